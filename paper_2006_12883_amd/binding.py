"""ctypes binding of libstmg.so (the C ABI in include/stmg.h).

Argument marshalling only: every numerical step runs in the HIP library.
Device arrays are torch tensors (float64, contiguous, on the handle's
device); torch supplies memory and the current stream.  If the library has
not been built the binding raises -- there is no fallback.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libstmg.so")

STMG_OK, STMG_EINVAL, STMG_ENOMEM, STMG_EHIP = 0, -1, -2, -3
STMG_ENOTCONV, STMG_EDIVERGED, STMG_ENAN, STMG_EUNSUPPORTED = -4, -5, -6, -7
BC = {"periodic": 0, "neumann": 1}
REACTION = {"linear": 0, "allen_cahn": 1}
PRECISION = {"fp64": 0, "mixed": 1}
COARSEN = {"auto": 0, "space": 1, "spacetime": 2, "smmg": 3}
FORM = {"dg": 0, "colloc": 1}
SMOOTHER = {"pbj": 0, "sdc": 1}
COARSE_OP = {"redisc": 0, "galerkin": 1}

# every symbol the header declares
EXPORTS = [
    "stmg_default_options", "stmg_workspace_bytes", "stmg_setup", "stmg_num_levels",
    "stmg_level_shape", "stmg_level_nodes", "stmg_residual", "stmg_residual_noalloc", "stmg_vcycle", "stmg_solve", "stmg_solve_end",
    "stmg_num_windows", "stmg_tuned_shape", "stmg_adjoint",
    "stmg_sdc_sweep", "stmg_pfasst_solve", "stmg_level_smooth", "stmg_level_restrict_residual",
    "stmg_level_prolong", "stmg_level_prolong_smooth", "stmg_level_smooth_restrict", "stmg_coarse_solve", "stmg_destroy",
    "stmg_batch_workspace_bytes", "stmg_batch_setup", "stmg_batch_solve",
    "stmg_batch_destroy", "stmg_status_string", "stmg_last_error",
]


class Problem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nx", ctypes.c_int32 * 2), ("length", ctypes.c_double * 2),
                ("bc", ctypes.c_int32), ("nu", ctypes.c_double), ("reaction", ctypes.c_int32),
                ("lambda_", ctypes.c_double), ("gamma", ctypes.c_double), ("M", ctypes.c_int32),
                ("N", ctypes.c_int32), ("dt", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("coarsen", ctypes.c_int32), ("mu_crit", ctypes.c_double),
                ("omega", ctypes.c_double), ("chunk", ctypes.c_int32), ("chunk_coarse", ctypes.c_int32),
                ("nu_pre", ctypes.c_int32),
                ("nu_post", ctypes.c_int32), ("max_levels", ctypes.c_int32), ("min_coarse", ctypes.c_int32),
                ("max_cycles", ctypes.c_int32), ("rtol", ctypes.c_double), ("newton_rtol", ctypes.c_double),
                ("max_newton", ctypes.c_int32), ("mem_budget", ctypes.c_size_t), ("sdc", ctypes.c_int32),
                ("autotune", ctypes.c_int32), ("inner_cycles", ctypes.c_int32),
                ("fft_coarse", ctypes.c_int32), ("krylov", ctypes.c_int32),
                ("krylov_left", ctypes.c_int32), ("inner_adapt", ctypes.c_int32),
                ("form", ctypes.c_int32), ("smoother", ctypes.c_int32), ("coarse_op", ctypes.c_int32),
                ("pfasst_levels", ctypes.c_int32), ("pfasst_sweeps", ctypes.c_int32),
                ("pfasst_inner_cycles", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int32), ("newton_its", ctypes.c_int32), ("refinements", ctypes.c_int32),
                ("status", ctypes.c_int32), ("rel_res", ctypes.c_double), ("seconds", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libstmg.so is not built; run `python -m paper_2006_12883_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, dp, ip, sz = ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_int, ctypes.c_size_t
        P, O, S = ctypes.POINTER(Problem), ctypes.POINTER(Options), ctypes.POINTER(Stats)
        sig = {
            "stmg_default_options": (None, [O]),
            "stmg_workspace_bytes": (sz, [P, O]),
            "stmg_setup": (ip, [P, O, vp, sz, vp, ctypes.POINTER(vp)]),
            "stmg_num_levels": (ip, [vp]),
            "stmg_level_shape": (ip, [vp, ip, ctypes.POINTER(ctypes.c_int32), dp]),
            "stmg_level_nodes": (ip, [vp, ip]),
            "stmg_residual": (ip, [vp, vp, vp, vp, dp]),
            "stmg_residual_noalloc": (ip, [P, vp, vp, vp, dp, vp]),
            "stmg_vcycle": (ip, [vp, vp, vp, dp]),
            "stmg_solve": (ip, [vp, vp, vp, S]),
            "stmg_adjoint": (ip, [vp, vp, vp, vp, vp, dp, S]),
            "stmg_solve_end": (ip, [vp, vp, vp, S]),
            "stmg_num_windows": (ip, [vp]),
            "stmg_tuned_shape": (ip, [vp, ip]),
            "stmg_sdc_sweep": (ip, [vp, vp, vp, ctypes.c_int32, dp]),
            "stmg_pfasst_solve": (ip, [vp, vp, vp, S]),
            "stmg_level_smooth": (ip, [vp, ip, vp, vp, vp, vp]),
            "stmg_level_restrict_residual": (ip, [vp, ip, vp, vp, vp, vp]),
            "stmg_level_prolong": (ip, [vp, ip, vp, vp, vp]),
            "stmg_level_prolong_smooth": (ip, [vp, ip, vp, vp, vp, vp, vp]),
            "stmg_level_smooth_restrict": (ip, [vp, ip, vp, vp, vp, vp, vp, vp]),
            "stmg_coarse_solve": (ip, [vp, vp, vp]),
            "stmg_destroy": (None, [vp]),
            "stmg_batch_workspace_bytes": (sz, [ctypes.c_int32, P, O]),
            "stmg_batch_setup": (ip, [ctypes.c_int32, P, O, vp, sz, vp, ctypes.POINTER(vp)]),
            "stmg_batch_solve": (ip, [vp, ctypes.POINTER(vp), ctypes.POINTER(vp), S]),
            "stmg_batch_destroy": (None, [vp]),
            "stmg_status_string": (ctypes.c_char_p, [ip]),
            "stmg_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


class STMGError(RuntimeError):
    def __init__(self, status, where):
        L = lib()
        self.status = status
        msg = "%s: %s (%s)" % (where, L.stmg_status_string(status).decode(), L.stmg_last_error().decode())
        super().__init__(msg)


def check(rc, where):
    if rc != STMG_OK:
        raise STMGError(rc, where)
    return rc


def make_problem(d):
    p = Problem()
    p.dim = int(d["dim"])
    p.nx[0] = int(d["nx"][0])
    p.nx[1] = int(d["nx"][1]) if d["dim"] == 2 else 1
    p.length[0] = float(d["length"][0])
    p.length[1] = float(d["length"][1])
    p.bc = BC[d.get("bc", "periodic")]
    p.nu = float(d["nu"])
    p.reaction = REACTION[d.get("reaction", "linear")]
    p.lambda_ = float(d.get("lambda", 0.0))
    p.gamma = float(d.get("gamma", 0.0))
    p.M = int(d["M"])
    p.N = int(d["N"])
    p.dt = float(d["dt"])
    return p


def make_options(**kw):
    o = Options()
    lib().stmg_default_options(ctypes.byref(o))
    for k, v in kw.items():
        if k == "precision":
            v = PRECISION[v] if isinstance(v, str) else v
        if k == "coarsen":
            v = COARSEN[v] if isinstance(v, str) else v
        if k == "form":
            v = FORM[v] if isinstance(v, str) else v
        if k == "smoother":
            v = SMOOTHER[v] if isinstance(v, str) else v
        if k == "coarse_op":
            v = COARSE_OP[v] if isinstance(v, str) else v
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def workspace_bytes(prob, **opts):
    n = lib().stmg_workspace_bytes(ctypes.byref(make_problem(prob)), ctypes.byref(make_options(**opts)))
    if n == 0:
        raise STMGError(STMG_EINVAL, "stmg_workspace_bytes")
    return n
