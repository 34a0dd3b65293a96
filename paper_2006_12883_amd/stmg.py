"""Python front end of the space-time multigrid library.

`Handle` owns the workspace tensor and the library handle of one problem.
Every method forwards to one C-ABI call; tensors must be float64,
contiguous and on the handle's device.
"""
import ctypes

import torch

from . import binding as B


def _ptr(t):
    if t is None:
        return None
    if t.dtype != torch.float64 or not t.is_contiguous() or not t.is_cuda:
        raise ValueError("expected a contiguous float64 device tensor")
    return ctypes.c_void_p(t.data_ptr())


def residual_noalloc(prob, u0, U, r=None):
    """||b - A(U)|| (and r when given) through stmg_residual_noalloc: no
    handle, no workspace, nothing allocated by the library; the work goes on
    the current stream of U's device."""
    n = ctypes.c_double()
    stream = torch.cuda.current_stream(U.device)
    B.check(B.lib().stmg_residual_noalloc(ctypes.byref(B.make_problem(prob)), _ptr(u0), _ptr(U), _ptr(r),
                                          ctypes.byref(n), ctypes.c_void_p(stream.cuda_stream)),
            "stmg_residual_noalloc")
    return n.value


class Handle:
    def __init__(self, prob, device="cuda", **opts):
        self.prob = dict(prob)
        self.device = torch.device(device)
        self._p = B.make_problem(prob)
        self._o = B.make_options(**opts)
        L = B.lib()
        nbytes = L.stmg_workspace_bytes(ctypes.byref(self._p), ctypes.byref(self._o))
        if nbytes == 0:
            raise B.STMGError(B.STMG_EINVAL, "stmg_workspace_bytes")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        B.check(L.stmg_setup(ctypes.byref(self._p), ctypes.byref(self._o), ctypes.c_void_p(base + off),
                             nbytes, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "stmg_setup")
        self.h = h
        ny = 1 if prob["dim"] == 1 else prob["nx"][1] + (0 if prob.get("bc", "periodic") == "periodic" else 1)
        nx = prob["nx"][0] + (0 if prob.get("bc", "periodic") == "periodic" else 1)
        self.space_shape = (ny, nx)
        self.shape = (prob["N"], prob["M"], ny, nx)

    def close(self):
        if getattr(self, "h", None):
            B.lib().stmg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- hierarchy -------------------------------------------------------
    def levels(self):
        L = B.lib()
        out = []
        for l in range(L.stmg_num_levels(self.h)):
            a = (ctypes.c_int32 * 4)()
            dt = ctypes.c_double()
            B.check(L.stmg_level_shape(self.h, l, a, ctypes.byref(dt)), "stmg_level_shape")
            m = L.stmg_level_nodes(self.h, l)
            B.check(min(m, 0), "stmg_level_nodes")
            out.append(dict(nx=a[0], ny=a[1], N=a[2], kind=a[3], dt=dt.value, M=m))
        return out

    def level_shape(self, l):
        d = self.levels()[l]
        return (d["N"], d["M"], d["ny"], d["nx"])

    # --- main entry points -----------------------------------------------
    def residual(self, u0, U, r=None):
        n = ctypes.c_double()
        B.check(B.lib().stmg_residual(self.h, _ptr(u0), _ptr(U), _ptr(r), ctypes.byref(n)), "stmg_residual")
        return n.value

    def vcycle(self, u0, U):
        rel = ctypes.c_double()
        B.check(B.lib().stmg_vcycle(self.h, _ptr(u0), _ptr(U), ctypes.byref(rel)), "stmg_vcycle")
        return rel.value

    def solve(self, u0, U=None, check=True):
        if U is None:
            U = torch.zeros(self.shape, dtype=torch.float64, device=self.device)
        st = B.Stats()
        rc = B.lib().stmg_solve(self.h, _ptr(u0), _ptr(U), ctypes.byref(st))
        if check:
            B.check(rc, "stmg_solve")
        return U, st.as_dict()

    def num_windows(self):
        return B.lib().stmg_num_windows(self.h)

    def solve_end(self, u0, check=True):
        """Solve and return only u(T) (windowed handles: no trajectory stored)."""
        uT = torch.empty(self.space_shape, dtype=torch.float64, device=self.device)
        st = B.Stats()
        rc = B.lib().stmg_solve_end(self.h, _ptr(u0), _ptr(uT), ctypes.byref(st))
        if check:
            B.check(rc, "stmg_solve_end")
        return uT, st.as_dict()

    def adjoint(self, U, gT, u0=None):
        """(dL/du0, dL/dnu, stats) for L with dL/du(T) = gT; U may be None on a
        windowed handle (the trajectory is recomputed from u0)."""
        g = torch.empty(self.space_shape, dtype=torch.float64, device=self.device)
        gnu = ctypes.c_double()
        st = B.Stats()
        B.check(B.lib().stmg_adjoint(self.h, _ptr(u0), _ptr(U), _ptr(gT), _ptr(g), ctypes.byref(gnu),
                                     ctypes.byref(st)), "stmg_adjoint")
        return g, gnu.value, st.as_dict()

    def sdc_sweep(self, u0, U, sweeps=1):
        rel = ctypes.c_double()
        B.check(B.lib().stmg_sdc_sweep(self.h, _ptr(u0), _ptr(U), int(sweeps), ctypes.byref(rel)),
                "stmg_sdc_sweep")
        return rel.value

    def pfasst(self, u0, U=None, check=True):
        """PFASST iterations (handle set up with pfasst_levels >= 2) from U
        (zero if None); returns (U, stats)."""
        if U is None:
            U = torch.zeros(self.shape, dtype=torch.float64, device=self.device)
        st = B.Stats()
        rc = B.lib().stmg_pfasst_solve(self.h, _ptr(u0), _ptr(U), ctypes.byref(st))
        if check:
            B.check(rc, "stmg_pfasst_solve")
        return U, st.as_dict()

    # --- components --------------------------------------------------------
    def smooth(self, level, Uin, Uout, f=None, u0=None):
        B.check(B.lib().stmg_level_smooth(self.h, level, _ptr(f), _ptr(u0), _ptr(Uin), _ptr(Uout)),
                "stmg_level_smooth")

    def restrict_residual(self, level, U, fc, f=None, u0=None):
        B.check(B.lib().stmg_level_restrict_residual(self.h, level, _ptr(f), _ptr(u0), _ptr(U), _ptr(fc)),
                "stmg_level_restrict_residual")

    def prolong(self, level, ec, Uout, Uin=None):
        B.check(B.lib().stmg_level_prolong(self.h, level, _ptr(Uin), _ptr(ec), _ptr(Uout)),
                "stmg_level_prolong")

    def smooth_restrict(self, level, Uout, fc, Uin=None, uc=None, f=None, u0=None):
        B.check(B.lib().stmg_level_smooth_restrict(self.h, level, _ptr(f), _ptr(u0), _ptr(Uin), _ptr(Uout),
                                                   _ptr(fc), _ptr(uc)), "stmg_level_smooth_restrict")

    def prolong_smooth(self, level, ec, Uout, Uin=None, f=None, u0=None):
        B.check(B.lib().stmg_level_prolong_smooth(self.h, level, _ptr(f), _ptr(u0), _ptr(Uin), _ptr(ec),
                                                  _ptr(Uout)), "stmg_level_prolong_smooth")

    def coarse_solve(self, f, U):
        B.check(B.lib().stmg_coarse_solve(self.h, _ptr(f), _ptr(U)), "stmg_coarse_solve")


def solve(u0, prob, **opts):
    """Solve the all-at-once system for one problem; returns (U, stats)."""
    h = Handle(prob, device=u0.device, **opts)
    try:
        return h.solve(u0)
    finally:
        h.close()


class Batch:
    """Many independent 2D periodic linear problems solved together
    (stmg_batch_*): FP32 V-cycles inside FP64 refinement, one graph replay
    per refinement step for all problems."""

    def __init__(self, probs, device="cuda", **opts):
        self.probs = [dict(p) for p in probs]
        self.device = torch.device(device)
        n = len(probs)
        self._p = (B.Problem * n)(*[B.make_problem(p) for p in probs])
        self._o = B.make_options(**opts)
        L = B.lib()
        nbytes = L.stmg_batch_workspace_bytes(n, self._p, ctypes.byref(self._o))
        if nbytes == 0:
            raise B.STMGError(B.STMG_EUNSUPPORTED, "stmg_batch_workspace_bytes")
        self.ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.ws.data_ptr()
        off = (-base) % 256
        self.stream = torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        B.check(L.stmg_batch_setup(n, self._p, ctypes.byref(self._o), ctypes.c_void_p(base + off), nbytes,
                                   ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)), "stmg_batch_setup")
        self.h = h
        self.shapes = []
        for p in probs:
            ny, nx = p["nx"][1], p["nx"][0]
            self.shapes.append((p["N"], p["M"], ny, nx))

    def solve(self, u0s, Us=None, check=True):
        n = len(self.probs)
        if Us is None:
            Us = [torch.zeros(s, dtype=torch.float64, device=self.device) for s in self.shapes]
        pu0 = (ctypes.c_void_p * n)(*[_ptr(u).value for u in u0s])
        pU = (ctypes.c_void_p * n)(*[_ptr(U).value for U in Us])
        st = (B.Stats * n)()
        rc = B.lib().stmg_batch_solve(self.h, pu0, pU, st)
        if check:
            B.check(rc, "stmg_batch_solve")
        return Us, [s.as_dict() for s in st]

    def close(self):
        if getattr(self, "h", None):
            B.lib().stmg_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
