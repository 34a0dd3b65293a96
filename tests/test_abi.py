"""The C-ABI library loads and exports every symbol the header declares;
host-side argument checks (no GPU needed)."""
import ctypes
import os
import re

import pytest

from paper_2006_12883_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_header_symbols_exported():
    hdr = open(os.path.join(ROOT, "include", "stmg.h")).read()
    declared = set(re.findall(r"\b(stmg_[a-z_0-9]+)\s*\(", hdr))
    assert declared == set(B.EXPORTS)
    L = B.lib()
    for name in declared:
        assert hasattr(L, name), name


def test_status_strings():
    L = B.lib()
    assert L.stmg_status_string(0) == b"ok"
    assert L.stmg_status_string(-4) == b"not converged"


def test_workspace_and_validation():
    import stmg_inputs as si
    prob = si.config("rd2d")
    n = B.workspace_bytes(prob)
    # level 0 needs at least a ping-pong and a right-hand-side FP64 vector
    assert n > 2 * 8 * 256 * 256 * 3 * 256
    for bad in [dict(prob, M=0), dict(prob, M=9), dict(prob, N=0), dict(prob, dt=-1.0),
                dict(prob, nu=0.0), dict(prob, dim=3), dict(prob, nx=[2, 2])]:
        assert B.lib().stmg_workspace_bytes(ctypes.byref(B.make_problem(bad)),
                                            ctypes.byref(B.make_options())) == 0
    assert B.lib().stmg_setup(None, None, None, 0, None, None) == B.STMG_EINVAL
    for bad in (0, 65):
        assert B.lib().stmg_workspace_bytes(ctypes.byref(B.make_problem(prob)),
                                            ctypes.byref(B.make_options(inner_cycles=bad))) == 0
    for bad in (-1, 33):
        assert B.lib().stmg_workspace_bytes(ctypes.byref(B.make_problem(prob)),
                                            ctypes.byref(B.make_options(krylov=bad))) == 0
    # the Krylov method adds 2 (m + 1) level-0 FP64 vectors
    m = 4
    extra = B.workspace_bytes(prob, krylov=m) - n
    assert extra >= 2 * (m + 1) * 8 * 256 * 256 * 3 * 256


def test_options_defaults():
    o = B.make_options()
    assert o.omega == 0.8 and o.chunk == 16 and o.chunk_coarse == 4 and o.nu_pre == 1 and o.nu_post == 1
    assert o.mu_crit == 0.5
    assert o.rtol == 1e-12 and o.coarsen == 0 and o.precision == 0
    assert o.krylov == 0 and o.inner_cycles == 5 and o.inner_adapt == 1


def test_batch_workspace_counts_inner_cycles():
    """The batch work-item table grows with the FP32 cycles per refinement
    step (one level-0 sweep item per further cycle and problem)."""
    import stmg_inputs as si
    probs = [si.problem(2, 32, 2, 16, 1.0, nu=1e-2, lam=0.5), si.problem(2, 48, 3, 8, 1.0, nu=1e-1, lam=1.0)]
    arr = (B.Problem * len(probs))(*[B.make_problem(p) for p in probs])
    sizes = [B.lib().stmg_batch_workspace_bytes(len(probs), arr, ctypes.byref(B.make_options(inner_cycles=k)))
             for k in (1, 5, 64)]
    assert all(x > 0 for x in sizes)
    assert sizes[0] < sizes[1] < sizes[2]


def test_undersized_workspace_is_refused_on_the_host():
    """stmg_setup checks the workspace size before it touches the device:
    one byte short of stmg_workspace_bytes gives STMG_ENOMEM (the pointer
    below is never dereferenced)."""
    import stmg_inputs as si
    prob = si.problem(2, 32, 3, 16, 0.5, nu=1e-2, lam=1.0)
    P, O = B.make_problem(prob), B.make_options()
    need = B.lib().stmg_workspace_bytes(ctypes.byref(P), ctypes.byref(O))
    assert need > 0
    h = ctypes.c_void_p()
    rc = B.lib().stmg_setup(ctypes.byref(P), ctypes.byref(O), ctypes.c_void_p(1 << 20), need - 1, None,
                            ctypes.byref(h))
    assert rc == B.STMG_ENOMEM
    assert b"workspace too small" in B.lib().stmg_last_error()
    # misaligned workspace: EINVAL, also before any device access
    rc = B.lib().stmg_setup(ctypes.byref(P), ctypes.byref(O), ctypes.c_void_p((1 << 20) + 8), need, None,
                            ctypes.byref(h))
    assert rc == B.STMG_EINVAL


def test_galerkin_option_validation_and_workspace():
    """Galerkin coarse levels: accepted for space coarsening of periodic linear
    problems with a Fourier coarsest level, and then take one more level-sized
    vector per coarse level plus the mass symbol; refused (workspace 0)
    otherwise."""
    import stmg_inputs as si
    prob = si.config("rd2d")
    ws = lambda p, **o: B.lib().stmg_workspace_bytes(ctypes.byref(B.make_problem(p)),
                                                     ctypes.byref(B.make_options(**o)))
    n = ws(prob, coarsen="space")
    g = ws(prob, coarsen="space", coarse_op="galerkin")
    assert n > 0 and g > n
    # levels 128^2 and 64^2 (the Fourier coarsest), N = 256, M = 3; the
    # rediscretized hierarchy also holds the fused level-0 sweep's planes at
    # its 7 run boundaries (runs of 32 slabs, 256^2 points)
    assert g - n + 8 * 7 * 256 * 256 >= 8 * 3 * 256 * (128 * 128 + 64 * 64)
    assert ws(prob, coarse_op="galerkin") == 0                      # coarsen auto
    assert ws(dict(prob, bc="neumann"), coarsen="space", coarse_op="galerkin") == 0
    ac = si.config("ac2d")
    assert ws(ac, coarsen="space", coarse_op="galerkin") == 0       # nonlinear
    # fft_coarse = 0: the hierarchy runs down to min_coarse, still Fourier-solved
    assert ws(prob, coarsen="space", coarse_op="galerkin", fft_coarse=0) > 0
    assert ws(prob, coarsen="space", coarse_op=2) == 0


def test_pfasst_option_validation_and_workspace():
    """PFASST levels: accepted for FP64 problems (Allen-Cahn IMEX) whose
    element counts stay even down the levels, adding the coarse levels' vectors and solvers
    to the workspace; refused (workspace 0) otherwise."""
    import stmg_inputs as si
    prob = si.config("rd2d")
    ws = lambda p, **o: B.lib().stmg_workspace_bytes(ctypes.byref(B.make_problem(p)),
                                                     ctypes.byref(B.make_options(**o)))
    n = ws(prob)
    assert ws(prob, pfasst_levels=2) > n and ws(prob, pfasst_levels=3) > ws(prob, pfasst_levels=2)
    assert ws(prob, pfasst_levels=1) == 0
    assert ws(prob, pfasst_levels=9) == 0
    assert ws(prob, pfasst_levels=2, pfasst_sweeps=0) == 0
    assert ws(prob, pfasst_levels=2, precision="mixed") == 0
    assert ws(prob, pfasst_levels=2, pfasst_inner_cycles=2) > 0
    assert ws(prob, pfasst_levels=2, pfasst_inner_cycles=-1) == 0
    assert ws(prob, pfasst_levels=2, pfasst_inner_cycles=101) == 0
    assert ws(si.config("ac2d"), pfasst_levels=2) > 0                   # IMEX
    assert ws(si.config("ac2d"), pfasst_levels=2, precision="mixed") == 0
    assert ws(dict(prob, nx=[10, 10]), pfasst_levels=3) == 0  # 10 -> 5 elements, odd: no second halving
    assert ws(dict(prob, nx=[12, 12]), pfasst_levels=3) > 0   # 12 -> 6 -> 3
    assert ws(dict(prob, nx=[8, 8]), pfasst_levels=2) > 0     # 8 -> 4
    assert ws(dict(prob, nx=[8, 8]), pfasst_levels=3) == 0    # 4 -> 2: fewer than 3 points
