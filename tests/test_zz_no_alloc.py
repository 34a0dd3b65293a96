"""The no-allocation residual (stmg_residual_noalloc) against the handle-based
stmg_residual: same kernels and launch shapes, so r and ||r|| agree bitwise.
Two calls in a row share the library's fixed device scratch, the second on a
smaller problem; a problem whose partial sums exceed the scratch is refused
on the host before any launch."""
import ctypes

import numpy as np
import pytest
import torch

import stmg_inputs as si
from paper_2006_12883_amd import binding as B
from paper_2006_12883_amd import stmg
from tests.gpu_util import T, H
from oracle import allatonce

pytestmark = pytest.mark.gpu


def _case(prob, seed):
    u0 = si.random_field(si.grid_points(prob), seed)
    N, M = prob["N"], prob["M"]
    U = si.random_field((N, M) + tuple(si.grid_points(prob)), seed + 1)
    return u0, U


def _both(prob, seed):
    u0, U = _case(prob, seed)
    du0, dU = T(u0), T(U)
    r_na = torch.full_like(dU, float("nan"))
    n_na = stmg.residual_noalloc(prob, du0, dU, r_na)
    h = H(prob)
    r_h = torch.full_like(dU, float("nan"))
    n_h = h.residual(du0, dU, r_h)
    torch.cuda.synchronize()
    return u0, U, r_na.cpu().numpy(), n_na, r_h.cpu().numpy(), n_h


def test_noalloc_residual_matches_handle_two_calls():
    big = si.problem(2, 64, 3, 40, 0.5, nu=1e-2, lam=1.0)        # 16 blocks x 5 slab runs
    small = si.problem(2, 32, 2, 9, 0.25, nu=5e-2, lam=0.5)      # 4 blocks x 2 slab runs
    for prob, seed in ((big, 11), (small, 21)):
        u0, U, r_na, n_na, r_h, n_h = _both(prob, seed)
        assert np.array_equal(r_na, r_h)
        assert n_na == n_h
        # and the residual is the system's: the oracle's entry-by-entry residual
        ref = allatonce.residual(prob, u0, U)
        scale = max(1.0, float(np.abs(ref).max()))
        assert float(np.abs(r_na - ref).max()) <= 1e-12 * scale
        assert abs(n_na - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)


def test_noalloc_residual_allen_cahn_norm_only():
    prob = si.problem(2, 32, 3, 16, 0.5, nu=1e-3, gamma=1.0, reaction="allen_cahn")
    u0, U = _case(prob, 31)
    U *= 0.5
    du0, dU = T(u0), T(U)
    n1 = stmg.residual_noalloc(prob, du0, dU)
    n2 = H(prob).residual(du0, dU)
    assert n1 == n2


def test_noalloc_refuses_oversized_problem_on_host():
    # 1024 x 1024 points need 4096 blocks per slab run; 257 runs exceed the scratch
    prob = si.problem(2, 1024, 1, 2056, 1.0, nu=1e-2, lam=1.0)
    dummy = torch.zeros(8, dtype=torch.float64, device="cuda:0")
    n = ctypes.c_double()
    rc = B.lib().stmg_residual_noalloc(ctypes.byref(B.make_problem(prob)), ctypes.c_void_p(dummy.data_ptr()),
                                       ctypes.c_void_p(dummy.data_ptr()), None, ctypes.byref(n), None)
    assert rc == B.STMG_EINVAL
    assert b"scratch" in B.lib().stmg_last_error()
