"""Pins for the assembled multigrid: the sparse transfer matrices equal the
oracle's transfer functions, rediscretized assembled levels equal the
matrix-free ones, the Galerkin products satisfy R A P on random vectors,
SMMG's node transfer is Galerkin in the time structure (its Galerkin and
rediscretized level-1 operators agree), and the assembled V-cycle with the
block-Jacobi-free ILU(0)-GMRES smoother reaches the dense solution."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import allatonce, galerkin, ilu, mg


@pytest.mark.parametrize("coarsen", ["space", "spacetime", "smmg", "auto"])
def test_transfer_matrices_match_functions(coarsen):
    prob = si.problem(1, 32, 3, 8, 0.5, nu=1.0)
    levels, kinds = mg.hierarchy(prob, coarsen=coarsen, fft_coarse=0, min_coarse=8)
    rng = np.random.default_rng(1)
    for l in range(len(levels) - 1):
        P, R = galerkin.transfers(levels[l], levels[l + 1], kinds[l])
        e = rng.standard_normal(levels[l + 1].shape)
        r = rng.standard_normal(levels[l].shape)
        assert np.abs(P @ e.ravel() - mg.prolong(e, kinds[l], 1, levels[l].Pm).ravel()).max() <= 1e-14
        assert np.abs(R @ r.ravel() - mg.restrict(r, kinds[l], 1, levels[l].Pm).ravel()).max() <= 1e-13


def test_assembled_vcycle_equals_matrix_free_with_same_smoother():
    # rediscretized assembled levels, ILU(0)-GMRES smoothing: the assembled
    # V-cycle and oracle.mg's V-cycle with the same smoothers agree
    prob = si.problem(1, 32, 2, 8, 0.5, nu=1.0)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0, min_coarse=16)
    As, Ps, Rs = galerkin.operators(levels, kinds, galerkin=False)
    sms = [ilu.ilu_gmres_smoother(A, 3) for A in As[:-1]]
    rng = np.random.default_rng(2)
    x = rng.standard_normal(levels[0].shape)
    f = rng.standard_normal(levels[0].shape)
    got = galerkin.vcycle(As, Ps, Rs, sms, galerkin.exact_coarse(As[-1]), x.ravel(), f.ravel())
    ref = mg.vcycle(levels, kinds, x.copy(), f, smoothers=[lambda v, g, s=s: s(v, g) for s in sms])
    assert np.abs(got - ref.ravel()).max() <= 1e-10 * np.abs(ref).max()


def test_galerkin_products_and_node_transfer():
    prob = si.problem(1, 32, 3, 8, 0.5, nu=1.0)
    levels, kinds = mg.hierarchy(prob, coarsen="smmg", fft_coarse=0, min_coarse=16)
    Ag, Ps, Rs = galerkin.operators(levels, kinds, galerkin=True)
    Ar, _, _ = galerkin.operators(levels, kinds, galerkin=False)
    rng = np.random.default_rng(3)
    e = rng.standard_normal(Ag[1].shape[0])
    assert np.abs(Ag[1] @ e - Rs[0] @ (Ag[0] @ (Ps[0] @ e))).max() <= 1e-10 * np.abs(Ag[1] @ e).max()
    # space coarsening of the 1D Laplacian and the Lagrange node transfer are
    # Galerkin-exact for the stiffness and time parts; what differs is the
    # identity in space, which becomes R_s P_s (a three-point average)
    D = (Ag[1] - Ar[1]).toarray()
    assert np.abs(D).max() > 1e-6


def test_assembled_galerkin_vcycle_converges():
    prob = si.problem(1, 64, 2, 16, 0.5, nu=1.0)
    u0 = si.u0_heat1d(prob)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0, min_coarse=16)
    As, Ps, Rs = galerkin.operators(levels, kinds, galerkin=True)
    sms = [ilu.ilu_gmres_smoother(A, 3) for A in As[:-1]]
    coarse = galerkin.exact_coarse(As[-1])
    f = mg.rhs(levels, u0).ravel()
    x = np.zeros_like(f)
    for _ in range(40):
        x = galerkin.vcycle(As, Ps, Rs, sms, coarse, x, f)
        if np.linalg.norm(f - As[0] @ x) <= 1e-10 * np.linalg.norm(f):
            break
    ref = allatonce.dense_solve(prob, u0)
    assert np.abs(x - ref.ravel()).max() <= 1e-8 * np.abs(ref).max()
