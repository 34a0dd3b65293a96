"""Pins for the oracle's ILU(0) and the ILU(0)-GMRES smoother: the factors
reproduce A on its pattern and vanish off it, the factorisation is exact for
a matrix whose LU has no fill (block lower-bidiagonal in time with
tridiagonal blocks), the level operators assemble to the matrix-free ones,
and the smoother reduces the preconditioned residual as GMRES must."""
import numpy as np
import pytest
import scipy.sparse as sp

import stmg_inputs as si
from oracle import allatonce, ilu, mg


def _rand_sparse(n, seed):
    rng = np.random.default_rng(seed)
    A = sp.random(n, n, density=0.08, random_state=np.random.RandomState(seed), format="csr")
    A = A + sp.diags(4.0 + rng.random(n))
    return sp.csr_matrix(A)


def test_factors_reproduce_a_on_its_pattern():
    A = _rand_sparse(60, 1)
    L, U = ilu.ilu0(A)
    LU = (L @ U).toarray()
    Ad = A.toarray()
    pat = Ad != 0
    assert np.abs(LU[pat] - Ad[pat]).max() <= 1e-13 * np.abs(Ad).max()
    # no entry of L or U outside the pattern of A
    assert not ((L.toarray() != 0) & ~pat & ~np.eye(60, dtype=bool)).any()
    assert not ((U.toarray() != 0) & ~pat).any()


def test_exact_without_fill():
    # the LU factors of a tridiagonal matrix (here block diagonal with
    # tridiagonal blocks) have no fill, so ILU(0) is the exact LU
    n, nb = 12, 5
    rng = np.random.default_rng(2)
    T = sp.diags([-1.0 * np.ones(n - 1), 4.0 + rng.random(n), -1.3 * np.ones(n - 1)], [-1, 0, 1])
    A = sp.csr_matrix(sp.kron(sp.identity(nb), T))
    L, U = ilu.ilu0(A)
    assert np.abs((L @ U - A).toarray()).max() <= 1e-13
    b = rng.standard_normal(A.shape[0])
    x = ilu.ilu_solve(L, U, b)
    assert np.abs(A @ x - b).max() <= 1e-12
    # with a lower block coupling the factorisation is no longer exact: the
    # dropped fill shows up off the pattern only
    A2 = sp.csr_matrix(A + sp.kron(sp.diags([np.ones(nb - 1)], [-1]), -0.5 * sp.identity(n)))
    L2, U2 = ilu.ilu0(A2)
    D = (L2 @ U2 - A2).toarray()
    pat = A2.toarray() != 0
    assert np.abs(D[pat]).max() <= 1e-13 and np.abs(D[~pat]).max() > 1e-3


def test_level_matrices_match_matrix_free_operators():
    prob = si.problem(1, 32, 3, 8, 0.5, nu=1.0)
    levels, kinds = mg.hierarchy(prob, coarsen="smmg", fft_coarse=0, min_coarse=16)
    rng = np.random.default_rng(3)
    for lev in levels:
        A = allatonce.matrix(mg.level_problem(lev))
        U = rng.standard_normal(lev.shape)
        assert np.abs(A @ U.ravel() - lev.apply(U).ravel()).max() <= 1e-11 * np.abs(lev.apply(U)).max()


@pytest.mark.parametrize("nu", [1, 3])
def test_gmres_smoothing_reduces_preconditioned_residual(nu):
    prob = si.problem(1, 32, 2, 8, 0.5, nu=1.0)
    levels, _ = mg.hierarchy(prob, fft_coarse=0, min_coarse=16)
    lev = levels[0]
    A = allatonce.matrix(mg.level_problem(lev))
    L, U = ilu.ilu0(A)
    sm = ilu.ilu_gmres_smoother(A, nu)
    rng = np.random.default_rng(4)
    x = rng.standard_normal(lev.shape)
    f = rng.standard_normal(lev.shape)

    def pres(v):
        return np.linalg.norm(ilu.ilu_solve(L, U, f.ravel() - A @ v.ravel()))

    x1 = sm(x, f)
    assert pres(x1) < pres(x)
    # more iterations never increase the minimised norm
    assert pres(ilu.ilu_gmres_smoother(A, nu + 2)(x, f)) <= pres(x1) * (1 + 1e-12)


def test_vcycle_with_ilu_gmres_converges():
    prob = si.problem(1, 64, 2, 16, 0.5, nu=1.0)
    u0 = si.u0_heat1d(prob)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0, min_coarse=16)
    sms = [ilu.ilu_gmres_smoother(allatonce.matrix(mg.level_problem(lev)), 3) for lev in levels[:-1]]
    f = mg.rhs(levels, u0)
    U = np.zeros(levels[0].shape)
    nb = np.linalg.norm(f)
    for _ in range(30):
        U = mg.vcycle(levels, kinds, U, f, smoothers=sms)
        if np.linalg.norm(f - levels[0].apply(U)) <= 1e-10 * nb:
            break
    ref = allatonce.dense_solve(prob, u0)
    assert np.abs(U - ref).max() <= 1e-8 * np.abs(ref).max()
