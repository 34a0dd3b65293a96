"""Pins for the assembled multigrid: the sparse transfer matrices equal the
oracle's transfer functions, rediscretized assembled levels equal the
matrix-free ones, the Galerkin products satisfy R A P on random vectors,
SMMG's node transfer is Galerkin in the time structure (its Galerkin and
rediscretized level-1 operators agree), and the assembled V-cycle with the
block-Jacobi-free ILU(0)-GMRES smoother reaches the dense solution."""
import numpy as np
import pytest

import stmg_inputs as si
import scipy.sparse as sp

from oracle import allatonce, galerkin, ilu, mg, stepper


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


# --- 2D Galerkin coarse operators (space coarsening, periodic) ---------------
def _stencil(vx, vy):
    """3 x 3 stencil [dy][dx] of the tensor product of 1D 3-point stencils."""
    return np.outer(np.asarray(vy), np.asarray(vx))


@pytest.mark.parametrize("M", [1, 2, 3])
def test_galerkin_2d_coarse_stencils_closed_form(M):
    """R A P for bilinear P and full weighting R = P^T / 4 on the FD-scaled
    operator: in 1D, R I P = [1/8, 3/4, 1/8], R D2_h P = D2_{2h}, and a
    symmetric stencil [a, b, a] becomes [a/2 + b/8, a + 3b/4, a/2 + b/8]
    (worked out by hand from the transfer definitions); in 2D the products are
    tensor products, so the Galerkin levels are
      K_q (x) Mc + dt diag(b) (x) (-nu (Dxx (x) m_y + m_x (x) Dyy) + lambda Mc)
    on the diagonal and -l(0) e_M^T (x) Mc below, with 9-point stencils."""
    from oracle import radau
    prob = si.problem(2, 16, M, 3, 0.3, nu=0.05, lam=0.7)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0, min_coarse=1)
    As, _, _ = galerkin.operators(levels, kinds, galerkin=True)
    t = radau.tables(M)
    m = np.array([0.0, 1.0, 0.0])
    for l in range(1, min(3, len(levels))):
        lev = levels[l]
        m = np.array([m[0] / 2 + m[1] / 8, m[0] + 3 * m[1] / 4, m[0] / 2 + m[1] / 8])
        H = lev.hx
        d2 = np.array([1.0, -2.0, 1.0]) / H ** 2
        Mc = _stencil(m, m)
        Kc = -prob["nu"] * (_stencil(d2, m) + _stencil(m, d2)) + prob["lambda"] * Mc
        diag, sub = galerkin.space_stencils(As[l], lev.shape)
        for i in range(M):
            for j in range(M):
                want = t["Kq"][i, j] * Mc + (lev.dt * t["b"][i] * Kc if i == j else 0.0)
                assert np.abs(diag[i, j] - want).max() < 1e-12 * max(1.0, np.abs(want).max())
                wsub = -t["l0"][i] * Mc if j == M - 1 else 0.0 * Mc
                assert np.abs(sub[i, j] - wsub).max() < 1e-13
        # nothing outside the 3 x 3 neighbourhood: row sums match
        row = sp.csr_matrix(As[l])[lev.M * lev.nx * lev.ny]
        assert abs(row.sum() - (diag[0].sum() + sub[0].sum())) < 1e-10 * np.abs(row.data).sum()


def test_galerkin_2d_products_on_random_vectors():
    """The assembled Galerkin matrix applied to a vector equals R (A (P x))."""
    prob = si.problem(2, 16, 2, 4, 0.5, nu=0.02, lam=1.0)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0)
    As, Ps, Rs = galerkin.operators(levels, kinds, galerkin=True)
    rng = np.random.default_rng(3)
    for l in range(len(levels) - 1):
        x = rng.standard_normal(As[l + 1].shape[0])
        assert np.abs(As[l + 1] @ x - Rs[l] @ (As[l] @ (Ps[l] @ x))).max() < 1e-12 * np.abs(x).max() * 1e3


@pytest.mark.parametrize("chunk", [1, 4])
def test_point_block_smoother_equals_matrix_free_on_rediscretized_levels(chunk):
    """On rediscretized levels the generic assembled point-block smoother is
    the matrix-free block-Jacobi sweep of oracle.mg (itself pinned against the
    dense chunk-matrix form)."""
    prob = si.problem(2, 8, 3, 8, 0.5, nu=0.02, lam=1.0)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0)
    As, _, _ = galerkin.operators(levels, kinds, galerkin=False)
    rng = np.random.default_rng(5)
    for l, lev in enumerate(levels):
        U = rng.standard_normal(lev.shape)
        f = rng.standard_normal(lev.shape)
        got = galerkin.point_block_smooth(As[l], lev.shape, U, f, 0.8, chunk)
        assert np.abs(got - lev.smooth(U, f, 0.8, chunk)).max() < 1e-12


def test_galerkin_smg_2d_converges_to_stepper():
    """SMG V-cycles with Galerkin coarse levels and the point-block smoother
    (chunks of 16 / 4 slabs) reach the stepper's solution."""
    prob = si.problem(2, 16, 2, 8, 0.5, nu=0.02, lam=1.0)
    u0 = si.u0_rd2d(prob, 4)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0)
    As, Ps, Rs = galerkin.operators(levels, kinds, galerkin=True)
    sms = [(lambda x, g, l=l: galerkin.point_block_smooth(As[l], levels[l].shape, x, g, 0.8,
                                                           16 if l == 0 else 4).reshape(-1))
           for l in range(len(levels))]
    coarse = galerkin.exact_coarse(As[-1])
    f = mg.rhs(levels, u0).reshape(-1)
    x = np.zeros_like(f)
    nb = np.linalg.norm(f)
    for _ in range(40):
        x = galerkin.vcycle(As, Ps, Rs, sms, coarse, x, f)
        if np.linalg.norm(f - As[0] @ x) <= 1e-12 * nb:
            break
    Ue = stepper.solve_linear(prob, u0)
    assert np.linalg.norm(x - Ue.reshape(-1)) <= 1e-10 * np.linalg.norm(Ue)


def test_damping_closed_form():
    """Rediscretized levels: omega itself.  Galerkin levels: the mass stencil
    sums to one (R I P conserves the row sum: P has unit row sums, R = P^T / 2^d
    has column sums of 2^d / 2^d = 1 per coarse point), so the factor is the
    centre weight, (3/4)^d after one coarsening and (11/16)^d after two
    (1D recurrence [a, b, a] -> [a/2 + b/8, a + 3b/4, a/2 + b/8] from [0, 1, 0])."""
    for dim, n in [(1, 64), (2, 16)]:
        prob = si.problem(dim, n, 2, 4, 0.2, nu=0.05, lam=0.5)
        levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0)
        Ar, _, _ = galerkin.operators(levels, kinds, galerkin=False)
        Ag, _, _ = galerkin.operators(levels, kinds, galerkin=True)
        for l, lev in enumerate(levels):
            assert galerkin.damping(Ar[l], lev.shape, 0.8) == pytest.approx(0.8, abs=1e-15)
        want = [1.0, 0.75 ** dim, (11 / 16) ** dim]
        for l in range(3):
            assert galerkin.damping(Ag[l], levels[l].shape, 0.8) == pytest.approx(0.8 * want[l], rel=1e-13)
