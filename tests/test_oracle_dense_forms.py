"""Pins of the oracle's SDC sweep and block-Jacobi smoother against dense
formulations of the same iterations.

Both are stationary iterations U <- U + P^{-1} (b - C U) whose splitting is
fixed by what the method computes; here P and C are assembled as explicit
matrices and applied with a dense solve, instead of the forward
substitutions the oracle runs:

* SDC (Sec. 2.1; the sweep of PFASST, Sec. 4.1): per slab the collocation
  matrix C = I - dt Q (x) L and the preconditioner P = I - dt Q_Delta (x) L,
  Q_Delta the implicit-Euler lower-triangular matrix Q_Delta[m, j] = c_j - c_{j-1}
  (j <= m, c_0 = 0), with the previous slab's end value taken from the
  incoming iterate (Jacobi across slabs).
* block-Jacobi over chunks of slabs (Sec. 4.2): C is the all-at-once DG
  matrix assembled from the integral definitions of K_q, M_q and J_q, and P
  is the part of it that couples unknowns at the same grid point inside one
  chunk of slabs (the M x M point blocks on the diagonal and the
  -l(0) e_M^T couplings between consecutive slabs of the chunk), damped by
  omega.

A flipped sign or a wrong index in the oracle's substitution (the accumulated
explicit part of the SDC sweep, or the in-chunk coupling l(0) d_{n-1,M} of
the smoother) changes the iterate and fails these tests; the fixed-point
tests alone would not see it.
"""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import allatonce, mg, radau, sdc


def _lap_dense(nx, ny, hx, hy):
    """Periodic 5-point (or 3-point) Laplacian as a dense matrix on [y][x]."""
    P = nx * ny
    D = np.zeros((P, P))
    for y in range(ny):
        for x in range(nx):
            p = y * nx + x
            for dx in (-1, 1):
                D[p, y * nx + (x + dx) % nx] += 1.0 / hx ** 2
            D[p, p] -= 2.0 / hx ** 2
            if ny > 1:
                for dy in (-1, 1):
                    D[p, ((y + dy) % ny) * nx + x] += 1.0 / hy ** 2
                D[p, p] -= 2.0 / hy ** 2
    return D


def _sdc_dense(prob, u0, U):
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    nx = prob["nx"][0]
    ny = prob["nx"][1] if prob["dim"] == 2 else 1
    hx = prob["length"][0] / nx
    hy = prob["length"][1] / ny if prob["dim"] == 2 else 1.0
    L = prob["nu"] * _lap_dense(nx, ny, hx, hy) - prob["lambda"] * np.eye(nx * ny)
    t = radau.tables(M)
    c, Q = t["c"], t["Q"]
    QD = np.zeros((M, M))
    for m in range(M):
        for j in range(m + 1):
            QD[m, j] = c[j] - (c[j - 1] if j > 0 else 0.0)
    P = nx * ny
    I = np.eye(M * P)
    C = I - dt * np.kron(Q, L)
    Pre = I - dt * np.kron(QD, L)
    V = np.asarray(U).reshape(N, M * P)
    out = np.empty_like(V)
    for n in range(N):
        prev = np.asarray(u0).reshape(P) if n == 0 else V[n - 1, (M - 1) * P:]
        r = np.tile(prev, M) - C @ V[n]
        out[n] = V[n] + np.linalg.solve(Pre, r)
    return out.reshape(np.shape(U))


@pytest.mark.parametrize("M", [2, 3, 4])
@pytest.mark.parametrize("dim", [1, 2])
def test_sdc_sweep_is_dense_preconditioned_richardson(M, dim):
    """One oracle sweep = U + (I - dt Q_Delta (x) L)^{-1} (1 (x) u_{n-1} - (I - dt Q (x) L) U_n)
    per slab, from a random (non-converged) iterate."""
    nx = 12 if dim == 1 else 5
    prob = si.problem(dim, nx, M, 5, 0.4, nu=0.07, lam=0.6)
    rng = np.random.default_rng(100 + 10 * M + dim)
    shape = (prob["N"], M, nx if dim == 2 else 1, nx)
    U = rng.standard_normal(shape)
    u0 = rng.standard_normal(shape[2:])
    got = sdc.sweep(prob, u0, U)
    ref = _sdc_dense(prob, u0, U)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    # the sweep changes a non-converged iterate (the comparison is not vacuous)
    assert np.abs(got - U).max() > 1e-2


def _smooth_dense(prob, level, f, U, omega, chunk):
    """U + omega P^{-1} (f - A U) with A the assembled DG matrix and P its
    point-local part inside each chunk of slabs."""
    A = allatonce.matrix(prob).toarray()
    N, M, ny, nx = level.shape
    P = nx * ny
    K = M * P
    r = f.reshape(-1) - A @ U.reshape(-1)
    # unknown index = (n M + i) P + p: keep entries whose grid point agrees and
    # whose slabs lie in the same chunk (same slab, or n = m + 1 in the chunk)
    idx = np.arange(N * K)
    slab, point = idx // K, idx % P
    same_point = point[:, None] == point[None, :]
    same_chunk = (slab[:, None] // chunk) == (slab[None, :] // chunk)
    Pre = np.where(same_point & same_chunk, A, 0.0)
    d = np.linalg.solve(Pre, r)
    return U + omega * d.reshape(U.shape)


@pytest.mark.parametrize("chunk", [1, 4, 16])
@pytest.mark.parametrize("dim", [1, 2])
def test_smoother_is_dense_chunk_block_jacobi(chunk, dim):
    """One oracle smoothing sweep = U + omega C^{-1} (f - A U), C the point-local
    block lower-bidiagonal part of the assembled A on each chunk (N = 20 slabs:
    chunk 16 leaves a ragged chunk of 4)."""
    nx = 10 if dim == 1 else 4
    prob = si.problem(dim, nx, 3, 20, 0.8, nu=0.03, lam=0.7)
    levels, _ = mg.hierarchy(prob, min_coarse=10 ** 9)
    lev = levels[0]
    rng = np.random.default_rng(200 + chunk + dim)
    U = rng.standard_normal(lev.shape)
    u0 = rng.standard_normal(lev.shape[2:])
    f = mg.rhs(levels, u0)
    got = lev.smooth(U, f, 0.8, chunk)
    ref = _smooth_dense(prob, lev, f, U, 0.8, chunk)
    assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
    assert np.abs(got - U).max() > 1e-2


@pytest.mark.parametrize("prob", [si.problem(1, 12, 3, 4, 0.3, nu=0.5, lam=0.4),
                                  si.problem(2, 6, 2, 3, 0.5, nu=0.05, lam=1.0, bc="neumann"),
                                  si.problem(2, 6, 4, 3, 0.5, nu=0.01, gamma=1.0, reaction="allen_cahn")])
def test_collocation_residual(prob):
    """The collocation-form residual (built from Q) vanishes at the stepper's
    solution and equals Q diag(b)^-1 applied per slab and point to the DG
    residual (built from the integral definitions of K_q, M_q, J_q): the two
    forms have the same solution and residuals that differ by this factor."""
    from oracle import stepper
    rng = np.random.default_rng(12)
    ny, nx = si.grid_points(prob)
    u0 = 0.5 * rng.standard_normal((ny, nx))
    U = 0.5 * rng.standard_normal((prob["N"], prob["M"], ny, nx))
    t = radau.tables(prob["M"])
    G = t["Q"] / t["b"][None, :]
    rdg = allatonce.residual(prob, u0, U)
    rc = allatonce.residual_colloc(prob, u0, U)
    assert np.abs(rc - np.einsum("ij,njyx->niyx", G, rdg)).max() < 1e-12 * max(1.0, np.abs(rc).max())
    # G l(0) = 1: the collocation right-hand side is 1 (x) u0
    assert np.abs(G @ t["l0"] - 1.0).max() < 1e-13
    Ue = stepper.solve(prob, u0)
    assert np.abs(allatonce.residual_colloc(prob, u0, Ue)).max() < 1e-12
