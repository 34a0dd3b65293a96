"""Assembled multigrid: the oracle's transfers as sparse matrices and
Galerkin coarse operators A_{l+1} = R_l A_l P_l, for comparing the
rediscretized coarse levels with the paper's Galerkin ones (Sec. 4.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Vectors are ordered [N][M][ny][nx] as everywhere in the oracle, so a
transfer that coarsens time, nodes and space is the Kronecker product
P = P_t (x) P_m (x) P_s of the one-dimensional factors of oracle.mg
(periodic grids; in 2D P_s = P_y (x) P_x):
  space  P_s[2X, X] = 1, P_s[2X+1, X] = P_s[2X+1, X+1] = 1/2 (periodic),
         R_s = P_s^T / 2^d;
  time   P_t[2J+1, J] = 1, P_t[2J, J] = P_t[2J, J-1] = 1/2 (J > 0),
         R_t = P_t^T;
  nodes  P_m = the Lagrange node prolongation, R_m = P_m^T.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import allatonce, mg


def _space_p(nc):
    rows, cols, vals = [], [], []
    for X in range(nc):
        rows += [2 * X, 2 * X + 1, 2 * X + 1]
        cols += [X, X, (X + 1) % nc]
        vals += [1.0, 0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * nc, nc))


def _time_p(Nc):
    rows, cols, vals = [], [], []
    for J in range(Nc):
        rows += [2 * J + 1, 2 * J]
        cols += [J, J]
        vals += [1.0, 0.5]
        if J > 0:
            rows.append(2 * J)
            cols.append(J - 1)
            vals.append(0.5)
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * Nc, Nc))


def transfers(fine, coarse, kind):
    """(P, R) between two consecutive levels of oracle.mg.hierarchy (periodic)."""
    assert fine.bc == "periodic"
    P1 = fine.nx * fine.ny
    if "s" in kind:
        Ps = _space_p(coarse.nx)
        if fine.dim == 2:
            Ps = sp.kron(_space_p(coarse.ny), Ps, format="csr")
        Rs = (0.5 ** fine.dim) * Ps.T
    else:
        Ps = sp.identity(P1, format="csr")
        Rs = Ps
    Pt = _time_p(coarse.N) if "t" in kind else sp.identity(fine.N, format="csr")
    Pm = sp.csr_matrix(fine.Pm) if "m" in kind else sp.identity(fine.M, format="csr")
    P = sp.kron(sp.kron(Pt, Pm), Ps, format="csr")
    R = sp.kron(sp.kron(Pt.T, Pm.T), Rs, format="csr")
    return P, R


def operators(levels, kinds, galerkin):
    """Level matrices: rediscretized (each level's own problem) or Galerkin
    products starting from the finest level's matrix."""
    As = [allatonce.matrix(mg.level_problem(levels[0]))]
    Ps, Rs = [], []
    for l in range(len(levels) - 1):
        P, R = transfers(levels[l], levels[l + 1], kinds[l])
        Ps.append(P)
        Rs.append(R)
        if galerkin:
            As.append(sp.csr_matrix(R @ As[l] @ P))
        else:
            As.append(allatonce.matrix(mg.level_problem(levels[l + 1])))
    return As, Ps, Rs


def vcycle(As, Ps, Rs, smoothers, coarse, x, f, l=0):
    """One V-cycle on assembled levels; smoothers[l](x, f) -> x' (one call
    before and one after the coarse correction), coarse(f) solves the last
    level exactly."""
    if l == len(As) - 1:
        return coarse(f)
    x = smoothers[l](x, f)
    fc = Rs[l] @ (f - As[l] @ x)
    ec = vcycle(As, Ps, Rs, smoothers, coarse, np.zeros(As[l + 1].shape[0]), fc, l + 1)
    x = x + Ps[l] @ ec
    return smoothers[l](x, f)


def exact_coarse(A):
    lu = spla.splu(sp.csc_matrix(A))
    return lu.solve


def point_block_smooth(A, shape, U, f, omega, chunk):
    """One sweep of the block-Jacobi smoother over chunks of `chunk` slabs on
    an assembled level matrix A (vectors [N][M][P]): r = f - A U; inside a
    chunk, forward substitution with the point-diagonal parts of the slab
    blocks, d_n(x) = B_n(x)^-1 (r_n(x) - [n not first in chunk] C_n(x)
    d_{n-1}(x)) with B_n(x) = A[(n, :, x), (n, :, x)] and C_n(x) =
    A[(n, :, x), (n-1, :, x)] (M x M each); U' = U + omega d.  On a
    rediscretized level B = K_q + dt diag(b) (2 nu/hx^2 + 2 nu/hy^2 + lam) and
    C = -l(0) e_M^T, which is the smoother of oracle.mg; on a Galerkin level
    the mass stencil's centre weight enters both."""
    N, M = shape[0], shape[1]
    P = int(np.prod(shape[2:]))
    A = sp.csr_matrix(A)
    u = np.asarray(U, dtype=np.float64).reshape(-1)
    r = (np.asarray(f, dtype=np.float64).reshape(-1) - A @ u).reshape(N, M, P)
    d = np.zeros((N, M, P))
    idx = lambda n, x: n * M * P + np.arange(M) * P + x
    for n in range(N):
        for x in range(P):
            rows = idx(n, x)
            B = A[rows][:, rows].toarray()
            rhs = r[n, :, x].copy()
            if n % chunk != 0:
                C = A[rows][:, idx(n - 1, x)].toarray()
                rhs -= C @ d[n - 1, :, x]
            d[n, :, x] = np.linalg.solve(B, rhs)
    return (u + omega * d.reshape(-1)).reshape(shape)


def damping(A, shape, omega):
    """Damping of the point-block sweep on a level matrix (N >= 2 slabs):
    omega m_0 / sum_x |m_x|, with m the mass stencil read off the coupling
    block to the previous slab, -l(0) e_M^T (x) Ms (row: slab 1, node 0,
    point 0).  The point block keeps only m_0, so a spatially smooth error
    sees the step omega sum|m| / m_0; the factor gives it the step omega of a
    level with identity mass (a rediscretized level, where the result is
    omega itself).  The centre entry and the row sum are those of the stencil
    on any periodic grid of two or more points."""
    N, M = shape[0], shape[1]
    P = int(np.prod(shape[2:]))
    assert N >= 2
    row = sp.csr_matrix(A)[M * P].toarray().ravel()
    c = row[(M - 1) * P:M * P]          # slab 0, node M-1, every point
    return omega * abs(c[0]) / np.abs(c).sum()


def space_stencils(A, shape):
    """Couplings of a translation-invariant level matrix (periodic grid, at
    least two slabs) read off one row block: diag[i, j, dy+1, dx+1] couples
    unknown (slab 1, node i, point (0, 0)) to (slab 1, node j, point (dy, dx))
    and sub[...] to the same point of slab 0.  Couplings beyond the 3 x 3
    neighbourhood are not returned (the tests check the row sums)."""
    N, M, ny, nx = shape
    A = sp.csr_matrix(A)
    P = nx * ny
    diag = np.zeros((M, M, 3, 3))
    sub = np.zeros((M, M, 3, 3))
    n = 1
    for i in range(M):
        row = A[n * M * P + i * P + 0]
        for j in range(M):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    x, y = dx % nx, dy % ny
                    diag[i, j, dy + 1, dx + 1] = row[0, n * M * P + j * P + y * nx + x]
                    sub[i, j, dy + 1, dx + 1] = row[0, (n - 1) * M * P + j * P + y * nx + x]
    return diag, sub

