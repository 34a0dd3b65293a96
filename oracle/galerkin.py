"""Assembled multigrid: the oracle's transfers as sparse matrices and
Galerkin coarse operators A_{l+1} = R_l A_l P_l, for comparing the
rediscretized coarse levels with the paper's Galerkin ones (Sec. 4.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Vectors are ordered [N][M][ny][nx] as everywhere in the oracle, so a
transfer that coarsens time, nodes and space is the Kronecker product
P = P_t (x) P_m (x) P_s of the one-dimensional factors of oracle.mg (1D
grids):
  space  P_s[2X, X] = 1, P_s[2X+1, X] = P_s[2X+1, X+1] = 1/2 (periodic),
         R_s = P_s^T / 2;
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
    """(P, R) between two consecutive 1D levels of oracle.mg.hierarchy."""
    assert fine.dim == 1
    Ps = _space_p(coarse.nx) if "s" in kind else sp.identity(fine.nx, format="csr")
    Rs = 0.5 * Ps.T if "s" in kind else Ps
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
