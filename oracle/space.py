"""Second-order finite-difference Laplacian (Sec. 3).

The paper uses linear finite elements with a lumped mass matrix and
homogeneous Neumann conditions (Eq. spatial operators and the remark on the
lumped mass at the end of Sec. 3).  Dividing each row of K_h by the lumped
mass gives the central 3-point difference in the interior and, at the two
boundary nodes, the ghost-reflection formula 2(u_1 - u_0)/h^2.  The
periodic variant (same stencil, wrapped) is used by the synthetic
workloads.  Grids:
  periodic : n points per dimension, h = length / n, x_j = j h
  neumann  : n + 1 points per dimension, h = length / n, x_j = j h
Vectors are ordered [y][x] with x fastest; a 1D problem has ny = 1.
"""
import numpy as np
import scipy.sparse as sp


def npoints(n, bc):
    return n if bc == "periodic" else n + 1


def lap1d(n, h, bc):
    """Sparse 1D second difference (not yet divided by nothing else): D2 u / h^2."""
    m = npoints(n, bc)
    D = sp.lil_matrix((m, m))
    for j in range(m):
        if bc == "periodic":
            D[j, (j - 1) % m] += 1.0
            D[j, (j + 1) % m] += 1.0
            D[j, j] -= 2.0
        else:
            # ghost reflection: u_{-1} = u_1, u_{m} = u_{m-2}
            left = 1 if j == 0 else j - 1
            right = m - 2 if j == m - 1 else j + 1
            D[j, left] += 1.0
            D[j, right] += 1.0
            D[j, j] -= 2.0
    return (D.tocsr() / (h * h))


def laplacian(prob):
    """Delta_h for the problem's grid, as a sparse matrix on [y][x] vectors."""
    bc = prob["bc"]
    nx = prob["nx"][0]
    hx = prob["length"][0] / nx
    Dx = lap1d(nx, hx, bc)
    if prob["dim"] == 1:
        return Dx.tocsr()
    ny = prob["nx"][1]
    hy = prob["length"][1] / ny
    Dy = lap1d(ny, hy, bc)
    Ix = sp.identity(Dx.shape[0], format="csr")
    Iy = sp.identity(Dy.shape[0], format="csr")
    return (sp.kron(Iy, Dx) + sp.kron(Dy, Ix)).tocsr()


def grid_shape(prob):
    """(ny, nx) point counts of the spatial grid."""
    bc = prob["bc"]
    nx = npoints(prob["nx"][0], bc)
    ny = npoints(prob["nx"][1], bc) if prob["dim"] == 2 else 1
    return ny, nx


def linear_operator(prob):
    """L = nu * Delta_h - lambda * I  (the linear right-hand side f(u) = L u)."""
    D = laplacian(prob)
    return (prob["nu"] * D - prob.get("lambda", 0.0) * sp.identity(D.shape[0])).tocsr()
