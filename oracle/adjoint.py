"""Discrete adjoint of the sequential Radau IIA stepper (linear problems).

Forward (collocation form, Sec. 2.1): S U_n = 1 (x) u_{n-1}, with
S = I - dt (Q (x) L), L = nu Delta_h - lambda I and u_n = (e_M^T (x) I) U_n.
Loss L = || u_N - u_tgt ||^2.  Lagrange multipliers, backward in time:
  mu_N = S^{-T} (e_M (x) g),             g = 2 (u_N - u_tgt)
  mu_n = S^{-T} (e_M (x) (1^T (x) I) mu_{n+1})
Gradients:
  dL/du0 = (1^T (x) I) mu_1
  dL/dnu = sum_n mu_n^T (dt Q (x) Delta_h) U_n     (since dS/dnu = -dt Q (x) Delta_h)
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import radau, space, stepper


def loss(prob, U, u_tgt):
    d = U[-1, -1] - np.asarray(u_tgt).reshape(U.shape[2:])
    return float(np.sum(d * d))


def gradients(prob, u0, u_tgt, U=None):
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    if U is None:
        U = stepper.solve_linear(prob, u0)
    Q = radau.tables(M)["Q"]
    D = space.laplacian(prob)
    L = space.linear_operator(prob)
    S = (sp.identity(M * L.shape[0]) - dt * sp.kron(sp.csr_matrix(Q), L)).tocsc()
    lu = spla.splu(S)
    n = L.shape[0]
    QD = sp.kron(sp.csr_matrix(Q), D).tocsr()
    g = 2.0 * (U[-1, -1].reshape(-1) - np.asarray(u_tgt).reshape(-1))
    rhs = np.zeros(M * n)
    rhs[(M - 1) * n:] = g
    dnu = 0.0
    mu = None
    for k in range(N - 1, -1, -1):
        mu = lu.solve(rhs, trans="T")
        dnu += float(mu @ (dt * (QD @ U[k].reshape(-1))))
        s = mu.reshape(M, n).sum(axis=0)
        rhs = np.zeros(M * n)
        rhs[(M - 1) * n:] = s
    du0 = mu.reshape(M, n).sum(axis=0)
    return du0.reshape(U.shape[2:]), dnu
