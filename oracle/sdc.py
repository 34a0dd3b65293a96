"""SDC sweeps on the collocation form (Sec. 2.1 and Sec. 4.1), plain NumPy.

One sweep is one step of the preconditioned Richardson iteration on the
collocation problem U_n = 1 (x) u_{n-1} + dt (Q (x) I) F(U_n) of every slab,
with the implicit-Euler lower-triangular Q_Delta (Q_Delta[m][j] = c_j - c_{j-1}
for j <= m, c_0 = 0).  All slabs are swept at once with the previous slab's
end value taken from the incoming iterate (Jacobi across slabs), u_{-1} = u0:

  r_n     = 1 (x) u_{n-1} + dt (Q (x) L) U_n - U_n          (collocation residual)
  (I - dt dc_m L) delta_m = r_{n,m} + dt sum_{j<m} dc_j L delta_j,   m = 1..M
  U_n    <- U_n + delta

Linear problems (F = L U, L = nu Lap - lambda).  Spatial solves are direct.
The paper does not give Q_Delta; implicit Euler is the standard choice of the
SISDC method it cites.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import radau, space


def sweep(prob, u0, U):
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    t = radau.tables(M)
    c, Q = t["c"], t["Q"]
    dc = np.diff(np.concatenate([[0.0], c]))
    L = space.linear_operator(prob)
    n = L.shape[0]
    I = sp.identity(n, format="csc")
    solvers = [spla.splu((I - dt * dc[m] * L).tocsc()) for m in range(M)]
    V = np.asarray(U, dtype=np.float64).reshape(N, M, n)
    out = V.copy()
    u_prev = np.asarray(u0, dtype=np.float64).reshape(n)
    for k in range(N):
        prev = u_prev if k == 0 else V[k - 1, M - 1]
        LU = np.array([L @ V[k, j] for j in range(M)])
        acc = np.zeros(n)
        for m in range(M):
            r = prev + dt * (Q[m] @ LU) - V[k, m]
            d = solvers[m].solve(r + acc)
            acc = acc + dt * dc[m] * (L @ d)
            out[k, m] = V[k, m] + d
    return out.reshape(np.shape(U))
