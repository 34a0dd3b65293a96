"""The all-at-once DG space-time system (Eq. st_system) assembled literally.

Blocks (Eq. A_B_ops) with the lumped mass divided out of every spatial row
(so M_h -> I and K_h -> -nu Delta_h + lambda I, the FD-scaled form):
  A = K_q (x) I + M_q (x) (-nu Delta_h + lambda I)
  B = -J_q (x) I
and right-hand side -B u_0pad with u_0pad = [0, ..., 0, u0] (u0 in the last
node's slot, Sec. 3).  K_q, M_q = dt * Mq1, J_q come from their integral
definitions (Eqs. Kq, Mq) in oracle.radau -- not from Q.  Allen-Cahn adds
gamma (I (x) M_q (x) I) r(U) with r(u) = u^3 - u (Sec. 3), for the equation
u_t = nu Delta_h u + gamma (u - u^3).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import radau, space


def blocks(prob):
    t = radau.tables(prob["M"])
    dt = prob["dt"]
    D = space.laplacian(prob)
    I = sp.identity(D.shape[0], format="csr")
    K_h = -prob["nu"] * D + prob.get("lambda", 0.0) * I
    if prob.get("reaction", "linear") == "allen_cahn":
        K_h = -prob["nu"] * D
    Mq = dt * t["Mq1"]
    A = sp.kron(sp.csr_matrix(t["Kq"]), I) + sp.kron(sp.csr_matrix(Mq), K_h)
    B = -sp.kron(sp.csr_matrix(t["Jq"]), I)
    return A.tocsr(), B.tocsr(), Mq, t


def matrix(prob):
    """Sparse N*M*n x N*M*n matrix of the linear part of Eq. st_system."""
    A, B, _, _ = blocks(prob)
    N = prob["N"]
    main = sp.kron(sp.identity(N), A)
    sub = sp.kron(sp.diags([np.ones(N - 1)], [-1], shape=(N, N)), B)
    return (main + sub).tocsr()


def rhs(prob, u0):
    """-B u_0pad in the first slab, zero elsewhere."""
    _, B, _, _ = blocks(prob)
    M, N = prob["M"], prob["N"]
    u = np.asarray(u0, dtype=np.float64).reshape(-1)
    pad = np.zeros(M * u.size)
    pad[(M - 1) * u.size:] = u
    b = np.zeros(N * M * u.size)
    b[:M * u.size] = -(B @ pad)
    return b


def apply(prob, U):
    """Action of the all-at-once operator (Allen-Cahn: nonlinear) on U."""
    ny, nx = space.grid_shape(prob)
    v = np.asarray(U, dtype=np.float64).reshape(-1)
    out = matrix(prob) @ v
    if prob.get("reaction", "linear") == "allen_cahn":
        _, _, Mq, _ = blocks(prob)
        n = ny * nx
        N, M = prob["N"], prob["M"]
        Rm = sp.kron(sp.identity(N), sp.kron(sp.csr_matrix(Mq), sp.identity(n)))
        out = out + prob["gamma"] * (Rm @ (v ** 3 - v))
    return out.reshape(np.shape(U))


def residual(prob, u0, U):
    """b - A(U) for the all-at-once system, shape (N, M, ny, nx)."""
    return rhs(prob, u0).reshape(np.shape(U)) - apply(prob, U)


def residual_entry(prob, u0, U, n, i, y, x):
    """One entry of b - A(U), evaluated straight from the block definitions.

    Reads only the stencil neighbourhood of (y, x) in slabs n-1 and n, so it
    can be used on full-size arrays where assembling the matrix is too big.
    """
    t = radau.tables(prob["M"])
    M, dt, nu = prob["M"], prob["dt"], prob["nu"]
    lam = prob.get("lambda", 0.0)
    ac = prob.get("reaction", "linear") == "allen_cahn"
    bc = prob["bc"]
    ny, nx = space.grid_shape(prob)
    hx = prob["length"][0] / prob["nx"][0]
    hy = prob["length"][1] / prob["nx"][1] if prob["dim"] == 2 else 1.0

    def nb(j, m, d):
        if bc == "periodic":
            return (j + d) % m
        k = j + d
        if k < 0:
            return 1
        if k > m - 1:
            return m - 2
        return k

    def lap(V, yy, xx):
        s = (V[yy, nb(xx, nx, -1)] + V[yy, nb(xx, nx, 1)] - 2 * V[yy, xx]) / hx ** 2
        if prob["dim"] == 2:
            s += (V[nb(yy, ny, -1), xx] + V[nb(yy, ny, 1), xx] - 2 * V[yy, xx]) / hy ** 2
        return s

    acc = 0.0
    for j in range(M):
        Vj = U[n, j]
        acc += t["Kq"][i, j] * Vj[y, x]
        kh = -nu * lap(Vj, y, x) + (0.0 if ac else lam * Vj[y, x])
        acc += dt * t["Mq1"][i, j] * kh
        if ac:
            acc += prob["gamma"] * dt * t["Mq1"][i, j] * (Vj[y, x] ** 3 - Vj[y, x])
    prev = np.asarray(u0).reshape(ny, nx)[y, x]
    for j in range(M):
        if n == 0:
            pj = prev if j == M - 1 else 0.0
        else:
            pj = U[n - 1, j][y, x]
        acc -= t["Jq"][i, j] * pj
    b = 0.0  # the u0 term has been folded into the j loop above for n == 0
    return b - acc


def dense_solve(prob, u0, tol=1e-14, max_newton=50):
    """Brute-force solve of the whole system with dense linear algebra."""
    ny, nx = space.grid_shape(prob)
    shape = (prob["N"], prob["M"], ny, nx)
    Amat = matrix(prob).toarray()
    b = rhs(prob, u0)
    if prob.get("reaction", "linear") != "allen_cahn":
        return np.linalg.solve(Amat, b).reshape(shape)
    _, _, Mq, _ = blocks(prob)
    n = ny * nx
    Rm = np.kron(np.eye(prob["N"]), np.kron(Mq, np.eye(n)))
    g = prob["gamma"]
    v = np.zeros(b.size)
    for _ in range(max_newton):
        G = Amat @ v + g * (Rm @ (v ** 3 - v)) - b
        if np.abs(G).max() <= tol * max(1.0, np.abs(v).max()):
            return v.reshape(shape)
        J = Amat + g * (Rm * (3 * v ** 2 - 1)[None, :])
        v = v - np.linalg.solve(J, G)
    raise RuntimeError("dense Newton did not converge")


def residual_colloc(prob, u0, U):
    """Residual of the collocation form (Sec. 2.1, Eq. collocation), slab by
    slab: r_n = 1 (x) u_{n-1} + dt (Q (x) I) F(U_n) - U_n with u_{n-1} the
    previous slab's last stage (u0 for the first slab) and F(u) = nu Lap_h u -
    lambda u, or nu Lap_h u + gamma (u - u^3) for Allen-Cahn.  Built from Q
    and the spatial operator directly, not from the DG blocks."""
    t = radau.tables(prob["M"])
    Q, dt = t["Q"], prob["dt"]
    D = space.laplacian(prob)
    U = np.asarray(U, dtype=np.float64)
    N, M = U.shape[0], U.shape[1]
    n = D.shape[0]
    V = U.reshape(N, M, n)
    ac = prob.get("reaction", "linear") == "allen_cahn"
    r = np.zeros_like(V)
    prev = np.asarray(u0, dtype=np.float64).reshape(n)
    for k in range(N):
        F = np.array([prob["nu"] * (D @ V[k, j]) + (prob["gamma"] * (V[k, j] - V[k, j] ** 3) if ac
                                                     else -prob.get("lambda", 0.0) * V[k, j])
                      for j in range(M)])
        for m in range(M):
            r[k, m] = prev + dt * (Q[m] @ F) - V[k, m]
        prev = V[k, M - 1]
    return r.reshape(U.shape)

