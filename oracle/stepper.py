"""Sequential Radau IIA time stepping with a direct sparse solve per step.

This is the plain definition of the discrete solution: the collocation form
of Sec. 2.1 (Eq. collocation), U = U_0 + dt Q F(U), applied slab after slab
with U_0 = 1 (x) u_{n-1}, where u_{n-1} is the previous step's last stage
(t_M = T_{n+1}, so the method is stiffly accurate).  The paper states that
the DG form (Eq. DG_problem2) has the same solution at the nodes, and that
the all-at-once system (Eq. st_system) couples exactly these steps.

Stage vectors are ordered [m][y][x]; the result is an array of shape
(N, M, ny, nx) holding every stage value of every step.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import radau, space


def _stage_matrix(Q, L, dt):
    M = Q.shape[0]
    n = L.shape[0]
    return (sp.identity(M * n) - dt * sp.kron(sp.csr_matrix(Q), L)).tocsc()


def solve_linear(prob, u0):
    """All stage values for f(u) = nu Delta_h u - lambda u.  FP64."""
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    ny, nx = space.grid_shape(prob)
    Q = radau.tables(M)["Q"]
    L = space.linear_operator(prob)
    lu = spla.splu(_stage_matrix(Q, L, dt))
    U = np.zeros((N, M, ny, nx))
    u = np.asarray(u0, dtype=np.float64).reshape(-1)
    for n in range(N):
        Un = lu.solve(np.tile(u, M))
        U[n] = Un.reshape(M, ny, nx)
        u = Un[(M - 1) * u.size:]
    return U


def solve_allen_cahn(prob, u0, tol=1e-14, max_newton=50, reuse=False, log=None):
    """All stage values for f(u) = nu Delta_h u + gamma (u - u^3).

    Each step solves G(U) = U - 1(x)u_{n-1} - dt (Q(x)I) F(U) = 0 by Newton
    with Jacobian I - dt (Q(x)I)(I(x)nu Delta_h + diag(gamma (1 - 3U^2))),
    starting from 1(x)u_{n-1}; stop when max|G| <= tol * max(1, max|U|).
    By default the Jacobian is refactored at every Newton iteration.  With
    reuse=True one factorization is kept across iterations and steps and
    refactored at the current iterate only when an iteration reduces max|G|
    by less than a factor 0.3 (a chord iteration): the stop rule, and so the
    computed solution, are the same; only the work differs.  `log`, if given,
    is called as log(step, iterations, refactorizations so far).
    """
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    g = prob["gamma"]
    ny, nx = space.grid_shape(prob)
    Q = radau.tables(M)["Q"]
    D = prob["nu"] * space.laplacian(prob)
    QI = sp.kron(sp.csr_matrix(Q), sp.identity(D.shape[0]))
    ID = sp.kron(sp.identity(M), D)
    U = np.zeros((N, M, ny, nx))
    u = np.asarray(u0, dtype=np.float64).reshape(-1)

    def jacobian(V):
        return (sp.identity(V.size) - dt * (QI @ (ID + sp.diags(g * (1.0 - 3.0 * V ** 2))))).tocsc()

    lu = None
    factors = 0
    for n in range(N):
        U0 = np.tile(u, M)
        V = U0.copy()
        gprev = None
        for it in range(max_newton):
            F = ID @ V + g * (V - V ** 3)
            G = V - U0 - dt * (QI @ F)
            gn = np.abs(G).max()
            if gn <= tol * max(1.0, np.abs(V).max()):
                break
            if not reuse:
                V = V - spla.spsolve(jacobian(V), G)
                continue
            if lu is None or (gprev is not None and gn > 0.3 * gprev):
                lu = spla.splu(jacobian(V))
                factors += 1
            gprev = gn
            V = V - lu.solve(G)
        else:
            raise RuntimeError("oracle Newton did not converge at step %d" % n)
        if log is not None:
            log(n, it, factors)
        U[n] = V.reshape(M, ny, nx)
        u = V[(M - 1) * u.size:]
    return U


def solve(prob, u0):
    if prob.get("reaction", "linear") == "allen_cahn":
        return solve_allen_cahn(prob, u0)
    return solve_linear(prob, u0)
