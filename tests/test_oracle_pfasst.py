"""Pins of the oracle's PFASST (oracle/pfasst.py) against what fixes it
independently: the collocation solution of the stepper (its fixed point), and
one iteration written as linear two- and three-level multigrid with the
composite collocation matrices assembled block by block from Q and L."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import mg, pfasst, radau, space, stepper


def _u0(prob, seed=1):
    ny, nx = space.grid_shape(prob)
    return np.random.default_rng(seed).standard_normal((ny, nx))


@pytest.mark.parametrize("dim,bc,levels", [(1, "periodic", 2), (1, "neumann", 3), (2, "periodic", 2),
                                           (2, "periodic", 3), (2, "neumann", 2)])
def test_fixed_point_is_the_collocation_solution(dim, bc, levels):
    """PFASST converges to the Radau IIA stage values of the time stepper."""
    if dim == 1:
        prob = si.problem(1, 32, 3, 8, 0.2, nu=0.1, lam=0.5, bc=bc)
    else:
        prob = si.problem(2, 16, 2, 6, 0.3, nu=0.02, lam=1.0, bc=bc)
    u0 = _u0(prob)
    ref = stepper.solve_linear(prob, u0)
    hist = []
    U, its = pfasst.solve(prob, u0, levels=levels, rtol=1e-13, max_iter=60, history=hist)
    assert hist[-1] <= 1e-13, hist
    assert np.linalg.norm(U - ref) <= 1e-11 * np.linalg.norm(ref)
    # the collocation residual of the stepper's solution is at rounding level
    assert pfasst.rel_residual(pfasst.PLevel(prob), u0.reshape(ref.shape[2:]), ref) < 1e-13


# --- the same iteration as linear multigrid on assembled matrices -----------
def _transfer_matrices(lev, coarse_grid):
    """R_s and P_s of one level (to / from the next one) as dense matrices,
    by applying oracle.mg's transfer functions to unit vectors."""
    n = int(np.prod(lev.grid))
    nc = int(np.prod(coarse_grid))
    Rs = np.array([mg.restrict_space(np.eye(n)[j].reshape(lev.grid), lev.dim, lev.bc).reshape(-1)
                   for j in range(n)]).T
    Ps = np.array([mg.prolong_space(np.eye(nc)[j].reshape(coarse_grid), lev.dim, lev.bc).reshape(-1)
                   for j in range(nc)]).T
    assert Rs.shape == (nc, n) and Ps.shape == (n, nc)
    return Rs, Ps


def _composite(prob):
    """C = blocks I - dt Q (x) L on the diagonal, -(1 e_M^T) (x) I below."""
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    Q = radau.tables(M)["Q"]
    L = space.linear_operator(prob).toarray()
    n = L.shape[0]
    D = np.eye(M * n) - dt * np.kron(Q, L)
    S = -np.kron(np.outer(np.ones(M), np.eye(M)[M - 1]), np.eye(n))
    A = np.kron(np.eye(N), D) + np.kron(np.eye(N, k=-1), S)
    return A


def _jacobi(prob):
    """Block diagonal of I - dt Q_Delta (x) L, Q_Delta[m][j] = c_j - c_{j-1} (j <= m)."""
    M, N, dt = prob["M"], prob["N"], prob["dt"]
    c = radau.tables(M)["c"]
    dc = np.diff(np.concatenate([[0.0], c]))
    QD = np.tril(np.tile(dc, (M, 1)))
    L = space.linear_operator(prob).toarray()
    n = L.shape[0]
    return np.kron(np.eye(N), np.eye(M * n) - dt * np.kron(QD, L))


def _transfers(levf, levc, prob_f):
    """Space-time R (end node, R_s) and P (linear in time from the previous
    slab's end, P_s) between a level and the next."""
    M, N = prob_f["M"], prob_f["N"]
    c = radau.tables(M)["c"]
    Rs, Ps = _transfer_matrices(levf, levc.grid)
    R = np.kron(np.eye(N), np.kron(np.eye(M)[M - 1][None, :], Rs))
    T = np.zeros((N * M, N))
    for k in range(N):
        for i in range(M):
            T[k * M + i, k] = c[i]
            if k > 0:
                T[k * M + i, k - 1] = 1.0 - c[i]
    return R, np.kron(T, Ps)


@pytest.mark.parametrize("dim,bc", [(1, "periodic"), (1, "neumann"), (2, "periodic")])
def test_one_iteration_is_two_level_multigrid(dim, bc):
    """x_s = x + B^-1 (b - C x) (Jacobi SDC sweep); x' = x_s + P C_c^-1 R (b - C x_s)."""
    prob = si.problem(1, 8, 3, 3, 0.3, nu=0.1, lam=0.4, bc=bc) if dim == 1 else \
        si.problem(2, 4, 2, 2, 0.3, nu=0.05, lam=0.7)
    levs = pfasst.hierarchy(prob, 2)
    u0 = _u0(prob, 3)
    u0s = pfasst.initial_values(levs, u0)
    x = np.random.default_rng(4).standard_normal(levs[0].shape)
    got = pfasst.iteration(levs, u0s, x, nu=1).reshape(-1)
    A0 = _composite(prob)
    A1 = _composite(levs[1].prob)
    n = u0.size
    b = np.zeros(A0.shape[0])
    b[:prob["M"] * n] = np.tile(u0.reshape(-1), prob["M"])
    B = _jacobi(prob)
    R, P = _transfers(levs[0], levs[1], prob)
    xs = x.reshape(-1) + np.linalg.solve(B, b - A0 @ x.reshape(-1))
    want = xs + P @ np.linalg.solve(A1, R @ (b - A0 @ xs))
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_one_iteration_is_three_level_multigrid():
    """Level 1 (M = 1): Jacobi sweep, exact level-2 correction, Jacobi sweep,
    on A_1 y = R (b - A_0 x_s) + A_1 y0 with y0 = R~ x_s."""
    prob = si.problem(1, 16, 2, 3, 0.3, nu=0.2, lam=0.3)
    levs = pfasst.hierarchy(prob, 3)
    u0 = _u0(prob, 5)
    u0s = pfasst.initial_values(levs, u0)
    x = np.random.default_rng(6).standard_normal(levs[0].shape)
    got = pfasst.iteration(levs, u0s, x, nu=1).reshape(-1)
    p1, p2 = levs[1].prob, levs[2].prob
    A0, A1, A2 = _composite(prob), _composite(p1), _composite(p2)
    B0, B1 = _jacobi(prob), _jacobi(p1)
    R0, P0 = _transfers(levs[0], levs[1], prob)
    R1, P1 = _transfers(levs[1], levs[2], p1)
    n = u0.size
    b = np.zeros(A0.shape[0])
    b[:prob["M"] * n] = np.tile(u0.reshape(-1), prob["M"])
    xs = x.reshape(-1) + np.linalg.solve(B0, b - A0 @ x.reshape(-1))
    y0 = R0 @ xs  # R~ x_s: the end node restricted, the same matrix as R
    bt = R0 @ (b - A0 @ xs) + A1 @ y0
    ys = y0 + np.linalg.solve(B1, bt - A1 @ y0)
    yc = ys + P1 @ np.linalg.solve(A2, R1 @ (bt - A1 @ ys))
    yf = yc + np.linalg.solve(B1, bt - A1 @ yc)
    want = xs + P0 @ (yf - y0)
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_coarse_serial_sweep_is_backward_euler():
    """At M = 1 the serial sweep with tau = 0 is backward Euler on the level's
    grid (u_n = (I - dt L)^-1 u_{n-1}), whatever the incoming iterate."""
    prob = pfasst.coarse_problem(si.problem(1, 32, 3, 5, 0.2, nu=0.3, lam=0.1))
    lev = pfasst.PLevel(prob)
    u0 = _u0(prob, 7)
    V = np.random.default_rng(8).standard_normal(lev.shape)
    got = lev.sweep(V, u0, np.zeros(lev.shape), serial=True)
    L = space.linear_operator(prob).toarray()
    u = u0.reshape(-1)
    for k in range(prob["N"]):
        u = np.linalg.solve(np.eye(L.shape[0]) - prob["dt"] * L, u)
        assert np.abs(got[k, 0].reshape(-1) - u).max() <= 1e-13 * max(1.0, np.abs(u).max())


# --- Allen-Cahn: the IMEX sweep ---------------------------------------------
@pytest.mark.parametrize("dim,levels", [(1, 2), (1, 3), (2, 2), (2, 3)])
def test_imex_pfasst_reaches_the_implicit_collocation_solution(dim, levels):
    """With the reaction explicit in the sweeps, PFASST still converges to the
    fully implicit Radau IIA solution of the Allen-Cahn problem (the time
    stepper with Newton per step)."""
    if dim == 1:
        prob = si.problem(1, 32, 3, 8, 0.4, nu=0.05, gamma=1.0, reaction="allen_cahn")
    else:
        prob = si.problem(2, 16, 2, 6, 0.3, nu=0.02, gamma=1.0, reaction="allen_cahn")
    u0 = 0.8 * np.tanh(_u0(prob, 11))
    ref = stepper.solve_allen_cahn(prob, u0)
    hist = []
    U, its = pfasst.solve(prob, u0, levels=levels, rtol=1e-13, max_iter=80, history=hist)
    assert hist[-1] <= 1e-13, hist[-5:]
    assert np.linalg.norm(U - ref) <= 1e-11 * np.linalg.norm(ref)


@pytest.mark.parametrize("serial", [False, True])
def test_imex_sweep_solves_its_defining_equation(serial):
    """One IMEX sweep V -> V' satisfies, slab by slab (u_0 the slab's initial
    value in the sweep, u_0^old the incoming one),
      V' = 1 u_0 + dt Q_I L V' + dt Q_E R([u_0; V'])
           + dt (Q F(V) - Q_I L V - Q_E R([u_0^old; V])) + tau
    with Q_I = implicit Euler (lower triangular, dc_j for j <= m) and Q_E the
    M x (M+1) explicit Euler matrix (dc_{j+1} for j < m, column 0 the initial
    value), written here with dense Kronecker products."""
    prob = si.problem(1, 16, 3, 4, 0.5, nu=0.1, gamma=2.0, reaction="allen_cahn")
    lev = pfasst.PLevel(prob)
    rng = np.random.default_rng(12)
    u0 = 0.7 * np.tanh(rng.standard_normal(lev.grid))
    V = 0.7 * np.tanh(rng.standard_normal(lev.shape))
    tau = 0.01 * rng.standard_normal(lev.shape)
    out = lev.sweep(V, u0, tau, serial=serial)
    M, dt, n = lev.M, lev.dt, int(np.prod(lev.grid))
    c = radau.tables(M)["c"]
    cc = np.concatenate([[0.0], c])
    QI = np.array([[cc[j + 1] - cc[j] if j <= m else 0.0 for j in range(M)] for m in range(M)])
    QE = np.array([[cc[j + 1] - cc[j] if j <= m else 0.0 for j in range(M + 1)] for m in range(M)])
    Q = radau.tables(M)["Q"]
    L = space.linear_operator(prob).toarray()
    R = lambda v: prob["gamma"] * (v - v ** 3)
    for k in range(prob["N"]):
        u_old = (u0 if k == 0 else V[k - 1, M - 1]).reshape(n)
        u_new = (u0 if k == 0 else (out if serial else V)[k - 1, M - 1]).reshape(n)
        Vk, Wk = V[k].reshape(M, n), out[k].reshape(M, n)
        FV = Vk @ L.T + R(Vk)
        ext_new = np.vstack([u_new, Wk])
        ext_old = np.vstack([u_old, Vk])
        rhs = (np.tile(u_new, (M, 1)) + dt * QI @ (Wk @ L.T) + dt * QE @ R(ext_new)
               + dt * (Q @ FV - QI @ (Vk @ L.T) - QE @ R(ext_old)) + tau[k].reshape(M, n))
        assert np.abs(Wk - rhs).max() <= 1e-12 * max(1.0, np.abs(Wk).max())
