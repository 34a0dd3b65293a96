"""Oracle pins: the sequential Radau IIA stepper against closed forms, the
paper's heat example, and a brute-force dense solve of the all-at-once
system."""
import json
import os

import numpy as np
import pytest

import stmg_inputs as si
from oracle import adjoint, allatonce, fourier, radau, space, stepper

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_heat_table.json")


def test_stepper_vs_fourier_1d():
    prob = si.config("heat1d")
    u0 = si.initial("heat1d", prob)
    U = stepper.solve_linear(prob, u0)
    V = fourier.solve_linear_periodic(prob, u0)
    assert np.abs(U - V).max() <= 1e-13 * np.abs(V).max()


@pytest.mark.parametrize("M", [1, 3, 4])
def test_stepper_vs_fourier_2d(M):
    prob = si.problem(2, 32, M, 8, 0.5, nu=1e-2, lam=1.0)
    u0 = si.u0_rd2d(prob, 7)
    U = stepper.solve_linear(prob, u0)
    V = fourier.solve_linear_periodic(prob, u0)
    assert np.abs(U - V).max() <= 1e-13 * np.abs(V).max()


def test_fourier_vs_stability_function_single_mode():
    """A single Fourier mode of the heat equation is multiplied by R(dt sigma_k) per step."""
    prob = si.problem(1, 64, 3, 10, 0.2, nu=1.0, lam=0.0)
    X, _ = si.coords(prob)
    k = 5
    u0 = np.cos(2 * np.pi * k * X)
    h = 1.0 / 64
    sig = -4.0 / h ** 2 * np.sin(np.pi * k * h) ** 2
    R = radau.stability_function(radau.tables(3)["Q"], prob["dt"] * sig)
    U = stepper.solve_linear(prob, u0)
    assert np.abs(U[-1, -1] - R ** 10 * u0).max() < 1e-14


def test_mean_and_norm():
    prob = si.config("heat1d")
    u0 = si.initial("heat1d", prob)
    U = stepper.solve_linear(prob, u0)
    m0 = u0.mean()
    for n in range(prob["N"]):
        assert abs(U[n, -1].mean() - m0) < 1e-14
    norms = [np.linalg.norm(u0)] + [np.linalg.norm(U[n, -1]) for n in range(prob["N"])]
    assert all(b <= a + 1e-14 for a, b in zip(norms, norms[1:]))
    # with lambda > 0 the mean decays by R(-dt lambda) per step
    p2 = si.problem(1, 16, 2, 5, 1.0, nu=0.3, lam=2.0)
    u = np.ones((1, 16))
    U2 = stepper.solve_linear(p2, u)
    R = radau.stability_function(radau.tables(2)["Q"], -p2["dt"] * 2.0)
    assert abs(U2[-1, -1].mean() - R ** 5) < 1e-14


@pytest.mark.parametrize("M", [1, 2, 3])
@pytest.mark.parametrize("dim", [1, 2])
def test_dense_allatonce_equals_stepper(M, dim):
    nx = 12 if dim == 1 else 6
    prob = si.problem(dim, nx, M, 5, 0.3, nu=0.05, lam=0.7)
    rng = np.random.default_rng(3)
    ny, nxp = si.grid_points(prob)
    u0 = rng.standard_normal((ny, nxp))
    U = stepper.solve_linear(prob, u0)
    V = allatonce.dense_solve(prob, u0)
    assert np.abs(U - V).max() <= 1e-13 * np.abs(V).max()
    r = allatonce.residual(prob, u0, U)
    assert np.abs(r).max() < 1e-13


def test_dense_allatonce_neumann():
    prob = si.problem(1, 10, 3, 4, 0.2, nu=1.0, lam=0.0, bc="neumann")
    u0 = np.random.default_rng(0).standard_normal((1, 11))
    U = stepper.solve_linear(prob, u0)
    V = allatonce.dense_solve(prob, u0)
    assert np.abs(U - V).max() <= 1e-13 * np.abs(V).max()


def test_residual_entry_matches_matrix():
    prob = si.problem(2, 6, 3, 3, 0.3, nu=0.1, lam=0.5)
    rng = np.random.default_rng(1)
    U = rng.standard_normal((3, 3, 6, 6))
    u0 = rng.standard_normal((6, 6))
    R = allatonce.residual(prob, u0, U)
    for (n, i, y, x) in [(0, 0, 0, 0), (0, 2, 5, 3), (1, 1, 2, 5), (2, 2, 0, 5), (2, 0, 3, 3)]:
        assert abs(allatonce.residual_entry(prob, u0, U, n, i, y, x) - R[n, i, y, x]) < 1e-13
    pa = dict(prob, reaction="allen_cahn", gamma=2.0)
    R = allatonce.residual(pa, u0, U)
    for (n, i, y, x) in [(0, 1, 1, 1), (2, 2, 4, 0)]:
        assert abs(allatonce.residual_entry(pa, u0, U, n, i, y, x) - R[n, i, y, x]) < 1e-12


def _paper_heat(M, Nt):
    g = json.load(open(GOLD))
    prob = si.problem(1, g["Nx"], M, Nt, 1.0, nu=1.0, bc="neumann")
    x = np.arange(g["Nx"] + 1) / g["Nx"]
    u0 = np.cos(np.pi * x) + 2 * np.cos(3 * np.pi * x) + 3 * np.cos(4 * np.pi * x)
    U = stepper.solve_linear(prob, u0[None])
    exact = (np.cos(np.pi * x) * np.exp(-np.pi ** 2) + 2 * np.cos(3 * np.pi * x) * np.exp(-9 * np.pi ** 2)
             + 3 * np.cos(4 * np.pi * x) * np.exp(-16 * np.pi ** 2))
    return np.abs(U[-1, -1, 0] - exact).max()


@pytest.mark.parametrize("M", [2, 3, 4, 5])
def test_paper_minimal_nt(M):
    """Sec. 5.3: the minimal power-of-two N_t with error < 1e-9 is the table header."""
    g = json.load(open(GOLD))
    nt = g["nt_by_M"][str(M)]
    assert _paper_heat(M, nt) < g["tol"]
    assert _paper_heat(M, nt // 2) >= g["tol"]


def test_paper_m1_and_spatial_error():
    g = json.load(open(GOLD))
    e1 = _paper_heat(1, g["M1"]["Nt"])
    assert 0.1 * g["M1"]["err_order_of_magnitude"] < e1 < 10 * g["M1"]["err_order_of_magnitude"]
    # semi-discrete solution (Eq. an_sol2) vs analytic (Eq. an_sol): spatial error
    h = 1.0 / g["Nx"]
    x = np.arange(g["Nx"] + 1) * h
    rho = lambda k: (2 * np.cos(k * np.pi * h) - 2) / h ** 2
    ut = (np.cos(np.pi * x) * np.exp(rho(1)) + 2 * np.cos(3 * np.pi * x) * np.exp(rho(3))
          + 3 * np.cos(4 * np.pi * x) * np.exp(rho(4)))
    ua = (np.cos(np.pi * x) * np.exp(-np.pi ** 2) + 2 * np.cos(3 * np.pi * x) * np.exp(-9 * np.pi ** 2)
          + 3 * np.cos(4 * np.pi * x) * np.exp(-16 * np.pi ** 2))
    es = np.abs(ut - ua).max()
    assert 0.1 * g["spatial_error_order_of_magnitude"] < es < 10 * g["spatial_error_order_of_magnitude"]


@pytest.mark.parametrize("M", [2, 3])
def test_order_semidiscrete(M):
    """Sec. 5.3 / Fig. accuracy: temporal error vs the semi-discrete solution has order 2M-1."""
    nx = 64
    h = 1.0 / nx
    x = np.arange(nx + 1) * h
    errs = []
    Ns = [4, 8, 16]
    for Nt in Ns:
        prob = si.problem(1, nx, M, Nt, 1.0, nu=1.0, bc="neumann")
        u0 = np.cos(np.pi * x) + 2 * np.cos(3 * np.pi * x)
        U = stepper.solve_linear(prob, u0[None])
        rho = lambda k: (2 * np.cos(k * np.pi * h) - 2) / h ** 2
        ut = np.cos(np.pi * x) * np.exp(rho(1)) + 2 * np.cos(3 * np.pi * x) * np.exp(rho(3))
        errs.append(np.abs(U[-1, -1, 0] - ut).max())
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(slopes[-1] - (2 * M - 1)) < 0.25, slopes


def _ac_exact(u0, g, t):
    return u0 * np.exp(g * t) / np.sqrt(1 + u0 ** 2 * (np.exp(2 * g * t) - 1))


@pytest.mark.parametrize("reuse", [False, True])
@pytest.mark.parametrize("M", [2, 3])
def test_allen_cahn_uniform_order(M, reuse):
    """Spatially uniform u0 reduces u_t = nu Lap u + g (u - u^3) to a logistic-type ODE
    (with and without reuse of the Jacobian's factorization)."""
    errs = []
    Ns = [4, 8, 16]
    for Nt in Ns:
        prob = si.problem(1, 8, M, Nt, 1.0, nu=0.1, gamma=2.0, reaction="allen_cahn")
        U = stepper.solve_allen_cahn(prob, np.full((1, 8), 0.3), reuse=reuse)
        errs.append(abs(U[-1, -1, 0, 3] - _ac_exact(0.3, 2.0, 1.0)))
        assert np.ptp(U[-1, -1]) < 1e-14
    slopes = [np.log2(errs[i] / errs[i + 1]) for i in range(len(errs) - 1)]
    assert abs(slopes[-1] - (2 * M - 1)) < 0.3, slopes


@pytest.mark.parametrize("reuse", [False, True])
def test_allen_cahn_fixed_points_and_dense(reuse):
    prob = si.problem(2, 4, 2, 3, 0.3, nu=0.05, gamma=3.0, reaction="allen_cahn")
    for c in (0.0, 1.0, -1.0):
        U = stepper.solve_allen_cahn(prob, np.full((4, 4), c), reuse=reuse)
        assert np.abs(U - c).max() < 1e-15
    u0 = np.random.default_rng(2).uniform(-0.8, 0.8, (4, 4))
    U = stepper.solve_allen_cahn(prob, u0, reuse=reuse)
    V = allatonce.dense_solve(prob, u0)
    assert np.abs(U - V).max() < 1e-13
    assert np.abs(allatonce.residual(prob, u0, U)).max() < 1e-13


def test_fourier_end_value_matches_stepper():
    prob = si.problem(2, 16, 3, 7, 0.4, nu=0.02, lam=0.6)
    u0 = si.u0_rd2d(prob, 3)
    U = stepper.solve_linear(prob, u0)
    assert np.abs(fourier.end_value_periodic(prob, u0) - U[-1, -1]).max() <= 1e-13 * np.abs(U).max()


def test_allen_cahn_jacobian_reuse_same_solution():
    """Keeping one factorization across Newton iterations and steps (chord
    iteration, refactored when the contraction is weaker than 0.3) stops on the
    same residual test, so the trajectory agrees with full Newton to rounding;
    here with fewer factorizations than steps."""
    prob = si.problem(2, 16, 3, 12, 0.6, nu=1e-3, gamma=1.0, reaction="allen_cahn")
    u0 = np.random.default_rng(7).uniform(-0.1, 0.1, (16, 16))
    seen = []
    Ur = stepper.solve_allen_cahn(prob, u0, reuse=True, log=lambda n, it, f: seen.append(f))
    Uf = stepper.solve_allen_cahn(prob, u0)
    assert np.abs(Ur - Uf).max() <= 1e-13
    assert seen[-1] < prob["N"]
