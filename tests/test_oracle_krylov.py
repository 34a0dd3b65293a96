"""Pins for the oracle's flexible GMRES: finite termination, the minimal
residual over the search space it built (checked by brute-force least
squares over the recorded directions and over an explicit Krylov basis),
one step with the exact inverse, monotone restarts, and the all-at-once
solve reaching the dense solution."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import allatonce, krylov, mg


def _system(n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 2.0 * np.eye(n)
    b = rng.standard_normal(n)
    return A, b


def test_finite_termination():
    # with no preconditioner, n steps span R^n: the exact solution
    A, b = _system(12, 0)
    x, hist, steps = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=12, rtol=0.0, max_steps=12)
    assert steps == 12
    ref = np.linalg.solve(A, b)
    assert np.abs(x - ref).max() <= 1e-10 * np.abs(ref).max()
    assert hist[-1] <= 1e-12


def test_exact_preconditioner_one_step():
    A, b = _system(20, 1)
    Ainv = np.linalg.inv(A)
    x, hist, steps = krylov.fgmres(lambda v: A @ v, lambda v: Ainv @ v, b, restart=5, rtol=1e-12)
    assert steps == 1
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)


@pytest.mark.parametrize("k", [1, 3, 6])
def test_minimal_residual_over_recorded_directions(k):
    # a preconditioner that changes every call (two alternating matrices);
    # the update must minimise ||b - A x|| over x0 + span of the directions
    # the preconditioner returned
    rng = np.random.default_rng(2)
    n = 30
    A, b = _system(n, 3)
    P = [np.eye(n) + 0.3 * rng.standard_normal((n, n)) / np.sqrt(n) for _ in range(2)]
    x0 = rng.standard_normal(n)
    Z = []

    def pre(v):
        z = P[len(Z) % 2] @ v
        Z.append(z)
        return z

    x, hist, steps = krylov.fgmres(lambda v: A @ v, pre, b, x0=x0, restart=10, rtol=0.0, max_steps=k)
    assert steps == k and len(Z) == k
    Zm = np.stack(Z, axis=1)
    y = np.linalg.lstsq(A @ Zm, b - A @ x0, rcond=None)[0]
    xs = x0 + Zm @ y
    assert np.abs(x - xs).max() <= 1e-10 * np.abs(xs).max()
    assert abs(hist[-1] - np.linalg.norm(b - A @ xs) / np.linalg.norm(b)) <= 1e-12


@pytest.mark.parametrize("k", [2, 5])
def test_search_space_is_preconditioned_krylov_space(k):
    # a fixed preconditioner P: the search space is P K_k(A P, r0), spanned
    # here by explicit powers (no orthogonalisation)
    rng = np.random.default_rng(4)
    n = 25
    A, b = _system(n, 5)
    P = np.eye(n) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    x, _, _ = krylov.fgmres(lambda v: A @ v, lambda v: P @ v, b, restart=10, rtol=0.0, max_steps=k)
    cols = [b]
    for _ in range(k - 1):
        cols.append(A @ (P @ cols[-1]))
    S = P @ np.stack(cols, axis=1)
    y = np.linalg.lstsq(A @ S, b, rcond=None)[0]
    xs = S @ y
    assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()


def test_least_squares_estimate_is_true_residual():
    # the Hessenberg least-squares residual after k steps equals ||b - A x_k||
    A, b = _system(40, 6)
    _, hist, _ = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=30, rtol=0.0, max_steps=8)
    for k in range(1, 8):
        x, hk, _ = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=30, rtol=0.0, max_steps=k)
        true = np.linalg.norm(b - A @ x) / np.linalg.norm(b)
        assert abs(hk[-1] - true) <= 1e-13
        assert abs(hist[k] - true) <= 1e-12 * max(true, 1e-3)


def test_restarts_monotone():
    A, b = _system(60, 7)
    x, hist, steps = krylov.fgmres(lambda v: A @ v, lambda v: v, b, restart=3, rtol=1e-10, max_steps=300)
    assert hist[-1] <= 1e-10
    assert all(hist[i + 1] <= hist[i] * (1 + 1e-12) for i in range(len(hist) - 1))
    assert np.linalg.norm(b - A @ x) <= 1e-10 * np.linalg.norm(b)


@pytest.mark.parametrize("coarsen,restart", [("space", 10), ("spacetime", 30), ("smmg", 10)])
def test_vcycle_preconditioned_solve(coarsen, restart):
    # FGMRES around the V-cycle reaches the dense all-at-once solution in
    # fewer steps than the plain V-cycle iteration takes to the same
    # tolerance; with full space-time coarsening at mu = 64 the plain
    # iteration diverges while the Krylov method still converges
    prob = si.problem(1, 32, 3, 8, 0.5, nu=1.0)
    u0 = si.u0_heat1d(prob)
    kw = dict(coarsen=coarsen, fft_coarse=0, min_coarse=16)
    U, hist, steps = krylov.solve(prob, u0, rtol=1e-10, restart=restart, max_steps=300, **kw)
    ref = allatonce.dense_solve(prob, u0)
    assert hist[-1] <= 1e-10
    assert np.abs(U - ref).max() <= 1e-8 * np.abs(ref).max()
    _, vh = mg.solve(prob, u0, rtol=1e-10, max_cycles=300, **kw)
    if coarsen == "spacetime":
        assert not vh[-1] <= 1e-10
    else:
        assert vh[-1] <= 1e-10
        assert steps < len(vh)


@pytest.mark.parametrize("k", [2, 4])
def test_left_preconditioned_minimises_preconditioned_residual(k):
    # GMRES on P A x = P b: after k steps x minimises ||P (b - A x)|| over
    # K_k(P A, P b), spanned here by explicit powers
    rng = np.random.default_rng(8)
    n = 25
    A, b = _system(n, 9)
    P = np.eye(n) + 0.2 * rng.standard_normal((n, n)) / np.sqrt(n)
    x, hist, _ = krylov.fgmres(lambda v: P @ (A @ v), lambda v: v, P @ b, restart=10, rtol=0.0, max_steps=k)
    cols = [P @ b]
    for _ in range(k - 1):
        cols.append(P @ (A @ cols[-1]))
    S = np.stack(cols, axis=1)
    y = np.linalg.lstsq(P @ A @ S, P @ b, rcond=None)[0]
    xs = S @ y
    assert np.abs(x - xs).max() <= 1e-9 * np.abs(xs).max()
    assert abs(hist[-1] - np.linalg.norm(P @ (b - A @ xs)) / np.linalg.norm(P @ b)) <= 1e-12


def test_left_preconditioned_vcycle_solve():
    prob = si.problem(1, 32, 3, 8, 0.5, nu=1.0)
    u0 = si.u0_heat1d(prob)
    kw = dict(coarsen="space", fft_coarse=0, min_coarse=16)
    U, hist, steps = krylov.solve(prob, u0, rtol=1e-11, restart=10, left=True, **kw)
    ref = allatonce.dense_solve(prob, u0)
    assert hist[-1] <= 1e-11
    assert np.abs(U - ref).max() <= 1e-8 * np.abs(ref).max()
