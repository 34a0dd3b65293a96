"""Flexible GMRES around the V-cycle (option krylov = restart length) against
the oracle's FGMRES step by step, and on the paper's 1D workloads."""
import json
import os

import numpy as np
import pytest

import stmg_inputs as si
from oracle import adjoint, fourier, krylov, stepper

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, assert_close, rel_err  # noqa: E402

GOLD = os.path.join(os.path.dirname(__file__), "golden", "paper_heat_table.json")
SMALL = si.problem(1, 32, 3, 8, 0.5, nu=1.0)
HIER = dict(fft_coarse=0, min_coarse=16)


@pytest.mark.parametrize("coarsen", ["space", "smmg", "spacetime"])
@pytest.mark.parametrize("k", [1, 2, 4, 7, 12])
def test_fgmres_steps_match_oracle(coarsen, k):
    """After k Krylov steps (restart 5, so k = 7 and 12 cross restarts) the
    iterate and its residual match the oracle's FGMRES."""
    print("case fgmres steps", coarsen, k, flush=True)
    u0 = si.u0_heat1d(SMALL)
    ref, hist, steps = krylov.solve(SMALL, u0, rtol=0.0, restart=5, max_steps=k, coarsen=coarsen, **HIER)
    assert steps == k
    h = H(SMALL, coarsen=coarsen, krylov=5, max_cycles=k, rtol=1e-30, **HIER)
    U, st = h.solve(T(u0), check=False)
    assert st["cycles"] == k and st["status"] == -4
    assert_close(U.cpu().numpy(), ref, 1e-9, "iterate after %d steps" % k)
    assert abs(st["rel_res"] - hist[-1]) <= 1e-7 * hist[-1] + 1e-14, (st["rel_res"], hist[-1])


@pytest.mark.parametrize("restart", [1, 3, 10, 32])
def test_fgmres_converges_to_stepper(restart):
    print("case fgmres restart", restart, flush=True)
    prob = si.problem(2, 64, 3, 32, 0.5, nu=1e-2, lam=1.0)
    u0 = si.u0_rd2d(prob, 2)
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, krylov=restart).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= 1e-12
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10
    _, plain = H(prob).solve(T(u0))
    if restart >= 3:
        assert st["cycles"] < plain["cycles"], (st["cycles"], plain["cycles"])


def test_fgmres_spacetime_where_vcycles_diverge():
    """Full space-time coarsening at mu = 64: the plain iteration diverges,
    FGMRES(30) around the same cycle converges to the stepper's solution."""
    print("case fgmres spacetime", flush=True)
    u0 = si.u0_heat1d(SMALL)
    ref = stepper.solve_linear(SMALL, u0)
    _, plain = H(SMALL, coarsen="spacetime", **HIER).solve(T(u0), check=False)
    assert plain["status"] != 0
    U, st = H(SMALL, coarsen="spacetime", krylov=30, max_cycles=400, **HIER).solve(T(u0))
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10


def test_fgmres_mixed_precision():
    """FP32 V-cycles as the (variable) preconditioner of FP64 FGMRES."""
    print("case fgmres mixed", flush=True)
    prob = si.problem(2, 64, 3, 32, 0.5, nu=1e-2, lam=1.0)
    u0 = si.u0_rd2d(prob, 2)
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, krylov=10, precision="mixed", rtol=1e-11).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= 1e-11
    assert rel_err(U.cpu().numpy(), ref) <= 1e-9


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fgmres_newton(prec):
    print("case fgmres newton", prec, flush=True)
    prob = si.problem(1, 64, 3, 16, 0.5, nu=1e-2, gamma=5.0, reaction="allen_cahn")
    u0 = np.random.default_rng(3).uniform(-0.1, 0.1, (1, 64))
    ref = stepper.solve_allen_cahn(prob, u0)
    tol = 1e-12 if prec == "fp64" else 1e-10
    U, st = H(prob, krylov=8, precision=prec, newton_rtol=tol).solve(T(u0))
    assert st["status"] == 0 and st["newton_its"] >= 2
    assert rel_err(U.cpu().numpy(), ref) <= (1e-10 if prec == "fp64" else 1e-9)


def test_fgmres_adjoint():
    print("case fgmres adjoint", flush=True)
    prob = si.problem(2, 32, 3, 16, 0.5, nu=1e-2, lam=1.0)
    ny, nx = si.grid_points(prob)
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal((ny, nx))
    tgt = rng.standard_normal((ny, nx))
    h = H(prob, krylov=6)
    U, st = h.solve(T(u0))
    assert st["status"] == 0
    gu0, gnu, ast = h.adjoint(U, 2.0 * (U[-1, -1] - T(tgt)))
    assert ast["status"] == 0
    ref_g, ref_nu = adjoint.gradients(prob, u0, tgt)
    assert rel_err(gu0.cpu().numpy(), ref_g) <= 1e-9
    assert abs(gnu - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))


def _exact_heat(prob):
    X, _ = si.coords(prob)
    return (np.cos(np.pi * X) * np.exp(-np.pi ** 2) + 2 * np.cos(3 * np.pi * X) * np.exp(-9 * np.pi ** 2)
            + 3 * np.cos(4 * np.pi * X) * np.exp(-16 * np.pi ** 2))


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5])
def test_paper_heat1d(M):
    """The paper's heat example (N_x = 1024, N_t from its tables, stop at
    1e-9): FGMRES around 7-level SMG cycles meets the paper's accuracy at T
    (max error below 1e-9 against the analytic solution for M >= 2), agrees
    with the sequential stepper, and takes fewer steps than the plain
    iteration."""
    coarsen = "space"
    print("case paper heat1d", M, coarsen, flush=True)
    g = json.load(open(GOLD))
    prob = si.paper_heat1d(M)
    nt = g["M1"]["Nt"] if M == 1 else g["nt_by_M"][str(M)]
    assert prob["N"] == nt and prob["nx"][0] == g["Nx"]
    u0 = si.u0_paper_heat1d(prob)
    kw = dict(coarsen=coarsen, max_levels=7, max_cycles=300)
    # the rounding floor of ||b - A U|| / ||b|| is near 1e-11 here (entries of
    # A up to dt nu / h^2 ~ 6e4)
    U, st = H(prob, krylov=10, rtol=1e-10, **kw).solve(T(u0))
    assert st["status"] == 0
    uT = U[-1, -1].cpu().numpy()
    err = np.abs(uT - _exact_heat(prob)).max()
    if M == 1:
        # backward Euler at N_t = 1024: about 1e-6 (the paper's footnote)
        assert 0.1 * g["M1"]["err_order_of_magnitude"] < err < 10 * g["M1"]["err_order_of_magnitude"]
    else:
        assert err < g["tol"]
    ref = stepper.solve_linear(prob, u0)
    assert np.abs(uT - ref[-1, -1]).max() <= 1e-10
    # steps to the paper's tolerance, against the plain iteration
    _, kst = H(prob, krylov=10, rtol=1e-9, **kw).solve(T(u0))
    _, plain = H(prob, rtol=1e-9, **kw).solve(T(u0))
    assert plain["status"] == 0 and kst["status"] == 0 and kst["cycles"] <= plain["cycles"]


def test_paper_monodomain_m3():
    """The paper's monodomain example (X = 10, T = 2, gamma = 5, M = 3,
    N_t = 32): Newton with FGMRES around SMG cycles against the stepper."""
    print("case paper monodomain", flush=True)
    prob = si.paper_monodomain(3)
    u0 = si.u0_paper_monodomain(prob)
    # h = 10/1024 puts the rounding floor of the stepper's Newton residual
    # near 1e-13, so its stop test is 1e-12 here
    ref = stepper.solve_allen_cahn(prob, u0, tol=1e-12)
    # the error is about 100x the relative Newton residual here (h = 10/1024,
    # mu = dt / h^2 = 655), so the solve stops at 1e-12 for a 1e-10 error
    U, st = H(prob, krylov=10, coarsen="space", max_levels=7, newton_rtol=1e-12).solve(T(u0))
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10


def test_fgmres_stops_at_rounding_floor():
    """A tolerance below the rounding floor ends once two restart cycles in a
    row were ended by the least-squares estimate while the true residual
    stayed above the tolerance, not after max_cycles."""
    print("case fgmres floor", flush=True)
    prob = si.paper_heat1d(4)
    u0 = si.u0_paper_heat1d(prob)
    U, st = H(prob, krylov=10, coarsen="space", max_levels=7, rtol=1e-16, max_cycles=1000).solve(
        T(u0), check=False)
    assert st["status"] == -4 and st["cycles"] < 100 and st["rel_res"] <= 1e-9, st


def test_fgmres_odd_length():
    """31 points x M = 3 x N = 5: an odd vector length (the vector kernels'
    tail element)."""
    print("case fgmres odd", flush=True)
    prob = si.problem(1, 30, 3, 5, 0.2, nu=1.0, bc="neumann")
    u0 = si.u0_paper_heat1d(prob)
    assert np.prod(si.grid_points(prob)) * 3 * 5 % 2 == 1
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, krylov=4, coarsen="space").solve(T(u0))
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10


def test_fgmres_windows():
    """Time windows (checkpointing) with the Krylov method in each window:
    the memory budget accounts for its 2 (m + 1) vectors."""
    print("case fgmres windows", flush=True)
    prob = si.problem(2, 32, 3, 48, 0.6, nu=1e-2, lam=0.5)
    ny, nx = si.grid_points(prob)
    m = 4
    slab = prob["M"] * nx * ny * 8
    budget = (5 + 2 * (m + 1) + 1) * slab * 16
    u0 = si.u0_rd2d(prob, 6)
    tgt = si.u_tgt_adj2d(prob, 7)
    ref = stepper.solve_linear(prob, u0)
    hw = H(prob, krylov=m, mem_budget=budget)
    assert hw.num_windows() == 3
    U, st = hw.solve(T(u0))
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10
    ref_g, ref_nu = adjoint.gradients(prob, u0, tgt)
    g, gnu, ast = hw.adjoint(U, 2.0 * (U[-1, -1] - T(tgt)))
    assert rel_err(g.cpu().numpy(), ref_g) <= 1e-9
    assert abs(gnu - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))


def test_fgmres_mixed_neumann():
    """Neumann grid (the unfused mixed path) with FP32 cycles preconditioning."""
    print("case fgmres mixed neumann", flush=True)
    prob = si.problem(2, 32, 3, 16, 0.5, nu=1e-2, lam=1.0, bc="neumann")
    u0 = np.random.default_rng(11).standard_normal(si.grid_points(prob))
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, krylov=6, precision="mixed", rtol=1e-11).solve(T(u0))
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-9


@pytest.mark.parametrize("M,Nt,L", [(2, 2048, 8), (5, 64, 7)])
def test_paper_heat1d_weak(M, Nt, L):
    """The longest runs of the paper's weak-scaling tables (Example ex_3):
    SMG^L with FGMRES against the sequential stepper."""
    print("case paper heat1d weak", M, Nt, flush=True)
    assert (Nt, L) in si.PAPER_WEAK[M]
    prob = si.paper_heat1d(M, Nt=Nt)
    u0 = si.u0_paper_heat1d(prob)
    # mu = dt / h^2 reaches 512 (M = 2) and 16384 (M = 5): the error of the
    # whole trajectory is up to ~100x the relative residual, so the solve
    # stops at 1e-12 for a 1e-10 error
    U, st = H(prob, krylov=10, coarsen="space", max_levels=L, nu_pre=3, nu_post=3, rtol=1e-12,
              max_cycles=300).solve(T(u0))
    assert st["status"] == 0
    ref = stepper.solve_linear(prob, u0)
    assert np.abs(U[-1, -1].cpu().numpy() - ref[-1, -1]).max() <= 1e-10
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10


def test_paper_heat1d_mixed_split_coarse():
    """Mixed precision on the paper's heat example (M = 2, N_t = 256): the FP32
    cycles' coarsest level (17 points x 256 slabs) takes the split recurrence."""
    print("case paper heat1d mixed", flush=True)
    prob = si.paper_heat1d(2)
    u0 = si.u0_paper_heat1d(prob)
    ref = stepper.solve_linear(prob, u0)
    for kr in (0, 10):
        U, st = H(prob, krylov=kr, precision="mixed", coarsen="space", max_levels=7, rtol=1e-10).solve(T(u0))
        assert st["status"] == 0
        assert np.abs(U[-1, -1].cpu().numpy() - ref[-1, -1]).max() <= 1e-10


def test_adjoint_split_coarse():
    """The transposed problem's coarsest level (8 x 8 points x 32 slabs) through
    the split recurrence: gradients against the oracle's adjoint."""
    print("case adjoint split coarse", flush=True)
    prob = si.problem(2, 32, 3, 32, 0.5, nu=1e-2, lam=1.0)
    ny, nx = si.grid_points(prob)
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal((ny, nx))
    tgt = rng.standard_normal((ny, nx))
    h = H(prob, coarsen="space", max_levels=3, fft_coarse=0)
    lv = h.levels()[-1]
    assert lv["nx"] * lv["ny"] == 64 and lv["N"] == 32
    U, st = h.solve(T(u0))
    assert st["status"] == 0
    g, gnu, ast = h.adjoint(U, 2.0 * (U[-1, -1] - T(tgt)))
    ref_g, ref_nu = adjoint.gradients(prob, u0, tgt)
    assert rel_err(g.cpu().numpy(), ref_g) <= 1e-9
    assert abs(gnu - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_fgmres_rd2d_full(prec):
    """The full 256^2 x M=3 x N=256 workload through FGMRES(5) (the bench's
    launch configuration) against the oracle's closed form."""
    print("case fgmres rd2d full", prec, flush=True)
    prob = si.config("rd2d")
    u0 = si.initial("rd2d", prob)
    U, st = H(prob, krylov=5, precision=prec, rtol=1e-10).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= 1e-10
    ref = fourier.solve_linear_periodic(prob, u0)
    got = U.cpu().numpy()
    assert rel_err(got, ref) <= 1e-9
    assert rel_err(got[-1, -1], ref[-1, -1]) <= 1e-9


@pytest.mark.parametrize("coarsen", ["space", "smmg"])
@pytest.mark.parametrize("k", [1, 3, 5, 7])
def test_left_preconditioned_steps_match_oracle(coarsen, k):
    """Left preconditioning (GMRES on M^-1 A U = M^-1 b, one V-cycle as M):
    the iterate after k Krylov steps (restart 5) against the oracle's GMRES
    on the same left-preconditioned system.  The V-cycle count is k plus one
    per restart residual plus the final check."""
    print("case left steps", coarsen, k, flush=True)
    u0 = si.u0_heat1d(SMALL)
    ref, hist, steps = krylov.solve(SMALL, u0, rtol=0.0, restart=5, max_steps=k, left=True, coarsen=coarsen,
                                    **HIER)
    assert steps == k
    cycles = k + 1 + (k - 1) // 5
    h = H(SMALL, coarsen=coarsen, krylov=5, krylov_left=1, max_cycles=cycles, rtol=1e-30, **HIER)
    U, st = h.solve(T(u0), check=False)
    assert st["status"] == -4 and st["cycles"] == cycles + 1
    assert_close(U.cpu().numpy(), ref, 1e-9, "left-preconditioned iterate after %d steps" % k)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_left_preconditioned_paper_heat1d(prec):
    """The paper's heat example (M = 3) with the preconditioned-residual stop
    at 1e-9: the end value against the stepper."""
    print("case left paper heat1d", prec, flush=True)
    prob = si.paper_heat1d(3)
    u0 = si.u0_paper_heat1d(prob)
    U, st = H(prob, krylov=10, krylov_left=1, precision=prec, coarsen="space", max_levels=7, rtol=1e-9).solve(T(u0))
    assert st["status"] == 0
    ref = stepper.solve_linear(prob, u0)
    assert np.abs(U[-1, -1].cpu().numpy() - ref[-1, -1]).max() <= 1e-9
