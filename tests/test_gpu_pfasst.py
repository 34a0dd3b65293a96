"""PFASST (stmg_pfasst_solve) against the oracle's PFASST iteration by
iteration, and its converged solution against the time stepper.

Each case prints its name before touching the GPU."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import pfasst, stepper

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, assert_close, rel_err  # noqa: E402


def _rect(prob, nx, ny, ly):
    prob = dict(prob)
    prob["nx"] = [nx, ny]
    prob["length"] = [prob["length"][0], ly]
    return prob


# (name, problem, levels, sweeps)
CASES = [
    ("2d-M3-L2", si.problem(2, 32, 3, 8, 0.25, nu=0.02, lam=1.0), 2, 1),
    ("2d-M2-L3", si.problem(2, 32, 2, 6, 0.3, nu=0.05, lam=0.5), 3, 1),
    ("2d-M4-L3-nu2", si.problem(2, 16, 4, 5, 0.2, nu=0.02, lam=0.3), 3, 2),
    ("2d-rect-L2", _rect(si.problem(2, 32, 3, 6, 0.3, nu=0.03, lam=0.7), 32, 16, 0.5), 2, 1),
    ("2d-neumann-L2", si.problem(2, 16, 2, 6, 0.3, nu=0.02, lam=1.0, bc="neumann"), 2, 1),
    ("1d-M3-L3", si.problem(1, 64, 3, 12, 0.2, nu=0.1, lam=0.5), 3, 1),
    ("1d-neumann-L3", si.problem(1, 32, 3, 8, 0.2, nu=0.1, lam=0.5, bc="neumann"), 3, 1),
    ("1d-M1-L2", si.problem(1, 64, 1, 16, 0.3, nu=0.2, lam=0.0), 2, 1),
    ("1d-M5-L3", si.problem(1, 64, 5, 6, 0.2, nu=0.1, lam=0.2), 3, 1),
]


def _u0(prob, seed):
    ny, nx = si.grid_points(prob)
    return np.random.default_rng(seed).standard_normal((ny, nx))


@pytest.mark.parametrize("name,prob,levels,nu", CASES)
def test_iterations_match_oracle(name, prob, levels, nu):
    """Four PFASST iterations from a random start, one call each (max_cycles
    1), against oracle.pfasst.iteration; inner solves to 1e-13."""
    print("case", name, flush=True)
    u0 = _u0(prob, 1)
    levs = pfasst.hierarchy(prob, levels)
    u0s = pfasst.initial_values(levs, u0)
    X = np.random.default_rng(2).standard_normal(levs[0].shape)
    h = H(prob, pfasst_levels=levels, pfasst_sweeps=nu, rtol=1e-13, max_cycles=1)
    Ud = T(X)
    ref = X
    for k in range(4):
        ref = pfasst.iteration(levs, u0s, ref, nu)
        _, st = h.pfasst(T(u0), Ud, check=False)
        assert st["cycles"] == 1 and st["status"] in (0, -4), st
        assert_close(Ud.cpu().numpy(), ref, 1e-10, "iteration %d" % (k + 1))


SOLVES = [
    ("rd2d-64-M3-L2", si.problem(2, 64, 3, 16, 0.5, nu=1e-2, lam=1.0), 2),
    ("rd2d-64-M3-L3", si.problem(2, 64, 3, 16, 0.5, nu=1e-2, lam=1.0), 3),
    ("heat1d-128-M2-L3", si.problem(1, 128, 2, 32, 0.1, nu=0.5, lam=0.0), 3),
    ("neumann1d-L2", si.problem(1, 64, 3, 16, 0.2, nu=0.05, lam=0.3, bc="neumann"), 2),
]


@pytest.mark.parametrize("name,prob,levels", SOLVES)
def test_converges_to_stepper(name, prob, levels):
    print("case", name, flush=True)
    ny, nx = si.grid_points(prob)
    u0 = si.u0_rd2d(prob, 3) if prob["dim"] == 2 else np.sin(2 * np.pi * np.arange(nx) / nx)[None, :]
    ref = stepper.solve_linear(prob, u0)
    h = H(prob, pfasst_levels=levels, rtol=1e-12, max_cycles=200)
    U, st = h.pfasst(T(u0))
    print("iterations", st["cycles"], "rel", st["rel_res"], flush=True)
    assert st["status"] == 0 and st["rel_res"] <= 1e-12
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10
    assert rel_err(U.cpu().numpy()[-1, -1], ref[-1, -1]) <= 1e-10


@pytest.mark.parametrize("inner", [1, 2])
def test_inexact_inner_solves_converge(inner):
    """With every inner solve cut to `inner` V-cycles PFASST still converges
    to the stepper's solution (more iterations, cheaper ones)."""
    print("case inexact", inner, flush=True)
    prob = si.problem(2, 64, 3, 16, 0.5, nu=1e-2, lam=1.0)
    u0 = si.u0_rd2d(prob, 3)
    ref = stepper.solve_linear(prob, u0)
    h = H(prob, pfasst_levels=2, pfasst_inner_cycles=inner, rtol=1e-12, max_cycles=300)
    U, st = h.pfasst(T(u0))
    print("iterations", st["cycles"], "rel", st["rel_res"], flush=True)
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10


# Allen-Cahn: IMEX sweeps (reaction explicit), the coarsest level swept slab
# after slab (one-slab Fourier or dense solves; the Neumann 33^2 plane takes
# the one-slab multigrid solver)
AC = [
    ("2d-AC-L2", si.problem(2, 32, 3, 8, 0.4, nu=0.02, gamma=1.0, reaction="allen_cahn"), 2, 1),
    ("2d-AC-L3-nu2", si.problem(2, 32, 2, 6, 0.3, nu=0.01, gamma=2.0, reaction="allen_cahn"), 3, 2),
    ("1d-AC-L3", si.problem(1, 64, 3, 12, 0.5, nu=0.05, gamma=1.0, reaction="allen_cahn"), 3, 1),
    ("1d-AC-neumann-L2", si.problem(1, 32, 2, 8, 0.4, nu=0.05, gamma=1.0, reaction="allen_cahn",
                                    bc="neumann"), 2, 1),
    ("2d-AC-neumann-L2", si.problem(2, 64, 2, 4, 0.1, nu=0.01, gamma=1.0, reaction="allen_cahn",
                                    bc="neumann"), 2, 1),
]


def _u0_ac(prob, seed):
    return 0.8 * np.tanh(_u0(prob, seed))


@pytest.mark.parametrize("name,prob,levels,nu", AC)
def test_imex_iterations_match_oracle(name, prob, levels, nu):
    print("case", name, flush=True)
    u0 = _u0_ac(prob, 1)
    levs = pfasst.hierarchy(prob, levels)
    u0s = pfasst.initial_values(levs, u0)
    X = 0.8 * np.tanh(np.random.default_rng(2).standard_normal(levs[0].shape))
    h = H(prob, pfasst_levels=levels, pfasst_sweeps=nu, rtol=1e-13, max_cycles=1)
    Ud = T(X)
    ref = X
    for k in range(3):
        ref = pfasst.iteration(levs, u0s, ref, nu)
        _, st = h.pfasst(T(u0), Ud, check=False)
        assert st["cycles"] == 1 and st["status"] in (0, -4), st
        assert_close(Ud.cpu().numpy(), ref, 1e-10, "IMEX iteration %d" % (k + 1))


def test_imex_sdc_sweep_matches_oracle():
    """stmg_sdc_sweep on an Allen-Cahn handle is the IMEX sweep (the oracle's
    level-0 PFASST sweep with tau = 0)."""
    print("case imex sdc sweep", flush=True)
    prob = si.problem(2, 32, 3, 8, 0.4, nu=0.02, gamma=1.5, reaction="allen_cahn")
    u0 = _u0_ac(prob, 3)
    lev = pfasst.PLevel(prob)
    X = 0.8 * np.tanh(np.random.default_rng(4).standard_normal(lev.shape))
    ref = X
    h = H(prob, sdc=1, rtol=1e-13)
    Ud = T(X)
    for k in range(3):
        ref = lev.sweep(ref, u0, np.zeros(lev.shape), serial=False)
        h.sdc_sweep(T(u0), Ud, 1)
        assert_close(Ud.cpu().numpy(), ref, 1e-10, "IMEX sweep %d" % (k + 1))


@pytest.mark.parametrize("levels", [2, 3])
def test_imex_converges_to_implicit_stepper(levels):
    print("case imex solve", levels, flush=True)
    prob = si.problem(2, 64, 3, 16, 0.5, nu=1e-3, gamma=1.0, reaction="allen_cahn")
    u0 = si.initial("ac2d", prob)
    ref = stepper.solve_allen_cahn(prob, u0)
    h = H(prob, pfasst_levels=levels, rtol=1e-12, max_cycles=300)
    U, st = h.pfasst(T(u0))
    print("iterations", st["cycles"], "rel", st["rel_res"], flush=True)
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10
    assert rel_err(U.cpu().numpy()[-1, -1], ref[-1, -1]) <= 1e-10


def test_pfasst_needs_its_levels():
    print("case no levels", flush=True)
    prob = si.problem(2, 16, 2, 4, 0.2, nu=0.05, lam=1.0)
    h = H(prob)
    with pytest.raises(Exception) as e:
        h.pfasst(T(_u0(prob, 1)))
    assert "pfasst_levels" in str(e.value)


def test_full_size_pfasst_matches_multigrid():
    """PFASST^3_1 with one V-cycle per inner solve on the 256^2 x 3 x 256
    workload, to 1e-12, against the multigrid solve of the same system."""
    print("case full pfasst", flush=True)
    prob = si.config("rd2d")
    u0 = T(si.initial("rd2d", prob))
    Up, sp = H(prob, pfasst_levels=3, pfasst_inner_cycles=1, max_cycles=300).pfasst(u0)
    Ur, sr = H(prob).solve(u0)
    print("iterations", sp["cycles"], flush=True)
    assert sp["status"] == 0 and sr["status"] == 0
    assert float(torch.linalg.norm(Up - Ur) / torch.linalg.norm(Ur)) <= 1e-10


def test_pfasst_nan_input_and_collocation_stop():
    """A NaN in u0 ends the iteration with STMG_ENAN; with form = COLLOC the
    stop test uses the collocation residual and reaches the same solution."""
    print("case pfasst nan / colloc", flush=True)
    prob = si.problem(2, 32, 3, 8, 0.25, nu=0.02, lam=1.0)
    u0 = _u0(prob, 5)
    bad = u0.copy()
    bad[3, 4] = np.nan
    _, st = H(prob, pfasst_levels=2).pfasst(T(bad), check=False)
    assert st["status"] == -6, st
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, pfasst_levels=2, form="colloc", rtol=1e-12).pfasst(T(u0))
    assert st["status"] == 0
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10
