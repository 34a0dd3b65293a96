"""SDC sweeps on the GPU (A11) against the oracle's sweep and the collocation
solution."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import sdc, stepper

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, assert_close, rel_err  # noqa: E402

CASES = [
    ("1d-M2", si.problem(1, 64, 2, 8, 0.1, nu=1.0)),
    ("2d-M3", si.problem(2, 32, 3, 8, 0.5, nu=1e-2, lam=1.0)),
    ("2d-M4-odd", si.problem(2, 20, 4, 5, 0.4, nu=2e-2, lam=0.3)),
]


@pytest.mark.parametrize("name,prob", CASES)
def test_one_sweep_matches_oracle(name, prob):
    print("case sdc sweep", name, flush=True)
    ny, nx = si.grid_points(prob)
    rng = np.random.default_rng(1)
    u0 = rng.standard_normal((ny, nx))
    U = rng.standard_normal((prob["N"], prob["M"], ny, nx))
    ref = sdc.sweep(prob, u0, U)
    h = H(prob, sdc=1)
    Ud = T(U)
    h.sdc_sweep(T(u0), Ud, 1)
    assert_close(Ud.cpu().numpy(), ref, 1e-10, "one SDC sweep")


@pytest.mark.parametrize("name,prob", CASES)
def test_fixed_point_and_convergence(name, prob):
    print("case sdc converge", name, flush=True)
    ny, nx = si.grid_points(prob)
    u0 = np.random.default_rng(2).standard_normal((ny, nx))
    ref = stepper.solve_linear(prob, u0)
    h = H(prob, sdc=1)
    Ue = T(ref)
    rel = h.sdc_sweep(T(u0), Ue, 1)
    assert rel_err(Ue.cpu().numpy(), ref) <= 1e-12 and rel <= 1e-11
    U = torch.zeros_like(Ue)
    rel = h.sdc_sweep(T(u0), U, 40)
    assert rel_err(U.cpu().numpy(), ref) <= 1e-9, rel


def test_sdc_needs_option():
    prob = CASES[0][1]
    h = H(prob)
    with pytest.raises(Exception):
        h.sdc_sweep(T(np.zeros((1, 64))), torch.zeros(h.shape, dtype=torch.float64, device="cuda:0"), 1)


@pytest.mark.parametrize("name,prob", CASES[:2])
def test_sdc_smoothed_vcycle_matches_oracle(name, prob):
    """One V-cycle with options.smoother = SDC (each finest-level smoothing
    step is one SDC sweep; coarser levels block-Jacobi) against the oracle's
    V-cycle with the same smoothers (its SDC sweep solves exactly; the GPU's
    spatial solves stop at rtol = 1e-13)."""
    from oracle import mg
    print("case sdc smoother vcycle", name, flush=True)
    ny, nx = si.grid_points(prob)
    u0 = np.random.default_rng(3).standard_normal((ny, nx))
    levels, kinds = mg.hierarchy(prob)
    smoothers = [lambda V, f: sdc.sweep(prob, u0, V)] + \
                [(lambda V, f, lev=lev: lev.smooth(V, f, 0.8, 4)) for lev in levels[1:]]
    f = mg.rhs(levels, u0)
    ref = mg.vcycle(levels, kinds, np.zeros(levels[0].shape), f, smoothers=smoothers)
    h = H(prob, smoother="sdc", rtol=1e-13)
    assert len(h.levels()) == len(levels)
    U = torch.zeros(levels[0].shape, dtype=torch.float64, device="cuda:0")
    h.vcycle(T(u0), U)
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10


@pytest.mark.parametrize("name,prob", CASES)
def test_sdc_smoother_solve(name, prob):
    """Solves with the SDC smoother reach the collocation (stepper) solution."""
    print("case sdc smoother solve", name, flush=True)
    ny, nx = si.grid_points(prob)
    u0 = np.random.default_rng(4).standard_normal((ny, nx))
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, smoother="sdc", rtol=1e-12).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= 1e-12
    assert rel_err(U.cpu().numpy(), ref) <= 1e-10
    print("sdc smoother: %d cycles" % st["cycles"])


def test_sdc_smoother_unsupported_combinations():
    """The SDC smoother is for FP64 linear problems without the Krylov method."""
    from paper_2006_12883_amd import binding as B
    prob = CASES[1][1]
    for kw in (dict(precision="mixed"), dict(krylov=4)):
        with pytest.raises(B.STMGError) as e:
            H(prob, smoother="sdc", **kw)
        assert "SDC smoother" in str(e.value)
    ac = si.problem(2, 16, 2, 4, 0.5, nu=1e-2, gamma=1.0, reaction="allen_cahn")
    with pytest.raises(B.STMGError):
        H(ac, smoother="sdc")
