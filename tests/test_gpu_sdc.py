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
