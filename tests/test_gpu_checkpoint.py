"""Time-window checkpointing and the autograd Function (GPU)."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import adjoint

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, rel_err  # noqa: E402


def _prob():
    return si.problem(2, 32, 3, 48, 0.6, nu=1e-2, lam=0.5)


def _budget(prob, slabs):
    """A memory budget that leaves windows of `slabs` slabs (power of two)."""
    ny, nx = si.grid_points(prob)
    return 6 * prob["M"] * nx * ny * 8 * slabs


def test_windowed_solve_matches_full():
    print("case windowed solve", flush=True)
    prob = _prob()
    u0 = si.u0_rd2d(prob, 5)
    U, st = H(prob).solve(T(u0))
    hw = H(prob, mem_budget=_budget(prob, 16))
    assert hw.num_windows() == 3
    Uw, stw = hw.solve(T(u0))
    assert stw["status"] == 0
    assert rel_err(Uw.cpu().numpy(), U.cpu().numpy()) <= 1e-10
    uT, ste = hw.solve_end(T(u0))
    assert rel_err(uT.cpu().numpy(), U[-1, -1].cpu().numpy()) <= 1e-10


@pytest.mark.parametrize("slabs", [16, 32])
def test_windowed_adjoint_matches_oracle(slabs):
    print("case windowed adjoint", slabs, flush=True)
    prob = _prob()
    u0 = si.u0_rd2d(prob, 6)
    tgt = si.u_tgt_adj2d(prob, 7)
    ref_g, ref_nu = adjoint.gradients(prob, u0, tgt)
    hw = H(prob, mem_budget=_budget(prob, slabs))
    assert hw.num_windows() == (3 if slabs == 16 else 2)
    uT, _ = hw.solve_end(T(u0))
    gT = 2.0 * (uT - T(tgt))
    g, gnu, st = hw.adjoint(None, gT, u0=T(u0))      # trajectory recomputed
    assert rel_err(g.cpu().numpy(), ref_g) <= 1e-9
    assert abs(gnu - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))
    U, _ = hw.solve(T(u0))                             # trajectory given
    g2, gnu2, _ = hw.adjoint(U, gT)
    assert rel_err(g2.cpu().numpy(), ref_g) <= 1e-9
    assert abs(gnu2 - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))


@pytest.mark.parametrize("budget", [None, 16])
def test_autograd_function(budget):
    print("case autograd", budget, flush=True)
    from paper_2006_12883_amd import autograd as ag
    prob = _prob()
    u0n = si.u0_rd2d(prob, 8)
    tgt = si.u_tgt_adj2d(prob, 9)
    ref_g, ref_nu = adjoint.gradients(prob, u0n, tgt)
    u0 = T(u0n).requires_grad_(True)
    nu = torch.tensor(prob["nu"], dtype=torch.float64, device="cuda:0", requires_grad=True)
    opts = {} if budget is None else {"mem_budget": _budget(prob, budget)}
    uT = ag.end_value(u0, nu, prob, **opts)
    L = ((uT - T(tgt)) ** 2).sum()
    L.backward()
    assert rel_err(u0.grad.cpu().numpy(), ref_g) <= 1e-9
    assert abs(float(nu.grad) - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))
