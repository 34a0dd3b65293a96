"""The level-0 pre-smoothing sweep fused with the restriction of the new
residual (stmg_level_smooth_restrict, Sec. 4.2) against the oracle's sweep
followed by its restriction and the coarse level's first sweep from zero.

Grids whose tiles of 64 x 16 fine points cover the plane: one workgroup run
in time (no run boundary), several runs of one smoother chunk, a ragged last
run, runs of two smoother chunks (the chunk start inside a run), with and
without a right-hand side array, from zero and from a random iterate.  Each
case prints its name before touching the GPU."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, assert_close  # noqa: E402


def _rect(prob, nx, ny):
    prob = dict(prob)
    prob["nx"] = [nx, ny]
    prob["length"] = [prob["length"][0], prob["length"][0] * ny / nx]
    return prob


# (name, problem, options): smoother chunk 16 / coarse chunk 4 unless given
CASES = [
    ("64x64-M3-N48", si.problem(2, 64, 3, 48, 0.3, nu=0.02, lam=1.0), {}),
    ("128x64-M2-N40", _rect(si.problem(2, 128, 2, 40, 0.25, nu=0.01, lam=0.5), 128, 64), {}),
    ("64x64-M4-N16", si.problem(2, 64, 4, 16, 0.2, nu=0.05, lam=0.0), {}),
    ("64x64-M1-N33", si.problem(2, 64, 1, 33, 0.4, nu=0.03, lam=2.0), {}),
    ("128x128-M2-N128-chunk2", si.problem(2, 128, 2, 128, 0.25, nu=0.01, lam=0.5),
     dict(chunk=2, chunk_coarse=2)),
    ("64x128-M3-N24-chunk8", _rect(si.problem(2, 64, 3, 24, 0.3, nu=0.02, lam=1.0), 64, 128),
     dict(chunk=8, chunk_coarse=4)),
]


def _ref(prob, opts, U, f):
    levels, kinds = mg.hierarchy(prob, coarsen="space")
    assert kinds[0] == "s"
    lev, nxt = levels[0], levels[1]
    chunk, cc = opts.get("chunk", 16), opts.get("chunk_coarse", 4)
    Us = lev.smooth(U, f, 0.8, chunk)
    fc = mg.restrict(f - lev.apply(Us), "s", lev.dim, bc=lev.bc)
    uc = nxt.smooth(np.zeros(nxt.shape), fc, 0.8, cc)
    return levels, Us, fc, uc


@pytest.mark.parametrize("name,prob,opts", CASES)
@pytest.mark.parametrize("zero", [False, True])
def test_smooth_restrict_matches_oracle(name, prob, opts, zero):
    print("case", name, zero, flush=True)
    rng = np.random.default_rng(7)
    h = H(prob, coarsen="space", **opts)
    levels, Us, fc, uc = None, None, None, None
    shape = (prob["N"], prob["M"], prob["nx"][1], prob["nx"][0])
    U = np.zeros(shape) if zero else rng.standard_normal(shape)
    f = rng.standard_normal(shape)
    levels, Us, fcr, ucr = _ref(prob, opts, U, f)
    out = torch.empty(shape, dtype=torch.float64, device="cuda:0")
    fc = torch.empty(levels[1].shape, dtype=torch.float64, device="cuda:0")
    uc = torch.empty(levels[1].shape, dtype=torch.float64, device="cuda:0")
    h.smooth_restrict(0, out, fc, Uin=None if zero else T(U), uc=uc, f=T(f))
    assert_close(out.cpu().numpy(), Us, 1e-12, "sweep")
    assert_close(fc.cpu().numpy(), fcr, 1e-12, "restricted residual")
    assert_close(uc.cpu().numpy(), ucr, 1e-12, "coarse first sweep")
    # without the coarse sweep, the same restriction
    fc2 = torch.empty_like(fc)
    h.smooth_restrict(0, out, fc2, Uin=None if zero else T(U), f=T(f))
    assert torch.equal(fc, fc2)


def test_smooth_restrict_right_hand_side_from_u0():
    """f = NULL: the right-hand side is the u0 coupling of slab 0."""
    print("case u0 rhs", flush=True)
    prob, opts = CASES[0][1], {}
    rng = np.random.default_rng(8)
    shape = (prob["N"], prob["M"], prob["nx"][1], prob["nx"][0])
    U = rng.standard_normal(shape)
    u0 = rng.standard_normal(shape[2:])
    levels, kinds = mg.hierarchy(prob, coarsen="space")
    f = mg.rhs(levels, u0)
    _, Us, fcr, ucr = _ref(prob, opts, U, f)
    h = H(prob, coarsen="space")
    out = torch.empty(shape, dtype=torch.float64, device="cuda:0")
    fc = torch.empty(levels[1].shape, dtype=torch.float64, device="cuda:0")
    uc = torch.empty(levels[1].shape, dtype=torch.float64, device="cuda:0")
    h.smooth_restrict(0, out, fc, Uin=T(U), uc=uc, u0=T(u0))
    assert_close(out.cpu().numpy(), Us, 1e-12, "sweep")
    assert_close(fc.cpu().numpy(), fcr, 1e-12, "restricted residual")
    assert_close(uc.cpu().numpy(), ucr, 1e-12, "coarse first sweep")


def test_smooth_restrict_vcycle_matches_oracle():
    """One V-cycle on a grid where level 0 runs the fused sweep, against the
    oracle's V-cycle (runs of two chunks, three levels)."""
    print("case fused vcycle", flush=True)
    prob, opts = CASES[4][1], CASES[4][2]
    rng = np.random.default_rng(9)
    u0 = rng.standard_normal((prob["nx"][1], prob["nx"][0]))
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=0, max_levels=3)
    f = mg.rhs(levels, u0)
    U0 = rng.standard_normal(levels[0].shape)
    ref = mg.vcycle(levels, kinds, U0.copy(), f, chunk=2, chunk_coarse=2)
    h = H(prob, coarsen="space", fft_coarse=0, max_levels=3, **opts)
    Ud = T(U0)
    h.vcycle(T(u0), Ud)
    assert_close(Ud.cpu().numpy(), ref, 1e-11, "V-cycle")


def test_smooth_restrict_unsupported_grids():
    print("case unsupported", flush=True)
    prob = si.problem(2, 32, 3, 8, 0.3, nu=0.02, lam=1.0)  # tiles of 64 points do not fit
    h = H(prob, coarsen="space")
    out = torch.empty((8, 3, 32, 32), dtype=torch.float64, device="cuda:0")
    fc = torch.empty((8, 3, 16, 16), dtype=torch.float64, device="cuda:0")
    with pytest.raises(Exception) as e:
        h.smooth_restrict(0, out, fc, f=out)
    assert "fused smoothing" in str(e.value)
