"""Galerkin coarse levels (A_{l+1} = R A_l P, Sec. 4.2) on the GPU against the
oracle's assembled Galerkin matrices: per level (9-point smoothing sweep,
residual restriction, prolongation + sweep, Fourier coarsest solve), one
V-cycle, and whole solves against the stepper, FP64 and mixed precision.

Each case prints its name before touching the GPU."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import stmg_inputs as si
from oracle import adjoint, galerkin, mg, stepper

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, assert_close, rel_err  # noqa: E402


def _rect(prob, nx, ny, ly):
    prob = dict(prob)
    prob["nx"] = [nx, ny]
    prob["length"] = [prob["length"][0], ly]
    return prob


# (name, problem, fft_coarse): fft_coarse chosen so that the hierarchy has at
# least two Galerkin levels above the Fourier coarsest one
CASES = [
    ("2d-M2", si.problem(2, 32, 2, 8, 0.5, nu=0.02, lam=1.0), 2048),
    ("2d-M3-tiles", si.problem(2, 48, 3, 9, 0.5, nu=0.05, lam=0.3), 2048),
    ("2d-M4", si.problem(2, 32, 4, 5, 1.0, nu=0.01, lam=0.5), 2048),
    ("2d-M1", si.problem(2, 32, 1, 12, 0.3, nu=0.1, lam=0.0), 1024),
    ("2d-rect", _rect(si.problem(2, 32, 3, 6, 0.5, nu=0.03, lam=0.7), 32, 16, 0.5), 512),
    ("1d-M2", si.problem(1, 128, 2, 16, 0.1, nu=1.0, lam=0.0), 1024),
    ("1d-M3", si.problem(1, 128, 3, 6, 0.2, nu=0.3, lam=0.1), 1024),
    # down to the 2 x 2 plane (fft_coarse 0), many slabs per smoother chunk run
    ("2d-deep", si.problem(2, 16, 3, 40, 40 / 256, nu=1e-2, lam=1.0), 0),
    ("1d-deep", si.problem(1, 64, 2, 24, 0.1, nu=0.05, lam=0.5), 0),
    ("2d-M6", si.problem(2, 16, 6, 4, 0.2, nu=0.05, lam=0.5), 512),
    ("1d-M8", si.problem(1, 36, 8, 3, 0.1, nu=0.2, lam=0.3), 256),
]


def _setup(prob, fc):
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=fc)
    assert len(levels) >= 3 and all(k == "s" for k in kinds)
    As, Ps, Rs = galerkin.operators(levels, kinds, galerkin=True)
    return levels, kinds, As, Ps, Rs


def _handle(prob, fc, **kw):
    return H(prob, coarsen="space", fft_coarse=fc, coarse_op="galerkin", **kw)


def _smooth_ref(levels, As, l, U, f):
    """The GPU smoothers: block Jacobi over 16-slab chunks on the (rediscretized)
    finest level, the point-block sweep over 4-slab chunks on Galerkin levels
    with the damping scaled by the mass stencil (galerkin.damping)."""
    lev = levels[l]
    if l == 0:
        return lev.smooth(U, f, 0.8, 16)
    om = galerkin.damping(As[l], lev.shape, 0.8)
    return galerkin.point_block_smooth(As[l], lev.shape, U, f, om, 4)


@pytest.mark.parametrize("name,prob,fc", CASES)
def test_hierarchy_same_as_rediscretized(name, prob, fc):
    print("case", name, flush=True)
    levels, _ = mg.hierarchy(prob, coarsen="space", fft_coarse=fc)
    got = _handle(prob, fc).levels()
    assert [(g["nx"], g["ny"], g["N"], g["M"]) for g in got] == [(o.nx, o.ny, o.N, o.M) for o in levels]


@pytest.mark.parametrize("name,prob,fc", CASES)
@pytest.mark.parametrize("zero", [False, True])
def test_smooth_each_galerkin_level(name, prob, fc, zero):
    print("case", name, zero, flush=True)
    levels, kinds, As, _, _ = _setup(prob, fc)
    h = _handle(prob, fc)
    for l in range(1, len(levels) - 1):
        lev = levels[l]
        rng = np.random.default_rng(40 + l)
        U = np.zeros(lev.shape) if zero else rng.standard_normal(lev.shape)
        f = rng.standard_normal(lev.shape)
        ref = _smooth_ref(levels, As, l, U, f)
        out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        h.smooth(l, None if zero else T(U), out, f=T(f))
        assert_close(out.cpu().numpy(), ref, 1e-12, "Galerkin smooth level %d" % l)


@pytest.mark.parametrize("name,prob,fc", CASES)
def test_transfers_each_galerkin_level(name, prob, fc):
    """f_c = R (f - A_l U) with the Galerkin A_l; prolongation alone and fused
    with the level's sweep."""
    print("case", name, flush=True)
    levels, kinds, As, Ps, Rs = _setup(prob, fc)
    h = _handle(prob, fc)
    for l in range(len(levels) - 1):
        lev, nxt = levels[l], levels[l + 1]
        rng = np.random.default_rng(60 + l)
        U = rng.standard_normal(lev.shape)
        f = rng.standard_normal(lev.shape)
        ref = (Rs[l] @ (f.reshape(-1) - As[l] @ U.reshape(-1))).reshape(nxt.shape)
        fc_d = torch.empty(nxt.shape, dtype=torch.float64, device="cuda:0")
        h.restrict_residual(l, T(U), fc_d, f=T(f))
        assert_close(fc_d.cpu().numpy(), ref, 1e-12, "restrict level %d" % l)
        ec = rng.standard_normal(nxt.shape)
        up = U + (Ps[l] @ ec.reshape(-1)).reshape(lev.shape)
        out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        h.prolong(l, T(ec), out, Uin=T(U))
        assert_close(out.cpu().numpy(), up, 1e-13, "prolong level %d" % l)
        ref_ps = _smooth_ref(levels, As, l, up, f)
        h.prolong_smooth(l, T(ec), out, Uin=T(U), f=T(f))
        assert_close(out.cpu().numpy(), ref_ps, 1e-12, "prolong + smooth level %d" % l)


@pytest.mark.parametrize("name,prob,fc", CASES)
def test_galerkin_coarse_solve(name, prob, fc):
    """Fourier solve of the Galerkin coarsest level (mass symbol divided out)
    against a sparse direct solve of the assembled R A P."""
    print("case", name, flush=True)
    levels, kinds, As, _, _ = _setup(prob, fc)
    h = _handle(prob, fc)
    lev = levels[-1]
    f = np.random.default_rng(3).standard_normal(lev.shape)
    ref = spla.spsolve(As[-1].tocsc(), f.reshape(-1)).reshape(lev.shape)
    out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
    h.coarse_solve(T(f), out)
    assert_close(out.cpu().numpy(), ref, 1e-11, "Galerkin coarse solve")


@pytest.mark.parametrize("name,prob,fc", CASES)
def test_one_galerkin_vcycle(name, prob, fc):
    print("case", name, flush=True)
    levels, kinds, As, Ps, Rs = _setup(prob, fc)
    u0 = np.random.default_rng(4).standard_normal(levels[0].shape[2:])
    f = mg.rhs(levels, u0)
    U = np.random.default_rng(5).standard_normal(levels[0].shape)
    sms = [(lambda x, g, l=l: _smooth_ref(levels, As, l, x.reshape(levels[l].shape),
                                          g.reshape(levels[l].shape)).reshape(-1))
           for l in range(len(levels))]
    coarse = galerkin.exact_coarse(As[-1])
    ref = galerkin.vcycle(As, Ps, Rs, sms, coarse, U.reshape(-1), f.reshape(-1)).reshape(U.shape)
    h = _handle(prob, fc)
    Ud = T(U)
    h.vcycle(T(u0), Ud)
    assert_close(Ud.cpu().numpy(), ref, 1e-11, "one Galerkin V-cycle")


SOLVES = [
    ("rd2d-64-M3", si.problem(2, 64, 3, 16, 0.5, nu=1e-2, lam=1.0), 1 << 14),
    ("rd2d-128-M2", si.problem(2, 128, 2, 32, 1.0, nu=1e-3, lam=0.5), 1 << 16),
    ("heat1d-256-M3", si.problem(1, 256, 3, 32, 0.5, nu=0.1, lam=0.0), 1024),
    # down to 2 x 2 with 128 slabs: diverges with the unscaled damping
    ("rd2d-32-deep", si.problem(2, 32, 3, 128, 0.5, nu=1e-2, lam=1.0), 0),
]


@pytest.mark.parametrize("name,prob,fc", SOLVES)
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_galerkin_solve_matches_stepper(name, prob, fc, precision):
    """Galerkin SMG to rtol reaches the time stepper's solution (1e-10 FP64,
    1e-9 mixed); cycle counts next to the rediscretized hierarchy's."""
    print("case", name, precision, flush=True)
    ny, nx = si.grid_points(prob)
    u0 = si.u0_rd2d(prob, 3) if prob["dim"] == 2 else np.sin(2 * np.pi * np.arange(nx) / nx)
    ref = stepper.solve_linear(prob, u0)
    Ug, sg = _handle(prob, fc, precision=precision, max_cycles=200).solve(T(u0))
    Ur, sr = H(prob, coarsen="space", fft_coarse=fc, precision=precision, max_cycles=200).solve(T(u0))
    print("cycles galerkin", sg["cycles"], "rediscretized", sr["cycles"], flush=True)
    assert sg["status"] == 0 and sr["status"] == 0
    tol = 1e-10 if precision == "fp64" else 1e-9
    assert rel_err(Ug.cpu().numpy(), ref) <= tol
    assert rel_err(Ug.cpu().numpy()[-1, -1], ref[-1, -1]) <= tol
    assert sg["cycles"] <= 2 * sr["cycles"] + 2


def test_galerkin_adjoint_matches_oracle():
    """The transposed Galerkin hierarchy (R A^T P = (R A P)^T) drives the
    adjoint solve to the oracle's discrete gradient."""
    print("case adjoint galerkin", flush=True)
    prob = si.problem(2, 32, 3, 16, 0.5, nu=1e-2, lam=1.0)
    ny, nx = si.grid_points(prob)
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal((ny, nx))
    tgt = rng.standard_normal((ny, nx))
    h = _handle(prob, 4096)
    U, st = h.solve(T(u0))
    assert st["status"] == 0
    uT = U[-1, -1]
    gu0, gnu, ast = h.adjoint(U, 2.0 * (uT - T(tgt)))
    assert ast["status"] == 0
    ref_g, ref_nu = adjoint.gradients(prob, u0, tgt)
    assert rel_err(gu0.cpu().numpy(), ref_g) <= 1e-9
    assert abs(gnu - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))


def test_full_size_galerkin_solve_matches_rediscretized():
    """The 256^2 x 3 x 256 workload with Galerkin coarse levels, FP64 to 1e-12,
    reaches the solution of the rediscretized solve (the same all-at-once
    system) to 1e-10."""
    print("case full galerkin", flush=True)
    prob = si.config("rd2d")
    u0 = T(si.initial("rd2d", prob))
    Ug, sg = H(prob, coarsen="space", coarse_op="galerkin").solve(u0)
    Ur, sr = H(prob).solve(u0)
    print("cycles galerkin", sg["cycles"], "rediscretized", sr["cycles"], flush=True)
    assert sg["status"] == 0 and sr["status"] == 0
    assert float(torch.linalg.norm(Ug - Ur) / torch.linalg.norm(Ur)) <= 1e-10
