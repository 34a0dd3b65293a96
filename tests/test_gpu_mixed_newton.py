"""Mixed precision (FP32 V-cycles inside FP64 refinement) and Newton for the
Allen-Cahn reaction, against the FP64 oracle."""
import functools
import os

import numpy as np
import pytest

import stmg_inputs as si
from oracle import allatonce, fourier, stepper

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, rel_err  # noqa: E402


def _errs(U, ref):
    return rel_err(U, ref), rel_err(U[-1, -1], ref[-1, -1])


def test_mixed_heat1d():
    print("case mixed heat1d", flush=True)
    prob = si.config("heat1d")
    u0 = si.initial("heat1d", prob)
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, precision="mixed", rtol=1e-10, inner_adapt=0).solve(T(u0))
    # five FP32 V-cycles per FP64 refinement step
    assert st["status"] == 0 and st["rel_res"] <= 1e-10 and st["cycles"] == 5 * st["refinements"]
    e, eT = _errs(U.cpu().numpy(), ref)
    assert e <= 1e-9 and eT <= 1e-9, (e, eT)
    # by default (inner_adapt) a step from the second on may stop short of five
    Ua, sa = H(prob, precision="mixed", rtol=1e-10).solve(T(u0))
    assert sa["status"] == 0 and sa["rel_res"] <= 1e-10
    assert sa["refinements"] <= sa["cycles"] <= 5 * sa["refinements"] and sa["cycles"] <= st["cycles"]
    e, eT = _errs(Ua.cpu().numpy(), ref)
    assert e <= 1e-9 and eT <= 1e-9, (e, eT)


@pytest.mark.parametrize("M", [2, 3, 4])
def test_mixed_rd2d_small(M):
    print("case mixed rd2d small", M, flush=True)
    prob = si.problem(2, 64, M, 32, 0.5, nu=1e-2, lam=1.0)
    u0 = si.u0_rd2d(prob, 2)
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, precision="mixed", rtol=1e-10).solve(T(u0))
    assert st["status"] == 0
    e, eT = _errs(U.cpu().numpy(), ref)
    assert e <= 1e-9 and eT <= 1e-9, (e, eT)


@pytest.mark.parametrize("inner", [1, 2, 3, 6])
@pytest.mark.parametrize("adapt", [0, 1])
def test_mixed_inner_cycles(inner, adapt):
    """Any number of FP32 cycles per refinement step reaches the FP64
    tolerance; with inner_adapt the steps after the first may be shorter."""
    print("case mixed inner cycles", inner, adapt, flush=True)
    prob = si.problem(2, 64, 3, 32, 0.5, nu=1e-2, lam=1.0)
    u0 = si.u0_rd2d(prob, 5)
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, precision="mixed", rtol=1e-10, inner_cycles=inner, inner_adapt=adapt).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= 1e-10
    if adapt:
        assert inner + st["refinements"] - 1 <= st["cycles"] <= inner * st["refinements"]
    else:
        assert st["cycles"] == inner * st["refinements"]
    e, eT = _errs(U.cpu().numpy(), ref)
    assert e <= 1e-9 and eT <= 1e-9, (e, eT)


@pytest.mark.parametrize("kw", [{"nu_post": 0}, {"max_levels": 1}])
def test_mixed_unfolded_update(kw):
    """Where the last level-0 kernel is not the fused prolongation + smoothing
    (V(1,0) cycles, a single level) the refinement sweep adds the FP32
    correction itself; the solve still reaches the FP64 tolerance."""
    print("case mixed unfolded update", kw, flush=True)
    prob = si.problem(2, 32, 3, 16, 0.5, nu=1e-2, lam=1.0)
    u0 = si.u0_rd2d(prob, 6)
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, precision="mixed", rtol=1e-10, max_cycles=400, **kw).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= 1e-10
    e, eT = _errs(U.cpu().numpy(), ref)
    assert e <= 1e-9 and eT <= 1e-9, (e, eT)


def test_mixed_neumann():
    """Neumann grids take the unfused refinement path (separate update)."""
    print("case mixed neumann", flush=True)
    prob = si.problem(2, 32, 3, 16, 0.5, nu=1e-2, lam=1.0, bc="neumann")
    u0 = np.random.default_rng(11).normal(size=si.grid_points(prob)[::-1])
    ref = stepper.solve_linear(prob, u0)
    U, st = H(prob, precision="mixed", rtol=1e-10).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= 1e-10
    e, eT = _errs(U.cpu().numpy(), ref)
    assert e <= 1e-9 and eT <= 1e-9, (e, eT)


def test_mixed_rd2d_full():
    print("case mixed rd2d full", flush=True)
    prob = si.config("rd2d")
    u0 = si.initial("rd2d", prob)
    U, st = H(prob, precision="mixed", rtol=1e-10).solve(T(u0))
    assert st["status"] == 0
    ref = fourier.solve_linear_periodic(prob, u0)
    e, eT = _errs(U.cpu().numpy(), ref)
    assert e <= 1e-9 and eT <= 1e-9, (e, eT)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("dim", [1, 2])
def test_newton_allen_cahn_small(prec, dim):
    print("case newton", prec, dim, flush=True)
    if dim == 1:
        prob = si.problem(1, 64, 3, 16, 0.5, nu=1e-2, gamma=5.0, reaction="allen_cahn")
        u0 = np.random.default_rng(3).uniform(-0.1, 0.1, (1, 64))
    else:
        prob = si.problem(2, 64, 3, 32, 0.5, nu=1e-3, gamma=1.0, reaction="allen_cahn")
        u0 = si.u0_ac2d(prob, 3)
    ref = stepper.solve_allen_cahn(prob, u0)
    # the error reaches about 30x the relative Newton residual on the 2D case;
    # both precisions stop two orders of magnitude below the error bound
    tol = 1e-12 if prec == "fp64" else 1e-11
    U, st = H(prob, precision=prec, newton_rtol=tol).solve(T(u0))
    assert st["status"] == 0 and st["newton_its"] >= 2
    e, eT = _errs(U.cpu().numpy(), ref)
    lim = 1e-10 if prec == "fp64" else 1e-9
    assert e <= lim and eT <= lim, (e, eT)


def test_newton_fixed_points():
    """u = 0, 1, -1 are fixed points of the reaction: one Newton residual check."""
    prob = si.problem(2, 16, 2, 4, 0.5, nu=1e-2, gamma=2.0, reaction="allen_cahn")
    for c in (1.0, -1.0):
        u0 = np.full((16, 16), c)
        U, st = H(prob, newton_rtol=1e-13).solve(T(u0))
        assert st["status"] == 0
        assert np.abs(U.cpu().numpy() - c).max() < 1e-11


def test_newton_ac2d_full_sampled():
    """The full 512^2 x M=3 x N=512 Allen-Cahn workload in mixed precision: the
    nonlinear residual reaches 1e-10, and sampled entries of the GPU residual of
    the GPU solution agree with the oracle's entry-by-entry definition."""
    print("case ac2d full", flush=True)
    prob = si.config("ac2d")
    u0 = si.initial("ac2d", prob)
    h = H(prob, precision="mixed", newton_rtol=1e-10)
    u0d = T(u0)
    U, st = h.solve(u0d)
    assert st["status"] == 0 and st["rel_res"] <= 1e-10
    r = torch.empty_like(U)
    h.residual(u0d, U, r)
    rng = np.random.default_rng(0)
    for _ in range(12):
        n = int(rng.integers(0, prob["N"]))
        i = int(rng.integers(0, prob["M"]))
        y, x = (int(v) for v in rng.integers(0, 512, 2))
        lo = max(n - 1, 0)
        Ul = U[lo:n + 1].cpu().numpy()
        ref = allatonce.residual_entry(prob, u0, Ul, n - lo, i, y, x) if n > 0 else \
            allatonce.residual_entry(prob, u0, Ul, 0, i, y, x)
        got = float(r[n, i, y, x])
        assert abs(got - ref) <= 1e-12 * max(1.0, float(np.abs(Ul).max())), (n, i, y, x, got, ref)


_AC2D_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "ac2d_512_golden.npz")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_ac2d_full_vs_oracle_golden(prec):
    """The full 512^2 x M=3 x N=512 Allen-Cahn workload against the stored
    oracle solution (tests/golden/make_ac2d_golden.py: the sequential Radau
    IIA stepper with Newton per step to 1e-14): u(T), u(T/2), and the norm and
    sum of every slab's node planes.  The error is about 30x the relative
    Newton residual, so FP64 stops at 1e-12 and mixed precision at 1e-11."""
    print("case ac2d full golden", prec, flush=True)
    g = np.load(_AC2D_GOLDEN)
    prob = si.config("ac2d")
    u0 = si.initial("ac2d", prob)
    tol = 1e-12 if prec == "fp64" else 1e-11
    U, st = H(prob, precision=prec, newton_rtol=tol).solve(T(u0))
    assert st["status"] == 0 and st["rel_res"] <= tol
    N, M = prob["N"], prob["M"]
    lim = 1e-10 if prec == "fp64" else 1e-9
    assert rel_err(U[-1, -1].cpu().numpy(), g["uT"]) <= lim
    assert rel_err(U[N // 2 - 1, -1].cpu().numpy(), g["umid"]) <= lim
    flat = U.reshape(N, M, -1)
    norms = torch.linalg.vector_norm(flat, dim=2).cpu().numpy()
    sums = flat.sum(dim=2).cpu().numpy()
    assert np.abs(norms - g["norms"]).max() <= lim * np.abs(g["norms"]).max()
    assert np.abs(sums - g["sums"]).max() <= lim * np.abs(g["norms"]).max() * 512
    print("ac2d %s: %d Newton its, %d cycles, err(T) %.2e" % (prec, st["newton_its"], st["cycles"],
                                                          rel_err(U[-1, -1].cpu().numpy(), g["uT"])))


@functools.lru_cache(maxsize=1)
def _ac2d_reduced_oracle():
    prob = si.problem(2, 128, 3, 128, 0.5, nu=1e-3, gamma=1.0, reaction="allen_cahn")
    u0 = si.u0_ac2d(prob, 3)
    return prob, u0, stepper.solve_allen_cahn(prob, u0, reuse=True)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_newton_ac2d_reduced_full_trajectory(prec):
    """The reduced Allen-Cahn workload (128^2, N = 128, T = 0.5, the same nu,
    gamma and initial-data recipe): every stage value against the oracle."""
    print("case ac2d reduced", prec, flush=True)
    prob, u0, ref = _ac2d_reduced_oracle()
    tol = 1e-12 if prec == "fp64" else 1e-11
    U, st = H(prob, precision=prec, newton_rtol=tol).solve(T(u0))
    assert st["status"] == 0
    e, eT = _errs(U.cpu().numpy(), ref)
    lim = 1e-10 if prec == "fp64" else 1e-9
    assert e <= lim and eT <= lim, (e, eT)
