"""Batched solves (A13): each problem against the closed form and against its
unbatched solve."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import fourier

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, rel_err  # noqa: E402


def _small_batch():
    return [
        si.problem(2, 32, 2, 16, 1.0, nu=1e-2, lam=0.5),
        si.problem(2, 64, 3, 32, 1.0, nu=3e-3, lam=1.5),
        si.problem(2, 24, 4, 8, 0.5, nu=5e-2, lam=0.0),
        si.problem(2, 48, 3, 64, 1.0, nu=1e-1, lam=1.0),
        si.problem(2, 16, 2, 4, 1.0, nu=2e-3, lam=0.2),
        si.problem(2, 96, 4, 16, 1.0, nu=1e-3, lam=1.9),
    ]


def test_small_batch_vs_closed_form_and_unbatched():
    from paper_2006_12883_amd import stmg
    probs = _small_batch()
    u0s = [si.batch_u0(p, i) for i, p in enumerate(probs)]
    b = stmg.Batch(probs, device="cuda:0", rtol=1e-10)
    Us, stats = b.solve([T(u) for u in u0s])
    for i, (p, u0, U, st) in enumerate(zip(probs, u0s, Us, stats)):
        print("problem", i, st, flush=True)
        assert st["status"] == 0 and st["rel_res"] <= 1e-10
        ref = fourier.solve_linear_periodic(p, u0)
        Un = U.cpu().numpy()
        assert rel_err(Un, ref) <= 1e-9, i
        V, sv = H(p, precision="mixed", rtol=1e-10).solve(T(u0))
        assert rel_err(Un, V.cpu().numpy()) <= 1e-9, i


def test_batch_repeat_and_warm_start():
    """A second solve from the converged iterate stops at once (every problem
    meets the tolerance at its first residual check)."""
    from paper_2006_12883_amd import stmg
    probs = _small_batch()[:3]
    u0s = [T(si.batch_u0(p, i)) for i, p in enumerate(probs)]
    b = stmg.Batch(probs, device="cuda:0", rtol=1e-10)
    Us, st1 = b.solve(u0s)
    Us2, st2 = b.solve(u0s, [U.clone() for U in Us])
    assert all(s["cycles"] == 0 for s in st2)
    assert all(torch.equal(a, c) for a, c in zip(Us, Us2))


def test_batch64_full():
    """The 64-problem workload (nx in {64..512}, N in {32..256}, M in {2,3,4},
    nu log-uniform, lambda uniform): every problem reaches 1e-10 and its end
    value u(T) matches the closed form R(dt sigma_k)^N u0_hat."""
    from paper_2006_12883_amd import stmg
    probs = si.batch64()
    u0s = [si.batch_u0(p, i) for i, p in enumerate(probs)]
    b = stmg.Batch(probs, device="cuda:0", rtol=1e-10)
    Us, stats = b.solve([T(u) for u in u0s])
    print("cycles", [s["cycles"] for s in stats], flush=True)
    for i, (p, u0, U, st) in enumerate(zip(probs, u0s, Us, stats)):
        assert st["status"] == 0 and st["rel_res"] <= 1e-10, (i, st)
        ref = fourier.end_value_periodic(p, u0)
        assert rel_err(U[-1, -1].cpu().numpy(), ref) <= 1e-9, i


@pytest.mark.parametrize("inner", [1, 3])
def test_batch_inner_cycles(inner):
    """One or several FP32 cycles per refinement step of the batch: every
    problem still reaches 1e-10 and the closed form, cycles = steps x inner."""
    from paper_2006_12883_amd import stmg
    print("case batch inner", inner, flush=True)
    probs = _small_batch()
    u0s = [si.batch_u0(p, i) for i, p in enumerate(probs)]
    b = stmg.Batch(probs, device="cuda:0", rtol=1e-10, inner_cycles=inner)
    Us, stats = b.solve([T(u) for u in u0s])
    for i, (p, u0, U, st) in enumerate(zip(probs, u0s, Us, stats)):
        assert st["status"] == 0 and st["rel_res"] <= 1e-10, (i, st)
        assert st["cycles"] == inner * st["refinements"]
        ref = fourier.solve_linear_periodic(p, u0)
        assert rel_err(U.cpu().numpy(), ref) <= 1e-9, i


def test_batch_autotune_bitwise_identical(tmp_path, monkeypatch):
    """The batch autotuner (the restrictions' slab run per level shape) changes
    launch shapes only: solutions are bitwise equal to the untuned batch, the
    choices are cached under "batch_" keys, and a second tuned batch reads
    them back."""
    import json
    from paper_2006_12883_amd import stmg
    print("case batch autotune", flush=True)
    cache = tmp_path / "tune.json"
    monkeypatch.setenv("STMG_TUNE_CACHE", str(cache))
    probs = _small_batch() + [si.problem(2, 256, 3, 64, 1.0, nu=1e-2, lam=1.0)]
    u0s = [T(si.batch_u0(p, i)) for i, p in enumerate(probs)]
    Ua, sa = stmg.Batch(probs, device="cuda:0", rtol=1e-10).solve(u0s)
    Ub, sb = stmg.Batch(probs, device="cuda:0", rtol=1e-10, autotune=1).solve(u0s)
    keys = json.loads(cache.read_text())
    assert any(k.startswith("batch_") for k in keys)
    assert all(v >= 1 and v % 4 == 0 for k, v in keys.items() if k.startswith("batch_"))
    Uc, sc = stmg.Batch(probs, device="cuda:0", rtol=1e-10, autotune=1).solve(u0s)
    for i in range(len(probs)):
        assert sa[i]["status"] == 0 and sb[i]["cycles"] == sa[i]["cycles"]
        assert torch.equal(Ua[i], Ub[i]) and torch.equal(Ua[i], Uc[i]), i
