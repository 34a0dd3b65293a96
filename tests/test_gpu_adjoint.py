"""Adjoint gradients (transposed system solved backward in time by the same
V-cycle kernels) against the oracle's discrete adjoint and central FD."""
import os

import numpy as np
import pytest

import stmg_inputs as si
from oracle import adjoint

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, rel_err  # noqa: E402


def _loss_and_grad(prob, u0, tgt, **opt):
    h = H(prob, **opt)
    U, st = h.solve(T(u0))
    uT = U[-1, -1]
    g = 2.0 * (uT - T(tgt))
    L = float(((uT - T(tgt)) ** 2).sum())
    gu0, gnu, ast = h.adjoint(U, g)
    return L, gu0.cpu().numpy(), gnu, ast


@pytest.mark.parametrize("dim,M", [(1, 2), (2, 3), (2, 4)])
def test_adjoint_vs_oracle(dim, M):
    print("case adjoint", dim, M, flush=True)
    if dim == 1:
        prob = si.problem(1, 64, M, 16, 0.2, nu=0.5, lam=0.5)
    else:
        prob = si.problem(2, 32, M, 16, 0.5, nu=1e-2, lam=1.0)
    ny, nx = si.grid_points(prob)
    rng = np.random.default_rng(7)
    u0 = rng.standard_normal((ny, nx))
    tgt = rng.standard_normal((ny, nx))
    L, gu0, gnu, st = _loss_and_grad(prob, u0, tgt)
    assert st["status"] == 0
    ref_g, ref_nu = adjoint.gradients(prob, u0, tgt)
    assert rel_err(gu0, ref_g) <= 1e-9
    assert abs(gnu - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))


def test_adjoint_adj2d_full_fd():
    """Full 256^2 x M=3 x N=256 workload: the u0-gradient against central FD
    (h = 1e-6) on 16 random unit directions, and dL/dnu against central FD.

    Each FD solve runs the same fixed number of V-cycles (enough to reach the
    rounding floor), so that the +h and -h solves take the same path: the
    V-cycle iteration is linear in u0, and the FD quotient is then not polluted
    by stopping-tolerance noise divided by h."""
    print("case adjoint full", flush=True)
    prob = si.config("adj2d")
    u0 = si.initial("adj2d", prob)
    tgt = si.u_tgt_adj2d(prob)
    L, gu0, gnu, st = _loss_and_grad(prob, u0, tgt)
    assert st["status"] == 0
    K = 80
    fixed = dict(rtol=1e-30, max_cycles=K)
    h = H(prob, **fixed)
    tg = T(tgt)

    def loss(hh, u):
        U, s = hh.solve(T(u), check=False)
        assert s["status"] in (0, -4) and s["cycles"] == K
        return float(((U[-1, -1] - tg) ** 2).sum())

    eps = 1e-6
    for d in si.directions(u0.shape, 16, seed=41):
        fd = (loss(h, u0 + eps * d) - loss(h, u0 - eps * d)) / (2 * eps)
        ad = float(np.sum(gu0 * d))
        assert abs(fd - ad) <= 1e-6 * np.linalg.norm(gu0) + 1e-6 * abs(ad), (fd, ad)
    hp = H(dict(prob, nu=prob["nu"] + eps), **fixed)
    hm = H(dict(prob, nu=prob["nu"] - eps), **fixed)
    fdnu = (loss(hp, u0) - loss(hm, u0)) / (2 * eps)
    assert abs(fdnu - gnu) <= 1e-5 * max(1.0, abs(gnu)), (fdnu, gnu)


@pytest.mark.parametrize("dim,M", [(1, 2), (2, 3), (2, 4)])
def test_adjoint_mixed_vs_oracle(dim, M):
    """Mixed precision (FP32 V-cycles on the transposed system inside FP64
    refinement) reaches the oracle's discrete adjoint to 1e-9."""
    print("case adjoint mixed", dim, M, flush=True)
    if dim == 1:
        prob = si.problem(1, 64, M, 16, 0.2, nu=0.5, lam=0.5)
    else:
        prob = si.problem(2, 32, M, 16, 0.5, nu=1e-2, lam=1.0)
    ny, nx = si.grid_points(prob)
    rng = np.random.default_rng(8)
    u0 = rng.standard_normal((ny, nx))
    tgt = rng.standard_normal((ny, nx))
    L, gu0, gnu, st = _loss_and_grad(prob, u0, tgt, precision="mixed", rtol=1e-11)
    assert st["status"] == 0 and st["rel_res"] <= 1e-11
    ref_g, ref_nu = adjoint.gradients(prob, u0, tgt)
    assert rel_err(gu0, ref_g) <= 1e-9
    assert abs(gnu - ref_nu) <= 1e-9 * max(1.0, abs(ref_nu))


_ADJ2D_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adj2d_256_golden.npz")


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_adjoint_adj2d_full_vs_oracle_golden(prec):
    """The full 256^2 x M=3 x N=256 gradient workload against the stored
    oracle gradients (tests/golden/make_adj2d_golden.py: the sequential
    stepper and its discrete adjoint with a direct solve per step)."""
    print("case adjoint full golden", prec, flush=True)
    g = np.load(_ADJ2D_GOLDEN)
    prob = si.config("adj2d")
    u0 = si.initial("adj2d", prob)
    tgt = si.u_tgt_adj2d(prob)
    opt = dict(rtol=1e-12) if prec == "fp64" else dict(precision="mixed", rtol=1e-11)
    L, gu0, gnu, st = _loss_and_grad(prob, u0, tgt, **opt)
    assert st["status"] == 0
    lim = 1e-10 if prec == "fp64" else 1e-9
    assert abs(L - float(g["loss"])) <= lim * abs(float(g["loss"]))
    assert rel_err(gu0, g["grad_u0"]) <= lim
    assert abs(gnu - float(g["grad_nu"])) <= lim * abs(float(g["grad_nu"]))
    print("adjoint %s: %d cycles, grad err %.2e, dnu err %.2e" % (
        prec, st["cycles"], rel_err(gu0, g["grad_u0"]), abs(gnu / float(g["grad_nu"]) - 1)))
