"""Oracle pins: the discrete adjoint against finite differences."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import adjoint, stepper


def _loss(prob, u0, tgt):
    return adjoint.loss(prob, stepper.solve_linear(prob, u0), tgt)


@pytest.mark.parametrize("dim,M", [(1, 2), (2, 3)])
def test_adjoint_u0_fd(dim, M):
    prob = si.problem(dim, 16 if dim == 1 else 8, M, 6, 0.4, nu=0.05, lam=0.5)
    ny, nx = si.grid_points(prob)
    rng = np.random.default_rng(5)
    u0 = rng.standard_normal((ny, nx))
    tgt = rng.standard_normal((ny, nx))
    g, _ = adjoint.gradients(prob, u0, tgt)
    for d in si.directions((ny, nx), 4, seed=11):
        h = 1e-3  # the loss is quadratic in u0: central FD is exact up to rounding
        fd = (_loss(prob, u0 + h * d, tgt) - _loss(prob, u0 - h * d, tgt)) / (2 * h)
        assert abs(fd - np.sum(g * d)) <= 1e-9 * max(1.0, abs(fd))


def test_adjoint_nu_fd():
    prob = si.problem(2, 8, 3, 6, 0.4, nu=0.05, lam=0.5)
    rng = np.random.default_rng(6)
    u0 = rng.standard_normal((8, 8))
    tgt = rng.standard_normal((8, 8))
    _, gnu = adjoint.gradients(prob, u0, tgt)
    h = 1e-5
    lp = _loss(dict(prob, nu=prob["nu"] + h), u0, tgt)
    lm = _loss(dict(prob, nu=prob["nu"] - h), u0, tgt)
    fd = (lp - lm) / (2 * h)
    assert abs(fd - gnu) <= 1e-7 * max(1.0, abs(fd))
