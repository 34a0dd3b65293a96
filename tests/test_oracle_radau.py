"""Oracle pins: Radau tables against textbook closed forms and identities."""
import json
import math
import os

import numpy as np
import pytest

from oracle import radau

GOLD = os.path.join(os.path.dirname(__file__), "golden", "radau_iia_closed_forms.json")


def _ev(expr, z=0.0):
    return eval(expr, {"s": math.sqrt(6.0), "z": z})


@pytest.mark.parametrize("M", [1, 2, 3])
def test_tableau_closed_form(M):
    g = json.load(open(GOLD))["M%d" % M]
    t = radau.tables(M)
    c = np.array([_ev(e) for e in g["c"]])
    A = np.array([[_ev(e) for e in row] for row in g["A"]])
    assert np.abs(t["c"] - c).max() < 1e-15
    assert np.abs(t["Q"] - A).max() < 1e-15
    assert np.abs(t["b"] - A[-1]).max() < 1e-15


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5, 6, 7, 8])
def test_order_conditions(M):
    t = radau.tables(M)
    c, Q, b = t["c"], t["Q"], t["b"]
    assert abs(c[-1] - 1.0) == 0.0
    assert np.all(np.diff(c) > 0) and c[0] > 0
    # quadrature exactness B(2M-1): sum_j b_j c_j^{k-1} = 1/k
    for k in range(1, 2 * M):
        assert abs(b @ c ** (k - 1) - 1.0 / k) < 1e-13
    # stage order C(M): sum_j q_mj c_j^{k-1} = c_m^k / k
    for k in range(1, M + 1):
        assert np.abs(Q @ c ** (k - 1) - c ** k / k).max() < 1e-13
    # B(2M) fails: the nodes are not Gauss nodes
    assert abs(b @ c ** (2 * M - 1) - 1.0 / (2 * M)) > 1e-12


@pytest.mark.parametrize("M", [1, 2, 3, 4, 5])
def test_dg_equals_collocation(M):
    """Z1-Z3 readings: M_q = dt diag(b), J_q = l(0) e_M^T, diag(b)^{-1} K_q = Q^{-1}."""
    t = radau.tables(M)
    assert np.abs(t["Mq1"] - np.diag(t["b"])).max() < 1e-15
    eM = np.zeros(M)
    eM[-1] = 1
    assert np.abs(t["Jq"] - np.outer(t["l0"], eM)).max() < 1e-13
    lhs = np.linalg.solve(np.diag(t["b"]), t["Kq"])
    assert np.abs(lhs - np.linalg.inv(t["Q"])).max() < 1e-11 * max(1, np.abs(lhs).max())
    # l(0) = diag(b) Q^{-1} 1
    assert np.abs(t["l0"] - np.diag(t["b"]) @ np.linalg.solve(t["Q"], np.ones(M))).max() < 1e-11


@pytest.mark.parametrize("M", [1, 2, 3])
@pytest.mark.parametrize("z", [-0.01, -1.0, -37.5, -1e4, 0.3])
def test_stability_function_pade(M, z):
    g = json.load(open(GOLD))["pade"]["M%d" % M]
    R = radau.stability_function(radau.tables(M)["Q"], z)
    assert abs(R - _ev(g, z)) <= 1e-14 * max(1.0, abs(R))


def test_a_stability_and_stiff_decay():
    for M in range(1, 6):
        Q = radau.tables(M)["Q"]
        for z in [-1e-3, -1.0, -10.0, -1e3, -1e6, 1j * 5, -2 + 3j]:
            assert abs(radau.stability_function(Q, z)) <= 1.0 + 1e-14
        assert abs(radau.stability_function(Q, -1e9)) < 1e-6  # L-stable
