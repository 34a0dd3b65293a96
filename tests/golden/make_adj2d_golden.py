"""Writes the stored oracle values of the 256^2 adjoint workload.

Runs only the CPU oracle on the seeded inputs of `stmg_inputs` (u0 seed 4,
u_tgt seed 40): the sequential Radau IIA stepper (`oracle.stepper`) for the
forward solution and its discrete adjoint (`oracle.adjoint`, transposed
stage solves backward in time) for the gradients of
L = || u(T) - u_tgt ||^2.  Stores, in `adj2d_256_golden.npz`:
  uT        u(T) of the forward solve             (256 x 256)
  loss      L
  grad_u0   dL/du0                                 (256 x 256)
  grad_nu   dL/dnu
  seconds   oracle wall time (forward, adjoint)
Usage: python tests/golden/make_adj2d_golden.py   (from the repository root;
about two minutes and 12 GB of memory on one host core).
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import stmg_inputs as si  # noqa: E402
from oracle import adjoint, stepper  # noqa: E402


def main():
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "adj2d_256_golden.npz")
    prob = si.config("adj2d")
    u0 = si.initial("adj2d", prob)
    tgt = si.u_tgt_adj2d(prob)
    t0 = time.perf_counter()
    U = stepper.solve_linear(prob, u0)
    t1 = time.perf_counter()
    g_u0, g_nu = adjoint.gradients(prob, u0, tgt, U=U)
    t2 = time.perf_counter()
    np.savez(out, uT=U[-1, -1], loss=adjoint.loss(prob, U, tgt), grad_u0=g_u0, grad_nu=g_nu,
             seconds=np.array([t1 - t0, t2 - t1]))
    print("wrote %s (forward %.0f s, adjoint %.0f s)" % (out, t1 - t0, t2 - t1))


if __name__ == "__main__":
    main()
