"""Writes the stored oracle values of the 512^2 Allen-Cahn workload.

Runs only the CPU oracle (`oracle.stepper.solve_allen_cahn`, sequential
Radau IIA with Newton per step and Jacobian reuse) on the seeded input of
`stmg_inputs` and stores, in `ac2d_512_golden.npz`:
  uT      u(T) = U[N-1, M-1]            (512 x 512, FP64)
  umid    U[N/2-1, M-1], the solution at t = T/2
  norms   ||U[n, m]||_2 for every slab n and node m   (N x M)
  sums    sum_x U[n, m](x)                            (N x M)
  seconds oracle wall time, factorizations, Newton iterations
Usage: python tests/golden/make_ac2d_golden.py [--nx 512 --N 512 --T 2]
(from the repository root).  The full run takes about an hour or more on
one host core and needs about 12 GB of memory.
"""
import argparse
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import stmg_inputs as si  # noqa: E402
from oracle import stepper  # noqa: E402


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--nx", type=int, default=512)
    ap.add_argument("--N", type=int, default=512)
    ap.add_argument("--T", type=float, default=2.0)
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                  "ac2d_512_golden.npz"))
    a = ap.parse_args()
    prob = si.problem(2, a.nx, 3, a.N, a.T, nu=1e-3, gamma=1.0, reaction="allen_cahn")
    u0 = si.u0_ac2d(prob, 3)
    stats = {"its": 0, "factors": 0}
    t0 = time.perf_counter()

    def log(n, its, factors):
        stats["its"] += its
        stats["factors"] = factors
        if n % 8 == 0 or n == prob["N"] - 1:
            print("step %d/%d: %d Newton its, %d factorizations, %.0f s"
                  % (n + 1, prob["N"], its, factors, time.perf_counter() - t0), flush=True)

    U = stepper.solve_allen_cahn(prob, u0, reuse=True, log=log)
    secs = time.perf_counter() - t0
    N = prob["N"]
    flat = U.reshape(N, prob["M"], -1)
    np.savez(a.out, uT=U[-1, -1], umid=U[N // 2 - 1, -1],
             norms=np.sqrt((flat ** 2).sum(axis=2)), sums=flat.sum(axis=2),
             seconds=secs, factors=stats["factors"], newton_its=stats["its"],
             shape=np.array(U.shape))
    print("wrote %s (%.0f s, %d factorizations, %d Newton its)" % (a.out, secs, stats["factors"], stats["its"]))


if __name__ == "__main__":
    main()
