"""Iteration counts of the paper's three hierarchies on its 1D heat example,
with the block-Jacobi smoother and with the paper's ILU(0)-GMRES smoother.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Run as

    python -m oracle.paper_hierarchies [--M 3] [--hier SMG7] [--workers 6]

and it prints one JSON line per case.  The oracle's transfers are periodic,
so the problem is the periodic analogue of the paper's Neumann example
(Sec. 5.3): N_x = 1024 points on [0, 1), u0 = cos 2 pi x + 2 cos 6 pi x +
3 cos 8 pi x, nu = 1, T = 1, M = 1..5 with N_t from the paper's tables;
SMG^7 (space coarsening, 7 levels), STMG^5 (space and time, 5 levels), SMMG^7
(space and nodes, 7 levels) as in Sec. 5.2; each smoothing step is either one
block-Jacobi sweep (chunk 16 / 4, omega 0.8) or three ILU(0)-GMRES iterations
(oracle.ilu), one step before and one after the coarse correction; coarse
levels rediscretized (ours) or Galerkin products R A P (the paper's, assembled
with oracle.galerkin; ILU(0)-GMRES smoothing only).  Counts:
plain V-cycle iterations, FGMRES(30) steps with one V-cycle as the
preconditioner (true residual), and GMRES(30) steps on the left-
preconditioned system (preconditioned residual, PETSc's default), all to a
relative residual of 1e-9 (at most 60 / 100 / 100).
"""
import argparse
import json
import time
from concurrent.futures import ProcessPoolExecutor

import numpy as np

from . import galerkin, ilu, krylov, mg

NT = {1: 1024, 2: 256, 3: 32, 4: 16, 5: 8}
HIERS = {"SMG7": ("space", 7), "STMG5": ("spacetime", 5), "SMMG7": ("smmg", 7)}


def problem(M, nx=1024):
    return dict(dim=1, nx=[nx, 1], length=[1.0, 1.0], bc="periodic", nu=1.0, reaction="linear",
                **{"lambda": 0.0}, gamma=0.0, M=M, N=NT[M], dt=1.0 / NT[M])


def initial(prob):
    x = np.arange(prob["nx"][0]) / prob["nx"][0]
    return (np.cos(2 * np.pi * x) + 2 * np.cos(6 * np.pi * x) + 3 * np.cos(8 * np.pi * x))[None, :]


def run_case(M, hier, smoother, ops="redisc", max_cycles=60, max_steps=100, tol=1e-9):
    t0 = time.time()
    prob = problem(M)
    coarsen, L = HIERS[hier]
    if coarsen == "smmg" and M == 1:
        return dict(M=M, hier=hier, smoother=smoother, ops=ops, skipped="SMMG with M = 1 is SMG")
    levels, kinds = mg.hierarchy(prob, coarsen=coarsen, max_levels=L, fft_coarse=0, min_coarse=1)
    f = mg.rhs(levels, initial(prob)).ravel()
    nb = np.linalg.norm(f)
    if smoother == "bj":
        assert ops == "redisc"
        shape = levels[0].shape

        def cycle(x, g):
            return mg.vcycle(levels, kinds, x.reshape(shape), g.reshape(shape)).ravel()

        def apply(v):
            return levels[0].apply(v.reshape(shape)).ravel()
    else:
        As, Ps, Rs = galerkin.operators(levels, kinds, galerkin=(ops == "galerkin"))
        sms = [ilu.ilu_gmres_smoother(A, 3) for A in As[:-1]]
        coarse = galerkin.exact_coarse(As[-1])

        def cycle(x, g):
            return galerkin.vcycle(As, Ps, Rs, sms, coarse, x, g)

        def apply(v):
            return As[0] @ v
    U = np.zeros_like(f)
    cycles, rel = None, None
    for k in range(1, max_cycles + 1):
        U = cycle(U, f)
        rel = np.linalg.norm(f - apply(U)) / nb
        if not np.isfinite(rel) or rel > 1e3:
            break
        if rel <= tol:
            cycles = k
            break

    def precond(v):
        return cycle(np.zeros_like(v), v)

    _, hist, steps = krylov.fgmres(apply, precond, f, restart=30, rtol=tol, max_steps=max_steps)
    # left preconditioning, stop on the preconditioned residual
    _, lhist, lsteps = krylov.fgmres(lambda v: precond(apply(v)), lambda v: v, precond(f), restart=30, rtol=tol,
                                     max_steps=max_steps)
    return dict(M=M, N_t=prob["N"], hier=hier, smoother=smoother, ops=ops, levels=len(levels),
                left_steps=lsteps if lhist[-1] <= tol else None, left_rel=float(lhist[-1]),
                coarsest=[levels[-1].nx, levels[-1].N, levels[-1].M],
                vcycles=cycles, last_rel=float(rel) if rel is not None else None,
                fgmres_steps=steps if hist[-1] <= tol else None, fgmres_rel=float(hist[-1]),
                seconds=time.time() - t0)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--M", type=int, nargs="*", default=[1, 2, 3, 4, 5])
    ap.add_argument("--hier", nargs="*", default=list(HIERS))
    ap.add_argument("--variants", nargs="*", default=["bj:redisc", "ilu3:redisc", "ilu3:galerkin"])
    ap.add_argument("--workers", type=int, default=1)
    a = ap.parse_args()
    cases = [(M, h) + tuple(v.split(":")) for M in a.M for h in a.hier for v in a.variants]
    if a.workers > 1:
        with ProcessPoolExecutor(a.workers) as ex:
            for r in ex.map(run_case, *zip(*cases)):
                print(json.dumps(r), flush=True)
    else:
        for c in cases:
            print(json.dumps(run_case(*c)), flush=True)


if __name__ == "__main__":
    main()
