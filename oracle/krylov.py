"""Restarted flexible GMRES with the V-cycle as right preconditioner.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper stops its multigrid runs on a preconditioned Krylov residual
(Sec. 5, the set-up of the numerical examples): the multigrid cycle sits
inside a Krylov method rather than being iterated on its own.  We read this
as restarted GMRES with one V-cycle from a zero guess as the right
preconditioner, in the flexible form (Saad, 1993): the preconditioned
directions z_j = M_j^-1 v_j are stored and the update is taken from them, so
the preconditioner may change from one step to the next (an FP32 V-cycle, a
cycle whose coarse solve is inexact) and the quantity minimised over the
search space is the true residual ||b - A x||_2.

One restart cycle, written in the order of the method:

  r0 = b - A x0,  beta = ||r0||,  v_1 = r0 / beta
  for j = 1..m:
      z_j = precond(v_j)
      w = A z_j
      h_ij = (w, v_i), w -= h_ij v_i        for i = 1..j (Gram-Schmidt)
      h_{j+1,j} = ||w||,  v_{j+1} = w / h_{j+1,j}
      y_j = argmin_y || beta e_1 - H_j y ||  ((j+1) x j Hessenberg H_j)
      stop the cycle when that minimum is <= tol
  x = x0 + [z_1 .. z_k] y_k

The small least-squares problem is handed to numpy.linalg.lstsq at every
step; no Givens rotations, no orthogonalisation tricks.  Gram-Schmidt is
the modified form, repeated once (a second pass over the same basis) so the
basis stays orthogonal to rounding for the restart lengths used here.
"""
import numpy as np


def fgmres(apply, precond, b, x0=None, restart=10, rtol=1e-9, max_steps=200):
    """Solve A x = b.

    apply(x) -> A x;  precond(v) -> z (any map; called once per step).
    Stops when ||b - A x|| <= rtol ||b|| (the least-squares estimate ends a
    cycle, the true residual of the updated x decides) or after `max_steps`
    Arnoldi steps in total.  Returns (x, hist, steps): hist[k] is the
    least-squares residual after k steps relative to ||b|| (hist[0] the
    initial one; at a restart the entry is the true residual instead).
    """
    b = np.asarray(b, dtype=np.float64)
    shape = b.shape
    bf = b.ravel()
    nb = np.linalg.norm(bf)
    scale = nb if nb > 0 else 1.0
    x = np.zeros_like(bf) if x0 is None else np.array(x0, dtype=np.float64).ravel()

    def A(v):
        return np.asarray(apply(v.reshape(shape)), dtype=np.float64).ravel()

    def P(v):
        return np.asarray(precond(v.reshape(shape)), dtype=np.float64).ravel()

    steps = 0
    hist = []
    while True:
        r = bf - A(x)
        beta = np.linalg.norm(r)
        if hist:
            hist[-1] = beta / scale
        else:
            hist.append(beta / scale)
        if beta <= rtol * scale or steps >= max_steps or beta == 0.0:
            break
        V = [r / beta]
        Z = []
        H = np.zeros((restart + 1, restart))
        e1 = np.zeros(restart + 1)
        e1[0] = beta
        y = np.zeros(0)
        for j in range(restart):
            Z.append(P(V[j]))
            w = A(Z[j])
            for _ in range(2):
                for i in range(j + 1):
                    hij = np.dot(w, V[i])
                    H[i, j] += hij
                    w = w - hij * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            steps += 1
            Hj = H[:j + 2, :j + 1]
            y = np.linalg.lstsq(Hj, e1[:j + 2], rcond=None)[0]
            res = np.linalg.norm(e1[:j + 2] - Hj @ y)
            hist.append(res / scale)
            if H[j + 1, j] == 0.0 or res <= rtol * scale or steps >= max_steps:
                break
            V.append(w / H[j + 1, j])
        for j in range(len(y)):
            x = x + y[j] * Z[j]
    return x.reshape(shape), hist, steps


def solve(prob, u0, rtol=1e-9, max_steps=200, restart=10, left=False, **kw):
    """FGMRES on the all-at-once system with one oracle V-cycle (from zero)
    as the preconditioner; keyword arguments as for `mg.solve`.  With left,
    GMRES on the left-preconditioned system M A x = M f (M = one V-cycle):
    the residual it minimises and stops on is the preconditioned one, and
    hist is relative to ||M f||."""
    from . import mg
    hk = {k: kw.pop(k) for k in ("coarsen", "mu_crit", "min_coarse", "max_levels", "fft_coarse") if k in kw}
    levels, kinds = mg.hierarchy(prob, **hk)
    f = mg.rhs(levels, u0)

    def precond(v):
        return mg.vcycle(levels, kinds, np.zeros(levels[0].shape), v, **kw)

    if left:
        return fgmres(lambda v: precond(levels[0].apply(v)), lambda v: v, precond(f), restart=restart,
                      rtol=rtol, max_steps=max_steps)
    return fgmres(levels[0].apply, precond, f, restart=restart, rtol=rtol, max_steps=max_steps)
