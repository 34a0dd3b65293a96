"""The paper's smoother: GMRES preconditioned by ILU(0), spelled out plainly.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper smooths every level with a few iterations of GMRES preconditioned
by an incomplete LU factorisation with no fill (Sec. 4.2, "ILU(0)-PGMRES").
Here:

* ilu0: the factorisation restricted to the sparsity pattern of A, rows in
  order; for each row i and each k < i in the row, the multiplier
  a_ik / a_kk is formed and row k is subtracted on the entries of row i's
  pattern only (entries outside the pattern are dropped).  L is unit lower
  triangular, U upper triangular; (L U)_ij = A_ij on every (i, j) of the
  pattern.
* a smoothing step: nu iterations of GMRES on the left-preconditioned
  system (LU)^-1 A x = (LU)^-1 f from the current iterate (left
  preconditioning is PETSc's default, which the paper used), using the
  oracle's GMRES with an identity inner preconditioner.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import krylov


def ilu0(A):
    """ILU(0) of a square sparse matrix: (L, U) in CSR."""
    A = sp.csr_matrix(A, dtype=np.float64)
    A.sort_indices()
    n = A.shape[0]
    indptr, indices = A.indptr, A.indices
    data = A.data.copy()
    diag = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        for p in range(indptr[i], indptr[i + 1]):
            if indices[p] == i:
                diag[i] = p
                break
    if (diag < 0).any():
        raise ValueError("ILU(0) needs every diagonal entry in the pattern")
    for i in range(1, n):
        row = {int(indices[p]): p for p in range(indptr[i], indptr[i + 1])}
        for p in range(indptr[i], indptr[i + 1]):
            k = int(indices[p])
            if k >= i:
                break
            data[p] /= data[diag[k]]
            lik = data[p]
            for q in range(diag[k] + 1, indptr[k + 1]):
                t = row.get(int(indices[q]))
                if t is not None:
                    data[t] -= lik * data[q]
    F = sp.csr_matrix((data, indices.copy(), indptr.copy()), shape=A.shape)
    L = sp.tril(F, k=-1, format="csr") + sp.identity(n, format="csr")
    U = sp.triu(F, k=0, format="csr")
    return L, U


def ilu_solve(L, U, b):
    y = spla.spsolve_triangular(L, b, lower=True, unit_diagonal=True)
    return spla.spsolve_triangular(U, y, lower=False)


def ilu_gmres_smoother(A, nu):
    """A smoothing map (x, f) -> x' doing nu left-preconditioned GMRES
    iterations from x (vectors of any shape, flattened inside)."""
    A = sp.csr_matrix(A)
    L, U = ilu0(A)

    def prec_apply(v):
        return ilu_solve(L, U, A @ v)

    def smooth(x, f):
        shape = x.shape
        b = ilu_solve(L, U, np.asarray(f, dtype=np.float64).ravel())
        xo, _, _ = krylov.fgmres(prec_apply, lambda v: v, b, x0=x.ravel(), restart=nu, rtol=0.0, max_steps=nu)
        return xo.reshape(shape)

    return smooth
