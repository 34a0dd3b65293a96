"""Right Gauss-Radau collocation tables, computed in mpmath.

Paper, Sec. 2.1 (collocation form): M right Radau nodes with t_M = T_{n+1};
q_{mj} = (1/dt) * integral from T_n to t_m of the Lagrange polynomial l_j.
Paper, Sec. 2.2, Eqs. (Kq) and (Mq): the DG-in-time matrices
  K_q[i,j] = -int l_i'(t) l_j(t) dt + l_i(T_{n+1}) l_j(T_{n+1}),
  M_q[i,j] =  int l_i(t) l_j(t) dt,
  J_q[i,j] =  l_i(T_n) l_j(T_{n+1}).
All integrals are over one step; on the unit step [0, 1] K_q and J_q do not
depend on dt and M_q scales with dt.

Everything is done with exact polynomial arithmetic in mpmath at `dps`
digits and returned as float64 numpy arrays (or as mpmath matrices on
request).  This is test infrastructure, not the library's table code.
"""
import mpmath as mp
import numpy as np

_DPS = 40


def _legendre_coeffs(n):
    """Monomial coefficients (ascending) of the Legendre polynomial P_n(x)."""
    p0 = [mp.mpf(1)]
    if n == 0:
        return p0
    p1 = [mp.mpf(0), mp.mpf(1)]
    for k in range(1, n):
        # (k+1) P_{k+1} = (2k+1) x P_k - k P_{k-1}
        xp = [mp.mpf(0)] + p1
        pm = p0 + [mp.mpf(0)] * (len(xp) - len(p0))
        p2 = [((2 * k + 1) * a - k * b) / (k + 1) for a, b in zip(xp, pm)]
        p0, p1 = p1, p2
    return p1


def _peval(c, x):
    s = mp.mpf(0)
    for a in reversed(c):
        s = s * x + a
    return s


def _pmul(a, b):
    out = [mp.mpf(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _pint(c, lo, hi):
    """Exact integral of a polynomial from lo to hi."""
    anti = [mp.mpf(0)] + [a / (k + 1) for k, a in enumerate(c)]
    return _peval(anti, hi) - _peval(anti, lo)


def _pder(c):
    return [k * c[k] for k in range(1, len(c))] or [mp.mpf(0)]


def nodes(M, dps=_DPS, as_mp=False):
    """Right Radau nodes on (0, 1]: the roots of P_M(2t-1) - P_{M-1}(2t-1).

    Sec. 2.1: T_n < t_1 < ... < t_M = T_{n+1}.  The last node is exactly 1.
    """
    with mp.workdps(dps + 10):
        pM = _legendre_coeffs(M)
        pM1 = _legendre_coeffs(M - 1)
        f = lambda t: _peval(pM, 2 * t - 1) - _peval(pM1, 2 * t - 1)
        # starting guesses from a float64 root finder, polished in mpmath
        lc = np.zeros(M + 1)
        lc[M] = 1.0
        lc[M - 1] -= 1.0
        guesses = np.sort((np.polynomial.legendre.legroots(lc).real + 1.0) / 2.0)
        c = []
        for g in guesses:
            c.append(mp.findroot(f, mp.mpf(g)))
        c[-1] = mp.mpf(1)
        c = sorted(c)
        if as_mp:
            return c
        return np.array([float(x) for x in c])


def lagrange_basis(c):
    """Monomial coefficients of the Lagrange polynomials at nodes c."""
    M = len(c)
    basis = []
    for j in range(M):
        p = [mp.mpf(1)]
        for k in range(M):
            if k != j:
                d = c[j] - c[k]
                p = _pmul(p, [-c[k] / d, 1 / d])
        basis.append(p)
    return basis


def tables(M, dps=_DPS):
    """Collocation and DG tables on the unit step.

    Returns a dict of float64 arrays:
      c   nodes (M,)
      Q   q_{mj} = int_0^{c_m} l_j                  (Sec. 2.1)
      b   last row of Q (the quadrature weights)
      Kq  -int_0^1 l_i' l_j + l_i(1) l_j(1)        (Eq. Kq)
      Mq1 int_0^1 l_i l_j  (M_q = dt * Mq1)          (Eq. Mq)
      Jq  l_i(0) l_j(1)                              (Eq. Mq)
      l0  l_i(0)
    """
    with mp.workdps(dps + 10):
        c = nodes(M, dps, as_mp=True)
        L = lagrange_basis(c)
        Q = mp.matrix(M, M)
        Kq = mp.matrix(M, M)
        Mq1 = mp.matrix(M, M)
        Jq = mp.matrix(M, M)
        for i in range(M):
            for j in range(M):
                Q[i, j] = _pint(L[j], 0, c[i])
                Kq[i, j] = -_pint(_pmul(_pder(L[i]), L[j]), 0, 1) + _peval(L[i], 1) * _peval(L[j], 1)
                Mq1[i, j] = _pint(_pmul(L[i], L[j]), 0, 1)
                Jq[i, j] = _peval(L[i], 0) * _peval(L[j], 1)
        l0 = [_peval(L[i], 0) for i in range(M)]
        tof = lambda A: np.array([[float(A[i, j]) for j in range(M)] for i in range(M)])
        Qf = tof(Q)
        return dict(c=np.array([float(x) for x in c]), Q=Qf, b=Qf[-1].copy(),
                    Kq=tof(Kq), Mq1=tof(Mq1), Jq=tof(Jq),
                    l0=np.array([float(x) for x in l0]))


def stability_function(Q, z):
    """R(z) = e_M^T (I - z Q)^{-1} 1 : one Radau IIA step applied to y' = z y."""
    M = Q.shape[0]
    return np.linalg.solve(np.eye(M) - z * Q, np.ones(M))[-1]
