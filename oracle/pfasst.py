"""PFASST (Sec. 4.1; Sec. 5.2, PFASST item), plain NumPy.

TEST INFRASTRUCTURE ONLY (see the package docstring).

PFASST runs SDC iterations on the collocation problem of every slab at once,
on a hierarchy of levels with a full approximation scheme (FAS) correction
between them; new initial values go forward in time after every sweep, and
only the coarsest level is serial in time (Sec. 4.1).  Level 0 is the
problem's grid with its M Radau nodes; every coarser level halves the
spatial elements (bisection, the space transfers of oracle.mg: full
weighting R_s, linear interpolation P_s) and has M = 1 (Sec. 5.2: M = 1 on
all coarse levels), with its own rediscretized L_l = nu Lap_l - lambda.

Level problem (collocation form, Sec. 2.1), slab n, node i:
  C_l(V)_{n,i} = V_{n,i} - dt (Q_l (x) L_l) V_n |_i - V_{n-1,M_l} = tau_{l,n,i}
with V_{-1,M} = u0_l (u0 on level 0, R_s u0_{l-1} below) and tau_0 = 0.

One iteration (a V-cycle over the levels):
  * levels l = 0 .. L-2, going down: nu SDC sweeps with the previous slab's end
    value from the incoming iterate (all slabs at once); then the FAS step
      Vt = R~ V_l = R_s V_{l,.,M_l}              (the end node, restricted)
      tau_{l+1} = R (tau_l - C_l(V_l)) + C_{l+1}(Vt),  R = R_s at the end node
    and V_{l+1} = Vt;
  * the coarsest level: nu sweeps in slab order, each slab taking the new end
    value of the slab before it (at M = 1 one such sweep solves the level
    exactly);
  * going up, l = L-2 .. 0: e_n = V_{l+1,n} - Vt_n (e_{-1} = 0), and the
    correction is interpolated in space and, between the slab's initial value
    (the previous slab's end) and its end, linearly in time:
      V_{l,n,i} += P_s ((1 - c_i) e_{n-1} + c_i e_n)
    then nu sweeps on l > 0 (level 0 sweeps at the start of the next
    iteration).

The SDC sweep is the one of oracle.sdc (implicit-Euler Q_Delta) with the
right-hand side tau; spatial solves are direct.  For the Allen-Cahn reaction
the sweep is semi-implicit (IMEX, Sec. 5.4: the reaction explicit, the
diffusion implicit): F = L + R with R(u) = gamma (u - u^3), L implicit with
Q_Delta as above and R explicit with the explicit-Euler Q_Delta^E, whose row
m weighs the values at the left ends of the node intervals,
Q_Delta^E[m][j] = c_{j+1} - c_j for j = 0 .. m-1 (j = 0 being the slab's
initial value, c_0 = 0).  In correction form, node by node:
  (I - dt dc_m L) d_m = r_m + dt sum_{j<m} dc_j L d_j
                        + dt sum_{j=0}^{m-1} dc_{j+1} (R(V_j + d_j) - R(V_j)),
with V_0 the initial value and d_0 its change (zero in the Jacobi sweep, the
change of the previous slab's end value in the serial one) and r_m the
collocation residual with the full F and the sweep's initial value.  The
fixed point is still the collocation solution.  The iteration stops on the
level-0 collocation residual relative to ||1 (x) u0||.  Readings: the paper
leaves the transfers, the time interpolation, the FAS form and the order of
sweeps to LibPFASST; the choices above are the standard ones of PFASST
(Emmett and Minion 2012) and of its multigrid description (Bolten, Moser
and Speck 2017).
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import mg, radau, space


def coarse_problem(prob):
    """The problem on the grid with half the elements (and M = 1)."""
    p = dict(prob)
    p["nx"] = [prob["nx"][0] // 2, prob["nx"][1] // 2 if prob["dim"] == 2 else 1]
    p["M"] = 1
    return p


class PLevel:
    def __init__(self, prob):
        self.prob = prob
        self.M, self.N, self.dt = prob["M"], prob["N"], prob["dt"]
        self.dim, self.bc = prob["dim"], prob.get("bc", "periodic")
        self.grid = space.grid_shape(prob)
        t = radau.tables(self.M)
        self.c, self.Q = t["c"], t["Q"]
        self.dc = np.diff(np.concatenate([[0.0], self.c]))
        self.L = space.linear_operator(prob)
        self.gamma = prob["gamma"] if prob.get("reaction", "linear") == "allen_cahn" else 0.0
        I = sp.identity(self.L.shape[0], format="csc")
        self.lu = [spla.splu((I - self.dt * self.dc[m] * self.L).tocsc()) for m in range(self.M)]

    @property
    def shape(self):
        return (self.N, self.M) + self.grid

    def R(self, v):
        """The explicit (reaction) part of F: gamma (u - u^3), zero when linear."""
        return self.gamma * (v - v ** 3)

    def F(self, V):
        """F = L + R applied to every node plane of V ([N][M][ny][nx])."""
        n = self.L.shape[0]
        flat = V.reshape(-1, n)
        return np.array([self.L @ v + self.R(v) for v in flat]).reshape(V.shape)

    def C(self, V, u0):
        """C_l(V): the collocation operator (full F) with u0 entering slab 0."""
        FV = self.F(V)
        out = np.empty_like(V)
        for k in range(self.N):
            prev = u0 if k == 0 else V[k - 1, self.M - 1]
            for i in range(self.M):
                out[k, i] = V[k, i] - self.dt * np.tensordot(self.Q[i], FV[k], axes=1) - prev
        return out

    def sweep(self, V, u0, tau, serial):
        """One SDC sweep on C_l(V) = tau: residual node by node, implicit-Euler
        substitution over the nodes (IMEX with a reaction); the previous
        slab's end value from V (serial False) or from the slabs already swept
        (serial True)."""
        n = self.L.shape[0]
        out = V.copy()
        for k in range(self.N):
            prev_old = (u0 if k == 0 else V[k - 1, self.M - 1]).reshape(n)
            prev = (u0 if k == 0 else (out if serial else V)[k - 1, self.M - 1]).reshape(n)
            FV = np.array([self.L @ V[k, j].reshape(n) + self.R(V[k, j].reshape(n)) for j in range(self.M)])
            acc = self.dt * self.dc[0] * (self.R(prev) - self.R(prev_old))
            for m in range(self.M):
                v = V[k, m].reshape(n)
                r = tau[k, m].reshape(n) + prev + self.dt * (self.Q[m] @ FV) - v
                d = self.lu[m].solve(r + acc)
                acc = acc + self.dt * self.dc[m] * (self.L @ d)
                if m + 1 < self.M:
                    acc = acc + self.dt * self.dc[m + 1] * (self.R(v + d) - self.R(v))
                out[k, m] = V[k, m] + d.reshape(self.grid)
        return out


def hierarchy(prob, levels):
    """PLevel list: the problem itself, then levels - 1 bisections in space
    with M = 1."""
    out = [PLevel(prob)]
    p = prob
    for _ in range(levels - 1):
        p = coarse_problem(p)
        out.append(PLevel(p))
    return out


def restrict_s(lev, v):
    return mg.restrict_space(v, lev.dim, lev.bc)


def prolong_s(lev, v):
    return mg.prolong_space(v, lev.dim, lev.bc)


def iteration(levs, u0s, U, nu=1):
    """One PFASST iteration from U (level-0 values [N][M][ny][nx])."""
    nl = len(levs)
    V = [np.asarray(U, dtype=np.float64).copy()] + [None] * (nl - 1)
    taus = [np.zeros(levs[0].shape)] + [None] * (nl - 1)
    Vt = [None] * (nl - 1)
    for l in range(nl - 1):
        f, c = levs[l], levs[l + 1]
        for _ in range(nu):
            V[l] = f.sweep(V[l], u0s[l], taus[l], serial=False)
        Vt[l] = restrict_s(f, V[l][:, f.M - 1])[:, None]
        r = taus[l] - f.C(V[l], u0s[l])
        taus[l + 1] = restrict_s(f, r[:, f.M - 1])[:, None] + c.C(Vt[l], u0s[l + 1])
        V[l + 1] = Vt[l].copy()
    for _ in range(nu):
        V[-1] = levs[-1].sweep(V[-1], u0s[-1], taus[-1], serial=True)
    for l in range(nl - 2, -1, -1):
        f = levs[l]
        e = (V[l + 1] - Vt[l])[:, 0]
        eprev = np.concatenate([np.zeros_like(e[:1]), e[:-1]])
        E = np.stack([(1.0 - f.c[i]) * eprev + f.c[i] * e for i in range(f.M)], axis=1)
        V[l] = V[l] + prolong_s(f, E)
        if l > 0:
            for _ in range(nu):
                V[l] = f.sweep(V[l], u0s[l], taus[l], serial=False)
    return V[0]


def initial_values(levs, u0):
    u0s = [np.asarray(u0, dtype=np.float64).reshape(levs[0].grid)]
    for l in range(len(levs) - 1):
        u0s.append(restrict_s(levs[l], u0s[-1]))
    return u0s


def rel_residual(lev, u0, U):
    """||C_0(U)|| / ||1 (x) u0|| (the collocation residual of level 0)."""
    r = lev.C(U, u0)
    return np.linalg.norm(r) / (np.sqrt(lev.M) * np.linalg.norm(u0))


def solve(prob, u0, levels=2, nu=1, rtol=1e-12, max_iter=100, U=None, history=None):
    levs = hierarchy(prob, levels)
    u0s = initial_values(levs, u0)
    U = np.zeros(levs[0].shape) if U is None else np.asarray(U, dtype=np.float64).copy()
    for k in range(max_iter):
        U = iteration(levs, u0s, U, nu)
        rel = rel_residual(levs[0], u0s[0], U)
        if history is not None:
            history.append(rel)
        if rel <= rtol:
            return U, k + 1
    return U, max_iter
