"""The multigrid components, spelled out plainly in NumPy.

This is the oracle for the pieces of the V-cycle (one smoothing sweep, one
restriction, one prolongation, one coarsest solve, one V-cycle), used to
check the GPU kernels element by element.  The paper fixes the system
(Eq. st_system), the transfer structure I = T (x) M (x) S (Eq.
space_time_tran) with bisection stencils [1 2 1]/4 (Sec. 5.2, SMG and STMG
items), a block-Jacobi smoother over time slabs (Sec. 4.2), an exact
coarsest solve and Newton around the linear solver.  What it leaves open
is read as follows (each reading is listed with its reason in the design
notes):

* operator: the DG form with the lumped mass divided out,
    (A U)_{n,i} = sum_j Kq[i,j] U_{n,j} + dt b_i (-nu Lap + lam) U_{n,i}
                  - [n > 0] l_i(0) U_{n-1,M}
  with M_q = dt diag(b) and J_q = l(0) e_M^T (exact for right Radau nodes);
  coarse levels rediscretize with their own h and dt;
* smoother: damped block-Jacobi over chunks of `chunk` consecutive slabs;
  each chunk is inverted approximately by forward substitution in time
  with a point-block (M x M) diagonal in space:
    d_n = B^{-1} (r_n + [n mod chunk != 0] l(0) d_{n-1,M}),  U += omega d,
  B = Kq + dt diag(b) (2 nu/hx^2 + 2 nu/hy^2 + lam);  chunk = 1 is the
  plain point-block Jacobi over slabs; the coarser levels use their own
  (shorter) `chunk_coarse`;
* space transfer: full weighting [1 2 1]/4 per dimension and linear
  interpolation, vertex-centred (coarse point X is fine point 2X); on
  Neumann grids (the paper's boundary condition, Sec. 3: nx elements, nx + 1
  points, lumped linear FE) the end points use the mirror value as their
  missing neighbour, in the Laplacian and in the restriction alike.  For the
  restriction this is the FE-consistent R = M_c^-1 P^T M_f with the lumped
  masses (half weight at the end points);
* time transfer: slab n is identified with its end point T_{n+1}; coarse
  slab J is fine slab 2J+1, the stencil is [1 2 1]/2 (restriction = P^T,
  scaled so that rediscretized coarse operators match R A P), T_0 carries a
  zero correction, the node index is left alone (M_l^{l+1} = I);
* semi-coarsening: at each level coarsen in space if
  mu = nu dt / h^2 >= mu_crit, else in time (Sec. 4.2: mu << 1 -> time,
  mu >> 1 -> space), falling back to the other direction when one is not
  possible, until the level holds at most `min_coarse` unknowns.  The paper
  gives no threshold; mu_crit = 0.5 by default.
* node coarsening (SMMG, Sec. 5.2): each level coarsens in space (as SMG) and
  lowers M by one until M = 1.  The paper calls the node transfer M_l^{l+1} a linear
  interpolation; we read it as Lagrange interpolation from the coarse Radau
  nodes to the fine ones, P[i, k] = l_k^coarse(c_i^fine) (exact for the coarse
  polynomials, the M-coarsening PFASST uses), with restriction R = P^T.  With
  these, P^T A_fine P equals the rediscretized coarse operator exactly in the
  time structure (K_q, the Radau mass diag(b), l(0) and the end-node
  coupling), so rediscretization and Galerkin agree for this transfer.
* coarsest level: coarsening also stops at the first level below the finest
  whose planes hold at most `fft_plane` points (or, in 2D, whose sides are
  powers of two of at most `fft_side` points) and which holds at most
  `fft_coarse` unknowns (0 disables the rule).  This is a choice of where the
  exact coarse solve sits (the paper fixes the number of levels per run); the
  exact solve itself is the same direct slab-by-slab solve on any level
  (one LU factorization of the slab matrix: dense up to 4096 unknowns per
  slab, sparse above).
"""
import numpy as np
import scipy.linalg
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import radau


class Level:
    def __init__(self, nx, ny, N, M, dt, nu, lam, length, dim, tab, bc="periodic"):
        # nx, ny: grid points; elements = points (periodic) or points - 1 (Neumann)
        self.nx, self.ny, self.N, self.M, self.dt = nx, ny, N, M, dt
        self.nu, self.lam, self.dim, self.bc = nu, lam, dim, bc
        self.length = [float(length[0]), float(length[1])]
        e = 0 if bc == "periodic" else 1
        self.ex, self.ey = nx - e, (ny - e if dim == 2 else 1)
        self.hx = length[0] / self.ex
        self.hy = length[1] / self.ey if dim == 2 else 1.0
        self.Kq, self.b, self.l0 = tab["Kq"], tab["b"], tab["l0"]
        cx = nu / self.hx ** 2
        cy = nu / self.hy ** 2 if dim == 2 else 0.0
        self.cx, self.cy = cx, cy
        dgl = 2 * cx + 2 * cy + lam
        self.B = self.Kq + dt * np.diag(self.b) * dgl
        self.Binv = np.linalg.inv(self.B)
        self.Pm = None  # node prolongation to the next coarser level (node coarsening only)

    @property
    def shape(self):
        return (self.N, self.M, self.ny, self.nx)

    def lap(self, U):
        out = self.cx * (_left(U, -1, self.bc) + _right(U, -1, self.bc) - 2 * U)
        if self.dim == 2:
            out = out + self.cy * (_left(U, -2, self.bc) + _right(U, -2, self.bc) - 2 * U)
        return out

    def apply(self, U):
        out = np.einsum("ij,njyx->niyx", self.Kq, U)
        out = out + self.dt * self.b[None, :, None, None] * (-self.lap(U) + self.lam * U)
        out[1:] -= self.l0[None, :, None, None] * U[:-1, -1][:, None]
        return out

    def smooth(self, U, f, omega, chunk):
        r = f - self.apply(U)
        d = np.zeros_like(U)
        for n in range(self.N):
            rhs = r[n].copy()
            if n % chunk != 0:
                rhs = rhs + self.l0[:, None, None] * d[n - 1, -1][None]
            d[n] = np.einsum("ij,jyx->iyx", self.Binv, rhs)
        return U + omega * d

    def slab_matrix(self):
        """Dense diagonal block of the level operator (one slab)."""
        K = self.M * self.ny * self.nx
        E = np.eye(K).reshape(K, 1, self.M, self.ny, self.nx)
        cols = []
        for k in range(K):
            e = E[k]
            v = np.einsum("ij,njyx->niyx", self.Kq, e) + \
                self.dt * self.b[None, :, None, None] * (-self.lap(e) + self.lam * e)
            cols.append(v.reshape(-1))
        return np.array(cols).T

    def slab_matrix_sparse(self):
        """The same slab block assembled from its Kronecker structure,
        Kq (x) I + diag(dt b) (x) (-Lap + lam I), with the periodic 1D second
        differences Lap = cx D_x (+ cy D_y) on the [y][x] ordering."""
        def d2(n, c):
            I = sp.identity(n, format="csr")
            if self.bc == "periodic":
                S = sp.csr_matrix((np.ones(n), (np.arange(n), (np.arange(n) + 1) % n)), shape=(n, n))
                return c * (S + S.T - 2 * I)
            # Neumann: the mirror point doubles the inner neighbour at both ends
            up = np.ones(n - 1)
            lo = np.ones(n - 1)
            up[0] = 2.0
            lo[-1] = 2.0
            return c * (sp.diags([lo, up], [-1, 1], shape=(n, n), format="csr") - 2 * I)
        lap = sp.kron(sp.identity(self.ny), d2(self.nx, self.cx))
        if self.dim == 2:
            lap = lap + sp.kron(d2(self.ny, self.cy), sp.identity(self.nx))
        P = self.nx * self.ny
        return sp.csc_matrix(sp.kron(self.Kq, sp.identity(P)) +
                             sp.kron(self.dt * np.diag(self.b), -lap + self.lam * sp.identity(P)))

    def exact_solve(self, f, dense=None):
        """Slab after slab, A_slab U_n = f_n + l(0) (x) U_{n-1,M}, with one LU
        factorization of the (shared) slab matrix: dense for at most 4096
        unknowns per slab, sparse (SuperLU) above, or as `dense` says."""
        if dense is None:
            dense = self.M * self.nx * self.ny <= 4096
        key = "_lu" if dense else "_splu"
        if getattr(self, key, None) is None:
            if dense:
                self._lu = scipy.linalg.lu_factor(self.slab_matrix())
            else:
                self._splu = spla.splu(self.slab_matrix_sparse())
        U = np.zeros(self.shape)
        for n in range(self.N):
            rhs = f[n].copy()
            if n > 0:
                rhs = rhs + self.l0[:, None, None] * U[n - 1, -1][None]
            b = rhs.reshape(-1)
            x = scipy.linalg.lu_solve(self._lu, b) if dense else self._splu.solve(b)
            U[n] = x.reshape(self.M, self.ny, self.nx)
        return U


def _left(U, axis, bc):
    """The neighbour at index i - 1 along `axis`: periodic wrap, or the mirror
    point i + 1 at the first point (Neumann)."""
    if bc == "periodic":
        return np.roll(U, 1, axis)
    n = U.shape[axis]
    idx = np.concatenate(([1], np.arange(n - 1)))
    return np.take(U, idx, axis=axis)


def _right(U, axis, bc):
    """The neighbour at index i + 1: periodic wrap, or the mirror point i - 1
    at the last point (Neumann)."""
    if bc == "periodic":
        return np.roll(U, -1, axis)
    n = U.shape[axis]
    idx = np.concatenate((np.arange(1, n), [n - 2]))
    return np.take(U, idx, axis=axis)


def restrict_space(r, dim, bc="periodic"):
    r = 0.25 * _left(r, -1, bc) + 0.5 * r + 0.25 * _right(r, -1, bc)
    r = r[..., ::2]
    if dim == 2:
        r = 0.25 * _left(r, -2, bc) + 0.5 * r + 0.25 * _right(r, -2, bc)
        r = r[..., ::2, :]
    return r


def _interp_axis(e, axis, bc):
    """Linear interpolation to the grid with half the spacing along `axis`:
    fine 2X = coarse X, fine 2X + 1 = mean of coarse X and X + 1 (periodic:
    nc -> 2 nc points; Neumann: nc -> 2 nc - 1 points, both ends kept)."""
    e = np.moveaxis(e, axis, -1)
    nc = e.shape[-1]
    nf = 2 * nc if bc == "periodic" else 2 * nc - 1
    f = np.zeros(e.shape[:-1] + (nf,))
    f[..., ::2] = e
    nxt = np.roll(e, -1, -1) if bc == "periodic" else e[..., 1:]
    f[..., 1::2] = 0.5 * ((e if bc == "periodic" else e[..., :-1]) + nxt)
    return np.moveaxis(f, -1, axis)


def prolong_space(e, dim, bc="periodic"):
    f = _interp_axis(e, -1, bc)
    if dim == 2:
        f = _interp_axis(f, -2, bc)
    return f


def restrict_time(r):
    N = r.shape[0]
    c = np.zeros((N // 2,) + r.shape[1:])
    for J in range(N // 2):
        c[J] = 0.5 * r[2 * J] + r[2 * J + 1]
        if 2 * J + 2 < N:
            c[J] += 0.5 * r[2 * J + 2]
    return c


def prolong_time(e):
    Nc = e.shape[0]
    f = np.zeros((2 * Nc,) + e.shape[1:])
    for J in range(Nc):
        f[2 * J + 1] = e[J]
        f[2 * J] = 0.5 * e[J] + (0.5 * e[J - 1] if J > 0 else 0.0)
    return f


def node_prolongation(Mf, Mc):
    """P (Mf x Mc): the coarse Lagrange basis at the Radau nodes of the fine
    level, P[i, k] = prod_{j != k} (c_i - C_j) / (C_k - C_j)."""
    cf = radau.tables(Mf)["c"]
    cc = radau.tables(Mc)["c"]
    P = np.ones((Mf, Mc))
    for k in range(Mc):
        for j in range(Mc):
            if j != k:
                P[:, k] *= (cf - cc[j]) / (cc[k] - cc[j])
    return P


def hierarchy(prob, coarsen="auto", mu_crit=0.5, min_coarse=64, max_levels=30, fft_coarse=1 << 22,
              fft_plane=1024, fft_side=64):
    """Level list and the coarsening kind between consecutive levels.

    kinds[l] is 's' (space), 't' (time) or 'st' (both) for the step l -> l+1.
    Periodic or Neumann grids; space coarsening halves the element count
    (which must be even and at least 4); the Fourier coarsest-level rule is
    for periodic grids only.
    """
    dim = prob["dim"]
    bc = prob.get("bc", "periodic")
    e = 0 if bc == "periodic" else 1
    nx = prob["nx"][0] + e
    ny = prob["nx"][1] + e if dim == 2 else 1
    N, dt = prob["N"], prob["dt"]
    mk = lambda nx_, ny_, N_, dt_, M_: Level(nx_, ny_, N_, M_, dt_, prob["nu"], prob.get("lambda", 0.0),
                                             prob["length"], dim, radau.tables(M_), bc)
    levels = [mk(nx, ny, N, dt, prob["M"])]
    kinds = []
    while len(levels) < max_levels:
        l = levels[-1]
        if l.M * l.nx * l.ny * l.N <= min_coarse:
            break
        pow2_sides = dim == 2 and all(n >= 2 and n & (n - 1) == 0 and n <= fft_side for n in (l.nx, l.ny))
        if bc == "periodic" and len(levels) > 1 and (l.nx * l.ny <= fft_plane or pow2_sides) and \
                l.M * l.nx * l.ny * l.N <= fft_coarse:
            break
        can_s = l.ex % 2 == 0 and l.ex >= 4 and (dim == 1 or (l.ey % 2 == 0 and l.ey >= 4))
        can_t = l.N % 2 == 0
        mu = l.nu * l.dt / min(l.hx, l.hy if dim == 2 else l.hx) ** 2
        if coarsen == "space":
            k = "s" if can_s else None
        elif coarsen == "smmg":
            k = ("sm" if l.M > 1 else "s") if can_s else None
        elif coarsen == "spacetime":
            k = "st" if (can_s and can_t) else ("s" if can_s else ("t" if can_t else None))
        else:
            if mu >= mu_crit and can_s:
                k = "s"
            elif can_t:
                k = "t"
            elif can_s:
                k = "s"
            else:
                k = None
        if k is None:
            break
        nx2 = l.ex // 2 + e if "s" in k else l.nx
        ny2 = (l.ey // 2 + e if dim == 2 else 1) if "s" in k else l.ny
        N2 = l.N // 2 if "t" in k else l.N
        dt2 = 2 * l.dt if "t" in k else l.dt
        M2 = l.M - 1 if "m" in k else l.M
        l.Pm = node_prolongation(l.M, M2) if "m" in k else None
        levels.append(mk(nx2, ny2, N2, dt2, M2))
        kinds.append(k)
    return levels, kinds


def restrict(r, kind, dim, Pm=None, bc="periodic"):
    if "s" in kind:
        r = restrict_space(r, dim, bc)
    if "t" in kind:
        r = restrict_time(r)
    if "m" in kind:
        r = np.einsum("ik,niyx->nkyx", Pm, r)
    return r


def prolong(e, kind, dim, Pm=None, bc="periodic"):
    if "m" in kind:
        e = np.einsum("ik,nkyx->niyx", Pm, e)
    if "t" in kind:
        e = prolong_time(e)
    if "s" in kind:
        e = prolong_space(e, dim, bc)
    return e


def vcycle(levels, kinds, U, f, omega=0.8, chunk=16, nu_pre=1, nu_post=1, l=0, chunk_coarse=4,
           smoothers=None):
    """One V-cycle; the smoother's block length is `chunk` slabs on the finest
    level and `chunk_coarse` on the coarser ones.  `smoothers`, if given, is
    one map (U, f) -> U' per level that replaces the block-Jacobi sweep (each
    pre- and post-smoothing step calls it once)."""
    lev = levels[l]
    if l == len(levels) - 1:
        return lev.exact_solve(f)
    ch = chunk if l == 0 else chunk_coarse

    def sweep(V):
        return smoothers[l](V, f) if smoothers is not None else lev.smooth(V, f, omega, ch)

    for _ in range(nu_pre):
        U = sweep(U)
    r = f - lev.apply(U)
    fc = restrict(r, kinds[l], lev.dim, lev.Pm, lev.bc)
    ec = vcycle(levels, kinds, np.zeros(levels[l + 1].shape), fc, omega, chunk, nu_pre, nu_post, l + 1,
                chunk_coarse, smoothers)
    U = U + prolong(ec, kinds[l], lev.dim, lev.Pm, lev.bc)
    for _ in range(nu_post):
        U = sweep(U)
    return U


def level_problem(lev):
    """The problem statement a level rediscretizes (periodic, same domain)."""
    nx = [lev.ex, lev.ey if lev.dim == 2 else 1]
    return dict(dim=lev.dim, nx=nx, length=list(lev.length), bc=lev.bc, nu=lev.nu,
                reaction="linear", **{"lambda": lev.lam}, gamma=0.0, M=lev.M, N=lev.N, dt=lev.dt)


def rhs(levels, u0):
    lev = levels[0]
    f = np.zeros(lev.shape)
    f[0] = lev.l0[:, None, None] * np.asarray(u0).reshape(lev.ny, lev.nx)[None]
    return f


def solve(prob, u0, rtol=1e-12, max_cycles=200, **kw):
    """V-cycles from a zero initial guess until ||b - A U|| <= rtol ||b||."""
    hk = {k: kw.pop(k) for k in ("coarsen", "mu_crit", "min_coarse", "max_levels", "fft_coarse") if k in kw}
    levels, kinds = hierarchy(prob, **hk)
    f = rhs(levels, u0)
    U = np.zeros(levels[0].shape)
    nb = np.linalg.norm(f)
    hist = []
    for _ in range(max_cycles):
        U = vcycle(levels, kinds, U, f, **kw)
        hist.append(np.linalg.norm(f - levels[0].apply(U)) / nb)
        if hist[-1] <= rtol:
            break
    return U, hist
