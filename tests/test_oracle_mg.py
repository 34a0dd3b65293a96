"""Oracle pins for the multigrid components: transfer identities, the
smoother's fixed point, the V-cycle's fixed point (the stepper's solution)."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import radau
from oracle import mg, stepper


def _inner(a, b):
    return float(np.sum(a * b))


@pytest.mark.parametrize("dim", [1, 2])
def test_space_transfer_adjoint(dim):
    rng = np.random.default_rng(0)
    shp_f = (3, 2, 8 if dim == 2 else 1, 16)
    shp_c = (3, 2, 4 if dim == 2 else 1, 8)
    f = rng.standard_normal(shp_f)
    c = rng.standard_normal(shp_c)
    # R = 2^{-d} P^T
    assert abs(_inner(mg.restrict_space(f, dim), c) - 2.0 ** (-dim) * _inner(f, mg.prolong_space(c, dim))) < 1e-12


def test_time_transfer_adjoint():
    rng = np.random.default_rng(1)
    f = rng.standard_normal((8, 3, 2, 2))
    c = rng.standard_normal((4, 3, 2, 2))
    # time restriction is exactly P^T
    assert abs(_inner(mg.restrict_time(f), c) - _inner(f, mg.prolong_time(c))) < 1e-12


def test_transfer_constants_and_linears():
    c = np.ones((2, 1, 4, 4))
    assert np.abs(mg.prolong_space(c, 2) - 1).max() == 0
    assert np.abs(mg.restrict_space(np.ones((2, 1, 8, 8)), 2) - 1).max() == 0
    # linear in slab end time is reproduced exactly (T_0 carries zero)
    Nc = 4
    e = (np.arange(Nc) + 1.0)[:, None, None, None] * 2.0 * np.ones((1, 2, 1, 3))
    f = mg.prolong_time(e)
    assert np.abs(f[:, 0, 0, 0] - (np.arange(2 * Nc) + 1.0)).max() == 0
    # interior time restriction of a constant gives 2 (rediscretization scale)
    r = mg.restrict_time(np.ones((8, 1, 1, 1)))
    assert np.allclose(r[:-1, 0, 0, 0], 2.0) and r[-1, 0, 0, 0] == 1.5


def test_hierarchy_auto_rule():
    prob = si.problem(2, 64, 3, 64, 1.0, nu=0.04, lam=1.0)  # mu = 2.56 on the finest level
    levels, kinds = mg.hierarchy(prob, fft_coarse=0)
    assert kinds[0] == "s"            # mu = 2.56 >= 0.5: space first
    assert kinds[1] == "s"            # mu = 0.64 after one space step
    assert kinds[2] == "t"            # mu = 0.16
    for l, k in zip(levels, kinds):
        mu = l.nu * l.dt / l.hx ** 2
        if k == "s":
            assert mu >= 0.5 or l.N % 2 == 1
    l1, k1 = mg.hierarchy(prob, mu_crit=1.0, fft_coarse=0)
    assert k1[:2] == ["s", "t"]
    last = levels[-1]
    assert last.M * last.nx * last.ny * last.N <= 64


def test_hierarchy_coarsest_rule():
    """The coarsest level is the first level below the finest with planes of at
    most 1024 points (or power-of-two sides of at most 64) and at most
    fft_coarse unknowns (else the AUTO rule runs on)."""
    prob = si.config("rd2d")                  # 256^2 x 3 x 256
    levels, kinds = mg.hierarchy(prob)
    assert kinds == ["s", "s"]
    last = levels[-1]
    assert (last.nx, last.ny, last.N) == (64, 64, 256)
    # planes of at most 1024 points only: down to 32^2 x 64
    lv1, k1 = mg.hierarchy(prob, fft_side=0)
    assert k1 == ["s", "s", "t", "t", "s"] and (lv1[-1].nx, lv1[-1].N) == (32, 64)
    lv2, k2 = mg.hierarchy(prob, fft_coarse=262144)
    assert k2 == k1
    deep, dk = mg.hierarchy(prob, fft_coarse=0)
    assert len(deep) == 15 and dk[:5] == k1
    # non-power-of-two sides: the 1024-point rule alone
    odd = si.problem(2, 96, 2, 8, 1.0, nu=0.02, lam=1.0)
    lo, ko = mg.hierarchy(odd)
    assert (lo[-1].nx, lo[-1].ny) == (24, 24)
    # the finest level itself never stops the coarsening
    small = si.problem(2, 16, 2, 4, 0.5, nu=0.02, lam=1.0)
    lv, kk = mg.hierarchy(small)
    assert len(lv) == 2


@pytest.mark.parametrize("Mf", [2, 3, 4, 5])
def test_node_prolongation_reproduces_polynomials(Mf):
    """The node transfer interpolates every polynomial of degree < Mc exactly
    and keeps the end node (t = 1 is a node of every Radau set)."""
    Mc = Mf - 1
    P = mg.node_prolongation(Mf, Mc)
    cf, cc = radau.tables(Mf)["c"], radau.tables(Mc)["c"]
    for p in range(Mc):
        assert np.abs(P @ cc ** p - cf ** p).max() < 1e-13
    assert np.abs(P[-1] - np.eye(Mc)[-1]).max() < 1e-14


@pytest.mark.parametrize("Mf", [2, 3, 4, 5])
def test_node_transfer_is_galerkin(Mf):
    """P^T A_fine P = A_coarse in the time structure (reading: Lagrange node
    transfer, R = P^T): Kq, the Radau mass diag(b), l(0) and the end-node
    coupling restrict exactly, so rediscretized coarse levels are Galerkin."""
    Mc = Mf - 1
    P = mg.node_prolongation(Mf, Mc)
    tf, tc = radau.tables(Mf), radau.tables(Mc)
    assert np.abs(P.T @ tf["Kq"] @ P - tc["Kq"]).max() < 1e-12
    assert np.abs(P.T @ np.diag(tf["b"]) @ P - np.diag(tc["b"])).max() < 1e-13
    assert np.abs(P.T @ tf["l0"] - tc["l0"]).max() < 1e-12


def test_smmg_hierarchy():
    """SMMG lowers M by one per level until M = 1 while coarsening in space
    (Sec. 5.2: M = max(M - l + 1, 1) on level l), then continues as SMG."""
    prob = si.problem(2, 32, 3, 4, 0.5, nu=0.05, lam=1.0)
    levels, kinds = mg.hierarchy(prob, coarsen="smmg", fft_coarse=0)
    assert kinds == ["sm", "sm", "s"]
    assert [(l.nx, l.M) for l in levels] == [(32, 3), (16, 2), (8, 1), (4, 1)]
    assert levels[0].Pm.shape == (3, 2) and levels[1].Pm.shape == (2, 1) and levels[2].Pm is None


@pytest.mark.parametrize("chunk", [1, 4, 16])
def test_smoother_fixed_point(chunk):
    prob = si.problem(2, 16, 3, 8, 0.5, nu=0.02, lam=1.0)
    u0 = si.u0_rd2d(prob, 9)
    levels, _ = mg.hierarchy(prob)
    Ue = stepper.solve_linear(prob, u0)
    f = mg.rhs(levels, u0)
    assert np.abs(levels[0].apply(Ue) - f).max() < 1e-13
    U1 = levels[0].smooth(Ue, f, 0.8, chunk)
    assert np.abs(U1 - Ue).max() < 1e-13


@pytest.mark.parametrize("dense", [True, False])
def test_exact_coarse_solve(dense):
    """Both factorizations of the slab matrix (dense LU, sparse LU) against the
    time stepper's direct solve per step."""
    prob = si.problem(2, 8, 2, 6, 0.5, nu=0.02, lam=1.0)
    levels, _ = mg.hierarchy(prob, min_coarse=10 ** 9)
    u0 = si.u0_rd2d(prob, 3)
    f = mg.rhs(levels, u0)
    U = levels[0].exact_solve(f, dense=dense)
    assert np.abs(U - stepper.solve_linear(prob, u0)).max() < 1e-13


@pytest.mark.parametrize("prob", [si.problem(2, 6, 3, 2, 0.5, nu=0.02, lam=1.0),
                                  si.problem(1, 10, 2, 2, 0.5, nu=0.3, lam=0.1),
                                  si.problem(2, 2, 2, 2, 0.5, nu=0.1, lam=0.0)])
def test_slab_matrix_kronecker_form(prob):
    """The Kronecker assembly of the slab block equals the block built column
    by column from the level operator (two sizes of 2D, 1D, and the 2-point
    periodic grid whose two neighbours coincide)."""
    lev = mg.hierarchy(prob, min_coarse=10 ** 9)[0][0]
    assert np.abs(lev.slab_matrix_sparse().toarray() - lev.slab_matrix()).max() == 0.0


@pytest.mark.parametrize("name,kw", [
    ("heat1d", {}),
    ("rd2d-small", {}),
    ("rd2d-small", {"coarsen": "space"}),
    ("rd2d-small", {"coarsen": "spacetime"}),
    ("rd2d-small", {"chunk": 1}),
    ("rd2d-small", {"fft_coarse": 0}),
    ("rd2d-small", {"coarsen": "smmg"}),
    ("rd2d-small", {"coarsen": "smmg", "fft_coarse": 0}),
    ("heat1d", {"coarsen": "smmg"}),
])
def test_vcycle_converges_to_stepper(name, kw):
    if name == "heat1d":
        prob = si.config("heat1d")
        u0 = si.initial("heat1d", prob)
    else:
        prob = si.problem(2, 32, 3, 32, 1.0, nu=1e-2 * 32 / 256 * 8, lam=1.0)
        u0 = si.u0_rd2d(prob, 2)
    # SMMG on the 1D heat workload (mu = 25.6) contracts by only ~0.84 per
    # cycle (the paper's Table 3 also has SMMG needing more iterations than SMG)
    slow = name == "heat1d" and kw.get("coarsen") == "smmg"
    U, hist = mg.solve(prob, u0, rtol=1e-12, max_cycles=300 if slow else 150, **kw)
    assert hist[-1] <= 1e-12
    Ue = stepper.solve_linear(prob, u0)
    assert np.linalg.norm(U - Ue) <= 1e-10 * np.linalg.norm(Ue)
    rates = [hist[i + 1] / hist[i] for i in range(len(hist) - 1)]
    if not kw:
        assert np.median(rates) < 0.5, rates


def test_sdc_fixed_point_and_convergence():
    """The collocation solution is a fixed point of the SDC sweep, and sweeps
    from zero converge to it (Sec. 2.1: SDC's fixed point is Radau IIA)."""
    from oracle import sdc
    prob = si.problem(1, 16, 3, 6, 0.3, nu=0.1, lam=0.5)
    u0 = np.random.default_rng(2).standard_normal((1, 16))
    Ue = stepper.solve_linear(prob, u0)
    assert np.abs(sdc.sweep(prob, u0, Ue) - Ue).max() < 1e-13
    U = np.zeros_like(Ue)
    for _ in range(60):
        U = sdc.sweep(prob, u0, U)
    assert np.abs(U - Ue).max() < 1e-11 * np.abs(Ue).max()


def test_sdc_m1_is_backward_euler():
    """With M = 1, Q_Delta = Q: one sweep solves each slab exactly for the
    lagged initial value, so N sweeps from zero give backward Euler exactly."""
    from oracle import sdc
    prob = si.problem(2, 6, 1, 4, 0.2, nu=0.05, lam=0.3)
    u0 = np.random.default_rng(3).standard_normal((6, 6))
    Ue = stepper.solve_linear(prob, u0)
    U = np.zeros_like(Ue)
    for _ in range(prob["N"]):
        U = sdc.sweep(prob, u0, U)
    assert np.abs(U - Ue).max() < 1e-13


# --- Neumann grids (the paper's boundary condition, Sec. 3) -----------------
def _interp_matrix(ec):
    """Linear interpolation from ec + 1 coarse to 2 ec + 1 fine points as an
    explicit matrix (fine 2J = coarse J, fine 2J + 1 = their mean)."""
    P = np.zeros((2 * ec + 1, ec + 1))
    for J in range(ec + 1):
        P[2 * J, J] = 1.0
        if J < ec:
            P[2 * J + 1, J] = 0.5
            P[2 * J + 1, J + 1] = 0.5
    return P


def _lumped_mass(e, h):
    m = np.full(e + 1, h)
    m[0] = m[-1] = 0.5 * h
    return np.diag(m)


@pytest.mark.parametrize("dim", [1, 2])
def test_neumann_restriction_is_fe_consistent(dim):
    """On Neumann grids the restriction equals R = M_c^-1 P^T M_f with the
    lumped linear-FE masses (half weight at the end points), built here as
    explicit matrices; a sign or weight slip at an end point fails this."""
    ef, h = 8, 0.125
    Rx = np.linalg.inv(_lumped_mass(ef // 2, 2 * h)) @ _interp_matrix(ef // 2).T @ _lumped_mass(ef, h)
    rng = np.random.default_rng(4)
    ny = ef + 1 if dim == 2 else 1
    r = rng.standard_normal((2, 3, ny, ef + 1))
    want = np.einsum("Xx,nmyx->nmyX", Rx, r)
    if dim == 2:
        want = np.einsum("Yy,nmyX->nmYX", Rx, want)
    got = mg.restrict_space(r, dim, "neumann")
    assert np.abs(got - want).max() < 1e-14


@pytest.mark.parametrize("dim", [1, 2])
def test_neumann_prolongation_reproduces_linears(dim):
    """Linear functions of x (and y) on the coarse Neumann grid, end points
    included, are interpolated exactly; the interpolation matrix matches."""
    ec = 4
    xc = np.arange(ec + 1) * 0.25
    xf = np.arange(2 * ec + 1) * 0.125
    if dim == 1:
        e = (1.5 + 2.0 * xc)[None, None, None, :]
        f = mg.prolong_space(e, 1, "neumann")
        assert np.abs(f[0, 0, 0] - (1.5 + 2.0 * xf)).max() < 1e-15
    else:
        e = (1.5 + 2.0 * xc[None, :] - 3.0 * xc[:, None])[None, None]
        f = mg.prolong_space(e, 2, "neumann")
        assert np.abs(f[0, 0] - (1.5 + 2.0 * xf[None, :] - 3.0 * xf[:, None])).max() < 1e-14
    rng = np.random.default_rng(5)
    v = rng.standard_normal((1, 1, 1, ec + 1))
    assert np.abs(mg.prolong_space(v, 1, "neumann")[0, 0, 0] - _interp_matrix(ec) @ v[0, 0, 0]).max() < 1e-15


NEUMANN = [si.problem(1, 16, 3, 8, 0.2, nu=0.5, lam=0.3, bc="neumann"),
           si.problem(2, 8, 2, 6, 0.5, nu=0.05, lam=1.0, bc="neumann")]


@pytest.mark.parametrize("prob", NEUMANN)
def test_neumann_operator_matches_allatonce(prob):
    """The level operator with mirror points equals the literal assembly of the
    all-at-once system (oracle.allatonce, built on oracle.space's Neumann
    Laplacian), and the slab block assembled from its Kronecker form equals
    the one built column by column."""
    from oracle import allatonce
    levels, _ = mg.hierarchy(prob, min_coarse=10 ** 9)
    lev = levels[0]
    rng = np.random.default_rng(6)
    U = rng.standard_normal(lev.shape)
    assert np.abs(lev.apply(U) - allatonce.apply(prob, U)).max() < 1e-12
    assert np.abs(lev.slab_matrix_sparse().toarray() - lev.slab_matrix()).max() < 1e-12


@pytest.mark.parametrize("prob", NEUMANN)
def test_neumann_fixed_points_and_vcycle(prob):
    """Smoother fixed point, exact slab solve and V-cycles on Neumann grids all
    reach the stepper's solution."""
    rng = np.random.default_rng(7)
    ny, nx = si.grid_points(prob)
    u0 = rng.standard_normal((ny, nx))
    Ue = stepper.solve_linear(prob, u0)
    levels, kinds = mg.hierarchy(prob, fft_coarse=0, min_coarse=16)
    assert any("s" in k for k in kinds)
    f = mg.rhs(levels, u0)
    assert np.abs(levels[0].smooth(Ue, f, 0.8, 4) - Ue).max() < 1e-12
    assert np.abs(levels[0].exact_solve(f) - Ue).max() < 1e-12
    U, hist = mg.solve(prob, u0, rtol=1e-12, max_cycles=150, fft_coarse=0, min_coarse=16)
    assert hist[-1] <= 1e-12
    assert np.linalg.norm(U - Ue) <= 1e-10 * np.linalg.norm(Ue)


@pytest.mark.parametrize("dim,M,chunk", [(2, 3, 16), (2, 2, 3), (1, 4, 1), (2, 1, 5)])
def test_swept_residual_identity(dim, M, chunk):
    """The residual after one block-Jacobi sweep (Sec. 4.2), f - A (U + omega d)
    with d = C^{-1}(f - A U), equals

      (1 - omega) r + omega dt b (cx (d_W + d_E) + cy (d_S + d_N))
        + omega l(0) d_{n-1,M} at chunk starts n > 0,

    the form in which the fused level-0 sweep + restriction forms it (C: the
    slab block on the diagonal and the chunk-internal coupling).  Periodic
    neighbours by rolling the arrays; a dropped coupling term, a wrong sign of
    the neighbour sum or a chunk-start term at the wrong slabs fails."""
    prob = si.problem(dim, 32 if dim == 2 else 64, M, 12, 0.3, nu=0.03, lam=0.7)
    levels, kinds = mg.hierarchy(prob, coarsen="space")
    lev = levels[0]
    rng = np.random.default_rng(11)
    U = rng.standard_normal(lev.shape)
    f = rng.standard_normal(lev.shape)
    omega = 0.8
    r = f - lev.apply(U)
    Us = lev.smooth(U, f, omega, chunk)
    d = (Us - U) / omega
    direct = f - lev.apply(Us)
    nb = lev.cx * (np.roll(d, 1, axis=-1) + np.roll(d, -1, axis=-1))
    if dim == 2:
        nb = nb + lev.cy * (np.roll(d, 1, axis=-2) + np.roll(d, -1, axis=-2))
    form = (1 - omega) * r + omega * lev.dt * lev.b[None, :, None, None] * nb
    for n in range(chunk, lev.N, chunk):
        form[n] += omega * lev.l0[:, None, None] * d[n - 1, -1][None]
    scale = np.abs(direct).max()
    assert np.abs(form - direct).max() <= 1e-12 * scale
    # the chunk-start term matters: without it the first slab of a chunk is off
    if chunk < lev.N:
        wrong = (1 - omega) * r + omega * lev.dt * lev.b[None, :, None, None] * nb
        assert np.abs(wrong - direct).max() > 1e-6 * scale
