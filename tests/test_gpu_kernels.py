"""GPU parity, kernel by kernel, against the oracle (element by element).

Each case prints its name before touching the GPU."""
import numpy as np
import pytest

import stmg_inputs as si
from oracle import allatonce, mg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
from gpu_util import H, T, assert_close, rel_err  # noqa: E402

CASES = [
    ("1d-M1", si.problem(1, 24, 1, 7, 0.3, nu=0.2, lam=0.5)),
    ("1d-M2", si.problem(1, 64, 2, 16, 0.1, nu=1.0, lam=0.0)),
    ("2d-M3-ragged", si.problem(2, 20, 3, 9, 0.5, nu=0.01, lam=1.0)),
    ("2d-M4", si.problem(2, 32, 4, 12, 1.0, nu=0.05, lam=0.3)),
    ("2d-M3-tiles", si.problem(2, 48, 3, 34, 1.0, nu=0.02, lam=1.0)),
    ("2d-M6", si.problem(2, 16, 6, 6, 0.2, nu=0.05, lam=0.5)),
    ("1d-odd", si.problem(1, 25, 2, 8, 0.2, nu=0.3, lam=0.1)),
]

# Neumann grids (the paper's boundary condition, Sec. 3): mirror points in the
# operator and the restriction, both ends kept by the interpolation
NEUMANN = [
    ("1d-neumann", si.problem(1, 32, 3, 8, 0.2, nu=0.5, lam=0.3, bc="neumann")),
    ("2d-neumann", si.problem(2, 16, 2, 6, 0.5, nu=0.05, lam=1.0, bc="neumann")),
    ("2d-neumann-M4", si.problem(2, 12, 4, 5, 0.3, nu=0.02, lam=0.5, bc="neumann")),
    ("2d-neumann-space", si.problem(2, 20, 3, 4, 0.2, nu=0.2, lam=0.1, bc="neumann")),
]


def _rng_fields(prob, seed):
    rng = np.random.default_rng(seed)
    ny, nx = si.grid_points(prob)
    shape = (prob["N"], prob["M"], ny, nx)
    return rng.standard_normal(shape), rng.standard_normal((ny, nx)), rng.standard_normal(shape)


@pytest.mark.parametrize("name,prob", CASES + [
    ("1d-neumann", si.problem(1, 30, 3, 5, 0.2, nu=1.0, bc="neumann")),
    ("2d-neumann", si.problem(2, 12, 2, 6, 0.2, nu=0.1, lam=0.2, bc="neumann")),
    ("2d-AC", si.problem(2, 16, 3, 5, 0.5, nu=0.01, gamma=1.0, reaction="allen_cahn")),
])
def test_residual_matches_allatonce(name, prob):
    print("case", name, flush=True)
    U, u0, _ = _rng_fields(prob, 1)
    ref = allatonce.residual(prob, u0, U)
    h = H(prob)
    r = torch.empty(U.shape, dtype=torch.float64, device="cuda:0")
    nrm = h.residual(T(u0), T(U), r)
    got = r.cpu().numpy()
    assert_close(got, ref, 1e-13 * np.abs(ref).max(), "residual")
    assert abs(nrm - np.linalg.norm(ref)) <= 1e-12 * np.linalg.norm(ref)


# fft_coarse: the default coarsest-level rule, and 0 (deep hierarchies down to
# a few dozen unknowns, which exercise every transfer kind on small grids)
FFT = [1 << 22, 0]


@pytest.mark.parametrize("name,prob", CASES + NEUMANN)
@pytest.mark.parametrize("fft", FFT)
def test_hierarchy_matches_oracle(name, prob, fft):
    print("case", name, fft, flush=True)
    levels, kinds = mg.hierarchy(prob, fft_coarse=fft)
    got = H(prob, fft_coarse=fft).levels()
    assert len(got) == len(levels)
    code = {"s": 1, "t": 2, "st": 3, "sm": 5}
    for l, (g, o) in enumerate(zip(got, levels)):
        assert (g["nx"], g["ny"], g["N"], g["M"]) == (o.nx, o.ny, o.N, o.M)
        assert abs(g["dt"] - o.dt) <= 1e-15 * o.dt
        assert g["kind"] == (code[kinds[l]] if l < len(kinds) else 0)


@pytest.mark.parametrize("name,prob", CASES + NEUMANN)
@pytest.mark.parametrize("zero", [False, True])
def test_smoother_each_level(name, prob, zero):
    print("case", name, zero, flush=True)
    levels, kinds = mg.hierarchy(prob, fft_coarse=0)
    h = H(prob, fft_coarse=0)
    for l, lev in enumerate(levels):
        rng = np.random.default_rng(10 + l)
        U = np.zeros(lev.shape) if zero else rng.standard_normal(lev.shape)
        f = rng.standard_normal(lev.shape)
        ref = lev.smooth(U, f, 0.8, 16 if l == 0 else 4)
        out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        h.smooth(l, None if zero else T(U), out, f=T(f))
        assert_close(out.cpu().numpy(), ref, 1e-12, "smooth level %d" % l)


@pytest.mark.parametrize("name,prob", CASES + NEUMANN)
def test_restrict_prolong_each_level(name, prob):
    print("case", name, flush=True)
    levels, kinds = mg.hierarchy(prob, fft_coarse=0)
    h = H(prob, fft_coarse=0)
    for l in range(len(levels) - 1):
        lev, nxt = levels[l], levels[l + 1]
        rng = np.random.default_rng(20 + l)
        U = rng.standard_normal(lev.shape)
        f = rng.standard_normal(lev.shape)
        ref = mg.restrict(f - lev.apply(U), kinds[l], lev.dim, bc=lev.bc)
        fc = torch.empty(nxt.shape, dtype=torch.float64, device="cuda:0")
        h.restrict_residual(l, T(U), fc, f=T(f))
        assert_close(fc.cpu().numpy(), ref, 1e-12, "restrict level %d kind %s" % (l, kinds[l]))
        ec = rng.standard_normal(nxt.shape)
        refp = U + mg.prolong(ec, kinds[l], lev.dim, bc=lev.bc)
        out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        h.prolong(l, T(ec), out, Uin=T(U))
        assert_close(out.cpu().numpy(), refp, 1e-13, "prolong level %d kind %s" % (l, kinds[l]))


@pytest.mark.parametrize("name,prob", CASES + NEUMANN)
@pytest.mark.parametrize("fft", FFT)
def test_coarse_solve(name, prob, fft):
    """Fourier coarsest solve (default rule, periodic) or the dense one (deep
    hierarchies) against the oracle's direct slab-by-slab solve."""
    print("case", name, fft, flush=True)
    levels, kinds = mg.hierarchy(prob, fft_coarse=fft)
    h = H(prob, fft_coarse=fft)
    lev = levels[-1]
    f = np.random.default_rng(3).standard_normal(lev.shape)
    ref = lev.exact_solve(f)
    out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
    h.coarse_solve(T(f), out)
    assert_close(out.cpu().numpy(), ref, 1e-12, "coarse solve")


# Coarsest planes with power-of-two sides of at most 64 points take the
# register transforms; long time axes (N (M + 2) > 768) the run-chained mode
# recurrence.  One space step from the finest level, fft_coarse large.
REG = [(128, 128, 3, 160), (128, 64, 2, 12), (64, 128, 4, 7), (16, 128, 1, 9), (8, 8, 2, 300),
       (4, 4, 5, 3), (128, 128, 2, 2)]


def _reg_problem(nx, ny, M, N):
    prob = si.problem(2, nx, M, N, 1.0, nu=0.02, lam=0.7)
    prob["nx"] = [nx, ny]
    return prob


@pytest.mark.parametrize("nx,ny,M,N", REG)
def test_coarse_solve_register_transforms(nx, ny, M, N):
    print("case reg", nx, ny, M, N, flush=True)
    prob = _reg_problem(nx, ny, M, N)
    opt = dict(coarsen="space", fft_coarse=1 << 24)
    levels, kinds = mg.hierarchy(prob, coarsen="space", fft_coarse=1 << 24)
    assert len(levels) == 2
    h = H(prob, **opt)
    assert [(g["nx"], g["ny"], g["N"]) for g in h.levels()] == [(l.nx, l.ny, l.N) for l in levels]
    lev = levels[-1]
    f = np.random.default_rng(31).standard_normal(lev.shape)
    ref = lev.exact_solve(f)
    out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
    h.coarse_solve(T(f), out)
    assert_close(out.cpu().numpy(), ref, 1e-12, "coarse solve")
    # one V-cycle through it
    u0 = np.random.default_rng(32).standard_normal(levels[0].shape[2:])
    U = np.random.default_rng(33).standard_normal(levels[0].shape)
    refv = mg.vcycle(levels, kinds, U.copy(), mg.rhs(levels, u0))
    Ud = T(U)
    h.vcycle(T(u0), Ud)
    assert_close(Ud.cpu().numpy(), refv, 1e-11, "one V-cycle")


@pytest.mark.parametrize("name,prob", CASES)
@pytest.mark.parametrize("fft", FFT)
def test_one_vcycle_matches_oracle(name, prob, fft):
    print("case", name, fft, flush=True)
    levels, kinds = mg.hierarchy(prob, fft_coarse=fft)
    u0 = np.random.default_rng(4).standard_normal(levels[0].shape[2:])
    f = mg.rhs(levels, u0)
    U = np.random.default_rng(5).standard_normal(levels[0].shape)
    ref = mg.vcycle(levels, kinds, U.copy(), f)
    h = H(prob, fft_coarse=fft)
    Ud = T(U)
    h.vcycle(T(u0), Ud)
    assert_close(Ud.cpu().numpy(), ref, 1e-11, "one V-cycle")


def test_repeatable_bitwise():
    prob = CASES[3][1]
    U, u0, _ = _rng_fields(prob, 7)
    h = H(prob)
    outs = []
    for _ in range(3):
        Ud = T(U)
        h.vcycle(T(u0), Ud)
        outs.append(Ud.cpu().numpy())
    assert all(np.array_equal(outs[0], o) for o in outs[1:])


# SMMG: space coarsening with M lowered by one per level (Sec. 5.2)
SMMG = [
    ("smmg-2d-M3", si.problem(2, 32, 3, 6, 0.5, nu=0.05, lam=1.0)),
    ("smmg-2d-M4-tiles", si.problem(2, 48, 4, 5, 0.5, nu=0.02, lam=0.5)),
    ("smmg-1d-M2", si.problem(1, 64, 2, 16, 0.1, nu=1.0, lam=0.0)),
]


@pytest.mark.parametrize("name,prob", SMMG)
@pytest.mark.parametrize("fft", FFT)
def test_smmg_hierarchy_matches_oracle(name, prob, fft):
    print("case", name, fft, flush=True)
    levels, kinds = mg.hierarchy(prob, coarsen="smmg", fft_coarse=fft)
    got = H(prob, coarsen="smmg", fft_coarse=fft).levels()
    assert len(got) == len(levels)
    code = {"s": 1, "sm": 5}
    for l, (g, o) in enumerate(zip(got, levels)):
        assert (g["nx"], g["ny"], g["N"], g["M"]) == (o.nx, o.ny, o.N, o.M)
        assert g["kind"] == (code[kinds[l]] if l < len(kinds) else 0)


@pytest.mark.parametrize("name,prob", SMMG)
def test_smmg_transfers_each_level(name, prob):
    """Residual restriction and prolongation across node sets against the oracle."""
    print("case", name, flush=True)
    levels, kinds = mg.hierarchy(prob, coarsen="smmg", fft_coarse=0)
    h = H(prob, coarsen="smmg", fft_coarse=0)
    for l in range(len(levels) - 1):
        lev, nxt = levels[l], levels[l + 1]
        rng = np.random.default_rng(40 + l)
        U = rng.standard_normal(lev.shape)
        f = rng.standard_normal(lev.shape)
        ref = mg.restrict(f - lev.apply(U), kinds[l], lev.dim, lev.Pm)
        fc = torch.empty(nxt.shape, dtype=torch.float64, device="cuda:0")
        h.restrict_residual(l, T(U), fc, f=T(f))
        assert_close(fc.cpu().numpy(), ref, 1e-12, "restrict level %d kind %s" % (l, kinds[l]))
        ec = rng.standard_normal(nxt.shape)
        refp = U + mg.prolong(ec, kinds[l], lev.dim, lev.Pm)
        out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        h.prolong(l, T(ec), out, Uin=T(U))
        assert_close(out.cpu().numpy(), refp, 1e-13, "prolong level %d kind %s" % (l, kinds[l]))
        ref_s = lev.smooth(U, f, 0.8, 16 if l == 0 else 4)
        out_s = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        h.smooth(l, T(U), out_s, f=T(f))
        assert_close(out_s.cpu().numpy(), ref_s, 1e-12, "smooth level %d (M=%d)" % (l, lev.M))


@pytest.mark.parametrize("name,prob", SMMG)
@pytest.mark.parametrize("fft", FFT)
def test_smmg_one_vcycle_matches_oracle(name, prob, fft):
    print("case", name, fft, flush=True)
    levels, kinds = mg.hierarchy(prob, coarsen="smmg", fft_coarse=fft)
    u0 = np.random.default_rng(4).standard_normal(levels[0].shape[2:])
    f = mg.rhs(levels, u0)
    U = np.random.default_rng(5).standard_normal(levels[0].shape)
    ref = mg.vcycle(levels, kinds, U.copy(), f)
    h = H(prob, coarsen="smmg", fft_coarse=fft)
    Ud = T(U)
    h.vcycle(T(u0), Ud)
    assert_close(Ud.cpu().numpy(), ref, 1e-11, "one SMMG V-cycle")


def test_smmg_coarse_solve_on_lowered_nodes():
    """The coarsest level of an SMMG hierarchy has fewer nodes than the finest;
    both coarsest solves (Fourier and dense) use that level's own tables."""
    prob = SMMG[0][1]
    for fft in FFT:
        levels, kinds = mg.hierarchy(prob, coarsen="smmg", fft_coarse=fft)
        lev = levels[-1]
        assert lev.M < prob["M"]
        h = H(prob, coarsen="smmg", fft_coarse=fft)
        f = np.random.default_rng(6).standard_normal(lev.shape)
        out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        h.coarse_solve(T(f), out)
        assert_close(out.cpu().numpy(), lev.exact_solve(f), 1e-12, "coarse solve M=%d" % lev.M)


@pytest.mark.parametrize("name,prob,levels", [
    ("1d-16pt-64slabs", si.problem(1, 32, 3, 64, 0.5, nu=1.0), 2),
    ("2d-8x8-40slabs", si.problem(2, 16, 2, 40, 0.5, nu=0.01, lam=1.0), 2),
    ("2d-neumann-5x5-48slabs", si.problem(2, 16, 3, 48, 0.5, nu=0.01, lam=1.0, bc="neumann"), 3),
])
def test_coarse_solve_split_recurrence(name, prob, levels):
    """Dense coarsest levels with at most 64 points per plane and at least 32
    slabs take the split recurrence (parallel A^-1 applications around a
    one-wave P-vector recurrence): against the oracle's slab-by-slab solve
    (periodic), or against the forward substitution of the assembled slab
    system (Neumann)."""
    print("case", name, flush=True)
    h = H(prob, coarsen="space", max_levels=levels, fft_coarse=0)
    lv = h.levels()[-1]
    shape = (lv["N"], lv["M"], lv["ny"], lv["nx"])
    assert lv["nx"] * lv["ny"] <= 64 and lv["N"] >= 32
    f = np.random.default_rng(8).standard_normal(shape)
    out = torch.empty(shape, dtype=torch.float64, device="cuda:0")
    h.coarse_solve(T(f), out)
    if prob["bc"] == "periodic":
        levels_o, _ = mg.hierarchy(prob, coarsen="space", max_levels=levels, fft_coarse=0)
        ref = levels_o[-1].exact_solve(f)
        assert ref.shape == shape
    else:
        # the coarsest level rediscretizes the problem on its own grid (same
        # domain, nx - 1 elements, its own dt): its all-at-once matrix with
        # zero u0, solved densely
        cp = si.problem(2, lv["nx"] - 1, prob["M"], lv["N"], lv["dt"] * lv["N"], nu=prob["nu"],
                        lam=prob["lambda"], bc="neumann")
        ref = np.linalg.solve(allatonce.matrix(cp).toarray(), f.reshape(-1)).reshape(shape)
    assert_close(out.cpu().numpy(), ref, 1e-12, "coarse solve (split recurrence)")


def test_full_size_smoother_and_vcycle():
    """The 256^2 x M=3 x N=256 workload in the benchmark's configuration: one
    level-0 smoothing sweep (right-hand side generated from u0, as the timed
    kernel runs it) and one whole V-cycle, element by element against the
    oracle."""
    print("case full-size smoother and V-cycle", flush=True)
    prob = si.config("rd2d")
    levels, kinds = mg.hierarchy(prob)
    u0 = si.initial("rd2d", prob)
    f = mg.rhs(levels, u0)
    U = np.random.default_rng(31).standard_normal(levels[0].shape)
    h = H(prob)
    assert [(l["nx"], l["N"]) for l in h.levels()] == [(lv.nx, lv.N) for lv in levels]
    ref = levels[0].smooth(U, f, 0.8, 16)
    out = torch.empty(levels[0].shape, dtype=torch.float64, device="cuda:0")
    h.smooth(0, T(U), out, u0=T(u0))
    assert_close(out.cpu().numpy(), ref, 1e-12, "full-size smooth")
    del out, ref
    ref = mg.vcycle(levels, kinds, U.copy(), f)
    Ud = T(U)
    h.vcycle(T(u0), Ud)
    assert_close(Ud.cpu().numpy(), ref, 1e-11, "full-size V-cycle")


@pytest.mark.parametrize("name,prob", CASES)
def test_prolong_smooth_each_level(name, prob):
    """The fused way up (stmg_level_prolong_smooth): U' = U + P e_c, then one
    block-Jacobi sweep, against the oracle's prolongation followed by its
    smoother, from a given and from a zero (NULL) iterate; on level 0 also
    with the right-hand side built from u0."""
    print("case", name, flush=True)
    levels, kinds = mg.hierarchy(prob, fft_coarse=0)
    h = H(prob, fft_coarse=0)
    ny, nx = si.grid_points(prob)
    blocked = prob["bc"] == "periodic" and nx % 2 == 0 and (ny == 1 or ny % 2 == 0)
    for l in range(len(levels) - 1):
        lev, nxt = levels[l], levels[l + 1]
        rng = np.random.default_rng(30 + l)
        U = rng.standard_normal(lev.shape)
        f = rng.standard_normal(lev.shape)
        ec = rng.standard_normal(nxt.shape)
        out = torch.empty(lev.shape, dtype=torch.float64, device="cuda:0")
        if not blocked:
            with pytest.raises(Exception):
                h.prolong_smooth(l, T(ec), out, Uin=T(U), f=T(f))
            return
        Up = U + mg.prolong(ec, kinds[l], lev.dim, lev.Pm)
        ref = lev.smooth(Up, f, 0.8, 16 if l == 0 else 4)
        h.prolong_smooth(l, T(ec), out, Uin=T(U), f=T(f))
        assert_close(out.cpu().numpy(), ref, 1e-12, "prolong+smooth level %d kind %s" % (l, kinds[l]))
        # zero iterate (U passed as NULL): U' = P e_c
        refz = lev.smooth(mg.prolong(ec, kinds[l], lev.dim, lev.Pm), f, 0.8, 16 if l == 0 else 4)
        h.prolong_smooth(l, T(ec), out, f=T(f))
        assert_close(out.cpu().numpy(), refz, 1e-12, "prolong+smooth level %d from zero" % l)
        if l == 0:
            u0 = rng.standard_normal((ny, nx))
            f0 = mg.rhs(levels, u0)
            ref0 = lev.smooth(Up, f0, 0.8, 16)
            h.prolong_smooth(0, T(ec), out, Uin=T(U), u0=T(u0))
            assert_close(out.cpu().numpy(), ref0, 1e-12, "prolong+smooth level 0 from u0")
