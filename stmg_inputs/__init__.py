"""Seeded synthetic inputs for the space-time multigrid workloads.

Shared by the GPU tests, the benchmark and the CPU oracle.  This module
only builds problem descriptions (plain dicts) and input arrays (initial
conditions, targets, directions); it contains none of the solver's
arithmetic.

A problem dict has the keys of the paper's problem statement (Sec. 3):
  dim (1|2), nx [nx, ny] (elements per dimension), length [X, Y],
  bc ('periodic'|'neumann'), nu, reaction ('linear'|'allen_cahn'),
  lambda (linear: f = nu Lap u - lambda u), gamma (Allen-Cahn:
  f = nu Lap u + gamma (u - u^3)), M (right Radau nodes), N (steps), dt.
Periodic grids hold nx points per dimension (h = X / nx, x_j = j h);
Neumann grids hold nx + 1 points.
"""
import numpy as np


def problem(dim, nx, M, N, T, nu=1.0, lam=0.0, gamma=0.0, reaction="linear",
            bc="periodic", length=1.0):
    if dim == 1:
        nxs = [int(nx), 1]
    else:
        nxs = [int(nx), int(nx)]
    return dict(dim=dim, nx=nxs, length=[float(length), float(length)], bc=bc,
                nu=float(nu), reaction=reaction, **{"lambda": float(lam)},
                gamma=float(gamma), M=int(M), N=int(N), dt=float(T) / int(N))


# The five synthetic workloads ---------------------------------------------
def config(name):
    if name == "heat1d":      # 1D heat, periodic, 64 points, M=2, N=16, T=0.1
        return problem(1, 64, 2, 16, 0.1, nu=1.0, lam=0.0)
    if name == "rd2d":        # 2D linear, 256^2, M=3, N=256, T=1
        return problem(2, 256, 3, 256, 1.0, nu=1e-2, lam=1.0)
    if name == "ac2d":        # 2D Allen-Cahn, 512^2, M=3, N=512, T=2
        return problem(2, 512, 3, 512, 2.0, nu=1e-3, gamma=1.0, reaction="allen_cahn")
    if name == "adj2d":       # adjoint workload: same PDE as rd2d
        return problem(2, 256, 3, 256, 1.0, nu=1e-2, lam=1.0)
    raise KeyError(name)


# The paper's 1D examples (Sec. 5): X = 1, N_x = 1024 elements, Neumann, and
# N_t per M from its table headers.
PAPER_NT = {1: 1024, 2: 256, 3: 32, 4: 16, 5: 8}


def paper_heat1d(M, nx=1024, Nt=None):
    """Heat equation (gamma = 0), T = 1, N_t from the table headers unless given."""
    return problem(1, nx, M, PAPER_NT[M] if Nt is None else Nt, 1.0, nu=1.0, bc="neumann")


# Weak scaling in N_t (Example ex_3, SMG tables): (N_t, levels L) per M.
PAPER_WEAK = {1: [(1024, 7), (2048, 8), (4096, 8), (8192, 8)],
              2: [(256, 7), (512, 7), (1024, 8), (2048, 8)],
              3: [(32, 7), (64, 7), (128, 8), (256, 8)],
              4: [(16, 7), (32, 7), (64, 7), (128, 8)],
              5: [(8, 7), (16, 7), (32, 7), (64, 7)]}


def u0_paper_heat1d(prob):
    """cos(pi x) + 2 cos(3 pi x) + 3 cos(4 pi x) on [0, 1]."""
    X, _ = coords(prob)
    return np.cos(np.pi * X) + 2 * np.cos(3 * np.pi * X) + 3 * np.cos(4 * np.pi * X)


def paper_monodomain(M, nx=1024):
    """Monodomain example: X = 10, T = 2, gamma = 5, N_t from the table headers."""
    return problem(1, nx, M, PAPER_NT[M], 2.0, nu=1.0, gamma=5.0, reaction="allen_cahn", bc="neumann",
                   length=10.0)


def u0_paper_monodomain(prob):
    """Narrow stimulus in the middle of [0, X]: 2 exp(-((x - X/2) / 0.1)^2)."""
    X, _ = coords(prob)
    L = prob["length"][0]
    return 2.0 * np.exp(-((X - 0.5 * L) / 0.1) ** 2)


def grid_points(prob):
    nx = prob["nx"][0] + (0 if prob["bc"] == "periodic" else 1)
    ny = 1 if prob["dim"] == 1 else prob["nx"][1] + (0 if prob["bc"] == "periodic" else 1)
    return ny, nx


def coords(prob):
    ny, nx = grid_points(prob)
    hx = prob["length"][0] / prob["nx"][0]
    x = np.arange(nx) * hx
    if prob["dim"] == 1:
        return x[None, :], np.zeros((1, nx))
    hy = prob["length"][1] / prob["nx"][1]
    y = np.arange(ny) * hy
    X, Y = np.meshgrid(x, y)
    return X, Y


def u0_heat1d(prob, seed=1):
    """sin(2 pi x) + sum_{k=1..8} (a_k cos 2 pi k x + b_k sin 2 pi k x), a, b ~ N(0, 0.1^2)."""
    rng = np.random.default_rng(seed)
    a = rng.normal(0.0, 0.1, 8)
    b = rng.normal(0.0, 0.1, 8)
    X, _ = coords(prob)
    u = np.sin(2 * np.pi * X)
    for k in range(1, 9):
        u = u + a[k - 1] * np.cos(2 * np.pi * k * X) + b[k - 1] * np.sin(2 * np.pi * k * X)
    return u


def fourier_modes_2d(prob, kmax, seed, kmin=1.0):
    """Random periodic field: all k in Z^2 with kmin <= |k| <= kmax (one of each
    +-k pair), cos and sin amplitudes iid N(0, 1/|k|^2)."""
    rng = np.random.default_rng(seed)
    X, Y = coords(prob)
    u = np.zeros_like(X)
    K = int(np.floor(kmax))
    for kx in range(0, K + 1):
        for ky in range(-K, K + 1):
            if kx == 0 and ky <= 0:
                continue
            r = np.hypot(kx, ky)
            if r < kmin or r > kmax:
                continue
            a, b = rng.normal(0.0, 1.0 / r, 2)
            ph = 2 * np.pi * (kx * X + ky * Y)
            u += a * np.cos(ph) + b * np.sin(ph)
    return u


def u0_rd2d(prob, seed=2):
    return fourier_modes_2d(prob, 16, seed)


def u0_ac2d(prob, seed=3):
    ny, nx = grid_points(prob)
    return np.random.default_rng(seed).uniform(-0.1, 0.1, (ny, nx))


def u_tgt_adj2d(prob, seed=40):
    return fourier_modes_2d(prob, 4, seed)


def directions(shape, count=16, seed=41):
    rng = np.random.default_rng(seed)
    d = rng.normal(0.0, 1.0, (count,) + tuple(shape))
    return d / np.sqrt((d.reshape(count, -1) ** 2).sum(axis=1)).reshape((count,) + (1,) * len(shape))


def initial(name, prob, seed=None):
    if name == "heat1d":
        return u0_heat1d(prob, 1 if seed is None else seed)
    if name in ("rd2d",):
        return u0_rd2d(prob, 2 if seed is None else seed)
    if name == "adj2d":
        return u0_rd2d(prob, 4 if seed is None else seed)
    if name == "ac2d":
        return u0_ac2d(prob, 3 if seed is None else seed)
    raise KeyError(name)


def batch64(seed=5, count=64):
    """64 independent 2D periodic linear problems of uneven shape (T = 1)."""
    rng = np.random.default_rng(seed)
    probs = []
    for p in range(count):
        nx = int(rng.choice([64, 128, 256, 384, 512]))
        N = int(rng.choice([32, 64, 128, 256]))
        M = int(rng.choice([2, 3, 4]))
        nu = float(np.exp(rng.uniform(np.log(1e-3), np.log(1e-1))))
        lam = float(rng.uniform(0.0, 2.0))
        probs.append(problem(2, nx, M, N, 1.0, nu=nu, lam=lam))
    return probs


def batch_u0(prob, p):
    return fourier_modes_2d(prob, 16, 5000 + p)


def random_field(shape, seed):
    return np.random.default_rng(seed).standard_normal(shape)
