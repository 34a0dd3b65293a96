// PFASST (Sec. 4.1; Sec. 5.2, PFASST item): multilevel SDC on the
// collocation form with FAS corrections between levels; an Allen-Cahn
// reaction R(u) = gamma (u - u^3) is explicit in every sweep (IMEX, Sec. 5.4)
// and enters F = L + R in the FAS terms.  Level 0
// is the handle's grid with its M Radau nodes, swept by the SDC sweep of the
// handle (Solver::sdc_core); every coarser level has M = 1 and half the
// elements of the one above, with its own M = 1 solver for the slab solves.
//
// Level problem, slab n, node i (V_{-1,M} = the level's initial value u0_l):
//   V_{n,i} - dt (Q (x) F_l) V_n |_i - V_{n-1,M} = tau_{l,n,i},   tau_0 = 0.
// FAS restriction to level l+1 (end node, space full weighting R_s):
//   tau_{l+1,n} = R_s [tau_{l,n,M} + dt (Q F_l V_n)_M] - dt F_{l+1} R_s V_{n,M},
//   V_{l+1} = R_s V_{.,M}   (the level's terms in V_{n-1,M} cancel).
// Correction of level l (linear in time between the slab's start and end):
//   V_{l,n,i} += P_s ((1 - c_i) e_{n-1} + c_i e_n),  e_n = V_{l+1,n} - R_s V_{l,n,M},
//   e_{-1} = 0.
#include <chrono>
#include <cmath>
#include <string>

#include "solver.hpp"

namespace stmg {
namespace {

constexpr int kPfBlock = 256;

__device__ __forceinline__ int pf_lo(int i, int n, int bc) { return i > 0 ? i - 1 : (bc == 0 ? n - 1 : 1); }
__device__ __forceinline__ int pf_hi(int i, int n, int bc) { return i < n - 1 ? i + 1 : (bc == 0 ? 0 : n - 2); }

// (L u)(x, y) = cx (u[x-1] + u[x+1] - 2u) + cy (u[y-1] + u[y+1] - 2u) - lam u
__device__ __forceinline__ double pf_lap(const double* __restrict__ u, int x, int y, int nx, int ny, int bc,
                                         double cx, double cy, double lam) {
  const double c = u[y * nx + x];
  double l = cx * (u[y * nx + pf_lo(x, nx, bc)] + u[y * nx + pf_hi(x, nx, bc)] - 2.0 * c);
  if (ny > 1) l += cy * (u[pf_lo(y, ny, bc) * nx + x] + u[pf_hi(y, ny, bc) * nx + x] - 2.0 * c);
  return l - lam * c;
}

struct PfGrid {
  int nx, ny, bc;
  double cx, cy, lam;
  double gamma;  // explicit Allen-Cahn reaction (0: linear)
};

// F(u) at a point: (L u) + gamma (u - u^3)
__device__ __forceinline__ double pf_F(const double* __restrict__ u, int x, int y, const PfGrid& g) {
  const double v = u[y * g.nx + x];
  return pf_lap(u, x, y, g.nx, g.ny, g.bc, g.cx, g.cy, g.lam) + g.gamma * (v - v * v * v);
}

// per-node weights passed by value (last row of Q, or the nodes c)
struct PfNodes {
  double w[kMaxM];
};

// z_n = tau_n + dt sum_j q_j F(V_{n,j})  on the finer grid (tau may be null).
__global__ __launch_bounds__(kPfBlock) void k_pf_z(const double* __restrict__ V, const double* __restrict__ tau,
                                                   double* __restrict__ z, int N, int M, PfGrid g, double dt,
                                                   PfNodes q) {
  const int P = g.nx * g.ny;
  const size_t total = (size_t)N * P;
  for (size_t e = (size_t)blockIdx.x * kPfBlock + threadIdx.x; e < total; e += (size_t)gridDim.x * kPfBlock) {
    const int n = (int)(e / P), p = (int)(e % P);
    const int x = p % g.nx, y = p / g.nx;
    double s = 0.0;
    for (int j = 0; j < M; ++j)
      s += q.w[j] * pf_F(V + ((size_t)n * M + j) * P, x, y, g);
    z[e] = (tau ? tau[e] : 0.0) + dt * s;
  }
}

// Full weighting at coarse point (X, Y) of a fine plane: weights 1/4, 1/2,
// 1/4 per dimension around fine (2X, 2Y), periodic wrap or Neumann mirror.
__device__ __forceinline__ double pf_fw(const double* __restrict__ f, int X, int Y, int nxf, int nyf, int bc) {
  const int x = 2 * X, xm = pf_lo(x, nxf, bc), xp = pf_hi(x, nxf, bc);
  auto row = [&](int y) { return 0.25 * f[y * nxf + xm] + 0.5 * f[y * nxf + x] + 0.25 * f[y * nxf + xp]; };
  if (nyf == 1) return row(0);
  const int y = 2 * Y;
  return 0.25 * row(pf_lo(y, nyf, bc)) + 0.5 * row(y) + 0.25 * row(pf_hi(y, nyf, bc));
}

// out[n][0] = R_s a_n, out[n][1] = R_s b_n (a_n = a + n sa, b_n = b + n sb)
__global__ __launch_bounds__(kPfBlock) void k_pf_restrict(const double* __restrict__ a, size_t sa,
                                                          const double* __restrict__ b, size_t sb,
                                                          double* __restrict__ out, int N, int nxf, int nyf,
                                                          int nxc, int nyc, int bc) {
  const int Pc = nxc * nyc;
  const size_t total = (size_t)N * Pc;
  for (size_t e = (size_t)blockIdx.x * kPfBlock + threadIdx.x; e < total; e += (size_t)gridDim.x * kPfBlock) {
    const int n = (int)(e / Pc), p = (int)(e % Pc);
    const int X = p % nxc, Y = p / nxc;
    out[((size_t)n * 2) * Pc + p] = pf_fw(a + n * sa, X, Y, nxf, nyf, bc);
    out[((size_t)n * 2 + 1) * Pc + p] = pf_fw(b + n * sb, X, Y, nxf, nyf, bc);
  }
}

// tau_n = (R z)_n - dt F (R V_M)_n;  V_n = (R V_M)_n   on the coarser grid
__global__ __launch_bounds__(kPfBlock) void k_pf_tau(const double* __restrict__ pack, double* __restrict__ tau,
                                                     double* __restrict__ V, int N, PfGrid g, double dt) {
  const int P = g.nx * g.ny;
  const size_t total = (size_t)N * P;
  for (size_t e = (size_t)blockIdx.x * kPfBlock + threadIdx.x; e < total; e += (size_t)gridDim.x * kPfBlock) {
    const int n = (int)(e / P), p = (int)(e % P);
    const int x = p % g.nx, y = p / g.nx;
    const double* rz = pack + ((size_t)n * 2) * P;
    const double* rv = rz + P;
    tau[e] = rz[p] - dt * pf_F(rv, x, y, g);
    V[e] = rv[p];
  }
}

// Linear interpolation to fine (x, y) of the coarse correction e = W - RV:
// fine 2X = coarse X, fine 2X + 1 = mean of coarse X and X + 1 (periodic
// wrap; on Neumann grids both ends are kept, so X + 1 stays inside), first
// along x, then along y.
__device__ __forceinline__ double pf_interp_e(const double* __restrict__ W, const double* __restrict__ RV, int x,
                                              int y, int nxc, int nyc) {
  auto e = [&](int X, int Y) { return W[Y * nxc + X] - RV[Y * nxc + X]; };
  const int X0 = x / 2, X1 = X0 + 1 == nxc ? 0 : X0 + 1;
  auto gx = [&](int Y) { return (x & 1) ? 0.5 * (e(X0, Y) + e(X1, Y)) : e(X0, Y); };
  const int Y0 = y / 2, Y1 = Y0 + 1 == nyc ? 0 : Y0 + 1;
  return (nyc > 1 && (y & 1)) ? 0.5 * (gx(Y0) + gx(Y1)) : gx(Y0);
}

// V_{n,i} += P_s ((1 - c_i) e_{n-1} + c_i e_n) on the finer grid
__global__ __launch_bounds__(kPfBlock) void k_pf_correct(double* __restrict__ V, int N, int M, int nxf, int nyf,
                                                         const double* __restrict__ W,
                                                         const double* __restrict__ pack, int nxc, int nyc,
                                                         PfNodes c) {
  const int P = nxf * nyf, Pc = nxc * nyc;
  const size_t total = (size_t)N * P;
  for (size_t e = (size_t)blockIdx.x * kPfBlock + threadIdx.x; e < total; e += (size_t)gridDim.x * kPfBlock) {
    const int n = (int)(e / P), p = (int)(e % P);
    const int x = p % nxf, y = p / nxf;
    const double en = pf_interp_e(W + (size_t)n * Pc, pack + ((size_t)n * 2 + 1) * Pc, x, y, nxc, nyc);
    const double ep =
        n > 0 ? pf_interp_e(W + (size_t)(n - 1) * Pc, pack + ((size_t)(n - 1) * 2 + 1) * Pc, x, y, nxc, nyc) : 0.0;
    for (int i = 0; i < M; ++i) V[((size_t)n * M + i) * P + p] += (1.0 - c.w[i]) * ep + c.w[i] * en;
  }
}

// rhs_n = V_{n-1} + tau_n + dt R(V_n)  (V_{-1} = u0): the slab solves
// (I - dt L) V'_n = rhs_n of a Jacobi sweep at M = 1 (R = 0 when linear)
__global__ __launch_bounds__(kPfBlock) void k_pf_jrhs(const double* __restrict__ V, const double* __restrict__ tau,
                                                      const double* __restrict__ u0, double* __restrict__ rhs, int N,
                                                      int P, double dt, double gamma) {
  const size_t total = (size_t)N * P;
  for (size_t e = (size_t)blockIdx.x * kPfBlock + threadIdx.x; e < total; e += (size_t)gridDim.x * kPfBlock) {
    const size_t n = e / P, p = e % P;
    const double v = V[e];
    rhs[e] = (n > 0 ? V[e - P] : u0[p]) + tau[e] + dt * gamma * (v - v * v * v);
  }
}

// The serial IMEX sweep at M = 1, slab n: rhs = a + dt (R(a) - R(a_old)) +
// dt R(V_old_n) + tau_n with a the new end value of slab n - 1 (u0 for n = 0)
// and a_old its incoming value; then (I - dt L) V_n = rhs.
__global__ __launch_bounds__(kPfBlock) void k_pf_srhs(const double* __restrict__ V, const double* __restrict__ Vold,
                                                      const double* __restrict__ tau, const double* __restrict__ u0,
                                                      double* __restrict__ rhs, int n, int P, double dt,
                                                      double gamma) {
  auto R = [&](double v) { return gamma * (v - v * v * v); };
  for (int p = blockIdx.x * kPfBlock + threadIdx.x; p < P; p += gridDim.x * kPfBlock) {
    const double a = n > 0 ? V[(size_t)(n - 1) * P + p] : u0[p];
    const double ao = n > 0 ? Vold[(size_t)(n - 1) * P + p] : u0[p];
    const double vo = Vold[(size_t)n * P + p];
    rhs[p] = a + dt * (R(a) - R(ao)) + dt * R(vo) + tau[(size_t)n * P + p];
  }
}

int pf_blocks(size_t total) {
  size_t b = (total + kPfBlock - 1) / kPfBlock;
  if (b > 8192) b = 8192;
  return b < 1 ? 1 : static_cast<int>(b);
}

}  // namespace

#define PF_CHECK(expr)                                                           \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return STMG_EHIP;                                                          \
    }                                                                            \
  } while (0)

int Solver::pfasst(const double* u0, double* U, stmg_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  if (pf.empty() || sdcn.empty()) {
    set_error("stmg_pfasst_solve: set up the handle with options.pfasst_levels >= 2 (linear problems)");
    return STMG_EUNSUPPORTED;
  }
  const int nl = static_cast<int>(pf.size()) + 1, nu = opt.pfasst_sweeps;
  // the inner-solve cap holds for this call only
  struct CapGuard {
    int& c;
    ~CapGuard() { c = 0; }
  } cap_guard{inner_cap};
  inner_cap = opt.pfasst_inner_cycles;
  const int N = lv[0].N, M0 = prob.M;
  const double dt = prob.dt;
  // level l: grid, nodes, iterate, FAS right-hand side
  const double gam = allen_cahn ? prob.gamma : 0.0;
  auto grid = [&](int l) {
    const OpParams& o = l == 0 ? lv[0].op : pf[l - 1].sol->lv[0].op;
    return PfGrid{o.nx, o.ny, o.bc, o.cx, o.cy, o.lam, gam};
  };
  auto nodes = [&](int l) { return l == 0 ? M0 : 1; };
  auto iter = [&](int l) { return l == 0 ? U : pf[l - 1].V; };
  PfNodes qM{}, c0{};
  for (int j = 0; j < M0; ++j) {
    qM.w[j] = static_cast<double>(tab.Q[M0 - 1][j]);
    c0.w[j] = static_cast<double>(tab.c[j]);
  }
  PfNodes q1{}, c1{};
  q1.w[0] = 1.0;  // Q = [1] and c = [1] at M = 1
  c1.w[0] = 1.0;
  // initial values of the coarser levels: u0_{l+1} = R_s u0_l
  for (int l = 0; l + 1 < nl; ++l) {
    const PfGrid f = grid(l), c = grid(l + 1);
    const double* src = l == 0 ? u0 : pf[l - 1].u0;
    // both outputs of the pair kernel land in the level's pack buffer (N * 2 planes)
    hipLaunchKernelGGL(k_pf_restrict, dim3(pf_blocks(static_cast<size_t>(c.nx) * c.ny)), dim3(kPfBlock), 0, stream,
                       src, 0, src, 0, pf[l].pack, 1, f.nx, f.ny, c.nx, c.ny, f.bc);
    PF_CHECK(hipGetLastError());
    PF_CHECK(hipMemcpyAsync(pf[l].u0, pf[l].pack, sizeof(double) * c.nx * c.ny, hipMemcpyDeviceToDevice, stream));
  }
  // An M = 1 level solve A V = f (+ u0 entering slab 0), warm-started from V,
  // to rtol relative to (||f||^2 + ||u0||^2)^{1/2}.  (Relative to the first
  // residual would ask a sweep that starts from an exact V for a reduction
  // below rounding.)
  auto level_solve = [&](PfLevel& q, const double* f, const double* u0l) -> int {
    const size_t P = static_cast<size_t>(q.nx) * q.ny;
    int np = 0;
    PF_CHECK(launch_sumsq(f, N * P, part, &np, stream));
    PF_CHECK(launch_sum_partials(part, np, scal + 2, stream));
    double s2[2] = {0.0, 0.0};
    if (u0l) {
      PF_CHECK(launch_sumsq(u0l, P, part, &np, stream));
      PF_CHECK(launch_sum_partials(part, np, scal + 3, stream));
    }
    PF_CHECK(hipMemcpyAsync(s2, scal + 2, 2 * sizeof(double), hipMemcpyDeviceToHost, stream));
    PF_CHECK(hipStreamSynchronize(stream));
    const double nb = std::sqrt(s2[0] + (u0l ? s2[1] : 0.0));
    if (!std::isfinite(nb)) return STMG_ENAN;
    if (nb == 0.0) {
      PF_CHECK(hipMemsetAsync(q.V, 0, N * P * sizeof(double), stream));
      return STMG_OK;
    }
    return inner_solve(q.sol.get(), f, u0l, q.V, nb);
  };
  // one Jacobi sweep on an M = 1 level: V_n <- (I - dt L)^-1 (V_{n-1} + tau_n)
  auto jacobi = [&](int l) -> int {
    PfLevel& q = pf[l - 1];
    const size_t P = static_cast<size_t>(q.nx) * q.ny;
    hipLaunchKernelGGL(k_pf_jrhs, dim3(pf_blocks(N * P)), dim3(kPfBlock), 0, stream, q.V, q.tau, q.u0, q.rhs, N,
                       static_cast<int>(P), dt, gam);
    PF_CHECK(hipGetLastError());
    return level_solve(q, q.rhs, nullptr);
  };
  const double nb = norm_u0_b(u0);
  if (nb < 0.0) return STMG_EHIP;
  stmg_stats s{};
  // the statistics are filled on every way out, an inner solve's failure too
  auto done = [&](int status) {
    s.status = status;
    s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    last = s;
    if (st) *st = s;
    return status;
  };
  int status = STMG_ENOTCONV;
  double rel = 0.0, rel0 = -1.0, prev = 0.0;
  int incr = 0;
  for (int it = 0; it < opt.max_cycles; ++it) {
    // down: sweeps, then the FAS restriction
    for (int l = 0; l + 1 < nl; ++l) {
      if (l == 0) {
        const int rc = sdc_core(u0, U, nu);
        if (rc) return done(rc);
      } else {
        for (int k = 0; k < nu; ++k) {
          const int rc = jacobi(l);
          if (rc) return done(rc);
        }
      }
      const PfGrid f = grid(l), c = grid(l + 1);
      const int Mf = nodes(l);
      const size_t Pf = static_cast<size_t>(f.nx) * f.ny, Pc = static_cast<size_t>(c.nx) * c.ny;
      const double* V = iter(l);
      hipLaunchKernelGGL(k_pf_z, dim3(pf_blocks(N * Pf)), dim3(kPfBlock), 0, stream, V,
                         l == 0 ? nullptr : pf[l - 1].tau, pf_pack, N, Mf, f, dt, l == 0 ? qM : q1);
      PF_CHECK(hipGetLastError());
      hipLaunchKernelGGL(k_pf_restrict, dim3(pf_blocks(N * Pc)), dim3(kPfBlock), 0, stream, pf_pack, Pf,
                         V + (Mf - 1) * Pf, Mf * Pf, pf[l].pack, N, f.nx, f.ny, c.nx, c.ny, f.bc);
      PF_CHECK(hipGetLastError());
      hipLaunchKernelGGL(k_pf_tau, dim3(pf_blocks(N * Pc)), dim3(kPfBlock), 0, stream, pf[l].pack, pf[l].tau,
                         pf[l].V, N, c, dt);
      PF_CHECK(hipGetLastError());
    }
    // the coarsest level: the serial sweep.  Linear: it solves the level's
    // block lower-bidiagonal system, done for all slabs at once.  IMEX: slab
    // after slab with the one-slab solver, nu times.
    if (!pf.back().serial) {
      const int rc = level_solve(pf.back(), pf.back().tau, pf.back().u0);
      if (rc) return done(rc);
    } else {
      PfLevel& q = pf.back();
      Solver* S1 = q.sol.get();
      const size_t P = static_cast<size_t>(q.nx) * q.ny;
      for (int k = 0; k < nu; ++k) {
        PF_CHECK(hipMemcpyAsync(q.rhs, q.V, N * P * sizeof(double), hipMemcpyDeviceToDevice, stream));
        for (int n = 0; n < N; ++n) {
          double* rhs = q.pack + static_cast<size_t>(n) * 2 * P;  // slot 0 (R z) is spent
          double* Vn = q.V + static_cast<size_t>(n) * P;
          hipLaunchKernelGGL(k_pf_srhs, dim3(pf_blocks(P)), dim3(kPfBlock), 0, stream, q.V, q.rhs, q.tau, q.u0, rhs,
                             n, static_cast<int>(P), dt, gam);
          PF_CHECK(hipGetLastError());
          if (S1->lv.size() == 1) {
            PF_CHECK(S1->coarse<double>(false, REACT_CONST, rhs, nullptr, Vn));  // exact
          } else {
            int np = 0;
            double b2 = 0.0;
            PF_CHECK(launch_sumsq(rhs, P, part, &np, stream));
            PF_CHECK(launch_sum_partials(part, np, scal + 2, stream));
            const int rc = read_scalar(scal + 2, &b2);
            if (rc) return done(rc);
            if (!std::isfinite(b2)) return done(STMG_ENAN);
            if (b2 == 0.0) {
              PF_CHECK(hipMemsetAsync(Vn, 0, P * sizeof(double), stream));
              continue;
            }
            const int rc2 = inner_solve(S1, rhs, nullptr, Vn, std::sqrt(b2));
            if (rc2) return done(rc2);
          }
        }
      }
    }
    // up: corrections, then the sweeps of the M = 1 levels
    for (int l = nl - 2; l >= 0; --l) {
      const PfGrid f = grid(l), c = grid(l + 1);
      const size_t Pf = static_cast<size_t>(f.nx) * f.ny;
      hipLaunchKernelGGL(k_pf_correct, dim3(pf_blocks(N * Pf)), dim3(kPfBlock), 0, stream, iter(l), N, nodes(l),
                         f.nx, f.ny, pf[l].V, pf[l].pack, c.nx, c.ny, l == 0 ? c0 : c1);
      PF_CHECK(hipGetLastError());
      if (l > 0) {
        for (int k = 0; k < nu; ++k) {
          const int rc = jacobi(l);
          if (rc) return done(rc);
        }
      }
    }
    // stop test on level 0
    PF_CHECK(residual64<double>(false, allen_cahn ? REACT_AC : REACT_CONST, U, nullptr, u0, nullptr, scal));
    double r2 = 0.0;
    const int rc = read_scalar(scal, &r2);
    if (rc) return done(rc);
    rel = nb > 0.0 ? std::sqrt(r2) / nb : std::sqrt(r2);
    s.cycles = it + 1;
    if (!std::isfinite(rel)) { status = STMG_ENAN; break; }
    if (rel <= opt.rtol) { status = STMG_OK; break; }
    if (rel0 < 0.0) rel0 = rel;
    if (rel > 1e3 * (rel0 > 0.0 ? rel0 : 1.0)) { status = STMG_EDIVERGED; break; }
    // growth of more than 10% per iteration, five in a row (not rounding-floor noise)
    incr = (it > 0 && rel > 1.1 * prev) ? incr + 1 : 0;
    if (incr >= 5) { status = STMG_EDIVERGED; break; }
    prev = rel;
  }
  s.rel_res = rel;
  return done(status);
}

}  // namespace stmg
