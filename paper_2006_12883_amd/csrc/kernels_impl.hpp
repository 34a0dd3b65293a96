// Device code of the space-time multigrid kernels (included by the
// instantiation units; internal to libstmg).
//
// All operator kernels work on space-time vectors laid out [N][M][ny][nx]
// (slab, node, space; Sec. 3).  A thread owns one spatial point and marches
// through a run of consecutive slabs: the M node values of its point and the
// coupling value from the previous slab stay in registers, so a slab's
// end-value plane is never re-read from memory inside a run.  Spatial
// neighbours come through the L1/L2 caches; the block index is remapped so
// that consecutive spatial tiles run on the same XCD (shared L2).  The small
// M x M time coupling is done with scalar constants from the kernel argument
// block; it is 2M flops per unknown, far too little to use matrix cores.
#pragma once
#include "kernels.hpp"

namespace stmg {

namespace {

// Consecutive logical blocks on one XCD: hardware places block b on XCD b % 8.
__device__ __forceinline__ int xcd_remap(int bid, int nb) {
  const int X = 8;
  const int q = nb / X, r = nb % X;
  const int xcd = bid % X, k = bid / X;
  return xcd * q + (xcd < r ? xcd : r) + k;
}

__device__ __forceinline__ int nb_lo(int i, int n, int bc) {
  return i > 0 ? i - 1 : (bc == 0 ? n - 1 : 1);
}
__device__ __forceinline__ int nb_hi(int i, int n, int bc) {
  return i < n - 1 ? i + 1 : (bc == 0 ? 0 : n - 2);
}

// Sum over the workgroup (256 threads); the result is valid in thread 0.
__device__ __forceinline__ double block_sum(double v) {
  __shared__ double red[kBlock / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kBlock / 64; ++i) t += red[i];
  }
  return t;
}

// Adds one point's contribution to ||r||^2 (FP64) in the form of the level: the
// DG residual as computed, or its collocation form G r with G = Q diag(b)^-1
// (the same solution; the residuals differ by this per-point factor).
template <int M, typename T>
__device__ __forceinline__ void ssq_add(const OpParams& p, const T r[M], double& ssq) {
  if (p.colloc) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j < M; ++j) v += p.G[i * M + j] * (double)r[j];
      ssq += v * v;
    }
  } else {
#pragma unroll
    for (int i = 0; i < M; ++i) ssq += (double)r[i] * (double)r[i];
  }
}

// Constants of a level converted to the arithmetic type T.
template <int M, typename T>
struct Consts {
  T K[M][M], Bi[M][M], db[M], cin[M], cout[M];
  T cx, cy, lam, gamma, omega;
  __device__ __forceinline__ explicit Consts(const OpParams& p) {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      db[i] = (T)p.db[i];
      cin[i] = (T)p.cin[i];
      cout[i] = (T)p.cout[i];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        K[i][j] = (T)p.K[i * M + j];
        Bi[i][j] = (T)p.Binv[i * M + j];
      }
    }
    cx = (T)p.cx;
    cy = (T)p.cy;
    lam = (T)p.lam;
    gamma = (T)p.gamma;
    omega = (T)p.omega;
  }
};

// Neighbour offsets of point q inside a plane.
struct Nbr {
  int xm, xp, ym, yp;
};

__device__ __forceinline__ Nbr neighbours(int x, int y, int nx, int ny, int bc) {
  Nbr o;
  o.xm = y * nx + nb_lo(x, nx, bc);
  o.xp = y * nx + nb_hi(x, nx, bc);
  o.ym = ny > 1 ? nb_lo(y, ny, bc) * nx + x : 0;
  o.yp = ny > 1 ? nb_hi(y, ny, bc) * nx + x : 0;
  return o;
}

// Loads the M node values at point q of slab `base` and their 5-point
// Laplacians (scaled by cx, cy).
template <int M, typename T>
__device__ __forceinline__ void load_point(const T* __restrict__ U, size_t base, int P, int q,
                                           const Nbr& nb, bool twod, T cx, T cy, T u[M],
                                           T lap[M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const T* Um = U + base + (size_t)m * P;
    const T c = Um[q];
    T l = cx * (Um[nb.xm] + Um[nb.xp] - c - c);
    if (twod) l += cy * (Um[nb.ym] + Um[nb.yp] - c - c);
    u[m] = c;
    lap[m] = l;
  }
}

// r_i = f_i - [sum_j K_ij u_j + db_i (-lap_i + react_i) - cin_i prev]
template <int M, typename T, int REACT>
__device__ __forceinline__ void point_residual(const Consts<M, T>& c, const T u[M],
                                               const T lap[M], const T* __restrict__ coef,
                                               const T* __restrict__ f, size_t base, int P,
                                               int q, T prev, T r[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T au = T(0);
#pragma unroll
    for (int j = 0; j < M; ++j) au += c.K[i][j] * u[j];
    T react;
    if (REACT == REACT_CONST) react = c.lam * u[i];
    else if (REACT == REACT_COEF) react = coef[base + (size_t)i * P + q] * u[i];
    else react = c.gamma * (u[i] * u[i] * u[i] - u[i]);
    au += c.db[i] * (react - lap[i]);
    au -= c.cin[i] * prev;
    const T fi = f ? f[base + (size_t)i * P + q] : T(0);
    r[i] = fi - au;
  }
}

// d = B^{-1} rhs with B = K + diag(db_i (dg + coef_i)), no pivoting
// (K has positive leading minors and the added diagonal is positive in
// practice; the constant-coefficient case uses the precomputed inverse).
template <int M, typename T>
__device__ __forceinline__ void point_block_solve(const Consts<M, T>& c, T dg, const T coefv[M],
                                                  T x[M]) {
  T A[M][M];
#pragma unroll
  for (int i = 0; i < M; ++i) {
#pragma unroll
    for (int j = 0; j < M; ++j) A[i][j] = c.K[i][j];
    A[i][i] += c.db[i] * (dg + coefv[i]);
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    const T inv = T(1) / A[k][k];
#pragma unroll
    for (int i = k + 1; i < M; ++i) {
      const T l = A[i][k] * inv;
#pragma unroll
      for (int j = k + 1; j < M; ++j) A[i][j] -= l * A[k][j];
      x[i] -= l * x[k];
    }
  }
#pragma unroll
  for (int k = M - 1; k >= 0; --k) {
    T s = x[k];
#pragma unroll
    for (int j = k + 1; j < M; ++j) s -= A[k][j] * x[j];
    x[k] = s / A[k][k];
  }
}

// ---------------------------------------------------------------------------
// Smoother: block-Jacobi over chunks of S slabs.  Inside a chunk the
// block lower-bidiagonal time coupling is inverted by forward substitution
// with the point-block (M x M) diagonal in space:
//   d_n = B^{-1} (r_n + [n > n0] cin (cout . d_{n-1})),  U_out = U + omega d,
// where r = f - A U uses the old iterate everywhere (Jacobi in space and
// across chunks).  One thread = one point x one chunk.
template <int M, typename T, int REACT>
__global__ __launch_bounds__(kBlock) void k_smooth(const OpParams p, const SweepPtrs<T> a, int S,
                                                   int tiles, int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int tile = lb % tiles;
  const int n0 = (lb / tiles) * S;
  const int P = p.nx * p.ny;
  const int q = tile * kBlock + threadIdx.x;
  double ssq = 0.0;  // ||f - A U||^2 of the input iterate (optional output)
  if (q < P && n0 < p.N) {
    const int n1 = min(n0 + S, p.N);
    const Consts<M, T> c(p);
    const bool twod = p.ny > 1;
    const Nbr nb = neighbours(q % p.nx, q / p.nx, p.nx, p.ny, p.bc);
    const T dg = T(2) * c.cx + (twod ? T(2) * c.cy : T(0));
    T* __restrict__ out = static_cast<T*>(a.out);

    T prev = T(0);
    if (n0 == 0) {
      if (a.u0) prev = (T)a.u0[q];
    } else if (a.U) {
      const size_t b = (size_t)(n0 - 1) * M * P;
#pragma unroll
      for (int j = 0; j < M; ++j) prev += c.cout[j] * a.U[b + (size_t)j * P + q];
    }
    T dprev = T(0);
    for (int n = n0; n < n1; ++n) {
      const size_t base = (size_t)n * M * P;
      T u[M], lap[M], r[M];
      if (a.U) {
        load_point<M, T>(a.U, base, P, q, nb, twod, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) u[m] = lap[m] = T(0);
      }
      point_residual<M, T, REACT>(c, u, lap, a.coef, a.f, base, P, q, prev, r);
      if (a.part) ssq_add<M, T>(p, r, ssq);
      if (n > n0) {
#pragma unroll
        for (int i = 0; i < M; ++i) r[i] += c.cin[i] * dprev;
      }
      T d[M];
      if (REACT == REACT_COEF) {
        T cv[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
          cv[i] = a.coef[base + (size_t)i * P + q];
          d[i] = r[i];
        }
        point_block_solve<M, T>(c, dg, cv, d);
      } else {
#pragma unroll
        for (int i = 0; i < M; ++i) {
          T sm = T(0);
#pragma unroll
          for (int k = 0; k < M; ++k) sm += c.Bi[i][k] * r[k];
          d[i] = sm;
        }
      }
      T np = T(0), nd = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        out[base + (size_t)i * P + q] = u[i] + c.omega * d[i];
        np += c.cout[i] * u[i];
        nd += c.cout[i] * d[i];
      }
      prev = np;
      dprev = nd;
    }
  }
  if (a.part) {
    const double t = block_sum(ssq);
    if (threadIdx.x == 0) a.part[lb] = t;
  }
}

// Residual r = f - A U (+ coupling of u0 into slab 0), optionally stored
// as TO, with per-block partial sums of r^2.
template <int M, typename T, typename TO, int REACT>
__global__ __launch_bounds__(kBlock) void k_residual(const OpParams p, const SweepPtrs<T> a, int S,
                                                     int tiles, int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int tile = lb % tiles;
  const int n0 = (lb / tiles) * S;
  const int P = p.nx * p.ny;
  const int q = tile * kBlock + threadIdx.x;
  double ssq = 0.0;
  if (q < P && n0 < p.N) {
    const int n1 = min(n0 + S, p.N);
    const Consts<M, T> c(p);
    const bool twod = p.ny > 1;
    const Nbr nb = neighbours(q % p.nx, q / p.nx, p.nx, p.ny, p.bc);
    TO* __restrict__ out = static_cast<TO*>(a.out);
    T prev = T(0);
    if (n0 == 0) {
      if (a.u0) prev = (T)a.u0[q];
    } else if (a.U) {
      const size_t b = (size_t)(n0 - 1) * M * P;
#pragma unroll
      for (int j = 0; j < M; ++j) prev += c.cout[j] * a.U[b + (size_t)j * P + q];
    }
    for (int n = n0; n < n1; ++n) {
      const size_t base = (size_t)n * M * P;
      T u[M], lap[M], r[M];
      if (a.U) {
        load_point<M, T>(a.U, base, P, q, nb, twod, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) u[m] = lap[m] = T(0);
      }
      point_residual<M, T, REACT>(c, u, lap, a.coef, a.f, base, P, q, prev, r);
      T np = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        if (out) out[base + (size_t)i * P + q] = (TO)r[i];
        np += c.cout[i] * u[i];
      }
      ssq_add<M, T>(p, r, ssq);
      prev = np;
    }
  }
  if (a.part) {
    const double t = block_sum(ssq);
    if (threadIdx.x == 0) a.part[lb] = t;
  }
}

// ---------------------------------------------------------------------------
// Fused residual + restriction.  One thread = one coarse point x a run of
// coarse slabs.  For every fine slab of the run it evaluates the fine
// residual at the (up to 3 x 3) fine points of the full-weighting stencil
// [1 2 1]/4 per coarsened dimension (coarse X = fine 2X; periodic wrap or
// Neumann reflection), then accumulates in time with the [1 2 1]/2 stencil
// over slab end points (coarse J = fine 2J+1; the slab after the last is
// absent).  The previous-slab coupling value of each fine point is carried
// in registers from one fine slab to the next.
template <int M, typename T, int REACT, bool SP, bool TM, bool TWOD>
__global__ __launch_bounds__(kBlock) void k_restrict(const OpParams p, const SweepPtrs<T> a,
                                                     int ncx, int ncy, int Nc, T* __restrict__ fc,
                                                     int S, int tiles, int nblocks) {
  constexpr int WX = SP ? 3 : 1;
  constexpr int WY = (SP && TWOD) ? 3 : 1;
  constexpr int NP = WX * WY;
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int tile = lb % tiles;
  const int J0 = (lb / tiles) * S;
  const int Pc = ncx * ncy;
  const int qc = tile * kBlock + threadIdx.x;
  if (qc >= Pc || J0 >= Nc) return;
  const int J1 = min(J0 + S, Nc);
  const Consts<M, T> c(p);
  const int nx = p.nx, ny = p.ny, P = nx * ny;
  const int X = qc % ncx, Y = qc / ncx;

  int qf[NP];
  Nbr nbf[NP];
  T w[NP];
  {
    int xs[WX], ys[WY];
    T wx[WX], wy[WY];
    if (SP) {
      xs[0] = nb_lo(2 * X, nx, p.bc); xs[WX / 2] = 2 * X; xs[WX - 1] = nb_hi(2 * X, nx, p.bc);
      wx[0] = T(0.25); wx[WX / 2] = T(0.5); wx[WX - 1] = T(0.25);
    } else {
      xs[0] = X; wx[0] = T(1);
    }
    if (SP && TWOD) {
      ys[0] = nb_lo(2 * Y, ny, p.bc); ys[WY / 2] = 2 * Y; ys[WY - 1] = nb_hi(2 * Y, ny, p.bc);
      wy[0] = T(0.25); wy[WY / 2] = T(0.5); wy[WY - 1] = T(0.25);
    } else {
      ys[0] = Y; wy[0] = T(1);
    }
#pragma unroll
    for (int j = 0; j < WY; ++j)
#pragma unroll
      for (int i = 0; i < WX; ++i) {
        const int k = j * WX + i;
        qf[k] = ys[j] * nx + xs[i];
        nbf[k] = neighbours(xs[i], ys[j], nx, ny, p.bc);
        w[k] = wx[i] * wy[j];
      }
  }
  // fine slab range of this run
  const int nlo = TM ? 2 * J0 : J0;
  const int nhi = TM ? min(2 * J1, p.N - 1) : J1 - 1;
  T prev[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    prev[k] = T(0);
    if (nlo == 0) {
      if (a.u0) prev[k] = (T)a.u0[qf[k]];
    } else if (a.U) {
      const size_t b = (size_t)(nlo - 1) * M * P;
#pragma unroll
      for (int j = 0; j < M; ++j) prev[k] += c.cout[j] * a.U[b + (size_t)j * P + qf[k]];
    }
  }
  T acc[M];
#pragma unroll
  for (int i = 0; i < M; ++i) acc[i] = T(0);
  const bool twod = ny > 1;  // the operator's dimension (TWOD only shapes the stencil)
  for (int n = nlo; n <= nhi; ++n) {
    const size_t base = (size_t)n * M * P;
    T rs[M];
#pragma unroll
    for (int i = 0; i < M; ++i) rs[i] = T(0);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      T u[M], lap[M], r[M];
      if (a.U) {
        load_point<M, T>(a.U, base, P, qf[k], nbf[k], twod, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) u[m] = lap[m] = T(0);
      }
      point_residual<M, T, REACT>(c, u, lap, a.coef, a.f, base, P, qf[k], prev[k], r);
      T np = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        rs[i] += w[k] * r[i];
        np += c.cout[i] * u[i];
      }
      prev[k] = np;
    }
    if (!TM) {
      const size_t cb = (size_t)n * M * Pc;
#pragma unroll
      for (int i = 0; i < M; ++i) fc[cb + (size_t)i * Pc + qc] = rs[i];
    } else if (n & 1) {  // n = 2J + 1: centre of coarse slab J
      const int J = n >> 1;
#pragma unroll
      for (int i = 0; i < M; ++i) acc[i] += rs[i];
      if (J == Nc - 1) {  // the fine slab 2J + 2 does not exist
        const size_t cb = (size_t)J * M * Pc;
#pragma unroll
        for (int i = 0; i < M; ++i) fc[cb + (size_t)i * Pc + qc] = acc[i];
      }
    } else {  // n = 2J: right neighbour of coarse J - 1, left neighbour of J
      const int J = n >> 1;
      if (J > J0) {
        const size_t cb = (size_t)(J - 1) * M * Pc;
#pragma unroll
        for (int i = 0; i < M; ++i) fc[cb + (size_t)i * Pc + qc] = acc[i] + T(0.5) * rs[i];
      }
#pragma unroll
      for (int i = 0; i < M; ++i) acc[i] = T(0.5) * rs[i];
    }
  }
}

// Fused residual + space restriction with an LDS tile.  A workgroup owns a
// TCX x TCY tile of coarse points and a run of coarse slabs.  For each fine
// slab it evaluates the residual once at every fine point of the
// (2 TCX + 1) x (2 TCY + 1) fine tile (coarse X = fine 2X, tile origin at fine
// 2 X0 - 1) into LDS, then every thread applies the [1 2 1]/4 full-weighting
// stencil of its coarse point from LDS and, with time coarsening, the
// [1 2 1]/2 stencil over slab end points in registers.  The coupling value of
// each fine point from the previous fine slab stays in the registers of the
// thread that owns that fine point.
template <int M, typename T, int REACT, bool TM, bool TWOD, int TCX, int TCY>
__global__ __launch_bounds__(kBlock) void k_restrict_lds(const OpParams p, const SweepPtrs<T> a,
                                                         int ncx, int ncy, int Nc,
                                                         T* __restrict__ fc, int S, int tiles_x,
                                                         int tiles, int nblocks) {
  constexpr int FW = 2 * TCX + 1;
  constexpr int FH = TWOD ? 2 * TCY + 1 : 1;
  constexpr int NF = FW * FH;
  constexpr int KMAX = (NF + kBlock - 1) / kBlock;
  __shared__ T rs[M][FH][FW];
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int tile = lb % tiles;
  const int J0 = (lb / tiles) * S;
  if (J0 >= Nc) return;  // whole workgroup leaves together
  const int J1 = min(J0 + S, Nc);
  const int X0 = (tile % tiles_x) * TCX;
  const int Y0 = TWOD ? (tile / tiles_x) * TCY : 0;
  const Consts<M, T> c(p);
  const int nx = p.nx, ny = p.ny, P = nx * ny;
  const bool twod = ny > 1;
  const int Pc = ncx * ncy;

  // fine points owned by this thread in the LDS tile
  int qf[KMAX];
  Nbr nbf[KMAX];
  T prev[KMAX];
  const int nlo = TM ? 2 * J0 : J0;
  const int nhi = TM ? min(2 * J1, p.N - 1) : J1 - 1;
#pragma unroll
  for (int kk = 0; kk < KMAX; ++kk) {
    const int k = threadIdx.x + kk * kBlock;
    int fx = 2 * X0 - 1 + (k % FW);
    int fy = TWOD ? 2 * Y0 - 1 + (k / FW) : 0;
    // periodic wrap or Neumann reflection, then clamp (points beyond the
    // coarse grid's extent are computed but never used)
    if (fx < 0) fx = nb_lo(0, nx, p.bc);
    if (fx >= nx) fx = p.bc == 0 ? fx - nx : 2 * (nx - 1) - fx;
    fx = fx < 0 ? 0 : (fx >= nx ? nx - 1 : fx);
    if (TWOD) {
      if (fy < 0) fy = nb_lo(0, ny, p.bc);
      if (fy >= ny) fy = p.bc == 0 ? fy - ny : 2 * (ny - 1) - fy;
      fy = fy < 0 ? 0 : (fy >= ny ? ny - 1 : fy);
    }
    qf[kk] = fy * nx + fx;
    nbf[kk] = neighbours(fx, fy, nx, ny, p.bc);
    prev[kk] = T(0);
    if (k < NF) {
      if (nlo == 0) {
        if (a.u0) prev[kk] = (T)a.u0[qf[kk]];
      } else if (a.U) {
        const size_t b = (size_t)(nlo - 1) * M * P;
#pragma unroll
        for (int j = 0; j < M; ++j) prev[kk] += c.cout[j] * a.U[b + (size_t)j * P + qf[kk]];
      }
    }
  }
  // this thread's coarse point
  const int tx = threadIdx.x % TCX, ty = threadIdx.x / TCX;
  const int X = X0 + tx, Y = Y0 + ty;
  const bool cvalid = (threadIdx.x < TCX * TCY) && X < ncx && Y < ncy;
  const int qc = Y * ncx + X;
  T acc[M];
#pragma unroll
  for (int i = 0; i < M; ++i) acc[i] = T(0);

  for (int n = nlo; n <= nhi; ++n) {
    const size_t base = (size_t)n * M * P;
#pragma unroll
    for (int kk = 0; kk < KMAX; ++kk) {
      const int k = threadIdx.x + kk * kBlock;
      if (k < NF) {
        T u[M], lap[M], r[M];
        if (a.U) {
          load_point<M, T>(a.U, base, P, qf[kk], nbf[kk], twod, c.cx, c.cy, u, lap);
        } else {
#pragma unroll
          for (int m = 0; m < M; ++m) u[m] = lap[m] = T(0);
        }
        point_residual<M, T, REACT>(c, u, lap, a.coef, a.f, base, P, qf[kk], prev[kk], r);
        T np = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          rs[i][k / FW][k % FW] = r[i];
          np += c.cout[i] * u[i];
        }
        prev[kk] = np;
      }
    }
    __syncthreads();
    if (cvalid) {
      T rc[M];
      const int cx0 = 2 * tx, cy0 = TWOD ? 2 * ty : 0;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        T sx0 = T(0.25) * rs[i][cy0][cx0] + T(0.5) * rs[i][cy0][cx0 + 1] + T(0.25) * rs[i][cy0][cx0 + 2];
        if (TWOD) {
          const T sx1 = T(0.25) * rs[i][cy0 + 1][cx0] + T(0.5) * rs[i][cy0 + 1][cx0 + 1] +
                        T(0.25) * rs[i][cy0 + 1][cx0 + 2];
          const T sx2 = T(0.25) * rs[i][cy0 + 2][cx0] + T(0.5) * rs[i][cy0 + 2][cx0 + 1] +
                        T(0.25) * rs[i][cy0 + 2][cx0 + 2];
          sx0 = T(0.25) * sx0 + T(0.5) * sx1 + T(0.25) * sx2;
        }
        rc[i] = sx0;
      }
      if (!TM) {
        const size_t cb = (size_t)n * M * Pc;
#pragma unroll
        for (int i = 0; i < M; ++i) fc[cb + (size_t)i * Pc + qc] = rc[i];
      } else if (n & 1) {
        const int J = n >> 1;
#pragma unroll
        for (int i = 0; i < M; ++i) acc[i] += rc[i];
        if (J == Nc - 1) {
          const size_t cb = (size_t)J * M * Pc;
#pragma unroll
          for (int i = 0; i < M; ++i) fc[cb + (size_t)i * Pc + qc] = acc[i];
        }
      } else {
        const int J = n >> 1;
        if (J > J0) {
          const size_t cb = (size_t)(J - 1) * M * Pc;
#pragma unroll
          for (int i = 0; i < M; ++i) fc[cb + (size_t)i * Pc + qc] = acc[i] + T(0.5) * rc[i];
        }
#pragma unroll
        for (int i = 0; i < M; ++i) acc[i] = T(0.5) * rc[i];
      }
    }
    __syncthreads();
  }
}

// U_out = U_in + P e_c: linear interpolation in space (fine 2X = coarse X,
// fine 2X+1 = mean of coarse X and X+1) and in slab end points (fine 2J+1 =
// coarse J, fine 2J = mean of coarse J-1 and J, coarse -1 = 0).
template <int M, typename T, bool SP, bool TM, bool TWOD>
__global__ __launch_bounds__(kBlock) void k_prolong(const OpParams p, int ncx, int ncy, int Nc,
                                                    const T* __restrict__ ec,
                                                    const T* __restrict__ Uin, T* __restrict__ Uout,
                                                    int S, int tiles, int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int tile = lb % tiles;
  const int n0 = (lb / tiles) * S;
  const int nx = p.nx, ny = p.ny, P = nx * ny;
  const int q = tile * kBlock + threadIdx.x;
  if (q >= P || n0 >= p.N) return;
  const int n1 = min(n0 + S, p.N);
  const int Pc = ncx * ncy;
  const int x = q % nx, y = q / nx;
  int cq[4];
  T cw[4];
  int ncq = 0;
  {
    int xs[2], ys[2];
    T wx[2], wy[2];
    int nxs = 1, nys = 1;
    if (SP) {
      if (x & 1) {
        xs[0] = x >> 1; xs[1] = ((x >> 1) + 1) % ncx; wx[0] = wx[1] = T(0.5); nxs = 2;
        if (p.bc != 0) xs[1] = (x >> 1) + 1;
      } else {
        xs[0] = x >> 1; wx[0] = T(1);
      }
      if (TWOD) {
        if (y & 1) {
          ys[0] = y >> 1; ys[1] = ((y >> 1) + 1) % ncy; wy[0] = wy[1] = T(0.5); nys = 2;
          if (p.bc != 0) ys[1] = (y >> 1) + 1;
        } else {
          ys[0] = y >> 1; wy[0] = T(1);
        }
      } else {
        ys[0] = y; wy[0] = T(1);
      }
    } else {
      xs[0] = x; ys[0] = y; wx[0] = wy[0] = T(1);
    }
    for (int j = 0; j < nys; ++j)
      for (int i = 0; i < nxs; ++i) {
        cq[ncq] = ys[j] * ncx + xs[i];
        cw[ncq] = wx[i] * wy[j];
        ++ncq;
      }
  }
  for (int n = n0; n < n1; ++n) {
    int js[2];
    T wt[2];
    int nt;
    if (!TM) {
      js[0] = n; wt[0] = T(1); nt = 1;
    } else if (n & 1) {
      js[0] = n >> 1; wt[0] = T(1); nt = 1;
    } else {
      const int J = n >> 1;
      js[0] = J; wt[0] = T(0.5); nt = 1;
      if (J > 0) { js[1] = J - 1; wt[1] = T(0.5); nt = 2; }
    }
    const size_t base = (size_t)n * M * P;
#pragma unroll
    for (int i = 0; i < M; ++i) {
      T e = T(0);
      for (int t = 0; t < nt; ++t) {
        const T* Ec = ec + (size_t)js[t] * M * Pc + (size_t)i * Pc;
        T s = T(0);
        for (int k = 0; k < ncq; ++k) s += cw[k] * Ec[cq[k]];
        e += wt[t] * s;
      }
      const size_t o = base + (size_t)i * P + q;
      Uout[o] = (Uin ? Uin[o] : T(0)) + e;
    }
  }
}

// ---------------------------------------------------------------------------
// Register-blocked kernels for periodic grids with even point counts.  A
// thread owns a 2 x BY block of points (BY = 2 in 2D, 1 in 1D) and marches
// through its slabs.  Per node and slab it issues BY + 2 two-wide row loads
// (its own rows and the halo rows y0 - 1, y0 + BY) and 2 BY single loads for
// the x halo, instead of five loads per point: the interior y-neighbours come
// from its own registers.  Results are identical to the single-point kernels.
template <typename T>
struct Vec2;
template <>
struct Vec2<double> { using type = double2; };
template <>
struct Vec2<float> { using type = float2; };

template <typename T>
__device__ __forceinline__ void ld2(const T* __restrict__ p, T& a, T& b) {
  const typename Vec2<T>::type v = *reinterpret_cast<const typename Vec2<T>::type*>(p);
  a = v.x;
  b = v.y;
}
template <typename T>
__device__ __forceinline__ void st2(T* __restrict__ p, T a, T b) {
  typename Vec2<T>::type v;
  v.x = a;
  v.y = b;
  *reinterpret_cast<typename Vec2<T>::type*>(p) = v;
}

// Global accesses through a wave-uniform base address plus a 32-bit
// per-lane byte offset.  The base is moved to scalar registers with
// readfirstlane (every lane of the wave holds the same value), so the loads
// take the scalar-base form: one 32-bit offset register per access pattern
// instead of a 64-bit address per load, which keeps the unrolled multi-plane
// stencil kernels at two or more waves per SIMD.  Callers guarantee that the
// pointer is the same on every active lane and that byte offsets fit in 32 bits
// (a plane of at most 2^32 bytes).
typedef const __attribute__((address_space(1))) char* gcptr;
typedef __attribute__((address_space(1))) char* gptr;
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v));
  const unsigned hi = __builtin_amdgcn_readfirstlane(static_cast<unsigned>(v >> 32));
  return (static_cast<unsigned long long>(hi) << 32) | lo;
}
__device__ __forceinline__ gcptr ubase(const void* p) {
  return (gcptr)uniform_u64(reinterpret_cast<unsigned long long>(p));
}
__device__ __forceinline__ gptr ubase_w(void* p) {
  return (gptr)uniform_u64(reinterpret_cast<unsigned long long>(p));
}
template <typename T>
__device__ __forceinline__ T ldo(gcptr b, unsigned o) {
  return *(const __attribute__((address_space(1))) T*)(b + o);
}
template <typename T>
__device__ __forceinline__ void ld2o(gcptr b, unsigned o, T& x, T& y) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 v = *(const __attribute__((address_space(1))) v2*)(b + o);
  x = v.x;
  y = v.y;
}
template <typename T>
__device__ __forceinline__ void st2o(gptr b, unsigned o, T x, T y) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = x;
  v.y = y;
  *(__attribute__((address_space(1))) v2*)(b + o) = v;
}
// The same with a non-temporal (streaming) hint: the stencil kernels' outputs
// are read again only by the next kernel, after the whole vector is written.
template <typename T>
__device__ __forceinline__ void st2o_nt(gptr b, unsigned o, T x, T y) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  v2 v;
  v.x = x;
  v.y = y;
  __builtin_nontemporal_store(v, (__attribute__((address_space(1))) v2*)(b + o));
}

// Lane exchanges inside a wave (DPP wavefront shifts): lane l receives the
// value of lane l - 1 (from_below) or lane l + 1 (from_above); a lane
// without a source lane receives 0.  Values move unchanged.  The whole wave
// must reach them (never inside a divergent branch).
__device__ __forceinline__ int dpp_from_below(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xf, 0xf, false);  // wave_shr:1
}
__device__ __forceinline__ int dpp_from_above(int v) {
  return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xf, 0xf, false);  // wave_shl:1
}
__device__ __forceinline__ float lane_from_below(float v) {
  return __int_as_float(dpp_from_below(__float_as_int(v)));
}
__device__ __forceinline__ float lane_from_above(float v) {
  return __int_as_float(dpp_from_above(__float_as_int(v)));
}
__device__ __forceinline__ double lane_from_below(double v) {
  const unsigned long long x = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(dpp_from_below(static_cast<int>(x)));
  const unsigned hi = static_cast<unsigned>(dpp_from_below(static_cast<int>(x >> 32)));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}
__device__ __forceinline__ double lane_from_above(double v) {
  const unsigned long long x = static_cast<unsigned long long>(__double_as_longlong(v));
  const unsigned lo = static_cast<unsigned>(dpp_from_above(static_cast<int>(x)));
  const unsigned hi = static_cast<unsigned>(dpp_from_above(static_cast<int>(x >> 32)));
  return __longlong_as_double(static_cast<long long>((static_cast<unsigned long long>(hi) << 32) | lo));
}

// Which x neighbours of a thread's block the adjacent lanes hold: xl, the
// block to the left is lane l - 1's; xr, the block to the right is lane
// l + 1's.  Callers that exchange through them guarantee that no lane has
// both false (it would need two loads).
struct LaneNbrs {
  bool xl, xr;
};

// Geometry of the 2 x BY block owned by thread t of a plane (periodic), with
// the element offsets (inside a plane) of its rows and side points.
template <int BY>
struct Blk {
  int x0, y0, xm, xp, ylo, yhi;
  unsigned orow[BY + 2];  // rows ylo, y0 .. y0 + BY - 1, yhi at column x0
  unsigned oside[BY][2];  // (y0 + j, xm) and (y0 + j, xp)
  __device__ __forceinline__ Blk(int t, int nx, int ny) {
    const int hx = nx >> 1;
    x0 = (t % hx) * 2;
    y0 = (t / hx) * BY;
    xm = x0 > 0 ? x0 - 1 : nx - 1;
    xp = x0 + 2 < nx ? x0 + 2 : 0;
    ylo = y0 > 0 ? y0 - 1 : ny - 1;
    yhi = y0 + BY < ny ? y0 + BY : 0;
    orow[0] = static_cast<unsigned>(ylo * nx + x0);
    orow[BY + 1] = static_cast<unsigned>(yhi * nx + x0);
#pragma unroll
    for (int j = 0; j < BY; ++j) {
      orow[j + 1] = static_cast<unsigned>((y0 + j) * nx + x0);
      oside[j][0] = static_cast<unsigned>((y0 + j) * nx + xm);
      oside[j][1] = static_cast<unsigned>((y0 + j) * nx + xp);
    }
  }
  // plane offset of block point k (k = j * 2 + i)
  __device__ __forceinline__ int q(int k, int nx) const { return (y0 + (k >> 1)) * nx + x0 + (k & 1); }
};

// Lane neighbours when thread t owns block t (consecutive lanes hold
// consecutive blocks of a row): the left block is lane l - 1's unless l is
// the wave's first lane or the block starts its row, the right block lane
// l + 1's unless l is the last lane or the block ends its row.  Lanes past
// the plane's last block are never a source (that block ends its row).  A
// row of nx / 2 blocks with nx a multiple of 4 never both starts and ends on
// one lane's block at a wave boundary, so no lane lacks both neighbours.
template <int BY>
__device__ __forceinline__ LaneNbrs lane_nbrs(const Blk<BY>& b, int nx) {
  const int lane = threadIdx.x & 63;
  return LaneNbrs{lane > 0 && b.x0 > 0, lane < 63 && b.x0 + 2 < nx};
}

// The block's own rows (x0, x0 + 1 of rows y0 .. y0 + BY - 1), all M nodes.
template <int M, typename T, int BY>
__device__ __forceinline__ void load_rows(const T* __restrict__ U, size_t base, int P,
                                          const Blk<BY>& b, T own[M][BY][2]) {
  constexpr unsigned E = sizeof(T);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const gcptr Um = ubase(U + base + (size_t)m * P);
#pragma unroll
    for (int j = 0; j < BY; ++j) ld2o(Um, b.orow[j + 1] * E, own[m][j][0], own[m][j][1]);
  }
}

// Values and scaled 5-point Laplacians of the block's points, all M nodes,
// from the block's own rows (already loaded) and its neighbours.
template <int M, typename T, int BY, bool TWOD>
__device__ __forceinline__ void blk_from_rows(const T* __restrict__ U, size_t base, int P,
                                              const Blk<BY>& b, T cx, T cy, const T own[M][BY][2],
                                              T u[2 * BY][M], T lap[2 * BY][M]) {
  constexpr unsigned E = sizeof(T);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const gcptr Um = ubase(U + base + (size_t)m * P);
    T rw[BY + 2][2];
#pragma unroll
    for (int j = 0; j < BY; ++j) {
      rw[j + 1][0] = own[m][j][0];
      rw[j + 1][1] = own[m][j][1];
    }
    if (TWOD) {
      ld2o(Um, b.orow[0] * E, rw[0][0], rw[0][1]);
      ld2o(Um, b.orow[BY + 1] * E, rw[BY + 1][0], rw[BY + 1][1]);
    }
#pragma unroll
    for (int j = 0; j < BY; ++j) {
      const T l = ldo<T>(Um, b.oside[j][0] * E), r = ldo<T>(Um, b.oside[j][1] * E);
      const T c0 = rw[j + 1][0], c1 = rw[j + 1][1];
      T l0 = cx * (l + c1 - c0 - c0);
      T l1 = cx * (c0 + r - c1 - c1);
      if (TWOD) {
        l0 += cy * (rw[j][0] + rw[j + 2][0] - c0 - c0);
        l1 += cy * (rw[j][1] + rw[j + 2][1] - c1 - c1);
      }
      u[2 * j][m] = c0;
      u[2 * j + 1][m] = c1;
      lap[2 * j][m] = l0;
      lap[2 * j + 1][m] = l1;
    }
  }
}

// Values and scaled 5-point Laplacians of the block's points, all M nodes.
template <int M, typename T, int BY, bool TWOD>
__device__ __forceinline__ void load_blk(const T* __restrict__ U, size_t base, int P, int nx,
                                         const Blk<BY>& b, T cx, T cy, T u[2 * BY][M],
                                         T lap[2 * BY][M]) {
  T own[M][BY][2];
  load_rows<M, T, BY>(U, base, P, b, own);
  blk_from_rows<M, T, BY, TWOD>(U, base, P, b, cx, cy, own, u, lap);
}

// Loads an M-node field (f or coef) on the block's own points.
template <int M, typename T, int BY>
__device__ __forceinline__ void load_own(const T* __restrict__ F, size_t base, int P, int nx,
                                         const Blk<BY>& b, T v[2 * BY][M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const gcptr Fm = ubase(F + base + (size_t)m * P);
#pragma unroll
    for (int j = 0; j < BY; ++j) ld2o(Fm, b.orow[j + 1] * sizeof(T), v[2 * j][m], v[2 * j + 1][m]);
  }
}

template <int M, typename T, int BY>
__device__ __forceinline__ void store_own(T* __restrict__ F, size_t base, int P, int nx,
                                          const Blk<BY>& b, const T v[2 * BY][M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const gptr Fm = ubase_w(F + base + (size_t)m * P);
#pragma unroll
    for (int j = 0; j < BY; ++j) st2o_nt(Fm, b.orow[j + 1] * sizeof(T), v[2 * j][m], v[2 * j + 1][m]);
  }
}

// Coupling value entering the run at slab n0 for every block point (nodes
// with a zero coupling weight are not read).
template <int M, typename T, int BY>
__device__ __forceinline__ void run_prev(const Consts<M, T>& c, const SweepPtrs<T>& a, int n0, int P,
                                         int nx, const Blk<BY>& b, T prev[2 * BY]) {
#pragma unroll
  for (int k = 0; k < 2 * BY; ++k) prev[k] = T(0);
  if (n0 == 0) {
    if (a.u0) {
#pragma unroll
      for (int j = 0; j < BY; ++j) {
        const double* q = a.u0 + (b.y0 + j) * nx + b.x0;
        prev[2 * j] = (T)q[0];
        prev[2 * j + 1] = (T)q[1];
      }
    }
  } else if (a.U) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (c.cout[m] == T(0)) continue;
      const gcptr Um = ubase(a.U + (size_t)((n0 - 1) * M + m) * P);
#pragma unroll
      for (int j = 0; j < BY; ++j) {
        T v0, v1;
        ld2o(Um, b.orow[j + 1] * sizeof(T), v0, v1);
        prev[2 * j] += c.cout[m] * v0;
        prev[2 * j + 1] += c.cout[m] * v1;
      }
    }
  }
}

// r = f - [K u + db (react - lap) - cin prev] with preloaded f and coef.
template <int M, typename T, int REACT>
__device__ __forceinline__ void resid_vals(const Consts<M, T>& c, const T u[M], const T lap[M],
                                           const T fv[M], const T cv[M], T prev, T r[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T au = T(0);
#pragma unroll
    for (int j = 0; j < M; ++j) au += c.K[i][j] * u[j];
    T react;
    if (REACT == REACT_CONST) react = c.lam * u[i];
    else if (REACT == REACT_COEF) react = cv[i] * u[i];
    else react = c.gamma * (u[i] * u[i] * u[i] - u[i]);
    au += c.db[i] * (react - lap[i]);
    au -= c.cin[i] * prev;
    r[i] = fv[i] - au;
  }
}

// One point's smoothing update: d = D^{-1} r (block solve with the point's
// reaction coefficient for REACT_COEF), returning cout . d.
template <int M, typename T, int REACT>
__device__ __forceinline__ T point_correction(const Consts<M, T>& c, T dg, const T cv[M], const T r[M],
                                              T d[M]) {
  if (REACT == REACT_COEF) {
#pragma unroll
    for (int i = 0; i < M; ++i) d[i] = r[i];
    point_block_solve<M, T>(c, dg, cv, d);
  } else {
#pragma unroll
    for (int i = 0; i < M; ++i) {
      T sm = T(0);
#pragma unroll
      for (int j = 0; j < M; ++j) sm += c.Bi[i][j] * r[j];
      d[i] = sm;
    }
  }
  T nd = T(0);
#pragma unroll
  for (int i = 0; i < M; ++i) nd += c.cout[i] * d[i];
  return nd;
}

// resid_vals in two steps for a coupling value known only later:
// au = K u + db (react - lap), then r = f - (au - cin prev).
template <int M, typename T, int REACT>
__device__ __forceinline__ void resid_partial(const Consts<M, T>& c, const T u[M], const T lap[M],
                                              const T cv[M], T au[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = T(0);
#pragma unroll
    for (int j = 0; j < M; ++j) s += c.K[i][j] * u[j];
    T react;
    if (REACT == REACT_CONST) react = c.lam * u[i];
    else if (REACT == REACT_COEF) react = cv[i] * u[i];
    else react = c.gamma * (u[i] * u[i] * u[i] - u[i]);
    s += c.db[i] * (react - lap[i]);
    au[i] = s;
  }
}
template <int M, typename T>
__device__ __forceinline__ void resid_finish(const Consts<M, T>& c, const T au[M], const T fv[M], T prev,
                                             T r[M]) {
#pragma unroll
  for (int i = 0; i < M; ++i) {
    T s = au[i];
    s -= c.cin[i] * prev;
    r[i] = fv[i] - s;
  }
}

// Smoother (same mathematics as k_smooth) on 2 x BY blocks.
template <int M, typename T, int REACT, int BY, bool TWOD>
__device__ __forceinline__ void smooth_blk_body(const OpParams& p, const SweepPtrs<T>& a, int S,
                                                int tile, int n0, int pslot) {
  constexpr int NP = 2 * BY;
  const int nx = p.nx, P = nx * p.ny;
  const int t = tile * kBlock + threadIdx.x;
  double ssq = 0.0;
  if (t < (nx >> 1) * (p.ny / BY) && n0 < p.N) {
    const int n1 = min(n0 + S, p.N);
    const Consts<M, T> c(p);
    const Blk<BY> b(t, nx, p.ny);
    const T dg = T(2) * c.cx + (TWOD ? T(2) * c.cy : T(0));
    T* __restrict__ out = static_cast<T*>(a.out);
    T prev[NP], dprev[NP];
    run_prev<M, T, BY>(c, a, n0, P, nx, b, prev);
#pragma unroll
    for (int k = 0; k < NP; ++k) dprev[k] = T(0);
    for (int n = n0; n < n1; ++n) {
      const size_t base = (size_t)n * M * P;
      T u[NP][M], lap[NP][M], fv[NP][M], cv[NP][M], o[NP][M];
      if (a.U) {
        load_blk<M, T, BY, TWOD>(a.U, base, P, nx, b, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) u[k][m] = lap[k][m] = T(0);
      }
      if (a.f) {
        load_own<M, T, BY>(a.f, base, P, nx, b, fv);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) fv[k][m] = T(0);
      }
      if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        T r[M], d[M];
        resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], r);
        if (a.part) ssq_add<M, T>(p, r, ssq);
        if (n > n0) {
#pragma unroll
          for (int i = 0; i < M; ++i) r[i] += c.cin[i] * dprev[k];
        }
        if (REACT == REACT_COEF) {
#pragma unroll
          for (int i = 0; i < M; ++i) d[i] = r[i];
          point_block_solve<M, T>(c, dg, cv[k], d);
        } else {
#pragma unroll
          for (int i = 0; i < M; ++i) {
            T sm = T(0);
#pragma unroll
            for (int j = 0; j < M; ++j) sm += c.Bi[i][j] * r[j];
            d[i] = sm;
          }
        }
        T np = T(0), nd = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          o[k][i] = u[k][i] + c.omega * d[i];
          np += c.cout[i] * u[k][i];
          nd += c.cout[i] * d[i];
        }
        prev[k] = np;
        dprev[k] = nd;
      }
      store_own<M, T, BY>(out, base, P, nx, b, o);
    }
  }
  if (a.part) {
    const double tt = block_sum(ssq);
    if (threadIdx.x == 0) a.part[pslot] = tt;
  }
}

template <int M, typename T, int REACT, int BY, bool TWOD>
__global__ __launch_bounds__(kBlock) void k_smooth_blk(const OpParams p, const SweepPtrs<T> a, int S,
                                                       int tiles, int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  smooth_blk_body<M, T, REACT, BY, TWOD>(p, a, S, lb % tiles, (lb / tiles) * S, lb);
}

// Residual (optionally stored as TO) with per-block partial sums of r^2.
template <int M, typename T, typename TO, int REACT, int BY, bool TWOD>
__device__ __forceinline__ void residual_blk_body(const OpParams& p, const SweepPtrs<T>& a, int S,
                                                  int tile, int n0, int pslot) {
  constexpr int NP = 2 * BY;
  const int nx = p.nx, P = nx * p.ny;
  const int t = tile * kBlock + threadIdx.x;
  double ssq = 0.0;
  if (t < (nx >> 1) * (p.ny / BY) && n0 < p.N) {
    const int n1 = min(n0 + S, p.N);
    const Consts<M, T> c(p);
    const Blk<BY> b(t, nx, p.ny);
    TO* __restrict__ out = static_cast<TO*>(a.out);
    T prev[NP];
    run_prev<M, T, BY>(c, a, n0, P, nx, b, prev);
    for (int n = n0; n < n1; ++n) {
      const size_t base = (size_t)n * M * P;
      T u[NP][M], lap[NP][M], fv[NP][M], cv[NP][M];
      TO o[NP][M];
      if (a.U) {
        load_blk<M, T, BY, TWOD>(a.U, base, P, nx, b, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) u[k][m] = lap[k][m] = T(0);
      }
      if (a.f) {
        load_own<M, T, BY>(a.f, base, P, nx, b, fv);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) fv[k][m] = T(0);
      }
      if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        T r[M];
        resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], r);
        T np = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          o[k][i] = (TO)r[i];
          np += c.cout[i] * u[k][i];
        }
        ssq_add<M, T>(p, r, ssq);
        prev[k] = np;
      }
      if (out) store_own<M, TO, BY>(out, base, P, nx, b, o);
    }
  }
  if (a.part) {
    const double tt = block_sum(ssq);
    if (threadIdx.x == 0) a.part[pslot] = tt;
  }
}

template <int M, typename T, typename TO, int REACT, int BY, bool TWOD>
__global__ __launch_bounds__(kBlock) void k_residual_blk(const OpParams p, const SweepPtrs<T> a, int S,
                                                         int tiles, int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  residual_blk_body<M, T, TO, REACT, BY, TWOD>(p, a, S, lb % tiles, (lb / tiles) * S, lb);
}

// Values and scaled Laplacians of U' = U + e on the block's points (U in
// FP64, the correction e in FP32, e may be null), all M nodes.  U' is formed
// with the same FP64 additions as a stored update would use.
template <int M, int BY, bool TWOD>
__device__ __forceinline__ void load_blk_sum(const double* __restrict__ U, const float* __restrict__ e,
                                             size_t base, int P, const Blk<BY>& b, double cx, double cy,
                                             double u[2 * BY][M], double lap[2 * BY][M]) {
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const gcptr Um = ubase(U + base + (size_t)m * P);
    const gcptr Em = e ? ubase(e + base + (size_t)m * P) : nullptr;
    double rw[BY + 2][2];
#pragma unroll
    for (int j = 0; j < BY + 2; ++j) {
      if (!TWOD && j != 1) continue;
      ld2o(Um, b.orow[j] * 8u, rw[j][0], rw[j][1]);
      if (Em) {
        float e0, e1;
        ld2o(Em, b.orow[j] * 4u, e0, e1);
        rw[j][0] = rw[j][0] + (double)e0;
        rw[j][1] = rw[j][1] + (double)e1;
      }
    }
#pragma unroll
    for (int j = 0; j < BY; ++j) {
      double l = ldo<double>(Um, b.oside[j][0] * 8u), r = ldo<double>(Um, b.oside[j][1] * 8u);
      if (Em) {
        l = l + (double)ldo<float>(Em, b.oside[j][0] * 4u);
        r = r + (double)ldo<float>(Em, b.oside[j][1] * 4u);
      }
      const double c0 = rw[j + 1][0], c1 = rw[j + 1][1];
      double l0 = cx * (l + c1 - c0 - c0);
      double l1 = cx * (c0 + r - c1 - c1);
      if (TWOD) {
        l0 += cy * (rw[j][0] + rw[j + 2][0] - c0 - c0);
        l1 += cy * (rw[j][1] + rw[j + 2][1] - c1 - c1);
      }
      u[2 * j][m] = c0;
      u[2 * j + 1][m] = c1;
      lap[2 * j][m] = l0;
      lap[2 * j + 1][m] = l1;
    }
  }
}

// One iterative-refinement step of the mixed-precision solve, fused into a
// single sweep over the finest level (2 x BY blocks, runs of S slabs = one
// smoother chunk):
//   U' = U + e                 (FP64 iterate plus FP32 correction, e may be null)
//   r  = f - A U'              (FP64, per-block partial sums of r^2 in a.part)
//   a.out <- U' (FP64, if a.out is set), r32 <- (float) r  (the next correction equation's
//   right-hand side), and with e1 set that equation's first smoothing sweep
//   from a zero iterate, in FP32: e1 = omega D^{-1} (r32 + cin (x) cout . d_prev).
// The results equal those of the separate update, FP64 residual and FP32
// smoothing kernels, operation for operation.
template <int M, int REACT, int BY, bool TWOD>
__device__ __forceinline__ void refine_blk_body(const OpParams& p, const SweepPtrs<double>& a,
                                                const float* __restrict__ e, float* __restrict__ r32,
                                                float* __restrict__ e1, const float* __restrict__ coef32,
                                                int S, int tile, int n0, int pslot) {
  constexpr int NP = 2 * BY;
  const int nx = p.nx, P = nx * p.ny;
  const int t = tile * kBlock + threadIdx.x;
  double ssq = 0.0;
  if (t < (nx >> 1) * (p.ny / BY) && n0 < p.N) {
    const int n1 = min(n0 + S, p.N);
    const Consts<M, double> c(p);
    const Blk<BY> b(t, nx, p.ny);
    double prev[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) prev[k] = 0.0;
    if (n0 == 0) {
      if (a.u0) {
#pragma unroll
        for (int j = 0; j < BY; ++j) {
          const double* q = a.u0 + (b.y0 + j) * nx + b.x0;
          prev[2 * j] = q[0];
          prev[2 * j + 1] = q[1];
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        if (c.cout[m] == 0.0) continue;
        const size_t off = (size_t)((n0 - 1) * M + m) * P;
        const gcptr Um = ubase(a.U + off);
        const gcptr Em = e ? ubase(e + off) : nullptr;
#pragma unroll
        for (int j = 0; j < BY; ++j) {
          double v0, v1;
          ld2o(Um, b.orow[j + 1] * 8u, v0, v1);
          if (Em) {
            float e0, e1v;
            ld2o(Em, b.orow[j + 1] * 4u, e0, e1v);
            v0 = v0 + (double)e0;
            v1 = v1 + (double)e1v;
          }
          prev[2 * j] += c.cout[m] * v0;
          prev[2 * j + 1] += c.cout[m] * v1;
        }
      }
    }
    float dprev[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) dprev[k] = 0.0f;
    for (int n = n0; n < n1; ++n) {
      const size_t base = (size_t)n * M * P;
      double u[NP][M], lap[NP][M], fv[NP][M], cv[NP][M];
      float rr[NP][M];
      load_blk_sum<M, BY, TWOD>(a.U, e, base, P, b, c.cx, c.cy, u, lap);
      if (a.f) {
        load_own<M, double, BY>(a.f, base, P, nx, b, fv);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) fv[k][m] = 0.0;
      }
      if (REACT == REACT_COEF) load_own<M, double, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        double r[M];
        resid_vals<M, double, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], r);
        double np = 0.0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
          rr[k][i] = (float)r[i];
          np += c.cout[i] * u[k][i];
        }
        ssq_add<M, double>(p, r, ssq);
        prev[k] = np;
      }
      if (a.out) store_own<M, double, BY>(static_cast<double*>(a.out), base, P, nx, b, u);
      store_own<M, float, BY>(r32, base, P, nx, b, rr);
      if (e1) {
        const Consts<M, float> c32(p);
        const float dg = 2.0f * c32.cx + (TWOD ? 2.0f * c32.cy : 0.0f);
        float cv32[NP][M], o[NP][M];
        if (REACT == REACT_COEF) load_own<M, float, BY>(coef32, base, P, nx, b, cv32);
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          float r[M], d[M];
#pragma unroll
          for (int i = 0; i < M; ++i) r[i] = rr[k][i];
          if (n > n0) {
#pragma unroll
            for (int i = 0; i < M; ++i) r[i] += c32.cin[i] * dprev[k];
          }
          dprev[k] = point_correction<M, float, REACT>(c32, dg, cv32[k], r, d);
#pragma unroll
          for (int i = 0; i < M; ++i) o[k][i] = c32.omega * d[i];
        }
        store_own<M, float, BY>(e1, base, P, nx, b, o);
      }
    }
  }
  if (a.part) {
    const double tt = block_sum(ssq);
    if (threadIdx.x == 0) a.part[pslot] = tt;
  }
}

template <int M, int REACT, int BY, bool TWOD>
__global__ __launch_bounds__(kBlock) void k_refine_blk(const OpParams p, const SweepPtrs<double> a,
                                                       const float* __restrict__ e, float* __restrict__ r32,
                                                       float* __restrict__ e1,
                                                       const float* __restrict__ coef32, int S, int tiles,
                                                       int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  refine_blk_body<M, REACT, BY, TWOD>(p, a, e, r32, e1, coef32, S, lb % tiles, (lb / tiles) * S, lb);
}

// Fused residual + restriction on 2 x BY blocks with an LDS tile.  A
// workgroup owns TCX x TCY coarse points; its 256 threads own the 2 x BY
// fine blocks whose lower-left point is fine (2X, 2Y), so the fine tile is
// (2 TCX) x (BY TCY) owned points plus one halo column (fine x = 2 X0 - 1)
// and, in 2D, one halo row (fine y = 2 Y0 - 1); the halo residuals are
// computed by single-point work items.  Space coarsening only (the time
// stencil, if any, is applied in registers as in k_restrict_lds).
//
// With ZS the kernel also does the coarse level's first smoothing sweep from
// a zero iterate (U_c = omega D_c^{-1} f_c along the coarse chunks of cs
// slabs, which the run [J0, J1) contains whole) and writes it to uc.
template <int M, typename T, int REACT, bool TM, bool TWOD, int TCX, int TCY, bool ZS>
__device__ __forceinline__ void restrict_blk_body(const OpParams& p, const SweepPtrs<T>& a, int ncx,
                                                  int ncy, int Nc, T* __restrict__ fc, int S,
                                                  int tiles_x, int tile, int J0, const OpParams& pc,
                                                  T* __restrict__ uc, const T* __restrict__ coefc,
                                                  int cs, T* lds) {
  constexpr int BY = TWOD ? 2 : 1;
  constexpr int FW = 2 * TCX + 1;
  constexpr int FH = TWOD ? 2 * TCY + 1 : 1;
  constexpr int NHALO = TWOD ? FW + FH - 1 : 1;  // halo column + halo row (corner once)
  static_assert(TCX * TCY == kBlock, "one owned fine block per thread");
  // LDS tile of fine residuals provided by the caller (one allocation per
  // kernel, M x FH x RW values): FH rows of FW = 2 TCX + 1 points, each row
  // stored as its even columns and then its odd columns (TCX + 1 slots each),
  // so that the lanes of a wave, which take every second column, touch
  // consecutive words
  constexpr int RH = TCX + 1;
  constexpr int RW = 2 * RH;
  auto rs = [lds](int i, int y, int x) -> T& { return lds[(i * FH + y) * RW + (x & 1) * RH + (x >> 1)]; };
  if (J0 >= Nc) return;
  const int J1 = min(J0 + S, Nc);
  const int X0 = (tile % tiles_x) * TCX;
  const int Y0 = TWOD ? (tile / tiles_x) * TCY : 0;
  const Consts<M, T> c(p);
  const int nx = p.nx, ny = p.ny, P = nx * ny;
  const int Pc = ncx * ncy;
  const int tx = threadIdx.x % TCX, ty = threadIdx.x / TCX;
  const int X = X0 + tx, Y = Y0 + ty;
  const bool own = X < ncx && Y < ncy;  // this thread's coarse point (and fine block) exists
  const int nlo = TM ? 2 * J0 : J0;
  const int nhi = TM ? min(2 * J1, p.N - 1) : J1 - 1;

  // owned block: fine (2X .. 2X+1) x (2Y .. 2Y+1) (1D: 2X .. 2X+1), the
  // block with plane index Y (nx / 2) + X
  const Blk<BY> b(own ? (TWOD ? Y : 0) * (nx >> 1) + X : 0, nx, ny);
  T prev[2 * BY];
#pragma unroll
  for (int k = 0; k < 2 * BY; ++k) prev[k] = T(0);
  if (own) run_prev<M, T, BY>(c, a, nlo, P, nx, b, prev);
  // halo work item of this thread (if any)
  const int hk = threadIdx.x;
  const bool hown = hk < NHALO;
  int hq = 0;
  Nbr hn{0, 0, 0, 0};
  bool hvalid = false;
  int hx = 0, hy = 0;  // LDS coordinates
  if (hown) {
    int fx, fy;
    if (hk < FH) {  // halo column, tile x = 0, tile y = hk
      hx = 0; hy = hk;
      fx = 2 * X0 - 1;
      fy = TWOD ? 2 * Y0 - 1 + hk : 0;
    } else {        // halo row, tile y = 0, tile x = hk - FH + 1
      hx = hk - FH + 1; hy = 0;
      fx = 2 * X0 - 1 + hx;
      fy = 2 * Y0 - 1;
    }
    if (fx < 0) fx += nx;
    if (fy < 0) fy += ny;
    // only needed if a coarse point of this tile uses it
    const int cxn = min(TCX, ncx - X0), cyn = TWOD ? min(TCY, ncy - Y0) : 1;
    hvalid = hx <= 2 * cxn && hy <= (TWOD ? 2 * cyn : 0) && fx < nx && fy < ny;
    if (hvalid) {
      hq = fy * nx + fx;
      hn = neighbours(fx, fy, nx, ny, 0);
    }
  }
  T hprev = T(0);
  if (hvalid) {
    if (nlo == 0) {
      if (a.u0) hprev = (T)a.u0[hq];
    } else if (a.U) {
      const size_t bb = (size_t)(nlo - 1) * M * P;
#pragma unroll
      for (int j = 0; j < M; ++j) hprev += c.cout[j] * a.U[bb + (size_t)j * P + hq];
    }
  }
  T acc[M];
#pragma unroll
  for (int i = 0; i < M; ++i) acc[i] = T(0);
  T zdprev = T(0);
  const int qc = Y * ncx + X;
  for (int n = nlo; n <= nhi; ++n) {
    const size_t base = (size_t)n * M * P;
    if (own) {
      T u[2 * BY][M], lap[2 * BY][M], fv[2 * BY][M], cv[2 * BY][M];
      if (a.U) {
        load_blk<M, T, BY, TWOD>(a.U, base, P, nx, b, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int k = 0; k < 2 * BY; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) u[k][m] = lap[k][m] = T(0);
      }
      if (a.f) {
        load_own<M, T, BY>(a.f, base, P, nx, b, fv);
      } else {
#pragma unroll
        for (int k = 0; k < 2 * BY; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) fv[k][m] = T(0);
      }
      if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
      for (int k = 0; k < 2 * BY; ++k) {
        T r[M];
        resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], r);
        T np = T(0);
        const int lx = 2 * tx + 1 + (k & 1), ly = TWOD ? 2 * ty + 1 + (k >> 1) : 0;
#pragma unroll
        for (int i = 0; i < M; ++i) {
          rs(i, ly, lx) = r[i];
          np += c.cout[i] * u[k][i];
        }
        prev[k] = np;
      }
    }
    if (hvalid) {
      T u[M], lap[M], r[M];
      if (a.U) {
        load_point<M, T>(a.U, base, P, hq, hn, TWOD, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) u[m] = lap[m] = T(0);
      }
      point_residual<M, T, REACT>(c, u, lap, a.coef, a.f, base, P, hq, hprev, r);
      T np = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) {
        rs(i, hy, hx) = r[i];
        np += c.cout[i] * u[i];
      }
      hprev = np;
    }
    __syncthreads();
    if (own) {
      T rc[M];
      const int cx0 = 2 * tx, cy0 = TWOD ? 2 * ty : 0;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        T sx0 = T(0.25) * rs(i, cy0, cx0) + T(0.5) * rs(i, cy0, cx0 + 1) + T(0.25) * rs(i, cy0, cx0 + 2);
        if (TWOD) {
          const T sx1 = T(0.25) * rs(i, cy0 + 1, cx0) + T(0.5) * rs(i, cy0 + 1, cx0 + 1) +
                        T(0.25) * rs(i, cy0 + 1, cx0 + 2);
          const T sx2 = T(0.25) * rs(i, cy0 + 2, cx0) + T(0.5) * rs(i, cy0 + 2, cx0 + 1) +
                        T(0.25) * rs(i, cy0 + 2, cx0 + 2);
          sx0 = T(0.25) * sx0 + T(0.5) * sx1 + T(0.25) * sx2;
        }
        rc[i] = sx0;
      }
      // complete coarse slab J: store f_c and, with ZS, one zero-guess sweep
      auto emit = [&](int J, const T* v) {
        const size_t cb = (size_t)J * M * Pc;
#pragma unroll
        for (int i = 0; i < M; ++i) __builtin_nontemporal_store(v[i], fc + cb + (size_t)i * Pc + qc);
        if (ZS) {
          const Consts<M, T> k(pc);
          T rr[M], d[M];
#pragma unroll
          for (int i = 0; i < M; ++i) rr[i] = v[i] + ((J % cs) != 0 ? k.cin[i] * zdprev : T(0));
          if (REACT == REACT_COEF) {
            T cvv[M];
#pragma unroll
            for (int i = 0; i < M; ++i) {
              cvv[i] = coefc[cb + (size_t)i * Pc + qc];
              d[i] = rr[i];
            }
            const T dgc = T(2) * k.cx + (TWOD ? T(2) * k.cy : T(0));
            point_block_solve<M, T>(k, dgc, cvv, d);
          } else {
#pragma unroll
            for (int i = 0; i < M; ++i) {
              T sm = T(0);
#pragma unroll
              for (int j = 0; j < M; ++j) sm += k.Bi[i][j] * rr[j];
              d[i] = sm;
            }
          }
          T nd = T(0);
#pragma unroll
          for (int i = 0; i < M; ++i) {
            __builtin_nontemporal_store(k.omega * d[i], uc + cb + (size_t)i * Pc + qc);
            nd += k.cout[i] * d[i];
          }
          zdprev = nd;
        }
      };
      if (!TM) {
        emit(n, rc);
      } else if (n & 1) {
        const int J = n >> 1;
#pragma unroll
        for (int i = 0; i < M; ++i) acc[i] += rc[i];
        if (J == Nc - 1) emit(J, acc);
      } else {
        const int J = n >> 1;
        if (J > J0) {
          T v[M];
#pragma unroll
          for (int i = 0; i < M; ++i) v[i] = acc[i] + T(0.5) * rc[i];
          emit(J - 1, v);
        }
#pragma unroll
        for (int i = 0; i < M; ++i) acc[i] = T(0.5) * rc[i];
      }
    }
    __syncthreads();
  }
}

template <int M, typename T, int REACT, bool TM, bool TWOD, int TCX, int TCY, bool ZS>
__global__ __launch_bounds__(kBlock) void k_restrict_blk(const OpParams p, const SweepPtrs<T> a,
                                                         int ncx, int ncy, int Nc,
                                                         T* __restrict__ fc, int S, int tiles_x,
                                                         int tiles, int nblocks, const OpParams pc,
                                                         T* __restrict__ uc,
                                                         const T* __restrict__ coefc, int cs) {
  constexpr int FW = 2 * TCX + 1;
  constexpr int FH = TWOD ? 2 * TCY + 1 : 1;
  __shared__ T rs[M * FH * 2 * (TCX + 1)];
  const int lb = xcd_remap(blockIdx.x, nblocks);
  restrict_blk_body<M, T, REACT, TM, TWOD, TCX, TCY, ZS>(p, a, ncx, ncy, Nc, fc, S, tiles_x, lb % tiles,
                                                         (lb / tiles) * S, pc, uc, coefc, cs, rs);
}

// Fused residual + time restriction (no space coarsening) on 2 x BY blocks:
// the coarse grid is the fine grid in space, coarse slab J = fine slab 2J+1
// with the [1 2 1]/2 stencil over slab end points; with ZS also the coarse
// level's first smoothing sweep from zero (as in restrict_blk_body).
template <int M, typename T, int REACT, int BY, bool TWOD, bool ZS>
__device__ __forceinline__ void restrict_t_body(const OpParams& p, const SweepPtrs<T>& a, int Nc,
                                                T* __restrict__ fc, int S, int tile, int J0,
                                                const OpParams& pc, T* __restrict__ uc,
                                                const T* __restrict__ coefc, int cs) {
  constexpr int NP = 2 * BY;
  const int nx = p.nx, P = nx * p.ny;
  const int t = tile * kBlock + threadIdx.x;
  if (t >= (nx >> 1) * (p.ny / BY) || J0 >= Nc) return;
  const int J1 = min(J0 + S, Nc);
  const Consts<M, T> c(p);
  const Blk<BY> b(t, nx, p.ny);
  const int nlo = 2 * J0, nhi = min(2 * J1, p.N - 1);
  T prev[NP];
  run_prev<M, T, BY>(c, a, nlo, P, nx, b, prev);
  T acc[NP][M];
  T zd[NP];
#pragma unroll
  for (int k = 0; k < NP; ++k) {
    zd[k] = T(0);
#pragma unroll
    for (int i = 0; i < M; ++i) acc[k][i] = T(0);
  }
  auto emit = [&](int J, T v[NP][M]) {
    const size_t cb = (size_t)J * M * P;
    store_own<M, T, BY>(fc, cb, P, nx, b, v);
    if (ZS) {
      const Consts<M, T> k(pc);
      T cvv[NP][M], o[NP][M];
      if (REACT == REACT_COEF) load_own<M, T, BY>(coefc, cb, P, nx, b, cvv);
      const T dgc = T(2) * k.cx + (TWOD ? T(2) * k.cy : T(0));
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        T d[M];
#pragma unroll
        for (int i = 0; i < M; ++i) d[i] = v[q][i] + ((J % cs) != 0 ? k.cin[i] * zd[q] : T(0));
        if (REACT == REACT_COEF) {
          point_block_solve<M, T>(k, dgc, cvv[q], d);
        } else {
          T rr[M];
#pragma unroll
          for (int i = 0; i < M; ++i) rr[i] = d[i];
#pragma unroll
          for (int i = 0; i < M; ++i) {
            T sm = T(0);
#pragma unroll
            for (int j = 0; j < M; ++j) sm += k.Bi[i][j] * rr[j];
            d[i] = sm;
          }
        }
        T nd = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          o[q][i] = k.omega * d[i];
          nd += k.cout[i] * d[i];
        }
        zd[q] = nd;
      }
      store_own<M, T, BY>(uc, cb, P, nx, b, o);
    }
  };
  for (int n = nlo; n <= nhi; ++n) {
    const size_t base = (size_t)n * M * P;
    T u[NP][M], lap[NP][M], fv[NP][M], cv[NP][M], rr[NP][M];
    if (a.U) {
      load_blk<M, T, BY, TWOD>(a.U, base, P, nx, b, c.cx, c.cy, u, lap);
    } else {
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) u[k][m] = lap[k][m] = T(0);
    }
    if (a.f) {
      load_own<M, T, BY>(a.f, base, P, nx, b, fv);
    } else {
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) fv[k][m] = T(0);
    }
    if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], rr[k]);
      T np = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) np += c.cout[i] * u[k][i];
      prev[k] = np;
    }
    if (n & 1) {
      const int J = n >> 1;
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int i = 0; i < M; ++i) acc[k][i] += rr[k][i];
      if (J == Nc - 1) emit(J, acc);
    } else {
      const int J = n >> 1;
      if (J > J0) {
        T v[NP][M];
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int i = 0; i < M; ++i) v[k][i] = acc[k][i] + T(0.5) * rr[k][i];
        emit(J - 1, v);
      }
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int i = 0; i < M; ++i) acc[k][i] = T(0.5) * rr[k][i];
    }
  }
}

template <int M, typename T, int REACT, int BY, bool TWOD, bool ZS>
__global__ __launch_bounds__(kBlock) void k_restrict_t_blk(const OpParams p, const SweepPtrs<T> a, int Nc,
                                                           T* __restrict__ fc, int S, int tiles,
                                                           int nblocks, const OpParams pc,
                                                           T* __restrict__ uc,
                                                           const T* __restrict__ coefc, int cs) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  restrict_t_body<M, T, REACT, BY, TWOD, ZS>(p, a, Nc, fc, S, lb % tiles, (lb / tiles) * S, pc, uc,
                                             coefc, cs);
}

// Slab-parallel form of restrict_t_body for small levels (latency-bound): a
// workgroup covers SL consecutive coarse slabs (one coarse smoother chunk, SL
// a power of two with kBlock / SL a multiple of the wave size) of
// kBlock / SL blocks.  The thread of coarse slab J forms the fine residuals of
// slabs 2J and 2J+1, the last slab row also of 2J+2; the coupling value of
// slab 2J-1 and the residual of slab 2J+2 come from the neighbouring slab row
// through LDS.  With ZS one thread per block then runs the coarse zero-guess
// sweep along the chunk.  Arithmetic as in restrict_t_body, operation for
// operation.  LDS: kBlock * 2BY * (M + 1) values of T, plus kBlock * 2BY * M
// for REACT_COEF.
template <int M, typename T, int REACT, int BY, bool TWOD, bool ZS>
__device__ __forceinline__ void restrict_t_sp_body(const OpParams& p, const SweepPtrs<T>& a, int Nc,
                                                   T* __restrict__ fc, int SL, int tile, int J0,
                                                   const OpParams& pc, T* __restrict__ uc,
                                                   const T* __restrict__ coefc, int cs, T* lds) {
  constexpr int NP = 2 * BY;
  const int NB = kBlock / SL;
  const int tid = threadIdx.x;
  const int sl = tid / NB, pb = tid - sl * NB;
  const int nx = p.nx, P = nx * p.ny;
  const int t = tile * NB + pb;
  const int J = J0 + sl;
  const bool blk_ok = t < (nx >> 1) * (p.ny / BY);
  const bool act = blk_ok && J < Nc;
  T (*sR)[NP][M] = reinterpret_cast<T (*)[NP][M]>(lds);
  T (*sP)[NP] = reinterpret_cast<T (*)[NP]>(lds + kBlock * NP * M);
  T (*sC)[NP][M] = reinterpret_cast<T (*)[NP][M]>(lds + kBlock * NP * (M + 1));
  const Consts<M, T> c(p);
  const Blk<BY> b(blk_ok ? t : 0, nx, p.ny);
  const int n = 2 * J;
  const bool last = J == Nc - 1;                     // no fine slab 2J+2
  const bool third = act && !last && sl == SL - 1;   // slab 2J+2 formed here
  T au0[NP][M], f0[NP][M], r1[NP][M], r2[NP][M], prev[NP];
  if (act) {
    T np0[NP];
    {
      T u[NP][M], lap[NP][M], cv[NP][M];
      const size_t base = (size_t)n * M * P;
      if (a.U) {
        load_blk<M, T, BY, TWOD>(a.U, base, P, nx, b, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) u[k][m] = lap[k][m] = T(0);
      }
      if (a.f) {
        load_own<M, T, BY>(a.f, base, P, nx, b, f0);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) f0[k][m] = T(0);
      }
      if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        resid_partial<M, T, REACT>(c, u[k], lap[k], cv[k], au0[k]);
        T np = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) np += c.cout[i] * u[k][i];
        np0[k] = np;
      }
    }
    // fine slabs 2J+1 and (last row) 2J+2, whose couplings are local
    const int nslab = third ? 2 : 1;
    for (int e = 0; e < nslab; ++e) {
      const size_t base = (size_t)(n + 1 + e) * M * P;
      T u[NP][M], lap[NP][M], fv[NP][M], cv[NP][M];
      if (a.U) {
        load_blk<M, T, BY, TWOD>(a.U, base, P, nx, b, c.cx, c.cy, u, lap);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) u[k][m] = lap[k][m] = T(0);
      }
      if (a.f) {
        load_own<M, T, BY>(a.f, base, P, nx, b, fv);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) fv[k][m] = T(0);
      }
      if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        T np = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) np += c.cout[i] * u[k][i];
        if (e == 0) {
          resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], np0[k], r1[k]);
          np0[k] = np;  // now the coupling value of slab 2J+1
        } else {
          resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], np0[k], r2[k]);
        }
      }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) sP[tid][k] = np0[k];
    if (sl == 0) run_prev<M, T, BY>(c, a, n, P, nx, b, prev);
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      if (sl > 0) prev[k] = sP[tid - NB][k];
      T r0[M];
      resid_finish<M, T>(c, au0[k], f0[k], prev[k], r0);
#pragma unroll
      for (int i = 0; i < M; ++i) sR[tid][k][i] = r0[i];
    }
  }
  __syncthreads();
  T v[NP][M];
  if (act) {
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int i = 0; i < M; ++i) {
        T acc = T(0.5) * sR[tid][k][i];
        acc += r1[k][i];
        if (!last) acc = acc + T(0.5) * (third ? r2[k][i] : sR[tid + NB][k][i]);
        v[k][i] = acc;
      }
    store_own<M, T, BY>(fc, (size_t)J * M * P, P, nx, b, v);
  }
  if (ZS) {
    __syncthreads();
    if (act) {
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int i = 0; i < M; ++i) sR[tid][k][i] = v[k][i];
      if (REACT == REACT_COEF) {
        T cvv[NP][M];
        load_own<M, T, BY>(coefc, (size_t)J * M * P, P, nx, b, cvv);
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int i = 0; i < M; ++i) sC[tid][k][i] = cvv[k][i];
      }
    }
    __syncthreads();
    const Consts<M, T> kc(pc);
    if (sl == 0 && blk_ok) {
      const T dgc = T(2) * kc.cx + (TWOD ? T(2) * kc.cy : T(0));
      T zd[NP];
#pragma unroll
      for (int k = 0; k < NP; ++k) zd[k] = T(0);
      for (int ss = 0; ss < SL && J0 + ss < Nc; ++ss) {
        const int q = ss * NB + pb;
        const bool cpl = ((J0 + ss) % cs) != 0;
#pragma unroll
        for (int k = 0; k < NP; ++k) {
          T r[M], d[M], cq[M];
#pragma unroll
          for (int i = 0; i < M; ++i) {
            r[i] = sR[q][k][i] + (cpl ? kc.cin[i] * zd[k] : T(0));
            cq[i] = REACT == REACT_COEF ? sC[q][k][i] : T(0);
          }
          zd[k] = point_correction<M, T, REACT>(kc, dgc, cq, r, d);
#pragma unroll
          for (int i = 0; i < M; ++i) sR[q][k][i] = d[i];
        }
      }
    }
    __syncthreads();
    if (act) {
      T o[NP][M];
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int i = 0; i < M; ++i) o[k][i] = kc.omega * sR[tid][k][i];
      store_own<M, T, BY>(uc, (size_t)J * M * P, P, nx, b, o);
    }
  }
}

template <int M, typename T, int REACT, int BY, bool TWOD, bool ZS>
__global__ __launch_bounds__(kBlock) void k_restrict_t_sp(const OpParams p, const SweepPtrs<T> a, int Nc,
                                                          T* __restrict__ fc, int SL, int tiles,
                                                          int nblocks, const OpParams pc,
                                                          T* __restrict__ uc,
                                                          const T* __restrict__ coefc, int cs) {
  extern __shared__ __align__(16) unsigned char smem_rt[];
  const int lb = xcd_remap(blockIdx.x, nblocks);
  restrict_t_sp_body<M, T, REACT, BY, TWOD, ZS>(p, a, Nc, fc, SL, lb % tiles, (lb / tiles) * SL, pc, uc,
                                                coefc, cs, reinterpret_cast<T*>(smem_rt));
}

// Prolongation + correction on 2 x BY fine blocks (space coarsening: the
// block of coarse point (X, Y) is fine (2X .. 2X+1) x (2Y .. 2Y+1); time
// interpolation as in k_prolong).
template <int M, typename T, bool SP, bool TM, int BY, bool TWOD>
__global__ __launch_bounds__(kBlock) void k_prolong_blk(const OpParams p, int ncx, int ncy, int Nc,
                                                        const T* __restrict__ ec,
                                                        const T* __restrict__ Uin,
                                                        T* __restrict__ Uout, int S, int tiles,
                                                        int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int tile = lb % tiles;
  const int n0 = (lb / tiles) * S;
  const int nx = p.nx, ny = p.ny, P = nx * ny;
  const int t = tile * kBlock + threadIdx.x;
  if (t >= (nx >> 1) * (ny / BY) || n0 >= p.N) return;
  const int n1 = min(n0 + S, p.N);
  const int Pc = ncx * ncy;
  const Blk<BY> b(t, nx, ny);
  // coarse points feeding the block (byte offsets)
  unsigned c00, c10, c01, c11;
  if (SP) {
    const int X = b.x0 >> 1, Y = TWOD ? (b.y0 >> 1) : 0;
    const int X1 = X + 1 < ncx ? X + 1 : 0, Y1 = TWOD ? (Y + 1 < ncy ? Y + 1 : 0) : 0;
    c00 = (Y * ncx + X) * sizeof(T); c10 = (Y * ncx + X1) * sizeof(T);
    c01 = (Y1 * ncx + X) * sizeof(T); c11 = (Y1 * ncx + X1) * sizeof(T);
  } else {
    c00 = c10 = c01 = c11 = 0;
  }
  for (int n = n0; n < n1; ++n) {
    int js[2];
    T wt[2];
    int nt;
    if (!TM) { js[0] = n; wt[0] = T(1); nt = 1; }
    else if (n & 1) { js[0] = n >> 1; wt[0] = T(1); nt = 1; }
    else {
      const int J = n >> 1;
      js[0] = J; wt[0] = T(0.5); nt = 1;
      if (J > 0) { js[1] = J - 1; wt[1] = T(0.5); nt = 2; }
    }
    const size_t base = (size_t)n * M * P;
    T v[2 * BY][M];
    if (Uin) load_own<M, T, BY>(Uin, base, P, nx, b, v);
    else {
#pragma unroll
      for (int k = 0; k < 2 * BY; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) v[k][m] = T(0);
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      T e[2 * BY];
#pragma unroll
      for (int k = 0; k < 2 * BY; ++k) e[k] = T(0);
      for (int tt = 0; tt < nt; ++tt) {
        const gcptr Ec = ubase(ec + (size_t)js[tt] * M * Pc + (size_t)m * Pc);
        if (SP) {
          const T a00 = ldo<T>(Ec, c00), a10 = ldo<T>(Ec, c10);
          e[0] += wt[tt] * a00;
          e[1] += wt[tt] * (T(0.5) * (a00 + a10));
          if (TWOD) {
            const T a01 = ldo<T>(Ec, c01), a11 = ldo<T>(Ec, c11);
            e[2] += wt[tt] * (T(0.5) * (a00 + a01));
            e[3] += wt[tt] * (T(0.25) * (a00 + a10 + a01 + a11));
          }
        } else {
          // time only: same spatial grid
          T a0, a1;
#pragma unroll
          for (int j = 0; j < BY; ++j) {
            ld2o(Ec, b.orow[j + 1] * sizeof(T), a0, a1);
            e[2 * j] += wt[tt] * a0;
            e[2 * j + 1] += wt[tt] * a1;
          }
        }
      }
#pragma unroll
      for (int k = 0; k < 2 * BY; ++k) v[k][m] += e[k];
    }
    store_own<M, T, BY>(Uout, base, P, nx, b, v);
  }
}

// Coarse neighbourhood of block b for the space prolongation: byte offsets of
// the coarse columns and rows -1, 0, +1 around coarse point (x0 / 2, y0 / 2).
template <typename T, bool SP, bool TWOD, int BY>
struct CoarseNbr {
  unsigned ocx[3] = {0, 0, 0}, ocy[3] = {0, 0, 0};
  __device__ __forceinline__ CoarseNbr(const Blk<BY>& b, int ncx, int ncy) {
    constexpr unsigned E = sizeof(T);
    if (SP) {
      const int X = b.x0 >> 1, Y = TWOD ? (b.y0 >> 1) : 0;
      ocx[0] = (X > 0 ? X - 1 : ncx - 1) * E;
      ocx[1] = X * E;
      ocx[2] = (X + 1 < ncx ? X + 1 : 0) * E;
      if (TWOD) {
        ocy[0] = (Y > 0 ? Y - 1 : ncy - 1) * ncx * E;
        ocy[1] = Y * ncx * E;
        ocy[2] = (Y + 1 < ncy ? Y + 1 : 0) * ncx * E;
      }
    }
  }
};

// Coarse correction interpolated to the 4 x (BY + 2) fine positions of
// block b (dx = -1..2, dy = -1..BY) for node m of fine slab n; only the own
// rows' dx = -1..2 and the halo rows' dx = 0..1 are used.  Space
// interpolation is linear per dimension (fine 2X = coarse X), time
// interpolation linear in slab end points (coarse slab -1 is zero).
// With XS (space prolongation) a lane loads its coarse column X and, for a
// lane at a row or wave end, the column beyond that end; column X + 1 comes
// from lane l + 1 where ln.xr (column X - 1 is needed only where !ln.xl).
template <int M, typename T, bool SP, bool TM, int BY, bool TWOD, bool XS = false>
__device__ __forceinline__ void corr_blk(const T* __restrict__ ec, int n, int m, int Pc,
                                         const Blk<BY>& b, const CoarseNbr<T, SP, TWOD, BY>& cn,
                                         T cr[BY + 2][4], LaneNbrs ln = LaneNbrs{false, false}) {
  constexpr unsigned E = sizeof(T);
  int js[2];
  T wt[2];
  int nt;
  if (!TM) { js[0] = n; wt[0] = T(1); nt = 1; }
  else if (n & 1) { js[0] = n >> 1; wt[0] = T(1); nt = 1; }
  else {
    const int J = n >> 1;
    js[0] = J; wt[0] = T(0.5); nt = 1;
    if (J > 0) { js[1] = J - 1; wt[1] = T(0.5); nt = 2; }
  }
#pragma unroll
  for (int j = 0; j < BY + 2; ++j)
#pragma unroll
    for (int i = 0; i < 4; ++i) cr[j][i] = T(0);
  for (int tt = 0; tt < nt; ++tt) {
    const gcptr Ec = ubase(ec + (size_t)js[tt] * M * Pc + (size_t)m * Pc);
    const T w = wt[tt];
    if (SP) {
      T cv[3][3];
      if (XS) {
        T ce[3];
#pragma unroll
        for (int yy = 0; yy < (TWOD ? 3 : 1); ++yy) {
          cv[yy][1] = ldo<T>(Ec, cn.ocy[yy] + cn.ocx[1]);
          ce[yy] = ldo<T>(Ec, cn.ocy[yy] + (ln.xl ? cn.ocx[2] : cn.ocx[0]));
        }
#pragma unroll
        for (int yy = 0; yy < (TWOD ? 3 : 1); ++yy) {
          const T fa = lane_from_above(cv[yy][1]);
          cv[yy][0] = ce[yy];
          cv[yy][2] = ln.xr ? fa : ce[yy];
        }
      } else {
#pragma unroll
        for (int yy = 0; yy < (TWOD ? 3 : 1); ++yy)
#pragma unroll
          for (int xx = 0; xx < 3; ++xx) cv[yy][xx] = ldo<T>(Ec, cn.ocy[yy] + cn.ocx[xx]);
      }
      // x interpolation of each coarse row at fine dx = -1, 0, 1, 2
      T rx[3][4];
#pragma unroll
      for (int yy = 0; yy < (TWOD ? 3 : 1); ++yy) {
        rx[yy][0] = T(0.5) * (cv[yy][0] + cv[yy][1]);
        rx[yy][1] = cv[yy][1];
        rx[yy][2] = T(0.5) * (cv[yy][1] + cv[yy][2]);
        rx[yy][3] = cv[yy][2];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        if (TWOD) {
          cr[0][i] += w * T(0.5) * (rx[0][i] + rx[1][i]);  // dy = -1
          cr[1][i] += w * rx[1][i];                         // dy = 0
          cr[2][i] += w * T(0.5) * (rx[1][i] + rx[2][i]);  // dy = 1
          cr[3][i] += w * rx[2][i];                         // dy = 2
        } else {
          cr[1][i] += w * rx[0][i];
        }
      }
    } else {
      // time only: the coarse grid is the fine grid
#pragma unroll
      for (int j = 0; j < BY + 2; ++j) {
        if (!TWOD && j != 1) continue;
        T v0, v1;
        ld2o(Ec, b.orow[j] * E, v0, v1);
        cr[j][1] += w * v0;
        cr[j][2] += w * v1;
        if (j >= 1 && j <= BY) {
          cr[j][0] += w * ldo<T>(Ec, b.oside[j - 1][0] * E);
          cr[j][3] += w * ldo<T>(Ec, b.oside[j - 1][1] * E);
        }
      }
    }
  }
}

// U' = U + P e_c on the own points of block b in fine slab n: node values
// and scaled 5-point Laplacians (U' is formed on the halo too, never stored).
// U may be null (zero).
// With XS the side values of U' come from the adjacent lanes where ln says
// so (each lane at a row or wave end loads its one missing side).  UM: 0
// tests U for null at every access, 1 and 2 take U as present and as null
// (zero), so that the loads of all nodes form one straight run the compiler
// issues together ahead of the lane exchanges.
template <int M, typename T, bool SP, bool TM, int BY, bool TWOD, bool XS, int UM>
__device__ __forceinline__ void prolonged_blk_u(const Consts<M, T>& c, const T* __restrict__ U,
                                                const T* __restrict__ ec, int n, int P, int Pc,
                                                const Blk<BY>& b,
                                                const CoarseNbr<T, SP, TWOD, BY>& cn,
                                                T u[2 * BY][M], T lap[2 * BY][M], LaneNbrs ln) {
  constexpr unsigned E = sizeof(T);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    T cr[BY + 2][4];
    corr_blk<M, T, SP, TM, BY, TWOD, XS && SP>(ec, n, m, Pc, b, cn, cr, ln);
    const gcptr Um = UM == 2 ? nullptr : (UM == 1 || U) ? ubase(U + (size_t)(n * M + m) * P) : nullptr;
    const bool hu = UM == 1 ? true : UM == 2 ? false : Um != nullptr;
    T rw[BY + 2][2];
#pragma unroll
    for (int j = 0; j < BY + 2; ++j) {
      if (!TWOD && j != 1) continue;
      T v0 = T(0), v1 = T(0);
      if (hu) ld2o(Um, b.orow[j] * E, v0, v1);
      rw[j][0] = v0 + cr[j][1];
      rw[j][1] = v1 + cr[j][2];
    }
    T es[BY];
    if (XS) {
#pragma unroll
      for (int j = 0; j < BY; ++j)
        es[j] = hu ? ldo<T>(Um, (ln.xl ? b.oside[j][1] : b.oside[j][0]) * E) : T(0);
    }
#pragma unroll
    for (int j = 0; j < BY; ++j) {
      const T c0 = rw[j + 1][0], c1 = rw[j + 1][1];
      T l, r;
      if (XS) {
        const T fl = lane_from_below(c1), fr = lane_from_above(c0);
        l = ln.xl ? fl : es[j] + cr[j + 1][0];
        r = ln.xr ? fr : es[j] + cr[j + 1][3];
      } else {
        l = (hu ? ldo<T>(Um, b.oside[j][0] * E) : T(0)) + cr[j + 1][0];
        r = (hu ? ldo<T>(Um, b.oside[j][1] * E) : T(0)) + cr[j + 1][3];
      }
      T l0 = c.cx * (l + c1 - c0 - c0);
      T l1 = c.cx * (c0 + r - c1 - c1);
      if (TWOD) {
        l0 += c.cy * (rw[j][0] + rw[j + 2][0] - c0 - c0);
        l1 += c.cy * (rw[j][1] + rw[j + 2][1] - c1 - c1);
      }
      u[2 * j][m] = c0;
      u[2 * j + 1][m] = c1;
      lap[2 * j][m] = l0;
      lap[2 * j + 1][m] = l1;
    }
  }
}

template <int M, typename T, bool SP, bool TM, int BY, bool TWOD, bool XS = false>
__device__ __forceinline__ void prolonged_blk(const Consts<M, T>& c, const T* __restrict__ U,
                                              const T* __restrict__ ec, int n, int P, int Pc,
                                              const Blk<BY>& b,
                                              const CoarseNbr<T, SP, TWOD, BY>& cn,
                                              T u[2 * BY][M], T lap[2 * BY][M],
                                              LaneNbrs ln = LaneNbrs{false, false}) {
  if (!XS) {
    prolonged_blk_u<M, T, SP, TM, BY, TWOD, false, 0>(c, U, ec, n, P, Pc, b, cn, u, lap, ln);
  } else if (U) {
    prolonged_blk_u<M, T, SP, TM, BY, TWOD, XS, 1>(c, U, ec, n, P, Pc, b, cn, u, lap, ln);
  } else {
    prolonged_blk_u<M, T, SP, TM, BY, TWOD, XS, 2>(c, U, ec, n, P, Pc, b, cn, u, lap, ln);
  }
}

// Coupling value cout . U'_n on the own points of block b (nodes with a zero
// weight are not read).
template <int M, typename T, bool SP, bool TM, int BY, bool TWOD>
__device__ __forceinline__ void prolonged_cout(const Consts<M, T>& c, const T* __restrict__ U,
                                               const T* __restrict__ ec, int n, int P, int Pc,
                                               const Blk<BY>& b,
                                               const CoarseNbr<T, SP, TWOD, BY>& cn,
                                               T prev[2 * BY]) {
  constexpr unsigned E = sizeof(T);
#pragma unroll
  for (int k = 0; k < 2 * BY; ++k) prev[k] = T(0);
#pragma unroll
  for (int m = 0; m < M; ++m) {
    if (c.cout[m] == T(0)) continue;
    T cr[BY + 2][4];
    corr_blk<M, T, SP, TM, BY, TWOD>(ec, n, m, Pc, b, cn, cr);
    const gcptr Um = U ? ubase(U + (size_t)(n * M + m) * P) : nullptr;
#pragma unroll
    for (int j = 0; j < BY; ++j) {
      T v0 = T(0), v1 = T(0);
      if (Um) ld2o(Um, b.orow[j + 1] * E, v0, v1);
      prev[2 * j] += c.cout[m] * (v0 + cr[j + 1][1]);
      prev[2 * j + 1] += c.cout[m] * (v1 + cr[j + 1][2]);
    }
  }
}

// Prolongation fused with the first post-smoothing sweep:
//   U' = U + P e_c,  U_out = U' + omega D^{-1} (f - A U')
// on 2 x BY blocks, each thread marching through its run of S slabs.
template <int M, typename T, int REACT, bool SP, bool TM, int BY, bool TWOD, bool XS = false>
__device__ __forceinline__ void prolong_smooth_body(const OpParams& p, const SweepPtrs<T>& a, int ncx,
                                                    int ncy, int Nc, const T* __restrict__ ec, int S,
                                                    int tile, int n0, int pslot) {
  constexpr int NP = 2 * BY;
  const int nx = p.nx, ny = p.ny, P = nx * ny;
  const int Pc = ncx * ncy;
  const int t = tile * kBlock + threadIdx.x;
  double ssq = 0.0;
  if (t < (nx >> 1) * (ny / BY) && n0 < p.N) {
    const int n1 = min(n0 + S, p.N);
    const Consts<M, T> c(p);
    const Blk<BY> b(t, nx, ny);
    const CoarseNbr<T, SP, TWOD, BY> cn(b, ncx, ncy);
    const T dg = T(2) * c.cx + (TWOD ? T(2) * c.cy : T(0));
    T* __restrict__ out = static_cast<T*>(a.out);
    T prev[NP], dprev[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) { prev[k] = T(0); dprev[k] = T(0); }
    if (n0 == 0) {
      if (a.u0) {
#pragma unroll
        for (int j = 0; j < BY; ++j) {
          const double* q = a.u0 + (b.y0 + j) * nx + b.x0;
          prev[2 * j] = (T)q[0];
          prev[2 * j + 1] = (T)q[1];
        }
      }
    } else {
      prolonged_cout<M, T, SP, TM, BY, TWOD>(c, a.U, ec, n0 - 1, P, Pc, b, cn, prev);
    }
    const LaneNbrs ln = lane_nbrs<BY>(b, nx);
    for (int n = n0; n < n1; ++n) {
      const size_t base = (size_t)n * M * P;
      T u[NP][M], lap[NP][M], fv[NP][M], cv[NP][M], o[NP][M];
      prolonged_blk<M, T, SP, TM, BY, TWOD, XS>(c, a.U, ec, n, P, Pc, b, cn, u, lap, ln);
      if (a.f) {
        load_own<M, T, BY>(a.f, base, P, nx, b, fv);
      } else {
#pragma unroll
        for (int k = 0; k < NP; ++k)
#pragma unroll
          for (int m = 0; m < M; ++m) fv[k][m] = T(0);
      }
      if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        T r[M], d[M];
        resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], r);
        if (a.part) ssq_add<M, T>(p, r, ssq);
        if (n > n0) {
#pragma unroll
          for (int i = 0; i < M; ++i) r[i] += c.cin[i] * dprev[k];
        }
        const T nd = point_correction<M, T, REACT>(c, dg, cv[k], r, d);
        T np = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          o[k][i] = u[k][i] + c.omega * d[i];
          np += c.cout[i] * u[k][i];
        }
        prev[k] = np;
        dprev[k] = nd;
      }
      store_own<M, T, BY>(out, base, P, nx, b, o);
      if constexpr (sizeof(T) == 4) {
        if (a.up64) {
          double v[NP][M];
          load_own<M, double, BY>(a.up64, base, P, nx, b, v);
#pragma unroll
          for (int k = 0; k < NP; ++k)
#pragma unroll
            for (int i = 0; i < M; ++i) v[k][i] = v[k][i] + (double)o[k][i];
          store_own<M, double, BY>(a.up64_out, base, P, nx, b, v);
        }
      }
    }
  }
  if (a.part) {
    const double tt = block_sum(ssq);
    if (threadIdx.x == 0) a.part[pslot] = tt;
  }
}

// XS: x neighbours exchanged between lanes (nx a multiple of 4).
template <int M, typename T, int REACT, bool SP, bool TM, int BY, bool TWOD, bool XS = false>
__global__ __launch_bounds__(kBlock) void k_prolong_smooth_blk(const OpParams p, const SweepPtrs<T> a,
                                                               int ncx, int ncy, int Nc,
                                                               const T* __restrict__ ec, int S,
                                                               int tiles, int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  prolong_smooth_body<M, T, REACT, SP, TM, BY, TWOD, XS>(p, a, ncx, ncy, Nc, ec, S, lb % tiles,
                                                         (lb / tiles) * S, lb);
}

// Slab-parallel form of the fused prolongation + post-smoothing for small
// levels, whose cost is latency: a workgroup covers SL consecutive slabs (one
// smoother chunk, SL a power of two) of kBlock / SL blocks, one slab per
// thread, so every slab's loads are in flight at once.  The residuals are
// formed in parallel (the coupling value of slab n - 1 comes from the thread
// below through LDS), then one thread per block runs the chunk's forward
// substitution over the M-vectors in LDS, then every thread writes its slab.
// The arithmetic is that of prolong_smooth_body, operation for operation.
// kBlock / SL must be a multiple of the wave size: each wave lies in one slab
// (its plane bases are wave-uniform).
// LDS: kBlock * 2BY * (M + 1) values of T, plus kBlock * 2BY * M for REACT_COEF.
template <int M, typename T, int REACT, bool SP, bool TM, int BY, bool TWOD>
__device__ __forceinline__ void prolong_smooth_sp_body(const OpParams& p, const SweepPtrs<T>& a,
                                                       int ncx, int ncy, const T* __restrict__ ec,
                                                       int SL, int tile, int n0, T* lds) {
  constexpr int NP = 2 * BY;
  const int NB = kBlock / SL;
  const int tid = threadIdx.x;
  const int sl = tid / NB, pb = tid - sl * NB;
  const int nx = p.nx, ny = p.ny, P = nx * ny;
  const int Pc = ncx * ncy;
  const int t = tile * NB + pb;
  const int n = n0 + sl;
  const bool blk_ok = t < (nx >> 1) * (ny / BY);
  const bool act = blk_ok && n < p.N;
  T (*sR)[NP][M] = reinterpret_cast<T (*)[NP][M]>(lds);
  T (*sP)[NP] = reinterpret_cast<T (*)[NP]>(lds + kBlock * NP * M);
  T (*sC)[NP][M] = reinterpret_cast<T (*)[NP][M]>(lds + kBlock * NP * (M + 1));
  const Consts<M, T> c(p);
  const Blk<BY> b(blk_ok ? t : 0, nx, ny);
  const CoarseNbr<T, SP, TWOD, BY> cn(b, ncx, ncy);
  const T dg = T(2) * c.cx + (TWOD ? T(2) * c.cy : T(0));
  T u[NP][M], lap[NP][M], fv[NP][M], cv[NP][M], prev[NP];
  if (act) {
    prolonged_blk<M, T, SP, TM, BY, TWOD>(c, a.U, ec, n, P, Pc, b, cn, u, lap);
    const size_t base = (size_t)n * M * P;
    if (a.f) {
      load_own<M, T, BY>(a.f, base, P, nx, b, fv);
    } else {
#pragma unroll
      for (int k = 0; k < NP; ++k)
#pragma unroll
        for (int m = 0; m < M; ++m) fv[k][m] = T(0);
    }
    if (REACT == REACT_COEF) load_own<M, T, BY>(a.coef, base, P, nx, b, cv);
    if (sl == 0) {
      if (n0 == 0) {
#pragma unroll
        for (int k = 0; k < NP; ++k) prev[k] = T(0);
        if (a.u0) {
#pragma unroll
          for (int j = 0; j < BY; ++j) {
            const double* q = a.u0 + (b.y0 + j) * nx + b.x0;
            prev[2 * j] = (T)q[0];
            prev[2 * j + 1] = (T)q[1];
          }
        }
      } else {
        prolonged_cout<M, T, SP, TM, BY, TWOD>(c, a.U, ec, n0 - 1, P, Pc, b, cn, prev);
      }
    }
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      T np = T(0);
#pragma unroll
      for (int i = 0; i < M; ++i) np += c.cout[i] * u[k][i];
      sP[tid][k] = np;
      if (REACT == REACT_COEF) {
#pragma unroll
        for (int i = 0; i < M; ++i) sC[tid][k][i] = cv[k][i];
      }
    }
  }
  __syncthreads();
  if (act) {
#pragma unroll
    for (int k = 0; k < NP; ++k) {
      if (sl > 0) prev[k] = sP[tid - NB][k];
      T r[M];
      resid_vals<M, T, REACT>(c, u[k], lap[k], fv[k], cv[k], prev[k], r);
#pragma unroll
      for (int i = 0; i < M; ++i) sR[tid][k][i] = r[i];
    }
  }
  __syncthreads();
  if (sl == 0 && blk_ok) {
    T dprev[NP];
#pragma unroll
    for (int k = 0; k < NP; ++k) dprev[k] = T(0);
    for (int ss = 0; ss < SL && n0 + ss < p.N; ++ss) {
      const int q = ss * NB + pb;
#pragma unroll
      for (int k = 0; k < NP; ++k) {
        T r[M], d[M], cq[M];
#pragma unroll
        for (int i = 0; i < M; ++i) {
          r[i] = sR[q][k][i];
          cq[i] = REACT == REACT_COEF ? sC[q][k][i] : T(0);
        }
        if (ss > 0) {
#pragma unroll
          for (int i = 0; i < M; ++i) r[i] += c.cin[i] * dprev[k];
        }
        dprev[k] = point_correction<M, T, REACT>(c, dg, cq, r, d);
#pragma unroll
        for (int i = 0; i < M; ++i) sR[q][k][i] = d[i];
      }
    }
  }
  __syncthreads();
  if (act) {
    T o[NP][M];
#pragma unroll
    for (int k = 0; k < NP; ++k)
#pragma unroll
      for (int i = 0; i < M; ++i) o[k][i] = u[k][i] + c.omega * sR[tid][k][i];
    store_own<M, T, BY>(static_cast<T*>(a.out), (size_t)n * M * P, P, nx, b, o);
  }
}

template <int M, typename T, int REACT, bool SP, bool TM, int BY, bool TWOD>
__global__ __launch_bounds__(kBlock) void k_prolong_smooth_sp(const OpParams p, const SweepPtrs<T> a,
                                                              int ncx, int ncy,
                                                              const T* __restrict__ ec, int SL,
                                                              int tiles, int nblocks) {
  extern __shared__ __align__(16) unsigned char smem_ps[];
  const int lb = xcd_remap(blockIdx.x, nblocks);
  prolong_smooth_sp_body<M, T, REACT, SP, TM, BY, TWOD>(p, a, ncx, ncy, ec, SL, lb % tiles,
                                                        (lb / tiles) * SL,
                                                        reinterpret_cast<T*>(smem_ps));
}

// ---------------------------------------------------------------------------
// Coarsest level: U_n = Ainv (f_n + cin (x) (cout . U_{n-1})) slab after slab
// in one workgroup; Ainv is the inverse of the (constant) slab matrix.
template <typename T>
__device__ __forceinline__ void coarse_solve_body(const OpParams& p, const double* __restrict__ Ainv,
                                                  const T* __restrict__ f,
                                                  const double* __restrict__ u0,
                                                  T* __restrict__ U, int nbeg_in, int nend_in);

template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve(const OpParams p, const double* __restrict__ Ainv,
                                                         const T* __restrict__ f,
                                                         const double* __restrict__ u0,
                                                         T* __restrict__ U) {
  // decoupled slabs (no time coupling): one workgroup per slab
  if (gridDim.x > 1) coarse_solve_body<T>(p, Ainv, f, u0, U, blockIdx.x, blockIdx.x + 1);
  else coarse_solve_body<T>(p, Ainv, f, u0, U, 0, p.N);
}

template <typename T>
__device__ __forceinline__ void coarse_solve_body(const OpParams& p, const double* __restrict__ Ainv,
                                                  const T* __restrict__ f,
                                                  const double* __restrict__ u0,
                                                  T* __restrict__ U, int nbeg, int nend) {
  extern __shared__ double sm[];
  __shared__ double s_cin[kMaxM], s_cout[kMaxM];
  const int P = p.nx * p.ny, M = p.M, K = M * P;
  double* v = sm;
  double* xv = sm + K;
  double* prv = xv + K;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kMaxM; ++i) { s_cin[i] = p.cin[i]; s_cout[i] = p.cout[i]; }
  }
  for (int q = threadIdx.x; q < P; q += kBlock) prv[q] = u0 ? u0[q] : 0.0;
  __syncthreads();
  for (int n = nbeg; n < nend; ++n) {
    for (int k = threadIdx.x; k < K; k += kBlock)
      v[k] = (f ? (double)f[(size_t)n * K + k] : 0.0) + s_cin[k / P] * prv[k % P];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) {
      const double* row = Ainv + (size_t)k * K;
      double s = 0.0;
      for (int j = 0; j < K; ++j) s += row[j] * v[j];
      xv[k] = s;
      U[(size_t)n * K + k] = (T)s;
    }
    __syncthreads();
    for (int q = threadIdx.x; q < P; q += kBlock) {
      double s = 0.0;
      for (int j = 0; j < M; ++j) s += s_cout[j] * xv[j * P + q];
      prv[q] = s;
    }
    __syncthreads();
  }
}

// Coarsest level with a per-DOF reaction coefficient: every slab has its own
// matrix A_n = K (x) I + diag(db) (x) (-Lap) + diag(db_i coef_{n,i}(q)), built
// in the scratch buffer, LU-factored with partial pivoting and solved, slab
// after slab, in one workgroup.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve_coef(const OpParams p, const T* __restrict__ coef,
                                                              double* __restrict__ A,
                                                              const T* __restrict__ f,
                                                              const double* __restrict__ u0,
                                                              T* __restrict__ U) {
  extern __shared__ double sm[];
  __shared__ double s_cin[kMaxM], s_cout[kMaxM], s_db[kMaxM], s_K[kMaxM * kMaxM];
  __shared__ int s_piv;
  const int nx = p.nx, ny = p.ny, P = nx * ny, M = p.M, K = M * P;
  double* v = sm;
  double* prv = sm + K;
  int* perm = reinterpret_cast<int*>(prv + P);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kMaxM; ++i) { s_cin[i] = p.cin[i]; s_cout[i] = p.cout[i]; s_db[i] = p.db[i]; }
#pragma unroll
    for (int i = 0; i < kMaxM * kMaxM; ++i) s_K[i] = p.K[i];
  }
  for (int q = threadIdx.x; q < P; q += kBlock) prv[q] = u0 ? u0[q] : 0.0;
  __syncthreads();
  for (int n = 0; n < p.N; ++n) {
    // assemble
    for (size_t e = threadIdx.x; e < (size_t)K * K; e += kBlock) {
      const int r = (int)(e / K), cI = (int)(e % K);
      const int i = r / P, q = r % P, j = cI / P, q2 = cI % P;
      double val = (q == q2) ? s_K[i * M + j] : 0.0;
      if (i == j) {
        const int x = q % nx, y = q / nx;
        double l = 0.0;  // (-Lap)[q][q2] scaled
        if (q == q2) l += 2.0 * p.cx + (ny > 1 ? 2.0 * p.cy : 0.0);
        if (q2 == y * nx + nb_lo(x, nx, p.bc)) l -= p.cx;
        if (q2 == y * nx + nb_hi(x, nx, p.bc)) l -= p.cx;
        if (ny > 1) {
          if (q2 == nb_lo(y, ny, p.bc) * nx + x) l -= p.cy;
          if (q2 == nb_hi(y, ny, p.bc) * nx + x) l -= p.cy;
        }
        if (q == q2) l += (double)coef[(size_t)n * K + r];
        val += s_db[i] * l;
      }
      A[e] = val;
    }
    for (int k = threadIdx.x; k < K; k += kBlock) {
      v[k] = (f ? (double)f[(size_t)n * K + k] : 0.0) + s_cin[k / P] * prv[k % P];
      perm[k] = k;
    }
    __syncthreads();
    // LU with partial pivoting (row swaps applied to v as well)
    for (int k = 0; k < K; ++k) {
      if (threadIdx.x == 0) {
        int pr = k;
        double best = fabs(A[(size_t)k * K + k]);
        for (int r = k + 1; r < K; ++r) {
          const double t = fabs(A[(size_t)r * K + k]);
          if (t > best) { best = t; pr = r; }
        }
        s_piv = pr;
      }
      __syncthreads();
      const int pr = s_piv;
      if (pr != k) {
        for (int j = threadIdx.x; j < K; j += kBlock) {
          const double t = A[(size_t)k * K + j];
          A[(size_t)k * K + j] = A[(size_t)pr * K + j];
          A[(size_t)pr * K + j] = t;
        }
        if (threadIdx.x == 0) {
          const double t = v[k]; v[k] = v[pr]; v[pr] = t;
        }
      }
      __syncthreads();
      const double piv = A[(size_t)k * K + k];
      for (int r = k + 1 + threadIdx.x; r < K; r += kBlock) {
        const double l = A[(size_t)r * K + k] / piv;
        A[(size_t)r * K + k] = l;
        for (int j = k + 1; j < K; ++j) A[(size_t)r * K + j] -= l * A[(size_t)k * K + j];
        v[r] -= l * v[k];
      }
      __syncthreads();
    }
    // back substitution (serial in k, parallel dot products would need more syncs)
    if (threadIdx.x == 0) {
      for (int k = K - 1; k >= 0; --k) {
        double s = v[k];
        for (int j = k + 1; j < K; ++j) s -= A[(size_t)k * K + j] * v[j];
        v[k] = s / A[(size_t)k * K + k];
      }
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += kBlock) U[(size_t)n * K + k] = (T)v[k];
    for (int q = threadIdx.x; q < P; q += kBlock) {
      double s = 0.0;
      for (int j = 0; j < M; ++j) s += s_cout[j] * v[j * P + q];
      prv[q] = s;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------




template <typename TX, typename TY>
__global__ __launch_bounds__(kBlock) void k_axpy_cast(size_t n, const TX* __restrict__ x, double alpha,
                                                      TY* __restrict__ y, int acc) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double v = alpha * (double)x[i];
    y[i] = acc ? (TY)((double)y[i] + v) : (TY)v;
  }
}

template <typename TE>
__global__ __launch_bounds__(kBlock) void k_update(size_t n, double* __restrict__ U,
                                                   const TE* __restrict__ e,
                                                   const double* __restrict__ scale) {
  const double s = scale ? scale[0] : 1.0;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    U[i] += s * (double)e[i];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_newton_coef(size_t n, const double* __restrict__ U,
                                                        double gamma, T* __restrict__ c) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) {
    const double u = U[i];
    c[i] = (T)(gamma * (3.0 * u * u - 1.0));
  }
}

// Coarse coefficient: weighted mean of the fine coefficient over the
// full-weighting neighbourhood in space and the [1 2 1] neighbourhood of
// slab end points in time (weights normalized to sum to one).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_restrict_coef(const OpParams p, int sp, int tm, int ncx, int ncy,
                                                          int Nc, const T* __restrict__ cf,
                                                          T* __restrict__ cc) {
  const int Pc = ncx * ncy;
  const size_t total = (size_t)Nc * p.M * Pc;
  const size_t stride = (size_t)gridDim.x * kBlock;
  const int nx = p.nx, ny = p.ny, P = nx * ny, M = p.M;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
    const int qc = (int)(e % Pc);
    const int i = (int)((e / Pc) % M);
    const int J = (int)(e / ((size_t)Pc * M));
    const int X = qc % ncx, Y = qc / ncx;
    int xs[3], ys[3], ns[3];
    double wx[3], wy[3], wt[3];
    int nxs = 1, nys = 1, nts = 1;
    if (sp) {
      xs[0] = nb_lo(2 * X, nx, p.bc); xs[1] = 2 * X; xs[2] = nb_hi(2 * X, nx, p.bc);
      wx[0] = 0.25; wx[1] = 0.5; wx[2] = 0.25; nxs = 3;
      if (ny > 1) {
        ys[0] = nb_lo(2 * Y, ny, p.bc); ys[1] = 2 * Y; ys[2] = nb_hi(2 * Y, ny, p.bc);
        wy[0] = 0.25; wy[1] = 0.5; wy[2] = 0.25; nys = 3;
      } else {
        ys[0] = Y; wy[0] = 1.0;
      }
    } else {
      xs[0] = X; ys[0] = Y; wx[0] = wy[0] = 1.0;
    }
    if (tm) {
      ns[0] = 2 * J; ns[1] = 2 * J + 1; wt[0] = 0.25; wt[1] = 0.5; nts = 2;
      if (2 * J + 2 < p.N) { ns[2] = 2 * J + 2; wt[2] = 0.25; nts = 3; }
    } else {
      ns[0] = J; wt[0] = 1.0;
    }
    double s = 0.0, ws = 0.0;
    for (int t = 0; t < nts; ++t)
      for (int b = 0; b < nys; ++b)
        for (int a = 0; a < nxs; ++a) {
          const double w = wt[t] * wy[b] * wx[a];
          s += w * (double)cf[((size_t)ns[t] * M + i) * P + (size_t)ys[b] * nx + xs[a]];
          ws += w;
        }
    cc[e] = (T)(s / ws);
  }
}







inline int grid_for(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}


// SDC: in-place per-point M x M transform r <- G r on [N][M][P] (G row-major).
__global__ __launch_bounds__(kBlock) void k_node_transform(double* __restrict__ r, int N, int M, int P,
                                                           const double* __restrict__ G) {
  __shared__ double g[kMaxM * kMaxM];
  if (threadIdx.x < kMaxM * kMaxM) g[threadIdx.x] = threadIdx.x < M * M ? G[threadIdx.x] : 0.0;
  __syncthreads();
  const size_t total = (size_t)N * P;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
    const size_t n = e / P, q = e % P;
    double v[kMaxM], w[kMaxM];
    for (int i = 0; i < M; ++i) v[i] = r[(n * M + i) * P + q];
    for (int i = 0; i < M; ++i) {
      double s = 0.0;
      for (int j = 0; j < M; ++j) s += g[i * M + j] * v[j];
      w[i] = s;
    }
    for (int i = 0; i < M; ++i) r[(n * M + i) * P + q] = w[i];
  }
}

// SDC: rhs[n][q] = r[n][m][q] + acc[n][q]
__global__ __launch_bounds__(kBlock) void k_sdc_gather(const double* __restrict__ r, const double* __restrict__ acc,
                                                       double* __restrict__ rhs, int N, int M, int P, int m) {
  const size_t total = (size_t)N * P;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
    const size_t n = e / P, q = e % P;
    rhs[e] = r[(n * M + m) * P + q] + acc[e];
  }
}

// SDC: U[n][m][q] += d[n][q];  acc[n][q] += w (nu Lap - lambda) d [n][q]
// (periodic or Neumann 5-point stencil on the plane of each slab).
__global__ __launch_bounds__(kBlock) void k_sdc_update(double* __restrict__ U, double* __restrict__ acc,
                                                       const double* __restrict__ d, int N, int M, int nx,
                                                       int ny, int bc, double cx, double cy, double lam,
                                                       double w, int m) {
  const int P = nx * ny;
  const size_t total = (size_t)N * P;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
    const size_t n = e / P;
    const int q = (int)(e % P);
    const int x = q % nx, y = q / nx;
    const double* D = d + n * P;
    const double c = D[q];
    double l = cx * (D[y * nx + nb_lo(x, nx, bc)] + D[y * nx + nb_hi(x, nx, bc)] - 2.0 * c);
    if (ny > 1) l += cy * (D[nb_lo(y, ny, bc) * nx + x] + D[nb_hi(y, ny, bc) * nx + x] - 2.0 * c);
    U[(n * M + m) * P + q] += c;
    acc[e] += w * (l - lam * c);
  }
}
}  // namespace
}  // namespace stmg
