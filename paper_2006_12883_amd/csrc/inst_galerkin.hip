// Galerkin coarse levels (Sec. 4.2 with A_{l+1} = R A_l P): the 9-point
// residual and smoothing kernels and their launchers, for FP64 and FP32.
#include "launchers.hpp"

namespace stmg {
namespace {
// Galerkin coarse levels (periodic, 3 x 3 mass and stiffness stencils,
// entry [(dy + 1) * 3 + dx + 1] weighing u(x + dx, y + dy)).  One thread =
// one pair of points (x0, x0 + 1), x0 even, x a run of slabs: each stencil row
// of a node plane is loaded as one pair and two single values (4 columns for
// both points), and the coupling values cout . U_{n-1} at the 3 x 4 positions
// stay in registers from one slab to the next.  SMOOTH false: residual
// r = f - A U; true: one block-Jacobi sweep over the run (one smoother chunk):
// r += cin m_0 (cout . d_{n-1}) inside the chunk, d = (K m_0 + diag(db) k_0)^-1 r,
// U' = U + omega d.
template <typename T>
__device__ __forceinline__ void ld_pair(const T* __restrict__ b, T& x, T& y) {
  typedef T v2 __attribute__((ext_vector_type(2)));
  const v2 w = *reinterpret_cast<const v2*>(b);
  x = w.x;
  y = w.y;
}

template <typename T, bool TWOD>
__device__ __forceinline__ T apply9c(const T w[9], const T v[3][4], int c0) {
  T s = T(0);
#pragma unroll
  for (int k = 0; k < 9; ++k)
    if (TWOD || k / 3 == 1) s += w[k] * v[k / 3][k % 3 + c0];
  return s;
}

struct PairGeo {
  int row[3];      // fine rows y - 1, y, y + 1 (wrapped; 1D: all y)
  int xm, x0, xp;  // fine columns x0 - 1, x0, x0 + 2
};

template <typename T, bool TWOD>
__device__ __forceinline__ void load_rows(const T* __restrict__ Um, const PairGeo& g, int nx, T v[3][4]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    if (!TWOD && r != 1) {
#pragma unroll
      for (int c = 0; c < 4; ++c) v[r][c] = T(0);
      continue;
    }
    const T* b = Um + (size_t)g.row[r] * nx;
    v[r][0] = b[g.xm];
    ld_pair(b + g.x0, v[r][1], v[r][2]);
    v[r][3] = b[g.xp];
  }
}

template <int M, typename T, bool TWOD, bool SMOOTH>
__global__ __launch_bounds__(kBlock) void k_level9x2(const OpParams p, const Stencil9 st, const T* __restrict__ U,
                                                     const T* __restrict__ f, T* __restrict__ out, int S, int tiles,
                                                     int nblocks) {
  const int lb = xcd_remap(blockIdx.x, nblocks);
  const int t = (lb % tiles) * kBlock + threadIdx.x;
  const int n0 = (lb / tiles) * S;
  const int nx = p.nx, ny = p.ny, P = nx * ny, hx = nx >> 1;
  if (t >= hx * ny || n0 >= p.N) return;
  const int n1 = min(n0 + S, p.N);
  PairGeo g;
  const int y = t / hx;
  g.x0 = (t % hx) * 2;
  g.xm = g.x0 > 0 ? g.x0 - 1 : nx - 1;
  g.xp = g.x0 + 2 < nx ? g.x0 + 2 : 0;
  g.row[0] = TWOD ? (y > 0 ? y - 1 : ny - 1) : y;
  g.row[1] = y;
  g.row[2] = TWOD ? (y + 1 < ny ? y + 1 : 0) : y;
  const Consts<M, T> c(p);
  T ms[9], ks[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    ms[k] = (T)st.m[k];
    ks[k] = (T)st.k[k];
  }
  auto node_vals = [&](int n, int m, T v[3][4]) {
    if (U) load_rows<T, TWOD>(U + ((size_t)n * M + m) * P, g, nx, v);
    else {
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) v[r][q] = T(0);
    }
  };
  T prev[3][4];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int q = 0; q < 4; ++q) prev[r][q] = T(0);
  if (n0 > 0 && U) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (c.cout[m] == T(0)) continue;
      T v[3][4];
      node_vals(n0 - 1, m, v);
#pragma unroll
      for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int q = 0; q < 4; ++q) prev[r][q] += c.cout[m] * v[r][q];
    }
  }
  T dprev[2] = {T(0), T(0)};
  for (int n = n0; n < n1; ++n) {
    const size_t base = (size_t)n * M * P;
    T v[M][3][4];
#pragma unroll
    for (int m = 0; m < M; ++m) node_vals(n, m, v[m]);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      T mv[M], r[M];
#pragma unroll
      for (int m = 0; m < M; ++m) mv[m] = apply9c<T, TWOD>(ms, v[m], h);
      const T mprev = apply9c<T, TWOD>(ms, prev, h);
      const size_t q = (size_t)y * nx + g.x0 + h;
#pragma unroll
      for (int i = 0; i < M; ++i) {
        T au = T(0);
#pragma unroll
        for (int j = 0; j < M; ++j) au += c.K[i][j] * mv[j];
        au += c.db[i] * apply9c<T, TWOD>(ks, v[i], h);
        au -= c.cin[i] * mprev;
        const T fi = f ? f[base + (size_t)i * P + q] : T(0);
        r[i] = fi - au;
      }
      if (!SMOOTH) {
#pragma unroll
        for (int i = 0; i < M; ++i) out[base + (size_t)i * P + q] = r[i];
      } else {
        if (n > n0) {
#pragma unroll
          for (int i = 0; i < M; ++i) r[i] += c.cin[i] * ms[4] * dprev[h];
        }
        T d[M], nd = T(0);
#pragma unroll
        for (int i = 0; i < M; ++i) {
          T sm = T(0);
#pragma unroll
          for (int j = 0; j < M; ++j) sm += c.Bi[i][j] * r[j];
          d[i] = sm;
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
          out[base + (size_t)i * P + q] = v[i][1][1 + h] + c.omega * d[i];
          nd += c.cout[i] * d[i];
        }
        dprev[h] = nd;
      }
    }
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        T s2 = T(0);
#pragma unroll
        for (int m = 0; m < M; ++m) s2 += c.cout[m] * v[m][r][q];
        prev[r][q] = s2;
      }
  }
}

}  // namespace

// Launch shape of the pair kernels: one thread per pair, runs of S slabs.
template <typename T, bool SMOOTH>
static hipError_t launch_pairs(const OpParams& p, const Stencil9& st, const T* U, const T* f, T* out, int S,
                               hipStream_t s) {
  const int thr = (p.nx / 2) * p.ny;
  const int tiles = (thr + kBlock - 1) / kBlock;
  const int nb = tiles * ((p.N + S - 1) / S);
#define L(MM)                                                                                               \
  if (p.ny > 1)                                                                                             \
    hipLaunchKernelGGL((k_level9x2<MM, T, true, SMOOTH>), dim3(nb), dim3(kBlock), 0, s, p, st, U, f, out, S, \
                       tiles, nb);                                                                          \
  else                                                                                                      \
    hipLaunchKernelGGL((k_level9x2<MM, T, false, SMOOTH>), dim3(nb), dim3(kBlock), 0, s, p, st, U, f, out, S, \
                       tiles, nb);
  STMG_DISPATCH_M(L)
#undef L
  return hipGetLastError();
}

// Galerkin levels: residual (runs of 8 slabs) and smoothing sweep (runs of
// one chunk).  A Galerkin level is coarsened again, so its point count is
// even (hipErrorNotSupported otherwise).
template <typename T>
hipError_t launch_residual9(const OpParams& p, const Stencil9& st, const T* U, const T* f, T* out,
                            hipStream_t s) {
  if (p.nx % 2 != 0) return hipErrorNotSupported;
  return launch_pairs<T, false>(p, st, U, f, out, 8, s);
}

template <typename T>
hipError_t launch_smooth9(const OpParams& p, const Stencil9& st, const T* U, const T* f, T* out, int chunk,
                          hipStream_t s) {
  if (p.nx % 2 != 0) return hipErrorNotSupported;
  return launch_pairs<T, true>(p, st, U, f, out, chunk, s);
}

template hipError_t launch_residual9<double>(const OpParams&, const Stencil9&, const double*, const double*, double*,
                                             hipStream_t);
template hipError_t launch_residual9<float>(const OpParams&, const Stencil9&, const float*, const float*, float*,
                                            hipStream_t);
template hipError_t launch_smooth9<double>(const OpParams&, const Stencil9&, const double*, const double*, double*,
                                           int, hipStream_t);
template hipError_t launch_smooth9<float>(const OpParams&, const Stencil9&, const float*, const float*, float*, int,
                                          hipStream_t);
}  // namespace stmg
