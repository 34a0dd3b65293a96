// Level-0 vector kernels of the flexible GMRES driver: Gram-Schmidt passes
// with fused dot products, column sums of their partials, and the final
// combination of the preconditioned directions.  All FP64, memory bound:
// each pass streams w and the k basis vectors once.
#include "launchers.hpp"

namespace stmg {

namespace {

inline int kgrid(size_t n) {
  size_t b = (n + kBlock - 1) / kBlock;
  if (b > static_cast<size_t>(kKrylovParts)) b = kKrylovParts;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}

// KM: compile-time bound on k (accumulators live in registers).  Each thread
// takes two consecutive doubles per step (16-byte loads); an odd last element
// is taken by thread 0 of block 0.
template <int KM>
__global__ __launch_bounds__(kBlock) void k_kortho(double* __restrict__ w, const KVecs V, int k,
                                                   const KCoef s, const double* __restrict__ d,
                                                   size_t n, int dots, double* __restrict__ part) {
  __shared__ double s_coef[KM];
  __shared__ double red[kBlock / 64][KM + 1];
  const bool upd = d != nullptr;
  if (threadIdx.x < KM) {
    const int i = threadIdx.x;
    s_coef[i] = (upd && i < k) ? s.c[i] * d[i] : 0.0;
  }
  __syncthreads();
  double acc[KM + 1];
#pragma unroll
  for (int i = 0; i <= KM; ++i) acc[i] = 0.0;
  const size_t n2 = n >> 1;
  const size_t stride = static_cast<size_t>(gridDim.x) * kBlock;
  for (size_t e = static_cast<size_t>(blockIdx.x) * kBlock + threadIdx.x; e < n2; e += stride) {
    double2 x = reinterpret_cast<const double2*>(w)[e];
    double2 v[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      if (i < k) {
        v[i] = reinterpret_cast<const double2*>(V.v[i])[e];
        x.x -= s_coef[i] * v[i].x;
        x.y -= s_coef[i] * v[i].y;
      }
    }
    if (upd) reinterpret_cast<double2*>(w)[e] = x;
    if (dots) {
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (i < k) acc[i] += x.x * v[i].x + x.y * v[i].y;
    }
    acc[KM] += x.x * x.x + x.y * x.y;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const size_t e = n - 1;
    double x = w[e];
    double v[KM];
#pragma unroll
    for (int i = 0; i < KM; ++i) {
      if (i < k) {
        v[i] = V.v[i][e];
        x -= s_coef[i] * v[i];
      }
    }
    if (upd) w[e] = x;
    if (dots) {
#pragma unroll
      for (int i = 0; i < KM; ++i)
        if (i < k) acc[i] += x * v[i];
    }
    acc[KM] += x * x;
  }
  // wave sums, then one cross-wave sum per column
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i <= KM; ++i) {
    double t = acc[i];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) t += __shfl_xor(t, off, 64);
    if (lane == 0) red[wv][i] = t;
  }
  __syncthreads();
  const int nb = gridDim.x;
  const int c = threadIdx.x;
  if (c <= KM) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < kBlock / 64; ++q) t += red[q][c];
    if (c == KM) part[static_cast<size_t>(k) * nb + blockIdx.x] = t;
    else if (dots && c < k) part[static_cast<size_t>(c) * nb + blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_kreduce(const double* __restrict__ part, int nb,
                                                    double* __restrict__ out, double* mirror) {
  const int c = blockIdx.x;
  double t = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) t += part[static_cast<size_t>(c) * nb + b];
  const double r = block_sum(t);
  if (threadIdx.x == 0) {
    out[c] = r;
    if (mirror) mirror[c] = r;
  }
}

// Two consecutive doubles per thread and step (all pointers 16-byte aligned).
__global__ __launch_bounds__(kBlock) void k_kcombine2(double* __restrict__ x, const KVecs Z, int k,
                                                      const KCoef y, size_t n) {
  const size_t n2 = n >> 1;
  const size_t stride = static_cast<size_t>(gridDim.x) * kBlock;
  for (size_t e = static_cast<size_t>(blockIdx.x) * kBlock + threadIdx.x; e < n2; e += stride) {
    double2 t = reinterpret_cast<const double2*>(x)[e];
    for (int i = 0; i < k; ++i) {
      const double2 z = reinterpret_cast<const double2*>(Z.v[i])[e];
      t.x += y.c[i] * z.x;
      t.y += y.c[i] * z.y;
    }
    reinterpret_cast<double2*>(x)[e] = t;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    double t = x[n - 1];
    for (int i = 0; i < k; ++i) t += y.c[i] * Z.v[i][n - 1];
    x[n - 1] = t;
  }
}

__global__ __launch_bounds__(kBlock) void k_kcombine(double* __restrict__ x, const KVecs Z, int k,
                                                     const KCoef y, size_t n) {
  const size_t stride = static_cast<size_t>(gridDim.x) * kBlock;
  for (size_t e = static_cast<size_t>(blockIdx.x) * kBlock + threadIdx.x; e < n; e += stride) {
    double t = x[e];
    for (int i = 0; i < k; ++i) t += y.c[i] * Z.v[i][e];
    x[e] = t;
  }
}

}  // namespace

hipError_t launch_kortho(double* w, const KVecs& V, int k, const KCoef& s, const double* d, size_t n,
                         bool dots, double* part, int* nb, hipStream_t st) {
  if (k < 0 || k > kKrylovMax + 1) return hipErrorInvalidValue;
  if (reinterpret_cast<uintptr_t>(w) & 15) return hipErrorInvalidValue;
  for (int i = 0; i < k; ++i)
    if (reinterpret_cast<uintptr_t>(V.v[i]) & 15) return hipErrorInvalidValue;
  const int g = kgrid(n >> 1);
  *nb = g;
  const int df = dots ? 1 : 0;
  if (k <= 8)
    hipLaunchKernelGGL((k_kortho<8>), dim3(g), dim3(kBlock), 0, st, w, V, k, s, d, n, df, part);
  else if (k <= 16)
    hipLaunchKernelGGL((k_kortho<16>), dim3(g), dim3(kBlock), 0, st, w, V, k, s, d, n, df, part);
  else
    hipLaunchKernelGGL((k_kortho<kKrylovMax + 1>), dim3(g), dim3(kBlock), 0, st, w, V, k, s, d, n, df, part);
  return hipGetLastError();
}

hipError_t launch_kreduce(const double* part, int nb, int cols, double* out, double* mirror,
                          hipStream_t st) {
  if (cols < 1) return hipSuccess;
  hipLaunchKernelGGL(k_kreduce, dim3(cols), dim3(kBlock), 0, st, part, nb, out, mirror);
  return hipGetLastError();
}

hipError_t launch_kcombine(double* x, const KVecs& Z, int k, const KCoef& y, size_t n, hipStream_t st) {
  if (k < 1) return hipSuccess;
  if (k > kKrylovMax + 1) return hipErrorInvalidValue;
  bool aligned = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  for (int i = 0; i < k; ++i) aligned = aligned && (reinterpret_cast<uintptr_t>(Z.v[i]) & 15) == 0;
  if (aligned)
    hipLaunchKernelGGL(k_kcombine2, dim3(grid_for(n >> 1)), dim3(kBlock), 0, st, x, Z, k, y, n);
  else
    hipLaunchKernelGGL(k_kcombine, dim3(grid_for(n)), dim3(kBlock), 0, st, x, Z, k, y, n);
  return hipGetLastError();
}

}  // namespace stmg
