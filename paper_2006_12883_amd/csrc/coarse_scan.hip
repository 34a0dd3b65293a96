// Coarsest level with a constant slab matrix A_s and at most kScanMaxP points
// per plane, split so that only a P-vector recurrence is sequential:
//   w_n = A_s^{-1} f_n,  g_n = (cout (x) I) w_n                  (all slabs)
//   p_{-1} = u0 (or 0),  p_n = g_n + G p_{n-1},  G = (cout (x) I) A_s^{-1} (cin (x) I)
//   U_n = w_n + H p_{n-1},  H = A_s^{-1} (cin (x) I)             (all slabs)
// which is U_n = A_s^{-1} (f_n + cin (x) p_{n-1}) with p_{n-1} = cout . U_{n-1}.
#include "launchers.hpp"

namespace stmg {

namespace {

// One thread per (slab n, point q): the M rows (m, q) of w_n and g_n[q].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cs_apply(const double* __restrict__ Ainv, const double* __restrict__ cout,
                                                     int M, int P, int N, const T* __restrict__ f, T* __restrict__ U,
                                                     double* __restrict__ g) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= static_cast<size_t>(N) * P) return;
  const int n = static_cast<int>(idx / P), q = static_cast<int>(idx % P);
  const int K = M * P;
  double gs = 0.0;
  for (int m = 0; m < M; ++m) {
    const int r = m * P + q;
    double s = 0.0;
    if (f) {
      const double* row = Ainv + static_cast<size_t>(r) * K;
      const T* fn = f + static_cast<size_t>(n) * K;
      for (int j = 0; j < K; ++j) s += row[j] * static_cast<double>(fn[j]);
    }
    U[static_cast<size_t>(n) * K + r] = static_cast<T>(s);
    gs += cout[m] * s;
  }
  g[idx] = gs;
}

// One wave: lane q keeps row q of G in registers and p_q; the vector p is
// shared through LDS each step.  pg holds g_n on entry and p_{n-1} on exit.
template <int PM>
__global__ __launch_bounds__(64) void k_cs_scan(const double* __restrict__ G, int P, int N,
                                                const double* __restrict__ u0, double* __restrict__ pg) {
  __shared__ double sp[PM];
  const int q = threadIdx.x;
  const bool on = q < P;
  double grow[PM];
#pragma unroll
  for (int j = 0; j < PM; ++j) grow[j] = (on && j < P) ? G[static_cast<size_t>(q) * P + j] : 0.0;
  double p = (on && u0) ? u0[q] : 0.0;
  for (int n = 0; n < N; ++n) {
    double g = 0.0;
    if (on) {
      g = pg[static_cast<size_t>(n) * P + q];
      pg[static_cast<size_t>(n) * P + q] = p;
    }
    if (q < PM) sp[q] = on ? p : 0.0;
    __syncthreads();
    double s = g;
#pragma unroll
    for (int j = 0; j < PM; ++j) s += grow[j] * sp[j];
    p = s;
    __syncthreads();
  }
}

// One thread per (slab n, row r): U_n[r] += sum_q' H[r][q'] p_{n-1}[q'].
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cs_finish(const double* __restrict__ H, int K, int P, int N,
                                                      const double* __restrict__ pin, T* __restrict__ U) {
  const size_t idx = static_cast<size_t>(blockIdx.x) * kBlock + threadIdx.x;
  if (idx >= static_cast<size_t>(N) * K) return;
  const int n = static_cast<int>(idx / K), r = static_cast<int>(idx % K);
  const double* hr = H + static_cast<size_t>(r) * P;
  const double* pn = pin + static_cast<size_t>(n) * P;
  double s = static_cast<double>(U[idx]);
  for (int j = 0; j < P; ++j) s += hr[j] * pn[j];
  U[idx] = static_cast<T>(s);
}

}  // namespace

template <typename T>
hipError_t launch_coarse_scan(const OpParams& p, const CoarseScan& cs, const T* f, const double* u0, T* U,
                              hipStream_t s) {
  const int P = p.nx * p.ny, M = p.M, K = M * P, N = p.N;
  if (P < 1 || P > kScanMaxP || N < 1) return hipErrorInvalidValue;
  const size_t np = static_cast<size_t>(N) * P, nk = static_cast<size_t>(N) * K;
  hipLaunchKernelGGL((k_cs_apply<T>), dim3(static_cast<unsigned>((np + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     cs.Ainv, cs.cout, M, P, N, f, U, cs.pg);
  if (P <= 16)
    hipLaunchKernelGGL((k_cs_scan<16>), dim3(1), dim3(64), 0, s, cs.G, P, N, u0, cs.pg);
  else if (P <= 32)
    hipLaunchKernelGGL((k_cs_scan<32>), dim3(1), dim3(64), 0, s, cs.G, P, N, u0, cs.pg);
  else
    hipLaunchKernelGGL((k_cs_scan<64>), dim3(1), dim3(64), 0, s, cs.G, P, N, u0, cs.pg);
  hipLaunchKernelGGL((k_cs_finish<T>), dim3(static_cast<unsigned>((nk + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     cs.H, K, P, N, cs.pg, U);
  return hipGetLastError();
}

template hipError_t launch_coarse_scan<double>(const OpParams&, const CoarseScan&, const double*, const double*,
                                               double*, hipStream_t);
template hipError_t launch_coarse_scan<float>(const OpParams&, const CoarseScan&, const float*, const double*,
                                              float*, hipStream_t);

}  // namespace stmg
