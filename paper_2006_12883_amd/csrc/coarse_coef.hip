// Coarsest level under Newton (per-point reaction coefficient).  Each slab
// has its own matrix A_n = K (x) I + diag(db) (x) (-Lap) + diag(db_i c_{n,i}(q)).
// The matrices depend only on the linearization, so they are inverted once
// per Newton step, all slabs in parallel; every V-cycle's coarsest solve is
// then the slab recurrence U_n = A_n^{-1} (f_n + cin (x) (cout . U_{n-1})),
// one matrix-vector product per slab.
#include "launchers.hpp"

namespace stmg {

namespace {

// Slab n (one workgroup): W_n = [A_n | I] (K x 2K, row-major) becomes
// [I | A_n^{-1}] by Gauss-Jordan elimination with partial pivoting (largest
// magnitude in the column, the smaller row index on ties).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_invert_coef(const OpParams p, const T* __restrict__ coef,
                                                               double* __restrict__ W) {
  extern __shared__ double fac[];  // K
  __shared__ double s_K[kMaxM * kMaxM], s_db[kMaxM];
  __shared__ int s_piv;
  const int nx = p.nx, ny = p.ny, P = nx * ny, M = p.M, K = M * P, L = 2 * K;
  const int n = blockIdx.x;
  double* A = W + static_cast<size_t>(n) * K * L;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kMaxM; ++i) s_db[i] = p.db[i];
#pragma unroll
    for (int i = 0; i < kMaxM * kMaxM; ++i) s_K[i] = p.K[i];
  }
  __syncthreads();
  for (size_t e = threadIdx.x; e < static_cast<size_t>(K) * L; e += kBlock) {
    const int r = static_cast<int>(e / L), c = static_cast<int>(e % L);
    double val;
    if (c >= K) {
      val = (c - K == r) ? 1.0 : 0.0;
    } else {
      const int i = r / P, q = r % P, j = c / P, q2 = c % P;
      val = (q == q2) ? s_K[i * M + j] : 0.0;
      if (i == j) {
        const int x = q % nx, y = q / nx;
        double l = 0.0;  // (-Lap + c)[q][q2]
        if (q == q2) l += 2.0 * p.cx + (ny > 1 ? 2.0 * p.cy : 0.0);
        if (q2 == y * nx + nb_lo(x, nx, p.bc)) l -= p.cx;
        if (q2 == y * nx + nb_hi(x, nx, p.bc)) l -= p.cx;
        if (ny > 1) {
          if (q2 == nb_lo(y, ny, p.bc) * nx + x) l -= p.cy;
          if (q2 == nb_hi(y, ny, p.bc) * nx + x) l -= p.cy;
        }
        if (q == q2) l += static_cast<double>(coef[static_cast<size_t>(n) * K + r]);
        val += s_db[i] * l;
      }
    }
    A[e] = val;
  }
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    if (threadIdx.x < 64) {
      double best = -1.0;
      int br = k;
      for (int r = k + static_cast<int>(threadIdx.x); r < K; r += 64) {
        const double t = fabs(A[static_cast<size_t>(r) * L + k]);
        if (t > best) { best = t; br = r; }
      }
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int orow = __shfl_xor(br, off, 64);
        if (ob > best || (ob == best && orow < br)) { best = ob; br = orow; }
      }
      if (threadIdx.x == 0) s_piv = br;
    }
    __syncthreads();
    const int pr = s_piv;
    if (pr != k) {
      for (int j = threadIdx.x; j < L; j += kBlock) {
        const double t = A[static_cast<size_t>(k) * L + j];
        A[static_cast<size_t>(k) * L + j] = A[static_cast<size_t>(pr) * L + j];
        A[static_cast<size_t>(pr) * L + j] = t;
      }
    }
    __syncthreads();
    const double inv = 1.0 / A[static_cast<size_t>(k) * L + k];
    for (int r = threadIdx.x; r < K; r += kBlock) fac[r] = (r == k) ? 0.0 : A[static_cast<size_t>(r) * L + k];
    __syncthreads();
    for (int j = k + threadIdx.x; j < L; j += kBlock) A[static_cast<size_t>(k) * L + j] *= inv;
    __syncthreads();
    const int w = L - k;
    for (size_t e = threadIdx.x; e < static_cast<size_t>(K) * w; e += kBlock) {
      const int r = static_cast<int>(e / w), j = k + static_cast<int>(e % w);
      if (r != k) A[static_cast<size_t>(r) * L + j] -= fac[r] * A[static_cast<size_t>(k) * L + j];
    }
    __syncthreads();
  }
}

// The slab recurrence with the stored inverses (right half of W_n).  With
// no coupling between slabs (cin = 0, no u0) every workgroup takes one slab.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_coarse_solve_slabs(const OpParams p, const double* __restrict__ W,
                                                               const T* __restrict__ f,
                                                               const double* __restrict__ u0,
                                                               T* __restrict__ U) {
  extern __shared__ double sm[];
  __shared__ double s_cin[kMaxM], s_cout[kMaxM];
  const int P = p.nx * p.ny, M = p.M, K = M * P, L = 2 * K;
  double* v = sm;
  double* xv = sm + K;
  double* prv = xv + K;
  const int nbeg = gridDim.x > 1 ? static_cast<int>(blockIdx.x) : 0;
  const int nend = gridDim.x > 1 ? nbeg + 1 : p.N;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kMaxM; ++i) { s_cin[i] = p.cin[i]; s_cout[i] = p.cout[i]; }
  }
  for (int q = threadIdx.x; q < P; q += kBlock) prv[q] = (u0 && nbeg == 0) ? u0[q] : 0.0;
  __syncthreads();
  for (int n = nbeg; n < nend; ++n) {
    for (int k = threadIdx.x; k < K; k += kBlock)
      v[k] = (f ? static_cast<double>(f[static_cast<size_t>(n) * K + k]) : 0.0) + s_cin[k / P] * prv[k % P];
    __syncthreads();
    const double* Ainv = W + static_cast<size_t>(n) * K * L + K;
    for (int k = threadIdx.x; k < K; k += kBlock) {
      const double* row = Ainv + static_cast<size_t>(k) * L;
      double s = 0.0;
      for (int j = 0; j < K; ++j) s += row[j] * v[j];
      xv[k] = s;
      U[static_cast<size_t>(n) * K + k] = static_cast<T>(s);
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

}  // namespace

size_t coarse_inverse_doubles(const OpParams& p) {
  const size_t K = static_cast<size_t>(p.M) * p.nx * p.ny;
  return static_cast<size_t>(p.N) * K * 2 * K;
}

template <typename T>
hipError_t launch_coarse_invert_coef(const OpParams& p, const T* coef, double* W, hipStream_t s) {
  const int K = p.M * p.nx * p.ny;
  if (K < 1 || p.N < 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_coarse_invert_coef<T>), dim3(p.N), dim3(kBlock), static_cast<size_t>(K) * sizeof(double), s,
                     p, coef, W);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve_slabs(const OpParams& p, const double* W, const T* f, const double* u0, T* U,
                                     hipStream_t s) {
  const int P = p.nx * p.ny;
  const size_t shm = static_cast<size_t>(2 * p.M * P + P) * sizeof(double);
  bool coupled = false;
  for (int i = 0; i < p.M; ++i) coupled = coupled || p.cin[i] != 0.0;
  const int grid = (!coupled && !u0) ? p.N : 1;
  hipLaunchKernelGGL((k_coarse_solve_slabs<T>), dim3(grid), dim3(kBlock), shm, s, p, W, f, u0, U);
  return hipGetLastError();
}

template hipError_t launch_coarse_invert_coef<double>(const OpParams&, const double*, double*, hipStream_t);
template hipError_t launch_coarse_invert_coef<float>(const OpParams&, const float*, double*, hipStream_t);
template hipError_t launch_coarse_solve_slabs<double>(const OpParams&, const double*, const double*, const double*,
                                                      double*, hipStream_t);
template hipError_t launch_coarse_solve_slabs<float>(const OpParams&, const double*, const float*, const double*,
                                                     float*, hipStream_t);

}  // namespace stmg
