// Non-template launchers and elementwise / reduction instantiations.
#include "launchers.hpp"

namespace stmg {

namespace {

__global__ __launch_bounds__(kBlock) void k_sum_partials(const double* __restrict__ part, int n,
                                                         double* __restrict__ out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += part[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) out[0] = t;
}

__global__ __launch_bounds__(kBlock) void k_sumsq(const double* __restrict__ x, size_t n,
                                                  double* __restrict__ part) {
  double s = 0.0;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride) s += x[i] * x[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ __launch_bounds__(kBlock) void k_reverse_slabs(const double* __restrict__ in,
                                                          double* __restrict__ out, int N,
                                                          size_t slab) {
  const size_t total = (size_t)N * slab;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
    const size_t n = e / slab, r = e % slab;
    out[(size_t)(N - 1 - n) * slab + r] = in[e];
  }
}

__global__ __launch_bounds__(kBlock) void k_node_combine(const double* __restrict__ lam, const double* w,
                                                         int M, size_t P, double* __restrict__ out) {
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t q = (size_t)blockIdx.x * kBlock + threadIdx.x; q < P; q += stride) {
    double s = 0.0;
    for (int i = 0; i < M; ++i) s += w[i] * lam[(size_t)i * P + q];
    out[q] = s;
  }
}

__global__ __launch_bounds__(kBlock) void k_grad_nu(const OpParams p, const double* __restrict__ U,
                                                    const double* __restrict__ lam, double* __restrict__ part) {
  __shared__ double s_db[kMaxM];
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < kMaxM; ++i) s_db[i] = p.db[i];
  }
  __syncthreads();
  const int nx = p.nx, ny = p.ny, P = nx * ny, M = p.M, N = p.N;
  const size_t total = (size_t)N * M * P;
  const size_t stride = (size_t)gridDim.x * kBlock;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += stride) {
    const int q = (int)(e % P);
    const int i = (int)((e / P) % M);
    const int n = (int)(e / ((size_t)P * M));
    const int x = q % nx, y = q / nx;
    const double* Um = U + ((size_t)n * M + i) * P;
    const double c = Um[q];
    double l = p.cx * (Um[y * nx + nb_lo(x, nx, p.bc)] + Um[y * nx + nb_hi(x, nx, p.bc)] - 2.0 * c);
    if (ny > 1) l += p.cy * (Um[nb_lo(y, ny, p.bc) * nx + x] + Um[nb_hi(y, ny, p.bc) * nx + x] - 2.0 * c);
    acc += lam[((size_t)(N - 1 - n) * M + i) * P + q] * s_db[i] * l;
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// c = gamma (3 u^2 - 1) into c64 and c32, two values per thread and step
// (U and c64 16-byte aligned, c32 8-byte aligned; the odd last value by
// thread 0 of block 0).
__global__ __launch_bounds__(kBlock) void k_newton_coef_pair(size_t n, const double* __restrict__ U, double gamma,
                                                             double* __restrict__ c64, float* __restrict__ c32) {
  const size_t n2 = n >> 1;
  const size_t stride = (size_t)gridDim.x * kBlock;
  for (size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x; e < n2; e += stride) {
    const double2 u = reinterpret_cast<const double2*>(U)[e];
    double2 c;
    c.x = gamma * (3.0 * u.x * u.x - 1.0);
    c.y = gamma * (3.0 * u.y * u.y - 1.0);
    reinterpret_cast<double2*>(c64)[e] = c;
    float2 f;
    f.x = (float)c.x;
    f.y = (float)c.y;
    reinterpret_cast<float2*>(c32)[e] = f;
  }
  if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const double u = U[n - 1];
    const double c = gamma * (3.0 * u * u - 1.0);
    c64[n - 1] = c;
    c32[n - 1] = (float)c;
  }
}

// SDC update with the explicit reaction of the IMEX sweep (see kernels.hpp).
__global__ __launch_bounds__(kBlock) void k_sdc_update_imex(double* __restrict__ U, double* __restrict__ acc,
                                                            const double* __restrict__ d, int N, int M, int nx,
                                                            int ny, int bc, double cx, double cy, double lam,
                                                            double w, double gamma, double we, int m) {
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
    double* u = U + (n * M + m) * P + q;
    const double uo = *u, un = uo + c;
    *u = un;
    acc[e] += w * (l - lam * c) + we * gamma * ((un - un * un * un) - (uo - uo * uo * uo));
  }
}
}  // namespace

hipError_t launch_newton_coef_pair(size_t n, const double* U, double gamma, double* c64, float* c32,
                                   hipStream_t s) {
  const bool aligned = (reinterpret_cast<uintptr_t>(U) & 15) == 0 && (reinterpret_cast<uintptr_t>(c64) & 15) == 0 &&
                       (reinterpret_cast<uintptr_t>(c32) & 7) == 0;
  if (!aligned) {
    hipError_t e = launch_newton_coef<double>(n, U, gamma, c64, s);
    if (e != hipSuccess) return e;
    return launch_newton_coef<float>(n, U, gamma, c32, s);
  }
  hipLaunchKernelGGL(k_newton_coef_pair, dim3(grid_for(n >> 1)), dim3(kBlock), 0, s, n, U, gamma, c64, c32);
  return hipGetLastError();
}

template <typename T>
__global__ __launch_bounds__(kBlock) void k_node_transfer(const T* __restrict__ in, int Min,
                                                          T* __restrict__ out, int Mout, const NodeMat W,
                                                          int N, size_t P) {
  const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
  if (idx >= (size_t)N * P) return;
  const size_t n = idx / P, q = idx - n * P;
  double v[kMaxM];
  for (int i = 0; i < Min; ++i) v[i] = (double)in[(n * Min + i) * P + q];
  for (int o = 0; o < Mout; ++o) {
    double s = 0.0;
    for (int i = 0; i < Min; ++i) s += W.W[o * Min + i] * v[i];
    out[(n * Mout + o) * P + q] = (T)s;
  }
}

template <typename T>
hipError_t launch_node_transfer(const T* in, int Min, T* out, int Mout, const NodeMat& W, int N,
                                size_t P, hipStream_t s) {
  if (Min < 1 || Min > kMaxM || Mout < 1 || Mout > kMaxM) return hipErrorInvalidValue;
  const size_t tot = (size_t)N * P;
  if (tot == 0) return hipSuccess;
  const unsigned nb = (unsigned)((tot + kBlock - 1) / kBlock);
  hipLaunchKernelGGL((k_node_transfer<T>), dim3(nb), dim3(kBlock), 0, s, in, Min, out, Mout, W, N, P);
  return hipGetLastError();
}
template hipError_t launch_node_transfer<double>(const double*, int, double*, int, const NodeMat&, int,
                                                 size_t, hipStream_t);
template hipError_t launch_node_transfer<float>(const float*, int, float*, int, const NodeMat&, int,
                                                size_t, hipStream_t);

int smooth_blocks(const OpParams& p, int chunk) {
  return ((plane_threads(p) + kBlock - 1) / kBlock) * ((p.N + chunk - 1) / chunk);
}

bool blocked_layout(const OpParams& p) { return blocked(p); }

hipError_t launch_sum_partials(const double* part, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_sum_partials, dim3(1), dim3(kBlock), 0, s, part, n, out);
  return hipGetLastError();
}

hipError_t launch_sumsq(const double* x, size_t n, double* part, int* nparts, hipStream_t s) {
  const int g = grid_for(n) > 1024 ? 1024 : grid_for(n);
  *nparts = g;
  hipLaunchKernelGGL(k_sumsq, dim3(g), dim3(kBlock), 0, s, x, n, part);
  return hipGetLastError();
}

hipError_t launch_reverse_slabs(const double* in, double* out, int N, int M, size_t P,
                                hipStream_t s) {
  const size_t slab = (size_t)M * P;
  hipLaunchKernelGGL(k_reverse_slabs, dim3(grid_for((size_t)N * slab)), dim3(kBlock), 0, s, in, out,
                     N, slab);
  return hipGetLastError();
}

hipError_t launch_node_combine(const double* lam, const double* w, int M, size_t P, double* out,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_node_combine, dim3(grid_for(P)), dim3(kBlock), 0, s, lam, w, M, P, out);
  return hipGetLastError();
}

hipError_t launch_grad_nu(const OpParams& p, const double* U, const double* lam, double* part,
                          int* nparts, hipStream_t s) {
  const size_t total = (size_t)p.N * p.M * p.nx * p.ny;
  int g = grid_for(total);
  if (g > 1024) g = 1024;
  *nparts = g;
  hipLaunchKernelGGL(k_grad_nu, dim3(g), dim3(kBlock), 0, s, p, U, lam, part);
  return hipGetLastError();
}

hipError_t launch_node_transform(double* r, int N, int M, int P, const double* G, hipStream_t s) {
  hipLaunchKernelGGL(k_node_transform, dim3(grid_for((size_t)N * P)), dim3(kBlock), 0, s, r, N, M, P, G);
  return hipGetLastError();
}

hipError_t launch_sdc_gather(const double* r, const double* acc, double* rhs, int N, int M, int P,
                             int m, hipStream_t s) {
  hipLaunchKernelGGL(k_sdc_gather, dim3(grid_for((size_t)N * P)), dim3(kBlock), 0, s, r, acc, rhs, N, M, P, m);
  return hipGetLastError();
}

hipError_t launch_sdc_update_imex(double* U, double* acc, const double* d, int N, int M, int nx, int ny,
                                  int bc, double cx, double cy, double lam, double w, double gamma,
                                  double we, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_sdc_update_imex, dim3(grid_for((size_t)N * nx * ny)), dim3(kBlock), 0, s, U, acc, d, N,
                     M, nx, ny, bc, cx, cy, lam, w, gamma, we, m);
  return hipGetLastError();
}

hipError_t launch_sdc_update(double* U, double* acc, const double* d, int N, int M, int nx, int ny,
                             int bc, double cx, double cy, double lam, double w, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_sdc_update, dim3(grid_for((size_t)N * nx * ny)), dim3(kBlock), 0, s, U, acc, d, N,
                     M, nx, ny, bc, cx, cy, lam, w, m);
  return hipGetLastError();
}

template hipError_t launch_coarse_solve<double>(const OpParams&, const double*, const double*, const double*, double*, hipStream_t);
template hipError_t launch_coarse_solve<float>(const OpParams&, const double*, const float*, const double*, float*, hipStream_t);
template hipError_t launch_coarse_solve_coef<double>(const OpParams&, const double*, double*, const double*, const double*, double*, hipStream_t);
template hipError_t launch_coarse_solve_coef<float>(const OpParams&, const float*, double*, const float*, const double*, float*, hipStream_t);
template hipError_t launch_axpy_cast<double, float>(size_t, const double*, double, float*, bool, hipStream_t);
template hipError_t launch_axpy_cast<float, double>(size_t, const float*, double, double*, bool, hipStream_t);
template hipError_t launch_axpy_cast<double, double>(size_t, const double*, double, double*, bool, hipStream_t);
template hipError_t launch_update<float>(size_t, double*, const float*, const double*, hipStream_t);
template hipError_t launch_update<double>(size_t, double*, const double*, const double*, hipStream_t);
template hipError_t launch_newton_coef<double>(size_t, const double*, double, double*, hipStream_t);
template hipError_t launch_newton_coef<float>(size_t, const double*, double, float*, hipStream_t);
template hipError_t launch_restrict_coef<double>(const OpParams&, bool, bool, int, int, int, const double*, double*, hipStream_t);
template hipError_t launch_restrict_coef<float>(const OpParams&, bool, bool, int, int, int, const float*, float*, hipStream_t);

}  // namespace stmg
