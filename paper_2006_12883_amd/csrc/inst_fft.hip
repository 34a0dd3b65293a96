// Exact coarsest-level solve by discrete Fourier diagonalization (periodic
// grids, constant reaction).  With periodic boundaries every slab matrix
// K (x) I + diag(dt b) (x) (-Lap + lambda) of Eq. (st_system) is diagonalized by
// the 2D DFT of the plane: Fourier mode q = (kx, ky) sees the M x M matrix
//   S_q = K + diag(dt b) (lambda_q + lambda),
//   lambda_q = cx (2 - 2 cos(2 pi kx / nx)) + cy (2 - 2 cos(2 pi ky / ny)),
// and the time coupling -cin (x) cout^T acts mode by mode as well.  So
//   1. transform every plane of f (and u0) to Fourier space (k_fft_fwd*),
//   2. run the slab recurrence u_n = S_q^{-1} (f_n + cin (cout . u_{n-1}))
//      per mode (k_fft_modes_*; u_{-1} enters as the transform of u0),
//   3. transform back (k_fft_inv*).
// The transforms are radix-2 FFTs for power-of-two sides (in registers for
// 2D planes with sides of at most kFftRegSide, else in LDS) and direct DFTs
// with twiddles from a table otherwise (planes of at most kFftMaxPlane
// points).  The arithmetic is FP64 whatever the storage type, except in
// launch_fft_coarse32 (the FP32 cycles of mixed precision on register-
// transform planes: FP32 tables, work space and arithmetic).
#include <type_traits>

#include "kernels.hpp"

namespace stmg {
namespace {

constexpr int kFftBlock = 256;

// complex pairs of the arithmetic type A (FP64, or FP32 for the FP32 cycles)
template <typename A>
struct V2;
template <>
struct V2<double> {
  typedef double2 t;
};
template <>
struct V2<float> {
  typedef float2 t;
};
template <typename A>
__device__ __forceinline__ typename V2<A>::t mk2(A x, A y) {
  typename V2<A>::t v;
  v.x = x;
  v.y = y;
  return v;
}

#define STMG_DISPATCH_M_FFT(MACRO) \
  switch (p.M) {                   \
    case 1: MACRO(1); break;       \
    case 2: MACRO(2); break;       \
    case 3: MACRO(3); break;       \
    case 4: MACRO(4); break;       \
    case 5: MACRO(5); break;       \
    case 6: MACRO(6); break;       \
    case 7: MACRO(7); break;       \
    case 8: MACRO(8); break;       \
    default: return hipErrorInvalidValue; \
  }

// Twiddle table layout: tw[2 j] = cos(2 pi j / nx), tw[2 j + 1] = sin(2 pi j / nx)
// for j < nx, then the same for ny (2D).  nx + ny <= kFftMaxPlane + 1 whenever
// nx ny <= kFftMaxPlane with both >= 1, so 2 (kFftMaxPlane + 1) entries hold it.
constexpr int kTwMax = 2 * (kFftMaxPlane + 1);

// f (T, [N][M][P], may be null) and u0 (FP64 [P], may be null) to Fourier
// space: out[pl][ky][kx] complex (re, im interleaved), planes pl < N M, then
// the u0 plane at index N M when u0 is given.
template <typename T>
__global__ __launch_bounds__(kFftBlock) void k_fft_fwd(int nx, int ny, int nplanes,
                                                       const T* __restrict__ f,
                                                       const double* __restrict__ u0,
                                                       const double* __restrict__ tw,
                                                       double* __restrict__ out) {
  __shared__ double X[kFftMaxPlane];
  __shared__ double A[2 * kFftMaxPlane];
  __shared__ double W[kTwMax];
  const int P = nx * ny;
  const int pl = blockIdx.x;
  const int tid = threadIdx.x;
  const int ntw = 2 * (nx + (ny > 1 ? ny : 0));
  for (int i = tid; i < ntw; i += kFftBlock) W[i] = tw[i];
  if (pl < nplanes) {
    for (int q = tid; q < P; q += kFftBlock) X[q] = f ? (double)f[(size_t)pl * P + q] : 0.0;
  } else {
    for (int q = tid; q < P; q += kFftBlock) X[q] = u0[q];
  }
  __syncthreads();
  const double* Wx = W;
  const double* Wy = W + 2 * nx;
  // along x: A[y][kx] = sum_x X[y][x] exp(-i 2 pi kx x / nx)
  for (int idx = tid; idx < P; idx += kFftBlock) {
    const int y = idx / nx, kx = idx - y * nx;
    double re = 0.0, im = 0.0;
    int j = 0;
    for (int x = 0; x < nx; ++x) {
      const double v = X[y * nx + x];
      re += v * Wx[2 * j];
      im -= v * Wx[2 * j + 1];
      j += kx;
      if (j >= nx) j -= nx;
    }
    A[2 * idx] = re;
    A[2 * idx + 1] = im;
  }
  __syncthreads();
  double* o = out + (size_t)pl * 2 * P;
  if (ny == 1) {
    for (int idx = tid; idx < P; idx += kFftBlock) {
      o[2 * idx] = A[2 * idx];
      o[2 * idx + 1] = A[2 * idx + 1];
    }
    return;
  }
  // along y: F[ky][kx] = sum_y A[y][kx] exp(-i 2 pi ky y / ny)
  for (int idx = tid; idx < P; idx += kFftBlock) {
    const int ky = idx / nx, kx = idx - ky * nx;
    double re = 0.0, im = 0.0;
    int j = 0;
    for (int y = 0; y < ny; ++y) {
      const double ar = A[2 * (y * nx + kx)], ai = A[2 * (y * nx + kx) + 1];
      const double c = Wy[2 * j], s = Wy[2 * j + 1];
      re += ar * c + ai * s;
      im += ai * c - ar * s;
      j += ky;
      if (j >= ny) j -= ny;
    }
    o[2 * idx] = re;
    o[2 * idx + 1] = im;
  }
}

// Radix-2 forms of the two transforms for power-of-two nx and ny: iterative
// decimation-in-time butterflies in LDS (log2 nx + log2 ny stages instead of
// nx + ny multiply-adds per value).  Same results as the direct DFTs up to
// rounding.
__device__ __forceinline__ int bitrev(int i, int lg) { return lg ? (int)(__brev((unsigned)i) >> (32 - lg)) : 0; }

// In-place butterflies along one dimension of the complex array A: `rows`
// lines of length n (power of two), element (r, i) at A + 2 (r * rs + i * es);
// input in bit-reversed order along the line; W holds cos, sin of 2 pi k / n;
// sgn = -1 forward, +1 inverse.
__device__ __forceinline__ void butterflies(double* A, int rows, int n, int rs, int es, const double* W,
                                            double sgn) {
  const int hn = n >> 1;
  for (int len = 2; len <= n; len <<= 1) {
    const int half = len >> 1, step = n / len;
    for (int b = threadIdx.x; b < rows * hn; b += kFftBlock) {
      const int r = b / hn, k = b - r * hn;
      const int g = k / half, j = k - g * half;
      const int i0 = g * len + j, i1 = i0 + half;
      const double c = W[2 * (j * step)], sn = sgn * W[2 * (j * step) + 1];
      double* p0 = A + 2 * (r * rs + i0 * es);
      double* p1 = A + 2 * (r * rs + i1 * es);
      const double ar = p1[0], ai = p1[1];
      const double tr = c * ar - sn * ai, ti = c * ai + sn * ar;
      const double br = p0[0], bi = p0[1];
      p1[0] = br - tr;
      p1[1] = bi - ti;
      p0[0] = br + tr;
      p0[1] = bi + ti;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kFftBlock) void k_fft_fwd2(int nx, int ny, int lgx, int lgy, int nplanes,
                                                        const T* __restrict__ f,
                                                        const double* __restrict__ u0,
                                                        const double* __restrict__ tw,
                                                        double* __restrict__ out) {
  __shared__ double A[2 * kFftMaxPlane];
  __shared__ double B[2 * kFftMaxPlane];
  __shared__ double W[kTwMax];
  const int P = nx * ny;
  const int pl = blockIdx.x;
  const int tid = threadIdx.x;
  const int ntw = 2 * (nx + (ny > 1 ? ny : 0));
  for (int i = tid; i < ntw; i += kFftBlock) W[i] = tw[i];
  // A[y][x] = X[y][bitrev(x)] (P <= kFftMaxPlane: at most 4 values per thread,
  // all loaded before the LDS writes)
  constexpr int kPer = kFftMaxPlane / kFftBlock;
  double v[kPer];
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int q = u * kFftBlock + tid;
    v[u] = 0.0;
    if (q < P) {
      const int y = q / nx, x = q - y * nx;
      const int src = y * nx + bitrev(x, lgx);
      if (pl < nplanes) v[u] = f ? (double)f[(size_t)pl * P + src] : 0.0;
      else v[u] = u0[src];
    }
  }
#pragma unroll
  for (int u = 0; u < kPer; ++u) {
    const int q = u * kFftBlock + tid;
    if (q < P) {
      A[2 * q] = v[u];
      A[2 * q + 1] = 0.0;
    }
  }
  __syncthreads();
  butterflies(A, ny, nx, nx, 1, W, -1.0);
  double* o = out + (size_t)pl * 2 * P;
  if (ny == 1) {
    for (int i = tid; i < 2 * P; i += kFftBlock) o[i] = A[i];
    return;
  }
  // B[y][x] = A[bitrev(y)][x], then butterflies along y
  for (int q = tid; q < P; q += kFftBlock) {
    const int y = q / nx, x = q - y * nx;
    const int src = bitrev(y, lgy) * nx + x;
    B[2 * q] = A[2 * src];
    B[2 * q + 1] = A[2 * src + 1];
  }
  __syncthreads();
  butterflies(B, nx, ny, 1, nx, W + 2 * nx, -1.0);
  for (int i = tid; i < 2 * P; i += kFftBlock) o[i] = B[i];
}

template <typename T>
__global__ __launch_bounds__(kFftBlock) void k_fft_inv2(int nx, int ny, int lgx, int lgy,
                                                        const double* __restrict__ F,
                                                        const double* __restrict__ tw,
                                                        T* __restrict__ U) {
  __shared__ double A[2 * kFftMaxPlane];
  __shared__ double B[2 * kFftMaxPlane];
  __shared__ double W[kTwMax];
  const int P = nx * ny;
  const int pl = blockIdx.x;
  const int tid = threadIdx.x;
  const int ntw = 2 * (nx + (ny > 1 ? ny : 0));
  for (int i = tid; i < ntw; i += kFftBlock) W[i] = tw[i];
  const double* src = F + (size_t)pl * 2 * P;
  constexpr int kPer = kFftMaxPlane / kFftBlock;
  if (ny > 1) {
    // B[ky][kx] = F[bitrev(ky)][kx], butterflies along y
    double vr[kPer], vi[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = u * kFftBlock + tid;
      if (q < P) {
        const int y = q / nx, x = q - y * nx;
        const int s2 = bitrev(y, lgy) * nx + x;
        vr[u] = src[2 * s2];
        vi[u] = src[2 * s2 + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = u * kFftBlock + tid;
      if (q < P) {
        B[2 * q] = vr[u];
        B[2 * q + 1] = vi[u];
      }
    }
    __syncthreads();
    butterflies(B, nx, ny, 1, nx, W + 2 * nx, 1.0);
    // A[y][kx] = B[y][bitrev(kx)]
    for (int q = tid; q < P; q += kFftBlock) {
      const int y = q / nx, x = q - y * nx;
      const int s2 = y * nx + bitrev(x, lgx);
      A[2 * q] = B[2 * s2];
      A[2 * q + 1] = B[2 * s2 + 1];
    }
  } else {
    double vr[kPer], vi[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = u * kFftBlock + tid;
      if (q < P) {
        const int s2 = bitrev(q, lgx);
        vr[u] = src[2 * s2];
        vi[u] = src[2 * s2 + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int q = u * kFftBlock + tid;
      if (q < P) {
        A[2 * q] = vr[u];
        A[2 * q + 1] = vi[u];
      }
    }
  }
  __syncthreads();
  butterflies(A, ny, nx, nx, 1, W, 1.0);
  const double scale = 1.0 / (double)P;
  T* dst = U + (size_t)pl * P;
  for (int q = tid; q < P; q += kFftBlock) dst[q] = (T)(A[2 * q] * scale);
}

// Per-mode slab recurrence in Fourier space, in place on F ([N][M][P]
// complex): u_n = Sinv_q (F_n + cin p), p = cout . u_n, starting from
// p = (transform of u0)(q) when u0F is given, else 0.  Sinv: [P][M][M] real.
// Here the workgroup's MB modes are staged in LDS for every slab.  With c = cout^T S_q, beta = c . cin and d = S_q cin the coupling
// values obey the scalar recurrence
//   p_n = c . F_n + beta p_{n-1},
// so every M-vector product runs in parallel over (slab, mode) and only the
// scalar chain is sequential: (A) a_n = c . F_n, (B) p_n = a_n + beta p_{n-1}
// per mode, (C) u_n = S_q F_n + d p_{n-1}.  Used when the workgroup's
// N (M + 2) MB complex values fit in kFftLds.
constexpr int kFftLds = 48 * 1024;
constexpr int kStage = 16;
template <int M, typename A>
__global__ __launch_bounds__(kFftBlock) void k_fft_modes_lds(int P, int N, int MB, A* __restrict__ F,
                                                             const A* __restrict__ u0F,
                                                             const A* __restrict__ Sinv,
                                                             const OpParams p,
                                                             const A* __restrict__ fscale) {
  __shared__ A L[kFftLds / sizeof(A)];
  const int q0 = blockIdx.x * MB;
  const int mb = min(MB, P - q0);
  const int tid = threadIdx.x;
  const int tot = N * M * mb;
  A* Lf = L;                          // [(n M + m) MB + qq] complex
  A* La = L + 2 * (size_t)N * M * MB;  // [n MB + qq] complex: a_n, then p_{n-1}
  // stage F (loads in batches, all in flight before the LDS writes)
  for (int i0 = 0; i0 < tot; i0 += kFftBlock * kStage) {
    A re[kStage], im[kStage];
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int i = i0 + u * kFftBlock + tid;
      if (i < tot) {
        const int nm = i / mb, qq = i - nm * mb;
        const size_t at = 2 * ((size_t)nm * P + q0 + qq);
        const A sc = fscale ? fscale[q0 + qq] : A(1.0);
        re[u] = sc * F[at];
        im[u] = sc * F[at + 1];
      }
    }
#pragma unroll
    for (int u = 0; u < kStage; ++u) {
      const int i = i0 + u * kFftBlock + tid;
      if (i < tot) {
        const int nm = i / mb, qq = i - nm * mb;
        Lf[2 * (nm * MB + qq)] = re[u];
        Lf[2 * (nm * MB + qq) + 1] = im[u];
      }
    }
  }
  __syncthreads();
  // (A) a_n = c . F_n
  for (int i = tid; i < N * mb; i += kFftBlock) {
    const int n = i / mb, qq = i - n * mb;
    const A* S = Sinv + (size_t)(q0 + qq) * M * M;
    A ar = A(0.0), ai = A(0.0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      A c = A(0.0);
#pragma unroll
      for (int k = 0; k < M; ++k) c += (A)p.cout[k] * S[k * M + j];
      const int at = 2 * ((n * M + j) * MB + qq);
      ar += c * Lf[at];
      ai += c * Lf[at + 1];
    }
    La[2 * (n * MB + qq)] = ar;
    La[2 * (n * MB + qq) + 1] = ai;
  }
  __syncthreads();
  // (B) per mode: La[n] <- p_{n-1} (the coupling value entering slab n)
  if (tid < mb) {
    const A* S = Sinv + (size_t)(q0 + tid) * M * M;
    A beta = A(0.0);
#pragma unroll
    for (int j = 0; j < M; ++j) {
      A c = A(0.0);
#pragma unroll
      for (int k = 0; k < M; ++k) c += (A)p.cout[k] * S[k * M + j];
      beta += c * (A)p.cin[j];
    }
    A pr = A(0.0), pi = A(0.0);
    if (u0F) {
      pr = u0F[2 * (q0 + tid)];
      pi = u0F[2 * (q0 + tid) + 1];
    }
    for (int n = 0; n < N; ++n) {
      const int at = 2 * (n * MB + tid);
      const A ar = La[at], ai = La[at + 1];
      La[at] = pr;
      La[at + 1] = pi;
      pr = ar + beta * pr;
      pi = ai + beta * pi;
    }
  }
  __syncthreads();
  // (C) u_n = S_q F_n + d p_{n-1}, in place in Lf
  for (int i = tid; i < N * mb; i += kFftBlock) {
    const int n = i / mb, qq = i - n * mb;
    const A* S = Sinv + (size_t)(q0 + qq) * M * M;
    const A pr = La[2 * (n * MB + qq)], pi = La[2 * (n * MB + qq) + 1];
    A fr[M], fi[M];
#pragma unroll
    for (int j = 0; j < M; ++j) {
      const int at = 2 * ((n * M + j) * MB + qq);
      fr[j] = Lf[at];
      fi[j] = Lf[at + 1];
    }
#pragma unroll
    for (int k = 0; k < M; ++k) {
      A sr = A(0.0), si = A(0.0), dk = A(0.0);
#pragma unroll
      for (int j = 0; j < M; ++j) {
        sr += S[k * M + j] * fr[j];
        si += S[k * M + j] * fi[j];
        dk += S[k * M + j] * (A)p.cin[j];
      }
      const int at = 2 * ((n * M + k) * MB + qq);
      Lf[at] = sr + dk * pr;
      Lf[at + 1] = si + dk * pi;
    }
  }
  __syncthreads();
  for (int i = tid; i < tot; i += kFftBlock) {
    const int nm = i / mb, qq = i - nm * mb;
    const size_t at = 2 * ((size_t)nm * P + q0 + qq);
    F[at] = Lf[2 * (nm * MB + qq)];
    F[at + 1] = Lf[2 * (nm * MB + qq) + 1];
  }
}

// Back to physical space: U[pl][y][x] = Re (1/P) sum F[pl][ky][kx] exp(+i ...).
template <typename T>
__global__ __launch_bounds__(kFftBlock) void k_fft_inv(int nx, int ny, const double* __restrict__ F,
                                                       const double* __restrict__ tw,
                                                       T* __restrict__ U) {
  __shared__ double B[2 * kFftMaxPlane];
  __shared__ double A[2 * kFftMaxPlane];
  __shared__ double W[kTwMax];
  const int P = nx * ny;
  const int pl = blockIdx.x;
  const int tid = threadIdx.x;
  const int ntw = 2 * (nx + (ny > 1 ? ny : 0));
  for (int i = tid; i < ntw; i += kFftBlock) W[i] = tw[i];
  const double* src = F + (size_t)pl * 2 * P;
  for (int i = tid; i < 2 * P; i += kFftBlock) B[i] = src[i];
  __syncthreads();
  const double* Wx = W;
  const double* Wy = W + 2 * nx;
  const double* R = B;
  if (ny > 1) {
    // along y: A[y][kx] = sum_ky B[ky][kx] exp(+i 2 pi ky y / ny)
    for (int idx = tid; idx < P; idx += kFftBlock) {
      const int y = idx / nx, kx = idx - y * nx;
      double re = 0.0, im = 0.0;
      int j = 0;
      for (int ky = 0; ky < ny; ++ky) {
        const double br = B[2 * (ky * nx + kx)], bi = B[2 * (ky * nx + kx) + 1];
        const double c = Wy[2 * j], s = Wy[2 * j + 1];
        re += br * c - bi * s;
        im += bi * c + br * s;
        j += y;
        if (j >= ny) j -= ny;
      }
      A[2 * idx] = re;
      A[2 * idx + 1] = im;
    }
    __syncthreads();
    R = A;
  }
  // along x, real part only: U[y][x] = (1/P) Re sum_kx R[y][kx] exp(+i 2 pi kx x / nx)
  const double scale = 1.0 / (double)P;
  T* dst = U + (size_t)pl * P;
  for (int idx = tid; idx < P; idx += kFftBlock) {
    const int y = idx / nx, x = idx - y * nx;
    double re = 0.0;
    int j = 0;
    for (int kx = 0; kx < nx; ++kx) {
      re += R[2 * (y * nx + kx)] * Wx[2 * j] - R[2 * (y * nx + kx) + 1] * Wx[2 * j + 1];
      j += x;
      if (j >= nx) j -= nx;
    }
    dst[idx] = (T)(re * scale);
  }
}

// ---------------------------------------------------------------------------
// Register-resident transforms for 2D planes with power-of-two sides of at
// most 64 points (fft_reg_plane).  A wave holds 64 / n lines of n points, lane
// l the point l mod n of line l / n; one radix-2 stage of span h pairs lane l
// with lane l ^ h.  The forward transform runs decimation in frequency
// (natural order in, bit-reversed order out), the inverse decimation in time
// (bit-reversed in, natural out), so no permutation is ever applied: the
// Fourier coefficients stay in bit-reversed order.  Between the two
// directions the plane is transposed through LDS (padded lines).
//
// Planes are real, so F(-kx, -ky) = conj F(kx, ky) and only the columns
// kx = 0 .. nx/2 are kept: in bit-reversed order these are the even columns
// kx' = 2c (kx < nx/2) and kx' = 1 (kx = nx/2), stored as compact columns
// c = 0 .. nx/2 (column nx/2 for kx' = 1): the spectrum of a plane is
// [nx/2 + 1][ny] complex, ky in bit-reversed order, and the per-mode tables
// follow that order.
constexpr int kRegBlock = 512;
constexpr int kRegWaves = kRegBlock / 64;
constexpr int kRegLds = kFftRegSide * (kFftRegSide / 2 + 2);

// Value held by lane (own lane xor H) of the wave; every lane must be active.
// Spans inside a row of 16 lanes move through DPP on the vector ALU (quad
// permutations, the half-row mirror, the row rotation by 8) instead of the
// LDS crossbar that ds_bpermute uses: xor 1 and xor 2 are quad permutations,
// xor 4 is the quad reversal (xor 3) followed by the half-row mirror (xor 7),
// xor 8 is the rotation of the 16-lane row by 8.  Wider spans use
// ds_bpermute.  The values are moved, never changed.
template <int H>
__device__ __forceinline__ int xor_lane_b32(int v) {
  if constexpr (H == 1) {
    return __builtin_amdgcn_update_dpp(v, v, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
  } else if constexpr (H == 2) {
    return __builtin_amdgcn_update_dpp(v, v, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
  } else if constexpr (H == 4) {
    const int t = __builtin_amdgcn_update_dpp(v, v, 0x1B, 0xF, 0xF, false);  // quad_perm [3,2,1,0]
    return __builtin_amdgcn_update_dpp(t, t, 0x141, 0xF, 0xF, false);       // row_half_mirror
  } else if constexpr (H == 8) {
    return __builtin_amdgcn_update_dpp(v, v, 0x128, 0xF, 0xF, false);  // row_ror:8
  } else {
    return __shfl_xor(v, H);
  }
}
template <int H, typename A>
__device__ __forceinline__ A xor_lane(A v) {
  if constexpr (sizeof(A) == 8) {
    const unsigned long long b = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = static_cast<unsigned>(xor_lane_b32<H>(static_cast<int>(b & 0xffffffffull)));
    const unsigned hi = static_cast<unsigned>(xor_lane_b32<H>(static_cast<int>(b >> 32)));
    return __builtin_bit_cast(A, (static_cast<unsigned long long>(hi) << 32) | lo);
  } else {
    return __builtin_bit_cast(A, xor_lane_b32<H>(__builtin_bit_cast(int, v)));
  }
}

// A thread takes R lines per direction (R = P / 512, at least 1): all R are
// loaded first and every butterfly stage runs over the R lines together, so
// the loads and the shuffles of different lines overlap.  The butterflies are
// branch-free: the lower lane of a pair uses the twiddle 1 and the sign +1.
// Lines have n <= 64 points (a power of two), so the stages are the spans
// H < n, unrolled with H a compile-time constant.
//
// Decimation in frequency along lines of n points.  W: cos, sin of 2 pi j / n
// for j < n; sgn -1 forward.  Lower lane of a pair: u + v; upper: (u - v) w^j
// with j = (l mod h) n / (2 h), i.e. (sigma own + partner) w with sigma = -1.
static_assert(kFftRegSide <= 64, "register lines span at most one wave (stages H <= 32)");
template <typename A, int R, int H>
__device__ __forceinline__ void dif_stage(A (&re)[R], A (&im)[R], int n, const A* W, A sgn) {
  if (H >= n) return;
  const int lane = threadIdx.x & 63;
  const bool up = (lane & H) != 0;
  const int j = (lane & (H - 1)) * (n / (2 * H));
  const A c = up ? W[2 * j] : A(1.0), s = up ? sgn * W[2 * j + 1] : A(0.0);
  const A sig = up ? -A(1.0) : A(1.0);
  A pr[R], pi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    pr[r] = xor_lane<H>(re[r]);
    pi[r] = xor_lane<H>(im[r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    const A ar = fma(sig, re[r], pr[r]), ai = fma(sig, im[r], pi[r]);
    re[r] = ar * c - ai * s;
    im[r] = ar * s + ai * c;
  }
}
template <typename A, int R>
__device__ __forceinline__ void dif_lines(A (&re)[R], A (&im)[R], int n, const A* W,
                                          A sgn) {
  dif_stage<A, R, 32>(re, im, n, W, sgn);
  dif_stage<A, R, 16>(re, im, n, W, sgn);
  dif_stage<A, R, 8>(re, im, n, W, sgn);
  dif_stage<A, R, 4>(re, im, n, W, sgn);
  dif_stage<A, R, 2>(re, im, n, W, sgn);
  dif_stage<A, R, 1>(re, im, n, W, sgn);
}

// Decimation in time along lines of n points (bit-reversed input): every lane
// forms x = own w^j (w = 1 on the lower lane), the pair exchanges x; lower:
// u + t, upper: u - t (t = v w^j).
template <typename A, int R, int H>
__device__ __forceinline__ void dit_stage(A (&re)[R], A (&im)[R], int n, const A* W, A sgn) {
  if (H >= n) return;
  const int lane = threadIdx.x & 63;
  const bool up = (lane & H) != 0;
  const int j = (lane & (H - 1)) * (n / (2 * H));
  const A c = up ? W[2 * j] : A(1.0), s = up ? sgn * W[2 * j + 1] : A(0.0);
  const A sig = up ? -A(1.0) : A(1.0);
  A xr[R], xi[R], pr[R], pi[R];
#pragma unroll
  for (int r = 0; r < R; ++r) {
    xr[r] = re[r] * c - im[r] * s;
    xi[r] = re[r] * s + im[r] * c;
    pr[r] = xor_lane<H>(xr[r]);
    pi[r] = xor_lane<H>(xi[r]);
  }
#pragma unroll
  for (int r = 0; r < R; ++r) {
    re[r] = fma(sig, xr[r], pr[r]);
    im[r] = fma(sig, xi[r], pi[r]);
  }
}
template <typename A, int R>
__device__ __forceinline__ void dit_lines(A (&re)[R], A (&im)[R], int n, const A* W,
                                          A sgn) {
  dit_stage<A, R, 1>(re, im, n, W, sgn);
  dit_stage<A, R, 2>(re, im, n, W, sgn);
  dit_stage<A, R, 4>(re, im, n, W, sgn);
  dit_stage<A, R, 8>(re, im, n, W, sgn);
  dit_stage<A, R, 16>(re, im, n, W, sgn);
  dit_stage<A, R, 32>(re, im, n, W, sgn);
}

// Lines handled by a thread: line r is (wid + kRegWaves r) lpw + line along
// the other direction.  R = P / 512 (at least 1) lines cover a full
// direction; the real-valued row passes pair rows r and r + RP in one complex
// line (RP = R / 2 when R >= 2); the compact columns (nx/2 + 1 of them) take
// RC = R / 2 + 1 lines (R >= 2).
template <int R>
struct RegLines {
  static constexpr int RP = R >= 2 ? R / 2 : 1;
  static constexpr int RC = R >= 2 ? R / 2 + 1 : 1;
};

__device__ __forceinline__ int brev_n(int i, int lg) { return (int)(__brev((unsigned)i) >> (32 - lg)); }

// Forward: plane pl of f (or u0 for pl == nplanes) -> out[pl][c][ky'].
// Rows: two real rows a, b form z = a + i b; after the transform
// A[k] = (Z[k] + conj Z[-k]) / 2, B[k] = (Z[k] - conj Z[-k]) / 2i, with Z[-k]
// read from the lane holding bit-reversed (n - k) mod n; lanes of the kept
// columns write them to the tile [c][y] (stride ny + 1).
template <typename T, typename A, int R>
__global__ __launch_bounds__(kRegBlock) void k_fft_fwd_reg(int nx, int ny, int lgx, int nplanes,
                                                           const T* __restrict__ f,
                                                           const double* __restrict__ u0,
                                                           const A* __restrict__ tw,
                                                           A* __restrict__ out) {
  constexpr int RP = RegLines<R>::RP, RC = RegLines<R>::RC;
  constexpr bool PACK = R >= 2;
  __shared__ A Tr[kRegLds];
  __shared__ A Ti[kRegLds];
  __shared__ A W[4 * kFftRegSide];
  const int P = nx * ny, nh = nx >> 1, Ph = (nh + 1) * ny;
  const int pl = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int i = tid; i < 2 * (nx + ny); i += kRegBlock) W[i] = tw[i];
  const double* src = pl < nplanes ? nullptr : u0;
  auto ld = [&](int y, int x) -> A {
    if (y >= ny) return A(0.0);
    if (src) return (A)src[y * nx + x];
    return f ? (A)f[(size_t)pl * P + y * nx + x] : A(0.0);
  };
  // rows: lane = x in, kx' = pos out
  {
    const int lpw = 64 / nx, line = lane / nx, pos = lane - line * nx;
    A re[RP], im[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      re[r] = ld((wid + kRegWaves * r) * lpw + line, pos);
      im[r] = PACK ? ld((wid + kRegWaves * (r + RP)) * lpw + line, pos) : A(0.0);
    }
    __syncthreads();  // W
    dif_lines<A, RP>(re, im, nx, W, -A(1.0));
    // lane of the partner coefficient Z[-k], k = bitrev(pos); kept column
    const int kn = (nx - brev_n(pos, lgx)) & (nx - 1);
    const int src_lane = line * nx + brev_n(kn, lgx);
    const bool keep = (pos & 1) == 0 || pos == 1;
    const int c = (pos & 1) ? nh : pos >> 1;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int ya = (wid + kRegWaves * r) * lpw + line;
      if (PACK) {
        const int yb = (wid + kRegWaves * (r + RP)) * lpw + line;
        const A wr = __shfl(re[r], src_lane), wi = __shfl(im[r], src_lane);
        if (keep && ya < ny) {
          Tr[c * (ny + 1) + ya] = A(0.5) * (re[r] + wr);
          Ti[c * (ny + 1) + ya] = A(0.5) * (im[r] - wi);
        }
        if (keep && yb < ny) {
          Tr[c * (ny + 1) + yb] = A(0.5) * (im[r] + wi);
          Ti[c * (ny + 1) + yb] = A(0.5) * (wr - re[r]);
        }
      } else if (keep && ya < ny) {
        Tr[c * (ny + 1) + ya] = re[r];
        Ti[c * (ny + 1) + ya] = im[r];
      }
    }
  }
  __syncthreads();
  // kept columns: lane = y in, ky' out
  {
    const int lpw = 64 / ny, line = lane / ny, pos = lane - line * ny;
    A re[RC], im[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int c = (wid + kRegWaves * r) * lpw + line;
      re[r] = c <= nh ? Tr[c * (ny + 1) + pos] : A(0.0);
      im[r] = c <= nh ? Ti[c * (ny + 1) + pos] : A(0.0);
    }
    dif_lines<A, RC>(re, im, ny, W + 2 * nx, -A(1.0));
    typename V2<A>::t* o = reinterpret_cast<typename V2<A>::t*>(out + (size_t)pl * 2 * Ph);
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int c = (wid + kRegWaves * r) * lpw + line;
      if (c <= nh) o[c * ny + pos] = mk2<A>(re[r], im[r]);
    }
  }
}

// Inverse: F[pl][c][ky'] -> U[pl][y][x] = Re (1/P) sum F exp(+i ...).
// Columns: the kept columns back to y (tile [y][c], stride nh + 2).  Rows:
// lane kx' takes its column from the tile, for the dropped columns (odd
// kx' != 1, kx > nx/2) as the conjugate of column nx - kx; the row spectra
// are Hermitian (the field is real), so two rows a, b go through one
// transform of A + i B and come out as its real and imaginary parts.
template <typename T, typename A, int R>
__global__ __launch_bounds__(kRegBlock) void k_fft_inv_reg(int nx, int ny, int lgx,
                                                           const A* __restrict__ F,
                                                           const A* __restrict__ tw,
                                                           T* __restrict__ U) {
  constexpr int RP = RegLines<R>::RP, RC = RegLines<R>::RC;
  constexpr bool PACK = R >= 2;
  __shared__ A Tr[kRegLds];
  __shared__ A Ti[kRegLds];
  __shared__ A W[4 * kFftRegSide];
  const int P = nx * ny, nh = nx >> 1, Ph = (nh + 1) * ny, ts = nh + 2;
  const int pl = blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  for (int i = tid; i < 2 * (nx + ny); i += kRegBlock) W[i] = tw[i];
  // kept columns: lane = ky' in, y out
  {
    const int lpw = 64 / ny, line = lane / ny, pos = lane - line * ny;
    const typename V2<A>::t* src = reinterpret_cast<const typename V2<A>::t*>(F + (size_t)pl * 2 * Ph);
    A re[RC], im[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int c = (wid + kRegWaves * r) * lpw + line;
      const typename V2<A>::t v = c <= nh ? src[c * ny + pos] : mk2<A>(A(0.0), A(0.0));
      re[r] = v.x;
      im[r] = v.y;
    }
    __syncthreads();  // W
    dit_lines<A, RC>(re, im, ny, W + 2 * nx, A(1.0));
#pragma unroll
    for (int r = 0; r < RC; ++r) {
      const int c = (wid + kRegWaves * r) * lpw + line;
      if (c <= nh) {
        Tr[pos * ts + c] = re[r];
        Ti[pos * ts + c] = im[r];
      }
    }
  }
  __syncthreads();
  // rows: lane = kx' in, x out
  {
    const int lpw = 64 / nx, line = lane / nx, pos = lane - line * nx;
    int c;
    A cs = A(1.0);  // -1: conjugate
    if ((pos & 1) == 0) c = pos >> 1;
    else if (pos == 1) c = nh;
    else {
      c = brev_n(nx - brev_n(pos, lgx), lgx) >> 1;
      cs = -A(1.0);
    }
    A re[RP], im[RP];
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int ya = (wid + kRegWaves * r) * lpw + line;
      const A ar = ya < ny ? Tr[ya * ts + c] : A(0.0);
      const A ai = ya < ny ? cs * Ti[ya * ts + c] : A(0.0);
      if (PACK) {
        const int yb = (wid + kRegWaves * (r + RP)) * lpw + line;
        const A br = yb < ny ? Tr[yb * ts + c] : A(0.0);
        const A bi = yb < ny ? cs * Ti[yb * ts + c] : A(0.0);
        re[r] = ar - bi;
        im[r] = ai + br;
      } else {
        re[r] = ar;
        im[r] = ai;
      }
    }
    dit_lines<A, RP>(re, im, nx, W, A(1.0));
    const A scale = A(1.0) / (A)P;
    T* dst = U + (size_t)pl * P;
#pragma unroll
    for (int r = 0; r < RP; ++r) {
      const int ya = (wid + kRegWaves * r) * lpw + line;
      if (ya < ny) dst[ya * nx + pos] = (T)(re[r] * scale);
      if (PACK) {
        const int yb = (wid + kRegWaves * (r + RP)) * lpw + line;
        if (yb < ny) dst[yb * nx + pos] = (T)(im[r] * scale);
      }
    }
  }
}

// Per-mode slab recurrence for long time axes (the workgroup's modes do not
// fit in LDS for all slabs): kChunkQ modes x kChunkC runs of consecutive
// slabs per workgroup; a run of at most ChunkG<M>::G slabs is read once.
// With c = cout^T S_q, beta = c . cin, d = S_q cin:
//   (1) each run folds a_n = c . F_n into s = a_n + beta s from s = 0 and
//       records s and beta^len;
//   (2) one thread per mode chains the runs: p entering run r+1 is
//       s_r + beta^len_r p entering run r (p entering run 0 = transform of
//       u0, or 0);
//   (3) each run replays its slabs from its entering p:
//       u_n = S_q F_n + d p_{n-1}, p_n = a_n + beta p_{n-1}, in place in F.
// The same recurrence as k_fft_modes_lds, with the chain regrouped by runs.
constexpr int kChunkQ = 16;
constexpr int kChunkC = kFftBlock / kChunkQ;
// slabs whose loads are issued together (a run of at most this many slabs
// keeps its values in registers from step (1) to step (3))
template <int M>
struct ChunkG {
  static constexpr int G = M <= 3 ? 16 : 48 / M;
};
template <int M, typename A>
__global__ __launch_bounds__(kFftBlock) void k_fft_modes_chunk(int P, int N, A* __restrict__ F,
                                                               const A* __restrict__ u0F,
                                                               const A* __restrict__ Sinv,
                                                               const OpParams p,
                                                               const A* __restrict__ fscale) {
  __shared__ A Sr[kChunkC][kChunkQ], Si[kChunkC][kChunkQ], Bp[kChunkC][kChunkQ];
  const int qq = threadIdx.x % kChunkQ, ch = threadIdx.x / kChunkQ;
  const int q = blockIdx.x * kChunkQ + qq;
  const bool act = q < P;
  const int len = (N + kChunkC - 1) / kChunkC;
  const int n0 = min(ch * len, N), n1 = min(n0 + len, N);
  A S[M][M], cv[M], dv[M], beta = A(0.0);
#pragma unroll
  for (int i = 0; i < M; ++i)
#pragma unroll
    for (int j = 0; j < M; ++j) S[i][j] = act ? Sinv[((size_t)q * M + i) * M + j] : A(0.0);
#pragma unroll
  for (int j = 0; j < M; ++j) {
    A cj = A(0.0);
#pragma unroll
    for (int k = 0; k < M; ++k) cj += (A)p.cout[k] * S[k][j];
    cv[j] = cj;
    beta += cj * (A)p.cin[j];
  }
#pragma unroll
  for (int k = 0; k < M; ++k) {
    A dk = A(0.0);
#pragma unroll
    for (int j = 0; j < M; ++j) dk += S[k][j] * (A)p.cin[j];
    dv[k] = dk;
  }
  typename V2<A>::t* Fc = reinterpret_cast<typename V2<A>::t*>(F);
  const A fsc = (fscale && act) ? fscale[q] : A(1.0);
  constexpr int G = ChunkG<M>::G;
  const bool cached = n1 - n0 <= G;
  typename V2<A>::t v[G][M];
  // (1)
  A sr = A(0.0), si = A(0.0), bp = A(1.0);
  if (act) {
    for (int g0 = n0; g0 < n1; g0 += G) {
#pragma unroll
      for (int g = 0; g < G; ++g)
#pragma unroll
        for (int m = 0; m < M; ++m) {
          v[g][m] = g0 + g < n1 ? Fc[((size_t)(g0 + g) * M + m) * P + q] : mk2<A>(A(0.0), A(0.0));
          v[g][m].x *= fsc;
          v[g][m].y *= fsc;
        }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g0 + g < n1) {
          A ar = A(0.0), ai = A(0.0);
#pragma unroll
          for (int j = 0; j < M; ++j) {
            ar += cv[j] * v[g][j].x;
            ai += cv[j] * v[g][j].y;
          }
          sr = ar + beta * sr;
          si = ai + beta * si;
          bp *= beta;
        }
      }
    }
  }
  Sr[ch][qq] = sr;
  Si[ch][qq] = si;
  Bp[ch][qq] = bp;
  __syncthreads();
  // (2): the entering p of every run replaces its (s, beta^len) in LDS
  if (ch == 0 && act) {
    A pr = A(0.0), pi = A(0.0);
    if (u0F) {
      pr = u0F[2 * q];
      pi = u0F[2 * q + 1];
    }
    for (int r = 0; r < kChunkC; ++r) {
      const A s0 = Sr[r][qq], s1 = Si[r][qq], b = Bp[r][qq];
      Sr[r][qq] = pr;
      Si[r][qq] = pi;
      pr = s0 + b * pr;
      pi = s1 + b * pi;
    }
  }
  __syncthreads();
  // (3)
  if (act) {
    A pr = Sr[ch][qq], pi = Si[ch][qq];
    for (int g0 = n0; g0 < n1; g0 += G) {
      if (!cached) {
#pragma unroll
        for (int g = 0; g < G; ++g)
#pragma unroll
          for (int m = 0; m < M; ++m) {
            v[g][m] = g0 + g < n1 ? Fc[((size_t)(g0 + g) * M + m) * P + q] : mk2<A>(A(0.0), A(0.0));
            v[g][m].x *= fsc;
            v[g][m].y *= fsc;
          }
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (g0 + g < n1) {
          A ar = A(0.0), ai = A(0.0);
#pragma unroll
          for (int k = 0; k < M; ++k) {
            A ur = dv[k] * pr, ui = dv[k] * pi;
#pragma unroll
            for (int j = 0; j < M; ++j) {
              ur += S[k][j] * v[g][j].x;
              ui += S[k][j] * v[g][j].y;
            }
            Fc[((size_t)(g0 + g) * M + k) * P + q] = mk2<A>(ur, ui);
            ar += cv[k] * v[g][k].x;
            ai += cv[k] * v[g][k].y;
          }
          pr = ar + beta * pr;
          pi = ai + beta * pi;
        }
      }
    }
  }
}

}  // namespace

// The three steps with arithmetic type A: FP64 on every plane the Fourier
// solve takes, FP32 on the register-transform planes only.
template <typename T, typename A>
static hipError_t fft_coarse_impl(const OpParams& p, const A* Sinv, const A* tw, A* work, const T* f,
                                  const double* u0, T* U, hipStream_t s, const A* fscale) {
  constexpr bool F64 = std::is_same<A, double>::value;
  const int P = p.nx * p.ny;
  const bool reg = fft_reg_plane(p.nx, p.ny);
  if ((!reg && (P > kFftMaxPlane || !F64)) || p.M < 1 || p.M > kMaxM) return hipErrorInvalidValue;
  const int planes = p.N * p.M;
  // modes per plane in Fourier space (the kept half for the register path)
  const int PF = reg ? (p.nx / 2 + 1) * p.ny : P;
  A* u0F = u0 ? work + (size_t)2 * planes * PF : nullptr;
  auto lg2 = [](int n) { int l = 0; while ((1 << l) < n) ++l; return (1 << l) == n ? l : -1; };
  const int lgx = lg2(p.nx), lgy = lg2(p.ny);
  const bool pow2 = lgx >= 0 && lgy >= 0;
  // lines per thread and direction for the register transforms
  const int R = P <= kRegBlock ? 1 : P / kRegBlock;
#define LREG(RR, KERNEL, GRID, ...)                                                        \
  switch (RR) {                                                                            \
    case 1: hipLaunchKernelGGL((KERNEL<T, A, 1>), dim3(GRID), dim3(kRegBlock), 0, s, __VA_ARGS__); break; \
    case 2: hipLaunchKernelGGL((KERNEL<T, A, 2>), dim3(GRID), dim3(kRegBlock), 0, s, __VA_ARGS__); break; \
    case 4: hipLaunchKernelGGL((KERNEL<T, A, 4>), dim3(GRID), dim3(kRegBlock), 0, s, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL((KERNEL<T, A, 8>), dim3(GRID), dim3(kRegBlock), 0, s, __VA_ARGS__); break; \
  }
  if (reg) {
    LREG(R, k_fft_fwd_reg, planes + (u0 ? 1 : 0), p.nx, p.ny, lgx, planes, f, u0, tw, work)
  } else if constexpr (F64) {
    if (pow2)
      hipLaunchKernelGGL((k_fft_fwd2<T>), dim3(planes + (u0 ? 1 : 0)), dim3(kFftBlock), 0, s, p.nx, p.ny,
                         lgx, lgy, planes, f, u0, tw, work);
    else
      hipLaunchKernelGGL((k_fft_fwd<T>), dim3(planes + (u0 ? 1 : 0)), dim3(kFftBlock), 0, s, p.nx, p.ny,
                         planes, f, u0, tw, work);
  }
  // modes per workgroup for the LDS-staged recurrence (at most 64, at least
  // 4), sized with 8-byte values whatever A is: where FP64 modes no longer fit
  // four to a workgroup the time axis is long enough that the run-chunked
  // recurrence, with 16 modes x 16 runs per workgroup, is the faster one in
  // FP32 too
  const long long per_mode = (long long)p.N * (p.M + 2) * 2 * sizeof(double);
  int MB = (int)(kFftLds / per_mode);
  if (MB > 64) MB = 64;
  if (MB >= 4) {
    const int gb = (PF + MB - 1) / MB;
#define L(MM)                                                                                        \
  hipLaunchKernelGGL((k_fft_modes_lds<MM, A>), dim3(gb), dim3(kFftBlock), 0, s, PF, p.N, MB, work, u0F, \
                     Sinv, p, fscale)
    STMG_DISPATCH_M_FFT(L)
#undef L
  } else {
    const int gb = (PF + kChunkQ - 1) / kChunkQ;
#define L(MM)                                                                                           \
  hipLaunchKernelGGL((k_fft_modes_chunk<MM, A>), dim3(gb), dim3(kFftBlock), 0, s, PF, p.N, work, u0F, Sinv, p, \
                     fscale)
    STMG_DISPATCH_M_FFT(L)
#undef L
  }
  if (reg) {
    LREG(R, k_fft_inv_reg, planes, p.nx, p.ny, lgx, work, tw, U)
  } else if constexpr (F64) {
    if (pow2)
      hipLaunchKernelGGL((k_fft_inv2<T>), dim3(planes), dim3(kFftBlock), 0, s, p.nx, p.ny, lgx, lgy, work,
                         tw, U);
    else
      hipLaunchKernelGGL((k_fft_inv<T>), dim3(planes), dim3(kFftBlock), 0, s, p.nx, p.ny, work, tw, U);
  }
#undef LREG
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fft_coarse(const OpParams& p, const double* Sinv, const double* tw, double* work,
                             const T* f, const double* u0, T* U, hipStream_t s, const double* fscale) {
  return fft_coarse_impl<T, double>(p, Sinv, tw, work, f, u0, U, s, fscale);
}

hipError_t launch_fft_coarse32(const OpParams& p, const float* Sinv, const float* tw, float* work, const float* f,
                               const double* u0, float* U, hipStream_t s, const float* fscale) {
  if (!fft_reg_plane(p.nx, p.ny)) return hipErrorNotSupported;
  return fft_coarse_impl<float, float>(p, Sinv, tw, work, f, u0, U, s, fscale);
}

template hipError_t launch_fft_coarse<double>(const OpParams&, const double*, const double*, double*,
                                              const double*, const double*, double*, hipStream_t, const double*);
template hipError_t launch_fft_coarse<float>(const OpParams&, const double*, const double*, double*,
                                             const float*, const double*, float*, hipStream_t, const double*);

}  // namespace stmg
