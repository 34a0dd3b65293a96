// Kernel parameter blocks and launch wrappers (internal to libstmg).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace stmg {

constexpr int kMaxM = 8;
constexpr int kBlock = 256;  // threads per workgroup (4 wave64)

// One level's operator, passed by value as a kernel argument.
//   (A U)_{n,i} = sum_j K[i][j] U_{n,j} + db_i (-(cx D_xx + cy D_yy) U_{n,i} + react)
//                 - cin_i * (sum_j cout_j U_{n-1,j})
// D_xx u = u[x-1] + u[x+1] - 2 u[x] (periodic wrap or Neumann reflection).
// Forward problem: K = Kq, cin = l(0), cout = e_M.  Transposed problem stored
// backward in time: K = Kq^T, cin = e_M, cout = l(0).
struct OpParams {
  int M;
  int nx, ny;      // grid points of this level (ny = 1 in 1D)
  int N;           // slabs
  int bc;          // 0 periodic, 1 Neumann
  int colloc;      // residual norms in the collocation form: ||G r|| per point, G = Q diag(b)^-1
  double cx, cy;   // nu / hx^2, nu / hy^2 (cy = 0 in 1D)
  double lam;      // constant linear reaction rate
  double gamma;    // Allen-Cahn intensity
  double omega;    // smoother damping
  double K[kMaxM * kMaxM];
  double db[kMaxM];    // dt * b_i
  double cin[kMaxM];
  double cout[kMaxM];
  double Binv[kMaxM * kMaxM];  // (K + diag(db) (2cx + 2cy + lam))^{-1}
  double G[kMaxM * kMaxM];     // Q diag(b)^-1 (collocation form of a DG residual), used when colloc
};

// Spatial stencils of a Galerkin coarse level (periodic, 3 x 3, entry
// [(dy + 1) * 3 + dx + 1] weighs u(x + dx, y + dy); 1D uses the middle row).
// The level operator is
//   (A U)_{n,i} = sum_j K[i][j] (Ms U_{n,j}) + db_i (Ks U_{n,i}) - cin_i (Ms (cout . U_{n-1}))
// with Ms = R Ms_fine P and Ks = R Ks_fine P (the finest level: Ms = I,
// Ks = -nu Lap_h + lambda).  OpParams.Binv holds (K m_0 + diag(db) k_0)^-1.
struct Stencil9 {
  double m[9];
  double k[9];
};

// Reaction modes of the operator kernels.
enum { REACT_CONST = 0, REACT_COEF = 1, REACT_AC = 2 };

template <typename T>
struct SweepPtrs {
  const T* U;        // current iterate; nullptr means U = 0
  const T* f;        // explicit right-hand side; nullptr means none
  const double* u0;  // value entering slab 0 through the coupling; may be null
  const T* coef;     // REACT_COEF: per-DOF reaction coefficient
  void* out;         // smoother: new iterate (T); residual: r (type TO), may be null
  double* part;      // per-block partial sums of ||f - A U||^2 (input iterate), may be null
  // FP32 prolongation + smoothing only: when set, also up64_out = up64 + out
  // in FP64 on the written points (the refinement update of mixed precision)
  const double* up64 = nullptr;
  double* up64_out = nullptr;
};

// Launchers return hipSuccess or the launch error.
// Workgroups of a smoothing sweep (= partial sums written when a.part is set).
int smooth_blocks(const OpParams& p, int chunk);
template <typename T>
hipError_t launch_smooth(const OpParams& p, int react, const SweepPtrs<T>& a,
                         int chunk, hipStream_t s);

// Residual r = f + (u0 coupling) - A U; out type TO (double or float).
template <typename T, typename TO>
hipError_t launch_residual(const OpParams& p, int react, const SweepPtrs<T>& a,
                           int slabs_per_block, int* nparts, hipStream_t s);

// One iterative-refinement step of the mixed-precision solve fused into one
// sweep (register-blocked layouts only, else hipErrorNotSupported): a.out =
// U' = a.U + e (e may be null), r = a.f + (u0 coupling) - A U' in FP64 with
// per-block partial sums of r^2 in a.part (*nparts blocks), r32 = (float) r,
// and with e1 set the first FP32 smoothing sweep from zero for A e = r32 over
// chunks of `chunk` slabs.  react: REACT_CONST or REACT_COEF (coef32 for the
// FP32 sweep).
hipError_t launch_refine(const OpParams& p, int react, const SweepPtrs<double>& a, const float* e,
                         float* r32, float* e1, const float* coef32, int chunk, int* nparts,
                         hipStream_t s);

// f_c = R (f - A U) on the fine level described by p; the coarse level has
// ncx x ncy points and Nc slabs; space/time select the coarsening.  If uc is
// given (with the coarse level's operator pc, coefficient coefc and smoother
// block length cs) the kernel may also write the coarse level's first
// smoothing sweep from a zero iterate into uc; *smoothed tells whether it did.
template <typename T>
hipError_t launch_restrict_residual(const OpParams& p, int react, const SweepPtrs<T>& a,
                                    bool space, bool time, int ncx, int ncy, int Nc,
                                    T* fc, int slabs_per_block, hipStream_t s,
                                    const OpParams* pc = nullptr, T* uc = nullptr,
                                    const T* coefc = nullptr, int cs = 0,
                                    bool* smoothed = nullptr);

// U_out = U_in + P e_c (U_in may be null: assign).  Fine level p.
template <typename T>
hipError_t launch_prolong(const OpParams& p, bool space, bool time, int ncx, int ncy,
                          int Nc, const T* ec, const T* Uin, T* Uout, int slabs_per_block,
                          hipStream_t s);

// Prolongation fused with one smoothing sweep: U' = U_in + P e_c, then
// out = U' + omega D^{-1} (f - A U') (a.U = U_in, may be null; a.out = out).
// Periodic grids with even sizes only (hipErrorNotSupported otherwise).
template <typename T>
hipError_t launch_prolong_smooth(const OpParams& p, int react, const SweepPtrs<T>& a, bool space,
                                 bool time, int ncx, int ncy, int Nc, const T* ec, int chunk,
                                 hipStream_t s);
bool blocked_layout(const OpParams& p);

// Level-0 smoothing sweep fused with the restriction of the swept iterate's
// residual (2D periodic, constant reaction or REACT_COEF with a.coef and the
// coarse coefficients coefc, space coarsening by 2, nx a
// multiple of 64, ny of 16, M <= 4; the smoother's chunks of `chunk` slabs,
// a multiple of the coarse chunk cs): a.out = U + omega C^{-1}(f - A U),
// fc = R (f - A a.out) and, with pc and uc, the coarse level's first sweep
// from zero into uc.  zbuf: smooth_restrict_zbuf elements (one plane per run
// boundary); a.part (may be null): one partial of ||f - A U||^2 per
// workgroup, smooth_restrict_blocks of them.
bool smooth_restrict_ok(const OpParams& p, int react, int ncx, int ncy, int Nc, int chunk, int cs);
int smooth_restrict_blocks(const OpParams& p, int chunk);
size_t smooth_restrict_zbuf(const OpParams& p, int chunk);
template <typename T>
hipError_t launch_smooth_restrict(const OpParams& p, int react, const SweepPtrs<T>& a, int ncx, int ncy, T* fc,
                                  int chunk, const OpParams* pc, T* uc, const T* coefc, int cs, T* zbuf,
                                  hipStream_t s);

// Galerkin levels: r = f - A U (U may be null: zero) into out, and one
// block-Jacobi sweep over chunks of `chunk` slabs (point-diagonal parts of
// the slab blocks: B = K m_0 + diag(db) k_0 and the coupling cin m_0 cout^T).
template <typename T>
hipError_t launch_residual9(const OpParams& p, const Stencil9& st, const T* U, const T* f, T* out,
                            hipStream_t s);
template <typename T>
hipError_t launch_smooth9(const OpParams& p, const Stencil9& st, const T* U, const T* f, T* out, int chunk,
                          hipStream_t s);


// Exact solve of the block lower-bidiagonal coarsest system:
// U_n = Ainv (f_n + cin (x) (cout . U_{n-1}))   (u0 enters slab 0 if given).
template <typename T>
hipError_t launch_coarse_solve(const OpParams& p, const double* Ainv, const T* f,
                               const double* u0, T* U, hipStream_t s);

// Exact coarsest solve by 2D discrete Fourier diagonalization (periodic
// grids, constant reaction, planes that fft_plane_ok takes): Sinv holds
// per mode q (in the storage order of the transforms) the M x M inverse of
// K + diag(db) (lambda_q + lam) ([P][M][M]), tw the twiddles cos, sin of
// 2 pi j / nx (j < nx) then of 2 pi j / ny, work 2 (N M + 1) P doubles.
// f may be null (zero), u0 enters slab 0 if given.
constexpr int kFftMaxPlane = 1024;
// 2D planes whose sides are powers of two of at most kFftRegSide points take
// radix-2 transforms held in registers: a wave holds 64 / n whole lines of n
// points and exchanges butterfly partners by lane shuffles.  Their Fourier
// coefficients are stored column-major in bit-reversed order (storage index
// kx' ny + ky' holds mode (bitrev kx', bitrev ky')), and Sinv follows that order.
constexpr int kFftRegSide = 64;
inline bool fft_pow2(int n) { return n >= 2 && (n & (n - 1)) == 0; }
inline bool fft_reg_plane(int nx, int ny) {
  return ny > 1 && fft_pow2(nx) && fft_pow2(ny) && nx <= kFftRegSide && ny <= kFftRegSide;
}
// Planes the Fourier coarsest solve takes.
inline bool fft_plane_ok(int nx, int ny) { return nx * ny <= kFftMaxPlane || fft_reg_plane(nx, ny); }
// fscale (may be null): per-mode factor applied to the transformed right-hand
// side (a Galerkin coarsest level: 1 / the mass stencil's symbol).
template <typename T>
hipError_t launch_fft_coarse(const OpParams& p, const double* Sinv, const double* tw, double* work,
                             const T* f, const double* u0, T* U, hipStream_t s,
                             const double* fscale = nullptr);
// The same in FP32 arithmetic with FP32 tables (Sinv, tw, fscale as in the
// FP64 solve, rounded) and work space, for the FP32 cycles of mixed
// precision; register-transform planes only (hipErrorNotSupported otherwise).
hipError_t launch_fft_coarse32(const OpParams& p, const float* Sinv, const float* tw, float* work, const float* f,
                               const double* u0, float* U, hipStream_t s, const float* fscale = nullptr);

// Coarsest solve with a different slab matrix per slab: the K x K slab
// matrices (K = M nx ny) are built from the per-DOF coefficient and factored
// in the kernel (dense LU, one workgroup), then the slabs are solved in order.
template <typename T>
hipError_t launch_coarse_solve_coef(const OpParams& p, const T* coef, double* scratch,
                                    const T* f, const double* u0, T* U, hipStream_t s);

// The same, with the per-slab matrices inverted once per linearization:
// W holds N blocks [A_n | A_n^{-1}] (K x 2K each, coarse_inverse_doubles(p)
// doubles).  launch_coarse_invert_coef builds and inverts them (one workgroup
// per slab); launch_coarse_solve_slabs runs the slab recurrence with them.
size_t coarse_inverse_doubles(const OpParams& p);
template <typename T>
hipError_t launch_coarse_invert_coef(const OpParams& p, const T* coef, double* W, hipStream_t s);
template <typename T>
hipError_t launch_coarse_solve_slabs(const OpParams& p, const double* W, const T* f, const double* u0, T* U,
                                     hipStream_t s);

// Coarsest level with a constant slab matrix and at most kScanMaxP points per
// plane: the slab recurrence split into parallel applications of A_s^{-1}
// and a P-vector recurrence p_n = g_n + G p_{n-1} in one wave.  Ainv is
// K x K, G is P x P, H = A_s^{-1} (cin (x) I) is K x P, cout has M entries,
// pg is N x P scratch.
constexpr int kScanMaxP = 64;
struct CoarseScan {
  const double* Ainv = nullptr;
  const double* G = nullptr;
  const double* H = nullptr;
  const double* cout = nullptr;
  double* pg = nullptr;
};
template <typename T>
hipError_t launch_coarse_scan(const OpParams& p, const CoarseScan& cs, const T* f, const double* u0, T* U,
                              hipStream_t s);

// out[0] = sum of part[0..n) in a fixed order (one workgroup).
hipError_t launch_sum_partials(const double* part, int n, double* out, hipStream_t s);

// Sum of squares of a double array into per-block partials.
hipError_t launch_sumsq(const double* x, size_t n, double* part, int* nparts, hipStream_t s);

// y[i] = (TY) (alpha * x[i])
template <typename TX, typename TY>
hipError_t launch_axpy_cast(size_t n, const TX* x, double alpha, TY* y, bool accumulate,
                            hipStream_t s);

// U64 += e32 (or e64)
template <typename TE>
hipError_t launch_update(size_t n, double* U, const TE* e, const double* scale, hipStream_t s);

// Newton coefficient c = gamma (3 U^2 - 1) (the derivative of the
// Allen-Cahn term gamma (u^3 - u)), written as T.
template <typename T>
hipError_t launch_newton_coef(size_t n, const double* U, double gamma, T* coef, hipStream_t s);
// The same coefficient written as FP64 and FP32 in one pass over U.
hipError_t launch_newton_coef_pair(size_t n, const double* U, double gamma, double* c64, float* c32,
                                   hipStream_t s);

// Coefficient on the next coarser level: average of the fine values
// (full-weighting pattern normalized to unit sum in space and time).
template <typename T>
hipError_t launch_restrict_coef(const OpParams& fine, bool space, bool time, int ncx, int ncy,
                                int Nc, const T* cf, T* cc, hipStream_t s);

// Node transfer between collocation node sets, pointwise in slab and space:
// out[n][o][q] = sum_i W[o * Min + i] in[n][i][q]  (W is Mout x Min).
struct NodeMat {
  double W[kMaxM * kMaxM];
};
template <typename T>
hipError_t launch_node_transfer(const T* in, int Min, T* out, int Mout, const NodeMat& W, int N,
                                size_t P, hipStream_t s);

// Reverse the slab order of a [N][M][P] array (out-of-place).
hipError_t launch_reverse_slabs(const double* in, double* out, int N, int M, size_t P,
                                hipStream_t s);

// grad_u0[q] = sum_i w_i lam_slab[i][q]
hipError_t launch_node_combine(const double* lam_slab, const double* w, int M, size_t P,
                               double* out, hipStream_t s);

// Per-block partials of sum_{n,i,q} lam[N-1-n][i][q] * db_i * (Lap U_{n,i})(q) with
// lam stored backward in time (adjoint) and U forward.
hipError_t launch_grad_nu(const OpParams& p, const double* U, const double* lam_rev,
                          double* part, int* nparts, hipStream_t s);

// SDC helpers: in-place r <- G r per point ([N][M][P], G M x M row-major on
// the device); rhs = r[:, m, :] + acc; U[:, m, :] += d and
// acc += w (cx D_xx + cy D_yy - lam) d.
hipError_t launch_node_transform(double* r, int N, int M, int P, const double* G, hipStream_t s);
hipError_t launch_sdc_gather(const double* r, const double* acc, double* rhs, int N, int M, int P,
                             int m, hipStream_t s);
hipError_t launch_sdc_update(double* U, double* acc, const double* d, int N, int M, int nx, int ny,
                             int bc, double cx, double cy, double lam, double w, int m, hipStream_t s);
// The same with an explicit Allen-Cahn reaction R(u) = gamma (u - u^3) (IMEX
// sweep): also acc += we (R(U + d) - R(U)) with U the node's value before the
// update (we = dt (c_{m+1} - c_m), zero after the last node).
hipError_t launch_sdc_update_imex(double* U, double* acc, const double* d, int N, int M, int nx, int ny,
                                  int bc, double cx, double cy, double lam, double w, double gamma,
                                  double we, int m, hipStream_t s);

// Flexible GMRES on level 0 (FP64).  A set of up to kKrylovMax + 1
// vectors of n doubles and one coefficient per vector, both passed by value.
constexpr int kKrylovMax = 32;
constexpr int kKrylovParts = 4096;  // upper bound on the blocks of one Krylov pass
struct KVecs {
  const double* v[kKrylovMax + 1];
};
struct KCoef {
  double c[kKrylovMax + 1];
};
// One Gram-Schmidt pass of w against V_0..V_{k-1} (k <= kKrylovMax + 1;
// w and every V_i 16-byte aligned):
// when d is given, w -= sum_i s.c[i] d[i] V_i (d on the device, typically the
// previous pass's dot products, s the host's 1 / ||V_i||^2); then per-block
// partials of (w, V_i) for i < k (when dots) in part[i * nb + block] and of
// (w, w) in part[k * nb + block].  *nb receives the block count.
hipError_t launch_kortho(double* w, const KVecs& V, int k, const KCoef& s, const double* d, size_t n,
                         bool dots, double* part, int* nb, hipStream_t st);
// out[c] = sum_b part[c * nb + b] for c < cols (fixed order), also written to
// the host-visible mirror when it is given.
hipError_t launch_kreduce(const double* part, int nb, int cols, double* out, double* mirror,
                          hipStream_t st);
// x += sum_{i < k} y.c[i] Z_i
hipError_t launch_kcombine(double* x, const KVecs& Z, int k, const KCoef& y, size_t n, hipStream_t st);

}  // namespace stmg
