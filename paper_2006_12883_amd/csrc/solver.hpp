// Host-side solver state behind the C ABI (internal to libstmg).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "../../include/stmg.h"
#include "kernels.hpp"
#include "tables.hpp"

namespace stmg {

void set_error(const std::string& msg);

// Autotuner cache: a flat JSON object {"key": integer} (file named by
// $STMG_TUNE_CACHE).
std::map<std::string, int> tune_cache_read(const char* path);
void tune_cache_write(const char* path, const std::map<std::string, int>& m);

struct Level {
  int nx = 0, ny = 1;  // grid points
  int ex = 0, ey = 1;  // elements (Neumann) / points (periodic), for h
  int N = 0;
  int M = 0;           // collocation nodes (lowered by node coarsening)
  double dt = 0.0, hx = 0.0, hy = 1.0;
  int kind = 0;        // coarsening to the next level: bits 1 space, 2 time, 4 nodes
  // node coarsening to the next level: prolongation Pn (M x M_next) and
  // restriction Rn = Pn^T, and the coarse-grid buffers with this level's M
  // that carry the transfers between the two node sets
  NodeMat Pn{}, Rn{};
  double* nt64 = nullptr;
  float* nt32 = nullptr;
  size_t n = 0;        // N * M * nx * ny
  OpParams op{}, opT{};
  // FP64 buffers (level 0: A is the caller's iterate, B is workspace)
  double *A64 = nullptr, *B64 = nullptr, *f64 = nullptr, *coef64 = nullptr;
  // FP32 buffers (mixed precision)
  float *A32 = nullptr, *B32 = nullptr, *f32 = nullptr, *coef32 = nullptr;
  // Galerkin coarse level (option coarse_op): its stencils and a level-sized
  // temporary (the residual before restriction, the prolonged iterate before
  // smoothing)
  bool g9 = false;
  Stencil9 st{};
  double* g64 = nullptr;
  float* g32 = nullptr;
};

// Byte-offset planner over one device buffer.
struct Plan {
  char* base = nullptr;
  size_t off = 0;
  template <typename T>
  T* take(size_t count) {
    off = (off + 255) & ~static_cast<size_t>(255);
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

// Pinned host slot and event for reading a device scalar without draining
// the stream (created on first use, on the device current at that time).
// Kernels write the slot through its device alias `d`, so no copy is queued.
struct HostScalar {
  double* h = nullptr;
  double* d = nullptr;
  size_t cap = 0;  // doubles
  hipEvent_t ev = nullptr;
  HostScalar() = default;
  HostScalar(const HostScalar&) = delete;
  HostScalar& operator=(const HostScalar&) = delete;
  ~HostScalar() {
    if (ev) (void)hipEventDestroy(ev);
    if (h) (void)hipHostFree(h);
  }
  hipError_t init(size_t count = 1) {
    if (h && cap < count) {
      // callers only grow the slot count before queuing work that uses it
      (void)hipHostFree(h);
      h = nullptr;
      d = nullptr;
      cap = 0;
    }
    if (!h) {
      hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&h), count * sizeof(double),
                                   hipHostMallocMapped | hipHostMallocCoherent);
      if (e != hipSuccess) { h = nullptr; return e; }
      cap = count;
      e = hipHostGetDevicePointer(reinterpret_cast<void**>(&d), h, 0);
      if (e != hipSuccess) return e;
    }
    if (!ev) {
      hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
      if (e != hipSuccess) { ev = nullptr; return e; }
    }
    return hipSuccess;
  }
};

struct Solver {
  stmg_problem prob{};
  stmg_options opt{};
  hipStream_t stream = nullptr;
  RadauTables tab{};                 // M of the problem (finest level)
  RadauTables mtab[kMaxM + 1]{};     // per node count (node coarsening), built on demand
  bool mtab_ok[kMaxM + 1] = {};
  const RadauTables* tables_for(int m);
  std::vector<Level> lv;
  bool allen_cahn = false;
  bool linearized = false;  // Allen-Cahn: a Newton step has set the Jacobian coefficients
  bool mixed = false;
  bool fuse = true;  // fused restriction+presmooth / prolongation+postsmooth kernels
  size_t ws_bytes = 0;
  // shared device scratch
  double* part = nullptr;   // per-block partial sums
  int max_parts = 0;
  double* scal = nullptr;   // device scalars
  double* Ainv = nullptr;   // coarsest slab inverse (forward)
  double* AinvT = nullptr;  // (transposed problem)
  double* coarse_scratch = nullptr;  // dense slab matrix for the Newton coarsest solve
  // Dense coarsest level with few points per plane and many slabs: the split
  // recurrence (forward and transposed problem); empty when not used
  CoarseScan scan{}, scanT{};
  // Newton coarsest level: the inverted slab matrices of the current
  // linearization (null when they would exceed kCoarseInvMaxBytes; the
  // coarsest solve then factors slab after slab inside the cycle)
  double* coarse_inv = nullptr;
  // Coarsest level solved by Fourier diagonalization (periodic grids, constant
  // reaction): per-mode M x M inverses, twiddles, complex workspace.
  bool fft = false;
  double* fft_sinv = nullptr;   // [P][M][M] (forward problem)
  double* fft_sinvT = nullptr;  // (transposed problem)
  double* fft_tw = nullptr;
  double* fft_work = nullptr;   // 2 (N M + 1) P
  double* fft_mscale = nullptr; // Galerkin coarsest level: 1 / mass symbol per mode
  // the same tables rounded to FP32 and an FP32 workspace, for the FP32
  // cycles of mixed precision on register-transform planes
  bool fft32 = false;
  float *fft_sinv32 = nullptr, *fft_sinvT32 = nullptr, *fft_tw32 = nullptr, *fft_work32 = nullptr,
        *fft_mscale32 = nullptr;
  double* delta64 = nullptr;  // Newton correction / adjoint multiplier (level 0, FP64)
  // Flexible GMRES (opt.krylov = m > 0): m + 1 basis vectors and m + 1
  // direction buffers (one spare for the V-cycle's ping-pong) on level 0,
  // block partials, and the dot products of the Gram-Schmidt passes on the
  // device (kdev) with a host-visible mirror (kh), both laid out as
  // [restart norm | pass 1 | pass 2 | pass 3], kKrylovMax + 2 slots a pass.
  double* kV = nullptr;
  double* kZ = nullptr;
  size_t kstride = 0;  // doubles between consecutive vectors (256-byte multiple)
  double* kpart = nullptr;
  double* kdev = nullptr;
  HostScalar kh;
  double* lw = nullptr;       // M weights l(0) on the device (gradient of u0)
  double* form_G = nullptr;   // Q diag(b)^-1 on the device (collocation-form residual output)
  // statistics of the last solve
  stmg_stats last{};
  // Stop test of the linear solve: the residual norm of the incoming iterate
  // is copied to pinned memory behind an event; the host waits on that event
  // only after the cycle's level-0 restriction is queued (gate0 is called
  // there by vcycle and may end the cycle, leaving the iterate untouched), so
  // the device never idles while the host decides.
  HostScalar hnorm;
  std::function<hipError_t(bool*)> gate0;
  // Mixed precision: when set, the level-0 FP32 prolongation + smoothing also
  // writes up_out = up_in + (its FP32 result) in FP64 (the refinement update)
  // and sets up_done.
  const double* up_in = nullptr;
  double* up_out = nullptr;
  bool up_done = false;
  // Level-0 pre-smoothing fused with the residual restriction
  // (launch_smooth_restrict): possible for this hierarchy (sr), its run
  // boundary planes, and the hand-over from the FP64 solve's norm sweep to
  // the cycle (sr_pending: the sweep in the cycle's iterate buffer has also
  // restricted; sr_smoothed: with the coarse first sweep).
  bool sr = false;
  double* sr_z64 = nullptr;
  float* sr_z32 = nullptr;
  bool sr_pending = false;
  bool sr_smoothed = false;

  // Time windows (adjoint checkpointing).  When the options' memory budget
  // cannot hold the trajectory, the handle drives a sub-solver for W slabs
  // (and one for the shorter last window): A is block lower-triangular, so
  // solving window after window, each started from the previous window's end
  // value, is exact.  Only window start values (checkpoints) are kept.
  int win_W = 0;        // 0: no windows
  int nwin = 0;
  std::unique_ptr<Solver> win, win_last;
  double* ckpt = nullptr;  // start value of window w >= 1, plane w
  double* Uw = nullptr;    // one window's trajectory
  double* gw = nullptr;    // two planes: coupling passed backward between windows
  Solver* sub(int w) { return (w == nwin - 1 && win_last) ? win_last.get() : win.get(); }
  int window_len(int w) const { return (w == nwin - 1) ? prob.N - (nwin - 1) * win_W : win_W; }
  int solve_end(const double* u0, double* uT, stmg_stats* st);

  // Independent slabs (no time coupling, space coarsening only): the
  // Helmholtz solves of the SDC sweep.
  bool decoupled = false;
  // Member of a batch: FP32 level buffers only, and space coarsening only
  // while the coarse grid keeps an even point count (register-blocked
  // kernels on every level).
  bool batch_member = false;
  // SDC: one M = 1 sub-solver per collocation node (operator
  // I - dt dc_m L on every slab), the accumulated explicit part, Q diag(b)^-1.
  std::vector<std::unique_ptr<Solver>> sdcn;
  double* sdc_acc = nullptr;
  double* sdc_G = nullptr;
  double sdc_w[kMaxM] = {0};  // dt * (c_m - c_{m-1})

  // PFASST (option pfasst_levels): the levels below level 0, each with M = 1
  // and half the elements of the one above; per level its iterate, FAS
  // right-hand side, the restricted pair (z, end values) from the level
  // above, its initial value and an M = 1 solver (independent slabs on the
  // intermediate levels, the coupled system on the coarsest).
  struct PfLevel {
    int nx = 0, ny = 1;
    double* V = nullptr;
    double* tau = nullptr;
    double* rhs = nullptr;
    double* pack = nullptr;  // [N][2][P]: R_s z, R_s V_M of the level above
    double* u0 = nullptr;
    std::unique_ptr<Solver> sol;
    bool serial = false;  // sol is a one-slab solver (the IMEX serial sweep)
  };
  std::vector<PfLevel> pf;
  double* pf_pack = nullptr;  // [N][2][P] on the finer level of a transfer
  double* pf_E = nullptr;     // [N][M][P] corrections on the coarser grid
  int pfasst(const double* u0, double* U, stmg_stats* st);
  // > 0 while PFASST runs with options.pfasst_inner_cycles: the cap on the
  // V-cycles of each inner solve (reaching it is not an error there)
  int inner_cap = 0;
  int inner_solve(Solver* S, const double* f, const double* u0, double* U, double norm_b);

  // --- setup ---
  int build(const stmg_problem* p, const stmg_options* o);
  size_t plan(char* ws);  // lays out (or sizes, ws = nullptr) the workspace
  int upload();           // copies tables into the workspace
  int upload_fft();       // tables of the Fourier coarsest solve
  int upload_dense();     // dense inverse of the coarsest slab matrix
  int galerkin_levels();  // Galerkin stencils and point blocks of the coarse levels

  int chunk_of(int l) const;        // smoother block length on level l
  int transfer_slabs(int l) const;  // slabs per thread in transfer kernels
  std::vector<int> tuned;           // autotuned transfer_slabs per level (0: default)
  int autotune();                   // time candidate shapes, keep the fastest
  // --- building blocks (FP64 or FP32 arithmetic) ---
  template <typename T>
  hipError_t smooth(int l, bool adj, int react, const T* U, const T* f, const double* u0, T* out);
  // f_c = R (f - A U); with uc also the coarse level's first smoothing sweep
  // from zero into uc when possible (*smoothed reports it).
  template <typename T>
  hipError_t restrict_residual(int l, bool adj, int react, const T* U, const T* f,
                               const double* u0, T* fc, T* uc = nullptr, bool* smoothed = nullptr);
  // Level 0: one smoothing sweep U -> out fused with f_c = R (f - A out)
  // (uc: the coarse first sweep), part: per-workgroup ||f - A U||^2 or null.
  bool sr_usable(int react, bool fp64) const;
  template <typename T>
  hipError_t smooth_restrict(bool adj, int react, const T* U, const T* f, const double* u0, T* out, T* fc, T* uc,
                             double* part_out, bool* smoothed);
  template <typename T>
  hipError_t prolong_smooth(int l, bool adj, int react, const T* Uin, const T* ec, const T* f,
                            const double* u0, T* out);
  template <typename T>
  hipError_t prolong(int l, const T* Uin, const T* ec, T* Uout);
  template <typename T>
  hipError_t coarse(bool adj, int react, const T* f, const double* u0, T* U);
  // One V-cycle on level l; `cur` holds the iterate (ignored if zero), `oth`
  // is the ping-pong partner; the result pointer is returned in *res.
  // skip_pre: pre-smoothing sweeps on level l already done by the caller.
  template <typename T>
  hipError_t vcycle(int l, bool adj, int react, T* cur, T* oth, const T* f, const double* u0,
                    bool zero, T** res, int skip_pre);

  // ||f + u0-coupling - A U||^2 on level 0 (FP64), optional store into r (TO).
  template <typename TO>
  hipError_t residual64(bool adj, int react, const double* U, const double* f,
                        const double* u0, TO* r, double* d_out);
  long long residual_parts() const;  // per-block partial sums residual64 writes
  int read_scalar(const double* d, double* h);

  // --- drivers ---
  int solve_linear(bool adj, int react, const double* f, const double* u0, double* U,
                   double rtol, double norm_b, int* cycles, double* rel, int* refinements = nullptr);
  int solve_fgmres(bool adj, int react, const double* f, const double* u0, double* U, double rtol,
                   double norm_b, int* cycles, double* rel);
  int solve(const double* u0, double* U, stmg_stats* st);
  int vcycle_user(const double* u0, double* U, double* h_rel);
  int residual_user(const double* u0, const double* U, double* r, double* h_norm);
  int adjoint(const double* u0, const double* U, const double* gT, double* grad_u0,
              double* grad_nu, stmg_stats* st);
  int sdc(const double* u0, double* U, int sweeps, double* h_rel);
  int sdc_core(const double* u0, double* U, int sweeps);  // the sweeps, no norm

  int newton_linearize(const double* U);  // coefficients on every level
  double norm_u0_b(const double* u0);     // ||b|| for b = l(0) (x) u0
};

}  // namespace stmg
