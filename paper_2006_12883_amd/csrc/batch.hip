// Batched solve of many independent linear problems (C ABI stmg_batch_*).
//
// Every problem keeps its own level hierarchy (a Solver in batch-member
// mode: FP32 level buffers, register-blocked layout on every level).  One
// refinement step of all problems is a fixed sequence of phase launches, each
// covering every problem that has work in that phase:
//
//   R   FP64 residual b - A U, stored as FP32, with per-block partial sums
//   NRM per-problem norm; a problem whose norm meets its threshold is done
//   S0  level-0 smoothing sweep from zero (FP32)
//   D_l restriction level l -> l+1, fused with the coarse level's first sweep
//   C   coarsest solves (one workgroup per problem)
//   U_l prolongation fused with the first post-smoothing sweep, l -> ... -> 0
//   (S, D_l, C, U_l again for each further FP32 cycle of the step, the level-0
//   sweep starting from the last cycle's e; inner_cycles cycles per step)
//   X   U += e (FP64)
//
// A workgroup finds its (problem, level) work item by binary search over the
// items of its phase and leaves at once if that problem is done.  The step is
// captured once in a HIP graph on the batch's own stream and replayed until
// every problem is done; the host reads back only the done flags and norms.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdlib>
#include <map>
#include <memory>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "launchers.hpp"
#include "solver.hpp"

#define HIP_CHECK_B(expr)                                                        \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return STMG_EHIP;                                                          \
    }                                                                            \
  } while (0)

namespace stmg {

namespace {

struct BItem {
  const OpParams* op;   // operator of this level
  const OpParams* opc;  // operator of the next coarser level
  const double* Ainv;   // coarsest inverse (phase C)
  const void* U;        // iterate
  const void* f;        // right-hand side
  void* out;            // output iterate / residual
  const void* ec;       // coarse correction (phase U)
  void* fc;             // coarse right-hand side (phase D)
  void* uc;             // coarse iterate (phase D with zs)
  double* part;         // partial sums (phase R)
  long long n;          // element count (phase X)
  int ncx, ncy, Nc, S, tiles, tiles_x, nblocks, blk0, cs, prob, M, zs;
};

enum { PH_R, PH_NRM, PH_S0, PH_DS, PH_DT, PH_C, PH_US, PH_UT, PH_X };

__device__ __forceinline__ int find_item(const BItem* __restrict__ it, int n, int b) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (it[mid].blk0 <= b) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

#define BDISPATCH(CALL)                 \
  switch (it.M) {                      \
    case 1: CALL(1); break;            \
    case 2: CALL(2); break;            \
    case 3: CALL(3); break;            \
    case 4: CALL(4); break;            \
    default: break;                    \
  }

__global__ __launch_bounds__(kBlock) void k_b_resid(const BItem* __restrict__ items, int nitems,
                                                    const int* __restrict__ done,
                                                    const double* const* __restrict__ Up,
                                                    const double* const* __restrict__ u0p) {
  const BItem& it = items[find_item(items, nitems, blockIdx.x)];
  if (done[it.prob]) return;
  const int lb = blockIdx.x - it.blk0;
  SweepPtrs<double> a{Up[it.prob], nullptr, u0p[it.prob], nullptr, it.out, it.part};
#define C_(MM) \
  residual_blk_body<MM, double, float, REACT_CONST, 2, true>(*it.op, a, it.S, lb % it.tiles, (lb / it.tiles) * it.S, lb)
  BDISPATCH(C_)
#undef C_
}

// per-problem norm^2 from its partials; done flag is sticky
__global__ __launch_bounds__(kBlock) void k_b_norm(const BItem* __restrict__ items, int* __restrict__ done,
                                                   double* __restrict__ norm2,
                                                   const double* __restrict__ thr) {
  const BItem& it = items[blockIdx.x];
  double s = 0.0;
  for (int i = threadIdx.x; i < it.nblocks; i += kBlock) s += it.part[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) {
    if (!done[it.prob]) {
      norm2[it.prob] = t;
      if (t <= thr[it.prob] || !(t == t)) done[it.prob] = 1;
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_b_smooth0(const BItem* __restrict__ items, int nitems,
                                                      const int* __restrict__ done) {
  const BItem& it = items[find_item(items, nitems, blockIdx.x)];
  if (done[it.prob]) return;
  const int lb = blockIdx.x - it.blk0;
  SweepPtrs<float> a{static_cast<const float*>(it.U), static_cast<const float*>(it.f), nullptr, nullptr, it.out,
                     nullptr};
#define C_(MM) \
  smooth_blk_body<MM, float, REACT_CONST, 2, true>(*it.op, a, it.S, lb % it.tiles, (lb / it.tiles) * it.S, 0)
  BDISPATCH(C_)
#undef C_
}

__global__ __launch_bounds__(kBlock) void k_b_restrict_s(const BItem* __restrict__ items, int nitems,
                                                         const int* __restrict__ done) {
  // restrict_blk_body's tile: M <= 4 nodes x 33 rows x 2 x 17 slots
  __shared__ float lds[4 * 33 * 2 * 17];
  const BItem& it = items[find_item(items, nitems, blockIdx.x)];
  if (done[it.prob]) return;
  const int lb = blockIdx.x - it.blk0;
  SweepPtrs<float> a{static_cast<const float*>(it.U), static_cast<const float*>(it.f), nullptr, nullptr,
                     nullptr, nullptr};
  float* fc = static_cast<float*>(it.fc);
  float* uc = static_cast<float*>(it.uc);
  const int tile = lb % it.tiles, J0 = (lb / it.tiles) * it.S;
#define C_(MM)                                                                                    \
  if (it.zs) restrict_blk_body<MM, float, REACT_CONST, false, true, 16, 16, true>(                 \
      *it.op, a, it.ncx, it.ncy, it.Nc, fc, it.S, it.tiles_x, tile, J0, *it.opc, uc, nullptr, it.cs, lds); \
  else restrict_blk_body<MM, float, REACT_CONST, false, true, 16, 16, false>(                      \
      *it.op, a, it.ncx, it.ncy, it.Nc, fc, it.S, it.tiles_x, tile, J0, *it.op, nullptr, nullptr, it.cs, lds)
  BDISPATCH(C_)
#undef C_
}

__global__ __launch_bounds__(kBlock) void k_b_restrict_t(const BItem* __restrict__ items, int nitems,
                                                         const int* __restrict__ done) {
  const BItem& it = items[find_item(items, nitems, blockIdx.x)];
  if (done[it.prob]) return;
  const int lb = blockIdx.x - it.blk0;
  SweepPtrs<float> a{static_cast<const float*>(it.U), static_cast<const float*>(it.f), nullptr, nullptr,
                     nullptr, nullptr};
  float* fc = static_cast<float*>(it.fc);
  float* uc = static_cast<float*>(it.uc);
  const int tile = lb % it.tiles, J0 = (lb / it.tiles) * it.S;
#define C_(MM)                                                                                   \
  if (it.zs) restrict_t_body<MM, float, REACT_CONST, 2, true, true>(*it.op, a, it.Nc, fc, it.S, tile, J0, \
                                                                     *it.opc, uc, nullptr, it.cs); \
  else restrict_t_body<MM, float, REACT_CONST, 2, true, false>(*it.op, a, it.Nc, fc, it.S, tile, J0,     \
                                                               *it.op, nullptr, nullptr, it.cs)
  BDISPATCH(C_)
#undef C_
}

__global__ __launch_bounds__(kBlock) void k_b_coarse(const BItem* __restrict__ items, int nitems,
                                                     const int* __restrict__ done) {
  const BItem& it = items[blockIdx.x];
  if (done[it.prob]) return;
  coarse_solve_body<float>(*it.op, it.Ainv, static_cast<const float*>(it.f), nullptr,
                           static_cast<float*>(it.out), 0, it.op->N);
}

template <bool SP>
__global__ __launch_bounds__(kBlock) void k_b_prolong(const BItem* __restrict__ items, int nitems,
                                                      const int* __restrict__ done) {
  const BItem& it = items[find_item(items, nitems, blockIdx.x)];
  if (done[it.prob]) return;
  const int lb = blockIdx.x - it.blk0;
  SweepPtrs<float> a{static_cast<const float*>(it.U), static_cast<const float*>(it.f), nullptr, nullptr,
                     it.out, nullptr};
  const float* ec = static_cast<const float*>(it.ec);
#define C_(MM)                                                                                   \
  prolong_smooth_body<MM, float, REACT_CONST, SP, !SP, 2, true>(*it.op, a, it.ncx, it.ncy, it.Nc, ec, \
                                                                it.S, lb % it.tiles, (lb / it.tiles) * it.S, 0)
  BDISPATCH(C_)
#undef C_
}

// U64 += e32, 1024 elements per workgroup
__global__ __launch_bounds__(kBlock) void k_b_update(const BItem* __restrict__ items, int nitems,
                                                     const int* __restrict__ done,
                                                     double* const* __restrict__ Up) {
  const BItem& it = items[find_item(items, nitems, blockIdx.x)];
  if (done[it.prob]) return;
  const long long base = (long long)(blockIdx.x - it.blk0) * 4 * kBlock;
  double* U = Up[it.prob];
  const float* e = static_cast<const float*>(it.ec);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const long long i = base + k * kBlock + threadIdx.x;
    if (i < it.n) U[i] += (double)e[i];
  }
}

__global__ __launch_bounds__(kBlock) void k_b_u0norm(const double* const* __restrict__ u0p,
                                                     const long long* __restrict__ npts,
                                                     double* __restrict__ out) {
  const double* u = u0p[blockIdx.x];
  const long long n = npts[blockIdx.x];
  double s = 0.0;
  for (long long i = threadIdx.x; i < n; i += kBlock) s += u[i] * u[i];
  const double t = block_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = t;
}

}  // namespace

}  // namespace stmg

struct stmg_batch {
  int n = 0;
  std::vector<std::unique_ptr<stmg::Solver>> S;
  stmg_options opt{};
  hipStream_t user = nullptr;
  hipStream_t own = nullptr;
  // device tables (inside the workspace)
  stmg::OpParams* d_ops = nullptr;
  stmg::BItem* d_items = nullptr;
  size_t items_cap = 0;  // entries of d_items
  double* d_part = nullptr;
  double* d_norm2 = nullptr;
  double* d_thr = nullptr;
  double* d_u0n = nullptr;
  int* d_done = nullptr;
  const double** d_u0p = nullptr;
  double** d_Up = nullptr;
  long long* d_npts = nullptr;
  struct Phase {
    int kind, first, count, blocks;
    size_t shm;
  };
  std::vector<Phase> phases;
  std::vector<stmg::BItem> items;
  // slabs per workgroup run of each problem's restriction to level l + 1
  // (autotuned; 0 = the default)
  std::vector<std::vector<int>> tune_S;
  int nparts = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  stmg_batch() = default;
  stmg_batch(const stmg_batch&) = delete;
  stmg_batch& operator=(const stmg_batch&) = delete;
  // releases what setup created, also when setup stops half-way
  ~stmg_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (own) (void)hipStreamDestroy(own);
  }
};

namespace stmg {
namespace {

bool batchable(const stmg_problem& p) {
  return p.dim == 2 && p.bc == STMG_BC_PERIODIC && p.reaction == STMG_REACT_LINEAR && p.M >= 1 &&
         p.M <= 4 && p.nx[0] % 2 == 0 && p.nx[1] % 2 == 0;
}

// Builds the solvers and returns the workspace bytes (ws == nullptr: size only).
int batch_build(stmg_batch* b, int32_t n, const stmg_problem* probs, const stmg_options* o,
                char* ws, size_t* bytes) {
  b->n = n;
  b->opt = *o;
  b->opt.precision = STMG_PREC_MIXED;
  b->opt.mem_budget = 0;
  b->opt.sdc = 0;
  b->opt.coarsen = STMG_COARSEN_AUTO;
  b->opt.form = STMG_FORM_DG;
  b->opt.smoother = STMG_SMOOTH_PBJ;
  b->opt.coarse_op = STMG_COARSE_REDISC;
  b->S.clear();
  Plan pl;
  pl.base = ws;
  for (int p = 0; p < n; ++p) {
    if (!batchable(probs[p])) {
      set_error("batch: problem " + std::to_string(p) +
                " is not a 2D periodic linear problem with even sizes and M <= 4");
      return STMG_EUNSUPPORTED;
    }
    std::unique_ptr<Solver> s(new Solver());
    s->batch_member = true;
    int rc = s->build(&probs[p], &b->opt);
    if (rc) return rc;
    const size_t need = s->plan(nullptr);
    char* base = pl.take<char>(need);
    if (ws) s->plan(base);
    b->S.push_back(std::move(s));
  }
  // operator table: all levels of all problems
  size_t nops = 0;
  for (auto& s : b->S) nops += s->lv.size();
  b->d_ops = pl.take<OpParams>(nops);
  // work items: an upper bound (per problem: R, NRM, S0, X, C, 2 per level,
  // and one level-0 sweep for each further FP32 cycle of a step)
  size_t nit = 0;
  for (auto& s : b->S) nit += 6 + 2 * s->lv.size() + static_cast<size_t>(b->opt.inner_cycles - 1);
  b->d_items = pl.take<BItem>(nit);
  b->items_cap = nit;
  // partials of phase R
  size_t nparts = 0;
  for (auto& s : b->S) {
    const OpParams& op = s->lv[0].op;
    nparts += static_cast<size_t>(smooth_blocks(op, 8));
  }
  b->d_part = pl.take<double>(nparts);
  b->d_norm2 = pl.take<double>(n);
  b->d_thr = pl.take<double>(n);
  b->d_u0n = pl.take<double>(n);
  b->d_done = pl.take<int>(n);
  b->d_u0p = pl.take<const double*>(n);
  b->d_Up = pl.take<double*>(n);
  b->d_npts = pl.take<long long>(n);
  *bytes = pl.off + 256;
  return STMG_OK;
}

// Work item of problem p's restriction from level l to l + 1 (space or time
// kind) with S slabs per workgroup run (0: the default); the caller sets
// blk0.  Returns the item's workgroup count.
int restrict_item(stmg_batch* b, int p, int l, const std::vector<std::vector<const OpParams*>>& opp, int S,
                  BItem* out) {
  Solver& s = *b->S[p];
  const int last = static_cast<int>(s.lv.size()) - 1;
  Level& F = s.lv[l];
  Level& C = s.lv[l + 1];
  BItem x{};
  x.prob = p;
  x.M = s.prob.M;
  x.op = opp[p][l];
  x.opc = opp[p][l + 1];
  x.U = F.A32;
  x.f = F.f32;
  x.fc = C.f32;
  x.zs = (l + 1 < last) ? 1 : 0;
  x.uc = x.zs ? C.A32 : nullptr;
  x.cs = s.chunk_of(l + 1);
  int spb = S > 0 ? S : s.transfer_slabs(l + 1);
  if (spb % x.cs) spb = ((spb + x.cs - 1) / x.cs) * x.cs;
  x.S = spb;
  x.ncx = C.nx;
  x.ncy = C.ny;
  x.Nc = C.N;
  if (F.kind & 1) {
    // 16 x 16 coarse points per workgroup.  The tile shape is not tuned: it
    // decides which fine residuals the single-point halo items compute and
    // which the 2 x 2 blocks do, and the two code paths may round differently.
    x.tiles_x = (C.nx + 15) / 16;
    x.tiles = x.tiles_x * ((C.ny + 15) / 16);
  } else {
    x.tiles = (plane_threads(F.op) + kBlock - 1) / kBlock;
  }
  *out = x;
  return x.tiles * ((C.N + spb - 1) / spb);
}

// Autotuner of the restriction launch shape (slabs per workgroup run, a
// multiple of the coarse level's smoother block, so that the fused coarse
// sweep stays possible; every choice gives bitwise identical results): per
// (level shape, M, coarse chunk) each candidate is timed on one problem's own
// level buffers, the fastest of three timed launches wins, and choices are
// cached in $STMG_TUNE_CACHE under "batch_..." keys.
int batch_autotune(stmg_batch* b, const std::vector<std::vector<const OpParams*>>& opp) {
  b->tune_S.assign(b->n, {});
  const char* path = std::getenv("STMG_TUNE_CACHE");
  std::map<std::string, int> cache;
  if (path) cache = tune_cache_read(path);
  bool dirty = false;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_CHECK_B(hipEventCreate(&e0));
  HIP_CHECK_B(hipEventCreate(&e1));
  struct EvScope {
    hipEvent_t a, b;
    ~EvScope() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); }
  } ev_scope{e0, e1};
  HIP_CHECK_B(hipMemsetAsync(b->d_done, 0, b->n * sizeof(int), b->own));
  for (int p = 0; p < b->n; ++p) {
    Solver& s = *b->S[p];
    const int L = static_cast<int>(s.lv.size());
    b->tune_S[p].assign(L, 0);
    for (int l = 0; l + 1 < L; ++l) {
      const Level& F = s.lv[l];
      const Level& C = s.lv[l + 1];
      const bool space = (F.kind & 1) != 0;
      std::ostringstream k;
      k << "batch_f32_M" << s.prob.M << "_" << F.nx << "x" << F.ny << "x" << F.N << "_k" << F.kind << "_c"
        << s.chunk_of(l + 1) << (l + 2 < L ? "_zs" : "");
      const std::string key = k.str();
      auto hit = cache.find(key);
      if (hit != cache.end() && hit->second > 0) {
        b->tune_S[p][l] = hit->second;
        continue;
      }
      const int cs = s.chunk_of(l + 1);
      float best = 1e30f;
      int best_S = cs;
      {
        for (int mult : {1, 2, 4, 8}) {
          const int S = cs * mult;
          if (S > 64 || (mult > 1 && S > C.N)) break;
          BItem x{};
          const int nb = restrict_item(b, p, l, opp, S, &x);
          x.blk0 = 0;
          x.nblocks = nb;
          HIP_CHECK_B(hipMemcpyAsync(b->d_items, &x, sizeof(BItem), hipMemcpyHostToDevice, b->own));
          float tot = 0.0f;
          for (int rep = 0; rep < 4; ++rep) {
            HIP_CHECK_B(hipEventRecord(e0, b->own));
            if (space)
              hipLaunchKernelGGL(k_b_restrict_s, dim3(nb), dim3(kBlock), 0, b->own, b->d_items, 1, b->d_done);
            else
              hipLaunchKernelGGL(k_b_restrict_t, dim3(nb), dim3(kBlock), 0, b->own, b->d_items, 1, b->d_done);
            HIP_CHECK_B(hipGetLastError());
            HIP_CHECK_B(hipEventRecord(e1, b->own));
            HIP_CHECK_B(hipEventSynchronize(e1));
            float ms = 0.0f;
            HIP_CHECK_B(hipEventElapsedTime(&ms, e0, e1));
            if (rep > 0) tot += ms;  // the first launch warms up
          }
          if (tot < best) { best = tot; best_S = S; }
        }
      }
      b->tune_S[p][l] = best_S;
      cache[key] = best_S;
      dirty = true;
    }
  }
  if (path && dirty) tune_cache_write(path, cache);
  return STMG_OK;
}

int batch_items(stmg_batch* b) {
  std::vector<OpParams> ops;
  std::vector<std::vector<const OpParams*>> opp(b->n);
  for (int p = 0; p < b->n; ++p)
    for (auto& l : b->S[p]->lv) {
      opp[p].push_back(b->d_ops + ops.size());
      ops.push_back(l.op);
    }
  HIP_CHECK_B(hipMemcpyAsync(b->d_ops, ops.data(), ops.size() * sizeof(OpParams), hipMemcpyHostToDevice, b->own));
  if (b->opt.autotune) {
    // the level buffers hold no data yet: zero the ones the candidates read
    for (auto& sp : b->S)
      for (auto& l : sp->lv) {
        if (l.A32) HIP_CHECK_B(hipMemsetAsync(l.A32, 0, l.n * sizeof(float), b->own));
        if (l.f32) HIP_CHECK_B(hipMemsetAsync(l.f32, 0, l.n * sizeof(float), b->own));
      }
    const int rc = batch_autotune(b, opp);
    if (rc) return rc;
  }
  std::vector<BItem>& it = b->items;
  it.clear();
  b->phases.clear();
  int maxL = 0;
  for (auto& s : b->S) maxL = std::max<int>(maxL, static_cast<int>(s->lv.size()));
  auto begin = [&](int kind) { b->phases.push_back({kind, static_cast<int>(it.size()), 0, 0, 0}); };
  auto end = [&]() {
    auto& ph = b->phases.back();
    ph.count = static_cast<int>(it.size()) - ph.first;
    if (ph.count == 0) b->phases.pop_back();
  };
  auto add = [&](BItem x, int nblocks) {
    auto& ph = b->phases.back();
    x.blk0 = ph.blocks;
    x.nblocks = nblocks;
    ph.blocks += nblocks;
    it.push_back(x);
  };
  auto blank = [&](int p, int l) {
    BItem x{};
    x.prob = p;
    x.M = b->S[p]->prob.M;
    x.op = opp[p][l];
    return x;
  };
  // R: FP64 residual -> FP32 f on level 0, partials
  size_t poff = 0;
  begin(PH_R);
  for (int p = 0; p < b->n; ++p) {
    Level& L = b->S[p]->lv[0];
    BItem x = blank(p, 0);
    x.out = L.f32;
    x.S = 8;
    x.tiles = (plane_threads(L.op) + kBlock - 1) / kBlock;
    x.part = b->d_part + poff;
    const int nb = smooth_blocks(L.op, 8);
    poff += nb;
    add(x, nb);
  }
  end();
  // NRM: one workgroup per problem (items reuse the R geometry)
  begin(PH_NRM);
  for (int p = 0; p < b->n; ++p) {
    BItem x = it[b->phases[0].first + p];
    x.blk0 = 0;
    add(x, 1);
    it.back().nblocks = smooth_blocks(b->S[p]->lv[0].op, 8);
  }
  end();
  // S0: level-0 sweep from zero into A32
  begin(PH_S0);
  for (int p = 0; p < b->n; ++p) {
    Solver& s = *b->S[p];
    Level& L = s.lv[0];
    BItem x = blank(p, 0);
    x.f = L.f32;
    x.out = L.A32;
    x.S = s.chunk_of(0);
    x.tiles = (plane_threads(L.op) + kBlock - 1) / kBlock;
    add(x, smooth_blocks(L.op, x.S));
  }
  end();
  // D_l: restrictions; on level l >= 1 the iterate is A32 (from the fused sweep)
  const size_t cyc0 = b->phases.size();  // first phase of the cycle below S0
  for (int l = 0; l + 1 < maxL; ++l) {
    for (int kind : {PH_DS, PH_DT}) {
      begin(kind);
      for (int p = 0; p < b->n; ++p) {
        Solver& s = *b->S[p];
        const int last = static_cast<int>(s.lv.size()) - 1;
        if (l + 1 > last) continue;
        Level& F = s.lv[l];
        Level& C = s.lv[l + 1];
        if ((kind == PH_DS) != ((F.kind & 1) != 0)) continue;
        (void)C;
        const bool tuned = !b->tune_S.empty() && l < static_cast<int>(b->tune_S[p].size());
        BItem x{};
        const int nb = restrict_item(b, p, l, opp, tuned ? b->tune_S[p][l] : 0, &x);
        add(x, nb);
      }
      end();
    }
  }
  // C: coarsest solves into A32 of the last level
  begin(PH_C);
  size_t shm = 0;
  for (int p = 0; p < b->n; ++p) {
    Solver& s = *b->S[p];
    const int last = static_cast<int>(s.lv.size()) - 1;
    Level& C = s.lv[last];
    BItem x = blank(p, last);
    x.Ainv = s.Ainv;
    x.f = C.f32;
    x.out = C.A32;
    const size_t P = static_cast<size_t>(C.nx) * C.ny;
    shm = std::max(shm, (2 * s.prob.M * P + P) * sizeof(double));
    add(x, 1);
  }
  b->phases.back().shm = shm;
  end();
  // U_l: prolongation + first post-sweep, level l result into B32
  for (int l = maxL - 2; l >= 0; --l) {
    for (int kind : {PH_US, PH_UT}) {
      begin(kind);
      for (int p = 0; p < b->n; ++p) {
        Solver& s = *b->S[p];
        const int last = static_cast<int>(s.lv.size()) - 1;
        if (l + 1 > last) continue;
        Level& F = s.lv[l];
        Level& C = s.lv[l + 1];
        if ((kind == PH_US) != ((F.kind & 1) != 0)) continue;
        BItem x = blank(p, l);
        x.U = F.A32;
        x.f = F.f32;
        x.out = F.B32;
        x.ec = (l + 1 == last) ? C.A32 : C.B32;
        x.S = s.chunk_of(l);
        x.ncx = C.nx;
        x.ncy = C.ny;
        x.Nc = C.N;
        x.tiles = (plane_threads(F.op) + kBlock - 1) / kBlock;
        add(x, smooth_blocks(F.op, x.S));
      }
      end();
    }
  }
  // further FP32 cycles of the step on the same correction equation: a
  // level-0 sweep from the last cycle's e (B32) into A32, then the same
  // restriction, coarsest and prolongation phases again
  const size_t ncycle = b->phases.size() - cyc0;
  for (int k = 1; k < b->opt.inner_cycles; ++k) {
    begin(PH_S0);
    for (int p = 0; p < b->n; ++p) {
      Solver& s = *b->S[p];
      if (s.lv.size() == 1) continue;  // the exact solve does not use the iterate
      Level& L = s.lv[0];
      BItem x = blank(p, 0);
      x.U = L.B32;
      x.f = L.f32;
      x.out = L.A32;
      x.S = s.chunk_of(0);
      x.tiles = (plane_threads(L.op) + kBlock - 1) / kBlock;
      add(x, smooth_blocks(L.op, x.S));
    }
    end();
    for (size_t q = 0; q < ncycle; ++q) {
      const auto ph = b->phases[cyc0 + q];
      b->phases.push_back(ph);
    }
  }
  // X: U += e (level-0 result in B32)
  begin(PH_X);
  for (int p = 0; p < b->n; ++p) {
    Level& L = b->S[p]->lv[0];
    BItem x = blank(p, 0);
    // single-level problems end with the coarsest solve's result in A32
    x.ec = b->S[p]->lv.size() == 1 ? L.A32 : L.B32;
    x.n = static_cast<long long>(L.n);
    add(x, static_cast<int>((L.n + 4 * kBlock - 1) / (4 * kBlock)));
  }
  end();
  b->nparts = static_cast<int>(poff);
  if (it.size() > b->items_cap) {
    set_error("batch: work item table overflow");
    return STMG_EINVAL;
  }
  HIP_CHECK_B(hipMemcpyAsync(b->d_items, it.data(), it.size() * sizeof(BItem), hipMemcpyHostToDevice, b->own));
  std::vector<long long> npts(b->n);
  for (int p = 0; p < b->n; ++p) npts[p] = static_cast<long long>(b->S[p]->lv[0].nx) * b->S[p]->lv[0].ny;
  HIP_CHECK_B(hipMemcpyAsync(b->d_npts, npts.data(), npts.size() * sizeof(long long), hipMemcpyHostToDevice, b->own));
  HIP_CHECK_B(hipStreamSynchronize(b->own));
  return STMG_OK;
}

// One refinement step of all problems (the sequence captured in the graph).
hipError_t batch_step(stmg_batch* b) {
  const hipStream_t s = b->own;
  for (const auto& ph : b->phases) {
    const BItem* items = b->d_items + ph.first;
    switch (ph.kind) {
      case PH_R:
        hipLaunchKernelGGL(k_b_resid, dim3(ph.blocks), dim3(kBlock), 0, s, items, ph.count, b->d_done,
                           b->d_Up, b->d_u0p);
        break;
      case PH_NRM:
        hipLaunchKernelGGL(k_b_norm, dim3(ph.count), dim3(kBlock), 0, s, items, b->d_done, b->d_norm2,
                           b->d_thr);
        break;
      case PH_S0:
        hipLaunchKernelGGL(k_b_smooth0, dim3(ph.blocks), dim3(kBlock), 0, s, items, ph.count, b->d_done);
        break;
      case PH_DS:
        hipLaunchKernelGGL(k_b_restrict_s, dim3(ph.blocks), dim3(kBlock), 0, s, items, ph.count, b->d_done);
        break;
      case PH_DT:
        hipLaunchKernelGGL(k_b_restrict_t, dim3(ph.blocks), dim3(kBlock), 0, s, items, ph.count, b->d_done);
        break;
      case PH_C:
        hipLaunchKernelGGL(k_b_coarse, dim3(ph.count), dim3(kBlock), ph.shm, s, items, ph.count, b->d_done);
        break;
      case PH_US:
        hipLaunchKernelGGL(k_b_prolong<true>, dim3(ph.blocks), dim3(kBlock), 0, s, items, ph.count, b->d_done);
        break;
      case PH_UT:
        hipLaunchKernelGGL(k_b_prolong<false>, dim3(ph.blocks), dim3(kBlock), 0, s, items, ph.count, b->d_done);
        break;
      case PH_X:
        hipLaunchKernelGGL(k_b_update, dim3(ph.blocks), dim3(kBlock), 0, s, items, ph.count, b->d_done, b->d_Up);
        break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace
}  // namespace stmg

using stmg::Solver;

extern "C" {

size_t stmg_batch_workspace_bytes(int32_t n, const stmg_problem* probs, const stmg_options* opt) {
  if (n < 1 || !probs) { stmg::set_error("bad batch"); return 0; }
  stmg_options d;
  if (!opt) { stmg_default_options(&d); opt = &d; }
  stmg_batch b;
  size_t bytes = 0;
  if (stmg::batch_build(&b, n, probs, opt, nullptr, &bytes) != STMG_OK) return 0;
  return bytes;
}

int stmg_batch_setup(int32_t n, const stmg_problem* probs, const stmg_options* opt, void* d_ws,
                     size_t ws_bytes, void* stream, stmg_batch** out) {
  if (n < 1 || !probs || !d_ws || !out) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) { stmg::set_error("workspace alignment"); return STMG_EINVAL; }
  stmg_options d;
  if (!opt) { stmg_default_options(&d); opt = &d; }
  std::unique_ptr<stmg_batch> b(new (std::nothrow) stmg_batch);
  if (!b) return STMG_ENOMEM;
  size_t need = 0;
  int rc = stmg::batch_build(b.get(), n, probs, opt, nullptr, &need);
  if (rc) return rc;
  if (ws_bytes < need) {
    stmg::set_error("batch workspace too small: need " + std::to_string(need) + " bytes");
    return STMG_ENOMEM;
  }
  rc = stmg::batch_build(b.get(), n, probs, opt, static_cast<char*>(d_ws), &need);
  if (rc) return rc;
  b->user = static_cast<hipStream_t>(stream);
  if (hipStreamCreateWithFlags(&b->own, hipStreamNonBlocking) != hipSuccess) {
    stmg::set_error("batch: stream creation failed");
    return STMG_EHIP;
  }
  for (auto& s : b->S) {
    s->stream = b->own;
    rc = s->upload();
    if (rc) return rc;
  }
  rc = stmg::batch_items(b.get());
  if (rc) return rc;
  // capture one refinement step
  if (hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    stmg::set_error("batch: graph capture failed to start");
    return STMG_EHIP;
  }
  hipError_t e = stmg::batch_step(b.get());
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(b->own, &g);
  b->graph = g;
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    stmg::set_error(std::string("batch: graph capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2));
    return STMG_EHIP;
  }
  if (hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0) != hipSuccess) {
    stmg::set_error("batch: graph instantiation failed");
    return STMG_EHIP;
  }
  *out = b.release();
  return STMG_OK;
}

int stmg_batch_solve(stmg_batch* b, const double* const* d_u0, double* const* d_U, stmg_stats* stats) {
  if (!b || !d_u0 || !d_U) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  const auto t0 = std::chrono::steady_clock::now();
  const int n = b->n;
  // inputs written on the caller's stream are complete before we start
  if (hipStreamSynchronize(b->user) != hipSuccess) { stmg::set_error("batch: stream sync"); return STMG_EHIP; }
  std::vector<const double*> u0p(d_u0, d_u0 + n);
  std::vector<double*> Up(d_U, d_U + n);
  hipStream_t s = b->own;
  if (hipMemcpyAsync(b->d_u0p, u0p.data(), n * sizeof(double*), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b->d_Up, Up.data(), n * sizeof(double*), hipMemcpyHostToDevice, s) != hipSuccess) {
    stmg::set_error("batch: pointer upload failed");
    return STMG_EHIP;
  }
  hipLaunchKernelGGL(stmg::k_b_u0norm, dim3(n), dim3(stmg::kBlock), 0, s, b->d_u0p, b->d_npts, b->d_u0n);
  std::vector<double> u0n(n), thr(n), norm2(n, 0.0);
  std::vector<int> done(n, 0), prevdone(n, 0), cycles(n, 0);
  if (hipMemcpyAsync(u0n.data(), b->d_u0n, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess) {
    stmg::set_error("batch: norm readback failed");
    return STMG_EHIP;
  }
  std::vector<double> nb(n);
  for (int p = 0; p < n; ++p) {
    long double w = 0.0L;
    for (int i = 0; i < b->S[p]->prob.M; ++i) w += b->S[p]->tab.l0[i] * b->S[p]->tab.l0[i];
    nb[p] = std::sqrt(static_cast<double>(w) * u0n[p]);
    const double t = b->opt.rtol * nb[p];
    thr[p] = t * t;
  }
  if (hipMemcpyAsync(b->d_thr, thr.data(), n * sizeof(double), hipMemcpyHostToDevice, s) != hipSuccess ||
      hipMemcpyAsync(b->d_done, done.data(), n * sizeof(int), hipMemcpyHostToDevice, s) != hipSuccess) {
    stmg::set_error("batch: upload failed");
    return STMG_EHIP;
  }
  int steps = 0;
  int status = STMG_OK;
  for (;;) {
    if (hipGraphLaunch(b->exec, s) != hipSuccess) { stmg::set_error("batch: graph launch failed"); return STMG_EHIP; }
    if (hipMemcpyAsync(done.data(), b->d_done, n * sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipMemcpyAsync(norm2.data(), b->d_norm2, n * sizeof(double), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess) {
      stmg::set_error("batch: readback failed");
      return STMG_EHIP;
    }
    ++steps;
    int all = 1;
    for (int p = 0; p < n; ++p) {
      if (!done[p]) { ++cycles[p]; all = 0; }
    }
    if (all) break;
    if (static_cast<long long>(steps) * b->opt.inner_cycles > b->opt.max_cycles) {
      status = STMG_ENOTCONV;
      break;
    }
  }
  const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (stats) {
    for (int p = 0; p < n; ++p) {
      stmg_stats st{};
      st.cycles = cycles[p] * b->opt.inner_cycles;
      st.refinements = cycles[p];
      st.rel_res = nb[p] > 0 ? std::sqrt(norm2[p]) / nb[p] : std::sqrt(norm2[p]);
      st.status = !std::isfinite(st.rel_res) ? STMG_ENAN : (done[p] ? STMG_OK : STMG_ENOTCONV);
      st.seconds = secs;
      stats[p] = st;
    }
  }
  if (status) stmg::set_error("batch: max_cycles reached before every problem converged");
  return status;
}

void stmg_batch_destroy(stmg_batch* b) { delete b; }

}  // extern "C"
