// Solver setup, V-cycle and solve drivers (host side of libstmg).
#include "solver.hpp"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <limits>
#include <map>
#include <sstream>

namespace stmg {

namespace {

constexpr int kResidSlabs = 8;   // slabs per thread in residual sweeps
constexpr size_t kCoarseInvMaxBytes = size_t(1) << 30;  // Newton coarsest inverses
constexpr int kScanMinSlabs = 32;  // shorter coarsest levels keep the one-kernel recurrence
constexpr int kTransferSlabs = 4;
constexpr int kInnerMax = 64;  // inner_cycles bound
constexpr double kGrowth = 1.1;  // divergence test: per-cycle growth that counts

// Elements -> points per dimension.
int points(int e, int bc) { return bc == STMG_BC_PERIODIC ? e : e + 1; }

}  // namespace

// Cap on the V-cycles of an inner solve (SDC node solves, PFASST level
// solves), which stop at rtol relative to their first residual.
constexpr int kInnerMaxCycles = 200;

#define HIP_TRY(expr)                                                            \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return e_;                                                                 \
    }                                                                            \
  } while (0)

#define HIP_CHECK(expr)                                                          \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      set_error(std::string("HIP error in ") + #expr + ": " + hipGetErrorString(e_)); \
      return STMG_EHIP;                                                          \
    }                                                                            \
  } while (0)

const RadauTables* Solver::tables_for(int m) {
  if (m < 1 || m > kMaxM) return nullptr;
  if (!mtab_ok[m]) {
    if (!radau_tables(m, &mtab[m])) return nullptr;
    mtab_ok[m] = true;
  }
  return &mtab[m];
}

// ---------------------------------------------------------------------------
// Hierarchy.  Semi-coarsening by the anisotropy ratio mu = nu dt / h^2
// (Sec. 4.2: coarsen in time when mu << 1 and in space when mu >> 1), with the
// SMG (space only) and STMG (space and time) variants of Sec. 5.2.
int Solver::build(const stmg_problem* p, const stmg_options* o) {
  prob = *p;
  opt = *o;
  if (p->dim != 1 && p->dim != 2) { set_error("dim must be 1 or 2"); return STMG_EINVAL; }
  if (p->M < 1 || p->M > kMaxM) { set_error("M must be in 1..8"); return STMG_EINVAL; }
  if (p->N < 1) { set_error("N must be >= 1"); return STMG_EINVAL; }
  if (!(p->dt > 0.0)) { set_error("dt must be > 0"); return STMG_EINVAL; }
  if (!(p->nu > 0.0)) { set_error("nu must be > 0"); return STMG_EINVAL; }
  if (p->bc != STMG_BC_PERIODIC && p->bc != STMG_BC_NEUMANN) { set_error("bad bc"); return STMG_EINVAL; }
  if (p->reaction != STMG_REACT_LINEAR && p->reaction != STMG_REACT_ALLEN_CAHN) {
    set_error("bad reaction");
    return STMG_EINVAL;
  }
  const int ex = p->nx[0], ey = p->dim == 2 ? p->nx[1] : 1;
  if (points(ex, p->bc) < 3 || (p->dim == 2 && points(ey, p->bc) < 3)) {
    set_error("need at least 3 grid points per dimension");
    return STMG_EINVAL;
  }
  if (!(p->length[0] > 0.0) || (p->dim == 2 && !(p->length[1] > 0.0))) {
    set_error("length must be > 0");
    return STMG_EINVAL;
  }
  if (o->chunk < 1 || o->chunk_coarse < 1 || o->nu_pre < 0 || o->nu_post < 0 || o->nu_pre + o->nu_post < 1 ||
      o->max_levels < 1 || o->max_cycles < 1 || !(o->rtol > 0.0) || !(o->omega > 0.0) ||
      o->inner_cycles < 1 || o->inner_cycles > kInnerMax || o->fft_coarse < 0 || o->krylov < 0 || o->krylov > kKrylovMax ||
      o->krylov_left < 0 || o->krylov_left > 1 || o->inner_adapt < 0 || o->inner_adapt > 1) {
    set_error("invalid options");
    return STMG_EINVAL;
  }
  if (o->precision != STMG_PREC_FP64 && o->precision != STMG_PREC_MIXED) {
    set_error("bad precision");
    return STMG_EINVAL;
  }
  if (o->form != STMG_FORM_DG && o->form != STMG_FORM_COLLOC) { set_error("bad form"); return STMG_EINVAL; }
  if (o->smoother != STMG_SMOOTH_PBJ && o->smoother != STMG_SMOOTH_SDC) {
    set_error("bad smoother");
    return STMG_EINVAL;
  }
  if (o->coarse_op != STMG_COARSE_REDISC && o->coarse_op != STMG_COARSE_GALERKIN) {
    set_error("bad coarse_op");
    return STMG_EINVAL;
  }
  if (o->coarse_op == STMG_COARSE_GALERKIN &&
      (o->coarsen != STMG_COARSEN_SPACE || p->bc != STMG_BC_PERIODIC ||
       p->reaction != STMG_REACT_LINEAR || batch_member)) {
    set_error("Galerkin coarse operators: space coarsening of periodic linear problems only");
    return STMG_EUNSUPPORTED;
  }
  if (o->form == STMG_FORM_COLLOC && o->krylov > 0) {
    set_error("collocation-form residuals with the Krylov method are not supported");
    return STMG_EUNSUPPORTED;
  }
  allen_cahn = p->reaction == STMG_REACT_ALLEN_CAHN;
  mixed = o->precision == STMG_PREC_MIXED;
  if (!radau_tables(p->M, &tab)) { set_error("Radau table construction failed"); return STMG_EINVAL; }
  if (o->coarsen == STMG_COARSEN_SMMG && allen_cahn) {
    set_error("SMMG coarsening: linear problems only");
    return STMG_EUNSUPPORTED;
  }
  if (o->coarsen < STMG_COARSEN_AUTO || o->coarsen > STMG_COARSEN_SMMG) {
    set_error("bad coarsen");
    return STMG_EINVAL;
  }

  const int M = p->M;
  const bool twod = p->dim == 2;
  lv.clear();
  Level L;
  L.ex = ex;
  L.ey = ey;
  L.nx = points(ex, p->bc);
  L.ny = twod ? points(ey, p->bc) : 1;
  L.N = p->N;
  L.M = M;
  L.dt = p->dt;
  lv.push_back(L);
  // Periodic grids with a constant reaction can stop at a larger coarsest
  // level: its exact solve by Fourier diagonalization costs two small DFTs
  // per plane, while the levels below it would be latency-bound launches.
  const bool fft_ok = p->bc == STMG_BC_PERIODIC && !allen_cahn && !batch_member;
  while (static_cast<int>(lv.size()) < o->max_levels) {
    Level& c = lv.back();
    if (static_cast<long long>(c.M) * c.nx * c.ny * c.N <= o->min_coarse) break;
    if (fft_ok && lv.size() > 1 && fft_plane_ok(c.nx, c.ny) &&
        static_cast<long long>(c.M) * c.nx * c.ny * c.N <= o->fft_coarse)
      break;
    const int q = batch_member ? 4 : 2;
    const bool cs_x = (c.ex % q == 0) && c.ex >= 4;
    const bool cs_y = !twod || ((c.ey % q == 0) && c.ey >= 4);
    const bool can_s = cs_x && cs_y;
    const bool can_t = c.N % 2 == 0 && !decoupled;
    const double hx = p->length[0] / c.ex;
    const double hy = twod ? p->length[1] / c.ey : hx;
    const double hmin = hx < hy ? hx : hy;
    const double mu = p->nu * c.dt / (hmin * hmin);
    int kind = 0;
    if (o->coarsen == STMG_COARSEN_SPACE) {
      kind = can_s ? 1 : 0;
    } else if (o->coarsen == STMG_COARSEN_SMMG) {
      kind = can_s ? (c.M > 1 ? 1 | 4 : 1) : 0;
    } else if (o->coarsen == STMG_COARSEN_SPACETIME) {
      kind = (can_s && can_t) ? 3 : (can_s ? 1 : (can_t ? 2 : 0));
    } else {
      if (mu >= o->mu_crit && can_s) kind = 1;
      else if (can_t) kind = 2;
      else if (can_s) kind = 1;
    }
    if (kind == 0) break;
    c.kind = kind;
    Level nl;
    nl.ex = (kind & 1) ? c.ex / 2 : c.ex;
    nl.ey = (kind & 1) && twod ? c.ey / 2 : c.ey;
    nl.nx = points(nl.ex, p->bc);
    nl.ny = twod ? points(nl.ey, p->bc) : 1;
    nl.N = (kind & 2) ? c.N / 2 : c.N;
    nl.M = (kind & 4) ? c.M - 1 : c.M;
    nl.dt = (kind & 2) ? 2.0 * c.dt : c.dt;
    if (kind & 4) {
      // Lagrange basis of the coarse Radau nodes at the fine ones
      const RadauTables* tf = tables_for(c.M);
      const RadauTables* tc = tables_for(nl.M);
      if (!tf || !tc) { set_error("Radau table construction failed"); return STMG_EINVAL; }
      for (int i = 0; i < c.M; ++i)
        for (int k = 0; k < nl.M; ++k) {
          long double v = 1.0L;
          for (int j = 0; j < nl.M; ++j)
            if (j != k) v *= (tf->c[i] - tc->c[j]) / (tc->c[k] - tc->c[j]);
          c.Pn.W[i * nl.M + k] = static_cast<double>(v);
          c.Rn.W[k * c.M + i] = static_cast<double>(v);
        }
    }
    lv.push_back(nl);
  }
  const Level& last = lv.back();
  const long long Kc = static_cast<long long>(last.M) * last.nx * last.ny;
  fft = fft_ok && fft_plane_ok(last.nx, last.ny);
  fft32 = fft && mixed && fft_reg_plane(last.nx, last.ny);
  if (!fft && Kc > 1024) {
    set_error("coarsest level has more than 1024 unknowns per slab");
    return STMG_EUNSUPPORTED;
  }

  // Operators per level (each with its own node count and tables).
  for (auto& l : lv) {
    l.hx = p->length[0] / l.ex;
    l.hy = twod ? p->length[1] / l.ey : 1.0;
    l.n = static_cast<size_t>(l.N) * l.M * l.nx * l.ny;
    const RadauTables* lt = tables_for(l.M);
    if (!lt) { set_error("Radau table construction failed"); return STMG_EINVAL; }
    const RadauTables& tab = *lt;
    const int M = l.M;
    OpParams op{};
    op.M = M;
    op.nx = l.nx;
    op.ny = l.ny;
    op.N = l.N;
    op.bc = p->bc == STMG_BC_PERIODIC ? 0 : 1;
    op.cx = p->nu / (l.hx * l.hx);
    op.cy = twod ? p->nu / (l.hy * l.hy) : 0.0;
    op.lam = allen_cahn ? 0.0 : p->lambda;
    op.gamma = allen_cahn ? p->gamma : 0.0;
    op.omega = o->omega;
    OpParams opT = op;
    const long double dg = 2.0L * op.cx + 2.0L * op.cy + op.lam;
    std::vector<long double> B(static_cast<size_t>(M) * M), BT(static_cast<size_t>(M) * M);
    for (int i = 0; i < M; ++i) {
      op.db[i] = static_cast<double>(l.dt * tab.b[i]);
      opT.db[i] = op.db[i];
      op.cin[i] = decoupled ? 0.0 : static_cast<double>(tab.l0[i]);
      op.cout[i] = (i == M - 1 && !decoupled) ? 1.0 : 0.0;
      opT.cin[i] = op.cout[i];
      opT.cout[i] = op.cin[i];
      for (int j = 0; j < M; ++j) {
        op.K[i * M + j] = static_cast<double>(tab.Kq[i][j]);
        opT.K[i * M + j] = static_cast<double>(tab.Kq[j][i]);
        B[static_cast<size_t>(i) * M + j] = tab.Kq[i][j] + (i == j ? l.dt * tab.b[i] * dg : 0.0L);
        BT[static_cast<size_t>(i) * M + j] = tab.Kq[j][i] + (i == j ? l.dt * tab.b[i] * dg : 0.0L);
      }
    }
    if (!invert_ld(B, M) || !invert_ld(BT, M)) { set_error("singular point block"); return STMG_EINVAL; }
    for (int i = 0; i < M * M; ++i) {
      op.Binv[i] = static_cast<double>(B[i]);
      opT.Binv[i] = static_cast<double>(BT[i]);
    }
    // collocation form of the residual norms (finest level, forward problem)
    if (&l == &lv[0] && o->form == STMG_FORM_COLLOC) {
      op.colloc = 1;
      for (int i = 0; i < M; ++i)
        for (int j = 0; j < M; ++j) op.G[i * M + j] = static_cast<double>(tab.Q[i][j] / tab.b[j]);
    }
    l.op = op;
    l.opT = opT;
  }
  if (o->coarse_op == STMG_COARSE_GALERKIN && lv.size() > 1) {
    if (!fft) {
      set_error("Galerkin coarse operators need a Fourier-solvable coarsest plane");
      return STMG_EUNSUPPORTED;
    }
    int rc = galerkin_levels();
    if (rc) return rc;
  }
  // SDC node solvers
  sdcn.clear();
  if (o->smoother == STMG_SMOOTH_SDC &&
      (allen_cahn || o->precision != STMG_PREC_FP64 || o->krylov > 0 || batch_member || decoupled)) {
    set_error("SDC smoother: FP64 linear problems without the Krylov method only");
    return STMG_EUNSUPPORTED;
  }
  if (o->pfasst_levels != 0 &&
      (o->pfasst_levels < 2 || o->pfasst_levels > 8 || o->pfasst_sweeps < 1 || o->pfasst_sweeps > 16 ||
       o->pfasst_inner_cycles < 0 || o->pfasst_inner_cycles > 100)) {
    set_error("pfasst_levels must be 0 or 2..8, pfasst_sweeps 1..16, pfasst_inner_cycles 0..100");
    return STMG_EINVAL;
  }
  if (o->pfasst_levels >= 2 && (o->precision != STMG_PREC_FP64 || o->krylov > 0 || batch_member || decoupled)) {
    set_error("PFASST: FP64 without the Krylov method only");
    return STMG_EUNSUPPORTED;
  }
  if ((o->sdc || o->smoother == STMG_SMOOTH_SDC || o->pfasst_levels >= 2) && !decoupled) {
    // node solves with the implicit (linear) part only: an Allen-Cahn reaction
    // is explicit in the sweep (IMEX)
    for (int m = 0; m < M; ++m) {
      const long double dc = tab.c[m] - (m > 0 ? tab.c[m - 1] : 0.0L);
      sdc_w[m] = static_cast<double>(p->dt * dc);
      stmg_problem sp = *p;
      sp.M = 1;
      sp.dt = sdc_w[m];
      sp.reaction = STMG_REACT_LINEAR;
      sp.gamma = 0.0;
      stmg_options so = *o;
      so.sdc = 0;
      so.pfasst_levels = 0;
      so.mem_budget = 0;
      so.krylov = 0;
      so.max_cycles = std::max(o->max_cycles, kInnerMaxCycles);
      so.precision = STMG_PREC_FP64;
      so.coarsen = STMG_COARSEN_SPACE;
      so.smoother = STMG_SMOOTH_PBJ;
      so.form = STMG_FORM_DG;
      std::unique_ptr<Solver> sub(new Solver());
      sub->decoupled = true;
      int rc = sub->build(&sp, &so);
      if (rc) return rc;
      sdcn.push_back(std::move(sub));
    }
  }
  // PFASST levels: bisection in space, M = 1
  pf.clear();
  if (o->pfasst_levels >= 2 && !decoupled) {
    int ex = lv[0].ex, ey = lv[0].ey;
    for (int l = 1; l < o->pfasst_levels; ++l) {
      if (ex % 2 != 0 || ex / 2 < 2 || (twod && (ey % 2 != 0 || ey / 2 < 2))) {
        set_error("PFASST: element counts must stay even down to at least 2 per dimension");
        return STMG_EINVAL;
      }
      ex /= 2;
      if (twod) ey /= 2;
      stmg_problem sp = *p;
      sp.nx[0] = ex;
      sp.nx[1] = twod ? ey : 1;
      sp.M = 1;
      sp.reaction = STMG_REACT_LINEAR;  // the reaction stays explicit (IMEX)
      sp.gamma = 0.0;
      stmg_options so = *o;
      so.pfasst_levels = 0;
      so.sdc = 0;
      so.mem_budget = 0;
      so.krylov = 0;
      so.max_cycles = std::max(o->max_cycles, kInnerMaxCycles);
      so.precision = STMG_PREC_FP64;
      so.smoother = STMG_SMOOTH_PBJ;
      so.form = STMG_FORM_DG;
      so.coarse_op = STMG_COARSE_REDISC;
      PfLevel q;
      q.sol.reset(new Solver());
      if (l + 1 < o->pfasst_levels) {
        so.coarsen = STMG_COARSEN_SPACE;
        q.sol->decoupled = true;
      } else if (allen_cahn) {
        // the serial IMEX sweep solves slab after slab: a one-slab solver,
        // exact in one level where the plane allows (Fourier or dense)
        sp.N = 1;
        q.serial = true;
        const int px = p->bc == STMG_BC_PERIODIC ? ex : ex + 1;
        const int py = twod ? (p->bc == STMG_BC_PERIODIC ? ey : ey + 1) : 1;
        if ((p->bc == STMG_BC_PERIODIC && fft_plane_ok(px, py)) || px * py <= 1024) so.max_levels = 1;
      }
      int rc = q.sol->build(&sp, &so);
      if (rc) return rc;
      q.nx = q.sol->lv[0].nx;
      q.ny = q.sol->lv[0].ny;
      pf.push_back(std::move(q));
    }
  }
  // Windows: the FP64 path keeps about five full vectors on level 0 (the
  // caller's U, ping-pong, right-hand side, Newton/adjoint vector and the
  // adjoint's own ping-pong), plus 2 (m + 1) with the Krylov method.
  win_W = 0;
  nwin = 0;
  win.reset();
  win_last.reset();
  const size_t P = static_cast<size_t>(lv[0].nx) * lv[0].ny;
  const size_t slab = static_cast<size_t>(M) * P * sizeof(double);
  const size_t vecs = 5 + (o->krylov > 0 ? 2 * static_cast<size_t>(o->krylov + 1) : 0);
  if (o->mem_budget > 0 && vecs * slab * static_cast<size_t>(p->N) > o->mem_budget) {
    long long W = static_cast<long long>(o->mem_budget / ((vecs + 1) * slab));
    if (W < 1) W = 1;
    // largest power of two not above the budget, so windows coarsen in time
    long long w2 = 1;
    while (w2 * 2 <= W) w2 *= 2;
    W = w2;
    if (W < p->N) {
      if (!pf.empty()) {
        set_error("PFASST needs the whole trajectory in memory (mem_budget too small)");
        return STMG_EUNSUPPORTED;
      }
      sdcn.clear();  // SDC sweeps act on the whole trajectory
      win_W = static_cast<int>(W);
      nwin = (p->N + win_W - 1) / win_W;
      stmg_options so = *o;
      so.mem_budget = 0;
      stmg_problem sp = *p;
      sp.N = win_W;
      win.reset(new Solver());
      int rc = win->build(&sp, &so);
      if (rc) return rc;
      const int lastN = p->N - (nwin - 1) * win_W;
      if (lastN != win_W) {
        sp.N = lastN;
        win_last.reset(new Solver());
        rc = win_last->build(&sp, &so);
        if (rc) return rc;
      }
    }
  }
  return STMG_OK;
}

size_t Solver::plan(char* ws) {
  Plan pl;
  pl.base = ws;
  if (batch_member) {
    for (auto& l : lv) {
      l.A32 = pl.take<float>(l.n);
      l.B32 = pl.take<float>(l.n);
      l.f32 = pl.take<float>(l.n);
    }
    max_parts = 1024;
    part = pl.take<double>(1024);
    scal = pl.take<double>(32);
    const Level& c = lv.back();
    const size_t K = static_cast<size_t>(prob.M) * c.nx * c.ny;
    Ainv = pl.take<double>(K * K);
    AinvT = pl.take<double>(K * K);
    lw = pl.take<double>(kMaxM);
    form_G = pl.take<double>(kMaxM * kMaxM);
    return pl.off + 256;
  }
  if (win) {
    // windowed handle: the sub-solvers' workspaces, checkpoints, one window
    const size_t P = static_cast<size_t>(lv[0].nx) * lv[0].ny;
    const size_t wb = win->plan(nullptr);
    char* wbase = pl.take<char>(wb);
    win->plan(wbase);
    if (win_last) {
      const size_t lb = win_last->plan(nullptr);
      char* lbase = pl.take<char>(lb);
      win_last->plan(lbase);
    }
    ckpt = pl.take<double>(static_cast<size_t>(nwin) * P);
    Uw = pl.take<double>(static_cast<size_t>(win_W) * prob.M * P);
    gw = pl.take<double>(2 * P);
    return pl.off + 256;
  }
  for (size_t i = 0; i < lv.size(); ++i) {
    Level& l = lv[i];
    if ((l.kind & 4) && i + 1 < lv.size()) {
      const Level& c = lv[i + 1];
      const size_t nt = static_cast<size_t>(c.N) * l.M * c.nx * c.ny;
      l.nt64 = pl.take<double>(nt);
      if (mixed) l.nt32 = pl.take<float>(nt);
    }
    if (i > 0) l.A64 = pl.take<double>(l.n);
    l.B64 = pl.take<double>(l.n);
    l.f64 = pl.take<double>(l.n);
    if (mixed) {
      l.A32 = pl.take<float>(l.n);
      l.B32 = pl.take<float>(l.n);
      l.f32 = pl.take<float>(l.n);
    }
    if (allen_cahn) {
      if (i == 0 || !mixed) l.coef64 = pl.take<double>(l.n);
      if (mixed) l.coef32 = pl.take<float>(l.n);
    }
    if (l.g9) {
      l.g64 = pl.take<double>(l.n);
      if (mixed) l.g32 = pl.take<float>(l.n);
    }
  }
  delta64 = pl.take<double>(lv[0].n);
  if (opt.krylov > 0) {
    const size_t vecs = static_cast<size_t>(opt.krylov) + 1;
    kstride = (lv[0].n + 31) & ~static_cast<size_t>(31);
    kV = pl.take<double>(vecs * kstride);
    kZ = pl.take<double>(vecs * kstride);
    kpart = pl.take<double>(static_cast<size_t>(kKrylovParts) * (kKrylovMax + 2));
    kdev = pl.take<double>(1 + 3 * (kKrylovMax + 2));
  }
  // level-0 pre-smoothing fused with the restriction: space coarsening by
  // two of a 2D periodic level whose tiles cover the coarse grid, linear
  // constant reaction, the point-block smoother on both levels
  sr = false;
  if (lv.size() >= 2) {
    const Level& l = lv[0];
    const Level& c = lv[1];
    sr = fuse && !l.g9 && !c.g9 && (l.kind & 1) && !(l.kind & 2) && !(l.kind & 4) &&
         smooth_restrict_ok(l.op, REACT_CONST, c.nx, c.ny, c.N, chunk_of(0), chunk_of(1)) &&
         smooth_restrict_ok(l.opT, REACT_CONST, c.nx, c.ny, c.N, chunk_of(0), chunk_of(1));
    if (sr) {
      const size_t zn = smooth_restrict_zbuf(l.op, chunk_of(0));
      sr_z64 = zn ? pl.take<double>(zn) : nullptr;
      sr_z32 = (zn && mixed) ? pl.take<float>(zn) : nullptr;
    }
  }
  // partial sums: the largest residual launch is on level 0
  {
    const Level& l = lv[0];
    const int tiles = (l.nx * l.ny + kBlock - 1) / kBlock;
    const int chunks = (l.N + kResidSlabs - 1) / kResidSlabs;
    max_parts = tiles * chunks;
    const int sb = smooth_blocks(l.op, chunk_of(0));
    if (max_parts < sb) max_parts = sb;
    if (sr && max_parts < smooth_restrict_blocks(l.op, chunk_of(0))) max_parts = smooth_restrict_blocks(l.op, chunk_of(0));
    if (max_parts < 1024) max_parts = 1024;
  }
  part = pl.take<double>(static_cast<size_t>(max_parts));
  scal = pl.take<double>(32);
  const Level& c = lv.back();
  const size_t K = static_cast<size_t>(c.M) * c.nx * c.ny;
  if (fft) {
    const size_t Pc = static_cast<size_t>(c.nx) * c.ny;
    fft_sinv = pl.take<double>(Pc * c.M * c.M);
    fft_sinvT = pl.take<double>(Pc * c.M * c.M);
    fft_tw = pl.take<double>(2 * (static_cast<size_t>(c.nx) + c.ny));
    fft_work = pl.take<double>(2 * (static_cast<size_t>(c.N) * c.M + 1) * Pc);
    if (c.g9) fft_mscale = pl.take<double>(Pc);
    if (fft32) {
      fft_sinv32 = pl.take<float>(Pc * c.M * c.M);
      fft_sinvT32 = pl.take<float>(Pc * c.M * c.M);
      fft_tw32 = pl.take<float>(2 * (static_cast<size_t>(c.nx) + c.ny));
      fft_work32 = pl.take<float>(2 * (static_cast<size_t>(c.N) * c.M + 1) * Pc);
      if (c.g9) fft_mscale32 = pl.take<float>(Pc);
    }
  } else {
    Ainv = pl.take<double>(K * K);
    AinvT = pl.take<double>(K * K);
  }
  coarse_scratch = allen_cahn ? pl.take<double>(K * K) : nullptr;
  scan = CoarseScan{};
  scanT = CoarseScan{};
  if (!fft && !decoupled && !batch_member && static_cast<int>(c.nx * c.ny) <= kScanMaxP && c.N >= kScanMinSlabs) {
    const size_t Pc = static_cast<size_t>(c.nx) * c.ny;
    double* g = pl.take<double>(Pc * Pc);
    double* h = pl.take<double>(K * Pc);
    double* gT = pl.take<double>(Pc * Pc);
    double* hT = pl.take<double>(K * Pc);
    double* co = pl.take<double>(2 * kMaxM);
    double* pg = pl.take<double>(static_cast<size_t>(c.N) * Pc);
    if (ws) {
      scan = CoarseScan{Ainv, g, h, co, pg};
      scanT = CoarseScan{AinvT, gT, hT, co + kMaxM, pg};
    }
  }
  coarse_inv = nullptr;
  if (allen_cahn && !batch_member) {
    const size_t d = coarse_inverse_doubles(c.op);
    if (d * sizeof(double) <= kCoarseInvMaxBytes) coarse_inv = pl.take<double>(d);
  }
  lw = pl.take<double>(kMaxM);
  form_G = pl.take<double>(kMaxM * kMaxM);
  if (!sdcn.empty()) {
    for (auto& sub : sdcn) {
      const size_t b = sub->plan(nullptr);
      sub->plan(pl.take<char>(b));
    }
    sdc_acc = pl.take<double>(static_cast<size_t>(lv[0].N) * lv[0].nx * lv[0].ny);
    sdc_G = pl.take<double>(kMaxM * kMaxM);
  }
  if (!pf.empty()) {
    const size_t N = static_cast<size_t>(lv[0].N);
    pf_pack = pl.take<double>(N * 2 * lv[0].nx * lv[0].ny);
    pf_E = pl.take<double>(N * prob.M * pf[0].nx * pf[0].ny);
    for (auto& q : pf) {
      const size_t P = static_cast<size_t>(q.nx) * q.ny;
      q.V = pl.take<double>(N * P);
      q.tau = pl.take<double>(N * P);
      q.rhs = pl.take<double>(N * P);
      q.pack = pl.take<double>(N * 2 * P);
      q.u0 = pl.take<double>(P);
      const size_t b = q.sol->plan(nullptr);
      q.sol->plan(pl.take<char>(b));
    }
  }
  return pl.off + 256;
}

// Tables of the Fourier coarsest solve: per mode q = (kx, ky) the inverses of
// Kq + diag(dt b) (lambda_q + lambda) and of its transpose (the transposed
// problem), lambda_q = cx (2 - 2 cos(2 pi kx / nx)) + cy (2 - 2 cos(2 pi ky / ny)),
// in long double; the DFT twiddles cos, sin of 2 pi j / n.
// Galerkin coarse levels (space coarsening, periodic): the 3 x 3 mass and
// stiffness stencils of A_{l+1} = R A_l P, obtained by applying R S P to a
// coarse delta on a small periodic grid (16 x 16 fine points; bilinear P,
// full weighting R = P^T / 2^d) in long double, starting from Ms = I and
// Ks = -nu Lap_h + lambda on the finest level; and the point-block inverses
// (K m_0 + diag(db) k_0)^-1 of the smoother.
int Solver::galerkin_levels() {
  const bool twod = prob.dim == 2;
  constexpr int nc = 8, nf = 16;
  const int nyc = twod ? nc : 1, nyf = twod ? nf : 1;
  long double ms[9] = {0}, ks[9] = {0};
  ms[4] = 1.0L;
  {
    const Level& L0 = lv[0];
    const long double cx = L0.op.cx, cy = L0.op.cy, lam = L0.op.lam;
    ks[4] = 2.0L * cx + (twod ? 2.0L * cy : 0.0L) + lam;
    ks[3] = ks[5] = -cx;
    if (twod) ks[1] = ks[7] = -cy;
  }
  auto rap = [&](const long double* sf, long double* out) -> bool {
    // coarse delta at (4, 4) (1D: x = 4), prolongated, stencil, restricted
    std::vector<long double> ec(static_cast<size_t>(nc) * nyc, 0.0L), uf(static_cast<size_t>(nf) * nyf, 0.0L),
        vf(uf.size(), 0.0L), rc(ec.size(), 0.0L);
    const int X0 = 4, Y0 = twod ? 4 : 0;
    ec[static_cast<size_t>(Y0) * nc + X0] = 1.0L;
    auto cval = [&](int X, int Y) { return ec[static_cast<size_t>(((Y % nyc) + nyc) % nyc) * nc + ((X % nc) + nc) % nc]; };
    for (int y = 0; y < nyf; ++y)
      for (int x = 0; x < nf; ++x) {
        // bilinear: average of the coarse points around fine (x, y)
        const int X = x / 2, Y = twod ? y / 2 : 0;
        const bool ox = x & 1, oy = twod && (y & 1);
        long double v = cval(X, Y);
        if (ox && oy) v = 0.25L * (cval(X, Y) + cval(X + 1, Y) + cval(X, Y + 1) + cval(X + 1, Y + 1));
        else if (ox) v = 0.5L * (cval(X, Y) + cval(X + 1, Y));
        else if (oy) v = 0.5L * (cval(X, Y) + cval(X, Y + 1));
        uf[static_cast<size_t>(y) * nf + x] = v;
      }
    auto fval = [&](const std::vector<long double>& a, int x, int y) {
      return a[static_cast<size_t>(((y % nyf) + nyf) % nyf) * nf + ((x % nf) + nf) % nf];
    };
    for (int y = 0; y < nyf; ++y)
      for (int x = 0; x < nf; ++x) {
        long double v = 0.0L;
        for (int k = 0; k < 9; ++k) {
          const int dx = k % 3 - 1, dy = k / 3 - 1;
          if (!twod && dy != 0) continue;
          v += sf[k] * fval(uf, x + dx, y + dy);
        }
        vf[static_cast<size_t>(y) * nf + x] = v;
      }
    const long double w1[3] = {0.25L, 0.5L, 0.25L};
    for (int Y = 0; Y < nyc; ++Y)
      for (int X = 0; X < nc; ++X) {
        long double v = 0.0L;
        for (int dy = -1; dy <= 1; ++dy) {
          if (!twod && dy != 0) continue;
          for (int dx = -1; dx <= 1; ++dx)
            v += (twod ? w1[dy + 1] : 1.0L) * w1[dx + 1] * fval(vf, 2 * X + dx, 2 * Y + dy);
        }
        rc[static_cast<size_t>(Y) * nc + X] = v;
      }
    // (A delta_{X0})(X) = s[X0 - X]: read the 3 x 3 neighbourhood, require zeros outside
    long double outside = 0.0L, total = 0.0L;
    for (int Y = 0; Y < nyc; ++Y)
      for (int X = 0; X < nc; ++X) {
        const long double v = rc[static_cast<size_t>(Y) * nc + X];
        const int dx = X0 - X, dy = Y0 - Y;
        total += std::fabs(v);
        if (std::abs(dx) <= 1 && std::abs(dy) <= 1) out[(dy + 1) * 3 + dx + 1] = v;
        else outside += std::fabs(v);
      }
    return outside <= 1e-15L * total;
  };
  for (size_t l = 1; l < lv.size(); ++l) {
    if (lv[l - 1].kind != 1) {
      set_error("Galerkin coarse operators: space coarsening only");
      return STMG_EUNSUPPORTED;
    }
    long double m2[9] = {0}, k2[9] = {0};
    if (!rap(ms, m2) || !rap(ks, k2)) { set_error("Galerkin stencil is not 3 x 3"); return STMG_EINVAL; }
    for (int k = 0; k < 9; ++k) {
      ms[k] = m2[k];
      ks[k] = k2[k];
    }
    Level& L = lv[l];
    L.g9 = true;
    for (int k = 0; k < 9; ++k) {
      L.st.m[k] = static_cast<double>(ms[k]);
      L.st.k[k] = static_cast<double>(ks[k]);
    }
    const RadauTables* lt = tables_for(L.M);
    if (!lt) { set_error("Radau table construction failed"); return STMG_EINVAL; }
    const int M = L.M;
    std::vector<long double> B(static_cast<size_t>(M) * M), BT(static_cast<size_t>(M) * M);
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) {
        const long double d = (i == j) ? static_cast<long double>(L.dt) * lt->b[i] * ks[4] : 0.0L;
        B[static_cast<size_t>(i) * M + j] = lt->Kq[i][j] * ms[4] + d;
        BT[static_cast<size_t>(i) * M + j] = lt->Kq[j][i] * ms[4] + d;
      }
    if (!invert_ld(B, M) || !invert_ld(BT, M)) { set_error("singular Galerkin point block"); return STMG_EINVAL; }
    for (int i = 0; i < M * M; ++i) {
      L.op.Binv[i] = static_cast<double>(B[i]);
      L.opT.Binv[i] = static_cast<double>(BT[i]);
    }
    // damping: the point block keeps only the mass stencil's centre m_0, so
    // on a spatially smooth error the sweep's step is omega sum|m| / m_0;
    // scaling omega by m_0 / sum|m| gives that mode the step omega of a
    // rediscretized level (identity mass)
    long double msum = 0.0L;
    for (int k = 0; k < 9; ++k) msum += std::fabs(ms[k]);
    L.op.omega = static_cast<double>(static_cast<long double>(L.op.omega) * ms[4] / msum);
    L.opT.omega = L.op.omega;
  }
  return STMG_OK;
}

int Solver::upload_fft() {
  const Level& c = lv.back();
  const int M = c.M, nx = c.nx, ny = c.ny, P = nx * ny;
  const RadauTables* lt = tables_for(M);
  if (!lt) { set_error("Radau table construction failed"); return STMG_EINVAL; }
  const RadauTables& tab = *lt;
  const long double twopi = 6.283185307179586476925286766559L;
  const OpParams& op = c.op;
  std::vector<double> S(static_cast<size_t>(P) * M * M), ST(static_cast<size_t>(P) * M * M);
  std::vector<double> mscale(c.g9 ? static_cast<size_t>(P) : 0);
  std::vector<long double> a(static_cast<size_t>(M) * M);
  // storage order of the modes: row-major (ky, kx), or for the register
  // transforms the kept half kx = 0 .. nx/2 in compact columns c (kx < nx/2:
  // c = bitrev(kx) / 2; kx = nx/2: c = nx/2), ky bit-reversed: c ny + ky'
  const bool reg = fft_reg_plane(nx, ny);
  auto brev = [](int i, int n) {
    int r = 0;
    for (int b = 1; b < n; b <<= 1) r = (r << 1) | ((i & b) ? 1 : 0);
    return r;
  };
  for (int ky = 0; ky < ny; ++ky)
    for (int kx = 0; kx < nx; ++kx) {
      if (reg && kx > nx / 2) continue;  // conjugate of a kept mode
      const int q = reg ? (kx < nx / 2 ? brev(kx, nx) / 2 : nx / 2) * ny + brev(ky, ny) : ky * nx + kx;
      long double lq = static_cast<long double>(op.cx) * (2.0L - 2.0L * std::cos(twopi * kx / nx));
      if (ny > 1) lq += static_cast<long double>(op.cy) * (2.0L - 2.0L * std::cos(twopi * ky / ny));
      lq += static_cast<long double>(op.lam);
      if (c.g9) {
        // Galerkin level: multiplied through by the mass stencil's inverse
        // (symbols real: the stencils are symmetric), the slab coupling is
        // pointwise again, the spatial symbol is khat / mhat and the
        // transformed right-hand side is scaled by 1 / mhat (fft_mscale)
        long double mh = 0.0L, kh = 0.0L;
        for (int k = 0; k < 9; ++k) {
          const int dx = k % 3 - 1, dy = k / 3 - 1;
          if (ny == 1 && dy != 0) continue;
          const long double ph = twopi * (static_cast<long double>(kx) * dx / nx +
                                          (ny > 1 ? static_cast<long double>(ky) * dy / ny : 0.0L));
          mh += static_cast<long double>(c.st.m[k]) * std::cos(ph);
          kh += static_cast<long double>(c.st.k[k]) * std::cos(ph);
        }
        if (!(mh > 0.0L)) { set_error("Galerkin mass symbol not positive"); return STMG_EINVAL; }
        lq = kh / mh;
        mscale[q] = static_cast<double>(1.0L / mh);
      }
      for (int tr = 0; tr < 2; ++tr) {
        for (int i = 0; i < M; ++i)
          for (int j = 0; j < M; ++j) {
            long double v = tr ? tab.Kq[j][i] : tab.Kq[i][j];
            if (i == j) v += c.dt * tab.b[i] * lq;
            a[static_cast<size_t>(i) * M + j] = v;
          }
        if (!invert_ld(a, M)) { set_error("singular Fourier mode matrix"); return STMG_EINVAL; }
        double* dst = (tr ? ST.data() : S.data()) + static_cast<size_t>(q) * M * M;
        for (int i = 0; i < M * M; ++i) dst[i] = static_cast<double>(a[i]);
      }
    }
  std::vector<double> tw(2 * (static_cast<size_t>(nx) + ny));
  for (int j = 0; j < nx; ++j) {
    tw[2 * j] = static_cast<double>(std::cos(twopi * j / nx));
    tw[2 * j + 1] = static_cast<double>(std::sin(twopi * j / nx));
  }
  for (int j = 0; j < ny; ++j) {
    tw[2 * (nx + j)] = static_cast<double>(std::cos(twopi * j / ny));
    tw[2 * (nx + j) + 1] = static_cast<double>(std::sin(twopi * j / ny));
  }
  HIP_CHECK(hipMemcpyAsync(fft_sinv, S.data(), S.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipMemcpyAsync(fft_sinvT, ST.data(), ST.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipMemcpyAsync(fft_tw, tw.data(), tw.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  if (c.g9)
    HIP_CHECK(hipMemcpyAsync(fft_mscale, mscale.data(), mscale.size() * sizeof(double), hipMemcpyHostToDevice,
                             stream));
  std::vector<float> S32, ST32, tw32, ms32;
  if (fft32) {
    auto cast = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
    S32 = cast(S);
    ST32 = cast(ST);
    tw32 = cast(tw);
    ms32 = cast(mscale);
    HIP_CHECK(hipMemcpyAsync(fft_sinv32, S32.data(), S32.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(fft_sinvT32, ST32.data(), ST32.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(fft_tw32, tw32.data(), tw32.size() * sizeof(float), hipMemcpyHostToDevice, stream));
    if (c.g9)
      HIP_CHECK(hipMemcpyAsync(fft_mscale32, ms32.data(), ms32.size() * sizeof(float), hipMemcpyHostToDevice,
                               stream));
  }
  HIP_CHECK(hipStreamSynchronize(stream));  // host vectors go out of scope
  return STMG_OK;
}

// Dense inverse of the coarsest slab matrix K (x) I + diag(db) (x) (-Lap + lambda)
// (and its transpose, for the transposed problem), in long double.
int Solver::upload_dense() {
  const Level& c = lv.back();
  const int M = c.M, P = c.nx * c.ny, K = M * P;
  const RadauTables* lt = tables_for(M);
  if (!lt) { set_error("Radau table construction failed"); return STMG_EINVAL; }
  const RadauTables& tab = *lt;
  std::vector<long double> A(static_cast<size_t>(K) * K, 0.0L);
  const OpParams& op = c.op;
  auto lo = [&](int i, int n) { return i > 0 ? i - 1 : (op.bc == 0 ? n - 1 : 1); };
  auto hi = [&](int i, int n) { return i < n - 1 ? i + 1 : (op.bc == 0 ? 0 : n - 2); };
  for (int i = 0; i < M; ++i)
    for (int q = 0; q < P; ++q) {
      const int r = i * P + q;
      for (int j = 0; j < M; ++j) A[static_cast<size_t>(r) * K + j * P + q] += tab.Kq[i][j];
      const int x = q % c.nx, y = q / c.nx;
      const long double db = c.dt * tab.b[i];
      auto add = [&](int q2, long double v) { A[static_cast<size_t>(r) * K + i * P + q2] += db * v; };
      add(q, 2.0L * op.cx + (c.ny > 1 ? 2.0L * op.cy : 0.0L) + op.lam);
      add(y * c.nx + lo(x, c.nx), -op.cx);
      add(y * c.nx + hi(x, c.nx), -op.cx);
      if (c.ny > 1) {
        add(lo(y, c.ny) * c.nx + x, -op.cy);
        add(hi(y, c.ny) * c.nx + x, -op.cy);
      }
    }
  if (!invert_ld(A, K)) { set_error("singular coarsest slab matrix"); return STMG_EINVAL; }
  std::vector<double> Ad(static_cast<size_t>(K) * K), AdT(static_cast<size_t>(K) * K);
  for (int r = 0; r < K; ++r)
    for (int s = 0; s < K; ++s) {
      Ad[static_cast<size_t>(r) * K + s] = static_cast<double>(A[static_cast<size_t>(r) * K + s]);
      AdT[static_cast<size_t>(s) * K + r] = static_cast<double>(A[static_cast<size_t>(r) * K + s]);
    }
  HIP_CHECK(hipMemcpyAsync(Ainv, Ad.data(), Ad.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipMemcpyAsync(AinvT, AdT.data(), AdT.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  // split recurrence: G = (cout (x) I) A^{-1} (cin (x) I), H = A^{-1} (cin (x) I)
  // for the forward problem and, with the transposed inverse and exchanged
  // coupling vectors, for the transposed one
  std::vector<double> Gd, Hd, GTd, HTd, cod;
  if (scan.G) {
    auto build = [&](bool tr, const OpParams& o, std::vector<double>& Gv, std::vector<double>& Hv) {
      Gv.assign(static_cast<size_t>(P) * P, 0.0);
      Hv.assign(static_cast<size_t>(K) * P, 0.0);
      auto inv = [&](int r, int s) -> long double {
        return tr ? A[static_cast<size_t>(s) * K + r] : A[static_cast<size_t>(r) * K + s];
      };
      for (int r = 0; r < K; ++r)
        for (int q2 = 0; q2 < P; ++q2) {
          long double h = 0.0L;
          for (int m2 = 0; m2 < M; ++m2) h += inv(r, m2 * P + q2) * static_cast<long double>(o.cin[m2]);
          Hv[static_cast<size_t>(r) * P + q2] = static_cast<double>(h);
        }
      for (int q = 0; q < P; ++q)
        for (int q2 = 0; q2 < P; ++q2) {
          long double g = 0.0L;
          for (int m = 0; m < M; ++m) {
            long double h = 0.0L;
            for (int m2 = 0; m2 < M; ++m2) h += inv(m * P + q, m2 * P + q2) * static_cast<long double>(o.cin[m2]);
            g += static_cast<long double>(o.cout[m]) * h;
          }
          Gv[static_cast<size_t>(q) * P + q2] = static_cast<double>(g);
        }
    };
    build(false, c.op, Gd, Hd);
    build(true, c.opT, GTd, HTd);
    cod.assign(2 * kMaxM, 0.0);
    for (int m = 0; m < M; ++m) {
      cod[m] = c.op.cout[m];
      cod[kMaxM + m] = c.opT.cout[m];
    }
    HIP_CHECK(hipMemcpyAsync(const_cast<double*>(scan.G), Gd.data(), Gd.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(const_cast<double*>(scan.H), Hd.data(), Hd.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(const_cast<double*>(scanT.G), GTd.data(), GTd.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(const_cast<double*>(scanT.H), HTd.data(), HTd.size() * sizeof(double), hipMemcpyHostToDevice, stream));
    HIP_CHECK(hipMemcpyAsync(const_cast<double*>(scan.cout), cod.data(), cod.size() * sizeof(double), hipMemcpyHostToDevice, stream));
  }
  HIP_CHECK(hipStreamSynchronize(stream));  // host vectors go out of scope
  return STMG_OK;
}

int Solver::upload() {
  if (win) {
    win->stream = stream;
    int rc = win->upload();
    if (rc) return rc;
    if (win_last) {
      win_last->stream = stream;
      rc = win_last->upload();
      if (rc) return rc;
    }
    return STMG_OK;
  }
  const int M = prob.M;
  {
    const int rc = fft ? upload_fft() : upload_dense();
    if (rc) return rc;
  }
  double w[kMaxM] = {0};
  for (int i = 0; i < M; ++i) w[i] = static_cast<double>(tab.l0[i]);
  HIP_CHECK(hipMemcpyAsync(lw, w, sizeof(w), hipMemcpyHostToDevice, stream));
  HIP_CHECK(hipMemcpyAsync(form_G, lv[0].op.G, sizeof(lv[0].op.G), hipMemcpyHostToDevice, stream));
  double G[kMaxM * kMaxM] = {0};
  if (!sdcn.empty()) {
    // collocation residual = Q diag(b)^{-1} (DG residual), per slab and point
    for (int i = 0; i < M; ++i)
      for (int j = 0; j < M; ++j) G[i * M + j] = static_cast<double>(tab.Q[i][j] / tab.b[j]);
    HIP_CHECK(hipMemcpyAsync(sdc_G, G, sizeof(G), hipMemcpyHostToDevice, stream));
    for (auto& sub : sdcn) {
      sub->stream = stream;
      int rc = sub->upload();
      if (rc) return rc;
    }
  }
  for (auto& q : pf) {
    q.sol->stream = stream;
    int rc = q.sol->upload();
    if (rc) return rc;
  }
  HIP_CHECK(hipStreamSynchronize(stream));  // host vectors go out of scope
  return STMG_OK;
}

// ---------------------------------------------------------------------------
int Solver::chunk_of(int l) const { return l == 0 ? opt.chunk : opt.chunk_coarse; }

// Slabs per thread in the transfer kernels of level l: long runs on big
// levels (fewer re-reads at run boundaries), single slabs on small levels
// (more parallelism; their cost is latency, not bandwidth).  No effect on
// results.
int Solver::transfer_slabs(int l) const {
  if (l < static_cast<int>(tuned.size()) && tuned[l] > 0) return tuned[l];
  const Level& L = lv[l];
  const long long pts = static_cast<long long>(L.nx) * L.ny;
  return pts * L.N >= (1LL << 22) ? kTransferSlabs : 1;
}

template <typename T>
static const T* coef_of(const Level& l);
template <>
const double* coef_of<double>(const Level& l) { return l.coef64; }
template <>
const float* coef_of<float>(const Level& l) { return l.coef32; }
template <typename T>
static T* nt_of(const Level& l);
template <>
double* nt_of<double>(const Level& l) { return l.nt64; }
template <>
float* nt_of<float>(const Level& l) { return l.nt32; }

template <typename T>
static T* g9_tmp(const Level& l);
template <>
double* g9_tmp<double>(const Level& l) { return l.g64; }
template <>
float* g9_tmp<float>(const Level& l) { return l.g32; }

template <typename T>
hipError_t Solver::smooth(int l, bool adj, int react, const T* U, const T* f, const double* u0,
                          T* out) {
  const Level& L = lv[l];
  if (L.g9) return launch_smooth9<T>(adj ? L.opT : L.op, L.st, U, f, out, chunk_of(l), stream);
  SweepPtrs<T> a{U, f, u0, coef_of<T>(L), out, nullptr};
  return launch_smooth<T>(adj ? L.opT : L.op, react, a, chunk_of(l), stream);
}

bool Solver::sr_usable(int react, bool fp64) const {
  // a reaction coefficient (Newton) in FP32 only: the FP64 kernel with it needs
  // too many registers, the separate kernels serve it
  return sr && fuse && (react == REACT_CONST || (react == REACT_COEF && !fp64)) && opt.smoother == STMG_SMOOTH_PBJ;
}

template <typename T>
T* sr_zbuf(double* z64, float* z32);
template <>
double* sr_zbuf<double>(double* z64, float*) { return z64; }
template <>
float* sr_zbuf<float>(double*, float* z32) { return z32; }

template <typename T>
hipError_t Solver::smooth_restrict(bool adj, int react, const T* U, const T* f, const double* u0, T* out, T* fc,
                                   T* uc, double* part_out, bool* smoothed) {
  const Level& L = lv[0];
  const Level& C = lv[1];
  SweepPtrs<T> a{U, f, u0, react == REACT_COEF ? coef_of<T>(L) : nullptr, out, part_out};
  if (part_out && smooth_restrict_blocks(L.op, chunk_of(0)) > max_parts) {
    set_error("partial buffer too small");
    return hipErrorInvalidValue;
  }
  if (smoothed) *smoothed = uc != nullptr;
  return launch_smooth_restrict<T>(adj ? L.opT : L.op, react, a, C.nx, C.ny, fc, chunk_of(0),
                                   adj ? &C.opT : &C.op, uc, react == REACT_COEF ? coef_of<T>(C) : nullptr,
                                   chunk_of(1), sr_zbuf<T>(sr_z64, sr_z32), stream);
}

template <typename T>
hipError_t Solver::restrict_residual(int l, bool adj, int react, const T* U, const T* f,
                                     const double* u0, T* fc, T* uc, bool* smoothed) {
  const Level& L = lv[l];
  const Level& C = lv[l + 1];
  SweepPtrs<T> a{U, f, u0, coef_of<T>(L), nullptr, nullptr};
  int spb = transfer_slabs(l + 1);
  const int cs = chunk_of(l + 1);
  if (L.kind & 4) {
    // node coarsening: restrict in space with this level's nodes into the
    // transfer buffer, then R = P^T over the nodes (no fused coarse sweep)
    if (smoothed) *smoothed = false;
    T* nt = nt_of<T>(L);
    HIP_TRY(launch_restrict_residual<T>(adj ? L.opT : L.op, react, a, (L.kind & 1) != 0,
                                        (L.kind & 2) != 0, C.nx, C.ny, C.N, nt, spb, stream));
    return launch_node_transfer<T>(nt, L.M, fc, C.M, L.Rn, C.N, static_cast<size_t>(C.nx) * C.ny,
                                   stream);
  }
  if (L.g9) {
    // Galerkin level: its residual into the level's temporary, then the
    // transfer of that vector (the restriction kernels with a zero iterate)
    T* tmp = g9_tmp<T>(L);
    HIP_TRY(launch_residual9<T>(adj ? L.opT : L.op, L.st, U, f, tmp, stream));
    a = SweepPtrs<T>{nullptr, tmp, nullptr, nullptr, nullptr, nullptr};
    uc = nullptr;
  }
  // a Galerkin coarse level smooths with its own operator: no fused first sweep
  if (C.g9) uc = nullptr;
  if (smoothed) *smoothed = false;
  if (uc && spb % cs != 0) spb = ((spb + cs - 1) / cs) * cs;
  return launch_restrict_residual<T>(adj ? L.opT : L.op, react, a, (L.kind & 1) != 0,
                                     (L.kind & 2) != 0, C.nx, C.ny, C.N, fc, spb, stream,
                                     adj ? &C.opT : &C.op, uc, coef_of<T>(C), cs, smoothed);
}

template <typename T>
hipError_t Solver::prolong(int l, const T* Uin, const T* ec, T* Uout) {
  const Level& L = lv[l];
  const Level& C = lv[l + 1];
  if (L.kind & 4) {
    T* nt = nt_of<T>(L);
    HIP_TRY(launch_node_transfer<T>(ec, C.M, nt, L.M, L.Pn, C.N, static_cast<size_t>(C.nx) * C.ny, stream));
    ec = nt;
  }
  return launch_prolong<T>(L.op, (L.kind & 1) != 0, (L.kind & 2) != 0, C.nx, C.ny, C.N, ec, Uin,
                           Uout, transfer_slabs(l), stream);
}

template <typename T>
hipError_t Solver::coarse(bool adj, int react, const T* f, const double* u0, T* U) {
  const Level& C = lv.back();
  const OpParams& op = adj ? C.opT : C.op;
  if (react == REACT_COEF) {
    if (coarse_inv && !adj) return launch_coarse_solve_slabs<T>(op, coarse_inv, f, u0, U, stream);
    return launch_coarse_solve_coef<T>(op, coef_of<T>(C), coarse_scratch, f, u0, U, stream);
  }
  if constexpr (sizeof(T) == 4) {
    if (fft32)
      return launch_fft_coarse32(op, adj ? fft_sinvT32 : fft_sinv32, fft_tw32, fft_work32, f, u0, U, stream,
                                 C.g9 ? fft_mscale32 : nullptr);
  }
  if (fft)
    return launch_fft_coarse<T>(op, adj ? fft_sinvT : fft_sinv, fft_tw, fft_work, f, u0, U, stream,
                                C.g9 ? fft_mscale : nullptr);
  if (scan.G) return launch_coarse_scan<T>(op, adj ? scanT : scan, f, u0, U, stream);
  return launch_coarse_solve<T>(op, adj ? AinvT : Ainv, f, u0, U, stream);
}

template <typename T>
hipError_t Solver::prolong_smooth(int l, bool adj, int react, const T* Uin, const T* ec,
                                  const T* f, const double* u0, T* out) {
  const Level& L = lv[l];
  const Level& C = lv[l + 1];
  SweepPtrs<T> a{Uin, f, u0, coef_of<T>(L), out, nullptr};
  if (L.kind & 4) {
    T* nt = nt_of<T>(L);
    HIP_TRY(launch_node_transfer<T>(ec, C.M, nt, L.M, L.Pn, C.N, static_cast<size_t>(C.nx) * C.ny, stream));
    ec = nt;
  }
  if (L.g9) {
    // Galerkin level: U' = U_in + P e_c into the level's temporary, then the
    // 9-point smoothing sweep
    T* tmp = g9_tmp<T>(L);
    HIP_TRY(launch_prolong<T>(L.op, (L.kind & 1) != 0, (L.kind & 2) != 0, C.nx, C.ny, C.N, ec, Uin, tmp,
                              transfer_slabs(l), stream));
    return launch_smooth9<T>(adj ? L.opT : L.op, L.st, tmp, f, out, chunk_of(l), stream);
  }
  if constexpr (sizeof(T) == 4) {
    if (l == 0 && up_in) {
      a.up64 = up_in;
      a.up64_out = up_out;
      up_done = true;
    }
  }
  return launch_prolong_smooth<T>(adj ? L.opT : L.op, react, a, (L.kind & 1) != 0,
                                  (L.kind & 2) != 0, C.nx, C.ny, C.N, ec, chunk_of(l), stream);
}

template <typename T>
hipError_t Solver::vcycle(int l, bool adj, int react, T* cur, T* oth, const T* f,
                          const double* u0, bool zero, T** res, int skip_pre) {
  const int last = static_cast<int>(lv.size()) - 1;
  if (l == last) {
    HIP_TRY(coarse<T>(adj, react, f, u0, cur));
    *res = cur;
    return hipSuccess;
  }
  if constexpr (sizeof(T) == 8) {
    if (l == 0 && opt.smoother == STMG_SMOOTH_SDC && !sdcn.empty()) {
      // Finest level smoothed by SDC sweeps (in place, right-hand side from
      // u0), unfused transfers; the coarser levels are as below.
      if (zero) HIP_TRY(hipMemsetAsync(cur, 0, lv[0].n * sizeof(double), stream));
      for (int s = skip_pre; s < opt.nu_pre; ++s)
        if (sdc_core(u0, cur, 1) != STMG_OK) return hipErrorLaunchFailure;
      Level& C = lv[1];
      const bool want = fuse && l + 1 < last;
      bool smoothed = false;
      HIP_TRY(restrict_residual<double>(0, adj, react, cur, f, u0, C.f64, want ? C.A64 : nullptr, &smoothed));
      if (gate0) {
        bool stop = false;
        HIP_TRY(gate0(&stop));
        if (stop) {
          *res = nullptr;
          return hipSuccess;
        }
      }
      double* ec = nullptr;
      HIP_TRY(vcycle<double>(1, adj, react, C.A64, C.B64, C.f64, nullptr, !smoothed, &ec, smoothed ? 1 : 0));
      HIP_TRY(prolong<double>(0, cur, ec, cur));
      for (int s = 0; s < opt.nu_post; ++s)
        if (sdc_core(u0, cur, 1) != STMG_OK) return hipErrorLaunchFailure;
      *res = cur;
      return hipSuccess;
    }
  }
  Level& C = lv[l + 1];
  T* cf = nullptr;
  T* ca = nullptr;
  T* cb = nullptr;
  if constexpr (sizeof(T) == 8) { cf = C.f64; ca = C.A64; cb = C.B64; }
  else { cf = C.f32; ca = C.A32; cb = C.B32; }
  // Descend: the restriction also does the coarse level's first smoothing
  // sweep from a zero iterate when the kernel supports it.  On level 0 the
  // last pre-smoothing sweep and the restriction are one kernel where the
  // grid allows it (or were, when the caller's sweep already restricted).
  const bool want = fuse && opt.nu_pre >= 1 && l + 1 < last;
  bool smoothed = false;
  bool restricted = false;
  if (l == 0 && skip_pre >= 1 && sr_pending) {
    restricted = true;
    smoothed = sr_smoothed;
    sr_pending = false;
  }
  const bool use_sr = l == 0 && !restricted && sr_usable(react, sizeof(T) == 8) && opt.nu_pre > skip_pre;
  for (int s = skip_pre; s < opt.nu_pre; ++s) {
    if (use_sr && s == opt.nu_pre - 1) {
      HIP_TRY(smooth_restrict<T>(adj, react, zero ? nullptr : cur, f, u0, oth, cf, want ? ca : nullptr, nullptr,
                                 &smoothed));
      restricted = true;
    } else {
      HIP_TRY(smooth<T>(l, adj, react, zero ? nullptr : cur, f, u0, oth));
    }
    std::swap(cur, oth);
    zero = false;
  }
  if (!restricted)
    HIP_TRY(restrict_residual<T>(l, adj, react, zero ? nullptr : cur, f, u0, cf,
                                 want ? ca : nullptr, &smoothed));
  if (l == 0 && gate0) {
    // Nothing written so far touches the caller's iterate.
    bool stop = false;
    HIP_TRY(gate0(&stop));
    if (stop) {
      *res = nullptr;
      return hipSuccess;
    }
  }
  T* ec = nullptr;
  HIP_TRY(vcycle<T>(l + 1, adj, react, ca, cb, cf, nullptr, !smoothed, &ec, smoothed ? 1 : 0));
  // Ascend: prolongation fused with the first post-smoothing sweep where the
  // grid layout allows it.
  int post = opt.nu_post;
  const OpParams& op = adj ? lv[l].opT : lv[l].op;
  if (fuse && post >= 1 && blocked_layout(op)) {
    HIP_TRY(prolong_smooth<T>(l, adj, react, zero ? nullptr : cur, ec, f, u0, oth));
    std::swap(cur, oth);
    --post;
  } else {
    // Keep an even number of buffer flips so that level 0 ends where it began.
    const bool flip = ((opt.nu_pre + opt.nu_post) & 1) != 0;
    if (flip) {
      HIP_TRY(prolong<T>(l, zero ? nullptr : cur, ec, oth));
      std::swap(cur, oth);
    } else {
      HIP_TRY(prolong<T>(l, zero ? nullptr : cur, ec, cur));
    }
  }
  for (int s = 0; s < post; ++s) {
    HIP_TRY(smooth<T>(l, adj, react, cur, f, u0, oth));
    std::swap(cur, oth);
  }
  *res = cur;
  return hipSuccess;
}

template <typename TO>
hipError_t Solver::residual64(bool adj, int react, const double* U, const double* f,
                              const double* u0, TO* r, double* d_out) {
  const Level& L = lv[0];
  if (residual_parts() > max_parts) {
    set_error("partial buffer too small");
    return hipErrorInvalidValue;
  }
  SweepPtrs<double> a{U, f, u0, L.coef64, r, part};
  int launched = 0;
  HIP_TRY((launch_residual<double, TO>(adj ? L.opT : L.op, react, a, kResidSlabs, &launched, stream)));
  return launch_sum_partials(part, launched, d_out, stream);
}

long long Solver::residual_parts() const {
  const Level& L = lv[0];
  return ((static_cast<long long>(L.nx) * L.ny + kBlock - 1) / kBlock) *
         ((L.N + kResidSlabs - 1) / kResidSlabs);
}

int Solver::read_scalar(const double* d, double* h) {
  HIP_CHECK(hipMemcpyAsync(h, d, sizeof(double), hipMemcpyDeviceToHost, stream));
  HIP_CHECK(hipStreamSynchronize(stream));
  return STMG_OK;
}

double Solver::norm_u0_b(const double* u0) {
  // ||b||^2 = sum_i l_i(0)^2 ||u0||^2 for b_{0,i} = l_i(0) u0.
  const Level& L = lv[0];
  const size_t P = static_cast<size_t>(L.nx) * L.ny;
  int np = 0;
  if (launch_sumsq(u0, P, part, &np, stream) != hipSuccess) return -1.0;
  if (launch_sum_partials(part, np, scal + 1, stream) != hipSuccess) return -1.0;
  double s = 0.0;
  if (read_scalar(scal + 1, &s) != STMG_OK) return -1.0;
  // collocation form: b_{0,i} = (G l(0))_i u0 with G = Q diag(b)^-1
  long double w = 0.0L;
  for (int i = 0; i < prob.M; ++i) {
    long double v = tab.l0[i];
    if (L.op.colloc) {
      v = 0.0L;
      for (int j = 0; j < prob.M; ++j) v += tab.Q[i][j] / tab.b[j] * tab.l0[j];
    }
    w += v * v;
  }
  return std::sqrt(static_cast<double>(w) * s);
}

// ---------------------------------------------------------------------------
// Linear solve on level 0: FP64 V-cycles, or (mixed) FP32 V-cycles on the
// FP64 residual with FP64 updates (iterative refinement).  `U` holds the
// initial guess and receives the result.
int Solver::solve_linear(bool adj, int react, const double* f, const double* u0, double* U,
                         double rtol, double norm_b, int* cycles, double* rel_out, int* refinements) {
  if (opt.krylov > 0) return solve_fgmres(adj, react, f, u0, U, rtol, norm_b, cycles, rel_out);
  Level& L0 = lv[0];
  const OpParams& op0 = adj ? L0.opT : L0.op;
  // FP64 with pre-smoothing: the first sweep of every cycle also returns
  // ||f - A U_k|| of the incoming iterate U_k, which stays untouched in `U`
  // (the sweep writes the ping-pong partner), so the stop test costs no extra
  // pass over the data.
  const bool fused = !mixed && opt.nu_pre >= 1 && opt.smoother == STMG_SMOOTH_PBJ;
  // Mixed precision on the register-blocked layout: one fused sweep per
  // refinement step forms U' = U + e, its FP64 residual and norm, the FP32
  // right-hand side and the first FP32 smoothing sweep (k_refine_blk); the
  // iterate ping-pongs between U and L0.B64.
  const bool refine = mixed && opt.nu_pre >= 1 && blocked_layout(op0) &&
                      (react == REACT_CONST || react == REACT_COEF);
  const int inner = mixed ? opt.inner_cycles : 1;
  HIP_CHECK(hnorm.init());
  double* Ucur = U;
  double* Unext = L0.B64;
  const float* ecur = nullptr;
  float* e1 = L0.A32;
  // Queues ||f - A U||^2 of the current iterate, written straight into the
  // pinned host slot, and an event behind it.
  double* const out = hnorm.d;
  sr_pending = false;
  auto launch_norm = [&]() -> hipError_t {
    if (fused && opt.nu_pre == 1 && lv.size() > 1 && sr_usable(react, true)) {
      // the only pre-smoothing sweep also restricts
      Level& C = lv[1];
      const bool want = fuse && lv.size() > 2;
      HIP_TRY(smooth_restrict<double>(adj, react, U, f, u0, L0.B64, C.f64, want ? C.A64 : nullptr, part,
                                      &sr_smoothed));
      sr_pending = true;
      HIP_TRY(launch_sum_partials(part, smooth_restrict_blocks(op0, chunk_of(0)), out, stream));
    } else if (fused) {
      SweepPtrs<double> a{U, f, u0, L0.coef64, L0.B64, part};
      HIP_TRY(launch_smooth<double>(op0, react, a, chunk_of(0), stream));
      HIP_TRY(launch_sum_partials(part, smooth_blocks(op0, chunk_of(0)), out, stream));
    } else if (refine) {
      // U' = Ucur + ecur when the correction was not folded into the last
      // FP32 kernel of the previous step (ecur set), else Ucur as it is
      SweepPtrs<double> a{Ucur, f, u0, L0.coef64, ecur ? Unext : nullptr, part};
      e1 = (ecur == L0.A32) ? L0.B32 : L0.A32;
      int np = 0;
      if (smooth_blocks(op0, chunk_of(0)) > max_parts) {
        set_error("partial buffer too small");
        return hipErrorInvalidValue;
      }
      HIP_TRY(launch_refine(op0, react, a, ecur, L0.f32, e1, L0.coef32, chunk_of(0), &np, stream));
      HIP_TRY(launch_sum_partials(part, np, out, stream));
    } else if (!mixed) {
      HIP_TRY(residual64<double>(adj, react, U, f, u0, nullptr, out));
    } else {
      HIP_TRY(residual64<float>(adj, react, U, f, u0, L0.f32, out));
    }
    return hipEventRecord(hnorm.ev, stream);
  };
  double rel = 0.0, rel0 = 0.0, prev = 0.0;
  double step_rel = 0.0;  // mixed: residual at the start of the previous step
  int step_k = 0;         // and its FP32 cycles
  bool first = true;
  int incr = 0;
  int c = 0;   // outer steps (V-cycles in FP64, refinement steps in mixed precision)
  int vc = 0;  // V-cycles
  int status = STMG_OK;
  // Waits for the queued norm and applies the stop tests to U_c.  A negative
  // norm_b means: relative to the first residual (||b|| for a zero initial
  // guess), so the caller needs no separate pass and read for ||b||.
  double nb = norm_b;
  auto decide = [&](bool* stop) -> hipError_t {
    HIP_TRY(hipEventSynchronize(hnorm.ev));
    const double rn2 = *hnorm.h;
    if (first && nb < 0.0) nb = rn2 > 0.0 ? std::sqrt(rn2) : 1.0;
    rel = nb > 0.0 ? std::sqrt(rn2) / nb : std::sqrt(rn2);
    if (first) { rel0 = rel; prev = rel; first = false; }
    *stop = true;
    if (!std::isfinite(rel)) { status = STMG_ENAN; return hipSuccess; }
    if (rel <= rtol) return hipSuccess;
    if (c > 0) {
      if (rel > 1e3 * (rel0 > 0 ? rel0 : 1.0)) { status = STMG_EDIVERGED; return hipSuccess; }
      // growth of more than 10% per cycle, five cycles in a row (at the rounding
      // floor the norm moves by far less, either way)
      incr = rel > kGrowth * prev ? incr + 1 : 0;
      if (incr >= 5) { status = STMG_EDIVERGED; return hipSuccess; }
    }
    prev = rel;
    if (vc >= opt.max_cycles) { status = STMG_ENOTCONV; return hipSuccess; }
    *stop = false;
    return hipSuccess;
  };
  struct GateScope {
    Solver* s;
    ~GateScope() { s->gate0 = nullptr; }
  } scope{this};
  // With one level there is no restriction to overlap: decide up front.
  const bool gated = lv.size() > 1;
  if (gated) gate0 = decide;
  HIP_CHECK(launch_norm());
  for (;;) {
    if (!gated) {
      bool stop = false;
      HIP_CHECK(decide(&stop));
      if (stop) break;
    }
    if (fused) {
      // the first pre-smoothing sweep already sits in L0.B64
      double* res = nullptr;
      HIP_CHECK(vcycle<double>(0, adj, react, L0.B64, U, f, u0, false, &res, 1));
      if (!res) break;
      if (res != U) HIP_CHECK(hipMemcpyAsync(U, res, L0.n * sizeof(double), hipMemcpyDeviceToDevice, stream));
      ++vc;
    } else if (!mixed) {
      double* res = nullptr;
      HIP_CHECK(vcycle<double>(0, adj, react, U, L0.B64, f, u0, false, &res, 0));
      if (!res) break;
      if (res != U) HIP_CHECK(hipMemcpyAsync(U, res, L0.n * sizeof(double), hipMemcpyDeviceToDevice, stream));
      ++vc;
    } else {
      // FP32 V-cycles on A e = r: the first starts from the sweep already in
      // e1 (fused refinement) or from zero.
      // With the fused refinement the last cycle's level-0 post-smoothing also
      // writes Unext = Ucur + e in FP64 (up_in / up_out) when it is the fused
      // prolongation kernel; otherwise the next refinement sweep adds e.
      float* res = nullptr;
      float* oth = (e1 == L0.A32) ? L0.B32 : L0.A32;
      if (refine) {
        // at the refinement sweep the iterate is Unext when it formed U' there
        if (ecur) std::swap(Ucur, Unext);
        ecur = nullptr;
      }
      struct UpScope {
        Solver* s;
        ~UpScope() { s->up_in = nullptr; s->up_out = nullptr; }
      } up_scope{this};
      up_done = false;
      if (refine && inner == 1) { up_in = Ucur; up_out = Unext; }
      if (refine) HIP_CHECK(vcycle<float>(0, adj, react, e1, oth, L0.f32, nullptr, false, &res, 1));
      else HIP_CHECK(vcycle<float>(0, adj, react, L0.A32, L0.B32, L0.f32, nullptr, true, &res, 0));
      if (!res) break;
      ++vc;
      // Cycles of this step: inner_cycles, or with inner_adapt (from the
      // second step on) the count that the previous step's contraction per
      // cycle says takes the current residual (known here: the stop test ran
      // inside the first cycle) down to rtol.
      int inner_now = inner;
      if (opt.inner_adapt && step_k > 0 && rel > 0.0 && rel < step_rel) {
        const double rho = std::pow(rel / step_rel, 1.0 / step_k);
        const double need = std::log(rtol / rel) / std::log(rho);
        if (need < inner) inner_now = std::max(1, static_cast<int>(std::ceil(need)));
      }
      step_rel = rel;
      step_k = inner_now;
      for (int k = 1; k < inner_now; ++k) {
        float* other = (res == L0.A32) ? L0.B32 : L0.A32;
        float* r2 = nullptr;
        if (refine && k == inner_now - 1) { up_in = Ucur; up_out = Unext; }
        const auto g = std::move(gate0);
        gate0 = nullptr;
        const hipError_t e = vcycle<float>(0, adj, react, res, other, L0.f32, nullptr, false, &r2, 0);
        gate0 = g;
        HIP_CHECK(e);
        res = r2;
        ++vc;
      }
      up_in = nullptr;
      up_out = nullptr;
      if (refine) {
        if (up_done) std::swap(Ucur, Unext);  // Unext = Ucur + e is written
        else ecur = res;                      // the next sweep forms Ucur + e
      } else {
        HIP_CHECK(launch_update<float>(L0.n, U, res, nullptr, stream));
      }
    }
    ++c;
    HIP_CHECK(launch_norm());
  }
  // Fused refinement: the final iterate is the last refinement sweep's U',
  // Unext when that sweep added the correction, else Ucur.
  if (refine) {
    double* fin = ecur ? Unext : Ucur;
    if (fin != U) HIP_CHECK(hipMemcpyAsync(U, fin, L0.n * sizeof(double), hipMemcpyDeviceToDevice, stream));
  }
  sr_pending = false;
  *cycles += vc;
  if (refinements) *refinements += mixed ? c : 0;
  *rel_out = rel;
  if (status != STMG_OK) {
    set_error(std::string("linear solve stopped: ") + stmg_status_string(status));
  }
  return status;
}

// Restarted flexible GMRES (Saad, 1993) on A U = b with one V-cycle from a
// zero guess as the right preconditioner: the paper stops its multigrid runs
// on a preconditioned Krylov residual (Sec. 5).  The minimised residual is
// the true one, ||b - A U||, so the stop test is the plain iteration's.
//
// Storage and scaling: basis vectors are kept unnormalised (V_i raw, with
// v_i = V_i / ||V_i||); the host holds 1 / ||V_i||^2.  Step j runs the
// preconditioner on V_j into Z_j and the residual kernel on Z_j with no
// right-hand side, W = -A Z_j, so the direction taken is zhat_j = -Z_j and
// A zhat_j = W.  Then h_ij = (W, v_i) and the projections W -= h_ij v_i are
// W -= (W, V_i) / ||V_i||^2 V_i.  Classical Gram-Schmidt, whose dot products
// are fused into the projection pass, repeated when the projection removed
// more than half of ||W||^2 (Daniel, Gragg, Kaufman, Stewart 1976); the
// remainder, unnormalised, is V_{j+1}.  The (m + 1) x m Hessenberg matrix is
// reduced by Givens rotations on the host; the estimate |g_{j+1}| ends the
// cycle, U += sum_j y_j zhat_j, and the true residual of the new U starts the
// next cycle or ends the solve.  Host waits: one per step, two when the
// second Gram-Schmidt pass runs, one per restart.
int Solver::solve_fgmres(bool adj, int react, const double* f, const double* u0, double* U,
                         double rtol, double norm_b, int* cycles, double* rel_out) {
  Level& L0 = lv[0];
  const int m = opt.krylov;
  const size_t n = L0.n;
  constexpr int kCol = kKrylovMax + 2;
  HIP_CHECK(kh.init(1 + 3 * kCol));
  double* const hres = kh.h;
  double* const h1 = kh.h + 1;
  double* const h2 = h1 + kCol;
  double* const h3 = h2 + kCol;
  double* const m1 = kh.d + 1;
  double* const m2 = m1 + kCol;
  double* const m3 = m2 + kCol;
  double* const d1 = kdev + 1;
  double* const d2 = d1 + kCol;
  double* const d3 = d2 + kCol;
  double* Vb[kKrylovMax + 1];
  double* Zb[kKrylovMax + 1];
  for (int i = 0; i <= m; ++i) {
    Vb[i] = kV + static_cast<size_t>(i) * kstride;
    Zb[i] = kZ + static_cast<size_t>(i) * kstride;
  }
  KVecs Vs{};
  for (int i = 0; i <= m; ++i) Vs.v[i] = Vb[i];
  // norm_b < 0: relative to the first residual (as in solve_linear)
  double scale = norm_b > 0.0 ? norm_b : 1.0;
  bool scale_first = norm_b < 0.0;
  std::vector<double> H(static_cast<size_t>(m + 1) * m), cs(m), sn(m), g(m + 1), inv2(m + 1);
  auto Hs = [&](int i, int j) -> double& { return H[static_cast<size_t>(i) * m + j]; };
  auto wait = [&]() -> hipError_t {
    HIP_TRY(hipEventRecord(kh.ev, stream));
    return hipEventSynchronize(kh.ev);
  };
  // out = M^-1 (alpha in): one V-cycle from zero (FP32 on a cast copy in
  // mixed precision); the result lands in *out, which may trade places with
  // the ping-pong partner *spare
  int vcount = 0;
  auto vcyc = [&](const double* in, double alpha, double** out, double** spare) -> hipError_t {
    ++vcount;
    if (!mixed) {
      double* res = nullptr;
      HIP_TRY(vcycle<double>(0, adj, react, *out, *spare, in, nullptr, true, &res, 0));
      if (res == *spare) std::swap(*out, *spare);
      else if (res != *out) return hipErrorInvalidValue;
      return hipSuccess;
    }
    HIP_TRY((launch_axpy_cast<double, float>(n, in, alpha, L0.f32, false, stream)));
    float* res = nullptr;
    HIP_TRY(vcycle<float>(0, adj, react, L0.A32, L0.B32, L0.f32, nullptr, true, &res, 0));
    if (!res) return hipErrorInvalidValue;
    return launch_axpy_cast<float, double>(n, res, 1.0, *out, false, stream);
  };
  // Left preconditioning (GMRES on M^-1 A U = M^-1 b, stop on the
  // preconditioned residual): the basis is built from W = M^-1 (-A V_j) in
  // place of -A M^-1 V_j; Zb[0] holds -A V_j (or the restart residual) and
  // Zb[1] is the cycle's ping-pong partner.
  const bool left = opt.krylov_left != 0;
  double* T = Zb[0];
  double* spare = Zb[1];
  double pscale = 0.0;  // first preconditioned residual norm (left)
  auto sync_vs = [&]() {
    for (int i = 0; i <= m; ++i) Vs.v[i] = Vb[i];
  };
  int steps = 0;
  int status = STMG_OK;
  double rel = 0.0;
  // cycles in a row that the least-squares estimate ended (estimate <=
  // rtol) while the true residual of the updated iterate stayed above rtol:
  // the estimate keeps falling in exact arithmetic, the true residual stops
  // at its rounding floor, so two misses in a row mean rtol is below it
  bool est_done = false;
  int miss = 0;
  for (;;) {
    // r = b - A U is the first (unnormalised) basis vector; with left
    // preconditioning M^-1 r is
    HIP_CHECK(residual64<double>(adj, react, U, f, u0, left ? T : Vb[0], kh.d));
    HIP_CHECK(wait());
    const double rnorm = std::sqrt(*hres);
    if (scale_first) {
      scale = rnorm > 0.0 ? rnorm : 1.0;
      scale_first = false;
    }
    rel = rnorm / scale;
    if (!std::isfinite(rel)) { status = STMG_ENAN; break; }
    if (rnorm == 0.0) break;
    double beta = rnorm;
    double crit = rel;  // the quantity the stop test compares with rtol
    if (left) {
      // (this cycle also checks the final iterate, so the count may end one
      // above max_cycles)
      HIP_CHECK(vcyc(T, 1.0, &Vb[0], &spare));
      sync_vs();
      int nb = 0;
      HIP_CHECK(launch_kortho(Vb[0], Vs, 0, KCoef{}, nullptr, n, false, kpart, &nb, stream));
      HIP_CHECK(launch_kreduce(kpart, nb, 1, d1, m1, stream));
      HIP_CHECK(wait());
      beta = std::sqrt(h1[0]);
      if (!std::isfinite(beta)) { status = STMG_ENAN; break; }
      if (pscale == 0.0) pscale = beta;
      if (beta == 0.0) break;
      crit = beta / pscale;
    }
    if (crit <= rtol) break;
    if ((left ? vcount : steps) >= opt.max_cycles) { status = STMG_ENOTCONV; break; }
    miss = est_done ? miss + 1 : 0;
    if (miss >= 2) { status = STMG_ENOTCONV; break; }
    est_done = false;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    inv2[0] = 1.0 / (beta * beta);
    int k = 0;
    bool bad = false;
    for (int j = 0; j < m; ++j) {
      if (left) {
        HIP_CHECK(residual64<double>(adj, react, Vb[j], nullptr, nullptr, T, kdev));
        HIP_CHECK(vcyc(T, 1.0, &Vb[j + 1], &spare));
        sync_vs();
      } else {
        HIP_CHECK(vcyc(Vb[j], std::sqrt(inv2[j]), &Zb[j], &Zb[m]));
        HIP_CHECK(residual64<double>(adj, react, Zb[j], nullptr, nullptr, Vb[j + 1], kdev));
      }
      KCoef s{};
      for (int i = 0; i <= j; ++i) s.c[i] = inv2[i];
      int nb = 0;
      // pass 1: (W, V_i) and ||W||^2; pass 2: project, and the same again
      HIP_CHECK(launch_kortho(Vb[j + 1], Vs, j + 1, s, nullptr, n, true, kpart, &nb, stream));
      HIP_CHECK(launch_kreduce(kpart, nb, j + 2, d1, m1, stream));
      HIP_CHECK(launch_kortho(Vb[j + 1], Vs, j + 1, s, d1, n, true, kpart, &nb, stream));
      HIP_CHECK(launch_kreduce(kpart, nb, j + 2, d2, m2, stream));
      HIP_CHECK(wait());
      double hcol[kKrylovMax + 1];
      for (int i = 0; i <= j; ++i) hcol[i] = h1[i];
      double nw2 = h2[j + 1];
      if (nw2 < 0.5 * h1[j + 1]) {
        // pass 3: project out the pass-2 components
        HIP_CHECK(launch_kortho(Vb[j + 1], Vs, j + 1, s, d2, n, false, kpart, &nb, stream));
        HIP_CHECK(launch_kreduce(kpart + static_cast<size_t>(j + 1) * nb, nb, 1, d3 + j + 1, m3 + j + 1,
                                 stream));
        HIP_CHECK(wait());
        for (int i = 0; i <= j; ++i) hcol[i] += h2[i];
        nw2 = h3[j + 1];
      }
      // right: the direction is zhat_j = -Z_j with A zhat_j = W; left: the
      // basis vector v_j = V_j / ||V_j|| itself, with (-M^-1 A) v_j = W / ||V_j||
      const double aj = left ? std::sqrt(inv2[j]) : 1.0;
      for (int i = 0; i <= j; ++i) Hs(i, j) = aj * std::sqrt(inv2[i]) * hcol[i];
      const double hn = aj * std::sqrt(nw2);
      Hs(j + 1, j) = hn;
      ++steps;
      k = j + 1;
      // apply the earlier rotations to column j, then eliminate H(j+1, j)
      for (int i = 0; i < j; ++i) {
        const double a = Hs(i, j), b = Hs(i + 1, j);
        Hs(i, j) = cs[i] * a + sn[i] * b;
        Hs(i + 1, j) = -sn[i] * a + cs[i] * b;
      }
      const double a = Hs(j, j), b = Hs(j + 1, j);
      const double r = std::hypot(a, b);
      if (!std::isfinite(r)) { bad = true; break; }
      cs[j] = r > 0.0 ? a / r : 1.0;
      sn[j] = r > 0.0 ? b / r : 0.0;
      Hs(j, j) = r;
      Hs(j + 1, j) = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      if (std::fabs(g[j + 1]) <= rtol * (left ? pscale : scale)) { est_done = true; break; }
      if ((left ? vcount : steps) >= opt.max_cycles || hn == 0.0) break;
      inv2[j + 1] = 1.0 / nw2;
    }
    if (bad) { status = STMG_ENAN; rel = std::numeric_limits<double>::quiet_NaN(); break; }
    // y = R^-1 g; right: U += sum_j y_j zhat_j = U - sum_j y_j Z_j; left:
    // the operator of the Arnoldi relation is -M^-1 A, so U -= sum_j y_j v_j
    KCoef y{};
    for (int i = k - 1; i >= 0; --i) {
      double t = g[i];
      for (int q = i + 1; q < k; ++q) t -= Hs(i, q) * y.c[q];
      y.c[i] = Hs(i, i) != 0.0 ? t / Hs(i, i) : 0.0;
    }
    KVecs Zs{};
    for (int i = 0; i < k; ++i) {
      Zs.v[i] = left ? Vb[i] : Zb[i];
      y.c[i] = left ? -y.c[i] * std::sqrt(inv2[i]) : -y.c[i];
    }
    HIP_CHECK(launch_kcombine(U, Zs, k, y, n, stream));
  }
  *cycles += vcount;
  *rel_out = rel;
  if (status != STMG_OK) set_error(std::string("Krylov solve stopped: ") + stmg_status_string(status));
  return status;
}

int Solver::newton_linearize(const double* U) {
  // c = gamma (3 U^2 - 1) on level 0, restricted to the coarser levels.
  Level& L0 = lv[0];
  if (L0.coef64 && mixed) {
    HIP_CHECK(launch_newton_coef_pair(L0.n, U, prob.gamma, L0.coef64, L0.coef32, stream));
  } else {
    if (L0.coef64) HIP_CHECK(launch_newton_coef<double>(L0.n, U, prob.gamma, L0.coef64, stream));
    if (mixed) HIP_CHECK(launch_newton_coef<float>(L0.n, U, prob.gamma, L0.coef32, stream));
  }
  for (size_t l = 0; l + 1 < lv.size(); ++l) {
    const Level& F = lv[l];
    Level& C = lv[l + 1];
    const bool sp = (F.kind & 1) != 0, tm = (F.kind & 2) != 0;
    if (!mixed) HIP_CHECK(launch_restrict_coef<double>(F.op, sp, tm, C.nx, C.ny, C.N, F.coef64, C.coef64, stream));
    else HIP_CHECK(launch_restrict_coef<float>(F.op, sp, tm, C.nx, C.ny, C.N, F.coef32, C.coef32, stream));
  }
  if (coarse_inv) {
    const Level& C = lv.back();
    if (!mixed) HIP_CHECK(launch_coarse_invert_coef<double>(C.op, C.coef64, coarse_inv, stream));
    else HIP_CHECK(launch_coarse_invert_coef<float>(C.op, C.coef32, coarse_inv, stream));
  }
  linearized = true;
  return STMG_OK;
}

int Solver::solve(const double* u0, double* U, stmg_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  stmg_stats s{};
  if (win) {
    // window after window; window w starts from the end value of window w-1
    const size_t P = static_cast<size_t>(lv[0].nx) * lv[0].ny;
    const size_t slab = static_cast<size_t>(prob.M) * P;
    int rc = STMG_OK;
    for (int w = 0; w < nwin && rc == STMG_OK; ++w) {
      const double* us = w == 0 ? u0 : U + (static_cast<size_t>(w) * win_W - 1) * slab + (prob.M - 1) * P;
      stmg_stats sw{};
      rc = sub(w)->solve(us, U + static_cast<size_t>(w) * win_W * slab, &sw);
      s.cycles += sw.cycles;
      s.newton_its += sw.newton_its;
      s.refinements += sw.refinements;
      s.rel_res = std::max(s.rel_res, sw.rel_res);
    }
    s.status = rc;
    s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    last = s;
    if (st) *st = s;
    return rc;
  }
  const double nb = norm_u0_b(u0);
  if (nb < 0.0) return STMG_EHIP;
  int rc = STMG_OK;
  if (!allen_cahn) {
    rc = solve_linear(false, REACT_CONST, nullptr, u0, U, opt.rtol, nb, &s.cycles, &s.rel_res,
                      &s.refinements);
  } else {
    // Newton on G(U) = b - A_AC(U) (Sec. 4.2), inexact: each correction solve
    // stops at a relative tolerance eta_k (Eisenstat-Walker, choice 2).
    Level& L0 = lv[0];
    double gprev = -1.0, eta = 1e-2;
    for (int k = 0;; ++k) {
      HIP_CHECK(residual64<double>(false, REACT_AC, U, nullptr, u0, L0.f64, scal));
      double g2 = 0.0;
      rc = read_scalar(scal, &g2);
      if (rc) break;
      const double g = std::sqrt(g2) / nb;
      s.rel_res = g;
      if (!std::isfinite(g)) { rc = STMG_ENAN; break; }
      if (g <= opt.newton_rtol) { rc = STMG_OK; break; }
      if (k >= opt.max_newton) { rc = STMG_ENOTCONV; break; }
      if (gprev > 0.0) {
        const double r = g / gprev;
        eta = 0.9 * r * r;
        if (eta > 1e-1) eta = 1e-1;
      }
      // never ask for more than the final target needs
      const double floor = 0.5 * opt.newton_rtol / g;
      if (eta < floor) eta = floor;
      if (eta < 1e-12) eta = 1e-12;
      gprev = g;
      rc = newton_linearize(U);
      if (rc) break;
      HIP_CHECK(hipMemsetAsync(delta64, 0, L0.n * sizeof(double), stream));
      double rel = 0.0;
      int lrc = solve_linear(false, REACT_COEF, L0.f64, nullptr, delta64, eta, std::sqrt(g2),
                             &s.cycles, &rel, &s.refinements);
      if (lrc == STMG_ENAN || lrc == STMG_EHIP) { rc = lrc; break; }
      HIP_CHECK(launch_update<double>(L0.n, U, delta64, nullptr, stream));
      ++s.newton_its;
    }
  }
  HIP_CHECK(hipStreamSynchronize(stream));
  s.status = rc;
  s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  last = s;
  if (st) *st = s;
  return rc;
}

int Solver::vcycle_user(const double* u0, double* U, double* h_rel) {
  if (win) { set_error("stmg_vcycle: not available on a windowed handle"); return STMG_EUNSUPPORTED; }
  if (allen_cahn && !linearized) {
    set_error("stmg_vcycle: no linearization point yet (run stmg_solve first)");
    return STMG_EINVAL;
  }
  Level& L0 = lv[0];
  const bool lin = !allen_cahn;
  const int react = lin ? REACT_CONST : REACT_COEF;
  const double* f = lin ? nullptr : L0.f64;
  const double* uu = lin ? u0 : nullptr;
  if (!mixed) {
    double* res = nullptr;
    HIP_CHECK(vcycle<double>(0, false, react, U, L0.B64, f, uu, false, &res, 0));
    if (res != U) HIP_CHECK(hipMemcpyAsync(U, res, L0.n * sizeof(double), hipMemcpyDeviceToDevice, stream));
  } else {
    HIP_CHECK(residual64<float>(false, react, U, f, uu, L0.f32, scal));
    float* res = nullptr;
    HIP_CHECK(vcycle<float>(0, false, react, L0.A32, L0.B32, L0.f32, nullptr, true, &res, 0));
    HIP_CHECK(launch_update<float>(L0.n, U, res, nullptr, stream));
  }
  if (h_rel) {
    HIP_CHECK(residual64<double>(false, react, U, f, uu, nullptr, scal));
    double r2 = 0.0;
    int rc = read_scalar(scal, &r2);
    if (rc) return rc;
    double nb = 1.0;
    if (lin) {
      nb = norm_u0_b(u0);
    } else if (L0.op.colloc) {
      // ||f|| in the collocation form: the residual of a zero iterate
      HIP_CHECK(residual64<double>(false, REACT_COEF, nullptr, f, nullptr, nullptr, scal + 2));
      double f2 = 0.0;
      rc = read_scalar(scal + 2, &f2);
      if (rc) return rc;
      nb = std::sqrt(f2);
    } else {
      int np = 0;
      HIP_CHECK(launch_sumsq(L0.f64, L0.n, part, &np, stream));
      HIP_CHECK(launch_sum_partials(part, np, scal + 2, stream));
      double f2 = 0.0;
      rc = read_scalar(scal + 2, &f2);
      if (rc) return rc;
      nb = std::sqrt(f2);
    }
    *h_rel = nb > 0 ? std::sqrt(r2) / nb : std::sqrt(r2);
  }
  return STMG_OK;
}

int Solver::residual_user(const double* u0, const double* U, double* r, double* h_norm) {
  if (win) { set_error("stmg_residual: not available on a windowed handle"); return STMG_EUNSUPPORTED; }
  const int react = allen_cahn ? REACT_AC : REACT_CONST;
  HIP_CHECK(residual64<double>(false, react, U, nullptr, u0, r, scal));
  if (r && lv[0].op.colloc) {
    const Level& L0 = lv[0];
    HIP_CHECK(launch_node_transform(r, L0.N, prob.M, L0.nx * L0.ny, form_G, stream));
  }
  if (h_norm) {
    double r2 = 0.0;
    int rc = read_scalar(scal, &r2);
    if (rc) return rc;
    *h_norm = std::sqrt(r2);
  }
  return STMG_OK;
}

// Solve and keep only the end value u(T) = U_{N,M} (P values).  On a
// windowed handle the trajectory is never stored: one window at a time, the
// window start values go to the checkpoint planes.
int Solver::solve_end(const double* u0, double* uT, stmg_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!win) {
    set_error("stmg_solve_end needs a memory budget that requires time windows");
    return STMG_EUNSUPPORTED;
  }
  const size_t P = static_cast<size_t>(lv[0].nx) * lv[0].ny;
  stmg_stats s{};
  int rc = STMG_OK;
  for (int w = 0; w < nwin && rc == STMG_OK; ++w) {
    const double* us = w == 0 ? u0 : ckpt + static_cast<size_t>(w) * P;
    stmg_stats sw{};
    HIP_CHECK(hipMemsetAsync(Uw, 0, static_cast<size_t>(window_len(w)) * prob.M * P * sizeof(double), stream));
    rc = sub(w)->solve(us, Uw, &sw);
    s.cycles += sw.cycles;
    s.newton_its += sw.newton_its;
    s.rel_res = std::max(s.rel_res, sw.rel_res);
    const double* end = Uw + (static_cast<size_t>(window_len(w) - 1) * prob.M + (prob.M - 1)) * P;
    double* dst = (w + 1 < nwin) ? ckpt + static_cast<size_t>(w + 1) * P : uT;
    HIP_CHECK(hipMemcpyAsync(dst, end, P * sizeof(double), hipMemcpyDeviceToDevice, stream));
  }
  HIP_CHECK(hipStreamSynchronize(stream));
  s.status = rc;
  s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = s;
  return rc;
}

// Adjoint: A^T lam = g with g = dL/du(T) in slab N, node M.  A^T is block
// upper-bidiagonal; stored backward in time (slab n' = N-1-n) it has the
// lower-bidiagonal form of A with K -> Kq^T and the coupling roles of l(0)
// and e_M exchanged, so the forward V-cycle kernels solve it unchanged.
int Solver::adjoint(const double* u0, const double* U, const double* gT, double* grad_u0,
                    double* grad_nu, stmg_stats* st) {
  const auto t0 = std::chrono::steady_clock::now();
  if (allen_cahn) { set_error("adjoint: linear problems only"); return STMG_EUNSUPPORTED; }
  // The transposed kernels reuse the symmetric periodic Laplacian; the
  // ghost-reflection Neumann operator is not symmetric.
  if (prob.bc != STMG_BC_PERIODIC) { set_error("adjoint: periodic grids only"); return STMG_EUNSUPPORTED; }
  if (win) {
    // Windows backward in time.  Window w's transposed system receives from
    // window w+1 the coupling e_M (x) (l(0)^T lam_{first slab of w+1}), which is
    // exactly the "dL/du0" output of window w+1; the window's trajectory is
    // taken from U or recomputed from its checkpoint.
    if (!U && !u0) { set_error("adjoint: need the trajectory or u0"); return STMG_EINVAL; }
    const auto t0 = std::chrono::steady_clock::now();
    const size_t P = static_cast<size_t>(lv[0].nx) * lv[0].ny;
    const size_t slab = static_cast<size_t>(prob.M) * P;
    stmg_stats s{};
    int rc = STMG_OK;
    if (!U) {
      stmg_stats sf{};
      rc = solve_end(u0, gw + P, &sf);  // fills the checkpoints
      if (rc) return rc;
      s.cycles += sf.cycles;
    }
    double gsum = 0.0;
    const double* g = gT;
    for (int w = nwin - 1; w >= 0; --w) {
      const double* Uwin = nullptr;
      if (U) {
        Uwin = U + static_cast<size_t>(w) * win_W * slab;
      } else {
        const double* us = w == 0 ? u0 : ckpt + static_cast<size_t>(w) * P;
        HIP_CHECK(hipMemsetAsync(Uw, 0, static_cast<size_t>(window_len(w)) * slab * sizeof(double), stream));
        stmg_stats sw{};
        rc = sub(w)->solve(us, Uw, &sw);
        if (rc) return rc;
        s.cycles += sw.cycles;
        Uwin = Uw;
      }
      double gn = 0.0;
      stmg_stats sa{};
      double* gout = (w == 0) ? grad_u0 : gw + static_cast<size_t>(w & 1) * P;
      rc = sub(w)->adjoint(nullptr, Uwin, g, gout, &gn, &sa);
      if (rc && rc != STMG_ENOTCONV) return rc;
      s.cycles += sa.cycles;
      s.rel_res = std::max(s.rel_res, sa.rel_res);
      gsum += gn;
      g = gout;
    }
    *grad_nu = gsum;
    s.status = rc;
    s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (st) *st = s;
    return rc;
  }
  if (!U) { set_error("adjoint: forward trajectory required"); return STMG_EINVAL; }
  (void)u0;
  Level& L0 = lv[0];
  stmg_stats s{};
  // ||g||: the right-hand side is cin (x) gT = e_M (x) gT in (reversed) slab 0
  const size_t P = static_cast<size_t>(L0.nx) * L0.ny;
  int np = 0;
  HIP_CHECK(launch_sumsq(gT, P, part, &np, stream));
  HIP_CHECK(launch_sum_partials(part, np, scal + 3, stream));
  double g2 = 0.0;
  int rc = read_scalar(scal + 3, &g2);
  if (rc) return rc;
  HIP_CHECK(hipMemsetAsync(delta64, 0, L0.n * sizeof(double), stream));
  rc = solve_linear(true, REACT_CONST, nullptr, gT, delta64, opt.rtol, std::sqrt(g2), &s.cycles,
                    &s.rel_res);
  if (rc != STMG_OK && rc != STMG_ENOTCONV) return rc;
  // dL/du0 = sum_i l_i(0) lam_{0,i}: forward slab 0 is reversed slab N-1
  HIP_CHECK(launch_node_combine(delta64 + static_cast<size_t>(L0.N - 1) * prob.M * P, lw, prob.M, P,
                                grad_u0, stream));
  // dL/dnu = sum lam dt b_i (Lap U) = (1/nu) sum lam db_i (nu Lap U)
  HIP_CHECK(launch_grad_nu(L0.op, U, delta64, part, &np, stream));
  HIP_CHECK(launch_sum_partials(part, np, scal + 4, stream));
  double gn = 0.0;
  int rc2 = read_scalar(scal + 4, &gn);
  if (rc2) return rc2;
  *grad_nu = gn / prob.nu;
  s.status = rc;
  s.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  if (st) *st = s;
  return rc;
}

// SDC sweeps (Sec. 2.1, 3.1).  One sweep: r_col = Q diag(b)^{-1} r_DG, then
// for m = 1..M:  (I - dt dc_m L) delta_m = r_col,m + dt sum_{j<m} dc_j L delta_j
// with the node solves as batched spatial V-cycles, U_m += delta_m.
int Solver::sdc(const double* u0, double* U, int sweeps, double* h_rel) {
  if (sdcn.empty() || win) {
    set_error("stmg_sdc_sweep: set up the handle with options.sdc = 1");
    return STMG_EUNSUPPORTED;
  }
  const int rc = sdc_core(u0, U, sweeps);
  if (rc) return rc;
  if (h_rel) {
    HIP_CHECK(residual64<double>(false, allen_cahn ? REACT_AC : REACT_CONST, U, nullptr, u0, nullptr, scal));
    double r2 = 0.0;
    const int rc2 = read_scalar(scal, &r2);
    if (rc2) return rc2;
    const double nb = norm_u0_b(u0);
    *h_rel = nb > 0.0 ? std::sqrt(r2) / nb : std::sqrt(r2);
  }
  return STMG_OK;
}

// An inner solve of the SDC sweep or of PFASST: to rtol (relative to the
// first residual when norm_b < 0), or with inner_cap > 0 for at most that
// many V-cycles, the cap being no failure.
int Solver::inner_solve(Solver* S, const double* f, const double* u0, double* U, double norm_b) {
  int cyc = 0;
  double rel = 0.0;
  if (inner_cap <= 0) return S->solve_linear(false, REACT_CONST, f, u0, U, opt.rtol, norm_b, &cyc, &rel);
  const int keep = S->opt.max_cycles;
  S->opt.max_cycles = inner_cap;
  int rc = S->solve_linear(false, REACT_CONST, f, u0, U, opt.rtol, norm_b, &cyc, &rel);
  S->opt.max_cycles = keep;
  if (rc == STMG_ENOTCONV) rc = STMG_OK;
  return rc;
}

int Solver::sdc_core(const double* u0, double* U, int sweeps) {
  Level& L0 = lv[0];
  const int N = L0.N, M = prob.M, P = L0.nx * L0.ny;
  const size_t NP = static_cast<size_t>(N) * P;
  for (int s = 0; s < sweeps; ++s) {
    HIP_CHECK(residual64<double>(false, allen_cahn ? REACT_AC : REACT_CONST, U, nullptr, u0, delta64, scal));
    HIP_CHECK(launch_node_transform(delta64, N, M, P, sdc_G, stream));
    HIP_CHECK(hipMemsetAsync(sdc_acc, 0, NP * sizeof(double), stream));
    for (int m = 0; m < M; ++m) {
      Solver* S = sdcn[m].get();
      double* rhs = S->lv[0].f64;
      HIP_CHECK(launch_sdc_gather(delta64, sdc_acc, rhs, N, M, P, m, stream));
      HIP_CHECK(hipMemsetAsync(S->delta64, 0, NP * sizeof(double), stream));
      // from a zero guess: the stop test is relative to the first residual,
      // which is ||rhs|| (no separate norm pass or host read per node)
      int cyc = 0;
      double rel = 0.0;
      const int rc = inner_solve(S, rhs, nullptr, S->delta64, -1.0);
      if (rc) return rc;
      if (allen_cahn)
        HIP_CHECK(launch_sdc_update_imex(U, sdc_acc, S->delta64, N, M, L0.nx, L0.ny, L0.op.bc, L0.op.cx,
                                         L0.op.cy, L0.op.lam, sdc_w[m], L0.op.gamma,
                                         m + 1 < M ? sdc_w[m + 1] : 0.0, m, stream));
      else
        HIP_CHECK(launch_sdc_update(U, sdc_acc, S->delta64, N, M, L0.nx, L0.ny, L0.op.bc, L0.op.cx,
                                    L0.op.cy, L0.op.lam, sdc_w[m], m, stream));
    }
  }
  return STMG_OK;
}

// explicit instantiations used by the C ABI
template hipError_t Solver::smooth<double>(int, bool, int, const double*, const double*, const double*, double*);
template hipError_t Solver::restrict_residual<double>(int, bool, int, const double*, const double*, const double*, double*, double*, bool*);
template hipError_t Solver::smooth_restrict<double>(bool, int, const double*, const double*, const double*, double*,
                                                    double*, double*, double*, bool*);
template hipError_t Solver::prolong<double>(int, const double*, const double*, double*);
template hipError_t Solver::coarse<double>(bool, int, const double*, const double*, double*);
template hipError_t Solver::residual64<double>(bool, int, const double*, const double*, const double*, double*,
                                               double*);

}  // namespace stmg

namespace stmg {

// Autotuner for the launch shape (slabs per workgroup run) of the restriction
// kernels, level by level: each candidate is a multiple of the coarse level's
// smoother block (so the fused coarse sweep stays possible) and gives bitwise
// identical results; the fastest of three timed launches wins.  Choices are
// kept in a JSON object {"key": slabs} in $STMG_TUNE_CACHE.
namespace {
std::string tune_key(const Solver& s, int l) {
  const Level& F = s.lv[l];
  std::ostringstream k;
  k << (s.mixed ? "f32" : "f64") << "_M" << s.prob.M << "_" << F.nx << "x" << F.ny << "x" << F.N << "_k"
    << F.kind << "_c" << s.chunk_of(l + 1);
  return k.str();
}

}  // namespace

std::map<std::string, int> tune_cache_read(const char* path) {
  std::map<std::string, int> m;
  std::ifstream in(path);
  if (!in) return m;
  std::stringstream ss;
  ss << in.rdbuf();
  const std::string t = ss.str();
  size_t i = 0;
  while ((i = t.find('"', i)) != std::string::npos) {
    const size_t j = t.find('"', i + 1);
    if (j == std::string::npos) break;
    const std::string key = t.substr(i + 1, j - i - 1);
    const size_t c = t.find(':', j);
    if (c == std::string::npos) break;
    m[key] = std::atoi(t.c_str() + c + 1);
    i = t.find_first_of(",}", c);
    if (i == std::string::npos) break;
  }
  return m;
}

void tune_cache_write(const char* path, const std::map<std::string, int>& m) {
  std::ofstream out(path);
  out << "{";
  bool first = true;
  for (const auto& kv : m) {
    out << (first ? "" : ",") << "\n  \"" << kv.first << "\": " << kv.second;
    first = false;
  }
  out << "\n}\n";
}

int Solver::autotune() {
  if (win || lv.size() < 2) return STMG_OK;
  tuned.assign(lv.size(), 0);
  const char* path = std::getenv("STMG_TUNE_CACHE");
  std::map<std::string, int> cache;
  if (path) cache = tune_cache_read(path);
  bool dirty = false;
  hipEvent_t e0, e1;
  HIP_CHECK(hipEventCreate(&e0));
  HIP_CHECK(hipEventCreate(&e1));
  for (size_t l = 0; l + 1 < lv.size(); ++l) {
    const std::string key = tune_key(*this, static_cast<int>(l));
    auto it = cache.find(key);
    if (it != cache.end() && it->second > 0) {
      tuned[l + 1] = it->second;
      continue;
    }
    const int cs = chunk_of(static_cast<int>(l) + 1);
    float best = 1e30f;
    int bestS = 0;
    for (int mult : {1, 2, 4, 8}) {
      const int S = cs * mult;
      if (S > 64 || (mult > 1 && S > lv[l + 1].N)) break;
      tuned[l + 1] = S;
      Level& F = lv[l];
      Level& C = lv[l + 1];
      float tot = 0.0f;
      for (int rep = 0; rep < 4; ++rep) {
        HIP_CHECK(hipEventRecord(e0, stream));
        if (!mixed) {
          const bool zs = l + 2 < lv.size();
          HIP_CHECK(restrict_residual<double>(static_cast<int>(l), false, REACT_CONST, l == 0 ? lv[0].B64 : F.A64,
                                              l == 0 ? nullptr : F.f64, nullptr, C.f64, zs ? C.A64 : nullptr,
                                              nullptr));
        } else {
          const bool zs = l + 2 < lv.size();
          HIP_CHECK(restrict_residual<float>(static_cast<int>(l), false, REACT_CONST, F.A32, F.f32, nullptr,
                                             C.f32, zs ? C.A32 : nullptr, nullptr));
        }
        HIP_CHECK(hipEventRecord(e1, stream));
        HIP_CHECK(hipEventSynchronize(e1));
        float ms = 0.0f;
        HIP_CHECK(hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tot += ms;  // first launch warms up
      }
      if (tot < best) { best = tot; bestS = S; }
    }
    tuned[l + 1] = bestS;
    cache[key] = bestS;
    dirty = true;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (path && dirty) tune_cache_write(path, cache);
  return STMG_OK;
}

template hipError_t Solver::restrict_residual<float>(int, bool, int, const float*, const float*, const double*, float*, float*, bool*);
template hipError_t Solver::smooth_restrict<float>(bool, int, const float*, const float*, const double*, float*,
                                                   float*, float*, double*, bool*);

}  // namespace stmg
