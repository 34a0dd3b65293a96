// C ABI of libstmg (declared in include/stmg.h).
#include <mutex>
#include <new>
#include <string>

#include "solver.hpp"

struct stmg_handle {
  stmg::Solver s;
};

namespace stmg {
namespace {
thread_local std::string g_last_error;

// Device scratch of the no-allocation residual (stmg_residual_noalloc): the
// per-block partial sums of ||r||^2 and, in the last slot, their total.  One
// copy per GPU, held until the process ends.  Host code never uses the name
// `scratch` as an address: it takes the device address from
// hipGetSymbolAddress once per device (noalloc_scratch below).
constexpr int kNoAllocParts = 131072;  // 1 MiB of partial sums
static __device__ __align__(256) double scratch[kNoAllocParts + 32];
constexpr int kNoAllocMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[kNoAllocMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first
// call on that device, with the device current).
int noalloc_scratch(double** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kNoAllocMaxDevices) {
    set_error("stmg_residual_noalloc: no usable current device");
    return STMG_EHIP;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      set_error(std::string("stmg_residual_noalloc: hipGetSymbolAddress failed: ") + hipGetErrorString(e));
      return STMG_EHIP;
    }
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return STMG_OK;
}
}  // namespace
void set_error(const std::string& msg) { g_last_error = msg; }
}  // namespace stmg

using stmg::Solver;

extern "C" {

const char* stmg_status_string(int status) {
  switch (status) {
    case STMG_OK: return "ok";
    case STMG_EINVAL: return "invalid argument";
    case STMG_ENOMEM: return "workspace too small";
    case STMG_EHIP: return "HIP runtime error";
    case STMG_ENOTCONV: return "not converged";
    case STMG_EDIVERGED: return "diverged";
    case STMG_ENAN: return "NaN or Inf in residual";
    case STMG_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

const char* stmg_last_error(void) { return stmg::g_last_error.c_str(); }

void stmg_default_options(stmg_options* o) {
  if (!o) return;
  o->precision = STMG_PREC_FP64;
  o->coarsen = STMG_COARSEN_AUTO;
  o->mu_crit = 0.5;
  o->omega = 0.8;
  o->chunk = 16;
  o->chunk_coarse = 4;
  o->nu_pre = 1;
  o->nu_post = 1;
  o->max_levels = 30;
  o->min_coarse = 64;
  o->max_cycles = 200;
  o->rtol = 1e-12;
  o->newton_rtol = 1e-10;
  o->max_newton = 30;
  o->mem_budget = 0;
  o->sdc = 0;
  o->autotune = 0;
  o->inner_cycles = 5;
  o->fft_coarse = 1 << 22;
  o->krylov = 0;
  o->krylov_left = 0;
  o->inner_adapt = 1;
  o->form = STMG_FORM_DG;
  o->smoother = STMG_SMOOTH_PBJ;
  o->coarse_op = STMG_COARSE_REDISC;
  o->pfasst_levels = 0;
  o->pfasst_sweeps = 1;
  o->pfasst_inner_cycles = 0;
}

size_t stmg_workspace_bytes(const stmg_problem* prob, const stmg_options* opt) {
  if (!prob) { stmg::set_error("null problem"); return 0; }
  stmg_options d;
  if (!opt) { stmg_default_options(&d); opt = &d; }
  Solver s;
  if (s.build(prob, opt) != STMG_OK) return 0;
  return s.plan(nullptr);
}

int stmg_setup(const stmg_problem* prob, const stmg_options* opt, void* d_ws, size_t ws_bytes,
               void* stream, stmg_handle** out) {
  if (!prob || !d_ws || !out) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  if (reinterpret_cast<uintptr_t>(d_ws) % 256 != 0) {
    stmg::set_error("workspace must be 256-byte aligned");
    return STMG_EINVAL;
  }
  stmg_options d;
  if (!opt) { stmg_default_options(&d); opt = &d; }
  stmg_handle* h = new (std::nothrow) stmg_handle;
  if (!h) return STMG_ENOMEM;
  int rc = h->s.build(prob, opt);
  if (rc) { delete h; return rc; }
  const size_t need = h->s.plan(nullptr);
  if (ws_bytes < need) {
    stmg::set_error("workspace too small: need " + std::to_string(need) + " bytes");
    delete h;
    return STMG_ENOMEM;
  }
  h->s.stream = static_cast<hipStream_t>(stream);
  h->s.ws_bytes = ws_bytes;
  h->s.plan(static_cast<char*>(d_ws));
  rc = h->s.upload();
  if (rc) { delete h; return rc; }
  if (opt->autotune) {
    rc = h->s.autotune();
    if (rc) { delete h; return rc; }
  }
  *out = h;
  return STMG_OK;
}

int stmg_num_levels(const stmg_handle* h) { return h ? static_cast<int>(h->s.lv.size()) : 0; }

int stmg_level_shape(const stmg_handle* h, int level, int32_t out[4], double* dt) {
  if (!h || !out || level < 0 || level >= static_cast<int>(h->s.lv.size())) {
    stmg::set_error("bad level");
    return STMG_EINVAL;
  }
  const auto& l = h->s.lv[level];
  out[0] = l.nx;
  out[1] = l.ny;
  out[2] = l.N;
  out[3] = l.kind;
  if (dt) *dt = l.dt;
  return STMG_OK;
}

int stmg_level_nodes(const stmg_handle* h, int level) {
  if (!h || level < 0 || level >= static_cast<int>(h->s.lv.size())) {
    stmg::set_error("bad level");
    return STMG_EINVAL;
  }
  return h->s.lv[level].M;
}

int stmg_residual(stmg_handle* h, const double* d_u0, const double* d_U, double* d_r,
                  double* h_norm) {
  if (!h || !d_U) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  return h->s.residual_user(d_u0, d_U, d_r, h_norm);
}

int stmg_residual_noalloc(const stmg_problem* prob, const double* d_u0, const double* d_U,
                          double* d_r, double* h_norm, void* stream) {
  if (!prob || !d_U) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  stmg_options o;
  stmg_default_options(&o);
  // Host-only set-up: the same tables and level-0 operator as stmg_setup builds.
  Solver s;
  int rc = s.build(prob, &o);
  if (rc) return rc;
  const long long parts = s.residual_parts();
  if (parts > stmg::kNoAllocParts) {
    stmg::set_error("stmg_residual_noalloc: problem needs " + std::to_string(parts) +
                    " partial sums, the fixed scratch holds " + std::to_string(stmg::kNoAllocParts));
    return STMG_EINVAL;
  }
  double* ptr = nullptr;
  rc = stmg::noalloc_scratch(&ptr);
  if (rc) return rc;
  s.stream = static_cast<hipStream_t>(stream);
  s.part = ptr;
  s.max_parts = stmg::kNoAllocParts;
  s.scal = ptr + stmg::kNoAllocParts;
  return s.residual_user(d_u0, d_U, d_r, h_norm);
}

int stmg_vcycle(stmg_handle* h, const double* d_u0, double* d_U, double* h_rel) {
  if (!h || !d_U) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  if (!h->s.allen_cahn && !d_u0) { stmg::set_error("null u0"); return STMG_EINVAL; }
  return h->s.vcycle_user(d_u0, d_U, h_rel);
}

int stmg_solve(stmg_handle* h, const double* d_u0, double* d_U, stmg_stats* stats) {
  if (!h || !d_u0 || !d_U) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  return h->s.solve(d_u0, d_U, stats);
}

int stmg_solve_end(stmg_handle* h, const double* d_u0, double* d_uT, stmg_stats* stats) {
  if (!h || !d_u0 || !d_uT) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  return h->s.solve_end(d_u0, d_uT, stats);
}

int stmg_adjoint(stmg_handle* h, const double* d_u0, const double* d_U, const double* d_gT,
                 double* d_grad_u0, double* h_grad_nu, stmg_stats* stats) {
  if (!h || !d_gT || !d_grad_u0 || !h_grad_nu) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  return h->s.adjoint(d_u0, d_U, d_gT, d_grad_u0, h_grad_nu, stats);
}

int stmg_sdc_sweep(stmg_handle* h, const double* d_u0, double* d_U, int32_t sweeps,
                   double* h_rel) {
  if (!h || !d_u0 || !d_U || sweeps < 0) { stmg::set_error("bad argument"); return STMG_EINVAL; }
  return h->s.sdc(d_u0, d_U, sweeps, h_rel);
}

int stmg_pfasst_solve(stmg_handle* h, const double* d_u0, double* d_U, stmg_stats* stats) {
  if (!h || !d_u0 || !d_U) { stmg::set_error("null pointer"); return STMG_EINVAL; }
  return h->s.pfasst(d_u0, d_U, stats);
}

int stmg_num_windows(const stmg_handle* h) { return h ? h->s.nwin : 0; }

int stmg_tuned_shape(const stmg_handle* h, int level) {
  if (!h || level < 0 || level + 1 >= static_cast<int>(h->s.lv.size())) return 0;
  return h->s.transfer_slabs(level + 1);
}

int stmg_level_smooth(stmg_handle* h, int level, const double* d_f, const double* d_u0,
                      const double* d_Uin, double* d_Uout) {
  if (!h || !d_Uout || level < 0 || level >= static_cast<int>(h->s.lv.size())) {
    stmg::set_error("bad argument");
    return STMG_EINVAL;
  }
  if (h->s.win) { stmg::set_error("windowed handle"); return STMG_EUNSUPPORTED; }
  hipError_t e = h->s.smooth<double>(level, false, stmg::REACT_CONST, d_Uin, d_f,
                                     level == 0 ? d_u0 : nullptr, d_Uout);
  return e == hipSuccess ? STMG_OK : STMG_EHIP;
}

int stmg_level_restrict_residual(stmg_handle* h, int level, const double* d_f,
                                 const double* d_u0, const double* d_U, double* d_fc) {
  if (!h || !d_fc || level < 0 || level + 1 >= static_cast<int>(h->s.lv.size())) {
    stmg::set_error("bad argument");
    return STMG_EINVAL;
  }
  if (h->s.win) { stmg::set_error("windowed handle"); return STMG_EUNSUPPORTED; }
  hipError_t e = h->s.restrict_residual<double>(level, false, stmg::REACT_CONST, d_U, d_f,
                                                level == 0 ? d_u0 : nullptr, d_fc, nullptr, nullptr);
  return e == hipSuccess ? STMG_OK : STMG_EHIP;
}

int stmg_level_prolong(stmg_handle* h, int level, const double* d_Uin, const double* d_ec,
                       double* d_Uout) {
  if (!h || !d_ec || !d_Uout || level < 0 || level + 1 >= static_cast<int>(h->s.lv.size())) {
    stmg::set_error("bad argument");
    return STMG_EINVAL;
  }
  if (h->s.win) { stmg::set_error("windowed handle"); return STMG_EUNSUPPORTED; }
  hipError_t e = h->s.prolong<double>(level, d_Uin, d_ec, d_Uout);
  return e == hipSuccess ? STMG_OK : STMG_EHIP;
}

int stmg_level_prolong_smooth(stmg_handle* h, int level, const double* d_f, const double* d_u0,
                              const double* d_Uin, const double* d_ec, double* d_Uout) {
  if (!h || !d_ec || !d_Uout || level < 0 || level + 1 >= static_cast<int>(h->s.lv.size())) {
    stmg::set_error("bad argument");
    return STMG_EINVAL;
  }
  if (h->s.win) { stmg::set_error("windowed handle"); return STMG_EUNSUPPORTED; }
  if (!stmg::blocked_layout(h->s.lv[level].op)) {
    stmg::set_error("fused prolongation + smoothing: periodic grids with even point counts only");
    return STMG_EUNSUPPORTED;
  }
  hipError_t e = h->s.prolong_smooth<double>(level, false, stmg::REACT_CONST, d_Uin, d_ec, d_f,
                                             level == 0 ? d_u0 : nullptr, d_Uout);
  return e == hipSuccess ? STMG_OK : STMG_EHIP;
}

int stmg_level_smooth_restrict(stmg_handle* h, int level, const double* d_f, const double* d_u0,
                               const double* d_Uin, double* d_Uout, double* d_fc, double* d_uc) {
  if (!h || !d_Uout || !d_fc || level != 0 || h->s.lv.size() < 2) {
    stmg::set_error("bad argument");
    return STMG_EINVAL;
  }
  if (h->s.win) { stmg::set_error("windowed handle"); return STMG_EUNSUPPORTED; }
  if (h->s.allen_cahn || !h->s.sr_usable(stmg::REACT_CONST, true)) {
    stmg::set_error("fused smoothing + restriction: 2D periodic linear problems with space coarsening on level 0, "
                    "nx a multiple of 64, ny of 16, M <= 4, the smoother chunk a multiple of the coarse one");
    return STMG_EUNSUPPORTED;
  }
  hipError_t e = h->s.smooth_restrict<double>(false, stmg::REACT_CONST, d_Uin, d_f, d_u0, d_Uout, d_fc, d_uc, nullptr,
                                              nullptr);
  return e == hipSuccess ? STMG_OK : STMG_EHIP;
}

int stmg_coarse_solve(stmg_handle* h, const double* d_f, double* d_U) {
  if (!h || !d_U) { stmg::set_error("bad argument"); return STMG_EINVAL; }
  if (h->s.win) { stmg::set_error("windowed handle"); return STMG_EUNSUPPORTED; }
  hipError_t e = h->s.coarse<double>(false, stmg::REACT_CONST, d_f, nullptr, d_U);
  return e == hipSuccess ? STMG_OK : STMG_EHIP;
}

void stmg_destroy(stmg_handle* h) { delete h; }



}  // extern "C"
