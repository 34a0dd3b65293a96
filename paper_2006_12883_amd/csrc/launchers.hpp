// Kernel launchers (templates; instantiated in the inst_*.hip units).
#pragma once
#include "kernels_impl.hpp"

namespace stmg {

// ---------------------------------------------------------------------------
// Launchers: dispatch on M and on the reaction mode.
#define STMG_DISPATCH_M(MACRO) \
  switch (p.M) {               \
    case 1: MACRO(1); break;   \
    case 2: MACRO(2); break;   \
    case 3: MACRO(3); break;   \
    case 4: MACRO(4); break;   \
    case 5: MACRO(5); break;   \
    case 6: MACRO(6); break;   \
    case 7: MACRO(7); break;   \
    case 8: MACRO(8); break;   \
    default: return hipErrorInvalidValue; \
  }

// The register-blocked kernels cover periodic grids with even point counts.
inline bool blocked(const OpParams& p) {
  return p.bc == 0 && (p.nx % 2) == 0 && (p.ny == 1 || (p.ny % 2) == 0);
}
inline int plane_threads(const OpParams& p) {
  if (blocked(p)) return (p.nx / 2) * (p.ny > 1 ? p.ny / 2 : 1);
  return p.nx * p.ny;
}

// Slab-parallel kernels (one slab of a smoother chunk per thread) serve the
// small levels, where a thread marching through its slabs waits on one
// memory round trip per slab.  Returns the workgroup's slab count (the chunk,
// or the next power of two >= N when one chunk holds every slab), or 0 when
// the level is large or the chunk is not a power of two.  Every wave must
// lie inside one slab (the kernels address each slab's planes through a
// wave-uniform base), so a workgroup holds at most kBlock / 64 slabs.
// level sizes (points x slabs) up to which the slab-parallel form is faster
constexpr long long kSlabParallelMaxWork = 1LL << 19;          // prolongation + smoothing
constexpr long long kSlabParallelMaxWorkRestrict = 1LL << 20;  // time restriction
constexpr size_t kSlabParallelLds = 64 * 1024;
constexpr int kSlabParallelMaxLen = kBlock / 64;
inline int slab_parallel_len(int M, long long work, int nslabs, int chunk,
                             long long max_work = kSlabParallelMaxWork) {
  if (M > 4 || chunk < 1 || (chunk & (chunk - 1)) != 0) return 0;
  if (work > max_work) return 0;
  int sl = chunk;
  while (sl > 1 && (sl >> 1) >= nslabs) sl >>= 1;
  return (sl >= 2 && sl <= kSlabParallelMaxLen) ? sl : 0;
}
inline long long level_work(const OpParams& p) { return (long long)p.nx * p.ny * p.N; }





template <typename T>
hipError_t launch_smooth(const OpParams& p, int react, const SweepPtrs<T>& a, int chunk,
                         hipStream_t s) {
  const int nb = smooth_blocks(p, chunk);
  const int tiles = (plane_threads(p) + kBlock - 1) / kBlock;
  if (blocked(p)) {
#define LB(MM, RE, BYc, TWc) \
  hipLaunchKernelGGL((k_smooth_blk<MM, T, RE, BYc, TWc>), dim3(nb), dim3(kBlock), 0, s, p, a, chunk, tiles, nb)
#define L(MM)                                                                 \
  if (p.ny > 1) { if (react == REACT_COEF) LB(MM, REACT_COEF, 2, true); else LB(MM, REACT_CONST, 2, true); } \
  else { if (react == REACT_COEF) LB(MM, REACT_COEF, 1, false); else LB(MM, REACT_CONST, 1, false); }
    STMG_DISPATCH_M(L)
#undef L
#undef LB
    return hipGetLastError();
  }
#define L(MM)                                                                                   \
  if (react == REACT_COEF)                                                                      \
    hipLaunchKernelGGL((k_smooth<MM, T, REACT_COEF>), dim3(nb), dim3(kBlock), 0, s, p, a, chunk, \
                       tiles, nb);                                                              \
  else                                                                                          \
    hipLaunchKernelGGL((k_smooth<MM, T, REACT_CONST>), dim3(nb), dim3(kBlock), 0, s, p, a,       \
                       chunk, tiles, nb);
  STMG_DISPATCH_M(L)
#undef L
  return hipGetLastError();
}

template <typename T, typename TO>
hipError_t launch_residual(const OpParams& p, int react, const SweepPtrs<T>& a, int spb,
                           int* nparts, hipStream_t s) {
  const int tiles = (plane_threads(p) + kBlock - 1) / kBlock;
  const int chunks = (p.N + spb - 1) / spb;
  const int nb = tiles * chunks;
  if (nparts) *nparts = nb;
  if (blocked(p)) {
#define LB(MM, RE, BYc, TWc)                                                                     \
  hipLaunchKernelGGL((k_residual_blk<MM, T, TO, RE, BYc, TWc>), dim3(nb), dim3(kBlock), 0, s, p, a, \
                     spb, tiles, nb)
#define LBR(MM, BYc, TWc)                                                    \
  if (react == REACT_COEF) LB(MM, REACT_COEF, BYc, TWc);                     \
  else if (react == REACT_AC) LB(MM, REACT_AC, BYc, TWc);                    \
  else LB(MM, REACT_CONST, BYc, TWc);
#define L(MM) \
  if (p.ny > 1) { LBR(MM, 2, true) } else { LBR(MM, 1, false) }
    STMG_DISPATCH_M(L)
#undef L
#undef LBR
#undef LB
    return hipGetLastError();
  }
#define L(MM)                                                                                    \
  if (react == REACT_COEF)                                                                       \
    hipLaunchKernelGGL((k_residual<MM, T, TO, REACT_COEF>), dim3(nb), dim3(kBlock), 0, s, p, a,   \
                       spb, tiles, nb);                                                          \
  else if (react == REACT_AC)                                                                    \
    hipLaunchKernelGGL((k_residual<MM, T, TO, REACT_AC>), dim3(nb), dim3(kBlock), 0, s, p, a,     \
                       spb, tiles, nb);                                                          \
  else                                                                                           \
    hipLaunchKernelGGL((k_residual<MM, T, TO, REACT_CONST>), dim3(nb), dim3(kBlock), 0, s, p, a,  \
                       spb, tiles, nb);
  STMG_DISPATCH_M(L)
#undef L
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_residual(const OpParams& p, int react, const SweepPtrs<T>& a,
                                    bool space, bool time, int ncx, int ncy, int Nc, T* fc,
                                    int spb, hipStream_t s, const OpParams* pc, T* uc,
                                    const T* coefc, int cs, bool* smoothed) {
  const bool twod = p.ny > 1;
  if (smoothed) *smoothed = false;
  if (space && blocked(p) && p.M <= 4) {
    const bool zs = uc != nullptr && pc != nullptr && cs >= 1 && (spb % cs) == 0;
    if (smoothed) *smoothed = zs;
    const OpParams& pcc = zs ? *pc : p;
    // register-blocked fine tiles, 32 x 8 coarse points (2D: 512-byte fine
    // row segments) or 256 (1D)
    const int tcx = twod ? 32 : 256;
    const int tcy = twod ? 8 : 1;
    const int tiles_x = (ncx + tcx - 1) / tcx;
    const int tiles = tiles_x * ((ncy + tcy - 1) / tcy);
    const int nb = tiles * ((Nc + spb - 1) / spb);
#define LRB(MM, RE, TMc, TWc, CX, CY)                                                            \
  if (zs)                                                                                           \
    hipLaunchKernelGGL((k_restrict_blk<MM, T, RE, TMc, TWc, CX, CY, true>), dim3(nb), dim3(kBlock), 0, \
                       s, p, a, ncx, ncy, Nc, fc, spb, tiles_x, tiles, nb, pcc, uc, coefc, cs);     \
  else                                                                                              \
    hipLaunchKernelGGL((k_restrict_blk<MM, T, RE, TMc, TWc, CX, CY, false>), dim3(nb), dim3(kBlock), 0, \
                       s, p, a, ncx, ncy, Nc, fc, spb, tiles_x, tiles, nb, pcc, uc, coefc, cs)
#define LRBE(MM, RE)                                          \
  if (twod) {                                                 \
    if (time) LRB(MM, RE, true, true, 32, 8);                 \
    else LRB(MM, RE, false, true, 32, 8);                     \
  } else {                                                    \
    if (time) LRB(MM, RE, true, false, 256, 1);               \
    else LRB(MM, RE, false, false, 256, 1);                   \
  }
#define LB4(MM) \
  if (react == REACT_COEF) { LRBE(MM, REACT_COEF) } else { LRBE(MM, REACT_CONST) }
    switch (p.M) {
      case 1: LB4(1); break;
      case 2: LB4(2); break;
      case 3: LB4(3); break;
      case 4: LB4(4); break;
      default: return hipErrorInvalidValue;
    }
#undef LB4
#undef LRBE
#undef LRB
    return hipGetLastError();
  }
  if (space) {
    // LDS-tiled kernel: coarse tiles of 16 x 16 (M <= 4) or 16 x 8 in 2D, 256 in 1D
    const int tcx = twod ? 16 : 256;
    const int tcy = twod ? (p.M <= 4 ? 16 : 8) : 1;
    const int tiles_x = (ncx + tcx - 1) / tcx;
    const int tiles_y = (ncy + tcy - 1) / tcy;
    const int tiles = tiles_x * tiles_y;
    const int chunks = (Nc + spb - 1) / spb;
    const int nb = tiles * chunks;
#define LRS(MM, RE, TMc, TWc, CX, CY)                                                        \
  hipLaunchKernelGGL((k_restrict_lds<MM, T, RE, TMc, TWc, CX, CY>), dim3(nb), dim3(kBlock), 0, s, \
                     p, a, ncx, ncy, Nc, fc, spb, tiles_x, tiles, nb)
#define LRSE(MM, RE, CY)                                     \
  if (twod) {                                                \
    if (time) LRS(MM, RE, true, true, 16, CY);               \
    else LRS(MM, RE, false, true, 16, CY);                   \
  } else {                                                   \
    if (time) LRS(MM, RE, true, false, 256, 1);              \
    else LRS(MM, RE, false, false, 256, 1);                  \
  }
#define L(MM)                                                                     \
  if (react == REACT_COEF) { LRSE(MM, REACT_COEF, (MM <= 4 ? 16 : 8)) }           \
  else { LRSE(MM, REACT_CONST, (MM <= 4 ? 16 : 8)) }
    STMG_DISPATCH_M(L)
#undef L
#undef LRSE
#undef LRS
    return hipGetLastError();
  }
  if (!space && time && blocked(p)) {
    const bool want_zs = uc != nullptr && pc != nullptr && cs >= 1;
    const int sl = slab_parallel_len(p.M, level_work(p), Nc, want_zs ? cs : kSlabParallelMaxLen,
                                    kSlabParallelMaxWorkRestrict);
    const int NP = twod ? 4 : 2;
    const size_t lds = (size_t)kBlock * NP *
                       (p.M + 1 + (react == REACT_COEF && want_zs ? p.M : 0)) * sizeof(T);
    if (sl > 0 && lds <= kSlabParallelLds) {
      if (smoothed) *smoothed = want_zs;
      const OpParams& pcc = want_zs ? *pc : p;
      const int nbk = kBlock / sl;
      const int tiles = (plane_threads(p) + nbk - 1) / nbk;
      const int nb = tiles * ((Nc + sl - 1) / sl);
#define LT(MM, RE, BYc, TWc)                                                                       \
  if (want_zs)                                                                                      \
    hipLaunchKernelGGL((k_restrict_t_sp<MM, T, RE, BYc, TWc, true>), dim3(nb), dim3(kBlock), lds, s, p, \
                       a, Nc, fc, sl, tiles, nb, pcc, uc, coefc, cs);                               \
  else                                                                                              \
    hipLaunchKernelGGL((k_restrict_t_sp<MM, T, RE, BYc, TWc, false>), dim3(nb), dim3(kBlock), lds, s, p, \
                       a, Nc, fc, sl, tiles, nb, pcc, uc, coefc, cs)
#define LTS(MM, RE) \
  if (twod) { LT(MM, RE, 2, true); } else { LT(MM, RE, 1, false); }
#define L(MM) \
  if (react == REACT_COEF) { LTS(MM, REACT_COEF) } else { LTS(MM, REACT_CONST) }
      switch (p.M) {
        case 1: L(1); break;
        case 2: L(2); break;
        case 3: L(3); break;
        case 4: L(4); break;
        default: return hipErrorInvalidValue;
      }
#undef L
#undef LTS
#undef LT
      return hipGetLastError();
    }
    const bool zs = want_zs && (spb % cs) == 0;
    if (smoothed) *smoothed = zs;
    const OpParams& pcc = zs ? *pc : p;
    const int tiles = (plane_threads(p) + kBlock - 1) / kBlock;
    const int nb = tiles * ((Nc + spb - 1) / spb);
#define LT(MM, RE, BYc, TWc)                                                                       \
  if (zs)                                                                                           \
    hipLaunchKernelGGL((k_restrict_t_blk<MM, T, RE, BYc, TWc, true>), dim3(nb), dim3(kBlock), 0, s, p, a, \
                       Nc, fc, spb, tiles, nb, pcc, uc, coefc, cs);                                 \
  else                                                                                              \
    hipLaunchKernelGGL((k_restrict_t_blk<MM, T, RE, BYc, TWc, false>), dim3(nb), dim3(kBlock), 0, s, p, a, \
                       Nc, fc, spb, tiles, nb, pcc, uc, coefc, cs)
#define LTS(MM, RE) \
  if (twod) { LT(MM, RE, 2, true); } else { LT(MM, RE, 1, false); }
#define L(MM) \
  if (react == REACT_COEF) { LTS(MM, REACT_COEF) } else { LTS(MM, REACT_CONST) }
    STMG_DISPATCH_M(L)
#undef L
#undef LTS
#undef LT
    return hipGetLastError();
  }
  const int Pc = ncx * ncy;
  const int tiles = (Pc + kBlock - 1) / kBlock;
  const int chunks = (Nc + spb - 1) / spb;
  const int nb = tiles * chunks;
#define LR(MM, RE, TMc)                                                                        \
  hipLaunchKernelGGL((k_restrict<MM, T, RE, false, TMc, false>), dim3(nb), dim3(kBlock), 0, s, p, \
                     a, ncx, ncy, Nc, fc, spb, tiles, nb)
#define L(MM)                                                             \
  if (react == REACT_COEF) { if (time) LR(MM, REACT_COEF, true); else LR(MM, REACT_COEF, false); } \
  else { if (time) LR(MM, REACT_CONST, true); else LR(MM, REACT_CONST, false); }
  STMG_DISPATCH_M(L)
#undef L
#undef LR
  return hipGetLastError();
}

template <typename T>
hipError_t launch_prolong(const OpParams& p, bool space, bool time, int ncx, int ncy, int Nc,
                          const T* ec, const T* Uin, T* Uout, int spb, hipStream_t s) {
  const bool twod = p.ny > 1;
  const int tiles = (plane_threads(p) + kBlock - 1) / kBlock;
  const int chunks = (p.N + spb - 1) / spb;
  const int nb = tiles * chunks;
  if (blocked(p)) {
#define LPB(MM, SPc, TMc, BYc, TWc)                                                             \
  hipLaunchKernelGGL((k_prolong_blk<MM, T, SPc, TMc, BYc, TWc>), dim3(nb), dim3(kBlock), 0, s, p, \
                     ncx, ncy, Nc, ec, Uin, Uout, spb, tiles, nb)
#define LPS(MM, BYc, TWc)                                 \
  if (space && time) LPB(MM, true, true, BYc, TWc);       \
  else if (space) LPB(MM, true, false, BYc, TWc);         \
  else if (time) LPB(MM, false, true, BYc, TWc);          \
  else LPB(MM, false, false, BYc, TWc);
#define L(MM) \
  if (twod) { LPS(MM, 2, true) } else { LPS(MM, 1, false) }
    STMG_DISPATCH_M(L)
#undef L
#undef LPS
#undef LPB
    return hipGetLastError();
  }
#define LP(MM, SPc, TMc, TWc)                                                                  \
  hipLaunchKernelGGL((k_prolong<MM, T, SPc, TMc, TWc>), dim3(nb), dim3(kBlock), 0, s, p, ncx, ncy, \
                     Nc, ec, Uin, Uout, spb, tiles, nb)
#define L(MM)                                                            \
  if (space && time) {                                                   \
    if (twod) LP(MM, true, true, true); else LP(MM, true, true, false);  \
  } else if (space) {                                                    \
    if (twod) LP(MM, true, false, true); else LP(MM, true, false, false); \
  } else if (time) {                                                     \
    LP(MM, false, true, false);                                          \
  } else {                                                               \
    LP(MM, false, false, false);                                         \
  }
  STMG_DISPATCH_M(L)
#undef L
#undef LP
  return hipGetLastError();
}


template <typename T>
hipError_t launch_prolong_smooth(const OpParams& p, int react, const SweepPtrs<T>& a, bool space,
                                 bool time, int ncx, int ncy, int Nc, const T* ec, int chunk,
                                 hipStream_t s) {
  if (!blocked(p)) return hipErrorNotSupported;
  const bool twod = p.ny > 1;
  const int sl = slab_parallel_len(p.M, level_work(p), p.N, chunk);
  const int NP = twod ? 4 : 2;
  const size_t lds = (size_t)kBlock * NP * (p.M + 1 + (react == REACT_COEF ? p.M : 0)) * sizeof(T);
  if (sl > 0 && a.part == nullptr && a.up64 == nullptr && lds <= kSlabParallelLds) {
    const int nbk = kBlock / sl;
    const int tiles = (plane_threads(p) + nbk - 1) / nbk;
    const int nb = tiles * ((p.N + sl - 1) / sl);
#define LF(MM, RE, SPc, TMc, BYc, TWc)                                                           \
  hipLaunchKernelGGL((k_prolong_smooth_sp<MM, T, RE, SPc, TMc, BYc, TWc>), dim3(nb), dim3(kBlock), \
                     lds, s, p, a, ncx, ncy, ec, sl, tiles, nb)
#define LFS(MM, RE, BYc, TWc)                                   \
  if (space && time) LF(MM, RE, true, true, BYc, TWc);          \
  else if (space) LF(MM, RE, true, false, BYc, TWc);            \
  else LF(MM, RE, false, true, BYc, TWc);
#define LFR(MM, RE) \
  if (twod) { LFS(MM, RE, 2, true) } else { LFS(MM, RE, 1, false) }
#define L(MM) \
  if (react == REACT_COEF) { LFR(MM, REACT_COEF) } else { LFR(MM, REACT_CONST) }
    switch (p.M) {
      case 1: L(1); break;
      case 2: L(2); break;
      case 3: L(3); break;
      case 4: L(4); break;
      default: return hipErrorInvalidValue;
    }
#undef L
#undef LFR
#undef LFS
#undef LF
    return hipGetLastError();
  }
  const int nb = smooth_blocks(p, chunk);
  const int tiles = (plane_threads(p) + kBlock - 1) / kBlock;
  // x neighbours exchanged between lanes (2D, nx a multiple of 4; M = 3,
  // where it cuts the loads per slab without costing a wave per SIMD)
  const bool xs = twod && (p.nx % 4) == 0;
#define LF(MM, RE, SPc, TMc, BYc, TWc, XSc)                                                          \
  hipLaunchKernelGGL((k_prolong_smooth_blk<MM, T, RE, SPc, TMc, BYc, TWc, XSc>), dim3(nb), dim3(kBlock), \
                     0, s, p, a, ncx, ncy, Nc, ec, chunk, tiles, nb)
#define LFS(MM, RE, BYc, TWc, XSc)                                   \
  if (space && time) LF(MM, RE, true, true, BYc, TWc, XSc);          \
  else if (space) LF(MM, RE, true, false, BYc, TWc, XSc);            \
  else LF(MM, RE, false, true, BYc, TWc, XSc);
#define LFR(MM, RE)                                                   \
  if (twod && xs) { LFS(MM, RE, 2, true, (MM == 3)) }                \
  else if (twod) { LFS(MM, RE, 2, true, false) }                      \
  else { LFS(MM, RE, 1, false, false) }
#define L(MM) \
  if (react == REACT_COEF) { LFR(MM, REACT_COEF) } else { LFR(MM, REACT_CONST) }
  STMG_DISPATCH_M(L)
#undef L
#undef LFR
#undef LFS
#undef LF
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve(const OpParams& p, const double* Ainv, const T* f,
                               const double* u0, T* U, hipStream_t s) {
  const int P = p.nx * p.ny;
  const size_t shm = (size_t)(2 * p.M * P + P) * sizeof(double);
  bool coupled = false;
  for (int i = 0; i < p.M; ++i) coupled = coupled || p.cin[i] != 0.0;
  const int grid = (!coupled && !u0) ? p.N : 1;  // independent slabs in parallel
  hipLaunchKernelGGL((k_coarse_solve<T>), dim3(grid), dim3(kBlock), shm, s, p, Ainv, f, u0, U);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_coarse_solve_coef(const OpParams& p, const T* coef, double* scratch, const T* f,
                                    const double* u0, T* U, hipStream_t s) {
  const int P = p.nx * p.ny;
  const int K = p.M * P;
  const size_t shm = (size_t)(K + P) * sizeof(double) + (size_t)K * sizeof(int);
  hipLaunchKernelGGL((k_coarse_solve_coef<T>), dim3(1), dim3(kBlock), shm, s, p, coef, scratch, f,
                     u0, U);
  return hipGetLastError();
}





template <typename TX, typename TY>
hipError_t launch_axpy_cast(size_t n, const TX* x, double alpha, TY* y, bool acc, hipStream_t s) {
  hipLaunchKernelGGL((k_axpy_cast<TX, TY>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, x, alpha, y,
                     acc ? 1 : 0);
  return hipGetLastError();
}

template <typename TE>
hipError_t launch_update(size_t n, double* U, const TE* e, const double* scale, hipStream_t s) {
  hipLaunchKernelGGL((k_update<TE>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, U, e, scale);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_newton_coef(size_t n, const double* U, double gamma, T* coef, hipStream_t s) {
  hipLaunchKernelGGL((k_newton_coef<T>), dim3(grid_for(n)), dim3(kBlock), 0, s, n, U, gamma, coef);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_restrict_coef(const OpParams& fine, bool space, bool time, int ncx, int ncy,
                                int Nc, const T* cf, T* cc, hipStream_t s) {
  const size_t total = (size_t)Nc * fine.M * ncx * ncy;
  hipLaunchKernelGGL((k_restrict_coef<T>), dim3(grid_for(total)), dim3(kBlock), 0, s, fine,
                     space ? 1 : 0, time ? 1 : 0, ncx, ncy, Nc, cf, cc);
  return hipGetLastError();
}







}  // namespace stmg
