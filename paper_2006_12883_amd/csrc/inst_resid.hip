// Explicit instantiations of the kernel launchers (one unit per family,
// compiled in parallel).
#include "launchers.hpp"

namespace stmg {
template hipError_t launch_residual<double, double>(const OpParams&, int, const SweepPtrs<double>&, int, int*, hipStream_t);
template hipError_t launch_residual<double, float>(const OpParams&, int, const SweepPtrs<double>&, int, int*, hipStream_t);
template hipError_t launch_residual<float, float>(const OpParams&, int, const SweepPtrs<float>&, int, int*, hipStream_t);

hipError_t launch_refine(const OpParams& p, int react, const SweepPtrs<double>& a, const float* e,
                         float* r32, float* e1, const float* coef32, int chunk, int* nparts,
                         hipStream_t s) {
  if (!blocked(p)) return hipErrorNotSupported;
  if (react != REACT_CONST && react != REACT_COEF) return hipErrorInvalidValue;
  if (chunk < 1) return hipErrorInvalidValue;
  const int tiles = (plane_threads(p) + kBlock - 1) / kBlock;
  const int nb = tiles * ((p.N + chunk - 1) / chunk);
  if (nparts) *nparts = nb;
#define LB(MM, RE, BYc, TWc)                                                                    \
  hipLaunchKernelGGL((k_refine_blk<MM, RE, BYc, TWc>), dim3(nb), dim3(kBlock), 0, s, p, a, e, r32, \
                     e1, coef32, chunk, tiles, nb)
#define L(MM)                                                                            \
  if (p.ny > 1) {                                                                        \
    if (react == REACT_COEF) LB(MM, REACT_COEF, 2, true); else LB(MM, REACT_CONST, 2, true); \
  } else {                                                                               \
    if (react == REACT_COEF) LB(MM, REACT_COEF, 1, false); else LB(MM, REACT_CONST, 1, false); \
  }
  STMG_DISPATCH_M(L)
#undef L
#undef LB
  return hipGetLastError();
}

}  // namespace stmg
