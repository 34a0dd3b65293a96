// Explicit instantiations of the kernel launchers (one unit per family,
// compiled in parallel).
#include "launchers.hpp"

namespace stmg {
template hipError_t launch_residual<double, double>(const OpParams&, int, const SweepPtrs<double>&, int, int*, hipStream_t);
template hipError_t launch_residual<double, float>(const OpParams&, int, const SweepPtrs<double>&, int, int*, hipStream_t);
template hipError_t launch_residual<float, float>(const OpParams&, int, const SweepPtrs<float>&, int, int*, hipStream_t);

}  // namespace stmg
