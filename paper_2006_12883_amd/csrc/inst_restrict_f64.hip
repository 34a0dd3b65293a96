// Explicit instantiations of the kernel launchers (one unit per family,
// compiled in parallel).
#include "launchers.hpp"

namespace stmg {
template hipError_t launch_restrict_residual<double>(const OpParams&, int, const SweepPtrs<double>&, bool, bool, int, int, int, double*, int, hipStream_t, const OpParams*, double*, const double*, int, bool*);

}  // namespace stmg
