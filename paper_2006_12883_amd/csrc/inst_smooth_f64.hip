// Explicit instantiations of the kernel launchers (one unit per family,
// compiled in parallel).
#include "launchers.hpp"

namespace stmg {
template hipError_t launch_smooth<double>(const OpParams&, int, const SweepPtrs<double>&, int, hipStream_t);
template hipError_t launch_prolong_smooth<double>(const OpParams&, int, const SweepPtrs<double>&, bool, bool, int, int, int, const double*, int, hipStream_t);

}  // namespace stmg
