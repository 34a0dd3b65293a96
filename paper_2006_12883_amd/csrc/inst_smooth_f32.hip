// Explicit instantiations of the kernel launchers (one unit per family,
// compiled in parallel).
#include "launchers.hpp"

namespace stmg {
template hipError_t launch_smooth<float>(const OpParams&, int, const SweepPtrs<float>&, int, hipStream_t);
template hipError_t launch_prolong_smooth<float>(const OpParams&, int, const SweepPtrs<float>&, bool, bool, int, int, int, const float*, int, hipStream_t);

}  // namespace stmg
