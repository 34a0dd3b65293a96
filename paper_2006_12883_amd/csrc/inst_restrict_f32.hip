// Explicit instantiations of the kernel launchers (one unit per family,
// compiled in parallel).
#include "launchers.hpp"

namespace stmg {
template hipError_t launch_restrict_residual<float>(const OpParams&, int, const SweepPtrs<float>&, bool, bool, int, int, int, float*, int, hipStream_t, const OpParams*, float*, const float*, int, bool*);

}  // namespace stmg
