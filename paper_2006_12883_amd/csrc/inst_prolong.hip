// Explicit instantiations of the kernel launchers (one unit per family,
// compiled in parallel).
#include "launchers.hpp"

namespace stmg {
template hipError_t launch_prolong<double>(const OpParams&, bool, bool, int, int, int, const double*, const double*, double*, int, hipStream_t);
template hipError_t launch_prolong<float>(const OpParams&, bool, bool, int, int, int, const float*, const float*, float*, int, hipStream_t);

}  // namespace stmg
