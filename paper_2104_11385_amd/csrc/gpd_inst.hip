// One group of gather-push-deposit kernels: precision PB_GPD_REAL, shape
// order PB_GPD_ORDER (every compiled tile shape, both particle orders, and
// the global-path kernel).  The build compiles this file once per group, in
// parallel.
#include "gpd_kernel.hpp"

#if !defined(PB_GPD_REAL) || !defined(PB_GPD_ORDER)
#error "PB_GPD_REAL and PB_GPD_ORDER must be defined"
#endif

namespace pb {
template hipError_t gpd_tile<PB_GPD_REAL, PB_GPD_ORDER>(const GpdLaunch &, hipStream_t);
template hipError_t gpd_global<PB_GPD_REAL, PB_GPD_ORDER>(const GpdLaunch &, int, unsigned, hipStream_t);
}  // namespace pb
