// Patch-hierarchy kernel instantiations for one lattice (LBM_Q = 19 or 27),
// every storage type the hierarchy supports (float64, float32, shifted
// float32).
#define LBM_PATCH_DEFINITIONS
#include "patch_kernels.hpp"

#if !defined(LBM_Q)
#error "compile with -DLBM_Q=19 or -DLBM_Q=27"
#endif

namespace lbm {
LBM_INSTANTIATE_PATCH(LBM_Q, double, double, false)
LBM_INSTANTIATE_PATCH(LBM_Q, float, float, false)
LBM_INSTANTIATE_PATCH(LBM_Q, float, float, true)
}  // namespace lbm
