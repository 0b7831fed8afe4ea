// Patch-hierarchy kernel instantiations for one lattice (LBM_Q = 19 or 27)
// and one family of storage types (LBM_PATCH_SET 0: float64, float32,
// shifted float32; 1: the shifted half and bfloat16 storages, rounding to
// nearest or stochastically), so that the families compile in parallel.
#define LBM_PATCH_DEFINITIONS
#include "patch_kernels.hpp"

#if !defined(LBM_Q) || !defined(LBM_PATCH_SET)
#error "compile with -DLBM_Q=19 or -DLBM_Q=27 and -DLBM_PATCH_SET=0 or 1"
#endif

namespace lbm {
#if LBM_PATCH_SET == 0
LBM_INSTANTIATE_PATCH(LBM_Q, double, double, false)
LBM_INSTANTIATE_PATCH(LBM_Q, float, float, false)
LBM_INSTANTIATE_PATCH(LBM_Q, float, float, true)
#else
LBM_INSTANTIATE_PATCH(LBM_Q, _Float16, float, true)
LBM_INSTANTIATE_PATCH(LBM_Q, __bf16, float, true)
LBM_INSTANTIATE_PATCH(LBM_Q, half_sr, float, true)
LBM_INSTANTIATE_PATCH(LBM_Q, bf16_sr, float, true)
#endif
}  // namespace lbm
