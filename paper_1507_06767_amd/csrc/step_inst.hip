// One step-kernel instantiation per object file.  The build compiles this
// source once per (lattice, storage type, arithmetic type, shifted) with
// LBM_Q, LBM_T, LBM_C and LBM_SH defined, so that the variants compile in
// parallel; lbm.hip only sees the declaration in launch.hpp.
#define LBM_LAUNCH_DEFINITIONS
#include "launch.hpp"

#if !defined(LBM_Q) || !defined(LBM_T) || !defined(LBM_C) || !defined(LBM_SH)
#error "compile with -DLBM_Q=... -DLBM_T=... -DLBM_C=... -DLBM_SH=..."
#endif

namespace lbm {
template void launch_step_kernel<LBM_Q, LBM_T, LBM_C, LBM_SH>(const StepArgs<LBM_C> &, const LaunchCfg &);
template void launch_multi_kernel<LBM_Q, LBM_T, LBM_C, LBM_SH>(const StepArgs<LBM_C> &, int, const LaunchCfg &);
}  // namespace lbm
