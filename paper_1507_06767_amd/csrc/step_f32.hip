// Step-kernel instantiations for float32 storage, plain and shifted.
#define LBM_LAUNCH_DEFINITIONS
#include "launch.hpp"

namespace lbm {
template void launch_step_kernel<9, float, float, false>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<9, float, float, true>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<19, float, float, false>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<19, float, float, true>(const StepArgs<float> &, const LaunchCfg &);
}  // namespace lbm
