// Step-kernel instantiations for shifted bfloat16 storage, rounding to
// nearest and stochastic.
#define LBM_LAUNCH_DEFINITIONS
#include "launch.hpp"

namespace lbm {
template void launch_step_kernel<9, __bf16, float, true>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<9, bf16_sr, float, true>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<19, __bf16, float, true>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<19, bf16_sr, float, true>(const StepArgs<float> &, const LaunchCfg &);
}  // namespace lbm
