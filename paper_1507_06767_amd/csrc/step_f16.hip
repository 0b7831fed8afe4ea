// Step-kernel instantiations for shifted IEEE-half storage, rounding to
// nearest and stochastic.
#define LBM_LAUNCH_DEFINITIONS
#include "launch.hpp"

namespace lbm {
template void launch_step_kernel<9, _Float16, float, true>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<9, half_sr, float, true>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<19, _Float16, float, true>(const StepArgs<float> &, const LaunchCfg &);
template void launch_step_kernel<19, half_sr, float, true>(const StepArgs<float> &, const LaunchCfg &);
}  // namespace lbm
