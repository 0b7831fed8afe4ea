// Step-kernel instantiations for float64 storage.
#define LBM_LAUNCH_DEFINITIONS
#include "launch.hpp"

namespace lbm {
template void launch_step_kernel<9, double, double, false>(const StepArgs<double> &, const LaunchCfg &);
template void launch_step_kernel<19, double, double, false>(const StepArgs<double> &, const LaunchCfg &);
}  // namespace lbm
