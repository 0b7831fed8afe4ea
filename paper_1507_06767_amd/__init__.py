"""MI355X lattice Boltzmann step fused with the kinetic mesh-refinement sensor.

The compute lives in the HIP library ``liblbm.so`` (sources in ``csrc/``,
interface in ``include/lbm.h``).  This package is its Python binding: the
functions of ``abi`` carry the C names and only marshal arguments, and
``Blocks`` sizes and allocates the caller-owned device buffers as torch
tensors.  Nothing here computes any part of the method.  If the library has
not been built the import of ``abi`` raises.
"""
from .abi import (  # noqa: F401
    LbmError, LBM_OK, LBM_EINVAL, LBM_ENOTSUP, LBM_EHIP, LBM_ESTATE, LBM_ENONFINITE,
    LBM_D2Q9, LBM_D3Q19, LBM_D3Q27, LBM_F64, LBM_F32, LBM_F32_SHIFTED, LBM_F16_SHIFTED, LBM_BF16_SHIFTED,
    LBM_F16_SHIFTED_SR, LBM_BF16_SHIFTED_SR,
    LBM_SENSOR_L2, LBM_SENSOR_KKN,
    LBM_BC_PERIODIC, LBM_BC_WALL, LBM_PROFILE_UNIFORM, LBM_PROFILE_SMOOTH,
    LBM_STREAMING_AUTO, LBM_STREAMING_PINGPONG, LBM_STREAMING_INPLACE, lbm_desc, lbm_box, make_desc, library_path,
    lbm_required_bytes, lbm_create_blocks, lbm_step_n, lbm_sensor_flags, lbm_get_macros, lbm_block_means,
    lbm_get_populations, lbm_set_populations, lbm_set_equilibrium, lbm_get_step, lbm_set_step, lbm_get_scheme,
    lbm_set_multistep, lbm_get_multistep,
    lbm_conservation, lbm_tau_from_reynolds, lbm_destroy, lbm_last_error,
    lbm_sensor_levels, lbm_sensor_average_begin, lbm_sensor_average, lbm_sensor_average_end,
    lbm_autotune, lbm_use_graphs, lbm_hierarchy_required_bytes, lbm_create_hierarchy, lbm_hierarchy_step, lbm_hierarchy_sensor,
    lbm_hierarchy_patch_fields, lbm_hierarchy_info, lbm_hierarchy_autotune, lbm_hierarchy_profile,
    lbm_destroy_hierarchy,
)
from .blocks import Blocks  # noqa: F401
from .hierarchy import Hierarchy  # noqa: F401
