// launch.hpp -- host-side launch of the step kernels.
//
// The kernel variants (lattice x storage x sensor kind x collision model x
// tile width x streaming scheme) are instantiated in one translation unit per storage
// family (step_f64.hip, step_f32.hip, step_f16.hip, step_bf16.hip) so that
// they compile in parallel; lbm.hip only sees the declaration.
#pragma once

#include <hip/hip_runtime.h>

#include "step_kernel.hpp"

namespace lbm {

struct LaunchCfg {
    hipStream_t stream;
    int tile_x;        // 32, 64 or 128 cells x 8 rows; kRowTileX: one row, 3D ping-pong
                       // only (step_zmarch: 64)
    int scheme;        // kPingPong, kStream or kLocal
    bool sensor;       // evaluate sensor, block maxima and flags in this step
    int sensor_kind;   // kSensorL2 or kSensorKKn
    bool force;        // body force present
    bool smag;         // Smagorinsky subgrid model on
};

// 3D float64 marches over z inside a workgroup (a 64-bit block maximum
// leaves no room for the arrival count of step_cells); every other form runs
// one cell per thread.
template <int Q, typename C>
constexpr bool uses_zmarch() {
    return Lattice<Q>::D == 3 && sizeof(C) == 8;
}

// Enqueues one step of lattice Q, storage policy T and arithmetic C.
template <int Q, typename T, typename C, bool SH>
void launch_step_kernel(const StepArgs<C> &a, const LaunchCfg &c);

// Enqueues nsteps (1 .. kMultiMaxSteps) sensor-free ping-pong steps of a 2D
// grid as one step_multi launch (a.src -> a.dst); a no-op for 3D lattices
// and stochastic rounding, which the host never sends here.
template <int Q, typename T, typename C, bool SH>
void launch_multi_kernel(const StepArgs<C> &a, int nsteps, const LaunchCfg &c);

#ifdef LBM_LAUNCH_DEFINITIONS
template <bool ZM, int Q, typename T, typename C, bool SH, bool SENS, int SK, int MODEL, int BX, int SCH>
void launch_one(hipStream_t st, const StepArgs<C> &a) {
    constexpr int TY = (BX == kRowTileX) ? 1 : kTileY;
    const dim3 g(a.ntiles), b(BX, TY);
    if constexpr (ZM) hipLaunchKernelGGL((step_zmarch<Q, T, C, SH, SENS, SK, MODEL, BX>), g, b, 0, st, a);
    else hipLaunchKernelGGL((step_cells<Q, T, C, SH, SENS, SK, MODEL, BX, SCH, TY>), g, b, 0, st, a);
}

template <bool ZM, int Q, typename T, typename C, bool SH, bool SENS, int SK, int BX, int SCH>
void launch_model(const StepArgs<C> &a, const LaunchCfg &c) {
    switch ((c.force ? kModelForce : 0) | (c.smag ? kModelSmag : 0)) {
        case kModelForce: launch_one<ZM, Q, T, C, SH, SENS, SK, kModelForce, BX, SCH>(c.stream, a); break;
        case kModelSmag: launch_one<ZM, Q, T, C, SH, SENS, SK, kModelSmag, BX, SCH>(c.stream, a); break;
        case kModelForce | kModelSmag:
            launch_one<ZM, Q, T, C, SH, SENS, SK, kModelForce | kModelSmag, BX, SCH>(c.stream, a);
            break;
        default: launch_one<ZM, Q, T, C, SH, SENS, SK, 0, BX, SCH>(c.stream, a); break;
    }
}

template <bool ZM, int Q, typename T, typename C, bool SH, int BX, int SCH>
void launch_sk(const StepArgs<C> &a, const LaunchCfg &c) {
    if (!c.sensor) launch_model<ZM, Q, T, C, SH, false, kSensorL2, BX, SCH>(a, c);
    else if (c.sensor_kind == kSensorL2) launch_model<ZM, Q, T, C, SH, true, kSensorL2, BX, SCH>(a, c);
    else launch_model<ZM, Q, T, C, SH, true, kSensorKKn, BX, SCH>(a, c);
}

template <int Q, typename T, typename C, bool SH, int BX>
void launch_scheme(const StepArgs<C> &a, const LaunchCfg &c) {
    switch (c.scheme) {
        case kStream: launch_sk<false, Q, T, C, SH, BX, kStream>(a, c); break;
        case kLocal: launch_sk<false, Q, T, C, SH, BX, kLocal>(a, c); break;
        default: launch_sk<false, Q, T, C, SH, BX, kPingPong>(a, c); break;
    }
}

template <int Q, typename T, typename C, bool SH>
void launch_multi_kernel(const StepArgs<C> &a, int nsteps, const LaunchCfg &c) {
    if constexpr (Lattice<Q>::D == 2 && !Storage<T>::sr) {
        const int ntx = (a.nx + kMultiTile - 1) / kMultiTile, nty = (a.ny + kMultiTile - 1) / kMultiTile;
        const dim3 g(ntx * nty), b(kMultiEdge * kMultiEdge);
        switch ((c.force ? kModelForce : 0) | (c.smag ? kModelSmag : 0)) {
            case kModelForce:
                hipLaunchKernelGGL((step_multi<Q, T, C, SH, kModelForce>), g, b, 0, c.stream, a, nsteps);
                break;
            case kModelSmag:
                hipLaunchKernelGGL((step_multi<Q, T, C, SH, kModelSmag>), g, b, 0, c.stream, a, nsteps);
                break;
            case kModelForce | kModelSmag:
                hipLaunchKernelGGL((step_multi<Q, T, C, SH, kModelForce | kModelSmag>), g, b, 0, c.stream, a,
                                   nsteps);
                break;
            default: hipLaunchKernelGGL((step_multi<Q, T, C, SH, 0>), g, b, 0, c.stream, a, nsteps); break;
        }
    } else {
        (void)a, (void)nsteps, (void)c;
    }
}

template <int Q, typename T, typename C, bool SH>
void launch_step_kernel(const StepArgs<C> &a, const LaunchCfg &c) {
    if constexpr (uses_zmarch<Q, C>()) {
        launch_sk<true, Q, T, C, SH, 64, kPingPong>(a, c);
    } else if (Lattice<Q>::D == 3 && c.tile_x == kRowTileX && c.scheme == kPingPong) {
        if constexpr (Lattice<Q>::D == 3) launch_sk<false, Q, T, C, SH, kRowTileX, kPingPong>(a, c);
    } else {
        switch (c.tile_x) {
            case 32: launch_scheme<Q, T, C, SH, 32>(a, c); break;
            case 64: launch_scheme<Q, T, C, SH, 64>(a, c); break;
            default: launch_scheme<Q, T, C, SH, 128>(a, c); break;
        }
    }
}
#endif

}  // namespace lbm
