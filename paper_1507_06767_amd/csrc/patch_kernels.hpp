// patch_kernels.hpp -- kernels of the two-level patch hierarchy: a batch of
// fine patches (refinement factor 2) over a coarse grid, advanced in one
// persistent launch per fine step.
//
// Coupling (the grid-refinement scheme the paper's AMR runs rely on, Sec. 5.2,
// after Dupuis & Chopard): acoustic scaling, dt_f = dt_c / 2, dx_f = dx_c / 2,
// so tau_f = 2 tau_c - 1/2 keeps the physical viscosity.  Populations are
// split into f^eq(rho, u) and a non-equilibrium part; across levels the
// pre-collision f^neq scales by tau_f / (2 tau_c), so for the stored
// post-collision values S = f^eq + (1 - 1/tau) f^neq the non-equilibrium part
// of S scales by
//     alpha = (tau_f - 1) / (2 (tau_c - 1))     (coarse -> fine; 1/alpha back).
//
// Layout of the fine level.  Patch p is a box of ex x ey x ez fine cells (all
// multiples of 8) with a one-cell ghost layer: its (ex+2)(ey+2)(ez+2) padded
// cells sit at offset off_p of every population plane, x fastest.  Streaming
// pulls from the padded neighbours, so interior cells never branch on
// boundaries; the ghost layer is refilled before every fine step, from the
// abutting patch where there is one, else by interpolation of the coarse
// level.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"
#include "step_kernel.hpp"

namespace lbm {

// Per-patch record in device memory (int32 fields).
struct PatchRec {
    int o[3];       // fine-cell origin (twice the coarse box origin)
    int e[3];       // fine-cell extent
    int off;        // first padded cell of the patch in each plane
    int blk0;       // first 8^3 sensor block of the patch
    int coff;       // first covered coarse cell (restriction enumeration)
    int pad[3];
};
static_assert(sizeof(PatchRec) == 48, "PatchRec layout");

template <typename C>
struct PatchArgs {
    const void *src;          // fine state read by the step (padded planes)
    void *dst;                // fine state written by the step
    int64_t pitch;            // elements between fine planes
    const PatchRec *patch;    // [npatch]
    const int *blk_patch;     // [nblocks]: patch of each sensor block
    int npatch, nblocks;
    C shift[kMaxQ];           // w_i rho0 in C
    C rho0, omega;            // fine relaxation rate 1 / tau_f
    double theta_r, theta_c;
    C *block_max;             // [nblocks] (finished sensor values)
    int8_t *flags;            // [nblocks]
};

// Coarse-level view used by the ghost fill and the restriction.
template <typename C>
struct CoarseView {
    const void *s0;           // coarse post-collision state at the earlier time
    const void *s1;           // ... at the later time (== s0 when w1 == 0)
    void *out;                // restriction target (coarse state being completed)
    int64_t pitch;            // elements between coarse planes
    int nx, ny, nz;
    const int *cover;         // [coarse cells]: patch covering the cell, or -1
    C w1;                     // weight of s1 in the time interpolation
    C alpha;                  // coarse -> fine scaling of the non-equilibrium part
};

// Per-cell pieces of the BGK collision shared by the kernels below, in the
// deviation form d_i = f_i - w_i rho0 of the step kernel.
template <int Q, typename C>
struct Moments {
    C drho, j[3], u[3], usq;
};

template <int Q, typename C>
__device__ __forceinline__ Moments<Q, C> moments_of(const C (&d)[Q], C rho0) {
    Moments<Q, C> m;
    m.drho = C(0);
    m.j[0] = m.j[1] = m.j[2] = C(0);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        m.drho += d[i];
        if constexpr (V::x != 0) m.j[0] += C(V::x) * d[i];
        if constexpr (V::y != 0) m.j[1] += C(V::y) * d[i];
        if constexpr (V::z != 0) m.j[2] += C(V::z) * d[i];
    });
    const C inv_rho = C(1) / (rho0 + m.drho);
    for (int a = 0; a < 3; ++a) m.u[a] = m.j[a] * inv_rho;
    m.usq = m.u[0] * m.u[0] + m.u[1] * m.u[1] + m.u[2] * m.u[2];
    return m;
}

// f^eq_i - w_i rho0 (Eq. feq_i), the same arithmetic as the step kernel.
template <int Q, int I, typename C>
__device__ __forceinline__ C deq_of(const Moments<Q, C> &m, C rho0) {
    const C cu = dot_c<Q, I>(m.u);
    const C cj = dot_c<Q, I>(m.j);
    const C p2 = C(4.5) * cu * cu - C(1.5) * m.usq;
    return wmul<C, Vel<Q, I>::w>(m.drho + C(3) * cj + (rho0 * p2 + m.drho * p2));
}

template <typename T, typename C>
__device__ __forceinline__ C load_dev(const void *buf, int64_t idx, C shift, bool shifted) {
    const C v = static_cast<C>(static_cast<const T *>(buf)[idx]);
    return shifted ? v : v - shift;
}

template <typename T, typename C>
__device__ __forceinline__ void store_dev(void *buf, int64_t idx, C d, C shift, bool shifted) {
    static_cast<T *>(buf)[idx] = static_cast<T>(shifted ? d : d + shift);
}

// Padded index of fine cell (x, y, z) of a patch (interior cells 0..e-1).
__device__ __forceinline__ int64_t padded_index(const PatchRec &p, int x, int y, int z) {
    return (int64_t)p.off + ((int64_t)(z + 1) * (p.e[1] + 2) + (y + 1)) * (p.e[0] + 2) + (x + 1);
}

// One fine step of every patch.  A workgroup of 8 x 8 x BZ threads owns one
// 8^3 sensor block at a time (each thread marches 8/BZ z-slices) and loops
// over the blocks of all patches with a fixed stride (a persistent launch of
// fewer workgroups than blocks): pull-stream from the padded neighbours,
// BGK collision, and on sensor steps the block maximum and flag, reduced in
// the workgroup without atomics.
template <int Q, typename T, typename C, bool SH, bool SENSOR, int SKIND, int BZ>
__global__ __launch_bounds__(64 * BZ) void patch_step(const PatchArgs<C> a) {
    static_assert(Lattice<Q>::D == 3 && 8 % BZ == 0, "3D patches, BZ divides 8");
    const int tx = threadIdx.x & 7, ty = (threadIdx.x >> 3) & 7, tz = threadIdx.x >> 6;
    __shared__ C red[BZ];
    for (int b = blockIdx.x; b < a.nblocks; b += gridDim.x) {
        const PatchRec p = a.patch[a.blk_patch[b]];
        const int lb = b - p.blk0;
        const int nbx = p.e[0] >> 3, nby = p.e[1] >> 3;
        const int bx = lb % nbx, by = (lb / nbx) % nby, bz = lb / (nbx * nby);
        const int64_t sy = p.e[0] + 2, sz = sy * (p.e[1] + 2);
        C m = C(0);
#pragma unroll 1
        for (int zz = tz; zz < 8; zz += BZ) {
            const int64_t c = padded_index(p, 8 * bx + tx, 8 * by + ty, 8 * bz + zz);
            C d[Q];
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                using V = Vel<Q, i>;
                const int64_t from = c - (V::x + V::y * sy + V::z * sz);
                d[i] = load_dev<T>(a.src, i * a.pitch + from, a.shift[i], SH);
            });
            const Moments<Q, C> mo = moments_of<Q>(d, a.rho0);
            C num = C(0), den = C(0), kkn = C(0);
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                const C deq = deq_of<Q, i>(mo, a.rho0);
                const C fneq = d[i] - deq;
                if constexpr (SENSOR) {
                    const C feq = a.shift[i] + deq;
                    if constexpr (SKIND == kSensorL2) {
                        num += fneq * fneq;
                        den += feq * feq;
                    } else {
                        kkn += fabs(fneq / feq);
                    }
                }
                store_dev<T>(a.dst, i * a.pitch + c, d[i] - a.omega * fneq, a.shift[i], SH);
            });
            if constexpr (SENSOR) m = nan_max(m, SKIND == kSensorL2 ? num / den : kkn * C(1.0 / Q));
        }
        if constexpr (SENSOR) {
            // a wave is one 8 x 8 slice: reduce it with shuffles, then the BZ waves in LDS
#pragma unroll
            for (int s = 1; s < 64; s <<= 1) m = nan_max(m, static_cast<C>(__shfl_xor(m, s)));
            if ((threadIdx.x & 63) == 0) red[tz] = m;
            __syncthreads();
            if (threadIdx.x == 0) {
                C M = red[0];
                for (int k = 1; k < BZ; ++k) M = nan_max(M, red[k]);
                M = finish<SKIND>(M);
                a.block_max[b] = M;
                const double Md = static_cast<double>(M);
                a.flags[b] = (!(Md == Md) || Md == HUGE_VAL) ? 2 : (Md > a.theta_r ? 1 : (Md < a.theta_c ? -1 : 0));
            }
            __syncthreads();
        }
    }
}

// Trilinear interpolation of the coarse populations (time-interpolated
// between s0 and s1) at coarse-index position (px, py, pz), rescaled to the
// fine level: d_f = deq + alpha (d - deq).
template <int Q, typename T, typename C, bool SH>
__device__ __forceinline__ void coarse_to_fine(const CoarseView<C> &v, const C (&shift)[kMaxQ], C rho0, C px,
                                               C py, C pz, C (&d)[Q]) {
    const int x0 = (int)floor(px), y0 = (int)floor(py), z0 = (int)floor(pz);
    const C fx = px - C(x0), fy = py - C(y0), fz = pz - C(z0);
    static_for<0, Q>([&](auto ic) { d[decltype(ic)::value] = C(0); });
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
        const C w = (dx ? fx : C(1) - fx) * (dy ? fy : C(1) - fy) * (dz ? fz : C(1) - fz);
        const int64_t cc = ((int64_t)(z0 + dz) * v.ny + (y0 + dy)) * v.nx + (x0 + dx);
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            C s = load_dev<T>(v.s0, i * v.pitch + cc, shift[i], SH);
            if (v.w1 != C(0)) s += v.w1 * (load_dev<T>(v.s1, i * v.pitch + cc, shift[i], SH) - s);
            d[i] += w * s;
        });
    }
    const Moments<Q, C> mo = moments_of<Q>(d, rho0);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const C deq = deq_of<Q, i>(mo, rho0);
        d[i] = deq + v.alpha * (d[i] - deq);
    });
}

// Ghost layer of every patch (or, with all_cells, every padded cell: the
// initial state).  One thread per padded cell; a ghost cell copies from the
// patch whose interior holds it, else interpolates the coarse level.
template <int Q, typename T, typename C, bool SH>
__global__ __launch_bounds__(256) void patch_fill(const PatchArgs<C> a, const CoarseView<C> v, void *state, int64_t total_padded,
                           int all_cells) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= total_padded) return;
    int lo = 0, hi = a.npatch - 1;               // last patch with off <= g
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.patch[mid].off <= g) lo = mid; else hi = mid - 1;
    }
    const PatchRec p = a.patch[lo];
    const int64_t r = g - p.off;
    const int px = (int)(r % (p.e[0] + 2)), py = (int)((r / (p.e[0] + 2)) % (p.e[1] + 2));
    const int pz = (int)(r / ((int64_t)(p.e[0] + 2) * (p.e[1] + 2)));
    const bool ghost = px == 0 || py == 0 || pz == 0 || px == p.e[0] + 1 || py == p.e[1] + 1 || pz == p.e[2] + 1;
    if (!ghost && !all_cells) return;
    const int gx = p.o[0] + px - 1, gy = p.o[1] + py - 1, gz = p.o[2] + pz - 1;   // global fine cell
    if (ghost && !all_cells) {
        const int owner = v.cover[((int64_t)(gz >> 1) * v.ny + (gy >> 1)) * v.nx + (gx >> 1)];
        if (owner >= 0) {
            const PatchRec q = a.patch[owner];
            const int64_t from = padded_index(q, gx - q.o[0], gy - q.o[1], gz - q.o[2]);
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                static_cast<T *>(state)[i * a.pitch + g] = static_cast<const T *>(state)[i * a.pitch + from];
            });
            return;
        }
    }
    // fine cell centre in coarse-index coordinates: (g + 1/2) / 2 - 1/2
    C d[Q];
    coarse_to_fine<Q, T, C, SH>(v, a.shift, a.rho0, C(0.5) * C(gx) - C(0.25), C(0.5) * C(gy) - C(0.25),
                                C(0.5) * C(gz) - C(0.25), d);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        store_dev<T>(state, i * a.pitch + g, d[i], a.shift[i], SH);
    });
}

// Restriction: every coarse cell covered by a patch takes the mean of its 8
// fine cells, rescaled to the coarse level: d_c = deq + (d - deq) / alpha.
// One thread per covered coarse cell.
template <int Q, typename T, typename C, bool SH>
__global__ __launch_bounds__(256) void patch_restrict(const PatchArgs<C> a, const CoarseView<C> v, const void *fine, int64_t covered) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= covered) return;
    int lo = 0, hi = a.npatch - 1;               // last patch with coff <= t
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (a.patch[mid].coff <= t) lo = mid; else hi = mid - 1;
    }
    const PatchRec p = a.patch[lo];
    const int64_t r = t - p.coff;
    const int cex = p.e[0] >> 1, cey = p.e[1] >> 1;
    const int cx = (int)(r % cex), cy = (int)((r / cex) % cey), cz = (int)(r / ((int64_t)cex * cey));
    C d[Q];
    static_for<0, Q>([&](auto ic) { d[decltype(ic)::value] = C(0); });
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t c = padded_index(p, 2 * cx + (k & 1), 2 * cy + ((k >> 1) & 1), 2 * cz + (k >> 2));
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            d[i] += load_dev<T>(fine, i * a.pitch + c, a.shift[i], SH);
        });
    }
    static_for<0, Q>([&](auto ic) { d[decltype(ic)::value] *= C(0.125); });
    const Moments<Q, C> mo = moments_of<Q>(d, a.rho0);
    const int64_t cc = ((int64_t)(p.o[2] / 2 + cz) * v.ny + (p.o[1] / 2 + cy)) * v.nx + (p.o[0] / 2 + cx);
    const C inv_alpha = C(1) / v.alpha;
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const C deq = deq_of<Q, i>(mo, a.rho0);
        store_dev<T>(v.out, i * v.pitch + cc, deq + inv_alpha * (d[i] - deq), a.shift[i], SH);
    });
}

// Fine-level macroscopic fields of one patch's interior (float64 output,
// [z][y][x]), u from the stored post-collision populations (no body force).
template <int Q, typename T, typename C, bool SH>
__global__ __launch_bounds__(256) void patch_macros(const PatchArgs<C> a, const void *state, int patch, double *rho, double *u,
                             double *f_out) {
    const PatchRec p = a.patch[patch];
    const int64_t n = (int64_t)p.e[0] * p.e[1] * p.e[2];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int x = (int)(t % p.e[0]), y = (int)((t / p.e[0]) % p.e[1]), z = (int)(t / ((int64_t)p.e[0] * p.e[1]));
    const int64_t c = padded_index(p, x, y, z);
    double r = 0.0, m[3] = {0.0, 0.0, 0.0};
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        const double s = static_cast<double>(static_cast<const T *>(state)[i * a.pitch + c]);
        const double f = SH ? s + static_cast<double>(V::w) * static_cast<double>(a.rho0) : s;
        if (f_out) f_out[i * n + t] = f;
        r += f;
        m[0] += V::x * f;
        m[1] += V::y * f;
        m[2] += V::z * f;
    });
    if (rho) rho[t] = r;
    if (u) {
        u[t] = m[0] / r;
        u[n + t] = m[1] / r;
        u[2 * n + t] = m[2] / r;
    }
}

}  // namespace lbm

namespace lbm {

// Host-side launchers, instantiated per lattice in patch_inst.hip.
struct PatchLaunch {
    hipStream_t stream;
    bool sensor;
    int sensor_kind;
    int bz;          // tile depth: 8 x 8 x bz threads per workgroup
    int nwg;         // workgroups of the persistent launch
};

template <int Q, typename T, typename C, bool SH>
void launch_patch_step(const PatchArgs<C> &a, const PatchLaunch &l);
template <int Q, typename T, typename C, bool SH>
void launch_patch_fill(const PatchArgs<C> &a, const CoarseView<C> &v, void *state, int64_t total_padded,
                       bool all_cells, hipStream_t st);
template <int Q, typename T, typename C, bool SH>
void launch_patch_restrict(const PatchArgs<C> &a, const CoarseView<C> &v, const void *fine, int64_t covered,
                           hipStream_t st);
template <int Q, typename T, typename C, bool SH>
void launch_patch_macros(const PatchArgs<C> &a, const void *state, int patch, int64_t cells, double *rho,
                         double *u, double *f, hipStream_t st);

#ifdef LBM_PATCH_DEFINITIONS
template <int Q, typename T, typename C, bool SH, bool S, int K>
void launch_patch_bz(const PatchArgs<C> &a, const PatchLaunch &l) {
    switch (l.bz) {
        case 2: hipLaunchKernelGGL((patch_step<Q, T, C, SH, S, K, 2>), dim3(l.nwg), dim3(128), 0, l.stream, a); break;
        case 4: hipLaunchKernelGGL((patch_step<Q, T, C, SH, S, K, 4>), dim3(l.nwg), dim3(256), 0, l.stream, a); break;
        default: hipLaunchKernelGGL((patch_step<Q, T, C, SH, S, K, 8>), dim3(l.nwg), dim3(512), 0, l.stream, a); break;
    }
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_step(const PatchArgs<C> &a, const PatchLaunch &l) {
    if (!l.sensor) launch_patch_bz<Q, T, C, SH, false, kSensorL2>(a, l);
    else if (l.sensor_kind == kSensorL2) launch_patch_bz<Q, T, C, SH, true, kSensorL2>(a, l);
    else launch_patch_bz<Q, T, C, SH, true, kSensorKKn>(a, l);
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_fill(const PatchArgs<C> &a, const CoarseView<C> &v, void *state, int64_t total_padded,
                       bool all_cells, hipStream_t st) {
    hipLaunchKernelGGL((patch_fill<Q, T, C, SH>), dim3((unsigned)((total_padded + 255) / 256)), dim3(256), 0, st,
                       a, v, state, total_padded, all_cells ? 1 : 0);
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_restrict(const PatchArgs<C> &a, const CoarseView<C> &v, const void *fine, int64_t covered,
                           hipStream_t st) {
    hipLaunchKernelGGL((patch_restrict<Q, T, C, SH>), dim3((unsigned)((covered + 255) / 256)), dim3(256), 0, st,
                       a, v, fine, covered);
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_macros(const PatchArgs<C> &a, const void *state, int patch, int64_t cells, double *rho,
                         double *u, double *f, hipStream_t st) {
    hipLaunchKernelGGL((patch_macros<Q, T, C, SH>), dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, a,
                       state, patch, rho, u, f);
}

#define LBM_INSTANTIATE_PATCH(Q, T, C, SH)                                                                   \
    template void launch_patch_step<Q, T, C, SH>(const PatchArgs<C> &, const PatchLaunch &);                 \
    template void launch_patch_fill<Q, T, C, SH>(const PatchArgs<C> &, const CoarseView<C> &, void *, int64_t, \
                                                 bool, hipStream_t);                                         \
    template void launch_patch_restrict<Q, T, C, SH>(const PatchArgs<C> &, const CoarseView<C> &,            \
                                                     const void *, int64_t, hipStream_t);                    \
    template void launch_patch_macros<Q, T, C, SH>(const PatchArgs<C> &, const void *, int, int64_t, double *, \
                                                   double *, double *, hipStream_t);
#endif

}  // namespace lbm
