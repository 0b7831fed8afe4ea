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
    int xoff;       // first element of its two x-face ghost arrays (low x side, then high)
    int pad[2];
};
static_assert(sizeof(PatchRec) == 48, "PatchRec layout");

// A tile of the fine step: W x 8 x 8 cells (W = 8, 16 or 32) of one patch,
// i.e. W/8 sensor blocks side by side along x.
struct PatchTile {
    int patch;      // patch index
    int x0, y0, z0; // first interior cell (multiples of 8; x0 + W <= e_x)
    int w;          // W
    int blk;        // sensor block of the tile's first 8 x-cells
    int pad[2];
};
static_assert(sizeof(PatchTile) == 32, "PatchTile layout");

// A tile of the ghost fill: up to 256 ghost cells of one face of one patch
// (a 16 x 16 piece of the face), entries k0 .. k0+n-1 of the ghost list, and
// the box of coarse cells their interpolation stencils cover (origin o,
// extent dx x dy x dz <= kGhostBox cells; extent 0 when every ghost of the
// tile copies from an abutting patch).
constexpr int kGhostBox = 200;
// gmask bit of a ghost on an x face: its values go to the patch's compact
// x-face array (element gdst & 0x1FFFFFFF of each x-ghost plane), not to its
// slot in the padded rows (population bits stay below bit 27).
constexpr uint32_t kGhostXFace = 1u << 31;
struct GhostTile {
    int k0, n;
    int ox, oy, oz;
    int dx, dy, dz;
};
static_assert(sizeof(GhostTile) == 32, "GhostTile layout");

template <typename C>
struct PatchArgs {
    const void *src;          // fine state read by the step (padded planes)
    void *dst;                // fine state written by the step
    int64_t pitch;            // elements between fine planes
    int64_t xg_base;          // first element of the x-face ghost planes (after the q padded planes)
    int64_t xg_pitch;         // elements between x-face ghost planes
    const PatchRec *patch;    // [npatch]
    const PatchTile *tile;    // [ntiles]
    int npatch, ntiles;
    C shift[kMaxQ];           // w_i rho0 in C
    C rho0, omega;            // fine relaxation rate 1 / tau_f
    double theta_r, theta_c;
    C *block_max;             // [nblocks] (finished sensor values)
    int8_t *flags;            // [nblocks]
    uint32_t step;            // fine step index: the key of stochastic rounding on store
};

// Stored representation of storage policy T (see Storage in step_kernel.hpp).
template <typename T>
using raw_t = typename Storage<T>::raw;

// Stochastic-rounding keys of the hierarchy's stores: cell_key of a cell
// index and a step, the index xor-ed with a salt per kind of store so that
// the fine step, the ghost fill, the restriction and the initial fill draw
// different bits from the coarse step kernel's (whose indices are coarse
// cells) and from each other.
constexpr uint32_t kSaltFine = 0x40000000u, kSaltGhost = 0x80000000u, kSaltRestrict = 0xC0000000u,
                   kSaltInit = 0x20000000u;

template <typename T>
__device__ __forceinline__ uint32_t sr_cell_key(uint32_t cell, uint32_t salt, uint32_t step) {
    return Storage<T>::sr ? cell_key(cell ^ salt, step) : 0u;
}

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
    const C v = static_cast<C>(static_cast<const raw_t<T> *>(buf)[idx]);
    return shifted ? v : v - shift;
}

// Store of the deviation d (shift added back for unshifted storage) with the
// rounding of policy T; ckey is the cell's stochastic-rounding key.
template <typename T, typename C>
__device__ __forceinline__ void store_dev(void *buf, int64_t idx, C d, C shift, bool shifted, uint32_t ckey,
                                          int pop) {
    static_cast<raw_t<T> *>(buf)[idx] =
        to_storage<T>(shifted ? d : d + shift, Storage<T>::sr ? round_key(ckey, pop) : 0u);
}

// Element of population i of ghost entry g: its slot in the padded rows, or
// for an x-face ghost its element of the compact x-face array.
template <typename C>
__device__ __forceinline__ int64_t ghost_index(const PatchArgs<C> &a, uint32_t need, int i, int64_t g) {
    return (need & kGhostXFace) ? a.xg_base + i * a.xg_pitch + g : i * a.pitch + g;
}

// Padded index of fine cell (x, y, z) of a patch (interior cells 0..e-1).
__device__ __forceinline__ int64_t padded_index(const PatchRec &p, int x, int y, int z) {
    return (int64_t)p.off + ((int64_t)(z + 1) * (p.e[1] + 2) + (y + 1)) * (p.e[0] + 2) + (x + 1);
}

// Restriction sums in 64-bit fixed point with 2^-59 resolution: integer
// additions are exact and associative, so the sum of a coarse cell's 8 fine
// values does not depend on the order in which its contributions arrive
// (LDS atomics in the band step) and equals the exact sum for float32 values
// (multiples of 2^-59 down to |r| = 2^-35); float64 values are rounded to
// 2^-59 each.  Deviations |r| < 1 keep the sum of 8 within range.
constexpr double kFixScale = 0x1p59;
template <typename C>
__device__ __forceinline__ long long to_fixed(C r) {
    return __double2ll_rn(static_cast<double>(r) * kFixScale);
}
template <typename C>
__device__ __forceinline__ C fixed_mean8(long long sum) {
    return static_cast<C>(static_cast<double>(sum) * (0.125 / kFixScale));
}

// One fine step of every patch.  A workgroup of 512 threads owns one tile
// (W x 8 x 8 cells) at a time: thread t takes x = t mod W, y = (t / W) mod 8
// and marches z from t / 8W in steps of 64 / W, so a wave reads W
// consecutive cells of 64 / W rows (rows of up to 128 bytes in float32).  It
// loops over the tiles of all patches (a persistent launch of fewer
// workgroups than tiles, each XCD taking a contiguous part of the list):
// pull-stream from the padded
// neighbours, BGK collision, and on sensor steps the maxima and flags of the
// tile's W/8 blocks, reduced in the workgroup without atomics.
//
// Addressing: the pull source of population i is the cell's padded index c
// minus delta_i = xi_x + xi_y sy + xi_z sz, the same for every cell of a
// patch, so it is folded into the population's plane base (one scalar
// address per population and tile) and every load and store of the cell
// uses the one 32-bit byte offset c * sizeof(T).  The collision is the step
// kernel's: moments in population order, the even part of the equilibrium
// shared by each opposite pair.
template <int Q, typename T, typename C, bool SH, bool SENSOR, int SKIND, bool RESTRICT>
__global__ __launch_bounds__(512) void patch_step(const PatchArgs<C> a, const CoarseView<C> v) {
    static_assert(Lattice<Q>::D == 3, "3D patches");
    __shared__ C red[8][4];      // [wave][block of the tile]
    // restriction: per coarse cell of the tile (at most 16 x 4 x 4) and
    // population, the sum of its 8 fine cells (two partial sums of 4)
    constexpr int kCoarsePerTile = 256;
    __shared__ long long racc[RESTRICT ? Q * kCoarsePerTile : 1];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    using R = raw_t<T>;
    const char *src = static_cast<const char *>(a.src);
    char *dst = static_cast<char *>(a.dst);
    const int64_t plane_bytes = a.pitch * (int64_t)sizeof(R);
    // Workgroups are dealt to the 8 XCDs round-robin by id.  With at least 8
    // workgroups, XCD j works through the j-th eighth of the tile list (tiles
    // are listed x fastest, patch by patch), so that tiles sharing halo lines
    // are fetched into one L2; every tile is visited exactly once either way.
    int k0 = blockIdx.x, k1 = a.ntiles, kstep = gridDim.x;
    if (gridDim.x >= 8) {
        const int xcd = blockIdx.x & 7;
        k0 = (int)((int64_t)a.ntiles * xcd / 8) + (int)(blockIdx.x >> 3);
        k1 = (int)((int64_t)a.ntiles * (xcd + 1) / 8);
        kstep = (int)((gridDim.x - xcd + 7) >> 3);
    }
    for (int k = k0; k < k1; k += kstep) {
        const PatchTile tl = a.tile[k];
        const PatchRec p = a.patch[tl.patch];
        const int W = tl.w;
        const int x = t % W, y = (t / W) & 7, zstep = 64 / W;
        const int sy = p.e[0] + 2, sz = sy * (p.e[1] + 2);
        // the first and last cell of a row also write their value into the
        // row's ghost slot beside them (refilled before it is read): every
        // padded row is then written whole, and the memory system sees whole
        // lines instead of lines with a 4-byte hole at each row end
        const bool xlo = tl.x0 + x == 0, xhi = tl.x0 + x == p.e[0] - 1;
        const bool xedge = xlo || xhi;
        const int xoff = xlo ? -(int)sizeof(R) : (int)sizeof(R);
        // the first and last cell of a row pull their x-face ghosts from the
        // compact x-face arrays: element (z + 1) P1 + (y + 1) of the low or
        // high side, minus the population's (y, z) offset
        const int P1 = p.e[1] + 2;
        const int64_t xg_side = (int64_t)P1 * (p.e[2] + 2);
        const R *xg0 = static_cast<const R *>(a.src) + a.xg_base + p.xoff + (xhi ? xg_side : 0) + (tl.y0 + y + 1);
        C m = C(0);
        if constexpr (RESTRICT) {
            for (int r = t; r < Q * kCoarsePerTile; r += 512) racc[r] = 0;
            __syncthreads();
        }
#pragma unroll 1
        for (int zz = t / (8 * W); zz < 8; zz += zstep) {
            // padded cell index (< 2^29, checked on the host) as a byte offset
            const R *xgc = xg0 + (int64_t)(tl.z0 + zz + 1) * P1;
            const uint32_t cidx = (uint32_t)(p.off + (tl.z0 + zz + 1) * sz + (tl.y0 + y + 1) * sy + (tl.x0 + x + 1));
            const uint32_t cb = cidx * (uint32_t)sizeof(R);
            const uint32_t ckey = sr_cell_key<T>(cidx, kSaltFine, a.step);
            const int rslot = ((zz >> 1) * 4 + (y >> 1)) * (W >> 1) + (x >> 1);
            (void)rslot;
            C d[Q];
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                using V = Vel<Q, i>;
                const int64_t delta = V::x + (int64_t)V::y * sy + (int64_t)V::z * sz;
                const char *base = src + i * plane_bytes - delta * (int64_t)sizeof(R);
                const R *from = reinterpret_cast<const R *>(base + cb);
                if constexpr (V::x > 0) {
                    if (xlo) from = xgc + (i * a.xg_pitch - (V::z * P1 + V::y));
                } else if constexpr (V::x < 0) {
                    if (xhi) from = xgc + (i * a.xg_pitch - (V::z * P1 + V::y));
                }
                const C v = static_cast<C>(*from);
                if constexpr (SH) d[i] = v;
                else d[i] = v - a.shift[i];
            });
            C drho, j[3];
            cell_moments<Q>(d, drho, j);
            const C inv_rho = C(1) / (a.rho0 + drho);
            const C u[3] = {j[0] * inv_rho, j[1] * inv_rho, j[2] * inv_rho};
            const C m15usq = C(-1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            C num = C(0), den = C(0), kkn = C(0);
            auto relax = [&](auto ic, C br) {
                constexpr int i = decltype(ic)::value;
                const C deq = wmul<C, Vel<Q, i>::w>(br);
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
                C out = d[i] - a.omega * fneq;
                if constexpr (!SH) out += a.shift[i];
                const R stored = to_storage<T>(out, Storage<T>::sr ? round_key(ckey, i) : 0u);
                *reinterpret_cast<R *>(dst + i * plane_bytes + cb) = stored;
                if (xedge) *reinterpret_cast<R *>(dst + i * plane_bytes + cb + xoff) = stored;
                if constexpr (RESTRICT) {
                    // the value the level below reads back, as a deviation, added
                    // to its coarse cell's sum in fixed point (exact, any order)
                    C r = static_cast<C>(stored);
                    if constexpr (!SH) r -= a.shift[i];
                    atomicAdd(reinterpret_cast<unsigned long long *>(&racc[i * kCoarsePerTile + rslot]),
                              static_cast<unsigned long long>(to_fixed(r)));
                }
            };
            relax(std::integral_constant<int, 0>{}, drho + (a.rho0 * m15usq + drho * m15usq));
            static_for<0, (Q - 1) / 2>([&](auto kc) {
                constexpr int i = 2 * decltype(kc)::value + 1;
                const C cu = dot_c<Q, i>(u);
                const C cj = dot_c<Q, i>(j);
                const C p2 = C(4.5) * cu * cu + m15usq;
                const C even = drho + (a.rho0 * p2 + drho * p2);
                relax(std::integral_constant<int, i>{}, even + C(3) * cj);
                relax(std::integral_constant<int, i + 1>{}, even - C(3) * cj);
            });
            if constexpr (SENSOR) m = nan_max(m, SKIND == kSensorL2 ? num / den : kkn * C(1.0 / Q));
        }
        if constexpr (RESTRICT) {
            // each coarse cell of the tile takes the mean of its 8 fine cells,
            // rescaled to the coarse level: d_c = deq + (d - deq) / alpha
            __syncthreads();
            const int ncoarse = 8 * W;   // (W / 2) x 4 x 4
            if (t < ncoarse) {
                const int hx = W >> 1;
                const int cxl = t % hx, cyl = (t / hx) & 3, czl = t / (4 * hx);
                const int cx = ((p.o[0] + tl.x0) >> 1) + cxl;
                const int cy = ((p.o[1] + tl.y0) >> 1) + cyl;
                const int cz = ((p.o[2] + tl.z0) >> 1) + czl;
                const int64_t cc = ((int64_t)cz * v.ny + cy) * v.nx + cx;
                C dr[Q];
                static_for<0, Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    dr[i] = fixed_mean8<C>(racc[i * kCoarsePerTile + t]);
                });
                const Moments<Q, C> mo = moments_of<Q>(dr, a.rho0);
                const C inv_alpha = C(1) / v.alpha;
                const uint32_t rkey = sr_cell_key<T>((uint32_t)cc, kSaltRestrict, a.step);
                static_for<0, Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    const C deq = deq_of<Q, i>(mo, a.rho0);
                    store_dev<T>(v.out, i * v.pitch + cc, deq + inv_alpha * (dr[i] - deq), a.shift[i], SH, rkey, i);
                });
            }
            __syncthreads();   // the next tile zeroes racc
        }
        if constexpr (SENSOR) {
            // lane bits 3.. log2(W)-1 number the block of the lane's x: reduce
            // over every other lane bit, then over the 8 waves in LDS
#pragma unroll
            for (int s = 1; s < 64; s <<= 1)
                if ((s & (W - 8)) == 0) m = nan_max(m, static_cast<C>(__shfl_xor(m, s)));
            if ((lane & 7) == 0 && lane < W) red[wave][lane >> 3] = m;
            __syncthreads();
            if (t < W / 8) {
                C M = red[0][t];
                for (int w = 1; w < 8; ++w) M = nan_max(M, red[w][t]);
                M = finish<SKIND>(M);
                a.block_max[tl.blk + t] = M;
                const double Md = static_cast<double>(M);
                a.flags[tl.blk + t] =
                    (!(Md == Md) || Md == HUGE_VAL) ? 2 : (Md > a.theta_r ? 1 : (Md < a.theta_c ? -1 : 0));
            }
            __syncthreads();
        }
    }
}

// Widest tile of the band step (interior cells along x).
constexpr int kBandMaxW = 48;

// One fine step of every patch, band form.  A tile is a band of one patch:
// W <= 48 interior cells along x (the whole row when it fits) by 8 rows by 8
// slices, i.e. one row of 8^3 sensor blocks.  Its cells are numbered row by
// row, slice by slice, and the 512 threads take consecutive numbers, so a
// wave's 64 lanes read and write 64 consecutive cells of every population
// plane: where the tile spans the patch row, the row-end ghost slots are
// numbered too and a row's 8 rows are one contiguous run of memory.  Lanes on
// a ghost slot (never read: x-face ghosts live in the compact arrays) store
// zeros, so every line is written whole.  Per cell: the pull, BGK collision
// and stores of patch_step, the same arithmetic in the same order (the same
// bits).  Sensor: an LDS atomic max per block; restriction: each stored
// value, as a deviation, is added to its coarse cell's LDS sum in fixed
// point (exact and order independent), then one thread per coarse cell
// takes the mean and rescales the non-equilibrium part by 1/alpha.
//
// Addresses: the host runs bands only on state buffers below 4 GiB, so every
// access is one 64-bit base plus a 32-bit byte offset (a per-population
// scalar plus the cell's offset), which keeps the scalar registers of 2Q
// plane pointers out of the loop; at most 128 VGPRs (4 waves per SIMD).
// Barriers keep the waves of a workgroup on neighbouring cells, so that the
// lines that two waves share are written while both halves are in L2 and
// the chip's window of memory in use stays compact (measured: without
// them the step is 25% slower): one at the start of every tile, and after
// every pass of the 512 threads, except with the restriction, whose LDS
// atomics make the passes uneven (there one barrier after the tile's last
// pass completes the sums).  The epilogue's thread that reads an LDS sum
// also clears it for the next tile.
template <int Q, typename T, typename C, bool SH, bool SENSOR, int SKIND, bool RESTRICT>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void patch_band_step(
    const PatchArgs<C> a, const CoarseView<C> v) {
    static_assert(Lattice<Q>::D == 3, "3D patches");
    using R = raw_t<T>;
    constexpr int kRC = 4 * 4 * (kBandMaxW / 2);   // coarse cells of a tile: 4 slices x 4 rows x W/2
    constexpr bool kPassSync = !RESTRICT;
    // block maxima as the bits of the sensor value: it is >= 0, +inf or NaN,
    // so the unsigned order of its bits is a NaN-propagating max order
    using U = std::conditional_t<sizeof(C) == 8, unsigned long long, unsigned>;
    __shared__ U red[kBandMaxW / 8];
    __shared__ long long racc[RESTRICT ? Q * kRC : 1];
    const int t = threadIdx.x;
    const char *src = static_cast<const char *>(a.src);
    char *dst = static_cast<char *>(a.dst);
    const uint32_t plane_bytes = (uint32_t)a.pitch * (uint32_t)sizeof(R);
    int k0 = blockIdx.x, k1 = a.ntiles, kstep = gridDim.x;
    if (gridDim.x >= 8) {   // XCD j works through the j-th eighth of the tile list
        const int xcd = blockIdx.x & 7;
        k0 = (int)((int64_t)a.ntiles * xcd / 8) + (int)(blockIdx.x >> 3);
        k1 = (int)((int64_t)a.ntiles * (xcd + 1) / 8);
        kstep = (int)((gridDim.x - xcd + 7) >> 3);
    }
    if constexpr (SENSOR)
        if (t < kBandMaxW / 8) red[t] = U(0);
    if constexpr (RESTRICT)
        for (int r = t; r < Q * kRC; r += 512) racc[r] = 0;
    for (int k = k0; k < k1; k += kstep) {
        __syncthreads();   // the previous tile's epilogue has read and cleared the LDS sums
        const PatchTile tl = a.tile[k];
        const PatchRec p = a.patch[tl.patch];
        const int W = tl.w, hx = W >> 1;
        const int sy = p.e[0] + 2, sz = sy * (p.e[1] + 2);
        const int P1 = p.e[1] + 2;
        const uint32_t xg_side = (uint32_t)P1 * (uint32_t)(p.e[2] + 2);
        // lanes of a row segment: the W interior cells, plus a row-end ghost
        // slot where the tile reaches the patch's end
        const int g0 = tl.x0 == 0, g1 = tl.x0 + W == p.e[0];
        const int L = W + g0 + g1, xs = tl.x0 + 1 - g0;   // first padded x of a segment
        const int per_slice = 8 * L, total = 8 * per_slice;
        // (slice, row, lane of the segment) of number j = t, then advanced by 512
        int sl = t / per_slice;
        int rem = t - sl * per_slice;
        int row = rem / L, xl = rem - row * L;
        const int drow = 512 / L, dxl = 512 - drow * L;
#pragma unroll 1
        for (int j0 = 0; j0 < total; j0 += 512) {
            if (j0 + t < total) {
                const int xp = xs + xl;                   // padded x
                const uint32_t cidx = (uint32_t)(p.off + (tl.z0 + sl + 1) * sz + (tl.y0 + row + 1) * sy + xp);
                const uint32_t cb = cidx * (uint32_t)sizeof(R);
                const int x = xp - 1;                     // interior x; -1 or e_x on a ghost slot
                if (x < 0 || x >= p.e[0]) {
                    static_for<0, Q>([&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        *reinterpret_cast<R *>(dst + (cb + i * plane_bytes)) = R(0);
                    });
                } else {
                    const bool xlo = x == 0, xhi = x == p.e[0] - 1;
                    // element of the cell's row in the x-face ghost arrays of its side
                    const uint32_t xgc = (uint32_t)a.xg_base + (uint32_t)p.xoff + (xhi ? xg_side : 0u) +
                                         (uint32_t)((tl.z0 + sl + 1) * P1 + (tl.y0 + row + 1));
                    const uint32_t ckey = sr_cell_key<T>(cidx, kSaltFine, a.step);
                    C d[Q];
                    static_for<0, Q>([&](auto ic) {
                        constexpr int i = decltype(ic)::value;
                        using V = Vel<Q, i>;
                        // byte offsets modulo 2^32: the true offset lies in [0, 2^32)
                        const uint32_t delta = (uint32_t)(V::x + V::y * sy + V::z * sz) * (uint32_t)sizeof(R);
                        uint32_t off = cb + i * plane_bytes - delta;
                        if constexpr (V::x != 0) {
                            const uint32_t xoff =
                                (xgc + (uint32_t)i * (uint32_t)a.xg_pitch - (uint32_t)(V::z * P1 + V::y)) *
                                (uint32_t)sizeof(R);
                            if (V::x > 0 ? xlo : xhi) off = xoff;
                        }
                        const C vv = static_cast<C>(*reinterpret_cast<const R *>(src + off));
                        if constexpr (SH) d[i] = vv;
                        else d[i] = vv - a.shift[i];
                    });
                    C drho, j3[3];
                    cell_moments<Q>(d, drho, j3);
                    const C inv_rho = C(1) / (a.rho0 + drho);
                    const C u[3] = {j3[0] * inv_rho, j3[1] * inv_rho, j3[2] * inv_rho};
                    const C m15usq = C(-1.5) * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
                    C num = C(0), den = C(0), kkn = C(0);
                    const int rslot = ((sl >> 1) * 4 + (row >> 1)) * hx + ((x - tl.x0) >> 1);
                    (void)rslot;
                    auto relax = [&](auto ic, C br) {
                        constexpr int i = decltype(ic)::value;
                        const C deq = wmul<C, Vel<Q, i>::w>(br);
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
                        C out = d[i] - a.omega * fneq;
                        if constexpr (!SH) out += a.shift[i];
                        const R stored = to_storage<T>(out, Storage<T>::sr ? round_key(ckey, i) : 0u);
                        *reinterpret_cast<R *>(dst + (cb + i * plane_bytes)) = stored;
                        if constexpr (RESTRICT) {
                            C r = static_cast<C>(stored);
                            if constexpr (!SH) r -= a.shift[i];
                            atomicAdd(reinterpret_cast<unsigned long long *>(&racc[i * kRC + rslot]),
                                      static_cast<unsigned long long>(to_fixed(r)));
                        }
                    };
                    relax(std::integral_constant<int, 0>{}, drho + (a.rho0 * m15usq + drho * m15usq));
                    static_for<0, (Q - 1) / 2>([&](auto kc) {
                        constexpr int i = 2 * decltype(kc)::value + 1;
                        const C cu = dot_c<Q, i>(u);
                        const C cj = dot_c<Q, i>(j3);
                        const C p2 = C(4.5) * cu * cu + m15usq;
                        const C even = drho + (a.rho0 * p2 + drho * p2);
                        relax(std::integral_constant<int, i>{}, even + C(3) * cj);
                        relax(std::integral_constant<int, i + 1>{}, even - C(3) * cj);
                    });
                    if constexpr (SENSOR) {
                        const C sv = SKIND == kSensorL2 ? num / den : kkn * C(1.0 / Q);
                        atomicMax(&red[(x - tl.x0) >> 3], __builtin_bit_cast(U, sv));
                    }
                }
            }
            xl += dxl;
            row += drow;
            if (xl >= L) {
                xl -= L;
                ++row;
            }
            sl += row >> 3;
            row &= 7;
            if constexpr (kPassSync) __syncthreads();
        }
        if constexpr (RESTRICT) __syncthreads();   // the tile's LDS sums are complete
        // epilogue: each sum is read and cleared by one thread
        if constexpr (SENSOR) {
            if (t < W / 8) {
                const C M = finish<SKIND>(__builtin_bit_cast(C, red[t]));
                red[t] = U(0);
                a.block_max[tl.blk + t] = M;
                a.flags[tl.blk + t] = block_flag(static_cast<double>(M), a.theta_r, a.theta_c);
            }
        }
        if constexpr (RESTRICT) {
            // each coarse cell of the tile takes the mean of its 8 fine cells,
            // rescaled to the coarse level: d_c = deq + (d - deq) / alpha
            for (int c = t; c < 16 * hx; c += 512) {
                const int cxl = c % hx, cyl = (c / hx) & 3, czl = c / (4 * hx);
                const int cx = ((p.o[0] + tl.x0) >> 1) + cxl;
                const int cy = ((p.o[1] + tl.y0) >> 1) + cyl;
                const int cz = ((p.o[2] + tl.z0) >> 1) + czl;
                const int64_t cc = ((int64_t)cz * v.ny + cy) * v.nx + cx;
                C dr[Q];
                static_for<0, Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    dr[i] = fixed_mean8<C>(racc[i * kRC + c]);
                    racc[i * kRC + c] = 0;
                });
                const Moments<Q, C> mo = moments_of<Q>(dr, a.rho0);
                const C inv_alpha = C(1) / v.alpha;
                const uint32_t rkey = sr_cell_key<T>((uint32_t)cc, kSaltRestrict, a.step);
                static_for<0, Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    const C deq = deq_of<Q, i>(mo, a.rho0);
                    store_dev<T>(v.out, i * v.pitch + cc, deq + inv_alpha * (dr[i] - deq), a.shift[i], SH, rkey, i);
                });
            }
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
    // corners one at a time: q accumulators and q loads in flight keep the
    // register count (and so the occupancy) of this gather-bound loop moderate
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
        const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
        const C w = (dx ? fx : C(1) - fx) * (dy ? fy : C(1) - fy) * (dz ? fz : C(1) - fz);
        const int64_t cc = ((int64_t)(z0 + dz) * v.ny + (y0 + dy)) * v.nx + (x0 + dx);
        // the time-interpolation test outside the population loop (all loads
        // of a corner in flight together)
        C s0[Q];
        if (v.w1 != C(0)) {
            C s1[Q];
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                s0[i] = load_dev<T>(v.s0, i * v.pitch + cc, shift[i], SH);
                s1[i] = load_dev<T>(v.s1, i * v.pitch + cc, shift[i], SH);
            });
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                d[i] += w * (s0[i] + v.w1 * (s1[i] - s0[i]));
            });
        } else {
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                s0[i] = load_dev<T>(v.s0, i * v.pitch + cc, shift[i], SH);
            });
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                d[i] += w * s0[i];
            });
        }
    }
    const Moments<Q, C> mo = moments_of<Q>(d, rho0);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const C deq = deq_of<Q, i>(mo, rho0);
        d[i] = deq + v.alpha * (d[i] - deq);
    });
}

// Ghost layers from the precomputed list: entry k fills padded cell
// gdst[k] & 0x1FFFFFFF; gsrc[k] >= 0 is the padded cell of an abutting
// patch to copy, else -gsrc[k] - 1 is the coarse cell at the low corner of
// the interpolation stencil, and bit 29 + a of gdst[k] is set when the
// weight of the upper neighbour along axis a is 3/4 (else 1/4).  Only the
// populations some interior cell pulls from the ghost (bit i of gmask[k]:
// ghost + xi_i is an interior cell) are written; the rest of a ghost cell
// is never read.
template <int Q, typename T, typename C, bool SH>
__global__ __launch_bounds__(256) void patch_ghosts(const PatchArgs<C> a, const CoarseView<C> v, void *state,
                                                    const uint32_t *gdst, const int *gsrc, const uint32_t *gmask,
                                                    int64_t nghost) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nghost) return;
    const uint32_t code = gdst[k];
    const int64_t g = code & 0x1FFFFFFFu;
    const int src = gsrc[k];
    const uint32_t need = gmask[k];
    if (src >= 0) {
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if ((need >> i) & 1u)
                static_cast<raw_t<T> *>(state)[ghost_index(a, need, i, g)] =
                    static_cast<const raw_t<T> *>(state)[i * a.pitch + src];
        });
        return;
    }
    const int base = -src - 1;               // coarse cells < 2^31
    const int x0 = base % v.nx, y0 = (base / v.nx) % v.ny, z0 = base / (v.nx * v.ny);
    const C fx = (code >> 29) & 1u ? C(0.75) : C(0.25);
    const C fy = (code >> 30) & 1u ? C(0.75) : C(0.25);
    const C fz = (code >> 31) & 1u ? C(0.75) : C(0.25);
    C d[Q];
    coarse_to_fine<Q, T, C, SH>(v, a.shift, a.rho0, C(x0) + fx, C(y0) + fy, C(z0) + fz, d);
    const uint32_t gkey = sr_cell_key<T>((uint32_t)k, kSaltGhost, a.step);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        if ((need >> i) & 1u) store_dev<T>(state, ghost_index(a, need, i, g), d[i], a.shift[i], SH, gkey, i);
    });
}

// The same ghost fill, one workgroup per ghost tile: the tile's coarse box,
// interpolated in time, is staged once in LDS ([population][cell]) and every
// ghost of the tile interpolates from there, so each coarse value is read
// from memory once per tile instead of up to eight times per ghost.  Same
// arithmetic, in the same order, as patch_ghosts.
template <int Q, typename T, typename C, bool SH>
__global__ __launch_bounds__(256) void patch_ghosts_lds(const PatchArgs<C> a, const CoarseView<C> v, void *state,
                                                        const GhostTile *tiles, const uint32_t *gdst,
                                                        const int *gsrc, const int *gloc, const uint32_t *gmask) {
    static_assert(kGhostBox <= 256, "one box cell per thread");
    __shared__ C box[Q * kGhostBox];
    // neighbouring tiles of a face share coarse lines: give each XCD a run of them
    const GhostTile tl = tiles[xcd_tile(blockIdx.x, gridDim.x)];
    const int ncell = tl.dx * tl.dy * tl.dz;
    if ((int)threadIdx.x < ncell) {
        const int cell = threadIdx.x;
        const int lx = cell % tl.dx, ly = (cell / tl.dx) % tl.dy, lz = cell / (tl.dx * tl.dy);
        const int64_t cc = ((int64_t)(tl.oz + lz) * v.ny + (tl.oy + ly)) * v.nx + (tl.ox + lx);
        // the time-interpolation test outside the population loop, so that all
        // of a cell's loads are in flight before the first is used (a test
        // per population had made the compiler wait for each load in turn)
        C s0[Q];
        if (v.w1 != C(0)) {
            C s1[Q];
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                s0[i] = load_dev<T>(v.s0, i * v.pitch + cc, a.shift[i], SH);
                s1[i] = load_dev<T>(v.s1, i * v.pitch + cc, a.shift[i], SH);
            });
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                box[i * kGhostBox + cell] = s0[i] + v.w1 * (s1[i] - s0[i]);
            });
        } else {
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                s0[i] = load_dev<T>(v.s0, i * v.pitch + cc, a.shift[i], SH);
            });
            static_for<0, Q>([&](auto ic) {
                constexpr int i = decltype(ic)::value;
                box[i * kGhostBox + cell] = s0[i];
            });
        }
    }
    __syncthreads();
    if ((int)threadIdx.x >= tl.n) return;
    const int64_t k = (int64_t)tl.k0 + threadIdx.x;
    const uint32_t code = gdst[k];
    const int64_t g = code & 0x1FFFFFFFu;
    const int src = gsrc[k];
    const uint32_t need = gmask[k];
    if (src >= 0) {
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            if ((need >> i) & 1u)
                static_cast<raw_t<T> *>(state)[ghost_index(a, need, i, g)] =
                    static_cast<const raw_t<T> *>(state)[i * a.pitch + src];
        });
        return;
    }
    const int c0 = gloc[k];                  // low stencil corner inside the tile's box
    const C fx = (code >> 29) & 1u ? C(0.75) : C(0.25);
    const C fy = (code >> 30) & 1u ? C(0.75) : C(0.25);
    const C fz = (code >> 31) & 1u ? C(0.75) : C(0.25);
    C d[Q];
    static_for<0, Q>([&](auto ic) { d[decltype(ic)::value] = C(0); });
#pragma unroll 1
    for (int c = 0; c < 8; ++c) {
        const int ddx = c & 1, ddy = (c >> 1) & 1, ddz = c >> 2;
        const C w = (ddx ? fx : C(1) - fx) * (ddy ? fy : C(1) - fy) * (ddz ? fz : C(1) - fz);
        const int cell = c0 + (ddz * tl.dy + ddy) * tl.dx + ddx;
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            d[i] += w * box[i * kGhostBox + cell];
        });
    }
    const Moments<Q, C> mo = moments_of<Q>(d, a.rho0);
    const uint32_t gkey = sr_cell_key<T>((uint32_t)k, kSaltGhost, a.step);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const C deq = deq_of<Q, i>(mo, a.rho0);
        if ((need >> i) & 1u)
            store_dev<T>(state, ghost_index(a, need, i, g), deq + v.alpha * (d[i] - deq), a.shift[i], SH, gkey, i);
    });
}

// Every padded cell of every patch interpolated from the coarse level: the
// initial fine state.  One thread per padded cell.
template <int Q, typename T, typename C, bool SH>
__global__ __launch_bounds__(256) void patch_init(const PatchArgs<C> a, const CoarseView<C> v, void *state,
                                                  int64_t total_padded) {
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
    const int gx = p.o[0] + px - 1, gy = p.o[1] + py - 1, gz = p.o[2] + pz - 1;   // global fine cell
    // fine cell centre in coarse-index coordinates: (g + 1/2) / 2 - 1/2
    C d[Q];
    coarse_to_fine<Q, T, C, SH>(v, a.shift, a.rho0, C(0.5) * C(gx) - C(0.25), C(0.5) * C(gy) - C(0.25),
                                C(0.5) * C(gz) - C(0.25), d);
    const uint32_t ikey = sr_cell_key<T>((uint32_t)g, kSaltInit, a.step);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        store_dev<T>(state, i * a.pitch + g, d[i], a.shift[i], SH, ikey, i);
    });
}

// Restriction: every coarse cell covered by a patch takes the mean of its 8
// fine cells, rescaled to the coarse level: d_c = deq + (d - deq) / alpha.
// One thread per entry of the precomputed list: coarse cell rc[k], padded
// cell rf[k] of the fine group's low corner, patch rp[k].
template <int Q, typename T, typename C, bool SH>
__global__ __launch_bounds__(256) void patch_restrict(const PatchArgs<C> a, const CoarseView<C> v, const void *fine,
                                                      const int *rc, const int *rf, const int *rp,
                                                      int64_t covered) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= covered) return;
    const PatchRec &p = a.patch[rp[t]];
    const int64_t sy = p.e[0] + 2, sz = sy * (p.e[1] + 2);
    const int64_t c0 = rf[t];
    long long acc[Q];
    static_for<0, Q>([&](auto ic) { acc[decltype(ic)::value] = 0; });
#pragma unroll
    for (int k = 0; k < 8; ++k) {
        const int64_t c = c0 + (k & 1) + ((k >> 1) & 1) * sy + (k >> 2) * sz;
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            acc[i] += to_fixed(load_dev<T>(fine, i * a.pitch + c, a.shift[i], SH));
        });
    }
    C d[Q];
    static_for<0, Q>([&](auto ic) { d[decltype(ic)::value] = fixed_mean8<C>(acc[decltype(ic)::value]); });
    const Moments<Q, C> mo = moments_of<Q>(d, a.rho0);
    const int64_t cc = rc[t];
    const C inv_alpha = C(1) / v.alpha;
    const uint32_t rkey = sr_cell_key<T>((uint32_t)cc, kSaltRestrict, a.step);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const C deq = deq_of<Q, i>(mo, a.rho0);
        store_dev<T>(v.out, i * v.pitch + cc, deq + inv_alpha * (d[i] - deq), a.shift[i], SH, rkey, i);
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
        const double s = static_cast<double>(static_cast<const raw_t<T> *>(state)[i * a.pitch + c]);
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
    bool restrict_to_coarse;   // also restrict to the coarse state (CoarseView::out)
    int nwg;         // workgroups of the persistent launch
    bool bands;      // the tile list holds bands (patch_band_step), else W x 8 x 8 tiles
};

// Lists the fine step and the coupling kernels read (device pointers).
struct PatchLists {
    const uint32_t *gdst;
    const int *gsrc;
    const int *gloc;        // per ghost: low stencil corner inside its tile's box (LDS path)
    const uint32_t *gmask;  // per ghost: populations some interior cell pulls from it
    int64_t nghost;
    const GhostTile *gtile;
    int64_t ngtile;
    const int *rc, *rf, *rp;
    int64_t covered;
};

template <int Q, typename T, typename C, bool SH>
void launch_patch_step(const PatchArgs<C> &a, const CoarseView<C> &v, const PatchLaunch &l);
template <int Q, typename T, typename C, bool SH>
void launch_patch_init(const PatchArgs<C> &a, const CoarseView<C> &v, void *state, int64_t total_padded,
                       hipStream_t st);
template <int Q, typename T, typename C, bool SH>
void launch_patch_ghosts(const PatchArgs<C> &a, const CoarseView<C> &v, void *state, const PatchLists &L,
                         hipStream_t st);
template <int Q, typename T, typename C, bool SH>
void launch_patch_restrict(const PatchArgs<C> &a, const CoarseView<C> &v, const void *fine, const PatchLists &L,
                           hipStream_t st);
template <int Q, typename T, typename C, bool SH>
void launch_patch_macros(const PatchArgs<C> &a, const void *state, int patch, int64_t cells, double *rho,
                         double *u, double *f, hipStream_t st);

#ifdef LBM_PATCH_DEFINITIONS
template <int Q, typename T, typename C, bool SH>
void launch_patch_step(const PatchArgs<C> &a, const CoarseView<C> &v, const PatchLaunch &l) {
    const dim3 g(l.nwg), b(512);
    auto go = [&](auto kern) { hipLaunchKernelGGL(kern, g, b, 0, l.stream, a, v); };
    if (l.bands) {
        if (l.restrict_to_coarse) {
            if (!l.sensor) go(patch_band_step<Q, T, C, SH, false, kSensorL2, true>);
            else if (l.sensor_kind == kSensorL2) go(patch_band_step<Q, T, C, SH, true, kSensorL2, true>);
            else go(patch_band_step<Q, T, C, SH, true, kSensorKKn, true>);
        } else {
            if (!l.sensor) go(patch_band_step<Q, T, C, SH, false, kSensorL2, false>);
            else if (l.sensor_kind == kSensorL2) go(patch_band_step<Q, T, C, SH, true, kSensorL2, false>);
            else go(patch_band_step<Q, T, C, SH, true, kSensorKKn, false>);
        }
    } else if (l.restrict_to_coarse) {
        if (!l.sensor) go(patch_step<Q, T, C, SH, false, kSensorL2, true>);
        else if (l.sensor_kind == kSensorL2) go(patch_step<Q, T, C, SH, true, kSensorL2, true>);
        else go(patch_step<Q, T, C, SH, true, kSensorKKn, true>);
    } else {
        if (!l.sensor) go(patch_step<Q, T, C, SH, false, kSensorL2, false>);
        else if (l.sensor_kind == kSensorL2) go(patch_step<Q, T, C, SH, true, kSensorL2, false>);
        else go(patch_step<Q, T, C, SH, true, kSensorKKn, false>);
    }
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_init(const PatchArgs<C> &a, const CoarseView<C> &v, void *state, int64_t total_padded,
                       hipStream_t st) {
    hipLaunchKernelGGL((patch_init<Q, T, C, SH>), dim3((unsigned)((total_padded + 255) / 256)), dim3(256), 0, st,
                       a, v, state, total_padded);
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_ghosts(const PatchArgs<C> &a, const CoarseView<C> &v, void *state, const PatchLists &L,
                         hipStream_t st) {
    if (L.nghost == 0) return;
    if (L.gtile)
        hipLaunchKernelGGL((patch_ghosts_lds<Q, T, C, SH>), dim3((unsigned)L.ngtile), dim3(256), 0, st, a, v, state,
                           L.gtile, L.gdst, L.gsrc, L.gloc, L.gmask);
    else
        hipLaunchKernelGGL((patch_ghosts<Q, T, C, SH>), dim3((unsigned)((L.nghost + 255) / 256)), dim3(256), 0,
                           st, a, v, state, L.gdst, L.gsrc, L.gmask, L.nghost);
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_restrict(const PatchArgs<C> &a, const CoarseView<C> &v, const void *fine, const PatchLists &L,
                           hipStream_t st) {
    hipLaunchKernelGGL((patch_restrict<Q, T, C, SH>), dim3((unsigned)((L.covered + 255) / 256)), dim3(256), 0, st,
                       a, v, fine, L.rc, L.rf, L.rp, L.covered);
}

template <int Q, typename T, typename C, bool SH>
void launch_patch_macros(const PatchArgs<C> &a, const void *state, int patch, int64_t cells, double *rho,
                         double *u, double *f, hipStream_t st) {
    hipLaunchKernelGGL((patch_macros<Q, T, C, SH>), dim3((unsigned)((cells + 255) / 256)), dim3(256), 0, st, a,
                       state, patch, rho, u, f);
}

#define LBM_INSTANTIATE_PATCH(Q, T, C, SH)                                                                   \
    template void launch_patch_step<Q, T, C, SH>(const PatchArgs<C> &, const CoarseView<C> &,                \
                                                 const PatchLaunch &);                                       \
    template void launch_patch_init<Q, T, C, SH>(const PatchArgs<C> &, const CoarseView<C> &, void *, int64_t, \
                                                 hipStream_t);                                               \
    template void launch_patch_ghosts<Q, T, C, SH>(const PatchArgs<C> &, const CoarseView<C> &, void *,      \
                                                   const PatchLists &, hipStream_t);                         \
    template void launch_patch_restrict<Q, T, C, SH>(const PatchArgs<C> &, const CoarseView<C> &,            \
                                                     const void *, const PatchLists &, hipStream_t);         \
    template void launch_patch_macros<Q, T, C, SH>(const PatchArgs<C> &, const void *, int, int64_t, double *, \
                                                   double *, double *, hipStream_t);
#endif

}  // namespace lbm
