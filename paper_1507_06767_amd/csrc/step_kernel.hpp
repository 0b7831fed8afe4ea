// step_kernel.hpp -- the fused lattice Boltzmann step + kinetic sensor for gfx950.
//
// One launch advances every cell by one step S_k = C(T(S_{k-1})) (Sec. 2.2:
// Eq. bgklb, equilibrium Eq. feq_i, moments Eqs. rho and u, then the
// collide-and-stream split) and, on sensor steps, evaluates the kinetic sensor
// of Sec. 3.2 on the pre-collision populations, reduces it to one maximum per
// sensor block and writes the refine / keep / coarsen flag of that block
// (Sec. 3.4).
//
// Layout: structure of arrays, population plane i at element offset i*pitch,
// cell (x,y,z) at (z*ny + y)*nx + x.  Streaming is a PULL: population i of
// cell x is read from cell x - xi_i of the other buffer, so every stored value
// is read exactly once and the 64 lanes of a wave read 64 consecutive values
// of one plane.  Walls are recognised from the coordinates (no geometry array)
// and handled without branches: a bounced link reads the opposite population
// of its own cell instead of the neighbour's, selected per lane.  Addresses
// are a uniform plane base plus a 32-bit lane offset, which keeps the kernel
// at ~40 VGPRs (8 waves per SIMD) so that enough loads are in flight.
//
// Two work decompositions:
//  * step_cells: one cell per thread; a workgroup is BX x 8 cells of one
//    z-slice, i.e. BX/8 block columns of one 8x8 block row.  The workgroup
//    reduces its part of each block maximum with 8-lane shuffles and one LDS
//    exchange; in 2D that is the whole block.  In 3D the 8 z-slices of a block
//    are combined through one 64-bit word per block holding (arrival count <<
//    32 | max bits): each contributor folds its value in with a
//    compare-and-swap, and the one that completes the count writes the block
//    maximum and flag and clears the word for the next sensor step.  The max
//    is order independent, so the result is deterministic.  Used for float
//    storage (a float's bits fit beside the count).
//  * step_zmarch: one thread marches over the 8 z-slices of a block column, so
//    a BX x 8 workgroup holds whole 8x8x8 blocks and finishes their maxima
//    itself.  Used for 3D float64 storage, whose 64-bit maximum leaves no room
//    for a count.
//
// Arithmetic is done on the shifted populations d_i = f_i - w_i rho0, which
// keeps the float32 variants accurate: every quantity the sensor and the
// collision need (rho - rho0, rho u, f^neq, f^eq - w_i rho0) is a small
// number formed without cancellation.  Two more choices keep float32
// arithmetic from drifting over thousands of steps: the equilibrium's
// first-order term is formed from the momentum j = sum_i xi_i f_i (+ F/2)
// itself rather than from rho * u, and its product with the weight w_i uses
// a two-float weight (w_hi + w_lo, one extra FMA), so that sum_i w_i = 1 and
// sum_i w_i xi_i xi_i = c_s^2 I hold to rounding instead of being off by the
// float rounding of 1/3, 1/18, 1/36 -- an error that would otherwise add the
// same small momentum at every collision.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbm {

constexpr int kBlockEdge = 8;       // sensor block edge along every active axis
constexpr int kTileY = 8;           // rows per workgroup (one block row)
constexpr int kSensorL2 = 0;
constexpr int kSensorKKn = 1;

template <typename C>
struct StepArgs {
    const void *src;        // S_{k-1}
    void *dst;              // S_k
    uint32_t pitch;         // elements between population planes
    int nx, ny, nz;
    int ntx, nty, ntiles;   // tiles along x, y; total tiles (workgroups)
    int nbx, nby;           // sensor blocks along x, y
    uint32_t wall;          // bit f set: face f (-x,+x,-y,+y,-z,+z) is a wall
    C wcorr[19][6];         // 6 w_i rho0 (xi_i . u_face): moving-wall term per face
    C shift[19];            // w_i rho0 rounded to C
    C omega;                // 1 / tau
    C guo;                  // 1 - 1 / (2 tau)
    C rho0;
    C F[3];                 // body-force density
    double theta_r, theta_c;
    C *block_max;           // [nbz][nby][nbx]
    int8_t *flags;          // [nbz][nby][nbx]
    unsigned long long *acc;  // per block (count << 32 | max bits), zero between sensor steps
};

// Workgroups are dealt to the 8 XCDs round-robin by workgroup id.  Renumber
// tiles so that XCD j receives one contiguous run of tiles (x fastest): the
// cache lines that straddle two x-neighbouring tiles are then fetched into
// the same L2 by consecutive workgroups.  Bijective for any tile count.
__device__ __forceinline__ int xcd_tile(int b, int n) {
    const int q = n >> 3, r = n & 7;
    const int xcd = b & 7, local = b >> 3;
    return xcd * q + min(xcd, r) + local;
}

// Maximum that propagates NaN from either side.
template <typename C>
__device__ __forceinline__ C nan_max(C a, C b) {
    return (a != a || b > a || b != b) ? ((a != a) ? a : b) : a;
}

template <int Q, int I, typename C>
__device__ __forceinline__ C dot_c(const C (&u)[3]) {
    using V = Vel<Q, I>;
    C s = C(0);
    if constexpr (V::x != 0) s += C(V::x) * u[0];
    if constexpr (V::y != 0) s += C(V::y) * u[1];
    if constexpr (V::z != 0) s += C(V::z) * u[2];
    return s;
}

// x * w for a lattice weight w known at compile time.  In float the weight
// is carried as w_hi + w_lo (w_hi = w rounded to float) and the product
// formed with one FMA, which rounds x * w almost always correctly.
template <typename C, double W>
__device__ __forceinline__ C wmul(C x) {
    if constexpr (sizeof(C) == 4) {
        constexpr float hi = static_cast<float>(W);
        constexpr float lo = static_cast<float>(W - static_cast<double>(hi));
        return __builtin_fmaf(x, hi, x * lo);
    } else {
        return x * C(W);
    }
}

// Pull-stream with boundary conditions: the q shifted populations of cell
// (x, y, z) after streaming, d_i = f_i(x) - w_i rho0.
template <int Q, typename T, typename C, bool SHIFTED>
__device__ __forceinline__ void pull(const StepArgs<C> &a, int x, int y, int z, C (&d)[Q]) {
    constexpr int D = Lattice<Q>::D;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    // "m": source of a population moving in +axis (coordinate - 1); "p": in -axis
    const bool wxm = (x == 0) && (a.wall & 1u);
    const bool wxp = (x == nx - 1) && (a.wall & 2u);
    const bool wym = (y == 0) && (a.wall & 4u);
    const bool wyp = (y == ny - 1) && (a.wall & 8u);
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;
    bool wzm = false, wzp = false;
    int zm = z, zp = z;
    if constexpr (D == 3) {
        wzm = (z == 0) && (a.wall & 16u);
        wzp = (z == nz - 1) && (a.wall & 32u);
        zm = (z == 0) ? nz - 1 : z - 1;
        zp = (z == nz - 1) ? 0 : z + 1;
    }
    const uint32_t cell = (uint32_t)((z * ny + y) * nx + x);
    const char *base = static_cast<const char *>(a.src);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        // both candidate sources lie in planes i and opp(i): address them from
        // the lower of the two so that the lane offset stays non-negative
        constexpr int lo = (V::opp < i) ? V::opp : i;
        const int sx = (V::x > 0) ? xm : ((V::x < 0) ? xp : x);
        const int sy = (V::y > 0) ? ym : ((V::y < 0) ? yp : y);
        const int sz = (V::z > 0) ? zm : ((V::z < 0) ? zp : z);
        bool wall = false;
        C corr = C(0);
        if constexpr (V::x > 0) { wall = wall || wxm; corr += wxm ? a.wcorr[i][0] : C(0); }
        if constexpr (V::x < 0) { wall = wall || wxp; corr += wxp ? a.wcorr[i][1] : C(0); }
        if constexpr (V::y > 0) { wall = wall || wym; corr += wym ? a.wcorr[i][2] : C(0); }
        if constexpr (V::y < 0) { wall = wall || wyp; corr += wyp ? a.wcorr[i][3] : C(0); }
        if constexpr (V::z > 0) { wall = wall || wzm; corr += wzm ? a.wcorr[i][4] : C(0); }
        if constexpr (V::z < 0) { wall = wall || wzp; corr += wzp ? a.wcorr[i][5] : C(0); }
        const uint32_t nbr = (uint32_t)((sz * ny + sy) * nx + sx);
        const uint32_t e_pull = (uint32_t)(i - lo) * a.pitch + nbr;
        const uint32_t e_bounce = (uint32_t)(V::opp - lo) * a.pitch + cell;
        const uint32_t boff = (wall ? e_bounce : e_pull) * (uint32_t)sizeof(T);
        const T *p = reinterpret_cast<const T *>(base + (size_t)lo * a.pitch * sizeof(T) + boff);
        C v = static_cast<C>(*p);
        if constexpr (!SHIFTED) v -= a.shift[i];   // shift[i] == shift[opp(i)]
        d[i] = v + corr;                             // moving-wall term, 0 off walls
    });
}

// Moments, equilibrium, sensor, BGK + Guo collision and the store of one
// cell.  Returns the cell's sensor value: ||f^neq||^2 / ||f^eq||^2 (L2; the
// square root is taken once per block) or K_Kn.
template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, bool FORCE>
__device__ __forceinline__ C collide_store(const StepArgs<C> &a, uint32_t cell, const C (&d)[Q]) {
    // moments (Eqs. rho and u), Guo's half-force shift
    C drho = C(0), mx = C(0), my = C(0), mz = C(0);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        drho += d[i];
        if constexpr (V::x != 0) mx += C(V::x) * d[i];
        if constexpr (V::y != 0) my += C(V::y) * d[i];
        if constexpr (V::z != 0) mz += C(V::z) * d[i];
    });
    const C rho = a.rho0 + drho;
    const C inv_rho = C(1) / rho;
    C j[3] = {mx, my, mz};   // rho u
    if constexpr (FORCE) {
        j[0] += C(0.5) * a.F[0];
        j[1] += C(0.5) * a.F[1];
        j[2] += C(0.5) * a.F[2];
    }
    const C u[3] = {j[0] * inv_rho, j[1] * inv_rho, j[2] * inv_rho};
    const C usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    C uF = C(0);
    if constexpr (FORCE) uF = u[0] * a.F[0] + u[1] * a.F[1] + u[2] * a.F[2];

    C num = C(0), den = C(0), kkn = C(0);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        const C cu = dot_c<Q, i>(u);
        const C cj = dot_c<Q, i>(j);
        // f^eq_i - w_i rho0 = w_i [ (rho - rho0) + 3 xi.(rho u) + rho (9/2 cu^2 - 3/2 u^2) ],
        // rho (...) taken as rho0 (...) + (rho - rho0) (...)
        const C p2 = C(4.5) * cu * cu - C(1.5) * usq;
        const C br = drho + C(3) * cj + (a.rho0 * p2 + drho * p2);
        const C deq = wmul<C, V::w>(br);
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
        if constexpr (FORCE) {
            C cF = C(0);
            if constexpr (V::x != 0) cF += C(V::x) * a.F[0];
            if constexpr (V::y != 0) cF += C(V::y) * a.F[1];
            if constexpr (V::z != 0) cF += C(V::z) * a.F[2];
            out += a.guo * wmul<C, V::w>(C(3) * (cF - uF) + C(9) * cu * cF);
        }
        if constexpr (!SHIFTED) out += a.shift[i];
        // streaming store: the value is read back only in the next launch
        __builtin_nontemporal_store(static_cast<T>(out), dst + (size_t)i * a.pitch + cell);
    });
    if constexpr (SENSOR) {
        if constexpr (SKIND == kSensorL2) return num / den;
        else return kkn * C(1.0 / Q);
    }
    return C(0);
}

template <typename C>
__device__ __forceinline__ void write_block(const StepArgs<C> &a, int b, C M) {
    a.block_max[b] = M;
    const double Md = static_cast<double>(M);
    int8_t fl;
    if (!(Md == Md) || Md == HUGE_VAL) fl = 2;
    else if (Md > a.theta_r) fl = 1;
    else if (Md < a.theta_c) fl = -1;
    else fl = 0;
    a.flags[b] = fl;
}

// In-workgroup part of the block maximum: lanes 8k..8k+7 of a row hold one
// block column; returns, for threads (tx < BX/8, ty == 0), the maximum over
// the workgroup's 8 rows of block column tx.
template <int BX, typename C>
__device__ __forceinline__ C tile_block_max(C m) {
    m = nan_max(m, static_cast<C>(__shfl_xor(m, 1)));
    m = nan_max(m, static_cast<C>(__shfl_xor(m, 2)));
    m = nan_max(m, static_cast<C>(__shfl_xor(m, 4)));
    __shared__ C red[kTileY][BX / kBlockEdge];
    if ((threadIdx.x & (kBlockEdge - 1)) == 0) red[threadIdx.y][threadIdx.x / kBlockEdge] = m;
    __syncthreads();
    C M = C(0);
    if (threadIdx.y == 0 && threadIdx.x < BX / kBlockEdge) {
        M = red[0][threadIdx.x];
#pragma unroll
        for (int r = 1; r < kTileY; ++r) M = nan_max(M, red[r][threadIdx.x]);
    }
    return M;
}

template <int SKIND, typename C>
__device__ __forceinline__ C finish(C M) {
    if constexpr (SKIND == kSensorL2) return sqrt(M);   // sqrt is monotone
    else return M;
}

template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, bool FORCE, int BX>
__global__ __launch_bounds__(BX *kTileY) void step_cells(const StepArgs<C> a) {
    constexpr int D = Lattice<Q>::D;
    static_assert(BX % kBlockEdge == 0, "tile width must hold whole blocks");
    static_assert(D == 2 || !SENSOR || sizeof(C) == 4, "3D float64 uses step_zmarch");

    const int tile = xcd_tile(blockIdx.x, a.ntiles);
    const int tix = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int tiy = rest % a.nty;
    const int z = rest / a.nty;
    const int x = tix * BX + (int)threadIdx.x;
    const int y = tiy * kTileY + (int)threadIdx.y;

    C s = C(0);
    if (x < a.nx && y < a.ny) {
        C d[Q];
        pull<Q, T, C, SHIFTED>(a, x, y, z, d);
        s = collide_store<Q, T, C, SHIFTED, SENSOR, SKIND, FORCE>(a, (uint32_t)((z * a.ny + y) * a.nx + x), d);
    }
    if constexpr (SENSOR) {
        const C M = tile_block_max<BX>(s);
        if (threadIdx.y == 0 && threadIdx.x < BX / kBlockEdge) {
            const int bx = tix * (BX / kBlockEdge) + (int)threadIdx.x;
            if (bx < a.nbx) {
                if constexpr (D == 2) {
                    write_block(a, tiy * a.nbx + bx, finish<SKIND>(M));
                } else {
                    const int bz = z / kBlockEdge;
                    const int b = (bz * a.nby + tiy) * a.nbx + bx;
                    const unsigned need = (unsigned)min(kBlockEdge, a.nz - kBlockEdge * bz);
                    // M >= 0, +inf or NaN: unsigned order of the bits is a
                    // NaN-propagating max order
                    const unsigned mine = __float_as_uint(static_cast<float>(M));
                    unsigned long long old = a.acc[b], seen;
                    unsigned cnt, top;
                    do {
                        seen = old;
                        cnt = (unsigned)(seen >> 32) + 1u;
                        top = max(mine, (unsigned)seen);
                        const unsigned long long next =
                            (cnt == need) ? 0ull : (((unsigned long long)cnt << 32) | top);
                        old = atomicCAS(&a.acc[b], seen, next);
                    } while (old != seen);
                    if (cnt == need) write_block(a, b, finish<SKIND>(static_cast<C>(__uint_as_float(top))));
                }
            }
        }
    }
}

template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, bool FORCE, int BX>
__global__ __launch_bounds__(BX *kTileY) void step_zmarch(const StepArgs<C> a) {
    static_assert(Lattice<Q>::D == 3, "z-march is for 3D grids");
    const int tile = xcd_tile(blockIdx.x, a.ntiles);
    const int tix = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int tiy = rest % a.nty;
    const int tiz = rest / a.nty;
    const int x = tix * BX + (int)threadIdx.x;
    const int y = tiy * kTileY + (int)threadIdx.y;
    const int z0 = tiz * kBlockEdge;

    C m = C(0);
    if (x < a.nx && y < a.ny) {
        const int zend = min(z0 + kBlockEdge, a.nz);
#pragma unroll 1
        for (int z = z0; z < zend; ++z) {
            C d[Q];
            pull<Q, T, C, SHIFTED>(a, x, y, z, d);
            const C s = collide_store<Q, T, C, SHIFTED, SENSOR, SKIND, FORCE>(
                a, (uint32_t)((z * a.ny + y) * a.nx + x), d);
            if constexpr (SENSOR) m = nan_max(m, s);
        }
    }
    if constexpr (SENSOR) {
        const C M = tile_block_max<BX>(m);
        if (threadIdx.y == 0 && threadIdx.x < BX / kBlockEdge) {
            const int bx = tix * (BX / kBlockEdge) + (int)threadIdx.x;
            if (bx < a.nbx) write_block(a, (tiz * a.nby + tiy) * a.nbx + bx, finish<SKIND>(M));
        }
    }
}

}  // namespace lbm
