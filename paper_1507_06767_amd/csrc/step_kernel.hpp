// step_kernel.hpp -- the fused lattice Boltzmann step + kinetic sensor for gfx950.
//
// One launch advances every cell by one step S_k = C(T(S_{k-1})) (Sec. 2.2:
// Eq. bgklb, equilibrium Eq. feq_i, moments Eqs. rho and u, then the
// collide-and-stream split) and, on sensor steps, evaluates the kinetic sensor
// of Sec. 3.2 on the pre-collision populations, reduces it to one maximum per
// sensor block and writes the refine / keep / coarsen flag of that block.
//
// Layout: structure of arrays, population plane i at element offset i*pitch,
// cell (x,y,z) at (z*ny + y)*nx + x.  Streaming is a PULL: population i of
// cell x is read from cell x - xi_i of the other buffer, so every stored value
// is read exactly once and every lane of a wave reads consecutive addresses of
// one plane (a row of 64 cells = 256 contiguous bytes in float32).  Walls are
// recognised from the coordinates; no geometry array is read.
//
// Work decomposition: a workgroup is BX x 8 threads; it owns a tile of BX
// cells in x by 8 rows in y and marches through 8 z-slices (1 in 2D), so a
// tile is exactly (BX/8) whole sensor blocks of 8x8x8 cells and the block
// maximum is finished inside the workgroup: 8-lane shuffles within a wave,
// then one LDS exchange across the 8 rows.  No atomics, no second pass.
//
// Arithmetic is done on the shifted populations d_i = f_i - w_i rho0, which
// keeps the float32 variants accurate: every quantity the sensor and the
// collision need (rho - rho0, rho u, f^neq, f^eq - w_i rho0) is a small
// number formed without cancellation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"

namespace lbm {

constexpr int kBlockEdge = 8;       // sensor block edge along every active axis
constexpr int kTileY = 8;           // rows per workgroup
constexpr int kSensorL2 = 0;
constexpr int kSensorKKn = 1;

template <typename C>
struct StepArgs {
    const void *src;        // S_{k-1}
    void *dst;              // S_k
    int64_t pitch;          // elements between population planes
    int nx, ny, nz;
    int ntx, nty, ntiles;   // tiles along x, y; total tiles
    int nbx, nby;           // sensor blocks along x, y
    uint32_t wall;          // bit f set: face f (-x,+x,-y,+y,-z,+z) is a wall
    C uw[6][3];             // wall velocity per face
    C shift[19];            // w_i rho0 rounded to C: the storage shift
    C omega;                // 1 / tau
    C guo;                  // 1 - 1 / (2 tau)
    C rho0;
    C F[3];                 // body-force density
    double theta_r, theta_c;
    C *block_max;           // [nbz][nby][nbx]
    int8_t *flags;          // [nbz][nby][nbx]
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

template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, bool FORCE, int BX>
__global__ __launch_bounds__(BX *kTileY) void step_kernel(const StepArgs<C> a) {
    constexpr int D = Lattice<Q>::D;
    constexpr int BZ = (D == 3) ? kBlockEdge : 1;
    static_assert(BX % kBlockEdge == 0, "tile width must hold whole blocks");

    const int tile = xcd_tile(blockIdx.x, a.ntiles);
    const int tix = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int tiy = rest % a.nty;
    const int tiz = rest / a.nty;

    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int x = tix * BX + (int)threadIdx.x;
    const int y = tiy * kTileY + (int)threadIdx.y;
    const int z0 = tiz * BZ;
    const bool active = (x < nx) && (y < ny);

    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const int64_t P = a.pitch;

    // Pull sources along x and y.  "m" is the source of a population moving
    // in +axis (it comes from coordinate - 1), "p" of one moving in -axis.
    const bool wxm = (x == 0) && (a.wall & 1u);
    const bool wxp = (x == nx - 1) && (a.wall & 2u);
    const int xm = (x == 0) ? nx - 1 : x - 1;
    const int xp = (x == nx - 1) ? 0 : x + 1;
    const bool wym = (y == 0) && (a.wall & 4u);
    const bool wyp = (y == ny - 1) && (a.wall & 8u);
    const int ym = (y == 0) ? ny - 1 : y - 1;
    const int yp = (y == ny - 1) ? 0 : y + 1;

    C run_max = C(0);   // ratio^2 (L2) or K_Kn, maximum over this thread's cells

    for (int dz = 0; dz < BZ; ++dz) {
        const int z = z0 + dz;
        if (!active || z >= nz) continue;
        bool wzm = false, wzp = false;
        int zm = z, zp = z;
        if constexpr (D == 3) {
            wzm = (z == 0) && (a.wall & 16u);
            wzp = (z == nz - 1) && (a.wall & 32u);
            zm = (z == 0) ? nz - 1 : z - 1;
            zp = (z == nz - 1) ? 0 : z + 1;
        }
        const int cell = (z * ny + y) * nx + x;

        // ---- pull-stream with boundary conditions ---------------------------
        C d[Q];
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            using V = Vel<Q, i>;
            const int sx = (V::x > 0) ? xm : ((V::x < 0) ? xp : x);
            const int sy = (V::y > 0) ? ym : ((V::y < 0) ? yp : y);
            const int sz = (V::z > 0) ? zm : ((V::z < 0) ? zp : z);
            bool wall = false;
            if constexpr (V::x > 0) wall = wall || wxm;
            if constexpr (V::x < 0) wall = wall || wxp;
            if constexpr (V::y > 0) wall = wall || wym;
            if constexpr (V::y < 0) wall = wall || wyp;
            if constexpr (V::z > 0) wall = wall || wzm;
            if constexpr (V::z < 0) wall = wall || wzp;
            const int off = wall ? cell : (sz * ny + sy) * nx + sx;
            const T *plane = src + (wall ? (int64_t)V::opp * P : (int64_t)i * P);
            C v = static_cast<C>(plane[off]);
            if constexpr (!SHIFTED) v -= a.shift[i];   // shift[i] == shift[opp(i)]
            if (wall) {
                // moving-wall term 6 w_i rho0 (xi_i . u_w), u_w summed over the
                // wall faces this link crosses
                C cuw = C(0);
                if constexpr (V::x > 0) { if (wxm) cuw += dot_c<Q, i>(a.uw[0]); }
                if constexpr (V::x < 0) { if (wxp) cuw += dot_c<Q, i>(a.uw[1]); }
                if constexpr (V::y > 0) { if (wym) cuw += dot_c<Q, i>(a.uw[2]); }
                if constexpr (V::y < 0) { if (wyp) cuw += dot_c<Q, i>(a.uw[3]); }
                if constexpr (V::z > 0) { if (wzm) cuw += dot_c<Q, i>(a.uw[4]); }
                if constexpr (V::z < 0) { if (wzp) cuw += dot_c<Q, i>(a.uw[5]); }
                v += C(6.0 * V::w) * a.rho0 * cuw;
            }
            d[i] = v;
        });

        // ---- moments (Eqs. rho and u), Guo's half-force shift ---------------
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
        C u[3];
        if constexpr (FORCE) {
            u[0] = (mx + C(0.5) * a.F[0]) * inv_rho;
            u[1] = (my + C(0.5) * a.F[1]) * inv_rho;
            u[2] = (mz + C(0.5) * a.F[2]) * inv_rho;
        } else {
            u[0] = mx * inv_rho;
            u[1] = my * inv_rho;
            u[2] = mz * inv_rho;
        }
        const C usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];

        // ---- equilibrium, sensor, BGK + Guo collision, store ----------------
        C num = C(0), den = C(0), kkn = C(0);
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            using V = Vel<Q, i>;
            constexpr C w = C(V::w);
            const C cu = dot_c<Q, i>(u);
            // f^eq_i - w_i rho0 = w_i [ (rho - rho0) + rho (3 cu + 9/2 cu^2 - 3/2 u^2) ]
            const C deq = w * (drho + rho * (cu * (C(3) + C(4.5) * cu) - C(1.5) * usq));
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
                const C uF = u[0] * a.F[0] + u[1] * a.F[1] + u[2] * a.F[2];
                out += a.guo * w * (C(3) * (cF - uF) + C(9) * cu * cF);
            }
            if constexpr (!SHIFTED) out += a.shift[i];
            dst[(int64_t)i * P + cell] = static_cast<T>(out);
        });

        if constexpr (SENSOR) {
            if constexpr (SKIND == kSensorL2) run_max = nan_max(run_max, num / den);
            else run_max = nan_max(run_max, kkn * C(1.0 / Q));
        }
    }

    if constexpr (SENSOR) {
        // lanes 8k..8k+7 of a wave hold the 8 x-columns of one block row
        C m = run_max;
        m = nan_max(m, static_cast<C>(__shfl_xor(m, 1)));
        m = nan_max(m, static_cast<C>(__shfl_xor(m, 2)));
        m = nan_max(m, static_cast<C>(__shfl_xor(m, 4)));
        __shared__ C red[kTileY][BX / kBlockEdge];
        if ((threadIdx.x & (kBlockEdge - 1)) == 0) red[threadIdx.y][threadIdx.x / kBlockEdge] = m;
        __syncthreads();
        if (threadIdx.y == 0 && threadIdx.x < BX / kBlockEdge) {
            C M = red[0][threadIdx.x];
#pragma unroll
            for (int r = 1; r < kTileY; ++r) M = nan_max(M, red[r][threadIdx.x]);
            if constexpr (SKIND == kSensorL2) M = sqrt(M);   // sqrt is monotone
            const int bx = tix * (BX / kBlockEdge) + (int)threadIdx.x;
            if (bx < a.nbx) {
                const int b = (tiz * a.nby + tiy) * a.nbx + bx;
                a.block_max[b] = M;
                const double Md = static_cast<double>(M);
                int8_t fl;
                if (!(Md == Md) || Md == HUGE_VAL) fl = 2;
                else if (Md > a.theta_r) fl = 1;
                else if (Md < a.theta_c) fl = -1;
                else fl = 0;
                a.flags[b] = fl;
            }
        }
    }
}

}  // namespace lbm
