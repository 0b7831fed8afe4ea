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
// Three streaming schemes share the arithmetic:
//  * kPingPong: read S_{k-1} from one buffer (pull), write S_k to the other.
//  * In-place ("AA" pattern, one buffer): steps alternate between
//    kStream, which gathers the pre-collision populations from the
//    neighbours' opposite slots and scatters the post-collision ones to the
//    neighbours' own slots, and kLocal, which reads a cell's own slots and
//    writes its post-collision values back into the opposite slots.  After a
//    kStream step the buffer holds T(S_k) in natural order; after a kLocal
//    step it holds S_k with slot i <-> opp(i) exchanged.  A cell reads and
//    writes the same set of locations, so one buffer suffices, and the
//    working set of a step is half that of ping-pong: a 128^3 D3Q19 float
//    state (152 MiB) then stays in the 256 MB Infinity Cache.  Bounce-back
//    folds into the addressing of both halves of kStream.
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

#include <type_traits>

#include "lattice.hpp"

namespace lbm {

constexpr int kBlockEdge = 8;       // sensor block edge along every active axis
constexpr int kTileY = 8;           // rows per workgroup (one block row)
constexpr int kRowTileX = 256;      // row tiles: 256 cells of one grid row per workgroup
constexpr int kSensorL2 = 0;
constexpr int kSensorKKn = 1;
constexpr int kPingPong = 0;   // streaming schemes, see above
constexpr int kStream = 1;
constexpr int kLocal = 2;
constexpr int kModelForce = 1;   // collision-model bits: Guo body force
constexpr int kModelSmag = 2;    //                       Smagorinsky subgrid model

template <typename C>
struct StepArgs {
    const void *src;        // S_{k-1} (in-place schemes: the single buffer)
    void *dst;              // S_k (in-place schemes: the same buffer)
    uint32_t pitch;         // elements between population planes
    int nx, ny, nz;
    int ntx, nty, ntiles;   // tiles along x, y; total tiles (workgroups)
    int nbx, nby;           // sensor blocks along x, y
    uint32_t wall;          // bit f set: face f (-x,+x,-y,+y,-z,+z) is a wall
    C wcorr[kMaxQ][6];      // 6 w_i rho0 (xi_i . u_face): moving-wall term per face
    uint32_t profile;       // bit f set: face f's velocity is smoothed (axis_profile)
    C shift[kMaxQ];         // w_i rho0 rounded to C
    C omega;                // 1 / tau
    C guo;                  // 1 - 1 / (2 tau)
    C tau0;                 // tau (Smagorinsky: the molecular part)
    C smag;                 // 18 sqrt(2) C_smag^2 (Smagorinsky closed form)
    C rho0;
    C F[3];                 // body-force density
    double theta_r, theta_c;
    uint32_t step;          // index of the step this launch computes (stochastic rounding key)
    double *avg;            // per-cell running sums of the sensor in float64 (time average); nullptr: off
    C *block_max;           // [nbz][nby][nbx]
    int8_t *flags;          // [nbz][nby][nbx]
    unsigned long long *acc;  // per block (count << 32 | max bits), zero between steps; row tiles
                              // fold max bits into its low 32-bit half
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

// threadIdx.y of a BX x 8 workgroup.  When BX is a multiple of the wave
// width every wave lies in one row, so the value is read once per wave into
// a scalar register and everything derived from y stays scalar.
template <int BX>
__device__ __forceinline__ int wave_row() {
    if constexpr (BX % 64 == 0) return __builtin_amdgcn_readfirstlane((int)threadIdx.y);
    else return (int)threadIdx.y;
}

// Maximum that propagates NaN from either side.
template <typename C>
__device__ __forceinline__ C nan_max(C a, C b) {
    return (a != a || b > a || b != b) ? ((a != a) ? a : b) : a;
}

// xi_I . v, summed over the non-zero components of xi_I only (IEEE rules
// keep a compiler from dropping an addition of +0, so none is written).
template <int Q, int I, typename C>
__device__ __forceinline__ C dot_c(const C (&u)[3]) {
    constexpr int c[3] = {Vel<Q, I>::x, Vel<Q, I>::y, Vel<Q, I>::z};
    constexpr int f = c[0] ? 0 : (c[1] ? 1 : (c[2] ? 2 : 3));
    if constexpr (f == 3) {
        return C(0);
    } else {
        C s = (c[f] > 0) ? u[f] : -u[f];
        static_for<f + 1, 3>([&](auto ac) {
            constexpr int k = decltype(ac)::value;
            if constexpr (c[k] > 0) s += u[k];
            else if constexpr (c[k] < 0) s -= u[k];
        });
        return s;
    }
}

// First population with a non-zero component along axis A, or Q if none.
template <int Q, int A>
constexpr int first_on_axis() {
    for (int i = 1; i < Q; ++i)
        if (Lattice<Q>::c[i][A] != 0) return i;
    return Q;
}

// Density offset rho - rho0 and momentum sum_i xi_i d_i of the shifted
// populations, each summed in population order starting from its first
// term.  (Pairing opposite populations, d_I - d_opp(I), would save a few
// additions but biases float32 rounding of the momentum: in a force-driven
// channel the drift of the velocity profile grows threefold.)
template <int Q, typename C>
__device__ __forceinline__ void cell_moments(const C (&d)[Q], C &drho, C (&m)[3]) {
    drho = d[0];
    m[0] = m[1] = m[2] = C(0);
    static_for<1, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        drho += d[i];
        constexpr int c[3] = {V::x, V::y, V::z};
        static_for<0, 3>([&](auto ac) {
            constexpr int k = decltype(ac)::value;
            if constexpr (c[k] != 0) {
                const C t = (c[k] > 0) ? d[i] : -d[i];
                if constexpr (i == first_on_axis<Q, k>()) m[k] = t;
                else m[k] += t;
            }
        });
    });
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

// Wall-velocity factor of a smoothed face along one in-plane axis (the lid
// profile of Sec. 5.1): (1 - s^18)^2 with s = (2 c + 1 - n) / n the cell
// centre mapped to (-1, 1).  An axis of one cell has s = 0, factor 1.
template <typename C>
__device__ __forceinline__ C axis_profile(int c, int n) {
    const C s = C(2 * c + 1 - n) / C(n);
    const C s2 = s * s, s4 = s2 * s2, s8 = s4 * s4;
    const C t = C(1) - s8 * s8 * s2;
    return t * t;
}

// Neighbourhood of one cell: the element offsets from the cell to its x - 1
// ("m") and x + 1 ("p") neighbours along each axis, with periodic wrap,
// whether that neighbour lies beyond a wall face, and per face the factor of
// that face's wall velocity at the cell: 0 off the face, 1 next to it, or for
// a smoothed face the product of axis_profile over the face's in-plane axes.
// Formed once per cell, so that every link is a sum of offsets and a
// branch-free moving-wall term.  When y and z are the same across a wave
// (one grid row per wave) their offsets and flags are wave-uniform and live
// in scalar registers.
template <typename C>
struct Geo {
    int x, y, z;
    uint32_t cell;
    int dxm, dxp, dym, dyp, dzm, dzp;
    bool wxm, wxp, wym, wyp, wzm, wzp;
    C fw[6];
};

template <int D, typename C>
__device__ __forceinline__ Geo<C> make_geo(const StepArgs<C> &a, int x, int y, int z) {
    Geo<C> g;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int row = nx, slab = nx * ny;
    g.x = x; g.y = y; g.z = z;
    g.wxm = (x == 0) && (a.wall & 1u);
    g.wxp = (x == nx - 1) && (a.wall & 2u);
    g.wym = (y == 0) && (a.wall & 4u);
    g.wyp = (y == ny - 1) && (a.wall & 8u);
    g.dxm = (x == 0) ? nx - 1 : -1;
    g.dxp = (x == nx - 1) ? 1 - nx : 1;
    g.dym = (y == 0) ? (ny - 1) * row : -row;
    g.dyp = (y == ny - 1) ? (1 - ny) * row : row;
    g.wzm = g.wzp = false;
    g.dzm = g.dzp = 0;
    if constexpr (D == 3) {
        g.wzm = (z == 0) && (a.wall & 16u);
        g.wzp = (z == nz - 1) && (a.wall & 32u);
        g.dzm = (z == 0) ? (nz - 1) * slab : -slab;
        g.dzp = (z == nz - 1) ? (1 - nz) * slab : slab;
    }
    g.cell = (uint32_t)(z * slab + y * row + x);
    C pf[6] = {C(1), C(1), C(1), C(1), C(1), C(1)};
    if (a.profile) {
        const C t[3] = {axis_profile<C>(x, nx), axis_profile<C>(y, ny), axis_profile<C>(z, nz)};
        const C face[3] = {t[1] * t[2], t[0] * t[2], t[0] * t[1]};
#pragma unroll
        for (int f = 0; f < 6; ++f)
            if ((a.profile >> f) & 1u) pf[f] = face[f / 2];
    }
    const bool on[6] = {g.wxm, g.wxp, g.wym, g.wyp, g.wzm, g.wzp};
#pragma unroll
    for (int f = 0; f < 6; ++f) g.fw[f] = on[f] ? pf[f] : C(0);
    return g;
}

// The pull link of population I at the cell: its source cell x - xi_I (after
// periodic wrap), whether the source lies beyond a wall (then the link is
// bounced), and the moving-wall term 6 w_I rho0 (xi_I . u_w) summed over the
// faces xi_I crosses, each face's velocity times its factor at the cell (0
// off walls).
template <typename C>
struct Link {
    bool wall;
    uint32_t src;
    C corr;
};

template <int Q, int I, typename C>
__device__ __forceinline__ Link<C> link(const StepArgs<C> &a, const Geo<C> &g) {
    using V = Vel<Q, I>;
    // offset to x - xi_I: the row and slab parts first (wave-uniform when y, z are)
    int dyz = 0;
    if constexpr (V::y > 0) dyz += g.dym;
    if constexpr (V::y < 0) dyz += g.dyp;
    if constexpr (V::z > 0) dyz += g.dzm;
    if constexpr (V::z < 0) dyz += g.dzp;
    int dx = 0;
    if constexpr (V::x > 0) dx = g.dxm;
    if constexpr (V::x < 0) dx = g.dxp;
    Link<C> l;
    l.wall = false;
    l.corr = C(0);
    if constexpr (V::x > 0) { l.wall = l.wall || g.wxm; l.corr += a.wcorr[I][0] * g.fw[0]; }
    if constexpr (V::x < 0) { l.wall = l.wall || g.wxp; l.corr += a.wcorr[I][1] * g.fw[1]; }
    if constexpr (V::y > 0) { l.wall = l.wall || g.wym; l.corr += a.wcorr[I][2] * g.fw[2]; }
    if constexpr (V::y < 0) { l.wall = l.wall || g.wyp; l.corr += a.wcorr[I][3] * g.fw[3]; }
    if constexpr (V::z > 0) { l.wall = l.wall || g.wzm; l.corr += a.wcorr[I][4] * g.fw[4]; }
    if constexpr (V::z < 0) { l.wall = l.wall || g.wzp; l.corr += a.wcorr[I][5] * g.fw[5]; }
    l.src = g.cell + (uint32_t)(dx + dyz);
    return l;
}

// Storage policies.  A plain type (double, float, _Float16, __bf16) is stored
// with its conversion's rounding, to nearest even.  half_sr / bf16_sr store
// IEEE half / bfloat16 with stochastic rounding: a value between two
// representable neighbours goes to the upper one with probability equal to
// its distance from the lower one, in units of their spacing.  Rounding is
// then unbiased, so per-step increments smaller than half a unit in the last
// place are not lost (round-to-nearest would return the same stored value
// step after step).  The random bits come from a hash of (cell, population,
// step), so a run is reproducible bit for bit.
struct half_sr {};
struct bf16_sr {};

template <typename T>
struct Storage {
    using raw = T;
    static constexpr bool sr = false;
};
template <>
struct Storage<half_sr> {
    using raw = _Float16;
    static constexpr bool sr = true;
};
template <>
struct Storage<bf16_sr> {
    using raw = __bf16;
    static constexpr bool sr = true;
};

// MurmurHash3's 32-bit finaliser (Appleby), a bijective avalanche mix.
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

// Random bits for population `pop` of a cell: one full mix per (cell, step)
// (cell_key), then a cheap multiply-xorshift per population, whose upper bits
// are the ones the rounding uses.
__device__ __forceinline__ uint32_t cell_key(uint32_t cell, uint32_t step) {
    return mix32(cell * 0x9E3779B1u + step * 0x7FEB352Du + 0x2545F491u);
}

__device__ __forceinline__ uint32_t round_key(uint32_t ckey, int pop) {
    uint32_t h = (ckey ^ ((uint32_t)pop * 0x9E3779B9u)) * 0x85EBCA6Bu;
    return h ^ (h >> 15);
}

// x converted to the stored representation of policy T.
template <typename T, typename C>
__device__ __forceinline__ typename Storage<T>::raw to_storage(C x, uint32_t key) {
    if constexpr (std::is_same_v<T, bf16_sr>) {
        // bfloat16 keeps the upper 16 bits of a float: add a uniform 16-bit
        // dither to the dropped bits and truncate (finite values only)
        uint32_t b = __float_as_uint(static_cast<float>(x));
        if ((b & 0x7F800000u) != 0x7F800000u) b += key >> 16;
        return __builtin_bit_cast(__bf16, static_cast<uint16_t>(b >> 16));
    } else if constexpr (std::is_same_v<T, half_sr>) {
        // add uniform noise of one half-precision spacing, centred, then
        // round to nearest: the upper neighbour wins with the right probability
        const float xf = static_cast<float>(x);
        int e = (int)((__float_as_uint(xf) >> 23) & 0xFFu) - 127;
        e = e < -14 ? -14 : e;                                   // subnormal spacing 2^-24
        const float ulp = __uint_as_float((uint32_t)(e - 10 + 127) << 23);
        const float u = static_cast<float>(key >> 8) * 0x1p-24f;  // [0, 1)
        return static_cast<_Float16>(xf + (u - 0.5f) * ulp);
    } else {
        (void)key;
        return static_cast<T>(x);
    }
}

// Planes {I, opp(I)} hold both candidates of every access of population I,
// so an access is the base of the lower of the two planes (wave-uniform)
// plus a 32-bit byte offset: plane_of(I, plane) * pitch + cell elements,
// where plane_of is 0 for the lower plane and 1 for the upper one.  Choosing
// between a bounced and a streamed source is then a select of two offsets.
template <int Q, int I, typename T>
__device__ __forceinline__ typename Storage<T>::raw *pair_base(void *buf, uint32_t pitch) {
    using R = typename Storage<T>::raw;
    constexpr int lo = (Vel<Q, I>::opp < I) ? Vel<Q, I>::opp : I;
    return reinterpret_cast<R *>(static_cast<char *>(buf) + (size_t)lo * pitch * sizeof(R));
}

template <int Q, int I, typename T>
__device__ __forceinline__ uint32_t pair_off(uint32_t pitch, int plane, uint32_t cell) {
    using R = typename Storage<T>::raw;
    constexpr int lo = (Vel<Q, I>::opp < I) ? Vel<Q, I>::opp : I;
    return ((uint32_t)(plane - lo) * pitch + cell) * (uint32_t)sizeof(R);
}

template <typename R>
__device__ __forceinline__ R *at_byte(R *base, uint32_t off) {
    return reinterpret_cast<R *>(reinterpret_cast<char *>(base) + off);
}

template <int Q, int I, typename T>
__device__ __forceinline__ typename Storage<T>::raw *pair_addr(void *buf, uint32_t pitch, int plane,
                                                                uint32_t cell) {
    return at_byte(pair_base<Q, I, T>(buf, pitch), pair_off<Q, I, T>(pitch, plane, cell));
}

// The q pre-collision populations of the cell as shifted values
// d_i = f_i - w_i rho0, read according to the streaming scheme:
//   kPingPong: f_i = S_i(x - xi_i), or S_opp(i)(x) + term on a bounced link;
//   kStream  : the same values, found in the opposite slots of the single
//              buffer (S_i(y) is kept in slot opp(i) of y);
//   kLocal   : f_i is in slot i of the cell itself.
template <int Q, typename T, typename C, bool SHIFTED, int SCHEME>
__device__ __forceinline__ void load_cell(const StepArgs<C> &a, const Geo<C> &g, C (&d)[Q]) {
    void *src = const_cast<void *>(a.src);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int o = Vel<Q, i>::opp;
        if constexpr (SCHEME == kLocal || i == 0) {
            // no link crosses a face: the value is the cell's own
            const int plane = (SCHEME == kStream) ? o : i;
            C v = static_cast<C>(*pair_addr<Q, i, T>(src, a.pitch, plane, g.cell));
            if constexpr (!SHIFTED) v -= a.shift[i];
            d[i] = v;
        } else {
            const Link<C> l = link<Q, i>(a, g);
            const int plane_pull = (SCHEME == kPingPong) ? i : o;
            const int plane_bounce = (SCHEME == kPingPong) ? o : i;
            const uint32_t off = l.wall ? pair_off<Q, i, T>(a.pitch, plane_bounce, g.cell)
                                        : pair_off<Q, i, T>(a.pitch, plane_pull, l.src);
            C v = static_cast<C>(*at_byte(pair_base<Q, i, T>(src, a.pitch), off));
            if constexpr (!SHIFTED) v -= a.shift[i];   // shift[i] == shift[opp(i)]
            d[i] = v + l.corr;
        }
    });
}

// Store of the post-collision value of population I of the cell:
//   kPingPong: slot I of the cell in the other buffer (non-temporal);
//   kLocal   : slot opp(I) of the cell;
//   kStream  : slot I of the neighbour x + xi_I, the pre-collision place of
//              the next step; if x + xi_I lies beyond a wall the value
//              returns to the cell as opp(I) with the moving-wall term.
template <int Q, int I, typename T, typename C, int SCHEME>
__device__ __forceinline__ void store_pop(const StepArgs<C> &a, const Geo<C> &g, C out, uint32_t ckey) {
    constexpr int o = Vel<Q, I>::opp;
    const uint32_t key = Storage<T>::sr ? round_key(ckey, I) : 0u;
    if constexpr (SCHEME == kPingPong) {
        __builtin_nontemporal_store(to_storage<T>(out, key), pair_addr<Q, I, T>(a.dst, a.pitch, I, g.cell));
    } else if constexpr (SCHEME == kLocal || I == 0) {
        *pair_addr<Q, I, T>(a.dst, a.pitch, o, g.cell) = to_storage<T>(out, key);
    } else {
        // the scatter link of I is the pull link of opp(I) read backwards
        const Link<C> l = link<Q, o>(a, g);
        const uint32_t off = l.wall ? pair_off<Q, I, T>(a.pitch, o, g.cell) : pair_off<Q, I, T>(a.pitch, I, l.src);
        *at_byte(pair_base<Q, I, T>(a.dst, a.pitch), off) = to_storage<T>(out + l.corr, key);
    }
}

// Moments, equilibrium, sensor and BGK + Guo collision of one cell; each
// post-collision value (a shifted population plus shift for the plain
// storages) goes to sink(integral_constant<I>, value, cell key).  Returns the
// cell's sensor value: ||f^neq||^2 / ||f^eq||^2 (L2; the square root is taken
// once per block) or K_Kn.
template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, int MODEL, typename Sink>
__device__ __forceinline__ C collide(const StepArgs<C> &a, const Geo<C> &g, const C (&d)[Q], Sink &&sink) {
    constexpr bool FORCE = (MODEL & kModelForce) != 0;
    constexpr bool SMAG = (MODEL & kModelSmag) != 0;
    // moments (Eqs. rho and u), Guo's half-force shift
    C drho, j[3];   // rho - rho0, rho u
    cell_moments<Q>(d, drho, j);
    const C rho = a.rho0 + drho;
    const C inv_rho = C(1) / rho;
    if constexpr (FORCE) {
        j[0] += C(0.5) * a.F[0];
        j[1] += C(0.5) * a.F[1];
        j[2] += C(0.5) * a.F[2];
    }
    const C u[3] = {j[0] * inv_rho, j[1] * inv_rho, j[2] * inv_rho};
    const C usq = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    C uF = C(0);
    if constexpr (FORCE) uF = u[0] * a.F[0] + u[1] * a.F[1] + u[2] * a.F[2];

    // Smagorinsky (the subgrid model of Sec. 4): the cell's relaxation time
    // tau_e = (tau + sqrt(tau^2 + 18 sqrt(2) C^2 |Pi| / rho)) / 2 from the
    // non-equilibrium momentum flux Pi = sum_i xi_i xi_i f^neq_i.
    C omega = a.omega, guo = a.guo;
    if constexpr (SMAG) {
        C pxx = C(0), pyy = C(0), pzz = C(0), pxy = C(0), pxz = C(0), pyz = C(0);
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            using V = Vel<Q, i>;
            const C cu = dot_c<Q, i>(u);
            const C cj = dot_c<Q, i>(j);
            const C p2 = C(4.5) * cu * cu - C(1.5) * usq;
            const C fneq = d[i] - wmul<C, V::w>(drho + C(3) * cj + (a.rho0 * p2 + drho * p2));
            if constexpr (V::x != 0) pxx += fneq;
            if constexpr (V::y != 0) pyy += fneq;
            if constexpr (V::z != 0) pzz += fneq;
            if constexpr (V::x * V::y != 0) pxy += C(V::x * V::y) * fneq;
            if constexpr (V::x * V::z != 0) pxz += C(V::x * V::z) * fneq;
            if constexpr (V::y * V::z != 0) pyz += C(V::y * V::z) * fneq;
        });
        const C pp = pxx * pxx + pyy * pyy + pzz * pzz + C(2) * (pxy * pxy + pxz * pxz + pyz * pyz);
        const C tau_e = C(0.5) * (a.tau0 + sqrt(a.tau0 * a.tau0 + a.smag * sqrt(pp) * inv_rho));
        omega = C(1) / tau_e;
        guo = C(1) - C(0.5) * omega;
    }

    C num = C(0), den = C(0), kkn = C(0);
    const uint32_t ckey = Storage<T>::sr ? cell_key(g.cell, a.step) : 0u;
    const C m15usq = C(-1.5) * usq;
    // Relaxation of population I given the bracket of its equilibrium,
    // f^eq_I - w_I rho0 = w_I [ (rho - rho0) + 3 xi_I.(rho u) + rho (9/2 (xi_I.u)^2 - 3/2 u^2) ].
    auto relax = [&](auto ic, C br, C cu) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
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
        C out = d[i] - omega * fneq;
        if constexpr (FORCE) {
            C cF = C(0);
            if constexpr (V::x != 0) cF += C(V::x) * a.F[0];
            if constexpr (V::y != 0) cF += C(V::y) * a.F[1];
            if constexpr (V::z != 0) cF += C(V::z) * a.F[2];
            out += guo * wmul<C, V::w>(C(3) * (cF - uF) + C(9) * cu * cF);
        }
        if constexpr (!SHIFTED) out += a.shift[i];
        sink(ic, out, ckey);
    };
    // rest population: xi = 0
    relax(std::integral_constant<int, 0>{}, drho + (a.rho0 * m15usq + drho * m15usq), C(0));
    // opposite pairs I, I + 1 share (xi.u)^2 and so the even part of the bracket,
    // rho - rho0 + rho (9/2 (xi.u)^2 - 3/2 u^2), with rho taken as rho0 + (rho - rho0)
    static_for<0, (Q - 1) / 2>([&](auto kc) {
        constexpr int i = 2 * decltype(kc)::value + 1;
        const C cu = dot_c<Q, i>(u);
        const C cj = dot_c<Q, i>(j);
        const C p2 = C(4.5) * cu * cu + m15usq;
        const C even = drho + (a.rho0 * p2 + drho * p2);
        relax(std::integral_constant<int, i>{}, even + C(3) * cj, cu);
        relax(std::integral_constant<int, i + 1>{}, even - C(3) * cj, -cu);
    });
    if constexpr (SENSOR) {
        if constexpr (SKIND == kSensorL2) return num / den;
        else return kkn * C(1.0 / Q);
    }
    return C(0);
}

// collide with the stores of the streaming scheme.
template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, int MODEL, int SCHEME>
__device__ __forceinline__ C collide_store(const StepArgs<C> &a, const Geo<C> &g, const C (&d)[Q]) {
    return collide<Q, T, C, SHIFTED, SENSOR, SKIND, MODEL>(a, g, d, [&](auto ic, C out, uint32_t ckey) {
        store_pop<Q, decltype(ic)::value, T, C, SCHEME>(a, g, out, ckey);
    });
}

// Refine / keep / coarsen decision of a block maximum (non-finite: 2).
__host__ __device__ __forceinline__ int8_t block_flag(double Md, double theta_r, double theta_c) {
    if (!(Md == Md) || Md == HUGE_VAL) return 2;
    if (Md > theta_r) return 1;
    if (Md < theta_c) return -1;
    return 0;
}

template <typename C>
__device__ __forceinline__ void write_block(const StepArgs<C> &a, int b, C M) {
    a.block_max[b] = M;
    a.flags[b] = block_flag(static_cast<double>(M), a.theta_r, a.theta_c);
}

// In-workgroup part of the block maximum: lanes 8k..8k+7 of a row hold one
// block column; returns, for threads (tx < BX/8, ty == 0), the maximum over
// the workgroup's TY rows of block column tx.
template <int BX, int TY, typename C>
__device__ __forceinline__ C tile_block_max(C m) {
    if constexpr (sizeof(C) == 4) {
        // Sensor values are >= 0, +inf or NaN, so the unsigned order of their
        // bits is a NaN-propagating max order: the max over each group of 8
        // lanes takes three DPP moves (swap neighbours, swap pairs, mirror
        // the half row) and unsigned maxima, with every lane active.
        unsigned u = __float_as_uint(static_cast<float>(m));
        u = max(u, static_cast<unsigned>(__builtin_amdgcn_mov_dpp(static_cast<int>(u), 0xB1, 0xF, 0xF, false)));
        u = max(u, static_cast<unsigned>(__builtin_amdgcn_mov_dpp(static_cast<int>(u), 0x4E, 0xF, 0xF, false)));
        u = max(u, static_cast<unsigned>(__builtin_amdgcn_mov_dpp(static_cast<int>(u), 0x141, 0xF, 0xF, false)));
        m = static_cast<C>(__uint_as_float(u));
    } else {
        m = nan_max(m, static_cast<C>(__shfl_xor(m, 1)));
        m = nan_max(m, static_cast<C>(__shfl_xor(m, 2)));
        m = nan_max(m, static_cast<C>(__shfl_xor(m, 4)));
    }
    __shared__ C red[TY][BX / kBlockEdge];
    if ((threadIdx.x & (kBlockEdge - 1)) == 0) red[threadIdx.y][threadIdx.x / kBlockEdge] = m;
    __syncthreads();
    C M = C(0);
    if (threadIdx.y == 0 && threadIdx.x < BX / kBlockEdge) {
        M = red[0][threadIdx.x];
#pragma unroll
        for (int r = 1; r < TY; ++r) M = nan_max(M, red[r][threadIdx.x]);
    }
    return M;
}

template <int SKIND, typename C>
__device__ __forceinline__ C finish(C M) {
    if constexpr (SKIND == kSensorL2) return sqrt(M);   // sqrt is monotone
    else return M;
}

// Time average of the cell sensor (the averaged sensor of Sec. 5.1): adds the
// cell's sensor value to its running sum when averaging is switched on.  The
// sums are float64 whatever the arithmetic type: over windows of 10^4 sensor
// steps a float32 sum would lose ~10^4 half-ulps, far above the sensor's own
// float32 error.
template <int SKIND, typename C>
__device__ __forceinline__ void accumulate(const StepArgs<C> &a, uint32_t cell, C s) {
    if (a.avg) a.avg[cell] += static_cast<double>(finish<SKIND>(s));
}

// Tiles of BX x TY cells of one z-slice.  TY = 8 (one block row) is dealt to
// the XCDs in contiguous runs (xcd_tile), which keeps the lines shared by
// x-neighbouring tiles in one L2: the better order while the state fits the
// Infinity Cache.  TY = 1 (row tiles, 3D ping-pong only) takes the natural
// order instead, so that the whole chip streams through one compact window
// of every population plane: measured on a 256^3 float32 state (2.5 GB per
// step), the plain pull pattern runs at 73% of the HBM peak with row tiles
// in natural order and at 68% with 128 x 8 tiles in XCD runs.  Row tiles
// complete a block maximum across 8 rows x 8 slices of workgroups.
template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, int MODEL, int BX, int SCHEME,
          int TY = kTileY>
__global__ __launch_bounds__(BX *TY) void step_cells(const StepArgs<C> a) {
    constexpr int D = Lattice<Q>::D;
    static_assert(BX % kBlockEdge == 0, "tile width must hold whole blocks");
    static_assert(D == 2 || !SENSOR || sizeof(C) == 4, "3D float64 uses step_zmarch");
    static_assert(TY == kTileY || (D == 3 && kTileY % TY == 0), "row tiles are for 3D grids");

    const int tile = (TY == kTileY) ? xcd_tile(blockIdx.x, a.ntiles) : (int)blockIdx.x;
    const int tix = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int tiy = rest % a.nty;
    const int z = rest / a.nty;
    const int x = tix * BX + (int)threadIdx.x;
    const int y = tiy * TY + wave_row<BX>();

    C s = C(0);
    if (x < a.nx && y < a.ny) {
        const Geo<C> g = make_geo<D>(a, x, y, z);
        C d[Q];
        load_cell<Q, T, C, SHIFTED, SCHEME>(a, g, d);
        s = collide_store<Q, T, C, SHIFTED, SENSOR, SKIND, MODEL, SCHEME>(a, g, d);
        if constexpr (SENSOR) accumulate<SKIND>(a, g.cell, s);
    }
    if constexpr (SENSOR) {
        const C M = tile_block_max<BX, TY>(s);
        if (threadIdx.y == 0 && threadIdx.x < BX / kBlockEdge) {
            const int bx = tix * (BX / kBlockEdge) + (int)threadIdx.x;
            if (bx < a.nbx) {
                if constexpr (D == 2) {
                    write_block(a, tiy * a.nbx + bx, finish<SKIND>(M));
                } else {
                    const int bz = z / kBlockEdge;
                    const int by = (tiy * TY) / kBlockEdge;
                    const int b = (bz * a.nby + by) * a.nbx + bx;
                    // M >= 0, +inf or NaN: unsigned order of the bits is a
                    // NaN-propagating max order
                    const unsigned mine = __float_as_uint(static_cast<float>(M));
                    if constexpr (TY < kTileY) {
                        // Row tiles: 64 workgroups meet in a block, most of them at
                        // the same time, so a compare-and-swap loop would retry
                        // (measured: +50% on a 256^3 step).  Each folds its maximum
                        // into the low half of the block's word with one atomic max
                        // and nothing else; finish_blocks_kernel, launched right
                        // after the step, writes the block maxima and flags and
                        // clears the words.
                        unsigned *w32 = reinterpret_cast<unsigned *>(a.acc);
                        __hip_atomic_fetch_max(&w32[2 * b], mine, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        return;
                    }
                    // contributions to block (bx, by, bz): one per z-slice of the block
                    const unsigned need = (unsigned)min(kBlockEdge, a.nz - kBlockEdge * bz);
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

template <int Q, typename T, typename C, bool SHIFTED, bool SENSOR, int SKIND, int MODEL, int BX>
__global__ __launch_bounds__(BX *kTileY) void step_zmarch(const StepArgs<C> a) {
    static_assert(Lattice<Q>::D == 3, "z-march is for 3D grids");
    const int tile = xcd_tile(blockIdx.x, a.ntiles);
    const int tix = tile % a.ntx;
    const int rest = tile / a.ntx;
    const int tiy = rest % a.nty;
    const int tiz = rest / a.nty;
    const int x = tix * BX + (int)threadIdx.x;
    const int y = tiy * kTileY + wave_row<BX>();
    const int z0 = tiz * kBlockEdge;

    C m = C(0);
    if (x < a.nx && y < a.ny) {
        const int zend = min(z0 + kBlockEdge, a.nz);
#pragma unroll 1
        for (int z = z0; z < zend; ++z) {
            const Geo<C> g = make_geo<3>(a, x, y, z);
            C d[Q];
            load_cell<Q, T, C, SHIFTED, kPingPong>(a, g, d);
            const C s = collide_store<Q, T, C, SHIFTED, SENSOR, SKIND, MODEL, kPingPong>(a, g, d);
            if constexpr (SENSOR) {
                m = nan_max(m, s);
                accumulate<SKIND>(a, g.cell, s);
            }
        }
    }
    if constexpr (SENSOR) {
        const C M = tile_block_max<BX, kTileY>(m);
        if (threadIdx.y == 0 && threadIdx.x < BX / kBlockEdge) {
            const int bx = tix * (BX / kBlockEdge) + (int)threadIdx.x;
            if (bx < a.nbx) write_block(a, (tiz * a.nby + tiy) * a.nbx + bx, finish<SKIND>(M));
        }
    }
}

// Several sensor-free ping-pong steps of a 2D grid in one launch (temporal
// blocking), for grids too small to fill the chip, where a step lasts about
// as long as the latency of one small kernel.  A workgroup owns a tile of
// kMultiTile x kMultiTile cells and steps it together with a halo of
// kMultiHalo cells on every side, one cell per thread, keeping the
// post-collision populations in LDS between steps (two buffers, one barrier
// per step).  The first step pulls from global memory exactly as step_cells
// does; each later one pulls from the neighbours' LDS slots, a bounced link
// from the cell's own opposite slot with the moving-wall term, and the last
// stores the tile's own cells to the other buffer.  Across a periodic axis
// the halo holds the wrapped cells; across a wall it lies outside the grid
// and is never pulled from.  The outermost ring of the halo pulls from
// beyond it and so turns wrong one cell deeper at every step after the
// first: nsteps <= kMultiHalo + 1 leaves the tile exact.  The values kept in
// LDS are the stored values of the storage type, and the arithmetic is
// collide's, so the result equals nsteps launches of step_cells bit for bit.
constexpr int kMultiTile = 8;
constexpr int kMultiHalo = 4;
constexpr int kMultiEdge = kMultiTile + 2 * kMultiHalo;   // one cell per thread
constexpr int kMultiMaxSteps = kMultiHalo + 1;

template <int Q, typename T, typename C, bool SHIFTED, int MODEL>
__global__ __launch_bounds__(kMultiEdge *kMultiEdge) void step_multi(const StepArgs<C> a, int nsteps) {
    static_assert(Lattice<Q>::D == 2, "temporal blocking is for 2D grids");
    static_assert(!Storage<T>::sr, "stochastic rounding keys on the step index");
    using R = typename Storage<T>::raw;
    constexpr int E = kMultiEdge, NC = E * E;
    __shared__ R pop[2][Q * NC];
    const int me = threadIdx.x;
    const int ex = me % E, ey = me / E;
    const int ntx = (a.nx + kMultiTile - 1) / kMultiTile;
    const int x0 = (int)(blockIdx.x % ntx) * kMultiTile, y0 = (int)(blockIdx.x / ntx) * kMultiTile;
    const int ux = x0 - kMultiHalo + ex, uy = y0 - kMultiHalo + ey;   // unwrapped coordinates
    // an axis is periodic when neither of its faces is a wall (the host runs
    // this kernel only when both are, or neither)
    const int x = (a.wall & 3u) ? ux : ((ux % a.nx) + a.nx) % a.nx;
    const int y = (a.wall & 12u) ? uy : ((uy % a.ny) + a.ny) % a.ny;
    const bool inside = x >= 0 && x < a.nx && y >= 0 && y < a.ny;
    const bool own = ex >= kMultiHalo && ex < kMultiHalo + kMultiTile && ey >= kMultiHalo &&
                     ey < kMultiHalo + kMultiTile && ux < a.nx && uy < a.ny;
    Geo<C> g{};
    if (inside) g = make_geo<2>(a, x, y, 0);
    int cur = 0;
#pragma unroll 1
    for (int s = 0; s < nsteps; ++s) {
        if (inside) {
            C d[Q];
            if (s == 0) {
                load_cell<Q, T, C, SHIFTED, kPingPong>(a, g, d);
            } else {
                static_for<0, Q>([&](auto ic) {
                    constexpr int i = decltype(ic)::value;
                    using V = Vel<Q, i>;
                    const Link<C> l = link<Q, i>(a, g);
                    // the halo's outer ring reads a clamped (wrong, unused) neighbour
                    const int sx = min(max(ex - V::x, 0), E - 1), sy = min(max(ey - V::y, 0), E - 1);
                    const R raw = l.wall ? pop[cur][V::opp * NC + me] : pop[cur][i * NC + sy * E + sx];
                    C v = static_cast<C>(raw);
                    if constexpr (!SHIFTED) v -= a.shift[i];
                    if constexpr (i == 0) d[i] = v;
                    else d[i] = v + l.corr;
                });
            }
            if (s == nsteps - 1) {
                if (own)
                    collide<Q, T, C, SHIFTED, false, kSensorL2, MODEL>(a, g, d, [&](auto ic, C out, uint32_t ckey) {
                        store_pop<Q, decltype(ic)::value, T, C, kPingPong>(a, g, out, ckey);
                    });
            } else {
                collide<Q, T, C, SHIFTED, false, kSensorL2, MODEL>(a, g, d, [&](auto ic, C out, uint32_t) {
                    pop[cur ^ 1][decltype(ic)::value * NC + me] = to_storage<T>(out, 0u);
                });
            }
        }
        cur ^= 1;
        if (s + 1 < nsteps) __syncthreads();
    }
}

// Inverse of one in-place kStream step's scatter: from a buffer that holds
// T(S_k) in natural order (after kStream), writes S_k in natural order to
// `out` (same pitch).  S_i(x) sits in slot i of x + xi_i, or, when that
// neighbour lies beyond a wall, in slot opp(i) of x with the moving-wall term
// added.  One thread per cell.
template <int Q, typename T, typename C>
__global__ void unstream_kernel(const StepArgs<C> a, T *out) {
    constexpr int D = Lattice<Q>::D;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.nx * a.ny * a.nz) return;
    const int x = c % a.nx;
    const int y = (c / a.nx) % a.ny;
    const int z = c / (a.nx * a.ny);
    const Geo<C> g = make_geo<D>(a, x, y, z);
    void *src = const_cast<void *>(a.src);
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        constexpr int o = Vel<Q, i>::opp;
        const Link<C> l = link<Q, o>(a, g);
        const T *p = l.wall ? pair_addr<Q, i, T>(src, a.pitch, o, g.cell)
                            : pair_addr<Q, i, T>(src, a.pitch, i, l.src);
        const C v = static_cast<C>(*p) - l.corr;
        out[(size_t)i * a.pitch + g.cell] = static_cast<T>(v);
    });
}

}  // namespace lbm
