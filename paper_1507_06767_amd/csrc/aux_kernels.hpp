// aux_kernels.hpp -- kernels outside the time loop: state initialisation,
// host-transfer conversion, macroscopic fields and the conservation totals.
// None of them runs per step; all of them read or write the same SoA planes
// as the step kernel.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lattice.hpp"
#include "step_kernel.hpp"

namespace lbm {

// Conversions between the storage type and float64 (16-bit types go
// through float32).
template <typename T>
__device__ __forceinline__ T to_store(double v) {
    if constexpr (sizeof(T) == 2) return static_cast<T>(static_cast<float>(v));
    else return static_cast<T>(v);
}

template <typename T>
__device__ __forceinline__ double from_store(T v) {
    if constexpr (sizeof(T) == 2) return static_cast<double>(static_cast<float>(v));
    else return static_cast<double>(v);
}

template <typename T>
struct Planes {
    T *f;              // plane i at f + i*pitch
    int64_t pitch;
    int cells;
    double shift[kMaxQ];  // storage shift per population (0 for plain storage)
};

// Rest state: f_i = w_i rho0 (stored as f_i - shift_i).
template <int Q, typename T>
__global__ void init_rest_kernel(Planes<T> p, double rho0) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.cells) return;
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        p.f[(int64_t)i * p.pitch + c] = to_store<T>(Vel<Q, i>::w * rho0 - p.shift[i]);
    });
}

// Clears n 64-bit words (the per-block accumulators of the step kernel).
__global__ void zero_words_kernel(unsigned long long *p, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// out[opp(i)][c] = in[i][c]: between natural order and the exchanged-slot
// order of the in-place scheme (an involution).
template <int Q, typename T>
__global__ void swap_planes_kernel(const T *in, T *out, int64_t pitch, int cells) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cells) return;
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        out[(int64_t)Vel<Q, i>::opp * pitch + c] = in[(int64_t)i * pitch + c];
    });
}

// One plane from float64 staging: out = (T)(in - shift).
template <typename T>
__global__ void import_plane_kernel(const double *in, T *out, int cells, double shift) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < cells) out[c] = to_store<T>(in[c] - shift);
}

// One plane to float64 staging: out = (double)in + shift.
template <typename T>
__global__ void export_plane_kernel(const T *in, double *out, int cells, double shift) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c < cells) out[c] = from_store<T>(in[c]) + shift;
}

// f^eq(rho, u) of Eq. feq_i in float64, stored as f^eq_i - shift_i.
// rho == nullptr: rho0 everywhere; u == nullptr: at rest.  u has 3 planes.
template <int Q, typename T>
__global__ void equilibrium_kernel(Planes<T> p, const double *rho, const double *u, double rho0) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.cells) return;
    const double r = rho ? rho[c] : rho0;
    double uu[3] = {0.0, 0.0, 0.0};
    if (u) {
        uu[0] = u[c];
        uu[1] = u[(int64_t)p.cells + c];
        uu[2] = (Lattice<Q>::D == 3) ? u[2 * (int64_t)p.cells + c] : 0.0;
    }
    const double usq = uu[0] * uu[0] + uu[1] * uu[1] + uu[2] * uu[2];
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        const double cu = V::x * uu[0] + V::y * uu[1] + V::z * uu[2];
        const double feq = V::w * r * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq);
        p.f[(int64_t)i * p.pitch + c] = to_store<T>(feq - p.shift[i]);
    });
}

// rho = sum_i S_i and u = (sum_i xi_i S_i - F/2) / rho in float64.
template <int Q, typename T>
__global__ void macros_kernel(Planes<T> p, double *rho_out, double *u_out, double Fx, double Fy,
                              double Fz) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= p.cells) return;
    double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        const double v = from_store<T>(p.f[(int64_t)i * p.pitch + c]);
        rho += v + p.shift[i];
        if constexpr (V::x != 0) m[0] += V::x * v;   // the shifts cancel in pairs
        if constexpr (V::y != 0) m[1] += V::y * v;
        if constexpr (V::z != 0) m[2] += V::z * v;
    });
    if (rho_out) rho_out[c] = rho;
    if (u_out) {
        u_out[c] = (m[0] - 0.5 * Fx) / rho;
        u_out[(int64_t)p.cells + c] = (m[1] - 0.5 * Fy) / rho;
        u_out[2 * (int64_t)p.cells + c] = (m[2] - 0.5 * Fz) / rho;
    }
}

// Per-block means of (rho - rho0, u_x, u_y, u_z) from per-cell fields (one
// thread per block, cells summed in z, y, x order); edge blocks average the
// cells they hold.  Output [block][4].
__global__ void block_means_kernel(const double *rho, const double *u, int nx, int ny, int nz, int nbx, int nby,
                                   int nbz, int bz, double rho0, double *out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nbx * nby * nbz) return;
    const int ib = b % nbx, jb = (b / nbx) % nby, kb = b / (nbx * nby);
    const int64_t cells = (int64_t)nx * ny * nz;
    const int x1 = min(nx, 8 * ib + 8), y1 = min(ny, 8 * jb + 8), z1 = min(nz, bz * kb + bz);
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int z = bz * kb; z < z1; ++z)
        for (int y = 8 * jb; y < y1; ++y)
            for (int x = 8 * ib; x < x1; ++x) {
                const int64_t c = ((int64_t)z * ny + y) * nx + x;
                s[0] += rho[c] - rho0;
                s[1] += u[c];
                s[2] += u[cells + c];
                s[3] += u[2 * cells + c];
            }
    const double n = (double)((x1 - 8 * ib) * (y1 - 8 * jb) * (z1 - bz * kb));
    for (int k = 0; k < 4; ++k) out[4 * (int64_t)b + k] = s[k] / n;
}

// Refinement level of every block from its sensor maximum (Sec. 3.4):
// l = clamp(floor(a log2 M + b), lmin, lmax); non-finite M -> lmax, M <= 0 -> lmin.
template <typename C>
__global__ void levels_kernel(const C *bmax, int8_t *lev, int nblocks, double a, double b, int lmin,
                              int lmax) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nblocks) return;
    const double K = static_cast<double>(bmax[i]);
    int l;
    if (!(K == K) || K == HUGE_VAL) l = lmax;
    else if (K <= 0.0) l = lmin;
    else {
        const double x = floor(a * log2(K) + b);
        l = (x < lmin) ? lmin : (x > lmax) ? lmax : (int)x;
    }
    lev[i] = (int8_t)l;
}

// Buffer layer (Sec. 5.2): every block takes the largest level within `r`
// blocks of it (Chebyshev distance).
__global__ void dilate_kernel(const int8_t *in, int8_t *out, int nbx, int nby, int nbz, int r) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbx * nby * nbz) return;
    const int x = i % nbx, y = (i / nbx) % nby, z = i / (nbx * nby);
    int best = -128;
    for (int dz = -r; dz <= r; ++dz)
        for (int dy = -r; dy <= r; ++dy)
            for (int dx = -r; dx <= r; ++dx) {
                const int xx = x + dx, yy = y + dy, zz = z + dz;
                if (xx < 0 || yy < 0 || zz < 0 || xx >= nbx || yy >= nby || zz >= nbz) continue;
                const int v = in[(zz * nby + yy) * nbx + xx];
                best = v > best ? v : best;
            }
    out[i] = (int8_t)best;
}

// Block maxima and flags of a row-tile sensor step from the max bits its
// workgroups folded into the low halves of the accumulator words, which are
// cleared for the next sensor step; the L2 sensor's square root is taken
// here, once per block.
template <typename C>
__global__ void finish_blocks_kernel(unsigned *w32, int nblocks, bool l2, C *block_max, int8_t *flags,
                                     double theta_r, double theta_c) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    float M = __uint_as_float(w32[2 * b]);
    w32[2 * b] = 0u;
    if (l2) M = sqrtf(M);
    block_max[b] = static_cast<C>(M);
    flags[b] = block_flag(static_cast<double>(M), theta_r, theta_c);
}

// Per block: the largest time-averaged cell sensor, sum / samples, NaN-propagating
// (the per-cell sums are float64).
__global__ void average_block_max_kernel(const double *sum, double *out, int nx, int ny, int nz, int bx, int by,
                                         int bz, int nbx, int nby, int nbz, double inv_samples) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nbx * nby * nbz) return;
    const int x0 = (i % nbx) * bx, y0 = ((i / nbx) % nby) * by, z0 = (i / (nbx * nby)) * bz;
    double m = 0.0;
    bool nan = false;
    for (int z = z0; z < min(z0 + bz, nz); ++z)
        for (int y = y0; y < min(y0 + by, ny); ++y)
            for (int x = x0; x < min(x0 + bx, nx); ++x) {
                const double v = sum[((int64_t)z * ny + y) * nx + x] * inv_samples;
                if (!(v == v)) nan = true;
                else if (v > m) m = v;
            }
    out[i] = nan ? __longlong_as_double(0x7ff8000000000000ll) : m;
}

constexpr int kReduceThreads = 256;

// Fixed-order tree over the workgroup's 256 slots of 4 doubles.
__device__ __forceinline__ void tree_reduce4(double (*sh)[4], double acc[4]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < 4; ++k) sh[t][k] = acc[k];
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
#pragma unroll
            for (int k = 0; k < 4; ++k) sh[t][k] += sh[t + s][k];
        }
        __syncthreads();
    }
}

// Pass 1: workgroup g sums cells g*256 + t, stepping by the grid size, into
// partial[g][4] = (mass, momentum x, y, z).
template <int Q, typename T>
__global__ __launch_bounds__(kReduceThreads) void conservation_pass1(Planes<T> p, double *partial) {
    __shared__ double sh[kReduceThreads][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    const int stride = gridDim.x * kReduceThreads;
    for (int c = blockIdx.x * kReduceThreads + threadIdx.x; c < p.cells; c += stride) {
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            using V = Vel<Q, i>;
            const double v = from_store<T>(p.f[(int64_t)i * p.pitch + c]);
            acc[0] += v + p.shift[i];
            if constexpr (V::x != 0) acc[1] += V::x * v;
            if constexpr (V::y != 0) acc[2] += V::y * v;
            if constexpr (V::z != 0) acc[3] += V::z * v;
        });
    }
    tree_reduce4(sh, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) partial[4 * blockIdx.x + k] = sh[0][k];
}

// Pass 2: one workgroup folds the partials in a fixed order.
__global__ __launch_bounds__(kReduceThreads) void conservation_pass2(const double *partial, int n,
                                                                     double *out) {
    __shared__ double sh[kReduceThreads][4];
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int j = threadIdx.x; j < n; j += kReduceThreads)
        for (int k = 0; k < 4; ++k) acc[k] += partial[4 * j + k];
    tree_reduce4(sh, acc);
    if (threadIdx.x == 0)
        for (int k = 0; k < 4; ++k) out[k] = sh[0][k];
}

}  // namespace lbm
