// lbm.hip -- host runtime behind the C interface of include/lbm.h.
//
// Validates descriptors, lays out the caller's buffers, selects the kernel
// variant for (lattice, storage, sensor, force) and enqueues it on the
// caller's stream.  The library allocates no device memory; the only host
// allocation is the handle itself.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <type_traits>
#include <vector>

#include "lbm.h"
#include "aux_kernels.hpp"
#include "launch.hpp"
#include "step_kernel.hpp"

using namespace lbm;

namespace {

thread_local std::string g_error;

lbm_status fail(lbm_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(LBM_EHIP, "%s failed: %s", #expr, hipGetErrorString(e_));          \
    } while (0)

constexpr int kAuxThreads = 256;
constexpr int kMaxPartials = 1024;
constexpr size_t kAlign = 256;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Tile width: the narrowest of 32, 64, 128 that spans the grid's x extent,
// capped at 64 for the in-place scheme (measured best on the 128^3 cavity,
// whose state stays in the Infinity Cache); 3D ping-pong grids wider than 128
// cells take row tiles (kRowTileX cells of one row, natural dispatch order),
// which stream a state too large for that cache faster than 128 x 8 tiles in
// XCD runs (256^3: 73% against 68% of the HBM peak for the bare access
// pattern).  LBM_TILE_X (32, 64, 128, or 256 for row tiles) overrides it for
// tuning; row tiles are only taken by 3D ping-pong.
int tile_x_setting(int nx, bool inplace, int dim) {
    const bool rows_ok = !inplace && dim == 3;
    const char *s = std::getenv("LBM_TILE_X");
    if (s) {
        int v = std::atoi(s);
        if (v == 32 || v == 64 || v == 128) return v;
        if (v == kRowTileX) return rows_ok ? v : 128;
    }
    if (rows_ok && nx > 128) return kRowTileX;
    const int cap = inplace ? 64 : 128;
    const int fit = nx <= 32 ? 32 : (nx <= 64 ? 64 : 128);
    return fit < cap ? fit : cap;
}

// Rows of a tile of width tile_x.
int tile_rows(int tile_x) { return tile_x == kRowTileX ? 1 : kTileY; }

size_t plane_pad_setting() {
    const char *s = std::getenv("LBM_PLANE_PAD");
    if (s) {
        long v = std::atol(s);
        if (v >= 0 && v % 256 == 0 && v <= (1l << 24)) return (size_t)v;
    }
    return 512;
}

struct Layout {
    int q, dim;
    int64_t cells;
    int64_t pitch;        // elements between planes
    size_t elem;          // bytes per stored population value
    size_t cbytes;        // bytes per compute-type value (block maxima)
    int nb[3];
    int64_t nblocks;
    size_t bytes[LBM_NBUF];
    size_t acc_off;       // per-block accumulator words inside BLOCK_MAX
    size_t staging_off, partial_off, out_off;
    size_t avg_off;       // per-cell running sensor sums in float64 (time average)
    size_t lev_off;       // two per-block int8 level arrays
    size_t avgmax_off;    // per-block float64 maxima of the averaged sensor
    size_t means_off;     // per-block float64 means of (rho - rho0, u)
};

bool is_fin(double v) { return std::isfinite(v); }

lbm_status check_desc(const lbm_desc *d, Layout *L) {
    if (!d) return fail(LBM_EINVAL, "descriptor is NULL");
    if (d->abi_version != LBM_ABI_VERSION)
        return fail(LBM_EINVAL, "abi_version %u, library has %u", d->abi_version, LBM_ABI_VERSION);
    if (d->lattice != LBM_D2Q9 && d->lattice != LBM_D3Q19 && d->lattice != LBM_D3Q27)
        return fail(LBM_ENOTSUP, "lattice %d not supported (9, 19 or 27)", d->lattice);
    if (d->storage < LBM_F64 || d->storage > LBM_BF16_SHIFTED_SR)
        return fail(LBM_ENOTSUP, "storage %d not supported", d->storage);
    if (d->sensor_kind != LBM_SENSOR_L2 && d->sensor_kind != LBM_SENSOR_KKN)
        return fail(LBM_EINVAL, "sensor_kind %d", d->sensor_kind);
    const int dim = (d->lattice == LBM_D2Q9) ? 2 : 3;
    int64_t cells = 1;
    for (int a = 0; a < 3; ++a) {
        if (d->extent[a] < 1) return fail(LBM_EINVAL, "extent[%d] = %d < 1", a, d->extent[a]);
        cells *= d->extent[a];
    }
    if (dim == 2 && d->extent[2] != 1) return fail(LBM_EINVAL, "D2Q9 needs extent[2] == 1");
    if (cells >= (int64_t(1) << 31) - 1024) return fail(LBM_ENOTSUP, "grid of %lld cells exceeds 2^31", (long long)cells);
    const int want_bz = (dim == 3) ? kBlockEdge : 1;
    if (d->block[0] != kBlockEdge || d->block[1] != kBlockEdge || d->block[2] != want_bz)
        return fail(LBM_ENOTSUP, "sensor block {%d,%d,%d}: only {8,8,%d} is supported", d->block[0],
                    d->block[1], d->block[2], want_bz);
    for (int f = 0; f < 6; ++f)
        if (d->face_bc[f] != LBM_BC_PERIODIC && d->face_bc[f] != LBM_BC_WALL)
            return fail(LBM_EINVAL, "face_bc[%d] = %d", f, d->face_bc[f]);
    for (int a = 0; a < 3; ++a)
        if ((d->face_bc[2 * a] == LBM_BC_PERIODIC) != (d->face_bc[2 * a + 1] == LBM_BC_PERIODIC))
            return fail(LBM_EINVAL, "axis %d: a periodic face needs a periodic opposite face", a);
    if (dim == 2 && (d->face_bc[4] != LBM_BC_PERIODIC || d->face_bc[5] != LBM_BC_PERIODIC))
        return fail(LBM_EINVAL, "D2Q9: the z faces must be periodic");
    if (!is_fin(d->tau) || !(d->tau > 0.5)) return fail(LBM_EINVAL, "tau = %g must be > 1/2", d->tau);
    if (!is_fin(d->rho0) || !(d->rho0 > 0.0)) return fail(LBM_EINVAL, "rho0 = %g must be > 0", d->rho0);
    for (int a = 0; a < 3; ++a)
        if (!is_fin(d->force[a])) return fail(LBM_EINVAL, "force[%d] not finite", a);
    for (int f = 0; f < 6; ++f)
        for (int a = 0; a < 3; ++a)
            if (!is_fin(d->wall_u[f][a])) return fail(LBM_EINVAL, "wall_u[%d][%d] not finite", f, a);
    if (dim == 2 && (d->force[2] != 0.0)) return fail(LBM_EINVAL, "D2Q9: force[2] must be 0");
    if (!is_fin(d->theta_refine) || !is_fin(d->theta_coarsen) || d->theta_coarsen > d->theta_refine)
        return fail(LBM_EINVAL, "thresholds must be finite with theta_coarsen <= theta_refine");
    if (!is_fin(d->smagorinsky) || d->smagorinsky < 0.0 || d->smagorinsky > 1.0)
        return fail(LBM_EINVAL, "smagorinsky = %g must be in [0, 1]", d->smagorinsky);
    for (int f = 0; f < 6; ++f)
        if (d->wall_profile[f] != LBM_PROFILE_UNIFORM && d->wall_profile[f] != LBM_PROFILE_SMOOTH)
            return fail(LBM_EINVAL, "wall_profile[%d] = %d", f, d->wall_profile[f]);
    if (d->streaming < LBM_STREAMING_AUTO || d->streaming > LBM_STREAMING_INPLACE)
        return fail(LBM_EINVAL, "streaming = %d", d->streaming);
    if (d->streaming == LBM_STREAMING_INPLACE && d->lattice != LBM_D2Q9 && d->storage == LBM_F64)
        return fail(LBM_ENOTSUP, "3D float64 streams ping-pong only");

    L->q = d->lattice;
    L->dim = dim;
    L->cells = cells;
    L->elem = (d->storage == LBM_F64) ? 8 : (d->storage <= LBM_F32_SHIFTED ? 4 : 2);
    L->cbytes = (d->storage == LBM_F64) ? 8 : 4;   // block maxima in the arithmetic type
    const size_t plane = round_up((size_t)cells * L->elem, kAlign) + plane_pad_setting();
    L->pitch = (int64_t)(plane / L->elem);
    // the kernels address two adjacent planes with a 32-bit byte offset
    if (2 * plane >= (size_t(1) << 32))
        return fail(LBM_ENOTSUP, "grid of %lld cells: two population planes exceed 4 GiB", (long long)cells);
    L->nblocks = 1;
    for (int a = 0; a < 3; ++a) {
        const int e = (a == 2 && dim == 2) ? 1 : kBlockEdge;
        L->nb[a] = (d->extent[a] + e - 1) / e;
        L->nblocks *= L->nb[a];
    }
    L->bytes[LBM_BUF_F_A] = L->bytes[LBM_BUF_F_B] = plane * L->q;
    L->acc_off = round_up((size_t)L->nblocks * L->cbytes, kAlign);
    L->bytes[LBM_BUF_BLOCK_MAX] = L->acc_off + round_up((size_t)L->nblocks * 8, kAlign);
    L->bytes[LBM_BUF_FLAGS] = round_up((size_t)L->nblocks, kAlign);
    L->staging_off = 0;
    L->partial_off = round_up((size_t)cells * 8 * 4, kAlign);
    L->out_off = L->partial_off + round_up((size_t)kMaxPartials * 4 * 8, kAlign);
    L->avg_off = L->out_off + kAlign;
    L->lev_off = L->avg_off + round_up((size_t)cells * 8, kAlign);
    L->avgmax_off = L->lev_off + round_up((size_t)L->nblocks * 2, kAlign);
    L->means_off = L->avgmax_off + round_up((size_t)L->nblocks * 8, kAlign);
    L->bytes[LBM_BUF_SCRATCH] = L->means_off + round_up((size_t)L->nblocks * 4 * 8, kAlign);
    return LBM_OK;
}

lbm_status check_buffers(const lbm_desc *d, const Layout &L) {
    static const char *names[LBM_NBUF] = {"F_A", "F_B", "BLOCK_MAX", "FLAGS", "SCRATCH"};
    for (int b = 0; b < LBM_NBUF; ++b) {
        if (!d->buf[b]) return fail(LBM_EINVAL, "buffer %s is NULL", names[b]);
        if (d->buf_bytes[b] < L.bytes[b])
            return fail(LBM_EINVAL, "buffer %s has %zu bytes, needs %zu", names[b], d->buf_bytes[b],
                        L.bytes[b]);
        const size_t align = (b <= LBM_BUF_F_B) ? kAlign : 16;
        if ((uintptr_t)d->buf[b] % align)
            return fail(LBM_EINVAL, "buffer %s is not %zu-byte aligned", names[b], align);
        hipPointerAttribute_t attr;
        if (hipPointerGetAttributes(&attr, d->buf[b]) != hipSuccess || attr.type != hipMemoryTypeDevice) {
            (void)hipGetLastError();
            return fail(LBM_EINVAL, "buffer %s is not device memory", names[b]);
        }
    }
    for (int b = 0; b < LBM_NBUF; ++b)
        for (int c = b + 1; c < LBM_NBUF; ++c) {
            const uintptr_t b0 = (uintptr_t)d->buf[b], b1 = b0 + L.bytes[b];
            const uintptr_t c0 = (uintptr_t)d->buf[c], c1 = c0 + L.bytes[c];
            if (b0 < c1 && c0 < b1) return fail(LBM_EINVAL, "buffers %s and %s overlap", names[b], names[c]);
        }
    return LBM_OK;
}

}  // namespace

struct lbm_blocks {
    lbm_desc d;
    Layout L;
    hipStream_t stream;
    int device;
    int tile_x;
    bool inplace;             // in-place (single buffer) streaming, else ping-pong
    int cur;                  // ping-pong: 0 state in F_A, 1 state in F_B
    int phase;                // in-place: 0 F_A holds S_k with slots i <-> opp(i)
                              // exchanged; 1 F_A holds T(S_k) in natural order
    int64_t step;
    int64_t last_sensor_step; // -1: none since the state was set
    bool has_force;
    bool averaging;           // sensor steps add the cell sensor to running sums
    bool avg_started;         // the sums were cleared by lbm_sensor_average_begin
    int64_t avg_samples;      // sensor steps summed since averaging began
    uint32_t wall_mask;
    int multi;                // most sensor-free steps per step_multi launch (small 2D
                              // ping-pong grids), 0: one launch per step
    int graph_chunk;          // steps per graph replay (even), 0: launch step by step
    hipGraphExec_t graph[2];  // graph_chunk steps, by buffer parity
    std::vector<int8_t> flags_host;
    std::vector<unsigned char> bmax_host;
};

namespace {

// Streaming scheme: in place (one buffer, the AA pattern) when a buffer is at
// most 512 MiB, so that the working set of a step can stay in the Infinity
// Cache; ping-pong above, where the two are on par and ping-pong streams its
// stores non-temporally.  3D float64 always uses ping-pong (its z-march
// kernel).  An explicit choice in the descriptor wins; under
// LBM_STREAMING_AUTO the environment variable LBM_STREAMING=pingpong|inplace
// overrides the size rule (tests run both schemes that way).
bool multi_setting(const lbm_desc *d, const Layout &L);

bool inplace_setting(const lbm_desc *d, const Layout &L) {
    if (d->lattice != LBM_D2Q9 && d->storage == LBM_F64) return false;
    if (d->streaming == LBM_STREAMING_PINGPONG) return false;
    if (d->streaming == LBM_STREAMING_INPLACE) return true;
    const char *s = std::getenv("LBM_STREAMING");
    if (s && std::strcmp(s, "pingpong") == 0) return false;
    if (s && std::strcmp(s, "inplace") == 0) return true;
    if (multi_setting(d, L)) return false;   // small 2D grids: ping-pong, several steps per launch
    return L.bytes[LBM_BUF_F_A] <= (size_t(512) << 20);
}

// Several sensor-free steps per launch (step_multi, temporal blocking) for
// 2D grids of at most kMultiMaxCells cells, whose single steps are too short
// to fill the chip (4096 cells: 64 workgroups of 256 threads), in ping-pong
// streaming, without stochastic rounding (its random bits key on the step
// index); lbm_set_multistep switches it off or changes the step count.  Both
// faces of an axis are walls or both periodic (checked at creation).
constexpr int64_t kMultiMaxCells = int64_t(1) << 16;
bool multi_setting(const lbm_desc *d, const Layout &L) {
    if (d->lattice != LBM_D2Q9 || L.cells > kMultiMaxCells) return false;
    return d->storage != LBM_F16_SHIFTED_SR && d->storage != LBM_BF16_SHIFTED_SR;
}

// Buffer the step kernel reads.
void *state_ptr(lbm_blocks *h) {
    if (h->inplace) return h->d.buf[LBM_BUF_F_A];
    return h->d.buf[h->cur ? LBM_BUF_F_B : LBM_BUF_F_A];
}

double *scratch_d(lbm_blocks *h, size_t off) {
    return reinterpret_cast<double *>(static_cast<char *>(h->d.buf[LBM_BUF_SCRATCH]) + off);
}

// Storage shift of the auxiliary kernels: w_i rho0 for the shifted storage
// (exact in float64), 0 for the plain ones.
template <int Q, typename T>
Planes<T> planes_of(lbm_blocks *h, void *buf) {
    Planes<T> p{};
    p.f = static_cast<T *>(buf);
    p.pitch = h->L.pitch;
    p.cells = (int)h->L.cells;
    const bool shifted = h->d.storage >= LBM_F32_SHIFTED;
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        p.shift[i] = shifted ? Vel<Q, i>::w * h->d.rho0 : 0.0;
    });
    return p;
}

template <int Q, typename C>
StepArgs<C> step_args(lbm_blocks *h, const void *src, void *dst, bool zmarch, int tile_x) {
    StepArgs<C> a{};
    const lbm_desc &d = h->d;
    constexpr int D = Lattice<Q>::D;
    const int BZ = (D == 3) ? kBlockEdge : 1;
    a.src = src;
    a.dst = dst;
    a.pitch = (uint32_t)h->L.pitch;
    a.nx = d.extent[0];
    a.ny = d.extent[1];
    a.nz = d.extent[2];
    a.ntx = (a.nx + tile_x - 1) / tile_x;
    a.nty = (a.ny + tile_rows(tile_x) - 1) / tile_rows(tile_x);
    const int ntz = zmarch ? (a.nz + BZ - 1) / BZ : a.nz;
    a.ntiles = a.ntx * a.nty * ntz;
    a.nbx = h->L.nb[0];
    a.nby = h->L.nb[1];
    a.wall = h->wall_mask;
    a.profile = 0;
    for (int f = 0; f < 6; ++f)
        if (d.face_bc[f] == LBM_BC_WALL && d.wall_profile[f] == LBM_PROFILE_SMOOTH) a.profile |= 1u << f;
    static_for<0, Q>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        using V = Vel<Q, i>;
        a.shift[i] = (C)(V::w * d.rho0);
        for (int f = 0; f < 6; ++f) {
            const double cu = V::x * d.wall_u[f][0] + V::y * d.wall_u[f][1] + V::z * d.wall_u[f][2];
            a.wcorr[i][f] = (C)(6.0 * V::w * d.rho0 * cu);
        }
    });
    a.omega = (C)(1.0 / d.tau);
    a.guo = (C)(1.0 - 0.5 / d.tau);
    a.tau0 = (C)d.tau;
    a.smag = (C)(18.0 * std::sqrt(2.0) * d.smagorinsky * d.smagorinsky);
    a.rho0 = (C)d.rho0;
    for (int c = 0; c < 3; ++c) a.F[c] = (C)d.force[c];
    a.theta_r = d.theta_refine;
    a.theta_c = d.theta_coarsen;
    a.step = (uint32_t)(h->step + 1);
    a.avg = h->averaging ? reinterpret_cast<double *>(static_cast<char *>(d.buf[LBM_BUF_SCRATCH]) + h->L.avg_off)
                         : nullptr;
    a.block_max = static_cast<C *>(d.buf[LBM_BUF_BLOCK_MAX]);
    a.flags = static_cast<int8_t *>(d.buf[LBM_BUF_FLAGS]);
    a.acc = reinterpret_cast<unsigned long long *>(static_cast<char *>(d.buf[LBM_BUF_BLOCK_MAX]) +
                                                   h->L.acc_off);
    return a;
}

// Calls f.template operator()<Q, T>() for the handle's lattice and storage type.
template <int Q, typename F>
void with_storage_type(lbm_blocks *h, F &&f) {
    switch (h->d.storage) {
        case LBM_F64: f.template operator()<Q, double>(); break;
        case LBM_F16_SHIFTED:
        case LBM_F16_SHIFTED_SR: f.template operator()<Q, _Float16>(); break;
        case LBM_BF16_SHIFTED:
        case LBM_BF16_SHIFTED_SR: f.template operator()<Q, __bf16>(); break;
        default: f.template operator()<Q, float>(); break;
    }
}

template <typename F>
void with_types(lbm_blocks *h, F &&f) {
    if (h->d.lattice == 9) with_storage_type<9>(h, f);
    else if (h->d.lattice == 19) with_storage_type<19>(h, f);
    else with_storage_type<27>(h, f);
}

unsigned grid_for(int64_t n) { return (unsigned)((n + kAuxThreads - 1) / kAuxThreads); }

// The step kernel's per-block (count | max) words must read zero before a
// sensor step; they are cleared whenever a state is installed.
void reset_accumulators(lbm_blocks *h) {
    auto *acc = reinterpret_cast<unsigned long long *>(static_cast<char *>(h->d.buf[LBM_BUF_BLOCK_MAX]) +
                                                       h->L.acc_off);
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid_for(h->L.nblocks)), dim3(kAuxThreads), 0, h->stream,
                       acc, (int)h->L.nblocks);
}

// Row tiles leave a sensor step's block maxima as max bits in the
// accumulator words: the block maxima and flags are written from them right
// after the step (and the words cleared).
void finish_blocks(lbm_blocks *h) {
    auto *w32 = reinterpret_cast<unsigned *>(static_cast<char *>(h->d.buf[LBM_BUF_BLOCK_MAX]) + h->L.acc_off);
    const bool l2 = h->d.sensor_kind == LBM_SENSOR_L2;
    auto *fl = static_cast<int8_t *>(h->d.buf[LBM_BUF_FLAGS]);
    const unsigned g = grid_for(h->L.nblocks);
    // float storages only: 3D float64 steps with the z-march kernel
    hipLaunchKernelGGL(finish_blocks_kernel<float>, dim3(g), dim3(kAuxThreads), 0, h->stream, w32,
                       (int)h->L.nblocks, l2, static_cast<float *>(h->d.buf[LBM_BUF_BLOCK_MAX]), fl,
                       h->d.theta_refine, h->d.theta_coarsen);
}

template <int Q, typename T, typename C, bool SH>
void launch_step(lbm_blocks *h, bool sens) {
    void *src = state_ptr(h);
    void *dst = h->inplace ? src : h->d.buf[h->cur ? LBM_BUF_F_A : LBM_BUF_F_B];
    LaunchCfg c;
    c.stream = h->stream;
    c.scheme = !h->inplace ? kPingPong : (h->phase == 0 ? kStream : kLocal);
    c.sensor = sens;
    c.sensor_kind = h->d.sensor_kind;
    c.force = h->has_force;
    c.smag = h->d.smagorinsky > 0.0;
    constexpr bool zm = uses_zmarch<Q, C>();
    c.tile_x = zm ? 64 : h->tile_x;
    const StepArgs<C> a = step_args<Q, C>(h, src, dst, zm, c.tile_x);
    launch_step_kernel<Q, T, C, SH>(a, c);
    if (sens && c.tile_x == kRowTileX && c.scheme == kPingPong) finish_blocks(h);
}

// Where host data and initial states are written: the state buffer for
// ping-pong; F_B as staging for the in-place scheme (then exchanged into F_A
// by finish_import).
void *import_target(lbm_blocks *h) { return h->inplace ? h->d.buf[LBM_BUF_F_B] : state_ptr(h); }

void finish_import(lbm_blocks *h) {
    if (!h->inplace) return;
    with_types(h, [&]<int Q, typename T>() {
        hipLaunchKernelGGL((swap_planes_kernel<Q, T>), dim3(grid_for(h->L.cells)), dim3(kAuxThreads), 0,
                           h->stream, static_cast<const T *>(h->d.buf[LBM_BUF_F_B]),
                           static_cast<T *>(h->d.buf[LBM_BUF_F_A]), h->L.pitch, (int)h->L.cells);
    });
    h->phase = 0;
}

// A buffer holding S_k in natural order: the state buffer for ping-pong; for
// the in-place scheme, F_B after undoing the slot exchange or the last
// scatter of F_A.
void *canonical_state(lbm_blocks *h) {
    if (!h->inplace) return state_ptr(h);
    void *A = h->d.buf[LBM_BUF_F_A];
    void *B = h->d.buf[LBM_BUF_F_B];
    with_types(h, [&]<int Q, typename T>() {
        if (h->phase == 0) {
            hipLaunchKernelGGL((swap_planes_kernel<Q, T>), dim3(grid_for(h->L.cells)), dim3(kAuxThreads), 0,
                               h->stream, static_cast<const T *>(A), static_cast<T *>(B), h->L.pitch,
                               (int)h->L.cells);
        } else {
            using C = std::conditional_t<sizeof(T) == 8, double, float>;
            const StepArgs<C> a = step_args<Q, C>(h, A, B, false, h->tile_x);
            hipLaunchKernelGGL((unstream_kernel<Q, T, C>), dim3(grid_for(h->L.cells)), dim3(kAuxThreads), 0,
                               h->stream, a, static_cast<T *>(B));
        }
    });
    return B;
}

template <int Q>
void launch_step_q(lbm_blocks *h, bool sens) {
    switch (h->d.storage) {
        case LBM_F64: launch_step<Q, double, double, false>(h, sens); break;
        case LBM_F32: launch_step<Q, float, float, false>(h, sens); break;
        case LBM_F32_SHIFTED: launch_step<Q, float, float, true>(h, sens); break;
        case LBM_F16_SHIFTED: launch_step<Q, _Float16, float, true>(h, sens); break;
        case LBM_BF16_SHIFTED: launch_step<Q, __bf16, float, true>(h, sens); break;
        case LBM_F16_SHIFTED_SR: launch_step<Q, half_sr, float, true>(h, sens); break;
        default: launch_step<Q, bf16_sr, float, true>(h, sens); break;
    }
}

void launch_step_any(lbm_blocks *h, bool sens) {
    if (h->d.lattice == 9) launch_step_q<9>(h, sens);
    else if (h->d.lattice == 19) launch_step_q<19>(h, sens);
    else launch_step_q<27>(h, sens);
}

template <typename T, typename C, bool SH>
void launch_multi(lbm_blocks *h, int m) {
    LaunchCfg c;
    c.stream = h->stream;
    c.tile_x = h->tile_x;
    c.scheme = kPingPong;
    c.sensor = false;
    c.sensor_kind = h->d.sensor_kind;
    c.force = h->has_force;
    c.smag = h->d.smagorinsky > 0.0;
    const StepArgs<C> a = step_args<9, C>(h, state_ptr(h), h->d.buf[h->cur ? LBM_BUF_F_A : LBM_BUF_F_B], false,
                                          h->tile_x);
    launch_multi_kernel<9, T, C, SH>(a, m, c);
}

// m (2 .. h->multi) sensor-free steps in one step_multi launch: the state
// moves to the other buffer once, whatever m.
void multi_once(lbm_blocks *h, int m) {
    switch (h->d.storage) {
        case LBM_F64: launch_multi<double, double, false>(h, m); break;
        case LBM_F32: launch_multi<float, float, false>(h, m); break;
        case LBM_F32_SHIFTED: launch_multi<float, float, true>(h, m); break;
        case LBM_F16_SHIFTED: launch_multi<_Float16, float, true>(h, m); break;
        default: launch_multi<__bf16, float, true>(h, m); break;   // LBM_BF16_SHIFTED
    }
    h->cur ^= 1;
    h->step += m;
}

void drop_graphs(lbm_blocks *h) {
    for (int p = 0; p < 2; ++p)
        if (h->graph[p]) {
            (void)hipGraphExecDestroy(h->graph[p]);
            h->graph[p] = nullptr;
        }
}

// One step with the usual bookkeeping (no graph).
void step_once(lbm_blocks *h, int32_t sensor_every) {
    const int64_t step = h->step + 1;
    const bool sens = sensor_every > 0 && step % sensor_every == 0;
    launch_step_any(h, sens);
    if (h->inplace) h->phase ^= 1;
    else h->cur ^= 1;
    h->step = step;
    if (sens) h->last_sensor_step = step;
    if (sens && h->averaging) ++h->avg_samples;
}

// c >= 2 sensor-free steps in an even number of step_multi launches (so that
// the state ends in the buffer it started in, as a captured graph needs) of
// at most h->multi steps each, as even as possible.
void multi_run(lbm_blocks *h, int64_t c) {
    int64_t nl = (c + h->multi - 1) / h->multi;
    if (nl % 2) ++nl;   // c even (graph chunks): nl <= c
    for (int64_t l = 0; l < nl; ++l) {
        const int64_t m = c / nl + (l < c % nl ? 1 : 0);
        if (m >= 2) multi_once(h, (int)m);
        else step_once(h, 0);
    }
}

// Captures graph_chunk sensor-free steps for the current buffer parity.
lbm_status capture_steps(lbm_blocks *h, int parity) {
    const int64_t s0 = h->step;
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    if (h->multi) multi_run(h, h->graph_chunk);
    else
        for (int k = 0; k < h->graph_chunk; ++k) step_once(h, 0);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(h->stream, &g));
    h->step = s0;   // captured, not run; an even chunk leaves the parity as it was
    hipError_t e = hipGraphInstantiate(&h->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        h->graph[parity] = nullptr;
        return fail(LBM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

lbm_status check_handle(lbm_blocks *h) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != h->device)
        return fail(LBM_EINVAL, "current device %d differs from the handle's device %d", dev, h->device);
    return LBM_OK;
}

lbm_status import_state(lbm_blocks *h, const double *f_host) {
    double *stage = scratch_d(h, h->L.staging_off);
    const int64_t cells = h->L.cells;
    lbm_status st = LBM_OK;
    reset_accumulators(h);
    with_types(h, [&]<int Q, typename T>() {
        Planes<T> p = planes_of<Q, T>(h, import_target(h));
        for (int i = 0; i < Q && st == LBM_OK; ++i) {
            hipError_t e = hipMemcpyAsync(stage, f_host + (int64_t)i * cells, cells * sizeof(double),
                                          hipMemcpyHostToDevice, h->stream);
            if (e != hipSuccess) { st = fail(LBM_EHIP, "hipMemcpyAsync: %s", hipGetErrorString(e)); break; }
            hipLaunchKernelGGL((import_plane_kernel<T>), dim3(grid_for(cells)), dim3(kAuxThreads), 0,
                               h->stream, stage, p.f + (int64_t)i * p.pitch, (int)cells, p.shift[i]);
            // the staging plane is reused by the next population: wait for the kernel
            e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) st = fail(LBM_EHIP, "import: %s", hipGetErrorString(e));
        }
    });
    if (st != LBM_OK) return st;
    finish_import(h);
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_required_bytes(const lbm_desc *d, size_t bytes[LBM_NBUF]) {
    Layout L;
    lbm_status st = check_desc(d, &L);
    if (st != LBM_OK) return st;
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    for (int b = 0; b < LBM_NBUF; ++b) bytes[b] = L.bytes[b];
    return LBM_OK;
}

lbm_status lbm_create_blocks(const lbm_desc *d, const double *f0_host, lbm_blocks **out) {
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    Layout L;
    lbm_status st = check_desc(d, &L);
    if (st != LBM_OK) return st;
    st = check_buffers(d, L);
    if (st != LBM_OK) return st;
    lbm_blocks *h = new (std::nothrow) lbm_blocks();
    if (!h) return fail(LBM_EINVAL, "out of host memory");
    h->d = *d;
    h->L = L;
    h->stream = static_cast<hipStream_t>(d->stream);
    h->inplace = inplace_setting(d, L);
    // 3D float64 has one tile shape (the z-march kernel, 64 x 8)
    h->tile_x = (L.dim == 3 && d->storage == LBM_F64) ? 64 : tile_x_setting(d->extent[0], h->inplace, L.dim);
    h->phase = 0;
    h->cur = 0;
    h->step = 0;
    h->last_sensor_step = -1;
    h->averaging = false;
    h->avg_started = false;
    h->avg_samples = 0;
    h->has_force = d->force[0] != 0.0 || d->force[1] != 0.0 || d->force[2] != 0.0;
    h->wall_mask = 0;
    h->graph_chunk = 0;
    h->multi = (!h->inplace && multi_setting(d, L)) ? kMultiMaxSteps : 0;
    h->graph[0] = h->graph[1] = nullptr;
    for (int f = 0; f < 6; ++f)
        if (d->face_bc[f] == LBM_BC_WALL) h->wall_mask |= 1u << f;
    h->flags_host.resize(L.nblocks);
    h->bmax_host.resize(L.nblocks * L.cbytes);
    hipError_t e = hipGetDevice(&h->device);
    if (e != hipSuccess) {
        delete h;
        return fail(LBM_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    }
    if (f0_host) {
        st = import_state(h, f0_host);
    } else {
        reset_accumulators(h);
        with_types(h, [&]<int Q, typename T>() {
            hipLaunchKernelGGL((init_rest_kernel<Q, T>), dim3(grid_for(L.cells)), dim3(kAuxThreads), 0,
                               h->stream, planes_of<Q, T>(h, import_target(h)), d->rho0);
        });
        finish_import(h);
        e = hipStreamSynchronize(h->stream);
        if (e == hipSuccess) e = hipGetLastError();
        if (e != hipSuccess) st = fail(LBM_EHIP, "initial state: %s", hipGetErrorString(e));
    }
    if (st != LBM_OK) {
        delete h;
        return st;
    }
    *out = h;
    return LBM_OK;
}

lbm_status lbm_step_n(lbm_blocks *h, int64_t n, int32_t sensor_every) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (n < 0) return fail(LBM_EINVAL, "n = %lld < 0", (long long)n);
    if (sensor_every < 0) return fail(LBM_EINVAL, "sensor_every = %d < 0", sensor_every);
    int64_t k = 0;
    while (k < n) {
        const int64_t c = h->graph_chunk;
        // a graph replay covers steps step+1 .. step+c when none of them is a sensor step
        const bool free = c > 0 && n - k >= c && !h->averaging &&
                          (sensor_every == 0 || (h->step + c) / sensor_every == h->step / sensor_every);
        if (free) {
            const int parity = h->inplace ? h->phase : h->cur;
            if (!h->graph[parity]) {
                st = capture_steps(h, parity);
                if (st != LBM_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(h->graph[parity], h->stream));
            h->step += c;
            k += c;
            continue;
        }
        if (h->multi && !h->averaging) {
            // the sensor-free steps before the next sensor step, in one launch
            int64_t r = n - k;
            if (sensor_every > 0) r = std::min(r, sensor_every - 1 - h->step % sensor_every);
            if (r >= 2) {
                const int m = (int)std::min<int64_t>(r, h->multi);
                multi_once(h, m);
                k += m;
                continue;
            }
        }
        step_once(h, sensor_every);
        ++k;
    }
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_use_graphs(lbm_blocks *h, int32_t chunk) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (chunk < 0 || chunk % 2) return fail(LBM_EINVAL, "chunk = %d must be an even number >= 0", chunk);
    if (chunk > 0 && !h->stream) return fail(LBM_ENOTSUP, "graphs need a non-NULL stream");
    if (chunk > 0 && (h->d.storage == LBM_F16_SHIFTED_SR || h->d.storage == LBM_BF16_SHIFTED_SR))
        return fail(LBM_ENOTSUP, "stochastic rounding keys on the step index: no graph replay");
    HIP_TRY(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    h->graph_chunk = chunk;
    return LBM_OK;
}

lbm_status lbm_sensor_flags(lbm_blocks *h, double *block_max_host, int8_t *flags_host,
                            int64_t *step_index) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (h->last_sensor_step < 0) return fail(LBM_ESTATE, "no sensor step has run since the state was set");
    const int64_t nb = h->L.nblocks;
    HIP_TRY(hipMemcpyAsync(h->bmax_host.data(), h->d.buf[LBM_BUF_BLOCK_MAX], nb * h->L.cbytes,
                           hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipMemcpyAsync(h->flags_host.data(), h->d.buf[LBM_BUF_FLAGS], nb, hipMemcpyDeviceToHost,
                           h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    bool nonfinite = false;
    for (int64_t b = 0; b < nb; ++b) {
        const double v = (h->L.cbytes == 8) ? reinterpret_cast<const double *>(h->bmax_host.data())[b]
                                            : reinterpret_cast<const float *>(h->bmax_host.data())[b];
        if (block_max_host) block_max_host[b] = v;
        if (flags_host) flags_host[b] = h->flags_host[b];
        if (h->flags_host[b] == LBM_FLAG_NONFINITE) nonfinite = true;
    }
    if (step_index) *step_index = h->last_sensor_step;
    if (nonfinite) return fail(LBM_ENONFINITE, "a sensor block holds a non-finite value");
    return LBM_OK;
}

lbm_status lbm_sensor_levels(lbm_blocks *h, double a, double b, int32_t lmin, int32_t lmax,
                             int32_t buffer, int8_t *levels_host) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (!levels_host) return fail(LBM_EINVAL, "levels_host is NULL");
    if (!is_fin(a) || !is_fin(b) || lmin > lmax || lmin < -127 || lmax > 127 || buffer < 0 || buffer > 8)
        return fail(LBM_EINVAL, "need finite a, b, -127 <= lmin <= lmax <= 127 and 0 <= buffer <= 8");
    if (h->last_sensor_step < 0) return fail(LBM_ESTATE, "no sensor step has run since the state was set");
    const int nb = (int)h->L.nblocks;
    int8_t *lev = reinterpret_cast<int8_t *>(static_cast<char *>(h->d.buf[LBM_BUF_SCRATCH]) + h->L.lev_off);
    const unsigned g = grid_for(nb);
    if (h->L.cbytes == 8)
        hipLaunchKernelGGL(levels_kernel<double>, dim3(g), dim3(kAuxThreads), 0, h->stream,
                           static_cast<const double *>(h->d.buf[LBM_BUF_BLOCK_MAX]), lev, nb, a, b, lmin, lmax);
    else
        hipLaunchKernelGGL(levels_kernel<float>, dim3(g), dim3(kAuxThreads), 0, h->stream,
                           static_cast<const float *>(h->d.buf[LBM_BUF_BLOCK_MAX]), lev, nb, a, b, lmin, lmax);
    hipLaunchKernelGGL(dilate_kernel, dim3(g), dim3(kAuxThreads), 0, h->stream, lev, lev + nb, h->L.nb[0],
                       h->L.nb[1], h->L.nb[2], buffer);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(levels_host, lev + nb, nb, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status lbm_sensor_average_begin(lbm_blocks *h) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    const size_t bytes = (size_t)h->L.cells * 8;
    char *p = static_cast<char *>(h->d.buf[LBM_BUF_SCRATCH]) + h->L.avg_off;
    // cleared with a kernel (no memset node if the caller captures the stream)
    hipLaunchKernelGGL(zero_words_kernel, dim3(grid_for((int64_t)(bytes / 8))), dim3(kAuxThreads), 0,
                       h->stream, reinterpret_cast<unsigned long long *>(p), (int)(bytes / 8));
    HIP_TRY(hipGetLastError());
    drop_graphs(h);   // the step kernels take the averaging pointer
    h->averaging = true;
    h->avg_started = true;
    h->avg_samples = 0;
    return LBM_OK;
}

lbm_status lbm_sensor_average(lbm_blocks *h, double *block_max_host, int64_t *samples) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (!h->avg_started) return fail(LBM_ESTATE, "averaging has not been started");
    if (samples) *samples = h->avg_samples;
    if (!block_max_host) return LBM_OK;
    if (h->avg_samples == 0) return fail(LBM_ESTATE, "no sensor step since averaging began");
    const int nb = (int)h->L.nblocks;
    const int bz = (h->L.dim == 3) ? kBlockEdge : 1;
    const char *scr = static_cast<const char *>(h->d.buf[LBM_BUF_SCRATCH]);
    double *out = reinterpret_cast<double *>(static_cast<char *>(h->d.buf[LBM_BUF_SCRATCH]) + h->L.avgmax_off);
    const double inv = 1.0 / (double)h->avg_samples;
    const lbm_desc &d = h->d;
    hipLaunchKernelGGL(average_block_max_kernel, dim3(grid_for(nb)), dim3(kAuxThreads), 0, h->stream,
                       reinterpret_cast<const double *>(scr + h->L.avg_off), out, d.extent[0], d.extent[1],
                       d.extent[2], kBlockEdge, kBlockEdge, bz, h->L.nb[0], h->L.nb[1], h->L.nb[2], inv);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(block_max_host, out, nb * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status lbm_sensor_average_end(lbm_blocks *h) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    h->averaging = false;
    return LBM_OK;
}

lbm_status lbm_get_macros(lbm_blocks *h, double *rho_host, double *u_host) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    const int64_t cells = h->L.cells;
    double *rho_d = scratch_d(h, h->L.staging_off);
    double *u_d = rho_d + cells;
    void *canon = canonical_state(h);
    with_types(h, [&]<int Q, typename T>() {
        hipLaunchKernelGGL((macros_kernel<Q, T>), dim3(grid_for(cells)), dim3(kAuxThreads), 0, h->stream,
                           planes_of<Q, T>(h, canon), rho_d, u_d, h->d.force[0], h->d.force[1],
                           h->d.force[2]);
    });
    HIP_TRY(hipGetLastError());
    if (rho_host) HIP_TRY(hipMemcpyAsync(rho_host, rho_d, cells * 8, hipMemcpyDeviceToHost, h->stream));
    if (u_host) HIP_TRY(hipMemcpyAsync(u_host, u_d, 3 * cells * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status lbm_block_means(lbm_blocks *h, double *means_host) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (!means_host) return fail(LBM_EINVAL, "means_host is NULL");
    const int64_t cells = h->L.cells;
    double *rho_d = scratch_d(h, h->L.staging_off);
    double *u_d = rho_d + cells;
    double *out = scratch_d(h, h->L.means_off);
    void *canon = canonical_state(h);
    with_types(h, [&]<int Q, typename T>() {
        hipLaunchKernelGGL((macros_kernel<Q, T>), dim3(grid_for(cells)), dim3(kAuxThreads), 0, h->stream,
                           planes_of<Q, T>(h, canon), rho_d, u_d, h->d.force[0], h->d.force[1],
                           h->d.force[2]);
    });
    const int bz = h->L.dim == 2 ? 1 : kBlockEdge;
    hipLaunchKernelGGL(block_means_kernel, dim3(grid_for(h->L.nblocks)), dim3(kAuxThreads), 0, h->stream, rho_d,
                       u_d, h->d.extent[0], h->d.extent[1], h->d.extent[2], h->L.nb[0], h->L.nb[1], h->L.nb[2], bz,
                       h->d.rho0, out);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(means_host, out, h->L.nblocks * 4 * 8, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status lbm_get_populations(lbm_blocks *h, double *f_host) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (!f_host) return fail(LBM_EINVAL, "f_host is NULL");
    const int64_t cells = h->L.cells;
    double *stage = scratch_d(h, h->L.staging_off);
    void *canon = canonical_state(h);
    with_types(h, [&]<int Q, typename T>() {
        Planes<T> p = planes_of<Q, T>(h, canon);
        for (int i = 0; i < Q && st == LBM_OK; ++i) {
            hipLaunchKernelGGL((export_plane_kernel<T>), dim3(grid_for(cells)), dim3(kAuxThreads), 0,
                               h->stream, p.f + (int64_t)i * p.pitch, stage, (int)cells, p.shift[i]);
            hipError_t e = hipMemcpyAsync(f_host + (int64_t)i * cells, stage, cells * 8,
                                          hipMemcpyDeviceToHost, h->stream);
            if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
            if (e != hipSuccess) st = fail(LBM_EHIP, "export: %s", hipGetErrorString(e));
        }
    });
    return st;
}

lbm_status lbm_set_populations(lbm_blocks *h, const double *f_host) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (!f_host) return fail(LBM_EINVAL, "f_host is NULL");
    st = import_state(h, f_host);
    if (st == LBM_OK) h->last_sensor_step = -1;
    return st;
}

lbm_status lbm_set_equilibrium(lbm_blocks *h, const double *rho_host, const double *u_host) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    const int64_t cells = h->L.cells;
    double *rho_d = scratch_d(h, h->L.staging_off);
    double *u_d = rho_d + cells;
    if (rho_host) HIP_TRY(hipMemcpyAsync(rho_d, rho_host, cells * 8, hipMemcpyHostToDevice, h->stream));
    if (u_host) {
        const int planes = h->L.dim;
        HIP_TRY(hipMemcpyAsync(u_d, u_host, planes * cells * 8, hipMemcpyHostToDevice, h->stream));
    }
    reset_accumulators(h);
    with_types(h, [&]<int Q, typename T>() {
        hipLaunchKernelGGL((equilibrium_kernel<Q, T>), dim3(grid_for(cells)), dim3(kAuxThreads), 0,
                           h->stream, planes_of<Q, T>(h, import_target(h)), rho_host ? rho_d : nullptr,
                           u_host ? u_d : nullptr, h->d.rho0);
    });
    finish_import(h);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(h->stream));
    h->last_sensor_step = -1;
    return LBM_OK;
}

lbm_status lbm_get_scheme(lbm_blocks *h, int32_t *inplace, int32_t *next_is_gather, int32_t *tile_x) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (inplace) *inplace = h->inplace ? 1 : 0;
    if (next_is_gather) *next_is_gather = (h->inplace && h->phase == 0) ? 1 : 0;
    if (tile_x) *tile_x = h->tile_x;
    return LBM_OK;
}

lbm_status lbm_set_multistep(lbm_blocks *h, int32_t steps) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (steps != 0 && (steps < 2 || steps > kMultiMaxSteps))
        return fail(LBM_EINVAL, "steps = %d: 0 (off) or 2 .. %d", steps, kMultiMaxSteps);
    if (steps > 0 && (h->inplace || !multi_setting(&h->d, h->L)))
        return fail(LBM_ENOTSUP, "several steps per launch need a ping-pong D2Q9 handle of at most %lld cells "
                                 "without stochastic rounding", (long long)kMultiMaxCells);
    HIP_TRY(hipStreamSynchronize(h->stream));
    drop_graphs(h);   // captured with the old setting
    h->multi = steps;
    return LBM_OK;
}

lbm_status lbm_get_multistep(lbm_blocks *h, int32_t *steps) {
    if (!h || !steps) return fail(LBM_EINVAL, "NULL argument");
    *steps = h->multi;
    return LBM_OK;
}

lbm_status lbm_get_step(lbm_blocks *h, int64_t *step) {
    if (!h || !step) return fail(LBM_EINVAL, "NULL argument");
    *step = h->step;
    return LBM_OK;
}

lbm_status lbm_set_step(lbm_blocks *h, int64_t step) {
    if (!h) return fail(LBM_EINVAL, "handle is NULL");
    if (step < 0) return fail(LBM_EINVAL, "step = %lld < 0", (long long)step);
    h->step = step;
    h->last_sensor_step = -1;
    return LBM_OK;
}

lbm_status lbm_conservation(lbm_blocks *h, double out[4]) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    const int64_t cells = h->L.cells;
    double *partial = scratch_d(h, h->L.partial_off);
    double *res = scratch_d(h, h->L.out_off);
    const int nwg = (int)std::min<int64_t>(kMaxPartials, (cells + kReduceThreads - 1) / kReduceThreads);
    void *canon = canonical_state(h);
    with_types(h, [&]<int Q, typename T>() {
        hipLaunchKernelGGL((conservation_pass1<Q, T>), dim3(nwg), dim3(kReduceThreads), 0, h->stream,
                           planes_of<Q, T>(h, canon), partial);
    });
    hipLaunchKernelGGL(conservation_pass2, dim3(1), dim3(kReduceThreads), 0, h->stream, partial, nwg, res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

}  // extern "C"

// Workspace of lbm_conservation_noalloc, owned by the library: the first
// pass's partial sums (4 doubles for each of at most kMaxPartials
// workgroups) and the 4 totals, 32 KiB.  Each GPU the library runs on holds
// its own copy until the process ends.  In host code `scratch` names a host
// stand-in, not device memory: only the address from hipGetSymbolAddress,
// kept per device in g_scratch_dev, is passed to kernels and copies.
static __device__ __align__(256) double scratch[kMaxPartials * 4 + 4];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), looked up
// once per device.
lbm_status noalloc_scratch(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return fail(LBM_ENOTSUP, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LBM_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
        g_scratch_dev[device] = static_cast<double *>(p);
    }
    *out = g_scratch_dev[device];
    return LBM_OK;
}

}  // namespace

extern "C" {

lbm_status lbm_conservation_noalloc(lbm_blocks *h, double out[4]) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    const int64_t cells = h->L.cells;
    // the first pass caps its workgroups at kMaxPartials (each then sums
    // more cells), so every grid a handle accepts fits the workspace
    const int nwg = (int)std::min<int64_t>(kMaxPartials, (cells + kReduceThreads - 1) / kReduceThreads);
    double *ws = nullptr;
    st = noalloc_scratch(h->device, &ws);
    if (st != LBM_OK) return st;
    double *partial = ws;
    double *res = ws + (size_t)kMaxPartials * 4;
    // The same kernels, workgroup count and summation order as
    // lbm_conservation, so the totals are the same bits.  Every partial the
    // second pass reads is written by the first, so nothing needs clearing.
    void *canon = canonical_state(h);
    with_types(h, [&]<int Q, typename T>() {
        hipLaunchKernelGGL((conservation_pass1<Q, T>), dim3(nwg), dim3(kReduceThreads), 0, h->stream,
                           planes_of<Q, T>(h, canon), partial);
    });
    hipLaunchKernelGGL(conservation_pass2, dim3(1), dim3(kReduceThreads), 0, h->stream, partial, nwg, res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out, res, 4 * sizeof(double), hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    return LBM_OK;
}

lbm_status lbm_autotune(lbm_blocks *h, int32_t reps, int32_t *tile_x) {
    lbm_status st = check_handle(h);
    if (st != LBM_OK) return st;
    if (reps < 1) return fail(LBM_EINVAL, "reps = %d < 1", reps);
    const bool zm = h->d.lattice != LBM_D2Q9 && h->d.storage == LBM_F64;
    if (zm) {   // the z-march kernel has one tile shape
        if (tile_x) *tile_x = 64;
        return LBM_OK;
    }
    // Timed launches must leave the state alone.  Ping-pong: they read the
    // state and write the other buffer.  In place: they run on a copy of F_A
    // in F_B (the staging buffer), with the two buffers exchanged meanwhile.
    const size_t bytes = (size_t)h->L.q * h->L.pitch * h->L.elem;
    if (h->inplace) {
        HIP_TRY(hipMemcpyAsync(h->d.buf[LBM_BUF_F_B], h->d.buf[LBM_BUF_F_A], bytes, hipMemcpyDeviceToDevice,
                               h->stream));
        std::swap(h->d.buf[LBM_BUF_F_A], h->d.buf[LBM_BUF_F_B]);
    }
    const int saved_tile = h->tile_x, saved_phase = h->phase;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    float best = 1e30f;
    int best_tile = saved_tile;
    hipError_t e = hipSuccess;
    const bool rows_ok = !h->inplace && h->L.dim == 3;
    for (int tx : {32, 64, 128, kRowTileX}) {
        if (tx == kRowTileX && !rows_ok) continue;
        h->tile_x = tx;
        auto one = [&]() {
            launch_step_any(h, false);
            if (h->inplace) h->phase ^= 1;
        };
        one();
        one();   // warm-up (both halves of the in-place pair)
        e = hipEventRecord(e0, h->stream);
        for (int r = 0; r < 2 * reps && e == hipSuccess; ++r) one();
        if (e == hipSuccess) e = hipEventRecord(e1, h->stream);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) break;
        if (ms < best) {
            best = ms;
            best_tile = tx;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (h->inplace) std::swap(h->d.buf[LBM_BUF_F_A], h->d.buf[LBM_BUF_F_B]);
    h->phase = saved_phase;
    h->tile_x = (e == hipSuccess) ? best_tile : saved_tile;
    if (h->tile_x != saved_tile) drop_graphs(h);   // captured with the old tiling
    if (e != hipSuccess) return fail(LBM_EHIP, "autotune: %s", hipGetErrorString(e));
    if (tile_x) *tile_x = h->tile_x;
    return LBM_OK;
}

lbm_status lbm_tau_from_reynolds(double u, double n_across, double re, double *tau) {
    if (!tau) return fail(LBM_EINVAL, "tau is NULL");
    if (!is_fin(u) || !is_fin(n_across) || !is_fin(re) || !(re > 0.0) || !(n_across > 0.0))
        return fail(LBM_EINVAL, "need finite u, n_across > 0 and re > 0");
    const double cs2 = 1.0 / 3.0;
    const double nu = std::fabs(u) * n_across / re;
    *tau = nu / cs2 + 0.5;
    return LBM_OK;
}

void lbm_destroy(lbm_blocks *h) {
    if (!h) return;
    (void)hipStreamSynchronize(h->stream);
    drop_graphs(h);
    delete h;
}

const char *lbm_last_error(void) { return g_error.c_str(); }

}  // extern "C"

// The two-level patch hierarchy (lbm_create_hierarchy and friends).
#include "hierarchy_host.hpp"
