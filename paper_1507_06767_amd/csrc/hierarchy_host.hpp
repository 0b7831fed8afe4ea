// hierarchy_host.hpp -- host side of the two-level patch hierarchy
// (include/lbm.h, lbm_create_hierarchy and friends).  Part of the lbm.hip
// translation unit: it uses that file's handle internals and helpers.
//
// One coarse step of the hierarchy (coarse state X -> Y, fine A -> B -> A):
//   1. ghost layers of the fine state A from X (and from abutting patches);
//   2. fine step A -> B;
//   3. coarse step X -> Y (every coarse cell, the step kernel of the handle);
//   4. ghost layers of B from (X + Y) / 2 (linear time interpolation);
//   5. fine step B -> A (with the fine sensor on sensor steps);
//   6. restriction: covered coarse cells of Y from the fine state A.
// Steps 1-6 of two consecutive coarse steps are captured once into a HIP
// graph per coarse parity and replayed (the kernels' arguments repeat every
// two coarse steps).  The fine step walks a tile list, the ghost fill a
// ghost list and the separate restriction kernel (a comparison path; the
// second fine step restricts by default) a list of covered coarse cells, all
// built here on the host at creation.

#include <array>
#include <string>

#include "patch_kernels.hpp"

struct lbm_hierarchy {
    lbm_blocks *coarse;
    int q;
    int npatch;
    std::vector<lbm_box> boxes;
    std::vector<PatchRec> rec;
    int64_t total_padded, covered, nblocks, fine_cells, max_patch_cells;
    int64_t pitch;            // elements between fine planes
    int64_t xg_pitch;         // elements between the x-face ghost planes (after the q fine planes)
    size_t elem;              // bytes per stored value
    size_t meta_patch, meta_tile, meta_cover, meta_gdst, meta_gsrc, meta_gloc, meta_gmask, meta_gtile, meta_rc,
        meta_rf, meta_rp,
        meta_stage;           // offsets inside META
    int64_t nghost, ntiles;   // ghost cells; tiles of the current tile list
    int64_t ngtile, ngtile_max;   // ghost tiles in use (0: list-only ghost kernel); their bound
    std::vector<PatchTile> tiles;
    size_t bytes[LBM_NHBUF];
    void *buf[LBM_NHBUF];
    int cur;                  // fine state in F_A (0) or F_B (1)
    double tau_f, alpha;
    int wmax, nwg;            // widest fine tile (8, 16, 32; kBandMaxW: bands) and persistent workgroups
    int nwg_restrict;         // persistent workgroups of the restricting fine step
    bool use_graph;
    hipGraphExec_t graph[2];  // two coarse steps, by the coarse buffer parity
    int64_t step;             // coarse steps taken through the hierarchy
    int64_t last_sensor_step;
    std::vector<unsigned char> bmax_host;
};

namespace {

constexpr int kHierCUs = 256;

// Layout of the hierarchy for a coarse handle and boxes; validates both.
lbm_status hier_layout(const lbm_blocks *h, int32_t nbox, const lbm_box *boxes, lbm_hierarchy *H) {
    if (!h) return fail(LBM_EINVAL, "coarse handle is NULL");
    if (nbox < 1 || !boxes) return fail(LBM_EINVAL, "need at least one box");
    const lbm_desc &d = h->d;
    if (d.lattice == LBM_D2Q9) return fail(LBM_ENOTSUP, "the hierarchy is 3D (D3Q19 or D3Q27)");
    if (d.storage < LBM_F64 || d.storage > LBM_BF16_SHIFTED_SR)
        return fail(LBM_ENOTSUP, "storage %d", d.storage);
    if (h->inplace) return fail(LBM_ENOTSUP, "the coarse handle must stream ping-pong (LBM_STREAMING_PINGPONG)");
    if (h->has_force || d.smagorinsky > 0.0)
        return fail(LBM_ENOTSUP, "the hierarchy couples plain BGK without body force");
    const double tau_c = d.tau, tau_f = 2.0 * tau_c - 0.5;
    if (std::fabs(tau_c - 1.0) < 0.05 || std::fabs(tau_f - 1.0) < 0.05)
        return fail(LBM_ENOTSUP, "tau = %g: the non-equilibrium rescaling needs tau and 2 tau - 1/2 away from 1",
                    tau_c);
    const int n[3] = {d.extent[0], d.extent[1], d.extent[2]};
    std::vector<int> cover((size_t)h->L.cells, -1);
    H->q = d.lattice;
    H->npatch = nbox;
    H->boxes.assign(boxes, boxes + nbox);
    H->rec.assign(nbox, PatchRec{});
    int64_t padded = 0, blocks = 0, cov = 0, maxc = 0, xg = 0;
    for (int p = 0; p < nbox; ++p) {
        const lbm_box &b = boxes[p];
        PatchRec &r = H->rec[p];
        for (int a = 0; a < 3; ++a) {
            if (b.lo[a] < 1 || b.hi[a] > n[a] - 1 || b.hi[a] <= b.lo[a])
                return fail(LBM_EINVAL, "box %d axis %d: need 1 <= lo < hi <= n - 1 (coarse cells)", p, a);
            if ((b.hi[a] - b.lo[a]) % 4)
                return fail(LBM_EINVAL, "box %d axis %d: extent %d is not a multiple of 4 coarse cells", p, a,
                            b.hi[a] - b.lo[a]);
            r.o[a] = 2 * b.lo[a];
            r.e[a] = 2 * (b.hi[a] - b.lo[a]);
        }
        for (int z = b.lo[2]; z < b.hi[2]; ++z)
            for (int y = b.lo[1]; y < b.hi[1]; ++y)
                for (int x = b.lo[0]; x < b.hi[0]; ++x) {
                    int &c = cover[((size_t)z * n[1] + y) * n[0] + x];
                    if (c >= 0) return fail(LBM_EINVAL, "boxes %d and %d overlap", c, p);
                    c = p;
                }
        r.off = (int)padded;
        r.blk0 = (int)blocks;
        r.coff = (int)cov;
        r.xoff = (int)xg;                         // the patch's two x-face ghost arrays
        xg += 2 * (int64_t)(r.e[1] + 2) * (r.e[2] + 2);
        const int64_t pc = (int64_t)(r.e[0] + 2) * (r.e[1] + 2) * (r.e[2] + 2);
        const int64_t cells = (int64_t)r.e[0] * r.e[1] * r.e[2];
        padded += pc;
        blocks += cells / 512;
        cov += cells / 8;
        maxc = std::max(maxc, cells);
    }
    // the ghost list packs a padded index and three interpolation bits in 32 bits
    if (padded >= (int64_t(1) << 29) || xg >= (int64_t(1) << 29))
        return fail(LBM_ENOTSUP, "patches hold more than 2^29 padded cells");
    H->total_padded = padded;
    H->nblocks = blocks;
    H->covered = cov;
    H->fine_cells = 8 * cov;
    H->max_patch_cells = maxc;
    H->elem = h->L.elem;
    H->pitch = (int64_t)round_up((size_t)padded, 64) + 64;
    H->xg_pitch = (int64_t)round_up((size_t)xg, 64) + 64;
    H->tau_f = tau_f;
    H->alpha = (tau_f - 1.0) / (2.0 * (tau_c - 1.0));
    H->bytes[LBM_HBUF_F_A] = H->bytes[LBM_HBUF_F_B] =
        round_up((size_t)H->q * (H->pitch + H->xg_pitch) * H->elem, kAlign);
    H->bytes[LBM_HBUF_BLOCK_MAX] = round_up((size_t)blocks * h->L.cbytes, kAlign);
    H->bytes[LBM_HBUF_FLAGS] = round_up((size_t)blocks, kAlign);
    H->nghost = padded - 8 * cov;
    H->meta_patch = 0;
    H->meta_tile = round_up((size_t)nbox * sizeof(PatchRec), kAlign);
    H->meta_cover = H->meta_tile + round_up((size_t)blocks * sizeof(PatchTile), kAlign);   // <= one tile per block
    H->meta_gdst = H->meta_cover + round_up((size_t)h->L.cells * 4, kAlign);
    H->meta_gsrc = H->meta_gdst + round_up((size_t)H->nghost * 4, kAlign);
    // ghost tiles: 16 x 16 pieces of the six faces of every patch
    int64_t ngt = 0;
    for (int p = 0; p < nbox; ++p) {
        const PatchRec &r = H->rec[p];
        const int64_t P0 = r.e[0] + 2, P1 = r.e[1] + 2, P2 = r.e[2] + 2;
        auto t16 = [](int64_t m) { return (m + 15) / 16; };
        ngt += 2 * (t16(P1) * t16(P2) + t16(P0 - 2) * t16(P2) + t16(P0 - 2) * t16(P1 - 2));
    }
    H->ngtile_max = ngt;
    H->meta_gloc = H->meta_gsrc + round_up((size_t)H->nghost * 4, kAlign);
    H->meta_gmask = H->meta_gloc + round_up((size_t)H->nghost * 4, kAlign);
    H->meta_gtile = H->meta_gmask + round_up((size_t)H->nghost * 4, kAlign);
    H->meta_rc = H->meta_gtile + round_up((size_t)ngt * sizeof(GhostTile), kAlign);
    H->meta_rf = H->meta_rc + round_up((size_t)cov * 4, kAlign);
    H->meta_rp = H->meta_rf + round_up((size_t)cov * 4, kAlign);
    H->meta_stage = H->meta_rp + round_up((size_t)cov * 4, kAlign);
    H->bytes[LBM_HBUF_META] = H->meta_stage + round_up((size_t)maxc * (H->q + 4) * 8, kAlign);
    H->bmax_host.assign((size_t)blocks * h->L.cbytes, 0);
    return LBM_OK;
}

// fine_step: index of the fine step the launch belongs to (the stochastic
// rounding key of its stores)
template <typename C>
PatchArgs<C> patch_args(lbm_hierarchy *H, const void *src, void *dst, int64_t fine_step = 0) {
    const lbm_desc &d = H->coarse->d;
    PatchArgs<C> a{};
    a.src = src;
    a.dst = dst;
    a.pitch = H->pitch;
    a.xg_base = (int64_t)H->q * H->pitch;
    a.xg_pitch = H->xg_pitch;
    char *meta = static_cast<char *>(H->buf[LBM_HBUF_META]);
    a.patch = reinterpret_cast<const PatchRec *>(meta + H->meta_patch);
    a.tile = reinterpret_cast<const PatchTile *>(meta + H->meta_tile);
    a.npatch = H->npatch;
    a.ntiles = (int)H->ntiles;
    for (int i = 0; i < kMaxQ; ++i) a.shift[i] = C(0);
    auto fill_shift = [&]<int Q>() {
        static_for<0, Q>([&](auto ic) {
            constexpr int i = decltype(ic)::value;
            a.shift[i] = (C)(Vel<Q, i>::w * d.rho0);
        });
    };
    if (H->q == 19) fill_shift.template operator()<19>();
    else fill_shift.template operator()<27>();
    a.rho0 = (C)d.rho0;
    a.omega = (C)(1.0 / H->tau_f);
    a.theta_r = d.theta_refine;
    a.theta_c = d.theta_coarsen;
    a.block_max = static_cast<C *>(H->buf[LBM_HBUF_BLOCK_MAX]);
    a.flags = static_cast<int8_t *>(H->buf[LBM_HBUF_FLAGS]);
    a.step = (uint32_t)fine_step;
    return a;
}

template <typename C>
CoarseView<C> coarse_view(lbm_hierarchy *H, const void *s0, const void *s1, double w1, void *out) {
    const lbm_blocks *h = H->coarse;
    CoarseView<C> v{};
    v.s0 = s0;
    v.s1 = s1;
    v.out = out;
    v.pitch = h->L.pitch;
    v.nx = h->d.extent[0];
    v.ny = h->d.extent[1];
    v.nz = h->d.extent[2];
    v.cover = reinterpret_cast<const int *>(static_cast<char *>(H->buf[LBM_HBUF_META]) + H->meta_cover);
    v.w1 = (C)w1;
    v.alpha = (C)H->alpha;
    return v;
}

// Calls f.template operator()<Q, T, C, SH>() for the hierarchy's types.
template <typename F>
void with_hier_types(lbm_hierarchy *H, F &&f) {
    const int s = H->coarse->d.storage;
    auto by_q = [&]<int Q>() {
        switch (s) {
            case LBM_F64: f.template operator()<Q, double, double, false>(); break;
            case LBM_F32: f.template operator()<Q, float, float, false>(); break;
            case LBM_F16_SHIFTED: f.template operator()<Q, _Float16, float, true>(); break;
            case LBM_BF16_SHIFTED: f.template operator()<Q, __bf16, float, true>(); break;
            case LBM_F16_SHIFTED_SR: f.template operator()<Q, half_sr, float, true>(); break;
            case LBM_BF16_SHIFTED_SR: f.template operator()<Q, bf16_sr, float, true>(); break;
            default: f.template operator()<Q, float, float, true>(); break;
        }
    };
    if (H->q == 19) by_q.template operator()<19>();
    else by_q.template operator()<27>();
}

void *fine_buf(lbm_hierarchy *H, int which) { return H->buf[which ? LBM_HBUF_F_B : LBM_HBUF_F_A]; }

PatchLists patch_lists(lbm_hierarchy *H) {
    char *meta = static_cast<char *>(H->buf[LBM_HBUF_META]);
    PatchLists L;
    L.gdst = reinterpret_cast<const uint32_t *>(meta + H->meta_gdst);
    L.gsrc = reinterpret_cast<const int *>(meta + H->meta_gsrc);
    L.gloc = reinterpret_cast<const int *>(meta + H->meta_gloc);
    L.gmask = reinterpret_cast<const uint32_t *>(meta + H->meta_gmask);
    L.nghost = H->nghost;
    L.gtile = H->ngtile > 0 ? reinterpret_cast<const GhostTile *>(meta + H->meta_gtile) : nullptr;
    L.ngtile = H->ngtile;
    L.rc = reinterpret_cast<const int *>(meta + H->meta_rc);
    L.rf = reinterpret_cast<const int *>(meta + H->meta_rf);
    L.rp = reinterpret_cast<const int *>(meta + H->meta_rp);
    L.covered = H->covered;
    return L;
}

// Tiles of the fine step: per patch, rows of 8 x 8 x 8 blocks cut along x
// into the widest of 32, 16, 8 cells (at most wmax) that still fit (the
// W x 8 x 8 tiles of patch_step), or for wmax = kBandMaxW into bands of
// patch_band_step: the whole row when it is at most 48 cells wide, else
// pieces of 48 cells and the rest (a multiple of 8).  Bands address a state
// buffer with 32-bit byte offsets: above 4 GiB the tiles of 32 take over.
void build_tiles(lbm_hierarchy *H, int wmax) {
    if (wmax == kBandMaxW && H->bytes[LBM_HBUF_F_A] > (size_t(1) << 32)) wmax = 32;
    H->tiles.clear();
    for (int p = 0; p < H->npatch; ++p) {
        const PatchRec &r = H->rec[p];
        const int nbx = r.e[0] / 8, nby = r.e[1] / 8;
        for (int bz = 0; bz < r.e[2] / 8; ++bz)
            for (int by = 0; by < nby; ++by)
                for (int x0 = 0; x0 < r.e[0];) {
                    const int left = r.e[0] - x0;
                    int w;
                    if (wmax == kBandMaxW) w = std::min(left, kBandMaxW);
                    else w = (wmax >= 32 && left >= 32) ? 32 : ((wmax >= 16 && left >= 16) ? 16 : 8);
                    PatchTile t{};
                    t.patch = p;
                    t.x0 = x0;
                    t.y0 = 8 * by;
                    t.z0 = 8 * bz;
                    t.w = w;
                    t.blk = r.blk0 + (bz * nby + by) * nbx + x0 / 8;
                    H->tiles.push_back(t);
                    x0 += w;
                }
    }
    H->ntiles = (int64_t)H->tiles.size();
    H->wmax = wmax;
}

hipError_t upload_tiles(lbm_hierarchy *H) {
    char *meta = static_cast<char *>(H->buf[LBM_HBUF_META]);
    return hipMemcpyAsync(meta + H->meta_tile, H->tiles.data(), H->tiles.size() * sizeof(PatchTile),
                          hipMemcpyHostToDevice, H->coarse->stream);
}

// A fine step over all patches; with `restrict_out` (the coarse state being
// completed) it also restricts every covered coarse cell to it.
void hier_fine_step(lbm_hierarchy *H, const void *src, void *dst, bool sensor, int64_t fine_step,
                    void *restrict_out = nullptr) {
    with_hier_types(H, [&]<int Q, typename T, typename C, bool SH>() {
        PatchLaunch l{H->coarse->stream, sensor, H->coarse->d.sensor_kind, restrict_out != nullptr,
                      restrict_out ? H->nwg_restrict : H->nwg, H->wmax == kBandMaxW};
        launch_patch_step<Q, T, C, SH>(patch_args<C>(H, src, dst, fine_step),
                                       coarse_view<C>(H, restrict_out, restrict_out, 0.0, restrict_out), l);
    });
}

// The fine step's default tiling: bands (patch_band_step); LBM_HIER_TILES=8,
// 16 or 32 selects W x 8 x 8 tiles of patch_step (for comparison).
int fine_tiling_setting() {
    const char *s = std::getenv("LBM_HIER_TILES");
    if (s) {
        const int v = std::atoi(s);
        if (v == 8 || v == 16 || v == 32) return v;
    }
    return kBandMaxW;
}

// The restriction runs inside the second fine step unless LBM_HIER_RESTRICT
// is "separate" (its own kernel over the precomputed list; for comparison).
bool restriction_fused() {
    const char *s = std::getenv("LBM_HIER_RESTRICT");
    return !(s && std::string(s) == "separate");
}

void hier_ghosts(lbm_hierarchy *H, void *state, const void *s0, const void *s1, double w1, int64_t fine_step) {
    with_hier_types(H, [&]<int Q, typename T, typename C, bool SH>() {
        launch_patch_ghosts<Q, T, C, SH>(patch_args<C>(H, state, state, fine_step),
                                         coarse_view<C>(H, s0, s1, w1, nullptr),
                                         state, patch_lists(H), H->coarse->stream);
    });
}

// One coarse step (steps 1-6 above; step 6 inside step 5 by default)
// enqueued on the coarse handle's stream.
// With `ev` (7 events), the events are recorded before, between and after
// the six launches, for lbm_hierarchy_profile.
void hier_coarse_step(lbm_hierarchy *H, bool sens, hipEvent_t *ev = nullptr) {
    lbm_blocks *h = H->coarse;
    auto mark = [&](int i) {
        if (ev) (void)hipEventRecord(ev[i], h->stream);
    };
    void *X = state_ptr(h);
    void *Y = h->d.buf[h->cur ? LBM_BUF_F_A : LBM_BUF_F_B];
    void *A = fine_buf(H, H->cur), *B = fine_buf(H, H->cur ^ 1);
    const int64_t f1 = 2 * H->step + 1, f2 = f1 + 1;   // fine steps of this coarse step
    mark(0);
    hier_ghosts(H, A, X, X, 0.0, f1);
    mark(1);
    hier_fine_step(H, A, B, false, f1);
    mark(2);
    const int64_t step = h->step + 1;
    launch_step_any(h, sens);
    mark(3);
    h->cur ^= 1;
    h->step = step;
    if (sens) h->last_sensor_step = step;
    hier_ghosts(H, B, X, Y, 0.5, f2);
    mark(4);
    const bool fused = restriction_fused();
    hier_fine_step(H, B, A, sens, f2, fused ? Y : nullptr);
    mark(5);
    if (!fused)
        with_hier_types(H, [&]<int Q, typename T, typename C, bool SH>() {
            launch_patch_restrict<Q, T, C, SH>(patch_args<C>(H, A, A, f2), coarse_view<C>(H, Y, Y, 0.0, Y), A,
                                               patch_lists(H), h->stream);
        });
    mark(6);
    H->step += 1;
    if (sens) H->last_sensor_step = H->step;
}

lbm_status hier_capture(lbm_hierarchy *H, int parity) {
    lbm_blocks *h = H->coarse;
    const int64_t s0 = h->step, s1 = h->last_sensor_step, s2 = H->step, s3 = H->last_sensor_step;
    HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
    hier_coarse_step(H, false);
    hier_coarse_step(H, false);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamEndCapture(h->stream, &g));
    h->step = s0;
    h->last_sensor_step = s1;
    H->step = s2;
    H->last_sensor_step = s3;
    hipError_t e = hipGraphInstantiate(&H->graph[parity], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        H->graph[parity] = nullptr;
        return fail(LBM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    }
    return LBM_OK;
}

lbm_status hier_check(lbm_hierarchy *H) {
    if (!H) return fail(LBM_EINVAL, "hierarchy is NULL");
    return check_handle(H->coarse);
}

}  // namespace

extern "C" {

lbm_status lbm_hierarchy_required_bytes(const lbm_blocks *coarse, int32_t nbox, const lbm_box *boxes,
                                        size_t bytes[LBM_NHBUF]) {
    if (!bytes) return fail(LBM_EINVAL, "bytes is NULL");
    lbm_hierarchy H;
    lbm_status st = hier_layout(coarse, nbox, boxes, &H);
    if (st != LBM_OK) return st;
    for (int b = 0; b < LBM_NHBUF; ++b) bytes[b] = H.bytes[b];
    return LBM_OK;
}

lbm_status lbm_create_hierarchy(lbm_blocks *coarse, int32_t nbox, const lbm_box *boxes, void *const buf[LBM_NHBUF],
                                const size_t buf_bytes[LBM_NHBUF], int32_t use_graph, lbm_hierarchy **out) {
    if (!out || !buf || !buf_bytes) return fail(LBM_EINVAL, "out, buf and buf_bytes must not be NULL");
    lbm_status st = check_handle(coarse);
    if (st != LBM_OK) return st;
    lbm_hierarchy *H = new (std::nothrow) lbm_hierarchy();
    if (!H) return fail(LBM_EINVAL, "out of host memory");
    st = hier_layout(coarse, nbox, boxes, H);
    if (st != LBM_OK) {
        delete H;
        return st;
    }
    static const char *names[LBM_NHBUF] = {"F_A", "F_B", "BLOCK_MAX", "FLAGS", "META"};
    for (int b = 0; b < LBM_NHBUF; ++b) {
        if (!buf[b] || buf_bytes[b] < H->bytes[b] || (uintptr_t)buf[b] % kAlign) {
            delete H;
            return fail(LBM_EINVAL, "hierarchy buffer %s: NULL, smaller than %zu bytes or not 256-byte aligned",
                        names[b], H->bytes[b]);
        }
        H->buf[b] = buf[b];
    }
    H->coarse = coarse;
    H->cur = 0;
    build_tiles(H, fine_tiling_setting());
    H->nwg = (int)std::min<int64_t>(H->ntiles, 8 * kHierCUs);
    // the restricting step's LDS sums leave room for one or two workgroups per CU
    H->nwg_restrict = (int)std::min<int64_t>(H->ntiles, kHierCUs);
    const bool sr = coarse->d.storage == LBM_F16_SHIFTED_SR || coarse->d.storage == LBM_BF16_SHIFTED_SR;
    if (use_graph != 0 && sr) {
        delete H;
        return fail(LBM_ENOTSUP, "stochastic rounding keys on the step index: no graph replay");
    }
    H->use_graph = use_graph != 0 && coarse->stream != nullptr;
    H->graph[0] = H->graph[1] = nullptr;
    H->step = 0;
    H->last_sensor_step = -1;
    // coarse cover map
    const int nx = coarse->d.extent[0], ny = coarse->d.extent[1];
    std::vector<int> cover((size_t)coarse->L.cells, -1);
    for (int p = 0; p < H->npatch; ++p) {
        const lbm_box &b = H->boxes[p];
        for (int z = b.lo[2]; z < b.hi[2]; ++z)
            for (int y = b.lo[1]; y < b.hi[1]; ++y)
                for (int x = b.lo[0]; x < b.hi[0]; ++x) cover[((size_t)z * ny + y) * nx + x] = p;
    }
    // ghost list, grouped into tiles of at most 16 x 16 cells of one face: a
    // ghost copies from the patch that holds its cell, else it carries the low
    // corner of its coarse interpolation stencil and the 3/4-weight bits.
    // Faces own their cells without overlap: x faces whole, y faces without
    // the x rims, z faces without the x and y rims.  The two faces normal to
    // an axis alternate piece by piece: the pieces of the low and the high x
    // face at the same (y, z) read the same coarse rows (two cells at each
    // end), and as neighbours in the list they run side by side on one XCD.
    std::vector<uint32_t> gdst;
    std::vector<int> gsrc;
    std::vector<GhostTile> gtiles;
    std::vector<int> gloc;
    std::vector<uint32_t> gmask;
    gloc.reserve(H->nghost);
    gmask.reserve(H->nghost);
    // velocity table of the lattice (interface order)
    const int(*vel)[3] = (H->q == 19) ? Lattice<19>::c : Lattice<27>::c;
    gdst.reserve(H->nghost);
    gsrc.reserve(H->nghost);
    bool tiles_ok = true;
    for (int p = 0; p < H->npatch; ++p) {
        const PatchRec &r = H->rec[p];
        const int P[3] = {r.e[0] + 2, r.e[1] + 2, r.e[2] + 2};
        for (int na = 0; na < 3; ++na) {
            const int ua = (na == 0) ? 1 : 0, va = (na == 2) ? 1 : 2;
            const int ulo = (na == 0) ? 0 : 1, uhi = (na == 0) ? P[1] : P[0] - 1;
            const int vlo = (na == 2) ? 1 : 0, vhi = (na == 2) ? P[1] - 1 : P[2];
            for (int v0 = vlo; v0 < vhi; v0 += 16)
                for (int u0 = ulo; u0 < uhi; u0 += 16)
                    for (int f = 2 * na; f < 2 * na + 2; ++f) {   // the low face's piece, then the high face's
                        const int pn = (f & 1) ? P[na] - 1 : 0;
                        GhostTile t{};
                        t.k0 = (int)gdst.size();
                        std::vector<std::array<int, 3>> corner;   // stencil corner of each entry (-1: copy)
                        int bmin[3] = {1 << 30, 1 << 30, 1 << 30}, bmax[3] = {-1, -1, -1};
                        for (int vv = v0; vv < std::min(v0 + 16, vhi); ++vv)
                            for (int uu = u0; uu < std::min(u0 + 16, uhi); ++uu) {
                                int pc[3];
                                pc[na] = pn;
                                pc[ua] = uu;
                                pc[va] = vv;
                                const int g[3] = {r.o[0] + pc[0] - 1, r.o[1] + pc[1] - 1, r.o[2] + pc[2] - 1};
                                // an x-face ghost lives in its side's compact array [pc2][pc1]
                                const uint32_t dst =
                                    (na == 0) ? (uint32_t)(r.xoff + ((int64_t)(f & 1) * P[2] + pc[2]) * P[1] + pc[1])
                                              : (uint32_t)(r.off + ((int64_t)pc[2] * P[1] + pc[1]) * P[0] + pc[0]);
                                uint32_t need = 0;   // populations an interior cell pulls from this ghost
                                for (int i = 0; i < H->q; ++i) {
                                    bool in = true;
                                    for (int a = 0; a < 3; ++a) {
                                        const int t2 = pc[a] + vel[i][a];
                                        in = in && t2 >= 1 && t2 <= P[a] - 2;
                                    }
                                    if (in) need |= 1u << i;
                                }
                                if (na == 0) need |= kGhostXFace;
                                gmask.push_back(need);
                                const int owner = cover[((size_t)(g[2] >> 1) * ny + (g[1] >> 1)) * nx + (g[0] >> 1)];
                                if (owner >= 0) {
                                    const PatchRec &o = H->rec[owner];
                                    const int64_t src =
                                        o.off + ((int64_t)(g[2] - o.o[2] + 1) * (o.e[1] + 2) + (g[1] - o.o[1] + 1)) *
                                                    (o.e[0] + 2) + (g[0] - o.o[0] + 1);
                                    gdst.push_back(dst);
                                    gsrc.push_back((int)src);
                                    corner.push_back({-1, -1, -1});
                                    continue;
                                }
                                // centre (g + 1/2) / 2 - 1/2: even g -> g/2 - 1 + 3/4, odd g -> (g - 1)/2 + 1/4
                                uint32_t code = 0;
                                int b[3];
                                for (int a = 0; a < 3; ++a) {
                                    const bool even = (g[a] & 1) == 0;
                                    b[a] = even ? g[a] / 2 - 1 : (g[a] - 1) / 2;
                                    if (even) code |= 1u << (29 + a);
                                    bmin[a] = std::min(bmin[a], b[a]);
                                    bmax[a] = std::max(bmax[a], b[a] + 1);
                                }
                                gdst.push_back(dst | code);
                                gsrc.push_back((int)(-(((int64_t)b[2] * ny + b[1]) * nx + b[0]) - 1));
                                corner.push_back({b[0], b[1], b[2]});
                            }
                        t.n = (int)gdst.size() - t.k0;
                        if (bmax[0] >= 0) {
                            t.ox = bmin[0];
                            t.oy = bmin[1];
                            t.oz = bmin[2];
                            t.dx = bmax[0] - bmin[0] + 1;
                            t.dy = bmax[1] - bmin[1] + 1;
                            t.dz = bmax[2] - bmin[2] + 1;
                            if (t.dx * t.dy * t.dz > kGhostBox || t.n > 256) tiles_ok = false;
                        }
                        for (const auto &c : corner)
                            gloc.push_back(c[0] < 0 ? 0
                                                    : ((c[2] - t.oz) * t.dy + (c[1] - t.oy)) * t.dx + (c[0] - t.ox));
                        gtiles.push_back(t);
                    }
        }
    }
    H->ngtile = tiles_ok ? (int64_t)gtiles.size() : 0;
    const char *gmode = std::getenv("LBM_HIER_GHOSTS");
    if (gmode && std::strcmp(gmode, "plain") == 0) H->ngtile = 0;   // the list-only kernel (tests compare both)
    // restriction list: each covered coarse cell, its fine group and patch
    std::vector<int> rc, rf, rp;
    for (int p = 0; p < H->npatch; ++p) {
        const PatchRec &r = H->rec[p];
        const lbm_box &b = H->boxes[p];
        for (int z = b.lo[2]; z < b.hi[2]; ++z)
            for (int y = b.lo[1]; y < b.hi[1]; ++y)
                for (int x = b.lo[0]; x < b.hi[0]; ++x) {
                    rc.push_back((int)(((int64_t)z * ny + y) * nx + x));
                    const int fx = 2 * (x - b.lo[0]) + 1, fy = 2 * (y - b.lo[1]) + 1, fz = 2 * (z - b.lo[2]) + 1;
                    rf.push_back((int)(r.off + ((int64_t)fz * (r.e[1] + 2) + fy) * (r.e[0] + 2) + fx));
                    rp.push_back(p);
                }
    }
    char *meta = static_cast<char *>(H->buf[LBM_HBUF_META]);
    hipStream_t s = coarse->stream;
    hipError_t e = hipMemcpyAsync(meta + H->meta_patch, H->rec.data(), H->rec.size() * sizeof(PatchRec),
                                  hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = upload_tiles(H);
    if (e == hipSuccess)
        e = hipMemcpyAsync(meta + H->meta_cover, cover.data(), cover.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(meta + H->meta_gdst, gdst.data(), gdst.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(meta + H->meta_gsrc, gsrc.data(), gsrc.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && (int64_t)gtiles.size() > H->ngtile_max) e = hipErrorInvalidValue;   // before the copy
    if (e == hipSuccess && (gloc.size() != gdst.size() || gmask.size() != gdst.size())) e = hipErrorInvalidValue;
    if (e == hipSuccess) e = hipMemcpyAsync(meta + H->meta_gmask, gmask.data(), gmask.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(meta + H->meta_gloc, gloc.data(), gloc.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && H->ngtile > 0)
        e = hipMemcpyAsync(meta + H->meta_gtile, gtiles.data(), gtiles.size() * sizeof(GhostTile),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(meta + H->meta_rc, rc.data(), rc.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(meta + H->meta_rf, rf.data(), rf.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipMemcpyAsync(meta + H->meta_rp, rp.data(), rp.size() * 4, hipMemcpyHostToDevice, s);
    if (e == hipSuccess && (int64_t)gdst.size() != H->nghost) e = hipErrorInvalidValue;
    if (e == hipSuccess) {
        // the initial fine state: every padded cell interpolated from the coarse state
        void *X = state_ptr(coarse);
        with_hier_types(H, [&]<int Q, typename T, typename C, bool SH>() {
            launch_patch_init<Q, T, C, SH>(patch_args<C>(H, fine_buf(H, 0), fine_buf(H, 0)),
                                           coarse_view<C>(H, X, X, 0.0, nullptr), fine_buf(H, 0), H->total_padded, s);
        });
        e = hipGetLastError();
        // the x-face ghost arrays start defined (every fine step is preceded by a ghost fill)
        for (int b = 0; b < 2 && e == hipSuccess; ++b)
            e = hipMemsetAsync(static_cast<char *>(H->buf[LBM_HBUF_F_A + b]) + (size_t)H->q * H->pitch * H->elem, 0,
                               (size_t)H->q * H->xg_pitch * H->elem, s);
    }
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) {
        delete H;
        return fail(LBM_EHIP, "hierarchy set-up: %s", hipGetErrorString(e));
    }
    *out = H;
    return LBM_OK;
}

lbm_status lbm_hierarchy_step(lbm_hierarchy *H, int64_t n, int32_t sensor_every) {
    lbm_status st = hier_check(H);
    if (st != LBM_OK) return st;
    if (n < 0 || sensor_every < 0) return fail(LBM_EINVAL, "n and sensor_every must be >= 0");
    lbm_blocks *h = H->coarse;
    int64_t k = 0;
    while (k < n) {
        const int64_t step = h->step + 1;
        const bool sens = sensor_every > 0 && step % sensor_every == 0;
        const bool sens2 = sensor_every > 0 && (step + 1) % sensor_every == 0;
        if (H->use_graph && !sens && !sens2 && n - k >= 2) {
            const int parity = h->cur;
            if (!H->graph[parity]) {
                st = hier_capture(H, parity);
                if (st != LBM_OK) return st;
            }
            HIP_TRY(hipGraphLaunch(H->graph[parity], h->stream));
            h->step += 2;
            H->step += 2;
            k += 2;   // two coarse steps: both parities are back where they were
            continue;
        }
        hier_coarse_step(H, sens);
        ++k;
    }
    HIP_TRY(hipGetLastError());
    return LBM_OK;
}

lbm_status lbm_hierarchy_sensor(lbm_hierarchy *H, double *block_max_host, int8_t *flags_host, int64_t *step) {
    lbm_status st = hier_check(H);
    if (st != LBM_OK) return st;
    if (H->last_sensor_step < 0) return fail(LBM_ESTATE, "no fine sensor step has run");
    lbm_blocks *h = H->coarse;
    if (block_max_host)
        HIP_TRY(hipMemcpyAsync(H->bmax_host.data(), H->buf[LBM_HBUF_BLOCK_MAX], H->bmax_host.size(),
                               hipMemcpyDeviceToHost, h->stream));
    if (flags_host)
        HIP_TRY(hipMemcpyAsync(flags_host, H->buf[LBM_HBUF_FLAGS], H->nblocks, hipMemcpyDeviceToHost, h->stream));
    HIP_TRY(hipStreamSynchronize(h->stream));
    if (block_max_host) {
        for (int64_t b = 0; b < H->nblocks; ++b) {
            if (h->L.cbytes == 8) block_max_host[b] = reinterpret_cast<const double *>(H->bmax_host.data())[b];
            else block_max_host[b] = reinterpret_cast<const float *>(H->bmax_host.data())[b];
        }
    }
    if (step) *step = H->last_sensor_step;
    return LBM_OK;
}

lbm_status lbm_hierarchy_patch_fields(lbm_hierarchy *H, int32_t patch, double *rho_host, double *u_host,
                                      double *f_host) {
    lbm_status st = hier_check(H);
    if (st != LBM_OK) return st;
    if (patch < 0 || patch >= H->npatch) return fail(LBM_EINVAL, "patch %d out of range", patch);
    const PatchRec &r = H->rec[patch];
    const int64_t n = (int64_t)r.e[0] * r.e[1] * r.e[2];
    double *stage = reinterpret_cast<double *>(static_cast<char *>(H->buf[LBM_HBUF_META]) + H->meta_stage);
    double *rho_d = stage, *u_d = stage + n, *f_d = stage + 4 * n;
    hipStream_t s = H->coarse->stream;
    with_hier_types(H, [&]<int Q, typename T, typename C, bool SH>() {
        launch_patch_macros<Q, T, C, SH>(patch_args<C>(H, fine_buf(H, H->cur), nullptr), fine_buf(H, H->cur), patch,
                                         n, rho_d, u_d, f_host ? f_d : nullptr, s);
    });
    HIP_TRY(hipGetLastError());
    if (rho_host) HIP_TRY(hipMemcpyAsync(rho_host, rho_d, n * 8, hipMemcpyDeviceToHost, s));
    if (u_host) HIP_TRY(hipMemcpyAsync(u_host, u_d, 3 * n * 8, hipMemcpyDeviceToHost, s));
    if (f_host) HIP_TRY(hipMemcpyAsync(f_host, f_d, H->q * n * 8, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return LBM_OK;
}

lbm_status lbm_hierarchy_info(lbm_hierarchy *H, int64_t *fine_cells, int64_t *fine_blocks, double *n_eff,
                              double *tau_fine, int32_t *tile_x, int32_t *workgroups) {
    lbm_status st = hier_check(H);
    if (st != LBM_OK) return st;
    if (fine_cells) *fine_cells = H->fine_cells;
    if (fine_blocks) *fine_blocks = H->nblocks;
    // effective cells (Sec. 5.2): cells of level i weighted by 2^-(L - i); the
    // coarse level (i = 0) steps once per two fine steps (L = 1)
    if (n_eff) *n_eff = 0.5 * (double)H->coarse->L.cells + (double)H->fine_cells;
    if (tau_fine) *tau_fine = H->tau_f;
    if (tile_x) *tile_x = H->wmax;
    if (workgroups) *workgroups = H->nwg;
    return LBM_OK;
}

lbm_status lbm_hierarchy_autotune(lbm_hierarchy *H, int32_t reps, int32_t *tile_x, int32_t *workgroups,
                                  double *step_us) {
    lbm_status st = hier_check(H);
    if (st != LBM_OK) return st;
    if (reps < 1) return fail(LBM_EINVAL, "reps = %d < 1", reps);
    hipStream_t s = H->coarse->stream;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // the timed launches read the fine state and write the other fine buffer,
    // which the next step overwrites, and the restricting ones also write the
    // coarse buffer that the next coarse step overwrites: the state is left
    // unchanged
    const void *src = fine_buf(H, H->cur);
    void *dst = fine_buf(H, H->cur ^ 1);
    lbm_blocks *h = H->coarse;
    void *coarse_next = h->d.buf[h->cur ? LBM_BUF_F_A : LBM_BUF_F_B];
    hipError_t e = hipSuccess;
    auto time_steps = [&](void *restrict_out, float &ms) {
        hier_fine_step(H, src, dst, false, 0, restrict_out);   // warm-up
        e = hipEventRecord(e0, s);
        for (int r = 0; r < reps && e == hipSuccess; ++r) hier_fine_step(H, src, dst, false, 0, restrict_out);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        return e == hipSuccess;
    };
    float best = 1e30f;
    int best_w = H->wmax, best_nwg = H->nwg;
    const int per_cu[5] = {1, 2, 4, 8, 16};
    for (int w : {8, 16, 32, kBandMaxW}) {
        build_tiles(H, w);
        e = upload_tiles(H);
        if (e != hipSuccess) break;
        for (int pc : per_cu) {
            H->nwg = (int)std::min<int64_t>(H->ntiles, (int64_t)pc * kHierCUs);
            float ms = 0.0f;
            if (!time_steps(nullptr, ms)) break;
            if (ms < best) {
                best = ms;
                best_w = w;
                best_nwg = H->nwg;
            }
        }
        if (e != hipSuccess) break;
    }
    // the restricting step on the chosen tiling: its LDS sums hold the
    // resident workgroups to one or two per CU, so fewer candidates
    build_tiles(H, best_w);
    if (e == hipSuccess) e = upload_tiles(H);
    H->nwg = best_nwg;
    float best_r = 1e30f;
    int best_nwg_r = H->nwg_restrict;
    for (int pc : {1, 2, 4}) {
        if (e != hipSuccess) break;
        H->nwg_restrict = (int)std::min<int64_t>(H->ntiles, (int64_t)pc * kHierCUs);
        float ms = 0.0f;
        if (!time_steps(coarse_next, ms)) break;
        if (ms < best_r) {
            best_r = ms;
            best_nwg_r = H->nwg_restrict;
        }
    }
    H->nwg_restrict = best_nwg_r;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    // graphs captured with the old tile list are stale
    for (int p = 0; p < 2; ++p)
        if (H->graph[p]) {
            (void)hipGraphExecDestroy(H->graph[p]);
            H->graph[p] = nullptr;
        }
    if (e != hipSuccess) return fail(LBM_EHIP, "autotune: %s", hipGetErrorString(e));
    if (tile_x) *tile_x = H->wmax;
    if (workgroups) *workgroups = H->nwg;
    if (step_us) *step_us = 1e3 * (double)best / reps;
    return LBM_OK;
}

lbm_status lbm_hierarchy_profile(lbm_hierarchy *H, int32_t steps, double *us) {
    lbm_status st = hier_check(H);
    if (st != LBM_OK) return st;
    if (steps < 1) return fail(LBM_EINVAL, "steps = %d < 1", steps);
    if (!us) return fail(LBM_EINVAL, "us is NULL");
    hipEvent_t ev[7] = {};
    hipError_t e = hipSuccess;
    for (int i = 0; i < 7 && e == hipSuccess; ++i) e = hipEventCreate(&ev[i]);
    // sums over launches: coarse, ghosts (two per step), first fine step,
    // second fine step (with the restriction) plus the separate restriction if any
    double sum[4] = {0.0, 0.0, 0.0, 0.0};
    for (int32_t k = 0; k < steps && e == hipSuccess; ++k) {
        hier_coarse_step(H, false, ev);
        e = hipGetLastError();
        if (e == hipSuccess) e = hipEventSynchronize(ev[6]);
        float ms[6] = {};
        for (int i = 0; i < 6 && e == hipSuccess; ++i) e = hipEventElapsedTime(&ms[i], ev[i], ev[i + 1]);
        // launch order: ghosts, fine, coarse, ghosts, fine (+ restriction), [restriction]
        sum[1] += ms[0] + ms[3];
        sum[2] += ms[1];
        sum[0] += ms[2];
        sum[3] += ms[4] + ms[5];
    }
    for (int i = 0; i < 7; ++i)
        if (ev[i]) (void)hipEventDestroy(ev[i]);
    if (e != hipSuccess) return fail(LBM_EHIP, "profile: %s", hipGetErrorString(e));
    us[0] = 1e3 * sum[0] / steps;
    us[1] = 1e3 * sum[1] / (2.0 * steps);
    us[2] = 1e3 * sum[2] / steps;
    us[3] = 1e3 * sum[3] / steps;
    return LBM_OK;
}

void lbm_destroy_hierarchy(lbm_hierarchy *H) {
    if (!H) return;
    for (int p = 0; p < 2; ++p)
        if (H->graph[p]) (void)hipGraphExecDestroy(H->graph[p]);
    delete H;
}

}  // extern "C"
