/*
 * lbm.h -- C interface of the MI355X lattice Boltzmann step with the kinetic
 * mesh-refinement sensor (Thorimbert et al., "Local mesh refinement sensor for
 * the lattice Boltzmann method", arXiv:1507.06767).
 *
 * One handle owns one uniform grid of cells.  Each step advances the BGK
 * lattice Boltzmann equation (Sec. 2.2, Eq. bgklb with the equilibrium of
 * Eq. feq_i and the moments of Eqs. rho and u) by one collide-and-stream
 * cycle, fused on the GPU with the kinetic sensor of Sec. 3.2 (Eq. sensor /
 * Eq. kkn, or the L2 ratio ||f^neq||_2 / ||f^eq||_2), its maximum over sensor
 * blocks and the refine / keep / coarsen decision of Sec. 3.4.
 *
 * Conventions that hold for every entry point:
 *   - Every function returns an lbm_status (0 on success, < 0 on error) and
 *     never aborts or throws; on error, lbm_last_error() returns a message
 *     for the calling thread.
 *   - Device memory is OWNED BY THE CALLER.  The library never allocates
 *     device memory: the caller sizes the five buffers with
 *     lbm_required_bytes(), allocates them (for instance as torch tensors)
 *     and keeps them alive until lbm_destroy().  The one exception is the
 *     32 KiB static workspace of lbm_conservation_noalloc, part of the
 *     library's code object.  Host arrays are only read or written during
 *     the call that receives them.
 *   - Work is enqueued on the caller's HIP stream (lbm_desc.stream; NULL is
 *     the null stream).  lbm_step_n() is asynchronous; the calls that return
 *     host data synchronise that stream.  One handle must not be used from
 *     two host threads at once.
 *   - Host population arrays are float64, shape [q][nz][ny][nx] (x fastest),
 *     in the velocity order below.  Host macroscopic arrays are float64:
 *     rho [nz][ny][nx], u [3][nz][ny][nx] (u_z = 0 in 2D).
 *   - The stored state is the set of post-collision populations S_k.  Step k
 *     (1-based) computes S_k = C(T(S_{k-1})): T streams with the boundary
 *     conditions, C is the BGK collision with Guo's body-force term.  The
 *     sensor of step k is evaluated on the pre-collision populations
 *     T(S_{k-1}).
 *
 * Velocity order (opposite of i: i+1 for odd i, i-1 for even i > 0):
 *   D2Q9 : 0 (0,0) 1 (1,0) 2 (-1,0) 3 (0,1) 4 (0,-1) 5 (1,1) 6 (-1,-1)
 *          7 (1,-1) 8 (-1,1)
 *   D3Q19: 0 (0,0,0) 1 (1,0,0) 2 (-1,0,0) 3 (0,1,0) 4 (0,-1,0) 5 (0,0,1)
 *          6 (0,0,-1) 7 (1,1,0) 8 (-1,-1,0) 9 (1,-1,0) 10 (-1,1,0)
 *          11 (1,0,1) 12 (-1,0,-1) 13 (1,0,-1) 14 (-1,0,1) 15 (0,1,1)
 *          16 (0,-1,-1) 17 (0,1,-1) 18 (0,-1,1)
 *   D3Q27: 0..18 as D3Q19, then 19 (1,1,1) 20 (-1,-1,-1) 21 (1,1,-1)
 *          22 (-1,-1,1) 23 (1,-1,1) 24 (-1,1,-1) 25 (-1,1,1) 26 (1,-1,-1)
 *
 * Boundary faces, in the order -x,+x,-y,+y,-z,+z, are periodic or walls.
 * Walls use halfway bounce-back: all n cells along an axis are fluid and the
 * wall lies half a cell beyond the outer ones.  A link pulled from beyond a
 * wall returns the opposite population of the same cell plus the moving-wall
 * term 6 w_i rho0 (xi_i . u_w) (the moving bounce-back rule cited in
 * Sec. 4.1), where u_w is the sum of the wall velocities of every wall face
 * the link crosses (so a moving lid acts on the links through its edges and
 * corners too, which keeps mass exactly conserved).
 */
#ifndef LBM_H
#define LBM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBM_ABI_VERSION 2u

typedef int32_t lbm_status;
enum {
    LBM_OK = 0,
    LBM_EINVAL = -1,      /* bad argument or descriptor; nothing was enqueued */
    LBM_ENOTSUP = -2,     /* valid but not supported by this library */
    LBM_EHIP = -3,        /* a HIP call failed; lbm_last_error() has its text */
    LBM_ESTATE = -4,      /* call not valid in the handle's state */
    LBM_ENONFINITE = -5   /* a sensor block holds a NaN or Inf (data still written) */
};

enum { LBM_D2Q9 = 9, LBM_D3Q19 = 19, LBM_D3Q27 = 27 };         /* lbm_desc.lattice */
enum { LBM_F64 = 0, LBM_F32 = 1, LBM_F32_SHIFTED = 2,          /* lbm_desc.storage */
       LBM_F16_SHIFTED = 3, LBM_BF16_SHIFTED = 4,
       LBM_F16_SHIFTED_SR = 5, LBM_BF16_SHIFTED_SR = 6 };
enum { LBM_SENSOR_L2 = 0, LBM_SENSOR_KKN = 1 };                 /* lbm_desc.sensor_kind */
enum { LBM_BC_PERIODIC = 0, LBM_BC_WALL = 1 };                  /* lbm_desc.face_bc[] */
enum { LBM_BUF_F_A = 0, LBM_BUF_F_B = 1, LBM_BUF_BLOCK_MAX = 2,  /* lbm_desc.buf[] */
       LBM_BUF_FLAGS = 3, LBM_BUF_SCRATCH = 4, LBM_NBUF = 5 };

/* Refinement decision per sensor block. */
enum { LBM_FLAG_COARSEN = -1, LBM_FLAG_KEEP = 0, LBM_FLAG_REFINE = 1, LBM_FLAG_NONFINITE = 2 };

typedef struct lbm_blocks lbm_blocks;   /* opaque handle */

enum { LBM_PROFILE_UNIFORM = 0, LBM_PROFILE_SMOOTH = 1 };      /* lbm_desc.wall_profile[] */
enum { LBM_STREAMING_AUTO = 0, LBM_STREAMING_PINGPONG = 1,    /* lbm_desc.streaming */
       LBM_STREAMING_INPLACE = 2 };

typedef struct {
    uint32_t abi_version;   /* LBM_ABI_VERSION */
    int32_t lattice;        /* LBM_D2Q9, LBM_D3Q19 or LBM_D3Q27 */
    int32_t storage;        /* LBM_F64: populations and arithmetic in float64.
                               LBM_F32: float32 populations f_i, float32 arithmetic.
                               LBM_F32_SHIFTED: float32 stores f_i - w_i rho0,
                               float32 arithmetic (same bytes, finer rounding).
                               LBM_F16_SHIFTED / LBM_BF16_SHIFTED: IEEE half / bfloat16
                               store f_i - w_i rho0 (half the bytes), float32
                               arithmetic, rounding to nearest even on store.
                               LBM_F16_SHIFTED_SR / LBM_BF16_SHIFTED_SR: the same with
                               stochastic rounding on store (unbiased; the random
                               bits hash (cell, population, step), so runs are
                               reproducible bit for bit). */
    int32_t sensor_kind;    /* LBM_SENSOR_L2: ||f^neq||_2 / ||f^eq||_2;
                               LBM_SENSOR_KKN: (1/q) sum_i |f^neq_i / f^eq_i| (Eq. kkn) */
    int32_t extent[3];      /* cells along x, y, z; extent[2] == 1 for D2Q9;
                               extent[0]*extent[1]*extent[2] < 2^31 */
    int32_t block[3];       /* sensor block edge: {8,8,1} for D2Q9, {8,8,8} in 3D
                               (other sizes: LBM_ENOTSUP).  Blocks start at
                               the origin; partial blocks at the far faces are
                               allowed and take the maximum of the cells they hold. */
    int32_t face_bc[6];     /* -x,+x,-y,+y,-z,+z: LBM_BC_PERIODIC or LBM_BC_WALL; a
                               periodic face needs a periodic opposite face; the z
                               faces are periodic for D2Q9 */
    double wall_u[6][3];    /* wall velocity per face (ignored on periodic faces) */
    double tau;             /* BGK relaxation time (Eq. bgklb), > 1/2 */
    double rho0;            /* reference density: initial density, wall density of
                               the moving-wall term, and shift of LBM_F32_SHIFTED */
    double force[3];        /* body-force density (Guo scheme); zeros mean none */
    double theta_refine;    /* flag REFINE iff block max > theta_refine */
    double theta_coarsen;   /* flag COARSEN iff block max < theta_coarsen
                               (<= theta_refine) */
    double smagorinsky;     /* Smagorinsky constant C in [0, 1] (0: plain BGK).  The
                               subgrid model the paper adds to BGK at high Reynolds
                               number (Sec. 4, C = 0.14): per cell the relaxation time
                               tau_e = (tau + sqrt(tau^2 + 18 sqrt(2) C^2 |Pi| / rho)) / 2,
                               Pi = sum_i xi_i xi_i (f_i - f^eq_i), i.e. the viscosity
                               c_s^2 (tau - 1/2) plus C^2 |S|, |S| = sqrt(2 S:S) */
    int32_t wall_profile[6];  /* per face: LBM_PROFILE_UNIFORM, or LBM_PROFILE_SMOOTH
                               for the smoothed lid of the 3D cavity (Sec. 5.1): the
                               face's wall_u times prod over its in-plane axes of
                               (1 - s^18)^2, s = (2 x + 1 - n) / n in (-1, 1) at the
                               fluid cell's centre (ignored on periodic faces) */
    int32_t streaming;      /* LBM_STREAMING_AUTO: in place (one buffer, the AA pattern)
                               when a buffer is at most 512 MiB, except 3D float64
                               and the 2D grids of lbm_set_multistep;
                               PINGPONG: read F_A, write F_B, swap (required by
                               lbm_create_hierarchy); INPLACE: in place (not for 3D
                               float64).  Results are identical bit for bit. */
    void *buf[LBM_NBUF];    /* caller-owned device buffers, see lbm_required_bytes();
                               F_A and F_B must be 256-byte aligned; no two overlap */
    size_t buf_bytes[LBM_NBUF];  /* their sizes in bytes, >= the required sizes */
    void *stream;           /* hipStream_t for all work of this handle */
} lbm_desc;

/* Sizes in bytes of the five device buffers for descriptor d (its buf and
 * buf_bytes fields are ignored).  Pure host computation, no HIP call.
 *   F_A, F_B   : two population arrays of q padded planes each.  Ping-pong
 *                streaming alternates between them; the in-place scheme
 *                (chosen for arrays up to 512 MiB) steps F_A only and uses F_B
 *                as staging when states are read or written;
 *   BLOCK_MAX  : one float32 (float32/16-bit storages) or float64 (F64) per block,
 *                followed by one 64-bit accumulator word per block;
 *   FLAGS      : one int8 per sensor block;
 *   SCRATCH    : staging for host transfers, the conservation partial sums, the
 *                per-cell sums of the time-averaged sensor and the level maps.
 * Returns LBM_EINVAL / LBM_ENOTSUP for a bad descriptor. */
lbm_status lbm_required_bytes(const lbm_desc *d, size_t bytes[LBM_NBUF]);

/* Validates d (including buffer sizes and alignment), creates a handle and
 * writes the initial state S_0 into F_A: f0_host (float64 [q][cells]) if not
 * NULL, otherwise the rest state f_i = w_i rho0.  Synchronises the stream.
 * The step counter starts at 0.  *out is set only on success. */
lbm_status lbm_create_blocks(const lbm_desc *d, const double *f0_host, lbm_blocks **out);

/* Enqueues n >= 0 steps k = s+1 .. s+n, s being the current step counter.
 * Step k also evaluates the sensor, its block maxima and the flags when
 * sensor_every > 0 and k % sensor_every == 0 (sensor_every == 0: never).
 * Asynchronous: returns once the launches are enqueued. */
lbm_status lbm_step_n(lbm_blocks *h, int64_t n, int32_t sensor_every);

/* Replays runs of `chunk` sensor-free steps (an even number; 0 switches it
 * off, the default) in lbm_step_n from a HIP graph captured once per buffer
 * parity, instead of launching each step: for small grids, whose steps are
 * bound by launch overhead.  Steps whose run would contain a sensor step,
 * and all steps while the time average is on, are launched one by one.
 * Results are identical bit for bit.  Needs a non-NULL stream
 * (LBM_ENOTSUP otherwise) and is refused for stochastic rounding (its
 * random bits depend on the step index).  Synchronises the stream. */
lbm_status lbm_use_graphs(lbm_blocks *h, int32_t chunk);

/* Synchronises the stream and returns the block maxima (as float64) and the
 * flags of the latest step that evaluated the sensor, and that step's index.
 * Any of the host pointers may be NULL.  Blocks are ordered [nbz][nby][nbx].
 * LBM_ESTATE if no sensor step has run since the state was last set;
 * LBM_ENONFINITE if some block maximum is NaN or Inf (outputs still written). */
lbm_status lbm_sensor_flags(lbm_blocks *h, double *block_max_host, int8_t *flags_host,
                            int64_t *step_index);

/* Refinement level of every sensor block from the block maxima M of the
 * latest sensor step (Sec. 3.4): phi = log2 M, l = clamp(floor(a phi + b),
 * lmin, lmax); a non-finite M gives lmax and M = 0 gives lmin.  The offset b
 * is this library's addition: with a alone, sensor values near 1e-3
 * (phi ~ -10) cannot be placed on levels >= 0.  Then the buffer layer of
 * Sec. 5.2: each block takes the largest level within `buffer` blocks
 * (Chebyshev distance, 0..8).  levels_host: int8 [nbz][nby][nbx].
 * Synchronises the stream; LBM_ESTATE if no sensor step has run. */
lbm_status lbm_sensor_levels(lbm_blocks *h, double a, double b, int32_t lmin, int32_t lmax,
                             int32_t buffer, int8_t *levels_host);

/* Time-averaged sensor (Sec. 5.1 averages the sensor over a period before
 * building its mesh).  _begin clears per-cell running sums; from then on
 * every sensor step adds each cell's sensor value.  lbm_sensor_average
 * returns, per block, the largest time-averaged cell value (float64,
 * [nbz][nby][nbx]; NULL allowed) and the number of sensor steps summed.
 * _end stops accumulating (the sums stay readable).  The sums live in the
 * scratch buffer; lbm_sensor_average synchronises the stream. */
lbm_status lbm_sensor_average_begin(lbm_blocks *h);
lbm_status lbm_sensor_average(lbm_blocks *h, double *block_max_host, int64_t *samples);
lbm_status lbm_sensor_average_end(lbm_blocks *h);

/* Synchronises the stream and returns the macroscopic fields of the stored
 * state computed in float64: rho = sum_i S_i, u = (sum_i xi_i S_i - F/2) / rho
 * (the velocity of the last collision, Eqs. rho and u).  Either pointer may
 * be NULL. */
lbm_status lbm_get_macros(lbm_blocks *h, double *rho_host, double *u_host);

/* Synchronises the stream and returns per-block means of the fields of
 * lbm_get_macros: means_host[nbz][nby][nbx][4] = (rho - rho0, u_x, u_y, u_z)
 * averaged over the cells of each 8^d block (edge blocks average the cells
 * they hold), float64.  These are the inputs of the learned flag predictor
 * (include/lbm_cnn.h); the blocks are those of the sensor (Sec. 3.4). */
lbm_status lbm_block_means(lbm_blocks *h, double *means_host);

/* Stored populations S_k as float64 [q][cells] (checkpointing, tests). */
lbm_status lbm_get_populations(lbm_blocks *h, double *f_host);

/* Replaces the stored state by f_host (float64 [q][cells], converted to the
 * storage type).  Non-finite values are accepted; the next sensor step flags
 * their blocks LBM_FLAG_NONFINITE.  Synchronises the stream. */
lbm_status lbm_set_populations(lbm_blocks *h, const double *f_host);

/* Replaces the stored state by the equilibrium f^eq(rho, u) of Eq. feq_i,
 * computed on the GPU in float64 from rho_host [cells] (NULL: rho0 everywhere)
 * and u_host [3][cells] (NULL: at rest).  Synchronises the stream. */
lbm_status lbm_set_equilibrium(lbm_blocks *h, const double *rho_host, const double *u_host);

/* How the handle streams: *inplace = 1 for the single-buffer scheme (steps
 * alternate between a gather-scatter launch and a local launch; the step
 * counter's parity says which comes next via *next_is_gather), 0 for
 * ping-pong; *tile_x = workgroup tile width in cells (256: row tiles of one
 * row, otherwise tiles of 8 rows).  Any pointer may be NULL.  Pure host
 * query. */
lbm_status lbm_get_scheme(lbm_blocks *h, int32_t *inplace, int32_t *next_is_gather, int32_t *tile_x);

/* Several steps per launch for small 2D grids (temporal blocking; not in the
 * paper: a launch of one step of a 64^2 grid lasts about as long as the
 * latency of one small kernel).  Runs of sensor-free steps of a ping-pong
 * D2Q9 handle of at most 65,536 cells are taken up to `steps` at a time by
 * one launch, in which each workgroup steps an 8 x 8 tile of the grid and a
 * halo of 4 cells around it in LDS; the results equal one launch per step bit
 * for bit (sensor steps are launched alone).  On by default with 5 steps
 * where it applies: D2Q9, ping-pong (LBM_STREAMING_AUTO picks ping-pong for
 * such grids), no stochastic rounding.  steps = 0 switches it off, 2 .. 5
 * sets the most steps per launch; LBM_EINVAL for other values, LBM_ENOTSUP
 * for steps > 0 on a handle where it does not apply.  Synchronises the stream
 * and drops captured graphs.  lbm_get_multistep reads the setting (0: off);
 * pure host query. */
lbm_status lbm_set_multistep(lbm_blocks *h, int32_t steps);
lbm_status lbm_get_multistep(lbm_blocks *h, int32_t *steps);

/* Step counter (number of steps taken since it was last set). */
lbm_status lbm_get_step(lbm_blocks *h, int64_t *step);
lbm_status lbm_set_step(lbm_blocks *h, int64_t step);

/* Totals over all cells of the stored state, accumulated in float64 by a
 * fixed-order two-pass tree (bitwise reproducible): out[0] = sum rho,
 * out[1..3] = sum_i xi_i S_i summed over cells.  Synchronises the stream. */
lbm_status lbm_conservation(lbm_blocks *h, double out[4]);

/* For callers that cannot allocate device memory or pass a workspace (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): lbm_conservation with the same result bits, whose partial sums
 * and totals live in a 32 KiB array the library holds in device memory of
 * each GPU it runs on (kept until the process ends; its address is looked
 * up once per device, on the first call there) instead of the handle's
 * scratch buffer.  No grid is too large for it: the first pass caps its
 * workgroups at 1024, each then summing more cells.  Allocates nothing and
 * calls no allocating routine; for an in-place handle the natural-order
 * copy of the state is built in F_B, which the caller already provided.
 * All calls on one GPU share the array: calls that overlap in time on one
 * GPU (two host threads, or two streams) race and must be serialised by the
 * caller.  Synchronises the stream. */
lbm_status lbm_conservation_noalloc(lbm_blocks *h, double out[4]);

/* tau = nu / c_s^2 + 1/2 with nu = u * n_across / re (Eq. nu_omega, c_s^2 = 1/3). */
lbm_status lbm_tau_from_reynolds(double u, double n_across, double re, double *tau);

/* Synchronises the stream and releases the handle; caller buffers are left
 * untouched.  NULL is a no-op. */
void lbm_destroy(lbm_blocks *h);

/* Message of the last failed call on this thread ("" if none). */
const char *lbm_last_error(void);

/* Picks the fastest tile for the handle's step kernel, 32, 64 or 128 cells
 * along x by 8 rows, or for 3D ping-pong also row tiles of 256 cells of one
 * row (*tile_x = 256), by timing `reps` launches (in-place: `reps` pairs) of
 * each on the handle's stream, and keeps it for later steps.  The state is not
 * changed: ping-pong timings write only the spare buffer, in-place ones run
 * on a copy in F_B.  Every tile width gives bit-identical results.  3D
 * float64 (one tile shape) returns 64 at once.  Synchronises the stream. */
lbm_status lbm_autotune(lbm_blocks *h, int32_t reps, int32_t *tile_x);

/* ---------------------------------------------------------------------------
 * Two-level patch hierarchy: boxes of the handle's grid refined by a factor 2
 * (the static refinement built from the sensor in Sec. 5.1, coupled as in the
 * AMR runs of Sec. 5.2, after Dupuis & Chopard).  Acoustic scaling: every
 * coarse step is two fine steps with tau_f = 2 tau - 1/2.  Coupling:
 *   - ghost layer of each patch: from an abutting patch where one holds the
 *     cell, else trilinear interpolation of the coarse post-collision
 *     populations (linear in time between coarse steps), whose
 *     non-equilibrium part S - f^eq(rho, u) is scaled by
 *     alpha = (tau_f - 1) / (2 (tau - 1));
 *   - restriction: after each coarse step every covered coarse cell takes the
 *     mean of its 8 fine cells, non-equilibrium part scaled by 1/alpha.
 * The coarse handle keeps stepping every cell; it must stream ping-pong
 * (lbm_desc.streaming = LBM_STREAMING_PINGPONG), be 3D, have no body force
 * and no Smagorinsky model, and have tau and 2 tau - 1/2 at least 0.05 away
 * from 1 (else LBM_ENOTSUP).  The fine level stores its populations in the
 * coarse handle's storage type, 16-bit shifted storages included; every
 * kernel of the hierarchy computes in float32 for them (float64 for
 * LBM_F64).  While the hierarchy exists the coarse handle must only be
 * stepped through lbm_hierarchy_step.
 *
 * Boxes are in coarse cells, [lo, hi) per axis, with 1 <= lo, hi <= n - 1,
 * extents multiples of 4 (fine extents multiples of 8, whole 8^3 sensor
 * blocks), and may touch but not overlap (LBM_EINVAL otherwise).  Fine
 * sensor blocks are numbered patch by patch, x fastest within a patch.
 * ------------------------------------------------------------------------- */
typedef struct lbm_hierarchy lbm_hierarchy;   /* opaque handle */

typedef struct {
    int32_t lo[3];   /* first coarse cell of the box along x, y, z */
    int32_t hi[3];   /* one past the last */
} lbm_box;

enum { LBM_HBUF_F_A = 0, LBM_HBUF_F_B = 1, LBM_HBUF_BLOCK_MAX = 2,   /* hierarchy buffers */
       LBM_HBUF_FLAGS = 3, LBM_HBUF_META = 4, LBM_NHBUF = 5 };

/* Sizes of the five caller-owned device buffers of a hierarchy: the fine
 * populations twice (padded patches, then the compact x-face ghost arrays;
 * ping-pong), the fine block maxima (the
 * coarse handle's compute precision), the fine flags, and META (patch table,
 * block-to-patch map, coarse cover map, staging).  Host computation only. */
lbm_status lbm_hierarchy_required_bytes(const lbm_blocks *coarse, int32_t nbox, const lbm_box *boxes,
                                        size_t bytes[LBM_NHBUF]);

/* Creates the hierarchy over `coarse`; buffers must be 256-byte aligned device
 * memory of at least the required sizes.  The fine state starts as the
 * interpolation of the coarse state.  use_graph != 0 replays pairs of coarse
 * steps from a captured HIP graph (needs a non-NULL stream; with the NULL
 * stream the steps are launched one by one; LBM_ENOTSUP for the stochastic
 * rounding storages, whose random bits depend on the step index).
 * Synchronises the stream. */
lbm_status lbm_create_hierarchy(lbm_blocks *coarse, int32_t nbox, const lbm_box *boxes, void *const buf[LBM_NHBUF],
                                const size_t buf_bytes[LBM_NHBUF], int32_t use_graph, lbm_hierarchy **out);

/* n coarse steps (2n fine steps), asynchronous.  On coarse steps k with
 * k % sensor_every == 0 (sensor_every > 0) the coarse sensor runs as in
 * lbm_step_n and the fine sensor on the second fine step. */
lbm_status lbm_hierarchy_step(lbm_hierarchy *H, int64_t n, int32_t sensor_every);

/* Fine block maxima (float64, NULL allowed), flags (int8, NULL allowed) of
 * the last fine sensor step, and that coarse step index.  Synchronises. */
lbm_status lbm_hierarchy_sensor(lbm_hierarchy *H, double *block_max_host, int8_t *flags_host, int64_t *step);

/* Interior fields of one patch, float64 [ez][ey][ex] (x fastest): rho, u
 * [3][...], and populations [q][...] in the interface velocity order; each
 * may be NULL.  Synchronises. */
lbm_status lbm_hierarchy_patch_fields(lbm_hierarchy *H, int32_t patch, double *rho_host, double *u_host,
                                      double *f_host);

/* Fine cells and blocks, effective cells N_eff = n_coarse / 2 + n_fine (the
 * cost measure of Sec. 5.2: cells of level i weighted by their update rate),
 * tau_f, and the fine step's widest tile and persistent workgroup count.
 * Any pointer may be NULL. */
lbm_status lbm_hierarchy_info(lbm_hierarchy *H, int64_t *fine_cells, int64_t *fine_blocks, double *n_eff,
                              double *tau_fine, int32_t *tile_x, int32_t *workgroups);

/* Picks the fine step's tiling and its persistent workgroup count (1 to 16
 * per compute unit) by timing `reps` launches of each with HIP events on the
 * handle's stream, then the workgroup count (1, 2 or 4 per compute unit) of
 * the fine step that also restricts to the coarse level, on that tiling; the
 * state is not changed (the timed launches write the buffers that the next
 * fine and coarse steps overwrite).  Tilings (512 threads): bands
 * (*tile_x = 48, the default) of 8 rows x 8 slices of a patch, the whole row
 * when it is at most 48 cells wide, whose cells the threads take in memory
 * order (only on fine buffers below 4 GiB: they address them with 32-bit
 * offsets); or tiles of W x 8 x 8 cells, W the widest of 8, 16, 32 not above
 * tile_x that fits the patch row.  Every tiling gives the same bits.
 * *workgroups receives the plain fine step's count; step_us (NULL allowed)
 * the chosen configuration's mean duration of one plain fine step over all
 * patches, in microseconds.  Synchronises. */
lbm_status lbm_hierarchy_autotune(lbm_hierarchy *H, int32_t reps, int32_t *tile_x, int32_t *workgroups,
                                  double *step_us);

/* Advances the hierarchy by `steps` coarse steps (no sensor) launched one by
 * one, with HIP events recorded between the kernels on the handle's stream,
 * and writes mean durations in microseconds: us[0] the coarse step, us[1] a
 * ghost fill, us[2] the first fine step over all patches, us[3] the second
 * fine step, which also restricts the fine level to the covered coarse
 * cells.  The kernels run in their production order
 * and on production data, so their caches are warm or cold as they would be
 * in stepping; each bracket also times a few microseconds of event packets.
 * steps >= 1; us must hold 4 doubles.  Synchronises. */
lbm_status lbm_hierarchy_profile(lbm_hierarchy *H, int32_t steps, double *us);

/* Releases the hierarchy (host memory and graphs); buffers are untouched. */
void lbm_destroy_hierarchy(lbm_hierarchy *H);

#ifdef __cplusplus
}
#endif

#endif /* LBM_H */
