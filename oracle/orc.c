/*
 * orc.c -- FP64 CPU oracle for the lattice Boltzmann BGK step and the kinetic
 * refinement sensor of Thorimbert et al., "Local mesh refinement sensor for the
 * lattice Boltzmann method" (arXiv:1507.06767).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP path is checked against.  Only the tests, the smoke check and the CPU
 * baseline leg of the benchmark may load it; the product path never does.  It
 * shares no code, header or table with the HIP library: its velocity set is
 * enumerated here, its populations are stored cell-major (AoS) in its own
 * order, and it streams by PUSHING populations to their neighbours, whereas the
 * GPU kernel PULLS them.
 *
 * What one step computes (Sec. 2.2, Eqs. bgklb, feq_i, rho, u and the
 * collide-and-stream split that follows them):
 *   S_k = C(T(S_{k-1})), where the state S is the set of post-collision
 *   populations f^out, T is the streaming with boundary conditions and C the
 *   BGK collision.  This is the paper's collide-then-stream loop cut after the
 *   collision, which is the order AMROC-LBM uses (stream first, then collide;
 *   Sec. 2.1).  The sensor of Sec. 3.2 (Eq. sensor / Eq. kkn) is evaluated on
 *   the pre-collision populations f = T(S_{k-1}) of the step.
 *
 * Readings of the paper that this file takes (the paper is silent on them):
 *   - halfway bounce-back on wall faces; all n cells along an axis are fluid;
 *   - the moving-wall term is the one of the moving bounce-back rule the
 *     paper cites for its cavity (Sec. 4.1), with the wall density equal to
 *     the reference density rho0;
 *   - a link that leaves the domain through several wall faces (an edge or a
 *     corner) takes the SUM of those faces' wall velocities, so that a single
 *     moving lid acts on every link that crosses it;
 *   - body force by Guo's scheme (the paper cites it for the droplet case,
 *     Sec. 4.5): rho*u = sum_i xi_i f_i + F/2 and a source term in the
 *     collision;
 *   - second sensor form: the L2 ratio ||f^neq||_2 / ||f^eq||_2 next to the
 *     paper's mean |f^neq_i / f^eq_i|;
 *   - per-block maximum of the cell sensor over blocks that start at the
 *     origin (partial blocks at the far faces allowed), NaN-propagating, and
 *     the flags +2 non-finite, +1 refine (M > theta_r), -1 coarsen
 *     (M < theta_c), 0 keep.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAXQ 27

typedef struct {
    int q, d;
    int c[ORC_MAXQ][3];
    double w[ORC_MAXQ];
    int opp[ORC_MAXQ];
    double cs2;
} orc_lattice;

/* Parameters of one uniform grid.  Face order: -x,+x,-y,+y,-z,+z. */
typedef struct {
    int32_t q;               /* 9 (D2Q9), 19 (D3Q19) or 27 (D3Q27) */
    int32_t n[3];            /* cells per axis; n[2] == 1 in 2D */
    int32_t bc[6];           /* 0 periodic, 1 wall (halfway bounce-back) */
    double wall_u[6][3];     /* wall velocity per face */
    double tau;              /* BGK relaxation time, > 1/2 */
    double rho0;             /* reference density (wall density too) */
    double force[3];         /* body-force density F (Guo) */
    int32_t sensor_kind;     /* 0: L2 ratio, 1: mean |f^neq/f^eq| (Eq. kkn) */
    int32_t block[3];        /* sensor block edge per axis */
    double theta_refine;     /* refine iff M > theta_refine */
    double theta_coarsen;    /* coarsen iff M < theta_coarsen */
    double smagorinsky;      /* Smagorinsky constant C (0: plain BGK) */
    int32_t wall_profile[6]; /* 1: smoothed wall velocity on that face */
} orc_params;

/* ---------------------------------------------------------------------------
 * Velocity sets (Sec. 2.2: discrete velocities xi_i, weights w_i, c_s^2 = 1/3).
 * The velocities are enumerated from {-1,0,1}^d, keeping those whose squared
 * length is allowed by the model; the weight depends on the squared length
 * only.  DdQq tables are the standard ones (Qian, d'Humieres, Lallemand).
 * ------------------------------------------------------------------------- */
static int build_lattice(int q, orc_lattice *L)
{
    int d, maxlen2;
    double wt[4];
    if (q == 9) {
        d = 2; maxlen2 = 2;
        wt[0] = 4.0 / 9.0; wt[1] = 1.0 / 9.0; wt[2] = 1.0 / 36.0; wt[3] = 0.0;
    } else if (q == 19) {
        d = 3; maxlen2 = 2;
        wt[0] = 1.0 / 3.0; wt[1] = 1.0 / 18.0; wt[2] = 1.0 / 36.0; wt[3] = 0.0;
    } else if (q == 27) {
        d = 3; maxlen2 = 3;
        wt[0] = 8.0 / 27.0; wt[1] = 2.0 / 27.0; wt[2] = 1.0 / 54.0; wt[3] = 1.0 / 216.0;
    } else {
        return -1;
    }
    int k = 0;
    int zlo = (d == 3) ? -1 : 0, zhi = (d == 3) ? 1 : 0;
    for (int cz = zlo; cz <= zhi; ++cz)
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                int len2 = cx * cx + cy * cy + cz * cz;
                if (len2 > maxlen2) continue;
                L->c[k][0] = cx; L->c[k][1] = cy; L->c[k][2] = cz;
                L->w[k] = wt[len2];
                ++k;
            }
    if (k != q) return -1;
    for (int i = 0; i < q; ++i) {
        L->opp[i] = -1;
        for (int j = 0; j < q; ++j)
            if (L->c[j][0] == -L->c[i][0] && L->c[j][1] == -L->c[i][1] &&
                L->c[j][2] == -L->c[i][2])
                L->opp[i] = j;
    }
    L->q = q; L->d = d; L->cs2 = 1.0 / 3.0;
    return 0;
}

/* Exported so that the tests can pin the tables against exact identities. */
int orc_lattice_tables(int q, int *c, double *w, int *opp)
{
    orc_lattice L;
    if (build_lattice(q, &L) != 0) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) c[3 * i + a] = L.c[i][a];
        w[i] = L.w[i];
        opp[i] = L.opp[i];
    }
    return L.d;
}

/* ---------------------------------------------------------------------------
 * Equilibrium, Eq. feq_i: f^eq_i = w_i rho (1 + xi_i.u / c_s^2
 *                                          + Q_i : uu / (2 c_s^4)),
 * with Q_i = xi_i xi_i - c_s^2 I, written with the tensor contraction spelled
 * out rather than expanded.
 * ------------------------------------------------------------------------- */
static void equilibrium(const orc_lattice *L, double rho, const double u[3], double *feq)
{
    const double cs2 = L->cs2;
    for (int i = 0; i < L->q; ++i) {
        double xu = 0.0;
        for (int a = 0; a < 3; ++a) xu += L->c[i][a] * u[a];
        double Quu = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double Q = (double)(L->c[i][a] * L->c[i][b]) - (a == b ? cs2 : 0.0);
                Quu += Q * u[a] * u[b];
            }
        feq[i] = L->w[i] * rho * (1.0 + xu / cs2 + Quu / (2.0 * cs2 * cs2));
    }
}

int orc_equilibrium(int q, double rho, const double *u, double *feq)
{
    orc_lattice L;
    if (build_lattice(q, &L) != 0) return -1;
    double uu[3] = {u[0], u[1], u[2]};
    equilibrium(&L, rho, uu, feq);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Moments, Eqs. rho and u: rho = sum_i f_i, rho u = sum_i xi_i f_i, plus
 * half the body force (Guo) on the pre-collision populations.
 * ------------------------------------------------------------------------- */
static void moments(const orc_lattice *L, const double *fc, const double F[3], double half_force_sign,
                    double *rho_out, double u_out[3])
{
    double rho = 0.0, m[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < L->q; ++i) {
        rho += fc[i];
        for (int a = 0; a < 3; ++a) m[a] += L->c[i][a] * fc[i];
    }
    for (int a = 0; a < 3; ++a) u_out[a] = (m[a] + half_force_sign * 0.5 * F[a]) / rho;
    *rho_out = rho;
}

static int64_t ncells(const orc_params *p) { return (int64_t)p->n[0] * p->n[1] * p->n[2]; }

static int check_params(const orc_params *p, orc_lattice *L)
{
    if (build_lattice(p->q, L) != 0) return -1;
    for (int a = 0; a < 3; ++a) if (p->n[a] < 1) return -1;
    if (L->d == 2 && p->n[2] != 1) return -1;
    if (!(p->tau > 0.5)) return -1;
    if (!(p->smagorinsky >= 0.0)) return -1;
    for (int f = 0; f < 6; ++f) if (p->wall_profile[f] != 0 && p->wall_profile[f] != 1) return -1;
    /* a periodic face needs its opposite face to be periodic as well */
    for (int a = 0; a < 3; ++a)
        if ((p->bc[2 * a] == 0) != (p->bc[2 * a + 1] == 0)) return -1;
    return 0;
}

/* f^eq(rho, u) for every cell; rho has one value per cell, u three. */
int orc_equilibrium_field(const orc_params *p, const double *rho, const double *u, double *f)
{
    orc_lattice L;
    if (check_params(p, &L) != 0) return -1;
    const int64_t N = ncells(p);
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < N; ++cell) equilibrium(&L, rho[cell], u + 3 * cell, f + cell * L.q);
    return 0;
}

/* Smoothed wall velocity (the lid profile of the 3D cavity, Sec. 5.1): the
 * face's velocity times prod over the face's in-plane axes a of
 * (1 - s_a^18)^2, s_a = 2 (x_a + 1/2) / n_a - 1 the cell-centre coordinate
 * mapped to (-1, 1), i.e. x/h - 1 on a side of length 2h.  An axis with one
 * cell (the z axis of a 2D grid) has s = 0 and contributes 1. */
static double wall_profile_factor(const orc_params *p, int face, const int *x)
{
    if (!p->wall_profile[face]) return 1.0;
    double g = 1.0;
    for (int a = 0; a < 3; ++a) {
        if (a == face / 2) continue;
        const double s = 2.0 * (x[a] + 0.5) / p->n[a] - 1.0;
        const double t = 1.0 - pow(s, 18.0);
        g *= t * t;
    }
    return g;
}

/* ---------------------------------------------------------------------------
 * Streaming with boundary conditions (push form of the streaming step of
 * Sec. 2.2): every post-collision population S_i(x) moves to x + xi_i.  If
 * x + xi_i leaves the domain through a periodic face it re-enters on the
 * opposite face; if it leaves through a wall face it is reflected back into
 * x as the opposite population (halfway bounce-back), with the moving-wall
 * correction of the moving bounce-back rule,
 *   f_{opp(i)}(x) = S_i(x) - 2 w_i rho_w (xi_i . u_w) / c_s^2 ,
 * u_w the sum of the velocities of the wall faces crossed, each times its
 * profile factor at x (1 unless the face is smoothed).
 * ------------------------------------------------------------------------- */
int orc_stream(const orc_params *p, const double *S, double *f)
{
    orc_lattice L;
    if (check_params(p, &L) != 0) return -1;
    const int q = L.q, nx = p->n[0], ny = p->n[1], nz = p->n[2];
    const int64_t N = ncells(p);
    const double rho_w = p->rho0;
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < N; ++cell) {
        int x[3];
        x[0] = (int)(cell % nx);
        x[1] = (int)((cell / nx) % ny);
        x[2] = (int)(cell / ((int64_t)nx * ny));
        for (int i = 0; i < q; ++i) {
            int t[3];
            int solid = 0;
            double uw[3] = {0.0, 0.0, 0.0};
            for (int a = 0; a < 3; ++a) {
                t[a] = x[a] + L.c[i][a];
                int face = -1;
                if (t[a] < 0) face = 2 * a;
                else if (t[a] >= p->n[a]) face = 2 * a + 1;
                if (face < 0) continue;
                if (p->bc[face] == 0) {
                    t[a] = (t[a] + p->n[a]) % p->n[a];
                } else {
                    solid = 1;
                    const double g = wall_profile_factor(p, face, x);
                    for (int b = 0; b < 3; ++b) uw[b] += g * p->wall_u[face][b];
                }
            }
            const double Si = S[cell * q + i];
            if (solid) {
                double xu = 0.0;
                for (int b = 0; b < 3; ++b) xu += L.c[i][b] * uw[b];
                f[cell * q + L.opp[i]] = Si - 2.0 * L.w[i] * rho_w * xu / L.cs2;
            } else {
                int64_t tc = ((int64_t)t[2] * ny + t[1]) * nx + t[0];
                f[tc * q + i] = Si;
            }
        }
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Cell sensor on the pre-collision populations f (Sec. 3.2).
 *   kind 1: K_Kn = (1/q) sum_i |f^neq_i / f^eq_i|            (Eqs. sensor, kkn)
 *   kind 0: ||f^neq||_2 / ||f^eq||_2
 * with f^eq = f^eq(rho, u) from the moments of f and f^neq = f - f^eq.
 * ------------------------------------------------------------------------- */
static double cell_sensor(const orc_lattice *L, const orc_params *p, const double *fc)
{
    double rho, u[3], feq[ORC_MAXQ];
    moments(L, fc, p->force, +1.0, &rho, u);
    equilibrium(L, rho, u, feq);
    if (p->sensor_kind == 1) {
        double acc = 0.0;
        for (int i = 0; i < L->q; ++i) acc += fabs((fc[i] - feq[i]) / feq[i]);
        return acc / L->q;
    }
    double num = 0.0, den = 0.0;
    for (int i = 0; i < L->q; ++i) {
        double fneq = fc[i] - feq[i];
        num += fneq * fneq;
        den += feq[i] * feq[i];
    }
    return sqrt(num) / sqrt(den);
}

int orc_sensor(const orc_params *p, const double *f, double *s)
{
    orc_lattice L;
    if (check_params(p, &L) != 0) return -1;
    const int64_t N = ncells(p);
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < N; ++cell) s[cell] = cell_sensor(&L, p, f + cell * L.q);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Relaxation time of a cell.  Plain BGK: tau.  With the Smagorinsky model
 * (the subgrid model the paper adds to BGK at high Reynolds number, Sec. 4)
 * the viscosity is c_s^2 (tau_e - 1/2) = c_s^2 (tau - 1/2) + C^2 |S|, with
 * |S| = sqrt(2 S:S) and the strain rate read from the non-equilibrium
 * momentum flux of the cell, Pi = sum_i xi_i xi_i (f_i - f^eq_i) =
 * -2 rho c_s^2 tau_e S.  Then tau_e (tau_e - tau) = C^2 sqrt(2) |Pi| /
 * (2 rho c_s^4), |Pi| = sqrt(Pi:Pi), whose positive root is taken.
 * ------------------------------------------------------------------------- */
static double relaxation_time(const orc_lattice *L, const orc_params *p, const double *fc, const double *feq,
                              double rho)
{
    if (p->smagorinsky == 0.0) return p->tau;
    double Pi[3][3] = {{0.0}};
    for (int i = 0; i < L->q; ++i) {
        const double fneq = fc[i] - feq[i];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Pi[a][b] += L->c[i][a] * L->c[i][b] * fneq;
    }
    double pp = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) pp += Pi[a][b] * Pi[a][b];
    const double C2 = p->smagorinsky * p->smagorinsky;
    const double k = C2 * sqrt(2.0) * sqrt(pp) / (2.0 * rho * L->cs2 * L->cs2);
    return 0.5 * (p->tau + sqrt(p->tau * p->tau + 4.0 * k));
}

/* ---------------------------------------------------------------------------
 * BGK collision (Eq. bgklb): f^out_i = f_i - (f_i - f^eq_i) / tau, plus Guo's
 * forcing term (1 - 1/(2 tau)) w_i [ (xi_i - u)/c_s^2 + (xi_i.u) xi_i / c_s^4 ].F,
 * tau the cell's relaxation time (relaxation_time).
 * ------------------------------------------------------------------------- */
static void collide_cell(const orc_lattice *L, const orc_params *p, const double *fc, double *Sc)
{
    double rho, u[3], feq[ORC_MAXQ];
    moments(L, fc, p->force, +1.0, &rho, u);
    equilibrium(L, rho, u, feq);
    const double tau = relaxation_time(L, p, fc, feq, rho);
    const double cs2 = L->cs2;
    for (int i = 0; i < L->q; ++i) {
        double xu = 0.0;
        for (int a = 0; a < 3; ++a) xu += L->c[i][a] * u[a];
        double src = 0.0;
        for (int a = 0; a < 3; ++a)
            src += ((L->c[i][a] - u[a]) / cs2 + xu * L->c[i][a] / (cs2 * cs2)) * p->force[a];
        src *= L->w[i] * (1.0 - 1.0 / (2.0 * tau));
        Sc[i] = fc[i] - (fc[i] - feq[i]) / tau + src;
    }
}

int orc_collide(const orc_params *p, const double *f, double *S)
{
    orc_lattice L;
    if (check_params(p, &L) != 0) return -1;
    const int64_t N = ncells(p);
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < N; ++cell) collide_cell(&L, p, f + cell * L.q, S + cell * L.q);
    return 0;
}

/* Macroscopic fields; sign = +1 for pre-collision f (u carries +F/2), -1 for
 * the post-collision state S (whose momentum already holds the full F). */
int orc_moments(const orc_params *p, const double *f, double sign, double *rho, double *u)
{
    orc_lattice L;
    if (check_params(p, &L) != 0) return -1;
    const int64_t N = ncells(p);
#pragma omp parallel for schedule(static)
    for (int64_t cell = 0; cell < N; ++cell) {
        double r, uu[3];
        moments(&L, f + cell * L.q, p->force, sign, &r, uu);
        rho[cell] = r;
        for (int a = 0; a < 3; ++a) u[cell * 3 + a] = uu[a];
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Per-block maximum of the cell sensor.  NaN-propagating: any NaN in a block
 * makes its maximum NaN.
 * ------------------------------------------------------------------------- */
int orc_block_max(const orc_params *p, const double *s, double *bmax)
{
    int nb[3];
    for (int a = 0; a < 3; ++a) {
        if (p->block[a] < 1) return -1;
        nb[a] = (p->n[a] + p->block[a] - 1) / p->block[a];
    }
    const int64_t NB = (int64_t)nb[0] * nb[1] * nb[2];
    for (int64_t b = 0; b < NB; ++b) bmax[b] = -INFINITY;
    for (int z = 0; z < p->n[2]; ++z)
        for (int y = 0; y < p->n[1]; ++y)
            for (int x = 0; x < p->n[0]; ++x) {
                int64_t cell = ((int64_t)z * p->n[1] + y) * p->n[0] + x;
                int64_t b = ((int64_t)(z / p->block[2]) * nb[1] + y / p->block[1]) * nb[0] + x / p->block[0];
                double v = s[cell];
                if (isnan(v) || isnan(bmax[b])) bmax[b] = NAN;
                else if (v > bmax[b]) bmax[b] = v;
            }
    return 0;
}

/* Thresholding of the block maxima into refinement decisions. */
int orc_flags(const orc_params *p, const double *bmax, int64_t nblocks, int8_t *flags)
{
    for (int64_t b = 0; b < nblocks; ++b) {
        double m = bmax[b];
        if (!isfinite(m)) flags[b] = 2;
        else if (m > p->theta_refine) flags[b] = 1;
        else if (m < p->theta_coarsen) flags[b] = -1;
        else flags[b] = 0;
    }
    return 0;
}

/* One step: f = T(S); optional sensor on f; S_next = C(f). */
int orc_step(const orc_params *p, const double *S, double *S_next, double *f_work, double *s_cell)
{
    if (orc_stream(p, S, f_work) != 0) return -1;
    if (s_cell && orc_sensor(p, f_work, s_cell) != 0) return -1;
    return orc_collide(p, f_work, S_next);
}

/* n steps k = k0+1 .. k0+n.  The sensor runs when k % sensor_every == 0
 * (sensor_every > 0); the block maxima of each such step are appended to
 * bmax_hist (nblocks values per sensor step) if it is not NULL.
 * S holds S_{k0} on entry and S_{k0+n} on return; work holds 2 more states
 * plus one double per cell. Returns the number of sensor steps done. */
int64_t orc_run(const orc_params *p, double *S, double *work, int64_t k0, int64_t n,
                int32_t sensor_every, double *bmax_hist)
{
    orc_lattice L;
    if (check_params(p, &L) != 0) return -1;
    const int64_t N = ncells(p);
    double *f = work;
    double *S2 = work + N * L.q;
    double *s = work + 2 * N * L.q;
    int nb[3];
    for (int a = 0; a < 3; ++a) nb[a] = (p->n[a] + p->block[a] - 1) / p->block[a];
    const int64_t NB = (int64_t)nb[0] * nb[1] * nb[2];
    int64_t nsens = 0;
    double *cur = S, *next = S2;
    for (int64_t k = k0 + 1; k <= k0 + n; ++k) {
        int sense = sensor_every > 0 && (k % sensor_every) == 0;
        if (orc_step(p, cur, next, f, sense ? s : NULL) != 0) return -1;
        double *t = cur; cur = next; next = t;
        if (sense) {
            if (bmax_hist) orc_block_max(p, s, bmax_hist + nsens * NB);
            ++nsens;
        }
    }
    if (cur != S) memcpy(S, cur, sizeof(double) * N * L.q);
    return nsens;
}

/* Totals of the stored state: sum of rho and of the momentum sum_i xi_i S_i,
 * accumulated in long double, in cell order. */
int orc_conservation(const orc_params *p, const double *S, double *out)
{
    orc_lattice L;
    if (check_params(p, &L) != 0) return -1;
    const int64_t N = ncells(p);
    long double acc[4] = {0, 0, 0, 0};
    for (int64_t cell = 0; cell < N; ++cell)
        for (int i = 0; i < L.q; ++i) {
            double v = S[cell * L.q + i];
            acc[0] += v;
            for (int a = 0; a < 3; ++a) acc[1 + a] += (long double)L.c[i][a] * v;
        }
    for (int a = 0; a < 4; ++a) out[a] = (double)acc[a];
    return 0;
}

/* ---------------------------------------------------------------------------
 * Refinement level map (Sec. 3.4): phi = log2 K and
 *   l = l_min if [a phi] < l_min, l_max if [a phi] > l_max, [a phi] otherwise,
 * with [x] the integral part.  Reading taken here: an offset b is added
 * (l from [a phi + b]) because with a alone the sensor values met in practice
 * (K ~ 1e-3, phi ~ -10) cannot be mapped onto levels >= 0; "integral part" is
 * read as floor.  A non-finite K gives l_max (refine where the sensor is
 * broken); K = 0 gives l_min.  Then the buffer layer of Sec. 5.2: every block
 * takes the maximum level found within `buffer` blocks of it (Chebyshev
 * distance), so refinement spreads one layer (or more) around tagged blocks.
 * ------------------------------------------------------------------------- */
int orc_levels(const orc_params *p, const double *bmax, double a, double b, int lmin, int lmax,
               int buffer, int8_t *levels)
{
    int nb[3];
    for (int k = 0; k < 3; ++k) nb[k] = (p->n[k] + p->block[k] - 1) / p->block[k];
    const int64_t NB = (int64_t)nb[0] * nb[1] * nb[2];
    int8_t *raw = (int8_t *)malloc((size_t)NB);
    if (!raw) return -1;
    for (int64_t i = 0; i < NB; ++i) {
        double K = bmax[i];
        int l;
        if (!isfinite(K)) l = lmax;
        else if (K <= 0.0) l = lmin;
        else {
            double x = floor(a * log2(K) + b);
            l = (x < lmin) ? lmin : (x > lmax) ? lmax : (int)x;
        }
        raw[i] = (int8_t)l;
    }
    for (int z = 0; z < nb[2]; ++z)
        for (int y = 0; y < nb[1]; ++y)
            for (int x = 0; x < nb[0]; ++x) {
                int best = -128;
                for (int dz = -buffer; dz <= buffer; ++dz)
                    for (int dy = -buffer; dy <= buffer; ++dy)
                        for (int dx = -buffer; dx <= buffer; ++dx) {
                            int xx = x + dx, yy = y + dy, zz = z + dz;
                            if (xx < 0 || yy < 0 || zz < 0 || xx >= nb[0] || yy >= nb[1] || zz >= nb[2])
                                continue;
                            int v = raw[((int64_t)zz * nb[1] + yy) * nb[0] + xx];
                            if (v > best) best = v;
                        }
                levels[((int64_t)z * nb[1] + y) * nb[0] + x] = (int8_t)best;
            }
    free(raw);
    return 0;
}

/* Threads of the OpenMP loops (timing the oracle on one core or all). */
int orc_set_threads(int n)
{
    if (n < 1) return -1;
    omp_set_num_threads(n);
    return 0;
}

int orc_max_threads(void) { return omp_get_max_threads(); }
