/*
 * oracle.c -- plain, slow, obviously-correct FP64 CPU reference of the pixelated-LArTPC charge path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header, table or constant generator with the HIP library;
 * the only thing both sides consume in common is the seeded input (segments, parameters, response table).
 *
 * What it computes (arXiv 2212.09807):
 *   1. Recombination, Sec. 3.1, eq. (birks) / eq. (box):  R, Q_0 = E / W_ion, Q_R = R * Q_0.
 *   2. Drift, Sec. 3.2, eq. (drift), eq. (lifetime), sigma = sqrt(2 D t):  evaluated at the segment midpoint.
 *   3. Charge density, Sec. 3.3.2, eq. (rho): N points evenly spaced along the segment (midpoints of N equal
 *      pieces, N = ceil(L / 10 um)), each carrying Q_a / N; the M Gaussian perturbations of each point are
 *      replaced by their M -> infinity expectation ("D-exact"): the probability that the perturbed point
 *      falls in each sub-pixel bin (x, y) and each tick (arrival time), a product of truncated-Gaussian
 *      bin masses (truncated at n_sigma and renormalised).
 *      With mc_draws = M > 0 the paper's own estimator is used instead: each point is moved M times by Philox-keyed
 *      Gaussian draws (truncated at n_sigma) and each moved copy puts Q_a / (N M) into the cell containing it.
 *      With per_point = 1 lifetime and diffusion are evaluated at every sample point's own drift time instead of
 *      the segment midpoint's (charge Q_R / N * exp(-t_mu / tau), widths sqrt(2 D t_mu)).
 *   4. Induced current, Sec. 3.3.2, eq. (current): each charge cell (tick a, bin u, v) adds
 *      q * R[k, i, j] to pixel p at tick a - (T_R - 1) + k, where (i, j) is the bin's mirror-folded offset
 *      from the pixel centre (the table is quadrant-symmetric, Sec. 3.3.1) and the table is arrival-aligned.
 *   5. Per-pixel sum over segments (Sec. 3.4).
 *   6. Electronics, Sec. 3.4: integrate, discriminate (>= threshold), hold, digitise (8-bit ADC), reset,
 *      with reset / discriminator / uncorrelated Gaussian noise drawn from a counter-based Philox4x32-10
 *      generator (Salmon et al., SC'11) through Box-Muller.
 *
 * Readings of points the paper leaves open that change arithmetic here:
 *   - the number of points N is an integer decided by floating point, so it is decided in FP32 exactly as
 *     the device decides it (sqrt / divide / ceil in IEEE single, no contraction);
 *   - arrival time of a point = its interpolated time + |z - z_anode| / v_d;
 *   - ticks outside [0, n_ticks) are dropped and their (signed) contribution is reported as "clipped";
 *     cells outside the pixel grid are reported as "off-grid" charge.
 *
 * Precision: IEEE double everywhere except the FP32 decision of N noted above.  Build with
 * -ffp-contract=off so the FP32 decision is bit-identical to the device's.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <limits.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t recomb_model;
    double e_field, lar_density, w_ion, birks_ab, birks_kb, box_alpha, box_beta;
    double v_drift, lifetime, d_long, d_tran, z_anode, sample_step, n_sigma;
    int32_t mc_draws;       /* 0: expectation over the perturbations (D-exact); M > 0: M random draws per point */
    int32_t per_point;      /* 0: lifetime and diffusion at the segment midpoint; 1: at every sample point */
} orc_physics_params;

/* Key of the Monte Carlo perturbations (used only when mc_draws > 0). */
typedef struct {
    uint64_t seed;          /* Philox key */
    uint64_t event_id;
} orc_mc_key;

typedef struct {
    double pitch;
    int32_t n_x, n_y;
    double x0, y0;
    int32_t n_sub;
    double tick;
    int32_t n_ticks;
    double t_begin;
} orc_readout_params;

typedef struct {
    double threshold;
    int32_t hold_ticks, min_spacing;
    double q_lsb;
    int32_t pedestal, adc_bits;
    double sigma_reset, sigma_disc, sigma_unc;
    int32_t max_packets;
    uint64_t seed;
    int32_t reset_period;
} orc_electronics_params;

typedef struct {
    const float *x0, *y0, *z0, *t0, *x1, *y1, *z1, *t1, *energy, *dedx;
    int64_t n;
} orc_segments;

/* Per-segment results of steps 1-2 (and the point count of step 3). */
typedef struct {
    double length, dedx, recomb, q0, q_r, t_drift, q_a, sigma_t, sigma_time;
    int32_t n_points;
    int32_t flags;          /* bit0: Box factor clamped at 0; bit1: invalid (zero length without dE/dx) */
} orc_seginfo;

#define ORC_FLAG_BOX_CLAMP 1
#define ORC_FLAG_INVALID 2

/* ------------------------------------------------------------------------------------------------
 * Steps 1-2: recombination and drift, one segment.
 * ------------------------------------------------------------------------------------------------ */
static int32_t point_count_fp32(float dx, float dy, float dz, float step)
{
    /* N = max(1, ceil(L / step)) decided in IEEE single precision. */
    volatile float sxx = dx * dx;
    volatile float syy = dy * dy;
    volatile float szz = dz * dz;
    volatile float s2 = sxx + syy;
    volatile float s3 = s2 + szz;
    float L = sqrtf(s3);
    volatile float q = L / step;
    float c = ceilf(q);
    if (!(c >= 1.0f)) return 1;
    if (c > 1.0e8f) c = 1.0e8f;
    return (int32_t)c;
}

static void segment_physics(const orc_physics_params *ph, const orc_segments *sg, int64_t i, orc_seginfo *o)
{
    memset(o, 0, sizeof(*o));
    double dx = (double)sg->x1[i] - sg->x0[i];
    double dy = (double)sg->y1[i] - sg->y0[i];
    double dz = (double)sg->z1[i] - sg->z0[i];
    double L = sqrt(dx * dx + dy * dy + dz * dz);
    double E = sg->energy[i];
    o->length = L;
    if (L > 0.0) {
        o->dedx = E / L;                                   /* dE/dx constant within a segment, Sec. 2 */
    } else if (sg->dedx && !isnan(sg->dedx[i])) {
        o->dedx = sg->dedx[i];
    } else {
        o->flags |= ORC_FLAG_INVALID;
        o->dedx = 0.0;
    }
    double eps = ph->e_field * ph->lar_density;            /* field x density, Sec. 3.1 */
    if (ph->recomb_model == 0) {                           /* Birks, eq. (birks) */
        o->recomb = ph->birks_ab / (1.0 + ph->birks_kb / eps * o->dedx);
    } else {                                               /* modified Box, eq. (box) */
        double xi = ph->box_beta / eps * o->dedx;
        double r = xi > 0.0 ? log(ph->box_alpha + xi) / xi : -INFINITY;
        if (!(r >= 0.0)) { r = 0.0; o->flags |= ORC_FLAG_BOX_CLAMP; }
        o->recomb = r;
    }
    o->q0 = E / ph->w_ion;
    o->q_r = o->recomb * o->q0;
    double zm = 0.5 * ((double)sg->z0[i] + (double)sg->z1[i]);
    o->t_drift = fabs(zm - ph->z_anode) / ph->v_drift;     /* eq. (drift), at the midpoint */
    o->q_a = o->q_r * exp(-o->t_drift / ph->lifetime);     /* eq. (lifetime) */
    o->sigma_t = sqrt(2.0 * ph->d_tran * o->t_drift);      /* transverse, cm */
    o->sigma_time = sqrt(2.0 * ph->d_long * o->t_drift) / ph->v_drift;   /* longitudinal, in us */
    o->n_points = point_count_fp32(sg->x1[i] - sg->x0[i], sg->y1[i] - sg->y0[i], sg->z1[i] - sg->z0[i],
                                   (float)ph->sample_step);
    if (ph->per_point) {                                   /* collected charge = sum over the points' charges */
        double qa = 0.0;
        for (int32_t mu = 0; mu < o->n_points; ++mu) {
            double s = ((double)mu + 0.5) / (double)o->n_points;
            double pz = sg->z0[i] + s * ((double)sg->z1[i] - sg->z0[i]);
            qa += o->q_r / o->n_points * exp(-fabs(pz - ph->z_anode) / ph->v_drift / ph->lifetime);
        }
        o->q_a = qa;
    }
}

/* ------------------------------------------------------------------------------------------------
 * Step 3: truncated-Gaussian bin masses.
 * ------------------------------------------------------------------------------------------------ */
/* Phi(b) - Phi(a) for a <= b, using erfc on the side away from the mean to avoid cancellation. */
static double phi_diff(double a, double b)
{
    const double r = 0.70710678118654752440;
    if (a >= 0.0) return 0.5 * (erfc(a * r) - erfc(b * r));
    if (b <= 0.0) return 0.5 * (erfc(-b * r) - erfc(-a * r));
    return 1.0 - 0.5 * erfc(b * r) - 0.5 * erfc(-a * r);
}

/* P(mean + sigma * g in [lo, hi)) with g ~ N(0,1) truncated to |g| <= nsig and renormalised.
 * sigma == 0: the point mass lies in the half-open bin that contains the mean. */
static double tn_mass(double mean, double sigma, double nsig, double lo, double hi)
{
    if (sigma <= 0.0) return (mean >= lo && mean < hi) ? 1.0 : 0.0;
    double za = (lo - mean) / sigma, zb = (hi - mean) / sigma;
    if (za < -nsig) za = -nsig;
    if (zb > nsig) zb = nsig;
    if (za >= zb) return 0.0;
    return phi_diff(za, zb) / phi_diff(-nsig, nsig);
}

/* Index range [k_lo, k_hi] of the bins (edges origin + k * width) that the truncated cloud can touch. */
static void support(double mean, double sigma, double nsig, double origin, double width, int64_t *k_lo, int64_t *k_hi)
{
    if (sigma <= 0.0) {
        int64_t k = (int64_t)floor((mean - origin) / width);
        *k_lo = *k_hi = k;
        return;
    }
    *k_lo = (int64_t)floor((mean - nsig * sigma - origin) / width);
    *k_hi = (int64_t)floor((mean + nsig * sigma - origin) / width);
}

/* Points of a segment: position (x, y) and arrival time. */
static void point_at(const orc_physics_params *ph, const orc_segments *sg, int64_t i, int32_t n, int32_t mu,
                     double *x, double *y, double *tarr)
{
    double s = ((double)mu + 0.5) / (double)n;
    double px = sg->x0[i] + s * ((double)sg->x1[i] - sg->x0[i]);
    double py = sg->y0[i] + s * ((double)sg->y1[i] - sg->y0[i]);
    double pz = sg->z0[i] + s * ((double)sg->z1[i] - sg->z0[i]);
    double pt = sg->t0[i] + s * ((double)sg->t1[i] - sg->t0[i]);
    *x = px;
    *y = py;
    *tarr = pt + fabs(pz - ph->z_anode) / ph->v_drift;
}

/* Drift of sample point mu: its charge (lifetime applied at the point's own drift time) and its cloud widths.
 * With per_point == 0 every point takes the segment midpoint's values. */
static void point_drift(const orc_physics_params *ph, const orc_segments *sg, int64_t i, const orc_seginfo *si,
                        int32_t mu, double *q, double *sig_t, double *sig_time)
{
    if (!ph->per_point) {
        *q = si->q_a / si->n_points;
        *sig_t = si->sigma_t;
        *sig_time = si->sigma_time;
        return;
    }
    double s = ((double)mu + 0.5) / (double)si->n_points;
    double pz = sg->z0[i] + s * ((double)sg->z1[i] - sg->z0[i]);
    double td = fabs(pz - ph->z_anode) / ph->v_drift;                  /* eq. (drift) at the point */
    *q = si->q_r / si->n_points * exp(-td / ph->lifetime);             /* eq. (lifetime) at the point */
    *sig_t = sqrt(2.0 * ph->d_tran * td);
    *sig_time = sqrt(2.0 * ph->d_long * td) / ph->v_drift;
}

typedef struct {
    int64_t a0, na, u0, nu, v0, nv;   /* box: ticks [a0, a0+na), bins [u0, u0+nu) x [v0, v0+nv) */
    double *c;                        /* c[((a-a0)*nu + (u-u0))*nv + (v-v0)] */
} orc_cells;

static void segment_box(const orc_physics_params *ph, const orc_readout_params *ro, const orc_segments *sg, int64_t i,
                        const orc_seginfo *si, orc_cells *cb)
{
    double b = ro->pitch / ro->n_sub;
    int64_t ulo = INT64_MAX, uhi = INT64_MIN, vlo = INT64_MAX, vhi = INT64_MIN, alo = INT64_MAX, ahi = INT64_MIN;
    for (int32_t mu = 0; mu < si->n_points; ++mu) {
        double x, y, t, q, st, stime;
        int64_t lo, hi;
        point_at(ph, sg, i, si->n_points, mu, &x, &y, &t);
        point_drift(ph, sg, i, si, mu, &q, &st, &stime);
        support(x, st, ph->n_sigma, ro->x0, b, &lo, &hi);
        if (lo < ulo) ulo = lo;
        if (hi > uhi) uhi = hi;
        support(y, st, ph->n_sigma, ro->y0, b, &lo, &hi);
        if (lo < vlo) vlo = lo;
        if (hi > vhi) vhi = hi;
        support(t, stime, ph->n_sigma, ro->t_begin, ro->tick, &lo, &hi);
        if (lo < alo) alo = lo;
        if (hi > ahi) ahi = hi;
    }
    cb->a0 = alo; cb->na = ahi - alo + 1;
    cb->u0 = ulo; cb->nu = uhi - ulo + 1;
    cb->v0 = vlo; cb->nv = vhi - vlo + 1;
    cb->c = NULL;
}

/* c[a,u,v] = sum over points of q * Fx[u] * Fy[v] * Ft[a]  (expectation of eq. (rho) on the grid). */
static int segment_cells(const orc_physics_params *ph, const orc_readout_params *ro, const orc_segments *sg, int64_t i,
                         const orc_seginfo *si, orc_cells *cb)
{
    segment_box(ph, ro, sg, i, si, cb);
    size_t ncell = (size_t)(cb->na * cb->nu * cb->nv);
    cb->c = (double *)calloc(ncell ? ncell : 1, sizeof(double));
    if (!cb->c) return -1;
    double b = ro->pitch / ro->n_sub;
    double *fx = (double *)malloc(sizeof(double) * (size_t)(cb->nu + cb->nv + cb->na));
    if (!fx) return -1;
    double *fy = fx + cb->nu, *ft = fy + cb->nv;
    for (int32_t mu = 0; mu < si->n_points; ++mu) {
        double x, y, t, q, st, stime;
        point_at(ph, sg, i, si->n_points, mu, &x, &y, &t);
        point_drift(ph, sg, i, si, mu, &q, &st, &stime);
        for (int64_t u = 0; u < cb->nu; ++u) {
            double lo = ro->x0 + (double)(cb->u0 + u) * b;
            fx[u] = tn_mass(x, st, ph->n_sigma, lo, lo + b);
        }
        for (int64_t v = 0; v < cb->nv; ++v) {
            double lo = ro->y0 + (double)(cb->v0 + v) * b;
            fy[v] = tn_mass(y, st, ph->n_sigma, lo, lo + b);
        }
        for (int64_t a = 0; a < cb->na; ++a) {
            double lo = ro->t_begin + (double)(cb->a0 + a) * ro->tick;
            ft[a] = tn_mass(t, stime, ph->n_sigma, lo, lo + ro->tick);
        }
        for (int64_t a = 0; a < cb->na; ++a) {
            if (ft[a] == 0.0) continue;
            for (int64_t u = 0; u < cb->nu; ++u) {
                double w = q * ft[a] * fx[u];
                if (w == 0.0) continue;
                double *row = cb->c + (a * cb->nu + u) * cb->nv;
                for (int64_t v = 0; v < cb->nv; ++v) row[v] += w * fy[v];
            }
        }
    }
    free(fx);
    return 0;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* Four standard normals from one Philox block: Box-Muller on words (0, 1) gives g[0] (cosine branch) and g[1]
 * (sine branch), on words (2, 3) g[2] and g[3]; each word x maps to u = (x + 1/2) 2^-32 in (0, 1). */
static void philox_normals(const uint32_t ctr[4], const uint32_t key[2], double g[4])
{
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const double two_m32 = 2.3283064365386963e-10, two_pi = 6.283185307179586477;
    for (int h = 0; h < 2; ++h) {
        double u0 = ((double)x[2 * h] + 0.5) * two_m32;
        double u1 = ((double)x[2 * h + 1] + 0.5) * two_m32;
        double r = sqrt(-2.0 * log(u0));
        g[2 * h] = r * cos(two_pi * u1);
        g[2 * h + 1] = r * sin(two_pi * u1);
    }
}

#define ORC_MC_TRIES 9

/* Perturbation of draw (mu, m) of segment seg: normals (g_x, g_y, g_t) from the cosine and sine branches of words
 * (0, 1) and the cosine branch of words (2, 3).  Each is a standard normal truncated to |g| <= nsig: a component
 * outside is replaced by the same component of the next try (try r uses stream 3 + r; a component with no accepted
 * value after nine tries, probability below 1e-50 at nsig >= 1, is set to 0).  Counter of try r:
 * (seg, mu * M + m, event id low word, (event id high word << 4) | (3 + r)). */
static void mc_perturbation(const orc_mc_key *k, double nsig, uint32_t seg, uint32_t draw, double g[3])
{
    const uint32_t key[2] = {(uint32_t)k->seed, (uint32_t)(k->seed >> 32)};
    int have[3] = {0, 0, 0};
    g[0] = g[1] = g[2] = 0.0;
    for (uint32_t r = 0; r < ORC_MC_TRIES && !(have[0] && have[1] && have[2]); ++r) {
        const uint32_t ctr[4] = {seg, draw, (uint32_t)k->event_id,
                                 (uint32_t)((k->event_id >> 32) << 4) | ((3u + r) & 15u)};
        double gg[4];
        philox_normals(ctr, key, gg);
        for (int a = 0; a < 3; ++a)
            if (!have[a] && fabs(gg[a]) <= nsig) { g[a] = gg[a]; have[a] = 1; }
    }
}

/* Draws that land within a small margin of a sub-pixel or tick edge (1e-5 of the bin) are those whose cell an FP32
 * evaluation of the same position may legitimately decide differently; their (u, v) bins are recorded so a
 * comparison can flag the pixels in their reach.  The record is cleared by orc_mc_clear_near_edges. */
#define ORC_NEAR_CAP 65536
static int64_t g_near_n = 0;
static int32_t g_near_uv[2 * ORC_NEAR_CAP];

static int near_edge(double y, double origin, double width)
{
    double f = (y - origin) / width;
    double d = f - floor(f);
    return d < 1e-5 || d > 1.0 - 1e-5;
}

void orc_mc_clear_near_edges(void) { g_near_n = 0; }

/* Number of near-edge draws recorded since the last clear; copies up to cap (u, v) pairs to uv. */
int64_t orc_mc_near_edges(int32_t *uv, int64_t cap)
{
    int64_t n = g_near_n < ORC_NEAR_CAP ? g_near_n : ORC_NEAR_CAP;
    for (int64_t k = 0; k < n && k < cap; ++k) { uv[2 * k] = g_near_uv[2 * k]; uv[2 * k + 1] = g_near_uv[2 * k + 1]; }
    return g_near_n;
}

/* The paper's estimator of the charge density (eq. (rho)): every point is moved M times by a random 3-D Gaussian
 * perturbation (transverse sigma_T in x and y, longitudinal sigma_L / v_d in arrival time) and each moved copy
 * carries q / M into the cell (tick, sub-pixel bin) that contains it.  Cells are integer hit counts times q / M. */
static int segment_cells_mc(const orc_physics_params *ph, const orc_readout_params *ro, const orc_segments *sg,
                            int64_t i, const orc_seginfo *si, const orc_mc_key *key, orc_cells *cb)
{
    segment_box(ph, ro, sg, i, si, cb);
    size_t ncell = (size_t)(cb->na * cb->nu * cb->nv);
    int64_t *hits = (int64_t *)calloc(ncell ? ncell : 1, sizeof(int64_t));
    cb->c = (double *)calloc(ncell ? ncell : 1, sizeof(double));
    if (!hits || !cb->c) return -1;
    const double b = ro->pitch / ro->n_sub;
    const int32_t M = ph->mc_draws;
    for (int32_t mu = 0; mu < si->n_points; ++mu) {
        double x, y, t;
        point_at(ph, sg, i, si->n_points, mu, &x, &y, &t);
        for (int32_t m = 0; m < M; ++m) {
            double g[3];
            mc_perturbation(key, ph->n_sigma, (uint32_t)i, (uint32_t)((int64_t)mu * M + m), g);
            int64_t u = (int64_t)floor((x + si->sigma_t * g[0] - ro->x0) / b);
            int64_t v = (int64_t)floor((y + si->sigma_t * g[1] - ro->y0) / b);
            int64_t a = (int64_t)floor((t + si->sigma_time * g[2] - ro->t_begin) / ro->tick);
            if (near_edge(x + si->sigma_t * g[0], ro->x0, b) || near_edge(y + si->sigma_t * g[1], ro->y0, b) ||
                near_edge(t + si->sigma_time * g[2], ro->t_begin, ro->tick)) {
#pragma omp critical(orc_near)
                {
                    if (g_near_n < ORC_NEAR_CAP) {
                        g_near_uv[2 * g_near_n] = (int32_t)u;
                        g_near_uv[2 * g_near_n + 1] = (int32_t)v;
                    }
                    ++g_near_n;
                }
            }
            if (u < cb->u0 || u >= cb->u0 + cb->nu || v < cb->v0 || v >= cb->v0 + cb->nv || a < cb->a0 ||
                a >= cb->a0 + cb->na) {
                free(hits);
                return -4;                        /* cannot happen: the box holds the truncated cloud */
            }
            hits[((a - cb->a0) * cb->nu + (u - cb->u0)) * cb->nv + (v - cb->v0)] += 1;
        }
    }
    const double w = si->q_a / si->n_points / M;
    for (size_t c = 0; c < ncell; ++c) cb->c[c] = (double)hits[c] * w;
    free(hits);
    return 0;
}

/* cells of one segment by the estimator the parameters select */
static int cells_of(const orc_physics_params *ph, const orc_readout_params *ro, const orc_segments *sg, int64_t i,
                    const orc_seginfo *si, const orc_mc_key *key, orc_cells *cb)
{
    if (ph->mc_draws > 0 && ph->per_point) return -5;     /* the Monte Carlo form uses the midpoint drift */
    if (ph->mc_draws > 0) return key ? segment_cells_mc(ph, ro, sg, i, si, key, cb) : -3;
    return segment_cells(ph, ro, sg, i, si, cb);
}

/* mirror fold of a bin offset k from the pixel centre: k >= 0 -> k, k < 0 -> -k-1 */
static inline int64_t fold(int64_t k) { return k >= 0 ? k : -k - 1; }

/* ------------------------------------------------------------------------------------------------
 * Public API
 * ------------------------------------------------------------------------------------------------ */

/* Steps 1-2 for every segment. out: n x 9 doubles (length, dedx, R, Q0, Q_R, t_drift, Q_a, sigma_T,
 * sigma_t[us]); n_points[n]; flags[n]. */
int orc_quench_drift(const orc_physics_params *ph, const orc_segments *sg, double *out, int32_t *n_points, int32_t *flags)
{
    for (int64_t i = 0; i < sg->n; ++i) {
        orc_seginfo si;
        segment_physics(ph, sg, i, &si);
        double *o = out + 9 * i;
        o[0] = si.length; o[1] = si.dedx; o[2] = si.recomb; o[3] = si.q0; o[4] = si.q_r;
        o[5] = si.t_drift; o[6] = si.q_a; o[7] = si.sigma_t; o[8] = si.sigma_time;
        n_points[i] = si.n_points;
        flags[i] = si.flags;
    }
    return 0;
}

/* Truncated-Gaussian masses of nk consecutive bins [origin + k*width, origin + (k+1)*width), k = k0.. */
void orc_bin_masses(double mean, double sigma, double nsig, double origin, double width, int64_t k0, int64_t nk,
                    double *out)
{
    for (int64_t k = 0; k < nk; ++k) {
        double lo = origin + (double)(k0 + k) * width;
        out[k] = tn_mass(mean, sigma, nsig, lo, lo + width);
    }
}

/* Charge cells of one segment (index i of the event's segments).  box[6] = a0, na, u0, nu, v0, nv.  If cells == NULL
 * only the box is returned; otherwise cells must hold na*nu*nv doubles (layout [a][u][v]).  key: Monte Carlo key,
 * required when ph->mc_draws > 0 (else -3). */
int orc_segment_cells(const orc_physics_params *ph, const orc_readout_params *ro, const orc_segments *sg, int64_t i,
                      const orc_mc_key *key, int64_t *box, double *cells)
{
    orc_seginfo si;
    segment_physics(ph, sg, i, &si);
    if (si.flags & ORC_FLAG_INVALID) return -2;
    orc_cells cb;
    if (!cells) {
        segment_box(ph, ro, sg, i, &si, &cb);
    } else {
        int rc = cells_of(ph, ro, sg, i, &si, key, &cb);
        if (rc) return rc;
        memcpy(cells, cb.c, sizeof(double) * (size_t)(cb.na * cb.nu * cb.nv));
        free(cb.c);
    }
    box[0] = cb.a0; box[1] = cb.na; box[2] = cb.u0; box[3] = cb.nu; box[4] = cb.v0; box[5] = cb.nv;
    return 0;
}

/* pixel range of the grid whose reach (|bin offset| < B from the pixel centre) meets a cell box */
static void box_pixels(const orc_readout_params *ro, int32_t bx, int32_t by, const orc_cells *cb,
                       int64_t *ix0, int64_t *ix1, int64_t *iy0, int64_t *iy1)
{
    int64_t ns = ro->n_sub, h = ro->n_sub / 2;
    /* pixel ix reaches cells u in [ix*ns + h - bx, ix*ns + h + bx - 1] */
    int64_t ulo = cb->u0, uhi = cb->u0 + cb->nu - 1, vlo = cb->v0, vhi = cb->v0 + cb->nv - 1;
    int64_t a = ulo - h - bx + 1, bb = uhi - h + bx;           /* ix*ns in [a, bb] */
    *ix0 = (a >= 0) ? (a + ns - 1) / ns : -((-a) / ns);
    *ix1 = (bb >= 0) ? bb / ns : -((-bb + ns - 1) / ns);
    a = vlo - h - by + 1; bb = vhi - h + by;
    *iy0 = (a >= 0) ? (a + ns - 1) / ns : -((-a) / ns);
    *iy1 = (bb >= 0) ? bb / ns : -((-bb + ns - 1) / ns);
    if (*ix0 < 0) *ix0 = 0;
    if (*iy0 < 0) *iy0 = 0;
    if (*ix1 > ro->n_x - 1) *ix1 = ro->n_x - 1;
    if (*iy1 > ro->n_y - 1) *iy1 = ro->n_y - 1;
}

/* Sorted list of in-grid pixels (tile-local id iy*n_x + ix) that some segment's charge box reaches.
 * Returns the count; writes at most cap ids into out (out may be NULL). */
int64_t orc_active_pixels(const orc_physics_params *ph, const orc_readout_params *ro, int32_t t_r, int32_t bx, int32_t by,
                          const orc_segments *sg, int32_t *out, int64_t cap)
{
    (void)t_r;
    int64_t npx = (int64_t)ro->n_x * ro->n_y;
    uint8_t *mark = (uint8_t *)calloc((size_t)npx, 1);
    if (!mark) return -1;
    for (int64_t i = 0; i < sg->n; ++i) {
        orc_seginfo si;
        segment_physics(ph, sg, i, &si);
        if (si.flags & ORC_FLAG_INVALID) continue;
        orc_cells cb;
        segment_box(ph, ro, sg, i, &si, &cb);
        int64_t ix0, ix1, iy0, iy1;
        box_pixels(ro, bx, by, &cb, &ix0, &ix1, &iy0, &iy1);
        for (int64_t iy = iy0; iy <= iy1; ++iy)
            for (int64_t ix = ix0; ix <= ix1; ++ix) mark[iy * ro->n_x + ix] = 1;
    }
    int64_t cnt = 0;
    for (int64_t p = 0; p < npx; ++p)
        if (mark[p]) {
            if (out && cnt < cap) out[cnt] = (int32_t)p;
            ++cnt;
        }
    free(mark);
    return cnt;
}

/*
 * Steps 3-5: waveforms I[p, n] (n in [0, n_ticks)) for the listed pixels, in FP64.
 *   table: FP32 [t_r][bx][by] exactly as given to the device.
 *   wave:  n_pix * n_ticks doubles (output).
 *   clipped: per listed pixel, the summed contribution that fell outside [0, n_ticks) (output, may be NULL).
 *   seg_sums (may be NULL): 3 doubles: sum Q_R, sum Q_a, off-grid charge (cells outside the pixel grid).
 *   key: Monte Carlo key (event id, seed), required when ph->mc_draws > 0.
 * Returns 0, or -2 if a segment is invalid, -1 on allocation failure or a missing key.
 */
/* The induction loop dominates the oracle's run time; it is also compiled for AVX2 and picked at load time when the
   host has it (the same IEEE double operations in the same order either way, no contraction). */
__attribute__((target_clones("avx2", "default")))
int orc_waveforms(const orc_physics_params *ph, const orc_readout_params *ro, const float *table, int32_t t_r, int32_t bx,
                  int32_t by, const orc_segments *sg, const int32_t *pixels, int64_t n_pix, double *wave,
                  double *clipped, double *seg_sums, const orc_mc_key *key)
{
    int64_t nseg = sg->n;
    int64_t nt = ro->n_ticks;
    orc_seginfo *si = (orc_seginfo *)malloc(sizeof(orc_seginfo) * (size_t)(nseg ? nseg : 1));
    orc_cells *cb = (orc_cells *)calloc((size_t)(nseg ? nseg : 1), sizeof(orc_cells));
    int64_t *prng = (int64_t *)malloc(sizeof(int64_t) * 4 * (size_t)(nseg ? nseg : 1));
    uint8_t *need = (uint8_t *)calloc((size_t)(nseg ? nseg : 1), 1);
    double *tab = (double *)malloc(sizeof(double) * (size_t)t_r * bx * by);
    if (!si || !cb || !prng || !need || !tab) return -1;
    /* table in [i][j][k] order, same values in double */
    for (int64_t k = 0; k < t_r; ++k)
        for (int64_t i = 0; i < bx; ++i)
            for (int64_t j = 0; j < by; ++j)
                tab[(i * by + j) * t_r + k] = (double)table[(k * bx + i) * by + j];

    int bad = 0;
    for (int64_t s = 0; s < nseg; ++s) {
        segment_physics(ph, sg, s, &si[s]);
        if (si[s].flags & ORC_FLAG_INVALID) bad = 1;
    }
    if (bad) { free(si); free(cb); free(prng); free(need); free(tab); return -2; }

    /* which segments reach the listed pixels */
    for (int64_t s = 0; s < nseg; ++s) {
        segment_box(ph, ro, sg, s, &si[s], &cb[s]);
        box_pixels(ro, bx, by, &cb[s], &prng[4 * s], &prng[4 * s + 1], &prng[4 * s + 2], &prng[4 * s + 3]);
    }
    for (int64_t q = 0; q < n_pix; ++q) {
        int64_t ix = pixels[q] % ro->n_x, iy = pixels[q] / ro->n_x;
        for (int64_t s = 0; s < nseg; ++s)
            if (ix >= prng[4 * s] && ix <= prng[4 * s + 1] && iy >= prng[4 * s + 2] && iy <= prng[4 * s + 3])
                need[s] = 1;
    }
    int err = 0;
    if (seg_sums) {
        for (int64_t s = 0; s < nseg; ++s) need[s] = 1;
    }
#pragma omp parallel for schedule(dynamic, 1) reduction(| : err)
    for (int64_t s = 0; s < nseg; ++s)
        if (need[s] && cells_of(ph, ro, sg, s, &si[s], key, &cb[s])) err = 1;
    if (err) return -1;

    if (seg_sums) {
        double qr = 0.0, qa = 0.0, off = 0.0;
        int64_t ugrid = (int64_t)ro->n_x * ro->n_sub, vgrid = (int64_t)ro->n_y * ro->n_sub;
        for (int64_t s = 0; s < nseg; ++s) {
            qr += si[s].q_r;
            qa += si[s].q_a;
            for (int64_t a = 0; a < cb[s].na; ++a)
                for (int64_t u = 0; u < cb[s].nu; ++u)
                    for (int64_t v = 0; v < cb[s].nv; ++v) {
                        int64_t uu = cb[s].u0 + u, vv = cb[s].v0 + v;
                        if (uu < 0 || uu >= ugrid || vv < 0 || vv >= vgrid)
                            off += cb[s].c[(a * cb[s].nu + u) * cb[s].nv + v];
                    }
        }
        seg_sums[0] = qr; seg_sums[1] = qa; seg_sums[2] = off;
    }

    int64_t h = ro->n_sub / 2;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_pix; ++q) {
        double *w = wave + q * nt;
        double clip = 0.0;
        memset(w, 0, sizeof(double) * (size_t)nt);
        int64_t ix = pixels[q] % ro->n_x, iy = pixels[q] / ro->n_x;
        int64_t uc = ix * ro->n_sub + h, vc = iy * ro->n_sub + h;
        for (int64_t s = 0; s < nseg; ++s) {              /* fixed segment order */
            if (!(ix >= prng[4 * s] && ix <= prng[4 * s + 1] && iy >= prng[4 * s + 2] && iy <= prng[4 * s + 3]))
                continue;
            const orc_cells *c = &cb[s];
            for (int64_t u = 0; u < c->nu; ++u) {
                int64_t i = fold(c->u0 + u - uc);
                if (i >= bx) continue;
                for (int64_t v = 0; v < c->nv; ++v) {
                    int64_t j = fold(c->v0 + v - vc);
                    if (j >= by) continue;
                    const double *col = tab + (i * by + j) * t_r;
                    for (int64_t a = 0; a < c->na; ++a) {
                        double cv = c->c[(a * c->nu + u) * c->nv + v];
                        if (cv == 0.0) continue;
                        int64_t n0 = c->a0 + a - (t_r - 1);     /* tick of table entry k = 0 */
                        /* entries k < k_lo land before tick 0 and k >= k_hi after the window: their products go to
                           the clipped charge, in ascending k as in one pass over the column */
                        int64_t k_lo = n0 < 0 ? -n0 : 0, k_hi = nt - n0;
                        if (k_lo > t_r) k_lo = t_r;
                        if (k_hi > t_r) k_hi = t_r;
                        if (k_hi < k_lo) k_hi = k_lo;
                        for (int64_t k = 0; k < k_lo; ++k) clip += cv * col[k];
                        for (int64_t k = k_lo; k < k_hi; ++k) w[n0 + k] += cv * col[k];
                        for (int64_t k = k_hi; k < t_r; ++k) clip += cv * col[k];
                    }
                }
            }
        }
        if (clipped) clipped[q] = clip;
    }
    for (int64_t s = 0; s < nseg; ++s) free(cb[s].c);
    free(si); free(cb); free(prng); free(need); free(tab);
    return 0;
}

/* ------------------------------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11), written from its published description:
 * ten rounds of two 32x32->64 multiplies with the round constants, the key bumped by the Weyl
 * increments between rounds.
 * ------------------------------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; ++r) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

enum { ORC_STREAM_DISC = 0, ORC_STREAM_RESET = 1, ORC_STREAM_SAMPLE = 2, ORC_STREAM_MC = 3 };
#define ORC_TICK_INITIAL 0xFFFFFFFFu

/* Standard normal for (pixel, tick, event, stream): Box-Muller on the first two words, in FP64. */
double orc_noise_normal(uint64_t seed, uint32_t pixel, uint32_t tick, uint64_t event_id, uint32_t stream)
{
    uint32_t ctr[4] = {pixel, tick, (uint32_t)event_id, (uint32_t)((event_id >> 32) << 4) | (stream & 15u)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    const double two_m32 = 2.3283064365386963e-10;
    double u0 = ((double)x[0] + 0.5) * two_m32;
    double u1 = ((double)x[1] + 0.5) * two_m32;
    return sqrt(-2.0 * log(u0)) * cos(6.283185307179586477 * u1);
}

/*
 * Step 6: electronics for n_pix pixels (tile-local ids), FP64 arithmetic.
 *   wave: n_pix x n_ticks input currents (electrons per tick).
 *   Per pixel up to el->max_packets packets: tick, adc, flag.  flag bit0: the ADC value lies within eps of
 *   an LSB boundary; bit1: an earlier (or this) discriminator decision of this pixel lay within eps of the
 *   threshold, so this packet's timing may legitimately differ from a finite-precision evaluation.
 *   eps = eps_abs + eps_rel * (running sum of |I| since the last reset + threshold).
 *   counts[n_pix]: packets emitted (capped); stats[3] += (samples dropped past the window, packets over
 *   the cap, decisions flagged); uncertain_from[n_pix] (may be NULL): first tick at which a threshold
 *   decision lay within eps, INT32_MAX if none.
 */
int orc_electronics(const orc_electronics_params *el, const orc_readout_params *ro, uint64_t event_id, int64_t n_pix,
                    const int32_t *pixels, const double *wave, double eps_rel, double eps_abs,
                    int32_t *pkt_tick, int32_t *pkt_adc, int32_t *pkt_flag, int32_t *counts, int64_t *stats,
                    int32_t *uncertain_from)
{
    int64_t nt = ro->n_ticks;
    int64_t dropped = 0, over = 0, nflag = 0;
    const int32_t adc_max = (1 << el->adc_bits) - 1;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : dropped, over, nflag)
    for (int64_t q = 0; q < n_pix; ++q) {
        uint32_t pid = (uint32_t)pixels[q];
        const double *w = wave + q * nt;
        double Q = 0.0, absum = 0.0;
        if (el->sigma_reset > 0.0)
            Q = el->sigma_reset * orc_noise_normal(el->seed, pid, ORC_TICK_INITIAL, event_id, ORC_STREAM_RESET);
        int pending = 0, uncertain = 0;
        int64_t ns = 0, ready = 0, last_s = INT64_MIN / 4;
        int32_t cnt = 0;
        int32_t ufrom = INT32_MAX;
        for (int64_t n = 0; n < nt; ++n) {
            /* periodic reset (Sec. 3.4): at every multiple of the period, a pixel without a pending sample
             * discards its integrated charge before this tick's charge arrives */
            if (el->reset_period > 0 && n > 0 && n % el->reset_period == 0 && !pending) {
                Q = 0.0;
                if (el->sigma_reset > 0.0)
                    Q = el->sigma_reset * orc_noise_normal(el->seed, pid, (uint32_t)n, event_id, ORC_STREAM_RESET);
                absum = 0.0;
            }
            Q += w[n];
            absum += fabs(w[n]);
            if (!pending && n >= ready) {
                double disc = 0.0;
                if (el->sigma_disc > 0.0)
                    disc = el->sigma_disc * orc_noise_normal(el->seed, pid, (uint32_t)n, event_id, ORC_STREAM_DISC);
                double m = Q + disc - el->threshold;
                double eps = eps_abs + eps_rel * (absum + fabs(Q) + el->threshold);
                if (fabs(m) < eps) {
                    if (!uncertain) { ++nflag; ufrom = (int32_t)n; }
                    uncertain = 1;
                }
                if (m >= 0.0) {
                    pending = 1;
                    ns = n + el->hold_ticks;
                    if (last_s + el->min_spacing > ns) ns = last_s + el->min_spacing;
                    if (ns >= nt) { ++dropped; break; }
                }
            }
            if (pending && n == ns) {
                double qs = Q;
                if (el->sigma_unc > 0.0)
                    qs += el->sigma_unc * orc_noise_normal(el->seed, pid, (uint32_t)n, event_id, ORC_STREAM_SAMPLE);
                double x = qs / el->q_lsb;
                double fl = floor(x);
                int64_t code = (int64_t)fl + el->pedestal;
                if (code < 0) code = 0;
                if (code > adc_max) code = adc_max;
                double eps = eps_abs + eps_rel * (absum + fabs(qs) + el->threshold);
                int32_t flag = uncertain ? 2 : 0;
                double dist = (x - fl) * el->q_lsb;
                double dist2 = el->q_lsb - dist;
                if (dist < eps || dist2 < eps) flag |= 1;
                if (cnt < el->max_packets) {
                    int64_t o = q * el->max_packets + cnt;
                    pkt_tick[o] = (int32_t)n;
                    pkt_adc[o] = (int32_t)code;
                    pkt_flag[o] = flag;
                    ++cnt;
                } else {
                    ++over;
                }
                Q = 0.0;
                if (el->sigma_reset > 0.0)
                    Q = el->sigma_reset * orc_noise_normal(el->seed, pid, (uint32_t)n, event_id, ORC_STREAM_RESET);
                absum = 0.0;
                pending = 0;
                ready = n + 1;
                last_s = n;
            }
        }
        counts[q] = cnt;
        if (uncertain_from) uncertain_from[q] = ufrom;
    }
    stats[0] += dropped;
    stats[1] += over;
    stats[2] += nflag;
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Number of OpenMP threads of later calls (timing of the oracle alone; no effect on its results). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ================================================================================================
 * Light simulation, Sec. 4 (on given photocurrents; the visibility table is an input of the caller).
 * ================================================================================================ */
typedef struct {
    double tick;            /* ns per light tick */
    double tau_p, tau_s;    /* ns: prompt and slow scintillation decay times */
    double f_prompt;        /* fraction of the light in the prompt component */
    double trunc;           /* the scintillation kernel is truncated after trunc * tau_s */
    double gain;            /* ADC counts per photoelectron */
    double normal_above;    /* expected p.e. per tick above which the normal approximation replaces Poisson */
    int32_t n_det, n_ticks;
    uint64_t seed;
} orc_light_params;

#define ORC_STREAM_LIGHT_PE 12u
#define ORC_STREAM_LIGHT_NOISE 13u

/* Number of taps of the truncated scintillation kernel: lags 0 .. trunc * tau_s / tick. */
int32_t orc_light_taps(const orc_light_params *lp)
{
    return (int32_t)floor(lp->trunc * lp->tau_s / lp->tick) + 1;
}

/* Expected photoelectrons per tick after scintillation (Sec. 4.2, the truncated direct convolution):
 * mu[d][t] = sum_{k=0}^{K-1} ipe[d][t-k] * f_scint(k * tick) * tick, with the two-component time profile
 * f_scint(t) = f_p / tau_p exp(-t / tau_p) + (1 - f_p) / tau_s exp(-t / tau_s) sampled at the lag. */
void orc_light_scint(const orc_light_params *lp, const float *ipe, double *mu)
{
    const int32_t K = orc_light_taps(lp), T = lp->n_ticks;
    double *w = (double *)malloc(sizeof(double) * (size_t)K);
    for (int32_t k = 0; k < K; ++k) {
        double t = k * lp->tick;
        w[k] = lp->tick * (lp->f_prompt / lp->tau_p * exp(-t / lp->tau_p) +
                           (1.0 - lp->f_prompt) / lp->tau_s * exp(-t / lp->tau_s));
    }
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)lp->n_det * T; ++e) {
        const int64_t d = e / T;
        const int32_t t = (int32_t)(e % T);
        const float *x = ipe + d * T;
        double acc = 0.0;
        for (int32_t k = 0; k < K && k <= t; ++k) acc += (double)x[t - k] * w[k];
        mu[e] = acc;
    }
    free(w);
}

/* Photoelectron counting statistics (Sec. 4.2): per (detector, tick) a Poisson draw of mean mu by inverse transform
 * sampling (sequential search of the cumulative distribution from 0), or, above normal_above, mu + sqrt(mu) * g
 * with g standard normal.  One Philox4x32-10 block per element: counter (detector, tick, event id low word, (event id
 * high word << 4) | 12); u = (x0 + 1/2) 2^-32 for the search, Box-Muller on words (0, 1) for g.
 * near[e] = 1 when u lies within 1e-12 of a cumulative value the search compared it with (a decision that a different
 * rounding of mu or exp could change). */
void orc_light_fluct(const orc_light_params *lp, uint64_t event_id, const double *mu, double *n, int32_t *near)
{
    const uint32_t key[2] = {(uint32_t)lp->seed, (uint32_t)(lp->seed >> 32)};
    const int32_t T = lp->n_ticks;
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < (int64_t)lp->n_det * T; ++e) {
        const uint32_t ctr[4] = {(uint32_t)(e / T), (uint32_t)(e % T), (uint32_t)event_id,
                                 (uint32_t)((event_id >> 32) << 4) | ORC_STREAM_LIGHT_PE};
        uint32_t x[4];
        orc_philox4x32_10(ctr, key, x);
        const double two_m32 = 2.3283064365386963e-10;
        const double u = ((double)x[0] + 0.5) * two_m32;
        const double m = mu[e];
        int32_t flag = 0;
        if (m > lp->normal_above) {
            const double u1 = ((double)x[1] + 0.5) * two_m32;
            n[e] = m + sqrt(m) * sqrt(-2.0 * log(u)) * cos(6.283185307179586477 * u1);
        } else {
            double p = exp(-m), F = p;
            int32_t k = 0;
            if (fabs(u - F) < 1e-12) flag = 1;
            while (u > F && k < 1000) {
                ++k;
                p *= m / k;
                F += p;
                if (fabs(u - F) < 1e-12) flag = 1;
            }
            n[e] = (double)k;
        }
        if (near) near[e] = flag;
    }
}

/* Noise phases (Sec. 4.3: random-phase sinusoids): phi[d][f - 1] = 2 pi u for f = 1 .. n_freq, u from word 0 of the
 * Philox block with counter (detector, f, event id low word, (event id high word << 4) | 13). */
void orc_light_noise_phases(const orc_light_params *lp, uint64_t event_id, int32_t n_freq, double *phi)
{
    const uint32_t key[2] = {(uint32_t)lp->seed, (uint32_t)(lp->seed >> 32)};
    for (int32_t d = 0; d < lp->n_det; ++d)
        for (int32_t f = 1; f <= n_freq; ++f) {
            const uint32_t ctr[4] = {(uint32_t)d, (uint32_t)f, (uint32_t)event_id,
                                     (uint32_t)((event_id >> 32) << 4) | ORC_STREAM_LIGHT_NOISE};
            uint32_t x[4];
            orc_philox4x32_10(ctr, key, x);
            phi[(int64_t)d * n_freq + f - 1] = 6.283185307179586477 * (((double)x[0] + 0.5) * 2.3283064365386963e-10);
        }
}
