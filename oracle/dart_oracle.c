/*
 * dart_oracle.c -- plain, slow FP64 CPU oracle for the lookback intensity sum.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or call
 * this file; only the tests, the smoke check and the bench's CPU-baseline leg do.
 * It shares no code, header, table or helper with the HIP library.
 *
 * What it computes (paper, Sec. 2.3 Eqs. 4-9 and Sec. 2.5 Eqs. 14-19):
 *
 *   I(ray) = sum over cells n the ray crosses with chord ds_n > 0, and whose
 *            retarded time tbar_n lies inside [t_0, t_{M-1}], of
 *            ds_n * sum_m W_m(tbar_n) * D_{n,m}^p * j_{n,m}
 *
 *   - ds_n   : exact chord of the ray inside the half-open box of cell n;
 *   - tbar_n : t_obs - s_mid / c (Eq. 2) with c = 1, s_mid the chord midpoint,
 *              s measured along the ray from the plane through the grid centre;
 *   - W_m    : the linear hat weight of Eqs. 6-7 between the two epochs that
 *              bracket tbar_n (generalised to strictly increasing epoch times);
 *   - D      : Doppler factor sqrt(1-beta^2) / (1 + beta . s_hat) (Eq. 14), with
 *              s_hat pointing from the observer into the domain;
 *   - p      : 2 + alpha, the exponent of Eq. 18-19 for a rest-frame spectrum
 *              S ~ nu^-alpha (alpha > 0 for the usual synchrotron slope).
 *
 * Camera: orthographic, distant observer.  n_hat = (sin th cos ph, sin th sin ph,
 * cos th) points toward the observer, s_hat = -n_hat; image basis
 * e_u = (-sin ph, cos ph, 0), e_v = (-cos th cos ph, -cos th sin ph, sin th).
 * Pixel (i, j) sits at u = (i + 1/2 - W/2) p, v = (j + 1/2 - H/2) p; row j = 0 is
 * the most negative v.  Ray: x(s) = C + u e_u + v e_v + s s_hat, C = grid centre.
 *
 * Segmentation (O1): every crossing of a cell plane inside (s_in, s_out) is
 * collected together with s_in and s_out and the list is sorted; consecutive
 * entries bound the per-cell chords.  This is deliberately not a DDA.
 * Brute force (O2): the ray is intersected with every cell box of the grid.
 *
 * Sub-domains (the labelled mode of Sec. 4): a grid may be placed inside a
 * larger domain (placed = 1): its lower corner sits at `origin` and the camera
 * is centred on the domain point `centre`, through which the s = 0 plane of
 * the retarded time also passes.  Everything else is computed in the grid's
 * own coordinates.  A render of the domain is the sum of the renders of its
 * non-overlapping sub-domains (optically thin emission adds along the ray).
 *
 * Flags: ORC_NO_LOOKBACK (tbar = t_obs for every cell, Eq. 3 / Eq. 10),
 * ORC_NO_BEAMING (D = 1), ORC_NEAREST (weight 1 on the epoch closest to tbar,
 * ties to the earlier epoch), ORC_EXACT_TIME (every chord is also cut where
 * the ray's retarded time passes an epoch time, s = t_obs - t_m; each piece
 * then lies in one cell and one epoch interval, where the interpolated
 * emissivity is linear along the ray, so the midpoint rule per piece is the
 * exact integral of the piecewise-linear-in-time field, window ends included.
 * A cell counts as one cell-step however many pieces it has.)
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_NO_LOOKBACK 1u
#define ORC_NO_BEAMING 2u
#define ORC_NEAREST 4u
#define ORC_EXACT_TIME 8u

#define ORC_DT_F64 0
#define ORC_DT_F32 1
#define ORC_DT_F16 2  /* IEEE binary16 bit patterns (uint16) */
#define ORC_DT_BF16 3 /* bfloat16 bit patterns (uint16): the top half of a binary32 */
#define ORC_DT_F32_AS_BF16 4 /* float32 arrays, each value rounded to bfloat16 when read */
#define ORC_DT_F32_AS_F16 5  /* float32 arrays, each value rounded to binary16 when read */

typedef struct {
    int n[3];             /* cells along x, y, z */
    double cell[3];       /* cell size along x, y, z */
    int n_epochs;         /* M */
    const double *times;  /* [M], strictly increasing */
    int dtype;            /* ORC_DT_F64 or ORC_DT_F32 for the two arrays below */
    const void *j;        /* [M][nz][ny][nx] rest-frame emissivity */
    const void *beta;     /* [M][nz][ny][nx][3] velocity / c */
    int placed;           /* 0: the grid is the whole domain */
    double origin[3];     /* placed: position of the grid's lower corner in the domain */
    double centre[3];     /* placed: the domain point the camera is centred on */
} orc_grid;

typedef struct {
    double theta_deg, phi_deg;
    int width, height;
    double pixel_scale;
    double t_obs;
    double alpha;
    unsigned flags;
} orc_view;

/* ---- small helpers ------------------------------------------------------ */

/* sin and cos of an angle in degrees, exact at multiples of 90 degrees */
static void sincos_deg(double deg, double *s, double *c) {
    double r = fmod(deg, 360.0);
    if (r < 0) r += 360.0;
    if (r == 0.0) { *s = 0.0; *c = 1.0; return; }
    if (r == 90.0) { *s = 1.0; *c = 0.0; return; }
    if (r == 180.0) { *s = 0.0; *c = -1.0; return; }
    if (r == 270.0) { *s = -1.0; *c = 0.0; return; }
    *s = sin(deg * (M_PI / 180.0));
    *c = cos(deg * (M_PI / 180.0));
}

/* binary16 -> double from the bit fields: sign, 5-bit exponent (bias 15),
 * 10-bit fraction; subnormals scale the fraction by 2^-24 */
static double half_to_double(uint16_t h) {
    int sign = h >> 15, ex = (h >> 10) & 31, fr = h & 1023;
    double v;
    if (ex == 0) v = ldexp((double)fr, -24);
    else if (ex == 31) v = fr ? NAN : INFINITY;
    else v = ldexp(1.0 + fr / 1024.0, ex - 15);
    return sign ? -v : v;
}

/* Round-to-nearest-even of a finite binary32 to the nearest bfloat16, done on
 * the integer representation: add half an ulp of the 16 kept bits (rounding
 * ties toward the even kept pattern) and drop the low 16 bits. */
static double f32_round_bf16(float f) {
    uint32_t u;
    memcpy(&u, &f, sizeof(u));
    u = (u + 0x7fffu + ((u >> 16) & 1u)) & 0xffff0000u;
    memcpy(&f, &u, sizeof(f));
    return (double)f;
}

/* Round-to-nearest-even of a binary32 to binary16 (finite, normal range and
 * subnormals), returned widened: the value is scaled so that the binary16
 * ulp at its exponent becomes 1, rounded to an integer with ties to even by
 * nearbyint (default rounding mode), and scaled back. */
static double f32_round_f16(float f) {
    double x = (double)f, a = fabs(x);
    if (a == 0.0) return x;
    int e;
    frexp(a, &e);                 /* a = m 2^e, m in [0.5, 1) */
    int ulp_exp = (e - 1) - 10;   /* 10 fraction bits */
    if (ulp_exp < -24) ulp_exp = -24; /* subnormal spacing 2^-24 */
    double q = nearbyint(ldexp(x, -ulp_exp));
    double r = ldexp(q, ulp_exp);
    if (fabs(r) > 65504.0) return x > 0 ? INFINITY : -INFINITY;
    return r;
}

static double load_val(const void *p, int dtype, size_t idx) {
    if (dtype == ORC_DT_F32) return (double)((const float *)p)[idx];
    if (dtype == ORC_DT_F32_AS_BF16) return f32_round_bf16(((const float *)p)[idx]);
    if (dtype == ORC_DT_F32_AS_F16) return f32_round_f16(((const float *)p)[idx]);
    if (dtype == ORC_DT_F16) return half_to_double(((const uint16_t *)p)[idx]);
    if (dtype == ORC_DT_BF16) {
        uint32_t u = (uint32_t)((const uint16_t *)p)[idx] << 16;
        float f;
        memcpy(&f, &u, sizeof(f));
        return (double)f;
    }
    return ((const double *)p)[idx];
}

typedef struct {
    double shat[3], eu[3], ev[3], centre[3];
} orc_camera;

void orc_camera_basis(const orc_grid *g, const orc_view *v, double *out12) {
    double st, ct, sp, cp;
    sincos_deg(v->theta_deg, &st, &ct);
    sincos_deg(v->phi_deg, &sp, &cp);
    double nhat[3] = {st * cp, st * sp, ct};
    for (int a = 0; a < 3; a++) out12[a] = -nhat[a];
    out12[3] = -sp; out12[4] = cp; out12[5] = 0.0;
    out12[6] = -ct * cp; out12[7] = -ct * sp; out12[8] = st;
    for (int a = 0; a < 3; a++)
        out12[9 + a] = g->placed ? g->centre[a] - g->origin[a] : 0.5 * g->n[a] * g->cell[a];
}

static void make_camera(const orc_grid *g, const orc_view *v, orc_camera *cam) {
    double b[12];
    orc_camera_basis(g, v, b);
    memcpy(cam->shat, b, 3 * sizeof(double));
    memcpy(cam->eu, b + 3, 3 * sizeof(double));
    memcpy(cam->ev, b + 6, 3 * sizeof(double));
    memcpy(cam->centre, b + 9, 3 * sizeof(double));
}

static void pixel_ray(const orc_view *v, const orc_camera *cam, int i, int j, double o[3]) {
    double u = (i + 0.5 - 0.5 * v->width) * v->pixel_scale;
    double w = (j + 0.5 - 0.5 * v->height) * v->pixel_scale;
    for (int a = 0; a < 3; a++) o[a] = cam->centre[a] + u * cam->eu[a] + w * cam->ev[a];
}

/* Ray against the box [lo, hi) per axis.  Returns 1 and the chord [s0, s1] when
 * the ray meets the box with s1 > s0; axes with zero direction use the
 * half-open membership test of the origin. */
static int ray_box(const double o[3], const double d[3], const double lo[3], const double hi[3],
                   double *s0, double *s1) {
    double a = -INFINITY, b = INFINITY;
    for (int k = 0; k < 3; k++) {
        if (d[k] == 0.0) {
            if (o[k] < lo[k] || o[k] >= hi[k]) return 0;
            continue;
        }
        double t0 = (lo[k] - o[k]) / d[k];
        double t1 = (hi[k] - o[k]) / d[k];
        if (t0 > t1) { double t = t0; t0 = t1; t1 = t; }
        if (t0 > a) a = t0;
        if (t1 < b) b = t1;
    }
    if (!(b > a)) return 0;
    *s0 = a;
    *s1 = b;
    return 1;
}

/* Interpolation weights of Eqs. 6-7 on strictly increasing epoch times.
 * Writes at most two (epoch, weight) pairs and returns their count; returns 0
 * when tbar lies outside [t_0, t_{M-1}] (the hard temporal window). */
int orc_epoch_weights(const double *t, int M, double tbar, unsigned flags, int *m_out,
                      double *w_out) {
    if (!(tbar >= t[0] && tbar <= t[M - 1])) return 0;
    if (M == 1) { m_out[0] = 0; w_out[0] = 1.0; return 1; }
    int m = 0;
    while (m + 1 < M - 1 && t[m + 1] <= tbar) m++;
    if (flags & ORC_NEAREST) {
        /* the epoch of smallest |tbar - t_m|; an exact tie goes to the earlier one */
        double dl = tbar - t[m], dr = t[m + 1] - tbar;
        m_out[0] = (dr < dl) ? m + 1 : m;
        w_out[0] = 1.0;
        return 1;
    }
    double delta = (tbar - t[m]) / (t[m + 1] - t[m]);
    m_out[0] = m;     w_out[0] = 1.0 - delta;
    m_out[1] = m + 1; w_out[1] = delta;
    return 2;
}

/* D^p for one stored velocity, Eq. 14 raised to p = 2 + alpha */
static double doppler_pow(const double beta[3], const double shat[3], double p) {
    double b2 = beta[0] * beta[0] + beta[1] * beta[1] + beta[2] * beta[2];
    double bs = beta[0] * shat[0] + beta[1] * shat[1] + beta[2] * shat[2];
    double D = sqrt(1.0 - b2) / (1.0 + bs);
    return pow(D, p);
}

/* Epoch-interval restriction for the snapshot-outer form: only the epochs
 * [e0, e0 + ne) are present in the grid's arrays, and only cells whose
 * retarded time lies in [t_lo, t_hi) (closed at t_hi when hi_closed) are
 * summed.  The default (ne = 0) means every epoch is present and no
 * restriction applies. */
typedef struct {
    int e0, ne;
    double t_lo, t_hi;
    int hi_closed;
    int ring; /* 0: epoch e is at slot e - e0; 1: at slot e mod ne (a ring of ne epochs) */
} orc_window;

static __thread const orc_window *tl_win = NULL;

/* Contribution of one chord [sa, sb] inside cell (ix, iy, iz).  Returns 1 when
 * the cell lies inside the temporal window (a counted cell-step). */
static int cell_term(const orc_grid *g, const orc_view *v, const double shat[3], int ix,
                     int iy, int iz, double sa, double sb, double *acc) {
    double ds = sb - sa;
    double smid = 0.5 * (sa + sb);
    double tbar = (v->flags & ORC_NO_LOOKBACK) ? v->t_obs : v->t_obs - smid;
    const orc_window *w = tl_win;
    if (w && w->ne > 0) {
        if (!(tbar >= w->t_lo && (tbar < w->t_hi || (w->hi_closed && tbar == w->t_hi)))) return 0;
    }
    int ms[2];
    double ws[2];
    int k = orc_epoch_weights(g->times, g->n_epochs, tbar, v->flags, ms, ws);
    if (k == 0) return 0;
    size_t ncell = (size_t)g->n[0] * g->n[1] * g->n[2];
    size_t c = ((size_t)iz * g->n[1] + iy) * g->n[0] + ix;
    double p = 2.0 + v->alpha;
    double sum = 0.0;
    for (int q = 0; q < k; q++) {
        if (ws[q] == 0.0) continue;
        int me = ms[q];
        if (w && w->ne > 0) {
            if (me < w->e0 || me >= w->e0 + w->ne) return -1; /* the caller did not load it */
            me = w->ring ? me % w->ne : me - w->e0;
        }
        size_t r = (size_t)me * ncell + c;
        double jv = load_val(g->j, g->dtype, r);
        double dp = 1.0;
        if (!(v->flags & ORC_NO_BEAMING)) {
            double b[3] = {load_val(g->beta, g->dtype, 3 * r), load_val(g->beta, g->dtype, 3 * r + 1),
                           load_val(g->beta, g->dtype, 3 * r + 2)};
            dp = doppler_pow(b, shat, p);
        }
        sum += ws[q] * dp * jv;
    }
    *acc += ds * sum;
    return 1;
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

static __thread int tl_err = 0;

/* Appends the crossings of the planes x_a = k dx_a (0 < k < n_a) that lie
 * strictly inside (s0, s1); only the k whose plane can be reached in that
 * range are visited. */
static int add_crossings(const orc_grid *g, const double o[3], const double d[3], double s0,
                         double s1, double *out, int cnt) {
    for (int a = 0; a < 3; a++) {
        if (d[a] == 0.0) continue;
        double x0 = (o[a] + s0 * d[a]) / g->cell[a], x1 = (o[a] + s1 * d[a]) / g->cell[a];
        if (x0 > x1) { double t = x0; x0 = x1; x1 = t; }
        long k0 = (long)floor(x0) - 1, k1 = (long)ceil(x1) + 1;
        if (k0 < 1) k0 = 1;
        if (k1 > g->n[a] - 1) k1 = g->n[a] - 1;
        for (long k = k0; k <= k1; k++) {
            double s = (k * g->cell[a] - o[a]) / d[a];
            if (s > s0 && s < s1) out[cnt++] = s;
        }
    }
    return cnt;
}

/* O1: one pixel by sorted plane crossings */
static double ray_sorted(const orc_grid *g, const orc_view *v, const orc_camera *cam, int i,
                         int j, long long *steps, double *scratch) {
    double o[3];
    pixel_ray(v, cam, i, j, o);
    const double *d = cam->shat;
    double lo[3] = {0, 0, 0}, hi[3];
    for (int a = 0; a < 3; a++) hi[a] = g->n[a] * g->cell[a];
    double s_in, s_out;
    if (!ray_box(o, d, lo, hi, &s_in, &s_out)) return 0.0;
    const orc_window *w = tl_win;
    if (w && w->ne > 0 && !(v->flags & ORC_NO_LOOKBACK)) {
        /* snapshot-outer form: only chords whose midpoint can fall inside the
         * window are needed; a margin of one cell diagonal keeps every such
         * chord whole, and the partial chords at the clipped ends have their
         * midpoints outside the window */
        double diag = sqrt(g->cell[0] * g->cell[0] + g->cell[1] * g->cell[1] +
                           g->cell[2] * g->cell[2]);
        double c0 = v->t_obs - w->t_hi - diag, c1 = v->t_obs - w->t_lo + diag;
        if (c0 > s_in) s_in = c0;
        if (c1 < s_out) s_out = c1;
        if (!(s_out > s_in)) return 0.0;
    }
    int cnt = 0;
    scratch[cnt++] = s_in;
    scratch[cnt++] = s_out;
    cnt = add_crossings(g, o, d, s_in, s_out, scratch, cnt);
    if ((v->flags & ORC_EXACT_TIME) && !(v->flags & ORC_NO_LOOKBACK))
        for (int m = 0; m < g->n_epochs; m++) {
            double s = v->t_obs - g->times[m];
            if (s > s_in && s < s_out) scratch[cnt++] = s;
        }
    qsort(scratch, (size_t)cnt, sizeof(double), cmp_double);
    double acc = 0.0;
    long long n_steps = 0;
    long long last_cell = -1;  /* a cell cut in pieces counts once */
    for (int q = 0; q + 1 < cnt; q++) {
        double sa = scratch[q], sb = scratch[q + 1];
        if (!(sb > sa)) continue;
        double smid = 0.5 * (sa + sb);
        int idx[3], inside = 1;
        for (int a = 0; a < 3; a++) {
            idx[a] = (int)floor((o[a] + smid * d[a]) / g->cell[a]);
            if (idx[a] < 0 || idx[a] >= g->n[a]) inside = 0;
        }
        if (!inside) continue;
        int r = cell_term(g, v, d, idx[0], idx[1], idx[2], sa, sb, &acc);
        const long long lin = ((long long)idx[2] * g->n[1] + idx[1]) * g->n[0] + idx[0];
        if (r < 0) tl_err = 1;
        else if (r > 0 && lin != last_cell) {
            n_steps++;
            last_cell = lin;
        }
    }
    if (steps) *steps += n_steps;
    return acc;
}

/* O2: one pixel by testing every cell box of the grid */
static double ray_brute(const orc_grid *g, const orc_view *v, const orc_camera *cam, int i,
                        int j, long long *steps) {
    double o[3];
    pixel_ray(v, cam, i, j, o);
    const double *d = cam->shat;
    double acc = 0.0;
    long long n_steps = 0;
    for (int iz = 0; iz < g->n[2]; iz++)
        for (int iy = 0; iy < g->n[1]; iy++)
            for (int ix = 0; ix < g->n[0]; ix++) {
                double lo[3] = {ix * g->cell[0], iy * g->cell[1], iz * g->cell[2]};
                double hi[3] = {(ix + 1) * g->cell[0], (iy + 1) * g->cell[1], (iz + 1) * g->cell[2]};
                double sa, sb;
                if (!ray_box(o, d, lo, hi, &sa, &sb)) continue;
                /* exact-time mode: the chord cut at every epoch time inside it */
                double cuts[2 + 64];  /* (exact-time brute force: at most 64 epochs) */
                int nc = 0;
                cuts[nc++] = sa;
                if ((v->flags & ORC_EXACT_TIME) && !(v->flags & ORC_NO_LOOKBACK))
                    for (int m = 0; m < g->n_epochs && m < 64; m++) {
                        double s = v->t_obs - g->times[m];
                        if (s > sa && s < sb) cuts[nc++] = s;
                    }
                cuts[nc++] = sb;
                qsort(cuts, (size_t)nc, sizeof(double), cmp_double);
                int any = 0;
                for (int q = 0; q + 1 < nc; q++) {
                    int r = cell_term(g, v, d, ix, iy, iz, cuts[q], cuts[q + 1], &acc);
                    if (r < 0) tl_err = 1;
                    else any |= r;
                }
                n_steps += any;
            }
    if (steps) *steps += n_steps;
    return acc;
}

/* ---- threaded drivers ---------------------------------------------------- */

typedef struct {
    const orc_grid *g;
    const orc_view *v;
    const orc_camera *cam;
    const int32_t *pix; /* pairs (i, j), or NULL for the whole image in row order */
    long long n_pix;
    double *out;
    long long steps;
    int tid, nthreads, brute;
    const orc_window *win;
    int accumulate, err;
} orc_job;

static void *worker(void *arg) {
    orc_job *jb = (orc_job *)arg;
    const orc_grid *g = jb->g;
    tl_win = jb->win;
    tl_err = 0;
    size_t cap = 2 + (size_t)g->n[0] + g->n[1] + g->n[2] + (size_t)g->n_epochs;
    double *scratch = (double *)malloc(cap * sizeof(double));
    for (long long q = jb->tid; q < jb->n_pix; q += jb->nthreads) {
        int i, j;
        if (jb->pix) { i = jb->pix[2 * q]; j = jb->pix[2 * q + 1]; }
        else { i = (int)(q % jb->v->width); j = (int)(q / jb->v->width); }
        double val = jb->brute ? ray_brute(g, jb->v, jb->cam, i, j, &jb->steps)
                               : ray_sorted(g, jb->v, jb->cam, i, j, &jb->steps, scratch);
        if (jb->accumulate) jb->out[q] += val;
        else jb->out[q] = val;
    }
    free(scratch);
    jb->err = tl_err;
    tl_win = NULL;
    return NULL;
}

static int run_ex(const orc_grid *g, const orc_view *v, const int32_t *pix, long long n_pix,
                  double *out, long long *steps_out, int nthreads, int brute,
                  const orc_window *win, int accumulate) {
    if (!g || !v || !out || g->n_epochs < 1) return -1;
    for (int a = 0; a < 3; a++)
        if (g->n[a] < 1 || !(g->cell[a] > 0)) return -1;
    for (int m = 0; m + 1 < g->n_epochs; m++)
        if (!(g->times[m + 1] > g->times[m])) return -1;
    if (!pix) n_pix = (long long)v->width * v->height;
    if (nthreads < 1) nthreads = 1;
    orc_camera cam;
    make_camera(g, v, &cam);
    orc_job *jobs = (orc_job *)calloc((size_t)nthreads, sizeof(orc_job));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    for (int t = 0; t < nthreads; t++) {
        orc_job jb = {g, v, &cam, pix, n_pix, out, 0, t, nthreads, brute, win, accumulate, 0};
        jobs[t] = jb;
        if (nthreads > 1) pthread_create(&th[t], NULL, worker, &jobs[t]);
    }
    if (nthreads == 1) worker(&jobs[0]);
    long long steps = 0;
    int err = 0;
    for (int t = 0; t < nthreads; t++) {
        if (nthreads > 1) pthread_join(th[t], NULL);
        steps += jobs[t].steps;
        err |= jobs[t].err;
    }
    if (steps_out) *steps_out = steps;
    free(jobs);
    free(th);
    return err ? -2 : 0;
}

static int run(const orc_grid *g, const orc_view *v, const int32_t *pix, long long n_pix,
               double *out, long long *steps_out, int nthreads, int brute) {
    return run_ex(g, v, pix, n_pix, out, steps_out, nthreads, brute, NULL, 0);
}

/* O1 over a pixel list (pix = (i, j) pairs) or over the whole image (pix = NULL,
 * out in row order [height][width]).  steps_out receives the number of counted
 * cell-steps (cells with a positive chord inside the temporal window). */
int orc_render(const orc_grid *g, const orc_view *v, const int32_t *pix, long long n_pix,
               double *out, long long *steps_out, int nthreads) {
    return run(g, v, pix, n_pix, out, steps_out, nthreads, 0);
}

/* Snapshot-outer form of O1 (the chronology of the paper's Fig. 5): the grid's
 * arrays hold only epochs [e0, e0 + ne) (times still lists all M epochs), and
 * the call ADDS to out[] the contributions of the cells whose retarded time
 * lies in [t_lo, t_hi) (or [t_lo, t_hi] with hi_closed).  With ring != 0 the
 * arrays are a ring of ne slots and epoch e sits in slot e mod ne.  Summing the calls
 * over the intervals [t_m, t_{m+1}) with epochs {m, m+1} loaded, the last one
 * closed, gives the whole image while only two epochs are held at a time.
 * Returns -2 when a cell in the interval needs an epoch that was not loaded. */
int orc_render_window(const orc_grid *g, const orc_view *v, int e0, int ne, int ring, double t_lo,
                      double t_hi, int hi_closed, const int32_t *pix, long long n_pix, double *out,
                      long long *steps_out, int nthreads) {
    if (ne < 1 || e0 < 0 || e0 + ne > g->n_epochs) return -1;
    orc_window w = {e0, ne, t_lo, t_hi, hi_closed, ring};
    return run_ex(g, v, pix, n_pix, out, steps_out, nthreads, 0, &w, 1);
}

/* O2, same interface; cost grows with every cell of the grid per pixel */
int orc_render_brute(const orc_grid *g, const orc_view *v, const int32_t *pix, long long n_pix,
                     double *out, long long *steps_out, int nthreads) {
    return run(g, v, pix, n_pix, out, steps_out, nthreads, 1);
}

/* Chord segmentation of one pixel ray as used by O1: writes up to cap triples
 * (s_a, s_b, linear cell index) and returns the number of chords. */
int orc_segments(const orc_grid *g, const orc_view *v, int i, int j, double *out, int cap) {
    orc_camera cam;
    make_camera(g, v, &cam);
    double o[3];
    pixel_ray(v, &cam, i, j, o);
    const double *d = cam.shat;
    double lo[3] = {0, 0, 0}, hi[3];
    for (int a = 0; a < 3; a++) hi[a] = g->n[a] * g->cell[a];
    double s_in, s_out;
    if (!ray_box(o, d, lo, hi, &s_in, &s_out)) return 0;
    size_t n_all = 2 + (size_t)g->n[0] + g->n[1] + g->n[2];
    double *s = (double *)malloc(n_all * sizeof(double));
    int cnt = 0;
    s[cnt++] = s_in;
    s[cnt++] = s_out;
    for (int a = 0; a < 3; a++) {
        if (d[a] == 0.0) continue;
        for (int k = 1; k < g->n[a]; k++) {
            double t = (k * g->cell[a] - o[a]) / d[a];
            if (t > s_in && t < s_out) s[cnt++] = t;
        }
    }
    qsort(s, (size_t)cnt, sizeof(double), cmp_double);
    int nseg = 0;
    for (int q = 0; q + 1 < cnt && nseg < cap; q++) {
        if (!(s[q + 1] > s[q])) continue;
        double smid = 0.5 * (s[q] + s[q + 1]);
        int idx[3], inside = 1;
        for (int a = 0; a < 3; a++) {
            idx[a] = (int)floor((o[a] + smid * d[a]) / g->cell[a]);
            if (idx[a] < 0 || idx[a] >= g->n[a]) inside = 0;
        }
        if (!inside) continue;
        out[3 * nseg] = s[q];
        out[3 * nseg + 1] = s[q + 1];
        out[3 * nseg + 2] = (double)(((size_t)idx[2] * g->n[1] + idx[1]) * g->n[0] + idx[0]);
        nseg++;
    }
    free(s);
    return nseg;
}

/* Number of distinct (block, epoch) pairs that receive a positive weight on
 * any ray of the image, for blocks of bx x by x bz cells (1 x 1 x 1: the
 * compulsory samples an image must read).  Reads no field values. */
long long orc_count_blocks(const orc_grid *g, const orc_view *v, int bx, int by, int bz) {
    int nbx = (g->n[0] + bx - 1) / bx, nby = (g->n[1] + by - 1) / by, nbz = (g->n[2] + bz - 1) / bz;
    size_t ncell = (size_t)nbx * nby * nbz;
    size_t nbits = ncell * (size_t)g->n_epochs;
    uint8_t *seen = (uint8_t *)calloc(nbits, 1);
    if (!seen) return -1;
    int cap = 2 + g->n[0] + g->n[1] + g->n[2];
    double *seg = (double *)malloc((size_t)cap * 3 * sizeof(double));
    long long count = 0;
    for (int j = 0; j < v->height; j++)
        for (int i = 0; i < v->width; i++) {
            int ns = orc_segments(g, v, i, j, seg, cap);
            for (int q = 0; q < ns; q++) {
                double smid = 0.5 * (seg[3 * q] + seg[3 * q + 1]);
                double tbar = (v->flags & ORC_NO_LOOKBACK) ? v->t_obs : v->t_obs - smid;
                int ms[2];
                double ws[2];
                int k = orc_epoch_weights(g->times, g->n_epochs, tbar, v->flags, ms, ws);
                for (int r = 0; r < k; r++) {
                    if (!(ws[r] > 0.0)) continue;
                    size_t c = (size_t)seg[3 * q + 2];
                    size_t x = c % g->n[0], y = (c / g->n[0]) % g->n[1], z = c / ((size_t)g->n[0] * g->n[1]);
                    size_t blk = ((z / bz) * nby + y / by) * nbx + x / bx;
                    size_t bit = (size_t)ms[r] * ncell + blk;
                    if (!seen[bit]) { seen[bit] = 1; count++; }
                }
            }
        }
    free(seg);
    free(seen);
    return count;
}

long long orc_count_samples(const orc_grid *g, const orc_view *v) {
    return orc_count_blocks(g, v, 1, 1, 1);
}
