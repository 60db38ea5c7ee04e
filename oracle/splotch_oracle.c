/*
 * Splotch render oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU evaluation of the Splotch render as
 * defined in Jin et al., "High-performance astrophysical visualization using
 * Splotch" (ICCS 2010), Section 2:
 *   - every particle p carries a Gaussian density rho_p(r) = rho0_p exp(-r^2/sigma_p^2)
 *     that is cut to zero at f*sigma_p (Section 2, first assumption);
 *   - r, g and b are transported independently (second assumption);
 *   - along each ray the intensity obeys dI/dx = (E_p - A_p I) rho_p(x)
 *     (Section 2, Eq. (1));
 *   - E_p and A_p come from a scalar through a colour look-up table, or from
 *     the three components of a vector quantity, and the optical depth may
 *     be scaled by another per-particle scalar (Section 2, last paragraph);
 *   - the render stage transforms particles to screen coordinates, assigns
 *     colours, finds the screen area each particle affects and combines the
 *     contributions (Section 3.2).
 *
 * Everything continuous is computed in double precision.  The integer
 * decisions (which particles are visible, their pixel bounding boxes, the
 * screen tiles they touch, the depth key that orders them, and which pixels
 * a particle covers) follow a written recipe of IEEE operations in a fixed
 * order so that another implementation can reproduce them bit for bit:
 *   projection, bounding box:   binary64, no fused multiply-add;
 *   depth key:                  binary32 rounding of the camera depth;
 *   pixel membership:           binary32, no fused multiply-add.
 * This file must be compiled with -ffp-contract=off.
 *
 * Compositing: particles covering a pixel are ordered by (depth key, index)
 * front to back.  Each particle's contribution is the exact solution of
 * Eq. (1) across that particle alone, I <- I exp(-A tau) + E tau phi(A tau)
 * with phi(x) = (1 - exp(-x))/x and tau the line-of-sight column of the
 * particle's density at the pixel:
 *   kernel 0 (cut on the impact parameter): tau = rho0 exp(-q^2);
 *   kernel 1 (density cut to the sphere r <= f sigma):
 *            tau = rho0 exp(-q^2) erf(sqrt(f^2 - q^2));
 * q = d/sigma_s, both normalised so that the untruncated column at zero
 * impact parameter is rho0.  The oracle applies the particles back to front
 * (painter's order), starting from the input image.  Emission-only steps
 * (A = 0, a plain sum) are added with Neumaier's compensated summation; an
 * absorbing step scales the carried compensation by its transmittance.
 *
 * The brute-force ray marcher integrates Eq. (1) along each pixel ray
 * through the summed density of all particles, without any splatting.
 *
 * Nothing here is shared with the GPU implementation and nothing in the
 * GPU implementation may call it; only tests and the CPU-baseline timing do.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_SPECIES 8
#define ORC_PI 3.14159265358979323846

enum { ORC_VISIBLE = 0, ORC_INVALID = 1, ORC_DEPTH = 2, ORC_OFFSCREEN = 3 };

/* Particle set: host arrays of n.  value_g and value_b are the second and
 * third components of a vector quantity whose first component is value;
 * they are read only for species coloured by a vector. */
typedef struct {
    int64_t n;
    const float *x, *y, *z, *h, *value, *rho0, *value_g, *value_b;
    const uint8_t *species;
} orc_particles;

/* Render settings.  colour[s]: 0 = scalar through the palette, 1 = the
 * three vector components map to r, g, b directly.  mode[s]: 0 additive
 * (A = 0), 1 ordered (A = absorb * colour).  kernel: 0 or 1 as above.
 * emission_is_source: 1 reads the emission of absorbing species as a source
 * function S, i.e. Eq. (1) runs with E := A * S.  pal_abs (KA entries) is
 * the absorption palette; NULL means the emission palette. */
typedef struct {
    int ns;
    float vmin[ORC_MAX_SPECIES], vmax[ORC_MAX_SPECIES];
    float bright[ORC_MAX_SPECIES], absorb[ORC_MAX_SPECIES];
    int log_scale[ORC_MAX_SPECIES], mode[ORC_MAX_SPECIES], colour[ORC_MAX_SPECIES];
    float sigma_over_h, trunc_f;
    int kernel, emission_is_source;
    int K, KA;
    const float *pal, *pal_abs;
} orc_settings;

/* Camera as flat FP32 values, promoted to FP64 exactly:
 * cam[0..2] eye, [3..5] right, [6..8] up, [9..11] fwd,
 * cam[12] focal length in px (perspective), cam[13] px per unit (ortho),
 * cam[14] z_near, cam[15] z_far. */
typedef struct {
    int persp, W, H;
    double eye[3], right[3], up[3], fwd[3];
    double focal, ppu, znear, zfar;
} cam64;

static cam64 cam_promote(const float *cam, int projection, int W, int H) {
    cam64 c;
    c.persp = projection == 1;
    c.W = W;
    c.H = H;
    for (int k = 0; k < 3; ++k) {
        c.eye[k] = (double)cam[k];
        c.right[k] = (double)cam[3 + k];
        c.up[k] = (double)cam[6 + k];
        c.fwd[k] = (double)cam[9 + k];
    }
    c.focal = (double)cam[12];
    c.ppu = (double)cam[13];
    c.znear = (double)cam[14];
    c.zfar = (double)cam[15];
    return c;
}

/* Monotone unsigned image of a binary32 value (for ordering). */
static uint32_t order_bits(float f) {
    uint32_t b;
    memcpy(&b, &f, 4);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

typedef struct {
    int status;
    int i0, i1, j0, j1;
    float u_rel, v_rel, r2;  /* binary32 fields that decide pixel membership */
    uint32_t key;            /* depth ordering key */
    double u, v, sig, zc;    /* exact screen position, screen sigma, camera depth */
} proj_t;

static int finitef(float a) { return isfinite(a) != 0; }

/* Camera transform and projection of one particle to screen coordinates
 * (Section 3.2, the display step) plus its screen footprint. */
static proj_t project_one(const cam64 *c, float x, float y, float z, float h,
                          double soh, double f) {
    proj_t p;
    memset(&p, 0, sizeof p);
    double d0 = (double)x - c->eye[0];
    double d1 = (double)y - c->eye[1];
    double d2 = (double)z - c->eye[2];
    double xc = (d0 * c->right[0] + d1 * c->right[1]) + d2 * c->right[2];
    double yc = (d0 * c->up[0] + d1 * c->up[1]) + d2 * c->up[2];
    double zc = (d0 * c->fwd[0] + d1 * c->fwd[1]) + d2 * c->fwd[2];
    p.zc = zc;
    if (!(zc > c->znear && zc <= c->zfar)) {
        p.status = ORC_DEPTH;
        return p;
    }
    double s = c->persp ? c->focal / zc : c->ppu;
    double u = xc * s + 0.5 * (double)c->W;
    double v = yc * s + 0.5 * (double)c->H;
    double sig = ((double)h * soh) * s;
    double r = f * sig;
    p.u = u;
    p.v = v;
    p.sig = sig;
    double a = (u - r) - 0.5, b = (u + r) - 0.5;
    double cc = (v - r) - 0.5, d = (v + r) - 0.5;
    if (!(a <= b) || !(cc <= d)) {
        p.status = ORC_OFFSCREEN;
        return p;
    }
    double i0 = ceil(a), i1 = floor(b), j0 = ceil(cc), j1 = floor(d);
    if (i0 < 0.0) i0 = 0.0;
    if (i1 > (double)(c->W - 1)) i1 = (double)(c->W - 1);
    if (j0 < 0.0) j0 = 0.0;
    if (j1 > (double)(c->H - 1)) j1 = (double)(c->H - 1);
    if (!(i0 <= i1) || !(j0 <= j1)) {
        p.status = ORC_OFFSCREEN;
        return p;
    }
    p.i0 = (int)i0;
    p.i1 = (int)i1;
    p.j0 = (int)j0;
    p.j1 = (int)j1;
    p.u_rel = (float)(u - i0);
    p.v_rel = (float)(v - j0);
    p.r2 = (float)(r * r);
    p.key = order_bits((float)zc);
    p.status = ORC_VISIBLE;
    return p;
}

/* Binary32 membership of pixel (i, j) in a particle's footprint disk. */
static int member32(const proj_t *p, int i, int j) {
    if (i < p->i0 || i > p->i1 || j < p->j0 || j > p->j1) return 0;
    float dx = ((float)(i - p->i0) + 0.5f) - p->u_rel;
    float dy = ((float)(j - p->j0) + 0.5f) - p->v_rel;
    float dd = dx * dx + dy * dy;
    return dd <= p->r2;
}

static int is_vector(const orc_settings *st, int s) { return st->colour[s] == 1; }

static int particle_valid(const orc_particles *P, int64_t k, const orc_settings *st) {
    if (!finitef(P->x[k]) || !finitef(P->y[k]) || !finitef(P->z[k]) || !finitef(P->h[k]) ||
        !finitef(P->value[k]))
        return 0;
    if (!(P->h[k] > 0.0f)) return 0;
    if (P->species && (int)P->species[k] >= st->ns) return 0;
    if (P->rho0 && (!finitef(P->rho0[k]) || P->rho0[k] < 0.0f)) return 0;
    int s = P->species ? P->species[k] : 0;
    if (is_vector(st, s) && (!finitef(P->value_g[k]) || !finitef(P->value_b[k]))) return 0;
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Colour (Section 2: a scalar is mapped to colour through a look-up
 * table, or a vector's components map to r, g, b; Section 3.2: particle
 * values are normalised before display).                                  */
/* ---------------------------------------------------------------------- */

/* Resolve each species' value range.  Given (vmin < vmax) ranges are kept;
 * otherwise the range is the exact min/max of the species' valid particles
 * (positive values only when the species uses a log scale), over all three
 * components for vector-coloured species. */
void orc_value_range(const orc_particles *P, const orc_settings *st, float *vmin_out,
                     float *vmax_out) {
    int have[ORC_MAX_SPECIES] = {0};
    float lo[ORC_MAX_SPECIES], hi[ORC_MAX_SPECIES];
    for (int64_t k = 0; k < P->n; ++k) {
        if (!particle_valid(P, k, st)) continue;
        int s = P->species ? P->species[k] : 0;
        float comp[3] = {P->value[k], 0.0f, 0.0f};
        int nc = 1;
        if (is_vector(st, s)) {
            comp[1] = P->value_g[k];
            comp[2] = P->value_b[k];
            nc = 3;
        }
        for (int c = 0; c < nc; ++c) {
            float v = comp[c];
            if (st->log_scale[s] && !(v > 0.0f)) continue;
            if (!have[s]) {
                lo[s] = hi[s] = v;
                have[s] = 1;
            } else {
                if (v < lo[s]) lo[s] = v;
                if (v > hi[s]) hi[s] = v;
            }
        }
    }
    for (int s = 0; s < st->ns; ++s) {
        vmin_out[s] = st->vmin[s];
        vmax_out[s] = st->vmax[s];
        if (st->vmin[s] < st->vmax[s]) continue;
        vmin_out[s] = have[s] ? lo[s] : 0.0f;
        vmax_out[s] = have[s] ? hi[s] : 0.0f;
    }
}

/* Normalised scalar t in [0, 1]. */
double orc_normalise(float value, float vmin, float vmax, int log_scale) {
    double gv, g0, g1;
    if (log_scale) {
        if (!(value > 0.0f) || !(vmin > 0.0f) || !(vmax > 0.0f)) return 0.0;
        gv = log10((double)value);
        g0 = log10((double)vmin);
        g1 = log10((double)vmax);
    } else {
        gv = value;
        g0 = vmin;
        g1 = vmax;
    }
    double den = g1 - g0;
    if (!(den > 0.0)) return 0.0;
    double t = (gv - g0) / den;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    return t;
}

/* Linear interpolation in a K-entry RGB palette at t*(K-1), clamped. */
void orc_palette(double t, int K, const float *pal, double *rgb) {
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double p = t * (double)(K - 1);
    int k = (int)floor(p);
    if (k > K - 2) k = K - 2;
    double w = p - (double)k;
    for (int c = 0; c < 3; ++c)
        rgb[c] = (double)pal[3 * k + c] * (1.0 - w) + (double)pal[3 * (k + 1) + c] * w;
}

/* Emission and absorption coefficients of particle k per channel
 * (Section 2, last paragraph).  lo/hi: the resolved value ranges. */
static void particle_colour(const orc_particles *P, int64_t k, const orc_settings *st,
                            const float *lo, const float *hi, double *E, double *A) {
    int s = P->species ? P->species[k] : 0;
    double ce[3], ca[3];
    if (is_vector(st, s)) {
        const float comp[3] = {P->value[k], P->value_g[k], P->value_b[k]};
        for (int c = 0; c < 3; ++c) ce[c] = ca[c] = orc_normalise(comp[c], lo[s], hi[s],
                                                                  st->log_scale[s]);
    } else {
        double t = orc_normalise(P->value[k], lo[s], hi[s], st->log_scale[s]);
        orc_palette(t, st->K, st->pal, ce);
        if (st->pal_abs)
            orc_palette(t, st->KA, st->pal_abs, ca);
        else
            for (int c = 0; c < 3; ++c) ca[c] = ce[c];
    }
    for (int c = 0; c < 3; ++c) {
        E[c] = (double)st->bright[s] * ce[c];
        A[c] = st->mode[s] == 1 ? (double)st->absorb[s] * ca[c] : 0.0;
        /* source-function reading: Eq. (1) with E := A * S */
        if (st->emission_is_source && st->mode[s] == 1) E[c] = A[c] * E[c];
    }
}

/* Column through the particle at squared normalised impact parameter q2,
 * per unit rho0 (Section 2, first assumption; see the header comment). */
static double column(const orc_settings *st, double q2) {
    double g = exp(-q2);
    if (st->kernel == 1) {
        double f = (double)st->trunc_f;
        double rem = f * f - q2;
        g *= erf(sqrt(rem > 0.0 ? rem : 0.0));
    }
    return g;
}

/* ---------------------------------------------------------------------- */
/* Projection outputs for index checks.                                    */
/* ---------------------------------------------------------------------- */
void orc_project(const orc_particles *P, const orc_settings *st, const float *cam,
                 int projection, int W, int H, int tile, int8_t *status, int32_t *bbox,
                 float *spec, uint32_t *key, uint32_t *ntiles, double *cont) {
    cam64 c = cam_promote(cam, projection, W, H);
    for (int64_t k = 0; k < P->n; ++k) {
        proj_t p;
        memset(&p, 0, sizeof p);
        if (!particle_valid(P, k, st))
            p.status = ORC_INVALID;
        else
            p = project_one(&c, P->x[k], P->y[k], P->z[k], P->h[k], (double)st->sigma_over_h,
                            (double)st->trunc_f);
        status[k] = (int8_t)p.status;
        bbox[4 * k + 0] = p.i0;
        bbox[4 * k + 1] = p.i1;
        bbox[4 * k + 2] = p.j0;
        bbox[4 * k + 3] = p.j1;
        spec[3 * k + 0] = p.u_rel;
        spec[3 * k + 1] = p.v_rel;
        spec[3 * k + 2] = p.r2;
        key[k] = p.key;
        ntiles[k] = 0;
        if (p.status == ORC_VISIBLE && tile > 0)
            ntiles[k] = (uint32_t)((p.i1 / tile - p.i0 / tile + 1) *
                                   (p.j1 / tile - p.j0 / tile + 1));
        cont[4 * k + 0] = p.u;
        cont[4 * k + 1] = p.v;
        cont[4 * k + 2] = p.sig;
        cont[4 * k + 3] = p.zc;
    }
}

/* ---------------------------------------------------------------------- */
/* Rendering.                                                               */
/* ---------------------------------------------------------------------- */
typedef struct {
    proj_t p;
    int64_t idx;
    double E[3], A[3], rho0;
} vis_t;

static int cmp_canonical(const void *a, const void *b) {
    const vis_t *x = (const vis_t *)a, *y = (const vis_t *)b;
    if (x->p.key != y->p.key) return x->p.key < y->p.key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* phi(x) = (1 - exp(-x))/x, phi(0) = 1. */
static double phi(double xx) { return xx > 0.0 ? -expm1(-xx) / xx : 1.0; }

/* Build the visible-particle list with colours, in canonical front-to-back
 * order.  Returns the count; *out is malloc'ed. */
static int64_t build_visible(const orc_particles *P, const orc_settings *st, const cam64 *c,
                             vis_t **out) {
    float lo[ORC_MAX_SPECIES], hi[ORC_MAX_SPECIES];
    orc_value_range(P, st, lo, hi);
    vis_t *v = (vis_t *)malloc(sizeof(vis_t) * (size_t)(P->n > 0 ? P->n : 1));
    int64_t m = 0;
    for (int64_t k = 0; k < P->n; ++k) {
        if (!particle_valid(P, k, st)) continue;
        proj_t p = project_one(c, P->x[k], P->y[k], P->z[k], P->h[k], (double)st->sigma_over_h,
                               (double)st->trunc_f);
        if (p.status != ORC_VISIBLE) continue;
        vis_t e;
        e.p = p;
        e.idx = k;
        e.rho0 = P->rho0 ? (double)P->rho0[k] : 1.0;
        particle_colour(P, k, st, lo, hi, e.E, e.A);
        v[m++] = e;
    }
    qsort(v, (size_t)m, sizeof(vis_t), cmp_canonical);
    *out = v;
    return m;
}

/* One step of Eq. (1) across one particle with column tau, on the
 * intensity I of one channel and its carried compensation cmp. */
static void rt_step(double E, double A, double tau, double *I, double *cmp) {
    double xx = A * tau;
    if (xx > 0.0) {
        double ex = exp(-xx);
        *I = *I * ex + E * tau * phi(xx);
        *cmp *= ex;
    } else {
        /* A = 0: I + E tau, summed with Neumaier's compensation */
        double y = E * tau;
        double t = *I + y;
        if (fabs(*I) >= fabs(y))
            *cmp += (*I - t) + y;
        else
            *cmp += (y - t) + *I;
        *I = t;
    }
}

/* Apply one particle's exact single-particle solution of Eq. (1) to the
 * three channels of pixel (i, j). */
static void apply_particle(const orc_settings *st, const vis_t *e, int i, int j, double *I,
                           double *cmp) {
    double dx = ((double)i + 0.5) - e->p.u;
    double dy = ((double)j + 0.5) - e->p.v;
    double q2 = (dx * dx + dy * dy) / (e->p.sig * e->p.sig);
    double tau = e->rho0 * column(st, q2);
    for (int ch = 0; ch < 3; ++ch) rt_step(e->E[ch], e->A[ch], tau, &I[ch], &cmp[ch]);
}

/* Paint the visible particles v[0..m) back to front on rows [ra, rb) of
 * the image (img: planar [3][H][W], holding the incoming light). */
static void paint_rows(const orc_settings *st, const vis_t *v, const int64_t *list,
                       int64_t nlist, int W, int H, int ra, int rb, double *img) {
    size_t np = (size_t)W * (size_t)H;
    double *cmp = (double *)calloc(3 * (size_t)W * (size_t)(rb - ra) + 1, sizeof(double));
    for (int64_t a = nlist - 1; a >= 0; --a) {
        const vis_t *e = &v[list ? list[a] : a];
        int j0 = e->p.j0 > ra ? e->p.j0 : ra;
        int j1 = e->p.j1 < rb - 1 ? e->p.j1 : rb - 1;
        for (int j = j0; j <= j1; ++j)
            for (int i = e->p.i0; i <= e->p.i1; ++i) {
                if (!member32(&e->p, i, j)) continue;
                size_t o = (size_t)j * W + i;
                size_t oc = (size_t)(j - ra) * W + i, pc = (size_t)W * (size_t)(rb - ra);
                double I[3] = {img[o], img[np + o], img[2 * np + o]};
                double c3[3] = {cmp[oc], cmp[pc + oc], cmp[2 * pc + oc]};
                apply_particle(st, e, i, j, I, c3);
                img[o] = I[0];
                img[np + o] = I[1];
                img[2 * np + o] = I[2];
                cmp[oc] = c3[0];
                cmp[pc + oc] = c3[1];
                cmp[2 * pc + oc] = c3[2];
            }
    }
    /* fold the carried compensation in */
    size_t pc = (size_t)W * (size_t)(rb - ra);
    for (int ch = 0; ch < 3; ++ch)
        for (int j = ra; j < rb; ++j)
            for (int i = 0; i < W; ++i)
                img[ch * np + (size_t)j * W + i] += cmp[ch * pc + (size_t)(j - ra) * W + i];
    free(cmp);
    (void)H;
}

/* Full render.  img_in (planar [3][H][W], may be NULL = zero) is the light
 * entering from behind all particles; img_out receives the result. */
int64_t orc_render(const orc_particles *P, const orc_settings *st, const float *cam,
                   int projection, int W, int H, const double *img_in, double *img_out) {
    cam64 c = cam_promote(cam, projection, W, H);
    vis_t *v;
    int64_t m = build_visible(P, st, &c, &v);
    size_t np = (size_t)W * (size_t)H;
    for (size_t q = 0; q < 3 * np; ++q) img_out[q] = img_in ? img_in[q] : 0.0;
    paint_rows(st, v, NULL, m, W, H, 0, H, img_out);
    free(v);
    return m;
}

/* The same render with the rows cut into bands of `band` rows painted by
 * the OpenMP threads (each band is the same back-to-front sequence, so the
 * image is identical to orc_render's).  For timing on many cores. */
int64_t orc_render_rows(const orc_particles *P, const orc_settings *st, const float *cam,
                        int projection, int W, int H, int band, const double *img_in,
                        double *img_out) {
    cam64 c = cam_promote(cam, projection, W, H);
    vis_t *v;
    int64_t m = build_visible(P, st, &c, &v);
    size_t np = (size_t)W * (size_t)H;
    for (size_t q = 0; q < 3 * np; ++q) img_out[q] = img_in ? img_in[q] : 0.0;
    if (band < 1) band = 1;
    int nb = (H + band - 1) / band;
    /* per band, the canonical positions of the particles whose rows meet it */
    int64_t *cnt = (int64_t *)calloc((size_t)nb + 1, sizeof(int64_t));
    for (int64_t a = 0; a < m; ++a)
        for (int b = v[a].p.j0 / band; b <= v[a].p.j1 / band; ++b) cnt[b + 1]++;
    for (int b = 0; b < nb; ++b) cnt[b + 1] += cnt[b];
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt[nb] > 0 ? cnt[nb] : 1));
    int64_t *fill = (int64_t *)calloc((size_t)nb, sizeof(int64_t));
    for (int64_t a = 0; a < m; ++a)
        for (int b = v[a].p.j0 / band; b <= v[a].p.j1 / band; ++b)
            list[cnt[b] + fill[b]++] = a;
    free(fill);
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int b = 0; b < nb; ++b) {
        int ra = b * band, rb = ra + band < H ? ra + band : H;
        paint_rows(st, v, list + cnt[b], cnt[b + 1] - cnt[b], W, H, ra, rb, img_out);
    }
    free(list);
    free(cnt);
    free(v);
    return m;
}

/* Threads the OpenMP runtime will use. */
int orc_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Render a list of sample pixels only (for checks at sizes where a full
 * FP64 image is too slow).  in_px/out_px hold 3 values per sample. */
typedef struct {
    uint32_t key;
    int64_t idx;
    int32_t sample;
    double contrib_tau, E[3], A[3];
} hit_t;

static int cmp_hit(const void *a, const void *b) {
    const hit_t *x = (const hit_t *)a, *y = (const hit_t *)b;
    if (x->sample != y->sample) return x->sample < y->sample ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

int64_t orc_render_pixels(const orc_particles *P, const orc_settings *st, const float *cam,
                          int projection, int W, int H, int64_t npx, const int32_t *pi,
                          const int32_t *pj, const double *in_px, double *out_px) {
    cam64 c = cam_promote(cam, projection, W, H);
    float lo[ORC_MAX_SPECIES], hi[ORC_MAX_SPECIES];
    orc_value_range(P, st, lo, hi);
    /* samples bucketed by row */
    int64_t *row_first = (int64_t *)calloc((size_t)H + 1, sizeof(int64_t));
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(npx > 0 ? npx : 1));
    for (int64_t s = 0; s < npx; ++s) row_first[pj[s] + 1]++;
    for (int j = 0; j < H; ++j) row_first[j + 1] += row_first[j];
    int64_t *fill = (int64_t *)calloc((size_t)H, sizeof(int64_t));
    for (int64_t s = 0; s < npx; ++s) order[row_first[pj[s]] + fill[pj[s]]++] = s;
    free(fill);
    /* The particle scan is split over threads; each keeps its own hit list.
     * The lists are concatenated and put in the total order
     * (sample, depth key, index), so the result does not depend on the
     * number of threads. */
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    hit_t **tl = (hit_t **)calloc((size_t)nthr, sizeof(hit_t *));
    size_t *tn = (size_t *)calloc((size_t)nthr, sizeof(size_t));
#ifdef _OPENMP
#pragma omp parallel num_threads(nthr)
#endif
    {
        int me = 0;
#ifdef _OPENMP
        me = omp_get_thread_num();
#endif
        size_t cap = 1024, nh = 0;
        hit_t *hits = (hit_t *)malloc(sizeof(hit_t) * cap);
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
        for (int64_t k = 0; k < P->n; ++k) {
            if (!particle_valid(P, k, st)) continue;
            proj_t p = project_one(&c, P->x[k], P->y[k], P->z[k], P->h[k],
                                   (double)st->sigma_over_h, (double)st->trunc_f);
            if (p.status != ORC_VISIBLE) continue;
            int colour_done = 0;
            double E[3], A[3];
            for (int j = p.j0; j <= p.j1; ++j)
                for (int64_t q = row_first[j]; q < row_first[j + 1]; ++q) {
                    int64_t smp = order[q];
                    if (!member32(&p, pi[smp], j)) continue;
                    if (!colour_done) {
                        particle_colour(P, k, st, lo, hi, E, A);
                        colour_done = 1;
                    }
                    if (nh == cap) {
                        cap *= 2;
                        hits = (hit_t *)realloc(hits, sizeof(hit_t) * cap);
                    }
                    hit_t *e = &hits[nh++];
                    e->key = p.key;
                    e->idx = k;
                    e->sample = (int32_t)smp;
                    double dx = ((double)pi[smp] + 0.5) - p.u;
                    double dy = ((double)j + 0.5) - p.v;
                    double q2 = (dx * dx + dy * dy) / (p.sig * p.sig);
                    e->contrib_tau = (P->rho0 ? (double)P->rho0[k] : 1.0) * column(st, q2);
                    for (int ch = 0; ch < 3; ++ch) {
                        e->E[ch] = E[ch];
                        e->A[ch] = A[ch];
                    }
                }
        }
        tl[me] = hits;
        tn[me] = nh;
    }
    size_t nh = 0;
    for (int t = 0; t < nthr; ++t) nh += tn[t];
    hit_t *hits = (hit_t *)malloc(sizeof(hit_t) * (nh > 0 ? nh : 1));
    size_t at = 0;
    for (int t = 0; t < nthr; ++t) {
        if (tn[t]) memcpy(hits + at, tl[t], tn[t] * sizeof(hit_t));
        at += tn[t];
        free(tl[t]);
    }
    free(tl);
    free(tn);
    qsort(hits, nh, sizeof(hit_t), cmp_hit);
    double *cmp = (double *)calloc(3 * (size_t)(npx > 0 ? npx : 1), sizeof(double));
    for (int64_t s = 0; s < npx; ++s)
        for (int ch = 0; ch < 3; ++ch) out_px[3 * s + ch] = in_px ? in_px[3 * s + ch] : 0.0;
    /* per sample, back to front */
    for (size_t a = nh; a-- > 0;) {
        const hit_t *e = &hits[a];
        for (int ch = 0; ch < 3; ++ch)
            rt_step(e->E[ch], e->A[ch], e->contrib_tau, &out_px[3 * e->sample + ch],
                    &cmp[3 * e->sample + ch]);
    }
    for (int64_t s = 0; s < 3 * npx; ++s) out_px[s] += cmp[s];
    free(cmp);
    free(hits);
    free(order);
    free(row_first);
    return (int64_t)nh;
}

/* ---------------------------------------------------------------------- */
/* Brute-force ray marching (orthographic cameras, tiny inputs).           */
/* ---------------------------------------------------------------------- */
/* Integrates Eq. (1) with the summed density of all particles along the
 * ray through each pixel centre, from far to near, by classical RK4.  Each
 * particle's 3-D density is (rho0/(sigma sqrt(pi))) exp(-r^2/sigma^2);
 * kernel 0 keeps it on rays of impact parameter b <= f sigma (and cuts the
 * line at 10 sigma, where it is below e^-100); kernel 1 keeps it inside
 * the sphere r <= f sigma.  The ray is cut at every particle's entry and
 * exit points, and each piece between consecutive cuts (where the
 * integrand is smooth) is marched with `steps` steps per unit sigma_min.
 * E and A per particle are given directly (E[3n], A[3n]) to keep this
 * independent of the colour mapping. */
typedef struct {
    double s0, amp, inv_s2, lo, hi, E[3], A[3];
} seg_t;

static void rhs(const seg_t *g, int m, double s, const double *I, double *dI) {
    dI[0] = dI[1] = dI[2] = 0.0;
    for (int k = 0; k < m; ++k) {
        double ds = s - g[k].s0;
        double rho = g[k].amp * exp(-ds * ds * g[k].inv_s2);
        for (int ch = 0; ch < 3; ++ch) dI[ch] += (g[k].E[ch] - g[k].A[ch] * I[ch]) * rho;
    }
}

static int cmp_double(const void *a, const void *b) {
    double x = *(const double *)a, y = *(const double *)b;
    return x < y ? -1 : (x > y);
}

int orc_raymarch(int64_t n, const float *x, const float *y, const float *z, const float *h,
                 const double *rho0, const double *E, const double *A, const float *cam,
                 int W, int H, float sigma_over_h, float trunc_f, int kernel,
                 int steps_per_sigma, const double *img_in, double *img_out) {
    cam64 c = cam_promote(cam, 0, W, H);
    seg_t *g = (seg_t *)malloc(sizeof(seg_t) * (size_t)(n > 0 ? n : 1));
    seg_t *act = (seg_t *)malloc(sizeof(seg_t) * (size_t)(n > 0 ? n : 1));
    double *cuts = (double *)malloc(sizeof(double) * (size_t)(2 * n + 2));
    double sigmin = INFINITY;
    for (int64_t k = 0; k < n; ++k) {
        double sig = (double)h[k] * (double)sigma_over_h;
        if (sig < sigmin) sigmin = sig;
    }
    double f = (double)trunc_f;
    size_t np = (size_t)W * (size_t)H;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            /* ray: world point at camera-plane offset (xc, yc), direction fwd */
            double xc = ((double)i + 0.5 - 0.5 * W) / c.ppu;
            double yc = ((double)j + 0.5 - 0.5 * H) / c.ppu;
            int m = 0;
            for (int64_t k = 0; k < n; ++k) {
                double d[3] = {(double)x[k] - c.eye[0], (double)y[k] - c.eye[1],
                               (double)z[k] - c.eye[2]};
                double px = d[0] * c.right[0] + d[1] * c.right[1] + d[2] * c.right[2];
                double py = d[0] * c.up[0] + d[1] * c.up[1] + d[2] * c.up[2];
                double pz = d[0] * c.fwd[0] + d[1] * c.fwd[1] + d[2] * c.fwd[2];
                double sig = (double)h[k] * (double)sigma_over_h;
                double b2 = (px - xc) * (px - xc) + (py - yc) * (py - yc);
                if (b2 > f * f * sig * sig) continue;
                seg_t *e = &g[m];
                e->s0 = pz;
                e->inv_s2 = 1.0 / (sig * sig);
                e->amp = rho0[k] / (sig * sqrt(ORC_PI)) * exp(-b2 / (sig * sig));
                double half = kernel == 1 ? sqrt(f * f * sig * sig - b2) : 10.0 * sig;
                e->lo = pz - half;
                e->hi = pz + half;
                for (int ch = 0; ch < 3; ++ch) {
                    e->E[ch] = E[3 * k + ch];
                    e->A[ch] = A[3 * k + ch];
                }
                cuts[2 * m] = e->lo;
                cuts[2 * m + 1] = e->hi;
                ++m;
            }
            size_t o = (size_t)j * W + i;
            double I[3] = {img_in ? img_in[o] : 0.0, img_in ? img_in[np + o] : 0.0,
                           img_in ? img_in[2 * np + o] : 0.0};
            qsort(cuts, (size_t)(2 * m), sizeof(double), cmp_double);
            /* radiation travels towards the eye: from depth max to min; with
             * x = -depth, dI/dx = sum_k (E_k - A_k I) rho_k. */
            for (int q = 2 * m - 1; q > 0; --q) {
                double s_hi = cuts[q], s_lo = cuts[q - 1];
                if (!(s_hi > s_lo)) continue;
                double mid = 0.5 * (s_lo + s_hi);
                int ma = 0;
                for (int k = 0; k < m; ++k)
                    if (g[k].lo <= mid && mid <= g[k].hi) act[ma++] = g[k];
                if (ma == 0) continue;
                long nsteps = (long)ceil((s_hi - s_lo) / sigmin * steps_per_sigma);
                if (nsteps < 4) nsteps = 4;
                double hs = (s_hi - s_lo) / (double)nsteps;
                for (long st = 0; st < nsteps; ++st) {
                    double s = s_hi - hs * (double)st;
                    double k1[3], k2[3], k3[3], k4[3], t[3];
                    rhs(act, ma, s, I, k1);
                    for (int ch = 0; ch < 3; ++ch) t[ch] = I[ch] + 0.5 * hs * k1[ch];
                    rhs(act, ma, s - 0.5 * hs, t, k2);
                    for (int ch = 0; ch < 3; ++ch) t[ch] = I[ch] + 0.5 * hs * k2[ch];
                    rhs(act, ma, s - 0.5 * hs, t, k3);
                    for (int ch = 0; ch < 3; ++ch) t[ch] = I[ch] + hs * k3[ch];
                    rhs(act, ma, s - hs, t, k4);
                    for (int ch = 0; ch < 3; ++ch)
                        I[ch] += hs / 6.0 * (k1[ch] + 2.0 * k2[ch] + 2.0 * k3[ch] + k4[ch]);
                }
            }
            img_out[o] = I[0];
            img_out[np + o] = I[1];
            img_out[2 * np + o] = I[2];
        }
    free(cuts);
    free(act);
    free(g);
    return 0;
}
