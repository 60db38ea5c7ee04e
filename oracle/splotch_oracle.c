/*
 * Splotch render oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously correct CPU evaluation of the Splotch render as
 * defined in Jin et al., "High-performance astrophysical visualization using
 * Splotch" (ICCS 2010), Section 2:
 *   - every particle p carries a Gaussian density rho_p(r) = rho0_p exp(-r^2/sigma_p^2)
 *     that is cut to zero for rays passing farther than f*sigma_p
 *     (Section 2, first assumption);
 *   - r, g and b are transported independently (second assumption);
 *   - along each ray the intensity obeys dI/dx = (E_p - A_p I) rho_p(x)
 *     (Section 2, Eq. (1));
 *   - E_p and A_p come from a scalar through a colour look-up table, and
 *     the optical depth may be scaled by another per-particle scalar
 *     (Section 2, last paragraph);
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
 * with tau = rho0 exp(-q^2) (the line-of-sight column of the density,
 * normalised to rho0 at zero impact parameter), q = d/sigma_s and
 * phi(x) = (1 - exp(-x))/x.  The oracle applies it back to front (painter's
 * order), starting from the input image.  With A = 0 this is a plain sum.
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

static int particle_valid(int64_t k, const float *x, const float *y, const float *z,
                          const float *h, const float *value, const float *rho0,
                          const uint8_t *species, int ns) {
    if (!finitef(x[k]) || !finitef(y[k]) || !finitef(z[k]) || !finitef(h[k]) ||
        !finitef(value[k]))
        return 0;
    if (!(h[k] > 0.0f)) return 0;
    if (species && (int)species[k] >= ns) return 0;
    if (rho0 && (!finitef(rho0[k]) || rho0[k] < 0.0f)) return 0;
    return 1;
}

/* ---------------------------------------------------------------------- */
/* Colour (Section 2: a scalar is mapped to colour through a look-up
 * table; Section 3.2: particle values are normalised before display).     */
/* ---------------------------------------------------------------------- */

/* Resolve each species' value range.  Given (vmin < vmax) ranges are kept;
 * otherwise the range is the exact min/max of the species' valid particles
 * (positive values only when the species uses a log scale). */
void orc_value_range(int64_t n, const float *x, const float *y, const float *z,
                     const float *h, const float *value, const float *rho0,
                     const uint8_t *species, int ns, const float *vmin_in,
                     const float *vmax_in, const int *log_scale, float *vmin_out,
                     float *vmax_out) {
    int have[ORC_MAX_SPECIES] = {0};
    for (int s = 0; s < ns; ++s) {
        vmin_out[s] = vmin_in[s];
        vmax_out[s] = vmax_in[s];
    }
    float lo[ORC_MAX_SPECIES], hi[ORC_MAX_SPECIES];
    for (int64_t k = 0; k < n; ++k) {
        if (!particle_valid(k, x, y, z, h, value, rho0, species, ns)) continue;
        int s = species ? species[k] : 0;
        float v = value[k];
        if (log_scale[s] && !(v > 0.0f)) continue;
        if (!have[s]) {
            lo[s] = hi[s] = v;
            have[s] = 1;
        } else {
            if (v < lo[s]) lo[s] = v;
            if (v > hi[s]) hi[s] = v;
        }
    }
    for (int s = 0; s < ns; ++s) {
        if (vmin_in[s] < vmax_in[s]) continue;
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

/* ---------------------------------------------------------------------- */
/* Projection outputs for index checks.                                    */
/* ---------------------------------------------------------------------- */
void orc_project(int64_t n, const float *x, const float *y, const float *z, const float *h,
                 const float *value, const float *rho0, const uint8_t *species, int ns,
                 const float *cam, int projection, int W, int H, float sigma_over_h,
                 float trunc_f, int tile, int8_t *status, int32_t *bbox, float *spec,
                 uint32_t *key, uint32_t *ntiles, double *cont) {
    cam64 c = cam_promote(cam, projection, W, H);
    for (int64_t k = 0; k < n; ++k) {
        proj_t p;
        memset(&p, 0, sizeof p);
        if (!particle_valid(k, x, y, z, h, value, rho0, species, ns))
            p.status = ORC_INVALID;
        else
            p = project_one(&c, x[k], y[k], z[k], h[k], (double)sigma_over_h,
                            (double)trunc_f);
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

typedef struct {
    int ns;
    const float *vmin, *vmax;
    const int *log_scale, *mode;
    const float *bright, *absorb;
} species_t;

/* Build the visible-particle list with colours, in canonical front-to-back
 * order.  Returns the count; *out is malloc'ed. */
static int64_t build_visible(int64_t n, const float *x, const float *y, const float *z,
                             const float *h, const float *value, const float *rho0,
                             const uint8_t *species, const species_t *sp, const cam64 *c,
                             float sigma_over_h, float trunc_f, int K, const float *pal,
                             vis_t **out) {
    float lo[ORC_MAX_SPECIES], hi[ORC_MAX_SPECIES];
    orc_value_range(n, x, y, z, h, value, rho0, species, sp->ns, sp->vmin, sp->vmax,
                    sp->log_scale, lo, hi);
    vis_t *v = (vis_t *)malloc(sizeof(vis_t) * (size_t)(n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t k = 0; k < n; ++k) {
        if (!particle_valid(k, x, y, z, h, value, rho0, species, sp->ns)) continue;
        proj_t p = project_one(c, x[k], y[k], z[k], h[k], (double)sigma_over_h,
                               (double)trunc_f);
        if (p.status != ORC_VISIBLE) continue;
        int s = species ? species[k] : 0;
        double t = orc_normalise(value[k], lo[s], hi[s], sp->log_scale[s]);
        double col[3];
        orc_palette(t, K, pal, col);
        vis_t e;
        e.p = p;
        e.idx = k;
        e.rho0 = rho0 ? (double)rho0[k] : 1.0;
        for (int ch = 0; ch < 3; ++ch) {
            e.E[ch] = (double)sp->bright[s] * col[ch];
            e.A[ch] = sp->mode[s] == 1 ? (double)sp->absorb[s] * col[ch] : 0.0;
        }
        v[m++] = e;
    }
    qsort(v, (size_t)m, sizeof(vis_t), cmp_canonical);
    *out = v;
    return m;
}

/* Apply one particle's exact single-particle solution of Eq. (1) to I. */
static void apply_particle(const vis_t *e, int i, int j, double *I) {
    double dx = ((double)i + 0.5) - e->p.u;
    double dy = ((double)j + 0.5) - e->p.v;
    double q2 = (dx * dx + dy * dy) / (e->p.sig * e->p.sig);
    double tau = e->rho0 * exp(-q2);
    for (int ch = 0; ch < 3; ++ch) {
        double xx = e->A[ch] * tau;
        I[ch] = I[ch] * exp(-xx) + e->E[ch] * tau * phi(xx);
    }
}

/* Full render.  img_in (planar [3][H][W], may be NULL = zero) is the light
 * entering from behind all particles; img_out receives the result. */
int64_t orc_render(int64_t n, const float *x, const float *y, const float *z, const float *h,
                   const float *value, const float *rho0, const uint8_t *species, int ns,
                   const float *vmin, const float *vmax, const int *log_scale,
                   const float *bright, const float *absorb, const int *mode,
                   const float *cam, int projection, int W, int H, float sigma_over_h,
                   float trunc_f, int K, const float *pal, const double *img_in,
                   double *img_out) {
    species_t sp = {ns, vmin, vmax, log_scale, mode, bright, absorb};
    cam64 c = cam_promote(cam, projection, W, H);
    vis_t *v;
    int64_t m = build_visible(n, x, y, z, h, value, rho0, species, &sp, &c, sigma_over_h,
                              trunc_f, K, pal, &v);
    size_t np = (size_t)W * (size_t)H;
    for (size_t q = 0; q < 3 * np; ++q) img_out[q] = img_in ? img_in[q] : 0.0;
    /* back to front: reverse canonical order */
    for (int64_t a = m - 1; a >= 0; --a) {
        const vis_t *e = &v[a];
        for (int j = e->p.j0; j <= e->p.j1; ++j)
            for (int i = e->p.i0; i <= e->p.i1; ++i) {
                if (!member32(&e->p, i, j)) continue;
                size_t o = (size_t)j * W + i;
                double I[3] = {img_out[o], img_out[np + o], img_out[2 * np + o]};
                apply_particle(e, i, j, I);
                img_out[o] = I[0];
                img_out[np + o] = I[1];
                img_out[2 * np + o] = I[2];
            }
    }
    free(v);
    return m;
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

int64_t orc_render_pixels(int64_t n, const float *x, const float *y, const float *z,
                          const float *h, const float *value, const float *rho0,
                          const uint8_t *species, int ns, const float *vmin,
                          const float *vmax, const int *log_scale, const float *bright,
                          const float *absorb, const int *mode, const float *cam,
                          int projection, int W, int H, float sigma_over_h, float trunc_f,
                          int K, const float *pal, int64_t npx, const int32_t *pi,
                          const int32_t *pj, const double *in_px, double *out_px) {
    species_t sp = {ns, vmin, vmax, log_scale, mode, bright, absorb};
    cam64 c = cam_promote(cam, projection, W, H);
    float lo[ORC_MAX_SPECIES], hi[ORC_MAX_SPECIES];
    orc_value_range(n, x, y, z, h, value, rho0, species, ns, vmin, vmax, log_scale, lo, hi);
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
        for (int64_t k = 0; k < n; ++k) {
            if (!particle_valid(k, x, y, z, h, value, rho0, species, ns)) continue;
            proj_t p = project_one(&c, x[k], y[k], z[k], h[k], (double)sigma_over_h,
                                   (double)trunc_f);
            if (p.status != ORC_VISIBLE) continue;
            int s = species ? species[k] : 0;
            int colour_done = 0;
            double col[3];
            for (int j = p.j0; j <= p.j1; ++j)
                for (int64_t q = row_first[j]; q < row_first[j + 1]; ++q) {
                    int64_t smp = order[q];
                    if (!member32(&p, pi[smp], j)) continue;
                    if (!colour_done) {
                        double t = orc_normalise(value[k], lo[s], hi[s], log_scale[s]);
                        orc_palette(t, K, pal, col);
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
                    e->contrib_tau = (rho0 ? (double)rho0[k] : 1.0) * exp(-q2);
                    for (int ch = 0; ch < 3; ++ch) {
                        e->E[ch] = (double)bright[s] * col[ch];
                        e->A[ch] = mode[s] == 1 ? (double)absorb[s] * col[ch] : 0.0;
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
    for (int64_t s = 0; s < npx; ++s)
        for (int ch = 0; ch < 3; ++ch) out_px[3 * s + ch] = in_px ? in_px[3 * s + ch] : 0.0;
    /* per sample, back to front */
    for (size_t a = nh; a-- > 0;) {
        const hit_t *e = &hits[a];
        double *I = &out_px[3 * e->sample];
        for (int ch = 0; ch < 3; ++ch) {
            double xx = e->A[ch] * e->contrib_tau;
            I[ch] = I[ch] * exp(-xx) + e->E[ch] * e->contrib_tau * phi(xx);
        }
    }
    free(hits);
    free(order);
    free(row_first);
    return (int64_t)nh;
}

/* ---------------------------------------------------------------------- */
/* Brute-force ray marching (orthographic cameras, tiny inputs).           */
/* ---------------------------------------------------------------------- */
/* Integrates Eq. (1) with the summed density of all particles along the
 * ray through each pixel centre, from far to near, by classical RK4 with
 * `steps` steps per unit sigma_min.  Each particle's 3-D density is
 * (rho0/(sigma sqrt(pi))) exp(-(b^2 + s^2)/sigma^2) for impact parameter
 * b <= f sigma, zero otherwise; its column along a ray is then
 * rho0 exp(-b^2/sigma^2).  E and A per particle are given directly
 * (E[3n], A[3n]) to keep this independent of the colour mapping. */
typedef struct {
    double s0, amp, inv_s2, E[3], A[3];
} seg_t;

static void rhs(const seg_t *g, int m, double s, const double *I, double *dI) {
    dI[0] = dI[1] = dI[2] = 0.0;
    for (int k = 0; k < m; ++k) {
        double ds = s - g[k].s0;
        double rho = g[k].amp * exp(-ds * ds * g[k].inv_s2);
        for (int ch = 0; ch < 3; ++ch) dI[ch] += (g[k].E[ch] - g[k].A[ch] * I[ch]) * rho;
    }
}

int orc_raymarch(int64_t n, const float *x, const float *y, const float *z, const float *h,
                 const double *rho0, const double *E, const double *A, const float *cam,
                 int W, int H, float sigma_over_h, float trunc_f, int steps_per_sigma,
                 const double *img_in, double *img_out) {
    cam64 c = cam_promote(cam, 0, W, H);
    seg_t *g = (seg_t *)malloc(sizeof(seg_t) * (size_t)(n > 0 ? n : 1));
    double sigmin = INFINITY;
    for (int64_t k = 0; k < n; ++k) {
        double sig = (double)h[k] * (double)sigma_over_h;
        if (sig < sigmin) sigmin = sig;
    }
    size_t np = (size_t)W * (size_t)H;
    for (int j = 0; j < H; ++j)
        for (int i = 0; i < W; ++i) {
            /* ray: world point at camera-plane offset (xc, yc), direction fwd */
            double xc = ((double)i + 0.5 - 0.5 * W) / c.ppu;
            double yc = ((double)j + 0.5 - 0.5 * H) / c.ppu;
            int m = 0;
            double smin = INFINITY, smax = -INFINITY;
            for (int64_t k = 0; k < n; ++k) {
                double d[3] = {(double)x[k] - c.eye[0], (double)y[k] - c.eye[1],
                               (double)z[k] - c.eye[2]};
                double px = d[0] * c.right[0] + d[1] * c.right[1] + d[2] * c.right[2];
                double py = d[0] * c.up[0] + d[1] * c.up[1] + d[2] * c.up[2];
                double pz = d[0] * c.fwd[0] + d[1] * c.fwd[1] + d[2] * c.fwd[2];
                double sig = (double)h[k] * (double)sigma_over_h;
                double b2 = (px - xc) * (px - xc) + (py - yc) * (py - yc);
                if (b2 > (double)trunc_f * (double)trunc_f * sig * sig) continue;
                seg_t *e = &g[m++];
                e->s0 = pz;
                e->inv_s2 = 1.0 / (sig * sig);
                e->amp = rho0[k] / (sig * sqrt(ORC_PI)) * exp(-b2 / (sig * sig));
                for (int ch = 0; ch < 3; ++ch) {
                    e->E[ch] = E[3 * k + ch];
                    e->A[ch] = A[3 * k + ch];
                }
                if (pz - 10.0 * sig < smin) smin = pz - 10.0 * sig;
                if (pz + 10.0 * sig > smax) smax = pz + 10.0 * sig;
            }
            size_t o = (size_t)j * W + i;
            double I[3] = {img_in ? img_in[o] : 0.0, img_in ? img_in[np + o] : 0.0,
                           img_in ? img_in[2 * np + o] : 0.0};
            if (m > 0) {
                long nsteps = (long)ceil((smax - smin) / sigmin * steps_per_sigma);
                double hs = (smax - smin) / (double)nsteps;
                /* radiation travels towards the eye: from depth smax to smin;
                 * with x = -depth, dI/dx = sum_k (E_k - A_k I) rho_k. */
                for (long st = 0; st < nsteps; ++st) {
                    double s = smax - hs * (double)st;
                    double k1[3], k2[3], k3[3], k4[3], t[3];
                    rhs(g, m, s, I, k1);
                    for (int ch = 0; ch < 3; ++ch) t[ch] = I[ch] + 0.5 * hs * k1[ch];
                    rhs(g, m, s - 0.5 * hs, t, k2);
                    for (int ch = 0; ch < 3; ++ch) t[ch] = I[ch] + 0.5 * hs * k2[ch];
                    rhs(g, m, s - 0.5 * hs, t, k3);
                    for (int ch = 0; ch < 3; ++ch) t[ch] = I[ch] + hs * k3[ch];
                    rhs(g, m, s - hs, t, k4);
                    for (int ch = 0; ch < 3; ++ch)
                        I[ch] += hs / 6.0 * (k1[ch] + 2.0 * k2[ch] + 2.0 * k3[ch] + k4[ch]);
                }
            }
            img_out[o] = I[0];
            img_out[np + o] = I[1];
            img_out[2 * np + o] = I[2];
        }
    free(g);
    return 0;
}
