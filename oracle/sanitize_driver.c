/*
 * Driver for sanitizer builds of the oracle -- TEST INFRASTRUCTURE ONLY
 * (only tests/ compile and run it).
 *
 * Linked with splotch_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer (any report aborts), it runs every oracle entry
 * point on small seeded inputs with every setting: orthographic and
 * perspective cameras, additive and ordered species, vector colours, an
 * absorption table, both column kernels, the source-function reading, an
 * incoming image, invalid particles, empty sets, sample pixels and the ray
 * marcher.  It prints one checksum line; the test only needs it to finish.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    const float *x, *y, *z, *h, *value, *rho0, *value_g, *value_b;
    const uint8_t *species;
} orc_particles;

typedef struct {
    int ns;
    float vmin[8], vmax[8];
    float bright[8], absorb[8];
    int log_scale[8], mode[8], colour[8];
    float sigma_over_h, trunc_f;
    int kernel, emission_is_source;
    int K, KA;
    const float *pal, *pal_abs;
} orc_settings;

void orc_value_range(const orc_particles *, const orc_settings *, float *, float *);
void orc_project(const orc_particles *, const orc_settings *, const float *, int, int, int, int,
                 int8_t *, int32_t *, float *, uint32_t *, uint32_t *, double *);
int64_t orc_render(const orc_particles *, const orc_settings *, const float *, int, int, int,
                   const double *, double *);
int64_t orc_render_rows(const orc_particles *, const orc_settings *, const float *, int, int, int,
                        int, const double *, double *);
int64_t orc_render_pixels(const orc_particles *, const orc_settings *, const float *, int, int,
                          int, int64_t, const int32_t *, const int32_t *, const double *,
                          double *);
int orc_raymarch(int64_t, const float *, const float *, const float *, const float *,
                 const double *, const double *, const double *, const float *, int, int, float,
                 float, int, int, const double *, double *);

static uint64_t rng_state = 0x243F6A8885A308D3ull;
static double uni(void) {
    rng_state = rng_state * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(rng_state >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    enum { N = 600, W = 37, H = 29, K = 16 };
    static float x[N], y[N], z[N], h[N], v[N], r0[N], vg[N], vb[N], pal[3 * K], pala[3 * K];
    static uint8_t sp[N];
    for (int k = 0; k < N; ++k) {
        x[k] = (float)(uni() * 1.4 - 0.2);
        y[k] = (float)(uni() * 1.4 - 0.2);
        z[k] = (float)(uni() * 1.5 - 0.5);
        h[k] = (float)(0.002 + 0.05 * uni() * uni());
        v[k] = (float)exp(uni() * 4.0 - 2.0);
        r0[k] = (float)(0.2 + uni());
        vg[k] = (float)(uni() * 3.0);
        vb[k] = (float)(uni() * 3.0 - 0.5);
        sp[k] = (uint8_t)(k % 3);
    }
    x[0] = NAN;
    h[1] = 0.0f;
    h[2] = -1.0f;
    sp[3] = 9;
    r0[4] = -1.0f;
    vg[5] = INFINITY;
    h[6] = 5.0f; /* covers everything */
    for (int k = 0; k < 3 * K; ++k) {
        pal[k] = (float)(k % 3 == 0 ? k / (3.0 * K) : 0.3 + 0.02 * k);
        pala[k] = (float)(1.0 - k / (3.0 * K));
    }
    float cam_ortho[16] = {0.5f, 0.5f, -1.0f, 1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 30.0f, 0.05f, 1e30f};
    float cam_persp[16] = {0.5f, 0.5f, -1.5f, 1, 0, 0, 0, 1, 0, 0, 0, 1, 32.0f, 0, 0.05f, 1e30f};
    orc_particles P = {N, x, y, z, h, v, r0, vg, vb, sp};
    orc_settings st;
    memset(&st, 0, sizeof st);
    st.ns = 3;
    for (int s = 0; s < 3; ++s) {
        st.vmin[s] = 0.0f;
        st.vmax[s] = s == 1 ? 4.0f : 0.0f;
        st.bright[s] = 0.5f + 0.2f * s;
        st.absorb[s] = s == 0 ? 0.5f : 0.9f;
        st.log_scale[s] = s == 0;
        st.mode[s] = s == 2 ? 0 : 1;
        st.colour[s] = s == 1;
    }
    st.sigma_over_h = 1.0f;
    st.trunc_f = 2.0f;
    st.K = K;
    st.pal = pal;
    double sum = 0.0;
    static double img[3 * W * H], iin[3 * W * H], out_px[3 * 40], in_px[3 * 40];
    static int8_t status[N];
    static int32_t bbox[4 * N], pi[40], pj[40];
    static float spec[3 * N];
    static uint32_t key[N], nt[N];
    static double cont[4 * N];
    for (int q = 0; q < 3 * W * H; ++q) iin[q] = 0.1 * uni();
    for (int q = 0; q < 40; ++q) {
        pi[q] = (int32_t)(uni() * W);
        pj[q] = (int32_t)(uni() * H);
    }
    for (int q = 0; q < 120; ++q) in_px[q] = 0.05;
    float lo[8], hi[8];
    for (int variant = 0; variant < 16; ++variant) {
        st.kernel = variant & 1;
        st.emission_is_source = (variant >> 1) & 1;
        st.pal_abs = (variant >> 2) & 1 ? pala : NULL;
        st.KA = st.pal_abs ? K : 0;
        const float *cam = (variant >> 3) & 1 ? cam_persp : cam_ortho;
        const int proj = (variant >> 3) & 1;
        orc_value_range(&P, &st, lo, hi);
        orc_project(&P, &st, cam, proj, W, H, 8, status, bbox, spec, key, nt, cont);
        sum += (double)orc_render(&P, &st, cam, proj, W, H, variant & 1 ? iin : NULL, img);
        for (int q = 0; q < 3 * W * H; ++q) sum += img[q];
        sum += (double)orc_render_rows(&P, &st, cam, proj, W, H, 5, iin, img);
        sum += (double)orc_render_pixels(&P, &st, cam, proj, W, H, 40, pi, pj,
                                         variant & 2 ? in_px : NULL, out_px);
        for (int q = 0; q < 120; ++q) sum += out_px[q];
    }
    orc_particles E = {0, x, y, z, h, v, r0, vg, vb, sp};
    sum += (double)orc_render(&E, &st, cam_ortho, 0, W, H, NULL, img);
    enum { M = 5 };
    double rr[M], ee[3 * M], aa[3 * M];
    for (int k = 0; k < M; ++k) {
        rr[k] = 0.5;
        for (int c = 0; c < 3; ++c) {
            ee[3 * k + c] = 0.3;
            aa[3 * k + c] = c * 0.4;
        }
    }
    static double ray[3 * 9 * 7];
    float hm[M] = {0.1f, 0.12f, 0.08f, 0.1f, 0.2f};
    for (int kern = 0; kern < 2; ++kern) {
        orc_raymarch(M, x + 10, y + 10, z + 10, hm, rr, ee, aa, cam_ortho, 9, 7, 1.0f, 2.0f, kern,
                     20, NULL, ray);
        for (int q = 0; q < 3 * 9 * 7; ++q) sum += ray[q];
    }
    printf("checksum %.17g\n", sum);
    return 0;
}
