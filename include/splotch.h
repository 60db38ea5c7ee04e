/*
 * splotch.h -- C ABI of the MI355X Splotch renderer (libsplotch.so).
 *
 * The library renders a particle set into an RGB image the way Splotch
 * defines it (Jin et al., ICCS 2010):
 *   - Section 2: each particle is a Gaussian density rho0 exp(-r^2/sigma^2)
 *     cut to zero for rays passing farther than f*sigma; r, g and b are
 *     transported independently; along each ray dI/dx = (E_p - A_p I) rho_p(x)
 *     (Eq. (1)); E_p and A_p follow a scalar through a colour look-up
 *     table, and rho0 (the optical depth) may be scaled per particle.
 *   - Section 3.2: per particle, normalise its values, transform it to
 *     screen coordinates, assign its colour, find the pixels it affects and
 *     combine all contributions into the image.
 *
 * Conventions for every entry point:
 *   - Pointers marked "device" are HIP device pointers on the current
 *     device; pointers marked "host" are ordinary host memory.  The caller
 *     owns every buffer; the library keeps no reference after a call
 *     returns and allocates no device memory of its own.
 *   - Work is enqueued on params->stream (a hipStream_t; NULL = the null
 *     stream) and the call returns without waiting for the image, except
 *     that splotch_render reads back a few bytes (the pair total, the chunk
 *     plan and, if requested, the statistics), which synchronises that
 *     stream.
 *   - Errors are reported through the return status; nothing is thrown.
 *     Argument errors are detected on the host before any work is queued
 *     and leave the image untouched.  Particles with non-finite fields,
 *     h <= 0, a negative rho0 or an out-of-range species tag are not errors:
 *     they are skipped and counted in the statistics.
 *   - Calls on distinct streams with distinct workspaces may run
 *     concurrently.
 */
#ifndef SPLOTCH_H
#define SPLOTCH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SPLOTCH_OK = 0,
    SPLOTCH_E_INVALID_ARG = 1, /* a host-checkable argument is wrong */
    SPLOTCH_E_WORKSPACE = 2,   /* workspace missing or too small for n particles */
    SPLOTCH_E_DEVICE = 3,      /* a HIP runtime call failed */
    SPLOTCH_E_UNSUPPORTED = 4, /* valid but not supported (e.g. tile size) */
    SPLOTCH_E_CAPACITY = 5,    /* one particle needs more pair slots than the workspace holds */
    SPLOTCH_E_SCRATCH = 6      /* splotch_render_static: the input needs more than the
                                  library's static scratch buffer */
} splotch_status;

enum { SPLOTCH_ORTHO = 0, SPLOTCH_PERSPECTIVE = 1 };
enum { SPLOTCH_ADDITIVE = 0, SPLOTCH_ORDERED = 1 };
/* How a species' particles get their colour (Section 2, last paragraph). */
enum { SPLOTCH_COLOUR_PALETTE = 0, SPLOTCH_COLOUR_VECTOR = 1 };
/* Which column of the particle's density a pixel ray sees (Section 2,
 * first assumption: the density is set to zero beyond f sigma).
 * GAUSS2D: the cut is on the ray's impact parameter d, tau = rho0 exp(-q^2)
 *          with q = d / sigma_s, for d <= f sigma_s.
 * TRUNC3D: the density is cut to the ball r <= f sigma, so the column is
 *          tau = rho0 exp(-q^2) erf(sqrt(f^2 - q^2)).
 * Both are normalised so that the untruncated column at d = 0 is rho0. */
enum { SPLOTCH_KERNEL_GAUSS2D = 0, SPLOTCH_KERNEL_TRUNC3D = 1 };

#define SPLOTCH_MAX_SPECIES 8
#define SPLOTCH_MAX_DIM 16384 /* maximum image width and height in pixels */

/* Particle set, structure of arrays, all device pointers of n elements.
 * x, y, z: world position; h: smoothing length (sigma = sigma_over_h * h);
 * value: the scalar mapped to colour (Section 2, colour look-up table), or
 *        the first component of a vector quantity for species coloured by
 *        a vector;
 * rho0: optional density amplitude / optical-depth scale per particle
 *       (Section 2, optical depth modulated by another scalar), NULL = 1;
 * species: optional species tag per particle, NULL = species 0;
 * value_g, value_b: second and third vector components (Section 2, last
 *       paragraph: a vector's components mapped directly to r, g, b).
 *       Required when any species uses SPLOTCH_COLOUR_VECTOR, else unread
 *       (may be NULL).
 * n may be 0; n must be below 2^32. */
typedef struct splotch_particles {
    int64_t n;
    const float *x, *y, *z;
    const float *h;
    const float *value;
    const float *rho0;
    const uint8_t *species;
    const float *value_g, *value_b;
} splotch_particles;

/* Camera (host struct).  right, up, fwd: orthonormal FP32 frame with
 * right x up = fwd.  Camera coordinates of a point p are
 * (p-eye).right, (p-eye).up, (p-eye).fwd = (xc, yc, zc).  Perspective:
 * screen u = xc*F/zc + W/2, v = yc*F/zc + H/2, screen sigma = sigma*F/zc,
 * with F = focal_px.  Orthographic: the same with F/zc replaced by
 * px_per_unit.  Pixel (i, j) has its centre at (i + 1/2, j + 1/2); row 0
 * is the bottom row.  Particles with zc outside (z_near, z_far] are culled
 * whole.  The projection itself is evaluated in binary64 with the
 * operation order given in the library source, so that visibility,
 * bounding boxes and tile lists are reproducible bit for bit. */
typedef struct splotch_camera {
    int32_t projection; /* SPLOTCH_ORTHO or SPLOTCH_PERSPECTIVE */
    int32_t width, height;
    float eye[3], right[3], up[3], fwd[3];
    float focal_px;    /* perspective only, > 0 */
    float px_per_unit; /* orthographic only, > 0 */
    float z_near, z_far;
} splotch_camera;

/* Colour look-up tables (Section 2): n_entries >= 2 RGB triples, device,
 * interleaved r,g,b, float32.  A normalised scalar t in [0,1] is mapped by
 * linear interpolation at t*(n_entries-1).  rgb gives the emission colour;
 * rgb_absorb (n_entries_absorb >= 2 triples) gives the absorption colour of
 * ORDERED species, so that E and A may differ per channel (Section 2: the
 * paper's E = A restriction lifted).  rgb_absorb = NULL uses rgb for both
 * (n_entries_absorb is then ignored). */
typedef struct splotch_colourmap {
    int32_t n_entries;
    const float *rgb;
    int32_t n_entries_absorb;
    const float *rgb_absorb;
} splotch_colourmap;

/* Per-species colour and transfer settings.
 * t = (g(value) - g(vmin)) / (g(vmax) - g(vmin)) clamped to [0,1] with
 * g = log10 when log_scale (values <= 0 give t = 0) or the identity;
 * vmin >= vmax asks the library for the exact min/max of the species'
 * valid particles (positive ones only under log_scale).
 * E_p = brightness * colour(t), A_p = absorption * colour_A(t) for ORDERED
 * species and A_p = 0 for ADDITIVE species (Eq. (1)); colour_A is the
 * absorption table when the colour map has one, else the emission table.
 * Absorption equal to brightness with one table is the paper's recommended
 * E = A setting.
 * colour = SPLOTCH_COLOUR_VECTOR maps the three components (value, value_g,
 * value_b) to r, g, b directly: channel c uses t_c, the normalised c-th
 * component (same range and scale for all three; an automatic range spans
 * all three components), for both E and A. */
typedef struct splotch_species {
    float vmin, vmax;
    int32_t log_scale;
    float brightness;
    float absorption;
    int32_t mode;   /* SPLOTCH_ADDITIVE or SPLOTCH_ORDERED */
    int32_t colour; /* SPLOTCH_COLOUR_PALETTE (0) or SPLOTCH_COLOUR_VECTOR */
} splotch_species;

/* Optional statistics (host struct), filled after the render. */
typedef struct splotch_stats {
    int64_t n_visible;      /* particles that touch at least one tile */
    int64_t n_invalid;      /* non-finite fields, h <= 0, rho0 < 0, bad species */
    int64_t n_depth_culled; /* zc outside (z_near, z_far] */
    int64_t n_offscreen;    /* footprint box misses the screen */
    int64_t n_pairs;        /* (tile, particle) pairs over all chunks */
    int32_t n_chunks;       /* workspace-bounded passes */
    int32_t tile;           /* tile edge used, in pixels */
    int32_t ordered;        /* 1 if the depth-ordered path ran */
    int32_t reserved;
    float vmin[SPLOTCH_MAX_SPECIES], vmax[SPLOTCH_MAX_SPECIES]; /* ranges used */
    /* Filled only when params->profile is set: milliseconds per stage,
     * measured with HIP events on params->stream and summed over chunks:
     * [0] value range + projection, [1] depth sort + reorder,
     * [2] pair-offset scan, [3] pair emission, [4] tile sort + ranges,
     * [5] splat; the number of (pixel, particle) contributions the splat
     * composited, and how many of them came from absorbing particles. */
    float stage_ms[6];
    int64_t n_member_pairs;
    int64_t n_member_absorbing;
} splotch_stats;

/* Render settings (host struct). */
typedef struct splotch_params {
    int32_t n_species; /* 1..SPLOTCH_MAX_SPECIES */
    splotch_species species[SPLOTCH_MAX_SPECIES];
    float sigma_over_h; /* sigma_p = sigma_over_h * h_p, > 0 (default 1) */
    float trunc_f;      /* f: footprint radius f*sigma, > 0 (default 2) */
    int32_t accumulate; /* 0: image = render; 1: composite over the image (it is
                           the light entering from behind every particle) */
    int32_t compensated; /* 1: compensated (Kahan) summation of emission */
    int32_t tile;        /* tile edge in pixels: 0 (= 16), 8, 16 or 32 */
    int32_t profile;     /* 1: time each stage (needs stats) */
    int32_t seg_records; /* least records per tile-list segment (one workgroup
                            each); 0 = 1024.  Long lists are cut into segments
                            whose partial (C, T) are merged front to back:
                            this changes speed and, within rounding, how a
                            tile's sums are associated. */
    int32_t splat_variant; /* how a tile's list is walked (speed only, the
                            image is the same):
                            0 = default (1);
                            1 = one lane per pixel: the wave of each 8x8
                                block walks the records whose box meets
                                its block;
                            2 = one lane per pixel: each lane first lists
                                its member records, then composites them;
                            3 = one wave per tile, pixel state in LDS, the
                                lanes laid over each record's footprint box.
                            Other values: SPLOTCH_E_INVALID_ARG. */
    int32_t batch_streams; /* splotch_render_batch only: views in flight at
                            once, 0 or 1 = one after another on params->stream,
                            2..4 = round-robin over that many streams (the
                            caller's plus library-owned ones, forked from and
                            joined back to params->stream).  The workspace is
                            split into that many equal parts, each sized as
                            splotch_workspace_size gives for one view.
                            Other values: SPLOTCH_E_INVALID_ARG. */
    const uint8_t *tile_mask; /* device, one byte per screen tile (row-major,
                            tiles of params->tile px), or NULL = all tiles.
                            Tiles whose byte is 0 are skipped: no pairs, no
                            compositing, their pixels are left untouched. */
    void *stream;        /* hipStream_t */
    void *workspace;     /* device, >= splotch_workspace_size() bytes, 256-aligned */
    size_t workspace_bytes;
    splotch_stats *stats; /* host, may be NULL */
    int32_t kernel;      /* SPLOTCH_KERNEL_GAUSS2D (0) or SPLOTCH_KERNEL_TRUNC3D */
    int32_t emission_is_source; /* 0: Eq. (1) as written, each particle adds
                            I <- I exp(-A tau) + E tau phi(A tau),
                            phi(x) = (1 - exp(-x))/x.  1: for ORDERED species
                            E is read as the source function S = E/A, i.e.
                            Eq. (1) runs with E := A * E, and the update is
                            I <- (I - E) exp(-A tau) + E.  ADDITIVE species
                            are unaffected. */
} splotch_params;

/* Output image: planar float32 [3][height][width], device. */
typedef struct splotch_image {
    float *rgb;
    int32_t width, height;
} splotch_image;

/* Human-readable name of a status code (static string, never NULL). */
const char *splotch_status_string(splotch_status s);

/* Fill *cam with a camera at eye looking at `at` with the given up hint
 * (host arrays of 3).  projection PERSPECTIVE: fov_or_scale is the
 * horizontal field of view in degrees (0 < fov < 180); ORTHO: it is
 * px_per_unit.  Returns SPLOTCH_E_INVALID_ARG for degenerate frames. */
splotch_status splotch_camera_look_at(splotch_camera *cam, const float eye[3],
                                      const float at[3], const float up[3],
                                      int32_t projection, float fov_or_scale,
                                      int32_t width, int32_t height, float z_near,
                                      float z_far);

/* Bytes of workspace needed to render n particles at the camera's size
 * with room for max_pairs (tile, particle) pairs per pass (max_pairs <= 0
 * picks 4n + 65536).  A render whose pairs exceed the capacity runs in
 * several passes (chunks) over the same workspace.  Host only. */
splotch_status splotch_workspace_size(int64_t n, const splotch_camera *cam,
                                      const splotch_params *params, int64_t max_pairs,
                                      size_t *bytes);

/* Render particles into image (Section 2 model, Section 3.2 stages):
 * project and cull, normalise and colour, bin each particle into the
 * screen tiles its footprint box touches, order each tile's list by depth
 * (front to back, ties by particle index) when any species is ORDERED,
 * and composite every pixel.  Additive-only sets skip the depth order.
 * All pointers in the structs are as documented above; image dimensions
 * must equal the camera's. */
splotch_status splotch_render(const splotch_particles *particles, const splotch_camera *cam,
                              const splotch_colourmap *cmap, const splotch_params *params,
                              splotch_image *image);

/* Allocation-free render, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation).  Same arguments, result and errors as splotch_render, except
 * that params->workspace and params->workspace_bytes are ignored: the
 * workspace is a static device buffer of SPLOTCH_STATIC_SCRATCH_BYTES that
 * the library holds on each GPU it runs on until the process ends (its
 * address is looked up once per device, on the first call there).  The
 * call allocates no device memory.
 * Limits: the render's smallest workspace, splotch_workspace_size(n, cam,
 * params, 1, ...), must fit in the buffer, else SPLOTCH_E_SCRATCH before
 * any work is queued (about 4e6 particles at 1024x1024 with an ordered
 * species); pairs beyond what the buffer holds are rendered in several
 * passes, as with a small workspace.  params->profile must be 0 (stage
 * timing creates events), else SPLOTCH_E_INVALID_ARG.
 * Every call on one GPU uses that GPU's single buffer, which keeps the
 * last call's contents (the render clears what it needs): calls that
 * overlap on one GPU, from several host threads or on several streams,
 * race and must be serialised by the caller. */
#define SPLOTCH_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
splotch_status splotch_render_static(const splotch_particles *particles,
                                     const splotch_camera *cam, const splotch_colourmap *cmap,
                                     const splotch_params *params, splotch_image *image);

/* Stage outputs for inspection and exact comparison (Section 3.2: the
 * screen transform and footprint of each particle).  For every particle
 * (device arrays of n): status (0 visible, 1 invalid, 2 depth-culled,
 * 3 off-screen), bbox (4 int32: i0, i1, j0, j1 of its clipped pixel box),
 * spec (3 float32: u - i0, v - j0, (f sigma_s)^2, the binary32 fields that
 * decide pixel membership), depth key (uint32, monotone image of the
 * binary32 camera depth) and tile count (uint32, for params->tile).  Any
 * output pointer may be NULL.  Uses the workspace like splotch_render. */
splotch_status splotch_project(const splotch_particles *particles, const splotch_camera *cam,
                               const splotch_params *params, int8_t *status, int32_t *bbox,
                               float *spec, uint32_t *key, uint32_t *ntiles);

/* Binning outputs: the per-tile particle lists of one render pass, as the
 * splat consumes them.  tile_start/tile_end (device, n_tiles uint32 each)
 * bound each tile's slice of pair_particle (device, capacity max_out
 * uint32), which lists particle indices tile by tile, front to back for
 * depth-ordered renders and by index otherwise.  *n_pairs (host) receives
 * the pair total; SPLOTCH_E_CAPACITY if it exceeds max_out or the
 * workspace's pair capacity. */
splotch_status splotch_bin(const splotch_particles *particles, const splotch_camera *cam,
                           const splotch_params *params, uint32_t *tile_start,
                           uint32_t *tile_end, uint32_t *pair_particle, int64_t max_out,
                           int64_t *n_pairs);

/* Render n_views camera views (1..SPLOTCH_MAX_VIEWS, sizes may differ) of
 * one particle set with shared colour settings into images[v] (Section 3.2
 * stages per view).  Nothing is read back between stages: every size is
 * kept on the device, so the whole batch is one stream-ordered sequence.
 * With use_graph = 1 the sequence is captured into a HIP graph on the first
 * call and replayed by later calls whose arguments (all pointers, sizes and
 * settings) are identical; params->stream must then be a created stream
 * (not the null stream).  The workspace is sized with
 * splotch_workspace_size for the view with the most tiles, times
 * params->batch_streams when that is above 1; views are rendered one after
 * another through each part of it.  There is no chunking: a view
 * whose pairs exceed the workspace's pair capacity is left incomplete and
 * flagged.  params->tile_mask must be NULL (SPLOTCH_E_UNSUPPORTED).
 * If params->stats is not NULL it must point to n_views structs;
 * the call then waits for the batch, fills n_pairs (and tile, ordered) per
 * view, and returns SPLOTCH_E_CAPACITY if any view overflowed (its
 * n_chunks is then 0).  Without stats the call returns as soon as the work
 * is queued. */
#define SPLOTCH_MAX_VIEWS 1024
splotch_status splotch_render_batch(const splotch_particles *particles, int32_t n_views,
                                    const splotch_camera *cams, const splotch_colourmap *cmap,
                                    const splotch_params *params, splotch_image *images,
                                    int32_t use_graph);

/* Destroy every cached HIP graph (see splotch_render_batch).  Returns the
 * number destroyed. */
int32_t splotch_graph_cache_clear(void);

/* ------------------------------------------------------------------------
 * Learned decimation: kernels of the reconstruction network.  A render of
 * a seeded 1/16 particle subset is mapped back towards the full render by
 * a convolutional encoder-decoder trained on pairs this library renders.
 * All pointers are device pointers; bf16 tensors are uint16 bit patterns
 * (bfloat16, round to nearest even); activations are NHWC.  Every call is
 * asynchronous on `stream`; argument errors return SPLOTCH_E_INVALID_ARG
 * before any launch.
 * ------------------------------------------------------------------------ */

/* C[z][M][N] (float32) = sum over the z-th K range of A[m][k] * B[k][n]
 * on BF16 matrix cores with FP32 accumulation.  A is [M][K] with row
 * stride lda, or with trans_a = 1 stored as [K][M] (stride lda); B is
 * [K][N] with stride ldb.  K is cut into splotch_nn_gemm_splits(K, splits)
 * ranges; C must hold that many M x N slices (sum them with
 * splotch_nn_epilogue). */
splotch_status splotch_nn_gemm(const uint16_t *A, const uint16_t *B, float *C, int32_t M,
                               int32_t N, int32_t K, int32_t lda, int32_t ldb, int32_t trans_a,
                               int32_t splits, void *stream);
int32_t splotch_nn_gemm_splits(int32_t K, int32_t splits);

/* 3x3 patches with zero padding: out[p][tap*c + ch] = in[p + offset(tap)][ch],
 * taps (ky, kx) row-major, p = (image, y, x); in is [n][h][w][c], c a
 * multiple of 8; out is [n*h*w][9*c]. */
splotch_status splotch_nn_im2col3x3(const uint16_t *in, uint16_t *out, int32_t n, int32_t h,
                                    int32_t w, int32_t c, void *stream);

/* Weights of the adjoint convolution.  Forward weights are the GEMM
 * operand w[tap][ci][co] ([9*cin][cout]); the adjoint operand is
 * wt[tap'][co][ci] = w[8-tap'][ci][co] ([9*cout][cin]). */
splotch_status splotch_nn_flip_weights(const uint16_t *w, uint16_t *wt, int32_t cout, int32_t cin,
                                       void *stream);

/* out[r][c] = act(sum_z partials[z][r][c] + bias[c]) + residual[r][c];
 * act = ReLU when relu, else identity; bias and residual may be NULL;
 * writes out_bf16 and/or out_f32 (either may be NULL, not both). */
splotch_status splotch_nn_epilogue(const float *partials, int32_t splits, int64_t rows,
                                   int32_t cols, const float *bias, int32_t relu,
                                   const float *residual, uint16_t *out_bf16, float *out_f32,
                                   void *stream);

/* Forward-convolution weights: wf[co][tap*cin + ci] = w[tap*cin + ci][co]
 * (w is the GEMM operand [9*cin][cout]; wf is [cout][9*cin], bf16). */
splotch_status splotch_nn_conv3x3_weights(const uint16_t *w, uint16_t *wf, int32_t cin,
                                          int32_t cout, void *stream);

/* Fused 3x3 convolution, stride 1, zero padding, NHWC bf16 x [n][h][w][cin]:
 * out[p][co] = act(sum over taps and ci of x[p + offset(tap)][ci] *
 * wf[co][tap*cin + ci] + bias[co]) + residual[p][co], with the epilogue of
 * splotch_nn_epilogue and the same meaning of relu, bias, residual and the
 * two outputs.  The same result as im2col + GEMM + epilogue up to the order
 * of the FP32 accumulation, without the [n*h*w][9*cin] patch buffer.
 * cin and cout are multiples of 32, x and wf 16-byte aligned; wf comes from
 * splotch_nn_conv3x3_weights.
 * Device pointers, caller-owned; asynchronous on stream. */
splotch_status splotch_nn_conv3x3(const uint16_t *x, const uint16_t *wf, const float *bias,
                                  int32_t relu, const float *residual, uint16_t *out_bf16,
                                  float *out_f32, int32_t n, int32_t h, int32_t w, int32_t cin,
                                  int32_t cout, void *stream);

/* ReLU adjoint: dz = dy where y > 0 (or everywhere when relu = 0), as bf16
 * and optionally float32. */
splotch_status splotch_nn_relu_bwd(const float *dy, const uint16_t *y, int32_t relu,
                                   uint16_t *dz_bf16, float *dz_f32, int64_t n, void *stream);

/* out[c] = sum over rows of in[row][c], cols <= 256 (bias gradients,
 * image sums); scratch holds 1024 * cols floats. */
splotch_status splotch_nn_colsum(const float *in, int64_t rows, int32_t cols, float *out,
                                 float *scratch, void *stream);

/* 2x2 average pool [n][h][w][c] -> [n][h/2][w/2][c] (bf16) and its adjoint
 * (float32; accumulate adds into din).  The forward pool takes c a multiple
 * of 8 and 16-byte aligned in and out. */
splotch_status splotch_nn_pool2(const uint16_t *in, uint16_t *out, int32_t n, int32_t h, int32_t w,
                                int32_t c, void *stream);
splotch_status splotch_nn_pool2_bwd(const float *dout, float *din, int32_t n, int32_t h,
                                    int32_t w, int32_t c, int32_t accumulate, void *stream);

/* Nearest 2x upsample of a ([n][h/2][w/2][ca]) concatenated along channels
 * with s ([n][h][w][cs]) into out ([n][h][w][ca+cs]), and its adjoint:
 * da = 2x2 sums of the first ca channels, ds = the other cs channels.
 * The forward takes ca and cs multiples of 8 and 16-byte aligned a, s and
 * out. */
splotch_status splotch_nn_up2_concat(const uint16_t *a, int32_t ca, const uint16_t *s, int32_t cs,
                                     uint16_t *out, int32_t n, int32_t h, int32_t w,
                                     void *stream);
splotch_status splotch_nn_up2_concat_bwd(const float *dout, int32_t ca, int32_t cs, float *da,
                                         float *ds, int32_t n, int32_t h, int32_t w,
                                         void *stream);

/* Mean squared error over the first `used` of c channels of [pixels][c]:
 * grad = 2 (pred - target) / (pixels*used) (zero in unused channels);
 * loss_partials[b] (nblocks floats) sum to the squared-error total. */
splotch_status splotch_nn_mse(const float *pred, const float *target, float *grad, int64_t pixels,
                              int32_t c, int32_t used, float *loss_partials, int32_t nblocks,
                              void *stream);

/* Adam step (bias-corrected, step >= 1) on float32 master weights w with
 * moments m, v; also writes the bf16 copy when w_bf16 is not NULL. */
splotch_status splotch_nn_adam(float *w, uint16_t *w_bf16, const float *g, float *m, float *v,
                               int64_t n, float lr, float b1, float b2, float eps, int32_t step,
                               void *stream);

/* Tone map a planar [3][h][w] image into NHWC with c >= 3 channels (extra
 * channels zero): out = log1p(max(img, 0) / scale); and back (first three
 * channels): img = scale * expm1(in). */
splotch_status splotch_nn_tonemap(const float *img, int32_t h, int32_t w, float scale, int32_t c,
                                  float *out_f32, uint16_t *out_bf16, void *stream);
splotch_status splotch_nn_untonemap(const float *in, int32_t h, int32_t w, float scale, int32_t c,
                                    float *img, void *stream);

/* float32 -> bfloat16 (round to nearest even). */
splotch_status splotch_nn_f32_to_bf16(const float *in, uint16_t *out, int64_t n, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* SPLOTCH_H */
