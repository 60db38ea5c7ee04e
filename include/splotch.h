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
     * [5] splat.  With profile = 2 also the number of (pixel, particle)
     * contributions the splat composited and how many of them came from
     * absorbing particles (the splat then runs its counting variant). */
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
    int32_t tile;        /* tile edge in pixels: 0 (= 16), 8, 16, 32 or 64 (64 with
                            the row walk only, splat_variant 0 or 1) */
    int32_t profile;     /* 1: time each stage (needs stats); 2: also count the
                            composited contributions; other values:
                            SPLOTCH_E_INVALID_ARG */
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
                                its block (less a box's corner blocks
                                that hold no pixel within the radius);
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
    int32_t split_pixels; /* split particles (Section 3.2): a particle whose
                            footprint box covers more pixels than this has
                            its (tile, particle) pairs written by a whole
                            workgroup instead of one thread.  0 = (W + H) / 2
                            of the camera, the paper's suggestion; < 0 =
                            never.  Speed only: the pairs and the image are
                            the same bits either way (not used with a
                            tile_mask). */
    int32_t batch_persistent; /* splotch_render_batch only: 1 = views are
                            prepared in groups of batch_streams (one per
                            stream, projection to tile lists) and each group
                            is splatted by one persistent launch whose
                            workgroups take (view, tile segment, 8x8 block)
                            units until none is left; needs the row walk
                            (splat_variant 0 or 1, else
                            SPLOTCH_E_UNSUPPORTED).  Images are the same
                            bits as with 0. */
} splotch_params;

/* Output image: planar float32 [3][height][width], device. */
typedef struct splotch_image {
    float *rgb;
    int32_t width, height;
} splotch_image;

/* Human-readable name of a status code (static string, never NULL).  The
 * argument is a plain integer so that any value a caller holds is valid;
 * one that names no splotch_status gives "unknown status". */
const char *splotch_status_string(int32_t code);

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

/* Out-of-core render (Section 3.2: the subset loop that renders one part of
 * the data while the fragments of the previous parts are combined; here
 * the combination happens on the device).  host: the particle set in host
 * memory (the same fields as splotch_particles, host pointers; pinned
 * memory lets the copies overlap the work); n may exceed 2^32.  The set is
 * copied to the device `subset` particles at a time, on a library-owned
 * stream (default priority), into two staging buffers, overlapped with the
 * work on params->stream.
 *   - Additive-only sets: each subset is rendered and added into the image.
 *   - With an ORDERED species: a first pass projects every subset and
 *     histograms the depth keys (top 20 bits of the binary32 depth image,
 *     i.e. bins 2^-11 of the depth wide); slabs are runs of bins holding at
 *     most `slab` particles; from the farthest slab to the nearest, every
 *     subset is projected again, its particles in the slab are gathered (in
 *     index order) into a device buffer and the slab is rendered over the
 *     image (C + T I_in).  The result equals splotch_render of the whole set
 *     up to rounding (the composite is associative); the whole set is read
 *     once per slab.  A depth bin with more than `slab` particles gives
 *     SPLOTCH_E_CAPACITY.
 * Automatic value ranges are those of the whole set (found in the first
 * pass).  params->workspace: splotch_stream_workspace_size bytes (device,
 * 256-aligned); params->tile_mask must be NULL.  stats (optional): counts
 * over the whole set, n_pairs and n_chunks (renders) summed.  Returns after
 * the last render is queued (the renders read back their pair totals). */
splotch_status splotch_stream_workspace_size(const splotch_particles *host, int64_t subset,
                                             int64_t slab, const splotch_camera *cam,
                                             const splotch_params *params, size_t *bytes);
splotch_status splotch_render_stream(const splotch_particles *host, int64_t subset, int64_t slab,
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

/* ------------------------------------------------------------------------
 * The reconstruction network as an object.  n_levels levels with
 * channels[l] features each (multiples of 32, <= 256); each level applies
 * two 3x3 convolutions with ReLU; the encoder halves the resolution with
 * 2x2 average pooling, the decoder doubles it with nearest upsampling and
 * concatenates the encoder features of the same level; a last 3x3
 * convolution (no activation) adds a correction to the tone-mapped input:
 *   x = log1p(I_dec / s),  y = x + net(x),  I = s expm1(y),
 * s = the mean of the decimated render (found on the device).  in_channels
 * (a multiple of 32) carries the three tone-mapped colours, the rest zero.
 * Weights live in caller-owned device memory of splotch_nn_param_bytes
 * (FP32 master weights and biases, their gradients, Adam moments, BF16
 * copies); activations in a caller-owned workspace of
 * splotch_nn_workspace_bytes for the batch shape (n images of h x w, h and
 * w multiples of 2^(n_levels-1), n h w below 2^31; other shapes are
 * SPLOTCH_E_INVALID_ARG).  The object itself is host memory; it is
 * not thread-safe.  All device work is asynchronous on `stream` except
 * create, save and load, which wait for their copies.
 * ------------------------------------------------------------------------ */
#define SPLOTCH_NN_MAX_LEVELS 8
typedef struct splotch_nn splotch_nn;
typedef struct splotch_nn_config {
    int32_t n_levels;
    int32_t channels[SPLOTCH_NN_MAX_LEVELS];
    int32_t in_channels;
} splotch_nn_config;
/* Where layer k keeps its tensors, as byte offsets: w, b, gw, gb (float32)
 * and w_bf16 into the parameter memory; x (its bf16 input), y (its output:
 * bf16, float32 for the last layer), dy and dx (float32 gradients of its
 * output and input; dx = SIZE_MAX for the first layer, which has none) into
 * the workspace laid out for the (n, h, w) given to splotch_nn_layer_info.
 * Layers are ordered: encoder levels top down (two each), decoder levels
 * from the deepest up (two each), then the output layer.  Weights are laid
 * out [tap][cin][cout], taps (ky, kx) row-major; level l runs at h >> l. */
typedef struct splotch_nn_layer {
    int32_t cin, cout, relu, level;
    size_t w, b, gw, gb, w_bf16;
    size_t x, y, dy, dx;
} splotch_nn_layer;

splotch_status splotch_nn_param_bytes(const splotch_nn_config *cfg, size_t *bytes);
/* Initialise the network in `params` (256-byte aligned): He-normal weights
 * from a seeded generator (the output layer scaled by 0.1), zero biases and
 * Adam moments, step 0. */
splotch_status splotch_nn_create(const splotch_nn_config *cfg, void *params, size_t params_bytes,
                                 uint64_t seed, void *stream, splotch_nn **net);
splotch_status splotch_nn_destroy(splotch_nn *net);
int32_t splotch_nn_n_layers(const splotch_nn *net);
int32_t splotch_nn_get_step(const splotch_nn *net);
splotch_status splotch_nn_workspace_bytes(splotch_nn *net, int32_t n, int32_t h, int32_t w,
                                          size_t *bytes);
splotch_status splotch_nn_layer_info(splotch_nn *net, int32_t k, int32_t n, int32_t h, int32_t w,
                                     splotch_nn_layer *out);
/* Network on tone-mapped NHWC input [n][h][w][in_channels] (x_f32 is the
 * residual, x_bf16 the first convolution's input); y (may be NULL) receives
 * the float32 output of the same shape.  Keeps the activations in the
 * workspace for splotch_nn_backward. */
splotch_status splotch_nn_forward(splotch_nn *net, const float *x_f32, const uint16_t *x_bf16,
                                  int32_t n, int32_t h, int32_t w, float *y, void *workspace,
                                  size_t workspace_bytes, void *stream);
/* Mean squared error over the three colour channels of y against target
 * (both [n][h][w][in_channels]) and its gradient; loss_partials (256 floats)
 * sum to the squared-error total. */
splotch_status splotch_nn_loss_grad(splotch_nn *net, const float *y, const float *target,
                                    int32_t n, int32_t h, int32_t w, float *grad,
                                    float *loss_partials, void *stream);
/* Gradients of every weight and bias for the output gradient grad_y, from
 * the activations the last splotch_nn_forward left in the workspace. */
splotch_status splotch_nn_backward(splotch_nn *net, const float *grad_y, void *workspace,
                                   size_t workspace_bytes, void *stream);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8, bias-corrected) on every layer;
 * refreshes the BF16 copies. */
splotch_status splotch_nn_adam_step(splotch_nn *net, float lr, void *stream);
/* Training checkpoint: configuration, step, seed, FP32 weights, biases and
 * Adam moments (host file, little-endian binary).  load requires the same
 * configuration and resumes from the stored step. */
splotch_status splotch_nn_save(const splotch_nn *net, const char *path, void *stream);
splotch_status splotch_nn_load(splotch_nn *net, const char *path, void *stream);
/* Image level: tone map the planar [3][h][w] decimated render with its own
 * mean, run the network, map back into out_img (may equal dec_img). */
splotch_status splotch_nn_reconstruct(splotch_nn *net, const float *dec_img, int32_t h, int32_t w,
                                      float *out_img, void *workspace, size_t workspace_bytes,
                                      void *stream);
/* One training step on n (decimated, full) render pairs: dec_imgs and
 * full_imgs are host arrays of n device pointers to planar [3][h][w]
 * images; both are tone-mapped with the decimated render's mean; forward,
 * loss, backward, Adam.  loss_partials: NULL or 256 device floats. */
splotch_status splotch_nn_train_step(splotch_nn *net, const float *const *dec_imgs,
                                     const float *const *full_imgs, int32_t n, int32_t h,
                                     int32_t w, float lr, float *loss_partials, void *workspace,
                                     size_t workspace_bytes, void *stream);

/* Decimation: an exact seeded subset of m = max(1, n / keep) particles (a
 * keyed permutation of the indices; kept particles in index order), with h
 * and rho0 multiplied by keep^(1/3) (rho0 = keep^(1/3) where in->rho0 is
 * NULL), which keeps the expected flux, proportional to rho0 sigma^2 per
 * particle.  out holds caller-allocated device arrays of out->n = m
 * elements: x, y, z, h, value, rho0, and species / value_g / value_b when
 * the input has them.  workspace: splotch_decimate_workspace_bytes(n). */
size_t splotch_decimate_workspace_bytes(int64_t n);
splotch_status splotch_decimate(const splotch_particles *in, int32_t keep, uint64_t seed,
                                splotch_particles *out, void *workspace, size_t workspace_bytes,
                                void *stream);
/* Probe tiles: mask (device, one byte per tile of `tile` px, row-major) = 1
 * for a seeded sample of about frac of the tiles (at least one). */
splotch_status splotch_probe_mask(int32_t width, int32_t height, int32_t tile, float frac,
                                  uint64_t seed, uint8_t *mask, void *stream);
splotch_status splotch_learned_workspace_bytes(splotch_nn *net, int32_t width, int32_t height,
                                               int32_t tile, size_t *bytes);
/* Learned decimated render with fallback.  Renders `dec` (the decimated
 * set, tiles of dec_tile px; 0 = 16) into image, replaces it in place by the
 * network's reconstruction, and renders `full` on the probe tiles of
 * probe_mask (tiles of params->tile px) on a library-owned stream while the
 * network runs.  The PSNR of the reconstruction against that probe, after
 * the tone map T(I) = log1p(I/s) / log1p(max/s) with s the probe's mean,
 * is computed on the device and returned in *probe_psnr (+inf when they
 * agree exactly or the probe is dark); below psnr_threshold the full render
 * replaces the image and *used_fallback = 1.  params: render settings,
 * stream and a workspace that fits both renders; params->tile_mask must be
 * NULL.  nn_workspace: splotch_learned_workspace_bytes.  Waits for the
 * probe PSNR (one value read back). */
splotch_status splotch_render_learned(const splotch_particles *full,
                                      const splotch_particles *dec, const splotch_camera *cam,
                                      const splotch_colourmap *cmap, const splotch_params *params,
                                      int32_t dec_tile, splotch_nn *net, void *nn_workspace,
                                      size_t nn_workspace_bytes, const uint8_t *probe_mask,
                                      float psnr_threshold, splotch_image *image,
                                      int32_t *used_fallback, float *probe_psnr);

#ifdef __cplusplus
}
#endif
#endif /* SPLOTCH_H */
