// Learned decimation on the device: the seeded 1/keep particle subset, the
// probe tile mask, the probe's PSNR, and the render-reconstruct-probe-
// fallback sequence of splotch_render_learned.
//
// The decimated set keeps an exact seeded subset of n/keep particles (in
// index order) with smoothing lengths and density amplitudes scaled by
// keep^(1/3): a particle's emitted flux is proportional to rho0 sigma^2,
// so the expected total flux is unchanged.  The probe renders the full set
// on a seeded sample of screen tiles; its PSNR against the reconstruction,
// after the tone map T(I) = log1p(I/s) / log1p(max/s) with s the probe's
// mean, decides whether the full render replaces the reconstruction.
#include <math.h>

#include <map>
#include <mutex>

#include "../../include/splotch.h"
#include "internal.h"

using namespace splotch;

namespace {

inline hipStream_t st(void *s) { return reinterpret_cast<hipStream_t>(s); }
inline size_t al(size_t v) { return (v + 255) / 256 * 256; }

#define L_TRY(expr)                                         \
    do {                                                    \
        if ((expr) != hipSuccess) return SPLOTCH_E_DEVICE;  \
    } while (0)

__host__ __device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// A keyed bijection of [0, n): a balanced Feistel network on 2b bits
// (4^b >= n) with cycle walking back into [0, n).
struct Perm {
    uint64_t n, key;
    uint32_t half;  // b
    __device__ uint64_t round(uint64_t r, int k) const {
        return mix64(key ^ (r * 0x9E3779B97F4A7C15ull) ^ ((uint64_t)k << 58)) &
               ((1ull << half) - 1);
    }
    __device__ uint64_t once(uint64_t x) const {
        const uint64_t m = (1ull << half) - 1;
        uint64_t l = x >> half, r = x & m;
        for (int k = 0; k < 4; ++k) {
            const uint64_t t = l ^ round(r, k);
            l = r;
            r = t;
        }
        return (l << half) | r;
    }
    __device__ uint64_t operator()(uint64_t x) const {
        do {
            x = once(x);
        } while (x >= n);
        return x;
    }
};

__global__ void k_decimate_flags(Perm perm, uint64_t keep_count, uint32_t *flags) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < perm.n) flags[i] = perm(i) < keep_count ? 1u : 0u;
}

struct DecArgs {
    splotch_particles in, out;
    const uint32_t *flags, *pos;  // flag and exclusive scan
    uint64_t n;
    float scale;  // keep^(1/3)
};

__global__ void k_decimate_gather(DecArgs a) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.n || !a.flags[i]) return;
    const uint64_t o = a.pos[i];
    float *ox = const_cast<float *>(a.out.x), *oy = const_cast<float *>(a.out.y),
          *oz = const_cast<float *>(a.out.z), *oh = const_cast<float *>(a.out.h),
          *ov = const_cast<float *>(a.out.value), *orho = const_cast<float *>(a.out.rho0);
    ox[o] = a.in.x[i];
    oy[o] = a.in.y[i];
    oz[o] = a.in.z[i];
    oh[o] = a.in.h[i] * a.scale;
    ov[o] = a.in.value[i];
    orho[o] = (a.in.rho0 ? a.in.rho0[i] : 1.0f) * a.scale;
    if (a.in.species) const_cast<uint8_t *>(a.out.species)[o] = a.in.species[i];
    if (a.in.value_g) const_cast<float *>(a.out.value_g)[o] = a.in.value_g[i];
    if (a.in.value_b) const_cast<float *>(a.out.value_b)[o] = a.in.value_b[i];
}

// Tile t is probed when its keyed hash falls below frac; if none is, the
// tile with the smallest hash is.
__global__ void k_probe_mask(uint32_t n_tiles, uint64_t seed, double frac, uint8_t *mask) {
    __shared__ unsigned long long s_min;
    __shared__ int s_any;
    if (threadIdx.x == 0) {
        s_min = ~0ull;
        s_any = 0;
    }
    __syncthreads();
    const uint64_t thr = frac >= 1.0 ? ~0ull : (uint64_t)(frac * 18446744073709551616.0);
    for (uint32_t t = threadIdx.x; t < n_tiles; t += blockDim.x) {
        const uint64_t hsh = mix64(seed * 0x9E3779B97F4A7C15ull + t + 1);
        const bool on = hsh < thr;
        mask[t] = on ? 1 : 0;
        if (on) s_any = 1;
        // smallest hash with the tile in the low bits (ties broken by index)
        atomicMin(&s_min, (unsigned long long)((hsh & ~0xFFFFFFFFull) | t));
    }
    __syncthreads();
    if (threadIdx.x == 0 && !s_any) mask[(uint32_t)(s_min & 0xFFFFFFFFull)] = 1;
}

// Per probed tile, over its pixels and channels: sum and max of the probe,
// the number of pixels, and the max of the image being judged (FP64).
__global__ void k_probe_stats(const float *probe, const float *img, const uint8_t *mask, int W,
                              int H, int T, int ntx, double *part) {
    __shared__ double s_sum[256], s_max[256], s_img[256];
    const uint32_t t = blockIdx.x;
    const int tid = threadIdx.x;
    double sum = 0.0, mx = 0.0, mi = 0.0;
    int cnt = 0;
    if (mask[t]) {
        const int x0 = (int)(t % (uint32_t)ntx) * T, y0 = (int)(t / (uint32_t)ntx) * T;
        const size_t plane = (size_t)W * H;
        for (int p = tid; p < T * T; p += blockDim.x) {
            const int x = x0 + p % T, y = y0 + p / T;
            if (x >= W || y >= H) continue;
            ++cnt;
            for (int c = 0; c < 3; ++c) {
                const size_t o = c * plane + (size_t)y * W + x;
                const double v = probe[o];
                sum += v;
                mx = fmax(mx, v);
                mi = fmax(mi, (double)img[o]);
            }
        }
    }
    s_sum[tid] = sum;
    s_max[tid] = mx;
    s_img[tid] = mi;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            s_sum[tid] += s_sum[tid + o];
            s_max[tid] = fmax(s_max[tid], s_max[tid + o]);
            s_img[tid] = fmax(s_img[tid], s_img[tid + o]);
        }
        __syncthreads();
    }
    __shared__ int s_cnt;
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    if (cnt) atomicAdd(&s_cnt, cnt);
    __syncthreads();
    if (tid == 0) {
        part[4 * t] = s_sum[0];
        part[4 * t + 1] = s_max[0];
        part[4 * t + 2] = (double)s_cnt;
        part[4 * t + 3] = s_img[0];
    }
}

// Fold per-tile partials in tile order (one workgroup).  Mode 0 (stride 4):
// out[0] = mean of the probe, out[1] = its max, out[2] = number of values
// (3 per pixel), out[4] = max of the image.  Mode 1 (stride 1): out[3] =
// PSNR from the summed squared differences of the tone maps.  A dark probe
// (mean 0) gives +inf when the image is dark there too and -inf otherwise.
__global__ void k_probe_fold(const double *part, uint32_t n_tiles, int stride, int mode,
                             double *out) {
    __shared__ double s_a[256], s_b[256], s_c[256], s_d[256];
    const int tid = threadIdx.x;
    double a = 0.0, b = 0.0, c = 0.0, d = 0.0;
    for (uint32_t t = tid; t < n_tiles; t += blockDim.x) {
        a += part[(size_t)stride * t];
        if (mode == 0) {
            b = fmax(b, part[(size_t)stride * t + 1]);
            c += part[(size_t)stride * t + 2];
            d = fmax(d, part[(size_t)stride * t + 3]);
        }
    }
    s_a[tid] = a;
    s_b[tid] = b;
    s_c[tid] = c;
    s_d[tid] = d;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
            s_a[tid] += s_a[tid + o];
            s_b[tid] = fmax(s_b[tid], s_b[tid + o]);
            s_c[tid] += s_c[tid + o];
            s_d[tid] = fmax(s_d[tid], s_d[tid + o]);
        }
        __syncthreads();
    }
    if (tid == 0) {
        if (mode == 0) {
            const double nv = 3.0 * s_c[0];
            out[0] = nv > 0 ? s_a[0] / nv : 0.0;
            out[1] = s_b[0];
            out[2] = nv;
            out[4] = s_d[0];
        } else {
            const double nv = out[2];
            const double mse = nv > 0 ? s_a[0] / nv : 0.0;
            if (!(out[0] > 0.0))
                out[3] = out[4] > 0.0 ? -INFINITY : INFINITY;
            else
                out[3] = mse == 0.0 ? INFINITY : 10.0 * log10(1.0 / mse);
        }
    }
}

// Per probed tile: sum over its pixels and channels of (T(img) - T(probe))^2.
__global__ void k_probe_sqdiff(const float *img, const float *probe, const uint8_t *mask, int W,
                               int H, int T, int ntx, const double *stats, double *part) {
    __shared__ double s_sq[256];
    const uint32_t t = blockIdx.x;
    const int tid = threadIdx.x;
    double sq = 0.0;
    const double s = stats[0];
    if (mask[t] && s > 0.0) {
        const double den = log1p(stats[1] / s);
        const int x0 = (int)(t % (uint32_t)ntx) * T, y0 = (int)(t / (uint32_t)ntx) * T;
        const size_t plane = (size_t)W * H;
        for (int p = tid; p < T * T; p += blockDim.x) {
            const int x = x0 + p % T, y = y0 + p / T;
            if (x >= W || y >= H) continue;
            for (int c = 0; c < 3; ++c) {
                const size_t o = c * plane + (size_t)y * W + x;
                const double a = log1p(fmax((double)img[o], 0.0) / s) / den;
                const double b = log1p(fmax((double)probe[o], 0.0) / s) / den;
                sq += (a - b) * (a - b);
            }
        }
    }
    s_sq[tid] = sq;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) s_sq[tid] += s_sq[tid + o];
        __syncthreads();
    }
    if (tid == 0) part[t] = s_sq[0];
}

// Library-owned side stream (default priority) and events, per device.
struct Side {
    hipStream_t s;
    hipEvent_t fork, join;
};
std::mutex g_side_mu;
std::map<int, Side> g_side;

splotch_status side_stream(Side **out) {
    int dev = 0;
    L_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_side_mu);
    auto it = g_side.find(dev);
    if (it == g_side.end()) {
        Side q;
        L_TRY(hipStreamCreateWithFlags(&q.s, hipStreamNonBlocking));
        L_TRY(hipEventCreateWithFlags(&q.fork, hipEventDisableTiming));
        L_TRY(hipEventCreateWithFlags(&q.join, hipEventDisableTiming));
        it = g_side.emplace(dev, q).first;
    }
    *out = &it->second;
    return SPLOTCH_OK;
}

struct LearnedLayout {
    size_t nn, probe, part, stats, total;
};

LearnedLayout learned_layout(size_t nn_bytes, int W, int H, uint32_t n_tiles) {
    LearnedLayout L;
    size_t o = 0;
    L.nn = o;
    o += al(nn_bytes);
    L.probe = o;
    o += al((size_t)3 * W * H * 4);
    L.part = o;
    o += al((size_t)n_tiles * 4 * 8);
    L.stats = o;
    o += al(5 * 8);
    L.total = o;
    return L;
}

}  // namespace

extern "C" {

size_t splotch_decimate_workspace_bytes(int64_t n) {
    if (n < 0) return 0;
    return al((size_t)n * 4) * 2 + al(scan_u32_scratch_bytes((size_t)n));
}

splotch_status splotch_decimate(const splotch_particles *in, int32_t keep, uint64_t seed,
                                splotch_particles *out, void *workspace, size_t workspace_bytes,
                                void *stream) {
    if (!in || !out || keep < 1 || in->n < 0 || (uint64_t)in->n >= (1ull << 32))
        return SPLOTCH_E_INVALID_ARG;
    if (in->n > 0 && (!in->x || !in->y || !in->z || !in->h || !in->value))
        return SPLOTCH_E_INVALID_ARG;
    const uint64_t n = (uint64_t)in->n;
    const uint64_t m = n / (uint64_t)keep > 0 ? n / (uint64_t)keep : (n > 0 ? 1 : 0);
    if (out->n != (int64_t)m || (m > 0 && (!out->x || !out->y || !out->z || !out->h ||
                                           !out->value || !out->rho0)))
        return SPLOTCH_E_INVALID_ARG;
    if ((in->species && !out->species) || (in->value_g && !out->value_g) ||
        (in->value_b && !out->value_b))
        return SPLOTCH_E_INVALID_ARG;
    if (!workspace || workspace_bytes < splotch_decimate_workspace_bytes(in->n))
        return SPLOTCH_E_WORKSPACE;
    if (n == 0) return SPLOTCH_OK;
    hipStream_t s = st(stream);
    char *ws = static_cast<char *>(workspace);
    uint32_t *flags = reinterpret_cast<uint32_t *>(ws);
    uint32_t *pos = reinterpret_cast<uint32_t *>(ws + al(n * 4));
    void *scratch = ws + 2 * al(n * 4);
    Perm perm;
    perm.n = n;
    perm.key = mix64(seed ^ 0xD1B54A32D192ED03ull);
    perm.half = 1;
    while ((1ull << (2 * perm.half)) < n) ++perm.half;
    const unsigned grid = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_decimate_flags, dim3(grid), dim3(256), 0, s, perm, m, flags);
    L_TRY(hipGetLastError());
    L_TRY(hipMemcpyAsync(pos, flags, n * 4, hipMemcpyDeviceToDevice, s));
    L_TRY(launch_scan_u32(pos, n, scratch, s));
    DecArgs a;
    a.in = *in;
    a.out = *out;
    a.flags = flags;
    a.pos = pos;
    a.n = n;
    a.scale = (float)cbrt((double)keep);
    hipLaunchKernelGGL(k_decimate_gather, dim3(grid), dim3(256), 0, s, a);
    L_TRY(hipGetLastError());
    return SPLOTCH_OK;
}

splotch_status splotch_probe_mask(int32_t width, int32_t height, int32_t tile, float frac,
                                  uint64_t seed, uint8_t *mask, void *stream) {
    if (width <= 0 || height <= 0 || width > SPLOTCH_MAX_DIM || height > SPLOTCH_MAX_DIM ||
        (tile != 8 && tile != 16 && tile != 32 && tile != 64) || !(frac > 0.f) || !(frac <= 1.f) || !mask)
        return SPLOTCH_E_INVALID_ARG;
    const uint32_t nt = (uint32_t)((width + tile - 1) / tile) * (uint32_t)((height + tile - 1) / tile);
    hipLaunchKernelGGL(k_probe_mask, dim3(1), dim3(1024), 0, st(stream), nt, seed, (double)frac,
                       mask);
    L_TRY(hipGetLastError());
    return SPLOTCH_OK;
}

splotch_status splotch_learned_workspace_bytes(splotch_nn *net, int32_t width, int32_t height,
                                               int32_t tile, size_t *bytes) {
    size_t nn = 0;
    splotch_status r = splotch_nn_workspace_bytes(net, 1, height, width, &nn);
    if (r != SPLOTCH_OK) return r;
    if (!bytes || (tile != 8 && tile != 16 && tile != 32 && tile != 64)) return SPLOTCH_E_INVALID_ARG;
    const uint32_t nt = (uint32_t)((width + tile - 1) / tile) * (uint32_t)((height + tile - 1) / tile);
    *bytes = learned_layout(nn, width, height, nt).total;
    return SPLOTCH_OK;
}

splotch_status splotch_render_learned(const splotch_particles *full,
                                      const splotch_particles *dec, const splotch_camera *cam,
                                      const splotch_colourmap *cmap, const splotch_params *params,
                                      int32_t dec_tile, splotch_nn *net, void *nn_workspace,
                                      size_t nn_workspace_bytes, const uint8_t *probe_mask,
                                      float psnr_threshold, splotch_image *image,
                                      int32_t *used_fallback, float *probe_psnr) {
    TraceRange trace("splotch_render_learned");
    if (!full || !dec || !cam || !params || !net || !probe_mask || !image || !image->rgb ||
        !used_fallback || !probe_psnr || params->tile_mask || isnan(psnr_threshold))
        return SPLOTCH_E_INVALID_ARG;
    if (dec_tile != 0 && dec_tile != 8 && dec_tile != 16 && dec_tile != 32 && dec_tile != 64)
        return SPLOTCH_E_UNSUPPORTED;
    if (image->width != cam->width || image->height != cam->height) return SPLOTCH_E_INVALID_ARG;
    const int W = cam->width, H = cam->height;
    const int T = params->tile == 0 ? 16 : params->tile;
    if (T != 8 && T != 16 && T != 32 && T != 64) return SPLOTCH_E_UNSUPPORTED;
    const int ntx = (W + T - 1) / T, nty = (H + T - 1) / T;
    const uint32_t n_tiles = (uint32_t)(ntx * nty);
    size_t nn_bytes = 0;
    splotch_status r = splotch_nn_workspace_bytes(net, 1, H, W, &nn_bytes);
    if (r != SPLOTCH_OK) return r;
    const LearnedLayout LL = learned_layout(nn_bytes, W, H, n_tiles);
    if (!nn_workspace || nn_workspace_bytes < LL.total) return SPLOTCH_E_WORKSPACE;
    char *lw = static_cast<char *>(nn_workspace);
    float *probe = reinterpret_cast<float *>(lw + LL.probe);
    double *part = reinterpret_cast<double *>(lw + LL.part);
    double *stats = reinterpret_cast<double *>(lw + LL.stats);
    hipStream_t s = st(params->stream);
    Side *side = nullptr;
    if ((r = side_stream(&side)) != SPLOTCH_OK) return r;

    // 1. the decimated render, into the output image
    splotch_params pd = *params;
    pd.tile = dec_tile;
    pd.stats = nullptr;
    pd.profile = 0;
    if ((r = splotch_render(dec, cam, cmap, &pd, image)) != SPLOTCH_OK) return r;
    // 2. the probe (full set on the probe tiles) on the side stream, after
    // the decimated render (both use params->workspace), while the network
    // runs on the caller's stream
    L_TRY(hipEventRecord(side->fork, s));
    L_TRY(hipStreamWaitEvent(side->s, side->fork, 0));
    // 3. reconstruction in place: the tone map reads the decimated render
    // before the inverse tone map overwrites it
    if ((r = splotch_nn_reconstruct(net, image->rgb, H, W, image->rgb, lw + LL.nn, nn_bytes,
                                    params->stream)) != SPLOTCH_OK)
        return r;
    splotch_params pp = *params;
    pp.tile = T;
    pp.tile_mask = probe_mask;
    pp.stats = nullptr;
    pp.profile = 0;
    pp.accumulate = 0;
    pp.stream = side->s;
    splotch_image pimg{probe, W, H};
    if ((r = splotch_render(full, cam, cmap, &pp, &pimg)) != SPLOTCH_OK) return r;
    L_TRY(hipEventRecord(side->join, side->s));
    L_TRY(hipStreamWaitEvent(s, side->join, 0));
    // 4. probe PSNR on the device, one value read back
    hipLaunchKernelGGL(k_probe_stats, dim3(n_tiles), dim3(256), 0, s, probe, image->rgb,
                       probe_mask, W, H, T, ntx, part);
    L_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_probe_fold, dim3(1), dim3(256), 0, s, part, n_tiles, 4, 0, stats);
    L_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_probe_sqdiff, dim3(n_tiles), dim3(256), 0, s, image->rgb, probe,
                       probe_mask, W, H, T, ntx, stats, part);
    L_TRY(hipGetLastError());
    hipLaunchKernelGGL(k_probe_fold, dim3(1), dim3(256), 0, s, part, n_tiles, 1, 1, stats);
    L_TRY(hipGetLastError());
    double psnr = 0.0;
    L_TRY(hipMemcpyAsync(&psnr, stats + 3, 8, hipMemcpyDeviceToHost, s));
    L_TRY(hipStreamSynchronize(s));
    *probe_psnr = (float)psnr;
    *used_fallback = psnr < (double)psnr_threshold ? 1 : 0;
    // 5. fallback: the full render replaces the reconstruction
    if (*used_fallback) {
        splotch_params pf = *params;
        pf.stats = nullptr;
        pf.profile = 0;
        if ((r = splotch_render(full, cam, cmap, &pf, image)) != SPLOTCH_OK) return r;
    }
    return SPLOTCH_OK;
}

}  // extern "C"
