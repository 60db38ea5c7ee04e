// Out-of-core render: particles that stay in host memory (larger than the
// device, or simply not resident) streamed to the device in subsets, the
// way Section 3.2's loop renders one subset while the previous fragments
// are combined, here with the combination done on the device.
//
// Additive-only sets: each subset is rendered and summed into the image.
// Sets with an ordered species need the global depth order, so the render
// runs in depth slabs: a first pass over all subsets projects them and
// builds a histogram of the depth keys (top 20 bits of the binary32 depth
// image); slabs are runs of histogram bins holding at most `slab`
// particles; then, from the farthest slab to the nearest, every subset is
// projected again, its particles in the slab are compacted (in index
// order) into a device slab buffer, and the slab is rendered over the
// image (C + T I_in).  Per-species automatic value ranges are taken over
// the whole set in the first pass and passed to every slab render.
//
// Host-to-device copies run on a library-owned copy stream into two staging
// buffers, overlapped with the projection, compaction and render of the
// previous subset on the caller's stream.
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <vector>

#include "../../include/splotch.h"
#include "internal.h"

using namespace splotch;

namespace {

constexpr int kBinShift = 12;  // histogram bins: the top 20 bits of a depth key
constexpr uint32_t kBins = 1u << (32 - kBinShift);

#define S_TRY(expr)                                         \
    do {                                                    \
        if ((expr) != hipSuccess) return SPLOTCH_E_DEVICE;  \
    } while (0)

inline size_t al(size_t v) { return (v + 255) / 256 * 256; }

// Which optional fields a particle set carries.
struct Fields {
    bool rho0, species, vg, vb;
};

Fields fields_of(const splotch_particles *P) {
    return Fields{P->rho0 != nullptr, P->species != nullptr, P->value_g != nullptr,
                  P->value_b != nullptr};
}

size_t soa_bytes(size_t n, Fields f) {
    size_t b = 5 * al(n * 4);
    if (f.rho0) b += al(n * 4);
    if (f.vg) b += al(n * 4);
    if (f.vb) b += al(n * 4);
    if (f.species) b += al(n);
    return b;
}

// Device structure-of-arrays views at base for n particles.
splotch_particles soa_at(char *base, size_t n, Fields f) {
    splotch_particles P;
    memset(&P, 0, sizeof P);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        char *p = base + o;
        o += al(bytes);
        return p;
    };
    P.n = (int64_t)n;
    P.x = reinterpret_cast<float *>(take(n * 4));
    P.y = reinterpret_cast<float *>(take(n * 4));
    P.z = reinterpret_cast<float *>(take(n * 4));
    P.h = reinterpret_cast<float *>(take(n * 4));
    P.value = reinterpret_cast<float *>(take(n * 4));
    if (f.rho0) P.rho0 = reinterpret_cast<float *>(take(n * 4));
    if (f.vg) P.value_g = reinterpret_cast<float *>(take(n * 4));
    if (f.vb) P.value_b = reinterpret_cast<float *>(take(n * 4));
    if (f.species) P.species = reinterpret_cast<uint8_t *>(take(n));
    return P;
}

struct StreamLayout {
    size_t stage[2], rec, cnt, key, counters, range, flags, pos, scan, hist, slab, slab_n, render;
    size_t render_bytes, total;
};

StreamLayout stream_layout(int64_t subset, int64_t slab, Fields f, size_t render_bytes) {
    StreamLayout L;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += al(bytes ? bytes : 1);
        return at;
    };
    const size_t S = (size_t)subset;
    L.stage[0] = take(soa_bytes(S, f));
    L.stage[1] = take(soa_bytes(S, f));
    L.rec = take(S * sizeof(Rec));
    L.cnt = take(S * 4);
    L.key = take(S * 4);
    L.counters = take(kCntN * 8);
    L.range = take(kRangeSlots * 4);
    L.flags = take(S * 4);
    L.pos = take(S * 4);
    L.scan = take(scan_u32_scratch_bytes(S));
    L.hist = take((size_t)kBins * 4);
    L.slab = take(soa_bytes((size_t)slab, f));
    L.slab_n = take(8);
    L.render = take(render_bytes);
    L.render_bytes = render_bytes;
    L.total = o;
    return L;
}

__global__ void k_key_hist(const uint32_t *key, size_t n, uint32_t *hist) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t k = key[i];
        if (k != kEmptyKey) atomicAdd(&hist[k >> kBinShift], 1u);
    }
}

__global__ void k_slab_flags(const uint32_t *key, size_t n, uint32_t bin_lo, uint32_t bin_hi,
                             uint32_t *flags) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x) {
        const uint32_t k = key[i];
        const uint32_t b = k >> kBinShift;
        flags[i] = (k != kEmptyKey && b >= bin_lo && b < bin_hi) ? 1u : 0u;
    }
}

// Append the flagged particles of a subset to the slab buffer at
// *slab_n + pos[i] (pos: exclusive scan of the flags), then advance *slab_n.
struct Compact {
    splotch_particles src, dst;
    const uint32_t *flags, *pos;
    size_t n;
    unsigned long long *slab_n;
};

__global__ void k_slab_compact(Compact c) {
    const unsigned long long base = *c.slab_n;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < c.n;
         i += (size_t)gridDim.x * blockDim.x) {
        if (!c.flags[i]) continue;
        const size_t o = base + c.pos[i];
        const_cast<float *>(c.dst.x)[o] = c.src.x[i];
        const_cast<float *>(c.dst.y)[o] = c.src.y[i];
        const_cast<float *>(c.dst.z)[o] = c.src.z[i];
        const_cast<float *>(c.dst.h)[o] = c.src.h[i];
        const_cast<float *>(c.dst.value)[o] = c.src.value[i];
        if (c.src.rho0) const_cast<float *>(c.dst.rho0)[o] = c.src.rho0[i];
        if (c.src.value_g) const_cast<float *>(c.dst.value_g)[o] = c.src.value_g[i];
        if (c.src.value_b) const_cast<float *>(c.dst.value_b)[o] = c.src.value_b[i];
        if (c.src.species) const_cast<uint8_t *>(c.dst.species)[o] = c.src.species[i];
    }
}

__global__ void k_slab_advance(const uint32_t *flags, const uint32_t *pos, size_t n,
                               unsigned long long *slab_n) {
    if (threadIdx.x == 0 && blockIdx.x == 0 && n > 0) *slab_n += pos[n - 1] + flags[n - 1];
}

unsigned grid_of(size_t n) {
    size_t g = (n + 255) / 256;
    return (unsigned)std::max<size_t>(1, std::min<size_t>(g, 16384));
}

// Library-owned copy stream and events, per device.
struct CopyLane {
    hipStream_t s;
    hipEvent_t copied[2], used[2];
};
std::mutex g_copy_mu;
std::map<int, CopyLane> g_copy;

splotch_status copy_lane(CopyLane **out) {
    int dev = 0;
    S_TRY(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lock(g_copy_mu);
    auto it = g_copy.find(dev);
    if (it == g_copy.end()) {
        CopyLane q;
        S_TRY(hipStreamCreateWithFlags(&q.s, hipStreamNonBlocking));
        for (int b = 0; b < 2; ++b) {
            S_TRY(hipEventCreateWithFlags(&q.copied[b], hipEventDisableTiming));
            S_TRY(hipEventCreateWithFlags(&q.used[b], hipEventDisableTiming));
        }
        it = g_copy.emplace(dev, q).first;
    }
    *out = &it->second;
    return SPLOTCH_OK;
}

// Streams every subset of the host set through the two staging buffers and
// calls work(k, device view, stream) for each on the caller's stream.
template <typename Work>
splotch_status for_each_subset(const splotch_particles *H, int64_t subset, char *ws,
                               const StreamLayout &L, Fields f, hipStream_t s, CopyLane *cl,
                               Work work) {
    const int64_t n = H->n;
    const int64_t nsub = (n + subset - 1) / subset;
    auto issue = [&](int64_t k) -> splotch_status {
        const int b = (int)(k & 1);
        const size_t first = (size_t)(k * subset);
        const size_t cnt = (size_t)std::min<int64_t>(subset, n - k * subset);
        splotch_particles D = soa_at(ws + L.stage[b], cnt, f);
        // the buffer's previous subset must be done with before it is refilled
        S_TRY(hipStreamWaitEvent(cl->s, cl->used[b], 0));
        const float *src[8] = {H->x, H->y, H->z, H->h, H->value, H->rho0, H->value_g, H->value_b};
        const float *dst[8] = {D.x, D.y, D.z, D.h, D.value, D.rho0, D.value_g, D.value_b};
        for (int q = 0; q < 8; ++q)
            if (src[q])
                S_TRY(hipMemcpyAsync(const_cast<float *>(dst[q]), src[q] + first, cnt * 4,
                                     hipMemcpyHostToDevice, cl->s));
        if (H->species)
            S_TRY(hipMemcpyAsync(const_cast<uint8_t *>(D.species), H->species + first, cnt,
                                 hipMemcpyHostToDevice, cl->s));
        S_TRY(hipEventRecord(cl->copied[b], cl->s));
        return SPLOTCH_OK;
    };
    // both buffers start free
    for (int b = 0; b < 2; ++b) S_TRY(hipEventRecord(cl->used[b], s));
    splotch_status r;
    if (nsub > 0 && (r = issue(0)) != SPLOTCH_OK) return r;
    for (int64_t k = 0; k < nsub; ++k) {
        const int b = (int)(k & 1);
        if (k + 1 < nsub && (r = issue(k + 1)) != SPLOTCH_OK) return r;
        const size_t cnt = (size_t)std::min<int64_t>(subset, n - k * subset);
        S_TRY(hipStreamWaitEvent(s, cl->copied[b], 0));
        if ((r = work(k, soa_at(ws + L.stage[b], cnt, f))) != SPLOTCH_OK) return r;
        S_TRY(hipEventRecord(cl->used[b], s));
    }
    return SPLOTCH_OK;
}

splotch_status validate_host_set(const splotch_particles *H) {
    if (!H || H->n < 0) return SPLOTCH_E_INVALID_ARG;
    if (H->n > 0 && (!H->x || !H->y || !H->z || !H->h || !H->value)) return SPLOTCH_E_INVALID_ARG;
    return SPLOTCH_OK;
}

}  // namespace

extern "C" {

splotch_status splotch_stream_workspace_size(const splotch_particles *host, int64_t subset,
                                             int64_t slab, const splotch_camera *cam,
                                             const splotch_params *params, size_t *bytes) {
    splotch_status r = validate_host_set(host);
    if (r != SPLOTCH_OK) return r;
    if (!bytes || subset < 1 || slab < 1 || (uint64_t)slab >= (1ull << 32) ||
        (uint64_t)subset >= (1ull << 32))
        return SPLOTCH_E_INVALID_ARG;
    size_t rb = 0;
    if ((r = splotch_workspace_size(std::max(subset, slab), cam, params, 0, &rb)) != SPLOTCH_OK)
        return r;
    *bytes = stream_layout(subset, slab, fields_of(host), rb).total;
    return SPLOTCH_OK;
}

splotch_status splotch_render_stream(const splotch_particles *host, int64_t subset, int64_t slab,
                                     const splotch_camera *cam, const splotch_colourmap *cmap,
                                     const splotch_params *params, splotch_image *image) {
    TraceRange trace("splotch_render_stream");
    splotch_status r = validate_host_set(host);
    if (r != SPLOTCH_OK) return r;
    if (!params || !image || !image->rgb || params->tile_mask) return SPLOTCH_E_INVALID_ARG;
    size_t need = 0;
    if ((r = splotch_stream_workspace_size(host, subset, slab, cam, params, &need)) != SPLOTCH_OK)
        return r;
    if (!params->workspace || params->workspace_bytes < need ||
        (reinterpret_cast<uintptr_t>(params->workspace) & 255u))
        return SPLOTCH_E_WORKSPACE;
    if (image->width != cam->width || image->height != cam->height) return SPLOTCH_E_INVALID_ARG;
    const Fields f = fields_of(host);
    size_t rb = 0;
    if ((r = splotch_workspace_size(std::max(subset, slab), cam, params, 0, &rb)) != SPLOTCH_OK)
        return r;
    const StreamLayout L = stream_layout(subset, slab, f, rb);
    char *ws = static_cast<char *>(params->workspace);
    hipStream_t s = reinterpret_cast<hipStream_t>(params->stream);
    CopyLane *cl = nullptr;
    if ((r = copy_lane(&cl)) != SPLOTCH_OK) return r;
    bool ordered = false, any_auto = false;
    for (int q = 0; q < params->n_species; ++q) {
        ordered |= params->species[q].mode == SPLOTCH_ORDERED;
        any_auto |= !(params->species[q].vmin < params->species[q].vmax);
    }
    // render settings of the per-subset / per-slab renders
    splotch_params rp = *params;
    rp.workspace = ws + L.render;
    rp.workspace_bytes = L.render_bytes;
    rp.stats = nullptr;
    rp.profile = 0;
    int64_t n_pairs = 0;
    int32_t n_renders = 0;
    auto render_set = [&](const splotch_particles &D) -> splotch_status {
        rp.accumulate = n_renders == 0 ? params->accumulate : 1;
        splotch_stats stt;
        rp.stats = &stt;
        splotch_status rr = splotch_render(&D, cam, cmap, &rp, image);
        rp.stats = nullptr;
        if (rr == SPLOTCH_OK) {
            n_pairs += stt.n_pairs;
            ++n_renders;
        }
        return rr;
    };

    // projection of one staged subset: record, tile count, depth key
    uint32_t *range = reinterpret_cast<uint32_t *>(ws + L.range);
    unsigned long long *counters = reinterpret_cast<unsigned long long *>(ws + L.counters);
    auto project = [&](const splotch_particles &D, const splotch_params *pp) -> splotch_status {
        ProjectArgs a;
        memset(&a, 0, sizeof a);
        a.cam = cam_dev(cam);
        a.sp = species_dev(pp);
        a.x = D.x;
        a.y = D.y;
        a.z = D.z;
        a.h = D.h;
        a.value = D.value;
        a.rho0 = D.rho0;
        a.species = D.species;
        a.value_g = D.value_g;
        a.value_b = D.value_b;
        a.n = D.n;
        a.soh = (double)pp->sigma_over_h;
        a.f = (double)pp->trunc_f;
        a.tile = pp->tile == 0 ? 16 : pp->tile;
        a.ntx = (cam->width + a.tile - 1) / a.tile;
        a.range_bits = range;
        a.rec = reinterpret_cast<Rec *>(ws + L.rec);
        a.cnt = reinterpret_cast<uint32_t *>(ws + L.cnt);
        a.key = reinterpret_cast<uint32_t *>(ws + L.key);
        a.counters = counters;
        S_TRY(launch_project(a, s));
        return SPLOTCH_OK;
    };

    // pass 1: statistics, value ranges and (ordered) the depth histogram
    uint32_t *hist = reinterpret_cast<uint32_t *>(ws + L.hist);
    std::vector<uint32_t> h_hist;
    unsigned long long cnt_host[kCntN] = {0, 0, 0, 0};
    if (ordered || any_auto || params->stats) {
        S_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(counters), 0u, 2 * kCntN, s));
        S_TRY(launch_range_init(range, s));
        if (ordered) S_TRY(launch_fill_u32(hist, 0u, kBins, s));
        r = for_each_subset(host, subset, ws, L, f, s, cl,
                            [&](int64_t, const splotch_particles &D) -> splotch_status {
                                splotch_status q = project(D, params);
                                if (q != SPLOTCH_OK || !ordered) return q;
                                hipLaunchKernelGGL(k_key_hist, dim3(grid_of((size_t)D.n)),
                                                   dim3(256), 0, s,
                                                   reinterpret_cast<uint32_t *>(ws + L.key),
                                                   (size_t)D.n, hist);
                                S_TRY(hipGetLastError());
                                return SPLOTCH_OK;
                            });
        if (r != SPLOTCH_OK) return r;
        uint32_t rng[2 * kMaxSpecies];
        S_TRY(hipMemcpyAsync(rng, range, sizeof rng, hipMemcpyDeviceToHost, s));
        S_TRY(hipMemcpyAsync(cnt_host, counters, sizeof cnt_host, hipMemcpyDeviceToHost, s));
        if (ordered) {
            h_hist.resize(kBins);
            S_TRY(hipMemcpyAsync(h_hist.data(), hist, (size_t)kBins * 4, hipMemcpyDeviceToHost,
                                 s));
        }
        S_TRY(hipStreamSynchronize(s));
        // the whole set's ranges, given to every render
        for (int q = 0; q < params->n_species; ++q) {
            if (params->species[q].vmin < params->species[q].vmax) continue;
            float lo = 0.f, hi = 0.f;
            if (rng[2 * q] != 0xFFFFFFFFu) {
                const uint32_t bl = from_order_bits_u(rng[2 * q]);
                const uint32_t bh = from_order_bits_u(rng[2 * q + 1]);
                memcpy(&lo, &bl, 4);
                memcpy(&hi, &bh, 4);
            }
            rp.species[q].vmin = lo;
            rp.species[q].vmax = hi;
        }
    }

    if (!ordered) {
        // additive: every subset rendered and summed into the image
        r = for_each_subset(host, subset, ws, L, f, s, cl,
                            [&](int64_t, const splotch_particles &D) { return render_set(D); });
        if (r != SPLOTCH_OK) return r;
    } else {
        // slabs: runs of histogram bins with at most `slab` particles
        std::vector<std::pair<uint32_t, uint32_t>> slabs;  // [bin_lo, bin_hi)
        uint64_t acc = 0;
        uint32_t lo = 0;
        for (uint32_t b = 0; b < kBins; ++b) {
            const uint64_t c = h_hist[b];
            if (c > (uint64_t)slab) return SPLOTCH_E_CAPACITY;  // one depth bin exceeds a slab
            if (acc + c > (uint64_t)slab) {
                slabs.push_back({lo, b});
                lo = b;
                acc = 0;
            }
            acc += c;
        }
        if (acc > 0) slabs.push_back({lo, kBins});
        unsigned long long *slab_n = reinterpret_cast<unsigned long long *>(ws + L.slab_n);
        uint32_t *flags = reinterpret_cast<uint32_t *>(ws + L.flags);
        uint32_t *pos = reinterpret_cast<uint32_t *>(ws + L.pos);
        for (size_t q = slabs.size(); q-- > 0;) {  // farthest slab first
            const uint32_t blo = slabs[q].first, bhi = slabs[q].second;
            uint64_t count = 0;
            for (uint32_t b = blo; b < bhi; ++b) count += h_hist[b];
            // the slab buffer's fields are laid out for `slab` particles
            splotch_particles S = soa_at(ws + L.slab, (size_t)slab, f);
            S.n = (int64_t)count;
            S_TRY(launch_fill_u32(reinterpret_cast<uint32_t *>(slab_n), 0u, 2, s));
            r = for_each_subset(
                host, subset, ws, L, f, s, cl,
                [&](int64_t, const splotch_particles &D) -> splotch_status {
                    splotch_status qq = project(D, &rp);
                    if (qq != SPLOTCH_OK) return qq;
                    const size_t n = (size_t)D.n;
                    hipLaunchKernelGGL(k_slab_flags, dim3(grid_of(n)), dim3(256), 0, s,
                                       reinterpret_cast<uint32_t *>(ws + L.key), n, blo, bhi,
                                       flags);
                    S_TRY(hipGetLastError());
                    S_TRY(hipMemcpyAsync(pos, flags, n * 4, hipMemcpyDeviceToDevice, s));
                    S_TRY(launch_scan_u32(pos, n, ws + L.scan, s));
                    Compact c;
                    c.src = D;
                    c.dst = soa_at(ws + L.slab, (size_t)slab, f);
                    c.flags = flags;
                    c.pos = pos;
                    c.n = n;
                    c.slab_n = slab_n;
                    hipLaunchKernelGGL(k_slab_compact, dim3(grid_of(n)), dim3(256), 0, s, c);
                    S_TRY(hipGetLastError());
                    hipLaunchKernelGGL(k_slab_advance, dim3(1), dim3(64), 0, s, flags, pos, n,
                                       slab_n);
                    S_TRY(hipGetLastError());
                    return SPLOTCH_OK;
                });
            if (r != SPLOTCH_OK) return r;
            if ((r = render_set(S)) != SPLOTCH_OK) return r;
        }
    }
    if (n_renders == 0) {
        // nothing visible: the image is still written (cleared or kept)
        splotch_particles E;
        memset(&E, 0, sizeof E);
        if ((r = render_set(E)) != SPLOTCH_OK) return r;
    }
    if (params->stats) {
        splotch_stats *st = params->stats;
        memset(st, 0, sizeof *st);
        st->n_visible = (int64_t)cnt_host[kCntVisible];
        st->n_invalid = (int64_t)cnt_host[kCntInvalid];
        st->n_depth_culled = (int64_t)cnt_host[kCntDepth];
        st->n_offscreen = (int64_t)cnt_host[kCntOffscreen];
        st->n_pairs = n_pairs;
        st->n_chunks = n_renders;
        st->tile = params->tile == 0 ? 16 : params->tile;
        st->ordered = ordered ? 1 : 0;
        for (int q = 0; q < params->n_species; ++q) {
            st->vmin[q] = rp.species[q].vmin;
            st->vmax[q] = rp.species[q].vmax;
        }
    }
    return SPLOTCH_OK;
}

}  // extern "C"
