// Host side of libsplotch: argument validation, workspace layout, stage
// orchestration on the caller's stream, chunking when the (tile, particle)
// pairs exceed the workspace, and the C ABI declared in include/splotch.h.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <list>
#include <map>
#include <mutex>
#include <utility>
#include <vector>

#include "../../include/splotch.h"
#include "internal.h"

using namespace splotch;

namespace {

constexpr uint32_t kMaxChunks = 4096;
constexpr uint64_t kMaxPairCap = 0xFFFF0000ull;  // pair indices are 32-bit
constexpr uint32_t kSegMin = 1024;               // least records per list segment
constexpr int kMaxLanes = 4;                     // batch views in flight at once
static_assert(kMaxLanes <= kMaxGroup, "a persistent group holds one view per lane");

struct Layout {
    size_t rec, cnt, key0, key1, val0, val1, off, scan, radix, counters, range, bounds;
    size_t tstart, tend, mcount, seg_len, nseg, nmulti, seg_off, part_off, seg_scan, item_tile;
    size_t partial, flags, sargs, unit_next, split, split_cnt, split_off;
    size_t pk0, pk1, pv0, pv1;
    uint64_t max_items, max_slots;
    size_t total;
    uint64_t pair_cap;
    uint32_t n_tiles;
    int ntx, nty, tile;
    bool ordered;
};

int tile_of(const splotch_params *p) { return p->tile == 0 ? 16 : p->tile; }

bool any_ordered(const splotch_params *p) {
    for (int s = 0; s < p->n_species; ++s)
        if (p->species[s].mode == SPLOTCH_ORDERED) return true;
    return false;
}

// Lay out the workspace for n particles and pair capacity cap.
Layout layout(int64_t n, const splotch_camera *cam, const splotch_params *p, uint64_t cap) {
    Layout L;
    memset(&L, 0, sizeof L);
    L.tile = tile_of(p);
    L.ntx = (cam->width + L.tile - 1) / L.tile;
    L.nty = (cam->height + L.tile - 1) / L.tile;
    L.n_tiles = (uint32_t)(L.ntx * L.nty);
    L.ordered = any_ordered(p);
    L.pair_cap = cap;
    const size_t N = (size_t)n;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += align_up(bytes ? bytes : 1, 256);
        return at;
    };
    L.rec = take(N * sizeof(Rec));
    L.cnt = take(N * 4);
    if (L.ordered) {
        L.key0 = take(N * 4);
        L.key1 = take(N * 4);
        L.val0 = take(N * 4);
        L.val1 = take(N * 4);
    }
    L.off = take((N + 1) * 8);
    // split particles: a queue part and a count per emission workgroup and
    // the counts' scan (the dense queue reuses cnt, which the pair-offset
    // scan has consumed by then, and the scan's scratch that of that scan)
    const size_t emit_groups = (N + kEmitGroup - 1) / kEmitGroup;
    L.split = take(emit_groups * kEmitGroup * 4);
    L.split_cnt = take(emit_groups * 4);
    L.split_off = take((emit_groups + 1) * 8);
    L.scan = take(scan_u32_u64_scratch_bytes(N));
    L.radix = take(radix_scratch_bytes(std::max<size_t>(L.ordered ? N : 0, (size_t)cap)));
    L.counters = take(kCntN * 8);
    L.range = take(kRangeSlots * 4);
    L.bounds = take((2 + 2 * (kMaxChunks + 1)) * 8);
    L.tstart = take((size_t)L.n_tiles * 4);
    L.tend = take((size_t)L.n_tiles * 4);
    L.mcount = take((size_t)L.n_tiles * 16);
    // segments: seg_len >= max(seg_min, pairs / kSegTarget) keeps the number
    // of items <= n_tiles + kSegTarget; a tile of L > seg_len records has
    // ceil(L / seg_len) < 2 L / seg_len segments, so the partial slots of a
    // pass number < 2 pairs / seg_len <= 2 min(kSegTarget, cap / seg_min)
    const uint64_t seg_min = p->seg_records > 0 ? (uint64_t)p->seg_records : kSegMin;
    L.max_items = (uint64_t)L.n_tiles + kSegTarget + 64;
    L.max_slots = std::min<uint64_t>(2 * kSegTarget, 2 * (cap / seg_min) + 2);
    L.seg_len = take(4);
    L.flags = take((size_t)SPLOTCH_MAX_VIEWS * 12);  // per view: overflow flag (u32), pairs (u64)
    L.sargs = take(kMaxGroup * sizeof(SplatArgs));    // splat settings of a persistent group
    L.unit_next = take(kUnitCounters * 4);            // its per-XCD unit counters
    L.nseg = take((size_t)L.n_tiles * 4);
    L.nmulti = take((size_t)L.n_tiles * 4);
    L.seg_off = take(((size_t)L.n_tiles + 1) * 8);
    L.part_off = take(((size_t)L.n_tiles + 1) * 8);
    L.seg_scan = take(scan_u32_u64_scratch_bytes(L.n_tiles));
    L.item_tile = take(L.max_items * 4);
    L.partial = take(L.max_slots * 6 * (size_t)L.tile * L.tile * 4);
    L.pk0 = take(cap * 4);
    L.pk1 = take(cap * 4);
    L.pv0 = take(cap * 4);
    L.pv1 = take(cap * 4);
    L.total = o;
    return L;
}

// Largest pair capacity whose layout fits in `bytes`.
bool fit_capacity(int64_t n, const splotch_camera *cam, const splotch_params *p, size_t bytes,
                  Layout *out) {
    Layout L0 = layout(n, cam, p, 1);
    if (L0.total > bytes) return false;
    uint64_t lo = 1, hi = kMaxPairCap;
    // per pair: 16 bytes plus about 0.26 bytes of radix scratch
    uint64_t guess = (uint64_t)((bytes - L0.total) / 16.3);
    hi = std::min<uint64_t>(hi, guess + 4096);
    while (lo < hi) {
        uint64_t mid = lo + (hi - lo + 1) / 2;
        if (layout(n, cam, p, mid).total <= bytes)
            lo = mid;
        else
            hi = mid - 1;
    }
    *out = layout(n, cam, p, lo);
    return true;
}

bool finite3(const float *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

splotch_status validate_camera(const splotch_camera *c) {
    if (!c) return SPLOTCH_E_INVALID_ARG;
    if (c->projection != SPLOTCH_ORTHO && c->projection != SPLOTCH_PERSPECTIVE)
        return SPLOTCH_E_INVALID_ARG;
    if (c->width <= 0 || c->height <= 0 || c->width > SPLOTCH_MAX_DIM ||
        c->height > SPLOTCH_MAX_DIM)
        return SPLOTCH_E_INVALID_ARG;
    if (!finite3(c->eye) || !finite3(c->right) || !finite3(c->up) || !finite3(c->fwd))
        return SPLOTCH_E_INVALID_ARG;
    const float *b[3] = {c->right, c->up, c->fwd};
    for (int a = 0; a < 3; ++a)
        for (int q = 0; q < 3; ++q) {
            double d = (double)b[a][0] * b[q][0] + (double)b[a][1] * b[q][1] +
                       (double)b[a][2] * b[q][2];
            if (fabs(d - (a == q ? 1.0 : 0.0)) > 1e-5) return SPLOTCH_E_INVALID_ARG;
        }
    if (c->projection == SPLOTCH_PERSPECTIVE) {
        if (!(c->focal_px > 0.0f) || !isfinite(c->focal_px)) return SPLOTCH_E_INVALID_ARG;
        if (!(c->z_near > 0.0f)) return SPLOTCH_E_INVALID_ARG;
    } else {
        if (!(c->px_per_unit > 0.0f) || !isfinite(c->px_per_unit)) return SPLOTCH_E_INVALID_ARG;
    }
    if (isnan(c->z_near) || isnan(c->z_far) || !(c->z_far > c->z_near))
        return SPLOTCH_E_INVALID_ARG;
    return SPLOTCH_OK;
}

splotch_status validate_params(const splotch_params *p) {
    if (!p) return SPLOTCH_E_INVALID_ARG;
    if (p->n_species < 1 || p->n_species > SPLOTCH_MAX_SPECIES) return SPLOTCH_E_INVALID_ARG;
    if (!(p->sigma_over_h > 0.0f) || !isfinite(p->sigma_over_h)) return SPLOTCH_E_INVALID_ARG;
    if (!(p->trunc_f > 0.0f) || !isfinite(p->trunc_f)) return SPLOTCH_E_INVALID_ARG;
    if (p->tile != 0 && p->tile != 8 && p->tile != 16 && p->tile != 32 && p->tile != 64)
        return SPLOTCH_E_UNSUPPORTED;
    // 64 px tiles only with the row walk (the other strategies hold a whole
    // tile in one workgroup)
    if (p->tile == 64 && p->splat_variant != 0 && p->splat_variant != 1)
        return SPLOTCH_E_UNSUPPORTED;
    if (p->accumulate != 0 && p->accumulate != 1) return SPLOTCH_E_INVALID_ARG;
    if (p->seg_records < 0) return SPLOTCH_E_INVALID_ARG;
    if (p->profile < 0 || p->profile > 2) return SPLOTCH_E_INVALID_ARG;
    if (p->splat_variant < 0 || p->splat_variant > 3) return SPLOTCH_E_INVALID_ARG;
    if (p->batch_streams < 0 || p->batch_streams > kMaxLanes) return SPLOTCH_E_INVALID_ARG;
    if (p->batch_persistent != 0 && p->batch_persistent != 1) return SPLOTCH_E_INVALID_ARG;
    // the persistent batch splat is a row walk
    if (p->batch_persistent && p->splat_variant != 0 && p->splat_variant != 1)
        return SPLOTCH_E_UNSUPPORTED;
    for (int s = 0; s < p->n_species; ++s) {
        const splotch_species &q = p->species[s];
        if (q.mode != SPLOTCH_ADDITIVE && q.mode != SPLOTCH_ORDERED) return SPLOTCH_E_INVALID_ARG;
        if (!isfinite(q.brightness) || !isfinite(q.absorption) || q.absorption < 0.0f)
            return SPLOTCH_E_INVALID_ARG;
        if (isnan(q.vmin) || isnan(q.vmax)) return SPLOTCH_E_INVALID_ARG;
        if (q.log_scale && q.vmin < q.vmax && !(q.vmin > 0.0f)) return SPLOTCH_E_INVALID_ARG;
        if (q.colour != SPLOTCH_COLOUR_PALETTE && q.colour != SPLOTCH_COLOUR_VECTOR)
            return SPLOTCH_E_INVALID_ARG;
    }
    if (p->kernel != SPLOTCH_KERNEL_GAUSS2D && p->kernel != SPLOTCH_KERNEL_TRUNC3D)
        return SPLOTCH_E_INVALID_ARG;
    if (p->emission_is_source != 0 && p->emission_is_source != 1) return SPLOTCH_E_INVALID_ARG;
    return SPLOTCH_OK;
}

splotch_status validate_particles(const splotch_particles *P) {
    if (!P || P->n < 0 || (uint64_t)P->n >= (1ull << 32)) return SPLOTCH_E_INVALID_ARG;
    if (P->n > 0 && (!P->x || !P->y || !P->z || !P->h || !P->value)) return SPLOTCH_E_INVALID_ARG;
    return SPLOTCH_OK;
}

}  // namespace

namespace splotch {

CamDev cam_dev(const splotch_camera *c) {
    CamDev d;
    for (int k = 0; k < 3; ++k) {
        d.eye[k] = c->eye[k];
        d.right[k] = c->right[k];
        d.up[k] = c->up[k];
        d.fwd[k] = c->fwd[k];
    }
    d.focal = c->focal_px;
    d.ppu = c->px_per_unit;
    d.znear = c->z_near;
    d.zfar = c->z_far;
    d.half_w = 0.5 * (double)c->width;
    d.half_h = 0.5 * (double)c->height;
    d.wmax = (double)(c->width - 1);
    d.hmax = (double)(c->height - 1);
    d.persp = c->projection == SPLOTCH_PERSPECTIVE;
    d.width = c->width;
    d.height = c->height;
    return d;
}

SpeciesDev species_dev(const splotch_params *p) {
    SpeciesDev s;
    memset(&s, 0, sizeof s);
    s.n = p->n_species;
    for (int k = 0; k < p->n_species; ++k) {
        const splotch_species &q = p->species[k];
        s.vmin[k] = q.vmin;
        s.vmax[k] = q.vmax;
        s.brightness[k] = q.brightness;
        s.absorption[k] = q.absorption;
        s.log_scale[k] = q.log_scale ? 1 : 0;
        s.ordered[k] = q.mode == SPLOTCH_ORDERED;
        s.auto_range[k] = !(q.vmin < q.vmax);
        s.vector[k] = q.colour == SPLOTCH_COLOUR_VECTOR;
        s.any_vector |= s.vector[k];
    }
    return s;
}

}  // namespace splotch

namespace {

splotch_status validate_colourmap(const splotch_colourmap *m) {
    if (!m || m->n_entries < 2 || !m->rgb) return SPLOTCH_E_INVALID_ARG;
    if (m->rgb_absorb && m->n_entries_absorb < 2) return SPLOTCH_E_INVALID_ARG;
    return SPLOTCH_OK;
}

// Colour and column settings of the splat (shared by single and batched
// renders).
void splat_colour_args(SplatArgs *sa, const splotch_particles *P, const splotch_colourmap *m,
                       const splotch_params *p) {
    sa->palette = m->rgb;
    sa->n_pal = m->n_entries;
    sa->pal_abs = m->rgb_absorb;
    sa->n_pal_abs = m->rgb_absorb ? m->n_entries_absorb : 0;
    sa->value_g = P->value_g;
    sa->value_b = P->value_b;
    sa->kernel3d = p->kernel == SPLOTCH_KERNEL_TRUNC3D ? 1 : 0;
    sa->source = p->emission_is_source ? 1 : 0;
    sa->sp = species_dev(p);
    // E = A for every record of an ordered species with equal brightness
    // and absorption, one colour table and E read as emission (Section 2's
    // recommended setting); anything else may give E != A
    sa->general = 0;
    for (int s = 0; s < p->n_species; ++s) {
        const splotch_species &q = p->species[s];
        if (q.mode != SPLOTCH_ORDERED || q.absorption == 0.0f) continue;
        if (q.brightness != q.absorption || m->rgb_absorb || p->emission_is_source)
            sa->general = 1;
    }
}

#define TRY(expr)                                      \
    do {                                               \
        if ((expr) != hipSuccess) return SPLOTCH_E_DEVICE; \
    } while (0)

// Names of the stages in the timer and in the trace markers.
const char *const kStageName[] = {"splotch: project", "splotch: depth sort", "splotch: scan",
                                  "splotch: emit", "splotch: tile sort", "splotch: splat"};

// Stage timer: HIP events recorded on the render's stream between stages,
// and a trace marker at the end of each stage's launches.
struct Prof {
    bool on = false;
    hipStream_t s = nullptr;
    std::vector<hipEvent_t> ev;
    std::vector<int> stage;  // stage of the interval ending at ev[k]
    hipError_t start(bool enable, hipStream_t st) {
        on = enable;
        s = st;
        if (!on) return hipSuccess;
        return mark(-1);
    }
    hipError_t mark(int stg) {
        if (stg >= 0 && stg < 6) roctxMarkA(kStageName[stg]);
        if (!on) return hipSuccess;
        hipEvent_t e;
        hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) return r;
        ev.push_back(e);
        stage.push_back(stg);
        return hipEventRecord(e, s);
    }
    // Sum intervals per stage (synchronises the stream).
    hipError_t finish(float *ms, int nstages) {
        if (!on) return hipSuccess;
        hipError_t r = hipStreamSynchronize(s);
        for (int k = 0; k < nstages; ++k) ms[k] = 0.0f;
        for (size_t k = 1; k < ev.size() && r == hipSuccess; ++k) {
            float t = 0.0f;
            r = hipEventElapsedTime(&t, ev[k - 1], ev[k]);
            if (stage[k] >= 0 && stage[k] < nstages) ms[stage[k]] += t;
        }
        return r;
    }
    ~Prof() {
        for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    }
};

// Split threshold in pixels of a footprint box (Section 3.2: particles
// influencing more pixels than a threshold are split; about the mean of
// the window's width and height works well): 0 = (W + H) / 2, negative =
// no splitting.
uint64_t split_threshold(const splotch_params *p, const splotch_camera *cam) {
    if (p->split_pixels < 0) return 0;
    if (p->split_pixels == 0) return (uint64_t)(cam->width + cam->height) / 2;
    return (uint64_t)p->split_pixels;
}

// Public splat_variant -> walking strategy (0 = the default).
int splat_variant_of(int v) {
    switch (v) {
        case 2: return kSplatLists;
        case 3: return kSplatBox;
        default: return kSplatRows;
    }
}

struct Ctx {
    Layout L;
    char *ws;
    hipStream_t s;
    uint64_t split = 0;  // split threshold in pixels, 0 = no splitting
    uint32_t seg_min = kSegMin;
    const uint8_t *tile_mask = nullptr;
    Prof prof;
    template <typename T>
    T *at(size_t off) const {
        return reinterpret_cast<T *>(ws + off);
    }
};

// Stage 1: auto value ranges + projection.  Fills rec, cnt, key0 (if ordered).
splotch_status run_project(const Ctx &c, const splotch_particles *P, const splotch_camera *cam,
                           const splotch_params *p, int8_t *o_status, int32_t *o_bbox,
                           float *o_spec, uint32_t *o_key) {
    ProjectArgs a;
    memset(&a, 0, sizeof a);
    a.cam = cam_dev(cam);
    a.sp = species_dev(p);
    a.x = P->x;
    a.y = P->y;
    a.z = P->z;
    a.h = P->h;
    a.value = P->value;
    a.rho0 = P->rho0;
    a.species = P->species;
    a.value_g = P->value_g;
    a.value_b = P->value_b;
    a.n = P->n;
    a.soh = (double)p->sigma_over_h;
    a.f = (double)p->trunc_f;
    a.tile = c.L.tile;
    a.ntx = c.L.ntx;
    a.tile_mask = p->tile_mask;
    a.rec = c.at<Rec>(c.L.rec);
    a.cnt = c.at<uint32_t>(c.L.cnt);
    a.key = c.L.ordered ? c.at<uint32_t>(c.L.key0) : nullptr;
    a.counters = c.at<unsigned long long>(c.L.counters);
    a.o_status = o_status;
    a.o_bbox = o_bbox;
    a.o_spec = o_spec;
    a.o_key = o_key;
    TRY(launch_fill_u32(c.at<uint32_t>(c.L.counters), 0u, 2 * kCntN, c.s));
    uint32_t *range = c.at<uint32_t>(c.L.range);
    TRY(launch_range_init(range, c.s));
    a.range_bits = range;
    TRY(launch_project(a, c.s));
    TRY(const_cast<Prof &>(c.prof).mark(0));
    return SPLOTCH_OK;
}

// Stage 2: processing order (depth sort when ordered) and pair offsets
// (L.off, in processing order).  Returns the order (or null = particle
// order) and the mask of an order entry's index bits: up to 2^30 particles
// the entries carry their tile counts in the top bits, which the scan
// decodes, so no gather of counts into the sorted order is needed.
// trim_keys: read the visible depth-key range back (one stream sync) and
// sort only the digits it spans; particles outside it have no pairs, so
// where they land does not matter.  Off where the caller cannot sync
// (graph capture).
splotch_status run_order_and_scan(const Ctx &c, int64_t n, bool trim_keys,
                                  const uint32_t **order, uint32_t *idx_mask) {
    const uint32_t *cnt = c.at<uint32_t>(c.L.cnt);
    uint64_t *off = c.at<uint64_t>(c.L.off);
    *order = nullptr;
    *idx_mask = 0xFFFFFFFFu;
    if (c.L.ordered && n > 0) {
        bool in1 = false;
        uint32_t *k0 = c.at<uint32_t>(c.L.key0), *k1 = c.at<uint32_t>(c.L.key1);
        uint32_t *v0 = c.at<uint32_t>(c.L.val0), *v1 = c.at<uint32_t>(c.L.val1);
        int bits = 32;
        uint32_t bias = 0;
        if (trim_keys) {
            uint32_t kr[2];
            TRY(hipMemcpyAsync(kr, c.at<uint32_t>(c.L.range) + 2 * kMaxSpecies, sizeof kr,
                               hipMemcpyDeviceToHost, c.s));
            TRY(hipStreamSynchronize(c.s));
            if (kr[0] <= kr[1]) {
                bias = kr[0];
                const uint32_t span = kr[1] - kr[0];
                bits = span == 0 ? 1 : 32 - __builtin_clz(span);
            } else {
                bits = 1;  // nothing visible
            }
        }
        const bool tag = (uint64_t)n <= (1ull << kTagShift);
        // without the read-back, the passes find the key range on the device
        const uint32_t *key_range =
            trim_keys ? nullptr : c.at<uint32_t>(c.L.range) + 2 * kMaxSpecies;
        TRY(radix_sort_pairs(k0, v0, k1, v1, true, (size_t)n, nullptr, bits, bias, false,
                             c.at<void>(c.L.radix), &in1, c.s, tag ? cnt : nullptr, key_range));
        const uint32_t *ord = in1 ? v1 : v0;
        *order = ord;
        if (tag) {
            *idx_mask = kIdxMask;
            TRY(const_cast<Prof &>(c.prof).mark(1));
            TRY(launch_scan_tagged_counts(ord, cnt, off, (size_t)n, c.at<void>(c.L.scan), c.s));
            TRY(const_cast<Prof &>(c.prof).mark(2));
            return SPLOTCH_OK;
        }
        // key buffers are free after the sort: counts in processing order
        TRY(launch_gather_u32(cnt, ord, k0, (size_t)n, c.s));
        cnt = k0;
    }
    TRY(const_cast<Prof &>(c.prof).mark(1));
    TRY(launch_scan_u32_u64(cnt, off, (size_t)n, c.at<void>(c.L.scan), c.s));
    TRY(const_cast<Prof &>(c.prof).mark(2));
    return SPLOTCH_OK;
}

// Bin one chunk [first, last) of processing positions: emit, sort by tile,
// tile ranges.  Returns the sorted pair values via *vals.
splotch_status run_bin_chunk(const Ctx &c, const uint32_t *order, uint32_t idx_mask,
                             uint64_t first, uint64_t last, uint64_t off_first, uint64_t npairs,
                             const uint32_t **vals, const uint32_t **keys_out = nullptr) {
    uint32_t *pk0 = c.at<uint32_t>(c.L.pk0), *pk1 = c.at<uint32_t>(c.L.pk1);
    uint32_t *pv0 = c.at<uint32_t>(c.L.pv0), *pv1 = c.at<uint32_t>(c.L.pv1);
    EmitArgs e;
    e.rec = c.at<Rec>(c.L.rec);
    e.order = order;
    e.idx_mask = idx_mask;
    e.off = c.at<uint64_t>(c.L.off);
    e.first = first;
    e.last = last;
    e.base = off_first;
    e.cap = c.L.pair_cap;
    e.overflow = nullptr;
    e.tile_mask = c.tile_mask;
    e.tile = c.L.tile;
    e.qshift = block_mask_shift(c.L.tile, c.L.n_tiles);
    e.ntx = c.L.ntx;
    e.pair_key = pk0;
    e.pair_val = pv0;
    e.split_pixels = c.split;
    e.split_list = c.split ? c.at<uint32_t>(c.L.split) : nullptr;
    e.split_count = c.at<uint32_t>(c.L.split_cnt);
    e.split_off = c.at<uint64_t>(c.L.split_off);
    e.split_scratch = c.at<void>(c.L.scan);
    e.split_dense = c.at<uint32_t>(c.L.cnt);
    TRY(launch_emit(e, c.s));
    TRY(const_cast<Prof &>(c.prof).mark(3));
    int bits = 0;
    while ((1ull << bits) < (uint64_t)c.L.n_tiles) ++bits;
    bool in1 = false;
    TRY(radix_sort_pairs(pk0, pv0, pk1, pv1, false, (size_t)npairs, nullptr, bits, 0u, true,
                         c.at<void>(c.L.radix), &in1, c.s));
    const uint32_t *keys = in1 ? pk1 : pk0;
    *vals = in1 ? pv1 : pv0;
    const uint32_t key_mask = e.qshift ? (1u << e.qshift) - 1u : 0xFFFFFFFFu;
    TRY(launch_tile_ranges(keys, (size_t)npairs, nullptr, c.at<uint32_t>(c.L.tstart),
                           c.at<uint32_t>(c.L.tend), c.L.n_tiles, key_mask, c.s));
    if (keys_out) *keys_out = keys;
    TRY(const_cast<Prof &>(c.prof).mark(4));
    return SPLOTCH_OK;
}

// Read the pair total and plan chunks.  plan receives (position, offset)
// boundaries: chunk k covers [plan[2k], plan[2k+2]).
splotch_status plan_chunks(const Ctx &c, int64_t n, std::vector<uint64_t> *plan) {
    uint64_t total = 0;
    uint64_t *off = c.at<uint64_t>(c.L.off);
    TRY(hipMemcpyAsync(&total, off + n, 8, hipMemcpyDeviceToHost, c.s));
    TRY(hipStreamSynchronize(c.s));
    plan->clear();
    if (total <= c.L.pair_cap) {
        *plan = {0, 0, (uint64_t)n, total};
        return SPLOTCH_OK;
    }
    uint64_t *bounds = c.at<uint64_t>(c.L.bounds);
    TRY(launch_chunk_plan(off, (uint64_t)n, c.L.pair_cap, bounds, kMaxChunks, c.s));
    std::vector<uint64_t> hb(2 + 2 * (kMaxChunks + 1));
    TRY(hipMemcpyAsync(hb.data(), bounds, hb.size() * 8, hipMemcpyDeviceToHost, c.s));
    TRY(hipStreamSynchronize(c.s));
    if (hb[1] != 0) return SPLOTCH_E_CAPACITY;
    const uint64_t nch = hb[0];
    plan->assign(hb.begin() + 2, hb.begin() + 2 + 2 * (nch + 1));
    return SPLOTCH_OK;
}

splotch_status run_splat_pass(Ctx &c, SplatArgs &sa, uint64_t npairs) {
    const uint32_t nt = (uint32_t)(c.L.tile * c.L.tile);
    const uint32_t seg_len = seg_len_rule(npairs, nt, c.seg_min);
    TRY(launch_segments(sa.tile_start, sa.tile_end, c.L.n_tiles, npairs, nullptr, nt, c.seg_min,
                        c.at<uint32_t>(c.L.seg_len), c.at<uint32_t>(c.L.nseg),
                        c.at<uint32_t>(c.L.nmulti), c.at<uint64_t>(c.L.seg_off),
                        c.at<uint64_t>(c.L.part_off), c.at<uint32_t>(c.L.item_tile),
                        c.L.max_items, c.at<void>(c.L.seg_scan), c.s));
    TRY(launch_splat(sa, splat_grid(c.L.n_tiles, npairs, seg_len), c.s));
    TRY(c.prof.mark(5));
    return SPLOTCH_OK;
}

splotch_status read_stats(Ctx &c, const splotch_params *p, int64_t pairs, int chunks) {
    if (!p->stats) return SPLOTCH_OK;
    float stage_ms[6] = {0, 0, 0, 0, 0, 0};
    TRY(c.prof.finish(stage_ms, 6));
    int64_t members = 0, absorbing = 0;
    if (c.prof.on) {
        std::vector<unsigned long long> mc(2 * (size_t)c.L.n_tiles);
        TRY(hipMemcpyAsync(mc.data(), c.at<void>(c.L.mcount), mc.size() * 8,
                           hipMemcpyDeviceToHost, c.s));
        TRY(hipStreamSynchronize(c.s));
        for (size_t k = 0; k < mc.size(); k += 2) {
            members += (int64_t)mc[k];
            absorbing += (int64_t)mc[k + 1];
        }
    }
    unsigned long long cnt[kCntN];
    uint32_t range[2 * kMaxSpecies];
    TRY(hipMemcpyAsync(cnt, c.at<void>(c.L.counters), sizeof cnt, hipMemcpyDeviceToHost, c.s));
    TRY(hipMemcpyAsync(range, c.at<void>(c.L.range), sizeof range, hipMemcpyDeviceToHost, c.s));
    TRY(hipStreamSynchronize(c.s));
    splotch_stats *st = p->stats;
    memset(st, 0, sizeof *st);
    st->n_visible = (int64_t)cnt[kCntVisible];
    st->n_invalid = (int64_t)cnt[kCntInvalid];
    st->n_depth_culled = (int64_t)cnt[kCntDepth];
    st->n_offscreen = (int64_t)cnt[kCntOffscreen];
    st->n_pairs = pairs;
    st->n_chunks = chunks;
    st->tile = c.L.tile;
    st->ordered = c.L.ordered ? 1 : 0;
    for (int k = 0; k < 6; ++k) st->stage_ms[k] = stage_ms[k];
    st->n_member_pairs = members;
    st->n_member_absorbing = absorbing;
    for (int s = 0; s < p->n_species; ++s) {
        const splotch_species &q = p->species[s];
        if (q.vmin < q.vmax) {
            st->vmin[s] = q.vmin;
            st->vmax[s] = q.vmax;
        } else if (range[2 * s] == 0xFFFFFFFFu) {
            st->vmin[s] = st->vmax[s] = 0.0f;
        } else {
            for (int w = 0; w < 2; ++w) {
                uint32_t k = range[2 * s + w];
                uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
                float f;
                memcpy(&f, &b, 4);
                (w ? st->vmax : st->vmin)[s] = f;
            }
        }
    }
    return SPLOTCH_OK;
}

splotch_status prepare(const splotch_particles *P, const splotch_camera *cam,
                       const splotch_params *p, Ctx *c) {
    splotch_status st;
    if ((st = validate_particles(P)) != SPLOTCH_OK) return st;
    if ((st = validate_camera(cam)) != SPLOTCH_OK) return st;
    if ((st = validate_params(p)) != SPLOTCH_OK) return st;
    for (int s = 0; s < p->n_species; ++s)
        if (p->species[s].colour == SPLOTCH_COLOUR_VECTOR && P->n > 0 &&
            (!P->value_g || !P->value_b))
            return SPLOTCH_E_INVALID_ARG;
    if (!p->workspace || (reinterpret_cast<uintptr_t>(p->workspace) & 255u) != 0)
        return SPLOTCH_E_WORKSPACE;
    if (!fit_capacity(P->n, cam, p, p->workspace_bytes, &c->L)) return SPLOTCH_E_WORKSPACE;
    c->ws = reinterpret_cast<char *>(p->workspace);
    c->s = reinterpret_cast<hipStream_t>(p->stream);
    c->seg_min = p->seg_records > 0 ? (uint32_t)p->seg_records : kSegMin;
    c->tile_mask = p->tile_mask;
    c->split = split_threshold(p, cam);
    if (c->prof.start(p->profile != 0 && p->stats != nullptr, c->s) != hipSuccess)
        return SPLOTCH_E_DEVICE;
    return SPLOTCH_OK;
}


// ------------------------------------------------------------------ batch
__global__ void k_copy_u64(const uint64_t *src, uint64_t *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = *src;
}

struct GraphEntry {
    std::vector<uint64_t> key;
    hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::list<GraphEntry> g_graphs;  // most recently used first
constexpr size_t kMaxGraphs = 16;

void key_bytes(std::vector<uint64_t> *k, const void *p, size_t n) {
    const unsigned char *b = static_cast<const unsigned char *>(p);
    for (size_t i = 0; i < n; i += 8) {
        uint64_t w = 0;
        memcpy(&w, b + i, std::min<size_t>(8, n - i));
        k->push_back(w);
    }
}

// Library-owned streams and events for the batch lanes, one set per
// device, created on first use (default priority).
struct LaneSet {
    hipStream_t s[kMaxLanes - 1];
    hipEvent_t fork, join[kMaxLanes - 1];
};
std::mutex g_lane_mu;  // held while a batch is queued
std::map<int, LaneSet> g_lanes;

splotch_status lane_set(LaneSet **out) {
    int dev = 0;
    TRY(hipGetDevice(&dev));
    auto it = g_lanes.find(dev);
    if (it == g_lanes.end()) {
        LaneSet L;
        for (int k = 0; k < kMaxLanes - 1; ++k) {
            TRY(hipStreamCreateWithFlags(&L.s[k], hipStreamNonBlocking));
            TRY(hipEventCreateWithFlags(&L.join[k], hipEventDisableTiming));
        }
        TRY(hipEventCreateWithFlags(&L.fork, hipEventDisableTiming));
        it = g_lanes.emplace(dev, L).first;
    }
    *out = &it->second;
    return SPLOTCH_OK;
}

// Queue view v on lane c (its workspace part and stream).  flags/totals
// (per view) live in the first lane's workspace part.
// With defer (persistent batches) the splat is not launched: its settings
// are returned in *defer for the group launch.
splotch_status enqueue_view(Ctx &c, int32_t v, uint32_t *flags, uint64_t *totals,
                            const splotch_particles *P, const splotch_camera *cam,
                            const splotch_colourmap *cmap, const splotch_params *p,
                            splotch_image *image, SplatArgs *defer = nullptr) {
    const int64_t n = P->n;
    const uint64_t cap = c.L.pair_cap;
    const uint32_t nt = (uint32_t)(c.L.tile * c.L.tile);
    {
        Layout Lv = c.L;  // same buffers; per-view tile grid
        Lv.ntx = (cam->width + c.L.tile - 1) / c.L.tile;
        Lv.nty = (cam->height + c.L.tile - 1) / c.L.tile;
        Lv.n_tiles = (uint32_t)(Lv.ntx * Lv.nty);
        Ctx cv;  // fresh context (no stage events) over the same workspace
        cv.L = Lv;
        cv.ws = c.ws;
        cv.s = c.s;
        cv.seg_min = c.seg_min;
        cv.tile_mask = c.tile_mask;
        splotch_status st;
        // the value range does not depend on the camera: the projection of
        // every view recomputes it from the same particles
        if ((st = run_project(cv, P, cam, p, nullptr, nullptr, nullptr, nullptr)) != SPLOTCH_OK)
            return st;
        const uint32_t *order;
        uint32_t idx_mask;
        if ((st = run_order_and_scan(cv, n, false, &order, &idx_mask)) != SPLOTCH_OK) return st;
        const uint64_t *total = c.at<uint64_t>(c.L.off) + n;
        EmitArgs e;
        e.rec = c.at<Rec>(c.L.rec);
        e.order = order;
        e.idx_mask = idx_mask;
        e.off = c.at<uint64_t>(c.L.off);
        e.first = 0;
        e.last = (uint64_t)n;
        e.base = 0;
        e.cap = cap;
        e.overflow = flags + v;
        e.tile_mask = p->tile_mask;
        e.tile = c.L.tile;
        e.ntx = Lv.ntx;
        e.qshift = block_mask_shift(c.L.tile, Lv.n_tiles);
        e.split_pixels = split_threshold(p, cam);
        e.split_list = e.split_pixels ? c.at<uint32_t>(c.L.split) : nullptr;
        e.split_count = c.at<uint32_t>(c.L.split_cnt);
        e.split_off = c.at<uint64_t>(c.L.split_off);
        e.split_scratch = c.at<void>(c.L.scan);
        e.split_dense = c.at<uint32_t>(c.L.cnt);
        uint32_t *pk0 = c.at<uint32_t>(c.L.pk0), *pk1 = c.at<uint32_t>(c.L.pk1);
        uint32_t *pv0 = c.at<uint32_t>(c.L.pv0), *pv1 = c.at<uint32_t>(c.L.pv1);
        e.pair_key = pk0;
        e.pair_val = pv0;
        TRY(launch_emit(e, c.s));
        hipLaunchKernelGGL(k_copy_u64, dim3(1), dim3(64), 0, c.s, total, totals + v);
        TRY(hipGetLastError());
        int bits = 0;
        while ((1ull << bits) < (uint64_t)Lv.n_tiles) ++bits;
        bool in1 = false;
        TRY(radix_sort_pairs(pk0, pv0, pk1, pv1, false, (size_t)cap, total, bits, 0u, true,
                             c.at<void>(c.L.radix), &in1, c.s));
        const uint32_t *keys = in1 ? pk1 : pk0;
        const uint32_t *vals = in1 ? pv1 : pv0;
        uint32_t *ts = c.at<uint32_t>(c.L.tstart), *te = c.at<uint32_t>(c.L.tend);
        TRY(launch_tile_ranges(keys, (size_t)cap, total, ts, te, Lv.n_tiles,
                               e.qshift ? (1u << e.qshift) - 1u : 0xFFFFFFFFu, c.s));
        TRY(launch_segments(ts, te, Lv.n_tiles, cap, total, nt, c.seg_min,
                            c.at<uint32_t>(c.L.seg_len), c.at<uint32_t>(c.L.nseg),
                            c.at<uint32_t>(c.L.nmulti), c.at<uint64_t>(c.L.seg_off),
                            c.at<uint64_t>(c.L.part_off), c.at<uint32_t>(c.L.item_tile),
                            c.L.max_items, c.at<void>(c.L.seg_scan), c.s));
        SplatArgs sa;
        memset(&sa, 0, sizeof sa);
        sa.rec = c.at<Rec>(c.L.rec);
        sa.pair_val = vals;
        sa.pair_key = keys;
        sa.qshift = e.qshift;
        sa.tile_start = ts;
        sa.tile_end = te;
        sa.seg_off = c.at<uint64_t>(c.L.seg_off);
        sa.part_off = c.at<uint64_t>(c.L.part_off);
        sa.item_tile = c.at<uint32_t>(c.L.item_tile);
        sa.partial = c.at<float>(c.L.partial);
        sa.max_slots = c.L.max_slots;
        sa.max_items = c.L.max_items;
        sa.seg_len = c.at<uint32_t>(c.L.seg_len);
        splat_colour_args(&sa, P, cmap, p);
        sa.image = image->rgb;
        sa.member_count = c.at<unsigned long long>(c.L.mcount);
        sa.tile_mask = p->tile_mask;
        sa.range_bits = c.at<uint32_t>(c.L.range);
        sa.width = cam->width;
        sa.height = cam->height;
        sa.tile = c.L.tile;
        sa.ntx = Lv.ntx;
        sa.nty = Lv.nty;
        sa.accumulate = p->accumulate;
        sa.compensated = p->compensated ? 1 : 0;
        sa.ordered = c.L.ordered ? 1 : 0;
        sa.variant = splat_variant_of(p->splat_variant);
        // a view that overflowed writes nothing (it is rendered again in
        // chunks, or reported)
        sa.skip = flags + v;
        if (defer) {
            *defer = sa;
            return SPLOTCH_OK;
        }
        if (sa.variant == kSplatRows) {
            // the item count is on the device: a persistent launch over
            // the view's units instead of a grid sized to the most items
            SplatArgs *dev = c.at<SplatArgs>(c.L.sargs);
            TRY(store_splat_args(sa, dev, c.s));
            TRY(launch_splat_multi(dev, 1, sa, c.at<uint32_t>(c.L.unit_next), c.s));
            TRY(launch_merge(sa, c.s));
        } else {
            const uint32_t q = 64;
            const uint32_t grid = (uint32_t)((Lv.n_tiles + kSegTarget + q - 1) / q * q);
            TRY(launch_splat(sa, grid, c.s));
        }
    }
    return SPLOTCH_OK;
}

// Queue the whole batch without any host read-back: views round-robin over
// the lanes (lane 0 runs on the caller's stream), forked from and joined
// back to the caller's stream with events.
splotch_status enqueue_batch(std::vector<Ctx> &lanes, const LaneSet *ls,
                             const splotch_particles *P, int32_t nv, const splotch_camera *cams,
                             const splotch_colourmap *cmap, const splotch_params *p,
                             splotch_image *images) {
    Ctx &c0 = lanes[0];
    const int K = (int)lanes.size();
    uint32_t *flags = c0.at<uint32_t>(c0.L.flags);
    uint64_t *totals = reinterpret_cast<uint64_t *>(flags + SPLOTCH_MAX_VIEWS);
    TRY(launch_fill_u32(flags, 0u, (size_t)nv, c0.s));
    if (p->batch_persistent) {
        // groups of K views: each lane prepares one view (projection to
        // segments), then one persistent splat over the group on the
        // caller's stream, then the views' merges; the next group's lanes
        // start after them (they reuse the workspace parts)
        SplatArgs *views = c0.at<SplatArgs>(c0.L.sargs);
        for (int32_t g0 = 0; g0 < nv; g0 += K) {
            const int G = std::min<int>(K, nv - g0);
            if (G > 1) {
                TRY(hipEventRecord(ls->fork, c0.s));
                for (int k = 1; k < G; ++k) TRY(hipStreamWaitEvent(lanes[k].s, ls->fork, 0));
            }
            SplatArgs sa[kMaxGroup];
            for (int k = 0; k < G; ++k) {
                splotch_status st = enqueue_view(lanes[k], g0 + k, flags, totals, P, &cams[g0 + k],
                                                 cmap, p, &images[g0 + k], &sa[k]);
                if (st != SPLOTCH_OK) return st;
                TRY(store_splat_args(sa[k], views + k, lanes[k].s));
            }
            if (G > 1) {
                for (int k = 1; k < G; ++k) {
                    TRY(hipEventRecord(ls->join[k - 1], lanes[k].s));
                    TRY(hipStreamWaitEvent(c0.s, ls->join[k - 1], 0));
                }
            }
            TRY(launch_splat_multi(views, G, sa[0], c0.at<uint32_t>(c0.L.unit_next), c0.s));
            for (int k = 0; k < G; ++k) TRY(launch_merge(sa[k], c0.s));
        }
        return SPLOTCH_OK;
    }
    if (K > 1) {
        TRY(hipEventRecord(ls->fork, c0.s));
        for (int k = 1; k < K; ++k) TRY(hipStreamWaitEvent(lanes[k].s, ls->fork, 0));
    }
    for (int32_t v = 0; v < nv; ++v) {
        splotch_status st = enqueue_view(lanes[v % K], v, flags, totals, P, &cams[v], cmap, p,
                                         &images[v]);
        if (st != SPLOTCH_OK) return st;
    }
    if (K > 1) {
        for (int k = 1; k < K; ++k) {
            TRY(hipEventRecord(ls->join[k - 1], lanes[k].s));
            TRY(hipStreamWaitEvent(c0.s, ls->join[k - 1], 0));
        }
    }
    return SPLOTCH_OK;
}

}  // namespace

extern "C" {

const char *splotch_status_string(int32_t code) {
    switch (code) {
        case SPLOTCH_OK: return "ok";
        case SPLOTCH_E_INVALID_ARG: return "invalid argument";
        case SPLOTCH_E_WORKSPACE: return "workspace missing, misaligned or too small";
        case SPLOTCH_E_DEVICE: return "HIP runtime error";
        case SPLOTCH_E_UNSUPPORTED: return "unsupported setting";
        case SPLOTCH_E_CAPACITY: return "a particle needs more pair slots than the workspace holds";
        case SPLOTCH_E_SCRATCH: return "input needs more than the static scratch buffer holds";
    }
    return "unknown status";
}

splotch_status splotch_camera_look_at(splotch_camera *cam, const float eye[3], const float at[3],
                                      const float up[3], int32_t projection, float fov_or_scale,
                                      int32_t width, int32_t height, float z_near, float z_far) {
    if (!cam || !eye || !at || !up) return SPLOTCH_E_INVALID_ARG;
    double f[3], r[3], u[3];
    for (int k = 0; k < 3; ++k) f[k] = (double)at[k] - (double)eye[k];
    double nf = sqrt(f[0] * f[0] + f[1] * f[1] + f[2] * f[2]);
    if (!(nf > 0.0) || !isfinite(nf)) return SPLOTCH_E_INVALID_ARG;
    for (int k = 0; k < 3; ++k) f[k] /= nf;
    // right = up x fwd, up' = fwd x right  (right x up' = fwd)
    r[0] = (double)up[1] * f[2] - (double)up[2] * f[1];
    r[1] = (double)up[2] * f[0] - (double)up[0] * f[2];
    r[2] = (double)up[0] * f[1] - (double)up[1] * f[0];
    double nr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(nr > 1e-12) || !isfinite(nr)) return SPLOTCH_E_INVALID_ARG;
    for (int k = 0; k < 3; ++k) r[k] /= nr;
    u[0] = f[1] * r[2] - f[2] * r[1];
    u[1] = f[2] * r[0] - f[0] * r[2];
    u[2] = f[0] * r[1] - f[1] * r[0];
    splotch_camera c;
    memset(&c, 0, sizeof c);
    c.projection = projection;
    c.width = width;
    c.height = height;
    for (int k = 0; k < 3; ++k) {
        c.eye[k] = eye[k];
        c.right[k] = (float)r[k];
        c.up[k] = (float)u[k];
        c.fwd[k] = (float)f[k];
    }
    if (projection == SPLOTCH_PERSPECTIVE) {
        if (!(fov_or_scale > 0.0f && fov_or_scale < 180.0f)) return SPLOTCH_E_INVALID_ARG;
        c.focal_px = (float)((0.5 * width) / tan(0.5 * (double)fov_or_scale * M_PI / 180.0));
    } else if (projection == SPLOTCH_ORTHO) {
        c.px_per_unit = fov_or_scale;
    } else {
        return SPLOTCH_E_INVALID_ARG;
    }
    c.z_near = z_near;
    c.z_far = z_far;
    splotch_status st = validate_camera(&c);
    if (st != SPLOTCH_OK) return st;
    *cam = c;
    return SPLOTCH_OK;
}

splotch_status splotch_workspace_size(int64_t n, const splotch_camera *cam,
                                      const splotch_params *params, int64_t max_pairs,
                                      size_t *bytes) {
    if (!bytes || n < 0 || (uint64_t)n >= (1ull << 32)) return SPLOTCH_E_INVALID_ARG;
    splotch_status st;
    if ((st = validate_camera(cam)) != SPLOTCH_OK) return st;
    if ((st = validate_params(params)) != SPLOTCH_OK) return st;
    uint64_t cap = max_pairs > 0 ? (uint64_t)max_pairs : 4ull * (uint64_t)n + 65536ull;
    if (cap > kMaxPairCap) cap = kMaxPairCap;
    *bytes = layout(n, cam, params, cap).total;
    return SPLOTCH_OK;
}

splotch_status splotch_render(const splotch_particles *P, const splotch_camera *cam,
                              const splotch_colourmap *cmap, const splotch_params *p,
                              splotch_image *img) {
    TraceRange trace("splotch_render");
    Ctx c;
    splotch_status st = prepare(P, cam, p, &c);
    if (st != SPLOTCH_OK) return st;
    if ((st = validate_colourmap(cmap)) != SPLOTCH_OK) return st;
    if (!img || !img->rgb || img->width != cam->width || img->height != cam->height)
        return SPLOTCH_E_INVALID_ARG;
    const int64_t n = P->n;
    if ((st = run_project(c, P, cam, p, nullptr, nullptr, nullptr, nullptr)) != SPLOTCH_OK)
        return st;
    const uint32_t *order;
    uint32_t idx_mask;
    if ((st = run_order_and_scan(c, n, true, &order, &idx_mask)) != SPLOTCH_OK) return st;
    std::vector<uint64_t> plan;
    if ((st = plan_chunks(c, n, &plan)) != SPLOTCH_OK) return st;
    const int nch = (int)(plan.size() / 2) - 1;

    SplatArgs sa;
    memset(&sa, 0, sizeof sa);
    sa.rec = c.at<Rec>(c.L.rec);
    sa.tile_start = c.at<uint32_t>(c.L.tstart);
    sa.tile_end = c.at<uint32_t>(c.L.tend);
    splat_colour_args(&sa, P, cmap, p);
    sa.image = img->rgb;
    sa.width = cam->width;
    sa.height = cam->height;
    sa.tile = c.L.tile;
    sa.ntx = c.L.ntx;
    sa.nty = c.L.nty;
    sa.compensated = p->compensated ? 1 : 0;
    sa.ordered = c.L.ordered ? 1 : 0;
    sa.variant = splat_variant_of(p->splat_variant);
    sa.member_count = c.at<unsigned long long>(c.L.mcount);
    sa.tile_mask = p->tile_mask;
    sa.range_bits = c.at<uint32_t>(c.L.range);
    sa.seg_off = c.at<uint64_t>(c.L.seg_off);
    sa.part_off = c.at<uint64_t>(c.L.part_off);
    sa.item_tile = c.at<uint32_t>(c.L.item_tile);
    sa.partial = c.at<float>(c.L.partial);
    sa.max_slots = c.L.max_slots;
    sa.max_items = c.L.max_items;
    sa.seg_len = c.at<uint32_t>(c.L.seg_len);
    sa.qshift = block_mask_shift(c.L.tile, c.L.n_tiles);
    // member statistics only where they are asked for (profile level 2)
    sa.count = (p->stats != nullptr && p->profile >= 2) ? 1 : 0;
    TRY(launch_fill_u32(c.at<uint32_t>(c.L.mcount), 0u, (size_t)c.L.n_tiles * 4, c.s));

    const uint64_t total = plan.back();
    if (total == 0) {
        // nothing on screen: the splat still writes every pixel
        TRY(launch_fill_u32(c.at<uint32_t>(c.L.tstart), 0u, c.L.n_tiles, c.s));
        TRY(launch_fill_u32(c.at<uint32_t>(c.L.tend), 0u, c.L.n_tiles, c.s));
        sa.pair_val = c.at<uint32_t>(c.L.pv0);
        sa.pair_key = c.at<uint32_t>(c.L.pk0);
        sa.accumulate = p->accumulate;
        if ((st = run_splat_pass(c, sa, 0)) != SPLOTCH_OK) return st;
        return read_stats(c, p, 0, 0);
    }
    // depth-ordered chunks are depth slabs: composite back to front
    for (int q = 0; q < nch; ++q) {
        const int k = c.L.ordered ? nch - 1 - q : q;
        const uint64_t first = plan[2 * k], last = plan[2 * k + 2];
        const uint64_t o0 = plan[2 * k + 1], o1 = plan[2 * k + 3];
        const uint32_t *vals, *keys;
        if ((st = run_bin_chunk(c, order, idx_mask, first, last, o0, o1 - o0, &vals, &keys)) !=
            SPLOTCH_OK)
            return st;
        sa.pair_val = vals;
        sa.pair_key = keys;
        sa.accumulate = q == 0 ? p->accumulate : 1;
        if ((st = run_splat_pass(c, sa, o1 - o0)) != SPLOTCH_OK) return st;
    }
    return read_stats(c, p, (int64_t)total, nch);
}

splotch_status splotch_project(const splotch_particles *P, const splotch_camera *cam,
                               const splotch_params *p, int8_t *status, int32_t *bbox,
                               float *spec, uint32_t *key, uint32_t *ntiles) {
    Ctx c;
    splotch_status st = prepare(P, cam, p, &c);
    if (st != SPLOTCH_OK) return st;
    if ((st = run_project(c, P, cam, p, status, bbox, spec, key)) != SPLOTCH_OK) return st;
    if (ntiles && P->n > 0)
        TRY(hipMemcpyAsync(ntiles, c.at<void>(c.L.cnt), (size_t)P->n * 4,
                           hipMemcpyDeviceToDevice, c.s));
    return read_stats(c, p, 0, 0);
}

splotch_status splotch_bin(const splotch_particles *P, const splotch_camera *cam,
                           const splotch_params *p, uint32_t *tile_start, uint32_t *tile_end,
                           uint32_t *pair_particle, int64_t max_out, int64_t *n_pairs) {
    Ctx c;
    splotch_status st = prepare(P, cam, p, &c);
    if (st != SPLOTCH_OK) return st;
    if (!tile_start || !tile_end || !pair_particle || !n_pairs || max_out < 0)
        return SPLOTCH_E_INVALID_ARG;
    const int64_t n = P->n;
    if ((st = run_project(c, P, cam, p, nullptr, nullptr, nullptr, nullptr)) != SPLOTCH_OK)
        return st;
    const uint32_t *order;
    uint32_t idx_mask;
    if ((st = run_order_and_scan(c, n, true, &order, &idx_mask)) != SPLOTCH_OK) return st;
    uint64_t total = 0;
    TRY(hipMemcpyAsync(&total, c.at<uint64_t>(c.L.off) + n, 8, hipMemcpyDeviceToHost, c.s));
    TRY(hipStreamSynchronize(c.s));
    *n_pairs = (int64_t)total;
    if (total > c.L.pair_cap || total > (uint64_t)max_out) return SPLOTCH_E_CAPACITY;
    const uint32_t *vals = c.at<uint32_t>(c.L.pv0);
    if (total > 0) {
        if ((st = run_bin_chunk(c, order, idx_mask, 0, (uint64_t)n, 0, total, &vals)) !=
            SPLOTCH_OK)
            return st;
    } else {
        TRY(launch_fill_u32(c.at<uint32_t>(c.L.tstart), 0u, c.L.n_tiles, c.s));
        TRY(launch_fill_u32(c.at<uint32_t>(c.L.tend), 0u, c.L.n_tiles, c.s));
    }
    TRY(hipMemcpyAsync(tile_start, c.at<void>(c.L.tstart), (size_t)c.L.n_tiles * 4,
                       hipMemcpyDeviceToDevice, c.s));
    TRY(hipMemcpyAsync(tile_end, c.at<void>(c.L.tend), (size_t)c.L.n_tiles * 4,
                       hipMemcpyDeviceToDevice, c.s));
    if (total > 0)
        TRY(hipMemcpyAsync(pair_particle, vals, (size_t)total * 4, hipMemcpyDeviceToDevice, c.s));
    return read_stats(c, p, (int64_t)total, 1);
}

splotch_status splotch_render_batch(const splotch_particles *P, int32_t n_views,
                                    const splotch_camera *cams, const splotch_colourmap *cmap,
                                    const splotch_params *p, splotch_image *images,
                                    int32_t use_graph) {
    TraceRange trace("splotch_render_batch");
    if (n_views < 1 || n_views > SPLOTCH_MAX_VIEWS || !cams || !images || !p)
        return SPLOTCH_E_INVALID_ARG;
    if (use_graph != 0 && use_graph != 1) return SPLOTCH_E_INVALID_ARG;
    if (p->tile_mask) return SPLOTCH_E_UNSUPPORTED;  // one mask cannot fit views of several sizes
    splotch_status st;
    int32_t big = 0;
    uint64_t big_tiles = 0;
    const int T = p->tile == 0 ? 16 : p->tile;
    for (int32_t v = 0; v < n_views; ++v) {
        if ((st = validate_camera(&cams[v])) != SPLOTCH_OK) return st;
        if (!images[v].rgb || images[v].width != cams[v].width ||
            images[v].height != cams[v].height)
            return SPLOTCH_E_INVALID_ARG;
        const uint64_t nt = (uint64_t)((cams[v].width + T - 1) / T) * ((cams[v].height + T - 1) / T);
        if (nt > big_tiles) {
            big_tiles = nt;
            big = v;
        }
    }
    if ((st = validate_colourmap(cmap)) != SPLOTCH_OK) return st;
    if (p->batch_streams < 0 || p->batch_streams > kMaxLanes) return SPLOTCH_E_INVALID_ARG;
    const int K = std::max(1, std::min<int>(p->batch_streams, n_views));
    Ctx c;
    splotch_params q = *p;  // stats are read after the batch, not per stage
    q.stats = nullptr;
    q.workspace_bytes = p->workspace_bytes / (size_t)K / 256 * 256;  // one lane's part
    if ((st = prepare(P, &cams[big], &q, &c)) != SPLOTCH_OK) return st;
    if (use_graph && c.s == nullptr) return SPLOTCH_E_INVALID_ARG;
    std::lock_guard<std::mutex> lane_lock(g_lane_mu);
    LaneSet *ls = nullptr;
    std::vector<Ctx> lanes(K);
    if (K > 1 && (st = lane_set(&ls)) != SPLOTCH_OK) return st;
    for (int k = 0; k < K; ++k) {
        lanes[k].L = c.L;
        lanes[k].ws = c.ws + (size_t)k * q.workspace_bytes;
        lanes[k].s = k == 0 ? c.s : ls->s[k - 1];
        lanes[k].seg_min = c.seg_min;
        lanes[k].tile_mask = c.tile_mask;
        lanes[k].split = c.split;
    }
    if (!use_graph) {
        if ((st = enqueue_batch(lanes, ls, P, n_views, cams, cmap, p, images)) != SPLOTCH_OK)
            return st;
    } else {
        std::vector<uint64_t> key;
        key_bytes(&key, P, sizeof *P);
        key_bytes(&key, cams, sizeof(splotch_camera) * (size_t)n_views);
        key_bytes(&key, cmap, sizeof *cmap);
        splotch_params kp = *p;
        kp.stats = nullptr;
        kp.stream = nullptr;
        kp.profile = 0;
        key_bytes(&key, &kp, sizeof kp);
        key_bytes(&key, images, sizeof(splotch_image) * (size_t)n_views);
        std::lock_guard<std::mutex> lock(g_graph_mu);
        auto it = std::find_if(g_graphs.begin(), g_graphs.end(),
                               [&](const GraphEntry &g) { return g.key == key; });
        if (it == g_graphs.end()) {
            hipGraph_t graph;
            TRY(hipStreamBeginCapture(c.s, hipStreamCaptureModeThreadLocal));
            st = enqueue_batch(lanes, ls, P, n_views, cams, cmap, p, images);
            hipError_t ec = hipStreamEndCapture(c.s, &graph);
            if (st != SPLOTCH_OK) {
                if (ec == hipSuccess) (void)hipGraphDestroy(graph);
                return st;
            }
            TRY(ec);
            hipGraphExec_t exec;
            hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            TRY(ei);
            g_graphs.push_front(GraphEntry{key, exec});
            if (g_graphs.size() > kMaxGraphs) {
                (void)hipGraphExecDestroy(g_graphs.back().exec);
                g_graphs.pop_back();
            }
            it = g_graphs.begin();
        } else if (it != g_graphs.begin()) {
            g_graphs.splice(g_graphs.begin(), g_graphs, it);
            it = g_graphs.begin();
        }
        TRY(hipGraphLaunch(it->exec, c.s));
    }
    // Eager batches wait for the overflow flags: a view whose pairs exceeded
    // the capacity wrote nothing and is rendered again here in
    // workspace-bounded chunks, as splotch_render does.  A graph replay
    // cannot branch on them: without stats it returns at once, with stats
    // it reports the overflowed views.
    if (use_graph && !p->stats) return SPLOTCH_OK;
    std::vector<uint32_t> fl(n_views);
    std::vector<uint64_t> tot(n_views);
    uint32_t *flags = c.at<uint32_t>(c.L.flags);
    TRY(hipMemcpyAsync(fl.data(), flags, 4 * (size_t)n_views, hipMemcpyDeviceToHost, c.s));
    TRY(hipMemcpyAsync(tot.data(), flags + SPLOTCH_MAX_VIEWS, 8 * (size_t)n_views,
                       hipMemcpyDeviceToHost, c.s));
    TRY(hipStreamSynchronize(c.s));
    bool over = false;
    for (int32_t v = 0; v < n_views; ++v) {
        splotch_stats one;
        memset(&one, 0, sizeof one);
        one.n_pairs = (int64_t)tot[v];
        one.n_chunks = fl[v] ? 0 : 1;
        one.tile = c.L.tile;
        one.ordered = c.L.ordered ? 1 : 0;
        if (fl[v] && !use_graph) {
            // lane 0's part of the workspace: the pair capacity of one view
            splotch_params r = q;
            r.stats = p->stats ? &one : nullptr;
            r.batch_streams = 0;
            r.batch_persistent = 0;
            r.profile = 0;
            if ((st = splotch_render(P, &cams[v], cmap, &r, &images[v])) != SPLOTCH_OK) return st;
        }
        over = over || one.n_chunks == 0;
        if (p->stats) p->stats[v] = one;
    }
    return over ? SPLOTCH_E_CAPACITY : SPLOTCH_OK;
}

int32_t splotch_graph_cache_clear(void) {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    int32_t k = 0;
    for (GraphEntry &g : g_graphs) {
        (void)hipGraphExecDestroy(g.exec);
        ++k;
    }
    g_graphs.clear();
    return k;
}

}  // extern "C"
