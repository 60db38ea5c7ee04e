// Internal declarations shared by the HIP translation units of libsplotch.
#pragma once

#include <hip/hip_runtime.h>
#include <rocprofiler-sdk-roctx/roctx.h>
#include <stdint.h>

namespace splotch {

constexpr int kMaxSpecies = 8;
constexpr int kBboxBits = 14;  // i0, i1 packed in 14 bits each (W, H <= 16384)
constexpr uint32_t kBboxMask = (1u << kBboxBits) - 1u;
// Bits 28..31 of a record's second word (above j0, j1): whether the box's
// corner 8x8 block (lowest or highest block column, lowest or highest block
// row: bit 28 + (x high) + 2 (y high)) holds no pixel within the radius.
constexpr int kCornerShift = 28;
constexpr uint32_t kEmptyKey = 0xFFFFFFFFu;

// Status codes written per particle by the projection kernel.
enum : int8_t { kVisible = 0, kInvalid = 1, kDepthCulled = 2, kOffscreen = 3 };

// Camera promoted to binary64 on the host (exact: every FP32 value is a
// binary64 value).
struct CamDev {
    double eye[3], right[3], up[3], fwd[3];
    double focal, ppu, znear, zfar;
    double half_w, half_h, wmax, hmax;  // W/2, H/2, W-1, H-1
    int persp, width, height;
};

// Per-species settings as the kernels see them.
struct SpeciesDev {
    float vmin[kMaxSpecies], vmax[kMaxSpecies];
    float brightness[kMaxSpecies], absorption[kMaxSpecies];
    int log_scale[kMaxSpecies], ordered[kMaxSpecies], auto_range[kMaxSpecies];
    int vector[kMaxSpecies];  // 1: the three vector components are r, g, b
    int n;
    int any_vector;
};

// Projected particle record: 32 bytes, two uint4.
//   a.x = i0 | i1 << 14 | species << 28     a.y = j0 | j1 << 14
//   a.z = float(u - i0)                     a.w = float(v - j0)
//   b.x = float((f sigma_s)^2)              b.y = float(log2(e) / sigma_s^2)
//   b.z = value (raw scalar)                b.w = rho0
struct Rec {
    uint4 a, b;
};

// Counters accumulated by the projection kernel (device, 64-bit).
enum { kCntVisible = 0, kCntInvalid, kCntDepth, kCntOffscreen, kCntN };

struct ProjectArgs {
    CamDev cam;
    SpeciesDev sp;
    const float *x, *y, *z, *h, *value, *rho0;
    const uint8_t *species;
    const float *value_g, *value_b;  // vector components 2 and 3 (vector species)
    int64_t n;
    double soh, f;
    int tile, ntx;
    const uint8_t *tile_mask;    // per tile, 0 = skip; null = all tiles
    uint32_t *range_bits;        // [2*kMaxSpecies] ordered bits of auto min/max (atomics),
                                 // then [2]: min/max depth key of visible particles
    Rec *rec;
    uint32_t *cnt;   // tile count per particle
    uint32_t *key;   // depth key per particle (kEmptyKey when not visible), may be null
    unsigned long long *counters;  // [kCntN]
    // optional stage outputs
    int8_t *o_status;
    int32_t *o_bbox;
    float *o_spec;
    uint32_t *o_key;
};

}  // namespace splotch

struct splotch_camera;
struct splotch_params;

namespace splotch {

// Device views of the camera (promoted to binary64) and of the per-species
// settings (api.hip).
CamDev cam_dev(const splotch_camera *c);
SpeciesDev species_dev(const splotch_params *p);

// Workgroups are dealt to the 8 XCDs round-robin.  This maps workgroup b
// of nblocks to the chunk it processes so that each XCD gets a contiguous
// range of chunks: outputs of neighbouring chunks that share cache lines
// then meet in one XCD's L2 instead of leaving partial lines in two.  A
// bijection on [0, nblocks).
__device__ __forceinline__ uint32_t xcd_contiguous(uint32_t b, uint32_t nblocks) {
    const uint32_t q = nblocks / 8, r = nblocks % 8, x = b % 8;
    return x * q + (x < r ? x : r) + b / 8;
}

// ---- launchers (one per kernel family) ------------------------------------
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_fill_f32(float *p, float v, size_t n, hipStream_t s);
// Reset the auto-range and depth-key-range slots (min = all ones, max = 0)
// before the projection.
constexpr int kRangeSlots = 2 * kMaxSpecies + 2;
hipError_t launch_range_init(uint32_t *range_bits, hipStream_t s);
hipError_t launch_project(const ProjectArgs &a, hipStream_t s);

// Exclusive scan of n uint32 counts into n+1 uint64 offsets (out[n] = total).
size_t scan_u32_u64_scratch_bytes(size_t n);
hipError_t launch_scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, void *scratch,
                               hipStream_t s);
// In-place exclusive scan of n uint32 values.
size_t scan_u32_scratch_bytes(size_t n);
hipError_t launch_scan_u32(uint32_t *data, size_t n, void *scratch, hipStream_t s);

// Stable LSD radix sort of (key, value) pairs on bits [0, bits) of
// key - bias (unsigned; keys below bias or at or above bias + 2^bits are
// placed in an unspecified order, which callers use only for entries that
// do not matter).  vals_in may be null (values = 0..n-1).  With n_dev non-null the live
// count is min(*n_dev, n) read on the device and n only sizes the grid
// (graph-capturable).  Buffers k0/v0 hold the input;
// k1/v1 are the second half of the ping-pong.  *result_in_1 tells which
// half holds the output.  keys_needed = false lets the last pass skip
// writing keys.
size_t radix_scratch_bytes(size_t n);
// tag_counts (with vals_identity, n <= 2^30): the identity values carry the
// element's count from tag_counts in bits 30-31 (1, 2, 4; 0 = other), so a
// sorted order also gives the counts in that order without a gather.
// key_range (device [smallest, largest] key, with n on the host, values
// only): instead of bits and bias, the passes take the bias and the number
// of 8-bit digits from the range on the device, and the values land in v0.
hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                            bool vals_identity, size_t n, const uint64_t *n_dev, int bits,
                            uint32_t bias, bool keys_needed, void *scratch, bool *result_in_1,
                            hipStream_t s, const uint32_t *tag_counts = nullptr,
                            const uint32_t *key_range = nullptr);
constexpr int kTagShift = 30;
constexpr uint32_t kIdxMask = (1u << kTagShift) - 1u;
// Exclusive scan of the counts a tagged order carries (cnt: counts by
// particle, read where the tag says "other") into n+1 offsets.
hipError_t launch_scan_tagged_counts(const uint32_t *order, const uint32_t *cnt, uint64_t *out,
                                     size_t n, void *scratch, hipStream_t s);

// Binning.
hipError_t launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst,
                             size_t n, hipStream_t s);
struct EmitArgs {
    const Rec *rec;
    const uint32_t *order;   // processing order -> particle index (null = identity)
    uint32_t idx_mask;       // bits of an order entry that hold the index
    const uint64_t *off;     // pair offsets in processing order
    uint64_t first, last;    // processing positions [first, last)
    uint64_t base;           // off[first]
    uint64_t cap;            // pair slots; a particle past it sets *overflow
    uint32_t *overflow;      // may be null when cap is known to suffice
    int tile, ntx;
    const uint8_t *tile_mask;  // per tile, 0 = skip; null = all tiles
    int qshift;                // > 0: key bit qshift + b set when the box meets 8x8 block b
    uint32_t *pair_key, *pair_val;
    // split particles: boxes of more than split_pixels pixels are queued
    // and their pairs written a wave per particle.  Emission workgroup b
    // (256 positions) queues its split particles at split_list[256 b ...]
    // and their number at split_count[b] (capacities of 256 and 1 entries
    // per workgroup of the launch; null split_list = no splitting); the
    // counts' exclusive scan (split_off, one entry more, with
    // split_scratch for launch_scan_u32_u64) places them in one dense
    // queue (split_dense, last - first entries).
    uint64_t split_pixels;
    uint32_t *split_list;    // processing positions (n < 2^32)
    uint32_t *split_count;
    uint64_t *split_off;
    void *split_scratch;
    uint32_t *split_dense;
};
constexpr uint32_t kEmitGroup = 256;  // positions per emission workgroup
hipError_t launch_emit(const EmitArgs &a, hipStream_t s);
// Bit of a pair key where the mask of the tile's 8x8 blocks that the
// particle's box meets begins (bit qshift + b for block b, row-major), or 0
// when tiles have one block or the tile sort's 8-bit digits reach those bits.
inline int block_mask_shift(int tile, uint32_t n_tiles) {
    const int nb = (tile / 8) * (tile / 8);
    if (nb <= 1 || nb > 24) return 0;
    int bits = 0;
    while ((1ull << bits) < (uint64_t)n_tiles) ++bits;
    const int sorted = (bits + 7) / 8 * 8;
    const int qs = 32 - nb;
    return sorted <= qs ? qs : 0;
}
// n_pairs_dev (nullable): live pair count on the device, capped at n_pairs.
// key_mask: the bits of a pair key that hold the tile index.
hipError_t launch_tile_ranges(const uint32_t *sorted_keys, size_t n_pairs,
                              const uint64_t *n_pairs_dev, uint32_t *start, uint32_t *end,
                              uint32_t n_tiles, uint32_t key_mask, hipStream_t s);
hipError_t launch_chunk_plan(const uint64_t *off, uint64_t n, uint64_t capacity,
                             uint64_t *bounds, uint32_t max_chunks, hipStream_t s);

// Splat.  Work items are (tile, segment): each tile's list is cut into
// segments of at most seg_len records; a tile with one segment writes its
// pixels directly, a tile with several writes one partial (C, Tr) per
// segment that the merge kernel folds front to back.
struct SplatArgs {
    const Rec *rec;
    const uint32_t *pair_val;
    const uint32_t *pair_key;   // sorted keys (block masks from bit qshift)
    int qshift;                 // see EmitArgs; 0 = no block masks
    const uint32_t *tile_start, *tile_end;
    const uint64_t *seg_off;    // [n_tiles + 1] first item of each tile
    const uint64_t *part_off;   // [n_tiles + 1] first partial slot of each multi-segment tile
    const uint32_t *item_tile;  // item -> tile
    float *partial;             // [slot][6][T*T]: C0 C1 C2 Tr0 Tr1 Tr2
    uint64_t max_slots;         // partial slots in the buffer
    uint64_t max_items;         // entries of item_tile
    const uint32_t *seg_len;    // device: records per segment for this pass
    const float *palette;
    int n_pal;
    const float *pal_abs;        // absorption table, null = the emission table
    int n_pal_abs;
    const float *value_g, *value_b;  // vector components 2 and 3 (vector species)
    int kernel3d;                // 1: column of the density cut to the f sigma ball
    int general;                 // 1: some ordered species may have E != A
    int source;                  // 1: emission of ordered species is a source function
    SpeciesDev sp;
    float *image;
    unsigned long long *member_count;  // [2 per tile]: all, absorbing; summed over chunks
    const uint8_t *tile_mask;          // per tile, 0 = leave untouched; null = all tiles
    const uint32_t *range_bits;        // auto value ranges found by the projection
    int width, height, tile, ntx, nty;
    int accumulate, compensated, ordered;
    int variant;  // kSplatBox, kSplatRows or kSplatLists (see splat.hip)
    int count;    // 1: accumulate the member statistics (the row walk skips them otherwise)
    const uint32_t *skip;  // device flag or null: nonzero = write nothing (a batched view
                           // whose pairs overflowed the capacity)
};
// How a workgroup walks a tile's list.
constexpr int kSplatBox = 0, kSplatRows = 1, kSplatLists = 2;
// Segment length rule (shared by host and device): a multiple of the
// staging batch nt, at least seg_min, and at least pairs / kSegTarget so
// that a pass has at most n_tiles + kSegTarget items.
constexpr uint64_t kSegTarget = 65536;
__host__ __device__ inline uint32_t seg_len_rule(uint64_t npairs, uint32_t nt, uint32_t seg_min) {
    uint64_t s = (npairs + kSegTarget - 1) / kSegTarget;
    if (s < seg_min) s = seg_min;
    s = (s + nt - 1) / nt * nt;
    return (uint32_t)(s < 0x7FFFFFFFull ? s : 0x7FFFFFFFull);
}
// Segment bookkeeping for one pass: segment length (from the pair count,
// host value or device pointer), counts per tile, their scans and the
// item -> tile map.  scratch: scan_u32_u64_scratch_bytes(n_tiles).
hipError_t launch_segments(const uint32_t *tile_start, const uint32_t *tile_end,
                           uint32_t n_tiles, uint64_t npairs, const uint64_t *npairs_dev,
                           uint32_t nt, uint32_t seg_min, uint32_t *seg_len, uint32_t *nseg,
                           uint32_t *nmulti, uint64_t *seg_off, uint64_t *part_off,
                           uint32_t *item_tile, uint64_t max_items, void *scratch,
                           hipStream_t s);
// Grid size (upper bound on items) for a pass with npairs pairs.
uint32_t splat_grid(uint32_t n_tiles, uint64_t npairs, uint32_t seg_len);
hipError_t launch_splat(const SplatArgs &a, uint32_t grid, hipStream_t s);
// Persistent multi-view splat (row walk): views (device array of nv <=
// kMaxGroup SplatArgs, written by store_splat_args) share one launch; like
// holds the settings that pick the kernel (tile, ordering, compensation,
// counting, column kernel) and must match every view's.  The views' merge
// kernels follow separately (launch_merge).
// Work is handed out dynamically: next (kUnitCounters uint32, device) holds
// one unit counter per XCD, cleared by the launcher.
constexpr int kMaxGroup = 4;
constexpr int kUnitCounters = 8;
hipError_t store_splat_args(const SplatArgs &a, SplatArgs *dst, hipStream_t s);
hipError_t launch_splat_multi(const SplatArgs *views, int nv, const SplatArgs &like,
                              uint32_t *next, hipStream_t s);
hipError_t launch_merge(const SplatArgs &a, hipStream_t s);

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// Monotone unsigned image of a binary32 value, and its inverse.
__host__ __device__ inline uint32_t order_bits_u(uint32_t b) {
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ inline uint32_t from_order_bits_u(uint32_t k) {
    return (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
}

// Normalised scalar t in [0, 1] (Section 3.2: values are normalised before
// colouring): (g(v) - g(vmin)) / (g(vmax) - g(vmin)) clamped, g = log10 or
// the identity; t = 0 for non-positive values under log10 or an empty range.
__device__ __forceinline__ float normalise_value(float v, float vmin, float vmax, int log_scale) {
    float gv, g0, g1;
    if (log_scale) {
        if (!(v > 0.0f) || !(vmin > 0.0f) || !(vmax > 0.0f)) return 0.0f;
        gv = log10f(v);
        g0 = log10f(vmin);
        g1 = log10f(vmax);
    } else {
        gv = v;
        g0 = vmin;
        g1 = vmax;
    }
    float den = g1 - g0;
    if (!(den > 0.0f)) return 0.0f;
    float t = (gv - g0) / den;
    return fminf(fmaxf(t, 0.0f), 1.0f);
}

// Value range of species s as used for colouring: the given one, or the
// device min/max of the species' valid values (0, 0 when it has none).
__device__ __forceinline__ void species_range(const SpeciesDev &sp, const uint32_t *range_bits,
                                              int s, float *lo, float *hi) {
    *lo = sp.vmin[s];
    *hi = sp.vmax[s];
    if (s < sp.n && sp.auto_range[s] && range_bits) {
        const uint32_t bl = range_bits[2 * s], bh = range_bits[2 * s + 1];
        if (bl == 0xFFFFFFFFu) {
            *lo = *hi = 0.0f;
        } else {
            *lo = __uint_as_float(from_order_bits_u(bl));
            *hi = __uint_as_float(from_order_bits_u(bh));
        }
    }
}

// A named range on the host timeline of a trace (roctx: rocprofv3
// --marker-trace shows it; a plain call into a stub when no tool listens).
struct TraceRange {
    explicit TraceRange(const char *name) { roctxRangePushA(name); }
    ~TraceRange() { roctxRangePop(); }
    TraceRange(const TraceRange &) = delete;
    TraceRange &operator=(const TraceRange &) = delete;
};

}  // namespace splotch
