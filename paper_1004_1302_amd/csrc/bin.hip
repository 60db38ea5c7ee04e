// Screen-tile binning: each visible particle emits one (tile, particle)
// pair per tile its footprint box touches (Section 3.2: the screen area a
// particle affects; the paper's split of large particles into pixel
// subsets becomes this per-tile duplication).  Pairs are emitted in
// processing order (particle index, or front-to-back depth order), so a
// stable sort by tile leaves every tile's list in that order.
#include <algorithm>

#include "internal.h"

namespace splotch {

namespace {

constexpr int kThreads = 256;
static_assert(kThreads == (int)kEmitGroup, "one split-queue part per emission workgroup");

__global__ void k_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, size_t n) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride)
        dst[k] = src[idx[k]];
}

// The pair key of tile (tx, ty) for a particle box [i0, i1] x [j0, j1]
// (its second record word b1 carries the corner bits): the tile index, and
// above it (qshift > 0) the mask of the tile's 8x8 blocks the box meets (a
// rectangle of them), less the box's corner blocks in this tile that the
// corner bits mark as holding no pixel within the radius.
__device__ __forceinline__ uint32_t pair_key(const EmitArgs &a, int tx, int ty, int i0, int i1,
                                             int j0, int j1, uint32_t b1) {
    const int T = a.tile, QW = T / 8;
    uint32_t key = (uint32_t)(ty * a.ntx + tx);
    if (a.qshift) {
        const int x0 = tx * T, y0 = ty * T;
        const int qx0 = (max(i0, x0) - x0) >> 3, qx1 = (min(i1, x0 + T - 1) - x0) >> 3;
        const int qy0 = (max(j0, y0) - y0) >> 3, qy1 = (min(j1, y0 + T - 1) - y0) >> 3;
        const uint32_t row = ((2u << qx1) - 1u) & ~((1u << qx0) - 1u);
        uint32_t m = 0;
        for (int qy = qy0; qy <= qy1; ++qy) m |= row << (qy * QW);
        const uint32_t cb = b1 >> kCornerShift;
        if (cb) {
            // a box corner lies in this tile when the box's edges do
            const bool lo_x = i0 >= x0, hi_x = i1 <= x0 + T - 1;
            const bool lo_y = j0 >= y0, hi_y = j1 <= y0 + T - 1;
            if ((cb & 1u) && lo_x && lo_y) m &= ~(1u << (qy0 * QW + qx0));
            if ((cb & 2u) && hi_x && lo_y) m &= ~(1u << (qy0 * QW + qx1));
            if ((cb & 4u) && lo_x && hi_y) m &= ~(1u << (qy1 * QW + qx0));
            if ((cb & 8u) && hi_x && hi_y) m &= ~(1u << (qy1 * QW + qx1));
        }
        key |= m << a.qshift;
    }
    return key;
}

// One thread per particle in processing order writes its pairs at its
// offset, tile rows bottom to top, tiles left to right, skipping the tiles
// a tile mask leaves out.  Used with a tile mask; no particle is split.
__global__ __launch_bounds__(kThreads) void k_emit(EmitArgs a) {
    const uint64_t k = a.first + (uint64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= a.last) return;
    const uint64_t o0 = a.off[k];
    const uint32_t c = (uint32_t)(a.off[k + 1] - o0);
    if (c == 0) return;
    const uint32_t i = a.order ? (a.order[k] & a.idx_mask) : (uint32_t)k;
    const uint2 bb = *reinterpret_cast<const uint2 *>(&a.rec[i].a);
    const int T = a.tile;
    const int tx0 = (int)(bb.x & kBboxMask) / T, tx1 = (int)((bb.x >> kBboxBits) & kBboxMask) / T;
    const int ty0 = (int)(bb.y & kBboxMask) / T, ty1 = (int)((bb.y >> kBboxBits) & kBboxMask) / T;
    uint64_t o = o0 - a.base;
    // Past the capacity (possible only where no host plan chunks the pass):
    // write the pairs that fit, so every slot below the capacity holds a
    // valid pair, and flag the pass.
    if (o + c > a.cap && a.overflow) *a.overflow = 1u;
    const int i0 = (int)(bb.x & kBboxMask), i1 = (int)((bb.x >> kBboxBits) & kBboxMask);
    const int j0 = (int)(bb.y & kBboxMask), j1 = (int)((bb.y >> kBboxBits) & kBboxMask);
    for (int ty = ty0; ty <= ty1; ++ty)
        for (int tx = tx0; tx <= tx1; ++tx) {
            if (a.tile_mask && !a.tile_mask[ty * a.ntx + tx]) continue;
            if (o >= a.cap) return;
            a.pair_key[o] = pair_key(a, tx, ty, i0, i1, j0, j1, bb.y);
            a.pair_val[o] = i;
            ++o;
        }
}

// The same pairs written by waves: a wave takes 64 consecutive processing
// positions, whose pairs fill one run of slots, and lane l writes the
// run's slots l, l + 64, ...  A slot's particle is the last of the wave's
// 64 whose first slot is at or before it (a binary search over the first
// slots, kept in LDS), and its tile is the slot's rank in that particle's
// box in k_emit's order (rows bottom to top, tiles left to right).  Every
// lane then does the same work however unevenly the tile counts spread,
// and each store writes consecutive slots.  Split particles are left out
// of the run (their slots are written by k_emit_split) and queued in the
// workgroup's own part of the split list, counted in LDS: a counter shared
// by the whole grid would take one device-scope atomic per queued particle
// or wave, and those are serialised beyond the XCDs' L2 caches.  Used without a tile
// mask, where a particle's t-th pair is the t-th tile of its box.
__global__ __launch_bounds__(kThreads) void k_emit_waves(EmitArgs a) {
    __shared__ uint32_t s_first[kThreads];  // first slot in the wave's run
    __shared__ uint32_t s_off[kThreads];    // first slot, from the wave's first pair
    __shared__ uint32_t s_b0[kThreads], s_b1[kThreads], s_idx[kThreads];
    __shared__ uint32_t s_nsplit;
    if (threadIdx.x == 0) s_nsplit = 0;
    __syncthreads();
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t w0 = threadIdx.x & ~63u;
    const uint64_t k0 = a.first + (uint64_t)blockIdx.x * kThreads + w0;
    const uint64_t k = k0 + lane;
    const bool valid = k < a.last;
    uint64_t o0 = 0;
    uint32_t c = 0, i = 0;
    bool split = false;
    uint2 bb = make_uint2(0u, 0u);
    if (valid) {
        o0 = a.off[k];
        c = (uint32_t)(a.off[k + 1] - o0);
        if (c) {
            i = a.order ? (a.order[k] & a.idx_mask) : (uint32_t)k;
            bb = *reinterpret_cast<const uint2 *>(&a.rec[i].a);
            if (a.split_list) {
                const uint64_t bw = ((bb.x >> kBboxBits) & kBboxMask) - (bb.x & kBboxMask) + 1;
                const uint64_t bh = ((bb.y >> kBboxBits) & kBboxMask) - (bb.y & kBboxMask) + 1;
                split = bw * bh > a.split_pixels;
            }
            if (split) {
                const uint32_t q = atomicAdd(&s_nsplit, 1u);
                a.split_list[(size_t)blockIdx.x * kThreads + q] = (uint32_t)k;
            } else if (o0 - a.base + c > a.cap && a.overflow) {
                *a.overflow = 1u;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x == 0 && a.split_list) a.split_count[blockIdx.x] = s_nsplit;
    if (k0 >= a.last) return;  // the whole wave is past the end
    // the wave's run: its particles' slots in order, split ones left out
    // (at most 64 particles of at most (16384 / 8)^2 tiles each)
    const uint32_t ce = split ? 0u : c;
    uint32_t incl = ce;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t t = (uint32_t)__shfl_up((int)incl, d, 64);
        if ((int)lane >= d) incl += t;
    }
    const uint32_t total = (uint32_t)__shfl((int)incl, 63, 64);
    const uint64_t wb = a.off[k0];
    s_first[threadIdx.x] = incl - ce;
    s_off[threadIdx.x] = (uint32_t)(o0 - wb);
    s_b0[threadIdx.x] = bb.x;
    s_b1[threadIdx.x] = bb.y;
    s_idx[threadIdx.x] = i;
    // the wave reads back its own entries (a wave's LDS requests complete
    // in order)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const int T = a.tile;
    const uint64_t slot0 = wb - a.base;
    for (uint32_t j = lane; j < total; j += 64) {
        // lane 0's first slot is 0 and the first slots never decrease; a
        // particle without slots in the run shares its first slot with the
        // next particle, which the search then takes
        uint32_t p = 0;
#pragma unroll
        for (uint32_t step = 32; step > 0; step >>= 1)
            if (s_first[w0 + p + step] <= j) p += step;
        const uint32_t e = w0 + p;
        const uint32_t t = j - s_first[e];
        const uint64_t slot = slot0 + s_off[e] + t;
        if (slot >= a.cap) continue;
        const uint32_t b0 = s_b0[e], b1 = s_b1[e];
        const int i0 = (int)(b0 & kBboxMask), i1 = (int)((b0 >> kBboxBits) & kBboxMask);
        const int j0 = (int)(b1 & kBboxMask), j1 = (int)((b1 >> kBboxBits) & kBboxMask);
        const int tx0 = i0 / T, ty0 = j0 / T;
        const uint32_t nx = (uint32_t)(i1 / T - tx0 + 1);
        const uint32_t row = t / nx;
        const int tx = tx0 + (int)(t - row * nx), ty = ty0 + (int)row;
        a.pair_key[slot] = pair_key(a, tx, ty, i0, i1, j0, j1, b1);
        a.pair_val[slot] = s_idx[e];
    }
}

// The queued split particles into one dense queue: thread b copies the
// part of emission workgroup b to its place in the counts' scan.
__global__ void k_split_compact(EmitArgs a, uint32_t nblocks) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nblocks) return;
    const uint32_t m = a.split_count[b];
    const uint64_t o = a.split_off[b];
    for (uint32_t q = 0; q < m; ++q) a.split_dense[o + q] = a.split_list[(size_t)b * kThreads + q];
}

// Split particles: the waves of the grid take the dense queue's particles
// in turn, and a wave's lanes write pair t of its particle (its t-th tile,
// in k_emit's order) at the particle's offset + t.
__global__ __launch_bounds__(kThreads) void k_emit_split(EmitArgs a, uint32_t nblocks) {
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t total = a.split_off[nblocks];
    const uint64_t waves = (uint64_t)gridDim.x * (kThreads / 64);
    for (uint64_t e = (uint64_t)blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6); e < total;
         e += waves) {
        const uint64_t k = a.split_dense[e];
        const uint64_t o0 = a.off[k];
        const uint32_t c = (uint32_t)(a.off[k + 1] - o0);
        const uint32_t i = a.order ? (a.order[k] & a.idx_mask) : (uint32_t)k;
        const uint2 bb = *reinterpret_cast<const uint2 *>(&a.rec[i].a);
        const int T = a.tile;
        const int i0 = (int)(bb.x & kBboxMask), i1 = (int)((bb.x >> kBboxBits) & kBboxMask);
        const int j0 = (int)(bb.y & kBboxMask), j1 = (int)((bb.y >> kBboxBits) & kBboxMask);
        const int tx0 = i0 / T, ty0 = j0 / T, nx = i1 / T - tx0 + 1;
        const uint64_t o = o0 - a.base;
        if (o + c > a.cap && a.overflow && lane == 0) *a.overflow = 1u;
        for (uint32_t t = lane; t < c; t += 64) {
            if (o + t >= a.cap) break;
            const int tx = tx0 + (int)(t % (uint32_t)nx), ty = ty0 + (int)(t / (uint32_t)nx);
            a.pair_key[o + t] = pair_key(a, tx, ty, i0, i1, j0, j1, bb.y);
            a.pair_val[o + t] = i;
        }
    }
}

// Boundaries of each tile's run in the sorted pair keys.  Each thread
// takes four consecutive keys (one 16-byte load) plus its right neighbour.
__global__ void k_tile_ranges(const uint32_t *keys, size_t n_cap, const uint64_t *n_dev,
                              uint32_t *start, uint32_t *end, uint32_t n_tiles,
                              uint32_t key_mask) {
    size_t n = n_cap;
    if (n_dev && *n_dev < n) n = (size_t)*n_dev;
    const size_t nq = (n + 3) / 4;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t q = (size_t)blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += stride) {
        const size_t p0 = 4 * q;
        uint32_t k[5];
        if (p0 + 4 <= n) {
            const uint4 v = *reinterpret_cast<const uint4 *>(keys + p0);
            k[0] = v.x & key_mask;
            k[1] = v.y & key_mask;
            k[2] = v.z & key_mask;
            k[3] = v.w & key_mask;
        } else {
            for (int j = 0; j < 4; ++j) k[j] = p0 + j < n ? (keys[p0 + j] & key_mask) : 0xFFFFFFFFu;
        }
        const uint32_t prev = p0 > 0 ? (keys[p0 - 1] & key_mask) : 0xFFFFFFFFu;
        k[4] = p0 + 4 < n ? (keys[p0 + 4] & key_mask) : 0xFFFFFFFFu;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const size_t p = p0 + j;
            if (p >= n) break;
            const uint32_t key = k[j];
            if (key >= n_tiles) continue;  // cannot happen for emitted pairs; keeps stores in bounds
            const uint32_t before = j == 0 ? prev : k[j - 1];
            if (p == 0 || before != key) start[key] = (uint32_t)p;
            if (p == n - 1 || k[j + 1] != key) end[key] = (uint32_t)(p + 1);
        }
    }
}

// Greedy chunk plan over the pair offsets: chunk c covers processing
// positions [bounds[2c], bounds[2c+2]) with pair offsets bounds[2c+1] ...
// Layout: bounds[0] = number of chunks, bounds[1] = 1 if one particle
// alone exceeds the capacity; then pairs (position, offset) for each
// boundary starting at (0, 0).
__global__ void k_chunk_plan(const uint64_t *off, uint64_t n, uint64_t cap, uint64_t *bounds,
                             uint32_t max_chunks) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    uint64_t b = 0;
    uint32_t c = 0;
    bounds[1] = 0;
    bounds[2] = 0;
    bounds[3] = off[0];
    while (b < n && c < max_chunks) {
        const uint64_t target = off[b] + cap;
        uint64_t lo = b, hi = n;  // invariant: off[lo] <= target
        while (lo < hi) {
            uint64_t mid = lo + (hi - lo + 1) / 2;
            if (off[mid] <= target)
                lo = mid;
            else
                hi = mid - 1;
        }
        if (lo == b) {
            bounds[1] = 1;
            break;
        }
        ++c;
        bounds[2 + 2 * c] = lo;
        bounds[3 + 2 * c] = off[lo];
        b = lo;
    }
    if (b < n && bounds[1] == 0) bounds[1] = 2;  // ran out of chunk slots
    bounds[0] = c;
}

unsigned grid_for(size_t n, unsigned cap) {
    size_t g = (n + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_gather_u32(const uint32_t *src, const uint32_t *idx, uint32_t *dst, size_t n,
                             hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_u32, dim3(grid_for(n, 1u << 20)), dim3(kThreads), 0, s, src, idx,
                       dst, n);
    return hipGetLastError();
}

hipError_t launch_emit(const EmitArgs &a, hipStream_t s) {
    const uint64_t n = a.last - a.first;
    if (n == 0) return hipSuccess;
    EmitArgs e = a;
    if (e.tile_mask) e.split_list = nullptr;  // split only where pair t is tile t
    const uint32_t nblocks = (uint32_t)((n + kThreads - 1) / kThreads);
    if (e.tile_mask)
        hipLaunchKernelGGL(k_emit, dim3(nblocks), dim3(kThreads), 0, s, e);
    else
        hipLaunchKernelGGL(k_emit_waves, dim3(nblocks), dim3(kThreads), 0, s, e);
    hipError_t r = hipGetLastError();
    if (r != hipSuccess || !e.split_list) return r;
    if ((r = launch_scan_u32_u64(e.split_count, e.split_off, nblocks, e.split_scratch, s)) !=
        hipSuccess)
        return r;
    hipLaunchKernelGGL(k_split_compact, dim3((nblocks + kThreads - 1) / kThreads), dim3(kThreads),
                       0, s, e, nblocks);
    if ((r = hipGetLastError()) != hipSuccess) return r;
    hipLaunchKernelGGL(k_emit_split, dim3(2048), dim3(kThreads), 0, s, e, nblocks);
    return hipGetLastError();
}

hipError_t launch_tile_ranges(const uint32_t *sorted_keys, size_t n_pairs,
                              const uint64_t *n_pairs_dev, uint32_t *start, uint32_t *end,
                              uint32_t n_tiles, uint32_t key_mask, hipStream_t s) {
    hipError_t e = launch_fill_u32(start, 0u, n_tiles, s);
    if (e != hipSuccess) return e;
    e = launch_fill_u32(end, 0u, n_tiles, s);
    if (e != hipSuccess || n_pairs == 0) return e;
    // a count on the device (capacity-sized arrays): a capped grid strides
    // over the live pairs
    const unsigned cap = n_pairs_dev ? 8192u : (1u << 20);
    hipLaunchKernelGGL(k_tile_ranges, dim3(grid_for((n_pairs + 3) / 4, cap)), dim3(kThreads), 0, s,
                       sorted_keys, n_pairs, n_pairs_dev, start, end, n_tiles, key_mask);
    return hipGetLastError();
}

hipError_t launch_chunk_plan(const uint64_t *off, uint64_t n, uint64_t capacity, uint64_t *bounds,
                             uint32_t max_chunks, hipStream_t s) {
    hipLaunchKernelGGL(k_chunk_plan, dim3(1), dim3(64), 0, s, off, n, capacity, bounds,
                       max_chunks);
    return hipGetLastError();
}

}  // namespace splotch
