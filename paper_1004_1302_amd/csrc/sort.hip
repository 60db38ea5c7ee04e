// Device-wide exclusive scans and a stable LSD radix sort of (key, value)
// pairs, written for wave64: 256-thread workgroups, 4096 keys per
// workgroup tile, 8-bit digits.
//
// Each radix pass is reduce-then-scan: a histogram kernel counts digits per
// tile (digit-major, so one exclusive scan yields every tile's output
// offset per digit), then the scatter kernel ranks keys inside the tile
// (wave ballots find equal digits, lanes in order, waves in order: stable),
// reorders the tile in LDS and writes each digit run contiguously.
#include <algorithm>

#include "internal.h"

namespace splotch {

namespace {

constexpr int kT = 256;
constexpr int kW = kT / 64;
constexpr int kIpt = 16;
constexpr int kTile = kT * kIpt;  // 4096

__device__ __forceinline__ uint32_t shfl_up_u32(uint32_t v, int o) {
    return (uint32_t)__shfl_up((int)v, o, 64);
}
__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t v, int o) {
    uint32_t lo = shfl_up_u32((uint32_t)v, o), hi = shfl_up_u32((uint32_t)(v >> 32), o);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint32_t shfl_up_t(uint32_t v, int o) { return shfl_up_u32(v, o); }
__device__ __forceinline__ uint64_t shfl_up_t(uint64_t v, int o) { return shfl_up_u64(v, o); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T t = shfl_up_t(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

// Exclusive scan across the workgroup (NW waves); s_w has NW slots.
template <int NW, typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *s_w, T *total) {
    T inc = wave_incl_scan(v);
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (lane == 63) s_w[w] = inc;
    __syncthreads();
    T pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        T x = s_w[k];
        if (k < w) pre += x;
        tot += x;
    }
    *total = tot;
    __syncthreads();
    return pre + inc - v;
}

__device__ __forceinline__ int pad(int i) { return i + (i >> 4); }

// Scan inputs: plain values, or tile counts decoded from a tagged
// processing order (see radix_sort_pairs).
// A load is split in two steps, raw() and finish(), so that a workgroup
// issues all of its streaming loads before the rare dependent ones.
template <typename TI>
struct LoadPlain {
    const TI *p;
    __device__ __forceinline__ TI raw(size_t i) const { return p[i]; }
    __device__ __forceinline__ TI finish(TI r) const { return r; }
};
struct LoadTaggedCount {
    const uint32_t *order, *cnt;
    __device__ __forceinline__ uint32_t raw(size_t i) const { return order[i]; }
    __device__ __forceinline__ uint32_t finish(uint32_t v) const {
        const uint32_t code = v >> kTagShift;
        return code == 0 ? cnt[v & kIdxMask] : (code == 3 ? 4u : code);
    }
};

template <typename L, typename TO>
__global__ __launch_bounds__(kT) void k_scan_reduce(L in, size_t n, TO *partial) {
    __shared__ TO s_w[kW];
    const size_t base = (size_t)blockIdx.x * kTile;
    decltype(in.raw(0)) r[kIpt];
#pragma unroll
    for (int q = 0; q < kIpt; ++q) {
        size_t idx = base + (size_t)q * kT + threadIdx.x;
        if (idx < n) r[q] = in.raw(idx);
    }
    TO s = 0;
#pragma unroll
    for (int q = 0; q < kIpt; ++q) {
        size_t idx = base + (size_t)q * kT + threadIdx.x;
        if (idx < n) s += (TO)in.finish(r[q]);
    }
    TO tot;
    block_excl_scan<kW>(s, s_w, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

template <typename TO>
__global__ __launch_bounds__(1024) void k_scan_partials(TO *partial, size_t m, TO *total_out) {
    __shared__ TO s_w[16];
    TO carry = 0;
    for (size_t base = 0; base < m; base += 1024) {
        size_t idx = base + threadIdx.x;
        TO v = idx < m ? partial[idx] : (TO)0;
        TO tot;
        TO ex = block_excl_scan<16>(v, s_w, &tot);
        if (idx < m) partial[idx] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename L, typename TO>
__global__ __launch_bounds__(kT) void k_scan_down(L in, TO *out, size_t n, const TO *partial) {
    __shared__ TO s[kTile + kTile / 16];
    __shared__ TO s_w[kW];
    const size_t base = (size_t)blockIdx.x * kTile;
    decltype(in.raw(0)) r[kIpt];
#pragma unroll
    for (int q = 0; q < kIpt; ++q) {
        size_t idx = base + (size_t)q * kT + threadIdx.x;
        if (idx < n) r[q] = in.raw(idx);
    }
#pragma unroll
    for (int q = 0; q < kIpt; ++q) {
        int l = q * kT + threadIdx.x;
        size_t idx = base + l;
        s[pad(l)] = idx < n ? (TO)in.finish(r[q]) : (TO)0;
    }
    __syncthreads();
    TO v[kIpt];
    TO sum = 0;
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
        v[i] = s[pad(threadIdx.x * kIpt + i)];
        sum += v[i];
    }
    TO tot;
    TO run = partial[blockIdx.x] + block_excl_scan<kW>(sum, s_w, &tot);
#pragma unroll
    for (int i = 0; i < kIpt; ++i) {
        s[pad(threadIdx.x * kIpt + i)] = run;
        run += v[i];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kIpt; ++q) {
        int l = q * kT + threadIdx.x;
        size_t idx = base + l;
        if (idx < n) out[idx] = s[pad(l)];
    }
}

// A scan of at most kSmallTiles tiles in one workgroup: the tiles one after
// another, each as in k_scan_down with the running total as its partial.
// One launch instead of three for the short scans (digit histograms and
// segment counts of small views, where launches dominate).
constexpr size_t kSmallTiles = 4;

template <typename L, typename TO>
__global__ __launch_bounds__(kT) void k_scan_small(L in, TO *out, size_t n, TO *total_out) {
    __shared__ TO s[kTile + kTile / 16];
    __shared__ TO s_w[kW];
    TO carry = 0;
    for (size_t base = 0; base < n; base += kTile) {
        decltype(in.raw(0)) r[kIpt];
#pragma unroll
        for (int q = 0; q < kIpt; ++q) {
            size_t idx = base + (size_t)q * kT + threadIdx.x;
            if (idx < n) r[q] = in.raw(idx);
        }
#pragma unroll
        for (int q = 0; q < kIpt; ++q) {
            int l = q * kT + threadIdx.x;
            size_t idx = base + l;
            s[pad(l)] = idx < n ? (TO)in.finish(r[q]) : (TO)0;
        }
        __syncthreads();
        TO v[kIpt];
        TO sum = 0;
#pragma unroll
        for (int i = 0; i < kIpt; ++i) {
            v[i] = s[pad(threadIdx.x * kIpt + i)];
            sum += v[i];
        }
        TO tot;
        TO run = carry + block_excl_scan<kW>(sum, s_w, &tot);
#pragma unroll
        for (int i = 0; i < kIpt; ++i) {
            s[pad(threadIdx.x * kIpt + i)] = run;
            run += v[i];
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kIpt; ++q) {
            int l = q * kT + threadIdx.x;
            size_t idx = base + l;
            if (idx < n) out[idx] = s[pad(l)];
        }
        carry += tot;
        __syncthreads();  // before the next tile overwrites s
    }
    if (threadIdx.x == 0 && total_out) *total_out = carry;
}

template <typename TO>
__global__ void k_set_value(TO *p, TO v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

// Partials one workgroup scans in turn; more than that are scanned by the
// same three kernels (one level down), which the scratch then also holds.
constexpr size_t kPartialsOneGroup = 16 * 1024;

size_t scan_scratch_words(size_t n) {
    const size_t nb = (n + kTile - 1) / kTile;
    size_t w = nb + 1;
    if (nb > kPartialsOneGroup) w += scan_scratch_words(nb);
    return w;
}

template <typename L, typename TO>
hipError_t scan_impl(L in, TO *out, size_t n, TO *total_out, void *scratch, hipStream_t s) {
    if (n == 0) {
        if (total_out) hipLaunchKernelGGL(k_set_value<TO>, dim3(1), dim3(64), 0, s, total_out, (TO)0);
        return hipGetLastError();
    }
    size_t nb = (n + kTile - 1) / kTile;
    if (nb <= kSmallTiles) {
        hipLaunchKernelGGL((k_scan_small<L, TO>), dim3(1), dim3(kT), 0, s, in, out, n, total_out);
        return hipGetLastError();
    }
    TO *partial = reinterpret_cast<TO *>(scratch);
    hipLaunchKernelGGL((k_scan_reduce<L, TO>), dim3((unsigned)nb), dim3(kT), 0, s, in, n,
                       partial);
    if (nb > kPartialsOneGroup) {
        // the partials' exclusive scan in place, its own partials after them
        hipError_t e = scan_impl<LoadPlain<TO>, TO>(LoadPlain<TO>{partial}, partial, nb, total_out,
                                                    partial + nb + 1, s);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_scan_partials<TO>, dim3(1), dim3(1024), 0, s, partial, nb,
                           total_out);
    }
    hipLaunchKernelGGL((k_scan_down<L, TO>), dim3((unsigned)nb), dim3(kT), 0, s, in, out, n,
                       partial);
    return hipGetLastError();
}

// ---------------------------------------------------------------- radix sort
__device__ __forceinline__ size_t live_count(size_t n, const uint64_t *n_dev) {
    if (!n_dev) return n;
    const uint64_t d = *n_dev;
    return d < n ? (size_t)d : n;
}

// Identity value with the tile count in the top bits (0 = look it up).
__device__ __forceinline__ uint32_t tag_value(uint32_t idx, uint32_t count) {
    const uint32_t code = count == 1 ? 1u : (count == 2 ? 2u : (count == 4 ? 3u : 0u));
    return idx | (code << kTagShift);
}

// Tiles of a radix pass: one workgroup per tile.  With a count on the
// device (batched views: the pair arrays are sized to their capacity) the
// live tiles are those the device count fills, and the XCD-contiguous
// order is taken over them, so every XCD shares the live work; the
// capacity's other workgroups write zero histogram columns or return.
struct PassTiles {
    uint32_t live;  // tiles holding elements
    uint32_t all;   // tiles of the capacity (the histogram's columns)
    __device__ PassTiles(size_t n_live, uint32_t nblocks) {
        const size_t t = (n_live + kTile - 1) / kTile;
        live = t < nblocks ? (uint32_t)t : nblocks;
        all = nblocks;
    }
    // tile of workgroup b (b < live: XCD-contiguous among the live)
    __device__ uint32_t tile(uint32_t b) const {
        return b < live ? xcd_contiguous(b, live) : b;
    }
};

// A sort whose key range is on the device (the views of a batch, where
// nothing is read back): the passes subtract the smallest key and sort as
// many digits as the range spans; the remaining pass slots return at once.
// The values go from slot to slot so that the last sorting pass writes v0,
// and that pass writes no keys.
struct DeviceKeys {
    const uint32_t *range;  // [smallest, largest] key (smallest > largest: none); null: host plan
    uint32_t *v0, *v1;
    int slot;
    // false when this slot has nothing to sort
    __device__ bool resolve(int db, uint32_t *bias, int *passes) const {
        const uint32_t lo = range[0], hi = range[1];
        int bits = 1;
        *bias = 0;
        if (lo <= hi) {
            *bias = lo;
            const uint32_t span = hi - lo;
            bits = span == 0 ? 1 : 32 - __clz((int)span);
        }
        *passes = (bits + db - 1) / db;
        return slot < *passes;
    }
};

// Digit histogram of one tile.  16 copies of the counters (by lane mod 16)
// keep a wave whose keys share a digit from serialising on one LDS address.
constexpr int kHistCopies = 16;

// One workgroup per tile of the capacity.  DB: digit bits (7 or 8): the
// histogram has 2^DB columns per tile.
template <int DB>
__global__ __launch_bounds__(kT) void k_rs_hist(const uint32_t *keys, size_t n_cap,
                                                const uint64_t *n_dev, int shift, uint32_t bias,
                                                uint32_t *hist, uint32_t nblocks, DeviceKeys dk) {
    constexpr uint32_t ND = 1u << DB, DM = ND - 1u;
    if (dk.range) {
        int passes;
        if (!dk.resolve(DB, &bias, &passes)) return;
    }
    const size_t n = live_count(n_cap, n_dev);
    const PassTiles pt(n, nblocks);
    __shared__ uint32_t sh[kHistCopies][ND];
    const int c = threadIdx.x & (kHistCopies - 1);
    // neighbouring tiles' counts share lines of the digit-major histogram
    const uint32_t b = blockIdx.x;
    const uint32_t t = pt.tile(b);
    if (b >= pt.live) {
        if (threadIdx.x < ND) hist[(size_t)threadIdx.x * nblocks + t] = 0u;
        return;
    }
    for (int d = threadIdx.x; d < kHistCopies * (int)ND; d += kT) (&sh[0][0])[d] = 0;
    __syncthreads();
    const size_t base = (size_t)t * kTile;
#pragma unroll
    for (int q = 0; q < kIpt; ++q) {
        size_t idx = base + (size_t)q * kT + threadIdx.x;
        if (idx < n) atomicAdd(&sh[c][((keys[idx] - bias) >> shift) & DM], 1u);
    }
    __syncthreads();
    if (threadIdx.x < ND) {
        uint32_t sum = 0;
#pragma unroll
        for (int k = 0; k < kHistCopies; ++k) sum += sh[k][threadIdx.x];
        hist[(size_t)threadIdx.x * nblocks + t] = sum;
    }
}

// Rank the keys of tile t inside the tile (wave ballots find equal digits,
// lanes in order, waves in order: stable), reorder the tile in LDS and
// write each digit run contiguously.
template <int DB>
struct ScatterLds {
    uint32_t k[kTile], v[kTile];
    uint32_t wc[kW][1 << DB];
    uint32_t bs[1 << DB], go[1 << DB], sw[kW];
};

template <int DB>
__device__ __forceinline__ void scatter_tile(ScatterLds<DB> &L, uint32_t t, size_t n,
                                             const uint32_t *kin, const uint32_t *vin,
                                             uint32_t *kout, uint32_t *vout, int shift,
                                             uint32_t bias, const uint32_t *hist,
                                             uint32_t nblocks, int write_keys,
                                             const uint32_t *tag) {
    constexpr uint32_t ND = 1u << DB, DM = ND - 1u;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const size_t base = (size_t)t * kTile;
    for (int d = tid; d < kW * (int)ND; d += kT) (&L.wc[0][0])[d] = 0;
    // dg: the key's digit; entries past the live count take digit 255 so
    // that they rank after every live entry of the tile
    uint32_t k[kIpt], v[kIpt], r[kIpt], dg[kIpt];
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        size_t idx = base + (size_t)w * (kIpt * 64) + (size_t)j * 64 + lane;
        if (idx < n) {
            k[j] = kin[idx];
            v[j] = vin ? vin[idx] : (tag ? tag_value((uint32_t)idx, tag[idx]) : (uint32_t)idx);
            dg[j] = ((k[j] - bias) >> shift) & DM;
        } else {
            k[j] = 0xFFFFFFFFu;
            v[j] = 0u;
            dg[j] = DM;
        }
    }
    __syncthreads();
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t d = dg[j];
        uint64_t m = ~0ull;
#pragma unroll
        for (int b = 0; b < DB; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bal = __ballot(bit);
            m &= bit ? bal : ~bal;
        }
        const uint32_t rank = (uint32_t)__popcll(m & lt);
        const uint32_t c = L.wc[w][d];
        r[j] = c + rank;
        if (rank == 0) L.wc[w][d] = c + (uint32_t)__popcll(m);
    }
    __syncthreads();
    // one thread per digit; the others add nothing to the scan
    const int dd = tid & (int)DM;
    uint32_t wpre[kW];
    uint32_t dtot = 0;
#pragma unroll
    for (int ww = 0; ww < kW; ++ww) {
        wpre[ww] = dtot;
        dtot += L.wc[ww][dd];
    }
    if (tid >= (int)ND) dtot = 0;
    uint32_t tot;
    uint32_t ex = block_excl_scan<kW>(dtot, L.sw, &tot);
    if (tid < (int)ND) {
        L.bs[tid] = ex;
#pragma unroll
        for (int ww = 0; ww < kW; ++ww) L.wc[ww][tid] = wpre[ww];
        L.go[tid] = hist[(size_t)tid * nblocks + t];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kIpt; ++j) {
        const uint32_t d = dg[j];
        const uint32_t pos = L.bs[d] + L.wc[w][d] + r[j];
        L.k[pos] = k[j];
        L.v[pos] = v[j];
    }
    __syncthreads();
    const size_t rem = n - base;
    const int nvalid = rem < (size_t)kTile ? (int)rem : kTile;
#pragma unroll
    for (int q = 0; q < kIpt; ++q) {
        int p = q * kT + tid;
        if (p < nvalid) {
            uint32_t key = L.k[p];
            uint32_t d = ((key - bias) >> shift) & DM;
            size_t g = (size_t)L.go[d] + (size_t)(p - (int)L.bs[d]);
            if (write_keys) kout[g] = key;
            vout[g] = L.v[p];
        }
    }
}

template <int DB>
__global__ __launch_bounds__(kT) void k_rs_scatter(const uint32_t *kin, const uint32_t *vin,
                                                   uint32_t *kout, uint32_t *vout, size_t n_cap,
                                                   const uint64_t *n_dev, int shift,
                                                   uint32_t bias, const uint32_t *hist,
                                                   uint32_t nblocks, int write_keys,
                                                   const uint32_t *tag, DeviceKeys dk) {
    const size_t n = live_count(n_cap, n_dev);
    __shared__ ScatterLds<DB> L;
    if (dk.range) {
        int passes;
        if (!dk.resolve(DB, &bias, &passes)) return;
        if (dk.slot > 0) vin = ((passes - dk.slot) & 1) ? dk.v1 : dk.v0;
        vout = ((passes - 1 - dk.slot) & 1) ? dk.v1 : dk.v0;
        if (dk.slot == passes - 1) write_keys = 0;
    }
    // one workgroup per tile of the capacity; those past the live tiles (a
    // count on the device) return at once.  The runs two neighbouring tiles
    // write for one digit are adjacent in the output.
    const PassTiles pt(n, nblocks);
    if (blockIdx.x < pt.live)
        scatter_tile(L, pt.tile(blockIdx.x), n, kin, vin, kout, vout, shift, bias, hist, nblocks,
                     write_keys, tag);
}

}  // namespace

size_t scan_u32_u64_scratch_bytes(size_t n) {
    return align_up(scan_scratch_words(n) * sizeof(uint64_t), 256);
}

hipError_t launch_scan_u32_u64(const uint32_t *in, uint64_t *out, size_t n, void *scratch,
                               hipStream_t s) {
    return scan_impl<LoadPlain<uint32_t>, uint64_t>(LoadPlain<uint32_t>{in}, out, n, out + n,
                                                    scratch, s);
}

hipError_t launch_scan_tagged_counts(const uint32_t *order, const uint32_t *cnt, uint64_t *out,
                                     size_t n, void *scratch, hipStream_t s) {
    return scan_impl<LoadTaggedCount, uint64_t>(LoadTaggedCount{order, cnt}, out, n, out + n,
                                                scratch, s);
}

size_t scan_u32_scratch_bytes(size_t n) {
    return align_up(scan_scratch_words(n) * sizeof(uint32_t), 256);
}

hipError_t launch_scan_u32(uint32_t *data, size_t n, void *scratch, hipStream_t s) {
    return scan_impl<LoadPlain<uint32_t>, uint32_t>(LoadPlain<uint32_t>{data}, data, n, nullptr,
                                                    scratch, s);
}

size_t radix_scratch_bytes(size_t n) {
    size_t nb = (n + kTile - 1) / kTile;
    if (nb == 0) nb = 1;
    size_t hist = align_up(nb * 256 * sizeof(uint32_t), 256);
    return hist + scan_u32_scratch_bytes(nb * 256);
}

// One pass: digit histogram per tile, its scan, the scatter.  A count on
// the device (n_dev) bounds the live tiles; the grid covers the capacity.
template <int DB>
hipError_t radix_pass(const uint32_t *kin, const uint32_t *vin, uint32_t *kout, uint32_t *vout,
                      size_t n, const uint64_t *n_dev, int shift, uint32_t bias, uint32_t *hist,
                      uint32_t nb, int write_keys, const uint32_t *tag, DeviceKeys dk,
                      void *scan_scratch, hipStream_t s) {
    hipLaunchKernelGGL((k_rs_hist<DB>), dim3(nb), dim3(kT), 0, s, kin, n, n_dev, shift, bias, hist,
                       nb, dk);
    hipError_t e = launch_scan_u32(hist, (size_t)nb << DB, scan_scratch, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_rs_scatter<DB>), dim3(nb), dim3(kT), 0, s, kin, vin, kout, vout, n,
                       n_dev, shift, bias, hist, nb, write_keys, tag, dk);
    return hipGetLastError();
}

hipError_t radix_sort_pairs(uint32_t *k0, uint32_t *v0, uint32_t *k1, uint32_t *v1,
                            bool vals_identity, size_t n, const uint64_t *n_dev, int bits,
                            uint32_t bias, bool keys_needed, void *scratch, bool *result_in_1,
                            hipStream_t s, const uint32_t *tag_counts,
                            const uint32_t *key_range) {
    *result_in_1 = false;
    if (n == 0) return hipSuccess;
    if (key_range && (keys_needed || n_dev)) return hipErrorInvalidValue;
    const uint32_t nb = (uint32_t)((n + kTile - 1) / kTile);
    uint32_t *hist = reinterpret_cast<uint32_t *>(scratch);
    void *scan_scratch =
        reinterpret_cast<char *>(scratch) + align_up((size_t)nb * 256 * sizeof(uint32_t), 256);
    if (key_range) bits = 32;  // the passes the range needs are found on the device
    const int passes = bits <= 0 ? 1 : (bits + 7) / 8;
    // 7-bit digits when they cover the key in as many passes: half the
    // histogram, and digit runs twice as long in the scatter's writes
    const int db = !key_range && bits > 0 && bits <= 7 * passes ? 7 : 8;
    int src = 0;
    for (int p = 0; p < passes; ++p) {
        uint32_t *kin = src ? k1 : k0, *vin = src ? v1 : v0;
        uint32_t *kout = src ? k0 : k1, *vout = src ? v0 : v1;
        const int shift = db * p;
        const bool last = p == passes - 1;
        const uint32_t *vsrc = (p == 0 && vals_identity) ? (const uint32_t *)nullptr : vin;
        const uint32_t *tag = (p == 0 && vals_identity) ? tag_counts : nullptr;
        const int wk = (!last || keys_needed) ? 1 : 0;
        const DeviceKeys dk{key_range, v0, v1, p};
        hipError_t e = db == 7 ? radix_pass<7>(kin, vsrc, kout, vout, n, n_dev, shift, bias, hist,
                                               nb, wk, tag, dk, scan_scratch, s)
                               : radix_pass<8>(kin, vsrc, kout, vout, n, n_dev, shift, bias, hist,
                                               nb, wk, tag, dk, scan_scratch, s);
        if (e != hipSuccess) return e;
        src ^= 1;
    }
    // a device plan leaves the values in v0
    *result_in_1 = !key_range && src == 1;
    return hipSuccess;
}

}  // namespace splotch
