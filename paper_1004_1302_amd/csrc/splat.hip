// Splat / composite: one workgroup per screen tile, one lane per pixel.
//
// Section 2 of the paper: each particle's density is rho0 exp(-r^2/sigma^2)
// cut at f sigma; along a pixel's line of sight it contributes the column
// tau = rho0 exp(-q^2), q = d/sigma_s, and the radiative-transfer equation
// dI/dx = (E - A I) rho (Eq. (1)) integrates across it to
//   I <- I exp(-A tau) + E tau phi(A tau),  phi(x) = (1 - exp(-x))/x.
// Front to back this is carried as colour C and transmittance Tr:
//   C += Tr E tau phi(A tau),  Tr *= exp(-A tau),  I_out = C + Tr I_in.
// With A = 0 (additive species) it is a plain sum.
//
// The tile's list (particle indices, front to back or by index) is staged
// through LDS in batches: each lane gathers one 32-byte record and expands
// its colour from the palette once.  Every wave then walks the batch in
// order, skipping records whose footprint box misses the wave's pixel rows
// (a wave-uniform test), and each lane applies the binary32 membership
// test of the index recipe before compositing.  No global atomics: each
// pixel is owned by one lane and written once.
#include "internal.h"

namespace splotch {

namespace {

// Pixel membership: binary32, no contraction (part of the index recipe).
__device__ __forceinline__ float member_d2(int i, int i0, float ur, int j, int j0, float vr) {
#pragma clang fp contract(off)
    float dx = ((float)(i - i0) + 0.5f) - ur;
    float dy = ((float)(j - j0) + 0.5f) - vr;
    return dx * dx + dy * dy;
}

// phi(x) = (1 - exp(-x))/x and exp(-x) = 1 - x phi(x).  For x < 1/32,
// phi comes from its Taylor series to x^3 (the first dropped term, x^4/120,
// is below 8e-9 relative, under binary32 resolution) and exp(-x) from one
// fused multiply-add: this keeps the product of thousands of transmittance
// factors free of the bias a transcendental's last-place error would add,
// and avoids the cancellation in 1 - exp(-x).
constexpr float kSeriesMax = 0.03125f;

__device__ __forceinline__ void ex_phi_small(float x, float &ex, float &ph) {
    ph = 1.0f + x * (-0.5f + x * (1.0f / 6.0f + x * (-1.0f / 24.0f)));
    ex = __builtin_fmaf(-x, ph, 1.0f);
}

__device__ __forceinline__ void ex_phi(float x, float &ex, float &ph) {
    if (x < kSeriesMax) {
        ex_phi_small(x, ex, ph);
    } else {
        ex = __builtin_amdgcn_exp2f(-x * 1.4426950408889634f);
        ph = (1.0f - ex) / x;
    }
}

__device__ __forceinline__ void kahan_add(float &s, float &c, float v) {
    float y = v - c;
    float t = s + y;
    c = (t - s) - y;
    s = t;
}

constexpr uint32_t kRun = 8;  // consecutive items per XCD run

// Final pixel value: composite over the incoming image when accumulating.
template <bool ORDERED>
__device__ __forceinline__ void write_pixel(const SplatArgs &a, int i, int j, float C0, float C1,
                                            float C2, float T0, float T1, float T2) {
    if (i >= a.width || j >= a.height) return;
    const size_t plane = (size_t)a.width * a.height;
    const size_t o = (size_t)j * a.width + i;
    float *img = a.image;
    if (a.accumulate) {
        const float in0 = img[o], in1 = img[plane + o], in2 = img[2 * plane + o];
        if (ORDERED) {
            C0 += T0 * in0;
            C1 += T1 * in1;
            C2 += T2 * in2;
        } else {
            C0 += in0;
            C1 += in1;
            C2 += in2;
        }
    }
    img[o] = C0;
    img[plane + o] = C1;
    img[2 * plane + o] = C2;
}

// Records staged per batch: B indices of at most 8 bits per lane list.
template <int T>
struct Batch {
    static constexpr int NT = T * T;
    static constexpr int B = (32768 / NT) < 128 ? (32768 / NT) : 128;
};

// Two strategies for walking a staged batch (chosen per launch):
//  LISTS = false: every wave walks the batch in order; for each record whose
//    box meets its rows, each lane tests its pixel and members composite
//    (cheap emission-only path, but lanes outside the footprint idle);
//  LISTS = true: phase 1 builds, per lane, the ordered list of member
//    records in LDS; phase 2 walks the lists so every active lane composites
//    (full lane use, at the price of per-lane LDS gathers).
template <int T, bool ORDERED, bool KAHAN, bool LISTS>
__global__ __launch_bounds__(T *T) void k_splat(SplatArgs a) {
    constexpr int NT = T * T;
    constexpr int B = LISTS ? Batch<T>::B : NT;
    constexpr int ROWS = 64 / T;  // pixel rows per wave
    __shared__ uint32_t s_b0[B], s_b1[B];
    __shared__ float s_ur[B], s_vr[B], s_r2[B], s_qs[B];
    __shared__ float s_e[3][B];
    __shared__ float s_a[3][B];
    // per-lane member lists: entry m of lane l at s_list[m * NT + l]
    __shared__ uint8_t s_list[LISTS ? B * NT : 4];

    // Blocks are dealt to the 8 XCDs round-robin.  Give each XCD runs of
    // kRun consecutive items (neighbouring tiles share that XCD's L2) while
    // the runs stay interleaved across XCDs (dense regions spread out).
    const uint32_t b = blockIdx.x, k = b >> 3;
    const uint32_t item = (k / kRun) * (8 * kRun) + (b & 7) * kRun + (k % kRun);
    const uint32_t ntiles = (uint32_t)(a.ntx * a.nty);
    if (item >= a.seg_off[ntiles]) return;
    const uint32_t tile = a.item_tile[item];
    if (a.tile_mask && !a.tile_mask[tile]) return;
    const uint32_t seg = item - (uint32_t)a.seg_off[tile];
    const uint32_t nseg = (uint32_t)(a.seg_off[tile + 1] - a.seg_off[tile]);
    const int tx = (int)(tile % (uint32_t)a.ntx), ty = (int)(tile / (uint32_t)a.ntx);
    const int tid = threadIdx.x;
    const int i = tx * T + (tid % T), j = ty * T + (tid / T);
    const int wave = tid >> 6;
    const int wx0 = tx * T, wx1 = tx * T + T - 1;
    const int wy0 = ty * T + wave * ROWS, wy1 = wy0 + ROWS - 1;
    const uint32_t seg_len = *a.seg_len;
    const uint32_t tend = a.tile_end[tile];
    const uint32_t start = a.tile_start[tile] + seg * seg_len;
    const uint32_t end = (tend - start) > seg_len ? start + seg_len : tend;
    __shared__ float s_vmin[kMaxSpecies], s_vmax[kMaxSpecies];
    if (tid < kMaxSpecies) species_range(a.sp, a.range_bits, tid, &s_vmin[tid], &s_vmax[tid]);
    __syncthreads();

    uint32_t n_member = 0, n_absorb = 0;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f;
    float K0 = 0.f, K1 = 0.f, K2 = 0.f;  // compensation terms
    float T0 = 1.f, T1 = 1.f, T2 = 1.f;

    for (uint32_t base = start; base < end; base += B) {
        // stage: gather records, expand colours once per record
        for (int r = tid; r < B; r += NT) {
            const uint32_t kk2 = base + r;
            if (kk2 < end) {
                const uint32_t idx = a.pair_val[kk2];
                const uint4 ra = a.rec[idx].a, rb = a.rec[idx].b;
                const int sp = (int)(ra.x >> 28);
                const float t = normalise_value(__uint_as_float(rb.z), s_vmin[sp], s_vmax[sp],
                                                a.sp.log_scale[sp]);
                const float rho0 = __uint_as_float(rb.w);
                const float pp = t * (float)(a.n_pal - 1);
                int kk = (int)floorf(pp);
                kk = kk > a.n_pal - 2 ? a.n_pal - 2 : kk;
                const float w1 = pp - (float)kk, w0 = 1.0f - w1;
                const float *c0 = a.palette + 3 * kk;
                const float cr = c0[0] * w0 + c0[3] * w1;
                const float cg = c0[1] * w0 + c0[4] * w1;
                const float cb = c0[2] * w0 + c0[5] * w1;
                const float eb = a.sp.brightness[sp] * rho0;
                const bool ord = a.sp.ordered[sp] != 0;
                const float ab = ord ? a.sp.absorption[sp] * rho0 : 0.0f;
                s_b0[r] = ra.x;
                s_b1[r] = (ra.y & 0x0FFFFFFFu) | ((ab == 0.0f) ? 0x80000000u : 0u);
                s_ur[r] = __uint_as_float(ra.z);
                s_vr[r] = __uint_as_float(ra.w);
                s_r2[r] = __uint_as_float(rb.x);
                s_qs[r] = __uint_as_float(rb.y);
                s_e[0][r] = eb * cr;
                s_e[1][r] = eb * cg;
                s_e[2][r] = eb * cb;
                s_a[0][r] = ab * cr;
                s_a[1][r] = ab * cg;
                s_a[2][r] = ab * cb;
            }
        }
        __syncthreads();
        const int nb = (int)((end - base) < (uint32_t)B ? (end - base) : (uint32_t)B);
        if (!LISTS) {
            for (int r = 0; r < nb; ++r) {
                // record fields are the same for every lane: decode and cull
                // the footprint box in scalar registers
                const uint32_t b0 = __builtin_amdgcn_readfirstlane(s_b0[r]);
                const uint32_t b1 = __builtin_amdgcn_readfirstlane(s_b1[r]);
                const int i0 = (int)(b0 & kBboxMask), i1 = (int)((b0 >> kBboxBits) & kBboxMask);
                const int j0 = (int)(b1 & kBboxMask), j1 = (int)((b1 >> kBboxBits) & kBboxMask);
                if (i1 < wx0 || i0 > wx1 || j1 < wy0 || j0 > wy1) continue;
                const float d2 = member_d2(i, i0, s_ur[r], j, j0, s_vr[r]);
                const bool in = (uint32_t)(i - i0) <= (uint32_t)(i1 - i0) &&
                                (uint32_t)(j - j0) <= (uint32_t)(j1 - j0) && d2 <= s_r2[r];
                if (!in) continue;
                ++n_member;
                const float w = __builtin_amdgcn_exp2f(-d2 * s_qs[r]);  // exp(-q^2)
                const float e0 = s_e[0][r] * w, e1 = s_e[1][r] * w, e2 = s_e[2][r] * w;
                if (!ORDERED || (b1 >> 31)) {
                    const float v0 = ORDERED ? T0 * e0 : e0;
                    const float v1 = ORDERED ? T1 * e1 : e1;
                    const float v2 = ORDERED ? T2 * e2 : e2;
                    if (KAHAN) {
                        kahan_add(C0, K0, v0);
                        kahan_add(C1, K1, v1);
                        kahan_add(C2, K2, v2);
                    } else {
                        C0 += v0;
                        C1 += v1;
                        C2 += v2;
                    }
                } else {
                    ++n_absorb;
                    const float x0 = s_a[0][r] * w, x1 = s_a[1][r] * w, x2 = s_a[2][r] * w;
                    float ex0, ex1, ex2, ph0, ph1, ph2;
                    if (fmaxf(x0, fmaxf(x1, x2)) < kSeriesMax) {
                        ex_phi_small(x0, ex0, ph0);
                        ex_phi_small(x1, ex1, ph1);
                        ex_phi_small(x2, ex2, ph2);
                    } else {
                        ex_phi(x0, ex0, ph0);
                        ex_phi(x1, ex1, ph1);
                        ex_phi(x2, ex2, ph2);
                    }
                    if (KAHAN) {
                        kahan_add(C0, K0, T0 * (e0 * ph0));
                        kahan_add(C1, K1, T1 * (e1 * ph1));
                        kahan_add(C2, K2, T2 * (e2 * ph2));
                    } else {
                        C0 += T0 * (e0 * ph0);
                        C1 += T1 * (e1 * ph1);
                        C2 += T2 * (e2 * ph2);
                    }
                    T0 *= ex0;
                    T1 *= ex1;
                    T2 *= ex2;
                }
            }
        } else {
        // phase 1: each lane lists, in order, the staged records whose
        // footprint holds its pixel (binary32 membership of the index recipe)
        int cnt = 0;
        for (int r = 0; r < nb; ++r) {
            // record fields are the same for every lane: decode and cull the
            // footprint box in scalar registers
            const uint32_t b0 = __builtin_amdgcn_readfirstlane(s_b0[r]);
            const uint32_t b1 = __builtin_amdgcn_readfirstlane(s_b1[r]);
            const int i0 = (int)(b0 & kBboxMask), i1 = (int)((b0 >> kBboxBits) & kBboxMask);
            const int j0 = (int)(b1 & kBboxMask), j1 = (int)((b1 >> kBboxBits) & kBboxMask);
            if (i1 < wx0 || i0 > wx1 || j1 < wy0 || j0 > wy1) continue;
            const float d2 = member_d2(i, i0, s_ur[r], j, j0, s_vr[r]);
            const bool in = (uint32_t)(i - i0) <= (uint32_t)(i1 - i0) &&
                            (uint32_t)(j - j0) <= (uint32_t)(j1 - j0) && d2 <= s_r2[r];
            if (in) {
                s_list[cnt * NT + tid] = (uint8_t)r;
                ++cnt;
            }
        }
        // phase 2: composite each lane's list front to back; lanes work on
        // different records at once, so every active lane does useful work.
        // Emission-only records take the same path: with A = 0 the series
        // gives phi = 1 and exp(-x) = 1 exactly.
        for (int m = 0; __ballot(m < cnt) != 0ull; ++m) {
            if (m < cnt) {
                const int r = s_list[m * NT + tid];
                const uint32_t b0 = s_b0[r], b1 = s_b1[r];
                const int i0 = (int)(b0 & kBboxMask), j0 = (int)(b1 & kBboxMask);
                const float d2 = member_d2(i, i0, s_ur[r], j, j0, s_vr[r]);
                const float w = __builtin_amdgcn_exp2f(-d2 * s_qs[r]);  // exp(-q^2)
                const float e0 = s_e[0][r] * w, e1 = s_e[1][r] * w, e2 = s_e[2][r] * w;
                ++n_member;
                if (!ORDERED) {
                    if (KAHAN) {
                        kahan_add(C0, K0, e0);
                        kahan_add(C1, K1, e1);
                        kahan_add(C2, K2, e2);
                    } else {
                        C0 += e0;
                        C1 += e1;
                        C2 += e2;
                    }
                } else {
                    n_absorb += (b1 >> 31) ^ 1u;
                    const float x0 = s_a[0][r] * w, x1 = s_a[1][r] * w, x2 = s_a[2][r] * w;
                    float ex0, ex1, ex2, ph0, ph1, ph2;
                    if (fmaxf(x0, fmaxf(x1, x2)) < kSeriesMax) {
                        ex_phi_small(x0, ex0, ph0);
                        ex_phi_small(x1, ex1, ph1);
                        ex_phi_small(x2, ex2, ph2);
                    } else {
                        ex_phi(x0, ex0, ph0);
                        ex_phi(x1, ex1, ph1);
                        ex_phi(x2, ex2, ph2);
                    }
                    if (KAHAN) {
                        kahan_add(C0, K0, T0 * (e0 * ph0));
                        kahan_add(C1, K1, T1 * (e1 * ph1));
                        kahan_add(C2, K2, T2 * (e2 * ph2));
                    } else {
                        C0 += T0 * (e0 * ph0);
                        C1 += T1 * (e1 * ph1);
                        C2 += T2 * (e2 * ph2);
                    }
                    T0 *= ex0;
                    T1 *= ex1;
                    T2 *= ex2;
                }
            }
        }
        }
        __syncthreads();
    }
    // per-tile count of composited (pixel, particle) contributions
    __shared__ uint32_t s_cnt[2][NT / 64];
    uint32_t wsum = n_member, asum = n_absorb;
    for (int o = 32; o > 0; o >>= 1) {
        wsum += __shfl_xor(wsum, o, 64);
        asum += __shfl_xor(asum, o, 64);
    }
    if ((tid & 63) == 0) {
        s_cnt[0][wave] = wsum;
        s_cnt[1][wave] = asum;
    }
    __syncthreads();
    if (tid == 0) {
        unsigned long long t = 0, ta = 0;
        for (int w = 0; w < NT / 64; ++w) {
            t += s_cnt[0][w];
            ta += s_cnt[1][w];
        }
        // statistics only; compositing itself uses no atomics
        if (t) atomicAdd(&a.member_count[2 * tile], t);
        if (ta) atomicAdd(&a.member_count[2 * tile + 1], ta);
    }
    if (nseg == 1) {
        write_pixel<ORDERED>(a, i, j, C0, C1, C2, T0, T1, T2);
    } else {
        float *slot = a.partial + (size_t)(a.part_off[tile] + seg) * 6 * NT;
        slot[0 * NT + tid] = C0;
        slot[1 * NT + tid] = C1;
        slot[2 * NT + tid] = C2;
        if (ORDERED) {
            slot[3 * NT + tid] = T0;
            slot[4 * NT + tid] = T1;
            slot[5 * NT + tid] = T2;
        }
    }
}

// Fold the partial (C, Tr) of a multi-segment tile front to back:
// C += Tr * C_s, Tr *= Tr_s (the associative "over"); a plain sum when
// nothing absorbs.
template <int T, bool ORDERED, bool KAHAN>
__global__ __launch_bounds__(T *T) void k_merge(SplatArgs a) {
    constexpr int NT = T * T;
    const uint32_t tile = blockIdx.x;
    const uint32_t nseg = (uint32_t)(a.seg_off[tile + 1] - a.seg_off[tile]);
    if (nseg <= 1 || (a.tile_mask && !a.tile_mask[tile])) return;
    const int tx = (int)(tile % (uint32_t)a.ntx), ty = (int)(tile / (uint32_t)a.ntx);
    const int tid = threadIdx.x;
    const int i = tx * T + (tid % T), j = ty * T + (tid / T);
    float C0 = 0.f, C1 = 0.f, C2 = 0.f, K0 = 0.f, K1 = 0.f, K2 = 0.f;
    float T0 = 1.f, T1 = 1.f, T2 = 1.f;
    const float *slot = a.partial + (size_t)a.part_off[tile] * 6 * NT;
    for (uint32_t s = 0; s < nseg; ++s, slot += 6 * NT) {
        const float c0 = slot[tid], c1 = slot[NT + tid], c2 = slot[2 * NT + tid];
        if (KAHAN) {
            kahan_add(C0, K0, ORDERED ? T0 * c0 : c0);
            kahan_add(C1, K1, ORDERED ? T1 * c1 : c1);
            kahan_add(C2, K2, ORDERED ? T2 * c2 : c2);
        } else {
            C0 += ORDERED ? T0 * c0 : c0;
            C1 += ORDERED ? T1 * c1 : c1;
            C2 += ORDERED ? T2 * c2 : c2;
        }
        if (ORDERED) {
            T0 *= slot[3 * NT + tid];
            T1 *= slot[4 * NT + tid];
            T2 *= slot[5 * NT + tid];
        }
    }
    write_pixel<ORDERED>(a, i, j, C0, C1, C2, T0, T1, T2);
}

__global__ void k_seg_count(const uint32_t *ts, const uint32_t *te, uint32_t n_tiles,
                            uint64_t npairs, const uint64_t *npairs_dev, uint32_t nt,
                            uint32_t seg_min, uint32_t *seg_len_out, uint32_t *nseg,
                            uint32_t *nmulti) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t np = npairs_dev ? (*npairs_dev < npairs ? *npairs_dev : npairs) : npairs;
    const uint32_t seg_len = seg_len_rule(np, nt, seg_min);
    if (t == 0) *seg_len_out = seg_len;
    if (t >= n_tiles) return;
    const uint32_t len = te[t] - ts[t];
    const uint32_t n = len == 0 ? 1u : (len + seg_len - 1) / seg_len;
    nseg[t] = n;
    nmulti[t] = n > 1 ? n : 0u;
}

__global__ void k_item_tiles(const uint64_t *seg_off, uint32_t n_tiles, uint32_t *item_tile) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    for (uint64_t k = seg_off[t]; k < seg_off[t + 1]; ++k) item_tile[k] = t;
}

template <int T, bool ORDERED, bool KAHAN, bool LISTS>
hipError_t launch_tok(const SplatArgs &a, uint32_t grid, hipStream_t s) {
    hipLaunchKernelGGL((k_splat<T, ORDERED, KAHAN, LISTS>), dim3(grid), dim3(T * T), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_merge<T, ORDERED, KAHAN>), dim3((uint32_t)(a.ntx * a.nty)), dim3(T * T),
                       0, s, a);
    return hipGetLastError();
}

template <int T, bool LISTS>
hipError_t launch_tl(const SplatArgs &a, uint32_t grid, hipStream_t s) {
    if (a.ordered)
        return a.compensated ? launch_tok<T, true, true, LISTS>(a, grid, s)
                             : launch_tok<T, true, false, LISTS>(a, grid, s);
    return a.compensated ? launch_tok<T, false, true, LISTS>(a, grid, s)
                         : launch_tok<T, false, false, LISTS>(a, grid, s);
}

template <int T>
hipError_t launch_t(const SplatArgs &a, uint32_t grid, hipStream_t s) {
    return a.lists ? launch_tl<T, true>(a, grid, s) : launch_tl<T, false>(a, grid, s);
}

}  // namespace

uint32_t splat_grid(uint32_t n_tiles, uint64_t npairs, uint32_t seg_len) {
    const uint64_t items = (uint64_t)n_tiles + (npairs + seg_len - 1) / seg_len;
    const uint64_t q = 8 * kRun;
    return (uint32_t)((items + q - 1) / q * q);
}

hipError_t launch_segments(const uint32_t *tile_start, const uint32_t *tile_end,
                           uint32_t n_tiles, uint64_t npairs, const uint64_t *npairs_dev,
                           uint32_t nt, uint32_t seg_min, uint32_t *seg_len, uint32_t *nseg,
                           uint32_t *nmulti, uint64_t *seg_off, uint64_t *part_off,
                           uint32_t *item_tile, void *scratch, hipStream_t s) {
    const uint32_t g = (n_tiles + 255) / 256;
    hipLaunchKernelGGL(k_seg_count, dim3(g), dim3(256), 0, s, tile_start, tile_end, n_tiles,
                       npairs, npairs_dev, nt, seg_min, seg_len, nseg, nmulti);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_scan_u32_u64(nseg, seg_off, n_tiles, scratch, s)) != hipSuccess) return e;
    if ((e = launch_scan_u32_u64(nmulti, part_off, n_tiles, scratch, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_item_tiles, dim3(g), dim3(256), 0, s, seg_off, n_tiles, item_tile);
    return hipGetLastError();
}

hipError_t launch_splat(const SplatArgs &a, uint32_t grid, hipStream_t s) {
    switch (a.tile) {
        case 8: return launch_t<8>(a, grid, s);
        case 16: return launch_t<16>(a, grid, s);
        case 32: return launch_t<32>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace splotch
