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

// exp(-x) and phi(x) = (1 - exp(-x))/x.  For x < 1/32 both come from
// their Taylor series (truncation below 3e-10), which keeps the product of
// thousands of transmittance factors free of the bias a transcendental's
// last-place error would add, and avoids the cancellation in 1 - exp(-x).
__device__ __forceinline__ void ex_phi(float x, float &ex, float &ph) {
    if (x < 0.03125f) {
        ex = 1.0f + x * (-1.0f + x * (0.5f + x * (-1.0f / 6.0f + x * (1.0f / 24.0f))));
        ph = 1.0f + x * (-0.5f + x * (1.0f / 6.0f + x * (-1.0f / 24.0f + x * (1.0f / 120.0f))));
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

template <int T, bool ORDERED, bool KAHAN>
__global__ __launch_bounds__(T *T) void k_splat(SplatArgs a) {
    constexpr int NT = T * T;
    constexpr int ROWS = 64 / T;  // pixel rows per wave
    __shared__ uint32_t s_b0[NT], s_b1[NT];
    __shared__ float s_ur[NT], s_vr[NT], s_r2[NT], s_qs[NT];
    __shared__ float s_e[3][NT];
    __shared__ float s_a[3][NT];

    const uint32_t ntiles = (uint32_t)(a.ntx * a.nty);
    const uint32_t per = gridDim.x / 8;
    // workgroups are dealt to the 8 XCDs round-robin; give each XCD a
    // contiguous band of tiles so neighbouring tiles share its L2
    const uint32_t tile = (blockIdx.x % 8) * per + blockIdx.x / 8;
    if (tile >= ntiles) return;
    const int tx = (int)(tile % (uint32_t)a.ntx), ty = (int)(tile / (uint32_t)a.ntx);
    const int tid = threadIdx.x;
    const int i = tx * T + (tid % T), j = ty * T + (tid / T);
    const int wave = tid >> 6;
    const int wx0 = tx * T, wx1 = tx * T + T - 1;
    const int wy0 = ty * T + wave * ROWS, wy1 = wy0 + ROWS - 1;
    const uint32_t start = a.tile_start[tile], end = a.tile_end[tile];

    uint32_t n_member = 0, n_absorb = 0;
    float C0 = 0.f, C1 = 0.f, C2 = 0.f;
    float K0 = 0.f, K1 = 0.f, K2 = 0.f;  // compensation terms
    float T0 = 1.f, T1 = 1.f, T2 = 1.f;

    for (uint32_t base = start; base < end; base += NT) {
        const uint32_t k = base + tid;
        if (k < end) {
            const uint32_t idx = a.pair_val[k];
            const uint4 ra = a.rec[idx].a, rb = a.rec[idx].b;
            const int sp = (int)(ra.x >> 28);
            const float t = __uint_as_float(rb.z);
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
            s_b0[tid] = ra.x;
            s_b1[tid] = (ra.y & 0x0FFFFFFFu) | ((ab == 0.0f) ? 0x80000000u : 0u);
            s_ur[tid] = __uint_as_float(ra.z);
            s_vr[tid] = __uint_as_float(ra.w);
            s_r2[tid] = __uint_as_float(rb.x);
            s_qs[tid] = __uint_as_float(rb.y);
            s_e[0][tid] = eb * cr;
            s_e[1][tid] = eb * cg;
            s_e[2][tid] = eb * cb;
            s_a[0][tid] = ab * cr;
            s_a[1][tid] = ab * cg;
            s_a[2][tid] = ab * cb;
        }
        __syncthreads();
        const int nb = (int)((end - base) < (uint32_t)NT ? (end - base) : (uint32_t)NT);
        for (int b = 0; b < nb; ++b) {
            const uint32_t b0 = s_b0[b], b1 = s_b1[b];
            const int i0 = (int)(b0 & kBboxMask), i1 = (int)((b0 >> kBboxBits) & kBboxMask);
            const int j0 = (int)(b1 & kBboxMask), j1 = (int)((b1 >> kBboxBits) & kBboxMask);
            if (i1 < wx0 || i0 > wx1 || j1 < wy0 || j0 > wy1) continue;  // wave-uniform
            const float d2 = member_d2(i, i0, s_ur[b], j, j0, s_vr[b]);
            const bool in = i >= i0 && i <= i1 && j >= j0 && j <= j1 && d2 <= s_r2[b];
            if (!in) continue;
            ++n_member;
            const float w = __builtin_amdgcn_exp2f(-d2 * s_qs[b]);  // exp(-q^2)
            const float e0 = s_e[0][b] * w, e1 = s_e[1][b] * w, e2 = s_e[2][b] * w;
            if (!ORDERED || (b1 >> 31)) {
                if (ORDERED) {
                    if (KAHAN) {
                        kahan_add(C0, K0, T0 * e0);
                        kahan_add(C1, K1, T1 * e1);
                        kahan_add(C2, K2, T2 * e2);
                    } else {
                        C0 += T0 * e0;
                        C1 += T1 * e1;
                        C2 += T2 * e2;
                    }
                } else {
                    if (KAHAN) {
                        kahan_add(C0, K0, e0);
                        kahan_add(C1, K1, e1);
                        kahan_add(C2, K2, e2);
                    } else {
                        C0 += e0;
                        C1 += e1;
                        C2 += e2;
                    }
                }
            } else {
                ++n_absorb;
                float ex, ph;
                ex_phi(s_a[0][b] * w, ex, ph);
                if (KAHAN) kahan_add(C0, K0, T0 * e0 * ph); else C0 += T0 * e0 * ph;
                T0 *= ex;
                ex_phi(s_a[1][b] * w, ex, ph);
                if (KAHAN) kahan_add(C1, K1, T1 * e1 * ph); else C1 += T1 * e1 * ph;
                T1 *= ex;
                ex_phi(s_a[2][b] * w, ex, ph);
                if (KAHAN) kahan_add(C2, K2, T2 * e2 * ph); else C2 += T2 * e2 * ph;
                T2 *= ex;
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
        a.member_count[2 * tile] += t;
        a.member_count[2 * tile + 1] += ta;
    }
    if (i < a.width && j < a.height) {
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
}

template <int T>
hipError_t launch_t(const SplatArgs &a, hipStream_t s) {
    const uint32_t ntiles = (uint32_t)(a.ntx * a.nty);
    const uint32_t grid = (ntiles + 7) / 8 * 8;
    if (a.ordered) {
        if (a.compensated)
            hipLaunchKernelGGL((k_splat<T, true, true>), dim3(grid), dim3(T * T), 0, s, a);
        else
            hipLaunchKernelGGL((k_splat<T, true, false>), dim3(grid), dim3(T * T), 0, s, a);
    } else {
        if (a.compensated)
            hipLaunchKernelGGL((k_splat<T, false, true>), dim3(grid), dim3(T * T), 0, s, a);
        else
            hipLaunchKernelGGL((k_splat<T, false, false>), dim3(grid), dim3(T * T), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_splat(const SplatArgs &a, hipStream_t s) {
    switch (a.tile) {
        case 8: return launch_t<8>(a, s);
        case 16: return launch_t<16>(a, s);
        case 32: return launch_t<32>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace splotch
