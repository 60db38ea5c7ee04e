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
    ph = __builtin_fmaf(x, __builtin_fmaf(x, __builtin_fmaf(x, -1.0f / 24.0f, 1.0f / 6.0f), -0.5f),
                        1.0f);
    ex = __builtin_fmaf(-x, ph, 1.0f);
}

__device__ __forceinline__ void ex_phi(float x, float &ex, float &ph) {
#pragma clang fp contract(off)
    if (x < kSeriesMax) {
        ex_phi_small(x, ex, ph);
    } else {
        ex = __builtin_amdgcn_exp2f(-x * 1.4426950408889634f);
        ph = (1.0f - ex) / x;
    }
}

// Compensated (Kahan) accumulation into (C, K) of a term y from which the
// running compensation K has already been subtracted.
__device__ __forceinline__ void kahan_step(float &C, float &K, float y) {
#pragma clang fp contract(off)
    const float t = C + y;
    K = (t - C) - y;
    C = t;
}

// Adds T v to C (T = 1 when unordered), fused, optionally compensated.
// Every splat strategy goes through here, so a pixel's value does not
// depend on which one ran.
template <bool ORDERED, bool KAHAN>
__device__ __forceinline__ void add_term(float &C, float &K, float T, float v) {
#pragma clang fp contract(off)
    if (KAHAN)
        kahan_step(C, K, ORDERED ? __builtin_fmaf(T, v, -K) : v - K);
    else
        C = ORDERED ? __builtin_fmaf(T, v, C) : C + v;
}

// Kinds of record (uniform per record): emission only (A = 0), E = A per
// channel, and any other absorber.
enum : int { kKindEmit = 0, kKindEqual = 1, kKindGeneral = 2 };

constexpr float kLog2e = 1.4426950408889634f;

// The column a member pixel's ray sees, per unit rho0, as 2^-q g: the
// Gaussian exp(-d^2/sigma_s^2) = 2^-q with q = d2 log2(e)/sigma_s^2, and
// g = erf(sqrt(f^2 - d^2/sigma_s^2)) when the density is cut to the f sigma
// ball (f^2 - d^2/sigma_s^2 = (r2 - d2)/sigma_s^2), else 1.
struct Col {
    float q, g;
};

template <bool K3D>
__device__ __forceinline__ Col column(float d2, float r2, float qs) {
#pragma clang fp contract(off)
    Col c;
    c.q = d2 * qs;
    c.g = 1.0f;
    if (K3D) {
        const float rem = fmaxf(r2 - d2, 0.0f) * (qs * 0.6931471805599453f);
        c.g = erff(sqrtf(rem));
    }
    return c;
}

// Per-pixel state: colour C with its compensation K; for ordered sets the
// optical depth L crossed so far per channel (the transmittance is
// exp(-L)) and, when the set has absorbers with E != A (GEN), the
// transmittance D those absorbers removed and whether an E = A absorber
// covered the pixel.  P: colour terms not yet added to C (see fold).
struct Px {
    float C0, C1, C2, K0, K1, K2, L0, L1, L2, D0, D1, D2, seen, P0, P1, P2;
};

__device__ __forceinline__ void px_init(Px &p) {
    p.C0 = p.C1 = p.C2 = 0.f;
    p.K0 = p.K1 = p.K2 = 0.f;
    p.P0 = p.P1 = p.P2 = 0.f;
    p.L0 = p.L1 = p.L2 = 0.f;
    p.D0 = p.D1 = p.D2 = 0.f;
    p.seen = 0.f;
}

// exp(-x) and phi(x) for three channels: the series almost always; the rare
// large optical depth redoes its channels (one branch, skipped when no lane
// needs it).
__device__ __forceinline__ void ex_phi3(float x0, float x1, float x2, float &ex0, float &ex1,
                                        float &ex2, float &ph0, float &ph1, float &ph2) {
    ex_phi_small(x0, ex0, ph0);
    ex_phi_small(x1, ex1, ph1);
    ex_phi_small(x2, ex2, ph2);
    if (fmaxf(x0, fmaxf(x1, x2)) >= kSeriesMax) {
        ex_phi(x0, ex0, ph0);
        ex_phi(x1, ex1, ph1);
        ex_phi(x2, ex2, ph2);
    }
}

// Transmittance exp(-L) of one channel times the column 2^-q g.
__device__ __forceinline__ float trans_col(float L, Col c) {
    return __builtin_amdgcn_exp2f(-__builtin_fmaf(L, kLog2e, c.q)) * c.g;
}

// One member contribution of a particle with emission e = E c rho0 and
// absorption a = A c rho0 per channel and column c at this pixel: the exact
// per-particle solution of Eq. (1), front to back, with T = exp(-L):
//   Emission only (A = 0): C += T e w.
//   E = A: I <- I e^{-x} + (1 - e^{-x}) with x = a w, so the particle adds
//     exactly the transmittance it removes, T (1 - e^{-x}).  Only the
//     optical depth is carried (L += x); the sum of those additions,
//     (1 - exp(-L)) less what other absorbers removed (D), is added once at
//     the end (finish).  Carrying L rather than a product of factors keeps
//     faint pixels exact to rounding: 1 - exp(-L) = -expm1(-L).
//   Other absorbers: C += T e w phi(x), D += T x phi(x), L += x.
// Additive (unordered) sets: C += e w.
// A colour term s t (s, t its two factors) is added to C compensated, or,
// with DEFER (compensated sums only), fused into the partial sum P, which
// fold() adds to C compensated: a two-level compensated sum that costs
// one fused multiply-add per term instead of five operations.
template <bool KAHAN, bool DEFER>
__device__ __forceinline__ void add_colour(float &C, float &K, float &P, float s, float t) {
#pragma clang fp contract(off)
    if (KAHAN && DEFER)
        P = __builtin_fmaf(s, t, P);
    else
        add_term<false, KAHAN>(C, K, 1.f, s * t);
}

// member: false for a lane that runs the arithmetic without being covered
// (its column is 2^-inf = 0, so every term is an exact zero); it then only
// keeps `seen` as it was.
template <bool ORDERED, bool KAHAN, bool GEN, bool DEFER = false>
__device__ __forceinline__ void composite(int kind, Col c, float e0, float e1, float e2, float a0,
                                          float a1, float a2, Px &p, bool member = true) {
#pragma clang fp contract(off)
    if (!ORDERED) {
        const float w = __builtin_amdgcn_exp2f(-c.q) * c.g;
        add_colour<KAHAN, DEFER>(p.C0, p.K0, p.P0, e0, w);
        add_colour<KAHAN, DEFER>(p.C1, p.K1, p.P1, e1, w);
        add_colour<KAHAN, DEFER>(p.C2, p.K2, p.P2, e2, w);
    } else if (kind == kKindEmit) {
        add_colour<KAHAN, DEFER>(p.C0, p.K0, p.P0, e0, trans_col(p.L0, c));
        add_colour<KAHAN, DEFER>(p.C1, p.K1, p.P1, e1, trans_col(p.L1, c));
        add_colour<KAHAN, DEFER>(p.C2, p.K2, p.P2, e2, trans_col(p.L2, c));
    } else if (kind == kKindEqual) {
        const float w = __builtin_amdgcn_exp2f(-c.q) * c.g;
        p.L0 = __builtin_fmaf(e0, w, p.L0);
        p.L1 = __builtin_fmaf(e1, w, p.L1);
        p.L2 = __builtin_fmaf(e2, w, p.L2);
        if (GEN) p.seen = member ? 1.f : p.seen;
    } else {
        const float w = __builtin_amdgcn_exp2f(-c.q) * c.g;
        const float x0 = a0 * w, x1 = a1 * w, x2 = a2 * w;
        float ex0, ex1, ex2, ph0, ph1, ph2;
        ex_phi3(x0, x1, x2, ex0, ex1, ex2, ph0, ph1, ph2);
        const float t0 = __builtin_amdgcn_exp2f(-p.L0 * kLog2e);
        const float t1 = __builtin_amdgcn_exp2f(-p.L1 * kLog2e);
        const float t2 = __builtin_amdgcn_exp2f(-p.L2 * kLog2e);
        add_colour<KAHAN, DEFER>(p.C0, p.K0, p.P0, t0, (e0 * w) * ph0);
        add_colour<KAHAN, DEFER>(p.C1, p.K1, p.P1, t1, (e1 * w) * ph1);
        add_colour<KAHAN, DEFER>(p.C2, p.K2, p.P2, t2, (e2 * w) * ph2);
        if (GEN) {
            p.D0 = __builtin_fmaf(t0, x0 * ph0, p.D0);
            p.D1 = __builtin_fmaf(t1, x1 * ph1, p.D1);
            p.D2 = __builtin_fmaf(t2, x2 * ph2, p.D2);
        }
        p.L0 += x0;
        p.L1 += x1;
        p.L2 += x2;
        (void)ex0;
        (void)ex1;
        (void)ex2;
    }
}

// Adds the partial sums P to C, compensated, and clears them.
template <bool KAHAN>
__device__ __forceinline__ void fold(Px &p) {
#pragma clang fp contract(off)
    if (!KAHAN) return;
    kahan_step(p.C0, p.K0, p.P0 - p.K0);
    kahan_step(p.C1, p.K1, p.P1 - p.K1);
    kahan_step(p.C2, p.K2, p.P2 - p.K2);
    p.P0 = p.P1 = p.P2 = 0.f;
}

// End of a pixel's list: adds the E = A absorbers' contribution,
// (1 - exp(-L)) - D (0 when none covered the pixel), to C once,
// compensated, and returns the transmittance exp(-L) per channel.
template <bool ORDERED, bool KAHAN, bool GEN>
__device__ __forceinline__ void finish(Px &p, float &T0, float &T1, float &T2) {
#pragma clang fp contract(off)
    T0 = T1 = T2 = 1.f;
    if (!ORDERED) return;
    float g0 = -expm1f(-p.L0), g1 = -expm1f(-p.L1), g2 = -expm1f(-p.L2);
    T0 = expf(-p.L0);
    T1 = expf(-p.L1);
    T2 = expf(-p.L2);
    if (GEN) {
        const bool s = p.seen != 0.f;
        g0 = s ? g0 - p.D0 : 0.f;
        g1 = s ? g1 - p.D1 : 0.f;
        g2 = s ? g2 - p.D2 : 0.f;
    }
    if (KAHAN) {
        p.C0 = p.C0 + (g0 != 0.f ? g0 - p.K0 : 0.f);
        p.C1 = p.C1 + (g1 != 0.f ? g1 - p.K1 : 0.f);
        p.C2 = p.C2 + (g2 != 0.f ? g2 - p.K2 : 0.f);
    } else {
        p.C0 += g0;
        p.C1 += g1;
        p.C2 += g2;
    }
}

constexpr uint32_t kRun = 2;  // consecutive items per XCD run

// Final pixel value: composite over the incoming image when accumulating.
template <bool ORDERED>
__device__ __forceinline__ void write_pixel(const SplatArgs &a, int i, int j, float C0, float C1,
                                            float C2, float T0, float T1, float T2) {
#pragma clang fp contract(off)
    if (i >= a.width || j >= a.height) return;
    const size_t plane = (size_t)a.width * a.height;
    const size_t o = (size_t)j * a.width + i;
    float *img = a.image;
    if (a.accumulate) {
        const float in0 = img[o], in1 = img[plane + o], in2 = img[2 * plane + o];
        if (ORDERED) {
            C0 = __builtin_fmaf(T0, in0, C0);
            C1 = __builtin_fmaf(T1, in1, C1);
            C2 = __builtin_fmaf(T2, in2, C2);
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

// Flags in the top bits of a staged record's packed row box.
constexpr uint32_t kEmitOnly = 0x80000000u;      // A = 0: emission only
constexpr uint32_t kEmitEqAbsorb = 0x40000000u;  // E = A per channel (same colour terms)
constexpr uint32_t kRowMask = 0x0FFFFFFFu;       // j0 | j1 << 14

// Kind of a staged record from its flags.
__device__ __forceinline__ int record_kind(uint32_t flags) {
    return (flags & kEmitOnly) ? kKindEmit : ((flags & kEmitEqAbsorb) ? kKindEqual : kKindGeneral);
}

// One record as the compositing loop needs it: packed box (flags above),
// membership fields, Gaussian
// exponent scale and the emission / absorption colours E c(t) rho0 and
// A c(t) rho0 (Section 3.2: value -> normalised t -> palette colour).
struct Expanded {
    uint32_t b0, b1;
    float ur, vr, r2, qs;
    float e[3], ab[3];
};

// Linear interpolation in a K-entry RGB table at t (K - 1), t in [0, 1].
__device__ __forceinline__ void palette_rgb(const float *pal, int K, float t, float &r, float &g,
                                            float &b) {
#pragma clang fp contract(off)
    const float pp = t * (float)(K - 1);
    int kk = (int)floorf(pp);
    kk = kk > K - 2 ? K - 2 : kk;
    const float w1 = pp - (float)kk, w0 = 1.0f - w1;
    const float *c0 = pal + 3 * kk;
    r = c0[0] * w0 + c0[3] * w1;
    g = c0[1] * w0 + c0[4] * w1;
    b = c0[2] * w0 + c0[5] * w1;
}

// Section 2, last paragraph: E = brightness c_E, A = absorption c_A with the
// colours from the look-up tables at the normalised scalar, or, for
// vector-coloured species, the three normalised components as r, g, b for
// both.  Under the source-function reading an ordered species emits A S.
// idx: the particle's index (vector components are read from the particle
// arrays; the record keeps only the first).
__device__ __forceinline__ Expanded expand_loaded(const SplatArgs &a, uint4 ra, uint4 rb,
                                                  uint32_t idx, const float *vmin,
                                                  const float *vmax) {
#pragma clang fp contract(off)
    const int sp = (int)(ra.x >> 28);
    const int ls = a.sp.log_scale[sp];
    const float rho0 = __uint_as_float(rb.w);
    const bool ord = a.sp.ordered[sp] != 0;
    float cr, cg, cb, ar, ag, abb;
    if (a.sp.any_vector && a.sp.vector[sp]) {
        cr = normalise_value(__uint_as_float(rb.z), vmin[sp], vmax[sp], ls);
        cg = normalise_value(a.value_g[idx], vmin[sp], vmax[sp], ls);
        cb = normalise_value(a.value_b[idx], vmin[sp], vmax[sp], ls);
        ar = cr;
        ag = cg;
        abb = cb;
    } else {
        const float t = normalise_value(__uint_as_float(rb.z), vmin[sp], vmax[sp], ls);
        palette_rgb(a.palette, a.n_pal, t, cr, cg, cb);
        if (a.pal_abs && ord) {
            palette_rgb(a.pal_abs, a.n_pal_abs, t, ar, ag, abb);
        } else {
            ar = cr;
            ag = cg;
            abb = cb;
        }
    }
    const float eb = a.sp.brightness[sp] * rho0;
    const float ab = ord ? a.sp.absorption[sp] * rho0 : 0.0f;
    Expanded x;
    x.b0 = ra.x;
    x.ur = __uint_as_float(ra.z);
    x.vr = __uint_as_float(ra.w);
    x.r2 = __uint_as_float(rb.x);
    x.qs = __uint_as_float(rb.y);
    x.e[0] = eb * cr;
    x.e[1] = eb * cg;
    x.e[2] = eb * cb;
    x.ab[0] = ab * ar;
    x.ab[1] = ab * ag;
    x.ab[2] = ab * abb;
    if (a.source && ord) {
        // E := A S per channel: rho0 (A c_A) (E c_E)
        const float a0 = a.sp.absorption[sp];
        x.e[0] *= a0 * ar;
        x.e[1] *= a0 * ag;
        x.e[2] *= a0 * abb;
    }
    // finite colours (an overflow saturates): the row walk multiplies them
    // by an exact zero on pixels a record does not cover
    for (int c = 0; c < 3; ++c) {
        x.e[c] = fminf(x.e[c], 3.40282347e38f);
        x.ab[c] = fminf(x.ab[c], 3.40282347e38f);
    }
    const bool same = x.e[0] == x.ab[0] && x.e[1] == x.ab[1] && x.e[2] == x.ab[2];
    x.b1 = (ra.y & 0x0FFFFFFFu) | ((ab == 0.0f) ? kEmitOnly : 0u) |
           ((ab != 0.0f && same) ? kEmitEqAbsorb : 0u);
    return x;
}

__device__ __forceinline__ Expanded expand_record(const SplatArgs &a, uint32_t idx,
                                                  const float *vmin, const float *vmax) {
    return expand_loaded(a, a.rec[idx].a, a.rec[idx].b, idx, vmin, vmax);
}

// Records staged per batch: B indices of at most 8 bits per lane list.
template <int T>
struct Batch {
    static constexpr int NT = T * T;
    static constexpr int B = (32768 / NT) < 128 ? (32768 / NT) : 128;
};

// Member lists (one lane per pixel, 64-pixel rows of waves): phase 1
// builds, per lane, the ordered list of its member records in LDS; phase 2
// walks the lists, so every active lane composites (full lane use, at the
// price of per-lane LDS gathers).
template <int T, bool ORDERED, bool KAHAN, bool GEN>
__global__ __launch_bounds__(T *T) void k_splat_lists(SplatArgs a) {
    constexpr int NT = T * T;
    constexpr int B = Batch<T>::B;
    constexpr int ROWS = 64 / T;  // pixel rows per wave
    __shared__ uint32_t s_b0[B], s_b1[B];
    __shared__ float s_ur[B], s_vr[B], s_r2[B], s_qs[B];
    __shared__ float s_e[3][B];
    __shared__ float s_a[3][B];
    // per-lane member lists: entry m of lane l at s_list[m * NT + l]
    __shared__ uint8_t s_list[B * NT];

    // Blocks are dealt to the 8 XCDs round-robin.  Give each XCD runs of
    // kRun consecutive items (neighbouring tiles share that XCD's L2) while
    // the runs stay interleaved across XCDs (dense regions spread out).
    const uint32_t b = blockIdx.x, k = b >> 3;
    const uint32_t item = (k / kRun) * (8 * kRun) + (b & 7) * kRun + (k % kRun);
    const uint32_t ntiles = (uint32_t)(a.ntx * a.nty);
    if (item >= a.seg_off[ntiles] || item >= a.max_items) return;
    if (a.skip && *a.skip) return;
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
    Px px;
    px_init(px);

    for (uint32_t base = start; base < end; base += B) {
        // stage: gather records, expand colours once per record
        for (int r = tid; r < B; r += NT) {
            const uint32_t kk2 = base + r;
            if (kk2 < end) {
                const Expanded x = expand_record(a, a.pair_val[kk2], s_vmin, s_vmax);
                s_b0[r] = x.b0;
                s_b1[r] = x.b1;
                s_ur[r] = x.ur;
                s_vr[r] = x.vr;
                s_r2[r] = x.r2;
                s_qs[r] = x.qs;
                s_e[0][r] = x.e[0];
                s_e[1][r] = x.e[1];
                s_e[2][r] = x.e[2];
                s_a[0][r] = x.ab[0];
                s_a[1][r] = x.ab[1];
                s_a[2][r] = x.ab[2];
            }
        }
        __syncthreads();
        const int nb = (int)((end - base) < (uint32_t)B ? (end - base) : (uint32_t)B);
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
        for (int m = 0; __ballot(m < cnt) != 0ull; ++m) {
            if (m < cnt) {
                const int r = s_list[m * NT + tid];
                const uint32_t b0 = s_b0[r], b1 = s_b1[r];
                const int i0 = (int)(b0 & kBboxMask), j0 = (int)(b1 & kBboxMask);
                const float d2 = member_d2(i, i0, s_ur[r], j, j0, s_vr[r]);
                const Col cw = a.kernel3d ? column<true>(d2, s_r2[r], s_qs[r])
                                          : column<false>(d2, s_r2[r], s_qs[r]);
                ++n_member;
                if (ORDERED) n_absorb += (b1 >> 31) ^ 1u;
                composite<ORDERED, KAHAN, GEN>(record_kind(b1), cw, s_e[0][r], s_e[1][r],
                                               s_e[2][r], s_a[0][r], s_a[1][r], s_a[2][r], px);
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
    float T0, T1, T2;
    finish<ORDERED, KAHAN, GEN>(px, T0, T1, T2);
    if (nseg == 1) {
        write_pixel<ORDERED>(a, i, j, px.C0, px.C1, px.C2, T0, T1, T2);
    } else if (a.part_off[tile] + seg < a.max_slots) {
        float *slot = a.partial + (size_t)(a.part_off[tile] + seg) * 6 * NT;
        slot[0 * NT + tid] = px.C0;
        slot[1 * NT + tid] = px.C1;
        slot[2 * NT + tid] = px.C2;
        if (ORDERED) {
            slot[3 * NT + tid] = T0;
            slot[4 * NT + tid] = T1;
            slot[5 * NT + tid] = T2;
        }
    }
}

// Row walk (one lane per pixel, state in registers).  Each wave owns an
// 8x8 block of the tile and streams the item's list on its own, with no
// barrier between waves (waves whose blocks see fewer records do not wait
// for the others).  Pair keys carry, above the tile index, the mask of the
// tile's blocks that the particle's box meets: the wave scans keys 64 at a
// time and queues, in list order, the particle indices of the pairs whose
// mask holds its block, so it gathers and expands only those.  Up to 64
// queued records at a time are staged in the wave's own LDS rows,
// 64 bytes per record, read back as four broadcast 16-byte rows:
//   {u - i0, v - j0, r^2, log2(e)/sigma^2}, {2 i0, 2 j0, 2 (i1 - i0) + 1,
//   2 (j1 - j0) + 1} as floats, {E c rho0, flags}, {A c rho0, 0}.
// Without block masks (one block per tile, or tile indices that need the
// bits) every pair is queued; the per-pixel box test below keeps the
// result the same.  Membership: with a = (2 i + 1) - 2 i0 = 2 (i - i0) + 1
// (exact), a in [1, 2 (i1 - i0) + 1] is the box test and
// fma(1/2, a, -(u - i0)) rounds (i - i0 + 1/2) - (u - i0) once, which is
// the binary32 offset of the index recipe bit for bit.
// One 8x8 block (sub) of one item: the body of the row walk, shared by the
// per-view launch and the persistent multi-view launch.
// Bits lo..hi of an 8-bit row or column mask (0 when the range misses
// 0..7).
__device__ __forceinline__ uint32_t span8(int lo, int hi) {
    lo = lo < 0 ? 0 : lo;
    hi = hi > 7 ? 7 : hi;
    return lo > hi ? 0u : (((2u << hi) - 1u) & ~((1u << lo) - 1u));
}

template <int T, bool ORDERED, bool KAHAN, bool COUNT, bool K3D, bool GEN>
__device__ __forceinline__ void rows_unit(const SplatArgs &a, uint32_t item, uint32_t sub) {
    constexpr int NT = T * T;
    constexpr int QW = T / 8;    // blocks per tile row
    constexpr uint32_t kB = 64;   // records staged per batch (one per lane)
    constexpr int kS = 1;         // 64-key chunks per scan
    constexpr uint32_t kQ = 128;  // queue ring: < kB left over + 64 kS scanned
    static_assert(kB <= 64, "one record per lane");
    static_assert(kB - 1 + 64 * kS <= kQ && (kQ & (kQ - 1)) == 0, "queue ring");
    __shared__ float4 s_r[4][kB];
    __shared__ uint32_t s_q[kQ];
    __shared__ float s_vmin[kMaxSpecies], s_vmax[kMaxSpecies];

    const uint32_t ntiles = (uint32_t)(a.ntx * a.nty);
    if (item >= a.seg_off[ntiles] || item >= a.max_items) return;
    if (a.skip && *a.skip) return;
    const uint32_t tile = a.item_tile[item];
    if (a.tile_mask && !a.tile_mask[tile]) return;
    const uint32_t seg = item - (uint32_t)a.seg_off[tile];
    const uint32_t nseg = (uint32_t)(a.seg_off[tile + 1] - a.seg_off[tile]);
    const int tx0 = (int)(tile % (uint32_t)a.ntx) * T, ty0 = (int)(tile / (uint32_t)a.ntx) * T;
    const int lane = threadIdx.x;
    const int bx = tx0 + (int)(sub % QW) * 8, by = ty0 + (int)(sub / QW) * 8;
    const int i = bx + (lane & 7), j = by + (lane >> 3);
    const float tfx = (float)(2 * i + 1), tfy = (float)(2 * j + 1);
    // this lane's column and row bits in a record's block box
    const uint32_t sel = (1u << (lane & 7)) | (1u << (8 + (lane >> 3)));
    const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint32_t seg_len = *a.seg_len;
    const uint32_t tend = a.tile_end[tile];
    const uint32_t start = a.tile_start[tile] + seg * seg_len;
    const uint32_t end = (tend - start) > seg_len ? start + seg_len : tend;
    if (lane < kMaxSpecies) species_range(a.sp, a.range_bits, lane, &s_vmin[lane], &s_vmax[lane]);
    __syncthreads();

    uint32_t n_member = 0, n_absorb = 0;  // this lane's contributions
    Px px;
    px_init(px);

    // Keys and values of the next 64 kS positions are loaded one scan ahead,
    // at positions clamped to the segment's last pair (always valid).
    const bool masked = a.qshift != 0;
    const uint32_t bit = masked ? (uint32_t)a.qshift + sub : 0u;
    const uint32_t last = end > start ? end - 1 : start;
    uint32_t kq[kS] = {}, vq[kS] = {};
    uint32_t pos = start;
    auto load_scan = [&](uint32_t p) {
#pragma unroll
        for (int c = 0; c < kS; ++c) {
            const uint32_t q = p + 64 * c + lane;
            const uint32_t qc = q < last ? q : last;
            if (masked) kq[c] = a.pair_key[qc];
            vq[c] = a.pair_val[qc];
        }
    };
    uint32_t head = 0, qn = 0;  // queue ring: entries [head, head + qn)
    auto fill = [&]() {
        while (qn < kB && pos < end) {
#pragma unroll
            for (int c = 0; c < kS; ++c) {
                const bool hit = pos + 64 * c + lane < end && (!masked || ((kq[c] >> bit) & 1u));
                const uint64_t m = __ballot(hit);
                if (hit) s_q[(head + qn + __popcll(m & below)) & (kQ - 1)] = vq[c];
                qn += (uint32_t)__popcll(m);
            }
            pos += 64 * kS;
            if (pos < end) load_scan(pos);
        }
    };
    if (end > start) load_scan(start);
    fill();
    // the records of the next batch are in flight while a batch composites
    uint4 ra = make_uint4(0u, 0u, 0u, 0u), rb = ra;
    uint32_t gidx = 0;
    auto gather = [&](uint32_t n) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (n > 0) {
            // lanes past the batch load its first record again: no lane
            // keeps an old value, so nothing waits on the loads until the
            // batch is expanded
            gidx = s_q[(head + ((uint32_t)lane < n ? (uint32_t)lane : 0u)) & (kQ - 1)];
            ra = a.rec[gidx].a;
            rb = a.rec[gidx].b;
        }
        head += n;
        qn -= n;
    };
    uint32_t ncur = qn < kB ? qn : kB;
    gather(ncur);
    while (ncur > 0) {
        uint32_t kflags = 0;
        if ((uint32_t)lane < ncur) {
            const Expanded x = expand_loaded(a, ra, rb, gidx, s_vmin, s_vmax);
            const int i0 = (int)(x.b0 & kBboxMask), i1 = (int)((x.b0 >> kBboxBits) & kBboxMask);
            const int j0 = (int)(x.b1 & kBboxMask), j1 = (int)((x.b1 >> kBboxBits) & kBboxMask);
            // the block's columns and rows inside the record's box
            const uint32_t box = span8(i0 - bx, i1 - bx) | (span8(j0 - by, j1 - by) << 8);
            s_r[0][lane] = make_float4(x.ur, x.vr, x.r2, x.qs);
            s_r[1][lane] = make_float4((float)(2 * i0), (float)(2 * j0), __uint_as_float(box), 0.0f);
            s_r[2][lane] = make_float4(x.e[0], x.e[1], x.e[2], 0.0f);
            s_r[3][lane] = make_float4(x.ab[0], x.ab[1], x.ab[2], 0.0f);
            kflags = x.b1;
        }
        // kinds of the staged records, one bit per record
        const uint64_t m_emit = __ballot((kflags & kEmitOnly) != 0);
        const uint64_t m_equal = __ballot((kflags & kEmitEqAbsorb) != 0);
        fill();
        const uint32_t nnext = qn < kB ? qn : kB;
        gather(nnext);
        // the wave reads back its own rows (a wave's LDS requests complete
        // in order)
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // each visit reads the next record's rows before working on its
        // own, so no visit waits on the LDS for its rows
        float4 fn = s_r[0][0], gn = s_r[1][0], en = s_r[2][0];
        auto visit = [&](uint32_t r) {
            const float4 f = fn, g = gn, e = en;
            const uint32_t rn = r + 1 < ncur ? r + 1 : r;
            fn = s_r[0][rn];
            gn = s_r[1][rn];
            en = s_r[2][rn];
            const float ax = tfx - g.x, ay = tfy - g.y;
            float d2;
            {
#pragma clang fp contract(off)
                const float dx = __builtin_fmaf(0.5f, ax, -f.x);
                const float dy = __builtin_fmaf(0.5f, ay, -f.y);
                d2 = dx * dx + dy * dy;
            }
            // box: this lane's column and row bits both set; no
            // short-circuit, so one mask and no branch around the tests
            const bool in = ((__float_as_uint(g.z) & sel) == sel) & (d2 <= f.z);
            // a wave with no member lane skips the rest
            if (__builtin_amdgcn_ballot_w64(in) == 0ull) return;
            // Every lane runs the member arithmetic: a vector instruction
            // with at most 8 active lanes issues at about a fifth of the
            // full rate, and no branch means no copies at a join.  A
            // non-member's column is 2^-inf = 0, so its terms are exact
            // zeros.
            Col cw = column<K3D>(d2, f.z, f.w);
            cw.q = in ? cw.q : __builtin_inff();
            const uint32_t one = in ? 1u : 0u;
            if (COUNT) n_member += one;
            if (!ORDERED || ((m_emit >> r) & 1ull)) {
                composite<ORDERED, KAHAN, GEN, true>(kKindEmit, cw, e.x, e.y, e.z, 0.f, 0.f, 0.f,
                                                     px, in);
            } else if (!GEN || ((m_equal >> r) & 1ull)) {
                // without absorbers of E != A every absorbing record is
                // E = A: only the optical depth is carried
                if (COUNT) n_absorb += one;
                composite<ORDERED, KAHAN, GEN, true>(kKindEqual, cw, e.x, e.y, e.z, 0.f, 0.f,
                                                     0.f, px, in);
            } else {
                if (COUNT) n_absorb += one;
                const float4 x = s_r[3][r];
                composite<ORDERED, KAHAN, GEN, true>(kKindGeneral, cw, e.x, e.y, e.z, x.x, x.y,
                                                     x.z, px, in);
            }
        };
        // four visits per trip: the register allocator rotates the running
        // sums and the prefetched rows between them instead of copying them
        // back each trip (one visit per trip measured 18% slower)
        uint32_t r = 0;
        for (; r + 3 < ncur; r += 4) {
            visit(r);
            visit(r + 1);
            visit(r + 2);
            visit(r + 3);
        }
        for (; r < ncur; ++r) visit(r);
        // the batch's colour terms into the compensated sum
        fold<KAHAN>(px);
        // before the next batch overwrites the rows
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        ncur = nnext;
    }
    if (COUNT) {
        for (int o = 32; o > 0; o >>= 1) {
            n_member += __shfl_xor(n_member, o, 64);
            n_absorb += __shfl_xor(n_absorb, o, 64);
        }
    }
    if (COUNT && lane == 0) {
        // statistics only; compositing itself uses no atomics
        if (n_member) atomicAdd(&a.member_count[2 * tile], (unsigned long long)n_member);
        if (n_absorb) atomicAdd(&a.member_count[2 * tile + 1], (unsigned long long)n_absorb);
    }
    float T0, T1, T2;
    finish<ORDERED, KAHAN, GEN>(px, T0, T1, T2);
    if (nseg == 1) {
        write_pixel<ORDERED>(a, i, j, px.C0, px.C1, px.C2, T0, T1, T2);
    } else if (a.part_off[tile] + seg < a.max_slots) {
        const int p = (j - ty0) * T + (i - tx0);
        float *slot = a.partial + (size_t)(a.part_off[tile] + seg) * 6 * NT;
        slot[0 * NT + p] = px.C0;
        slot[1 * NT + p] = px.C1;
        slot[2 * NT + p] = px.C2;
        if (ORDERED) {
            slot[3 * NT + p] = T0;
            slot[4 * NT + p] = T1;
            slot[5 * NT + p] = T2;
        }
    }
}

// Workgroups are dealt to the 8 XCDs round-robin.  In each XCD's own
// sequence k, the NW blocks of an item come one after another (they read
// the same keys and records, through that XCD's L2), items in runs of kRun.
template <int T>
__device__ __forceinline__ void unit_of(uint32_t b, uint32_t *item, uint32_t *sub,
                                        uint32_t *run_base) {
    constexpr uint32_t NW = (uint32_t)(T * T / 64);
    const uint32_t k = (b >> 3) / NW;
    *sub = (b >> 3) % NW;
    *run_base = (k / kRun) * (8 * kRun);
    *item = *run_base + (b & 7) * kRun + (k % kRun);
}

template <int T, bool ORDERED, bool KAHAN, bool COUNT, bool K3D, bool GEN>
__global__ __launch_bounds__(64) void k_splat_rows(SplatArgs a) {
    uint32_t item, sub, base;
    unit_of<T>(blockIdx.x, &item, &sub, &base);
    rows_unit<T, ORDERED, KAHAN, COUNT, K3D, GEN>(a, item, sub);
}

// Persistent row walk over the items of several views at once: the views'
// settings sit in device memory and their item counts are read on the
// device.  Units (item, 8x8 block) of the concatenated item sequence are
// handed out dynamically, one counter per XCD: a workgroup on XCD x (the
// hardware deals workgroups to the 8 XCDs round-robin) takes that XCD's
// next unit of the per-view launch's order, so units keep their XCD and
// a tile's blocks still share one L2, while long and short units balance
// as they would under the hardware's own dispatch.  Units past the last
// item end the loop: their run base only grows with the counter.
template <int T, bool ORDERED, bool KAHAN, bool COUNT, bool K3D, bool GEN>
__global__ __launch_bounds__(64) void k_splat_rows_multi(const SplatArgs *__restrict__ views,
                                                         int nv, uint32_t *next) {
    // The views' settings are read through the constant address space with
    // a wave-uniform index, so their fields come in by scalar loads into
    // scalar registers, as a kernel argument's do.  (Read as global memory,
    // the fields sit in vector registers, about 24 more, and 5 waves fit on
    // a SIMD instead of 7.)  Nothing writes them during the launch.
    typedef const __attribute__((address_space(4))) SplatArgs *ConstArgs;
    const ConstArgs cviews = (ConstArgs)views;
    uint32_t first[kMaxGroup + 1];
    first[0] = 0;
#pragma unroll
    for (int v = 0; v < kMaxGroup; ++v) {
        uint32_t n = 0;
        if (v < nv) {
            const uint64_t items = cviews[v].seg_off[(uint32_t)(cviews[v].ntx * cviews[v].nty)];
            n = (uint32_t)(items < cviews[v].max_items ? items : cviews[v].max_items);
        }
        first[v + 1] = first[v] + n;
    }
    uint32_t total = first[1];
#pragma unroll
    for (int v = 2; v <= kMaxGroup; ++v) total = v <= nv ? first[v] : total;
    const uint32_t x = blockIdx.x & 7u;
    for (;;) {
        uint32_t k = 0;
        if (threadIdx.x == 0) k = atomicAdd(&next[x], 1u);
        // lane 0's counter value into a scalar register
        k = __builtin_amdgcn_readfirstlane(k);
        uint32_t item, sub, base;
        unit_of<T>(8u * k + x, &item, &sub, &base);
        if (base >= total) break;
        if (item >= total) continue;
        int v = 0;
        uint32_t f = 0;
#pragma unroll
        for (int w = 1; w < kMaxGroup; ++w) {
            if (w < nv && item >= first[w]) {
                v = w;
                f = first[w];
            }
        }
        v = __builtin_amdgcn_readfirstlane(v);
        f = __builtin_amdgcn_readfirstlane(f);
        rows_unit<T, ORDERED, KAHAN, COUNT, K3D, GEN>(*(const SplatArgs *)(cviews + v), item - f,
                                                      sub);
        __syncthreads();  // the next unit reuses the staging rows
    }
}

// Box-mapped lanes (one wave per item).  Footprints are often a few pixels
// across, so with one lane per pixel most lanes idle on each record.  Here
// the tile's pixel state (C, Tr and the compensation terms) lives in LDS and
// for each record the 64 lanes are laid over the record's footprint box
// clipped to the tile, 8, 16 or 32 columns wide, in as many passes of
// 64 >> log2(width) rows as the box needs.  One wave walks the records in
// list order and LDS requests of a wave complete in order, so each pixel
// still sees its particles front to back; per pixel the arithmetic is that
// of the other strategies.
//
// State index of tile pixel (x, y): y T + (x ^ swz(y)).  The XOR spreads the
// rows a pass touches over distinct LDS banks (8- and 16-wide passes for
// T = 16, 8- and 32-wide ones for T = 32).
template <int T>
__device__ __forceinline__ int state_index(int x, int y) {
    const int sw = T == 16 ? ((y >> 1) & 1) << 3 : (T == 32 ? (y & 3) << 3 : 0);
    return y * T + (x ^ sw);
}

template <int T, bool ORDERED, bool KAHAN, bool GEN>
__global__ __launch_bounds__(64) void k_splat_box(SplatArgs a) {
    constexpr int NT = T * T;
    constexpr int NS = ORDERED ? NT : 1;
    constexpr int NK = KAHAN ? NT : 1;
    constexpr int NG = GEN ? NT : 1;
    __shared__ float s_C[3][NT];
    __shared__ float s_T[3][NS];  // optical depth L per channel
    __shared__ float s_K[3][NK];
    __shared__ float s_D[4][NG];  // D per channel, then the E = A flag
    // staged records, three 16-byte rows each: {b0, b1, ur, vr},
    // {r2, qs, e0, e1}, {e2, a0, a1, a2}
    __shared__ uint4 s_rec[3][64];
    __shared__ float s_vmin[kMaxSpecies], s_vmax[kMaxSpecies];

    const uint32_t b = blockIdx.x, k = b >> 3;
    const uint32_t item = (k / kRun) * (8 * kRun) + (b & 7) * kRun + (k % kRun);
    const uint32_t ntiles = (uint32_t)(a.ntx * a.nty);
    if (item >= a.seg_off[ntiles] || item >= a.max_items) return;
    if (a.skip && *a.skip) return;
    const uint32_t tile = a.item_tile[item];
    if (a.tile_mask && !a.tile_mask[tile]) return;
    const uint32_t seg = item - (uint32_t)a.seg_off[tile];
    const uint32_t nseg = (uint32_t)(a.seg_off[tile + 1] - a.seg_off[tile]);
    const int tx0 = (int)(tile % (uint32_t)a.ntx) * T, ty0 = (int)(tile / (uint32_t)a.ntx) * T;
    const int lane = threadIdx.x;
    const uint32_t seg_len = *a.seg_len;
    const uint32_t tend = a.tile_end[tile];
    const uint32_t start = a.tile_start[tile] + seg * seg_len;
    const uint32_t end = (tend - start) > seg_len ? start + seg_len : tend;
    if (lane < kMaxSpecies) species_range(a.sp, a.range_bits, lane, &s_vmin[lane], &s_vmax[lane]);
    for (int p = lane; p < NT; p += 64) {
        s_C[0][p] = 0.f;
        s_C[1][p] = 0.f;
        s_C[2][p] = 0.f;
        if (ORDERED) {
            s_T[0][p] = 0.f;  // optical depth
            s_T[1][p] = 0.f;
            s_T[2][p] = 0.f;
        }
        if (KAHAN) {
            s_K[0][p] = 0.f;
            s_K[1][p] = 0.f;
            s_K[2][p] = 0.f;
        }
        if (GEN) {
            s_D[0][p] = 0.f;
            s_D[1][p] = 0.f;
            s_D[2][p] = 0.f;
            s_D[3][p] = 0.f;
        }
    }
    __syncthreads();

    uint32_t n_member = 0, n_absorb = 0;
    for (uint32_t base = start; base < end; base += 64) {
        if (base + lane < end) {
            const Expanded x = expand_record(a, a.pair_val[base + lane], s_vmin, s_vmax);
            s_rec[0][lane] = make_uint4(x.b0, x.b1, __float_as_uint(x.ur), __float_as_uint(x.vr));
            s_rec[1][lane] = make_uint4(__float_as_uint(x.r2), __float_as_uint(x.qs),
                                        __float_as_uint(x.e[0]), __float_as_uint(x.e[1]));
            s_rec[2][lane] = make_uint4(__float_as_uint(x.e[2]), __float_as_uint(x.ab[0]),
                                        __float_as_uint(x.ab[1]), __float_as_uint(x.ab[2]));
        }
        __syncthreads();
        const int nb = (int)((end - base) < 64u ? (end - base) : 64u);
        for (int r = 0; r < nb; ++r) {
            const uint4 q0 = s_rec[0][r];
            const uint32_t b0 = __builtin_amdgcn_readfirstlane(q0.x);
            const uint32_t b1 = __builtin_amdgcn_readfirstlane(q0.y);
            const int i0 = (int)(b0 & kBboxMask), i1 = (int)((b0 >> kBboxBits) & kBboxMask);
            const int j0 = (int)(b1 & kBboxMask), j1 = (int)((b1 >> kBboxBits) & kBboxMask);
            const int ci0 = i0 > tx0 ? i0 : tx0, ci1 = i1 < tx0 + T - 1 ? i1 : tx0 + T - 1;
            const int cj0 = j0 > ty0 ? j0 : ty0, cj1 = j1 < ty0 + T - 1 ? j1 : ty0 + T - 1;
            if (ci0 > ci1 || cj0 > cj1) continue;
            const int bw = ci1 - ci0 + 1;
            const int gs = (T == 8 || bw <= 8) ? 3 : ((T == 16 || bw <= 16) ? 4 : 5);
            const int lx = lane & ((1 << gs) - 1), ly = lane >> gs;
            const int i = ci0 + lx;
            const bool col_in = lx < bw;
            const uint4 q1 = s_rec[1][r], q2 = s_rec[2][r];
            const float ur = __uint_as_float(q0.z), vr = __uint_as_float(q0.w);
            const float r2 = __uint_as_float(q1.x), qs = __uint_as_float(q1.y);
            const bool emit_only = (b1 >> 31) != 0;
            const int kind = record_kind(b1);
            for (int y0 = cj0; y0 <= cj1; y0 += 64 >> gs) {
                const int j = y0 + ly;
                if (!col_in || j > cj1) continue;
                const float d2 = member_d2(i, i0, ur, j, j0, vr);
                if (!(d2 <= r2)) continue;
                ++n_member;
                if (ORDERED && !emit_only) ++n_absorb;
                const Col cw = a.kernel3d ? column<true>(d2, r2, qs) : column<false>(d2, r2, qs);
                const int o = state_index<T>(i - tx0, j - ty0);
                Px px;
                px_init(px);
                px.C0 = s_C[0][o];
                px.C1 = s_C[1][o];
                px.C2 = s_C[2][o];
                if (ORDERED) {
                    px.L0 = s_T[0][o];
                    px.L1 = s_T[1][o];
                    px.L2 = s_T[2][o];
                }
                if (KAHAN) {
                    px.K0 = s_K[0][o];
                    px.K1 = s_K[1][o];
                    px.K2 = s_K[2][o];
                }
                if (GEN) {
                    px.D0 = s_D[0][o];
                    px.D1 = s_D[1][o];
                    px.D2 = s_D[2][o];
                    px.seen = s_D[3][o];
                }
                composite<ORDERED, KAHAN, GEN>(kind, cw, __uint_as_float(q1.z),
                                               __uint_as_float(q1.w), __uint_as_float(q2.x),
                                               __uint_as_float(q2.y), __uint_as_float(q2.z),
                                               __uint_as_float(q2.w), px);
                s_C[0][o] = px.C0;
                s_C[1][o] = px.C1;
                s_C[2][o] = px.C2;
                if (ORDERED) {
                    s_T[0][o] = px.L0;
                    s_T[1][o] = px.L1;
                    s_T[2][o] = px.L2;
                }
                if (KAHAN) {
                    s_K[0][o] = px.K0;
                    s_K[1][o] = px.K1;
                    s_K[2][o] = px.K2;
                }
                if (GEN) {
                    s_D[0][o] = px.D0;
                    s_D[1][o] = px.D1;
                    s_D[2][o] = px.D2;
                    s_D[3][o] = px.seen;
                }
            }
            // the next record may map another lane onto these pixels: keep
            // its LDS reads after these writes (a wave's LDS requests are
            // served in order, so no wait is needed)
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        __syncthreads();
    }
    uint32_t wsum = n_member, asum = n_absorb;
    for (int o = 32; o > 0; o >>= 1) {
        wsum += __shfl_xor(wsum, o, 64);
        asum += __shfl_xor(asum, o, 64);
    }
    if (lane == 0) {
        // statistics only; compositing itself uses no atomics
        if (wsum) atomicAdd(&a.member_count[2 * tile], (unsigned long long)wsum);
        if (asum) atomicAdd(&a.member_count[2 * tile + 1], (unsigned long long)asum);
    }
    for (int p = lane; p < NT; p += 64) {
        const int x = p % T, y = p / T;
        const int o = state_index<T>(x, y);
        Px px;
        px_init(px);
        px.C0 = s_C[0][o];
        px.C1 = s_C[1][o];
        px.C2 = s_C[2][o];
        if (ORDERED) {
            px.L0 = s_T[0][o];
            px.L1 = s_T[1][o];
            px.L2 = s_T[2][o];
        }
        if (KAHAN) {
            px.K0 = s_K[0][o];
            px.K1 = s_K[1][o];
            px.K2 = s_K[2][o];
        }
        if (GEN) {
            px.D0 = s_D[0][o];
            px.D1 = s_D[1][o];
            px.D2 = s_D[2][o];
            px.seen = s_D[3][o];
        }
        float T0, T1, T2;
        finish<ORDERED, KAHAN, GEN>(px, T0, T1, T2);
        const float C0 = px.C0, C1 = px.C1, C2 = px.C2;
        if (nseg == 1) {
            write_pixel<ORDERED>(a, tx0 + x, ty0 + y, C0, C1, C2, T0, T1, T2);
        } else if (a.part_off[tile] + seg < a.max_slots) {
            float *slot = a.partial + (size_t)(a.part_off[tile] + seg) * 6 * NT;
            slot[0 * NT + p] = C0;
            slot[1 * NT + p] = C1;
            slot[2 * NT + p] = C2;
            if (ORDERED) {
                slot[3 * NT + p] = T0;
                slot[4 * NT + p] = T1;
                slot[5 * NT + p] = T2;
            }
        }
    }
}

// Fold the partial (C, Tr) of a multi-segment tile front to back:
// C += Tr * C_s, Tr *= Tr_s (the associative "over"); a plain sum when
// nothing absorbs.
template <int T, bool ORDERED, bool KAHAN>
__global__ __launch_bounds__(T *T < 1024 ? T *T : 1024) void k_merge(SplatArgs a) {
    constexpr int NT = T * T;
    const uint32_t tile = blockIdx.x;
    const uint32_t nseg = (uint32_t)(a.seg_off[tile + 1] - a.seg_off[tile]);
    if (nseg <= 1 || (a.tile_mask && !a.tile_mask[tile])) return;
    if (a.skip && *a.skip) return;
    if (a.part_off[tile] + nseg > a.max_slots) return;  // never: the slot bound holds
    const int tx = (int)(tile % (uint32_t)a.ntx), ty = (int)(tile / (uint32_t)a.ntx);
    for (int p = threadIdx.x; p < NT; p += blockDim.x) {
        const int i = tx * T + (p % T), j = ty * T + (p / T);
        float C0 = 0.f, C1 = 0.f, C2 = 0.f, K0 = 0.f, K1 = 0.f, K2 = 0.f;
        float T0 = 1.f, T1 = 1.f, T2 = 1.f;
        const float *slot = a.partial + (size_t)a.part_off[tile] * 6 * NT;
        for (uint32_t s = 0; s < nseg; ++s, slot += 6 * NT) {
            const float c0 = slot[p], c1 = slot[NT + p], c2 = slot[2 * NT + p];
            add_term<ORDERED, KAHAN>(C0, K0, T0, c0);
            add_term<ORDERED, KAHAN>(C1, K1, T1, c1);
            add_term<ORDERED, KAHAN>(C2, K2, T2, c2);
            if (ORDERED) {
                T0 *= slot[3 * NT + p];
                T1 *= slot[4 * NT + p];
                T2 *= slot[5 * NT + p];
            }
        }
        write_pixel<ORDERED>(a, i, j, C0, C1, C2, T0, T1, T2);
    }
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

__global__ void k_item_tiles(const uint64_t *seg_off, uint32_t n_tiles, uint32_t *item_tile,
                             uint64_t max_items) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_tiles) return;
    const uint64_t e = seg_off[t + 1] < max_items ? seg_off[t + 1] : max_items;
    for (uint64_t k = seg_off[t]; k < e; ++k) item_tile[k] = t;
}

template <int T, bool ORDERED, bool KAHAN, bool GEN>
hipError_t launch_tok(const SplatArgs &a, uint32_t grid, hipStream_t s) {
    switch (a.variant) {
        case kSplatRows: {
            // one single-wave workgroup per 8x8 block of every item
            const dim3 g(grid * (T * T / 64)), b(64);
            if (a.kernel3d) {
                if (a.count)
                    hipLaunchKernelGGL((k_splat_rows<T, ORDERED, KAHAN, true, true, GEN>), g, b,
                                       0, s, a);
                else
                    hipLaunchKernelGGL((k_splat_rows<T, ORDERED, KAHAN, false, true, GEN>), g, b,
                                       0, s, a);
            } else {
                if (a.count)
                    hipLaunchKernelGGL((k_splat_rows<T, ORDERED, KAHAN, true, false, GEN>), g, b,
                                       0, s, a);
                else
                    hipLaunchKernelGGL((k_splat_rows<T, ORDERED, KAHAN, false, false, GEN>), g,
                                       b, 0, s, a);
            }
            break;
        }
        default:
            // member lists and box-mapped lanes hold a whole tile in one
            // workgroup: up to 32 px tiles
            if constexpr (T <= 32) {
                if (a.variant == kSplatLists)
                    hipLaunchKernelGGL((k_splat_lists<T, ORDERED, KAHAN, GEN>), dim3(grid),
                                       dim3(T * T), 0, s, a);
                else
                    hipLaunchKernelGGL((k_splat_box<T, ORDERED, KAHAN, GEN>), dim3(grid), dim3(64),
                                       0, s, a);
            } else {
                return hipErrorInvalidValue;
            }
            break;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_merge<T, ORDERED, KAHAN>), dim3((uint32_t)(a.ntx * a.nty)),
                       dim3(T * T < 1024 ? T * T : 1024), 0, s, a);
    return hipGetLastError();
}

template <int T>
hipError_t launch_t(const SplatArgs &a, uint32_t grid, hipStream_t s) {
    // absorbers with E != A exist only in ordered sets
    if (a.ordered) {
        if (a.general)
            return a.compensated ? launch_tok<T, true, true, true>(a, grid, s)
                                 : launch_tok<T, true, false, true>(a, grid, s);
        return a.compensated ? launch_tok<T, true, true, false>(a, grid, s)
                             : launch_tok<T, true, false, false>(a, grid, s);
    }
    return a.compensated ? launch_tok<T, false, true, false>(a, grid, s)
                         : launch_tok<T, false, false, false>(a, grid, s);
}

__global__ void k_store_args(SplatArgs a, SplatArgs *dst) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst = a;
}

template <int T, bool ORDERED, bool KAHAN, bool GEN>
hipError_t launch_multi_tok(const SplatArgs *views, int nv, const SplatArgs &a, uint32_t *next,
                            hipStream_t s) {
    // a persistent grid: 8 single-wave workgroups per SIMD, a multiple of 8
    const dim3 g(256 * 4 * 8), b(64);
    hipError_t e = launch_fill_u32(next, 0u, kUnitCounters, s);
    if (e != hipSuccess) return e;
    if (a.kernel3d) {
        if (a.count)
            hipLaunchKernelGGL((k_splat_rows_multi<T, ORDERED, KAHAN, true, true, GEN>), g, b, 0, s,
                               views, nv, next);
        else
            hipLaunchKernelGGL((k_splat_rows_multi<T, ORDERED, KAHAN, false, true, GEN>), g, b, 0,
                               s, views, nv, next);
    } else {
        if (a.count)
            hipLaunchKernelGGL((k_splat_rows_multi<T, ORDERED, KAHAN, true, false, GEN>), g, b, 0,
                               s, views, nv, next);
        else
            hipLaunchKernelGGL((k_splat_rows_multi<T, ORDERED, KAHAN, false, false, GEN>), g, b, 0,
                               s, views, nv, next);
    }
    return hipGetLastError();
}

template <int T>
hipError_t launch_multi_t(const SplatArgs *views, int nv, const SplatArgs &a, uint32_t *next,
                          hipStream_t s) {
    if (a.ordered) {
        if (a.general)
            return a.compensated ? launch_multi_tok<T, true, true, true>(views, nv, a, next, s)
                                 : launch_multi_tok<T, true, false, true>(views, nv, a, next, s);
        return a.compensated ? launch_multi_tok<T, true, true, false>(views, nv, a, next, s)
                             : launch_multi_tok<T, true, false, false>(views, nv, a, next, s);
    }
    return a.compensated ? launch_multi_tok<T, false, true, false>(views, nv, a, next, s)
                         : launch_multi_tok<T, false, false, false>(views, nv, a, next, s);
}

template <int T>
hipError_t launch_merge_t(const SplatArgs &a, hipStream_t s) {
    const dim3 g((uint32_t)(a.ntx * a.nty)), b(T * T < 1024 ? T * T : 1024);
    if (a.ordered) {
        if (a.compensated)
            hipLaunchKernelGGL((k_merge<T, true, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_merge<T, true, false>), g, b, 0, s, a);
    } else {
        if (a.compensated)
            hipLaunchKernelGGL((k_merge<T, false, true>), g, b, 0, s, a);
        else
            hipLaunchKernelGGL((k_merge<T, false, false>), g, b, 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t store_splat_args(const SplatArgs &a, SplatArgs *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_store_args, dim3(1), dim3(64), 0, s, a, dst);
    return hipGetLastError();
}

hipError_t launch_splat_multi(const SplatArgs *views, int nv, const SplatArgs &a,
                              uint32_t *next, hipStream_t s) {
    if (nv < 1 || nv > kMaxGroup || a.variant != kSplatRows) return hipErrorInvalidValue;
    switch (a.tile) {
        case 8: return launch_multi_t<8>(views, nv, a, next, s);
        case 16: return launch_multi_t<16>(views, nv, a, next, s);
        case 32: return launch_multi_t<32>(views, nv, a, next, s);
        case 64: return launch_multi_t<64>(views, nv, a, next, s);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_merge(const SplatArgs &a, hipStream_t s) {
    switch (a.tile) {
        case 8: return launch_merge_t<8>(a, s);
        case 16: return launch_merge_t<16>(a, s);
        case 32: return launch_merge_t<32>(a, s);
        case 64: return launch_merge_t<64>(a, s);
        default: return hipErrorInvalidValue;
    }
}

uint32_t splat_grid(uint32_t n_tiles, uint64_t npairs, uint32_t seg_len) {
    const uint64_t items = (uint64_t)n_tiles + (npairs + seg_len - 1) / seg_len;
    const uint64_t q = 8 * kRun;
    return (uint32_t)((items + q - 1) / q * q);
}

hipError_t launch_segments(const uint32_t *tile_start, const uint32_t *tile_end,
                           uint32_t n_tiles, uint64_t npairs, const uint64_t *npairs_dev,
                           uint32_t nt, uint32_t seg_min, uint32_t *seg_len, uint32_t *nseg,
                           uint32_t *nmulti, uint64_t *seg_off, uint64_t *part_off,
                           uint32_t *item_tile, uint64_t max_items, void *scratch,
                           hipStream_t s) {
    const uint32_t g = (n_tiles + 255) / 256;
    hipLaunchKernelGGL(k_seg_count, dim3(g), dim3(256), 0, s, tile_start, tile_end, n_tiles,
                       npairs, npairs_dev, nt, seg_min, seg_len, nseg, nmulti);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = launch_scan_u32_u64(nseg, seg_off, n_tiles, scratch, s)) != hipSuccess) return e;
    if ((e = launch_scan_u32_u64(nmulti, part_off, n_tiles, scratch, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_item_tiles, dim3(g), dim3(256), 0, s, seg_off, n_tiles, item_tile,
                       max_items);
    return hipGetLastError();
}

hipError_t launch_splat(const SplatArgs &a, uint32_t grid, hipStream_t s) {
    switch (a.tile) {
        case 8: return launch_t<8>(a, grid, s);
        case 16: return launch_t<16>(a, grid, s);
        case 32: return launch_t<32>(a, grid, s);
        case 64: return launch_t<64>(a, grid, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace splotch
