// Per-particle stage of the render (Section 3.2: normalise, transform to
// screen coordinates, find the affected screen area): one coalesced pass
// over the structure-of-arrays particle set that writes a 32-byte record,
// the number of screen tiles the footprint box touches and the depth key.
//
// The integer decisions follow a fixed recipe of IEEE operations so that
// any conforming implementation reproduces them bit for bit:
//   binary64, no contraction:
//     d = p - eye;  xc = (d0 r0 + d1 r1) + d2 r2  (same for yc with up, zc with fwd)
//     cull unless z_near < zc <= z_far
//     s = F / zc (perspective) or px_per_unit (orthographic)
//     u = xc s + W/2,  v = yc s + H/2,  sigma_s = (h * sigma_over_h) * s,  r = f sigma_s
//     i0 = max(ceil((u - r) - 1/2), 0),  i1 = min(floor((u + r) - 1/2), W-1)  (same for j)
//     off-screen unless i0 <= i1 and j0 <= j1
//   binary32 rounding: u - i0, v - j0, r^2 (membership fields), zc (depth key).
// Colour normalisation and the kernel scale are continuous values computed
// in binary32 and are not part of the recipe.
#include <algorithm>

#include "internal.h"

#include <float.h>

namespace splotch {

namespace {

constexpr int kThreads = 256;

__device__ __forceinline__ uint32_t order_bits(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ float from_order_bits(uint32_t k) {
    uint32_t b = (k & 0x80000000u) ? (k & 0x7FFFFFFFu) : ~k;
    return __uint_as_float(b);
}

__device__ __forceinline__ bool finite_f(float v) {
    return (__float_as_uint(v) & 0x7F800000u) != 0x7F800000u;
}

struct Proj {
    int status;
    int i0, i1, j0, j1;
    float ur, vr, r2;
    double zc, sig;
};

__device__ Proj project_spec(const CamDev &c, float x, float y, float z, float h, double soh,
                             double f) {
#pragma clang fp contract(off)
    Proj p;
    p.i0 = p.i1 = p.j0 = p.j1 = 0;
    p.ur = p.vr = p.r2 = 0.0f;
    p.sig = 0.0;
    double d0 = (double)x - c.eye[0];
    double d1 = (double)y - c.eye[1];
    double d2 = (double)z - c.eye[2];
    double xc = (d0 * c.right[0] + d1 * c.right[1]) + d2 * c.right[2];
    double yc = (d0 * c.up[0] + d1 * c.up[1]) + d2 * c.up[2];
    double zc = (d0 * c.fwd[0] + d1 * c.fwd[1]) + d2 * c.fwd[2];
    p.zc = zc;
    if (!(zc > c.znear && zc <= c.zfar)) {
        p.status = kDepthCulled;
        return p;
    }
    double s = c.persp ? c.focal / zc : c.ppu;
    double u = xc * s + c.half_w;
    double v = yc * s + c.half_h;
    double sig = ((double)h * soh) * s;
    double r = f * sig;
    p.sig = sig;
    double a = (u - r) - 0.5, b = (u + r) - 0.5;
    double cc = (v - r) - 0.5, dd = (v + r) - 0.5;
    if (!(a <= b) || !(cc <= dd)) {
        p.status = kOffscreen;
        return p;
    }
    double i0 = ceil(a), i1 = floor(b), j0 = ceil(cc), j1 = floor(dd);
    if (i0 < 0.0) i0 = 0.0;
    if (i1 > c.wmax) i1 = c.wmax;
    if (j0 < 0.0) j0 = 0.0;
    if (j1 > c.hmax) j1 = c.hmax;
    if (!(i0 <= i1) || !(j0 <= j1)) {
        p.status = kOffscreen;
        return p;
    }
    p.i0 = (int)i0;
    p.i1 = (int)i1;
    p.j0 = (int)j0;
    p.j1 = (int)j1;
    p.ur = (float)(u - i0);
    p.vr = (float)(v - j0);
    p.r2 = (float)(r * r);
    p.status = kVisible;
    return p;
}

// Along one axis, the squared offset the splat's row walk computes between
// the footprint's centre c (relative to the box origin o) and the nearest
// pixel centre of lo..hi, or 0 when that range holds the pixel pc at or
// left of c or the next one.  dx = fl((p - o + 0.5) - c) grows with p, so a
// range on one side of c is nearest at its edge on c's side (pc comes from
// floor(c - 0.5), whose rounding can only put it one pixel right).
__device__ __forceinline__ float axis_gap2(int lo, int hi, int o, int pc, float c) {
#pragma clang fp contract(off)
    if (lo <= pc + 1 && pc <= hi) return 0.0f;
    const int p = hi < pc ? hi : lo;
    const float g = __builtin_fmaf(0.5f, (float)(2 * (p - o) + 1), -c);
    return g * g;
}

// The corner bits of a record: which of the box's four corner 8x8 blocks
// (when it spans two block columns and rows or more) lie off the centre's
// block row and column with even their nearest pixel outside the radius by
// the row walk's own rounded distance (dx dx + dy dy, each step rounded).
// That distance is no larger there than at the block's other pixels, so
// the row walk would find no member in such a block.
__device__ __forceinline__ uint32_t corner_bits(const Proj &p) {
#pragma clang fp contract(off)
    const int bc0 = p.i0 >> 3, bc1 = p.i1 >> 3, br0 = p.j0 >> 3, br1 = p.j1 >> 3;
    if (bc1 == bc0 || br1 == br0) return 0u;
    const int pcx = p.i0 + (int)floorf(p.ur - 0.5f), pcy = p.j0 + (int)floorf(p.vr - 0.5f);
    const float gx[2] = {axis_gap2(p.i0, min(p.i1, 8 * bc0 + 7), p.i0, pcx, p.ur),
                         axis_gap2(max(p.i0, 8 * bc1), p.i1, p.i0, pcx, p.ur)};
    const float gy[2] = {axis_gap2(p.j0, min(p.j1, 8 * br0 + 7), p.j0, pcy, p.vr),
                         axis_gap2(max(p.j0, 8 * br1), p.j1, p.j0, pcy, p.vr)};
    uint32_t bits = 0;
#pragma unroll
    for (int yh = 0; yh < 2; ++yh)
#pragma unroll
        for (int xh = 0; xh < 2; ++xh)
            if (gx[xh] != 0.0f && gy[yh] != 0.0f && gx[xh] + gy[yh] > p.r2)
                bits |= 1u << (xh + 2 * yh);
    return bits;
}

__device__ __forceinline__ bool particle_valid(float x, float y, float z, float h, float v,
                                               float r0, int sp, int ns) {
    return finite_f(x) && finite_f(y) && finite_f(z) && finite_f(h) && finite_f(v) &&
           h > 0.0f && sp < ns && finite_f(r0) && r0 >= 0.0f;
}

__device__ __forceinline__ unsigned wave_sum(unsigned v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

__global__ void k_fill_f32(float *p, float v, size_t n) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += stride) p[k] = v;
}

// Min slots start at all-ones, max slots at zero.
__global__ void k_init_range(uint32_t *range_bits) {
    int t = threadIdx.x;
    if (t < kRangeSlots) range_bits[t] = (t & 1) ? 0u : 0xFFFFFFFFu;
}

// The projection also finds the exact per-species min/max of valid values
// for auto ranges (order-free: min and max of binary32 values through their
// monotone unsigned images); the colour is normalised later, when the splat
// stages each record.
__global__ __launch_bounds__(kThreads) void k_project(ProjectArgs a) {
    __shared__ unsigned s_cnt[kCntN];
    // per species value range, then the depth-key range of visible particles
    __shared__ uint32_t s_lo[kMaxSpecies + 1], s_hi[kMaxSpecies + 1];
    if (threadIdx.x < kCntN) s_cnt[threadIdx.x] = 0;
    if (threadIdx.x <= kMaxSpecies) {
        s_lo[threadIdx.x] = 0xFFFFFFFFu;
        s_hi[threadIdx.x] = 0u;
    }
    __syncthreads();
    uint32_t lo[kMaxSpecies], hi[kMaxSpecies];
#pragma unroll
    for (int q = 0; q < kMaxSpecies; ++q) {
        lo[q] = 0xFFFFFFFFu;
        hi[q] = 0u;
    }
    uint32_t klo = 0xFFFFFFFFu, khi = 0u;
    unsigned my[kCntN] = {0, 0, 0, 0};
    const int T = a.tile;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x; k < (size_t)a.n; k += stride) {
        float x = a.x[k], y = a.y[k], z = a.z[k], h = a.h[k], v = a.value[k];
        int sp = a.species ? (int)a.species[k] : 0;
        float r0 = a.rho0 ? a.rho0[k] : 1.0f;
        Proj p;
        bool valid = particle_valid(x, y, z, h, v, r0, sp, a.sp.n);
        // vector-coloured species: all three components must be finite, and
        // an automatic range spans all three
        const bool vec = a.sp.any_vector && valid && a.sp.vector[sp];
        float vg = 0.0f, vb = 0.0f;
        if (vec) {
            vg = a.value_g[k];
            vb = a.value_b[k];
            valid = finite_f(vg) && finite_f(vb);
        }
        if (valid && a.sp.auto_range[sp]) {
            const int ls = a.sp.log_scale[sp];
            uint32_t olo = 0xFFFFFFFFu, ohi = 0u;
            if (!ls || v > 0.0f) olo = ohi = order_bits(v);
            if (vec) {
                if (!ls || vg > 0.0f) {
                    olo = min(olo, order_bits(vg));
                    ohi = max(ohi, order_bits(vg));
                }
                if (!ls || vb > 0.0f) {
                    olo = min(olo, order_bits(vb));
                    ohi = max(ohi, order_bits(vb));
                }
            }
#pragma unroll
            for (int q = 0; q < kMaxSpecies; ++q)
                if (q == sp) {
                    lo[q] = min(lo[q], olo);
                    hi[q] = max(hi[q], ohi);
                }
        }
        if (!valid) {
            p.status = kInvalid;
            p.i0 = p.i1 = p.j0 = p.j1 = 0;
            p.ur = p.vr = p.r2 = 0.0f;
            p.zc = 0.0;
            p.sig = 0.0;
        } else {
            p = project_spec(a.cam, x, y, z, h, a.soh, a.f);
        }
        uint32_t cnt = 0, key = kEmptyKey;
        if (p.status == kVisible) {
            double qs = 1.4426950408889634 / (p.sig * p.sig);
            float qsf = (float)fmin(qs, (double)FLT_MAX);
            Rec r;
            r.a.x = (uint32_t)p.i0 | ((uint32_t)p.i1 << kBboxBits) | ((uint32_t)sp << 28);
            r.a.y = (uint32_t)p.j0 | ((uint32_t)p.j1 << kBboxBits) | (corner_bits(p) << kCornerShift);
            r.a.z = __float_as_uint(p.ur);
            r.a.w = __float_as_uint(p.vr);
            r.b.x = __float_as_uint(p.r2);
            r.b.y = __float_as_uint(qsf);
            r.b.z = __float_as_uint(v);
            r.b.w = __float_as_uint(r0);
            a.rec[k] = r;
            if (!a.tile_mask) {
                cnt = (uint32_t)((p.i1 / T - p.i0 / T + 1) * (p.j1 / T - p.j0 / T + 1));
            } else {
                for (int ty = p.j0 / T; ty <= p.j1 / T; ++ty)
                    for (int tx = p.i0 / T; tx <= p.i1 / T; ++tx)
                        cnt += a.tile_mask[ty * a.ntx + tx] ? 1u : 0u;
            }
            key = order_bits((float)p.zc);
            klo = min(klo, key);
            khi = max(khi, key);
        }
        a.cnt[k] = cnt;
        if (a.key) a.key[k] = key;
        if (a.o_status) a.o_status[k] = (int8_t)p.status;
        if (a.o_bbox) {
            int4 bb = make_int4(p.i0, p.i1, p.j0, p.j1);
            reinterpret_cast<int4 *>(a.o_bbox)[k] = bb;
        }
        if (a.o_spec) {
            a.o_spec[3 * k + 0] = p.ur;
            a.o_spec[3 * k + 1] = p.vr;
            a.o_spec[3 * k + 2] = p.r2;
        }
        if (a.o_key) a.o_key[k] = p.status == kVisible ? key : 0u;
        my[p.status] += 1;
    }
#pragma unroll
    for (int c = 0; c < kCntN; ++c) {
        unsigned w = wave_sum(my[c]);
        if ((threadIdx.x & 63) == 0 && w) atomicAdd(&s_cnt[c], w);
    }
    for (int q = 0; q < a.sp.n; ++q) {
        uint32_t l = lo[q], h = hi[q];
        for (int o = 32; o > 0; o >>= 1) {
            l = min(l, (uint32_t)__shfl_xor((int)l, o, 64));
            h = max(h, (uint32_t)__shfl_xor((int)h, o, 64));
        }
        if ((threadIdx.x & 63) == 0 && l != 0xFFFFFFFFu) {
            atomicMin(&s_lo[q], l);
            atomicMax(&s_hi[q], h);
        }
    }
    if (a.key) {
        for (int o = 32; o > 0; o >>= 1) {
            klo = min(klo, (uint32_t)__shfl_xor((int)klo, o, 64));
            khi = max(khi, (uint32_t)__shfl_xor((int)khi, o, 64));
        }
        if ((threadIdx.x & 63) == 0 && klo != 0xFFFFFFFFu) {
            atomicMin(&s_lo[kMaxSpecies], klo);
            atomicMax(&s_hi[kMaxSpecies], khi);
        }
    }
    __syncthreads();
    if (threadIdx.x < kCntN && s_cnt[threadIdx.x])
        atomicAdd(&a.counters[threadIdx.x], (unsigned long long)s_cnt[threadIdx.x]);
    if (threadIdx.x < a.sp.n && s_lo[threadIdx.x] != 0xFFFFFFFFu) {
        atomicMin(&a.range_bits[2 * threadIdx.x], s_lo[threadIdx.x]);
        atomicMax(&a.range_bits[2 * threadIdx.x + 1], s_hi[threadIdx.x]);
    }
    if (threadIdx.x == 0 && s_lo[kMaxSpecies] != 0xFFFFFFFFu) {
        atomicMin(&a.range_bits[2 * kMaxSpecies], s_lo[kMaxSpecies]);
        atomicMax(&a.range_bits[2 * kMaxSpecies + 1], s_hi[kMaxSpecies]);
    }
}

unsigned grid_for(size_t n, unsigned cap) {
    size_t g = (n + kThreads - 1) / kThreads;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 65536)), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_fill_f32(float *p, float v, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 65536)), dim3(kThreads), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_range_init(uint32_t *range_bits, hipStream_t s) {
    hipLaunchKernelGGL(k_init_range, dim3(1), dim3(64), 0, s, range_bits);
    return hipGetLastError();
}

hipError_t launch_project(const ProjectArgs &a, hipStream_t s) {
    if (a.n == 0) return hipSuccess;
    // grid-stride, at least 16 particles a thread between 2048 and 16384
    // workgroups: each workgroup publishes its counters and value ranges
    // with device-scope atomics on a few words, which are serialised beyond
    // the XCDs' L2 caches (16384 workgroups took 0.2 ms more than 2048 on a
    // 1e7-particle set), while a 1e9-particle set runs faster on 16384 than
    // on 2048 (13.2 against 15.0 ms)
    const size_t cap = std::min<size_t>(std::max<size_t>((size_t)a.n / (16 * kThreads), 2048), 16384);
    hipLaunchKernelGGL(k_project, dim3(grid_for((size_t)a.n, (unsigned)cap)), dim3(kThreads), 0, s,
                       a);
    return hipGetLastError();
}

}  // namespace splotch
