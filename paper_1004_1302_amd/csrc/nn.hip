// Kernels of the reconstruction network (learned decimation): a BF16 GEMM
// on gfx950 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation),
// im2col for 3x3 convolutions, and the elementwise pieces of training
// (bias + ReLU epilogue, ReLU backward, 2x2 average pool and nearest
// upsample with their adjoints, channel concat/split, loss, Adam, tone
// map).  Activations are NHWC; every image dimension and channel count the
// network uses is a multiple of 8 and 32.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nn_internal.h"

namespace splotch {
namespace nn {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float bf2f(bf16_t v) { return __uint_as_float((uint32_t)v << 16); }
__device__ __forceinline__ bf16_t f2bf(float f) {
    // round to nearest even; NaN stays NaN
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x7FFFFFu)) return (bf16_t)((u >> 16) | 0x40u);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}

// ------------------------------------------------------------------ GEMM
// C[z][M][N] (FP32) = sum over k in split z of A[m][k] * B[k][n].
// A is [M][K] (lda) or, with TRANS_A, stored as [K][M] (lda).  B is [K][N].
// Workgroup tile BM x BN x 32 with 4 waves; each wave owns (BM/WM) x
// (BN/WN) outputs as 16x16 MFMA tiles.
constexpr int BK = 32;
constexpr int PAD = 8;  // LDS row pad (bf16) keeps 16-byte fragment reads aligned

template <int BM, int BN, bool TRANS_A>
__global__ __launch_bounds__(256) void k_gemm(const bf16_t *A, const bf16_t *B, float *C, int M,
                                              int N, int K, int lda, int ldb, int k_per_split) {
    constexpr int WN = BN / 32 >= 2 ? 2 : 1;  // waves along N
    constexpr int WM = 4 / WN;                // waves along M
    constexpr int TM = BM / WM / 16, TN = BN / WN / 16;  // MFMA tiles per wave
    __shared__ __attribute__((aligned(16))) bf16_t sA[BM][BK + PAD];
    __shared__ __attribute__((aligned(16))) bf16_t sB[BN][BK + PAD];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int wm = wave / WN, wn = wave % WN;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    const int kbeg = blockIdx.z * k_per_split;
    const int kend = min(K, kbeg + k_per_split);
    f32x4 acc[TM][TN];
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int k0 = kbeg; k0 < kend; k0 += BK) {
        // stage A tile as sA[m][k]
        for (int e = tid; e < BM * BK / 8; e += 256) {
            if (!TRANS_A) {
                const int r = e / (BK / 8), c8 = (e % (BK / 8)) * 8;
                const int m = m0 + r, k = k0 + c8;
                const bf16_t *src = A + (size_t)m * lda + k;
                if (m < M && k + 8 <= kend && ((reinterpret_cast<uintptr_t>(src) & 15u) == 0)) {
                    *reinterpret_cast<uint4 *>(&sA[r][c8]) = *reinterpret_cast<const uint4 *>(src);
                } else {
#pragma unroll
                    for (int q = 0; q < 8; ++q)
                        sA[r][c8 + q] = (m < M && k + q < kend) ? src[q] : (bf16_t)0;
                }
            } else {
                const int kr = e / (BM / 8), m8 = (e % (BM / 8)) * 8;
                const int k = k0 + kr;
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int m = m0 + m8 + q;
                    sA[m8 + q][kr] = (m < M && k < kend) ? A[(size_t)k * lda + m] : (bf16_t)0;
                }
            }
        }
        // stage B tile transposed as sB[n][k]
        for (int e = tid; e < BN * BK / 8; e += 256) {
            const int kr = e / (BN / 8), n8 = (e % (BN / 8)) * 8;
            const int k = k0 + kr;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int n = n0 + n8 + q;
                sB[n8 + q][kr] = (n < N && k < kend) ? B[(size_t)k * ldb + n] : (bf16_t)0;
            }
        }
        __syncthreads();
        const int kq = (lane >> 4) * 8;
        bf16x8 af[TM], bfr[TN];
#pragma unroll
        for (int a = 0; a < TM; ++a)
            af[a] = *reinterpret_cast<const bf16x8 *>(&sA[(wm * TM + a) * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int b = 0; b < TN; ++b)
            bfr[b] = *reinterpret_cast<const bf16x8 *>(&sB[(wn * TN + b) * 16 + (lane & 15)][kq]);
#pragma unroll
        for (int a = 0; a < TM; ++a)
#pragma unroll
            for (int b = 0; b < TN; ++b)
                acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b], 0, 0, 0);
        __syncthreads();
    }
    float *Cz = C + (size_t)blockIdx.z * M * N;
#pragma unroll
    for (int a = 0; a < TM; ++a)
#pragma unroll
        for (int b = 0; b < TN; ++b) {
            const int n = n0 + (wn * TN + b) * 16 + (lane & 15);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int m = m0 + (wm * TM + a) * 16 + (lane >> 4) * 4 + q;
                if (m < M && n < N) Cz[(size_t)m * N + n] = acc[a][b][q];
            }
        }
}

// ------------------------------------------------------- fused 3x3 convolution
// Forward weights [cout][9 cin] from the GEMM operand [9 cin][cout]: row n
// holds output channel n's taps (tap-major, then input channel), so a
// lane's 8 consecutive reduction terms are one 16-byte read.
__global__ void k_conv_wf(const bf16_t *w, bf16_t *wf, int cin, int cout) {
    const size_t k9 = (size_t)9 * cin, total = k9 * cout;
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const size_t n = e / k9, k = e % k9;
        wf[e] = w[k * cout + n];
    }
}

// out = epilogue(conv3x3(x, W) + bias) for NHWC BF16 x, without an im2col
// buffer: the implicit GEMM (pixels x cout, reduction over 9 taps x cin)
// runs on the matrix cores from LDS.  A workgroup owns an 8 x 16 pixel
// tile and CO output channels; per 32-channel slice of the input it stages
// the tile with its one-pixel halo (zeros outside the image) and the
// slice's weights for all 9 taps, then each wave accumulates 2 rows of 16
// pixels x CO channels, one MFMA per (row, 16 channels) per tap.
constexpr int kCTH = 8, kCTW = 16;           // output tile rows, columns
constexpr int kCHW = kCTW + 2;               // halo tile width
constexpr int kCHP = (kCTH + 2) * kCHW;      // halo tile pixels
constexpr int kCK = 32;                      // input channels per stage
constexpr int kCRow = kCK + PAD;             // LDS row (bf16); 80 B spreads the banks

template <int CO>
__global__ __launch_bounds__(256) void k_conv3x3(const bf16_t *x, const bf16_t *wf,
                                                 const float *bias, int relu,
                                                 const float *residual, bf16_t *out_bf,
                                                 float *out_f, int h, int w, int cin, int cout) {
    constexpr int NT = CO / 16;
    __shared__ __attribute__((aligned(16))) bf16_t sX[kCHP][kCRow];
    __shared__ __attribute__((aligned(16))) bf16_t sW[9 * CO][kCRow];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int tiles_x = (w + kCTW - 1) / kCTW, tiles_y = (h + kCTH - 1) / kCTH;
    const int tile = (int)(blockIdx.x % (unsigned)(tiles_x * tiles_y));
    const int img = (int)(blockIdx.x / (unsigned)(tiles_x * tiles_y));
    const int y0 = (tile / tiles_x) * kCTH, x0 = (tile % tiles_x) * kCTW;
    const int n0 = (int)blockIdx.y * CO;
    const size_t k9 = (size_t)9 * cin;
    const size_t plane = (size_t)img * h;
    f32x4 acc[2][NT];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < NT; ++b) acc[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int kq = (lane >> 4) * 8;
    for (int c0 = 0; c0 < cin; c0 += kCK) {
        __syncthreads();  // the previous slice's fragments are read
        for (int e = tid; e < kCHP * 4; e += 256) {
            const int p = e >> 2, q = (e & 3) * 8;
            const int yy = y0 - 1 + p / kCHW, xx = x0 - 1 + p % kCHW;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (yy >= 0 && yy < h && xx >= 0 && xx < w)
                v = *reinterpret_cast<const uint4 *>(x + ((plane + yy) * w + xx) * cin + c0 + q);
            *reinterpret_cast<uint4 *>(&sX[p][q]) = v;
        }
        for (int e = tid; e < 9 * CO * 4; e += 256) {
            const int r = e >> 2, q = (e & 3) * 8;
            const int tap = r / CO, nl = r % CO;
            *reinterpret_cast<uint4 *>(&sW[r][q]) = *reinterpret_cast<const uint4 *>(
                wf + (size_t)(n0 + nl) * k9 + (size_t)tap * cin + c0 + q);
        }
        __syncthreads();
#pragma unroll
        for (int tap = 0; tap < 9; ++tap) {
            const int dy = tap / 3, dx = tap % 3;
            bf16x8 af[2], bfr[NT];
#pragma unroll
            for (int a = 0; a < 2; ++a)
                af[a] = *reinterpret_cast<const bf16x8 *>(
                    &sX[(2 * wave + a + dy) * kCHW + (lane & 15) + dx][kq]);
#pragma unroll
            for (int b = 0; b < NT; ++b)
                bfr[b] = *reinterpret_cast<const bf16x8 *>(&sW[tap * CO + b * 16 + (lane & 15)][kq]);
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < NT; ++b)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[a], bfr[b], acc[a][b],
                                                                        0, 0, 0);
        }
    }
    // output (pixel, channel) of acc[a][b][q]: row 2 wave + a, column
    // 4 (lane / 16) + q of the tile; channel n0 + 16 b + lane % 16
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        const int yy = y0 + 2 * wave + a;
        if (yy >= h) continue;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int xx = x0 + (lane >> 4) * 4 + q;
            if (xx >= w) continue;
            const size_t pix = (plane + yy) * w + xx;
#pragma unroll
            for (int b = 0; b < NT; ++b) {
                const int n = n0 + b * 16 + (lane & 15);
                const size_t e = pix * cout + n;
                float v = acc[a][b][q];
                if (bias) v += bias[n];
                if (relu) v = v > 0.f ? v : 0.f;
                if (residual) v += residual[e];
                if (out_bf) out_bf[e] = f2bf(v);
                if (out_f) out_f[e] = v;
            }
        }
    }
}

// ------------------------------------------------------------------ im2col
// out[p][tap*C + c] = in[p shifted by tap][c] (zero outside the image),
// taps in (ky, kx) row-major order, p = (img, y, x).
__global__ void k_im2col3x3(const bf16_t *in, bf16_t *out, int n, int h, int w, int c) {
    const size_t total = (size_t)n * h * w * 9 * (c / 8);
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        const int c8 = (int)(e % (c / 8)) * 8;
        size_t r = e / (c / 8);
        const int tap = (int)(r % 9);
        const size_t p = r / 9;
        const int x = (int)(p % w), y = (int)((p / w) % h), img = (int)(p / ((size_t)w * h));
        const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
        uint4 v = make_uint4(0, 0, 0, 0);
        if (yy >= 0 && yy < h && xx >= 0 && xx < w)
            v = *reinterpret_cast<const uint4 *>(in + (((size_t)img * h + yy) * w + xx) * c + c8);
        *reinterpret_cast<uint4 *>(out + (p * 9 + tap) * c + c8) = v;
    }
}

// Weights of the adjoint (backward-data) convolution.  Forward weights are
// stored as the GEMM operand w[tap][ci][co]; the adjoint operand is
// wt[tap'][co][ci] = w[8 - tap'][ci][co] (taps mirrored, channels swapped).
__global__ void k_flip_weights(const bf16_t *w, bf16_t *wt, int cout, int cin) {
    const int total = 9 * cin * cout;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < total; e += gridDim.x * blockDim.x) {
        const int co = e % cout, ci = (e / cout) % cin, tap = e / (cout * cin);
        wt[((size_t)(8 - tap) * cout + co) * cin + ci] = w[e];
    }
}

// Sum split-K partials, add bias, apply ReLU; write BF16 and/or FP32,
// optionally adding a residual (FP32) after the activation.
__global__ void k_epilogue(const float *Cp, int splits, size_t mn, int n, const float *bias,
                           int relu, const float *residual, bf16_t *out_bf, float *out_f) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < mn; e += stride) {
        float v = 0.f;
        for (int z = 0; z < splits; ++z) v += Cp[(size_t)z * mn + e];
        if (bias) v += bias[e % n];
        if (relu) v = v > 0.f ? v : 0.f;
        if (residual) v += residual[e];
        if (out_bf) out_bf[e] = f2bf(v);
        if (out_f) out_f[e] = v;
    }
}

// dZ = dY * [Y > 0] (ReLU adjoint), written as BF16 for the GEMMs and
// reduced per channel into the bias gradient (one atomic per block and
// channel is avoided: per-block partial sums, reduced by k_colsum).
__global__ void k_relu_bwd(const float *dy, const bf16_t *y, int relu, bf16_t *dz_bf,
                           float *dz_f, size_t total) {
    size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += stride) {
        float g = dy[e];
        if (relu && !(bf2f(y[e]) > 0.f)) g = 0.f;
        dz_bf[e] = f2bf(g);
        if (dz_f) dz_f[e] = g;
    }
}

// Column sums of in[rows][cols] (cols <= 256) in two passes: each block
// sums a contiguous chunk of rows for every column (lanes spread over
// columns, coalesced), then one pass adds the per-block partials in order.
__global__ void k_colsum_part(const float *in, size_t rows, int cols, size_t rows_per_block,
                              float *part) {
    __shared__ float sh[256];
    const int per_row = 256 / cols;  // rows covered by one sweep of the block
    const int t = threadIdx.x, c = t % cols, r0 = t / cols;
    const size_t beg = (size_t)blockIdx.x * rows_per_block;
    const size_t end = beg + rows_per_block < rows ? beg + rows_per_block : rows;
    float s = 0.f;
    if (r0 < per_row)
        for (size_t r = beg + r0; r < end; r += per_row) s += in[r * cols + c];
    sh[t] = s;
    __syncthreads();
    if (t < cols) {
        float tot = 0.f;
        for (int k = 0; k < per_row; ++k) tot += sh[k * cols + t];
        part[(size_t)blockIdx.x * cols + t] = tot;
    }
}

__global__ void k_colsum_final(const float *part, int nblocks, int cols, float *out) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= cols) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += part[(size_t)b * cols + c];
    out[c] = s;
}

// 2x2 average pool (NHWC, BF16 in/out) and its adjoint (FP32 in/out).
// Eight channels per thread (one 16-byte load per input pixel).
__global__ void k_pool2(const bf16_t *in, bf16_t *out, int n, int h, int w, int c) {
    const int ho = h / 2, wo = w / 2, c8 = c / 8;
    const size_t total = (size_t)n * ho * wo * c8;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(e % c8) * 8;
        size_t p = e / c8;
        const int x = (int)(p % wo), y = (int)((p / wo) % ho), img = (int)(p / ((size_t)wo * ho));
        const size_t b = (((size_t)img * h + 2 * y) * w + 2 * x) * c + ch;
        const size_t row = (size_t)w * c;
        union U {
            uint4 v;
            bf16_t s[8];
        } q0, q1, q2, q3, o;
        q0.v = *reinterpret_cast<const uint4 *>(in + b);
        q1.v = *reinterpret_cast<const uint4 *>(in + b + c);
        q2.v = *reinterpret_cast<const uint4 *>(in + b + row);
        q3.v = *reinterpret_cast<const uint4 *>(in + b + row + c);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const float sum = bf2f(q0.s[k]) + bf2f(q1.s[k]) + bf2f(q2.s[k]) + bf2f(q3.s[k]);
            o.s[k] = f2bf(0.25f * sum);
        }
        *reinterpret_cast<uint4 *>(out + p * c + ch) = o.v;
    }
}

__global__ void k_pool2_bwd(const float *dout, float *din, int n, int h, int w, int c,
                            int accumulate) {
    const size_t total = (size_t)n * h * w * c;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(e % c);
        size_t p = e / c;
        const int x = (int)(p % w), y = (int)((p / w) % h), img = (int)(p / ((size_t)w * h));
        const float g = 0.25f * dout[(((size_t)img * (h / 2) + y / 2) * (w / 2) + x / 2) * c + ch];
        din[e] = accumulate ? din[e] + g : g;
    }
}

// Nearest 2x upsample of `a` (ca channels, h/2 x w/2) concatenated with
// `s` (cs channels, h x w) along channels: out has ca + cs channels.
// Eight channels per thread; ca and cs are multiples of 8, so a group of
// eight never straddles the two sources.
__global__ void k_up2_concat(const bf16_t *a, int ca, const bf16_t *s, int cs, bf16_t *out, int n,
                             int h, int w) {
    const int co = ca + cs, c8 = co / 8;
    const size_t total = (size_t)n * h * w * c8;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(e % c8) * 8;
        size_t p = e / c8;
        const int x = (int)(p % w), y = (int)((p / w) % h), img = (int)(p / ((size_t)w * h));
        const bf16_t *src = ch < ca
            ? a + (((size_t)img * (h / 2) + y / 2) * (w / 2) + x / 2) * ca + ch
            : s + p * cs + (ch - ca);
        *reinterpret_cast<uint4 *>(out + p * co + ch) = *reinterpret_cast<const uint4 *>(src);
    }
}

// Adjoint of k_up2_concat: da (FP32, h/2 x w/2 x ca) = 2x2 sums of the first
// ca channels; ds (FP32, h x w x cs) = the remaining channels.
__global__ void k_up2_concat_bwd(const float *dout, int ca, int cs, float *da, float *ds, int n,
                                 int h, int w) {
    const int co = ca + cs;
    const size_t plow = (size_t)n * (h / 2) * (w / 2);
    const size_t total_a = plow * ca, total_s = (size_t)n * h * w * cs;
    const size_t total = total_a + total_s;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        if (e < total_a) {
            const int ch = (int)(e % ca);
            const size_t p = e / ca;
            const int x = (int)(p % (w / 2)), y = (int)((p / (w / 2)) % (h / 2));
            const int img = (int)(p / ((size_t)(w / 2) * (h / 2)));
            const size_t b = (((size_t)img * h + 2 * y) * w + 2 * x) * co + ch;
            da[e] = dout[b] + dout[b + co] + dout[b + (size_t)w * co] + dout[b + (size_t)w * co + co];
        } else {
            const size_t f = e - total_a;
            const int ch = (int)(f % cs);
            const size_t p = f / cs;
            ds[f] = dout[p * co + ca + ch];
        }
    }
}

// Mean-squared error over the first `used` of `c` channels and its
// gradient; partial sums per block in loss_part.
__global__ void k_mse(const float *pred, const float *target, float *grad, size_t pixels, int c,
                      int used, float *loss_part) {
    __shared__ float sh[256];
    float s = 0.f;
    const float scale = 2.0f / (float)(pixels * used);
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < pixels * c;
         e += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(e % c);
        float d = 0.f;
        if (ch < used) {
            d = pred[e] - target[e];
            s += d * d;
        }
        grad[e] = scale * d;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = sh[0];
}

// Adam with bias correction; FP32 master weights, BF16 copy for the GEMMs.
__global__ void k_adam(float *w, bf16_t *w_bf, const float *g, float *m, float *v, size_t n,
                       float lr, float b1, float b2, float eps, float c1, float c2) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x) {
        const float gi = g[e];
        const float mi = b1 * m[e] + (1.f - b1) * gi;
        const float vi = b2 * v[e] + (1.f - b2) * gi * gi;
        m[e] = mi;
        v[e] = vi;
        const float wi = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[e] = wi;
        if (w_bf) w_bf[e] = f2bf(wi);
    }
}

// Tone-map scale: the host value, or the device sum times inv_count (the
// image mean); a non-positive or non-finite scale becomes 1.
__device__ __forceinline__ float tone_scale(const float *sum, float inv_count, float s) {
    if (sum) s = sum[0] * inv_count;
    return (s > 0.f && s < 3.0e38f) ? s : 1.f;
}

// Tone map of a planar float image [3][h][w] into NHWC with c channels
// (channels >= 3 zero): out = log1p(img / s), s > 0 per image.
__global__ void k_tonemap(const float *img, int h, int w, const float *sum, float inv_count,
                          float s0, int c, float *out_f, bf16_t *out_bf) {
    const float s = tone_scale(sum, inv_count, s0);
    const size_t total = (size_t)h * w * c;
    const size_t plane = (size_t)h * w;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(e % c);
        const size_t p = e / c;
        float v = 0.f;
        if (ch < 3) v = log1pf(fmaxf(img[ch * plane + p], 0.f) / s);
        if (out_f) out_f[e] = v;
        if (out_bf) out_bf[e] = f2bf(v);
    }
}

// Inverse tone map from NHWC (first 3 channels) to planar [3][h][w].
__global__ void k_untonemap(const float *in, int h, int w, const float *sum, float inv_count,
                            float s0, int c, float *img) {
    const float s = tone_scale(sum, inv_count, s0);
    const size_t plane = (size_t)h * w;
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < 3 * plane;
         e += (size_t)gridDim.x * blockDim.x) {
        const int ch = (int)(e / plane);
        const size_t p = e % plane;
        img[e] = s * expm1f(in[p * c + ch]);
    }
}

__global__ void k_f2bf(const float *in, bf16_t *out, size_t n) {
    for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (size_t)gridDim.x * blockDim.x)
        out[e] = f2bf(in[e]);
}

unsigned grid_for(size_t n) {
    size_t g = (n + 255) / 256;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

}  // namespace

hipError_t gemm(const bf16_t *A, const bf16_t *B, float *C, int M, int N, int K, int lda, int ldb,
                int trans_a, int splits, hipStream_t s) {
    if (splits < 1) splits = 1;
    int kps = (K + splits - 1) / splits;
    kps = (kps + BK - 1) / BK * BK;
    splits = (K + kps - 1) / kps;
    if (splits < 1) splits = 1;
    const int bn = N <= 32 ? 32 : 64;
    dim3 grid((M + 63) / 64, (N + bn - 1) / bn, splits);
    if (bn == 32) {
        if (trans_a)
            hipLaunchKernelGGL((k_gemm<64, 32, true>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
        else
            hipLaunchKernelGGL((k_gemm<64, 32, false>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
    } else {
        if (trans_a)
            hipLaunchKernelGGL((k_gemm<64, 64, true>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
        else
            hipLaunchKernelGGL((k_gemm<64, 64, false>), grid, dim3(256), 0, s, A, B, C, M, N, K, lda, ldb, kps);
    }
    return hipGetLastError();
}

int gemm_splits(int K, int splits) {
    if (splits < 1) splits = 1;
    int kps = (K + splits - 1) / splits;
    kps = (kps + BK - 1) / BK * BK;
    splits = (K + kps - 1) / kps;
    return splits < 1 ? 1 : splits;
}

hipError_t im2col3x3(const bf16_t *in, bf16_t *out, int n, int h, int w, int c, hipStream_t s) {
    const size_t total = (size_t)n * h * w * 9 * (c / 8);
    hipLaunchKernelGGL(k_im2col3x3, dim3(grid_for(total)), dim3(256), 0, s, in, out, n, h, w, c);
    return hipGetLastError();
}

hipError_t flip_weights(const bf16_t *w, bf16_t *wt, int cout, int cin, hipStream_t s) {
    hipLaunchKernelGGL(k_flip_weights, dim3(grid_for((size_t)cout * 9 * cin)), dim3(256), 0, s, w,
                       wt, cout, cin);
    return hipGetLastError();
}

hipError_t epilogue(const float *Cp, int splits, size_t mn, int n, const float *bias, int relu,
                    const float *residual, bf16_t *out_bf, float *out_f, hipStream_t s) {
    hipLaunchKernelGGL(k_epilogue, dim3(grid_for(mn)), dim3(256), 0, s, Cp, splits, mn, n, bias,
                       relu, residual, out_bf, out_f);
    return hipGetLastError();
}

hipError_t conv3x3_weights(const bf16_t *w, bf16_t *wf, int cin, int cout, hipStream_t s) {
    const size_t total = (size_t)9 * cin * cout;
    hipLaunchKernelGGL(k_conv_wf, dim3(grid_for(total)), dim3(256), 0, s, w, wf, cin, cout);
    return hipGetLastError();
}

hipError_t conv3x3(const bf16_t *x, const bf16_t *wf, const float *bias, int relu,
                   const float *residual, bf16_t *out_bf, float *out_f, int n, int h, int w,
                   int cin, int cout, hipStream_t s) {
    const unsigned tiles = (unsigned)((h + kCTH - 1) / kCTH) * (unsigned)((w + kCTW - 1) / kCTW);
    // 64 output channels per workgroup where that still gives the GPU
    // enough workgroups, 32 on the small deep levels
    if (cout % 64 == 0 && (uint64_t)tiles * (uint64_t)n * (uint64_t)(cout / 64) >= 1024) {
        hipLaunchKernelGGL(k_conv3x3<64>, dim3(tiles * (unsigned)n, (unsigned)(cout / 64)),
                           dim3(256), 0, s, x, wf, bias, relu, residual, out_bf, out_f, h, w, cin,
                           cout);
    } else {
        hipLaunchKernelGGL(k_conv3x3<32>, dim3(tiles * (unsigned)n, (unsigned)(cout / 32)),
                           dim3(256), 0, s, x, wf, bias, relu, residual, out_bf, out_f, h, w, cin,
                           cout);
    }
    return hipGetLastError();
}

hipError_t relu_bwd(const float *dy, const bf16_t *y, int relu, bf16_t *dz_bf, float *dz_f,
                    size_t total, hipStream_t s) {
    hipLaunchKernelGGL(k_relu_bwd, dim3(grid_for(total)), dim3(256), 0, s, dy, y, relu, dz_bf,
                       dz_f, total);
    return hipGetLastError();
}

hipError_t colsum(const float *in, size_t rows, int cols, float *out, float *part, hipStream_t s) {
    size_t rpb = (rows + kColsumBlocks - 1) / kColsumBlocks;
    if (rpb < 256) rpb = 256;
    const int nb = (int)((rows + rpb - 1) / rpb);
    hipLaunchKernelGGL(k_colsum_part, dim3(nb), dim3(256), 0, s, in, rows, cols, rpb, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, s, part, nb, cols,
                       out);
    return hipGetLastError();
}

hipError_t pool2(const bf16_t *in, bf16_t *out, int n, int h, int w, int c, hipStream_t s) {
    hipLaunchKernelGGL(k_pool2, dim3(grid_for((size_t)n * h * w * c / 32)), dim3(256), 0, s, in,
                       out, n, h, w, c);
    return hipGetLastError();
}

hipError_t pool2_bwd(const float *dout, float *din, int n, int h, int w, int c, int accumulate,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_pool2_bwd, dim3(grid_for((size_t)n * h * w * c)), dim3(256), 0, s, dout,
                       din, n, h, w, c, accumulate);
    return hipGetLastError();
}

hipError_t up2_concat(const bf16_t *a, int ca, const bf16_t *sk, int cs, bf16_t *out, int n,
                      int h, int w, hipStream_t s) {
    hipLaunchKernelGGL(k_up2_concat, dim3(grid_for((size_t)n * h * w * (ca + cs) / 8)), dim3(256), 0,
                       s, a, ca, sk, cs, out, n, h, w);
    return hipGetLastError();
}

hipError_t up2_concat_bwd(const float *dout, int ca, int cs, float *da, float *ds, int n, int h,
                          int w, hipStream_t s) {
    const size_t total = (size_t)n * (h / 2) * (w / 2) * ca + (size_t)n * h * w * cs;
    hipLaunchKernelGGL(k_up2_concat_bwd, dim3(grid_for(total)), dim3(256), 0, s, dout, ca, cs, da,
                       ds, n, h, w);
    return hipGetLastError();
}

hipError_t mse(const float *pred, const float *target, float *grad, size_t pixels, int c,
               int used, float *loss_part, int nblocks, hipStream_t s) {
    hipLaunchKernelGGL(k_mse, dim3(nblocks), dim3(256), 0, s, pred, target, grad, pixels, c, used,
                       loss_part);
    return hipGetLastError();
}

hipError_t adam(float *w, bf16_t *w_bf, const float *g, float *m, float *v, size_t n, float lr,
                float b1, float b2, float eps, int step, hipStream_t s) {
    const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(n)), dim3(256), 0, s, w, w_bf, g, m, v, n, lr, b1, b2,
                       eps, c1, c2);
    return hipGetLastError();
}

hipError_t tonemap(const float *img, int h, int w, float scale, int c, float *out_f,
                   bf16_t *out_bf, hipStream_t s, const float *sum, float inv_count) {
    hipLaunchKernelGGL(k_tonemap, dim3(grid_for((size_t)h * w * c)), dim3(256), 0, s, img, h, w,
                       sum, inv_count, scale, c, out_f, out_bf);
    return hipGetLastError();
}

hipError_t untonemap(const float *in, int h, int w, float scale, int c, float *img, hipStream_t s,
                     const float *sum, float inv_count) {
    hipLaunchKernelGGL(k_untonemap, dim3(grid_for((size_t)h * w * 3)), dim3(256), 0, s, in, h, w,
                       sum, inv_count, scale, c, img);
    return hipGetLastError();
}

hipError_t f2bf(const float *in, bf16_t *out, size_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_f2bf, dim3(grid_for(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace splotch
