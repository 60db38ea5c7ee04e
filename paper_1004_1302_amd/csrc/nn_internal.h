// Launchers of the reconstruction-network kernels (nn.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace splotch {
namespace nn {

typedef uint16_t bf16_t;  // bfloat16 bits

hipError_t gemm(const bf16_t *A, const bf16_t *B, float *C, int M, int N, int K, int lda, int ldb,
                int trans_a, int splits, hipStream_t s);
int gemm_splits(int K, int splits);
hipError_t im2col3x3(const bf16_t *in, bf16_t *out, int n, int h, int w, int c, hipStream_t s);
hipError_t flip_weights(const bf16_t *w, bf16_t *wt, int cout, int cin, hipStream_t s);
// Fused 3x3 convolution (zero padding) with the epilogue below: cin and cout
// multiples of 32; wf from conv3x3_weights ([cout][9 cin]).
hipError_t conv3x3_weights(const bf16_t *w, bf16_t *wf, int cin, int cout, hipStream_t s);
hipError_t conv3x3(const bf16_t *x, const bf16_t *wf, const float *bias, int relu,
                   const float *residual, bf16_t *out_bf, float *out_f, int n, int h, int w,
                   int cin, int cout, hipStream_t s);
hipError_t epilogue(const float *Cp, int splits, size_t mn, int n, const float *bias, int relu,
                    const float *residual, bf16_t *out_bf, float *out_f, hipStream_t s);
hipError_t relu_bwd(const float *dy, const bf16_t *y, int relu, bf16_t *dz_bf, float *dz_f,
                    size_t total, hipStream_t s);
// Column sums (cols <= 256); part: scratch of kColsumBlocks * cols floats.
constexpr int kColsumBlocks = 1024;
hipError_t colsum(const float *in, size_t rows, int cols, float *out, float *part, hipStream_t s);
hipError_t pool2(const bf16_t *in, bf16_t *out, int n, int h, int w, int c, hipStream_t s);
hipError_t pool2_bwd(const float *dout, float *din, int n, int h, int w, int c, int accumulate,
                     hipStream_t s);
hipError_t up2_concat(const bf16_t *a, int ca, const bf16_t *sk, int cs, bf16_t *out, int n,
                      int h, int w, hipStream_t s);
hipError_t up2_concat_bwd(const float *dout, int ca, int cs, float *da, float *ds, int n, int h,
                          int w, hipStream_t s);
hipError_t mse(const float *pred, const float *target, float *grad, size_t pixels, int c,
               int used, float *loss_part, int nblocks, hipStream_t s);
hipError_t adam(float *w, bf16_t *w_bf, const float *g, float *m, float *v, size_t n, float lr,
                float b1, float b2, float eps, int step, hipStream_t s);
// Tone map with scale s: `scale`, or, when sum is not null, sum[0] *
// inv_count read on the device (the image mean, no host read-back).
hipError_t tonemap(const float *img, int h, int w, float scale, int c, float *out_f,
                   bf16_t *out_bf, hipStream_t s, const float *sum = nullptr,
                   float inv_count = 0.f);
hipError_t untonemap(const float *in, int h, int w, float scale, int c, float *img, hipStream_t s,
                     const float *sum = nullptr, float inv_count = 0.f);
hipError_t f2bf(const float *in, bf16_t *out, size_t n, hipStream_t s);

}  // namespace nn
}  // namespace splotch
