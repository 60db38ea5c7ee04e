// C ABI of the reconstruction-network kernels (declared in include/splotch.h).
#include "../../include/splotch.h"
#include "nn_internal.h"

using namespace splotch::nn;

namespace {
inline hipStream_t st(void *s) { return reinterpret_cast<hipStream_t>(s); }
inline splotch_status ok(hipError_t e) { return e == hipSuccess ? SPLOTCH_OK : SPLOTCH_E_DEVICE; }
inline bool m8(int v) { return v > 0 && v % 8 == 0; }
// 16-byte aligned (the vectorised kernels move eight bf16 at a time)
inline bool a16(const void *p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }
}  // namespace

extern "C" {

splotch_status splotch_nn_gemm(const uint16_t *A, const uint16_t *B, float *C, int32_t M,
                               int32_t N, int32_t K, int32_t lda, int32_t ldb, int32_t trans_a,
                               int32_t splits, void *stream) {
    if (!A || !B || !C || M <= 0 || N <= 0 || K <= 0 || splits < 1) return SPLOTCH_E_INVALID_ARG;
    if ((!trans_a && lda < K) || (trans_a && lda < M) || ldb < N) return SPLOTCH_E_INVALID_ARG;
    return ok(gemm(A, B, C, M, N, K, lda, ldb, trans_a ? 1 : 0, splits, st(stream)));
}

int32_t splotch_nn_gemm_splits(int32_t K, int32_t splits) { return gemm_splits(K, splits); }

splotch_status splotch_nn_im2col3x3(const uint16_t *in, uint16_t *out, int32_t n, int32_t h,
                                    int32_t w, int32_t c, void *stream) {
    if (!in || !out || n <= 0 || h <= 0 || w <= 0 || !m8(c)) return SPLOTCH_E_INVALID_ARG;
    return ok(im2col3x3(in, out, n, h, w, c, st(stream)));
}

splotch_status splotch_nn_flip_weights(const uint16_t *w, uint16_t *wt, int32_t cout, int32_t cin,
                                       void *stream) {
    if (!w || !wt || cout <= 0 || cin <= 0) return SPLOTCH_E_INVALID_ARG;
    return ok(flip_weights(w, wt, cout, cin, st(stream)));
}

splotch_status splotch_nn_epilogue(const float *partials, int32_t splits, int64_t rows,
                                   int32_t cols, const float *bias, int32_t relu,
                                   const float *residual, uint16_t *out_bf16, float *out_f32,
                                   void *stream) {
    if (!partials || splits < 1 || rows <= 0 || cols <= 0 || (!out_bf16 && !out_f32))
        return SPLOTCH_E_INVALID_ARG;
    return ok(epilogue(partials, splits, (size_t)rows * cols, cols, bias, relu, residual, out_bf16,
                       out_f32, st(stream)));
}

splotch_status splotch_nn_conv3x3_weights(const uint16_t *w, uint16_t *wf, int32_t cin,
                                         int32_t cout, void *stream) {
    if (!w || !wf || cin <= 0 || cout <= 0) return SPLOTCH_E_INVALID_ARG;
    return ok(conv3x3_weights(w, wf, cin, cout, st(stream)));
}

splotch_status splotch_nn_conv3x3(const uint16_t *x, const uint16_t *wf, const float *bias,
                                  int32_t relu, const float *residual, uint16_t *out_bf16,
                                  float *out_f32, int32_t n, int32_t h, int32_t w, int32_t cin,
                                  int32_t cout, void *stream) {
    if (!x || !wf || (!out_bf16 && !out_f32) || n <= 0 || h <= 0 || w <= 0)
        return SPLOTCH_E_INVALID_ARG;
    if (cin <= 0 || cin % 32 || cout <= 0 || cout % 32) return SPLOTCH_E_INVALID_ARG;
    if (!a16(x) || !a16(wf)) return SPLOTCH_E_INVALID_ARG;
    const uint64_t tiles = (uint64_t)((h + 7) / 8) * (uint64_t)((w + 15) / 16) * (uint64_t)n;
    if (tiles >= (1ull << 31)) return SPLOTCH_E_INVALID_ARG;
    return ok(conv3x3(x, wf, bias, relu ? 1 : 0, residual, out_bf16, out_f32, n, h, w, cin, cout,
                      st(stream)));
}

splotch_status splotch_nn_relu_bwd(const float *dy, const uint16_t *y, int32_t relu,
                                   uint16_t *dz_bf16, float *dz_f32, int64_t n, void *stream) {
    if (!dy || !dz_bf16 || n <= 0 || (relu && !y)) return SPLOTCH_E_INVALID_ARG;
    return ok(relu_bwd(dy, y, relu, dz_bf16, dz_f32, (size_t)n, st(stream)));
}

splotch_status splotch_nn_colsum(const float *in, int64_t rows, int32_t cols, float *out,
                                 float *scratch, void *stream) {
    if (!in || !out || !scratch || rows <= 0 || cols <= 0 || cols > 256)
        return SPLOTCH_E_INVALID_ARG;
    return ok(colsum(in, (size_t)rows, cols, out, scratch, st(stream)));
}

splotch_status splotch_nn_pool2(const uint16_t *in, uint16_t *out, int32_t n, int32_t h, int32_t w,
                                int32_t c, void *stream) {
    if (!in || !out || n <= 0 || h <= 0 || w <= 0 || h % 2 || w % 2 || !m8(c))
        return SPLOTCH_E_INVALID_ARG;
    if (!a16(in) || !a16(out)) return SPLOTCH_E_INVALID_ARG;
    return ok(pool2(in, out, n, h, w, c, st(stream)));
}

splotch_status splotch_nn_pool2_bwd(const float *dout, float *din, int32_t n, int32_t h,
                                    int32_t w, int32_t c, int32_t accumulate, void *stream) {
    if (!dout || !din || n <= 0 || h <= 0 || w <= 0 || h % 2 || w % 2 || c <= 0)
        return SPLOTCH_E_INVALID_ARG;
    return ok(pool2_bwd(dout, din, n, h, w, c, accumulate, st(stream)));
}

splotch_status splotch_nn_up2_concat(const uint16_t *a, int32_t ca, const uint16_t *s, int32_t cs,
                                     uint16_t *out, int32_t n, int32_t h, int32_t w,
                                     void *stream) {
    if (!a || !s || !out || !m8(ca) || !m8(cs) || n <= 0 || h <= 0 || w <= 0 || h % 2 || w % 2)
        return SPLOTCH_E_INVALID_ARG;
    if (!a16(a) || !a16(s) || !a16(out)) return SPLOTCH_E_INVALID_ARG;
    return ok(up2_concat(a, ca, s, cs, out, n, h, w, st(stream)));
}

splotch_status splotch_nn_up2_concat_bwd(const float *dout, int32_t ca, int32_t cs, float *da,
                                         float *ds, int32_t n, int32_t h, int32_t w,
                                         void *stream) {
    if (!dout || !da || !ds || ca <= 0 || cs <= 0 || n <= 0 || h % 2 || w % 2)
        return SPLOTCH_E_INVALID_ARG;
    return ok(up2_concat_bwd(dout, ca, cs, da, ds, n, h, w, st(stream)));
}

splotch_status splotch_nn_mse(const float *pred, const float *target, float *grad, int64_t pixels,
                              int32_t c, int32_t used, float *loss_partials, int32_t nblocks,
                              void *stream) {
    if (!pred || !target || !grad || !loss_partials || pixels <= 0 || c <= 0 || used <= 0 ||
        used > c || nblocks < 1)
        return SPLOTCH_E_INVALID_ARG;
    return ok(mse(pred, target, grad, (size_t)pixels, c, used, loss_partials, nblocks, st(stream)));
}

splotch_status splotch_nn_adam(float *w, uint16_t *w_bf16, const float *g, float *m, float *v,
                               int64_t n, float lr, float b1, float b2, float eps, int32_t step,
                               void *stream) {
    if (!w || !g || !m || !v || n <= 0 || step < 1) return SPLOTCH_E_INVALID_ARG;
    return ok(adam(w, w_bf16, g, m, v, (size_t)n, lr, b1, b2, eps, step, st(stream)));
}

splotch_status splotch_nn_tonemap(const float *img, int32_t h, int32_t w, float scale, int32_t c,
                                  float *out_f32, uint16_t *out_bf16, void *stream) {
    if (!img || h <= 0 || w <= 0 || !(scale > 0.0f) || c < 3 || (!out_f32 && !out_bf16))
        return SPLOTCH_E_INVALID_ARG;
    return ok(tonemap(img, h, w, scale, c, out_f32, out_bf16, st(stream)));
}

splotch_status splotch_nn_untonemap(const float *in, int32_t h, int32_t w, float scale, int32_t c,
                                    float *img, void *stream) {
    if (!in || !img || h <= 0 || w <= 0 || !(scale > 0.0f) || c < 3) return SPLOTCH_E_INVALID_ARG;
    return ok(untonemap(in, h, w, scale, c, img, st(stream)));
}

splotch_status splotch_nn_f32_to_bf16(const float *in, uint16_t *out, int64_t n, void *stream) {
    if (!in || !out || n <= 0) return SPLOTCH_E_INVALID_ARG;
    return ok(f2bf(in, out, (size_t)n, st(stream)));
}

}  // extern "C"
