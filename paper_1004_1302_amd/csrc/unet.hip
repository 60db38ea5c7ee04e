// The reconstruction network of the learned-decimation path as a library
// object: parameter layout in caller-owned memory, seeded initialisation,
// forward and backward passes over the network kernels of nn.hip, the MSE
// loss, Adam, checkpoints, and the image-level steps (tone map with the
// image mean found on the device, reconstruction, one training step).
//
// Network: n_levels levels with channels c_0..c_{L-1}.  Each level applies
// two 3x3 convolutions with ReLU; the encoder halves the resolution with 2x2
// average pooling between levels, the decoder doubles it with nearest
// upsampling and concatenates the encoder features of the same level; a
// last 3x3 convolution (no activation) adds a correction to the tone-mapped
// input:  x = log1p(I_dec / s),  y = x + net(x),  I = s expm1(y),  s the
// mean of the decimated render.  Activations are NHWC bf16, convolution
// outputs accumulate in FP32 on the matrix cores.
#include <math.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "../../include/splotch.h"
#include "internal.h"
#include "nn_internal.h"

using namespace splotch::nn;

namespace {

inline size_t al(size_t v) { return (v + 255) / 256 * 256; }
inline hipStream_t st(void *s) { return reinterpret_cast<hipStream_t>(s); }

constexpr size_t kNone = (size_t)-1;
constexpr int kLossBlocks = 256;
constexpr uint32_t kMagic[2] = {0x4e4e4c53u, 0x00000001u};  // "SLNN", version 1

struct Conv {
    int cin, cout, relu, level;
    size_t w, b, gw, gb, mw, vw, mb, vb;  // float32 byte offsets in the parameters
    size_t w_bf, wt_bf, wf_bf;            // bf16 copies: [9cin][cout], [9cout][cin], [cout][9cin]
    // activations (byte offsets in the workspace; set by the layout)
    size_t x, y, dy, dx;
};

// Workspace layout for one (n, h, w).
struct Acts {
    int n = 0, h = 0, w = 0;
    size_t x_f, x_bf, t_f, gy, y, loss, sum, csum;
    std::vector<size_t> pin, ea, e, cat, da, dd, gdn, ge;
    size_t dz_bf, dz_f, col, colz, gemm;
    size_t total = 0;
};

}  // namespace

struct splotch_nn {
    splotch_nn_config cfg;
    std::vector<Conv> conv;  // enc0a enc0b .. enc(L-1)b, dec(L-2)a dec(L-2)b .. dec0a dec0b, out
    char *pm = nullptr;
    size_t pbytes = 0;
    int32_t step = 0;
    uint64_t seed = 0;
    Acts A;
    int fn = 0, fh = 0, fw = 0;  // shape of the last forward pass
};

namespace {

int enc_a(int l) { return 2 * l; }
int enc_b(int l) { return 2 * l + 1; }
int dec_a(const splotch_nn_config &c, int l) { return 2 * c.n_levels + 2 * (c.n_levels - 2 - l); }
int dec_b(const splotch_nn_config &c, int l) { return dec_a(c, l) + 1; }
int out_layer(const splotch_nn_config &c) { return 4 * c.n_levels - 2; }

bool valid_config(const splotch_nn_config *c) {
    if (!c || c->n_levels < 1 || c->n_levels > SPLOTCH_NN_MAX_LEVELS) return false;
    if (c->in_channels < 32 || c->in_channels % 32 || c->in_channels > 256) return false;
    for (int l = 0; l < c->n_levels; ++l)
        if (c->channels[l] < 32 || c->channels[l] % 32 || c->channels[l] > 256) return false;
    return true;
}

// Layers and their parameter offsets.
size_t build_layers(const splotch_nn_config &c, std::vector<Conv> *out) {
    std::vector<Conv> v;
    const int L = c.n_levels;
    auto add = [&](int cin, int cout, int relu, int level) {
        Conv k;
        memset(&k, 0, sizeof k);
        k.cin = cin;
        k.cout = cout;
        k.relu = relu;
        k.level = level;
        v.push_back(k);
    };
    for (int l = 0; l < L; ++l) {
        add(l == 0 ? c.in_channels : c.channels[l - 1], c.channels[l], 1, l);
        add(c.channels[l], c.channels[l], 1, l);
    }
    for (int l = L - 2; l >= 0; --l) {
        add(c.channels[l + 1] + c.channels[l], c.channels[l], 1, l);
        add(c.channels[l], c.channels[l], 1, l);
    }
    add(c.channels[0], c.in_channels, 0, 0);
    size_t o = 0;
    for (Conv &k : v) {
        const size_t nw = (size_t)9 * k.cin * k.cout, nb = (size_t)k.cout;
        k.w = o;
        o += al(nw * 4);
        k.b = o;
        o += al(nb * 4);
        k.gw = o;
        o += al(nw * 4);
        k.gb = o;
        o += al(nb * 4);
        k.mw = o;
        o += al(nw * 4);
        k.vw = o;
        o += al(nw * 4);
        k.mb = o;
        o += al(nb * 4);
        k.vb = o;
        o += al(nb * 4);
        k.w_bf = o;
        o += al(nw * 2);
        k.wt_bf = o;
        o += al(nw * 2);
        k.wf_bf = o;
        o += al(nw * 2);
    }
    if (out) *out = v;
    return o;
}

int gemm_want(size_t P) {
    size_t want = P / 2048;
    if (want < 1) want = 1;
    if (want > 256) want = 256;
    return (int)want;
}

// Activation and scratch layout for a batch of n images of h x w.
Acts layout_acts(splotch_nn *net, int n, int h, int w) {
    const splotch_nn_config &c = net->cfg;
    const int L = c.n_levels, CI = c.in_channels;
    Acts A;
    A.n = n;
    A.h = h;
    A.w = w;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o += al(bytes ? bytes : 1);
        return at;
    };
    const size_t P0 = (size_t)n * h * w;
    A.x_f = take(P0 * CI * 4);
    A.x_bf = take(P0 * CI * 2);
    A.t_f = take(P0 * CI * 4);
    A.gy = take(P0 * CI * 4);
    A.y = take(P0 * CI * 4);
    A.loss = take(kLossBlocks * 4);
    A.sum = take((size_t)n * 4);
    A.csum = take((size_t)kColsumBlocks * 256 * 4);
    A.pin.assign(L, kNone);
    A.ea.assign(L, kNone);
    A.e.assign(L, kNone);
    A.cat.assign(L, kNone);
    A.da.assign(L, kNone);
    A.dd.assign(L, kNone);
    A.gdn.assign(L, kNone);
    A.ge.assign(L, kNone);
    auto P = [&](int l) { return (size_t)n * (size_t)(h >> l) * (size_t)(w >> l); };
    for (int l = 0; l < L; ++l) {
        if (l > 0) A.pin[l] = take(P(l) * c.channels[l - 1] * 2);
        A.ea[l] = take(P(l) * c.channels[l] * 2);
        A.e[l] = take(P(l) * c.channels[l] * 2);
        A.ge[l] = take(P(l) * c.channels[l] * 4);
    }
    for (int l = L - 2; l >= 0; --l) {
        A.cat[l] = take(P(l) * (c.channels[l + 1] + c.channels[l]) * 2);
        A.da[l] = take(P(l) * c.channels[l] * 2);
        A.dd[l] = take(P(l) * c.channels[l] * 2);
        A.gdn[l] = take(P(l + 1) * c.channels[l + 1] * 4);
    }
    // shared backward scratch: the largest over the layers
    size_t dz = 0, col = 0, colz = 0, gemm = 0;
    for (const Conv &k : net->conv) {
        const size_t p = P(k.level);
        dz = std::max(dz, p * k.cout);
        col = std::max(col, p * 9 * k.cin);
        colz = std::max(colz, p * 9 * k.cout);
        const int s = gemm_splits((int)std::min<size_t>(p, 0x7FFFFFFF), gemm_want(p));
        gemm = std::max(gemm, (size_t)s * 9 * k.cin * k.cout);
    }
    A.dz_bf = take(dz * 2);
    A.dz_f = take(dz * 4);
    A.col = take(col * 2);
    A.colz = take(colz * 2);
    A.gemm = take(gemm * 4);
    // per-layer inputs, outputs and gradients
    for (int l = 0; l < L; ++l) {
        Conv &a = net->conv[enc_a(l)], &b = net->conv[enc_b(l)];
        a.x = l == 0 ? A.x_bf : A.pin[l];
        a.y = A.ea[l];
        b.x = A.ea[l];
        b.y = A.e[l];
        b.dy = A.ge[l];
        a.dy = kNone;  // set below: enc_b's dx
    }
    for (int l = L - 2; l >= 0; --l) {
        Conv &a = net->conv[dec_a(c, l)], &b = net->conv[dec_b(c, l)];
        a.x = A.cat[l];
        a.y = A.da[l];
        b.x = A.da[l];
        b.y = A.dd[l];
    }
    Conv &oc = net->conv[out_layer(c)];
    oc.x = L > 1 ? A.dd[0] : A.e[0];
    oc.y = A.y;
    oc.dy = A.gy;
    for (size_t k = 0; k < net->conv.size(); ++k) {
        Conv &q = net->conv[k];
        const bool first = (int)k == enc_a(0);
        q.dx = first ? kNone : take(P(q.level) * q.cin * 4);
    }
    for (int l = 0; l < L; ++l) net->conv[enc_a(l)].dy = net->conv[enc_b(l)].dx;
    for (int l = 0; l <= L - 2; ++l) {
        net->conv[dec_a(c, l)].dy = net->conv[dec_b(c, l)].dx;
        // dec_b(l) sees the gradient of its output: from the output layer
        // (l = 0) or the decoder level below, after the up-concat adjoint
        net->conv[dec_b(c, l)].dy = l == 0 ? oc.dx : A.gdn[l - 1];
    }
    if (L > 1) net->conv[enc_b(L - 1)].dy = A.gdn[L - 2];
    else net->conv[enc_b(0)].dy = oc.dx;
    A.total = o;
    return A;
}

bool valid_shape(const splotch_nn *net, int n, int h, int w) {
    const int m = 1 << (net->cfg.n_levels - 1);
    // the pixel count is a GEMM dimension (int); every buffer offset is
    // 64-bit
    return n >= 1 && h >= 1 && w >= 1 && h % m == 0 && w % m == 0 &&
           (uint64_t)n * h * w < (1ull << 31);
}

Acts &acts(splotch_nn *net, int n, int h, int w) {
    if (net->A.n != n || net->A.h != h || net->A.w != w) net->A = layout_acts(net, n, h, w);
    return net->A;
}

template <typename T>
T *P_(splotch_nn *net, size_t off) {
    return reinterpret_cast<T *>(net->pm + off);
}
template <typename T>
T *W_(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

#define NN_TRY(expr)                                        \
    do {                                                    \
        if ((expr) != hipSuccess) return SPLOTCH_E_DEVICE;  \
    } while (0)

// BF16 copies (and the fused-convolution transpose) of a layer's weights.
splotch_status refresh_bf16(splotch_nn *net, const Conv &k, hipStream_t s) {
    NN_TRY(f2bf(P_<float>(net, k.w), P_<bf16_t>(net, k.w_bf), (size_t)9 * k.cin * k.cout, s));
    NN_TRY(conv3x3_weights(P_<bf16_t>(net, k.w_bf), P_<bf16_t>(net, k.wf_bf), k.cin, k.cout, s));
    return SPLOTCH_OK;
}

// Seeded normal deviates (splitmix64 bits, Box-Muller) for the weights.
struct Rng {
    uint64_t s;
    uint64_t next() {
        uint64_t z = (s += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    double uniform() { return ((double)(next() >> 11) + 0.5) * (1.0 / 9007199254740992.0); }
    double normal() {
        const double u = uniform(), v = uniform();
        return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
    }
};

splotch_status conv_forward(splotch_nn *net, const Conv &k, void *ws, int n, int hh, int ww,
                            const float *residual, float *out_f, hipStream_t s) {
    bf16_t *out_bf = k.relu ? W_<bf16_t>(ws, k.y) : nullptr;
    NN_TRY(conv3x3(W_<bf16_t>(ws, k.x), P_<bf16_t>(net, k.wf_bf), P_<float>(net, k.b), k.relu,
                   residual, out_bf, out_f, n, hh, ww, k.cin, k.cout, s));
    return SPLOTCH_OK;
}

// Gradients of one convolution: dW, db and (need_dx) the input gradient.
splotch_status conv_backward(splotch_nn *net, const Conv &k, const Acts &A, void *ws, int n,
                             int hh, int ww, const float *dy, bool need_dx, hipStream_t s) {
    const size_t P = (size_t)n * hh * ww;
    bf16_t *dz_bf = W_<bf16_t>(ws, A.dz_bf);
    float *dz_f = W_<float>(ws, A.dz_f);
    NN_TRY(relu_bwd(dy, k.relu ? W_<bf16_t>(ws, k.y) : nullptr, k.relu, dz_bf, dz_f, P * k.cout,
                    s));
    NN_TRY(colsum(dz_f, P, k.cout, P_<float>(net, k.gb), W_<float>(ws, A.csum), s));
    bf16_t *col = W_<bf16_t>(ws, A.col);
    NN_TRY(im2col3x3(W_<bf16_t>(ws, k.x), col, n, hh, ww, k.cin, s));
    const int want = gemm_want(P);
    const int splits = gemm_splits((int)P, want);
    float *cw = W_<float>(ws, A.gemm);
    NN_TRY(gemm(col, dz_bf, cw, 9 * k.cin, k.cout, (int)P, 9 * k.cin, k.cout, 1, want, s));
    NN_TRY(epilogue(cw, splits, (size_t)9 * k.cin * k.cout, k.cout, nullptr, 0, nullptr, nullptr,
                    P_<float>(net, k.gw), s));
    if (!need_dx) return SPLOTCH_OK;
    NN_TRY(flip_weights(P_<bf16_t>(net, k.w_bf), P_<bf16_t>(net, k.wt_bf), k.cout, k.cin, s));
    bf16_t *colz = W_<bf16_t>(ws, A.colz);
    NN_TRY(im2col3x3(dz_bf, colz, n, hh, ww, k.cout, s));
    NN_TRY(gemm(colz, P_<bf16_t>(net, k.wt_bf), W_<float>(ws, k.dx), (int)P, k.cin, 9 * k.cout,
                9 * k.cout, k.cin, 0, 1, s));
    return SPLOTCH_OK;
}

splotch_status run_forward(splotch_nn *net, const float *x_f, const bf16_t *x_bf, int n, int h,
                           int w, float *y, void *ws, size_t ws_bytes, hipStream_t s) {
    if (!valid_shape(net, n, h, w)) return SPLOTCH_E_INVALID_ARG;
    Acts &A = acts(net, n, h, w);
    if (!ws || ws_bytes < A.total) return SPLOTCH_E_WORKSPACE;
    net->fn = n;
    net->fh = h;
    net->fw = w;
    const splotch_nn_config &c = net->cfg;
    const int L = c.n_levels;
    // the caller's input goes where the layout expects it
    if (x_bf != W_<bf16_t>(ws, A.x_bf))
        NN_TRY(hipMemcpyAsync(W_<bf16_t>(ws, A.x_bf), x_bf, (size_t)n * h * w * c.in_channels * 2,
                              hipMemcpyDeviceToDevice, s));
    splotch_status r;
    for (int l = 0; l < L; ++l) {
        const int hh = h >> l, ww = w >> l;
        if (l > 0)
            NN_TRY(pool2(W_<bf16_t>(ws, A.e[l - 1]), W_<bf16_t>(ws, A.pin[l]), n, 2 * hh, 2 * ww,
                         c.channels[l - 1], s));
        if ((r = conv_forward(net, net->conv[enc_a(l)], ws, n, hh, ww, nullptr, nullptr, s)) !=
            SPLOTCH_OK)
            return r;
        if ((r = conv_forward(net, net->conv[enc_b(l)], ws, n, hh, ww, nullptr, nullptr, s)) !=
            SPLOTCH_OK)
            return r;
    }
    size_t d = A.e[L - 1];
    for (int l = L - 2; l >= 0; --l) {
        const int hh = h >> l, ww = w >> l;
        NN_TRY(up2_concat(W_<bf16_t>(ws, d), c.channels[l + 1], W_<bf16_t>(ws, A.e[l]),
                          c.channels[l], W_<bf16_t>(ws, A.cat[l]), n, hh, ww, s));
        if ((r = conv_forward(net, net->conv[dec_a(c, l)], ws, n, hh, ww, nullptr, nullptr, s)) !=
            SPLOTCH_OK)
            return r;
        if ((r = conv_forward(net, net->conv[dec_b(c, l)], ws, n, hh, ww, nullptr, nullptr, s)) !=
            SPLOTCH_OK)
            return r;
        d = A.dd[l];
    }
    float *yo = W_<float>(ws, A.y);
    if ((r = conv_forward(net, net->conv[out_layer(c)], ws, n, h, w, x_f, yo, s)) != SPLOTCH_OK)
        return r;
    if (y && y != yo)
        NN_TRY(hipMemcpyAsync(y, yo, (size_t)n * h * w * c.in_channels * 4,
                              hipMemcpyDeviceToDevice, s));
    return SPLOTCH_OK;
}

splotch_status run_backward(splotch_nn *net, const float *gy, void *ws, size_t ws_bytes,
                            hipStream_t s) {
    if (net->fn == 0) return SPLOTCH_E_INVALID_ARG;  // no forward pass yet
    Acts &A = acts(net, net->fn, net->fh, net->fw);
    if (!ws || ws_bytes < A.total) return SPLOTCH_E_WORKSPACE;
    const splotch_nn_config &c = net->cfg;
    const int L = c.n_levels, n = A.n, h = A.h, w = A.w;
    if (gy != W_<float>(ws, A.gy))
        NN_TRY(hipMemcpyAsync(W_<float>(ws, A.gy), gy, (size_t)n * h * w * c.in_channels * 4,
                              hipMemcpyDeviceToDevice, s));
    splotch_status r;
    const Conv &oc = net->conv[out_layer(c)];
    if ((r = conv_backward(net, oc, A, ws, n, h, w, W_<float>(ws, A.gy), true, s)) != SPLOTCH_OK)
        return r;
    size_t gd = oc.dx;
    for (int l = 0; l <= L - 2; ++l) {
        const int hh = h >> l, ww = w >> l;
        const Conv &b = net->conv[dec_b(c, l)], &a = net->conv[dec_a(c, l)];
        if ((r = conv_backward(net, b, A, ws, n, hh, ww, W_<float>(ws, gd), true, s)) !=
            SPLOTCH_OK)
            return r;
        if ((r = conv_backward(net, a, A, ws, n, hh, ww, W_<float>(ws, b.dx), true, s)) !=
            SPLOTCH_OK)
            return r;
        NN_TRY(up2_concat_bwd(W_<float>(ws, a.dx), c.channels[l + 1], c.channels[l],
                              W_<float>(ws, A.gdn[l]), W_<float>(ws, A.ge[l]), n, hh, ww, s));
        gd = A.gdn[l];
    }
    // the deepest encoder level sees the last decoder gradient directly
    const size_t ge_last = L > 1 ? A.gdn[L - 2] : oc.dx;
    for (int l = L - 1; l >= 0; --l) {
        const int hh = h >> l, ww = w >> l;
        const Conv &b = net->conv[enc_b(l)], &a = net->conv[enc_a(l)];
        const float *gin = W_<float>(ws, l == L - 1 ? ge_last : A.ge[l]);
        if ((r = conv_backward(net, b, A, ws, n, hh, ww, gin, true, s)) != SPLOTCH_OK) return r;
        if ((r = conv_backward(net, a, A, ws, n, hh, ww, W_<float>(ws, b.dx), l > 0, s)) !=
            SPLOTCH_OK)
            return r;
        if (l > 0)
            NN_TRY(pool2_bwd(W_<float>(ws, a.dx), W_<float>(ws, A.ge[l - 1]), n, 2 * hh, 2 * ww,
                             c.channels[l - 1], 1, s));
    }
    return SPLOTCH_OK;
}

// Tone map n planar images into the workspace's NHWC input (scale = the
// mean of each decimated image, summed on the device) and optionally their
// targets with the same scales.
splotch_status tonemap_batch(splotch_nn *net, const Acts &A, void *ws, const float *const *dec,
                             const float *const *full, int n, int h, int w, hipStream_t s) {
    const int CI = net->cfg.in_channels;
    const size_t P = (size_t)h * w;
    const float inv = 1.0f / (float)(3 * P);
    for (int k = 0; k < n; ++k) {
        float *sum = W_<float>(ws, A.sum) + k;
        NN_TRY(colsum(dec[k], 3 * P, 1, sum, W_<float>(ws, A.csum), s));
        NN_TRY(tonemap(dec[k], h, w, 1.0f, CI, W_<float>(ws, A.x_f) + k * P * CI,
                       W_<bf16_t>(ws, A.x_bf) + k * P * CI, s, sum, inv));
        if (full)
            NN_TRY(tonemap(full[k], h, w, 1.0f, CI, W_<float>(ws, A.t_f) + k * P * CI, nullptr, s,
                           sum, inv));
    }
    return SPLOTCH_OK;
}

}  // namespace

extern "C" {

splotch_status splotch_nn_param_bytes(const splotch_nn_config *cfg, size_t *bytes) {
    if (!valid_config(cfg) || !bytes) return SPLOTCH_E_INVALID_ARG;
    *bytes = build_layers(*cfg, nullptr);
    return SPLOTCH_OK;
}

splotch_status splotch_nn_create(const splotch_nn_config *cfg, void *params, size_t params_bytes,
                                 uint64_t seed, void *stream, splotch_nn **out) {
    if (!valid_config(cfg) || !out) return SPLOTCH_E_INVALID_ARG;
    std::vector<Conv> layers;
    const size_t need = build_layers(*cfg, &layers);
    if (!params || params_bytes < need || (reinterpret_cast<uintptr_t>(params) & 255u))
        return SPLOTCH_E_WORKSPACE;
    splotch_nn *net = new splotch_nn();
    net->cfg = *cfg;
    net->conv = layers;
    net->pm = static_cast<char *>(params);
    net->pbytes = need;
    net->seed = seed;
    hipStream_t s = st(stream);
    // He-normal weights (the output layer scaled by 0.1 so the network
    // starts close to the identity on its residual input), zero biases and
    // moments
    Rng rng{seed};
    std::vector<float> host;
    splotch_status r = SPLOTCH_OK;
    for (size_t k = 0; k < layers.size() && r == SPLOTCH_OK; ++k) {
        const Conv &q = layers[k];
        const size_t nw = (size_t)9 * q.cin * q.cout;
        const double gain = (int)k == out_layer(*cfg) ? 0.1 : 1.0;
        const double sd = gain * sqrt(2.0 / (9.0 * q.cin));
        host.resize(nw);
        for (size_t e = 0; e < nw; ++e) host[e] = (float)(rng.normal() * sd);
        if (hipMemcpyAsync(net->pm + q.w, host.data(), nw * 4, hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            r = SPLOTCH_E_DEVICE;
    }
    for (size_t k = 0; k < layers.size() && r == SPLOTCH_OK; ++k) {
        const Conv &q = layers[k];
        const size_t nw = (size_t)9 * q.cin * q.cout;
        float *zero[6] = {P_<float>(net, q.b), P_<float>(net, q.mw), P_<float>(net, q.vw),
                          P_<float>(net, q.mb), P_<float>(net, q.vb), P_<float>(net, q.gb)};
        const size_t cnt[6] = {(size_t)q.cout, nw, nw, (size_t)q.cout, (size_t)q.cout,
                               (size_t)q.cout};
        for (int z = 0; z < 6 && r == SPLOTCH_OK; ++z)
            if (splotch::launch_fill_f32(zero[z], 0.f, cnt[z], s) != hipSuccess) r = SPLOTCH_E_DEVICE;
        if (r == SPLOTCH_OK) r = refresh_bf16(net, q, s);
    }
    if (r != SPLOTCH_OK) {
        delete net;
        return r;
    }
    *out = net;
    return SPLOTCH_OK;
}

splotch_status splotch_nn_destroy(splotch_nn *net) {
    delete net;
    return SPLOTCH_OK;
}

int32_t splotch_nn_n_layers(const splotch_nn *net) { return net ? (int32_t)net->conv.size() : 0; }

splotch_status splotch_nn_workspace_bytes(splotch_nn *net, int32_t n, int32_t h, int32_t w,
                                          size_t *bytes) {
    if (!net || !bytes || !valid_shape(net, n, h, w)) return SPLOTCH_E_INVALID_ARG;
    *bytes = acts(net, n, h, w).total;
    return SPLOTCH_OK;
}

splotch_status splotch_nn_layer_info(splotch_nn *net, int32_t k, int32_t n, int32_t h, int32_t w,
                                     splotch_nn_layer *out) {
    if (!net || !out || k < 0 || k >= (int32_t)net->conv.size() || !valid_shape(net, n, h, w))
        return SPLOTCH_E_INVALID_ARG;
    acts(net, n, h, w);
    const Conv &q = net->conv[(size_t)k];
    out->cin = q.cin;
    out->cout = q.cout;
    out->relu = q.relu;
    out->level = q.level;
    out->w = q.w;
    out->b = q.b;
    out->gw = q.gw;
    out->gb = q.gb;
    out->w_bf16 = q.w_bf;
    out->x = q.x;
    out->y = q.y;
    out->dy = q.dy;
    out->dx = q.dx;
    return SPLOTCH_OK;
}

splotch_status splotch_nn_forward(splotch_nn *net, const float *x_f32, const uint16_t *x_bf16,
                                  int32_t n, int32_t h, int32_t w, float *y, void *workspace,
                                  size_t workspace_bytes, void *stream) {
    if (!net || !x_f32 || !x_bf16) return SPLOTCH_E_INVALID_ARG;
    return run_forward(net, x_f32, x_bf16, n, h, w, y, workspace, workspace_bytes, st(stream));
}

splotch_status splotch_nn_loss_grad(splotch_nn *net, const float *y, const float *target,
                                    int32_t n, int32_t h, int32_t w, float *grad,
                                    float *loss_partials, void *stream) {
    if (!net || !y || !target || !grad || !loss_partials || !valid_shape(net, n, h, w))
        return SPLOTCH_E_INVALID_ARG;
    NN_TRY(mse(y, target, grad, (size_t)n * h * w, net->cfg.in_channels, 3, loss_partials,
               kLossBlocks, st(stream)));
    return SPLOTCH_OK;
}

splotch_status splotch_nn_backward(splotch_nn *net, const float *grad_y, void *workspace,
                                   size_t workspace_bytes, void *stream) {
    if (!net || !grad_y) return SPLOTCH_E_INVALID_ARG;
    return run_backward(net, grad_y, workspace, workspace_bytes, st(stream));
}

splotch_status splotch_nn_adam_step(splotch_nn *net, float lr, void *stream) {
    if (!net || !(lr > 0.f)) return SPLOTCH_E_INVALID_ARG;
    hipStream_t s = st(stream);
    ++net->step;
    for (const Conv &q : net->conv) {
        const size_t nw = (size_t)9 * q.cin * q.cout;
        NN_TRY(adam(P_<float>(net, q.w), P_<bf16_t>(net, q.w_bf), P_<float>(net, q.gw),
                    P_<float>(net, q.mw), P_<float>(net, q.vw), nw, lr, 0.9f, 0.999f, 1e-8f,
                    net->step, s));
        NN_TRY(adam(P_<float>(net, q.b), nullptr, P_<float>(net, q.gb), P_<float>(net, q.mb),
                    P_<float>(net, q.vb), (size_t)q.cout, lr, 0.9f, 0.999f, 1e-8f, net->step, s));
        NN_TRY(conv3x3_weights(P_<bf16_t>(net, q.w_bf), P_<bf16_t>(net, q.wf_bf), q.cin, q.cout,
                               s));
    }
    return SPLOTCH_OK;
}

int32_t splotch_nn_get_step(const splotch_nn *net) { return net ? net->step : -1; }

splotch_status splotch_nn_save(const splotch_nn *net, const char *path, void *stream) {
    if (!net || !path) return SPLOTCH_E_INVALID_ARG;
    hipStream_t s = st(stream);
    FILE *f = fopen(path, "wb");
    if (!f) return SPLOTCH_E_INVALID_ARG;
    bool okw = fwrite(kMagic, 4, 2, f) == 2 && fwrite(&net->cfg, sizeof net->cfg, 1, f) == 1 &&
               fwrite(&net->step, 4, 1, f) == 1 && fwrite(&net->seed, 8, 1, f) == 1;
    std::vector<float> host;
    splotch_status r = SPLOTCH_OK;
    for (const Conv &q : net->conv) {
        if (!okw) break;
        const size_t nw = (size_t)9 * q.cin * q.cout, nb = (size_t)q.cout;
        const size_t offs[6] = {q.w, q.b, q.mw, q.vw, q.mb, q.vb};
        const size_t cnt[6] = {nw, nb, nw, nw, nb, nb};
        for (int z = 0; z < 6 && okw; ++z) {
            host.resize(cnt[z]);
            if (hipMemcpyAsync(host.data(), net->pm + offs[z], cnt[z] * 4, hipMemcpyDeviceToHost,
                               s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                r = SPLOTCH_E_DEVICE;
                okw = false;
                break;
            }
            okw = fwrite(host.data(), 4, cnt[z], f) == cnt[z];
        }
    }
    if (fclose(f) != 0) okw = false;
    if (r != SPLOTCH_OK) return r;
    return okw ? SPLOTCH_OK : SPLOTCH_E_INVALID_ARG;
}

splotch_status splotch_nn_load(splotch_nn *net, const char *path, void *stream) {
    if (!net || !path) return SPLOTCH_E_INVALID_ARG;
    hipStream_t s = st(stream);
    FILE *f = fopen(path, "rb");
    if (!f) return SPLOTCH_E_INVALID_ARG;
    uint32_t magic[2];
    splotch_nn_config cfg;
    int32_t step;
    uint64_t seed;
    bool okr = fread(magic, 4, 2, f) == 2 && magic[0] == kMagic[0] && magic[1] == kMagic[1] &&
               fread(&cfg, sizeof cfg, 1, f) == 1 && fread(&step, 4, 1, f) == 1 &&
               fread(&seed, 8, 1, f) == 1;
    // the checkpoint must describe this network
    okr = okr && memcmp(&cfg, &net->cfg, sizeof cfg) == 0 && step >= 0;
    std::vector<std::vector<float>> blocks;
    for (const Conv &q : net->conv) {
        if (!okr) break;
        const size_t nw = (size_t)9 * q.cin * q.cout, nb = (size_t)q.cout;
        const size_t cnt[6] = {nw, nb, nw, nw, nb, nb};
        for (int z = 0; z < 6 && okr; ++z) {
            blocks.emplace_back(cnt[z]);
            okr = fread(blocks.back().data(), 4, cnt[z], f) == cnt[z];
        }
    }
    fclose(f);
    if (!okr) return SPLOTCH_E_INVALID_ARG;
    size_t bi = 0;
    for (const Conv &q : net->conv) {
        const size_t offs[6] = {q.w, q.b, q.mw, q.vw, q.mb, q.vb};
        for (int z = 0; z < 6; ++z, ++bi)
            NN_TRY(hipMemcpyAsync(net->pm + offs[z], blocks[bi].data(), blocks[bi].size() * 4,
                                  hipMemcpyHostToDevice, s));
        NN_TRY(hipStreamSynchronize(s));
        splotch_status r = refresh_bf16(net, q, s);
        if (r != SPLOTCH_OK) return r;
    }
    net->step = step;
    net->seed = seed;
    return SPLOTCH_OK;
}

splotch_status splotch_nn_reconstruct(splotch_nn *net, const float *dec_img, int32_t h, int32_t w,
                                      float *out_img, void *workspace, size_t workspace_bytes,
                                      void *stream) {
    if (!net || !dec_img || !out_img || !valid_shape(net, 1, h, w)) return SPLOTCH_E_INVALID_ARG;
    hipStream_t s = st(stream);
    Acts &A = acts(net, 1, h, w);
    if (!workspace || workspace_bytes < A.total) return SPLOTCH_E_WORKSPACE;
    const float *dec[1] = {dec_img};
    splotch_status r = tonemap_batch(net, A, workspace, dec, nullptr, 1, h, w, s);
    if (r != SPLOTCH_OK) return r;
    if ((r = run_forward(net, W_<float>(workspace, A.x_f), W_<bf16_t>(workspace, A.x_bf), 1, h, w,
                         nullptr, workspace, workspace_bytes, s)) != SPLOTCH_OK)
        return r;
    NN_TRY(untonemap(W_<float>(workspace, A.y), h, w, 1.0f, net->cfg.in_channels, out_img, s,
                     W_<float>(workspace, A.sum), 1.0f / (float)(3 * (size_t)h * w)));
    return SPLOTCH_OK;
}

splotch_status splotch_nn_train_step(splotch_nn *net, const float *const *dec_imgs,
                                     const float *const *full_imgs, int32_t n, int32_t h,
                                     int32_t w, float lr, float *loss_partials, void *workspace,
                                     size_t workspace_bytes, void *stream) {
    if (!net || !dec_imgs || !full_imgs || !valid_shape(net, n, h, w) || !(lr > 0.f))
        return SPLOTCH_E_INVALID_ARG;
    for (int k = 0; k < n; ++k)
        if (!dec_imgs[k] || !full_imgs[k]) return SPLOTCH_E_INVALID_ARG;
    hipStream_t s = st(stream);
    Acts &A = acts(net, n, h, w);
    if (!workspace || workspace_bytes < A.total) return SPLOTCH_E_WORKSPACE;
    splotch_status r = tonemap_batch(net, A, workspace, dec_imgs, full_imgs, n, h, w, s);
    if (r != SPLOTCH_OK) return r;
    if ((r = run_forward(net, W_<float>(workspace, A.x_f), W_<bf16_t>(workspace, A.x_bf), n, h, w,
                         nullptr, workspace, workspace_bytes, s)) != SPLOTCH_OK)
        return r;
    float *loss = loss_partials ? loss_partials : W_<float>(workspace, A.loss);
    NN_TRY(mse(W_<float>(workspace, A.y), W_<float>(workspace, A.t_f), W_<float>(workspace, A.gy),
               (size_t)n * h * w, net->cfg.in_channels, 3, loss, kLossBlocks, s));
    if ((r = run_backward(net, W_<float>(workspace, A.gy), workspace, workspace_bytes, s)) !=
        SPLOTCH_OK)
        return r;
    return splotch_nn_adam_step(net, lr, stream);
}

}  // extern "C"
