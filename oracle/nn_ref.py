"""FP64 reference of the reconstruction network -- TEST INFRASTRUCTURE ONLY.

Plain numpy definitions of what the network computes, used to check the
HIP kernels: 3x3 "same" convolution with zero padding, ReLU, 2x2 average
pooling, nearest 2x upsampling with channel concatenation, mean squared
error and the Adam update, each with its adjoint written out by hand.
Activations are NHWC float64; a convolution's weights are
W[tap][ci][co] with taps (ky, kx) row-major, i.e. the output is
  y[n, y, x, co] = b[co] + sum_{ky,kx,ci} x[n, y+ky-1, x+kx-1, ci] W[3ky+kx, ci, co].
`bf16` reproduces bfloat16 rounding (nearest even) so the reference can see
exactly the BF16 operands the GPU sees.  The manual adjoints are pinned by
central finite differences (tests/test_nn_reference.py).
"""
from __future__ import annotations

import numpy as np


def bf16(a):
    """Round float values to bfloat16 (nearest even), returned as float64."""
    f = np.asarray(a, np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def conv3x3(x, W, b):
    n, h, w, ci = x.shape
    co = W.shape[2]
    xp = np.zeros((n, h + 2, w + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((n, h, w, co))
    for ky in range(3):
        for kx in range(3):
            y += xp[:, ky:ky + h, kx:kx + w, :] @ W[3 * ky + kx]
    return y + (0 if b is None else b)


def conv3x3_adjoint(x, W, dz):
    """Gradients of sum(dz * conv3x3(x, W, b)) with respect to x, W, b."""
    n, h, w, ci = x.shape
    xp = np.zeros((n, h + 2, w + 2, ci))
    xp[:, 1:-1, 1:-1] = x
    dW = np.zeros_like(W)
    dxp = np.zeros_like(xp)
    for ky in range(3):
        for kx in range(3):
            t = 3 * ky + kx
            patch = xp[:, ky:ky + h, kx:kx + w, :]
            dW[t] = patch.reshape(-1, ci).T @ dz.reshape(-1, dz.shape[-1])
            dxp[:, ky:ky + h, kx:kx + w, :] += dz @ W[t].T
    db = dz.reshape(-1, dz.shape[-1]).sum(axis=0)
    return dxp[:, 1:-1, 1:-1], dW, db


def pool2(x):
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).mean(axis=(2, 4))


def pool2_adjoint(dy):
    return 0.25 * np.repeat(np.repeat(dy, 2, axis=1), 2, axis=2)


def up2_concat(a, s):
    up = np.repeat(np.repeat(a, 2, axis=1), 2, axis=2)
    return np.concatenate([up, s], axis=-1)


def up2_concat_adjoint(dout, ca):
    n, h, w, _ = dout.shape
    da = dout[..., :ca].reshape(n, h // 2, 2, w // 2, 2, ca).sum(axis=(2, 4))
    return da, dout[..., ca:]


def mse(pred, target, used):
    d = pred[..., :used] - target[..., :used]
    g = np.zeros_like(pred)
    g[..., :used] = 2.0 * d / d.size
    return float((d * d).mean()), g


def adam(w, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    w = w - lr * (m / (1 - b1 ** step)) / (np.sqrt(v / (1 - b2 ** step)) + eps)
    return w, m, v


class UNetRef:
    """The encoder-decoder of the learned path in float64.  With
    round_bf16=True every tensor the GPU stores or feeds to a GEMM in
    bfloat16 (weights, activations, the masked output gradients) is rounded
    the same way, so only accumulation order differs from the GPU."""

    def __init__(self, levels, weights, cin=32, round_bf16=True):
        # weights: list of (W [9, ci, co], b [co]) in the order
        # enc0a, enc0b, ..., enc{L-1}b, dec{L-2}a, dec{L-2}b, ..., dec0a, dec0b, out
        self.levels = levels
        self.cin = cin
        self.r = bf16 if round_bf16 else (lambda a: np.asarray(a, np.float64))
        self.W = [(np.asarray(W, np.float64), np.asarray(b, np.float64)) for W, b in weights]

    def _layers(self):
        L = len(self.levels)
        enc = [(2 * l, 2 * l + 1) for l in range(L)]
        dec = {}
        k = 2 * L
        for l in range(L - 2, -1, -1):
            dec[l] = (k, k + 1)
            k += 2
        return enc, dec, k

    def forward(self, x):
        r = self.r
        L = len(self.levels)
        enc, dec, out_k = self._layers()
        self.cache = {}

        def conv(k, inp, relu):
            W, b = self.W[k]
            z = conv3x3(inp, r(W), b)
            y = np.maximum(z, 0) if relu else z
            self.cache[k] = (inp, y if relu else None)
            return y

        xb = r(x)
        e = []
        inp = xb
        for l in range(L):
            if l > 0:
                inp = r(pool2(e[l - 1]))
            a = r(conv(enc[l][0], inp, True))
            e.append(r(conv(enc[l][1], a, True)))
        d = e[L - 1]
        for l in range(L - 2, -1, -1):
            cat = up2_concat(d, e[l])
            a = r(conv(dec[l][0], cat, True))
            d = r(conv(dec[l][1], a, True))
        y = conv(out_k, d, False) + x
        self.shapes = [ei.shape for ei in e]
        return y

    def backward(self, gy):
        """Returns the list of (dW, db) in the layer order of __init__."""
        r = self.r
        L = len(self.levels)
        enc, dec, out_k = self._layers()
        grads = [None] * (out_k + 1)

        def conv_b(k, g, relu, need_dx=True):
            inp, y = self.cache[k]
            dz = r(g * (y > 0)) if relu else r(g)
            W, _ = self.W[k]
            dx, dW, db = conv3x3_adjoint(inp, r(W), dz)
            grads[k] = (dW, db)
            return dx

        gd = conv_b(out_k, gy, False)
        ge = [None] * L
        for l in range(L - 1):
            g = conv_b(dec[l][1], gd, True)
            g = conv_b(dec[l][0], g, True)
            gd, ge[l] = up2_concat_adjoint(g, self.levels[l + 1])
        ge[L - 1] = gd
        for l in range(L - 1, -1, -1):
            g = conv_b(enc[l][1], ge[l], True)
            g = conv_b(enc[l][0], g, True)
            if l > 0:
                ge[l - 1] = ge[l - 1] + pool2_adjoint(g)
        return grads
