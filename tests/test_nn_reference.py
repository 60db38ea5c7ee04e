"""Pins of the FP64 network reference (oracle/nn_ref.py): the convolution
against scipy's correlation, every hand-written adjoint against central
finite differences, and the Adam step against its textbook closed form
on a constant gradient."""
import numpy as np
import pytest
from scipy import signal

from oracle import nn_ref as R


def test_conv_matches_scipy_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 7, 9, 3))
    W = rng.standard_normal((9, 3, 4))
    b = rng.standard_normal(4)
    y = R.conv3x3(x, W, b)
    for n in range(2):
        for co in range(4):
            ref = b[co] + sum(signal.correlate2d(x[n, :, :, ci], W[:, ci, co].reshape(3, 3),
                                                 mode="same", boundary="fill")
                              for ci in range(3))
            assert np.allclose(y[n, :, :, co], ref, atol=1e-12)


def _fd(f, a, idx, eps=1e-6):
    a1, a2 = a.copy(), a.copy()
    a1[idx] += eps
    a2[idx] -= eps
    return (f(a1) - f(a2)) / (2 * eps)


def test_conv_adjoint_finite_differences():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((1, 5, 6, 3))
    W = rng.standard_normal((9, 3, 2))
    b = rng.standard_normal(2)
    dz = rng.standard_normal((1, 5, 6, 2))
    dx, dW, db = R.conv3x3_adjoint(x, W, dz)
    for idx in [(0, 0, 0, 0), (0, 4, 5, 2), (0, 2, 3, 1)]:
        assert dx[idx] == pytest.approx(_fd(lambda a: (R.conv3x3(a, W, b) * dz).sum(), x, idx), rel=1e-6)
    for idx in [(0, 0, 0), (4, 2, 1), (8, 1, 0)]:
        assert dW[idx] == pytest.approx(_fd(lambda a: (R.conv3x3(x, a, b) * dz).sum(), W, idx), rel=1e-6)
    assert db[1] == pytest.approx(_fd(lambda a: (R.conv3x3(x, W, a) * dz).sum(), b, (1,)), rel=1e-6)


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((1, 4, 6, 3))
    dy = rng.standard_normal((1, 2, 3, 3))
    g = R.pool2_adjoint(dy)
    for idx in [(0, 0, 0, 0), (0, 3, 5, 2)]:
        assert g[idx] == pytest.approx(_fd(lambda a: (R.pool2(a) * dy).sum(), x, idx), rel=1e-7)
    a = rng.standard_normal((1, 2, 3, 2))
    s = rng.standard_normal((1, 4, 6, 3))
    dout = rng.standard_normal((1, 4, 6, 5))
    da, ds = R.up2_concat_adjoint(dout, 2)
    assert da[0, 1, 2, 1] == pytest.approx(
        _fd(lambda t: (R.up2_concat(t, s) * dout).sum(), a, (0, 1, 2, 1)), rel=1e-7)
    assert ds[0, 3, 4, 2] == pytest.approx(
        _fd(lambda t: (R.up2_concat(a, t) * dout).sum(), s, (0, 3, 4, 2)), rel=1e-7)


def test_mse_gradient():
    rng = np.random.default_rng(3)
    p = rng.standard_normal((10, 4))
    t = rng.standard_normal((10, 4))
    _, g = R.mse(p, t, 3)
    assert np.all(g[:, 3] == 0)
    assert g[4, 1] == pytest.approx(_fd(lambda a: R.mse(a, t, 3)[0], p, (4, 1)), rel=1e-6)


def test_unet_reference_backward_finite_differences():
    rng = np.random.default_rng(4)
    levels = (4, 6, 8)
    cin = 3
    shapes = []
    L = len(levels)
    for l in range(L):
        ci = cin if l == 0 else levels[l - 1]
        shapes += [(ci, levels[l]), (levels[l], levels[l])]
    for l in range(L - 2, -1, -1):
        shapes += [(levels[l + 1] + levels[l], levels[l]), (levels[l], levels[l])]
    shapes.append((levels[0], cin))
    weights = [(rng.standard_normal((9, a, b)) * np.sqrt(2 / (9 * a)), rng.standard_normal(b) * 0.1)
               for a, b in shapes]
    x = rng.standard_normal((1, 8, 8, cin))
    t = rng.standard_normal((1, 8, 8, cin))

    def loss(ws):
        net = R.UNetRef(levels, ws, cin=cin, round_bf16=False)
        return R.mse(net.forward(x), t, cin)[0]

    net = R.UNetRef(levels, weights, cin=cin, round_bf16=False)
    _, g = R.mse(net.forward(x), t, cin)
    grads = net.backward(g)
    for k in (0, 3, 5, 7, len(weights) - 1):
        W, b = weights[k]
        idx = tuple(rng.integers(0, s) for s in W.shape)

        def f(Wk, k=k):
            ws = list(weights)
            ws[k] = (Wk, weights[k][1])
            return loss(ws)
        assert grads[k][0][idx] == pytest.approx(_fd(f, W, idx), rel=1e-5, abs=1e-10), k


def test_adam_closed_form_constant_gradient():
    """With a constant gradient g the bias-corrected moments are exactly g
    and g^2, so every step moves w by -lr * g/(|g| + eps)."""
    w = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -0.1, 2.0])
    m = np.zeros(3)
    v = np.zeros(3)
    for step in range(1, 6):
        w_new, m, v = R.adam(w, g, m, v, step, lr=0.01)
        assert np.allclose(w_new - w, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-9)
        w = w_new


def test_bf16_rounding():
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -3.140625, 1e-3], np.float32)
    r = R.bf16(vals)
    assert r[0] == 1.0 and r[1] == 1.0          # tie to even
    assert r[2] == 1.0 + 2 ** -7                # rounds up
    assert r[3] == -3.140625                    # exactly representable
    assert abs(r[4] - 1e-3) / 1e-3 < 2 ** -8
