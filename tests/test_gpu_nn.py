"""GPU checks of the reconstruction network's kernels against the FP64
reference (oracle/nn_ref.py) on the same BF16-rounded operands, and of
what the trained network gains over the decimated render alone."""
import math

import numpy as np
import pytest

from oracle import nn_ref as R
from paper_1004_1302_amd import binding as B
from paper_1004_1302_amd import learned as LN
from paper_1004_1302_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as T
    assert T.cuda.is_available()
    return T


def to_bf16_bits(torch, a):
    r = R.bf16(a).astype(np.float32)
    return torch.from_numpy(r.view(np.uint32).astype(np.uint32) >> 16).to(torch.int32) \
        .to(torch.int16).cuda(), r.astype(np.float64)


def bits_to_f64(t):
    u = t.cpu().numpy().astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


@pytest.mark.parametrize("M,N,K,trans,splits", [
    (64, 32, 32, 0, 1), (100, 48, 70, 0, 1), (256, 64, 288, 0, 1), (96, 64, 1000, 1, 7),
    (576, 32, 4096, 1, 4), (37, 17, 33, 1, 1)])
def test_gemm_bf16_mfma(torch, M, N, K, trans, splits):
    """Checks the matrix-core fragment layout and the split-K partials."""
    ops = LN.Ops()
    rng = np.random.default_rng(M + N + K)
    a = rng.standard_normal((K, M) if trans else (M, K))
    b = rng.standard_normal((K, N))
    A, a64 = to_bf16_bits(torch, a)
    Bt, b64 = to_bf16_bits(torch, b)
    s = ops.splits(K, splits)
    C = torch.empty(s * M * N, dtype=torch.float32, device="cuda")
    lda = M if trans else K
    ops.gemm(A, Bt, C, M, N, K, lda, N, trans, splits)
    out = torch.empty(M * N, dtype=torch.float32, device="cuda")
    ops.epilogue(C, s, M, N, None, 0, None, None, out)
    torch.cuda.synchronize()
    ref = (a64.T if trans else a64) @ b64
    got = out.cpu().numpy().reshape(M, N)
    assert np.allclose(got, ref, rtol=1e-5, atol=1e-4 * np.abs(ref).max())


@pytest.mark.parametrize("n,h,w,ci,co,relu,res", [
    (1, 13, 21, 32, 32, True, False), (2, 16, 24, 96, 128, True, False),
    (1, 9, 40, 64, 32, False, True), (1, 32, 32, 256, 128, True, False),
    (3, 8, 16, 32, 64, True, True)])
def test_fused_conv3x3(torch, n, h, w, ci, co, relu, res):
    """The fused convolution (halo tile and weights in LDS, implicit GEMM on
    the matrix cores) against the FP64 reference on the same BF16 operands,
    and against im2col + GEMM + epilogue: ragged tiles, several images,
    several 32-channel slices, both channel groupings, residual input."""
    rng = np.random.default_rng(ci + co + h)
    ops = LN.Ops()
    P = n * h * w
    xb, x64 = to_bf16_bits(torch, rng.standard_normal((P, ci)))
    wb, w64 = to_bf16_bits(torch, rng.standard_normal((9 * ci, co)) * math.sqrt(2.0 / (9 * ci)))
    b = rng.standard_normal(co).astype(np.float32) * 0.1
    bt = torch.from_numpy(b).cuda()
    r = rng.standard_normal((P, co)).astype(np.float32) if res else None
    rt = torch.from_numpy(r).cuda() if res else None
    wf = torch.empty((co, 9 * ci), dtype=torch.int16, device="cuda")
    ops.conv_weights(wb, wf, ci, co)
    out_f = torch.full((P, co), float("nan"), dtype=torch.float32, device="cuda")
    out_b = torch.zeros((P, co), dtype=torch.int16, device="cuda")
    ops.conv3x3(xb, wf, bt, relu, rt, out_b, out_f, n, h, w, ci, co)
    col = torch.empty((P, 9 * ci), dtype=torch.int16, device="cuda")
    ops.im2col(xb, col, n, h, w, ci)
    cb = torch.empty((P, co), dtype=torch.float32, device="cuda")
    ops.gemm(col, wb, cb, P, co, 9 * ci, 9 * ci, co, 0, 1)
    ref_f = torch.empty((P, co), dtype=torch.float32, device="cuda")
    ops.epilogue(cb, 1, P, co, bt, relu, rt, None, ref_f)
    torch.cuda.synchronize()
    z = R.conv3x3(x64.reshape(n, h, w, ci), w64.reshape(9, ci, co), b.astype(np.float64))
    if relu:
        z = np.maximum(z, 0)
    if res:
        z = z + r.reshape(n, h, w, co)
    got = out_f.cpu().numpy().reshape(n, h, w, co)
    scale = np.abs(z).max()
    assert np.abs(got - z).max() <= 1e-5 * scale
    assert np.abs(got - ref_f.cpu().numpy().reshape(n, h, w, co)).max() <= 1e-5 * scale
    gb = bits_to_f64(out_b).reshape(n, h, w, co)
    assert np.array_equal(gb, R.bf16(got.astype(np.float64)))


def test_pool_and_upsample_concat_exact(torch):
    """The 2x2 average pool (FP32 sum in a fixed order, one rounding to
    BF16) and the nearest upsample + channel concat (a copy) are exact."""
    rng = np.random.default_rng(21)
    ops = LN.Ops()
    n, h, w, c = 2, 6, 10, 40
    xb, x64 = to_bf16_bits(torch, rng.standard_normal((n * h * w, c)))
    out = torch.empty((n * (h // 2) * (w // 2), c), dtype=torch.int16, device="cuda")
    ops.pool2(xb, out, n, h, w, c)
    x = x64.reshape(n, h, w, c).astype(np.float32)
    sm = ((x[:, 0::2, 0::2] + x[:, 0::2, 1::2]) + x[:, 1::2, 0::2]) + x[:, 1::2, 1::2]
    ref = R.bf16((np.float32(0.25) * sm).astype(np.float64))
    assert np.array_equal(bits_to_f64(out).reshape(ref.shape), ref)
    ca, cs = 24, 40
    ab, a64 = to_bf16_bits(torch, rng.standard_normal((n * (h // 2) * (w // 2), ca)))
    sb, s64 = to_bf16_bits(torch, rng.standard_normal((n * h * w, cs)))
    cat = torch.empty((n * h * w, ca + cs), dtype=torch.int16, device="cuda")
    ops.up2_concat(ab, ca, sb, cs, cat, n, h, w)
    up = np.repeat(np.repeat(a64.reshape(n, h // 2, w // 2, ca), 2, 1), 2, 2)
    ref = np.concatenate([up, s64.reshape(n, h, w, cs)], axis=3)
    assert np.array_equal(bits_to_f64(cat).reshape(ref.shape), ref)


def test_conv_layer_forward_backward(torch):
    rng = np.random.default_rng(5)
    n, h, w, ci, co = 2, 16, 24, 32, 64
    layer = LN.Conv3x3(ci, co, True, rng, "cuda")
    layer.b.copy_(torch.from_numpy(rng.standard_normal(co).astype(np.float32) * 0.1))
    x = rng.standard_normal((n, h, w, ci))
    xb, x64 = to_bf16_bits(torch, x.reshape(-1, ci))
    sc = LN.Scratch("cuda")
    y = torch.empty(n * h * w * co, dtype=torch.int16, device="cuda")
    layer.forward(xb, n, h, w, y, sc, "t")
    W64 = bits_to_f64(layer.w_bf).reshape(9, ci, co)
    b64 = layer.b.cpu().numpy().astype(np.float64)
    z = R.conv3x3(x64.reshape(n, h, w, ci), W64, b64)
    yref = np.maximum(z, 0)
    got = bits_to_f64(y).reshape(n, h, w, co)
    assert np.allclose(got, R.bf16(yref), rtol=2 ** -7, atol=1e-3 * np.abs(yref).max())
    dy = rng.standard_normal((n * h * w, co)).astype(np.float32)
    dy_t = torch.from_numpy(dy).cuda()
    dx = layer.backward(xb, y, dy_t, n, h, w, sc, True)
    torch.cuda.synchronize()
    yg = got
    dz = R.bf16(dy.reshape(n, h, w, co) * (yg > 0))
    dx_r, dW_r, db_r = R.conv3x3_adjoint(x64.reshape(n, h, w, ci), W64, dz)
    gw = layer.gw.cpu().numpy().reshape(9, ci, co)
    assert np.allclose(gw, dW_r, rtol=1e-4, atol=1e-4 * np.abs(dW_r).max())
    gb = layer.gb.cpu().numpy()
    db_exact = (dy.reshape(-1, co) * (yg.reshape(-1, co) > 0)).sum(0)
    assert np.allclose(gb, db_exact, rtol=1e-4, atol=1e-4 * np.abs(db_exact).max())
    assert np.allclose(dx.cpu().numpy().reshape(n, h, w, ci), dx_r, rtol=1e-4,
                       atol=1e-4 * np.abs(dx_r).max())


def _net_weights_for_ref(net):
    out = []
    for c in net.layers():
        out.append((bits_to_f64(c.w_bf).reshape(9, c.cin, c.cout), c.b.cpu().numpy().astype(np.float64)))
    return out


def test_unet_gradients_against_reference(torch):
    """Whole-network forward and backward on the GPU against the FP64
    reference fed the same BF16 weights and rounding points."""
    levels = (32, 32, 64)
    net = LN.UNet(seed=3, levels=levels)
    rng = np.random.default_rng(6)
    for c in net.layers():
        c.b.copy_(torch.from_numpy(rng.standard_normal(c.cout).astype(np.float32) * 0.05))
    n, h, w = 1, 16, 16
    x = np.zeros((n * h * w, LN.CIN))
    x[:, :3] = rng.uniform(0, 2, (n * h * w, 3))
    t = x.copy()
    t[:, :3] += rng.normal(0, 0.2, (n * h * w, 3))
    x_f = torch.from_numpy(x.astype(np.float32)).cuda()
    x_bf, x64 = to_bf16_bits(torch, x)
    t_f = torch.from_numpy(t.astype(np.float32)).cuda()
    y = net.forward(x_f, x_bf, n, h, w)
    gy = torch.empty_like(y)
    part = torch.empty(256, dtype=torch.float32, device="cuda")
    ops = LN.Ops()
    ops.mse(y, t_f, gy, n * h * w, LN.CIN, 3, part, 256)
    net.backward(gy)
    torch.cuda.synchronize()
    ref = R.UNetRef(levels, _net_weights_for_ref(net), cin=LN.CIN, round_bf16=True)
    yr = ref.forward(x.reshape(n, h, w, LN.CIN).astype(np.float32).astype(np.float64))
    yg = y.cpu().numpy().reshape(n, h, w, LN.CIN)
    assert np.abs(yg - yr).max() <= 2e-2 * np.abs(yr).max()
    _, gr = R.mse(yr, t.reshape(n, h, w, LN.CIN), 3)
    grads = ref.backward(gr.astype(np.float32).astype(np.float64))
    for k, c in enumerate(net.layers()):
        gw = c.gw.cpu().numpy().reshape(9, c.cin, c.cout)
        rel = np.linalg.norm(gw - grads[k][0]) / max(np.linalg.norm(grads[k][0]), 1e-30)
        assert rel < 3e-2, (k, rel)
        gb = c.gb.cpu().numpy()
        relb = np.linalg.norm(gb - grads[k][1]) / max(np.linalg.norm(grads[k][1]), 1e-30)
        assert relb < 3e-2, (k, relb)


def test_adam_kernel(torch):
    ops = LN.Ops()
    rng = np.random.default_rng(8)
    w = rng.standard_normal(1000)
    m = np.zeros(1000)
    v = np.zeros(1000)
    tw = torch.from_numpy(w.astype(np.float32)).cuda()
    tm = torch.zeros(1000, device="cuda")
    tv = torch.zeros(1000, device="cuda")
    for step in range(1, 4):
        g = rng.standard_normal(1000)
        tg = torch.from_numpy(g.astype(np.float32)).cuda()
        ops.adam(tw, None, tg, tm, tv, 1000, 1e-2, 0.9, 0.999, 1e-8, step)
        w, m, v = R.adam(w, g.astype(np.float32).astype(np.float64), m, v, step, 1e-2)
    torch.cuda.synchronize()
    assert np.allclose(tw.cpu().numpy(), w, rtol=1e-5, atol=1e-6)


def _pairs(torch, n_pairs, size, seed):
    sc = synth.plummer_mix(400_000, seed=seed, h_mean=0.004)
    parts, pal = B.scene_to_device(sc)
    dec = LN.decimate(parts, seed=seed + 1)
    cams = synth.orbit_cameras(n_pairs, seed + 2, [(size, size)])
    out = []
    for cam in cams:
        full = B.render(parts, cam, pal, sc.species_params, compensated=True)
        d = B.render(dec, cam, pal, sc.species_params, compensated=True)
        out.append((d.clone(), full.clone()))
    return out, parts, dec, pal, sc, cams


def test_training_gains_over_decimated_render(torch):
    """A short training run on renderer-made pairs: the network's output is
    closer to the full render than the decimated render is (tone-mapped
    PSNR on held-out views)."""
    pairs, parts, dec, pal, sc, cams = _pairs(torch, 40, 128, 11)
    train, test = pairs[:32], pairs[32:]
    net = LN.UNet(seed=0)
    rec = LN.Reconstructor(net)
    for it in range(240):
        k = (it * 4) % len(train)
        batch = train[k:k + 4]
        rec.train_step([d for d, _ in batch], [f for _, f in batch], lr=1e-3)
    torch.cuda.synchronize()
    gains = []
    for d, f in test:
        out = rec.infer(d)
        torch.cuda.synchronize()
        p_net = LN.psnr_tonemapped(out.cpu().numpy(), f.cpu().numpy())
        p_dec = LN.psnr_tonemapped(d.cpu().numpy(), f.cpu().numpy())
        gains.append(p_net - p_dec)
    print("PSNR gain per held-out view (dB):", np.round(gains, 2))
    assert np.mean(gains) > 1.0


def test_probe_and_fallback(torch):
    """Threshold 0 dB never falls back; an unreachable threshold always does
    and then returns exactly the full render."""
    pairs, parts, dec, pal, sc, cams = _pairs(torch, 1, 128, 21)
    net = LN.UNet(seed=1)
    rec = LN.Reconstructor(net)
    img, info = LN.render_learned(parts, dec, cams[0], pal, sc.species_params, rec,
                                  threshold_db=0.0, compensated=True)
    assert not info["fallback"] and info["probe_tiles"] >= 1
    # the probe (rendered on a side stream while the network runs) against
    # the same steps one after another on the caller's stream
    d = B.render(dec, cams[0], pal, sc.species_params, tile=32, compensated=True)
    r = rec.infer(d)
    mask_t, mask = LN.probe_mask(128, 128, 16, 0.02, 0, "cuda")
    probe = torch.zeros_like(r)
    B.render(parts, cams[0], pal, sc.species_params, probe, tile=16, tile_mask=mask_t,
             compensated=True)
    torch.cuda.synchronize()
    sel = np.repeat(np.repeat(mask, 16, 0), 16, 1).astype(bool)
    p_serial = LN.psnr_tonemapped(r.cpu().numpy()[:, sel], probe.cpu().numpy()[:, sel])
    assert info["probe_psnr"] == p_serial
    assert np.array_equal(img.cpu().numpy(), r.cpu().numpy())
    img2, info2 = LN.render_learned(parts, dec, cams[0], pal, sc.species_params, rec,
                                    threshold_db=1e9, compensated=True)
    assert info2["fallback"]
    full = B.render(parts, cams[0], pal, sc.species_params, compensated=True)
    torch.cuda.synchronize()
    assert np.array_equal(img2.cpu().numpy(), full.cpu().numpy())


def test_tile_mask_renders_only_selected_tiles(torch, orc):
    sc = synth.plummer_mix(50_000, seed=4)
    parts, pal = B.scene_to_device(sc)
    mask_t, mask = LN.probe_mask(256, 256, 16, 0.1, 3, "cuda")
    img = torch.full((3, 256, 256), -7.0, device="cuda")
    B.render(parts, sc.camera, pal, sc.species_params, img, tile=16, tile_mask=mask_t)
    torch.cuda.synchronize()
    got = img.cpu().numpy()
    ref = orc.render(sc)
    sel = np.repeat(np.repeat(mask, 16, 0), 16, 1).astype(bool)
    assert np.all(got[:, ~sel] == -7.0)
    rel = np.abs(got[:, sel] - ref[:, sel]).max() / np.abs(ref).max()
    assert rel <= 1e-4
