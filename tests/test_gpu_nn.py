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
    (3, 8, 16, 32, 64, True, True),
    # 8 * 8 tiles * 8 images * 2 groups of 64 channels = 1024 workgroups:
    # the 64-channel grouping
    (8, 64, 128, 32, 128, True, True)])
def test_fused_conv3x3(torch, n, h, w, ci, co, relu, res):
    """The fused convolution (halo tile and weights in LDS, implicit GEMM on
    the matrix cores) against the FP64 reference on the same BF16 operands,
    and against im2col + GEMM + epilogue: ragged tiles, several images,
    several 32-channel slices, both channel groupings (32 output channels
    per workgroup on small grids, 64 once the grid has 1024 workgroups),
    residual input."""
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


def _layer_index(L):
    enc_a = lambda l: 2 * l
    enc_b = lambda l: 2 * l + 1
    dec_a = lambda l: 2 * L + 2 * (L - 2 - l)
    dec_b = lambda l: dec_a(l) + 1
    return enc_a, enc_b, dec_a, dec_b, 4 * L - 2


def _run_net(torch, levels, n, h, w, seed):
    net = LN.UNet(seed=seed, levels=levels)
    rng = np.random.default_rng(seed + 3)
    for c in net.layers():
        c.b.copy_(torch.from_numpy(rng.standard_normal(c.cout).astype(np.float32) * 0.05))
    x = np.zeros((n * h * w, LN.CIN))
    x[:, :3] = rng.uniform(0, 2, (n * h * w, 3))
    t = x.copy()
    t[:, :3] += rng.normal(0, 0.2, (n * h * w, 3))
    x_f = torch.from_numpy(x.astype(np.float32)).cuda()
    x_bf, _ = to_bf16_bits(torch, x)
    t_f = torch.from_numpy(t.astype(np.float32)).cuda()
    y = net.forward(x_f, x_bf, n, h, w)
    g, _ = net.loss_grad(y, t_f, n, h, w)
    net.backward(g)
    torch.cuda.synchronize()
    return net, x.astype(np.float32).astype(np.float64), t, y, g


def test_unet_every_layer_elementwise(torch):
    """The six-level network of the learned path (2 images of 64x64, so the
    deepest level runs at 2x2) checked layer by layer, element by element,
    against the FP64 reference fed the GPU's own BF16 inputs, weights and
    output gradients: every convolution's output, dW, db and input
    gradient, and every connection between layers (pooling, upsampling and
    concatenation, their adjoints, the residual).  Bounds: a BF16 output may
    differ by one BF16 step (2^-8 relative) where the FP32 sum lands on the
    other side of a rounding boundary, plus 1e-5 of the layer's largest
    value for the FP32 accumulation order; FP32 gradients within 1e-4 of
    the largest value (sums over up to 9 x 8192 terms)."""
    levels = LN.LEVELS
    L = len(levels)
    n, h, w = 2, 64, 64
    net, x, t, y, g = _run_net(torch, levels, n, h, w, seed=3)
    enc_a, enc_b, dec_a, dec_b, out_k = _layer_index(L)
    info = [net.layer_info(k, n, h, w) for k in range(out_k + 1)]
    bf = lambda off, numel: bits_to_f64(net.tensor(off, numel, torch.int16))
    f32 = lambda off, numel: net.tensor(off, numel, torch.float32).cpu().numpy().astype(np.float64)
    X, Y, DY, DX = {}, {}, {}, {}
    for k, (lay, inf) in enumerate(zip(net.layers(), info)):
        hh, ww = h >> inf.level, w >> inf.level
        P = n * hh * ww
        ci, co = inf.cin, inf.cout
        X[k] = bf(inf.x, P * ci).reshape(n, hh, ww, ci)
        Wb = bits_to_f64(lay.w_bf).reshape(9, ci, co)
        b = lay.b.cpu().numpy().astype(np.float64)
        z = R.conv3x3(X[k], Wb, b)
        if inf.relu:
            Y[k] = bf(inf.y, P * co).reshape(n, hh, ww, co)
            ref = np.maximum(z, 0)
            scale = np.abs(ref).max()
            assert np.all(np.abs(Y[k] - ref) <= 2.0 ** -8 * np.abs(ref) + 1e-5 * scale), k
        else:
            Y[k] = f32(inf.y, P * co).reshape(n, hh, ww, co)
            ref = z + x.reshape(n, hh, ww, co)
            assert np.abs(Y[k] - ref).max() <= 1e-5 * np.abs(ref).max(), k
        DY[k] = f32(inf.dy, P * co).reshape(n, hh, ww, co)
        mask = (Y[k] > 0) if inf.relu else np.ones_like(Y[k], bool)
        dz = R.bf16(DY[k] * mask)
        dx_r, dW_r, _ = R.conv3x3_adjoint(X[k], Wb, dz)
        db_r = (DY[k] * mask).reshape(-1, co).sum(axis=0)
        gw = lay.gw.cpu().numpy().astype(np.float64).reshape(9, ci, co)
        gb = lay.gb.cpu().numpy().astype(np.float64)
        assert np.abs(gw - dW_r).max() <= 1e-4 * np.abs(dW_r).max(), k
        assert np.abs(gb - db_r).max() <= 1e-4 * max(np.abs(db_r).max(), 1e-30), k
        if inf.dx != LN.NONE:
            DX[k] = f32(inf.dx, P * ci).reshape(n, hh, ww, ci)
            assert np.abs(DX[k] - dx_r).max() <= 1e-4 * np.abs(dx_r).max(), k
        else:
            assert k == enc_a(0)
    # forward connections: pooled and concatenated inputs are exact
    for l in range(1, L):
        e = Y[enc_b(l - 1)].astype(np.float32)
        pooled = np.float32(0.25) * (((e[:, 0::2, 0::2] + e[:, 0::2, 1::2]) + e[:, 1::2, 0::2])
                                     + e[:, 1::2, 1::2])
        assert np.array_equal(X[enc_a(l)], R.bf16(pooled.astype(np.float64)))
    for l in range(L - 2, -1, -1):
        below = Y[enc_b(L - 1)] if l == L - 2 else Y[dec_b(l + 1)]
        assert np.array_equal(X[dec_a(l)], R.up2_concat(below, Y[enc_b(l)]))
    assert np.array_equal(X[out_k], Y[dec_b(0)])
    assert np.array_equal(X[enc_a(0)], R.bf16(x).reshape(X[enc_a(0)].shape))
    # backward connections: the output gradient of each layer from the
    # input gradients of the layers it feeds
    yo = Y[out_k].reshape(-1, LN.CIN)
    _, gref = R.mse(yo, t, 3)
    # the loss gradient 2 (y - t) / (3 P): y - t rounds in FP32
    assert np.abs(DY[out_k].reshape(-1, LN.CIN) - gref).max() <= 1e-6 * np.abs(gref).max()
    close = lambda a, b: np.abs(a - b).max() <= 1e-6 * max(np.abs(b).max(), 1e-30)
    for l in range(L - 1):
        assert info[dec_a(l)].dy == info[dec_b(l)].dx
        src = DX[out_k] if l == 0 else R.up2_concat_adjoint(DX[dec_a(l - 1)], levels[l])[0]
        assert close(DY[dec_b(l)], src), l
    for l in range(L):
        assert info[enc_a(l)].dy == info[enc_b(l)].dx
        if l == L - 1:
            src = R.up2_concat_adjoint(DX[dec_a(L - 2)], levels[L - 1])[0]
        else:
            src = R.up2_concat_adjoint(DX[dec_a(l)], levels[l + 1])[1] + \
                R.pool2_adjoint(DX[enc_a(l + 1)])
        assert close(DY[enc_b(l)], src), l


def test_unet_end_to_end_against_reference(torch):
    """The same network run end to end against the FP64 reference with BF16
    rounding at the same points (no GPU values fed back): the output and the
    output-layer gradients agree element by element within a bound that
    allows one-step BF16 flips to propagate through 22 layers."""
    levels = LN.LEVELS
    n, h, w = 2, 64, 64
    net, x, t, y, g = _run_net(torch, levels, n, h, w, seed=4)
    ref = R.UNetRef(levels, [(bits_to_f64(c.w_bf).reshape(9, c.cin, c.cout),
                              c.b.cpu().numpy().astype(np.float64)) for c in net.layers()],
                    cin=LN.CIN, round_bf16=True)
    yr = ref.forward(x.reshape(n, h, w, LN.CIN))
    yg = y.cpu().numpy().reshape(n, h, w, LN.CIN).astype(np.float64)
    assert np.all(np.abs(yg - yr) <= 1e-2 * np.abs(yr).max())
    _, gr = R.mse(yr, t.reshape(n, h, w, LN.CIN), 3)
    grads = ref.backward(gr)
    last = net.layers()[-1]
    gw = last.gw.cpu().numpy().astype(np.float64).reshape(9, last.cin, last.cout)
    assert np.all(np.abs(gw - grads[-1][0]) <= 3e-2 * np.abs(grads[-1][0]).max())


def test_checkpoint_resume_is_exact(torch, tmp_path):
    """Weights, biases, Adam moments and the step count round-trip through a
    checkpoint: training resumed from it gives bit-identical weights."""
    levels = (32, 32, 64)
    n, h, w = 2, 16, 16
    rng = np.random.default_rng(9)
    batches = []
    for _ in range(5):
        d = [torch.from_numpy(rng.uniform(0, 1, (3, h, w)).astype(np.float32)).cuda()
             for _ in range(n)]
        f = [(t * 1.3).contiguous() for t in d]
        batches.append((d, f))
    a = LN.UNet(seed=5, levels=levels)
    ra = LN.Reconstructor(a)
    for d, f in batches[:3]:
        ra.train_step(d, f, lr=1e-3)
    path = tmp_path / "net.ckpt"
    a.save(path)
    for d, f in batches[3:]:
        ra.train_step(d, f, lr=1e-3)
    b = LN.UNet(seed=6, levels=levels)
    b.load(path)
    assert b.step == 3
    rb = LN.Reconstructor(b)
    for d, f in batches[3:]:
        rb.train_step(d, f, lr=1e-3)
    torch.cuda.synchronize()
    assert a.step == b.step == 5
    for ca, cb in zip(a.layers(), b.layers()):
        assert torch.equal(ca.w, cb.w) and torch.equal(ca.b, cb.b)
    other = LN.UNet(seed=5, levels=(32, 64, 64))
    with pytest.raises(B.SplotchError):
        other.load(path)


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
    """(decimated, full) render pairs of one particle set (generator seed
    `seed`, decimation seed seed + 1) from seeded orbit cameras."""
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
    """A short training run on renderer-made pairs from three particle sets
    (generator and decimation seeds of their own): on views of a fourth,
    unseen particle set the network's output is closer to the full render
    than the decimated render is, and than the decimated render blurred by
    the best of three Gaussian widths (tone-mapped PSNR)."""
    train = []
    for seed in (11, 31, 51):
        train += _pairs(torch, 12, 128, seed)[0]
    test = _pairs(torch, 8, 128, 71)[0]
    net = LN.UNet(seed=0)
    rec = LN.Reconstructor(net)
    order = np.random.default_rng(2).permutation(len(train))
    for it in range(240):
        k = [order[(it * 4 + j) % len(train)] for j in range(4)]
        rec.train_step([train[i][0] for i in k], [train[i][1] for i in k], lr=1e-3)
    torch.cuda.synchronize()
    from scipy.ndimage import gaussian_filter
    gains, over_blur = [], []
    for d, f in test:
        out = rec.infer(d)
        torch.cuda.synchronize()
        fh, dh = f.cpu().numpy(), d.cpu().numpy()
        p_net = LN.psnr_tonemapped(out.cpu().numpy(), fh)
        p_dec = LN.psnr_tonemapped(dh, fh)
        # a non-learned baseline: the decimated render blurred, best of
        # three widths for each view
        p_blur = max(LN.psnr_tonemapped(gaussian_filter(dh, (0, sg, sg)), fh)
                     for sg in (0.5, 1.0, 2.0))
        gains.append(p_net - p_dec)
        over_blur.append(p_net - p_blur)
    print("PSNR gain per view of the unseen set (dB):", np.round(gains, 2))
    print("PSNR gain over the best blurred decimated render (dB):", np.round(over_blur, 2))
    assert np.mean(gains) > 1.0
    assert np.mean(over_blur) > 0.0


def test_training_step_at_full_size(torch):
    """One training step at the learned path's shape (4 images of 1024^2,
    the largest activations: 4 Mpx x 9 taps x 64 channels in the
    backward GEMMs) and one reconstruction: finite loss and output.
    Shapes of 2^31 pixels or more are refused on the host."""
    net = LN.UNet(seed=3)
    rec = LN.Reconstructor(net)
    g = torch.Generator(device="cuda").manual_seed(9)
    full = [torch.rand((3, 1024, 1024), device="cuda", generator=g) for _ in range(4)]
    dec = [f * torch.rand((3, 1024, 1024), device="cuda", generator=g) for f in full]
    part = rec.train_step(dec, full, lr=1e-3)
    out = rec.infer(dec[0])
    torch.cuda.synchronize()
    assert math.isfinite(float(part.sum())) and float(part.sum()) > 0
    assert bool(torch.isfinite(out).all())
    import ctypes as C
    nb = C.c_size_t(0)
    assert net.L.splotch_nn_workspace_bytes(net.h, 4, 1024, 1024, C.byref(nb)) == 0
    assert net.L.splotch_nn_workspace_bytes(net.h, 2048, 1024, 1024, C.byref(nb)) == 1


def test_probe_and_fallback(torch):
    """Threshold 0 dB never falls back; an unreachable threshold always does
    and then returns exactly the full render.  The device PSNR of the probe
    matches the same steps run one after another and evaluated on the
    host."""
    pairs, parts, dec, pal, sc, cams = _pairs(torch, 1, 128, 21)
    net = LN.UNet(seed=1)
    rec = LN.Reconstructor(net)
    img, info = LN.render_learned(parts, dec, cams[0], pal, sc.species_params, rec,
                                  threshold_db=0.0, compensated=True, probe_frac=0.1)
    assert not info["fallback"] and info["probe_tiles"] >= 1
    # the probe (rendered on a side stream while the network runs) against
    # the same steps one after another on the caller's stream
    d = B.render(dec, cams[0], pal, sc.species_params, tile=32, compensated=True)
    r = rec.infer(d)
    mask_t, mask = LN.probe_mask(128, 128, 16, 0.1, 0, "cuda")
    probe = torch.zeros_like(r)
    B.render(parts, cams[0], pal, sc.species_params, probe, tile=16, tile_mask=mask_t,
             compensated=True)
    torch.cuda.synchronize()
    sel = np.repeat(np.repeat(mask, 16, 0), 16, 1).astype(bool)
    p_serial = LN.psnr_tonemapped(r.cpu().numpy()[:, sel], probe.cpu().numpy()[:, sel])
    assert np.isfinite(p_serial) and info["probe_psnr"] == pytest.approx(p_serial, rel=1e-6)
    assert np.array_equal(img.cpu().numpy(), r.cpu().numpy())
    img2, info2 = LN.render_learned(parts, dec, cams[0], pal, sc.species_params, rec,
                                    threshold_db=1e9, compensated=True, probe_frac=0.1)
    assert info2["fallback"], info2
    full = B.render(parts, cams[0], pal, sc.species_params, compensated=True)
    torch.cuda.synchronize()
    assert np.array_equal(img2.cpu().numpy(), full.cpu().numpy())


def test_decimate_exact_seeded_subset(torch):
    """splotch_decimate keeps exactly n/16 particles, in index order, each
    an input particle with h and rho0 scaled by 16^(1/3); the same seed
    gives the same subset, another seed another one; kept indices spread
    over the whole set."""
    sc = synth.plummer_mix(100_003, seed=8)
    sc.rho0 = np.random.default_rng(1).uniform(0.5, 2.0, sc.n).astype(np.float32)
    sc.value = np.arange(1, sc.n + 1, dtype=np.float32)  # labels: value = index + 1
    parts, _ = B.scene_to_device(sc)
    a = LN.decimate(parts, seed=3)
    b = LN.decimate(parts, seed=3)
    c = LN.decimate(parts, seed=4)
    m = 100_003 // 16
    assert a["x"].numel() == m
    for k in a:
        assert torch.equal(a[k], b[k])
    assert not torch.equal(a["x"], c["x"])
    idx = a["value"].cpu().numpy().astype(np.int64) - 1
    assert np.all(np.diff(idx) > 0)
    assert np.array_equal(a["x"].cpu().numpy(), sc.x[idx])
    assert np.array_equal(a["z"].cpu().numpy(), sc.z[idx])
    k3 = np.float32(16.0 ** (1.0 / 3.0))
    assert np.array_equal(a["h"].cpu().numpy(), sc.h[idx] * k3)
    assert np.array_equal(a["rho0"].cpu().numpy(), sc.rho0[idx] * k3)
    hist = np.histogram(idx, bins=10, range=(0, sc.n))[0]
    assert hist.min() > 0.8 * m / 10


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
