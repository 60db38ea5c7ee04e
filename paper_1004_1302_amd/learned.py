"""Learned decimation: render a seeded 1/16 subset of the particles and
reconstruct the full render with a convolutional encoder-decoder; fall back
to the full render when a cheap probe says the reconstruction is not good
enough.

Every step runs in libsplotch: the decimation, the renders, the network
(splotch_nn: forward and backward passes, loss, Adam, checkpoints), the
tone map with its scale found on the device, the probe and its PSNR, and
the fallback decision (splotch_render_learned).  This module marshals
arguments; torch holds the buffers and the stream.  `psnr_tonemapped` is a
host helper for evaluating results, not part of the render path.

Network: six levels with 32, 32, 64, 64, 128, 128 channels.  Each level has
two 3x3 convolutions with ReLU; the encoder halves the resolution with 2x2
average pooling, the decoder doubles it with nearest upsampling and
concatenates the encoder features of the same level; a final 3x3
convolution (no activation) adds a correction to the tone-mapped input:
    x = log1p(I_dec / s),  y = x + net(x),  I = s * expm1(y),
s being the mean of the decimated render.  About 1.46M parameters.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import binding as B

LEVELS = (32, 32, 64, 64, 128, 128)
CIN = 32          # tone-mapped RGB, zero-padded to a matrix-core friendly width
DECIMATE = 16     # keep 1 particle in 16
H_SCALE = DECIMATE ** (1.0 / 3.0)

_declared = False


def _lib():
    global _declared
    L = B.lib()
    if not _declared:
        P, I32, I64, F32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
        sig = {
            "splotch_nn_gemm": [P, P, P, I32, I32, I32, I32, I32, I32, I32, P],
            "splotch_nn_im2col3x3": [P, P, I32, I32, I32, I32, P],
            "splotch_nn_flip_weights": [P, P, I32, I32, P],
            "splotch_nn_epilogue": [P, I32, I64, I32, P, I32, P, P, P, P],
            "splotch_nn_conv3x3_weights": [P, P, I32, I32, P],
            "splotch_nn_conv3x3": [P, P, P, I32, P, P, P, I32, I32, I32, I32, I32, P],
            "splotch_nn_relu_bwd": [P, P, I32, P, P, I64, P],
            "splotch_nn_colsum": [P, I64, I32, P, P, P],
            "splotch_nn_pool2": [P, P, I32, I32, I32, I32, P],
            "splotch_nn_pool2_bwd": [P, P, I32, I32, I32, I32, I32, P],
            "splotch_nn_up2_concat": [P, I32, P, I32, P, I32, I32, I32, P],
            "splotch_nn_up2_concat_bwd": [P, I32, I32, P, P, I32, I32, I32, P],
            "splotch_nn_mse": [P, P, P, I64, I32, I32, P, I32, P],
            "splotch_nn_adam": [P, P, P, P, P, I64, F32, F32, F32, F32, I32, P],
            "splotch_nn_tonemap": [P, I32, I32, F32, I32, P, P, P],
            "splotch_nn_untonemap": [P, I32, I32, F32, I32, P, P],
            "splotch_nn_f32_to_bf16": [P, P, I64, P],
            "splotch_nn_param_bytes": [P, P],
            "splotch_nn_create": [P, P, C.c_size_t, C.c_uint64, P, P],
            "splotch_nn_destroy": [P],
            "splotch_nn_workspace_bytes": [P, I32, I32, I32, P],
            "splotch_nn_layer_info": [P, I32, I32, I32, I32, P],
            "splotch_nn_forward": [P, P, P, I32, I32, I32, P, P, C.c_size_t, P],
            "splotch_nn_loss_grad": [P, P, P, I32, I32, I32, P, P, P],
            "splotch_nn_backward": [P, P, P, C.c_size_t, P],
            "splotch_nn_adam_step": [P, F32, P],
            "splotch_nn_save": [P, C.c_char_p, P],
            "splotch_nn_load": [P, C.c_char_p, P],
            "splotch_nn_reconstruct": [P, P, I32, I32, P, P, C.c_size_t, P],
            "splotch_nn_train_step": [P, P, P, I32, I32, I32, F32, P, P, C.c_size_t, P],
            "splotch_decimate": [P, I32, C.c_uint64, P, P, C.c_size_t, P],
            "splotch_probe_mask": [I32, I32, I32, F32, C.c_uint64, P, P],
            "splotch_learned_workspace_bytes": [P, I32, I32, I32, P],
            "splotch_render_learned": [P, P, P, P, P, I32, P, P, C.c_size_t, P, F32, P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.restype = C.c_int
            fn.argtypes = args
        L.splotch_nn_gemm_splits.restype = C.c_int32
        L.splotch_nn_gemm_splits.argtypes = [C.c_int32, C.c_int32]
        for name in ("splotch_nn_n_layers", "splotch_nn_get_step"):
            getattr(L, name).restype = C.c_int32
            getattr(L, name).argtypes = [P]
        L.splotch_decimate_workspace_bytes.restype = C.c_size_t
        L.splotch_decimate_workspace_bytes.argtypes = [I64]
        _declared = True
    return L


def _p(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _s():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ok(code, what):
    if code != 0:
        raise B.SplotchError(code, what)


# ------------------------------------------------------------------ ops
class Ops:
    """Thin wrappers over the C ABI; tensors are torch device tensors
    (bf16 data held as int16 bit patterns)."""

    def __init__(self):
        self.L = _lib()

    def gemm(self, A, Bm, Cbuf, M, N, K, lda, ldb, trans_a, splits):
        _ok(self.L.splotch_nn_gemm(_p(A), _p(Bm), _p(Cbuf), M, N, K, lda, ldb, trans_a, splits,
                                   _s()), "nn_gemm")

    def splits(self, K, want):
        return int(self.L.splotch_nn_gemm_splits(K, want))

    def im2col(self, x, col, n, h, w, c):
        _ok(self.L.splotch_nn_im2col3x3(_p(x), _p(col), n, h, w, c, _s()), "nn_im2col3x3")

    def flip(self, w, wt, cout, cin):
        _ok(self.L.splotch_nn_flip_weights(_p(w), _p(wt), cout, cin, _s()), "nn_flip_weights")

    def epilogue(self, Cp, splits, rows, cols, bias, relu, residual, out_bf, out_f):
        _ok(self.L.splotch_nn_epilogue(_p(Cp), splits, rows, cols, _p(bias), int(relu),
                                       _p(residual), _p(out_bf), _p(out_f), _s()), "nn_epilogue")

    def conv_weights(self, w, wf, cin, cout):
        _ok(self.L.splotch_nn_conv3x3_weights(_p(w), _p(wf), cin, cout, _s()),
            "nn_conv3x3_weights")

    def conv3x3(self, x, wf, bias, relu, residual, out_bf, out_f, n, h, w, cin, cout):
        _ok(self.L.splotch_nn_conv3x3(_p(x), _p(wf), _p(bias), int(relu), _p(residual),
                                      _p(out_bf), _p(out_f), n, h, w, cin, cout, _s()),
            "nn_conv3x3")

    def relu_bwd(self, dy, y, relu, dz_bf, dz_f, n):
        _ok(self.L.splotch_nn_relu_bwd(_p(dy), _p(y), int(relu), _p(dz_bf), _p(dz_f), n, _s()),
            "nn_relu_bwd")

    def colsum(self, x, rows, cols, out, scratch):
        _ok(self.L.splotch_nn_colsum(_p(x), rows, cols, _p(out), _p(scratch), _s()), "nn_colsum")

    def pool2(self, x, out, n, h, w, c):
        _ok(self.L.splotch_nn_pool2(_p(x), _p(out), n, h, w, c, _s()), "nn_pool2")

    def pool2_bwd(self, dout, din, n, h, w, c, acc):
        _ok(self.L.splotch_nn_pool2_bwd(_p(dout), _p(din), n, h, w, c, int(acc), _s()),
            "nn_pool2_bwd")

    def up2_concat(self, a, ca, sk, cs, out, n, h, w):
        _ok(self.L.splotch_nn_up2_concat(_p(a), ca, _p(sk), cs, _p(out), n, h, w, _s()),
            "nn_up2_concat")

    def up2_concat_bwd(self, dout, ca, cs, da, ds, n, h, w):
        _ok(self.L.splotch_nn_up2_concat_bwd(_p(dout), ca, cs, _p(da), _p(ds), n, h, w, _s()),
            "nn_up2_concat_bwd")

    def mse(self, pred, target, grad, pixels, c, used, part, nblocks):
        _ok(self.L.splotch_nn_mse(_p(pred), _p(target), _p(grad), pixels, c, used, _p(part),
                                  nblocks, _s()), "nn_mse")

    def adam(self, w, w_bf, g, m, v, n, lr, b1, b2, eps, step):
        _ok(self.L.splotch_nn_adam(_p(w), _p(w_bf), _p(g), _p(m), _p(v), n, lr, b1, b2, eps, step,
                                   _s()), "nn_adam")

    def tonemap(self, img, h, w, scale, c, out_f, out_bf):
        _ok(self.L.splotch_nn_tonemap(_p(img), h, w, float(scale), c, _p(out_f), _p(out_bf),
                                      _s()), "nn_tonemap")

    def untonemap(self, x, h, w, scale, c, img):
        _ok(self.L.splotch_nn_untonemap(_p(x), h, w, float(scale), c, _p(img), _s()),
            "nn_untonemap")

    def f2bf(self, x, out, n):
        _ok(self.L.splotch_nn_f32_to_bf16(_p(x), _p(out), n, _s()), "nn_f32_to_bf16")


class NNConfig(C.Structure):
    _fields_ = [("n_levels", C.c_int32), ("channels", C.c_int32 * 8), ("in_channels", C.c_int32)]


class NNLayer(C.Structure):
    _fields_ = [("cin", C.c_int32), ("cout", C.c_int32), ("relu", C.c_int32), ("level", C.c_int32),
                ("w", C.c_size_t), ("b", C.c_size_t), ("gw", C.c_size_t), ("gb", C.c_size_t),
                ("w_bf16", C.c_size_t), ("x", C.c_size_t), ("y", C.c_size_t),
                ("dy", C.c_size_t), ("dx", C.c_size_t)]


NONE = (1 << 64) - 1  # SIZE_MAX: tensor not kept


def _view(buf, off, numel, dtype):
    """numel elements of dtype at byte offset off of a uint8 device tensor."""
    import torch
    size = torch.empty(0, dtype=dtype).element_size()
    return buf[off:off + numel * size].view(dtype)


class LayerView:
    """Views of one convolution's parameters in the network's memory."""

    def __init__(self, net, k, info):
        import torch
        self.k, self.cin, self.cout, self.relu = k, info.cin, info.cout, info.relu
        nw = 9 * self.cin * self.cout
        pm = net.params
        self.w = _view(pm, info.w, nw, torch.float32)
        self.b = _view(pm, info.b, self.cout, torch.float32)
        self.gw = _view(pm, info.gw, nw, torch.float32)
        self.gb = _view(pm, info.gb, self.cout, torch.float32)
        self.w_bf = _view(pm, info.w_bf16, nw, torch.int16)

    def n_params(self):
        return self.w.numel() + self.b.numel()


class UNet:
    """The library's reconstruction network (splotch_nn): weights in a
    device buffer this object owns, activations in a workspace grown per
    batch shape."""

    def __init__(self, seed=0, device="cuda", levels=LEVELS, cin=CIN):
        import torch
        self.L = _lib()
        self.levels, self.cin, self.dev = tuple(levels), cin, device
        cfg = NNConfig()
        cfg.n_levels = len(levels)
        for k, c in enumerate(levels):
            cfg.channels[k] = int(c)
        cfg.in_channels = cin
        self.cfg = cfg
        nb = C.c_size_t(0)
        _ok(self.L.splotch_nn_param_bytes(C.byref(cfg), C.byref(nb)), "nn_param_bytes")
        self.params = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
        h = C.c_void_p()
        _ok(self.L.splotch_nn_create(C.byref(cfg), _p(self.params), int(nb.value), int(seed),
                                     _s(), C.byref(h)), "nn_create")
        self.h = h
        self.ws = None
        self._layers = [LayerView(self, k, self.layer_info(k))
                        for k in range(self.L.splotch_nn_n_layers(h))]

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and h.value:
            self.L.splotch_nn_destroy(h)
            self.h = None

    def layer_info(self, k, n=1, h=None, w=None):
        m = 1 << (len(self.levels) - 1)
        info = NNLayer()
        _ok(self.L.splotch_nn_layer_info(self.h, k, n, h or m, w or m, C.byref(info)),
            "nn_layer_info")
        return info

    def layers(self):
        """Encoder levels top-down, decoder levels from the deepest up, then
        the output convolution (the order the FP64 reference uses)."""
        return self._layers

    def n_params(self):
        return sum(c.n_params() for c in self._layers)

    @property
    def step(self):
        return int(self.L.splotch_nn_get_step(self.h))

    def workspace(self, n, h, w):
        import torch
        nb = C.c_size_t(0)
        _ok(self.L.splotch_nn_workspace_bytes(self.h, n, h, w, C.byref(nb)), "nn_workspace_bytes")
        if self.ws is None or self.ws.numel() < nb.value:
            self.ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.dev)
        return self.ws, int(nb.value)

    def tensor(self, off, numel, dtype):
        """A view of the workspace (activations and gradients of the last
        pass, offsets from layer_info)."""
        return _view(self.ws, off, numel, dtype)

    def forward(self, x_f, x_bf, n, h, w):
        """x_f, x_bf: tone-mapped input [n*h*w, in_channels] (FP32 and BF16).
        Returns the FP32 output of the same shape."""
        import torch
        ws, nb = self.workspace(n, h, w)
        y = torch.empty(n * h * w * self.cin, dtype=torch.float32, device=self.dev)
        _ok(self.L.splotch_nn_forward(self.h, _p(x_f), _p(x_bf), n, h, w, _p(y), _p(ws), nb,
                                      _s()), "nn_forward")
        return y

    def loss_grad(self, y, target, n, h, w):
        import torch
        g = torch.empty_like(y)
        part = torch.empty(256, dtype=torch.float32, device=self.dev)
        _ok(self.L.splotch_nn_loss_grad(self.h, _p(y), _p(target), n, h, w, _p(g), _p(part),
                                        _s()), "nn_loss_grad")
        return g, part

    def backward(self, gy):
        """gy: FP32 gradient of the last forward's output.  Fills every
        layer's weight and bias gradients."""
        _ok(self.L.splotch_nn_backward(self.h, _p(gy), _p(self.ws), self.ws.numel(), _s()),
            "nn_backward")

    def adam_step(self, lr):
        _ok(self.L.splotch_nn_adam_step(self.h, float(lr), _s()), "nn_adam_step")

    def save(self, path):
        _ok(self.L.splotch_nn_save(self.h, str(path).encode(), _s()), "nn_save")

    def load(self, path):
        _ok(self.L.splotch_nn_load(self.h, str(path).encode(), _s()), "nn_load")


def decimate(parts: dict, seed=7, keep=DECIMATE):
    """splotch_decimate: an exact seeded 1/keep subset (index order) with
    smoothing lengths and density amplitudes scaled by keep^(1/3)."""
    import torch
    L = _lib()
    n = int(parts["x"].numel())
    m = max(1, n // keep) if n > 0 else 0
    dev = parts["x"].device
    out = {k: torch.empty(m, dtype=torch.float32, device=dev)
           for k in ("x", "y", "z", "h", "value", "rho0")}
    for k in ("value_g", "value_b"):
        if parts.get(k) is not None:
            out[k] = torch.empty(m, dtype=torch.float32, device=dev)
    if parts.get("species") is not None:
        out["species"] = torch.empty(m, dtype=torch.uint8, device=dev)
    ws = torch.empty(max(1, int(L.splotch_decimate_workspace_bytes(n))), dtype=torch.uint8,
                     device=dev)
    P_in = B.particles_struct(parts)
    P_out = B.particles_struct(out)
    _ok(L.splotch_decimate(C.byref(P_in), int(keep), int(seed), C.byref(P_out), _p(ws),
                           ws.numel(), _s()), "decimate")
    return out


class Reconstructor:
    """Image-level use of the network: training steps on render pairs and
    reconstruction of a decimated render (all on the device)."""

    def __init__(self, net: UNet):
        self.net = net

    def train_step(self, dec_imgs, full_imgs, lr=1e-3):
        """One step on lists of planar [3,H,W] renders; returns the 256 loss
        partials (device) of the step."""
        import torch
        n = len(dec_imgs)
        _, h, w = dec_imgs[0].shape
        ws, nb = self.net.workspace(n, h, w)
        D = (C.c_void_p * n)(*[t.data_ptr() for t in dec_imgs])
        Fi = (C.c_void_p * n)(*[t.data_ptr() for t in full_imgs])
        part = torch.empty(256, dtype=torch.float32, device=self.net.dev)
        _ok(self.net.L.splotch_nn_train_step(self.net.h, D, Fi, n, h, w, float(lr), _p(part),
                                             _p(ws), nb, _s()), "nn_train_step")
        return part

    def infer(self, dec_img):
        """Reconstructed planar [3,H,W] image from one decimated render."""
        import torch
        _, h, w = dec_img.shape
        ws, nb = self.net.workspace(1, h, w)
        out = torch.empty_like(dec_img)
        _ok(self.net.L.splotch_nn_reconstruct(self.net.h, _p(dec_img), h, w, _p(out), _p(ws), nb,
                                              _s()), "nn_reconstruct")
        return out


def psnr_tonemapped(img, ref):
    """PSNR of img against ref after the tone map T(I) = log1p(I/s) /
    log1p(max(ref)/s), s = mean of ref (host numpy arrays [3,H,W])."""
    ref = np.asarray(ref, np.float64)
    img = np.asarray(img, np.float64)
    s = ref.mean()
    if not s > 0:
        # a dark reference: agreement only if the image is dark too
        return float("inf") if not img.max() > 0 else float("-inf")
    den = math.log1p(ref.max() / s)
    a = np.log1p(np.maximum(img, 0) / s) / den
    b = np.log1p(np.maximum(ref, 0) / s) / den
    mse = float(((a - b) ** 2).mean())
    return float("inf") if mse == 0 else 10.0 * math.log10(1.0 / mse)


def psnr_linear(img, ref):
    """PSNR of img against ref with the reference's largest value as the
    peak (host numpy arrays [3,H,W])."""
    ref = np.asarray(ref, np.float64)
    img = np.asarray(img, np.float64)
    peak = float(np.abs(ref).max())
    mse = float(((img - ref) ** 2).mean())
    if mse == 0:
        return float("inf")
    return float("-inf") if peak == 0 else 10.0 * math.log10(peak * peak / mse)


def probe_mask(width, height, tile, frac, seed, device):
    """splotch_probe_mask: a seeded sample of about frac of the screen tiles
    (at least one), as a device uint8 mask and its host copy [nty, ntx]."""
    import torch
    ntx, nty = -(-width // tile), -(-height // tile)
    m = torch.empty(ntx * nty, dtype=torch.uint8, device=device)
    _ok(_lib().splotch_probe_mask(width, height, tile, float(frac), int(seed), _p(m), _s()),
        "probe_mask")
    return m, m.cpu().numpy().reshape(nty, ntx)


_probe_cache = {}
_nn_ws = {}


def render_learned(parts_full, parts_dec, cam, palette, species, recon, *,
                   threshold_db=40.0, probe_frac=0.02, seed=0, tile=16, dec_tile=32, **kw):
    """splotch_render_learned: decimated render, reconstruction, probe on a
    seeded sample of tiles (rendered on a library stream while the network
    runs), PSNR on the device, and the full render if the PSNR is below
    threshold_db.  recon: a Reconstructor or UNet.  Returns (image, info)
    with the probe PSNR and whether the full render was used."""
    import torch
    net = recon.net if isinstance(recon, Reconstructor) else recon
    L = _lib()
    dev = parts_full["x"].device
    key = (cam.width, cam.height, tile, probe_frac, seed, str(dev))
    if key not in _probe_cache:
        _probe_cache[key] = probe_mask(cam.width, cam.height, tile, probe_frac, seed, dev)
    mask_t, mask = _probe_cache[key]
    cs = cam if isinstance(cam, B.CameraS) else B.camera_struct(cam)
    pk = {k: v for k, v in kw.items() if k in ("sigma_over_h", "trunc_f", "compensated",
                                               "accumulate", "seg_records", "splat_variant",
                                               "kernel", "emission_is_source")}
    prm = B.params_struct(species, tile=tile, **pk)
    mp = int(kw.get("max_pairs") or 0)
    Pf, Pd = B.particles_struct(parts_full), B.particles_struct(parts_dec)
    prm_d = B.params_struct(species, tile=dec_tile, **pk)
    need = max(B.workspace_bytes(Pf.n, cs, prm, mp), B.workspace_bytes(Pd.n, cs, prm_d, mp))
    ws = B.get_workspace(need, dev)
    prm.workspace = C.c_void_p(ws.data_ptr())
    prm.workspace_bytes = need
    prm.stream = _s()
    nb = C.c_size_t(0)
    _ok(L.splotch_learned_workspace_bytes(net.h, cam.width, cam.height, tile, C.byref(nb)),
        "learned_workspace_bytes")
    lw = _nn_ws.get(str(dev))
    if lw is None or lw.numel() < nb.value:
        lw = torch.empty(int(nb.value), dtype=torch.uint8, device=dev)
        _nn_ws[str(dev)] = lw
    image = torch.empty((3, cs.height, cs.width), dtype=torch.float32, device=dev)
    cm = B.colourmap_struct(palette, kw.get("palette_absorb"))
    img = B.Image(C.c_void_p(image.data_ptr()), cs.width, cs.height)
    fb = C.c_int32(0)
    ps = C.c_float(0)
    _ok(L.splotch_render_learned(C.byref(Pf), C.byref(Pd), C.byref(cs), C.byref(cm),
                                 C.byref(prm), int(dec_tile), net.h, _p(lw), int(nb.value),
                                 _p(mask_t), float(threshold_db), C.byref(img), C.byref(fb),
                                 C.byref(ps)), "render_learned")
    info = dict(probe_psnr=float(ps.value), fallback=bool(fb.value), probe_tiles=int(mask.sum()))
    return image, info
