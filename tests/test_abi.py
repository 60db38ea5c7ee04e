"""Host-side checks of the C ABI: no GPU needed, no compute launched.

Every argument error below is detected on the host before any HIP call,
so these run on a machine without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1004_1302_amd import binding as B
from paper_1004_1302_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "splotch.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(splotch_\w+)\s*\(", txt, re.M)))


def test_exports_every_declared_symbol():
    lib = B.lib()
    names = declared_functions()
    assert len(names) >= 6
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(B.EXPORTS)


def test_status_strings():
    for code in range(6):
        s = B.status_string(code)
        assert isinstance(s, str) and s
    assert B.status_string(0) == "ok"
    assert B.status_string(99) == "unknown status"


def _params(**kw):
    return B.params_struct([synth.Species()], **kw)


def test_camera_look_at_frame():
    c = B.camera_look_at((1, 2, 3), (4, -2, 9), (0, 1, 0), B.PERSPECTIVE, 60.0, 640, 480, 0.1, 100)
    R, U, F = (np.array(list(getattr(c, k)), np.float64) for k in ("right", "up", "fwd"))
    assert np.allclose([R @ R, U @ U, F @ F], 1, atol=1e-6)
    assert np.allclose([R @ U, R @ F, U @ F], 0, atol=1e-6)
    assert np.allclose(np.cross(R, U), F, atol=1e-6)
    assert c.focal_px == pytest.approx(320 / np.tan(np.radians(30)), rel=1e-6)
    # agrees with the generator's frame construction
    g = synth.look_at((1, 2, 3), (4, -2, 9), (0, 1, 0), B.PERSPECTIVE, 640, 480, 60.0)
    assert np.allclose(R, g.right, atol=1e-6) and np.allclose(U, g.up, atol=1e-6)
    with pytest.raises(B.SplotchError):
        B.camera_look_at((0, 0, 0), (0, 0, 0), (0, 1, 0), B.PERSPECTIVE, 60.0, 64, 64, 0.1, 10)
    with pytest.raises(B.SplotchError):
        B.camera_look_at((0, 0, 0), (0, 1, 0), (0, 1, 0), B.PERSPECTIVE, 60.0, 64, 64, 0.1, 10)


def _ws_size(n, cam, prm, pairs=0):
    out = C.c_size_t()
    code = B.lib().splotch_workspace_size(n, C.byref(cam), C.byref(prm), pairs, C.byref(out))
    return code, out.value


def test_workspace_size_monotone():
    cam = B.camera_struct(synth.ortho_unit_square(256, 256))
    prm = _params()
    sizes = [_ws_size(n, cam, prm)[1] for n in (0, 1, 1000, 10 ** 5, 10 ** 7)]
    assert all(b > a for a, b in zip(sizes, sizes[1:]))
    assert _ws_size(1000, cam, prm, 10 ** 6)[1] > _ws_size(1000, cam, prm, 10 ** 4)[1]
    # an ordered species needs the depth-sort buffers
    prm_o = B.params_struct([synth.Species(mode=synth.ORDERED, absorption=1.0)])
    assert _ws_size(10 ** 5, cam, prm_o)[1] > _ws_size(10 ** 5, cam, prm)[1]
    assert _ws_size(-1, cam, prm)[0] == 1


SEG_TARGET = 65536  # kSegTarget of the library


def _seg_len_rule(npairs, nt, seg_min, target=SEG_TARGET):
    s = max(-(-npairs // target), seg_min)
    return -(-s // nt) * nt


def test_segment_slot_bound():
    """A tile of L > s records is cut into ceil(L/s) < 2L/s segments, so a
    pass with P pairs fills fewer than 2P/s partial slots; with s at least
    the segment minimum and at least P/65536, that is at most
    2 min(65536, P/seg_min).  Checked on skewed tile-length mixes, and the
    workspace grows when a shorter segment minimum needs more slots."""
    rng = np.random.default_rng(0)
    for trial in range(3000):
        seg_min = int(rng.choice([1, 7, 64, 256, 300, 1024, 5000]))
        nt = int(rng.choice([64, 256, 1024]))
        L = (rng.pareto(0.8, int(rng.integers(1, 3000))) * seg_min).astype(np.int64)
        if trial % 3 == 0:
            L[:] = max(seg_min, nt) + 1
        P = int(L.sum())
        s = _seg_len_rule(P, nt, seg_min)
        nseg = np.where(L == 0, 1, -(-L // s))
        assert nseg[nseg > 1].sum() <= min(2 * SEG_TARGET, 2 * (P // seg_min) + 2)
        assert nseg.sum() <= L.size + SEG_TARGET
    cam = B.camera_struct(synth.ortho_unit_square(256, 256))
    short, default = _params(seg_records=256), _params()
    assert _ws_size(1000, cam, short, 10 ** 6)[1] > _ws_size(1000, cam, default, 10 ** 6)[1]


@pytest.mark.parametrize("field,value,code", [
    ("width", 0, 1), ("height", -3, 1), ("width", 20000, 1), ("projection", 7, 1),
    ("px_per_unit", 0.0, 1), ("z_far", -5.0, 1),
])
def test_camera_validation(field, value, code):
    cam = B.camera_struct(synth.ortho_unit_square(64, 64))
    setattr(cam, field, value)
    assert _ws_size(10, cam, _params())[0] == code


def test_non_orthonormal_frame_rejected():
    cam = B.camera_struct(synth.ortho_unit_square(64, 64))
    cam.up[:] = [0.0, 1.0, 0.1]
    assert _ws_size(10, cam, _params())[0] == 1


def test_perspective_needs_positive_near_and_focal():
    cam = B.camera_struct(synth.look_at((0, 0, -5), (0, 0, 0), (0, 1, 0), B.PERSPECTIVE, 64, 64))
    assert _ws_size(10, cam, _params())[0] == 0
    cam.z_near = 0.0
    assert _ws_size(10, cam, _params())[0] == 1
    cam.z_near = 0.1
    cam.focal_px = -1.0
    assert _ws_size(10, cam, _params())[0] == 1


@pytest.mark.parametrize("kw,code", [
    (dict(sigma_over_h=0.0), 1), (dict(trunc_f=-1.0), 1), (dict(tile=12), 4), (dict(tile=128), 4),
    (dict(tile=64), 0), (dict(tile=64, splat_variant=2), 4), (dict(tile=64, splat_variant=3), 4),
    (dict(splat_variant=4), 1), (dict(splat_variant=-1), 1), (dict(splat_variant=3), 0),
    (dict(seg_records=-5), 1), (dict(batch_streams=5), 1), (dict(batch_streams=-1), 1),
    (dict(batch_streams=4), 0), (dict(kernel=2), 1), (dict(kernel=-1), 1), (dict(kernel=1), 0),
    (dict(emission_is_source=2), 1), (dict(emission_is_source=1), 0),
])
def test_param_validation(kw, code):
    cam = B.camera_struct(synth.ortho_unit_square(64, 64))
    assert _ws_size(10, cam, _params(**kw))[0] == code


def test_species_validation():
    cam = B.camera_struct(synth.ortho_unit_square(64, 64))
    bad = [synth.Species(mode=5), synth.Species(absorption=-1.0),
           synth.Species(vmin=-1.0, vmax=2.0, log_scale=1), synth.Species(colour=2),
           synth.Species(colour=-1)]
    for s in bad:
        assert _ws_size(10, cam, B.params_struct([s]))[0] == 1
    p = B.params_struct([synth.Species()])
    p.n_species = 0
    assert _ws_size(10, cam, p)[0] == 1
    p.n_species = 9
    assert _ws_size(10, cam, p)[0] == 1


def test_render_rejects_before_launch():
    """Argument errors come back before any device work (no GPU here)."""
    cam = B.camera_struct(synth.ortho_unit_square(64, 64))
    prm = _params()
    P = B.Particles()
    P.n = 10  # null pointers with n > 0
    cm = B.Colourmap(256, C.c_void_p(0x1000))
    img = B.Image(C.c_void_p(0x2000), 64, 64)
    lib = B.lib()
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm), C.byref(img)) == 1
    P.n = 0
    # no workspace
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm), C.byref(img)) == 2
    # misaligned workspace
    prm.workspace = C.c_void_p(0x1001)
    prm.workspace_bytes = 1 << 30
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm), C.byref(img)) == 2
    # too small
    prm.workspace = C.c_void_p(0x100000)
    prm.workspace_bytes = 100
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm), C.byref(img)) == 2
    prm.workspace_bytes = 1 << 30
    # palette with one entry, image of the wrong size
    bad_cm = B.Colourmap(1, C.c_void_p(0x1000))
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(bad_cm), C.byref(prm), C.byref(img)) == 1
    # absorption table with one entry
    bad_cm = B.Colourmap(256, C.c_void_p(0x1000), 1, C.c_void_p(0x3000))
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(bad_cm), C.byref(prm), C.byref(img)) == 1
    # a vector-coloured species without its second and third components
    vec = B.params_struct([synth.Species(colour=synth.COLOUR_VECTOR)])
    vec.workspace, vec.workspace_bytes = prm.workspace, prm.workspace_bytes
    Pv = B.Particles()
    Pv.n = 4
    Pv.x = Pv.y = Pv.z = Pv.h = Pv.value = C.c_void_p(0x4000)
    assert lib.splotch_render(C.byref(Pv), C.byref(cam), C.byref(cm), C.byref(vec), C.byref(img)) == 1
    bad_img = B.Image(C.c_void_p(0x2000), 32, 64)
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm), C.byref(bad_img)) == 1
    P.n = 1 << 32
    assert lib.splotch_render(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm), C.byref(img)) == 1


def test_bin_and_project_validate():
    cam = B.camera_struct(synth.ortho_unit_square(64, 64))
    prm = _params(tile=24)
    P = B.Particles()
    lib = B.lib()
    assert lib.splotch_project(C.byref(P), C.byref(cam), C.byref(prm), None, None, None, None, None) == 4
    n = C.c_int64()
    assert lib.splotch_bin(C.byref(P), C.byref(cam), C.byref(prm), None, None, None, 0, C.byref(n)) == 4


def test_batch_validates_before_launch():
    cam = B.camera_struct(synth.ortho_unit_square(64, 64))
    prm = _params()
    P = B.Particles()
    cm = B.Colourmap(256, C.c_void_p(0x1000))
    cams = (B.CameraS * 2)(cam, cam)
    ims = (B.Image * 2)(B.Image(C.c_void_p(0x2000), 64, 64), B.Image(C.c_void_p(0x3000), 64, 64))
    lib = B.lib()
    assert lib.splotch_render_batch(C.byref(P), 0, cams, C.byref(cm), C.byref(prm), ims, 0) == 1
    assert lib.splotch_render_batch(C.byref(P), 2, cams, C.byref(cm), None, ims, 0) == 1
    bad = (B.Image * 2)(B.Image(C.c_void_p(0x2000), 64, 64), B.Image(C.c_void_p(0x3000), 32, 64))
    assert lib.splotch_render_batch(C.byref(P), 2, cams, C.byref(cm), C.byref(prm), bad, 0) == 1
    # no workspace
    assert lib.splotch_render_batch(C.byref(P), 2, cams, C.byref(cm), C.byref(prm), ims, 0) == 2
    assert lib.splotch_render_batch(C.byref(P), 2, cams, C.byref(cm), C.byref(prm), ims, 3) == 1
    assert B.graph_cache_clear() == 0


def test_fused_conv_argument_checks():
    """Host-side checks of the fused convolution's arguments, before any
    launch: channel counts must be multiples of 32, sizes positive, and at
    least one output given."""
    import ctypes as C
    from paper_1004_1302_amd import learned as LN
    L = LN._lib()
    p = C.c_void_p(16)
    bad = [
        (p, p, None, 1, None, p, None, 1, 8, 16, 48, 32),   # cin % 32
        (p, p, None, 1, None, p, None, 1, 8, 16, 32, 40),   # cout % 32
        (p, p, None, 1, None, None, None, 1, 8, 16, 32, 32),  # no output
        (None, p, None, 1, None, p, None, 1, 8, 16, 32, 32),  # no input
        (p, p, None, 1, None, p, None, 0, 8, 16, 32, 32),   # n = 0
        (p, p, None, 1, None, p, None, 1, 8, -1, 32, 32),   # w < 0
    ]
    for args in bad:
        assert L.splotch_nn_conv3x3(*args, None) == 1, args  # SPLOTCH_E_INVALID_ARG
    assert L.splotch_nn_conv3x3_weights(None, p, 32, 32, None) == 1


def test_static_render_refuses_before_device_work():
    """splotch_render_static checks sizes and settings on the host: an input
    beyond the static buffer and stage timing are refused before any HIP
    call (no GPU here)."""
    cam = B.camera_struct(synth.ortho_unit_square(4096, 4096))
    P = B.Particles()
    P.n = 100_000_000
    P.x = P.y = P.z = P.h = P.value = C.c_void_p(0x1000)
    cm = B.Colourmap(256, C.c_void_p(0x1000), 0, None)
    img = B.Image(C.c_void_p(0x2000), 4096, 4096)
    lib = B.lib()
    prm = _params()
    assert lib.splotch_render_static(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm),
                                     C.byref(img)) == 6
    prm.profile = 1
    assert lib.splotch_render_static(C.byref(P), C.byref(cam), C.byref(cm), C.byref(prm),
                                     C.byref(img)) == 1
    assert "static scratch" in B.status_string(6)


def test_network_and_learned_arguments_checked_on_host():
    """Configuration and argument checks of the network object and the
    learned path that need no device."""
    from paper_1004_1302_amd import learned as LN
    L = LN._lib()
    cfg = LN.NNConfig()
    cfg.n_levels = 6
    for k, c in enumerate(LN.LEVELS):
        cfg.channels[k] = c
    cfg.in_channels = LN.CIN
    nb = C.c_size_t(0)
    assert L.splotch_nn_param_bytes(C.byref(cfg), C.byref(nb)) == 0
    # per layer: FP32 weights, gradients and two moments, three BF16 copies
    nw = 9 * 32 * 32 * 2 + 9 * 32 * 64 + 9 * 64 * 64 * 3 + 9 * 64 * 128 + 9 * 128 * 128 * 3 + \
        9 * 96 * 32 + 9 * 128 * 64 + 9 * 192 * 64 + 9 * 256 * 128 + 9 * 32 * 32
    assert nb.value >= nw * (4 * 4 + 2 * 3)
    for bad in (dict(n_levels=0), dict(n_levels=9), dict(in_channels=16), dict(ch0=48)):
        c2 = LN.NNConfig()
        C.memmove(C.byref(c2), C.byref(cfg), C.sizeof(cfg))
        if "n_levels" in bad:
            c2.n_levels = bad["n_levels"]
        if "in_channels" in bad:
            c2.in_channels = bad["in_channels"]
        if "ch0" in bad:
            c2.channels[0] = bad["ch0"]
        assert L.splotch_nn_param_bytes(C.byref(c2), C.byref(nb)) == 1
    h = C.c_void_p()
    assert L.splotch_nn_create(C.byref(cfg), None, 0, 1, None, C.byref(h)) == 2
    assert L.splotch_decimate_workspace_bytes(1000) >= 8000
    assert L.splotch_probe_mask(64, 64, 12, 0.1, 0, C.c_void_p(0x1000), None) == 1
    assert L.splotch_probe_mask(64, 64, 16, 0.0, 0, C.c_void_p(0x1000), None) == 1
    P = B.Particles()
    P.n = 100
    out = B.Particles()
    out.n = 7  # must be 100 // 16 = 6
    ws = C.c_void_p(0x1000)
    assert L.splotch_decimate(C.byref(P), 16, 0, C.byref(out), ws, 1 << 20, None) == 1
