"""Python binding of libsplotch (ctypes).

Argument marshalling only: every stage of the render runs in the HIP
library.  torch supplies device memory (particles, palette, image,
workspace) and the stream.  If the library is missing this module raises;
there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsplotch.so")

MAX_SPECIES = 8
ORTHO, PERSPECTIVE = 0, 1
ADDITIVE, ORDERED = 0, 1
COLOUR_PALETTE, COLOUR_VECTOR = 0, 1
KERNEL_GAUSS2D, KERNEL_TRUNC3D = 0, 1

STATUS = {0: "ok", 1: "invalid argument", 2: "workspace", 3: "device", 4: "unsupported",
          5: "capacity", 6: "scratch"}


class SplotchError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {_lib().splotch_status_string(code).decode()} (status {code})")


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", C.c_void_p), ("y", C.c_void_p), ("z", C.c_void_p),
                ("h", C.c_void_p), ("value", C.c_void_p), ("rho0", C.c_void_p),
                ("species", C.c_void_p), ("value_g", C.c_void_p), ("value_b", C.c_void_p)]


class CameraS(C.Structure):
    _fields_ = [("projection", C.c_int32), ("width", C.c_int32), ("height", C.c_int32),
                ("eye", C.c_float * 3), ("right", C.c_float * 3), ("up", C.c_float * 3),
                ("fwd", C.c_float * 3), ("focal_px", C.c_float), ("px_per_unit", C.c_float),
                ("z_near", C.c_float), ("z_far", C.c_float)]


class Colourmap(C.Structure):
    _fields_ = [("n_entries", C.c_int32), ("rgb", C.c_void_p), ("n_entries_absorb", C.c_int32),
                ("rgb_absorb", C.c_void_p)]


class SpeciesS(C.Structure):
    _fields_ = [("vmin", C.c_float), ("vmax", C.c_float), ("log_scale", C.c_int32),
                ("brightness", C.c_float), ("absorption", C.c_float), ("mode", C.c_int32),
                ("colour", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("n_visible", C.c_int64), ("n_invalid", C.c_int64),
                ("n_depth_culled", C.c_int64), ("n_offscreen", C.c_int64),
                ("n_pairs", C.c_int64), ("n_chunks", C.c_int32), ("tile", C.c_int32),
                ("ordered", C.c_int32), ("reserved", C.c_int32),
                ("vmin", C.c_float * MAX_SPECIES), ("vmax", C.c_float * MAX_SPECIES),
                ("stage_ms", C.c_float * 6), ("n_member_pairs", C.c_int64),
                ("n_member_absorbing", C.c_int64)]

    STAGES = ("project", "depth_sort", "scan", "emit", "tile_sort", "splat")

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_
             if k not in ("vmin", "vmax", "reserved", "stage_ms")}
        d["vmin"] = list(self.vmin)
        d["vmax"] = list(self.vmax)
        d["stage_ms"] = dict(zip(self.STAGES, list(self.stage_ms)))
        return d


class Params(C.Structure):
    _fields_ = [("n_species", C.c_int32), ("species", SpeciesS * MAX_SPECIES),
                ("sigma_over_h", C.c_float), ("trunc_f", C.c_float),
                ("accumulate", C.c_int32), ("compensated", C.c_int32), ("tile", C.c_int32),
                ("profile", C.c_int32), ("seg_records", C.c_int32),
                ("splat_variant", C.c_int32), ("batch_streams", C.c_int32),
                ("tile_mask", C.c_void_p),
                ("stream", C.c_void_p), ("workspace", C.c_void_p),
                ("workspace_bytes", C.c_size_t), ("stats", C.POINTER(Stats)),
                ("kernel", C.c_int32), ("emission_is_source", C.c_int32),
                ("split_pixels", C.c_int32), ("batch_persistent", C.c_int32)]


class Image(C.Structure):
    _fields_ = [("rgb", C.c_void_p), ("width", C.c_int32), ("height", C.c_int32)]


_L = None

EXPORTS = ("splotch_status_string", "splotch_camera_look_at", "splotch_workspace_size",
           "splotch_render", "splotch_render_static", "splotch_project", "splotch_bin", "splotch_render_batch",
           "splotch_graph_cache_clear", "splotch_nn_gemm", "splotch_nn_gemm_splits",
           "splotch_nn_im2col3x3", "splotch_nn_flip_weights", "splotch_nn_epilogue",
           "splotch_nn_conv3x3_weights", "splotch_nn_conv3x3",
           "splotch_nn_relu_bwd", "splotch_nn_colsum", "splotch_nn_pool2", "splotch_nn_pool2_bwd",
           "splotch_nn_up2_concat", "splotch_nn_up2_concat_bwd", "splotch_nn_mse",
           "splotch_nn_adam", "splotch_nn_tonemap", "splotch_nn_untonemap",
           "splotch_nn_f32_to_bf16", "splotch_nn_param_bytes", "splotch_nn_create",
           "splotch_nn_destroy", "splotch_nn_n_layers", "splotch_nn_get_step",
           "splotch_nn_workspace_bytes", "splotch_nn_layer_info", "splotch_nn_forward",
           "splotch_nn_loss_grad", "splotch_nn_backward", "splotch_nn_adam_step",
           "splotch_nn_save", "splotch_nn_load", "splotch_nn_reconstruct",
           "splotch_nn_train_step", "splotch_decimate_workspace_bytes", "splotch_decimate",
           "splotch_probe_mask", "splotch_learned_workspace_bytes", "splotch_render_learned",
           "splotch_stream_workspace_size", "splotch_render_stream")
MAX_VIEWS = 1024


def _lib():
    global _L
    if _L is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libsplotch.so not built ({LIB_PATH}); run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.splotch_status_string.restype = C.c_char_p
        L.splotch_status_string.argtypes = [C.c_int]
        L.splotch_camera_look_at.restype = C.c_int
        L.splotch_camera_look_at.argtypes = [C.POINTER(CameraS), C.POINTER(C.c_float * 3),
                                             C.POINTER(C.c_float * 3), C.POINTER(C.c_float * 3),
                                             C.c_int32, C.c_float, C.c_int32, C.c_int32,
                                             C.c_float, C.c_float]
        L.splotch_workspace_size.restype = C.c_int
        L.splotch_workspace_size.argtypes = [C.c_int64, C.POINTER(CameraS), C.POINTER(Params),
                                             C.c_int64, C.POINTER(C.c_size_t)]
        L.splotch_render.restype = C.c_int
        L.splotch_render.argtypes = [C.POINTER(Particles), C.POINTER(CameraS),
                                     C.POINTER(Colourmap), C.POINTER(Params), C.POINTER(Image)]
        L.splotch_render_static.restype = C.c_int
        L.splotch_render_static.argtypes = [C.POINTER(Particles), C.POINTER(CameraS),
                                            C.POINTER(Colourmap), C.POINTER(Params),
                                            C.POINTER(Image)]
        L.splotch_stream_workspace_size.restype = C.c_int
        L.splotch_stream_workspace_size.argtypes = [C.POINTER(Particles), C.c_int64, C.c_int64,
                                                    C.POINTER(CameraS), C.POINTER(Params),
                                                    C.POINTER(C.c_size_t)]
        L.splotch_render_stream.restype = C.c_int
        L.splotch_render_stream.argtypes = [C.POINTER(Particles), C.c_int64, C.c_int64,
                                            C.POINTER(CameraS), C.POINTER(Colourmap),
                                            C.POINTER(Params), C.POINTER(Image)]
        L.splotch_project.restype = C.c_int
        L.splotch_project.argtypes = [C.POINTER(Particles), C.POINTER(CameraS), C.POINTER(Params),
                                      C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p]
        L.splotch_render_batch.restype = C.c_int
        L.splotch_render_batch.argtypes = [C.POINTER(Particles), C.c_int32, C.POINTER(CameraS),
                                           C.POINTER(Colourmap), C.POINTER(Params),
                                           C.POINTER(Image), C.c_int32]
        L.splotch_graph_cache_clear.restype = C.c_int32
        L.splotch_graph_cache_clear.argtypes = []
        L.splotch_bin.restype = C.c_int
        L.splotch_bin.argtypes = [C.POINTER(Particles), C.POINTER(CameraS), C.POINTER(Params),
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64,
                                  C.POINTER(C.c_int64)]
        _L = L
    return _L


def lib():
    return _lib()


def status_string(code: int) -> str:
    return _lib().splotch_status_string(code).decode()


def _check(code, where):
    if code != 0:
        raise SplotchError(code, where)


# ---------------------------------------------------------------- structs
def camera_struct(cam) -> CameraS:
    """From any object with the splotch_camera fields (e.g. synth.Camera)."""
    c = CameraS()
    c.projection = int(cam.projection)
    c.width = int(cam.width)
    c.height = int(cam.height)
    for name in ("eye", "right", "up", "fwd"):
        v = [float(t) for t in getattr(cam, name)]
        getattr(c, name)[:] = v
    c.focal_px = float(cam.focal_px)
    c.px_per_unit = float(cam.px_per_unit)
    c.z_near = float(cam.z_near)
    c.z_far = float(cam.z_far)
    return c


def camera_look_at(eye, at, up, projection, fov_or_scale, width, height, z_near, z_far) -> CameraS:
    c = CameraS()
    f3 = C.c_float * 3
    _check(_lib().splotch_camera_look_at(C.byref(c), C.byref(f3(*eye)), C.byref(f3(*at)),
                                         C.byref(f3(*up)), projection, fov_or_scale, width,
                                         height, z_near, z_far), "splotch_camera_look_at")
    return c


def params_struct(species, sigma_over_h=1.0, trunc_f=2.0, accumulate=False, compensated=False,
                  tile=0, profile=False, seg_records=0, tile_mask=None,
                  splat_variant=0, batch_streams=0, kernel=0, emission_is_source=0,
                  split_pixels=0, batch_persistent=0) -> Params:
    p = Params()
    if not 1 <= len(species) <= MAX_SPECIES:
        raise ValueError("1..8 species")
    p.n_species = len(species)
    for k, s in enumerate(species):
        p.species[k] = SpeciesS(float(s.vmin), float(s.vmax), int(s.log_scale),
                                float(s.brightness), float(s.absorption), int(s.mode),
                                int(getattr(s, "colour", COLOUR_PALETTE)))
    p.sigma_over_h = float(sigma_over_h)
    p.trunc_f = float(trunc_f)
    p.accumulate = 1 if accumulate else 0
    p.compensated = 1 if compensated else 0
    p.tile = int(tile)
    p.profile = int(profile)
    p.seg_records = int(seg_records)
    p.tile_mask = None if tile_mask is None else C.c_void_p(tile_mask.data_ptr())
    p.splat_variant = int(splat_variant)
    p.batch_streams = int(batch_streams)
    p.kernel = int(kernel)
    p.emission_is_source = int(emission_is_source)
    p.split_pixels = int(split_pixels)
    p.batch_persistent = int(batch_persistent)
    return p


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _table(t, what):
    import torch
    if t.dtype != torch.float32 or not t.is_contiguous() or t.dim() != 2 or t.shape[1] != 3:
        raise ValueError(f"{what} must be contiguous float32 [K, 3]")
    return int(t.shape[0]), C.c_void_p(t.data_ptr())


def colourmap_struct(palette, palette_absorb=None) -> Colourmap:
    """Emission table and optional absorption table (device [K, 3] float32)."""
    k, p = _table(palette, "palette")
    cm = Colourmap(k, p, 0, None)
    if palette_absorb is not None:
        cm.n_entries_absorb, cm.rgb_absorb = _table(palette_absorb, "palette_absorb")
    return cm


def particles_struct(parts: dict) -> Particles:
    """parts: dict of contiguous device tensors x, y, z, h, value (float32)
    and optional rho0, value_g, value_b (float32), species (uint8)."""
    import torch
    P = Particles()
    n = int(parts["x"].numel())
    for k in ("x", "y", "z", "h", "value", "rho0", "value_g", "value_b"):
        t = parts.get(k)
        if t is not None:
            if t.dtype != torch.float32 or not t.is_contiguous() or t.numel() != n:
                raise ValueError(f"particle field {k} must be contiguous float32 of length {n}")
    sp = parts.get("species")
    if sp is not None and (sp.dtype != torch.uint8 or not sp.is_contiguous() or sp.numel() != n):
        raise ValueError("species must be contiguous uint8")
    P.n = n
    P.x, P.y, P.z, P.h, P.value = (_ptr(parts[k]) for k in ("x", "y", "z", "h", "value"))
    P.rho0 = _ptr(parts.get("rho0"))
    P.species = _ptr(sp)
    P.value_g = _ptr(parts.get("value_g"))
    P.value_b = _ptr(parts.get("value_b"))
    return P


# ---------------------------------------------------------------- workspace
_ws_cache: dict = {}


def workspace_bytes(n, cam: CameraS, prm: Params, max_pairs=0) -> int:
    out = C.c_size_t(0)
    _check(_lib().splotch_workspace_size(int(n), C.byref(cam), C.byref(prm), int(max_pairs),
                                         C.byref(out)), "splotch_workspace_size")
    return int(out.value)


def get_workspace(nbytes: int, device):
    """A cached uint8 device tensor of at least nbytes (256-byte aligned)."""
    import torch
    key = str(device)
    t = _ws_cache.get(key)
    if t is None or t.numel() < nbytes:
        _ws_cache.pop(key, None)
        t = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws_cache[key] = t
    assert t.data_ptr() % 256 == 0
    return t


def reserve_workspace(parts: dict, cam, species, max_pairs=0, **kw):
    """Grow the cached workspace, on the current stream, to what a render of
    these particles needs, so that a later render (on any stream) does not
    replace it."""
    P = particles_struct(parts)
    cs = cam if isinstance(cam, CameraS) else camera_struct(cam)
    return get_workspace(workspace_bytes(P.n, cs, params_struct(species, **kw), max_pairs),
                         parts["x"].device)


def release_workspace():
    _ws_cache.clear()


def _stream_ptr(device):
    import torch
    return C.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _setup(parts, cam, species, max_pairs, workspace, **kw):
    P = particles_struct(parts)
    cs = cam if isinstance(cam, CameraS) else camera_struct(cam)
    prm = params_struct(species, **kw)
    dev = parts["x"].device
    if workspace is None:
        need = workspace_bytes(P.n, cs, prm, max_pairs or 0)
        workspace = get_workspace(need, dev)
        nbytes = need  # the cached buffer may be larger; the pair capacity follows max_pairs
    else:
        nbytes = int(workspace.numel())
    prm.workspace = C.c_void_p(workspace.data_ptr())
    prm.workspace_bytes = nbytes
    prm.stream = _stream_ptr(dev)
    return P, cs, prm, dev


def render(parts: dict, cam, palette, species, image=None, *, sigma_over_h=1.0, trunc_f=2.0,
           accumulate=False, compensated=False, tile=0, max_pairs=0, workspace=None,
           stats=False, profile=False, seg_records=0, tile_mask=None, splat_variant=0,
           palette_absorb=None, kernel=KERNEL_GAUSS2D, emission_is_source=0, split_pixels=0):
    """Render into image (planar float32 [3, H, W] device tensor; allocated
    if None).  Returns the image, or (image, stats dict) with stats=True
    (profile=1 adds per-stage milliseconds to the stats, profile=2 also the
    composited-contribution counts)."""
    import torch
    P, cs, prm, dev = _setup(parts, cam, species, max_pairs, workspace, sigma_over_h=sigma_over_h,
                             trunc_f=trunc_f, accumulate=accumulate, compensated=compensated,
                             tile=tile, profile=profile, seg_records=seg_records,
                             tile_mask=tile_mask, splat_variant=splat_variant, kernel=kernel,
                             emission_is_source=emission_is_source, split_pixels=split_pixels)
    stats = stats or profile
    if image is None:
        image = torch.empty((3, cs.height, cs.width), dtype=torch.float32, device=dev)
    if image.dtype != torch.float32 or not image.is_contiguous() or \
            tuple(image.shape) != (3, cs.height, cs.width):
        raise ValueError("image must be contiguous float32 [3, H, W]")
    cm = colourmap_struct(palette, palette_absorb)
    img = Image(C.c_void_p(image.data_ptr()), cs.width, cs.height)
    st = Stats()
    if stats:
        prm.stats = C.pointer(st)
    _check(_lib().splotch_render(C.byref(P), C.byref(cs), C.byref(cm), C.byref(prm),
                                 C.byref(img)), "splotch_render")
    return (image, st.as_dict()) if stats else image


def render_static(parts: dict, cam, palette, species, image, *, sigma_over_h=1.0, trunc_f=2.0,
                  accumulate=False, compensated=False, tile=0, stats=False, seg_records=0,
                  tile_mask=None, splat_variant=0, palette_absorb=None, kernel=KERNEL_GAUSS2D,
                  emission_is_source=0):
    """splotch_render_static: the render with the library's static scratch
    buffer as its workspace (no device allocation anywhere in the call;
    image must be given).  Returns the image, or (image, stats dict)."""
    import torch
    P = particles_struct(parts)
    cs = cam if isinstance(cam, CameraS) else camera_struct(cam)
    prm = params_struct(species, sigma_over_h=sigma_over_h, trunc_f=trunc_f,
                        accumulate=accumulate, compensated=compensated, tile=tile,
                        seg_records=seg_records, tile_mask=tile_mask,
                        splat_variant=splat_variant, kernel=kernel,
                        emission_is_source=emission_is_source)
    dev = parts["x"].device
    prm.stream = _stream_ptr(dev)
    if image.dtype != torch.float32 or not image.is_contiguous() or \
            tuple(image.shape) != (3, cs.height, cs.width):
        raise ValueError("image must be contiguous float32 [3, H, W]")
    cm = colourmap_struct(palette, palette_absorb)
    img = Image(C.c_void_p(image.data_ptr()), cs.width, cs.height)
    st = Stats()
    if stats:
        prm.stats = C.pointer(st)
    _check(_lib().splotch_render_static(C.byref(P), C.byref(cs), C.byref(cm), C.byref(prm),
                                        C.byref(img)), "splotch_render_static")
    return (image, st.as_dict()) if stats else image


def host_particles_struct(parts: dict) -> Particles:
    """parts: dict of contiguous host (CPU) tensors with the fields of
    particles_struct; pinned memory lets the copies overlap the work."""
    import torch
    for k, t in parts.items():
        if t is not None and t.device.type != "cpu":
            raise ValueError(f"host particle field {k} must be a CPU tensor")
    P = Particles()
    n = int(parts["x"].numel())
    for k in ("x", "y", "z", "h", "value", "rho0", "value_g", "value_b"):
        t = parts.get(k)
        if t is not None and (t.dtype != torch.float32 or not t.is_contiguous() or
                              t.numel() != n):
            raise ValueError(f"particle field {k} must be contiguous float32 of length {n}")
    P.n = n
    P.x, P.y, P.z, P.h, P.value = (_ptr(parts[k]) for k in ("x", "y", "z", "h", "value"))
    P.rho0 = _ptr(parts.get("rho0"))
    P.species = _ptr(parts.get("species"))
    P.value_g = _ptr(parts.get("value_g"))
    P.value_b = _ptr(parts.get("value_b"))
    return P


def render_stream(host_parts: dict, cam, palette, species, image=None, *, subset=1 << 22,
                  slab=1 << 24, device="cuda", stats=False, palette_absorb=None, **kw):
    """splotch_render_stream: render a host-resident particle set (dict of
    CPU tensors, ideally pinned) in subsets of `subset` particles and, with
    ordered species, depth slabs of at most `slab` particles.  Returns the
    image (or (image, stats))."""
    import torch
    P = host_particles_struct(host_parts)
    cs = cam if isinstance(cam, CameraS) else camera_struct(cam)
    prm = params_struct(species, **kw)
    out = C.c_size_t(0)
    _check(_lib().splotch_stream_workspace_size(C.byref(P), int(subset), int(slab), C.byref(cs),
                                                C.byref(prm), C.byref(out)),
           "splotch_stream_workspace_size")
    ws = get_workspace(int(out.value), torch.device(device))
    prm.workspace = C.c_void_p(ws.data_ptr())
    prm.workspace_bytes = int(out.value)
    prm.stream = _stream_ptr(torch.device(device))
    if image is None:
        image = torch.empty((3, cs.height, cs.width), dtype=torch.float32, device=device)
    cm = colourmap_struct(palette, palette_absorb)
    img = Image(C.c_void_p(image.data_ptr()), cs.width, cs.height)
    st = Stats()
    if stats:
        prm.stats = C.pointer(st)
    _check(_lib().splotch_render_stream(C.byref(P), int(subset), int(slab), C.byref(cs),
                                        C.byref(cm), C.byref(prm), C.byref(img)),
           "splotch_render_stream")
    return (image, st.as_dict()) if stats else image


def project(parts: dict, cam, species, *, sigma_over_h=1.0, trunc_f=2.0, tile=0,
            workspace=None):
    """Per-particle stage outputs: dict of device tensors status (int8),
    bbox (int32 [n,4]), spec (float32 [n,3]), key (uint32 as int32 view
    bits), ntiles (uint32 bits in int32)."""
    import torch
    P, cs, prm, dev = _setup(parts, cam, species, 1, workspace, sigma_over_h=sigma_over_h,
                             trunc_f=trunc_f, tile=tile)
    n = P.n
    out = dict(status=torch.empty(n, dtype=torch.int8, device=dev),
               bbox=torch.empty((n, 4), dtype=torch.int32, device=dev),
               spec=torch.empty((n, 3), dtype=torch.float32, device=dev),
               key=torch.empty(n, dtype=torch.int32, device=dev),
               ntiles=torch.empty(n, dtype=torch.int32, device=dev))
    st = Stats()
    prm.stats = C.pointer(st)
    _check(_lib().splotch_project(C.byref(P), C.byref(cs), C.byref(prm), _ptr(out["status"]),
                                  _ptr(out["bbox"]), _ptr(out["spec"]), _ptr(out["key"]),
                                  _ptr(out["ntiles"])), "splotch_project")
    out["stats"] = st.as_dict()
    return out


def bin_pairs(parts: dict, cam, species, *, sigma_over_h=1.0, trunc_f=2.0, tile=0,
              max_pairs=0, workspace=None, split_pixels=0):
    """Per-tile particle lists: (tile_start, tile_end, pair_particle) device
    int32 tensors (uint32 bits) and the pair count."""
    import torch
    P, cs, prm, dev = _setup(parts, cam, species, max_pairs, workspace, sigma_over_h=sigma_over_h,
                             trunc_f=trunc_f, tile=tile, split_pixels=split_pixels)
    T = tile or 16
    nt = ((cs.width + T - 1) // T) * ((cs.height + T - 1) // T)
    cap = max_pairs or (4 * P.n + 65536)
    ts = torch.empty(nt, dtype=torch.int32, device=dev)
    te = torch.empty(nt, dtype=torch.int32, device=dev)
    pp = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
    npairs = C.c_int64(0)
    _check(_lib().splotch_bin(C.byref(P), C.byref(cs), C.byref(prm), _ptr(ts), _ptr(te),
                              _ptr(pp), int(cap), C.byref(npairs)), "splotch_bin")
    return ts, te, pp[: npairs.value], int(npairs.value)


_streams: dict = {}


def _side_stream(device):
    """A created (non-null) stream per device for graph capture and replay."""
    import torch
    key = str(device)
    if key not in _streams:
        _streams[key] = torch.cuda.Stream(device=device)
    return _streams[key]


def render_batch(parts: dict, cams, palette, species, images=None, *, graph=False,
                 sigma_over_h=1.0, trunc_f=2.0, accumulate=False, compensated=False, tile=0,
                 max_pairs=0, seg_records=0, workspace=None, stats=False, splat_variant=0,
                 streams=1, palette_absorb=None, kernel=KERNEL_GAUSS2D, emission_is_source=0,
                 split_pixels=0, persistent=False):
    """Render several camera views of one particle set (splotch_render_batch).
    images: list of [3, H_v, W_v] float32 device tensors (allocated if None).
    graph=True captures the batch into a HIP graph on first use and replays
    it while every argument stays the same (same tensors, same settings).
    streams: views in flight at once (1..4); the workspace holds that many
    view layouts.  Returns images, or (images, per-view stats) with
    stats=True."""
    import torch
    P = particles_struct(parts)
    dev = parts["x"].device
    nv = len(cams)
    if not 1 <= nv <= MAX_VIEWS:
        raise ValueError(f"1..{MAX_VIEWS} views")
    cs = (CameraS * nv)(*[c if isinstance(c, CameraS) else camera_struct(c) for c in cams])
    prm = params_struct(species, sigma_over_h=sigma_over_h, trunc_f=trunc_f,
                        accumulate=accumulate, compensated=compensated, tile=tile,
                        seg_records=seg_records, splat_variant=splat_variant,
                        batch_streams=streams, kernel=kernel,
                        emission_is_source=emission_is_source, split_pixels=split_pixels,
                        batch_persistent=1 if persistent else 0)
    T = tile or 16
    big = max(range(nv), key=lambda v: (-(-cs[v].width // T)) * (-(-cs[v].height // T)))
    if workspace is None:
        one = workspace_bytes(P.n, cs[big], prm, max_pairs or 0)
        need = (one + 255) // 256 * 256 * max(1, int(streams))
        workspace = get_workspace(need, dev)
        nbytes = need
    else:
        nbytes = int(workspace.numel())
    prm.workspace = C.c_void_p(workspace.data_ptr())
    prm.workspace_bytes = nbytes
    if images is None:
        images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device=dev) for c in cs]
    for im, c in zip(images, cs):
        if im.dtype != torch.float32 or not im.is_contiguous() or \
                tuple(im.shape) != (3, c.height, c.width):
            raise ValueError("each image must be contiguous float32 [3, H, W] of its camera")
    ims = (Image * nv)(*[Image(C.c_void_p(im.data_ptr()), c.width, c.height)
                         for im, c in zip(images, cs)])
    cm = colourmap_struct(palette, palette_absorb)
    st = (Stats * nv)()
    if stats:
        prm.stats = C.cast(st, C.POINTER(Stats))
    cur = torch.cuda.current_stream(dev)
    if graph:
        side = _side_stream(dev)
        side.wait_stream(cur)
        prm.stream = C.c_void_p(side.cuda_stream)
    else:
        prm.stream = C.c_void_p(cur.cuda_stream)
    code = _lib().splotch_render_batch(C.byref(P), nv, cs, C.byref(cm), C.byref(prm), ims,
                                       1 if graph else 0)
    if graph:
        cur.wait_stream(side)
    _check(code, "splotch_render_batch")
    return (images, [s.as_dict() for s in st]) if stats else images


def graph_cache_clear() -> int:
    return int(_lib().splotch_graph_cache_clear())


@dataclass
class SpeciesParams:
    vmin: float = 0.0
    vmax: float = 0.0
    log_scale: int = 0
    brightness: float = 1.0
    absorption: float = 0.0
    mode: int = ADDITIVE
    colour: int = COLOUR_PALETTE


def scene_to_device(scene, device="cuda"):
    """Copy a host synth.Scene's particle arrays to device tensors."""
    import torch

    def t(a, dt):
        return None if a is None else torch.from_numpy(a).to(device=device, dtype=dt).contiguous()
    parts = dict(x=t(scene.x, torch.float32), y=t(scene.y, torch.float32),
                 z=t(scene.z, torch.float32), h=t(scene.h, torch.float32),
                 value=t(scene.value, torch.float32))
    if scene.rho0 is not None:
        parts["rho0"] = t(scene.rho0, torch.float32)
    if scene.species is not None:
        parts["species"] = t(scene.species, torch.uint8)
    for k in ("value_g", "value_b"):
        a = getattr(scene, k, None)
        if a is not None:
            parts[k] = t(a, torch.float32)
    pal = torch.from_numpy(scene.palette).to(device=device, dtype=torch.float32).contiguous()
    return parts, pal


def scene_options(scene, device="cuda") -> dict:
    """Render keyword arguments a host synth.Scene carries besides its
    particles, palette and species: footprint scale and cut, column kernel,
    emission reading and the absorption table (copied to the device)."""
    import torch
    pa = getattr(scene, "palette_absorb", None)
    return dict(sigma_over_h=float(scene.sigma_over_h), trunc_f=float(scene.trunc_f),
                kernel=int(getattr(scene, "kernel", KERNEL_GAUSS2D)),
                emission_is_source=int(getattr(scene, "emission_is_source", 0)),
                palette_absorb=None if pa is None else
                torch.from_numpy(np.ascontiguousarray(pa, np.float32)).to(device))
