"""FP64 CPU oracle for the Splotch render -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path never calls it.

The arithmetic lives in ``splotch_oracle.c`` (plain C, double precision,
compiled with ``-ffp-contract=off``); this module builds it with gcc and
marshals numpy arrays.  Every function cites the part of the paper it
follows in the C source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "splotch_oracle.c")
_LIB = os.path.join(_HERE, "libsplotch_oracle.so")
# A test may point the wrapper at a deliberately broken build of the same
# source to show that the pins detect the breakage.
_LIB_OVERRIDE = os.environ.get("SPLOTCH_ORACLE_LIB")

VISIBLE, INVALID, DEPTH, OFFSCREEN = 0, 1, 2, 3


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no FMA contraction, IEEE semantics)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = f"{_LIB}.{os.getpid()}.tmp"  # concurrent builders do not share it
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math",
                               "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            _lib = C.CDLL(_LIB_OVERRIDE)
            _declare(_lib)
            return _lib
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = C.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = C.c_void_p
I64 = C.c_int64
I32 = C.c_int
F32 = C.c_float
MAXS = 8


class OrcParticles(C.Structure):
    _fields_ = [("n", C.c_int64), ("x", P), ("y", P), ("z", P), ("h", P), ("value", P),
                ("rho0", P), ("value_g", P), ("value_b", P), ("species", P)]


class OrcSettings(C.Structure):
    _fields_ = [("ns", C.c_int), ("vmin", C.c_float * MAXS), ("vmax", C.c_float * MAXS),
                ("bright", C.c_float * MAXS), ("absorb", C.c_float * MAXS),
                ("log_scale", C.c_int * MAXS), ("mode", C.c_int * MAXS),
                ("colour", C.c_int * MAXS), ("sigma_over_h", C.c_float),
                ("trunc_f", C.c_float), ("kernel", C.c_int), ("emission_is_source", C.c_int),
                ("K", C.c_int), ("KA", C.c_int), ("pal", P), ("pal_abs", P)]


def _declare(L):
    PP, PS = C.POINTER(OrcParticles), C.POINTER(OrcSettings)
    L.orc_value_range.restype = None
    L.orc_value_range.argtypes = [PP, PS, P, P]
    L.orc_normalise.restype = C.c_double
    L.orc_normalise.argtypes = [F32, F32, F32, I32]
    L.orc_palette.restype = None
    L.orc_palette.argtypes = [C.c_double, I32, P, P]
    L.orc_project.restype = None
    L.orc_project.argtypes = [PP, PS, P, I32, I32, I32, I32, P, P, P, P, P, P]
    L.orc_render.restype = I64
    L.orc_render.argtypes = [PP, PS, P, I32, I32, I32, P, P]
    L.orc_render_rows.restype = I64
    L.orc_render_rows.argtypes = [PP, PS, P, I32, I32, I32, I32, P, P]
    L.orc_threads.restype = I32
    L.orc_threads.argtypes = []
    L.orc_render_pixels.restype = I64
    L.orc_render_pixels.argtypes = [PP, PS, P, I32, I32, I32, I64, P, P, P, P]
    L.orc_raymarch.restype = I32
    L.orc_raymarch.argtypes = [I64, P, P, P, P, P, P, P, P, I32, I32, F32, F32, I32, I32, P, P]


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f32(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float32)


def cam_array(cam) -> np.ndarray:
    return np.concatenate([np.asarray(cam.eye, np.float32), np.asarray(cam.right, np.float32),
                           np.asarray(cam.up, np.float32), np.asarray(cam.fwd, np.float32),
                           np.array([cam.focal_px, cam.px_per_unit, cam.z_near, cam.z_far],
                                    np.float32)]).astype(np.float32)


class _Marshalled:
    """Particle and settings structs for one scene; keeps the arrays they
    point to alive."""

    def __init__(self, scene):
        sp = None if scene.species is None else np.ascontiguousarray(scene.species, np.uint8)
        self.keep = [_f32(scene.x), _f32(scene.y), _f32(scene.z), _f32(scene.h),
                     _f32(scene.value), _f32(scene.rho0), _f32(getattr(scene, "value_g", None)),
                     _f32(getattr(scene, "value_b", None)), sp]
        x, y, z, h, v, r0, vg, vb, spc = self.keep
        self.parts = OrcParticles(scene.n, _p(x), _p(y), _p(z), _p(h), _p(v), _p(r0), _p(vg),
                                  _p(vb), _p(spc))
        st = OrcSettings()
        sps = scene.species_params
        st.ns = len(sps)
        for k, s in enumerate(sps):
            st.vmin[k], st.vmax[k] = float(s.vmin), float(s.vmax)
            st.bright[k], st.absorb[k] = float(s.brightness), float(s.absorption)
            st.log_scale[k], st.mode[k] = int(s.log_scale), int(s.mode)
            st.colour[k] = int(getattr(s, "colour", 0))
            if st.colour[k] == 1 and (vg is None or vb is None):
                raise ValueError("vector-coloured species need value_g and value_b")
        st.sigma_over_h, st.trunc_f = float(scene.sigma_over_h), float(scene.trunc_f)
        st.kernel = int(getattr(scene, "kernel", 0))
        st.emission_is_source = int(getattr(scene, "emission_is_source", 0))
        pal = np.ascontiguousarray(scene.palette, np.float32)
        pa = getattr(scene, "palette_absorb", None)
        pa = None if pa is None else np.ascontiguousarray(pa, np.float32)
        self.keep += [pal, pa]
        st.K, st.pal = pal.shape[0], _p(pal)
        st.KA, st.pal_abs = (0, None) if pa is None else (pa.shape[0], _p(pa))
        self.st = st
        self.cam = cam_array(scene.camera)

    def args(self):
        return C.byref(self.parts), C.byref(self.st)


def value_range(scene):
    m = _Marshalled(scene)
    ns = m.st.ns
    lo = np.zeros(ns, np.float32)
    hi = np.zeros(ns, np.float32)
    lib().orc_value_range(*m.args(), _p(lo), _p(hi))
    return lo, hi


def normalise(value, vmin, vmax, log_scale):
    return lib().orc_normalise(float(value), float(vmin), float(vmax), int(log_scale))


def palette_lookup(t, pal):
    pal = np.ascontiguousarray(pal, np.float32)
    out = np.zeros(3, np.float64)
    lib().orc_palette(float(t), pal.shape[0], _p(pal), _p(out))
    return out


def project(scene, tile=16):
    """Per-particle projection fields (status, bbox, binary32 membership
    fields, depth key, tile count and the exact FP64 u, v, sigma_s, z_c)."""
    m = _Marshalled(scene)
    n = scene.n
    cam = scene.camera
    out = dict(status=np.zeros(n, np.int8), bbox=np.zeros((n, 4), np.int32),
               spec=np.zeros((n, 3), np.float32), key=np.zeros(n, np.uint32),
               ntiles=np.zeros(n, np.uint32), cont=np.zeros((n, 4), np.float64))
    lib().orc_project(*m.args(), _p(m.cam), cam.projection, cam.width, cam.height, tile,
                      _p(out["status"]), _p(out["bbox"]), _p(out["spec"]), _p(out["key"]),
                      _p(out["ntiles"]), _p(out["cont"]))
    return out


def render(scene, img_in=None) -> np.ndarray:
    """FP64 image, planar [3][H][W] (single thread)."""
    m = _Marshalled(scene)
    cam = scene.camera
    out = np.zeros((3, cam.height, cam.width), np.float64)
    iin = None if img_in is None else np.ascontiguousarray(img_in, np.float64)
    lib().orc_render(*m.args(), _p(m.cam), cam.projection, cam.width, cam.height, _p(iin),
                     _p(out))
    return out


def render_rows(scene, img_in=None, band=16) -> np.ndarray:
    """The same image as render(), with bands of `band` rows painted in
    parallel by the OpenMP threads (OMP_NUM_THREADS)."""
    m = _Marshalled(scene)
    cam = scene.camera
    out = np.zeros((3, cam.height, cam.width), np.float64)
    iin = None if img_in is None else np.ascontiguousarray(img_in, np.float64)
    lib().orc_render_rows(*m.args(), _p(m.cam), cam.projection, cam.width, cam.height,
                          int(band), _p(iin), _p(out))
    return out


def threads() -> int:
    """OpenMP threads the oracle's parallel parts use."""
    return int(lib().orc_threads())


def render_pixels(scene, pi, pj, in_px=None) -> np.ndarray:
    """FP64 values (npx, 3) at the sample pixels (pi[k], pj[k]).  The scan
    over particles runs on all OpenMP threads; the composite is the same
    for any thread count."""
    m = _Marshalled(scene)
    cam = scene.camera
    pi = np.ascontiguousarray(pi, np.int32)
    pj = np.ascontiguousarray(pj, np.int32)
    out = np.zeros((pi.shape[0], 3), np.float64)
    iin = None if in_px is None else np.ascontiguousarray(in_px, np.float64)
    lib().orc_render_pixels(*m.args(), _p(m.cam), cam.projection, cam.width, cam.height,
                            pi.shape[0], _p(pi), _p(pj), _p(iin), _p(out))
    return out


def raymarch(x, y, z, h, rho0, E, A, cam, sigma_over_h=1.0, trunc_f=2.0, steps_per_sigma=120,
             img_in=None, kernel=0) -> np.ndarray:
    """Brute-force RK4 integration of Eq. (1) through the summed density,
    orthographic cameras only.  E, A: (n, 3) per-particle emission and
    absorption.  kernel 0: density kept on rays within f sigma of the
    centre; kernel 1: density cut to the sphere of radius f sigma.
    Returns planar [3][H][W] FP64."""
    x, y, z, h = (_f32(a) for a in (x, y, z, h))
    rho0 = np.ascontiguousarray(rho0, np.float64)
    E = np.ascontiguousarray(E, np.float64)
    A = np.ascontiguousarray(A, np.float64)
    W, H = cam.width, cam.height
    out = np.zeros((3, H, W), np.float64)
    iin = None if img_in is None else np.ascontiguousarray(img_in, np.float64)
    ca = cam_array(cam)
    lib().orc_raymarch(x.shape[0], _p(x), _p(y), _p(z), _p(h), _p(rho0), _p(E), _p(A), _p(ca),
                       W, H, sigma_over_h, trunc_f, int(kernel), steps_per_sigma, _p(iin),
                       _p(out))
    return out


def rel_linf(gpu: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Per-channel relative L-infinity error max|g - o| / max|o| over the
    image (planar [3][...])."""
    g = np.asarray(gpu, np.float64).reshape(3, -1)
    o = np.asarray(ref, np.float64).reshape(3, -1)
    den = np.abs(o).max(axis=1)
    den = np.where(den > 0, den, 1.0)
    return np.abs(g - o).max(axis=1) / den
