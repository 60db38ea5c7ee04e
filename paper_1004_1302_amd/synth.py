"""Seeded synthetic particle sets, palettes and cameras.

This module only constructs inputs: particle positions, smoothing lengths,
scalar values, species tags, a colour palette and camera frames.  It holds
none of the rendering arithmetic and is shared by the GPU path, the oracle
tests and the benchmark.

The paper renders N-body extracts (1M/10M/100M/850M particles) and the
Millennium II snapshot (Section 4).  Those data sets are not available, so
these generators stand in for them with clustered distributions of the same
kind: Plummer spheres over a uniform background, NFW halos with a power-law
mass function, and a lognormal density field sampled per cell.

All host generators use numpy's PCG64 with an explicit seed.  The
large-scale lognormal-field generator is written with torch so that it can
run on the GPU (a billion particles); its random stream depends on the
device it runs on, and callers copy its output to wherever it is checked.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

ORTHO = 0
PERSPECTIVE = 1
ADDITIVE = 0
ORDERED = 1
COLOUR_PALETTE = 0   # a scalar through the colour look-up table
COLOUR_VECTOR = 1    # three vector components map to r, g, b
KERNEL_GAUSS2D = 0   # Gaussian column cut at impact parameter f sigma
KERNEL_TRUNC3D = 1   # Gaussian density cut to the sphere r <= f sigma


# --------------------------------------------------------------------------
# Cameras and palettes
# --------------------------------------------------------------------------
@dataclass
class Camera:
    """Pinhole or orthographic camera with an FP32 orthonormal frame."""

    projection: int
    width: int
    height: int
    eye: np.ndarray
    right: np.ndarray
    up: np.ndarray
    fwd: np.ndarray
    focal_px: float = 0.0
    px_per_unit: float = 0.0
    z_near: float = 1e-3
    z_far: float = 1e30


def look_at(eye, at, up, projection, width, height, fov_x_deg=60.0,
            px_per_unit=None, z_near=1e-3, z_far=1e30) -> Camera:
    """Build a camera frame looking from ``eye`` towards ``at``.

    ``fwd`` points from the eye into the scene, ``right`` = up x fwd is the
    screen x axis and ``up`` = fwd x right the screen y axis, so that
    right x up = fwd (row 0 of the image is the bottom row).  Perspective
    cameras use a horizontal field of view; the focal length in pixels is
    (W/2)/tan(fov_x/2).
    """
    eye = np.asarray(eye, np.float64)
    at = np.asarray(at, np.float64)
    upv = np.asarray(up, np.float64)
    f = at - eye
    f /= np.linalg.norm(f)
    r = np.cross(upv, f)
    r /= np.linalg.norm(r)
    u = np.cross(f, r)
    cam = Camera(projection, int(width), int(height),
                 eye.astype(np.float32), r.astype(np.float32),
                 u.astype(np.float32), f.astype(np.float32),
                 z_near=float(z_near), z_far=float(z_far))
    if projection == PERSPECTIVE:
        cam.focal_px = float(np.float32((width / 2.0) / math.tan(math.radians(fov_x_deg) / 2.0)))
    else:
        cam.px_per_unit = float(np.float32(px_per_unit if px_per_unit is not None else 1.0))
    return cam


def ortho_unit_square(width=256, height=256) -> Camera:
    """Orthographic view along +z of the unit square [0,1]^2 (x right, y up)."""
    return Camera(ORTHO, width, height,
                  eye=np.array([0.5, 0.5, -1.0], np.float32),
                  right=np.array([1.0, 0.0, 0.0], np.float32),
                  up=np.array([0.0, 1.0, 0.0], np.float32),
                  fwd=np.array([0.0, 0.0, 1.0], np.float32),
                  px_per_unit=float(width), z_near=0.0, z_far=10.0)


def orbit_cameras(n_views, seed, sizes, centre=(0.5, 0.5, 0.5), radius=2.0, fov_x_deg=60.0,
                  z_near=0.05, z_far=100.0):
    """Perspective cameras at seeded random points of a sphere of `radius`
    around `centre`, looking at it, with resolutions drawn from `sizes`
    (a list of (width, height))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    cams = []
    for _ in range(n_views):
        th = math.acos(rng.uniform(-1.0, 1.0))
        ph = rng.uniform(0.0, 2.0 * math.pi)
        eye = np.asarray(centre, np.float64) + radius * np.array(
            [math.sin(th) * math.cos(ph), math.sin(th) * math.sin(ph), math.cos(th)])
        w, h = sizes[int(rng.integers(0, len(sizes)))]
        up = (0.0, 1.0, 0.0) if abs(math.cos(th)) < 0.9 else (1.0, 0.0, 0.0)
        cams.append(look_at(eye, centre, up, PERSPECTIVE, w, h, fov_x_deg, z_near=z_near,
                            z_far=z_far))
    return cams


def palette(n_entries: int = 256) -> np.ndarray:
    """A project-defined analytic RGB ramp (black -> red -> yellow -> white,
    with a blue lift in the mid range), as ``(K, 3)`` float32."""
    t = np.linspace(0.0, 1.0, n_entries)
    r = np.clip(1.6 * t, 0.0, 1.0)
    g = np.clip(1.6 * t - 0.45, 0.0, 1.0)
    b = np.clip(0.35 * np.sin(np.pi * t) + np.clip(2.0 * t - 1.2, 0.0, 1.0), 0.0, 1.0)
    return np.stack([r, g, b], axis=1).astype(np.float32)


# --------------------------------------------------------------------------
# Particle sets
# --------------------------------------------------------------------------
@dataclass
class Species:
    vmin: float = 0.0
    vmax: float = 0.0          # vmin >= vmax: range found from the data
    log_scale: int = 0
    brightness: float = 1.0
    absorption: float = 0.0
    mode: int = ADDITIVE
    colour: int = COLOUR_PALETTE


@dataclass
class Scene:
    """A particle set (SoA, float32 numpy) plus the render settings."""

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    h: np.ndarray
    value: np.ndarray
    camera: Camera
    species_params: list = field(default_factory=lambda: [Species()])
    species: np.ndarray | None = None   # uint8 tag per particle
    rho0: np.ndarray | None = None      # per-particle density amplitude
    palette: np.ndarray = field(default_factory=palette)
    sigma_over_h: float = 1.0
    trunc_f: float = 2.0
    name: str = ""
    value_g: np.ndarray | None = None   # 2nd and 3rd vector components
    value_b: np.ndarray | None = None   # (vector-coloured species)
    palette_absorb: np.ndarray | None = None  # absorption palette; None = palette
    kernel: int = KERNEL_GAUSS2D
    emission_is_source: int = 0

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def subset(self, idx) -> "Scene":
        def s(a):
            return None if a is None else np.ascontiguousarray(a[idx])
        return Scene(s(self.x), s(self.y), s(self.z), s(self.h), s(self.value),
                     self.camera, self.species_params, s(self.species), s(self.rho0),
                     self.palette, self.sigma_over_h, self.trunc_f, self.name,
                     s(self.value_g), s(self.value_b), self.palette_absorb, self.kernel,
                     self.emission_is_source)


def _lognormal_mean(rng, mean, sigma, n):
    # mean of a lognormal is exp(mu + sigma^2/2)
    mu = math.log(mean) - 0.5 * sigma * sigma
    return rng.lognormal(mu, sigma, n)


def _plummer_offsets(rng, n, a, rcut_over_a=10.0):
    # enclosed mass fraction M(r) = r^3/(r^2+a^2)^{3/2}; invert M(r)=u
    umax = rcut_over_a ** 3 / (rcut_over_a ** 2 + 1.0) ** 1.5
    u = rng.uniform(0.0, umax, n)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    return r[:, None] * _iso_dirs(rng, n)


def _iso_dirs(rng, n):
    cz = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - cz * cz)
    return np.stack([s * np.cos(ph), s * np.sin(ph), cz], axis=1)


def plummer_mix(n=100_000, seed=1, n_spheres=10, a=0.02, h_mean=0.005, h_sigma=0.5,
                width=256, height=256, camera=None, brightness=1.0) -> Scene:
    """Uniform particles in [0,1]^3 mixed 50/50 with ``n_spheres`` Plummer
    spheres of scale ``a`` at seeded centres; lognormal smoothing lengths
    and scalar values; all additive; orthographic view along z."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_u = n // 2
    n_p = n - n_u
    pos_u = rng.uniform(0.0, 1.0, (n_u, 3))
    centres = rng.uniform(0.1, 0.9, (n_spheres, 3))
    per = np.full(n_spheres, n_p // n_spheres)
    per[: n_p - per.sum()] += 1
    pos_p = np.concatenate([c + _plummer_offsets(rng, k, a) for c, k in zip(centres, per)])
    pos = np.concatenate([pos_u, pos_p])
    h = _lognormal_mean(rng, h_mean, h_sigma, n)
    val = rng.lognormal(0.0, 1.0, n)
    cam = camera if camera is not None else ortho_unit_square(width, height)
    sp = [Species(brightness=brightness, mode=ADDITIVE)]
    return Scene(pos[:, 0].astype(np.float32), pos[:, 1].astype(np.float32),
                 pos[:, 2].astype(np.float32), h.astype(np.float32),
                 val.astype(np.float32), cam, sp, name=f"plummer_mix_{n}")


def _nfw_x_of_m(c):
    # tabulated inverse of m(x) = ln(1+x) - x/(1+x) on [0, c]
    xs = np.concatenate([[0.0], np.geomspace(1e-6, c, 4096)])
    ms = np.log1p(xs) - xs / (1.0 + xs)
    return xs, ms


def nfw_halos(n=10_000_000, seed=2, n_halos=1000, box=100.0, bg_frac=0.2,
              slope=-1.9, mass_range=(1.0, 1000.0), conc=10.0, rvir_max=5.0,
              grid=256, width=1920, height=1080, fov_x_deg=60.0,
              gas_frac=0.5, brightness=None, camera=None) -> Scene:
    """NFW halos with a power-law mass function plus a uniform background in
    a box of side ``box``; two species: gas (depth-ordered, absorption equal
    to emission) and dark matter (additive).  Smoothing lengths follow the
    local density, h = l (rho/mean)^{-1/3} clipped to [0.01, 2]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_bg = int(round(n * bg_frac))
    n_h = n - n_bg
    m0, m1 = mass_range
    g = slope + 1.0
    u = rng.uniform(0.0, 1.0, n_halos)
    mass = (m0 ** g + u * (m1 ** g - m0 ** g)) ** (1.0 / g)
    counts = np.floor(n_h * mass / mass.sum()).astype(np.int64)
    counts[: n_h - counts.sum()] += 1
    centres = rng.uniform(0.0, box, (n_halos, 3))
    rvir = rvir_max * (mass / mass.max()) ** (1.0 / 3.0)
    xs, ms = _nfw_x_of_m(conc)
    hidx = np.repeat(np.arange(n_halos), counts)
    q = rng.uniform(0.0, ms[-1], n_h)
    xr = np.interp(q, ms, xs)
    r = xr * (rvir[hidx] / conc)
    pos_h = centres[hidx] + r[:, None] * _iso_dirs(rng, n_h)
    pos_bg = rng.uniform(0.0, box, (n_bg, 3))
    pos = np.concatenate([pos_h, pos_bg])
    # local density from nearest-grid-point counts
    cell = np.clip((pos / box * grid).astype(np.int64), 0, grid - 1)
    flat = (cell[:, 0] * grid + cell[:, 1]) * grid + cell[:, 2]
    cnt = np.bincount(flat, minlength=grid ** 3)
    rho = cnt[flat] / (n / grid ** 3)
    ell = box / n ** (1.0 / 3.0)
    h = np.clip(ell * rho ** (-1.0 / 3.0), 0.01, 2.0)
    species = (rng.uniform(0.0, 1.0, n) >= gas_frac).astype(np.uint8)  # 0 gas, 1 dm
    if camera is None:
        camera = look_at((box / 2, box / 2, -box), (box / 2, box / 2, box / 2), (0, 1, 0),
                         PERSPECTIVE, width, height, fov_x_deg, z_near=1.0, z_far=10 * box)
    if brightness is None:
        brightness = 0.15
    sp = [Species(log_scale=1, brightness=brightness, absorption=brightness, mode=ORDERED),
          Species(log_scale=1, brightness=brightness, absorption=0.0, mode=ADDITIVE)]
    return Scene(pos[:, 0].astype(np.float32), pos[:, 1].astype(np.float32),
                 pos[:, 2].astype(np.float32), h.astype(np.float32),
                 rho.astype(np.float32), camera, sp, species=species,
                 name=f"nfw_halos_{n}")


def lognormal_field(n_target=1_000_000_000, grid=512, sigma=1.5, box=100.0, seed=3,
                    width=4096, height=4096, fov_x_deg=60.0, gas_frac=0.5,
                    brightness=None, device="cpu", with_rho0=True):
    """Particles drawn from a lognormal density field on a ``grid``^3 mesh
    with per-cell Poisson sampling (torch; runs on the GPU for 1e9).

    The Gaussian field has power spectrum P(k) ~ k^-2 and unit variance;
    delta = exp(sigma g - sigma^2/2) has mean one.  Each cell receives
    Poisson(lambda delta) particles at uniform positions inside the cell,
    with lambda = n_target / grid^3.  Cells are enumerated with z fastest,
    so particles adjacent along z are adjacent in memory.  Returns a dict of
    torch tensors on ``device`` plus the camera and species settings.
    """
    import torch

    gen = torch.Generator(device=device)
    gen.manual_seed(seed)
    dev = torch.device(device)
    k1 = torch.fft.fftfreq(grid, device=dev)
    kz = torch.fft.rfftfreq(grid, device=dev)
    noise = torch.randn((grid, grid, grid), generator=gen, device=dev, dtype=torch.float32)
    fk = torch.fft.rfftn(noise)
    del noise
    k2 = (k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + kz[None, None, :] ** 2)
    amp = torch.where(k2 > 0, k2.rsqrt(), torch.zeros_like(k2))   # sqrt(P(k)) ~ 1/k
    fk *= amp
    del amp, k2
    g = torch.fft.irfftn(fk, s=(grid, grid, grid))
    del fk
    g = (g - g.mean()) / g.std()
    delta = torch.exp(sigma * g - 0.5 * sigma * sigma)
    del g
    lam = n_target / grid ** 3
    ncell = torch.poisson(delta * lam, generator=gen).to(torch.int32).reshape(-1)
    del delta
    n = int(ncell.sum().item())
    cell_id = torch.repeat_interleave(torch.arange(grid ** 3, device=dev, dtype=torch.int32),
                                      ncell.to(torch.int64), output_size=n)
    dcell = box / grid
    out = {}
    cz = cell_id % grid
    cy = (cell_id // grid) % grid
    cx = cell_id // (grid * grid)
    for name, c in (("x", cx), ("y", cy), ("z", cz)):
        r = torch.rand(n, generator=gen, device=dev, dtype=torch.float32)
        out[name] = ((c.to(torch.float32) + r) * dcell).contiguous()
        del r
    del cx, cy, cz
    nc = ncell[cell_id.to(torch.int64)].to(torch.float32)
    del cell_id, ncell
    out["h"] = torch.clamp(dcell * nc.pow(-1.0 / 3.0), dcell / 8, 4 * dcell).contiguous()
    out["value"] = nc.contiguous()
    del nc
    out["species"] = (torch.rand(n, generator=gen, device=dev) >= gas_frac).to(torch.uint8)
    if with_rho0:
        out["rho0"] = torch.ones(n, device=dev, dtype=torch.float32)
    camera = look_at((box / 2, box / 2, -box), (box / 2, box / 2, box / 2), (0, 1, 0),
                     PERSPECTIVE, width, height, fov_x_deg, z_near=1.0, z_far=10 * box)
    if brightness is None:
        brightness = 0.02
    sp = [Species(log_scale=1, brightness=brightness, absorption=brightness, mode=ORDERED),
          Species(log_scale=1, brightness=brightness, absorption=0.0, mode=ADDITIVE)]
    return out, camera, sp


def torch_scene_to_numpy(parts: dict, camera, species_params, name="") -> Scene:
    """Copy a dict of torch particle tensors into a host Scene."""
    def h(k):
        t = parts.get(k)
        return None if t is None else t.detach().cpu().numpy()
    return Scene(h("x"), h("y"), h("z"), h("h"), h("value"), camera, species_params,
                 species=h("species"), rho0=h("rho0"), name=name)
