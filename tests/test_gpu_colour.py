"""GPU parity for the general colour model and the two alternative readings
of Section 2, through the C ABI against the FP64 oracle:

* a separate absorption look-up table (E and A differ per channel);
* vector quantities whose three components are r, g, b directly;
* emission of absorbing species read as a source function (E := A E);
* the density cut to the f sigma ball (column times erf(sqrt(f^2 - q^2))).

Bars as elsewhere: images within 1e-4 relative L-infinity per channel;
the three splat strategies bit-identical to each other; projections of
vector-coloured species bit-exact (validity, boxes, keys)."""
import numpy as np
import pytest

from paper_1004_1302_amd import binding as B
from paper_1004_1302_amd import synth

from test_gpu_parity import c1, c2_small, check_image, gpu_render, same_composite

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def absorb_palette(K=64):
    """An absorption table unlike the emission one: strong in blue, weak in
    red, with a bump in green."""
    t = np.linspace(0.0, 1.0, K)
    return np.stack([0.2 + 0.3 * t, 0.5 + 0.5 * np.sin(np.pi * t), 1.2 - 0.4 * t],
                    axis=1).astype(np.float32)


def vector_scene(n=120_000, seed=31, w=240, h=180, log_scale=0):
    """NFW halos with two species: gas coloured by a 3-vector (ordered),
    dark matter through the palette (additive)."""
    sc = c2_small(n, seed=seed, w=w, h=h)
    rng = np.random.default_rng(seed + 1)
    sc.value_g = rng.lognormal(0.3, 0.8, sc.n).astype(np.float32)
    sc.value_b = rng.lognormal(-0.2, 0.6, sc.n).astype(np.float32)
    sc.species_params = [
        synth.Species(log_scale=log_scale, brightness=0.3, absorption=0.3, mode=synth.ORDERED,
                      colour=synth.COLOUR_VECTOR),
        synth.Species(log_scale=1, brightness=0.2, mode=synth.ADDITIVE)]
    return sc


def all_variants(scene, ref, **kw):
    """Render with every splat strategy: each within tolerance of the
    oracle, and all three the same composite (bit-identical without
    compensation, the grouping bound with it)."""
    imgs = [gpu_render(scene, splat_variant=v, **kw) for v in (1, 2, 3)]
    for im in imgs:
        check_image(im, ref)
    comp = kw.get("compensated", False)
    same_composite(imgs[0], imgs[1], comp, "lists")
    same_composite(imgs[0], imgs[2], comp, "box")
    return imgs[0]


def test_absorption_palette_ordered(torch_cuda, orc):
    sc = c2_small(80_000, seed=21, w=240, h=160)
    sc.palette_absorb = absorb_palette()
    sc.species_params = [
        synth.Species(log_scale=1, brightness=0.4, absorption=0.7, mode=synth.ORDERED),
        synth.Species(log_scale=1, brightness=0.3, mode=synth.ADDITIVE)]
    ref = orc.render(sc)
    img = all_variants(sc, ref, compensated=True)
    # the table matters: the same render with one table is far from it
    sc1 = c2_small(80_000, seed=21, w=240, h=160)
    sc1.species_params = sc.species_params
    assert np.abs(orc.render(sc1) - ref).max() > 1e-2 * np.abs(ref).max()
    assert img.shape == ref.shape


@pytest.mark.parametrize("log_scale", [0, 1])
def test_vector_colour(torch_cuda, orc, log_scale):
    sc = vector_scene(log_scale=log_scale)
    ref = orc.render(sc)
    img, st = gpu_render(sc, stats=True)
    check_image(img, ref)
    lo, hi = orc.value_range(sc)
    assert np.array_equal(np.array(st["vmin"][:2], np.float32), lo)
    assert np.array_equal(np.array(st["vmax"][:2], np.float32), hi)
    all_variants(sc, ref, compensated=True)


def test_vector_colour_invalid_components(torch_cuda, orc):
    """Non-finite second or third components make a vector-coloured
    particle invalid (skipped and counted); palette species ignore them."""
    sc = vector_scene(30_000, seed=33, w=160, h=120)
    sc.value_g[:40] = np.nan
    sc.value_b[40:80] = np.inf
    ref = orc.render(sc)
    img, st = gpu_render(sc, stats=True)
    check_image(img, ref)
    is_vec = sc.species[:80] == 0
    assert st["n_invalid"] == int(is_vec.sum())
    parts, _ = B.scene_to_device(sc)
    pr = B.project(parts, sc.camera, sc.species_params)
    want = orc.project(sc)["status"]
    assert np.array_equal(pr["status"].cpu().numpy(), want)


def test_vector_colour_needs_components(torch_cuda):
    sc = vector_scene(1000, seed=34, w=64, h=64)
    parts, pal = B.scene_to_device(sc)
    del parts["value_g"]
    with pytest.raises(B.SplotchError) as e:
        B.render(parts, sc.camera, pal, sc.species_params)
    assert e.value.code == 1


@pytest.mark.parametrize("palette_absorb", [False, True])
def test_emission_is_source(torch_cuda, orc, palette_absorb):
    """Source-function reading: ordered species update I <- (I - S) e^{-A tau}
    + S; additive species unchanged."""
    sc = c2_small(80_000, seed=22, w=240, h=160)
    sc.emission_is_source = 1
    if palette_absorb:
        sc.palette_absorb = absorb_palette()
    sc.species_params = [
        synth.Species(log_scale=1, brightness=0.8, absorption=0.5, mode=synth.ORDERED),
        synth.Species(log_scale=1, brightness=0.2, mode=synth.ADDITIVE)]
    iin = np.random.default_rng(5).uniform(0, 0.3, (3, 160, 240))
    ref = orc.render(sc, img_in=iin)
    img = gpu_render(sc, img_in=iin, compensated=True)
    check_image(img, ref)
    sc.emission_is_source = 0
    assert np.abs(orc.render(sc, img_in=iin) - ref).max() > 1e-2 * np.abs(ref).max()


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_trunc3d_additive(torch_cuda, orc, tile):
    sc = c1(60_000, seed=23)
    sc.kernel = synth.KERNEL_TRUNC3D
    ref = orc.render(sc)
    check_image(gpu_render(sc, tile=tile, compensated=True), ref)


def test_trunc3d_ordered_all_variants(torch_cuda, orc):
    sc = c2_small(80_000, seed=24, w=240, h=160)
    sc.kernel = synth.KERNEL_TRUNC3D
    ref = orc.render(sc)
    all_variants(sc, ref, compensated=True)
    # the kernel matters: the 2-D cut differs from the ball cut
    sc.kernel = synth.KERNEL_GAUSS2D
    assert np.abs(orc.render(sc) - ref).max() > 1e-3 * np.abs(ref).max()


def test_trunc3d_single_particle_closed_form(torch_cuda):
    """At the footprint centre the column is rho0 erf(f); one sigma out it is
    rho0 e^{-1} erf(sqrt(f^2 - 1))."""
    from math import erf, exp, sqrt
    cam = synth.ortho_unit_square(64, 64)
    sc = synth.Scene(np.array([20.5 / 64], np.float32), np.array([30.5 / 64], np.float32),
                     np.array([0.5], np.float32), np.array([4.0 / 64], np.float32),
                     np.array([1.0], np.float32), cam,
                     [synth.Species(vmin=0.0, vmax=2.0, brightness=1.0)],
                     rho0=np.array([0.5], np.float32), kernel=synth.KERNEL_TRUNC3D)
    sc.palette = np.ones((2, 3), np.float32)
    img = gpu_render(sc)
    assert img[0, 30, 20] == pytest.approx(0.5 * erf(2.0), rel=2e-6)
    assert img[1, 30, 24] == pytest.approx(0.5 * exp(-1.0) * erf(sqrt(3.0)), rel=2e-5)
    assert img[2, 30, 29] == 0.0


def test_everything_together_chunked_batched(torch_cuda, orc):
    """All four settings at once, rendered whole, in forced chunks, and as a
    two-view batch: each against the oracle."""
    import torch
    sc = vector_scene(60_000, seed=35, w=200, h=150, log_scale=1)
    sc.palette_absorb = absorb_palette(32)
    sc.species_params.append(
        synth.Species(log_scale=1, brightness=0.6, absorption=1.1, mode=synth.ORDERED))
    sc.species = np.random.default_rng(8).integers(0, 3, sc.n).astype(np.uint8)
    sc.kernel = synth.KERNEL_TRUNC3D
    sc.emission_is_source = 1
    ref = orc.render(sc)
    full = gpu_render(sc, compensated=True)
    check_image(full, ref)
    img, st = gpu_render(sc, compensated=True, max_pairs=4000, stats=True)
    assert st["n_chunks"] > 3
    check_image(img, ref)
    parts, pal = B.scene_to_device(sc)
    cam2 = synth.look_at((50.0, 60.0, -90.0), (50.0, 50.0, 50.0), (0.0, 1.0, 0.0),
                         synth.PERSPECTIVE, 96, 80)
    opts = B.scene_options(sc)
    ims = B.render_batch(parts, [sc.camera, cam2], pal, sc.species_params, compensated=True,
                         **opts)
    torch.cuda.synchronize()
    check_image(ims[0].cpu().numpy(), ref)
    sc2 = sc.subset(np.arange(sc.n))
    sc2.camera = cam2
    check_image(ims[1].cpu().numpy(), orc.render(sc2))
