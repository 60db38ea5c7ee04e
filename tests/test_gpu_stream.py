"""Out-of-core render (splotch_render_stream): particles in pinned host
memory, streamed to the device in subsets; ordered sets in depth slabs.
Checked against the device-resident render of the same set (equal up to
rounding: 2e-5 relative L-infinity) and against the FP64 oracle (1e-4)."""
import numpy as np
import pytest

from paper_1004_1302_amd import binding as B
from paper_1004_1302_amd import synth

from test_gpu_parity import c1, c2_small, check_image, gpu_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def host_parts(torch, scene):
    """The scene's particle arrays as pinned host tensors."""
    out = {}
    for k in ("x", "y", "z", "h", "value", "rho0", "value_g", "value_b"):
        a = getattr(scene, k, None)
        if a is not None:
            out[k] = torch.from_numpy(np.ascontiguousarray(a, np.float32)).pin_memory()
    if scene.species is not None:
        out["species"] = torch.from_numpy(np.ascontiguousarray(scene.species, np.uint8)) \
            .pin_memory()
    return out


def streamed(torch, scene, **kw):
    _, pal = B.scene_to_device(scene)
    opts = B.scene_options(scene)
    opts.update(kw)
    img, st = B.render_stream(host_parts(torch, scene), scene.camera, pal,
                              scene.species_params, stats=True, **opts)
    torch.cuda.synchronize()
    return img.cpu().numpy(), st


def test_stream_additive_subsets(torch_cuda, orc):
    scene = c1(200_000, seed=61)
    img, st = streamed(torch_cuda, scene, subset=30_000, compensated=True)
    assert st["n_chunks"] == 7 and st["ordered"] == 0
    dev = gpu_render(scene, compensated=True)
    check_image(img, dev.astype(np.float64), tol=2e-5)
    check_image(img, orc.render(scene))


@pytest.mark.parametrize("slab", [40_000, 1 << 20])
def test_stream_ordered_depth_slabs(torch_cuda, orc, slab):
    """Mixed species (ordered gas, additive dark matter) over a background
    image: several depth slabs composited back to front, or one."""
    scene = c2_small(200_000, seed=62, w=320, h=200)
    iin = np.random.default_rng(4).uniform(0, 0.3, (3, 200, 320)).astype(np.float32)
    import torch
    image = torch.from_numpy(iin).cuda()
    _, pal = B.scene_to_device(scene)
    img, st = B.render_stream(host_parts(torch, scene), scene.camera, pal, scene.species_params,
                              image, subset=37_000, slab=slab, stats=True, compensated=True,
                              accumulate=True, **B.scene_options(scene))
    torch.cuda.synchronize()
    img = img.cpu().numpy()
    dev, dst = gpu_render(scene, img_in=iin, compensated=True, stats=True)
    assert st["ordered"] == 1 and st["n_visible"] == dst["n_visible"]
    assert (st["n_chunks"] > 3) == (slab < 100_000)
    check_image(img, dev.astype(np.float64), tol=2e-5)
    check_image(img, orc.render(scene, img_in=iin.astype(np.float64)))


def test_stream_whole_set_value_range(torch_cuda, orc):
    """Automatic value ranges are those of the whole set, not of a subset
    or slab (the colours would differ otherwise)."""
    scene = c2_small(120_000, seed=63, w=200, h=150)
    img, st = streamed(torch_cuda, scene, subset=10_000, slab=30_000)
    lo, hi = orc.value_range(scene)
    assert np.array_equal(np.array(st["vmin"][:2], np.float32), lo)
    assert np.array_equal(np.array(st["vmax"][:2], np.float32), hi)
    check_image(img, orc.render(scene))


def test_stream_general_colour_settings(torch_cuda, orc):
    """Vector colours, an absorption table, the ball-cut column and the
    source-function reading through the streamed path."""
    scene = c2_small(80_000, seed=64, w=200, h=150)
    rng = np.random.default_rng(64)
    scene.value_g = rng.lognormal(0, 0.5, scene.n).astype(np.float32)
    scene.value_b = rng.lognormal(0, 0.5, scene.n).astype(np.float32)
    scene.species_params = [
        synth.Species(log_scale=1, brightness=0.3, absorption=0.5, mode=synth.ORDERED,
                      colour=synth.COLOUR_VECTOR),
        synth.Species(log_scale=1, brightness=0.2, absorption=0.9, mode=synth.ORDERED)]
    scene.palette_absorb = np.linspace([0.2, 0.8, 1.0], [1.0, 0.3, 0.1], 16).astype(np.float32)
    scene.kernel = synth.KERNEL_TRUNC3D
    scene.emission_is_source = 1
    img, st = streamed(torch_cuda, scene, subset=9_000, slab=20_000, compensated=True)
    assert st["n_chunks"] > 2
    check_image(img, orc.render(scene))


def test_stream_nfw_full_size_sampled(torch_cuda, orc):
    """The full NFW set (1e7 particles, 1920x1080, mixed species) streamed
    from pinned host memory in 2^21-particle subsets and 2^22-particle
    slabs: against the device-resident render, and against the oracle on
    sampled pixels (the brightest and random ones)."""
    import torch
    scene = synth.nfw_halos(10_000_000, seed=2)
    img, st = streamed(torch, scene, subset=1 << 21, slab=1 << 22, compensated=True)
    assert st["n_chunks"] >= 2
    dev = gpu_render(scene, compensated=True)
    check_image(img, dev.astype(np.float64), tol=2e-5)
    rng = np.random.default_rng(1)
    flat = img.sum(0).ravel()
    idx = np.concatenate([np.argsort(flat)[-64:], rng.integers(0, flat.size, 448)])
    pj, pi = np.unravel_index(idx, (1080, 1920))
    ref = orc.render_pixels(scene, pi, pj)
    got = img[:, pj, pi].T.astype(np.float64)
    scale = np.abs(ref).max(axis=0)
    assert np.all(np.abs(got - ref).max(axis=0) / scale <= 1e-4)


def test_stream_empty_and_capacity(torch_cuda):
    import torch
    scene = c2_small(20_000, seed=65, w=64, h=48)
    empty = scene.subset(np.arange(0))
    _, pal = B.scene_to_device(scene)
    img = torch.full((3, 48, 64), 3.0, device="cuda")
    out = B.render_stream(host_parts(torch, empty), scene.camera, pal, scene.species_params,
                          img, subset=1000, slab=1000)
    torch.cuda.synchronize()
    assert torch.count_nonzero(out) == 0
    # every particle at one depth: one histogram bin larger than a slab
    same = scene.subset(np.arange(scene.n))
    same.z = np.full(scene.n, 50.0, np.float32)
    with pytest.raises(B.SplotchError) as e:
        B.render_stream(host_parts(torch, same), scene.camera, pal, scene.species_params,
                        subset=5000, slab=1000)
    assert e.value.code == 5
