"""Split particles (Section 3.2): particles whose footprint box covers more
pixels than the threshold have their (tile, particle) pairs written by a
whole workgroup.  Speed only: per-tile lists and images are bit-identical
with splitting off, at the paper's (W+H)/2 and at a tiny threshold, and
match the oracle."""
import numpy as np
import pytest

from paper_1004_1302_amd import binding as B
from paper_1004_1302_amd import synth

from test_gpu_parity import check_image, expected_bins, gpu_render

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def closeup(n=60_000, seed=71, w=400, h=300):
    """NFW halos seen from close by: footprints from a few pixels to the
    whole window."""
    sc = synth.nfw_halos(n, seed=seed, n_halos=40, grid=64, width=w, height=h)
    sc.camera = synth.look_at((50.0, 50.0, 20.0), (50.0, 50.0, 60.0), (0.0, 1.0, 0.0),
                              synth.PERSPECTIVE, w, h, z_near=0.5, z_far=500.0)
    return sc


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_split_lists_and_images_identical(torch_cuda, orc, tile):
    sc = closeup()
    parts, pal = B.scene_to_device(sc)
    lists = []
    for split in (-1, 0, 16):
        ts, te, pp, n = B.bin_pairs(parts, sc.camera, sc.species_params, tile=tile,
                                    split_pixels=split)
        lists.append((ts.cpu().numpy(), te.cpu().numpy(), pp.cpu().numpy(), n))
    ref = orc.project(sc, tile=tile)
    es, ee, ep = expected_bins(ref, sc, tile, True)
    for ts, te, pp, n in lists:
        assert n == ep.size
        assert np.array_equal(pp.view(np.uint32).astype(np.int64), ep)
        assert np.array_equal(ts.view(np.uint32), es.astype(np.uint32))
    # some particles are split at (W+H)/2: boxes above 350 px
    big = (ref["bbox"][:, 1] - ref["bbox"][:, 0] + 1) * (ref["bbox"][:, 3] - ref["bbox"][:, 2] + 1)
    assert np.sum((ref["status"] == 0) & (big > 350)) > 100
    imgs = [gpu_render(sc, tile=tile, compensated=True, split_pixels=s) for s in (-1, 0, 16)]
    assert np.array_equal(imgs[0], imgs[1]) and np.array_equal(imgs[0], imgs[2])
    check_image(imgs[0], orc.render(sc))


def test_split_chunked_and_batched(torch_cuda, orc):
    """Splitting inside workspace-bounded chunks and in a batch of views."""
    import torch
    sc = closeup(40_000, seed=72, w=320, h=240)
    ref = orc.render(sc)
    a, st = gpu_render(sc, max_pairs=5_000, stats=True, split_pixels=16)
    assert st["n_chunks"] > 3
    check_image(a, ref)
    parts, pal = B.scene_to_device(sc)
    ims = B.render_batch(parts, [sc.camera, sc.camera], pal, sc.species_params,
                         split_pixels=16, streams=2)
    torch.cuda.synchronize()
    plain = gpu_render(sc, split_pixels=-1)
    assert np.array_equal(ims[0].cpu().numpy(), plain)
    assert np.array_equal(ims[1].cpu().numpy(), plain)
