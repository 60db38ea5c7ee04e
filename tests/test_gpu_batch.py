"""Batched views: several cameras of differing resolutions rendered from
one device-resident particle set in one stream-ordered sequence (optionally
one HIP graph), checked against single-view renders through the same
C ABI, and against the oracle."""
import numpy as np
import pytest

from paper_1004_1302_amd import autotune
from paper_1004_1302_amd import binding as B
from paper_1004_1302_amd import synth

pytestmark = pytest.mark.gpu


def orbit_cameras(n_views, seed, sizes):
    return synth.orbit_cameras(n_views, seed, sizes)


@pytest.fixture(scope="module")
def scene():
    import torch
    assert torch.cuda.is_available()
    sc = synth.plummer_mix(200_000, seed=31)
    # two species so the depth-ordered path runs: half absorbing, half additive
    sc.species = (np.arange(sc.n) % 2).astype(np.uint8)
    sc.species_params = [
        synth.Species(log_scale=1, brightness=0.05, absorption=0.05, mode=synth.ORDERED),
        synth.Species(log_scale=1, brightness=0.05, mode=synth.ADDITIVE)]
    return sc


def single(parts, cam, pal, sp, **kw):
    import torch
    img = B.render(parts, cam, pal, sp, compensated=True, **kw)
    torch.cuda.synchronize()
    return img.cpu().numpy()


def test_batch_matches_single_views(scene, orc):
    import torch
    parts, pal = B.scene_to_device(scene)
    cams = orbit_cameras(6, 1, [(96, 96), (160, 120), (200, 90), (64, 128)])
    imgs, st = B.render_batch(parts, cams, pal, scene.species_params, compensated=True,
                              stats=True)
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        ref = single(parts, cam, pal, scene.species_params)
        assert np.array_equal(imgs[v].cpu().numpy(), ref), f"view {v}"
        assert st[v]["n_chunks"] == 1 and st[v]["n_pairs"] > 0
    # and one view against the oracle
    sc = synth.Scene(scene.x, scene.y, scene.z, scene.h, scene.value, cams[2],
                     scene.species_params, species=scene.species)
    o = orc.render(sc)
    got = imgs[2].cpu().numpy().astype(np.float64)
    rel = np.abs(got - o).reshape(3, -1).max(1) / np.abs(o).reshape(3, -1).max(1)
    assert np.all(rel <= 1e-4), rel


def test_batch_at_the_batched_views_sizes(scene, orc):
    """The batched-views workload's shape at a reduced particle count:
    cameras on the seeded orbit at 512², 1024², 1920x1080 and 2048², one
    batch on four streams captured as a graph, every view bit-identical to
    its single render; the 2048² view against the oracle on sampled pixels
    (the 64 brightest and 192 random ones)."""
    import torch
    parts, pal = B.scene_to_device(scene)
    sizes = [(512, 512), (1024, 1024), (1920, 1080), (2048, 2048)]
    cams = orbit_cameras(8, 11, sizes)
    cams[-1] = orbit_cameras(1, 12, [(2048, 2048)])[0]
    # room for every view's pairs (the 2048² views bin about 4.5 per
    # particle), so that no render here is cut into depth slabs
    mp = 1 << 23
    refs = [single(parts, c, pal, scene.species_params, max_pairs=mp) for c in cams]
    _, st = B.render_batch(parts, cams, pal, scene.species_params, compensated=True,
                           streams=4, max_pairs=mp, stats=True)
    assert all(s["n_chunks"] == 1 and s["n_pairs"] > 0 for s in st)
    B.graph_cache_clear()
    images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device="cuda")
              for c in cams]
    for rep in range(2):
        out = B.render_batch(parts, cams, pal, scene.species_params, images, graph=True,
                             compensated=True, streams=4, max_pairs=mp)
        torch.cuda.synchronize()
        for v in range(len(cams)):
            assert np.array_equal(out[v].cpu().numpy(), refs[v]), f"replay {rep} view {v}"
    B.graph_cache_clear()
    cam = cams[-1]
    got = refs[-1].astype(np.float64)
    lum = got.sum(0).ravel()
    rng = np.random.default_rng(13)
    pick = np.concatenate([np.argsort(lum)[-64:], rng.integers(0, lum.size, 192)])
    pj, pi = np.divmod(pick, cam.width)
    sc = synth.Scene(scene.x, scene.y, scene.z, scene.h, scene.value, cam,
                     scene.species_params, species=scene.species)
    o = orc.render_pixels(sc, pi.astype(np.int32), pj.astype(np.int32)).T
    g = got.reshape(3, -1)[:, pick]
    rel = np.abs(g - o).max(1) / np.abs(o).max(1)
    assert np.all(rel <= 1e-4), rel


@pytest.mark.parametrize("streams", [2, 3, 4])
def test_batch_on_several_streams_matches_single_views(scene, streams):
    """Views round-robin over several streams (each with its own workspace
    part) give the same bits as one render call per view, eager and as a
    replayed graph."""
    import torch
    parts, pal = B.scene_to_device(scene)
    cams = orbit_cameras(7, 5, [(96, 96), (160, 120), (200, 90), (64, 128)])
    refs = [single(parts, c, pal, scene.species_params) for c in cams]
    imgs, st = B.render_batch(parts, cams, pal, scene.species_params, compensated=True,
                              stats=True, streams=streams)
    torch.cuda.synchronize()
    for v in range(len(cams)):
        assert np.array_equal(imgs[v].cpu().numpy(), refs[v]), f"view {v}"
        assert st[v]["n_chunks"] == 1 and st[v]["n_pairs"] > 0
    B.graph_cache_clear()
    images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device="cuda")
              for c in cams]
    for rep in range(3):
        for im in images:
            im.fill_(-1.0)
        torch.cuda.synchronize()
        out = B.render_batch(parts, cams, pal, scene.species_params, images, graph=True,
                             compensated=True, streams=streams)
        torch.cuda.synchronize()
        for v in range(len(cams)):
            assert np.array_equal(out[v].cpu().numpy(), refs[v]), f"replay {rep} view {v}"
    assert B.graph_cache_clear() == 1


def test_graph_replays_track_eager(scene):
    """The captured graph is replayed several times with eager work and
    synchronisations in between; particle values change in place between
    replays, and every replay must equal an eager render of the same data."""
    import torch
    parts, pal = B.scene_to_device(scene)
    cams = orbit_cameras(4, 2, [(128, 96), (80, 80), (150, 110)])
    B.graph_cache_clear()
    images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device="cuda")
              for c in cams]
    for rep in range(4):
        if rep:
            parts["value"].mul_(1.7)              # same pointers, new data
            parts["h"].mul_(1.05)
        junk = torch.randn(1 << 20, device="cuda").sum()   # eager work between replays
        torch.cuda.synchronize()
        out = B.render_batch(parts, cams, pal, scene.species_params, images, graph=True,
                             compensated=True)
        torch.cuda.synchronize()
        float(junk)
        for v, cam in enumerate(cams):
            ref = single(parts, cam, pal, scene.species_params)
            assert np.array_equal(out[v].cpu().numpy(), ref), f"replay {rep} view {v}"
    assert B.graph_cache_clear() == 1


def test_batch_overflow_is_chunked(scene):
    """A view whose pairs exceed the capacity of its part of the workspace
    writes nothing in the batch; an eager batch then renders it in
    workspace-bounded chunks, the same bits as a single render with that
    capacity.  A graph replay cannot branch on the flag: it reports the
    view (SPLOTCH_E_CAPACITY with stats) and leaves its image untouched."""
    import torch
    parts, pal = B.scene_to_device(scene)
    cams = orbit_cameras(3, 3, [(128, 128)])
    kw = dict(max_pairs=20_000, compensated=True)
    imgs, st = B.render_batch(parts, cams, pal, scene.species_params, stats=True, **kw)
    torch.cuda.synchronize()
    for v, cam in enumerate(cams):
        ref, one = B.render(parts, cam, pal, scene.species_params, stats=True, **kw)
        torch.cuda.synchronize()
        assert one["n_chunks"] > 1 and st[v]["n_chunks"] == one["n_chunks"]
        assert np.array_equal(imgs[v].cpu().numpy(), ref.cpu().numpy()), v
    for im in imgs:
        im.fill_(-1.0)
    with pytest.raises(B.SplotchError) as e:
        B.render_batch(parts, cams, pal, scene.species_params, imgs, stats=True, graph=True, **kw)
    assert e.value.code == 5
    torch.cuda.synchronize()
    assert all(bool((im == -1.0).all()) for im in imgs)
    B.graph_cache_clear()
    # the library is still usable afterwards
    imgs = B.render_batch(parts, cams, pal, scene.species_params, compensated=True)
    torch.cuda.synchronize()
    ref = single(parts, cams[0], pal, scene.species_params)
    assert np.array_equal(imgs[0].cpu().numpy(), ref)


def test_autotune_picks_and_caches(scene, tmp_path):
    parts, pal = B.scene_to_device(scene)
    cam = orbit_cameras(1, 4, [(256, 192)])[0]
    path = str(tmp_path / "tune.json")
    r1 = autotune.tune(parts, cam, pal, scene.species_params, cache_path=path, repeats=2,
                       compensated=True)
    assert r1["tile"] in autotune.DEFAULT_TILES and r1["seg_records"] in autotune.DEFAULT_SEGS
    assert len(r1["table"]) == len(autotune.DEFAULT_TILES) * len(autotune.DEFAULT_SEGS)
    assert not r1["cached"]
    r2 = autotune.tune(parts, cam, pal, scene.species_params, cache_path=path)
    assert r2["cached"] and r2["tile"] == r1["tile"]
    # every tuned shape renders the same image (within rounding of the merge order)
    base = single(parts, cam, pal, scene.species_params, tile=16)
    for row in r1["table"]:
        img = single(parts, cam, pal, scene.species_params, tile=row["tile"],
                     seg_records=row["seg_records"])
        rel = np.abs(img - base).max() / np.abs(base).max()
        assert rel <= 1e-5


@pytest.mark.timeout(900)
def test_batched_views_full_size(orc):
    """The batched-views workload at its stated size: 5e7 particles of the
    small-configuration generator, 64 orbit cameras at 512², 1024²,
    1920x1080 and 2048², rendered as one batch on four streams (pair
    capacity 3e8 per view).  Every view is checked against a single render
    of the same view (bit-identical), and four views, among them a 2048²
    one, against the oracle on 2048 sampled pixels each (the 64 brightest
    and random ones), 1e-4 relative L-infinity per channel."""
    import torch
    sc = synth.plummer_mix(50_000_000, seed=41)
    parts, pal = B.scene_to_device(sc)
    sizes = [(512, 512), (1024, 1024), (1920, 1080), (2048, 2048)]
    cams = synth.orbit_cameras(64, 7, sizes)
    kw = dict(compensated=True, tile=32, seg_records=4096, max_pairs=300_000_000)
    imgs, st = B.render_batch(parts, cams, pal, sc.species_params, streams=4, stats=True, **kw)
    torch.cuda.synchronize()
    assert all(s["n_chunks"] == 1 for s in st)
    print(f"batch: most pairs in a view {max(s['n_pairs'] for s in st)}", flush=True)
    big = [v for v, c in enumerate(cams) if (c.width, c.height) == (2048, 2048)]
    check = [big[0]] + [v for v in (0, 21, 42) if v != big[0]][:3]
    rng = np.random.default_rng(3)
    for v in range(len(cams)):
        ref = single(parts, cams[v], pal, sc.species_params, tile=32, seg_records=4096,
                     max_pairs=300_000_000)
        assert np.array_equal(imgs[v].cpu().numpy(), ref), f"view {v}"
    for v in check:
        cam = cams[v]
        img = imgs[v].cpu().numpy()
        flat = img.sum(0).ravel()
        idx = np.concatenate([np.argsort(flat)[-64:], rng.integers(0, flat.size, 1984)])
        pj, pi = np.unravel_index(idx, (cam.height, cam.width))
        view = synth.Scene(sc.x, sc.y, sc.z, sc.h, sc.value, cam, sc.species_params)
        ref = orc.render_pixels(view, pi, pj)
        got = img[:, pj, pi].T.astype(np.float64)
        scale = np.abs(ref).max(axis=0)
        rel = np.abs(got - ref).max(axis=0) / np.where(scale > 0, scale, 1)
        print(f"view {v} {cam.width}x{cam.height}: sampled relative Linf {rel}", flush=True)
        assert np.all(rel <= 1e-4), (v, rel)


@pytest.mark.parametrize("streams", [1, 3, 4])
def test_persistent_batch_bit_identical(scene, streams):
    """Views prepared in groups of `streams` and splatted by one persistent
    launch per group: every image the same bits as a single render, eager
    and as graph replays (with work and syncs between replays); 64 px tiles
    too."""
    import torch
    parts, pal = B.scene_to_device(scene)
    cams = orbit_cameras(7, 4, [(96, 96), (160, 120), (200, 90), (64, 128)])
    for tile in (16, 64):
        refs = [single(parts, c, pal, scene.species_params, tile=tile) for c in cams]
        imgs = B.render_batch(parts, cams, pal, scene.species_params, compensated=True,
                              persistent=True, streams=streams, tile=tile)
        torch.cuda.synchronize()
        for v in range(len(cams)):
            assert np.array_equal(imgs[v].cpu().numpy(), refs[v]), (tile, v)
        B.graph_cache_clear()
        for rep in range(3):
            for im in imgs:
                im.fill_(-1.0)
            B.render_batch(parts, cams, pal, scene.species_params, imgs, compensated=True,
                           persistent=True, streams=streams, tile=tile, graph=True)
            torch.cuda.synchronize()
            for v in range(len(cams)):
                assert np.array_equal(imgs[v].cpu().numpy(), refs[v]), (tile, rep, v)
        B.graph_cache_clear()
