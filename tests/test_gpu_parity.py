"""GPU parity: the HIP path, called through the C ABI, against the FP64
oracle on the same seeded inputs.

Bars: integer outputs (visibility, pixel boxes, tile counts, depth keys,
per-tile lists) and the binary32 membership fields are bit-exact; images
agree to a relative L-infinity error of 1e-4 per channel
(max |gpu - oracle| / max |oracle|)."""
import numpy as np
import pytest

from paper_1004_1302_amd import binding as B
from paper_1004_1302_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def gpu_render(scene, img_in=None, **kw):
    import torch
    parts, pal = B.scene_to_device(scene)
    image = None
    if img_in is not None:
        image = torch.from_numpy(np.ascontiguousarray(img_in, np.float32)).cuda()
        kw["accumulate"] = True
    opts = B.scene_options(scene)
    opts.update(kw)
    out = B.render(parts, scene.camera, pal, scene.species_params, image, **opts)
    st = None
    if isinstance(out, tuple):
        out, st = out
    torch.cuda.synchronize()
    img = out.cpu().numpy()
    return (img, st) if st is not None else img


def check_image(gpu, ref, tol=TOL):
    err = np.abs(gpu.astype(np.float64) - ref).reshape(3, -1).max(axis=1)
    den = np.abs(ref).reshape(3, -1).max(axis=1)
    rel = err / np.where(den > 0, den, 1.0)
    assert np.all(rel <= tol), f"relative Linf per channel {rel}"
    return rel


def check_pixels(gpu, ref, rel=1e-4, floor=1e-6):
    """Per-pixel bound for compensated renders: every pixel within rel of
    its own oracle value, plus an absolute floor of `floor` times the
    channel's largest oracle value (pixels that faint are at the level of
    the FP32 resolution of the bright ones).  Arrays are [3][...] or
    [..., 3] with channel_axis 0."""
    g = gpu.astype(np.float64).reshape(3, -1)
    o = np.asarray(ref, np.float64).reshape(3, -1)
    bound = rel * np.abs(o) + floor * np.abs(o).max(axis=1, keepdims=True)
    worst = (np.abs(g - o) / np.where(bound > 0, bound, 1.0)).max(axis=1)
    assert np.all(np.abs(g - o) <= bound), f"per-pixel error over the bound: {worst}"
    return worst


def expected_bins(pr, scene, tile, ordered):
    W, H = scene.camera.width, scene.camera.height
    ntx, nty = -(-W // tile), -(-H // tile)
    vis = np.nonzero(pr["status"] == 0)[0]
    i0, i1, j0, j1 = pr["bbox"][vis].T
    tiles, parts = [], []
    for k, p in enumerate(vis):
        tx = np.arange(i0[k] // tile, i1[k] // tile + 1)
        ty = np.arange(j0[k] // tile, j1[k] // tile + 1)
        t = (ty[:, None] * ntx + tx[None, :]).ravel()
        tiles.append(t)
        parts.append(np.full(t.size, p))
    tiles = np.concatenate(tiles) if tiles else np.zeros(0, np.int64)
    parts = np.concatenate(parts) if parts else np.zeros(0, np.int64)
    if ordered:
        order = np.lexsort((parts, pr["key"][parts], tiles))
    else:
        order = np.lexsort((parts, tiles))
    tiles, parts = tiles[order], parts[order]
    start = np.zeros(ntx * nty, np.int64)
    end = np.zeros(ntx * nty, np.int64)
    if tiles.size:
        b = np.nonzero(np.diff(tiles))[0] + 1
        firsts = np.concatenate([[0], b])
        lasts = np.concatenate([b, [tiles.size]])
        start[tiles[firsts]] = firsts
        end[tiles[firsts]] = lasts
    return start, end, parts


# ----------------------------------------------------------------- scenes
def c1(n=100_000, seed=1, **kw):
    return synth.plummer_mix(n, seed=seed, **kw)


def c2_small(n=200_000, seed=2, w=480, h=270):
    return synth.nfw_halos(n, seed=seed, n_halos=60, grid=64, width=w, height=h)


def edge_scene():
    """Ragged sizes, off-screen and behind-camera particles, non-finite
    fields, a particle covering the whole screen, sub-pixel particles."""
    rng = np.random.default_rng(7)
    n = 3000
    x = rng.uniform(-0.2, 1.2, n).astype(np.float32)
    y = rng.uniform(-0.2, 1.2, n).astype(np.float32)
    z = rng.uniform(-0.5, 1.0, n).astype(np.float32)
    h = rng.lognormal(np.log(0.01), 1.0, n).astype(np.float32)
    v = rng.lognormal(0, 1, n).astype(np.float32)
    x[:5] = np.nan
    y[5:10] = np.inf
    h[10:15] = 0.0
    h[15:20] = -1.0
    v[20:25] = np.nan
    h[30] = 3.0          # covers everything
    h[31:40] = 1e-5      # sub-pixel
    x[40:50] = 50.0      # far off screen
    cam = synth.ortho_unit_square(101, 77)
    cam.px_per_unit = 90.0
    cam.z_near = 0.3
    sp = [synth.Species(log_scale=1, brightness=0.5, absorption=0.9, mode=synth.ORDERED),
          synth.Species(brightness=0.7, mode=synth.ADDITIVE)]
    spc = rng.integers(0, 2, n).astype(np.uint8)
    spc[60:70] = 5       # unknown species: invalid
    r0 = rng.uniform(0.2, 1.5, n).astype(np.float32)
    r0[70:75] = -1.0     # negative density: invalid
    return synth.Scene(x, y, z, h, v, cam, sp, species=spc, rho0=r0, name="edges")


def wide_scene(w, h, n=200_000, seed=12):
    """Mixed species over an orthographic w x h view, footprints of a few
    pixels (sigma about 3 px) whatever the image size."""
    rng = np.random.default_rng(seed)
    x = rng.uniform(0.0, 1.0, n).astype(np.float32)
    y = rng.uniform(0.5 - 0.6 * h / w, 0.5 + 0.6 * h / w, n).astype(np.float32)
    z = rng.uniform(0.0, 1.0, n).astype(np.float32)
    hh = rng.lognormal(np.log(3.0 / w), 0.5, n).astype(np.float32)
    v = rng.lognormal(0, 1, n).astype(np.float32)
    sp = [synth.Species(log_scale=1, brightness=0.6, absorption=0.6, mode=synth.ORDERED),
          synth.Species(brightness=0.4, mode=synth.ADDITIVE)]
    spc = rng.integers(0, 2, n).astype(np.uint8)
    return synth.Scene(x, y, z, hh, v, synth.ortho_unit_square(w, h), sp, species=spc,
                       name=f"wide_{w}x{h}")


# ----------------------------------------------------------------- indices
@pytest.mark.parametrize("name", ["c1", "c2_small", "edges"])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_projection_bit_exact(torch_cuda, orc, name, tile):
    scene = {"c1": c1, "c2_small": c2_small, "edges": edge_scene}[name]()
    parts, _ = B.scene_to_device(scene)
    out = B.project(parts, scene.camera, scene.species_params, sigma_over_h=scene.sigma_over_h,
                    trunc_f=scene.trunc_f, tile=tile)
    ref = orc.project(scene, tile=tile)
    st = out["status"].cpu().numpy()
    assert np.array_equal(st, ref["status"])
    vis = ref["status"] == 0
    assert vis.sum() > 0
    assert np.array_equal(out["bbox"].cpu().numpy()[vis], ref["bbox"][vis])
    spec = out["spec"].cpu().numpy()
    assert np.array_equal(spec[vis].view(np.uint32), ref["spec"][vis].view(np.uint32))
    key = out["key"].cpu().numpy().view(np.uint32)
    assert np.array_equal(key[vis], ref["key"][vis])
    nt = out["ntiles"].cpu().numpy().view(np.uint32)
    assert np.array_equal(nt, ref["ntiles"])
    s = out["stats"]
    for code, k in ((0, "n_visible"), (1, "n_invalid"), (2, "n_depth_culled"), (3, "n_offscreen")):
        assert s[k] == int((ref["status"] == code).sum())


@pytest.mark.parametrize("name", ["c1", "c2_small", "edges"])
@pytest.mark.parametrize("tile", [8, 16, 32])
def test_tile_lists_bit_exact(torch_cuda, orc, name, tile):
    scene = {"c1": c1, "c2_small": c2_small, "edges": edge_scene}[name]()
    parts, _ = B.scene_to_device(scene)
    ts, te, pp, n = B.bin_pairs(parts, scene.camera, scene.species_params,
                                sigma_over_h=scene.sigma_over_h, trunc_f=scene.trunc_f, tile=tile)
    ref = orc.project(scene, tile=tile)
    ordered = any(s.mode == synth.ORDERED for s in scene.species_params)
    es, ee, ep = expected_bins(ref, scene, tile, ordered)
    assert n == ep.size
    assert np.array_equal(ts.cpu().numpy().astype(np.int64), es)
    assert np.array_equal(te.cpu().numpy().astype(np.int64), ee)
    assert np.array_equal(pp.cpu().numpy().view(np.uint32).astype(np.int64), ep)


# ----------------------------------------------------------------- images
@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("compensated", [False, True])
def test_c1_full_additive(torch_cuda, orc, tile, compensated):
    """100k particles, Plummer spheres over a uniform background, 256x256,
    additive, orthographic (the small configuration in full)."""
    scene = c1()
    ref = orc.render(scene)
    img, st = gpu_render(scene, tile=tile, compensated=compensated, stats=True)
    check_image(img, ref)
    if compensated:
        check_pixels(img, ref)
    assert st["ordered"] == 0 and st["n_chunks"] == 1


@pytest.mark.parametrize("compensated", [False, True])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_c2_small_mixed_ordered(torch_cuda, orc, compensated, variant):
    """NFW halos, gas depth-ordered with E = A plus additive dark matter,
    perspective, at reduced size; both splat strategies."""
    scene = c2_small()
    ref = orc.render(scene)
    img, st = gpu_render(scene, compensated=compensated, stats=True, splat_variant=variant)
    check_image(img, ref)
    if compensated:
        check_pixels(img, ref)
    assert st["ordered"] == 1


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_list_variant_additive_and_edges(torch_cuda, orc, tile):
    scene = c1(30_000, seed=8)
    check_image(gpu_render(scene, tile=tile, splat_variant=2), orc.render(scene))
    scene = edge_scene()
    iin = np.random.default_rng(4).uniform(0, 0.6, (3, 77, 101))
    check_image(gpu_render(scene, img_in=iin, tile=tile, splat_variant=2),
                orc.render(scene, img_in=iin))


def _big_footprints(n=4000, seed=12):
    """Footprints from one pixel to several tiles across (box widths past
    16 and 32 px), depth-ordered, with a background."""
    sc = c2_small(n, seed=seed, w=180, h=140)
    sc.h = (sc.h * np.random.default_rng(seed).lognormal(2.0, 1.0, n)).astype(np.float32)
    return sc


def _strategy_scenes():
    big = _big_footprints()
    tau = c2_small(30_000, seed=10, w=160, h=120)
    tau.species_params = [
        synth.Species(log_scale=1, brightness=3.0, absorption=3.0, mode=synth.ORDERED),
        synth.Species(log_scale=1, brightness=0.5, absorption=0.0, mode=synth.ADDITIVE)]
    tau.rho0 = np.random.default_rng(1).uniform(0.1, 4.0, tau.n).astype(np.float32)
    return {"c1": (c1(40_000, seed=6), None), "c2": (c2_small(80_000, seed=5, w=240, h=150), None),
            "edges": (edge_scene(), np.random.default_rng(4).uniform(0, 0.6, (3, 77, 101))),
            "big": (big, np.random.default_rng(5).uniform(0, 0.3, (3, 140, 180))),
            "tau": (tau, None)}


def same_composite(a, b, compensated, what=""):
    """Two renders that composite each pixel's particles in the same order
    with the same arithmetic.  Uncompensated: bit-identical.  Compensated,
    the row walk adds its colour terms (all >= 0) in groups of at most 64
    (a fused multiply-add into a partial sum, then a compensated add of
    the partial) where the other strategies add each term compensated: a
    partial of n terms is off by at most n u of its sum (u = 2^-24) and
    each compensated add by 2u of the total, so a pixel differs by at most
    (64 + 4) u = 4.1e-6 of its value; the check allows 1e-5."""
    if not compensated:
        assert np.array_equal(a, b), what
        return
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    bound = 1e-5 * np.maximum(np.abs(a64), np.abs(b64)) + 1e-30
    assert np.all(np.abs(a64 - b64) <= bound), (what, float(np.max(np.abs(a64 - b64) / bound)))


@pytest.mark.parametrize("tile", [8, 16, 32])
@pytest.mark.parametrize("compensated", [False, True])
def test_box_mapped_lanes_bitwise_equal_rows(torch_cuda, orc, tile, compensated):
    """Box-mapped lanes (variant 3) composite each pixel's particles in the
    same order with the same arithmetic as the row walk (variant 1), also
    with short segments (partials merged): bit-identical images without
    compensation, the grouping bound with it (same_composite); both agree
    with the oracle."""
    for name, (scene, iin) in _strategy_scenes().items():
        for seg in (0, 256):
            kw = dict(tile=tile, compensated=compensated, seg_records=seg)
            rows = gpu_render(scene, img_in=iin, splat_variant=1, **kw)
            box = gpu_render(scene, img_in=iin, splat_variant=3, **kw)
            same_composite(rows, box, compensated, (name, seg))
        check_image(box, orc.render(scene, img_in=iin))


def test_box_mapped_lanes_chunked(torch_cuda, orc):
    scene = c2_small(40_000, seed=4, w=240, h=160)
    img, st = gpu_render(scene, max_pairs=5000, stats=True, splat_variant=3)
    assert st["n_chunks"] > 3
    check_image(img, orc.render(scene))


def test_statistics_do_not_change_the_image(torch_cuda):
    """Frames that do not report member statistics (they are reported with
    profiled stats) run the row walk without its member counters; the image
    is the same bits either way."""
    scene = c2_small(60_000, seed=9, w=320, h=200)
    plain = gpu_render(scene, compensated=True)
    counted, st = gpu_render(scene, compensated=True, profile=2)
    assert np.array_equal(plain, counted)
    assert st["n_member_pairs"] > 0 and 0 < st["n_member_absorbing"] < st["n_member_pairs"]


def test_block_masks_on_and_off_bitwise_equal(torch_cuda):
    """Pair keys carry the mask of the tile's 8x8 blocks a footprint meets
    when the tile index leaves room above the sort's digits: 16 px tiles
    here, and 32 px tiles of a small image.  On a 16384 x 4160 image the
    66,560 tiles of 32 px need 17 bits, the sort orders 24, and the masks
    are off (every pair queued for every block); 8 px tiles never carry
    masks.  With one list segment per tile each pixel composites the same
    particles in the same order through the same arithmetic, so without
    compensation all of these images are bit-identical; with it the
    groups of colour terms differ (a block's batches hold other records
    when the masks are off) and the images agree to the grouping bound."""
    def one(scene, tile, compensated):
        img, st = gpu_render(scene, tile=tile, compensated=compensated, seg_records=1 << 24,
                             splat_variant=1, max_pairs=1 << 24, stats=True)
        assert st["n_chunks"] == 1, (tile, st["n_pairs"])
        return img

    for w, h in ((16384, 4160), (480, 270)):
        scene = wide_scene(w, h)
        for compensated in (False, True):
            ref = one(scene, 16, compensated)
            assert np.any(ref > 0)
            for tile in (32, 8):
                same_composite(one(scene, tile, compensated), ref, compensated, (w, tile))


def corner_scene(n=30_000, seed=19, w=256):
    """Footprints centred near the corners where four 8x8 blocks meet, with
    radii that put the circle at, just inside or just outside the nearest
    pixel centre of the diagonal block: the cases where a box's corner block
    is left out of a pair's block mask or kept by one rounding."""
    rng = np.random.default_rng(seed)
    cam = synth.ortho_unit_square(w, w)
    cx = 8.0 * rng.integers(2, w // 8 - 2, n) + rng.choice([-1.5, -0.75, -0.5, 0.0, 0.25, 0.5, 1.0], n)
    cy = 8.0 * rng.integers(2, w // 8 - 2, n) + rng.choice([-1.25, -0.5, 0.0, 0.5, 0.75, 1.5], n)
    # distance to the nearest pixel centre across the block corner (8a, 8b)
    dx = np.abs(np.round(cx / 8.0) * 8.0 + np.where(cx < np.round(cx / 8.0) * 8.0, 0.5, -0.5) - cx)
    dy = np.abs(np.round(cy / 8.0) * 8.0 + np.where(cy < np.round(cy / 8.0) * 8.0, 0.5, -0.5) - cy)
    d = np.hypot(dx, dy)
    r = d * rng.choice([1.0 - 1e-3, 1.0 - 1e-7, 1.0, 1.0 + 1e-7, 1.0 + 1e-3, 1.6], n)
    r = np.maximum(r, 0.3)
    sc = synth.Scene((cx / w).astype(np.float32), (cy / w).astype(np.float32),
                     rng.uniform(0.0, 1.0, n).astype(np.float32),
                     (r / (2.0 * w)).astype(np.float32),  # trunc_f 2, sigma_over_h 1
                     rng.lognormal(0, 1, n).astype(np.float32), cam,
                     [synth.Species(log_scale=1, brightness=0.5, absorption=0.5,
                                    mode=synth.ORDERED),
                      synth.Species(brightness=0.4, mode=synth.ADDITIVE)],
                     species=rng.integers(0, 2, n).astype(np.uint8), name="corners")
    return sc


def test_corner_blocks_left_out_keep_every_member(torch_cuda, orc):
    """A pair's block mask leaves out the box's corner blocks whose nearest
    pixel is outside the radius by the row walk's own rounding.  With
    footprints placed on block corners at the threshold, renders with the
    masks (16 and 32 px tiles) match the unmasked 8 px tiles bit for bit
    without compensation, and every render matches the oracle."""
    scene = corner_scene()
    ref = orc.render(scene)

    def one(tile, compensated):
        img, st = gpu_render(scene, tile=tile, compensated=compensated, seg_records=1 << 24,
                             splat_variant=1, max_pairs=1 << 24, stats=True)
        assert st["n_chunks"] == 1
        return img

    for compensated in (False, True):
        base = one(8, compensated)
        check_image(base, ref)
        for tile in (16, 32):
            img = one(tile, compensated)
            same_composite(img, base, compensated, ("corners", tile))
            check_image(img, ref)


@pytest.mark.parametrize("spread", [0.0, 1e-6, 0.25])
def test_depth_sort_over_the_visible_key_span(torch_cuda, orc, spread):
    """The depth sort runs only over the digits the visible depth keys span:
    equal depths (span 0, the index decides), a span of a few ulps across a
    power of two, and a wide one; invisible particles (behind the camera,
    invalid) carry keys outside the span.  Pair lists are bit-exact."""
    rng = np.random.default_rng(int(spread * 1e6) + 3)
    n = 20_000
    cam = synth.ortho_unit_square(96, 80)
    z = (0.5 + spread * rng.uniform(-1, 1, n)).astype(np.float32)
    z[:50] = -3.0                     # behind the camera: not visible
    x = rng.uniform(0, 1, n).astype(np.float32)
    x[50:60] = np.nan                 # invalid
    sp = [synth.Species(log_scale=1, brightness=0.4, absorption=0.6, mode=synth.ORDERED),
          synth.Species(brightness=0.3, mode=synth.ADDITIVE)]
    scene = synth.Scene(x, rng.uniform(0, 1, n).astype(np.float32), z,
                        rng.lognormal(np.log(0.02), 0.5, n).astype(np.float32),
                        rng.lognormal(0, 1, n).astype(np.float32), cam, sp,
                        species=rng.integers(0, 2, n).astype(np.uint8))
    if spread == 1e-6:
        # view depths 2 and 2 - 2^-22: keys on both sides of an exponent step
        scene.z = np.where(np.arange(n) % 2 == 0, np.float32(1.0),
                           np.float32(1.0 - 2.0 ** -22)).astype(np.float32)
        scene.z[:50] = -3.0
    parts, pal = B.scene_to_device(scene)
    ts, te, pp, npairs = B.bin_pairs(parts, scene.camera, scene.species_params,
                                      sigma_over_h=scene.sigma_over_h, trunc_f=scene.trunc_f,
                                      tile=16)
    ref = orc.project(scene, tile=16)
    es, ee, ep = expected_bins(ref, scene, 16, True)
    assert npairs == ep.size
    assert np.array_equal(pp.cpu().numpy().view(np.uint32).astype(np.int64), ep)
    check_image(gpu_render(scene), orc.render(scene))
    # A batch reads nothing back: its depth passes take the key range from
    # the device and return past its digits; the images are the single
    # render's bits.
    for compensated in (False, True):
        kw = dict(sigma_over_h=scene.sigma_over_h, trunc_f=scene.trunc_f, tile=16,
                  compensated=compensated)
        one = B.render(parts, scene.camera, pal, scene.species_params, **kw).cpu().numpy()
        for streams in (1, 2):
            imgs = B.render_batch(parts, [scene.camera, scene.camera], pal,
                                  scene.species_params, streams=streams, **kw)
            for im in imgs:
                assert np.array_equal(im.cpu().numpy(), one), (spread, compensated, streams)


@pytest.mark.parametrize("n", [4096, 16384, 16385, 20480, 20481])
def test_scans_around_the_one_workgroup_size(torch_cuda, orc, n):
    """Scans of at most four 4096-element tiles run in one workgroup, longer
    ones in three kernels: particle counts at and just past both sizes give
    bit-exact pair lists (the pair offsets are a scan over the particles)."""
    rng = np.random.default_rng(n)
    cam = synth.ortho_unit_square(80, 64)
    sp = [synth.Species(log_scale=1, brightness=0.4, absorption=0.6, mode=synth.ORDERED),
          synth.Species(brightness=0.3, mode=synth.ADDITIVE)]
    scene = synth.Scene(rng.uniform(0, 1, n).astype(np.float32),
                        rng.uniform(0, 1, n).astype(np.float32),
                        rng.uniform(0, 1, n).astype(np.float32),
                        rng.lognormal(np.log(0.03), 0.6, n).astype(np.float32),
                        rng.lognormal(0, 1, n).astype(np.float32), cam, sp,
                        species=rng.integers(0, 2, n).astype(np.uint8))
    parts, pal = B.scene_to_device(scene)
    ts, te, pp, npairs = B.bin_pairs(parts, scene.camera, scene.species_params,
                                      sigma_over_h=scene.sigma_over_h, trunc_f=scene.trunc_f,
                                      tile=16)
    ref = orc.project(scene, tile=16)
    es, ee, ep = expected_bins(ref, scene, 16, True)
    assert npairs == ep.size
    assert np.array_equal(pp.cpu().numpy().view(np.uint32).astype(np.int64), ep)
    assert np.array_equal(ts.cpu().numpy().astype(np.int64), es)
    assert np.array_equal(te.cpu().numpy().astype(np.int64), ee)
    check_image(gpu_render(scene, compensated=True), orc.render(scene))


def test_batch_with_nothing_visible(torch_cuda):
    """Every particle behind the camera: the depth-key range on the device is
    empty (smallest above largest), the batch's one sorting pass orders
    nothing, and the images stay black like the single render's."""
    rng = np.random.default_rng(5)
    n = 5_000
    cam = synth.ortho_unit_square(64, 48)
    sp = [synth.Species(log_scale=1, brightness=0.4, absorption=0.6, mode=synth.ORDERED)]
    scene = synth.Scene(rng.uniform(0, 1, n).astype(np.float32),
                        rng.uniform(0, 1, n).astype(np.float32),
                        np.full(n, -3.0, np.float32),
                        np.full(n, 0.02, np.float32), np.ones(n, np.float32), cam, sp)
    parts, pal = B.scene_to_device(scene)
    one = B.render(parts, cam, pal, scene.species_params, tile=16).cpu().numpy()
    assert not np.any(one)
    imgs, st = B.render_batch(parts, [cam, cam], pal, scene.species_params, tile=16, streams=2,
                              stats=True)
    assert all(v["n_pairs"] == 0 for v in st)
    for im in imgs:
        assert np.array_equal(im.cpu().numpy(), one)


def test_edges_ordered_with_background(torch_cuda, orc):
    scene = edge_scene()
    iin = np.random.default_rng(3).uniform(0, 0.6, (3, 77, 101))
    ref = orc.render(scene, img_in=iin)
    img = gpu_render(scene, img_in=iin)
    check_image(img, ref)


def test_general_e_not_a_two_species(torch_cuda, orc):
    """Species with different source functions E/A: order matters."""
    scene = c2_small(60_000, seed=9, w=200, h=150)
    scene.species_params = [
        synth.Species(log_scale=1, brightness=0.1, absorption=0.4, mode=synth.ORDERED),
        synth.Species(log_scale=1, brightness=0.3, absorption=0.05, mode=synth.ORDERED)]
    ref = orc.render(scene)
    check_image(gpu_render(scene), ref)


def test_large_optical_depth_steps(torch_cuda, orc):
    """Absorption large enough that single-particle optical depths exceed
    the series threshold."""
    scene = c2_small(30_000, seed=10, w=160, h=120)
    scene.species_params = [
        synth.Species(log_scale=1, brightness=3.0, absorption=3.0, mode=synth.ORDERED),
        synth.Species(log_scale=1, brightness=0.5, absorption=0.0, mode=synth.ADDITIVE)]
    scene.rho0 = np.random.default_rng(1).uniform(0.1, 4.0, scene.n).astype(np.float32)
    ref = orc.render(scene)
    check_image(gpu_render(scene), ref)


def test_chunked_equals_unchunked(torch_cuda, orc):
    """A workspace too small for all pairs forces several passes; additive
    chunks add, ordered chunks are depth slabs composited back to front."""
    for scene in (c1(20_000, seed=3), c2_small(40_000, seed=4, w=240, h=160)):
        ref = orc.render(scene)
        full = gpu_render(scene)
        img, st = gpu_render(scene, max_pairs=5000, stats=True)
        assert st["n_chunks"] > 3
        check_image(img, ref)
        check_image(img, full.astype(np.float64), tol=2e-5)


def test_empty_and_all_culled(torch_cuda, orc):
    import torch
    scene = c1(10, seed=5)
    empty = scene.subset(np.arange(0))
    iin = np.full((3, 256, 256), 0.25, np.float32)
    assert np.array_equal(gpu_render(empty), np.zeros((3, 256, 256), np.float32))
    assert np.array_equal(gpu_render(empty, img_in=iin), iin)
    culled = scene.subset(np.arange(10))
    culled.z = np.full(10, -50.0, np.float32)
    img, st = gpu_render(culled, stats=True)
    assert np.array_equal(img, np.zeros((3, 256, 256), np.float32))
    assert st["n_depth_culled"] == 10 and st["n_pairs"] == 0


def test_one_particle_closed_form(torch_cuda):
    """Pixel centred on the particle holds E rho0; one sigma away E rho0/e."""
    cam = synth.ortho_unit_square(64, 64)
    sc = synth.Scene(np.array([20.5 / 64], np.float32), np.array([30.5 / 64], np.float32),
                     np.array([0.5], np.float32), np.array([3.0 / 64], np.float32),
                     np.array([1.0], np.float32), cam,
                     [synth.Species(vmin=0.0, vmax=2.0, brightness=2.0)],
                     rho0=np.array([0.7], np.float32))
    sc.palette = np.ones((2, 3), np.float32)
    img = gpu_render(sc)
    peak = 2.0 * np.float32(0.7)
    assert img[0, 30, 20] == pytest.approx(peak, rel=1e-6)
    assert img[1, 30, 23] == pytest.approx(peak * np.exp(-1.0), rel=1e-5)
    assert img[2, 37, 20] == 0.0


def test_kahan_many_identical(torch_cuda):
    """n identical particles on one pixel: the compensated sum is n w to
    within (g + 2) u, u = 2^-24: the row walk adds at most g = 64 terms of a
    batch into a partial sum (off by at most g u of the partial) and adds
    the partials compensated (2 u of the total).  Identical terms are the
    worst case for the partials, whose rounding errors all have one sign.
    The plain FP32 sum drifts further (its segments of the tile's list are
    also partial sums, merged plainly)."""
    n = 200_000
    cam = synth.ortho_unit_square(16, 16)
    sc = synth.Scene(np.full(n, 8.5 / 16, np.float32), np.full(n, 8.5 / 16, np.float32),
                     np.linspace(0.1, 0.9, n).astype(np.float32), np.full(n, 1.3 / 16, np.float32),
                     np.ones(n, np.float32), cam, [synth.Species(vmin=0.0, vmax=2.0, brightness=0.1)])
    sc.palette = np.ones((2, 3), np.float32)
    ref = n * float(np.float32(0.1))
    k = gpu_render(sc, compensated=True)[0, 8, 8]
    p = gpu_render(sc, compensated=False)[0, 8, 8]
    assert abs(k - ref) / ref < 66 * 2.0 ** -24
    assert abs(k - ref) < abs(p - ref)


def test_deterministic_and_permutation(torch_cuda, orc):
    """Two runs are bit-identical; with distinct depth keys the ordered path
    is bit-identical under a permutation of the input (same sorted order)."""
    scene = c2_small(50_000, seed=11, w=200, h=120)
    a = gpu_render(scene)
    b = gpu_render(scene)
    assert np.array_equal(a, b)
    key = orc.project(scene)["key"]
    _, first, counts = np.unique(key, return_index=True, return_counts=True)
    keep = np.sort(first[counts == 1])
    sub = scene.subset(keep)
    ref = gpu_render(sub)
    perm = np.random.default_rng(2).permutation(sub.n)
    c = gpu_render(sub.subset(perm))
    assert np.array_equal(ref, c)


def test_c2_full_size_sampled(torch_cuda, orc):
    """The full NFW configuration (1e7 particles, 1920x1080, mixed species)
    in the launch configuration the benchmark uses, checked on sampled
    pixels the oracle evaluates one by one, plus bit-exact projection."""
    scene = synth.nfw_halos(10_000_000, seed=2)
    img, st = gpu_render(scene, compensated=True, stats=True)
    rng = np.random.default_rng(0)
    # random pixels plus the brightest ones
    flat = img.sum(0).ravel()
    top = np.argsort(flat)[-64:]
    rnd = rng.integers(0, flat.size, 448)
    idx = np.concatenate([top, rnd])
    pj, pi = np.unravel_index(idx, (1080, 1920))
    ref = orc.render_pixels(scene, pi, pj)
    got = img[:, pj, pi].T.astype(np.float64)
    scale = np.abs(ref).max(axis=0)
    rel = np.abs(got - ref).max(axis=0) / np.where(scale > 0, scale, 1)
    assert np.all(rel <= TOL), rel
    assert st["n_visible"] > 7_000_000  # the 16:9 frame crops the box top and bottom


@pytest.mark.parametrize("name", ["c1", "c2_small", "edges"])
def test_tile64_row_walk(torch_cuda, orc, name):
    """64 px tiles (row walk only: 64 single-wave workgroups per tile, no
    block masks in the keys) against the oracle, whole and in chunks."""
    scene = {"c1": lambda: c1(60_000, seed=13), "c2_small": lambda: c2_small(80_000, seed=14),
             "edges": edge_scene}[name]()
    ref = orc.render(scene)
    img, st = gpu_render(scene, tile=64, compensated=True, stats=True)
    assert st["tile"] == 64
    check_image(img, ref)
    img, st = gpu_render(scene, tile=64, max_pairs=max(64, st["n_pairs"] // 4), seg_records=64,
                         stats=True)
    assert st["n_chunks"] > 1
    check_image(img, ref)
