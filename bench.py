#!/usr/bin/env python3
"""Benchmark: one render of a device-resident synthetic particle set per step.

Default workload: 1e9 particles drawn from a lognormal density field on a
512^3 grid (sigma 1.5, per-cell Poisson sampling, box 100), two species
(gas depth-ordered with absorption equal to emission, dark matter additive),
perspective camera with a 60 degree field of view, 4096x4096 float32 RGB,
compensated accumulation.  Particles are generated on the GPU and resident
in HBM before the timed region starts.

Prints one JSON line: Mparticles/s (whole job), frames/s, the roofline
figure of the dominant kernel (timed with HIP events inside the library on
the stream it runs on) and the FP64 CPU oracle's rate on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mparticles/s and frames/s at 4096² (1 GPU); learned vs plain at PSNR≥40dB"
HBM_PEAK_GBS = 8000.0
# MI355X published FP32 vector peak (256 CUs x 2.4 GHz x 256 flops/clk, which
# counts packed FP32 FMA); the kernels are built without packed FP32, so
# the unpacked FMA rate (256 CU x 64 lanes x 2 x 2.4 GHz) is given beside it
FP32_VECTOR_PEAK_TFLOPS = 157.3
FP32_FMA_UNPACKED_TFLOPS = 78.6
# algorithmic FP32 operations per composited (pixel, particle) contribution:
# emission only, about 10 flops (weight: scale and exp; per channel E w, and
# T E w) plus 1 exp and 12 for the compensated add of three channels;
# absorbing, about 25 flops plus 4 exp (weight and three transmittances)
FLOPS_EMISSION = 23
FLOPS_ABSORBING = 29


SPLAT_KERNELS = {0: "k_splat_rows", 1: "k_splat_rows", 2: "k_splat_lists", 3: "k_splat_box"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def measured_traffic(kernel, cfg, args):
    """HBM bytes per launch of the dominant kernel from the committed
    counter record (two rocprofv3 --pmc runs, FETCH_SIZE then WRITE_SIZE,
    each scaled by the same counter's reading for a copy of known size), or
    None when no record covers this kernel and workload or the kernel's
    sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_lognormal_1e9_4096.json")
    if not os.path.exists(path) or cfg.get("workload") != "lognormal_field":
        return None
    if cfg.get("n_target") != 1_000_000_000 or args.max_pairs:
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec or rec.get("tile") != args.tile:
        return None
    h = hashlib.sha256()
    for src in rec["sources"]:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    if h.hexdigest() != rec["sources_sha256"]:
        return None
    return rec["traffic_bytes_per_launch"]


def make_workload(args, torch):
    from paper_1004_1302_amd import binding as B
    from paper_1004_1302_amd import synth
    dev = torch.device("cuda:0")
    if args.workload == "lognormal":
        n = int(args.n or 1_000_000_000)
        grid = args.grid or 512
        parts, cam, sp = synth.lognormal_field(n_target=n, grid=grid, sigma=1.5, seed=3,
                                               width=4096, height=4096, device="cuda:0")
        pal = torch.from_numpy(synth.palette(256)).to(dev)
        cfg = dict(workload="lognormal_field", n_target=n, grid=grid, sigma=1.5, box=100.0,
                   width=4096, height=4096, camera="perspective fov 60",
                   species="gas ordered E=A + dark matter additive", compensated=True)
    elif args.workload == "nfw":
        n = int(args.n or 10_000_000)
        sc = synth.nfw_halos(n, seed=2)
        parts, pal = B.scene_to_device(sc, "cuda:0")
        cam, sp = sc.camera, sc.species_params
        cfg = dict(workload="nfw_halos", n_target=n, width=1920, height=1080,
                   camera="perspective fov 60", species="gas ordered E=A + dark matter additive",
                   compensated=True)
    elif args.workload == "plummer":
        n = int(args.n or 100_000)
        sc = synth.plummer_mix(n, seed=1)
        parts, pal = B.scene_to_device(sc, "cuda:0")
        cam, sp = sc.camera, sc.species_params
        cfg = dict(workload="plummer_mix", n_target=n, width=256, height=256, camera="ortho z",
                   species="additive", compensated=True)
    else:
        raise SystemExit(f"unknown workload {args.workload}")
    return parts, cam, sp, pal, cfg


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_scene(parts, cam, sp, idx=None):
    """Host copy of (a subset of) the device particles as an oracle scene."""
    from paper_1004_1302_amd import synth
    pick = (lambda t: t[idx]) if idx is not None else (lambda t: t)
    host = {key: pick(t).cpu().numpy() for key, t in parts.items()}
    return synth.Scene(host["x"], host["y"], host["z"], host["h"], host["value"], cam, sp,
                       species=host.get("species"), rho0=host.get("rho0"))


def cpu_baseline(parts, cam, sp, args, np, torch):
    """The FP64 oracle timed on the host cores: row bands of the image
    painted by all OpenMP threads (the same image as the single-thread
    definition, bit for bit).  Sets above 1e7 particles are timed on a
    seeded random subsample (--cpu-fraction, default 1/50: about 8 s a run
    on 16 threads, where the full set in FP64 would not fit host memory) and
    the per-particle rate is extrapolated; smaller sets are timed whole."""
    import oracle
    n = int(parts["x"].numel())
    frac = 1.0 if n <= 10_000_000 else float(args.cpu_fraction)
    k = max(1, int(round(n * frac)))
    if k < n:
        gen = torch.Generator(device="cpu")
        gen.manual_seed(17)
        idx = torch.unique(torch.randint(0, n, (k,), generator=gen)).to(parts["x"].device)
        k = int(idx.numel())
        scene = host_scene(parts, cam, sp, idx)
    else:
        scene = host_scene(parts, cam, sp)
    oracle.lib()
    threads = oracle.threads()
    runs = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.render_rows(scene, band=16)
        runs.append(time.perf_counter() - t0)
    dt = float(np.median(runs))
    what = (f"seeded random subsample of {k} of {n} particles (1/{round(n / k)}), rate "
            f"extrapolated per particle" if k < n else f"all {n} particles")
    return dict(value=round(k / dt / 1e6, 6), unit="Mparticles/s", cores=threads, kind="oracle",
                nproc=os.cpu_count(), cpu_model=cpu_model(), extrapolated=k < n,
                sample=f"{what}; same camera and {cam.width}x{cam.height} image; FP64, row "
                       f"bands on {threads} OpenMP threads; median of 3 runs, {dt:.2f} s each")


def sampled_error(parts, cam, sp, image, np, n_random=1984, n_top=64):
    """Oracle check of the timed frame on sampled pixels (the brightest plus
    random ones), each evaluated by the oracle over every particle.
    Returns the relative L-infinity error per channel (normalised by the
    largest sampled oracle value) and the largest per-pixel relative error
    with an absolute floor of 1e-6 of that value."""
    import oracle
    img = image.cpu().numpy()
    H, W = img.shape[1:]
    rng = np.random.default_rng(0)
    flat = img.sum(0).ravel()
    pix = np.concatenate([np.argsort(flat)[-n_top:], rng.integers(0, flat.size, n_random)])
    pj, pi = np.unravel_index(pix, (H, W))
    scene = host_scene(parts, cam, sp)
    t0 = time.perf_counter()
    ref = oracle.render_pixels(scene, pi, pj)
    dt = time.perf_counter() - t0
    got = img[:, pj, pi].T.astype(np.float64)
    scale = np.abs(ref).max(axis=0)
    scale = np.where(scale > 0, scale, 1.0)
    rel = np.abs(got - ref).max(axis=0) / scale
    per_px = (np.abs(got - ref) / (np.abs(ref) + 1e-6 * scale)).max(axis=0)
    return dict(pixels=int(pix.size), rel_linf_per_channel=[float(f"{v:.3e}") for v in rel],
                per_pixel_rel_max=[float(f"{v:.3e}") for v in per_px],
                per_pixel_floor="1e-6 of the largest sampled value", oracle_seconds=round(dt, 1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal",
                    choices=["lognormal", "nfw", "plummer", "learned", "batch", "copy", "split"])
    ap.add_argument("--copy-mib", type=int, default=2048)
    ap.add_argument("--views", type=int, default=32)
    ap.add_argument("--batch-set", default="nfw", choices=["nfw", "plummer"])
    ap.add_argument("--train-pairs", type=int, default=4000)
    ap.add_argument("--train-sets", type=int, default=8)
    ap.add_argument("--test-views", type=int, default=20)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--n", type=float, default=0)
    ap.add_argument("--grid", type=int, default=0)
    # 32 px tiles: 1.46 pairs per particle on the 1e9 field against 2.02
    # at 16 px, so a shorter tile sort and emission for a splat 2% longer
    ap.add_argument("--tile", type=int, default=32)
    ap.add_argument("--splat-variant", type=int, default=0)
    ap.add_argument("--max-pairs", type=float, default=0)
    ap.add_argument("--cpu-fraction", type=float, default=0.02)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the renderer "
              "has no multi-GPU path", file=sys.stderr)
        raise SystemExit(2)

    import numpy as np
    import torch
    from paper_1004_1302_amd import binding as B
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.workload == "learned":
        return learned_leg(args, np, torch)
    if args.workload == "batch":
        return batch_leg(args, np, torch)
    if args.workload == "copy":
        return copy_leg(args, torch)
    if args.workload == "split":
        return split_leg(args, np, torch)

    t0 = time.perf_counter()
    parts, cam, sp, pal, cfg = make_workload(args, torch)
    torch.cuda.synchronize()
    n = int(parts["x"].numel())
    log(f"workload {cfg['workload']}: {n} particles generated in {time.perf_counter() - t0:.1f} s")
    W, H = cam.width, cam.height
    image = torch.empty((3, H, W), dtype=torch.float32, device="cuda:0")
    max_pairs = int(args.max_pairs) if args.max_pairs else 4 * n + 65536
    kw = dict(compensated=True, tile=args.tile, max_pairs=max_pairs,
              splat_variant=args.splat_variant)

    def step(profile=False):
        return B.render(parts, cam, pal, sp, image, profile=profile, **kw)

    for w in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {w + 1}/{args.warmup} done")
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for s in range(args.steps):
        step()
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    log(f"timed {args.steps} steps: {ms:.3f} ms/step")

    # per-stage breakdown with the library's own HIP events, from frames
    # that run the same kernels as the timed ones (profile level 1), then
    # one frame that also counts the composited (pixel, particle) pairs
    # (profile level 2: the splat's counting variant)
    stage_runs = []
    for s in range(max(1, min(args.steps, 5))):
        _, st = step(profile=1)
        stage_runs.append(st)
    stages = {k: float(np.mean([r["stage_ms"][k] for r in stage_runs]))
              for k in stage_runs[0]["stage_ms"]}
    _, st = step(profile=2)
    dominant = max(stages, key=stages.get)
    log(f"stages ms: {json.dumps({k: round(v, 3) for k, v in stages.items()})}")
    n_mem, n_abs = st["n_member_pairs"], st["n_member_absorbing"]
    pairs = st["n_pairs"]
    # algorithmic work of the dominant stage per launch
    if dominant == "splat":
        flops = FLOPS_EMISSION * (n_mem - n_abs) + FLOPS_ABSORBING * n_abs
        ach = flops / (stages["splat"] * 1e-3) / 1e12
        kern = SPLAT_KERNELS.get(args.splat_variant, "k_splat_rows")
        roof = dict(bound="alu", achieved=round(ach, 3), peak=FP32_VECTOR_PEAK_TFLOPS,
                    unit="TFLOP/s", frac=round(ach / FP32_VECTOR_PEAK_TFLOPS, 4),
                    traffic=measured_traffic(kern, cfg, args), kernel=kern,
                    kernel_ms=round(stages["splat"], 3), flops_per_launch=flops,
                    flops_per_pair=dict(emission_only=FLOPS_EMISSION, absorbing=FLOPS_ABSORBING),
                    member_pairs=n_mem, member_pairs_absorbing=n_abs,
                    peak_fma_unpacked=FP32_FMA_UNPACKED_TFLOPS,
                    frac_fma_unpacked=round(ach / FP32_FMA_UNPACKED_TFLOPS, 4))
    else:
        algo_bytes = {
            "project": n * (24 + 4 + 1) + st["n_visible"] * 32 + n * 8,
            "depth_sort": n * 4 * 20 + n * 12,
            "scan": n * 12,
            "emit": n * 16 + pairs * 8,
            "tile_sort": pairs * 20 * 2 + pairs * 8,
        }[dominant]
        ach = algo_bytes / (stages[dominant] * 1e-3) / 1e9
        roof = dict(bound="hbm", achieved=round(ach, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(ach / HBM_PEAK_GBS, 4), traffic=None, kernel=dominant)
    out = {
        "metric": METRIC,
        "value": round(n / (ms * 1e-3) / 1e6, 3),
        "unit": "Mparticles/s",
        "fps": round(1000.0 / ms, 4),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(cfg, n_particles=n, tile=args.tile, splat_variant=args.splat_variant,
                       pairs=pairs,
                       chunks=st["n_chunks"], visible=st["n_visible"]),
        "stages_ms": {k: round(v, 3) for k, v in stages.items()},
        "roofline": roof,
    }
    if not args.no_check:
        log("oracle check of the timed frame on sampled pixels ...")
        out["parity"] = sampled_error(parts, cam, sp, image, np)
        log(f"parity: {out['parity']}")
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(parts, cam, sp, args, np, torch)
    print(json.dumps(out), flush=True)
    # hand the device memory back before the process ends
    del parts, image
    B.release_workspace()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()


def split_leg(args, np, torch):
    """Split particles (Section 3.2, Table 2): NFW halo sets of the three
    sizes of the paper's table (370,852, 2,646,991 and 16,202,527 particles)
    seen from inside the box at 1920x1080, so that footprints range from a
    pixel to the whole window.  For each set: frame time and the pair
    emission stage with splitting off, at the paper's threshold (W+H)/2 =
    1500 pixels, and at other thresholds (median of --steps frames each)."""
    from paper_1004_1302_amd import binding as B
    from paper_1004_1302_amd import synth
    W, H = 1920, 1080
    cam = synth.look_at((50.0, 50.0, 10.0), (50.0, 50.0, 60.0), (0.0, 1.0, 0.0),
                        synth.PERSPECTIVE, W, H, z_near=0.5, z_far=500.0)
    thresholds = [-1, 64, 256, (W + H) // 2, 4096, 16384, 65536]
    sets = []
    for name, n in (("small", 370_852), ("medium", 2_646_991), ("large", 16_202_527)):
        sc = synth.nfw_halos(n, seed=2)
        parts, pal = B.scene_to_device(sc, "cuda:0")
        sp = sc.species_params
        image = torch.empty((3, H, W), dtype=torch.float32, device="cuda:0")
        rows = {}
        ref = None
        for thr in thresholds:
            kw = dict(compensated=True, split_pixels=thr)
            B.render(parts, cam, pal, sp, image, **kw)
            torch.cuda.synchronize()
            if ref is None:
                ref = image.clone()
            elif not torch.equal(image, ref):
                raise SystemExit(f"split threshold {thr} changed the image")
            frame, emit = [], []
            for _ in range(max(3, args.steps)):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                B.render(parts, cam, pal, sp, image, **kw)
                e1.record()
                _, st = B.render(parts, cam, pal, sp, image, profile=1, **kw)
                torch.cuda.synchronize()
                frame.append(e0.elapsed_time(e1))
                emit.append(st["stage_ms"]["emit"])
            rows[str(thr)] = dict(frame_ms=round(float(np.median(frame)), 3),
                                  emit_ms=round(float(np.median(emit)), 3))
        _, st = B.render(parts, cam, pal, sp, image, stats=True, compensated=True)
        del parts, image
        B.release_workspace()
        torch.cuda.empty_cache()
        sets.append(dict(set=name, n_particles=n, pairs=st["n_pairs"], timings=rows,
                         split_vs_none_frame=round(rows[str((W + H) // 2)]["frame_ms"] /
                                                   rows["-1"]["frame_ms"], 4),
                         split_vs_none_emit=round(rows[str((W + H) // 2)]["emit_ms"] /
                                                  rows["-1"]["emit_ms"], 4)))
        log(f"split: {name} {json.dumps(rows)}")
    out = {"metric": "frame ms with and without split particles", "value":
           sets[-1]["timings"][str((W + H) // 2)]["frame_ms"], "unit": "ms (large set, (W+H)/2)",
           "higher_is_better": False, "n_gpus": 1, "dtype": "f32", "data": "synthetic",
           "config": dict(workload="split_particles", width=W, height=H,
                          camera="inside the NFW box, 60 deg", thresholds_px=thresholds,
                          paper_threshold_px=(W + H) // 2),
           "sets": sets}
    print(json.dumps(out), flush=True)


def copy_leg(args, torch):
    """Plain device-to-device copies of --copy-mib MiB: the achieved
    streaming rate (read + write) the HBM-bound passes are compared with,
    and, run under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE), the
    known bytes that calibrate those counters."""
    n = args.copy_mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)  # first touch
    torch.cuda.synchronize()
    reps = max(3, args.steps)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
    ev[0].record()
    for k in range(reps):
        dst.copy_(src)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(reps)]
    best = min(ms)
    print(json.dumps({"metric": "device copy bandwidth (read + write)",
                      "value": round(2 * n * 4 / (best * 1e-3) / 1e12, 3), "unit": "TB/s",
                      "copy_bytes_read": n * 4, "copy_bytes_written": n * 4,
                      "dispatches": reps + 1, "ms": [round(m, 4) for m in ms]}), flush=True)


def batch_leg(args, np, torch):
    """Many views of one device-resident particle set.  --batch-set nfw: the
    NFW halo set (--n particles, default 1e7, mixed ordered species),
    --views cameras on a seeded orbit, each of one of four sizes (1920x1080,
    1280x720, 1024x1024, 640x480; for 1e6 particles or fewer 320x240,
    256x256, 200x150, 128x128).  --batch-set plummer: the batched-views
    workload, the small-config generator (default 5e7 particles, additive)
    seen from the unit-cube orbit at 512², 1024², 1920x1080 and 2048² (pass
    --max-pairs for the largest views).  The autotuner picks tile and
    segment length on the first view; one checked batch (stats on) runs
    before timing.  Timed: one render call per view, one batch call (eager), and
    replays of the batch captured as a HIP graph, each on one stream and on
    four; wall clock per batch with the device synchronised on both
    sides.  `value` is the fastest batch mode's views/s."""
    from paper_1004_1302_amd import autotune
    from paper_1004_1302_amd import binding as B
    from paper_1004_1302_amd import synth
    if args.batch_set == "plummer":
        # the batched-views workload: the small-config generator (one
        # additive species) on the unit-cube orbit, 512² to 2048² views
        n = int(args.n or 50_000_000)
        sc = synth.plummer_mix(n, seed=41)
        sizes = [(512, 512), (1024, 1024), (1920, 1080), (2048, 2048)]
        cams = synth.orbit_cameras(args.views, 7, sizes)
        name = "plummer_mix_multiview"
    else:
        n = int(args.n or 10_000_000)
        sc = synth.nfw_halos(n, seed=2)
        # light sets use thumbnail sizes, where launch overhead is a large share
        sizes = ([(1920, 1080), (1280, 720), (1024, 1024), (640, 480)] if n > 1_000_000 else
                 [(320, 240), (256, 256), (200, 150), (128, 128)])
        cams = synth.orbit_cameras(args.views, 7, sizes, centre=(50.0, 50.0, 50.0),
                                   radius=150.0, z_near=1.0, z_far=1000.0)
        name = "nfw_halos_multiview"
    parts, pal = B.scene_to_device(sc, "cuda:0")
    sp = sc.species_params
    tuned = autotune.tune(parts, cams[0], pal, sp, use_cache=False, compensated=True)
    log(f"autotune: tile {tuned['tile']} seg_records {tuned['seg_records']}")
    kw = dict(compensated=True, tile=tuned["tile"], seg_records=tuned["seg_records"],
              max_pairs=int(args.max_pairs or 0))
    images = [torch.empty((3, c.height, c.width), dtype=torch.float32, device="cuda:0")
              for c in cams]
    px = sum(c.width * c.height for c in cams)

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
        return float(np.median(t))

    def singles():
        for c, im in zip(cams, images):
            B.render(parts, c, pal, sp, im, **kw)

    # one checked batch first: a view whose pairs exceed the capacity raises
    _, st = B.render_batch(parts, cams, pal, sp, images, stats=True, streams=4, **kw)
    log(f"batch: most pairs in a view {max(v['n_pairs'] for v in st)}, "
        f"chunks {max(v['n_chunks'] for v in st)}")
    reps = max(3, args.steps)
    ms_single = timed(singles, reps)
    ms_batch = timed(lambda: B.render_batch(parts, cams, pal, sp, images, **kw), reps)
    B.graph_cache_clear()
    ms_graph = timed(lambda: B.render_batch(parts, cams, pal, sp, images, graph=True, **kw), reps)
    B.graph_cache_clear()
    ms_batch4 = timed(lambda: B.render_batch(parts, cams, pal, sp, images, streams=4, **kw), reps)
    ms_graph4 = timed(lambda: B.render_batch(parts, cams, pal, sp, images, graph=True, streams=4,
                                             **kw), reps)
    B.graph_cache_clear()
    # one persistent splat launch per group of four views
    ms_pers4 = timed(lambda: B.render_batch(parts, cams, pal, sp, images, streams=4,
                                            persistent=True, **kw), reps)
    ms_pgraph4 = timed(lambda: B.render_batch(parts, cams, pal, sp, images, graph=True,
                                              streams=4, persistent=True, **kw), reps)
    B.graph_cache_clear()
    best = min(ms_graph, ms_batch4, ms_graph4, ms_batch, ms_pers4, ms_pgraph4)
    out = {
        "metric": METRIC,
        "value": round(len(cams) / (best * 1e-3), 2),
        "unit": "views/s (fastest batch mode)",
        "higher_is_better": True,
        "n_gpus": 1,
        "dtype": "f32",
        "data": "synthetic",
        "config": dict(workload=name, n_particles=n, views=len(cams),
                       sizes=sizes, pixels_per_batch=px, tile=tuned["tile"],
                       seg_records=tuned["seg_records"], compensated=True),
        "ms_per_batch_single_calls": round(ms_single, 3),
        "ms_per_batch_eager": round(ms_batch, 3),
        "ms_per_batch_graph": round(ms_graph, 3),
        "ms_per_batch_eager_4_streams": round(ms_batch4, 3),
        "ms_per_batch_graph_4_streams": round(ms_graph4, 3),
        "ms_per_batch_persistent_4_streams": round(ms_pers4, 3),
        "ms_per_batch_persistent_graph_4_streams": round(ms_pgraph4, 3),
        "speedup_best_vs_single_calls": round(ms_single / best, 3),
        "mparticle_views_per_s": round(n * len(cams) / (best * 1e-3) / 1e6, 1),
        "autotune_table": tuned["table"],
    }
    print(json.dumps(out), flush=True)


def learned_leg(args, np, torch):
    """Learned decimation against the plain render: particle sets of the
    Plummer-mix generator (20M particles each), square images of --size px
    from cameras on a seeded orbit.  The network trains on pairs the
    renderer makes on the fly (--train-pairs views, 4 per step) from
    --train-sets particle sets, each with its own generator and decimation
    seed (every pair turned by a random multiple of 90 degrees and mirrored
    at random: the render of a turned view is the turned render), and is
    evaluated on --test-views held-out views of one of those sets (seen)
    and of a set whose seeds training never saw (unseen):
    tone-mapped PSNR, max error, fallback rate at 40 dB, and frame times of
    the learned path (decimated render + network + probe) and of the full
    render."""
    from paper_1004_1302_amd import binding as B
    from paper_1004_1302_amd import learned as LN
    from paper_1004_1302_amd import synth
    n = int(args.n or 20_000_000)
    t0 = time.perf_counter()

    def particle_set(seed):
        sc = synth.plummer_mix(n, seed=seed)
        parts, pal = B.scene_to_device(sc, "cuda:0")
        return parts, LN.decimate(parts, seed=seed + 1), pal, sc.species_params

    seeds = [5 + 10 * k for k in range(args.train_sets)]
    unseen_seed = 1001
    train_sets = [particle_set(sd) for sd in seeds]
    unseen = particle_set(unseen_seed)
    pal, sp = train_sets[0][2], train_sets[0][3]
    size = args.size
    cams = synth.orbit_cameras(args.train_pairs + 2 * args.test_views, 9, [(size, size)])
    train = cams[:args.train_pairs]
    test_seen = cams[args.train_pairs:args.train_pairs + args.test_views]
    test_unseen = cams[args.train_pairs + args.test_views:]
    log(f"learned: {len(seeds) + 1} sets of {n} particles ({int(unseen[1]['x'].numel())} decimated) in "
        f"{time.perf_counter() - t0:.1f} s")
    net = LN.UNet(seed=0)
    rec = LN.Reconstructor(net)
    kw = dict(compensated=True)
    t1 = time.perf_counter()
    batch = 4
    steps = max(1, len(train) // batch)
    aug = np.random.default_rng(17)

    def turned(img, k, flip):
        img = torch.rot90(img, k, dims=(1, 2))
        return (torch.flip(img, dims=(2,)) if flip else img).contiguous()

    for it in range(steps):
        parts, dec = train_sets[it % len(train_sets)][:2]
        views = train[it * batch:(it + 1) * batch]
        d = [B.render(dec, c, pal, sp, **kw) for c in views]
        f = [B.render(parts, c, pal, sp, **kw) for c in views]
        ks, fl = aug.integers(0, 4, len(views)), aug.integers(0, 2, len(views))
        d = [turned(x, int(k), int(m)) for x, k, m in zip(d, ks, fl)]
        f = [turned(x, int(k), int(m)) for x, k, m in zip(f, ks, fl)]
        lr = 1e-3 if it < 0.7 * steps else 3e-4
        part = rec.train_step(d, f, lr=lr)
        if it % 50 == 0 or it == steps - 1:
            loss = float(part.sum().item()) / (batch * size * size * 3)
            log(f"train step {it + 1}/{steps} loss {loss:.3e}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1

    from scipy.ndimage import gaussian_filter
    blur_sigmas = (0.5, 1.0, 2.0)

    def evaluate(pset, views):
        parts, dec = pset[:2]
        psnr_net, psnr_dec, maxerr, fb = [], [], [], 0
        lin_net, lin_dec = [], []
        psnr_blur = {sg: [] for sg in blur_sigmas}
        ev = lambda: torch.cuda.Event(enable_timing=True)
        t_learn, t_full = [], []
        for c in views:
            e0, e1, e2 = ev(), ev(), ev()
            e0.record()
            full = B.render(parts, c, pal, sp, **kw)
            e1.record()
            img, info = LN.render_learned(parts, dec, c, pal, sp, rec, threshold_db=40.0, **kw)
            e2.record()
            torch.cuda.synchronize()
            t_full.append(e0.elapsed_time(e1))
            t_learn.append(e1.elapsed_time(e2))
            d = B.render(dec, c, pal, sp, **kw)
            out = rec.infer(d)
            torch.cuda.synchronize()
            fh, oh, dh = full.cpu().numpy(), out.cpu().numpy(), d.cpu().numpy()
            psnr_net.append(LN.psnr_tonemapped(oh, fh))
            psnr_dec.append(LN.psnr_tonemapped(dh, fh))
            lin_net.append(LN.psnr_linear(oh, fh))
            lin_dec.append(LN.psnr_linear(dh, fh))
            # a non-learned baseline: the decimated render blurred by a
            # Gaussian of sigma px
            for sg in blur_sigmas:
                psnr_blur[sg].append(LN.psnr_tonemapped(gaussian_filter(dh, (0, sg, sg)), fh))
            maxerr.append(float(np.abs(oh - fh).max() / max(np.abs(fh).max(), 1e-30)))
            fb += int(info["fallback"])
        med = lambda a: float(np.median(a))
        return {
            "psnr_net_median_db": round(med(psnr_net), 3),
            "psnr_decimated_median_db": round(med(psnr_dec), 3),
            "psnr_gain_median_db": round(med(np.array(psnr_net) - np.array(psnr_dec)), 3),
            "psnr_blurred_decimated_median_db": {str(sg): round(med(v), 3)
                                                 for sg, v in psnr_blur.items()},
            "psnr_gain_over_best_blur_median_db": round(
                med(np.array(psnr_net) - np.max([psnr_blur[sg] for sg in blur_sigmas], axis=0)),
                3),
            "psnr_linear_net_median_db": round(med(lin_net), 3),
            "psnr_linear_decimated_median_db": round(med(lin_dec), 3),
            "max_rel_error_median": round(med(maxerr), 5),
            "fallback_rate_at_40db": fb / len(views),
            "ms_full_render_median": round(med(t_full), 3),
            "ms_learned_path_median": round(med(t_learn), 3),
        }

    seen = evaluate(train_sets[0], test_seen)
    new = evaluate(unseen, test_unseen)
    out = {
        "metric": METRIC,
        "value": new["psnr_net_median_db"],
        "unit": "dB (tone-mapped PSNR of the learned reconstruction vs the full render, "
                "particle set unseen in training)",
        "higher_is_better": True,
        "n_gpus": 1,
        "dtype": "bf16 network, f32 render",
        "data": "synthetic",
        "config": dict(workload="learned_decimation", n_particles=n, decimation=LN.DECIMATE,
                       width=size, height=size, train_pairs=len(train),
                       train_sets=f"generator seeds {seeds} (decimation seed + 1), views "
                                  "turned by multiples of 90 degrees and mirrored at random",
                       test_views=len(test_unseen),
                       unseen_set=f"generator seed {unseen_seed} (decimation seed + 1)",
                       params=net.n_params(), levels=list(LN.LEVELS)),
        "unseen_set": new,
        "seen_set_new_views": seen,
        "train_seconds": round(train_s, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
