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
FP32_VECTOR_PEAK_TFLOPS = 78.6  # non-packed FP32 FMA rate: 256 CU x 64 lanes x 2 x 2.4 GHz
# algorithmic FP32 operations per composited (pixel, particle) contribution
FLOPS_EMISSION = 11   # weight (scale, exp) + per channel E*w, *T, +=
FLOPS_ABSORBING = 29  # weight + per channel E*w, A*w, exp, 1-e, /x, *T*phi (2), +=, T*=


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
    if cfg.get("n_target") != 1_000_000_000 or args.tile != 16 or args.max_pairs:
        return None
    rec = json.load(open(path)).get(kernel)
    if not rec:
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


def cpu_baseline(parts, cam, sp, args, np, torch):
    """The FP64 oracle on a seeded random subsample of the same particles
    (same smoothing lengths, same camera and image size), single thread."""
    import oracle
    from paper_1004_1302_amd import synth
    n = int(parts["x"].numel())
    k = min(n, int(args.cpu_sample))
    gen = torch.Generator(device="cpu")
    gen.manual_seed(17)
    idx = torch.unique(torch.randint(0, n, (k,), generator=gen)).to(parts["x"].device)
    k = int(idx.numel())
    host = {key: t[idx].cpu().numpy() for key, t in parts.items()}
    scene = synth.Scene(host["x"], host["y"], host["z"], host["h"], host["value"], cam, sp,
                        species=host.get("species"), rho0=host.get("rho0"))
    oracle.lib()
    t0 = time.perf_counter()
    oracle.render(scene)
    dt = time.perf_counter() - t0
    return dict(value=round(k / dt / 1e6, 6), unit="Mparticles/s", cores=1, kind="oracle",
                sample=f"seeded random subsample of {k} of {n} particles, same camera and "
                       f"{cam.width}x{cam.height} image, FP64 single thread, {dt:.2f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="lognormal",
                    choices=["lognormal", "nfw", "plummer", "learned", "batch"])
    ap.add_argument("--views", type=int, default=32)
    ap.add_argument("--batch-set", default="nfw", choices=["nfw", "plummer"])
    ap.add_argument("--train-pairs", type=int, default=2000)
    ap.add_argument("--test-views", type=int, default=20)
    ap.add_argument("--size", type=int, default=1024)
    ap.add_argument("--n", type=float, default=0)
    ap.add_argument("--grid", type=int, default=0)
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--splat-variant", type=int, default=0)
    ap.add_argument("--max-pairs", type=float, default=0)
    ap.add_argument("--cpu-sample", type=float, default=5_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    # per-stage breakdown with the library's own HIP events
    stage_runs = []
    for s in range(max(1, min(args.steps, 5))):
        _, st = step(profile=True)
        stage_runs.append(st)
    st = stage_runs[-1]
    stages = {k: float(np.mean([r["stage_ms"][k] for r in stage_runs])) for k in st["stage_ms"]}
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
                    member_pairs=n_mem, member_pairs_absorbing=n_abs)
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
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(parts, cam, sp, args, np, torch)
    print(json.dumps(out), flush=True)


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
    best = min(ms_graph, ms_batch4, ms_graph4, ms_batch)
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
        "mparticle_views_per_s": round(n * len(cams) / (best * 1e-3) / 1e6, 1),
        "autotune_table": tuned["table"],
    }
    print(json.dumps(out), flush=True)


def learned_leg(args, np, torch):
    """Learned decimation against the plain render: 20M particles of the
    Plummer-mix generator, square images of --size px from cameras on a
    seeded orbit; the network trains on pairs the renderer makes on the fly
    (--train-pairs views, 4 per step) and is evaluated on --test-views
    held-out views (tone-mapped PSNR, max error), with frame times of the
    learned path (decimated render + network + probe) and of the full
    render."""
    from paper_1004_1302_amd import binding as B
    from paper_1004_1302_amd import learned as LN
    from paper_1004_1302_amd import synth
    n = int(args.n or 20_000_000)
    t0 = time.perf_counter()
    sc = synth.plummer_mix(n, seed=5)
    parts, pal = B.scene_to_device(sc, "cuda:0")
    dec = LN.decimate(parts, seed=6)
    sp = sc.species_params
    size = args.size
    cams = synth.orbit_cameras(args.train_pairs + args.test_views, 9, [(size, size)])
    train, test = cams[:args.train_pairs], cams[args.train_pairs:]
    log(f"learned: {n} particles ({int(dec['x'].numel())} decimated) in "
        f"{time.perf_counter() - t0:.1f} s")
    net = LN.UNet(seed=0)
    rec = LN.Reconstructor(net)
    kw = dict(compensated=True)
    t1 = time.perf_counter()
    batch = 4
    steps = max(1, len(train) // batch)
    for it in range(steps):
        views = train[it * batch:(it + 1) * batch]
        d = [B.render(dec, c, pal, sp, **kw).clone() for c in views]
        f = [B.render(parts, c, pal, sp, **kw).clone() for c in views]
        lr = 1e-3 if it < 0.7 * steps else 3e-4
        part = rec.train_step(d, f, lr=lr)
        if it % 50 == 0 or it == steps - 1:
            loss = float(part.sum().item()) / (batch * size * size * 3)
            log(f"train step {it + 1}/{steps} loss {loss:.3e}")
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t1
    psnr_net, psnr_dec, maxerr, fb = [], [], [], 0
    ev = lambda: torch.cuda.Event(enable_timing=True)
    t_learn, t_full = [], []
    for c in test:
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
        maxerr.append(float(np.abs(oh - fh).max() / max(np.abs(fh).max(), 1e-30)))
        fb += int(info["fallback"])
    med = lambda a: float(np.median(a))
    out = {
        "metric": METRIC,
        "value": round(med(psnr_net), 3),
        "unit": "dB (tone-mapped PSNR of the learned reconstruction vs the full render)",
        "higher_is_better": True,
        "n_gpus": 1,
        "dtype": "bf16 network, f32 render",
        "data": "synthetic",
        "config": dict(workload="learned_decimation", n_particles=n, decimation=LN.DECIMATE,
                       width=size, height=size, train_pairs=len(train), test_views=len(test),
                       params=net.n_params(), levels=list(LN.LEVELS)),
        "psnr_net_median_db": round(med(psnr_net), 3),
        "psnr_decimated_median_db": round(med(psnr_dec), 3),
        "psnr_gain_median_db": round(med(np.array(psnr_net) - np.array(psnr_dec)), 3),
        "max_rel_error_median": round(med(maxerr), 5),
        "fallback_rate_at_40db": fb / len(test),
        "ms_full_render_median": round(med(t_full), 3),
        "ms_learned_path_median": round(med(t_learn), 3),
        "train_seconds": round(train_s, 1),
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
