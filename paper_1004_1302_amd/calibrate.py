"""Plain device-to-device copies of a known size, for calibrating HBM
traffic counters: run under `rocprofv3 --pmc FETCH_SIZE` (then WRITE_SIZE)
and divide the known bytes by what the counter reports for the copy kernel
to get the factor applied to the render kernels' counter readings."""
import argparse
import json


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=2048)
    ap.add_argument("--repeats", type=int, default=3)
    args = ap.parse_args()
    import torch
    n = args.mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)  # first touch
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.repeats + 1)]
    ev[0].record()
    for k in range(args.repeats):
        dst.copy_(src)
        ev[k + 1].record()
    torch.cuda.synchronize()
    ms = [ev[k].elapsed_time(ev[k + 1]) for k in range(args.repeats)]
    best = min(ms)
    # achieved streaming rate (read + write) of a plain device copy: the
    # practical ceiling the HBM-bound passes are compared with
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4,
                      "repeats": args.repeats + 1, "ms": [round(m, 4) for m in ms],
                      "copy_tb_per_s": round(2 * n * 4 / (best * 1e-3) / 1e12, 3)}), flush=True)


if __name__ == "__main__":
    main()
