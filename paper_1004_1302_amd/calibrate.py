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
    for _ in range(args.repeats):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4,
                      "repeats": args.repeats}), flush=True)


if __name__ == "__main__":
    main()
