"""Build libsplotch.so (HIP, gfx950) in-tree with hipcc."""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsplotch.so")
SOURCES = ["api.hip", "project.hip", "sort.hip", "bin.hip", "splat.hip", "nn.hip", "nn_api.hip", "unet.hip",
           "learned.hip", "stream.hip", "render_static.hip"]
ARCH = os.environ.get("SPLOTCH_OFFLOAD_ARCH", "gfx950")

ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast-honor-pragmas",
    "-Wall", "-Wno-unused-function",
]

# Host-side AddressSanitizer + UndefinedBehaviorSanitizer build of the same
# sources: every -fsanitize= goes to the host pass only (the device code is
# built as usual), and the library leaves the sanitizer runtime's symbols to
# a preloaded libclang_rt.asan.
SAN_DIR = os.path.join(CSRC, "_build", "hsan")
SAN_LIB = os.path.join(SAN_DIR, "libsplotch_hsan.so")
SAN_FLAGS = [
    "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast-honor-pragmas",
    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
    "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
]


def build(verbose: bool = False) -> str:
    """Compile every HIP source and link the shared library (always
    recompiles: this is the build check)."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objs = []
    procs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, "_build", src.replace(".hip", ".o"))
        os.makedirs(os.path.dirname(obj), exist_ok=True)
        cmd = [hipcc, *HIPCC_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        text = out.decode(errors="replace")
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln
                 and "not a recognized feature for this target" not in ln]
        if pr.returncode != 0:
            failed.append(src)
            print("\n".join(lines), file=sys.stderr)
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        raise RuntimeError(f"hipcc failed for {failed}")
    tmp = LIB + ".tmp"
    # trace ranges and markers (roctx) for rocprofv3 --marker-trace
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
           f"-L{ROCM}/lib", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM}/lib"]
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


def _sources_digest(flags) -> str:
    h = hashlib.sha256(" ".join(flags).encode())
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")):
            h.update(name.encode())
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(f.read())
    with open(os.path.join(os.path.dirname(HERE), "include", "splotch.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()


def build_host_sanitized() -> str:
    """Build libsplotch_hsan.so (host code under ASan + UBSan) unless the one
    on disk was built from the same sources and flags; returns its path.
    Load it only with the sanitizer runtime preloaded."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    stamp = os.path.join(SAN_DIR, "sources.sha256")
    digest = _sources_digest(SAN_FLAGS)
    if os.path.exists(SAN_LIB) and os.path.exists(stamp) and open(stamp).read() == digest:
        return SAN_LIB
    os.makedirs(SAN_DIR, exist_ok=True)
    objs, procs = [], []
    for src in SOURCES:
        obj = os.path.join(SAN_DIR, src.replace(".hip", ".o"))
        cmd = [hipcc, *SAN_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        objs.append(obj)
    failed = []
    for src, pr in procs:
        out, _ = pr.communicate()
        if pr.returncode != 0:
            failed.append(src)
            print(out.decode(errors="replace"), file=sys.stderr)
    if failed:
        raise RuntimeError(f"hipcc (sanitized host build) failed for {failed}")
    tmp = SAN_LIB + ".tmp"
    subprocess.check_call([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs,
                           f"-L{ROCM}/lib", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM}/lib"])
    os.replace(tmp, SAN_LIB)
    with open(stamp, "w") as f:
        f.write(digest)
    return SAN_LIB


if __name__ == "__main__":
    print(build(verbose=True))
