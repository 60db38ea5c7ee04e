"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds libsplotch_hsan.so (every -fsanitize= on the host pass only; the
device code is the ordinary build) and runs the host-only ABI checks of
test_abi.py against it in a child process with the ASan runtime preloaded
(an uninstrumented python needs it first in the link order).  Any sanitizer
report aborts the child and fails this test; no GPU is needed.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CLANG = "/opt/rocm/llvm/bin/clang"

RUNNER = r"""
import sys
sys.path.insert(0, sys.argv[1])
from paper_1004_1302_amd import binding as B
B.LIB_PATH = sys.argv[2]
import pytest
sys.exit(pytest.main(["-q", "-x", "-s", "-p", "no:cacheprovider", sys.argv[3]]))
"""


def _asan_runtime():
    if not os.path.exists(CLANG):
        return None
    out = subprocess.run([CLANG, "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True).stdout.strip()
    return out if os.path.isabs(out) and os.path.exists(out) else None


@pytest.mark.timeout(600)
def test_abi_checks_under_host_sanitizers():
    rt = _asan_runtime()
    if rt is None or shutil.which(os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")) is None:
        pytest.skip("hipcc or the clang ASan runtime is not installed")
    from paper_1004_1302_amd import build
    lib = build.build_host_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = " ".join(p for p in (rt, env.get("LD_PRELOAD", "")) if p)
    # leaks: python's own; shadow gap: the HIP runtime maps fixed ranges
    env["ASAN_OPTIONS"] = "detect_leaks=0:protect_shadow_gap=0:abort_on_error=0:exitcode=86"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=87"
    r = subprocess.run([sys.executable, "-c", RUNNER, ROOT, lib, os.path.join(ROOT, "tests", "test_abi.py")],
                       env=env, capture_output=True, text=True, timeout=300)
    report = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, report
    assert "passed" in r.stdout and "runtime error" not in report and "AddressSanitizer" not in report, report
