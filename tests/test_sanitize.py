"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code, on
the CPU: the oracle (every entry point, degenerate inputs included) and the
library's host runtime (argument checks, workspace layout, the Morton sort of
strips into culling bins, the view queue and orders), each driven by a small
program under tests/sanitize/.  Device code is built as usual and never runs
here; the sanitizers instrument host code only."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_19641_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r.stdout


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not installed")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    # plain C build of the oracle with the sanitizers (host compiler, no HIP)
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(SAN, "oracle_main.c"), "-lm", "-o", exe]
    subprocess.run(cmd, check=True, timeout=300)
    assert "oracle sanitize driver ok" in _run(exe)


HIPCC = "/opt/rocm/bin/hipcc"


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_runtime_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "runtime_asan")
    srcs = [os.path.join(CSRC, f) for f in ("gp_runtime.hip", "gp_kernels.hip", "gp_raster.hip", "gp_chip.hip",
                                            "gp_raycast.hip")]
    # the sanitizers go to the host pass only (each -fsanitize right after -Xarch_host)
    cmd = [HIPCC, "--offload-arch=gfx950", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Wno-unused-command-line-argument",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           *srcs, os.path.join(SAN, "runtime_main.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, timeout=900, capture_output=True)
    assert "runtime sanitize driver ok" in _run(exe)
