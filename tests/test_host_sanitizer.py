"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

abi.cpp and schedule.cpp (the orchestration: job tables, staging, the schedule check, the
host model of the task graph) are compiled with both sanitizers on their host side, linked
with the library's kernel objects as built, and a driver (tests/sanitize/host_entry_points.cpp)
calls every host-only entry point over a grid of shapes (empty, ragged and invalid ones too).
No GPU is touched.  Skipped when the kernel objects or hipcc are not there."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_00136_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def test_host_entry_points_under_sanitizers(tmp_path):
    kernels = [p for p in glob.glob(os.path.join(BUILD, "*.hip.o"))]
    if not kernels or not os.path.exists(HIPCC) or not os.path.exists(CLANG) or shutil.which("ldd") is None:
        pytest.skip("kernel objects (python -m paper_2505_00136_amd.build) or the toolchain missing")
    objs = []
    for src in [os.path.join(CSRC, "abi.cpp"), os.path.join(CSRC, "schedule.cpp"),
                os.path.join(ROOT, "tests", "sanitize", "host_entry_points.cpp")]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        cmd = [HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature",
               "-Xclang", "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC] + SAN + \
              ["-c", src, "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "host_entry_points")
    # the host-side link (no device code is compiled here): the sanitizer runtimes and HIP's
    link = [CLANG, "-fsanitize=address,undefined", "-o", exe] + objs + kernels + \
           ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-lpthread"]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 failure(s)" in r.stdout
