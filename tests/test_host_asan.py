"""The library's host code under AddressSanitizer (host only; the GPU code is
built as usual): every source is compiled with ASan on the host side, linked
with a C driver (`host_asan/driver.c`) that calls every entry point of the C
ABI with NULL handles and pointers, and the host-only calls (action checks
with truncated message buffers, the traversal query, the footprint model)
over many argument sets; any out-of-bounds access or use of freed memory in
those paths aborts the driver with an ASan report.  Leak checking is off: the
HIP runtime keeps allocations until exit."""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1810_01609_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang"


def _have_asan():
    return bool(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG) and _have_asan()),
                    reason="hipcc / ROCm clang with the ASan runtime not available")
def test_host_abi_under_asan(tmp_path):
    srcs = [f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp"))]
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-I", os.path.join(ROOT, "include"),
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]

    def comp(f):
        o = str(tmp_path / (f + ".o"))
        r = subprocess.run([HIPCC, "-x", "hip", "-c", os.path.join(CSRC, f), "-o", o] + common,
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return o

    with cf.ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    drv = str(tmp_path / "driver.o")
    r = subprocess.run([CLANG, "-c", os.path.join(HERE, "host_asan", "driver.c"), "-o", drv, "-I",
                        os.path.join(ROOT, "include"), "-g", "-O1", "-fsanitize=address", "-fno-omit-frame-pointer"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    exe = str(tmp_path / "driver")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-o", exe, drv] + objs + ["-Xarch_host", "-fsanitize=address"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
    assert "0 failed" in r.stdout
