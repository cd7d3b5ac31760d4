"""The partition builder of the C ABI under host AddressSanitizer (CPU only).

tests/asan_partition_walk.cpp calls dd_partition and every partition query on
14 layouts, into output arrays of exactly the documented sizes.  The library's
host source is rebuilt with -fsanitize=address for the host pass (device code
is built as usual and never launched) and linked with the device objects that
build() left in _build/.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"
DEVICE_OBJS = ["ie.o", "rs.o", "pcg.o", "mlp.o", "fft.o"]


@pytest.mark.slow
def test_partition_walk_is_clean_under_address_sanitizer(tmp_path):
    objdir = os.path.join(ROOT, "_build")
    if not os.path.exists(HIPCC) or not all(os.path.exists(os.path.join(objdir, o)) for o in DEVICE_OBJS):
        pytest.skip("needs hipcc and the objects of a previous build()")
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I" + os.path.join(ROOT, "include")]
    asan = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]
    srcs = [(os.path.join(ROOT, "paper_2108_12574_amd", "csrc", "host.cpp"), "host.o"),
            (os.path.join(ROOT, "tests", "asan_partition_walk.cpp"), "walk.o")]
    for src, obj in srcs:
        r = subprocess.run([HIPCC, "-x", "hip", "-c", src, "-o", str(tmp_path / obj)] + flags + asan,
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
    exe = str(tmp_path / "walk")
    objs = [str(tmp_path / o) for _, o in srcs] + [os.path.join(objdir, o) for o in DEVICE_OBJS]
    r = subprocess.run([HIPCC, "--offload-arch=gfx950"] + objs + ["-o", exe, "-Xarch_host", "-fsanitize=address"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "asan partition walk ok" in r.stdout
    assert "rc " not in r.stdout, r.stdout
