"""CPU tests of the C ABI: the library loads and exports every declared symbol,
and its host-only partition logic matches the oracle's decomposition exactly."""
import os
import re

import numpy as np
import pytest

import paper_2108_12574_amd as cbd
from paper_2108_12574_amd import _lib
from oracle import dd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "cbd.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\*?\s+\**(\w+)\s*\(", src, flags=re.M)))


def test_library_exports_every_declared_symbol():
    L = cbd.lib()
    names = _declared_functions()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    # the binding declares exactly the header's functions
    assert sorted(n for n, _, _ in _lib.SIGNATURES) == names


def test_errors_are_reported_without_gpu():
    L = cbd.lib()
    import ctypes
    h = ctypes.c_void_p()
    assert L.dd_partition(2, 30, 4, 1, cbd.MODE_CBD, 0, ctypes.byref(h)) == _lib.EARG
    assert b"multiple" in L.cbd_last_error()
    assert L.dd_partition(2, 32, 8, 3, cbd.MODE_CBD, 0, ctypes.byref(h)) == _lib.EARG
    assert L.dd_partition(4, 32, 8, 1, cbd.MODE_CBD, 0, ctypes.byref(h)) == _lib.EARG
    with pytest.raises(cbd.CbdError):
        cbd.Partition((2, 30), 4)


def test_every_compute_entry_point_rejects_bad_arguments_on_the_host():
    """Each entry point checks its arguments before any device call, so a
    NULL handle or pointer, a nonpositive count or an unknown option returns
    EARG with a message naming the call, with no GPU present."""
    L = cbd.lib()
    import ctypes
    h = ctypes.c_void_p()
    buf = ctypes.c_void_p(16)  # never dereferenced: each call fails before
    it, rr = ctypes.c_int(), ctypes.c_double()
    opts = _lib.RSOpts()
    cases = [
        ("ie_assemble", lambda: L.ie_assemble(4, 16, 0, None, None, buf, buf, buf, buf, None, ctypes.byref(h))),
        ("ie_assemble", lambda: L.ie_assemble(2, 1, 0, None, None, buf, buf, buf, buf, None, ctypes.byref(h))),
        ("ie_assemble", lambda: L.ie_assemble(2, 16, 0, None, None, None, buf, buf, buf, None, ctypes.byref(h))),
        ("kernel_matvec", lambda: L.kernel_matvec(None, 1, buf, ctypes.c_void_p(32), None)),
        ("kernel_matvec_fft", lambda: L.kernel_matvec_fft(None, 1, buf, ctypes.c_void_p(32), None)),
        ("cbd_fft_prepare", lambda: L.cbd_fft_prepare(None, 1, buf, 1 << 20, None)),
        ("cbd_autotune_matvec", lambda: L.cbd_autotune_matvec(None, 1, buf, ctypes.c_void_p(32), None, None)),
        ("cbd_matvec_set_shape", lambda: L.cbd_matvec_set_shape(None, 1, 4)),
        ("rs_factor_batched", lambda: L.rs_factor_batched(None, None, ctypes.byref(opts), None, buf, 1 << 20,
                                                          None, None, None, ctypes.byref(h))),
        ("rs_factor_workspace", lambda: L.rs_factor_workspace(None, None, ctypes.byref(opts), None, None)),
        ("rs_factor_rank_count", lambda: L.rs_factor_rank_count(None, ctypes.byref(opts), None)),
        ("rs_apply", lambda: L.rs_apply(None, 1, buf, ctypes.c_void_p(32), None)),
        ("rs_apply_sub", lambda: L.rs_apply_sub(None, 0, 1, buf, ctypes.c_void_p(32), None)),
        ("pcg_solve", lambda: L.pcg_solve(None, None, 1, buf, buf, 1e-10, 10, 0, buf, 0,
                                          ctypes.byref(it), ctypes.byref(rr), None)),
        ("rank_mlp_forward", lambda: L.rank_mlp_forward(None, 4, buf, buf, None)),
        ("rank_mlp_adam", lambda: L.rank_mlp_adam(buf, buf, buf, buf, 0, ctypes.c_float(1e-3), None)),
        ("dd_partition_info", lambda: L.dd_partition_info(None, None, None, None, None)),
        ("rs_factor_stats", lambda: L.rs_factor_stats(None, None, None, None, None)),
        ("cbd_timing_get", lambda: L.cbd_timing_get(None, None, None)),
    ]
    for name, call in cases:
        assert call() == _lib.EARG, name
        assert L.cbd_last_error().startswith(name.encode()), (name, L.cbd_last_error())


CASES = [
    (2, 64, 16, 1, dd.CBD, 0),
    (2, 256, 4, 8, dd.SCHWARZ, 8),
    (2, 48, 12, 1, dd.CBD, 0),
    (2, 60, 6, 2, dd.CBD, 4),
    (2, 32, 4, 1, dd.JACOBI, 0),
    (2, 16, 2, 1, dd.CBD, 0),
    (3, 32, 4, 1, dd.CBD, 0),
    (3, 12, 4, 1, dd.SCHWARZ, 3),
    (2, 512, 64, 1, dd.CBD, 0),
]


@pytest.mark.parametrize("d,n,m,delta,mode,leaf", CASES)
def test_partition_matches_oracle(d, n, m, delta, mode, leaf):
    ref = dd.Partition(d, n, m, delta, mode, leaf)
    got = cbd.Partition((d, n), m, delta, mode, leaf)
    assert got.D == ref.D and got.Lt == ref.Lt and got.Lr == ref.Lr
    assert got.total == sum(len(s.index) for s in ref.subdomains)
    for i, sd in enumerate(ref.subdomains):
        idx, nleaves, root = got.subdomain(i)
        assert np.array_equal(np.array(idx), sd.index)
        assert nleaves == len(sd.leaves) and root == sd.root_level
        for l in range(sd.root_level + 1):
            boxes, parent = got.level_boxes(i, l)
            assert len(boxes) == len(sd.levels[l])
            for b, box in enumerate(sd.levels[l]):
                assert boxes[b] == (box.lo, box.hi)
            if l < sd.root_level:
                for c, pb in enumerate(sd.levels[l + 1]):
                    for ch in pb.children:
                        assert parent[ch] == c
            else:
                assert parent == [-1]


def test_header_constants_match_the_binding():
    # every #define CBD_<NAME> <int> of the header equals the binding's <NAME> where it has one
    hdr = open(os.path.join(ROOT, "include", "cbd.h")).read()
    seen = 0
    for name, val in re.findall(r"#define CBD_([A-Z0-9_]+)\s+\(?(-?\d+)\)?", hdr):
        if hasattr(_lib, name):
            assert getattr(_lib, name) == int(val), name
            seen += 1
    assert seen >= 15


@pytest.mark.parametrize("d,n,m,mode,leaf", [(2, 64, 16, cbd.MODE_CBD, 0), (2, 64, 4, cbd.MODE_SCHWARZ, 8),
                                             (3, 16, 4, cbd.MODE_CBD, 0), (2, 32, 1, cbd.MODE_JACOBI, 4)])
def test_rank_count_is_the_number_of_compressed_boxes(d, n, m, mode, leaf):
    # the length of rank_hint / ranks_out: boxes of every level below the highest root,
    # of the subdomains whose root lies above that level
    import ctypes
    part = cbd.Partition((d, n), m, 1, mode, leaf)
    roots = [part.subdomain(i)[2] for i in range(part.D)]
    Lmax = max(roots)
    want = sum(len(part.level_boxes(i, l)[0]) for l in range(Lmax) for i in range(part.D) if roots[i] > l)
    opts = _lib.RSOpts(1e-6, 64, 1.5, 0, 0, None, 0, 0, 0, 0, 0)
    cnt = ctypes.c_int()
    assert cbd.lib().rs_factor_rank_count(part.handle, ctypes.byref(opts), ctypes.byref(cnt)) == 0
    assert cnt.value == want
    opts.exact = 1      # exact subsolves: no compressed level
    assert cbd.lib().rs_factor_rank_count(part.handle, ctypes.byref(opts), ctypes.byref(cnt)) == 0
    assert cnt.value == 0


def test_fft_workspace_size():
    L = cbd.lib()
    # 512^2: P = 1024, kernel transform + twiddles + 3 complex work arrays
    want = 8 * 1024 ** 2 + 16 * 512 + 16 * 1024 ** 2 * 3
    assert L.cbd_fft_workspace_bytes(2, 512, 3) == want
    assert L.cbd_fft_workspace_bytes(4, 512, 3) == 0 and L.cbd_fft_workspace_bytes(2, 512, 0) == 0


def test_bench_refuses_several_gpus():
    """bench.py runs on one GPU: --gpus above 1 exits with status 2 and says why, before
    touching a device."""
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300, cwd=root)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
