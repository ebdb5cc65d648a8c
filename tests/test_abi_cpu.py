"""C ABI checks that need no GPU: the library loads, exports every declared entry point,
and rejects bad arguments before touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hcc.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hcc_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def H():
    import paper_2305_16652_amd as H
    return H


def test_header_declares_the_five_verbs():
    names = _declared()
    for verb in ("hcc_build_bvh", "hcc_select_cut", "hcc_encode", "hcc_sort", "hcc_trace"):
        assert verb in names


def test_library_exports_every_declared_symbol(H):
    for name in _declared():
        assert hasattr(H.lib, name), name


def test_validation_without_device(H):
    lib = H.lib
    bad = C.c_void_p(0)
    b = C.c_size_t()
    assert lib.hcc_sort_workspace(1 << 30, 32, C.byref(b)) == 1
    assert lib.hcc_sort_workspace(10, 0, C.byref(b)) == 1
    assert lib.hcc_sort_workspace(10, 65, C.byref(b)) == 1
    assert lib.hcc_sort_workspace(10, 32, C.byref(b)) == 0 and b.value > 0
    assert lib.hcc_encode(bad, bad, 1, 32, None, 10, None, None) == 1
    assert "invalid" in lib.hcc_last_error().decode()
    assert lib.hcc_trace(bad, None, None, 10, 0, None, None, None) == 1
    assert lib.hcc_build_bvh(None, 10, None, C.byref(C.c_void_p())) == 1
    assert lib.hcc_build_bvh(C.c_void_p(16), 0, None, C.byref(C.c_void_p())) == 1
    assert lib.hcc_select_cut(bad, 8, 0.125, None, C.byref(C.c_void_p())) == 1
    assert lib.hcc_sort(None, 32, 0, None, None, None, 0, None) == 0          # n = 0: nothing to do
    assert lib.hcc_sort(None, 33, 10, None, None, None, 0, None) == 1
    # the no-allocation sort refuses bad sizes before touching the device
    assert lib.hcc_sort_static(None, 32, 0, None, None, None) == 0     # n = 0: nothing to do
    assert lib.hcc_sort_static(C.c_void_p(16), 32, (1 << 20) + 1, C.c_void_p(16), None, None) == 1
    assert lib.hcc_sort_static(C.c_void_p(16), 0, 10, C.c_void_p(16), None, None) == 1
    assert lib.hcc_sort_static_bytes(C.byref(b)) == 0 and b.value >= H.sort_workspace_bytes(1 << 20, 64)
    lib.hcc_bvh_destroy(bad)      # ignored
    lib.hcc_cut_destroy(bad)


def test_sort_workspace_grows_with_n_and_bits(H):
    assert H.sort_workspace_bytes(1 << 20, 64) > H.sort_workspace_bytes(1 << 20, 32) > \
        H.sort_workspace_bytes(1 << 10, 32)


def test_set_allocator_validation(H):
    """Both hooks or neither; a Python pair can be installed and removed without a device."""
    keep = H.ALLOC_FN(lambda n, s, c: None)
    assert H.lib.hcc_set_allocator(C.cast(keep, C.c_void_p), None, None) == 1
    assert H.lib.hcc_set_allocator(None, None, None) == 0
    with pytest.raises(ValueError):
        H.set_allocator(alloc=lambda n, s: 0)
    H.set_allocator(lambda n, s: 0, lambda p, s: None)
    H.set_allocator()


def test_entry_points_open_roctx_ranges(H):
    """The library imports ROCm's roctx range calls (rocprofv3 --marker-trace shows each entry
    point's host call) and its entry points still run their argument checks without a device."""
    import subprocess
    out = subprocess.run(["nm", "-D", H.LIB_PATH], capture_output=True, text=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
    assert H.lib.hcc_encode(C.c_void_p(0), C.c_void_p(0), 1, 32, None, 10, None, None) == 1
