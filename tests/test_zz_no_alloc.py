"""hcc_sort_static, the sort that allocates nothing (its workspace is a fixed device array of the
library): through the C ABI its permutation and sorted keys equal hcc_sort's bit for bit, on
two calls in a row where the second is smaller (the array keeps the first call's contents, so
whatever must start at zero has to be cleared by the call), for 32- and 64-bit keys, up to the
largest size it accepts; larger sizes are refused."""
import ctypes as C

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H():
    assert torch.cuda.is_available()
    import paper_2305_16652_amd as H
    return H


def _keys(n: int, key_bits: int, seed: int, skew: bool) -> np.ndarray:
    k = W.u64_hash(seed, 0, np.arange(n, dtype=np.uint64))
    if skew:   # few distinct values in long runs, like the reordering keys of coherent rays
        k = k >> np.uint64(58)
        k = np.repeat(k[: (n + 15) // 16], 16)[:n]
    k &= np.uint64((1 << key_bits) - 1) if key_bits < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    return k.astype(np.uint32) if key_bits <= 32 else k


def _reference(H, keys_d, key_bits):
    """hcc_sort with its own workspace (the existing entry point)."""
    n = keys_d.shape[0]
    perm = torch.empty(n, dtype=torch.int32, device="cuda")
    sk = torch.empty_like(keys_d)
    ws = torch.empty(max(H.sort_workspace_bytes(n, key_bits), 256), dtype=torch.uint8, device="cuda")
    assert H.lib.hcc_sort(keys_d.data_ptr(), key_bits, n, perm.data_ptr(), sk.data_ptr(), ws.data_ptr(),
                          ws.numel(), None) == 0
    return perm, sk


def _static(H, keys_d, key_bits, with_keys=True):
    n = keys_d.shape[0]
    perm = torch.full((n,), -1, dtype=torch.int32, device="cuda")
    sk = torch.zeros_like(keys_d) if with_keys else None
    st = H.lib.hcc_sort_static(keys_d.data_ptr(), key_bits, n, perm.data_ptr(),
                               sk.data_ptr() if sk is not None else None, None)
    assert st == 0, H.lib.hcc_last_error().decode()
    return perm, sk


@pytest.mark.parametrize("key_bits,n1,n2,skew", [
    (32, 1 << 20, 70_001, False),          # the largest accepted size, then a ragged smaller one
    (32, 1_000_003, 4_097, True),
    (64, 1 << 20, 123_457, False),
    (64, 500_000, 1, True),
    (20, 300_000, 299_999, False),
    (7, 65_536, 65_535, True),
])
def test_static_sort_equals_sort_on_two_calls(H, key_bits, n1, n2, skew):
    for call, n in enumerate((n1, n2)):
        k = _keys(n, key_bits, seed=31 + call + key_bits, skew=skew)
        kd = torch.from_numpy(k.view(np.int32) if key_bits <= 32 else k.view(np.int64)).cuda()
        p_ref, sk_ref = _reference(H, kd, key_bits)
        p, sk = _static(H, kd, key_bits, with_keys=(call == 0))
        torch.cuda.synchronize()
        assert torch.equal(p, p_ref), f"call {call}: permutation differs from hcc_sort (n={n})"
        if sk is not None:
            assert torch.equal(sk, sk_ref), f"call {call}: sorted keys differ from hcc_sort (n={n})"
        # the permutation sorts the keys stably (independent of hcc_sort)
        order = np.argsort(k, kind="stable")
        assert np.array_equal(p.cpu().numpy().astype(np.int64), order), f"call {call}: not the stable order"


def test_static_sort_limits(H):
    b = C.c_size_t()
    assert H.lib.hcc_sort_static_bytes(C.byref(b)) == 0
    assert b.value >= (1 << 20) * 20 and b.value < (64 << 20)
    kd = torch.zeros(16, dtype=torch.int32, device="cuda")
    perm = torch.empty(16, dtype=torch.int32, device="cuda")
    big = H.SORT_STATIC_MAX_KEYS + 1
    assert H.lib.hcc_sort_static(kd.data_ptr(), 32, big, perm.data_ptr(), None, None) == 1
    assert "HCC_SORT_STATIC_MAX_KEYS" in H.lib.hcc_last_error().decode()
    assert H.lib.hcc_sort_static(kd.data_ptr(), 0, 16, perm.data_ptr(), None, None) == 1
    assert H.lib.hcc_sort_static(None, 32, 16, perm.data_ptr(), None, None) == 1
    assert H.lib.hcc_sort_static(kd.data_ptr(), 32, 0, None, None, None) == 0
