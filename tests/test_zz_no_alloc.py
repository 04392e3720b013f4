"""The allocation-free entry point against ms_shuffle_ex, through the C ABI.

ms_shuffle_noalloc keeps its scratch in a fixed device array that every call
on the device shares; two calls in a row (the second smaller, so it runs over
what the first left in the array) must each give exactly what ms_shuffle_ex
gives for the same arguments, bits included, and oversize calls are refused
before anything is launched.
"""
import ctypes
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1508_03167_amd as M

    M.lib()
    return M


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _call(M, fn, x, seed):
    import torch

    L = M.lib()
    bits = torch.zeros(1, dtype=torch.int64, device=x.device)
    eb = x.element_size() * (x[0].numel() if x.dim() > 1 else 1)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    rc = getattr(L, fn)(ctypes.c_void_p(x.data_ptr()), x.shape[0], eb, seed, stream, None,
                        ctypes.c_void_p(bits.data_ptr()))
    assert rc == 0, (fn, rc, L.ms_last_error())
    torch.cuda.synchronize()
    assert M.device_status() == 0
    return int(bits.item())


@pytest.mark.parametrize("eb,sizes", [(4, (3_000_017, 70_001)), (8, (1_500_007, 9_001)),
                                      (16, (600_011, 8_193))])
def test_noalloc_equals_shuffle_ex_twice(M, eb, sizes):
    import torch

    for n, seed in zip(sizes, (12345, 678)):
        _say(f"[gpu] noalloc eb={eb} n={n} seed={seed}")
        rng = np.random.default_rng(n)
        vals = rng.integers(0, 2**62, size=(n, eb // 4), dtype=np.int64).astype(np.int32)
        a = torch.from_numpy(vals.copy()).cuda()
        b = a.clone()
        ba = _call(M, "ms_shuffle_ex", a, seed)
        bb = _call(M, "ms_shuffle_noalloc", b, seed)
        assert torch.equal(a, b), f"first mismatch at row {int((a != b).any(dim=1).nonzero()[0])}"
        assert ba == bb


def test_noalloc_refuses_oversize_calls(M):
    import torch

    L = M.lib()
    n = 1 << 24  # 64 MiB of uint32 plus the plan: above the fixed scratch
    x = torch.arange(n, dtype=torch.int32, device="cuda")
    rc = L.ms_shuffle_noalloc(ctypes.c_void_p(x.data_ptr()), n, 4, 1,
                              ctypes.c_void_p(torch.cuda.current_stream().cuda_stream), None, None)
    assert rc == M._lib.MS_ERR_UNSUPPORTED
    torch.cuda.synchronize()
    assert torch.equal(x, torch.arange(n, dtype=torch.int32, device="cuda"))
