"""GPU parity of BalancedShuffle (Section 2; MS_CFG_PLACEMENT_BALANCED):
every merge interleaves its halves by the side labels Algorithm 2 leaves on
0^n1 1^n2, so the permutation and the bit count must equal the oracle's
BalancedShuffle merge at every size, cutoff and element size, and in batched
calls."""
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1508_03167_amd as M

    M.lib()
    return M


def _want(n, B, seed):
    p = np.arange(n, dtype=np.uint32)
    bits = O.shuffle_u32(p, B, seed, O.BALANCED)
    return p, bits


@pytest.mark.parametrize("n,B,seed", [(5, 1, 3), (17, 2, 4), (100, 3, 5), (1000, 7, 6), (4097, 4096, 7),
                                      (8193, 4096, 8), (70001, 4096, 9), (123457, 100, 10), (300007, 4096, 11),
                                      (1 << 18, 1000, 12), ((1 << 20) + 12345, 4096, 13), (40000, 16, 14),
                                      ((1 << 22) + 77, 4096, 15)])
def test_permutation_equals_the_oracle(M, n, B, seed):
    import torch

    print(f"[gpu] balanced n={n} B={B} seed={seed}", flush=True)
    sys.stdout.flush()
    want, wbits = _want(n, B, seed)
    x = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(x, seed, bits=bits, leaf_B=B, placement="BAL")
    torch.cuda.synchronize()
    assert M.device_status() == 0
    assert np.array_equal(x.cpu().numpy().view(np.uint32), want)
    assert int(bits.item()) == wbits


def test_bench_size_balanced(M):
    # the size and seed bench.py times BalancedShuffle at
    import torch

    n, seed = 1 << 26, 7
    print(f"[gpu] balanced n={n} seed={seed}", flush=True)
    want = np.arange(n, dtype=np.uint32)
    wbits = O.shuffle_u32(want, 4096, seed, O.BALANCED, threads=O.max_threads())
    x = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(x, seed, bits=bits, placement="BAL")
    torch.cuda.synchronize()
    assert M.device_status() == 0
    assert np.array_equal(x.cpu().numpy().view(np.uint32), want)
    assert int(bits.item()) == wbits


@pytest.mark.parametrize("eb", [8, 16])
def test_records_move_with_the_permutation(M, eb):
    import torch

    n = 123457
    print(f"[gpu] balanced records eb={eb}", flush=True)
    host = np.random.default_rng(eb).integers(0, 2**62, size=(n, eb // 8), dtype=np.int64)
    x = torch.from_numpy(host.copy()).cuda()
    M.shuffle_(x, 21, placement="BAL")
    torch.cuda.synchronize()
    want, _ = _want(n, 4096, 21)
    assert np.array_equal(x.cpu().numpy(), host[want.astype(np.int64)])


def test_batched_balanced(M):
    import torch

    sizes = [3, 5000, 70001, (1 << 21) + 5, 9000]
    print("[gpu] balanced batched", flush=True)
    dev = [torch.arange(n, dtype=torch.int32, device="cuda") for n in sizes]
    from paper_1508_03167_amd._lib import MS_CFG_PLACEMENT_BALANCED

    with M.BatchGraph(dev, [40 + a for a in range(len(sizes))],
                      cfgs=[M.config(flags=MS_CFG_PLACEMENT_BALANCED)] * len(sizes)) as g:
        g.launch()
        assert g.status() == 0
    for a, n in enumerate(sizes):
        want, _ = _want(n, 4096, 40 + a)
        assert np.array_equal(dev[a].cpu().numpy().view(np.uint32), want), (a, n)
