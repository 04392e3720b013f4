"""GPU parity of the listing's placement (MS_CFG_PLACEMENT_R1): the printed
Merge listing places the coin-flip loop's elements by in-place swaps (the B
element of a one swaps with the slot; a zero keeps what the slot holds).  The
GPU result must equal the oracle's R1 run element by element, with the same
bit count, which is also the stable-interleave run's count (both readings
consume the same flips and draws)."""
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


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _oracle_r1(n, cutoff, seed):
    a = np.arange(n, dtype=np.uint32)
    bits = O.shuffle_u32(a, cutoff, seed, placement=O.R1, threads=O.max_threads())
    return a, bits


@pytest.mark.parametrize("n", [2, 3, 4097, 8197, 65536 + 123, (1 << 20) + 7777, 3_000_001])
def test_permutation_matches_oracle_r1(M, n):
    import torch

    _say(f"[gpu] r1 permutation n={n}")
    seed = 1000 + n
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, seed, bits=bits, placement="R1")
    torch.cuda.synchronize()
    assert M.device_status() == 0
    want, wbits = _oracle_r1(n, 4096, seed)
    got = out.cpu().numpy().view(np.uint32)
    assert np.array_equal(got, want)
    assert int(bits.item()) == wbits


def test_bench_size_r1(M):
    # the size and seed bench.py times the listing placement at
    import torch

    n, seed = 1 << 26, 7
    _say(f"[gpu] r1 permutation n={n} seed={seed}")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, seed, bits=bits, placement="R1")
    torch.cuda.synchronize()
    assert M.device_status() == 0
    want, wbits = _oracle_r1(n, 4096, seed)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
    assert int(bits.item()) == wbits


def test_same_bits_as_stable_interleave_but_another_permutation(M):
    import torch

    n, seed = (1 << 18) + 99, 5
    a = torch.empty(n, dtype=torch.int32, device="cuda")
    b = torch.empty(n, dtype=torch.int32, device="cuda")
    ba = torch.zeros(1, dtype=torch.int64, device="cuda")
    bb = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(a, seed, bits=ba, placement="R1")
    M.permutation(b, seed, bits=bb)
    torch.cuda.synchronize()
    assert int(ba.item()) == int(bb.item())
    assert not torch.equal(a, b)
    want2, _ = O.permutation(n, 4096, seed)
    assert np.array_equal(b.cpu().numpy().view(np.uint32), want2)


@pytest.mark.parametrize("eb", [8, 16])
def test_records_match_oracle_r1(M, eb):
    import torch

    n, seed = 200_003, 77 + eb
    _say(f"[gpu] r1 records eb={eb}")
    rng = np.random.default_rng(eb)
    host = rng.integers(0, 2**63, size=(n, eb // 8), dtype=np.int64)
    dev = torch.from_numpy(host.copy()).cuda()
    M.shuffle_(dev, seed, placement="R1")
    torch.cuda.synchronize()
    want, _ = _oracle_r1(n, 4096, seed)
    assert np.array_equal(dev.cpu().numpy(), host[want.astype(np.int64)])


def test_small_cutoff_many_levels(M):
    import torch

    n, seed, cut = 50_000, 9, 16
    _say("[gpu] r1 cutoff 16")
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, seed, bits=bits, leaf_B=cut, placement="R1")
    torch.cuda.synchronize()
    want, wbits = _oracle_r1(n, cut, seed)
    assert np.array_equal(out.cpu().numpy().view(np.uint32), want)
    assert int(bits.item()) == wbits


def test_batched_r1_equals_one_call_per_array(M):
    import torch

    sizes = [5000, 70001, 3, 300_000]
    a = [torch.arange(n, dtype=torch.int32, device="cuda") for n in sizes]
    b = [t.clone() for t in a]
    M.shuffle_batched_(a, 31, placement="R1")
    for i, t in enumerate(b):
        M.shuffle_(t, 31 + i, placement="R1")
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)
