"""GPU parity at the benchmark sizes, in the launch configuration bench.py times.

The oracle's results at these sizes are stored in tests/golden/configs.json
(written by tests/golden/make_golden.py from the oracle alone): the random-bit
count, two order-sensitive fingerprints of the whole permutation and 512
sampled slots.  The GPU side computes the same fingerprints on the device.
The benchmark workload itself (n = 2^30, seed 7) is also compared element by
element with the oracle run on the host.
"""
import json
import os
import sys

import numpy as np
import pytest

import hashing

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden(name):
    return json.load(open(os.path.join(HERE, "golden", "configs.json")))[name]


@pytest.fixture(scope="module")
def M():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    import paper_1508_03167_amd as M

    M.lib()
    return M


def test_permutation_n2p30_seed7(M):
    import torch

    g = _golden("perm_n2^30_seed7")
    print(f"[gpu] full-size permutation n={g['n']} seed={g['seed']}", flush=True)
    out = torch.empty(g["n"], dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, g["seed"], bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    assert int(bits.item()) == g["bits"]
    pos = torch.tensor([p for p, _ in g["samples"]], dtype=torch.int64, device="cuda")
    got = (out[pos].to(torch.int64) & 0xFFFFFFFF).cpu().numpy()
    assert got.tolist() == [v for _, v in g["samples"]]
    assert list(hashing.fingerprint_torch(out)) == g["fingerprint"]
    # shuffling the identity in place gives the same array
    x = torch.arange(g["n"], dtype=torch.int32, device="cuda")
    M.shuffle_(x, g["seed"])
    assert torch.equal(x, out)
    del out, x
    M.release()
    torch.cuda.empty_cache()


def test_permutation_n2p30_seed7_every_element(M):
    # the benchmark workload compared element by element with the oracle run
    # on the host's cores (about 20 s at 16 threads)
    import torch

    from oracle import oracle as O

    n, seed = 1 << 30, 7
    print(f"[gpu] full-size permutation n={n} seed={seed}, every element", flush=True)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, seed, bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    got = out.cpu().numpy().view(np.uint32)
    del out
    M.release()
    torch.cuda.empty_cache()
    want, want_bits = O.permutation(n, 4096, seed, threads=O.max_threads())
    assert int(bits.item()) == want_bits
    assert np.array_equal(got, want)


def test_ragged_n_near_2p30_every_element(M):
    # n = 2^30 - 12345: leaves of 4095 and 4096 elements, every merge and
    # tile of the fused passes ragged
    import torch

    from oracle import oracle as O

    n, seed = (1 << 30) - 12345, 21
    print(f"[gpu] ragged permutation n={n} seed={seed}, every element", flush=True)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, seed, bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    got = out.cpu().numpy().view(np.uint32)
    del out
    M.release()
    torch.cuda.empty_cache()
    want, want_bits = O.permutation(n, 4096, seed, threads=O.max_threads())
    assert int(bits.item()) == want_bits
    assert np.array_equal(got, want)


def test_records8_n2p28_every_element(M):
    # 8-byte elements at scale: x[i] = i as uint64, shuffled in place, equals
    # the oracle's permutation of 0..n-1
    import torch

    from oracle import oracle as O

    n, seed = (1 << 28) + 7, 13
    print(f"[gpu] 8-byte shuffle n={n} seed={seed}, every element", flush=True)
    x = torch.arange(n, dtype=torch.int64, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.shuffle_(x, seed, bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    got = x.cpu().numpy()
    del x
    M.release()
    torch.cuda.empty_cache()
    want, want_bits = O.permutation(n, 4096, seed, threads=O.max_threads())
    assert int(bits.item()) == want_bits
    assert np.array_equal(got, want.astype(np.int64))


def test_permutation_largest_accepted_size(M):
    # n = 2^32 - 2^16, the largest n the library accepts: slot indices use all
    # 32 bits, the top merge spans the whole array
    import torch

    g = _golden("perm_n2^32-2^16_seed5")
    n = g["n"]
    print(f"[gpu] largest-size permutation n={n} seed={g['seed']}", flush=True)
    out = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, g["seed"], bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    assert int(bits.item()) == g["bits"]
    pos = torch.tensor([p for p, _ in g["samples"]], dtype=torch.int64, device="cuda")
    got = (out[pos].to(torch.int64) & 0xFFFFFFFF).cpu().numpy()
    assert got.tolist() == [v for _, v in g["samples"]]
    assert list(hashing.fingerprint_torch(out)) == g["fingerprint"]
    # a permutation of 0..n-1: the sums of the values and of their squares
    # (modulo 2^64) are those of the identity
    s1 = s2 = 0
    for a in range(0, n, 1 << 26):
        v = out[a:a + (1 << 26)].to(torch.int64) & 0xFFFFFFFF
        s1 += int(v.sum().item())
        s2 = (s2 + int((v * v).sum().item())) % (1 << 64)
    assert s1 == n * (n - 1) // 2
    assert s2 == ((n - 1) * n * (2 * n - 1) // 6) % (1 << 64)
    del out
    M.release()
    torch.cuda.empty_cache()


def test_records16_n2p27_seed11(M):
    import torch

    from paper_1508_03167_amd.inputs import records16

    g = _golden("perm_n2^27_seed11")
    print(f"[gpu] full-size records n={g['n']} seed={g['seed']}", flush=True)
    host = records16(g["n"], g["seed"])
    rec = torch.from_numpy(host.view(np.int64)).cuda()
    keys0 = rec[:, 0].clone()
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.shuffle_(rec, g["seed"], bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    assert int(bits.item()) == g["bits"]
    payload = rec[:, 1]
    assert list(hashing.fingerprint_torch(payload)) == g["fingerprint"]
    pos = torch.tensor([p for p, _ in g["samples"]], dtype=torch.int64, device="cuda")
    assert payload[pos].cpu().numpy().tolist() == [v for _, v in g["samples"]]
    assert torch.equal(rec[:, 0], keys0[payload])
    # every record: the payloads are the oracle's permutation of 0..n-1
    from oracle import oracle as O

    want, _ = O.permutation(g["n"], 4096, g["seed"], threads=O.max_threads())
    assert np.array_equal(payload.cpu().numpy(), want.astype(np.int64))
    del rec, keys0, payload
    M.release()
    torch.cuda.empty_cache()
