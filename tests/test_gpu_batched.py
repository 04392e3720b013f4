"""GPU parity of the batched entry point: every array of a batch, whatever its
size, element size or position in the batch, gets exactly the permutation the
oracle gives for (its n, cutoff 4096, seed + its index), and the bits it used.

Small arrays (every merge level inside one leaf workgroup) run together, up to
64 per launch; larger ones take the full path on side streams.
"""
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


def _make(sizes, ebs, seed):
    import torch

    rng = np.random.default_rng(seed)
    host, dev = [], []
    for n, eb in zip(sizes, ebs):
        if eb == 4:
            v = np.arange(n, dtype=np.int32)
            host.append(v)
            dev.append(torch.from_numpy(v.copy()).cuda())
        else:
            v = rng.integers(0, 2**63, size=(n, eb // 8), dtype=np.int64)
            host.append(v)
            dev.append(torch.from_numpy(v.copy()).cuda())
    return host, dev


def _check(M, sizes, ebs, seed):
    import torch

    host, dev = _make(sizes, ebs, seed)
    bits = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    M.shuffle_batched_(dev, seed, bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    got_bits = bits.cpu().numpy()
    for a, (n, eb) in enumerate(zip(sizes, ebs)):
        want, wbits = O.permutation(n, 4096, seed + a)
        got = dev[a].cpu().numpy()
        if eb == 4:
            assert np.array_equal(got.view(np.uint32), want), (a, n)
        else:
            assert np.array_equal(got, host[a][want.astype(np.int64)]), (a, n, eb)
        assert got_bits[a] == wbits, (a, n)


def test_mixed_sizes_and_element_sizes(M):
    sizes = [0, 1, 2, 3, 100, 4096, 4097, 16384, 16385, 50000, 300007, 7, 8192, 65537]
    ebs = [4, 4, 4, 8, 16, 4, 8, 4, 4, 16, 4, 8, 16, 4]
    _say("[gpu] batched mixed")
    _check(M, sizes, ebs, 21)


def test_many_small_arrays_span_several_launches(M):
    rng = np.random.default_rng(5)
    sizes = [int(x) for x in rng.integers(2, 16385, size=150)]
    _say("[gpu] batched 150 small")
    _check(M, sizes, [4] * len(sizes), 1000)


def test_log_uniform_sizes(M):
    # sizes 2^(8 + 12u) as in the batched workload, capped for the oracle's sake
    rng = np.random.default_rng(3)
    sizes = [int(2 ** (8 + 9 * u)) for u in rng.random(120)]
    _say("[gpu] batched log-uniform")
    _check(M, sizes, [4] * len(sizes), 3)


def test_batched_workload_at_full_size(M):
    # the batched workload bench.py times: 4096 uint32 identity arrays, sizes
    # floor(2^(8 + 12u)) from seed 3, array a shuffled with seed 3 + a; the
    # eager call, then one replay of its captured graph on fresh arrays,
    # every array against the oracle
    import torch

    from paper_1508_03167_amd import inputs

    sizes = [int(x) for x in inputs.batched_sizes(4096, 3)]
    seeds = [3 + a for a in range(len(sizes))]
    _say(f"[gpu] batched workload: {len(sizes)} arrays, {sum(sizes)} elements")
    dev = [torch.arange(n, dtype=torch.int32, device="cuda") for n in sizes]
    bits = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    M.shuffle_batched_(dev, 3, bits=bits)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    got_bits = bits.cpu().numpy()
    wants, wbitss = [], []
    for a, n in enumerate(sizes):
        want, wbits = O.permutation(n, 4096, seeds[a], threads=O.max_threads())
        assert np.array_equal(dev[a].cpu().numpy().view(np.uint32), want), (a, n)
        assert got_bits[a] == wbits, (a, n)
        wants.append(want)
        wbitss.append(wbits)
    for a, n in enumerate(sizes):
        dev[a].copy_(torch.arange(n, dtype=torch.int32, device="cuda"))
    bits.zero_()
    torch.cuda.synchronize()
    with M.BatchGraph(dev, seeds, bits=bits) as g:
        g.launch()
        assert g.status() == 0
        torch.cuda.synchronize()
    got_bits = bits.cpu().numpy()
    for a, n in enumerate(sizes):
        assert np.array_equal(dev[a].cpu().numpy().view(np.uint32), wants[a]), ("graph", a, n)
        assert got_bits[a] == wbitss[a], ("graph", a, n)
    del dev
    M.release()
    torch.cuda.empty_cache()


def test_batched_equals_one_call_per_array(M):
    import torch

    sizes = [5000, 20000, 3, 70000, 16384]
    a = [torch.arange(n, dtype=torch.int32, device="cuda") for n in sizes]
    b = [t.clone() for t in a]
    M.shuffle_batched_(a, 77)
    for i, t in enumerate(b):
        M.shuffle_(t, 77 + i)
    torch.cuda.synchronize()
    for x, y in zip(a, b):
        assert torch.equal(x, y)


def test_arrays_in_several_waves(M, monkeypatch):
    # arrays with HBM passes run in waves; three arrays per wave here
    monkeypatch.setenv("MS_WAVE_ARRAYS", "3")
    sizes = [16385, 40000, 3, 100000, 65536, 131073, 5000, 20000, 300001, 16384 * 3]
    ebs = [4, 8, 4, 16, 4, 8, 4, 16, 4, 8]
    _say("[gpu] batched waves of 3")
    _check(M, sizes, ebs, 606)


def test_full_path_arrays_beside_waves(M):
    # arrays above the wave limit (2^21 elements) take the full path on the
    # side streams while the others run in a wave
    sizes = [(1 << 21) + 5, 40000, 1 << 21, 70001, (1 << 21) + 4096 * 3, 9000]
    ebs = [4, 4, 8, 16, 4, 4]
    _say("[gpu] batched full path + wave")
    _check(M, sizes, ebs, 4242)


def test_two_host_threads_on_two_streams(M):
    # two host threads batch full-path arrays (spread over each caller
    # stream's own side streams) and wave arrays at the same time, each on
    # its own stream; every result and every stream's status stays its own
    import threading

    import torch

    _say("[gpu] batched from two host threads")
    sizes = [(1 << 21) + 5, 40000, (1 << 21) + 4096, 9000, 1 << 22]
    ebs = [4, 8, 4, 4, 8]
    jobs = []
    for k in range(2):
        host, dev = _make(sizes, ebs, 900 + k)
        jobs.append((900 + k, host, dev, torch.zeros(len(sizes), dtype=torch.int64, device="cuda"),
                     torch.cuda.Stream()))
    torch.cuda.synchronize()
    errors = []

    def work(seed, dev, bits, st):
        try:
            with torch.cuda.stream(st):
                for _ in range(3):  # the same batch three times in a row
                    M.shuffle_batched_(dev, seed, bits=bits, stream=st)
            errors.append((seed, M.device_status(st)))
        except Exception as e:  # noqa: BLE001
            errors.append((seed, repr(e)))

    th = [threading.Thread(target=work, args=(s, d, b, st)) for s, _, d, b, st in jobs]
    for t in th:
        t.start()
    for t in th:
        t.join()
    torch.cuda.synchronize()
    assert sorted(errors) == [(900, 0), (901, 0)], errors
    for seed, host, dev, bits, _ in jobs:
        got_bits = bits.cpu().numpy()
        for a, (n, eb) in enumerate(zip(sizes, ebs)):
            p, b = O.permutation(n, 4096, seed + a)
            want = np.arange(n, dtype=np.int64)
            for _ in range(3):
                want = want[p.astype(np.int64)]
            got = dev[a].cpu().numpy()
            if eb == 4:
                assert np.array_equal(got.view(np.uint32), want), (seed, a, n)
            else:
                assert np.array_equal(got, host[a][want]), (seed, a, n, eb)
            assert got_bits[a] == 3 * b, (seed, a, n)
