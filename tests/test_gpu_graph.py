"""GPU parity of batched calls captured in a HIP graph (ms_batch_graph_*):
every replay shuffles each array exactly as ms_shuffle_ex with its own seed
and knobs would, so the k-th replay leaves the oracle's permutation applied
k times, with k times its bits.  Replays are separated by other work and
synchronizations, and run on two different streams in turn."""
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


def _arrays(sizes, ebs, seed):
    import torch

    rng = np.random.default_rng(seed)
    host, dev = [], []
    for n, eb in zip(sizes, ebs):
        if eb == 4:
            v = np.arange(n, dtype=np.int32)
        else:
            v = rng.integers(0, 2**62, size=(n, eb // 8), dtype=np.int64)
        host.append(v)
        dev.append(torch.from_numpy(v.copy()).cuda())
    return host, dev


def _check(host, dev, sizes, Bs, seeds, bits, reps):
    got_bits = bits.cpu().numpy()
    for a, n in enumerate(sizes):
        p, wb = O.permutation(n, Bs[a] or 4096, seeds[a])
        idx = np.arange(n, dtype=np.int64)
        for _ in range(reps):
            idx = idx[p.astype(np.int64)]
        assert np.array_equal(dev[a].cpu().numpy(), host[a][idx]), (reps, a, n)
        assert got_bits[a] == reps * wb, (reps, a, n)


def test_graph_replays_equal_the_oracle(M):
    import torch

    sizes = [3, 40000, 100000, (1 << 21) + 5, 70001, 5000, (1 << 21) + 4096 * 3, 9000, 300007, 1]
    ebs = [4, 4, 8, 4, 16, 4, 8, 4, 4, 4]
    Bs = [0, 1000, 0, 0, 2048, 100, 0, 4096, 3000, 0]
    seeds = [11 + 7 * i for i in range(len(sizes))]
    _say("[gpu] graph: mixed arrays, per-array cutoffs")
    host, dev = _arrays(sizes, ebs, 5)
    bits = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    other = torch.arange(1 << 20, dtype=torch.int32, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    torch.cuda.synchronize()
    with M.BatchGraph(dev, seeds, cfgs=[M.config(leaf_B=b) for b in Bs], bits=bits) as g:
        assert g.scratch_bytes > 0
        for rep in range(1, 4):
            st = s1 if rep % 2 else s2
            g.launch(st)
            assert g.status(st) == 0
            torch.cuda.synchronize()
            _check(host, dev, sizes, Bs, seeds, bits, rep)
            # eager work between replays
            M.shuffle_(other, rep)
            torch.cuda.synchronize()


def test_graph_of_many_small_arrays(M):
    import torch

    from paper_1508_03167_amd import inputs

    sizes = [int(x) for x in inputs.batched_sizes(600, 3)]
    ebs = [4] * len(sizes)
    seeds = [3 + a for a in range(len(sizes))]
    _say("[gpu] graph: 600 log-uniform arrays")
    host, dev = _arrays(sizes, ebs, 6)
    bits = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    g = M.BatchGraph(dev, seeds, bits=bits)
    try:
        g.launch()
        torch.cuda.synchronize()
        _check(host, dev, sizes, [0] * len(sizes), seeds, bits, 1)
        # the same arrays batched eagerly from the same state: one more step
        ref = [d.clone() for d in dev]
        M.shuffle_batched_(ref, 3)
        g.launch()
        torch.cuda.synchronize()
        assert all(torch.equal(x, y) for x, y in zip(dev, ref))
    finally:
        g.destroy()


def test_graph_rejects_bad_arguments(M):
    import torch

    x = torch.zeros(1001, dtype=torch.int32, device="cuda")
    with pytest.raises(M.MSError):  # cutoff above 4096
        M.BatchGraph([x], [1], cfgs=[M.config(leaf_B=5000)])
    with pytest.raises(ValueError):
        M.BatchGraph([x], [1, 2])


def _check_tuned(M, dev, host, sizes, seeds, bits):
    got_bits = bits.cpu().numpy()
    for a, n in enumerate(sizes):
        B = M.leaf_B_for(n)
        p, wb = O.permutation(n, B, seeds[a])
        assert np.array_equal(dev[a].cpu().numpy(), host[a][p.astype(np.int64)]), (a, n, B)
        assert got_bits[a] == wb, (a, n, B)


def test_tuned_calls_take_the_table_and_report_the_cutoff(M):
    import torch

    sizes = [5000, 70000, 100, 8191, (1 << 16) + 7, 300000]
    seeds = [50 + a for a in range(len(sizes))]
    table = [{"elem_bytes": 4, "log2_n": 12, "leaf_B": 1000, "levels_per_pass": 2, "leaf_big": True},
             {"elem_bytes": 4, "log2_n": 16, "leaf_B": 2048, "levels_per_pass": 4, "leaf_big": False},
             {"elem_bytes": 4, "log2_n": 18, "leaf_B": 3000, "levels_per_pass": 1, "leaf_big": True}]
    _say("[gpu] tuned batched and graph calls, synthetic table")
    try:
        M.tune_set(table)
        assert [M.leaf_B_for(n) for n in sizes] == [1000, 2048, 4096, 1000, 2048, 3000]
        host, dev = _arrays(sizes, [4] * len(sizes), 8)
        bits = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
        M.shuffle_batched_(dev, 50, bits=bits, tuned=True)
        torch.cuda.synchronize()
        assert M.device_status() == 0
        _check_tuned(M, dev, host, sizes, seeds, bits)
        host, dev = _arrays(sizes, [4] * len(sizes), 9)
        bits.zero_()
        with M.BatchGraph(dev, seeds, cfgs=[M.config(tuned=True)] * len(sizes), bits=bits) as g:
            g.launch()
            assert g.status() == 0
        _check_tuned(M, dev, host, sizes, seeds, bits)
    finally:
        M.tune_set([])


def test_autotuner_writes_its_cache_and_the_table_follows_it(M, tmp_path):
    import json

    import torch

    from paper_1508_03167_amd import autotune

    path = str(tmp_path / "tune.json")
    _say("[gpu] autotuner on two buckets")
    try:
        rec = autotune.ensure_tuned([(4, 12), (4, 17)], path=path, budget=1 << 19, reps=1)
        saved = json.load(open(path))
        assert saved["entries"] == rec["entries"] and len(rec["entries"]) == 2
        for e in rec["entries"]:
            assert e["leaf_B"] in autotune.CUTOFFS and e["ms"] <= e["default_ms"] + 1e-9
            assert M.leaf_B_for(1 << e["log2_n"]) == e["leaf_B"]
        sizes = [4100, 6000, 140000, 200000]
        seeds = [70 + a for a in range(len(sizes))]
        host, dev = _arrays(sizes, [4] * len(sizes), 10)
        bits = torch.zeros(len(sizes), dtype=torch.int64, device="cuda")
        M.shuffle_batched_(dev, 70, bits=bits, tuned=True)
        torch.cuda.synchronize()
        _check_tuned(M, dev, host, sizes, seeds, bits)
    finally:
        M.tune_set([])
