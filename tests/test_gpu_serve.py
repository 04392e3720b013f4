"""The serving loop on the GPU: every request's result in the mix equals its
result alone (ms_shuffle with the request's seed) and the oracle's
permutation of its original values.  The HBM budget is small, so requests
queue for admission while several batches are in flight; the payload pool
is not recycled in this test, so every request's buffer still holds its
result when the stream ends.
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


@pytest.mark.parametrize("inflight,budget_mb", [(1, 1024), (3, 64)])
def test_results_in_the_mix_equal_results_alone(M, inflight, budget_mb):
    import torch

    from paper_1508_03167_amd.serve import GpuExecutor, Request, Server

    print(f"[gpu] serve mix inflight={inflight} budget={budget_mb} MiB", flush=True)
    sys.stdout.flush()
    rng = np.random.default_rng(inflight * 7 + budget_mb)
    sizes = [int(2 ** (10 + 10 * u)) for u in rng.random(50)] + [2, 3, 4097, 8193, (1 << 21) + 7]
    ebs = [int(x) for x in rng.choice([4, 8], size=len(sizes))]
    reqs, t = [], 0.0
    for i, (n, eb) in enumerate(zip(sizes, ebs)):
        t += float(rng.exponential(2e-4))
        reqs.append(Request(i, n, eb, 1000 + 7 * i, t))
    vals = {}

    def fill(pool):
        off = 0
        for r in reqs:
            v = rng.integers(0, 2**62, size=r.n, dtype=np.int64)
            if r.elem_bytes == 4:
                v = (v & 0x7FFFFFFF).astype(np.int32)
            vals[r.rid] = (off, v)
            raw = torch.from_numpy(v.view(np.uint8)).cuda()
            pool[off:off + raw.numel()].copy_(raw)
            off += -(-r.n * r.elem_bytes // 256) * 256

    class KeepExecutor(GpuExecutor):
        def release(self, r):  # no reuse: every buffer keeps its result
            pass

    payload = sum(-(-r.n * r.elem_bytes // 256) * 256 for r in reqs)
    ex = KeepExecutor(payload, max_inflight=inflight, fill=fill)
    budget = budget_mb << 20
    srv = Server(ex, budget, max_inflight=inflight)
    import time

    def wait(dt):
        if dt > 0:
            time.sleep(min(dt, 0.0005))

    done, rej = srv.run(reqs, time.perf_counter, wait)
    torch.cuda.synchronize()
    assert not rej and len(done) == len(reqs)
    assert srv.peak_used <= budget
    assert srv.batches < len(reqs)
    for r in reqs:
        off, v = vals[r.rid]
        assert r.offset == off  # first fit in arrival order, nothing released
        got = ex.view(r).cpu().numpy()
        alone = torch.from_numpy(v.copy()).cuda()
        M.shuffle_(alone, r.seed)
        assert np.array_equal(got, alone.cpu().numpy()), r.rid
        want, _ = O.permutation(r.n, 4096, r.seed)
        assert np.array_equal(got, v[want.astype(np.int64)]), r.rid
