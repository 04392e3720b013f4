"""GPU parity under the library's tuning knobs, each read once per process
(so each runs in a child process): the 1024-thread leaf with 128 KiB
super-blocks (MS_LEAF_BIG=1), the window-tree fused pass (MS_PASS_IMPL=tree)
and its 2048-slot tiles (MS_GROUP_TILE=2048), every other tile shape of the
table pass (MS_PASS_TILE=<slots>, which picks the shape of that many slots
for the element sizes that have one) and the one-level pass's other tile
sizes and staging modes (MS_PASS_VARIANT=1..5, with one-level passes).  The
permutation must not depend on any of them.

The capacity test shrinks the plan's insertion-loop pools (MS_CAP_SCALE) so
that they overflow: the calls must end normally, flag the overflow in the
status word (bit 0: target pool, bit 1: tail pool) and leave later calls
with the normal capacity exact."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))

CHILD = r"""
import sys
sys.path.insert(0, %r)
import numpy as np, torch
import paper_1508_03167_amd as M
from oracle import oracle as O
KW = %r
for n, seed, eb in [(70001, 3, 4), ((1 << 20) + 3, 4, 4), (3_000_017, 5, 4), (300_007, 6, 8), (123_457, 7, 16)]:
    want, wbits = O.permutation(n, 4096, seed)
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    if eb == 4:
        x = torch.empty(n, dtype=torch.int32, device="cuda")
        M.permutation(x, seed, bits=bits, **KW)
        got = x.cpu().numpy().view(np.uint32)
        ok = np.array_equal(got, want)
    else:
        host = np.random.default_rng(eb).integers(0, 2**63, size=(n, eb // 8), dtype=np.int64)
        x = torch.from_numpy(host.copy()).cuda()
        M.shuffle_(x, seed, bits=bits, **KW)
        ok = np.array_equal(x.cpu().numpy(), host[want.astype(np.int64)])
    torch.cuda.synchronize()
    status = M.device_status()
    print("case", n, eb, "ok" if ok and int(bits.item()) == wbits and status == 0 else "BAD", flush=True)
"""


KNOBS = [({"MS_LEAF_BIG": "1"}, {}), ({"MS_PASS_IMPL": "tree"}, {}),
         ({"MS_PASS_IMPL": "tree", "MS_GROUP_TILE": "2048"}, {})] + [
    ({"MS_PASS_TILE": str(t)}, {}) for t in (4096, 2048, 8192, 7168, 1792, 1024, 640, 512)] + [
    ({"MS_PASS_VARIANT": str(v)}, {"one_level_passes": True}) for v in range(1, 6)]


@pytest.mark.parametrize("knob,kw", KNOBS)
def test_tuning_knob_keeps_the_permutation(knob, kw):
    print(f"[gpu] knob {knob} {kw}", flush=True)
    env = dict(os.environ, **knob)
    r = subprocess.run([sys.executable, "-c", CHILD % (os.path.dirname(HERE), kw)], env=env, capture_output=True,
                       text=True, timeout=300)
    lines = [l for l in r.stdout.splitlines() if l.startswith("case")]
    assert r.returncode == 0 and len(lines) == 5, (r.stdout, r.stderr[-2000:])
    assert all(l.endswith(" ok") for l in lines), r.stdout


CAP_CHILD = r"""
import os, sys
sys.path.insert(0, %r)
import numpy as np, torch
import paper_1508_03167_amd as M
from oracle import oracle as O
x = torch.empty((1 << 22) + 5, dtype=torch.int32, device="cuda")
r = torch.arange(((1 << 19) + 3) * 2, dtype=torch.int64, device="cuda").view(-1, 2)
arrs = [torch.arange(n, dtype=torch.int32, device="cuda") for n in (40000, 3, 100000, (1 << 21) + 5, 70001)]
for scale in ("0.01", "0.000001"):
    os.environ["MS_CAP_SCALE"] = scale
    M.permutation(x, 5)
    print("flags perm", scale, M.device_status(), flush=True)
    M.shuffle_(r, 6)
    print("flags records", scale, M.device_status(), flush=True)
    M.shuffle_batched_(arrs, 7)
    print("flags batched", scale, M.device_status(), flush=True)
del os.environ["MS_CAP_SCALE"]
n = x.numel()
bits = torch.zeros(1, dtype=torch.int64, device="cuda")
M.permutation(x, 5, bits=bits)
want, wbits = O.permutation(n, 4096, 5)
ok = np.array_equal(x.cpu().numpy().view(np.uint32), want) and int(bits.item()) == wbits
print("after", "ok" if ok and M.device_status() == 0 else "BAD", flush=True)
"""


def test_pool_overflow_is_flagged_and_harmless():
    print("[gpu] capacity overflow (MS_CAP_SCALE)", flush=True)
    r = subprocess.run([sys.executable, "-c", CAP_CHILD % (os.path.dirname(HERE),)], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, (r.stdout, r.stderr[-2000:])
    flags = [int(l.split()[-1]) for l in r.stdout.splitlines() if l.startswith("flags")]
    assert len(flags) == 6 and all(f != 0 and f & ~3 == 0 for f in flags), r.stdout
    assert "after ok" in r.stdout, r.stdout
