"""GPU parity: the HIP path against the CPU oracle, element by element.

Every case runs the library through its C ABI (via the ctypes binding) on the
GPU and compares the permutation and the random-bit count with the oracle on
the same (n, cutoff, seed).  Integer work: the bar is bit-exact.
"""
import json
import os
import sys

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))


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


def gpu_perm(M, n, seed, **kw):
    import torch

    out = torch.empty(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.permutation(out, seed, bits=bits, **kw)
    torch.cuda.synchronize()
    assert M.device_status() == 0
    return out.cpu().numpy().view(np.uint32), int(bits.item())


SIZES = [2, 3, 5, 17, 100, 1000, 4095, 4096, 4097, 5000, 8192, 8193, 12289, 32768, 32769, 40000,
         65536, 65537, 100003, 262144, 300007, 1 << 20]


@pytest.mark.parametrize("n", SIZES)
def test_permutation_matches_oracle(M, n):
    for seed in (1, 2**40 + 3):
        _say(f"[gpu] permutation n={n} seed={seed}")
        got, gbits = gpu_perm(M, n, seed)
        want, wbits = O.permutation(n, 4096, seed)
        assert np.array_equal(got, want), f"first mismatch at {np.argmax(got != want)}"
        assert gbits == wbits


@pytest.mark.parametrize("n,B", [(10, 1), (100, 1), (1000, 2), (5000, 3), (100000, 4), (77777, 16),
                                 (200000, 100), (123457, 1000), (1 << 18, 64), (999999, 4095)])
def test_small_cutoffs_match_oracle(M, n, B):
    _say(f"[gpu] cutoff n={n} B={B}")
    got, gbits = gpu_perm(M, n, 99, leaf_B=B)
    want, wbits = O.permutation(n, B, 99)
    assert np.array_equal(got, want)
    assert gbits == wbits


@pytest.mark.parametrize("n", [4097, 50000, 1 << 17, 700001])
def test_result_independent_of_lds_levels(M, n):
    _say(f"[gpu] lds-level variants n={n}")
    want, wbits = O.permutation(n, 4096, 5)
    for kw in ({}, {"hbm_only": True}, {"lds_levels_max": 1}, {"lds_levels_max": 2}):
        got, gbits = gpu_perm(M, n, 5, **kw)
        assert np.array_equal(got, want), kw
        assert gbits == wbits, kw


@pytest.mark.parametrize("n,B", [(65537, 4096), (300007, 4096), (1048576 + 12345, 4096), (3000017, 4096),
                                 (200000, 100), (777777, 7), (1 << 21, 2048)])
def test_result_independent_of_levels_per_pass(M, n, B):
    _say(f"[gpu] levels-per-pass variants n={n} B={B}")
    want, wbits = O.permutation(n, B, 11)
    for kw in ({"levels_per_pass": 1}, {"levels_per_pass": 2}, {"levels_per_pass": 3}, {"levels_per_pass": 4},
               {"levels_per_pass": 2, "hbm_only": True}, {"levels_per_pass": 3, "hbm_only": True},
               {"levels_per_pass": 4, "hbm_only": True}, {"one_level_passes": True},
               {"one_level_passes": True, "hbm_only": True}):
        got, gbits = gpu_perm(M, n, 11, leaf_B=B, **kw)
        assert np.array_equal(got, want), (kw, int(np.argmax(got != want)))
        assert gbits == wbits, kw


@pytest.mark.parametrize("n", [1000, 4097, 65537, 300007])
def test_shuffle_u32_equals_permutation_of_identity(M, n):
    import torch

    _say(f"[gpu] shuffle_ u32 n={n}")
    x = torch.arange(n, dtype=torch.int32, device="cuda")
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.shuffle_(x, 42, bits=bits)
    want, wbits = O.permutation(n, 4096, 42)
    assert np.array_equal(x.cpu().numpy().view(np.uint32), want)
    assert int(bits.item()) == wbits


@pytest.mark.parametrize("eb", [8, 16])
@pytest.mark.parametrize("n", [3, 4097, 8193, 20000, 123457, (1 << 20) + 7, 4096 * 2**9 + 300])
def test_records_follow_the_index_permutation(M, eb, n):
    # 8193, 2^20 + 7 and 4096 * 2^9 + 300 have leaves of cutoff + 1 = 4097
    # elements (16-byte leaves of that size take the 128 KiB super-block)
    import torch

    _say(f"[gpu] records eb={eb} n={n}")
    rng = np.random.default_rng(n + eb)
    vals = rng.integers(0, 2**63, size=(n, eb // 8), dtype=np.int64)
    x = torch.from_numpy(vals.copy()).cuda()
    M.shuffle_(x, 1234)
    want, _ = O.permutation(n, 4096, 1234)
    assert np.array_equal(x.cpu().numpy(), vals[want.astype(np.int64)])


def test_trivial_sizes(M):
    import torch

    for n in (0, 1):
        x = torch.arange(max(n, 1), dtype=torch.int32, device="cuda")[:n]
        M.shuffle_(x, 3)
    torch.cuda.synchronize()


def test_config_small_golden(M):
    g = json.load(open(os.path.join(HERE, "golden", "configs.json")))["perm_n2^20_seed1"]
    got, gbits = gpu_perm(M, g["n"], g["seed"])
    import hashing

    assert gbits == g["bits"]
    assert list(hashing.fingerprint_np(got)) == g["fingerprint"]
    for p, v in g["samples"]:
        assert got[p] == v


def test_repeat_calls_deterministic(M):
    a, ab = gpu_perm(M, 300007, 8)
    b, bb = gpu_perm(M, 300007, 8)
    assert np.array_equal(a, b) and ab == bb


@pytest.mark.parametrize("off", [1, 2, 3])
@pytest.mark.parametrize("n", [70001, 300007])
def test_views_not_16_byte_aligned(M, n, off):
    # 4-byte aligned but not 16-byte aligned arrays take the scalar staging path
    import torch

    _say(f"[gpu] unaligned view n={n} off={off}")
    base = torch.zeros(n + 4, dtype=torch.int32, device="cuda")
    x = base[off:off + n]
    x.copy_(torch.arange(n, dtype=torch.int32, device="cuda"))
    bits = torch.zeros(1, dtype=torch.int64, device="cuda")
    M.shuffle_(x, 17, bits=bits)
    want, wbits = O.permutation(n, 4096, 17)
    assert np.array_equal(x.cpu().numpy().view(np.uint32), want)
    assert int(bits.item()) == wbits
    assert int(base[:off].abs().sum().item()) == 0 and int(base[off + n:].abs().sum().item()) == 0


def test_allocation_failure_is_reported(M):
    # the library's scratch allocation refused (test hook): the call fails
    # cleanly with MS_ERR_NOMEM and leaves the array untouched
    import subprocess

    code = (
        "import sys, torch; sys.path.insert(0, %r)\n"
        "import paper_1508_03167_amd as M\n"
        "x = torch.arange(1 << 20, dtype=torch.int32, device='cuda')\n"
        "try:\n"
        "    M.shuffle_(x, 1)\n"
        "    print('no error')\n"
        "except M.MSError as e:\n"
        "    torch.cuda.synchronize()\n"
        "    ok = bool(torch.equal(x, torch.arange(1 << 20, dtype=torch.int32, device='cuda')))\n"
        "    print('code', e.code, 'untouched', ok)\n" % os.path.dirname(HERE))
    env = dict(os.environ, MS_FAIL_ALLOC="1")
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=120)
    assert "code -3 untouched True" in r.stdout, (r.stdout, r.stderr[-2000:])
