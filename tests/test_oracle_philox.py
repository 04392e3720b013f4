"""Pins for the oracle's generator: Philox-4x32-10 and the stream rule.

Philox is pinned against values the generator's authors publish and against
PyTorch's independent host implementation.  The stream rule (which Philox
word and bit a flip or a bounded draw reads) is this implementation's own convention
for a paper that names no generator; its test states the rule once more.
"""
import os
import random
import shutil
import subprocess

import numpy as np
import pytest

from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _kat():
    rows = []
    with open(os.path.join(HERE, "golden", "philox_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            w = [int(x, 16) for x in line.split()]
            rows.append((w[0:4], w[4:6], tuple(w[6:10])))
    return rows


def test_philox_random123_kat():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, want in rows:
        assert O.philox4x32_10(ctr, key) == want


@pytest.fixture(scope="module")
def aten_kat(tmp_path_factory):
    import torch

    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    gxx = shutil.which("g++")
    if gxx is None or not os.path.exists(os.path.join(inc, "ATen", "core", "PhiloxRNGEngine.h")):
        pytest.skip("no g++ or no ATen Philox header")
    exe = str(tmp_path_factory.mktemp("aten") / "kat")
    subprocess.check_call([gxx, "-O1", "-std=c++17", "-I" + inc, "-o", exe,
                           os.path.join(HERE, "aten_philox_kat.cpp")])
    return exe


def test_philox_matches_aten(aten_kat):
    rng = random.Random(12345)
    cases = [(rng.getrandbits(64), rng.getrandbits(64), rng.getrandbits(64)) for _ in range(500)]
    cases += [(0, 0, 0), (2**64 - 1, 2**64 - 1, 2**64 - 1), (7, 1 << 40, 3)]
    inp = "".join(f"{s} {sub} {off}\n" for s, sub, off in cases)
    out = subprocess.run([aten_kat], input=inp, capture_output=True, text=True, check=True).stdout.split("\n")
    for (s, sub, off), line in zip(cases, out):
        want = tuple(int(x) for x in line.split())
        ctr = (off & 0xFFFFFFFF, off >> 32, sub & 0xFFFFFFFF, sub >> 32)
        key = (s & 0xFFFFFFFF, s >> 32)
        assert O.philox4x32_10(ctr, key) == want


def test_flip_stream_rule():
    # FLIP(L, m, t) = bit (t & 31) of word ((t >> 5) & 3) of Philox((t >> 7, m, L, 1 << 28)).
    rng = random.Random(5)
    for _ in range(300):
        seed = rng.getrandbits(64)
        L, m, t = rng.randrange(1, 33), rng.getrandbits(32), rng.getrandbits(32)
        w = O.philox4x32_10((t >> 7, m, L, 1 << 28), (seed & 0xFFFFFFFF, seed >> 32))
        assert O.random_bit(seed, L, m, t) == (w[(t >> 5) & 3] >> (t & 31)) & 1


def test_draw_stream_rule():
    # DRAW(L, u, d) feeds the Fast Dice Roller with word (d & 3) of
    # Philox((d >> 2, u, L, 2 << 28)) most-significant bit first, then with
    # Philox((d, u, L, (3 << 28) | j)), j = 0, 1, ..., words x0..x3.
    rng = random.Random(6)
    for it in range(300):
        seed = rng.getrandbits(64)
        L, u, d = rng.randrange(0, 33), rng.getrandbits(32), rng.getrandbits(32)
        k = rng.choice([2, 3, 5, 4097, rng.randrange(2, 2**32), 2**31 + 1, 2**32 - 1])
        key = (seed & 0xFFFFFFFF, seed >> 32)
        bits = []
        w = O.philox4x32_10((d >> 2, u, L, 2 << 28), key)[d & 3]
        bits += [(w >> (31 - i)) & 1 for i in range(32)]
        for j in range(4):
            for x in O.philox4x32_10((d, u, L, (3 << 28) | j), key):
                bits += [(x >> (31 - i)) & 1 for i in range(32)]
        v, used = O.fdr_on_bits(k, bits)
        got, gbits = O.random_int(seed, L, u, d, k)
        assert v >= 0 and got == v and gbits == used


def test_draw_continuation_is_exercised():
    # k = 2^31 + 1 rejects about half the time after 32 bits, so continuation
    # blocks are read; the value must still be in range and the count > 32.
    seen_long = 0
    for d in range(400):
        v, b = O.random_int(99, 3, 17, d, 2**31 + 1)
        assert 0 <= v <= 2**31
        seen_long += b > 32
    assert seen_long > 100
