"""Pins for the oracle's BalancedShuffle (Section 2): merges that interleave
the two shuffled halves by a uniformly random word of C(n1+n2, n1).

* exact: enumerating every coin flip and bounded draw, the word each merge
  uses is uniform over C(n1+n2, n1), and the whole routine is uniform over
  S_n for n <= 6 (Section 2.2: the map S_n1 x S_n2 x C(n1+n2, n1) -> S_n1+n2 is
  a bijection, so uniform inputs and a uniform word give a uniform output);
* structural: a merge keeps the relative order of each half (the word only
  says which side each slot takes from);
* the word is drawn by Algorithm 2's coin-flip loop and insertion run on the
  side labels, so it consumes exactly the bits MergeShuffle's merge does.
"""
import math
from collections import defaultdict
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O


def _enumerate_shuffle(n, cutoff):
    probs = defaultdict(Fraction)
    stack = [((), Fraction(1))]
    while stack:
        sc, p = stack.pop()
        perm, _, need = O.shuffle_scripted(n, cutoff, sc, O.BALANCED)
        if perm is None:
            for ch in range(need):
                stack.append((sc + (ch,), p / need))
        else:
            probs[tuple(perm.tolist())] += p
    return probs


@pytest.mark.parametrize("n,B", [(n, B) for n in range(1, 6) for B in (1, 2, 3)] + [(6, 3), (6, 6)])
def test_exact_uniformity_over_permutations(n, B):
    probs = _enumerate_shuffle(n, B)
    assert len(probs) == math.factorial(n)
    assert set(probs.values()) == {Fraction(1, math.factorial(n))}


@pytest.mark.parametrize("n1,n2", [(1, 1), (2, 1), (1, 2), (2, 2), (3, 2), (3, 3), (4, 3), (4, 4)])
def test_merge_word_is_uniform(n1, n2):
    # merge 0..n1-1 (A) with n1..n1+n2-1 (B); the word is where the A values land
    words = defaultdict(Fraction)
    stack = [((), Fraction(1))]
    vals = np.arange(n1 + n2, dtype=np.uint32)
    while stack:
        sc, p = stack.pop()
        out, r = O.merge_scripted(vals, n1, sc, O.BALANCED)
        if out is None:
            for ch in range(r):
                stack.append((sc + (ch,), p / r))
        else:
            words[tuple(int(v >= n1) for v in out)] += p
    assert len(words) == math.comb(n1 + n2, n1)
    assert set(words.values()) == {Fraction(1, math.comb(n1 + n2, n1))}
    assert all(sum(w) == n2 for w in words)


@pytest.mark.parametrize("n1,n2", [(1, 1), (7, 8), (100, 100), (1000, 999), (4096, 4097)])
def test_merge_keeps_each_half_in_order(n1, n2):
    rng = np.random.default_rng(n1 * 31 + n2)
    vals = rng.permutation(n1 + n2).astype(np.uint32)
    for m in range(5):
        out, P, bits = O.merge_seeded(vals, n1, 9 + m, 3, m, O.BALANCED)
        a_pos = np.isin(out, vals[:n1])
        assert a_pos.sum() == n1
        assert np.array_equal(out[a_pos], vals[:n1])
        assert np.array_equal(out[~a_pos], vals[n1:])


@pytest.mark.parametrize("n,B", [(1000, 16), (65537, 4096), (300007, 4096), (123456, 100)])
def test_same_bits_as_mergeshuffle(n, B):
    for seed in (1, 5, 2**33 + 7):
        a = np.arange(n, dtype=np.uint32)
        b = np.arange(n, dtype=np.uint32)
        ba = O.shuffle_u32(a, B, seed, O.BALANCED)
        bb = O.shuffle_u32(b, B, seed, O.R2)
        assert ba == bb
        assert np.array_equal(np.sort(a), np.arange(n, dtype=np.uint32))
        if n > B:
            assert not np.array_equal(a, b)


def test_cutoff_at_least_n_is_fisher_yates():
    # no merge level: BalancedShuffle and MergeShuffle are both Algorithm 1
    a = np.arange(3000, dtype=np.uint32)
    b = a.copy()
    O.shuffle_u32(a, 4096, 3, O.BALANCED)
    O.shuffle_u32(b, 4096, 3, O.R2)
    assert np.array_equal(a, b)
