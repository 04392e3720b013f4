"""Pins for the whole oracle: MergeShuffle yields a uniformly random permutation.

* exact: enumerate every outcome of every coin flip (probability 1/2) and
  every bounded draw (probability 1/k) for n <= 6 and several cutoffs; each
  of the n! permutations must get probability exactly 1/n! (Lemma 1 applied
  level by level; with cutoff >= n the top-level routine is Algorithm 1 alone);
* statistical: seeded runs through the Philox streams, chi-square over all of
  S_n for small n and over position marginals for larger n;
* structural: the top-level routine's partition (Appendix A.2: c, q, block bounds).
"""
import math
from collections import defaultdict
from fractions import Fraction

import numpy as np
import pytest
from scipy.stats import chisquare

from oracle import oracle as O


def _enumerate(n, cutoff, placement):
    probs = defaultdict(Fraction)
    stack = [((), Fraction(1))]
    while stack:
        sc, p = stack.pop()
        perm, _, need = O.shuffle_scripted(n, cutoff, sc, placement)
        if perm is None:
            for ch in range(need):
                stack.append((sc + (ch,), p / need))
        else:
            probs[tuple(perm.tolist())] += p
    return probs


CASES = [(n, B) for n in range(1, 6) for B in (1, 2, 3)] + [(6, 3), (6, 6), (5, 5)]


@pytest.mark.parametrize("n,B", CASES)
@pytest.mark.parametrize("placement", [O.R2, O.R1])
def test_exact_uniformity_small_n(n, B, placement):
    probs = _enumerate(n, B, placement)
    assert len(probs) == math.factorial(n)
    assert set(probs.values()) == {Fraction(1, math.factorial(n))}


@pytest.mark.slow
@pytest.mark.parametrize("B", [1, 2])
def test_exact_uniformity_n6_deep(B):
    probs = _enumerate(6, B, O.R2)
    assert set(probs.values()) == {Fraction(1, 720)} and len(probs) == 720


def _lehmer_rank(perms):
    perms = np.asarray(perms, dtype=np.int64)
    cnt, n = perms.shape
    rank = np.zeros(cnt, dtype=np.int64)
    for i in range(n):
        smaller = (perms[:, i + 1:] < perms[:, i:i + 1]).sum(axis=1)
        rank = rank * (n - i) + smaller
    return rank


@pytest.mark.parametrize("n,B,count", [(3, 1, 30000), (4, 1, 48000), (5, 2, 120000), (6, 1, 144000),
                                       (7, 2, 200000)])
def test_chi_square_over_all_permutations(n, B, count):
    perms, _ = O.sample_permutations(n, B, 10**6 * n + B, count)
    obs = np.bincount(_lehmer_rank(perms), minlength=math.factorial(n))
    assert obs.size == math.factorial(n)
    assert chisquare(obs).pvalue > 1e-5


@pytest.mark.parametrize("n,B,count", [(9, 2, 40000), (10, 1, 40000), (10, 3, 40000), (33, 4, 20000),
                                       (100, 8, 8000)])
def test_position_marginals(n, B, count):
    perms, _ = O.sample_permutations(n, B, 7 * 10**6 + n, count)
    # element x lands at slot p with probability 1/n
    table = np.zeros((n, n), dtype=np.int64)
    for p in range(n):
        table[p] += np.bincount(perms[:, p], minlength=n)
    assert chisquare(table.ravel()).pvalue > 1e-5
    # pairs of neighbouring slots: ordered pairs (x, y) equally likely
    if n <= 10:
        pair = perms[:, 0].astype(np.int64) * n + perms[:, 1]
        obs = np.bincount(pair, minlength=n * n).reshape(n, n)
        off = obs[~np.eye(n, dtype=bool)]
        assert obs.trace() == 0
        assert chisquare(off).pvalue > 1e-5


def test_driver_partition():
    # Appendix A.2: c = least c with (n >> c) <= cutoff, blocks of n*i >> c.
    assert O.levels(1 << 20, 4096) == 8
    assert O.levels(1 << 30, 4096) == 18
    assert O.levels(1 << 27, 4096) == 15
    assert O.levels(4096, 4096) == 0
    assert O.levels(4097, 4096) == 1
    assert O.levels(8193, 4096) == 1   # blocks of 4096 and 4097
    assert O.levels(8194, 4096) == 2
    for n, B in [(8193, 4096), (10**5, 1000), (12345, 77)]:
        c = O.levels(n, B)
        sizes = np.diff([(n * i) >> c for i in range((1 << c) + 1)])
        assert sizes.min() >= 1 and sizes.max() <= B + 1 and sizes.sum() == n


def test_cutoff_at_least_n_is_fisher_yates():
    # with c = 0 the whole array is one leaf: Algorithm 1 with unit 0
    for n in (2, 3, 17, 1000):
        pi, bits = O.permutation(n, n, 31)
        fy, fbits = O.fisher_yates_seeded(np.arange(n, dtype=np.uint32), 31, 0)
        assert np.array_equal(pi, fy) and bits == fbits


def test_trivial_sizes_and_threads():
    assert O.permutation(0, 4, 1)[1] == 0
    pi, bits = O.permutation(1, 4, 1)
    assert pi.tolist() == [0] and bits == 0
    # OpenMP over blocks and merges does not change the result
    a, ba = O.permutation(300000, 1000, 77, threads=1)
    b, bb = O.permutation(300000, 1000, 77, threads=4)
    assert np.array_equal(a, b) and ba == bb
    assert np.array_equal(np.sort(a), np.arange(300000))
