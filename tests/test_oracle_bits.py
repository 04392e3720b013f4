"""Pins for the oracle's random-bit count.

* the paper's own numbers: its Table (Section 3) prints the mean bits of
  Fisher-Yates over 100 trials; the exact mean with Fast Dice Roller draws
  (bitstats.py) must sit within the sampling error of a 100-trial mean, and
  so must the oracle's own 100-trial mean (leaf only: cutoff >= n);
* Lemma 2 / Section 1.2: the oracle's total bits against the exact mean and
  variance of the whole shuffle, for single seeds (5 sd) and for means over
  many seeds (5 standard errors), at power-of-two and ragged sizes;
* n log2 n + Theta(n): E/n - log2 n stays bounded as n grows;
* the paper's MergeShuffle row (cutoff unstated) lies just above the
  Fisher-Yates cost, and some power-of-two cutoff reproduces it to 0.3 %
  (a loose pin, since the cutoff is not printed).
"""
import math
import os

import numpy as np
import pytest

import bitstats
from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _paper_table():
    rows = {}
    with open(os.path.join(HERE, "golden", "paper_bit_table.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            rows[k] = [int(x) for x in v]
    return rows


@pytest.mark.parametrize("col,n", [(0, 10**5), (1, 10**6)])
def test_paper_fisher_yates_row_matches_exact_mean(col, n):
    paper = _paper_table()["fisher_yates"][col]
    e, v = bitstats.fisher_yates_moments(n)
    se100 = math.sqrt(v / 100)
    assert abs(paper - e) < 4 * se100, (paper, e, se100)


def test_oracle_fisher_yates_100_trials_vs_paper():
    n = 10**5
    paper = _paper_table()["fisher_yates"][0]
    e, v = bitstats.fisher_yates_moments(n)
    bits = [O.permutation(n, n, 5000 + s)[1] for s in range(100)]
    mean = float(np.mean(bits))
    se100 = math.sqrt(v / 100)
    assert abs(mean - e) < 5 * se100
    assert abs(mean - paper) < 6 * se100


@pytest.mark.parametrize("n,B", [(2, 1), (3, 1), (4, 1), (4, 2), (7, 2)])
def test_tiny_exact_means(n, B):
    e, v = bitstats.shuffle_moments(n, B)
    bits = O.sample_permutations(n, B, 123, 40000)[1].astype(np.float64)
    if v == 0:
        assert set(bits.tolist()) == {e} or np.allclose(bits, e)
    else:
        assert abs(bits.mean() - e) < 5 * math.sqrt(v / bits.size)
    if (n, B) == (2, 1):
        assert np.all(bits == 3)


def test_config_small_single_seed():
    # n = 2^20 identity, seed 1, cutoff 2^12
    e, v = bitstats.shuffle_moments(1 << 20, 4096)
    assert abs(e - 20936140.04) < 0.1
    _, bits = O.permutation(1 << 20, 4096, 1)
    assert abs(bits - e) < 5 * math.sqrt(v)


@pytest.mark.parametrize("n,B,trials", [(1 << 14, 64, 300), (100007, 1000, 60), (5000, 4096, 400),
                                        (777, 5, 2000)])
def test_mean_bits_over_seeds(n, B, trials):
    e, v = bitstats.shuffle_moments(n, B)
    _, bits = O.sample_permutations(n, B, 31337 + n, trials)
    mean = float(bits.astype(np.float64).mean())
    assert abs(mean - e) < 5 * math.sqrt(v / trials), (mean, e)


def test_bits_are_n_log_n_plus_linear():
    vals = []
    for k in range(10, 19, 2):
        n = 1 << k
        e, _ = bitstats.shuffle_moments(n, 64)
        vals.append(e / n - k)
    # the linear term converges (Section 1.2: the sum of i / 2^(i/2) is finite)
    steps = np.diff(vals)
    assert all(0 < x < 2 for x in vals), vals
    assert np.all(steps > 0) and np.all(steps[1:] < 0.75 * steps[:-1]), vals


@pytest.mark.parametrize("col,n", [(0, 10**5), (1, 10**6)])
def test_paper_mergeshuffle_row_band(col, n):
    t = _paper_table()
    fy = t["fisher_yates"][col]
    ms = t["mergeshuffle"][col]
    assert fy < ms < 1.01 * fy
    rel = []
    for B in (1 << 12, 1 << 14, 1 << 15, 1 << 16):
        e, _ = bitstats.shuffle_moments(n, B)
        assert fy < e < 1.03 * fy
        rel.append(abs(e - ms) / ms)
    # some power-of-two cutoff reproduces the printed row to 0.3 %
    assert min(rel) < 0.003, rel
