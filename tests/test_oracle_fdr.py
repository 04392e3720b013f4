"""Pins for the oracle's bounded draw (Fast Dice Roller, [Lumbroso13]).

The draw must be exactly uniform on {0..k-1} whatever k: enumerating every bit
string, the strings accepted at each length must split evenly over the k
values.  Its mean cost is checked against closed forms worked by hand and
against the independent phase-sum in bitstats.py.
"""
from fractions import Fraction

import numpy as np
import pytest

import bitstats
from oracle import oracle as O


def _enumerate(k, max_len):
    """{length: [count per value]} over all bit strings up to max_len."""
    per_len = {}
    stack = [()]
    while stack:
        s = stack.pop()
        v, used = O.fdr_on_bits(k, list(s))
        if v >= 0:
            per_len.setdefault(len(s), [0] * k)[v] += 1
            continue
        if len(s) < max_len:
            stack.append(s + (0,))
            stack.append(s + (1,))
    return per_len


@pytest.mark.parametrize("k", list(range(2, 41)) + [64, 96, 100, 127, 128, 129])
def test_fdr_exact_uniform_law(k):
    depth = (k - 1).bit_length() + 7
    per_len = _enumerate(k, depth)
    mass = Fraction(0)
    for ln, counts in per_len.items():
        # every value gets the same number of accepted strings of each length
        assert len(set(counts)) == 1, (k, ln, counts)
        mass += Fraction(sum(counts), 2**ln)
    # what is left unaccepted at this depth shrinks geometrically
    assert 1 - mass <= Fraction(1, 2**7)


def test_fdr_k1_and_powers_of_two():
    assert O.fdr_on_bits(1, []) == (0, 0)
    for j in range(1, 12):
        per_len = _enumerate(2**j, j + 3)
        assert list(per_len) == [j]  # always exactly j bits


def test_fdr_mean_cost_closed_forms():
    # k = 3: two bits accept with probability 3/4, else the state is back to
    # its start, so E = 2 + E/4, E = 8/3.  k = 5: three bits accept with
    # probability 5/8; else v = 3 and one bit gives v = 6 >= 5, accepted with
    # probability 5/6, else v = 1 (the start): E = 3 + 3/8 * (1 + 1/6 * E).
    def mean(k, depth):
        tot = Fraction(0)
        for ln, counts in _enumerate(k, depth).items():
            tot += Fraction(ln * sum(counts), 2**ln)
        return tot

    e3 = mean(3, 40)
    assert abs(float(e3) - 8 / 3) < 1e-9
    e5 = mean(5, 60)
    # E5 = 3 + 3/8 + (3/8)(1/6) E5  ->  E5 (1 - 1/16) = 27/8
    want5 = Fraction(27, 8) / (1 - Fraction(1, 16))
    assert abs(float(e5) - float(want5)) < 1e-9
    m, _ = bitstats.fdr_moments([3, 5])
    assert abs(m[0] - 8 / 3) < 1e-12 and abs(m[1] - float(want5)) < 1e-12


@pytest.mark.parametrize("k", [6, 7, 11, 12, 13, 100, 1000])
def test_fdr_phase_sum_matches_enumeration(k):
    depth = (k - 1).bit_length() + 24
    tot = Fraction(0)
    for ln, counts in _enumerate(k, depth).items():
        tot += Fraction(ln * sum(counts), 2**ln)
    m, _ = bitstats.fdr_moments([k])
    assert abs(float(tot) - m[0]) < 1e-4


def test_seeded_draws_chi_square():
    from scipy.stats import chisquare

    for k in (3, 7, 10, 4097):
        vals = np.array([O.random_int(2024, 1, 5, d, k)[0] for d in range(20000)])
        assert vals.min() >= 0 and vals.max() < k
        if k <= 10:
            obs = np.bincount(vals, minlength=k)
            assert chisquare(obs).pvalue > 1e-4
        else:
            obs = np.bincount(vals * 16 // k, minlength=16)
            assert chisquare(obs).pvalue > 1e-4
