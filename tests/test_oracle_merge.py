"""Pins for the oracle's Merge (Algorithm 2, appendix listing merge()).

* the hand-worked example in tests/golden/worked_merge.txt;
* Lemma 1's proof: before the insertion loop, slot i holds an element of A
  exactly when flip i is 0 -- for both placements, which also share P, the
  bits, the draws and the B slots;
* merge of two singletons always uses exactly 3 bits (Lemma 2's sum for
  n1 = n2 = 1: either the second flip repeats the first and one 1-bit draw
  follows, or both sides empty and a third flip ends the loop);
* brute force of every flip and draw outcome for small sizes: averaged over
  uniformly shuffled A and B, the output is a uniformly random permutation
  of the union (Lemma 1), for both placements;
* the mean bit count of one Merge against Lemma 2's sum (bitstats.py).
"""
import itertools
import math
import os
from collections import defaultdict
from fractions import Fraction

import numpy as np
import pytest

import bitstats
from oracle import oracle as O

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden():
    d = {}
    with open(os.path.join(HERE, "golden", "worked_merge.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            d[k] = [int(x) for x in v]
    return d


def test_worked_example():
    g = _golden()
    out2, P2 = O.merge_scripted(g["values"], g["n1"][0], g["flips"], placement=O.R2)
    out1, P1 = O.merge_scripted(g["values"], g["n1"][0], g["flips"], placement=O.R1)
    assert P2 == P1 == g["P"][0]
    assert out2.tolist() == g["r2"]
    assert out1.tolist() == g["r1"]
    # one flip fewer does not end the loop: the oracle asks for another bit
    out, need = O.merge_scripted(g["values"], g["n1"][0], g["flips"][:-1], placement=O.R2)
    assert out is None and need == 2


def _all_outcomes(n1, n2, placement):
    """{tuple(out): probability} with every flip and draw enumerated."""
    vals = list(range(n1 + n2))
    probs = defaultdict(Fraction)
    stack = [((), Fraction(1))]
    while stack:
        sc, p = stack.pop()
        out, P_or_need = O.merge_scripted(vals, n1, sc, placement=placement)
        if out is None:
            need = P_or_need
            for ch in range(need):
                stack.append((sc + (ch,), p / need))
        else:
            probs[tuple(out.tolist())] += p
    return probs


@pytest.mark.parametrize("n1,n2", [(1, 1), (1, 2), (2, 1), (2, 2), (1, 4), (3, 2), (3, 3), (2, 4)])
@pytest.mark.parametrize("placement", [O.R2, O.R1])
def test_merge_of_shuffled_halves_is_uniform(n1, n2, placement):
    # Lemma 1: average the merge's output law over uniformly shuffled A and B.
    n = n1 + n2
    merged = _all_outcomes(n1, n2, placement)
    total = defaultdict(Fraction)
    pa = list(itertools.permutations(range(n1)))
    pb = list(itertools.permutations(range(n1, n)))
    w = Fraction(1, len(pa) * len(pb))
    for a in pa:
        for b in pb:
            src = list(a) + list(b)
            for out, p in merged.items():
                total[tuple(src[i] for i in out)] += w * p
    assert len(total) == math.factorial(n)
    assert set(total.values()) == {Fraction(1, math.factorial(n))}


def test_prefix_slots_follow_flips_and_readings_agree():
    rng = np.random.default_rng(7)
    for it in range(300):
        n1 = int(rng.integers(1, 40))
        n2 = int(rng.integers(1, 40))
        seed = int(rng.integers(0, 2**63))
        L, m = int(rng.integers(1, 20)), int(rng.integers(0, 1000))
        vals = np.arange(n1 + n2, dtype=np.uint32)
        o2, P2, b2 = O.merge_seeded(vals, n1, seed, L, m, placement=O.R2)
        o1, P1, b1 = O.merge_seeded(vals, n1, seed, L, m, placement=O.R1)
        assert (P2, b2) == (P1, b1)
        flips = [O.random_bit(seed, L, m, t) for t in range(P2 + 1)]
        # the loop ends on a flip whose side is empty
        side = flips[P2]
        assert flips[:P2].count(side) == (n2 if side else n1)
        assert sorted(o2.tolist()) == list(range(n1 + n2))
        # bits = P + 1 flips + the insertion loop's draws of ranges P+1..n
        draws = sum(O.random_int(seed, L, m, i, i + 1)[1] for i in range(P2, n1 + n2))
        assert b2 == P2 + 1 + draws
        if P2 == n1 + n2:
            # no insertion: slot i holds A's next element iff flip i is 0,
            # and R1 places B's elements at the same slots as R2
            ra = iter(range(n1))
            rb = iter(range(n1, n1 + n2))
            want = [next(rb) if f else next(ra) for f in flips[:P2]]
            assert o2.tolist() == want
            for i, f in enumerate(flips[:P2]):
                assert (o1[i] >= n1) == bool(f)


def test_merge_two_singletons_costs_three_bits():
    for seed in range(500):
        _, _, bits = O.merge_seeded([5, 9], 1, seed, 1, 0)
        assert bits == 3


@pytest.mark.parametrize("n1,n2", [(2, 2), (3, 3), (4, 4), (5, 3), (16, 16), (100, 101)])
def test_merge_mean_bits_matches_lemma2_sum(n1, n2):
    pre = bitstats._Prefix(n1 + n2)
    e, v = bitstats.merge_moments(n1, n2, pre)
    trials = 4000
    tot = 0
    vals = np.arange(n1 + n2, dtype=np.uint32)
    for s in range(trials):
        tot += O.merge_seeded(vals, n1, 1000 + s, 2, s)[2]
    mean = tot / trials
    se = math.sqrt(v / trials)
    assert abs(mean - e) < 5 * se + 1e-9, (mean, e, se)
