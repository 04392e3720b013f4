"""Exact mean and variance of the random-bit count of MergeShuffle.

An independent derivation used to pin the oracle's bit accounting; it never
runs the shuffle.  It follows the paper's own cost formulas:

* bounded draws: the Fast Dice Roller [Lumbroso13] (cited in the paragraph on
  the random-bit model as the draw the simulations use).  Its bit count has a
  law that does not depend on the bits' values: from v = 1 the range doubles
  until v >= k, the draw is accepted with probability k/v, otherwise v -= k and
  it continues.  Mean and variance follow by summing over the phases.
* one Merge of sizes (n1, n2), Lemma 2: the coin-flip loop ends either with
  the (n1+1)-th zero after i ones (probability C(n1+i, n1)/2^(n1+1+i)) or with
  the (n2+1)-th one after i zeros; it has used P+1 bits with P = n1+i (resp.
  n2+i), and the insertion loop then draws ranges P+1, ..., n.  Lemma 2 prices
  a draw of range k at ceil(log2 k); here the draw's exact cost replaces it.
* the whole shuffle: sum over leaves (Fisher-Yates draws of ranges 2..b) plus
  sum over merges, all independent (Section 1.2 sums the same terms for
  n = 2^m).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import gammaln


def fdr_moments(k):
    """(E[bits], Var[bits]) of one Fast Dice Roller draw of range k (array ok)."""
    k = np.atleast_1d(np.asarray(k, dtype=np.float64))
    v = np.ones_like(k)
    reach = np.ones_like(k)   # probability that this phase is reached
    used = np.zeros_like(k)   # bits read by the end of this phase
    m1 = np.zeros_like(k)
    m2 = np.zeros_like(k)
    live = k > 1
    while live.any():
        # least d with v * 2^d >= k (exact: all values are integers < 2^53)
        vs = np.where(live, v, 1.0)
        d = (np.frexp(k)[1] - np.frexp(vs)[1]).astype(np.float64)
        d = np.where(vs * np.exp2(d) < k, d + 1, d)
        d = np.where(live, np.maximum(d, 0.0), 0.0)
        v = np.where(live, vs * np.exp2(d), v)
        used = used + d
        with np.errstate(divide="ignore", invalid="ignore"):
            pa = np.where(live, k / v, 0.0)  # accept: the value read is < k
        m1 = m1 + np.where(live, reach * pa * used, 0.0)
        m2 = m2 + np.where(live, reach * pa * used * used, 0.0)
        reach = np.where(live, reach * (1 - pa), 0.0)
        v = np.where(live, v - k, v)
        live = live & (reach > 1e-30)
    return m1, np.maximum(m2 - m1 * m1, 0.0)


class _Prefix:
    """Prefix sums of E and Var of draw costs for ranges 1..K."""

    def __init__(self, K: int):
        ks = np.arange(1, K + 1, dtype=np.float64)
        e, v = fdr_moments(ks)
        self.E = np.concatenate([[0.0], np.cumsum(e)])  # E[j] = sum_{k=1..j}
        self.V = np.concatenate([[0.0], np.cumsum(v)])

    def sum_e(self, a, b):
        """sum of E over ranges a..b inclusive (empty if a > b)."""
        a = np.asarray(a)
        return np.where(a <= b, self.E[b] - self.E[np.minimum(a, b + 1) - 1], 0.0)

    def sum_v(self, a, b):
        a = np.asarray(a)
        return np.where(a <= b, self.V[b] - self.V[np.minimum(a, b + 1) - 1], 0.0)


def merge_moments(n1: int, n2: int, pre: _Prefix):
    """(E, Var) of the bits of one Merge of sizes n1, n2 (Lemma 2's sum)."""
    n = n1 + n2
    m1 = 0.0
    m2 = 0.0
    for a, b in ((n1, n2), (n2, n1)):
        # break on the (a+1)-th draw of one side after i draws of the other
        i = np.arange(0, b + 1, dtype=np.int64)
        logp = gammaln(a + i + 1) - gammaln(a + 1) - gammaln(i + 1) - (a + 1 + i) * math.log(2.0)
        p = np.exp(logp)
        P = a + i
        flips = P + 1.0
        se = pre.sum_e(P + 1, n)
        sv = pre.sum_v(P + 1, n)
        m1 += float(np.sum(p * (flips + se)))
        m2 += float(np.sum(p * ((flips + se) ** 2 + sv)))
    return m1, max(m2 - m1 * m1, 0.0)


def shuffle_moments(n: int, cutoff: int):
    """(E, Var) of the total bits of MergeShuffle(n, cutoff)."""
    if n <= 1:
        return 0.0, 0.0
    c = 0
    while (n >> c) > cutoff:
        c += 1
    q = 1 << c
    pre = _Prefix(n)
    E = 0.0
    V = 0.0
    bounds = [(n * i) >> c for i in range(q + 1)]
    # leaves: Fisher-Yates draws of ranges 2..b
    sizes = np.diff(np.asarray(bounds, dtype=np.int64))
    for b, cnt in zip(*np.unique(sizes, return_counts=True)):
        E += cnt * float(pre.sum_e(2, int(b)))
        V += cnt * float(pre.sum_v(2, int(b)))
    cache = {}
    for L in range(1, c + 1):
        p = 1 << (L - 1)
        for i in range(0, q, 2 * p):
            n1 = bounds[i + p] - bounds[i]
            n2 = bounds[i + 2 * p] - bounds[i + p]
            key = (n1, n2)
            if key not in cache:
                cache[key] = merge_moments(n1, n2, pre)
            e, v = cache[key]
            E += e
            V += v
    return E, V


def fisher_yates_moments(n: int):
    """(E, Var) of the bits of Algorithm 1 on n elements (ranges 2..n)."""
    pre = _Prefix(n)
    return float(pre.sum_e(2, n)), float(pre.sum_v(2, n))
