"""The serving loop's scheduling on a simulated executor (no GPU).

The executor completes a batch after a time proportional to its elements
plus a fixed launch cost, in simulated time, and models the payload pool as
a byte budget.  Checked: every request is served or (only if it can never
fit) refused; the HBM budget is never exceeded; at most max_inflight batches
are on the device; requests are admitted and launched in arrival order;
requests that arrive while batches run are batched together (continuous
batching); latencies are arrival-to-completion.
"""
import random

import pytest

from paper_1508_03167_amd.serve import Request, Server, percentile


class SimClock:
    def __init__(self):
        self.t = 0.0

    def now(self):
        return self.t

    def wait(self, dt):
        self.t += max(dt, 1e-6)


class FakeExecutor:
    poll_is_cheap = False

    def __init__(self, clock, pool_bytes, rate=1e9, launch_cost=20e-6, scratch=lambda n, eb: n * eb + 4096):
        self.clock = clock
        self.pool = pool_bytes
        self.used = 0
        self.rate = rate
        self.launch_cost = launch_cost
        self.scratch = scratch
        self.inflight = 0
        self.max_seen = 0
        self.launches = []

    def footprint(self, n, eb):
        return n * eb + self.scratch(n, eb)

    def acquire(self, r):
        if self.used + r.n * r.elem_bytes > self.pool:
            return None
        self.used += r.n * r.elem_bytes
        return 0

    def release(self, r):
        self.used -= r.n * r.elem_bytes

    def launch(self, reqs, slot):
        self.inflight += 1
        self.max_seen = max(self.max_seen, self.inflight)
        self.launches.append([r.rid for r in reqs])
        return [self.clock.now() + self.launch_cost + sum(r.n for r in reqs) / self.rate, False]

    def done(self, h):
        if not h[1] and self.clock.now() >= h[0]:
            h[1] = True
            self.inflight -= 1
        return h[1]


def _requests(count, seed, max_n=1 << 22, rate=2000.0):
    rnd = random.Random(seed)
    t = 0.0
    out = []
    for i in range(count):
        t += rnd.expovariate(rate)
        n = int(2 ** (10 + rnd.random() * (max_n.bit_length() - 11)))
        out.append(Request(i, n, rnd.choice((4, 8)), 5 + i, t))
    return out


def _run(reqs, budget, inflight=2, pool=None, max_batch_elems=None, **kw):
    clock = SimClock()
    ex = FakeExecutor(clock, pool if pool is not None else budget, **kw)
    srv = Server(ex, budget, max_inflight=inflight, max_batch_elems=max_batch_elems)
    done, rej = srv.run(reqs, clock.now, clock.wait)
    return srv, ex, done, rej


def test_every_request_is_served_in_arrival_order():
    reqs = _requests(500, 1)
    srv, ex, done, rej = _run(reqs, budget=8 << 30)
    assert not rej and len(done) == 500
    by_arrival = sorted(done, key=lambda r: r.arrival)
    adm = [r.admitted for r in by_arrival]
    lau = [r.launched for r in by_arrival]
    assert adm == sorted(adm) and lau == sorted(lau)
    for r in done:
        assert r.arrival <= r.admitted <= r.launched <= r.done
        assert r.latency == pytest.approx(r.done - r.arrival)


def test_budget_is_never_exceeded_and_inflight_is_bounded():
    reqs = _requests(400, 2, rate=20000.0)
    budget = 512 << 20
    srv, ex, done, rej = _run(reqs, budget=budget, inflight=3)
    assert len(done) + len(rej) == 400
    assert srv.peak_used <= budget
    assert ex.max_seen <= 3
    assert srv.used == 0 and ex.used == 0


def test_oversize_requests_are_refused_at_once():
    reqs = [Request(0, 1000, 4, 1, 0.0), Request(1, 1 << 28, 8, 2, 0.0), Request(2, 5000, 4, 3, 0.001)]
    srv, ex, done, rej = _run(reqs, budget=1 << 24)
    assert [r.rid for r in rej] == [1] and rej[0].rejected
    assert sorted(r.rid for r in done) == [0, 2]


def test_arrivals_during_a_batch_are_batched_together():
    # a long first request keeps both slots busy; the many small requests
    # that arrive meanwhile go out in a few batches, not one launch each
    reqs = [Request(0, 1 << 26, 4, 1, 0.0), Request(1, 1 << 26, 4, 2, 0.0)]
    reqs += [Request(2 + i, 2048, 4, 10 + i, 1e-3 + i * 1e-6) for i in range(300)]
    srv, ex, done, rej = _run(reqs, budget=8 << 30, rate=1e9)
    assert len(done) == 302
    assert srv.batches <= 6
    assert max(len(b) for b in ex.launches) >= 100


def test_head_of_line_request_waits_for_space():
    # the second request needs the whole budget: it waits until the first is
    # done, and later small requests do not overtake it
    budget = 1 << 20
    scratch = lambda n, eb: 0  # noqa: E731
    reqs = [Request(0, 100000, 4, 1, 0.0), Request(1, 200000, 4, 2, 1e-6), Request(2, 100, 4, 3, 2e-6)]
    srv, ex, done, rej = _run(reqs, budget=budget, scratch=scratch)
    r = {q.rid: q for q in done}
    assert r[1].admitted >= r[0].done
    assert r[2].admitted >= r[1].admitted


def test_percentile():
    assert percentile([1, 2, 3, 4, 5], 50) == 3
    assert percentile([0, 10], 99) == pytest.approx(9.9)


def test_element_cap_keeps_small_requests_out_of_large_batches():
    # with a cap, a large request is launched alone and the small requests
    # that follow it go out in batches of their own
    reqs = [Request(0, 1 << 24, 4, 1, 0.0)]
    reqs += [Request(1 + i, 1000, 4, 10 + i, 0.0) for i in range(50)]
    reqs += [Request(51, 1 << 24, 4, 2, 0.0)]
    srv, ex, done, rej = _run(reqs, budget=8 << 30, inflight=3, max_batch_elems=1 << 20)
    assert len(done) == 52
    assert ex.launches[0] == [0]
    assert ex.launches[1] == list(range(1, 51))
    assert ex.launches[2] == [51]
    for b in ex.launches:
        assert len(b) == 1 or sum(1000 for _ in b) <= 1 << 20


def test_large_requests_take_turns_and_small_ones_pass_them():
    # two large requests arrive together with small ones: with one large
    # request on the device at a time, the second large one waits for the
    # first to finish while the small ones behind it are launched
    reqs = [Request(0, 1 << 24, 4, 1, 0.0), Request(1, 1 << 24, 4, 2, 0.0)]
    reqs += [Request(2 + i, 1000, 4, 10 + i, 0.0) for i in range(20)]
    clock = SimClock()
    ex = FakeExecutor(clock, 8 << 30)
    srv = Server(ex, 8 << 30, max_inflight=3, max_batch_elems=1 << 20, max_large_inflight=1)
    done, rej = srv.run(reqs, clock.now, clock.wait)
    r = {q.rid: q for q in done}
    assert len(done) == 22 and not rej
    assert r[1].launched >= r[0].done
    assert all(r[2 + i].launched < r[1].launched for i in range(20))
    assert ex.launches[0] == [0]
