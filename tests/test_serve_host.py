"""Host-side checks of the request loop: admission policy and loop accounting
with a simulated clock and executor (no GPU)."""

import collections

import numpy as np
import pytest

from paper_1510_04331_amd.serve import Admission, Request, run


def _req(rid, arrival, T, N):
    z = np.zeros(T)
    return Request(rid=rid, arrival=arrival, T=T, N=N, dx=z, dy=z, parang=z)


def _bytes(group):
    return sum(r.cube_bytes for r in group) + (1 << 20) * bool(group)


def test_admission_fifo_budget_and_slots():
    adm = Admission(budget_bytes=10 << 20, slots=2, max_batch=3, group_bytes=_bytes)
    # 1 MiB cubes: T=4, N=256 -> 1 MiB each
    w = collections.deque(_req(i, 0.0, 4, 256) for i in range(10))
    groups = adm.admit(w, used_bytes=0, free_slots=2)
    assert [len(g) for g, _, _ in groups] == [3, 3]              # max_batch per slot, one group per slot
    assert [r.rid for g, _, _ in groups for r in g] == list(range(6))  # first come, first served
    assert sum(b for _, b, _ in groups) <= 10 << 20
    assert [r.rid for r in w] == list(range(6, 10))


def test_admission_head_of_line_not_overtaken():
    adm = Admission(budget_bytes=(8 << 20) - 1, slots=4, max_batch=4, group_bytes=_bytes)
    big = _req(0, 0.0, 24, 256)          # 6 MiB + 1 MiB workspace
    small = _req(1, 0.0, 4, 256)
    w = collections.deque([big, small])
    got = adm.admit(w, used_bytes=2 << 20, free_slots=4)    # big does not fit next to 2 MiB in use
    assert got == [] and list(w) == [big, small]
    got = adm.admit(w, used_bytes=0, free_slots=4)
    assert [r.rid for g, _, _ in got for r in g] == [0]      # small would push the pair over budget
    assert [r.rid for r in w] == [1]


def _cost(r):
    return r.T * r.N * r.N * 1e-6


def test_admission_large_requests_one_at_a_time_with_backfill():
    adm = Admission(budget_bytes=4 << 30, slots=4, max_batch=4, group_bytes=_bytes, cost=_cost, big_cost=100.0)
    b0, b1 = _req(0, 0.0, 64, 2048), _req(1, 0.0, 64, 2048)      # cost 268: large
    s2, s3 = _req(2, 0.0, 8, 64), _req(3, 0.0, 8, 64)            # small
    w = collections.deque([b0, b1, s2, s3])
    got = adm.admit(w, used_bytes=0, free_slots=4)
    # b0 starts alone; b1 must wait for it; the small ones backfill as one group
    assert [([r.rid for r in g], big) for g, _, big in got] == [([0], True), ([2, 3], False)]
    assert list(w) == [b1]
    got = adm.admit(w, used_bytes=0, free_slots=2, big_inflight=1)
    assert got == [] and list(w) == [b1]
    got = adm.admit(w, used_bytes=0, free_slots=2, big_inflight=0)
    assert [([r.rid for r in g], big) for g, _, big in got] == [([1], True)]
    # a small request never overtakes a large one that could start
    w = collections.deque([_req(4, 0.0, 64, 2048), _req(5, 0.0, 8, 64)])
    got = adm.admit(w, used_bytes=(4 << 30) - (1 << 20), free_slots=4)
    assert got == [] and [r.rid for r in w] == [4, 5]


def test_admission_rejects_oversized_request():
    adm = Admission(budget_bytes=4 << 20, slots=1, max_batch=1, group_bytes=_bytes)
    with pytest.raises(ValueError):
        adm.check(_req(0, 0.0, 64, 256))
    with pytest.raises(ValueError):
        Admission(budget_bytes=0, slots=1, max_batch=1, group_bytes=_bytes)


class _Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class _FakeExecutor:
    """Each group finishes a fixed time after its launch, proportional to its
    pixels."""

    def __init__(self, clock, rate=1e9):
        self.clock = clock
        self.rate = rate
        self.live = []
        self.launched = []

    def launch(self, group, slot):
        h = {"end": self.clock() + sum(r.T * r.N * r.N for r in group) / self.rate, "group": group,
             "slot": slot}
        self.live.append(h)
        self.launched.append([r.rid for r in group])
        return h

    def done(self, h):
        return self.clock() >= h["end"]

    def release(self, h):
        self.live.remove(h)
        return [("final", r.rid) for r in h["group"]]


def test_loop_accounting_with_simulated_clock():
    clk = _Clock()
    rng = np.random.default_rng(3)
    arr = np.cumsum(rng.exponential(1 / 50.0, size=40))
    reqs = [_req(i, float(a), int(rng.integers(8, 64)), int(rng.choice([64, 128, 256]))) for i, a in enumerate(arr)]
    budget = 24 << 20
    adm = Admission(budget_bytes=budget, slots=3, max_batch=4, group_bytes=_bytes)
    ex = _FakeExecutor(clk, rate=2e8)
    st = run(reqs, ex, adm, clock=clk, sleep=clk.sleep)
    assert st.n == 40 and len(st.latencies_s) == 40
    for r in reqs:
        assert r.final == ("final", r.rid)
        assert r.arrival <= r.admitted <= r.done
        assert r.latency >= r.T * r.N * r.N / 2e8 - 1e-9   # at least its own run time
    order = [rid for g in ex.launched for rid in g]
    assert order == sorted(order)                          # all small: admitted in arrival order
    assert st.max_used_bytes <= budget
    assert 1 <= st.max_inflight <= 3
    s = st.summary()
    assert s["latency_ms"]["p50"] <= s["latency_ms"]["p99"] <= s["latency_ms"]["max"]
    assert s["frames"] == sum(r.T for r in reqs)


def test_loop_overlaps_when_requests_pile_up():
    clk = _Clock()
    reqs = [_req(i, 0.001 * i, 32, 128) for i in range(12)]
    adm = Admission(budget_bytes=64 << 20, slots=4, max_batch=2, group_bytes=_bytes)
    st = run(reqs, _FakeExecutor(clk, rate=1e7), adm, clock=clk, sleep=clk.sleep)
    assert st.max_inflight >= 2         # later arrivals were admitted while earlier groups ran
    assert all(r.done is not None for r in reqs)


def test_loop_large_requests_never_overlap_each_other():
    clk = _Clock()
    rng = np.random.default_rng(5)
    reqs = [_req(i, 0.002 * i, int(rng.integers(16, 64)), int(rng.choice([64, 1024]))) for i in range(30)]
    adm = Admission(budget_bytes=1 << 32, slots=4, max_batch=4, group_bytes=_bytes, cost=_cost, big_cost=10.0)
    ex = _FakeExecutor(clk, rate=1e9)
    live_big = []

    class Watch(_FakeExecutor):
        def launch(self, group, slot):
            h = super().launch(group, slot)
            if adm.is_big(group[0]):
                assert len(group) == 1
                assert not any(not self.done(x) for x in live_big)   # no other large one still running
                live_big.append(h)
            return h
    ex = Watch(clk, rate=1e9)
    st = run(reqs, ex, adm, clock=clk, sleep=clk.sleep)
    assert all(r.done is not None for r in reqs) and len(live_big) == sum(r.N == 1024 for r in reqs)
    assert st.max_inflight >= 2
