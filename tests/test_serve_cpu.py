"""Serving scheduler on the CPU with a fake executor and a deterministic clock:
bucketing, FIFO order, continuous batching (overlap), HBM-budget admission,
rejection of oversized / unsupported requests and failure isolation."""
import numpy as np
import pytest

import synth
from paper_1811_03882_amd.serve import (Executor, PoolAllocator, Request, Scheduler, device_overlap, make_requests,
                                        next_pow2)


class Clock:
    """Advances by `dt` seconds on every read: the scheduler loop drives time."""

    def __init__(self, dt=1e-5):
        self.t = 0.0
        self.dt = dt

    def __call__(self):
        self.t += self.dt
        return self.t


class FakeExecutor(Executor):
    def __init__(self, clock, n_slots=4, per_image_s=2e-4, fail_ids=(), launch_fail_ids=()):
        self.clock = clock
        self.n_slots = n_slots
        self.per_image_s = per_image_s
        self.fail_ids = set(fail_ids)
        self.launch_fail_ids = set(launch_fail_ids)
        self.log = []  # (launch time, done time, slot, size, ids)

    def batch_bytes(self, batch, size):
        return batch * size * size * 100

    def launch(self, slot, reqs, padded, size, offset):
        if any(r.rid in self.launch_fail_ids for r in reqs):
            raise RuntimeError("injected launch failure")
        t = self.clock()
        done = t + 1e-4 + self.per_image_s * padded * (size / 160.0) ** 2
        self.log.append((t, done, slot, size, [r.rid for r in reqs]))
        return (done, [r.rid for r in reqs], size)

    def done(self, h):
        return self.clock() >= h[0]

    def finish(self, h, reqs):
        if any(r.rid in self.fail_ids for r in reqs):
            raise RuntimeError("injected execution failure")
        for r in reqs:
            r.output = np.full(3, float(r.rid))


def _trace(n=400, rate=2000.0, seed=3):
    return make_requests(synth.serving_trace(n, rate, seed))


def test_pool_allocator_first_fit_and_coalesce():
    p = PoolAllocator(4096)
    a = p.alloc(1000)
    b = p.alloc(1000)
    c = p.alloc(1000)
    assert (a, b, c) == (0, 1024, 2048)
    assert p.alloc(2000) is None
    p.free(b, 1000)
    assert p.alloc(900) == 1024
    p.free(1024, 900)
    p.free(a, 1000)
    p.free(c, 1000)
    assert p.in_use == 0
    assert p.alloc(4096) == 0


def test_next_pow2():
    assert [next_pow2(n) for n in (1, 2, 3, 5, 33, 64)] == [1, 2, 4, 8, 64, 64]


def test_all_requests_complete_with_their_own_outputs():
    clk = Clock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, budget_bytes=1 << 34, sizes=(160, 224, 320, 416, 608), max_batch=64, clock=clk)
    reqs = _trace()
    st = sch.run(reqs)
    assert st.completed == len(reqs) and st.failed == 0 and st.rejected == 0
    for r in reqs:
        assert r.output is not None and r.output[0] == r.rid
        assert r.latency > 0
    # every batch holds one resolution only, and never more than max_batch requests
    for t, d, slot, size, ids in ex.log:
        assert len(ids) <= 64
        assert {reqs[i].size for i in ids} == {size}


def test_fifo_within_a_bucket():
    clk = Clock()
    ex = FakeExecutor(clk, n_slots=2)
    sch = Scheduler(ex, budget_bytes=1 << 34, sizes=(160, 224, 320, 416, 608), clock=clk)
    reqs = _trace(300)
    sch.run(reqs)
    launched = {}
    for order, (t, d, slot, size, ids) in enumerate(ex.log):
        for i in ids:
            launched[i] = order
    for s in (160, 224, 320, 416, 608):
        same = sorted((r.arrival, launched[r.rid]) for r in reqs if r.size == s)
        orders = [o for _, o in same]
        assert orders == sorted(orders)


def test_continuous_batching_overlaps_in_flight_batches():
    clk = Clock()
    ex = FakeExecutor(clk, n_slots=4, per_image_s=2e-3)  # slow device: batches overlap
    sch = Scheduler(ex, budget_bytes=1 << 34, sizes=(160, 224, 320, 416, 608), clock=clk)
    sch.run(_trace(300))
    assert sch.max_inflight >= 2
    # some batch was launched while an earlier one was still running
    log = sorted(ex.log)
    assert any(log[k][0] < log[k - 1][1] for k in range(1, len(log)))


def test_budget_admission_limits_concurrency():
    clk = Clock()
    ex = FakeExecutor(clk, n_slots=8, per_image_s=2e-3)
    one_batch = ex.batch_bytes(64, 608)
    sch = Scheduler(ex, budget_bytes=one_batch, sizes=(608,), clock=clk)
    reqs = [Request(i, 608, 0.0) for i in range(200)]
    st = sch.run(reqs)
    assert st.completed == 200
    assert sch.max_inflight == 1  # the budget admits one batch of 64 at a time
    clk2 = Clock()
    ex2 = FakeExecutor(clk2, n_slots=8, per_image_s=2e-3)
    sch2 = Scheduler(ex2, budget_bytes=8 * one_batch, sizes=(608,), clock=clk2)
    sch2.run([Request(i, 608, 0.0) for i in range(200)])
    assert sch2.max_inflight > 1


def test_oversized_and_unsupported_requests_are_rejected_others_served():
    clk = Clock()
    ex = FakeExecutor(clk)
    sch = Scheduler(ex, budget_bytes=ex.batch_bytes(2, 320), sizes=(160, 320, 608), clock=clk)
    reqs = [Request(0, 608, 0.0), Request(1, 160, 0.0), Request(2, 999, 0.0), Request(3, 320, 0.0)]
    st = sch.run(reqs)
    assert st.rejected == 2 and st.completed == 2
    assert reqs[0].error and reqs[2].error
    assert reqs[1].output is not None and reqs[3].output is not None


def test_failure_is_isolated_to_its_batch():
    clk = Clock()
    ex = FakeExecutor(clk, n_slots=2, fail_ids={5}, launch_fail_ids={50})
    sch = Scheduler(ex, budget_bytes=1 << 34, sizes=(160, 224, 320, 416, 608), clock=clk)
    reqs = _trace(200)
    st = sch.run(reqs)
    bad = [r for r in reqs if r.error]
    assert any(r.rid == 5 for r in bad) and any(r.rid == 50 for r in bad)
    assert st.failed == len(bad)
    assert st.completed == len(reqs) - len(bad) > 150


def test_plain_fifo_path_batch_one():
    clk = Clock()
    ex = FakeExecutor(clk, n_slots=1)
    sch = Scheduler(ex, budget_bytes=1 << 34, sizes=(160, 224, 320, 416, 608), max_batch=1,
                    pad_pow2=False, bucketed=False, clock=clk)
    reqs = _trace(100)
    st = sch.run(reqs)
    assert st.completed == 100 and st.mean_batch == 1.0 and sch.max_inflight == 1
    order = [ids[0] for _, _, _, _, ids in ex.log]
    assert order == sorted(order)  # arrival order (ids follow the trace order)


def test_padded_batch_over_budget_on_an_idle_pool_shrinks_instead_of_waiting():
    # the budget holds a padded batch of 2 at S=320: three requests pad to 4,
    # which never fits; with nothing in flight the scheduler must split them
    clk = Clock()
    ex = FakeExecutor(clk, n_slots=4)
    sch = Scheduler(ex, budget_bytes=ex.batch_bytes(2, 320), sizes=(320,), clock=clk)
    reqs = [Request(i, 320, 0.0) for i in range(3)]
    st = sch.run(reqs)
    assert st.completed == 3 and st.failed == 0 and st.rejected == 0
    assert sorted(len(ids) for _, _, _, _, ids in ex.log) == [1, 2]
    for r in reqs:
        assert r.output[0] == r.rid


def test_budget_of_one_image_serves_a_burst_one_by_one():
    clk = Clock()
    ex = FakeExecutor(clk, n_slots=2)
    sch = Scheduler(ex, budget_bytes=ex.batch_bytes(1, 608), sizes=(608,), clock=clk)
    st = sch.run([Request(i, 608, 0.0) for i in range(9)])
    assert st.completed == 9 and sch.max_inflight == 1
    assert all(len(ids) == 1 for _, _, _, _, ids in ex.log)


class _Ev:
    """Stand-in for a completed timing event: elapsed_time(other) = other.t - self.t (ms)."""

    def __init__(self, t):
        self.t = t

    def elapsed_time(self, other):
        return other.t - self.t


def test_device_overlap_from_event_intervals():
    ref = _Ev(0.0)
    # [1, 4], [2, 3], [3.5, 6], [8, 9]: busy 1..6 and 8..9 = 6 ms; two or more
    # in flight over [2, 3] and [3.5, 4] = 1.5 ms; interval sum 3 + 1 + 2.5 + 1 = 7.5
    iv = [(_Ev(1.0), _Ev(4.0), 1), (_Ev(2.0), _Ev(3.0), 1), (_Ev(3.5), _Ev(6.0), 1), (_Ev(8.0), _Ev(9.0), 1)]
    d = device_overlap(iv, ref)
    assert d["busy_ms"] == pytest.approx(6.0)
    assert d["sum_batch_ms"] == pytest.approx(7.5)
    assert d["mean_in_flight"] == pytest.approx(7.5 / 6.0)
    assert d["overlap_frac"] == pytest.approx(1.5 / 6.0)
    assert d["max_in_flight"] == 2
    # back to back (one ends where the next starts): no overlap
    d = device_overlap([(_Ev(0.0), _Ev(1.0), 1), (_Ev(1.0), _Ev(2.0), 1)], ref)
    assert d["overlap_frac"] == 0.0 and d["max_in_flight"] == 1 and d["busy_ms"] == pytest.approx(2.0)
    assert device_overlap([], ref)["busy_ms"] == 0.0
