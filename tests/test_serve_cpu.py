"""Serving loop on the CPU: scheduling, continuous batching, HBM admission and
latency accounting, with a mock executor standing in for the GPU."""
import numpy as np
import pytest

from fio_synth import gaussian_complex, serving_mix
from paper_2105_02995_amd.serve import (MockExecutor, Scheduler, ServeRequest, latency_stats,
                                        throughput)


def _key(i):
    return (1, 1024 * (1 + i % 3), "1d_ex1", 1e-6)


def _requests(count, rate, seed=0, max_rhs=8, keys=3):
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, count))
    out = []
    for j in range(count):
        k = _key(int(rng.integers(keys)))
        nr = int(rng.integers(1, max_rhs + 1))
        out.append(ServeRequest(j, k, float(t[j]), gaussian_complex((16, nr), 100 + j)))
    return out


def _transform(key, u):
    return u * (1.0 + key[1] / 1024.0)  # a per-key linear map, columnwise


def test_every_request_gets_its_own_columns_back():
    ex = MockExecutor(cost=lambda key, nr: 0.01 + 1e-4 * nr, transform=_transform)
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=32)
    for k in {_key(i) for i in range(3)}:
        assert s.register(k)
    reqs = _requests(200, rate=500.0)
    done = s.run(reqs)
    assert len(done) == 200
    for r in done:
        np.testing.assert_array_equal(r.result, _transform(r.key, r.u))
        assert r.done >= r.start >= r.arrival


def test_requests_arriving_during_a_batch_are_merged_into_the_next():
    ex = MockExecutor(cost=lambda key, nr: 0.05)
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=1024)
    s.register(_key(0))
    reqs = [ServeRequest(j, _key(0), 0.001 * j, gaussian_complex((8, 2), j)) for j in range(100)]
    s.run(reqs)
    # 100 requests over 0.1 s with 50 ms batches: a handful of batches, not 100
    assert s.batches_started <= 5
    assert len(s.finished) == 100


def test_batch_never_exceeds_max_columns():
    sizes = []

    class Ex(MockExecutor):
        def start(self, batch, now):
            sizes.append((batch.nrhs, len(batch.requests)))
            return super().start(batch, now)

    ex = Ex(cost=lambda key, nr: 0.01)
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=10)
    s.register(_key(0))
    reqs = [ServeRequest(j, _key(0), 0.0, gaussian_complex((4, 3 if j != 5 else 10), j)) for j in range(12)]
    done = s.run(reqs)
    assert len(done) == 12
    assert all(n <= 10 for n, k in sizes)
    assert any(n == 10 and k == 1 for n, k in sizes)


def test_hbm_admission_bounds_inflight_bytes_and_refuses_oversized_keys():
    inflight = []
    per_rhs = 1000

    class Ex(MockExecutor):
        def start(self, batch, now):
            inflight.append(sched.inflight_bytes)  # counts every batch admitted so far, this one included
            return super().start(batch, now)

    ex = Ex(cost=lambda key, nr: 0.02, factor_bytes=lambda key: 100_000 if key[0] == 2 else 10_000,
            ws_bytes_per_rhs=lambda key: per_rhs)
    sched = Scheduler(ex, hbm_budget=10_000 * 3 + 40 * per_rhs, max_batch_rhs=16)
    for i in range(3):
        assert sched.register(_key(i))
    assert not sched.register((2, 256, "2d_radon", 1e-4))  # would exceed the budget
    sched.run(_requests(300, rate=2000.0, max_rhs=8))
    assert len(sched.finished) == 300
    assert max(inflight) <= 40 * per_rhs
    assert sched.rejected_keys == [(2, 256, "2d_radon", 1e-4)]


def test_different_keys_overlap_and_latency_accounting():
    ex = MockExecutor(cost=lambda key, nr: 0.03)
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=64)
    for i in range(3):
        s.register(_key(i))
    done = s.run(_requests(150, rate=1000.0, keys=3))
    assert s.peak_inflight >= 2
    st = latency_stats(done)
    assert st["p50_ms"] >= 30.0 - 1e-6  # at least one batch duration
    assert st["p99_ms"] >= st["p50_ms"]
    assert throughput(done) > 0


def test_serving_mix_generator_shapes():
    mix = serving_mix(50, rate=10.0, seed=2000)
    assert len(mix) == 50
    assert all(m.nrhs >= 1 and m.nrhs <= 32 for m in mix)
    assert {m.d for m in mix} <= {1, 2}
    arr = [m.arrival for m in mix]
    assert arr == sorted(arr)


def test_oldest_request_first_with_more_keys_than_slots():
    """Twelve keys share four slots: dispatch goes by the arrival of each queue's
    head, so no key starves behind keys that were submitted first, and the oldest
    request never waits longer than a few batch durations."""
    cost = 0.01
    ex = MockExecutor(cost=lambda key, nr: cost)
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=8, max_inflight=4)
    keys = [(1, 1024 * (i + 1), "1d_ex1", 1e-6) for i in range(12)]
    for k in keys:
        assert s.register(k)
    rng = np.random.default_rng(3)
    reqs = []
    t = 0.0
    for j in range(600):  # offered load just under the four slots' capacity
        t += rng.exponential(cost / 3.6)
        reqs.append(ServeRequest(j, keys[j % 12], t, np.zeros((4, 8))))
    done = s.run(reqs)
    assert len(done) == 600
    waits = np.array([r.start - r.arrival for r in done])
    # a request waits at most for the batches ahead of it in arrival order: with
    # 12 keys over 4 slots that is about 3 rounds of batches
    assert waits.max() < 6 * cost, waits.max()
    assert s.peak_inflight <= 4


def test_scheduler_never_exceeds_executor_concurrency():
    ex = MockExecutor(cost=lambda key, nr: 0.01)
    ex.max_concurrent = 2
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=8, max_inflight=8)
    assert s.max_inflight == 2
    for i in range(5):
        assert s.register(_key(i))
    done = s.run(_requests(50, rate=1e4, keys=5, max_rhs=4))
    assert len(done) == 50 and s.peak_inflight <= 2


def test_oversized_request_is_refused_before_anything_runs():
    ex = MockExecutor(cost=lambda key, nr: 0.01)
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=16)
    assert s.register(_key(0))
    ok = ServeRequest(0, _key(0), 0.0, np.zeros((4, 3)))
    big = ServeRequest(1, _key(0), 0.0, np.zeros((4, 17)))
    with pytest.raises(ValueError):
        s.run([ok, big])
    assert s.batches_started == 0
    with pytest.raises(ValueError):
        s.submit(ServeRequest(2, _key(0), 0.0, np.zeros((4, 0))))


def test_multi_instance_groups_hold_batches_of_similar_work():
    """The GPU executor groups batches admitted together into multi-instance solves
    only when their estimated work (butterfly nonzeros x padded columns) is within a
    factor GROUP_SPREAD; a much larger batch runs on its own, and no group exceeds
    MULTI_MAX instances."""
    from paper_2105_02995_amd.serve import Batch, GpuExecutor

    class Fake(GpuExecutor):
        def __init__(self, stats):  # no device: only the grouping logic
            self.stats = stats
            self.max_batch_rhs = 256

    nnz = {("k%d" % i,): 1e6 * (1 + i % 3) for i in range(10)}
    nnz[("big",)] = 1e9
    ex = Fake({k: {"bf_nnz": v} for k, v in nnz.items()})
    batches = [Batch(k, [], 16, 0) for k in nnz]
    groups = ex._groups(batches)
    assert sorted(i for g in groups for i in g) == list(range(len(batches)))
    for g in groups:
        assert len(g) <= ex.MULTI_MAX
        w = [ex._work(batches[i]) for i in g]
        assert max(w) <= ex.GROUP_SPREAD * min(w)
    big = [g for g in groups if any(batches[i].key == ("big",) for i in g)]
    assert len(big) == 1 and len(big[0]) == 1


def test_cancel_withdraws_queued_and_running_requests():
    """A queued request leaves its queue at once; a running one is dropped when its
    batch completes; the other requests are served as usual."""
    ex = MockExecutor(cost=lambda key, nr: 0.05, transform=_transform)
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=64)
    k = _key(0)
    s.register(k)
    r = [ServeRequest(j, k, 0.0, gaussian_complex((16, 2), 500 + j)) for j in range(4)]
    s.submit(r[0])
    s.step(ex.clock())                 # r0 runs
    for q in r[1:]:
        s.submit(q)                    # r1..r3 wait for the key's slot
    assert s.cancel(1)                 # queued
    assert s.cancel(0)                 # running
    assert not s.cancel(99)
    while not s.idle():
        ex.wait()
        s.step(ex.clock())
    assert sorted(q.rid for q in s.finished) == [2, 3]
    assert sorted(q.rid for q in s.cancelled) == [0, 1]
    for q in s.cancelled:
        assert q.result is None and q.error == "cancelled"
    for q in s.finished:
        np.testing.assert_array_equal(q.result, _transform(k, q.u))
    assert not s.cancel(2)             # done: nothing to withdraw
    assert s.inflight_bytes == 0


def test_executor_failure_fails_only_that_batch():
    """The executor raising for one batch (a modelled allocation failure on its
    second start) fails that batch's requests with the error; the loop serves every
    other request and releases the batch's memory."""
    ex = MockExecutor(cost=lambda key, nr: 0.01, transform=_transform, ws_bytes_per_rhs=lambda key: 1000,
                      fail_starts={1})
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=32)
    for k in {_key(i) for i in range(3)}:
        s.register(k)
    reqs = _requests(60, rate=2000.0, seed=3)
    s.run(reqs)
    assert len(s.finished) + len(s.failed) == 60
    assert s.failed and all("MemoryError" in q.error and q.result is None for q in s.failed)
    assert len({q.key for q in s.failed}) == 1       # one batch: one key
    for q in s.finished:
        np.testing.assert_array_equal(q.result, _transform(q.key, q.u))
    assert s.inflight_bytes == 0 and not s.running


def test_per_key_batch_cap_bounds_large_keys_only():
    """The executor's per-key column cap (a bound on one batch's device time): the
    capped key's batches stay within it, a request wider than the cap still runs
    (alone), the other key batches up to max_batch_rhs, and every request is served."""
    sizes = {}
    big, small = _key(0), _key(1)

    class Ex(MockExecutor):
        def start(self, batch, now):
            sizes.setdefault(batch.key, []).append((batch.nrhs, len(batch.requests)))
            return super().start(batch, now)

    ex = Ex(cost=lambda key, nr: 0.02, transform=_transform, batch_caps={big: 8})
    s = Scheduler(ex, hbm_budget=1 << 40, max_batch_rhs=64)
    assert s.register(big) and s.register(small)
    reqs = [ServeRequest(j, big if j % 2 == 0 else small, 0.0,
                         gaussian_complex((4, 12 if j == 4 else 3), 500 + j)) for j in range(40)]
    done = s.run(reqs)
    assert len(done) == 40
    for r in done:
        np.testing.assert_array_equal(r.result, _transform(r.key, r.u))
    assert all(n <= 8 or k == 1 for n, k in sizes[big])
    assert any(n == 12 and k == 1 for n, k in sizes[big])
    assert max(n for n, _ in sizes[small]) > 8
