"""Scheduler logic of the continuous-batching server, on the CPU.

A fake executor stands in for the GPU: it sorts with the oracle, records
every batch it is handed and how many batches run at once, and sleeps to
keep batches in flight while others arrive.
"""
import threading
import time

import numpy as np
import pytest

import paper_2003_01216_amd.serve as serve
from paper_2003_01216_amd import HSORT_ERR_BUDGET, HsortError


class FakeExecutor:
    def __init__(self, orc, delay=0.02, per_key=8):
        self.orc = orc
        self.delay = delay
        self.per_key = per_key
        self.lock = threading.Lock()
        self.batches = []
        self.running = 0
        self.max_running = 0

    def batch_bytes(self, keys, nseg):
        return self.per_key * keys + 8 * (nseg + 1)

    def make_slot(self):
        return {}

    def run(self, slot, arrays):
        with self.lock:
            self.running += 1
            self.max_running = max(self.max_running, self.running)
            self.batches.append([int(a[0]) if a.size else -1 for a in arrays])
        time.sleep(self.delay)
        out = [self.orc.sort_keys(a) for a in arrays]
        with self.lock:
            self.running -= 1
        return out


def tagged(i, n, rng):
    """int64 request whose first key is its id (to follow it through batches)."""
    a = rng.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, n, dtype=np.int64, endpoint=True)
    a[0] = i
    return a


def test_results_alone_and_in_mix(orc):
    rng = np.random.default_rng(0)
    reqs = [tagged(i, int(rng.integers(1, 3000)), rng) for i in range(60)]
    ex = FakeExecutor(orc, delay=0.005)
    with serve.SortServer(hbm_budget=1 << 30, streams=3, executor=ex) as srv:
        futs = [srv.submit(r) for r in reqs]
        mixed = [f.result(timeout=60) for f in futs]
    alone = []
    for r in reqs:
        with serve.SortServer(hbm_budget=1 << 30, streams=1, executor=FakeExecutor(orc, 0)) as srv:
            alone.append(srv.submit(r).result(timeout=60))
    for r, m, a in zip(reqs, mixed, alone):
        assert np.array_equal(m, a) and np.array_equal(m, np.sort(r))
    assert max(len(b) for b in ex.batches) > 1  # requests were really batched


def test_budget_never_exceeded_and_admission_blocks(orc):
    rng = np.random.default_rng(1)
    ex = FakeExecutor(orc, delay=0.03)
    budget = 8 * 5000 + 64  # room for about one 5000-key batch
    with serve.SortServer(hbm_budget=budget, streams=4, executor=ex, max_batch_keys=1 << 20) as srv:
        futs = [srv.submit(tagged(i, 3000, rng)) for i in range(12)]
        for f in futs:
            f.result(timeout=60)
        st = srv.stats()
    assert st["peak_in_flight_bytes"] <= budget
    assert ex.max_running == 1  # the budget, not the 4 streams, limited concurrency
    assert all(len(b) == 1 for b in ex.batches)
    assert st["budget_waits"] > 0  # free workers found requests waiting and no budget


def test_oversized_request_is_rejected_others_proceed(orc):
    ex = FakeExecutor(orc, delay=0.0)
    with serve.SortServer(hbm_budget=8 * 1000 + 64, streams=2, executor=ex) as srv:
        big = srv.submit(np.arange(5000, dtype=np.int64))
        ok = srv.submit(np.arange(100, 0, -1, dtype=np.int64))
        with pytest.raises(HsortError) as e:
            big.result(timeout=10)
        assert e.value.code == HSORT_ERR_BUDGET
        assert np.array_equal(ok.result(timeout=10), np.arange(1, 101))


def test_fifo_admission(orc):
    rng = np.random.default_rng(2)
    ex = FakeExecutor(orc, delay=0.01)
    with serve.SortServer(hbm_budget=1 << 30, streams=2, executor=ex, max_batch_keys=2500) as srv:
        futs = [srv.submit(tagged(i, int(rng.integers(100, 1200)), rng)) for i in range(40)]
        for f in futs:
            f.result(timeout=60)
    taken = [i for b in ex.batches for i in b]
    # every batch is a prefix of what was waiting: ids are taken in submission order
    assert taken == sorted(taken) and sorted(taken) == list(range(40))


def _wait_running(ex, k, timeout=10.0):
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < timeout:
        with ex.lock:
            if ex.running >= k:
                return
        time.sleep(0.001)
    raise AssertionError(f"executor never reached {k} running batches")


def test_arrivals_during_flight_overlap(orc):
    rng = np.random.default_rng(3)
    ex = FakeExecutor(orc, delay=0.2)
    with serve.SortServer(hbm_budget=1 << 30, streams=2, executor=ex) as srv:
        futs = [srv.submit(tagged(0, 500, rng))]
        _wait_running(ex, 1)  # the first request is on one stream...
        futs.append(srv.submit(tagged(1, 500, rng)))
        _wait_running(ex, 2)  # ...the second on the other
        # both streams busy: these four wait and leave together in one batch
        futs += [srv.submit(tagged(i, 500, rng)) for i in range(2, 6)]
        for f in futs:
            f.result(timeout=60)
        st = srv.stats()
    assert ex.max_running == 2
    assert st["overlap_s"] > 0
    assert [2, 3, 4, 5] in ex.batches  # arrivals during flight were batched together


def test_close_drains_and_rejects_new(orc):
    ex = FakeExecutor(orc, delay=0.01)
    srv = serve.SortServer(hbm_budget=1 << 30, streams=2, executor=ex)
    futs = [srv.submit(np.arange(50, dtype=np.int64)[::-1].copy()) for _ in range(5)]
    srv.close()
    assert all(f.done() for f in futs)
    with pytest.raises(RuntimeError):
        srv.submit(np.arange(3, dtype=np.int64))


def test_executor_error_reaches_callers(orc):
    class Broken(FakeExecutor):
        def run(self, slot, arrays):
            raise HsortError(3, "device failure")

    with serve.SortServer(hbm_budget=1 << 30, streams=1, executor=Broken(orc)) as srv:
        f = srv.submit(np.arange(10, dtype=np.int64))
        with pytest.raises(HsortError):
            f.result(timeout=10)
        # the budget was released: a later request still gets admitted
        assert srv._in_flight_bytes == 0
