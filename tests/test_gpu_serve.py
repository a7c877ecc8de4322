"""The continuous-batching server on the GPU: every result equals the oracle
and is bit-identical to the same request served alone; the budget holds."""
import threading
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def srvmod():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd.serve as serve

    return serve


def test_mix_equals_alone_and_oracle(srvmod, orc):
    sizes = W.request_sizes(48, 2**10, 2**19, seed=4)
    rng = np.random.default_rng(4)
    I = np.iinfo(np.int64)
    reqs = [rng.integers(I.min, I.max, int(s), dtype=np.int64, endpoint=True) for s in sizes]
    gaps = rng.exponential(0.002, len(reqs))
    futs = [None] * len(reqs)
    with srvmod.SortServer(hbm_budget=64 << 30, streams=3) as srv:
        def client(idx):
            for i in idx:
                time.sleep(gaps[i])
                futs[i] = srv.submit(reqs[i])

        ths = [threading.Thread(target=client, args=(list(range(c, len(reqs), 3)),)) for c in range(3)]
        for t in ths:
            t.start()
        for t in ths:
            t.join()
        mixed = [f.result(timeout=120) for f in futs]
        st = srv.stats()
    print("serving stats", st, flush=True)
    with srvmod.SortServer(hbm_budget=64 << 30, streams=1) as srv:
        alone = [srv.submit(r).result(timeout=120) for r in reqs]
    for r, m, a in zip(reqs, mixed, alone):
        assert np.array_equal(m, a)
        assert np.array_equal(m, orc.sort_keys(r))
    assert st["batches"] < len(reqs)  # requests were batched


def test_small_budget_blocks_admission(srvmod):
    import paper_2003_01216_amd as hs

    n = 1 << 18
    one = 8 * n + 16 + hs.scratch_bytes(hs.SEG_I64, n, 1)
    budget = int(1.5 * one)  # one request at a time
    rng = np.random.default_rng(5)
    reqs = [rng.integers(-(10**12), 10**12, n, dtype=np.int64) for _ in range(6)]
    with srvmod.SortServer(hbm_budget=budget, streams=3, max_batch_keys=n) as srv:
        res = [f.result(timeout=120) for f in [srv.submit(r) for r in reqs]]
        st = srv.stats()
    assert st["peak_in_flight_bytes"] <= budget
    for r, o in zip(reqs, res):
        assert np.array_equal(o, np.sort(r))


def test_oversized_request_rejected(srvmod):
    import paper_2003_01216_amd as hs

    with srvmod.SortServer(hbm_budget=1 << 20, streams=1) as srv:
        f = srv.submit(np.arange(1 << 18, dtype=np.int64))
        with pytest.raises(hs.HsortError) as e:
            f.result(timeout=30)
        assert e.value.code == hs.HSORT_ERR_BUDGET
        ok = srv.submit(np.array([3, 1, 2], np.int64)).result(timeout=30)
        assert ok.tolist() == [1, 2, 3]
