"""Per-kernel timing records (hsort_timing_enable / hsort_timing_read).

The benchmark's per-kernel figures come from these records: HIP events
around each group of launches on the sorting stream, and each group's
algorithmic bytes (a merge round's from the bucket table the sort leaves in
scratch: the keys of the buckets that still merge in that round).  Checked
on a plain int32 sort whose figures are known in advance -- every key in
one bucket of the three-digit rule, so that bucket holds n keys and needs
every merge round the host launches: one range, scatter and local-sort
launch with 4n, 8n and 8n bytes, one merge record per round with 8n bytes
each; no records while timing is off, and none from a call replayed as a
captured graph (graph mode, on a stream other than the null stream).
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    hs.load_library()
    hs.hsort_timing_enable(False)
    hs.hsort_timing_read()
    yield hs
    hs.hsort_timing_enable(False)
    hs.hsort_timing_read()
    hs.hsort_graph_mode(False)
    hs.hsort_graph_clear()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def merge_rounds(n, tile, fanin):
    runs, r, cover = -(-n // tile), 0, 1
    while cover < runs:
        cover *= fanin
        r += 1
    return r


def one_bucket_keys(n, seed):
    # u = k (no negative key), ten digits: floor(u / 10^7) = 100 for every key
    r = np.random.default_rng(seed)
    return r.integers(10**9, 10**9 + 10**6, n).astype(np.int32)


def sorted_once(hs, k, s):
    t = torch.from_numpy(k).cuda()
    hs.hsort_keys(t, scratch=s)
    torch.cuda.synchronize()
    return t


def test_records_of_a_plain_sort(hs):
    n = 2**20
    cfg = hs.hsort_get_config(hs.KEYS_I32, n=n)
    if cfg[5] != 4 or cfg[6] != 3:
        pytest.skip(f"the tuned table for 2^20 int32 is not fan-in 4 with three digits: {cfg}")
    rounds = merge_rounds(n, cfg[0], 4)
    say(f"timing records: n={n} cfg={cfg} rounds={rounds}")
    k = one_bucket_keys(n, 3)
    s = torch.empty(hs.scratch_bytes(hs.KEYS_I32, n), dtype=torch.uint8, device="cuda")
    sorted_once(hs, k, s)  # warm-up
    hs.hsort_timing_read()
    hs.hsort_timing_enable(True)
    t = sorted_once(hs, k, s)
    hs.hsort_timing_enable(False)
    rec = hs.hsort_timing_read()
    assert np.array_equal(t.cpu().numpy(), np.sort(k))
    assert rec["range"][0] == 1 and rec["range"][2] == 4 * n
    assert rec["scatter"][0] == 1 and rec["scatter"][2] == 8 * n
    assert rec["tilesort"][0] == 1 and rec["tilesort"][2] == 8 * n
    assert rec["merge"][0] == rounds and rec["partition"][0] == rounds
    assert rec["merge"][2] == rounds * 8 * n  # the one bucket merges in every round
    for name in ("range", "scatter", "tilesort", "merge"):
        assert rec[name][1] > 0, name
    # timing off: nothing recorded
    sorted_once(hs, k, s)
    assert hs.hsort_timing_read() == {}


def test_no_records_from_graph_replays(hs):
    n = 2**20
    k = one_bucket_keys(n, 4)
    s = torch.empty(hs.scratch_bytes(hs.KEYS_I32, n), dtype=torch.uint8, device="cuda")
    say("timing records: graph mode")
    side = torch.cuda.Stream()  # graph mode captures on a stream of the caller's, not the null stream
    hs.hsort_graph_mode(True)
    try:
        hs.hsort_timing_read()
        hs.hsort_timing_enable(True)
        with torch.cuda.stream(side):
            t = torch.from_numpy(k).cuda()
            base = t.clone()
            for _ in range(2):  # the first call captures, both replay the graph
                t.copy_(base)
                hs.hsort_keys(t, scratch=s)
            side.synchronize()
        assert np.array_equal(t.cpu().numpy(), np.sort(k))
        hs.hsort_timing_enable(False)
        assert hs.hsort_timing_read() == {}
        assert hs.hsort_graph_count() >= 1
    finally:
        hs.hsort_timing_enable(False)
        hs.hsort_graph_mode(False)
        hs.hsort_graph_clear()
