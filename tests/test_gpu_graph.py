"""hipGraph replay of the launch sequence equals eager launches and the oracle.

Each test replays several times with fresh data and unrelated eager GPU work
(and host synchronisations) between the replays, and checks every replay.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    hs.load_library()
    yield hs
    hs.hsort_graph_mode(False)
    hs.hsort_graph_clear()


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def eager_noise():
    x = torch.randn(1 << 16, device="cuda")
    return float((x * x).sum().item())


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_segmented_graph_replays(hs, orc, dtype):
    keys0, off = W.segments_i32(3000, 2**15, 7)
    n = keys0.size
    max_len = int(np.diff(off).max())
    kind = hs.SEG_I32 if dtype == np.int32 else hs.SEG_I64
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        t = torch.empty(n, dtype=torch.int32 if dtype == np.int32 else torch.int64, device="cuda")
        o = dev(off)
        s = torch.empty(hs.scratch_bytes(kind, n, 3000), dtype=torch.uint8, device="cuda")
        hs.hsort_graph_mode(True)
        try:
            before = hs.hsort_graph_count()
            for rep in range(4):
                r = np.random.default_rng(100 + rep)
                if dtype == np.int32:
                    k = r.integers(0, 2**31 - 1, n, dtype=np.int32)
                else:
                    k = r.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, n, dtype=np.int64)
                t.copy_(dev(k))
                eager_noise()
                say(f"segmented graph replay {rep} {np.dtype(dtype).name}")
                hs.hsort_segmented(t, o, max_seg_len=max_len, scratch=s)
                side.synchronize()
                assert np.array_equal(t.cpu().numpy(), orc.sort_segmented(k, off)[0]), rep
            assert hs.hsort_graph_count() == before + 1  # captured once, replayed after
        finally:
            hs.hsort_graph_mode(False)


def test_segmented_graph_new_offsets(hs, orc):
    """Same sizes, different offsets values: the graph reads them on the device."""
    n, nseg = 200_000, 500
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        o = torch.empty(nseg + 1, dtype=torch.int64, device="cuda")
        s = torch.empty(hs.scratch_bytes(hs.SEG_I32, n, nseg), dtype=torch.uint8, device="cuda")
        hs.hsort_graph_mode(True)
        try:
            for rep in range(3):
                r = np.random.default_rng(rep)
                cuts = np.sort(r.choice(np.arange(1, n), nseg - 1, replace=False))
                off = np.concatenate([[0], cuts, [n]]).astype(np.int64)
                k = r.integers(-(10**6), 10**6, n).astype(np.int32)
                t.copy_(dev(k))
                o.copy_(dev(off))
                say(f"new offsets replay {rep}")
                hs.hsort_segmented(t, o, max_seg_len=n, scratch=s)
                side.synchronize()
                assert np.array_equal(t.cpu().numpy(), orc.sort_segmented(k, off)[0]), rep
        finally:
            hs.hsort_graph_mode(False)


def test_graph_replay_with_segment_beyond_hint(hs, orc):
    """A graph captured for max_seg_len = 4096 and replayed with offsets whose
    segment is longer: the device check reports it and leaves the keys, and a
    later replay with valid offsets sorts again."""
    n, nseg = 40_000, 20
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        t = torch.empty(n, dtype=torch.int32, device="cuda")
        o = torch.empty(nseg + 1, dtype=torch.int64, device="cuda")
        s = torch.empty(hs.scratch_bytes(hs.SEG_I32, n, nseg), dtype=torch.uint8, device="cuda")
        good = np.linspace(0, n, nseg + 1).astype(np.int64)  # 2000 keys each
        bad = good.copy()
        bad[6:9] = bad[9]  # segment 5 spans 8000 keys, beyond the 4096 hint; 6 to 8 are empty
        hs.hsort_graph_mode(True)
        try:
            for rep, off in enumerate([good, bad, good]):
                k = np.random.default_rng(200 + rep).integers(0, 2**31 - 1, n, dtype=np.int32)
                t.copy_(dev(k))
                o.copy_(dev(off))
                eager_noise()
                say(f"graph replay against the hint {rep}")
                hs.hsort_segmented(t, o, max_seg_len=4096, scratch=s)
                if off is bad:
                    with pytest.raises(hs.HsortError) as e:
                        hs.hsort_check(s)
                    assert "max_seg_len" in str(e.value)
                    assert np.array_equal(t.cpu().numpy(), k)
                else:
                    hs.hsort_check(s)
                    assert np.array_equal(t.cpu().numpy(), orc.sort_segmented(k, off)[0]), rep
        finally:
            hs.hsort_graph_mode(False)


@pytest.mark.parametrize("what", ["keys_i32", "keys_i64", "pairs"])
def test_plain_graph_replays(hs, orc, what):
    n = 3_000_017
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        dt = torch.int64 if what == "keys_i64" else torch.int32
        t = torch.empty(n, dtype=dt, device="cuda")
        v = torch.empty(n, dtype=torch.int32, device="cuda")
        hs.hsort_graph_mode(True)
        try:
            for rep in range(3):
                r = np.random.default_rng(50 + rep)
                if what == "keys_i64":
                    k = r.integers(np.iinfo(np.int64).min, np.iinfo(np.int64).max, n, dtype=np.int64)
                elif what == "pairs":
                    k = r.integers(0, 1000, n).astype(np.int32)
                else:
                    k = r.integers(-(2**31), 2**31 - 1, n, dtype=np.int32)
                t.copy_(dev(k))
                eager_noise()
                say(f"plain graph {what} replay {rep}")
                if what == "pairs":
                    vals = np.arange(n, dtype=np.uint32)
                    v.copy_(dev(vals.view(np.int32)))
                    hs.hsort_pairs(t, v)
                    side.synchronize()
                    ok, ov = orc.sort_pairs(k, vals)
                    assert np.array_equal(t.cpu().numpy(), ok)
                    assert np.array_equal(v.cpu().numpy().view(np.uint32), ov)
                else:
                    hs.hsort_keys(t)
                    side.synchronize()
                    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k)), rep
        finally:
            hs.hsort_graph_mode(False)


def test_call_inside_user_capture(hs, orc):
    """A call made while the caller captures a torch CUDA graph becomes part of it."""
    keys0, off = W.segments_i32(800, 2**13, 9)
    n = keys0.size
    t = dev(keys0)
    o = dev(off)
    s = torch.empty(hs.scratch_bytes(hs.SEG_I32, n, 800), dtype=torch.uint8, device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        hs.hsort_segmented(t, o, max_seg_len=2**13, scratch=s)  # warm-up outside capture
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        hs.hsort_segmented(t, o, max_seg_len=2**13, scratch=s)
    for rep in range(3):
        k = np.random.default_rng(7 + rep).integers(0, 2**31 - 1, n, dtype=np.int32)
        t.copy_(dev(k))
        torch.cuda.synchronize()
        eager_noise()
        say(f"user graph replay {rep}")
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), orc.sort_segmented(k, off)[0]), rep
