"""Element-by-element oracle parity at the full sizes of the measured workloads.

Each workload is the one the benchmark times, with the same generator and
seed: 2^28 uniform int32 keys (the headline sort), 2^28 stable pairs with
keys in [0, 1000) and payload = index, 2^26 int64 keys over the full range,
the batched segmented call over 16384 arrays of log-uniform sizes in
[1, 2^16] (eager and as hipGraph replays), and a 2^24-key int64 request
sorted by the serving loop in a mix of other requests.  The oracle sorts
each in seconds to tens of seconds on the host; every output is compared
with it bit for bit (integer sorting has one answer, stable pairs one
order).
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


def test_metric_2e28_uniform_i32_equals_oracle(hs, orc):
    n = 2**28
    k = W.uniform_i32(n, 0)
    say("2^28 uniform int32 (seed 0): GPU sort")
    t = dev(k)
    s = torch.empty(hs.scratch_bytes(hs.KEYS_I32, n), dtype=torch.uint8, device="cuda")
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    got = t.cpu().numpy()
    bounds = hs.read_bounds(s, hs.KEYS_I32, n).cpu().numpy()[0]
    del t, s
    torch.cuda.empty_cache()
    say("2^28 uniform int32: oracle")
    assert np.array_equal(got, orc.sort_keys(k))
    assert np.array_equal(bounds, orc.bounds(k))


def test_pairs_2e28_dup_equals_oracle(hs, orc):
    n = 2**28
    k, v = W.dup_pairs_i32(n, 0)
    say("2^28 stable pairs, keys in [0, 1000): GPU sort")
    tk, tv = dev(k), dev(v.view(np.int32))
    hs.hsort_pairs(tk, tv)
    gk, gv = tk.cpu().numpy(), tv.cpu().numpy().view(np.uint32)
    del tk, tv
    torch.cuda.empty_cache()
    say("2^28 stable pairs: oracle")
    ok, ov = orc.sort_pairs(k, v)
    assert np.array_equal(gk, ok)
    assert np.array_equal(gv, ov)


def test_int64_2e26_full_range_equals_oracle(hs, orc):
    n = 2**26
    k = W.uniform_i64(n, 0)
    say("2^26 int64 full range: GPU sort")
    t = dev(k)
    s = torch.empty(hs.scratch_bytes(hs.KEYS_I64, n), dtype=torch.uint8, device="cuda")
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    got = t.cpu().numpy()
    bounds = hs.read_bounds(s, hs.KEYS_I64, n).cpu().numpy()[0]
    del t, s
    say("2^26 int64: oracle")
    assert np.array_equal(got, orc.sort_keys(k))
    assert np.array_equal(bounds, orc.bounds(k))


def test_segmented_16384_arrays_eager_and_graph_equal_oracle(hs, orc):
    keys, off = W.segments_i32(16384, 2**16, 0)
    n, nseg = keys.size, off.size - 1
    max_len = int(np.diff(off).max())
    say(f"segmented 16384 arrays, {n} keys: oracle")
    ok, ob = orc.sort_segmented(keys, off)
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        t = dev(keys)
        o = dev(off)
        s = torch.empty(hs.scratch_bytes(hs.SEG_I32, n, nseg), dtype=torch.uint8, device="cuda")
        say("segmented 16384 arrays: eager")
        hs.hsort_segmented(t, o, max_seg_len=max_len, scratch=s)
        hs.hsort_check(s)
        assert np.array_equal(t.cpu().numpy(), ok)
        assert np.array_equal(hs.read_bounds(s, hs.SEG_I32, n, nseg).cpu().numpy(), ob)
        hs.hsort_graph_mode(True)
        try:
            for rep in range(3):
                say(f"segmented 16384 arrays: graph replay {rep}")
                t.copy_(dev(keys))
                x = torch.randn(1 << 16, device="cuda")  # unrelated eager work between replays
                float((x * x).sum().item())
                hs.hsort_segmented(t, o, max_seg_len=max_len, scratch=s)
                hs.hsort_check(s)
                assert np.array_equal(t.cpu().numpy(), ok), rep
                assert np.array_equal(hs.read_bounds(s, hs.SEG_I32, n, nseg).cpu().numpy(), ob), rep
        finally:
            hs.hsort_graph_mode(False)
            hs.hsort_graph_clear()


def test_serving_2e24_int64_request_equals_oracle(hs, orc):
    import paper_2003_01216_amd.serve as serve

    info = np.iinfo(np.int64)
    big = np.random.default_rng((0, 2**24)).integers(info.min, info.max, 2**24, dtype=np.int64, endpoint=True)
    others = [W.uniform_i64(int(m), 50 + i) for i, m in enumerate([1 << 10, 70_001, 1 << 20, 3_000_017])]
    say("serving: a 2^24-key int64 request in a mix")
    with serve.SortServer(hbm_budget=64 << 30, streams=2) as srv:
        futs = [srv.submit(a) for a in others[:2]] + [srv.submit(big)] + [srv.submit(a) for a in others[2:]]
        outs = [f.result() for f in futs]
    reqs = others[:2] + [big] + others[2:]
    for a, o in zip(reqs, outs):
        say(f"serving: oracle for {a.size} keys")
        assert np.array_equal(o, orc.sort_keys(a)), a.size
