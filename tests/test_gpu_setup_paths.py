"""GPU parity around the plain-sort setup paths.

A plain sort (one array) takes its segment's counts and its partition-tile
list from the setup kernel, and an array of at most 64 partition tiles (one
group) builds its offsets, bucket table, the scans of its tile and chunk
counts and its local-sort descriptors in one workgroup; larger arrays take
the general launches, as segmented calls always do.  Sizes on either side of
64 partition tiles -- 16384-key tiles for int32 keys with one thousand
buckets, 4096-key tiles with ten or one hundred buckets and for stable pairs
-- are compared with the oracle (keys, payloads and the ten-bucket bounds),
on uniform keys and on keys crowded into one bucket, and the same keys as a
one-segment segmented call.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GROUP_TILES = 64


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    hs.load_library()
    kinds = (hs.KEYS_I32, hs.PAIRS_I32_U32)
    saved = {(k, c): hs.hsort_get_config(k, size_class=c) for k in kinds for c in range(4)}
    yield hs
    for (k, c), cfg in saved.items():
        hs.hsort_set_config(k, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=c)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def use_digits(hs, kind, digits):
    for c in range(4):
        cfg = hs.hsort_get_config(kind, size_class=c)
        hs.hsort_set_config(kind, *cfg[:5], fanin=cfg[5], digits=digits, local=cfg[7], size_class=c)


def partition_tile(digits, pairs):
    return 16384 if digits == 3 and not pairs else 4096


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def scratch(hs, kind, n, nseg=0):
    return torch.empty(max(hs.scratch_bytes(kind, n, nseg), 1), dtype=torch.uint8, device="cuda")


def keys_of(dist, n, seed):
    if dist == "uniform":
        return W.uniform_i32(n, seed)
    # nine keys in ten inside one bucket of the array's plan (its maximum
    # has ten digits), the rest uniform: one bucket spans many tiles
    k = W.uniform_i32(n, seed)
    r = np.random.default_rng(seed + 1)
    m = r.random(n) < 0.9
    k[m] = r.integers(10**9, 10**9 + 10**6, int(m.sum())).astype(np.int32)
    return k


def sizes(ptile):
    edge = GROUP_TILES * ptile
    return [edge - 1, edge, edge + 1, edge + ptile - 1]


@pytest.mark.parametrize("dist", ["uniform", "one_bucket"])
@pytest.mark.parametrize("digits", [1, 2, 3])
def test_keys_around_one_group(hs, orc, digits, dist):
    use_digits(hs, hs.KEYS_I32, digits)
    for n in sizes(partition_tile(digits, False)):
        k = keys_of(dist, n, n + digits)
        say(f"setup paths: int32 keys digits={digits} {dist} n={n}")
        t = dev(k)
        s = scratch(hs, hs.KEYS_I32, n)
        hs.hsort_keys(t, scratch=s)
        hs.hsort_check(s)
        assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k)), n
        assert np.array_equal(hs.read_bounds(s, hs.KEYS_I32, n).cpu().numpy()[0], orc.bounds(k)), n


@pytest.mark.parametrize("digits", [1, 3])
def test_pairs_around_one_group(hs, orc, digits):
    use_digits(hs, hs.PAIRS_I32_U32, digits)
    for n in sizes(partition_tile(digits, True)):
        k = keys_of("one_bucket" if n % 2 else "uniform", n, n)
        v = np.arange(n, dtype=np.uint32)
        say(f"setup paths: int32 pairs digits={digits} n={n}")
        tk, tv = dev(k), dev(v.view(np.int32))
        s = scratch(hs, hs.PAIRS_I32_U32, n)
        hs.hsort_pairs(tk, tv, scratch=s)
        hs.hsort_check(s)
        ok, ov = orc.sort_pairs(k, v)
        assert np.array_equal(tk.cpu().numpy(), ok), n
        assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov), n
        assert np.array_equal(hs.read_bounds(s, hs.PAIRS_I32_U32, n).cpu().numpy()[0], orc.bounds(k)), n


@pytest.mark.parametrize("n", [8193, GROUP_TILES * 4096, GROUP_TILES * 16384 + 1])
def test_one_segment_segmented_equals_plain(hs, orc, n):
    # the segmented call takes the general setup launches for the same array
    k = W.uniform_i32(n, 7)
    say(f"setup paths: one-segment segmented n={n}")
    t = dev(k)
    off = torch.tensor([0, n], dtype=torch.int64, device="cuda")
    s = scratch(hs, hs.SEG_I32, n, 1)
    hs.hsort_segmented(t, off, scratch=s)
    hs.hsort_check(s)
    ok, ob = orc.sort_segmented(k, np.array([0, n], np.int64))
    assert np.array_equal(t.cpu().numpy(), ok)
    assert np.array_equal(hs.read_bounds(s, hs.SEG_I32, n, 1).cpu().numpy(), ob)
    p = dev(k)
    hs.hsort_keys(p)
    assert np.array_equal(p.cpu().numpy(), ok)
