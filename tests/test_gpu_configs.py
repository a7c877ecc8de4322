"""Every configuration the autotuner can pick (local-sort tile shape, merge
shape, fan-in 2 or 4, small-segment threshold, ten, one hundred or one thousand buckets)
sorts bit-exactly like the oracle, so a tuning table can select none that is
untested.  Inputs are sized so that the largest bucket holds more than four
local-sort tiles (two fan-in-4 rounds, three fan-in-2 rounds) and end in a
ragged tile; with one hundred or one thousand buckets, four fifths of the
keys are drawn from the lowest bucket so that it still needs merge rounds."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_2003_01216_amd as hsmod  # noqa: E402
from paper_2003_01216_amd import autotune  # noqa: E402

RAGGED = 1234
I32, I64 = np.iinfo(np.int32), np.iinfo(np.int64)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cands(kind):
    return [pytest.param(c, id="t{}x{}-m{}x{}-s{}-f{}-d{}-l{}".format(*c)) for c in autotune.candidates(kind)]


def skew(keys, cfg, lo, width, seed):
    """With one hundred buckets (cfg[6] == 2), put four fifths of the keys in
    [lo, lo + width), the lowest two-digit bucket of the array's plan; with
    one thousand (cfg[6] == 3) in the lowest three-digit bucket, a tenth of
    that."""
    if cfg[6] == 1:
        return keys
    if cfg[6] == 3:
        width //= 10
    r = np.random.default_rng(seed)
    k = keys.copy()
    m = r.random(k.size) < 0.8
    k[m] = (lo + r.integers(0, width, int(m.sum()))).astype(k.dtype)
    return k


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    hsmod.load_library()
    saved = {(k, c): hsmod.hsort_get_config(k, size_class=c) for k in range(6) for c in range(4)}
    yield hsmod
    for (k, c), cfg in saved.items():
        hsmod.hsort_set_config(k, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=c)


def use(hs, kind, cfg):
    for c in range(4):
        hs.hsort_set_config(kind, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=c)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def scratch(hs, kind, n, nseg=1):
    return torch.empty(hs.scratch_bytes(kind, n, nseg), dtype=torch.uint8, device="cuda")


@pytest.mark.parametrize("cfg", _cands(hsmod.KEYS_I32))
def test_keys_i32(hs, orc, cfg):
    # full int32 range: buckets 0..4 of the shifted keys, the largest ~23 %
    n = 18 * cfg[0] + RAGGED
    k = np.random.default_rng(cfg[0] + cfg[2] + cfg[5]).integers(I32.min, I32.max, n, dtype=np.int32, endpoint=True)
    k = skew(k, cfg, int(I32.min), 10**8, n)  # u up to 2^32 - 1: D = 10, two-digit buckets of 10^8
    say(f"config keys_i32 {cfg} n={n}")
    use(hs, hs.KEYS_I32, cfg)
    t = dev(k)
    s = scratch(hs, hs.KEYS_I32, n)
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))


@pytest.mark.parametrize("cfg", _cands(hsmod.KEYS_I64))
def test_keys_i64(hs, orc, cfg):
    # full int64 range: two buckets of the shifted keys, the larger ~55 %
    n = 8 * cfg[0] + RAGGED
    k = np.random.default_rng(cfg[0] + cfg[2] + cfg[5]).integers(I64.min, I64.max, n, dtype=np.int64, endpoint=True)
    k = skew(k, cfg, int(I64.min), 10**18, n)  # D = 20, two-digit buckets of 10^18
    say(f"config keys_i64 {cfg} n={n}")
    use(hs, hs.KEYS_I64, cfg)
    t = dev(k)
    s = scratch(hs, hs.KEYS_I64, n)
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))


@pytest.mark.parametrize("span", ["dup", "full"])
@pytest.mark.parametrize("cfg", _cands(hsmod.PAIRS_I32_U32))
def test_pairs(hs, orc, cfg, span):
    # "dup": keys in [0, 1000), ten buckets of ~10 %, narrow merge words;
    # "full": the whole int32 range, wide merge words
    if span == "dup":
        n = 45 * cfg[0] + RAGGED
        k, v = W.dup_pairs_i32(n, cfg[0] + cfg[2])
        k = skew(k, cfg, 0, 10, n)  # D = 3: two-digit buckets of ten values
    else:
        n = 18 * cfg[0] + RAGGED
        r = np.random.default_rng(cfg[0] + cfg[2] + 7)
        k = r.integers(I32.min, I32.max, n, dtype=np.int32, endpoint=True)
        v = r.integers(0, 2**32 - 1, n, dtype=np.uint32, endpoint=True)
        k = skew(k, cfg, int(I32.min), 10**8, n)
    say(f"config pairs {span} {cfg} n={n}")
    use(hs, hs.PAIRS_I32_U32, cfg)
    t, tv = dev(k), dev(v.view(np.int32))
    s = scratch(hs, hs.PAIRS_I32_U32, n)
    hs.hsort_pairs(t, tv, scratch=s)
    hs.hsort_check(s)
    ok, ov = orc.sort_pairs(k, v)
    assert np.array_equal(t.cpu().numpy(), ok)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov)


@pytest.mark.parametrize("span", ["dup", "full"])
@pytest.mark.parametrize("cfg", _cands(hsmod.PAIRS_I64_U32))
def test_pairs_i64(hs, orc, cfg, span):
    # "dup": keys in [0, 1000) (narrow 8-byte words); "full": the whole int64
    # range (16-byte words)
    r = np.random.default_rng(cfg[0] + cfg[2] + 13)
    if span == "dup":
        n = 45 * cfg[0] + RAGGED
        k = r.integers(0, 1000, n).astype(np.int64)
        k = skew(k, cfg, 0, 10, n)
    else:
        n = 18 * cfg[0] + RAGGED
        k = r.integers(I64.min, I64.max, n, dtype=np.int64, endpoint=True)
        k = skew(k, cfg, int(I64.min), 10**18, n)
    v = r.integers(0, 2**32 - 1, n, dtype=np.uint32, endpoint=True)
    say(f"config pairs_i64 {span} {cfg} n={n}")
    use(hs, hs.PAIRS_I64_U32, cfg)
    t, tv = dev(k), dev(v.view(np.int32))
    s = scratch(hs, hs.PAIRS_I64_U32, n)
    hs.hsort_sort(t, tv, scratch=s)
    hs.hsort_check(s)
    ok, ov = orc.sort_typed(k, v)
    assert np.array_equal(t.cpu().numpy(), ok)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov)


def _segments(dtype, cfg, seed):
    """One segment of 18 tiles, then 59 of log-uniform sizes in [1, 2 tiles]
    (whole-LDS and pipeline segments both), keys over the full range (the
    first segment skewed as above with one hundred buckets)."""
    tile = cfg[0]
    r = np.random.default_rng(seed)
    sizes = [18 * tile + 5] + np.exp(r.uniform(0, np.log(2 * tile), 59)).astype(np.int64).tolist()
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    info = np.iinfo(dtype)
    keys = r.integers(info.min, info.max, int(off[-1]), dtype=dtype, endpoint=True)
    first = keys[: sizes[0]]
    first[:] = skew(first, cfg, int(info.min), 10**8 if dtype == np.int32 else 10**18, seed)
    return keys, off


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_segmented_every_config(hs, orc, dtype):
    kind = hs.SEG_I32 if dtype == np.int32 else hs.SEG_I64
    for cfg in autotune.candidates(kind):
        keys, off = _segments(dtype, cfg, cfg[0] + cfg[4] + cfg[5])
        nseg = off.size - 1
        say(f"config seg {np.dtype(dtype).name} {cfg} n={keys.size}")
        use(hs, kind, cfg)
        t, o = dev(keys), dev(off)
        s = scratch(hs, kind, keys.size, nseg)
        hs.hsort_segmented(t, o, scratch=s)
        hs.hsort_check(s)
        ok, ob = orc.sort_segmented(keys, off)
        assert np.array_equal(t.cpu().numpy(), ok), cfg
        assert np.array_equal(hs.read_bounds(s, kind, keys.size, nseg).cpu().numpy(), ob), cfg
