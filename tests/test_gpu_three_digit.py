"""GPU parity of the three-digit one-step partition (one thousand buckets).

The splitter reads the first three of the D decimal digits of u = k - beta:
bucket floor(u / 10^(D-3)), or the digits of a shorter u followed by zeros
(100u when D = 1, 10u when D = 2).  It is offered for plain int32 sorts,
keys only (16384-key partition tiles, an unstable cursor scatter) and stable
pairs (4096-key tiles, three stable counting passes), and for the 32-bit
images of hsort_sort.  Every int32 keys and pairs shape is switched to it
here; the intermediate results (the keys-only scatter as each bucket's
multiset of keys, the pairs scatter bit for bit; the local sorts), the
exported ten-bucket bounds and the final sorts are compared with the
oracle's three-digit mode.  Keys of at most three digits put one key value
in each bucket: such buckets are copied, not sorted, and no merge round
follows.  Inputs reach
the cases the range and histogram passes treat apart: tiles whose own power
of ten is below their array's, negative keys, arrays of one to three digits,
heavy duplicates, skewed buckets, and sizes around the partition tile.
"""
import sys

import numpy as np
import pytest

import workloads as W
from stage_check import check_keys_stage

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I32 = np.iinfo(np.int32)
PTILE = 16384  # keys per partition tile with one thousand buckets


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    hs.load_library()
    saved = {(k, c): hs.hsort_get_config(k, size_class=c) for k in (hs.KEYS_I32, hs.PAIRS_I32_U32) for c in range(4)}
    for (k, c), cfg in saved.items():
        hs.hsort_set_config(k, *cfg[:5], fanin=cfg[5], digits=3, local=cfg[7], size_class=c)
    print("three-digit partition on int32 keys and pairs", flush=True)
    yield hs
    for (k, c), cfg in saved.items():
        hs.hsort_set_config(k, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=c)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def scratch(hs, kind, n):
    return torch.empty(max(hs.scratch_bytes(kind, n), 1), dtype=torch.uint8, device="cuda")


def _mixed_magnitudes(seed):
    """Whole partition tiles whose maxima have 1 to 10 digits, in random
    order: tiles with the array's power of ten, a tenth and a hundredth of it
    (their keys counted again under the array's plan) and less."""
    r = np.random.default_rng(seed)
    tops = [10, 100, 1000, 10**5, 10**7, 10**8, 10**9, 2**31 - 1]
    blocks = [r.integers(0, top, PTILE * int(r.integers(1, 3)), dtype=np.int32) for top in tops for _ in range(2)]
    order = r.permutation(len(blocks))
    return np.concatenate([blocks[i] for i in order] + [r.integers(0, 1000, 777, dtype=np.int32)])


def _inputs():
    r = np.random.default_rng(161)
    skew = W.uniform_i32(400_000, 162)
    m = r.random(skew.size) < 0.85
    skew[m] = r.integers(0, 10**7, int(m.sum())).astype(np.int32)  # 85 % in the lowest bucket
    return {
        "uniform": W.uniform_i32(600_000, 163),
        "loguniform": W.loguniform_i32(400_000, 164),
        "skewed": skew,
        "four_digit": r.integers(0, 10_000, 200_000).astype(np.int32),
        "three_digit": r.integers(0, 1000, 150_000).astype(np.int32),
        "two_digit": r.integers(0, 100, 60_000).astype(np.int32),
        "one_digit": r.integers(0, 10, 50_000).astype(np.int32),
        "negatives": r.integers(I32.min, I32.max, 300_000, dtype=np.int32, endpoint=True),
        "small_negative": r.integers(-5000, 300, 70_000).astype(np.int32),
        "mixed_magnitudes": _mixed_magnitudes(165),
        "all_equal": np.full(40_000, 123456, np.int32),
        "extremes": r.choice(np.array([I32.min, I32.min + 1, -1, 0, 1, I32.max - 1, I32.max], np.int32), 50_000),
    }


@pytest.mark.parametrize("name", sorted(_inputs().keys()))
def test_stages_and_sort(hs, orc, name):
    k = _inputs()[name]
    cfg = hs.hsort_get_config(hs.KEYS_I32, n=k.size)
    assert cfg[6] == 3
    say(f"three-digit int32 {name} n={k.size} cfg={cfg}")
    t = dev(k)
    hs.hsort_debug_stage(t, 1)
    ok, _, b = orc.scatter(k, digits=3)
    check_keys_stage(t.cpu().numpy(), ok, b, 1, 0, stable=False)
    t = dev(k)
    hs.hsort_debug_stage(t, 2)
    check_keys_stage(t.cpu().numpy(), orc.bucket_tiles(k, cfg[0], digits=3)[0], b, 2, cfg[0], stable=False)
    t = dev(k)
    s = scratch(hs, hs.KEYS_I32, k.size)
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k)), "sort"
    assert np.array_equal(hs.read_bounds(s, hs.KEYS_I32, k.size).cpu().numpy()[0], orc.bounds(k)), "bounds"


@pytest.mark.parametrize("n", [8193, PTILE - 1, PTILE, PTILE + 1, 2 * PTILE + 3, 100_000, 2**20 + 7])
def test_sizes_around_tiles(hs, orc, n):
    k = W.uniform_i32(n, n + 9)
    say(f"three-digit sizes n={n}")
    t = dev(k)
    hs.hsort_keys(t)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))


@pytest.mark.parametrize("name", sorted(W.adversarial_i32().keys()))
def test_adversarial(hs, orc, name):
    k = W.adversarial_i32()[name]
    say(f"three-digit adversarial {name} n={k.size}")
    t = dev(k)
    hs.hsort_keys(t)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))


@pytest.mark.parametrize("dtype", [np.uint32, np.float32])
@pytest.mark.parametrize("desc", [False, True])
def test_typed(hs, orc, dtype, desc):
    n = 300_001
    k = W.typed_keys(dtype, n, 171)
    kt = hs.U32 if dtype == np.uint32 else hs.F32
    say(f"three-digit typed {np.dtype(dtype).name} desc={desc} n={n}")
    t = dev(k.view(np.int32))  # the keys' bits
    hs.hsort_debug_stage_typed(t, 1, descending=desc, key_type=kt)
    ok, _, b = orc.stage_typed(k, None, desc, 0, 3)
    check_keys_stage(t.cpu().numpy().view(dtype), ok, b, 1, 0, stable=False)
    t = dev(k.view(np.int32))
    hs.hsort_sort(t, descending=desc, key_type=kt)
    assert np.array_equal(t.cpu().numpy().view(np.uint8), orc.sort_typed(k, descending=desc)[0].view(np.uint8))


@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
def test_2e24(hs, orc, dist):
    n = 2**24
    k = W.uniform_i32(n, 5) if dist == "uniform" else W.loguniform_i32(n, 5)
    say(f"three-digit 2^24 {dist}")
    t = dev(k)
    s = scratch(hs, hs.KEYS_I32, n)
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))
    assert np.array_equal(hs.read_bounds(s, hs.KEYS_I32, n).cpu().numpy()[0], orc.bounds(k)), "bounds"


def test_noalloc(hs, orc):
    # the allocation-free entry point shares the int32 table, so it runs the
    # three-digit partition here too
    for n in (3_000_001, 70_000):
        k = W.uniform_i32(n, n)
        say(f"three-digit noalloc n={n}")
        t = dev(k)
        hs.hsort_keys_i32_noalloc(t)
        torch.cuda.synchronize()
        assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))


def _pair_inputs():
    r = np.random.default_rng(181)
    n = 300_007
    out = {
        "dup": W.dup_pairs_i32(n, 182),  # keys in [0, 1000): one key value per bucket
        "narrow": (r.integers(0, 10**7, n).astype(np.int32), np.arange(n, dtype=np.uint32)),
        "full": (r.integers(I32.min, I32.max, n, dtype=np.int32, endpoint=True),
                 r.integers(0, 2**32 - 1, n, dtype=np.uint32, endpoint=True)),
    }
    k = r.integers(0, 1000, 2_000_003).astype(np.int32)
    k[r.random(k.size) < 0.7] = 7  # one bucket far above a tile: copied, not merged
    out["dup_heavy"] = (k, np.arange(k.size, dtype=np.uint32))
    return out


@pytest.mark.parametrize("name", sorted(_pair_inputs().keys()))
def test_pairs_stages_and_sort(hs, orc, name):
    k, v = _pair_inputs()[name]
    cfg = hs.hsort_get_config(hs.PAIRS_I32_U32, n=k.size)
    assert cfg[6] == 3
    say(f"three-digit pairs {name} n={k.size} cfg={cfg}")
    for stage in (1, 2, 3):
        tk, tv = dev(k), dev(v.view(np.int32))
        hs.hsort_debug_stage(tk, stage, vals=tv)
        if stage == 1:
            ok, ov, _ = orc.scatter(k, v, digits=3)
        elif stage == 2:
            ok, ov, _ = orc.bucket_tiles(k, cfg[0], v, digits=3)
        else:
            ok, ov = orc.sort_pairs(k, v)
        assert np.array_equal(tk.cpu().numpy(), ok), stage
        assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov), stage
    tk, tv = dev(k), dev(v.view(np.int32))
    s = scratch(hs, hs.PAIRS_I32_U32, k.size)
    hs.hsort_pairs(tk, tv, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(hs.read_bounds(s, hs.PAIRS_I32_U32, k.size).cpu().numpy()[0], orc.bounds(k)), "bounds"


@pytest.mark.parametrize("n", [5_000, 70_000, 3_000_001])
def test_keys_one_value_per_bucket(hs, orc, n):
    # keys of at most three digits: every bucket spans one key value, and the
    # largest holds many tiles
    r = np.random.default_rng(n)
    k = r.integers(0, 1000, n).astype(np.int32)
    k[r.random(n) < 0.5] = 999
    say(f"three-digit keys of one value per bucket n={n}")
    t = dev(k)
    hs.hsort_debug_stage(t, 2)
    ok, _, b = orc.scatter(k, digits=3)
    check_keys_stage(t.cpu().numpy(), ok, b, 2, hs.hsort_get_config(hs.KEYS_I32, n=n)[0], stable=False)
    t = dev(k)
    hs.hsort_keys(t)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))

