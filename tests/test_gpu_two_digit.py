"""GPU parity of the two-digit one-step partition (one hundred buckets).

The finer splitter reads the first two of the D decimal digits of
u = k - beta: bucket floor(u / 10^(D-2)), or 10u when D = 1.  Every shape of
every kind is switched to it here, and the intermediate results (the stable
bucket scatter, the local sorts of each bucket's partitions, the exported
ten-bucket bounds) and the final sorts are compared bit for bit with the
oracle's two-digit mode.  Inputs reach the cases the range and histogram
passes treat apart: tiles whose own power of ten is a tenth or at most a
hundredth of their segment's, negative keys, one- and two-digit arrays,
heavy duplicates, segments of every size class.
"""
import sys

import numpy as np
import pytest

import workloads as W
from stage_check import check_keys_stage

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I32, I64 = np.iinfo(np.int32), np.iinfo(np.int64)


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    hs.load_library()
    saved = {(k, c): hs.hsort_get_config(k, size_class=c) for k in range(6) for c in range(4)}
    for (k, c), cfg in saved.items():
        hs.hsort_set_config(k, *cfg[:5], fanin=cfg[5], digits=2, local=cfg[7], size_class=c)
    print("two-digit partition on every kind", flush=True)
    yield hs
    for (k, c), cfg in saved.items():
        hs.hsort_set_config(k, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=c)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def scratch(hs, kind, n, nseg=1):
    return torch.empty(max(hs.scratch_bytes(kind, n, nseg), 1), dtype=torch.uint8, device="cuda")


def _mixed_magnitudes(dtype, seed):
    """Whole 4096-key tiles whose maxima have 1 to 10 (int64: up to 19)
    digits in random order: tiles with the array's power of ten, a tenth of
    it (counted again from the keys) and a hundredth or less (all bucket 0)."""
    r = np.random.default_rng(seed)
    tops = [10, 100, 1000, 10**5, 10**7, 10**8, 10**9, 2**31 - 1]
    if dtype == np.int64:
        tops += [10**17, 10**18, 2**62]
    blocks = [r.integers(0, top, 4096 * int(r.integers(1, 4)), dtype=dtype) for top in tops for _ in range(2)]
    order = r.permutation(len(blocks))
    return np.concatenate([blocks[i] for i in order] + [r.integers(0, 1000, 777, dtype=dtype)])


def _inputs_i32():
    r = np.random.default_rng(61)
    return {
        "uniform": W.uniform_i32(300_000, 62),
        "loguniform": W.loguniform_i32(200_000, 63),
        "three_digit": r.integers(0, 1000, 150_000).astype(np.int32),
        "two_digit": r.integers(0, 100, 60_000).astype(np.int32),
        "one_digit": r.integers(0, 10, 50_000).astype(np.int32),
        "negatives": r.integers(I32.min, I32.max, 120_000, dtype=np.int32, endpoint=True),
        "small_negative": r.integers(-5000, 300, 70_000).astype(np.int32),
        "mixed_magnitudes": _mixed_magnitudes(np.int32, 64),
        "all_equal": np.full(40_000, 123456, np.int32),
        "tiny": np.array([523, 17, 999, 0, 140, 523, 88, 301], np.int32),
    }


@pytest.mark.parametrize("name", sorted(_inputs_i32().keys()))
def test_stages_and_sort_i32(hs, orc, name):
    k = _inputs_i32()[name]
    cfg = hs.hsort_get_config(hs.KEYS_I32, n=k.size)
    assert cfg[6] == 2
    say(f"two-digit int32 {name} n={k.size} cfg={cfg}")
    t = dev(k)
    hs.hsort_debug_stage(t, 1)
    ok, _, b = orc.scatter(k, digits=2)
    check_keys_stage(t.cpu().numpy(), ok, b, 1, 0, stable=False)
    t = dev(k)
    hs.hsort_debug_stage(t, 2)
    check_keys_stage(t.cpu().numpy(), orc.bucket_tiles(k, cfg[0], digits=2)[0], b, 2, cfg[0], stable=False)
    t = dev(k)
    s = scratch(hs, hs.KEYS_I32, k.size)
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k)), "sort"
    assert np.array_equal(hs.read_bounds(s, hs.KEYS_I32, k.size).cpu().numpy()[0], orc.bounds(k)), "bounds"


def _inputs_i64():
    r = np.random.default_rng(71)
    return {
        "full": r.integers(I64.min, I64.max, 100_003, dtype=np.int64, endpoint=True),
        "nonneg_19digit": r.integers(0, I64.max, 80_000, dtype=np.int64),
        "small_range": r.integers(-500, 500, 50_000).astype(np.int64),
        "extremes": r.choice(np.array([I64.min, I64.min + 1, -1, 0, 1, I64.max - 1, I64.max], np.int64), 30_000),
        "mixed_magnitudes": _mixed_magnitudes(np.int64, 72),
    }


@pytest.mark.parametrize("name", sorted(_inputs_i64().keys()))
def test_stages_and_sort_i64(hs, orc, name):
    k = _inputs_i64()[name]
    cfg = hs.hsort_get_config(hs.KEYS_I64, n=k.size)
    say(f"two-digit int64 {name} n={k.size} cfg={cfg}")
    t = dev(k)
    hs.hsort_debug_stage(t, 1)
    ok, _, b = orc.scatter(k, digits=2)
    check_keys_stage(t.cpu().numpy(), ok, b, 1, 0, stable=False)
    t = dev(k)
    hs.hsort_debug_stage(t, 2)
    check_keys_stage(t.cpu().numpy(), orc.bucket_tiles(k, cfg[0], digits=2)[0], b, 2, cfg[0], stable=False)
    t = dev(k)
    s = scratch(hs, hs.KEYS_I64, k.size)
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k)), "sort"
    assert np.array_equal(hs.read_bounds(s, hs.KEYS_I64, k.size).cpu().numpy()[0], orc.bounds(k)), "bounds"


@pytest.mark.parametrize("name", ["dup", "narrow_buckets", "full_range"])
def test_stages_and_sort_pairs(hs, orc, name):
    r = np.random.default_rng(81)
    n = 250_007
    if name == "dup":
        k, v = W.dup_pairs_i32(n, 82)
    elif name == "narrow_buckets":  # D = 7: two-digit buckets of 10^5 values, narrow local-sort words
        k = r.integers(0, 10**7, n).astype(np.int32)
        v = np.arange(n, dtype=np.uint32)
    else:
        k = r.integers(I32.min, I32.max, n, dtype=np.int32, endpoint=True)
        v = r.integers(0, 2**32 - 1, n, dtype=np.uint32, endpoint=True)
    cfg = hs.hsort_get_config(hs.PAIRS_I32_U32, n=n)
    say(f"two-digit pairs {name} cfg={cfg}")
    for stage in (1, 2, 3):
        tk, tv = dev(k), dev(v.view(np.int32))
        hs.hsort_debug_stage(tk, stage, vals=tv)
        if stage == 1:
            ok, ov, _ = orc.scatter(k, v, digits=2)
        elif stage == 2:
            ok, ov, _ = orc.bucket_tiles(k, cfg[0], v, digits=2)
        else:
            ok, ov = orc.sort_pairs(k, v)
        assert np.array_equal(tk.cpu().numpy(), ok), stage
        assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov), stage


@pytest.mark.parametrize("n", [1, 2, 4095, 4096, 4097, 8193, 16385, 40_000, 2**20 + 7])
def test_sizes_around_tiles(hs, orc, n):
    k = W.uniform_i32(n, n + 5)
    say(f"two-digit sizes n={n}")
    t = dev(k)
    hs.hsort_keys(t)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))


@pytest.mark.parametrize("name", sorted(W.adversarial_i32().keys()))
def test_adversarial(hs, orc, name):
    k = W.adversarial_i32()[name]
    say(f"two-digit adversarial {name} n={k.size}")
    t = dev(k)
    hs.hsort_keys(t)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_segmented(hs, orc, dtype):
    r = np.random.default_rng(91)
    parts = []
    for i in range(40):
        m = int(np.exp(r.uniform(0, np.log(120_000))))
        if i % 4 == 0:
            parts.append(r.integers(-(10**6), 10**6, m).astype(dtype))
        elif i % 4 == 1:
            parts.append(_mixed_magnitudes(dtype, 200 + i)[:m])
        elif i % 4 == 2:
            parts.append(r.integers(0, 10 ** int(r.integers(1, 10)), m).astype(dtype))
        else:
            info = np.iinfo(dtype)
            parts.append(r.integers(info.min, info.max, m, dtype=dtype, endpoint=True))
    keys = np.concatenate(parts)
    off = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
    kind = hs.SEG_I32 if dtype == np.int32 else hs.SEG_I64
    say(f"two-digit segmented {np.dtype(dtype).name} n={keys.size}")
    t, o = dev(keys), dev(off)
    s = scratch(hs, kind, keys.size, off.size - 1)
    hs.hsort_segmented(t, o, scratch=s)
    hs.hsort_check(s)
    ok, ob = orc.sort_segmented(keys, off)
    assert np.array_equal(t.cpu().numpy(), ok)
    assert np.array_equal(hs.read_bounds(s, kind, keys.size, off.size - 1).cpu().numpy(), ob)


@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
def test_2e24(hs, orc, dist):
    n = 2**24
    k = W.uniform_i32(n, 3) if dist == "uniform" else W.loguniform_i32(n, 3)
    say(f"two-digit 2^24 {dist}")
    t = dev(k)
    hs.hsort_keys(t)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))
