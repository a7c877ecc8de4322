"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Integer sorting has one correct answer, so every comparison is bit-exact,
element by element (the full workload sizes are in
test_gpu_full_configs.py).  Only the largest array one call accepts
(2^31 - 1 keys) is checked through properties that fix the result (sorted,
same sum and value counts) plus order statistics sampled by the oracle's
counting definition.
"""
import sys

import numpy as np
import pytest

import workloads as W
from stage_check import check_keys_stage

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    hs.load_library()
    return hs


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def gpu_keys(hs, k):
    t = dev(k)
    hs.hsort_keys(t)
    return t.cpu().numpy()


def gpu_pairs(hs, k, v):
    tk = dev(k)
    tv = dev(v.view(np.int32))
    hs.hsort_pairs(tk, tv)
    return tk.cpu().numpy(), tv.cpu().numpy().view(np.uint32)


# ------------------------------------------------------------ plain int32
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_uniform_2e20_matches_oracle(hs, orc, seed):
    k = W.uniform_i32(2**20, seed)
    say(f"uniform 2^20 seed {seed}")
    assert np.array_equal(gpu_keys(hs, k), orc.sort_keys(k))


@pytest.mark.parametrize("name", sorted(W.adversarial_i32().keys()))
def test_adversarial_i32(hs, orc, name):
    k = W.adversarial_i32()[name]
    say(f"adversarial {name} n={k.size}")
    assert np.array_equal(gpu_keys(hs, k), orc.sort_keys(k))


@pytest.mark.parametrize("n", [1, 2, 255, 256, 257, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193, 12289, 40000])
def test_sizes_around_tiles_i32(hs, orc, n):
    k = W.uniform_i32(n, n)
    say(f"sizes n={n}")
    assert np.array_equal(gpu_keys(hs, k), orc.sort_keys(k))


# ------------------------------------------------------------ plain int64
def _i64_cases():
    r = np.random.default_rng(5)
    I = np.iinfo(np.int64)
    cases = {}
    for n in [1, 3, 300, 4095, 4096, 4097, 9000, 100_003, 2**20]:
        cases[f"full_n{n}"] = r.integers(I.min, I.max, n, dtype=np.int64, endpoint=True)
    cases["extremes"] = r.choice(np.array([I.min, I.min + 1, -1, 0, 1, I.max - 1, I.max], np.int64), 30000)
    cases["small_range"] = r.integers(-500, 500, 50000).astype(np.int64)
    cases["all_equal"] = np.full(20000, -77, np.int64)
    cases["reverse"] = np.sort(r.integers(I.min, I.max, 50000, dtype=np.int64))[::-1].copy()
    cases["nonneg_19digit"] = r.integers(0, I.max, 50000, dtype=np.int64)
    return cases


@pytest.mark.parametrize("name", sorted(_i64_cases().keys()))
def test_int64(hs, orc, name):
    k = _i64_cases()[name]
    say(f"int64 {name} n={k.size}")
    assert np.array_equal(gpu_keys(hs, k), orc.sort_keys(k))


# ------------------------------------------------------------ stable pairs
@pytest.mark.parametrize("n", [1, 5, 1000, 4095, 4096, 4097, 65537, 2**20 + 11])
def test_pairs_duplicates(hs, orc, n):
    k, v = W.dup_pairs_i32(n, n)
    say(f"pairs dup n={n}")
    gk, gv = gpu_pairs(hs, k, v)
    ok, ov = orc.sort_pairs(k, v)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


@pytest.mark.parametrize("kind", ["uniform", "all_equal", "two_values", "random_payload"])
def test_pairs_variants(hs, orc, kind):
    r = np.random.default_rng(9)
    n = 300_001
    if kind == "uniform":
        k = W.uniform_i32(n, 4)
    elif kind == "all_equal":
        k = np.full(n, 5, np.int32)
    elif kind == "two_values":
        k = r.choice(np.array([-3, 1 << 30], np.int32), n)
    else:
        k = r.integers(-1000, 1000, n).astype(np.int32)
    v = np.arange(n, dtype=np.uint32) if kind != "random_payload" else r.integers(0, 2**32, n, dtype=np.uint32)
    say(f"pairs {kind}")
    gk, gv = gpu_pairs(hs, k, v)
    ok, ov = orc.sort_pairs(k, v)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


# -------------------------------------------------- intermediate results
def _stage_inputs():
    return {
        "uniform": W.uniform_i32(100_000, 21),
        "three_digit": np.random.default_rng(22).integers(0, 1000, 70_000).astype(np.int32),
        "loguniform": W.loguniform_i32(90_000, 23),
        "negatives": np.random.default_rng(24).integers(-(2**31), 2**31 - 1, 50_000, dtype=np.int32),
        "tiny": np.array([523, 17, 999, 0, 140, 523, 88, 301], np.int32),
    }


@pytest.mark.parametrize("name", sorted(_stage_inputs().keys()))
def test_bounds_match_oracle(hs, orc, name):
    k = _stage_inputs()[name]
    say(f"bounds {name}")
    t = dev(k)
    s = torch.empty(hs.scratch_bytes(hs.KEYS_I32, k.size), dtype=torch.uint8, device="cuda")
    hs.hsort_keys(t, scratch=s)
    torch.cuda.synchronize()
    got = hs.read_bounds(s, hs.KEYS_I32, k.size).cpu().numpy()[0]
    assert np.array_equal(got, orc.bounds(k))


@pytest.mark.parametrize("name", sorted(_stage_inputs().keys()))
def test_stage_scatter_matches_oracle(hs, orc, name):
    k = _stage_inputs()[name]
    digits = hs.hsort_get_config(hs.KEYS_I32, n=k.size)[6]
    say(f"stage scatter {name} digits={digits}")
    t = dev(k)
    hs.hsort_debug_stage(t, 1)
    ok, _, b = orc.scatter(k, digits=digits)
    check_keys_stage(t.cpu().numpy(), ok, b, 1, 0, stable=digits == 1)


@pytest.mark.parametrize("name", sorted(_stage_inputs().keys()))
def test_stage_local_sorts_match_oracle(hs, orc, name):
    k = _stage_inputs()[name]
    cfg = hs.hsort_get_config(hs.KEYS_I32, n=k.size)
    tile, digits = cfg[0], cfg[6]
    say(f"stage tiles {name} tile={tile} digits={digits}")
    t = dev(k)
    hs.hsort_debug_stage(t, 2)
    ok, _, b = orc.bucket_tiles(k, tile, digits=digits)
    check_keys_stage(t.cpu().numpy(), ok, b, 2, tile, stable=digits == 1)


def test_stage_pairs_scatter_and_tiles(hs, orc):
    k, v = W.dup_pairs_i32(200_003, 31)
    cfg = hs.hsort_get_config(hs.PAIRS_I32_U32, n=k.size)
    tile, digits = cfg[0], cfg[6]
    for stage in (1, 2):
        say(f"pairs stage {stage} digits={digits}")
        tk, tv = dev(k), dev(v.view(np.int32))
        hs.hsort_debug_stage(tk, stage, vals=tv)
        if stage == 1:
            ok, ov, _ = orc.scatter(k, v, digits=digits)
        else:
            ok, ov, _ = orc.bucket_tiles(k, tile, v, digits=digits)
        assert np.array_equal(tk.cpu().numpy(), ok)
        assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov)


def test_stage_int64(hs, orc):
    k = _i64_cases()["full_n100003"]
    cfg = hs.hsort_get_config(hs.KEYS_I64, n=k.size)
    tile, digits = cfg[0], cfg[6]
    for stage in (1, 2):
        say(f"int64 stage {stage} digits={digits}")
        t = dev(k)
        hs.hsort_debug_stage(t, stage)
        ok, _, b = orc.scatter(k, digits=digits) if stage == 1 else orc.bucket_tiles(k, tile, digits=digits)
        check_keys_stage(t.cpu().numpy(), ok, b, stage, tile, stable=digits == 1)


def _mixed_magnitudes(dtype, seed):
    """Blocks of whole 4096-key histogram tiles whose maxima have 1, 3, 5, 8, 10 (and, for int64, 19)
    digits, in random block order, so that the tiles' own powers of ten differ from the array's."""
    r = np.random.default_rng(seed)
    tops = [10, 1000, 10**5, 10**8, 2**31 - 1] + ([2**62] if dtype == np.int64 else [])
    blocks = [r.integers(0, top, 4096 * int(r.integers(1, 4)), dtype=dtype) for top in tops for _ in range(2)]
    order = r.permutation(len(blocks))
    return np.concatenate([blocks[i] for i in order] + [r.integers(0, 1000, 777, dtype=dtype)])


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_tiles_with_smaller_digit_plans(hs, orc, dtype):
    # the range pass counts each tile under the tile's own plan; tiles whose
    # maxima have fewer digits than the array's must end up all in bucket 0
    k = _mixed_magnitudes(dtype, 5)
    kind = hs.KEYS_I32 if dtype == np.int32 else hs.KEYS_I64
    say(f"mixed magnitudes {np.dtype(dtype).name} n={k.size}")
    t = dev(k)
    s = torch.empty(hs.scratch_bytes(kind, k.size), dtype=torch.uint8, device="cuda")
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_keys(k))
    assert np.array_equal(hs.read_bounds(s, kind, k.size).cpu().numpy()[0], orc.bounds(k))


def test_segmented_mixed_signs_and_magnitudes(hs, orc):
    # one call in which some large segments hold negative keys (their tiles
    # are counted again from the keys) and others do not (counts from the
    # range pass, some tiles with smaller digit plans than their segment)
    r = np.random.default_rng(9)
    parts = []
    for i in range(12):
        m = int(r.integers(20_000, 60_000))
        if i % 3 == 0:
            parts.append(r.integers(-(10**6), 10**6, m, dtype=np.int32))
        elif i % 3 == 1:
            parts.append(_mixed_magnitudes(np.int32, 100 + i)[:m])
        else:
            parts.append(r.integers(0, 10 ** int(r.integers(1, 10)), m, dtype=np.int32))
    keys = np.concatenate(parts)
    off = np.concatenate([[0], np.cumsum([p.size for p in parts])]).astype(np.int64)
    say(f"segmented mixed signs n={keys.size}")
    t, o = dev(keys), dev(off)
    s = torch.empty(hs.scratch_bytes(hs.SEG_I32, keys.size, off.size - 1), dtype=torch.uint8, device="cuda")
    hs.hsort_segmented(t, o, scratch=s)
    hs.hsort_check(s)
    ok, ob = orc.sort_segmented(keys, off)
    assert np.array_equal(t.cpu().numpy(), ok)
    assert np.array_equal(hs.read_bounds(s, hs.SEG_I32, keys.size, off.size - 1).cpu().numpy(), ob)


# --------------------------------------------------------------- segmented
def _segmented_case(dtype, nseg, max_len, seed):
    keys, off = W.segments_i32(nseg, max_len, seed)
    sizes = np.diff(off)
    r = np.random.default_rng(seed)
    sizes[r.integers(0, nseg, max(1, nseg // 20))] = 0  # some empty segments
    sizes[r.integers(0, nseg, max(1, nseg // 20))] = 1
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    n = int(off[-1])
    if dtype == np.int64:
        I = np.iinfo(np.int64)
        keys = r.integers(I.min, I.max, n, dtype=np.int64, endpoint=True)
    else:
        keys = keys[:n].copy()
    return keys, off


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
@pytest.mark.parametrize("nseg,max_len", [(1, 100_000), (7, 3000), (300, 2**16), (2000, 2**13)])
def test_segmented_matches_oracle(hs, orc, dtype, nseg, max_len):
    keys, off = _segmented_case(dtype, nseg, max_len, 40 + nseg)
    say(f"segmented {np.dtype(dtype).name} nseg={nseg} n={keys.size}")
    t, o = dev(keys), dev(off)
    kind = hs.SEG_I32 if dtype == np.int32 else hs.SEG_I64
    s = torch.empty(hs.scratch_bytes(kind, keys.size, nseg), dtype=torch.uint8, device="cuda")
    hs.hsort_segmented(t, o, scratch=s)
    hs.hsort_check(s)
    ok, ob = orc.sort_segmented(keys, off)
    assert np.array_equal(t.cpu().numpy(), ok)
    assert np.array_equal(hs.read_bounds(s, kind, keys.size, nseg).cpu().numpy(), ob)


def test_segmented_subrange_leaves_outside_untouched(hs, orc):
    r = np.random.default_rng(3)
    keys = r.integers(0, 10**9, 50_000).astype(np.int32)
    off = np.array([1000, 1000, 5000, 30000, 45000], np.int64)
    say("segmented subrange")
    t = dev(keys)
    hs.hsort_segmented(t, dev(off))
    got = t.cpu().numpy()
    assert np.array_equal(got[:1000], keys[:1000]) and np.array_equal(got[45000:], keys[45000:])
    ok, _ = orc.sort_segmented(keys, off)
    assert np.array_equal(got[1000:45000], ok[1000:45000])


def test_invalid_offsets_are_reported(hs):
    keys = np.arange(1000, 0, -1).astype(np.int32)
    off = np.array([0, 600, 300, 1000], np.int64)  # decreasing
    say("invalid offsets")
    t = dev(keys)
    s = torch.empty(hs.scratch_bytes(hs.SEG_I32, 1000, 3), dtype=torch.uint8, device="cuda")
    hs.hsort_segmented(t, dev(off), scratch=s)
    with pytest.raises(hs.HsortError) as e:
        hs.hsort_check(s)
    assert e.value.code == hs.HSORT_ERR_INVALID
    assert np.array_equal(t.cpu().numpy(), keys)  # nothing was touched
    off2 = np.array([0, 600, 1001], np.int64)  # past the end
    hs.hsort_segmented(t, dev(off2), scratch=s)
    with pytest.raises(hs.HsortError):
        hs.hsort_check(s)


def test_understated_max_seg_len_is_reported(hs, orc):
    # a segment longer than the caller's bound would need merge rounds the
    # call does not launch: the device flags it, nothing is touched, and
    # hsort_check reports it instead of returning partly merged keys
    r = np.random.default_rng(12)
    keys = r.integers(0, 2**31 - 1, 60_000, dtype=np.int32)
    off = np.array([0, 3000, 50_000, 60_000], np.int64)
    for hint in (10_000, 47_000 - 1):
        say(f"understated max_seg_len {hint}")
        t = dev(keys)
        s = torch.empty(hs.scratch_bytes(hs.SEG_I32, keys.size, 3), dtype=torch.uint8, device="cuda")
        hs.hsort_segmented(t, dev(off), max_seg_len=hint, scratch=s)
        with pytest.raises(hs.HsortError) as e:
            hs.hsort_check(s)
        assert e.value.code == hs.HSORT_ERR_INVALID and "max_seg_len" in str(e.value)
        assert np.array_equal(t.cpu().numpy(), keys)
    # the exact bound is accepted
    t = dev(keys)
    s = torch.empty(hs.scratch_bytes(hs.SEG_I32, keys.size, 3), dtype=torch.uint8, device="cuda")
    hs.hsort_segmented(t, dev(off), max_seg_len=47_000, scratch=s)
    hs.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_segmented(keys, off)[0])


def test_repeat_is_deterministic(hs):
    k = W.uniform_i32(3_000_001, 8)
    a = gpu_keys(hs, k)
    b = gpu_keys(hs, k)
    assert np.array_equal(a, b)


# ------------------------------------------------------------- full sizes
@pytest.mark.parametrize("dist", ["uniform", "loguniform"])
def test_2e26_matches_oracle(hs, orc, dist):
    n = 2**26
    k = W.uniform_i32(n, 0) if dist == "uniform" else W.loguniform_i32(n, 0)
    say(f"2^26 {dist}")
    got = gpu_keys(hs, k)
    assert np.array_equal(got, orc.sort_keys(k))


def _sampled_order_statistics(orc, inp, out, count=12, seed=0):
    r = np.random.default_rng(seed)
    js = np.concatenate([[0, out.size - 1], r.integers(0, out.size, count)])
    for j in js:
        lt, le = orc.count_lt_le(inp, out[j])
        assert lt <= j < le, (j, out[j], lt, le)


def test_max_keys_properties_and_samples(hs, orc):
    """The largest array one call accepts (2^31 - 1 int32 keys, about a billion
    per decimal bucket: eight fan-in-4 rounds with runs up to 2^30 keys).
    Checked on the device (order, 64-bit sum, count of one value) and by
    order statistics the oracle computes one by one."""
    n = 2**31 - 1
    k = W.uniform_i32(n, 9)
    say("2^31 - 1 uniform keys")
    t = dev(k)
    s = torch.empty(hs.scratch_bytes(hs.KEYS_I32, n), dtype=torch.uint8, device="cuda")
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    del s
    assert bool(torch.all(t[1:] >= t[:-1]).item())
    assert int(t.sum(dtype=torch.int64).item()) == int(k.sum(dtype=np.int64))
    probe = int(k[12345])
    assert int((t == probe).sum().item()) == int(np.count_nonzero(k == probe))
    r = np.random.default_rng(9)
    for j in np.concatenate([[0, n - 1], r.integers(0, n, 4)]):
        x = int(t[int(j)].item())
        lt, le = orc.count_lt_le(k, x)
        assert lt <= j < le, (j, x, lt, le)
