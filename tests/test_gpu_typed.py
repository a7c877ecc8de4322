"""GPU parity of the other key types (uint32/uint64, float32/float64 in
IEEE-754 total order, int32/int64), ascending and descending, keys only and
with a uint32 payload (stable), through the C ABI's hsort_sort, against the
oracle's typed sort bit for bit (NaNs included: every bit pattern has one
place).  Also the intermediates (stable bucket scatter, local sorts) and the
exported bounds of the order image, and int64 keys with a payload (the
16-byte sort words) at every size class."""
import sys

import numpy as np
import pytest

import workloads as W
from stage_check import check_keys_stage

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

DTYPES = [np.int32, np.uint32, np.float32, np.int64, np.uint64, np.float64]


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


def key_type(hs, dt):
    return {np.int32: hs.I32, np.uint32: hs.U32, np.float32: hs.F32, np.int64: hs.I64, np.uint64: hs.U64,
            np.float64: hs.F64}[dt]


def bits_dev(k):
    """The keys' bits on the device as a signed tensor of the same width."""
    b = k.view(np.int32 if k.dtype.itemsize == 4 else np.int64)
    return torch.from_numpy(np.ascontiguousarray(b)).cuda()


def host_keys(t, dt):
    return t.cpu().numpy().view(dt)


def same_bits(a, b):
    return a.dtype == b.dtype and np.array_equal(a.view(np.uint8), b.view(np.uint8))


def gpu_sort(hs, k, vals, desc, scratch=None):
    t = bits_dev(k)
    tv = None if vals is None else torch.from_numpy(vals.view(np.int32)).cuda()
    hs.hsort_sort(t, tv, descending=desc, key_type=key_type(hs, k.dtype.type), scratch=scratch)
    return host_keys(t, k.dtype), (None if tv is None else tv.cpu().numpy().view(np.uint32))


@pytest.mark.parametrize("desc", [False, True], ids=["asc", "desc"])
@pytest.mark.parametrize("dt", DTYPES, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("n", [1, 2, 4095, 4097, 70_001, 2**20 + 3])
def test_keys(hs, orc, dt, desc, n):
    k = W.typed_keys(dt, n, n + 7)
    say(f"typed keys {np.dtype(dt).name} desc={desc} n={n}")
    gk, _ = gpu_sort(hs, k, None, desc)
    ok, _ = orc.sort_typed(k, descending=desc)
    assert same_bits(gk, ok)


@pytest.mark.parametrize("desc", [False, True], ids=["asc", "desc"])
@pytest.mark.parametrize("dt", DTYPES, ids=lambda d: np.dtype(d).name)
@pytest.mark.parametrize("n", [3, 5000, 200_003, 300_007])
def test_pairs(hs, orc, dt, desc, n):
    k = W.typed_keys(dt, n, n + 11)
    v = np.arange(n, dtype=np.uint32)
    say(f"typed pairs {np.dtype(dt).name} desc={desc} n={n}")
    gk, gv = gpu_sort(hs, k, v, desc)
    ok, ov = orc.sort_typed(k, v, descending=desc)
    assert same_bits(gk, ok)
    assert np.array_equal(gv, ov)


@pytest.mark.parametrize("desc", [False, True], ids=["asc", "desc"])
@pytest.mark.parametrize("dt", DTYPES, ids=lambda d: np.dtype(d).name)
def test_stages_and_bounds(hs, orc, dt, desc):
    n = 150_001
    k = W.typed_keys(dt, n, 99)
    v = np.arange(n, dtype=np.uint32)
    kt = key_type(hs, dt)
    wide = np.dtype(dt).itemsize == 8
    for with_vals in (False, True):
        kind = (hs.PAIRS_I64_U32 if wide else hs.PAIRS_I32_U32) if with_vals else (hs.KEYS_I64 if wide else hs.KEYS_I32)
        cfg = hs.hsort_get_config(kind, n=n)
        say(f"typed stages {np.dtype(dt).name} desc={desc} vals={with_vals} cfg={cfg}")
        for stage in (1, 2):
            t = bits_dev(k)
            tv = torch.from_numpy(v.view(np.int32)).cuda() if with_vals else None
            hs.hsort_debug_stage_typed(t, stage, vals=tv, descending=desc, key_type=kt)
            ok, ov, b = orc.stage_typed(k, v if with_vals else None, desc, cfg[0] if stage == 2 else 0, cfg[6])
            got = host_keys(t, k.dtype)
            check_keys_stage(got, ok, b, stage, cfg[0], stable=with_vals or cfg[6] == 1,
                             is_sorted=lambda part: same_bits(part, orc.sort_typed(part, descending=desc)[0]))
            if with_vals:
                assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov), (stage, with_vals)
        s = torch.empty(hs.sort_scratch_bytes(kt, with_vals, n), dtype=torch.uint8, device="cuda")
        gpu_sort(hs, k, v if with_vals else None, desc, scratch=s)
        torch.cuda.synchronize()
        assert np.array_equal(hs.read_bounds(s, kind, n).cpu().numpy()[0], orc.bounds_typed(k, desc))


@pytest.mark.parametrize("kind", ["full", "dup", "narrow", "extremes"])
@pytest.mark.parametrize("n", [1, 4096, 4097, 65_537, 2**20 + 5, 2**23 + 1])
def test_int64_pairs(hs, orc, kind, n):
    """int64 keys with a payload: 16-byte sort words (narrow 8-byte ones when a
    bucket or a merge chunk spans few values), every size class."""
    r = np.random.default_rng(n + len(kind))
    I = np.iinfo(np.int64)
    if kind == "full":
        k = r.integers(I.min, I.max, n, dtype=np.int64, endpoint=True)
    elif kind == "dup":
        k = r.integers(-500, 500, n).astype(np.int64)
    elif kind == "narrow":
        k = r.integers(0, 10**12, n, dtype=np.int64)
    else:
        k = r.choice(np.array([I.min, I.min + 1, -1, 0, 1, I.max - 1, I.max], np.int64), n)
    v = r.integers(0, 2**32 - 1, n, dtype=np.uint32, endpoint=True)
    say(f"int64 pairs {kind} n={n}")
    tk, tv = torch.from_numpy(k).cuda(), torch.from_numpy(v.view(np.int32)).cuda()
    hs.hsort_sort(tk, tv)
    ok, ov = orc.sort_typed(k, v)
    assert np.array_equal(tk.cpu().numpy(), ok)
    assert np.array_equal(tv.cpu().numpy().view(np.uint32), ov)


def test_descending_int32_matches_reversed_stable(hs, orc):
    # the ten-bucket and hundred-bucket plans both, through the full pipeline
    k = W.uniform_i32(3_000_001, 5)
    gk, _ = gpu_sort(hs, k, None, True)
    assert np.array_equal(gk, orc.sort_typed(k, descending=True)[0])
    assert np.array_equal(gk, np.sort(k)[::-1])

