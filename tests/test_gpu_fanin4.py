"""The full pipeline with fan-in-4 merge rounds (every size class, every key
kind) against the oracle, bit-exact, including the device-side consistency
check of the split points."""
import sys

import numpy as np
import pytest

import workloads as W
from stage_check import check_keys_stage

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# fan-in-4 merge shapes compiled for every key kind: (sampling stride S =
# outputs per workgroup, outputs per thread); a workgroup holds up to 2S keys
SHAPES = [(4096, 16), (2048, 16), (2048, 8)]


@pytest.fixture(scope="module", params=SHAPES, ids=lambda s: f"S{s[0]}x{s[1]}")
def hs4(request):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    hs.load_library()
    nv, vt = request.param
    # kinds 0-4 (int64 pairs have 16-byte words and their own shapes, covered by test_gpu_configs)
    saved = {(k, c): hs.hsort_get_config(k, size_class=c) for k in range(5) for c in range(4)}
    for (k, c), cfg in saved.items():
        # the tuned local sort when this merge shape divides its tile, else the default network sort
        t, tv, lc = (cfg[0], cfg[1], cfg[7]) if cfg[0] % nv == 0 else ({1: 8192, 4: 8192}.get(k, 16384), 16 if k in (1, 4) else 32, 0)
        hs.hsort_set_config(k, t, tv, nv, vt, cfg[4], fanin=4, digits=cfg[6], local=lc, size_class=c)
    say(f"fanin4 shape S={nv} VT={vt}")
    yield hs
    for (k, c), cfg in saved.items():
        hs.hsort_set_config(k, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=c)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def sort_checked(hs, k, vals=None):
    kind = (hs.PAIRS_I32_U32 if vals is not None else hs.KEYS_I32 if k.dtype == np.int32 else hs.KEYS_I64)
    t = dev(k)
    s = torch.empty(hs.scratch_bytes(kind, k.size), dtype=torch.uint8, device="cuda")
    if vals is not None:
        tv = dev(vals.view(np.int32))
        hs.hsort_pairs(t, tv, scratch=s)
        hs.hsort_check(s)
        return t.cpu().numpy(), tv.cpu().numpy().view(np.uint32)
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    return t.cpu().numpy()


@pytest.mark.parametrize("n", [8193, 16385, 40000, 65536 * 4 + 7, 2**20, 3_000_001, 2**23 + 5])
def test_uniform_sizes(hs4, orc, n):
    k = W.uniform_i32(n, n % 97)
    say(f"fanin4 uniform n={n}")
    assert np.array_equal(sort_checked(hs4, k), orc.sort_keys(k))


@pytest.mark.parametrize("name", ["all_equal", "sorted", "reverse", "extremes", "full_range", "three_digit",
                                  "two_values", "loguniform", "sawtooth", "one_bucket"])
def test_adversarial(hs4, orc, name):
    base = W.adversarial_i32()[name]
    k = np.tile(base, 8)[: 400_003]  # long enough for several rounds
    say(f"fanin4 adversarial {name}")
    assert np.array_equal(sort_checked(hs4, k), orc.sort_keys(k))


@pytest.mark.parametrize("n", [5000, 300_001, 2**21 + 3])
def test_int64(hs4, orc, n):
    I = np.iinfo(np.int64)
    k = np.random.default_rng(n).integers(I.min, I.max, n, dtype=np.int64, endpoint=True)
    say(f"fanin4 int64 n={n}")
    assert np.array_equal(sort_checked(hs4, k), orc.sort_keys(k))


@pytest.mark.parametrize("n", [4097, 300_001, 2**21 + 3])
def test_pairs_stable(hs4, orc, n):
    k, v = W.dup_pairs_i32(n, n)
    say(f"fanin4 pairs n={n}")
    gk, gv = sort_checked(hs4, k, v)
    ok, ov = orc.sort_pairs(k, v)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


@pytest.mark.parametrize("span", ["full_range", "near_narrow_limit", "small_negative"])
def test_pairs_word_widths(hs4, orc, span):
    # chunks spanning more or fewer than 2^19 - 1 key values merge on 64- or
    # 32-bit words; these mixes exercise both, and the limit itself
    n = 600_001
    r = np.random.default_rng(len(span))
    I = np.iinfo(np.int32)
    lo, hi = {"full_range": (I.min, I.max), "near_narrow_limit": (0, 2**19), "small_negative": (-300_000, 200_000)}[span]
    k = r.integers(lo, hi, n, dtype=np.int32, endpoint=True)
    v = r.integers(0, 2**32, n, dtype=np.uint32)
    say(f"fanin4 pairs word widths {span}")
    gk, gv = sort_checked(hs4, k, v)
    ok, ov = orc.sort_pairs(k, v)
    assert np.array_equal(gk, ok) and np.array_equal(gv, ov)


@pytest.mark.parametrize("dtype", [np.int32, np.int64])
def test_segmented(hs4, orc, dtype):
    keys, off = W.segments_i32(400, 2**17, 12)
    if dtype == np.int64:
        I = np.iinfo(np.int64)
        keys = np.random.default_rng(3).integers(I.min, I.max, keys.size, dtype=np.int64, endpoint=True)
    say(f"fanin4 segmented {np.dtype(dtype).name} n={keys.size}")
    kind = hs4.SEG_I32 if dtype == np.int32 else hs4.SEG_I64
    t, o = dev(keys), dev(off)
    s = torch.empty(hs4.scratch_bytes(kind, keys.size, 400), dtype=torch.uint8, device="cuda")
    hs4.hsort_segmented(t, o, max_seg_len=int(np.diff(off).max()), scratch=s)
    hs4.hsort_check(s)
    assert np.array_equal(t.cpu().numpy(), orc.sort_segmented(keys, off)[0])


def test_stage_local_sorts_parity_follows_fanin(hs4, orc):
    k = W.uniform_i32(300_000, 5)
    cfg = hs4.hsort_get_config(hs4.KEYS_I32, n=k.size)
    t = dev(k)
    hs4.hsort_debug_stage(t, 2)
    ok, _, b = orc.bucket_tiles(k, cfg[0], digits=cfg[6])
    check_keys_stage(t.cpu().numpy(), ok, b, 2, cfg[0], stable=cfg[6] == 1)
