"""The C-ABI library loads on the CPU and exports every symbol its header
declares; host-only entry points behave (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsort.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hsort_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    import paper_2003_01216_amd as hs

    return hs.load_library()


def test_header_lists_the_boundary():
    names = declared_functions()
    for must in ["hsort_keys_i32", "hsort_keys_i64", "hsort_pairs", "hsort_segmented", "hsort_segmented_i64",
                 "hsort_scratch_bytes", "hsort_check", "hsort_last_error"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_names_match_header():
    import paper_2003_01216_amd as hs

    assert sorted(hs.EXPORTS) == declared_functions()


def test_scratch_bytes_host_only(lib):
    import paper_2003_01216_amd as hs

    small = hs.scratch_bytes(hs.KEYS_I32, 1000)
    big = hs.scratch_bytes(hs.KEYS_I32, 1 << 20)
    assert 0 < small < big
    assert big >= 4 * (1 << 20)  # at least the ping-pong copy of the keys
    assert hs.scratch_bytes(hs.PAIRS_I32_U32, 1 << 20) >= 8 * (1 << 20)
    assert hs.scratch_bytes(hs.KEYS_I64, 1 << 20) >= 8 * (1 << 20)
    assert hs.scratch_bytes(hs.SEG_I32, 1 << 20, 5000) > hs.scratch_bytes(hs.SEG_I32, 1 << 20, 1)
    assert hs.scratch_bytes(99, 10, 1) == 0


def test_argument_errors_are_synchronous(lib):
    # rejected before any device work: no GPU is touched
    assert lib.hsort_keys_i32(None, 10, None, 0, None) == 1
    assert b"null" in lib.hsort_last_error()
    assert lib.hsort_keys_i32(None, -1, None, 0, None) == 1
    assert lib.hsort_keys_i32(None, 0, None, 0, None) == 0  # n == 0 is a no-op
    assert lib.hsort_keys_i64(None, 1 << 40, None, 0, None) == 4
    assert lib.hsort_segmented(None, 10, None, -1, 0, None, 0, None) == 1
    assert lib.hsort_segmented(None, 0, None, 0, 0, None, 0, None) == 0
    fake = ctypes.c_void_p(0x1000)
    assert lib.hsort_keys_i32(fake, 1 << 20, fake, 16, None) == 2  # scratch too small
    assert b"scratch" in lib.hsort_last_error()


def test_segment_count_and_hint_limits(lib):
    # more segments than the per-bucket tables can index: rejected before
    # anything is enqueued (10 * nseg buckets must stay within 32 bits)
    fake = ctypes.c_void_p(0x1000)
    big = (1 << 24) + 1
    assert lib.hsort_segmented(fake, 10, fake, big, 0, fake, 1 << 40, None) == 4
    assert b"HSORT_MAX_SEGMENTS" in lib.hsort_last_error()
    assert lib.hsort_segmented_i64(fake, 10, fake, (1 << 31) - 1, 0, fake, 1 << 40, None) == 4
    assert lib.hsort_segmented(fake, 10, fake, 3, -5, fake, 1 << 40, None) == 1  # negative hint
    assert b"max_seg_len" in lib.hsort_last_error()
    assert 10 * (1 << 24) < 2**31 - 1


def test_binding_passes_byte_counts(monkeypatch):
    # a scratch tensor of a wider dtype is sized in bytes, not elements
    import paper_2003_01216_amd as hs
    import torch

    t = torch.empty(7, dtype=torch.int64)
    assert hs._nbytes(t) == 56
    src = open(os.path.join(ROOT, "paper_2003_01216_amd", "__init__.py")).read()
    assert "s.numel()," not in src and "scratch.numel()," not in src


def test_config_roundtrip(lib):
    import paper_2003_01216_amd as hs

    assert [hs.hsort_size_class(n) for n in (1, 1 << 18, (1 << 18) + 1, 1 << 22, 1 << 26, 1 << 28)] == [0, 0, 1, 1, 2, 3]
    cfg = hs.hsort_get_config(hs.KEYS_I32, size_class=3)
    t, tvt, m, mvt, s, fanin, digits, local = cfg
    assert t % m == 0 and s <= 8192 and t % tvt == 0 and m % mvt == 0 and fanin in (2, 4) and digits in (1, 2, 3)
    with pytest.raises(hs.HsortError):
        hs.hsort_set_config(hs.KEYS_I32, 1000, 16, 4096, 16, 100)
    with pytest.raises(hs.HsortError):  # merge chunk does not divide the tile
        hs.hsort_set_config(hs.KEYS_I32, 4096, 16, 8192, 32, 100)
    with pytest.raises(hs.HsortError):  # fan-in must be 2 or 4
        hs.hsort_set_config(hs.KEYS_I32, t, tvt, m, mvt, s, fanin=3, size_class=3)
    with pytest.raises(hs.HsortError):  # digits must be 1, 2 or 3
        hs.hsort_set_config(hs.KEYS_I32, t, tvt, m, mvt, s, fanin=fanin, digits=4, size_class=3)
    with pytest.raises(hs.HsortError):  # one thousand buckets: plain int32 keys only
        hs.hsort_set_config(hs.SEG_I32, t, tvt, m, mvt, s, fanin=fanin, digits=3, size_class=3)
    with pytest.raises(hs.HsortError):
        hs.hsort_set_config(hs.PAIRS_I64_U32, 4096, 8, 2048, 8, 4096, fanin=4, digits=3, size_class=3)
    with pytest.raises(hs.HsortError):
        hs.hsort_set_config(hs.KEYS_I64, 4096, 16, 4096, 16, 4096, fanin=4, digits=3, size_class=3)
    pc = hs.hsort_get_config(hs.PAIRS_I32_U32, size_class=3)  # int32 pairs take one thousand buckets too
    hs.hsort_set_config(hs.PAIRS_I32_U32, *pc[:5], fanin=pc[5], digits=3, local=pc[7], size_class=3)
    assert hs.hsort_get_config(hs.PAIRS_I32_U32, size_class=3)[6] == 3
    hs.hsort_set_config(hs.PAIRS_I32_U32, *pc[:5], fanin=pc[5], digits=pc[6], local=pc[7], size_class=3)
    for d in (1, 2, 3):
        hs.hsort_set_config(hs.KEYS_I32, t, tvt, m, mvt, s, fanin=4, digits=d, size_class=3)
        assert hs.hsort_get_config(hs.KEYS_I32, size_class=3)[5:] == (4, d, local)
    with pytest.raises(hs.HsortError):  # local must be 0 or 1
        hs.hsort_set_config(hs.KEYS_I32, t, tvt, m, mvt, s, fanin=fanin, local=2, size_class=3)
    with pytest.raises(hs.HsortError):  # no bottom-up local sort of this shape
        hs.hsort_set_config(hs.KEYS_I32, 16384, 32, m, mvt, s, fanin=fanin, local=1, size_class=3)
    hs.hsort_set_config(hs.KEYS_I32, 2048, 2, 2048, 16, s, fanin=4, local=1, size_class=3)
    assert hs.hsort_get_config(hs.KEYS_I32, size_class=3)[7] == 1
    hs.hsort_set_config(hs.KEYS_I32, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=3)
    assert hs.hsort_get_config(hs.KEYS_I32, size_class=3) == cfg


def test_tuning_file(lib, tmp_path):
    import paper_2003_01216_amd as hs

    before = [hs.hsort_get_config(hs.KEYS_I64, size_class=c) for c in range(4)]
    f = tmp_path / "t.txt"
    f.write_text("# kind class tile tile_vt merge_nv merge_vt small_max fanin [digits]\n"
                 "1 2 8192 16 4096 16 2048 4\n1 3 8192 16 4096 16 2048 4 2\n")
    hs.hsort_load_tuning(str(f))
    assert hs.hsort_get_config(hs.KEYS_I64, size_class=2) == (8192, 16, 4096, 16, 2048, 4, 1, 0)
    assert hs.hsort_get_config(hs.KEYS_I64, size_class=3) == (8192, 16, 4096, 16, 2048, 4, 2, 0)
    assert hs.hsort_get_config(hs.KEYS_I64, size_class=1) == before[1]
    f.write_text("1 2 8192 16 4096 16 2048 4 5\n")
    with pytest.raises(hs.HsortError):
        hs.hsort_load_tuning(str(f))
    f.write_text("1 2 999 16 4096 16 2048 2\n")
    with pytest.raises(hs.HsortError):
        hs.hsort_load_tuning(str(f))
    for c, cfg in enumerate(before):
        hs.hsort_set_config(hs.KEYS_I64, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=c)


def test_noalloc_argument_errors(lib):
    # sizes beyond the library-owned scratch array are refused before any
    # device work, with a message naming the limit
    import paper_2003_01216_amd as hs

    assert hs.NOALLOC_MAX_KEYS == 4194304
    assert lib.hsort_keys_i32_noalloc(None, hs.NOALLOC_MAX_KEYS + 1, None) == hs.HSORT_ERR_UNSUPPORTED
    assert b"HSORT_NOALLOC_MAX_KEYS" in lib.hsort_last_error()
    assert lib.hsort_keys_i32_noalloc(None, -1, None) == hs.HSORT_ERR_INVALID
    assert lib.hsort_keys_i32_noalloc(None, 5, None) == hs.HSORT_ERR_INVALID
    assert lib.hsort_keys_i32_noalloc(None, 0, None) == hs.HSORT_OK
    # every size class's tuned shapes fit the array at the largest size
    assert hs.scratch_bytes(hs.KEYS_I32, hs.NOALLOC_MAX_KEYS) <= 24 << 20


def test_typed_sort_argument_errors(lib):
    import paper_2003_01216_amd as hs

    assert lib.hsort_sort(None, None, 10, 6, 0, None, 0, None) == hs.HSORT_ERR_INVALID  # unknown key type
    assert lib.hsort_sort(None, None, 10, 0, 2, None, 0, None) == hs.HSORT_ERR_INVALID  # unknown flag
    assert lib.hsort_sort(None, None, 10, hs.F32, hs.DESCENDING, None, 0, None) == hs.HSORT_ERR_INVALID  # null
    assert lib.hsort_sort(None, None, 0, hs.U64, 0, None, 0, None) == hs.HSORT_OK
    assert lib.hsort_debug_stage_typed(None, None, 10, hs.I32, 0, 4, None, 0, None) == hs.HSORT_ERR_INVALID
    n = 1 << 20
    assert hs.sort_scratch_bytes(hs.U32, False, n) == hs.scratch_bytes(hs.KEYS_I32, n)
    assert hs.sort_scratch_bytes(hs.F64, False, n) == hs.scratch_bytes(hs.KEYS_I64, n)
    assert hs.sort_scratch_bytes(hs.F32, True, n) == hs.scratch_bytes(hs.PAIRS_I32_U32, n)
    assert hs.sort_scratch_bytes(hs.I64, True, n) == hs.scratch_bytes(hs.PAIRS_I64_U32, n) >= 12 * n
    assert hs.sort_scratch_bytes(9, False, n) == 0
