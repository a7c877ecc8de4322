"""hsort: MI355X (gfx950) hybrid MSD-radix / tile-sort / merge-path integer sort.

A thin ctypes binding of ``libhsort.so`` (the C ABI in ``include/hsort.h``):
argument marshalling only, every step of the sort runs in the library's HIP
kernels.  PyTorch supplies device memory and the current stream.  The
functions have the C ABI's names and sort device tensors in place.

Method: Alghamdi & Alaghband, "High Performance Parallel Sort for Shared and
Distributed Memory MIMD" (arXiv 2003.01216), Section 3.4 -- a one-step decimal
most-significant-digit partition into ten buckets, a local sort of each
bucket's partitions, then non-recursive merge rounds of the sorted runs.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhsort.so")
# table written by `python -m paper_2003_01216_amd.autotune`; applied at load
TUNING_PATH = os.path.join(_HERE, "tuning.txt")

HSORT_OK = 0
HSORT_ERR_INVALID = 1
HSORT_ERR_SCRATCH = 2
HSORT_ERR_HIP = 3
HSORT_ERR_UNSUPPORTED = 4
HSORT_ERR_BUDGET = 5

KEYS_I32 = 0
KEYS_I64 = 1
PAIRS_I32_U32 = 2
SEG_I32 = 3
SEG_I64 = 4
PAIRS_I64_U32 = 5

# key types of hsort_sort
I32, U32, F32, I64, U64, F64 = range(6)
DESCENDING = 1
_KEY_TYPE_OF_DTYPE = {torch.int32: I32, torch.float32: F32, torch.int64: I64, torch.float64: F64}
for _name, _kt in (("uint32", U32), ("uint64", U64)):
    if hasattr(torch, _name):
        _KEY_TYPE_OF_DTYPE[getattr(torch, _name)] = _kt

EXPORTS = [
    "hsort_scratch_bytes",
    "hsort_keys_i32",
    "hsort_keys_i64",
    "hsort_keys_i32_noalloc",
    "hsort_pairs",
    "hsort_sort",
    "hsort_sort_scratch_bytes",
    "hsort_segmented",
    "hsort_segmented_i64",
    "hsort_bounds_offset",
    "hsort_check",
    "hsort_last_error",
    "hsort_set_config",
    "hsort_get_config",
    "hsort_size_class",
    "hsort_load_tuning",
    "hsort_debug_stage",
    "hsort_debug_stage_typed",
    "hsort_graph_mode",
    "hsort_graph_clear",
    "hsort_graph_count",
    "hsort_timing_enable",
    "hsort_timing_read",
    "hsort_copy",
]


class HsortError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hsort error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libhsort.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2003_01216_amd.build`")
    lib = ctypes.CDLL(path)
    P, I64, SZ, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t, ctypes.c_int
    sig = {
        "hsort_scratch_bytes": ([I, I64, I64], SZ),
        "hsort_keys_i32": ([P, I64, P, SZ, P], I),
        "hsort_keys_i64": ([P, I64, P, SZ, P], I),
        "hsort_keys_i32_noalloc": ([P, I64, P], I),
        "hsort_pairs": ([P, P, I64, P, SZ, P], I),
        "hsort_sort": ([P, P, I64, I, I, P, SZ, P], I),
        "hsort_sort_scratch_bytes": ([I, I, I64], SZ),
        "hsort_debug_stage_typed": ([P, P, I64, I, I, I, P, SZ, P], I),
        "hsort_segmented": ([P, I64, P, I64, I64, P, SZ, P], I),
        "hsort_segmented_i64": ([P, I64, P, I64, I64, P, SZ, P], I),
        "hsort_bounds_offset": ([I, I64, I64], SZ),
        "hsort_check": ([P, P], I),
        "hsort_last_error": ([], ctypes.c_char_p),
        "hsort_set_config": ([I, I, I64, I64, I64, I64, I64, I64, I64, I64], I),
        "hsort_get_config": ([I, I, P, P, P, P, P, P, P, P], I),
        "hsort_size_class": ([I64], I),
        "hsort_load_tuning": ([ctypes.c_char_p], I),
        "hsort_debug_stage": ([I, P, P, I64, I, P, SZ, P], I),
        "hsort_graph_mode": ([I], I),
        "hsort_graph_clear": ([], I),
        "hsort_graph_count": ([], I64),
        "hsort_timing_enable": ([I], I),
        "hsort_timing_read": ([P, I64], I64),
        "hsort_copy": ([P, P, I64, P], I),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    tune = os.environ.get("HSORT_TUNE_FILE", TUNING_PATH)
    if tune and os.path.exists(tune):
        _check(lib.hsort_load_tuning(tune.encode()))
    return lib


def _check(rc: int):
    if rc != HSORT_OK:
        raise HsortError(rc, load_library().hsort_last_error().decode())


def _stream(t: torch.Tensor):
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _dev_tensor(t, dtypes, what):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{what} must be a CUDA (HIP) tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{what} dtype must be one of {dtypes}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what} must be contiguous")


def scratch_bytes(kind: int, n: int, nseg: int = 1) -> int:
    return int(load_library().hsort_scratch_bytes(kind, n, nseg))


def bounds_offset(kind: int, n: int, nseg: int = 1) -> int:
    return int(load_library().hsort_bounds_offset(kind, n, nseg))


def _scratch(kind, n, nseg, device, scratch):
    need = scratch_bytes(kind, n, nseg)
    if scratch is None:
        return torch.empty(max(need, 1), dtype=torch.uint8, device=device)
    if _nbytes(scratch) < need:
        raise HsortError(HSORT_ERR_SCRATCH, f"scratch needs {need} bytes")
    return scratch


def _nbytes(t: torch.Tensor) -> int:
    return t.numel() * t.element_size()


def hsort_keys(keys: torch.Tensor, scratch: torch.Tensor | None = None) -> torch.Tensor:
    """Sort int32/int64 device keys in place (ascending); returns `keys`."""
    _dev_tensor(keys, (torch.int32, torch.int64), "keys")
    kind = KEYS_I32 if keys.dtype == torch.int32 else KEYS_I64
    n = keys.numel()
    s = _scratch(kind, n, 1, keys.device, scratch)
    fn = load_library().hsort_keys_i32 if kind == KEYS_I32 else load_library().hsort_keys_i64
    _check(fn(_ptr(keys), n, _ptr(s), _nbytes(s), _stream(keys)))
    return keys


def hsort_keys_i32(keys, scratch=None):
    if keys.dtype != torch.int32:
        raise TypeError("hsort_keys_i32 takes int32 keys")
    return hsort_keys(keys, scratch)


def hsort_keys_i64(keys, scratch=None):
    if keys.dtype != torch.int64:
        raise TypeError("hsort_keys_i64 takes int64 keys")
    return hsort_keys(keys, scratch)


def hsort_keys_i32_noalloc(keys: torch.Tensor) -> torch.Tensor:
    """Sort int32 device keys in place with the library's own scratch array (no allocation; at most
    HSORT_NOALLOC_MAX_KEYS keys; calls that overlap on one GPU race)."""
    _dev_tensor(keys, (torch.int32,), "keys")
    n = keys.numel()
    _check(load_library().hsort_keys_i32_noalloc(_ptr(keys), n, _stream(keys)))
    return keys


NOALLOC_MAX_KEYS = 4194304


def hsort_pairs(keys: torch.Tensor, vals: torch.Tensor, scratch: torch.Tensor | None = None):
    """Stable sort of int32 keys with a 32-bit payload (uint32 bits in an int32 tensor), in place."""
    _dev_tensor(keys, (torch.int32,), "keys")
    _dev_tensor(vals, (torch.int32, torch.uint32), "vals")
    if vals.numel() != keys.numel():
        raise ValueError("keys and vals differ in length")
    n = keys.numel()
    s = _scratch(PAIRS_I32_U32, n, 1, keys.device, scratch)
    _check(load_library().hsort_pairs(_ptr(keys), _ptr(vals), n, _ptr(s), _nbytes(s), _stream(keys)))
    return keys, vals


def _key_type(keys, key_type):
    if not isinstance(keys, torch.Tensor) or not keys.is_cuda:
        raise TypeError("keys must be a CUDA (HIP) tensor")
    if not keys.is_contiguous():
        raise ValueError("keys must be contiguous")
    if key_type is None:
        if keys.dtype not in _KEY_TYPE_OF_DTYPE:
            raise TypeError(f"no key type for dtype {keys.dtype}; pass key_type")
        key_type = _KEY_TYPE_OF_DTYPE[keys.dtype]
    if key_type not in range(6):
        raise ValueError("key_type must be one of I32, U32, F32, I64, U64, F64")
    if keys.element_size() != (4 if key_type < I64 else 8):
        raise TypeError("keys' element size does not match the key type")
    return key_type


def sort_scratch_bytes(key_type: int, with_vals: bool, n: int) -> int:
    return int(load_library().hsort_sort_scratch_bytes(key_type, 1 if with_vals else 0, n))


def hsort_sort(keys: torch.Tensor, vals: torch.Tensor | None = None, descending: bool = False,
               key_type: int | None = None, scratch: torch.Tensor | None = None):
    """Sort keys of any supported type in place (int32/uint32/float32/int64/uint64/float64, the type taken
    from the dtype or given as key_type for a tensor holding the bits), ascending or descending, stable,
    permuting a 32-bit payload `vals` with them; floats in IEEE-754 total order."""
    kt = _key_type(keys, key_type)
    n = keys.numel()
    if vals is not None:
        _dev_tensor(vals, (torch.int32,) + ((torch.uint32,) if hasattr(torch, "uint32") else ()), "vals")
        if vals.numel() != n:
            raise ValueError("keys and vals differ in length")
    need = sort_scratch_bytes(kt, vals is not None, n)
    if scratch is None:
        scratch = torch.empty(max(need, 1), dtype=torch.uint8, device=keys.device)
    elif _nbytes(scratch) < need:
        raise HsortError(HSORT_ERR_SCRATCH, f"scratch needs {need} bytes")
    _check(load_library().hsort_sort(_ptr(keys), _ptr(vals), n, kt, DESCENDING if descending else 0, _ptr(scratch),
                                     _nbytes(scratch), _stream(keys)))
    return keys, vals


def hsort_debug_stage_typed(keys: torch.Tensor, stage: int, vals: torch.Tensor | None = None,
                            descending: bool = False, key_type: int | None = None) -> torch.Tensor:
    """hsort_sort's pipeline up to `stage` (1 scatter, 2 local sorts, 3 all), in place."""
    kt = _key_type(keys, key_type)
    n = keys.numel()
    s = torch.empty(max(sort_scratch_bytes(kt, vals is not None, n), 1), dtype=torch.uint8, device=keys.device)
    _check(load_library().hsort_debug_stage_typed(_ptr(keys), _ptr(vals), n, kt, DESCENDING if descending else 0,
                                                  stage, _ptr(s), _nbytes(s), _stream(keys)))
    return keys


def hsort_segmented(keys: torch.Tensor, offsets: torch.Tensor, max_seg_len: int = 0,
                    scratch: torch.Tensor | None = None) -> torch.Tensor:
    """Sort every keys[offsets[i]:offsets[i+1]] in place (int32 or int64 keys, int64 offsets)."""
    _dev_tensor(keys, (torch.int32, torch.int64), "keys")
    _dev_tensor(offsets, (torch.int64,), "offsets")
    nseg = offsets.numel() - 1
    if nseg < 0:
        raise ValueError("offsets needs at least one entry")
    kind = SEG_I32 if keys.dtype == torch.int32 else SEG_I64
    n = keys.numel()
    s = _scratch(kind, n, max(nseg, 0), keys.device, scratch)
    fn = load_library().hsort_segmented if kind == SEG_I32 else load_library().hsort_segmented_i64
    _check(fn(_ptr(keys), n, _ptr(offsets), nseg, int(max_seg_len), _ptr(s), _nbytes(s), _stream(keys)))
    return keys


def hsort_check(scratch: torch.Tensor) -> None:
    """Synchronise the current stream and raise if the last call on `scratch` saw bad offsets."""
    _check(load_library().hsort_check(_ptr(scratch), _stream(scratch)))


def read_bounds(scratch: torch.Tensor, kind: int, n: int, nseg: int = 1) -> torch.Tensor:
    """The int64 [nseg, 11] bucket bounds the last call left in `scratch` (a view)."""
    off = bounds_offset(kind, n, nseg)
    return scratch[off: off + 8 * 11 * nseg].view(torch.int64).view(nseg, 11)


def hsort_set_config(kind: int, tile: int, tile_vt: int, merge_nv: int, merge_vt: int, small_max: int,
                     fanin: int = 2, size_class: int = -1, digits: int = 1, local: int = 0) -> None:
    _check(load_library().hsort_set_config(kind, size_class, tile, tile_vt, merge_nv, merge_vt, small_max, fanin,
                                           digits, local))


def hsort_set_config_tuple(kind: int, cfg, size_class: int = -1) -> None:
    """Apply a (tile, tile_vt, merge_nv, merge_vt, small_max, fanin, digits, local) tuple."""
    hsort_set_config(kind, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=size_class)


def hsort_get_config(kind: int, size_class: int | None = None, n: int | None = None):
    """(tile, tile_vt, merge_nv, merge_vt, small_max, fanin, digits, local) of a kind, for a size class or
    for n keys (default: 2^28)."""
    lib = load_library()
    if size_class is None:
        size_class = lib.hsort_size_class(n if n is not None else 1 << 28)
    vals = [ctypes.c_int64() for _ in range(8)]
    _check(lib.hsort_get_config(kind, size_class, *[ctypes.byref(v) for v in vals]))
    return tuple(v.value for v in vals)


def hsort_size_class(n: int) -> int:
    return int(load_library().hsort_size_class(n))


def hsort_load_tuning(path: str) -> None:
    _check(load_library().hsort_load_tuning(path.encode()))


def hsort_debug_stage(keys: torch.Tensor, stage: int, vals: torch.Tensor | None = None,
                      scratch: torch.Tensor | None = None) -> torch.Tensor:
    """Run the plain pipeline up to `stage` (1 scatter, 2 local sorts, 3 all) in place."""
    _dev_tensor(keys, (torch.int32, torch.int64), "keys")
    if vals is not None:
        kind = PAIRS_I32_U32
    else:
        kind = KEYS_I32 if keys.dtype == torch.int32 else KEYS_I64
    n = keys.numel()
    s = _scratch(kind, n, 1, keys.device, scratch)
    _check(load_library().hsort_debug_stage(kind, _ptr(keys), _ptr(vals), n, stage, _ptr(s), _nbytes(s),
                                            _stream(keys)))
    return keys


def hsort_graph_mode(on: bool) -> None:
    """Capture each distinct call into a hipGraph once and replay it afterwards."""
    load_library().hsort_graph_mode(1 if on else 0)


def hsort_graph_clear() -> None:
    load_library().hsort_graph_clear()


def hsort_graph_count() -> int:
    return int(load_library().hsort_graph_count())


def hsort_timing_enable(on: bool) -> None:
    load_library().hsort_timing_enable(1 if on else 0)


def hsort_timing_read() -> dict:
    """{kernel name: (launches, total_ms, algorithmic_bytes)} since the last read."""
    lib = load_library()
    buf = ctypes.create_string_buffer(1 << 16)
    lib.hsort_timing_read(buf, len(buf))
    out = {}
    for line in buf.value.decode().splitlines():
        name, launches, ms, by = line.split()
        out[name] = (int(launches), float(ms), float(by))
    return out


def hsort_copy(src: torch.Tensor, dst: torch.Tensor) -> None:
    nbytes = src.numel() * src.element_size()
    _check(load_library().hsort_copy(_ptr(src), _ptr(dst), nbytes, _stream(src)))
