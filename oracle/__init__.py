"""CPU oracle for the hybrid MSD-radix / quicksort / merge sort.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2003_01216_amd``) and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, single-threaded): chunked
quicksort (Figure 1c) and bottom-up merge (Figure 1b, Section 3.2) on the
composite (key, input index), plus the one-step decimal MSD bucket rule of
Section 3.4 computed with a real division.  This module only marshals numpy
arrays to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# the paper's method on the host's cores (OpenMP): a CPU comparison point for
# the benchmark, not the oracle
_OMP_SRC = os.path.join(_HERE, "omp_hybrid.c")
_OMP_LIB = os.path.join(_HERE, "libomp_hybrid.so")


def build(force: bool = False, src: str = _SRC, out: str = _LIB) -> str:
    """Compile oracle.c into liboracle.so with gcc (plain -O2, no OpenMP)."""
    if force or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(src):
        tmp = out + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared", "-o", tmp, src])
        os.replace(tmp, out)
    return out


def build_omp(force: bool = False) -> str:
    """Compile omp_hybrid.c into libomp_hybrid.so (gcc -O2 -fopenmp)."""
    if force or not os.path.exists(_OMP_LIB) or os.path.getmtime(_OMP_LIB) < os.path.getmtime(_OMP_SRC):
        tmp = _OMP_LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fopenmp", "-fPIC", "-shared", "-o", tmp,
                               _OMP_SRC])
        os.replace(tmp, _OMP_LIB)
    return _OMP_LIB


_omp = None


def omp_hybrid_sort(keys, threads: int = 0):
    """(sorted int32 keys, threads used): Section 3.4's one-step decimal MSD
    partition and the shared-memory quicksort + merge-round hybrid of
    Sections 3.2-3.3 on `threads` host threads (0: all OpenMP allows)."""
    global _omp
    if _omp is None:
        _omp = ctypes.CDLL(build_omp())
        _omp.omp_hybrid_sort_i32.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int]
        _omp.omp_hybrid_sort_i32.restype = ctypes.c_int
    k = np.ascontiguousarray(keys, dtype=np.int32).copy()
    used = _omp.omp_hybrid_sort_i32(_ptr(k), k.size, int(threads))
    if used < 0:
        raise RuntimeError("omp_hybrid_sort: allocation failed")
    return k, used


def _bind(path):
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64 = ctypes.c_int64
    I = ctypes.c_int
    sigs = {
        "oracle_plan_i32": [P, I64, P, P, P],
        "oracle_plan_i64": [P, I64, P, P, P],
        "oracle_bounds_i32": [P, I64, P],
        "oracle_bounds_i64": [P, I64, P],
        "oracle_sort_keys_i32": [P, I64],
        "oracle_sort_keys_i64": [P, I64],
        "oracle_sort_pairs_i32": [P, P, I64],
        "oracle_radix_sort_keys_i32": [P, I64, P],
        "oracle_radix_sort_keys_i64": [P, I64, P],
        "oracle_radix_sort_pairs_i32": [P, P, I64, P],
        "oracle_scatter_i32": [P, P, I64, P],
        "oracle_scatter_i64": [P, I64, P],
        "oracle_bucket_tiles_i32": [P, P, I64, I64, P],
        "oracle_bucket_tiles_i64": [P, I64, I64, P],
        "oracle_sort_segmented_i32": [P, P, I64, P],
        "oracle_sort_segmented_i64": [P, P, I64, P],
        "oracle_bounds_digits_i32": [P, I64, I, P],
        "oracle_bounds_digits_i64": [P, I64, I, P],
        "oracle_radix_sort_keys_digits_i32": [P, I64, I, P],
        "oracle_radix_sort_keys_digits_i64": [P, I64, I, P],
        "oracle_radix_sort_pairs_digits_i32": [P, P, I64, I, P],
        "oracle_scatter_digits_i32": [P, P, I64, I, P],
        "oracle_scatter_digits_i64": [P, I64, I, P],
        "oracle_bucket_tiles_digits_i32": [P, P, I64, I64, I, P],
        "oracle_bucket_tiles_digits_i64": [P, I64, I64, I, P],
    }
    for name, args in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    for name, args in {"oracle_sort_typed": [P, P, I, I, I64],
                       "oracle_bounds_typed": [P, I, I, I64, I, P],
                       "oracle_radix_sort_typed": [P, P, I, I, I64, I, P],
                       "oracle_stage_typed": [P, P, I, I, I64, I64, I, P]}.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.oracle_count_lt_le_i32.argtypes = [P, I64, ctypes.c_int32, P, P]
    lib.oracle_count_lt_le_i32.restype = None
    lib.oracle_count_lt_le_i64.argtypes = [P, I64, ctypes.c_int64, P, P]
    lib.oracle_count_lt_le_i64.restype = None
    return lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle: {what} failed (rc={rc})")


def _keys(a):
    a = np.ascontiguousarray(a)
    if a.dtype not in (np.int32, np.int64):
        raise TypeError("keys must be int32 or int64")
    return a.copy()


def _sfx(a):
    return "i32" if a.dtype == np.int32 else "i64"


# key types of the typed entry points (int32, uint32, float32, int64, uint64, float64)
KEY_TYPES = {np.dtype(np.int32): 0, np.dtype(np.uint32): 1, np.dtype(np.float32): 2,
             np.dtype(np.int64): 3, np.dtype(np.uint64): 4, np.dtype(np.float64): 5}


def _typed(a):
    a = np.ascontiguousarray(a)
    if a.dtype not in KEY_TYPES:
        raise TypeError(f"keys must be one of {[str(d) for d in KEY_TYPES]}")
    return a.copy(), KEY_TYPES[a.dtype]


def _vals(vals, n):
    if vals is None:
        return None
    v = np.ascontiguousarray(vals, dtype=np.uint32).copy()
    if v.size != n:
        raise ValueError("keys and vals differ in length")
    return v


def _nb(digits):
    if digits not in (1, 2, 3):
        raise ValueError("digits must be 1 (ten buckets), 2 (one hundred) or 3 (one thousand)")
    return 10**digits


class Oracle:
    """One loaded copy of the oracle library (the default one, or a variant)."""

    def __init__(self, path: str):
        self.path = path
        self._lib = _bind(path)

    def plan(self, keys):
        """(beta, D, p) of the decimal digit rule for this array."""
        k = np.ascontiguousarray(keys)
        beta = ctypes.c_int64()
        D = ctypes.c_int32()
        p = ctypes.c_uint64()
        fn = getattr(self._lib, "oracle_plan_" + _sfx(k))
        _check(fn(_ptr(k), k.size, ctypes.byref(beta), ctypes.byref(D), ctypes.byref(p)), "plan")
        return beta.value, D.value, p.value

    def bounds(self, keys, digits=1):
        """int64[10^digits + 1]: bounds[b] = number of keys whose bucket is below b (digits = 1: the
        ten-bucket rule, 2: the two-digit, hundred-bucket rule)."""
        k = np.ascontiguousarray(keys)
        out = np.zeros(_nb(digits) + 1, np.int64)
        if digits == 1:
            _check(getattr(self._lib, "oracle_bounds_" + _sfx(k))(_ptr(k), k.size, _ptr(out)), "bounds")
        else:
            _check(getattr(self._lib, "oracle_bounds_digits_" + _sfx(k))(_ptr(k), k.size, digits, _ptr(out)), "bounds")
        return out

    def sort_keys(self, keys):
        k = _keys(keys)
        _check(getattr(self._lib, "oracle_sort_keys_" + _sfx(k))(_ptr(k), k.size), "sort_keys")
        return k

    def sort_pairs(self, keys, vals):
        k = _keys(keys)
        if k.dtype != np.int32:
            raise TypeError("pairs take int32 keys")
        v = np.ascontiguousarray(vals, dtype=np.uint32).copy()
        _check(self._lib.oracle_sort_pairs_i32(_ptr(k), _ptr(v), k.size), "sort_pairs")
        return k, v

    def radix_sort_keys(self, keys, digits=1):
        """Section 3.4 run sequentially: scatter into the buckets, sort each."""
        k = _keys(keys)
        b = np.zeros(_nb(digits) + 1, np.int64)
        if digits == 1:
            fn, args = getattr(self._lib, "oracle_radix_sort_keys_" + _sfx(k)), (_ptr(k), k.size, _ptr(b))
        else:
            fn, args = getattr(self._lib, "oracle_radix_sort_keys_digits_" + _sfx(k)), (_ptr(k), k.size, digits, _ptr(b))
        _check(fn(*args), "radix_sort_keys")
        return k, b

    def radix_sort_pairs(self, keys, vals, digits=1):
        k = _keys(keys)
        v = np.ascontiguousarray(vals, dtype=np.uint32).copy()
        b = np.zeros(_nb(digits) + 1, np.int64)
        if digits == 1:
            _check(self._lib.oracle_radix_sort_pairs_i32(_ptr(k), _ptr(v), k.size, _ptr(b)), "radix_sort_pairs")
        else:
            _check(self._lib.oracle_radix_sort_pairs_digits_i32(_ptr(k), _ptr(v), k.size, digits, _ptr(b)),
                   "radix_sort_pairs")
        return k, v, b

    def scatter(self, keys, vals=None, digits=1):
        """The stable one-step MSD scatter alone: (keys, vals, bounds)."""
        k = _keys(keys)
        b = np.zeros(_nb(digits) + 1, np.int64)
        if k.dtype == np.int32:
            v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
            if digits == 1:
                _check(self._lib.oracle_scatter_i32(_ptr(k), _ptr(v), k.size, _ptr(b)), "scatter")
            else:
                _check(self._lib.oracle_scatter_digits_i32(_ptr(k), _ptr(v), k.size, digits, _ptr(b)), "scatter")
            return k, v, b
        if vals is not None:
            raise TypeError("int64 pairs are not supported")
        if digits == 1:
            _check(self._lib.oracle_scatter_i64(_ptr(k), k.size, _ptr(b)), "scatter")
        else:
            _check(self._lib.oracle_scatter_digits_i64(_ptr(k), k.size, digits, _ptr(b)), "scatter")
        return k, None, b

    def bucket_tiles(self, keys, tile, vals=None, digits=1):
        """Scatter, then sort each `tile`-key partition of every bucket."""
        k = _keys(keys)
        b = np.zeros(_nb(digits) + 1, np.int64)
        if k.dtype == np.int32:
            v = None if vals is None else np.ascontiguousarray(vals, dtype=np.uint32).copy()
            if digits == 1:
                rc = self._lib.oracle_bucket_tiles_i32(_ptr(k), _ptr(v), k.size, int(tile), _ptr(b))
            else:
                rc = self._lib.oracle_bucket_tiles_digits_i32(_ptr(k), _ptr(v), k.size, int(tile), digits, _ptr(b))
            _check(rc, "bucket_tiles")
            return k, v, b
        if vals is not None:
            raise TypeError("int64 pairs are not supported")
        if digits == 1:
            rc = self._lib.oracle_bucket_tiles_i64(_ptr(k), k.size, int(tile), _ptr(b))
        else:
            rc = self._lib.oracle_bucket_tiles_digits_i64(_ptr(k), k.size, int(tile), digits, _ptr(b))
        _check(rc, "bucket_tiles")
        return k, None, b

    def sort_segmented(self, keys, offsets):
        """Each [off[i], off[i+1]) sorted on its own.  Returns (keys, bounds[nseg,11])."""
        k = _keys(keys)
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        nseg = off.size - 1
        b = np.zeros((max(nseg, 0), 11), np.int64)
        fn = getattr(self._lib, "oracle_sort_segmented_" + _sfx(k))
        _check(fn(_ptr(k), _ptr(off), nseg, _ptr(b)), "sort_segmented")
        return k, b

    # -------------------------------------------------- other key types
    def sort_typed(self, keys, vals=None, descending=False):
        """Stable sort of int32/uint32/float32/int64/uint64/float64 keys (and a uint32 payload),
        ascending or descending; floats in IEEE-754 total order.  Returns (keys, vals)."""
        k, t = _typed(keys)
        v = _vals(vals, k.size)
        _check(self._lib.oracle_sort_typed(_ptr(k), _ptr(v), t, int(bool(descending)), k.size), "sort_typed")
        return k, v

    def bounds_typed(self, keys, descending=False, digits=1):
        """Bucket bounds of the keys' order image (see oracle.c) under the one-step rule."""
        k, t = _typed(keys)
        out = np.zeros(_nb(digits) + 1, np.int64)
        _check(self._lib.oracle_bounds_typed(_ptr(k), t, int(bool(descending)), k.size, digits, _ptr(out)),
               "bounds_typed")
        return out

    def radix_sort_typed(self, keys, vals=None, descending=False, digits=1):
        """Section 3.4 run sequentially on the order image: (keys, vals, bounds)."""
        k, t = _typed(keys)
        v = _vals(vals, k.size)
        b = np.zeros(_nb(digits) + 1, np.int64)
        _check(self._lib.oracle_radix_sort_typed(_ptr(k), _ptr(v), t, int(bool(descending)), k.size, digits,
                                                 _ptr(b)), "radix_sort_typed")
        return k, v, b

    def stage_typed(self, keys, vals=None, descending=False, tile=0, digits=1):
        """The stable bucket scatter (tile = 0) or the scatter followed by the local sorts of every
        `tile`-key partition of every bucket: (keys, vals, bounds)."""
        k, t = _typed(keys)
        v = _vals(vals, k.size)
        b = np.zeros(_nb(digits) + 1, np.int64)
        _check(self._lib.oracle_stage_typed(_ptr(k), _ptr(v), t, int(bool(descending)), k.size, int(tile), digits,
                                            _ptr(b)), "stage_typed")
        return k, v, b

    def count_lt_le(self, keys, x):
        """(#{k < x}, #{k <= x}): o[j] == x iff lt <= j < le."""
        k = np.ascontiguousarray(keys)
        lt = ctypes.c_int64()
        le = ctypes.c_int64()
        if k.dtype == np.int32:
            self._lib.oracle_count_lt_le_i32(_ptr(k), k.size, ctypes.c_int32(int(x)), ctypes.byref(lt), ctypes.byref(le))
        else:
            self._lib.oracle_count_lt_le_i64(_ptr(k), k.size, ctypes.c_int64(int(x)), ctypes.byref(lt), ctypes.byref(le))
        return lt.value, le.value


_default = None


def default() -> Oracle:
    global _default
    if _default is None:
        _default = Oracle(build())
    return _default


def load_variant(path: str) -> Oracle:
    """Bind a separately compiled copy of the oracle (used by mutation tests)."""
    return Oracle(path)


def __getattr__(name):
    if name in _PUBLIC:
        return getattr(default(), name)
    raise AttributeError(name)


_PUBLIC = {"plan", "bounds", "sort_keys", "sort_pairs", "radix_sort_keys", "radix_sort_pairs", "scatter",
           "bucket_tiles", "sort_segmented", "count_lt_le", "sort_typed", "bounds_typed", "radix_sort_typed",
           "stage_typed"}
