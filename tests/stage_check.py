"""Comparison of a keys-only sort's intermediate with the oracle's.

With ten buckets, and for every pair sort, the GPU's bucket scatter is
stable, so its intermediates are compared bit for bit.  Keys-only sorts with
one hundred buckets place keys inside a bucket in any order (equal keys are
identical and the local sorts order the rest, so nothing of it reaches the
result): then what is unique is compared -- each bucket holds the oracle's
multiset of keys -- and what is left is checked for validity -- after the
local sorts every tile-key partition of every bucket is sorted.
"""
import numpy as np


def _bits(a):
    return np.ascontiguousarray(a).view(np.uint8).reshape(a.size, a.dtype.itemsize)


def same_multiset(a, b):
    """Equal as multisets of bit patterns (NaNs included)."""
    if a.size != b.size:
        return False
    ka = np.sort(np.ascontiguousarray(a).view(np.int32 if a.dtype.itemsize == 4 else np.int64))
    kb = np.sort(np.ascontiguousarray(b).view(np.int32 if b.dtype.itemsize == 4 else np.int64))
    return np.array_equal(ka, kb)


def check_keys_stage(got, want, bounds, stage, tile, stable, is_sorted=None):
    """got: GPU intermediate; want: the oracle's (stable) intermediate; bounds:
    the bucket bounds (10 or 100 buckets) of the input; stage 1 (scatter) or 2
    (local sorts of `tile`-key partitions).  is_sorted(part) tells whether a
    partition is in the sort's order (default: ascending signed order)."""
    if stable:
        assert np.array_equal(_bits(got), _bits(want)), f"stage {stage} differs from the oracle"
        return
    if is_sorted is None:
        def is_sorted(part):
            return bool(np.all(part[1:] >= part[:-1]))
    for b in range(len(bounds) - 1):
        lo, hi = int(bounds[b]), int(bounds[b + 1])
        assert same_multiset(got[lo:hi], want[lo:hi]), f"stage {stage}: bucket {b} holds other keys"
        if stage == 2:
            for s in range(lo, hi, tile):
                part = got[s:min(s + tile, hi)]
                assert is_sorted(part), f"stage 2: partition at {s} of bucket {b} is not sorted"
