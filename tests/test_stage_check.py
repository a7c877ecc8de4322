"""The GPU tests' comparison of unstable keys-only intermediates must reject
a key in the wrong bucket and an unsorted partition, and accept any order
inside a bucket."""
import numpy as np
import pytest

from stage_check import check_keys_stage


def test_accepts_reordered_buckets_and_rejects_mistakes(orc):
    r = np.random.default_rng(5)
    k = r.integers(0, 10**6, 5000).astype(np.int32)
    want, _, b = orc.scatter(k, digits=2)
    got = want.copy()
    for i in range(100):  # any order inside each bucket
        lo, hi = int(b[i]), int(b[i + 1])
        got[lo:hi] = r.permutation(got[lo:hi])
    check_keys_stage(got, want, b, 1, 0, stable=False)
    with pytest.raises(AssertionError):
        check_keys_stage(got, want, b, 1, 0, stable=True)
    nz = [i for i in range(99) if b[i + 1] > b[i] and b[i + 2] > b[i + 1]][0]
    bad = got.copy()
    bad[b[nz + 1] - 1], bad[b[nz + 1]] = bad[b[nz + 1]], bad[b[nz + 1] - 1]  # swap across a bucket edge
    if not np.array_equal(np.sort(bad[b[nz]:b[nz + 1]]), np.sort(want[b[nz]:b[nz + 1]])):
        with pytest.raises(AssertionError):
            check_keys_stage(bad, want, b, 1, 0, stable=False)
    T = 64
    tiles, _, tb = orc.bucket_tiles(k, T, digits=2)
    check_keys_stage(tiles, tiles, tb, 2, T, stable=False)
    big = int(np.argmax(np.diff(tb)))
    unsorted = tiles.copy()
    seg = unsorted[tb[big]:tb[big] + T]
    seg[[0, -1]] = seg[[-1, 0]]
    with pytest.raises(AssertionError):
        check_keys_stage(unsorted, tiles, tb, 2, T, stable=False)
