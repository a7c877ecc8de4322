"""The largest plain sort the library accepts: HSORT_MAX_KEYS = 2^31 - 1 int32 keys.

Every element index of the path is 32-bit (destinations, in-tile offsets,
descriptor counts) and the scans recurse over levels of block sums; this
size reaches the top of both.  The oracle would take minutes here, so the
output is checked by properties that fix it: it is sorted; it has the
input's multiset by independent sums over all keys (plain, sum of squares
and a multiplicative hash with 64-bit wraparound, and the exact histogram of
the low 16 bits); and
sampled order statistics meet the counting definition against the input on
the host (#(k < v) <= r < #(k <= v) for the key v at rank r).  The ten
bucket bounds are compared with counts of the input on the host.
"""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MAX_KEYS = 2**31 - 1


@pytest.fixture(scope="module")
def hs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if torch.cuda.get_device_properties(0).total_memory < (48 << 30):
        pytest.skip("needs about 26 GiB of device memory")
    import paper_2003_01216_amd as hs

    hs.load_library()
    return hs


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def sums(t):
    """Plain sum, sum of squares and a multiplicative hash (64-bit wraparound),
    and the exact histogram of the low 16 bits, in pieces of 2^27 keys."""
    mod = 1 << 64
    plain, squares, hashed = 0, 0, 0
    low = torch.zeros(1 << 16, dtype=torch.int64, device=t.device)
    for i in range(0, t.numel(), 1 << 27):
        x = t[i:i + (1 << 27)].to(torch.int64)
        plain += int(x.sum())
        squares = (squares + int((x * x).sum())) % mod
        hashed = (hashed + int(((x * -7046029254386353131) ^ (x >> 7)).sum())) % mod
        low += torch.bincount(x & 0xFFFF, minlength=1 << 16)
    return plain, squares, hashed, low.cpu().numpy()


def test_max_keys_uniform_int32(hs):
    n = MAX_KEYS
    assert hs.scratch_bytes(hs.KEYS_I32, n) < (16 << 30)
    k = W.uniform_i32(n, 31)
    say(f"max size: int32 keys n={n} cfg={hs.hsort_get_config(hs.KEYS_I32, n=n)}")
    t = torch.from_numpy(k).cuda()
    before = sums(t)
    torch.cuda.synchronize()
    s = torch.empty(hs.scratch_bytes(hs.KEYS_I32, n), dtype=torch.uint8, device="cuda")
    hs.hsort_keys(t, scratch=s)
    hs.hsort_check(s)
    torch.cuda.synchronize()
    say("max size: sorted, checking")
    assert bool(torch.all(t[1:] >= t[:-1]).item()), "not sorted"
    after = sums(t)
    assert after[:3] == before[:3], "multiset sums"
    assert np.array_equal(after[3], before[3]), "multiset low-16-bit histogram"
    for r in (0, 1, n // 7, n // 3, n // 2, n - 2, n - 1):
        v = int(t[r].item())
        lt = int(np.count_nonzero(k < v))
        le = lt + int(np.count_nonzero(k == v))
        assert lt <= r < le, (r, v, lt, le)
    # the ten-bucket bounds: keys in [0, 2^31-1) have ten digits, bucket b holds [b*10^9, (b+1)*10^9)
    b = hs.read_bounds(s, hs.KEYS_I32, n).cpu().numpy()[0]
    expect = [int(np.count_nonzero(k < d * 10**9)) for d in range(10)] + [n]
    assert np.array_equal(b, np.array(expect, np.int64)), (b, expect)
