"""The allocation-free entry point (hsort_keys_i32_noalloc, scratch in a
library-owned device array) against the entry point it is a variant of
(hsort_keys_i32 with a caller scratch buffer), called through the C ABI:
bit-exact on consecutive calls whose sizes shrink (the largest size the
array holds first), and equal to the oracle."""
import ctypes
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def test_noalloc_matches_scratch_entry_point(orc):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2003_01216_amd as hs

    lib = hs.load_library()
    r = np.random.default_rng(77)
    cases = [
        W.uniform_i32(hs.NOALLOC_MAX_KEYS, 1),
        r.integers(-(2**31), 2**31 - 1, 1_000_003, dtype=np.int32, endpoint=True),
        r.integers(0, 1000, 40_001).astype(np.int32),
        W.uniform_i32(5000, 3),
    ]
    for k in cases:
        print(f"noalloc n={k.size}", flush=True)
        sys.stdout.flush()
        a = torch.from_numpy(k).cuda()
        b = a.clone()
        stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        rc = lib.hsort_keys_i32_noalloc(ctypes.c_void_p(a.data_ptr()), k.size, stream)
        assert rc == hs.HSORT_OK, lib.hsort_last_error()
        s = torch.empty(hs.scratch_bytes(hs.KEYS_I32, k.size), dtype=torch.uint8, device="cuda")
        rc = lib.hsort_keys_i32(ctypes.c_void_p(b.data_ptr()), k.size, ctypes.c_void_p(s.data_ptr()), s.numel(),
                                stream)
        assert rc == hs.HSORT_OK, lib.hsort_last_error()
        torch.cuda.synchronize()
        ga = a.cpu().numpy()
        assert np.array_equal(ga, b.cpu().numpy()), k.size
        assert np.array_equal(ga, orc.sort_keys(k)), k.size
