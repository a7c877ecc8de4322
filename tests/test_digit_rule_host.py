"""The GPU library's decimal digit rules, checked on the host.

`tests/host/digit_rule_check.cpp` includes the library's device header and
compares digit_of (ten buckets), bucket2_of (one hundred buckets),
bucket3_of (one thousand, int32 keys) and bucket_span with integer division
by powers of ten written out in the check itself, for int32 and int64 keys
over every digit count, the edges of every bucket, negative minima and the
types' extremes (the one-step rule of Section 3.4 and its two- and
three-digit refinements).  No GPU is needed: the functions
are host-callable and the program launches nothing.
"""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_digit_rules_match_division(tmp_path):
    exe = tmp_path / "digit_rule_check"
    src = os.path.join(ROOT, "tests", "host", "digit_rule_check.cpp")
    inc = os.path.join(ROOT, "paper_2003_01216_amd", "csrc")
    subprocess.run([HIPCC, "--offload-arch=gfx950", "-O1", "-std=c++17", "-I", inc, src, "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "mismatches 0" in r.stdout
