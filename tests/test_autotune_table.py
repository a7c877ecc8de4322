"""The tuner's table file: what it writes reads back the same, rows written
without the optional digits and local-sort columns take their defaults, and
an --update run keeps the rows it does not measure.  Host only."""
import pytest

torch = pytest.importorskip("torch")

from paper_2003_01216_amd import autotune  # noqa: E402


def test_roundtrip_and_defaults(tmp_path):
    t = {(0, 3): (16384, 32, 2048, 16, 8192, 4, 3, 0), (5, 1): (2048, 8, 2048, 8, 4096, 2, 2, 0)}
    p = tmp_path / "t.txt"
    autotune.write_table(t, str(p))
    assert autotune.read_table(str(p)) == t
    p.write_text("# comment\n1 2 4096 16 4096 16 4096 2\n2 0 4096 16 4096 16 4096 4 2\n")
    assert autotune.read_table(str(p)) == {(1, 2): (4096, 16, 4096, 16, 4096, 2, 1, 0),
                                          (2, 0): (4096, 16, 4096, 16, 4096, 4, 2, 0)}


def test_update_keeps_other_rows(tmp_path, monkeypatch):
    p = tmp_path / "t.txt"
    old = {(0, 3): (16384, 32, 2048, 16, 8192, 4, 2, 0), (1, 3): (8192, 16, 4096, 16, 4096, 2, 2, 0)}
    autotune.write_table(old, str(p))
    new = {(0, 3): (32768, 32, 2048, 16, 8192, 4, 3, 0)}
    monkeypatch.setattr(autotune, "tune", lambda *a, **k: (new, []))
    autotune.main(["--out", str(p), "--kinds", "keys_i32", "--classes", "3", "--update"])
    assert autotune.read_table(str(p)) == {**old, **new}
    autotune.main(["--out", str(p), "--kinds", "keys_i32", "--classes", "3"])
    assert autotune.read_table(str(p)) == new
