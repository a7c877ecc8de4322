"""Autotuner for the local-sort and merge shapes.

For every key kind and size class it times each compiled shape on the
device -- tile (keys per local-sort partition) x keys per thread, merge
outputs per workgroup x per thread, the largest segment sorted wholly in
LDS, the merge fan-in (2 or 4 runs per round), the decimal digits of the
one-step partition (1: ten buckets, 2: one hundred) and the local sort (0:
network and lane merges, 1: bottom-up LDS merge) -- on a representative
synthetic workload of that class, and writes the
fastest to a table (``tuning.txt``, applied by the binding when the library
loads; see ``hsort_load_tuning``), and, with ``--report PATH``, a JSON log
of every measurement (a log, kept out of the package).

    python -m paper_2003_01216_amd.autotune [--quick] [--out tuning.txt]

Size classes (``hsort_size_class``): 0 up to 2^18 keys, 1 up to 2^22, 2 up
to 2^26, 3 above; a segmented call is classed by its longest segment.
"""
from __future__ import annotations

import argparse
import itertools
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import (KEYS_I32, KEYS_I64, PAIRS_I32_U32, PAIRS_I64_U32, SEG_I32, SEG_I64, TUNING_PATH, HsortError,
               hsort_graph_mode, hsort_keys, hsort_pairs, hsort_segmented, hsort_set_config, hsort_sort, load_library,
               scratch_bytes)

TILES = {
    KEYS_I32: [(8192, 16), (8192, 32), (16384, 32), (32768, 32)],
    KEYS_I64: [(4096, 16), (8192, 16)],
    PAIRS_I32_U32: [(4096, 16), (8192, 16)],
    PAIRS_I64_U32: [(2048, 8), (4096, 8)],
}
# merge shapes (outputs per workgroup, per thread) by fan-in; for fan-in 4
# the first number is also the sampling stride S (a workgroup holds <= 2S)
MERGES = {
    2: {KEYS_I32: [(4096, 16), (8192, 16), (8192, 32)], KEYS_I64: [(4096, 16)], PAIRS_I32_U32: [(4096, 16)],
        PAIRS_I64_U32: [(2048, 8)]},
    4: {KEYS_I32: [(4096, 16), (2048, 16), (2048, 8)], KEYS_I64: [(4096, 16), (2048, 16), (2048, 8)],
        PAIRS_I32_U32: [(4096, 16), (2048, 16), (2048, 8)], PAIRS_I64_U32: [(1024, 8), (2048, 8)]},
}
SMALL = {KEYS_I32: [8192], KEYS_I64: [4096], PAIRS_I32_U32: [4096], PAIRS_I64_U32: [4096]}
SEG_SMALL = [2048, 4096, 8192]
KEY_TYPE = {KEYS_I32: KEYS_I32, SEG_I32: KEYS_I32, KEYS_I64: KEYS_I64, SEG_I64: KEYS_I64, PAIRS_I32_U32: PAIRS_I32_U32,
            PAIRS_I64_U32: PAIRS_I64_U32}
CLASS_SIZES = {0: 1 << 18, 1: 1 << 22, 2: 1 << 26, 3: 1 << 28}
NAMES = {KEYS_I32: "keys_i32", KEYS_I64: "keys_i64", PAIRS_I32_U32: "pairs_i32", SEG_I32: "seg_i32", SEG_I64: "seg_i64",
         PAIRS_I64_U32: "pairs_i64"}


FANINS = [2, 4]
# decimal digits of the one-step partition: ten, one hundred or (plain
# int32 keys or pairs only) one thousand buckets
DIGITS = {KEYS_I32: [1, 2, 3], PAIRS_I32_U32: [1, 2, 3]}
DIGITS_DEFAULT = [1, 2]
# local-sort shapes of the bottom-up LDS merge (local = 1; Figure 1b from pairs when tile_vt = 2)
TILES_BU = {KEYS_I32: [(2048, 2), (4096, 8)], PAIRS_I32_U32: [(2048, 2)], KEYS_I64: [(2048, 2)]}


def candidates(kind):
    kt = KEY_TYPE[kind]
    smalls = SEG_SMALL if kind in (SEG_I32, SEG_I64) else SMALL[kt]
    tiles = [(t, tv, 0) for t, tv in TILES[kt]] + [(t, tv, 1) for t, tv in TILES_BU.get(kt, [])]
    for f in FANINS:
        for (t, tv, lc), (m, mv), s, d in itertools.product(tiles, MERGES[f][kt], smalls,
                                                            DIGITS.get(kind, DIGITS_DEFAULT)):
            if t % m == 0:
                yield (t, tv, m, mv, s, f, d, lc)


def _rng_keys(kind, n, seed):
    rng = np.random.default_rng(seed)
    if KEY_TYPE[kind] in (KEYS_I64, PAIRS_I64_U32):
        info = np.iinfo(np.int64)
        return rng.integers(info.min, info.max, n, dtype=np.int64, endpoint=True)
    return rng.integers(0, 2**31 - 1, n, dtype=np.int32)


def _segments(nseg, max_len, seed):
    rng = np.random.default_rng(seed)
    s = np.floor(np.exp(rng.random(nseg) * math.log(max_len + 1))).astype(np.int64)
    s = np.clip(s, 1, max_len)
    off = np.zeros(nseg + 1, np.int64)
    np.cumsum(s, out=off[1:])
    return off


class Workload:
    """A resident input of one class and a callable that sorts a fresh copy."""

    def __init__(self, kind, cls, quick):
        self.kind = kind
        dev = torch.device("cuda")
        if kind in (SEG_I32, SEG_I64):
            if cls == 0:
                nseg, max_len = (4096 if quick else 16384), 1 << 16
            else:
                max_len = min(CLASS_SIZES[cls], 1 << 24)
                nseg = max(4, (1 << (25 if not quick else 23)) // max_len * 4)
            off = _segments(nseg, max_len, 11 + cls)
            self.n = int(off[-1])
            self.max_len = int(np.diff(off).max())
            self.off = torch.from_numpy(off).to(dev)
            self.base = torch.from_numpy(_rng_keys(kind, self.n, 5 + cls)).to(dev)
            self.nseg = nseg
        else:
            n = CLASS_SIZES[cls]
            if KEY_TYPE[kind] != KEYS_I32 and cls == 3:
                n = 1 << 27
            if quick:
                n = min(n, 1 << 24)
            self.n = n
            self.base = torch.from_numpy(_rng_keys(kind, n, 5 + cls)).to(dev)
            if kind in (PAIRS_I32_U32, PAIRS_I64_U32):
                self.vals = torch.arange(n, dtype=torch.int32, device=dev)
            self.nseg = 1

    def scratch(self):
        return torch.empty(max(scratch_bytes(self.kind, self.n, self.nseg), 1), dtype=torch.uint8, device="cuda")

    def run(self, keys, vals, scratch):
        if self.kind in (SEG_I32, SEG_I64):
            hsort_segmented(keys, self.off, max_seg_len=self.max_len, scratch=scratch)
        elif self.kind == PAIRS_I32_U32:
            hsort_pairs(keys, vals, scratch=scratch)
        elif self.kind == PAIRS_I64_U32:
            hsort_sort(keys, vals, scratch=scratch)
        else:
            hsort_keys(keys, scratch=scratch)


def time_config(wl, cfg, cls, reps):
    """Median time of `reps` sorts of a fresh copy, after one warm-up call.

    The same buffers are sorted every time (refilled outside the timed
    window), so in graph mode the warm-up captures and the timed calls replay.
    """
    hsort_set_config(wl.kind, *cfg[:5], fanin=cfg[5], digits=cfg[6], local=cfg[7], size_class=cls)
    scratch = wl.scratch()
    work = wl.base.clone()
    wv = wl.vals.clone() if wl.kind in (PAIRS_I32_U32, PAIRS_I64_U32) else None
    times = []
    for r in range(reps + 1):
        work.copy_(wl.base)
        if wv is not None:
            wv.copy_(wl.vals)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        wl.run(work, wv, scratch)
        b.record()
        torch.cuda.synchronize()
        if r > 0:
            times.append(a.elapsed_time(b))
    if wl.kind not in (SEG_I32, SEG_I64):
        assert bool(torch.all(work[1:] >= work[:-1]).item()), f"unsorted output for {cfg}"
    del work, wv, scratch
    return float(np.median(times))


def tune(kinds, classes, quick=False, reps=5, log=print):
    load_library()
    hsort_graph_mode(True)
    table, report = {}, []
    try:
        for kind in kinds:
            for cls in classes:
                wl = Workload(kind, cls, quick)
                best = None
                for cfg in candidates(kind):
                    try:
                        ms = time_config(wl, cfg, cls, reps)
                    except HsortError as e:
                        log(f"  {NAMES[kind]} class {cls} {cfg}: {e}")
                        continue
                    gk = wl.n / ms / 1e6
                    report.append({"kind": NAMES[kind], "class": cls, "n": wl.n, "config": cfg, "ms": round(ms, 4),
                                   "Gkeys_s": round(gk, 3)})
                    log(f"  {NAMES[kind]:9s} class {cls} n={wl.n:>10d} {cfg}: {ms:8.3f} ms  {gk:7.2f} Gkeys/s")
                    # the bottom-up local sort must win by 2 % (it is slower at every measured size; a
                    # closer call on a small sample is noise)
                    if best is None or ms * (1.02 if cfg[7] else 1.0) < best[0] * (1.02 if best[1][7] else 1.0):
                        best = (ms, cfg)
                table[(kind, cls)] = best[1]
                hsort_set_config(kind, *best[1][:5], fanin=best[1][5], digits=best[1][6], local=best[1][7], size_class=cls)
                del wl
                torch.cuda.empty_cache()
    finally:
        hsort_graph_mode(False)
    return table, report


def read_table(path):
    """{(kind, class): config tuple} of an existing tuning file (missing columns take their defaults)."""
    table = {}
    with open(path) as f:
        for line in f:
            if not line.strip() or line.startswith("#"):
                continue
            x = [int(v) for v in line.split()]
            cfg = tuple(x[2:10]) + (1, 0)[len(x) - 8:] if len(x) < 10 else tuple(x[2:10])
            table[(x[0], x[1])] = cfg
    return table


def write_table(table, path, report=None, report_path=None):
    lines = ["# hsort tuning table: kind size_class tile tile_vt merge_nv merge_vt small_max fanin digits local",
             f"# written by paper_2003_01216_amd.autotune on {time.strftime('%Y-%m-%d %H:%M:%S')}"]
    for (kind, cls), cfg in sorted(table.items()):
        lines.append(f"{kind} {cls} " + " ".join(str(x) for x in cfg))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")
    if report is not None and report_path:
        os.makedirs(os.path.dirname(os.path.abspath(report_path)), exist_ok=True)
        with open(report_path, "w") as f:
            json.dump(report, f, indent=1)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--out", default=TUNING_PATH)
    ap.add_argument("--report", default="", help="write the JSON log of every measurement to this path")
    ap.add_argument("--quick", action="store_true", help="smaller workloads (sizes capped at 2^24)")
    ap.add_argument("--kinds", default="keys_i32,keys_i64,pairs_i32,seg_i32,seg_i64,pairs_i64")
    ap.add_argument("--classes", default="0,1,2,3")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--update", action="store_true",
                    help="keep the rows of the existing --out file that this run does not tune")
    args = ap.parse_args(argv)
    by_name = {v: k for k, v in NAMES.items()}
    kinds = [by_name[k] for k in args.kinds.split(",")]
    classes = [int(c) for c in args.classes.split(",")]
    t0 = time.time()
    table, report = tune(kinds, classes, args.quick, args.reps, log=lambda m: print(m, flush=True))
    if args.update and os.path.exists(args.out):
        table = {**read_table(args.out), **table}
    write_table(table, args.out, report, args.report)
    print(f"wrote {args.out} ({len(table)} entries) in {time.time() - t0:.0f} s", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
