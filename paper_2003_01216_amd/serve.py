"""Continuous-batching sort server over the segmented int64 sort.

Requests (host int64 arrays) arrive at any time through ``submit``; each
returns a Future that resolves to the sorted array.  Requests wait in one
FIFO queue.  ``streams`` workers each own a HIP stream; a free worker takes
the longest FIFO prefix of waiting requests that fits both its batch cap and
the HBM budget still free, copies them into one device buffer, sorts every
request as its own segment with one ``hsort_segmented_i64`` call, copies the
result back and resolves the futures.  Requests that arrive while batches
are on the GPU join the next batch as soon as a worker and memory free up,
so work from several batches overlaps on the device.

Budget accounting: a batch holds device bytes for its keys, its offsets and
the sort's scratch until its results are back on the host; the sum over
batches in flight never exceeds ``hbm_budget``.  A request that cannot fit
the whole budget on its own is rejected at once with HSORT_ERR_BUDGET.

Each request is sorted independently of the others it is batched with, so
its result is bit-identical alone and in any mix.

The executor is pluggable: ``GpuExecutor`` (default) runs on the device;
tests drive the scheduler with a CPU executor.
"""
from __future__ import annotations

import collections
import os
import threading
import time
from concurrent.futures import Future, ThreadPoolExecutor

import numpy as np

from . import HSORT_ERR_BUDGET, HsortError

_SEG_I64 = 4


_PIECE = 1 << 20  # elements per host copy task


def _copy_pieces(pool, pairs):
    """Copies every (dst, src) pair of equal-size arrays, large ones split into
    pieces, on the thread pool (numpy releases the GIL while it copies: one
    thread moves about 6 GB/s, eight about 30 GB/s on a host here)."""
    tasks = []
    for dst, src in pairs:
        for i in range(0, src.size, _PIECE):
            tasks.append(pool.submit(np.copyto, dst[i: i + _PIECE], src[i: i + _PIECE]))
    for t in tasks:
        t.result()


class GpuExecutor:
    """Sorts a batch on one HIP stream; buffers come from torch's caching
    allocator (they stay on the device between batches) and pinned staging
    buffers that grow as needed.  Host copies into and out of the staging
    buffers run on a thread pool shared by all streams."""

    def __init__(self, device="cuda", copy_threads=None):
        import torch

        from . import load_library

        self.torch = torch
        self.device = torch.device(device)
        self.lib = load_library()
        self.pool = ThreadPoolExecutor(copy_threads or min(16, os.cpu_count() or 4), thread_name_prefix="hsort-copy")

    def batch_bytes(self, total_keys, nseg):
        return 8 * total_keys + 8 * (nseg + 1) + int(self.lib.hsort_scratch_bytes(_SEG_I64, total_keys, nseg))

    def make_slot(self):
        torch = self.torch
        return {"stream": torch.cuda.Stream(self.device), "pin_in": None, "pin_out": None}

    def _pinned(self, slot, name, n):
        torch = self.torch
        buf = slot[name]
        if buf is None or buf.numel() < n:
            buf = torch.empty(max(n, 1 << 20), dtype=torch.int64, pin_memory=True)
            slot[name] = buf
        return buf[:n]

    def run(self, slot, arrays):
        import ctypes

        torch = self.torch
        from . import _check

        sizes = np.array([a.size for a in arrays], np.int64)
        off = np.zeros(sizes.size + 1, np.int64)
        np.cumsum(sizes, out=off[1:])
        n = int(off[-1])
        pin_in = self._pinned(slot, "pin_in", n)
        host_in = pin_in.numpy()
        _copy_pieces(self.pool, [(host_in[s: s + a.size], a) for a, s in zip(arrays, off[:-1])])
        st = slot["stream"]
        with torch.cuda.stream(st):
            keys = torch.empty(n, dtype=torch.int64, device=self.device)
            doff = torch.empty(off.size, dtype=torch.int64, device=self.device)
            scratch = torch.empty(max(int(self.lib.hsort_scratch_bytes(_SEG_I64, n, sizes.size)), 1),
                                  dtype=torch.uint8, device=self.device)
            keys.copy_(pin_in, non_blocking=True)
            doff.copy_(torch.from_numpy(off), non_blocking=False)
            _check(self.lib.hsort_segmented_i64(ctypes.c_void_p(keys.data_ptr()), n, ctypes.c_void_p(doff.data_ptr()),
                                                sizes.size, int(sizes.max()), ctypes.c_void_p(scratch.data_ptr()),
                                                scratch.numel() * scratch.element_size(),
                                                ctypes.c_void_p(st.cuda_stream)))
            pin_out = self._pinned(slot, "pin_out", n)
            pin_out.copy_(keys, non_blocking=True)
            st.synchronize()
            _check(self.lib.hsort_check(ctypes.c_void_p(scratch.data_ptr()), ctypes.c_void_p(st.cuda_stream)))
            host_out = pin_out.numpy()
            results = [np.empty(a.size, np.int64) for a in arrays]
            _copy_pieces(self.pool, [(r, host_out[s: s + a.size]) for r, a, s in zip(results, arrays, off[:-1])])
            del keys, doff, scratch  # back to the caching allocator, after the stream is idle
        return results


class _Request:
    __slots__ = ("keys", "future", "t_submit", "t_done")

    def __init__(self, keys):
        self.keys = keys
        self.future = Future()
        self.t_submit = time.perf_counter()
        self.t_done = None


class SortServer:
    def __init__(self, hbm_budget=64 << 30, streams=2, max_batch_keys=1 << 26, max_batch_requests=4096,
                 executor=None):
        self.executor = executor if executor is not None else GpuExecutor()
        self.hbm_budget = int(hbm_budget)
        self.max_batch_keys = int(max_batch_keys)
        self.max_batch_requests = int(max_batch_requests)
        self._queue = collections.deque()
        self._cv = threading.Condition()
        self._in_flight_bytes = 0
        self._peak_bytes = 0
        self._closed = False
        self._done = []
        self._batches = []  # (t_start, t_end, requests, keys) per batch
        self._keys_done = 0
        self._budget_waits = 0  # times a free worker found requests waiting but too little budget free
        self._workers = []
        for i in range(streams):
            th = threading.Thread(target=self._worker, args=(self.executor.make_slot(),), daemon=True,
                                  name=f"hsort-serve-{i}")
            th.start()
            self._workers.append(th)

    # ------------------------------------------------------------- clients
    def submit(self, keys) -> Future:
        a = np.ascontiguousarray(keys, dtype=np.int64)
        req = _Request(a)
        need = self.executor.batch_bytes(a.size, 1)
        if need > self.hbm_budget:
            req.future.set_exception(HsortError(HSORT_ERR_BUDGET, f"request of {a.size} keys needs {need} bytes, "
                                                                   f"more than the {self.hbm_budget}-byte budget"))
            return req.future
        with self._cv:
            if self._closed:
                raise RuntimeError("server is closed")
            self._queue.append(req)
            self._cv.notify_all()
        return req.future

    def close(self, wait=True):
        with self._cv:
            self._closed = True
            self._cv.notify_all()
        if wait:
            for th in self._workers:
                th.join()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # ------------------------------------------------------------ batching
    def _take_batch(self):
        """Longest FIFO prefix that fits the batch caps and the free budget."""
        batch, keys = [], 0
        while self._queue and len(batch) < self.max_batch_requests:
            r = self._queue[0]
            if batch and keys + r.keys.size > self.max_batch_keys:
                break
            need = self.executor.batch_bytes(keys + r.keys.size, len(batch) + 1)
            if self._in_flight_bytes + need > self.hbm_budget:
                break
            batch.append(self._queue.popleft())
            keys += r.keys.size
        if not batch:
            return None, 0
        need = self.executor.batch_bytes(keys, len(batch))
        self._in_flight_bytes += need
        self._peak_bytes = max(self._peak_bytes, self._in_flight_bytes)
        return batch, need

    def _worker(self, slot):
        while True:
            with self._cv:
                while True:
                    if self._queue:
                        batch, need = self._take_batch()
                        if batch:
                            break
                        self._budget_waits += 1
                    elif self._closed:
                        return
                    self._cv.wait()
            t0 = time.perf_counter()
            try:
                results = self.executor.run(slot, [r.keys for r in batch])
                err = None
            except Exception as e:  # noqa: BLE001 -- delivered to every caller of the batch
                results, err = None, e
            t1 = time.perf_counter()
            with self._cv:
                self._in_flight_bytes -= need
                self._batches.append((t0, t1, len(batch), sum(r.keys.size for r in batch)))
                self._cv.notify_all()
            for i, r in enumerate(batch):
                r.t_done = time.perf_counter()
                if err is None:
                    r.future.set_result(results[i])
                    with self._cv:
                        self._done.append(r)
                        self._keys_done += r.keys.size
                else:
                    r.future.set_exception(err)

    # --------------------------------------------------------------- stats
    def stats(self):
        with self._cv:
            done = list(self._done)
            batches = list(self._batches)
            peak = self._peak_bytes
            waits = self._budget_waits
        if not done:
            return {"requests": 0, "budget_waits": waits}
        lat = np.array([(r.t_done - r.t_submit) * 1e3 for r in done])
        t0 = min(r.t_submit for r in done)
        t1 = max(r.t_done for r in done)
        keys = sum(r.keys.size for r in done)
        overlap = 0.0
        if len(batches) > 1:  # time during which two or more batches were in the executor
            ev = sorted([(b[0], 1) for b in batches] + [(b[1], -1) for b in batches])
            depth, last = 0, None
            for t, d in ev:
                if depth >= 2 and last is not None:
                    overlap += t - last
                depth += d
                last = t
        return {"requests": len(done), "keys": int(keys), "wall_s": t1 - t0,
                "Gkeys_s": keys / (t1 - t0) / 1e9, "p50_ms": float(np.percentile(lat, 50)),
                "p99_ms": float(np.percentile(lat, 99)), "mean_ms": float(lat.mean()), "batches": len(batches),
                "mean_batch_requests": float(np.mean([b[2] for b in batches])) if batches else 0.0,
                "peak_in_flight_bytes": int(peak), "overlap_s": overlap, "budget_waits": waits}
