"""Serving: continuous batching of encode/decode requests (Python side).

The request loop itself is native (``pyrit_server_run`` in the library);
this module stages inputs, turns a request trace into the C request array and
summarises latencies.  Inputs are resident in HBM before the run starts:
every request reads its blocks from one device pool of seeded random bytes
(read-only, so requests may share bytes); outputs come from the server's own
pool, whose size caps the working set.
"""
from __future__ import annotations

import ctypes
import dataclasses

import numpy as np

from . import Plan, PyritError, _check, _stream_handle  # noqa: F401
from ._lib import (BATCH_MODES, Request, RequestResult, ServeConfig, ServeStats, Tune, lib)


class InputPool:
    """Device bytes from the seeded generator; hands out block addresses."""

    def __init__(self, nbytes: int, key: int):
        import torch

        from . import fill_random
        self.nbytes = nbytes // 256 * 256
        self.key = key
        self.buf = torch.empty(self.nbytes, dtype=torch.uint8, device="cuda")
        fill_random(self.buf, key)
        torch.cuda.synchronize()
        self.base = int(self.buf.data_ptr())

    def offset(self, req: int, j: int, block_len: int) -> int:
        """Deterministic, spread-out offset of input block j of request req."""
        span = self.nbytes - block_len
        assert span > 0, "input pool smaller than one block"
        h = (req * 0x9E3779B1 + j * 0x85EBCA77 + 0x2545F491) & 0xFFFFFFFFFFFF
        return (h % (span // 256 + 1)) * 256


class Server:
    """The library's request loop (pyrit_server_*) with its output pool."""

    def __init__(self, pool_bytes: int = 64 << 30, slots: int = 4, max_batch: int = 0,
                 per_request: bool = False, release_outputs: bool = True,
                 block_skew: int = 4352, mode: str = "grid", wg_threads: int = 0,
                 tile_bytes: int = 0, slot_bytes: int = 0, large_bytes: int = 64 << 20,
                 xcd_order: int = 0, split_k: int = 0):
        cfg = ServeConfig(pool_bytes, slots, max_batch, 1 if per_request else 0,
                          1 if release_outputs else 0, block_skew, slot_bytes, large_bytes,
                          Tune(BATCH_MODES[mode], tile_bytes, 0, wg_threads, xcd_order, split_k))
        h = ctypes.c_void_p()
        _check(lib().pyrit_server_create(ctypes.byref(cfg), ctypes.byref(h)))
        self._h = h
        self.pool_base = int(lib().pyrit_server_pool(h))
        self.pool_bytes = pool_bytes

    def run(self, reqs):
        """Serve a prepared request array (see `prepare`); returns the
        per-request results (numpy structured array) and run statistics."""
        n = len(reqs)
        res = (RequestResult * max(1, n))()
        st = ServeStats()
        _check(lib().pyrit_server_run(self._h, reqs, n, res, ctypes.byref(st)))
        dt = np.dtype([("admit_s", "f8"), ("launch_s", "f8"), ("done_s", "f8"),
                       ("out_offset", "u8"), ("out_stride", "u8"), ("launch", "i4")])
        arr = np.array([(r.admit_s, r.launch_s, r.done_s, r.out_offset, r.out_stride, r.launch)
                        for r in res[:n]], dtype=dt)
        stats = {f: getattr(st, f) for f, _ in ServeStats._fields_}
        return arr, stats

    def close(self):
        if getattr(self, "_h", None):
            lib().pyrit_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Prepared:
    """C request array for a trace, plus what keeps it alive."""

    def __init__(self, array, keep, meta):
        self.array, self.keep, self.meta = array, keep, meta

    def __len__(self):
        return len(self.meta)


def prepare(trace, inputs: InputPool, plans: dict, pitch_align: int = 0) -> Prepared:
    """trace: workload Requests (arrival_s, stripe, large).  plans: dict keyed
    by (w, n, p, k, m) (filled as needed).  Blocks are packed (slice pitch =
    S) when ``pitch_align`` is 0; else each slice starts at the next multiple
    of ``pitch_align`` bytes (the stripes in ``meta`` then carry that padding)."""
    n = len(trace)
    arr = (Request * max(1, n))()
    keep, meta = [], []
    for i, rq in enumerate(trace):
        st = rq.stripe
        if pitch_align:
            st = dataclasses.replace(st, pad=-(-st.S // pitch_align) * pitch_align - st.S)
        key = (st.w, st.n, st.p, st.k, st.m)
        if key not in plans:
            plans[key] = Plan(*key)
        plan = plans[key]
        offs = [inputs.offset(i, j, st.block_len) for j in range(st.k)]
        ins = (ctypes.c_void_p * st.k)(*[inputs.base + o for o in offs])
        er = (ctypes.c_int * max(1, len(st.erased)))(*st.erased)
        keep += [ins, er]
        arr[i].arrival_s = rq.arrival_s
        arr[i].plan = plan._h
        arr[i].n_erased = len(st.erased)
        arr[i].erased = ctypes.cast(er, ctypes.POINTER(ctypes.c_int))
        arr[i].inputs = ctypes.cast(ins, ctypes.POINTER(ctypes.c_void_p))
        arr[i].slice_bytes = st.S
        arr[i].slice_pitch = st.pitch
        meta.append((st, offs, rq.large))
    return Prepared(arr, keep + [plans], meta)


def summarize(prep: Prepared, res, stats) -> dict:
    """Latency percentiles (arrival to observed completion, ms) overall and
    for small / large requests, and served throughput."""
    n = len(prep)
    arrival = np.array([prep.array[i].arrival_s for i in range(n)])
    lat = (res["done_s"] - arrival) * 1e3
    large = np.array([m[2] for m in prep.meta], dtype=bool)
    user = sum(st.k * st.B for st, _, _ in prep.meta)
    el = max(stats["elapsed_s"], 1e-9)

    def pct(x, q):
        return round(float(np.percentile(x, q)), 4) if len(x) else None

    return {"requests": n, "large": int(large.sum()),
            "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "mean_ms": round(float(lat.mean()), 4),
            "p50_ms_small": pct(lat[~large], 50), "p99_ms_small": pct(lat[~large], 99),
            "p50_ms_large": pct(lat[large], 50), "p99_ms_large": pct(lat[large], 99),
            "GBps_data": round(user / el / 1e9, 1),
            "GBps_moved": round(stats["moved_bytes"] / el / 1e9, 1),
            "elapsed_s": round(el, 4), "launches": stats["launches"],
            "mean_batch": round(stats["mean_batch"], 2), "max_batch": stats["max_batch_seen"],
            "peak_pool_GiB": round(stats["peak_pool_bytes"] / 2**30, 3),
            "admission_waits": stats["admission_waits"]}
