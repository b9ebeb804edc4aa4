"""Autotuner for batched launches.

For a batch it times a small set of executors (queue drain mode, threads per
workgroup, split-K, tile width, XCD-contiguous item order) in both launch forms (hipGraph
replay and direct dispatch) with HIP events on the caller's stream and keeps
the fastest.  Results are cached per batch signature (rings, k and output
ranges, slice-size class, decode share, stripe-count class, slice alignment)
in memory and in a JSON file
(``PYRIT_AUTOTUNE_CACHE``, default ``~/.cache/pyrit_mi355x_autotune.json``),
so a signature is only tuned once per machine.

Timing launches the batch itself, so tuning writes the batch's outputs (with
the bytes a real launch writes).
"""
from __future__ import annotations

import json
import math
import os
import threading

from . import Batch

CANDIDATES = [
    {"mode": "grid", "wg_threads": 128, "split_k": 2},
    {"mode": "grid", "wg_threads": 128, "split_k": 2, "xcd_order": 1},
    {"mode": "grid", "wg_threads": 256, "split_k": 2},
    {"mode": "grid", "wg_threads": 256, "split_k": 2, "xcd_order": 1},
    {"mode": "grid", "wg_threads": 64, "split_k": 1},
    {"mode": "grid", "wg_threads": 128, "split_k": 1},
    {"mode": "grid", "wg_threads": 256, "split_k": 1},
    {"mode": "grid", "wg_threads": 64, "split_k": 1, "xcd_order": 1},
    {"mode": "grid", "wg_threads": 128, "split_k": 1, "xcd_order": 1},
    {"mode": "grid", "wg_threads": 256, "split_k": 1, "xcd_order": 1},
    {"mode": "queue", "wg_threads": 256, "tile_bytes": 0},
    {"mode": "queue", "wg_threads": 256, "tile_bytes": 4096},
    {"mode": "static", "wg_threads": 128, "tile_bytes": 0},
]

_lock = threading.Lock()
_mem: dict = {}


def cache_path() -> str:
    return os.environ.get("PYRIT_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache",
                                       "pyrit_mi355x_autotune.json"))


def _load_file() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _save_file(d: dict) -> None:
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses persistence


def signature(items) -> str:
    """Batch class: rings present, k/outputs ranges, log2 slice size range,
    decode share, stripe-count class and the slice alignment (the largest
    power of two up to 4096 dividing every slice pitch)."""
    rings, ks, outs, sizes, dec, align = set(), [], [], [], 0, 4096
    for it in items:
        plan, erased, _, S = it[:4]
        pitch = it[4] if len(it) > 4 and it[4] else S
        rings.add((plan.w, plan.n, plan.p))
        ks.append(plan.k)
        outs.append(len(erased) if erased else plan.m)
        sizes.append(S)
        dec += 1 if erased else 0
        align = min(align, pitch & -pitch)
    n = len(ks)
    if n == 0:
        return "empty"
    return "|".join([
        "v5", ",".join(f"{w}/{nn}/{p:x}" for w, nn, p in sorted(rings)),
        f"k{min(ks)}-{max(ks)}", f"o{min(outs)}-{max(outs)}",
        f"s{int(math.log2(min(sizes)))}-{int(math.log2(max(sizes)))}",
        f"d{round(10 * dec / n)}", f"n{int(math.log2(n))}", f"a{align}",
    ])


def time_batch(batch, stream, reps: int = 5, form: str = "graph") -> float:
    import torch
    fn = batch.launch if form == "graph" else batch.launch_direct
    fn(stream)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(reps):
        fn(stream)
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b) / reps


def tuned_batch(items, stream=None, candidates=None, retune: bool = False, log=None):
    """A Batch of `items` built with the fastest known executor for their
    signature (tuning it now if unknown).  Returns (batch, config, timings)."""
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    items = list(items)
    sig = signature(items)
    with _lock:
        if not _mem:
            _mem.update(_load_file())
        cfg = None if retune else _mem.get(sig)
    if cfg is not None:
        return Batch(items, **cfg), cfg, None
    timings = []
    best, best_ms = None, float("inf")
    for cand in candidates or CANDIDATES:
        b = Batch(items, **cand)
        for form in ("graph", "direct"):
            c = dict(cand, launch=form)
            ms = time_batch(b, stream, form=form)
            timings.append((c, ms))
            if log:
                log(f"autotune {sig}: {c} {ms:.4f} ms")
            if ms < best_ms:
                best, best_ms = c, ms
        b.close()
    with _lock:
        _mem[sig] = dict(best)
        disk = _load_file()
        disk[sig] = dict(best)
        _save_file(disk)
    return Batch(items, **best), dict(best), timings
