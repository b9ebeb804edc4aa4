"""Host side of the autotuner and the benchmark (no GPU needed): batch
signatures, the cache file, every candidate executor being one
pyrit_batch_describe accepts, and the benchmark's one-GPU rule."""
import json

import paper_1709_00178_amd as P
from paper_1709_00178_amd import autotune
from paper_1709_00178_amd import workloads as W

BASE = 1 << 36


def items_for(stripes, align=0):
    plans, items, addr = {}, [], BASE
    for st in stripes:
        key = (st.w, st.n, st.p, st.k, st.m)
        plans.setdefault(key, P.Plan(*key))
        pitch = -(-st.S // align) * align if align else st.S
        blocks = []
        for _ in range(st.k + st.m):
            blocks.append(addr)
            addr += (st.w * pitch + 255) // 256 * 256 + 4352
        items.append((plans[key], list(st.erased), blocks, st.S, pitch))
    return items


def test_signature_classes():
    """The signature separates what changes the best executor: the rings,
    k and output ranges, slice-size class, decode share, stripe count and
    slice alignment; it ignores the block addresses."""
    c3 = W.c3()[:256]
    a = autotune.signature(items_for(c3))
    assert a == autotune.signature(items_for(c3))
    assert a != autotune.signature(items_for(c3, align=256))            # alignment
    assert a != autotune.signature(items_for(c3[:16]))                  # stripe count
    assert a != autotune.signature(items_for([s for s in c3 if s.w == 8]))  # rings
    enc = [W.Stripe(*W.RING_W8, k=10, m=4, B=1 << 20, stripe=i) for i in range(8)]
    dec = [W.Stripe(*W.RING_W8, k=10, m=4, B=1 << 20, erased=(0, 1), stripe=i) for i in range(8)]
    assert autotune.signature(items_for(enc)) != autotune.signature(items_for(dec))
    assert autotune.signature([]) == "empty"
    assert "|a4096" in autotune.signature(items_for(enc))
    assert "|a64" in autotune.signature(items_for([W.Stripe(*W.RING_W8, k=4, m=2, B=8 * 4160)]))


def test_every_candidate_is_a_valid_executor():
    items = items_for(W.c3()[:64])
    for cand in autotune.CANDIDATES:
        args = dict(cand)
        if args["mode"] != "grid":
            args["grid"] = 1024  # the resident grid is a device query otherwise
        d = P.batch_describe(items, **args)
        assert d["work_items"] > 0 and d["moved_bytes"] > 0, cand


def test_cache_file_round_trip(tmp_path, monkeypatch):
    path = tmp_path / "tune.json"
    monkeypatch.setenv("PYRIT_AUTOTUNE_CACHE", str(path))
    assert autotune._load_file() == {}
    autotune._save_file({"sig": {"mode": "grid", "wg_threads": 256, "split_k": 2}})
    assert json.loads(path.read_text()) == {"sig": {"mode": "grid", "wg_threads": 256, "split_k": 2}}
    path.write_text("not json")
    assert autotune._load_file() == {}


def test_bench_refuses_more_than_one_gpu():
    """bench.py measures one GPU: --gpus N > 1 exits with a message, before
    touching any device."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "single GPU" in r.stderr and r.stdout == ""


def test_bench_records_the_host_cpu():
    import bench
    h = bench.host_cpu()
    assert h["logical_cpus_usable"] >= 1
    assert h["model"] is None or isinstance(h["model"], str)
