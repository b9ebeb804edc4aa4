"""The allocation-free batch run (pyrit_batch_run_noalloc) against the entry
points it stands for (pyrit_batch_create + pyrit_batch_launch_direct), bit
for bit, through the C ABI: two calls in a row, the second with fewer
stripes, in each executor.  The reference batches are themselves checked
against the CPU oracle by the batch tests."""
import numpy as np
import pytest

import paper_1709_00178_amd as P
from paper_1709_00178_amd import workloads as W
from tests.gpu_util import Arena, fill_inputs, stripe_buffers, stripe_bytes_needed, torch_mod

pytestmark = pytest.mark.gpu


def _sync():
    torch_mod().cuda.synchronize()


def _outputs(bufs):
    """Host copy of every output block of every stripe."""
    torch = torch_mod()
    return [torch.cat([blocks[b] for b in outs]).cpu().numpy() for blocks, _, outs in bufs]


def _clear(bufs, value):
    for blocks, _, outs in bufs:
        for b in outs:
            blocks[b].fill_(value)


@pytest.mark.parametrize("mode,wg", [("grid", 128), ("grid", 256), ("queue", 128),
                                     ("static", 256)])
def test_noalloc_matches_batch_two_calls(mode, wg):
    """Uneven stripes of the batched distribution (encodes and decodes, three
    fields): 40 stripes, then 12 others.  Each call's outputs equal those of
    a batch created and launched directly on the same items; the second,
    smaller call finds the first call's image (and, in the queue executor,
    its claim counters) in the shared array."""
    assert torch_mod().cuda.is_available(), "GPU tests need a GPU"
    stripes = W.c3(52)
    groups = [stripes[:40], stripes[40:]]
    plans = {}

    def plan(st):
        key = (st.w, st.n, st.p, st.k, st.m)
        if key not in plans:
            plans[key] = P.Plan(*key)
        return plans[key]

    arena = Arena(sum(stripe_bytes_needed(st) for st in stripes) + 4096)
    runs = []
    for sts in groups:
        bufs = [stripe_buffers(st, arena, fill=False) for st in sts]
        fill_inputs(sts, bufs)
        items = [(plan(st), list(st.erased), b[0], st.S, st.pitch) for st, b in zip(sts, bufs)]
        _clear(bufs, 0x5A)
        ref = P.Batch(items, mode=mode, wg_threads=wg, launch="direct")
        ref.run()
        _sync()
        want = _outputs(bufs)
        ref.close()
        _clear(bufs, 0xA5)
        runs.append((bufs, items, want))
    _sync()
    for _, items, _ in runs:  # two calls in a row, the second smaller
        P.batch_run_noalloc(items, mode=mode, wg_threads=wg)
    _sync()
    for ci, (bufs, items, want) in enumerate(runs):
        got = _outputs(bufs)
        for si, (g, w_) in enumerate(zip(got, want)):
            assert np.array_equal(g, w_), (mode, wg, "call", ci, "stripe", si)


def test_noalloc_refuses_an_image_larger_than_its_array():
    """16384 single-pass items (their pointer and lift tables alone exceed
    the array) are refused with PYRIT_ETOOBIG before anything is copied or
    launched.  The items point at real buffers, so even a launch would stay
    in bounds."""
    torch = torch_mod()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    w, n, p = W.RING_W10
    pl = P.Plan(w, n, p, 16, 4)
    blocks = [torch.zeros(w * 64, dtype=torch.uint8, device="cuda") for _ in range(20)]
    items = [(pl, [], blocks, 64)] * 16384
    with pytest.raises(P.PyritError) as e:
        P.batch_run_noalloc(items)
    assert e.value.code == -14  # PYRIT_ETOOBIG
    _sync()
