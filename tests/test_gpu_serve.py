"""Served form: continuous batching of requests through the native request
loop.  Each request's bytes in the mix must equal its bytes coded alone."""
import dataclasses

import numpy as np
import pytest

import oracle
import paper_1709_00178_amd as P
from paper_1709_00178_amd import serve
from paper_1709_00178_amd import workloads as W
from tests.gpu_util import sample_cols, torch_mod

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    torch = torch_mod()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build()
    yield
    torch.cuda.synchronize()


def small_trace(n=240, rate=60000.0, seed=7, large_every=40):
    """Uneven requests (blocks capped at 256 KiB) plus some k=10 m=4 GF(2^8)
    requests of 2 MiB blocks, Poisson arrivals fast enough to batch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t, out = 0.0, []
    for i in range(n):
        t += float(rng.exponential(1.0 / rate))
        if i % large_every == large_every - 1:
            st = W.Stripe(*W.RING_W8, k=10, m=4, B=2 * 1024 * 1024, stripe=i, seed=seed)
            if i % 80 == 79:
                st = dataclasses.replace(st, erased=(1, 5, 12))
            out.append(W.Request(t, st, True))
        else:
            st = W.draw_stripe(rng, i, seed)
            B = min(st.B, 256 * 1024) // 64 * 64
            out.append(W.Request(t, dataclasses.replace(st, B=B), False))
    return out


def _pool_view(server, off, nbytes):
    torch = torch_mod()
    # a host copy of pool bytes [off, off + nbytes)
    buf = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    import ctypes
    lib = P._lib.lib()
    rc = lib.pyrit_copy(ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(server.pool_base + off),
                        nbytes // 16 * 16, None)
    assert rc == 0
    torch.cuda.synchronize()
    return buf.cpu().numpy()


def _alone(plan, st, inputs, offs):
    """Outputs of one request coded by itself (plain kernel, fresh buffers)."""
    torch = torch_mod()
    blocks = [None] * (st.k + st.m)
    er = set(st.erased)
    ins = [b for b in range(st.k + st.m) if b not in er][:st.k] if st.erased else list(range(st.k))
    for b, o in zip(ins, offs):
        blocks[b] = inputs.buf[o:o + st.block_len]
    outs = list(st.erased) if st.erased else list(range(st.k, st.k + st.m))
    for b in outs:
        blocks[b] = torch.empty(st.block_len, dtype=torch.uint8, device="cuda")
    if st.erased:
        plan.decode(list(st.erased), blocks, st.S, pitch=st.pitch)
    else:
        plan.encode(blocks[:st.k], blocks[st.k:], st.S, pitch=st.pitch)
    torch.cuda.synchronize()
    return [blocks[b].cpu().numpy() for b in outs], ins


def test_served_mix_equals_alone_and_oracle():
    torch = torch_mod()
    trace = small_trace()
    inputs = serve.InputPool(256 << 20, key=0xC0FFEE)
    plans = {}
    prep = serve.prepare(trace, inputs, plans)
    sv = serve.Server(pool_bytes=4 << 30, slots=3, release_outputs=False)
    res, stats = sv.run(prep.array)
    summ = serve.summarize(prep, res, stats)
    # continuous batching: fewer launches than requests, and some launches
    # enqueued while an earlier launch was still running
    assert stats["launches"] < len(trace) and summ["mean_batch"] > 1.0, summ
    launch_done = {}
    for r in res:
        launch_done[r["launch"]] = max(launch_done.get(r["launch"], 0.0), r["done_s"])
    overlapped = sum(1 for r in res if any(l < r["launch"] and d > r["launch_s"]
                                           for l, d in launch_done.items()))
    assert overlapped > 0
    assert (res["admit_s"] <= res["launch_s"]).all() and (res["launch_s"] <= res["done_s"]).all()
    f_cache = {}
    for i, (st, offs, large) in enumerate(prep.meta):
        plan = plans[(st.w, st.n, st.p, st.k, st.m)]
        alone, ins = _alone(plan, st, inputs, offs)
        for q, blk in enumerate(alone):
            mixed = _pool_view(sv, int(res[i]["out_offset"] + q * res[i]["out_stride"]), st.block_len)
            assert np.array_equal(mixed[:st.block_len], blk), (i, q, st)
        if i % 10 == 0:  # oracle on sampled columns
            cols = sample_cols(st.S, 8, i)
            f = f_cache.setdefault((st.w, st.p), oracle.Field(st.w, st.p))
            G = plan.decode_matrix(list(st.erased))[1] if st.erased else plan.G
            mini = []
            for o in offs:
                idx = (o + np.arange(st.w)[:, None] * st.S + cols[None, :]).reshape(-1)
                mini.append(inputs.buf[torch.as_tensor(idx, device="cuda")].cpu().numpy())
            want = f.encode(G, mini, len(cols))
            for q, blk in enumerate(alone):
                got = np.stack([blk[t * st.S + cols] for t in range(st.w)]).reshape(-1)
                assert np.array_equal(got, want[q]), (i, q)
    sv.close()
    del torch


def test_burst_takes_both_launch_forms():
    """Bursts of requests on one launch slot: a launch of few requests runs
    plain kernels back to back, a launch of many one batch kernel.  Every
    request's outputs equal its outputs coded alone."""
    # three requests at once, then 40 more at once 20 ms later: the first
    # launch carries three requests, the later ones twelve
    trace = small_trace(n=43, rate=1e9, seed=29, large_every=1000)
    trace = trace[:3] + [dataclasses.replace(r, arrival_s=r.arrival_s + 0.02) for r in trace[3:]]
    inputs = serve.InputPool(256 << 20, key=0xB0B)
    plans = {}
    prep = serve.prepare(trace, inputs, plans)
    sv = serve.Server(pool_bytes=4 << 30, slots=1, max_batch=12, release_outputs=False)
    res, stats = sv.run(prep.array)
    sizes = np.bincount(res["launch"])
    assert sizes.max() > 4 and sizes.min() <= 4, sizes  # both launch forms ran
    for i, (st, offs, large) in enumerate(prep.meta):
        plan = plans[(st.w, st.n, st.p, st.k, st.m)]
        alone, _ = _alone(plan, st, inputs, offs)
        for q, blk in enumerate(alone):
            mixed = _pool_view(sv, int(res[i]["out_offset"] + q * res[i]["out_stride"]), st.block_len)
            assert np.array_equal(mixed[:st.block_len], blk), (i, q, st)
    sv.close()


def test_served_mix_with_256_byte_aligned_slices():
    """Requests whose slices start at 256-byte boundaries (slice pitch = S
    rounded up to 256, as the benchmark serves them): every coded slice equals
    the same request coded alone at that pitch."""
    trace = small_trace(n=120, seed=13)
    inputs = serve.InputPool(256 << 20, key=0xA11CE)
    plans = {}
    prep = serve.prepare(trace, inputs, plans, pitch_align=256)
    assert all(st.pitch % 256 == 0 and st.S <= st.pitch < st.S + 256 for st, _, _ in prep.meta)
    assert sum(st.pitch != st.S for st, _, _ in prep.meta) > len(trace) // 2
    sv = serve.Server(pool_bytes=2 << 30, slots=3, release_outputs=False)
    res, stats = sv.run(prep.array)
    assert stats["launches"] < len(trace)
    for i, (st, offs, large) in enumerate(prep.meta):
        plan = plans[(st.w, st.n, st.p, st.k, st.m)]
        alone, _ = _alone(plan, st, inputs, offs)
        for q, blk in enumerate(alone):
            mixed = _pool_view(sv, int(res[i]["out_offset"] + q * res[i]["out_stride"]), st.block_len)
            for t in range(st.w):
                sl = slice(t * st.pitch, t * st.pitch + st.S)
                assert np.array_equal(mixed[sl], blk[sl]), (i, q, t, st)
    sv.close()


def test_served_mix_with_parity_transform_plans():
    """Requests over GF(2^4) and GF(2^10) served with parity-transform plans
    (the paper's other transform, a different code) next to embedding plans
    over GF(2^8): every request's bytes equal the same plan coding it alone."""
    trace = small_trace(n=90, seed=17)
    inputs = serve.InputPool(128 << 20, key=0xD00D)
    plans = {}
    for rq in trace:
        st = rq.stripe
        key = (st.w, st.n, st.p, st.k, st.m)
        if key not in plans and st.w in (4, 10):
            plans[key] = P.Plan(*key, transform="parity")
    assert plans
    prep = serve.prepare(trace, inputs, plans)
    sv = serve.Server(pool_bytes=1 << 30, slots=2, release_outputs=False)
    res, stats = sv.run(prep.array)
    n_parity = 0
    for i, (st, offs, large) in enumerate(prep.meta):
        plan = plans[(st.w, st.n, st.p, st.k, st.m)]
        n_parity += plan.transform == "parity"
        alone, _ = _alone(plan, st, inputs, offs)
        for q, blk in enumerate(alone):
            mixed = _pool_view(sv, int(res[i]["out_offset"] + q * res[i]["out_stride"]), st.block_len)
            assert np.array_equal(mixed[:st.block_len], blk), (i, q, st)
    assert n_parity > len(trace) // 3
    sv.close()


def test_per_request_mode_same_bytes():
    trace = small_trace(n=60, seed=11)
    inputs = serve.InputPool(64 << 20, key=0xBEEF)
    plans = {}
    prep = serve.prepare(trace, inputs, plans)
    a = serve.Server(pool_bytes=1 << 30, slots=2, release_outputs=False)
    b = serve.Server(pool_bytes=1 << 30, slots=2, release_outputs=False, per_request=True)
    ra, sa = a.run(prep.array)
    rb, sb = b.run(prep.array)
    assert sb["launches"] == len(trace) and sb["max_batch_seen"] == 1
    for i, (st, offs, large) in enumerate(prep.meta):
        n_out = len(st.erased) if st.erased else st.m
        for q in range(n_out):
            x = _pool_view(a, int(ra[i]["out_offset"] + q * ra[i]["out_stride"]), st.block_len)
            y = _pool_view(b, int(rb[i]["out_offset"] + q * rb[i]["out_stride"]), st.block_len)
            assert np.array_equal(x, y), (i, q)


def test_admission_respects_the_pool_cap():
    """A pool holding only a few requests' outputs: requests wait for space,
    every request still completes, occupancy never exceeds the cap."""
    trace = small_trace(n=120, rate=200000.0, seed=13, large_every=10)
    inputs = serve.InputPool(64 << 20, key=0xABC)
    plans = {}
    prep = serve.prepare(trace, inputs, plans)
    biggest = max(st.block_len * (len(st.erased) if st.erased else st.m) for st, _, _ in prep.meta)
    cap = int(2.5 * (biggest + 4 * 4352)) // 256 * 256
    sv = serve.Server(pool_bytes=cap, slots=2, release_outputs=True)
    res, stats = sv.run(prep.array)
    assert stats["admission_waits"] > 0
    assert 0 < stats["peak_pool_bytes"] <= cap
    assert (res["done_s"] > 0).all()


def test_pool_too_small_is_an_error():
    """Outputs kept and a pool smaller than their sum: the loop reports that
    the head request can never be admitted instead of waiting forever."""
    trace = small_trace(n=30, seed=17, large_every=10)
    inputs = serve.InputPool(32 << 20, key=1)
    plans = {}
    prep = serve.prepare(trace, inputs, plans)
    total = sum((len(st.erased) if st.erased else st.m) * (st.block_len + 4352)
                for st, _, _ in prep.meta)
    cap = 20 << 20
    assert total > cap
    sv = serve.Server(pool_bytes=cap, slots=1, release_outputs=False)
    with pytest.raises(P.PyritError) as e:
        sv.run(prep.array)
    assert e.value.code == -12


class _DeviceBytes:
    """A device address range seen by torch (CUDA array interface, no copy)."""

    def __init__(self, ptr, nbytes):
        self.__cuda_array_interface__ = {"shape": (nbytes,), "typestr": "|u1",
                                         "data": (ptr, False), "version": 3}


def _check_window(sv, pool, trace, inputs, plans, f_cache, oracle_every):
    """Serve one window of the trace; every request's outputs against the
    plain kernel on the same inputs (compared on the device), sampled
    columns of every `oracle_every`-th request against the oracle."""
    torch = torch_mod()
    prep = serve.prepare(trace, inputs, plans)
    res, stats = sv.run(prep.array)
    assert (res["done_s"] > 0).all() and stats["launches"] <= len(trace)
    for i, (st, offs, large) in enumerate(prep.meta):
        plan = plans[(st.w, st.n, st.p, st.k, st.m)]
        blocks = [None] * (st.k + st.m)
        er = set(st.erased)
        ins = [b for b in range(st.k + st.m) if b not in er][:st.k] if st.erased else list(range(st.k))
        for b, o in zip(ins, offs):
            blocks[b] = inputs.buf[o:o + st.block_len]
        outs = list(st.erased) if st.erased else list(range(st.k, st.k + st.m))
        for b in outs:
            blocks[b] = torch.empty(st.block_len, dtype=torch.uint8, device="cuda")
        if st.erased:
            plan.decode(list(st.erased), blocks, st.S)
        else:
            plan.encode(blocks[:st.k], blocks[st.k:], st.S)
        for q, b in enumerate(outs):
            at = int(res[i]["out_offset"] + q * res[i]["out_stride"])
            assert torch.equal(pool[at:at + st.block_len], blocks[b]), (i, q)
        if i % oracle_every == 0:
            cols = sample_cols(st.S, 6, i)
            f = f_cache.setdefault((st.w, st.p), oracle.Field(st.w, st.p))
            G = plan.decode_matrix(list(st.erased))[1] if st.erased else plan.G
            rows = (np.arange(st.w)[:, None] * st.S + cols[None, :]).reshape(-1)
            mini = [inputs.buf[torch.as_tensor(o + rows, device="cuda")].cpu().numpy() for o in offs]
            want = f.encode(G, mini, len(cols))
            idx = torch.as_tensor(rows, device="cuda")
            for q, b in enumerate(outs):
                assert np.array_equal(blocks[b][idx].cpu().numpy(), want[q]), (i, q)
        del blocks
    return len(trace)


def test_c4_full_trace_in_windows():
    """The served mix at its full configuration (Poisson 20k req/s over 2 s,
    5% C1-shaped 64 MiB-block requests, 4 slots, 64 GiB pool), every request
    of the trace: the trace is served in twenty consecutive windows of 0.1 s
    (each window's outputs are kept for checking; a whole 2 s of kept outputs
    would exceed the pool).  Every request's outputs equal the plain
    kernel's on the same inputs, compared on the device; sampled columns of
    every 20th request equal the oracle's."""
    torch = torch_mod()
    full = W.c4()
    assert any(r.large for r in full) and len(full) > 38000
    inputs = serve.InputPool(16 << 30, key=W.BASE_SEED + 4)
    plans, f_cache = {}, {}
    sv = serve.Server(pool_bytes=64 << 30, slots=4, release_outputs=False, block_skew=4352)
    pool = torch.as_tensor(_DeviceBytes(sv.pool_base, sv.pool_bytes), device="cuda")
    checked = 0
    for wdx in range(20):
        t0 = 0.1 * wdx
        win = [dataclasses.replace(r, arrival_s=r.arrival_s - t0) for r in full
               if t0 <= r.arrival_s < t0 + 0.1]
        checked += _check_window(sv, pool, win, inputs, plans, f_cache, oracle_every=20)
        torch.cuda.synchronize()
    assert checked == len(full)
    del pool
    sv.close()
    del inputs
    torch.cuda.empty_cache()
