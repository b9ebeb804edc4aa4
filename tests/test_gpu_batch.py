"""Persistent batched kernel (one launch, hipGraph replay) against the CPU
oracle, bit-exact, through the C ABI."""
import numpy as np
import pytest

import oracle
import paper_1709_00178_amd as P
from paper_1709_00178_amd import workloads as W
from tests.gpu_util import (Arena, fill_inputs, gather_cols, oracle_cols, sample_cols, stripe_buffers,
                            stripe_bytes_needed, to_host, torch_mod)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _setup():
    torch = torch_mod()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build()
    yield
    torch.cuda.synchronize()


def sync():
    torch_mod().cuda.synchronize()


class PlanCache:
    def __init__(self):
        self.plans = {}

    def get(self, st):
        key = (st.w, st.n, st.p, st.k, st.m)
        if key not in self.plans:
            self.plans[key] = P.Plan(*key)
        return self.plans[key]


def _check_stripes(stripes, bufs, plans, ncols=16, seed=0):
    """Sampled columns of every output of every stripe against the oracle
    (columns gathered on the device, copied back, compared on the host)."""
    torch = torch_mod()
    for si, st in enumerate(stripes):
        blocks, ins, outs = bufs[si]
        plan = plans.get(st)
        G = plan.decode_matrix(list(st.erased))[1] if st.erased else plan.G
        cols = sample_cols(st.S, ncols, seed + st.stripe)
        want = oracle_cols(st, G, ins, cols, nthreads=1)
        idx = torch.as_tensor((np.arange(st.w)[:, None] * st.pitch + cols[None, :]).reshape(-1),
                              device="cuda")
        got_all = torch.stack([blocks[b][idx] for b in outs]).cpu().numpy()
        for r, b in enumerate(outs):
            assert np.array_equal(got_all[r], want[r]), (si, st, b)


def _build(stripes, plans, arena):
    bufs = [stripe_buffers(st, arena, fill=False) for st in stripes]
    fill_inputs(stripes, bufs)
    items = [(plans.get(st), list(st.erased), bufs[i][0], st.S, st.pitch)
             for i, st in enumerate(stripes)]
    return bufs, items


def _clear_outputs(bufs, value):
    for blocks, ins, outs in bufs:
        for b in outs:
            blocks[b].fill_(value)


def test_batch_single_stripe_every_shape():
    """C0 stripe in every launch shape: graph and direct launch, dynamic and
    static queues, 64/128/256-thread workgroups, several tile widths."""
    st = W.c0()
    plans = PlanCache()
    arena = Arena(stripe_bytes_needed(st) + 4096)
    bufs, items = _build([st], plans, arena)
    host = W.host_blocks(st)
    want = oracle.Field(st.w, st.p).encode(plans.get(st).G, host, st.S, nthreads=4)
    shapes = [("grid", 0, 0, 1), ("grid", 0, 1, 1), ("grid", 0, 0, 2), ("grid", 0, 1, 2),
              ("queue", 0, 0, 1), ("queue", 512, 0, 1), ("queue", 4096, 0, 1), ("static", 0, 0, 1),
              ("static", 512, 0, 1), ("static", 4096, 0, 1)]
    for wg in [64, 128, 256]:
        for mode, tile, xcd, split in shapes:
            if split == 2 and wg == 64:
                continue
            b = P.Batch(items, mode=mode, tile_bytes=tile, wg_threads=wg, xcd_order=xcd,
                        split_k=split)
            for launch in [b.launch, b.launch_direct, b.launch, b.run]:
                _clear_outputs(bufs, 0xEE)
                launch()
                sync()
                for i in range(st.m):
                    got = to_host(bufs[0][0][st.k + i])
                    assert np.array_equal(got, want[i]), (wg, mode, tile, xcd, split, i)
            b.close()


@pytest.mark.parametrize("mode", ["grid", "queue", "static"])
def test_batch_graph_replays_with_eager_work_between(mode):
    """Each replay recomputes every output; eager fills between replays (the
    queue mode's claim counters carry over from launch to launch)."""
    stripes = W.c2(8)
    plans = PlanCache()
    arena = Arena(sum(stripe_bytes_needed(s) for s in stripes) + 4096)
    bufs, items = _build(stripes, plans, arena)
    b = P.Batch(items, mode=mode, tile_bytes=4096 if mode != "grid" else 0)
    for rep in range(5):
        _clear_outputs(bufs, rep * 17)
        b.launch()
        sync()
        _check_stripes(stripes, bufs, plans, ncols=8, seed=rep)


@pytest.mark.parametrize("mode,xcd,split,wg", [("grid", 0, 1, 0), ("grid", 1, 1, 0), ("grid", 1, 2, 0),
                                               ("grid", 1, 2, 256), ("grid", 0, 2, 256),
                                               ("queue", 0, 1, 0), ("static", 0, 1, 0)])
def test_c2_all_stripes_one_launch(mode, xcd, split, wg):
    """All 256 stripes in one launch, including the executors the autotuner
    picks for them (256-thread workgroups of two split-K pairs)."""
    stripes = W.c2()
    plans = PlanCache()
    arena = Arena(sum(stripe_bytes_needed(s) for s in stripes) + 4096)
    bufs, items = _build(stripes, plans, arena)
    b = P.Batch(items, mode=mode, xcd_order=xcd, split_k=split, wg_threads=wg)
    info = b.info()
    assert info["passes"] == 256
    assert info["moved_bytes"] == sum(s.moved_bytes() for s in stripes)
    b.launch()
    sync()
    _check_stripes(stripes, bufs, plans, ncols=12)


@pytest.mark.parametrize("mode,xcd,split,wg", [("grid", 0, 1, 0), ("grid", 1, 1, 0), ("grid", 0, 2, 0),
                                               ("grid", 1, 2, 0), ("grid", 1, 2, 256),
                                               ("grid", 1, 1, 64), ("queue", 0, 1, 0),
                                               ("static", 0, 1, 0)])
def test_c3_all_4096_uneven_stripes_one_launch(mode, xcd, split, wg):
    """The uneven batch: w in {4,8,10}, k in [4,16], m in [2,4], 4 KiB..4 MiB
    blocks, 30% decodes, all in one launch (also with the 256- and 64-thread
    executors the autotuner has picked for it)."""
    stripes = W.c3()
    plans = PlanCache()
    arena = Arena(sum(stripe_bytes_needed(s) for s in stripes) + 4096)
    bufs, items = _build(stripes, plans, arena)
    b = P.Batch(items, mode=mode, xcd_order=xcd, split_k=split, wg_threads=wg)
    info = b.info()
    assert info["moved_bytes"] == sum(s.moved_bytes() for s in stripes)
    if mode == "grid":  # the host-only description sets up the same launch
        d = P.batch_describe(items, mode=mode, xcd_order=xcd, split_k=split, wg_threads=wg)
        assert [d[f] for f in ("passes", "work_items", "moved_bytes", "grid")] == \
               [info[f] for f in ("passes", "work_items", "moved_bytes", "grid")]
    _clear_outputs(bufs, 0x77)
    b.launch()
    sync()
    _check_stripes(stripes, bufs, plans, ncols=10)


@pytest.mark.parametrize("wg", [256, 128])
def test_c1_full_size_as_benched(wg):
    """The headline stripe in the benchmark's own layout and launch: 64 MiB
    blocks, slices 8 MiB + 4 KiB apart, blocks 4352 B apart, the grid
    executor with split-K workgroups of two pairs (the benched form) or one
    pair, direct dispatch.  Sampled
    columns of every parity slice against the oracle; the gaps between
    slices untouched; then the workload's 4-erasure decode the same way."""
    import dataclasses
    torch = torch_mod()
    st = dataclasses.replace(W.c1(), pad=4096)
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    skew = 4352
    stride = (st.block_len + 255) // 256 * 256 + skew
    pool = torch.empty(stride * (st.k + st.m + 4) + 4096, dtype=torch.uint8, device="cuda")
    blocks = [pool[i * stride:i * stride + st.block_len] for i in range(st.k + st.m)]
    for j in range(st.k):
        P.fill_random(blocks[j], st.key(j), nrandom=st.nrandom)
    for b in blocks[st.k:]:
        b.fill_(0xA5)
    b = P.Batch([(plan, [], blocks, st.S, st.pitch)], mode="grid", wg_threads=wg, xcd_order=0,
                split_k=2, launch="direct")
    b.run()
    sync()
    cols = sample_cols(st.S, 2048, 3)
    want = oracle_cols(st, plan.G, range(st.k), cols)
    idx = torch.as_tensor((np.arange(st.w)[:, None] * st.pitch + cols[None, :]).reshape(-1),
                          device="cuda")
    for i in range(st.m):
        assert np.array_equal(blocks[st.k + i][idx].cpu().numpy(), want[i]), i
        for t in range(st.w):
            gap = blocks[st.k + i][t * st.pitch + st.S:(t + 1) * st.pitch]
            assert bool((gap == 0xA5).all()), (i, t)
    # decode: the erased blocks come back bit-exact
    er = list(W.c1_erasure_patterns()[0])
    spare = [pool[(st.k + st.m + q) * stride:(st.k + st.m + q) * stride + st.block_len]
             for q in range(len(er))]
    dec = [spare[er.index(i)] if i in er else blk for i, blk in enumerate(blocks)]
    d = P.Batch([(plan, er, dec, st.S, st.pitch)], mode="grid", wg_threads=wg, split_k=2,
                launch="direct")
    d.run()
    sync()
    for q, e in enumerate(er):
        for t in range(st.w):
            sl = slice(t * st.pitch, t * st.pitch + st.S)
            assert torch.equal(spare[q][sl], blocks[e][sl]), (e, t)
    b.close()
    d.close()
    del pool


@pytest.mark.parametrize("xcd,wg", [(0, 128), (1, 128), (0, 256), (1, 256)])
def test_c3_with_256_byte_aligned_slices(xcd, wg):
    """The uneven batch as the benchmark codes it: every slice pitch rounded
    up to 256 bytes (blocks random over their whole memory, so B = w * S),
    the split-K grid executor in both item orders."""
    import dataclasses
    stripes = [dataclasses.replace(st, B=st.w * st.S, pad=-(-st.S // 256) * 256 - st.S)
               for st in W.c3()]
    assert sum(st.pad > 0 for st in stripes) > len(stripes) // 2
    plans = PlanCache()
    arena = Arena(sum(stripe_bytes_needed(s) for s in stripes) + 4096)
    bufs, items = _build(stripes, plans, arena)
    b = P.Batch(items, mode="grid", wg_threads=wg, split_k=2, xcd_order=xcd, launch="direct")
    _clear_outputs(bufs, 0x3C)
    b.run()
    sync()
    _check_stripes(stripes, bufs, plans, ncols=10, seed=5)
    b.close()


def test_c1_code_64_stripes_one_launch():
    """The headline code over 64 stripes of 1 MiB blocks in one launch (the
    bench's many-stripe leg), every stripe against the oracle."""
    base = W.c1()
    stripes = [W.Stripe(base.w, base.n, base.p, k=base.k, m=base.m, B=1 << 20, stripe=i,
                        seed=base.seed) for i in range(64)]
    plans = PlanCache()
    arena = Arena(sum(stripe_bytes_needed(s) for s in stripes) + 4096)
    bufs, items = _build(stripes, plans, arena)
    for cfg in [dict(split_k=2), dict(split_k=2, xcd_order=1), dict(wg_threads=256, split_k=1)]:
        _clear_outputs(bufs, 0x5A)
        b = P.Batch(items, mode="grid", **cfg)
        b.run()
        sync()
        _check_stripes(stripes, bufs, plans, ncols=8)
        b.close()


@pytest.mark.parametrize("split,wg", [(1, 128), (2, 128), (2, 256)])
def test_every_ring_in_one_batch(split, wg):
    """All five rings (both degree-8 factors of x^17+1 and the ESP ring
    x^6+x^3+1 included), encodes and decodes, uneven sizes, one launch."""
    rings = [(4, 5, 0x1F), (8, 17, 0x139), (8, 17, 0x1D7), (10, 11, 0x7FF), (6, 9, 0x49)]
    stripes = []
    for i, (w, n, p) in enumerate(rings * 3):
        k, m = (4 + i % 7, 2 + i % 3) if w != 4 else (4 + i % 5, 2 + i % 3)
        erased = () if i % 3 == 0 else tuple(sorted({(i * 5) % (k + m), (i * 7 + 1) % (k + m)}))[:m]
        B = (37 + 91 * i) * 64 * w
        stripes.append(W.Stripe(w, n, p, k=k, m=m, B=B, erased=erased, stripe=i, seed=99))
    plans = PlanCache()
    arena = Arena(sum(stripe_bytes_needed(s) for s in stripes) + 4096)
    bufs, items = _build(stripes, plans, arena)
    _clear_outputs(bufs, 0x3C)
    b = P.Batch(items, mode="grid", wg_threads=wg, split_k=split)
    b.run()
    sync()
    _check_stripes(stripes, bufs, plans, ncols=16)


def test_batch_matches_plain_kernel_bytes():
    """Batched and plain outputs are identical for C1-shaped stripes with
    6 outputs (two passes) and a decode."""
    torch = torch_mod()
    st = W.Stripe(8, 17, 0x139, k=10, m=6, B=8 * 64 * 1000, seed=21)
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    arena = Arena(3 * (st.k + st.m) * st.block_len + 8192)
    data = [arena.take(st.block_len) for _ in range(st.k)]
    for j, t in enumerate(data):
        P.fill_random(t, st.key(j))
    par_plain = [arena.take(st.block_len) for _ in range(st.m)]
    par_batch = [arena.take(st.block_len) for _ in range(st.m)]
    plan.encode(data, par_plain, st.S)
    for mode, split in [("grid", 1), ("grid", 2), ("queue", 1), ("static", 1)]:
        for t in par_batch:
            t.zero_()
        b = P.Batch([(plan, [], data + par_batch, st.S)], mode=mode, split_k=split)
        b.launch()
        sync()
        for a, c in zip(par_plain, par_batch):
            assert torch.equal(a, c), (mode, split)
    # decode two data blocks and two parity blocks through the batch path
    er = [1, 7, 11, 14]
    blocks = data + par_plain
    outs = {e: arena.take(st.block_len) for e in er}
    bl = [outs.get(i, blocks[i]) for i in range(st.k + st.m)]
    b2 = P.Batch([(plan, er, bl, st.S)])
    b2.launch()
    sync()
    for e in er:
        assert torch.equal(outs[e], blocks[e]), e


def test_batch_errors():
    st = W.c0()
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    arena = Arena(8 * st.block_len + 8192)
    blocks = [arena.take(st.block_len) for _ in range(6)]
    with pytest.raises(P.PyritError) as e:
        P.Batch([(plan, [], [blocks[0].data_ptr() + 4] + blocks[1:], st.S)])
    assert e.value.code == -8
    with pytest.raises(P.PyritError) as e:
        P.Batch([(plan, [0, 1, 2], blocks, st.S)])
    assert e.value.code == -6
    bad = P.Plan(3, 7, 0xB, 3, 2)
    with pytest.raises(P.PyritError) as e:
        P.Batch([(bad, [], blocks[:5], 64)])
    assert e.value.code == -9
    with pytest.raises(P.PyritError) as e:
        P.Batch([(plan, [], blocks, st.S)], wg_threads=96)
    assert e.value.code == -1
    with pytest.raises(P.PyritError) as e:
        P.Batch([(plan, [], blocks, st.S)], xcd_order=2)
    assert e.value.code == -1
    for bad_split in [dict(split_k=3), dict(split_k=2, wg_threads=64),
                      dict(split_k=2, mode="queue", wg_threads=128)]:
        with pytest.raises(P.PyritError) as e:
            P.Batch([(plan, [], blocks, st.S)], **bad_split)
        assert e.value.code == -1, bad_split
    with pytest.raises(ValueError):
        P.Batch([(plan, [], blocks, st.S)], mode="fifo")
    with pytest.raises(ValueError):
        P.Batch([(plan, [], blocks, st.S)], launch="stream")
    empty = P.Batch([])
    empty.launch()
    sync()


@pytest.mark.parametrize("mode,split,wg", [("grid", 1, 128), ("grid", 2, 128), ("grid", 2, 256),
                                           ("queue", 1, 128), ("static", 1, 128)])
def test_parity_and_embedding_stripes_in_one_batch(mode, split, wg):
    """Parity-transform stripes (encodes and decodes) next to embedding ones
    in one launch, each against the oracle's definition of its code."""
    torch = torch_mod()
    specs = [((4, 5, 0x1F), 4, 2), ((10, 11, 0x7FF), 6, 3), ((6, 9, 0x49), 5, 4), ((8, 17, 0x139), 5, 3)]
    plans, items, checks = [], [], []
    keep = []
    for i, ((w, n, p), k, m) in enumerate(specs * 2):
        transform = "parity" if (w != 8 and i % 2 == 0) else "embedding"
        plan = P.Plan(w, n, p, k, m, transform=transform)
        S = 64 * (40 + 17 * i)
        rng = np.random.Generator(np.random.PCG64(100 + i))
        data = [rng.integers(0, 256, w * S, dtype=np.uint8) for _ in range(k)]
        f = oracle.Field(w, p)
        if transform == "parity":
            code = data + oracle.encode_parity_transform(f, n, plan.G, data, S)
        else:
            code = data + f.encode(plan.G, data, S)
        er = [] if i < 4 else [0, k + m - 1]
        dev = [torch.from_numpy(c.copy()).cuda() for c in code]
        outs = er if er else list(range(k, k + m))
        for o in outs:
            dev[o].fill_(0x99)
        keep.append((plan, dev))
        items.append((plan, er, dev, S))
        checks.append((dev, code, outs))
    b = P.Batch(items, mode=mode, split_k=split, wg_threads=wg)
    b.run()
    sync()
    for i, (dev, code, outs) in enumerate(checks):
        for o in outs:
            assert np.array_equal(to_host(dev[o]), code[o]), (i, o)
