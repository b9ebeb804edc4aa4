"""Host side of the batch builder (no GPU needed): pyrit_batch_describe
computes, on the host, the passes, work items, bytes moved, grid and per-XCD
byte ranges that pyrit_batch_create would set up.  Block addresses here are
plain integers: nothing is dereferenced."""
import math

import pytest

import paper_1709_00178_amd as P
from paper_1709_00178_amd import workloads as W

EINVAL, EALIGN = -1, -8
BASE = 1 << 36  # a 256-byte aligned fake device address


def fake_items(stripes, plans, align=0):
    """Batch items with distinct, aligned, non-overlapping fake block addresses."""
    items, addr = [], BASE
    for st in stripes:
        key = (st.w, st.n, st.p, st.k, st.m)
        if key not in plans:
            plans[key] = P.Plan(*key)
        pitch = -(-st.S // align) * align if align else st.S
        blocks = []
        for _ in range(st.k + st.m):
            blocks.append(addr)
            addr += (st.w * pitch + 4351) // 256 * 256 + 4352
        items.append((plans[key], list(st.erased), blocks, st.S, pitch))
    return items


def moved(stripes):
    return sum((st.k + (len(st.erased) if st.erased else st.m)) * st.w * st.S for st in stripes)


@pytest.fixture(scope="module")
def c3():
    stripes = W.c3()
    return stripes, fake_items(stripes, {})


def test_uneven_batch_totals(c3):
    """Every stripe of the uneven batch fits one pass (at most four outputs);
    bytes moved are (k + outputs) * w * S summed; one work item per column
    chunk of at least 256 bytes."""
    stripes, items = c3
    d = P.batch_describe(items, mode="grid", wg_threads=128, split_k=2)
    assert d["passes"] == len(stripes)
    assert d["moved_bytes"] == moved(stripes)
    upper = sum(math.ceil(st.S / 256) for st in stripes)
    lower = sum(math.ceil(st.S / 512) for st in stripes)
    assert lower <= d["work_items"] <= upper
    assert d["grid"] == d["work_items"]
    assert d["xcd_bytes"] == [0] * 8


def test_xcd_ranges_carry_equal_bytes(c3):
    """With the XCD-contiguous order the queue is cut into eight ranges of
    equal bytes moved: they add up to the total and differ by at most two
    items' bytes (an item moves at most (16 + 4) * 10 slices * 512 bytes).
    The grid holds eight times the longest range, which has more items than
    the mean where its items are cheap; the surplus workgroups exit at once."""
    stripes, items = c3
    d = P.batch_describe(items, mode="grid", wg_threads=128, split_k=2, xcd_order=1)
    xb = d["xcd_bytes"]
    assert sum(xb) == d["moved_bytes"] == moved(stripes)
    assert max(xb) - min(xb) <= 2 * 20 * 10 * 512
    assert d["grid"] % 8 == 0 and d["work_items"] <= d["grid"] <= 1.5 * d["work_items"]


def test_xcd_ranges_of_a_skewed_order():
    """Stripes sorted by cost put all the expensive items at the end of the
    queue; equal item counts per XCD would leave the last XCD with far more
    bytes, equal-byte ranges do not."""
    stripes = sorted(W.c3()[:1024], key=lambda s: (s.k + (len(s.erased) or s.m)) * s.w)
    d = P.batch_describe(fake_items(stripes, {}), xcd_order=1)
    xb = d["xcd_bytes"]
    assert max(xb) <= 1.01 * sum(xb) / 8 + 2 * 20 * 10 * 512


def test_single_stripe_ranges_are_exact():
    """One C1-shaped stripe: 32768 equal items, an eighth of the bytes each."""
    st = W.c1()
    d = P.batch_describe(fake_items([st], {}), xcd_order=1)
    assert d["passes"] == 1 and d["work_items"] == st.S // 256 and d["grid"] == d["work_items"]
    assert d["xcd_bytes"] == [st.moved_bytes() // 8] * 8


def test_wide_codes_split_into_passes():
    """Parity blocks beyond four per pass open more passes, each re-reading
    the data blocks: GF(2^8) k=10 m=9 is three passes (4 + 4 + 1 outputs)."""
    st = W.Stripe(*W.RING_W8, k=10, m=9, B=8 * 4096)
    d = P.batch_describe(fake_items([st], {}))
    assert d["passes"] == 3
    assert d["moved_bytes"] == (3 * 10 + 9) * st.w * st.S


def test_two_split_k_pairs_per_workgroup(c3):
    """256-thread split-K workgroups hold two pairs on adjacent chunks: half
    as many items as 128-thread ones (one pair), and the same bytes."""
    stripes, items = c3
    one = P.batch_describe(items, wg_threads=128, split_k=2)
    two = P.batch_describe(items, wg_threads=256, split_k=2)
    assert two["moved_bytes"] == one["moved_bytes"]
    assert two["work_items"] == sum(math.ceil(st.S / (2 * 256 * (2 if st.w == 4 else 1)))
                                    for st in stripes)
    assert one["work_items"] == sum(math.ceil(st.S / (256 * (2 if st.w == 4 else 1)))
                                    for st in stripes)


def test_persistent_modes_need_a_grid(c3):
    stripes, items = c3
    for mode in ("queue", "static"):
        with pytest.raises(P.PyritError) as e:
            P.batch_describe(items[:50], mode=mode)
        assert e.value.code == EINVAL
        d = P.batch_describe(items[:50], mode=mode, grid=512, wg_threads=256)
        assert d["grid"] == 512 and d["moved_bytes"] == moved(stripes[:50])


def test_describe_errors():
    st = W.Stripe(*W.RING_W8, k=4, m=2, B=8 * 1024)
    plans = {}
    (plan, er, blocks, S, pitch), = fake_items([st], plans)
    with pytest.raises(P.PyritError) as e:
        P.batch_describe([(plan, er, [blocks[0] + 8] + blocks[1:], S, pitch)])
    assert e.value.code == EALIGN
    with pytest.raises(P.PyritError) as e:
        P.batch_describe([(plan, er, blocks, S, S - 64)])
    assert e.value.code == EINVAL
    with pytest.raises(P.PyritError) as e:
        P.batch_describe([(plan, er, blocks, S, pitch)], split_k=2, wg_threads=64)
    assert e.value.code == EINVAL
    with pytest.raises(P.PyritError) as e:
        P.batch_describe([(plan, [0, 1, 2], blocks, S, pitch)])
    assert e.value.code == -6
    assert P.batch_describe([])["work_items"] == 0


def test_largest_slice_window():
    """(w - 1) * pitch + S must stay below 2^31: the largest accepted block
    ends 64 bytes short of it, one more 64 bytes of pitch is refused."""
    S = (1 << 28) - 64
    st = W.Stripe(*W.RING_W8, k=2, m=1, B=8 * S)
    plan = P.Plan(*W.RING_W8, 2, 1)
    blocks = [BASE + i * (1 << 32) for i in range(3)]
    d = P.batch_describe([(plan, [], blocks, S, S + 64)])
    assert d["moved_bytes"] == 3 * 8 * S and 7 * (S + 64) + S == (1 << 31) - 64
    with pytest.raises(P.PyritError) as e:
        P.batch_describe([(plan, [], blocks, S, S + 128)])
    assert e.value.code == EINVAL
    assert st.S == S


def test_grid_of_more_than_2_32_threads_is_refused():
    """Grid mode launches one workgroup per work item and the dispatch counts
    threads in 32 bits: 32 stripes of 2^28-byte slice windows at 512 column
    bytes per 256-thread workgroup make 2^24 workgroups, 2^32 threads, one
    too many; 31 stripes fit."""
    S = (1 << 28) - 64
    plan = P.Plan(*W.RING_W8, 2, 1)
    items = [(plan, [], [BASE + (3 * s + i) * (1 << 32) for i in range(3)], S, S)
             for s in range(32)]
    with pytest.raises(P.PyritError) as e:
        P.batch_describe(items, wg_threads=256, split_k=2)
    assert e.value.code == EINVAL
    d = P.batch_describe(items[:31], wg_threads=256, split_k=2)
    assert d["grid"] == d["work_items"] == 31 << 19
