"""The seeded synthetic workloads (CPU): shapes, the readings taken where the
workload description is loose (slice rounding, the GF(2^4) length limit,
erasure draws, the served mix), and determinism."""
import collections
import itertools

import numpy as np

from paper_1709_00178_amd import workloads as W


def test_fixed_shapes():
    """C0, C1, C2: the slice size of each block is ceil(B / w) rounded up to
    64 bytes (C2: 4 MiB / 10 slices -> 419 456 bytes)."""
    c0, c1 = W.c0(), W.c1()
    assert (c0.w, c0.k, c0.m, c0.S) == (4, 4, 2, 16 * 1024)
    assert (c1.w, c1.n, c1.p, c1.k, c1.m, c1.S) == (8, 17, 0x139, 10, 4, 8 << 20)
    c2 = W.c2()
    assert len(c2) == 256 and {(s.w, s.k, s.m, s.S) for s in c2} == {(10, 16, 4, 419456)}
    per_slice = -(-(4 << 20) // 10)              # ceil(4 MiB / 10) = 419 431
    assert -(-per_slice // 64) * 64 == 419456
    assert c1.moved_bytes() == 14 * 8 * (8 << 20)


def test_slice_rounding():
    for B, w in [(4096, 4), (4160, 10), (1 << 20, 8), (12345 * 64, 10), (64, 8)]:
        S = W.slice_bytes(B, w)
        assert S % 64 == 0 and S * w >= B and (S - 64) * w < B, (B, w, S)


def test_uneven_batch_distribution():
    stripes = W.c3()
    assert len(stripes) == 4096
    ws = collections.Counter(s.w for s in stripes)
    assert set(ws) == {4, 8, 10} and min(ws.values()) > 1200
    for s in stripes:
        assert 4 <= s.k <= 16 and 2 <= s.m <= 4
        assert 4096 <= s.B <= 4 << 20 and s.B % 64 == 0
        if s.w == 4:
            assert s.k + s.m <= 16   # the GF(2^4) code-length limit: (k, m) redrawn
        if s.erased:
            assert 1 <= len(s.erased) <= s.m
            assert list(s.erased) == sorted(set(s.erased)) and max(s.erased) < s.k + s.m
    dec = sum(1 for s in stripes if s.erased) / len(stripes)
    assert 0.27 < dec < 0.33
    # block sizes log-uniform over [4 KiB, 4 MiB]: about half below 128 KiB
    lo = sum(1 for s in stripes if s.B < 128 * 1024) / len(stripes)
    assert 0.45 < lo < 0.55


def test_workloads_are_deterministic():
    a, b = W.c3(64), W.c3(64)
    assert a == b
    assert W.c1_erasure_patterns() == W.c1_erasure_patterns()
    st = W.c1()
    x = W.block_bytes(st.key(3), 4096, 4096)
    assert np.array_equal(x, W.block_bytes(st.key(3), 4096, 4096))
    assert not np.array_equal(x, W.block_bytes(st.key(4), 4096, 4096))


def test_c1_erasure_patterns():
    pick, lead = W.c1_erasure_patterns()
    assert lead == (0, 1, 2, 3)
    assert len(pick) == 4 and list(pick) == sorted(set(pick)) and max(pick) < 14
    assert pick in set(itertools.combinations(range(14), 4))


def test_packed_block_is_zero_past_B():
    st = W.Stripe(*W.RING_W10, k=4, m=2, B=4160)
    mem = W.block_bytes(st.key(0), st.block_len, st.nrandom)
    assert st.block_len == 10 * st.S > st.B
    assert mem[st.B:].max() == 0 and mem[:st.B].any()


def test_survivors():
    st = W.Stripe(*W.RING_W8, k=4, m=3, B=8 * 64, erased=(0, 5))
    assert W.survivors(st) == (1, 2, 3, 4)
    assert W.survivors(W.Stripe(*W.RING_W8, k=4, m=3, B=8 * 64)) == (0, 1, 2, 3)


def test_served_mix():
    """20 000 requests/s for 2 s: Poisson arrivals, 5% C1-shaped large
    requests (30% of them decodes), the rest drawn like the uneven batch."""
    trace = W.c4()
    assert 39000 < len(trace) < 41000
    t = np.array([r.arrival_s for r in trace])
    assert (np.diff(t) > 0).all() and t[-1] < 2.0
    gaps = np.diff(t)
    assert abs(gaps.mean() - 1 / 20000) < 0.05 / 20000 and abs(gaps.std() / gaps.mean() - 1) < 0.05
    large = [r for r in trace if r.large]
    assert 0.045 < len(large) / len(trace) < 0.055
    assert {(r.stripe.w, r.stripe.k, r.stripe.m, r.stripe.B) for r in large} == {(8, 10, 4, 64 << 20)}
    small = [r.stripe for r in trace if not r.large]
    assert all(4 <= s.k <= 16 and 4096 <= s.B <= 4 << 20 for s in small)
