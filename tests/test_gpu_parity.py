"""GPU outputs against the CPU oracle, bit-exact, through the C ABI."""
import itertools

import numpy as np
import pytest

import oracle
import paper_1709_00178_amd as P
from paper_1709_00178_amd import workloads as W
from tests.gpu_util import (dev_block, dev_empty, gather_cols, gen_cols, oracle_cols, sample_cols,
                            to_host, torch_mod)

pytestmark = pytest.mark.gpu

RINGS = [(4, 5, 0x1F), (8, 17, 0x139), (8, 17, 0x1D7), (10, 11, 0x7FF), (6, 9, 0x49)]


@pytest.fixture(scope="module", autouse=True)
def _setup():
    torch = torch_mod()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    oracle.build()
    yield
    torch.cuda.synchronize()


def sync():
    torch_mod().cuda.synchronize()


def test_fill_random_matches_generator():
    for nbytes, nrandom, key in [(1 << 20, 1 << 20, 1), (4096, 1000, 12345), (64, 3, 2**64 - 5)]:
        t = dev_empty(nbytes)
        P.fill_random(t, key, nrandom=nrandom)
        got = to_host(t)
        assert np.array_equal(got, W.block_bytes(key, nbytes, nrandom))


def test_fill_random_blocks_matches_generator():
    """Many buffers in one launch (sizes from 8 bytes to several tiles of
    32 KiB, random prefixes of every length class, an empty buffer), each
    against the host generator; bytes around each buffer stay untouched."""
    rng = np.random.Generator(np.random.PCG64(11))
    sizes = [8, 64, 4096, 32768, 32768 + 8, 3 * 32768 + 1000, 1 << 20, 0, 200000]
    sizes = [s // 8 * 8 for s in sizes]
    nrand = [s if i % 3 == 0 else int(rng.integers(0, s + 1)) for i, s in enumerate(sizes)]
    keys = [int(rng.integers(0, 2**63)) * 2 + 1 for _ in sizes]
    guard = 256
    arena = dev_empty(sum(s + 2 * guard for s in sizes))
    arena.fill_(0xC3)
    bufs, off = [], 0
    for s in sizes:
        bufs.append(arena[off + guard:off + guard + s])
        off += s + 2 * guard
    P.fill_random_blocks(bufs, keys, nrand)
    host = to_host(arena)
    off = 0
    for s, nr, key in zip(sizes, nrand, keys):
        assert np.all(host[off:off + guard] == 0xC3)
        assert np.array_equal(host[off + guard:off + guard + s], W.block_bytes(key, s, nr)), (s, nr)
        assert np.all(host[off + guard + s:off + s + 2 * guard] == 0xC3)
        off += s + 2 * guard
    with pytest.raises(P.PyritError):
        P.fill_random_blocks([arena[1:9]], [1])  # not 8-byte aligned


@pytest.mark.parametrize("nbytes", [16, 1008, 1024, 1 << 20, (1 << 20) + 48])
def test_copy_kernel(nbytes):
    """The copy kernel (16-byte loads, two 8-byte stores per lane) at sizes
    that end mid-wave and mid-workgroup; the bytes after the copy stay."""
    src = dev_empty(nbytes)
    P.fill_random(src, 7 + nbytes)
    dst = dev_empty(nbytes + 256)
    dst.fill_(0x5A)
    P.copy(dst, src, nbytes=nbytes)
    got = to_host(dst)
    assert np.array_equal(got[:nbytes], to_host(src))
    assert np.all(got[nbytes:] == 0x5A)


def _full_check(st, G, vec_bytes=0, seed_ids=None):
    """Encode a whole stripe on the GPU and compare every byte with the oracle."""
    k, m = G.shape[1], G.shape[0]
    plan = P.Plan(st.w, st.n, st.p, k, m, G=G)
    data = [dev_block(st, j) for j in range(k)]
    par = [dev_empty(st.block_len) for _ in range(m)]
    for t in par:
        t.fill_(0xA5)
    plan.encode(data, par, st.S, vec_bytes=vec_bytes)
    sync()
    host = [W.block_bytes(st.key(j), st.block_len, st.B) for j in range(k)]
    want = oracle.Field(st.w, st.p).encode(G, host, st.S, nthreads=4)
    for i in range(m):
        got = to_host(par[i])
        assert np.array_equal(got, want[i]), f"parity {i} differs at {np.flatnonzero(got != want[i])[:8]}"


@pytest.mark.parametrize("vec", [0, 4, 8, 16])
def test_c0_encode_bit_exact(vec):
    st = W.c0()
    _full_check(st, P.cauchy(st.w, st.p, st.k, st.m), vec_bytes=vec)


def test_c0_decode_every_two_erasure_pattern():
    st = W.c0()
    torch = torch_mod()
    f = oracle.Field(st.w, st.p)
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    data = W.host_blocks(st)
    code = data + f.encode(plan.G, data, st.S, nthreads=4)
    dev = [torch.from_numpy(b).cuda() for b in code]
    pats = W.c0_erasure_patterns() + [(e,) for e in range(6)]
    for er in pats:
        blocks = [b.clone() for b in dev]
        for e in er:
            blocks[e].fill_(0x5A)
        plan.decode(list(er), blocks, st.S)
        sync()
        for i in range(6):
            assert np.array_equal(to_host(blocks[i]), code[i]), (er, i)


# S spans several 256-lane workgroups and ends in a ragged tail for every
# lane width (4, 8 and 16 bytes per lane).
RAGGED_S = 64 * (4 * 256 + 3)


@pytest.mark.parametrize("w,n,p", RINGS)
@pytest.mark.parametrize("vec", [4, 8, 16])
def test_random_matrix_ragged_sizes(w, n, p, vec):
    k, m = 5, 4
    rng = np.random.Generator(np.random.PCG64(w * 100 + vec))
    G = rng.integers(0, 1 << w, size=(m, k)).astype(np.uint16)
    st = W.Stripe(w, n, p, k=k, m=m, B=RAGGED_S * w - 40, stripe=w + vec, seed=99)
    assert st.S == RAGGED_S
    _full_check(st, G, vec_bytes=vec)


@pytest.mark.parametrize("w,n,p,k,m", [(8, 17, 0x139, 8, 6), (10, 11, 0x7FF, 12, 9),
                                       (4, 5, 0x1F, 3, 1), (6, 9, 0x49, 40, 20)])
def test_many_outputs_and_shapes(w, n, p, k, m):
    st = W.Stripe(w, n, p, k=k, m=m, B=64 * 300 * w, stripe=k, seed=5)
    _full_check(st, P.cauchy(w, p, k, m))


@pytest.mark.parametrize("w,n,p,k,m", [(8, 17, 0x139, 10, 4), (10, 11, 0x7FF, 16, 4),
                                       (6, 9, 0x49, 12, 4), (4, 5, 0x1F, 4, 2)])
def test_light_cauchy_encode_and_decode(w, n, p, k, m):
    """The generalized Cauchy matrix of small lifted weight: encode every byte
    against the oracle with the same matrix, then decode a pattern with data
    and parity erased."""
    G = P.cauchy_light(w, n, p, k, m)[0]
    st = W.Stripe(w, n, p, k=k, m=m, B=RAGGED_S * w, stripe=k + m, seed=11)
    _full_check(st, G)
    torch = torch_mod()
    f = oracle.Field(w, p)
    host = [W.block_bytes(st.key(j), st.block_len, st.B) for j in range(k)]
    code = host + f.encode(G, host, st.S, nthreads=4)
    dev = [torch.from_numpy(b).cuda() for b in code]
    er = [0, k - 1, k + m - 1][:m]
    for e in er:
        dev[e].fill_(0x33)
    P.Plan(w, n, p, k, m, G=G).decode(er, dev, st.S)
    sync()
    for e in er:
        assert np.array_equal(to_host(dev[e]), code[e]), e


@pytest.mark.parametrize("w,n,p", [(8, 17, 0x139), (10, 11, 0x7FF), (4, 5, 0x1F)])
def test_minimum_slice_and_single_input(w, n, p):
    st = W.Stripe(w, n, p, k=1, m=3, B=64 * w, seed=6)
    assert st.S == 64
    _full_check(st, np.array([[1], [2], [(1 << w) - 1]], dtype=np.uint16))


def test_xor_parity_closed_form():
    """An all-ones row: parity = XOR of the data blocks (RAID-5)."""
    st = W.Stripe(8, 17, 0x139, k=7, m=1, B=8 * 4096, seed=8)
    plan = P.Plan(st.w, st.n, st.p, 7, 1, G=np.ones((1, 7), dtype=np.uint16))
    data = [dev_block(st, j) for j in range(7)]
    par = [dev_empty(st.block_len)]
    plan.encode(data, par, st.S)
    sync()
    want = np.bitwise_xor.reduce(np.stack([W.block_bytes(st.key(j), st.block_len) for j in range(7)]))
    assert np.array_equal(to_host(par[0]), want)


@pytest.mark.parametrize("s", [1, 5, 7])
def test_multiply_by_x_power_closed_form(s):
    """G = [x^s]: shift slices up by s, folding each overflow through p."""
    w, n, p, S = 8, 17, 0x139, 4096
    st = W.Stripe(w, n, p, k=1, m=1, B=w * S, seed=9 + s)
    plan = P.Plan(w, n, p, 1, 1, G=np.array([[1 << s]], dtype=np.uint16))
    d = dev_block(st, 0)
    out = dev_empty(st.block_len)
    plan.encode([d], [out], S)
    sync()
    host = W.block_bytes(st.key(0), st.block_len)
    sl = [host[t * S:(t + 1) * S].copy() for t in range(w)]
    for _ in range(s):
        top = sl[w - 1]
        sl = [np.zeros(S, dtype=np.uint8)] + sl[:w - 1]
        for t in range(w):
            if (p >> t) & 1:
                sl[t] = sl[t] ^ top
    assert np.array_equal(to_host(out), np.concatenate(sl))


def test_c1_full_size_encode_sampled():
    """GF(2^8) k=10 m=4, 64 MiB blocks: every launch shape the benchmark uses,
    checked on sampled columns of every slice of every parity block."""
    st = W.c1()
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    data = [dev_block(st, j) for j in range(st.k)]
    cols = sample_cols(st.S, 2048, 1)
    want = oracle_cols(st, plan.G, range(st.k), cols)
    for vec in [0, 8]:
        par = [dev_empty(st.block_len) for _ in range(st.m)]
        plan.encode(data, par, st.S, vec_bytes=vec)
        sync()
        for i in range(st.m):
            got = gather_cols(to_host(par[i]), st.S, st.w, cols)
            assert np.array_equal(got, want[i]), (vec, i)


def test_c1_decode_roundtrip_full_size():
    """Encode, erase the workload's patterns, decode: recovered data blocks
    equal the generator's bytes everywhere; recovered parity equals the oracle
    on sampled columns."""
    st = W.c1()
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    code = [dev_block(st, j) for j in range(st.k)] + [dev_empty(st.block_len) for _ in range(st.m)]
    plan.encode(code[:st.k], code[st.k:], st.S)
    cols = sample_cols(st.S, 1024, 2)
    want_par = oracle_cols(st, plan.G, range(st.k), cols)
    for er in W.c1_erasure_patterns():
        blocks = [b.clone() for b in code]
        for e in er:
            blocks[e].fill_(0xC3)
        plan.decode(list(er), blocks, st.S)
        sync()
        for e in er:
            got = to_host(blocks[e])
            if e < st.k:
                assert np.array_equal(got, W.block_bytes(st.key(e), st.block_len, st.B)), (er, e)
            else:
                assert np.array_equal(gather_cols(got, st.S, st.w, cols), want_par[e - st.k]), (er, e)


def test_c2_all_stripes_sampled():
    """GF(2^10) k=16 m=4, 256 stripes of 4 MiB blocks, plain kernel per stripe."""
    stripes = W.c2()
    st0 = stripes[0]
    plan = P.Plan(st0.w, st0.n, st0.p, st0.k, st0.m)
    torch = torch_mod()
    cols = sample_cols(st0.S, 24, 3)
    data = torch.empty((len(stripes), st0.k, st0.block_len), dtype=torch.uint8, device="cuda")
    par = torch.empty((len(stripes), st0.m, st0.block_len), dtype=torch.uint8, device="cuda")
    for s, st in enumerate(stripes):
        for j in range(st.k):
            P.fill_random(data[s, j], st.key(j), nrandom=st.B)
        plan.encode([data[s, j] for j in range(st.k)], [par[s, i] for i in range(st.m)], st.S)
    sync()
    idx = torch.as_tensor((np.arange(st0.w)[:, None] * st0.S + cols[None, :]).reshape(-1),
                          device="cuda")
    got_all = par[:, :, idx].cpu().numpy()
    for s, st in enumerate(stripes):
        want = oracle_cols(st, plan.G, range(st.k), cols, nthreads=2)
        for i in range(st.m):
            assert np.array_equal(got_all[s, i], want[i]), (s, i)


def test_c3_stripes_plain_sampled():
    """The uneven batch distribution through the plain path, first 192 stripes."""
    torch = torch_mod()
    plans = {}
    for st in W.c3()[:192]:
        key = (st.w, st.k, st.m)
        if key not in plans:
            plans[key] = P.Plan(st.w, st.n, st.p, st.k, st.m)
        plan = plans[key]
        ins = W.survivors(st)
        blocks = [None] * (st.k + st.m)
        for b in ins:
            blocks[b] = dev_block(st, b)
        outs = list(st.erased) if st.erased else list(range(st.k, st.k + st.m))
        for b in outs:
            blocks[b] = dev_empty(st.block_len)
        if st.erased:
            # survivors not read by the decoder may be absent; give them a buffer anyway
            for b in range(st.k + st.m):
                if blocks[b] is None:
                    blocks[b] = dev_empty(64)
            plan.decode(list(st.erased), blocks, st.S)
            _, D = plan.decode_matrix(list(st.erased))
            G = D
        else:
            plan.encode(blocks[:st.k], blocks[st.k:], st.S)
            G = plan.G
        sync()
        cols = sample_cols(st.S, 16, st.stripe)
        want = oracle_cols(st, G, ins, cols, nthreads=1)
        for r, b in enumerate(outs):
            got = gather_cols(to_host(blocks[b]), st.S, st.w, cols)
            assert np.array_equal(got, want[r]), (st, b)
    del torch


def test_parity_only_and_empty_erasures():
    st = W.Stripe(10, 11, 0x7FF, k=6, m=4, B=10 * 64 * 64, seed=11)
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    torch = torch_mod()
    f = oracle.Field(st.w, st.p)
    data = W.host_blocks(st)
    code = data + f.encode(plan.G, data, st.S)
    dev = [torch.from_numpy(b).cuda() for b in code]
    for er in [(6, 9), (7,), (6, 7, 8, 9), ()]:
        blocks = [b.clone() for b in dev]
        for e in er:
            blocks[e].zero_()
        plan.decode(list(er), blocks, st.S)
        sync()
        for i in range(st.k + st.m):
            assert np.array_equal(to_host(blocks[i]), code[i]), (er, i)


def test_error_paths():
    st = W.Stripe(8, 17, 0x139, k=2, m=2, B=8 * 256, seed=12)
    plan = P.Plan(st.w, st.n, st.p, 2, 2)
    a = dev_empty(st.block_len + 64)
    bufs = [dev_empty(st.block_len) for _ in range(3)]
    with pytest.raises(P.PyritError) as e:
        plan.encode([a.data_ptr() + 1, bufs[0]], bufs[1:], st.S)
    assert e.value.code == -8
    with pytest.raises(P.PyritError) as e:
        plan.encode([a, bufs[0]], bufs[1:], 100)
    assert e.value.code == -8
    with pytest.raises(P.PyritError) as e:
        plan.decode([0, 1, 2], [a] + bufs, st.S)
    assert e.value.code == -6
    with pytest.raises(P.PyritError) as e:
        plan.encode([a, bufs[0]], bufs[1:], st.S, vec_bytes=12)
    assert e.value.code == -1
    sync()


@pytest.mark.parametrize("w,n,p,pad", [(8, 17, 0x139, 4096), (10, 11, 0x7FF, 320), (4, 5, 0x1F, 64)])
def test_slice_pitch_plain_and_batched(w, n, p, pad):
    """Blocks whose slices sit `pad` bytes apart: the padding is never read or
    written, and the coded bytes equal the oracle on the packed slices."""
    torch = torch_mod()
    k, m = 6, 3
    st = W.Stripe(w, n, p, k=k, m=m, B=w * 64 * 300, seed=31, pad=pad)
    plan = P.Plan(w, n, p, k, m)
    data = [dev_block(st, j) for j in range(k)]
    host = W.host_blocks(st)
    want = oracle.Field(w, p).encode(plan.G, host, st.S, nthreads=4)
    for path in ["plain", "grid", "queue"]:
        par = [dev_empty(st.block_len) for _ in range(m)]
        for t in par:
            t.fill_(0xB7)
        if path == "plain":
            plan.encode(data, par, st.S, pitch=st.pitch)
        else:
            P.Batch([(plan, [], data + par, st.S, st.pitch)], mode=path).launch()
        sync()
        for i in range(m):
            mem = to_host(par[i])
            assert np.array_equal(W.logical(st, mem), want[i]), (path, i)
            for t in range(w):
                gap = mem[t * st.pitch + st.S:(t + 1) * st.pitch]
                assert (gap == 0xB7).all(), (path, i, t)
    # decode through the pitch-aware path
    code = data + [dev_empty(st.block_len) for _ in range(m)]
    plan.encode(data, code[k:], st.S, pitch=st.pitch)
    er = [0, 4, 7]
    saved = [code[e].clone() for e in er]
    for e in er:
        code[e].fill_(0)
    plan.decode(er, code, st.S, pitch=st.pitch)
    sync()
    for e, s_ in zip(er, saved):
        a, b = W.logical(st, to_host(code[e])), W.logical(st, to_host(s_))
        assert np.array_equal(a, b), e
    # the library's own refusals (raw addresses skip the binding's size check)
    din, dout = [t.data_ptr() for t in data], [t.data_ptr() for t in code[k:]]
    with pytest.raises(P.PyritError):
        plan.encode(din, dout, st.S, pitch=st.S - 64)
    with pytest.raises(P.PyritError):
        plan.encode(din, dout, st.S, pitch=st.S + 32)
    del torch


def test_largest_code_the_abi_accepts():
    """k = m = 64 (PYRIT_KMAX, PYRIT_MMAX) over GF(2^8), ragged slices: the
    plain encode (16 passes of four outputs, each re-reading the 64 data
    blocks) against the oracle, the same code in one batch launch, and a
    decode of all 64 data blocks from the 64 parity blocks."""
    torch = torch_mod()
    w, n, p, k, m = 8, 17, 0x139, 64, 64
    st = W.Stripe(w, n, p, k=k, m=m, B=w * 64 * 41, seed=71)
    assert st.S == 64 * 41
    plan = P.Plan(w, n, p, k, m)
    data = [dev_block(st, j) for j in range(k)]
    par = [dev_empty(st.block_len) for _ in range(m)]
    plan.encode(data, par, st.S)
    sync()
    want = oracle.Field(w, p).encode(plan.G, W.host_blocks(st), st.S, nthreads=4)
    for i in range(m):
        assert np.array_equal(to_host(par[i]), want[i]), i
    par2 = [dev_empty(st.block_len) for _ in range(m)]
    b = P.Batch([(plan, [], data + par2, st.S)], mode="grid", wg_threads=256, split_k=2)
    assert b.info()["passes"] == 16
    b.launch_direct()
    sync()
    for i in range(m):
        assert torch.equal(par2[i], par[i]), i
    saved = [d.clone() for d in data]
    for d in data:
        d.fill_(0)
    plan.decode(list(range(k)), data + par, st.S)
    sync()
    for j in range(k):
        assert torch.equal(data[j], saved[j]), j
    with pytest.raises(P.PyritError) as e:
        P.Plan(w, n, p, k + 1, 1)
    assert e.value.code == -1


def test_largest_block_the_abi_accepts():
    """A block whose slices reach the end of the 31-bit slice window: S just
    under 256 MiB at a pitch of S + 64, so (w - 1) * pitch + S = 2^31 - 64.
    Plain and batched encodes and a decode, checked on sampled columns (the
    last byte of the last slice included); one more 64 bytes of pitch is
    refused before anything runs."""
    torch = torch_mod()
    w, n, p, k, m = 8, 17, 0x139, 2, 1
    S = (1 << 28) - 64
    st = W.Stripe(w, n, p, k=k, m=m, B=w * S, seed=41, pad=64)
    assert st.S == S and (w - 1) * st.pitch + S == (1 << 31) - 64
    plan = P.Plan(w, n, p, k, m)
    data = [dev_block(st, j) for j in range(k)]
    cols = sample_cols(S, 512, 6)
    want = oracle_cols(st, plan.G, range(k), cols)
    idx = torch.from_numpy((np.arange(w)[:, None] * st.pitch + cols[None, :]).reshape(-1)).cuda()

    def at_cols(t):
        return t[idx].cpu().numpy()

    par = dev_empty(st.block_len)
    for path in ["plain", "grid"]:
        par.fill_(0x5A)
        if path == "plain":
            plan.encode(data, [par], S, pitch=st.pitch)
        else:
            P.Batch([(plan, [], data + [par], S, st.pitch)], mode="grid", wg_threads=128,
                    split_k=2).launch_direct()
        sync()
        assert np.array_equal(at_cols(par), want[0]), path
    lost = data[0].clone()
    data[0].fill_(0)
    plan.decode([0], [data[0], data[1], par], S, pitch=st.pitch)
    sync()
    assert np.array_equal(at_cols(data[0]), gen_cols(st, 0, cols))
    for t in range(w):
        sl = slice(t * st.pitch, t * st.pitch + S)
        assert torch.equal(data[0][sl], lost[sl]), t
    # refused by the library (raw addresses skip the binding's size check)
    with pytest.raises(P.PyritError) as e:
        plan.encode([t.data_ptr() for t in data], [par.data_ptr()], S, pitch=st.pitch + 64)
    assert e.value.code == -1
    del torch


# Symbol-major <-> bit-sliced conversions on the device against the oracle's.
# 512 * 257 symbols: 4112 lanes, not a multiple of the 256-lane workgroup.
N_SYM = 512 * 257


@pytest.mark.parametrize("w", [1, 4, 6, 8, 10, 16])
@pytest.mark.parametrize("extra_pitch", [0, 192])
def test_to_and_from_sliced(w, extra_pitch):
    torch = torch_mod()
    rng = np.random.Generator(np.random.PCG64(w * 10 + extra_pitch))
    dt = np.uint8 if w <= 8 else np.uint16
    sym = rng.integers(0, 1 << (8 if w <= 8 else 16), N_SYM).astype(dt)  # high bits set too
    S = N_SYM // 8
    pitch = S + extra_pitch
    dsym = torch.from_numpy(sym.view(np.uint8).copy()).cuda()
    dsl = dev_empty(w * pitch)
    dsl.fill_(0x77)
    P.to_sliced(w, dsym, dsl, n_symbols=N_SYM, pitch=pitch if extra_pitch else 0)
    back = dev_empty(sym.nbytes)
    back.fill_(0xEE)
    P.from_sliced(w, dsl, back, n_symbols=N_SYM, pitch=pitch if extra_pitch else 0)
    sync()
    want = oracle.to_sliced(w, sym.astype(np.uint32) & ((1 << w) - 1)).reshape(w, S)
    got = to_host(dsl).reshape(w, pitch)[:, :S]
    assert np.array_equal(got, want)
    masked = (sym.astype(np.uint32) & ((1 << w) - 1)).astype(dt)
    assert np.array_equal(to_host(back).view(dt), masked)


def test_symbols_to_parity_symbols_end_to_end():
    """GF(2^8) k=10 m=4: symbols -> slices -> encode -> parity symbols equals
    the symbol-by-symbol product with the oracle's multiply."""
    torch = torch_mod()
    w, n, p, k, m = 8, 17, 0x139, 10, 4
    nsym = 512 * 64
    S = nsym // 8
    rng = np.random.Generator(np.random.PCG64(77))
    data = [rng.integers(0, 256, nsym).astype(np.uint8) for _ in range(k)]
    plan = P.Plan(w, n, p, k, m)
    sliced = [dev_empty(w * S) for _ in range(k + m)]
    for j in range(k):
        P.to_sliced(w, torch.from_numpy(data[j]).cuda(), sliced[j])
    plan.encode(sliced[:k], sliced[k:], S)
    out = [dev_empty(nsym) for _ in range(m)]
    for i in range(m):
        P.from_sliced(w, sliced[k + i], out[i])
    sync()
    f = oracle.Field(w, p)
    for i in range(m):
        want = np.zeros(nsym, dtype=np.uint32)
        for j in range(k):
            want ^= f.mul_many(np.full(nsym, plan.G[i, j], dtype=np.uint32), data[j])
        assert np.array_equal(to_host(out[i]), want.astype(np.uint8)), i


def test_sliced_conversion_errors():
    a, b = dev_empty(8192), dev_empty(8192)
    for bad in [dict(w=0), dict(w=17), dict(n_symbols=500), dict(n_symbols=0)]:
        args = dict(w=8, n_symbols=512)
        args.update(bad)
        with pytest.raises(P.PyritError) as e:
            P.to_sliced(args["w"], a, b, n_symbols=args["n_symbols"])
        assert e.value.code == -1, bad
    with pytest.raises(P.PyritError) as e:
        P.to_sliced(8, a.data_ptr() + 4, b, n_symbols=512)
    assert e.value.code == -8
    with pytest.raises(P.PyritError) as e:
        P.from_sliced(8, a, b, n_symbols=512, pitch=96)
    assert e.value.code in (-1, -8)


# Parity transform (Sec. II-C.1, II-D.1): a different code, checked against
# the oracle's definition of it.
PT_RINGS = [(4, 5, 0x1F), (10, 11, 0x7FF), (6, 9, 0x49)]


@pytest.mark.parametrize("w,n,p", PT_RINGS)
@pytest.mark.parametrize("vec", [0, 4, 8, 16])
def test_parity_transform_encode(w, n, p, vec):
    k, m = (4, 3) if w == 4 else (7, 4)
    st = W.Stripe(w, n, p, k=k, m=m, B=RAGGED_S * w - 8, stripe=n + vec, seed=31)
    plan = P.Plan(w, n, p, k, m, transform="parity")
    data = [dev_block(st, j) for j in range(k)]
    par = [dev_empty(st.block_len) for _ in range(m)]
    plan.encode(data, par, st.S, vec_bytes=vec)
    sync()
    host = [W.block_bytes(st.key(j), st.block_len, st.B) for j in range(k)]
    want = oracle.encode_parity_transform(oracle.Field(w, p), n, plan.G, host, st.S)
    for i in range(m):
        assert np.array_equal(to_host(par[i]), want[i]), i


@pytest.mark.parametrize("w,n,p", PT_RINGS)
def test_parity_transform_decode(w, n, p):
    torch = torch_mod()
    k, m = (4, 2) if w == 4 else (8, 4)
    st = W.Stripe(w, n, p, k=k, m=m, B=64 * 96 * w, stripe=7, seed=32)
    plan = P.Plan(w, n, p, k, m, transform="parity")
    f = oracle.Field(w, p)
    host = [W.block_bytes(st.key(j), st.block_len, st.B) for j in range(k)]
    code = host + oracle.encode_parity_transform(f, n, plan.G, host, st.S)
    pats = list(itertools.combinations(range(k + m), m))[::max(1, len(list(itertools.combinations(range(k + m), m))) // 25)]
    for er in pats:
        dev = [torch.from_numpy(b.copy()).cuda() for b in code]
        for e in er:
            dev[e].fill_(0xC3)
        plan.decode(list(er), dev, st.S)
        sync()
        for e in er:
            assert np.array_equal(to_host(dev[e]), code[e]), (er, e)


# Passes of up to ring_max_out outputs: 8 for n <= 9, 6 for n = 11, 4 for
# n = 17; m above the limit splits into several passes (or wide launches),
# for the encode and for a decode of m erasures (the paper's (60,40) shape
# among them).
@pytest.mark.parametrize("w,n,p,k,m,transform", [
    (4, 5, 0x1F, 8, 8, "embedding"), (4, 5, 0x1F, 7, 9, "parity"),
    (6, 9, 0x49, 10, 8, "embedding"), (6, 9, 0x49, 11, 17, "parity"),
    (10, 11, 0x7FF, 10, 6, "embedding"), (10, 11, 0x7FF, 9, 7, "parity"),
    (8, 17, 0x1D7, 6, 5, "embedding"), (6, 9, 0x49, 40, 20, "embedding")])
def test_wide_passes_encode_and_decode(w, n, p, k, m, transform):
    torch = torch_mod()
    st = W.Stripe(w, n, p, k=k, m=m, B=64 * 200 * w, stripe=m, seed=41)
    plan = P.Plan(w, n, p, k, m, transform=transform)
    f = oracle.Field(w, p)
    host = [W.block_bytes(st.key(j), st.block_len, st.B) for j in range(k)]
    if transform == "parity":
        code = host + oracle.encode_parity_transform(f, n, plan.G, host, st.S)
    else:
        code = host + f.encode(plan.G, host, st.S, nthreads=4)
    dev = [torch.from_numpy(c.copy()).cuda() for c in code]
    for i in range(m):
        dev[k + i].fill_(0x11)
    plan.encode(dev[:k], dev[k:], st.S)
    sync()
    for i in range(m):
        assert np.array_equal(to_host(dev[k + i]), code[k + i]), i
    er = list(range(0, k + m, max(1, (k + m) // m)))[:m]
    for e in er:
        dev[e].fill_(0x22)
    plan.decode(er, dev, st.S)
    sync()
    for e in er:
        assert np.array_equal(to_host(dev[e]), code[e]), (er, e)


# Wide launches: outputs beyond one pass are coded by G waves sharing one
# column chunk (G output groups per launch, as many as the kernel arguments
# hold).  Each case against the oracle, whole blocks, ragged S over several
# workgroups, and against the one-pass-per-group path (vec_bytes = 4).
# Cases: three uneven groups in one launch on every ring and transform (odd k
# on the rings coding two blocks per barrier, so the last step holds one);
# the paper's (60,40) and (60,20) shapes; codes whose outputs need several
# wide launches (k = 64).
@pytest.mark.parametrize("w,n,p,k,m,transform", [
    (4, 5, 0x1F, 5, 11, "embedding"), (4, 5, 0x1F, 3, 13, "parity"),
    (8, 17, 0x139, 9, 11, "embedding"), (8, 17, 0x1D7, 7, 9, "embedding"),
    (10, 11, 0x7FF, 12, 13, "embedding"), (10, 11, 0x7FF, 11, 17, "parity"),
    (6, 9, 0x49, 40, 20, "embedding"), (6, 9, 0x49, 20, 40, "parity"),
    (6, 9, 0x49, 20, 40, "embedding"), (6, 9, 0x49, 7, 12, "embedding"),
    (6, 9, 0x49, 9, 11, "parity"), (10, 11, 0x7FF, 64, 40, "embedding"),
    (8, 17, 0x139, 64, 14, "embedding")])
def test_wide_launches_match_oracle_and_passes(w, n, p, k, m, transform):
    torch = torch_mod()
    st = W.Stripe(w, n, p, k=k, m=m, B=RAGGED_S * w - 24, stripe=k * 100 + m, seed=43)
    assert st.S == RAGGED_S
    plan = P.Plan(w, n, p, k, m, transform=transform)
    f = oracle.Field(w, p)
    host = [W.block_bytes(st.key(j), st.block_len, st.B) for j in range(k)]
    if transform == "parity":
        want = oracle.encode_parity_transform(f, n, plan.G, host, st.S)
    else:
        want = f.encode(plan.G, host, st.S, nthreads=8)
    data = [torch.from_numpy(h).cuda() for h in host]
    wide = [dev_empty(st.block_len) for _ in range(m)]
    passes = [dev_empty(st.block_len) for _ in range(m)]
    for a, b in zip(wide, passes):
        a.fill_(0x3C)
        b.fill_(0xC3)
    plan.encode(data, wide, st.S)
    plan.encode(data, passes, st.S, vec_bytes=4)
    sync()
    for i in range(m):
        got = to_host(wide[i])
        assert np.array_equal(got, want[i]), (i, np.flatnonzero(got != want[i])[:8])
        assert torch.equal(wide[i], passes[i]), i


def test_one_plan_on_concurrent_streams():
    """One plan coding on four streams at once: each stream encodes its own
    copy of the data and decodes its own erasure pattern (the decode cache
    fills from several host calls in flight)."""
    torch = torch_mod()
    st = W.Stripe(8, 17, 0x139, k=10, m=4, B=64 * 512 * 8, seed=61)
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    f = oracle.Field(st.w, st.p)
    host = [W.block_bytes(st.key(j), st.block_len, st.B) for j in range(st.k)]
    code = host + f.encode(plan.G, host, st.S, nthreads=4)
    pats = [[0, 3, 11], [1, 2, 12, 13], [4], [5, 6, 7, 8]]
    sets = []
    for er in pats:
        data = [torch.from_numpy(h.copy()).cuda() for h in host]
        par = [dev_empty(st.block_len) for _ in range(st.m)]
        word = [torch.from_numpy(c.copy()).cuda() for c in code]
        sets.append((torch.cuda.Stream(), er, data, par, word))
    torch.cuda.synchronize()
    for rep in range(3):
        for s, er, data, par, word in sets:
            with torch.cuda.stream(s):
                for e in er:
                    word[e].fill_(rep + 1)
                for t in par:
                    t.fill_(rep + 1)
            plan.encode(data, par, st.S, stream=s)
            plan.decode(er, word, st.S, stream=s)
        torch.cuda.synchronize()
        for s, er, data, par, word in sets:
            for i in range(st.m):
                assert np.array_equal(to_host(par[i]), code[st.k + i]), (rep, er, i)
            for e in er:
                assert np.array_equal(to_host(word[e]), code[e]), (rep, er, e)
