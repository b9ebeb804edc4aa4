"""Host side of the library through its C ABI (no GPU needed): ring checks,
the sparse transform, reduction, ring products, Cauchy matrices, decoding
matrices.  Pinned to the paper's worked values, brute force and the oracle."""
import ctypes
import itertools
import json
import os
import re

import numpy as np
import pytest

import oracle
import paper_1709_00178_amd as P
from paper_1709_00178_amd import _lib
from paper_1709_00178_amd import workloads as W
from tests import gf_schoolbook as sb

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
GOLD = json.load(open(os.path.join(HERE, "golden", "paper_examples.json")))
RINGS = [(4, 5, 0x1F), (8, 17, 0x139), (8, 17, 0x1D7), (10, 11, 0x7FF), (6, 9, 0x49)]
E = {"EINVAL": -1, "ENOTIRRED": -2, "ENOTDIV": -3, "ETOOLONG": -4, "ERANGE": -5,
     "ETOOMANY": -6, "ESINGULAR": -7, "EALIGN": -8, "EUNSUPPORTED": -9}


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "pyrit.h")).read()
    declared = set(re.findall(r"\b(pyrit_[a-z0-9_]+)\s*\(", hdr))
    assert declared, "no declarations parsed"
    L = _lib.lib()
    missing = [s for s in sorted(declared) if not hasattr(L, s)]
    assert not missing, missing
    assert declared <= set(_lib.SIGNATURES), declared - set(_lib.SIGNATURES)


def test_error_strings():
    for code in list(E.values()) + [0, -10, -11, -12]:
        assert P._lib.lib().pyrit_strerror(code)


def test_paper_r25_product():
    ex = GOLD["r25_product"]
    assert P.ring_mul(ex["n"], ex["a"], ex["b"]) == ex["product"]


def test_paper_r25_factors_and_idempotents():
    f = GOLD["r25_factors"]
    a, b = f["factors"]
    assert sb.poly_mul(a, b) == (1 << f["n"]) | 1      # x^5 + 1 = p1 * p2
    assert P.ring_mul(f["n"], a, b) == 0
    ex = GOLD["r25_idempotents"]
    n, t1, t2 = ex["n"], ex["theta_field_ideal"], ex["theta_other_ideal"]
    assert P.ring_mul(n, t1, t1) == t1 and P.ring_mul(n, t2, t2) == t2
    assert t1 ^ t2 == 1 and P.ring_mul(n, t1, t2) == 0
    # theta_1 acts as 1 on the field: its reduction mod p is 1
    assert P.ring_reduce(4, 5, ex["p"], t1) == 1


def test_paper_r25_sparse_representative():
    ex = GOLD["r25_sparse_example"]
    w, n, p, u = ex["w"], ex["n"], ex["p"], ex["u"]
    theta = GOLD["r25_idempotents"]["theta_field_ideal"]
    img = P.ring_mul(n, u, theta)
    assert img == ex["image"]
    assert img ^ p == ex["image_plus_p"]
    assert P.ring_reduce(w, n, p, img) == u
    cands = [c for c in range(1 << n) if sb.poly_mod(c, p) == u]
    assert len(cands) == ex["n_candidates"] == 2 ** (n - w)
    assert set(cands) == {img, img ^ p}
    assert P.lift(w, n, p, u) == ex["image_plus_p"]


@pytest.mark.parametrize("key", ["aop_embedding_inverse", "esp_embedding_inverse"])
def test_paper_inverse_embedding_closed_forms(key):
    ex = GOLD[key]
    for i, want in ex["x_pow_mod_p"].items():
        assert P.ring_reduce(ex["w"], ex["n"], ex["p"], 1 << int(i)) == want


def test_paper_esp_structure():
    ex = GOLD["esp_structure"]
    assert sb.poly_mul(ex["p"], ex["cofactor"]) == (1 << ex["n"]) | 1
    th = ex["theta"]
    assert P.ring_mul(ex["n"], th, th) == th
    assert P.ring_reduce(ex["w"], ex["n"], ex["p"], th) == 1
    assert P.ring_check(ex["w"], ex["n"], ex["p"]) == 0


def test_paper_aop_irreducibility():
    ex = GOLD["aop_irreducible"]
    for w in ex["irreducible_w"]:
        assert P.ring_check(w, w + 1, (1 << (w + 1)) - 1) == 0
    for w in ex["reducible_w"]:
        n = w + 1 if (w + 1) % 2 else w + 2
        rc = P.ring_check(w, n, (1 << (w + 1)) - 1)
        assert rc in (E["ENOTIRRED"], E["ENOTDIV"]), (w, rc)
        if (w + 1) % 2:
            assert rc == E["ENOTIRRED"], w


def test_ring_check_errors():
    assert P.ring_check(8, 17, 0x139) == 0
    assert P.ring_check(8, 17, 0x11D) == E["ENOTDIV"]    # irreducible, does not divide x^17+1
    assert P.ring_check(8, 16, 0x139) == E["ENOTDIV"]    # n even
    assert P.ring_check(4, 5, 0x11) == E["ENOTIRRED"]
    assert P.ring_check(4, 5, 0x3F) == E["EINVAL"]       # degree 5, not 4
    assert P.ring_check(4, 4, 0x1F) == E["EINVAL"]       # n must exceed w
    assert P.ring_check(4, 25, 0x1F) == E["EINVAL"]      # n above 24


@pytest.mark.parametrize("w,n,p", RINGS)
def test_ring_parameters_valid(w, n, p):
    assert sb.is_irreducible(p)
    assert sb.poly_mod((1 << n) | 1, p) == 0
    assert P.ring_check(w, n, p) == 0
    assert P.ring_supported(w, n, p)


@pytest.mark.parametrize("w,n,p", RINGS)
def test_lift_is_minimum_weight_representative(w, n, p):
    """Brute force over every ring element: group by residue mod p, keep the
    least weight, smallest integer on ties (Sec. II-B)."""
    c = np.arange(1 << n, dtype=np.int64)
    r = c.copy()
    for d in range(n - 1, w - 1, -1):
        r ^= np.where((r >> d) & 1, p << (d - w), 0)
    wt = np.array([bin(x).count("1") for x in range(1 << n)])
    for u in range(1 << w):
        sel = c[r == u]
        assert len(sel) == 2 ** (n - w)
        best = sel[np.lexsort((sel, wt[sel]))[0]]
        assert P.lift(w, n, p, u) == best, u


@pytest.mark.parametrize("w,n,p", RINGS)
def test_reduction_is_ring_homomorphism(w, n, p):
    """(a * b in R_{2,n}) mod p == (a mod p) * (b mod p) in GF(2^w)."""
    rng = np.random.Generator(np.random.PCG64(n))
    if n == 5:
        pairs = list(itertools.product(range(32), repeat=2))
    else:
        pairs = [tuple(int(v) for v in rng.integers(0, 1 << n, 2)) for _ in range(4000)]
    for a, b in pairs:
        lhs = P.ring_reduce(w, n, p, P.ring_mul(n, a, b))
        rhs = int(sb.mul(sb.poly_mod(a, p), sb.poly_mod(b, p), w, p))
        assert lhs == rhs, (a, b)


@pytest.mark.parametrize("w,n,p", RINGS)
def test_gf_mul_matches_schoolbook(w, n, p):
    q = 1 << w
    rng = np.random.Generator(np.random.PCG64(w))
    for a, b in rng.integers(0, q, size=(3000, 2)):
        assert P.gf_mul(w, p, int(a), int(b)) == int(sb.mul(a, b, w, p))


@pytest.mark.parametrize("st", [W.c0(), W.c1(), W.c2(1)[0]], ids=["c0", "c1", "c2"])
def test_cauchy_matches_oracle(st):
    G = P.cauchy(st.w, st.p, st.k, st.m)
    Go = oracle.Field(st.w, st.p).cauchy(st.k, st.m)
    assert np.array_equal(G, Go)


# Total lifted weight W (XOR terms per column) and the largest single weight,
# derived by brute force for the Cauchy matrices of the three workloads.
@pytest.mark.parametrize("st,total,maxw", [(W.c0(), 12, 2), (W.c1(), 92, 3),
                                           (W.c2(1)[0], 244, 5)], ids=["c0", "c1", "c2"])
def test_plan_lift_and_weights(st, total, maxw):
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    L = plan.lifted
    G = plan.G
    for i in range(st.m):
        for j in range(st.k):
            assert sb.poly_mod(int(L[i, j]), st.p) == int(G[i, j])
    wt = np.vectorize(lambda x: bin(int(x)).count("1"))(L)
    assert plan.weight == int(wt.sum()) == total
    assert wt.max() == maxw


def test_plan_create_errors():
    G = np.ones((2, 4), dtype=np.uint16)
    h = ctypes.c_void_p()
    L = _lib.lib()
    assert L.pyrit_plan_create(4, 5, 0x11, 4, 2, G.ctypes.data, ctypes.byref(h)) == E["ENOTIRRED"]
    assert L.pyrit_plan_create(4, 5, 0x1F, 0, 2, G.ctypes.data, ctypes.byref(h)) == E["EINVAL"]
    G16 = np.ones((4, 13), dtype=np.uint16)
    assert L.pyrit_plan_create(4, 5, 0x1F, 13, 4, G16.ctypes.data, ctypes.byref(h)) == E["ETOOLONG"]
    Gbad = np.full((2, 4), 16, dtype=np.uint16)
    assert L.pyrit_plan_create(4, 5, 0x1F, 4, 2, Gbad.ctypes.data, ctypes.byref(h)) == E["ERANGE"]
    # a ring without a device kernel: plan exists, device calls refuse
    plan = P.Plan(3, 7, 0xB, 3, 2)
    assert not P.ring_supported(3, 7, 0xB)
    with pytest.raises(P.PyritError) as e:
        plan.encode([1, 2, 3], [4, 5], 64, stream=0)
    assert e.value.code == E["EUNSUPPORTED"]


def _decode_check(st, patterns):
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    f = oracle.Field(st.w, st.p)
    rng = np.random.Generator(np.random.PCG64(3))
    S = 64
    data = [rng.integers(0, 256, st.w * S, dtype=np.uint8) for _ in range(st.k)]
    code = data + f.encode(plan.G, data, S)
    for er in patterns:
        surv, D = plan.decode_matrix(list(er))
        assert list(surv) == [i for i in range(st.k + st.m) if i not in er][:st.k]
        # recover with the oracle's multiply, by the binary-matrix form
        rec = sb.bitmatrix_encode(D, [code[s] for s in surv], st.w, st.p, S)
        for e, blk in zip(er, rec):
            assert np.array_equal(blk, code[e]), (er, e)


def test_decode_matrix_every_pattern_c0():
    st = W.c0()
    pats = [(e,) for e in range(6)] + W.c0_erasure_patterns() + [(5, 0)]
    _decode_check(st, pats)


def test_decode_matrix_c1_patterns():
    st = W.c1()
    rng = np.random.Generator(np.random.PCG64(4))
    pats = W.c1_erasure_patterns() + [tuple(rng.choice(14, 4, replace=False)) for _ in range(20)]
    _decode_check(st, pats)


def test_decode_matrix_errors():
    plan = P.Plan(4, 5, 0x1F, 4, 2)
    with pytest.raises(P.PyritError) as e:
        plan.decode_matrix([0, 1, 2])
    assert e.value.code == E["ETOOMANY"]
    with pytest.raises(P.PyritError) as e:
        plan.decode_matrix([1, 1])
    assert e.value.code == E["EINVAL"]
    sing = P.Plan(4, 5, 0x1F, 4, 2, G=np.ones((2, 4), dtype=np.uint16))
    with pytest.raises(P.PyritError) as e:
        sing.decode_matrix([0, 1])
    assert e.value.code == E["ESINGULAR"]


# Generalized Cauchy of small ring weight.  Pins: the rank-1 scaling
# structure against the oracle's multiply, nonsingular square submatrices by
# schoolbook elimination, the weight against brute-force popcounts of the
# lifted entries, and recovery from every pattern with the oracle's decoder.
LIGHT = [((4, 5, 0x1F), 4, 2, 12), ((8, 17, 0x139), 10, 4, 72), ((10, 11, 0x7FF), 16, 4, 168),
         ((8, 17, 0x1D7), 10, 4, 76), ((6, 9, 0x49), 12, 4, None)]


@pytest.mark.parametrize("ring,k,m,want", LIGHT, ids=[f"{r[0]}-{r[1]}-{k}-{m}" for r, k, m, _ in LIGHT])
def test_cauchy_light_structure_and_weight(ring, k, m, want):
    w, n, p = ring
    G, rs, cs, W_ = P.cauchy_light(w, n, p, k, m)
    G2, rs2, cs2, W2 = P.cauchy_light(w, n, p, k, m)
    assert np.array_equal(G, G2) and W_ == W2  # deterministic
    f = oracle.Field(w, p)
    C = f.cauchy(k, m)
    assert (rs != 0).all() and (cs != 0).all()
    for i in range(m):
        for j in range(k):
            assert int(G[i, j]) == f.mul(f.mul(int(rs[i]), int(C[i, j])), int(cs[j]))
    lifted = [P.lift(w, n, p, int(g)) for g in G.ravel()]
    assert W_ == sum(bin(c).count("1") for c in lifted)
    assert W_ <= P.Plan(w, n, p, k, m).weight
    if want is not None:
        assert W_ == want
    assert P.Plan(w, n, p, k, m, G=G).weight == W_


@pytest.mark.parametrize("ring,k,m", [((4, 5, 0x1F), 4, 2), ((8, 17, 0x139), 10, 4)])
def test_cauchy_light_is_mds(ring, k, m):
    w, n, p = ring
    G = P.cauchy_light(w, n, p, k, m)[0]
    mats = []
    for s in range(1, m + 1):
        for rows in itertools.combinations(range(m), s):
            for cols in itertools.combinations(range(k), s):
                mats.append(G[np.ix_(rows, cols)])
        ok = sb.det_nonzero_all(mats, w, p)
        assert ok.all(), s
        mats = []


# Generalized Cauchy with chosen points.  Pins: the entries are exactly
# row_scale[i] * col_scale[j] / (X[i] + Y[j]) by the oracle's field (a Cauchy
# matrix scaled by rows and columns, over distinct points), nonsingular
# square submatrices by schoolbook elimination on small codes, the weight
# against popcounts of the lifted entries, and recovery by the oracle.
SEARCH = [((4, 5, 0x1F), 8, 4), ((8, 17, 0x139), 10, 4), ((10, 11, 0x7FF), 16, 4),
          ((6, 9, 0x49), 40, 20), ((6, 9, 0x49), 20, 40), ((8, 17, 0x1D7), 6, 3)]


@pytest.mark.parametrize("ring,k,m", SEARCH, ids=[f"{r[0]}-{k}-{m}" for r, k, m in SEARCH])
def test_cauchy_search_structure_and_weight(ring, k, m):
    w, n, p = ring
    G, X, Y, rs, cs, W_ = P.cauchy_search(w, n, p, k, m)
    G2, X2, Y2, _, _, W2 = P.cauchy_search(w, n, p, k, m)
    assert np.array_equal(G, G2) and np.array_equal(X, X2) and W_ == W2  # deterministic
    pts = [int(v) for v in X] + [int(v) for v in Y]
    assert len(set(pts)) == k + m and max(pts) < (1 << w)
    assert (rs != 0).all() and (cs != 0).all()
    f = oracle.Field(w, p)
    for i in range(m):
        for j in range(k):
            want = f.mul(f.mul(int(rs[i]), int(cs[j])), f.inv(int(X[i]) ^ int(Y[j])))
            assert int(G[i, j]) == want, (i, j)
    lifted = [P.lift(w, n, p, int(g)) for g in G.ravel()]
    assert W_ == sum(bin(c).count("1") for c in lifted)
    assert W_ <= P.cauchy_light(w, n, p, k, m)[3]
    assert P.Plan(w, n, p, k, m, G=G).weight == W_
    # no sweep: the point sets stay {0..m-1} and {m..m+k-1}
    G0, X0, Y0, *_ = P.cauchy_search(w, n, p, k, m, sweeps=0)
    assert list(X0) == list(range(m)) and list(Y0) == list(range(m, m + k))


@pytest.mark.parametrize("ring,k,m", [((4, 5, 0x1F), 8, 4), ((8, 17, 0x139), 10, 4),
                                      ((6, 9, 0x49), 6, 3)])
def test_cauchy_search_is_mds(ring, k, m):
    w, n, p = ring
    G = P.cauchy_search(w, n, p, k, m)[0]
    for s in range(1, m + 1):
        mats = [G[np.ix_(rows, cols)] for rows in itertools.combinations(range(m), s)
                for cols in itertools.combinations(range(k), s)]
        assert sb.det_nonzero_all(mats, w, p).all(), s


def test_cauchy_search_errors():
    with pytest.raises(P.PyritError) as e:
        P.cauchy_search(4, 5, 0x1F, 12, 5)  # 17 points in GF(16)
    assert e.value.code == -4
    with pytest.raises(P.PyritError) as e:
        P.cauchy_search(4, 5, 0x1F, 4, 2, sweeps=-1)
    assert e.value.code == -1
    with pytest.raises(P.PyritError) as e:
        P.cauchy_search(4, 5, 0x1B, 4, 2)  # not the ring's polynomial
    assert e.value.code < 0


@pytest.mark.parametrize("make", [P.cauchy_light, P.cauchy_search], ids=["light", "search"])
def test_generalized_cauchy_decodes_every_pattern_c0_and_c1(make):
    for st, pats in [(W.c0(), [c for s in (1, 2) for c in itertools.combinations(range(6), s)]),
                     (W.c1(), list(itertools.combinations(range(14), 4))[::7])]:
        G = make(st.w, st.n, st.p, st.k, st.m)[0]
        f = oracle.Field(st.w, st.p)
        rng = np.random.Generator(np.random.PCG64(5))
        S = 64
        data = [rng.integers(0, 256, st.w * S, dtype=np.uint8) for _ in range(st.k)]
        code = data + f.encode(G, data, S)
        plan = P.Plan(st.w, st.n, st.p, st.k, st.m, G=G)
        for er in pats:
            blocks = [c.copy() for c in code]
            for e in er:
                blocks[e][:] = 0
            f.decode(G, list(er), blocks, S)
            for e in er:
                assert np.array_equal(blocks[e], code[e]), (st.w, er)
            surv, D = plan.decode_matrix(list(er))
            rec = sb.bitmatrix_encode(D, [code[s] for s in surv], st.w, st.p, S)
            for e, blk in zip(er, rec):
                assert np.array_equal(blk, code[e]), (st.w, er, e)


def test_parity_transform_plans():
    plan = P.Plan(4, 5, 0x1F, 4, 2, transform="parity")
    t = ctypes.c_int()
    assert _lib.lib().pyrit_plan_transform(plan._h, ctypes.byref(t)) == 0 and t.value == 1
    assert plan.transform == "parity"
    # same lifted schedule as the embedding plan: only the ring entry/exit differ
    assert np.array_equal(plan.lifted, P.Plan(4, 5, 0x1F, 4, 2).lifted)
    G = np.ones((2, 4), dtype=np.uint16)
    h = ctypes.c_void_p()
    assert _lib.lib().pyrit_plan_create_ex(4, 5, 0x1F, 4, 2, G.ctypes.data, 2, ctypes.byref(h)) == E["EINVAL"]
    with pytest.raises(ValueError):
        P.Plan(4, 5, 0x1F, 4, 2, transform="other")
    # no parity-transform kernel for the (8,17) ring: plan exists, device calls refuse
    p8 = P.Plan(8, 17, 0x139, 4, 2, transform="parity")
    with pytest.raises(P.PyritError) as e:
        p8.encode([1, 2, 3, 4], [5, 6], 64, stream=0)
    assert e.value.code == E["EUNSUPPORTED"]


def test_decode_matrix_cache_under_threads():
    """Many threads ask one plan for decoding matrices at once (ctypes drops
    the GIL in the call): every answer equals the single-threaded one."""
    import concurrent.futures as cf
    st = W.c1()
    plan = P.Plan(st.w, st.n, st.p, st.k, st.m)
    pats = list(itertools.combinations(range(14), 4))[:120]
    ref = {er: plan.decode_matrix(list(er)) for er in pats[:40]}
    fresh = P.Plan(st.w, st.n, st.p, st.k, st.m)

    def work(i):
        er = pats[(i * 7) % len(pats)]
        surv, D = fresh.decode_matrix(list(er))
        return er, surv, D

    with cf.ThreadPoolExecutor(8) as ex:
        res = list(ex.map(work, range(400)))
    for er, surv, D in res:
        s2, D2 = plan.decode_matrix(list(er))
        assert list(surv) == list(s2) and np.array_equal(D, D2), er
    for er, (s, D) in ref.items():
        assert np.array_equal(D, fresh.decode_matrix(list(er))[1])


class _FakeDeviceTensor:
    """Just enough of a device tensor for the binding's argument checks."""

    def __init__(self, nbytes, contiguous=True, cuda=True):
        self.nbytes, self.contiguous, self.is_cuda = nbytes, contiguous, cuda

    def data_ptr(self):
        return 1 << 36

    def is_contiguous(self):
        return self.contiguous

    def numel(self):
        return self.nbytes

    def element_size(self):
        return 1


def test_binding_refuses_short_or_strided_buffers():
    """The kernels address a block as (w - 1) * pitch + S flat bytes from its
    first element: the binding refuses, before any library call, a tensor
    that holds fewer bytes, a non-contiguous one and a host one."""
    plan = P.Plan(*W.RING_W8, 2, 1)
    S, pitch = 4096, 8192
    need = 7 * pitch + S
    ok = [_FakeDeviceTensor(need) for _ in range(2)]
    for bad, what in [(_FakeDeviceTensor(need - 1), "needed"),
                      (_FakeDeviceTensor(need, contiguous=False), "contiguous"),
                      (_FakeDeviceTensor(need, cuda=False), "device tensors")]:
        with pytest.raises(ValueError, match=what):
            plan.encode(ok, [bad], S, pitch=pitch)
        with pytest.raises(ValueError, match=what):
            plan.decode([0], [bad] + ok, S, pitch=pitch)
        with pytest.raises(ValueError, match=what):
            P.batch_describe([(plan, [], ok + [bad], S, pitch)])
    assert P._block_bytes(8, S, 0) == 8 * S
    # a decode touches only the first k survivors and the erased blocks:
    # block 2 (a survivor past the first k) may be any buffer
    stub = _FakeDeviceTensor(64)
    assert P._coded_blocks(2, 1, [0]) == {0, 1, 2}
    assert P._coded_blocks(2, 2, [1]) == {0, 1, 2}
    assert P._coded_blocks(2, 2, []) == {0, 1, 2, 3}
    plan4 = P.Plan(*W.RING_W8, 2, 2)
    d = P.batch_describe([(plan4, [1], [ok[0], ok[1], _FakeDeviceTensor(need), stub], S, pitch)])
    assert d["moved_bytes"] == 3 * 8 * S
    with pytest.raises(ValueError, match="needed"):
        P.batch_describe([(plan4, [1], [ok[0], ok[1], stub, stub], S, pitch)])
    with pytest.raises(ValueError, match="needed"):
        P.to_sliced(8, _FakeDeviceTensor(4096), _FakeDeviceTensor(4096 - 1), n_symbols=4096)
    with pytest.raises(ValueError, match="needed"):
        P.from_sliced(10, _FakeDeviceTensor(5120), _FakeDeviceTensor(8191), n_symbols=4096)


def test_device_calls_refuse_bad_arguments_before_any_device_work():
    """Encode and decode check every argument on the host before they touch
    the device, so the refusals can be pinned without a GPU: the addresses
    below are never dereferenced and no stream is used."""
    plan = P.Plan(*W.RING_W8, 2, 2)
    A, GiB = 1 << 36, 1 << 30
    d, p = [A, A + GiB], [A + 2 * GiB, A + 3 * GiB]
    EINVAL, ETOOMANY, EALIGN, EUNSUPPORTED = -1, -6, -8, -9
    cases = [
        (lambda: plan.encode(d, p, 0, stream=0), EALIGN),                  # empty slices
        (lambda: plan.encode(d, p, 100, stream=0), EALIGN),                # S not a multiple of 64
        (lambda: plan.encode(d, p, 4096, stream=0, pitch=4032), EINVAL),   # pitch below S
        (lambda: plan.encode(d, p, 4096, stream=0, pitch=4128), EALIGN),   # pitch not a multiple of 64
        (lambda: plan.encode(d, p, 1 << 28, stream=0, pitch=(1 << 28) + (1 << 26)), EINVAL),  # 2^31 window
        (lambda: plan.encode([A + 8, A + GiB], p, 4096, stream=0), EALIGN),  # pointer not 16-byte aligned
        (lambda: plan.encode([None, A + GiB], p, 4096, stream=0), EINVAL),   # missing input
        (lambda: plan.encode(d, p, 4096, stream=0, vec_bytes=12), EINVAL),
        (lambda: plan.decode([0, 0], d + p, 4096, stream=0), EINVAL),      # repeated erasure
        (lambda: plan.decode([4], d + p, 4096, stream=0), EINVAL),         # id past k + m
        (lambda: plan.decode([-1], d + p, 4096, stream=0), EINVAL),
        (lambda: plan.decode([0, 1, 2], d + p, 4096, stream=0), ETOOMANY),
        (lambda: P.Plan(3, 7, 0xB, 2, 1).encode(d, [A + 2 * GiB], 4096, stream=0), EUNSUPPORTED),
    ]
    for i, (call, code) in enumerate(cases):
        with pytest.raises(P.PyritError) as e:
            call()
        assert e.value.code == code, i
