"""CPU oracle for systematic MDS erasure coding over GF(2^w).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The accelerated library never imports
this package, and this package never imports the library.

Thin ctypes binding over ``pyrit_oracle.c`` (plain C, log/antilog tables).
Blocks are numpy ``uint8`` arrays of ``w * S`` bytes: slice ``t`` of a block is
``block[t*S:(t+1)*S]`` (the paper's "w chunks" of a block, Sec. III).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pyrit_oracle.c")
# PYRIT_ORACLE_MUTANT=n builds and loads a copy with planted mistake n (see
# OR_MUTANT in the C source) under PYRIT_ORACLE_DIR; only the mutant test
# sets them, to show that the pins reject every planted mistake.
_MUTANT = int(os.environ.get("PYRIT_ORACLE_MUTANT", "0"))
_LIB_PATH = (os.path.join(_HERE, "liboracle.so") if _MUTANT == 0 else
             os.path.join(os.environ["PYRIT_ORACLE_DIR"], f"liboracle_m{_MUTANT}.so"))

ERRORS = {0: "ok", -1: "invalid argument", -2: "modulus not irreducible",
          -3: "code too long for the field", -4: "singular matrix",
          -5: "too many erasures", -6: "out of memory"}


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no intrinsics)."""
    # a temporary name of this process's own, so that builds running at the
    # same time (parallel test workers) each replace the library whole
    tmp = f"{_LIB_PATH}.tmp{os.getpid():x}"
    cmd = ["gcc", "-O2", "-fopenmp", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
           f"-DOR_MUTANT={_MUTANT}", _SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    vp, u32, i32, sz = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_int, ctypes.c_size_t
    lib.or_field_create.argtypes = [i32, u32, ctypes.POINTER(vp)]
    lib.or_field_create.restype = i32
    lib.or_field_free.argtypes = [vp]
    lib.or_field_free.restype = None
    lib.or_field_generator.argtypes = [vp]
    lib.or_field_generator.restype = u32
    lib.or_mul.argtypes = [vp, u32, u32]
    lib.or_mul.restype = u32
    lib.or_inv.argtypes = [vp, u32]
    lib.or_inv.restype = u32
    lib.or_mul_many.argtypes = [vp, vp, vp, vp, sz]
    lib.or_mul_many.restype = None
    lib.or_cauchy.argtypes = [vp, i32, i32, vp]
    lib.or_cauchy.restype = i32
    lib.or_invert.argtypes = [vp, i32, vp]
    lib.or_invert.restype = i32
    lib.or_encode.argtypes = [vp, i32, i32, vp, vp, vp, sz, sz, sz, i32]
    lib.or_encode.restype = i32
    lib.or_decode.argtypes = [vp, i32, i32, vp, vp, i32, vp, sz, sz, sz, i32]
    lib.or_decode.restype = i32
    lib.or_max_threads.argtypes = []
    lib.or_max_threads.restype = i32
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {ERRORS.get(code, 'unknown')}")
        self.code = code


def _check(rc: int) -> None:
    if rc != 0:
        raise OracleError(rc)


def max_threads() -> int:
    return int(_load().or_max_threads())


def _ptr_array(arrs):
    t = (ctypes.c_void_p * len(arrs))()
    for i, a in enumerate(arrs):
        assert a.dtype == np.uint8 and a.flags["C_CONTIGUOUS"]
        t[i] = a.ctypes.data
    return t


class Field:
    """GF(2^w) = F_2[x]/(p) with log/antilog tables (Sec. II-A)."""

    def __init__(self, w: int, p: int):
        lib = _load()
        h = ctypes.c_void_p()
        _check(lib.or_field_create(w, p, ctypes.byref(h)))
        self._h = h
        self.w, self.p = w, p

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and _lib is not None:
            _lib.or_field_free(h)
            self._h = None

    @property
    def generator(self) -> int:
        return int(_lib.or_field_generator(self._h))

    def mul(self, a: int, b: int) -> int:
        return int(_lib.or_mul(self._h, a, b))

    def inv(self, a: int) -> int:
        return int(_lib.or_inv(self._h, a))

    def mul_many(self, a, b) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.uint32)
        b = np.ascontiguousarray(b, dtype=np.uint32)
        out = np.empty_like(a)
        _lib.or_mul_many(self._h, a.ctypes.data, b.ctypes.data, out.ctypes.data, a.size)
        return out

    def cauchy(self, k: int, m: int) -> np.ndarray:
        C = np.zeros((m, k), dtype=np.uint16)
        _check(_lib.or_cauchy(self._h, k, m, C.ctypes.data))
        return C

    def invert(self, A) -> np.ndarray:
        A = np.array(A, dtype=np.uint16, order="C")
        _check(_lib.or_invert(self._h, A.shape[0], A.ctypes.data))
        return A

    def encode(self, C, data, S: int, o0: int = 0, o1: int | None = None,
               nthreads: int = 1, parity=None):
        """Parity blocks for ``data`` (list of k blocks of w*S bytes)."""
        C = np.ascontiguousarray(C, dtype=np.uint16)
        m, k = C.shape
        assert len(data) == k
        if o1 is None:
            o1 = S
        if parity is None:
            parity = [np.zeros(self.w * S, dtype=np.uint8) for _ in range(m)]
        _check(_lib.or_encode(self._h, k, m, C.ctypes.data, _ptr_array(data),
                              _ptr_array(parity), S, o0, o1, nthreads))
        return parity

    def decode(self, C, erased, blocks, S: int, o0: int = 0, o1: int | None = None,
               nthreads: int = 1):
        """Overwrite the erased entries of ``blocks`` (k+m blocks) in place."""
        C = np.ascontiguousarray(C, dtype=np.uint16)
        m, k = C.shape
        assert len(blocks) == k + m
        if o1 is None:
            o1 = S
        er = (ctypes.c_int * max(1, len(erased)))(*erased)
        _check(_lib.or_decode(self._h, k, m, C.ctypes.data, er, len(erased),
                              _ptr_array(blocks), S, o0, o1, nthreads))
        return blocks


def to_sliced(w: int, symbols) -> np.ndarray:
    """Bit-sliced block of ``symbols`` (n symbols, n a multiple of 8): slice t
    holds bit t of every symbol, symbol 8o + b at bit b of byte o (the
    block's w chunks, Sec. III).  Returns w * n/8 bytes, slice after slice."""
    u = np.asarray(symbols).astype(np.uint32).reshape(-1)
    n = u.size
    assert n % 8 == 0
    S = n // 8
    out = np.zeros((w, S), dtype=np.uint32)
    for t in range(w):
        bits = ((u >> t) & 1).reshape(S, 8)
        for b in range(8):
            out[t] |= bits[:, b] << b
    return out.astype(np.uint8).reshape(-1)


def from_sliced(w: int, sliced, n: int) -> np.ndarray:
    """Inverse of `to_sliced`: the n symbols (uint16) of a bit-sliced block."""
    S = n // 8
    blk = np.asarray(sliced, dtype=np.uint8).reshape(w, S).astype(np.uint32)
    sym = np.zeros((S, 8), dtype=np.uint32)
    for t in range(w):
        for b in range(8):
            sym[:, b] |= ((blk[t] >> b) & 1) << t
    return sym.reshape(-1).astype(np.uint16)


# ---------------------------------------------------------------------------
# The parity transform (Sec. II-C.1 for the all-one polynomial, Sec. II-D.1
# for the equally spaced x^6+x^3+1).  A symbol b enters the ring as the one
# element of the ideal isomorphic to the field whose low w coefficients are
# b (the ideal is generated by h = (x^n + 1) / p: for the AOP the even-weight
# words, for the ESP three interleaved even-weight words); results leave the
# ring by dropping the n - w high coefficients.  This is a bijection, not the
# field isomorphism, so the code differs from [I; C]: with
# psi(b) = phi_P(b) mod p, parity_i = psi^-1(sum_j C[i][j] psi(d_j)).

def _poly_mod(a: int, m: int) -> int:
    dm = m.bit_length() - 1
    while a and a.bit_length() - 1 >= dm:
        a ^= m << (a.bit_length() - 1 - dm)
    return a


def _poly_div(a: int, m: int) -> int:
    q, dm = 0, m.bit_length() - 1
    while a and a.bit_length() - 1 >= dm:
        s = a.bit_length() - 1 - dm
        q |= 1 << s
        a ^= m << s
    assert a == 0, "p must divide x^n + 1"
    return q


def parity_embed_table(w: int, n: int, p: int) -> np.ndarray:
    """phi_P(b) for every symbol b: b plus the high coefficients q (deg q <
    n - w) that make it a multiple of h = (x^n + 1) / p, found by search."""
    h = _poly_div((1 << n) | 1, p)
    out = np.zeros(1 << w, dtype=np.uint32)
    for b in range(1 << w):
        hits = [q for q in range(1 << (n - w)) if _poly_mod(b | (q << w), h) == 0]
        assert len(hits) == 1
        out[b] = b | (hits[0] << w)
    return out


def psi_table(w: int, n: int, p: int) -> np.ndarray:
    """psi(b) = phi_P(b) mod p for every symbol b."""
    return np.array([_poly_mod(int(a), p) for a in parity_embed_table(w, n, p)], dtype=np.uint32)


def _map_symbols(w: int, block: np.ndarray, table: np.ndarray) -> np.ndarray:
    n = block.size // w * 8
    return to_sliced(w, table[from_sliced(w, block, n)])


def encode_parity_transform(f: "Field", n: int, C, data, S: int):
    """Parity blocks of the parity-transform code over ring R_{2,n}."""
    psi = psi_table(f.w, n, f.p)
    inv = np.argsort(psi).astype(np.uint32)
    tdata = [_map_symbols(f.w, np.ascontiguousarray(d), psi) for d in data]
    return [_map_symbols(f.w, b, inv) for b in f.encode(C, tdata, S)]


def decode_parity_transform(f: "Field", n: int, C, erased, blocks, S: int):
    """Overwrite the erased blocks of a parity-transform codeword in place."""
    psi = psi_table(f.w, n, f.p)
    inv = np.argsort(psi).astype(np.uint32)
    er = set(erased)
    tb = [b if i in er else _map_symbols(f.w, b, psi) for i, b in enumerate(blocks)]
    tb = [np.ascontiguousarray(b) for b in tb]
    f.decode(C, list(erased), tb, S)
    for e in erased:
        blocks[e][:] = _map_symbols(f.w, tb[e], inv)
    return blocks
