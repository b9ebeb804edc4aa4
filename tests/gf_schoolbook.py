"""Textbook GF(2)[x] arithmetic written independently for the tests.

Schoolbook carry-less multiplication with reduction after every shift, and the
binary-matrix form of multiplication by a constant (column b of the matrix of
u is u * x^b mod p).  Neither the oracle nor the library is imported here.
"""
import numpy as np


def mul(a, b, w, p):
    """Vectorised schoolbook product of field elements a*b mod p."""
    a = np.array(a, dtype=np.int64, copy=True)
    b = np.asarray(b, dtype=np.int64)
    r = np.zeros(np.broadcast(a, b).shape, dtype=np.int64)
    for i in range(w):
        r ^= np.where((b >> i) & 1, a, 0)
        a = a << 1
        a ^= np.where((a >> w) & 1, p, 0)
    return r


def poly_mul(a: int, b: int) -> int:
    """Carry-less product of two polynomials over GF(2) (no reduction)."""
    r = 0
    while b:
        if b & 1:
            r ^= a
        a <<= 1
        b >>= 1
    return r


def poly_mod(a: int, p: int) -> int:
    dp = p.bit_length() - 1
    while a and a.bit_length() - 1 >= dp:
        a ^= p << (a.bit_length() - 1 - dp)
    return a


def ring_mul(a: int, b: int, n: int) -> int:
    """Product in F_2[x]/(x^n + 1)."""
    return poly_mod(poly_mul(a, b), (1 << n) | 1)


def is_irreducible(p: int) -> bool:
    """Trial division by every polynomial of degree 1 .. deg(p)/2."""
    d = p.bit_length() - 1
    for q in range(2, 1 << (d // 2 + 1)):
        if poly_mod(p, q) == 0:
            return False
    return True


def inverse_table(w, p):
    """inv[a] by exhaustive search over the schoolbook product."""
    q = 1 << w
    a = np.arange(q, dtype=np.int64)
    inv = np.zeros(q, dtype=np.int64)
    for b in range(1, q):
        hit = mul(a, b, w, p) == 1
        inv[hit] = b
    return inv


def mul_table(w, p):
    q = 1 << w
    a = np.arange(q, dtype=np.int64)
    return mul(a[:, None], a[None, :], w, p)


def bitmatrix(u, w, p):
    """w x w binary matrix M with M[t][b] = bit t of u * x^b mod p."""
    M = np.zeros((w, w), dtype=np.uint8)
    col = int(u)
    for b in range(w):
        for t in range(w):
            M[t, b] = (col >> t) & 1
        col <<= 1
        if (col >> w) & 1:
            col ^= p
    return M


def bitmatrix_encode(G, data, w, p, S):
    """Parity blocks from the binary-matrix form: slice t of parity i is the
    XOR of slice b of data j over all ones M(G[i][j])[t][b]."""
    G = np.asarray(G)
    m, k = G.shape
    out = []
    for i in range(m):
        blk = np.zeros(w * S, dtype=np.uint8)
        for j in range(k):
            M = bitmatrix(G[i, j], w, p)
            for t in range(w):
                for b in range(w):
                    if M[t, b]:
                        blk[t * S:(t + 1) * S] ^= data[j][b * S:(b + 1) * S]
        out.append(blk)
    return out


def det_nonzero_all(mats, w, p, mt=None, inv=None):
    """For a stack of square matrices over GF(2^w), True where invertible.

    Gaussian elimination vectorised over the stack with table lookups built
    from the schoolbook product.
    """
    if mt is None:
        mt = mul_table(w, p)
    if inv is None:
        inv = inverse_table(w, p)
    A = np.array(mats, dtype=np.int64, copy=True)
    nb, k, _ = A.shape
    ok = np.ones(nb, dtype=bool)
    idx = np.arange(nb)
    for c in range(k):
        col = A[:, c:, c]
        nz = col != 0
        has = nz.any(axis=1)
        ok &= has
        piv = c + np.argmax(nz, axis=1)
        rows_c = A[idx, c, :].copy()
        A[idx, c, :] = A[idx, piv, :]
        A[idx, piv, :] = rows_c
        s = inv[A[:, c, c]]
        A[:, c, :] = mt[s[:, None], A[:, c, :]]
        for r in range(k):
            if r == c:
                continue
            e = A[:, r, c]
            A[:, r, :] ^= mt[e[:, None], A[:, c, :]]
    return ok
