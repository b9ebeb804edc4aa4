"""Seeded synthetic workloads: code parameters, input bytes, erasure patterns.

This module holds no coding arithmetic (no field, ring or matrix operation).
It only fixes *what* is coded: the code parameters of each workload, the
seeded random bytes of every block, the erasure patterns and the request
trace.  Both the accelerated library and the CPU oracle consume its outputs.

Input bytes come from a counter-based generator so that any byte of any block
can be produced on its own (the GPU fills whole buffers with the library's
own implementation; the tests regenerate sampled bytes here):

  SplitMix64 (Steele, Lea & Flood, OOPSLA 2014): with golden gamma
  G = 0x9E3779B97F4A7C15 and finaliser
      mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9;
              z ^= z >> 27; z *= 0x94D049BB133111EB; z ^= z >> 31
  the i-th output (i >= 1) of a generator with state s is mix(s + i*G).

  block key  K(seed, stripe, block) = mix(seed + (stripe*256 + block + 1) * G)
  word q     of a block              = mix(K + (q + 1) * G)
  byte i     of a block              = byte (i mod 8) of word (i div 8), little
                                       endian, for i < nrandom; 0 beyond.

A block is ``w`` slices of ``S`` bytes (slice t holds coefficient t of every
symbol, Sec. III of the paper); for a user block of B bytes,
``S = roundup(ceil(B / w), 64)`` and bytes ``B .. w*S`` are zero.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
MASK64 = (1 << 64) - 1
BASE_SEED = 170900178

# (w, n, p): the fields and rings used by the workloads.  p includes x^w.
RING_W4 = (4, 5, 0x1F)      # x^4+x^3+x^2+x+1, all-one polynomial, n = w + 1
RING_W8 = (8, 17, 0x139)    # x^8+x^5+x^4+x^3+1, a degree-8 factor of x^17+1
RING_W10 = (10, 11, 0x7FF)  # all-one polynomial of degree 10, n = w + 1
RING_W6 = (6, 9, 0x49)      # x^6+x^3+1, equally spaced polynomial, n = 9
RINGS = {4: RING_W4, 8: RING_W8, 10: RING_W10, 6: RING_W6}


def _mix_scalar(z: int) -> int:
    z &= MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.astype(np.uint64, copy=True)
    with np.errstate(over="ignore"):
        z ^= z >> np.uint64(30)
        z *= np.uint64(0xBF58476D1CE4E5B9)
        z ^= z >> np.uint64(27)
        z *= np.uint64(0x94D049BB133111EB)
        z ^= z >> np.uint64(31)
    return z


def block_key(seed: int, stripe: int, block: int) -> int:
    return _mix_scalar(seed + ((stripe * 256 + block + 1) * GAMMA))


def words(key: int, q0: int, q1: int) -> np.ndarray:
    """Words q0..q1-1 of the stream with the given key."""
    q = np.arange(q0, q1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        s = np.uint64(key) + (q + np.uint64(1)) * np.uint64(GAMMA)
    return _mix(s)


def block_bytes(key: int, nbytes: int, nrandom: int | None = None) -> np.ndarray:
    """All bytes of one block buffer."""
    if nrandom is None:
        nrandom = nbytes
    nw = (nrandom + 7) // 8
    out = np.zeros(nbytes, dtype=np.uint8)
    out[:nrandom] = words(key, 0, nw).view(np.uint8)[:nrandom]
    return out


def block_bytes_at(key: int, offsets: np.ndarray, nrandom: int) -> np.ndarray:
    """Bytes of a block at the given offsets (for sampled checks at full size)."""
    offsets = np.asarray(offsets, dtype=np.int64)
    q = (offsets // 8).astype(np.uint64)
    with np.errstate(over="ignore"):
        wv = _mix(np.uint64(key) + (q + np.uint64(1)) * np.uint64(GAMMA))
    b = ((wv >> ((offsets % 8).astype(np.uint64) * np.uint64(8))) & np.uint64(0xFF)).astype(np.uint8)
    b[offsets >= nrandom] = 0
    return b


def slice_bytes(B: int, w: int) -> int:
    """Slice size S for a user block of B bytes: roundup(ceil(B/w), 64)."""
    s = -(-B // w)
    return -(-s // 64) * 64


@dataclasses.dataclass(frozen=True)
class Stripe:
    """One codeword to encode or decode."""
    w: int
    n: int
    p: int
    k: int
    m: int
    B: int                      # user bytes per block
    erased: tuple = ()          # empty: encode; else: decode of these blocks
    stripe: int = 0             # index used in block keys
    seed: int = BASE_SEED
    pad: int = 0                # bytes between consecutive slices in memory

    @property
    def S(self) -> int:
        return slice_bytes(self.B, self.w)

    @property
    def pitch(self) -> int:
        """Slice stride in memory: S for the packed layout, S + pad else."""
        return self.S + self.pad

    @property
    def data_len(self) -> int:
        """Bytes of the w slices (the logical block)."""
        return self.w * self.S

    @property
    def block_len(self) -> int:
        """Bytes a block occupies in memory: w slices at the pitch."""
        return self.w * self.pitch

    @property
    def nrandom(self) -> int:
        """Memory bytes of a block holding generator output (zero beyond).
        Packed blocks carry B random bytes; padded blocks (which require
        B == w * S) are random over their whole memory, padding included."""
        if self.pad == 0:
            return self.B
        assert self.B == self.w * self.S, "padded layouts need B == w * S"
        return self.block_len

    def key(self, block: int) -> int:
        return block_key(self.seed, self.stripe, block)

    def moved_bytes(self) -> int:
        """Bytes a coding pass reads and writes: (k + outputs) * w * S."""
        outs = len(self.erased) if self.erased else self.m
        return (self.k + outs) * self.data_len


# ---------------------------------------------------------------- workloads
def c0() -> Stripe:
    """GF(2^4) in R_{2,5}; k=4, m=2; 64 KiB blocks (S = 16 KiB)."""
    return Stripe(*RING_W4, k=4, m=2, B=64 * 1024, seed=BASE_SEED)


def c0_erasure_patterns():
    """All 15 two-erasure patterns of the 6 blocks."""
    n = 6
    return [(a, b) for a in range(n) for b in range(a + 1, n)]


def c1() -> Stripe:
    """GF(2^8) in R_{2,17}; k=10, m=4; one stripe of 64 MiB blocks (S = 8 MiB)."""
    return Stripe(*RING_W8, k=10, m=4, B=64 * 1024 * 1024, seed=BASE_SEED + 1)


def c1_erasure_patterns():
    """A seeded uniform 4-subset of the 14 blocks, plus all four leading data blocks."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 1))
    pick = tuple(sorted(int(x) for x in rng.choice(14, size=4, replace=False)))
    return [pick, (0, 1, 2, 3)]


def c2(n_stripes: int = 256) -> list:
    """GF(2^10) in R_{2,11}; k=16, m=4; 256 stripes of 16 x 4 MiB blocks."""
    return [Stripe(*RING_W10, k=16, m=4, B=4 * 1024 * 1024, stripe=s, seed=BASE_SEED + 2)
            for s in range(n_stripes)]


def draw_stripe(rng: np.random.Generator, stripe: int, seed: int,
                decode_frac: float = 0.3) -> Stripe:
    """One stripe of the uneven batch distribution.

    w uniform in {4, 8, 10}; k uniform in [4, 16]; m uniform in [2, 4]; for
    w = 4 (k, m) is redrawn until k + m <= 16, the symbol-count limit of
    GF(2^4) codes.  Block size log-uniform in [4 KiB, 4 MiB], rounded to a
    multiple of 64 bytes.  With probability ``decode_frac`` the stripe is a
    decode of e ~ U{1..m} erasures drawn uniformly among the k + m blocks.
    """
    w = int(rng.choice([4, 8, 10]))
    while True:
        k = int(rng.integers(4, 17))
        m = int(rng.integers(2, 5))
        if w != 4 or k + m <= 16:
            break
    lb = rng.uniform(math.log(4096), math.log(4 * 1024 * 1024))
    B = int(round(math.exp(lb) / 64.0)) * 64
    B = min(max(B, 4096), 4 * 1024 * 1024)
    erased = ()
    if rng.uniform() < decode_frac:
        e = int(rng.integers(1, m + 1))
        erased = tuple(sorted(int(x) for x in rng.choice(k + m, size=e, replace=False)))
    return Stripe(*RINGS[w], k=k, m=m, B=B, erased=erased, stripe=stripe, seed=seed)


def c3(n_stripes: int = 4096) -> list:
    """4096 uneven stripes (30% decodes), one batch."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 3))
    return [draw_stripe(rng, s, BASE_SEED + 3) for s in range(n_stripes)]


@dataclasses.dataclass(frozen=True)
class Request:
    arrival_s: float
    stripe: Stripe
    large: bool


def c4(rate: float = 20000.0, duration_s: float = 2.0, large_frac: float = 0.05) -> list:
    """Poisson arrivals of encode/decode requests: the uneven distribution plus
    ``large_frac`` of k=10, m=4, GF(2^8) requests with 64 MiB blocks."""
    rng = np.random.Generator(np.random.PCG64(BASE_SEED + 4))
    t, out, i = 0.0, [], 0
    while True:
        t += float(rng.exponential(1.0 / rate))
        if t >= duration_s:
            break
        if rng.uniform() < large_frac:
            st = Stripe(*RING_W8, k=10, m=4, B=64 * 1024 * 1024, stripe=i, seed=BASE_SEED + 4)
            if rng.uniform() < 0.3:
                e = int(rng.integers(1, 5))
                er = tuple(sorted(int(x) for x in rng.choice(14, size=e, replace=False)))
                st = dataclasses.replace(st, erased=er)
            out.append(Request(t, st, True))
        else:
            out.append(Request(t, draw_stripe(rng, i, BASE_SEED + 4), False))
        i += 1
    return out


def survivors(st: Stripe) -> tuple:
    """Input block ids of a pass: the k data blocks for an encode, else the
    first k block ids (in 0 .. k+m-1) that are not erased."""
    if not st.erased:
        return tuple(range(st.k))
    er = set(st.erased)
    return tuple(i for i in range(st.k + st.m) if i not in er)[: st.k]


def host_blocks(st: Stripe, blocks=None) -> list:
    """Host copies of the input blocks of a pass (or of the listed block ids).

    Every input block carries random bytes keyed by its block id.  A decode is
    a fixed linear map of its k survivors, so random survivor bytes are a
    valid input; codeword round trips are checked separately.
    """
    ids = survivors(st) if blocks is None else blocks
    return [logical(st, block_bytes(st.key(j), st.block_len, st.nrandom)) for j in ids]


def logical(st: Stripe, mem: np.ndarray) -> np.ndarray:
    """The w slices of a block's memory image, packed (w * S bytes)."""
    if st.pad == 0:
        return mem
    return np.concatenate([mem[t * st.pitch:t * st.pitch + st.S] for t in range(st.w)])
