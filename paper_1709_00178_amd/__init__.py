"""PYRIT on MI355X: systematic MDS erasure coding over GF(2^w) computed as
rotated-slice XORs in the ring F_2[x]/(x^n + 1) (Detchart & Lacan).

Python binding over the C ABI in ``include/pyrit.h``.  Every coding step runs
in the library's HIP kernels; torch is used only to hand over device pointers
and the current stream.  Block buffers are uint8 device tensors of w * S
bytes (w slices of S bytes).
"""
from __future__ import annotations

import ctypes

import numpy as np

from ._lib import lib

__all__ = ["PyritError", "Plan", "Batch", "batch_run_noalloc", "ring_check", "ring_supported", "lift", "ring_reduce",
           "ring_mul", "gf_mul", "cauchy", "cauchy_light", "cauchy_search", "fill_random", "fill_random_blocks", "copy", "version"]

PYRIT_OK = 0


class PyritError(RuntimeError):
    def __init__(self, code: int):
        msg = lib().pyrit_strerror(code).decode()
        super().__init__(f"pyrit error {code}: {msg}")
        self.code = code


def _check(rc: int) -> None:
    if rc != PYRIT_OK:
        raise PyritError(rc)


def version() -> str:
    return lib().pyrit_version().decode()


def ring_check(w: int, n: int, p: int) -> int:
    """0 when (w, n, p) is a valid field/ring pair, else the error code."""
    return int(lib().pyrit_ring_check(w, n, p))


def ring_supported(w: int, n: int, p: int) -> bool:
    return bool(lib().pyrit_ring_supported(w, n, p))


def lift(w: int, n: int, p: int, u: int) -> int:
    c = ctypes.c_uint32()
    _check(lib().pyrit_lift(w, n, p, u, ctypes.byref(c)))
    return c.value


def ring_reduce(w: int, n: int, p: int, c: int) -> int:
    u = ctypes.c_uint32()
    _check(lib().pyrit_ring_reduce(w, n, p, c, ctypes.byref(u)))
    return u.value


def ring_mul(n: int, a: int, b: int) -> int:
    c = ctypes.c_uint32()
    _check(lib().pyrit_ring_mul(n, a, b, ctypes.byref(c)))
    return c.value


def gf_mul(w: int, p: int, a: int, b: int) -> int:
    c = ctypes.c_uint32()
    _check(lib().pyrit_gf_mul(w, p, a, b, ctypes.byref(c)))
    return c.value


def cauchy(w: int, p: int, k: int, m: int) -> np.ndarray:
    G = np.zeros((m, k), dtype=np.uint16)
    _check(lib().pyrit_cauchy(w, p, k, m, G.ctypes.data))
    return G


def cauchy_light(w: int, n: int, p: int, k: int, m: int):
    """Generalized Cauchy matrix with row/column multipliers chosen for a
    small lifted weight in R_{2,n}: returns (G, row_scale, col_scale, weight)."""
    G = np.zeros((m, k), dtype=np.uint16)
    rs = np.zeros(m, dtype=np.uint16)
    cs = np.zeros(k, dtype=np.uint16)
    wt = ctypes.c_int()
    _check(lib().pyrit_cauchy_light(w, n, p, k, m, G.ctypes.data, rs.ctypes.data, cs.ctypes.data,
                                    ctypes.byref(wt)))
    return G, rs, cs, wt.value


def cauchy_search(w: int, n: int, p: int, k: int, m: int, sweeps: int = 4):
    """Generalized Cauchy matrix with points and row/column multipliers
    chosen for a small lifted weight in R_{2,n} (pyrit_cauchy_search):
    returns (G, X, Y, row_scale, col_scale, weight), G[i][j] =
    row_scale[i] * col_scale[j] / (X[i] + Y[j])."""
    G = np.zeros((m, k), dtype=np.uint16)
    X = np.zeros(m, dtype=np.uint16)
    Y = np.zeros(k, dtype=np.uint16)
    rs = np.zeros(m, dtype=np.uint16)
    cs = np.zeros(k, dtype=np.uint16)
    wt = ctypes.c_int()
    _check(lib().pyrit_cauchy_search(w, n, p, k, m, sweeps, G.ctypes.data, X.ctypes.data,
                                     Y.ctypes.data, rs.ctypes.data, cs.ctypes.data,
                                     ctypes.byref(wt)))
    return G, X, Y, rs, cs, wt.value


def _dev_ptr(x, need: int = 0) -> int:
    """Device address of a tensor (or a plain integer address, taken as is).
    A tensor must be a contiguous device tensor of at least ``need`` bytes:
    the kernels address a buffer as flat bytes from its first element."""
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        if not x.is_cuda:
            raise ValueError("block buffers must be device tensors")
        if not x.is_contiguous():
            raise ValueError("device buffers must be contiguous")
        have = x.numel() * x.element_size()
        if have < need:
            raise ValueError(f"device buffer holds {have} bytes, {need} needed")
        return int(x.data_ptr())
    raise TypeError(f"expected a device tensor or a pointer, got {type(x)}")


def _block_bytes(w: int, S: int, pitch: int) -> int:
    """Bytes a block of w slices of S bytes at a stride of pitch spans."""
    return (w - 1) * (pitch or S) + S


def _stream_handle(stream) -> int | None:
    if stream is None:
        import torch
        return int(torch.cuda.current_stream().cuda_stream) or None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


def _coded_blocks(k: int, m: int, erased) -> set:
    """Ids of the blocks a call reads or writes: all k + m for an encode; for
    a decode the first k survivors and the erased blocks (other entries are
    never touched)."""
    if not erased:
        return set(range(k + m))
    er = set(erased)
    return set([b for b in range(k + m) if b not in er][:k]) | er


def _ptr_array(xs, need: int = 0, used=None):
    """C array of device addresses; entries in ``used`` (default: all) must
    hold ``need`` bytes."""
    arr = (ctypes.c_void_p * max(1, len(xs)))()
    for i, x in enumerate(xs):
        n = need if used is None or i in used else 0
        arr[i] = _dev_ptr(x, n) if x is not None else None
    return arr


class Plan:
    """A code [I_k; G] over GF(2^w) = F_2[x]/(p), lifted into R_{2,n}.

    ``G`` (m x k) defaults to the plain Cauchy matrix 1 / (i + m + j).
    ``transform``: "embedding" (the field code [I; G]) or "parity" (the
    paper's parity transform, a different MDS code; see pyrit.h).
    """

    TRANSFORMS = {"embedding": 0, "parity": 1}

    def __init__(self, w: int, n: int, p: int, k: int, m: int, G=None,
                 transform: str = "embedding"):
        if G is None:
            G = cauchy(w, p, k, m)
        G = np.ascontiguousarray(G, dtype=np.uint16)
        if G.shape != (m, k):
            raise ValueError(f"G must be {m}x{k}")
        if transform not in self.TRANSFORMS:
            raise ValueError(f"transform must be one of {sorted(self.TRANSFORMS)}")
        h = ctypes.c_void_p()
        _check(lib().pyrit_plan_create_ex(w, n, p, k, m, G.ctypes.data, self.TRANSFORMS[transform],
                                          ctypes.byref(h)))
        self._h = h
        self.w, self.n, self.p, self.k, self.m = w, n, p, k, m
        self.transform = transform
        self.G = G.copy()

    def close(self):
        if getattr(self, "_h", None):
            lib().pyrit_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def handle(self) -> int:
        return self._h.value

    @property
    def lifted(self) -> np.ndarray:
        C = np.zeros((self.m, self.k), dtype=np.uint32)
        _check(lib().pyrit_plan_lifted(self._h, C.ctypes.data))
        return C

    @property
    def weight(self) -> int:
        wt = ctypes.c_int()
        _check(lib().pyrit_plan_weight(self._h, ctypes.byref(wt)))
        return wt.value

    def decode_matrix(self, erased):
        er = (ctypes.c_int * max(1, len(erased)))(*erased)
        surv = np.zeros(self.k, dtype=np.int32)
        D = np.zeros((len(erased), self.k), dtype=np.uint16)
        _check(lib().pyrit_decode_matrix(self._h, er, len(erased), surv.ctypes.data,
                                         D.ctypes.data))
        return surv, D

    def encode(self, data, parity, S: int, stream=None, vec_bytes: int = 0,
               pitch: int = 0) -> None:
        """parity[i] = sum_j G[i][j] * data[j]; blocks are w slices of S bytes
        at a stride of ``pitch`` bytes (0: packed, pitch = S)."""
        if len(data) != self.k or len(parity) != self.m:
            raise ValueError("need k data and m parity buffers")
        need = _block_bytes(self.w, S, pitch)
        _check(lib().pyrit_encode_ex(self._h, _ptr_array(data, need), _ptr_array(parity, need), S,
                                     pitch, vec_bytes, _stream_handle(stream)))

    def decode(self, erased, blocks, S: int, stream=None, pitch: int = 0) -> None:
        """Rewrite the erased entries of ``blocks`` (k + m buffers)."""
        if len(blocks) != self.k + self.m:
            raise ValueError("need k + m block buffers")
        er = (ctypes.c_int * max(1, len(erased)))(*erased)
        _check(lib().pyrit_decode_ex(self._h, er, len(erased),
                                     _ptr_array(blocks, _block_bytes(self.w, S, pitch),
                                                _coded_blocks(self.k, self.m, erased)), S, pitch,
                                     _stream_handle(stream)))


def _batch_items(items):
    """C item array for batch items; returns it with what keeps it alive."""
    from ._lib import BatchItem
    keep = []
    arr = (BatchItem * max(1, len(items)))()
    for i, it in enumerate(items):
        plan, erased, blocks, S = it[:4]
        pitch = it[4] if len(it) > 4 else 0
        if len(blocks) != plan.k + plan.m:
            raise ValueError("each item needs k + m block entries")
        er = (ctypes.c_int * max(1, len(erased)))(*erased)
        bl = _ptr_array(blocks, _block_bytes(plan.w, S, pitch),
                        _coded_blocks(plan.k, plan.m, erased))
        keep += [er, bl, plan]
        arr[i].plan = plan._h
        arr[i].n_erased = len(erased)
        arr[i].erased = ctypes.cast(er, ctypes.POINTER(ctypes.c_int))
        arr[i].blocks = ctypes.cast(bl, ctypes.POINTER(ctypes.c_void_p))
        arr[i].slice_bytes = S
        arr[i].slice_pitch = pitch
    return arr, keep


def _batch_tune(mode, tile_bytes, grid, wg_threads, xcd_order, split_k):
    from ._lib import BATCH_MODES, Tune
    if mode not in BATCH_MODES:
        raise ValueError(f"mode must be one of {sorted(BATCH_MODES)}")
    return Tune(BATCH_MODES[mode], tile_bytes, grid, wg_threads, xcd_order, split_k)


def batch_describe(items, mode: str = "grid", tile_bytes: int = 0, grid: int = 0,
                   wg_threads: int = 0, xcd_order: int = 0, split_k: int = 0) -> dict:
    """The work a `Batch` of these items would launch, computed on the host
    (pyrit_batch_describe): passes, work items, bytes moved, workgroups, and
    the bytes of each XCD's item range (grid mode with xcd_order=1).  Block
    entries may be plain integer addresses; nothing touches the device."""
    items = list(items)
    arr, keep = _batch_items(items)
    tune = _batch_tune(mode, tile_bytes, grid, wg_threads, xcd_order, split_k)
    np_, ni, gr = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    mv = ctypes.c_uint64()
    xb = (ctypes.c_uint64 * 8)()
    _check(lib().pyrit_batch_describe(arr, len(items), ctypes.byref(tune), ctypes.byref(np_),
                                      ctypes.byref(ni), ctypes.byref(mv), ctypes.byref(gr), xb))
    del keep
    return {"passes": np_.value, "work_items": ni.value, "moved_bytes": mv.value,
            "grid": gr.value, "xcd_bytes": list(xb)}


def batch_run_noalloc(items, mode: str = "grid", tile_bytes: int = 0, grid: int = 0,
                      wg_threads: int = 0, xcd_order: int = 0, split_k: int = 0,
                      stream=None) -> None:
    """One run of a batch of these items without allocating device memory
    (pyrit_batch_run_noalloc): the batch image goes into the library's fixed
    per-GPU array of SCRATCH_BYTES bytes.  Items and tuning as `Batch`.
    Calls that overlap on one GPU race on that array."""
    items = list(items)
    arr, keep = _batch_items(items)
    tune = _batch_tune(mode, tile_bytes, grid, wg_threads, xcd_order, split_k)
    _check(lib().pyrit_batch_run_noalloc(arr, len(items), ctypes.byref(tune),
                                         _stream_handle(stream)))
    del keep


SCRATCH_BYTES = 8 << 20  # PYRIT_SCRATCH_BYTES


class Batch:
    """Many stripes coded by one batch-kernel launch.

    ``items``: iterable of ``(plan, erased, blocks, S)`` or ``(plan, erased,
    blocks, S, pitch)``; ``erased`` empty for an encode; ``blocks`` holds
    k + m device buffers (entries that are neither inputs nor outputs may be
    None).  ``launch`` is the form `run` uses: ``"graph"`` replays the
    instantiated hipGraph (`launch`), ``"direct"`` dispatches the same kernel
    with the same arguments (`launch_direct`).
    """

    def __init__(self, items, mode: str = "grid", tile_bytes: int = 0, grid: int = 0,
                 wg_threads: int = 0, xcd_order: int = 0, split_k: int = 0,
                 launch: str = "graph"):
        if launch not in ("graph", "direct"):
            raise ValueError("launch must be 'graph' or 'direct'")
        self.launch_form = launch
        items = list(items)
        arr, self._keep = _batch_items(items)
        self.mode = mode
        tune = _batch_tune(mode, tile_bytes, grid, wg_threads, xcd_order, split_k)
        h = ctypes.c_void_p()
        _check(lib().pyrit_batch_create(arr, len(items), ctypes.byref(tune), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        _check(lib().pyrit_batch_launch(self._h, _stream_handle(stream)))

    def launch_direct(self, stream=None) -> None:
        _check(lib().pyrit_batch_launch_direct(self._h, _stream_handle(stream)))

    def run(self, stream=None) -> None:
        """Launch in the form chosen at construction."""
        if self.launch_form == "graph":
            self.launch(stream)
        else:
            self.launch_direct(stream)

    def info(self) -> dict:
        np_, ni, gr, wg = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        mv = ctypes.c_uint64()
        _check(lib().pyrit_batch_info(self._h, ctypes.byref(np_), ctypes.byref(ni),
                                      ctypes.byref(mv), ctypes.byref(gr), ctypes.byref(wg)))
        return {"passes": np_.value, "work_items": ni.value, "moved_bytes": mv.value,
                "grid": gr.value, "wg_threads": wg.value}

    def close(self):
        if getattr(self, "_h", None):
            lib().pyrit_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def fill_random(buf, key: int, nrandom: int | None = None, nbytes: int | None = None,
                stream=None) -> None:
    """Fill a device buffer with the seeded SplitMix64 byte stream."""
    if nbytes is None:
        nbytes = buf.numel() * buf.element_size()
    if nrandom is None:
        nrandom = nbytes
    _check(lib().pyrit_fill_random(_dev_ptr(buf, nbytes), nbytes, nrandom, key & ((1 << 64) - 1),
                                   _stream_handle(stream)))


def fill_random_blocks(bufs, keys, nrandom=None, stream=None) -> None:
    """Fill many device buffers with their seeded SplitMix64 streams in one
    kernel launch (pyrit_fill_random_blocks): buffer i gets key keys[i],
    random bytes up to nrandom[i] (None: the whole buffer), zeros beyond.
    Returns once the fill has completed."""
    bufs = list(bufs)
    n = len(bufs)
    if len(keys) != n or (nrandom is not None and len(nrandom) != n):
        raise ValueError("need one key (and one nrandom) per buffer")
    sizes = [b.numel() * b.element_size() for b in bufs]
    dst = (ctypes.c_void_p * max(1, n))(*[_dev_ptr(b, s) for b, s in zip(bufs, sizes)])
    nb = (ctypes.c_size_t * max(1, n))(*sizes)
    ks = (ctypes.c_uint64 * max(1, n))(*[k & ((1 << 64) - 1) for k in keys])
    nr = None if nrandom is None else (ctypes.c_size_t * max(1, n))(*nrandom)
    _check(lib().pyrit_fill_random_blocks(dst, nb, nr, ks, n, _stream_handle(stream)))


def copy(dst, src, nbytes: int | None = None, stream=None) -> None:
    if nbytes is None:
        nbytes = src.numel() * src.element_size()
    _check(lib().pyrit_copy(_dev_ptr(dst, nbytes), _dev_ptr(src, nbytes), nbytes,
                            _stream_handle(stream)))


def to_sliced(w: int, symbols, sliced, n_symbols: int | None = None, pitch: int = 0,
              stream=None) -> None:
    """Symbol-major block (one byte per symbol for w <= 8, one 16-bit word
    for larger w) -> bit-sliced block of w slices (see pyrit_to_sliced)."""
    if n_symbols is None:
        n_symbols = symbols.numel() * symbols.element_size() // (1 if w <= 8 else 2)
    sym_bytes = n_symbols * (1 if w <= 8 else 2)
    _check(lib().pyrit_to_sliced(w, _dev_ptr(symbols, sym_bytes), n_symbols,
                                 _dev_ptr(sliced, _block_bytes(w, n_symbols // 8, pitch)), pitch,
                                 _stream_handle(stream)))


def from_sliced(w: int, sliced, symbols, n_symbols: int | None = None, pitch: int = 0,
                stream=None) -> None:
    """Bit-sliced block -> symbol-major block (inverse of `to_sliced`)."""
    if n_symbols is None:
        n_symbols = symbols.numel() * symbols.element_size() // (1 if w <= 8 else 2)
    sym_bytes = n_symbols * (1 if w <= 8 else 2)
    _check(lib().pyrit_from_sliced(w, _dev_ptr(sliced, _block_bytes(w, n_symbols // 8, pitch)),
                                   pitch, n_symbols, _dev_ptr(symbols, sym_bytes),
                                   _stream_handle(stream)))
