"""Helpers shared by the GPU parity tests: device buffers filled with the
seeded generator, and oracle expectations on sampled columns."""
import numpy as np

import oracle
import paper_1709_00178_amd as P
from paper_1709_00178_amd import workloads as W


def torch_mod():
    import torch
    return torch


def dev_empty(nbytes):
    torch = torch_mod()
    return torch.empty(nbytes, dtype=torch.uint8, device="cuda")


def dev_block(st, block_id):
    """A device block holding the generator's bytes for block `block_id`."""
    t = dev_empty(st.block_len)
    P.fill_random(t, st.key(block_id), nrandom=st.nrandom)
    return t


def to_host(t):
    return t.cpu().numpy()


def gather_cols(buf, S, w, cols, pitch=None):
    """Mini block made of the given columns of every slice (w x len(cols));
    slice t starts at t * pitch (pitch defaults to S)."""
    pitch = S if pitch is None else pitch
    return np.ascontiguousarray(np.stack([buf[t * pitch + cols] for t in range(w)]).reshape(-1))


def gen_cols(st, block_id, cols):
    """Generator bytes of a block at the given columns of every slice."""
    offs = (np.arange(st.w)[:, None] * st.pitch + cols[None, :]).reshape(-1)
    return W.block_bytes_at(st.key(block_id), offs, st.nrandom)


def sample_cols(S, n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    extra = np.array([0, 1, 15, 16, 63, S - 64, S - 17, S - 16, S - 1])
    cols = np.unique(np.concatenate([rng.integers(0, S, n), extra]))
    return cols[(cols >= 0) & (cols < S)]


def oracle_cols(st, G, in_ids, cols, nthreads=4):
    """Oracle outputs (rows of G applied to the input blocks) at `cols`."""
    f = oracle.Field(st.w, st.p)
    ins = [gen_cols(st, j, cols) for j in in_ids]
    return f.encode(np.ascontiguousarray(G, dtype=np.uint16), ins, len(cols), nthreads=nthreads)


class Arena:
    """One device allocation carved into 256-byte aligned block buffers."""

    def __init__(self, nbytes):
        self.buf = dev_empty(nbytes)
        self.off = 0

    def take(self, nbytes):
        off = self.off
        self.off = off + (nbytes + 255) // 256 * 256
        assert self.off <= self.buf.numel(), "arena exhausted"
        return self.buf[off:off + nbytes]


def stripe_buffers(st, arena, fill=True):
    """Device blocks of one stripe: inputs filled with the generator, outputs
    allocated; returns (blocks list of k+m entries, input ids, output ids)."""
    ins = list(W.survivors(st))
    outs = list(st.erased) if st.erased else list(range(st.k, st.k + st.m))
    blocks = [None] * (st.k + st.m)
    for b in ins:
        blocks[b] = arena.take(st.block_len)
        if fill:
            P.fill_random(blocks[b], st.key(b), nrandom=st.nrandom)
    for b in outs:
        blocks[b] = arena.take(st.block_len)
    return blocks, ins, outs


def fill_inputs(stripes, bufs):
    """Fill the input blocks of many stripes (bufs from stripe_buffers with
    fill=False) with the generator in one launch."""
    dst, keys, nrand = [], [], []
    for st, (blocks, ins, _) in zip(stripes, bufs):
        for b in ins:
            dst.append(blocks[b])
            keys.append(st.key(b))
            nrand.append(st.nrandom)
    P.fill_random_blocks(dst, keys, nrand)


def stripe_bytes_needed(st):
    n_out = len(st.erased) if st.erased else st.m
    return (st.k + n_out) * ((st.block_len + 255) // 256 * 256)
