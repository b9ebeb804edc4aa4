// The rings with device kernels and the argument block of one coding pass:
// everything the kernels are compiled from besides their own sources.
#pragma once
#include <stdint.h>

#include "../../include/pyrit.h"

namespace pyrit {

// Outputs computed by one kernel pass: the accumulators of every output live
// in registers, so a pass covers at most this many output blocks (the bound
// of every per-pass array; each ring has its own limit, ring_max_out).
constexpr int kMaxOut = 8;

// Rings with a device kernel.  The kernels are templates on (w, n, p), so the
// reduction modulo p and every rotation index are compile-time constants.
// `parity` selects the parity transform (Sec. II-C.1, II-D.1) in place of the
// embedding transform (Sec. II-C.2, II-D.2): data enter the ring with n - w
// parity slices instead of zero slices, and results leave it by dropping
// those slices instead of reducing modulo p.
struct RingDesc {
  int w, n;
  uint32_t p;
  bool parity;
};
constexpr int kNumRings = 8;
constexpr RingDesc kRings[kNumRings] = {
    {4, 5, 0x1Fu, false},     // all-one polynomial of degree 4 (Sec. II-C)
    {8, 17, 0x139u, false},   // x^8+x^5+x^4+x^3+1, divides x^17+1
    {8, 17, 0x1D7u, false},   // x^8+x^7+x^6+x^4+x^2+x+1, the other factor
    {10, 11, 0x7FFu, false},  // all-one polynomial of degree 10
    {6, 9, 0x49u, false},     // equally spaced x^6+x^3+1 (Sec. II-D)
    {4, 5, 0x1Fu, true},      // the AOP and ESP rings again, parity transform
    {10, 11, 0x7FFu, true},
    {6, 9, 0x49u, true},
};
// Outputs per pass of a ring: outputs x n ring slices of accumulators stay
// near 70 registers per lane (4 for n = 17, 6 for n = 11, 8 for n <= 9).
constexpr int ring_max_out(int ring) {
  return kRings[ring].n <= 9 ? 8 : kRings[ring].n <= 11 ? 6 : 4;
}

// Rings whose kernels take each coefficient as its field element u rather
// than its lifted ring element: the kernel branches on the w bits of u to a
// body compiled for lift(u) (2^w bodies per output, so only for small
// fields), in which the terms that land on one accumulator are summed two
// at a time by three-input XORs.  Other rings take the lifted element c and
// branch on its n bits, one rotation per set bit.
constexpr bool ring_fused(int ring) { return kRings[ring].n <= 9; }

// ---- how a lane addresses a block (kernels and host-side checks share it)
// A block's w slices start at base + t * pitch (t < w); the block spans
// (w - 1) * pitch + S bytes.  A lane reads the 4V bytes of its column `col`
// of slice t through a raw buffer descriptor of `span` records, with
// voffset = col and soffset = t * pitch.  Lanes whose column lies at or past
// S code nothing (the last chunk of a slice is often partial); their loads
// take the voffset kDeadOffset instead.  It exceeds every record count
// (spans stay below 2^31), so those loads return zero without touching
// memory whether or not the hardware adds soffset before its range check,
// and kDeadOffset + soffset still fits in 32 bits.
constexpr uint32_t kDeadOffset = 0x80000000u;
constexpr uint32_t block_span(uint32_t w, uint32_t S, uint32_t pitch) {
  return (w - 1) * pitch + S;
}
constexpr uint32_t lane_load_voffset(uint32_t col, uint32_t S) {
  return col < S ? col : kDeadOffset;
}
// Column of lane `lane` (lanes of V dwords) in the chunk of 64 lanes that
// starts at chunk_base.
constexpr uint32_t lane_col(uint32_t chunk_base, uint32_t lane, uint32_t V) {
  return chunk_base + lane * 4u * V;
}
// Plain kernel: workgroup b codes the chunk at b * 256 V bytes.
constexpr uint32_t plain_chunk_base(uint32_t b, uint32_t V) { return b * 64u * 4u * V; }
// Batch grid kernel: the i-th workgroup of a pass holds `pairs` chunks (one
// per wave, or per split-K pair of waves); wave `wave` codes chunk
// i * pairs + wave / ks.
constexpr uint32_t grid_chunk_base(uint32_t i, uint32_t wave, uint32_t pairs, uint32_t ks,
                                   uint32_t chunk) {
  return (i * pairs + wave / ks) * chunk;
}

// Arguments of one coding pass: outputs out[r] (r < nout) are
// sum_j coef[j][r] (*) in[j] in the ring, reduced mod p.  A coefficient word
// is the field element (rings with ring_fused) or its lifted ring element.
struct PassArgs {
  const uint8_t *in[PYRIT_KMAX];
  uint8_t *out[kMaxOut];
  uint32_t lift[PYRIT_KMAX][kMaxOut];  // coefficient words
  uint32_t k;
  uint32_t S;      // column bytes per slice
  uint32_t pitch;  // bytes from one slice to the next (>= S)
};

}  // namespace pyrit

namespace pyrit {

// ---- wide passes: codes with more outputs than one pass holds ----------
// One launch codes G output groups of up to wide_max_out outputs each; the
// G waves of a workgroup share one column chunk of 64 lanes x 4 bytes,
// wave g coding group g, and each input block is fetched from HBM once per
// launch into LDS, where every wave reads it.  Everything travels in the
// kernel-argument segment, packed into kWideWords 8-byte words:
//   word 0: k | S << 32;  word 1: pitch | groups << 32;
//   words 2, 3: the number of outputs of group g (1..15) in bits 4g..4g+3
//     of the 128-bit value word 2 | word 3 << 64;
//   words 4..4+k: input pointers;
//   then G x wide_max_out output pointers (group g's at g * wide_max_out);
//   then G x k records of wide_rec_words words, (g, j) at (g * k + j): the
//   coefficient words of input j for group g's outputs, as 16-bit words
//   (n <= 16) or 32-bit words (n = 17).
constexpr int kWideWords = 500;         // 4000 bytes of kernel arguments
constexpr int kWideMaxGroups = 16;      // waves per workgroup
constexpr int kWideV = 1;               // dwords per lane
struct WideArgs {
  uint64_t w[kWideWords];
};
constexpr int wide_header_words() { return 4; }
// Outputs per wave (output group) of a wide launch, with lanes of 4 bytes.
// On the ring (6,9), five: the embedding transform keeps all nine ring
// slices of an output until the reduction, and five outputs (45
// accumulators) fit eight waves per SIMD with no register spill, where six
// (54) spilled and eight (72) allowed five waves; the parity transform
// keeps six slices per output.  Groups of five also split the paper's
// (60,40) and (60,20) shapes (20 and 40 parity blocks) evenly, so no wave
// dispatches on padding coefficients.  Against six (embedding) and eight
// (parity) outputs per wave this ran those codes 5-20% faster; four per
// wave ran 10-25% slower (more waves, each reading every input block from
// LDS).  8-byte lanes, which halve the scalar dispatch work per byte,
// measured slower at every group size tried.
constexpr int wide_max_out(int ring) {
  return kRings[ring].n == 9 ? 5 : ring_max_out(ring);
}
// Record words per (group, input): 16-bit coefficient words, four per word
// (n <= 16), or 32-bit ones, two per word (n = 17).
constexpr int wide_rec_words(int ring) {
  return kRings[ring].n <= 16 ? (wide_max_out(ring) + 3) / 4 : (wide_max_out(ring) + 1) / 2;
}
// Blocks staged in LDS per workgroup of a wide pass (D stages of w slices x
// 256 bytes, D a power of two: 8 KiB to 12 KiB).
constexpr int wide_stages(int ring) { return kRings[ring].w <= 6 ? 8 : 4; }
// Blocks coded between two barriers of a wide pass: two where eight stages
// leave room to prefetch six blocks ahead (half the barriers, and waves
// whose coefficients cost more on one block catch up on the next: 2-9%
// faster on the (60,40) and (60,20) codes than one block per barrier; four
// per barrier, or two with sixteen stages, ran slower), else one.
constexpr int wide_blocks_per_barrier(int ring) { return wide_stages(ring) >= 8 ? 2 : 1; }
// Output groups that fit one launch of a k-input code on `ring`.
constexpr int wide_groups_fit(int ring, int k) {
  const int per_group = wide_max_out(ring) + wide_rec_words(ring) * k;
  // (two words stay free after the last record: the kernel reads one record
  // past each group's last)
  const int g = (kWideWords - 2 - wide_header_words() - k) / per_group;
  return g < kWideMaxGroups ? g : kWideMaxGroups;
}

}  // namespace pyrit
