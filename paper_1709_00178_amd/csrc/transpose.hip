// Symbol-major <-> bit-sliced block layout, the steps either side of the
// coding path when data arrives as ordinary GF(2^w) symbols.
//
// Symbol s of a block (one byte for w <= 8, one little-endian 16-bit word for
// 8 < w <= 16) maps to bit s mod 8 of byte s div 8 of each slice: bit t of the
// symbol lives in slice t.  This is the bit-slice view the coding kernels and
// the oracle use (a block as w chunks, Sec. III).
//
// One lane handles 32 consecutive symbols: 8 of them fill one byte of every
// slice, so the lane writes (or reads) one 32-bit word per slice and the 64
// lanes of a wave cover 256 contiguous bytes of each slice.  The symbol side
// goes through LDS so that every vector access of a wave covers contiguous
// bytes (lane i moves 16 bytes at 16 i of each 1 KiB row) while each lane
// still works on its own 32 symbols.  The byte-to-slice reshuffle of 8
// symbols is an 8 x 8 bit-matrix transpose done with three masked delta swaps
// on a 64-bit word (an involution, so both directions use it).
#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace pyrit {
namespace {

constexpr int kTransposeWG = 256;

// Bit (r, c) of the 8 x 8 matrix whose row r is byte r of x moves to (c, r).
// The standard three-step delta-swap transpose of an 8 x 8 bit matrix held in
// one 64-bit word (H. S. Warren, "Hacker's Delight", 2nd ed., Sec. 7-3,
// transposing a bit matrix): swap 1 x 1, then 2 x 2, then 4 x 4 sub-blocks.
__device__ __forceinline__ uint64_t transpose8(uint64_t x) {
  uint64_t t;
  t = (x ^ (x >> 7)) & 0x00AA00AA00AA00AAull;
  x = x ^ t ^ (t << 7);
  t = (x ^ (x >> 14)) & 0x0000CCCC0000CCCCull;
  x = x ^ t ^ (t << 14);
  t = (x ^ (x >> 28)) & 0x00000000F0F0F0F0ull;
  x = x ^ t ^ (t << 28);
  return x;
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Byte select from the 8 bytes {hi, lo} (lo = bytes 0-3, hi = bytes 4-7):
// result byte i = byte (sel >> 8i) & 0xFF of them, 12 gives zero.
__device__ __forceinline__ uint32_t bsel(uint32_t hi, uint32_t lo, uint32_t sel) {
  return __builtin_amdgcn_perm(hi, lo, sel);
}
__device__ __forceinline__ uint32_t lo32(uint64_t x) { return (uint32_t)x; }
__device__ __forceinline__ uint32_t hi32(uint64_t x) { return (uint32_t)(x >> 32); }

// Byte b (0..7) of each of x0..x3, in that order: one 32-bit word.
__device__ __forceinline__ uint32_t gather_byte(uint64_t x0, uint64_t x1, uint64_t x2, uint64_t x3,
                                                int b) {
  const uint32_t sel = 0x0C0C0000u | ((4u + (b & 3)) << 8) | (uint32_t)(b & 3);
  const uint32_t p01 = b < 4 ? bsel(lo32(x1), lo32(x0), sel) : bsel(hi32(x1), hi32(x0), sel);
  const uint32_t p23 = b < 4 ? bsel(lo32(x3), lo32(x2), sel) : bsel(hi32(x3), hi32(x2), sel);
  return bsel(p23, p01, 0x05040100u);
}

// BYTES = bytes per symbol (1 or 2).  Lane g: symbols 32g .. 32g+31.  The
// lane count is a multiple of 16, so the last wave may be partial: 16-byte
// units owned by lanes past the end are neither loaded nor stored.
template <int BYTES>
__global__ __launch_bounds__(kTransposeWG) void to_sliced_kernel(const uint8_t *sym, uint8_t *out,
                                                                   uint32_t w, uint32_t pitch,
                                                                   uint32_t lanes) {
  __shared__ u32x4 stage[kTransposeWG / 64][2 * BYTES][64];
  const uint32_t g = blockIdx.x * kTransposeWG + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t g0 = g - lane;  // first lane of this wave
  // coalesced: row i of the wave's 32 * 64 * BYTES bytes is lane-contiguous
  const u32x4 *src = (const u32x4 *)(sym + (size_t)g0 * 32 * BYTES);
#pragma unroll
  for (int i = 0; i < 2 * BYTES; ++i) {
    const uint32_t e = i * 64 + lane;  // 16-byte unit of the wave's span
    if (g0 + e / (2 * BYTES) < lanes) stage[wv][e % (2 * BYTES)][e / (2 * BYTES)] = __builtin_nontemporal_load(src + e);
  }
  __syncthreads();
  if (g >= lanes) return;
  // 32 symbols = 32 * BYTES bytes as 64-bit words: word q holds symbols
  // 8q/BYTES ..; for BYTES = 2, byte 2i is the low half of symbol i.
  uint64_t v[4 * BYTES];
#pragma unroll
  for (int i = 0; i < 2 * BYTES; ++i) {
    const u32x4 x = stage[wv][i][lane];
    v[2 * i] = ((uint64_t)x.y << 32) | x.x;
    v[2 * i + 1] = ((uint64_t)x.w << 32) | x.z;
  }
  // lo[q], hi[q]: the low / high bytes of symbols 8q .. 8q+7, one per byte
  uint64_t lo[4], hi[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if constexpr (BYTES == 1) {
      lo[q] = transpose8(v[q]);
      hi[q] = 0;
    } else {
      // symbols 8q .. 8q+7 are words 2q and 2q+1: the even bytes of both
      // are the symbols' low bytes, the odd bytes their high bytes
      const uint64_t a = v[2 * q], b = v[2 * q + 1];
      const uint64_t l = ((uint64_t)bsel(hi32(b), lo32(b), 0x06040200u) << 32) |
                         bsel(hi32(a), lo32(a), 0x06040200u);
      const uint64_t h = ((uint64_t)bsel(hi32(b), lo32(b), 0x07050301u) << 32) |
                         bsel(hi32(a), lo32(a), 0x07050301u);
      lo[q] = transpose8(l);
      hi[q] = transpose8(h);
    }
  }
  // slice t word = byte t of lo[0..3] (or byte t-8 of hi[0..3])
  uint8_t *dst = out + (size_t)g * 4;
#pragma unroll
  for (int t = 0; t < 8 * BYTES; ++t) {
    if ((uint32_t)t >= w) break;
    const uint32_t word = t < 8 ? gather_byte(lo[0], lo[1], lo[2], lo[3], t)
                                : gather_byte(hi[0], hi[1], hi[2], hi[3], t - 8);
    *(uint32_t *)(dst + (size_t)t * pitch) = word;
  }
}

template <int BYTES>
__global__ __launch_bounds__(kTransposeWG) void from_sliced_kernel(const uint8_t *in, uint8_t *sym,
                                                                     uint32_t w, uint32_t pitch,
                                                                     uint32_t lanes) {
  __shared__ u32x4 stage[kTransposeWG / 64][2 * BYTES][64];
  const uint32_t g = blockIdx.x * kTransposeWG + threadIdx.x;
  const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
  const uint32_t g0 = g - lane;
  const bool live = g < lanes;
  uint64_t lo[4] = {0, 0, 0, 0}, hi[4] = {0, 0, 0, 0};
  const uint8_t *src = in + (size_t)g * 4;
  // all slice words in flight before any is used
  uint32_t words[8 * BYTES];
#pragma unroll
  for (int t = 0; t < 8 * BYTES; ++t)
    words[t] = (live && (uint32_t)t < w)
                   ? __builtin_nontemporal_load((const uint32_t *)(src + (size_t)t * pitch))
                   : 0u;
  // byte t of lo[q] (hi[q]) = byte q of slice word t (t + 8)
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t sel = 0x0C0C0000u | ((4u + q) << 8) | (uint32_t)q;
    const uint32_t l0 = bsel(bsel(words[3], words[2], sel), bsel(words[1], words[0], sel), 0x05040100u);
    const uint32_t l1 = bsel(bsel(words[7], words[6], sel), bsel(words[5], words[4], sel), 0x05040100u);
    lo[q] = ((uint64_t)l1 << 32) | l0;
    if constexpr (BYTES == 2) {
      const uint32_t h0 = bsel(bsel(words[11], words[10], sel), bsel(words[9], words[8], sel), 0x05040100u);
      const uint32_t h1 = bsel(bsel(words[15], words[14], sel), bsel(words[13], words[12], sel), 0x05040100u);
      hi[q] = ((uint64_t)h1 << 32) | h0;
    }
  }
  uint64_t v[4 * BYTES];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint64_t l = transpose8(lo[q]);
    if constexpr (BYTES == 1) {
      v[q] = l;
    } else {
      const uint64_t h = transpose8(hi[q]);
      // interleave: symbol i = low byte i of l, high byte i of h
      v[2 * q] = ((uint64_t)bsel(lo32(h), lo32(l), 0x07030602u) << 32) |
                 bsel(lo32(h), lo32(l), 0x05010400u);
      v[2 * q + 1] = ((uint64_t)bsel(hi32(h), hi32(l), 0x07030602u) << 32) |
                     bsel(hi32(h), hi32(l), 0x05010400u);
    }
  }
#pragma unroll
  for (int i = 0; i < 2 * BYTES; ++i) {
    u32x4 x;
    x.x = (uint32_t)v[2 * i];
    x.y = (uint32_t)(v[2 * i] >> 32);
    x.z = (uint32_t)v[2 * i + 1];
    x.w = (uint32_t)(v[2 * i + 1] >> 32);
    stage[wv][i][lane] = x;
  }
  __syncthreads();
  // coalesced: 16-byte unit e of the wave's span belongs to lane e / (2 BYTES).
  // Each unit is stored as two 8-byte stores, never one 16-byte store: a
  // store wider than 64 bits reads its data registers after it issues, and
  // generated code has been seen to overwrite them in the very next
  // instruction (here an LDS read of the next unit would be one), corrupting
  // stored bytes now and then.  The empty asm keeps the halves apart.
  uint64_t *dst = (uint64_t *)(sym + (size_t)g0 * 32 * BYTES);
#pragma unroll
  for (int i = 0; i < 2 * BYTES; ++i) {
    const uint32_t e = i * 64 + lane;
    if (g0 + e / (2 * BYTES) < lanes) {
      const u32x4 x = stage[wv][e % (2 * BYTES)][e / (2 * BYTES)];
      dst[2 * e] = ((uint64_t)x.y << 32) | x.x;
      __asm__ volatile("" ::: "memory");
      dst[2 * e + 1] = ((uint64_t)x.w << 32) | x.z;
    }
  }
}

int check_transpose(int w, const void *a, const void *b, size_t n_symbols, size_t *pitch) {
  if (w < 1 || w > 16 || !a || !b) return PYRIT_EINVAL;
  if (n_symbols == 0 || n_symbols % 512 != 0 || n_symbols / 32 > 0xFFFFFFFFull) return PYRIT_EINVAL;
  if (((uintptr_t)a & 15u) || ((uintptr_t)b & 15u)) return PYRIT_EALIGN;
  return check_slices(w, n_symbols / 8, pitch);
}

}  // namespace
}  // namespace pyrit

using namespace pyrit;

extern "C" {

int pyrit_to_sliced(int w, const void *symbols, size_t n_symbols, uint8_t *sliced, size_t slice_pitch,
                    void *stream) {
  int rc = check_transpose(w, symbols, sliced, n_symbols, &slice_pitch);
  if (rc) return rc;
  const uint32_t lanes = (uint32_t)(n_symbols / 32);
  const dim3 grid((lanes + kTransposeWG - 1) / kTransposeWG);
  if (w <= 8)
    hipLaunchKernelGGL(to_sliced_kernel<1>, grid, dim3(kTransposeWG), 0, (hipStream_t)stream,
                       (const uint8_t *)symbols, sliced, (uint32_t)w, (uint32_t)slice_pitch, lanes);
  else
    hipLaunchKernelGGL(to_sliced_kernel<2>, grid, dim3(kTransposeWG), 0, (hipStream_t)stream,
                       (const uint8_t *)symbols, sliced, (uint32_t)w, (uint32_t)slice_pitch, lanes);
  return hipGetLastError() == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

int pyrit_from_sliced(int w, const uint8_t *sliced, size_t slice_pitch, size_t n_symbols, void *symbols,
                      void *stream) {
  int rc = check_transpose(w, sliced, symbols, n_symbols, &slice_pitch);
  if (rc) return rc;
  const uint32_t lanes = (uint32_t)(n_symbols / 32);
  const dim3 grid((lanes + kTransposeWG - 1) / kTransposeWG);
  if (w <= 8)
    hipLaunchKernelGGL(from_sliced_kernel<1>, grid, dim3(kTransposeWG), 0, (hipStream_t)stream,
                       sliced, (uint8_t *)symbols, (uint32_t)w, (uint32_t)slice_pitch, lanes);
  else
    hipLaunchKernelGGL(from_sliced_kernel<2>, grid, dim3(kTransposeWG), 0, (hipStream_t)stream,
                       sliced, (uint8_t *)symbols, (uint32_t)w, (uint32_t)slice_pitch, lanes);
  return hipGetLastError() == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

}  // extern "C"
