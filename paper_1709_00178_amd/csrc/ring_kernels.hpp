// Device side of one coding pass, for gfx950 (CDNA4, wave64).
//
// Each lane owns a column of 4*V bytes (V dwords) at byte offset `col` of
// every slice.  For one output block r the lane keeps the n ring slices of
// its column in registers (acc[r][0..n-1]).  Input block j contributes, for
// every exponent s set in the lifted coefficient c[r][j] (Sec. II-B), its w
// slices rotated by s: acc[r][(t + s) mod n] ^= slice t (multiplying by x^s
// in R_{2,n}).  The embedding transform pads a block with n - w zero slices
// (Sec. II-C.2), so those slices are never loaded.  After the last input,
// ring slices w..n-1 are folded into the field slices through x^i mod p
// (inverse embedding, Prop. 2) and the w field slices are stored.
//
// The set bits of a lifted coefficient are wave-uniform (scalar registers),
// so each rotation is a scalar branch around an unrolled body whose
// accumulator indices are compile-time constants: the accumulators never
// leave registers and no schedule is read per XOR (the GPU form of the
// paper's unrolled, schedule-free XOR code of Sec. III).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rings.hpp"

namespace pyrit {
namespace dev {

typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// The lifted coefficients of one input block for up to eight outputs.
struct Lift8 {
  u32x4 lo, hi;
  __device__ __forceinline__ uint32_t operator[](int r) const { return r < 4 ? lo[r] : hi[r - 4]; }
};

template <int V> struct Vec;
template <> struct Vec<1> { typedef uint32_t T; };
template <> struct Vec<2> { typedef u32x2 T; };
template <> struct Vec<4> { typedef u32x4 T; };

// Raw-buffer descriptor word 3 for gfx9-family parts (32-bit data format).
constexpr int kBufDword3 = 0x00020000;
// Cache policy bits of buffer instructions on gfx94x/gfx950: bit 0 = SC0,
// bit 1 = NT, bit 4 = SC1.  Inputs are read once: non-temporal loads.
// Outputs are stored with SC1 set and NT clear: on MI355X a 10-read/4-write
// stream measured 6.3 TB/s this way against 5.5 TB/s with NT stores.
constexpr int kLoadPolicy = 2;
constexpr int kStorePolicy = 16;

// x^i mod p for p of degree w, as a compile-time constant.
constexpr uint32_t xpow_mod(int i, uint32_t p, int w) {
  uint32_t v = 1;
  for (int e = 0; e < i; ++e) {
    v <<= 1;
    if (v >> w & 1u) v ^= p;
  }
  return v;
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t block_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes,
                                           kBufDword3);
}

template <int V>
__device__ __forceinline__ typename Vec<V>::T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                    uint32_t soff) {
  if constexpr (V == 1)
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, kLoadPolicy);
  else if constexpr (V == 2)
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, kLoadPolicy);
  else
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, kLoadPolicy);
}

template <int V>
__device__ __forceinline__ void bstore(typename Vec<V>::T x, __amdgpu_buffer_rsrc_t r,
                                       uint32_t voff, uint32_t soff) {
  if constexpr (V == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(x, r, voff, soff, kStorePolicy);
  } else if constexpr (V == 2) {
    __builtin_amdgcn_raw_buffer_store_b64(x, r, voff, soff, kStorePolicy);
  } else {
    // Two 8-byte stores, not one 16-byte store: a store of more than 64 bits
    // reads its data registers after issue, and the compiler has been seen
    // to let the next instruction overwrite them with no wait state between
    // (a VALU write right after buffer_store_dwordx4, on gfx950), which
    // corrupts the stored data now and then.
    // (The empty asm keeps the two halves from being merged back into one
    // 16-byte store.)
    const u32x2 lo = {x.x, x.y}, hi = {x.z, x.w};
    __builtin_amdgcn_raw_buffer_store_b64(lo, r, voff, soff, kStorePolicy);
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_raw_buffer_store_b64(hi, r, voff + 8u, soff, kStorePolicy);
  }
}

// ---- parity transform (Sec. II-C.1, II-D.1), all at compile time --------
// Carry-less product and remainder of small polynomials (bit i = x^i).
constexpr uint32_t cl_mul(uint32_t a, uint32_t b) {
  uint32_t r = 0;
  for (int i = 0; i < 32; ++i)
    if (b >> i & 1u) r ^= a << i;
  return r;
}
constexpr int cl_deg(uint32_t a) {
  int d = -1;
  for (int i = 0; i < 32; ++i)
    if (a >> i & 1u) d = i;
  return d;
}
constexpr uint32_t cl_mod(uint32_t a, uint32_t m) {
  const int dm = cl_deg(m);
  for (int d = cl_deg(a); d >= dm; d = cl_deg(a)) a ^= m << (d - dm);
  return a;
}
// h = (x^N + 1) / P: the ideal of multiples of h is the copy of the field
// inside R_{2,N} (the AOP case: h = x + 1, the ESP x^6+x^3+1: h = x^3 + 1).
constexpr uint32_t ideal_gen(int N, uint32_t P) {
  uint32_t a = (1u << N) | 1u, q = 0;
  const int dp = cl_deg(P);
  for (int d = cl_deg(a); d >= dp; d = cl_deg(a)) {
    q |= 1u << (d - dp);
    a ^= P << (d - dp);
  }
  return q;
}
// The parity transform sends b (deg < W) to b + x^W q with q = b x^-W mod h,
// the one element of the ideal whose low W coefficients are b.  Bit i of
// pt_mask(t) is set when coefficient i of b feeds coefficient t (W <= t < N).
constexpr uint32_t pt_mask(int t, int W, int N, uint32_t P) {
  const uint32_t h = ideal_gen(N, P);
  const uint32_t xw = cl_mod(1u << W, h);
  uint32_t y = 1;
  for (uint32_t c = 1; c < (1u << (N - W)); ++c)
    if (cl_mod(cl_mul(c, xw), h) == 1u) y = c;
  uint32_t mask = 0;
  for (int i = 0; i < W; ++i)
    if (cl_mod(cl_mul(1u << i, y), h) >> (t - W) & 1u) mask |= 1u << i;
  return mask;
}

template <int W, int N, uint32_t P>
struct PtMasks {
  uint32_t m[N > W ? N : 1];
  constexpr PtMasks() : m() {
    for (int t = W; t < N; ++t) m[t] = pt_mask(t, W, N, P);
  }
};

// Embedded block of the parity transform: the W loaded slices, then the
// N - W parity slices built from them.
template <int W, int N, uint32_t P, typename T>
__device__ __forceinline__ void parity_embed(T (&e)[N], const T (&d)[W]) {
  constexpr PtMasks<W, N, P> M{};
#pragma unroll
  for (int t = 0; t < W; ++t) e[t] = d[t];
#pragma unroll
  for (int t = W; t < N; ++t) {
    T x = (T)0;
#pragma unroll
    for (int i = 0; i < W; ++i)
      if (M.m[t] >> i & 1u) x ^= d[i];
    e[t] = x;
  }
}

// acc[(t + s) mod N] ^= d[t] for t < W and every s >= S0 set in c.
template <int W, int N, int S0, typename T>
__device__ __forceinline__ void rot_acc(T (&acc)[N], const T (&d)[W], uint32_t c) {
  if constexpr (S0 < N) {
    if (c & (1u << S0)) {
#pragma unroll
      for (int t = 0; t < W; ++t) acc[(t + S0) % N] ^= d[t];
    }
    rot_acc<W, N, S0 + 1, T>(acc, d, c);
  }
}

// Fold ring slices W..N-1 into the field slices: slice i adds itself to
// every field slice b with bit b of x^i mod p set.
template <int W, int N, uint32_t P, typename T>
__device__ __forceinline__ void reduce_mod_p(T (&acc)[N]) {
#pragma unroll
  for (int i = W; i < N; ++i) {
    const uint32_t red = xpow_mod(i, P, W);
#pragma unroll
    for (int b = 0; b < W; ++b)
      if (red >> b & 1u) acc[b] ^= acc[i];
  }
}

// One input block into the ring accumulators of MO outputs: embedding
// transform (the block as is, zero slices implied) or parity transform (the
// block extended by its parity slices).
template <int W, int N, uint32_t P, int MO, bool PT, typename T>
__device__ __forceinline__ void accumulate(T (&acc)[MO][N], const T (&d)[W], const Lift8 &cf) {
  if constexpr (PT) {
    T e[N];
    parity_embed<W, N, P, T>(e, d);
#pragma unroll
    for (int r = 0; r < MO; ++r) rot_acc<N, N, 0, T>(acc[r], e, cf[r]);
  } else {
#pragma unroll
    for (int r = 0; r < MO; ++r) rot_acc<W, N, 0, T>(acc[r], d, cf[r]);
  }
}

// Ring slices back to field slices: reduction modulo p (embedding transform)
// or nothing, the high slices being dropped (parity transform).
template <int W, int N, uint32_t P, bool PT, typename T>
__device__ __forceinline__ void leave_ring(T (&acc)[N]) {
  if constexpr (!PT) reduce_mod_p<W, N, P, T>(acc);
}

// Load the W slices of one block at this lane's voffset (its column, or
// kDeadOffset for a lane past the end of the slice).  bytes == 0 gives an
// empty descriptor: every load is out of range and returns zero without any
// memory traffic (used for prefetches past the last block).
template <int W, int V>
__device__ __forceinline__ void load_block(typename Vec<V>::T (&d)[W], const uint8_t *base,
                                           uint32_t bytes, uint32_t pitch, uint32_t voff) {
  const __amdgpu_buffer_rsrc_t r = block_rsrc(base, bytes);
#pragma unroll
  for (int t = 0; t < W; ++t) d[t] = bload<V>(r, voff, t * pitch);
}

// One lane column of one pass.  Src supplies wave-uniform values:
//   k(), S(), pitch(), nout(), in(j), out(r), lift(j, r) and lift8(j) (the
//   kMaxOut lifted coefficients of input j, two 16-byte loads); slice t of a block
//   starts t * pitch() bytes after its base.  Rows r >= nout() must have
//   zero lifted coefficients; they are neither reduced nor stored.
//
// KS = 1: the wave codes every input block of its column chunk.
// KS = 2 (split-K): a pair of waves of one workgroup shares one column
// chunk.  Wave `part` codes input blocks part, part + 2, ...; each reduces
// its partial sums mod p (reduction is linear), wave part keeps outputs
// r = part, part + 2, ... and hands the other outputs' partial slices to the
// other wave through LDS (`xch`: MO x W x 64 lane values, one writer each;
// the workgroup's one barrier sits between the writes and the reads).
// Half as many columns are in flight for the same number of waves, which
// shrinks the set of HBM rows open at once (measured on MI355X: 6.6 -> 7.0
// TB/s for the 10-in/4-out, 8-slice access pattern).
template <int W, int N, uint32_t P, int MO, int V, int KS = 1, bool PT = false, class Src>
__device__ __forceinline__ void code_column(const Src &src, uint32_t col, bool live,
                                            uint32_t part = 0,
                                            typename Vec<V>::T *xch = nullptr) {
  static_assert(KS == 1 || KS == 2, "split factor");
  typedef typename Vec<V>::T T;
  const int k = src.k();
  const uint32_t S = src.S();
  const uint32_t pitch = src.pitch();    // slice stride (>= S)
  const uint32_t span = block_span(W, S, pitch);  // bytes of a block holding slices
  const uint32_t voff = lane_load_voffset(col, S);  // dead lanes load nothing
  T acc[MO][N];
#pragma unroll
  for (int r = 0; r < MO; ++r)
#pragma unroll
    for (int i = 0; i < N; ++i) acc[r][i] = (T)0;

  // Two register sets: the wave's next block is in flight while the current
  // one is accumulated.  The prefetch after the last block uses an empty
  // descriptor.  (Deeper register prefetch measured no faster on MI355X: it
  // costs occupancy.)
  T d[2][W];
  auto clampj = [&](int jj) { return jj < k ? jj : k - 1; };
  auto prefetch = [&](int slot, int jj, const uint8_t *base) {
    load_block<W, V>(d[slot], base, jj < k ? span : 0u, pitch, voff);
  };
  // Scalar operands run ahead of their use: the block pointer one prefetch
  // ahead and the lifted coefficients one block ahead (one 16-byte scalar
  // load), so no scalar-load wait sits between the vector loads and XORs.
  prefetch(0, (int)part, src.in(clampj((int)part)));
  const uint8_t *ip = src.in(clampj((int)part + KS));
  Lift8 cf = src.lift8(clampj((int)part));
  for (int j = (int)part; j < k; j += 2 * KS) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int jq = j + q * KS;
      if (jq >= k) break;
      prefetch(q ^ 1, jq + KS, ip);
      ip = src.in(clampj(jq + 2 * KS));
      const Lift8 cn = src.lift8(clampj(jq + KS));
      accumulate<W, N, P, MO, PT, T>(acc, d[q], cf);
      cf = cn;
    }
  }

  if constexpr (KS == 1) {
    if (!live) return;
#pragma unroll
    for (int r = 0; r < MO; ++r) {
      if (r >= src.nout()) break;
      leave_ring<W, N, P, PT, T>(acc[r]);
      const __amdgpu_buffer_rsrc_t o = block_rsrc(src.out(r), span);
#pragma unroll
      for (int t = 0; t < W; ++t) bstore<V>(acc[r][t], o, col, t * pitch);
    }
  } else {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int r = 0; r < MO; ++r) {
      if (r >= src.nout()) break;
      leave_ring<W, N, P, PT, T>(acc[r]);
      if ((uint32_t)(r & 1) != part) {
#pragma unroll
        for (int t = 0; t < W; ++t) xch[(r * W + t) * 64 + lane] = acc[r][t];
      }
    }
    __syncthreads();
    if (!live) return;
#pragma unroll
    for (int r = 0; r < MO; ++r) {
      if (r >= src.nout()) break;
      if ((uint32_t)(r & 1) != part) continue;
      const __amdgpu_buffer_rsrc_t o = block_rsrc(src.out(r), span);
#pragma unroll
      for (int t = 0; t < W; ++t) bstore<V>(acc[r][t] ^ xch[(r * W + t) * 64 + lane], o, col, t * pitch);
    }
  }
}

// A run of consecutive chunks [col0, col1) of one pass, coded by one wave
// (chunk = 64 lanes x 4V bytes).  The block loads form one continuous
// stream: while chunk c's last block is accumulated, chunk c+1's first block
// is already in flight, so the wave never drains its load pipeline between
// chunks.
template <int W, int N, uint32_t P, int MO, int V, bool PT = false, class Src>
__device__ __forceinline__ void code_tile(const Src &src, uint32_t col0, uint32_t col1,
                                          uint32_t lane) {
  typedef typename Vec<V>::T T;
  constexpr uint32_t kChunk = 64u * 4u * V;
  const int k = src.k();
  const uint32_t S = src.S();
  const uint32_t pitch = src.pitch();    // slice stride (>= S)
  const uint32_t span = block_span(W, S, pitch);  // bytes of a block holding slices
  T acc[MO][N];
#pragma unroll
  for (int r = 0; r < MO; ++r)
#pragma unroll
    for (int i = 0; i < N; ++i) acc[r][i] = (T)0;

  T d[2][W];
  // prefetch of (chunk base cb, block jj); cb >= col1 means past the end
  // (empty descriptor), and lanes past the end of the slice load nothing
  auto prefetch = [&](int slot, uint32_t cb, int jj) {
    const bool ok = cb < col1;
    load_block<W, V>(d[slot], src.in(ok ? jj : 0), ok ? span : 0u, pitch,
                     lane_load_voffset(lane_col(cb, lane, V), S));
  };
  uint32_t cb = col0;  // chunk being accumulated
  int j = 0;           // block being accumulated
  prefetch(0, cb, 0);
  while (cb < col1) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      // next step: block j+1 of this chunk, or block 0 of the next chunk
      const bool last = j + 1 == k;
      prefetch(q ^ 1, last ? cb + kChunk : cb, last ? 0 : j + 1);
      accumulate<W, N, P, MO, PT, T>(acc, d[q], src.lift8(j));
      if (last) {
        const uint32_t col = lane_col(cb, lane, V);
        if (col < S) {
#pragma unroll
          for (int r = 0; r < MO; ++r) {
            if (r >= src.nout()) break;
            leave_ring<W, N, P, PT, T>(acc[r]);
            const __amdgpu_buffer_rsrc_t o = block_rsrc(src.out(r), span);
#pragma unroll
            for (int t = 0; t < W; ++t) bstore<V>(acc[r][t], o, col, t * pitch);
          }
        }
#pragma unroll
        for (int r = 0; r < MO; ++r)
#pragma unroll
          for (int i = 0; i < N; ++i) acc[r][i] = (T)0;
        cb += kChunk;
        j = 0;
        if (cb >= col1) break;
      } else {
        ++j;
      }
    }
  }
}

// Source of pass arguments held in the kernel-argument segment.
struct KernargSrc {
  const PassArgs &a;
  __device__ int k() const { return (int)a.k; }
  __device__ uint32_t S() const { return a.S; }
  __device__ uint32_t pitch() const { return a.pitch; }
  __device__ int nout() const { return kMaxOut; }
  __device__ const uint8_t *in(int j) const { return a.in[j]; }
  __device__ uint8_t *out(int r) const { return a.out[r]; }
  __device__ uint32_t lift(int j, int r) const { return a.lift[j][r]; }
  __device__ Lift8 lift8(int j) const {
    return Lift8{*(const u32x4 *)&a.lift[j][0], *(const u32x4 *)&a.lift[j][4]};
  }
};

}  // namespace dev
}  // namespace pyrit
