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

#include <type_traits>

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

// f(std::integral_constant<int, I>) for I = B, B+1, ..., E-1: a loop whose
// index is a compile-time constant in the body without relying on the loop
// unroller (which gives up on bodies as large as the fused rotations, and
// would then leave register arrays indexed at run time, i.e. in scratch).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

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

template <int V, int LP = kLoadPolicy>
__device__ __forceinline__ typename Vec<V>::T bload(__amdgpu_buffer_rsrc_t r, uint32_t voff,
                                                    uint32_t soff) {
  if constexpr (V == 1)
    return __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, LP);
  else if constexpr (V == 2)
    return __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, LP);
  else
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, LP);
}

template <int V, int SP = kStorePolicy>
__device__ __forceinline__ void bstore(typename Vec<V>::T x, __amdgpu_buffer_rsrc_t r,
                                       uint32_t voff, uint32_t soff) {
  if constexpr (V == 1) {
    __builtin_amdgcn_raw_buffer_store_b32(x, r, voff, soff, SP);
  } else if constexpr (V == 2) {
    __builtin_amdgcn_raw_buffer_store_b64(x, r, voff, soff, SP);
  } else {
    // Two 8-byte stores, not one 16-byte store: a store of more than 64 bits
    // reads its data registers after issue, and the compiler has been seen
    // to let the next instruction overwrite them with no wait state between
    // (a VALU write right after buffer_store_dwordx4, on gfx950), which
    // corrupts the stored data now and then.
    // (The empty asm keeps the two halves from being merged back into one
    // 16-byte store.)
    const u32x2 lo = {x.x, x.y}, hi = {x.z, x.w};
    __builtin_amdgcn_raw_buffer_store_b64(lo, r, voff, soff, SP);
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_raw_buffer_store_b64(hi, r, voff + 8u, soff, SP);
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

// ---- fused rotations for the small fields (rings with ring_fused) -------
// Three-input XOR: gfx950's v_bitop3_b32 with truth table 0x96 (the output
// bit is set where an odd number of the three inputs is set).
__device__ __forceinline__ uint32_t xor3(uint32_t a, uint32_t b, uint32_t c) {
  return __builtin_amdgcn_bitop3_b32(a, b, c, 0x96);
}
__device__ __forceinline__ u32x2 xor3(u32x2 a, u32x2 b, u32x2 c) {
  return u32x2{xor3(a.x, b.x, c.x), xor3(a.y, b.y, c.y)};
}
__device__ __forceinline__ u32x4 xor3(u32x4 a, u32x4 b, u32x4 c) {
  return u32x4{xor3(a.x, b.x, c.x), xor3(a.y, b.y, c.y), xor3(a.z, b.z, c.z),
               xor3(a.w, b.w, c.w)};
}

constexpr int popc(uint32_t x) {
  int c = 0;
  for (; x; x >>= 1) c += (int)(x & 1u);
  return c;
}
// Sparse transform (Sec. II-B) at compile time: among the ring elements
// u + t p (deg t < N - W), the one of fewest nonzero coefficients, ties
// going to the smallest integer (the host plan's rule).
constexpr uint32_t lift_const(uint32_t u, int W, int N, uint32_t P) {
  uint32_t best = u;
  int bw = popc(u);
  for (uint32_t t = 1; t < (1u << (N - W)); ++t) {
    const uint32_t c = u ^ cl_mul(t, P);
    const int cw = popc(c);
    if (cw < bw || (cw == bw && c < best)) {
      best = c;
      bw = cw;
    }
  }
  return best;
}

// The terms of a product by the ring element C, grouped by accumulator:
// slice term[i][q] (q < cnt[i]) of a WD-slice operand lands on
// accumulator i.
template <int WD, int N, uint32_t C>
struct RotTerms {
  int cnt[N];
  int term[N][N];
  constexpr RotTerms() : cnt(), term() {
    for (int i = 0; i < N; ++i)
      for (int s = 0; s < N; ++s) {
        const int t = (i - s + N) % N;
        if ((C >> s & 1u) && t < WD) term[i][cnt[i]++] = t;
      }
  }
};

// acc += x^s d for every s set in C (a product by C in R_{2,N}), two terms
// per instruction: acc[i] = acc[i] ^ d[a] ^ d[b].
template <int WD, int N, uint32_t C, typename T>
__device__ __forceinline__ void rot_acc_fused(T (&acc)[N], const T (&d)[WD]) {
  constexpr RotTerms<WD, N, C> R{};
  // (constant trip counts, so both loops unroll fully and every index
  // folds to a constant: the operands stay in registers)
#pragma unroll
  for (int i = 0; i < N; ++i) {
#pragma unroll
    for (int q = 0; q < N; q += 2) {
      if (q + 1 < R.cnt[i]) acc[i] = xor3(acc[i], d[R.term[i][q]], d[R.term[i][q + 1]]);
      else if (q < R.cnt[i]) acc[i] ^= d[R.term[i][q]];
    }
  }
}

// acc += lift(u) d for a wave-uniform field element u in [LO, HI): a
// binary search of scalar compares reaches the body compiled for lift(u).
// (Each node compares u with its own constant, one s_cmp and one branch on
// SCC; tests of u's bits, the same at every node of a level, would be
// computed once up front and kept as 64-bit lane masks, costing an extra
// scalar AND per node.)
// SH = 16: u is the high half of the word (the low half is another
// element's, which the compares u < MID << 16 ignore).
template <int WD, int N, int W, uint32_t P, uint32_t LO, uint32_t HI, typename T, int SH = 0>
__device__ __forceinline__ void acc_field(T (&acc)[N], const T (&d)[WD], uint32_t u) {
  if constexpr (HI - LO == 1) {
    rot_acc_fused<WD, N, lift_const(LO, W, N, P), T>(acc, d);
  } else {
    constexpr uint32_t MID = (LO + HI) / 2;
    if (u < (MID << SH))
      acc_field<WD, N, W, P, LO, MID, T, SH>(acc, d, u);
    else
      acc_field<WD, N, W, P, MID, HI, T, SH>(acc, d, u);
  }
}

// acc[(t + s) mod N] ^= d[t] for t < W and every s >= S0 set in c.
// (SH: the element sits SH bits up in the word c; the bits below are others'.)
template <int W, int N, int S0, typename T, int SH = 0>
__device__ __forceinline__ void rot_acc(T (&acc)[N], const T (&d)[W], uint32_t c) {
  if constexpr (S0 < N) {
    if (c & (1u << (S0 + SH))) {
#pragma unroll
      for (int t = 0; t < W; ++t) acc[(t + S0) % N] ^= d[t];
    }
    rot_acc<W, N, S0 + 1, T, SH>(acc, d, c);
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
// block extended by its parity slices).  cf holds the coefficient words:
// field elements for the small fields (N <= 9, fused rotations), lifted
// ring elements otherwise.
//
// HI16: the coefficient words of odd rows r are 32-bit words whose high
// half is the coefficient (two 16-bit coefficients per word, the even row's
// in the low half, already isolated): they are used without a shift.
template <int W, int N, uint32_t P, int MO, bool PT, typename T, bool HI16 = false>
__device__ __forceinline__ void accumulate(T (&acc)[MO][N], const T (&d)[W], const Lift8 &cf) {
  constexpr bool kFused = N <= 9;
  if constexpr (PT) {
    T e[N];
    parity_embed<W, N, P, T>(e, d);
    static_for<0, MO>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      constexpr int SH = HI16 && (r & 1) ? 16 : 0;
      if constexpr (kFused) acc_field<N, N, W, P, 0, (1u << W), T, SH>(acc[r], e, cf[r]);
      else rot_acc<N, N, 0, T, SH>(acc[r], e, cf[r]);
    });
  } else {
    static_for<0, MO>([&](auto rc) {
      constexpr int r = decltype(rc)::value;
      constexpr int SH = HI16 && (r & 1) ? 16 : 0;
      if constexpr (kFused) acc_field<W, N, W, P, 0, (1u << W), T, SH>(acc[r], d, cf[r]);
      else rot_acc<W, N, 0, T, SH>(acc[r], d, cf[r]);
    });
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
template <int W, int V, int LP = kLoadPolicy>
__device__ __forceinline__ void load_block(typename Vec<V>::T (&d)[W], const uint8_t *base,
                                           uint32_t bytes, uint32_t pitch, uint32_t voff) {
  const __amdgpu_buffer_rsrc_t r = block_rsrc(base, bytes);
#pragma unroll
  for (int t = 0; t < W; ++t) d[t] = bload<V, LP>(r, voff, t * pitch);
}

// One lane column of one pass.  Src supplies wave-uniform values:
//   k(), S(), pitch(), nout(), in(j), out(r) and lift8(j) (the kMaxOut
//   coefficient words of input j: field elements on the small fields, lifted
//   ring elements otherwise); slice t of a block starts t * pitch() bytes
//   after its base.  Rows r >= nout() must have zero coefficient words; they
//   are neither reduced nor stored.
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
// LP: cache policy of the block loads (non-temporal by default; a kernel
// whose waves share their loads takes the default policy instead).
template <int W, int N, uint32_t P, int MO, int V, int KS = 1, bool PT = false,
          int LP = kLoadPolicy, class Src>
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
  auto prefetch = [&](T (&dst)[W], int jj, const uint8_t *base) {
    load_block<W, V, LP>(dst, base, jj < k ? span : 0u, pitch, voff);
  };
  // Scalar operands run ahead of their use: the block pointer one prefetch
  // ahead and the lifted coefficients one block ahead (one 16-byte scalar
  // load), so no scalar-load wait sits between the vector loads and XORs.
  prefetch(d[0], (int)part, src.in(clampj((int)part)));
  const uint8_t *ip = src.in(clampj((int)part + KS));
  Lift8 cf = src.lift8(clampj((int)part));
  // One step: block jq (in register set Q) into the accumulators while block
  // jq + KS loads into the other set.  The set is a compile-time constant.
  auto step = [&](auto qc, int jq) {
    constexpr int q = decltype(qc)::value;
    prefetch(d[q ^ 1], jq + KS, ip);
    ip = src.in(clampj(jq + 2 * KS));
    const Lift8 cn = src.lift8(clampj(jq + KS));
    accumulate<W, N, P, MO, PT, T>(acc, d[q], cf);
    cf = cn;
  };
  for (int j = (int)part; j < k; j += 2 * KS) {
    step(std::integral_constant<int, 0>{}, j);
    if (j + KS >= k) break;
    step(std::integral_constant<int, 1>{}, j + KS);
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
  auto prefetch = [&](T (&dst)[W], uint32_t cb, int jj) {
    const bool ok = cb < col1;
    load_block<W, V>(dst, src.in(ok ? jj : 0), ok ? span : 0u, pitch,
                     lane_load_voffset(lane_col(cb, lane, V), S));
  };
  uint32_t cb = col0;  // chunk being accumulated
  int j = 0;           // block being accumulated
  prefetch(d[0], cb, 0);
  // One step: block j of chunk cb (in register set Q) into the accumulators
  // while the next step's block loads into the other set: block j+1 of this
  // chunk, or block 0 of the next chunk.  False once the tile is done.
  auto step = [&](auto qc) -> bool {
    constexpr int q = decltype(qc)::value;
    const bool last = j + 1 == k;
    prefetch(d[q ^ 1], last ? cb + kChunk : cb, last ? 0 : j + 1);
    accumulate<W, N, P, MO, PT, T>(acc, d[q], src.lift8(j));
    if (!last) {
      ++j;
      return true;
    }
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
    return cb < col1;
  };
  while (cb < col1) {
    if (!step(std::integral_constant<int, 0>{})) break;
    if (!step(std::integral_constant<int, 1>{})) break;
  }
}

// ---- wide passes: one read of the inputs for several output groups -----
// s_waitcnt with vmcnt = N and the other counters at their maxima (gfx9
// encoding: vmcnt bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
template <int N>
__device__ __forceinline__ void wait_vmcnt() {
  static_assert(N >= 0 && N < 64, "vmcnt range");
  __builtin_amdgcn_s_waitcnt((N & 15) | ((N >> 4) << 14) | (7 << 4) | (15 << 8));
}

// One column chunk (64 lanes x 4V bytes) of a wide pass, coded by the G
// waves of a workgroup: wave g accumulates its MO outputs from every input
// block, and the blocks reach the waves through a ring of D stages in LDS
// (`stage`: D x W x V x 64 dwords, then a 64-dword sink) that the waves
// fill together, each block loaded from HBM once.  A block is W V dword
// loads (load q: dword q mod V of every lane of slice q / V, straight into
// LDS with buffer loads to LDS, no registers held); wave g issues loads g,
// g + G, ..., NG = ceil(W V / G) of them per block, a slot past the last
// load repeating load (its index mod W V) into the sink, so that every wave
// has the same known count of loads per block in flight and no slot needs a
// per-block test.  The blocks are coded B at a time: at step j (a multiple
// of B) each wave waits until its loads of blocks j .. j + B - 1 have
// completed (the D - 2B blocks it issued since may still be in flight), then
// a barrier makes every wave's part visible; the B stages read by every
// wave before that barrier are then refilled with blocks j + D - B ..
// j + D - 1.  Loads past the last block use an empty descriptor (no
// traffic).  Lanes past the end of the slice load nothing and store
// nothing.
//
// Src supplies k(), S(), pitch(), nout(), out(r), in_words() (the k input
// block addresses, wave-uniform, readable up to D + B words past k: those
// reads only address loads with an empty descriptor, or go unused),
// records() (this wave's coefficient
// records, one per input block, readable one past the last; at most B - 1
// blocks past the last are skipped), unpack(record)
// -> Lift8 and kHi16 (see accumulate).  The per-block scalar work is kept
// small (running pointers, per-wave constants hoisted): the coefficient
// dispatch already costs the scalar unit about as many instructions as the
// XORs cost the vector unit.
template <int W, int N, uint32_t P, int MO, bool PT, int D, int B, int NG, int V, class Src>
__device__ __forceinline__ void code_column_staged(const Src &src, uint32_t col, uint32_t lane,
                                                   uint32_t g, uint32_t G, uint32_t *stage) {
  static_assert((D - 2 * B) * NG < 64, "awaited loads must fit vmcnt");
  static_assert(B == 1 || B == 2, "blocks per barrier");
  static_assert((D & (D - 1)) == 0, "stages: a power of two");
  static_assert(V == 1 || V == 2, "lane width");
  typedef typename Vec<V>::T T;
  typedef __attribute__((address_space(3))) void *lds_ptr;
  constexpr uint32_t kLoads = W * V;
  const int k = src.k();
  const uint32_t S = src.S();
  const uint32_t pitch = src.pitch();
  const uint32_t span = block_span(W, S, pitch);
  const uint32_t voff = lane_load_voffset(col, S);
  T acc[MO][N];
#pragma unroll
  for (int r = 0; r < MO; ++r)
#pragma unroll
    for (int i = 0; i < N; ++i) acc[r][i] = (T)0;

  // this wave's NG loads per block: load q_u = g + u G (slice q / V, dword
  // q mod V of each lane), or past the last, load q_u mod W V again into the
  // sink after the stages
  // (the LDS target of load u for the block in stage `slot` is
  // (slot & smask[u]) + loff[u]: the stage row of a live load, the sink for
  // any block otherwise)
  uint32_t soff[NG], loff[NG], smask[NG];
  static_for<0, NG>([&](auto uc) {
    constexpr int u = decltype(uc)::value;
    const uint32_t q = g + (uint32_t)u * G;
    const bool live = q < kLoads;
    const uint32_t qq = live ? q : q % kLoads;
    soff[u] = (qq / V) * pitch + (qq % V) * 4u;
    loff[u] = (live ? q * 64u : D * kLoads * 64u) * 4u;  // bytes
    smask[u] = live ? 0xFFFFFFFFu : 0u;
    // (held as plain scalar words, opaque to the compiler: otherwise it
    // rebuilds the mask from `live` at every load, a compare-and-select of
    // four scalar instructions instead of one AND)
    smask[u] = __builtin_amdgcn_readfirstlane(smask[u]);
    loff[u] = __builtin_amdgcn_readfirstlane(loff[u]);
    __asm__ volatile("" : "+s"(smask[u]), "+s"(loff[u]));
  });
  const auto *ip = src.in_words();     // address of input block jj at ip[jj]
  const auto *rec = src.records();     // coefficient record of block j at rec[j]
  constexpr uint32_t kStage = kLoads * 64u;
  auto issue = [&](int jj, const uint8_t *in) {
    const uint32_t bytes = jj < k ? span : 0u;
    const uint32_t slot = (uint32_t)(jj & (D - 1)) * (kStage * 4u);  // bytes
    static_for<0, NG>([&](auto uc) {
      constexpr int u = decltype(uc)::value;
      const __amdgpu_buffer_rsrc_t r = block_rsrc(in, bytes);
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          r, (lds_ptr)((char *)stage + ((slot & smask[u]) + loff[u])), 4, voff, soff[u], 0, 0);
    });
  };
  for (int jj = 0; jj < D - B; ++jj) issue(jj, (const uint8_t *)ip[jj]);
  // the addresses of the blocks issued at the next step, read a step ahead
  const uint8_t *pin[B];
  static_for<0, B>([&](auto bc) {
    pin[decltype(bc)::value] = (const uint8_t *)ip[D - B + decltype(bc)::value];
  });
  Lift8 cf = src.unpack(rec[0]);
  for (int j = 0; j < k; j += B) {
    wait_vmcnt<(D - 2 * B) * NG>();
    // (the empty asm statements keep the compiler from moving LDS reads
    // across the barrier, which it does not see as a memory operation)
    __asm__ volatile("" ::: "memory");
    __builtin_amdgcn_s_barrier();
    __asm__ volatile("" ::: "memory");
    static_for<0, B>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      issue(j + D - B + b, pin[b]);
      pin[b] = (const uint8_t *)ip[j + D + b];
    });
    static_for<0, B>([&](auto bc) {
      constexpr int b = decltype(bc)::value;
      const int jb = j + b;
      if (b > 0 && jb >= k) return;
      const auto next = rec[jb + 1];  // (one record past this group's last: padding)
      const uint32_t *blk = stage + (uint32_t)(jb & (D - 1)) * kStage + lane;
      T d[W];
#pragma unroll
      for (int t = 0; t < W; ++t) {
        if constexpr (V == 1)
          d[t] = blk[t * 64];
        else
          d[t] = T{blk[(2 * t) * 64], blk[(2 * t + 1) * 64]};
      }
      accumulate<W, N, P, MO, PT, T, Src::kHi16>(acc, d, cf);
      cf = src.unpack(next);
    });
  }
  // The loads issued past the last block (empty descriptors) still write
  // their LDS slots: let them land before the wave can end and the
  // workgroup's LDS pass to another workgroup.
  wait_vmcnt<0>();
  if (col >= S) return;
#pragma unroll
  for (int r = 0; r < MO; ++r) {
    if (r >= src.nout()) break;
    leave_ring<W, N, P, PT, T>(acc[r]);
    const __amdgpu_buffer_rsrc_t o = block_rsrc(src.out(r), span);
#pragma unroll
    for (int t = 0; t < W; ++t) bstore<V>(acc[r][t], o, col, t * pitch);
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
