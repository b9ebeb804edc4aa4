// Plain per-stripe kernel: one launch codes one pass (up to ring_max_out outputs)
// of one stripe.  Workgroup b is two waves sharing the column chunk of 64
// lanes x 4V bytes at b * 256V (split-K: each wave codes every other input
// block; partial sums meet in LDS).
#pragma once
#include "ring_kernels.hpp"

namespace pyrit {

constexpr uint32_t kPlainWG = 128;

template <int RING, int MO, int V>
__global__ __launch_bounds__(kPlainWG) void plain_pass_kernel(const PassArgs a) {
  constexpr RingDesc R = kRings[RING];
  typedef typename dev::Vec<V>::T T;
  __shared__ T xch[MO * R.w * 64];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t part = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t col = lane_col(plain_chunk_base(blockIdx.x, V), lane, V);
  dev::code_column<R.w, R.n, R.p, MO, V, 2, R.parity>(dev::KernargSrc{a}, col, col < a.S, part, xch);
}

// Wide pass: workgroup b = G waves on the column chunk at b * 256 bytes
// (4-byte lanes); wave g codes output group g from every input block, the
// blocks staged once per workgroup in LDS (code_column_staged).
#define PYRIT_AS4 __attribute__((address_space(4)))

struct WideSrc {
  const WideArgs &a;
  uint32_t g;  // this wave's output group
  static constexpr uint32_t kH = wide_header_words();
  __device__ int k() const { return (int)(uint32_t)a.w[0]; }
  __device__ uint32_t S() const { return (uint32_t)(a.w[0] >> 32); }
  __device__ uint32_t pitch() const { return (uint32_t)a.w[1]; }
  __device__ uint32_t groups() const { return (uint32_t)(a.w[1] >> 32); }
  __device__ int nout() const { return (int)((a.w[2 + g / 16] >> (4 * (g % 16))) & 15u); }
  // the input addresses (read up to D + B words past the k-th: output pointers and
  // records, all inside the argument block)
  __device__ const PYRIT_AS4 uint64_t *in_words() const {
    return (const PYRIT_AS4 uint64_t *)&a.w[kH];
  }
};
// Records of RW words: RW = 1 holds up to four 16-bit coefficient words (or
// two 32-bit ones), RW = 2 up to eight (four).
template <int MO, int RW, bool WORDS16>
struct WideGroupSrc : WideSrc {
  typedef typename dev::Vec<2 * RW>::T Rec;
  // 16-bit words: odd rows read their coefficient from the high half of the
  // 32-bit word in place (accumulate's HI16)
  static constexpr bool kHi16 = WORDS16;
  __device__ uint8_t *out(int r) const { return (uint8_t *)a.w[kH + k() + g * MO + r]; }
  __device__ const PYRIT_AS4 Rec *records() const {
    return (const PYRIT_AS4 Rec *)&a.w[kH + k() + groups() * MO + RW * g * (uint32_t)k()];
  }
  __device__ dev::Lift8 unpack(Rec x) const {
    if constexpr (RW == 1) {
      if constexpr (WORDS16)
        return dev::Lift8{dev::u32x4{x.x & 0xFFFFu, x.x, x.y & 0xFFFFu, x.y},
                          dev::u32x4{0u, 0u, 0u, 0u}};
      else
        return dev::Lift8{dev::u32x4{x.x, x.y, 0u, 0u}, dev::u32x4{0u, 0u, 0u, 0u}};
    } else {
      if constexpr (WORDS16)
        return dev::Lift8{dev::u32x4{x.x & 0xFFFFu, x.x, x.y & 0xFFFFu, x.y},
                          dev::u32x4{x.z & 0xFFFFu, x.z, x.w & 0xFFFFu, x.w}};
      else
        return dev::Lift8{x, dev::u32x4{0u, 0u, 0u, 0u}};
    }
  }
};

// NG: the dword loads each wave issues per block.  The embedding transform
// on the ring (6,9) asks for eight waves per SIMD (at most 64 VGPRs), which
// its five outputs per wave fit.
template <int RING>
constexpr int wide_min_waves() {
  return (kRings[RING].n == 9 && !kRings[RING].parity) ? 8 : 1;
}
template <int RING, int NG>
__global__ __launch_bounds__(64 * kWideMaxGroups)
__attribute__((amdgpu_waves_per_eu(wide_min_waves<RING>()))) void wide_pass_kernel(const WideArgs a) {
  constexpr RingDesc R = kRings[RING];
  constexpr int MO = wide_max_out(RING);
  constexpr int D = wide_stages(RING);
  constexpr int V = kWideV;
  __shared__ uint32_t stage[(D * R.w * V + 1) * 64];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t g = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t G = blockDim.x >> 6;
  const WideGroupSrc<MO, wide_rec_words(RING), (R.n <= 16)> src{{a, g}};
  const uint32_t col = lane_col(plain_chunk_base(blockIdx.x, V), lane, V);
  dev::code_column_staged<R.w, R.n, R.p, MO, R.parity, D, wide_blocks_per_barrier(RING), NG, V>(
      src, col, lane, g, G, stage);
}

// NG: the power of two at or above ceil(2 w / G) (slots past the block's
// loads repeat loads into the sink).
template <int RING, int NG>
static int launch_wide_ng(int groups, const WideArgs &a, hipStream_t st) {
  constexpr int kLoads = kRings[RING].w * kWideV;  // dword loads per block
  if constexpr (NG > 2 * ((kLoads + 1) / 2)) {
    return PYRIT_EINVAL;
  } else {
    if (NG * groups < kLoads) return launch_wide_ng<RING, 2 * NG>(groups, a, st);
    const uint32_t S = (uint32_t)(a.w[0] >> 32);
    const uint32_t chunk = 256u * kWideV;
    const uint32_t blocks = (S + chunk - 1) / chunk;
    hipLaunchKernelGGL((wide_pass_kernel<RING, NG>), dim3(blocks), dim3(64 * groups), 0, st, a);
    return hipGetLastError() == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
  }
}

template <int RING>
int launch_wide_ring(int groups, const WideArgs &a, hipStream_t st) {
  if (groups < 2 || groups > kWideMaxGroups) return PYRIT_EINVAL;
  return launch_wide_ng<RING, 1>(groups, a, st);
}

template <int RING, int MO, int V>
static int launch_plain(const PassArgs &a, hipStream_t st) {
  const uint32_t per_block = 64u * 4u * V;
  const uint32_t blocks = (a.S + per_block - 1) / per_block;
  hipLaunchKernelGGL((plain_pass_kernel<RING, MO, V>), dim3(blocks), dim3(kPlainWG), 0, st, a);
  return hipGetLastError() == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

template <int RING, int MO>
static int launch_plain_v(int vec_bytes, const PassArgs &a, hipStream_t st) {
  switch (vec_bytes) {
    case 4: return launch_plain<RING, MO, 1>(a, st);
    case 8: return launch_plain<RING, MO, 2>(a, st);
    case 16: return launch_plain<RING, MO, 4>(a, st);
    default: return PYRIT_EINVAL;
  }
}

template <int RING, int MO>
static int launch_plain_mo(int nout, int vec_bytes, const PassArgs &a, hipStream_t st) {
  if constexpr (MO > ring_max_out(RING)) {
    return PYRIT_EINVAL;
  } else {
    if (nout == MO) return launch_plain_v<RING, MO>(vec_bytes, a, st);
    if constexpr (MO < kMaxOut) return launch_plain_mo<RING, MO + 1>(nout, vec_bytes, a, st);
    return PYRIT_EINVAL;
  }
}

template <int RING>
int launch_plain_ring(int nout, int vec_bytes, const PassArgs &a, hipStream_t st) {
  return launch_plain_mo<RING, 1>(nout, vec_bytes, a, st);
}

}  // namespace pyrit
