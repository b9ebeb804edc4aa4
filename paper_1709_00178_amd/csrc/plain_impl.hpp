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
