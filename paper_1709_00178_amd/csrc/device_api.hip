// C ABI device entry points: encode, decode, fill, copy.
#include <hip/hip_runtime.h>

#include <cstring>

#include "internal.hpp"

namespace pyrit {

template <int RING>
int launch_plain_ring(int nout, int vec_bytes, const PassArgs &a, hipStream_t st);

int default_vec_bytes(int ring, int nout) {
  // Column bytes per lane of the plain kernel, chosen by measurement on
  // MI355X (encodes of 16 MiB blocks, every ring and output count against
  // 4-, 8- and 16-byte lanes): the 8-slice field takes 4-byte lanes at every
  // output count (16-byte lanes lost up to 13%); the 4-slice field 8-byte
  // lanes up to four outputs (16-byte lanes lost up to 35%); the 6- and
  // 10-slice fields 16-byte lanes for one output, 8-byte lanes up to four and
  // 4-byte lanes beyond (8-byte lanes also gave C2's 256 launches of 4 MiB
  // blocks +6% over 4-byte ones).  The widest lane that fits a register
  // budget is not the fastest: at the same accumulator count, 6-slice codes
  // ran 11% faster with four outputs on 8-byte lanes than with two outputs on
  // 16-byte lanes.
  const int n = kRings[ring].n;
  if (n >= 17) return 4;
  if (n <= 5) return nout <= 4 ? 8 : 4;
  return nout == 1 ? 16 : nout <= 4 ? 8 : 4;
}

int launch_pass(int ring, int nout, int vec_bytes, const PassArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  if (vec_bytes == 0) vec_bytes = default_vec_bytes(ring, nout);
  switch (ring) {
    case 0: return launch_plain_ring<0>(nout, vec_bytes, a, st);
    case 1: return launch_plain_ring<1>(nout, vec_bytes, a, st);
    case 2: return launch_plain_ring<2>(nout, vec_bytes, a, st);
    case 3: return launch_plain_ring<3>(nout, vec_bytes, a, st);
    case 4: return launch_plain_ring<4>(nout, vec_bytes, a, st);
    case 5: return launch_plain_ring<5>(nout, vec_bytes, a, st);
    case 6: return launch_plain_ring<6>(nout, vec_bytes, a, st);
    case 7: return launch_plain_ring<7>(nout, vec_bytes, a, st);
    default: return PYRIT_EUNSUPPORTED;
  }
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Run the passes for `nout` outputs of a lifted k-column matrix L (row r of
// L belongs to out[r]), at most ring_max_out outputs per pass.
static int run_passes(const pyrit_plan *pl, const uint8_t *const *in, uint8_t *const *out, int nout,
                      const uint32_t *L, size_t S, size_t pitch, int vec_bytes, void *stream) {
  PassArgs a;
  std::memset(&a, 0, sizeof(a));
  a.k = (uint32_t)pl->k;
  a.S = (uint32_t)S;
  a.pitch = (uint32_t)pitch;
  for (int j = 0; j < pl->k; ++j) {
    if (!in[j]) return PYRIT_EINVAL;
    if (!aligned16(in[j])) return PYRIT_EALIGN;
    a.in[j] = in[j];
  }
  const int per_pass = ring_max_out(pl->ring);
  for (int r0 = 0; r0 < nout; r0 += per_pass) {
    const int cnt = nout - r0 < per_pass ? nout - r0 : per_pass;
    for (int r = 0; r < kMaxOut; ++r) a.out[r] = nullptr;
    for (int r = 0; r < cnt; ++r) {
      if (!out[r0 + r]) return PYRIT_EINVAL;
      if (!aligned16(out[r0 + r])) return PYRIT_EALIGN;
      a.out[r] = out[r0 + r];
      for (int j = 0; j < pl->k; ++j) a.lift[j][r] = L[(size_t)(r0 + r) * pl->k + j];
    }
    for (int r = cnt; r < kMaxOut; ++r)
      for (int j = 0; j < pl->k; ++j) a.lift[j][r] = 0;
    int rc = launch_pass(pl->ring, cnt, vec_bytes, a, stream);
    if (rc) return rc;
  }
  return PYRIT_OK;
}

}  // namespace pyrit

using namespace pyrit;

extern "C" {

int pyrit_encode_ex(const pyrit_plan *plan, const uint8_t *const *data, uint8_t *const *parity,
                    size_t slice_bytes, size_t slice_pitch, int vec_bytes, void *stream) {
  if (!plan || !data || !parity) return PYRIT_EINVAL;
  if (plan->ring < 0) return PYRIT_EUNSUPPORTED;
  if (vec_bytes != 0 && vec_bytes != 4 && vec_bytes != 8 && vec_bytes != 16) return PYRIT_EINVAL;
  int rc = check_slices(plan->w, slice_bytes, &slice_pitch);
  if (rc) return rc;
  return run_passes(plan, data, parity, plan->m, plan->L.data(), slice_bytes, slice_pitch,
                    vec_bytes, stream);
}

int pyrit_encode(const pyrit_plan *plan, const uint8_t *const *data, uint8_t *const *parity,
                 size_t slice_bytes, void *stream) {
  return pyrit_encode_ex(plan, data, parity, slice_bytes, 0, 0, stream);
}

int pyrit_decode_ex(const pyrit_plan *plan, const int *erased, int n_erased, uint8_t *const *blocks,
                    size_t slice_bytes, size_t slice_pitch, void *stream) {
  if (!plan || !blocks) return PYRIT_EINVAL;
  if (plan->ring < 0) return PYRIT_EUNSUPPORTED;
  int rc = check_slices(plan->w, slice_bytes, &slice_pitch);
  if (rc) return rc;
  std::shared_ptr<const DecodeEntry> ent;
  rc = decode_entry(plan, erased, n_erased, &ent);
  if (rc) return rc;
  if (ent->outs.empty()) return PYRIT_OK;
  const uint8_t *in[PYRIT_KMAX];
  uint8_t *out[PYRIT_MMAX];
  for (int j = 0; j < plan->k; ++j) in[j] = blocks[ent->surv[j]];
  for (size_t e = 0; e < ent->outs.size(); ++e) out[e] = blocks[ent->outs[e]];
  return run_passes(plan, in, out, (int)ent->outs.size(), ent->L.data(), slice_bytes, slice_pitch,
                    0, stream);
}

int pyrit_decode(const pyrit_plan *plan, const int *erased, int n_erased, uint8_t *const *blocks,
                 size_t slice_bytes, void *stream) {
  return pyrit_decode_ex(plan, erased, n_erased, blocks, slice_bytes, 0, stream);
}

}  // extern "C"

// ------------------------------------------------------------------ utilities
namespace pyrit {

__device__ __forceinline__ uint64_t splitmix_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Word q of the buffer: mix(key + (q + 1) * golden gamma); bytes past
// nrandom are zero.
__global__ __launch_bounds__(256) void fill_random_kernel(uint64_t *dst, uint64_t nwords,
                                                          uint64_t nrandom, uint64_t key) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t q = (uint64_t)blockIdx.x * 256u + threadIdx.x; q < nwords; q += stride) {
    uint64_t v = splitmix_mix(key + (q + 1) * 0x9E3779B97F4A7C15ull);
    const uint64_t b0 = q * 8;
    if (b0 + 8 > nrandom) {
      const uint64_t keep = nrandom > b0 ? nrandom - b0 : 0;  // 0..7 bytes kept
      v = keep ? (v & ((1ull << (8 * keep)) - 1)) : 0;
    }
    dst[q] = v;
  }
}

typedef uint32_t cu32x4 __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void copy_kernel(cu32x4 *dst, const cu32x4 *src, uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < n16; i += stride)
    __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

static unsigned grid_for(uint64_t items) {
  uint64_t g = (items + 255) / 256;
  const uint64_t cap = 256ull * 64;  // 64 workgroups per CU on 256 CUs
  if (g > cap) g = cap;
  return (unsigned)(g ? g : 1);
}

}  // namespace pyrit

extern "C" {

int pyrit_fill_random(uint8_t *dst, size_t nbytes, size_t nrandom, uint64_t key, void *stream) {
  if (!dst || nbytes % 8 != 0 || ((uintptr_t)dst & 7u)) return PYRIT_EINVAL;
  if (nbytes == 0) return PYRIT_OK;
  if (nrandom > nbytes) nrandom = nbytes;
  const uint64_t nw = nbytes / 8;
  hipLaunchKernelGGL(fill_random_kernel, dim3(grid_for(nw)), dim3(256), 0, (hipStream_t)stream,
                     (uint64_t *)dst, (uint64_t)nw, (uint64_t)nrandom, (uint64_t)key);
  return hipGetLastError() == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

int pyrit_copy(uint8_t *dst, const uint8_t *src, size_t nbytes, void *stream) {
  if (!dst || !src || nbytes % 16 != 0 || ((uintptr_t)dst & 15u) || ((uintptr_t)src & 15u))
    return PYRIT_EINVAL;
  if (nbytes == 0) return PYRIT_OK;
  const uint64_t n16 = nbytes / 16;
  hipLaunchKernelGGL(copy_kernel, dim3(grid_for(n16)), dim3(256), 0, (hipStream_t)stream,
                     (cu32x4 *)dst, (const cu32x4 *)src, (uint64_t)n16);
  return hipGetLastError() == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

}  // extern "C"
