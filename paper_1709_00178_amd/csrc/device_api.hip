// C ABI device entry points: encode, decode, fill, copy.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "internal.hpp"
#include "ring_kernels.hpp"

namespace pyrit {

template <int RING>
int launch_plain_ring(int nout, int vec_bytes, const PassArgs &a, hipStream_t st);
template <int RING>
int launch_wide_ring(int groups, const WideArgs &a, hipStream_t st);

static int launch_wide(int ring, int groups, const WideArgs &a, void *stream) {
  hipStream_t st = (hipStream_t)stream;
  switch (ring) {
    case 0: return launch_wide_ring<0>(groups, a, st);
    case 1: return launch_wide_ring<1>(groups, a, st);
    case 2: return launch_wide_ring<2>(groups, a, st);
    case 3: return launch_wide_ring<3>(groups, a, st);
    case 4: return launch_wide_ring<4>(groups, a, st);
    case 5: return launch_wide_ring<5>(groups, a, st);
    case 6: return launch_wide_ring<6>(groups, a, st);
    case 7: return launch_wide_ring<7>(groups, a, st);
    default: return PYRIT_EUNSUPPORTED;
  }
}

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

// Run the passes for `nout` outputs of a k-column matrix of coefficient
// words (coef_words; row r belongs to out[r]), at most ring_max_out outputs
// per pass.
static int run_passes(const pyrit_plan *pl, const uint8_t *const *in, uint8_t *const *out, int nout,
                      const uint32_t *coef, size_t S, size_t pitch, int vec_bytes, void *stream) {
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
      for (int j = 0; j < pl->k; ++j) a.lift[j][r] = coef[(size_t)(r0 + r) * pl->k + j];
    }
    for (int r = cnt; r < kMaxOut; ++r)
      for (int j = 0; j < pl->k; ++j) a.lift[j][r] = 0;
    int rc = launch_pass(pl->ring, cnt, vec_bytes, a, stream);
    if (rc) return rc;
  }
  return PYRIT_OK;
}

// The same outputs in wide launches: each launch codes 2 to
// wide_groups_fit groups of up to wide_max_out outputs with one read of the
// inputs (all arguments in the kernel-argument segment, laid out as rings.hpp
// describes).  The outputs of a launch are spread over its groups as evenly
// as possible; a last pass's worth of outputs alone takes a plain pass.
static int run_wide(const pyrit_plan *pl, const uint8_t *const *in, uint8_t *const *out, int nout,
                    const uint32_t *coef, size_t S, size_t pitch, void *stream) {
  const int k = pl->k, ring = pl->ring;
  const int MO = wide_max_out(ring);
  const int RW = wide_rec_words(ring);
  const int fit = wide_groups_fit(ring, k);
  const bool words16 = kRings[ring].n <= 16;
  const uint32_t H = wide_header_words();
  for (int j = 0; j < k; ++j) {
    if (!in[j]) return PYRIT_EINVAL;
    if (!aligned16(in[j])) return PYRIT_EALIGN;
  }
  for (int r = 0; r < nout; ++r) {
    if (!out[r]) return PYRIT_EINVAL;
    if (!aligned16(out[r])) return PYRIT_EALIGN;
  }
  for (int r0 = 0; r0 < nout;) {
    const int left = nout - r0;
    if (left <= ring_max_out(ring))  // one pass left: the plain kernel (split-K) codes it
      return run_passes(pl, in, out + r0, left, coef + (size_t)r0 * k, S, pitch, 0, stream);
    const int G = std::min(fit, (left + MO - 1) / MO);
    const int cnt = std::min(left, G * MO);
    WideArgs a;
    std::memset(&a, 0, sizeof(a));
    a.w[0] = (uint64_t)(uint32_t)k | (uint64_t)S << 32;
    a.w[1] = (uint64_t)pitch | (uint64_t)G << 32;
    const uint32_t rec0 = H + (uint32_t)k + (uint32_t)(G * MO);  // first record word
    for (int j = 0; j < k; ++j) a.w[H + j] = (uint64_t)(uintptr_t)in[j];
    for (int g = 0; g < G; ++g) {
      const int first = cnt * g / G, n_g = cnt * (g + 1) / G - first;  // 1..MO outputs
      a.w[2 + g / 16] |= (uint64_t)n_g << (4 * (g % 16));
      for (int r = 0; r < n_g; ++r) {
        const int o = r0 + first + r;
        a.w[H + k + g * MO + r] = (uint64_t)(uintptr_t)out[o];
        for (int j = 0; j < k; ++j) {
          const uint32_t cw = coef[(size_t)o * k + j];
          uint8_t *rec = (uint8_t *)&a.w[rec0 + RW * (g * k + j)];
          if (words16) {
            const uint16_t v = (uint16_t)cw;
            std::memcpy(rec + 2 * r, &v, 2);
          } else {
            std::memcpy(rec + 4 * r, &cw, 4);
          }
        }
      }
    }
    int rc = launch_wide(ring, G, a, stream);
    if (rc) return rc;
    r0 += cnt;
  }
  return PYRIT_OK;
}

// Codes whose outputs need more than one pass take wide launches when at
// least two output groups fit one launch and the caller left the lane width
// to the library; otherwise one plain pass per ring_max_out outputs.
static int run_outputs(const pyrit_plan *pl, const uint8_t *const *in, uint8_t *const *out,
                       int nout, const uint32_t *coef, size_t S, size_t pitch, int vec_bytes,
                       void *stream) {
  if (vec_bytes == 0 && nout > ring_max_out(pl->ring) && wide_groups_fit(pl->ring, pl->k) >= 2)
    return run_wide(pl, in, out, nout, coef, S, pitch, stream);
  return run_passes(pl, in, out, nout, coef, S, pitch, vec_bytes, stream);
}

}  // namespace pyrit

using namespace pyrit;

extern "C" {

int pyrit_encode_ex(const pyrit_plan *plan, const uint8_t *const *data, uint8_t *const *parity,
                    size_t slice_bytes, size_t slice_pitch, int vec_bytes, void *stream) {
  return abi_guard([&]() -> int {
    if (!plan || !data || !parity) return PYRIT_EINVAL;
    if (plan->ring < 0) return PYRIT_EUNSUPPORTED;
    if (vec_bytes != 0 && vec_bytes != 4 && vec_bytes != 8 && vec_bytes != 16) return PYRIT_EINVAL;
    int rc = check_slices(plan->w, slice_bytes, &slice_pitch);
    if (rc) return rc;
    return run_outputs(plan, data, parity, plan->m, plan->K.data(), slice_bytes, slice_pitch,
                       vec_bytes, stream);
  });
}

int pyrit_encode(const pyrit_plan *plan, const uint8_t *const *data, uint8_t *const *parity,
                 size_t slice_bytes, void *stream) {
  return pyrit_encode_ex(plan, data, parity, slice_bytes, 0, 0, stream);
}

int pyrit_decode_ex(const pyrit_plan *plan, const int *erased, int n_erased, uint8_t *const *blocks,
                    size_t slice_bytes, size_t slice_pitch, void *stream) {
  return abi_guard([&]() -> int {
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
    return run_outputs(plan, in, out, (int)ent->outs.size(), ent->K.data(), slice_bytes,
                       slice_pitch, 0, stream);
  });
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

// Word q of a buffer: mix(key + (q + 1) * golden gamma); bytes past
// nrandom are zero.
__device__ __forceinline__ uint64_t fill_word(uint64_t key, uint64_t q, uint64_t nrandom) {
  uint64_t v = splitmix_mix(key + (q + 1) * 0x9E3779B97F4A7C15ull);
  const uint64_t b0 = q * 8;
  if (b0 + 8 > nrandom) {
    const uint64_t keep = nrandom > b0 ? nrandom - b0 : 0;  // 0..7 bytes kept
    v = keep ? (v & ((1ull << (8 * keep)) - 1)) : 0;
  }
  return v;
}

__global__ __launch_bounds__(256) void fill_random_kernel(uint64_t *dst, uint64_t nwords,
                                                          uint64_t nrandom, uint64_t key) {
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t q = (uint64_t)blockIdx.x * 256u + threadIdx.x; q < nwords; q += stride)
    dst[q] = fill_word(key, q, nrandom);
}

// Many buffers in one launch.  Buffer i is cut into tiles of kFillTile
// words; tiles are numbered buffer by buffer (first_tile[i] is buffer i's
// first), and a workgroup finds its buffer by a binary search over them.
constexpr uint64_t kFillTile = 256u * 16u;

struct FillRec {
  uint64_t dst, nwords, nrandom, key, first_tile;
};

__global__ __launch_bounds__(256) void fill_blocks_kernel(const FillRec *recs, uint32_t n,
                                                          uint64_t n_tiles) {
  for (uint64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) >> 1;
      if (recs[mid].first_tile <= t) lo = mid;
      else hi = mid;
    }
    const FillRec r = recs[lo];
    uint64_t *dst = (uint64_t *)r.dst;
    const uint64_t q0 = (t - r.first_tile) * kFillTile;
    const uint64_t q1 = q0 + kFillTile < r.nwords ? q0 + kFillTile : r.nwords;
    for (uint64_t q = q0 + threadIdx.x; q < q1; q += 256u) dst[q] = fill_word(r.key, q, r.nrandom);
  }
}

// Device copy: non-temporal 16-byte loads, each 16-byte unit stored as two
// 8-byte stores with the default cache policy.  (On MI355X a 1:1 copy of
// 0.9 GiB ran 5.4 TB/s this way, 4.7-5.2 TB/s with non-temporal 8-byte
// stores and 2.5 TB/s with the coding kernels' SC1 8-byte stores, which
// suit their 10:4 read/write streams.)
// A wave copies kCopyUnits x 1 KiB per step, and its loads run one step
// ahead of its stores: on gfx9-family parts one in-order counter covers
// loads and stores, so waiting for loads issued after a step's stores would
// also wait for those stores to complete, while loads issued before them
// can be awaited alone.  Each step's bytes are addressed through a buffer
// descriptor of exactly the bytes that remain (none past the last step), so
// lanes past the end neither load nor store.  Every 16-byte unit is stored
// as two 8-byte stores (a wider store reads its data registers after it
// issues, which generated code has been seen to overwrite before the read).
constexpr uint32_t kCopyUnits = 4;
constexpr uint64_t kCopyStep = 64u * 16u * kCopyUnits;  // bytes per wave step

__device__ __forceinline__ uint32_t copy_step_bytes(uint64_t s, uint64_t steps, uint64_t nbytes) {
  if (s >= steps) return 0u;
  const uint64_t left = nbytes - s * kCopyStep;
  return (uint32_t)(left < kCopyStep ? left : kCopyStep);
}

// Load step s into x (nothing, through an empty descriptor, past the end).
__device__ __forceinline__ void copy_load(dev::u32x4 (&x)[kCopyUnits], const uint8_t *src,
                                          uint64_t s, uint64_t steps, uint64_t nbytes,
                                          uint32_t lane) {
  const __amdgpu_buffer_rsrc_t r =
      dev::block_rsrc(src + (s < steps ? s * kCopyStep : 0), copy_step_bytes(s, steps, nbytes));
#pragma unroll
  for (uint32_t u = 0; u < kCopyUnits; ++u) x[u] = dev::bload<4>(r, (u * 64u + lane) * 16u, 0u);
}

__device__ __forceinline__ void copy_store(const dev::u32x4 (&x)[kCopyUnits], uint8_t *dst,
                                           uint64_t s, uint64_t steps, uint64_t nbytes,
                                           uint32_t lane) {
  const __amdgpu_buffer_rsrc_t r =
      dev::block_rsrc(dst + s * kCopyStep, copy_step_bytes(s, steps, nbytes));
#pragma unroll
  for (uint32_t u = 0; u < kCopyUnits; ++u) dev::bstore<4, 0>(x[u], r, (u * 64u + lane) * 16u, 0u);
}

__global__ __launch_bounds__(256) void copy_kernel(uint8_t *dst, const uint8_t *src,
                                                   uint64_t nbytes) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t steps = (nbytes + kCopyStep - 1) / kCopyStep;
  const uint64_t stride = (uint64_t)gridDim.x * 4u;
  uint64_t s = (uint64_t)blockIdx.x * 4u + wave;
  if (s >= steps) return;
  // two register sets in turn: step s + stride is in flight while step s is
  // stored
  dev::u32x4 x[kCopyUnits], y[kCopyUnits];
  copy_load(x, src, s, steps, nbytes, lane);
  while (true) {
    copy_load(y, src, s + stride, steps, nbytes, lane);
    copy_store(x, dst, s, steps, nbytes, lane);
    s += stride;
    if (s >= steps) break;
    copy_load(x, src, s + stride, steps, nbytes, lane);
    copy_store(y, dst, s, steps, nbytes, lane);
    s += stride;
    if (s >= steps) break;
  }
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

int pyrit_fill_random_blocks(uint8_t *const *dst, const size_t *nbytes, const size_t *nrandom,
                             const uint64_t *keys, int n, void *stream) {
  return abi_guard([&]() -> int {
    if (n < 0 || (n > 0 && (!dst || !nbytes || !keys))) return PYRIT_EINVAL;
    std::vector<FillRec> recs;
    recs.reserve((size_t)n);
    uint64_t tiles = 0;
    for (int i = 0; i < n; ++i) {
      if (nbytes[i] == 0) continue;  // nothing to fill: the address may be NULL
      if (!dst[i] || nbytes[i] % 8 != 0 || ((uintptr_t)dst[i] & 7u)) return PYRIT_EINVAL;
      const uint64_t nr = nrandom ? std::min<uint64_t>(nrandom[i], nbytes[i]) : nbytes[i];
      const uint64_t nw = nbytes[i] / 8;
      recs.push_back({(uint64_t)(uintptr_t)dst[i], nw, nr, keys[i], tiles});
      tiles += (nw + kFillTile - 1) / kFillTile;
    }
    if (recs.empty()) return PYRIT_OK;
    if (recs.size() > 0xFFFFFFFFull) return PYRIT_EINVAL;
    hipStream_t st = (hipStream_t)stream;
    const size_t bytes = recs.size() * sizeof(FillRec);
    void *table = nullptr;
    if (hipMalloc(&table, bytes) != hipSuccess) return PYRIT_ENOMEM;
    int rc = PYRIT_OK;
    if (hipMemcpyAsync(table, recs.data(), bytes, hipMemcpyHostToDevice, st) != hipSuccess) {
      rc = PYRIT_EHIP;
    } else {
      const uint64_t grid = std::min<uint64_t>(tiles, 256ull * 32);
      hipLaunchKernelGGL(fill_blocks_kernel, dim3((unsigned)grid), dim3(256), 0, st,
                         (const FillRec *)table, (uint32_t)recs.size(), tiles);
      if (hipGetLastError() != hipSuccess) rc = PYRIT_EHIP;
    }
    // the table (and the host records the copy reads) must outlive the work
    if (hipStreamSynchronize(st) != hipSuccess && rc == PYRIT_OK) rc = PYRIT_EHIP;
    (void)hipFree(table);
    return rc;
  });
}

int pyrit_copy(uint8_t *dst, const uint8_t *src, size_t nbytes, void *stream) {
  if (!dst || !src || nbytes % 16 != 0 || ((uintptr_t)dst & 15u) || ((uintptr_t)src & 15u))
    return PYRIT_EINVAL;
  if (nbytes == 0) return PYRIT_OK;
  const uint64_t steps = (nbytes + kCopyStep - 1) / kCopyStep;  // one per wave
  const uint64_t wgs = std::min<uint64_t>((steps + 3) / 4, 256ull * 8);
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)wgs), dim3(256), 0, (hipStream_t)stream, dst,
                     src, (uint64_t)nbytes);
  return hipGetLastError() == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

}  // extern "C"
