// Batched form: one launch codes a queue of (pass, column-tile) work items
// covering many stripes of any supported ring; the launch is a hipGraph.
//
// Three ways to drain the queue (pyrit_tune.mode):
//   grid   - one workgroup per item; the hardware dispatcher hands items to
//            CUs in queue order as slots free up.
//   queue  - persistent: a resident grid; each wave codes one item from a
//            static slot, then claims items from one of eight atomic
//            sub-queues (one per group of workgroups, so claims spread over
//            eight counters).  Every launch makes a known number of claims
//            per sub-queue, so the counters never need resetting: a claim's
//            position in the current launch is its value modulo that number.
//   static - persistent: the host assigns items to waves, longest first onto
//            the least-loaded wave; waves walk their own lists.
//
// This file holds the kernels; batch_host.cpp builds their work on the host.
#include <hip/hip_runtime.h>

#include "batch_abi.hpp"
#include "ring_kernels.hpp"

namespace pyrit {

// Pointer to the constant address space: values read through it are wave
// uniform and immutable during the kernel, so they are fetched with scalar
// loads.
#define AS4 __attribute__((address_space(4)))

struct TableSrc {
  const AS4 uint64_t *in_tab;
  const AS4 uint64_t *out_tab;
  const AS4 uint32_t *lift_tab;
  int k_;
  uint32_t S_;
  uint32_t pitch_;
  int nout_;
  __device__ int k() const { return k_; }
  __device__ uint32_t S() const { return S_; }
  __device__ uint32_t pitch() const { return pitch_; }
  __device__ int nout() const { return nout_; }
  __device__ const uint8_t *in(int j) const { return (const uint8_t *)in_tab[j]; }
  __device__ uint8_t *out(int r) const { return (uint8_t *)out_tab[r]; }
  __device__ uint32_t lift(int j, int r) const { return lift_tab[j * kMaxOut + r]; }
  __device__ dev::Lift8 lift8(int j) const {
    const AS4 dev::u32x4 *row = (const AS4 dev::u32x4 *)(lift_tab + j * kMaxOut);
    return dev::Lift8{row[0], row[1]};
  }
};

__device__ __forceinline__ TableSrc table_src(const PassDesc &d) {
  return TableSrc{(const AS4 uint64_t *)d.in_tab, (const AS4 uint64_t *)d.out_tab,
                  (const AS4 uint32_t *)d.lift_tab, (int)d.k, d.S, d.pitch, (int)d.nout};
}

// A register copy of a descriptor (field by field: a constant-address-space
// object has no implicit copy into a generic one).
__device__ __forceinline__ PassDesc load_desc(const AS4 PassDesc *p) {
  PassDesc d;
  d.in_tab = p->in_tab;
  d.out_tab = p->out_tab;
  d.lift_tab = p->lift_tab;
  d.k = p->k;
  d.nout = p->nout;
  d.S = p->S;
  d.ring = p->ring;
  d.pitch = p->pitch;
  d.pad = p->pad;
  return d;
}

__device__ __forceinline__ TableSrc table_src(const AS4 PassDesc *pd) {
  return table_src(load_desc(pd));
}

template <int RING>
__device__ __forceinline__ void run_tile(const AS4 PassDesc *pd, uint32_t col0, uint32_t col1,
                                         uint32_t lane) {
  constexpr RingDesc R = kRings[RING];
  dev::code_tile<R.w, R.n, R.p, batch_max_out(RING), kBatchV[RING], R.parity>(table_src(pd), col0, col1, lane);
}

// LDS exchange of the split-K grid kernel, in dwords: the largest
// outputs x w x V over the rings, x 64 lanes.
constexpr int xch_dwords() {
  int m = 0;
  for (int i = 0; i < kNumRings; ++i) {
    const int x = batch_max_out(i) * kRings[i].w * kBatchV[i];
    m = x > m ? x : m;
  }
  return m * 64;
}

template <int RING, int KS>
__device__ __forceinline__ void run_chunk(const PassDesc &pd, uint32_t base, uint32_t lane,
                                          uint32_t part, uint32_t *xch) {
  constexpr RingDesc R = kRings[RING];
  constexpr int V = kBatchV[RING];
  typedef typename dev::Vec<V>::T T;
  const TableSrc src = table_src(pd);
  const uint32_t col = lane_col(base, lane, V);
  dev::code_column<R.w, R.n, R.p, batch_max_out(RING), V, KS, R.parity>(src, col, col < src.S(), part,
                                                                          (T *)xch);
}

__device__ __forceinline__ void code_item(const AS4 PassDesc *passes, const AS4 WorkItem *it,
                                          uint32_t lane) {
  const AS4 PassDesc *pd = passes + it->pass;
  const uint32_t c0 = it->col0, c1 = it->col1;
  switch (it->ring) {
    case 0: run_tile<0>(pd, c0, c1, lane); break;
    case 1: run_tile<1>(pd, c0, c1, lane); break;
    case 2: run_tile<2>(pd, c0, c1, lane); break;
    case 3: run_tile<3>(pd, c0, c1, lane); break;
    case 4: run_tile<4>(pd, c0, c1, lane); break;
    case 5: run_tile<5>(pd, c0, c1, lane); break;
    case 6: run_tile<6>(pd, c0, c1, lane); break;
    case 7: run_tile<7>(pd, c0, c1, lane); break;
    default: break;
  }
}

// grid mode: workgroup b codes item b, one chunk per wave (one per split-K
// pair of waves when KS = 2).  Items are
// numbered pass by pass, so the workgroup finds its pass by binary search
// over the per-pass start indices (a small array every workgroup reads, hot
// in the scalar cache) instead of loading a per-item record.
//
// The dispatcher deals workgroups round-robin over the XCDs (workgroup i to
// XCD i mod 8).  With XCD_ORDER the workgroup-to-item map is permuted so that
// each XCD walks its own contiguous range of the queue.  The host cuts the
// queue into eight ranges of equal bytes moved (items of different codes
// differ up to 10x in cost), and the grid holds eight times the longest
// range: workgroups past the end of their XCD's range leave at once.
//
// KS = 2 (split-K): each pair of waves shares one chunk, each wave coding
// every other input block (see code_column); a 256-thread workgroup holds
// two pairs on adjacent chunks.
template <int WG, bool XCD_ORDER, int KS>
__global__ __launch_bounds__(WG) void batch_grid_kernel(const BatchArgs a) {
  static_assert(KS == 1 || WG % (64 * KS) == 0, "split-K workgroups hold whole pairs");
  constexpr int kPairs = WG / 64 / KS;  // chunks per workgroup
  __shared__ __attribute__((aligned(16))) uint32_t xch[KS > 1 ? kPairs * xch_dwords() : 1];
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const AS4 uint32_t *starts = (const AS4 uint32_t *)a.starts;
  uint32_t b = blockIdx.x;
  if constexpr (XCD_ORDER) {
    const uint32_t x = b % kXcds, i = b / kXcds;
    const uint32_t first = a.xcd_start[x];
    if (i >= a.xcd_start[x + 1] - first) return;
    b = first + i;
  }
  uint32_t lo = 0, hi = a.n_passes;
  while (hi - lo > 1) {
    const uint32_t mid = (lo + hi) >> 1;
    if (starts[mid] <= b) lo = mid;
    else hi = mid;
  }
  // the whole descriptor and the pass's first item index in one round of
  // scalar loads
  const PassDesc pd = load_desc((const AS4 PassDesc *)a.passes + lo);
  const uint32_t first = starts[lo];
  const uint32_t ring = pd.ring;
  const uint32_t chunk = chunk_bytes(ring);
  const uint32_t base = grid_chunk_base(b - first, wave, kPairs, KS, chunk);
  const uint32_t part = wave % KS;
  // A workgroup's first chunk never starts past the end of its pass; a later
  // one may.  Such a chunk has nothing to code.  A split-K pair still meets
  // the one barrier the other pairs of its workgroup wait at.
  if constexpr (kPairs > 1) {
    if (base >= pd.S) {
      if constexpr (KS > 1) __syncthreads();
      return;
    }
  }
  uint32_t *px = xch + (KS > 1 ? (wave / KS) * xch_dwords() : 0);
  switch (ring) {
    case 0: run_chunk<0, KS>(pd, base, lane, part, px); break;
    case 1: run_chunk<1, KS>(pd, base, lane, part, px); break;
    case 2: run_chunk<2, KS>(pd, base, lane, part, px); break;
    case 3: run_chunk<3, KS>(pd, base, lane, part, px); break;
    case 4: run_chunk<4, KS>(pd, base, lane, part, px); break;
    case 5: run_chunk<5, KS>(pd, base, lane, part, px); break;
    case 6: run_chunk<6, KS>(pd, base, lane, part, px); break;
    case 7: run_chunk<7, KS>(pd, base, lane, part, px); break;
    default: break;
  }
}

__device__ __forceinline__ uint64_t claim(uint64_t *counter, uint32_t lane) {
  uint64_t v = 0;
  if (lane == 0) v = __hip_atomic_fetch_add(counter, (uint64_t)1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

__device__ __forceinline__ uint64_t first_lane64(uint64_t v) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

template <int WG, uint32_t MODE>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(5))) void batch_persistent_kernel(const BatchArgs a) {
  constexpr uint32_t wpw = WG / 64;  // waves per workgroup
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const AS4 WorkItem *items = (const AS4 WorkItem *)a.items;
  const AS4 PassDesc *passes = (const AS4 PassDesc *)a.passes;
  const AS4 uint32_t *starts = (const AS4 uint32_t *)a.starts;
  if constexpr (MODE == kModeStatic) {
    const uint32_t w = blockIdx.x * wpw + wave;
    const uint32_t e = starts[w + 1];
    for (uint32_t i = starts[w]; i < e; ++i) code_item(passes, items + i, lane);
  } else {
    const uint32_t g = blockIdx.x % kGroups;
    const uint32_t l = (blockIdx.x / kGroups) * wpw + wave;       // wave within its group
    const uint32_t wg_in_g = (gridDim.x - g + kGroups - 1) / kGroups;
    const uint32_t W_g = wg_in_g * wpw;                            // waves in the group
    const uint32_t q0 = starts[g], n_g = starts[g + 1] - q0;
    const uint32_t dyn = n_g > W_g ? n_g - W_g : 0u;               // items claimed dynamically
    const uint64_t C_g = (uint64_t)dyn + W_g;                      // claims per launch
    uint64_t *ctr = a.counters + g * 8;
    if (l < n_g) code_item(passes, items + q0 + l, lane);
    // Claims are made between items (holding a claim in flight across an
    // item would cost the registers of a sixth wave per SIMD).
    while (true) {
      const uint64_t pos = first_lane64(claim(ctr, lane)) % C_g;
      if (pos >= dyn) break;
      code_item(passes, items + q0 + W_g + (uint32_t)pos, lane);
    }
  }
}

static const void *grid_fn(int wg, bool xcd, int split) {
  if (split == 2) switch (wg) {
      case 128: return xcd ? (const void *)batch_grid_kernel<128, true, 2> : (const void *)batch_grid_kernel<128, false, 2>;
      case 256: return xcd ? (const void *)batch_grid_kernel<256, true, 2> : (const void *)batch_grid_kernel<256, false, 2>;
      default: return nullptr;
    }
  switch (wg) {
    case 64: return xcd ? (const void *)batch_grid_kernel<64, true, 1> : (const void *)batch_grid_kernel<64, false, 1>;
    case 128: return xcd ? (const void *)batch_grid_kernel<128, true, 1> : (const void *)batch_grid_kernel<128, false, 1>;
    case 256: return xcd ? (const void *)batch_grid_kernel<256, true, 1> : (const void *)batch_grid_kernel<256, false, 1>;
    default: return nullptr;
  }
}

static const void *persistent_fn(int wg, int mode) {
  if (mode == kModeQueue) switch (wg) {
      case 64: return (const void *)batch_persistent_kernel<64, kModeQueue>;
      case 128: return (const void *)batch_persistent_kernel<128, kModeQueue>;
      case 256: return (const void *)batch_persistent_kernel<256, kModeQueue>;
      default: return nullptr;
    }
  if (mode == kModeStatic) switch (wg) {
      case 64: return (const void *)batch_persistent_kernel<64, kModeStatic>;
      case 128: return (const void *)batch_persistent_kernel<128, kModeStatic>;
      case 256: return (const void *)batch_persistent_kernel<256, kModeStatic>;
      default: return nullptr;
    }
  return nullptr;
}

const void *kernel_fn(int mode, int wg, int xcd_order, int split) {
  return mode == kModeGrid ? grid_fn(wg, xcd_order != 0, split) : persistent_fn(wg, mode);
}

}  // namespace pyrit

// ------------------------------------------------------------------------
// A batch run without allocation (pyrit_batch_run_noalloc).  The batch image
// goes into `scratch`, a fixed array of device memory that every call on a
// GPU shares.  In host code `scratch` names a host-side stand-in, not the
// array: its device address is looked up once per GPU with
// hipGetSymbolAddress and only that address is handed to copies and kernels.

#include <mutex>

#include "batch_host.hpp"
#include "internal.hpp"

namespace pyrit {

static __device__ __align__(256) uint8_t scratch[PYRIT_SCRATCH_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kMaxDevices];  // the array's device address per GPU, once looked up

// Device address of the current GPU's scratch array (looked up on the first
// call on that GPU, with that GPU current).
int scratch_address(void **out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PYRIT_EHIP;
  if (dev < 0 || dev >= kMaxDevices) return PYRIT_EHIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PYRIT_EHIP;
    g_scratch_dev[dev] = p;
  }
  *out = g_scratch_dev[dev];
  return PYRIT_OK;
}

}  // namespace
}  // namespace pyrit

extern "C" int pyrit_batch_run_noalloc(const pyrit_batch_item *items, int n_items,
                                       const pyrit_tune *tune, void *stream) {
  using namespace pyrit;
  return abi_guard([&]() -> int {
    if (n_items < 0 || (n_items > 0 && !items)) return PYRIT_EINVAL;
    pyrit_tune t{};
    if (tune) t = *tune;
    int rc = batch_check_tune(&t);
    if (rc) return rc;
    int grid = 0;
    if (t.mode != kModeGrid) {
      rc = batch_resident_grid(t, &grid);
      if (rc) return rc;
    }
    // Under stream capture the copy below would become a graph node that
    // reads the host image after this call has released it.
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cap) != hipSuccess) return PYRIT_EHIP;
    if (cap != hipStreamCaptureStatusNone) return PYRIT_EINVAL;
    void *dev = nullptr;
    rc = scratch_address(&dev);
    if (rc) return rc;
    BatchImage bi;
    rc = build_batch_image(items, n_items, t, grid, (uint64_t)(uintptr_t)dev, &bi);
    if (rc) return rc;
    if (bi.n_items == 0) return PYRIT_OK;
    if (bi.img.size() > (size_t)PYRIT_SCRATCH_BYTES) return PYRIT_ETOOBIG;
    // From pageable host memory: the copy completes before hipMemcpyAsync
    // returns, so the host image may be released afterwards.  The image's
    // counter words are zero, which resets the queue counters of this run.
    if (hipMemcpyAsync(dev, bi.img.data(), bi.img.size(), hipMemcpyHostToDevice,
                       (hipStream_t)stream) != hipSuccess)
      return PYRIT_EHIP;
    return launch_batch_image(bi, dev, stream);
  });
}
