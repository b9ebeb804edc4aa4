// Batched form: one persistent kernel drains a queue of (pass, column-tile)
// work items covering many stripes of any supported ring, and the launch is
// captured once in a hipGraph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <vector>

#include "internal.hpp"
#include "ring_kernels.hpp"

namespace pyrit {

// Pointer to the constant address space: values read through it are wave
// uniform and immutable during the kernel, so they are fetched with scalar
// loads.
#define AS4 __attribute__((address_space(4)))

struct PassDesc {
  uint64_t in_tab;    // k input block pointers
  uint64_t out_tab;   // nout output block pointers
  uint64_t lift_tab;  // k x kMaxOut lifted coefficients (row j, column r)
  uint32_t k, nout, S, ring;
};

struct WorkItem {
  uint32_t pass, col0, col1, ring;
};

struct BatchArgs {
  const PassDesc *passes;
  const WorkItem *items;
  uint32_t *counters;  // [0] next item, [1] waves finished
  uint32_t n_items;
  uint32_t total_waves;
  uint32_t dynamic;
};

// Lane width per ring inside the batch kernel: the widest that keeps every
// ring at or below the (8,17) ring's register count (85 VGPRs at 4 outputs).
constexpr int kBatchV[kNumRings] = {2, 1, 1, 1, 1};

struct TableSrc {
  const AS4 uint64_t *in_tab;
  const AS4 uint64_t *out_tab;
  const AS4 uint32_t *lift_tab;
  int k_;
  uint32_t S_;
  int nout_;
  __device__ int k() const { return k_; }
  __device__ uint32_t S() const { return S_; }
  __device__ int nout() const { return nout_; }
  __device__ const uint8_t *in(int j) const { return (const uint8_t *)in_tab[j]; }
  __device__ uint8_t *out(int r) const { return (uint8_t *)out_tab[r]; }
  __device__ uint32_t lift(int j, int r) const { return lift_tab[j * kMaxOut + r]; }
};

template <int RING>
__device__ __forceinline__ void run_item(const AS4 PassDesc *pd, uint32_t col0, uint32_t col1,
                                         uint32_t lane) {
  constexpr RingDesc R = kRings[RING];
  constexpr int V = kBatchV[RING];
  const TableSrc src{(const AS4 uint64_t *)pd->in_tab, (const AS4 uint64_t *)pd->out_tab,
                     (const AS4 uint32_t *)pd->lift_tab, (int)pd->k, pd->S, (int)pd->nout};
  for (uint32_t c = col0; c < col1; c += 64u * 4u * V) {
    const uint32_t col = c + lane * 4u * V;
    dev::code_column<R.w, R.n, R.p, kMaxOut, V>(src, col, col < src.S());
  }
}

__device__ __forceinline__ uint32_t queue_fetch(uint32_t *counter, uint32_t lane) {
  uint32_t v = 0;
  if (lane == 0) v = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return v;
}

template <int WG>
__global__ __launch_bounds__(WG) void batch_kernel(const BatchArgs a) {
  const uint32_t lane = threadIdx.x & 63u;
  const uint32_t wave_id = __builtin_amdgcn_readfirstlane(blockIdx.x * (WG / 64) + (threadIdx.x >> 6));
  const AS4 WorkItem *items = (const AS4 WorkItem *)a.items;
  const AS4 PassDesc *passes = (const AS4 PassDesc *)a.passes;
  uint32_t item = a.dynamic ? __builtin_amdgcn_readfirstlane(queue_fetch(a.counters, lane)) : wave_id;
  while (item < a.n_items) {
    // Claim the next item before coding this one; the claim completes while
    // this item's first loads are in flight.
    const uint32_t next_v = a.dynamic ? queue_fetch(a.counters, lane) : 0u;
    const AS4 WorkItem *it = items + item;
    const AS4 PassDesc *pd = passes + it->pass;
    switch (it->ring) {
      case 0: run_item<0>(pd, it->col0, it->col1, lane); break;
      case 1: run_item<1>(pd, it->col0, it->col1, lane); break;
      case 2: run_item<2>(pd, it->col0, it->col1, lane); break;
      case 3: run_item<3>(pd, it->col0, it->col1, lane); break;
      case 4: run_item<4>(pd, it->col0, it->col1, lane); break;
      default: break;
    }
    item = a.dynamic ? __builtin_amdgcn_readfirstlane(next_v) : item + a.total_waves;
  }
  if (a.dynamic && lane == 0) {
    // The last wave to finish rewinds the queue for the next launch.
    const uint32_t done =
        __hip_atomic_fetch_add(&a.counters[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (done == a.total_waves - 1) {
      __hip_atomic_store(&a.counters[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.counters[1], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

static const void *batch_kernel_fn(int wg) {
  switch (wg) {
    case 64: return (const void *)batch_kernel<64>;
    case 128: return (const void *)batch_kernel<128>;
    case 256: return (const void *)batch_kernel<256>;
    default: return nullptr;
  }
}

}  // namespace pyrit

using namespace pyrit;

struct pyrit_batch {
  void *dmem = nullptr;
  BatchArgs args{};
  int grid = 0, wg = 256;
  int n_passes = 0;
  uint64_t moved = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~pyrit_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (dmem) (void)hipFree(dmem);
  }
};

namespace {

struct HostPass {
  std::vector<uint64_t> in, out;
  std::vector<uint32_t> lift;  // k x kMaxOut
  uint32_t k, nout, S;
  int ring;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Resolve one batch item into passes of at most kMaxOut outputs.
int item_passes(const pyrit_batch_item &it, std::vector<HostPass> *out, uint64_t *moved) {
  const pyrit_plan *pl = it.plan;
  if (!pl || !it.blocks) return PYRIT_EINVAL;
  if (pl->ring < 0) return PYRIT_EUNSUPPORTED;
  int rc = check_slices(pl->w, it.slice_bytes);
  if (rc) return rc;
  std::vector<int> ins, outs;
  const uint32_t *L = nullptr;
  std::shared_ptr<const DecodeEntry> ent;
  if (it.n_erased == 0) {
    for (int j = 0; j < pl->k; ++j) ins.push_back(j);
    for (int i = 0; i < pl->m; ++i) outs.push_back(pl->k + i);
    L = pl->L.data();
  } else {
    rc = decode_entry(pl, it.erased, it.n_erased, &ent);
    if (rc) return rc;
    ins = ent->surv;
    outs = ent->outs;
    L = ent->L.data();
  }
  for (int b : ins)
    if (!it.blocks[b]) return PYRIT_EINVAL;
    else if ((uintptr_t)it.blocks[b] & 15u) return PYRIT_EALIGN;
  for (int b : outs)
    if (!it.blocks[b]) return PYRIT_EINVAL;
    else if ((uintptr_t)it.blocks[b] & 15u) return PYRIT_EALIGN;
  const int nout = (int)outs.size();
  for (int r0 = 0; r0 < nout; r0 += kMaxOut) {
    HostPass hp;
    hp.k = (uint32_t)pl->k;
    hp.S = (uint32_t)it.slice_bytes;
    hp.ring = pl->ring;
    hp.nout = (uint32_t)std::min(kMaxOut, nout - r0);
    for (int b : ins) hp.in.push_back((uint64_t)(uintptr_t)it.blocks[b]);
    for (uint32_t r = 0; r < hp.nout; ++r) hp.out.push_back((uint64_t)(uintptr_t)it.blocks[outs[r0 + r]]);
    hp.lift.assign((size_t)pl->k * kMaxOut, 0);
    for (int j = 0; j < pl->k; ++j)
      for (uint32_t r = 0; r < hp.nout; ++r)
        hp.lift[(size_t)j * kMaxOut + r] = L[(size_t)(r0 + r) * pl->k + j];
    *moved += (uint64_t)(pl->k + hp.nout) * pl->w * it.slice_bytes;
    out->push_back(std::move(hp));
  }
  return PYRIT_OK;
}

}  // namespace

extern "C" {

int pyrit_batch_create(const pyrit_batch_item *items, int n_items, const pyrit_tune *tune,
                       pyrit_batch **out) {
  if (!out || n_items < 0 || (n_items > 0 && !items)) return PYRIT_EINVAL;
  *out = nullptr;
  pyrit_tune t{};
  if (tune) t = *tune;
  if (t.wg_threads == 0) t.wg_threads = 256;
  if (!batch_kernel_fn(t.wg_threads)) return PYRIT_EINVAL;
  if (t.tile_bytes < 0 || t.grid < 0) return PYRIT_EINVAL;

  std::unique_ptr<pyrit_batch> b(new (std::nothrow) pyrit_batch());
  if (!b) return PYRIT_ENOMEM;
  std::vector<HostPass> passes;
  for (int i = 0; i < n_items; ++i) {
    int rc = item_passes(items[i], &passes, &b->moved);
    if (rc) return rc;
  }

  // Resident grid: as many workgroups as fit on every CU at once.
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PYRIT_EHIP;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return PYRIT_EHIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel_fn(t.wg_threads),
                                                   t.wg_threads, 0) != hipSuccess)
    return PYRIT_EHIP;
  const int grid = t.grid ? t.grid : std::max(1, per_cu * ncu);
  const uint32_t total_waves = (uint32_t)grid * (uint32_t)(t.wg_threads / 64);

  // Tile width: enough items for every wave to take several, at least one
  // wave-wide chunk, at most 64 KiB of columns.
  uint64_t cols = 0;
  for (auto &hp : passes) cols += hp.S;
  std::vector<WorkItem> work;
  for (size_t pi = 0; pi < passes.size(); ++pi) {
    const HostPass &hp = passes[pi];
    const uint32_t chunk = 64u * 4u * kBatchV[hp.ring];
    uint64_t T = t.tile_bytes ? (uint64_t)t.tile_bytes : cols / ((uint64_t)total_waves * 4 + 1);
    T = std::max<uint64_t>(chunk, std::min<uint64_t>(T, 65536));
    T = align_up(T, chunk);
    const uint32_t end = (uint32_t)align_up(hp.S, chunk);
    for (uint64_t c = 0; c < end; c += T)
      work.push_back({(uint32_t)pi, (uint32_t)c, (uint32_t)std::min<uint64_t>(c + T, end),
                      (uint32_t)hp.ring});
  }
  // Ring-major order keeps one ring's code hot in each CU's instruction cache;
  // within a ring, tiles stay in stripe order.
  std::stable_sort(work.begin(), work.end(),
                   [](const WorkItem &x, const WorkItem &y) { return x.ring < y.ring; });

  // Device image: counters | passes | items | pointer and lift tables.
  const size_t off_pass = 256;
  const size_t off_item = align_up(off_pass + passes.size() * sizeof(PassDesc), 256);
  size_t off_tab = align_up(off_item + work.size() * sizeof(WorkItem), 256);
  size_t tab_bytes = 0;
  for (auto &hp : passes)
    tab_bytes += align_up(hp.in.size() * 8, 16) + align_up(hp.out.size() * 8, 16) + hp.lift.size() * 4;
  const size_t total = align_up(off_tab + tab_bytes, 256);
  std::vector<uint8_t> img(total, 0);
  if (hipMalloc(&b->dmem, total) != hipSuccess) return PYRIT_ENOMEM;
  const uint64_t base = (uint64_t)(uintptr_t)b->dmem;
  size_t cur = off_tab;
  for (size_t pi = 0; pi < passes.size(); ++pi) {
    const HostPass &hp = passes[pi];
    PassDesc d{};
    d.k = hp.k;
    d.nout = hp.nout;
    d.S = hp.S;
    d.ring = (uint32_t)hp.ring;
    d.in_tab = base + cur;
    std::memcpy(&img[cur], hp.in.data(), hp.in.size() * 8);
    cur += align_up(hp.in.size() * 8, 16);
    d.out_tab = base + cur;
    std::memcpy(&img[cur], hp.out.data(), hp.out.size() * 8);
    cur += align_up(hp.out.size() * 8, 16);
    d.lift_tab = base + cur;
    std::memcpy(&img[cur], hp.lift.data(), hp.lift.size() * 4);
    cur += hp.lift.size() * 4;
    std::memcpy(&img[off_pass + pi * sizeof(PassDesc)], &d, sizeof(d));
  }
  if (!work.empty()) std::memcpy(&img[off_item], work.data(), work.size() * sizeof(WorkItem));
  if (hipMemcpy(b->dmem, img.data(), total, hipMemcpyHostToDevice) != hipSuccess) return PYRIT_EHIP;

  b->args.counters = (uint32_t *)b->dmem;
  b->args.passes = (const PassDesc *)((uint8_t *)b->dmem + off_pass);
  b->args.items = (const WorkItem *)((uint8_t *)b->dmem + off_item);
  b->args.n_items = (uint32_t)work.size();
  b->args.total_waves = total_waves;
  b->args.dynamic = t.static_queue ? 0u : 1u;
  b->grid = grid;
  b->wg = t.wg_threads;
  b->n_passes = (int)passes.size();

  if (hipGraphCreate(&b->graph, 0) != hipSuccess) return PYRIT_EHIP;
  hipKernelNodeParams kp{};
  void *kargs[] = {&b->args};
  kp.func = const_cast<void *>(batch_kernel_fn(b->wg));
  kp.gridDim = dim3(b->grid);
  kp.blockDim = dim3(b->wg);
  kp.sharedMemBytes = 0;
  kp.kernelParams = kargs;
  kp.extra = nullptr;
  hipGraphNode_t node;
  if (hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kp) != hipSuccess) return PYRIT_EHIP;
  if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return PYRIT_EHIP;
  *out = b.release();
  return PYRIT_OK;
}

int pyrit_batch_launch(pyrit_batch *batch, void *stream) {
  if (!batch) return PYRIT_EINVAL;
  if (batch->args.n_items == 0) return PYRIT_OK;
  return hipGraphLaunch(batch->exec, (hipStream_t)stream) == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

int pyrit_batch_launch_direct(pyrit_batch *batch, void *stream) {
  if (!batch) return PYRIT_EINVAL;
  if (batch->args.n_items == 0) return PYRIT_OK;
  void *kargs[] = {&batch->args};
  return hipLaunchKernel(batch_kernel_fn(batch->wg), dim3(batch->grid), dim3(batch->wg), kargs, 0,
                         (hipStream_t)stream) == hipSuccess
             ? PYRIT_OK
             : PYRIT_EHIP;
}

int pyrit_batch_info(const pyrit_batch *batch, int *n_passes, int *n_work_items,
                     uint64_t *moved_bytes, int *grid, int *wg_threads) {
  if (!batch) return PYRIT_EINVAL;
  if (n_passes) *n_passes = batch->n_passes;
  if (n_work_items) *n_work_items = (int)batch->args.n_items;
  if (moved_bytes) *moved_bytes = batch->moved;
  if (grid) *grid = batch->grid;
  if (wg_threads) *wg_threads = batch->wg;
  return PYRIT_OK;
}

void pyrit_batch_destroy(pyrit_batch *batch) { delete batch; }

}  // extern "C"
