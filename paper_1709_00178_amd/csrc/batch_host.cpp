// Host side of the batched form: resolving batch items into passes and work
// items, the executors' queue layouts, the device image of a batch, and the
// pyrit_batch_* entry points.  The kernels are in batch.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <queue>
#include <vector>

#include "batch_abi.hpp"
#include "batch_host.hpp"
#include "internal.hpp"

using namespace pyrit;

namespace {

struct HostPass {
  std::vector<uint64_t> in, out;
  std::vector<uint32_t> lift;  // k x kMaxOut
  uint32_t k, nout, S, pitch, w;
  int ring;
};

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Resolve one batch item into passes of at most batch_max_out outputs.
int item_passes(const pyrit_batch_item &it, std::vector<HostPass> *out, uint64_t *moved) {
  const pyrit_plan *pl = it.plan;
  if (!pl || !it.blocks) return PYRIT_EINVAL;
  if (pl->ring < 0) return PYRIT_EUNSUPPORTED;
  size_t pitch = it.slice_pitch;
  int rc = check_slices(pl->w, it.slice_bytes, &pitch);
  if (rc) return rc;
  std::vector<int> ins, outs;
  const uint32_t *coef = nullptr;  // coefficient words (coef_words), outputs x k
  std::shared_ptr<const DecodeEntry> ent;
  if (it.n_erased == 0) {
    for (int j = 0; j < pl->k; ++j) ins.push_back(j);
    for (int i = 0; i < pl->m; ++i) outs.push_back(pl->k + i);
    coef = pl->K.data();
  } else {
    rc = decode_entry(pl, it.erased, it.n_erased, &ent);
    if (rc) return rc;
    ins = ent->surv;
    outs = ent->outs;
    coef = ent->K.data();
  }
  for (int b : ins) {
    if (!it.blocks[b]) return PYRIT_EINVAL;
    if ((uintptr_t)it.blocks[b] & 15u) return PYRIT_EALIGN;
  }
  for (int b : outs) {
    if (!it.blocks[b]) return PYRIT_EINVAL;
    if ((uintptr_t)it.blocks[b] & 15u) return PYRIT_EALIGN;
  }
  const int nout = (int)outs.size();
  const int per_pass = batch_max_out(pl->ring);
  for (int r0 = 0; r0 < nout; r0 += per_pass) {
    HostPass hp;
    hp.k = (uint32_t)pl->k;
    hp.S = (uint32_t)it.slice_bytes;
    hp.pitch = (uint32_t)pitch;
    hp.w = (uint32_t)pl->w;
    hp.ring = pl->ring;
    hp.nout = (uint32_t)std::min(per_pass, nout - r0);
    for (int b : ins) hp.in.push_back((uint64_t)(uintptr_t)it.blocks[b]);
    for (uint32_t r = 0; r < hp.nout; ++r) hp.out.push_back((uint64_t)(uintptr_t)it.blocks[outs[r0 + r]]);
    hp.lift.assign((size_t)pl->k * kMaxOut, 0);
    for (int j = 0; j < pl->k; ++j)
      for (uint32_t r = 0; r < hp.nout; ++r)
        hp.lift[(size_t)j * kMaxOut + r] = coef[(size_t)(r0 + r) * pl->k + j];
    *moved += (uint64_t)(pl->k + hp.nout) * pl->w * it.slice_bytes;
    out->push_back(std::move(hp));
  }
  return PYRIT_OK;
}

// Bytes an item moves, plus a fixed per-item charge for its start-up.
uint64_t item_cost(const HostPass &hp, const WorkItem &wi) {
  return (uint64_t)(hp.k + hp.nout) * hp.w * (wi.col1 - wi.col0) + (uint64_t)hp.k * hp.w * 1024u;
}


}  // namespace

namespace pyrit {

int batch_check_tune(pyrit_tune *t) {
  if (t->mode < 0 || t->mode > 2 || t->tile_bytes < 0 || t->grid < 0) return PYRIT_EINVAL;
  if (t->xcd_order != 0 && t->xcd_order != 1) return PYRIT_EINVAL;
  if (t->wg_threads == 0) t->wg_threads = 128;
  if (t->wg_threads != 64 && t->wg_threads != 128 && t->wg_threads != 256) return PYRIT_EINVAL;
  if (t->split_k < 0 || t->split_k > 2) return PYRIT_EINVAL;
  if (t->split_k == 0) t->split_k = (t->mode == kModeGrid && t->wg_threads == 128) ? 2 : 1;
  if (t->split_k == 2 && (t->mode != kModeGrid || t->wg_threads == 64)) return PYRIT_EINVAL;
  return PYRIT_OK;
}

int batch_resident_grid(const pyrit_tune &t, int *grid) {
  int dev = 0, ncu = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PYRIT_EHIP;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return PYRIT_EHIP;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel_fn(t.mode, t.wg_threads, 0, 1),
                                                   t.wg_threads, 0) != hipSuccess)
    return PYRIT_EHIP;
  int g = t.grid ? t.grid : std::max(1, per_cu * ncu);
  // every sub-queue needs at least one workgroup to drain it
  if (t.mode == kModeQueue) g = std::max(g, kGroups);
  *grid = g;
  return PYRIT_OK;
}

int build_batch_image(const pyrit_batch_item *items, int n_items, const pyrit_tune &t,
                      int resident_grid, uint64_t dev_base, BatchImage *bi) {
  std::vector<HostPass> passes;
  bi->moved = 0;
  for (int i = 0; i < n_items; ++i) {
    int rc = item_passes(items[i], &passes, &bi->moved);
    if (rc) return rc;
  }
  const uint32_t wpw = (uint32_t)t.wg_threads / 64;
  const bool persistent = t.mode != kModeGrid;
  const int grid = persistent ? resident_grid : 0;
  const uint32_t total_waves = persistent ? (uint32_t)grid * wpw : 0u;

  // Work items.  grid mode: one item per workgroup, one chunk per wave (per
  // split-K pair), the
  // passes in ring order so each ring's workgroups are dispatched together.
  // persistent modes: tiles of several chunks, enough for every wave to take
  // a few, at most 64 KiB of columns.
  if (!persistent)
    std::stable_sort(passes.begin(), passes.end(),
                     [](const HostPass &x, const HostPass &y) { return x.ring < y.ring; });
  uint64_t cols = 0;
  for (auto &hp : passes) cols += hp.S;
  std::vector<WorkItem> work;
  for (size_t pi = 0; pi < passes.size(); ++pi) {
    const HostPass &hp = passes[pi];
    const uint32_t chunk = chunk_bytes(hp.ring);
    uint64_t T;
    if (!persistent) {
      T = (uint64_t)chunk * (wpw / (uint32_t)t.split_k);
    } else {
      T = t.tile_bytes ? (uint64_t)t.tile_bytes : cols / ((uint64_t)total_waves * 4 + 1);
      T = align_up(std::max<uint64_t>(chunk, std::min<uint64_t>(T, 65536)), chunk);
    }
    const uint32_t end = (uint32_t)align_up(hp.S, chunk);
    for (uint64_t c = 0; c < end; c += T)
      work.push_back({(uint32_t)pi, (uint32_t)c, (uint32_t)std::min<uint64_t>(c + T, end),
                      (uint32_t)hp.ring});
  }
  // Ring-major order keeps one ring's code hot in each CU's instruction
  // cache; within a ring, tiles stay in stripe order.
  std::stable_sort(work.begin(), work.end(),
                   [](const WorkItem &x, const WorkItem &y) { return x.ring < y.ring; });

  std::vector<uint32_t> starts;
  if (t.mode == kModeQueue) {
    // sub-queue g takes items g, g + kGroups, ... (each stays ring-major)
    std::vector<WorkItem> reord;
    reord.reserve(work.size());
    starts.push_back(0);
    for (int g = 0; g < kGroups; ++g) {
      for (size_t i = g; i < work.size(); i += kGroups) reord.push_back(work[i]);
      starts.push_back((uint32_t)reord.size());
    }
    work.swap(reord);
  } else if (t.mode == kModeStatic) {
    // longest item first onto the least-loaded wave
    std::vector<uint32_t> order(work.size());
    for (size_t i = 0; i < order.size(); ++i) order[i] = (uint32_t)i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
      return item_cost(passes[work[x].pass], work[x]) > item_cost(passes[work[y].pass], work[y]);
    });
    typedef std::pair<uint64_t, uint32_t> LW;
    std::priority_queue<LW, std::vector<LW>, std::greater<LW>> heap;
    for (uint32_t w = 0; w < total_waves; ++w) heap.push({0, w});
    std::vector<std::vector<uint32_t>> lists(total_waves);
    for (uint32_t i : order) {
      LW top = heap.top();
      heap.pop();
      lists[top.second].push_back(i);
      heap.push({top.first + item_cost(passes[work[i].pass], work[i]), top.second});
    }
    std::vector<WorkItem> reord;
    reord.reserve(work.size());
    starts.push_back(0);
    for (auto &ls : lists) {
      std::sort(ls.begin(), ls.end());  // ring-major, stripe order within a wave
      for (uint32_t i : ls) reord.push_back(work[i]);
      starts.push_back((uint32_t)reord.size());
    }
    work.swap(reord);
  } else {
    // start index of each pass's items (items are in pass order)
    starts.assign(passes.size() + 1, (uint32_t)work.size());
    for (size_t i = work.size(); i-- > 0;) starts[work[i].pass] = (uint32_t)i;
  }
  // grid mode with XCD order: eight contiguous ranges of equal bytes moved
  bi->xcd_start.assign(kXcds + 1, (uint32_t)work.size());
  bi->xcd_start[0] = 0;
  bi->xcd_bytes.assign(kXcds, 0);
  uint32_t longest = 0;
  if (!persistent && t.xcd_order) {
    auto cost = [&](const WorkItem &it) {
      const HostPass &hp = passes[it.pass];
      const uint64_t c1 = std::min<uint64_t>(it.col1, hp.S);
      return (uint64_t)(hp.k + hp.nout) * hp.w * (c1 > it.col0 ? c1 - it.col0 : 0);
    };
    uint64_t total = 0;
    for (const WorkItem &it : work) total += cost(it);
    uint64_t acc = 0;
    uint32_t x = 1;
    for (size_t i = 0; i < work.size(); ++i) {
      while (x < kXcds && acc * kXcds >= total * x) bi->xcd_start[x++] = (uint32_t)i;
      acc += cost(work[i]);
    }
    for (uint32_t y = 0; y < kXcds; ++y) {
      longest = std::max(longest, bi->xcd_start[y + 1] - bi->xcd_start[y]);
      for (uint32_t i = bi->xcd_start[y]; i < bi->xcd_start[y + 1]; ++i)
        bi->xcd_bytes[y] += cost(work[i]);
    }
  }

  // Image: counters | starts | passes | items | pointer and lift tables.
  bi->off_start = (size_t)kGroups * 64;
  bi->off_pass = align_up(bi->off_start + starts.size() * 4, 256);
  // grid mode derives each workgroup's item from the pass start indices, so
  // its image carries no item records
  const size_t n_item_recs = persistent ? work.size() : 0;
  bi->off_item = align_up(bi->off_pass + passes.size() * sizeof(PassDesc), 256);
  const size_t off_tab = align_up(bi->off_item + n_item_recs * sizeof(WorkItem), 256);
  size_t tab_bytes = 0;
  for (auto &hp : passes)
    tab_bytes += align_up(hp.in.size() * 8, 16) + align_up(hp.out.size() * 8, 16) + hp.lift.size() * 4;
  const size_t total = align_up(off_tab + tab_bytes, 256);
  bi->img.assign(total, 0);
  size_t cur = off_tab;
  for (size_t pi = 0; pi < passes.size(); ++pi) {
    const HostPass &hp = passes[pi];
    PassDesc d{};
    d.k = hp.k;
    d.nout = hp.nout;
    d.S = hp.S;
    d.pitch = hp.pitch;
    d.ring = (uint32_t)hp.ring;
    d.in_tab = dev_base + cur;
    std::memcpy(&bi->img[cur], hp.in.data(), hp.in.size() * 8);
    cur += align_up(hp.in.size() * 8, 16);
    d.out_tab = dev_base + cur;
    std::memcpy(&bi->img[cur], hp.out.data(), hp.out.size() * 8);
    cur += align_up(hp.out.size() * 8, 16);
    d.lift_tab = dev_base + cur;
    std::memcpy(&bi->img[cur], hp.lift.data(), hp.lift.size() * 4);
    cur += hp.lift.size() * 4;
    std::memcpy(&bi->img[bi->off_pass + pi * sizeof(PassDesc)], &d, sizeof(d));
  }
  if (!starts.empty()) std::memcpy(&bi->img[bi->off_start], starts.data(), starts.size() * 4);
  if (n_item_recs) std::memcpy(&bi->img[bi->off_item], work.data(), n_item_recs * sizeof(WorkItem));
  bi->n_items = (uint32_t)work.size();
  bi->n_passes = (uint32_t)passes.size();
  bi->total_waves = total_waves;
  bi->mode = t.mode;
  bi->wg = t.wg_threads;
  bi->xcd_order = t.xcd_order;
  bi->split = t.split_k;
  // The dispatch packet counts the grid in threads, in 32 bits.
  const uint64_t wgs = persistent ? (uint64_t)grid : t.xcd_order ? (uint64_t)kXcds * longest : work.size();
  if (wgs * (uint64_t)t.wg_threads > 0xFFFFFFFFull) return PYRIT_EINVAL;
  bi->grid = (int)wgs;
  return PYRIT_OK;
}

static BatchArgs image_args(const BatchImage &bi, void *dev) {
  BatchArgs a{};
  a.counters = (uint64_t *)dev;
  a.starts = (const uint32_t *)((uint8_t *)dev + bi.off_start);
  a.passes = (const PassDesc *)((uint8_t *)dev + bi.off_pass);
  a.items = (const WorkItem *)((uint8_t *)dev + bi.off_item);
  a.n_items = bi.n_items;
  a.total_waves = bi.total_waves;
  a.n_passes = bi.n_passes;
  for (uint32_t x = 0; x <= kXcds; ++x) a.xcd_start[x] = bi.xcd_start[x];
  return a;
}

int launch_batch_image(const BatchImage &bi, void *dev, void *stream) {
  if (bi.n_items == 0) return PYRIT_OK;
  BatchArgs a = image_args(bi, dev);
  void *kargs[] = {&a};
  return hipLaunchKernel(kernel_fn(bi.mode, bi.wg, bi.xcd_order, bi.split), dim3(bi.grid), dim3(bi.wg), kargs, 0,
                         (hipStream_t)stream) == hipSuccess
             ? PYRIT_OK
             : PYRIT_EHIP;
}

}  // namespace pyrit

struct pyrit_batch {
  void *dmem = nullptr;
  BatchImage bi;
  BatchArgs args{};
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~pyrit_batch() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (dmem) (void)hipFree(dmem);
  }
};

extern "C" {

int pyrit_batch_create(const pyrit_batch_item *items, int n_items, const pyrit_tune *tune,
                       pyrit_batch **out) {
  return abi_guard([&]() -> int {
    if (!out || n_items < 0 || (n_items > 0 && !items)) return PYRIT_EINVAL;
    *out = nullptr;
    pyrit_tune t{};
    if (tune) t = *tune;
    int rc = batch_check_tune(&t);
    if (rc) return rc;
    std::unique_ptr<pyrit_batch> b(new (std::nothrow) pyrit_batch());
    if (!b) return PYRIT_ENOMEM;
    // Validate the items before touching the device; the image embeds device
    // addresses, so it is built again once the allocation exists.
    BatchImage probe;
    rc = build_batch_image(items, n_items, t, 1, 0, &probe);
    if (rc) return rc;
    int grid = 0;
    if (t.mode != kModeGrid) {
      rc = batch_resident_grid(t, &grid);
      if (rc) return rc;
      rc = build_batch_image(items, n_items, t, grid, 0, &probe);
      if (rc) return rc;
    }
    if (hipMalloc(&b->dmem, probe.img.size()) != hipSuccess) return PYRIT_ENOMEM;
    rc = build_batch_image(items, n_items, t, grid, (uint64_t)(uintptr_t)b->dmem, &b->bi);
    if (rc) return rc;
    if (hipMemcpy(b->dmem, b->bi.img.data(), b->bi.img.size(), hipMemcpyHostToDevice) != hipSuccess)
      return PYRIT_EHIP;
    b->args = image_args(b->bi, b->dmem);
    if (b->bi.n_items == 0) {
      *out = b.release();
      return PYRIT_OK;
    }
    if (hipGraphCreate(&b->graph, 0) != hipSuccess) return PYRIT_EHIP;
    hipKernelNodeParams kp{};
    void *kargs[] = {&b->args};
    kp.func = const_cast<void *>(kernel_fn(b->bi.mode, b->bi.wg, b->bi.xcd_order, b->bi.split));
    kp.gridDim = dim3(b->bi.grid);
    kp.blockDim = dim3(b->bi.wg);
    kp.sharedMemBytes = 0;
    kp.kernelParams = kargs;
    kp.extra = nullptr;
    hipGraphNode_t node;
    if (hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kp) != hipSuccess) return PYRIT_EHIP;
    if (hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) return PYRIT_EHIP;
    *out = b.release();
    return PYRIT_OK;
  });
}

int pyrit_batch_launch(pyrit_batch *batch, void *stream) {
  if (!batch) return PYRIT_EINVAL;
  if (batch->bi.n_items == 0) return PYRIT_OK;
  return hipGraphLaunch(batch->exec, (hipStream_t)stream) == hipSuccess ? PYRIT_OK : PYRIT_EHIP;
}

int pyrit_batch_launch_direct(pyrit_batch *batch, void *stream) {
  if (!batch) return PYRIT_EINVAL;
  return launch_batch_image(batch->bi, batch->dmem, stream);
}

int pyrit_batch_info(const pyrit_batch *batch, int *n_passes, int *n_work_items,
                     uint64_t *moved_bytes, int *grid, int *wg_threads) {
  if (!batch) return PYRIT_EINVAL;
  if (n_passes) *n_passes = (int)batch->bi.n_passes;
  if (n_work_items) *n_work_items = (int)batch->bi.n_items;
  if (moved_bytes) *moved_bytes = batch->bi.moved;
  if (grid) *grid = batch->bi.grid;
  if (wg_threads) *wg_threads = batch->bi.wg;
  return PYRIT_OK;
}

void pyrit_batch_destroy(pyrit_batch *batch) { delete batch; }

int pyrit_batch_describe(const pyrit_batch_item *items, int n_items, const pyrit_tune *tune,
                         int *n_passes, int *n_work_items, uint64_t *moved_bytes, int *grid,
                         uint64_t *xcd_bytes) {
  return abi_guard([&]() -> int {
    if (n_items < 0 || (n_items > 0 && !items)) return PYRIT_EINVAL;
    pyrit_tune t{};
    if (tune) t = *tune;
    int rc = batch_check_tune(&t);
    if (rc) return rc;
    // the resident grid of the persistent modes is a device query: take it
    // from the caller instead
    if (t.mode != kModeGrid && t.grid <= 0) return PYRIT_EINVAL;
    const int resident = t.mode == kModeQueue ? std::max(t.grid, kGroups) : t.grid;
    BatchImage bi;
    rc = build_batch_image(items, n_items, t, t.mode == kModeGrid ? 0 : resident, 0, &bi);
    if (rc) return rc;
    if (n_passes) *n_passes = (int)bi.n_passes;
    if (n_work_items) *n_work_items = (int)bi.n_items;
    if (moved_bytes) *moved_bytes = bi.moved;
    if (grid) *grid = bi.grid;
    if (xcd_bytes)
      for (uint32_t x = 0; x < kXcds; ++x) xcd_bytes[x] = bi.xcd_bytes[x];
    return PYRIT_OK;
  });
}

}  // extern "C"
