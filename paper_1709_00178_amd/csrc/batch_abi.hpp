// Layout shared by the batch kernels and the host that builds their work:
// pass descriptors, work items, kernel arguments, and the per-ring pass
// width and lane width of the batch kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rings.hpp"

namespace pyrit {


constexpr int kGroups = 8;     // sub-queues (one per XCD-sized group of workgroups)
constexpr uint32_t kXcds = 8;  // XCDs of an MI355X

struct PassDesc {
  uint64_t in_tab;    // k input block pointers
  uint64_t out_tab;   // nout output block pointers
  uint64_t lift_tab;  // k x kMaxOut lifted coefficients (row j, column r)
  uint32_t k, nout, S, ring;
  uint32_t pitch, pad;  // slice stride
};

struct WorkItem {
  uint32_t pass, col0, col1, ring;
};

enum : uint32_t { kModeGrid = 0, kModeQueue = 1, kModeStatic = 2 };

struct BatchArgs {
  const PassDesc *passes;
  const WorkItem *items;
  const uint32_t *starts;  // queue: kGroups+1 sub-queue offsets; static: waves+1 list offsets
  uint64_t *counters;      // queue: kGroups claim counters, 64 bytes apart
  uint32_t n_items;
  uint32_t total_waves;
  uint32_t n_passes;
  // grid mode with XCD order: XCD x codes items [xcd_start[x], xcd_start[x+1])
  uint32_t xcd_start[kXcds + 1];
};

// Outputs per pass inside the batch kernels: four for every ring.  One kernel
// holds every ring, and its register count is the largest ring's; four
// outputs keep each ring near the (8,17) ring's count (about 88 VGPRs, five
// waves per SIMD), while wider passes would only pay off for codes with more
// than four parity blocks (the plain kernel takes those in wide passes).
constexpr int kBatchOut = 4;
constexpr int batch_max_out(int ring) {
  return ring_max_out(ring) < kBatchOut ? ring_max_out(ring) : kBatchOut;
}

// Lane width per ring inside the batch kernels: the widest that keeps every
// ring at or below that register count.
constexpr int kBatchV[kNumRings] = {2, 1, 1, 1, 1, 2, 1, 1};

// kBatchV packed four bits per ring, so a run-time ring id maps to its lane
// width with a shift instead of a table load.
constexpr uint32_t pack_batch_v() {
  uint32_t b = 0;
  for (int i = 0; i < kNumRings; ++i) b |= (uint32_t)kBatchV[i] << (4 * i);
  return b;
}
constexpr uint32_t kBatchVBits = pack_batch_v();

__host__ __device__ constexpr uint32_t chunk_bytes(int ring) {
  return 64u * 4u * ((kBatchVBits >> (4 * ring)) & 15u);
}

// The batch kernel for an executor (grid: wg 64/128/256, xcd_order 0/1,
// split 1, or 2 with wg 128; queue/static: wg 64/128/256), or nullptr.
const void *kernel_fn(int mode, int wg, int xcd_order, int split);

}  // namespace pyrit
