// Host-side batch image, shared by the batch entry points and the request
// loop.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "../../include/pyrit.h"

namespace pyrit {

// Host image of a batch (work queue, pass descriptors, pointer and lift
// tables) laid out for a device buffer at a given address.
struct BatchImage {
  std::vector<uint8_t> img;
  size_t off_start = 0, off_pass = 0, off_item = 0;
  uint32_t n_items = 0, n_passes = 0, total_waves = 0;
  int grid = 0, wg = 128, mode = 0, xcd_order = 0, split = 1;
  uint64_t moved = 0;
  std::vector<uint32_t> xcd_start;  // grid mode with XCD order: per-XCD item ranges
  std::vector<uint64_t> xcd_bytes;  // bytes moved by each of those ranges
};
int batch_check_tune(pyrit_tune *t);
int batch_resident_grid(const pyrit_tune &t, int *grid);
int build_batch_image(const pyrit_batch_item *items, int n_items, const pyrit_tune &t,
                      int resident_grid, uint64_t dev_base, BatchImage *bi);
// Launch the batch kernel on an image already copied to `dev`.
int launch_batch_image(const BatchImage &bi, void *dev, void *stream);

}  // namespace pyrit
