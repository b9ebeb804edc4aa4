// Internal declarations shared by the host plan, the launchers and the C ABI.
#pragma once
#include <array>
#include <cstdint>
#include <memory>
#include <mutex>
#include <unordered_map>
#include <vector>

#include "../../include/pyrit.h"

namespace pyrit {

// Outputs computed by one kernel pass: the accumulators of every output live
// in registers, so a pass covers at most this many output blocks (the bound
// of every per-pass array; each ring has its own limit, ring_max_out).
constexpr int kMaxOut = 8;

// Rings with a device kernel.  The kernels are templates on (w, n, p), so the
// reduction modulo p and every rotation index are compile-time constants.
// `parity` selects the parity transform (Sec. II-C.1, II-D.1) in place of the
// embedding transform (Sec. II-C.2, II-D.2): data enter the ring with n - w
// parity slices instead of zero slices, and results leave it by dropping
// those slices instead of reducing modulo p.
struct RingDesc {
  int w, n;
  uint32_t p;
  bool parity;
};
constexpr int kNumRings = 8;
constexpr RingDesc kRings[kNumRings] = {
    {4, 5, 0x1Fu, false},     // all-one polynomial of degree 4 (Sec. II-C)
    {8, 17, 0x139u, false},   // x^8+x^5+x^4+x^3+1, divides x^17+1
    {8, 17, 0x1D7u, false},   // x^8+x^7+x^6+x^4+x^2+x+1, the other factor
    {10, 11, 0x7FFu, false},  // all-one polynomial of degree 10
    {6, 9, 0x49u, false},     // equally spaced x^6+x^3+1 (Sec. II-D)
    {4, 5, 0x1Fu, true},      // the AOP and ESP rings again, parity transform
    {10, 11, 0x7FFu, true},
    {6, 9, 0x49u, true},
};
// Outputs per pass of a ring: outputs x n ring slices of accumulators stay
// near 70 registers per lane (4 for n = 17, 6 for n = 11, 8 for n <= 9).
constexpr int ring_max_out(int ring) {
  return kRings[ring].n <= 9 ? 8 : kRings[ring].n <= 11 ? 6 : 4;
}

// -1 when no kernel exists; transform: PYRIT_TRANSFORM_*
int ring_id(int w, int n, uint32_t p, int transform = PYRIT_TRANSFORM_EMBEDDING);

// Arguments of one coding pass: outputs out[r] (r < nout) are
// sum_j lift[j][r] (*) in[j] in the ring, reduced mod p.
struct PassArgs {
  const uint8_t *in[PYRIT_KMAX];
  uint8_t *out[kMaxOut];
  uint32_t lift[PYRIT_KMAX][kMaxOut];
  uint32_t k;
  uint32_t S;      // column bytes per slice
  uint32_t pitch;  // bytes from one slice to the next (>= S)
};

// Lanes' column width in bytes used when the caller does not choose.
int default_vec_bytes(int ring, int nout);

// Enqueue one pass (nout <= kMaxOut outputs) of the plain kernel.
int launch_pass(int ring, int nout, int vec_bytes, const PassArgs &a, void *stream);

struct DecodeEntry {
  std::vector<int> surv;      // k survivor block ids
  std::vector<int> outs;      // erased block ids, ascending
  std::vector<uint16_t> D;    // outs.size() x k decoding matrix
  std::vector<uint32_t> L;    // lifted D
  int weight = 0;
};

// Lifted representative of every field element of a ring (size 2^w).
const std::vector<uint32_t> &lift_table(int w, int n, uint32_t p);

}  // namespace pyrit

struct pyrit_plan {
  int w = 0, n = 0;
  uint32_t p = 0;
  int k = 0, m = 0;
  int ring = -1;
  int transform = PYRIT_TRANSFORM_EMBEDDING;
  std::vector<uint16_t> G;  // m x k
  std::vector<uint32_t> L;  // m x k lifted
  int weight = 0;
  mutable std::mutex mu;
  mutable std::unordered_map<std::string, std::shared_ptr<const pyrit::DecodeEntry>> dcache;
};

namespace pyrit {
// Decoding matrix for a pattern (cached on the plan).
int decode_entry(const pyrit_plan *plan, const int *erased, int n_erased,
                 std::shared_ptr<const DecodeEntry> *out);
// Validates slice size S and slice pitch (0 is replaced by S).
int check_slices(int w, size_t S, size_t *pitch);

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
