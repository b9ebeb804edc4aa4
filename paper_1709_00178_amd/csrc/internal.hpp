// Internal declarations shared by the host plan, the launchers and the C ABI.
#pragma once
#include <array>
#include <cstdint>
#include <memory>
#include <mutex>
#include <new>
#include <stdexcept>
#include <unordered_map>
#include <vector>

#include "../../include/pyrit.h"
#include "rings.hpp"

namespace pyrit {

// -1 when no kernel exists; transform: PYRIT_TRANSFORM_*
int ring_id(int w, int n, uint32_t p, int transform = PYRIT_TRANSFORM_EMBEDDING);

// Lanes' column width in bytes used when the caller does not choose.
int default_vec_bytes(int ring, int nout);

// Enqueue one pass (nout <= kMaxOut outputs) of the plain kernel.
int launch_pass(int ring, int nout, int vec_bytes, const PassArgs &a, void *stream);

struct DecodeEntry {
  std::vector<int> surv;      // k survivor block ids
  std::vector<int> outs;      // erased block ids, ascending
  std::vector<uint16_t> D;    // outs.size() x k decoding matrix
  std::vector<uint32_t> L;    // lifted D
  std::vector<uint32_t> K;    // kernel coefficient words of D (coef_words)
  int weight = 0;
};

// Coefficient words the kernels take for a matrix M (field elements) and its
// lifted form L: M itself on rings with ring_fused, else L.
std::vector<uint32_t> coef_words(int ring, const std::vector<uint16_t> &M,
                                 const std::vector<uint32_t> &L);

// Lifted representative of every field element of a ring (size 2^w).
const std::vector<uint32_t> &lift_table(int w, int n, uint32_t p);

// Runs the body of a C entry point so that no C++ exception crosses the C
// ABI: a failed host allocation becomes PYRIT_ENOMEM, anything else
// PYRIT_EINTERNAL.  Bodies hold their resources in RAII objects, so an
// exception leaves nothing behind.
template <class F>
int abi_guard(F &&body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc &) {
    return PYRIT_ENOMEM;
  } catch (const std::length_error &) {
    return PYRIT_ENOMEM;
  } catch (...) {
    return PYRIT_EINTERNAL;
  }
}

}  // namespace pyrit

struct pyrit_plan {
  int w = 0, n = 0;
  uint32_t p = 0;
  int k = 0, m = 0;
  int ring = -1;
  int transform = PYRIT_TRANSFORM_EMBEDDING;
  std::vector<uint16_t> G;  // m x k
  std::vector<uint32_t> L;  // m x k lifted
  std::vector<uint32_t> K;  // m x k kernel coefficient words (coef_words)
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

}  // namespace pyrit
