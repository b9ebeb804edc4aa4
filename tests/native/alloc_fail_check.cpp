// No C++ exception crosses the C ABI, and a failed host allocation leaves
// nothing behind: every allocating host entry point is called with the
// global operator new made to fail at its 1st, 2nd, ... allocation until
// the call gets through.  Each failing call must return PYRIT_ENOMEM; the
// call that gets through must return PYRIT_OK with the same result as an
// undisturbed call.  Built with AddressSanitizer (leak checking on) and
// UndefinedBehaviorSanitizer by tests/test_native_sanitizers.py; prints "ok"
// and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "../../include/pyrit.h"

namespace pyrit {
const void *kernel_fn(int, int, int, int) { return nullptr; }
}  // namespace pyrit

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

// ---- the failing allocator: allocation number fail_at (1-based) fails
static long fail_at = 0, count = 0;
static bool fired = false, fired_nothrow = false;

static void *take(size_t n, bool nothrow) {
  if (fail_at && ++count == fail_at) {
    fired = true;
    fired_nothrow = nothrow;
    if (nothrow) return nullptr;
    throw std::bad_alloc();
  }
  void *p = std::malloc(n ? n : 1);
  if (!p && !nothrow) throw std::bad_alloc();
  return p;
}
void *operator new(size_t n) { return take(n, false); }
void *operator new[](size_t n) { return take(n, false); }
void *operator new(size_t n, const std::nothrow_t &) noexcept { return take(n, true); }
void *operator new[](size_t n, const std::nothrow_t &) noexcept { return take(n, true); }
void operator delete(void *p) noexcept { std::free(p); }
void operator delete[](void *p) noexcept { std::free(p); }
void operator delete(void *p, size_t) noexcept { std::free(p); }
void operator delete[](void *p, size_t) noexcept { std::free(p); }

// Run f() with allocation 1, 2, ... failing until it gets through.  Returns
// the number of failing runs.  A failed throwing allocation must make the
// call return PYRIT_ENOMEM.  A failed nothrow allocation may instead be
// absorbed by the standard library (std::stable_sort falls back to an
// in-place sort when it gets no temporary buffer), so there PYRIT_OK is
// accepted too; the caller checks the final result against an undisturbed
// call.
template <class F>
static int until_through(F f) {
  for (long n = 1;; ++n) {
    fail_at = n;
    count = 0;
    fired = fired_nothrow = false;
    const int rc = f();
    const bool hit = fired;
    fail_at = 0;
    if (!hit) {
      CHECK(rc == PYRIT_OK);
      return (int)(n - 1);
    }
    if (rc != PYRIT_ENOMEM && !(fired_nothrow && rc == PYRIT_OK))
      std::fprintf(stderr, "allocation %ld failed, call returned %d\n", n, rc);
    CHECK(rc == PYRIT_ENOMEM || (fired_nothrow && rc == PYRIT_OK));
  }
}

int main() {
  // lift tables: a ring not used before builds its table (allocations)
  uint32_t c_ref = 0, c = 0;
  {
    const int fails = until_through([&] { return pyrit_lift(10, 11, 0x7FF, 0x155, &c); });
    CHECK(fails >= 1);
    CHECK(pyrit_lift(10, 11, 0x7FF, 0x155, &c_ref) == PYRIT_OK && c == c_ref);
  }
  // plan creation, both transforms, a ring whose table is not cached yet
  for (int tr = 0; tr < 2; ++tr) {
    std::vector<uint16_t> G(4 * 12);
    CHECK(pyrit_cauchy(6, 0x49, 12, 4, G.data()) == PYRIT_OK);
    pyrit_plan *pl = nullptr;
    const int fails = until_through([&] {
      pyrit_plan *q = nullptr;
      const int rc = pyrit_plan_create_ex(6, 9, 0x49, 12, 4, G.data(), tr, &q);
      if (rc == PYRIT_OK) pl = q;
      else CHECK(q == nullptr);
      return rc;
    });
    CHECK(fails >= 1 && pl);
    int wt = 0;
    CHECK(pyrit_plan_weight(pl, &wt) == PYRIT_OK && wt > 0);
    // decoding matrices: the per-plan cache is filled only by a call that
    // gets through; the result equals that of a second, cached call
    const int er[3] = {0, 5, 13};
    std::vector<uint16_t> D(3 * 12), D2(3 * 12);
    int surv[12], surv2[12];
    CHECK(until_through([&] { return pyrit_decode_matrix(pl, er, 3, surv, D.data()); }) >= 1);
    CHECK(pyrit_decode_matrix(pl, er, 3, surv2, D2.data()) == PYRIT_OK);
    CHECK(std::memcmp(surv, surv2, sizeof(surv)) == 0 && D == D2);
    pyrit_plan_destroy(pl);
  }
  // the light Cauchy search
  {
    std::vector<uint16_t> G(4 * 10), G2(4 * 10);
    int w1 = 0, w2 = 0;
    CHECK(until_through([&] {
            return pyrit_cauchy_light(8, 17, 0x139, 10, 4, G.data(), nullptr, nullptr, &w1);
          }) >= 1);
    CHECK(pyrit_cauchy_light(8, 17, 0x139, 10, 4, G2.data(), nullptr, nullptr, &w2) == PYRIT_OK);
    CHECK(G == G2 && w1 == w2);
  }
  // the batch builder (host only), every executor
  {
    std::vector<uint16_t> G(3 * 5);
    CHECK(pyrit_cauchy(8, 0x139, 5, 3, G.data()) == PYRIT_OK);
    pyrit_plan *pl = nullptr;
    CHECK(pyrit_plan_create(8, 17, 0x139, 5, 3, G.data(), &pl) == PYRIT_OK);
    std::vector<uint8_t *> bl[3];
    for (int s = 0; s < 3; ++s)
      for (int b = 0; b < 8; ++b)
        bl[s].push_back((uint8_t *)(uintptr_t)((1ull << 40) + ((uint64_t)s * 8 + b) * (1 << 22)));
    const int er[2] = {1, 6};
    pyrit_batch_item items[3] = {{pl, 0, nullptr, bl[0].data(), 4096, 0},
                                 {pl, 2, er, bl[1].data(), 65536, 65536 + 256},
                                 {pl, 0, nullptr, bl[2].data(), 8192, 0}};
    const int modes[3][2] = {{0, 0}, {1, 64}, {2, 32}};
    for (const auto &md : modes) {
      pyrit_tune t{};
      t.mode = md[0];
      t.grid = md[1];
      int np = 0, nw = 0, np2 = 0, nw2 = 0;
      uint64_t mv = 0, mv2 = 0;
      CHECK(until_through([&] {
              return pyrit_batch_describe(items, 3, &t, &np, &nw, &mv, nullptr, nullptr);
            }) >= 1);
      CHECK(pyrit_batch_describe(items, 3, &t, &np2, &nw2, &mv2, nullptr, nullptr) == PYRIT_OK);
      CHECK(np == np2 && nw == nw2 && mv == mv2 && np > 0);
    }
    pyrit_plan_destroy(pl);
  }
  std::printf("ok\n");
  return 0;
}
