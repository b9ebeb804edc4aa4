// Host plan under AddressSanitizer and UndefinedBehaviorSanitizer: every
// kernel ring and a few rings without kernels, plans of several shapes and
// both transforms, every decoding matrix of small codes (also from several
// threads at once, sharing the plan's cache), the light Cauchy search and
// the error paths.  Built and run by tests/test_native_sanitizers.py; prints
// "ok" and exits 0 when every check holds.
#include <cstdio>
#include <cstdlib>
#include <thread>
#include <vector>

#include "../../include/pyrit.h"

#define CHECK(c)                                                     \
  do {                                                               \
    if (!(c)) {                                                      \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                  \
    }                                                                \
  } while (0)

struct Ring {
  int w, n;
  uint32_t p;
};

int main() {
  const Ring rings[] = {{4, 5, 0x1F}, {8, 17, 0x139}, {8, 17, 0x1D7}, {10, 11, 0x7FF}, {6, 9, 0x49},
                        {3, 7, 0xB}, {2, 3, 0x7}};
  for (const Ring &r : rings) {
    CHECK(pyrit_ring_check(r.w, r.n, r.p) == PYRIT_OK);
    for (uint32_t u = 0; u < (1u << r.w); ++u) {
      uint32_t c = 0, back = 0;
      CHECK(pyrit_lift(r.w, r.n, r.p, u, &c) == PYRIT_OK);
      CHECK(pyrit_ring_reduce(r.w, r.n, r.p, c, &back) == PYRIT_OK && back == u);
    }
    const int kmax = r.w >= 8 ? 16 : (1 << r.w) - 2;
    for (int k = 1; k <= kmax; k += 3)
      for (int m = 1; m <= 4 && k + m <= (1 << r.w); ++m)
        for (int tr = 0; tr < 2; ++tr) {
          pyrit_plan *pl = nullptr;
          std::vector<uint16_t> G((size_t)k * m);
          CHECK(pyrit_cauchy(r.w, r.p, k, m, G.data()) == PYRIT_OK);
          const int rc = pyrit_plan_create_ex(r.w, r.n, r.p, k, m, G.data(), tr, &pl);
          if (rc != PYRIT_OK) {
            if (!(tr == 1 || rc == PYRIT_ETOOLONG))
              std::fprintf(stderr, "w=%d n=%d p=%#x k=%d m=%d tr=%d rc=%d\n", r.w, r.n, r.p, k, m, tr, rc);
            CHECK(tr == 1 || rc == PYRIT_ETOOLONG);  // parity transform: AOP / ESP rings only
            continue;
          }
          std::vector<uint32_t> L((size_t)k * m);
          CHECK(pyrit_plan_lifted(pl, L.data()) == PYRIT_OK);
          int wt = 0;
          CHECK(pyrit_plan_weight(pl, &wt) == PYRIT_OK && wt > 0);
          // every decoding pattern of up to two erasures (k + m <= 20 blocks)
          std::vector<int> surv(k);
          std::vector<uint16_t> D(2 * (size_t)k);
          for (int a = 0; a < k + m; ++a) {
            int e1[1] = {a};
            CHECK(pyrit_decode_matrix(pl, e1, 1, surv.data(), D.data()) == PYRIT_OK);
            for (int b = a + 1; b < k + m && m >= 2; ++b) {
              int e2[2] = {a, b};
              CHECK(pyrit_decode_matrix(pl, e2, 2, surv.data(), D.data()) == PYRIT_OK);
            }
          }
          int too_many[5] = {0, 1, 2, 3, 4};
          if (m < 5) CHECK(pyrit_decode_matrix(pl, too_many, m + 1, nullptr, nullptr) != PYRIT_OK);
          pyrit_plan_destroy(pl);
        }
  }
  // one plan's decode cache filled from eight threads at once
  pyrit_plan *pl = nullptr;
  std::vector<uint16_t> G1(40);
  CHECK(pyrit_cauchy(8, 0x139, 10, 4, G1.data()) == PYRIT_OK);
  CHECK(pyrit_plan_create(8, 17, 0x139, 10, 4, G1.data(), &pl) == PYRIT_OK);
  std::vector<std::thread> th;
  for (int t = 0; t < 8; ++t)
    th.emplace_back([pl, t] {
      std::vector<int> surv(10);
      std::vector<uint16_t> D(40);
      for (int a = 0; a < 14; ++a)
        for (int b = a + 1; b < 14; ++b) {
          int e[3] = {a, b, (a + b + t) % 14};
          const int ne = (e[2] == a || e[2] == b) ? 2 : 3;
          CHECK(pyrit_decode_matrix(pl, e, ne, surv.data(), D.data()) == PYRIT_OK);
        }
    });
  for (auto &x : th) x.join();
  pyrit_plan_destroy(pl);
  // the light Cauchy search
  std::vector<uint16_t> G(40), rs(4), cs(10);
  int weight = 0;
  CHECK(pyrit_cauchy_light(8, 17, 0x139, 10, 4, G.data(), rs.data(), cs.data(), &weight) == PYRIT_OK);
  CHECK(weight > 0 && weight <= 92);
  // the point search (a wide GF(2^6) code and the GF(2^10) code)
  {
    std::vector<uint16_t> Gs(20 * 40), X(20), Y(40), r2(20), c2(40);
    int ws = 0;
    CHECK(pyrit_cauchy_search(6, 9, 0x49, 40, 20, 2, Gs.data(), X.data(), Y.data(), r2.data(),
                              c2.data(), &ws) == PYRIT_OK);
    CHECK(ws > 0);
    CHECK(pyrit_cauchy_search(10, 11, 0x7FF, 16, 4, 1, Gs.data(), nullptr, nullptr, nullptr,
                              nullptr, &ws) == PYRIT_OK);
    CHECK(pyrit_cauchy_search(10, 11, 0x7FF, 16, 4, -1, Gs.data(), nullptr, nullptr, nullptr,
                              nullptr, nullptr) == PYRIT_EINVAL);
  }
  // error paths
  CHECK(pyrit_ring_check(8, 16, 0x139) != PYRIT_OK);
  CHECK(pyrit_ring_check(8, 17, 0x13B) != PYRIT_OK);
  CHECK(pyrit_plan_create(8, 17, 0x139, 10, 4, nullptr, &pl) == PYRIT_EINVAL);
  CHECK(pyrit_plan_create(8, 17, 0x139, 0, 4, G1.data(), &pl) != PYRIT_OK);
  std::vector<uint16_t> G2(18 * 4, 1);
  CHECK(pyrit_plan_create(4, 5, 0x1F, 14, 4, G2.data(), &pl) == PYRIT_ETOOLONG);
  uint16_t bad[2] = {1, 300};
  CHECK(pyrit_plan_create(8, 17, 0x139, 2, 1, bad, &pl) == PYRIT_ERANGE);
  for (int code = 0; code >= -12; --code) CHECK(pyrit_strerror(code) != nullptr);
  std::printf("ok\n");
  return 0;
}
