// The batch builder (pyrit_batch_describe: passes, work items, executor
// queue layouts, XCD ranges, the device image) under AddressSanitizer and
// UndefinedBehaviorSanitizer, on seeded random batches mixing every kernel
// ring, both transforms, encodes and decodes, ragged and padded slices, with
// every executor.  Nothing touches a device: block addresses are plain
// integers and the kernel table is a stub.  Built and run by
// tests/test_native_sanitizers.py; prints "ok" and exits 0 when every check
// holds.
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "../../include/pyrit.h"

namespace pyrit {
// describe never launches; the kernel table lives in the device code
const void *kernel_fn(int, int, int, int) { return nullptr; }
}  // namespace pyrit

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

namespace {

uint64_t rng_state = 0x9E3779B97F4A7C15ull;
uint32_t rnd(uint32_t n) {  // xorshift64*, uniform enough for test shapes
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 33) % n;
}

struct Ring {
  int w, n;
  uint32_t p;
  int transform;
};

struct Stripe {
  pyrit_plan *plan;
  int w, k, m;
  std::vector<int> erased;
  std::vector<uint8_t *> blocks;
  size_t S, pitch;
};

}  // namespace

int main() {
  const Ring rings[] = {{4, 5, 0x1F, 0}, {8, 17, 0x139, 0}, {8, 17, 0x1D7, 0}, {10, 11, 0x7FF, 0},
                        {6, 9, 0x49, 0},  {4, 5, 0x1F, 1},   {10, 11, 0x7FF, 1}, {6, 9, 0x49, 1}};
  const int n_rings = (int)(sizeof(rings) / sizeof(rings[0]));
  uint64_t next_addr = 1ull << 36;
  for (int round = 0; round < 12; ++round) {
    const int n_items = round == 0 ? 1 : 1 + (int)rnd(300);
    std::vector<Stripe> st(n_items);
    std::vector<pyrit_batch_item> items(n_items);
    uint64_t want_moved = 0;
    int want_passes = 0;
    for (int i = 0; i < n_items; ++i) {
      Stripe &s = st[i];
      const Ring &r = rings[rnd(n_rings)];
      const int maxlen = r.w >= 8 ? 40 : (1 << r.w);
      s.w = r.w;
      s.k = 1 + (int)rnd(r.w == 4 ? 10 : 24);
      s.m = 1 + (int)rnd(9);
      if (s.k + s.m > maxlen) s.m = maxlen - s.k;
      std::vector<uint16_t> G((size_t)s.k * s.m);
      CHECK(pyrit_cauchy(r.w, r.p, s.k, s.m, G.data()) == PYRIT_OK);
      CHECK(pyrit_plan_create_ex(r.w, r.n, r.p, s.k, s.m, G.data(), r.transform, &s.plan) ==
            PYRIT_OK);
      s.S = 64 * (1 + rnd(rnd(2) ? 64 : 20000));
      s.pitch = rnd(3) == 0 ? 0 : s.S + 64 * rnd(80);
      const size_t pitch = s.pitch ? s.pitch : s.S;
      if (rnd(3) == 0) {  // a decode of 1..m distinct erasures
        const int e = 1 + (int)rnd((uint32_t)s.m);
        std::vector<int> ids(s.k + s.m);
        for (int b = 0; b < s.k + s.m; ++b) ids[b] = b;
        for (int b = 0; b < e; ++b) {
          const int j = b + (int)rnd((uint32_t)(s.k + s.m - b));
          const int t = ids[b];
          ids[b] = ids[j];
          ids[j] = t;
          s.erased.push_back(ids[b]);
        }
      }
      for (int b = 0; b < s.k + s.m; ++b) {
        s.blocks.push_back((uint8_t *)(uintptr_t)next_addr);
        next_addr += ((s.w - 1) * pitch + s.S + 4351) / 256 * 256;
      }
      const int outs = s.erased.empty() ? s.m : (int)s.erased.size();
      const int passes = (outs + 3) / 4;  // the batch kernels code four outputs per pass
      want_passes += passes;
      want_moved += (uint64_t)(passes * s.k + outs) * s.w * s.S;
      pyrit_batch_item &it = items[i];
      it.plan = s.plan;
      it.n_erased = (int)s.erased.size();
      it.erased = s.erased.empty() ? nullptr : s.erased.data();
      it.blocks = s.blocks.data();
      it.slice_bytes = s.S;
      it.slice_pitch = s.pitch;
    }
    struct Exec {
      int mode, wg, split, xcd, grid, tile;
    } const execs[] = {{0, 64, 1, 0, 0, 0},   {0, 64, 1, 1, 0, 0},   {0, 128, 1, 0, 0, 0},
                       {0, 128, 2, 0, 0, 0},  {0, 128, 2, 1, 0, 0},  {0, 256, 1, 1, 0, 0},
                       {0, 256, 2, 0, 0, 0},  {0, 256, 2, 1, 0, 0},  {1, 256, 1, 0, 1024, 0},
                       {1, 128, 1, 0, 3, 4096}, {2, 128, 1, 0, 512, 0}, {2, 64, 1, 0, 7, 512}};
    for (const Exec &e : execs) {
      pyrit_tune t{};
      t.mode = e.mode;
      t.wg_threads = e.wg;
      t.split_k = e.split;
      t.xcd_order = e.xcd;
      t.grid = e.grid;
      t.tile_bytes = e.tile;
      int np = 0, nw = 0, grid = 0;
      uint64_t moved = 0, xb[8] = {0};
      CHECK(pyrit_batch_describe(items.data(), n_items, &t, &np, &nw, &moved, &grid, xb) ==
            PYRIT_OK);
      CHECK(np == want_passes);
      CHECK(moved == want_moved);
      CHECK(nw >= np && grid > 0);
      uint64_t xs = 0;
      for (int x = 0; x < 8; ++x) xs += xb[x];
      CHECK(xs == ((e.mode == 0 && e.xcd) ? moved : 0));
      if (e.mode == 0 && !e.xcd) CHECK(grid == nw);
      if (e.mode == 0 && e.xcd) CHECK(grid % 8 == 0 && grid >= nw);
      if (e.mode != 0) CHECK(grid == (e.mode == 1 && e.grid < 8 ? 8 : e.grid));
    }
    for (Stripe &s : st) pyrit_plan_destroy(s.plan);
  }
  // empty batch, a misaligned block, an unknown executor
  pyrit_tune t{};
  int nw = -1;
  CHECK(pyrit_batch_describe(nullptr, 0, &t, nullptr, &nw, nullptr, nullptr, nullptr) == PYRIT_OK &&
        nw == 0);
  pyrit_plan *pl = nullptr;
  std::vector<uint16_t> G(8);
  CHECK(pyrit_cauchy(8, 0x139, 4, 2, G.data()) == PYRIT_OK);
  CHECK(pyrit_plan_create(8, 17, 0x139, 4, 2, G.data(), &pl) == PYRIT_OK);
  uint8_t *bl[6];
  for (int b = 0; b < 6; ++b) bl[b] = (uint8_t *)(uintptr_t)((1ull << 40) + (uint64_t)b * (1 << 20));
  bl[2] += 8;
  pyrit_batch_item it{pl, 0, nullptr, bl, 4096, 0};
  CHECK(pyrit_batch_describe(&it, 1, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        PYRIT_EALIGN);
  bl[2] -= 8;
  t.mode = 5;
  CHECK(pyrit_batch_describe(&it, 1, &t, nullptr, nullptr, nullptr, nullptr, nullptr) ==
        PYRIT_EINVAL);
  pyrit_plan_destroy(pl);
  std::printf("ok\n");
  return 0;
}
