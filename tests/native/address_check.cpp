// Address model of every load and store the coding kernels issue, checked on
// the host: the plain kernel (every lane width), the wide kernel (every ring
// and group count) and the batch kernel's executors (grid with and without
// split-K pairs and XCD order, queue, static), on seeded mixed batches with
// ragged and padded slices.  The work
// comes from the real batch builder (build_batch_image) and the column of
// every lane from the formulas the kernels use (rings.hpp, batch_abi.hpp).
//
// A lane reads the 4V bytes at voffset + soffset from the base of a block
// through a raw buffer descriptor of num_records bytes.  Whether the
// hardware adds soffset before comparing against num_records is not assumed:
// an access counts as issued when either reading lets it through, and every
// issued access must lie inside the block, [0, (w-1)*pitch + S).  Stores
// must lie inside the first S bytes of their slice.
//
// The model is also run with the old rule (dead lanes loading at their own
// column); it must then find an access past the end of a block, which shows
// the check can fail.  Built and run by tests/test_native_sanitizers.py;
// prints "ok" and exits 0 when every check holds.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "../../include/pyrit.h"
#include "../../paper_1709_00178_amd/csrc/batch_abi.hpp"
#include "../../paper_1709_00178_amd/csrc/batch_host.hpp"

namespace pyrit {
const void *kernel_fn(int, int, int, int) { return nullptr; }
}  // namespace pyrit

using namespace pyrit;

#define CHECK(c)                                                          \
  do {                                                                    \
    if (!(c)) {                                                           \
      std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
      std::exit(1);                                                       \
    }                                                                     \
  } while (0)

namespace {

uint64_t rng_state = 0x2545F4914F6CDD1Dull;
uint32_t rnd(uint32_t n) {
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 0x2545F4914F6CDD1Dull) >> 33) % n;
}

bool old_rule = false;  // dead lanes load at their own column
uint64_t violations = 0, loads = 0, stores = 0;

// One lane's loads of the w slices of one input block (bytes = the
// descriptor's record count: span, or 0 for the empty prefetch descriptor).
void lane_loads(uint32_t w, uint32_t S, uint32_t pitch, uint32_t V, uint32_t col,
                uint32_t bytes) {
  const uint32_t span = block_span(w, S, pitch);
  const uint32_t voff = old_rule ? col : lane_load_voffset(col, S);
  for (uint32_t t = 0; t < w; ++t) {
    const uint64_t soff = (uint64_t)t * pitch;
    const bool in_a = voff < bytes;                       // soffset not range checked
    const bool in_b = (uint64_t)voff + soff < bytes;      // soffset range checked
    if (!in_a && !in_b) continue;
    ++loads;
    const uint64_t at = (uint64_t)voff + soff;
    if (at + 4u * V > span) ++violations;
  }
}

void lane_stores(uint32_t w, uint32_t S, uint32_t pitch, uint32_t V, uint32_t col) {
  if (col >= S) return;  // the kernels store live lanes only
  for (uint32_t t = 0; t < w; ++t) {
    ++stores;
    CHECK(col + 4u * V <= S);
    CHECK((uint64_t)col + (uint64_t)t * pitch + 4u * V <= block_span(w, S, pitch));
  }
}

// A wave coding one chunk of one pass: every input block's loads (the next
// block's prefetch included; past the last block it uses an empty
// descriptor) and the stores of the outputs.
void wave_chunk(uint32_t w, uint32_t S, uint32_t pitch, uint32_t V, uint32_t k, uint32_t base) {
  const uint32_t span = block_span(w, S, pitch);
  for (uint32_t lane = 0; lane < 64; ++lane) {
    const uint32_t col = lane_col(base, lane, V);
    for (uint32_t j = 0; j <= k; ++j) lane_loads(w, S, pitch, V, col, j < k ? span : 0u);
    lane_stores(w, S, pitch, V, col);
  }
}

struct Desc {
  uint32_t k, nout, S, pitch, ring;
};

Desc pass_desc(const BatchImage &bi, uint32_t pi) {
  PassDesc d;
  std::memcpy(&d, &bi.img[bi.off_pass + (size_t)pi * sizeof(PassDesc)], sizeof(d));
  return {d.k, d.nout, d.S, d.pitch, d.ring};
}

uint32_t ring_v(uint32_t ring) { return chunk_bytes((int)ring) / 256u; }

// The grid kernel: workgroup b (after the XCD permutation) finds its pass
// by the start indices and each wave (or split-K pair) codes one chunk.
void walk_grid(const BatchImage &bi) {
  std::vector<uint32_t> starts(bi.n_passes + 1);
  std::memcpy(starts.data(), &bi.img[bi.off_start], starts.size() * 4);
  const uint32_t ks = (uint32_t)bi.split, pairs = (uint32_t)bi.wg / 64u / ks;
  std::vector<uint32_t> coded(bi.n_items, 0);
  for (uint32_t b0 = 0; b0 < (uint32_t)bi.grid; ++b0) {
    uint32_t b = b0;
    if (bi.xcd_order) {
      const uint32_t x = b0 % kXcds, i = b0 / kXcds;
      if (i >= bi.xcd_start[x + 1] - bi.xcd_start[x]) continue;
      b = bi.xcd_start[x] + i;
    }
    CHECK(b < bi.n_items);
    ++coded[b];
    const uint32_t pi =
        (uint32_t)(std::upper_bound(starts.begin(), starts.begin() + bi.n_passes, b) - starts.begin()) - 1;
    const Desc d = pass_desc(bi, pi);
    const uint32_t w = (uint32_t)kRings[d.ring].w, V = ring_v(d.ring);
    for (uint32_t wave = 0; wave < (uint32_t)bi.wg / 64u; wave += ks) {
      const uint32_t base = grid_chunk_base(b - starts[pi], wave, pairs, ks, chunk_bytes((int)d.ring));
      CHECK(wave > 0 || base < d.S);  // a workgroup's first chunk is never past its pass
      if (base >= d.S) continue;      // later ones may be; they code nothing
      wave_chunk(w, d.S, d.pitch, V, d.k, base);
    }
  }
  for (uint32_t c : coded) CHECK(c == 1);  // every item exactly once
}

// The persistent kernels: each item is a tile [col0, col1) of chunks coded by
// one wave as one load stream (code_tile).
void walk_items(const BatchImage &bi) {
  std::vector<WorkItem> items(bi.n_items);
  std::memcpy(items.data(), &bi.img[bi.off_item], items.size() * sizeof(WorkItem));
  for (const WorkItem &it : items) {
    const Desc d = pass_desc(bi, it.pass);
    const uint32_t w = (uint32_t)kRings[d.ring].w, V = ring_v(d.ring);
    const uint32_t chunk = chunk_bytes((int)d.ring);
    CHECK(it.ring == d.ring && it.col0 < d.S && it.col1 > it.col0 && it.col0 % chunk == 0);
    CHECK(it.col1 <= (d.S + chunk - 1) / chunk * chunk);
    for (uint32_t cb = it.col0; cb < it.col1; cb += chunk) wave_chunk(w, d.S, d.pitch, V, d.k, cb);
    // the prefetch past the tile's last chunk uses an empty descriptor
    for (uint32_t lane = 0; lane < 64; ++lane)
      lane_loads(w, d.S, d.pitch, V, lane_col(it.col1, lane, V), 0u);
  }
}

// The plain kernel: one workgroup per chunk of 64 lanes x 4V bytes, both
// waves of its split-K pair on the same columns.
void walk_plain(uint32_t w, uint32_t S, uint32_t pitch, uint32_t V, uint32_t k) {
  const uint32_t per_block = 64u * 4u * V;
  const uint32_t blocks = (S + per_block - 1) / per_block;
  for (uint32_t b = 0; b < blocks; ++b) wave_chunk(w, S, pitch, V, k, plain_chunk_base(b, V));
}

// The wide kernel (plain_impl.hpp, ring_kernels.hpp code_column_staged):
// workgroup b = G waves on the chunk of 64 lanes x 4 kWideV bytes at
// plain_chunk_base(b, kWideV); each wave issues NG dword loads per block,
// load q = g + u G (q < w kWideV: dword q mod kWideV of every lane of slice
// q / kWideV; past that, load q mod w kWideV again into the sink), each
// lane loading 4 bytes at voffset lane_load_voffset(col, S) plus soffset.
// Blocks are issued B at a time, through block roundup(k, B) + D - B - 1
// (those at or past k with an empty descriptor).  Besides the global
// addresses, every LDS target must lie in the stage ring plus sink of
// D w kWideV + 1 rows of 64 dwords.
void walk_wide(uint32_t w, uint32_t S, uint32_t pitch, uint32_t k, uint32_t D, uint32_t B) {
  const uint32_t V = (uint32_t)kWideV, kLoads = w * V;
  const uint32_t span = block_span(w, S, pitch);
  const uint32_t chunk = 64u * 4u * V;
  const uint32_t blocks = (S + chunk - 1) / chunk;
  for (uint32_t G = 2; G <= (uint32_t)kWideMaxGroups; ++G) {
    uint32_t NG = 1;
    while (NG * G < kLoads) NG *= 2;
    for (uint32_t b = 0; b < blocks; ++b)
      for (uint32_t g = 0; g < G; ++g)
        for (uint32_t lane = 0; lane < 64; ++lane) {
          const uint32_t col = lane_col(plain_chunk_base(b, V), lane, V);
          const uint32_t voff = old_rule ? col : lane_load_voffset(col, S);
          for (uint32_t u = 0; u < NG; ++u) {
            const uint32_t q = g + u * G;
            const uint32_t qq = q < kLoads ? q : q % kLoads;
            const uint64_t soff = (uint64_t)(qq / V) * pitch + (qq % V) * 4u;
            const uint32_t loff = q < kLoads ? q * 64u : D * kLoads * 64u;
            const uint32_t smask = q < kLoads ? 0xFFFFFFFFu : 0u;
            const uint32_t issued = (k + B - 1) / B * B + D - B;
            for (uint32_t jj = 0; jj < issued; ++jj) {
              const uint32_t slot = (jj & (D - 1)) * kLoads * 64u;
              CHECK((slot & smask) + loff + lane < (D * kLoads + 1) * 64u);  // LDS target
              const uint32_t bytes = jj < k ? span : 0u;
              const bool in_a = voff < bytes, in_b = (uint64_t)voff + soff < bytes;
              if (!in_a && !in_b) continue;
              ++loads;
              if ((uint64_t)voff + soff + 4u > span) ++violations;
            }
          }
          lane_stores(w, S, pitch, V, col);
        }
  }
}

struct Ring {
  int w, n;
  uint32_t p;
  int transform;
};

struct Stripe {
  pyrit_plan *plan;
  int k, m;
  std::vector<int> erased;
  std::vector<uint8_t *> blocks;
};

void run_model() {
  // plain kernel: every lane width, ragged and padded slices
  for (uint32_t V : {1u, 2u, 4u})
    for (uint32_t w : {4u, 6u, 8u, 10u})
      for (int trial = 0; trial < 40; ++trial) {
        const uint32_t S = 64u * (1u + rnd(trial < 20 ? 40 : 3000));
        const uint32_t pitch = rnd(2) ? S : S + 64u * rnd(70);
        walk_plain(w, S, pitch, V, 1 + rnd(4));
      }
  // wide kernel: every ring's slice count and stage depth, ragged and padded
  for (int ring = 0; ring < kNumRings; ++ring)
    for (int trial = 0; trial < 6; ++trial) {
      const uint32_t w = (uint32_t)kRings[ring].w;
      const uint32_t S = 64u * (1u + rnd(trial < 3 ? 12 : 100));
      const uint32_t pitch = rnd(2) ? S : S + 64u * rnd(70);
      walk_wide(w, S, pitch, 1 + rnd(5), (uint32_t)wide_stages(ring),
                (uint32_t)wide_blocks_per_barrier(ring));
    }
  const Ring rings[] = {{4, 5, 0x1F, 0}, {8, 17, 0x139, 0}, {8, 17, 0x1D7, 0}, {10, 11, 0x7FF, 0},
                        {6, 9, 0x49, 0},  {4, 5, 0x1F, 1},   {10, 11, 0x7FF, 1}, {6, 9, 0x49, 1}};
  uint64_t next_addr = 1ull << 36;
  for (int round = 0; round < 6; ++round) {
    const int n_items = 1 + (int)rnd(60);
    std::vector<Stripe> st(n_items);
    std::vector<pyrit_batch_item> items(n_items);
    for (int i = 0; i < n_items; ++i) {
      Stripe &s = st[i];
      const Ring &r = rings[rnd(8)];
      s.k = 1 + (int)rnd(r.w == 4 ? 10 : 12);
      s.m = 1 + (int)rnd(6);
      if (r.w == 4 && s.k + s.m > 16) s.m = 16 - s.k;
      std::vector<uint16_t> G((size_t)s.k * s.m);
      CHECK(pyrit_cauchy(r.w, r.p, s.k, s.m, G.data()) == PYRIT_OK);
      CHECK(pyrit_plan_create_ex(r.w, r.n, r.p, s.k, s.m, G.data(), r.transform, &s.plan) == PYRIT_OK);
      const size_t S = 64 * (1 + rnd(rnd(2) ? 40 : 3000));
      const size_t pitch = rnd(2) ? 0 : S + 64 * rnd(70);
      if (rnd(3) == 0) s.erased.push_back((int)rnd((uint32_t)(s.k + s.m)));
      for (int b = 0; b < s.k + s.m; ++b) {
        s.blocks.push_back((uint8_t *)(uintptr_t)next_addr);
        next_addr += ((r.w - 1) * (pitch ? pitch : S) + S + 4351) / 256 * 256;
      }
      items[i] = {s.plan, (int)s.erased.size(), s.erased.empty() ? nullptr : s.erased.data(),
                  s.blocks.data(), S, pitch};
    }
    struct Exec {
      int mode, wg, split, xcd, grid, tile;
    } const execs[] = {{0, 64, 1, 0, 0, 0},  {0, 128, 1, 1, 0, 0},  {0, 128, 2, 0, 0, 0},
                       {0, 128, 2, 1, 0, 0}, {0, 256, 2, 0, 0, 0},  {0, 256, 2, 1, 0, 0},
                       {0, 256, 1, 0, 0, 0}, {1, 256, 1, 0, 64, 0}, {1, 128, 1, 0, 9, 4096},
                       {2, 128, 1, 0, 40, 0}, {2, 64, 1, 0, 7, 512}};
    for (const Exec &e : execs) {
      pyrit_tune t{};
      t.mode = e.mode;
      t.wg_threads = e.wg;
      t.split_k = e.split;
      t.xcd_order = e.xcd;
      t.grid = e.grid;
      t.tile_bytes = e.tile;
      CHECK(batch_check_tune(&t) == PYRIT_OK);
      BatchImage bi;
      CHECK(build_batch_image(items.data(), n_items, t, e.grid, 0, &bi) == PYRIT_OK);
      if (e.mode == 0) walk_grid(bi);
      else walk_items(bi);
    }
    for (Stripe &s : st) pyrit_plan_destroy(s.plan);
  }
}

}  // namespace

int main() {
  run_model();
  CHECK(violations == 0 && loads > 0 && stores > 0);
  // the check has teeth: loads of dead lanes at their own column reach past
  // the end of the last slice of a block
  old_rule = true;
  run_model();
  CHECK(violations > 0);
  std::printf("ok\n");
  return 0;
}
