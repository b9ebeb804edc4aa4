// Request loop with continuous batching over the batch kernels.
//
// One host thread drives the loop: arrivals (by wall clock) enter a FIFO;
// the head of the FIFO is admitted when its output blocks fit in the device
// pool (the working-set cap); whenever a launch slot is free, every admitted
// request not yet launched goes out as one batch on that slot's stream (the
// descriptor image is uploaded into the slot's own device buffer, so nothing
// is allocated per launch); a slot's completion event returns its requests'
// outputs to the pool.  Launches on different slots overlap on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <thread>
#include <vector>

#include "batch_host.hpp"
#include "internal.hpp"

namespace pyrit {
namespace {

// Requests launched as one plain kernel each rather than one batch kernel
// (see the launch step of pyrit_server_run).
constexpr int kPlainLaunchMax = 4;

// First-fit allocator over [0, size) with coalescing frees.
class PoolAlloc {
 public:
  explicit PoolAlloc(uint64_t size) : size_(size) { free_[0] = size; }
  bool alloc(uint64_t n, uint64_t *off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= n) {
        *off = it->first;
        const uint64_t rest = it->second - n, at = it->first + n;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += n;
        peak_ = std::max(peak_, used_);
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t n) {
    used_ -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t peak() const { return peak_; }
  uint64_t size() const { return size_; }

 private:
  uint64_t size_, used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void *dbuf = nullptr;
  uint8_t *hbuf = nullptr;  // pinned staging for the descriptor image
  bool busy = false;
  bool large = false;  // running one large request
  std::vector<int> reqs;
};

}  // namespace
}  // namespace pyrit

using namespace pyrit;

struct pyrit_server {
  pyrit_serve_config cfg{};
  void *pool = nullptr;
  std::vector<Slot> slots;
  int resident_grid = 0;
  ~pyrit_server() {
    for (auto &s : slots) {
      if (s.stream) (void)hipStreamSynchronize(s.stream);
      if (s.done) (void)hipEventDestroy(s.done);
      if (s.stream) (void)hipStreamDestroy(s.stream);
      if (s.dbuf) (void)hipFree(s.dbuf);
      if (s.hbuf) (void)hipHostFree(s.hbuf);
    }
    if (pool) (void)hipFree(pool);
  }
};

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int n_outputs(const pyrit_request &r) { return r.n_erased ? r.n_erased : r.plan->m; }

}  // namespace

extern "C" {

int pyrit_server_create(const pyrit_serve_config *cfg, pyrit_server **out) {
  return abi_guard([&]() -> int {
    if (!cfg || !out || cfg->pool_bytes == 0 || cfg->slots < 1 || cfg->slots > 16 ||
        cfg->max_batch < 0)
      return PYRIT_EINVAL;
    *out = nullptr;
    std::unique_ptr<pyrit_server> s(new (std::nothrow) pyrit_server());
    if (!s) return PYRIT_ENOMEM;
    s->cfg = *cfg;
    if (!s->cfg.slot_bytes) s->cfg.slot_bytes = 64u << 20;
    int rc = batch_check_tune(&s->cfg.tune);
    if (rc) return rc;
    if (s->cfg.tune.mode != 0) {
      rc = batch_resident_grid(s->cfg.tune, &s->resident_grid);
      if (rc) return rc;
    }
    if (hipMalloc(&s->pool, s->cfg.pool_bytes) != hipSuccess) return PYRIT_ENOMEM;
    s->slots.resize(s->cfg.slots);
    for (auto &sl : s->slots) {
      if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) return PYRIT_EHIP;
      if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) return PYRIT_EHIP;
      if (hipMalloc(&sl.dbuf, s->cfg.slot_bytes) != hipSuccess) return PYRIT_ENOMEM;
      if (hipHostMalloc((void **)&sl.hbuf, s->cfg.slot_bytes, hipHostMallocDefault) != hipSuccess)
        return PYRIT_ENOMEM;
    }
    *out = s.release();
    return PYRIT_OK;
  });
}

void *pyrit_server_pool(const pyrit_server *server) { return server ? server->pool : nullptr; }

void pyrit_server_destroy(pyrit_server *server) { delete server; }

int pyrit_server_run(pyrit_server *sv, const pyrit_request *reqs, int n, pyrit_request_result *res,
                     pyrit_serve_stats *stats) {
  return abi_guard([&]() -> int {
    if (!sv || n < 0 || (n > 0 && (!reqs || !res))) return PYRIT_EINVAL;
    const pyrit_serve_config &cfg = sv->cfg;
    // Validate every request up front and size its outputs.
    std::vector<uint64_t> need(n), stride(n), moved(n);
    uint64_t moved_total = 0;
    for (int i = 0; i < n; ++i) {
      const pyrit_request &r = reqs[i];
      if (!r.plan || !r.inputs || (i && r.arrival_s < reqs[i - 1].arrival_s)) return PYRIT_EINVAL;
      if (r.plan->ring < 0) return PYRIT_EUNSUPPORTED;
      size_t pitch = r.slice_pitch;
      int rc = check_slices(r.plan->w, r.slice_bytes, &pitch);
      if (rc) return rc;
      if (r.n_erased < 0 || r.n_erased > r.plan->m) return PYRIT_ETOOMANY;
      if (r.n_erased) {
        // the erasure list (ids in range, distinct) is checked, and its
        // decoding matrix built, before anything runs
        std::shared_ptr<const DecodeEntry> ent;
        rc = decode_entry(r.plan, r.erased, r.n_erased, &ent);
        if (rc) return rc;
        if ((int)ent->outs.size() != r.n_erased) return PYRIT_EINTERNAL;
      }
      stride[i] = align256((uint64_t)r.plan->w * pitch) + cfg.block_skew;
      need[i] = stride[i] * (uint64_t)n_outputs(r);
      if (need[i] > sv->cfg.pool_bytes) return PYRIT_EBUSY;
      moved[i] = (uint64_t)(r.plan->k + n_outputs(r)) * r.plan->w * r.slice_bytes;
      moved_total += moved[i];
      std::memset(&res[i], 0, sizeof(res[i]));
    }
    PoolAlloc pool(cfg.pool_bytes);
    int max_batch = cfg.max_batch;  // lowered if a batch's descriptors overflow a slot
    std::deque<int> pending, admitted, admitted_large;
    int next = 0, done = 0, launches = 0, max_batch_seen = 0, waits = 0;
    long batched = 0;
    std::vector<char> waited(n, 0);
    const auto t0 = std::chrono::steady_clock::now();
    auto now_s = [&] {
      return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    std::vector<uint8_t *> blocks;  // k + m pointers per request, rebuilt per launch
    std::vector<int> ids;
    std::vector<pyrit_batch_item> items;
    BatchImage bi;
    int err = PYRIT_OK;
    // Every slot's stream is drained before the call returns, also when an
    // exception (a failed host allocation) ends the loop early.
    struct DrainSlots {
      pyrit_server *sv;
      ~DrainSlots() {
        for (auto &sl : sv->slots) {
          (void)hipStreamSynchronize(sl.stream);
          sl.busy = false;
          sl.reqs.clear();
        }
      }
    } drain{sv};

    // Build the k + m block list of request i with its outputs in the pool.
    auto fill_blocks = [&](int i, uint8_t **bl) {
      const pyrit_request &r = reqs[i];
      const int k = r.plan->k, m = r.plan->m;
      for (int b = 0; b < k + m; ++b) bl[b] = nullptr;
      std::vector<char> er(k + m, 0);
      std::vector<int> outs;
      if (r.n_erased == 0) {
        for (int b = k; b < k + m; ++b) outs.push_back(b);
      } else {
        for (int e = 0; e < r.n_erased; ++e) er[r.erased[e]] = 1;
        for (int b = 0; b < k + m; ++b)
          if (er[b]) outs.push_back(b);
      }
      int j = 0;
      for (int b = 0; b < k + m && j < k; ++b)
        if (!er[b] && (r.n_erased || b < k)) bl[b] = const_cast<uint8_t *>(r.inputs[j++]);
      for (size_t q = 0; q < outs.size(); ++q)
        bl[outs[q]] = (uint8_t *)sv->pool + res[i].out_offset + q * stride[i];
    };

    while (done < n && err == PYRIT_OK) {
      bool progress = false;
      double t = now_s();
      while (next < n && reqs[next].arrival_s <= t) pending.push_back(next++), progress = true;
      // completions
      for (auto &sl : sv->slots) {
        if (!sl.busy) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
          err = PYRIT_EHIP;
          break;
        }
        t = now_s();
        for (int i : sl.reqs) {
          res[i].done_s = t;
          if (cfg.release_outputs) pool.release(res[i].out_offset, need[i]);
          ++done;
        }
        sl.reqs.clear();
        sl.busy = false;
        progress = true;
      }
      // admission, first come first served
      while (!pending.empty()) {
        const int i = pending.front();
        uint64_t off;
        if (!pool.alloc(need[i], &off)) {
          if (!waited[i]) waited[i] = 1, ++waits;
          break;
        }
        res[i].out_offset = off;
        res[i].out_stride = stride[i];
        res[i].admit_s = now_s();
        const bool large = !cfg.per_request && cfg.large_bytes && moved[i] >= cfg.large_bytes;
        (large ? admitted_large : admitted).push_back(i);
        pending.pop_front();
        progress = true;
      }
      // Launch on free slots.  A large request (moving at least large_bytes)
      // goes out alone, on at most slots-1 slots so that one slot stays for
      // small requests.  Admitted small requests that the idle slots can hold
      // go out one per slot, running side by side on their streams; more than
      // that go out together on one slot.
      for (auto &sl : sv->slots) {
        if (admitted.empty() && admitted_large.empty()) break;
        if (sl.busy) continue;
        int large_busy = 0;
        for (auto &o : sv->slots) large_busy += o.busy && o.large;
        const bool can_large = large_busy < (int)sv->slots.size() - 1 || sv->slots.size() == 1;
        std::deque<int> *src;
        int take;
        if (!admitted_large.empty() && (can_large || admitted.empty())) {
          if (!can_large) continue;  // wait for a slot small requests do not need
          src = &admitted_large;
          take = 1;
        } else {
          src = &admitted;
          take = (int)admitted.size();
          int idle = 0;  // this slot and the other idle ones
          for (auto &o : sv->slots) idle += !o.busy;
          if (cfg.per_request || take <= idle) take = 1;
          else if (max_batch) take = std::min(take, max_batch);
        }
        ids.assign(src->begin(), src->begin() + take);
        size_t nb = 0;
        for (int i : ids) nb += reqs[i].plan->k + reqs[i].plan->m;
        blocks.assign(nb, nullptr);
        items.resize(ids.size());
        size_t at = 0;
        for (size_t q = 0; q < ids.size(); ++q) {
          const int i = ids[q];
          fill_blocks(i, &blocks[at]);
          items[q] = {reqs[i].plan, reqs[i].n_erased, reqs[i].erased, &blocks[at],
                      reqs[i].slice_bytes, reqs[i].slice_pitch};
          at += reqs[i].plan->k + reqs[i].plan->m;
        }
        int rc;
        // A launch of up to kPlainLaunchMax requests runs the plain kernel
        // once per request, back to back on the slot's stream: the arguments
        // travel in the kernel-argument segment, with no descriptor upload
        // ahead of them (the upload cost a two-request batch more than a
        // second plain launch at 20 k req/s).
        if (take <= kPlainLaunchMax) {
          rc = PYRIT_OK;
          for (int q = 0; q < take && rc == PYRIT_OK; ++q) {
            const pyrit_batch_item &it = items[q];
            if (it.n_erased == 0)
              rc = pyrit_encode_ex(it.plan, (const uint8_t *const *)it.blocks,
                                   it.blocks + it.plan->k, it.slice_bytes, it.slice_pitch, 0,
                                   sl.stream);
            else
              rc = pyrit_decode_ex(it.plan, it.erased, it.n_erased, it.blocks, it.slice_bytes,
                                   it.slice_pitch, sl.stream);
          }
        } else {
          rc = build_batch_image(items.data(), (int)items.size(), cfg.tune, sv->resident_grid,
                                 (uint64_t)(uintptr_t)sl.dbuf, &bi);
          if (rc == PYRIT_OK && bi.img.size() > cfg.slot_bytes) {
            // halve the batch and retry on the next pass of the loop
            max_batch = std::max(1, take / 2);
            continue;
          }
          if (rc == PYRIT_OK) {
            std::memcpy(sl.hbuf, bi.img.data(), bi.img.size());
            if (hipMemcpyAsync(sl.dbuf, sl.hbuf, bi.img.size(), hipMemcpyHostToDevice, sl.stream) !=
                hipSuccess)
              rc = PYRIT_EHIP;
          }
          if (rc == PYRIT_OK) rc = launch_batch_image(bi, sl.dbuf, sl.stream);
        }
        if (rc == PYRIT_OK && hipEventRecord(sl.done, sl.stream) != hipSuccess) rc = PYRIT_EHIP;
        if (rc) {
          err = rc;
          break;
        }
        t = now_s();
        for (int i : ids) res[i].launch_s = t, res[i].launch = launches;
        src->erase(src->begin(), src->begin() + take);
        sl.reqs = ids;
        sl.busy = true;
        sl.large = src == &admitted_large;
        ++launches;
        batched += take;
        max_batch_seen = std::max(max_batch_seen, take);
        progress = true;
      }
      if (!progress && err == PYRIT_OK) {
        bool any_busy = false;
        for (auto &sl : sv->slots) any_busy |= sl.busy;
        // The head request failed admission and nothing in flight can free
        // space for it (outputs are kept): it can never run.
        if (!any_busy && admitted.empty() && admitted_large.empty() && !pending.empty()) {
          err = PYRIT_EBUSY;
          break;
        }
        std::this_thread::yield();
      }
    }
    for (auto &sl : sv->slots) (void)hipStreamSynchronize(sl.stream);
    if (stats) {
      double first = n ? reqs[0].arrival_s : 0, last = 0;
      for (int i = 0; i < n; ++i) last = std::max(last, res[i].done_s);
      stats->elapsed_s = last - first;
      stats->launches = launches;
      stats->max_batch_seen = max_batch_seen;
      stats->mean_batch = launches ? (double)batched / launches : 0;
      stats->peak_pool_bytes = pool.peak();
      stats->admission_waits = waits;
      stats->moved_bytes = moved_total;
    }
    return err;
  });
}

}  // extern "C"
