// Host plan: ring validation, the sparse transform, the lifted schedule and
// decoding matrices.  No device work happens here.
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <tuple>

#include "gf2.hpp"
#include "internal.hpp"

namespace pyrit {

int ring_id(int w, int n, uint32_t p, int transform) {
  const bool parity = transform == PYRIT_TRANSFORM_PARITY;
  for (int i = 0; i < kNumRings; ++i)
    if (kRings[i].w == w && kRings[i].n == n && kRings[i].p == p && kRings[i].parity == parity)
      return i;
  return -1;
}

int check_slices(int w, size_t S, size_t *pitch) {
  if (*pitch == 0) *pitch = S;
  if (S == 0 || S % 64 != 0 || *pitch % 64 != 0) return PYRIT_EALIGN;
  if (*pitch < S) return PYRIT_EINVAL;
  if ((uint64_t)(w - 1) * (uint64_t)*pitch + (uint64_t)S >= (uint64_t)PYRIT_SMAX_TOTAL)
    return PYRIT_EINVAL;
  return PYRIT_OK;
}

// Sparse transform (Sec. II-B): the ring elements that represent u are
// u + t*p for every t of degree < n - w (all c with c mod p == u).  Keep one
// of least weight; ties go to the smallest integer.
static uint32_t lift_one(int w, int n, uint32_t p, uint32_t u) {
  uint32_t best = u;
  int bw = __builtin_popcount(u);
  const uint64_t ncand = 1ull << (n - w);
  for (uint64_t t = 1; t < ncand; ++t) {
    const uint32_t c = u ^ (uint32_t)clmul(t, p);
    const int cw = __builtin_popcount(c);
    if (cw < bw || (cw == bw && c < best)) {
      best = c;
      bw = cw;
    }
  }
  return best;
}

const std::vector<uint32_t> &lift_table(int w, int n, uint32_t p) {
  static std::mutex mu;
  static std::map<std::tuple<int, int, uint32_t>, std::vector<uint32_t>> cache;
  std::lock_guard<std::mutex> g(mu);
  auto key = std::make_tuple(w, n, p);
  auto it = cache.find(key);
  if (it != cache.end()) return it->second;
  std::vector<uint32_t> t(1u << w);
  for (uint32_t u = 0; u < (1u << w); ++u) t[u] = lift_one(w, n, p, u);
  return cache.emplace(key, std::move(t)).first->second;
}

std::vector<uint32_t> coef_words(int ring, const std::vector<uint16_t> &M,
                                 const std::vector<uint32_t> &L) {
  if (ring >= 0 && ring_fused(ring)) return std::vector<uint32_t>(M.begin(), M.end());
  return L;
}

// Gauss-Jordan inverse of a k x k matrix over GF(2^w) = F_2[x]/(p).
static int gf_invert(std::vector<uint32_t> &A, int k, uint32_t p) {
  std::vector<uint32_t> I((size_t)k * k, 0);
  for (int i = 0; i < k; ++i) I[(size_t)i * k + i] = 1;
  for (int c = 0; c < k; ++c) {
    int piv = -1;
    for (int r = c; r < k; ++r)
      if (A[(size_t)r * k + c]) {
        piv = r;
        break;
      }
    if (piv < 0) return PYRIT_ESINGULAR;
    if (piv != c)
      for (int x = 0; x < k; ++x) {
        std::swap(A[(size_t)c * k + x], A[(size_t)piv * k + x]);
        std::swap(I[(size_t)c * k + x], I[(size_t)piv * k + x]);
      }
    const uint32_t s = gf_inv(A[(size_t)c * k + c], p);
    for (int x = 0; x < k; ++x) {
      A[(size_t)c * k + x] = gf_mul(A[(size_t)c * k + x], s, p);
      I[(size_t)c * k + x] = gf_mul(I[(size_t)c * k + x], s, p);
    }
    for (int r = 0; r < k; ++r) {
      const uint32_t e = A[(size_t)r * k + c];
      if (r == c || !e) continue;
      for (int x = 0; x < k; ++x) {
        A[(size_t)r * k + x] ^= gf_mul(e, A[(size_t)c * k + x], p);
        I[(size_t)r * k + x] ^= gf_mul(e, I[(size_t)c * k + x], p);
      }
    }
  }
  A.swap(I);
  return PYRIT_OK;
}

int decode_entry(const pyrit_plan *plan, const int *erased, int n_erased,
                 std::shared_ptr<const DecodeEntry> *out) {
  const int k = plan->k, m = plan->m, tot = k + m;
  if (n_erased < 0 || (n_erased > 0 && !erased)) return PYRIT_EINVAL;
  if (n_erased > m) return PYRIT_ETOOMANY;
  std::vector<char> is_er(tot, 0);
  for (int e = 0; e < n_erased; ++e) {
    if (erased[e] < 0 || erased[e] >= tot || is_er[erased[e]]) return PYRIT_EINVAL;
    is_er[erased[e]] = 1;
  }
  std::string key(is_er.begin(), is_er.end());
  {
    std::lock_guard<std::mutex> g(plan->mu);
    auto it = plan->dcache.find(key);
    if (it != plan->dcache.end()) {
      *out = it->second;
      return PYRIT_OK;
    }
  }
  auto ent = std::make_shared<DecodeEntry>();
  for (int i = 0; i < tot && (int)ent->surv.size() < k; ++i)
    if (!is_er[i]) ent->surv.push_back(i);
  for (int i = 0; i < tot; ++i)
    if (is_er[i]) ent->outs.push_back(i);
  // A: the survivors' rows of [I; G]
  std::vector<uint32_t> A((size_t)k * k, 0);
  for (int r = 0; r < k; ++r) {
    const int g = ent->surv[r];
    for (int c = 0; c < k; ++c)
      A[(size_t)r * k + c] = g < k ? (uint32_t)(g == c) : plan->G[(size_t)(g - k) * k + c];
  }
  int rc = gf_invert(A, k, plan->p);
  if (rc != PYRIT_OK) return rc;
  // D = G_E * A^{-1}: an erased data block j takes row j of A^{-1}; an erased
  // parity block i takes G row i times A^{-1}.
  const int ne = (int)ent->outs.size();
  ent->D.assign((size_t)ne * k, 0);
  for (int e = 0; e < ne; ++e) {
    const int g = ent->outs[e];
    for (int c = 0; c < k; ++c) {
      uint32_t acc = 0;
      if (g < k) {
        acc = A[(size_t)g * k + c];
      } else {
        for (int r = 0; r < k; ++r)
          acc ^= gf_mul(plan->G[(size_t)(g - k) * k + r], A[(size_t)r * k + c], plan->p);
      }
      ent->D[(size_t)e * k + c] = (uint16_t)acc;
    }
  }
  const auto &lt = lift_table(plan->w, plan->n, plan->p);
  ent->L.resize(ent->D.size());
  for (size_t i = 0; i < ent->D.size(); ++i) {
    ent->L[i] = lt[ent->D[i]];
    ent->weight += __builtin_popcount(ent->L[i]);
  }
  ent->K = coef_words(plan->ring, ent->D, ent->L);
  std::lock_guard<std::mutex> g(plan->mu);
  auto ins = plan->dcache.emplace(key, ent);
  *out = ins.first->second;
  return PYRIT_OK;
}

}  // namespace pyrit

using namespace pyrit;

extern "C" {

const char *pyrit_strerror(int code) {
  switch (code) {
    case PYRIT_OK: return "ok";
    case PYRIT_EINVAL: return "invalid argument";
    case PYRIT_ENOTIRRED: return "p is not irreducible of degree w";
    case PYRIT_ENOTDIV: return "n must be odd and p must divide x^n+1";
    case PYRIT_ETOOLONG: return "k+m exceeds the field size 2^w";
    case PYRIT_ERANGE: return "generator coefficient out of the field";
    case PYRIT_ETOOMANY: return "more erasures than parity blocks";
    case PYRIT_ESINGULAR: return "surviving rows are not invertible";
    case PYRIT_EALIGN: return "slice size must be a positive multiple of 64 and pointers 16-byte aligned";
    case PYRIT_EUNSUPPORTED: return "no device kernel for this ring";
    case PYRIT_EHIP: return "HIP runtime error";
    case PYRIT_ENOMEM: return "out of memory";
    case PYRIT_EBUSY: return "resource cap reached";
    case PYRIT_EINTERNAL: return "internal error";
    case PYRIT_ETOOBIG: return "work exceeds a fixed-size library buffer";
    default: return "unknown error";
  }
}

const char *pyrit_version(void) { return "pyrit-mi355x 0.1"; }

int pyrit_ring_check(int w, int n, uint32_t p) {
  if (w < 1 || w > 16 || n < 1 || n > 24 || n <= w) return PYRIT_EINVAL;
  if (deg(p) != w) return PYRIT_EINVAL;
  if (!irreducible(p)) return PYRIT_ENOTIRRED;
  if (n % 2 == 0) return PYRIT_ENOTDIV;
  if (pmod((1ull << n) | 1ull, p) != 0) return PYRIT_ENOTDIV;
  return PYRIT_OK;
}

int pyrit_ring_supported(int w, int n, uint32_t p) { return ring_id(w, n, p) >= 0 ? 1 : 0; }

int pyrit_lift(int w, int n, uint32_t p, uint32_t u, uint32_t *c) {
  return abi_guard([&]() -> int {
    int rc = pyrit_ring_check(w, n, p);
    if (rc) return rc;
    if (!c) return PYRIT_EINVAL;
    if (u >> w) return PYRIT_ERANGE;
    *c = lift_table(w, n, p)[u];
    return PYRIT_OK;
  });
}

int pyrit_ring_reduce(int w, int n, uint32_t p, uint32_t c, uint32_t *u) {
  int rc = pyrit_ring_check(w, n, p);
  if (rc) return rc;
  if (!u || (c >> n)) return PYRIT_EINVAL;
  *u = (uint32_t)pmod(c, p);
  return PYRIT_OK;
}

int pyrit_ring_mul(int n, uint32_t a, uint32_t b, uint32_t *c) {
  if (n < 1 || n > 31 || !c || (a >> n) || (b >> n)) return PYRIT_EINVAL;
  *c = ring_mul(a, b, n);
  return PYRIT_OK;
}

int pyrit_gf_mul(int w, uint32_t p, uint32_t a, uint32_t b, uint32_t *c) {
  if (w < 1 || w > 16 || deg(p) != w || !c) return PYRIT_EINVAL;
  if ((a >> w) || (b >> w)) return PYRIT_ERANGE;
  *c = gf_mul(a, b, p);
  return PYRIT_OK;
}

int pyrit_cauchy(int w, uint32_t p, int k, int m, uint16_t *G) {
  if (w < 1 || w > 16 || deg(p) != w || !G || k < 1 || m < 1) return PYRIT_EINVAL;
  if (!irreducible(p)) return PYRIT_ENOTIRRED;
  if ((uint64_t)k + (uint64_t)m > (1ull << w)) return PYRIT_ETOOLONG;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < k; ++j) G[(size_t)i * k + j] = (uint16_t)gf_inv((uint32_t)(i ^ (m + j)), p);
  return PYRIT_OK;
}

int pyrit_cauchy_light(int w, int n, uint32_t p, int k, int m, uint16_t *G, uint16_t *row_scale,
                       uint16_t *col_scale, int *weight) {
  return abi_guard([&]() -> int {
    int rc = pyrit_ring_check(w, n, p);
    if (rc) return rc;
    rc = pyrit_cauchy(w, p, k, m, G);
    if (rc) return rc;
    const auto &lt = lift_table(w, n, p);
    const uint32_t q = 1u << w;
    std::vector<uint32_t> C((size_t)m * k), d(m, 1u), c(k, 1u);
    for (size_t i = 0; i < C.size(); ++i) C[i] = G[i];
    auto wt = [&](uint32_t u) { return __builtin_popcount(lt[u]); };
    // Coordinate descent over the row and column multipliers: each step keeps
    // the multiplier with the smallest total lifted weight of its row or
    // column (ties: the smallest element), so the total never increases.
    for (int round = 0; round < 16; ++round) {
      bool changed = false;
      for (int j = 0; j < k; ++j) {
        uint32_t best = c[j];
        long best_w = -1;
        for (uint32_t a = 1; a < q; ++a) {
          long s = 0;
          for (int i = 0; i < m; ++i) s += wt(gf_mul(gf_mul(d[i], C[(size_t)i * k + j], p), a, p));
          if (best_w < 0 || s < best_w) { best_w = s; best = a; }
        }
        long cur = 0;
        for (int i = 0; i < m; ++i) cur += wt(gf_mul(gf_mul(d[i], C[(size_t)i * k + j], p), c[j], p));
        if (best_w < cur) { c[j] = best; changed = true; }
      }
      for (int i = 0; i < m; ++i) {
        uint32_t best = d[i];
        long best_w = -1;
        for (uint32_t a = 1; a < q; ++a) {
          long s = 0;
          for (int j = 0; j < k; ++j) s += wt(gf_mul(gf_mul(a, C[(size_t)i * k + j], p), c[j], p));
          if (best_w < 0 || s < best_w) { best_w = s; best = a; }
        }
        long cur = 0;
        for (int j = 0; j < k; ++j) cur += wt(gf_mul(gf_mul(d[i], C[(size_t)i * k + j], p), c[j], p));
        if (best_w < cur) { d[i] = best; changed = true; }
      }
      if (!changed) break;
    }
    int total = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < k; ++j) {
        const uint32_t g = gf_mul(gf_mul(d[i], C[(size_t)i * k + j], p), c[j], p);
        G[(size_t)i * k + j] = (uint16_t)g;
        total += wt(g);
      }
    if (row_scale)
      for (int i = 0; i < m; ++i) row_scale[i] = (uint16_t)d[i];
    if (col_scale)
      for (int j = 0; j < k; ++j) col_scale[j] = (uint16_t)c[j];
    if (weight) *weight = total;
    return PYRIT_OK;
  });
}

namespace {

// GF(2^w) products through logarithm and antilogarithm tables of one
// generator of the multiplicative group (the smallest element of order
// 2^w - 1), for the searches below.
struct GfTables {
  uint32_t q = 0;
  std::vector<uint32_t> ex, lg;  // ex[i] = g^i for i < 2(q - 1); lg[g^i] = i
  GfTables(int w, uint32_t p) : q(1u << w), ex(2 * (size_t)q), lg(q, 0) {
    uint32_t g = 2;
    for (;; ++g) {
      uint32_t x = g, ord = 1;
      while (x != 1) {
        x = gf_mul(x, g, p);
        ++ord;
      }
      if (ord == q - 1) break;
    }
    uint32_t x = 1;
    for (uint32_t i = 0; i < 2 * (q - 1); ++i) {
      ex[i] = x;
      if (i < q - 1) lg[x] = i;
      x = gf_mul(x, g, p);
    }
  }
  uint32_t mul(uint32_t a, uint32_t b) const { return a && b ? ex[lg[a] + lg[b]] : 0u; }
  uint32_t inv(uint32_t a) const { return ex[(q - 1) - lg[a]]; }
};

}  // namespace

int pyrit_cauchy_search(int w, int n, uint32_t p, int k, int m, int sweeps, uint16_t *G,
                        uint16_t *X, uint16_t *Y, uint16_t *row_scale, uint16_t *col_scale,
                        int *weight) {
  return abi_guard([&]() -> int {
    int rc = pyrit_ring_check(w, n, p);
    if (rc) return rc;
    if (!G || k < 1 || m < 1 || sweeps < 0) return PYRIT_EINVAL;
    if (w > 10) return PYRIT_EUNSUPPORTED;
    const uint32_t q = 1u << w;
    if ((uint64_t)k + (uint64_t)m > q) return PYRIT_ETOOLONG;
    const GfTables F(w, p);
    const auto &lt = lift_table(w, n, p);
    std::vector<int> wt(q);
    for (uint32_t u = 0; u < q; ++u) wt[u] = __builtin_popcount(lt[u]);
    std::vector<uint32_t> x(m), y(k), d(m, 1u), c(k, 1u);
    std::vector<char> used(q, 0);
    for (int i = 0; i < m; ++i) used[x[i] = (uint32_t)i] = 1;
    for (int j = 0; j < k; ++j) used[y[j] = (uint32_t)(m + j)] = 1;
    auto entry = [&](int i, int j) { return F.mul(F.mul(d[i], c[j]), F.inv(x[i] ^ y[j])); };
    // The multiplier a (a != 0) minimising sum_v wt(a * v) over the values
    // v; returns that sum.  Ties go to the smallest a.
    std::vector<uint32_t> vals;
    auto best_multiplier = [&](uint32_t *a_out) {
      long best = -1;
      for (uint32_t a = 1; a < q; ++a) {
        long s = 0;
        for (uint32_t v : vals) s += wt[F.mul(a, v)];
        if (best < 0 || s < best) {
          best = s;
          *a_out = a;
        }
      }
      return best;
    };
    // Coordinate descent over all multipliers (as pyrit_cauchy_light).
    auto descend = [&]() {
      for (int round = 0; round < 16; ++round) {
        bool changed = false;
        for (int j = 0; j < k; ++j) {
          vals.clear();
          long cur = 0;
          for (int i = 0; i < m; ++i) {
            vals.push_back(F.mul(d[i], F.inv(x[i] ^ y[j])));
            cur += wt[entry(i, j)];
          }
          uint32_t a = c[j];
          if (best_multiplier(&a) < cur) c[j] = a, changed = true;
        }
        for (int i = 0; i < m; ++i) {
          vals.clear();
          long cur = 0;
          for (int j = 0; j < k; ++j) {
            vals.push_back(F.mul(c[j], F.inv(x[i] ^ y[j])));
            cur += wt[entry(i, j)];
          }
          uint32_t a = d[i];
          if (best_multiplier(&a) < cur) d[i] = a, changed = true;
        }
        if (!changed) break;
      }
    };
    descend();
    for (int sweep = 0; sweep < sweeps; ++sweep) {
      bool improved = false;
      // each row point, then each column point, against every unused element
      for (int i = 0; i < m; ++i) {
        long cur = 0;
        for (int j = 0; j < k; ++j) cur += wt[entry(i, j)];
        for (uint32_t e = 0; e < q; ++e) {
          if (used[e]) continue;
          vals.clear();
          for (int j = 0; j < k; ++j) vals.push_back(F.mul(c[j], F.inv(e ^ y[j])));
          uint32_t a = 1;
          const long s = best_multiplier(&a);
          if (s < cur) {
            used[x[i]] = 0;
            used[x[i] = e] = 1;
            d[i] = a;
            cur = s;
            improved = true;
          }
        }
      }
      for (int j = 0; j < k; ++j) {
        long cur = 0;
        for (int i = 0; i < m; ++i) cur += wt[entry(i, j)];
        for (uint32_t e = 0; e < q; ++e) {
          if (used[e]) continue;
          vals.clear();
          for (int i = 0; i < m; ++i) vals.push_back(F.mul(d[i], F.inv(x[i] ^ e)));
          uint32_t a = 1;
          const long s = best_multiplier(&a);
          if (s < cur) {
            used[y[j]] = 0;
            used[y[j] = e] = 1;
            c[j] = a;
            cur = s;
            improved = true;
          }
        }
      }
      descend();
      if (!improved) break;
    }
    int total = 0;
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < k; ++j) {
        const uint32_t g = entry(i, j);
        G[(size_t)i * k + j] = (uint16_t)g;
        total += wt[g];
      }
    for (int i = 0; i < m; ++i) {
      if (X) X[i] = (uint16_t)x[i];
      if (row_scale) row_scale[i] = (uint16_t)d[i];
    }
    for (int j = 0; j < k; ++j) {
      if (Y) Y[j] = (uint16_t)y[j];
      if (col_scale) col_scale[j] = (uint16_t)c[j];
    }
    if (weight) *weight = total;
    return PYRIT_OK;
  });
}

int pyrit_plan_create(int w, int n, uint32_t p, int k, int m, const uint16_t *G,
                      pyrit_plan **out) {
  return pyrit_plan_create_ex(w, n, p, k, m, G, PYRIT_TRANSFORM_EMBEDDING, out);
}

int pyrit_plan_create_ex(int w, int n, uint32_t p, int k, int m, const uint16_t *G, int transform,
                         pyrit_plan **out) {
  return abi_guard([&]() -> int {
    if (transform != PYRIT_TRANSFORM_EMBEDDING && transform != PYRIT_TRANSFORM_PARITY)
      return PYRIT_EINVAL;
    if (!out || !G) return PYRIT_EINVAL;
    *out = nullptr;
    int rc = pyrit_ring_check(w, n, p);
    if (rc) return rc;
    if (k < 1 || k > PYRIT_KMAX || m < 1 || m > PYRIT_MMAX) return PYRIT_EINVAL;
    if ((uint64_t)k + (uint64_t)m > (1ull << w)) return PYRIT_ETOOLONG;
    for (int i = 0; i < m * k; ++i)
      if (G[i] >> w) return PYRIT_ERANGE;
    std::unique_ptr<pyrit_plan> pl(new (std::nothrow) pyrit_plan());
    if (!pl) return PYRIT_ENOMEM;
    pl->w = w;
    pl->n = n;
    pl->p = p;
    pl->k = k;
    pl->m = m;
    pl->ring = ring_id(w, n, p, transform);
    pl->transform = transform;
    pl->G.assign(G, G + (size_t)m * k);
    const auto &lt = lift_table(w, n, p);
    pl->L.resize(pl->G.size());
    for (size_t i = 0; i < pl->G.size(); ++i) {
      pl->L[i] = lt[pl->G[i]];
      pl->weight += __builtin_popcount(pl->L[i]);
    }
    pl->K = coef_words(pl->ring, pl->G, pl->L);
    *out = pl.release();
    return PYRIT_OK;
  });
}

void pyrit_plan_destroy(pyrit_plan *plan) { delete plan; }

int pyrit_plan_params(const pyrit_plan *plan, int *w, int *n, uint32_t *p, int *k, int *m) {
  if (!plan) return PYRIT_EINVAL;
  if (w) *w = plan->w;
  if (n) *n = plan->n;
  if (p) *p = plan->p;
  if (k) *k = plan->k;
  if (m) *m = plan->m;
  return PYRIT_OK;
}

int pyrit_plan_transform(const pyrit_plan *plan, int *transform) {
  if (!plan || !transform) return PYRIT_EINVAL;
  *transform = plan->transform;
  return PYRIT_OK;
}

int pyrit_plan_lifted(const pyrit_plan *plan, uint32_t *C) {
  if (!plan || !C) return PYRIT_EINVAL;
  std::memcpy(C, plan->L.data(), plan->L.size() * sizeof(uint32_t));
  return PYRIT_OK;
}

int pyrit_plan_weight(const pyrit_plan *plan, int *weight) {
  if (!plan || !weight) return PYRIT_EINVAL;
  *weight = plan->weight;
  return PYRIT_OK;
}

int pyrit_decode_matrix(const pyrit_plan *plan, const int *erased, int n_erased, int *survivors,
                        uint16_t *D) {
  return abi_guard([&]() -> int {
    if (!plan) return PYRIT_EINVAL;
    std::shared_ptr<const DecodeEntry> ent;
    int rc = decode_entry(plan, erased, n_erased, &ent);
    if (rc) return rc;
    if (survivors) std::copy(ent->surv.begin(), ent->surv.end(), survivors);
    if (D) {
      // rows in the caller's order
      for (int e = 0; e < n_erased; ++e) {
        const int row = (int)(std::find(ent->outs.begin(), ent->outs.end(), erased[e]) - ent->outs.begin());
        std::copy(ent->D.begin() + (size_t)row * plan->k, ent->D.begin() + (size_t)(row + 1) * plan->k,
                  D + (size_t)e * plan->k);
      }
    }
    return PYRIT_OK;
  });
}

}  // extern "C"
