// Host arithmetic on polynomials over GF(2) for the plan builder.
//
// A polynomial is an integer whose bit i is the coefficient of x^i.  The
// field GF(2^w) = F_2[x]/(p) and the ring R_{2,n} = F_2[x]/(x^n + 1) of the
// paper's Sec. II-A are both handled with carry-less products and remainders;
// no tables are involved.
#pragma once
#include <cstdint>

namespace pyrit {

inline int deg(uint64_t a) { return a ? 63 - __builtin_clzll(a) : -1; }

// Carry-less product (no reduction).
inline uint64_t clmul(uint64_t a, uint64_t b) {
  uint64_t r = 0;
  while (b) {
    if (b & 1u) r ^= a;
    a <<= 1;
    b >>= 1;
  }
  return r;
}

// Remainder of a modulo m (m != 0).
inline uint64_t pmod(uint64_t a, uint64_t m) {
  const int dm = deg(m);
  for (int d = deg(a); d >= dm; d = deg(a)) a ^= m << (d - dm);
  return a;
}

// Product in F_2[x]/(p) for reduced operands.
inline uint32_t gf_mul(uint32_t a, uint32_t b, uint32_t p) {
  return (uint32_t)pmod(clmul(a, b), p);
}

// Multiplicative inverse in F_2[x]/(p), p irreducible, a != 0: a^(2^w - 2).
inline uint32_t gf_inv(uint32_t a, uint32_t p) {
  const int w = deg(p);
  uint32_t r = 1, base = a;
  uint64_t e = (1ull << w) - 2;
  while (e) {
    if (e & 1u) r = gf_mul(r, base, p);
    base = gf_mul(base, base, p);
    e >>= 1;
  }
  return r;
}

// Product in R_{2,n}: reduce modulo x^n + 1 by folding the high part.
inline uint32_t ring_mul(uint32_t a, uint32_t b, int n) {
  uint64_t c = clmul(a, b);
  const uint64_t lo = c & ((1ull << n) - 1);
  const uint64_t hi = c >> n;
  return (uint32_t)(lo ^ hi);  // deg c <= 2n-2, so one fold suffices
}

// Irreducibility by trial division with every polynomial of degree 1..deg/2.
inline bool irreducible(uint32_t p) {
  const int d = deg(p);
  if (d < 1) return false;
  for (uint64_t q = 2; deg(q) <= d / 2; ++q)
    if (pmod(p, q) == 0) return false;
  return true;
}

}  // namespace pyrit
