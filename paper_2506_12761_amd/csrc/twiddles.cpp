// Host-side twiddle tables for the two-prime wave NTT.
#include <stdint.h>

#include <vector>

#include "internal.h"
#include "rns.h"

namespace vlp {
namespace {

uint32_t brv10(uint32_t x) {
  uint32_t r = 0;
  for (int i = 0; i < 10; ++i) r |= ((x >> i) & 1u) << (9 - i);
  return r;
}

// Smallest generator of the multiplicative group mod the prime p.
uint64_t generator(uint64_t p) {
  std::vector<uint64_t> f;
  uint64_t n = p - 1;
  for (uint64_t d = 2; d * d <= n; ++d)
    if (n % d == 0) {
      f.push_back(d);
      while (n % d == 0) n /= d;
    }
  if (n > 1) f.push_back(n);
  for (uint64_t g = 2;; ++g) {
    bool ok = true;
    for (uint64_t q : f) ok = ok && pow_mod(g, (p - 1) / q, p) != 1;
    if (ok) return g;
  }
}

}  // namespace

// Entry m: psi^brv10(m) mod each prime as its signed representative
// w in (-p/2, p/2), and floor(w 2^32 / p) (rounded down for negative w too).
void make_twiddles(uint32_t* tw) {
  const uint32_t primes[2] = {P1, P2};
  for (int k = 0; k < 2; ++k) {
    const int64_t p = primes[k];
    const uint64_t psi = pow_mod(generator(p), (p - 1) / 2048, p);  // order 2048
    for (uint32_t m = 0; m < (uint32_t)RING_N; ++m) {
      const int64_t w0 = (int64_t)pow_mod(psi, brv10(m), p);
      const int64_t w = w0 > p / 2 ? w0 - p : w0;
      const int64_t n = w * ((int64_t)1 << 32);
      const int64_t q = n / p - ((n % p != 0 && n < 0) ? 1 : 0);
      tw[4 * m + 2 * k] = (uint32_t)(int32_t)w;
      tw[4 * m + 2 * k + 1] = (uint32_t)(int32_t)q;
    }
  }
}

// Per prime: N^-1 * 2^32 mod p (Montgomery form of 1/1024) and its Shoup quotient.
void key_scale(uint32_t out[4]) {
  const uint32_t primes[2] = {P1, P2};
  for (int k = 0; k < 2; ++k) {
    const uint64_t p = primes[k];
    const uint64_t v = pow_mod(RING_N, p - 2, p) * ((1ull << 32) % p) % p;
    out[2 * k] = (uint32_t)v;
    out[2 * k + 1] = (uint32_t)((v << 32) / p);
  }
}

}  // namespace vlp
