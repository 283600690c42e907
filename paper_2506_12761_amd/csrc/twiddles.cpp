// Host-side twiddle tables for the two-prime wave NTT.
#include <stdint.h>

#include "internal.h"
#include "rns.h"

namespace vlp {

// Entry m: psi^brv10(m) mod each prime as its signed representative
// w in (-p/2, p/2), and floor(w 2^32 / p) (rounded down for negative w).
void make_twiddles(uint32_t* tw) {
  for (uint32_t m = 0; m < (uint32_t)RING_N; ++m) {
    const TwPair a = twiddle(P1, PSI1, m), b = twiddle(P2, PSI2, m);
    tw[4 * m + 0] = a.w;
    tw[4 * m + 1] = a.q;
    tw[4 * m + 2] = b.w;
    tw[4 * m + 3] = b.q;
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
