// Host-side twiddle tables for the wave NTT modulo the Goldilocks prime.
#include <stdint.h>

#include "internal.h"

namespace vlp {
namespace {

constexpr uint64_t P = 0xFFFFFFFF00000001ull;

uint64_t mulmod(uint64_t a, uint64_t b) { return (uint64_t)((unsigned __int128)a * b % P); }

uint64_t powmod(uint64_t b, uint64_t e) {
  uint64_t r = 1;
  while (e) {
    if (e & 1) r = mulmod(r, b);
    b = mulmod(b, b);
    e >>= 1;
  }
  return r;
}

uint32_t brv10(uint32_t x) {
  uint32_t r = 0;
  for (int i = 0; i < 10; ++i) r |= ((x >> i) & 1u) << (9 - i);
  return r;
}

}  // namespace

void make_twiddles(uint64_t* tw_fwd, uint64_t* tw_inv) {
  // 7 generates the multiplicative group mod p, so 7^((p-1)/2048) has order 2048.
  const uint64_t psi = powmod(7, (P - 1) / 2048);
  const uint64_t psi_inv = powmod(psi, P - 2);
  for (uint32_t m = 0; m < (uint32_t)RING_N; ++m) {
    tw_fwd[m] = powmod(psi, brv10(m));
    tw_inv[m] = powmod(psi_inv, brv10(m));
  }
}

}  // namespace vlp
