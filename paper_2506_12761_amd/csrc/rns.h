// Two-prime residue arithmetic for the exact negacyclic products.
//
// The blind rotation's polynomial products are integers of magnitude
// < 6 * 1024 * 64 * 2^32 < 2^50.6 (6 digit polynomials with |digit| <= 64
// times key words < 2^32, 1024 terms each).  They are computed modulo
// Q = P1 * P2 (~2^53.9) with two NTT primes P_i = 1 (mod 2048) and lifted
// back exactly: Q/2 > 2^52.9 exceeds every |coefficient|, so the centred
// residue is the integer itself and its low 32 bits are the torus result.
//
// Both primes are below 2^32 / 33 so that
//   - the forward transform never reduces: a Cooley-Tukey butterfly with a
//     Shoup twiddle (product in [0, 2P)) raises the bound of its values by 2P,
//     so inputs below 2P leave the ten stages below 22P < 2^32;
//   - six products of such values and canonical key residues sum below
//     132 P^2 < 4P * 2^32, the input range of one Montgomery reduction to
//     [0, 4P) (one reduction per accumulated coefficient);
//   - the inverse transform reduces only every third or fourth stage: a
//     Gentleman-Sande sum doubles the bound, and inputs below 4P may double
//     three times (32P < 2^32) before a Shoup product by 1 brings them back
//     below 2P.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlp {

constexpr uint32_t P1 = 130121729u;  // 0x07c18001 = 63536 * 2^11 + 1
constexpr uint32_t P2 = 130103297u;  // 0x07c13801 = 63527 * 2^11 + 1

// p^-1 mod 2^32 by Newton iteration (p odd).
constexpr uint32_t inv_mod_2_32(uint32_t p) {
  uint32_t x = p;
  for (int i = 0; i < 5; ++i) x *= 2u - p * x;
  return x;
}
constexpr uint64_t pow_mod(uint64_t b, uint64_t e, uint64_t m) {
  uint64_t r = 1;
  b %= m;
  while (e) {
    if (e & 1) r = r * b % m;
    b = b * b % m;
    e >>= 1;
  }
  return r;
}
constexpr uint32_t P1_INV = inv_mod_2_32(P1);
constexpr uint32_t P2_INV = inv_mod_2_32(P2);
// CRT: x = x1 + P1 * ((x2 - x1) * P1^-1 mod P2).
constexpr uint32_t C12 = (uint32_t)pow_mod(P1 % P2, P2 - 2, P2);
constexpr uint32_t C12_SHOUP = (uint32_t)(((uint64_t)C12 << 32) / P2);
constexpr uint64_t Q = (uint64_t)P1 * P2;

static_assert(33ull * P1 < (1ull << 32) && 33ull * P2 < (1ull << 32), "primes too large for lazy ranges");
static_assert((P1 - 1) % 2048 == 0 && (P2 - 1) % 2048 == 0, "primes need 2048-th roots of unity");
static_assert(Q / 2 > (6ull * 1024 * 64) << 32, "modulus too small for an exact lift");
static_assert(P1 < 2 * P2, "CRT difference range");

// Shoup product: y * w mod p in [0, 2p), for y < 2^32, w < p, wp = floor(w 2^32 / p).
__device__ __forceinline__ uint32_t shoup(uint32_t y, uint32_t w, uint32_t wp, uint32_t p) {
  const uint32_t q = __umulhi(y, wp);
  return w * y - q * p;
}

// x mod p in [0, 2p) for any 32-bit x: the Shoup product by 1 (whose
// quotient is floor(2^32 / p)).
__device__ __forceinline__ uint32_t reduce_2p(uint32_t x, uint32_t p) {
  return shoup(x, 1u, (uint32_t)((1ull << 32) / p), p);
}

// x - m if x >= m, else x (for x < 2m): one subtract and one unsigned min.
__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t m) { return min(x, x - m); }

// Montgomery reduction: T * 2^-32 mod p in [0, p) for T < p * 2^32, and in
// [0, 4p) for T < 4p * 2^32 (t is then in (-p, 4p) and 5p < 2^32).
__device__ __forceinline__ uint32_t redc(uint64_t T, uint32_t p, uint32_t pinv) {
  const uint32_t m = (uint32_t)T * pinv;
  const uint32_t t = (uint32_t)(T >> 32) - __umulhi(m, p);  // exact: low words cancel
  return min(t, t + p);                                      // t < 0 wraps high; t + p is then in [0, p)
}

// Six products of a lazy forward-transform value (< 22p) and a canonical key
// residue (< p) sum below 132 p^2 < 4p * 2^32 (< 2^64): one reduction to
// [0, 4p) and no reduction of the transform output.  Three such products
// (one half of an output, the four-wavefront kernel) stay below 66 p^2 <
// 2p * 2^32: one reduction to [0, 2p).
static_assert((unsigned __int128)132 * P1 * P1 < ((unsigned __int128)4 * P1 << 32) &&
                  (unsigned __int128)132 * P2 * P2 < ((unsigned __int128)4 * P2 << 32) &&
                  (unsigned __int128)66 * P1 * P1 < ((unsigned __int128)2 * P1 << 32) &&
                  (unsigned __int128)66 * P2 * P2 < ((unsigned __int128)2 * P2 << 32),
              "accumulator range");

// Low 32 bits of the centred lift of (x1 mod P1, x2 mod P2), canonical inputs.
__device__ __forceinline__ uint32_t crt_lift_u32(uint32_t x1, uint32_t x2) {
  const uint32_t d = x2 + 2u * P2 - x1;                 // = x2 - x1 (mod P2), in (0, 3 P2)
  const uint32_t h = csub(shoup(d, C12, C12_SHOUP, P2), P2);
  const uint64_t x = (uint64_t)P1 * h + x1;             // in [0, Q)
  return (uint32_t)x - (x > Q / 2 ? (uint32_t)Q : 0u);
}

// Residue of a signed digit.
__device__ __forceinline__ uint32_t res_of(int32_t d, uint32_t p) { return d < 0 ? (uint32_t)(d + (int32_t)p) : (uint32_t)d; }

}  // namespace vlp
