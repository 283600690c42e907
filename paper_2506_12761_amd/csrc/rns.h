// Two-prime residue arithmetic for the exact negacyclic products.
//
// The blind rotation's polynomial products are integers of magnitude
// < 6 * 1024 * 64 * 2^32 < 2^50.6 (6 digit polynomials with |digit| <= 64
// times key words < 2^32, 1024 terms each).  They are computed modulo
// Q = P1 * P2 (~2^52.0) with two NTT primes P_i = 1 (mod 2048) and lifted
// back exactly: Q/2 = 2^51.0 exceeds every |coefficient|, so the centred
// residue is the integer itself and its low 32 bits are the torus result.
//
// Residues on the transform path are signed: an int32 representative of
// the class (kept in 32-bit registers, two's complement) whose magnitude is
// tracked and stays below 2^31.  Twiddles are signed too, |w| < P/2, so that
// their Shoup quotients floor(w 2^32 / P) fit in an int32 and a product
// needs one signed high multiply, one low multiply and one multiply-add.
// Both primes are below 2^26 so that
//   - the forward transform never reduces: a Cooley-Tukey butterfly
//     (x + t, x - t) with t = w y in (-P/2, 3P/2) raises the magnitude bound
//     by 3P/2, so digits (|d| <= 64) leave the ten stages below 16P;
//   - six products of such values and canonical key residues stay far
//     inside the int64 range, and one Montgomery reduction of their sum
//     lands within (-4P, 4P);
//   - the inverse transform reduces only at three of its ten stages: a
//     Gentleman-Sande sum doubles the bound, and inputs below 4P may double
//     three times (32P < 2^31) before a Shoup product by 1 brings them back
//     into (-P/2, 3P/2).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlp {

constexpr uint32_t P1 = 67104769u;  // 0x03fff001 = 32766 * 2^11 + 1
constexpr uint32_t P2 = 67090433u;  // 0x03ffb801 = 32759 * 2^11 + 1

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

static_assert(P1 < (1u << 26) && P2 < (1u << 26), "primes too large for the signed lazy ranges");
static_assert((P1 - 1) % 2048 == 0 && (P2 - 1) % 2048 == 0, "primes need 2048-th roots of unity");
static_assert(Q / 2 > (6ull * 1024 * 64) << 32, "modulus too small for an exact lift");
static_assert(P2 < P1 && 2 * (uint64_t)P1 < 3 * (uint64_t)P2, "CRT difference range");

// Shoup product, unsigned: y * w mod p in [0, 2p), for y < 2^32, w < p,
// wp = floor(w 2^32 / p).
__device__ __forceinline__ uint32_t shoup(uint32_t y, uint32_t w, uint32_t wp, uint32_t p) {
  const uint32_t q = __umulhi(y, wp);
  return w * y - q * p;
}

// Shoup product, signed: y * w mod p in (-p/2, 3p/2) for |y| < 2^31, a
// signed twiddle |w| < p/2 and wq = floor(w 2^32 / p).  With z = y w / p, the
// signed high product q = floor(y wq / 2^32) = floor(z - e) for some
// |e| < 1/2, so y w - q p = p (z - q) and z - q lies in (-1/2, 3/2).  The
// result fits an int32, so the low words of the products give it exactly.
__device__ __forceinline__ uint32_t shoup_s(uint32_t y, uint32_t w, uint32_t wq, uint32_t p) {
  const uint32_t q = (uint32_t)__mulhi((int)y, (int)wq);
  return w * y - q * p;
}

// x mod p in (-p/2, 3p/2) for a signed |x| < 2^31: the signed Shoup product
// by 1 (whose quotient is floor(2^32 / p)).
__device__ __forceinline__ uint32_t reduce_s(uint32_t x, uint32_t p) {
  return shoup_s(x, 1u, (uint32_t)((1ull << 32) / p), p);
}

// x - m if x >= m, else x (for unsigned x < 2m): one subtract and one unsigned min.
__device__ __forceinline__ uint32_t csub(uint32_t x, uint32_t m) { return min(x, x - m); }

// Montgomery reduction of a signed 64-bit T: a representative of
// T * 2^-32 mod p in (floor(T / 2^32) - p, floor(T / 2^32)].  m p agrees with
// T in the low word, so T - m p is an exact multiple of 2^32.
__device__ __forceinline__ uint32_t redc_s(int64_t T, uint32_t p, uint32_t pinv) {
  const uint32_t m = (uint32_t)T * pinv;
  return (uint32_t)(int32_t)(T >> 32) - __umulhi(m, p);
}

// Ranges of the products (magnitudes): forward outputs below 16P times key
// residues below P.  Six of them (one output polynomial) sum below 96 P^2, so
// the high word is below 96 P^2 / 2^32 + 1 and the reduction lies in
// (-4P, 4P); three of them (one half of an output, the four-wavefront
// kernel) reduce into (-2P, 2P), and the two halves' sum again into (-4P, 4P).
static_assert(64 + 10 * (3 * (uint64_t)P1 / 2 + 1) < 16ull * P1, "forward-transform range");
static_assert(((unsigned __int128)96 * P1 * P1 >> 32) + 1 + P1 < 4ull * P1 &&
                  ((unsigned __int128)96 * P2 * P2 >> 32) + 1 + P2 < 4ull * P2,
              "accumulator range (six products)");
static_assert(((unsigned __int128)48 * P1 * P1 >> 32) + 1 + P1 < 2ull * P1 &&
                  ((unsigned __int128)48 * P2 * P2 >> 32) + 1 + P2 < 2ull * P2,
              "accumulator range (three products)");

// Low 32 bits of the centred lift of (x1 mod P1, x2 mod P2) for signed
// residues x1 in (-P1, 2 P1) and x2 in (-P2, 2 P2).  h = (x2 - x1) P1^-1 mod P2
// is made canonical; x = x1 + P1 h is then in (-P1, Q + P1) and congruent to
// the centred integer X (|X| < Q/2) mod Q, so it is X or X + Q, the latter
// exactly when x > Q/2.
__device__ __forceinline__ uint32_t crt_lift_s(uint32_t x1, uint32_t x2) {
  const uint32_t d = x2 - x1 + 4u * P2;                      // = x2 - x1 (mod P2), in (0, 7 P2)
  const uint32_t h = csub(shoup(d, C12, C12_SHOUP, P2), P2);  // [0, P2)
  const int64_t x = (int64_t)P1 * h + (int32_t)x1;
  return (uint32_t)x - (x > (int64_t)(Q / 2) ? (uint32_t)Q : 0u);
}

}  // namespace vlp
