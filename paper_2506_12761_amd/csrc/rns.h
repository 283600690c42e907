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
//   - the inverse transform reduces only at two of its ten stages: a
//     Gentleman-Sande sum doubles the bound, and inputs below 4P may double
//     three times (32P < 2^31) before a Shoup product by 1 brings them back
//     into (-P/2, 3P/2); its outputs, below 16P, go to the lift unreduced.
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

// Twiddles: psi_p, the 2048-th root of unity g^((p-1)/2048) of the smallest
// generator g mod p; entry m is psi_p^brv10(m) as its signed representative
// w in (-p/2, p/2) with floor(w 2^32 / p) (rounded down for negative w).  The
// host table (twiddles.cpp) and the kernels' compile-time constants of the
// first four stages both come from these.
constexpr uint32_t brv10(uint32_t x) {
  uint32_t r = 0;
  for (int i = 0; i < 10; ++i) r |= ((x >> i) & 1u) << (9 - i);
  return r;
}
constexpr uint64_t smallest_generator(uint64_t p) {
  uint64_t f[16] = {};
  int nf = 0;
  uint64_t n = p - 1;
  for (uint64_t d = 2; d * d <= n; ++d)
    if (n % d == 0) {
      f[nf++] = d;
      while (n % d == 0) n /= d;
    }
  if (n > 1) f[nf++] = n;
  for (uint64_t g = 2;; ++g) {
    bool ok = true;
    for (int i = 0; i < nf; ++i) ok = ok && pow_mod(g, (p - 1) / f[i], p) != 1;
    if (ok) return g;
  }
}
constexpr uint64_t root_2048(uint64_t p) { return pow_mod(smallest_generator(p), (p - 1) / 2048, p); }
struct TwPair {
  uint32_t w, q;  // signed twiddle and its signed Shoup quotient, as words
};
constexpr TwPair twiddle(uint64_t p, uint64_t psi, uint32_t m) {
  const int64_t w0 = (int64_t)pow_mod(psi, brv10(m), p);
  const int64_t w = w0 > (int64_t)p / 2 ? w0 - (int64_t)p : w0;
  const int64_t n = w * ((int64_t)1 << 32);
  const int64_t q = n / (int64_t)p - ((n % (int64_t)p != 0 && n < 0) ? 1 : 0);
  return TwPair{(uint32_t)(int32_t)w, (uint32_t)(int32_t)q};
}
constexpr uint64_t PSI1 = root_2048(P1), PSI2 = root_2048(P2);
static_assert(pow_mod(PSI1, 1024, P1) == P1 - 1 && pow_mod(PSI2, 1024, P2) == P2 - 1, "psi of order 2048");

// Entries 0..15 of each prime's table (the twiddles of stages 0..3).
struct TwHead {
  TwPair e[2][16];
};
constexpr TwHead make_tw_head() {
  TwHead t{};
  for (uint32_t m = 0; m < 16; ++m) {
    t.e[0][m] = twiddle(P1, PSI1, m);
    t.e[1][m] = twiddle(P2, PSI2, m);
  }
  return t;
}

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

// C12 as a signed representative (|C12S| < P2/2) with its signed Shoup quotient.
constexpr int64_t C12S = C12 > P2 / 2 ? (int64_t)C12 - P2 : (int64_t)C12;
constexpr int64_t C12S_Q = (C12S * ((int64_t)1 << 32) - ((C12S * ((int64_t)1 << 32)) % P2 + P2) % P2) / P2;

// Low 32 bits of the centred lift of (x1 mod P1, x2 mod P2) for signed
// residues |x1| < 16 P1 and |x2| < 16 P2 (so |x2 - x1| < 32 P1 < 2^31).  With
// h = (x2 - x1) P1^-1 mod P2 taken in (-P2/2, 3 P2/2) (one signed Shoup
// product), the integer X (|X| < 6 * 1024 * 64 * 2^32 < 0.37513 Q) is
// x1 + P1 h, or that minus Q: in the first case h < 0.37513 P2 + 16, in the
// second h > 0.62487 P2 - 16, so h > P2/2 tells them apart and only the low
// words are needed.
static_assert((6.0 * 1024 * 64 * 4294967296.0) / ((double)P1 * (double)P2) < 0.37513 &&
                  0.37513 * P2 + 16 < P2 / 2 && 0.62487 * P2 - 16 > P2 / 2 && 32ull * P1 < (1ull << 31),
              "CRT lift decision range");
__device__ __forceinline__ uint32_t crt_lift_s(uint32_t x1, uint32_t x2) {
  const uint32_t h = shoup_s(x2 - x1, (uint32_t)(int32_t)C12S, (uint32_t)(int32_t)C12S_Q, P2);
  const uint32_t lo = h * P1 + x1;
  return (int32_t)h > (int32_t)(P2 / 2) ? lo - (uint32_t)Q : lo;
}

}  // namespace vlp
