// Arithmetic modulo the Goldilocks prime p = 2^64 - 2^32 + 1 on gfx950.
//
// The exact negacyclic products of the blind rotation run in Z_p: a product
// of a decomposition digit polynomial (|digit| <= 64) with a bootstrapping-key
// polynomial (words < 2^32), summed over 6 rows and 1024 terms, is an integer
// of magnitude < 6 * 1024 * 64 * 2^32 < 2^51 < p/2, so the centred lift of
// the residue recovers it exactly and its low 32 bits are the torus result.
//
// p's shape makes reduction cheap with 32-bit pieces: 2^64 = 2^32 - 1 and
// 2^96 = -1 (mod p).  Values are carried "weakly reduced": any 64-bit word
// standing for its residue; canonical() maps to [0, p) where needed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace vlp {

constexpr uint64_t GL_P = 0xFFFFFFFF00000001ull;
constexpr uint64_t GL_EPS = 0xFFFFFFFFull;  // 2^64 mod p

// Weakly reduced x * y mod p.  The 128-bit product is built from four
// 32x32 -> 64 multiply-adds, then folded: lo + 2^64 * (h0 + 2^32 h1)
// = lo + h0 (2^32 - 1) - h1 (mod p).
__device__ __forceinline__ uint64_t gl_mul(uint64_t x, uint64_t y) {
  const uint32_t x0 = (uint32_t)x, x1 = (uint32_t)(x >> 32);
  const uint32_t y0 = (uint32_t)y, y1 = (uint32_t)(y >> 32);
  const uint64_t p00 = (uint64_t)x0 * y0;
  const uint64_t m0 = (uint64_t)x0 * y1 + (p00 >> 32);
  const uint64_t m1 = (uint64_t)x1 * y0 + (uint32_t)m0;
  const uint64_t hi = (uint64_t)x1 * y1 + (m0 >> 32) + (m1 >> 32);
  const uint64_t lo = ((uint64_t)(uint32_t)m1 << 32) | (uint32_t)p00;
  const uint32_t h0 = (uint32_t)hi, h1 = (uint32_t)(hi >> 32);
  uint64_t t0 = lo - h1;
  if (lo < h1) t0 -= GL_EPS;                       // borrow: wrapped by +2^64 = +EPS
  const uint64_t t1 = ((uint64_t)h0 << 32) - h0;   // h0 * (2^32 - 1), no overflow
  uint64_t r = t0 + t1;
  if (r < t1) r += GL_EPS;                         // carry: dropped 2^64 = EPS
  return r;
}

__device__ __forceinline__ uint64_t gl_canon(uint64_t x) { return x >= GL_P ? x - GL_P : x; }

// a + b for weakly reduced a and canonical b (< p): at most one correction.
__device__ __forceinline__ uint64_t gl_add_wc(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  return s < a ? s + GL_EPS : s;
}
// a - b for weakly reduced a and canonical b (< p): at most one correction.
__device__ __forceinline__ uint64_t gl_sub_wc(uint64_t a, uint64_t b) {
  uint64_t d = a - b;
  return a < b ? d - GL_EPS : d;
}
// a + b, both weakly reduced.
__device__ __forceinline__ uint64_t gl_add(uint64_t a, uint64_t b) {
  uint64_t s = a + b;
  if (s < a) {
    s += GL_EPS;
    if (s < GL_EPS) s += GL_EPS;
  }
  return s;
}
// a - b, both weakly reduced.
__device__ __forceinline__ uint64_t gl_sub(uint64_t a, uint64_t b) {
  uint64_t d = a - b;
  if (a < b) {
    uint64_t e = d - GL_EPS;
    if (d < GL_EPS) e -= GL_EPS;
    d = e;
  }
  return d;
}

// Residue of a signed 32-bit integer.
__device__ __forceinline__ uint64_t gl_from_i32(int32_t v) {
  return v >= 0 ? (uint64_t)v : GL_P - (uint64_t)(uint32_t)(-v);
}

// Low 32 bits of the centred lift of a residue: the integer in (-p/2, p/2)
// congruent to x, reduced mod 2^32.  Since p = 1 (mod 2^32), x - p has low
// word x_lo - 1.
__device__ __forceinline__ uint32_t gl_lift_u32(uint64_t x) {
  x = gl_canon(x);
  return (uint32_t)x - (x > (GL_P >> 1) ? 1u : 0u);
}

}  // namespace vlp
