// Register-resident negacyclic NTT of length 1024 for one 64-lane wavefront,
// computed modulo both primes of rns.h side by side.
//
// Each lane holds 16 coefficients, each as a residue pair (a mod P1, b mod P2).
// The transform is the merged negacyclic Cooley-Tukey form: stage s
// (s = 0..9) pairs elements j and j + (512 >> s) and multiplies by
// psi^brv10(2^s + (j >> (10 - s))), psi a primitive 2048-th root of unity
// mod each prime, brv10 the 10-bit reversal.  Output position k holds the
// evaluation at psi^(2 brv10(k) + 1).  The inverse runs the Gentleman-Sande
// stages in reverse with psi^-1 and no 1/N factor (folded into the key).
// It reads the forward table too: psi^-brv10(2^s + i) = -psi^brv10(2^(s+1) - 1 - i),
// so its stage s uses entry 2^(s+1) - 1 - i with the subtraction reversed.
//
// Butterflies are lazy and work on signed residues (rns.h): the forward
// transform never reduces (each stage raises the magnitude bound by 3P/2:
// digits end below 16P); the inverse takes inputs below 4P in magnitude, lets
// its sums double the bound and reduces them at two of its ten stages
// (inv_reduces), ending below 16P.  Twiddles are signed (|w| < P/2) and
// carry their Shoup quotient floor(w 2^32 / P).
//
// Three register layouts keep every butterfly inside a lane (a = lane & 15,
// h = lane >> 4):
//   A (coefficient order): j = 64 r + lane                                  stages 0..3
//   Y                      : j = 64 a + 4 r + h                              stages 4..7
//   Z (transform order)    : j = 64 a + 16 h + 4 (r & 3) + (r >> 2)          stages 8, 9
// An LDS transpose moves between A and Y (in LDS, element j sits at slot
// lds_slot(j), which spreads both access patterns over distinct banks); Y and
// Z differ only in two exchanged bit pairs, which the lane-swap instructions
// move in registers (swap_yz).
#pragma once
#include <type_traits>

#include "rns.h"

namespace vlp {

// Twiddle table entry: {w1, Shoup(w1), w2, Shoup(w2)}, w_i the signed
// representative (|w_i| < P_i / 2) of the twiddle mod P_i.
using Tw = uint4;

__device__ __forceinline__ int lay_a(int lane, int r) { return r * 64 + lane; }
__device__ __forceinline__ int lay_y(int lane, int r) { return ((lane & 15) << 6) | (r << 2) | (lane >> 4); }
__device__ __forceinline__ int lay_z(int lane, int r) {
  return ((lane & 15) << 6) | ((lane >> 4) << 4) | ((r & 3) << 2) | (r >> 2);
}
// LDS slot of element j: a bijection on each block of 64 (bits 1..4 take the
// block index, bit 5 takes bit 1).  Writes in layout A (one block per
// register, every lane a distinct slot of it) and reads in layout Y (64 a + 4 r
// + h: a and h vary over the lanes) both touch 64 distinct banks, and 32
// distinct ones in each half of the wavefront.
__device__ __forceinline__ int lds_slot(int j) { return j ^ (((j >> 6) & 15) << 1) ^ (((j >> 1) & 1) << 5); }

// Orders LDS accesses of one wavefront across its lanes.  The LDS performs
// one wavefront's operations in issue order, so a later read sees every
// lane's earlier write without waiting for it: the fences and the barrier
// only keep the compiler from moving accesses across this point.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct Poly2 {
  uint32_t a[16];  // residues mod P1
  uint32_t b[16];  // residues mod P2
};

template <int (*FROM)(int, int), int (*TO)(int, int)>
__device__ __forceinline__ void wave_transpose(Poly2& v, uint2* buf, int lane) {
  wave_lds_sync();  // earlier readers of buf are done
#pragma unroll
  for (int r = 0; r < 16; ++r) buf[lds_slot(FROM(lane, r))] = make_uint2(v.a[r], v.b[r]);
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const uint2 t = buf[lds_slot(TO(lane, r))];
    v.a[r] = t.x;
    v.b[r] = t.y;
  }
}

// Cooley-Tukey: (x, y) -> (x + w y, x - w y) with w y taken in (-P/2, 3P/2):
// for |x| below B (any |y| < 2^31) both outputs are below B + 3P/2 in
// magnitude.  No reduction.
__device__ __forceinline__ void bfly_ct(uint32_t& x, uint32_t& y, uint32_t w, uint32_t wq, uint32_t p) {
  const uint32_t u = x;
  const uint32_t t = shoup_s(y, w, wq, p);
  x = u + t;
  y = u - t;
}
// Gentleman-Sande with a negated twiddle -w: (x, y) -> (x + y, (y - x) w) for
// inputs below B P in magnitude.  The product is in (-P/2, 3P/2); the sum is
// below 2B P, or with RED reduced into (-P/2, 3P/2).
template <int B, bool RED>
__device__ __forceinline__ void bfly_gs_neg(uint32_t& x, uint32_t& y, uint32_t w, uint32_t wq, uint32_t p) {
  const uint32_t u = x, v = y;
  x = RED ? reduce_s(u + v, p) : u + v;
  y = shoup_s(v - u, w, wq, p);
}

// Bounds of the inverse stages (run from S = 9 down to 0), in multiples of P:
// the magnitude bound of stage S's inputs and whether it reduces its sums.
// Inputs start below 4P; a stage's outputs are below twice its input bound,
// or 2P if it reduces; no sum or difference reaches 32P.  The outputs end
// below 16P, the range the CRT lift takes (rns.h).
__host__ __device__ constexpr int inv_bound(int S) {
  return S == 9 ? 4 : S == 8 ? 8 : S == 7 ? 16 : S == 6 ? 2 : S == 5 ? 4 : S == 4 ? 8 : S == 3 ? 16 : S == 2 ? 2 : S == 1 ? 4 : 8;
}
__host__ __device__ constexpr bool inv_reduces(int S) { return S == 7 || S == 3; }
__host__ __device__ constexpr bool inv_bounds_hold() {
  for (int S = 9; S >= 0; --S) {
    if (2 * inv_bound(S) > 32) return false;
    const int out = inv_reduces(S) ? 2 : 2 * inv_bound(S);
    if (S > 0 && inv_bound(S - 1) != out) return false;
    if (S == 0 && out > 16) return false;
  }
  return inv_bound(9) == 4;
}
static_assert(inv_bounds_hold(), "inverse-transform ranges");
static_assert(32ull * P1 < (1ull << 31) && 32ull * P2 < (1ull << 31), "inverse sums overflow");

// Stages 0..3 read wavefront-uniform twiddles into scalar registers.  A
// signed high product with a scalar operand is expanded by the compiler into
// an unsigned one plus two sign corrections (four extra instructions per
// butterfly); a copy of the quotient into a vector register (one move per
// distinct twiddle) keeps it to one v_mul_hi_i32.
__device__ __forceinline__ void vgpr_quotient(uint32_t& wq) { asm("" : "+v"(wq)); }

// The eight butterflies of a stage: register r (bit RB clear) pairs with
// r | 2^RB.  All twiddle reads of the stage are issued before the first
// butterfly (the scheduling barrier keeps the compiler from sinking them to
// their uses), so the stage waits for one LDS round trip, not one per read.
template <int RB>
__device__ __forceinline__ constexpr int bfly_reg(int k) {
  return ((k >> RB) << (RB + 1)) | (k & ((1 << RB) - 1));
}
// Layouts Y and Z differ in two exchanged bit pairs: lane bit 5 with
// register bit 3 and lane bit 4 with register bit 2.  The lane-swap
// instructions exchange such a pair for two registers at once:
// permlane32_swap moves the upper 32 lanes of its first register and the lower
// 32 lanes of its second past each other, permlane16_swap the odd rows of 16
// lanes of its first and the even rows of its second.  The exchange is its
// own inverse, so it serves Y -> Z and Z -> Y alike.
__device__ __forceinline__ void swap_yz(uint32_t (&x)[16]) {
#pragma unroll
  for (int r = 0; r < 8; ++r) {  // register bit 3 <-> lane bit 5
    const auto t = __builtin_amdgcn_permlane32_swap(x[r], x[r | 8], false, false);
    x[r] = t[0];
    x[r | 8] = t[1];
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // register bit 2 <-> lane bit 4
    const int r = bfly_reg<2>(k);
    const auto t = __builtin_amdgcn_permlane16_swap(x[r], x[r | 4], false, false);
    x[r] = t[0];
    x[r | 4] = t[1];
  }
}
__device__ __forceinline__ void swap_yz(Poly2& v) {
  swap_yz(v.a);
  swap_yz(v.b);
}

template <int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ void fwd_stage(Poly2& v, const Tw* tw, int lane) {
  Tw w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    w[k] = tw[(1 << S) + (LAY(lane, bfly_reg<RB>(k)) >> (10 - S))];
    if (S < 4) vgpr_quotient(w[k].y), vgpr_quotient(w[k].w);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int r = bfly_reg<RB>(k);
    bfly_ct(v.a[r], v.a[r | (1 << RB)], w[k].x, w[k].y, P1);
    bfly_ct(v.b[r], v.b[r | (1 << RB)], w[k].z, w[k].w, P2);
  }
}
template <int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ void inv_stage(Poly2& v, const Tw* tw, int lane) {
  Tw w[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    w[k] = tw[(2 << S) - 1 - (LAY(lane, bfly_reg<RB>(k)) >> (10 - S))];
    if (S < 4) vgpr_quotient(w[k].y), vgpr_quotient(w[k].w);
  }
  __builtin_amdgcn_sched_barrier(0);
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int r = bfly_reg<RB>(k);
    bfly_gs_neg<inv_bound(S), inv_reduces(S)>(v.a[r], v.a[r | (1 << RB)], w[k].x, w[k].y, P1);
    bfly_gs_neg<inv_bound(S), inv_reduces(S)>(v.b[r], v.b[r | (1 << RB)], w[k].z, w[k].w, P2);
  }
}

// Forward: layout A (coefficient order, |values| <= 64) -> layout Z (transform order, |values| < 16P).
// Stages 0..3 use wavefront-uniform twiddles (their index depends only on the
// register), read through `gtw` (the table in global memory: scalar loads into
// SGPRs); the other stages read the LDS copy `tw` per lane.
__device__ __forceinline__ void ntt_fwd(Poly2& v, uint2* buf, const Tw* tw, const Tw* __restrict__ gtw, int lane) {
  fwd_stage<0, lay_a, 3>(v, gtw, lane);
  fwd_stage<1, lay_a, 2>(v, gtw, lane);
  fwd_stage<2, lay_a, 1>(v, gtw, lane);
  fwd_stage<3, lay_a, 0>(v, gtw, lane);
  wave_transpose<lay_a, lay_y>(v, buf, lane);
  fwd_stage<4, lay_y, 3>(v, tw, lane);
  fwd_stage<5, lay_y, 2>(v, tw, lane);
  fwd_stage<6, lay_y, 1>(v, tw, lane);
  fwd_stage<7, lay_y, 0>(v, tw, lane);
  swap_yz(v);  // layout Y -> Z
  fwd_stage<8, lay_z, 3>(v, tw, lane);
  fwd_stage<9, lay_z, 2>(v, tw, lane);
}

// Inverse without 1/N: layout Z (|values| < 4P) -> layout A (|values| < 16P).
__device__ __forceinline__ void ntt_inv(Poly2& v, uint2* buf, const Tw* tw, const Tw* __restrict__ gtw, int lane) {
  inv_stage<9, lay_z, 2>(v, tw, lane);
  inv_stage<8, lay_z, 3>(v, tw, lane);
  swap_yz(v);  // layout Z -> Y
  inv_stage<7, lay_y, 0>(v, tw, lane);
  inv_stage<6, lay_y, 1>(v, tw, lane);
  inv_stage<5, lay_y, 2>(v, tw, lane);
  inv_stage<4, lay_y, 3>(v, tw, lane);
  wave_transpose<lay_y, lay_a>(v, buf, lane);
  inv_stage<3, lay_a, 0>(v, gtw, lane);
  inv_stage<2, lay_a, 1>(v, gtw, lane);
  inv_stage<1, lay_a, 2>(v, gtw, lane);
  inv_stage<0, lay_a, 3>(v, gtw, lane);
}

// ---------------------------------------------------------------------------
// Single-prime form: one wavefront transforms the residues of one prime
// (two wavefronts per blind rotation).  Same stages, layouts and twiddle
// table (entry e of prime PR is the uint2 at index 2e + PR of the table).
// ---------------------------------------------------------------------------
template <int PR>
struct Prime;
template <>
struct Prime<0> {
  static constexpr uint32_t P = P1, PINV = P1_INV;
};
template <>
struct Prime<1> {
  static constexpr uint32_t P = P2, PINV = P2_INV;
};

// LDS word of element j in a single-prime transpose buffer: a bijection on
// [0, 1024) that puts j and j + 64 (registers 2k and 2k + 1 of one lane in
// layout A) in one aligned pair of words, so that side of a transpose moves
// two registers per 64-bit access.  Word bits: 0 = j6, 1..2 = j0..1,
// 3..5 = (j2..4 xor j7..9), 6 = j5, 7..9 = j7..9.  The 64-bit accesses of each
// half-wavefront in layout A and the 32-bit accesses of the wavefront in
// layout Y each touch all 64 banks once.
__device__ __forceinline__ int lds_slot1(int j) {
  return ((j >> 6) & 1) | ((j & 3) << 1) | ((((j >> 2) ^ (j >> 7)) & 7) << 3) | (((j >> 5) & 1) << 6) |
         (j & 0x380);
}

// Layout A -> Y and Y -> A through the wavefront's 8-byte-aligned LDS buffer.
__device__ __forceinline__ void transpose_a_to_y(uint32_t (&x)[16], uint32_t* buf, int lane) {
  wave_lds_sync();  // earlier readers of buf are done
#pragma unroll
  for (int k = 0; k < 8; ++k)
    *reinterpret_cast<uint2*>(buf + lds_slot1(lay_a(lane, 2 * k))) = make_uint2(x[2 * k], x[2 * k + 1]);
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = buf[lds_slot1(lay_y(lane, r))];
}
__device__ __forceinline__ void transpose_y_to_a(uint32_t (&x)[16], uint32_t* buf, int lane) {
  wave_lds_sync();  // earlier readers of buf are done
#pragma unroll
  for (int r = 0; r < 16; ++r) buf[lds_slot1(lay_y(lane, r))] = x[r];
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint2 t = *reinterpret_cast<const uint2*>(buf + lds_slot1(lay_a(lane, 2 * k)));
    x[2 * k] = t.x;
    x[2 * k + 1] = t.y;
  }
}

// Position of twiddle-table entry 2^S + o inside stage S's slice of a
// per-prime LDS plane.  Stage S >= 4 reads entry offsets o = j >> (10 - S)
// whose top bits hold lane bits (a = lane & 15 in layout Y; a and h = lane >> 4
// in layout Z) above bits set by the register index (c); the permutation
// moves the lane bits to the bottom, so for every butterfly slot the lanes
// read one contiguous run of entries (no bank conflicts).  A bijection on
// [0, 2^S) for every S.
__host__ __device__ __forceinline__ constexpr int tw_perm(int S, int o) {
  return S < 4    ? o
         : S <= 7 ? (((o & ((1 << (S - 4)) - 1)) << 4) | (o >> (S - 4)))          // o = a | c
         : S == 8 ? (((o & 3) << 6) | (((o >> 2) & 3) << 4) | ((o >> 4) & 15))      // o = a | h | c (2 bits)
                  : (((o & 7) << 6) | (((o >> 3) & 3) << 4) | ((o >> 5) & 15));     // o = a | h | c (3 bits)
}

// Calls f(std::integral_constant<int, k>) for k = 0..7.
template <class F>
__device__ __forceinline__ void for8(F&& f) {
  f(std::integral_constant<int, 0>{});
  f(std::integral_constant<int, 1>{});
  f(std::integral_constant<int, 2>{});
  f(std::integral_constant<int, 3>{});
  f(std::integral_constant<int, 4>{});
  f(std::integral_constant<int, 5>{});
  f(std::integral_constant<int, 6>{});
  f(std::integral_constant<int, 7>{});
}

// Signed Shoup product by a compile-time twiddle: the quotient stays a scalar
// operand of the high multiply (an SGPR constant, no vector register copy).
template <uint32_t W, uint32_t WQ, uint32_t P>
__device__ __forceinline__ uint32_t shoup_c(uint32_t y) {
  uint32_t q;
  asm("v_mul_hi_i32 %0, %1, %2" : "=v"(q) : "v"(y), "s"(WQ));
  return W * y - q * P;
}

// Stages 0..3 work in layout A (j = 64 r + lane), where entry 2^S + (j >> (10 - S))
// = 2^S + (r >> (4 - S)) depends only on the register: the twiddles are
// compile-time constants.  Stages 4..9 read this prime's permuted LDS plane tws.
template <int PR, int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ void fwd_stage1(uint32_t (&x)[16], const uint2* tws, int lane) {
  constexpr uint32_t P = Prime<PR>::P;
  if constexpr (S < 4) {
    for8([&](auto kc) {
      constexpr int r = bfly_reg<RB>(decltype(kc)::value);
      constexpr TwPair c = twiddle(P, PR ? PSI2 : PSI1, (1u << S) + (uint32_t)(r >> (4 - S)));
      const uint32_t u = x[r], t = shoup_c<c.w, c.q, P>(x[r | (1 << RB)]);
      x[r] = u + t;
      x[r | (1 << RB)] = u - t;
    });
  } else {
    uint2 w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) w[k] = tws[(1 << S) + tw_perm(S, LAY(lane, bfly_reg<RB>(k)) >> (10 - S))];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = bfly_reg<RB>(k);
      bfly_ct(x[r], x[r | (1 << RB)], w[k].x, w[k].y, P);
    }
  }
}
template <int PR, int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ void inv_stage1(uint32_t (&x)[16], const uint2* tws, int lane) {
  constexpr uint32_t P = Prime<PR>::P;
  if constexpr (S < 4) {
    for8([&](auto kc) {
      constexpr int r = bfly_reg<RB>(decltype(kc)::value);
      constexpr TwPair c = twiddle(P, PR ? PSI2 : PSI1, (2u << S) - 1 - (uint32_t)(r >> (4 - S)));
      const uint32_t u = x[r], v = x[r | (1 << RB)];
      x[r] = inv_reduces(S) ? reduce_s(u + v, P) : u + v;
      x[r | (1 << RB)] = shoup_c<c.w, c.q, P>(v - u);
    });
  } else {
    uint2 w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      w[k] = tws[(1 << S) + tw_perm(S, (1 << S) - 1 - (LAY(lane, bfly_reg<RB>(k)) >> (10 - S)))];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = bfly_reg<RB>(k);
      bfly_gs_neg<inv_bound(S), inv_reduces(S)>(x[r], x[r | (1 << RB)], w[k].x, w[k].y, P);
    }
  }
}

// Twiddle of butterfly k of forward stage S >= 4 (layout LAY, register bit
// RB) in this prime's permuted LDS plane tws.
template <int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ uint2 fwd_tw(const uint2* tws, int lane, int k) {
  return tws[(1 << S) + tw_perm(S, LAY(lane, bfly_reg<RB>(k)) >> (10 - S))];
}
// Forward transform, single prime; tws: this prime's permuted LDS plane
// (stages 4..9).  A wavefront's LDS reads return in issue order, so a
// twiddle read issued behind the transpose's reads comes back after all of
// them and holds up stage 4, which could otherwise start on each register
// pair as it arrives.  The twiddles of stages 4 and 5 are read before the
// transpose, those of stage 6 right behind it (needed only after stages 4
// and 5), those of stages 8 and 9 before the lane swaps of the Y -> Z move;
// stage 7 reads its own.  Per lane, stages 4..9 use 1, 2, 4, 8, 4, 8
// distinct twiddles: butterfly k of stage 5 shares with k & 4, of stage 6
// with k & 6, of stage 8 with k & 3.  (11.37 -> 10.85-10.97 ms per launch of
// the blind rotation against every stage reading its own.)
template <int PR>
__device__ __forceinline__ void ntt_fwd1(uint32_t (&x)[16], uint32_t* buf, const uint2* tws, int lane) {
  constexpr uint32_t P = Prime<PR>::P;
  const uint2 t4 = fwd_tw<4, lay_y, 3>(tws, lane, 0);
  const uint2 t5a = fwd_tw<5, lay_y, 2>(tws, lane, 0), t5b = fwd_tw<5, lay_y, 2>(tws, lane, 4);
  fwd_stage1<PR, 0, lay_a, 3>(x, tws, lane);
  fwd_stage1<PR, 1, lay_a, 2>(x, tws, lane);
  fwd_stage1<PR, 2, lay_a, 1>(x, tws, lane);
  fwd_stage1<PR, 3, lay_a, 0>(x, tws, lane);
  transpose_a_to_y(x, buf, lane);
  uint2 t6[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) t6[k] = fwd_tw<6, lay_y, 1>(tws, lane, 2 * k);
#pragma unroll
  for (int k = 0; k < 8; ++k) bfly_ct(x[k], x[k | 8], t4.x, t4.y, P);  // stage 4 (register bit 3)
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // stage 5 (register bit 2)
    const int r = bfly_reg<2>(k);
    const uint2 w = r < 8 ? t5a : t5b;
    bfly_ct(x[r], x[r | 4], w.x, w.y, P);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // stage 6 (register bit 1)
    const int r = bfly_reg<1>(k);
    bfly_ct(x[r], x[r | 2], t6[k >> 1].x, t6[k >> 1].y, P);
  }
  fwd_stage1<PR, 7, lay_y, 0>(x, tws, lane);
  uint2 t8[4], t9[8];
#pragma unroll
  for (int k = 0; k < 4; ++k) t8[k] = fwd_tw<8, lay_z, 3>(tws, lane, k);
#pragma unroll
  for (int k = 0; k < 8; ++k) t9[k] = fwd_tw<9, lay_z, 2>(tws, lane, k);
  swap_yz(x);  // layout Y -> Z
#pragma unroll
  for (int k = 0; k < 8; ++k) bfly_ct(x[k], x[k | 8], t8[k & 3].x, t8[k & 3].y, P);  // stage 8 (register bit 3)
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // stage 9 (register bit 2)
    const int r = bfly_reg<2>(k);
    bfly_ct(x[r], x[r | 4], t9[k].x, t9[k].y, P);
  }
}

// Twiddle of butterfly k of inverse stage S >= 4 (layout LAY, register bit
// RB) in this prime's permuted LDS plane tws.
template <int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ uint2 inv_tw(const uint2* tws, int lane, int k) {
  return tws[(1 << S) + tw_perm(S, (1 << S) - 1 - (LAY(lane, bfly_reg<RB>(k)) >> (10 - S)))];
}
// The twiddles of inverse stages 9 (eight per lane) and 8 (four: butterfly k
// shares with k & 3), for a caller that reads them ahead of other LDS reads
// the first stages must not wait behind.
struct InvTw98 {
  uint2 s9[8], s8[4];
};
__device__ __forceinline__ void inv_tw98_load(InvTw98& w, const uint2* tws, int lane) {
#pragma unroll
  for (int k = 0; k < 8; ++k) w.s9[k] = inv_tw<9, lay_z, 2>(tws, lane, k);
#pragma unroll
  for (int k = 0; k < 4; ++k) w.s8[k] = inv_tw<8, lay_z, 3>(tws, lane, k);
}

// Inverse transform, single prime (layout Z, |values| < 4P -> layout A, |values|
// < 16P), whose stages 9 and 8 take the twiddles read by inv_tw98_load.
template <int PR>
__device__ __forceinline__ void ntt_inv1(uint32_t (&x)[16], const InvTw98& w, uint32_t* buf, const uint2* tws,
                                         int lane) {
  constexpr uint32_t P = Prime<PR>::P;
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // stage 9 (register bit 2)
    const int r = bfly_reg<2>(k);
    bfly_gs_neg<inv_bound(9), inv_reduces(9)>(x[r], x[r | 4], w.s9[k].x, w.s9[k].y, P);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k)  // stage 8 (register bit 3)
    bfly_gs_neg<inv_bound(8), inv_reduces(8)>(x[k], x[k | 8], w.s8[k & 3].x, w.s8[k & 3].y, P);
  swap_yz(x);  // layout Z -> Y
  inv_stage1<PR, 7, lay_y, 0>(x, tws, lane);
  inv_stage1<PR, 6, lay_y, 1>(x, tws, lane);
  inv_stage1<PR, 5, lay_y, 2>(x, tws, lane);
  inv_stage1<PR, 4, lay_y, 3>(x, tws, lane);
  transpose_y_to_a(x, buf, lane);
  inv_stage1<PR, 3, lay_a, 0>(x, tws, lane);
  inv_stage1<PR, 2, lay_a, 1>(x, tws, lane);
  inv_stage1<PR, 1, lay_a, 2>(x, tws, lane);
  inv_stage1<PR, 0, lay_a, 3>(x, tws, lane);
}

// ---------------------------------------------------------------------------
// Two inverse transforms of one prime side by side (the two output
// polynomials of a CMux): every stage reads its twiddles once for both, and
// the two Y -> A transposes share one LDS round trip (bufx, bufy: the
// wavefront's two 8-byte-aligned buffers).
// ---------------------------------------------------------------------------
template <int PR, int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ void inv_stage1_pair(uint32_t (&x)[16], uint32_t (&y)[16], const uint2* tws, int lane) {
  constexpr uint32_t P = Prime<PR>::P;
  if constexpr (S < 4) {
    for8([&](auto kc) {
      constexpr int r = bfly_reg<RB>(decltype(kc)::value);
      constexpr TwPair c = twiddle(P, PR ? PSI2 : PSI1, (2u << S) - 1 - (uint32_t)(r >> (4 - S)));
      const uint32_t u = x[r], v = x[r | (1 << RB)], u2 = y[r], v2 = y[r | (1 << RB)];
      x[r] = inv_reduces(S) ? reduce_s(u + v, P) : u + v;
      x[r | (1 << RB)] = shoup_c<c.w, c.q, P>(v - u);
      y[r] = inv_reduces(S) ? reduce_s(u2 + v2, P) : u2 + v2;
      y[r | (1 << RB)] = shoup_c<c.w, c.q, P>(v2 - u2);
    });
  } else {
    uint2 w[8];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      w[k] = tws[(1 << S) + tw_perm(S, (1 << S) - 1 - (LAY(lane, bfly_reg<RB>(k)) >> (10 - S)))];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int r = bfly_reg<RB>(k);
      bfly_gs_neg<inv_bound(S), inv_reduces(S)>(x[r], x[r | (1 << RB)], w[k].x, w[k].y, P);
      bfly_gs_neg<inv_bound(S), inv_reduces(S)>(y[r], y[r | (1 << RB)], w[k].x, w[k].y, P);
    }
  }
}

__device__ __forceinline__ void transpose_y_to_a_pair(uint32_t (&x)[16], uint32_t (&y)[16], uint32_t* bufx,
                                                      uint32_t* bufy, int lane) {
  wave_lds_sync();  // earlier readers of the buffers are done
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    bufx[lds_slot1(lay_y(lane, r))] = x[r];
    bufy[lds_slot1(lay_y(lane, r))] = y[r];
  }
  wave_lds_sync();
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const uint2 t = *reinterpret_cast<const uint2*>(bufx + lds_slot1(lay_a(lane, 2 * k)));
    const uint2 u = *reinterpret_cast<const uint2*>(bufy + lds_slot1(lay_a(lane, 2 * k)));
    x[2 * k] = t.x;
    x[2 * k + 1] = t.y;
    y[2 * k] = u.x;
    y[2 * k + 1] = u.y;
  }
}

template <int PR>
__device__ __forceinline__ void ntt_inv1_pair(uint32_t (&x)[16], uint32_t (&y)[16], uint32_t* bufx, uint32_t* bufy,
                                              const uint2* tws, int lane) {
  inv_stage1_pair<PR, 9, lay_z, 2>(x, y, tws, lane);
  inv_stage1_pair<PR, 8, lay_z, 3>(x, y, tws, lane);
  swap_yz(x);  // layout Z -> Y
  swap_yz(y);
  inv_stage1_pair<PR, 7, lay_y, 0>(x, y, tws, lane);
  inv_stage1_pair<PR, 6, lay_y, 1>(x, y, tws, lane);
  inv_stage1_pair<PR, 5, lay_y, 2>(x, y, tws, lane);
  inv_stage1_pair<PR, 4, lay_y, 3>(x, y, tws, lane);
  transpose_y_to_a_pair(x, y, bufx, bufy, lane);
  inv_stage1_pair<PR, 3, lay_a, 0>(x, y, tws, lane);
  inv_stage1_pair<PR, 2, lay_a, 1>(x, y, tws, lane);
  inv_stage1_pair<PR, 1, lay_a, 2>(x, y, tws, lane);
  inv_stage1_pair<PR, 0, lay_a, 3>(x, y, tws, lane);
}

}  // namespace vlp
