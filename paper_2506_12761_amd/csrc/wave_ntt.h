// Register-resident negacyclic NTT of length 1024 for one 64-lane wavefront.
//
// Each lane holds 16 coefficients (two VGPRs each).  The transform is the
// merged negacyclic Cooley-Tukey form: stage s (s = 0..9) pairs the elements
// j and j + (512 >> s) and multiplies by psi^brv10(2^s + (j >> (10 - s))),
// where psi is a primitive 2048-th root of unity mod p and brv10 reverses 10
// bits.  The output at position k is the evaluation at psi^(2 brv10(k) + 1);
// the inverse runs the Gentleman-Sande stages in reverse with psi^-1 and no
// 1/N factor (the caller folds 1/N into the operand it multiplies by).
//
// Three register layouts keep every butterfly inside a lane; two LDS
// transposes per transform move between them:
//   A (coefficient order): j = 64 r + lane                 stages 0..3
//   B                      : j = 64 (lane>>2) + 4 r + (lane&3)      4..7
//   C (transform order)    : j = 64 (lane>>2) + 16 (r>>2) + 4 (lane&3) + (r&3)  8, 9
// In LDS, element j sits at j ^ ((j >> 6) & 15), which spreads every one of
// the three access patterns evenly over the banks.
#pragma once
#include "gl64.h"

namespace vlp {

__device__ __forceinline__ int lay_a(int lane, int r) { return r * 64 + lane; }
__device__ __forceinline__ int lay_b(int lane, int r) { return ((lane >> 2) << 6) | (r << 2) | (lane & 3); }
__device__ __forceinline__ int lay_c(int lane, int r) {
  return ((lane >> 2) << 6) | ((r >> 2) << 4) | ((lane & 3) << 2) | (r & 3);
}
__device__ __forceinline__ int lds_slot(int j) { return j ^ ((j >> 6) & 15); }

// Orders LDS accesses of one wavefront: every lane's earlier LDS writes are
// complete and visible before any later LDS read is issued.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int (*FROM)(int, int), int (*TO)(int, int)>
__device__ __forceinline__ void wave_transpose(uint64_t (&v)[16], uint64_t* buf, int lane) {
  wave_lds_sync();  // previous readers of buf are done
#pragma unroll
  for (int r = 0; r < 16; ++r) buf[lds_slot(FROM(lane, r))] = v[r];
  wave_lds_sync();
#pragma unroll
  for (int r = 0; r < 16; ++r) v[r] = buf[lds_slot(TO(lane, r))];
}

// Cooley-Tukey butterfly: (x, y) -> (x + w y, x - w y).
__device__ __forceinline__ void bfly_ct(uint64_t& x, uint64_t& y, uint64_t w) {
  const uint64_t t = gl_canon(gl_mul(y, w));
  const uint64_t a = x;
  x = gl_add_wc(a, t);
  y = gl_sub_wc(a, t);
}
// Gentleman-Sande butterfly: (x, y) -> (x + y, (x - y) w).
__device__ __forceinline__ void bfly_gs(uint64_t& x, uint64_t& y, uint64_t w) {
  const uint64_t a = x, b = y;
  x = gl_add(a, b);
  y = gl_mul(gl_sub(a, b), w);
}

// tw: psi^brv10(m) for m < 1024 (LDS or global).
template <int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ void fwd_stage(uint64_t (&v)[16], const uint64_t* tw, int lane) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << RB)) continue;
    const int j = LAY(lane, r);
    bfly_ct(v[r], v[r | (1 << RB)], tw[(1 << S) + (j >> (10 - S))]);
  }
}
template <int S, int (*LAY)(int, int), int RB>
__device__ __forceinline__ void inv_stage(uint64_t (&v)[16], const uint64_t* tw_inv, int lane) {
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    if (r & (1 << RB)) continue;
    const int j = LAY(lane, r);
    bfly_gs(v[r], v[r | (1 << RB)], tw_inv[(1 << S) + (j >> (10 - S))]);
  }
}

// Forward: v in layout A (coefficient order) -> layout C (transform order).
// Input values must be canonical (< p).
__device__ __forceinline__ void ntt_fwd(uint64_t (&v)[16], uint64_t* buf, const uint64_t* tw, int lane) {
  fwd_stage<0, lay_a, 3>(v, tw, lane);
  fwd_stage<1, lay_a, 2>(v, tw, lane);
  fwd_stage<2, lay_a, 1>(v, tw, lane);
  fwd_stage<3, lay_a, 0>(v, tw, lane);
  wave_transpose<lay_a, lay_b>(v, buf, lane);
  fwd_stage<4, lay_b, 3>(v, tw, lane);
  fwd_stage<5, lay_b, 2>(v, tw, lane);
  fwd_stage<6, lay_b, 1>(v, tw, lane);
  fwd_stage<7, lay_b, 0>(v, tw, lane);
  wave_transpose<lay_b, lay_c>(v, buf, lane);
  fwd_stage<8, lay_c, 1>(v, tw, lane);
  fwd_stage<9, lay_c, 0>(v, tw, lane);
}

// Inverse (without 1/N): v in layout C -> layout A.  Weakly reduced in/out.
__device__ __forceinline__ void ntt_inv(uint64_t (&v)[16], uint64_t* buf, const uint64_t* tw_inv, int lane) {
  inv_stage<9, lay_c, 0>(v, tw_inv, lane);
  inv_stage<8, lay_c, 1>(v, tw_inv, lane);
  wave_transpose<lay_c, lay_b>(v, buf, lane);
  inv_stage<7, lay_b, 0>(v, tw_inv, lane);
  inv_stage<6, lay_b, 1>(v, tw_inv, lane);
  inv_stage<5, lay_b, 2>(v, tw_inv, lane);
  inv_stage<4, lay_b, 3>(v, tw_inv, lane);
  wave_transpose<lay_b, lay_a>(v, buf, lane);
  inv_stage<3, lay_a, 0>(v, tw_inv, lane);
  inv_stage<2, lay_a, 1>(v, tw_inv, lane);
  inv_stage<1, lay_a, 2>(v, tw_inv, lane);
  inv_stage<0, lay_a, 3>(v, tw_inv, lane);
}

}  // namespace vlp
