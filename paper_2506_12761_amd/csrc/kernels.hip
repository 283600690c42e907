// Device kernels of libvlp: key preparation, batched blind rotation with
// sample extraction, batched key switching, and small helpers.
#include <hip/hip_runtime.h>

#include <cmath>
#include <type_traits>

#include "internal.h"
#include "rns.h"
#include "wave_ntt.h"

namespace vlp {

// ---------------------------------------------------------------------------
// Key preparation
// ---------------------------------------------------------------------------

// One wave per bootstrapping-key polynomial: residues of the coefficient words
// (integers in [0, 2^32)), forward transform, canonical, times the key scale
// 2^32 / 1024 (mod P_k), canonical again.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void bk_transform_kernel(const uint32_t* __restrict__ bk_coeff,
                                                                   uint32_t* __restrict__ bk_ntt,
                                                                   const Tw* __restrict__ tw_fwd,
                                                                   uint32_t n_polys, uint4 scale) {
  __shared__ Tw s_tw[RING_N];
  __shared__ uint2 s_buf[WAVES][RING_N];
  for (int k = threadIdx.x; k < RING_N; k += blockDim.x) s_tw[k] = tw_fwd[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  for (uint32_t poly = blockIdx.x * WAVES + wave; poly < n_polys; poly += gridDim.x * WAVES) {
    const uint32_t* src = bk_coeff + (size_t)poly * RING_N;
    Poly2 v;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t x = src[lay_a(lane, r)];
      v.a[r] = x % P1;
      v.b[r] = x % P2;
    }
    ntt_fwd(v, s_buf[wave], s_tw, tw_fwd, lane);
    uint32_t* dst = bk_ntt + (size_t)poly * 2 * RING_N;  // plane of P1, then plane of P2
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      // Canonical residues of the lazy signed forward output (|v| < 16P), once per key.
      const uint32_t a = (uint32_t)((int32_t)v.a[r] + 16 * (int32_t)P1) % P1;
      const uint32_t b = (uint32_t)((int32_t)v.b[r] + 16 * (int32_t)P2) % P2;
      dst[r * 64 + lane] = csub(shoup(a, scale.x, scale.y, P1), P1);
      dst[RING_N + r * 64 + lane] = csub(shoup(b, scale.z, scale.w, P2), P2);
    }
  }
}

// The key-switching key [1024][8][4][631] in the byte-plane layout of
// KSK_WORDS (internal.h), one output word per thread.
__global__ void ksk_relayout_kernel(const uint32_t* __restrict__ in, uint32_t* __restrict__ out) {
  for (size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x; idx < KSK_WORDS;
       idx += (size_t)gridDim.x * blockDim.x) {
    const uint32_t t = idx & 3, lane = (idx >> 2) & 63, p = (idx >> 8) & 3;
    const size_t rest = idx >> 10;
    const uint32_t tile = (uint32_t)(rest % KS_TILES), i = (uint32_t)(rest / KS_TILES);
    const uint32_t j = 4 * (lane >> 5) + t, w = 32 * tile + (lane & 31);
    uint32_t word = 0x80u;  // v = 0: the zero entry
    for (uint32_t v = 1; v < 4; ++v) {
      const uint32_t k = w < (uint32_t)CT_n ? in[(((size_t)i * KS_T + j) * 4 + v) * CT_n + w] : 0u;
      word |= (((k >> (8 * p)) & 0xFFu) ^ 0x80u) << (8 * v);
    }
    out[idx] = word;
  }
}

// ---------------------------------------------------------------------------
// Blind rotation + sample extraction, one wavefront per item.
// ---------------------------------------------------------------------------
constexpr uint32_t DEC_OFFSET = (1u << 31) + (1u << 24) + (1u << 17) + (1u << 10);
// Balanced digit l of D (with DEC_OFFSET added) is its 7-bit field minus 64,
// i.e. the field with bit 6 flipped read as a signed 7-bit number: flipping
// those bits once per coefficient lets one signed bit-field extract give
// each digit.
constexpr uint32_t DIGIT_FLIP = (1u << 31) | (1u << 24) | (1u << 17);
__device__ __forceinline__ uint32_t digit_of(uint32_t d_flipped, int shift) {
  return (uint32_t)__builtin_amdgcn_sbfe((int)d_flipped, (unsigned)shift, (unsigned)BG_BIT);
}

// Global-address-space views: loads through them are global (not flat)
// loads, so they are not counted by the LDS wait of the transposes.
typedef const uint32_t __attribute__((address_space(1))) g_u32;

// Up to 4 wavefronts per workgroup (one per SIMD) a wavefront may hold 512
// registers: the key rows are prefetched and the accumulators are 64-bit.
// With 8 (two per SIMD, so one hides the other's latencies) it has 256: the
// key is read where it is used and the accumulators are 32-bit.
template <int WAVES>
__global__ __launch_bounds__(64 * WAVES) void br_kernel(const BrItem* __restrict__ items, uint32_t count,
                                                         const Tw* __restrict__ tw_fwd) {
  constexpr bool kPrefetchKey = WAVES <= 4, kWideAcc = WAVES <= 4;
  using Acc = typename std::conditional<kWideAcc, int64_t, uint32_t>::type;
  __shared__ Tw s_tw[RING_N];                   // twiddles of both primes (16 KB)
  __shared__ uint2 s_buf[WAVES][RING_N];        // per-wave transpose scratch
  __shared__ uint32_t s_acc[WAVES][2][RING_N];  // per-wave accumulator (A, B), coefficient order
  __shared__ uint16_t s_abar[WAVES][CT_n + 1];  // modulus-switched input
  for (int k = threadIdx.x; k < RING_N; k += blockDim.x) s_tw[k] = tw_fwd[k];
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint2* buf = s_buf[wave];
  uint32_t* acc = s_acc[wave][0];
  uint16_t* abar = s_abar[wave];

  for (uint32_t it = blockIdx.x * WAVES + wave; it < count; it += gridDim.x * WAVES) {
    const BrItem I = items[it];
    // Gate pre-combination and modulus switch of all 631 words.
    wave_lds_sync();
    const g_u32* in_a = (const g_u32*)I.a;
    const g_u32* in_b = (const g_u32*)I.b;
    for (int w = lane; w < CT_n; w += 64) {
      uint32_t x = (uint32_t)I.ca * in_a[w];
      if (I.b) x += (uint32_t)I.cb * in_b[w];
      for (uint32_t t = 0; t < I.n_more; ++t) x += (uint32_t)I.cm * ((const g_u32*)I.more[t])[w];
      if (w == LWE_n) x += I.cst;
      abar[w] = (uint16_t)((x + (1u << 20)) >> 21);
    }
    wave_lds_sync();
    // acc = (0, X^(-bbar) * mu * (1 + X + ... + X^1023)); coefficient j = 64 r + lane.
    const uint32_t bbar = __builtin_amdgcn_readfirstlane(abar[LWE_n]);
    const uint32_t rot = (2048u - bbar) & 2047u;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t j = r * 64 + lane;
      const bool neg = (j < (rot & 1023u)) != (rot >= 1024u);
      acc[j] = 0;
      acc[RING_N + j] = neg ? (0u - I.mu) : I.mu;
    }
    const uint32_t* bk_i = I.bk;
    for (int i = 0; i < LWE_n; ++i, bk_i += BK_ROW_WORDS) {
      const uint32_t ab = __builtin_amdgcn_readfirstlane((uint32_t)abar[i]);
      if (ab == 0) continue;
      // External product BK_i x (X^ab acc - acc): the six digit polynomials are
      // transformed one at a time and multiplied into the accumulators.
      //  - wide (64-bit) accumulators take the lazy signed transform values
      //    (|x| < 16P): one Montgomery reduction of the six products at the
      //    end gives (-4P, 4P);
      //  - narrow (32-bit) accumulators reduce each product (|x b| < 16P^2)
      //    into (-5P/4, P/4 + 1) and sum the six lazily.
      Acc m0a[16], m0b[16], m1a[16], m1b[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) m0a[r] = m0b[r] = m1a[r] = m1b[r] = 0;
      wave_lds_sync();  // accumulator updates of the previous step are visible
#pragma unroll 1
      for (int c = 0; c < 2; ++c) {
        const uint32_t* poly = acc + c * RING_N;
        // D = X^ab p - p, plus the rounding offset of the decomposition.  All 32
        // reads are issued before the first use (one LDS round trip).
        uint32_t D[16], src[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t j = r * 64 + lane;
          src[r] = poly[((j + 2048u - ab) & 2047u) & 1023u];  // coefficient j of X^ab p is +-p[j - ab]
          D[r] = poly[j];
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const uint32_t s = (r * 64 + lane + 2048u - ab) & 2047u;
          D[r] = ((s >= 1024u ? 0u - src[r] : src[r]) - D[r] + DEC_OFFSET) ^ DIGIT_FLIP;
        }
#pragma unroll 1
        for (int lev = 0; lev < ELL; ++lev) {
          // Residues mod P1 and mod P2 of the two key rows of this digit (planes
          // of 1,024 words: row 0 P1, row 0 P2, row 1 P1, row 1 P2); with
          // registers to spare they are requested before the transform, which
          // hides their latency.
          const g_u32* k0 = (const g_u32*)(bk_i + (size_t)((c * ELL + lev) * 4) * RING_N);
          uint32_t b0a[16], b0b[16], b1a[16], b1b[16];
          if constexpr (kPrefetchKey) {
#pragma unroll
            for (int r = 0; r < 16; ++r) {
              b0a[r] = k0[r * 64 + lane];
              b0b[r] = k0[RING_N + r * 64 + lane];
              b1a[r] = k0[2 * RING_N + r * 64 + lane];
              b1b[r] = k0[3 * RING_N + r * 64 + lane];
            }
          }
          const int shift = 32 - BG_BIT * (lev + 1);
          Poly2 v;
#pragma unroll
          for (int r = 0; r < 16; ++r) v.a[r] = v.b[r] = digit_of(D[r], shift);  // signed, |d| <= 64
          ntt_fwd(v, buf, s_tw, tw_fwd, lane);
#pragma unroll
          for (int r = 0; r < 16; ++r) {
            if constexpr (!kPrefetchKey) {
              b0a[r] = k0[r * 64 + lane];
              b0b[r] = k0[RING_N + r * 64 + lane];
              b1a[r] = k0[2 * RING_N + r * 64 + lane];
              b1b[r] = k0[3 * RING_N + r * 64 + lane];
            }
            const int64_t da = (int32_t)v.a[r], db = (int32_t)v.b[r];  // |x| < 16P
            if constexpr (kWideAcc) {
              m0a[r] += da * (int32_t)b0a[r];
              m0b[r] += db * (int32_t)b0b[r];
              m1a[r] += da * (int32_t)b1a[r];
              m1b[r] += db * (int32_t)b1b[r];
            } else {
              m0a[r] += redc_s(da * (int32_t)b0a[r], P1, P1_INV);
              m0b[r] += redc_s(db * (int32_t)b0b[r], P2, P2_INV);
              m1a[r] += redc_s(da * (int32_t)b1a[r], P1, P1_INV);
              m1b[r] += redc_s(db * (int32_t)b1b[r], P2, P2_INV);
            }
          }
        }
      }
#pragma unroll 1
      for (int c = 0; c < 2; ++c) {
        Poly2 v;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if constexpr (kWideAcc) {  // (-4P, 4P), the inverse transform's input range
            v.a[r] = redc_s(c ? m1a[r] : m0a[r], P1, P1_INV);
            v.b[r] = redc_s(c ? m1b[r] : m0b[r], P2, P2_INV);
          } else {  // |sum| < 7.5P -> (-P/2, 3P/2)
            v.a[r] = reduce_s(c ? m1a[r] : m0a[r], P1);
            v.b[r] = reduce_s(c ? m1b[r] : m0b[r], P2);
          }
        }
        ntt_inv(v, buf, s_tw, tw_fwd, lane);
        uint32_t* poly = acc + c * RING_N;
        uint32_t old[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) old[r] = poly[r * 64 + lane];
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int r = 0; r < 16; ++r) poly[r * 64 + lane] = old[r] + crt_lift_s(v.a[r], v.b[r]);
      }
    }
    wave_lds_sync();
    // SampleExtract: a'_0 = A_0, a'_j = -A_(N-j), b' = B_0.
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int j = r * 64 + lane;
      const uint32_t a = acc[j];
      if (j == 0) I.out[0] = a;
      else I.out[RING_N - j] = 0u - a;
    }
    if (lane == 0) I.out[RING_N] = acc[RING_N];
  }
}

// ---------------------------------------------------------------------------
// Blind rotation split by prime: a workgroup of two wavefronts per item, wave
// PR computing every product modulo prime PR.  Each wavefront needs about half
// the registers of the one-wavefront form, so two fit on a SIMD and hide each
// other's memory and LDS latency.  Per CMux the two meet twice: after the
// inverse transforms (each hands the other the residues of the output
// polynomial that the other lifts) and after the accumulator update.
// ---------------------------------------------------------------------------
// SKIP: steps with abar_i = 0 (X^0 acc - acc = 0, an exact no-op) are skipped;
// workgroups holding several rotations run them all, so that every wavefront
// of the workgroup meets the same barriers.
template <int PR, bool SKIP>
__device__ __forceinline__ void br2_rotate(const BrItem& I, uint32_t* acc, const uint16_t* abar, uint32_t* buf,
                                           uint32_t* buf2, const uint32_t* other_buf, const uint2* tws, int lane) {
  constexpr uint32_t P = Prime<PR>::P, PINV = Prime<PR>::PINV;
  const uint32_t* bk_i = I.bk;
  for (int i = 0; i < LWE_n; ++i, bk_i += BK_ROW_WORDS) {
    const uint32_t ab = __builtin_amdgcn_readfirstlane((uint32_t)abar[i]);
    if (SKIP && ab == 0) continue;  // the same decision in both wavefronts: abar is shared
    // Signed 64-bit accumulators of the two output polynomials mod P: six
    // products of transform values (|x| < 16P) and key residues (< P); one
    // reduction at the end gives (-4P, 4P), the inverse transform's input range.
    int64_t m0[16], m1[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) m0[r] = m1[r] = 0;
#pragma unroll 1
    for (int c = 0; c < 2; ++c) {
      // Polynomial c and its negation side by side (2048 words): coefficient
      // j of X^ab p is word (j - ab) mod 2048 of that window.
      const uint32_t* poly = acc + c * 2 * RING_N;
      uint32_t D[16], src[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t j = r * 64 + lane;
        src[r] = poly[(j + 2048u - ab) & 2047u];
        D[r] = poly[j];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 16; ++r) D[r] = (src[r] - D[r] + DEC_OFFSET) ^ DIGIT_FLIP;
      // Unrolled: a quarter fewer scalar instructions per polynomial (the
      // loop's control and key addressing) and scheduling across the digits;
      // 1.1% less time per launch than a loop.
#pragma unroll
      for (int lev = 0; lev < ELL; ++lev) {
        // This prime's planes of the two key rows of the digit, requested
        // before the transform so that it hides their latency.
        const g_u32* k0 = (const g_u32*)(bk_i + (size_t)((c * ELL + lev) * 4 + PR) * RING_N);
        uint32_t b0[16], b1[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          b0[r] = k0[r * 64 + lane];
          b1[r] = k0[2 * RING_N + r * 64 + lane];
        }
        const int shift = 32 - BG_BIT * (lev + 1);
        uint32_t x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = digit_of(D[r], shift);  // balanced digit, signed
        ntt_fwd1<PR>(x, buf, tws, lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          m0[r] += (int64_t)(int32_t)x[r] * (int32_t)b0[r];
          m1[r] += (int64_t)(int32_t)x[r] * (int32_t)b1[r];
        }
      }
    }
    // Wave 0 lifts output 0 (A), wave 1 output 1 (B).  The kept output is
    // transformed first and stays in registers; the other one is transformed
    // next and parked in this wavefront's LDS buffer for the partner.
    constexpr int KEEP = PR;
    uint32_t keep[16], x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      keep[r] = redc_s(KEEP ? m1[r] : m0[r], P, PINV);
      x[r] = redc_s(KEEP ? m0[r] : m1[r], P, PINV);
    }
    ntt_inv1_pair<PR>(keep, x, buf, buf2, tws, lane);  // both end below 16P: the lift takes lazy residues
    wave_lds_sync();  // the transform's last reads of buf are done
#pragma unroll
    for (int r = 0; r < 16; ++r) buf[r * 64 + lane] = x[r];
    __syncthreads();  // both wavefronts have parked their residues
    uint32_t* poly = acc + KEEP * 2 * RING_N;
    uint32_t old[16], oth[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      old[r] = poly[r * 64 + lane];
      oth[r] = other_buf[r * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t v = old[r] + (PR == 0 ? crt_lift_s(keep[r], oth[r]) : crt_lift_s(oth[r], keep[r]));
      poly[r * 64 + lane] = v;
      poly[RING_N + r * 64 + lane] = 0u - v;
    }
    __syncthreads();  // accumulator updated; parked residues consumed
  }
}

// ROT rotations per workgroup (2 * ROT wavefronts): with ROT > 1 the
// rotations of a workgroup advance in lockstep (their wavefronts share every
// barrier), so they read each key row at the same time; a partial last
// workgroup repeats the last item in its idle rotations and writes nothing.
template <int ROT>
__global__ __launch_bounds__(128 * ROT) __attribute__((amdgpu_waves_per_eu(2))) void br2_kernel(
    const BrItem* __restrict__ items, uint32_t count, const Tw* __restrict__ tw_fwd) {
  __shared__ uint2 s_tw[2][RING_N];              // per prime: {w, Shoup(w)}, stage slices permuted (16 KB)
  __shared__ __align__(16) uint32_t s_buf[2 * ROT][RING_N];  // per wavefront: transpose scratch, then parked residues
  __shared__ __align__(16) uint32_t s_buf2[2 * ROT][RING_N]; // per wavefront: second transpose scratch
  __shared__ uint32_t s_acc[ROT][2][2 * RING_N];  // per rotation: accumulator A, -A, B, -B, coefficient order
  __shared__ uint16_t s_abar[ROT][CT_n + 1];     // per rotation: modulus-switched input
  for (int e = 16 + threadIdx.x; e < RING_N; e += blockDim.x) {  // stages 4..9 (entries 16..1023)
    const int S = 31 - __builtin_clz(e);
    const int slot = (1 << S) + tw_perm(S, e - (1 << S));
    const Tw w = tw_fwd[e];
    s_tw[0][slot] = make_uint2(w.x, w.y);
    s_tw[1][slot] = make_uint2(w.z, w.w);
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int rot_i = wave >> 1, pr = wave & 1, t = threadIdx.x & 127;  // t: thread within the rotation's pair
  // Wavefront w runs on SIMD w mod 4, so each SIMD holds rotation r and
  // rotation r + 2 of the same prime, which reach their LDS waits together.
  // Raising the first one's issue priority lets it run ahead until it waits
  // while the other fills the gaps (12.21 -> 12.12 ms per launch).
  if (ROT == 4 && rot_i < 2) __builtin_amdgcn_s_setprio(1);
  uint32_t* acc = s_acc[rot_i][0];
  uint16_t* abar = s_abar[rot_i];
  for (uint32_t g = blockIdx.x; g * ROT < count; g += gridDim.x) {
    const uint32_t idx = g * ROT + rot_i;
    const bool active = idx < count;
    const BrItem I = items[active ? idx : count - 1];
    __syncthreads();  // the previous item's readers of acc and abar are done
    const g_u32* in_a = (const g_u32*)I.a;
    const g_u32* in_b = (const g_u32*)I.b;
    for (int w = t; w < CT_n; w += 128) {
      uint32_t x = (uint32_t)I.ca * in_a[w];
      if (I.b) x += (uint32_t)I.cb * in_b[w];
      for (uint32_t k = 0; k < I.n_more; ++k) x += (uint32_t)I.cm * ((const g_u32*)I.more[k])[w];
      if (w == LWE_n) x += I.cst;
      abar[w] = (uint16_t)((x + (1u << 20)) >> 21);
    }
    __syncthreads();
    // acc = (0, X^(-bbar) * mu * (1 + X + ... + X^1023)): wave 0 of the pair writes A, wave 1 B.
    const uint32_t bbar = __builtin_amdgcn_readfirstlane(abar[LWE_n]);
    const uint32_t rot = (2048u - bbar) & 2047u;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t j = r * 64 + lane;
      const bool neg = (j < (rot & 1023u)) != (rot >= 1024u);
      const uint32_t v = pr == 0 ? 0u : (neg ? (0u - I.mu) : I.mu);
      acc[pr * 2 * RING_N + j] = v;
      acc[pr * 2 * RING_N + RING_N + j] = 0u - v;
    }
    __syncthreads();
    if (pr == 0)
      br2_rotate<0, ROT == 1>(I, acc, abar, s_buf[2 * rot_i], s_buf2[2 * rot_i], s_buf[2 * rot_i + 1], s_tw[0], lane);
    else
      br2_rotate<1, ROT == 1>(I, acc, abar, s_buf[2 * rot_i + 1], s_buf2[2 * rot_i + 1], s_buf[2 * rot_i], s_tw[1], lane);
    // SampleExtract: a'_0 = A_0, a'_j = -A_(N-j), b' = B_0 (the last update is
    // visible after the rotation's closing barrier, or the one above if no step ran).
    if (active) {
      for (int j = t; j < RING_N; j += 128) I.out[j] = j == 0 ? acc[0] : acc[2 * RING_N - j];  // -A_(N-j)
      if (t == 0) I.out[RING_N] = acc[2 * RING_N];
    }
  }
}

// ---------------------------------------------------------------------------
// Blind rotation split by prime and by accumulator half: a workgroup of four
// wavefronts per item; wave w = PR + 2H computes, modulo prime PR, the three
// digit polynomials of accumulator polynomial H and its products with the key
// rows for both outputs.  Per CMux each wavefront runs 3 forward and 1 inverse
// transform (half the split form's), so one rotation takes about half as
// long; three workgroup barriers per CMux:
//   B1  partial sums: wave (PR, H) receives from (PR, 1-H) the partial of
//       output H over the other three digits, adds it to its own and runs the
//       inverse transform of output H modulo PR;
//   B2  CRT: waves (0, H) and (1, H) swap half of their residues, each lifts
//       8 of the 16 registers of output H and updates the accumulator;
//   B3  the accumulator is complete for the next CMux.
// ---------------------------------------------------------------------------
template <int PR, int H>
__device__ __forceinline__ void br4_rotate(const BrItem& I, uint32_t* acc, const uint16_t* abar, uint32_t* buf,
                                           const uint32_t* prime_partner_buf, uint32_t* xbuf,
                                           const uint32_t* half_partner_xbuf, const uint2* tws,
                                           int lane) {
  constexpr uint32_t P = Prime<PR>::P, PINV = Prime<PR>::PINV;
  const uint32_t* bk_i = I.bk;
  for (int i = 0; i < LWE_n; ++i, bk_i += BK_ROW_WORDS) {
    const uint32_t ab = __builtin_amdgcn_readfirstlane((uint32_t)abar[i]);
    if (ab == 0) continue;  // the same decision in all four wavefronts: abar is shared
    // Three products of transform values (|x| < 16P) and key residues (< P)
    // per output: one reduction gives (-2P, 2P).
    int64_t m0[16], m1[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) m0[r] = m1[r] = 0;
    {
      const uint32_t* poly = acc + H * RING_N;
      uint32_t D[16], src[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t j = r * 64 + lane;
        src[r] = poly[((j + 2048u - ab) & 2047u) & 1023u];  // coefficient j of X^ab p is +-p[j - ab]
        D[r] = poly[j];
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const uint32_t s = (r * 64 + lane + 2048u - ab) & 2047u;
        D[r] = ((s >= 1024u ? 0u - src[r] : src[r]) - D[r] + DEC_OFFSET) ^ DIGIT_FLIP;
      }
      // Unrolled as in br2_rotate (5.5% less time per launch than a loop).
#pragma unroll
      for (int lev = 0; lev < ELL; ++lev) {
        const g_u32* k0 = (const g_u32*)(bk_i + (size_t)((H * ELL + lev) * 4 + PR) * RING_N);
        uint32_t b0[16], b1[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          b0[r] = k0[r * 64 + lane];
          b1[r] = k0[2 * RING_N + r * 64 + lane];
        }
        const int shift = 32 - BG_BIT * (lev + 1);
        uint32_t x[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) x[r] = digit_of(D[r], shift);  // balanced digit, signed
        ntt_fwd1<PR>(x, buf, tws, lane);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          m0[r] += (int64_t)(int32_t)x[r] * (int32_t)b0[r];
          m1[r] += (int64_t)(int32_t)x[r] * (int32_t)b1[r];
        }
      }
    }
    // Hand the partial of output 1-H to the other half; keep output H's.
    uint32_t x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      xbuf[r * 64 + lane] = redc_s(H ? m0[r] : m1[r], P, PINV);  // (-2P, 2P)
      x[r] = redc_s(H ? m1[r] : m0[r], P, PINV);
    }
    // The first two inverse stages' twiddles, read before the partner's
    // products so that they are not queued behind those reads.
    InvTw98 itw;
    inv_tw98_load(itw, tws, lane);
    __syncthreads();  // B1
    uint32_t oth[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) oth[r] = half_partner_xbuf[r * 64 + lane];
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] += oth[r];  // (-4P, 4P)
    ntt_inv1<PR>(x, itw, buf, tws, lane);
    // Wave (0, H) lifts registers 0..7, wave (1, H) registers 8..15: each parks
    // the half the other one lifts.
    wave_lds_sync();  // the transform's last reads of buf are done
    constexpr int MINE = PR * 8, THEIRS = 8 - PR * 8;
#pragma unroll
    for (int r = 0; r < 8; ++r) buf[(THEIRS + r) * 64 + lane] = x[THEIRS + r];  // lazy: the lift takes |x| < 16P
    __syncthreads();  // B2
    uint32_t* poly = acc + H * RING_N;
    uint32_t old[8], o2[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      old[r] = poly[(MINE + r) * 64 + lane];
      o2[r] = prime_partner_buf[(MINE + r) * 64 + lane];
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t mine = x[MINE + r];
      poly[(MINE + r) * 64 + lane] = old[r] + (PR == 0 ? crt_lift_s(mine, o2[r]) : crt_lift_s(o2[r], mine));
    }
    __syncthreads();  // B3
  }
}

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void br4_kernel(
    const BrItem* __restrict__ items, uint32_t count, const Tw* __restrict__ tw_fwd) {
  __shared__ uint2 s_tw[2][RING_N];      // per prime: {w, Shoup(w)}, stage slices permuted (16 KB)
  __shared__ __align__(16) uint32_t s_buf[4][RING_N];  // per wavefront: transpose scratch, then CRT hand-over
  __shared__ uint32_t s_x[4][RING_N];    // per wavefront: partial sum handed to the other half
  __shared__ uint32_t s_acc[2][RING_N];  // accumulator (A, B), coefficient order
  __shared__ uint16_t s_abar[CT_n + 1];  // modulus-switched input
  for (int e = 16 + threadIdx.x; e < RING_N; e += blockDim.x) {  // stages 4..9 (entries 16..1023)
    const int S = 31 - __builtin_clz(e);
    const int slot = (1 << S) + tw_perm(S, e - (1 << S));
    const Tw w = tw_fwd[e];
    s_tw[0][slot] = make_uint2(w.x, w.y);
    s_tw[1][slot] = make_uint2(w.z, w.w);
  }
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint32_t* acc = s_acc[0];
  for (uint32_t it = blockIdx.x; it < count; it += gridDim.x) {
    const BrItem I = items[it];
    __syncthreads();  // the previous item's readers of acc and abar are done
    const g_u32* in_a = (const g_u32*)I.a;
    const g_u32* in_b = (const g_u32*)I.b;
    for (int w = threadIdx.x; w < CT_n; w += 256) {
      uint32_t x = (uint32_t)I.ca * in_a[w];
      if (I.b) x += (uint32_t)I.cb * in_b[w];
      for (uint32_t t = 0; t < I.n_more; ++t) x += (uint32_t)I.cm * ((const g_u32*)I.more[t])[w];
      if (w == LWE_n) x += I.cst;
      s_abar[w] = (uint16_t)((x + (1u << 20)) >> 21);
    }
    __syncthreads();
    // acc = (0, X^(-bbar) * mu * (1 + X + ... + X^1023)): waves 0, 1 write A (halves), 2, 3 write B.
    const uint32_t bbar = __builtin_amdgcn_readfirstlane(s_abar[LWE_n]);
    const uint32_t rot = (2048u - bbar) & 2047u;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const uint32_t j = ((wave & 1) * 8 + r) * 64 + lane;
      const bool neg = (j < (rot & 1023u)) != (rot >= 1024u);
      acc[(wave >> 1) * RING_N + j] = (wave >> 1) == 0 ? 0u : (neg ? (0u - I.mu) : I.mu);
    }
    __syncthreads();
    switch (wave) {
      case 0: br4_rotate<0, 0>(I, acc, s_abar, s_buf[0], s_buf[1], s_x[0], s_x[2], s_tw[0], lane); break;
      case 1: br4_rotate<1, 0>(I, acc, s_abar, s_buf[1], s_buf[0], s_x[1], s_x[3], s_tw[1], lane); break;
      case 2: br4_rotate<0, 1>(I, acc, s_abar, s_buf[2], s_buf[3], s_x[2], s_x[0], s_tw[0], lane); break;
      default: br4_rotate<1, 1>(I, acc, s_abar, s_buf[3], s_buf[2], s_x[3], s_x[1], s_tw[1], lane); break;
    }
    for (int j = threadIdx.x; j < RING_N; j += 256) {
      const uint32_t a = acc[j];
      if (j == 0) I.out[0] = a;
      else I.out[RING_N - j] = 0u - a;
    }
    if (threadIdx.x == 0) I.out[RING_N] = acc[RING_N];
  }
}

// ---------------------------------------------------------------------------
// Key switching on the 8-bit matrix cores.
//
// The key switch of gate g subtracts, for every coefficient i < 1024 and
// level j < 8, the key entry selected by the digit d_ij of a'_i + 2^15.  With
// A[g][(i, j, v)] = [d_ij = v] (exactly one 1 per (i, j), the entry v = 0
// being zero) that sum is the product A x K of the one-hot matrix and the key
// K[(i, j, v)][w]; split K into byte planes K_p (so K = sum_p 2^(8p) K_p) and
// each plane's product is an exact integer (at most 8,192 terms below 2^8),
// computed by v_mfma_i32_32x32x32_i8 on signed bytes K_p - 128 (stored XOR
// 0x80); every (i, j) contributes exactly one -128, so the word is
// sum_p 2^(8p) C_p + 128 x (pairs) x 0x01010101 (mod 2^32).
//
// K-block of one MFMA = one coefficient i: lane n + 32 h supplies, in its 16
// operand bytes t*4 + v, the levels j = 4 h + t and the digit values v (the
// key lane of the same index supplies the same (j, v)); the gate rows of the
// A operand are the lanes' n, the output words of the B operand the lanes' n.
// A workgroup of 4 wavefronts covers 4 x RT x 32 gates and one tile of 32
// output words (4 planes = 4 accumulators per 32 gates); blockIdx.z takes a
// range of coefficients, whose partial results are added atomically into
// outputs zeroed first when there is more than one range.
// ---------------------------------------------------------------------------
typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// Digit bytes of count gates (input a' = u1 + u2):
// dig[(q * count + g) * 2 + h], byte c = bits [24 - 8h, 32 - 8h) of
// a'_(4q+c) + 2^15, i.e. the digits of levels 4h .. 4h + 3 of coefficient
// 4q + c, most significant first.  With zero_out the outputs are cleared
// (split key switching adds into them).  One thread per (q, g), g fastest.
__global__ void ks_prep_kernel(const KsItem* __restrict__ items, uint32_t count, uint2* __restrict__ dig,
                               int zero_out) {
  const size_t total = (size_t)count * (RING_N / 4);
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (size_t)gridDim.x * blockDim.x) {
    const uint32_t g = (uint32_t)(t % count), q = (uint32_t)(t / count);
    const KsItem& it = items[g];
    const g_u32* u1 = (const g_u32*)it.u1 + 4 * q;
    const g_u32* u2 = it.u2 ? (const g_u32*)it.u2 + 4 * q : nullptr;
    uint32_t hi = 0, lo = 0;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const uint32_t a = u1[c] + (u2 ? u2[c] : 0u) + 0x8000u;
      hi |= (a >> 24) << (8 * c);
      lo |= ((a >> 16) & 0xFFu) << (8 * c);
    }
    dig[t] = make_uint2(hi, lo);
    if (zero_out && 4 * q < (uint32_t)CT_n)
#pragma unroll
      for (int c = 0; c < 4; ++c)
        if (4 * q + c < (uint32_t)CT_n) it.out[4 * q + c] = 0u;
  }
}

template <int RT>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4 / RT))) void ks_mfma_kernel(
    const KsItem* __restrict__ items, uint32_t count,
                                                      const uint32_t* __restrict__ dig,
                                                      const uint4* __restrict__ ksk, uint32_t i_per_block) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint32_t tile = blockIdx.x;
  const uint32_t row0 = (blockIdx.y * 4 + wave) * (RT * 32);
  const uint32_t i0 = blockIdx.z * i_per_block, i_end = i0 + i_per_block;
  const int n = lane & 31, h = lane >> 5;
  // Digit words of this lane's gate rows (rows past the last gate read the
  // last gate's digits; their results are not stored).
  const g_u32* dp[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) dp[rt] = (const g_u32*)dig + (size_t)min(row0 + rt * 32 + n, count - 1) * 2 + h;
  const size_t dstep = (size_t)count * 2;  // words between coefficient groups
  v16i acc[RT][4];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[rt][p] = v16i{};
  // Key fragments of coefficient i: kb + i * KS_TILES * 256 (4 planes x 64 lanes).
  const g_u32* kb = (const g_u32*)(ksk + (size_t)tile * 256 + lane);
  auto load_b = [&](uint32_t i, v4i* b) {
    const uint4* k = (const uint4*)(kb) + (size_t)i * KS_TILES * 256;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const uint4 v = k[p * 64];
      b[p] = v4i{(int)v.x, (int)v.y, (int)v.z, (int)v.w};
    }
  };
  uint32_t dcur[RT], dnext[RT];
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) dcur[rt] = dp[rt][(size_t)(i0 / 4) * dstep];
  v4i b0[4], b1[4];
  load_b(i0, b0);
  load_b(i0 + 1, b1);
  for (uint32_t q = i0 / 4; q < i_end / 4; ++q) {
    const uint32_t qn = min(q + 1, i_end / 4 - 1);
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) dnext[rt] = dp[rt][(size_t)qn * dstep];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      v4i b[4];
#pragma unroll
      for (int p = 0; p < 4; ++p) {
        b[p] = b0[p];
        b0[p] = b1[p];
      }
      load_b(min(4 * q + c + 2, i_end - 1), b1);
#pragma unroll
      for (int rt = 0; rt < RT; ++rt) {
        const uint32_t x = dcur[rt] >> (8 * c);
        v4i a;
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = (int)(1u << (((x >> (6 - 2 * t)) & 3u) << 3));
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[rt][p] = __builtin_amdgcn_mfma_i32_32x32x32_i8(a, b[p], acc[rt][p], 0, 0, 0);
      }
    }
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) dcur[rt] = dnext[rt];
  }
  const uint32_t corr = 128u * 8u * i_per_block * 0x01010101u;
  const uint32_t w = tile * 32 + n;
  if (w >= (uint32_t)CT_n) return;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const uint32_t g = row0 + rt * 32 + 8 * (r >> 2) + 4 * h + (r & 3);
      if (g >= count) continue;
      const uint32_t sum = (uint32_t)acc[rt][0][r] + ((uint32_t)acc[rt][1][r] << 8) +
                           ((uint32_t)acc[rt][2][r] << 16) + ((uint32_t)acc[rt][3][r] << 24) + corr;
      const KsItem& it = items[g];
      uint32_t val = 0u - sum;
      if (w == (uint32_t)LWE_n && blockIdx.z == 0) val += it.u1[RING_N] + (it.u2 ? it.u2[RING_N] : 0u) + it.cst;
      if (gridDim.z == 1)
        it.out[w] = val;
      else
        atomicAdd(it.out + w, val);
    }
}

// ---------------------------------------------------------------------------
// Helpers
// ---------------------------------------------------------------------------
__global__ void make_br_items_kernel(BrItem* items, uint32_t count, const uint32_t* a, const uint32_t* b, int32_t ca,
                                     int32_t cb, uint32_t cst, uint32_t mu, uint32_t* out, const uint32_t* bk) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  BrItem it;
  it.a = a + (size_t)t * CT_n;
  it.b = b ? b + (size_t)t * CT_n : nullptr;
  it.out = out + (size_t)t * CT_N;
  it.bk = bk;
  it.ca = ca;
  it.cb = cb;
  it.cst = cst;
  it.mu = mu;
  it.more = nullptr;
  it.n_more = 0;
  it.cm = 0;
  items[t] = it;
}

__global__ void make_ks_items_kernel(KsItem* items, uint32_t count, const uint32_t* u1, const uint32_t* u2,
                                     uint32_t cst, uint32_t* out, const uint32_t* ksk) {
  const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count) return;
  KsItem it;
  it.u1 = u1 + (size_t)t * CT_N;
  it.u2 = u2 ? u2 + (size_t)t * CT_N : nullptr;
  it.out = out + (size_t)t * CT_n;
  it.ksk = ksk;
  it.cst = cst;
  it.pad = 0;
  items[t] = it;
}

__global__ void negate_kernel(const uint32_t* a, uint32_t* out, size_t words) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
    out[i] = 0u - a[i];
}

// ServerEnc (Alg. 2): ciphertext t of a flat [count][631] array becomes
// pk[t] + (0, Ecd(bit_t)).  bit_t is bit (t mod l) of the int64 value t / l
// (LSB first, two's complement) when `vals` is given, else bytes[t] != 0.
__device__ __forceinline__ uint32_t enc_word(const int64_t* vals, const uint8_t* bytes, uint32_t l, size_t t) {
  const uint32_t bit = vals ? (uint32_t)(((uint64_t)vals[t / l] >> (t % l)) & 1u) : (uint32_t)(bytes[t] != 0);
  return bit ? MU : 0u - MU;
}

// Out of place, 16-byte accesses (pk and out 16-byte aligned): each thread
// issues U loads of four consecutive words (a block's U loads cover U
// consecutive runs of blockDim quads) before it adds the body words and
// stores, so U x 16 bytes per lane are in flight; the last words % 4 words
// are done by the first threads.  IDX is the index type: 32-bit when the
// array has fewer than 2^32 words (cheaper division by 631), else 64-bit.
// Loads and stores are non-temporal: every word is touched once.
__device__ __forceinline__ void add_body(uint4& w, uint32_t r, uint32_t e) {
  switch (CT_n - 1 - r) {
    case 0: w.x += e; break;
    case 1: w.y += e; break;
    case 2: w.z += e; break;
    default: w.w += e; break;
  }
}

template <typename IDX, int U>
__global__ void server_enc_copy_kernel(const uint4* __restrict__ pk, uint4* __restrict__ out, size_t count,
                                       const int64_t* __restrict__ vals, const uint8_t* __restrict__ bytes,
                                       uint32_t l) {
  const IDX words = (IDX)(count * CT_n), quads = words / 4;
  const IDX stride = (IDX)gridDim.x * blockDim.x * U;
  for (IDX q0 = (IDX)blockIdx.x * blockDim.x * U + threadIdx.x; q0 < quads; q0 += stride) {
    uint4 w[U];
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const IDX q = q0 + (IDX)k * blockDim.x;
      if (q < quads) {
        w[k].x = __builtin_nontemporal_load(&pk[q].x);
        w[k].y = __builtin_nontemporal_load(&pk[q].y);
        w[k].z = __builtin_nontemporal_load(&pk[q].z);
        w[k].w = __builtin_nontemporal_load(&pk[q].w);
      }
    }
#pragma unroll
    for (int k = 0; k < U; ++k) {
      const IDX q = q0 + (IDX)k * blockDim.x;
      if (q < quads) {
        const IDX w0 = 4 * q;
        const IDX t = w0 / CT_n;
        const uint32_t r = (uint32_t)(w0 - t * CT_n);  // word index of w.x inside ciphertext t
        if (r >= CT_n - 4) add_body(w[k], r, enc_word(vals, bytes, l, t));  // the body word is one of the four
        __builtin_nontemporal_store(w[k].x, &out[q].x);
        __builtin_nontemporal_store(w[k].y, &out[q].y);
        __builtin_nontemporal_store(w[k].z, &out[q].z);
        __builtin_nontemporal_store(w[k].w, &out[q].w);
      }
    }
  }
  const IDX tid = (IDX)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid < words - 4 * quads) {
    const IDX wi = 4 * quads + tid;
    const IDX t = wi / CT_n;
    uint32_t v = reinterpret_cast<const uint32_t*>(pk)[wi];
    if (wi - t * CT_n == CT_n - 1) v += enc_word(vals, bytes, l, t);
    reinterpret_cast<uint32_t*>(out)[wi] = v;
  }
}

// Word-granular form of the copy for buffers that are not 16-byte aligned.
__global__ void server_enc_word_kernel(const uint32_t* __restrict__ pk, uint32_t* __restrict__ out, size_t count,
                                       const int64_t* __restrict__ vals, const uint8_t* __restrict__ bytes,
                                       uint32_t l) {
  const size_t words = count * CT_n;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x) {
    const size_t t = i / CT_n;
    uint32_t v = pk[i];
    if (i - t * CT_n == CT_n - 1) v += enc_word(vals, bytes, l, t);
    out[i] = v;
  }
}

// In place (out == pk): only the body words change.
__global__ void server_enc_inplace_kernel(uint32_t* ct, size_t count, const int64_t* __restrict__ vals,
                                          const uint8_t* __restrict__ bytes, uint32_t l) {
  for (size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x; t < count; t += (size_t)gridDim.x * blockDim.x)
    ct[t * CT_n + CT_n - 1] += enc_word(vals, bytes, l, t);
}

// ---------------------------------------------------------------------------
// Fixed scratch of the allocation-free gate call.  Each device holds its own
// copy for the life of the process.  On the host, `scratch` names a host-side
// stand-in, not device memory: host code uses only the address that
// noalloc_scratch_address() returns for the current device.
// ---------------------------------------------------------------------------
static __device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

int noalloc_scratch_address(void** p) {
  *p = nullptr;
  return (int)hipGetSymbolAddress(p, HIP_SYMBOL(scratch));
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
static inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

int launch_bk_transform(const uint32_t* bk_coeff, uint32_t* bk_ntt, const uint4* tw_fwd, void* stream) {
  const uint32_t n_polys = LWE_n * 2 * ELL * 2;
  uint32_t sc[4];
  key_scale(sc);
  const uint4 scale = make_uint4(sc[0], sc[1], sc[2], sc[3]);
  hipLaunchKernelGGL(bk_transform_kernel<4>, dim3((n_polys + 3) / 4), dim3(256), 0, S(stream), bk_coeff, bk_ntt, tw_fwd,
                     n_polys, scale);
  return (int)hipGetLastError();
}

int launch_ksk_relayout(const uint32_t* ksk_in, uint32_t* ksk_out, void* stream) {
  hipLaunchKernelGGL(ksk_relayout_kernel, dim3(4096), dim3(256), 0, S(stream), ksk_in, ksk_out);
  return (int)hipGetLastError();
}

int launch_br(const BrItem* items, uint32_t count, const uint4* tw_fwd, uint32_t waves_per_block, uint32_t blocks,
              void* stream) {
  if (count == 0) return 0;
  const uint32_t need = (count + waves_per_block - 1) / waves_per_block;
  if (blocks == 0 || blocks > need) blocks = need;
  switch (waves_per_block) {
    case 1: hipLaunchKernelGGL(br_kernel<1>, dim3(blocks), dim3(64), 0, S(stream), items, count, tw_fwd); break;
    case 2: hipLaunchKernelGGL(br_kernel<2>, dim3(blocks), dim3(128), 0, S(stream), items, count, tw_fwd); break;
    case 4: hipLaunchKernelGGL(br_kernel<4>, dim3(blocks), dim3(256), 0, S(stream), items, count, tw_fwd); break;
    case 8: hipLaunchKernelGGL(br_kernel<8>, dim3(blocks), dim3(512), 0, S(stream), items, count, tw_fwd); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_br2(const BrItem* items, uint32_t count, const uint4* tw_fwd, uint32_t rot_per_block, uint32_t blocks,
               void* stream) {
  if (count == 0) return 0;
  const uint32_t need = (count + rot_per_block - 1) / rot_per_block;
  if (blocks == 0 || blocks > need) blocks = need;
  switch (rot_per_block) {
    case 1: hipLaunchKernelGGL(br2_kernel<1>, dim3(blocks), dim3(128), 0, S(stream), items, count, tw_fwd); break;
    case 2: hipLaunchKernelGGL(br2_kernel<2>, dim3(blocks), dim3(256), 0, S(stream), items, count, tw_fwd); break;
    case 4: hipLaunchKernelGGL(br2_kernel<4>, dim3(blocks), dim3(512), 0, S(stream), items, count, tw_fwd); break;
    default: return (int)hipErrorInvalidValue;
  }
  return (int)hipGetLastError();
}

int launch_br4(const BrItem* items, uint32_t count, const uint4* tw_fwd, uint32_t blocks, void* stream) {
  if (count == 0) return 0;
  if (blocks == 0 || blocks > count) blocks = count;
  hipLaunchKernelGGL(br4_kernel, dim3(blocks), dim3(256), 0, S(stream), items, count, tw_fwd);
  return (int)hipGetLastError();
}

int launch_ks_group(const KsItem* items, uint32_t count, const uint32_t* ksk, uint32_t* dig,
                    uint32_t gates_per_block, uint32_t cus, void* stream) {
  if (!(gates_per_block == 128 || gates_per_block == 256 || gates_per_block == 512)) return (int)hipErrorInvalidValue;
  for (uint32_t first = 0; first < count; first += KS_CHUNK) {
    const uint32_t cnt = std::min(KS_CHUNK, count - first);
    // Gates per workgroup (gpb, at most gates_per_block; registers let a CU
    // hold 512 / gpb such workgroups) and coefficient ranges per gate tile
    // (sp): the pair that minimises the rounds of workgroups the device runs
    // times the cycles of a round on one SIMD -- 512 matrix-core cycles per
    // coefficient whatever the tile, plus the workgroups' epilogues (stores,
    // or atomic adds when the ranges are split); larger tiles on ties (fewer
    // key reads).
    uint32_t gpb = gates_per_block, best = 1, rows = 1;
    double best_cost = -1;
    for (uint32_t g = gates_per_block; g >= 128; g /= 2)
      for (uint32_t sp = 1; sp <= 32; sp *= 2) {
        const uint32_t r = (cnt + g - 1) / g;
        const double rounds = std::ceil((double)r * KS_TILES * sp / (cus * (512 / g)));
        const double cost = rounds * ((double)(RING_N / sp) * 512.0 + (sp > 1 ? 8192.0 : 4096.0));
        if (best_cost < 0 || cost < best_cost) {
          gpb = g;
          best = sp;
          rows = r;
          best_cost = cost;
        }
      }
    const KsItem* it = items + first;
    const size_t prep = (size_t)cnt * (RING_N / 4);
    hipLaunchKernelGGL(ks_prep_kernel, dim3((uint32_t)std::min<size_t>((prep + 255) / 256, 8192)), dim3(256), 0,
                       S(stream), it, cnt, reinterpret_cast<uint2*>(dig), best > 1 ? 1 : 0);
    const dim3 grid(KS_TILES, rows, best);
    const uint32_t ipb = RING_N / best;
    const uint4* k = reinterpret_cast<const uint4*>(ksk);
    switch (gpb) {
      case 128: hipLaunchKernelGGL(ks_mfma_kernel<1>, grid, dim3(256), 0, S(stream), it, cnt, dig, k, ipb); break;
      case 256: hipLaunchKernelGGL(ks_mfma_kernel<2>, grid, dim3(256), 0, S(stream), it, cnt, dig, k, ipb); break;
      default: hipLaunchKernelGGL(ks_mfma_kernel<4>, grid, dim3(256), 0, S(stream), it, cnt, dig, k, ipb); break;
    }
    const int e = (int)hipGetLastError();
    if (e != 0) return e;
  }
  return 0;
}

int launch_make_br_items(BrItem* items, uint32_t count, const uint32_t* a, const uint32_t* b, int32_t ca, int32_t cb,
                         uint32_t cst, uint32_t mu, uint32_t* out, const uint32_t* bk, void* stream) {
  if (count == 0) return 0;
  hipLaunchKernelGGL(make_br_items_kernel, dim3((count + 255) / 256), dim3(256), 0, S(stream), items, count, a, b, ca,
                     cb, cst, mu, out, bk);
  return (int)hipGetLastError();
}

int launch_make_ks_items(KsItem* items, uint32_t count, const uint32_t* u1, const uint32_t* u2, uint32_t cst,
                         uint32_t* out, const uint32_t* ksk, void* stream) {
  if (count == 0) return 0;
  hipLaunchKernelGGL(make_ks_items_kernel, dim3((count + 255) / 256), dim3(256), 0, S(stream), items, count, u1, u2,
                     cst, out, ksk);
  return (int)hipGetLastError();
}

int launch_negate(const uint32_t* a, uint32_t* out, size_t words, void* stream) {
  if (words == 0) return 0;
  hipLaunchKernelGGL(negate_kernel, dim3(1024), dim3(256), 0, S(stream), a, out, words);
  return (int)hipGetLastError();
}

int launch_server_enc(const uint32_t* pk, uint32_t* out, size_t count, const int64_t* vals, const uint8_t* bytes,
                      uint32_t l, void* stream) {
  if (count == 0) return 0;
  const size_t words = count * CT_n;
  if (pk == out) {
    const size_t blocks = std::min<size_t>((count + 255) / 256, 8192);
    hipLaunchKernelGGL(server_enc_inplace_kernel, dim3((uint32_t)blocks), dim3(256), 0, S(stream), out, count, vals,
                       bytes, l);
  } else if ((((uintptr_t)pk | (uintptr_t)out) & 15) == 0) {
    // One 16-byte word per thread in a grid that covers the buffer in one pass
    // (grid-stride only beyond 2^31 - 1 workgroups): measured 6.3 TB/s on a
    // plain copy, against 4.8 TB/s with 4,096 workgroups of 4 words per
    // thread.  The first workgroup also covers the word tail (< 4 words).
    const size_t quads = words / 4;
    const size_t blocks = std::max<size_t>(1, std::min<size_t>((quads + 255) / 256, 0x7fffffff));
    if (words < (1ull << 32))
      hipLaunchKernelGGL((server_enc_copy_kernel<uint32_t, 1>), dim3((uint32_t)blocks), dim3(256), 0, S(stream),
                         reinterpret_cast<const uint4*>(pk), reinterpret_cast<uint4*>(out), count, vals, bytes, l);
    else
      hipLaunchKernelGGL((server_enc_copy_kernel<uint64_t, 1>), dim3((uint32_t)blocks), dim3(256), 0, S(stream),
                         reinterpret_cast<const uint4*>(pk), reinterpret_cast<uint4*>(out), count, vals, bytes, l);
  } else {
    const size_t blocks = std::min<size_t>((words + 255) / 256, 8192);
    hipLaunchKernelGGL(server_enc_word_kernel, dim3((uint32_t)blocks), dim3(256), 0, S(stream), pk, out, count, vals,
                       bytes, l);
  }
  return (int)hipGetLastError();
}

}  // namespace vlp
