// Measured integer peak of the blind rotation's arithmetic.
//
// The algorithmic count of a blind rotation is its modular multiplications:
// per CMux, 8 transforms of (N/2) log2 N butterflies (one multiplication
// each) and 12 N pointwise key products (Section 2.2: the external product
// of a CMux, computed with negacyclic transforms); each is carried out as one
// residue butterfly per prime of the two-prime residue system.  The bound
// such a count is priced against can be derived from the instruction set
// (lanes x clock divided by the VALU instructions of one multiplication) or
// measured: this file measures it, with the very residue butterflies the
// transforms execute (wave_ntt.h: lazy signed Cooley-Tukey forward,
// Gentleman-Sande inverse, Shoup products), on register-resident values,
// every CU busy and no memory traffic inside the loop.
#include <hip/hip_runtime.h>

#include "vlp.h"
#include "wave_ntt.h"

namespace vlp {
namespace {

constexpr int PEAK_THREADS = 256;
constexpr int PEAK_WAVES_PER_CU = 32;  // 8 per SIMD: enough to hide the multiply latency
constexpr int PEAK_ITERS = 2048;
constexpr int BFLY_PER_ITER = 4 * 8;   // four stages (register strides 8, 4, 2, 1) of 8 butterflies

// One lane's 16 residues, transformed over and over by the stages a
// transform runs inside a lane.
template <bool INV>
__global__ __launch_bounds__(PEAK_THREADS) void butterfly_peak_kernel(uint32_t* out, uint32_t seed, int iters) {
  constexpr uint32_t p = Prime<0>::P;
  const uint32_t tid = blockIdx.x * PEAK_THREADS + threadIdx.x;
  uint32_t x[16], w[8], wp[8];
#pragma unroll
  for (int r = 0; r < 16; ++r) x[r] = ((seed ^ (tid * 16u + r)) * 2654435761u) % p;
#pragma unroll
  for (int k = 0; k < 8; ++k) {  // signed twiddles |w| < p/2 with floor(w 2^32 / p), as the tables hold
    const int64_t w0 = ((seed + tid) * (2u * k + 3u) + 12345u * k) % p;
    const int64_t ws = w0 > p / 2 ? w0 - (int64_t)p : w0;
    const int64_t n = ws * ((int64_t)1 << 32);
    w[k] = (uint32_t)(int32_t)ws;
    wp[k] = (uint32_t)(int32_t)(n / (int64_t)p - ((n % (int64_t)p != 0 && n < 0) ? 1 : 0));
    // Opaque from here on, as twiddles read from memory are: otherwise the
    // compiler folds their derivation into the products.
    asm volatile("" : "+v"(w[k]), "+v"(wp[k]));
  }
  for (int i = 0; i < iters; ++i) {
    // Forward: the transform's butterflies never reduce, so over the loop's
    // thousands of stages the values leave the residue ranges and wrap
    // modulo 2^32; the instructions, and so their timing, do not depend on
    // the values.  Inverse: sums double the bound three times (2P -> 16P) and
    // the fourth stage reduces them, the pattern of the inverse transform.
#pragma unroll
    for (int k = 0; k < 8; ++k) {  // register stride 8
      const int r = bfly_reg<3>(k);
      if (INV) bfly_gs_neg<2, false>(x[r], x[r | 8], w[k], wp[k], p); else bfly_ct(x[r], x[r | 8], w[k], wp[k], p);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {  // stride 4
      const int r = bfly_reg<2>(k);
      if (INV) bfly_gs_neg<4, false>(x[r], x[r | 4], w[k], wp[k], p); else bfly_ct(x[r], x[r | 4], w[k], wp[k], p);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {  // stride 2
      const int r = bfly_reg<1>(k);
      if (INV) bfly_gs_neg<8, false>(x[r], x[r | 2], w[k], wp[k], p); else bfly_ct(x[r], x[r | 2], w[k], wp[k], p);
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {  // stride 1
      const int r = bfly_reg<0>(k);
      if (INV) bfly_gs_neg<16, true>(x[r], x[r | 1], w[k], wp[k], p); else bfly_ct(x[r], x[r | 1], w[k], wp[k], p);
    }
  }
  uint32_t s = 0;
#pragma unroll
  for (int r = 0; r < 16; ++r) s ^= x[r];
  out[tid] = s;  // keeps the loop live; one word per thread, inside the buffer
}

}  // namespace
}  // namespace vlp

extern "C" vlp_status vlp_measure_modmul_peak(int device, double* fwd_per_s, double* inv_per_s, double* mixed_per_s) {
  using namespace vlp;
  if (!fwd_per_s || !inv_per_s || !mixed_per_s) return VLP_EINVAL;
  int n_dev = 0;
  if (hipGetDeviceCount(&n_dev) != hipSuccess) return VLP_EHIP;
  if (device < 0 || device >= n_dev) return VLP_EINVAL;
  int old = 0;
  if (hipGetDevice(&old) != hipSuccess || hipSetDevice(device) != hipSuccess) return VLP_EHIP;
  int cus = 0;
  uint32_t* out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  vlp_status status = VLP_OK;
  double rate[2] = {0, 0};
  do {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0) {
      status = VLP_EHIP;
      break;
    }
    const int blocks = cus * PEAK_WAVES_PER_CU * 64 / PEAK_THREADS;
    if (hipMalloc((void**)&out, (size_t)blocks * PEAK_THREADS * sizeof(uint32_t)) != hipSuccess ||
        hipStreamCreate(&st) != hipSuccess || hipEventCreate(&ev[0]) != hipSuccess ||
        hipEventCreate(&ev[1]) != hipSuccess) {
      status = VLP_EHIP;
      break;
    }
    const double bfly = (double)blocks * PEAK_THREADS * PEAK_ITERS * BFLY_PER_ITER;
    for (int inv = 0; inv < 2 && status == VLP_OK; ++inv) {
      float best = 0;
      for (int rep = 0; rep < 4; ++rep) {  // the first launch warms up; the fastest of the others counts
        if (hipEventRecord(ev[0], st) != hipSuccess) { status = VLP_EHIP; break; }
        if (inv)
          hipLaunchKernelGGL(butterfly_peak_kernel<true>, dim3(blocks), dim3(PEAK_THREADS), 0, st, out, 0x5EEDu + rep, PEAK_ITERS);
        else
          hipLaunchKernelGGL(butterfly_peak_kernel<false>, dim3(blocks), dim3(PEAK_THREADS), 0, st, out, 0x5EEDu + rep, PEAK_ITERS);
        float ms = 0;
        if (hipGetLastError() != hipSuccess || hipEventRecord(ev[1], st) != hipSuccess ||
            hipEventSynchronize(ev[1]) != hipSuccess || hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) {
          status = VLP_EHIP;
          break;
        }
        if (rep > 0 && (best == 0 || ms < best)) best = ms;
      }
      if (status == VLP_OK) rate[inv] = bfly / (best * 1e-3);
    }
  } while (0);
  if (ev[0]) (void)hipEventDestroy(ev[0]);
  if (ev[1]) (void)hipEventDestroy(ev[1]);
  if (st) (void)hipStreamDestroy(st);
  if (out) (void)hipFree(out);
  (void)hipSetDevice(old);
  if (status != VLP_OK) return status;
  *fwd_per_s = rate[0];
  *inv_per_s = rate[1];
  // A CMux runs six forward transforms and two inverse ones of equal size.
  *mixed_per_s = 8.0 / (6.0 / rate[0] + 2.0 / rate[1]);
  return VLP_OK;
}
