// Internal types shared by the kernels and the host runtime of libvlp.
#pragma once
#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime.h>

namespace vlp {

constexpr int LWE_n = 630;          // LWE dimension (Table 5)
constexpr int RING_N = 1024;        // ring degree
constexpr int BG_BIT = 7;           // gadget base 2^7
constexpr int ELL = 3;              // gadget levels
constexpr int KS_BASEBIT = 2;       // key-switching base 2^2
constexpr int KS_T = 8;             // key-switching levels
constexpr int CT_n = LWE_n + 1;     // words of an LWE_n ciphertext
constexpr int CT_N = RING_N + 1;    // words of an LWE_N ciphertext
constexpr uint32_t MU = 0x20000000u; // 1/8

// Transformed bootstrapping key: [630][6 rows][2 components][1024] residue
// pairs (mod P1, mod P2), each polynomial in the NTT's transform order
// (layout Z, stored as [r][lane] so a wave's loads are contiguous), scaled
// by 1/1024 and kept in Montgomery form (times 2^32 mod P).
constexpr size_t BK_ROW_WORDS = (size_t)2 * ELL * 2 * 2 * RING_N;  // one key row i: [6][2][2 primes][1024] words
constexpr size_t BK_NTT_WORDS = (size_t)LWE_n * BK_ROW_WORDS;
// Key-switching key laid out for the 8-bit matrix cores, as byte planes:
// [1024 coefficients i][20 tiles of 32 output words][4 byte planes p][64
// lanes][4 words t].  Lane n + 32 h, word t holds, for output word
// 32 * tile + n and level j = 4 h + t, byte p of the entries [i][j][v] for
// v = 0..3 in bytes v = 0..3, each XOR 0x80 (a signed byte: value - 128); the
// entry v = 0 and the words past 630 are zero.
constexpr int KS_TILES = 20;                                        // 640 words / 32
constexpr size_t KSK_WORDS = (size_t)RING_N * KS_TILES * 4 * 64 * 4;  // u32 words (83,886,080 B)

// One blind rotation: input = (0, cst) + ca * a + cb * b + cm * (more[0] +
// ... + more[n_more - 1]), output the sample-extracted LWE_N ciphertext of
// BlindRotate(input, mu).
struct BrItem {
  const uint32_t* a;
  const uint32_t* b;    // may be null (then cb is ignored)
  uint32_t* out;        // [1025]
  const uint32_t* bk;   // transformed bootstrapping key
  int32_t ca, cb;
  uint32_t cst, mu;
  const uint32_t* const* more;  // n_more further operands (k-input XOR), or null
  uint32_t n_more;
  int32_t cm;
};

// One key switch: input = u1 + u2 + (0, cst) in dimension N, output LWE_n.
struct KsItem {
  const uint32_t* u1;
  const uint32_t* u2;   // may be null
  uint32_t* out;        // [631]
  const uint32_t* ksk;  // re-laid key-switching key
  uint32_t cst;
  uint32_t pad;
};

// Fixed device scratch of the allocation-free gate call (vlp_gate_noalloc):
// the sample-extracted outputs of up to 2 blind rotations per gate, then the
// blind-rotation and key-switching work items and the key-switching digits
// (2 KiB per gate), for at most
// NOALLOC_MAX_GATES gates per call.  One copy per device, in kernels.hip.
constexpr size_t NOALLOC_MAX_GATES = 1024;
constexpr size_t NOALLOC_EXT_BYTES = 2 * NOALLOC_MAX_GATES * CT_N * 4;   // multiple of 256
constexpr size_t NOALLOC_BYTES = NOALLOC_EXT_BYTES + 2 * NOALLOC_MAX_GATES * sizeof(BrItem) +
                                 NOALLOC_MAX_GATES * sizeof(KsItem) + NOALLOC_MAX_GATES * RING_N * 2;
// Device address of the current device's copy of that scratch (the HIP error
// of the lookup; call with the device current).
int noalloc_scratch_address(void** p);

// Host-side launchers (kernels.hip).  All enqueue on `stream` and return the
// HIP error of the launch.
int launch_bk_transform(const uint32_t* bk_coeff, uint32_t* bk_ntt, const uint4* tw_fwd, void* stream);
int launch_ksk_relayout(const uint32_t* ksk_in, uint32_t* ksk_out, void* stream);
int launch_br(const BrItem* items, uint32_t count, const uint4* tw_fwd, uint32_t waves_per_block, uint32_t blocks,
              void* stream);
// ServerEnc over a flat [count][631] array; out == pk runs in place.
int launch_server_enc(const uint32_t* pk, uint32_t* out, size_t count, const int64_t* vals, const uint8_t* bytes,
                      uint32_t l, void* stream);
// Two wavefronts per rotation (one per prime), rot_per_block (1, 2, 4) rotations per workgroup.
int launch_br2(const BrItem* items, uint32_t count, const uint4* tw_fwd, uint32_t rot_per_block, uint32_t blocks,
               void* stream);
// Four wavefronts per rotation (prime x accumulator half), one rotation per workgroup.
int launch_br4(const BrItem* items, uint32_t count, const uint4* tw_fwd, uint32_t blocks, void* stream);
// Key switching of count items on the matrix cores, in launches of at most
// KS_CHUNK gates; dig: device scratch of ks_digit_bytes(count) bytes;
// gates_per_block is the most gates a workgroup takes (128, 256 or 512), cus
// the device's CUs.
constexpr uint32_t KS_CHUNK = 16384;
constexpr size_t ks_digit_bytes(size_t count) { return (count < KS_CHUNK ? count : KS_CHUNK) * (RING_N * 2); }
int launch_ks_group(const KsItem* items, uint32_t count, const uint32_t* ksk, uint32_t* dig,
                    uint32_t gates_per_block, uint32_t cus, void* stream);
int launch_make_br_items(BrItem* items, uint32_t count, const uint32_t* a, const uint32_t* b, int32_t ca, int32_t cb,
                         uint32_t cst, uint32_t mu, uint32_t* out, const uint32_t* bk, void* stream);
int launch_make_ks_items(KsItem* items, uint32_t count, const uint32_t* u1, const uint32_t* u2, uint32_t cst,
                         uint32_t* out, const uint32_t* ksk, void* stream);
int launch_negate(const uint32_t* a, uint32_t* out, size_t words, void* stream);

// Twiddle table (host), 4 words per m < 1024: {w1, Shoup(w1), w2, Shoup(w2)}
// with w_k = psi_k^brv10(m) mod P_k (the inverse transform reads it too).
void make_twiddles(uint32_t* tw);
// Per prime {N^-1 2^32 mod P, its Shoup quotient}: the key's scale factor.
void key_scale(uint32_t out[4]);

}  // namespace vlp
