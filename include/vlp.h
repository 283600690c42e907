/*
 * vlp.h -- C ABI of the MI355X TFHE gate-bootstrapping library (libvlp.so).
 *
 * The library is the server side of VeLoPIR (arXiv 2506.12761): it holds a
 * client's evaluation keys (Section 3.2, preprocessing: the client sends evk)
 * and evaluates the validation, zero-out and aggregation circuits of
 * Algorithm 3 over ciphertexts in device memory.  It generates no keys and
 * encrypts nothing: keys and ciphertexts come from the caller.
 *
 * Scheme and parameters (Table 5, 128-bit set): LWE dimension n = 630,
 * ring degree N = 1024, k = 1, bootstrapping-key gadget base 2^7 with 3
 * levels, key-switching base 2^2 with 8 levels.  All torus values are
 * uint32_t words modulo 2^32.  A bit m is encoded as m/4 - 1/8
 * (Section 2.2): 0x20000000 for 1, 0xE0000000 for 0.
 *
 * Data layouts (all arrays dense, row-major, little-endian uint32_t):
 *   LWE_n ciphertext : [631]  = a[0..629], b
 *   LWE_N ciphertext : [1025] = a[0..1023], b  (sample-extracted, key S)
 *   bootstrapping key: [630][6][2][1024], row r = c*3 + j of BK_i is a TRLWE
 *                      encryption of zero plus s_i * 2^(32-7(j+1)) on the
 *                      constant coefficient of component c (c = 0 mask, 1 body)
 *   key-switching key: [1024][8][4][631], entry [i][j][v] encrypts
 *                      v * S_i * 2^(32-2(j+1)) under s; entry v = 0 is ignored
 *
 * Conventions of the bootstrap (the paper names BlindRotate, SampleExtract and
 * KeySwitch in Section 2.2 and defers their definition to the TFHE method it
 * cites; these are the integer readings implemented):
 *   modulus switch  a~ = floor(((x + 2^20) mod 2^32) / 2^21) in [0, 2048)
 *   test polynomial v = mu * (1 + X + ... + X^1023), acc = (0, X^-b~ v)
 *   CMux i          acc += BK_i (x) (X^a~_i acc - acc), for i = 0..629
 *   decomposition   balanced base-2^7 digits in [-64, 63] of x rounded to 21 bits
 *   SampleExtract   a'_0 = A_0, a'_j = -A_(N-j), b' = B_0
 *   KeySwitch       r = (0, b') - sum over i < 1024, j < 8 of ksk[i][j][d_ij],
 *                   d_ij = bits [30-2j, 32-2j) of a'_i + 2^15
 * The polynomial products are exact (no rounding): the result words are a
 * deterministic function of the inputs and keys.
 *
 * Ownership and asynchrony: every pointer argument named *_dev is a device
 * pointer owned by the caller; the library never frees it.  Calls enqueue
 * work on the context's HIP stream and return without waiting; inputs must
 * stay valid and outputs unread until vlp_sync() returns (or the stream has
 * passed the call).  A vlp_keyset owns its transformed keys; a vlp_ctx owns
 * its scratch memory, bounded by the budget given at creation.
 *
 * Errors: every call returns a vlp_status; nothing is thrown across the ABI
 * and nothing aborts.  vlp_last_error() returns a message for the last failed
 * call on that context (valid until the next call on the same context).
 * A context is not thread-safe: one host thread at a time per context.
 */
#ifndef VLP_H
#define VLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VLP_OK = 0,
    VLP_EINVAL = -1,  /* bad argument: null pointer, size, shape or overlap */
    VLP_EBUDGET = -2, /* the call would exceed the context's device-memory budget */
    VLP_EHIP = -3,    /* a HIP runtime call failed (message holds its error string) */
    VLP_EPARAM = -4,  /* parameters differ from the supported Table 5 set */
    VLP_EBUSY = -5    /* object still in use (e.g. a keyset referenced by live programs) */
} vlp_status;

typedef enum { VLP_AND = 0, VLP_OR = 1, VLP_NAND = 2, VLP_XOR = 3, VLP_XNOR = 4, VLP_NOT = 5, VLP_MUX = 6 } vlp_gate_op;

/* Validation modes of Section 4: interval validation (Alg. 4), coordinate
 * validation (Alg. 8) and identifier matching (HomEQ on identifier bits). */
typedef enum { VLP_INTV = 0, VLP_COV = 1, VLP_IDM = 2 } vlp_mode;

/* Parameter set; must equal {630, 1024, 1, 7, 3, 2, 8} (Table 5). */
typedef struct {
    uint32_t n, N, k, bg_bit, ell, ks_basebit, ks_t;
} vlp_params;

/* Query shape (Section 3.2, "Secure Parameter Transmission"): M records,
 * l_I bits per coordinate or identifier, l_S payload bits per record,
 * d coordinates (1 or 2 for IntV and CoV; ignored for IdM). */
typedef struct {
    vlp_mode mode;
    uint32_t M, l_I, l_S, d;
} vlp_shape;

/* The circuits that evaluate a shape (Section 6.1).
 * optimized = 1 uses the OPT circuits (Alg. 11 comparators, Alg. 12 equality
 * tree, pairwise XOR aggregation); 0 uses Alg. 7's AND chain and Alg. 10's
 * XOR chain from a trivial zero.
 * agg_k = 0 aggregates as `optimized` says; 2 <= agg_k <= 16 replaces the
 * aggregation (HomSum, Alg. 10) by a tree of k-input XORs, each one bootstrap
 * of (0, (k-1)/4) + 2 * (sum of its k inputs): records' selected bits in
 * consecutive groups of k, a group of one passed through, repeated on the
 * group results.  Not in the paper; k <= 16 keeps the summed input noise
 * (4k times a gate output's) beyond 8 standard deviations of the 1/4
 * decision distance.
 * The calls that take a shape use {optimized = 1, agg_k = 0}; their _ex
 * forms take the circuits as an extra argument (NULL: that default).
 * VLP_EINVAL for agg_k = 1 or agg_k > 16. */
typedef struct {
    uint32_t optimized;
    uint32_t agg_k;
} vlp_circuit;

typedef struct vlp_ctx vlp_ctx;
typedef struct vlp_keyset vlp_keyset;
typedef struct vlp_program vlp_program;

/* Library version string (static storage). */
const char *vlp_version(void);

/* Fills *p with the supported parameter set. */
void vlp_default_params(vlp_params *p);

/* Create a context on HIP device `device`.  hip_stream: a hipStream_t to run
 * on, or NULL for a stream the context creates and owns.  hbm_budget: bytes
 * of device memory the context may allocate for keysets and programs
 * (0 = 90% of the device's memory).  VLP_EPARAM if *p is not Table 5. */
vlp_status vlp_ctx_create(vlp_ctx **out, const vlp_params *p, int device, void *hip_stream, size_t hbm_budget);

/* Destroys the context; every keyset and program made on it must be
 * destroyed first (VLP_EBUSY otherwise). */
vlp_status vlp_ctx_destroy(vlp_ctx *ctx);

/* Message for the last failed call on ctx ("" if none; ctx may be NULL for
 * failures of vlp_ctx_create). */
const char *vlp_last_error(const vlp_ctx *ctx);

/* Bytes of device memory the context currently holds, and its budget. */
vlp_status vlp_mem_info(const vlp_ctx *ctx, size_t *used, size_t *budget);

/* Load a client's evaluation keys (Section 3.2: evk = bootstrapping key and
 * key-switching key).  bk_dev: [630][6][2][1024], ksk_dev: [1024][8][4][631]
 * device arrays in the layouts above; they are read during the call's stream
 * work and may be freed after vlp_sync().  The keyset holds the bootstrapping
 * key transformed for the exact negacyclic products (61,931,520 B) and the
 * key-switching key as signed byte planes for the 8-bit matrix cores
 * (83,886,080 B).  VLP_EBUDGET if it does not fit. */
vlp_status vlp_keyset_load(vlp_ctx *ctx, const uint32_t *bk_dev, const uint32_t *ksk_dev, vlp_keyset **out);

/* Frees a keyset (VLP_EBUSY while programs made with it are alive). */
vlp_status vlp_keyset_destroy(vlp_keyset *ks);

/* Bootstrap without key switching, elementwise over B ciphertexts:
 * out[b] = SampleExtract(BlindRotate(in[b], mu)).
 * in_dev [B][631], out_dev [B][1025]; mu is the test-polynomial value
 * (0x20000000 for the gates).  B = 0 is a no-op. */
vlp_status vlp_bootstrap(vlp_ctx *ctx, const vlp_keyset *ks, const uint32_t *in_dev, uint32_t *out_dev, uint32_t mu, size_t B);

/* Key switching, elementwise: in_dev [B][1025] (key S) -> out_dev [B][631] (key s). */
vlp_status vlp_keyswitch(vlp_ctx *ctx, const vlp_keyset *ks, const uint32_t *in_dev, uint32_t *out_dev, size_t B);

/* Bootstrapped gates, elementwise over B: out[b] = op(a[b], b[b], c[b]).
 * Pre-combinations (Section 2.2 gives AND; the others are the same
 * construction with other constants):
 *   AND  (0,-1/8) + a + b     OR   (0, 1/8) + a + b    NAND (0, 1/8) - a - b
 *   XOR  (0, 1/4) + 2(a + b)  XNOR (0,-1/4) - 2(a + b) NOT  -a (no bootstrap)
 *   MUX(a = select, b = if 1, c = if 0): KS((0, 1/8) + u1 + u2) with
 *        u1 = BR+SE((0,-1/8) + a + b), u2 = BR+SE((0,-1/8) - a + c).
 * a_dev, b_dev, c_dev, out_dev: [B][631]; b_dev is ignored (may be NULL) for
 * NOT, c_dev must be NULL except for MUX.  out_dev may not overlap inputs. */
vlp_status vlp_gate(vlp_ctx *ctx, const vlp_keyset *ks, vlp_gate_op op, const uint32_t *a_dev, const uint32_t *b_dev,
                    const uint32_t *c_dev, uint32_t *out_dev, size_t B);

/* vlp_gate for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same gates, bit for bit, with the intermediate ciphertexts and work items
 * in a fixed scratch array that the library holds on each device for the
 * life of the process (10,665,984 B), so the call makes no hipMalloc/hipFree.
 * B <= 1024 gates per call (VLP_EINVAL above that).  Every call on one
 * device shares that device's array: calls that overlap in time on the same
 * device (two contexts or two streams) race and give wrong results; calls
 * ordered on one stream are safe.  Kernel timing (vlp_profile_enable) does
 * not cover this call.  Arguments and errors otherwise as vlp_gate. */
vlp_status vlp_gate_noalloc(vlp_ctx *ctx, const vlp_keyset *ks, vlp_gate_op op, const uint32_t *a_dev,
                            const uint32_t *b_dev, const uint32_t *c_dev, uint32_t *out_dev, size_t B);

/* Mode-level evaluation of Algorithm 3 for one query.
 *   query_dev : IntV/CoV [d][l_I][631] (coordinate k, bit j LSB first);
 *               IdM [l_I][631]
 *   db_loc_dev: IntV [M][d][2][l_I][631] (left bound, right bound, for the
 *               half-open interval left <= x < right, signed two's complement);
 *               CoV [M][d][l_I][631]; IdM [M][l_I][631]
 *   db_pay_dev: [M][l_S][631] payload bits, or NULL when l_S = 0
 *   R_dev     : [l_S][631] aggregated result (NULL when l_S = 0)
 *   v_out_dev : [M][631] validation bits, or NULL
 * The call builds (or reuses) the level schedule of the circuit and enqueues
 * it; intermediate ciphertexts are held within the context budget. */
vlp_status vlp_evaluate(vlp_ctx *ctx, const vlp_keyset *ks, const vlp_shape *shape, const uint32_t *query_dev,
                        const uint32_t *db_loc_dev, const uint32_t *db_pay_dev, uint32_t *R_dev, uint32_t *v_out_dev);
vlp_status vlp_evaluate_ex(vlp_ctx *ctx, const vlp_keyset *ks, const vlp_shape *shape, const vlp_circuit *circuit,
                           const uint32_t *query_dev, const uint32_t *db_loc_dev, const uint32_t *db_pay_dev,
                           uint32_t *R_dev, uint32_t *v_out_dev);

/* ServerEnc (Alg. 2): the server encrypts its plaintext database under the
 * client's public key (Alg. 1: one encryption of zero per database bit), so
 * no secret key is needed: each slot becomes pk + (0, Ecd(bit)).
 *   pk_loc / out_loc: location slots in db_loc_dev's layout of vlp_evaluate
 *                     (IntV [M][d][2][l_I][631], CoV [M][d][l_I][631],
 *                     IdM [M][l_I][631])
 *   loc             : int64 values, IntV [M][d][2] (left, right bound),
 *                     CoV [M][d], IdM [M]; slot bit j is bit j (LSB first) of
 *                     the value's two's-complement form
 *   pk_pay / out_pay: [M][l_S][631]; pay: [M][l_S] bytes, nonzero = bit 1
 *                     (all three NULL when l_S = 0)
 * All device pointers.  An output may equal its public key exactly (in
 * place: only body words are written); otherwise outputs may not overlap any
 * argument (VLP_EINVAL).  Enqueued on the context's stream; inputs must stay
 * valid until it has run. */
vlp_status vlp_server_encrypt(vlp_ctx *ctx, const vlp_shape *shape, const uint32_t *pk_loc, const uint32_t *pk_pay,
                              const int64_t *loc, const uint8_t *pay, uint32_t *out_loc, uint32_t *out_pay);

/* ---- Programs: an evaluation bound to its buffers, advanced level by level.
 * vlp_program_create builds the gate schedule of vlp_evaluate's arguments
 * and reserves its intermediate storage and its share of the context's
 * merged-step scratch (VLP_EBUDGET if the budget, or the device, cannot hold
 * it), so that vlp_step itself allocates nothing.  vlp_step advances every unfinished program in progs[] by one
 * circuit level in one merged batch of kernel launches, so gates of several
 * programs, keysets and modes share the same launches; *remaining receives
 * the number of programs in progs[] that still have levels to run; a program
 * listed twice is VLP_EINVAL (nothing is enqueued).
 * vlp_program_run runs all remaining levels of one program; with use_graph
 * != 0 the level sequence is captured once in a HIP graph and replayed on
 * later runs of the same program (inputs are re-read from the bound buffers
 * on every run; a change of vlp_set_tuning since the capture captures again;
 * a program that vlp_step has already advanced runs its remaining levels
 * without the graph). */
vlp_status vlp_program_create(vlp_ctx *ctx, const vlp_keyset *ks, const vlp_shape *shape, const uint32_t *query_dev,
                              const uint32_t *db_loc_dev, const uint32_t *db_pay_dev, uint32_t *R_dev,
                              uint32_t *v_out_dev, vlp_program **out);
vlp_status vlp_program_create_ex(vlp_ctx *ctx, const vlp_keyset *ks, const vlp_shape *shape,
                                 const vlp_circuit *circuit, const uint32_t *query_dev, const uint32_t *db_loc_dev,
                                 const uint32_t *db_pay_dev, uint32_t *R_dev, uint32_t *v_out_dev, vlp_program **out);
vlp_status vlp_program_reset(vlp_program *prog);
vlp_status vlp_step(vlp_ctx *ctx, vlp_program *const *progs, size_t n_progs, size_t *remaining);
vlp_status vlp_program_run(vlp_ctx *ctx, vlp_program *prog, int use_graph);
/* Static counts of a program: gates, blind rotations, key switches, levels. */
/* The same counts for a shape, computed on the host without a device. */
vlp_status vlp_plan_counts(const vlp_shape *shape, uint64_t *gates, uint64_t *blind_rotations, uint64_t *key_switches,
                           uint32_t *levels);
vlp_status vlp_plan_counts_ex(const vlp_shape *shape, const vlp_circuit *circuit, uint64_t *gates,
                              uint64_t *blind_rotations, uint64_t *key_switches, uint32_t *levels);
/* Device bytes vlp_program_create would reserve against the budget for a
 * shape (with or without a v_out buffer), computed on the host: work items,
 * intermediate ciphertexts, key-switching digits and the program's share of
 * the merged-step scratch that vlp_step uses.  A server can admit a request
 * only when these bytes (plus its input buffers) fit.  VLP_EINVAL for a bad
 * shape or a NULL argument. */
vlp_status vlp_plan_bytes(const vlp_shape *shape, int with_v_out, size_t *bytes);
vlp_status vlp_plan_bytes_ex(const vlp_shape *shape, const vlp_circuit *circuit, int with_v_out, size_t *bytes);
/* Blind rotations and key switches of one level (0-based) of a program;
 * VLP_EINVAL past the last level. */
vlp_status vlp_program_level_counts(const vlp_program *prog, uint32_t level, uint64_t *blind_rotations,
                                   uint64_t *key_switches);
vlp_status vlp_program_counts(const vlp_program *prog, uint64_t *gates, uint64_t *blind_rotations,
                              uint64_t *key_switches, uint32_t *levels);
vlp_status vlp_program_destroy(vlp_program *prog);

/* ---- Tuning knobs of the batched kernels (picked by the autotuner).
 * br_waves_per_rotation : wavefronts per blind rotation:
 *                          1 = both RNS primes in one wavefront;
 *                          2 = one wavefront per prime;
 *                          4 = one per prime and accumulator half (half the
 *                              latency of 2 per rotation, half the rotations
 *                              in flight; one rotation per workgroup);
 *                          0 = automatic (default): launches of at most 2
 *                              rotations per CU use 4 (2 workgroups per CU),
 *                              larger ones 2 in full rounds, a short last
 *                              round again 4
 * br_rotations_per_block: rotations per workgroup (1 wavefront per rotation:
 *                          1, 2, 4, 8 -- 8 puts two on a SIMD at half the
 *                          registers each; 2 wavefronts per rotation: 1, 2, 4
 *                          -- the rotations of a workgroup advance in
 *                          lockstep and share key reads; 4: 1)
 * br_blocks_per_cu      : workgroups per compute unit a launch is sized for
 *                          (1..64); one launch covers br_blocks_per_cu x
 *                          br_rotations_per_block rotations per CU
 * ks_gates_per_block    : most gates a key-switching workgroup takes, sharing
 *                          its reads of the key (128, 256, 512 (default));
 *                          each launch picks the tile (up to this) and the
 *                          split of the coefficients over workgroups */
typedef struct {
    uint32_t br_rotations_per_block;
    uint32_t br_blocks_per_cu;
    uint32_t ks_gates_per_block;
    uint32_t br_waves_per_rotation;
} vlp_tuning;
vlp_status vlp_get_tuning(const vlp_ctx *ctx, vlp_tuning *t);
vlp_status vlp_set_tuning(vlp_ctx *ctx, const vlp_tuning *t);

/* ---- Kernel timing.  While enabled, every blind-rotation and key-switching
 * kernel launch the context makes outside graph capture is bracketed by HIP
 * events on the context's stream.  vlp_profile_read waits for the stream,
 * returns the totals since the last read (or enable) and clears them. */
typedef struct {
    uint64_t launches;  /* kernel launches timed */
    uint64_t items;     /* blind rotations (or key switches) they processed */
    double ms;          /* summed launch durations, milliseconds */
} vlp_kernel_stats;
vlp_status vlp_profile_enable(vlp_ctx *ctx, int enable);
vlp_status vlp_profile_read(vlp_ctx *ctx, vlp_kernel_stats *br, vlp_kernel_stats *ks);

/* ---- Measured arithmetic peak.  The count a blind rotation is priced by is
 * its modular multiplications (per CMux of Section 2.2: 8 negacyclic
 * transforms of 512 x 10 butterflies and 12 x 1024 key products), each
 * computed as one residue butterfly per prime of the two-prime residue
 * system.  This call measures the rate at which HIP device `device` runs the
 * transforms' own residue butterflies (lazy signed forward Cooley-Tukey and
 * inverse Gentleman-Sande with Shoup products) on register-resident values
 * with every CU busy: *fwd_per_s and *inv_per_s for each kind, *mixed_per_s
 * for the 6:2 forward:inverse mix of a CMux (residue butterflies per second;
 * halve for modular multiplications per second).  It
 * blocks for about 0.1 s, allocates and frees a small device buffer and a
 * stream of its own, and needs no context.  VLP_EINVAL for a null output or
 * a bad device; VLP_EHIP if a HIP call fails (no message: there is no
 * context to hold it). */
vlp_status vlp_measure_modmul_peak(int device, double *fwd_per_s, double *inv_per_s, double *mixed_per_s);

/* Wait until all work enqueued on the context's stream has finished. */
vlp_status vlp_sync(vlp_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* VLP_H */
