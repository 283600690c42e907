/*
 * CPU oracle for TFHE gate bootstrapping (torus32, 128-bit parameter set).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant
 * generator with the GPU path: its number-theoretic transform runs modulo its
 * own prime P = 2^62 - 2^16 + 1, different from the GPU's.
 *
 * What is computed, and where it comes from (paper: VeLoPIR, arXiv 2506.12761):
 *   - Parameters: Table 5 (n = 630, N = 1024, k = 1, BK base 2^7 with 3
 *     levels, key switching base 2^2 with 8 levels).
 *   - Encoding Ecd(m) = m/4 - 1/8, encryption b = <a,s> + mu + e, decryption
 *     by the sign of the phase: Section 2.2 (TLWE encryption scheme).
 *   - Gate = Bootstrap(linear pre-combination): Section 2.2, HomAND equation;
 *     Bootstrap = BlindRotate, SampleExtract, KeySwitch, which the paper names
 *     and defers to the TFHE method it cites.  The integer conventions used
 *     for those three steps (rounding of the modulus switch, balanced digits,
 *     key-switching digits, test polynomial) are the readings recorded in the
 *     design notes; each function below states the one it implements.
 *
 * All torus arithmetic is exact arithmetic modulo 2^32 on uint32_t.  The
 * negacyclic polynomial products have a plain definition (the schoolbook sum
 * below); the default path reaches the same integers through an exact
 * negacyclic NTT, used as a library-style primitive and pinned against the
 * schoolbook sum by the test-suite.  Each product is computed on its own and
 * lifted back to an integer before it is summed, exactly as the external
 * product is defined.
 *
 * Parity status: every function here is pinned by tests (schoolbook and
 * brute force, closed-form bootstraps with degenerate keys, decryption of
 * every gate's truth table, plaintext predicates of the circuits).  The
 * ciphertext words themselves are not printed in the paper, so bit-level
 * values are pinned only through those properties.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_n 630
#define ORC_N 1024
#define ORC_BGBIT 7
#define ORC_ELL 3
#define ORC_KS_BASEBIT 2
#define ORC_KS_T 8
#define ORC_KS_BASE 4
#define ORC_MU 0x20000000u /* 1/8 on the torus */

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* Arithmetic modulo the oracle prime P = 2^62 - 2^16 + 1 (2^16 | P - 1).    */
/* ------------------------------------------------------------------------ */
#define ORC_P 0x3fffffffffff0001ull

static uint64_t addm(uint64_t a, uint64_t b) { uint64_t s = a + b; return s >= ORC_P ? s - ORC_P : s; }
static uint64_t subm(uint64_t a, uint64_t b) { return a >= b ? a - b : a + ORC_P - b; }
/* Multiply, then take the remainder of the full 128-bit product. */
static uint64_t mulm_slow(uint64_t a, uint64_t b) { return (uint64_t)(((u128)a * b) % ORC_P); }

static uint64_t powm(uint64_t b, uint64_t e) {
    uint64_t r = 1;
    b %= ORC_P;
    while (e) {
        if (e & 1) r = mulm_slow(r, b);
        b = mulm_slow(b, b);
        e >>= 1;
    }
    return r;
}

/* Montgomery multiplication with R = 2^64 (Montgomery, Math. Comp. 1985):
 * mont(x, y) = x*y*R^-1 mod P for x, y < P.  With y stored as y*R mod P
 * ("Montgomery form") it returns the plain product x*y mod P. */
static uint64_t g_pinv_neg; /* -P^-1 mod 2^64 */
static uint64_t g_r_mod_p;  /* 2^64 mod P */

static uint64_t mont(uint64_t x, uint64_t y) {
    u128 T = (u128)x * y;
    uint64_t m = (uint64_t)T * g_pinv_neg;
    u128 t = (T + (u128)m * ORC_P) >> 64;
    uint64_t r = (uint64_t)t;
    return r >= ORC_P ? r - ORC_P : r;
}
static uint64_t to_mont(uint64_t y) { return mulm_slow(y, g_r_mod_p); }

/* ------------------------------------------------------------------------ */
/* Negacyclic NTT of length N (power of two, 2 <= N <= 1024) modulo P.       */
/*   forward:  A_k = sum_j a_j psi^((2k+1) j),  k = 0..N-1 (natural order)   */
/*   inverse:  a_j = N^-1 psi^-j sum_k A_k psi^(-2jk)                         */
/* psi is a primitive 2N-th root of unity.  Implemented as the twist a_j*psi^j */
/* followed by a cyclic radix-2 transform in omega = psi^2.                  */
/* ------------------------------------------------------------------------ */
typedef struct {
    int N;
    uint64_t psi;                  /* primitive 2N-th root */
    uint64_t twist[ORC_N];         /* psi^j, Montgomery form */
    uint64_t untwist[ORC_N];       /* N^-1 psi^-j, Montgomery form */
    uint64_t w[ORC_N / 2];         /* omega^k, Montgomery form */
    uint64_t winv[ORC_N / 2];      /* omega^-k, Montgomery form */
} ntt_plan;

static ntt_plan g_plans[11]; /* index log2 N */
static int g_ready = 0;

static uint64_t primitive_root_2n(int N) {
    /* x^((P-1)/2N) has order dividing 2N; it is primitive iff its N-th power is -1. */
    for (uint64_t x = 2;; ++x) {
        uint64_t y = powm(x, (ORC_P - 1) / (uint64_t)(2 * N));
        if (powm(y, (uint64_t)N) == ORC_P - 1) return y;
    }
}

static void plan_init(ntt_plan *pl, int N) {
    pl->N = N;
    pl->psi = primitive_root_2n(N);
    uint64_t psi_inv = powm(pl->psi, ORC_P - 2);
    uint64_t ninv = powm((uint64_t)N, ORC_P - 2);
    uint64_t omega = mulm_slow(pl->psi, pl->psi), omega_inv = mulm_slow(psi_inv, psi_inv);
    uint64_t t = 1, ti = ninv;
    for (int j = 0; j < N; ++j) {
        pl->twist[j] = to_mont(t);
        pl->untwist[j] = to_mont(ti);
        t = mulm_slow(t, pl->psi);
        ti = mulm_slow(ti, psi_inv);
    }
    uint64_t w = 1, wi = 1;
    for (int k = 0; k < N / 2; ++k) {
        pl->w[k] = to_mont(w);
        pl->winv[k] = to_mont(wi);
        w = mulm_slow(w, omega);
        wi = mulm_slow(wi, omega_inv);
    }
}

void orc_init(void) {
    if (g_ready) return;
    /* Newton iteration for P^-1 mod 2^64 (P odd, so P*P = 1 mod 8 seeds it). */
    uint64_t inv = ORC_P;
    for (int i = 0; i < 6; ++i) inv *= 2 - ORC_P * inv;
    g_pinv_neg = (uint64_t)0 - inv;
    g_r_mod_p = (uint64_t)(((u128)1 << 64) % ORC_P);
    for (int lg = 1; lg <= 10; ++lg) plan_init(&g_plans[lg], 1 << lg);
    g_ready = 1;
}

static const ntt_plan *plan_for(int N) {
    int lg = 0;
    while ((1 << lg) < N) ++lg;
    return &g_plans[lg];
}

/* In-place cyclic transform A_k = sum_j a_j w^(jk) (w given as a power table). */
static void cyclic_ntt(uint64_t *a, int N, const uint64_t *wtab) {
    for (int i = 1, j = 0; i < N; ++i) { /* bit-reversal permutation */
        int bit = N >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) { uint64_t t = a[i]; a[i] = a[j]; a[j] = t; }
    }
    for (int len = 2; len <= N; len <<= 1) {
        int half = len >> 1, step = N / len;
        for (int i = 0; i < N; i += len)
            for (int k = 0; k < half; ++k) {
                uint64_t u = a[i + k];
                uint64_t v = mont(a[i + k + half], wtab[k * step]);
                a[i + k] = addm(u, v);
                a[i + k + half] = subm(u, v);
            }
    }
}

void orc_ntt_forward(int N, const uint64_t *in, uint64_t *out) {
    const ntt_plan *pl = plan_for(N);
    for (int j = 0; j < N; ++j) out[j] = mont(in[j] % ORC_P, pl->twist[j]);
    cyclic_ntt(out, N, pl->w);
}

void orc_ntt_inverse(int N, const uint64_t *in, uint64_t *out) {
    const ntt_plan *pl = plan_for(N);
    memcpy(out, in, sizeof(uint64_t) * (size_t)N);
    cyclic_ntt(out, N, pl->winv);
    for (int j = 0; j < N; ++j) out[j] = mont(out[j], pl->untwist[j]);
}

uint64_t orc_prime(void) { return ORC_P; }
uint64_t orc_psi(int N) { return plan_for(N)->psi; }

/* Residue of a signed integer, and the centred lift back from (-P/2, P/2). */
static uint64_t from_i64(int64_t x) { return x >= 0 ? (uint64_t)x % ORC_P : ORC_P - ((uint64_t)(-x) % ORC_P); }
static int64_t centred(uint64_t r) { return r > ORC_P / 2 ? -(int64_t)(ORC_P - r) : (int64_t)r; }

/* ------------------------------------------------------------------------ */
/* Negacyclic products in Z[X]/(X^N + 1), results reduced modulo 2^32.      */
/* ------------------------------------------------------------------------ */
static int g_schoolbook = 0; /* 1: every product by the schoolbook sum */
void orc_set_schoolbook(int on) { g_schoolbook = on; }

/* Definition: c_k = sum_{i+j=k} d_i t_j - sum_{i+j=k+N} d_i t_j  (mod 2^32). */
void orc_negamul_schoolbook(int N, const int32_t *d, const uint32_t *t, uint32_t *out) {
    for (int k = 0; k < N; ++k) {
        uint32_t acc = 0;
        for (int i = 0; i <= k; ++i) acc += (uint32_t)d[i] * t[k - i];
        for (int i = k + 1; i < N; ++i) acc -= (uint32_t)d[i] * t[k + N - i];
        out[k] = acc;
    }
}

/* Same product through the transform, given t already transformed (Montgomery
 * form).  Exact because |c_k| <= N * 2^31 * 2^32 < P/2 for |d_i| <= 2^31 and
 * t_j < 2^32 taken as non-negative integers... in practice |d_i| <= 64. */
static void negamul_ntt_pre(int N, const int32_t *d, const uint64_t *t_hat_mont, uint32_t *out) {
    uint64_t a[ORC_N], da[ORC_N], prod[ORC_N], c[ORC_N];
    for (int j = 0; j < N; ++j) a[j] = from_i64(d[j]);
    orc_ntt_forward(N, a, da);
    for (int k = 0; k < N; ++k) prod[k] = mont(da[k], t_hat_mont[k]);
    orc_ntt_inverse(N, prod, c);
    for (int k = 0; k < N; ++k) out[k] = (uint32_t)(uint64_t)centred(c[k]);
}

static void transform_torus_poly(int N, const uint32_t *t, uint64_t *t_hat_mont) {
    uint64_t a[ORC_N], ta[ORC_N];
    for (int j = 0; j < N; ++j) a[j] = t[j];
    orc_ntt_forward(N, a, ta);
    for (int k = 0; k < N; ++k) t_hat_mont[k] = to_mont(ta[k]);
}

void orc_negamul_ntt(int N, const int32_t *d, const uint32_t *t, uint32_t *out) {
    uint64_t th[ORC_N];
    transform_torus_poly(N, t, th);
    negamul_ntt_pre(N, d, th, out);
}

/* X^k * p in Z[X]/(X^N + 1), k in [0, 2N): a signed rotation. */
void orc_mul_by_xk(int N, const uint32_t *p, int k, uint32_t *out) {
    for (int j = 0; j < N; ++j) {
        int e = (j + k) % (2 * N);
        if (e < N) out[e] = p[j];
        else out[e - N] = (uint32_t)0 - p[j];
    }
}

/* ------------------------------------------------------------------------ */
/* Scalar conventions.                                                      */
/* ------------------------------------------------------------------------ */

/* Modulus switch to Z_2N with round-half-up: floor((x + 2^20 mod 2^32) / 2^21). */
uint32_t orc_modswitch(uint32_t x) { return (uint32_t)(x + (1u << 20)) >> 21; }

/* Gadget decomposition, base 2^7, 3 levels.  First round x to its top 21 bits,
 * u = floor((x + 2^10 mod 2^32) / 2^11); then write u (mod 2^21) in balanced
 * base 128 with digits in [-64, 63], least significant digit first, carrying
 * upward.  d[0] is the most significant digit (torus weight 2^25), d[2] the
 * least (weight 2^11).  The representation is unique. */
void orc_decompose(uint32_t x, int32_t d[3]) {
    uint32_t u = (uint32_t)(x + (1u << 10)) >> 11;
    int carry = 0;
    for (int j = ORC_ELL - 1; j >= 0; --j) {
        int v = (int)(u & 127u) + carry;
        u >>= 7;
        if (v >= 64) { v -= 128; carry = 1; } else carry = 0;
        d[j] = v;
    }
}

/* Key-switching digits: u = x + 2^15 (mod 2^32), digit j = bits [30-2j, 32-2j) of u. */
void orc_ks_digits(uint32_t x, uint32_t dig[8]) {
    uint32_t u = x + (1u << 15);
    for (int j = 0; j < ORC_KS_T; ++j) dig[j] = (u >> (32 - ORC_KS_BASEBIT * (j + 1))) & (ORC_KS_BASE - 1);
}

/* ------------------------------------------------------------------------ */
/* LWE / TRLWE encryption (client side; the randomness is passed in).       */
/* ------------------------------------------------------------------------ */

/* b = <a, s> + mu + e (mod 2^32); ct = (a[0..n-1], b). */
void orc_lwe_encrypt(int n, const uint32_t *s, const uint32_t *mask, int32_t noise, uint32_t mu, uint32_t *ct) {
    uint32_t b = 0;
    for (int i = 0; i < n; ++i) { ct[i] = mask[i]; b += mask[i] * s[i]; }
    ct[n] = b + mu + (uint32_t)noise;
}

/* phase = b - <a, s> (mod 2^32). */
uint32_t orc_lwe_phase(int n, const uint32_t *s, const uint32_t *ct) {
    uint32_t p = ct[n];
    for (int i = 0; i < n; ++i) p -= ct[i] * s[i];
    return p;
}

/* Nearest of {-1/8, +1/8}: bit 1 iff the phase, as a signed word, is >= 0. */
int orc_lwe_decrypt(int n, const uint32_t *s, const uint32_t *ct) {
    return (int32_t)orc_lwe_phase(n, s, ct) >= 0 ? 1 : 0;
}

/* TRLWE encryption of zero: (a, a*S + e), negacyclic product. */
static void trlwe_enc_zero(const uint32_t *S, const uint32_t *mask, const int32_t *noise, uint32_t out[2][ORC_N]) {
    int32_t Sd[ORC_N];
    uint32_t prod[ORC_N];
    for (int j = 0; j < ORC_N; ++j) Sd[j] = (int32_t)S[j];
    if (g_schoolbook) orc_negamul_schoolbook(ORC_N, Sd, mask, prod);
    else orc_negamul_ntt(ORC_N, Sd, mask, prod);
    for (int j = 0; j < ORC_N; ++j) {
        out[0][j] = mask[j];
        out[1][j] = prod[j] + (uint32_t)noise[j];
    }
}

/* Bootstrapping key: BK_i = TRGSW(s_i).  Row r = c*3 + j (c = 0 mask part,
 * c = 1 body part; j = level) is a fresh TRLWE encryption of zero to which
 * s_i * 2^(32 - 7(j+1)) is added on the constant coefficient of component c.
 * Layout bk[i][r][c'][k], u32 [630][6][2][1024].
 * mask, noise: [630][6][1024]. */
void orc_keygen_bk(const uint32_t *s, const uint32_t *S, const uint32_t *mask, const int32_t *noise, uint32_t *bk) {
    for (int i = 0; i < ORC_n; ++i)
        for (int r = 0; r < 2 * ORC_ELL; ++r) {
            uint32_t row[2][ORC_N];
            size_t off = ((size_t)i * 2 * ORC_ELL + r) * ORC_N;
            trlwe_enc_zero(S, mask + off, noise + off, row);
            int c = r / ORC_ELL, j = r % ORC_ELL;
            row[c][0] += s[i] << (32 - ORC_BGBIT * (j + 1));
            memcpy(bk + ((size_t)i * 2 * ORC_ELL + r) * 2 * ORC_N, row, sizeof(row));
        }
}

/* Key switching key: ksk[i][j][v] = LWE_s(v * S_i * 2^(32 - 2(j+1))) for v = 1..3,
 * and the all-zero word vector for v = 0.  Layout u32 [1024][8][4][631].
 * mask: [1024][8][3][630], noise: [1024][8][3]. */
void orc_keygen_ksk(const uint32_t *s, const uint32_t *S, const uint32_t *mask, const int32_t *noise, uint32_t *ksk) {
    for (int i = 0; i < ORC_N; ++i)
        for (int j = 0; j < ORC_KS_T; ++j)
            for (int v = 0; v < ORC_KS_BASE; ++v) {
                uint32_t *row = ksk + (((size_t)i * ORC_KS_T + j) * ORC_KS_BASE + v) * (ORC_n + 1);
                if (v == 0) { memset(row, 0, sizeof(uint32_t) * (ORC_n + 1)); continue; }
                size_t m = ((size_t)i * ORC_KS_T + j) * (ORC_KS_BASE - 1) + (v - 1);
                uint32_t mu = (uint32_t)v * S[i] << (32 - ORC_KS_BASEBIT * (j + 1));
                orc_lwe_encrypt(ORC_n, s, mask + m * ORC_n, noise[m], mu, row);
            }
}

/* ------------------------------------------------------------------------ */
/* Evaluation keys as the oracle holds them.                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint32_t *bk;          /* [630][6][2][1024] coefficient domain */
    uint64_t *bk_hat;      /* same, transformed, Montgomery form */
    uint32_t *ksk;         /* [1024][8][4][631] */
} orc_keys;

orc_keys *orc_keys_load(const uint32_t *bk, const uint32_t *ksk) {
    orc_init();
    size_t nbk = (size_t)ORC_n * 2 * ORC_ELL * 2 * ORC_N;
    size_t nks = (size_t)ORC_N * ORC_KS_T * ORC_KS_BASE * (ORC_n + 1);
    orc_keys *k = (orc_keys *)calloc(1, sizeof(orc_keys));
    if (!k) return NULL;
    k->bk = (uint32_t *)malloc(nbk * sizeof(uint32_t));
    k->bk_hat = (uint64_t *)malloc(nbk * sizeof(uint64_t));
    k->ksk = (uint32_t *)malloc(nks * sizeof(uint32_t));
    if (!k->bk || !k->bk_hat || !k->ksk) { free(k->bk); free(k->bk_hat); free(k->ksk); free(k); return NULL; }
    memcpy(k->bk, bk, nbk * sizeof(uint32_t));
    memcpy(k->ksk, ksk, nks * sizeof(uint32_t));
    for (size_t p = 0; p < nbk / ORC_N; ++p) transform_torus_poly(ORC_N, bk + p * ORC_N, k->bk_hat + p * ORC_N);
    return k;
}

void orc_keys_free(orc_keys *k) {
    if (!k) return;
    free(k->bk); free(k->bk_hat); free(k->ksk); free(k);
}

/* One polynomial product digit-poly x BK row component, by the selected route. */
static void bk_product(const orc_keys *K, int i, int r, int c, const int32_t *d, uint32_t *out) {
    size_t off = (((size_t)i * 2 * ORC_ELL + r) * 2 + c) * ORC_N;
    if (g_schoolbook) orc_negamul_schoolbook(ORC_N, d, K->bk + off, out);
    else negamul_ntt_pre(ORC_N, d, K->bk_hat + off, out);
}

/* External product BK_i x (A, B): sum_j dec_j(A) * BK_i[j] + sum_j dec_j(B) * BK_i[3 + j],
 * each product taken on its own and added modulo 2^32.  Adds the result to out. */
static void external_product_add(const orc_keys *K, int i, uint32_t D[2][ORC_N], uint32_t out[2][ORC_N]) {
    int32_t dig[2 * ORC_ELL][ORC_N];
    for (int c = 0; c < 2; ++c)
        for (int k = 0; k < ORC_N; ++k) {
            int32_t d3[ORC_ELL];
            orc_decompose(D[c][k], d3);
            for (int j = 0; j < ORC_ELL; ++j) dig[c * ORC_ELL + j][k] = d3[j];
        }
    uint32_t prod[ORC_N];
    for (int r = 0; r < 2 * ORC_ELL; ++r)
        for (int c = 0; c < 2; ++c) {
            bk_product(K, i, r, c, dig[r], prod);
            for (int k = 0; k < ORC_N; ++k) out[c][k] += prod[k];
        }
}

/* BlindRotate: acc = (0, X^(-b~) v) with v = mu (1 + X + ... + X^(N-1));
 * then for i = 0..629 with a~_i != 0: acc += BK_i x (X^(a~_i) acc - acc).
 * (Skipping a~_i = 0 changes nothing: the difference is then zero.)
 * in: LWE_n ciphertext u32[631]; out: TRLWE u32[2][1024]. */
void orc_blind_rotate(const orc_keys *K, const uint32_t *in, uint32_t mu, uint32_t *out) {
    uint32_t (*acc)[ORC_N] = (uint32_t (*)[ORC_N])out;
    uint32_t v[ORC_N];
    for (int j = 0; j < ORC_N; ++j) v[j] = mu;
    uint32_t bbar = orc_modswitch(in[ORC_n]);
    memset(acc[0], 0, sizeof(acc[0]));
    orc_mul_by_xk(ORC_N, v, (int)((2 * ORC_N - bbar) % (2 * ORC_N)), acc[1]);
    for (int i = 0; i < ORC_n; ++i) {
        uint32_t abar = orc_modswitch(in[i]);
        if (abar == 0) continue;
        uint32_t D[2][ORC_N], rot[ORC_N];
        for (int c = 0; c < 2; ++c) {
            orc_mul_by_xk(ORC_N, acc[c], (int)abar, rot);
            for (int k = 0; k < ORC_N; ++k) D[c][k] = rot[k] - acc[c][k];
        }
        external_product_add(K, i, D, acc);
    }
}

/* SampleExtract of coefficient 0: a'_0 = A_0, a'_j = -A_(N-j), b' = B_0.  out u32[1025]. */
void orc_sample_extract(const uint32_t *trlwe, uint32_t *out) {
    const uint32_t *A = trlwe, *B = trlwe + ORC_N;
    out[0] = A[0];
    for (int j = 1; j < ORC_N; ++j) out[j] = (uint32_t)0 - A[ORC_N - j];
    out[ORC_N] = B[0];
}

/* KeySwitch LWE_N -> LWE_n: start from (0, b'); for every i < 1024 and level
 * j < 8 with digit d != 0, subtract ksk[i][j][d].  in u32[1025], out u32[631]. */
void orc_keyswitch(const orc_keys *K, const uint32_t *in, uint32_t *out) {
    memset(out, 0, sizeof(uint32_t) * ORC_n);
    out[ORC_n] = in[ORC_N];
    for (int i = 0; i < ORC_N; ++i) {
        uint32_t dig[ORC_KS_T];
        orc_ks_digits(in[i], dig);
        for (int j = 0; j < ORC_KS_T; ++j) {
            if (!dig[j]) continue;
            const uint32_t *row = K->ksk + (((size_t)i * ORC_KS_T + j) * ORC_KS_BASE + dig[j]) * (ORC_n + 1);
            for (int w = 0; w <= ORC_n; ++w) out[w] -= row[w];
        }
    }
}

/* Bootstrap with output message mu: BlindRotate, SampleExtract (before KS). */
void orc_bootstrap_wo_ks(const orc_keys *K, const uint32_t *in, uint32_t mu, uint32_t *out_N) {
    uint32_t acc[2 * ORC_N];
    orc_blind_rotate(K, in, mu, acc);
    orc_sample_extract(acc, out_N);
}

void orc_bootstrap(const orc_keys *K, const uint32_t *in, uint32_t mu, uint32_t *out) {
    uint32_t ext[ORC_N + 1];
    orc_bootstrap_wo_ks(K, in, mu, ext);
    orc_keyswitch(K, ext, out);
}

/* ------------------------------------------------------------------------ */
/* Gates (Section 2.2: gate = Bootstrap of a linear pre-combination).       */
/* ------------------------------------------------------------------------ */
enum { ORC_AND = 0, ORC_OR = 1, ORC_NAND = 2, ORC_XOR = 3, ORC_XNOR = 4, ORC_NOT = 5, ORC_MUX = 6 };

/* t = (0, cst) + ca * a + cb * b on all 631 words. */
static void lin2(const uint32_t *a, int ca, const uint32_t *b, int cb, uint32_t cst, uint32_t *t) {
    for (int w = 0; w <= ORC_n; ++w) t[w] = (uint32_t)ca * a[w] + (uint32_t)cb * b[w];
    t[ORC_n] += cst;
}

/* op in {AND, OR, NAND, XOR, XNOR, NOT, MUX}; MUX(a = select, b = if 1, c = if 0). */
int orc_gate(const orc_keys *K, int op, const uint32_t *a, const uint32_t *b, const uint32_t *c, uint32_t *out) {
    const uint32_t mu = ORC_MU;
    uint32_t t[ORC_n + 1];
    switch (op) {
    case ORC_AND:  lin2(a, 1, b, 1, (uint32_t)0 - mu, t); break;
    case ORC_OR:   lin2(a, 1, b, 1, mu, t); break;
    case ORC_NAND: lin2(a, -1, b, -1, mu, t); break;
    case ORC_XOR:  lin2(a, 2, b, 2, 2 * mu, t); break;
    case ORC_XNOR: lin2(a, -2, b, -2, (uint32_t)0 - 2 * mu, t); break;
    case ORC_NOT:
        for (int w = 0; w <= ORC_n; ++w) out[w] = (uint32_t)0 - a[w];
        return 0;
    case ORC_MUX: {
        /* u1 = BR+SE of AND(sel, if1); u2 = BR+SE of AND(not sel, if0);
         * result = KS((0, mu) + u1 + u2). */
        uint32_t u1[ORC_N + 1], u2[ORC_N + 1], v[ORC_N + 1];
        lin2(a, 1, b, 1, (uint32_t)0 - mu, t);
        orc_bootstrap_wo_ks(K, t, mu, u1);
        lin2(a, -1, c, 1, (uint32_t)0 - mu, t);
        orc_bootstrap_wo_ks(K, t, mu, u2);
        for (int w = 0; w <= ORC_N; ++w) v[w] = u1[w] + u2[w];
        v[ORC_N] += mu;
        orc_keyswitch(K, v, out);
        return 0;
    }
    default:
        return -1;
    }
    orc_bootstrap(K, t, mu, out);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Array forms of the scalar conventions (for exhaustive property tests).   */
/* ------------------------------------------------------------------------ */
void orc_modswitch_arr(size_t cnt, const uint32_t *x, uint32_t *out) {
    for (size_t i = 0; i < cnt; ++i) out[i] = orc_modswitch(x[i]);
}
void orc_decompose_arr(size_t cnt, const uint32_t *x, int32_t *out /* [cnt][3] */) {
    for (size_t i = 0; i < cnt; ++i) orc_decompose(x[i], out + 3 * i);
}
void orc_ks_digits_arr(size_t cnt, const uint32_t *x, uint32_t *out /* [cnt][8] */) {
    for (size_t i = 0; i < cnt; ++i) orc_ks_digits(x[i], out + 8 * i);
}
