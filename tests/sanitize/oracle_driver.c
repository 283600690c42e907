/* Exercises the C oracle under AddressSanitizer and UndefinedBehaviorSanitizer:
 * key generation, key loading, every gate on every input combination, the
 * transforms and the exact products; exits non-zero on a wrong bit. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void orc_init(void);
void orc_ntt_forward(int N, const uint64_t *in, uint64_t *out);
void orc_ntt_inverse(int N, const uint64_t *in, uint64_t *out);
void orc_negamul_schoolbook(int N, const int32_t *d, const uint32_t *t, uint32_t *out);
void orc_negamul_ntt(int N, const int32_t *d, const uint32_t *t, uint32_t *out);
void orc_lwe_encrypt(int n, const uint32_t *s, const uint32_t *mask, int32_t noise, uint32_t mu, uint32_t *ct);
int orc_lwe_decrypt(int n, const uint32_t *s, const uint32_t *ct);
void orc_keygen_bk(const uint32_t *s, const uint32_t *S, const uint32_t *mask, const int32_t *noise, uint32_t *bk);
void orc_keygen_ksk(const uint32_t *s, const uint32_t *S, const uint32_t *mask, const int32_t *noise, uint32_t *ksk);
void *orc_keys_load(const uint32_t *bk, const uint32_t *ksk);
void orc_keys_free(void *k);
int orc_gate(const void *K, int op, const uint32_t *a, const uint32_t *b, const uint32_t *c, uint32_t *out);

enum { n = 630, N = 1024, ELL = 3, KT = 8 };
static uint64_t st = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(void) { /* xorshift64* */
    st ^= st >> 12; st ^= st << 25; st ^= st >> 27;
    return (uint32_t)((st * 0x2545F4914F6CDD1Dull) >> 32);
}
static int32_t small_noise(int bits) { return (int32_t)(rnd() % (1u << bits)) - (1 << (bits - 1)); }

int main(void) {
    orc_init();
    int bad = 0;
    /* Transforms: inverse(forward(x)) = N x; NTT product = schoolbook product. */
    {
        uint64_t a[N], f[N], b[N];
        for (int i = 0; i < N; ++i) a[i] = rnd() % 1000003u;
        orc_ntt_forward(N, a, f);
        orc_ntt_inverse(N, f, b);
        for (int i = 0; i < N; ++i) bad |= b[i] != a[i];
        int32_t d[64];
        uint32_t t[64], p1[64], p2[64];
        for (int i = 0; i < 64; ++i) { d[i] = (int32_t)(rnd() % 128) - 64; t[i] = rnd(); }
        orc_negamul_schoolbook(64, d, t, p1);
        orc_negamul_ntt(64, d, t, p2);
        for (int i = 0; i < 64; ++i) bad |= p1[i] != p2[i];
        if (bad) { printf("transform check failed\n"); return 1; }
    }
    uint32_t *s = malloc(n * 4), *S = malloc(N * 4);
    for (int i = 0; i < n; ++i) s[i] = rnd() & 1;
    for (int i = 0; i < N; ++i) S[i] = rnd() & 1;
    size_t nbm = (size_t)n * 2 * ELL * N, nks = (size_t)N * KT * 3;
    uint32_t *bmask = malloc(nbm * 4), *kmask = malloc(nks * n * 4);
    int32_t *bnoise = malloc(nbm * 4), *knoise = malloc(nks * 4);
    for (size_t i = 0; i < nbm; ++i) { bmask[i] = rnd(); bnoise[i] = small_noise(8); }
    for (size_t i = 0; i < nks * n; ++i) kmask[i] = rnd();
    for (size_t i = 0; i < nks; ++i) knoise[i] = small_noise(17);
    uint32_t *bk = malloc(nbm * 2 * 4), *ksk = malloc((size_t)N * KT * 4 * (n + 1) * 4);
    orc_keygen_bk(s, S, bmask, bnoise, bk);
    orc_keygen_ksk(s, S, kmask, knoise, ksk);
    void *K = orc_keys_load(bk, ksk);
    if (!K) { printf("key load failed\n"); return 1; }
    /* Every gate on every input pattern, fresh encryptions. */
    const uint32_t mu = 1u << 29;
    for (int op = 0; op < 7; ++op)
        for (int pat = 0; pat < 8; ++pat) {
            if (op != 6 && pat >= 4) continue;
            int x = pat & 1, y = (pat >> 1) & 1, z = (pat >> 2) & 1, want;
            uint32_t ca[n + 1], cb[n + 1], cc[n + 1], out[n + 1], m[n];
            for (int i = 0; i < n; ++i) m[i] = rnd();
            orc_lwe_encrypt(n, s, m, small_noise(17), x ? mu : 0u - mu, ca);
            for (int i = 0; i < n; ++i) m[i] = rnd();
            orc_lwe_encrypt(n, s, m, small_noise(17), y ? mu : 0u - mu, cb);
            for (int i = 0; i < n; ++i) m[i] = rnd();
            orc_lwe_encrypt(n, s, m, small_noise(17), z ? mu : 0u - mu, cc);
            switch (op) {
            case 0: want = x & y; break;
            case 1: want = x | y; break;
            case 2: want = !(x & y); break;
            case 3: want = x ^ y; break;
            case 4: want = !(x ^ y); break;
            case 5: want = !x; break;
            default: want = x ? y : z; break;
            }
            if (orc_gate(K, op, ca, cb, op == 6 ? cc : NULL, out) != 0 || orc_lwe_decrypt(n, s, out) != want) {
                printf("gate %d pattern %d wrong\n", op, pat);
                bad = 1;
            }
        }
    orc_keys_free(K);
    free(s); free(S); free(bmask); free(kmask); free(bnoise); free(knoise); free(bk); free(ksk);
    if (bad) return 1;
    printf("oracle OK\n");
    return 0;
}
