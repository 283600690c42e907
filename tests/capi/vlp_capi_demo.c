/* A C caller of libvlp (no Python): creates a context, loads evaluation keys
 * (uniform words; the check below does not depend on them), bootstraps and
 * switches keys on trivial ciphertexts (0, +-1/8), whose results are known in
 * closed form: every mask word is 0 after the rotation, the body is the input
 * body, so the blind rotation does nothing but select +-mu.  Also exercises
 * the error path of context creation.  Exit code 0 on success. */
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "vlp.h"

#define HIP_OK(x) do { if ((x) != hipSuccess) { printf("HIP call failed at line %d\n", __LINE__); return 1; } } while (0)

int main(void) {
    vlp_params p;
    vlp_default_params(&p);
    vlp_ctx *ctx = NULL;
    vlp_params bad = p;
    bad.N = 2048;
    if (vlp_ctx_create(&ctx, &bad, 0, NULL, 0) != VLP_EPARAM || ctx != NULL || vlp_last_error(NULL)[0] == 0) {
        printf("bad parameters were not rejected\n");
        return 1;
    }
    if (vlp_ctx_create(&ctx, &p, 0, NULL, 0) != VLP_OK) {
        printf("context: %s\n", vlp_last_error(NULL));
        return 1;
    }
    const size_t nbk = (size_t)630 * 6 * 2 * 1024, nksk = (size_t)1024 * 8 * 4 * 631;
    uint32_t *h = malloc(nksk * 4);
    uint64_t s = 12345;
    for (size_t i = 0; i < nksk; ++i) { s = s * 6364136223846793005ull + 1442695040888963407ull; h[i] = (uint32_t)(s >> 32); }
    uint32_t *d_bk, *d_ksk, *d_in, *d_mid, *d_out;
    HIP_OK(hipMalloc((void **)&d_bk, nbk * 4));
    HIP_OK(hipMalloc((void **)&d_ksk, nksk * 4));
    HIP_OK(hipMemcpy(d_bk, h, nbk * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemcpy(d_ksk, h, nksk * 4, hipMemcpyHostToDevice));
    vlp_keyset *ks = NULL;
    if (vlp_keyset_load(ctx, d_bk, d_ksk, &ks) != VLP_OK) { printf("keys: %s\n", vlp_last_error(ctx)); return 1; }
    /* Two trivial inputs: bodies +1/8 and -1/8. */
    const uint32_t mu = 1u << 29;
    uint32_t in[2][631] = {{0}}, mid[2][1025], out[2][631];
    in[0][630] = mu;
    in[1][630] = 0u - mu;
    HIP_OK(hipMalloc((void **)&d_in, sizeof in));
    HIP_OK(hipMalloc((void **)&d_mid, sizeof mid));
    HIP_OK(hipMalloc((void **)&d_out, sizeof out));
    HIP_OK(hipMemcpy(d_in, in, sizeof in, hipMemcpyHostToDevice));
    if (vlp_bootstrap(ctx, ks, d_in, d_mid, mu, 2) != VLP_OK || vlp_sync(ctx) != VLP_OK) {
        printf("bootstrap: %s\n", vlp_last_error(ctx));
        return 1;
    }
    HIP_OK(hipMemcpy(mid, d_mid, sizeof mid, hipMemcpyDeviceToHost));
    int bad_words = 0;
    for (int b = 0; b < 2; ++b) {
        for (int w = 0; w < 1024; ++w) bad_words += mid[b][w] != 0;
        bad_words += mid[b][1024] != (b == 0 ? mu : 0u - mu);
    }
    /* Key switching of (0, +-mu) keeps it: no digit of a zero mask selects a row. */
    if (vlp_keyswitch(ctx, ks, d_mid, d_out, 2) != VLP_OK || vlp_sync(ctx) != VLP_OK) {
        printf("keyswitch: %s\n", vlp_last_error(ctx));
        return 1;
    }
    HIP_OK(hipMemcpy(out, d_out, sizeof out, hipMemcpyDeviceToHost));
    for (int b = 0; b < 2; ++b) {
        for (int w = 0; w < 630; ++w) bad_words += out[b][w] != 0;
        bad_words += out[b][630] != (b == 0 ? mu : 0u - mu);
    }
    if (vlp_gate(ctx, ks, VLP_AND, d_in, d_in, d_in, d_out, 1) != VLP_EINVAL) {  /* c is for MUX only */
        printf("argument error not reported\n");
        return 1;
    }
    vlp_keyset_destroy(ks);
    if (vlp_ctx_destroy(ctx) != VLP_OK) { printf("destroy failed\n"); return 1; }
    hipFree(d_bk); hipFree(d_ksk); hipFree(d_in); hipFree(d_mid); hipFree(d_out);
    free(h);
    if (bad_words) { printf("%d words differ from the closed form\n", bad_words); return 1; }
    printf("C ABI OK (%s)\n", vlp_version());
    return 0;
}
