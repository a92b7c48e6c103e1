/*
 * A C program that uses the library through include/cleora.h alone (plus
 * the HIP runtime for device memory): embeds a small fixed graph and
 * prints the result, then checks that a bad edge list is reported.
 *
 * Graph: n = 97 nodes, edges (i, i+1 mod n) and (i, 7i+3 mod n), loops
 * skipped; d = 16, k = 3, seed 42, float32.
 * Output: "n d" on the first line, then n lines of d values, then
 * "blocked_maxdiff <x>": the largest difference between that result and the
 * same embedding computed 5 columns at a time into host memory
 * (cleora_embed_blocked); the last line is "bad_input <code> <message>".
 */
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "cleora.h"

#define CK(x)                                                                 \
    do {                                                                      \
        int rc_ = (x);                                                        \
        if (rc_ != 0) {                                                       \
            fprintf(stderr, "%s failed: %d %s\n", #x, rc_, cleora_last_error()); \
            return 1;                                                         \
        }                                                                     \
    } while (0)

#define HK(x)                                                                 \
    do {                                                                      \
        if ((x) != hipSuccess) {                                              \
            fprintf(stderr, "%s failed\n", #x);                               \
            return 1;                                                         \
        }                                                                     \
    } while (0)

int main(void)
{
    enum { N = 97, D = 16, K = 3 };
    int32_t src[2 * N], dst[2 * N];
    int64_t m = 0;
    for (int i = 0; i < N; ++i) {
        const int a = (i + 1) % N, b = (7 * i + 3) % N;
        if (a != i) { src[m] = i; dst[m] = a; ++m; }
        if (b != i) { src[m] = i; dst[m] = b; ++m; }
    }
    int32_t *d_src = NULL, *d_dst = NULL;
    float *d_out = NULL;
    HK(hipMalloc((void **)&d_src, sizeof(int32_t) * (size_t)m));
    HK(hipMalloc((void **)&d_dst, sizeof(int32_t) * (size_t)m));
    HK(hipMalloc((void **)&d_out, sizeof(float) * N * D));
    HK(hipMemcpy(d_src, src, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));
    HK(hipMemcpy(d_dst, dst, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));

    cleora_ctx *ctx = NULL;
    CK(cleora_create(&ctx, 0));
    CK(cleora_build_csr(ctx, N, m, d_src, d_dst, NULL, 0, NULL));
    CK(cleora_init(ctx, D, CLEORA_F32, 42, NULL));
    CK(cleora_propagate(ctx, K, NULL));
    CK(cleora_get_embedding(ctx, d_out, D, CLEORA_F32, NULL));
    CK(cleora_sync(ctx, NULL));
    static float out[N * D];
    HK(hipMemcpy(out, d_out, sizeof(out), hipMemcpyDeviceToHost));
    printf("%d %d\n", N, D);
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < D; ++j) printf(j ? " %.9g" : "%.9g", out[i * D + j]);
        printf("\n");
    }

    /* the column-blocked form, straight into (pageable) host memory */
    static float blk[N * D];
    CK(cleora_embed_blocked(ctx, D, 5, CLEORA_F32, 42, K, blk, D, NULL));
    double maxdiff = 0.0;
    for (int i = 0; i < N * D; ++i) {
        const double e = blk[i] > out[i] ? blk[i] - out[i] : out[i] - blk[i];
        if (e > maxdiff) maxdiff = e;
    }
    printf("blocked_maxdiff %.9g\n", maxdiff);

    /* an id outside [0, N) */
    dst[5] = N;
    HK(hipMemcpy(d_dst, dst, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice));
    const int rc = cleora_build_csr(ctx, N, m, d_src, d_dst, NULL, 0, NULL);
    printf("bad_input %d %s\n", rc, cleora_last_error());

    cleora_destroy(ctx);
    HK(hipFree(d_src));
    HK(hipFree(d_dst));
    HK(hipFree(d_out));
    return 0;
}
