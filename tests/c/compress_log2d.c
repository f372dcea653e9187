/*
 * Plain C use of the library (no Python, no PyTorch): compress the 2D log|x-y| kernel
 * matrix on a 40 x 40 cell-centred grid (5 x 5 boxes of 8 x 8 points) with rank 10 and
 * oversampling 10, then apply the compressed operator and measure its error.
 * Exit status 0 when every call succeeds and the relative Frobenius error is below 1e-3.
 */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

#include "blr_tag.h"

#define CHECK(call)                                                                            \
    do {                                                                                       \
        blr_status st_ = (call);                                                               \
        if (st_ != BLR_OK) {                                                                   \
            fprintf(stderr, "%s failed: %s (%s)\n", #call, blr_status_string(st_),               \
                    blr_last_error_message());                                                 \
            return 1;                                                                          \
        }                                                                                      \
    } while (0)
#define HCHECK(call)                                                                           \
    do {                                                                                       \
        if ((call) != hipSuccess) {                                                            \
            fprintf(stderr, "%s failed\n", #call);                                             \
            return 1;                                                                          \
        }                                                                                      \
    } while (0)

/* standard normal numbers: xorshift64* and the Box-Muller transform */
static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static double uniform01(void) {
    rng_state ^= rng_state >> 12;
    rng_state ^= rng_state << 25;
    rng_state ^= rng_state >> 27;
    return ((rng_state * 0x2545F4914F6CDD1Dull) >> 11) * (1.0 / 9007199254740992.0) + 1e-300;
}
static double normal(void) {
    return sqrt(-2.0 * log(uniform01())) * cos(6.283185307179586 * uniform01());
}

int main(void) {
    enum { B = 5, Q = 8, K = 10, P = 10 };
    const int nb = B * B, n = nb * Q * Q, r = K + P;
    int64_t box_ptr[B * B + 1];
    int32_t lattice[2 * B * B];
    double* pts = (double*)malloc(sizeof(double) * 2 * n);
    for (int bi = 0; bi < nb; ++bi) {
        const int bx = bi % B, by = bi / B;
        box_ptr[bi] = (int64_t)bi * Q * Q;
        lattice[2 * bi] = bx;
        lattice[2 * bi + 1] = by;
        for (int t = 0; t < Q * Q; ++t) {  /* points inside a box, x fastest */
            const int gx = bx * Q + t % Q, gy = by * Q + t / Q;
            pts[2 * (bi * Q * Q + t)] = (gx + 0.5) / (B * Q);
            pts[2 * (bi * Q * Q + t) + 1] = (gy + 0.5) / (B * Q);
        }
    }
    box_ptr[nb] = n;

    blr_geometry geom = {2, nb, box_ptr, lattice, NULL, NULL};
    int32_t ell = 0;
    CHECK(blr_tag_columns(&geom, 3, &ell));
    double* T = (double*)malloc(sizeof(double) * nb * ell);
    for (int q = 0; q < nb * ell; ++q) T[q] = normal();
    blr_tag_params prm = {K, P, 3, 1, T};
    blr_plan* plan = NULL;
    CHECK(blr_tag_plan(&geom, &prm, &plan));

    blr_operator* op = NULL;
    CHECK(blr_op_kernel_create(BLR_KERNEL_LOG, 2, n, pts, &op));

    const size_t gbytes = sizeof(double) * (size_t)n * r;
    double* hG = (double*)malloc(2 * gbytes);
    for (size_t q = 0; q < 2 * (size_t)n * r; ++q) hG[q] = normal();
    double *G = NULL, *H = NULL, *x = NULL, *y = NULL, *ya = NULL;
    HCHECK(hipMalloc((void**)&G, gbytes));
    HCHECK(hipMalloc((void**)&H, gbytes));
    HCHECK(hipMemcpy(G, hG, gbytes, hipMemcpyHostToDevice));
    HCHECK(hipMemcpy(H, hG + (size_t)n * r, gbytes, hipMemcpyHostToDevice));

    blr_ublr* h = NULL;
    blr_report rep;
    CHECK(blr_tag_compress(plan, op, G, H, NULL, NULL, &h, &rep));

    /* y = A_uBLR x against the operator's own product, for x = normal vector */
    double* hx = (double*)malloc(sizeof(double) * n);
    for (int q = 0; q < n; ++q) hx[q] = normal();
    HCHECK(hipMalloc((void**)&x, sizeof(double) * n));
    HCHECK(hipMalloc((void**)&y, sizeof(double) * n));
    HCHECK(hipMalloc((void**)&ya, sizeof(double) * n));
    HCHECK(hipMemcpy(x, hx, sizeof(double) * n, hipMemcpyHostToDevice));
    CHECK(blr_apply(h, 0, 1, x, n, y, n, NULL));
    CHECK(blr_op_apply(op, 0, 1, x, n, ya, n, NULL));
    HCHECK(hipDeviceSynchronize());
    double* hy = (double*)malloc(sizeof(double) * 2 * n);
    HCHECK(hipMemcpy(hy, y, sizeof(double) * n, hipMemcpyDeviceToHost));
    HCHECK(hipMemcpy(hy + n, ya, sizeof(double) * n, hipMemcpyDeviceToHost));
    double num = 0.0, den = 0.0;
    for (int q = 0; q < n; ++q) {
        num += (hy[q] - hy[n + q]) * (hy[q] - hy[n + q]);
        den += hy[n + q] * hy[n + q];
    }
    double err_fro = 0.0;
    CHECK(blr_error_fro(h, op, NULL, &err_fro));
    printf("compress_log2d: N=%d boxes=%d k=%d ell=%d  %.2f ms  applies A %lld  "
           "rel fro error %.3e  rel apply error %.3e\n",
           n, nb, K, ell, rep.ms_total, (long long)rep.applies_A, err_fro, sqrt(num / den));

    blr_ublr_destroy(h);
    blr_op_destroy(op);
    blr_plan_destroy(plan);
    hipFree(G);
    hipFree(H);
    hipFree(x);
    hipFree(y);
    hipFree(ya);
    free(pts);
    free(T);
    free(hG);
    free(hx);
    free(hy);
    return (err_fro < 1e-3 && sqrt(num / den) < 1e-3) ? 0 : 2;
}
