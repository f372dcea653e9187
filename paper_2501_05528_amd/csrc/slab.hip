// Thin-slab Schur complement operator (Section 7.2, eq. bvp): the second black box of the
// paper's experiments.  On an n x n x l grid (h = 1, zero Dirichlet values outside) the
// 7-point matrix of -Laplace - kappa^2 is split into the frontal face z = l - 1 and the
// internal planes; S = A_ff - A_fi A_ii^{-1} A_if.  The slab's constant coefficients make
// the exact solve separable: the orthonormal sine transform D (D_ap = sqrt(2/(n+1))
// sin(pi (a+1)(p+1)/(n+1)), symmetric, D D = I) diagonalises the in-plane 5-point part, so
// for every pair of sine modes (p, q) the internal planes reduce to one tridiagonal z-line
// whose last pivot is the eigenvalue s_pq of S.  A product is therefore
//     S x = D (s o (D X D)) D,   X = x as an n x n array (plane index x + n y),
// four passes of a tiled FP64 product with D, each storing its result transposed, with
// the scale applied between the second and third.  The operator only offers products:
// the compression treats it as any black box.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <sstream>
#include <string>
#include <vector>

#include "internal.hpp"

namespace blr {

namespace {

struct SlabCtx {
    int n = 0, l = 0;
    int64_t N = 0;
    int64_t* perm = nullptr;   // device [N]: plane index of plan row
    double* D = nullptr;       // device n x n sine transform
    double* sval = nullptr;    // device n x n eigenvalues s_pq (symmetric in p, q)
    ~SlabCtx() {
        if (perm) (void)hipFree(perm);
        if (D) (void)hipFree(D);
        if (sval) (void)hipFree(sval);
    }
};

// out[perm[row] + N c] = X[row + ldx c]
__global__ __launch_bounds__(256) void k_slab_gather(const double* __restrict__ X, int64_t ldx,
                                                     const int64_t* __restrict__ perm, double* __restrict__ out,
                                                     int64_t N) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (row < N) out[perm[row] + N * c] = X[row + ldx * c];
}

// Y[row + ldy c] = in[perm[row] + N c]
__global__ __launch_bounds__(256) void k_slab_scatter(const double* __restrict__ in,
                                                      const int64_t* __restrict__ perm, double* __restrict__ Y,
                                                      int64_t ldy, int64_t N) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t c = blockIdx.y;
    if (row < N) Y[row + ldy * c] = in[perm[row] + N * c];
}

// One pass: for every column c (an n x n array in_c, column-major), T = D in_c and
// out_c = T^T (times scale(p, b) elementwise when scale is given).  Grid (p tiles of 64,
// b tiles of 64, columns); each thread owns a 4 x 4 block of T.
__global__ __launch_bounds__(256) void k_dst_pass(const double* __restrict__ in, double* __restrict__ out,
                                                  const double* __restrict__ D, const double* __restrict__ scale,
                                                  int n, int64_t N) {
    __shared__ double sD[64][17];
    __shared__ double sX[16][65];
    const int tid = threadIdx.x;
    const int tp = tid >> 4, tb = tid & 15;
    const int p0 = blockIdx.x * 64, b0 = blockIdx.y * 64;
    const double* ic = in + N * blockIdx.z;
    double* oc = out + N * blockIdx.z;
    double acc[4][4] = {};
    for (int a0 = 0; a0 < n; a0 += 16) {
        for (int idx = tid; idx < 64 * 16; idx += 256) {
            const int pp = idx & 63, aa = idx >> 6;
            const int p = p0 + pp, a = a0 + aa;
            sD[pp][aa] = (p < n && a < n) ? D[p + static_cast<int64_t>(n) * a] : 0.0;
        }
        for (int idx = tid; idx < 16 * 64; idx += 256) {
            const int aa = idx & 15, bb = idx >> 4;
            const int a = a0 + aa, b = b0 + bb;
            sX[aa][bb] = (a < n && b < n) ? ic[a + static_cast<int64_t>(n) * b] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int aa = 0; aa < 16; ++aa) {
            double dv[4], xv[4];
#pragma unroll
            for (int i = 0; i < 4; ++i) dv[i] = sD[tp * 4 + i][aa];
#pragma unroll
            for (int j = 0; j < 4; ++j) xv[j] = sX[aa][tb * 4 + j];
#pragma unroll
            for (int i = 0; i < 4; ++i)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[i][j] = fma(dv[i], xv[j], acc[i][j]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int p = p0 + tp * 4 + i;
        if (p >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int b = b0 + tb * 4 + j;
            if (b >= n) continue;
            const double v = acc[i][j] * (scale ? scale[p + static_cast<int64_t>(n) * b] : 1.0);
            oc[b + static_cast<int64_t>(n) * p] = v;
        }
    }
}

int32_t slab_apply(void* ctx, int32_t /*trans: S is symmetric*/, int64_t ncols, const double* X, int64_t ldx,
                   double* Y, int64_t ldy, void* stream) {
    const SlabCtx& S = *static_cast<const SlabCtx*>(ctx);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (ncols <= 0) return 0;
    const int64_t N = S.N;
    const int64_t cc = std::max<int64_t>(1, std::min<int64_t>({ncols, (int64_t(1) << 27) / N, 65535}));
    void* A = nullptr;
    void* B = nullptr;
    if (hipMallocAsync(&A, static_cast<size_t>(N * cc) * sizeof(double), s) != hipSuccess) return 1;
    if (hipMallocAsync(&B, static_cast<size_t>(N * cc) * sizeof(double), s) != hipSuccess) {
        (void)hipFreeAsync(A, s);
        return 1;
    }
    double* a = static_cast<double*>(A);
    double* b = static_cast<double*>(B);
    const unsigned nt = static_cast<unsigned>((S.n + 63) / 64);
    for (int64_t c0 = 0; c0 < ncols; c0 += cc) {
        const unsigned nc = static_cast<unsigned>(std::min(cc, ncols - c0));
        const dim3 gv(static_cast<unsigned>((N + 255) / 256), nc);
        const dim3 gp(nt, nt, nc);
        hipLaunchKernelGGL(k_slab_gather, gv, dim3(256), 0, s, X + c0 * ldx, ldx, S.perm, a, N);
        hipLaunchKernelGGL(k_dst_pass, gp, dim3(256), 0, s, a, b, S.D, nullptr, S.n, N);    // (D X)^T
        hipLaunchKernelGGL(k_dst_pass, gp, dim3(256), 0, s, b, a, S.D, S.sval, S.n, N);     // s o (D X D)
        hipLaunchKernelGGL(k_dst_pass, gp, dim3(256), 0, s, a, b, S.D, nullptr, S.n, N);
        hipLaunchKernelGGL(k_dst_pass, gp, dim3(256), 0, s, b, a, S.D, nullptr, S.n, N);    // D (.) D
        hipLaunchKernelGGL(k_slab_scatter, gv, dim3(256), 0, s, a, S.perm, Y + c0 * ldy, ldy, N);
    }
    const hipError_t e = hipGetLastError();
    (void)hipFreeAsync(A, s);
    (void)hipFreeAsync(B, s);
    return e == hipSuccess ? 0 : 2;
}

void slab_free(void* ctx) { delete static_cast<SlabCtx*>(ctx); }

}  // namespace

// Builds the slab operator's context (host tables uploaded to the current device).
void* slab_create(int n, int l, double kappa_h, const int64_t* perm, int64_t N, blr_apply_fn* fn,
                  void (**free_fn)(void*)) {
    if (n < 1 || l < 1) fail(BLR_ERR_INVALID_ARG, "slab: need n >= 1 and l >= 1");
    if (!(kappa_h >= 0.0) || !std::isfinite(kappa_h)) fail(BLR_ERR_INVALID_ARG, "slab: kappa h must be finite, >= 0");
    if (!perm) fail(BLR_ERR_INVALID_ARG, "slab: NULL permutation");
    if (N != static_cast<int64_t>(n) * n) fail(BLR_ERR_INVALID_ARG, "slab: N must be n^2");
    std::vector<char> seen(static_cast<size_t>(N), 0);
    for (int64_t r = 0; r < N; ++r) {
        if (perm[r] < 0 || perm[r] >= N || seen[static_cast<size_t>(perm[r])])
            fail(BLR_ERR_INVALID_ARG, "slab: perm is not a permutation of 0 .. n^2 - 1");
        seen[static_cast<size_t>(perm[r])] = 1;
    }
    const double pi = 3.14159265358979323846;
    std::vector<double> D(static_cast<size_t>(n) * n), sv(static_cast<size_t>(n) * n), mu(n);
    const double sc = std::sqrt(2.0 / (n + 1));
    for (int a = 0; a < n; ++a)
        for (int p = 0; p < n; ++p) D[a + static_cast<size_t>(n) * p] = sc * std::sin(pi * (a + 1) * (p + 1) / (n + 1));
    for (int p = 0; p < n; ++p) {
        const double t = std::sin(pi * (p + 1) / (2.0 * (n + 1)));
        mu[p] = 4.0 * t * t;
    }
    const double k2 = kappa_h * kappa_h;
    for (int p = 0; p < n; ++p)
        for (int q = 0; q < n; ++q) {
            // z-line of mode (p, q): diagonal d, off-diagonal -1; eliminate z = 0 .. l-2
            const double d = 2.0 + mu[p] + mu[q] - k2;
            double e = d;
            for (int z = 0; z + 1 < l; ++z) {
                if (!(e > 0.0)) fail(BLR_ERR_INVALID_ARG, "slab: the internal block is not positive definite");
                e = d - 1.0 / e;
            }
            sv[p + static_cast<size_t>(n) * q] = e;
        }
    auto ctx = std::make_unique<SlabCtx>();
    ctx->n = n;
    ctx->l = l;
    ctx->N = N;
    auto up = [&](auto*& dst, const auto* src, size_t count) {
        using T = std::remove_pointer_t<std::remove_reference_t<decltype(dst)>>;
        if (hipMalloc(&dst, count * sizeof(T)) != hipSuccess) fail(BLR_ERR_OOM, "slab: device tables");
        if (hipMemcpy(dst, src, count * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
            fail(BLR_ERR_DEVICE, "slab: upload");
    };
    up(ctx->perm, perm, static_cast<size_t>(N));
    up(ctx->D, D.data(), D.size());
    up(ctx->sval, sv.data(), sv.size());
    *fn = slab_apply;
    *free_fn = slab_free;
    return ctx.release();
}

}  // namespace blr
