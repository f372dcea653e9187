// Kernels for operators given only by products with A and A* (the paper's
// black-box setting): the library forms the test matrices of each step
// explicitly, the caller's apply callback multiplies them, and these kernels
// turn the products into Atil and B (Table 1, reconstruct_tag).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "internal.hpp"
#include "kernels.hpp"

namespace blr {
namespace {

void check_launch_bb(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BLR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Omega(row, s*r + c) = T(box(row), s) G(row, c)  (eq. extend_test_mat), N x ell r.
__global__ __launch_bounds__(256) void k_expand_tagged(const double* __restrict__ G, int64_t n, int r,
                                                       int ell, const double* __restrict__ T,
                                                       const int32_t* __restrict__ rb,
                                                       double* __restrict__ Om) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t total = n * static_cast<int64_t>(ell) * r;
    if (idx >= total) return;
    const int64_t col = idx / n;
    const int64_t row = idx - col * n;
    const int s = static_cast<int>(col / r), c = static_cast<int>(col - static_cast<int64_t>(s) * r);
    Om[idx] = T[static_cast<int64_t>(rb[row]) * ell + s] * G[row + static_cast<int64_t>(c) * n];
}

// The same tagged test matrix with w columns per tag column, rounded to FP32 (the
// operand of a caller's low-precision products).
__global__ __launch_bounds__(256) void k_expand_tagged_f32(const double* __restrict__ G, int64_t n, int w,
                                                           int ell, const double* __restrict__ T,
                                                           const int32_t* __restrict__ rb,
                                                           float* __restrict__ Om) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t total = n * static_cast<int64_t>(ell) * w;
    if (idx >= total) return;
    const int64_t col = idx / n;
    const int64_t row = idx - col * n;
    const int s = static_cast<int>(col / w), c = static_cast<int>(col - static_cast<int64_t>(s) * w);
    Om[idx] = static_cast<float>(T[static_cast<int64_t>(rb[row]) * ell + s] * G[row + static_cast<int64_t>(c) * n]);
}

__global__ __launch_bounds__(256) void k_to_f32(const double* __restrict__ x, int64_t n, float* __restrict__ y) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx < n) y[idx] = static_cast<float>(x[idx]);
}

__global__ __launch_bounds__(256) void k_fill0(double* __restrict__ x, int64_t n) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx < n) x[idx] = 0.0;
}

// X(:, q) = e_{c0 + q} for q < w (n x w, leading dimension n): unit columns for the
// products that give a black box's entries.
__global__ __launch_bounds__(256) void k_unit_cols(double* __restrict__ X, int64_t n, int64_t c0, int64_t w) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= n * w) return;
    const int64_t q = idx / n, row = idx - q * n;
    X[idx] = row == c0 + q ? 1.0 : 0.0;
}

// S(row, c) += sum over boxes l in [j0, j1) that are far from box(row), in ascending order,
// of W(row, (l - j0) w + c): the far-field part of the products of A with a chunk of
// block-diagonal test columns (w columns per box).
__global__ __launch_bounds__(256) void k_far_gather(const double* __restrict__ W, int64_t n, int w,
                                                    const int32_t* __restrict__ rb,
                                                    const uint8_t* __restrict__ nearm, int nbox, int j0, int j1,
                                                    double* __restrict__ S) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= n * w) return;
    const int64_t c = idx / n;
    const int64_t row = idx - c * n;
    const int64_t i = rb[row];
    double acc = S[idx];
    for (int l = j0; l < j1; ++l)
        if (!nearm[i * nbox + l]) acc += W[row + (static_cast<int64_t>(l - j0) * w + c) * n];
    S[idx] = acc;
}

// X(:, (j - j0) w + t) = S(:, t) on the rows of box j, zero elsewhere, for boxes
// j0 <= j < j1 (a column chunk of blkdiag(S_1, ..., S_b) with w columns per box).
__global__ __launch_bounds__(256) void k_embed_blockdiag(const double* __restrict__ S, int64_t n, int w,
                                                         const int32_t* __restrict__ rb, int j0, int j1,
                                                         double* __restrict__ X) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t ncols = static_cast<int64_t>(j1 - j0) * w;
    if (idx >= n * ncols) return;
    const int64_t col = idx / n;
    const int64_t row = idx - col * n;
    const int j = j0 + static_cast<int>(col / w), t = static_cast<int>(col % w);
    X[idx] = rb[row] == j ? S[row + static_cast<int64_t>(t) * n] : 0.0;
}

// Om(row, (i - i0) r + c) = G(row, c) unless box(row) is a neighbour of box i, for
// boxes i0 <= i < i1: a column chunk of the masked test matrices of Alg. 3.
__global__ __launch_bounds__(256) void k_expand_masked(const double* __restrict__ G, int64_t n, int r,
                                                       const int32_t* __restrict__ rb,
                                                       const uint8_t* __restrict__ nearm, int nbox, int i0,
                                                       int i1, double* __restrict__ Om) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    const int64_t ncols = static_cast<int64_t>(i1 - i0) * r;
    if (idx >= n * ncols) return;
    const int64_t col = idx / n;
    const int64_t row = idx - col * n;
    const int i = i0 + static_cast<int>(col / r), c = static_cast<int>(col % r);
    Om[idx] = nearm[static_cast<int64_t>(i) * nbox + rb[row]] ? 0.0 : G[row + static_cast<int64_t>(c) * n];
}

// S(row, c) = Yc(row, (box(row) - i0) r + c) for the rows of boxes i0 <= i < i1: each
// box keeps its own rows of the product with its own masked test matrix (Alg. 3).
__global__ __launch_bounds__(256) void k_take_box_rows(const double* __restrict__ Yc, int64_t n, int r,
                                                       const int32_t* __restrict__ rb, int64_t row0,
                                                       int64_t nrows, int i0, double* __restrict__ S) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= nrows * r) return;
    const int64_t c = idx / nrows;
    const int64_t row = row0 + (idx - c * nrows);
    const int64_t q = rb[row] - i0;
    S[row + c * n] = Yc[row + (q * r + c) * n];
}

// S(row, c) = sum_t Y(row, t) P_box(row)(t, c): each box's rows of the sketch times its
// own null vectors (Alg. 1), Y N x s, P b x (s x r) column-major blocks.
__global__ __launch_bounds__(256) void k_bn_project(const double* __restrict__ Y, int64_t n, int64_t s, int r,
                                                    const int32_t* __restrict__ rb,
                                                    const double* __restrict__ Pall, double* __restrict__ S) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= n * r) return;
    const int64_t c = idx / n;
    const int64_t row = idx - c * n;
    const double* P = Pall + static_cast<int64_t>(rb[row]) * s * r + c * s;
    double acc = 0.0;
    for (int64_t t = 0; t < s; ++t) acc = fma(Y[row + t * n], P[t], acc);
    S[row + c * n] = acc;
}

__device__ inline double bb_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Null vectors of Alg. 1 for one box per workgroup: M = Omega^(i)* (s x nrows, the rows of
// the box's neighbours in ascending box order, built in the workspace), its Householder QR
// (reflector sign that avoids cancellation, as LAPACK's), then P^(i) = the r columns of the
// full orthogonal factor after its first nrows columns, formed by applying the reflectors in
// reverse to unit vectors.  The reflector of column j is kept in place (rows >= j).
// flag[0] is set to 1 if a neighbour block is numerically rank deficient.
__global__ __launch_bounds__(256) void k_bn_null(const double* __restrict__ Om, int64_t n, int64_t s, int r,
                                                 const int64_t* __restrict__ box_ptr,
                                                 const int32_t* __restrict__ near_ptr,
                                                 const int32_t* __restrict__ near_idx, int64_t ws_stride,
                                                 double* __restrict__ work, double* __restrict__ Pall,
                                                 double* __restrict__ flag) {
    extern __shared__ double xs[];        // the current reflector, s doubles
    __shared__ double vvs[2048];
    __shared__ double hs[2];
    constexpr int CB = 8;                 // columns a wave updates together (independent loads)
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int box = blockIdx.x;
    double* M = work + static_cast<int64_t>(box) * ws_stride;
    // build M: column q = row q of Omega^(i)
    int64_t nrows = 0;
    for (int q = near_ptr[box]; q < near_ptr[box + 1]; ++q) {
        const int j = near_idx[q];
        const int64_t r0 = box_ptr[j], mj = box_ptr[j + 1] - r0;
        for (int64_t e = tid; e < mj * s; e += 256) {
            const int64_t u = e / s, t = e - u * s;
            M[t + (nrows + u) * s] = Om[r0 + u + t * n];
        }
        nrows += mj;
    }
    __syncthreads();
    const int nc = static_cast<int>(nrows);
    double rmax = 0.0;
    for (int j = 0; j < nc; ++j) {
        double* x = M + static_cast<int64_t>(j) * s;
        if (wave == 0) {
            double s2 = 0.0;
            for (int64_t a = j + lane; a < s; a += 64) s2 = fma(x[a], x[a], s2);
            s2 = bb_wave_sum(s2);
            if (lane == 0) {
                const double nrm = sqrt(s2);
                rmax = fmax(rmax, nrm);
                const double x0 = x[j];
                const double alpha = x0 >= 0.0 ? -nrm : nrm;
                if (!(nrm > 1e-12 * rmax)) flag[0] = 1.0;
                x[j] = x0 - alpha;
                hs[0] = s2 - x0 * x0 + (x0 - alpha) * (x0 - alpha);
            }
        }
        __syncthreads();
        const double vv = hs[0];
        if (tid == 0) vvs[j] = vv;
        for (int64_t a = j + tid; a < s; a += 256) xs[a] = x[a];
        __syncthreads();
        for (int c0 = j + 1 + wave * CB; c0 < nc; c0 += 4 * CB) {
            const int cn = min(CB, nc - c0);
            double* y = M + static_cast<int64_t>(c0) * s;
            double d[CB];
#pragma unroll
            for (int u = 0; u < CB; ++u) d[u] = 0.0;
            for (int64_t a = j + lane; a < s; a += 64) {
                const double xa = xs[a];
#pragma unroll
                for (int u = 0; u < CB; ++u)
                    if (u < cn) d[u] = fma(xa, y[a + u * s], d[u]);
            }
#pragma unroll
            for (int u = 0; u < CB; ++u) d[u] = bb_wave_sum(d[u]);
            double f[CB];
#pragma unroll
            for (int u = 0; u < CB; ++u) f[u] = vv > 0.0 ? 2.0 * d[u] / vv : 0.0;
            for (int64_t a = j + lane; a < s; a += 64) {
                const double xa = xs[a];
#pragma unroll
                for (int u = 0; u < CB; ++u)
                    if (u < cn) y[a + u * s] -= f[u] * xa;
            }
        }
        __syncthreads();
    }
    // P^(i)(:, c) = H_0 ... H_{nc-1} e_{nc + c}: each wave applies every reflector (staged in
    // LDS) to its columns together
    double* Pb = Pall + static_cast<int64_t>(box) * s * r;
    for (int idx = tid; idx < s * r; idx += 256) {
        const int64_t c = idx / s, a = idx - c * s;
        Pb[idx] = (a == nc + c) ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int j = nc - 1; j >= 0; --j) {
        const double* x = M + static_cast<int64_t>(j) * s;
        for (int64_t a = j + tid; a < s; a += 256) xs[a] = x[a];
        __syncthreads();
        const double vv = vvs[j];
        for (int c0 = wave * CB; c0 < r; c0 += 4 * CB) {
            const int cn = min(CB, r - c0);
            double* y = Pb + static_cast<int64_t>(c0) * s;
            double d[CB];
#pragma unroll
            for (int u = 0; u < CB; ++u) d[u] = 0.0;
            for (int64_t a = j + lane; a < s; a += 64) {
                const double xa = xs[a];
#pragma unroll
                for (int u = 0; u < CB; ++u)
                    if (u < cn) d[u] = fma(xa, y[a + u * s], d[u]);
            }
#pragma unroll
            for (int u = 0; u < CB; ++u) d[u] = bb_wave_sum(d[u]);
            for (int64_t a = j + lane; a < s; a += 64) {
                const double xa = xs[a];
#pragma unroll
                for (int u = 0; u < CB; ++u)
                    if (u < cn) y[a + u * s] -= (vv > 0.0 ? 2.0 * d[u] / vv : 0.0) * xa;
            }
        }
        __syncthreads();
    }
}

// X_c(box_ptr[l] + u, u) = 1 for every box l of colour c and u < m_l, zero elsewhere
// (the sparse identity probe of Table 1 step 3), N x m_max.
__global__ __launch_bounds__(256) void k_identity_probe(int64_t n, int m_max, const int32_t* __restrict__ rb,
                                                        const int64_t* __restrict__ box_ptr,
                                                        const int32_t* __restrict__ colour, int c,
                                                        double* __restrict__ X) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= n * m_max) return;
    const int64_t col = idx / n;
    const int64_t row = idx - col * n;
    const int l = rb[row];
    X[idx] = (colour[l] == c && row - box_ptr[l] == col) ? 1.0 : 0.0;
}

// Atil(i k + a, j k + t) = sum_{row in I_i} U(row, a) W(row, (j - j0) k + t) for the
// boxes j0 <= j < j1 of one chunk: U_i* (A V)(I_i, J_j) (Table 1 step 2).  One
// workgroup per (row box i, 64-column tile of the chunk); rows staged in LDS.
__global__ __launch_bounds__(256) void k_cores_from_w(const double* __restrict__ U, int64_t n, int k,
                                                      const int64_t* __restrict__ box_ptr,
                                                      const double* __restrict__ W, int64_t ncols,
                                                      int j0, double* __restrict__ Atil, int64_t ldAt) {
    constexpr int RT = 16, CT = 64;
    __shared__ double sU[RT][64];
    __shared__ double sW[RT][CT];
    const int tid = threadIdx.x;
    const int i = blockIdx.x;
    const int64_t c0 = static_cast<int64_t>(blockIdx.y) * CT;
    const int64_t ri0 = box_ptr[i];
    const int mi = static_cast<int>(box_ptr[i + 1] - ri0);
    const int cc = tid % CT;            // tile column
    const int ab = tid / CT;            // rows a = ab, ab + 4, ...
    double acc[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    for (int a0 = 0; a0 < mi; a0 += RT) {
        __syncthreads();
        for (int e = tid; e < RT * 64; e += 256) {
            const int rr = e / 64, a = e % 64;
            sU[rr][a] = (a0 + rr < mi && a < k) ? U[ri0 + a0 + rr + static_cast<int64_t>(a) * n] : 0.0;
        }
        for (int e = tid; e < RT * CT; e += 256) {
            const int rr = e / CT, q = e % CT;
            sW[rr][q] = (a0 + rr < mi && c0 + q < ncols) ? W[ri0 + a0 + rr + (c0 + q) * n] : 0.0;
        }
        __syncthreads();
#pragma unroll 1
        for (int rr = 0; rr < RT; ++rr) {
            const double w = sW[rr][cc];
#pragma unroll
            for (int q = 0; q < 16; ++q) acc[q] += sU[rr][ab + 4 * q] * w;
        }
    }
    if (c0 + cc < ncols) {
        const int64_t col = static_cast<int64_t>(j0) * k + c0 + cc;
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const int a = ab + 4 * q;
            if (a < k) Atil[static_cast<int64_t>(i) * k + a + col * ldAt] = acc[q];
        }
    }
}

// B_il(a, col) = P_c(I_i[a], col) - sum_t U_i(a, t) Q_ic(col, t) for the neighbour l of
// box i that has colour c (Table 1 step 3, with P_c = A X_c from the caller's apply and
// Q_ic = X_c^T V Atil_{i,:}^T from the near-field workspace).
__global__ __launch_bounds__(256) void k_nf_from_probe(const double* __restrict__ Pc, int64_t ldP,
                                                       int c, const int64_t* __restrict__ box_ptr,
                                                       const int32_t* __restrict__ near_idx,
                                                       const int64_t* __restrict__ b_off,
                                                       const int32_t* __restrict__ nf_pair, int ncol,
                                                       const double* __restrict__ U, int64_t ldUV, int k,
                                                       int m_max, int kp, const double* __restrict__ Qg,
                                                       double* __restrict__ Bv) {
    const int i = blockIdx.x;
    const int pair = i * ncol + c;
    const int p = nf_pair[pair];
    if (p < 0) return;
    const int l = near_idx[p];
    const int64_t ri0 = box_ptr[i];
    const int mi = static_cast<int>(box_ptr[i + 1] - ri0);
    const int ml = static_cast<int>(box_ptr[l + 1] - box_ptr[l]);
    const double* Q = Qg + static_cast<int64_t>(pair) * m_max * kp;
    double* Bout = Bv + b_off[p];
    for (int64_t e = threadIdx.x; e < static_cast<int64_t>(mi) * ml; e += 256) {
        const int col = static_cast<int>(e / mi), a = static_cast<int>(e % mi);
        double v = Pc[ri0 + a + static_cast<int64_t>(col) * ldP];
        for (int t = 0; t < k; ++t) v -= U[ri0 + a + static_cast<int64_t>(t) * ldUV] * Q[static_cast<int64_t>(col) * kp + t];
        Bout[a + static_cast<int64_t>(col) * mi] = v;
    }
}

unsigned blocks_for(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

}  // namespace

void launch_expand_tagged(const PlanData& P, const DeviceTables& t, const double* G, double* Om,
                          hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(P.ell) * P.r;
    hipLaunchKernelGGL(k_expand_tagged, dim3(blocks_for(total)), dim3(256), 0, s, G, P.n, P.r, P.ell, t.T,
                       t.row_box, Om);
    check_launch_bb("tagged test matrix");
}

void launch_expand_tagged_f32(const PlanData& P, const DeviceTables& t, const double* G, int w, float* Om,
                              hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(P.ell) * w;
    hipLaunchKernelGGL(k_expand_tagged_f32, dim3(blocks_for(total)), dim3(256), 0, s, G, P.n, w, P.ell, t.T,
                       t.row_box, Om);
    check_launch_bb("FP32 tagged test matrix");
}

void launch_expand_tagged_w(const PlanData& P, const DeviceTables& t, const double* G, int w, double* Om,
                            hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(P.ell) * w;
    hipLaunchKernelGGL(k_expand_tagged, dim3(blocks_for(total)), dim3(256), 0, s, G, P.n, w, P.ell, t.T,
                       t.row_box, Om);
    check_launch_bb("tagged test matrix");
}

void launch_to_f32(const double* x, int64_t n, float* y, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3(blocks_for(n)), dim3(256), 0, s, x, n, y);
    check_launch_bb("FP32 rounding");
}

void launch_fill0(double* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_fill0, dim3(blocks_for(n)), dim3(256), 0, s, x, n);
    check_launch_bb("fill");
}

void launch_unit_cols(double* X, int64_t n, int64_t c0, int64_t w, hipStream_t s) {
    hipLaunchKernelGGL(k_unit_cols, dim3(blocks_for(n * w)), dim3(256), 0, s, X, n, c0, w);
    check_launch_bb("unit columns");
}

void launch_far_gather(const PlanData& P, const DeviceTables& t, const double* W, int w, int j0, int j1,
                       double* S, hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(w);
    hipLaunchKernelGGL(k_far_gather, dim3(blocks_for(total)), dim3(256), 0, s, W, P.n, w, t.row_box, t.nearm,
                       P.b, j0, j1, S);
    check_launch_bb("far-field gather");
}

void launch_embed_blockdiag(const PlanData& P, const DeviceTables& t, const double* S, int w, int j0,
                            int j1, double* X, hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(j1 - j0) * w;
    hipLaunchKernelGGL(k_embed_blockdiag, dim3(blocks_for(total)), dim3(256), 0, s, S, P.n, w, t.row_box,
                       j0, j1, X);
    check_launch_bb("block-diagonal test columns");
}

void launch_expand_masked(const PlanData& P, const DeviceTables& t, const double* G, int i0, int i1,
                          double* Om, hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(i1 - i0) * P.r;
    hipLaunchKernelGGL(k_expand_masked, dim3(blocks_for(total)), dim3(256), 0, s, G, P.n, P.r, t.row_box,
                       t.nearm, P.b, i0, i1, Om);
    check_launch_bb("masked test matrices");
}

void launch_take_box_rows(const PlanData& P, const DeviceTables& t, const double* Yc, int i0, int i1,
                          double* S, hipStream_t s) {
    const int64_t row0 = P.box_ptr[i0], nrows = P.box_ptr[i1] - P.box_ptr[i0];
    const int64_t total = nrows * P.r;
    hipLaunchKernelGGL(k_take_box_rows, dim3(blocks_for(total)), dim3(256), 0, s, Yc, P.n, P.r, t.row_box,
                       row0, nrows, i0, S);
    check_launch_bb("per-box sample rows");
}

void launch_bn_project(const PlanData& P, const DeviceTables& t, const double* Y, int64_t ns,
                       const double* Pall, double* S, hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(P.r);
    hipLaunchKernelGGL(k_bn_project, dim3(blocks_for(total)), dim3(256), 0, s, Y, P.n, ns, P.r, t.row_box,
                       Pall, S);
    check_launch_bb("block-nullified samples");
}

int64_t bn_null_workspace_doubles(const PlanData& P, int64_t ns) {
    return static_cast<int64_t>(P.b) * ns * (ns - P.r);
}

void launch_bn_null(const PlanData& P, const DeviceTables& t, const double* Om, int64_t ns, double* work,
                    double* Pall, double* flag, hipStream_t s) {
    if (ns - P.r > 2048) fail(BLR_ERR_UNSUPPORTED, "block nullification supports neighbourhoods of at most 2048 rows");
    hipLaunchKernelGGL(k_bn_null, dim3(P.b), dim3(256), static_cast<size_t>(ns) * sizeof(double), s, Om, P.n, ns,
                       P.r, t.box_ptr, t.near_ptr, t.near_idx, ns * (ns - P.r), work, Pall, flag);
    check_launch_bb("block-nullification null vectors");
}

void launch_identity_probe(const PlanData& P, const DeviceTables& t, int c, double* X, hipStream_t s) {
    const int64_t total = P.n * static_cast<int64_t>(P.m_max);
    hipLaunchKernelGGL(k_identity_probe, dim3(blocks_for(total)), dim3(256), 0, s, P.n, P.m_max, t.row_box,
                       t.box_ptr, t.colour, c, X);
    check_launch_bb("identity probe");
}

void launch_cores_from_w(const PlanData& P, const DeviceTables& t, const double* U, const double* W,
                         int j0, int j1, double* Atil, hipStream_t s) {
    if (P.k > 64) fail(BLR_ERR_UNSUPPORTED, "k > 64 is not supported by the cores kernel");
    const int64_t ncols = static_cast<int64_t>(j1 - j0) * P.k;
    const dim3 grid(P.b, static_cast<unsigned>((ncols + 63) / 64));
    hipLaunchKernelGGL(k_cores_from_w, grid, dim3(256), 0, s, U, P.n, P.k, t.box_ptr, W, ncols, j0, Atil,
                       static_cast<int64_t>(P.b) * P.k);
    check_launch_bb("cores from products");
}

void launch_nf_from_probe(const PlanData& P, const DeviceTables& t, const double* Pc, int c,
                          const double* U, const double* Qwork, double* Bv, hipStream_t s) {
    const int kp = 16 * ((P.k + 15) / 16);
    hipLaunchKernelGGL(k_nf_from_probe, dim3(P.b), dim3(256), 0, s, Pc, P.n, c, t.box_ptr, t.near_idx,
                       t.b_off, t.nf_pair, P.ncol, U, P.n, P.k, P.m_max, kp, Qwork, Bv);
    check_launch_bb("near field from probes");
}

}  // namespace blr
