// Truncation of a compressed uBLR to per-box ranks from a tolerance (the paper's remark
// that ranks can be chosen larger and truncated afterwards, Section 6, with the range
// finder's tolerance of Section 2.4).  Far block rows Atil(i, F_i) and, after the row
// step, far block columns Atil1(F_j, j) are reduced to k x k triangular factors by a
// streaming Householder QR held in LDS, whose one-sided Jacobi SVD gives the singular
// values and the rotation W_i (rows) or J_j (columns); the host picks the ranks and the
// remaining kernels rotate and cut U, V, Atil and fold the change of the near blocks
// into B.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "internal.hpp"
#include "kernels.hpp"

namespace blr {

namespace {

void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BLR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

__device__ inline double tr_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ inline int tr_player(int pos, int round, int n) {
    return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n - 1);
}

constexpr int kChunkRows = 128;   // rows of the far block row/column streamed per step

// One workgroup per box.  MODE 0: the far block row of box i, read as the
// (|F_i| k) x k matrix X_i^T with X_i^T((j, c), a) = Atil(i k + a, j k + c).  MODE 1: the far
// block column of box j, the (|F_j| k) x k matrix with ((i, a), c) = Atil(i k + a, j k + c).
// Either way the k x k factor R of its QR has the same right singular vectors, which are the
// left singular vectors of the far block row (MODE 0) or the right singular vectors of the
// far block column (MODE 1).  Output: W (k x k per box, column-major, columns by descending
// singular value, ties to the lower index) and sig (k per box).
template <int MODE>
__global__ __launch_bounds__(256) void k_trunc_svd(const double* __restrict__ At, int64_t ld, int nbox, int k,
                                                   const uint8_t* __restrict__ nearm, int max_sweeps,
                                                   double* __restrict__ Wout, double* __restrict__ sig) {
    extern __shared__ double smem[];
    __shared__ double hs[4];                   // alpha, v0, vv of the current reflector
    __shared__ double norms[64];
    __shared__ int order[64];
    __shared__ int cboxes[kChunkRows];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int box = blockIdx.x;
    double* R = smem;                          // k x k, column-major, upper triangular
    double* J = smem + k * k;                  // k x k rotations
    double* C = smem + 2 * k * k;              // kChunkRows x k chunk, column-major
    for (int idx = tid; idx < k * k; idx += 256) R[idx] = 0.0;
    const int per = kChunkRows / k;            // whole boxes per chunk
    int next = 0;                              // next candidate box of the far list
    __syncthreads();
    for (;;) {
        // collect up to `per` far boxes (all threads scan the same mask row)
        int nb = 0;
        while (next < nbox && nb < per) {
            if (!nearm[static_cast<int64_t>(box) * nbox + next]) {
                if (tid == 0) cboxes[nb] = next;
                ++nb;
            }
            ++next;
        }
        if (nb == 0) break;
        __syncthreads();
        const int nrows = nb * k;
        for (int idx = tid; idx < nrows * k; idx += 256) {
            const int col = idx / nrows, row = idx - col * nrows;
            const int q = row / k, w = row - q * k;
            const int64_t other = cboxes[q];
            double v;
            if (MODE == 0)   // row (other, w), column a = col
                v = At[(static_cast<int64_t>(box) * k + col) + (other * k + w) * ld];
            else             // row (other, w), column c = col
                v = At[(other * k + w) + (static_cast<int64_t>(box) * k + col) * ld];
            C[row + col * kChunkRows] = v;
        }
        __syncthreads();
        // Householder QR of [R; C]: the reflector of column j acts on row j of R and on C
        for (int j = 0; j < k; ++j) {
            const double* cj = C + j * kChunkRows;
            if (wave == 0) {
                double s2 = 0.0;
                for (int a = lane; a < nrows; a += 64) s2 = fma(cj[a], cj[a], s2);
                s2 = tr_wave_sum(s2);
                if (lane == 0) {
                    const double x0 = R[j + j * k];
                    const double tot = s2 + x0 * x0;
                    const double alpha = x0 >= 0.0 ? -sqrt(tot) : sqrt(tot);
                    const double v0 = x0 - alpha;
                    hs[0] = alpha;
                    hs[1] = v0;
                    hs[2] = s2 > 0.0 ? s2 + v0 * v0 : 0.0;     // no reflector when C(:, j) = 0
                }
            }
            __syncthreads();
            const double v0 = hs[1], vv = hs[2];
            if (vv > 0.0) {
                for (int t = j + 1 + wave; t < k; t += 4) {
                    double* ct = C + t * kChunkRows;
                    double d = 0.0;
                    for (int a = lane; a < nrows; a += 64) d = fma(cj[a], ct[a], d);
                    d = tr_wave_sum(d) + v0 * R[j + t * k];
                    const double f = 2.0 * d / vv;
                    for (int a = lane; a < nrows; a += 64) ct[a] -= f * cj[a];
                    if (lane == 0) R[j + t * k] -= f * v0;
                }
            }
            __syncthreads();
            if (tid == 0 && vv > 0.0) R[j + j * k] = hs[0];
            __syncthreads();
        }
    }
    for (int idx = tid; idx < k * k; idx += 256) {
        const int b = idx / k, a = idx - b * k;
        J[idx] = (a == b) ? 1.0 : 0.0;
    }
    __syncthreads();
    // one-sided Jacobi on the columns of R: R J = X Sigma, so R = X Sigma J^T and J holds the
    // right singular vectors of R.  Groups of 8 lanes rotate disjoint pairs (round robin).
    const double tol = sqrt(static_cast<double>(k)) * 2.220446049250313e-16;
    const int nr = k + (k & 1);
    const int grp = tid >> 3, gl = tid & 7;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        int rotated = 0;
        for (int round = 0; round < nr - 1; ++round) {
            for (int u = grp; u < nr / 2; u += 32) {
                int p = tr_player(u, round, nr), q = tr_player(nr - 1 - u, round, nr);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                if (q >= k) continue;
                double* xp = R + p * k;
                double* xq = R + q * k;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int a = gl; a < k; a += 8) {
                    const double x = xp[a], y = xq[a];
                    al = fma(x, x, al);
                    be = fma(y, y, be);
                    ga = fma(x, y, ga);
                }
#pragma unroll
                for (int o = 4; o >= 1; o >>= 1) {
                    al += __shfl_xor(al, o, 8);
                    be += __shfl_xor(be, o, 8);
                    ga += __shfl_xor(ga, o, 8);
                }
                if (ga != 0.0 && fabs(ga) > tol * sqrt(al * be)) {
                    const double zeta = (be - al) / (2.0 * ga);
                    const double t = copysign(1.0, zeta) / (fabs(zeta) + hypot(1.0, zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), sn = c * t;
                    double* jp = J + p * k;
                    double* jq = J + q * k;
                    for (int a = gl; a < k; a += 8) {
                        const double x = xp[a], y = xq[a];
                        xp[a] = c * x - sn * y;
                        xq[a] = sn * x + c * y;
                        const double u1 = jp[a], u2 = jq[a];
                        jp[a] = c * u1 - sn * u2;
                        jq[a] = sn * u1 + c * u2;
                    }
                    rotated = 1;
                }
            }
            __syncthreads();
        }
        if (!__syncthreads_or(rotated)) break;
    }
    for (int c = wave; c < k; c += 4) {
        double s2 = 0.0;
        for (int a = lane; a < k; a += 64) s2 = fma(R[c * k + a], R[c * k + a], s2);
        s2 = tr_wave_sum(s2);
        if (lane == 0) norms[c] = sqrt(s2);
    }
    __syncthreads();
    if (tid < k) {
        const double nv = norms[tid];
        int rank = 0;
        for (int c = 0; c < k; ++c) rank += (norms[c] > nv) || (norms[c] == nv && c < tid);
        order[rank] = tid;
    }
    __syncthreads();
    if (tid < k) sig[static_cast<int64_t>(box) * k + tid] = norms[order[tid]];
    double* Wb = Wout + static_cast<int64_t>(box) * k * k;
    for (int idx = tid; idx < k * k; idx += 256) {
        const int c = idx / k, a = idx - c * k;
        Wb[idx] = J[a + order[c] * k];
    }
}

// Row step: Aout(i k + a, col) = sum_s W_i(s, a) Ain(i k + s, col) for a < ku[i], 0 beyond.
// Grid (b, column tiles of 256); each thread owns one column of the block row (k contiguous
// values, whole cache lines).
__global__ __launch_bounds__(256) void k_trunc_rows(const double* __restrict__ Ain, double* __restrict__ Aout,
                                                    int64_t ld, int64_t ncol, int k,
                                                    const double* __restrict__ W,
                                                    const int32_t* __restrict__ ku) {
    __shared__ double sW[64 * 64];
    const int tid = threadIdx.x;
    const int i = blockIdx.x;
    const int kk = ku[i];
    const double* Wi = W + static_cast<int64_t>(i) * k * k;
    for (int idx = tid; idx < k * k; idx += 256) sW[idx] = Wi[idx];
    __syncthreads();
    const int64_t col = static_cast<int64_t>(blockIdx.y) * 256 + tid;
    if (col >= ncol) return;
    const double* in = Ain + static_cast<int64_t>(i) * k + col * ld;
    double* out = Aout + static_cast<int64_t>(i) * k + col * ld;
    double x[64];
#pragma unroll
    for (int s = 0; s < 64; ++s) x[s] = s < k ? in[s] : 0.0;
    for (int a = 0; a < k; ++a) {
        double acc = 0.0;
        if (a < kk) {
#pragma unroll
            for (int s = 0; s < 64; ++s)
                if (s < k) acc = fma(sW[s + a * k], x[s], acc);
        }
        out[a] = acc;
    }
}

// Column step, in place: A(row, j k + c) = sum_s A(row, j k + s) J_j(s, c) for c < kv[j],
// 0 beyond.  Grid (b, row tiles of 256); each thread owns one row of the block column.
__global__ __launch_bounds__(256) void k_trunc_cols(double* __restrict__ A, int64_t ld, int64_t nrow, int k,
                                                    const double* __restrict__ Jm,
                                                    const int32_t* __restrict__ kv) {
    __shared__ double sJ[64 * 64];
    const int tid = threadIdx.x;
    const int j = blockIdx.x;
    const int kk = kv[j];
    const double* Jj = Jm + static_cast<int64_t>(j) * k * k;
    for (int idx = tid; idx < k * k; idx += 256) sJ[idx] = Jj[idx];
    __syncthreads();
    const int64_t row = static_cast<int64_t>(blockIdx.y) * 256 + tid;
    if (row >= nrow) return;
    double* base = A + row + static_cast<int64_t>(j) * k * ld;
    double x[64];
#pragma unroll
    for (int s = 0; s < 64; ++s) x[s] = s < k ? base[s * ld] : 0.0;
    for (int c = 0; c < k; ++c) {
        double acc = 0.0;
        if (c < kk) {
#pragma unroll
            for (int s = 0; s < 64; ++s)
                if (s < k) acc = fma(x[s], sJ[s + c * k], acc);
        }
        base[c * ld] = acc;
    }
}

// Bases: Sout(row, a) = sum_s S(row, s) W_box(s, a) for a < kr[box], 0 beyond.  One
// workgroup per box.
__global__ __launch_bounds__(256) void k_trunc_basis(const double* __restrict__ S, double* __restrict__ Sout,
                                                     int64_t ldS, const int64_t* __restrict__ box_ptr, int k,
                                                     const double* __restrict__ W,
                                                     const int32_t* __restrict__ kr) {
    __shared__ double sW[64 * 64];
    const int tid = threadIdx.x;
    const int box = blockIdx.x;
    const int kk = kr[box];
    const double* Wb = W + static_cast<int64_t>(box) * k * k;
    for (int idx = tid; idx < k * k; idx += 256) sW[idx] = Wb[idx];
    __syncthreads();
    const int64_t r0 = box_ptr[box], r1 = box_ptr[box + 1];
    for (int64_t row = r0 + tid; row < r1; row += 256) {
        double x[64];
#pragma unroll
        for (int s = 0; s < 64; ++s) x[s] = s < k ? S[row + s * ldS] : 0.0;
        for (int a = 0; a < k; ++a) {
            double acc = 0.0;
            if (a < kk) {
#pragma unroll
                for (int s = 0; s < 64; ++s)
                    if (s < k) acc = fma(x[s], sW[s + a * k], acc);
            }
            Sout[row + a * ldS] = acc;
        }
    }
}

// Sum of squares of every k x k block of Atil: part[i b + j] (grid b x b).
__global__ __launch_bounds__(256) void k_block_sq(const double* __restrict__ At, int64_t ld, int k,
                                                  double* __restrict__ part) {
    __shared__ double red[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x, i = blockIdx.y;
    double s = 0.0;
    for (int idx = tid; idx < k * k; idx += 256) {
        const int c = idx / k, a = idx - c * k;
        const double v = At[(static_cast<int64_t>(i) * k + a) + (static_cast<int64_t>(j) * k + c) * ld];
        s = fma(v, v, s);
    }
    s = tr_wave_sum(s);
    if (lane == 0) red[wave] = s;
    __syncthreads();
    if (tid == 0) part[static_cast<int64_t>(i) * gridDim.x + j] = red[0] + red[1] + red[2] + red[3];
}

// Near pairs, one workgroup per pair q (i = pair_row[q], j = near_idx[q]):
// UPDATE = 0: part[q] = ||U_i Atil_ij V_j^T + B_ij||_F^2;
// UPDATE = 1: Bout_ij = B_ij + U_i D V_j^T with D = Aold_ij - W_i Anew_ij J_j^T, so that
//             U'_i Anew_ij V'_j^T + Bout_ij = U_i Aold_ij V_j^T + B_ij.
template <int UPDATE>
__global__ __launch_bounds__(256) void k_trunc_near(const int64_t* __restrict__ box_ptr,
                                                    const int32_t* __restrict__ pair_row,
                                                    const int32_t* __restrict__ near_idx,
                                                    const int64_t* __restrict__ b_off,
                                                    const double* __restrict__ U, const double* __restrict__ V,
                                                    int64_t ldUV, const double* __restrict__ Aold,
                                                    const double* __restrict__ Anew, int64_t ldA, int k,
                                                    const double* __restrict__ W, const double* __restrict__ Jm,
                                                    const double* __restrict__ Bin, double* __restrict__ Bout,
                                                    double* __restrict__ part) {
    constexpr int CH = 32;
    __shared__ double sD[64 * 64];
    __shared__ double sV[CH * 64];
    __shared__ double red[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int q = blockIdx.x;
    const int i = pair_row[q], j = near_idx[q];
    const int64_t ri0 = box_ptr[i], cj0 = box_ptr[j];
    const int mi = static_cast<int>(box_ptr[i + 1] - ri0);
    const int mj = static_cast<int>(box_ptr[j + 1] - cj0);
    auto blk = [&](const double* A, int a, int c) {
        return A[(static_cast<int64_t>(i) * k + a) + (static_cast<int64_t>(j) * k + c) * ldA];
    };
    if (UPDATE) {
        const double* Wi = W + static_cast<int64_t>(i) * k * k;
        const double* Jj = Jm + static_cast<int64_t>(j) * k * k;
        for (int idx = tid; idx < k * k; idx += 256) {      // T = W_i Anew_ij (in sD)
            const int c = idx / k, a = idx - c * k;
            double acc = 0.0;
            for (int s = 0; s < k; ++s) acc = fma(Wi[a + s * k], blk(Anew, s, c), acc);
            sD[idx] = acc;
        }
        __syncthreads();
        double d[16];                                        // D = Aold_ij - T J_j^T (k*k <= 16*256)
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int idx = tid + 256 * e;
            double acc = 0.0;
            if (idx < k * k) {
                const int c = idx / k, a = idx - c * k;
                for (int s = 0; s < k; ++s) acc = fma(sD[a + s * k], Jj[c + s * k], acc);
                acc = blk(Aold, a, c) - acc;
            }
            d[e] = acc;
        }
        __syncthreads();
#pragma unroll
        for (int e = 0; e < 16; ++e)
            if (tid + 256 * e < k * k) sD[tid + 256 * e] = d[e];
    } else {
        for (int idx = tid; idx < k * k; idx += 256) {
            const int c = idx / k, a = idx - c * k;
            sD[idx] = blk(Aold, a, c);
        }
    }
    __syncthreads();
    const double* Bq = Bin + b_off[q];
    double* Bo = UPDATE ? Bout + b_off[q] : nullptr;
    double sq = 0.0;
    for (int a0 = 0; a0 < mi; a0 += 256) {
        const int a = a0 + tid;
        const bool ok = a < mi;
        double w[64];
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            double acc = 0.0;
            if (ok && t < k)
                for (int s = 0; s < k; ++s) acc = fma(U[ri0 + a + static_cast<int64_t>(s) * ldUV], sD[s + t * k], acc);
            w[t] = acc;
        }
        for (int c0 = 0; c0 < mj; c0 += CH) {
            for (int idx = tid; idx < CH * 64; idx += 256) {
                const int cc = idx / 64, t = idx - cc * 64;
                sV[idx] = (c0 + cc < mj && t < k) ? V[cj0 + c0 + cc + static_cast<int64_t>(t) * ldUV] : 0.0;
            }
            __syncthreads();
            if (ok) {
                const int nc = min(CH, mj - c0);
                for (int cc = 0; cc < nc; ++cc) {
                    double rec = 0.0;
#pragma unroll
                    for (int t = 0; t < 64; ++t) rec = fma(w[t], sV[cc * 64 + t], rec);
                    const int64_t o = a + static_cast<int64_t>(c0 + cc) * mi;
                    const double v = rec + Bq[o];
                    if (UPDATE) Bo[o] = v;
                    else sq = fma(v, v, sq);
                }
            }
            __syncthreads();
        }
    }
    if (!UPDATE) {
        sq = tr_wave_sum(sq);
        if (lane == 0) red[wave] = sq;
        __syncthreads();
        if (tid == 0) part[q] = red[0] + red[1] + red[2] + red[3];
    }
}

}  // namespace

void launch_trunc_svd(const PlanData& P, const DeviceTables& t, int mode, const double* Atil, double* W,
                      double* sig, hipStream_t s) {
    const int k = P.k;
    if (k > 64) fail(BLR_ERR_UNSUPPORTED, "truncation supports k <= 64");
    const int64_t bk = static_cast<int64_t>(P.b) * k;
    const size_t lds = static_cast<size_t>(2 * k * k + kChunkRows * k) * sizeof(double);
    if (lds > 64 * 1024) {
        // raise the kernels' dynamic LDS limit once per device and size
        static std::mutex mu;
        static size_t set_bytes[64] = {};
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lock(mu);
        if (dev < 0 || dev >= 64 || lds > set_bytes[dev]) {
            for (const void* f : {reinterpret_cast<const void*>(k_trunc_svd<0>),
                                  reinterpret_cast<const void*>(k_trunc_svd<1>)}) {
                hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
                if (e != hipSuccess) fail(BLR_ERR_DEVICE, std::string("LDS attribute: ") + hipGetErrorString(e));
            }
            if (dev >= 0 && dev < 64) set_bytes[dev] = lds;
        }
    }
    if (mode == 0)
        hipLaunchKernelGGL(k_trunc_svd<0>, dim3(P.b), dim3(256), lds, s, Atil, bk, P.b, k, t.nearm, 60, W, sig);
    else
        hipLaunchKernelGGL(k_trunc_svd<1>, dim3(P.b), dim3(256), lds, s, Atil, bk, P.b, k, t.nearm, 60, W, sig);
    check_launch("truncation SVD");
}

void launch_trunc_rows(const PlanData& P, const double* Ain, double* Aout, const double* W, const int32_t* ku,
                       hipStream_t s) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    hipLaunchKernelGGL(k_trunc_rows, dim3(P.b, static_cast<unsigned>((bk + 255) / 256)), dim3(256), 0, s, Ain, Aout,
                       bk, bk, P.k, W, ku);
    check_launch("truncation rows");
}

void launch_trunc_cols(const PlanData& P, double* A, const double* Jm, const int32_t* kv, hipStream_t s) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    hipLaunchKernelGGL(k_trunc_cols, dim3(P.b, static_cast<unsigned>((bk + 255) / 256)), dim3(256), 0, s, A, bk, bk,
                       P.k, Jm, kv);
    check_launch("truncation columns");
}

void launch_trunc_basis(const PlanData& P, const DeviceTables& t, const double* S, double* Sout, const double* W,
                        const int32_t* kr, hipStream_t s) {
    hipLaunchKernelGGL(k_trunc_basis, dim3(P.b), dim3(256), 0, s, S, Sout, P.n, t.box_ptr, P.k, W, kr);
    check_launch("truncation bases");
}

void launch_block_sq(const PlanData& P, const double* Atil, double* part, hipStream_t s) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    hipLaunchKernelGGL(k_block_sq, dim3(P.b, P.b), dim3(256), 0, s, Atil, bk, P.k, part);
    check_launch("block norms");
}

void launch_near_repr_sq(const PlanData& P, const DeviceTables& t, const double* U, const double* V,
                         const double* Atil, const double* Bv, double* part, hipStream_t s) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    hipLaunchKernelGGL(k_trunc_near<0>, dim3(static_cast<unsigned>(P.near_nnz)), dim3(256), 0, s, t.box_ptr,
                       t.pair_row, t.near_idx, t.b_off, U, V, P.n, Atil, Atil, bk, P.k, nullptr, nullptr, Bv,
                       nullptr, part);
    check_launch("near-field norms");
}

void launch_trunc_near(const PlanData& P, const DeviceTables& t, const double* U, const double* V,
                       const double* Aold, const double* Anew, const double* W, const double* Jm,
                       const double* Bin, double* Bout, hipStream_t s) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    hipLaunchKernelGGL(k_trunc_near<1>, dim3(static_cast<unsigned>(P.near_nnz)), dim3(256), 0, s, t.box_ptr,
                       t.pair_row, t.near_idx, t.b_off, U, V, P.n, Aold, Anew, bk, P.k, W, Jm, Bin, Bout, nullptr);
    check_launch("truncation near field");
}

}  // namespace blr
