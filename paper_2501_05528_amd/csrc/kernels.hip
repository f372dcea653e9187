// HIP kernels (gfx950) of the tagged uBLR compression library.
//
// Dense contractions (the sketch, operator products, cores) run on FP64 MFMA
// (v_mfma_f64_16x16x4f64) with the A operand generated tile by tile into LDS
// (kernel matrices: from the point coordinates; dense operators: read in
// place).  Post-processing, probes, apply and error evaluation are
// bandwidth- or generation-bound and use plain VALU code (the near-field apply
// on 16 vectors at a time takes MFMA as well).
//
// MFMA f64 16x16x4 operand layout (wave64, lane l):
//   A (16x4):  lane l holds A[l % 16][l / 16]
//   B (4x16):  lane l holds B[l / 16][l % 16]
//   D (16x16): lane l, element v holds D[l / 16 + 4*v][l % 16]
#include <hip/hip_runtime.h>

#include <mutex>

#include <algorithm>
#include <cmath>
#include <sstream>
#include <type_traits>

#include "kernels.hpp"

namespace blr {

namespace {

typedef double d4 __attribute__((ext_vector_type(4)));

inline void check_launch(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        std::ostringstream os;
        os << what << ": " << hipGetErrorString(e);
        fail(BLR_ERR_DEVICE, os.str());
    }
}

__device__ inline d4 mfma64(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline int d_row(int lane, int v) { return (lane >> 4) + 4 * v; }
__device__ inline int d_col(int lane) { return lane & 15; }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ------------------------------------------------------------ entry sources
// A source yields A(i, j) from a row context and a column context.
// Natural logarithm of a positive, finite, normal x.  x = 2^e m with m in
// [1/sqrt(2), sqrt(2)); log m = 2 atanh(f) with f = (m - 1)/(m + 1), |f| <= 0.1716,
// summed as 2f (1 + f^2/3 + f^4/5 + ... + f^20/21) (the first omitted term is
// below 1e-18 relative); ln 2 is split into a head with 21 trailing zero bits
// (e * head is exact) and a tail.  The quotient f gets two Newton steps on the
// hardware reciprocal and one residual correction.  About 1 ulp.
__device__ inline double log_pos(double x) {
    double m = __builtin_amdgcn_frexp_mant(x);  // [0.5, 1)
    int e = __builtin_amdgcn_frexp_exp(x);
    const bool lo = m < 0.7071067811865476;
    m = lo ? 2.0 * m : m;
    e = lo ? e - 1 : e;
    const double num = m - 1.0, den = m + 1.0;
    double q = __builtin_amdgcn_rcp(den);
    q = fma(fma(-den, q, 1.0), q, q);
    q = fma(fma(-den, q, 1.0), q, q);
    double f = num * q;
    f = fma(fma(-den, f, num), q, f);
    const double s2 = f * f;
    double p = 1.0 / 21.0;
    p = fma(p, s2, 1.0 / 19.0);
    p = fma(p, s2, 1.0 / 17.0);
    p = fma(p, s2, 1.0 / 15.0);
    p = fma(p, s2, 1.0 / 13.0);
    p = fma(p, s2, 1.0 / 11.0);
    p = fma(p, s2, 1.0 / 9.0);
    p = fma(p, s2, 1.0 / 7.0);
    p = fma(p, s2, 1.0 / 5.0);
    p = fma(p, s2, 1.0 / 3.0);
    const double t = 2.0 * f;
    const double lm = fma(t * s2, p, t);
    const double de = static_cast<double>(e);
    return fma(de, 0.6931471803691238, fma(de, 1.9082149292705877e-10, lm));
}

#define BLR_LDS __attribute__((address_space(3)))
#define BLR_GLB __attribute__((address_space(1)))
// A pointer from a job descriptor in memory, marked as device global memory so
// that accesses through it compile to global (not flat) instructions.
template <class T>
__device__ inline BLR_GLB T* as_glb(T* p) {
    return (BLR_GLB T*)p;
}

// Table-driven natural logarithm for the kernel-matrix entries.  x = m 2^e with m in
// [1/2, 1); the top seven mantissa bits of m pick one of 128 centres c (spacing 1/256) with
// r = 1/c stored beside L = -ln r, so that
//   ln x = e ln2 + L + ln(1 + f),   f = m r - 1 (one fused multiply-add, |f| <= 2^-8),
// with ln(1 + f) from its Taylor series to f^6 (truncation below 3e-18).  The table is built
// per workgroup from log_pos.  Absolute error about 2e-16 for |ln x| < 1 (no split of the
// binade at sqrt 2: the entries need absolute, not relative, accuracy near x = 1).
__device__ inline void build_log_table(BLR_LDS double* tab) {
    const int t = threadIdx.x;
    if (t < 128) {
        const double c = 0.5 + (t + 0.5) / 256.0;
        const double r = 1.0 / c;
        tab[2 * t] = r;
        tab[2 * t + 1] = -log_pos(r);
    }
}

__device__ inline double log_tab(double x, const BLR_LDS double* tab) {
    const int e = __builtin_amdgcn_frexp_exp(x);
    const double m = __builtin_amdgcn_frexp_mant(x);
    const int idx = (__double2hiint(m) >> 13) & 127;
    const double r = tab[2 * idx], L = tab[2 * idx + 1];
    const double f = fma(m, r, -1.0);
    double q = -1.0 / 6.0;
    q = fma(q, f, 1.0 / 5.0);
    q = fma(q, f, -1.0 / 4.0);
    q = fma(q, f, 1.0 / 3.0);
    q = fma(q, f, -0.5);
    const double l1 = fma(f * f, q, f);
    const double de = static_cast<double>(e);
    return fma(de, 0.6931471803691238, fma(de, 1.9082149292705877e-10, L + l1));
}

// 1 / sqrt(x) for a positive, finite, normal x: the hardware estimate refined by two
// Newton steps y <- y + y (1 - x y^2) / 2 (each squares the relative error; the residual
// 1 - x y^2 is formed with one fused multiply-add).  About 1 ulp.
__device__ inline double rsqrt_pos(double x) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-(x * y), y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-(x * y), y, 1.0);
    return fma(0.5 * y, e, y);
}

// sqrt(x) for x >= 0 (finite): x / sqrt(x) from the refined reciprocal square root, 0 at 0.
__device__ inline double dist_pos(double x) {
    return x > 0.0 ? x * rsqrt_pos(x) : 0.0;
}

// 1 / x for a positive, finite, normal x: the hardware reciprocal refined by two Newton steps
// (each squares the relative error).  About 1 ulp.
__device__ inline double recip_pos(double x) {
    double q = __builtin_amdgcn_rcp(x);
    q = fma(fma(-x, q, 1.0), q, q);
    return fma(fma(-x, q, 1.0), q, q);
}

template <int KIND>
__device__ inline double kval(double r2) {
    if constexpr (KIND == BLR_KERNEL_LOG) {
        return 0.5 * log_pos(r2);
    } else if constexpr (KIND == BLR_KERNEL_INV_R) {
        return rsqrt_pos(r2);
    } else if constexpr (KIND == BLR_KERNEL_EXP) {
        return exp(-10.0 * dist_pos(r2));   // exp(-r / 0.1)
    } else {
        const double r = dist_pos(r2);
        return cos(20.0 * r) * recip_pos(r + 1e-3);
    }
}

template <int KIND>
struct KernelSrc {
    static constexpr int kKind = KIND;
    const double* px;
    const double* py;
    const double* pz;
    double diag;
    const BLR_LDS double* ltab = nullptr;  // log table in LDS (log kernel), set by prepare()
    // once per workgroup, before any entry (a __syncthreads() must follow)
    __device__ void prepare(BLR_LDS double* tab) {
        if constexpr (KIND == BLR_KERNEL_LOG) {
            build_log_table(tab);
            ltab = tab;
        }
    }
    struct P {
        double x, y, z;
        int64_t i;
    };
    __device__ P row(int64_t i) const { return P{px[i], py[i], pz[i], i}; }
    __device__ P col(int64_t j) const { return P{px[j], py[j], pz[j], j}; }
    // entry between two different points (i != j)
    __device__ double val_off(const P& a, const P& b) const {
        double dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
        const double r2 = dx * dx + dy * dy + dz * dz;
        if constexpr (KIND == BLR_KERNEL_LOG)
            return 0.5 * log_tab(r2, ltab);
        else
            return kval<KIND>(r2);
    }
    __device__ double val(const P& a, const P& b) const { return a.i == b.i ? diag : val_off(a, b); }
    // column contexts staged through LDS: 3 doubles per column
    static constexpr int STAGE = 3;
    __device__ void stage(int64_t j, double* c) const {
        c[0] = px[j];
        c[1] = py[j];
        c[2] = pz[j];
    }
    __device__ P col_staged(const double* c, int64_t j) const { return P{c[0], c[1], c[2], j}; }
    // split entry evaluation: pre() issues the loads of column j, fin() the arithmetic,
    // so a kernel can load the next step's columns before computing on the current one
    using Pre = P;
    __device__ Pre pre(const P&, int64_t j) const { return col(j); }
    __device__ double fin(const P& a, const Pre& b) const { return val(a, b); }
    __device__ double fin_off(const P& a, const Pre& b) const { return val_off(a, b); }
};

struct DenseSrc {  // A(i, j) = A[i + j*lda]
    static constexpr int kKind = -1;
    const double* A;
    int64_t lda;
    __device__ void prepare(BLR_LDS double*) {}
    struct P {
        int64_t i;
    };
    __device__ P row(int64_t i) const { return P{i}; }
    __device__ P col(int64_t j) const { return P{j}; }
    __device__ double val(const P& a, const P& b) const { return A[a.i + b.i * lda]; }
    __device__ double val_off(const P& a, const P& b) const { return val(a, b); }
    static constexpr int STAGE = 1;
    __device__ void stage(int64_t, double* c) const { c[0] = 0.0; }
    __device__ P col_staged(const double*, int64_t j) const { return P{j}; }
    using Pre = double;
    __device__ Pre pre(const P& a, int64_t j) const { return A[a.i + j * lda]; }
    __device__ double fin(const P&, Pre v) const { return v; }
    __device__ double fin_off(const P&, Pre v) const { return v; }
};

struct DenseTSrc {  // (A*)(i, j) = A[j + i*lda]
    static constexpr int kKind = -1;
    const double* A;
    int64_t lda;
    __device__ void prepare(BLR_LDS double*) {}
    struct P {
        int64_t i;
    };
    __device__ P row(int64_t i) const { return P{i}; }
    __device__ P col(int64_t j) const { return P{j}; }
    __device__ double val(const P& a, const P& b) const { return A[b.i + a.i * lda]; }
    __device__ double val_off(const P& a, const P& b) const { return val(a, b); }
    static constexpr int STAGE = 1;
    __device__ void stage(int64_t, double* c) const { c[0] = 0.0; }
    __device__ P col_staged(const double*, int64_t j) const { return P{j}; }
    using Pre = double;
    __device__ Pre pre(const P& a, int64_t j) const { return A[j + a.i * lda]; }
    __device__ double fin(const P&, Pre v) const { return v; }
    __device__ double fin_off(const P&, Pre v) const { return v; }
};

// ------------------------------------------------------------ B operands
// Tagged test matrix (eq. extend_test_mat): column q < LR belongs to Omega
// (from G0), q >= LR to Psi (from G1); within a side q = s*r + c and
// entry (j, q) = T(box(j), s) * G(j, c).
struct TaggedB {
    const double* T;    // row-major b x ell
    const int32_t* rb;  // box of each row
    const double* G0;
    const double* G1;
    int64_t n;
    int r, ell, LR;
    struct C {
        const double* g;
        int s;
    };
    __device__ C col(int q) const {
        int side = q >= LR ? 1 : 0;
        int qq = q - side * LR;
        int s = qq / r;
        int c = qq - s * r;
        return C{(side ? G1 : G0) + static_cast<int64_t>(c) * n, s};
    }
    __device__ double val(int64_t j, const C& c) const {
        return T[static_cast<int64_t>(rb[j]) * ell + c.s] * c.g[j];
    }
};

struct DenseB {
    const double* X;
    int64_t ldx;
    struct C {
        const double* x;
    };
    __device__ C col(int q) const { return C{X + static_cast<int64_t>(q) * ldx}; }
    __device__ double val(int64_t j, const C& c) const { return c.x[j]; }
};

struct SplitOut {  // column q < LR -> C0(:, q), else C1(:, q - LR)
    double* C0;
    double* C1;
    int64_t ld;
    int LR;
    __device__ void put(int64_t i, int q, double v) const {
        if (q < LR)
            C0[i + static_cast<int64_t>(q) * ld] = v;
        else
            C1[i + static_cast<int64_t>(q - LR) * ld] = v;
    }
};

// ------------------------------------------------------------ operator GEMM
// C(M x ncols) = A(M x K) * B(K x ncols), A generated by the source.  One
// workgroup (4 waves) computes a 64 x (4*WN) tile; wave w owns columns
// [w*WN, (w+1)*WN).  K is consumed KT = 8 at a time through double-buffered
// LDS with one barrier per step: while the MFMAs of step k read buffer k%2,
// the workgroup generates the A and B tiles of step k+1 into the other
// buffer, so entry generation overlaps the matrix cores.  Generation is
// branch-free (clamped indices, zero-select outside the matrix) and the
// source index of an A-tile column is wave-uniform (scalar loads).
template <class AS, class BS, class OUT, int WN>
__global__ __launch_bounds__(256, 2) void k_opgemm(AS A, BS B, OUT O, int64_t M, int64_t K,
                                                    int ncols) {
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    A.prepare((BLR_LDS double*)s_ltab);
    __syncthreads();
    constexpr int BM = 64, KT = 8, BN = 4 * WN, NT = WN / 16;
    constexpr int BPT = KT * BN / 256;  // B tile entries per thread
    static_assert((KT * BN) % 256 == 0, "B tile must split evenly over 256 threads");
    __shared__ double sA[2][KT * BM];
    __shared__ double sB[2][KT * BN];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * BM;
    const int col0 = blockIdx.y * BN;

    // A generation: thread (am = lane, kk = 2*wave + u), u < 2
    const int am = lane;
    const int64_t gi = row0 + am;
    const bool rowok = gi < M;
    const auto rp = A.row(rowok ? gi : M - 1);
    // B generation: element e = tid + 256*u of the KT x BN tile (fixed per thread)
    typename BS::C cpu[BPT];
    bool cok[BPT];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int e = tid + 256 * u;
        const int q = col0 + e % BN;
        cok[u] = q < ncols;
        cpu[u] = B.col(q < ncols ? q : ncols - 1);
    }

    auto gen = [&](int buf, int64_t k0) {
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int kk = 2 * wave + u;
            int64_t j = __builtin_amdgcn_readfirstlane(static_cast<int>(min<int64_t>(k0 + kk, K - 1)));
            double v = A.val(rp, A.col(j));
            sA[buf][kk * BM + am] = (rowok && k0 + kk < K) ? v : 0.0;
        }
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int e = tid + 256 * u;
            const int kk = e / BN;
            const int64_t j = min<int64_t>(k0 + kk, K - 1);
            const double v = B.val(j, cpu[u]);
            sB[buf][e] = (cok[u] && k0 + kk < K) ? v : 0.0;
        }
    };

    d4 acc[4][NT];
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = d4{0.0, 0.0, 0.0, 0.0};

    gen(0, 0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = 0; k0 < K; k0 += KT) {
        if (k0 + KT < K) gen(buf ^ 1, k0 + KT);
#pragma unroll
        for (int ks = 0; ks < KT / 4; ++ks) {
            const int kr = ks * 4 + (lane >> 4);
            double a[4], bb[NT];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt) a[mt] = sA[buf][kr * BM + mt * 16 + (lane & 15)];
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) bb[nt] = sB[buf][kr * BN + wave * WN + nt * 16 + (lane & 15)];
#pragma unroll
            for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma64(a[mt], bb[nt], acc[mt][nt]);
        }
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int mt = 0; mt < 4; ++mt)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int col = col0 + wave * WN + nt * 16 + d_col(lane);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t row = row0 + mt * 16 + d_row(lane, v);
                if (row < M && col < ncols) O.put(row, col, acc[mt][nt][v]);
            }
        }
}

// Column-tile width per wave: the widest of 64/48/32/16 that minimises padding.
inline int pick_wn(int ncols) {
    int best = 64;
    int64_t best_pad = -1;
    for (int wn : {64, 48, 32, 16}) {
        const int64_t bn = 4 * wn;
        const int64_t pad = ((ncols + bn - 1) / bn) * bn;
        if (best_pad < 0 || pad < best_pad) {
            best = wn;
            best_pad = pad;
        }
    }
    return best;
}

template <class AS, class BS, class OUT>
void gemm_launch(AS A, BS B, OUT O, int64_t M, int64_t K, int ncols, hipStream_t s) {
    if (M <= 0 || ncols <= 0) return;
    if (K <= 0 || K > INT32_MAX) fail(BLR_ERR_INVALID_ARG, "operator GEMM: bad inner dimension");
    const int wn = pick_wn(ncols);
    const int bn = 4 * wn;
    dim3 grid((M + 63) / 64, (ncols + bn - 1) / bn);
    switch (wn) {
        case 64: hipLaunchKernelGGL((k_opgemm<AS, BS, OUT, 64>), grid, dim3(256), 0, s, A, B, O, M, K, ncols); break;
        case 48: hipLaunchKernelGGL((k_opgemm<AS, BS, OUT, 48>), grid, dim3(256), 0, s, A, B, O, M, K, ncols); break;
        case 32: hipLaunchKernelGGL((k_opgemm<AS, BS, OUT, 32>), grid, dim3(256), 0, s, A, B, O, M, K, ncols); break;
        default: hipLaunchKernelGGL((k_opgemm<AS, BS, OUT, 16>), grid, dim3(256), 0, s, A, B, O, M, K, ncols); break;
    }
    check_launch("operator GEMM");
}

// ------------------------------------------------------------ tagged sketch
// Y(:, s*r + c) = sum_l T(l, s) A(:, I_l) G(I_l, c)  (and Z from H), i.e.
// Y = A Omega with Omega from eq. extend_test_mat.  The K loop walks the
// source boxes l in steps of KT (32) rows that never straddle a box, so within a
// step the tag weight T(l, s) is one scalar per tag column s: it scales the
// MFMA A fragments of the generated kernel tile, and the B tile is the plain
// rows of [G | H] (r columns each, padded to 16*NTR).
//
// Work split: a workgroup owns BM = 4*MA target rows and a group of up to
// 4*SPW "slots" (a slot is one (tag column s, side) pair, ordered s-major);
// its four waves take contiguous, balanced chunks of the slots, so a wave's
// Y and Z columns for the same s share one scaled A fragment.  One kernel
// entry generated into LDS feeds every slot of the workgroup.  Contractions
// use v_mfma_f64_4x4x4f64 with the A fragment replicated over the four
// blocks, i.e. one 4 x 16 x 4 product per instruction:
//   A lane l: A[l % 4][l / 16];  B lane l: B[l / 16][l % 16];
//   D lane l: D[l / 16][l % 16].
// When the last 16-column tile of a two-sided sketch holds at most 12 of the
// r columns (TG = 3, chosen by fp64_sketch_tail_groups where it measured
// faster), it runs in a narrow form instead: the four blocks take
// (4-row quad, 4-source half of an 8-source slice) pairs against 4 columns, so
// its 12 columns cost 3 instructions per 8 sources where the 4 x 16 x 4 form
// spends 4 (r = 42: 11 instead of 12 MFMAs per 4 sources and tag column).
// Tiles are double-buffered in LDS with one barrier per step; the next
// step's [G|H] rows are fetched into registers before the current step's
// MFMAs and stored afterwards.
__device__ inline double mfma44(double a, double b, double c) {
    return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// One workgroup tile of the sketch: target rows [BM rt_blk, BM rt_blk + BM) and tag
// column group grp of ngroups.  The split of the tag columns over groups and waves does
// not change any column's arithmetic.  sAp / sBp: the double-buffered LDS tiles (2 x KT*BM and
// 2 x (KT+1)*BW doubles).
template <class AS, int NTR, int NSIDE, int SVW, int KT, bool EVEN, int TG>
__device__ __attribute__((always_inline)) inline void sketch_tile(
    const AS& A, const double* __restrict__ T, const int64_t* __restrict__ box_ptr, int nbox,
    const double* __restrict__ G0, const double* __restrict__ G1, int64_t n, int r, int ell,
    double* __restrict__ Y0, double* __restrict__ Y1, int64_t rt_blk, int grp, int ngroups,
    BLR_LDS double* sAp, BLR_LDS double* sBp, int tid) {
    constexpr int MA = 2, BM = 4 * MA, CW = NTR * 16;            // rows, cols/side (KT sources/step)
    // TG > 0: the last 16-column tile holds at most 4 TG columns and runs in the narrow form
    constexpr int NTRF = TG > 0 ? NTR - 1 : NTR;                 // tiles in the 4 x 16 x 4 form
    constexpr int TGA = TG > 0 ? TG : 1;
    static_assert(TG >= 0 && TG <= 3 && KT % 8 == 0, "tile shape");
    constexpr int BW = NSIDE * CW;                               // B tile width
    constexpr int BPT = (KT * BW + 255) / 256;
    constexpr int AGEN = BM * KT;                                // A tile entries per step
    static_assert(AGEN <= 256, "tile shape");
    constexpr int KTP = KT + 1;                  // padded column stride of the B tile
    BLR_LDS double (*sA)[KT * BM] = reinterpret_cast<BLR_LDS double (*)[KT * BM]>(sAp);
    BLR_LDS double (*sB)[KTP * BW] = reinterpret_cast<BLR_LDS double (*)[KTP * BW]>(sBp);
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t row0 = rt_blk * BM;
    // this wave's tag columns: a balanced contiguous chunk of the group's.  Groups: 4 SVW
    // tag columns each (the last one the rest), or with EVEN the ell columns split evenly
    // over ngroups >= ell / (4 SVW) groups
    const int sg0 = EVEN ? (grp * ell) / ngroups : grp * 4 * SVW;
    const int sgn = EVEN ? ((grp + 1) * ell) / ngroups - sg0 : min(4 * SVW, ell - sg0);
    const int s_lo = sg0 + (wave * sgn) / 4;
    const int nsv = sg0 + ((wave + 1) * sgn) / 4 - s_lo;
    // A generation: threads t < AGEN own entry (row t % BM, kk = t / BM)
    const bool agen = tid < AGEN;
    const int arow = tid % BM, akk = tid / BM;
    const int64_t gi = row0 + arow;
    const auto rp = A.row(gi < n ? gi : n - 1);
    // B tile: element e = tid + 256*u -> row e % KT, column e / KT (side = column / CW), so
    // KT consecutive threads read one column's KT consecutive rows; LDS holds the tile
    // column-major with stride KTP
    const double* gptr[BPT];
    bool gcol[BPT], gin[BPT];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int e = tid + 256 * u;
        const int cc = e / KT;                   // tile column (coalesced: KT rows per column)
        const int side = cc / CW, c = cc % CW;
        gin[u] = e < KT * BW;
        gcol[u] = gin[u] && c < r;
        gptr[u] = (side ? G1 : G0) + static_cast<int64_t>(gcol[u] ? c : 0) * n;
    }
    double gv[BPT];
    auto fetch_b = [&](int64_t jb, int64_t jend) {
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int kk = (tid + 256 * u) % KT;
            gv[u] = gptr[u][min(jb + kk, jend - 1)];
        }
    };
    // the B tile is stored as read: rows past the box hold finite rows of the clamped read and
    // are cancelled by zero A entries (gen_a), and columns past r (read from column 0) only
    // reach output columns that are never stored
    auto store_b = [&](int buf) {
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int e = tid + 256 * u;
            const int kk = e % KT, cc = e / KT;
            if (gin[u]) sB[buf][cc * KTP + kk] = gv[u];
        }
    };
    // the next step's kernel column is loaded before the current step's MFMAs
    // (pre_a) and turned into an entry after them (gen_a); sources past the box give 0
    typename AS::Pre apre;
    bool ain = true;
    auto pre_a = [&](int64_t jb, int64_t jend) {
        ain = jb + akk < jend;
        if (agen) apre = A.pre(rp, min(jb + akk, jend - 1));
    };
    auto gen_a = [&](int buf) {
        if (agen) sA[buf][akk * BM + arow] = ain ? A.fin(rp, apre) : 0.0;
    };

    double acc[SVW][NSIDE][MA][NTRF > 0 ? NTRF : 1];
    double acct[SVW][NSIDE][TGA];
#pragma unroll
    for (int v = 0; v < SVW; ++v)
#pragma unroll
        for (int sd = 0; sd < NSIDE; ++sd) {
#pragma unroll
            for (int ma = 0; ma < MA; ++ma)
#pragma unroll
                for (int nt = 0; nt < NTRF; ++nt) acc[v][sd][ma][nt] = 0.0;
#pragma unroll
            for (int tg = 0; tg < TGA; ++tg) acct[v][sd][tg] = 0.0;
        }
    // narrow form of the last tile: v_mfma_f64_4x4x4f64 with its four blocks indexed by
    // (4-row quad q, source half h) = (b & 1, b >> 1), b = (lane >> 2) & 3: block b takes rows
    // 4q..4q+3, sources 8j + 4h..8j + 4h + 3 of an 8-source slice j and 4 columns, so one
    // instruction covers 8 rows x 4 columns x 8 sources; the two source halves are added
    // at the end
    const int tq = (lane >> 2) & 1, th = (lane >> 3) & 1;

    int l = 0;
    int64_t j0 = box_ptr[0], jend = box_ptr[1];
    double tw[SVW], twn[SVW];
    auto load_tw = [&](double* w, int lb) {
#pragma unroll
        for (int v = 0; v < SVW; ++v) w[v] = T[static_cast<int64_t>(lb) * ell + min(s_lo + v, ell - 1)];
    };
    fetch_b(j0, jend);
    pre_a(j0, jend);
    load_tw(tw, 0);
    store_b(0);
    gen_a(0);
    __syncthreads();
    int buf = 0;
    for (;;) {
        int ln = l;
        int64_t jn = j0 + KT, jendn = jend;
        if (jn >= jend) {
            ln = l + 1;
            if (ln < nbox) {
                jn = box_ptr[ln];
                jendn = box_ptr[ln + 1];
            }
        }
        const bool more = ln < nbox;
        if (more) {
            fetch_b(jn, jendn);
            pre_a(jn, jendn);
            load_tw(twn, ln);
        }
#pragma unroll
        for (int ks = 0; ks < KT / 4; ++ks) {
            if constexpr (NTRF > 0) {
                const int kr = ks * 4 + (lane >> 4);
                double a[MA];
#pragma unroll
                for (int ma = 0; ma < MA; ++ma) a[ma] = sA[buf][kr * BM + ma * 4 + (lane & 3)];
                double bb[NSIDE][NTRF > 0 ? NTRF : 1];
#pragma unroll
                for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                    for (int nt = 0; nt < NTRF; ++nt)
                        bb[sd][nt] = sB[buf][(sd * CW + nt * 16 + (lane & 15)) * KTP + kr];
#pragma unroll
                for (int v = 0; v < SVW; ++v) {
                    if (v < nsv) {
                        double as[MA];
#pragma unroll
                        for (int ma = 0; ma < MA; ++ma) as[ma] = a[ma] * tw[v];
#pragma unroll
                        for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                            for (int ma = 0; ma < MA; ++ma)
#pragma unroll
                                for (int nt = 0; nt < NTRF; ++nt)
                                    acc[v][sd][ma][nt] = mfma44(as[ma], bb[sd][nt], acc[v][sd][ma][nt]);
                    }
                }
            }
            if constexpr (TG > 0) {
                if (ks & 1) {
                    const int kt = (ks >> 1) * 8 + th * 4 + (lane >> 4);
                    const double at = sA[buf][kt * BM + tq * 4 + (lane & 3)];
                    double bt[NSIDE][TGA];
#pragma unroll
                    for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                        for (int tg = 0; tg < TG; ++tg)
                            bt[sd][tg] = sB[buf][(sd * CW + NTRF * 16 + tg * 4 + (lane & 3)) * KTP + kt];
#pragma unroll
                    for (int v = 0; v < SVW; ++v) {
                        if (v < nsv) {
                            const double ats = at * tw[v];
#pragma unroll
                            for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                                for (int tg = 0; tg < TG; ++tg)
                                    acct[v][sd][tg] = mfma44(ats, bt[sd][tg], acct[v][sd][tg]);
                        }
                    }
                }
            }
        }
        if (!more) break;
        store_b(buf ^ 1);
        gen_a(buf ^ 1);
        __syncthreads();
        buf ^= 1;
        l = ln;
        j0 = jn;
        jend = jendn;
#pragma unroll
        for (int v = 0; v < SVW; ++v) tw[v] = twn[v];
    }
    // epilogue: (s, side) column c -> Y_side(:, s*r + c)
#pragma unroll
    for (int v = 0; v < SVW; ++v) {
        if (v >= nsv) continue;
        const int sv = s_lo + v;
#pragma unroll
        for (int sd = 0; sd < NSIDE; ++sd) {
            double* Yo = sd ? Y1 : Y0;
#pragma unroll
            for (int ma = 0; ma < MA; ++ma) {
                const int64_t row = row0 + ma * 4 + (lane >> 4);
#pragma unroll
                for (int nt = 0; nt < NTRF; ++nt) {
                    const int c = nt * 16 + (lane & 15);
                    if (row < n && c < r) Yo[row + static_cast<int64_t>(sv * r + c) * n] = acc[v][sd][ma][nt];
                }
            }
            if constexpr (TG > 0) {
                const int64_t row = row0 + tq * 4 + (lane >> 4);
#pragma unroll
                for (int tg = 0; tg < TG; ++tg) {
                    // lanes l and l ^ 8 hold the two source halves of one output
                    const double sum = acct[v][sd][tg] + __shfl_xor(acct[v][sd][tg], 8);
                    const int c = NTRF * 16 + tg * 4 + (lane & 3);
                    if (th == 0 && row < n && c < r) Yo[row + static_cast<int64_t>(sv * r + c) * n] = sum;
                }
            }
        }
    }
}

template <class AS, int NTR, int NSIDE, int SVW, int KT, int TG>
__global__ __launch_bounds__(256, 2) void k_sketch(AS A, const double* __restrict__ T,
                                                    const int64_t* __restrict__ box_ptr, int nbox,
                                                    const double* __restrict__ G0,
                                                    const double* __restrict__ G1, int64_t n,
                                                    int r, int ell, double* __restrict__ Y0,
                                                    double* __restrict__ Y1) {
    constexpr int BM = 8, BW = NSIDE * NTR * 16;
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    __shared__ double sA[2 * KT * BM];
    __shared__ double sB[2 * (KT + 1) * BW];
    A.prepare((BLR_LDS double*)s_ltab);
    __syncthreads();
    sketch_tile<AS, NTR, NSIDE, SVW, KT, false, TG>(A, T, box_ptr, nbox, G0, G1, n, r, ell, Y0, Y1, blockIdx.x,
                                                blockIdx.y, gridDim.y, (BLR_LDS double*)sA, (BLR_LDS double*)sB,
                                                static_cast<int>(threadIdx.x));
}

// Persistent form over a batch of FP64 kernel-matrix jobs of one kernel kind (both
// sides): workgroups stride over a list of (job, 8-row block, tag column group) items,
// heaviest job first.  One kind per launch: a per-entry switch over the kinds makes the
// FP64 exp and cos paths spill registers.  The tag columns are split evenly over the
// groups, so a class can use one tag column per wave fewer than k_sketch when every job
// allows it (for ell = 13 and 4 column tiles: 2 groups of 6 and 7 instead of 12 and 1, and
// no spills).  TG is the last-tile form k_sketch takes for the class's kernel kind and r.
// Each tag column's sums run in the same order as in k_sketch, so a job's Y and Z equal
// its single-job sketch bit for bit.
template <int KIND, int NTR, int SVW, int TG>
__global__ __launch_bounds__(256, 2) void k_sketch_multi(const Fp64Job* __restrict__ jobs,
                                                         const int4* __restrict__ items, int nitems) {
    constexpr int KT = 32, BM = 8, BW = 2 * NTR * 16;
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    __shared__ double sA[2 * KT * BM];
    __shared__ double sB[2 * (KT + 1) * BW];
    KernelSrc<KIND> A{nullptr, nullptr, nullptr, 0.0};
    A.prepare((BLR_LDS double*)s_ltab);
    BLR_LDS double* lA = (BLR_LDS double*)sA;
    BLR_LDS double* lB = (BLR_LDS double*)sB;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        const Fp64Job& J = jobs[w.x];
        A.px = (const double*)as_glb(J.px);
        A.py = (const double*)as_glb(J.py);
        A.pz = (const double*)as_glb(J.pz);
        A.diag = J.diag;
        __syncthreads();  // the table is built; the previous item's last reads of LDS are done
        sketch_tile<KernelSrc<KIND>, NTR, 2, SVW, KT, true, TG>(
            A, (const double*)as_glb(J.T), (const int64_t*)as_glb(J.box_ptr), J.nbox,
            (const double*)as_glb(J.G0), (const double*)as_glb(J.G1), J.n, J.r, J.ell,
            (double*)as_glb(J.Y0), (double*)as_glb(J.Y1), w.y, w.z, J.ngroups, lA, lB,
            static_cast<int>(threadIdx.x));
    }
}

template <class AS>
void sketch_launch(AS A, const PlanData& P, const DeviceTables& t, const double* G0,
                   const double* G1, int nside, double* Y0, double* Y1, hipStream_t s) {
    const int ntr = (P.r + 15) / 16;
    // tag columns per wave bounded by the accumulator budget (SVW*NSIDE*2*NTR doubles)
    const int acc_per_sv = nside * 2 * ntr;
    const int svw = std::max(1, std::min(8, 48 / acc_per_sv));
    const int groups = (P.ell + 4 * svw - 1) / (4 * svw);
    dim3 grid((P.n + 7) / 8, groups);
#define BLR_SKETCH_CASE_TG(NTRV, NSV, SVWV, TGV)                                                          \
    hipLaunchKernelGGL((k_sketch<AS, NTRV, NSV, SVWV, 32, TGV>), grid, dim3(256), 0, s, A, t.T, t.box_ptr, \
                       P.b, G0, G1, P.n, P.r, P.ell, Y0, Y1)
#define BLR_SKETCH_CASE(NTRV, NSV, SVWV) BLR_SKETCH_CASE_TG(NTRV, NSV, SVWV, 0)
// both sides: the last column tile in the narrow form when it holds at most 12 columns
#define BLR_SKETCH_CASE2(NTRV, SVWV)                                           \
    do {                                                                       \
        if (fp64_sketch_tail_groups(AS::kKind, P.r) == 3) BLR_SKETCH_CASE_TG(NTRV, 2, SVWV, 3); \
        else BLR_SKETCH_CASE(NTRV, 2, SVWV);                                   \
    } while (0)
    if (nside == 2) {
        switch (ntr) {
            case 1: BLR_SKETCH_CASE2(1, 8); break;  // 48 / 4 = 12 -> 8
            case 2: BLR_SKETCH_CASE2(2, 6); break;
            case 3: BLR_SKETCH_CASE2(3, 4); break;
            case 4: BLR_SKETCH_CASE2(4, 3); break;
            case 5: BLR_SKETCH_CASE2(5, 2); break;
            default: fail(BLR_ERR_UNSUPPORTED, "k + p > 80 is not supported by the sketch kernel");
        }
    } else {
        switch (ntr) {
            case 1: BLR_SKETCH_CASE(1, 1, 8); break;
            case 2: BLR_SKETCH_CASE(2, 1, 8); break;
            case 3: BLR_SKETCH_CASE(3, 1, 8); break;
            case 4: BLR_SKETCH_CASE(4, 1, 6); break;
            case 5: BLR_SKETCH_CASE(5, 1, 4); break;
            default: fail(BLR_ERR_UNSUPPORTED, "k + p > 80 is not supported by the sketch kernel");
        }
    }
#undef BLR_SKETCH_CASE2
#undef BLR_SKETCH_CASE
#undef BLR_SKETCH_CASE_TG
    check_launch("tagged sketch");
}

}  // namespace

int fp64_sketch_svw(int ntr) { return std::max(1, std::min(8, 12 / std::max(1, ntr))); }

int fp64_sketch_tail_groups(int kind, int r) {
    const int ntr = (r + 15) / 16;
    if (r <= 0 || r - 16 * (ntr - 1) > 12) return 0;
    // measured on MI355X: faster with 2 or 3 column tiles for every entry source; with 4 only
    // for 1/r (exp and cos spill registers there and run slower, log gains nothing)
    return ntr == 2 || ntr == 3 || (ntr == 4 && kind == BLR_KERNEL_INV_R) ? 3 : 0;
}

void launch_sketch_multi(int kind, int ntr, int svw, int tg, const Fp64Job* jobs, const int4* items,
                         int nitems, int grid, hipStream_t s) {
    if (nitems <= 0) return;
    if (tg != 0 && tg != 3) fail(BLR_ERR_INVALID_ARG, "tail form of the persistent FP64 sketch must be 0 or 3");
    const dim3 g(static_cast<unsigned>(std::max(1, std::min(grid, nitems))));
    auto run = [&](auto kc) {
        constexpr int K = decltype(kc)::value;
        // SVW: fp64_sketch_svw(ntr) or one less
#define BLR_MULTI(NTRV, SVWV)                                                                                 \
    do {                                                                                                      \
        if (tg == 3) hipLaunchKernelGGL((k_sketch_multi<K, NTRV, SVWV, 3>), g, dim3(256), 0, s, jobs, items, nitems); \
        else hipLaunchKernelGGL((k_sketch_multi<K, NTRV, SVWV, 0>), g, dim3(256), 0, s, jobs, items, nitems);        \
    } while (0)
        if (ntr == 1 && svw == 8) BLR_MULTI(1, 8);
        else if (ntr == 1 && svw == 7) BLR_MULTI(1, 7);
        else if (ntr == 2 && svw == 6) BLR_MULTI(2, 6);
        else if (ntr == 2 && svw == 5) BLR_MULTI(2, 5);
        else if (ntr == 3 && svw == 4) BLR_MULTI(3, 4);
        else if (ntr == 3 && svw == 3) BLR_MULTI(3, 3);
        else if (ntr == 4 && svw == 3) BLR_MULTI(4, 3);
        else if (ntr == 4 && svw == 2) BLR_MULTI(4, 2);
        else if (ntr == 5 && svw == 2) BLR_MULTI(5, 2);
        else if (ntr == 5 && svw == 1) BLR_MULTI(5, 1);
        else fail(BLR_ERR_UNSUPPORTED, "no persistent FP64 sketch for this column-tile count and SVW");
#undef BLR_MULTI
    };
    switch (kind) {
        case BLR_KERNEL_LOG: run(std::integral_constant<int, BLR_KERNEL_LOG>{}); break;
        case BLR_KERNEL_INV_R: run(std::integral_constant<int, BLR_KERNEL_INV_R>{}); break;
        case BLR_KERNEL_EXP: run(std::integral_constant<int, BLR_KERNEL_EXP>{}); break;
        case BLR_KERNEL_COS: run(std::integral_constant<int, BLR_KERNEL_COS>{}); break;
        default: fail(BLR_ERR_INVALID_ARG, "unknown kernel kind");
    }
    check_launch("persistent tagged sketch");
}

namespace {

// Calls f(src) with the entry source of the operator (or of its adjoint).
template <class F>
void with_source(const OpData& op, int trans, F&& f) {
    if (op.type == OpType::Dense) {
        if (trans)
            f(DenseTSrc{op.A, op.lda});
        else
            f(DenseSrc{op.A, op.lda});
        return;
    }
    const double* px = op.pts;
    const double* py = op.pts + op.n;
    const double* pz = op.pts + 2 * op.n;
    switch (op.kind) {
        case BLR_KERNEL_LOG: f(KernelSrc<BLR_KERNEL_LOG>{px, py, pz, 0.0}); break;
        case BLR_KERNEL_INV_R: f(KernelSrc<BLR_KERNEL_INV_R>{px, py, pz, 0.0}); break;
        case BLR_KERNEL_EXP: f(KernelSrc<BLR_KERNEL_EXP>{px, py, pz, 1.0}); break;
        case BLR_KERNEL_COS: f(KernelSrc<BLR_KERNEL_COS>{px, py, pz, 1000.0}); break;
        default: fail(BLR_ERR_INVALID_ARG, "unknown kernel kind");
    }
}

// ------------------------------------------------------------ refinement sketch
// Far-field samples of the mixed-precision mode (one FP64 sketch on the
// mixed sample bases):
//   S0(I_i, :) = sum_{l in F_i} A(I_i, I_l) X0(I_l, :)   and S1 from X1,
// with the same kernel tile for both sides when the matrix is symmetric.  Near
// blocks are masked to zero as the tile is generated; a source box that is
// near to every row of the workgroup is skipped.  Workgroup: 16 MA target rows;
// wave w owns rows 4 MA w .. 4 MA (w + 1) - 1 (MA 4-row tiles of
// v_mfma_f64_4x4x4f64, the layout of k_sketch) and every column tile of both sides.
template <class AS, int NTR, int NSIDE, int MA>
__global__ __launch_bounds__(256, 2) void k_refine(AS A, const int64_t* __restrict__ box_ptr,
                                                   const int32_t* __restrict__ row_box,
                                                   const uint8_t* __restrict__ nearm, int nbox,
                                                   const double* __restrict__ X0,
                                                   const double* __restrict__ X1, int64_t n, int r,
                                                   double* __restrict__ S0, double* __restrict__ S1) {
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    A.prepare((BLR_LDS double*)s_ltab);
    __syncthreads();
    constexpr int BM = 16 * MA, KT = 16, CW = NTR * 16, BW = NSIDE * CW;
    constexpr int KSTEP = 256 / BM;              // source stride of one thread's entries
    constexpr int BPT = (KT * BW + 255) / 256;
    __shared__ double sA[2][KT * BM];
    constexpr int KTP = KT + 1;                  // padded column stride of the B tile
    __shared__ double sB[2][KTP * BW];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * BM;
    const int64_t rlast = min(row0 + BM, n) - 1;
    const int box_first = row_box[row0], box_last = row_box[rlast];
    const bool single = box_first == box_last;
    // generation: thread owns row tid % BM and sources tid / BM + KSTEP u, u < MA
    // with BM a multiple of 64 every thread of a wave takes the same source column in each
    // entry slot, so the column's points are loaded once per wave (scalar loads)
    const int arow = tid % BM;
    const int akk = BM % 64 == 0 ? __builtin_amdgcn_readfirstlane(tid / BM) : tid / BM;
    const int64_t gi = min(row0 + arow, n - 1);
    const auto rp = A.row(gi);
    const int64_t mybox_row = static_cast<int64_t>(row_box[gi]) * nbox;
    // B tile [X0 | X1]: element e = tid + 256*u -> row e % KT, column e / KT (coalesced
    // column reads), stored column-major in LDS with stride KTP
    const double* gptr[BPT];
    bool gcol[BPT], gin[BPT];
#pragma unroll
    for (int u = 0; u < BPT; ++u) {
        const int e = tid + 256 * u;
        const int cc = e / KT;                   // tile column (coalesced: KT rows per column)
        const int side = cc / CW, c = cc % CW;
        gin[u] = e < KT * BW;
        gcol[u] = gin[u] && c < r;
        gptr[u] = (side ? X1 : X0) + static_cast<int64_t>(gcol[u] ? c : 0) * n;
    }
    double gv[BPT];
    auto fetch_b = [&](int64_t jb, int64_t jend) {
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int kk = (tid + 256 * u) % KT;
            gv[u] = gptr[u][min(jb + kk, jend - 1)];
        }
    };
    // rows past the box and columns past r need no zeroing here: the A tile is zero in
    // those rows (gen_a) and the padding columns of the accumulators are never stored, and
    // the values read there are finite rows of X0 / X1
    auto store_b = [&](int buf) {
#pragma unroll
        for (int u = 0; u < BPT; ++u) {
            const int e = tid + 256 * u;
            const int kk = e % KT, cc = e / KT;
            if (gin[u]) sB[buf][cc * KTP + kk] = gv[u];
        }
    };
    // the next step's kernel columns and far mask are loaded before the current
    // step's MFMAs (pre_a) and turned into entries after them (gen_a)
    typename AS::Pre apre[MA];
    bool far_pre = true;
    auto pre_a = [&](int l, int64_t jb, int64_t jend) {
        far_pre = nearm[mybox_row + l] == 0;
#pragma unroll
        for (int u = 0; u < MA; ++u) {
            const int64_t j = jb + akk + KSTEP * u;
            apre[u] = A.pre(rp, j < jend ? j : jend - 1);
        }
    };
    // near blocks (the diagonal among them) are masked, so no entry needs the diagonal rule;
    // a masked value is discarded by the select, never multiplied
    auto gen_a = [&](int buf, int64_t jb, int64_t jend) {
#pragma unroll
        for (int u = 0; u < MA; ++u) {
            const int kk = akk + KSTEP * u;
            const double v = A.fin_off(rp, apre[u]);
            sA[buf][kk * BM + arow] = (far_pre && jb + kk < jend) ? v : 0.0;
        }
    };
    // next source box at or after l that is not near to the whole workgroup
    auto next_box = [&](int l) {
        while (l < nbox && single && nearm[static_cast<int64_t>(box_first) * nbox + l]) ++l;
        return l;
    };

    double acc[NSIDE][MA][NTR];
#pragma unroll
    for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
        for (int ma = 0; ma < MA; ++ma)
#pragma unroll
            for (int nt = 0; nt < NTR; ++nt) acc[sd][ma][nt] = 0.0;

    int l = next_box(0);
    if (l < nbox) {
        int64_t j0 = box_ptr[l], jend = box_ptr[l + 1];
        fetch_b(j0, jend);
        pre_a(l, j0, jend);
        store_b(0);
        gen_a(0, j0, jend);
        __syncthreads();
        int buf = 0;
        for (;;) {
            int ln = l;
            int64_t jn = j0 + KT, jendn = jend;
            if (jn >= jend) {
                ln = next_box(l + 1);
                if (ln < nbox) {
                    jn = box_ptr[ln];
                    jendn = box_ptr[ln + 1];
                }
            }
            const bool more = ln < nbox;
            if (more) {
                fetch_b(jn, jendn);
                pre_a(ln, jn, jendn);
            }
#pragma unroll
            for (int ks = 0; ks < KT / 4; ++ks) {
                const int kr = ks * 4 + (lane >> 4);
                double a[MA];
#pragma unroll
                for (int ma = 0; ma < MA; ++ma) a[ma] = sA[buf][kr * BM + wave * 4 * MA + ma * 4 + (lane & 3)];
                double bb[NSIDE][NTR];
#pragma unroll
                for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                    for (int nt = 0; nt < NTR; ++nt) bb[sd][nt] = sB[buf][(sd * CW + nt * 16 + (lane & 15)) * KTP + kr];
#pragma unroll
                for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                    for (int ma = 0; ma < MA; ++ma)
#pragma unroll
                        for (int nt = 0; nt < NTR; ++nt) acc[sd][ma][nt] = mfma44(a[ma], bb[sd][nt], acc[sd][ma][nt]);
            }
            if (!more) break;
            store_b(buf ^ 1);
            gen_a(buf ^ 1, jn, jendn);
            __syncthreads();
            buf ^= 1;
            l = ln;
            j0 = jn;
            jend = jendn;
        }
    }
#pragma unroll
    for (int sd = 0; sd < NSIDE; ++sd) {
        double* So = sd ? S1 : S0;
#pragma unroll
        for (int ma = 0; ma < MA; ++ma) {
            const int64_t row = row0 + wave * 4 * MA + ma * 4 + (lane >> 4);
#pragma unroll
            for (int nt = 0; nt < NTR; ++nt) {
                const int c = nt * 16 + (lane & 15);
                if (row < n && c < r) So[row + static_cast<int64_t>(c) * n] = acc[sd][ma][nt];
            }
        }
    }
}

template <class AS>
void refine_launch(AS A, const PlanData& P, const DeviceTables& t, const double* X0,
                   const double* X1, int nside, double* S0, double* S1, hipStream_t s) {
    const int ntr = (P.r + 15) / 16;
    constexpr int MAV = 4;  // 64 target rows per workgroup (32 measured slower)
    const dim3 grid(static_cast<unsigned>((P.n + 16 * MAV - 1) / (16 * MAV)));
#define BLR_REFINE_CASE(NTRV, NSV)                                                                      \
    hipLaunchKernelGGL((k_refine<AS, NTRV, NSV, MAV>), grid, dim3(256), 0, s, A, t.box_ptr, t.row_box, \
                       t.nearm, P.b, X0, X1, P.n, P.r, S0, S1)
    if (nside == 2) {
        switch (ntr) {
            case 1: BLR_REFINE_CASE(1, 2); break;
            case 2: BLR_REFINE_CASE(2, 2); break;
            case 3: BLR_REFINE_CASE(3, 2); break;
            case 4: BLR_REFINE_CASE(4, 2); break;
            case 5: BLR_REFINE_CASE(5, 2); break;
            default: fail(BLR_ERR_UNSUPPORTED, "k + p > 80 is not supported by the refinement sketch");
        }
    } else {
        switch (ntr) {
            case 1: BLR_REFINE_CASE(1, 1); break;
            case 2: BLR_REFINE_CASE(2, 1); break;
            case 3: BLR_REFINE_CASE(3, 1); break;
            case 4: BLR_REFINE_CASE(4, 1); break;
            case 5: BLR_REFINE_CASE(5, 1); break;
            default: fail(BLR_ERR_UNSUPPORTED, "k + p > 80 is not supported by the refinement sketch");
        }
    }
#undef BLR_REFINE_CASE
    check_launch("refinement sketch");
}

// ------------------------------------------------------------ post-processing
// Yhat(row, c) = sum_s z(box(row), s) * Y(row, s*r + c)   (Alg. 2 weighted sum)
template <class TIN>
__global__ __launch_bounds__(256) void k_postprocess(const TIN* __restrict__ Y,
                                                     double* __restrict__ Yh,
                                                     const double* __restrict__ z,
                                                     const int32_t* __restrict__ rb, int64_t n,
                                                     int r, int ell) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= n * r) return;
    const int c = static_cast<int>(idx / n);
    const int64_t row = idx - static_cast<int64_t>(c) * n;
    const double* zb = z + static_cast<int64_t>(rb[row]) * ell;
    double acc = 0.0;
    for (int s = 0; s < ell; ++s) acc += zb[s] * static_cast<double>(Y[row + static_cast<int64_t>(s * r + c) * n]);
    Yh[row + static_cast<int64_t>(c) * n] = acc;
}

// ------------------------------------------------------------ orthonormalisation
// col(S_i, k) for every box (one workgroup per box and side):
//   1. Householder QR of the m x r block S_i = Q R (reflectors kept below the
//      diagonal, in LDS when it fits, else in place in S);
//   2. one-sided (Hestenes) Jacobi on R^T: R^T J has orthogonal columns with
//      norms sigma, so R = J Sigma X^T and J holds the left singular vectors of
//      R.  Triangular preconditioning makes the sweep count small (about 8 for
//      samples whose singular values span 13 decades, against 23 on S_i itself);
//   3. the k columns of J with the largest sigma (descending, ties to the lower
//      index) give U_i = Q [W_k; 0], formed by applying the reflectors in reverse;
//   4. each column is signed so that its entry of largest magnitude (lowest row
//      on ties) is positive.
__device__ inline int rr_player(int pos, int round, int n) {
    return pos == 0 ? 0 : 1 + (pos - 1 + round) % (n - 1);
}

__global__ __launch_bounds__(256) void k_orth(double* S0, double* S1, int64_t ldS,
                                              const int64_t* box_ptr, int nbox, int r, int k,
                                              double* Q0, double* Q1, int64_t ldQ,
                                              double* sigma0, double* sigma1, int m_in_lds,
                                              int max_sweeps, int qr_only) {
    extern __shared__ double smem[];
    __shared__ double rdiag[128], vvs[128], norms[128];
    __shared__ int order[128];
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int side = blockIdx.x >= nbox ? 1 : 0;
    const int box = blockIdx.x - side * nbox;
    double* S = side ? S1 : S0;
    double* Q = side ? Q1 : Q0;
    double* sigma = side ? sigma1 : sigma0;
    const int64_t r0 = box_ptr[box];
    const int m = static_cast<int>(box_ptr[box + 1] - r0);
    double* Rt = smem;                      // r x r, column-major
    double* J = smem + r * r;               // r x r, column-major
    double* M;
    int64_t ldm;
    if (m_in_lds) {
        M = smem + 2 * r * r;
        ldm = m;
        for (int idx = tid; idx < m * r; idx += 256) {
            const int c = idx / m, a = idx - c * m;
            M[a + static_cast<int64_t>(c) * m] = S[r0 + a + static_cast<int64_t>(c) * ldS];
        }
    } else {
        M = S + r0;
        ldm = ldS;
    }
    __syncthreads();
    // 1. Householder QR.  Wave 0 forms reflector 0; afterwards the reflector of column j + 1
    // is formed by wave 0 right after it applies reflector j to that column (look-ahead), with
    // the same row-to-lane map as the update, so every column costs one barrier.
    auto reflector = [&](int j, double s2, double x0) {   // wave 0, after the wave sums
        const double alpha = x0 >= 0.0 ? -sqrt(s2) : sqrt(s2);
        if (lane == 0) {
            rdiag[j] = alpha;
            vvs[j] = s2 - x0 * x0 + (x0 - alpha) * (x0 - alpha);
        }
        return x0 - alpha;
    };
    if (wave == 0) {
        double s2 = 0.0;
        for (int a = lane; a < m; a += 64) s2 += M[a] * M[a];
        s2 = wave_sum(s2);
        const double x0 = M[0];
        const double h = reflector(0, s2, x0);
        if (lane == 0) M[0] = h;
    }
    __syncthreads();
    for (int j = 0; j < r; ++j) {
        double* x = M + static_cast<int64_t>(j) * ldm;
        const double vv = vvs[j];
        int c = j + 1 + wave;
        if (wave == 0 && j + 1 < r) {
            double* y = M + static_cast<int64_t>(j + 1) * ldm;
            double d = 0.0;
            for (int a = j + lane; a < m; a += 64) d = fma(x[a], y[a], d);
            d = wave_sum(d);
            const double f = vv > 0.0 ? 2.0 * d / vv : 0.0;
            double s2 = 0.0, y1 = 0.0;
            for (int a = j + lane; a < m; a += 64) {
                const double yn = y[a] - f * x[a];
                y[a] = yn;
                if (a > j) s2 = fma(yn, yn, s2);
                if (a == j + 1) y1 = yn;
            }
            s2 = wave_sum(s2);
            const double x0 = wave_sum(y1);                 // row j + 1 lives on lane 1 only
            const double h = reflector(j + 1, s2, x0);
            if (lane == 1) y[j + 1] = h;
            c += 4;
        }
        // two columns per wave at a time: their reductions and updates are independent
        for (; c + 4 < r; c += 8) {
            double* y = M + static_cast<int64_t>(c) * ldm;
            double* y2 = M + static_cast<int64_t>(c + 4) * ldm;
            double d = 0.0, d2 = 0.0;
            for (int a = j + lane; a < m; a += 64) {
                const double xa = x[a];
                d = fma(xa, y[a], d);
                d2 = fma(xa, y2[a], d2);
            }
            d = wave_sum(d);
            d2 = wave_sum(d2);
            const double f = vv > 0.0 ? 2.0 * d / vv : 0.0;
            const double f2 = vv > 0.0 ? 2.0 * d2 / vv : 0.0;
            for (int a = j + lane; a < m; a += 64) {
                const double xa = x[a];
                y[a] -= f * xa;
                y2[a] -= f2 * xa;
            }
        }
        if (c < r) {
            double* y = M + static_cast<int64_t>(c) * ldm;
            double d = 0.0;
            for (int a = j + lane; a < m; a += 64) d += x[a] * y[a];
            d = wave_sum(d);
            const double f = vv > 0.0 ? 2.0 * d / vv : 0.0;
            for (int a = j + lane; a < m; a += 64) y[a] -= f * x[a];
        }
        __syncthreads();
    }
    // Rt = R^T, J = I
    for (int idx = tid; idx < r * r; idx += 256) {
        const int b = idx / r, a = idx - b * r;       // Rt(a, b) = R(b, a)
        double v = 0.0;
        if (a == b) v = rdiag[b];
        else if (a > b) v = M[b + static_cast<int64_t>(a) * ldm];
        Rt[idx] = v;
        J[idx] = (a == b) ? 1.0 : 0.0;
    }
    __syncthreads();
    // 2. one-sided Jacobi on the columns of Rt, rotations accumulated in J
    // (skipped in QR-only mode: then U = the first k columns of Q).  Each round's
    // nr/2 column pairs (round-robin order) are disjoint; a group of 8 lanes
    // rotates one pair, its lanes striding over the r entries and reducing the
    // three inner products with in-group shuffles; 32 groups share a round, so
    // up to 64 columns take one pass per round.
    const double tol = sqrt(static_cast<double>(r)) * 2.220446049250313e-16;
    const int nr = r + (r & 1);
    const int grp = tid >> 3, gl = tid & 7;
    for (int sweep = 0; sweep < (qr_only ? 0 : max_sweeps); ++sweep) {
        int rotated = 0;
        for (int round = 0; round < nr - 1; ++round) {
            for (int u = grp; u < nr / 2; u += 32) {
                int p = rr_player(u, round, nr), q = rr_player(nr - 1 - u, round, nr);
                if (p > q) {
                    const int t = p;
                    p = q;
                    q = t;
                }
                if (q >= r) continue;
                double* xp = Rt + p * r;
                double* xq = Rt + q * r;
                double al = 0.0, be = 0.0, ga = 0.0;
                for (int a = gl; a < r; a += 8) {
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
                    double* jp = J + p * r;
                    double* jq = J + q * r;
                    for (int a = gl; a < r; a += 8) {
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
    // 3. singular values and their order
    for (int c = wave; c < r; c += 4) {
        double s2 = 0.0;
        for (int a = lane; a < r; a += 64) s2 += Rt[c * r + a] * Rt[c * r + a];
        s2 = wave_sum(s2);
        if (lane == 0) norms[c] = sqrt(s2);
    }
    __syncthreads();
    if (tid < r) {
        const double nv = norms[tid];
        int rank = 0;
        for (int c = 0; c < r; ++c) rank += (norms[c] > nv) || (norms[c] == nv && c < tid);
        order[qr_only ? tid : rank] = tid;
    }
    __syncthreads();
    if (sigma && tid < r) sigma[static_cast<int64_t>(box) * r + tid] = norms[order[tid]];
    // 4. U = Q [W_k; 0], applying H_{r-1} ... H_0; then the sign rule.  Boxes of at most 256
    // rows keep four output columns of a wave in registers (lane l holds rows l + 64 t), so
    // each reflector is read once for the four and their reductions overlap.
    if (m <= 256) {
        constexpr int MT = 4, CB = 4;
        const int ncw = (k - wave + 3) / 4;          // this wave's columns t = wave + 4 q
        for (int q0 = 0; q0 < ncw; q0 += CB) {
            double u[CB][MT];
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const bool valid = q0 + cb < ncw;
                const double* w = J + order[valid ? wave + 4 * (q0 + cb) : wave] * r;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int a = lane + 64 * mt;
                    u[cb][mt] = (valid && a < r) ? w[a] : 0.0;
                }
            }
            for (int j = r - 1; j >= 0; --j) {
                const double* x = M + static_cast<int64_t>(j) * ldm;
                double xv[MT];
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int a = lane + 64 * mt;
                    xv[mt] = (a >= j && a < m) ? x[a] : 0.0;
                }
                const double vv = vvs[j];
                double d[CB];
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    d[cb] = 0.0;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) d[cb] = fma(xv[mt], u[cb][mt], d[cb]);
                }
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) d[cb] = wave_sum(d[cb]);
#pragma unroll
                for (int cb = 0; cb < CB; ++cb) {
                    const double f = vv > 0.0 ? 2.0 * d[cb] / vv : 0.0;
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) u[cb][mt] -= f * xv[mt];
                }
            }
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                if (q0 + cb >= ncw) continue;
                const int t = wave + 4 * (q0 + cb);
                double best = -1.0, sval = 0.0;
                int bi = 0;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int a = lane + 64 * mt;
                    const double v = fabs(u[cb][mt]);
                    if (a < m && v > best) {
                        best = v;
                        bi = a;
                        sval = u[cb][mt];
                    }
                }
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    const double ob = __shfl_xor(best, o, 64);
                    const int oi = __shfl_xor(bi, o, 64);
                    const double os = __shfl_xor(sval, o, 64);
                    if (ob > best || (ob == best && oi < bi)) {
                        best = ob;
                        bi = oi;
                        sval = os;
                    }
                }
                const double sg = sval < 0.0 ? -1.0 : 1.0;
                double* uo = Q + r0 + static_cast<int64_t>(t) * ldQ;
#pragma unroll
                for (int mt = 0; mt < MT; ++mt) {
                    const int a = lane + 64 * mt;
                    if (a < m) uo[a] = sg * u[cb][mt];
                }
            }
        }
        return;
    }
    for (int t = wave; t < k; t += 4) {
        double* u = Q + r0 + static_cast<int64_t>(t) * ldQ;
        const double* w = J + order[t] * r;
        for (int a = lane; a < m; a += 64) u[a] = a < r ? w[a] : 0.0;
        for (int j = r - 1; j >= 0; --j) {
            const double* x = M + static_cast<int64_t>(j) * ldm;
            double d = 0.0;
            for (int a = j + lane; a < m; a += 64) d += x[a] * u[a];
            d = wave_sum(d);
            const double vv = vvs[j];
            const double f = vv > 0.0 ? 2.0 * d / vv : 0.0;
            for (int a = j + lane; a < m; a += 64) u[a] -= f * x[a];
        }
        double best = -1.0;
        int bi = 0;
        for (int a = lane; a < m; a += 64) {
            const double v = fabs(u[a]);
            if (v > best) {
                best = v;
                bi = a;
            }
        }
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            const double ob = __shfl_xor(best, o, 64);
            const int oi = __shfl_xor(bi, o, 64);
            if (ob > best || (ob == best && oi < bi)) {
                best = ob;
                bi = oi;
            }
        }
        if (u[bi] < 0.0)
            for (int a = lane; a < m; a += 64) u[a] = -u[a];
    }
}

// ------------------------------------------------------------ cores
// Atil_ij = U_i^T A_ij V_j for one pair per workgroup.  W = A_ij V_j is built
// on MFMA in 256-row chunks (wave w owns 64 rows); U_i^T W then reuses W
// straight from the MFMA accumulators: for a fixed element index v the
// accumulator holds rows {g + 4v} (g = lane/16) of a 16-row tile, which is
// exactly the 4-deep K slice of a B operand.
template <class AS, int NT>
__global__ __launch_bounds__(256, (NT >= 4 ? 1 : 2)) void k_cores(AS A, const int64_t* __restrict__ box_ptr,
                                                  const double* __restrict__ U,
                                                  const double* __restrict__ V, int64_t ldUV,
                                                  int k, double* __restrict__ Atil, int64_t ldAt) {
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    A.prepare((BLR_LDS double*)s_ltab);
    __syncthreads();
    constexpr int KT = 16, RC = 256, KP = NT * 16;
    __shared__ double sA[KT * RC];
    __shared__ double sV[KT * KP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x, i = blockIdx.y;
    const int64_t ri0 = box_ptr[i], cj0 = box_ptr[j];
    const int mi = static_cast<int>(box_ptr[i + 1] - ri0);
    const int mj = static_cast<int>(box_ptr[j + 1] - cj0);
    d4 accT[NT][NT];
#pragma unroll
    for (int at = 0; at < NT; ++at)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) accT[at][nt] = d4{0.0, 0.0, 0.0, 0.0};

    for (int rc0 = 0; rc0 < mi; rc0 += RC) {
        const int grow = rc0 + tid;
        const bool rowok = grow < mi;
        const auto rp = A.row(ri0 + (rowok ? grow : 0));
        d4 acc[4][NT];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = d4{0.0, 0.0, 0.0, 0.0};
        // a whole step of an off-diagonal pair needs neither the column bound nor the diagonal
        // rule; rows past the box repeat its first point (finite entries, and their products
        // meet zero rows of U and V below)
        const bool offdiag = i != j;
        for (int k0 = 0; k0 < mj; k0 += KT) {
            if (offdiag && k0 + KT <= mj) {
#pragma unroll 4
                for (int kk = 0; kk < KT; ++kk) sA[kk * RC + tid] = A.val_off(rp, A.col(cj0 + k0 + kk));
            } else {
#pragma unroll 4
                for (int kk = 0; kk < KT; ++kk) {
                    double v = 0.0;
                    if (rowok && k0 + kk < mj) v = A.val(rp, A.col(cj0 + k0 + kk));
                    sA[kk * RC + tid] = v;
                }
            }
            for (int idx = tid; idx < KT * KP; idx += 256) {
                const int kk = idx / KP, c = idx - kk * KP;
                double v = 0.0;
                if (k0 + kk < mj && c < k) v = V[cj0 + k0 + kk + static_cast<int64_t>(c) * ldUV];
                sV[idx] = v;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < KT / 4; ++ks) {
                const int kr = ks * 4 + (lane >> 4);
                double a[4], bb[NT];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) a[mt] = sA[kr * RC + wave * 64 + mt * 16 + (lane & 15)];
#pragma unroll
                for (int nt = 0; nt < NT; ++nt) bb[nt] = sV[kr * KP + nt * 16 + (lane & 15)];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) acc[mt][nt] = mfma64(a[mt], bb[nt], acc[mt][nt]);
            }
            __syncthreads();
        }
        // accT(a, c) += sum_rows U(row, a) W(row, c)
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int lrow = rc0 + wave * 64 + mt * 16 + d_row(lane, v);
#pragma unroll
                for (int at = 0; at < NT; ++at) {
                    const int acol = at * 16 + (lane & 15);
                    double ua = 0.0;
                    if (lrow < mi && acol < k) ua = U[ri0 + lrow + static_cast<int64_t>(acol) * ldUV];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) accT[at][nt] = mfma64(ua, acc[mt][nt][v], accT[at][nt]);
                }
            }
    }
    // reduce the four waves' partial products in a fixed order
    for (int w = 0; w < 4; ++w) {
        if (wave == w) {
#pragma unroll
            for (int at = 0; at < NT; ++at)
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                    for (int v = 0; v < 4; ++v) {
                        const int idx = (at * 16 + d_row(lane, v)) + (nt * 16 + d_col(lane)) * KP;
                        sA[idx] = (w == 0 ? 0.0 : sA[idx]) + accT[at][nt][v];
                    }
        }
        __syncthreads();
    }
    for (int idx = tid; idx < k * k; idx += 256) {
        const int a = idx % k, c = idx / k;
        Atil[(static_cast<int64_t>(i) * k + a) + (static_cast<int64_t>(j) * k + c) * ldAt] = sA[a + c * KP];
    }
}

// Cores for a symmetric operator (A_ji = A_ij^T): one workgroup per unordered pair i <= j
// generates A_ij once and multiplies it by [V_j | U_j]; then
//   Atil_ij = U_i^T (A_ij V_j)   and   Atil_ji = (V_i^T (A_ij U_j))^T,
// the second only for i < j.  Same MFMA scheme as k_cores with 2*NT column tiles.
template <class AS, int NT>
__global__ __launch_bounds__(256, 2) void k_cores_sym(
    AS A, const int64_t* __restrict__ box_ptr, const double* __restrict__ U,
    const double* __restrict__ V, int64_t ldUV, int k, double* __restrict__ Atil, int64_t ldAt) {
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    A.prepare((BLR_LDS double*)s_ltab);
    __syncthreads();
    constexpr int KT = 16, RC = 256, KP = NT * 16, NT2 = 2 * NT;
    __shared__ double sA[KT * RC];
    __shared__ double sV[KT * 2 * KP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x, i = blockIdx.y;
    if (i > j) return;
    const int64_t ri0 = box_ptr[i], cj0 = box_ptr[j];
    const int mi = static_cast<int>(box_ptr[i + 1] - ri0);
    const int mj = static_cast<int>(box_ptr[j + 1] - cj0);
    d4 accT[2][NT][NT];
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
        for (int at = 0; at < NT; ++at)
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) accT[h][at][nt] = d4{0.0, 0.0, 0.0, 0.0};

    for (int rc0 = 0; rc0 < mi; rc0 += RC) {
        const int grow = rc0 + tid;
        const bool rowok = grow < mi;
        const auto rp = A.row(ri0 + (rowok ? grow : 0));
        d4 acc[4][NT2];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int nt = 0; nt < NT2; ++nt) acc[mt][nt] = d4{0.0, 0.0, 0.0, 0.0};
        // a whole step of an off-diagonal pair needs neither the column bound nor the diagonal
        // rule; rows past the box repeat its first point (finite entries, and their products
        // meet zero rows of U and V below)
        const bool offdiag = i != j;
        for (int k0 = 0; k0 < mj; k0 += KT) {
            if (offdiag && k0 + KT <= mj) {
#pragma unroll 4
                for (int kk = 0; kk < KT; ++kk) sA[kk * RC + tid] = A.val_off(rp, A.col(cj0 + k0 + kk));
            } else {
#pragma unroll 4
                for (int kk = 0; kk < KT; ++kk) {
                    double v = 0.0;
                    if (rowok && k0 + kk < mj) v = A.val(rp, A.col(cj0 + k0 + kk));
                    sA[kk * RC + tid] = v;
                }
            }
            for (int idx = tid; idx < KT * 2 * KP; idx += 256) {
                const int kk = idx / (2 * KP), cc = idx - kk * 2 * KP;
                const int h = cc / KP, c = cc - h * KP;
                double v = 0.0;
                if (k0 + kk < mj && c < k) v = (h ? U : V)[cj0 + k0 + kk + static_cast<int64_t>(c) * ldUV];
                sV[idx] = v;
            }
            __syncthreads();
#pragma unroll
            for (int ks = 0; ks < KT / 4; ++ks) {
                const int kr = ks * 4 + (lane >> 4);
                double a[4], bb[NT2];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt) a[mt] = sA[kr * RC + wave * 64 + mt * 16 + (lane & 15)];
#pragma unroll
                for (int nt = 0; nt < NT2; ++nt) bb[nt] = sV[kr * 2 * KP + nt * 16 + (lane & 15)];
#pragma unroll
                for (int mt = 0; mt < 4; ++mt)
#pragma unroll
                    for (int nt = 0; nt < NT2; ++nt) acc[mt][nt] = mfma64(a[mt], bb[nt], acc[mt][nt]);
            }
            __syncthreads();
        }
        // accT[0](a, c) += sum_rows U_i(row, a) (A V_j)(row, c); accT[1] with V_i and A U_j
#pragma unroll
        for (int mt = 0; mt < 4; ++mt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int lrow = rc0 + wave * 64 + mt * 16 + d_row(lane, v);
#pragma unroll
                for (int at = 0; at < NT; ++at) {
                    const int acol = at * 16 + (lane & 15);
                    double ua = 0.0, va = 0.0;
                    if (lrow < mi && acol < k) {
                        ua = U[ri0 + lrow + static_cast<int64_t>(acol) * ldUV];
                        va = V[ri0 + lrow + static_cast<int64_t>(acol) * ldUV];
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        accT[0][at][nt] = mfma64(ua, acc[mt][nt][v], accT[0][at][nt]);
                        accT[1][at][nt] = mfma64(va, acc[mt][NT + nt][v], accT[1][at][nt]);
                    }
                }
            }
    }
    for (int h = 0; h < 2; ++h) {
        for (int w = 0; w < 4; ++w) {
            if (wave == w) {
#pragma unroll
                for (int at = 0; at < NT; ++at)
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                        for (int v = 0; v < 4; ++v) {
                            const int idx = (at * 16 + d_row(lane, v)) + (nt * 16 + d_col(lane)) * KP;
                            sA[idx] = (w == 0 ? 0.0 : sA[idx]) + accT[h][at][nt][v];
                        }
            }
            __syncthreads();
        }
        if (h == 0 || i < j) {
            for (int idx = tid; idx < k * k; idx += 256) {
                const int a = idx % k, c = idx / k;
                if (h == 0)
                    Atil[(static_cast<int64_t>(i) * k + a) + (static_cast<int64_t>(j) * k + c) * ldAt] = sA[a + c * KP];
                else  // Atil_ji(c, a) = (V_i^T A_ij U_j)(a, c)
                    Atil[(static_cast<int64_t>(j) * k + c) + (static_cast<int64_t>(i) * k + a) * ldAt] = sA[a + c * KP];
            }
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------ near field
// Near field in two launches.  k_nf_q: for every (box i, colour c) and probe column col,
//   Qg[(i, c)](col, t) = sum_{l' of colour c, col < m_l'} sum_s V_l'(col, s) Atil(i k + t, l' k + s)
// i.e. Q^T = X_c^T V Atil_{i,:}^T (m_max x KP per pair, zero beyond k).  k_nf_b:
//   B_il(a, col) = sum_{l'} A(I_i[a], I_l'[col]) - sum_t U_i(a, t) Qg(col, t).
template <int KP>
__global__ __launch_bounds__(256) void k_nf_q(const int64_t* __restrict__ box_ptr,
                                              const int32_t* __restrict__ colour_ptr,
                                              const int32_t* __restrict__ colour_boxes,
                                              const int32_t* __restrict__ nf_pair, int ncol,
                                              const double* __restrict__ V, int64_t ldUV,
                                              const double* __restrict__ Atil, int64_t ldAt, int k,
                                              int m_max, double* __restrict__ Qg) {
    __shared__ double sAt[KP * KP];  // sAt[s * KP + t] = Atil(i k + t, l' k + s)
    const int tid = threadIdx.x;
    const int pair = blockIdx.x;  // (i, c)
    const int i = pair / ncol, c = pair - (pair / ncol) * ncol;
    if (nf_pair[pair] < 0) return;
    const int cb0 = colour_ptr[c], cb1 = colour_ptr[c + 1];
    double* Q = Qg + static_cast<int64_t>(pair) * m_max * KP;
    for (int col0 = 0; col0 < m_max; col0 += 256) {
        const int col = col0 + tid;
        double q[KP];
#pragma unroll
        for (int t = 0; t < KP; ++t) q[t] = 0.0;
#pragma unroll 1
        for (int qq = cb0; qq < cb1; ++qq) {
            const int lp = colour_boxes[qq];
            const int64_t lp0 = box_ptr[lp];
            const int mlp = static_cast<int>(box_ptr[lp + 1] - lp0);
            __syncthreads();
            for (int idx = tid; idx < KP * KP; idx += 256) {
                const int t = idx % KP, sx = idx / KP;
                sAt[idx] = (t < k && sx < k)
                    ? Atil[(static_cast<int64_t>(i) * k + t) + (static_cast<int64_t>(lp) * k + sx) * ldAt] : 0.0;
            }
            __syncthreads();
            if (col < mlp) {
#pragma unroll 1
                for (int sx = 0; sx < k; ++sx) {
                    const double v = V[lp0 + col + static_cast<int64_t>(sx) * ldUV];
                    const double* at = sAt + sx * KP;
#pragma unroll
                    for (int t = 0; t < KP; ++t) q[t] += at[t] * v;
                }
            }
        }
        if (col < m_max) {
#pragma unroll
            for (int t = 0; t < KP; ++t) Q[static_cast<int64_t>(col) * KP + t] = q[t];
        }
    }
}

template <class AS, int KP>
__global__ __launch_bounds__(256) void k_nf_b(
    AS A, const int64_t* __restrict__ box_ptr, const int32_t* __restrict__ near_idx,
    const int64_t* __restrict__ b_off, const int32_t* __restrict__ colour_ptr,
    const int32_t* __restrict__ colour_boxes, const int32_t* __restrict__ nf_pair, int ncol,
    const double* __restrict__ U, int64_t ldUV, int k, int m_max, const double* __restrict__ Qg,
    double* __restrict__ Bv) {
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    A.prepare((BLR_LDS double*)s_ltab);
    __syncthreads();
    constexpr int CW = 16, NB = 32;
    __shared__ double scol[NB * CW * AS::STAGE];
    __shared__ int64_t sidx[NB * CW];
    __shared__ int svalid[NB * CW];
    __shared__ int sfull[NB];          // box bq of the block: another box, all CW columns valid
    __shared__ double sQ[CW * KP];
    const int tid = threadIdx.x;
    const int pair = blockIdx.x;
    const int i = pair / ncol, c = pair - (pair / ncol) * ncol;
    const int p = nf_pair[pair];
    if (p < 0) return;
    const int l = near_idx[p];
    const int64_t ri0 = box_ptr[i];
    const int mi = static_cast<int>(box_ptr[i + 1] - ri0);
    const int ml = static_cast<int>(box_ptr[l + 1] - box_ptr[l]);
    double* Bout = Bv + b_off[p];
    const int cb0 = colour_ptr[c], cb1 = colour_ptr[c + 1];
    const double* Q = Qg + static_cast<int64_t>(pair) * m_max * KP;
#pragma unroll 1
    for (int col0 = 0; col0 < ml; col0 += CW) {
        const int ncw = min(CW, ml - col0);
        __syncthreads();
        for (int e = tid; e < CW * KP; e += 256) {
            const int cc = e / KP;
            sQ[e] = (col0 + cc < m_max) ? Q[static_cast<int64_t>(col0) * KP + e] : 0.0;
        }
#pragma unroll 1
        for (int a0 = 0; a0 < mi; a0 += 256) {
            const int arow = a0 + tid;
            const bool rowok = arow < mi;
            const auto rp = A.row(ri0 + (rowok ? arow : 0));
            double acc[CW];
#pragma unroll
            for (int cc = 0; cc < CW; ++cc) acc[cc] = 0.0;
#pragma unroll 1
            for (int qb = cb0; qb < cb1; qb += NB) {
                const int nbq = min(NB, cb1 - qb);
                __syncthreads();
                for (int e = tid; e < nbq * CW; e += 256) {
                    const int bq = e / CW, cc = e - bq * CW;
                    const int lp = colour_boxes[qb + bq];
                    const int64_t lp0 = box_ptr[lp];
                    const int mlp = static_cast<int>(box_ptr[lp + 1] - lp0);
                    const bool ok = col0 + cc < mlp;
                    const int64_t j = lp0 + (ok ? col0 + cc : 0);
                    A.stage(j, scol + e * AS::STAGE);
                    sidx[e] = j;
                    svalid[e] = ok ? 1 : 0;
                    if (cc == 0) sfull[bq] = (lp != i && col0 + CW <= mlp) ? 1 : 0;
                }
                __syncthreads();
#pragma unroll 1
                for (int bq = 0; bq < nbq; ++bq) {
                    if (__builtin_amdgcn_readfirstlane(sfull[bq])) {
                        // another box and every column in it: no diagonal rule, no masking
#pragma unroll
                        for (int cc = 0; cc < CW; ++cc) {
                            const int e = bq * CW + cc;
                            acc[cc] += A.val_off(rp, A.col_staged(scol + e * AS::STAGE, sidx[e]));
                        }
                    } else {
#pragma unroll
                        for (int cc = 0; cc < CW; ++cc) {
                            const int e = bq * CW + cc;
                            const double v = A.val(rp, A.col_staged(scol + e * AS::STAGE, sidx[e]));
                            acc[cc] += svalid[e] ? v : 0.0;
                        }
                    }
                }
            }
            if (rowok) {
                const double* ur = U + ri0 + arow;
#pragma unroll 8
                for (int t = 0; t < k; ++t) {
                    const double u = ur[static_cast<int64_t>(t) * ldUV];
#pragma unroll
                    for (int cc = 0; cc < CW; ++cc) acc[cc] -= u * sQ[cc * KP + t];
                }
#pragma unroll
                for (int cc = 0; cc < CW; ++cc)
                    if (cc < ncw) Bout[arow + static_cast<int64_t>(col0 + cc) * mi] = acc[cc];
            }
        }
    }
}

// The same Q products on FP64 MFMA, for boxes of at most 16 RTW rows: the workgroup stages the
// k x k block Atil(i, l') of each box l' of the colour in LDS (B operand, transposed) and
// contracts it with V_l' read straight from HBM (A operand: 16 probe columns x 4 basis
// columns per lane group); wave w owns the 16-row tiles w, w + 4, ... of Q and all its
// KP / 16 column tiles, accumulated over the whole colour class.
template <int RTW, int NTT>
__global__ __launch_bounds__(256) void k_nf_q_m(const int64_t* __restrict__ box_ptr,
                                                const int32_t* __restrict__ colour_ptr,
                                                const int32_t* __restrict__ colour_boxes,
                                                const int32_t* __restrict__ nf_pair, int ncol,
                                                const double* __restrict__ V, int64_t ldUV,
                                                const double* __restrict__ Atil, int64_t ldAt, int k,
                                                int m_max, double* __restrict__ Qg) {
    constexpr int KP = NTT * 16, SP = KP + 1;
    __shared__ double sAt[KP * SP];  // sAt[s * SP + t] = Atil(i k + t, l' k + s), zero past k
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int pair = blockIdx.x;
    const int i = pair / ncol, c = pair - (pair / ncol) * ncol;
    if (nf_pair[pair] < 0) return;
    const int cb0 = colour_ptr[c], cb1 = colour_ptr[c + 1];
    const int nrt = (m_max + 15) / 16;
    d4 acc[RTW][NTT];
#pragma unroll
    for (int rr = 0; rr < RTW; ++rr)
#pragma unroll
        for (int nt = 0; nt < NTT; ++nt) acc[rr][nt] = d4{0.0, 0.0, 0.0, 0.0};
    const int srow = lane >> 4, lcol = lane & 15;
#pragma unroll 1
    for (int qq = cb0; qq < cb1; ++qq) {
        const int lp = colour_boxes[qq];
        const int64_t lp0 = box_ptr[lp];
        const int mlp = static_cast<int>(box_ptr[lp + 1] - lp0);
        __syncthreads();
        for (int idx = tid; idx < KP * KP; idx += 256) {
            const int t = idx % KP, sx = idx / KP;
            sAt[sx * SP + t] = (t < k && sx < k)
                ? Atil[(static_cast<int64_t>(i) * k + t) + (static_cast<int64_t>(lp) * k + sx) * ldAt] : 0.0;
        }
        __syncthreads();
        // V_lp operands are loaded one 4-deep slice ahead of the MFMAs that use them
        auto load_v = [&](double* a, int s0) {
            const int s2 = s0 + srow;
#pragma unroll
            for (int rr = 0; rr < RTW; ++rr) {
                const int col = (wave + 4 * rr) * 16 + lcol;
                a[rr] = (wave + 4 * rr < nrt && col < mlp && s2 < k)
                    ? V[lp0 + col + static_cast<int64_t>(s2) * ldUV] : 0.0;
            }
        };
        double an[RTW];
        load_v(an, 0);
        for (int s0 = 0; s0 < k; s0 += 4) {
            const int s2 = s0 + srow;                    // < KP: KP is a multiple of 16 >= k
            double a[RTW];
#pragma unroll
            for (int rr = 0; rr < RTW; ++rr) a[rr] = an[rr];
            if (s0 + 4 < k) load_v(an, s0 + 4);
            double bb[NTT];
#pragma unroll
            for (int nt = 0; nt < NTT; ++nt) bb[nt] = sAt[s2 * SP + nt * 16 + lcol];
#pragma unroll
            for (int rr = 0; rr < RTW; ++rr) {
                const int rt = wave + 4 * rr;
                if (rt >= nrt) continue;                 // uniform over the wave
#pragma unroll
                for (int nt = 0; nt < NTT; ++nt) acc[rr][nt] = mfma64(a[rr], bb[nt], acc[rr][nt]);
            }
        }
    }
    double* Q = Qg + static_cast<int64_t>(pair) * m_max * KP;
#pragma unroll
    for (int rr = 0; rr < RTW; ++rr) {
        const int rt = wave + 4 * rr;
        if (rt >= nrt) continue;
#pragma unroll
        for (int nt = 0; nt < NTT; ++nt)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int col = rt * 16 + d_row(lane, v);
                if (col < m_max) Q[static_cast<int64_t>(col) * KP + nt * 16 + d_col(lane)] = acc[rr][nt][v];
            }
    }
}

// out[idx] = sum_s part[s len + idx]: 64 outputs per workgroup; the four waves take every
// fourth split and their sums meet in LDS.
__global__ __launch_bounds__(256) void k_sum_parts(const double* __restrict__ part, int nsplit,
                                                   int64_t len, double* __restrict__ out) {
    __shared__ double red[256];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 64 + lane;
    double acc = 0.0;
    if (idx < len) {
#pragma unroll 8
        for (int s2 = wave; s2 < nsplit; s2 += 4) acc += part[static_cast<int64_t>(s2) * len + idx];
    }
    red[tid] = acc;
    __syncthreads();
    if (wave == 0 && idx < len) out[idx] = red[lane] + red[64 + lane] + red[128 + lane] + red[192 + lane];
}

// out(col_idx, col) = sum_row Atil(row, col_idx) t(row, col): one wave per output
__global__ __launch_bounds__(256) void k_gemv_t(const double* __restrict__ At, int64_t ld,
                                                int64_t bk, const double* __restrict__ t,
                                                double* __restrict__ out) {
    const int lane = threadIdx.x & 63;
    const int64_t c = static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6);
    const int col = blockIdx.y;
    if (c >= bk) return;
    const double* a = At + c * ld;
    const double* tc = t + static_cast<int64_t>(col) * bk;
    double acc = 0.0;
    for (int64_t q = lane; q < bk; q += 64) acc += a[q] * tc[q];
    acc = wave_sum(acc);
    if (lane == 0) out[c + static_cast<int64_t>(col) * bk] = acc;
}


// Multi-vector forms of the uBLR apply.  Vectors go in groups of NC; each kernel stages the
// small per-group operand (t or x) in LDS so every value of Atil, B, U or V read from HBM
// serves all NC vectors.

// t(j k + s, col) = sum_a S(I_j[a], s) x(I_j[a], col): one workgroup per (box j, vector
// group); rows of S_j and x_j staged in 32-row chunks, thread o owns outputs o + 256 u.
template <int NC>
__global__ __launch_bounds__(256) void k_proj_nc(const double* __restrict__ S, int64_t ldS,
                                                 const int64_t* __restrict__ box_ptr, int k,
                                                 const double* __restrict__ x, int64_t ldx, int ncols,
                                                 double* __restrict__ t, int64_t bk) {
    constexpr int RC = 32, SP = 65;
    __shared__ double sS[RC * SP];
    __shared__ double sX[RC * NC];
    const int tid = threadIdx.x;
    const int j = blockIdx.x, col0 = blockIdx.y * NC;
    const int nc = min(NC, ncols - col0);
    const int64_t r0 = box_ptr[j];
    const int m = static_cast<int>(box_ptr[j + 1] - r0);
    const int nout = k * NC;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a0 = 0; a0 < m; a0 += RC) {
        const int rows = min(RC, m - a0);
        __syncthreads();
        for (int e = tid; e < RC * k; e += 256) {
            const int rr = e % RC, s2 = e / RC;
            sS[rr * SP + s2] = rr < rows ? S[r0 + a0 + rr + static_cast<int64_t>(s2) * ldS] : 0.0;
        }
        for (int e = tid; e < RC * NC; e += 256) {
            const int rr = e % RC, v = e / RC;
            sX[rr * NC + v] = (rr < rows && v < nc) ? x[r0 + a0 + rr + static_cast<int64_t>(col0 + v) * ldx] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int o = tid + 256 * u;
            if (o < nout) {
                const int s2 = o % k, v = o / k;
#pragma unroll 8
                for (int rr = 0; rr < RC; ++rr) acc[u] = fma(sS[rr * SP + s2], sX[rr * NC + v], acc[u]);
            }
        }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int o = tid + 256 * u;
        if (o < nout) {
            const int s2 = o % k, v = o / k;
            if (v < nc) t[static_cast<int64_t>(j) * k + s2 + static_cast<int64_t>(col0 + v) * bk] = acc[u];
        }
    }
}

// part[split][row + col*bk] = sum over one column chunk of Atil(row, cc) t(cc, col) for the
// vectors of group blockIdx.z.  Each thread owns rows row0 and row0 + 256 of a 512-row block;
// the chunk of t (chunk x NC <= 4096 values) sits in dynamic LDS.
template <int NC>
__global__ __launch_bounds__(256) void k_gemv_nc(const double* __restrict__ At, int64_t ld, int64_t bk,
                                                 const double* __restrict__ t, int ncols,
                                                 double* __restrict__ part, int chunk) {
    extern __shared__ double st[];                      // chunk x NC values
    const int tid = threadIdx.x;
    const int split = blockIdx.y, col0 = blockIdx.z * NC;
    const int nc = min(NC, ncols - col0);
    const int64_t c0 = static_cast<int64_t>(split) * chunk;
    const int len = static_cast<int>(max<int64_t>(0, min<int64_t>(bk - c0, chunk)));
    for (int e = tid; e < len * NC; e += 256) {
        const int cc = e % len, v = e / len;
        st[cc * NC + v] = v < nc ? t[c0 + cc + static_cast<int64_t>(col0 + v) * bk] : 0.0;
    }
    __syncthreads();
    const int64_t row0 = static_cast<int64_t>(blockIdx.x) * 512 + tid;
    const int64_t row1 = row0 + 256;
    const int64_t ra = row0 < bk ? row0 : bk - 1, rb = row1 < bk ? row1 : bk - 1;
    const double* a = At + c0 * ld;
    double acc0[NC], acc1[NC];
#pragma unroll
    for (int v = 0; v < NC; ++v) acc0[v] = acc1[v] = 0.0;
#pragma unroll 4
    for (int cc = 0; cc < len; ++cc) {
        const double x0 = a[ra + static_cast<int64_t>(cc) * ld];
        const double x1 = a[rb + static_cast<int64_t>(cc) * ld];
#pragma unroll
        for (int v = 0; v < NC; ++v) {
            const double tv = st[cc * NC + v];
            acc0[v] = fma(x0, tv, acc0[v]);
            acc1[v] = fma(x1, tv, acc1[v]);
        }
    }
#pragma unroll
    for (int v = 0; v < NC; ++v) {
        if (v >= nc) continue;
        double* out = part + (static_cast<int64_t>(split) * ncols + col0 + v) * bk;
        if (row0 < bk) out[row0] = acc0[v];
        if (row1 < bk) out[row1] = acc1[v];
    }
}

// y(I_i, col) = U_i t(i-block, col) + sum over the neighbours j of i of B_ij x(I_j, col).
// One workgroup per (box i, vector group, 64-row slice of I_i); lane = row, so each column of
// U_i and B_ij is read as one coalesced 512-byte segment.  The terms (U_i first, then the
// neighbours in list order) go through LDS in chunks of up to 256 columns whose x values are
// staged there; the four waves split each chunk's columns and their sums meet in LDS.
template <int NC>
__global__ __launch_bounds__(256) void k_near_out_n(const double* __restrict__ U, int64_t ldU,
                                                    const int64_t* __restrict__ box_ptr, int k,
                                                    const double* __restrict__ t2, int64_t bk,
                                                    const int32_t* __restrict__ near_ptr,
                                                    const int32_t* __restrict__ near_idx,
                                                    const int64_t* __restrict__ b_off,
                                                    const double* __restrict__ Bv,
                                                    const double* __restrict__ x, int64_t ldx, int ncols,
                                                    double* __restrict__ y, int64_t ldy) {
    constexpr int CH = 256, SP = NC == 1 ? 1 : NC + 1;   // padded rows: conflict-free staging
    __shared__ double sx[CH * SP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int i = blockIdx.x, col0 = blockIdx.y * NC, slice = blockIdx.z;
    const int nc = min(NC, ncols - col0);
    const int64_t r0 = box_ptr[i];
    const int mi = static_cast<int>(box_ptr[i + 1] - r0);
    if (slice * 64 >= mi) return;                      // uniform over the workgroup
    const int a = slice * 64 + lane;
    const int arow = a < mi ? a : mi - 1;              // clamped row for the loads
    double acc[NC];
#pragma unroll
    for (int v = 0; v < NC; ++v) acc[v] = 0.0;
    const int q0 = near_ptr[i], q1 = near_ptr[i + 1];
    for (int item = q0 - 1; item < q1; ++item) {
        const double* M;
        const double* xs;
        int64_t ldm, ldxs;
        int len;
        if (item < q0) {
            M = U + r0;
            ldm = ldU;
            len = k;
            xs = t2 + static_cast<int64_t>(i) * k;
            ldxs = bk;
        } else {
            const int j = near_idx[item];
            const int64_t j0 = box_ptr[j];
            M = Bv + b_off[item];
            ldm = mi;
            len = static_cast<int>(box_ptr[j + 1] - j0);
            xs = x + j0;
            ldxs = ldx;
        }
        for (int c0 = 0; c0 < len; c0 += CH) {
            const int cl = min(CH, len - c0);
            __syncthreads();
            if (tid < cl) {
#pragma unroll
                for (int v = 0; v < NC; ++v)
                    sx[tid * SP + v] = v < nc ? xs[c0 + tid + static_cast<int64_t>(col0 + v) * ldxs] : 0.0;
            }
            __syncthreads();
            const int cq = (cl + 3) / 4;
            const int cb = wave * cq, ce = min(cl, cb + cq);
            const double* pm = M + static_cast<int64_t>(c0 + cb) * ldm + arow;
#pragma unroll 4
            for (int cc = cb; cc < ce; ++cc, pm += ldm) {
                const double bval = *pm;
#pragma unroll
                for (int v = 0; v < NC; ++v) acc[v] = fma(bval, sx[cc * SP + v], acc[v]);
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NC; ++v) sx[v * 256 + tid] = acc[v];
    __syncthreads();
    if (wave == 0 && a < mi) {
#pragma unroll
        for (int v = 0; v < NC; ++v)
            if (v < nc)
                y[r0 + a + static_cast<int64_t>(col0 + v) * ldy] =
                    sx[v * 256 + lane] + sx[v * 256 + 64 + lane] + sx[v * 256 + 128 + lane] + sx[v * 256 + 192 + lane];
    }
}

// Output stage of the apply for a group of 16 vectors, on FP64 MFMA.  Output box o = blockIdx.x,
// 64-row slice blockIdx.z; wave w owns output rows 16 w .. 16 w + 15 of the slice and all
// columns of every term, so no partial sums cross waves.
//   trans = 0: y(I_o) = U_o t2(o-block) + sum_{j in N(o)} B_oj x(I_j)
//   trans = 1: y(I_o) = V_o t2(o-block) + sum_{i in N(o)} B_io^T x(I_i)
// A term is a matrix M whose element (output row r, inner index c) sits at M[r rs + c ks]
// (rs = 1 for U, V and B_oj; rs = m_i, ks = 1 for B_io^T).  A operand = M's 16 x 4 block
// (lane l: row l % 16, inner index l / 16), B operand = the staged x rows (4 x 16), zero
// beyond the term's inner length.
template <int TRANS>
__global__ __launch_bounds__(256) void k_near_m16(const double* __restrict__ S, int64_t ldS,
                                                  const int64_t* __restrict__ box_ptr, int k,
                                                  const double* __restrict__ t2, int64_t bk,
                                                  const int32_t* __restrict__ near_ptr,
                                                  const int32_t* __restrict__ near_idx,
                                                  const int32_t* __restrict__ near_tpos,
                                                  const int64_t* __restrict__ b_off,
                                                  const double* __restrict__ Bv,
                                                  const double* __restrict__ x, int64_t ldx, int ncols,
                                                  double* __restrict__ y, int64_t ldy) {
    constexpr int CH = 128, NC = 16, SP = NC + 1;     // padded rows: conflict-free staging
    __shared__ double sx[CH * SP];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int o = blockIdx.x, col0 = blockIdx.y * NC, slice = blockIdx.z;
    const int nc = min(NC, ncols - col0);
    const int64_t r0 = box_ptr[o];
    const int mo = static_cast<int>(box_ptr[o + 1] - r0);
    if (slice * 64 >= mo) return;                      // uniform over the workgroup
    const int arow_l = slice * 64 + wave * 16 + (lane & 15);
    const int arow = arow_l < mo ? arow_l : mo - 1;    // rows past the box: clamped, never written
    const int kq = lane >> 4, col = lane & 15;
    d4 acc = {0.0, 0.0, 0.0, 0.0}, acc2 = {0.0, 0.0, 0.0, 0.0};
    const int q0 = near_ptr[o], q1 = near_ptr[o + 1];
    for (int item = q0 - 1; item < q1; ++item) {
        const double* M;
        const double* xs;
        int64_t rs, ks, ldxs;
        int len;
        if (item < q0) {
            M = S + r0;
            rs = 1;
            ks = ldS;
            len = k;
            xs = t2 + static_cast<int64_t>(o) * k;
            ldxs = bk;
        } else {
            const int j = near_idx[item];
            const int64_t j0 = box_ptr[j];
            const int mj = static_cast<int>(box_ptr[j + 1] - j0);
            if (TRANS) {
                M = Bv + b_off[near_tpos[item]];       // B_jo, m_j x m_o
                rs = mj;
                ks = 1;
            } else {
                M = Bv + b_off[item];                  // B_oj, m_o x m_j
                rs = 1;
                ks = mo;
            }
            len = mj;
            xs = x + j0;
            ldxs = ldx;
        }
        const double* Mr = M + static_cast<int64_t>(arow) * rs;
        for (int c0 = 0; c0 < len; c0 += CH) {
            const int cl = min(CH, len - c0);
            const int cl4 = (cl + 3) & ~3;
            __syncthreads();
            {
                const int cc = tid & (CH - 1);
                if (cc < cl4)
                    for (int v = tid >> 7; v < NC; v += 2)
                        sx[cc * SP + v] = (cc < cl && v < nc) ? xs[c0 + cc + static_cast<int64_t>(col0 + v) * ldxs] : 0.0;
            }
            __syncthreads();
            // Eight loads are issued before their MFMAs (two accumulators, steps alternating).
            // Inner indices past the term read a clamped in-range entry; their staged x rows are zero.
            const int64_t step4 = 4 * ks;
            const double* pa = Mr + static_cast<int64_t>(c0 + kq) * ks;
            int cc = 0;
            for (; cc + 32 <= cl; cc += 32) {
                double av[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) av[u] = pa[u * step4];
#pragma unroll
                for (int u = 0; u < 8; u += 2) {
                    acc = mfma64(av[u], sx[(cc + 4 * u + kq) * SP + col], acc);
                    acc2 = mfma64(av[u + 1], sx[(cc + 4 * u + 4 + kq) * SP + col], acc2);
                }
                pa += 8 * step4;
            }
            for (; cc + 4 <= cl; cc += 4, pa += step4) acc = mfma64(pa[0], sx[(cc + kq) * SP + col], acc);
            if (cc < cl4) {
                const int c = cc + kq;
                const double av = Mr[static_cast<int64_t>(c0 + (c < cl ? c : cl - 1)) * ks];
                acc = mfma64(av, sx[c * SP + col], acc);
            }
        }
    }
    const int dcol = d_col(lane);
    if (dcol < nc) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int a = slice * 64 + wave * 16 + d_row(lane, v);
            if (a < mo) y[r0 + a + static_cast<int64_t>(col0 + dcol) * ldy] = acc[v] + acc2[v];
        }
    }
}

// ------------------------------------------------------------ exact error
template <class AS>
__global__ __launch_bounds__(256) void k_err_fro(AS A, const int64_t* __restrict__ box_ptr,
                                                 const int32_t* __restrict__ near_ptr,
                                                 const int32_t* __restrict__ near_idx,
                                                 const int64_t* __restrict__ b_off,
                                                 const double* __restrict__ U,
                                                 const double* __restrict__ V, int64_t ldUV,
                                                 const double* __restrict__ Atil, int64_t ldAt,
                                                 int k, const double* __restrict__ Bv,
                                                 double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    A.prepare((BLR_LDS double*)s_ltab);
    __syncthreads();
    constexpr int CH = 64;
    __shared__ double sV[CH * 64];
    __shared__ double red[2][4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int j = blockIdx.x, i = blockIdx.y;
    const int64_t ri0 = box_ptr[i], cj0 = box_ptr[j];
    const int mi = static_cast<int>(box_ptr[i + 1] - ri0);
    const int mj = static_cast<int>(box_ptr[j + 1] - cj0);
    int p = -1;
    for (int q = near_ptr[i]; q < near_ptr[i + 1]; ++q)
        if (near_idx[q] == j) p = q;
    double se = 0.0, sa = 0.0;
    for (int a0 = 0; a0 < mi; a0 += 256) {
        const int a = a0 + tid;
        const bool ok = a < mi;
        double w[64];
#pragma unroll
        for (int t = 0; t < 64; ++t) {
            double acc = 0.0;
            if (ok && t < k)
                for (int s = 0; s < k; ++s)
                    acc += U[ri0 + a + static_cast<int64_t>(s) * ldUV] *
                           Atil[(static_cast<int64_t>(i) * k + s) + (static_cast<int64_t>(j) * k + t) * ldAt];
            w[t] = acc;
        }
        const auto rp = A.row(ri0 + (ok ? a : 0));
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
                    for (int t = 0; t < 64; ++t) rec += w[t] * sV[cc * 64 + t];
                    const double av = A.val(rp, A.col(cj0 + c0 + cc));
                    double e = av - rec;
                    if (p >= 0) e -= Bv[b_off[p] + a + static_cast<int64_t>(c0 + cc) * mi];
                    se += e * e;
                    sa += av * av;
                }
            }
            __syncthreads();
        }
    }
    se = wave_sum(se);
    sa = wave_sum(sa);
    if (lane == 0) {
        red[0][wave] = se;
        red[1][wave] = sa;
    }
    __syncthreads();
    if (tid == 0) {
        const int64_t pr = static_cast<int64_t>(i) * gridDim.x + j;
        part[2 * pr] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
        part[2 * pr + 1] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
    }
}

// ------------------------------------------------------------ small BLAS-1
constexpr int kDotBlocks = 512;

__global__ __launch_bounds__(256) void k_dot_stage1(const double* __restrict__ x,
                                                    const double* __restrict__ y, int64_t n,
                                                    double* __restrict__ part) {
    __shared__ double red[4];
    double acc = 0.0;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; q < n;
         q += static_cast<int64_t>(gridDim.x) * 256)
        acc += x[q] * y[q];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) part[1 + blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(64) void k_dot_stage2(double* part, int nb) {
    double acc = 0.0;
    for (int q = threadIdx.x; q < nb; q += 64) acc += part[1 + q];
    acc = wave_sum(acc);
    if (threadIdx.x == 0) part[0] = acc;
}

__global__ __launch_bounds__(256) void k_axpy(double a, const double* __restrict__ x,
                                              double* __restrict__ y, int64_t n) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (q < n) y[q] += a * x[q];
}

__global__ __launch_bounds__(256) void k_scale(double a, double* __restrict__ x, int64_t n) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (q < n) x[q] *= a;
}

}  // namespace

// ============================================================ launchers

void launch_sketch(const OpData& op, const PlanData& P, const DeviceTables& t, const double* G,
                   const double* H, double* Y, double* Z, hipStream_t s) {
    if (op.type == OpType::Kernel) {
        // A* = A: one pass over A serves Omega and Psi.
        with_source(op, 0, [&](auto A) { sketch_launch(A, P, t, G, H, 2, Y, Z, s); });
    } else {
        with_source(op, 0, [&](auto A) { sketch_launch(A, P, t, G, G, 1, Y, Y, s); });
        with_source(op, 1, [&](auto A) { sketch_launch(A, P, t, H, H, 1, Z, Z, s); });
    }
}

void launch_refine(const OpData& op, const PlanData& P, const DeviceTables& t, const double* X0,
                   const double* X1, double* S0, double* S1, hipStream_t s) {
    if (op.type == OpType::Kernel) {
        with_source(op, 0, [&](auto A) { refine_launch(A, P, t, X0, X1, 2, S0, S1, s); });
    } else {
        with_source(op, 0, [&](auto A) { refine_launch(A, P, t, X0, X0, 1, S0, S0, s); });
        with_source(op, 1, [&](auto A) { refine_launch(A, P, t, X1, X1, 1, S1, S1, s); });
    }
}

// Products with at most four columns on kernel-matrix operators: the matrix cores would
// idle on 16-column tiles, so each thread owns one target row and accumulates entry times
// x on the vector ALU, the source range split over gridDim.y workgroups whose partial sums
// a second kernel adds in split order.  Source contexts and x rows are staged in LDS in
// chunks of 256 and read as broadcasts.
template <class AS, int NC>
__global__ __launch_bounds__(256) void k_opgemv(AS A, const double* __restrict__ X, int64_t ldx, int ncols,
                                                int64_t M, int64_t K, int64_t chunk, double* __restrict__ part) {
    __shared__ __attribute__((aligned(16))) double s_ltab[256];
    A.prepare((BLR_LDS double*)s_ltab);
    constexpr int ST = AS::STAGE;
    __shared__ double sc[256 * ST];
    __shared__ double sx[256 * NC];
    const int tid = threadIdx.x;
    const int64_t i = static_cast<int64_t>(blockIdx.x) * 256 + tid;
    const bool rowok = i < M;
    const auto rp = A.row(rowok ? i : M - 1);
    const int64_t k0 = static_cast<int64_t>(blockIdx.y) * chunk;
    const int64_t k1 = min(K, k0 + chunk);
    double acc[NC];
#pragma unroll
    for (int v = 0; v < NC; ++v) acc[v] = 0.0;
    for (int64_t c0 = k0; c0 < k1; c0 += 256) {
        const int cl = static_cast<int>(min<int64_t>(256, k1 - c0));
        __syncthreads();
        if (tid < cl) {
            A.stage(c0 + tid, &sc[tid * ST]);
#pragma unroll
            for (int v = 0; v < NC; ++v) sx[tid * NC + v] = v < ncols ? X[c0 + tid + static_cast<int64_t>(v) * ldx] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int u = 0; u < cl; ++u) {
            const double a = A.val(rp, A.col_staged(&sc[u * ST], c0 + u));
#pragma unroll
            for (int v = 0; v < NC; ++v) acc[v] = fma(a, sx[u * NC + v], acc[v]);
        }
    }
    if (rowok) {
#pragma unroll
        for (int v = 0; v < NC; ++v)
            if (v < ncols) part[(static_cast<int64_t>(blockIdx.y) * ncols + v) * M + i] = acc[v];
    }
}

template <class OUT>
__global__ __launch_bounds__(256) void k_opgemv_sum(const double* __restrict__ part, int nsplit, int64_t M,
                                                    int ncols, OUT O) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= M * ncols) return;
    const int v = static_cast<int>(idx / M);
    const int64_t i = idx - static_cast<int64_t>(v) * M;
    double acc = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) acc += part[static_cast<int64_t>(sp) * ncols * M + idx];
    O.put(i, v, acc);
}

// source-range splits of k_opgemv: about eight waves per SIMD at this N
static int opgemv_nsplit(int64_t n) {
    const int64_t rowblocks = (n + 255) / 256;
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(32, (8 * 1024 / 4 + rowblocks - 1) / rowblocks)));
}

int64_t op_apply_workspace_doubles(const OpData& op, int64_t ncols) {
    if (op.type != OpType::Kernel || ncols > 4) return 0;
    return static_cast<int64_t>(opgemv_nsplit(op.n)) * ncols * op.n;
}

void launch_op_apply(const OpData& op, int trans, int64_t ncols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy, double* work, hipStream_t s) {
    if (ncols > (1 << 30)) fail(BLR_ERR_INVALID_ARG, "too many columns");
    SplitOut O{Y, Y, ldy, static_cast<int>(ncols)};
    if (op_apply_workspace_doubles(op, ncols) > 0 && ncols > 0) {
        if (!work) fail(BLR_ERR_INVALID_ARG, "operator product: missing workspace");
        const int ns = opgemv_nsplit(op.n);
        const int64_t chunk = (op.n + ns - 1) / ns;
        const dim3 grid(static_cast<unsigned>((op.n + 255) / 256), ns);
        const int nc = static_cast<int>(ncols);
        with_source(op, trans, [&](auto A) {
            using AS = decltype(A);
            if (nc == 1)
                hipLaunchKernelGGL((k_opgemv<AS, 1>), grid, dim3(256), 0, s, A, X, ldx, nc, op.n, op.n, chunk, work);
            else if (nc == 2)
                hipLaunchKernelGGL((k_opgemv<AS, 2>), grid, dim3(256), 0, s, A, X, ldx, nc, op.n, op.n, chunk, work);
            else
                hipLaunchKernelGGL((k_opgemv<AS, 4>), grid, dim3(256), 0, s, A, X, ldx, nc, op.n, op.n, chunk, work);
        });
        hipLaunchKernelGGL(k_opgemv_sum<SplitOut>, dim3(static_cast<unsigned>((op.n * ncols + 255) / 256)), dim3(256),
                           0, s, work, ns, op.n, nc, O);
        check_launch("operator product (few columns)");
        return;
    }
    DenseB B{X, ldx};
    with_source(op, trans, [&](auto A) { gemm_launch(A, B, O, op.n, op.n, static_cast<int>(ncols), s); });
}

void launch_postprocess(const PlanData& P, const DeviceTables& t, const double* Y, double* Yhat,
                        hipStream_t s) {
    const int64_t total = P.n * P.r;
    hipLaunchKernelGGL(k_postprocess<double>, dim3((total + 255) / 256), dim3(256), 0, s, Y, Yhat, t.z,
                       t.row_box, P.n, P.r, P.ell);
    check_launch("tag post-processing");
}

void launch_postprocess_lp(const PlanData& P, const DeviceTables& t, int r_lo, const float* Y,
                           double* Yhat, hipStream_t s) {
    const int64_t total = P.n * r_lo;
    hipLaunchKernelGGL(k_postprocess<float>, dim3((total + 255) / 256), dim3(256), 0, s, Y, Yhat, t.z,
                       t.row_box, P.n, r_lo, P.ell);
    check_launch("tag post-processing of the low-precision sketch");
}

void launch_orth2(const PlanData& P, const DeviceTables& t, double* S0, double* S1, double* Q0,
                  double* Q1, double* sig0, double* sig1, hipStream_t s) {
    launch_orth_cols(P, t, P.r, P.k, 0, S0, S1, Q0, Q1, sig0, sig1, s);
}

void launch_orth_cols(const PlanData& P, const DeviceTables& t, int r, int k, int qr_only,
                      double* S0, double* S1, double* Q0, double* Q1, double* sig0, double* sig1,
                      hipStream_t s) {
    if (r > 128) fail(BLR_ERR_UNSUPPORTED, "more than 128 sample columns are not supported by the basis kernel");
    if (r > P.m_min) fail(BLR_ERR_UNSUPPORTED, "sample columns exceed the smallest box size");
    if (k > r) fail(BLR_ERR_INVALID_ARG, "more basis columns than sample columns");
    const size_t small = static_cast<size_t>(2) * r * r * sizeof(double);
    const size_t big = static_cast<size_t>(P.m_max) * r * sizeof(double);
    const size_t lds_limit = 160 * 1024 - 4096;  // gfx950: 160 KiB per workgroup, minus statics
    if (small > lds_limit) fail(BLR_ERR_UNSUPPORTED, "k + p too large for the basis kernel");
    // The m x r block goes to LDS only while several workgroups still fit on a CU: with one
    // workgroup per CU (256 x 42 doubles) the barriers of the column loop are exposed, and
    // reading the block through the caches measured 30% faster.
    const int m_in_lds = (small + big <= 40 * 1024) ? 1 : 0;
    const size_t dyn = small + (m_in_lds ? big : 0);
    if (dyn > 64 * 1024) {
        // raise the kernel's dynamic LDS limit once per device and size (not during a
        // stream capture that follows an eager run of the same shapes)
        static std::mutex mu;
        static size_t set_bytes[64] = {};
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lock(mu);
        if (dev < 0 || dev >= 64 || dyn > set_bytes[dev]) {
            hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_orth),
                                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn));
            if (e != hipSuccess) fail(BLR_ERR_DEVICE, std::string("LDS attribute: ") + hipGetErrorString(e));
            if (dev >= 0 && dev < 64) set_bytes[dev] = dyn;
        }
    }
    const int nsides = S1 ? 2 : 1;
    hipLaunchKernelGGL(k_orth, dim3(nsides * P.b), dim3(256), dyn, s, S0, S1 ? S1 : S0, P.n, t.box_ptr,
                       P.b, r, k, Q0, Q1 ? Q1 : Q0, P.n, sig0, sig1, m_in_lds, 60, qr_only);
    check_launch("orthonormalisation");
}

void launch_orth(const PlanData& P, const DeviceTables& t, double* S, double* Q, double* sigma,
                 hipStream_t s) {
    launch_orth2(P, t, S, nullptr, Q, nullptr, sigma, nullptr, s);
}

void launch_cores(const OpData& op, const PlanData& P, const DeviceTables& t, const double* U,
                  const double* V, double* Atil, hipStream_t s) {
    if (P.k > 64) fail(BLR_ERR_UNSUPPORTED, "k > 64 is not supported by the cores kernel");
    const int64_t ldAt = static_cast<int64_t>(P.b) * P.k;
    dim3 grid(P.b, P.b);
    const int nt = (P.k + 15) / 16;
    if (op.type == OpType::Kernel && nt <= 2) {
        with_source(op, 0, [&](auto A) {
            using AS = decltype(A);
            switch (nt) {
                case 1: hipLaunchKernelGGL((k_cores_sym<AS, 1>), grid, dim3(256), 0, s, A, t.box_ptr, U, V, P.n, P.k, Atil, ldAt); break;
                default: hipLaunchKernelGGL((k_cores_sym<AS, 2>), grid, dim3(256), 0, s, A, t.box_ptr, U, V, P.n, P.k, Atil, ldAt); break;
            }
        });
        check_launch("cores");
        return;
    }
    with_source(op, 0, [&](auto A) {
        using AS = decltype(A);
        switch (nt) {
            case 1: hipLaunchKernelGGL((k_cores<AS, 1>), grid, dim3(256), 0, s, A, t.box_ptr, U, V, P.n, P.k, Atil, ldAt); break;
            case 2: hipLaunchKernelGGL((k_cores<AS, 2>), grid, dim3(256), 0, s, A, t.box_ptr, U, V, P.n, P.k, Atil, ldAt); break;
            case 3: hipLaunchKernelGGL((k_cores<AS, 3>), grid, dim3(256), 0, s, A, t.box_ptr, U, V, P.n, P.k, Atil, ldAt); break;
            default: hipLaunchKernelGGL((k_cores<AS, 4>), grid, dim3(256), 0, s, A, t.box_ptr, U, V, P.n, P.k, Atil, ldAt); break;
        }
    });
    check_launch("cores");
}

int64_t nearfield_workspace_doubles(const PlanData& P) {
    const int64_t kp = 16 * ((P.k + 15) / 16);
    return static_cast<int64_t>(P.b) * P.ncol * P.m_max * kp;
}

// Q products of the near field: the MFMA form while a wave's accumulators stay within 16
// tiles (boxes of at most 256 rows for k <= 64), else the VALU form.
template <int KP>
static void nf_q_launch(const PlanData& P, const DeviceTables& t, const double* V, const double* Atil,
                        int64_t ldAt, double* work, hipStream_t s) {
    constexpr int NTT = KP / 16;
    const dim3 grid(P.b * P.ncol);
    const int rtw = ((P.m_max + 15) / 16 + 3) / 4;
#define BLR_NFQ_M(RTWV)                                                                                   \
    hipLaunchKernelGGL((k_nf_q_m<RTWV, NTT>), grid, dim3(256), 0, s, t.box_ptr, t.colour_ptr, t.colour_boxes, \
                       t.nf_pair, P.ncol, V, P.n, Atil, ldAt, P.k, P.m_max, work)
    if (rtw * NTT <= 16) {
        switch (rtw) {
            case 1: BLR_NFQ_M(1); return;
            case 2: BLR_NFQ_M(2); return;
            case 3: BLR_NFQ_M(3); return;
            case 4: BLR_NFQ_M(4); return;
            default: break;
        }
    }
#undef BLR_NFQ_M
    hipLaunchKernelGGL((k_nf_q<KP>), grid, dim3(256), 0, s, t.box_ptr, t.colour_ptr, t.colour_boxes, t.nf_pair,
                       P.ncol, V, P.n, Atil, ldAt, P.k, P.m_max, work);
}

void launch_nearfield(const OpData& op, const PlanData& P, const DeviceTables& t, const double* U,
                      const double* V, const double* Atil, double* Bv, double* work, hipStream_t s) {
    if (P.k > 64) fail(BLR_ERR_UNSUPPORTED, "k > 64 is not supported by the near-field kernel");
    const int64_t ldAt = static_cast<int64_t>(P.b) * P.k;
    const int kp = 16 * ((P.k + 15) / 16);
    const dim3 grid(P.b * P.ncol);
    auto run = [&](auto kpc) {
        constexpr int KP = decltype(kpc)::value;
        nf_q_launch<KP>(P, t, V, Atil, ldAt, work, s);
        with_source(op, 0, [&](auto A) {
            using AS = decltype(A);
            hipLaunchKernelGGL((k_nf_b<AS, KP>), grid, dim3(256), 0, s, A, t.box_ptr, t.near_idx, t.b_off,
                               t.colour_ptr, t.colour_boxes, t.nf_pair, P.ncol, U, P.n, P.k, P.m_max, work, Bv);
        });
    };
    switch (kp) {
        case 16: run(std::integral_constant<int, 16>{}); break;
        case 32: run(std::integral_constant<int, 32>{}); break;
        case 48: run(std::integral_constant<int, 48>{}); break;
        default: run(std::integral_constant<int, 64>{}); break;
    }
    check_launch("near field");
}

void launch_nf_q(const PlanData& P, const DeviceTables& t, const double* V, const double* Atil,
                 double* work, hipStream_t s) {
    if (P.k > 64) fail(BLR_ERR_UNSUPPORTED, "k > 64 is not supported by the near-field kernel");
    const int64_t ldAt = static_cast<int64_t>(P.b) * P.k;
    const int kp = 16 * ((P.k + 15) / 16);
    const dim3 grid(P.b * P.ncol);
    auto run = [&](auto kpc) {
        constexpr int KP = decltype(kpc)::value;
        nf_q_launch<KP>(P, t, V, Atil, ldAt, work, s);
    };
    switch (kp) {
        case 16: run(std::integral_constant<int, 16>{}); break;
        case 32: run(std::integral_constant<int, 32>{}); break;
        case 48: run(std::integral_constant<int, 48>{}); break;
        default: run(std::integral_constant<int, 64>{}); break;
    }
    check_launch("near field (Q)");
}

// Vector group width and column split of Atil for an apply on ncols vectors: the split gives
// about 2048 workgroups, keeps the partial sums under 1/8 of Atil's bytes and a chunk of t
// within the 4096 LDS values of k_gemv_nc.
struct ApplyShape {
    int nc, groups, nsplit, chunk;
};

static ApplyShape apply_shape(int64_t bk, int64_t ncols) {
    ApplyShape a{};
    a.nc = ncols >= 16 ? 16 : ncols >= 8 ? 8 : ncols >= 4 ? 4 : (ncols >= 2 ? 2 : 1);
    a.groups = static_cast<int>((ncols + a.nc - 1) / a.nc);
    const int64_t rowblocks = (bk + 511) / 512;
    int64_t ns = (2048 + rowblocks * a.groups - 1) / (rowblocks * a.groups);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, bk / (8 * ncols)));
    ns = std::max<int64_t>(ns, (bk + 4096 / a.nc - 1) / (4096 / a.nc));
    ns = std::max<int64_t>(1, std::min<int64_t>(ns, bk));
    const int64_t chunk = (bk + ns - 1) / ns;
    a.chunk = static_cast<int>(chunk);
    a.nsplit = static_cast<int>((bk + chunk - 1) / chunk);
    return a;
}

int64_t apply_workspace_doubles(const PlanData& P, int64_t ncols) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    return (2 + apply_shape(bk, ncols).nsplit) * bk * ncols;
}

void launch_ublr_apply(const PlanData& P, const DeviceTables& t, const double* U, const double* V,
                       const double* Atil, const double* Bv, int trans, int64_t ncols,
                       const double* x, int64_t ldx, double* y, int64_t ldy, double* work,
                       hipStream_t s) {
    if (P.k > 64) fail(BLR_ERR_UNSUPPORTED, "k > 64 is not supported by the apply kernels");
    if (ncols > INT32_MAX / 16) fail(BLR_ERR_INVALID_ARG, "too many vectors");
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    const ApplyShape sh = apply_shape(bk, ncols);
    double* t1 = work;
    double* t2 = work + bk * ncols;
    double* part = work + 2 * bk * ncols;
    const double* Sin = trans ? U : V;
    const double* Sout = trans ? V : U;
    const int nv = static_cast<int>(ncols);
    const unsigned groups = static_cast<unsigned>(sh.groups);
    auto run = [&](auto ncv) {
        constexpr int NC = decltype(ncv)::value;
        hipLaunchKernelGGL((k_proj_nc<NC>), dim3(P.b, groups), dim3(256), 0, s, Sin, P.n, t.box_ptr, P.k, x,
                           ldx, nv, t1, bk);
        if (!trans) {
            hipLaunchKernelGGL((k_gemv_nc<NC>), dim3(static_cast<unsigned>((bk + 511) / 512), sh.nsplit, groups),
                               dim3(256), static_cast<size_t>(sh.chunk) * NC * sizeof(double), s, Atil, bk, bk, t1,
                               nv, part, sh.chunk);
            hipLaunchKernelGGL(k_sum_parts, dim3((bk * ncols + 63) / 64), dim3(256), 0, s, part, sh.nsplit,
                               bk * ncols, t2);
            const dim3 grid(P.b, groups, static_cast<unsigned>((P.m_max + 63) / 64));
            if constexpr (NC == 16)
                hipLaunchKernelGGL((k_near_m16<0>), grid, dim3(256), 0, s, Sout, P.n, t.box_ptr, P.k, t2, bk,
                                   t.near_ptr, t.near_idx, t.near_tpos, t.b_off, Bv, x, ldx, nv, y, ldy);
            else
                hipLaunchKernelGGL((k_near_out_n<NC>), grid, dim3(256), 0, s, Sout, P.n, t.box_ptr, P.k, t2, bk,
                                   t.near_ptr, t.near_idx, t.b_off, Bv, x, ldx, nv, y, ldy);
        }
    };
    if (sh.nc == 16) run(std::integral_constant<int, 16>{});
    else if (sh.nc == 8) run(std::integral_constant<int, 8>{});
    else if (sh.nc == 4) run(std::integral_constant<int, 4>{});
    else if (sh.nc == 2) run(std::integral_constant<int, 2>{});
    else run(std::integral_constant<int, 1>{});
    if (trans) {
        // B_io^T is read across its columns: the MFMA form reads 16 of them per wave as whole
        // cache lines, for any number of vectors
        hipLaunchKernelGGL(k_gemv_t, dim3((bk + 3) / 4, ncols), dim3(256), 0, s, Atil, bk, bk, t1, t2);
        const unsigned g16 = static_cast<unsigned>((ncols + 15) / 16);
        hipLaunchKernelGGL((k_near_m16<1>), dim3(P.b, g16, static_cast<unsigned>((P.m_max + 63) / 64)), dim3(256),
                           0, s, Sout, P.n, t.box_ptr, P.k, t2, bk, t.near_ptr, t.near_idx, t.near_tpos, t.b_off, Bv,
                           x, ldx, nv, y, ldy);
    }
    check_launch("uBLR apply");
}

void launch_err_fro(const OpData& op, const PlanData& P, const DeviceTables& t, const double* U,
                    const double* V, const double* Atil, const double* Bv, double* part,
                    hipStream_t s) {
    if (P.k > 64) fail(BLR_ERR_UNSUPPORTED, "k > 64 is not supported by the error kernel");
    const int64_t ldAt = static_cast<int64_t>(P.b) * P.k;
    with_source(op, 0, [&](auto A) {
        using AS = decltype(A);
        hipLaunchKernelGGL((k_err_fro<AS>), dim3(P.b, P.b), dim3(256), 0, s, A, t.box_ptr,
                           t.near_ptr, t.near_idx, t.b_off, U, V, P.n, Atil, ldAt, P.k, Bv, part);
    });
    check_launch("Frobenius error");
}

// flag[0] = 1 if any of the n values is not finite (flag[0] is set to 0 first by the
// launcher's one-block fill; every writer stores the same value).
__global__ __launch_bounds__(256) void k_zero1(double* __restrict__ flag) {
    if (threadIdx.x == 0) flag[0] = 0.0;
}

__global__ __launch_bounds__(256) void k_flag_nonfinite(const double* __restrict__ p, int64_t n,
                                                        double* __restrict__ flag) {
    bool bad = false;
    for (int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x; q < n;
         q += static_cast<int64_t>(gridDim.x) * 256)
        bad |= !isfinite(p[q]);
    if (bad) flag[0] = 1.0;
}

void launch_flag_nonfinite(const double* const* arrays, const int64_t* counts, int narrays, double* flag,
                           hipStream_t s) {
    hipLaunchKernelGGL(k_zero1, dim3(1), dim3(256), 0, s, flag);
    for (int q = 0; q < narrays; ++q) {
        if (counts[q] <= 0) continue;
        const int64_t blocks = std::min<int64_t>(4096, (counts[q] + 255) / 256);
        hipLaunchKernelGGL(k_flag_nonfinite, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, arrays[q],
                           counts[q], flag);
    }
    check_launch("finiteness check");
}

int dot_parts() { return 1 + kDotBlocks; }

void launch_dot(const double* x, const double* y, int64_t n, double* part, hipStream_t s) {
    hipLaunchKernelGGL(k_dot_stage1, dim3(kDotBlocks), dim3(256), 0, s, x, y, n, part);
    hipLaunchKernelGGL(k_dot_stage2, dim3(1), dim3(64), 0, s, part, kDotBlocks);
    check_launch("dot");
}

void launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy, dim3((n + 255) / 256), dim3(256), 0, s, a, x, y, n);
    check_launch("axpy");
}

void launch_scale(double a, double* x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3((n + 255) / 256), dim3(256), 0, s, a, x, n);
    check_launch("scale");
}

}  // namespace blr
