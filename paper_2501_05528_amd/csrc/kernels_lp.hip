// Low-precision tagged sketch of the mixed-precision mode: Y0 = A Omega and
// Z0 = A* Psi (Alg. 2, sketch step; eq. extend_test_mat) with kernel entries
// generated in FP32, contracted on BF16 or FP32 MFMA with FP32 accumulation,
// and written as FP32.  Also the packing of [G | H] into MFMA fragment order
// and the per-box mixing of sample bases used by the refinement sketch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.hpp"
#include "kernels.hpp"

namespace blr {
namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f4;
typedef float fv4 __attribute__((ext_vector_type(4)));
typedef unsigned int uv4 __attribute__((ext_vector_type(4)));

constexpr int LP_KT = 32;  // sources per K step: one 16x16x32 BF16 MFMA deep


void check_launch_lp(const char* what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) fail(BLR_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

// Address-space qualifiers: the tile body takes LDS tiles as LDS pointers and
// every array in device memory as a global pointer, so the compiler emits ds_*
// and global_* instructions (not flat ones) also when the pointers come from a
// job descriptor in memory.
#define BLR_LDS __attribute__((address_space(3)))
#define BLR_GLB __attribute__((address_space(1)))
template <class T>
__host__ __device__ inline BLR_GLB T* gptr(T* p) {
    return (BLR_GLB T*)p;
}

// ------------------------------------------------------------ FP32 entries
// Kernel functions in single precision from the hardware transcendentals
// (log2, exp2, reciprocal square root); accuracy a few ulp of FP32, far below
// the BF16 rounding of the operands and at the FP32 level of the sketch.
template <int KIND>
__device__ inline float kval32(float r2) {
    if constexpr (KIND == BLR_KERNEL_LOG) {
        return 0.34657359027997264f * __builtin_amdgcn_logf(r2);  // (ln 2 / 2) log2(r^2)
    } else if constexpr (KIND == BLR_KERNEL_INV_R) {
        return __builtin_amdgcn_rsqf(r2);
    } else if constexpr (KIND == BLR_KERNEL_EXP) {
        return __builtin_amdgcn_exp2f(-14.426950408889634f * __builtin_sqrtf(r2));  // e^(-r/0.1)
    } else {
        const float r = __builtin_sqrtf(r2);
        return __cosf(20.0f * r) / (r + 1e-3f);
    }
}

template <int KIND>
struct KernelSrc32 {
    const BLR_GLB float* px;
    const BLR_GLB float* py;
    const BLR_GLB float* pz;
    float diag;
    struct P {
        float x, y, z;
        int32_t i;  // row index (N < 2^31 is checked at launch)
    };
    __device__ P row(int64_t i) const { return P{px[i], py[i], pz[i], static_cast<int32_t>(i)}; }
    __device__ P col(int64_t j) const { return P{px[j], py[j], pz[j], static_cast<int32_t>(j)}; }
    __device__ float val(const P& a, const P& b) const {
        const float dx = a.x - b.x, dy = a.y - b.y, dz = a.z - b.z;
        const float v = kval32<KIND>(dx * dx + dy * dy + dz * dz);
        return a.i == b.i ? diag : v;
    }
    // split entry evaluation (loads of column j, then the arithmetic)
    using Pre = P;
    __device__ Pre pre(const P&, int64_t j) const { return col(j); }
    __device__ float fin(const P& a, const Pre& b) const { return val(a, b); }
    // column jb + off with jb the same for every thread and 0 <= off < 32: the points
    // arrays carry 32 readable entries past the end, so no clamp is needed (entries past
    // the box are discarded by the caller)
    static constexpr bool kPadded = true;
    __device__ Pre pre_at(int64_t jb, int off) const {
        const BLR_GLB float* bx = px + jb;
        const BLR_GLB float* by = py + jb;
        const BLR_GLB float* bz = pz + jb;
        const uint32_t o = static_cast<uint32_t>(off);
        return P{bx[o], by[o], bz[o], static_cast<int32_t>(jb) + off};
    }
};

struct DenseSrc32 {  // A(i, j) = A[i + j*lda], rounded to FP32
    const double* A;
    int64_t lda;
    struct P {
        int64_t i;
    };
    __device__ P row(int64_t i) const { return P{i}; }
    __device__ P col(int64_t j) const { return P{j}; }
    __device__ float val(const P& a, const P& b) const { return static_cast<float>(A[a.i + b.i * lda]); }
    using Pre = double;
    __device__ Pre pre(const P& a, int64_t j) const { return A[a.i + j * lda]; }
    __device__ float fin(const P&, Pre v) const { return static_cast<float>(v); }
};

struct DenseTSrc32 {  // (A*)(i, j) = A[j + i*lda], rounded to FP32
    const double* A;
    int64_t lda;
    struct P {
        int64_t i;
    };
    __device__ P row(int64_t i) const { return P{i}; }
    __device__ P col(int64_t j) const { return P{j}; }
    __device__ float val(const P& a, const P& b) const { return static_cast<float>(A[b.i + a.i * lda]); }
    using Pre = double;
    __device__ Pre pre(const P& a, int64_t j) const { return A[j + a.i * lda]; }
    __device__ float fin(const P&, Pre v) const { return static_cast<float>(v); }
};

// Sources whose point arrays are padded (KernelSrc32::kPadded) load a step's columns
// without clamping.
template <class AS, class = void>
struct PaddedSrc : std::false_type {};
template <class AS>
struct PaddedSrc<AS, std::void_t<decltype(AS::kPadded)>> : std::bool_constant<AS::kPadded> {};

template <int PREC>
struct LpElem;
template <>
struct LpElem<BLR_PREC_BF16_REFINE> {
    using T = __bf16;
};
template <>
struct LpElem<BLR_PREC_FP32_REFINE> {
    using T = float;
};

// ------------------------------------------------------------ packing
// The K loop of the sketch walks the source boxes in steps of LP_KT rows that
// never straddle a box (box l has ceil(m_l / LP_KT) steps, numbered box by box).
// Packed layout of one side (G or H, N x r): for step t, column tile nt (16
// columns), lane L and element e = 0..7 the value G(row, c) with
//   row = first row of the step + 8 (L / 16) + e,   c = 16 nt + L % 16,
// zero past the box or past column r, at ((t*NTR + nt)*64 + L)*8 + e.  Each
// lane of an MFMA B operand then reads its eight values as one 16-byte
// (BF16) or 32-byte (FP32) word.
template <class E>
__global__ __launch_bounds__(256) void k_pack_lp(const double* __restrict__ G, int64_t n, int r,
                                                 const int64_t* __restrict__ box_ptr,
                                                 const int32_t* __restrict__ kstep_ptr,
                                                 const int32_t* __restrict__ kstep_box, int nsteps,
                                                 int ntr, E* __restrict__ out) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;  // (t, nt, lane)
    const int64_t total = static_cast<int64_t>(nsteps) * ntr * 64;
    if (idx >= total) return;
    const int lane = static_cast<int>(idx & 63);
    const int64_t tn = idx >> 6;
    const int nt = static_cast<int>(tn % ntr);
    const int t = static_cast<int>(tn / ntr);
    const int l = kstep_box[t];
    const int64_t j0 = box_ptr[l] + static_cast<int64_t>(t - kstep_ptr[l]) * LP_KT;
    const int64_t jend = box_ptr[l + 1];
    const int c = nt * 16 + (lane & 15);
    E* o = out + idx * 8;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int64_t j = j0 + 8 * (lane >> 4) + e;
        const double v = (c < r && j < jend) ? G[j + static_cast<int64_t>(c) * n] : 0.0;
        o[e] = static_cast<E>(static_cast<float>(v));
    }
}

// ------------------------------------------------------------ sketch
// Y_sd(:, s*r + c) = sum_l T(l, s) A(:, I_l) G_sd(I_l, c) for every tag
// column s (sd = side: G for Y, H for Z with the same kernel tile when the
// matrix is symmetric).  Workgroup: 32 target rows and a group of tag columns;
// wave w takes row tile w & 1 (16 rows) and half w >> 1 of the group's tag
// columns.  Per K step the workgroup generates the 32 x 32 FP32 kernel tile
// into LDS and copies the packed [G|H] fragments for the step into LDS; each
// wave scales its A fragment by T(l, s) (one scalar per step, since steps stay
// inside box l), rounds it to the MFMA type and contracts it with every B
// fragment of both sides.  MFMA layouts (gfx950):
//   16x16x32 BF16: A lane L, element e: A[L % 16][8 (L / 16) + e];
//                  B lane L, element e: B[8 (L / 16) + e][L % 16];
//   16x16x4 F32 (8 of them per step, number e): A lane L: A[L % 16][8 (L / 16) + e],
//                  B lane L: B[8 (L / 16) + e][L % 16]  (the same K assignment);
//   D lane L, element v: D[4 (L / 16) + v][L % 16] for both.
template <int PREC, int NTR, int NSIDE>
struct LpTile {
    using E = typename LpElem<PREC>::T;
    static constexpr int BM = 32, KT = LP_KT, AST = KT + 4;    // rows, sources/step, LDS row stride
    static constexpr int FRAG = 64 * 8;                        // elements of one B fragment
    static constexpr int BEL = NSIDE * NTR * FRAG;             // B elements per step
};

// One workgroup tile of the sketch: target rows [32 rt_blk, 32 rt_blk + 32) and tag
// column group grp.  sAp / sBp: double-buffered LDS tiles (2 x BM*AST floats, 2 x BEL
// elements), 16-byte aligned.
template <class AS, int PREC, int NTR, int NSIDE, int SPW>
__device__ __attribute__((always_inline)) inline void sketch_lp_tile(AS A, const BLR_GLB float* __restrict__ Tf,
                                      const BLR_GLB int64_t* __restrict__ box_ptr, int nbox,
                                      const BLR_GLB typename LpElem<PREC>::T* __restrict__ B0,
                                      const BLR_GLB typename LpElem<PREC>::T* __restrict__ B1, int64_t n,
                                      int r, int ell, BLR_GLB float* __restrict__ Y0, BLR_GLB float* __restrict__ Y1,
                                      int64_t rt_blk, int grp, BLR_LDS float* sAp,
                                      BLR_LDS typename LpElem<PREC>::T* sBp) {
    using E = typename LpElem<PREC>::T;
    using TL = LpTile<PREC, NTR, NSIDE>;
    constexpr int BM = TL::BM, KT = TL::KT, AST = TL::AST, FRAG = TL::FRAG, BEL = TL::BEL;
    constexpr int CH_EL = 16 / sizeof(E);                      // elements per 16-byte chunk
    constexpr int NCH = BEL / CH_EL;                           // 16-byte chunks per step
    constexpr int CPT = (NCH + 255) / 256;                     // chunks per thread
    BLR_LDS float (*sA)[BM * AST] = reinterpret_cast<BLR_LDS float (*)[BM * AST]>(sAp);
    BLR_LDS E (*sB)[BEL] = reinterpret_cast<BLR_LDS E (*)[BEL]>(sBp);
    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int rt = wave & 1, half = wave >> 1;
    const int64_t row0 = rt_blk * BM;
    const int sg0 = grp * 2 * SPW;
    const int sgn = min(2 * SPW, ell - sg0);
    const int s_lo = sg0 + (half * sgn) / 2;
    const int nsv = sg0 + ((half + 1) * sgn) / 2 - s_lo;
    // A generation: thread owns row tid % 32 and sources (tid / 32) + 8u, u < 4
    const int arow = tid & 31, akk = tid >> 5;
    const int64_t gi = row0 + arow;
    const auto rp = A.row(gi < n ? gi : n - 1);

    uint64_t bv[CPT][2];
    auto fetch_b = [&](int64_t t) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int ch = tid + 256 * u;
            if (ch < NCH) {
                const int el = ch * CH_EL;                 // element within the step block
                const int sd = el / (NTR * FRAG);
                const BLR_GLB E* src = (sd ? B1 : B0) + t * (NTR * FRAG) + (el - sd * NTR * FRAG);
                const BLR_GLB uint64_t* q = reinterpret_cast<const BLR_GLB uint64_t*>(src);
                bv[u][0] = q[0];
                bv[u][1] = q[1];
            }
        }
    };
    auto store_b = [&](int buf) {
#pragma unroll
        for (int u = 0; u < CPT; ++u) {
            const int ch = tid + 256 * u;
            if (ch < NCH) {
                BLR_LDS uint64_t* q = reinterpret_cast<BLR_LDS uint64_t*>(&sB[buf][ch * CH_EL]);
                q[0] = bv[u][0];
                q[1] = bv[u][1];
            }
        }
    };
    // the next step's kernel columns are loaded before the current step's MFMAs
    // (pre) and turned into entries after them (gen_a)
    typename AS::Pre apre[4];
    auto pre_a = [&](int64_t jb, int64_t jend) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if constexpr (PaddedSrc<AS>::value) {
                apre[u] = A.pre_at(jb, akk + 8 * u);
            } else {
                const int64_t j = jb + akk + 8 * u;
                apre[u] = A.pre(rp, j < jend ? j : jend - 1);
            }
        }
    };
    auto gen_a = [&](int buf, int64_t jb, int64_t jend) {
        const int nvalid = static_cast<int>(min(jend - jb, static_cast<int64_t>(KT)));  // same for all threads
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int kk = akk + 8 * u;
            const float v = A.fin(rp, apre[u]);
            sA[buf][arow * AST + kk] = kk < nvalid ? v : 0.0f;
        }
    };

    f4 acc[SPW][NSIDE][NTR];
#pragma unroll
    for (int v = 0; v < SPW; ++v)
#pragma unroll
        for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
            for (int nt = 0; nt < NTR; ++nt) acc[v][sd][nt] = f4{0.0f, 0.0f, 0.0f, 0.0f};

    int l = 0;
    int64_t j0 = box_ptr[0], jend = box_ptr[1];
    int64_t t = 0;  // packed step index
    float tw[SPW], twn[SPW];
    auto load_tw = [&](float* w, int lb) {
#pragma unroll
        for (int v = 0; v < SPW; ++v) w[v] = Tf[static_cast<int64_t>(lb) * ell + min(s_lo + v, ell - 1)];
    };
    fetch_b(t);
    pre_a(j0, jend);
    load_tw(tw, 0);
    store_b(0);
    gen_a(0, j0, jend);
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
            fetch_b(t + 1);
            pre_a(jn, jendn);
            load_tw(twn, ln);
        }
        // this wave's A fragment: row rt*16 + lane % 16, sources 8 (lane / 16) + e
        float af[8];
        {
            const BLR_LDS float* ap = &sA[buf][(rt * 16 + (lane & 15)) * AST + 8 * (lane >> 4)];
            const fv4 lo = *reinterpret_cast<const BLR_LDS fv4*>(ap);
            const fv4 hi = *reinterpret_cast<const BLR_LDS fv4*>(ap + 4);
            af[0] = lo.x; af[1] = lo.y; af[2] = lo.z; af[3] = lo.w;
            af[4] = hi.x; af[5] = hi.y; af[6] = hi.z; af[7] = hi.w;
        }
        if constexpr (PREC == BLR_PREC_BF16_REFINE) {
            bf16x8 bq[NSIDE][NTR];
#pragma unroll
            for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                for (int nt = 0; nt < NTR; ++nt)
                    bq[sd][nt] = *reinterpret_cast<const BLR_LDS bf16x8*>(&sB[buf][((sd * NTR + nt) * 64 + lane) * 8]);
#pragma unroll
            for (int v = 0; v < SPW; ++v) {
                if (v < nsv) {
                    bf16x8 as;
#pragma unroll
                    for (int e = 0; e < 8; ++e) as[e] = static_cast<__bf16>(af[e] * tw[v]);
#pragma unroll
                    for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                        for (int nt = 0; nt < NTR; ++nt)
                            acc[v][sd][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as, bq[sd][nt], acc[v][sd][nt], 0, 0, 0);
                }
            }
        } else {
            float bq[NSIDE][NTR][8];
#pragma unroll
            for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                for (int nt = 0; nt < NTR; ++nt) {
                    const BLR_LDS float* bp = &sB[buf][((sd * NTR + nt) * 64 + lane) * 8];
                    const fv4 lo = *reinterpret_cast<const BLR_LDS fv4*>(bp);
                    const fv4 hi = *reinterpret_cast<const BLR_LDS fv4*>(bp + 4);
                    bq[sd][nt][0] = lo.x; bq[sd][nt][1] = lo.y; bq[sd][nt][2] = lo.z; bq[sd][nt][3] = lo.w;
                    bq[sd][nt][4] = hi.x; bq[sd][nt][5] = hi.y; bq[sd][nt][6] = hi.z; bq[sd][nt][7] = hi.w;
                }
#pragma unroll
            for (int v = 0; v < SPW; ++v) {
                if (v < nsv) {
                    float as[8];
#pragma unroll
                    for (int e = 0; e < 8; ++e) as[e] = af[e] * tw[v];
#pragma unroll
                    for (int e = 0; e < 8; ++e)
#pragma unroll
                        for (int sd = 0; sd < NSIDE; ++sd)
#pragma unroll
                            for (int nt = 0; nt < NTR; ++nt)
                                acc[v][sd][nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[e], bq[sd][nt][e], acc[v][sd][nt], 0, 0, 0);
                }
            }
        }
        if (!more) break;
        store_b(buf ^ 1);
        gen_a(buf ^ 1, jn, jendn);
        __syncthreads();
        buf ^= 1;
        l = ln;
        j0 = jn;
        jend = jendn;
        ++t;
#pragma unroll
        for (int v = 0; v < SPW; ++v) tw[v] = twn[v];
    }
    // epilogue: acc[v][sd][nt] element q -> row rt*16 + 4 (lane / 16) + q, column nt*16 + lane % 16
#pragma unroll
    for (int v = 0; v < SPW; ++v) {
        if (v >= nsv) continue;
        const int sv = s_lo + v;
#pragma unroll
        for (int sd = 0; sd < NSIDE; ++sd) {
            BLR_GLB float* Yo = sd ? Y1 : Y0;
#pragma unroll
            for (int nt = 0; nt < NTR; ++nt) {
                const int c = nt * 16 + (lane & 15);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int64_t row = row0 + rt * 16 + 4 * (lane >> 4) + q;
                    if (row < n && c < r) Yo[row + static_cast<int64_t>(sv * r + c) * n] = acc[v][sd][nt][q];
                }
            }
        }
    }
}

template <class AS, int PREC, int NTR, int NSIDE, int SPW>
__global__ __launch_bounds__(256, 2) void k_sketch_lp(AS A, const float* __restrict__ Tf,
                                                      const int64_t* __restrict__ box_ptr, int nbox,
                                                      const typename LpElem<PREC>::T* __restrict__ B0,
                                                      const typename LpElem<PREC>::T* __restrict__ B1,
                                                      int64_t n, int r, int ell,
                                                      float* __restrict__ Y0, float* __restrict__ Y1) {
    using TL = LpTile<PREC, NTR, NSIDE>;
    __shared__ __attribute__((aligned(16))) float sA[2 * TL::BM * TL::AST];
    __shared__ __attribute__((aligned(16))) typename TL::E sB[2 * TL::BEL];
    sketch_lp_tile<AS, PREC, NTR, NSIDE, SPW>(A, gptr(Tf), gptr(box_ptr), nbox, gptr(B0), gptr(B1), n, r,
                                              ell, gptr(Y0), gptr(Y1), blockIdx.x, blockIdx.y,
                                              (BLR_LDS float*)sA, (BLR_LDS typename TL::E*)sB);
}

// Persistent form over a batch of kernel-matrix jobs: workgroups stride over a
// list of (job, row block, tag column group) items, heaviest first; the kernel
// kind of each job is dispatched per item.
template <int PREC, int NTR, int SPW>
__global__ __launch_bounds__(256, 2) void k_sketch_lp_multi(const LpJob* __restrict__ jobs,
                                                            const int4* __restrict__ items,
                                                            int nitems) {
    using TL = LpTile<PREC, NTR, 2>;
    using E = typename TL::E;
    __shared__ __attribute__((aligned(16))) float sA[2 * TL::BM * TL::AST];
    __shared__ __attribute__((aligned(16))) E sB[2 * TL::BEL];
    BLR_LDS float* lA = (BLR_LDS float*)sA;
    BLR_LDS E* lB = (BLR_LDS E*)sB;
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int4 w = items[it];
        const LpJob& J = jobs[w.x];
        const int64_t rt_blk = static_cast<int64_t>(w.y);
        const BLR_GLB E* b0 = gptr(static_cast<const E*>(J.B0));
        const BLR_GLB E* b1 = gptr(static_cast<const E*>(J.B1));
        const BLR_GLB float* px = gptr(J.px);
        const BLR_GLB float* py = gptr(J.py);
        const BLR_GLB float* pz = gptr(J.pz);
        const BLR_GLB float* Tf = gptr(J.Tf);
        const BLR_GLB int64_t* bptr = gptr(J.box_ptr);
        BLR_GLB float* Y0 = gptr(J.Y0);
        BLR_GLB float* Y1 = gptr(J.Y1);
        __syncthreads();  // the previous item's last reads of LDS are done
        switch (J.kind) {
            case BLR_KERNEL_LOG:
                sketch_lp_tile<KernelSrc32<BLR_KERNEL_LOG>, PREC, NTR, 2, SPW>(
                    KernelSrc32<BLR_KERNEL_LOG>{px, py, pz, J.diag}, Tf, bptr, J.nbox, b0, b1,
                    J.n, J.r, J.ell, Y0, Y1, rt_blk, w.z, lA, lB);
                break;
            case BLR_KERNEL_INV_R:
                sketch_lp_tile<KernelSrc32<BLR_KERNEL_INV_R>, PREC, NTR, 2, SPW>(
                    KernelSrc32<BLR_KERNEL_INV_R>{px, py, pz, J.diag}, Tf, bptr, J.nbox, b0, b1,
                    J.n, J.r, J.ell, Y0, Y1, rt_blk, w.z, lA, lB);
                break;
            case BLR_KERNEL_EXP:
                sketch_lp_tile<KernelSrc32<BLR_KERNEL_EXP>, PREC, NTR, 2, SPW>(
                    KernelSrc32<BLR_KERNEL_EXP>{px, py, pz, J.diag}, Tf, bptr, J.nbox, b0, b1,
                    J.n, J.r, J.ell, Y0, Y1, rt_blk, w.z, lA, lB);
                break;
            default:
                sketch_lp_tile<KernelSrc32<BLR_KERNEL_COS>, PREC, NTR, 2, SPW>(
                    KernelSrc32<BLR_KERNEL_COS>{px, py, pz, J.diag}, Tf, bptr, J.nbox, b0, b1,
                    J.n, J.r, J.ell, Y0, Y1, rt_blk, w.z, lA, lB);
                break;
        }
    }
}

template <int PREC, class AS>
void sketch_lp_launch(AS A, const PlanData& P, const DeviceTables& t, int r, const void* B0,
                      const void* B1, int nside, float* Y0, float* Y1, hipStream_t s) {
    using E = typename LpElem<PREC>::T;
    const int ntr = (r + 15) / 16;
    const E* b0 = static_cast<const E*>(B0);
    const E* b1 = static_cast<const E*>(B1);
    // SPW (tag columns per wave) from the accumulator budget SPW * nside * ntr float4
    // per wave (about 168 floats for BF16, 120 for FP32), at most 8; a workgroup
    // covers 2 SPW tag columns and grid.y the groups of them.
#define BLR_LP_CASE(NTRV, NSV, SPWV)                                                               \
    hipLaunchKernelGGL((k_sketch_lp<AS, PREC, NTRV, NSV, SPWV>),                                   \
                       dim3(static_cast<unsigned>((P.n + 31) / 32), (P.ell + 2 * SPWV - 1) / (2 * SPWV)), \
                       dim3(256), 0, s, A, t.Tf, t.box_ptr, P.b, b0, b1, P.n, r, P.ell, Y0, Y1)
    if (PREC == BLR_PREC_BF16_REFINE) {
        if (nside == 2) {
            switch (ntr) {
                case 1: BLR_LP_CASE(1, 2, 8); break;
                case 2: BLR_LP_CASE(2, 2, 8); break;
                case 3: BLR_LP_CASE(3, 2, 7); break;
                case 4: BLR_LP_CASE(4, 2, 5); break;
                case 5: BLR_LP_CASE(5, 2, 4); break;
                default: fail(BLR_ERR_UNSUPPORTED, "r_lo > 80 is not supported by the low-precision sketch");
            }
        } else {
            switch (ntr) {
                case 1: BLR_LP_CASE(1, 1, 8); break;
                case 2: BLR_LP_CASE(2, 1, 8); break;
                case 3: BLR_LP_CASE(3, 1, 8); break;
                case 4: BLR_LP_CASE(4, 1, 8); break;
                case 5: BLR_LP_CASE(5, 1, 8); break;
                default: fail(BLR_ERR_UNSUPPORTED, "r_lo > 80 is not supported by the low-precision sketch");
            }
        }
    } else {
        if (nside == 2) {
            switch (ntr) {
                case 1: BLR_LP_CASE(1, 2, 8); break;
                case 2: BLR_LP_CASE(2, 2, 7); break;
                case 3: BLR_LP_CASE(3, 2, 5); break;
                case 4: BLR_LP_CASE(4, 2, 3); break;
                case 5: BLR_LP_CASE(5, 2, 3); break;
                default: fail(BLR_ERR_UNSUPPORTED, "r_lo > 80 is not supported by the low-precision sketch");
            }
        } else {
            switch (ntr) {
                case 1: BLR_LP_CASE(1, 1, 8); break;
                case 2: BLR_LP_CASE(2, 1, 8); break;
                case 3: BLR_LP_CASE(3, 1, 8); break;
                case 4: BLR_LP_CASE(4, 1, 7); break;
                case 5: BLR_LP_CASE(5, 1, 6); break;
                default: fail(BLR_ERR_UNSUPPORTED, "r_lo > 80 is not supported by the low-precision sketch");
            }
        }
    }
#undef BLR_LP_CASE
    check_launch_lp("low-precision tagged sketch");
}

// ------------------------------------------------------------ mixing
// X(I_l, c) = sum_a Q0(I_l, a) gamma[l](a, c), gamma C-ordered b x r_lo x r.
__global__ __launch_bounds__(256) void k_mix(const double* __restrict__ Q0, int64_t n, int r_lo,
                                             const double* __restrict__ gamma, int r,
                                             const int32_t* __restrict__ rb, double* __restrict__ X) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
    if (idx >= n * r) return;
    const int c = static_cast<int>(idx / n);
    const int64_t row = idx - static_cast<int64_t>(c) * n;
    const double* g = gamma + static_cast<int64_t>(rb[row]) * r_lo * r + c;
    double acc = 0.0;
    for (int a = 0; a < r_lo; ++a) acc = fma(Q0[row + static_cast<int64_t>(a) * n], g[static_cast<int64_t>(a) * r], acc);
    X[row + static_cast<int64_t>(c) * n] = acc;
}

}  // namespace

int64_t lp_packed_elems(const PlanData& P, int r_lo) {
    const int ntr = (r_lo + 15) / 16;
    return static_cast<int64_t>(P.kstep_ptr.back()) * ntr * 64 * 8;
}

void launch_pack_lp(const PlanData& P, const DeviceTables& t, int precision, int r_lo,
                    const double* G, void* out, hipStream_t s) {
    const int ntr = (r_lo + 15) / 16;
    const int nsteps = P.kstep_ptr.back();
    const int64_t total = static_cast<int64_t>(nsteps) * ntr * 64;
    const dim3 grid(static_cast<unsigned>((total + 255) / 256));
    if (precision == BLR_PREC_BF16_REFINE)
        hipLaunchKernelGGL(k_pack_lp<__bf16>, grid, dim3(256), 0, s, G, P.n, r_lo, t.box_ptr,
                           t.kstep_ptr, t.kstep_box, nsteps, ntr, static_cast<__bf16*>(out));
    else
        hipLaunchKernelGGL(k_pack_lp<float>, grid, dim3(256), 0, s, G, P.n, r_lo, t.box_ptr,
                           t.kstep_ptr, t.kstep_box, nsteps, ntr, static_cast<float*>(out));
    check_launch_lp("packing of the low-precision test blocks");
}

void launch_sketch_lp(const OpData& op, const PlanData& P, const DeviceTables& t, int precision,
                      int r_lo, const void* PG, const void* PH, float* Y, float* Z, hipStream_t s) {
    auto run = [&](auto prec_tag) {
        constexpr int PREC = decltype(prec_tag)::value;
        if (op.type == OpType::Kernel) {
            if (op.n >= (int64_t(1) << 31)) fail(BLR_ERR_UNSUPPORTED, "N >= 2^31 in the low-precision sketch");
            const BLR_GLB float* px = gptr(op.pts32);
            const BLR_GLB float* py = gptr(op.pts32 + op.n);
            const BLR_GLB float* pz = gptr(op.pts32 + 2 * op.n);
            auto go = [&](auto A) { sketch_lp_launch<PREC>(A, P, t, r_lo, PG, PH, 2, Y, Z, s); };
            switch (op.kind) {
                case BLR_KERNEL_LOG: go(KernelSrc32<BLR_KERNEL_LOG>{px, py, pz, 0.0f}); break;
                case BLR_KERNEL_INV_R: go(KernelSrc32<BLR_KERNEL_INV_R>{px, py, pz, 0.0f}); break;
                case BLR_KERNEL_EXP: go(KernelSrc32<BLR_KERNEL_EXP>{px, py, pz, 1.0f}); break;
                case BLR_KERNEL_COS: go(KernelSrc32<BLR_KERNEL_COS>{px, py, pz, 1000.0f}); break;
                default: fail(BLR_ERR_INVALID_ARG, "unknown kernel kind");
            }
        } else {
            sketch_lp_launch<PREC>(DenseSrc32{op.A, op.lda}, P, t, r_lo, PG, PG, 1, Y, Y, s);
            sketch_lp_launch<PREC>(DenseTSrc32{op.A, op.lda}, P, t, r_lo, PH, PH, 1, Z, Z, s);
        }
    };
    if (precision == BLR_PREC_BF16_REFINE)
        run(std::integral_constant<int, BLR_PREC_BF16_REFINE>{});
    else if (precision == BLR_PREC_FP32_REFINE)
        run(std::integral_constant<int, BLR_PREC_FP32_REFINE>{});
    else
        fail(BLR_ERR_INVALID_ARG, "not a low-precision mode");
}

int lp_multi_spw_candidates(int precision, int ntr, int* spw) {
    // (candidates keep the persistent kernel free of register spills)
    static const int bf16[6][2] = {{0, 0}, {8, 4}, {8, 4}, {6, 4}, {4, 3}, {3, 2}};
    static const int fp32[6][2] = {{0, 0}, {8, 4}, {7, 4}, {4, 3}, {3, 2}, {2, 1}};
    if (ntr < 1 || ntr > 5) fail(BLR_ERR_UNSUPPORTED, "r_lo > 80 is not supported by the low-precision sketch");
    const int(*tab)[2] = precision == BLR_PREC_BF16_REFINE ? bf16 : fp32;
    spw[0] = tab[ntr][0];
    spw[1] = tab[ntr][1];
    return 2;
}

void launch_sketch_lp_multi(int precision, int ntr, int spw, const LpJob* jobs, const int4* items,
                            int nitems, int grid, hipStream_t s) {
    if (nitems <= 0) return;
    const dim3 g(static_cast<unsigned>(std::max(1, std::min(grid, nitems))));
#define BLR_LPM(PRECV, NTRV, SPWV)                                                                 \
    if (precision == PRECV && ntr == NTRV && spw == SPWV) {                                        \
        hipLaunchKernelGGL((k_sketch_lp_multi<PRECV, NTRV, SPWV>), g, dim3(256), 0, s, jobs, items, nitems); \
        check_launch_lp("persistent low-precision sketch");                                        \
        return;                                                                                    \
    }
    BLR_LPM(BLR_PREC_BF16_REFINE, 1, 8) BLR_LPM(BLR_PREC_BF16_REFINE, 1, 4)
    BLR_LPM(BLR_PREC_BF16_REFINE, 2, 8) BLR_LPM(BLR_PREC_BF16_REFINE, 2, 4)
    BLR_LPM(BLR_PREC_BF16_REFINE, 3, 6) BLR_LPM(BLR_PREC_BF16_REFINE, 3, 4)
    BLR_LPM(BLR_PREC_BF16_REFINE, 4, 4) BLR_LPM(BLR_PREC_BF16_REFINE, 4, 3)
    BLR_LPM(BLR_PREC_BF16_REFINE, 5, 3) BLR_LPM(BLR_PREC_BF16_REFINE, 5, 2)
    BLR_LPM(BLR_PREC_FP32_REFINE, 1, 8) BLR_LPM(BLR_PREC_FP32_REFINE, 1, 4)
    BLR_LPM(BLR_PREC_FP32_REFINE, 2, 7) BLR_LPM(BLR_PREC_FP32_REFINE, 2, 4)
    BLR_LPM(BLR_PREC_FP32_REFINE, 3, 4) BLR_LPM(BLR_PREC_FP32_REFINE, 3, 3)
    BLR_LPM(BLR_PREC_FP32_REFINE, 4, 3) BLR_LPM(BLR_PREC_FP32_REFINE, 4, 2)
    BLR_LPM(BLR_PREC_FP32_REFINE, 5, 2) BLR_LPM(BLR_PREC_FP32_REFINE, 5, 1)
#undef BLR_LPM
    fail(BLR_ERR_INVALID_ARG, "no persistent sketch for this precision, column tiles and SPW");
}

void launch_mix(const PlanData& P, const DeviceTables& t, int r_lo, const double* Q0,
                const double* gamma, double* X, hipStream_t s) {
    const int64_t total = P.n * P.r;
    hipLaunchKernelGGL(k_mix, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, Q0,
                       P.n, r_lo, gamma, P.r, t.row_box, X);
    check_launch_lp("mixing of the sample bases");
}

}  // namespace blr
