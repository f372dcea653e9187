// Host-side launchers of the HIP kernels (kernels.hip).  All pointers are
// device memory; every launcher enqueues on `stream` and throws blr::Error
// on a launch failure.
#pragma once

#include <hip/hip_runtime.h>

#include "internal.hpp"

namespace blr {

// Y|Z sketch (Alg. 2): the tagged test matrices are formed in-kernel from T,
// the box of each row and the stacked Gaussian blocks.
void launch_sketch(const OpData& op, const PlanData& P, const DeviceTables& t, const double* G,
                   const double* H, double* Y, double* Z, hipStream_t s);

// Y = A X or A* X for a dense X (n x ncols).
// Y = op(A) X for a built-in operator; work holds op_apply_workspace_doubles(op, ncols)
// doubles (NULL when that is 0)
int64_t op_apply_workspace_doubles(const OpData& op, int64_t ncols);
void launch_op_apply(const OpData& op, int trans, int64_t ncols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy, double* work, hipStream_t s);

void launch_postprocess(const PlanData& P, const DeviceTables& t, const double* Y, double* Yhat,
                        hipStream_t s);

void launch_orth(const PlanData& P, const DeviceTables& t, double* S, double* Q, double* sigma,
                 hipStream_t s);
// General form: S has r columns, Q receives k <= r; qr_only = 1 gives the first k
// columns of the Householder Q (sign rule applied) without the SVD step.
void launch_orth_cols(const PlanData& P, const DeviceTables& t, int r, int k, int qr_only,
                      double* S0, double* S1, double* Q0, double* Q1, double* sig0, double* sig1,
                      hipStream_t s);
// Both sides in one launch (S1/Q1 may be null for one side).
void launch_orth2(const PlanData& P, const DeviceTables& t, double* S0, double* S1, double* Q0,
                  double* Q1, double* sig0, double* sig1, hipStream_t s);

void launch_cores(const OpData& op, const PlanData& P, const DeviceTables& t, const double* U,
                  const double* V, double* Atil, hipStream_t s);

// One kernel-matrix job of a persistent low-precision sketch launch (device array).
struct LpJob {
    int kind;                 // blr_kernel_kind
    float diag;               // kernel diagonal value
    const float* px;          // FP32 points, SoA
    const float* py;
    const float* pz;
    const float* Tf;          // b x ell row-major, FP32
    const int64_t* box_ptr;   // [b+1]
    int nbox;
    int r;                    // r_lo
    int ell;
    int64_t n;
    const void* B0;           // packed G (lp_packed_elems of the precision's type)
    const void* B1;           // packed H
    float* Y0;                // N x ell r_lo
    float* Y1;
};
// One kernel-matrix job of a persistent FP64 sketch launch (device array).
struct Fp64Job {
    int kind;                 // blr_kernel_kind (the same for every job of a launch)
    double diag;              // kernel diagonal value
    const double* px;         // FP64 points, SoA
    const double* py;
    const double* pz;
    const double* T;          // b x ell row-major
    const int64_t* box_ptr;   // [b+1]
    int nbox;
    int r;
    int ell;
    int64_t n;
    const double* G0;         // N x r
    const double* G1;
    double* Y0;               // N x ell r
    double* Y1;
    int ngroups;              // tag column groups (items carry the group index)
};
// Most tag columns per wave of the FP64 sketch for r = 16 ntr columns per side, both
// sides (the single-job choice); a workgroup covers 4 of them per group.
int fp64_sketch_svw(int ntr);
// Form of the last 16-column tile of the two-sided FP64 sketch for r columns per side and
// an entry source of the given kernel kind (-1: a dense matrix): 3 for the narrow form
// (three 4-column groups; the tile holds at most 12 columns), else 0.
int fp64_sketch_tail_groups(int kind, int r);
// Persistent FP64 sketch over items (job, 8-row block, tag column group) of jobs of
// one kernel kind; svw is fp64_sketch_svw(ntr) or one less, and every job's groups
// hold at most 4 svw tag columns; tg is fp64_sketch_tail_groups(kind, r) of every job.  Grid
// workgroups stride over the items.
void launch_sketch_multi(int kind, int ntr, int svw, int tg, const Fp64Job* jobs, const int4* items,
                         int nitems, int grid, hipStream_t s);
// Tag columns per wave (SPW) offered to the autotuner for a (precision, column
// tiles) class; a workgroup covers 2 SPW tag columns.  Returns the count (<= 2).
int lp_multi_spw_candidates(int precision, int ntr, int* spw);
// Persistent sketch over items (job, 32-row block, tag column group) built for the
// given SPW; grid workgroups stride over the items.
void launch_sketch_lp_multi(int precision, int ntr, int spw, const LpJob* jobs, const int4* items,
                            int nitems, int grid, hipStream_t s);

// Mixed-precision mode (kernels_lp.hip): [G|H] packed per side into MFMA
// fragment order (lp_packed_elems elements of 2 bytes for BF16, 4 for FP32),
// the low-precision tagged sketch into FP32 Y, Z (N x ell r_lo), and the mixing
// X(I_l) = Q0(I_l) gamma[l] (gamma C-ordered b x r_lo x r).
int64_t lp_packed_elems(const PlanData& P, int r_lo);
void launch_pack_lp(const PlanData& P, const DeviceTables& t, int precision, int r_lo,
                    const double* G, void* out, hipStream_t s);
void launch_sketch_lp(const OpData& op, const PlanData& P, const DeviceTables& t, int precision,
                      int r_lo, const void* PG, const void* PH, float* Y, float* Z, hipStream_t s);
void launch_postprocess_lp(const PlanData& P, const DeviceTables& t, int r_lo, const float* Y,
                           double* Yhat, hipStream_t s);
void launch_mix(const PlanData& P, const DeviceTables& t, int r_lo, const double* Q0,
                const double* gamma, double* X, hipStream_t s);
// FP64 far-field refinement sketch: S0 = far(A) X0, S1 = far(A*) X1 (N x r each).
void launch_refine(const OpData& op, const PlanData& P, const DeviceTables& t, const double* X0,
                   const double* X1, double* S0, double* S1, hipStream_t s);

// Black-box operators (blackbox.hip): explicit test matrices for the caller's
// products and the kernels that turn the products into Atil and B.
void launch_expand_tagged(const PlanData& P, const DeviceTables& t, const double* G, double* Om,
                          hipStream_t s);
void launch_embed_blockdiag(const PlanData& P, const DeviceTables& t, const double* S, int w, int j0,
                            int j1, double* X, hipStream_t s);
// Mixed precision on a black box: the tagged test matrix with w columns per tag column in
// FP64 or rounded to FP32, FP64 -> FP32 rounding, zero fill, and the far-field gather
// S(row, :) += sum_{l in [j0, j1), l far from box(row)} W(row, block l) of products with
// block-diagonal test columns.
void launch_expand_tagged_w(const PlanData& P, const DeviceTables& t, const double* G, int w, double* Om,
                            hipStream_t s);
void launch_expand_tagged_f32(const PlanData& P, const DeviceTables& t, const double* G, int w, float* Om,
                              hipStream_t s);
void launch_to_f32(const double* x, int64_t n, float* y, hipStream_t s);
void launch_fill0(double* x, int64_t n, hipStream_t s);
// X (n x w) = columns c0 .. c0 + w - 1 of the identity.
void launch_unit_cols(double* X, int64_t n, int64_t c0, int64_t w, hipStream_t s);
void launch_far_gather(const PlanData& P, const DeviceTables& t, const double* W, int w, int j0, int j1,
                       double* S, hipStream_t s);
// Alg. 3 on a black box: masked test matrices of boxes [i0, i1) (N x (i1 - i0) r) and
// each box's own rows of their products.
void launch_expand_masked(const PlanData& P, const DeviceTables& t, const double* G, int i0, int i1,
                          double* Om, hipStream_t s);
void launch_take_box_rows(const PlanData& P, const DeviceTables& t, const double* Yc, int i0, int i1,
                          double* S, hipStream_t s);
// Alg. 1: S(row, :) = Y(row, :) P_box(row) with Y N x ns and P b blocks of ns x r.
// Alg. 1 null vectors on the device: P (b blocks of ns x r) from the N x ns test matrix;
// work holds bn_null_workspace_doubles(P, ns) doubles; flag[0] = 1 on a rank-deficient
// neighbour block (the caller zeroes it first).
int64_t bn_null_workspace_doubles(const PlanData& P, int64_t ns);
void launch_bn_null(const PlanData& P, const DeviceTables& t, const double* Om, int64_t ns, double* work,
                    double* Pall, double* flag, hipStream_t s);
void launch_bn_project(const PlanData& P, const DeviceTables& t, const double* Y, int64_t ns,
                       const double* Pall, double* S, hipStream_t s);
void launch_identity_probe(const PlanData& P, const DeviceTables& t, int c, double* X, hipStream_t s);
void launch_cores_from_w(const PlanData& P, const DeviceTables& t, const double* U, const double* W,
                         int j0, int j1, double* Atil, hipStream_t s);
void launch_nf_from_probe(const PlanData& P, const DeviceTables& t, const double* Pc, int c,
                          const double* U, const double* Qwork, double* Bv, hipStream_t s);
// First half of the near field: Q_ic = X_c^T V Atil_{i,:}^T into the workspace.
void launch_nf_q(const PlanData& P, const DeviceTables& t, const double* V, const double* Atil,
                 double* work, hipStream_t s);

// Near field; work must hold nearfield_workspace_doubles(P) doubles.
int64_t nearfield_workspace_doubles(const PlanData& P);
void launch_nearfield(const OpData& op, const PlanData& P, const DeviceTables& t, const double* U,
                      const double* V, const double* Atil, double* Bv, double* work, hipStream_t s);

// y = A_uBLR x (or its transpose); work must hold 2 * b*k*ncols + nsplit*b*k*ncols doubles
// (see apply_workspace_doubles).
int64_t apply_workspace_doubles(const PlanData& P, int64_t ncols);
void launch_ublr_apply(const PlanData& P, const DeviceTables& t, const double* U, const double* V,
                       const double* Atil, const double* Bv, int trans, int64_t ncols,
                       const double* x, int64_t ldx, double* y, int64_t ldy, double* work,
                       hipStream_t s);

// Per-pair partial sums ||E_ij||_F^2 and ||A_ij||_F^2 into part[2*b*b].
void launch_err_fro(const OpData& op, const PlanData& P, const DeviceTables& t, const double* U,
                    const double* V, const double* Atil, const double* Bv, double* part,
                    hipStream_t s);

// Truncation to per-box ranks (truncate.hip).  mode 0: far block rows of Atil, mode 1:
// far block columns; W receives b k x k rotations (columns by descending singular value)
// and sig b x k singular values.
void launch_trunc_svd(const PlanData& P, const DeviceTables& t, int mode, const double* Atil, double* W,
                      double* sig, hipStream_t s);
// Aout = blockdiag(W_i(:, 1:ku_i))^T Ain (rows beyond ku_i zero)
void launch_trunc_rows(const PlanData& P, const double* Ain, double* Aout, const double* W, const int32_t* ku,
                       hipStream_t s);
// A = A blockdiag(J_j(:, 1:kv_j)) in place (columns beyond kv_j zero)
void launch_trunc_cols(const PlanData& P, double* A, const double* Jm, const int32_t* kv, hipStream_t s);
// Sout(I_i, :) = S(I_i, :) W_i(:, 1:kr_i) (columns beyond kr_i zero)
void launch_trunc_basis(const PlanData& P, const DeviceTables& t, const double* S, double* Sout, const double* W,
                        const int32_t* kr, hipStream_t s);
// part[i b + j] = ||Atil_ij||_F^2
void launch_block_sq(const PlanData& P, const double* Atil, double* part, hipStream_t s);
// part[q] = ||U_i Atil_ij V_j^T + B_ij||_F^2 for each neighbour pair q
void launch_near_repr_sq(const PlanData& P, const DeviceTables& t, const double* U, const double* V,
                         const double* Atil, const double* Bv, double* part, hipStream_t s);
// Bout_ij = B_ij + U_i (Aold_ij - W_i Anew_ij J_j^T) V_j^T for each neighbour pair
void launch_trunc_near(const PlanData& P, const DeviceTables& t, const double* U, const double* V,
                       const double* Aold, const double* Anew, const double* W, const double* Jm,
                       const double* Bin, double* Bout, hipStream_t s);

// Deterministic dot product: part needs dot_parts() doubles; result in part[0].
int dot_parts();
void launch_dot(const double* x, const double* y, int64_t n, double* part, hipStream_t s);
// flag[0] (device) = 1 if any value of the given device arrays is not finite, else 0
void launch_flag_nonfinite(const double* const* arrays, const int64_t* counts, int narrays, double* flag,
                           hipStream_t s);
// y = a*x + y
void launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t s);
void launch_scale(double a, double* x, int64_t n, hipStream_t s);

}  // namespace blr
