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
void launch_op_apply(const OpData& op, int trans, int64_t ncols, const double* X, int64_t ldx,
                     double* Y, int64_t ldy, hipStream_t s);

void launch_postprocess(const PlanData& P, const DeviceTables& t, const double* Y, double* Yhat,
                        hipStream_t s);

void launch_orth(const PlanData& P, const DeviceTables& t, double* S, double* Q, double* sigma,
                 hipStream_t s);
// Both sides in one launch (S1/Q1 may be null for one side).
void launch_orth2(const PlanData& P, const DeviceTables& t, double* S0, double* S1, double* Q0,
                  double* Q1, double* sig0, double* sig1, hipStream_t s);

void launch_cores(const OpData& op, const PlanData& P, const DeviceTables& t, const double* U,
                  const double* V, double* Atil, hipStream_t s);

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

// Deterministic dot product: part needs dot_parts() doubles; result in part[0].
int dot_parts();
void launch_dot(const double* x, const double* y, int64_t n, double* part, hipStream_t s);
// y = a*x + y
void launch_axpy(double a, const double* x, double* y, int64_t n, hipStream_t s);
void launch_scale(double a, double* x, int64_t n, hipStream_t s);

}  // namespace blr
