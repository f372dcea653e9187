/*
 * blr_tag.h -- C ABI of the MI355X (gfx950) library for black-box compression
 * of strongly admissible uniform Block Low-Rank (uBLR) matrices by tagging.
 *
 * Method: Pearce, Yesypenko, Levitt, Martinsson, "Randomized Block Low-Rank
 * Matrix Compression by Tagging" (arXiv 2501.05528).  The operator A is known
 * only through products X -> A X and X -> A* X (Section 1).  Compression
 * follows Table 1, column reconstruct_tag:
 *   (I)  [U, V] = tag(A, A*, k)           Alg. 2 (sketch, tag post-processing, col)
 *   (II) Atil = U* (A V)                  bk products
 *   (III) B from 3^d sparse identity probes (eq. sparse_struct_ids)
 * giving A ~ U Atil V* + B (eq. uniformBLRfull, eq. discrepancymatrix).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Status: every function returns blr_status; BLR_OK is 0.  On error the
 *    out-pointers are set to NULL, nothing is leaked, and
 *    blr_last_error_message() (thread-local) describes the failure.  No C++
 *    exception crosses the ABI.
 *  * Memory: "host" pointers are ordinary CPU memory read synchronously
 *    during the call; "device" pointers are HIP device memory on the device
 *    current at the call.  The caller owns every pointer it passes; the
 *    library owns the objects it creates (plan, operator, ublr) until the
 *    matching destroy call.
 *  * Layouts: matrices are column-major FP64 with the given leading
 *    dimension unless stated.  Rows are in box-major order: box i owns rows
 *    [box_ptr[i], box_ptr[i+1]).
 *  * Streams: `stream` is a hipStream_t passed as void* (NULL = the default
 *    stream).  Device work is enqueued asynchronously on it; results are
 *    valid once the stream has been synchronised.  Arguments are validated
 *    synchronously before anything is enqueued.
 */
#ifndef BLR_TAG_H
#define BLR_TAG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum blr_status {
    BLR_OK = 0,
    BLR_ERR_INVALID_ARG = 1, /* bad sizes/pointers, k + p > min m_i, wrong T shape ... */
    BLR_ERR_GEOMETRY = 2,    /* some box has an empty far field, or T(N_i,:) is rank deficient */
    BLR_ERR_OOM = 3,         /* device or host allocation failed */
    BLR_ERR_DEVICE = 4,      /* a HIP runtime call failed */
    BLR_ERR_OPERATOR = 5,    /* a user operator callback returned nonzero */
    BLR_ERR_NUMERICAL = 6,   /* non-finite sketch or basis */
    BLR_ERR_BUSY = 7,        /* server admission refused (over budget) */
    BLR_ERR_UNSUPPORTED = 8  /* combination not implemented (e.g. precision for this operator) */
} blr_status;

typedef struct blr_plan blr_plan;
typedef struct blr_operator blr_operator;
typedef struct blr_ublr blr_ublr;

/* Human-readable name of a status code (static storage). */
const char* blr_status_string(blr_status s);
/* Message of the last failed call on this thread (empty if none). */
const char* blr_last_error_message(void);
/* Library version string. */
const char* blr_version(void);

/* ------------------------------------------------------------------ plan
 * Geometry of the tessellation (Section 2.5): b boxes with index sets I_i
 * and their integer coordinates on a d-dimensional box lattice.  Strong
 * admissibility: the neighbours N_i of box i are the boxes at lattice
 * Chebyshev distance <= 1 (those sharing a boundary, i included; at most
 * 3^d), the far field is F_i = [b] \ N_i.
 */
typedef struct blr_geometry {
    int32_t dim;                /* d in {1, 2, 3} */
    int32_t nboxes;             /* b >= 2 */
    const int64_t* box_ptr;     /* host, b+1 entries, box_ptr[0] = 0, strictly increasing */
    const int32_t* box_lattice; /* host, b*dim entries, box i at [i*dim, i*dim+dim); may be
                                   NULL when near_ptr is given */
    /* Optional neighbour lists N_i as host CSR (near_ptr: b+1 entries from 0; near_idx:
     * near_ptr[b] box indices).  Each list strictly ascending, i in N_i, and the relation
     * symmetric (j in N_i iff i in N_j); every far field F_i = [b] \ N_i non-empty.
     * NULL: strong admissibility on the lattice, N_i = boxes at Chebyshev lattice
     * distance <= 1 (Section 2.5), with probe colours sum_t (lat_t mod 3) 3^t.  With
     * explicit lists the probe colours of Table 1 step (III) are assigned greedily in box
     * order: box i takes the smallest colour not held by an earlier box that shares a
     * neighbour with it, so the neighbours of every box carry distinct colours.
     * Errors: BLR_ERR_INVALID_ARG (malformed lists), BLR_ERR_GEOMETRY (asymmetric lists,
     * empty far field). */
    const int32_t* near_ptr;
    const int32_t* near_idx;
} blr_geometry;

/*
 * Number of columns ell of the tagging matrix T for a geometry: one more
 * than the largest neighbour count (Section 4.1) plus `extra_tag_cols`
 * additional columns that give every tag submatrix a null space of
 * dimension >= extra_tag_cols + 1 (Section 5.3; the paper's experiments use
 * 3 additional columns, Section 7).  Host only.
 */
blr_status blr_tag_columns(const blr_geometry* geom, int32_t extra_tag_cols, int32_t* ell_out);

typedef struct blr_tag_params {
    int32_t k;              /* block rank, >= 1 */
    int32_t p;              /* oversampling, r = k + p; requires r <= min_i m_i */
    int32_t extra_tag_cols; /* >= 0; ell = max|N_i| + 1 + extra_tag_cols */
    int32_t aspect_opt;     /* 1: minimise the aspect ratio (Section 5.3, LP per sign cell);
                               0: use the projection of the first start vector */
    const double* T;        /* host, b x ell column-major Gaussian tagging matrix (Alg. 2);
                               the caller draws it so results are reproducible */
} blr_tag_params;

/*
 * Build a compression plan (host only, no device calls): neighbour and far
 * lists, probe colours, and for every box the unit tag vector
 * z^(i) in null(T(N_i,:)) (Alg. 2; eq. tagsubmat) chosen to minimise the
 * aspect ratio rho^(i) of its projected tags (eq. aspect_ratio).  The plan is
 * immutable, reusable across operators, streams and threads, and uploads its
 * device tables lazily on first use per device.
 * Errors: BLR_ERR_INVALID_ARG (shapes, k + p > min m_i, NULL T),
 *         BLR_ERR_GEOMETRY (empty far field, rank-deficient T(N_i,:)).
 */
blr_status blr_tag_plan(const blr_geometry* geom, const blr_tag_params* params, blr_plan** out);
void blr_plan_destroy(blr_plan* plan);

typedef struct blr_plan_info {
    int64_t n;          /* N = box_ptr[b] */
    int32_t nboxes;     /* b */
    int32_t dim;        /* d */
    int32_t k, p, r;    /* rank, oversampling, r = k + p */
    int32_t ell;        /* columns of T */
    int32_t m_max;      /* largest box */
    int32_t m_min;      /* smallest box */
    int32_t ncolours;   /* 3^d probe colours */
    int64_t near_nnz;   /* number of neighbour pairs (i, j in N_i) */
    int64_t b_values;   /* doubles needed for all near-field blocks of B */
} blr_plan_info;

blr_status blr_plan_query(const blr_plan* plan, blr_plan_info* info);

/*
 * Copy the plan's lists to host arrays (any pointer may be NULL to skip it).
 *   near_ptr [b+1], near_idx [near_nnz]: CSR of N_i, ascending, self included
 *   colour   [b]: probe colour sum_t (lat_t mod 3) 3^t
 *   b_offset [near_nnz]: offset (in doubles) of block B_ij in the B value
 *            array; block (i, j) is m_i x m_j column-major, pairs in CSR order
 */
blr_status blr_plan_lists(const blr_plan* plan, int32_t* near_ptr, int32_t* near_idx,
                          int32_t* colour, int64_t* b_offset);

/* Copy tag vectors z (b x ell, column-major) and aspect ratios rho [b] to host. */
blr_status blr_plan_tags(const blr_plan* plan, double* z, double* rho);

/* ------------------------------------------------------------- operators
 * The black box A (N x N).  Built-in operators are evaluated by fused HIP
 * kernels that never form A (kernel matrices) or read it in place (dense).
 */
typedef enum blr_kernel_kind {
    BLR_KERNEL_LOG = 0,   /* log|x - y|, diagonal 0 (Section 7.1) */
    BLR_KERNEL_INV_R = 1, /* 1/|x - y|, diagonal 0 */
    BLR_KERNEL_EXP = 2,   /* exp(-|x - y| / 0.1), diagonal 1 */
    BLR_KERNEL_COS = 3    /* cos(20|x - y|) / (|x - y| + 1e-3), diagonal 1000 */
} blr_kernel_kind;

/*
 * Dense operator: A is device memory, n x n column-major with leading
 * dimension lda >= n, borrowed (must outlive the operator and every call
 * that uses it).  A* products read A transposed in place.
 */
blr_status blr_op_dense_create(int64_t n, const double* A, int64_t lda, blr_operator** out);

/*
 * Kernel-matrix operator A_ij = kappa(|x_i - x_j|) (A_ii = the diagonal
 * value), evaluated on the fly.  pts is host memory, n x dim row-major
 * (point i at pts[i*dim ...]); the library keeps its own device copy.
 * The matrix is symmetric, so A* = A.
 */
blr_status blr_op_kernel_create(int32_t kind, int32_t dim, int64_t n, const double* pts,
                                blr_operator** out);

/*
 * The caller's products with A and A* (Section 2, the black-box setting of the
 * problem statement): apply must enqueue Y = A X (trans = 0) or Y = A* X
 * (trans = 1) on `stream`, X: n x ncols device memory (ldx >= n), Y likewise
 * (ldy >= n), and return 0, or nonzero on failure (reported as
 * BLR_ERR_OPERATOR).  It is called from the thread that called the library.
 */
typedef int32_t (*blr_apply_fn)(void* ctx, int32_t trans, int64_t ncols, const double* X,
                                int64_t ldx, double* Y, int64_t ldy, void* stream);

/*
 * Black-box operator: every stage forms its test matrix explicitly and calls
 * apply -- 2 ell r columns for the sketches (Alg. 2), b k for the cores
 * (Table 1 step 2, in chunks of boxes) and 3^d m_max for the near-field
 * probes (Table 1 step 3).  ctx is borrowed and must outlive the operator.
 * In the mixed-precision modes the low-precision tagged sketch uses the
 * optional FP32-operand products (blr_op_callback_set_lp), else the FP64
 * products rounded to FP32; the refinement sketch applies A and A* to
 * block-diagonal test columns (b r per side, in chunks of boxes) and sums each
 * row box's far blocks.  blr_error_fro takes the entries from N products with
 * unit columns.  Batches need entry access and return BLR_ERR_UNSUPPORTED for
 * such operators.
 */
blr_status blr_op_callback_create(int64_t n, blr_apply_fn apply, void* ctx, blr_operator** out);

/*
 * Low-precision products for the mixed-precision modes: apply_lp must enqueue
 * Y = A X (trans = 0) or A* X (trans = 1) on `stream` with X, Y FP32 device
 * arrays (n x ncols, ldx, ldy >= n), computing in `precision`
 * (BLR_PREC_FP32_REFINE: FP32 arithmetic; BLR_PREC_BF16_REFINE: BF16 operands
 * with FP32 accumulation, or anything at least as accurate), and return 0 or
 * nonzero (BLR_ERR_OPERATOR).  Optional; NULL removes it.  Only for operators
 * made by blr_op_callback_create.
 */
typedef int32_t (*blr_apply_lp_fn)(void* ctx, int32_t trans, int32_t precision, int64_t ncols, const float* X,
                                   int64_t ldx, float* Y, int64_t ldy, void* stream);
blr_status blr_op_callback_set_lp(blr_operator* op, blr_apply_lp_fn apply_lp);

/*
 * The thin-slab Schur complement of Section 7.2 as a library-held black box
 * (products only, like a callback operator).  Grid n x n x l (h = 1, zero
 * Dirichlet values outside), 7-point finite differences of -Laplace - kappa^2
 * (diagonal 6 - kappa_h^2, -1 per neighbour; the paper's 100 points per
 * wavelength is kappa_h = 2 pi / 100), frontal face z = l - 1, internal planes
 * eliminated: S = A_ff - A_fi A_ii^{-1} A_if, N = n^2, symmetric (A* = A).
 * perm: host array of N, perm[row] = x + n y, the face point of operator row
 * `row` (a permutation; copied).  Products use the separable exact solve: sine
 * transforms in the plane and one tridiagonal z-line pivot per mode pair.
 * Errors: n < 1, l < 1, bad perm, or an internal block that is not positive
 * definite (a resonant slab) give BLR_ERR_INVALID_ARG.  Every call that takes a
 * callback operator takes this one (batches return BLR_ERR_UNSUPPORTED).
 */
blr_status blr_op_slab_create(int32_t n, int32_t l, double kappa_h, const int64_t* perm, blr_operator** out);
void blr_op_destroy(blr_operator* op);

/*
 * Y = A X (trans = 0) or Y = A* X (trans = 1) for X (n x ncols, device,
 * ldx >= n) into Y (n x ncols, device, ldy >= n).  The operator's own
 * black-box product, exposed for error estimation and testing.
 */
blr_status blr_op_apply(const blr_operator* op, int32_t trans, int64_t ncols, const double* X,
                        int64_t ldx, double* Y, int64_t ldy, void* stream);

/* ------------------------------------------------------- compression stages
 * Stage entry points of reconstruct_tag; blr_tag_compress chains them.  All
 * arrays are device memory, column-major with leading dimension N.
 */

/*
 * Tagged sketches (Alg. 2, sketch step; eq. extend_test_mat): Y = A Omega
 * and Z = A* Psi, each N x (ell*r), where block column j of Omega has block
 * row i equal to T(i,j) G_i (G: N x r stacked G_i) and Psi likewise from H
 * with the same T.  Omega and Psi are formed inside the kernel and never
 * stored.  Y, Z: N x ell*r, leading dimension N.
 */
blr_status blr_sketch(const blr_plan* plan, const blr_operator* op, const double* G,
                      const double* H, double* Y, double* Z, void* stream);

/*
 * Tag post-processing (Alg. 2, loop over boxes; eq. projected_tags):
 * Yhat(I_i,:) = sum_j z^(i)_j Y(I_i, (j-1)r+1 : jr), which cancels every
 * near-field contribution, and Zhat likewise from Z.  Yhat, Zhat: N x r.
 * Y or Yhat (Z or Zhat) may be NULL to skip that side.
 */
blr_status blr_tag_postprocess(const blr_plan* plan, const double* Y, const double* Z,
                               double* Yhat, double* Zhat, void* stream);

/*
 * Per-box bases (Alg. 2, U_i = col(Yhat(I_i,:), k); Section 2.3): the k
 * dominant left singular vectors of each m_i x r block of S, by batched
 * one-sided Jacobi in FP64, sorted by singular value, each column signed so
 * that its entry of largest magnitude is positive.  S is overwritten
 * (scratch).  Q: N x k output.  sigma: optional device array b x r of the
 * block singular values (descending), or NULL.
 */
blr_status blr_orthonormalize(const blr_plan* plan, double* S, double* Q, double* sigma,
                              void* stream);

/*
 * Cores (Table 1 step 2): Atil = U* (A V) with U = diag(U_i), V = diag(V_j),
 * i.e. Atil_ij = U_i* A_ij V_j for every pair (far pairs are the cores
 * S_ij of eq. uniformBLRblock; near pairs feed step III).  Atil: bk x bk
 * column-major (leading dimension b*k).
 */
blr_status blr_cores(const blr_plan* plan, const blr_operator* op, const double* U,
                     const double* V, double* Atil, void* stream);

/*
 * Near-field remainder (Table 1 step 3; eq. sparse_struct_ids): for every
 * colour c the probe P_c = (A - U Atil V*) X_c with X_c the identity blocks
 * on the boxes of colour c, and B_il = P_c(I_i, 1:m_l) for the neighbour l
 * of box i of colour c.  Bvals: b_values doubles laid out by b_offset.
 */
blr_status blr_nearfield(const blr_plan* plan, const blr_operator* op, const double* U,
                         const double* V, const double* Atil, double* Bvals, void* stream);

/*
 * Mixed modes, step 1: the tagged sketches of Alg. 2 with r_lo columns per tag
 * column in low precision (precision = BLR_PREC_FP32_REFINE or
 * BLR_PREC_BF16_REFINE): kernel entries in FP32 (dense operators: A rounded to
 * FP32), each entry scaled by T(i, j) in FP32 and rounded to the MFMA type,
 * G and H rounded likewise, FP32 accumulation.  G, H: N x r_lo (ld N);
 * Y0, Z0: float N x ell r_lo (ld N).  Returns BLR_ERR_UNSUPPORTED for r_lo > 80.
 */
blr_status blr_sketch_lowp(const blr_plan* plan, const blr_operator* op, int32_t precision,
                           int32_t r_lo, const double* G, const double* H, float* Y0, float* Z0,
                           void* stream);

/*
 * Mixed modes, post-processing of the FP32 sketches (eq. projected_tags, in
 * FP64): Yhat0(I_i,:) = sum_j z^(i)_j Y0(I_i, (j-1)r_lo+1 : j r_lo), N x r_lo.
 * Either side may be NULL (input and output together).
 */
blr_status blr_tag_postprocess_lowp(const blr_plan* plan, int32_t r_lo, const float* Y0,
                                    const float* Z0, double* Yhat0, double* Zhat0, void* stream);

/*
 * Orthonormal bases of per-box samples: for every box the m_i x ncols block
 * of S (ncols <= m_min, <= 128) is factored by Householder QR in FP64 and Q
 * receives the Q factor's ncols columns, each signed so that its entry of
 * largest magnitude (lowest row on ties) is positive.  S is overwritten.
 */
blr_status blr_sample_bases(const blr_plan* plan, int32_t ncols, double* S, double* Q, void* stream);

/*
 * Mixed modes, step 3 (FP64 refinement sketch on the far field):
 *   SY(I_i) = sum_{l in F_i} A(I_i, I_l) V0(I_l) gamma_v[l],
 *   SZ(I_i) = sum_{l in F_i} A(I_l, I_i)* U0(I_l) gamma_u[l],
 * U0, V0: N x r_lo; gamma_u, gamma_v: b x r_lo x r C-ordered (see
 * blr_compress_opts); SY, SZ: N x r.  All device memory.
 */
blr_status blr_refine_sketch(const blr_plan* plan, const blr_operator* op, int32_t r_lo,
                             const double* U0, const double* V0, const double* gamma_u,
                             const double* gamma_v, double* SY, double* SZ, void* stream);

/* ------------------------------------------------------------ compression */
/*
 * Precision of step (I).  The mixed modes are not in the paper (which runs
 * every step in one precision):
 *   1. the tagged sketches of Alg. 2 are taken with r_lo = k + p_lo columns
 *      per tag column, kernel entries in FP32, contracted on FP32 or BF16 MFMA
 *      with FP32 accumulation, and stored in FP32;
 *   2. FP64 tag post-processing and FP64 Householder QR give orthonormal
 *      bases U0_i, V0_i of all r_lo sample columns;
 *   3. one FP64 refinement sketch on the far field: with the caller's r_lo x r
 *      Gaussian blocks gamma_v[l], gamma_u[l],
 *        SY(I_i) = sum_{l in F_i} A_il V0_l gamma_v[l],
 *        SZ(I_i) = sum_{l in F_i} A_li* U0_l gamma_u[l],
 *      and U_i = col(SY(I_i), k), V_i = col(SZ(I_i), k) (as in Alg. 2);
 *   4. steps (II)-(III) of Table 1 in FP64, unchanged.
 * Step 3 uses block-sparse products with A (2 b r columns for a black box).
 */
typedef enum blr_precision {
    BLR_PREC_FP64 = 0,        /* every stage in FP64 */
    BLR_PREC_FP32_REFINE = 1, /* step (I) on FP32 MFMA, then the FP64 refinement sketch */
    BLR_PREC_BF16_REFINE = 2  /* step (I) on BF16 MFMA (FP32 accumulation), then refinement */
} blr_precision;

typedef struct blr_compress_opts {
    int32_t precision;          /* blr_precision */
    int32_t keep_intermediates; /* 1: keep the sketches, samples and sample bases for inspection */
    int32_t r_lo;               /* mixed modes: columns of G and H (k + p_lo, <= m_min, <= 80);
                                   0 means r; ignored in FP64 */
    int32_t reserved;           /* must be 0 */
    /* mixed modes: device arrays b x r_lo x r, C-ordered (entry (a, c) of box l
       at (l*r_lo + a)*r + c): gamma_v mixes V0 for the U side, gamma_u mixes U0
       for the V side.  Ignored in FP64. */
    const double* gamma_u;
    const double* gamma_v;
} blr_compress_opts;

typedef struct blr_report {
    /* stage times (ms, device events on the stream); in the mixed modes
       ms_sketch and ms_postprocess cover the low-precision sketch */
    double ms_sketch, ms_postprocess, ms_orth, ms_cores, ms_nearfield, ms_total;
    /* products in the paper's convention (columns applied to A and to A*);
       the mixed modes add the refinement's b r block-sparse columns per side */
    int64_t applies_A, applies_At;
    /* algorithmic work of the sketch launch (4 N^2 ell r, or 4 N^2 ell r_lo) */
    double sketch_flops;
    /* aspect ratios of the plan */
    double rho_min, rho_median, rho_max;
    /* mixed modes: sample bases + mixing + refinement sketch (ms), the
       refinement's algorithmic work (4 r sum_i m_i |F_i|-block flops), the
       precision and r_lo used; zero in FP64 */
    double ms_refine, refine_flops;
    int32_t precision, r_lo;
} blr_report;

/*
 * Full compression reconstruct_tag (Table 1): steps (I)-(III).  G and H
 * (device, N x r column-major, ld N; N x r_lo in the mixed modes) are the
 * stacked Gaussian blocks G_i, H_i of Alg. 2 drawn by the caller.  opts may
 * be NULL (FP64, no intermediates).  On success *out owns device U, V
 * (N x k), Atil (bk x bk) and B (b_values doubles); it keeps a reference to
 * the plan.  If rep is non-NULL the call synchronises the stream, checks U,
 * V, Atil and B for non-finite values (BLR_ERR_NUMERICAL, no handle returned:
 * a non-finite sketch or basis shows up in them) and fills the report; without
 * a report nothing waits and nothing is checked.
 */
blr_status blr_tag_compress(const blr_plan* plan, const blr_operator* op, const double* G,
                            const double* H, const blr_compress_opts* opts, void* stream,
                            blr_ublr** out, blr_report* rep);

/*
 * Alg. 3 (the paper's basic randomized SVD for step (I)) followed by steps
 * (II)-(III) of Table 1: the comparison method that tagging replaces.  For
 * every box i, A is applied to Omega^(i) = G with the rows of every box in
 * N_i set to zero, and A* to Psi^(i) = H masked likewise; U_i and V_i are the
 * top-k left singular vectors of the box's own rows of the two products (the
 * same per-box basis routine as blr_tag_compress).  G and H (device, N x r
 * column-major, ld N) are shared by all boxes: each box's sample sees an
 * N(0,1) test matrix on its far field, which is all Alg. 3 uses.  Costs b r
 * columns on each of A and A* (reported in applies_A / applies_At; ms_sketch
 * covers all of them, ms_postprocess is 0).  keep_samples != 0 keeps the
 * N x r per-box samples as BLR_PART_SY / BLR_PART_SZ.  Ownership, report and
 * error behaviour as for blr_tag_compress (FP64 only, any operator).
 */
blr_status blr_basic_compress(const blr_plan* plan, const blr_operator* op, const double* G,
                              const double* H, int32_t keep_samples, void* stream, blr_ublr** out,
                              blr_report* rep);

/*
 * Alg. 1 (block nullification for basis construction) followed by steps
 * (II)-(III) of Table 1: the method tagging improves on (Section 3).  One
 * sketch Y = A Omega, Z = A* Psi on s columns; for every box i, P^(i) = r
 * orthonormal vectors of null(Omega^(i)), where Omega^(i) stacks the rows of
 * the neighbour boxes (ascending box order), taken from the Householder QR of
 * Omega^(i)* (reflector signs that avoid cancellation; P^(i) = the r columns of
 * the orthogonal factor after its first |rows of N_i| columns); U_i = the
 * top-k left singular vectors of Y(I_i,:) P^(i), V_i likewise from Z and Psi.
 * Omega and Psi: device, N x s column-major, ld N; s >= blr_bn_min_columns
 * (r plus the rows of the largest neighbourhood, i.e. r + 3^d m on a uniform
 * tessellation; at most 2048 + r, else BLR_ERR_UNSUPPORTED) or
 * BLR_ERR_INVALID_ARG.  The null vectors are computed on the device, one
 * workgroup per box and side, in a stream-ordered workspace of b s (s - r)
 * doubles; a rank-deficient neighbour block gives BLR_ERR_NUMERICAL (the call
 * synchronises the stream to check).  Report: applies_A = s + b k + (colours)
 * m_max, applies_At = s; ms_sketch covers the two sketches, ms_postprocess the
 * null vectors and projections.
 * keep_samples != 0 keeps Y(I_i,:) P^(i) and Z(I_i,:) Q^(i) as BLR_PART_SY /
 * BLR_PART_SZ.  Ownership and errors as for blr_tag_compress (FP64, any operator).
 */
blr_status blr_bn_min_columns(const blr_plan* plan, int64_t* s);
blr_status blr_bn_compress(const blr_plan* plan, const blr_operator* op, int64_t s, const double* Omega,
                           const double* Psi, int32_t keep_samples, void* stream, blr_ublr** out,
                           blr_report* rep);

/*
 * A uniform rank from a singular-value threshold on the tagged samples (Section
 * 2.3: the range finder can pick its rank from a tolerance).  One tagged sketch
 * and post-processing at the plan's r = k + p columns (Alg. 2), then the
 * singular values of every box's m_i x r samples Yhat_i and Zhat_i.  *k_out =
 * the largest over boxes and sides of #{j : sigma_j(box) > tol * the largest
 * singular value of that side over all boxes}: the smallest uniform rank that
 * keeps every sample direction above the threshold.  *k_out = r means the
 * threshold was not reached within the sample (plan again with a larger k).
 * This is a per-direction threshold, not an error bound: the relative Frobenius
 * error summed over all b^2 blocks at rank *k_out can exceed tol (about 5 tol
 * on the 2D Laplace workload).  For a guaranteed tolerance compress at a larger
 * k and call blr_ublr_truncate.
 * G, H as for blr_tag_compress.  sigma: optional host array 2 x b x r
 * (Y side then Z side, each box's values descending).  Synchronises the
 * stream; tol < 0 or NaN gives BLR_ERR_INVALID_ARG, non-finite samples
 * BLR_ERR_NUMERICAL.  Any operator.
 */
blr_status blr_tag_rank(const blr_plan* plan, const blr_operator* op, const double* G, const double* H,
                        double tol, void* stream, int32_t* k_out, double* sigma);
void blr_ublr_destroy(blr_ublr* h);

/* Which device array of a compressed handle. */
typedef enum blr_ublr_part {
    BLR_PART_U = 0,     /* N x k */
    BLR_PART_V = 1,     /* N x k */
    BLR_PART_ATIL = 2,  /* bk x bk */
    BLR_PART_B = 3,     /* b_values */
    BLR_PART_Y = 4,     /* N x ell r   (keep_intermediates only) */
    BLR_PART_Z = 5,     /* N x ell r   (keep_intermediates only) */
    BLR_PART_YHAT = 6,  /* N x r  (N x r_lo in the mixed modes)  (keep_intermediates only) */
    BLR_PART_ZHAT = 7,  /* N x r  (N x r_lo in the mixed modes)  (keep_intermediates only) */
    BLR_PART_Y0 = 8,    /* float, N x ell r_lo: low-precision sketch  (mixed, keep_intermediates) */
    BLR_PART_Z0 = 9,    /* float, N x ell r_lo                        (mixed, keep_intermediates) */
    BLR_PART_U0 = 10,   /* N x r_lo sample bases                      (mixed, keep_intermediates) */
    BLR_PART_V0 = 11,   /* N x r_lo                                   (mixed, keep_intermediates) */
    BLR_PART_SY = 12,   /* N x r refinement samples (mixed, keep_intermediates); per-box samples of blr_basic_compress */
    BLR_PART_SZ = 13    /* N x r                                      (mixed, keep_intermediates) */
} blr_ublr_part;

/* Device pointer and element count of one part (the handle keeps ownership);
 * elements are double except for BLR_PART_Y0 and BLR_PART_Z0 (float). */
blr_status blr_ublr_part_ptr(const blr_ublr* h, int32_t part, const void** ptr, int64_t* count);

/*
 * Copies one part to host memory (element type and count as for
 * blr_ublr_part_ptr; `count` must equal the part's count).  Waits for the
 * copy on `stream` before returning.
 */
blr_status blr_ublr_export(const blr_ublr* h, int32_t part, void* host, int64_t count, void* stream);

/*
 * Per-box ranks from a tolerance by truncating a compressed operator (Section 6:
 * ranks can be chosen larger and truncated afterwards; Section 2.4: the range
 * finder can work to a tolerance).  From h (any precision), a new handle *out
 * whose far field is cut to the smallest per-box ranks that keep the change of
 * the represented matrix within tol ||A_uBLR||_F:
 *   rows: per box i the SVD of the far block row Atil(i, F_i); over all boxes
 *   the smallest singular values are dropped while their squares sum to at
 *   most half of (tol ||A_uBLR||_F)^2; U'_i = U_i W_i(:, 1:ku_i) and the block
 *   row is rotated and cut likewise;
 *   columns: the same on the far block columns of the row-truncated cores with
 *   the rest of the budget (V'_j, kv_j);
 *   near pairs: B'_ij = B_ij + U_i Atil_ij V_j* - U'_i Atil'_ij V'_j*, so every
 *   near block is represented as before.
 * The change of the far field is exactly the dropped squares (the two projections
 * are orthogonal), so ||A_uBLR' - A_uBLR||_F <= tol ||A_uBLR||_F and the error
 * against A grows by at most that much.  Layout stays uniform: U', V' are N x k
 * with the columns beyond the box's rank zero, Atil' bk x bk with the matching
 * rows and columns zero; apply, export and error calls work unchanged.
 * ranks_u, ranks_v: optional host arrays of b; rel_change: optional,
 * sqrt(dropped squares) / ||A_uBLR||_F.  h stays valid; *out is owned by the
 * caller.  Synchronises the stream.  tol < 0 or not finite: BLR_ERR_INVALID_ARG;
 * k > 64: BLR_ERR_UNSUPPORTED.
 */
blr_status blr_ublr_truncate(const blr_ublr* h, double tol, void* stream, blr_ublr** out, int32_t* ranks_u,
                             int32_t* ranks_v, double* rel_change);

/* Per-box ranks of a handle (host arrays of b): k everywhere unless truncated. */
blr_status blr_ublr_ranks(const blr_ublr* h, int32_t* ranks_u, int32_t* ranks_v);

/*
 * y = A_uBLR x = U (Atil (V* x)) + B x (trans = 0) or A_uBLR* x (trans = 1)
 * (eq. uniformBLRfull), x: N x ncols device (ldx >= N), y: N x ncols device
 * (ldy >= N), 1 <= ncols <= 65535 (0 does nothing).  The workspace
 * ((2 + s) b k ncols doubles, s the column split of the Atil product) is allocated
 * stream-ordered on `stream` for the call, so calls on one handle may run on
 * different streams at the same time.  Vectors go in groups of up to 16 that
 * read Atil and B once per group.
 */
blr_status blr_apply(const blr_ublr* h, int32_t trans, int64_t ncols, const double* x, int64_t ldx,
                     double* y, int64_t ldy, void* stream);

/*
 * blr_apply without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, results and kernels as blr_apply; the
 * workspace lives in a fixed 32 MiB array (4194304 doubles) that the library
 * holds on every device it runs on until the process ends.  A call whose
 * workspace ((2 + s) b k ncols doubles) exceeds that returns
 * BLR_ERR_INVALID_ARG naming the limit (split the columns over several calls).
 * All calls on one device share the array: calls that overlap in time on one
 * device (other streams, other threads) race and must be serialised by the
 * caller; calls queued on one stream are ordered.  Nothing in the array needs
 * to start at zero (every word a call reads, the same call writes first).
 */
blr_status blr_apply_noalloc(const blr_ublr* h, int32_t trans, int64_t ncols, const double* x,
                             int64_t ldx, double* y, int64_t ldy, void* stream);

/*
 * Exact relative Frobenius error ||A - A_uBLR||_F / ||A||_F (evaluation
 * harness; not part of the black-box method; Section 7's error metric).
 * Built-in operators: block by block with entry access.  Black-box operators:
 * from N products A e_j (unit columns in chunks of at most 512) against the
 * representation applied to the same columns, which costs N products.
 * Synchronises the stream.
 */
blr_status blr_error_fro(const blr_ublr* h, const blr_operator* op, void* stream, double* rel_err);

/*
 * The paper's accuracy metric (Section 7): ||A - A_uBLR||_2 / ||A||_2, each
 * norm by `iters` power iterations on M* M started from the given unit-norm
 * device vector x0 (N).  Only operator and uBLR products are used.
 * Synchronises the stream.  Outputs may be NULL.
 */
blr_status blr_error_power(const blr_ublr* h, const blr_operator* op, const double* x0,
                           int32_t iters, void* stream, double* err_norm, double* a_norm);

/* ----------------------------------------------------- batches of compressions
 * Many independent compressions of uneven N, box size, rank and kernel in one
 * object (not in the paper: the batched form of Table 1's reconstruct_tag).
 */

/*
 * Device bytes one blr_tag_compress call needs on `plan` in the given precision
 * (r_lo as in blr_compress_opts, 0 means r): the handle's outputs U, V, Atil, B
 * plus every temporary of the call.  Used for admission by HBM budget.
 */
blr_status blr_plan_footprint(const blr_plan* plan, int32_t precision, int32_t r_lo, int64_t* bytes);

typedef struct blr_batch blr_batch;

typedef struct blr_batch_job {
    const blr_plan* plan;
    const blr_operator* op;   /* built-in operator (dense or kernel); borrowed */
    const double* G;          /* device N x r (FP64) or N x r_lo (mixed); borrowed */
    const double* H;
    blr_compress_opts opts;   /* precision, r_lo, gamma_u, gamma_v (device, borrowed) */
} blr_batch_job;

enum {
    BLR_BATCH_GRAPH = 1,      /* capture the whole batch into a HIP graph on the second run
                                 and replay it on every later run */
    BLR_BATCH_AUTOTUNE = 2    /* first run: time each candidate tile shape of the persistent
                                 sketch per class and keep the fastest (cached per device) */
};

#define BLR_BATCH_MAX_CLASSES 32

typedef struct blr_batch_report {
    double ms_total;          /* the batch on the device (events on the batch stream) */
    double ms_sketch;         /* the persistent sketch launches (0 when a graph is replayed) */
    double sketch_flops;      /* sum over jobs of 4 N^2 ell r_lo (4 N^2 ell r for FP64 jobs) */
    double refine_flops;      /* sum over mixed jobs of the refinement's far-field flops */
    int64_t applies;          /* sum over jobs of the products in the paper's convention */
    int32_t graph_replayed;   /* 1 if this run replayed the captured graph */
    int32_t nclasses;         /* persistent sketch launches: one per (precision, 16-column tiles)
                                 and, for FP64, per kernel kind and form of the last column tile */
    int32_t class_precision[BLR_BATCH_MAX_CLASSES], class_ntr[BLR_BATCH_MAX_CLASSES];
    int32_t class_spw[BLR_BATCH_MAX_CLASSES];   /* tag columns per wave of the launch */
    int32_t class_jobs[BLR_BATCH_MAX_CLASSES];
    int32_t class_kind[BLR_BATCH_MAX_CLASSES];  /* blr_kernel_kind of an FP64 class, -1 otherwise */
    int32_t class_tail[BLR_BATCH_MAX_CLASSES];  /* FP64 class: 3 when the last 16-column tile (at
                                                   most 12 of the r columns) runs in the narrow form,
                                                   the choice blr_tag_compress makes for the same
                                                   kernel kind and r; else 0 */
} blr_batch_report;

/*
 * Plans the batch and allocates every output and temporary up front (no device
 * allocation happens in blr_batch_run).  Kernel-matrix jobs share persistent sketch
 * launches whose workgroups stride over (job, row block, tag column group) items,
 * heaviest job first: mixed-precision jobs one launch per (precision, 16-column
 * tiles of r_lo) class (32-row blocks, every kernel kind in one launch), FP64 jobs
 * one per (16-column tiles of r, kernel kind, last-tile form) class (8-row blocks).
 * At most BLR_BATCH_MAX_CLASSES classes (else BLR_ERR_UNSUPPORTED).  Every other stage
 * runs per job, the jobs spread over up to 4 streams of the batch (default priority)
 * forked after the sketches; jobs on dense operators use the single-job sketch
 * kernels.  Black-box
 * (callback) operators are not supported (BLR_ERR_UNSUPPORTED).  flags:
 * BLR_BATCH_GRAPH, BLR_BATCH_AUTOTUNE (low-precision classes only).
 */
blr_status blr_batch_create(int32_t njobs, const blr_batch_job* jobs, int32_t flags, blr_batch** out);

/*
 * Runs every compression of the batch on the batch's own streams, ordered after
 * the work already on `stream`; `stream` waits for the batch.  Results (and the
 * report) are valid after `stream` is synchronised.  Each job's arithmetic does not
 * depend on the other jobs, so its results equal those of blr_tag_compress on the
 * same inputs.
 */
blr_status blr_batch_run(blr_batch* b, void* stream, blr_batch_report* rep);

/* The compressed handle of job `job` (owned by the batch, valid until destroy). */
blr_status blr_batch_result(const blr_batch* b, int32_t job, const blr_ublr** h);

void blr_batch_destroy(blr_batch* b);

/* ------------------------------------------------------------ serving
 * A request loop for compression jobs (not in the paper): jobs are admitted in
 * arrival order as a slot and enough of the HBM budget are free, run
 * concurrently on the slots' own streams, and complete independently.
 */
typedef struct blr_server blr_server;

typedef struct blr_server_job_stats {
    double t_submit, t_start, t_end;   /* host monotonic clock, seconds */
    double ms_device;                  /* the job's compression on its stream (events) */
    double dev_start_ms, dev_end_ms;   /* the job's interval on its slot's stream (device
                                          events, ms since the server was created; -1 if
                                          the events failed) */
    int64_t footprint;                 /* bytes charged against the budget while it runs */
    int32_t slot;                      /* slot that ran the job */
    int32_t status;                    /* blr_status of the job */
} blr_server_job_stats;

/*
 * Creates a server on the current device with `slots` concurrent jobs (1..16, each
 * with its own stream) and an HBM budget in bytes for the admitted jobs' footprints
 * (blr_plan_footprint).  A running job is charged its whole footprint; once it
 * completes, its result (U, V, Atil, B; the whole footprint with
 * keep_intermediates) stays charged until blr_server_wait hands it over, so
 * results that nobody claims hold budget and can stall admission.
 */
blr_status blr_server_create(int64_t hbm_budget, int32_t slots, blr_server** out);

/*
 * Queues one compression (arguments as for blr_tag_compress; plan, op, G, H and
 * the gamma arrays are borrowed until the job completes).  Returns BLR_ERR_BUSY if
 * the job's footprint exceeds the whole budget.  *ticket identifies the job.
 */
blr_status blr_server_submit(blr_server* srv, const blr_plan* plan, const blr_operator* op,
                             const double* G, const double* H, const blr_compress_opts* opts,
                             uint64_t* ticket);

/* *done = 1 once the job has completed (successfully or not). */
blr_status blr_server_poll(blr_server* srv, uint64_t ticket, int32_t* done);

/*
 * Waits for the job, hands over its compressed handle (*out, owned by the caller;
 * NULL if the job failed) and fills stats (nullable); returns the job's status.
 * Each ticket can be waited for once.
 */
blr_status blr_server_wait(blr_server* srv, uint64_t ticket, blr_ublr** out,
                           blr_server_job_stats* stats);

/* Waits for every queued job, then releases the server (unclaimed handles are freed). */
void blr_server_destroy(blr_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* BLR_TAG_H */
