// Internal types shared by the host planner, the C ABI glue and the HIP
// kernels of the tagged uBLR library.  Not part of the public ABI.
#pragma once

#include <cstdint>
#include <memory>
#include <mutex>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/blr_tag.h"

namespace blr {

// Internal failures are thrown as Error and converted to a status code at
// the ABI boundary (no exception crosses it).
struct Error : std::runtime_error {
    blr_status status;
    Error(blr_status s, const std::string& m) : std::runtime_error(m), status(s) {}
};
[[noreturn]] inline void fail(blr_status s, const std::string& m) { throw Error(s, m); }

void set_last_error(const std::string& msg);

// Device copies of a plan's tables (one set per device that used the plan).
struct DeviceTables {
    int device = -1;
    int64_t* box_ptr = nullptr;      // [b+1]
    int32_t* row_box = nullptr;      // [N] box of each row
    double* T = nullptr;             // [b*ell] row-major (T(i, s) at i*ell + s)
    double* z = nullptr;             // [b*ell] row-major tag vectors
    int32_t* near_ptr = nullptr;     // [b+1]
    int32_t* near_idx = nullptr;     // [nnz]
    int32_t* near_tpos = nullptr;    // [nnz] index of pair (j, i) for pair (i, j)
    int64_t* b_off = nullptr;        // [nnz] offsets of B blocks
    int32_t* colour_ptr = nullptr;   // [ncol+1] CSR of boxes per colour
    int32_t* colour_boxes = nullptr; // [b]
    int32_t* nf_pair = nullptr;      // [b*ncol] near pair index of (i, colour) or -1
    float* Tf = nullptr;             // [b*ell] row-major T in FP32 (low-precision sketch)
    int32_t* kstep_ptr = nullptr;    // [b+1] first 32-row source step of each box
    int32_t* kstep_box = nullptr;    // [nsteps] box of each 32-row source step
    uint8_t* nearm = nullptr;        // [b*b] 1 if box j is in N_i (i-major)
    int32_t* colour = nullptr;       // [b] probe colour of each box
    int32_t* pair_row = nullptr;     // [nnz] row box i of neighbour pair q
    void release();
};

struct PlanData {
    int dim = 0, b = 0, k = 0, p = 0, r = 0, ell = 0, extra = 0, ncol = 0;
    int m_max = 0, m_min = 0;
    int aspect_opt = 1;
    int64_t n = 0, near_nnz = 0, b_values = 0;
    std::vector<int64_t> box_ptr;
    std::vector<int32_t> lattice;
    std::vector<int32_t> near_ptr, near_idx, near_tpos, colour, colour_ptr, colour_boxes, nf_pair, row_box;
    std::vector<int64_t> b_off;
    std::vector<int32_t> kstep_ptr, kstep_box;  // 32-row source steps per box
    std::vector<uint8_t> nearm;                 // b x b neighbour mask
    std::vector<int32_t> pair_row;              // row box of each neighbour pair
    bool custom_near = false;                   // neighbour lists given by the caller
    std::vector<double> T;    // column-major b x ell (as supplied)
    std::vector<double> z;    // column-major b x ell
    std::vector<double> rho;  // [b]

    std::mutex mu;
    std::vector<std::unique_ptr<DeviceTables>> dev;
    const DeviceTables& tables();  // tables for the current device (uploads on first use)
    const DeviceTables* resident_tables();  // tables for the current device if uploaded, else NULL
    ~PlanData();
};

// Bytes of a compressed handle's outputs U, V (N x k each), Atil (bk x bk) and B.
inline int64_t result_bytes(const PlanData& P) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    return static_cast<int64_t>(sizeof(double)) * (2 * P.n * P.k + bk * bk + P.b_values);
}

// Thin-slab Schur complement operator (slab.hip): a library-owned black box.  Returns its
// context and sets the product callback and the context's release function.
void* slab_create(int n, int l, double kappa_h, const int64_t* perm, int64_t N, blr_apply_fn* fn,
                  void (**free_fn)(void*));

// Host planner (plan.cpp).
std::shared_ptr<PlanData> build_plan(const blr_geometry* g, const blr_tag_params* prm);
int tag_columns(const blr_geometry* g, int extra);

// Block nullification (bn.cpp): the smallest test-matrix width that leaves r null
// vectors for every box.
int64_t bn_min_columns(const PlanData& P);

// Operators.
enum class OpType { Dense, Kernel, Callback };
struct OpData {
    OpType type = OpType::Dense;
    int64_t n = 0;
    int kind = 0;                 // blr_kernel_kind
    int dim = 0;
    const double* A = nullptr;    // dense, borrowed
    int64_t lda = 0;
    double* pts = nullptr;        // kernel: device SoA [3][n] (unused axes zero), owned
    float* pts32 = nullptr;       // kernel: the same points in FP32 (+32 zeros at the end), owned
    blr_apply_fn fn = nullptr;    // callback: the caller's products with A and A*
    blr_apply_lp_fn fn_lp = nullptr;  // callback: optional FP32-operand products (mixed modes)
    void* ctx = nullptr;          // callback: the caller's context, borrowed
    void (*ctx_free)(void*) = nullptr;  // set when the library owns ctx (built-in black boxes)
    int device = -1;
    ~OpData();
};

struct UblrData {
    std::shared_ptr<PlanData> plan;
    int device = -1;
    double* U = nullptr;
    double* V = nullptr;
    double* Atil = nullptr;
    double* B = nullptr;
    double* Y = nullptr;
    double* Z = nullptr;
    double* Yhat = nullptr;
    double* Zhat = nullptr;
    int precision = BLR_PREC_FP64;
    int r_lo = 0;                 // sample columns of the low-precision sketch
    float* Y0 = nullptr;          // mixed modes, keep_intermediates: FP32 sketches
    float* Z0 = nullptr;
    double* U0 = nullptr;         // mixed modes, keep_intermediates: sample bases (N x r_lo)
    double* V0 = nullptr;
    double* SY = nullptr;         // mixed modes, keep_intermediates: refinement samples (N x r)
    double* SZ = nullptr;
    std::vector<int32_t> ranks_u, ranks_v;  // per-box ranks after truncation (empty: all k)
    ~UblrData();
};

}  // namespace blr

struct blr_plan { std::shared_ptr<blr::PlanData> d; };
struct blr_operator { std::unique_ptr<blr::OpData> d; };
struct blr_ublr { std::unique_ptr<blr::UblrData> d; };
