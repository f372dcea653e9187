// C ABI of the tagged uBLR library (declared in include/blr_tag.h): argument
// validation, ownership, device tables, stage sequencing and reporting.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <tuple>
#include <mutex>
#include <map>
#include <cmath>
#include <cstring>
#include <sstream>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"

// Workspace of blr_apply_noalloc: one fixed array per device, resident until the
// process ends.  Host code never passes `scratch` itself to a kernel (on the host
// it names a stand-in, not device memory); it uses the per-device address that
// noalloc_scratch() obtains with hipGetSymbolAddress.
constexpr int64_t kNoAllocScratchDoubles = int64_t(1) << 22;   // 32 MiB
static __device__ __align__(256) double scratch[kNoAllocScratchDoubles];

namespace blr {

namespace {
thread_local std::string g_last_error;

#define HIPC(x)                                                                          \
    do {                                                                                 \
        hipError_t e_ = (x);                                                             \
        if (e_ != hipSuccess) fail(BLR_ERR_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

template <class T>
T* upload(const std::vector<T>& v) {
    T* p = nullptr;
    const size_t n = std::max<size_t>(1, v.size());
    if (hipMalloc(&p, n * sizeof(T)) != hipSuccess) fail(BLR_ERR_OOM, "device allocation of plan tables");
    if (!v.empty()) HIPC(hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice));
    return p;
}

template <class T>
void dfree(T*& p) {
    if (p) (void)hipFree(p);
    p = nullptr;
}

double* dalloc(int64_t count, hipStream_t s) {
    void* p = nullptr;
    const size_t bytes = static_cast<size_t>(std::max<int64_t>(1, count)) * sizeof(double);
    if (hipMallocAsync(&p, bytes, s) != hipSuccess) {
        (void)hipGetLastError();
        std::ostringstream os;
        os << "device allocation of " << bytes << " bytes failed";
        fail(BLR_ERR_OOM, os.str());
    }
    return static_cast<double*>(p);
}

double* dalloc_sync(int64_t count) {
    void* p = nullptr;
    const size_t bytes = static_cast<size_t>(std::max<int64_t>(1, count)) * sizeof(double);
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        std::ostringstream os;
        os << "device allocation of " << bytes << " bytes failed";
        fail(BLR_ERR_OOM, os.str());
    }
    return static_cast<double*>(p);
}

// Frees stream-ordered temporaries when a call leaves (normally or by error).
// Buffers handed to a caller's apply callback come from plain(): ordinary device
// allocations rather than stream-ordered pool memory, so that any framework the
// callback uses can wrap them.
struct AsyncTemps {
    hipStream_t s;
    std::vector<double*> ptrs, plain_ptrs;
    explicit AsyncTemps(hipStream_t st) : s(st) {}
    double* get(int64_t count) {
        ptrs.push_back(dalloc(count, s));
        return ptrs.back();
    }
    double* plain(int64_t count) {
        plain_ptrs.push_back(dalloc_sync(count));
        return plain_ptrs.back();
    }
    ~AsyncTemps() {
        for (double* p : ptrs) (void)hipFreeAsync(p, s);
        if (!plain_ptrs.empty()) {
            (void)hipStreamSynchronize(s);
            for (double* p : plain_ptrs) (void)hipFree(p);
        }
    }
};

int current_device() {
    int d = -1;
    HIPC(hipGetDevice(&d));
    return d;
}

// Device address of `scratch` on device `dev` (the current device), looked up once per
// device; every kernel argument and copy uses this address, never the array's name.
double* noalloc_scratch(int dev) {
    static std::mutex mu;
    static std::map<int, double*> addr;
    std::lock_guard<std::mutex> lock(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
        (void)hipGetLastError();
        fail(BLR_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    }
    addr[dev] = static_cast<double*>(p);
    return static_cast<double*>(p);
}

const blr::PlanData& plan_of(const blr_plan* p) {
    if (!p || !p->d) fail(BLR_ERR_INVALID_ARG, "NULL plan");
    return *p->d;
}

const blr::OpData& op_of(const blr_operator* o, const PlanData& P) {
    if (!o || !o->d) fail(BLR_ERR_INVALID_ARG, "NULL operator");
    if (o->d->n != P.n) fail(BLR_ERR_INVALID_ARG, "operator size differs from the plan's N");
    if (o->d->device != current_device()) fail(BLR_ERR_INVALID_ARG, "operator belongs to another device");
    return *o->d;
}

template <class F>
blr_status guard(F&& f) {
    try {
        f();
        g_last_error.clear();
        return BLR_OK;
    } catch (const Error& e) {
        g_last_error = e.what();
        return e.status;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return BLR_ERR_OOM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return BLR_ERR_INVALID_ARG;
    } catch (...) {
        g_last_error = "unknown error";
        return BLR_ERR_INVALID_ARG;
    }
}

void check_ld(int64_t ld, int64_t n, const char* what) {
    if (ld < n) fail(BLR_ERR_INVALID_ARG, std::string(what) + " leading dimension is smaller than N");
}

// ---- operator dispatch: built-in operators run fused kernels; a black-box
// operator gets explicit test matrices and the caller's products.
bool is_callback(const OpData& o) { return o.type == OpType::Callback; }

void require_entries(const OpData& o, const char* what) {
    if (is_callback(o))
        fail(BLR_ERR_UNSUPPORTED, std::string(what) + " needs entry access, which a black-box operator does not give");
}

void op_apply(const OpData& o, int trans, int64_t ncols, const double* X, int64_t ldx, double* Y,
              int64_t ldy, hipStream_t s) {
    if (!is_callback(o)) {
        const int64_t nw = op_apply_workspace_doubles(o, ncols);
        AsyncTemps tmp(s);
        launch_op_apply(o, trans, ncols, X, ldx, Y, ldy, nw > 0 ? tmp.get(nw) : nullptr, s);
        return;
    }
    const int32_t rc = o.fn(o.ctx, trans, ncols, X, ldx, Y, ldy, static_cast<void*>(s));
    if (rc != 0) {
        std::ostringstream os;
        os << "operator apply returned " << rc;
        fail(BLR_ERR_OPERATOR, os.str());
    }
}

// Columns of a block-diagonal test matrix per call: about 2^27 doubles (1 GiB).
int boxes_per_chunk(const PlanData& P, int w) {
    const int64_t per_box = P.n * static_cast<int64_t>(std::max(1, w));
    return static_cast<int>(std::max<int64_t>(1, std::min<int64_t>(P.b, (int64_t(1) << 27) / per_box)));
}

void sketch_any(const OpData& o, const PlanData& P, const DeviceTables& t, const double* G,
                const double* H, double* Y, double* Z, hipStream_t s, AsyncTemps& tmp) {
    if (!is_callback(o)) {
        launch_sketch(o, P, t, G, H, Y, Z, s);
        return;
    }
    const int64_t LR = static_cast<int64_t>(P.ell) * P.r;
    double* Om = tmp.plain(P.n * LR);
    double* Yo = tmp.plain(P.n * LR);
    launch_expand_tagged(P, t, G, Om, s);
    op_apply(o, 0, LR, Om, P.n, Yo, P.n, s);
    HIPC(hipMemcpyAsync(Y, Yo, P.n * LR * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_expand_tagged(P, t, H, Om, s);
    op_apply(o, 1, LR, Om, P.n, Yo, P.n, s);
    HIPC(hipMemcpyAsync(Z, Yo, P.n * LR * sizeof(double), hipMemcpyDeviceToDevice, s));
}

void cores_any(const OpData& o, const PlanData& P, const DeviceTables& t, const double* U,
               const double* V, double* Atil, hipStream_t s, AsyncTemps& tmp) {
    if (!is_callback(o)) {
        launch_cores(o, P, t, U, V, Atil, s);
        return;
    }
    const int cb = boxes_per_chunk(P, P.k);
    double* X = tmp.plain(P.n * static_cast<int64_t>(cb) * P.k);
    double* W = tmp.plain(P.n * static_cast<int64_t>(cb) * P.k);
    for (int j0 = 0; j0 < P.b; j0 += cb) {
        const int j1 = std::min(P.b, j0 + cb);
        launch_embed_blockdiag(P, t, V, P.k, j0, j1, X, s);
        op_apply(o, 0, static_cast<int64_t>(j1 - j0) * P.k, X, P.n, W, P.n, s);
        launch_cores_from_w(P, t, U, W, j0, j1, Atil, s);
    }
}

void nearfield_any(const OpData& o, const PlanData& P, const DeviceTables& t, const double* U,
                   const double* V, const double* Atil, double* Bv, hipStream_t s, AsyncTemps& tmp) {
    double* work = tmp.get(nearfield_workspace_doubles(P));
    if (!is_callback(o)) {
        launch_nearfield(o, P, t, U, V, Atil, Bv, work, s);
        return;
    }
    launch_nf_q(P, t, V, Atil, work, s);
    double* X = tmp.plain(P.n * static_cast<int64_t>(P.m_max));
    double* Pc = tmp.plain(P.n * static_cast<int64_t>(P.m_max));
    for (int c = 0; c < P.ncol; ++c) {
        launch_identity_probe(P, t, c, X, s);
        op_apply(o, 0, P.m_max, X, P.n, Pc, P.n, s);
        launch_nf_from_probe(P, t, Pc, c, U, work, Bv, s);
    }
}

}  // namespace

void set_last_error(const std::string& msg) { g_last_error = msg; }

void DeviceTables::release() {
    dfree(box_ptr);
    dfree(row_box);
    dfree(T);
    dfree(z);
    dfree(near_ptr);
    dfree(near_idx);
    dfree(near_tpos);
    dfree(b_off);
    dfree(colour_ptr);
    dfree(colour_boxes);
    dfree(nf_pair);
    dfree(Tf);
    dfree(kstep_ptr);
    dfree(kstep_box);
    dfree(nearm);
    dfree(colour);
    dfree(pair_row);
}

const DeviceTables* PlanData::resident_tables() {
    const int devid = current_device();
    std::lock_guard<std::mutex> lock(mu);
    for (auto& t : dev)
        if (t->device == devid) return t.get();
    return nullptr;
}

const DeviceTables& PlanData::tables() {
    const int devid = current_device();
    std::lock_guard<std::mutex> lock(mu);
    for (auto& t : dev)
        if (t->device == devid) return *t;
    auto t = std::make_unique<DeviceTables>();
    t->device = devid;
    try {
        std::vector<double> Trm(static_cast<size_t>(b) * ell), zrm(static_cast<size_t>(b) * ell);
        for (int i = 0; i < b; ++i)
            for (int s = 0; s < ell; ++s) {
                Trm[static_cast<size_t>(i) * ell + s] = T[i + static_cast<size_t>(s) * b];
                zrm[static_cast<size_t>(i) * ell + s] = z[i + static_cast<size_t>(s) * b];
            }
        t->box_ptr = upload(box_ptr);
        t->row_box = upload(row_box);
        t->T = upload(Trm);
        t->z = upload(zrm);
        t->near_ptr = upload(near_ptr);
        t->near_idx = upload(near_idx);
        t->near_tpos = upload(near_tpos);
        t->b_off = upload(b_off);
        t->colour_ptr = upload(colour_ptr);
        t->colour_boxes = upload(colour_boxes);
        t->nf_pair = upload(nf_pair);
        std::vector<float> Tf(Trm.begin(), Trm.end());
        t->Tf = upload(Tf);
        t->kstep_ptr = upload(kstep_ptr);
        t->kstep_box = upload(kstep_box);
        t->nearm = upload(nearm);
        t->colour = upload(colour);
        t->pair_row = upload(pair_row);
    } catch (...) {
        t->release();
        throw;
    }
    dev.push_back(std::move(t));
    return *dev.back();
}

PlanData::~PlanData() {
    if (dev.empty()) return;
    int cur = -1;
    (void)hipGetDevice(&cur);
    for (auto& t : dev) {
        (void)hipSetDevice(t->device);
        t->release();
    }
    if (cur >= 0) (void)hipSetDevice(cur);
}

OpData::~OpData() {
    dfree(pts);
    dfree(pts32);
    if (ctx_free && ctx) ctx_free(ctx);
}

UblrData::~UblrData() {
    dfree(U);
    dfree(V);
    dfree(Atil);
    dfree(B);
    dfree(Y);
    dfree(Z);
    dfree(Yhat);
    dfree(Zhat);
    dfree(Y0);
    dfree(Z0);
    dfree(U0);
    dfree(V0);
    dfree(SY);
    dfree(SZ);
}

}  // namespace blr

using namespace blr;

extern "C" {

const char* blr_status_string(blr_status s) {
    switch (s) {
        case BLR_OK: return "BLR_OK";
        case BLR_ERR_INVALID_ARG: return "BLR_ERR_INVALID_ARG";
        case BLR_ERR_GEOMETRY: return "BLR_ERR_GEOMETRY";
        case BLR_ERR_OOM: return "BLR_ERR_OOM";
        case BLR_ERR_DEVICE: return "BLR_ERR_DEVICE";
        case BLR_ERR_OPERATOR: return "BLR_ERR_OPERATOR";
        case BLR_ERR_NUMERICAL: return "BLR_ERR_NUMERICAL";
        case BLR_ERR_BUSY: return "BLR_ERR_BUSY";
        case BLR_ERR_UNSUPPORTED: return "BLR_ERR_UNSUPPORTED";
    }
    return "BLR_ERR_UNKNOWN";
}

const char* blr_last_error_message(void) { return g_last_error.c_str(); }

const char* blr_version(void) { return "blrtag-mi355x 0.1 (gfx950)"; }

blr_status blr_tag_columns(const blr_geometry* geom, int32_t extra_tag_cols, int32_t* ell_out) {
    if (ell_out) *ell_out = 0;
    return guard([&] {
        if (!ell_out) fail(BLR_ERR_INVALID_ARG, "NULL output");
        *ell_out = tag_columns(geom, extra_tag_cols);
    });
}

blr_status blr_tag_plan(const blr_geometry* geom, const blr_tag_params* params, blr_plan** out) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out) fail(BLR_ERR_INVALID_ARG, "NULL output");
        auto d = build_plan(geom, params);
        // T must have exactly ell columns; the caller sized it with blr_tag_columns.
        auto* p = new blr_plan;
        p->d = std::move(d);
        *out = p;
    });
}

void blr_plan_destroy(blr_plan* plan) { delete plan; }

blr_status blr_plan_query(const blr_plan* plan, blr_plan_info* info) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        if (!info) fail(BLR_ERR_INVALID_ARG, "NULL info");
        info->n = P.n;
        info->nboxes = P.b;
        info->dim = P.dim;
        info->k = P.k;
        info->p = P.p;
        info->r = P.r;
        info->ell = P.ell;
        info->m_max = P.m_max;
        info->m_min = P.m_min;
        info->ncolours = P.ncol;
        info->near_nnz = P.near_nnz;
        info->b_values = P.b_values;
    });
}

blr_status blr_plan_lists(const blr_plan* plan, int32_t* near_ptr, int32_t* near_idx,
                          int32_t* colour, int64_t* b_offset) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        if (near_ptr) std::copy(P.near_ptr.begin(), P.near_ptr.end(), near_ptr);
        if (near_idx) std::copy(P.near_idx.begin(), P.near_idx.end(), near_idx);
        if (colour) std::copy(P.colour.begin(), P.colour.end(), colour);
        if (b_offset) std::copy(P.b_off.begin(), P.b_off.end(), b_offset);
    });
}

blr_status blr_plan_tags(const blr_plan* plan, double* z, double* rho) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        if (z) std::copy(P.z.begin(), P.z.end(), z);
        if (rho) std::copy(P.rho.begin(), P.rho.end(), rho);
    });
}

blr_status blr_op_dense_create(int64_t n, const double* A, int64_t lda, blr_operator** out) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out || !A) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        if (n <= 0 || lda < n) fail(BLR_ERR_INVALID_ARG, "need n > 0 and lda >= n");
        auto d = std::make_unique<OpData>();
        d->type = OpType::Dense;
        d->n = n;
        d->A = A;
        d->lda = lda;
        d->device = current_device();
        auto* o = new blr_operator;
        o->d = std::move(d);
        *out = o;
    });
}

blr_status blr_op_kernel_create(int32_t kind, int32_t dim, int64_t n, const double* pts,
                                blr_operator** out) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out || !pts) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        if (kind < BLR_KERNEL_LOG || kind > BLR_KERNEL_COS) fail(BLR_ERR_INVALID_ARG, "unknown kernel kind");
        if (dim < 1 || dim > 3 || n <= 0) fail(BLR_ERR_INVALID_ARG, "need 1 <= dim <= 3 and n > 0");
        std::vector<double> soa(static_cast<size_t>(3) * n, 0.0);
        for (int64_t i = 0; i < n; ++i)
            for (int t = 0; t < dim; ++t) {
                const double v = pts[i * dim + t];
                if (!std::isfinite(v)) fail(BLR_ERR_INVALID_ARG, "non-finite point coordinate");
                soa[static_cast<size_t>(t) * n + i] = v;
            }
        auto d = std::make_unique<OpData>();
        d->type = OpType::Kernel;
        d->n = n;
        d->kind = kind;
        d->dim = dim;
        d->device = current_device();
        d->pts = dalloc_sync(3 * n);
        HIPC(hipMemcpy(d->pts, soa.data(), soa.size() * sizeof(double), hipMemcpyHostToDevice));
        // FP32 copy with 32 zero entries past the end: the low-precision sketch loads a
        // step's 32 source columns without clamping them to the box
        std::vector<float> soa32(soa.begin(), soa.end());
        soa32.resize(soa32.size() + 32, 0.0f);
        d->pts32 = reinterpret_cast<float*>(dalloc_sync((static_cast<int64_t>(soa32.size()) + 1) / 2));
        HIPC(hipMemcpy(d->pts32, soa32.data(), soa32.size() * sizeof(float), hipMemcpyHostToDevice));
        auto* o = new blr_operator;
        o->d = std::move(d);
        *out = o;
    });
}

blr_status blr_op_callback_create(int64_t n, blr_apply_fn apply, void* ctx, blr_operator** out) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out || !apply) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        if (n <= 0) fail(BLR_ERR_INVALID_ARG, "need n > 0");
        auto d = std::make_unique<OpData>();
        d->type = OpType::Callback;
        d->n = n;
        d->fn = apply;
        d->ctx = ctx;
        d->device = current_device();
        auto* o = new blr_operator;
        o->d = std::move(d);
        *out = o;
    });
}

blr_status blr_op_callback_set_lp(blr_operator* op, blr_apply_lp_fn apply_lp) {
    return guard([&] {
        if (!op || !op->d) fail(BLR_ERR_INVALID_ARG, "NULL operator");
        if (op->d->type != OpType::Callback) fail(BLR_ERR_INVALID_ARG, "not a callback operator");
        op->d->fn_lp = apply_lp;
    });
}

blr_status blr_op_slab_create(int32_t n, int32_t l, double kappa_h, const int64_t* perm, blr_operator** out) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        auto d = std::make_unique<OpData>();
        d->type = OpType::Callback;
        d->n = static_cast<int64_t>(n) * n;
        d->device = current_device();
        d->ctx = slab_create(n, l, kappa_h, perm, d->n, &d->fn, &d->ctx_free);
        auto* o = new blr_operator;
        o->d = std::move(d);
        *out = o;
    });
}

void blr_op_destroy(blr_operator* op) { delete op; }

blr_status blr_op_apply(const blr_operator* op, int32_t trans, int64_t ncols, const double* X,
                        int64_t ldx, double* Y, int64_t ldy, void* stream) {
    return guard([&] {
        if (!op || !op->d) fail(BLR_ERR_INVALID_ARG, "NULL operator");
        const OpData& o = *op->d;
        if (ncols < 0) fail(BLR_ERR_INVALID_ARG, "negative ncols");
        if (ncols == 0) return;
        if (!X || !Y) fail(BLR_ERR_INVALID_ARG, "NULL X or Y");
        check_ld(ldx, o.n, "X");
        check_ld(ldy, o.n, "Y");
        if (o.device != current_device()) fail(BLR_ERR_INVALID_ARG, "operator belongs to another device");
        op_apply(o, trans ? 1 : 0, ncols, X, ldx, Y, ldy, static_cast<hipStream_t>(stream));
    });
}

blr_status blr_sketch(const blr_plan* plan, const blr_operator* op, const double* G,
                      const double* H, double* Y, double* Z, void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!G || !H || !Y || !Z) fail(BLR_ERR_INVALID_ARG, "NULL G, H, Y or Z");
        const DeviceTables& t = plan->d->tables();
        hipStream_t s = static_cast<hipStream_t>(stream);
        AsyncTemps tmp(s);
        sketch_any(o, P, t, G, H, Y, Z, s, tmp);
    });
}

blr_status blr_tag_postprocess(const blr_plan* plan, const double* Y, const double* Z,
                               double* Yhat, double* Zhat, void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        if ((Y == nullptr) != (Yhat == nullptr) || (Z == nullptr) != (Zhat == nullptr))
            fail(BLR_ERR_INVALID_ARG, "input and output of a side must both be given");
        const DeviceTables& t = plan->d->tables();
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (Y) launch_postprocess(P, t, Y, Yhat, s);
        if (Z) launch_postprocess(P, t, Z, Zhat, s);
    });
}

blr_status blr_orthonormalize(const blr_plan* plan, double* S, double* Q, double* sigma,
                              void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        if (!S || !Q) fail(BLR_ERR_INVALID_ARG, "NULL S or Q");
        const DeviceTables& t = plan->d->tables();
        launch_orth(P, t, S, Q, sigma, static_cast<hipStream_t>(stream));
    });
}

blr_status blr_cores(const blr_plan* plan, const blr_operator* op, const double* U,
                     const double* V, double* Atil, void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!U || !V || !Atil) fail(BLR_ERR_INVALID_ARG, "NULL U, V or Atil");
        const DeviceTables& t = plan->d->tables();
        hipStream_t s = static_cast<hipStream_t>(stream);
        AsyncTemps tmp(s);
        cores_any(o, P, t, U, V, Atil, s, tmp);
    });
}

blr_status blr_nearfield(const blr_plan* plan, const blr_operator* op, const double* U,
                         const double* V, const double* Atil, double* Bvals, void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!U || !V || !Atil || !Bvals) fail(BLR_ERR_INVALID_ARG, "NULL U, V, Atil or B");
        const DeviceTables& t = plan->d->tables();
        hipStream_t s = static_cast<hipStream_t>(stream);
        AsyncTemps tmp(s);
        nearfield_any(o, P, t, U, V, Atil, Bvals, s, tmp);
    });
}

namespace {

bool is_mixed(int precision) {
    return precision == BLR_PREC_FP32_REFINE || precision == BLR_PREC_BF16_REFINE;
}

void check_r_lo(const PlanData& P, int r_lo) {
    if (r_lo < 1 || r_lo > 80) fail(BLR_ERR_UNSUPPORTED, "r_lo must be in 1..80");
    if (r_lo > P.m_min) fail(BLR_ERR_INVALID_ARG, "r_lo exceeds the smallest box size");
}

// Packs G (N x r_lo) for the low-precision sketch into a stream-ordered temporary.
void* pack_lp(AsyncTemps& tmp, const PlanData& P, const DeviceTables& t, int precision, int r_lo,
              const double* G, hipStream_t s) {
    const int64_t elems = lp_packed_elems(P, r_lo);
    const int64_t bytes = elems * (precision == BLR_PREC_BF16_REFINE ? 2 : 4);
    void* out = tmp.get((bytes + 7) / 8);
    launch_pack_lp(P, t, precision, r_lo, G, out, s);
    return out;
}

// 4 r sum_i m_i (N - sum_{l in N_i} m_l): the far-field products of both sides.
double refine_flops(const PlanData& P) {
    double f = 0.0;
    for (int i = 0; i < P.b; ++i) {
        double nearcols = 0.0;
        for (int q = P.near_ptr[i]; q < P.near_ptr[i + 1]; ++q) {
            const int j = P.near_idx[q];
            nearcols += static_cast<double>(P.box_ptr[j + 1] - P.box_ptr[j]);
        }
        f += static_cast<double>(P.box_ptr[i + 1] - P.box_ptr[i]) * (static_cast<double>(P.n) - nearcols);
    }
    return 4.0 * P.r * f;
}

// Low-precision tagged sketch (mixed modes) through a black box: the caller's FP32-operand
// products when it offers them, else its FP64 products rounded to FP32.
void sketch_lp_blackbox(const OpData& o, const PlanData& P, const DeviceTables& t, int precision, int r_lo,
                        const double* G, const double* H, float* Y0, float* Z0, hipStream_t s, AsyncTemps& tmp) {
    const int64_t LR = static_cast<int64_t>(P.ell) * r_lo;
    const int64_t nf = (P.n * LR + 1) / 2;
    if (o.fn_lp) {
        float* Om = reinterpret_cast<float*>(tmp.plain(nf));
        float* Yo = reinterpret_cast<float*>(tmp.plain(nf));
        for (int side = 0; side < 2; ++side) {
            launch_expand_tagged_f32(P, t, side ? H : G, r_lo, Om, s);
            const int32_t rc = o.fn_lp(o.ctx, side, precision, LR, Om, P.n, Yo, P.n, static_cast<void*>(s));
            if (rc != 0) {
                std::ostringstream os;
                os << "operator low-precision apply returned " << rc;
                fail(BLR_ERR_OPERATOR, os.str());
            }
            HIPC(hipMemcpyAsync(side ? Z0 : Y0, Yo, P.n * LR * sizeof(float), hipMemcpyDeviceToDevice, s));
        }
        return;
    }
    double* Om = tmp.plain(P.n * LR);
    double* Yo = tmp.plain(P.n * LR);
    for (int side = 0; side < 2; ++side) {
        launch_expand_tagged_w(P, t, side ? H : G, r_lo, Om, s);
        op_apply(o, side, LR, Om, P.n, Yo, P.n, s);
        launch_to_f32(Yo, P.n * LR, side ? Z0 : Y0, s);
    }
}

// Refinement sketch through a black box: A (or A*) applied to block-diagonal test columns
// (the mixing blocks X_l of every box, in chunks of boxes), then the far blocks of each
// row box summed: S(I_i) = sum_{l in F_i} A_il X_l (2 b r columns over both sides).
void refine_blackbox(const OpData& o, const PlanData& P, const DeviceTables& t, const double* Xv,
                     const double* Xu, double* SY, double* SZ, hipStream_t s, AsyncTemps& tmp) {
    const int cb = boxes_per_chunk(P, P.r);
    double* X = tmp.plain(P.n * static_cast<int64_t>(cb) * P.r);
    double* W = tmp.plain(P.n * static_cast<int64_t>(cb) * P.r);
    for (int side = 0; side < 2; ++side) {
        const double* Xs = side ? Xu : Xv;
        double* S = side ? SZ : SY;
        launch_fill0(S, P.n * P.r, s);
        for (int j0 = 0; j0 < P.b; j0 += cb) {
            const int j1 = std::min(P.b, j0 + cb);
            launch_embed_blockdiag(P, t, Xs, P.r, j0, j1, X, s);
            op_apply(o, side, static_cast<int64_t>(j1 - j0) * P.r, X, P.n, W, P.n, s);
            launch_far_gather(P, t, W, P.r, j0, j1, S, s);
        }
    }
}

}  // namespace

blr_status blr_sketch_lowp(const blr_plan* plan, const blr_operator* op, int32_t precision,
                           int32_t r_lo, const double* G, const double* H, float* Y0, float* Z0,
                           void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!is_mixed(precision)) fail(BLR_ERR_INVALID_ARG, "precision must be a mixed mode");
        check_r_lo(P, r_lo);
        if (!G || !H || !Y0 || !Z0) fail(BLR_ERR_INVALID_ARG, "NULL G, H, Y0 or Z0");
        const DeviceTables& t = plan->d->tables();
        hipStream_t s = static_cast<hipStream_t>(stream);
        AsyncTemps tmp(s);
        if (is_callback(o)) {
            sketch_lp_blackbox(o, P, t, precision, r_lo, G, H, Y0, Z0, s, tmp);
            return;
        }
        void* PG = pack_lp(tmp, P, t, precision, r_lo, G, s);
        void* PH = pack_lp(tmp, P, t, precision, r_lo, H, s);
        launch_sketch_lp(o, P, t, precision, r_lo, PG, PH, Y0, Z0, s);
    });
}

blr_status blr_tag_postprocess_lowp(const blr_plan* plan, int32_t r_lo, const float* Y0,
                                    const float* Z0, double* Yhat0, double* Zhat0, void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        check_r_lo(P, r_lo);
        if ((Y0 == nullptr) != (Yhat0 == nullptr) || (Z0 == nullptr) != (Zhat0 == nullptr))
            fail(BLR_ERR_INVALID_ARG, "input and output of a side must both be given");
        const DeviceTables& t = plan->d->tables();
        hipStream_t s = static_cast<hipStream_t>(stream);
        if (Y0) launch_postprocess_lp(P, t, r_lo, Y0, Yhat0, s);
        if (Z0) launch_postprocess_lp(P, t, r_lo, Z0, Zhat0, s);
    });
}

blr_status blr_sample_bases(const blr_plan* plan, int32_t ncols, double* S, double* Q, void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        if (!S || !Q) fail(BLR_ERR_INVALID_ARG, "NULL S or Q");
        if (ncols < 1) fail(BLR_ERR_INVALID_ARG, "ncols must be positive");
        const DeviceTables& t = plan->d->tables();
        launch_orth_cols(P, t, ncols, ncols, 1, S, nullptr, Q, nullptr, nullptr, nullptr,
                         static_cast<hipStream_t>(stream));
    });
}

blr_status blr_refine_sketch(const blr_plan* plan, const blr_operator* op, int32_t r_lo,
                             const double* U0, const double* V0, const double* gamma_u,
                             const double* gamma_v, double* SY, double* SZ, void* stream) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        check_r_lo(P, r_lo);
        if (!U0 || !V0 || !gamma_u || !gamma_v || !SY || !SZ) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        const DeviceTables& t = plan->d->tables();
        hipStream_t s = static_cast<hipStream_t>(stream);
        AsyncTemps tmp(s);
        double* Xv = tmp.get(P.n * P.r);
        double* Xu = tmp.get(P.n * P.r);
        launch_mix(P, t, r_lo, V0, gamma_v, Xv, s);
        launch_mix(P, t, r_lo, U0, gamma_u, Xu, s);
        if (is_callback(o)) refine_blackbox(o, P, t, Xv, Xu, SY, SZ, s, tmp);
        else launch_refine(o, P, t, Xv, Xu, SY, SZ, s);
    });
}

blr_status blr_tag_compress(const blr_plan* plan, const blr_operator* op, const double* G,
                            const double* H, const blr_compress_opts* opts, void* stream,
                            blr_ublr** out, blr_report* rep) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out) fail(BLR_ERR_INVALID_ARG, "NULL output");
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!G || !H) fail(BLR_ERR_INVALID_ARG, "NULL G or H");
        blr_compress_opts def{};
        def.precision = BLR_PREC_FP64;
        const blr_compress_opts& O = opts ? *opts : def;
        const bool mixed = is_mixed(O.precision);
        if (!mixed && O.precision != BLR_PREC_FP64) fail(BLR_ERR_UNSUPPORTED, "unsupported precision");
        if (O.reserved != 0) fail(BLR_ERR_INVALID_ARG, "reserved option field must be 0");
        const int r_lo = mixed ? (O.r_lo ? O.r_lo : P.r) : P.r;
        if (mixed) {
            check_r_lo(P, r_lo);
            if (!O.gamma_u || !O.gamma_v) fail(BLR_ERR_INVALID_ARG, "mixed modes need gamma_u and gamma_v");
        }
        hipStream_t s = static_cast<hipStream_t>(stream);
        const DeviceTables& t = plan->d->tables();
        const int64_t LR = static_cast<int64_t>(P.ell) * r_lo;
        const int64_t bk = static_cast<int64_t>(P.b) * P.k;
        const bool keep = O.keep_intermediates != 0;

        auto h = std::make_unique<UblrData>();
        h->plan = plan->d;
        h->device = current_device();
        h->precision = O.precision;
        h->r_lo = r_lo;
        h->U = dalloc_sync(P.n * P.k);
        h->V = dalloc_sync(P.n * P.k);
        h->Atil = dalloc_sync(bk * bk);
        h->B = dalloc_sync(P.b_values);
        AsyncTemps tmp(s);

        const bool timing = rep != nullptr;
        struct Events {  // destroyed on every exit, errors included
            hipEvent_t e[8] = {};
            ~Events() {
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } evs;
        hipEvent_t* ev = evs.e;
        if (timing)
            for (int q = 0; q < 8; ++q) HIPC(hipEventCreate(&ev[q]));
        auto mark = [&](int q) {
            if (timing) HIPC(hipEventRecord(ev[q], s));
        };
        auto keep_copy = [&](double*& dst, const double* src, int64_t count) {
            dst = dalloc_sync(count);
            HIPC(hipMemcpyAsync(dst, src, count * sizeof(double), hipMemcpyDeviceToDevice, s));
        };
        // events: 0 start | 1 sketch | 2 post-processing | 3 sample bases + mixing |
        //         4 refinement | 5 bases | 6 cores | 7 near field
        if (!mixed) {
            double *Y, *Z;
            if (keep) {
                h->Y = Y = dalloc_sync(P.n * LR);
                h->Z = Z = dalloc_sync(P.n * LR);
            } else {
                Y = tmp.get(P.n * LR);
                Z = tmp.get(P.n * LR);
            }
            double* Yh = tmp.get(P.n * P.r);
            double* Zh = tmp.get(P.n * P.r);
            mark(0);
            sketch_any(o, P, t, G, H, Y, Z, s, tmp);
            mark(1);
            launch_postprocess(P, t, Y, Yh, s);
            launch_postprocess(P, t, Z, Zh, s);
            if (keep) {
                keep_copy(h->Yhat, Yh, P.n * P.r);
                keep_copy(h->Zhat, Zh, P.n * P.r);
            }
            mark(2);
            mark(3);
            mark(4);
            launch_orth2(P, t, Yh, Zh, h->U, h->V, nullptr, nullptr, s);
        } else {
            const int64_t nf = (P.n * LR + 1) / 2;  // FP32 sketch in doubles
            float *Y0, *Z0;
            if (keep) {
                h->Y0 = Y0 = reinterpret_cast<float*>(dalloc_sync(nf));
                h->Z0 = Z0 = reinterpret_cast<float*>(dalloc_sync(nf));
            } else {
                Y0 = reinterpret_cast<float*>(tmp.get(nf));
                Z0 = reinterpret_cast<float*>(tmp.get(nf));
            }
            double* Yh = tmp.get(P.n * r_lo);
            double* Zh = tmp.get(P.n * r_lo);
            double* U0 = tmp.get(P.n * r_lo);
            double* V0 = tmp.get(P.n * r_lo);
            double* Xv = tmp.get(P.n * P.r);
            double* Xu = tmp.get(P.n * P.r);
            double* SY = tmp.get(P.n * P.r);
            double* SZ = tmp.get(P.n * P.r);
            mark(0);
            if (is_callback(o)) {
                sketch_lp_blackbox(o, P, t, O.precision, r_lo, G, H, Y0, Z0, s, tmp);
            } else {
                void* PG = pack_lp(tmp, P, t, O.precision, r_lo, G, s);
                void* PH = pack_lp(tmp, P, t, O.precision, r_lo, H, s);
                launch_sketch_lp(o, P, t, O.precision, r_lo, PG, PH, Y0, Z0, s);
            }
            mark(1);
            launch_postprocess_lp(P, t, r_lo, Y0, Yh, s);
            launch_postprocess_lp(P, t, r_lo, Z0, Zh, s);
            if (keep) {
                keep_copy(h->Yhat, Yh, P.n * r_lo);
                keep_copy(h->Zhat, Zh, P.n * r_lo);
            }
            mark(2);
            launch_orth_cols(P, t, r_lo, r_lo, 1, Yh, Zh, U0, V0, nullptr, nullptr, s);
            launch_mix(P, t, r_lo, V0, O.gamma_v, Xv, s);
            launch_mix(P, t, r_lo, U0, O.gamma_u, Xu, s);
            if (keep) {
                keep_copy(h->U0, U0, P.n * r_lo);
                keep_copy(h->V0, V0, P.n * r_lo);
            }
            mark(3);
            if (is_callback(o)) refine_blackbox(o, P, t, Xv, Xu, SY, SZ, s, tmp);
            else launch_refine(o, P, t, Xv, Xu, SY, SZ, s);
            mark(4);
            if (keep) {
                keep_copy(h->SY, SY, P.n * P.r);
                keep_copy(h->SZ, SZ, P.n * P.r);
            }
            launch_orth2(P, t, SY, SZ, h->U, h->V, nullptr, nullptr, s);
        }
        mark(5);
        cores_any(o, P, t, h->U, h->V, h->Atil, s, tmp);
        mark(6);
        nearfield_any(o, P, t, h->U, h->V, h->Atil, h->B, s, tmp);
        mark(7);
        if (timing) {
            // with a report the call waits for the device anyway: check U, V, Atil and B
            double* flag = tmp.get(1);
            const double* arrs[4] = {h->U, h->V, h->Atil, h->B};
            const int64_t cnts[4] = {P.n * P.k, P.n * P.k, bk * bk, P.b_values};
            launch_flag_nonfinite(arrs, cnts, 4, flag, s);
            double hflag = 0.0;
            HIPC(hipMemcpyAsync(&hflag, flag, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (hflag != 0.0)
                fail(BLR_ERR_NUMERICAL, "non-finite values in the compressed operator (sketch, bases, cores or near field)");
            float ms[7];
            for (int q = 0; q < 7; ++q) HIPC(hipEventElapsedTime(&ms[q], ev[q], ev[q + 1]));
            float tot;
            HIPC(hipEventElapsedTime(&tot, ev[0], ev[7]));
            std::memset(rep, 0, sizeof(*rep));
            rep->ms_sketch = ms[0];
            rep->ms_postprocess = ms[1];
            rep->ms_orth = ms[2] + ms[4];
            rep->ms_refine = ms[3];
            rep->ms_cores = ms[5];
            rep->ms_nearfield = ms[6];
            rep->ms_total = tot;
            const int64_t refine_cols = mixed ? static_cast<int64_t>(P.b) * P.r : 0;
            rep->applies_A = LR + refine_cols + bk + static_cast<int64_t>(P.ncol) * P.m_max;
            rep->applies_At = LR + refine_cols;
            rep->sketch_flops = 4.0 * static_cast<double>(P.n) * static_cast<double>(P.n) * static_cast<double>(LR);
            rep->refine_flops = mixed ? refine_flops(P) : 0.0;
            rep->precision = O.precision;
            rep->r_lo = mixed ? r_lo : 0;
            std::vector<double> rho = P.rho;
            std::sort(rho.begin(), rho.end());
            rep->rho_min = rho.front();
            rep->rho_max = rho.back();
            rep->rho_median = rho[rho.size() / 2];
        }
        auto* hh = new blr_ublr;
        hh->d = std::move(h);
        *out = hh;
    });
}

blr_status blr_basic_compress(const blr_plan* plan, const blr_operator* op, const double* G,
                              const double* H, int32_t keep_samples, void* stream, blr_ublr** out,
                              blr_report* rep) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out) fail(BLR_ERR_INVALID_ARG, "NULL output");
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!G || !H) fail(BLR_ERR_INVALID_ARG, "NULL G or H");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const DeviceTables& t = plan->d->tables();
        const int64_t bk = static_cast<int64_t>(P.b) * P.k;

        auto h = std::make_unique<UblrData>();
        h->plan = plan->d;
        h->device = current_device();
        h->precision = BLR_PREC_FP64;
        h->U = dalloc_sync(P.n * P.k);
        h->V = dalloc_sync(P.n * P.k);
        h->Atil = dalloc_sync(bk * bk);
        h->B = dalloc_sync(P.b_values);
        AsyncTemps tmp(s);
        // the basis routine overwrites its input: kept samples are copies
        double* SY = tmp.get(P.n * P.r);
        double* SZ = tmp.get(P.n * P.r);

        const bool timing = rep != nullptr;
        struct Events {
            hipEvent_t e[5] = {};
            ~Events() {
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } evs;
        hipEvent_t* ev = evs.e;
        if (timing)
            for (int q = 0; q < 5; ++q) HIPC(hipEventCreate(&ev[q]));
        auto mark = [&](int q) {
            if (timing) HIPC(hipEventRecord(ev[q], s));
        };
        // events: 0 start | 1 per-box samples | 2 bases | 3 cores | 4 near field
        mark(0);
        // Alg. 3: box i applies A (and A*) to G (H) with the rows of its neighbours
        // zeroed and keeps its own rows of the product; boxes go in chunks so that
        // one operator call sees many test matrices side by side.
        const int cb = boxes_per_chunk(P, P.r);
        const int64_t wmax = static_cast<int64_t>(cb) * P.r;
        double* Om = tmp.plain(P.n * wmax);
        double* Yc = tmp.plain(P.n * wmax);
        for (int side = 0; side < 2; ++side) {
            for (int i0 = 0; i0 < P.b; i0 += cb) {
                const int i1 = std::min(P.b, i0 + cb);
                launch_expand_masked(P, t, side ? H : G, i0, i1, Om, s);
                op_apply(o, side, static_cast<int64_t>(i1 - i0) * P.r, Om, P.n, Yc, P.n, s);
                launch_take_box_rows(P, t, Yc, i0, i1, side ? SZ : SY, s);
            }
        }
        if (keep_samples) {
            for (int side = 0; side < 2; ++side) {
                double*& dst = side ? h->SZ : h->SY;
                dst = dalloc_sync(P.n * P.r);
                HIPC(hipMemcpyAsync(dst, side ? SZ : SY, P.n * P.r * sizeof(double),
                                    hipMemcpyDeviceToDevice, s));
            }
        }
        mark(1);
        launch_orth2(P, t, SY, SZ, h->U, h->V, nullptr, nullptr, s);
        mark(2);
        cores_any(o, P, t, h->U, h->V, h->Atil, s, tmp);
        mark(3);
        nearfield_any(o, P, t, h->U, h->V, h->Atil, h->B, s, tmp);
        mark(4);
        if (timing) {
            double* flag = tmp.get(1);
            const double* arrs[4] = {h->U, h->V, h->Atil, h->B};
            const int64_t cnts[4] = {P.n * P.k, P.n * P.k, bk * bk, P.b_values};
            launch_flag_nonfinite(arrs, cnts, 4, flag, s);
            double hflag = 0.0;
            HIPC(hipMemcpyAsync(&hflag, flag, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            if (hflag != 0.0)
                fail(BLR_ERR_NUMERICAL, "non-finite values in the compressed operator (samples, bases, cores or near field)");
            float ms[4];
            for (int q = 0; q < 4; ++q) HIPC(hipEventElapsedTime(&ms[q], ev[q], ev[q + 1]));
            float tot;
            HIPC(hipEventElapsedTime(&tot, ev[0], ev[4]));
            std::memset(rep, 0, sizeof(*rep));
            rep->ms_sketch = ms[0];
            rep->ms_orth = ms[1];
            rep->ms_cores = ms[2];
            rep->ms_nearfield = ms[3];
            rep->ms_total = tot;
            const int64_t br = static_cast<int64_t>(P.b) * P.r;
            rep->applies_A = br + bk + static_cast<int64_t>(P.ncol) * P.m_max;
            rep->applies_At = br;
            rep->sketch_flops = 4.0 * static_cast<double>(P.n) * static_cast<double>(P.n) * static_cast<double>(br);
            rep->precision = BLR_PREC_FP64;
        }
        auto* hh = new blr_ublr;
        hh->d = std::move(h);
        *out = hh;
    });
}

blr_status blr_bn_min_columns(const blr_plan* plan, int64_t* s) {
    return guard([&] {
        if (!s) fail(BLR_ERR_INVALID_ARG, "NULL output");
        *s = bn_min_columns(plan_of(plan));
    });
}

blr_status blr_bn_compress(const blr_plan* plan, const blr_operator* op, int64_t s, const double* Omega,
                           const double* Psi, int32_t keep_samples, void* stream, blr_ublr** out,
                           blr_report* rep) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out) fail(BLR_ERR_INVALID_ARG, "NULL output");
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!Omega || !Psi) fail(BLR_ERR_INVALID_ARG, "NULL Omega or Psi");
        if (s < bn_min_columns(P))
            fail(BLR_ERR_INVALID_ARG, "s must be at least r plus the rows of the largest neighbourhood");
        hipStream_t st = static_cast<hipStream_t>(stream);
        const DeviceTables& t = plan->d->tables();
        const int64_t bk = static_cast<int64_t>(P.b) * P.k;
        const int64_t ns = P.n * s;

        auto h = std::make_unique<UblrData>();
        h->plan = plan->d;
        h->device = current_device();
        h->precision = BLR_PREC_FP64;
        h->U = dalloc_sync(P.n * P.k);
        h->V = dalloc_sync(P.n * P.k);
        h->Atil = dalloc_sync(bk * bk);
        h->B = dalloc_sync(P.b_values);
        AsyncTemps tmp(st);
        double* SY = tmp.get(P.n * P.r);
        double* SZ = tmp.get(P.n * P.r);
        double* Y = tmp.plain(ns);
        double* Z = tmp.plain(ns);
        double* dP = tmp.plain(static_cast<int64_t>(P.b) * s * P.r);
        double* dQ = tmp.plain(static_cast<int64_t>(P.b) * s * P.r);

        const bool timing = rep != nullptr;
        struct Events {
            hipEvent_t e[6] = {};
            ~Events() {
                for (hipEvent_t x : e)
                    if (x) (void)hipEventDestroy(x);
            }
        } evs;
        hipEvent_t* ev = evs.e;
        if (timing)
            for (int q = 0; q < 6; ++q) HIPC(hipEventCreate(&ev[q]));
        auto mark = [&](int q) {
            if (timing) HIPC(hipEventRecord(ev[q], st));
        };
        // events: 0 start | 1 sketches | 2 null vectors + projection | 3 bases | 4 cores | 5 near field
        mark(0);
        op_apply(o, 0, s, Omega, P.n, Y, P.n, st);
        op_apply(o, 1, s, Psi, P.n, Z, P.n, st);
        mark(1);
        {
            // the null vectors depend on the test matrices only: one Householder QR per box and side
            double* wsp = tmp.get(bn_null_workspace_doubles(P, s));
            double* flag = tmp.get(1);
            launch_fill0(flag, 1, st);
            launch_bn_null(P, t, Omega, s, wsp, dP, flag, st);
            launch_bn_null(P, t, Psi, s, wsp, dQ, flag, st);
            double hflag = 0.0;
            HIPC(hipMemcpyAsync(&hflag, flag, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPC(hipStreamSynchronize(st));
            if (hflag != 0.0)
                fail(BLR_ERR_NUMERICAL, "a neighbour block of the test matrix is rank deficient (block nullification)");
        }
        launch_bn_project(P, t, Y, s, dP, SY, st);
        launch_bn_project(P, t, Z, s, dQ, SZ, st);
        if (keep_samples) {
            for (int side = 0; side < 2; ++side) {
                double*& dst = side ? h->SZ : h->SY;
                dst = dalloc_sync(P.n * P.r);
                HIPC(hipMemcpyAsync(dst, side ? SZ : SY, P.n * P.r * sizeof(double),
                                    hipMemcpyDeviceToDevice, st));
            }
        }
        mark(2);
        launch_orth2(P, t, SY, SZ, h->U, h->V, nullptr, nullptr, st);
        mark(3);
        cores_any(o, P, t, h->U, h->V, h->Atil, st, tmp);
        mark(4);
        nearfield_any(o, P, t, h->U, h->V, h->Atil, h->B, st, tmp);
        mark(5);
        if (timing) {
            double* flag = tmp.get(1);
            const double* arrs[4] = {h->U, h->V, h->Atil, h->B};
            const int64_t cnts[4] = {P.n * P.k, P.n * P.k, bk * bk, P.b_values};
            launch_flag_nonfinite(arrs, cnts, 4, flag, st);
            double hflag = 0.0;
            HIPC(hipMemcpyAsync(&hflag, flag, sizeof(double), hipMemcpyDeviceToHost, st));
            HIPC(hipStreamSynchronize(st));
            if (hflag != 0.0)
                fail(BLR_ERR_NUMERICAL, "non-finite values in the compressed operator (samples, bases, cores or near field)");
            float ms[5];
            for (int q = 0; q < 5; ++q) HIPC(hipEventElapsedTime(&ms[q], ev[q], ev[q + 1]));
            float tot;
            HIPC(hipEventElapsedTime(&tot, ev[0], ev[5]));
            std::memset(rep, 0, sizeof(*rep));
            rep->ms_sketch = ms[0];
            rep->ms_postprocess = ms[1];
            rep->ms_orth = ms[2];
            rep->ms_cores = ms[3];
            rep->ms_nearfield = ms[4];
            rep->ms_total = tot;
            rep->applies_A = s + bk + static_cast<int64_t>(P.ncol) * P.m_max;
            rep->applies_At = s;
            rep->sketch_flops = 4.0 * static_cast<double>(P.n) * static_cast<double>(P.n) * static_cast<double>(s);
            rep->precision = BLR_PREC_FP64;
        }
        auto* hh = new blr_ublr;
        hh->d = std::move(h);
        *out = hh;
    });
}

blr_status blr_tag_rank(const blr_plan* plan, const blr_operator* op, const double* G, const double* H,
                        double tol, void* stream, int32_t* k_out, double* sigma) {
    return guard([&] {
        if (!k_out) fail(BLR_ERR_INVALID_ARG, "NULL output");
        const PlanData& P = plan_of(plan);
        const OpData& o = op_of(op, P);
        if (!G || !H) fail(BLR_ERR_INVALID_ARG, "NULL G or H");
        if (!(tol >= 0.0)) fail(BLR_ERR_INVALID_ARG, "tolerance must be a non-negative number");
        hipStream_t st = static_cast<hipStream_t>(stream);
        const DeviceTables& t = plan->d->tables();
        const int64_t LR = static_cast<int64_t>(P.ell) * P.r;
        const int64_t br = static_cast<int64_t>(P.b) * P.r;
        AsyncTemps tmp(st);
        double* Y = tmp.get(P.n * LR);
        double* Z = tmp.get(P.n * LR);
        double* Yh = tmp.get(P.n * P.r);
        double* Zh = tmp.get(P.n * P.r);
        double* Q0 = tmp.get(P.n * P.k);
        double* Q1 = tmp.get(P.n * P.k);
        double* sig = tmp.get(2 * br);
        sketch_any(o, P, t, G, H, Y, Z, st, tmp);
        launch_postprocess(P, t, Y, Yh, st);
        launch_postprocess(P, t, Z, Zh, st);
        launch_orth2(P, t, Yh, Zh, Q0, Q1, sig, sig + br, st);
        std::vector<double> hs(static_cast<size_t>(2 * br));
        HIPC(hipMemcpyAsync(hs.data(), sig, hs.size() * sizeof(double), hipMemcpyDeviceToHost, st));
        HIPC(hipStreamSynchronize(st));
        for (double v : hs)
            if (!std::isfinite(v)) fail(BLR_ERR_NUMERICAL, "non-finite singular values of the tagged samples");
        // k = max over boxes and sides of #{j : sigma_j(box) > tol * largest sigma of that side}
        int k = 0;
        for (int side = 0; side < 2; ++side) {
            const double* sg = hs.data() + side * br;
            double top = 0.0;
            for (int i = 0; i < P.b; ++i) top = std::max(top, sg[static_cast<int64_t>(i) * P.r]);
            if (top <= 0.0) continue;
            for (int i = 0; i < P.b; ++i) {
                int c = 0;
                for (int j = 0; j < P.r; ++j) c += sg[static_cast<int64_t>(i) * P.r + j] > tol * top ? 1 : 0;
                k = std::max(k, c);
            }
        }
        *k_out = k;
        if (sigma) std::memcpy(sigma, hs.data(), hs.size() * sizeof(double));
    });
}

void blr_ublr_destroy(blr_ublr* h) { delete h; }

// Choose per-box ranks: drop the globally smallest singular values (b x k table, each box's
// row descending) while the sum of their squares stays within `budget`.
static std::vector<int32_t> drop_to_budget(const std::vector<double>& sig, int b, int k, double budget,
                                           double* dropped) {
    std::vector<std::tuple<double, int, int>> all;
    all.reserve(static_cast<size_t>(b) * k);
    for (int i = 0; i < b; ++i)
        for (int j = 0; j < k; ++j) {
            const double v = sig[static_cast<size_t>(i) * k + j];
            all.emplace_back(v * v, i, j);
        }
    std::sort(all.begin(), all.end());
    std::vector<int32_t> ranks(b, k);
    double acc = 0.0;
    for (const auto& e : all) {
        if (acc + std::get<0>(e) > budget) break;
        acc += std::get<0>(e);
        --ranks[std::get<1>(e)];
    }
    *dropped = acc;
    return ranks;
}

blr_status blr_ublr_truncate(const blr_ublr* h, double tol, void* stream, blr_ublr** out, int32_t* ranks_u,
                             int32_t* ranks_v, double* rel_change) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!h || !h->d || !out) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        if (!(tol >= 0.0) || !std::isfinite(tol)) fail(BLR_ERR_INVALID_ARG, "tolerance must be a finite number >= 0");
        const UblrData& d = *h->d;
        const PlanData& P = *d.plan;
        if (d.device != current_device()) fail(BLR_ERR_INVALID_ARG, "handle belongs to another device");
        if (P.k > 64) fail(BLR_ERR_UNSUPPORTED, "truncation supports k <= 64");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const DeviceTables& t = d.plan->tables();
        const int b = P.b, k = P.k;
        const int64_t bk = static_cast<int64_t>(b) * k;
        auto o = std::make_unique<UblrData>();
        o->plan = d.plan;
        o->device = d.device;
        o->precision = d.precision;
        o->r_lo = d.r_lo;
        o->U = dalloc_sync(P.n * k);
        o->V = dalloc_sync(P.n * k);
        o->Atil = dalloc_sync(bk * bk);
        o->B = dalloc_sync(P.b_values);
        AsyncTemps tmp(s);
        double* W = tmp.get(static_cast<int64_t>(b) * k * k);
        double* Jm = tmp.get(static_cast<int64_t>(b) * k * k);
        double* sig = tmp.get(static_cast<int64_t>(b) * k);
        double* part = tmp.get(static_cast<int64_t>(b) * b + P.near_nnz);
        int32_t* kdev = reinterpret_cast<int32_t*>(tmp.get(b));    // b ranks (int32) in b doubles
        // ||A_uBLR||_F^2: far blocks ||Atil_ij||^2 (orthonormal bases), near blocks explicitly
        launch_block_sq(P, d.Atil, part, s);
        launch_near_repr_sq(P, t, d.U, d.V, d.Atil, d.B, part + static_cast<int64_t>(b) * b, s);
        std::vector<double> hp(static_cast<size_t>(b) * b + P.near_nnz);
        HIPC(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        std::vector<uint8_t> nm(P.nearm);
        HIPC(hipStreamSynchronize(s));
        double norm2 = 0.0;
        for (int i = 0; i < b; ++i)
            for (int j = 0; j < b; ++j)
                if (!nm[static_cast<size_t>(i) * b + j]) norm2 += hp[static_cast<size_t>(i) * b + j];
        for (int64_t q = 0; q < P.near_nnz; ++q) norm2 += hp[static_cast<size_t>(b) * b + q];
        if (!std::isfinite(norm2)) fail(BLR_ERR_NUMERICAL, "non-finite compressed operator");
        const double budget = tol * tol * norm2;
        std::vector<double> hs(static_cast<size_t>(b) * k);
        auto fetch_sig = [&] {
            HIPC(hipMemcpyAsync(hs.data(), sig, hs.size() * sizeof(double), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            for (double v : hs)
                if (!std::isfinite(v)) fail(BLR_ERR_NUMERICAL, "non-finite singular values in the truncation");
        };
        // rows: half of the budget
        launch_trunc_svd(P, t, 0, d.Atil, W, sig, s);
        fetch_sig();
        double drop_u = 0.0, drop_v = 0.0;
        std::vector<int32_t> ku = drop_to_budget(hs, b, k, 0.5 * budget, &drop_u);
        HIPC(hipMemcpyAsync(kdev, ku.data(), b * sizeof(int32_t), hipMemcpyHostToDevice, s));
        launch_trunc_rows(P, d.Atil, o->Atil, W, kdev, s);
        launch_trunc_basis(P, t, d.U, o->U, W, kdev, s);
        // columns of the row-truncated cores: what the rows left of the budget
        launch_trunc_svd(P, t, 1, o->Atil, Jm, sig, s);
        fetch_sig();
        std::vector<int32_t> kv = drop_to_budget(hs, b, k, budget - drop_u, &drop_v);
        HIPC(hipMemcpyAsync(kdev, kv.data(), b * sizeof(int32_t), hipMemcpyHostToDevice, s));
        launch_trunc_cols(P, o->Atil, Jm, kdev, s);
        launch_trunc_basis(P, t, d.V, o->V, Jm, kdev, s);
        // near pairs keep their represented blocks
        launch_trunc_near(P, t, d.U, d.V, d.Atil, o->Atil, W, Jm, d.B, o->B, s);
        HIPC(hipStreamSynchronize(s));
        o->ranks_u = ku;
        o->ranks_v = kv;
        if (ranks_u) std::memcpy(ranks_u, ku.data(), b * sizeof(int32_t));
        if (ranks_v) std::memcpy(ranks_v, kv.data(), b * sizeof(int32_t));
        if (rel_change) *rel_change = norm2 > 0.0 ? std::sqrt((drop_u + drop_v) / norm2) : 0.0;
        auto H = std::make_unique<blr_ublr>();
        H->d = std::move(o);
        *out = H.release();
    });
}

blr_status blr_ublr_ranks(const blr_ublr* h, int32_t* ranks_u, int32_t* ranks_v) {
    return guard([&] {
        if (!h || !h->d || !ranks_u || !ranks_v) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        const UblrData& d = *h->d;
        const int b = d.plan->b;
        for (int i = 0; i < b; ++i) {
            ranks_u[i] = d.ranks_u.empty() ? d.plan->k : d.ranks_u[i];
            ranks_v[i] = d.ranks_v.empty() ? d.plan->k : d.ranks_v[i];
        }
    });
}

blr_status blr_ublr_part_ptr(const blr_ublr* h, int32_t part, const void** ptr, int64_t* count) {
    if (ptr) *ptr = nullptr;
    return guard([&] {
        if (!h || !h->d || !ptr || !count) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        const UblrData& d = *h->d;
        const PlanData& P = *d.plan;
        const bool mixed = is_mixed(d.precision);
        const int rs = mixed ? d.r_lo : P.r;  // sample columns of the sketch
        const int64_t LR = static_cast<int64_t>(P.ell) * rs;
        const int64_t bk = static_cast<int64_t>(P.b) * P.k;
        switch (part) {
            case BLR_PART_U: *ptr = d.U; *count = P.n * P.k; break;
            case BLR_PART_V: *ptr = d.V; *count = P.n * P.k; break;
            case BLR_PART_ATIL: *ptr = d.Atil; *count = bk * bk; break;
            case BLR_PART_B: *ptr = d.B; *count = P.b_values; break;
            case BLR_PART_Y: *ptr = d.Y; *count = P.n * LR; break;
            case BLR_PART_Z: *ptr = d.Z; *count = P.n * LR; break;
            case BLR_PART_YHAT: *ptr = d.Yhat; *count = P.n * rs; break;
            case BLR_PART_ZHAT: *ptr = d.Zhat; *count = P.n * rs; break;
            case BLR_PART_Y0: *ptr = d.Y0; *count = P.n * LR; break;
            case BLR_PART_Z0: *ptr = d.Z0; *count = P.n * LR; break;
            case BLR_PART_U0: *ptr = d.U0; *count = P.n * rs; break;
            case BLR_PART_V0: *ptr = d.V0; *count = P.n * rs; break;
            case BLR_PART_SY: *ptr = d.SY; *count = P.n * P.r; break;
            case BLR_PART_SZ: *ptr = d.SZ; *count = P.n * P.r; break;
            default: fail(BLR_ERR_INVALID_ARG, "unknown part");
        }
        if (!*ptr) fail(BLR_ERR_INVALID_ARG, "part not kept (compress with keep_intermediates, in the mode that has it)");
    });
}

blr_status blr_ublr_export(const blr_ublr* h, int32_t part, void* host, int64_t count, void* stream) {
    return guard([&] {
        if (!host) fail(BLR_ERR_INVALID_ARG, "NULL host buffer");
        const void* ptr = nullptr;
        int64_t cnt = 0;
        const blr_status st = blr_ublr_part_ptr(h, part, &ptr, &cnt);
        if (st != BLR_OK) fail(st, g_last_error);
        if (count != cnt) fail(BLR_ERR_INVALID_ARG, "count differs from the part's element count");
        const size_t esize = (part == BLR_PART_Y0 || part == BLR_PART_Z0) ? sizeof(float) : sizeof(double);
        hipStream_t s = static_cast<hipStream_t>(stream);
        HIPC(hipMemcpyAsync(host, ptr, static_cast<size_t>(cnt) * esize, hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
    });
}

blr_status blr_apply(const blr_ublr* h, int32_t trans, int64_t ncols, const double* x, int64_t ldx,
                     double* y, int64_t ldy, void* stream) {
    return guard([&] {
        if (!h || !h->d) fail(BLR_ERR_INVALID_ARG, "NULL handle");
        const UblrData& d = *h->d;
        const PlanData& P = *d.plan;
        if (ncols < 0) fail(BLR_ERR_INVALID_ARG, "negative ncols");
        if (ncols == 0) return;
        if (ncols > 65535) fail(BLR_ERR_INVALID_ARG, "at most 65535 columns per call");
        if (!x || !y) fail(BLR_ERR_INVALID_ARG, "NULL x or y");
        check_ld(ldx, P.n, "x");
        check_ld(ldy, P.n, "y");
        if (d.device != current_device()) fail(BLR_ERR_INVALID_ARG, "handle belongs to another device");
        hipStream_t s = static_cast<hipStream_t>(stream);
        const DeviceTables& t = d.plan->tables();
        AsyncTemps tmp(s);
        double* work = tmp.get(apply_workspace_doubles(P, ncols));
        launch_ublr_apply(P, t, d.U, d.V, d.Atil, d.B, trans ? 1 : 0, ncols, x, ldx, y, ldy, work, s);
    });
}

blr_status blr_apply_noalloc(const blr_ublr* h, int32_t trans, int64_t ncols, const double* x, int64_t ldx,
                             double* y, int64_t ldy, void* stream) {
    return guard([&] {
        if (!h || !h->d) fail(BLR_ERR_INVALID_ARG, "NULL handle");
        const UblrData& d = *h->d;
        const PlanData& P = *d.plan;
        if (ncols < 0) fail(BLR_ERR_INVALID_ARG, "negative ncols");
        if (ncols == 0) return;
        if (ncols > 65535) fail(BLR_ERR_INVALID_ARG, "at most 65535 columns per call");
        if (!x || !y) fail(BLR_ERR_INVALID_ARG, "NULL x or y");
        check_ld(ldx, P.n, "x");
        check_ld(ldy, P.n, "y");
        if (d.device != current_device()) fail(BLR_ERR_INVALID_ARG, "handle belongs to another device");
        const int64_t need = apply_workspace_doubles(P, ncols);
        if (need > kNoAllocScratchDoubles) {
            std::ostringstream os;
            os << "blr_apply_noalloc: the workspace of " << need << " doubles exceeds the fixed scratch of "
               << kNoAllocScratchDoubles << " doubles (32 MiB); pass fewer columns per call or use blr_apply";
            fail(BLR_ERR_INVALID_ARG, os.str());
        }
        // The handle was built on this device, so the plan's tables are resident here.
        const DeviceTables* t = d.plan->resident_tables();
        if (!t) fail(BLR_ERR_INVALID_ARG, "the plan's device tables are not resident on this device");
        double* work = noalloc_scratch(d.device);
        launch_ublr_apply(P, *t, d.U, d.V, d.Atil, d.B, trans ? 1 : 0, ncols, x, ldx, y, ldy, work,
                          static_cast<hipStream_t>(stream));
    });
}

blr_status blr_error_fro(const blr_ublr* h, const blr_operator* op, void* stream, double* rel_err) {
    return guard([&] {
        if (!h || !h->d || !rel_err) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        const UblrData& d = *h->d;
        const PlanData& P = *d.plan;
        const OpData& o = op_of(op, P);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const DeviceTables& t = d.plan->tables();
        AsyncTemps tmp(s);
        if (is_callback(o)) {
            // A black box gives its entries only through products: A e_j for every column j,
            // in chunks of w unit columns, against the representation applied to the same
            // columns; both squared norms summed per chunk in a fixed order.
            const int64_t n = P.n;
            const int64_t w = std::max<int64_t>(16, std::min<int64_t>(512, ((int64_t(1) << 25) / n) / 16 * 16));
            double* X = tmp.plain(n * w);
            double* Y = tmp.plain(n * w);
            double* R = tmp.get(n * w);
            double* work = tmp.get(apply_workspace_doubles(P, w));
            double* part = tmp.get(dot_parts());
            auto sumsq = [&](const double* v, int64_t len) {
                launch_dot(v, v, len, part, s);
                double r = 0.0;
                HIPC(hipMemcpyAsync(&r, part, sizeof(double), hipMemcpyDeviceToHost, s));
                HIPC(hipStreamSynchronize(s));
                return r;
            };
            double se = 0.0, sa = 0.0;
            for (int64_t c0 = 0; c0 < n; c0 += w) {
                const int64_t wc = std::min(w, n - c0);
                launch_unit_cols(X, n, c0, wc, s);
                op_apply(o, 0, wc, X, n, Y, n, s);
                launch_ublr_apply(P, t, d.U, d.V, d.Atil, d.B, 0, wc, X, n, R, n, work, s);
                sa += sumsq(Y, n * wc);
                launch_axpy(-1.0, Y, R, n * wc, s);
                se += sumsq(R, n * wc);
            }
            if (!std::isfinite(se) || !std::isfinite(sa)) fail(BLR_ERR_NUMERICAL, "non-finite error sums");
            *rel_err = sa > 0.0 ? std::sqrt(se / sa) : std::sqrt(se);
            return;
        }
        const int64_t np = static_cast<int64_t>(P.b) * P.b;
        double* part = tmp.get(2 * np);
        require_entries(o, "the exact Frobenius error");
        launch_err_fro(o, P, t, d.U, d.V, d.Atil, d.B, part, s);
        std::vector<double> hp(2 * np);
        HIPC(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPC(hipStreamSynchronize(s));
        double se = 0.0, sa = 0.0;
        for (int64_t q = 0; q < np; ++q) {
            se += hp[2 * q];
            sa += hp[2 * q + 1];
        }
        *rel_err = sa > 0.0 ? std::sqrt(se / sa) : std::sqrt(se);
    });
}

blr_status blr_error_power(const blr_ublr* h, const blr_operator* op, const double* x0,
                           int32_t iters, void* stream, double* err_norm, double* a_norm) {
    return guard([&] {
        if (!h || !h->d || !x0) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        if (iters < 1) fail(BLR_ERR_INVALID_ARG, "iters must be >= 1");
        const UblrData& d = *h->d;
        const PlanData& P = *d.plan;
        const OpData& o = op_of(op, P);
        hipStream_t s = static_cast<hipStream_t>(stream);
        const DeviceTables& t = d.plan->tables();
        const int64_t n = P.n;
        AsyncTemps tmp(s);
        // x, y, w are operands of the operator's products (plain allocations for a callback)
        const bool cb = is_callback(o);
        double* x = cb ? tmp.plain(n) : tmp.get(n);
        double* y = cb ? tmp.plain(n) : tmp.get(n);
        double* w = cb ? tmp.plain(n) : tmp.get(n);
        double* u = tmp.get(n);
        double* part = tmp.get(dot_parts());
        double* work = tmp.get(apply_workspace_doubles(P, 1));
        auto norm2 = [&](const double* v) {
            launch_dot(v, v, n, part, s);
            double r = 0.0;
            HIPC(hipMemcpyAsync(&r, part, sizeof(double), hipMemcpyDeviceToHost, s));
            HIPC(hipStreamSynchronize(s));
            return std::sqrt(r);
        };
        // M v = A v - (use_ublr ? A_uBLR v : 0); M* likewise
        auto apply_M = [&](int trans, bool diff, const double* in, double* out) {
            op_apply(o, trans, 1, in, n, out, n, s);
            if (diff) {
                launch_ublr_apply(P, t, d.U, d.V, d.Atil, d.B, trans, 1, in, n, u, n, work, s);
                launch_axpy(-1.0, u, out, n, s);
            }
        };
        auto power = [&](bool diff) {
            HIPC(hipMemcpyAsync(x, x0, n * sizeof(double), hipMemcpyDeviceToDevice, s));
            const double n0 = norm2(x);
            if (n0 == 0.0) fail(BLR_ERR_INVALID_ARG, "x0 is zero");
            launch_scale(1.0 / n0, x, n, s);
            for (int it = 0; it < iters; ++it) {
                apply_M(0, diff, x, y);
                apply_M(1, diff, y, w);
                const double nw = norm2(w);
                if (nw == 0.0 || !std::isfinite(nw)) {
                    if (!std::isfinite(nw)) fail(BLR_ERR_NUMERICAL, "non-finite power iterate");
                    return 0.0;
                }
                launch_scale(1.0 / nw, w, n, s);
                std::swap(x, w);
            }
            apply_M(0, diff, x, y);
            return norm2(y);
        };
        const double e = power(true);
        if (err_norm) *err_norm = e;
        if (a_norm) *a_norm = power(false);
    });
}


// ------------------------------------------------------------------ batches
namespace {

// Bytes of one compression (outputs and temporaries), by the allocation plan of
// blr_tag_compress and of the batch.
int64_t footprint_bytes(const PlanData& P, int precision, int r_lo) {
    const int64_t bk = static_cast<int64_t>(P.b) * P.k;
    int64_t d = 2 * P.n * P.k + bk * bk + P.b_values + nearfield_workspace_doubles(P);
    int64_t bytes = 0;
    if (is_mixed(precision)) {
        const int64_t LR = static_cast<int64_t>(P.ell) * r_lo;
        const int64_t esize = precision == BLR_PREC_BF16_REFINE ? 2 : 4;
        bytes += 2 * P.n * LR * 4 + 2 * lp_packed_elems(P, r_lo) * esize;
        d += 4 * P.n * r_lo + 4 * P.n * P.r;
    } else {
        d += 2 * P.n * static_cast<int64_t>(P.ell) * P.r + 2 * P.n * P.r;
    }
    return bytes + d * static_cast<int64_t>(sizeof(double));
}

std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, int> g_tuned_spw;  // (device, precision, ntr) -> SPW

}  // namespace

blr_status blr_plan_footprint(const blr_plan* plan, int32_t precision, int32_t r_lo, int64_t* bytes) {
    return guard([&] {
        const PlanData& P = plan_of(plan);
        if (!bytes) fail(BLR_ERR_INVALID_ARG, "NULL output");
        if (!is_mixed(precision) && precision != BLR_PREC_FP64) fail(BLR_ERR_UNSUPPORTED, "unsupported precision");
        const int rl = is_mixed(precision) ? (r_lo ? r_lo : P.r) : P.r;
        if (is_mixed(precision)) check_r_lo(P, rl);
        *bytes = footprint_bytes(P, precision, rl);
    });
}

}  // extern "C"

namespace blr {
namespace {

struct BatchJob {
    std::shared_ptr<PlanData> plan;
    const OpData* op = nullptr;
    const double* G = nullptr;
    const double* H = nullptr;
    int precision = BLR_PREC_FP64;
    int r_lo = 0;
    const double* gamma_u = nullptr;
    const double* gamma_v = nullptr;
    blr_ublr* handle = nullptr;
    const DeviceTables* t = nullptr;
    bool persistent = false;  // sketch in a persistent class launch
    double *Y = nullptr, *Z = nullptr;
    float *Y0 = nullptr, *Z0 = nullptr;
    void *PG = nullptr, *PH = nullptr;
    double *Yh = nullptr, *Zh = nullptr, *U0 = nullptr, *V0 = nullptr;
    double *Xv = nullptr, *Xu = nullptr, *SY = nullptr, *SZ = nullptr, *nfw = nullptr;
};

struct SketchClass {
    int precision = 0, ntr = 0;
    int kind = -1;                 // FP64 classes: the kernel kind of every member
    int tg = 0;                    // FP64 classes: fp64_sketch_tail_groups(kind, r) of every member
    std::vector<int> members;
    LpJob* d_jobs = nullptr;
    Fp64Job* d_jobs64 = nullptr;
    int nspw = 0;
    int spw[2] = {0, 0};
    int4* d_items[2] = {nullptr, nullptr};
    int nitems[2] = {0, 0};
    int chosen = 0;
};

}  // namespace
}  // namespace blr

struct blr_batch {
    std::vector<blr::BatchJob> jobs;
    std::vector<blr::SketchClass> classes;
    std::vector<void*> mem;
    int device = -1;
    int flags = 0;
    int runs = 0;
    int grid = 512;
    hipStream_t own = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr, e0 = nullptr, e1 = nullptr, e2 = nullptr;
    // per-job stages after the sketch run on a few lanes (streams) forked from and joined to own
    std::vector<hipStream_t> lanes;
    std::vector<hipEvent_t> lane_done;
    hipEvent_t ev_fork = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~blr_batch() {
        int cur = -1;
        (void)hipGetDevice(&cur);
        if (device >= 0) (void)hipSetDevice(device);
        if (own) (void)hipStreamSynchronize(own);
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        for (auto& j : jobs) delete j.handle;
        for (void* p : mem) (void)hipFree(p);
        for (hipEvent_t e : {ev_in, ev_out, e0, e1, e2, ev_fork})
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : lane_done) (void)hipEventDestroy(e);
        for (hipStream_t l : lanes) {
            (void)hipStreamSynchronize(l);
            (void)hipStreamDestroy(l);
        }
        if (own) (void)hipStreamDestroy(own);
        if (cur >= 0) (void)hipSetDevice(cur);
    }
    template <class T>
    T* alloc(int64_t count) {
        void* p = nullptr;
        const size_t bytes = static_cast<size_t>(std::max<int64_t>(1, count)) * sizeof(T);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            blr::fail(BLR_ERR_OOM, "device allocation for the batch failed");
        }
        mem.push_back(p);
        return static_cast<T*>(p);
    }
};

namespace blr {
namespace {

void batch_enqueue(blr_batch& B, bool time_sketch) {
    hipStream_t s = B.own;
    for (auto& j : B.jobs) {
        const PlanData& P = *j.plan;
        if (is_mixed(j.precision)) {
            launch_pack_lp(P, *j.t, j.precision, j.r_lo, j.G, j.PG, s);
            launch_pack_lp(P, *j.t, j.precision, j.r_lo, j.H, j.PH, s);
            if (!j.persistent) launch_sketch_lp(*j.op, P, *j.t, j.precision, j.r_lo, j.PG, j.PH, j.Y0, j.Z0, s);
        } else {
            if (!j.persistent) launch_sketch(*j.op, P, *j.t, j.G, j.H, j.Y, j.Z, s);
        }
    }
    if (time_sketch) HIPC(hipEventRecord(B.e0, s));
    // the persistent launches one after another: each fills the device (run side by side on
    // the lanes they measured 17% slower)
    for (auto& c : B.classes) {
        if (c.precision == BLR_PREC_FP64)
            launch_sketch_multi(c.kind, c.ntr, c.spw[0], c.tg, c.d_jobs64, c.d_items[0], c.nitems[0], B.grid, s);
        else
            launch_sketch_lp_multi(c.precision, c.ntr, c.spw[c.chosen], c.d_jobs, c.d_items[c.chosen],
                                   c.nitems[c.chosen], B.grid, s);
    }
    if (time_sketch) HIPC(hipEventRecord(B.e1, s));
    // the jobs' remaining stages are independent of each other (every job owns its buffers):
    // job q runs on lane q mod lanes, so small jobs' launches overlap on the device
    HIPC(hipEventRecord(B.ev_fork, s));
    for (hipStream_t l : B.lanes) HIPC(hipStreamWaitEvent(l, B.ev_fork, 0));
    for (size_t q = 0; q < B.jobs.size(); ++q) {
        auto& j = B.jobs[q];
        const hipStream_t ls = B.lanes[q % B.lanes.size()];
        const PlanData& P = *j.plan;
        const DeviceTables& t = *j.t;
        UblrData& h = *j.handle->d;
        if (is_mixed(j.precision)) {
            launch_postprocess_lp(P, t, j.r_lo, j.Y0, j.Yh, ls);
            launch_postprocess_lp(P, t, j.r_lo, j.Z0, j.Zh, ls);
            launch_orth_cols(P, t, j.r_lo, j.r_lo, 1, j.Yh, j.Zh, j.U0, j.V0, nullptr, nullptr, ls);
            launch_mix(P, t, j.r_lo, j.V0, j.gamma_v, j.Xv, ls);
            launch_mix(P, t, j.r_lo, j.U0, j.gamma_u, j.Xu, ls);
            launch_refine(*j.op, P, t, j.Xv, j.Xu, j.SY, j.SZ, ls);
            launch_orth2(P, t, j.SY, j.SZ, h.U, h.V, nullptr, nullptr, ls);
        } else {
            launch_postprocess(P, t, j.Y, j.Yh, ls);
            launch_postprocess(P, t, j.Z, j.Zh, ls);
            launch_orth2(P, t, j.Yh, j.Zh, h.U, h.V, nullptr, nullptr, ls);
        }
        launch_cores(*j.op, P, t, h.U, h.V, h.Atil, ls);
        launch_nearfield(*j.op, P, t, h.U, h.V, h.Atil, h.B, j.nfw, ls);
    }
    for (size_t i = 0; i < B.lanes.size(); ++i) {
        HIPC(hipEventRecord(B.lane_done[i], B.lanes[i]));
        HIPC(hipStreamWaitEvent(s, B.lane_done[i], 0));
    }
}

// Times every SPW candidate of each class on the real items and keeps the fastest
// (the persistent sketch's results do not depend on SPW: each tag column's sums
// run in the same order).
void batch_autotune(blr_batch& B) {
    hipStream_t s = B.own;
    for (auto& c : B.classes) {
        if (c.precision == BLR_PREC_FP64) continue;  // one tile shape per FP64 class
        const auto key = std::make_tuple(B.device, c.precision, c.ntr);
        {
            std::lock_guard<std::mutex> lock(g_tune_mu);
            auto it = g_tuned_spw.find(key);
            if (it != g_tuned_spw.end()) {
                for (int q = 0; q < c.nspw; ++q)
                    if (c.spw[q] == it->second) c.chosen = q;
                continue;
            }
        }
        float best = 0.0f;
        int bq = 0;
        for (int q = 0; q < c.nspw; ++q) {
            HIPC(hipEventRecord(B.e0, s));
            launch_sketch_lp_multi(c.precision, c.ntr, c.spw[q], c.d_jobs, c.d_items[q], c.nitems[q], B.grid, s);
            HIPC(hipEventRecord(B.e1, s));
            HIPC(hipEventSynchronize(B.e1));
            float ms = 0.0f;
            HIPC(hipEventElapsedTime(&ms, B.e0, B.e1));
            if (q == 0 || ms < best) {
                best = ms;
                bq = q;
            }
        }
        c.chosen = bq;
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tuned_spw[key] = c.spw[bq];
    }
}

}  // namespace
}  // namespace blr

extern "C" {

blr_status blr_batch_create(int32_t njobs, const blr_batch_job* jobs, int32_t flags, blr_batch** out) {
    if (out) *out = nullptr;
    return guard([&] {
        if (!out || !jobs) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        if (njobs < 1) fail(BLR_ERR_INVALID_ARG, "njobs must be positive");
        auto B = std::make_unique<blr_batch>();
        B->device = current_device();
        B->flags = flags;
        int cus = 256;
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, B->device);
        B->grid = 2 * std::max(1, cus);
        B->jobs.resize(njobs);
        for (int q = 0; q < njobs; ++q) {
            const blr_batch_job& in = jobs[q];
            BatchJob& j = B->jobs[q];
            const PlanData& P = plan_of(in.plan);
            const OpData& o = op_of(in.op, P);
            if (is_callback(o)) fail(BLR_ERR_UNSUPPORTED, "batches need built-in operators");
            if (!in.G || !in.H) fail(BLR_ERR_INVALID_ARG, "NULL G or H");
            if (in.opts.reserved != 0) fail(BLR_ERR_INVALID_ARG, "reserved option field must be 0");
            j.plan = in.plan->d;
            j.op = &o;
            j.G = in.G;
            j.H = in.H;
            j.precision = in.opts.precision;
            if (!is_mixed(j.precision) && j.precision != BLR_PREC_FP64) fail(BLR_ERR_UNSUPPORTED, "unsupported precision");
            j.r_lo = is_mixed(j.precision) ? (in.opts.r_lo ? in.opts.r_lo : P.r) : P.r;
            if (is_mixed(j.precision)) {
                check_r_lo(P, j.r_lo);
                if (!in.opts.gamma_u || !in.opts.gamma_v) fail(BLR_ERR_INVALID_ARG, "mixed modes need gamma_u and gamma_v");
            }
            j.gamma_u = in.opts.gamma_u;
            j.gamma_v = in.opts.gamma_v;
            j.t = &j.plan->tables();
            // outputs
            auto h = std::make_unique<UblrData>();
            h->plan = j.plan;
            h->device = B->device;
            h->precision = j.precision;
            h->r_lo = j.r_lo;
            const int64_t bk = static_cast<int64_t>(P.b) * P.k;
            h->U = dalloc_sync(P.n * P.k);
            h->V = dalloc_sync(P.n * P.k);
            h->Atil = dalloc_sync(bk * bk);
            h->B = dalloc_sync(P.b_values);
            j.handle = new blr_ublr;
            j.handle->d = std::move(h);
            // temporaries
            const int64_t LR = static_cast<int64_t>(P.ell) * j.r_lo;
            if (is_mixed(j.precision)) {
                const int64_t esize = j.precision == BLR_PREC_BF16_REFINE ? 2 : 4;
                j.Y0 = B->alloc<float>(P.n * LR);
                j.Z0 = B->alloc<float>(P.n * LR);
                j.PG = B->alloc<char>(lp_packed_elems(P, j.r_lo) * esize);
                j.PH = B->alloc<char>(lp_packed_elems(P, j.r_lo) * esize);
                j.U0 = B->alloc<double>(P.n * j.r_lo);
                j.V0 = B->alloc<double>(P.n * j.r_lo);
                j.Xv = B->alloc<double>(P.n * P.r);
                j.Xu = B->alloc<double>(P.n * P.r);
                j.SY = B->alloc<double>(P.n * P.r);
                j.SZ = B->alloc<double>(P.n * P.r);
                j.persistent = o.type == OpType::Kernel;
                if (j.persistent && P.n >= (int64_t(1) << 31)) fail(BLR_ERR_UNSUPPORTED, "N >= 2^31 in a batch");
            } else {
                j.Y = B->alloc<double>(P.n * LR);
                j.Z = B->alloc<double>(P.n * LR);
                j.persistent = o.type == OpType::Kernel;
            }
            j.Yh = B->alloc<double>(P.n * j.r_lo);
            j.Zh = B->alloc<double>(P.n * j.r_lo);
            j.nfw = B->alloc<double>(nearfield_workspace_doubles(P));
        }
        // persistent sketch classes: (precision, column tiles), FP64 also by kernel kind and
        // the form of the last column tile
        for (int q = 0; q < njobs; ++q) {
            BatchJob& j = B->jobs[q];
            if (!j.persistent) continue;
            const int ntr = (j.r_lo + 15) / 16;
            const bool f64 = j.precision == BLR_PREC_FP64;
            const int kind = f64 ? j.op->kind : -1;
            const int tg = f64 ? fp64_sketch_tail_groups(kind, j.r_lo) : 0;
            SketchClass* c = nullptr;
            for (auto& x : B->classes)
                if (x.precision == j.precision && x.ntr == ntr && x.kind == kind && x.tg == tg) c = &x;
            if (!c) {
                if (B->classes.size() >= BLR_BATCH_MAX_CLASSES) fail(BLR_ERR_UNSUPPORTED, "too many sketch classes");
                B->classes.emplace_back();
                c = &B->classes.back();
                c->precision = j.precision;
                c->ntr = ntr;
                c->kind = kind;
                c->tg = tg;
            }
            c->members.push_back(q);
        }
        for (auto& c : B->classes) {
            if (c.precision != BLR_PREC_FP64) continue;
            // tag columns per wave: the fewest of {max, max - 1} that hold every member's
            // groups (ceil(ell / (4 max)) groups, split evenly)
            const int svw_max = fp64_sketch_svw(c.ntr);
            auto groups_of = [&](const PlanData& P) { return (P.ell + 4 * svw_max - 1) / (4 * svw_max); };
            int need = 1;
            for (int q : c.members) {
                const PlanData& P = *B->jobs[q].plan;
                const int ng = groups_of(P);
                need = std::max(need, ((P.ell + ng - 1) / ng + 3) / 4);
            }
            c.nspw = 1;
            c.spw[0] = (svw_max > 1 && need <= svw_max - 1) ? svw_max - 1 : svw_max;
            std::vector<Fp64Job> fj;
            for (int q : c.members) {
                const BatchJob& j = B->jobs[q];
                const PlanData& P = *j.plan;
                Fp64Job d{};
                d.kind = j.op->kind;
                d.diag = j.op->kind == BLR_KERNEL_EXP ? 1.0 : (j.op->kind == BLR_KERNEL_COS ? 1000.0 : 0.0);
                d.px = j.op->pts;
                d.py = j.op->pts + P.n;
                d.pz = j.op->pts + 2 * P.n;
                d.T = j.t->T;
                d.box_ptr = j.t->box_ptr;
                d.nbox = P.b;
                d.r = P.r;
                d.ell = P.ell;
                d.n = P.n;
                d.G0 = j.G;
                d.G1 = j.H;
                d.Y0 = j.Y;
                d.Y1 = j.Z;
                d.ngroups = groups_of(P);
                fj.push_back(d);
            }
            c.d_jobs64 = B->alloc<Fp64Job>(static_cast<int64_t>(fj.size()));
            HIPC(hipMemcpy(c.d_jobs64, fj.data(), fj.size() * sizeof(Fp64Job), hipMemcpyHostToDevice));
            // items: (job index in class, 8-row block, tag column group), heaviest job first
            std::vector<std::pair<double, int4>> items;
            for (size_t u = 0; u < c.members.size(); ++u) {
                const PlanData& P = *B->jobs[c.members[u]].plan;
                const int groups = groups_of(P);
                const int64_t blocks = (P.n + 7) / 8;
                if (blocks > INT32_MAX) fail(BLR_ERR_UNSUPPORTED, "job too large for the batch");
                const double cost = static_cast<double>(P.n) * P.ell;
                for (int64_t rb = 0; rb < blocks; ++rb)
                    for (int g = 0; g < groups; ++g)
                        items.push_back({cost, int4{static_cast<int>(u), static_cast<int>(rb), g, 0}});
            }
            std::stable_sort(items.begin(), items.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
            std::vector<int4> flat(items.size());
            for (size_t u = 0; u < items.size(); ++u) flat[u] = items[u].second;
            if (flat.size() > static_cast<size_t>(INT32_MAX)) fail(BLR_ERR_UNSUPPORTED, "batch too large");
            c.d_items[0] = B->alloc<int4>(static_cast<int64_t>(flat.size()));
            HIPC(hipMemcpy(c.d_items[0], flat.data(), flat.size() * sizeof(int4), hipMemcpyHostToDevice));
            c.nitems[0] = static_cast<int>(flat.size());
        }
        for (auto& c : B->classes) {
            if (c.precision == BLR_PREC_FP64) continue;
            std::vector<LpJob> lj;
            for (int q : c.members) {
                const BatchJob& j = B->jobs[q];
                const PlanData& P = *j.plan;
                LpJob d{};
                d.kind = j.op->kind;
                d.diag = j.op->kind == BLR_KERNEL_EXP ? 1.0f : (j.op->kind == BLR_KERNEL_COS ? 1000.0f : 0.0f);
                d.px = j.op->pts32;
                d.py = j.op->pts32 + P.n;
                d.pz = j.op->pts32 + 2 * P.n;
                d.Tf = j.t->Tf;
                d.box_ptr = j.t->box_ptr;
                d.nbox = P.b;
                d.r = j.r_lo;
                d.ell = P.ell;
                d.n = P.n;
                d.B0 = j.PG;
                d.B1 = j.PH;
                d.Y0 = j.Y0;
                d.Y1 = j.Z0;
                lj.push_back(d);
            }
            c.d_jobs = B->alloc<LpJob>(static_cast<int64_t>(lj.size()));
            HIPC(hipMemcpy(c.d_jobs, lj.data(), lj.size() * sizeof(LpJob), hipMemcpyHostToDevice));
            c.nspw = lp_multi_spw_candidates(c.precision, c.ntr, c.spw);
            for (int v = 0; v < c.nspw; ++v) {
                // items: (job index in class, 32-row block, tag column group), heaviest job first
                std::vector<std::pair<double, int4>> items;
                for (size_t u = 0; u < c.members.size(); ++u) {
                    const PlanData& P = *B->jobs[c.members[u]].plan;
                    const int groups = (P.ell + 2 * c.spw[v] - 1) / (2 * c.spw[v]);
                    const int64_t blocks = (P.n + 31) / 32;
                    if (blocks > INT32_MAX) fail(BLR_ERR_UNSUPPORTED, "job too large for the batch");
                    const double cost = static_cast<double>(P.n) * P.ell;
                    for (int64_t rb = 0; rb < blocks; ++rb)
                        for (int g = 0; g < groups; ++g)
                            items.push_back({cost, int4{static_cast<int>(u), static_cast<int>(rb), g, 0}});
                }
                std::stable_sort(items.begin(), items.end(),
                                 [](const auto& a, const auto& b) { return a.first > b.first; });
                std::vector<int4> flat(items.size());
                for (size_t u = 0; u < items.size(); ++u) flat[u] = items[u].second;
                c.d_items[v] = B->alloc<int4>(static_cast<int64_t>(flat.size()));
                HIPC(hipMemcpy(c.d_items[v], flat.data(), flat.size() * sizeof(int4), hipMemcpyHostToDevice));
                c.nitems[v] = static_cast<int>(flat.size());
            }
        }
        HIPC(hipStreamCreateWithFlags(&B->own, hipStreamNonBlocking));
        for (hipEvent_t* e : {&B->ev_in, &B->ev_out, &B->e0, &B->e1, &B->e2}) HIPC(hipEventCreate(e));
        HIPC(hipEventCreateWithFlags(&B->ev_fork, hipEventDisableTiming));
        const int nlanes = std::min(4, njobs);
        for (int i = 0; i < nlanes; ++i) {
            hipStream_t l = nullptr;
            HIPC(hipStreamCreateWithFlags(&l, hipStreamNonBlocking));
            B->lanes.push_back(l);
            hipEvent_t e = nullptr;
            HIPC(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            B->lane_done.push_back(e);
        }
        *out = B.release();
    });
}

blr_status blr_batch_run(blr_batch* b, void* stream, blr_batch_report* rep) {
    return guard([&] {
        if (!b) fail(BLR_ERR_INVALID_ARG, "NULL batch");
        if (b->device != current_device()) fail(BLR_ERR_INVALID_ARG, "batch belongs to another device");
        hipStream_t us = static_cast<hipStream_t>(stream);
        HIPC(hipEventRecord(b->ev_in, us));
        HIPC(hipStreamWaitEvent(b->own, b->ev_in, 0));
        const bool first = b->runs == 0;
        bool replayed = false;
        if (b->exec) {
            HIPC(hipEventRecord(b->e0, b->own));
            HIPC(hipGraphLaunch(b->exec, b->own));
            HIPC(hipEventRecord(b->e2, b->own));
            replayed = true;
        } else if ((b->flags & BLR_BATCH_GRAPH) && !first) {
            HIPC(hipStreamBeginCapture(b->own, hipStreamCaptureModeThreadLocal));
            try {
                batch_enqueue(*b, false);
            } catch (...) {
                hipGraph_t g = nullptr;
                (void)hipStreamEndCapture(b->own, &g);
                if (g) (void)hipGraphDestroy(g);
                throw;
            }
            HIPC(hipStreamEndCapture(b->own, &b->graph));
            HIPC(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
            HIPC(hipEventRecord(b->e0, b->own));
            HIPC(hipGraphLaunch(b->exec, b->own));
            HIPC(hipEventRecord(b->e2, b->own));
            replayed = true;
        } else {
            hipEvent_t start;
            HIPC(hipEventCreate(&start));
            HIPC(hipEventRecord(start, b->own));
            batch_enqueue(*b, true);
            HIPC(hipEventRecord(b->e2, b->own));
            if (rep) {
                HIPC(hipEventSynchronize(b->e2));
                float tot = 0.0f, sk = 0.0f;
                HIPC(hipEventElapsedTime(&tot, start, b->e2));
                HIPC(hipEventElapsedTime(&sk, b->e0, b->e1));
                std::memset(rep, 0, sizeof(*rep));
                rep->ms_total = tot;
                rep->ms_sketch = sk;
            }
            (void)hipEventDestroy(start);
            // after the first eager run (inputs packed): time the SPW candidates of each
            // persistent class on the real items; later runs use the fastest
            if (first && (b->flags & BLR_BATCH_AUTOTUNE)) batch_autotune(*b);
        }
        HIPC(hipEventRecord(b->ev_out, b->own));
        HIPC(hipStreamWaitEvent(us, b->ev_out, 0));
        ++b->runs;
        if (rep) {
            if (replayed) {
                HIPC(hipEventSynchronize(b->e2));
                float tot = 0.0f;
                HIPC(hipEventElapsedTime(&tot, b->e0, b->e2));
                std::memset(rep, 0, sizeof(*rep));
                rep->ms_total = tot;
                rep->graph_replayed = 1;
            }
            for (const auto& j : b->jobs) {
                const PlanData& P = *j.plan;
                const int64_t LR = static_cast<int64_t>(P.ell) * j.r_lo;
                const bool mixed = is_mixed(j.precision);
                rep->sketch_flops += 4.0 * static_cast<double>(P.n) * static_cast<double>(P.n) * static_cast<double>(LR);
                if (mixed) rep->refine_flops += refine_flops(P);
                const int64_t rc = mixed ? static_cast<int64_t>(P.b) * P.r : 0;
                rep->applies += 2 * (LR + rc) + static_cast<int64_t>(P.b) * P.k + static_cast<int64_t>(P.ncol) * P.m_max;
            }
            rep->nclasses = static_cast<int32_t>(b->classes.size());
            for (size_t q = 0; q < b->classes.size(); ++q) {
                rep->class_precision[q] = b->classes[q].precision;
                rep->class_kind[q] = b->classes[q].kind;
                rep->class_tail[q] = b->classes[q].tg;
                rep->class_ntr[q] = b->classes[q].ntr;
                rep->class_spw[q] = b->classes[q].spw[b->classes[q].chosen];
                rep->class_jobs[q] = static_cast<int32_t>(b->classes[q].members.size());
            }
        }
    });
}

blr_status blr_batch_result(const blr_batch* b, int32_t job, const blr_ublr** h) {
    if (h) *h = nullptr;
    return guard([&] {
        if (!b || !h) fail(BLR_ERR_INVALID_ARG, "NULL argument");
        if (job < 0 || job >= static_cast<int32_t>(b->jobs.size())) fail(BLR_ERR_INVALID_ARG, "job out of range");
        *h = b->jobs[job].handle;
    });
}

void blr_batch_destroy(blr_batch* b) { delete b; }
}  // extern "C"
