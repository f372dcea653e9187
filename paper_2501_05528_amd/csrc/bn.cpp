// Null vectors of Alg. 1 (block nullification for basis construction).
//
// For box i, Omega^(i) stacks the rows of the test matrix that belong to the
// neighbours of i (ascending box order, rows in order); P^(i) holds r
// orthonormal vectors of null(Omega^(i)).  They are taken from the Householder
// QR of Omega^(i)* (Section 3.2 costs the null spaces as Householder QRs):
// reflectors with the sign that avoids cancellation, P^(i) = the r columns of
// the full orthogonal factor that follow its first |rows of N_i| columns.
// The null vectors depend only on the test matrix and the geometry, so they
// are computed on the host, one box per thread.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>

#include "internal.hpp"

namespace blr {

namespace {

// A: rows x n column-major (overwritten).  out: rows x count, the columns n..n+count-1
// of Q = H_0 H_1 ... H_{n-1}.  False if A is numerically rank deficient.
bool householder_trailing(std::vector<double>& A, int rows, int n, int count, double* out) {
    std::vector<double> V(static_cast<size_t>(rows) * n, 0.0), vnorm2(n, 0.0);
    double rmax = 0.0;
    for (int j = 0; j < n; ++j) {
        double* a = &A[static_cast<size_t>(j) * rows];
        double nrm = 0.0;
        for (int i = j; i < rows; ++i) nrm += a[i] * a[i];
        nrm = std::sqrt(nrm);
        rmax = std::max(rmax, nrm);
        if (nrm <= 1e-12 * rmax) return false;
        double* v = &V[static_cast<size_t>(j) * rows];
        const double alpha = a[j] >= 0 ? -nrm : nrm;
        for (int i = j; i < rows; ++i) v[i] = a[i];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < rows; ++i) vv += v[i] * v[i];
        vnorm2[j] = vv;
        for (int c = j; c < n; ++c) {
            double* ac = &A[static_cast<size_t>(c) * rows];
            double d = 0.0;
            for (int i = j; i < rows; ++i) d += v[i] * ac[i];
            const double f = 2.0 * d / vv;
            for (int i = j; i < rows; ++i) ac[i] -= f * v[i];
        }
    }
    for (int c = 0; c < count; ++c) {
        double* col = out + static_cast<size_t>(c) * rows;
        std::fill(col, col + rows, 0.0);
        col[n + c] = 1.0;
        for (int j = n - 1; j >= 0; --j) {
            const double* v = &V[static_cast<size_t>(j) * rows];
            double d = 0.0;
            for (int i = j; i < rows; ++i) d += v[i] * col[i];
            const double f = 2.0 * d / vnorm2[j];
            for (int i = j; i < rows; ++i) col[i] -= f * v[i];
        }
    }
    return true;
}

}  // namespace

int64_t bn_min_columns(const PlanData& P) {
    int64_t worst = 0;
    for (int i = 0; i < P.b; ++i) {
        int64_t rows = 0;
        for (int q = P.near_ptr[i]; q < P.near_ptr[i + 1]; ++q) {
            const int j = P.near_idx[q];
            rows += P.box_ptr[j + 1] - P.box_ptr[j];
        }
        worst = std::max(worst, rows);
    }
    return worst + P.r;
}

void bn_null_vectors(const PlanData& P, const double* Om, int64_t s, double* Pall) {
    const int r = P.r;
    std::atomic<int> next{0};
    std::atomic<bool> bad{false};
    auto work = [&] {
        std::vector<double> Mt;
        for (int i = next++; i < P.b && !bad; i = next++) {
            int64_t nrows = 0;
            for (int q = P.near_ptr[i]; q < P.near_ptr[i + 1]; ++q) {
                const int j = P.near_idx[q];
                nrows += P.box_ptr[j + 1] - P.box_ptr[j];
            }
            // Omega^(i)*: s x nrows, column q = row q of Omega^(i)
            Mt.assign(static_cast<size_t>(s) * nrows, 0.0);
            int64_t col = 0;
            for (int q = P.near_ptr[i]; q < P.near_ptr[i + 1]; ++q) {
                const int j = P.near_idx[q];
                for (int64_t row = P.box_ptr[j]; row < P.box_ptr[j + 1]; ++row, ++col)
                    for (int64_t t = 0; t < s; ++t) Mt[t + col * s] = Om[row + t * P.n];
            }
            if (!householder_trailing(Mt, static_cast<int>(s), static_cast<int>(nrows), r,
                                      Pall + static_cast<size_t>(i) * s * r))
                bad = true;
        }
    };
    const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned t = 1; t < hw; ++t) th.emplace_back(work);
    work();
    for (auto& x : th) x.join();
    if (bad) fail(BLR_ERR_NUMERICAL, "a neighbour block of the test matrix is rank deficient (block nullification)");
}

}  // namespace blr
