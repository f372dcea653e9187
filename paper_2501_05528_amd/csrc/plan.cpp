// Host planner for tagged uBLR compression: admissibility lists, probe
// colours, tag vectors z^(i) and their aspect ratios.
//
// * Neighbours (Section 2.5): boxes sharing a boundary with box i, i
//   included; on a box lattice that is Chebyshev distance <= 1.
// * Tag vectors (Alg. 2; eq. tagsubmat): z^(i) lies in null(T(N_i,:)).  The
//   null space comes from a Householder QR of T(N_i,:)^T.
// * Aspect ratio (eq. aspect_ratio) and its minimisation (Section 5.3): on
//   each sign cell of the null space the ratio max|t_l^T x| / min|t_l^T x|
//   over the far field is minimised exactly as the linear program
//       min tau  s.t.  1 <= sigma_l t_l^T X alpha <= tau,  l in F_i,
//   in null-space coordinates alpha.  It is solved here through its dual
//   (s+1 equality rows) by a two-phase tableau simplex, and the primal
//   vertex is recovered from the optimal basis.  Start cells come from the
//   projections of e_1..e_ell onto the null space; ties within a relative
//   1e-9 go to the earliest start; z has unit norm and its largest-magnitude
//   entry positive.
#include <algorithm>
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <set>
#include <sstream>
#include <thread>

#include "internal.hpp"

namespace blr {

namespace {

void neighbour_csr(int dim, int b, const int32_t* lat, std::vector<int32_t>& ptr,
                   std::vector<int32_t>& idx) {
    ptr.assign(b + 1, 0);
    idx.clear();
    for (int i = 0; i < b; ++i) {
        for (int j = 0; j < b; ++j) {
            int cheb = 0;
            for (int t = 0; t < dim; ++t)
                cheb = std::max(cheb, std::abs(lat[i * dim + t] - lat[j * dim + t]));
            if (cheb <= 1) idx.push_back(j);
        }
        ptr[i + 1] = static_cast<int32_t>(idx.size());
    }
}

// Neighbour lists of a geometry: the caller's CSR (validated) or the lattice rule.
void geometry_near(const blr_geometry* g, std::vector<int32_t>& ptr, std::vector<int32_t>& idx) {
    const int b = g->nboxes;
    if (!g->near_ptr) {
        if (!g->box_lattice) fail(BLR_ERR_INVALID_ARG, "need box_lattice or explicit neighbour lists");
        neighbour_csr(g->dim, b, g->box_lattice, ptr, idx);
        return;
    }
    if (!g->near_idx) fail(BLR_ERR_INVALID_ARG, "near_ptr given without near_idx");
    if (g->near_ptr[0] != 0) fail(BLR_ERR_INVALID_ARG, "near_ptr[0] must be 0");
    for (int i = 0; i < b; ++i)
        if (g->near_ptr[i + 1] < g->near_ptr[i]) fail(BLR_ERR_INVALID_ARG, "near_ptr must be non-decreasing");
    if (static_cast<int64_t>(g->near_ptr[b]) > static_cast<int64_t>(b) * b)
        fail(BLR_ERR_INVALID_ARG, "more neighbour entries than box pairs");
    ptr.assign(g->near_ptr, g->near_ptr + b + 1);
    idx.assign(g->near_idx, g->near_idx + g->near_ptr[b]);
    for (int i = 0; i < b; ++i) {
        bool self = false;
        for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
            if (idx[q] < 0 || idx[q] >= b) fail(BLR_ERR_INVALID_ARG, "neighbour index out of range");
            if (q > ptr[i] && idx[q] <= idx[q - 1]) fail(BLR_ERR_INVALID_ARG, "neighbour lists must be strictly ascending");
            self |= idx[q] == i;
        }
        if (!self) fail(BLR_ERR_INVALID_ARG, "every box must be its own neighbour");
    }
}

// Greedy distance-2 colouring for explicit lists: box i (in index order) takes the smallest
// colour not held by an earlier box l with a common neighbour (l in N_j for some j in N_i).
int greedy_colours(int b, const std::vector<int32_t>& ptr, const std::vector<int32_t>& idx,
                   std::vector<int32_t>& colour) {
    colour.assign(b, -1);
    std::vector<int> seen;      // seen[c] == i + 1: colour c is taken for box i
    int ncol = 0;
    for (int i = 0; i < b; ++i) {
        for (int q = ptr[i]; q < ptr[i + 1]; ++q) {
            const int j = idx[q];
            for (int u = ptr[j]; u < ptr[j + 1]; ++u) {
                const int c = colour[idx[u]];
                if (c >= 0) {
                    if (c >= static_cast<int>(seen.size())) seen.resize(c + 1, 0);
                    seen[c] = i + 1;
                }
            }
        }
        int c = 0;
        while (c < static_cast<int>(seen.size()) && seen[c] == i + 1) ++c;
        colour[i] = c;
        ncol = std::max(ncol, c + 1);
    }
    return ncol;
}

// ---------------------------------------------------------------- null space
// Orthonormal basis (ell x s, column-major) of null(M) for M = T(N_i,:)
// (n x ell), from the Householder QR of M^T.  Returns false if M^T is
// numerically rank deficient.
bool null_basis(const std::vector<double>& Mt_in, int ell, int n, std::vector<double>& X) {
    std::vector<double> A = Mt_in;  // ell x n column-major
    std::vector<std::vector<double>> vs;
    double rmax = 0.0;
    for (int j = 0; j < n; ++j) {
        double nrm = 0.0;
        for (int i = j; i < ell; ++i) nrm += A[i + j * ell] * A[i + j * ell];
        nrm = std::sqrt(nrm);
        rmax = std::max(rmax, nrm);
        if (nrm <= 1e-12 * std::max(rmax, 1.0)) return false;
        std::vector<double> v(ell, 0.0);
        double x0 = A[j + j * ell];
        double alpha = x0 >= 0 ? -nrm : nrm;
        for (int i = j; i < ell; ++i) v[i] = A[i + j * ell];
        v[j] -= alpha;
        double vv = 0.0;
        for (int i = j; i < ell; ++i) vv += v[i] * v[i];
        for (int c = j; c < n; ++c) {
            double d = 0.0;
            for (int i = j; i < ell; ++i) d += v[i] * A[i + c * ell];
            double f = 2.0 * d / vv;
            for (int i = j; i < ell; ++i) A[i + c * ell] -= f * v[i];
        }
        vs.push_back(std::move(v));
        (void)alpha;
    }
    int s = ell - n;
    X.assign(static_cast<size_t>(ell) * s, 0.0);
    for (int c = 0; c < s; ++c) {
        double* col = &X[static_cast<size_t>(c) * ell];
        col[n + c] = 1.0;
        for (int j = n - 1; j >= 0; --j) {
            const std::vector<double>& v = vs[j];
            double d = 0.0, vv = 0.0;
            for (int i = j; i < ell; ++i) {
                d += v[i] * col[i];
                vv += v[i] * v[i];
            }
            double f = 2.0 * d / vv;
            for (int i = j; i < ell; ++i) col[i] -= f * v[i];
        }
    }
    return true;
}

// Solve the square system M y = rhs (M n x n column-major) by Gaussian
// elimination with partial pivoting.  Returns false if singular.
bool solve_square(std::vector<double> M, std::vector<double> rhs, int n, std::vector<double>& y) {
    for (int c = 0; c < n; ++c) {
        int piv = c;
        for (int i = c + 1; i < n; ++i)
            if (std::fabs(M[i + c * n]) > std::fabs(M[piv + c * n])) piv = i;
        if (std::fabs(M[piv + c * n]) < 1e-300) return false;
        if (piv != c) {
            for (int j = 0; j < n; ++j) std::swap(M[c + j * n], M[piv + j * n]);
            std::swap(rhs[c], rhs[piv]);
        }
        for (int i = c + 1; i < n; ++i) {
            double f = M[i + c * n] / M[c + c * n];
            if (f == 0.0) continue;
            for (int j = c; j < n; ++j) M[i + j * n] -= f * M[c + j * n];
            rhs[i] -= f * rhs[c];
        }
    }
    y.assign(n, 0.0);
    for (int i = n - 1; i >= 0; --i) {
        double acc = rhs[i];
        for (int j = i + 1; j < n; ++j) acc -= M[i + j * n] * y[j];
        y[i] = acc / M[i + i * n];
    }
    return true;
}

// ---------------------------------------------------------------- LP
// minimise tau s.t. 1 <= a_l^T alpha <= tau (l < F), alpha in R^s, where a is
// s x F column-major.  Solved through the dual
//   min -sum(lambda) s.t. sum_l (lambda_l - mu_l) a_l = 0, sum_l mu_l = 1,
//   lambda, mu >= 0,
// whose simplex multipliers y give alpha = -y(0:s).  Returns false on failure.
bool cell_lp(const std::vector<double>& a, int s, int F, std::vector<double>& alpha, double& tau) {
    const int R = s + 1;                 // rows
    const int nstruct = 2 * F;           // lambda_0..F-1, mu_0..F-1
    const int ncol = nstruct + R;        // + artificials
    const int W = ncol + 1;              // + rhs
    auto colvec = [&](int j, int row) -> double {
        if (j < F) return row < s ? a[row + static_cast<size_t>(j) * s] : 0.0;
        if (j < 2 * F) return row < s ? -a[row + static_cast<size_t>(j - F) * s] : 1.0;
        return (j - nstruct) == row ? 1.0 : 0.0;
    };
    std::vector<double> tab(static_cast<size_t>(R + 1) * W, 0.0);
    auto at = [&](int i, int j) -> double& { return tab[static_cast<size_t>(i) * W + j]; };
    for (int i = 0; i < R; ++i) {
        for (int j = 0; j < ncol; ++j) at(i, j) = colvec(j, i);
        at(i, ncol) = (i == R - 1) ? 1.0 : 0.0;
    }
    std::vector<int> basis(R);
    for (int i = 0; i < R; ++i) basis[i] = nstruct + i;
    const double eps = 1e-11;

    auto pivot = [&](int pr, int pc) {
        double pv = at(pr, pc);
        for (int j = 0; j < W; ++j) at(pr, j) /= pv;
        for (int i = 0; i <= R; ++i) {
            if (i == pr) continue;
            double f = at(i, pc);
            if (f == 0.0) continue;
            for (int j = 0; j < W; ++j) at(i, j) -= f * at(pr, j);
        }
        basis[pr] = pc;
    };
    // Runs the simplex on the current objective row; cols >= allowed are barred.
    auto run = [&](int allowed) -> int {
        const long max_it = 200L * (R + ncol) + 1000;
        int degenerate = 0;
        for (long it = 0; it < max_it; ++it) {
            bool bland = degenerate > 50;
            int pc = -1;
            double best = -eps;
            for (int j = 0; j < allowed; ++j) {
                double d = at(R, j);
                if (d < best) {
                    pc = j;
                    if (bland) break;
                    best = d;
                }
            }
            if (pc < 0) return 0;  // optimal
            int pr = -1;
            double rmin = 0.0;
            for (int i = 0; i < R; ++i) {
                double v = at(i, pc);
                if (v > eps) {
                    double ratio = at(i, ncol) / v;
                    if (pr < 0 || ratio < rmin - 1e-14 ||
                        (ratio <= rmin + 1e-14 && basis[i] < basis[pr])) {
                        pr = i;
                        rmin = ratio;
                    }
                }
            }
            if (pr < 0) return 2;  // unbounded
            degenerate = (rmin <= 1e-14) ? degenerate + 1 : 0;
            pivot(pr, pc);
        }
        return 1;  // iteration limit
    };
    // Phase I: minimise the sum of artificials.
    for (int j = 0; j < W; ++j) {
        double acc = 0.0;
        if (j < nstruct || j == ncol)
            for (int i = 0; i < R; ++i) acc -= at(i, j);
        at(R, j) = acc;
    }
    if (run(nstruct) != 0) return false;
    if (-at(R, ncol) > 1e-9) return false;  // infeasible
    for (int i = 0; i < R; ++i) {            // drive artificials out of the basis
        if (basis[i] < nstruct) continue;
        int pc = -1;
        for (int j = 0; j < nstruct; ++j)
            if (std::fabs(at(i, j)) > 1e-9) { pc = j; break; }
        if (pc >= 0) pivot(i, pc);
    }
    // Phase II objective: c = -1 on lambda, 0 elsewhere.
    auto cost = [&](int j) -> double { return j < F ? -1.0 : 0.0; };
    for (int j = 0; j < W; ++j) {
        double acc = (j < ncol) ? cost(j) : 0.0;
        for (int i = 0; i < R; ++i) acc -= cost(basis[i]) * at(i, j);
        at(R, j) = acc;
    }
    if (run(nstruct) != 0) return false;
    // Multipliers: B^T y = c_B.
    std::vector<double> Bt(static_cast<size_t>(R) * R), cb(R);
    for (int i = 0; i < R; ++i) {       // row i of B^T = column basis[i] of B
        for (int q = 0; q < R; ++q) Bt[i + static_cast<size_t>(q) * R] = colvec(basis[i], q);
        cb[i] = cost(basis[i]);
    }
    std::vector<double> y;
    if (!solve_square(Bt, cb, R, y)) return false;
    alpha.assign(s, 0.0);
    for (int q = 0; q < s; ++q) alpha[q] = -y[q];
    double lo = 1e300, hi = -1e300;
    for (int l = 0; l < F; ++l) {
        double v = 0.0;
        for (int q = 0; q < s; ++q) v += a[q + static_cast<size_t>(l) * s] * alpha[q];
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    if (!(lo > 0.5)) return false;  // the vertex must satisfy a_l^T alpha >= 1
    tau = hi / lo;
    for (int q = 0; q < s; ++q) alpha[q] /= lo;
    return true;
}

void canonical_sign(std::vector<double>& z) {
    int q = 0;
    for (size_t j = 1; j < z.size(); ++j)
        if (std::fabs(z[j]) > std::fabs(z[q])) q = static_cast<int>(j);
    if (z[q] < 0)
        for (double& v : z) v = -v;
}

double ratio_of(const PlanData& P, int i, const std::vector<double>& z) {
    double lo = 1e300, hi = 0.0;
    int b = P.b, ell = P.ell;
    for (int j = 0; j < b; ++j) {
        bool nearj = false;
        for (int q = P.near_ptr[i]; q < P.near_ptr[i + 1]; ++q) nearj |= (P.near_idx[q] == j);
        if (nearj) continue;
        double c = 0.0;
        for (int s = 0; s < ell; ++s) c += P.T[j + static_cast<size_t>(s) * b] * z[s];
        lo = std::min(lo, std::fabs(c));
        hi = std::max(hi, std::fabs(c));
    }
    return hi / lo;
}

// Tag vector and aspect ratio of box i.  Returns false if T(N_i,:) is rank deficient.
bool box_tag(PlanData& P, int i, std::vector<double>& zout, double& rho) {
    const int ell = P.ell, b = P.b;
    const int n0 = P.near_ptr[i], n1 = P.near_ptr[i + 1], nn = n1 - n0;
    std::vector<double> Mt(static_cast<size_t>(ell) * nn);
    for (int c = 0; c < nn; ++c)
        for (int s = 0; s < ell; ++s) Mt[s + static_cast<size_t>(c) * ell] = P.T[P.near_idx[n0 + c] + static_cast<size_t>(s) * b];
    std::vector<double> X;
    if (!null_basis(Mt, ell, nn, X)) return false;
    const int s = ell - nn;
    // far rows of T
    std::vector<int> far;
    for (int j = 0, q = n0; j < b; ++j) {
        if (q < n1 && P.near_idx[q] == j) { ++q; continue; }
        far.push_back(j);
    }
    const int F = static_cast<int>(far.size());
    // c_l(alpha) = t_l^T X alpha  ->  g_l = X^T t_l (s x F)
    std::vector<double> g(static_cast<size_t>(s) * F);
    for (int l = 0; l < F; ++l)
        for (int q = 0; q < s; ++q) {
            double acc = 0.0;
            for (int t = 0; t < ell; ++t) acc += X[t + static_cast<size_t>(q) * ell] * P.T[far[l] + static_cast<size_t>(t) * b];
            g[q + static_cast<size_t>(l) * s] = acc;
        }
    // starts: projections of e_j onto the null space, in alpha coordinates X(j,:)^T
    std::vector<std::vector<double>> starts;
    for (int j = 0; j < ell; ++j) {
        std::vector<double> al(s);
        double nrm = 0.0;
        for (int q = 0; q < s; ++q) {
            al[q] = X[j + static_cast<size_t>(q) * ell];
            nrm += al[q] * al[q];
        }
        if (std::sqrt(nrm) > 1e-12) starts.push_back(al);
    }
    std::vector<double> best_alpha;
    double best_tau = 0.0;
    bool have = false;
    if (P.aspect_opt) {
        std::set<std::vector<int8_t>> seen;
        for (const auto& al : starts) {
            std::vector<int8_t> sig(F);
            bool zero = false;
            for (int l = 0; l < F; ++l) {
                double c = 0.0;
                for (int q = 0; q < s; ++q) c += g[q + static_cast<size_t>(l) * s] * al[q];
                if (c == 0.0) zero = true;
                sig[l] = c > 0 ? 1 : -1;
            }
            if (zero) continue;
            if (sig[0] < 0)
                for (auto& v : sig) v = -v;
            if (!seen.insert(sig).second) continue;
            std::vector<double> a(static_cast<size_t>(s) * F);
            for (int l = 0; l < F; ++l)
                for (int q = 0; q < s; ++q) a[q + static_cast<size_t>(l) * s] = sig[l] * g[q + static_cast<size_t>(l) * s];
            std::vector<double> alpha;
            double tau;
            if (!cell_lp(a, s, F, alpha, tau)) continue;
            if (!have || tau < best_tau * (1.0 - 1e-9)) {
                best_alpha = alpha;
                best_tau = tau;
                have = true;
            }
        }
    }
    if (!have) best_alpha = starts.front();
    std::vector<double> z(ell, 0.0);
    for (int t = 0; t < ell; ++t)
        for (int q = 0; q < s; ++q) z[t] += X[t + static_cast<size_t>(q) * ell] * best_alpha[q];
    double nrm = 0.0;
    for (double v : z) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (double& v : z) v /= nrm;
    canonical_sign(z);
    zout = z;
    rho = ratio_of(P, i, z);
    return true;
}

}  // namespace

int tag_columns(const blr_geometry* g, int extra) {
    if (!g || g->dim < 1 || g->dim > 3 || g->nboxes < 2 || (!g->box_lattice && !g->near_ptr))
        fail(BLR_ERR_INVALID_ARG, "tag_columns: bad geometry");
    if (extra < 0) fail(BLR_ERR_INVALID_ARG, "extra_tag_cols must be >= 0");
    std::vector<int32_t> ptr, idx;
    geometry_near(g, ptr, idx);
    int mx = 0;
    for (int i = 0; i < g->nboxes; ++i) mx = std::max(mx, ptr[i + 1] - ptr[i]);
    return mx + 1 + extra;
}

std::shared_ptr<PlanData> build_plan(const blr_geometry* g, const blr_tag_params* prm) {
    if (!g || !prm) fail(BLR_ERR_INVALID_ARG, "NULL geometry or params");
    if (g->dim < 1 || g->dim > 3) fail(BLR_ERR_INVALID_ARG, "dim must be 1, 2 or 3");
    if (g->nboxes < 2) fail(BLR_ERR_INVALID_ARG, "need at least 2 boxes");
    if (!g->box_ptr) fail(BLR_ERR_INVALID_ARG, "NULL box_ptr");
    if (!g->box_lattice && !g->near_ptr) fail(BLR_ERR_INVALID_ARG, "need box_lattice or explicit neighbour lists");
    if (prm->k < 1 || prm->p < 0 || prm->extra_tag_cols < 0)
        fail(BLR_ERR_INVALID_ARG, "need k >= 1, p >= 0, extra_tag_cols >= 0");
    if (!prm->T) fail(BLR_ERR_INVALID_ARG, "NULL tagging matrix T");
    auto P = std::make_shared<PlanData>();
    P->dim = g->dim;
    P->b = g->nboxes;
    P->k = prm->k;
    P->p = prm->p;
    P->r = prm->k + prm->p;
    P->extra = prm->extra_tag_cols;
    P->aspect_opt = prm->aspect_opt ? 1 : 0;
    const int b = P->b, dim = P->dim;
    P->box_ptr.assign(g->box_ptr, g->box_ptr + b + 1);
    if (P->box_ptr[0] != 0) fail(BLR_ERR_INVALID_ARG, "box_ptr[0] must be 0");
    P->m_max = 0;
    P->m_min = INT32_MAX;
    for (int i = 0; i < b; ++i) {
        int64_t m = P->box_ptr[i + 1] - P->box_ptr[i];
        if (m <= 0) fail(BLR_ERR_INVALID_ARG, "box_ptr must be strictly increasing");
        if (m > (1 << 20)) fail(BLR_ERR_INVALID_ARG, "box too large");
        P->m_max = std::max<int>(P->m_max, static_cast<int>(m));
        P->m_min = std::min<int>(P->m_min, static_cast<int>(m));
    }
    P->n = P->box_ptr[b];
    if (P->r > P->m_min) {
        std::ostringstream os;
        os << "k + p = " << P->r << " exceeds the smallest box (" << P->m_min << " points)";
        fail(BLR_ERR_INVALID_ARG, os.str());
    }
    P->custom_near = g->near_ptr != nullptr;
    if (g->box_lattice) {
        P->lattice.assign(g->box_lattice, g->box_lattice + static_cast<size_t>(b) * dim);
        std::set<std::vector<int32_t>> uniq;
        for (int i = 0; i < b; ++i)
            if (!uniq.insert(std::vector<int32_t>(&P->lattice[i * dim], &P->lattice[i * dim] + dim)).second)
                fail(BLR_ERR_INVALID_ARG, "duplicate box lattice coordinates");
    }
    geometry_near(g, P->near_ptr, P->near_idx);
    P->near_nnz = static_cast<int64_t>(P->near_idx.size());
    int maxnear = 0;
    for (int i = 0; i < b; ++i) {
        int nn = P->near_ptr[i + 1] - P->near_ptr[i];
        maxnear = std::max(maxnear, nn);
        if (nn == b) {
            std::ostringstream os;
            os << "box " << i << " has an empty far field";
            fail(BLR_ERR_GEOMETRY, os.str());
        }
    }
    P->ell = maxnear + 1 + P->extra;
    // colours
    if (P->custom_near) {
        P->ncol = greedy_colours(b, P->near_ptr, P->near_idx, P->colour);
    } else {
        P->ncol = 1;
        for (int t = 0; t < dim; ++t) P->ncol *= 3;
        P->colour.resize(b);
        for (int i = 0; i < b; ++i) {
            int c = 0, w = 1;
            for (int t = 0; t < dim; ++t) {
                int v = P->lattice[i * dim + t] % 3;
                if (v < 0) v += 3;
                c += v * w;
                w *= 3;
            }
            P->colour[i] = c;
        }
    }
    P->colour_ptr.assign(P->ncol + 1, 0);
    for (int i = 0; i < b; ++i) P->colour_ptr[P->colour[i] + 1]++;
    for (int c = 0; c < P->ncol; ++c) P->colour_ptr[c + 1] += P->colour_ptr[c];
    P->colour_boxes.resize(b);
    {
        std::vector<int32_t> fill(P->colour_ptr.begin(), P->colour_ptr.end() - 1);
        for (int i = 0; i < b; ++i) P->colour_boxes[fill[P->colour[i]]++] = i;
    }
    P->nf_pair.assign(static_cast<size_t>(b) * P->ncol, -1);
    for (int i = 0; i < b; ++i)
        for (int q = P->near_ptr[i]; q < P->near_ptr[i + 1]; ++q) {
            int c = P->colour[P->near_idx[q]];
            if (P->nf_pair[static_cast<size_t>(i) * P->ncol + c] != -1)
                fail(BLR_ERR_GEOMETRY, "two neighbours share a probe colour");
            P->nf_pair[static_cast<size_t>(i) * P->ncol + c] = q;
        }
    P->b_off.resize(P->near_nnz);
    int64_t off = 0;
    for (int i = 0; i < b; ++i)
        for (int q = P->near_ptr[i]; q < P->near_ptr[i + 1]; ++q) {
            P->b_off[q] = off;
            int j = P->near_idx[q];
            off += (P->box_ptr[i + 1] - P->box_ptr[i]) * (P->box_ptr[j + 1] - P->box_ptr[j]);
        }
    P->b_values = off;
    P->near_tpos.resize(P->near_nnz);
    for (int i = 0; i < b; ++i)
        for (int q = P->near_ptr[i]; q < P->near_ptr[i + 1]; ++q) {
            const int j = P->near_idx[q];
            int pos = -1;
            for (int u = P->near_ptr[j]; u < P->near_ptr[j + 1]; ++u)
                if (P->near_idx[u] == i) pos = u;
            if (pos < 0) fail(BLR_ERR_GEOMETRY, "neighbour relation is not symmetric");
            P->near_tpos[q] = pos;
        }
    P->row_box.resize(P->n);
    for (int i = 0; i < b; ++i)
        for (int64_t a = P->box_ptr[i]; a < P->box_ptr[i + 1]; ++a) P->row_box[a] = i;
    // 32-row source steps of the low-precision sketch (steps never straddle a box)
    P->kstep_ptr.assign(b + 1, 0);
    for (int i = 0; i < b; ++i) {
        const int64_t steps = (P->box_ptr[i + 1] - P->box_ptr[i] + 31) / 32;
        if (P->kstep_ptr[i] + steps > INT32_MAX) fail(BLR_ERR_UNSUPPORTED, "too many source steps");
        P->kstep_ptr[i + 1] = P->kstep_ptr[i] + static_cast<int32_t>(steps);
    }
    P->kstep_box.resize(P->kstep_ptr[b]);
    for (int i = 0; i < b; ++i)
        for (int q = P->kstep_ptr[i]; q < P->kstep_ptr[i + 1]; ++q) P->kstep_box[q] = i;
    P->pair_row.resize(P->near_nnz);
    for (int i = 0; i < b; ++i)
        for (int q = P->near_ptr[i]; q < P->near_ptr[i + 1]; ++q) P->pair_row[q] = i;
    // neighbour mask for the far-field refinement sketch
    P->nearm.assign(static_cast<size_t>(b) * b, 0);
    for (int i = 0; i < b; ++i)
        for (int q = P->near_ptr[i]; q < P->near_ptr[i + 1]; ++q)
            P->nearm[static_cast<size_t>(i) * b + P->near_idx[q]] = 1;
    // tagging matrix and tag vectors
    P->T.assign(prm->T, prm->T + static_cast<size_t>(b) * P->ell);
    for (double v : P->T)
        if (!std::isfinite(v)) fail(BLR_ERR_INVALID_ARG, "non-finite entry in T");
    P->z.assign(static_cast<size_t>(b) * P->ell, 0.0);
    P->rho.assign(b, 0.0);
    std::atomic<int> next(0), bad(-1);
    unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    if (b < 64) nth = 1;
    auto worker = [&]() {
        std::vector<double> z;
        for (;;) {
            int i = next.fetch_add(1);
            if (i >= b) break;
            double rho = 0.0;
            if (!box_tag(*P, i, z, rho)) {
                bad.store(i);
                continue;
            }
            for (int s = 0; s < P->ell; ++s) P->z[i + static_cast<size_t>(s) * b] = z[s];
            P->rho[i] = rho;
        }
    };
    std::vector<std::thread> pool;
    for (unsigned t = 1; t < nth; ++t) pool.emplace_back(worker);
    worker();
    for (auto& th : pool) th.join();
    if (bad.load() >= 0) {
        std::ostringstream os;
        os << "tag submatrix T(N_i,:) is rank deficient for box " << bad.load();
        fail(BLR_ERR_GEOMETRY, os.str());
    }
    return P;
}

}  // namespace blr
