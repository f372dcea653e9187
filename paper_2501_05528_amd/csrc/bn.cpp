// Sizing of Alg. 1 (block nullification for basis construction): the test matrix needs
// r more columns than the rows of the largest neighbourhood, so that every box keeps r
// null vectors of its neighbours' rows (the null vectors themselves are computed on the
// device, k_bn_null).
#include <algorithm>

#include "internal.hpp"

namespace blr {

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

}  // namespace blr
