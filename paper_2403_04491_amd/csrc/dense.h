// Dense inverses of the coarsest AMG level's components (host, plain C++).
//
// Kept free of HIP and of exceptions so that it runs inside OpenMP regions (an
// exception escaping such a region would terminate the process) and can be
// compiled on its own for host tests.
#pragma once

#include <cmath>
#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

namespace knp {

// Pivots below this fraction of the matrix's largest entry count as zero: the
// inverse of such a block would carry no correct digits.
constexpr double DENSE_PIVOT_TOL = 64.0 * 2.220446049250313e-16;

// Gauss-Jordan with partial pivoting; a (row-major n x n) is replaced by its
// inverse.  Returns false, leaving a in an unspecified state, when a pivot falls
// below DENSE_PIVOT_TOL times the largest |a_ij| (or a holds a NaN/Inf).
inline bool invert_dense(int n, std::vector<double> &a) {
    double amax = 0.0;
    for (double v : a) {
        if (!std::isfinite(v)) return false;
        amax = std::fmax(amax, std::fabs(v));
    }
    if (n > 0 && amax == 0.0) return false;
    const double tiny = DENSE_PIVOT_TOL * amax;
    std::vector<double> inv(size_t(n) * n, 0.0);
    for (int i = 0; i < n; ++i) inv[size_t(i) * n + i] = 1.0;
    for (int c = 0; c < n; ++c) {
        int p = c;
        for (int r = c + 1; r < n; ++r)
            if (std::fabs(a[size_t(r) * n + c]) > std::fabs(a[size_t(p) * n + c])) p = r;
        if (!(std::fabs(a[size_t(p) * n + c]) > tiny)) return false;
        if (p != c)
            for (int k = 0; k < n; ++k) {
                std::swap(a[size_t(p) * n + k], a[size_t(c) * n + k]);
                std::swap(inv[size_t(p) * n + k], inv[size_t(c) * n + k]);
            }
        const double d = 1.0 / a[size_t(c) * n + c];
        for (int k = 0; k < n; ++k) {
            a[size_t(c) * n + k] *= d;
            inv[size_t(c) * n + k] *= d;
        }
        for (int r = 0; r < n; ++r) {
            if (r == c) continue;
            const double f = a[size_t(r) * n + c];
            if (f == 0.0) continue;
            for (int k = 0; k < n; ++k) {
                a[size_t(r) * n + k] -= f * a[size_t(c) * n + k];
                inv[size_t(r) * n + k] -= f * inv[size_t(c) * n + k];
            }
        }
    }
    a.swap(inv);
    return true;
}

}  // namespace knp
