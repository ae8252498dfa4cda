// Host-side simplex geometry shared by the operator builders (p2.cpp, rows.cpp).
#pragma once

#include <algorithm>
#include <cmath>
#include <cstdint>

namespace knp {
namespace host {

// volume and barycentric gradients (rows) of the simplex with vertices x[0..d]
inline double simplex_gradients(int d, const double *x, double *g) {
    double J[3][3] = {}, inv[3][3] = {}, det;
    for (int c = 0; c < d; ++c)
        for (int r = 0; r < d; ++r) J[r][c] = x[(c + 1) * d + r] - x[r];
    if (d == 2) {
        det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
        inv[0][0] = J[1][1] / det;
        inv[0][1] = -J[0][1] / det;
        inv[1][0] = -J[1][0] / det;
        inv[1][1] = J[0][0] / det;
    } else {
        const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
        const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
        const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
        det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
        inv[0][0] = c00 / det;
        inv[1][0] = c01 / det;
        inv[2][0] = c02 / det;
        inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    }
    for (int k = 0; k < d; ++k) {
        double s = 0.0;
        for (int a = 1; a <= d; ++a) {
            g[a * d + k] = inv[a - 1][k];
            s += inv[a - 1][k];
        }
        g[k] = -s;
    }
    return std::fabs(det) / (d == 2 ? 2.0 : 6.0);
}

// measure of the (d-1)-simplex with d vertices x of dimension d
inline double facet_measure(int d, const double *x) {
    if (d == 2) return std::hypot(x[2] - x[0], x[3] - x[1]);
    const double ax = x[3] - x[0], ay = x[4] - x[1], az = x[5] - x[2];
    const double bx = x[6] - x[0], by = x[7] - x[1], bz = x[8] - x[2];
    const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
    return 0.5 * std::sqrt(cx * cx + cy * cy + cz * cz);
}

// position of key in the ascending row[0..n), or -1
inline int find_sorted(const int32_t *row, int n, int32_t key) {
    const int32_t *p = std::lower_bound(row, row + n, key);
    if (p == row + n || *p != key) return -1;
    return int(p - row);
}

}  // namespace host
}  // namespace knp
