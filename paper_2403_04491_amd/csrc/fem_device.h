// Device helpers for P1 finite elements on simplices, shared by the assembly
// and vector-Jacobian-product kernels: barycentric gradients, exact simplex
// moments int prod lambda_a^{p_a} = m! |T| prod p_a! / (m + sum p_a)!, facet measures.
#pragma once

#include <hip/hip_runtime.h>

#include "knp_internal.h"

namespace knp {
namespace fem {

using launch::MeshArgs;

// Volume and barycentric gradients of a simplex with vertices x[a] (D = 2 or 3).
template <int D>
__device__ inline double simplex_grads(const double (&x)[D + 1][D], double (&g)[D + 1][D]) {
    double J[D][D];   // J[r][c] = x[c+1][r] - x[0][r]
#pragma unroll
    for (int c = 0; c < D; ++c)
#pragma unroll
        for (int r = 0; r < D; ++r) J[r][c] = x[c + 1][r] - x[0][r];
    double det, inv[D][D];
    if constexpr (D == 2) {
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
    // rows of J^{-1} are grad(lambda_1..D); grad(lambda_0) = -sum
#pragma unroll
    for (int d = 0; d < D; ++d) {
        double s = 0.0;
#pragma unroll
        for (int a = 1; a <= D; ++a) {
            g[a][d] = inv[a - 1][d];
            s += inv[a - 1][d];
        }
        g[0][d] = -s;
    }
    const double fact = (D == 2) ? 2.0 : 6.0;
    return fabs(det) / fact;
}

template <int D>
__device__ inline void load_simplex(const MeshArgs &ma, int32_t e, int32_t (&vg)[D + 1], double (&x)[D + 1][D]) {
#pragma unroll
    for (int a = 0; a <= D; ++a) {
        vg[a] = ma.elem[int64_t(e) * (D + 1) + a];
#pragma unroll
        for (int d = 0; d < D; ++d) x[a][d] = ma.xyz[int64_t(vg[a]) * D + d];
    }
}

// int over a D-simplex of lambda_a lambda_b, divided by |T|
template <int D>
__device__ inline double mass_moment(bool same) {
    return (same ? 2.0 : 1.0) / double((D + 1) * (D + 2));
}

// facet (dimension m = D-1) moments divided by |F|
template <int D>
__device__ inline double fmom2(int a, int b) {
    constexpr int m = D - 1;
    constexpr double base = (m == 1) ? 1.0 / 6.0 : 1.0 / 12.0;   // m!/(m+2)!
    return (a == b ? 2.0 : 1.0) * base;
}
template <int D>
__device__ inline double fmom3(int a, int b, int c) {
    constexpr int m = D - 1;
    constexpr double base = (m == 1) ? 1.0 / 24.0 : 1.0 / 60.0;  // m!/(m+3)!
    const int eq = (a == b) + (a == c) + (b == c);
    const double mult = eq == 3 ? 6.0 : (eq == 1 ? 2.0 : 1.0);
    return mult * base;
}

template <int D>
__device__ inline double facet_measure(const MeshArgs &ma, const int32_t *fv) {
    double x[D][D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
        for (int d = 0; d < D; ++d) x[a][d] = ma.xyz[int64_t(fv[a]) * D + d];
    if constexpr (D == 2) {
        const double dx = x[1][0] - x[0][0], dy = x[1][1] - x[0][1];
        return sqrt(dx * dx + dy * dy);
    } else {
        const double ax = x[1][0] - x[0][0], ay = x[1][1] - x[0][1], az = x[1][2] - x[0][2];
        const double bx = x[2][0] - x[0][0], by = x[2][1] - x[0][1], bz = x[2][2] - x[0][2];
        const double cx = ay * bz - az * by, cy = az * bx - ax * bz, cz = ax * by - ay * bx;
        return 0.5 * sqrt(cx * cx + cy * cy + cz * cz);
    }
}

}  // namespace fem
}  // namespace knp
