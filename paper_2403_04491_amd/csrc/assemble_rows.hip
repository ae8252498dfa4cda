// Per-step bulk values of an order-1 mesh from the row terms (see RowTerms): the
// c_r^k rows' phi_r block tilde-tau_k A_r^k, the phi_r row's phi_r block
// sum_k z_k tilde-tau_k A_r^k, f_r^k = M_r c^{k,n-1} and f_r^phi = 0, where A_r^k is the
// stiffness weighted by c^{k,n-1} (eq. ``lin_sys``).
//
// One wavefront per group of consecutive rows (at most 64 entries): lane x owns entry x
// of the group, loads its column's three concentrations once, and reads the
// concentrations at the weight vertices from the lanes of its row by cross-lane
// permutes, so every global load is coalesced and independent of the others.  The
// diagonal value (minus the row's off-diagonal sum) and f (the mass row times c) are
// segmented sums over the row's lanes.  Sums run in a fixed order and no atomics are
// used, so the values are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "knp_internal.h"

namespace knp {
namespace launch {

namespace {

constexpr int RBLK = 256;   // four wavefronts, one group each

template <int D>
__global__ void __launch_bounds__(RBLK) k_rows_dynamic(RegionArgs ra, RowView rv, PhysArgs p,
                                                        const int64_t *__restrict__ rowptr,
                                                        const int64_t *__restrict__ rstart, double *__restrict__ vals,
                                                        const double *__restrict__ sc, const double *__restrict__ u,
                                                        double *__restrict__ f, int64_t pin_dof) {
    const int64_t w = (int64_t(blockIdx.x) * RBLK + threadIdx.x) >> 6;
    const int lane = int(threadIdx.x & 63u);
    if (w >= rv.ngroups) return;   // the whole wavefront
    const RowGroup G = rv.groups[w];
    const int64_t e0 = ra.prow[G.row0];
    const int ne = int(ra.prow[rv.groups[w + 1].row0] - e0);
    const bool valid = lane < ne;
    // my row: the last row start at or below my lane; its end: the next start, or ne
    const uint64_t le = lane == 63 ? ~uint64_t(0) : (uint64_t(2) << lane) - 1;
    const uint64_t upto = G.starts & le, above = G.starts & ~le;
    const int rb = 63 - __builtin_clzll(upto);
    const int re = above ? __builtin_ctzll(above) : ne;
    const int64_t j = G.row0 + __popcll(upto) - 1;
    const int n = re - rb, q = lane - rb;
    const int64_t e = e0 + lane;
    const int64_t Nr = ra.Nr;
    const double *cb = u + ra.off;
    const int32_t col = valid ? ra.pcol[e] : 0;
    double cc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) cc[k] = valid ? cb[k * Nr + col] : 0.0;
    const bool diag = valid && col == j;
    const uint64_t dmask = __ballot(diag);
    const int dl = rb + __builtin_ctzll(dmask >> rb);
    double ci[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) ci[k] = __shfl(cc[k], dl);
    // ring sum of my entry: sum_t w_t c(slot_t), and sum_t w_t
    const int cnt = valid ? int(rv.tcount[e]) : 0;
    int incl = cnt;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int v = __shfl_up(incl, d);
        if (lane >= d) incl += v;
    }
    const int64_t t0 = G.term0 + (incl - cnt);
    double acc[3] = {0.0, 0.0, 0.0}, wsum = 0.0;
    for (int t = 0; t < G.tmax; ++t) {
        const bool has = t < cnt;
        const double wt = has ? rv.tval[t0 + t] : 0.0;
        const int src = rb + (has ? int(rv.tslot[t0 + t]) : 0);
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += wt * __shfl(cc[k], src);
        wsum += wt;
    }
    constexpr double inv_dm1 = 1.0 / double(D - 1);   // (c_i + c_j) / (d - 1)
    double V[3], red[6];
    const double mv = valid ? rv.mval[e] : 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        V[k] = acc[k] + wsum * (ci[k] + cc[k]) * inv_dm1;
        red[k] = (valid && !diag) ? V[k] : 0.0;
        red[3 + k] = mv * cc[k];
    }
    // segmented sums over my row's lanes: lane rb ends with the row's totals
    for (int d = 1; d < G.nmax; d <<= 1) {
        const bool take = lane + d < re;
#pragma unroll
        for (int k = 0; k < 6; ++k) {
            const double v = __shfl_down(red[k], d);
            if (take) red[k] += v;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double tot = __shfl(red[k], rb);
        if (diag) V[k] = -tot;
    }
    if (!valid) return;
    const int64_t phib = ra.off + 3 * Nr;
    const int64_t colg = phib + col;
    const double scol = sc[colg];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int64_t row = ra.off + k * Nr + j;
        const int gq = int(rowptr[row + 1] - rowptr[row]) - 2 * n;
        const int64_t seg = rstart[row] + (ra.r == 0 ? 0 : gq) + n;
        vals[seg + q] = colg == pin_dof ? 0.0 : p.ttau[k] * V[k] * sc[row] * scol;
        if (lane == rb) f[row] = red[3 + k];
    }
    const int64_t row = phib + j;
    const int gq = int(rowptr[row + 1] - rowptr[row]) - 4 * n;
    const int64_t seg = rstart[row] + (ra.r == 0 ? 0 : gq) + 3 * n;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) v += p.z[k] * p.ttau[k] * V[k];
    const bool keep = row == pin_dof ? (colg == row) : (colg != pin_dof);
    vals[seg + q] = keep ? v * sc[row] * scol : 0.0;
    if (lane == rb) f[row] = 0.0;
}

}  // namespace

void rows_dynamic(const RegionArgs &ra, const RowView &rv, const PhysArgs &p, const int64_t *rowptr,
                  const int64_t *rstart, double *vals, const double *sc, const double *u_prev, double *f,
                  int64_t pin_dof, hipStream_t s) {
    if (rv.ngroups == 0) return;
    const unsigned nb = unsigned((rv.ngroups * 64 + RBLK - 1) / RBLK);
    if (ra.dim == 2)
        hipLaunchKernelGGL(k_rows_dynamic<2>, dim3(nb), dim3(RBLK), 0, s, ra, rv, p, rowptr, rstart, vals, sc, u_prev,
                           f, pin_dof);
    else
        hipLaunchKernelGGL(k_rows_dynamic<3>, dim3(nb), dim3(RBLK), 0, s, ra, rv, p, rowptr, rstart, vals, sc, u_prev,
                           f, pin_dof);
}

}  // namespace launch
}  // namespace knp
