// Order-2 (P2) assembly of the IMEX-linearised KNP-EMI step (eq. ``lin_sys``): every value
// is a sparse product of the static operators built on the host (p2.cpp) with nodal
// data, one thread per entry of a region's scalar pattern or per membrane entry and
// region.  Sums run in the stored order; no atomics, so results are bitwise
// reproducible.  The row layout is that of the order-1 assembly: a c_r^k row holds its
// c_r^k block and its phi_r block (n entries each), a phi_r row the four field blocks,
// and either row the other region's phi at its membrane neighbours, first for the
// extracellular region and last for the intracellular one.
#include <hip/hip_runtime.h>

#include "knp_internal.h"

namespace knp {
namespace launch {

namespace {

inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }

// c_r^k rows, own block: M + tau_k A;  phi_r row, c_r^k blocks: z_k tau_k A.
__global__ void k_p2_static(RegionArgs ra, P2Bulk b, PhysArgs p, const int64_t *__restrict__ rowptr,
                            const int64_t *__restrict__ rstart, double *__restrict__ vals,
                            const double *__restrict__ sc, int64_t pin_dof) {
    const int64_t ent = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ent >= b.nent) return;
    const int64_t j = b.erow[ent];
    const int64_t p0 = ra.prow[j];
    const int n = int(ra.prow[j + 1] - p0);
    const int q = int(ent - p0);
    const int64_t lq = ra.pcol[ent];
    const int64_t Nr = ra.Nr;
    const double sv = b.sval[ent], mv = b.mval[ent];
    for (int k = 0; k < 3; ++k) {
        const int64_t row = ra.off + k * Nr + j;
        const int gq = int(rowptr[row + 1] - rowptr[row]) - 2 * n;
        const int64_t seg = rstart[row] + (ra.r == 0 ? 0 : gq);
        vals[seg + q] = (mv + p.tau[k] * sv) * sc[row] * sc[ra.off + k * Nr + lq];
    }
    const int64_t row = ra.off + 3 * Nr + j;
    const int gq = int(rowptr[row + 1] - rowptr[row]) - 4 * n;
    const int64_t seg0 = rstart[row] + (ra.r == 0 ? 0 : gq);
    const double sr = sc[row];
    const bool pinrow = row == pin_dof;
    for (int k = 0; k < 3; ++k)
        vals[seg0 + k * n + q] = pinrow ? 0.0 : p.z[k] * p.tau[k] * sv * sr * sc[ra.off + k * Nr + lq];
}

// c_r^k rows, phi_r block: tilde-tau_k A_r^k;  phi_r row, phi_r block: sum_k z_k tilde-tau_k
// A_r^k;  f_r^k = M_r c^{k,n-1}, f_r^phi = 0, with int c_h grad phi_j . grad phi_q =
// sum_t wval_t c(wnode_t) for the P2 field c_h of c^{k,n-1}.
__global__ void k_p2_dynamic(RegionArgs ra, P2Bulk b, PhysArgs p, const int64_t *__restrict__ rowptr,
                             const int64_t *__restrict__ rstart, double *__restrict__ vals,
                             const double *__restrict__ sc, const double *__restrict__ u, double *__restrict__ f,
                             int64_t pin_dof) {
    const int64_t ent = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (ent >= b.nent) return;
    const int64_t j = b.erow[ent];
    const int64_t p0 = ra.prow[j];
    const int n = int(ra.prow[j + 1] - p0);
    const int q = int(ent - p0);
    const int32_t lq = ra.pcol[ent];
    const int64_t Nr = ra.Nr;
    const double *cb = u + ra.off;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t t = b.wptr[ent]; t < b.wptr[ent + 1]; ++t) {
        const double w = b.wval[t];
        const int64_t m = b.wnode[t];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += w * cb[k * Nr + m];
    }
    const int64_t phib = ra.off + 3 * Nr;
    const int64_t col = phib + lq;
    const double scol = sc[col];
    const bool diag = lq == j;
    for (int k = 0; k < 3; ++k) {
        const int64_t row = ra.off + k * Nr + j;
        const int gq = int(rowptr[row + 1] - rowptr[row]) - 2 * n;
        const int64_t seg = rstart[row] + (ra.r == 0 ? 0 : gq) + n;
        vals[seg + q] = col == pin_dof ? 0.0 : p.ttau[k] * acc[k] * sc[row] * scol;
        if (diag) {
            double mc = 0.0;
            for (int qq = 0; qq < n; ++qq) mc += b.mval[p0 + qq] * cb[k * Nr + ra.pcol[p0 + qq]];
            f[row] = mc;
        }
    }
    const int64_t row = phib + j;
    const int gq = int(rowptr[row + 1] - rowptr[row]) - 4 * n;
    const int64_t seg = rstart[row] + (ra.r == 0 ? 0 : gq) + 3 * n;
    const bool pinrow = row == pin_dof;
    double v = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) v += p.z[k] * p.ttau[k] * acc[k];
    const bool keep = pinrow ? (col == row) : (col != pin_dof);
    vals[seg + q] = keep ? v * sc[row] * scol : 0.0;
    if (diag) f[row] = 0.0;
}

// Membrane part for the membrane node g of entry e and its neighbour a, region r (sgn_r
// in the coefficients): c_r^k row, phi_r block += int C_r^k phi_g phi_a and phi_q block
// = -int C_r^k phi_g phi_a; phi_r row, phi_r block += C_m/F int phi_g phi_a and phi_q
// block = -C_m/F int phi_g phi_a; the thread of g's first entry adds
// f_r^k -= int g_r^k phi_g and f_r^phi -= int h_r phi_g.
__global__ void k_p2_membrane(GammaArgs g, RegionArgs ra_i, RegionArgs ra_e, P2Mem mm, PhysArgs p,
                              const int64_t *__restrict__ rowptr, const int64_t *__restrict__ rstart,
                              double *__restrict__ vals, const double *__restrict__ sc,
                              const double *__restrict__ gc, double *__restrict__ f) {
    // threads [0, nmem) serve region i, [nmem, 2 nmem) region e: consecutive threads take
    // consecutive entries of one region, so a membrane row's values are written together
    const int64_t it = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (it >= 2 * mm.nmem) return;
    const int r = it < mm.nmem ? 0 : 1;
    const int64_t e = it - r * mm.nmem;
    const int64_t gi = mm.mrow[e];
    const int64_t e0 = mm.grow[gi];
    const int gn = int(mm.grow[gi + 1] - e0);
    const int idx = int(e - e0);
    const int32_t a = mm.gcol[e];
    const int64_t *prow = r == 0 ? ra_i.prow : ra_e.prow;
    const int32_t *loc_r = r == 0 ? g.gloc_i : g.gloc_e;   // by membrane index
    const int64_t Nr = r == 0 ? ra_i.Nr : ra_e.Nr, Nq = r == 0 ? ra_e.Nr : ra_i.Nr;
    const int64_t off = r == 0 ? ra_i.off : ra_e.off, offq = r == 0 ? ra_e.off : ra_i.off;
    const int64_t j = loc_r[gi];
    const int n = int(prow[j + 1] - prow[j]);
    const int qr = r == 0 ? mm.rpos_i[e] : mm.rpos_e[e];
    const int32_t ga = g.gidx[a];   // a is a membrane node too
    const int64_t la = r == 0 ? g.gloc_i[ga] : g.gloc_e[ga];
    const int64_t lqa = r == 0 ? g.gloc_e[ga] : g.gloc_i[ga];
    double val[3] = {0.0, 0.0, 0.0};
    for (int64_t t = mm.cptr[e]; t < mm.cptr[e + 1]; ++t) {
        const double w = mm.cval[t];
        const double *rec = gc + int64_t(mm.cnode[t]) * GC_STRIDE + r * GC_REGION;
#pragma unroll
        for (int k = 0; k < 3; ++k) val[k] += w * rec[GC_C + k];
    }
    const double S = p.C_m / p.F * mm.mg[e];
    const double scol_r = sc[off + 3 * Nr + la], scol_q = sc[offq + 3 * Nq + lqa];
    for (int k = 0; k < 4; ++k) {
        const int64_t row = off + k * Nr + j;
        const int64_t rp = rstart[row];
        const int nb = k < 3 ? 1 : 3;   // blocks preceding phi_r in this row
        const double sr = sc[row];
        const double v = k < 3 ? val[k] : S;
        vals[rp + (r == 0 ? 0 : gn) + int64_t(nb) * n + qr] += v * sr * scol_r;
        vals[(r == 0 ? rp + int64_t(nb + 1) * n : rp) + idx] = -v * sr * scol_q;
        if (idx == 0) {
            double fs = 0.0;
            for (int64_t e2 = e0; e2 < e0 + gn; ++e2) {
                const double *rec = gc + int64_t(g.gidx[mm.gcol[e2]]) * GC_STRIDE + r * GC_REGION;
                fs -= mm.mg[e2] * (k < 3 ? rec[GC_G + k] : rec[GC_H]);
            }
            f[row] += fs;
        }
    }
    (void)rowptr;
}

}  // namespace

void p2_static(const RegionArgs &ra, const P2Bulk &b, const PhysArgs &p, const int64_t *rowptr, const int64_t *rstart,
               double *vals, const double *sc, int64_t pin_dof, hipStream_t s) {
    if (b.nent == 0) return;
    hipLaunchKernelGGL(k_p2_static, dim3(nblocks(b.nent, 256)), dim3(256), 0, s, ra, b, p, rowptr, rstart, vals, sc,
                       pin_dof);
}

void p2_dynamic(const RegionArgs &ra, const P2Bulk &b, const PhysArgs &p, const int64_t *rowptr,
                const int64_t *rstart, double *vals, const double *sc, const double *u_prev, double *f,
                int64_t pin_dof, hipStream_t s) {
    if (b.nent == 0) return;
    hipLaunchKernelGGL(k_p2_dynamic, dim3(nblocks(b.nent, 256)), dim3(256), 0, s, ra, b, p, rowptr, rstart, vals, sc,
                       u_prev, f, pin_dof);
}

void p2_membrane(const GammaArgs &g, const RegionArgs &ra_i, const RegionArgs &ra_e, const P2Mem &mm, const PhysArgs &p,
                 const int64_t *rowptr, const int64_t *rstart, double *vals, const double *sc, const double *gcoef,
                 double *f, hipStream_t s) {
    if (mm.nmem == 0) return;
    hipLaunchKernelGGL(k_p2_membrane, dim3(nblocks(2 * mm.nmem, 256)), dim3(256), 0, s, g, ra_i, ra_e, mm, p, rowptr,
                       rstart, vals, sc, gcoef, f);
}

}  // namespace launch
}  // namespace knp
