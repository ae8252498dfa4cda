// Static operators of the product-form assembly, built on the host once per mesh: the
// path of quadratic (P2) elements, and of linear ones on meshes whose vertex degree
// exceeds what the element-walk kernels hold.
//
// The element integrals of the blocks of eq. ``lin_sys`` (Sec. "Algebraic structure and
// matrix assembly") for Lagrange elements of degree 1 or 2 (Sec. "Spatial discretization"):
// on an element T with barycentric gradients grad lambda_i and G_ij = grad lambda_i .
// grad lambda_j,
//   int_T grad phi_a . grad phi_b         = |T| sum_ij G_ij S[a][b][i][j],
//   int_T phi_c grad phi_a . grad phi_b   = |T| sum_ij G_ij W[c][a][b][i][j],
//   int_T phi_a phi_b                     = |T| M[a][b],
// and on a membrane facet F,  int_F phi_a phi_b = |F| F2[a][b],
// int_F phi_a phi_b phi_c = |F| F3[a][b][c], with the reference tensors of p2_ref.h.  The
// nonlinear coefficients (the concentrations in the weighted stiffness, the membrane
// coefficients) are P2 fields given by their nodal values, so every per-step value is a
// sum of stored weights times nodal values.  Sums run in the element (facet) order of
// each row node's incidence list, the weights of one weight node merged in order of
// first appearance, so the operators are deterministic.
#include <omp.h>

#include <algorithm>
#include <cmath>

#include "host_geom.h"
#include "knp_internal.h"
#include "p2_ref.h"

namespace knp {

namespace {

using host::facet_measure;
using host::find_sorted;
using host::simplex_gradients;

// one entry's weight terms, merged by weight node in order of first appearance
struct Terms {
    std::vector<int32_t> node;
    std::vector<double> val;
    void add(int32_t m, double v) {
        for (size_t i = 0; i < node.size(); ++i)
            if (node[i] == m) {
                val[i] += v;
                return;
            }
        node.push_back(m);
        val.push_back(v);
    }
};

[[noreturn]] void fail_internal(const char *what) { throw Error{KNP_E_ARG, std::string("internal: ") + what}; }

}  // namespace

void build_p2_operators(const HostMesh &m, P2Host &out) {
    build_p2_bulk(m, out);
    build_p2_membrane(m, out);
}

void build_p2_bulk(const HostMesh &m, P2Host &out) {
    const int d = m.dim, n = d + 1, nv = m.nv_elem, nf = m.nv_facet;
    const p2::RefTensors T = p2::reference_tensors(d, m.order);
    if (T.nb != nv || T.nf != nf) fail_internal("element node counts");
    for (int r = 0; r < 2; ++r) {
        const int64_t Nr = m.Nr[r], nent = m.prow[r][Nr];
        out.sval[r].assign(nent, 0.0);
        out.mval[r].assign(nent, 0.0);
        out.erow[r].assign(std::max<int64_t>(1, nent), 0);
        std::vector<std::vector<Terms>> rows(Nr);
        int bad = 0;
#pragma omp parallel
        {
            std::vector<double> x(size_t(n) * d), g(size_t(n) * d), G(size_t(n) * n);
            std::vector<int> qpos(nv);
#pragma omp for schedule(dynamic, 256)
            for (int64_t j = 0; j < Nr; ++j) {
                const int64_t p0 = m.prow[r][j];
                const int cnt = int(m.prow[r][j + 1] - p0);
                const int32_t *pc = &m.pcol[r][p0];
                rows[j].assign(cnt, Terms());
                for (int q = 0; q < cnt; ++q) out.erow[r][p0 + q] = int32_t(j);
                for (int64_t t = m.irow[r][j]; t < m.irow[r][j + 1]; ++t) {
                    const int32_t *ev = &m.elem[int64_t(m.ielem[r][t]) * nv];
                    // slot of the row node in the element (order 1: the low two bits)
                    const int s = int(m.order == 1 ? (m.ipos[r][t] & 3u) : m.ipos[r][t]);
                    for (int a = 0; a < n; ++a)
                        for (int k = 0; k < d; ++k) x[a * d + k] = m.xyz[int64_t(ev[a]) * d + k];
                    const double vol = simplex_gradients(d, x.data(), g.data());
                    for (int i = 0; i < n; ++i)
                        for (int jj = 0; jj < n; ++jj) {
                            double dot = 0.0;
                            for (int k = 0; k < d; ++k) dot += g[i * d + k] * g[jj * d + k];
                            G[i * n + jj] = dot;
                        }
                    for (int b = 0; b < nv; ++b) {
                        qpos[b] = find_sorted(pc, cnt, m.loc[r][ev[b]]);
                        if (qpos[b] < 0) {
#pragma omp atomic write
                            bad = 1;
                            qpos[b] = 0;
                        }
                    }
                    for (int b = 0; b < nv; ++b) {
                        const int64_t p = p0 + qpos[b];
                        double sv = 0.0;
                        for (int i = 0; i < n; ++i)
                            for (int jj = 0; jj < n; ++jj) sv += G[i * n + jj] * T.S[((size_t(s) * nv + b) * n + i) * n + jj];
                        out.sval[r][p] += vol * sv;
                        out.mval[r][p] += vol * T.M[size_t(s) * nv + b];
                        for (int c = 0; c < nv; ++c) {
                            double wv = 0.0;
                            for (int i = 0; i < n; ++i)
                                for (int jj = 0; jj < n; ++jj)
                                    wv += G[i * n + jj] * T.W[(((size_t(c) * nv + s) * nv + b) * n + i) * n + jj];
                            rows[j][qpos[b]].add(m.loc[r][ev[c]], vol * wv);
                        }
                    }
                }
            }
        }
        if (bad) fail_internal("element node outside the scalar pattern");
        std::vector<int64_t> &wp = out.wptr[r];
        wp.assign(nent + 1, 0);
        for (int64_t j = 0; j < Nr; ++j)
            for (size_t q = 0; q < rows[j].size(); ++q) wp[m.prow[r][j] + q + 1] = int64_t(rows[j][q].node.size());
        for (int64_t p = 0; p < nent; ++p) wp[p + 1] += wp[p];
        out.wnode[r].assign(std::max<int64_t>(1, wp[nent]), 0);
        out.wval[r].assign(std::max<int64_t>(1, wp[nent]), 0.0);
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < Nr; ++j)
            for (size_t q = 0; q < rows[j].size(); ++q) {
                const int64_t o = wp[m.prow[r][j] + q];
                std::copy(rows[j][q].node.begin(), rows[j][q].node.end(), out.wnode[r].begin() + o);
                std::copy(rows[j][q].val.begin(), rows[j][q].val.end(), out.wval[r].begin() + o);
            }
    }
}

void build_p2_membrane(const HostMesh &m, P2Host &out) {
    const int d = m.dim, nf = m.nv_facet;
    const p2::RefTensors T = p2::reference_tensors(d, m.order);
    if (T.nf != nf) fail_internal("facet node counts");
    const int64_t ng = int64_t(m.gamma.size()), nmem = m.grow[ng];
    out.mg.assign(std::max<int64_t>(1, nmem), 0.0);
    out.mrow.assign(std::max<int64_t>(1, nmem), 0);
    for (int64_t gi = 0; gi < ng; ++gi)
        for (int64_t e = m.grow[gi]; e < m.grow[gi + 1]; ++e) out.mrow[e] = int32_t(gi);
    for (int r = 0; r < 2; ++r) out.rpos[r].assign(std::max<int64_t>(1, nmem), 0);
    std::vector<Terms> ent(nmem);
    int bad = 0;
#pragma omp parallel
    {
        std::vector<double> x(size_t(d) * d);
        std::vector<int> epos(nf);
#pragma omp for schedule(dynamic, 256)
        for (int64_t gi = 0; gi < ng; ++gi) {
            const int32_t v = m.gamma[gi];
            const int64_t e0 = m.grow[gi];
            const int gn = int(m.grow[gi + 1] - e0);
            const int32_t *gc = &m.gcol[e0];
            for (int r = 0; r < 2; ++r) {
                const int32_t j = m.loc[r][v];
                const int32_t *pc = &m.pcol[r][m.prow[r][j]];
                const int cnt = int(m.prow[r][j + 1] - m.prow[r][j]);
                for (int e = 0; e < gn; ++e) {
                    const int q = find_sorted(pc, cnt, m.loc[r][gc[e]]);
                    if (q < 0) {
#pragma omp atomic write
                        bad = 1;
                    }
                    out.rpos[r][e0 + e] = q;
                }
            }
            for (int64_t t = m.frow[gi]; t < m.frow[gi + 1]; ++t) {
                const int32_t *fv = &m.facets[int64_t(m.ffacet[t]) * nf];
                int s = 0;
                for (int a = 0; a < nf; ++a)
                    if (fv[a] == v) s = a;
                for (int a = 0; a < d; ++a)
                    for (int k = 0; k < d; ++k) x[a * d + k] = m.xyz[int64_t(fv[a]) * d + k];
                const double meas = facet_measure(d, x.data());
                for (int b = 0; b < nf; ++b) {
                    epos[b] = find_sorted(gc, gn, fv[b]);
                    if (epos[b] < 0) {
#pragma omp atomic write
                        bad = 1;
                        epos[b] = 0;
                    }
                }
                for (int b = 0; b < nf; ++b) {
                    out.mg[e0 + epos[b]] += meas * T.F2[size_t(s) * nf + b];
                    for (int c = 0; c < nf; ++c)
                        ent[e0 + epos[b]].add(m.gidx[fv[c]], meas * T.F3[(size_t(s) * nf + b) * nf + c]);
                }
            }
        }
    }
    if (bad) fail_internal("membrane node outside the patterns");
    out.cptr.assign(nmem + 1, 0);
    for (int64_t e = 0; e < nmem; ++e) out.cptr[e + 1] = out.cptr[e] + int64_t(ent[e].node.size());
    out.cnode.assign(std::max<int64_t>(1, out.cptr[nmem]), 0);
    out.cval.assign(std::max<int64_t>(1, out.cptr[nmem]), 0.0);
    for (int64_t e = 0; e < nmem; ++e) {
        std::copy(ent[e].node.begin(), ent[e].node.end(), out.cnode.begin() + out.cptr[e]);
        std::copy(ent[e].val.begin(), ent[e].val.end(), out.cval.begin() + out.cptr[e]);
    }
}

}  // namespace knp
