// Row terms of the order-1 per-step bulk values (Sec. "Algebraic structure and matrix
// assembly": the blocks A_r^k of eq. ``lin_sys`` weighted by c^{k,n-1}), built on the
// host once per mesh.  For each row vertex i the element integrals are accumulated
// into a dense n x n table W[q][s] (entry q of row i, weight vertex at position s),
// walking i's elements in the order of its incidence list, so the terms are
// deterministic.  The ring identity behind the terms is stated with RowTerms.
#include <omp.h>

#include <cfloat>
#include <cmath>

#include "host_geom.h"
#include "knp_internal.h"

namespace knp {

namespace {

// W (ring weights, n x n, row-major) and M (mass row) of region vertex j
void row_tables(const HostMesh &m, int r, int64_t j, std::vector<double> &W, std::vector<double> &M) {
    const int d = m.dim, nv = d + 1;
    const int64_t p0 = m.prow[r][j];
    const int n = int(m.prow[r][j + 1] - p0);
    const int32_t *pc = &m.pcol[r][p0];
    W.assign(size_t(n) * n, 0.0);
    M.assign(n, 0.0);
    double x[4 * 3], g[4 * 3];
    int qa[4];
    const double mass_off = 1.0 / double((d + 1) * (d + 2));
    for (int64_t t = m.irow[r][j]; t < m.irow[r][j + 1]; ++t) {
        const int32_t *ev = &m.elem[int64_t(m.ielem[r][t]) * nv];
        const int s = int(m.ipos[r][t] & 3u);
        for (int a = 0; a < nv; ++a) {
            for (int k = 0; k < d; ++k) x[a * d + k] = m.xyz[int64_t(ev[a]) * d + k];
            qa[a] = host::find_sorted(pc, n, m.loc[r][ev[a]]);
            if (qa[a] < 0) throw Error{KNP_E_ARG, "internal: element vertex outside the scalar pattern"};
        }
        const double vol = host::simplex_gradients(d, x, g);
        for (int b = 0; b < nv; ++b) {
            M[qa[b]] += vol * (b == s ? 2.0 : 1.0) * mass_off;
            if (b == s) continue;
            double dot = 0.0;
            for (int k = 0; k < d; ++k) dot += g[s * d + k] * g[b * d + k];
            const double w = vol * dot / double(d + 1);
            for (int c = 0; c < nv; ++c)
                if (c != s && c != b) W[size_t(qa[b]) * n + qa[c]] += w;
        }
    }
}

// the terms kept of a row's table: |w| above 32 eps of the row's largest
double row_tolerance(const std::vector<double> &W) {
    double wmax = 0.0;
    for (double w : W) wmax = std::max(wmax, std::fabs(w));
    return 32.0 * DBL_EPSILON * wmax;
}

// consecutive rows with at most ROW_GROUP entries; ptr: row pointers, cnt: term counts
void make_groups(const int64_t *ptr, int64_t nrows, const std::vector<uint8_t> &cnt, std::vector<RowGroup> &out) {
    out.clear();
    int64_t j = 0, term = 0;
    while (j < nrows) {
        RowGroup g;
        g.row0 = int32_t(j);
        g.term0 = term;
        g.starts = 0;
        g.tmax = 0;
        g.nmax = 0;
        const int64_t e0 = ptr[j];
        while (j < nrows && ptr[j + 1] - e0 <= ROW_GROUP) {
            g.starts |= uint64_t(1) << (ptr[j] - e0);
            g.nmax = int16_t(std::max<int64_t>(g.nmax, ptr[j + 1] - ptr[j]));
            for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) {
                g.tmax = int16_t(std::max<int>(g.tmax, cnt[e]));
                term += cnt[e];
            }
            ++j;
        }
        out.push_back(g);
    }
    RowGroup end;
    end.row0 = int32_t(nrows);
    end.term0 = term;
    end.starts = 0;
    end.tmax = 0;
    end.nmax = 0;
    out.push_back(end);
}

}  // namespace

bool build_row_terms(const HostMesh &m, RowTerms out[2]) {
    if (m.order != 1) return false;
    for (int r = 0; r < 2; ++r)
        for (int64_t j = 0; j < m.Nr[r]; ++j)
            if (m.prow[r][j + 1] - m.prow[r][j] > ROW_GROUP) return false;
    for (int r = 0; r < 2; ++r) {
        RowTerms &o = out[r];
        const int64_t Nr = m.Nr[r], nent = m.prow[r][Nr];
        o.tcount.assign(std::max<int64_t>(1, nent), 0);
        o.mval.assign(std::max<int64_t>(1, nent), 0.0);
        std::vector<int64_t> rterm(Nr + 1, 0);   // terms of each row, then their offsets
        int err = 0;
#pragma omp parallel
        {
            std::vector<double> W, M;
#pragma omp for schedule(dynamic, 1024)
            for (int64_t j = 0; j < Nr; ++j) {
                try {
                    row_tables(m, r, j, W, M);
                } catch (const Error &) {
#pragma omp atomic write
                    err = 1;
                    continue;
                }
                const int64_t p0 = m.prow[r][j];
                const int n = int(m.prow[r][j + 1] - p0);
                const double tol = row_tolerance(W);
                int64_t tot = 0;
                for (int q = 0; q < n; ++q) {
                    int cnt = 0;
                    if (m.pcol[r][p0 + q] != j)
                        for (int s = 0; s < n; ++s) cnt += std::fabs(W[size_t(q) * n + s]) > tol;
                    o.tcount[p0 + q] = uint8_t(cnt);
                    o.mval[p0 + q] = M[q];
                    tot += cnt;
                }
                rterm[j + 1] = tot;
            }
        }
        if (err) throw Error{KNP_E_ARG, "internal: element vertex outside the scalar pattern"};
        for (int64_t j = 0; j < Nr; ++j) rterm[j + 1] += rterm[j];
        o.tslot.assign(std::max<int64_t>(1, rterm[Nr]), 0);
        o.tval.assign(std::max<int64_t>(1, rterm[Nr]), 0.0);
#pragma omp parallel
        {
            std::vector<double> W, M;
#pragma omp for schedule(dynamic, 1024)
            for (int64_t j = 0; j < Nr; ++j) {
                row_tables(m, r, j, W, M);
                const int64_t p0 = m.prow[r][j];
                const int n = int(m.prow[r][j + 1] - p0);
                const double tol = row_tolerance(W);
                int64_t t = rterm[j];
                for (int q = 0; q < n; ++q) {
                    if (m.pcol[r][p0 + q] == j) continue;
                    for (int s = 0; s < n; ++s) {
                        const double w = W[size_t(q) * n + s];
                        if (!(std::fabs(w) > tol)) continue;
                        o.tslot[t] = uint8_t(s);
                        o.tval[t] = w;
                        ++t;
                    }
                }
            }
        }
        make_groups(m.prow[r].data(), Nr, o.tcount, o.groups);
    }
    return true;
}

}  // namespace knp
