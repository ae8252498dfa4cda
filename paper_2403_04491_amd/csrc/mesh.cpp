// Host-side mesh setup: region DOF maps with duplicated membrane vertices,
// membrane facets, the structural CSR pattern of A (block rows of eq.
// ``lin_sys``) and the incidence lists the gather-assembly kernels walk.
// Runs once per mesh (the paper's "initialization" phase).
#include <omp.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <numeric>

#include "knp_internal.h"

namespace knp {

namespace {

[[noreturn]] void fail(const std::string &m) { throw Error{KNP_E_ARG, m}; }

struct Face {
    std::array<int32_t, 3> v;   // ascending; unused slots = -1
    int32_t owner;              // cell tag of the owning element
    bool operator<(const Face &o) const { return v < o.v; }
    bool same(const Face &o) const { return v == o.v; }
};

Face make_face(const int32_t *ev, int d1, int drop, int32_t owner) {
    Face f;
    f.v = {-1, -1, -1};
    int c = 0;
    for (int a = 0; a < d1; ++a)
        if (a != drop) f.v[c++] = ev[a];
    std::sort(f.v.begin(), f.v.begin() + c);
    f.owner = owner;
    return f;
}

int find_pos(const int32_t *row, int n, int32_t key) {
    const int32_t *p = std::lower_bound(row, row + n, key);
    if (p == row + n || *p != key) return -1;
    return int(p - row);
}

}  // namespace

void build_host_mesh(HostMesh &m, int dim, int order, int64_t n_vert, const double *xyz, int64_t n_elem,
                     const int32_t *elem_in, const int32_t *tag, int64_t pin_vertex) {
    if (dim != 2 && dim != 3) fail("dim must be 2 or 3");
    if (order != 1 && order != 2) fail("element order must be 1 or 2");
    if (n_vert <= 0 || n_elem <= 0) fail("empty mesh");
    if (n_vert >= (int64_t(1) << 31) - 1) fail("too many vertices for int32 indices");
    if (!xyz || !elem_in || !tag) fail("NULL mesh array");
    const int d1 = dim + 1;
    m = HostMesh();
    m.dim = dim;
    m.order = order;
    m.n_vert_p1 = n_vert;
    m.n_elem = n_elem;
    m.tag.assign(tag, tag + n_elem);

    int32_t maxtag = 0;
    for (int64_t e = 0; e < n_elem; ++e) {
        if (tag[e] < 0) fail("negative element tag");
        maxtag = std::max(maxtag, tag[e]);
        for (int a = 0; a < d1; ++a) {
            int32_t v = elem_in[e * d1 + a];
            if (v < 0 || v >= n_vert) fail("element vertex out of range");
            for (int b = 0; b < a; ++b)
                if (elem_in[e * d1 + b] == v) fail("degenerate element (repeated vertex)");
        }
    }
    m.n_cells = maxtag;

    // ---- nodes: the vertices, and for order 2 one node per edge (lexicographic)
    const int npair = d1 * (d1 - 1) / 2;
    std::vector<int64_t> ekeys;      // a * n_vert + b of the sorted edges (order 2)
    if (order == 1) {
        m.nv_elem = d1;
        m.nv_facet = dim;
        m.n_vert = n_vert;
        m.xyz.assign(xyz, xyz + n_vert * dim);
        m.elem.assign(elem_in, elem_in + n_elem * d1);
    } else {
        m.nv_elem = d1 + npair;
        m.nv_facet = dim + dim * (dim - 1) / 2;
        ekeys.reserve(size_t(n_elem) * npair);
        for (int64_t e = 0; e < n_elem; ++e)
            for (int i = 0; i < d1; ++i)
                for (int j = i + 1; j < d1; ++j) {
                    const int64_t a = std::min(elem_in[e * d1 + i], elem_in[e * d1 + j]);
                    const int64_t b = std::max(elem_in[e * d1 + i], elem_in[e * d1 + j]);
                    ekeys.push_back(a * n_vert + b);
                }
        std::sort(ekeys.begin(), ekeys.end());
        ekeys.erase(std::unique(ekeys.begin(), ekeys.end()), ekeys.end());
        const int64_t ne = int64_t(ekeys.size());
        m.n_vert = n_vert + ne;
        if (m.n_vert >= (int64_t(1) << 31) - 1) fail("too many nodes for int32 indices");
        m.edges.resize(size_t(ne) * 2);
        m.xyz.resize(size_t(m.n_vert) * dim);
        std::copy(xyz, xyz + n_vert * dim, m.xyz.begin());
        for (int64_t k = 0; k < ne; ++k) {
            const int64_t a = ekeys[k] / n_vert, b = ekeys[k] % n_vert;
            m.edges[2 * k] = int32_t(a);
            m.edges[2 * k + 1] = int32_t(b);
            for (int c = 0; c < dim; ++c) m.xyz[(n_vert + k) * dim + c] = 0.5 * (xyz[a * dim + c] + xyz[b * dim + c]);
        }
        m.elem.resize(size_t(n_elem) * m.nv_elem);
#pragma omp parallel for schedule(static)
        for (int64_t e = 0; e < n_elem; ++e) {
            int32_t *o = &m.elem[e * m.nv_elem];
            int c = 0;
            for (int i = 0; i < d1; ++i) o[c++] = elem_in[e * d1 + i];
            for (int i = 0; i < d1; ++i)
                for (int j = i + 1; j < d1; ++j) {
                    const int64_t a = std::min(elem_in[e * d1 + i], elem_in[e * d1 + j]);
                    const int64_t b = std::max(elem_in[e * d1 + i], elem_in[e * d1 + j]);
                    o[c++] = int32_t(n_vert + (std::lower_bound(ekeys.begin(), ekeys.end(), a * n_vert + b) - ekeys.begin()));
                }
        }
    }
    m.walk = order == 1;
    const int nv = m.nv_elem, nf = m.nv_facet;
    const int32_t *elem = m.elem.data();
    const int64_t n_node = m.n_vert;

    // ---- region membership, cell of each ICS vertex
    std::vector<uint8_t> in_r[2] = {std::vector<uint8_t>(n_node, 0), std::vector<uint8_t>(n_node, 0)};
    m.vcell.assign(n_node, 0);
    std::vector<uint8_t> cell_seen(maxtag + 1, 0);
    for (int64_t e = 0; e < n_elem; ++e) {
        int r = tag[e] >= 1 ? 0 : 1;
        cell_seen[tag[e]] = 1;
        for (int a = 0; a < nv; ++a) {
            int32_t v = elem[e * nv + a];
            in_r[r][v] = 1;
            if (r == 0) {
                if (m.vcell[v] == 0)
                    m.vcell[v] = tag[e];
                else if (m.vcell[v] != tag[e])
                    fail("two cells share a vertex");
            }
        }
    }
    for (int c = 1; c <= maxtag; ++c)
        if (!cell_seen[c]) fail("cell tags must be 1..n_cells without gaps");
    for (int r = 0; r < 2; ++r) {
        m.loc[r].assign(n_node, -1);
        for (int64_t v = 0; v < n_node; ++v)
            if (in_r[r][v]) {
                m.loc[r][v] = int32_t(m.verts[r].size());
                m.verts[r].push_back(int32_t(v));
            }
        m.Nr[r] = int64_t(m.verts[r].size());
    }
    if (m.Nr[1] == 0) fail("mesh has no extracellular elements");
    m.off[0] = 0;
    m.off[1] = 4 * m.Nr[0];
    m.N = 4 * (m.Nr[0] + m.Nr[1]);
    if (m.N >= (int64_t(1) << 31) - 1) fail("too many unknowns for int32 column indices");

    m.gidx.assign(n_node, -1);
    for (int64_t v = 0; v < n_node; ++v)
        if (in_r[0][v] && in_r[1][v]) {
            m.gidx[v] = int32_t(m.gamma.size());
            m.gamma.push_back(int32_t(v));
        }
    if (pin_vertex < 0 || pin_vertex >= n_vert || !in_r[1][pin_vertex] || m.gidx[pin_vertex] >= 0)
        fail("pin vertex must be an extracellular vertex off the membrane");
    m.pin_vertex = pin_vertex;

    // ---- membrane facets: ICS boundary faces that are also faces of ECS elements
    std::vector<Face> fi, fe;
    for (int64_t e = 0; e < n_elem; ++e) {
        const int32_t *ev = &elem[e * nv];   // its d + 1 vertices come first
        if (tag[e] >= 1) {
            for (int a = 0; a < d1; ++a) fi.push_back(make_face(ev, d1, a, tag[e]));
        } else {
            for (int a = 0; a < d1; ++a) {
                bool all_g = true;
                for (int b = 0; b < d1; ++b)
                    if (b != a && m.gidx[ev[b]] < 0) all_g = false;
                if (all_g) fe.push_back(make_face(ev, d1, a, 0));
            }
        }
    }
    std::sort(fi.begin(), fi.end());
    std::sort(fe.begin(), fe.end());
    std::vector<Face> gf;
    for (size_t i = 0; i < fi.size();) {
        size_t j = i + 1;
        while (j < fi.size() && fi[j].same(fi[i])) ++j;
        if (j - i > 2) fail("non-conforming mesh (face shared by more than two elements)");
        if (j - i == 1) {
            auto it = std::lower_bound(fe.begin(), fe.end(), fi[i]);
            if (it == fe.end() || !it->same(fi[i]))
                fail("a cell touches the outer boundary or another cell");
            gf.push_back(fi[i]);
        }
        i = j;
    }
    m.n_facets = int64_t(gf.size());
    m.facets.resize(gf.size() * nf);
    for (size_t f = 0; f < gf.size(); ++f) {
        int32_t *o = &m.facets[f * nf];
        for (int a = 0; a < dim; ++a) o[a] = gf[f].v[a];
        if (order == 2) {
            int c = dim;
            for (int i = 0; i < dim; ++i)
                for (int j = i + 1; j < dim; ++j) {
                    const int64_t key = int64_t(gf[f].v[i]) * n_vert + gf[f].v[j];   // ascending pair
                    const auto it = std::lower_bound(ekeys.begin(), ekeys.end(), key);
                    if (it == ekeys.end() || *it != key) fail("internal: facet edge not among the element edges");
                    o[c++] = int32_t(n_vert + (it - ekeys.begin()));
                }
        }
    }
    fi.clear();
    fi.shrink_to_fit();
    fe.clear();
    fe.shrink_to_fit();

    // ---- element incidence per region vertex
    for (int r = 0; r < 2; ++r) {
        const int64_t Nr = m.Nr[r];
        std::vector<int64_t> &irow = m.irow[r];
        irow.assign(Nr + 1, 0);
        for (int64_t e = 0; e < n_elem; ++e) {
            if ((tag[e] >= 1) != (r == 0)) continue;
            for (int a = 0; a < nv; ++a) irow[m.loc[r][elem[e * nv + a]] + 1]++;
        }
        for (int64_t j = 0; j < Nr; ++j) irow[j + 1] += irow[j];
        m.ielem[r].assign(irow[Nr], 0);
        m.ipos[r].assign(irow[Nr], 0);
        std::vector<int64_t> fill(irow.begin(), irow.end() - 1);
        for (int64_t e = 0; e < n_elem; ++e) {
            if ((tag[e] >= 1) != (r == 0)) continue;
            for (int a = 0; a < nv; ++a) {
                int32_t j = m.loc[r][elem[e * nv + a]];
                m.ielem[r][fill[j]] = int32_t(e);
                m.ipos[r][fill[j]] = uint32_t(a);     // slot; order 1: positions added below
                fill[j]++;
            }
        }
        // scalar pattern rows: union of incident element vertices
        std::vector<int64_t> &prow = m.prow[r];
        prow.assign(Nr + 1, 0);
        int bad = 0;
#pragma omp parallel
        {
            std::vector<int32_t> buf;
#pragma omp for schedule(static)
            for (int64_t j = 0; j < Nr; ++j) {
                buf.clear();
                for (int64_t t = irow[j]; t < irow[j + 1]; ++t) {
                    const int32_t *ev = &elem[int64_t(m.ielem[r][t]) * nv];
                    for (int a = 0; a < nv; ++a) buf.push_back(m.loc[r][ev[a]]);
                }
                std::sort(buf.begin(), buf.end());
                int64_t cnt = std::unique(buf.begin(), buf.end()) - buf.begin();
                if (cnt > MAXN) {
#pragma omp atomic write
                    bad = 1;
                }
                prow[j + 1] = cnt;
            }
        }
        if (bad) m.walk = false;
        for (int64_t j = 0; j < Nr; ++j) prow[j + 1] += prow[j];
        m.pcol[r].assign(prow[Nr], 0);
#pragma omp parallel
        {
            std::vector<int32_t> buf;
#pragma omp for schedule(static)
            for (int64_t j = 0; j < Nr; ++j) {
                buf.clear();
                for (int64_t t = irow[j]; t < irow[j + 1]; ++t) {
                    const int32_t *ev = &elem[int64_t(m.ielem[r][t]) * nv];
                    for (int a = 0; a < nv; ++a) buf.push_back(m.loc[r][ev[a]]);
                }
                std::sort(buf.begin(), buf.end());
                int64_t cnt = std::unique(buf.begin(), buf.end()) - buf.begin();
                int32_t *row = &m.pcol[r][prow[j]];
                std::copy(buf.begin(), buf.begin() + cnt, row);
                if (!m.walk) continue;
                for (int64_t t = irow[j]; t < irow[j + 1]; ++t) {
                    const int32_t *ev = &elem[int64_t(m.ielem[r][t]) * d1];
                    uint32_t packed = m.ipos[r][t] & 3u;
                    for (int a = 0; a < d1; ++a) {
                        int p = find_pos(row, int(cnt), m.loc[r][ev[a]]);
                        packed |= uint32_t(p) << (2 + 5 * a);
                    }
                    m.ipos[r][t] = packed;
                }
            }
        }
    }

    // ---- membrane adjacency and facet incidence per membrane vertex
    const int64_t ng = int64_t(m.gamma.size());
    m.frow.assign(ng + 1, 0);
    for (int64_t f = 0; f < m.n_facets; ++f)
        for (int a = 0; a < nf; ++a) m.frow[m.gidx[m.facets[f * nf + a]] + 1]++;
    for (int64_t g = 0; g < ng; ++g) m.frow[g + 1] += m.frow[g];
    m.ffacet.assign(m.frow[ng], 0);
    {
        std::vector<int64_t> fill(m.frow.begin(), m.frow.end() - 1);
        for (int64_t f = 0; f < m.n_facets; ++f)
            for (int a = 0; a < nf; ++a) {
                int32_t g = m.gidx[m.facets[f * nf + a]];
                m.ffacet[fill[g]++] = int32_t(f);
            }
    }
    m.grow.assign(ng + 1, 0);
    std::vector<std::vector<int32_t>> gnb(ng);
    int gbad = 0;
    for (int64_t g = 0; g < ng; ++g) {
        std::vector<int32_t> &buf = gnb[g];
        for (int64_t t = m.frow[g]; t < m.frow[g + 1]; ++t)
            for (int a = 0; a < nf; ++a) buf.push_back(m.facets[int64_t(m.ffacet[t]) * nf + a]);
        std::sort(buf.begin(), buf.end());
        buf.erase(std::unique(buf.begin(), buf.end()), buf.end());
        if (int(buf.size()) > MAXG) gbad = 1;
        m.grow[g + 1] = m.grow[g] + int64_t(buf.size());
    }
    if (gbad) m.walk = false;
    m.gcol.resize(m.grow[ng]);
    for (int64_t g = 0; g < ng; ++g) std::copy(gnb[g].begin(), gnb[g].end(), m.gcol.begin() + m.grow[g]);
    for (int r = 0; r < 2; ++r) m.fpos[r].assign(m.frow[ng], 0);
    for (int64_t g = 0; g < ng && order == 1; ++g) {   // slots (order 1), positions (walk)
        const int32_t v = m.gamma[g];
        const int32_t *grow_p = &m.gcol[m.grow[g]];
        const int gn = int(m.grow[g + 1] - m.grow[g]);
        for (int64_t t = m.frow[g]; t < m.frow[g + 1]; ++t) {
            const int32_t *fv = &m.facets[int64_t(m.ffacet[t]) * dim];
            int slot = 0;
            for (int a = 0; a < dim; ++a)
                if (fv[a] == v) slot = a;
            for (int r = 0; r < 2; ++r) {
                const int32_t j = m.loc[r][v];
                const int32_t *row = &m.pcol[r][m.prow[r][j]];
                const int n = int(m.prow[r][j + 1] - m.prow[r][j]);
                uint32_t packed = uint32_t(slot);
                for (int a = 0; a < dim && m.walk; ++a) {
                    int p = find_pos(row, n, m.loc[r][fv[a]]);
                    int pg = find_pos(grow_p, gn, fv[a]);
                    if (p < 0 || pg < 0) fail("internal: membrane facet outside the region pattern");
                    packed |= uint32_t(p) << (2 + 5 * a);
                    packed |= uint32_t(pg) << (17 + 4 * a);
                }
                m.fpos[r][t] = packed;
            }
        }
    }

    // ---- global CSR pattern in the block order of eq. lin_sys
    const int64_t N = m.N;
    m.rowptr.assign(N + 1, 0);
    auto glen = [&](int32_t v) -> int64_t {
        int32_t g = m.gidx[v];
        return g >= 0 ? m.grow[g + 1] - m.grow[g] : 0;
    };
    for (int r = 0; r < 2; ++r)
        for (int64_t j = 0; j < m.Nr[r]; ++j) {
            int64_t n = m.prow[r][j + 1] - m.prow[r][j];
            int64_t g = glen(m.verts[r][j]);
            for (int k = 0; k < 3; ++k) m.rowptr[m.off[r] + k * m.Nr[r] + j + 1] = 2 * n + g;
            m.rowptr[m.off[r] + 3 * m.Nr[r] + j + 1] = 4 * n + g;
        }
    for (int64_t i = 0; i < N; ++i) m.rowptr[i + 1] += m.rowptr[i];
    m.nnz = m.rowptr[N];
    m.nnz_p0 = 4 * (m.prow[0][m.Nr[0]] + m.prow[1][m.Nr[1]]);
    m.colidx.assign(m.nnz, 0);
    m.diag_pos.assign(N, 0);
    for (int r = 0; r < 2; ++r) {
        const int q = 1 - r;
        const int64_t Nr = m.Nr[r], Nq = m.Nr[q];
        const int64_t offr = m.off[r], offq = m.off[q];
#pragma omp parallel for schedule(static)
        for (int64_t j = 0; j < Nr; ++j) {
            const int32_t v = m.verts[r][j];
            const int32_t *pc = &m.pcol[r][m.prow[r][j]];
            const int64_t n = m.prow[r][j + 1] - m.prow[r][j];
            const int32_t g = m.gidx[v];
            const int32_t *gc = g >= 0 ? &m.gcol[m.grow[g]] : nullptr;
            const int64_t gn = g >= 0 ? m.grow[g + 1] - m.grow[g] : 0;
            const int self = find_pos(pc, int(n), int32_t(j));
            auto put_q = [&](int32_t *&o) {   // phi_q columns of the membrane neighbours
                for (int64_t t = 0; t < gn; ++t) *o++ = int32_t(offq + 3 * Nq + m.loc[q][gc[t]]);
            };
            auto put_blk = [&](int32_t *&o, int fld) {
                for (int64_t t = 0; t < n; ++t) *o++ = int32_t(offr + fld * Nr + pc[t]);
            };
            for (int k = 0; k < 3; ++k) {
                const int64_t row = offr + k * Nr + j;
                int32_t *o = &m.colidx[m.rowptr[row]];
                if (r == 1) put_q(o);
                put_blk(o, k);
                put_blk(o, 3);
                if (r == 0) put_q(o);
                m.diag_pos[row] = m.rowptr[row] + (r == 1 ? gn : 0) + self;
            }
            const int64_t row = offr + 3 * Nr + j;
            int32_t *o = &m.colidx[m.rowptr[row]];
            if (r == 1) put_q(o);
            for (int k = 0; k < 4; ++k) put_blk(o, k);
            if (r == 0) put_q(o);
            m.diag_pos[row] = m.rowptr[row] + (r == 1 ? gn : 0) + 3 * n + self;
        }
    }
    m.pin_dof = m.off[1] + 3 * m.Nr[1] + m.loc[1][pin_vertex];
}

}  // namespace knp
