// The C entry points of libknp (declared in include/knp.h).  Each call checks
// its arguments, converts every internal failure into a status code plus a
// message, and never lets a C++ exception cross the ABI.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>

#include "ctx.h"

namespace knp {

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) throw Error{KNP_E_HIP, std::string(what) + ": " + hipGetErrorString(e)};
}

template <typename T>
void DArray<T>::alloc(size_t count) {
    release();
    if (count == 0) count = 1;
    void *ptr = nullptr;
    hipError_t e = hipMalloc(&ptr, count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{KNP_E_NOMEM, "hipMalloc of " + std::to_string(count * sizeof(T)) + " bytes failed"};
    }
    p = static_cast<T *>(ptr);
    n = count;
}

template <typename T>
void DArray<T>::upload(const T *h, size_t count, hipStream_t s) {
    if (count == 0) return;
    if (count > n) throw Error{KNP_E_ARG, "internal: upload larger than buffer"};
    hip_check(hipMemcpyAsync(p, h, count * sizeof(T), hipMemcpyHostToDevice, s), "upload");
    hip_check(hipStreamSynchronize(s), "upload sync");
}

template <typename T>
void DArray<T>::download(T *h, size_t count, hipStream_t s) const {
    if (count == 0) return;
    hip_check(hipMemcpyAsync(h, p, count * sizeof(T), hipMemcpyDeviceToHost, s), "download");
    hip_check(hipStreamSynchronize(s), "download sync");
}

hipEvent_t Timers::begin(int k, hipStream_t s) {
    (void)k;
    if (!on) return nullptr;
    hipEvent_t e;
    if (!pool.empty()) {
        e = pool.back();
        pool.pop_back();
    } else {
        hip_check(hipEventCreate(&e), "event create");
    }
    hip_check(hipEventRecord(e, s), "event record");
    return e;
}

void Timers::end(int k, hipEvent_t start, double bytes, hipStream_t s) {
    if (!on || !start) return;
    hipEvent_t e = begin(k, s);
    cls[k].a.push_back(start);
    cls[k].b.push_back(e);
    cls[k].bytes.push_back(bytes);
}

void Timers::harvest() {
    for (auto &c : cls) {
        for (size_t i = 0; i < c.a.size(); ++i) {
            float ms = 0.0f;
            hip_check(hipEventElapsedTime(&ms, c.a[i], c.b[i]), "event elapsed");
            c.ms += ms;
            c.launches += 1;
            c.total_bytes += c.bytes[i];
            pool.push_back(c.a[i]);
            pool.push_back(c.b[i]);
        }
        c.a.clear();
        c.b.clear();
        c.bytes.clear();
    }
}

void Timers::reset() {
    for (auto &c : cls) {
        for (auto e : c.a) pool.push_back(e);
        for (auto e : c.b) pool.push_back(e);
        c = Cls();
    }
}

Timers::~Timers() {
    reset();
    for (auto e : pool) (void)hipEventDestroy(e);
}

template struct DArray<double>;
template struct DArray<float>;
template struct DArray<int32_t>;
template struct DArray<int64_t>;
template struct DArray<uint32_t>;
template struct DArray<uint8_t>;
template struct DArray<uint16_t>;
template struct DArray<RowGroup>;

}  // namespace knp

using namespace knp;

knp::launch::RegionArgs knp_ctx::region(int r) const {
    knp::launch::RegionArgs a{};
    a.r = r;
    a.dim = hm.dim;
    a.Nr = hm.Nr[r];
    a.off = hm.off[r];
    a.off_q = hm.off[1 - r];
    a.Nq = hm.Nr[1 - r];
    a.prow = d_prow[r].p;
    a.pcol = d_pcol[r].p;
    a.irow = d_irow[r].p;
    a.ielem = d_ielem[r].p;
    a.ipos = d_ipos[r].p;
    a.verts = d_verts[r].p;
    return a;
}

knp::launch::MeshArgs knp_ctx::mesh_args() const {
    knp::launch::MeshArgs a{};
    a.dim = hm.dim;
    a.xyz = d_xyz.p;
    a.elem = d_elem.p;
    a.loc_i = d_loc[0].p;
    a.loc_e = d_loc[1].p;
    return a;
}

knp::launch::GammaArgs knp_ctx::gamma_args() const {
    knp::launch::GammaArgs g{};
    g.n_gamma = int64_t(hm.gamma.size());
    g.gamma = d_gamma.p;
    g.gloc_i = d_gloc_i.p;
    g.gloc_e = d_gloc_e.p;
    g.gcell = d_gcell.p;
    g.frow = d_frow.p;
    g.ffacet = d_ffacet.p;
    g.fpos_i = d_fpos[0].p;
    g.fpos_e = d_fpos[1].p;
    g.facets = d_facets.p;
    g.gidx = d_gidx.p;
    g.cell_model = d_cell_model.p;
    g.cell_stim = d_cell_stim.p;
    return g;
}

knp::launch::PhysArgs knp_ctx::phys(double t, double dt) const {
    knp::launch::PhysArgs p{};
    const double psi = prm.R * prm.T / prm.F;
    for (int k = 0; k < 3; ++k) {
        p.z[k] = prm.z[k];
        p.D[k] = prm.D[k];
        p.tau[k] = dt * prm.D[k];
        p.ttau[k] = p.tau[k] * prm.z[k] / psi;
        p.g_leak[k] = prm.g_leak[k];
    }
    p.F = prm.F;
    p.C_m = prm.C_m;
    p.psi = psi;
    p.dt = dt;
    p.t = t;
    p.gbar_Na = prm.gbar_Na;
    p.gbar_K = prm.gbar_K;
    p.g_stim_bar = prm.g_stim_bar;
    p.stim_a = prm.stim_a;
    p.stim_tau = prm.stim_tau;
    p.phi_rest = prm.phi_rest;
    p.rho_pump = prm.rho_pump;
    p.P_Na = prm.P_Na;
    p.P_K = prm.P_K;
    p.K_e0 = prm.K_e0;
    p.E_K0 = any_kir ? psi / prm.z[1] * std::log(prm.K_e0 / prm.K_i0) : 0.0;
    p.n_ode = prm.n_ode;
    return p;
}

namespace {

knp_status fail(knp_ctx *c, knp_status st, const std::string &msg) {
    if (c) c->err = msg;
    return st;
}

template <typename F>
knp_status guarded(knp_ctx *c, F &&fn) {
    if (!c) return KNP_E_ARG;
    try {
        c->err.clear();
        return fn();
    } catch (const Error &e) {
        return fail(c, e.st, e.msg);
    } catch (const std::bad_alloc &) {
        return fail(c, KNP_E_NOMEM, "host allocation failed");
    } catch (const std::exception &e) {
        return fail(c, KNP_E_ARG, e.what());
    } catch (...) {
        return fail(c, KNP_E_ARG, "unknown error");
    }
}

void need_device(knp_ctx *c) {
    if (c->host_only) throw Error{KNP_E_STATE, "host-only context (created with device -1)"};
}

// The system matrix by vertex (VtxView): each vertex's neighbour list is the set of
// vertices its phi row touches, and every entry of its four rows is checked against
// the column the vertex view implies for that position.  If any row differs (or a
// vertex's rows exceed a block, or the pairs overflow int32) the view stays off and
// A x keeps the CSR stream.
void build_vertex_view(knp_ctx *c, const std::vector<int32_t> &cols) {
    c->vtx = false;
    const int64_t N = c->hm.N, nv = N / 4, nvi = c->hm.Nr[0];
    if (nv == 0 || 4 * nv != N) return;
    const std::vector<int64_t> &rp = c->rowptr_s;
    std::vector<int64_t> cnt(nv + 1, 0);
    std::vector<char> bad(nv, 0);
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        if (rp[4 * v + 4] - rp[4 * v] > VTX_CAP) {
            bad[v] = 1;
            continue;
        }
        std::vector<int32_t> w;
        for (int64_t k = rp[4 * v + 3]; k < rp[4 * v + 4]; ++k) w.push_back(cols[k] >> 2);
        std::sort(w.begin(), w.end());
        cnt[v + 1] = std::unique(w.begin(), w.end()) - w.begin();
    }
    for (int64_t v = 0; v < nv; ++v) cnt[v + 1] += cnt[v];
    if (cnt[nv] >= (int64_t(1) << 31)) return;
    std::vector<int32_t> nbr(std::max<int64_t>(1, cnt[nv]));
#pragma omp parallel for schedule(static)
    for (int64_t v = 0; v < nv; ++v) {
        if (bad[v]) continue;
        const int64_t pb = cnt[v], npv = cnt[v + 1] - cnt[v];
        std::vector<int32_t> w;
        for (int64_t k = rp[4 * v + 3]; k < rp[4 * v + 4]; ++k) w.push_back(cols[k] >> 2);
        std::sort(w.begin(), w.end());
        w.erase(std::unique(w.begin(), w.end()), w.end());
        const bool ext = v >= nvi;
        int64_t m = 0;
        for (int32_t u : w) m += (u >= nvi) == ext;
        const int64_t p = npv - m;
        const int64_t sb = ext ? p : 0, cb = ext ? 0 : m;
        // same-region neighbours and partners each form one contiguous run
        for (int64_t q = 0; q < npv; ++q) {
            nbr[pb + q] = w[q];
            if (((w[q] >= nvi) == ext) != (q >= sb && q < sb + m)) bad[v] = 1;
        }
        if (10 * m + 4 * p != rp[4 * v + 4] - rp[4 * v]) bad[v] = 1;
        for (int f = 0; f < 4 && !bad[v]; ++f) {
            const int64_t a = rp[4 * v + f], len = rp[4 * v + f + 1] - a;
            if (len != (f < 3 ? 2 * m + p : 4 * m + p)) {
                bad[v] = 1;
                break;
            }
            int64_t e = 0;
            auto seg = [&](int64_t base, int64_t n, int g) {
                for (int64_t i = 0; i < n; ++i, ++e)
                    if (cols[a + e] != 4 * w[base + i] + g) bad[v] = 1;
            };
            if (ext) seg(cb, p, 3);
            if (f < 3) {
                seg(sb, m, f);
                seg(sb, m, 3);
            } else {
                for (int g = 0; g < 4; ++g) seg(sb, m, g);
            }
            if (!ext) seg(cb, p, 3);
        }
    }
    for (int64_t v = 0; v < nv; ++v)
        if (bad[v]) return;
    std::vector<int64_t> vptr(nv + 1);
    for (int64_t v = 0; v <= nv; ++v) vptr[v] = rp[4 * v];
    std::vector<int32_t> nptr(nv + 1);
    for (int64_t v = 0; v <= nv; ++v) nptr[v] = int32_t(cnt[v]);
    std::vector<int32_t> blk{0};
    for (int64_t v = 0; v < nv;) {
        int64_t e = v;
        while (e < nv && vptr[e + 1] - vptr[v] <= VTX_CAP && e - v < VTX_VMAX) ++e;
        blk.push_back(int32_t(e));   // e > v: every vertex fits a block (checked above)
        v = e;
    }
    hipStream_t s = c->stream;
    c->d_vptr.alloc(vptr.size());
    c->d_vptr.upload(vptr, s);
    c->d_nptr.alloc(nptr.size());
    c->d_nptr.upload(nptr, s);
    c->d_nbr.alloc(nbr.size());
    c->d_nbr.upload(nbr, s);
    c->d_vblk.alloc(blk.size());
    c->d_vblk.upload(blk, s);
    std::vector<int64_t> kblk(blk.size());
    std::vector<int32_t> pblk(blk.size());
    for (size_t b = 0; b < blk.size(); ++b) {
        kblk[b] = vptr[blk[b]];
        pblk[b] = nptr[blk[b]];
    }
    c->d_kblk.alloc(kblk.size());
    c->d_kblk.upload(kblk, s);
    c->d_pblk.alloc(pblk.size());
    c->d_pblk.upload(pblk, s);
    c->npairs = cnt[nv];
    c->nvblk = int64_t(blk.size()) - 1;
    c->vtx = true;
}

}  // namespace

extern "C" {

// Text of the last failed knp_create on this thread (no context exists to hold it).
// the membrane operators of the product form (p2.cpp) and the membrane adjacency, on the
// device; returns their algorithmic bytes per assembly (terms, per-entry records, values)
static double upload_p2_membrane(knp_ctx *c, const P2Host &o) {
    const HostMesh &h = c->hm;
    hipStream_t s = c->stream;
    for (int r = 0; r < 2; ++r) {
        c->d_p2_rpos[r].alloc(o.rpos[r].size());
        c->d_p2_rpos[r].upload(o.rpos[r], s);
    }
    c->p2_nmem = h.grow.empty() ? 0 : h.grow.back();
    c->d_grow.alloc(h.grow.size());
    c->d_grow.upload(h.grow, s);
    c->d_gcol.alloc(std::max<size_t>(1, h.gcol.size()));
    if (!h.gcol.empty()) c->d_gcol.upload(h.gcol, s);
    c->d_p2_mrow.alloc(o.mrow.size());
    c->d_p2_mrow.upload(o.mrow, s);
    c->d_p2_mg.alloc(o.mg.size());
    c->d_p2_mg.upload(o.mg, s);
    c->d_p2_cptr.alloc(o.cptr.size());
    c->d_p2_cptr.upload(o.cptr, s);
    c->d_p2_cnode.alloc(o.cnode.size());
    c->d_p2_cnode.upload(o.cnode, s);
    c->d_p2_cval.alloc(o.cval.size());
    c->d_p2_cval.upload(o.cval, s);
    return 12.0 * double(o.cnode.size()) + 2.0 * (8.0 * 8.0 + 8.0 * 3.0) * double(c->p2_nmem);
}

// the product-form path (order 2, or order 1 beyond the element-walk kernels' limits):
// the static operators (p2.cpp) and the membrane adjacency, on the device
static void upload_p2(knp_ctx *c) {
    const HostMesh &h = c->hm;
    hipStream_t s = c->stream;
    P2Host o;
    build_p2_operators(h, o);
    for (int r = 0; r < 2; ++r) {
        c->p2_nent[r] = h.prow[r][h.Nr[r]];
        c->d_p2_wptr[r].alloc(o.wptr[r].size());
        c->d_p2_wptr[r].upload(o.wptr[r], s);
        c->d_p2_wnode[r].alloc(o.wnode[r].size());
        c->d_p2_wnode[r].upload(o.wnode[r], s);
        c->d_p2_wval[r].alloc(o.wval[r].size());
        c->d_p2_wval[r].upload(o.wval[r], s);
        c->d_p2_erow[r].alloc(o.erow[r].size());
        c->d_p2_erow[r].upload(o.erow[r], s);
        c->d_p2_sval[r].alloc(std::max<size_t>(1, o.sval[r].size()));
        if (!o.sval[r].empty()) c->d_p2_sval[r].upload(o.sval[r], s);
        c->d_p2_mval[r].alloc(std::max<size_t>(1, o.mval[r].size()));
        if (!o.mval[r].empty()) c->d_p2_mval[r].upload(o.mval[r], s);
    }
    const double bm = upload_p2_membrane(c, o);
    hip_check(hipStreamSynchronize(s), "P2 operator upload");
    // algorithmic bytes of one product-form assembly: the products' terms and row starts,
    // entry rows and columns, M, the values and f written, u read; membrane terms
    double b = 16.0 * double(h.N) + bm;
    for (int r = 0; r < 2; ++r)
        b += 12.0 * double(o.wnode[r].size()) + 56.0 * double(c->p2_nent[r]);
    c->assembly_bytes = b;
}

// order 1 within the walk limits: the row terms of the per-step bulk values (rows.cpp)
static void upload_rows(knp_ctx *c) {
    const HostMesh &h = c->hm;
    hipStream_t s = c->stream;
    RowTerms rt[2];
    if (!build_row_terms(h, rt)) throw Error{KNP_E_ARG, "internal: row longer than a row group"};
    // algorithmic bytes of one per-step bulk assembly, each array touched once: u_prev,
    // f and S; per region the groups, row pointers, and per row vertex the four rows'
    // lengths and storage starts; per entry its column, term count, mass weight and the
    // four values written; the terms (weight and position)
    double b = 24.0 * double(h.N);
    for (int r = 0; r < 2; ++r) {
        const RowTerms &o = rt[r];
        const int64_t nent = h.prow[r][h.Nr[r]];
        c->rows_ngroups[r] = int64_t(o.groups.size()) - 1;
        c->d_rgroups[r].alloc(o.groups.size());
        c->d_rgroups[r].upload(o.groups, s);
        c->d_rcount[r].alloc(o.tcount.size());
        c->d_rcount[r].upload(o.tcount, s);
        c->d_rslot[r].alloc(o.tslot.size());
        c->d_rslot[r].upload(o.tslot, s);
        c->d_rval[r].alloc(o.tval.size());
        c->d_rval[r].upload(o.tval, s);
        c->d_rmval[r].alloc(o.mval.size());
        c->d_rmval[r].upload(o.mval, s);
        b += 24.0 * double(o.groups.size()) + 8.0 * double(h.Nr[r] + 1) + 4.0 * 24.0 * double(h.Nr[r]);
        b += (4.0 + 1.0 + 8.0 + 4.0 * 8.0) * double(nent) + 9.0 * double(o.groups.back().term0);
    }
    // the membrane blocks: the product form's membrane operators
    P2Host o;
    build_p2_membrane(h, o);
    b += upload_p2_membrane(c, o);
    hip_check(hipStreamSynchronize(s), "row term upload");
    c->rows = true;
    c->assembly_bytes = b;
}

static thread_local std::string g_create_err = "no error";

static knp_status create_failed(knp_ctx *c, knp_status st, std::string msg) {
    delete c;
    g_create_err = std::move(msg);
    return st;
}

knp_status knp_create(knp_ctx **out, int hip_device, void *hip_stream) {
    if (!out) return KNP_E_ARG;
    *out = nullptr;
    knp_ctx *c = new (std::nothrow) knp_ctx();
    if (!c) return create_failed(nullptr, KNP_E_NOMEM, "out of host memory");
    c->device = hip_device;
    c->host_only = hip_device < 0;
    c->stream = static_cast<hipStream_t>(hip_stream);
    if (!c->host_only) {
        int n = 0;
        const hipError_t e = hipGetDeviceCount(&n);
        if (e != hipSuccess)
            return create_failed(c, KNP_E_HIP, std::string("hipGetDeviceCount: ") + hipGetErrorString(e));
        if (hip_device >= n)
            return create_failed(c, KNP_E_HIP, "device " + std::to_string(hip_device) + " of " +
                                                   std::to_string(n) + " visible");
        const hipError_t e2 = hipSetDevice(hip_device);
        if (e2 != hipSuccess)
            return create_failed(c, KNP_E_HIP, std::string("hipSetDevice: ") + hipGetErrorString(e2));
        try {
            c->d_flag.alloc(1);
        } catch (...) {
            return create_failed(c, KNP_E_NOMEM, "device allocation failed");
        }
        try {
            c->scratch = knp::launch::noalloc_scratch(hip_device);
        } catch (const Error &e) {
            return create_failed(c, e.st, e.msg);
        }
    }
    *out = c;
    return KNP_OK;
}

void knp_destroy(knp_ctx *c) {
    if (!c) return;
    if (!c->host_only) {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
    }
    delete c;
}

const char *knp_last_error(const knp_ctx *c) { return c ? c->err.c_str() : g_create_err.c_str(); }

static knp_status mesh_upload(knp_ctx *c, int order, int dim, int64_t n_vert, const double *xyz, int64_t n_elem,
                              const int32_t *elem_vert, const int32_t *elem_tag, int64_t pin_vertex,
                              knp_mesh_info *out) {
    return guarded(c, [&]() -> knp_status {
        if (c->have_mesh) return fail(c, KNP_E_STATE, "mesh already uploaded");
        HostMesh m;
        build_host_mesh(m, dim, order, n_vert, xyz, n_elem, elem_vert, elem_tag, pin_vertex);
        c->hm = std::move(m);
        HostMesh &h = c->hm;
        if (!c->host_only) {
            hip_check(hipSetDevice(c->device), "set device");
            hipStream_t s = c->stream;
            c->d_xyz.alloc(h.xyz.size());
            c->d_xyz.upload(h.xyz, s);
            c->d_elem.alloc(h.elem.size());
            c->d_elem.upload(h.elem, s);
            for (int r = 0; r < 2; ++r) {
                c->d_loc[r].alloc(h.loc[r].size());
                c->d_loc[r].upload(h.loc[r], s);
                c->d_verts[r].alloc(h.verts[r].size());
                c->d_verts[r].upload(h.verts[r], s);
                c->d_prow[r].alloc(h.prow[r].size());
                c->d_prow[r].upload(h.prow[r], s);
                c->d_pcol[r].alloc(h.pcol[r].size());
                c->d_pcol[r].upload(h.pcol[r], s);
                c->d_irow[r].alloc(h.irow[r].size());
                c->d_irow[r].upload(h.irow[r], s);
                c->d_ielem[r].alloc(h.ielem[r].size());
                c->d_ielem[r].upload(h.ielem[r], s);
                c->d_ipos[r].alloc(h.ipos[r].size());
                c->d_ipos[r].upload(h.ipos[r], s);
                c->d_fpos[r].alloc(h.fpos[r].size());
                c->d_fpos[r].upload(h.fpos[r], s);
            }
            const size_t ng = h.gamma.size();
            std::vector<int32_t> gli(ng), gle(ng), gcell(ng);
            for (size_t g = 0; g < ng; ++g) {
                gli[g] = h.loc[0][h.gamma[g]];
                gle[g] = h.loc[1][h.gamma[g]];
                gcell[g] = h.vcell[h.gamma[g]];
            }
            c->d_gamma.alloc(ng);
            c->d_gamma.upload(h.gamma, s);
            c->d_gloc_i.alloc(ng);
            c->d_gloc_i.upload(gli, s);
            c->d_gloc_e.alloc(ng);
            c->d_gloc_e.upload(gle, s);
            c->d_gcell.alloc(ng);
            c->d_gcell.upload(gcell, s);
            c->d_frow.alloc(h.frow.size());
            c->d_frow.upload(h.frow, s);
            c->d_ffacet.alloc(h.ffacet.size());
            c->d_ffacet.upload(h.ffacet, s);
            c->d_facets.alloc(h.facets.size());
            c->d_facets.upload(h.facets, s);
            c->d_gidx.alloc(h.gidx.size());
            c->d_gidx.upload(h.gidx, s);
            c->d_gcoef.alloc(std::max<size_t>(1, ng) * GC_STRIDE);
            c->d_thv.alloc(std::max<size_t>(1, ng));
            {
                std::vector<int64_t> row(h.n_cells + 1, 0);
                for (size_t g = 0; g < ng; ++g) row[gcell[g]]++;   // gcell is 1-based
                for (int32_t q = 0; q < h.n_cells; ++q) row[q + 1] += row[q];
                std::vector<int32_t> col(std::max<size_t>(1, ng));
                std::vector<int64_t> fill(row.begin(), row.end() - 1);
                for (size_t g = 0; g < ng; ++g) col[fill[gcell[g] - 1]++] = int32_t(g);
                c->d_cgrow.alloc(row.size());
                c->d_cgrow.upload(row, s);
                c->d_cgcol.alloc(col.size());
                c->d_cgcol.upload(col, s);
            }
            // storage order: by vertex, four fields side by side (one vertex's unknowns
            // share a cache line in every gather of x)
            {
                const int64_t N = h.N;
                c->int2ext.resize(N);
                c->ext2int.resize(N);
                for (int r = 0; r < 2; ++r)
                    for (int f = 0; f < 4; ++f)
                        for (int64_t j = 0; j < h.Nr[r]; ++j) {
                            const int64_t e = h.off[r] + f * h.Nr[r] + j, i = h.off[r] + 4 * j + f;
                            c->int2ext[i] = int32_t(e);
                            c->ext2int[e] = int32_t(i);
                        }
                c->rowptr_s.assign(N + 1, 0);
                for (int64_t i = 0; i < N; ++i)
                    c->rowptr_s[i + 1] = c->rowptr_s[i] + (h.rowptr[c->int2ext[i] + 1] - h.rowptr[c->int2ext[i]]);
                c->rstart.resize(N);
                for (int64_t i = 0; i < N; ++i) c->rstart[c->int2ext[i]] = c->rowptr_s[i];
                std::vector<int32_t> cols(std::max<int64_t>(1, h.nnz));
#pragma omp parallel for schedule(static)
                for (int64_t i = 0; i < N; ++i) {
                    const int64_t R = c->int2ext[i], a = h.rowptr[R], len = h.rowptr[R + 1] - a, o = c->rowptr_s[i];
                    for (int64_t q = 0; q < len; ++q) cols[o + q] = c->ext2int[h.colidx[a + q]];
                }
                std::vector<int64_t> diag(N);
                for (int64_t R = 0; R < N; ++R) diag[R] = c->rstart[R] + (h.diag_pos[R] - h.rowptr[R]);
                c->d_rowptr.alloc(h.rowptr.size());
                c->d_rowptr.upload(h.rowptr, s);
                c->d_rowptr_s.alloc(c->rowptr_s.size());
                c->d_rowptr_s.upload(c->rowptr_s, s);
                c->d_rstart.alloc(std::max<int64_t>(1, N));
                c->d_rstart.upload(c->rstart, s);
                c->d_int2ext.alloc(std::max<int64_t>(1, N));
                c->d_int2ext.upload(c->int2ext, s);
                c->d_colidx.alloc(cols.size());
                c->d_colidx.upload(cols, s);
                c->d_diag.alloc(std::max<int64_t>(1, N));
                c->d_diag.upload(diag, s);
                std::vector<int32_t> b = row_blocks(c->rowptr_s.data(), N);
                c->nblkA = int64_t(b.size()) - 1;
                c->d_blkA.alloc(b.size());
                c->d_blkA.upload(b, s);
                build_vertex_view(c, cols);
                hip_check(hipStreamSynchronize(s), "system upload");
            }
            c->d_vals.alloc(h.nnz);
            c->d_sc.alloc(h.N);
            c->nblk = launch::reduce_blocks(h.N);
            c->partial.alloc(size_t(c->nblk) * 16);
            c->w.alloc(h.N);
            c->bh.alloc(h.N);
            c->yh.alloc(h.N);
            c->dscal.alloc(64);
            if (!h.walk) upload_p2(c);
            if (h.walk) upload_rows(c);
            // element and incidence data stay; host copies of the big incidence
            // arrays are no longer needed
            for (int r = 0; r < 2; ++r) {
                std::vector<int32_t>().swap(h.ielem[r]);
                std::vector<uint32_t>().swap(h.ipos[r]);
                std::vector<int64_t>().swap(h.irow[r]);
            }
        }
        c->have_mesh = true;
        if (out) {
            out->n_vert = h.n_vert;
            out->n_elem = h.n_elem;
            out->N_i = h.Nr[0];
            out->N_e = h.Nr[1];
            out->N = h.N;
            out->nnz_A = h.nnz;
            out->nnz_P0 = h.nnz_p0;
            out->n_gamma = int64_t(h.gamma.size());
            out->n_facets = h.n_facets;
            out->n_cells = h.n_cells;
            out->dim = h.dim;
            out->pin_dof = h.pin_dof;
        }
        return KNP_OK;
    });
}

knp_status knp_mesh_upload(knp_ctx *c, int dim, int64_t n_vert, const double *xyz, int64_t n_elem,
                           const int32_t *elem_vert, const int32_t *elem_tag, int64_t pin_vertex,
                           knp_mesh_info *out) {
    return mesh_upload(c, 1, dim, n_vert, xyz, n_elem, elem_vert, elem_tag, pin_vertex, out);
}

knp_status knp_mesh_upload_p2(knp_ctx *c, int dim, int64_t n_vert, const double *xyz, int64_t n_elem,
                              const int32_t *elem_vert, const int32_t *elem_tag, int64_t pin_vertex,
                              knp_mesh_info *out) {
    return mesh_upload(c, 2, dim, n_vert, xyz, n_elem, elem_vert, elem_tag, pin_vertex, out);
}

knp_status knp_get_edges(knp_ctx *c, int64_t *n_edges, int32_t *edge_vertices) {
    return guarded(c, [&]() -> knp_status {
        if (!c->have_mesh) return fail(c, KNP_E_STATE, "no mesh");
        const HostMesh &h = c->hm;
        const int64_t ne = int64_t(h.edges.size() / 2);
        if (n_edges) *n_edges = ne;
        if (edge_vertices) std::copy(h.edges.begin(), h.edges.end(), edge_vertices);
        return KNP_OK;
    });
}

knp_status knp_get_layout(knp_ctx *c, int64_t *rowptr, int32_t *colidx, int32_t *dof_vertex) {
    return guarded(c, [&]() -> knp_status {
        if (!c->have_mesh) return fail(c, KNP_E_STATE, "no mesh");
        const HostMesh &h = c->hm;
        if (rowptr) std::memcpy(rowptr, h.rowptr.data(), h.rowptr.size() * sizeof(int64_t));
        if (colidx) std::memcpy(colidx, h.colidx.data(), h.colidx.size() * sizeof(int32_t));
        if (dof_vertex)
            for (int r = 0; r < 2; ++r)
                for (int f = 0; f < 4; ++f)
                    for (int64_t j = 0; j < h.Nr[r]; ++j) dof_vertex[h.off[r] + f * h.Nr[r] + j] = h.verts[r][j];
        return KNP_OK;
    });
}

knp_status knp_get_gamma(knp_ctx *c, int32_t *gamma_vertex) {
    return guarded(c, [&]() -> knp_status {
        if (!c->have_mesh) return fail(c, KNP_E_STATE, "no mesh");
        if (!gamma_vertex) return fail(c, KNP_E_ARG, "NULL output");
        std::memcpy(gamma_vertex, c->hm.gamma.data(), c->hm.gamma.size() * sizeof(int32_t));
        return KNP_OK;
    });
}

knp_status knp_set_params(knp_ctx *c, const knp_params *p) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->have_mesh) return fail(c, KNP_E_STATE, "knp_mesh_upload must come first");
        if (!p) return fail(c, KNP_E_ARG, "NULL params");
        if (p->n_cells != c->hm.n_cells) return fail(c, KNP_E_ARG, "n_cells does not match the mesh");
        if (p->n_cells > 0 && (!p->cell_model || !p->cell_stim)) return fail(c, KNP_E_ARG, "NULL cell arrays");
        if (!(p->F > 0 && p->R > 0 && p->T > 0 && p->C_m > 0) || p->n_ode < 1)
            return fail(c, KNP_E_ARG, "invalid physical constants");
        for (int k = 0; k < 3; ++k)
            if (p->z[k] == 0.0 || !(p->D[k] > 0.0)) return fail(c, KNP_E_ARG, "invalid valence or diffusivity");
        bool hh = false, kir = false;
        for (int32_t i = 0; i < p->n_cells; ++i) {
            const int32_t m = p->cell_model[i];
            if (m < 0 || m > 2) return fail(c, KNP_E_ARG, "cell model must be 0, 1 or 2");
            hh |= (m == 1);
            kir |= (m == 2);
        }
        if (kir && !(p->rho_pump >= 0.0 && std::isfinite(p->rho_pump) && p->P_Na > 0.0 && p->P_K > 0.0 &&
                     p->K_e0 > 0.0 && p->K_i0 > 0.0 && std::isfinite(p->P_Na + p->P_K + p->K_e0 + p->K_i0)))
            return fail(c, KNP_E_ARG, "invalid Kir-Na/K parameters");
        c->prm = *p;
        c->cell_model.assign(p->cell_model, p->cell_model + p->n_cells);
        c->cell_stim.assign(p->cell_stim, p->cell_stim + p->n_cells);
        c->any_hh = hh;
        c->any_kir = kir;
        c->prm.cell_model = nullptr;
        c->prm.cell_stim = nullptr;
        std::vector<int32_t> cm = c->cell_model, cs = c->cell_stim;
        if (cm.empty()) {
            cm.push_back(0);
            cs.push_back(0);
        }
        c->d_cell_model.alloc(cm.size());
        c->d_cell_model.upload(cm, c->stream);
        c->d_cell_stim.alloc(cs.size());
        c->d_cell_stim.upload(cs, c->stream);
        c->have_params = true;
        return KNP_OK;
    });
}

// The diagonal blocks (one per region and field, eq. ``P_prec``) of the stored
// matrix S A S, on the pattern of P_0, in the order the AMG setup reads them.
static std::vector<double> diagonal_blocks(knp_ctx *c) {
    const HostMesh &h = c->hm;
    std::vector<double> vals(h.nnz), out(h.nnz_p0);
    c->d_vals.download(vals.data(), h.nnz, c->stream);
    int64_t o = 0;
    for (int r = 0; r < 2; ++r)
        for (int f = 0; f < 4; ++f)
            for (int64_t j = 0; j < h.Nr[r]; ++j) {
                const int64_t row = h.off[r] + f * h.Nr[r] + j;
                const int64_t n = h.prow[r][j + 1] - h.prow[r][j];
                const int64_t len = h.rowptr[row + 1] - h.rowptr[row];
                const int64_t g = len - (f < 3 ? 2 : 4) * n;
                const int64_t seg = c->rstart[row] + (r == 0 ? 0 : g) + (f < 3 ? 0 : 3 * n);
                for (int64_t q = 0; q < n; ++q) out[o++] = vals[seg + q];
            }
    return out;
}

namespace {

knp_status check_assembly_args(knp_ctx *c, double t_n, double dt, const double *u_prev, const double *gates,
                               const double *f_out) {
    if (!c->have_mesh || !c->have_params) return fail(c, KNP_E_STATE, "mesh and params are required");
    if (!u_prev || !f_out) return fail(c, KNP_E_ARG, "NULL u_prev or f_out");
    if (c->any_hh && !gates) return fail(c, KNP_E_ARG, "gates required for Hodgkin-Huxley cells");
    if (!(dt > 0.0) || !std::isfinite(t_n)) return fail(c, KNP_E_ARG, "invalid dt or t_n");
    return KNP_OK;
}

// The assembly's device work on the context's stream: membrane coefficients into gcoef,
// then the values of A (scaled by the current S; the static part only when dt changed
// or force_static) and f.  The coefficients are computed once per call, so running the
// matrix part twice advances no gate twice.
void enqueue_assembly(knp_ctx *c, double t_n, double dt, const double *u_prev, double *gates, const double *theta,
                      double *gcoef, double *f_out, bool first) {
    const HostMesh &h = c->hm;
    hipStream_t s = c->stream;
    const auto p = c->phys(t_n, dt);
    const auto ma = c->mesh_args();
    const auto ga = c->gamma_args();
    // the point condition on the reference phi_e DOF (gauge 0) or none (gauge 1)
    const int64_t pin = c->gauge == 1 ? int64_t(-1) : h.pin_dof;
    launch::membrane_coefficients(ga, p, h.Nr[0], h.Nr[1], u_prev, gates, theta, gcoef, s);
    if (!h.walk) {   // product form: order 2, or order 1 beyond the walk kernels' limits
        auto p2_matrix_and_rhs = [&](bool force_static) {
            if (force_static || dt != c->dt_static) {
                for (int r = 0; r < 2; ++r)
                    launch::p2_static(c->region(r), c->p2_bulk(r), p, c->d_rowptr.p, c->d_rstart.p, c->d_vals.p,
                                      c->d_sc.p, pin, s);
                c->dt_static = dt;
            }
            for (int r = 0; r < 2; ++r)
                launch::p2_dynamic(c->region(r), c->p2_bulk(r), p, c->d_rowptr.p, c->d_rstart.p, c->d_vals.p,
                                   c->d_sc.p, u_prev, f_out, pin, s);
            launch::p2_membrane(ga, c->region(0), c->region(1), c->p2_mem(), p, c->d_rowptr.p, c->d_rstart.p,
                                c->d_vals.p, c->d_sc.p, gcoef, f_out, s);
        };
        p2_matrix_and_rhs(false);
        if (first) {
            launch::scaling_from_diag(h.N, c->d_vals.p, c->d_diag.p, c->d_sc.p, s);
            p2_matrix_and_rhs(true);
        }
        return;
    }
    auto matrix_and_rhs = [&](bool force_static) {
        if (force_static || dt != c->dt_static) {
            for (int r = 0; r < 2; ++r)
                launch::assemble_static(c->region(r), ma, p, c->d_rowptr.p, c->d_rstart.p, c->d_vals.p, c->d_sc.p,
                                        pin, s);
            c->dt_static = dt;
        }
        for (int r = 0; r < 2; ++r)
            launch::rows_dynamic(c->region(r), c->row_view(r), p, c->d_rowptr.p, c->d_rstart.p, c->d_vals.p,
                                 c->d_sc.p, u_prev, f_out, pin, s);
        launch::p2_membrane(ga, c->region(0), c->region(1), c->p2_mem(), p, c->d_rowptr.p, c->d_rstart.p,
                            c->d_vals.p, c->d_sc.p, gcoef, f_out, s);
    };
    matrix_and_rhs(false);
    if (first) {
        // S from the unscaled diagonal, then the same kernels again with S, so
        // that this step's values round exactly as a later call on the same
        // inputs (recomputed steps reproduce stored ones bit for bit)
        launch::scaling_from_diag(h.N, c->d_vals.p, c->d_diag.p, c->d_sc.p, s);
        matrix_and_rhs(true);
    }
}

void finish_assembly(knp_ctx *c, double t_n, double dt, const double *theta) {
    c->last_theta = theta;
    c->last_t = t_n;
    c->last_dt = dt;
    c->assembled = true;
    c->T_current = false;
    c->ns_stale = true;
}

}  // namespace

knp_status knp_assemble_step(knp_ctx *c, double t_n, double dt, const double *u_prev, double *gates,
                             const double *theta, double *f_out) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        const knp_status st = check_assembly_args(c, t_n, dt, u_prev, gates, f_out);
        if (st != KNP_OK) return st;
        hip_check(hipSetDevice(c->device), "set device");
        const HostMesh &h = c->hm;
        hipStream_t s = c->stream;
        int flag = 0;
        hip_check(hipMemsetAsync(c->d_flag.p, 0, sizeof(int), s), "flag");
        launch::check_finite(u_prev, h.N, c->d_flag.p, s);
        hip_check(hipMemcpyAsync(&flag, c->d_flag.p, sizeof(int), hipMemcpyDeviceToHost, s), "flag copy");
        hip_check(hipStreamSynchronize(s), "flag sync");
        if (flag) return fail(c, KNP_E_NUMERIC, "NaN or Inf in u_prev");
        const bool first = !c->assembled;
        if (first) {
            std::vector<double> ones(h.N, 1.0);
            c->d_sc.upload(ones, s);
        }
        hipEvent_t t0 = c->tm.begin(KNP_TIMER_ASSEMBLY, s);
        enqueue_assembly(c, t_n, dt, u_prev, gates, theta, c->d_gcoef.p, f_out, first);
        c->tm.end(KNP_TIMER_ASSEMBLY, t0, c->assembly_bytes, s);
        if (first) {
            // P_0: the diagonal blocks of the first (scaled) matrix, kept on the host for AMG setup
            std::vector<double> sc(h.N);
            c->p0_vals = diagonal_blocks(c);
            c->d_sc.download(sc.data(), h.N, s);
            c->near_null.resize(h.N);
            for (int64_t i = 0; i < h.N; ++i) c->near_null[i] = 1.0 / sc[i];
            c->dt_first = dt;
        }
        hip_check(hipGetLastError(), "assembly launch");
        // no synchronisation: the kernels run on after the return, in stream order with
        // whatever the caller enqueues next; their timer events are read at the next
        // synchronising call
        finish_assembly(c, t_n, dt, theta);
        return KNP_OK;
    });
}

// The same assembly with its scratch (the NaN counter and the membrane coefficient
// record) in the library's static device array instead of context memory: it enqueues
// kernels and copies only.  The first assembly of a context fixes S and P_0 (host work),
// so it must have been done by knp_assemble_step.
knp_status knp_assemble_step_noalloc(knp_ctx *c, double t_n, double dt, const double *u_prev, double *gates,
                                     const double *theta, double *f_out) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        const knp_status st = check_assembly_args(c, t_n, dt, u_prev, gates, f_out);
        if (st != KNP_OK) return st;
        if (!c->assembled)
            return fail(c, KNP_E_STATE, "knp_assemble_step must have been called once on this context (the "
                                        "first assembly fixes S and P_0)");
        const HostMesh &h = c->hm;
        if (int64_t(h.gamma.size()) > NOALLOC_MAX_GAMMA)
            return fail(c, KNP_E_ARG, "mesh has " + std::to_string(h.gamma.size()) +
                                          " membrane vertices; the static scratch holds at most " +
                                          std::to_string(NOALLOC_MAX_GAMMA));
        if (!c->scratch) return fail(c, KNP_E_STATE, "static scratch not resolved for this device");
        hip_check(hipSetDevice(c->device), "set device");
        hipStream_t s = c->stream;
        int *flag_d = reinterpret_cast<int *>(c->scratch);
        double *gcoef = c->scratch + NOALLOC_HEAD;
        int flag = 0;
        launch::clear_flag(flag_d, s);
        launch::check_finite(u_prev, h.N, flag_d, s);
        hip_check(hipMemcpyAsync(&flag, flag_d, sizeof(int), hipMemcpyDeviceToHost, s), "flag copy");
        hip_check(hipStreamSynchronize(s), "flag sync");
        if (flag) return fail(c, KNP_E_NUMERIC, "NaN or Inf in u_prev");
        enqueue_assembly(c, t_n, dt, u_prev, gates, theta, gcoef, f_out, false);
        hip_check(hipGetLastError(), "assembly launch");
        hip_check(hipStreamSynchronize(s), "assembly");
        finish_assembly(c, t_n, dt, theta);
        return KNP_OK;
    });
}

knp_status knp_set_gauge(knp_ctx *c, int32_t mode) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->have_mesh) return fail(c, KNP_E_STATE, "knp_mesh_upload must come first");
        if (c->assembled) return fail(c, KNP_E_STATE, "the gauge is fixed by the first knp_assemble_step");
        if (mode != 0 && mode != 1) return fail(c, KNP_E_ARG, "gauge must be 0 or 1");
        hip_check(hipSetDevice(c->device), "set device");
        if (mode == 1) gauge_build(c);
        c->gauge = mode;
        return KNP_OK;
    });
}

knp_status knp_amg_setup(knp_ctx *c, const knp_amg_opts *opts) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->assembled) return fail(c, KNP_E_STATE, "knp_assemble_step must come first");
        knp_amg_opts o{0, 0.6, 5, 2.5, 2000, 20, 0.01, 0, 0, 1, 0, 0, 0, 0};
        if (opts) o = *opts;
        if (o.precision != 0 && o.precision != 1) return fail(c, KNP_E_ARG, "precision must be 0 or 1");
        if (!(o.strength > 0.0 && o.strength < 1.0) || o.cheb_degree < 1 || !(o.cheb_ratio > 1.0) ||
            o.coarse_max < 1 || o.max_levels < 1 || !(o.coarse_drop >= 0.0 && o.coarse_drop < 1.0) ||
            o.cheb_pre_degree < 0 || o.coarse_pre_degree < 0 || o.coarse_post_degree < 1 ||
            (o.operator_step != 0 && o.operator_step != 1) || (o.field_split != 0 && o.field_split != 1) ||
            (o.shared_ion_aggregates != 0 && o.shared_ion_aggregates != 1) ||
            (o.coarse_graph != 0 && o.coarse_graph != 1))
            return fail(c, KNP_E_ARG, "invalid AMG options");
        hip_check(hipSetDevice(c->device), "set device");
        if (o.operator_step == 1)
            amg_build(c->amg, c->hm, diagonal_blocks(c), c->near_null, o, c->stream);
        else
            amg_build(c->amg, c->hm, c->p0_vals, c->near_null, o, c->stream);
        c->m_alloc = -1;   // Z precision may change
        return KNP_OK;
    });
}

knp_status knp_amg_stats(knp_ctx *c, int32_t *n_levels, int64_t *level_rows, int64_t *level_nnz) {
    return guarded(c, [&]() -> knp_status {
        if (!c->amg.ready) return fail(c, KNP_E_STATE, "knp_amg_setup has not been called");
        if (!n_levels || !level_rows || !level_nnz) return fail(c, KNP_E_ARG, "NULL output");
        const size_t L = std::min<size_t>(32, c->amg.level_n.size());
        *n_levels = int32_t(L);
        for (size_t l = 0; l < L; ++l) {
            level_rows[l] = c->amg.level_n[l];
            level_nnz[l] = c->amg.level_nnz[l];
        }
        return KNP_OK;
    });
}

static knp_status solve_common(knp_ctx *c, bool transpose, const double *b, double *x, const knp_solve_opts *opts,
                               knp_solve_info *info) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->assembled) return fail(c, KNP_E_STATE, "no assembled system");
        if (!b || !x) return fail(c, KNP_E_ARG, "NULL vector");
        knp_solve_opts o{1e-6, 30, 2000, 0, 1};
        if (opts) o = *opts;
        if (!(o.rtol >= 0.0) || o.restart < 1 || o.restart > 4096 || o.max_it < 0 ||
            (o.precond != 0 && o.precond != 1))
            return fail(c, KNP_E_ARG, "invalid solver options");
        if (transpose && c->gauge == 1)
            return fail(c, KNP_E_STATE, "the adjoint solve needs gauge 0 (the point condition in the system)");
        hip_check(hipSetDevice(c->device), "set device");
        return krylov_solve(c, transpose, b, x, o, info);
    });
}

knp_status knp_gmres_solve(knp_ctx *c, const double *b, double *x, const knp_solve_opts *opts,
                           knp_solve_info *info) {
    return solve_common(c, false, b, x, opts, info);
}

knp_status knp_adjoint_solve(knp_ctx *c, const double *rhs, double *lambda, const knp_solve_opts *opts,
                             knp_solve_info *info) {
    return solve_common(c, true, rhs, lambda, opts, info);
}

knp_status knp_apply(knp_ctx *c, int which, const double *x, double *y) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->assembled) return fail(c, KNP_E_STATE, "no assembled system");
        if (!x || !y) return fail(c, KNP_E_ARG, "NULL vector");
        if (which < 0 || which > 2) return fail(c, KNP_E_ARG, "which must be 0, 1 or 2");
        if (which == 1 && !c->amg.ready) return fail(c, KNP_E_STATE, "knp_amg_setup has not been called");
        hip_check(hipSetDevice(c->device), "set device");
        const int64_t N = c->hm.N;
        hipStream_t s = c->stream;
        double *xi = c->w.p, *yi = c->bh.p;   // solver-order copies of x and y
        launch::to_internal(N, c->d_int2ext.p, x, nullptr, xi, 2, s);
        if (which == 0) {
            apply_operator(c, false, xi, yi);
        } else if (which == 1) {
            if (c->amg.fp32) {
                knp::DArray<float> z;
                z.alloc(N);
                amg_vcycle(c->amg, xi, z.p, s, &c->tm);
                launch::convert<float, double>(N, z.p, yi, s);
                hip_check(hipStreamSynchronize(s), "apply");
            } else {
                amg_vcycle(c->amg, xi, yi, s, &c->tm);
            }
        } else {
            ensure_transpose(c);
            apply_operator(c, true, xi, yi);
        }
        launch::to_external(N, c->d_int2ext.p, yi, nullptr, y, 2, s);
        hip_check(hipStreamSynchronize(s), "apply");
        return KNP_OK;
    });
}

knp_status knp_get_scaling(knp_ctx *c, double *s) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->assembled) return fail(c, KNP_E_STATE, "no assembled system");
        if (!s) return fail(c, KNP_E_ARG, "NULL output");
        hip_check(hipMemcpyAsync(s, c->d_sc.p, sizeof(double) * c->hm.N, hipMemcpyDeviceToDevice, c->stream), "copy");
        hip_check(hipStreamSynchronize(c->stream), "sync");
        return KNP_OK;
    });
}

knp_status knp_extrapolate(knp_ctx *c, const double *u1, const double *u2, double *x0) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->have_mesh) return fail(c, KNP_E_STATE, "no mesh");
        if (!u1 || !u2 || !x0) return fail(c, KNP_E_ARG, "NULL vector");
        hip_check(hipSetDevice(c->device), "set device");
        launch::lincomb(c->hm.N, 2.0, u1, -1.0, u2, x0, c->stream);
        hip_check(hipGetLastError(), "extrapolate launch");
        return KNP_OK;
    });
}

knp_status knp_get_values(knp_ctx *c, double *vals) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!c->assembled) return fail(c, KNP_E_STATE, "no assembled system");
        if (!vals) return fail(c, KNP_E_ARG, "NULL output");
        launch::rows_to_external(c->hm.N, c->d_rowptr.p, c->d_rstart.p, c->d_vals.p, vals, c->stream);
        hip_check(hipStreamSynchronize(c->stream), "sync");
        return KNP_OK;
    });
}

knp_status knp_timing(knp_ctx *c, int enable) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        hip_check(hipStreamSynchronize(c->stream), "sync");
        c->tm.reset();
        c->tm.on = enable != 0;
        return KNP_OK;
    });
}

knp_status knp_timing_read(knp_ctx *c, knp_timer *out) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (!out) return fail(c, KNP_E_ARG, "NULL output");
        hip_check(hipStreamSynchronize(c->stream), "sync");
        c->tm.harvest();
        for (int k = 0; k < KNP_TIMER_COUNT; ++k) {
            out[k].launches = c->tm.cls[k].launches;
            out[k].total_ms = c->tm.cls[k].ms;
            out[k].bytes = c->tm.cls[k].total_bytes;
        }
        return KNP_OK;
    });
}

knp_status knp_step_vjp(knp_ctx *c, const double *u_prev, const double *u_n, const double *lambda_n,
                        double *u_prev_bar, double *theta_bar) {
    return guarded(c, [&]() -> knp_status {
        need_device(c);
        if (c->have_mesh && c->hm.order != 1) return fail(c, KNP_E_ARG, "knp_step_vjp supports order-1 meshes only");
        if (!c->assembled) return fail(c, KNP_E_STATE, "knp_assemble_step of this step must come first");
        if (c->gauge == 1) return fail(c, KNP_E_STATE, "the step VJP needs gauge 0 (the point condition in the system)");
        if (!u_prev || !u_n || !lambda_n || !u_prev_bar) return fail(c, KNP_E_ARG, "NULL vector");
        if (c->any_hh || c->any_kir)
            return fail(c, KNP_E_ARG, "vector-Jacobian products support passive-leak membranes only");
        hip_check(hipSetDevice(c->device), "set device");
        const HostMesh &h = c->hm;
        hipStream_t s = c->stream;
        const auto p = c->phys(c->last_t, c->last_dt);
        const auto ma = c->mesh_args();
        for (int r = 0; r < 2; ++r)
            launch::vjp_bulk(c->region(r), ma, p, u_n, lambda_n, u_prev_bar, h.pin_dof, s);
        launch::vjp_membrane(c->gamma_args(), ma, p, h.Nr[0], h.Nr[1], c->d_prow[0].p, c->d_prow[1].p, u_prev, u_n,
                             lambda_n, c->last_theta, u_prev_bar, c->d_thv.p, s);
        if (theta_bar) launch::reduce_theta(h.n_cells, c->d_cgrow.p, c->d_cgcol.p, c->d_thv.p, theta_bar, s);
        hip_check(hipGetLastError(), "vjp launch");
        hip_check(hipStreamSynchronize(s), "vjp");
        return KNP_OK;
    });
}

}  // extern "C"
