// The opaque context behind knp_ctx: mesh, device-resident system, AMG
// hierarchy and Krylov workspace of one HIP device and stream.
#pragma once

#include "knp_internal.h"

namespace knp {
// Pinned host buffer (hipHostMalloc): the target of the solver's small per-iteration
// device-to-host copies, which from pageable memory cost ~0.1 ms each.
template <typename T>
struct PinnedArray {
    T *p = nullptr;
    size_t n = 0;
    PinnedArray() = default;
    PinnedArray(const PinnedArray &) = delete;
    PinnedArray &operator=(const PinnedArray &) = delete;
    ~PinnedArray() { release(); }
    void release() {
        if (p) (void)hipHostFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count) {
        release();
        if (count == 0) return;
        hip_check(hipHostMalloc(reinterpret_cast<void **>(&p), count * sizeof(T), hipHostMallocDefault),
                  "pinned host allocation");
        n = count;
    }
};
}  // namespace knp

struct knp_ctx {
    int device = -1;
    bool host_only = true;
    hipStream_t stream = nullptr;
    std::string err;

    bool have_mesh = false, have_params = false, assembled = false;

    knp::HostMesh hm;

    // parameters
    knp_params prm{};
    std::vector<int32_t> cell_model, cell_stim;
    bool any_hh = false, any_kir = false;

    // device mesh data
    knp::DArray<double> d_xyz;
    knp::DArray<int32_t> d_elem, d_loc[2], d_verts[2];
    knp::DArray<int64_t> d_prow[2], d_irow[2];
    knp::DArray<int32_t> d_pcol[2], d_ielem[2];
    knp::DArray<uint32_t> d_ipos[2];
    knp::DArray<int32_t> d_gamma, d_gloc_i, d_gloc_e, d_gcell, d_ffacet, d_facets, d_gidx;
    knp::DArray<int64_t> d_frow;
    knp::DArray<uint32_t> d_fpos[2];
    knp::DArray<int32_t> d_cell_model, d_cell_stim;
    knp::DArray<double> d_gcoef;
    // order 2: the static P2 operators (knp::P2Host on the device) and the membrane adjacency
    knp::DArray<int64_t> d_p2_wptr[2], d_p2_cptr, d_grow;
    knp::DArray<int32_t> d_p2_wnode[2], d_p2_erow[2], d_p2_rpos[2], d_p2_mrow, d_p2_cnode, d_gcol;
    knp::DArray<double> d_p2_wval[2], d_p2_sval[2], d_p2_mval[2], d_p2_mg, d_p2_cval;
    int64_t p2_nent[2] = {0, 0}, p2_nmem = 0;
    // order 1 within the walk limits: the row terms of the per-step bulk values
    bool rows = false;
    int64_t rows_ngroups[2] = {0, 0};
    knp::DArray<knp::RowGroup> d_rgroups[2];
    knp::DArray<uint8_t> d_rcount[2], d_rslot[2];
    knp::DArray<double> d_rval[2], d_rmval[2];
    knp::DArray<int64_t> d_cgrow;   // membrane vertices of each cell (CSR)
    knp::DArray<int32_t> d_cgcol;
    knp::DArray<double> d_thv;      // per membrane vertex theta adjoint (VJP scratch)
    const double *last_theta = nullptr;
    double last_t = 0.0, last_dt = 0.0;

    // system.  Storage is by vertex with the four fields side by side: storage row
    // (and solver DOF) off_r + 4 j + f holds ABI row off_r + f N_r + j, with its
    // entries in the ABI row's order and columns renumbered to storage DOFs.
    knp::DArray<int64_t> d_rowptr;      // ABI-order row pointers (row lengths for the assembly)
    knp::DArray<int64_t> d_rowptr_s;    // storage row pointers
    knp::DArray<int64_t> d_rstart;      // [N] storage start of ABI row R
    knp::DArray<int64_t> d_diag;        // [N] storage position of ABI row R's diagonal
    knp::DArray<int32_t> d_int2ext;     // [N] storage DOF -> ABI DOF
    knp::DArray<int32_t> d_colidx;      // storage columns
    knp::DArray<double> d_vals, d_sc;   // values in storage order; S in ABI order
    std::vector<int64_t> rowptr_s, rstart;
    std::vector<int32_t> int2ext, ext2int;
    knp::DArray<int32_t> d_blkA;
    int64_t nblkA = 0;
    // A by vertex (knp::VtxView); used for A x when every row fits the pattern
    bool vtx = false;
    int64_t npairs = 0, nvblk = 0;
    knp::DArray<int64_t> d_vptr, d_kblk;
    knp::DArray<int32_t> d_nptr, d_nbr, d_vblk, d_pblk;
    knp::DArray<int32_t> d_flag;
    // this device's copy of the allocation-free assembly's static scratch (resolved at
    // knp_create); the NaN counter, then the membrane coefficient record
    double *scratch = nullptr;
    double dt_static = -1.0;
    double dt_first = -1.0;

    // transposed system (adjoint)
    bool have_T = false, T_current = false;
    knp::DArray<int64_t> d_rowptrT, d_permT;
    knp::DArray<int32_t> d_colT, d_blkT;
    int64_t nblkT = 0;
    knp::DArray<double> d_valsT;

    // gauge: 0 = the point condition phi_e = 0 at the reference DOF is part of the
    // assembled system; 1 = the system is assembled without it and the forward solve
    // handles the constant-potential nullspace (per-cell coarse correction, final shift)
    int gauge = 0;
    // gauge 1: per storage DOF the cell (0-based) whose intracellular potentials its
    // row couples to, or -1; the intracellular potential DOFs of each cell (CSR over
    // cells, storage indices ascending); their 1/S (ns_zs) and the same scattered into
    // a full vector (ns_u); W = S A S u (computed on the membrane rows, 0 elsewhere) and
    // E_k = zs_k^T W of the current system
    int32_t ns_ncell = 0;
    bool ns_basis = false, ns_stale = true;
    int64_t ns_nrows = 0;   // storage rows of membrane nodes (the rows W is computed on)
    knp::DArray<int32_t> d_ns_owner, d_ns_idx, d_ns_rows;
    knp::DArray<int64_t> d_ns_ptr, d_ns_wptr;   // cells' DOF lists; each membrane row's list below
    knp::DArray<uint16_t> d_ns_woff;            // in-row positions of its intracellular potential columns
    knp::DArray<double> d_ns_zs, d_ns_u, d_ns_w, d_ns_e, d_ns_sum, d_ns_part;

    // preconditioner
    std::vector<double> p0_vals, near_null;
    knp::Amg amg;

    knp::Timers tm;
    double assembly_bytes = 0.0;

    // Krylov workspace
    int m_alloc = -1;
    bool z32 = false;
    knp::DArray<double> V, Z64, w, bh, yh, partial, dscal;
    knp::PinnedArray<double> hbuf;   // host side of the Hessenberg column, norms and dots
    knp::DArray<float> Z32;
    int nblk = 1;

    knp::launch::RegionArgs region(int r) const;
    knp::launch::MeshArgs mesh_args() const;
    knp::launch::GammaArgs gamma_args() const;
    knp::launch::PhysArgs phys(double t, double dt) const;
    knp::launch::P2Bulk p2_bulk(int r) const {
        knp::launch::P2Bulk b;
        b.nent = p2_nent[r];
        b.wptr = d_p2_wptr[r].p;
        b.wnode = d_p2_wnode[r].p;
        b.erow = d_p2_erow[r].p;
        b.wval = d_p2_wval[r].p;
        b.sval = d_p2_sval[r].p;
        b.mval = d_p2_mval[r].p;
        return b;
    }
    knp::launch::RowView row_view(int r) const {
        knp::launch::RowView v;
        v.ngroups = rows_ngroups[r];
        v.groups = d_rgroups[r].p;
        v.tcount = d_rcount[r].p;
        v.tslot = d_rslot[r].p;
        v.tval = d_rval[r].p;
        v.mval = d_rmval[r].p;
        return v;
    }
    knp::launch::P2Mem p2_mem() const {
        knp::launch::P2Mem m;
        m.nmem = p2_nmem;
        m.grow = d_grow.p;
        m.cptr = d_p2_cptr.p;
        m.gcol = d_gcol.p;
        m.mrow = d_p2_mrow.p;
        m.cnode = d_p2_cnode.p;
        m.rpos_i = d_p2_rpos[0].p;
        m.rpos_e = d_p2_rpos[1].p;
        m.mg = d_p2_mg.p;
        m.cval = d_p2_cval.p;
        return m;
    }
    knp::CsrView viewA() const {
        knp::CsrView v;
        v.nrows = hm.N;
        v.nnz = hm.nnz;
        v.nblk = nblkA;
        v.rowptr = d_rowptr_s.p;
        v.col = d_colidx.p;
        v.blk = d_blkA.p;
        return v;
    }
    knp::VtxView viewV() const {
        knp::VtxView v;
        v.nv = hm.N / 4;
        v.nv_i = hm.Nr[0];
        v.nblk = nvblk;
        v.vptr = d_vptr.p;
        v.nptr = d_nptr.p;
        v.nbr = d_nbr.p;
        v.blk = d_vblk.p;
        v.kblk = d_kblk.p;
        v.pblk = d_pblk.p;
        return v;
    }
    // algorithmic bytes of one A x through the vertex view, x of xbytes per entry
    double vtx_bytes(double xbytes) const {
        const double nv = double(hm.N / 4);
        return 8.0 * double(hm.nnz) + 4.0 * double(npairs) + 12.0 * (nv + 1.0) + (xbytes + 8.0) * double(hm.N) +
               16.0 * double(nvblk + 1);
    }
    knp::CsrView viewT() const {
        knp::CsrView v;
        v.nrows = hm.N;
        v.nnz = hm.nnz;
        v.nblk = nblkT;
        v.rowptr = d_rowptrT.p;
        v.col = d_colT.p;
        v.blk = d_blkT.p;
        return v;
    }
};

namespace knp {
knp_status krylov_solve(knp_ctx *c, bool transpose, const double *b, double *x, const knp_solve_opts &o,
                        knp_solve_info *info);
void ensure_transpose(knp_ctx *c);
// y = (S A S) x or its transpose, FP64; timed under `timer` (a KNP_TIMER_* class)
void apply_operator(knp_ctx *c, bool transpose, const double *x, double *y, int timer = KNP_TIMER_SPMV_A);
// y = b - (S A S) x (or the transpose), FP64, timed as KNP_TIMER_RESID_A
void residual(knp_ctx *c, bool transpose, const double *x, const double *b, double *y);
// gauge 1: the cell ownership of every storage DOF and the per-cell lists of the
// intracellular potential DOFs (host work and upload; needs the mesh)
void gauge_build(knp_ctx *c);
}  // namespace knp
