// Internal declarations of libknp: host mesh structures, device buffers,
// AMG hierarchy, solver workspace and the kernel launchers shared between
// the host C++ translation units and the HIP kernel translation units.
#pragma once

#include <hip/hip_runtime_api.h>

#include <cstdint>
#include <memory>
#include <utility>
#include <string>
#include <vector>

#include "../../include/knp.h"

namespace knp {

// Kernel limits for the per-row gather assembly.
constexpr int MAXN = 32;   // scalar neighbours (incl. self) of a vertex in one region
constexpr int MAXG = 16;   // membrane neighbours (incl. self) of a membrane vertex

// Layout of the per-membrane-vertex coefficient record written by the membrane
// kernel: for r in {i, e}: C_r^k (3), g_r^k (3), h_r (1); then I_ch^k (3).
constexpr int GC_STRIDE = 20;
constexpr int GC_C = 0, GC_G = 3, GC_H = 6, GC_REGION = 7, GC_I = 14;

// Static scratch of the allocation-free assembly (knp_assemble_step_noalloc): NOALLOC_HEAD
// doubles (256 bytes) holding the NaN counter, then the coefficient record of at most
// NOALLOC_MAX_GAMMA membrane vertices (40 MiB in all, per device).
constexpr int64_t NOALLOC_HEAD = 32;
constexpr int64_t NOALLOC_MAX_GAMMA = 262144;

struct Error {
    knp_status st;
    std::string msg;
};

// ----------------------------------------------------------------------------- host mesh
struct HostMesh {
    int dim = 0;
    // Element order p.  For p = 2 the "vertices" of everything below are the P2 nodes:
    // the mesh vertices keep their ids, the edge (a, b), a < b, numbered in lexicographic
    // order of its vertex pair as e, is node n_vert_p1 + e at the edge midpoint; elements
    // list their d + 1 vertices and then their edges in lexicographic order of the local
    // pair, facets their d vertices (ascending) and then their edges the same way.
    int order = 1;
    int nv_elem = 0, nv_facet = 0;  // nodes per element and per membrane facet
    int64_t n_vert_p1 = 0;          // mesh vertices
    // order 1: every vertex within MAXN region and MAXG membrane neighbours, so the
    // element-walk kernels (packed positions) apply; otherwise the product-form path
    bool walk = false;
    std::vector<int32_t> edges;     // p = 2: [n_edges*2] vertex pairs of the edge nodes
    int64_t n_vert = 0, n_elem = 0;
    std::vector<double> xyz;        // [n_vert*dim]
    std::vector<int32_t> elem;      // [n_elem*nv_elem]
    std::vector<int32_t> tag;       // [n_elem]
    int32_t n_cells = 0;
    int64_t Nr[2] = {0, 0};
    int64_t off[2] = {0, 0};
    std::vector<int32_t> loc[2];    // [n_vert] region-local index or -1
    std::vector<int32_t> verts[2];  // region vertices (global ids, ascending)
    std::vector<int32_t> vcell;     // [n_vert] cell id of ICS vertices, 0 otherwise
    std::vector<int32_t> gamma;     // membrane vertices, ascending
    std::vector<int32_t> gidx;      // [n_vert] index into gamma or -1
    std::vector<int32_t> facets;    // [n_f*nv_facet] membrane facets (global ids, vertices ascending)
    int64_t n_facets = 0;
    // scalar pattern of each region (region-local indices, ascending)
    std::vector<int64_t> prow[2];
    std::vector<int32_t> pcol[2];
    // membrane adjacency: per membrane vertex, neighbour global ids (ascending)
    std::vector<int64_t> grow;
    std::vector<int32_t> gcol;
    // element incidence per region vertex; ipos packs the slot of the row vertex
    // in the element (bits 0-1) and the row positions of the element's vertices
    // (5 bits each from bit 2)
    std::vector<int64_t> irow[2];
    std::vector<int32_t> ielem[2];
    std::vector<uint32_t> ipos[2];
    // facet incidence per membrane vertex; fpos[r] packs the slot of the row vertex
    // (bits 0-1), the region-r row positions (5 bits each from bit 2) and the
    // membrane-row positions (4 bits each from bit 17)
    std::vector<int64_t> frow;
    std::vector<int32_t> ffacet;
    std::vector<uint32_t> fpos[2];
    // global CSR pattern
    int64_t N = 0, nnz = 0, nnz_p0 = 0;
    std::vector<int64_t> rowptr;
    std::vector<int32_t> colidx;
    std::vector<int64_t> diag_pos;  // [N]
    int64_t pin_vertex = 0, pin_dof = 0;
};

// Builds everything above from the raw mesh (elem: d + 1 vertices per element) for
// element order 1 or 2; throws Error.  The packed incidence positions (ipos, fpos) exist
// only where the element-walk kernels apply (walk); the slot (low bits) always.
void build_host_mesh(HostMesh &m, int dim, int order, int64_t n_vert, const double *xyz, int64_t n_elem,
                     const int32_t *elem, const int32_t *tag, int64_t pin_vertex);

// ----------------------------------------------------------------------------- P2 operators
// Static operators of the order-2 assembly, built on the host once per mesh from the
// element and facet integrals; every per-step value is then a sparse product with the
// nodal concentrations or membrane coefficients.
//   Bulk, per region r, on its scalar pattern (entry p = (row node j, column node q)):
//     sval[p] = int grad phi_j . grad phi_q,  mval[p] = int phi_j phi_q,
//     terms wptr[p]..wptr[p+1]: (wnode, wval) with wval = int phi_m grad phi_j . grad phi_q
//     summed over the elements containing j and q, one term per weight node m
//     (region-local), so that int c_h grad phi_j . grad phi_q = sum_t wval_t c(wnode_t).
//   Membrane, per membrane node g and membrane neighbour a (entry e of grow/gcol):
//     mg[e] = int_Gamma phi_g phi_a;  terms cptr[e]..cptr[e+1]: (cnode, cval), cnode the
//     membrane index of a weight node c, cval = int_Gamma phi_g phi_a phi_c;
//     rpos[r][e] = position of a in the region-r scalar row of g.
struct P2Host {
    std::vector<int32_t> mrow;      // [n_mem] membrane node of each membrane entry
    std::vector<int64_t> wptr[2];
    std::vector<int32_t> wnode[2], erow[2];
    std::vector<double> wval[2], sval[2], mval[2];
    std::vector<double> mg;
    std::vector<int64_t> cptr;
    std::vector<int32_t> cnode, rpos[2];
    std::vector<double> cval;
};
void build_p2_operators(const HostMesh &m, P2Host &out);   // throws Error
// the two halves of it: the bulk operators (sval, mval, erow, the w terms) and the
// membrane ones (mrow, mg, the c terms, rpos)
void build_p2_bulk(const HostMesh &m, P2Host &out);
void build_p2_membrane(const HostMesh &m, P2Host &out);

// ----------------------------------------------------------------------------- row terms
// The per-step bulk values of an order-1 mesh as sparse products with the nodal
// concentrations, laid out for one wavefront per group of consecutive rows.  For the
// row vertex i and an off-diagonal column j of region r,
//   int c_h grad phi_i . grad phi_j = sum_{T containing i, j} |T| G_ij(T) cbar_T,
// with G_ij = grad lambda_i . grad lambda_j and cbar_T the mean of c over the d + 1
// vertices of T (exact for P1).  Each element around the edge (i, j) holds d - 1 further
// vertices p (the edge's ring), so with w_p = sum_{T containing i, j, p} |T| G_ij(T)/(d+1)
//   int c_h grad phi_i . grad phi_j = sum_p w_p c_p + (sum_p w_p) (c_i + c_j)/(d - 1),
// and since sum_j G_ij(T) = 0 the diagonal value is minus the sum of the row's
// off-diagonal ones.  Every ring vertex is a neighbour of i, so a term is stored as
// (position of p in row i, w_p).  Weights below 32 eps of the row's largest are the
// rounding residue of integrals that vanish (right-angled elements) and are dropped.
struct RowGroup {
    int64_t term0;      // first term of the group
    uint64_t starts;    // bit x: the group's entry x is the first of a row
    int32_t row0;       // first row (region-local vertex)
    int16_t tmax;       // most terms of one entry in the group
    int16_t nmax;       // longest row of the group
};
struct RowTerms {
    std::vector<RowGroup> groups;   // [ngroups + 1]; the last holds row0 = N_r, term0 = all terms
    std::vector<uint8_t> tcount;    // [entries] terms of each entry of the region's pattern
    std::vector<uint8_t> tslot;     // [terms] position of the weight's vertex in the row
    std::vector<double> tval;       // [terms]
    std::vector<double> mval;       // [entries] int phi_i phi_j
};
constexpr int ROW_GROUP = 64;       // entries per group: one wavefront
// Builds both regions' row terms of an order-1 mesh; false (nothing built) if a row has
// more than ROW_GROUP entries.
bool build_row_terms(const HostMesh &m, RowTerms out[2]);

// ----------------------------------------------------------------------------- device buffer
template <typename T>
struct DArray {
    T *p = nullptr;
    size_t n = 0;
    DArray() = default;
    DArray(const DArray &) = delete;
    DArray &operator=(const DArray &) = delete;
    ~DArray() { release(); }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    void alloc(size_t count);                  // throws Error on failure
    void upload(const T *h, size_t count, hipStream_t s);
    void upload(const std::vector<T> &v, hipStream_t s) { upload(v.data(), v.size(), s); }
    void download(T *h, size_t count, hipStream_t s) const;
};

void hip_check(hipError_t e, const char *what);   // throws Error(KNP_E_HIP)

// ----------------------------------------------------------------------------- timing
// Event-bracketed launches per kernel class; elapsed times are harvested at the
// next host synchronisation point.
struct Timers {
    bool on = false;
    struct Cls {
        std::vector<hipEvent_t> a, b;   // pending start/stop pairs
        std::vector<double> bytes;      // pending algorithmic bytes
        int64_t launches = 0;
        double ms = 0.0, total_bytes = 0.0;
    } cls[KNP_TIMER_COUNT];
    std::vector<hipEvent_t> pool;
    hipEvent_t begin(int k, hipStream_t s);
    void end(int k, hipEvent_t start, double bytes, hipStream_t s);
    void harvest();   // call after the stream has been synchronised
    void reset();
    ~Timers();
};

// ----------------------------------------------------------------------------- AMG
// Host arrays of the AMG setup: resize() leaves new elements uninitialised (every
// producer writes all of them), so the multi-GB level arrays are not first zeroed by
// one thread; assign() and value-constructing calls still initialise.
template <class T>
struct NoInitAlloc : std::allocator<T> {
    template <class U>
    struct rebind {
        using other = NoInitAlloc<U>;
    };
    NoInitAlloc() = default;
    template <class U>
    NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
    template <class U>
    void construct(U *p) noexcept {
        ::new (static_cast<void *>(p)) U;
    }
    template <class U, class... Args>
    void construct(U *p, Args &&...args) {
        ::new (static_cast<void *>(p)) U(std::forward<Args>(args)...);
    }
};
template <class T>
using hvec = std::vector<T, NoInitAlloc<T>>;

struct Csr {
    int64_t nrows = 0, ncols = 0;
    hvec<int64_t> rowptr;
    hvec<int32_t> col;
    hvec<double> val;
    int64_t nnz() const { return rowptr.empty() ? 0 : rowptr.back(); }
};

// Device view of a CSR pattern for the block-streamed kernels: blk[b]..blk[b+1]
// are the rows of block b, whose entries fit one block's staging buffer.
struct CsrView {
    int64_t nrows = 0, nnz = 0, nblk = 0;
    const int64_t *rowptr = nullptr;
    const int32_t *col = nullptr;
    const int32_t *blk = nullptr;
};

// Device view of the system matrix by vertex.  Storage rows 4v..4v+3 are the four
// fields of vertex v (region i's vertices 0..nv_i-1 first, then region e's), and
// their columns follow from the vertex's neighbour list nbr[nptr[v]..nptr[v+1]),
// ascending: the m neighbours in its own region (itself among them) and the p
// membrane partners in the other region, which therefore come first for a region-e
// vertex and last for a region-i one.  In its entry order, a concentration row (f <
// 3) holds field f and then phi of the m neighbours, a phi row the fields 0, 1, 2,
// 3 of the m neighbours, and either row phi of the p partners before (region e) or
// after (region i) those.  The values stay in the CSR storage: vptr[v] is the
// first entry of row 4v, and m follows from the entry count 10 m + 4 p.  Block b
// owns vertices blk[b]..blk[b+1]-1 (at most VTX_VMAX), whose entries (at most
// VTX_CAP) start at kblk[b] = vptr[blk[b]] and whose pairs start at pblk[b] =
// nptr[blk[b]].
struct VtxView {
    int64_t nv = 0, nv_i = 0, nblk = 0;
    const int64_t *vptr = nullptr;
    const int32_t *nptr = nullptr;
    const int32_t *nbr = nullptr;
    const int32_t *blk = nullptr;
    const int64_t *kblk = nullptr;
    const int32_t *pblk = nullptr;
};
constexpr int VTX_CAP = 1536;
constexpr int VTX_VMAX = 32;
constexpr int VTX_RUNS = 14;   // runs per vertex: 3 per concentration row, 5 for phi

constexpr int STREAM_CAP = 2048;   // entries per row block (8 per thread of 256)
// Zeroed entries after the column indices and values of every level matrix: the
// FP32 stream reads 4 consecutive entries per lane from a 4-aligned start, up to
// 3 entries past a block's end.
constexpr int STREAM_PAD = 4;
// Row-block boundaries for the block-streamed kernels; throws if a row is longer
// than STREAM_CAP.
std::vector<int32_t> row_blocks(const int64_t *rowptr, int64_t nrows, int64_t cap = STREAM_CAP);

struct DevCsr {
    int64_t nrows = 0, ncols = 0, nnz = 0;
    DArray<int64_t> rowptr;
    DArray<int32_t> col;
    DArray<int32_t> blk;
    int64_t nblk = 0;
    DArray<double> val64;
    DArray<float> val32;
    void upload(const Csr &h, bool fp32, hipStream_t s);
    CsrView view() const {
        CsrView v;
        v.nrows = nrows;
        v.nnz = nnz;
        v.nblk = nblk;
        v.rowptr = rowptr.p;
        v.col = col.p;
        v.blk = blk.p;
        return v;
    }
};

// The finest AMG level is P_0, whose four field blocks in a region share that
// region's scalar pattern (rows and columns by region vertex).  It is stored once
// per vertex pair with the four field values side by side: block row v is region
// vertex v (region i first, then region e), its entries index region-local
// vertices, and vals[4k + f] is the field-f value of entry k.  Its vectors are in
// the solver's order, (region r, field f, local vertex j) at off_r + 4 j + f, except
// the residual handed to the restriction, which is field-major (off_r + f N_r + j).
constexpr int FB_CAP = 1024;        // vertex-pair entries per row block (4 products each)
struct FieldBlockView {
    int64_t nv = 0, nnz = 0, nblk = 0;   // block rows, entries, row blocks
    int64_t Ni = 0, Ne = 0;
    const int64_t *rowptr = nullptr;     // [nv+1]
    const int32_t *col = nullptr;        // [nnz + STREAM_PAD], region-local vertex
    const int32_t *blk = nullptr;        // [nblk+1]; no block straddles the regions
};
struct DevFieldBlock {
    int64_t nv = 0, nnz = 0, nblk = 0, Ni = 0, Ne = 0;
    DArray<int64_t> rowptr;
    DArray<int32_t> col, blk;
    DArray<double> val64;                // [4 (nnz + STREAM_PAD)]
    DArray<float> val32;
    FieldBlockView view() const {
        FieldBlockView v;
        v.nv = nv;
        v.nnz = nnz;
        v.nblk = nblk;
        v.Ni = Ni;
        v.Ne = Ne;
        v.rowptr = rowptr.p;
        v.col = col.p;
        v.blk = blk.p;
        return v;
    }
};

// blocks of a field-split level: one per region and field
constexpr int CHEB_BLOCKS = 8;

struct Level {
    int64_t n = 0;
    double lmax = 2.0;           // spectral radius estimate of the (unit-diagonal) operator
    DevCsr A, P, R;              // P: n x n_coarse, R = P^T (A unused on level 0)
    DevFieldBlock fb;            // level 0 only: P_0 in the field-block layout
    // field split (coarser levels): rows of block q (region r, field f: q = 4 r + f) are
    // [bstart[q], bstart[q+1]); blmax[q] bounds that block's spectrum (Gershgorin)
    int nblocks = 0;
    int32_t bstart[CHEB_BLOCKS + 1] = {};
    double blmax[CHEB_BLOCKS] = {};
    // level vectors (precision of the hierarchy); x, x2 and d are the three buffers the
    // Chebyshev recurrence in x rotates through, t the residual
    DArray<double> b64, x64, x2_64, t64, d64;
    DArray<float> b32, x32, x2_32, t32, d32;
};

struct Amg {
    bool ready = false;
    bool fp32 = false;
    int degree = 3;                  // finest level: post-smoothing degree
    int pre_degree = 2;              // finest level: pre-smoothing degree
    int coarse_pre = 1, coarse_post = 1;   // coarser levels (pre 0: restrict b directly)
    bool field_split = false;        // coarser levels: a smoothing interval per field block
    double ratio = 2.5;
    std::vector<Level *> levels;     // levels[0] is P_0
    // coarsest-level dense inverses, one per connected component
    int64_t n_coarse = 0;
    DArray<int32_t> ccomp;           // [n_coarse] component of each coarsest row
    DArray<int32_t> cloc;            // [n_coarse] position of the row inside its component
    DArray<int32_t> cmem;            // [n_coarse] rows of each component, concatenated
    DArray<int64_t> cstart;          // [n_blocks+1] start of each component in cmem
    DArray<int64_t> coff;            // [n_blocks] offset of the component's inverse
    DArray<double> cinv;             // packed dense inverses (row-major)
    DArray<double> cb64, cx64;       // coarse rhs / solution in FP64
    int64_t n_blocks = 0;
    std::vector<int64_t> level_nnz, level_n;
    double vcycle_bytes = 0.0;       // algorithmic bytes of one V-cycle (its timer class)
    // the levels below the finest as one HIP graph: captured (on a stream of its own; the
    // caller's may be the legacy default stream, which cannot be captured) at the first
    // V-cycle after a setup, replayed on the caller's stream; the levels' buffers are fixed,
    // so every replay runs the same kernels on the same data as the launches would
    bool coarse_graph = false;
    hipStream_t capture_stream = nullptr;
    hipGraphExec_t coarse_exec = nullptr;
    void *coarse_out = nullptr;      // the level-1 buffer the sub-cycle leaves its result in
    ~Amg();
    void clear();
};

void amg_build(Amg &amg, const HostMesh &m, const std::vector<double> &p0_vals,
               const std::vector<double> &near_null, const knp_amg_opts &o, hipStream_t s);
// z = V-cycle(v) on level 0; v is FP64; z is FP64 or FP32 per amg.fp32
void amg_vcycle(Amg &amg, const double *v, void *z, hipStream_t s, Timers *tm = nullptr);

}  // namespace knp

// ----------------------------------------------------------------------------- kernel launchers
namespace knp {
namespace launch {

struct RegionArgs {
    int r;                     // 0 = ICS, 1 = ECS
    int dim;
    int64_t Nr, off, off_q;    // region size, DOF offsets of this and the other region
    int64_t Nq;
    const int64_t *prow;       // scalar pattern row pointers
    const int32_t *pcol;
    const int64_t *irow;       // element incidence
    const int32_t *ielem;
    const uint32_t *ipos;
    const int32_t *verts;      // region vertices (global)
};

struct MeshArgs {
    int dim;
    const double *xyz;
    const int32_t *elem;
    const int32_t *loc_i, *loc_e;
};

struct PhysArgs {
    double z[3], D[3], tau[3], ttau[3];
    double F, C_m, psi, dt, t;
    double g_leak[3], gbar_Na, gbar_K, g_stim_bar, stim_a, stim_tau, phi_rest;
    double rho_pump, P_Na, P_K, K_e0, E_K0;   // Kir-Na/K
    int n_ode;
};

struct GammaArgs {
    int64_t n_gamma;
    const int32_t *gamma;      // global ids
    const int32_t *gloc_i, *gloc_e, *gcell;   // local indices and cell (1-based)
    const int64_t *frow;
    const int32_t *ffacet;
    const uint32_t *fpos_i, *fpos_e;
    const int32_t *facets;
    const int32_t *gidx;       // [n_vert]
    const int32_t *cell_model, *cell_stim;
};

// order-2 assembly: device views of the P2Host operators
struct P2Bulk {
    int64_t nent = 0;
    const int64_t *wptr = nullptr;
    const int32_t *wnode = nullptr, *erow = nullptr;
    const double *wval = nullptr, *sval = nullptr, *mval = nullptr;
};
struct P2Mem {
    int64_t nmem = 0;
    const int64_t *grow = nullptr, *cptr = nullptr;
    const int32_t *gcol = nullptr, *mrow = nullptr, *cnode = nullptr, *rpos_i = nullptr, *rpos_e = nullptr;
    const double *mg = nullptr, *cval = nullptr;
};
// order-1 per-step bulk values from the row terms (RowTerms on the device)
struct RowView {
    int64_t ngroups = 0;
    const RowGroup *groups = nullptr;   // [ngroups + 1]
    const uint8_t *tcount = nullptr, *tslot = nullptr;
    const double *tval = nullptr, *mval = nullptr;
};
void rows_dynamic(const RegionArgs &ra, const RowView &rv, const PhysArgs &p, const int64_t *rowptr,
                  const int64_t *rstart, double *vals, const double *sc, const double *u_prev, double *f,
                  int64_t pin_dof, hipStream_t s);
// the dt-dependent static blocks of one region (c rows: M + tau_k A; phi row: z_k tau_k A)
void p2_static(const RegionArgs &ra, const P2Bulk &b, const PhysArgs &p, const int64_t *rowptr, const int64_t *rstart,
               double *vals, const double *sc, int64_t pin_dof, hipStream_t s);
// the per-step bulk blocks and f of one region
void p2_dynamic(const RegionArgs &ra, const P2Bulk &b, const PhysArgs &p, const int64_t *rowptr,
                const int64_t *rstart, double *vals, const double *sc, const double *u_prev, double *f,
                int64_t pin_dof, hipStream_t s);
// the membrane blocks and terms of f of both regions, from the coefficient records
void p2_membrane(const GammaArgs &g, const RegionArgs &ra_i, const RegionArgs &ra_e, const P2Mem &mm, const PhysArgs &p,
                 const int64_t *rowptr, const int64_t *rstart, double *vals, const double *sc, const double *gcoef,
                 double *f, hipStream_t s);

void check_finite(const double *u, int64_t n, int *flag, hipStream_t s);
// *flag = 0 by a kernel (no memset node)
void clear_flag(int *flag, hipStream_t s);
// This device's address of the allocation-free assembly's static scratch; resolved with
// hipGetSymbolAddress the first time per device (the device must be current).  Throws.
double *noalloc_scratch(int device);
void membrane_coefficients(const GammaArgs &g, const PhysArgs &p, int64_t Ni, int64_t Ne, const double *u_prev,
                           double *gates, const double *theta, double *gcoef, hipStream_t s);
// rowptr: ABI-order row pointers (row lengths); rstart[R]: storage start of ABI row R
void assemble_static(const RegionArgs &ra, const MeshArgs &ma, const PhysArgs &p,
                     const int64_t *rowptr, const int64_t *rstart, double *vals, const double *sc, int64_t pin_dof,
                     hipStream_t s);
// solver order (off_r + 4 j + f) <-> ABI order (off_r + f N_r + j); int2ext maps the
// first to the second; mode 0: times sc, 1: divided by sc, 2: plain copy
void to_internal(int64_t n, const int32_t *int2ext, const double *x, const double *sc, double *y, int mode,
                 hipStream_t s);
void to_external(int64_t n, const int32_t *int2ext, const double *y, const double *sc, double *x, int mode,
                 hipStream_t s);
void rows_to_external(int64_t N, const int64_t *rowptr, const int64_t *rstart, const double *src, double *dst,
                      hipStream_t s);
void scaling_from_diag(int64_t N, const double *vals, const int64_t *diag_pos, double *sc, hipStream_t s);
void gather(int64_t n, const double *src, const int64_t *map, double *dst, hipStream_t s);

// sparse and dense linear algebra
template <typename TM, typename TX, typename TY>
void spmv(const CsrView &A, const TM *val, const TX *x, TY *y, hipStream_t s);
// y = A x for the system matrix by vertex (FP64 values and result)
template <typename TX>
void spmv_vtx(const VtxView &A, const double *val, const TX *x, double *y, hipStream_t s);
// y = b - A x
template <typename T>
void residual(const CsrView &A, const T *val, const T *x, const T *b, T *y, hipStream_t s);
// Chebyshev step in x alone: x_out = x_in + c1 (x_in - x_prev) + c2 (b - A x_in);
// x_in null: the first step from x = 0, x_out = c2 b; x_prev null: the zero vector
template <typename T>
void cheb_step(const CsrView &A, const T *val, const T *x_in, const T *b, const T *x_prev, T *x_out, double c1,
               double c2, hipStream_t s);
// the same step with coefficients per block of contiguous rows (one block per region and
// field: the field-split smoother); block q holds rows [start[q], start[q+1])
struct ChebBlocks {
    int nb;
    int32_t start[CHEB_BLOCKS + 1];
    double c1[CHEB_BLOCKS], c2[CHEB_BLOCKS];
};
template <typename T>
void cheb_step_blocks(const CsrView &A, const T *val, const T *x_in, const T *b, const T *x_prev, T *x_out,
                      const ChebBlocks &cb, hipStream_t s);
// x += P xc
template <typename T>
void prolong_add(const CsrView &P, const T *val, const T *xc, T *x, hipStream_t s);
// the same residual and Chebyshev step on the field-block layout of level 0; the
// residual y is written field-major (off_r + f N_r + j), the order of the
// restriction's columns on level 0
template <typename T>
void fb_residual(const FieldBlockView &A, const T *val, const T *x, const T *b, T *y, hipStream_t s);
template <typename T>
void fb_cheb_step(const FieldBlockView &A, const T *val, const T *x_in, const T *b, const T *x_prev, T *x_out,
                  double c1, double c2, hipStream_t s);
// a level-0 vector into field-major order (the restriction's column order)
template <typename T>
void to_field_major(const FieldBlockView &A, const T *src, T *dst, hipStream_t s);
template <typename TA, typename TB>
void convert(int64_t n, const TA *a, TB *b, hipStream_t s);
void coarse_solve(int64_t n, const int32_t *comp, const int32_t *cloc, const int32_t *cmem, const int64_t *cstart,
                  const int64_t *coff, const double *inv, const double *b, double *x, hipStream_t s);

// Krylov helpers (deterministic two-stage reductions)
void multi_dot(int64_t n, const double *V, int64_t ldv, int k, const double *w, double *out,
               double *partial, int nblk, hipStream_t s);
template <typename TZ>
void multi_axpy(int64_t n, const TZ *Z, int64_t ldz, int k, const double *coef, double *x, hipStream_t s);
void gs_update(int64_t n, const double *V, int64_t ldv, int k, const double *h, double *w,
               double *partial, int nblk, hipStream_t s);   // w -= V h; partial norms
void reduce_partials(int k, int nblk, const double *partial, double *out, hipStream_t s);
void scale_by_inv_norm(int64_t n, const double *w, const double *nrm2, double *v, hipStream_t s);
void add_scaled(int64_t n, double a, const double *x, double *y, hipStream_t s);   // y += a x
void axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s);
void sub(int64_t n, const double *a, const double *b, double *y, hipStream_t s);   // y = a - b
void lincomb(int64_t n, double a, const double *x, double b, const double *y, double *out,
             hipStream_t s);   // out = a x + b y
int reduce_blocks(int64_t n);

// the constant-potential gauge inside the solver (nullspace.hip)
// out[k] = sum_{q in [ptr[k], ptr[k+1])} zs[q] v[idx[q]]: CELL_SPLIT workgroups per cell
// write part[k * CELL_SPLIT + c], then the partials are added in order
constexpr int CELL_SPLIT = 8;
void cell_dot(int ncell, const int64_t *ptr, const int32_t *idx, const double *zs, const double *v, double *part,
              double *out, hipStream_t s);
// zs[q] = 1 / sc[int2ext[idx[q]]]; u = 0 except u[idx[q]] = zs[q]
void cell_basis(int64_t n, int64_t nidx, const int32_t *idx, const int32_t *int2ext, const double *sc, double *zs,
                double *u, hipStream_t s);
// c_k = sum[k] / E[k]; r[i] -= c_owner(i) W[i], y[i] += c_owner(i) u[i] where owner(i) >= 0
// (r or y null: that update skipped)
void cell_correct(int64_t n, const int32_t *owner, const double *W, const double *u, const double *sum,
                  const double *E, double *r, double *y, hipStream_t s);
// y[rows[t]] = sum of val[q] x[col[q]] over the listed entries q = rowptr[rows[t]] + off[e],
// e in [wptr[t], wptr[t+1]) (CSR storage view); other rows untouched
void rows_sub_spmv(int64_t n, const int32_t *rows, const int64_t *wptr, const uint16_t *off, const int64_t *rowptr,
                   const int32_t *col, const double *val, const double *x, double *y, hipStream_t s);
void fill_zero(int64_t n, double *y, hipStream_t s);
// x[j] -= *ref on [a0, a1) and [b0, b1)
void shift_potentials(int64_t a0, int64_t a1, int64_t b0, int64_t b1, const double *ref, double *x, hipStream_t s);

// adjoint
void vjp_bulk(const RegionArgs &ra, const MeshArgs &ma, const PhysArgs &p, const double *u_n, const double *lam,
              double *u_prev_bar, int64_t pin_dof, hipStream_t s);
void vjp_membrane(const GammaArgs &g, const MeshArgs &ma, const PhysArgs &p, int64_t Ni, int64_t Ne,
                  const int64_t *prow_i, const int64_t *prow_e, const double *u_prev, const double *u_n,
                  const double *lam, const double *theta, double *u_prev_bar, double *theta_vertex, hipStream_t s);
void reduce_theta(int n_cells, const int64_t *cg_row, const int32_t *cg_col, const double *theta_vertex,
                  double *theta_bar, hipStream_t s);

}  // namespace launch
}  // namespace knp
