// Algebraic multigrid for the frozen block-diagonal preconditioner P_0
// (eq. ``P_prec``; one V-cycle approximates P_0^{-1}, Sec. "Solution and
// preconditioning strategy").
//
// Setup (host, once per run): smoothed aggregation.  The operator arrives
// symmetrically scaled to unit diagonal.  Per level: strength of connection on
// negative couplings relative to the row's largest, greedy three-phase
// aggregation, tentative prolongator from the near-nullspace vector (the
// constant in unscaled variables), one damped-Jacobi smoothing step on the
// strength-filtered operator, Galerkin product R A P with R = P^T, weak couplings
// of the product dropped (lumped into the diagonal, near-nullspace weighted), and
// a symmetric rescaling of the coarse operator to unit diagonal (absorbed into P
// and R).  Aggregates never cross the blocks of P_0 because P_0 has no
// couplings between them.  The coarsest level is solved with one dense FP64
// inverse per connected component.
//
// Apply (device): V-cycle with Chebyshev smoothing (a recurrence in x alone) of a
// chosen degree before and after the coarse correction, separately for the finest
// level (field-block kernels) and the coarser ones (block-streamed CSR); degree 0
// before restricts the right-hand side as it is.  Residual, restriction and
// prolongation are fused CSR kernels; FP64 or FP32 (FP32 accumulation); the
// coarsest solve is always FP64.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <numeric>
#include <type_traits>

#include "dense.h"
#include "knp_internal.h"

namespace knp {

namespace {

// A^T with each row's entries in ascending column order (the order a serial
// transpose writes them): the threads take contiguous row ranges of A, count their
// entries per column, and each writes its range after the earlier threads' entries.
Csr transpose(const Csr &A) {
    Csr T;
    T.nrows = A.ncols;
    T.ncols = A.nrows;
    T.rowptr.assign(T.nrows + 1, 0);
    const int64_t nnz = A.nnz();
    const int nt = std::max(1, std::min<int>(omp_get_max_threads(), int(A.nrows / 4096) + 1));
    std::vector<std::vector<int64_t>> cnt(nt);
    std::vector<int64_t> r0(nt + 1);
    for (int t = 0; t <= nt; ++t) r0[t] = A.nrows * t / nt;
#pragma omp parallel for num_threads(nt) schedule(static, 1)
    for (int t = 0; t < nt; ++t) {
        cnt[t].assign(T.nrows, 0);
        for (int64_t k = A.rowptr[r0[t]]; k < A.rowptr[r0[t + 1]]; ++k) cnt[t][A.col[k]]++;
    }
    // per column: the start of each thread's entries, and the row pointers
    int64_t run = 0;
    for (int64_t c = 0; c < T.nrows; ++c) {
        T.rowptr[c] = run;
        for (int t = 0; t < nt; ++t) {
            const int64_t k = cnt[t][c];
            cnt[t][c] = run;
            run += k;
        }
    }
    T.rowptr[T.nrows] = run;
    T.col.resize(nnz);
    T.val.resize(nnz);
#pragma omp parallel for num_threads(nt) schedule(static, 1)
    for (int t = 0; t < nt; ++t) {
        std::vector<int64_t> &fill = cnt[t];
        for (int64_t i = r0[t]; i < r0[t + 1]; ++i)
            for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
                const int64_t p = fill[A.col[k]]++;
                T.col[p] = int32_t(i);
                T.val[p] = A.val[k];
            }
    }
    return T;
}

// sum over i < n of f(i) in fixed chunks, the chunk sums added in order: the result does
// not depend on the number of threads
template <class F>
double det_sum(int64_t n, F f) {
    constexpr int64_t CH = int64_t(1) << 14;
    const int64_t nch = (n + CH - 1) / CH;
    std::vector<double> part(nch);
#pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < nch; ++c) {
        double acc = 0.0;
        const int64_t e = std::min(n, (c + 1) * CH);
        for (int64_t i = c * CH; i < e; ++i) acc += f(i);
        part[c] = acc;
    }
    double tot = 0.0;
    for (double v : part) tot += v;
    return tot;
}

// Drops the couplings of a coarse operator with |a_ij| < tol sqrt(a_ii a_jj) and
// adds a_ij b_j / b_i to a_ii (b the coarse near-nullspace vector), so that A b is
// unchanged; the criterion is symmetric, so the result stays symmetric.  If that
// would take any diagonal below half its value, the operator is left exact.
void sparsify(Csr &A, const std::vector<double> &b, double tol) {
    const int64_t n = A.nrows;
    std::vector<double> dg(n, 0.0), lump(n, 0.0);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
            if (A.col[k] == i) dg[i] = A.val[k];
    std::vector<char> keep(A.nnz());
    std::vector<int64_t> cnt(n + 1, 0);
    bool ok = true;
#pragma omp parallel for schedule(static) reduction(&& : ok)
    for (int64_t i = 0; i < n; ++i) {
        int64_t c = 0;
        for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) {
            const int32_t j = A.col[k];
            const bool kp = j == i || std::fabs(A.val[k]) >= tol * std::sqrt(std::fabs(dg[i] * dg[j]));
            keep[k] = kp;
            c += kp;
            if (!kp && b[i] != 0.0) lump[i] += A.val[k] * b[j] / b[i];
        }
        cnt[i + 1] = c;
        ok = ok && dg[i] + lump[i] >= 0.5 * dg[i];
    }
    if (!ok) return;
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    Csr K;
    K.nrows = A.nrows;
    K.ncols = A.ncols;
    K.rowptr.assign(cnt.begin(), cnt.end());
    K.col.resize(cnt[n]);
    K.val.resize(cnt[n]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t o = K.rowptr[i];
        for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
            if (keep[k]) {
                K.col[o] = A.col[k];
                K.val[o] = A.val[k] + (A.col[k] == i ? lump[i] : 0.0);
                ++o;
            }
    }
    A = std::move(K);
}

// C = A B, rows computed independently (deterministic: accumulation follows the
// order of A's row and B's rows); columns sorted per row.
Csr spgemm(const Csr &A, const Csr &B) {
    Csr C;
    C.nrows = A.nrows;
    C.ncols = B.ncols;
    C.rowptr.assign(A.nrows + 1, 0);
    const int nt = omp_get_max_threads();
    std::vector<std::vector<int64_t>> marks(nt);
#pragma omp parallel
    {
        std::vector<int64_t> &mk = marks[omp_get_thread_num()];
        mk.assign(B.ncols, -1);
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < A.nrows; ++i) {
            int64_t cnt = 0;
            for (int64_t ka = A.rowptr[i]; ka < A.rowptr[i + 1]; ++ka) {
                const int32_t j = A.col[ka];
                for (int64_t kb = B.rowptr[j]; kb < B.rowptr[j + 1]; ++kb) {
                    const int32_t c = B.col[kb];
                    if (mk[c] != i) {
                        mk[c] = i;
                        ++cnt;
                    }
                }
            }
            C.rowptr[i + 1] = cnt;
        }
    }
    for (int64_t i = 0; i < A.nrows; ++i) C.rowptr[i + 1] += C.rowptr[i];
    C.col.resize(C.rowptr[A.nrows]);
    C.val.resize(C.rowptr[A.nrows]);
#pragma omp parallel
    {
        std::vector<int64_t> pos(B.ncols, -1);
        std::vector<int32_t> cols;
        std::vector<double> acc(B.ncols, 0.0);
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < A.nrows; ++i) {
            cols.clear();
            for (int64_t ka = A.rowptr[i]; ka < A.rowptr[i + 1]; ++ka) {
                const int32_t j = A.col[ka];
                const double a = A.val[ka];
                for (int64_t kb = B.rowptr[j]; kb < B.rowptr[j + 1]; ++kb) {
                    const int32_t c = B.col[kb];
                    if (pos[c] != i) {
                        pos[c] = i;
                        acc[c] = 0.0;
                        cols.push_back(c);
                    }
                    acc[c] += a * B.val[kb];
                }
            }
            std::sort(cols.begin(), cols.end());
            int64_t o = C.rowptr[i];
            for (int32_t c : cols) {
                C.col[o] = c;
                C.val[o] = acc[c];
                ++o;
            }
        }
    }
    return C;
}

double gershgorin(const Csr &A) {
    double m = 0.0;
#pragma omp parallel for reduction(max : m)
    for (int64_t i = 0; i < A.nrows; ++i) {
        double s = 0.0;
        for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) s += std::fabs(A.val[k]);
        m = std::max(m, s);
    }
    return m;
}

// power iteration on a symmetric unit-diagonal operator (deterministic start and sums)
double power_lmax(const Csr &A, int iters) {
    const int64_t n = A.nrows;
    std::vector<double> x(n), y(n);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) x[i] = 1.0 + 0.5 * std::sin(0.7 * double(i) + 0.3);
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
        const double nx = std::sqrt(det_sum(n, [&](int64_t i) { return x[i] * x[i]; }));
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) x[i] /= nx;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double s = 0.0;
            for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k) s += A.val[k] * x[A.col[k]];
            y[i] = s;
        }
        lam = det_sum(n, [&](int64_t i) { return x[i] * y[i]; });
        std::swap(x, y);
    }
    return lam;
}

// strong(i, j): a_ij < 0 and -a_ij >= theta * max_k(-a_ik)
void strength(const Csr &A, double theta, std::vector<int64_t> &srow, std::vector<int32_t> &scol) {
    const int64_t n = A.nrows;
    srow.assign(n + 1, 0);
    std::vector<double> thr(n, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double m = 0.0;
        int64_t cnt = 0;
        for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
            if (A.col[k] != i) m = std::max(m, -A.val[k]);
        thr[i] = theta * m;
        if (m > 0.0)
            for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
                if (A.col[k] != i && -A.val[k] >= thr[i] && A.val[k] < 0.0) ++cnt;
        srow[i + 1] = cnt;
    }
    for (int64_t i = 0; i < n; ++i) srow[i + 1] += srow[i];
    scol.resize(srow[n]);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        int64_t o = srow[i];
        if (thr[i] > 0.0)
            for (int64_t k = A.rowptr[i]; k < A.rowptr[i + 1]; ++k)
                if (A.col[k] != i && -A.val[k] >= thr[i] && A.val[k] < 0.0) scol[o++] = A.col[k];
    }
}

// three-phase greedy aggregation; returns number of aggregates
int64_t aggregate(int64_t n, const std::vector<int64_t> &srow, const std::vector<int32_t> &scol,
                  std::vector<int32_t> &agg) {
    agg.assign(n, -1);
    int64_t na = 0;
    for (int64_t i = 0; i < n; ++i) {   // phase 1: root + all-free strong neighbourhood
        if (agg[i] >= 0) continue;
        bool free_nb = true;
        for (int64_t k = srow[i]; k < srow[i + 1]; ++k)
            if (agg[scol[k]] >= 0) {
                free_nb = false;
                break;
            }
        if (!free_nb || srow[i + 1] == srow[i]) continue;
        agg[i] = int32_t(na);
        for (int64_t k = srow[i]; k < srow[i + 1]; ++k) agg[scol[k]] = int32_t(na);
        ++na;
    }
    std::vector<int32_t> agg1 = agg;
    for (int64_t i = 0; i < n; ++i) {   // phase 2: join a neighbouring phase-1 aggregate
        if (agg[i] >= 0) continue;
        for (int64_t k = srow[i]; k < srow[i + 1]; ++k)
            if (agg1[scol[k]] >= 0) {
                agg[i] = agg1[scol[k]];
                break;
            }
    }
    for (int64_t i = 0; i < n; ++i) {   // phase 3: leftovers with their free neighbours
        if (agg[i] >= 0) continue;
        agg[i] = int32_t(na);
        for (int64_t k = srow[i]; k < srow[i + 1]; ++k)
            if (agg[scol[k]] < 0) agg[scol[k]] = int32_t(na);
        ++na;
    }
    return na;
}

struct HostLevel {
    Csr A, P, R;
    double lmax;
    std::vector<int8_t> blk;   // (region, field) block of each row: 4 r + f
};

}  // namespace

std::vector<int32_t> row_blocks(const int64_t *rowptr, int64_t nrows, int64_t cap) {
    std::vector<int32_t> b;
    b.push_back(0);
    int64_t r = 0;
    while (r < nrows) {
        const int64_t k0 = rowptr[r];
        int64_t e = r;
        while (e < nrows && rowptr[e + 1] - k0 <= cap && e - r < cap) ++e;
        if (e == r) throw Error{KNP_E_ARG, "a matrix row is longer than the streaming block capacity"};
        b.push_back(int32_t(e));
        r = e;
    }
    return b;
}

void DevCsr::upload(const Csr &h, bool fp32, hipStream_t s) {
    nrows = h.nrows;
    ncols = h.ncols;
    nnz = h.nnz();
    rowptr.alloc(h.rowptr.size());
    rowptr.upload(h.rowptr.data(), h.rowptr.size(), s);
    {
        std::vector<int32_t> b = row_blocks(h.rowptr.data(), h.nrows);
        nblk = int64_t(b.size()) - 1;
        blk.alloc(b.size());
        blk.upload(b, s);
    }
    // columns and values, then STREAM_PAD zeros after each
    const size_t nz = h.col.size();
    const int32_t zc[STREAM_PAD] = {};
    col.alloc(nz + STREAM_PAD);
    if (nz) hip_check(hipMemcpyAsync(col.p, h.col.data(), nz * sizeof(int32_t), hipMemcpyHostToDevice, s), "col");
    hip_check(hipMemcpyAsync(col.p + nz, zc, sizeof(zc), hipMemcpyHostToDevice, s), "col pad");
    if (fp32) {
        std::unique_ptr<float[]> v(new float[nz + STREAM_PAD]);
#pragma omp parallel for schedule(static)
        for (int64_t k = 0; k < int64_t(nz); ++k) v[k] = float(h.val[k]);
        for (int k = 0; k < STREAM_PAD; ++k) v[nz + k] = 0.0f;
        val32.alloc(nz + STREAM_PAD);
        val32.upload(v.get(), nz + STREAM_PAD, s);
        hip_check(hipStreamSynchronize(s), "upload");
    } else {
        const double zv[STREAM_PAD] = {};
        val64.alloc(nz + STREAM_PAD);
        if (nz) hip_check(hipMemcpyAsync(val64.p, h.val.data(), nz * sizeof(double), hipMemcpyHostToDevice, s), "val");
        hip_check(hipMemcpyAsync(val64.p + nz, zv, sizeof(zv), hipMemcpyHostToDevice, s), "val pad");
        hip_check(hipStreamSynchronize(s), "upload");
    }
    hip_check(hipStreamSynchronize(s), "upload");
}

Amg::~Amg() {
    clear();
    if (capture_stream) (void)hipStreamDestroy(capture_stream);
    capture_stream = nullptr;
}

void Amg::clear() {
    if (coarse_exec) (void)hipGraphExecDestroy(coarse_exec);
    coarse_exec = nullptr;
    coarse_out = nullptr;
    for (Level *l : levels) delete l;
    levels.clear();
    ready = false;
    level_nnz.clear();
    level_n.clear();
}

namespace {

// P_0 in the field-block layout: the entries of region r's scalar pattern once,
// each with its four field values.  p0_vals holds P_0 block by block: for region
// r and field f the region's scalar pattern in row order.
void upload_field_blocks(DevFieldBlock &fb, const HostMesh &m, const std::vector<double> &p0_vals, bool fp32,
                         hipStream_t s) {
    const int64_t nnz0 = m.prow[0][m.Nr[0]], nnz1 = m.prow[1][m.Nr[1]];
    fb.Ni = m.Nr[0];
    fb.Ne = m.Nr[1];
    fb.nv = fb.Ni + fb.Ne;
    fb.nnz = nnz0 + nnz1;
    std::vector<int64_t> rp(fb.nv + 1);
    for (int64_t j = 0; j <= fb.Ni; ++j) rp[j] = m.prow[0][j];
    for (int64_t j = 1; j <= fb.Ne; ++j) rp[fb.Ni + j] = nnz0 + m.prow[1][j];
    std::vector<int32_t> col(std::max<int64_t>(1, fb.nnz));
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nnz0; ++k) col[k] = m.pcol[0][k];
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nnz1; ++k) col[nnz0 + k] = m.pcol[1][k];
    // row blocks per region, region e's rows after region i's
    std::vector<int32_t> blk = row_blocks(m.prow[0].data(), fb.Ni, FB_CAP);
    {
        std::vector<int32_t> be = row_blocks(m.prow[1].data(), fb.Ne, FB_CAP);
        for (size_t q = 1; q < be.size(); ++q) blk.push_back(int32_t(fb.Ni + be[q]));
    }
    fb.nblk = int64_t(blk.size()) - 1;
    // the four field values of each entry side by side, in the level's precision
    const size_t nv = size_t(std::max<int64_t>(4, 4 * fb.nnz));
    const int64_t pbase[2] = {0, 4 * nnz0}, nnzr[2] = {nnz0, nnz1}, kbase[2] = {0, nnz0};
    auto fill = [&](auto *v) {
        for (int r = 0; r < 2; ++r)
#pragma omp parallel for schedule(static)
            for (int64_t k = 0; k < nnzr[r]; ++k)
                for (int f = 0; f < 4; ++f)
                    v[4 * (kbase[r] + k) + f] = decltype(+v[0])(p0_vals[pbase[r] + f * nnzr[r] + k]);
        for (size_t k = size_t(4 * fb.nnz); k < nv; ++k) v[k] = 0;
    };
    fb.rowptr.alloc(rp.size());
    fb.rowptr.upload(rp, s);
    fb.col.alloc(col.size());
    fb.col.upload(col, s);
    fb.blk.alloc(blk.size());
    fb.blk.upload(blk, s);
    if (fp32) {
        std::unique_ptr<float[]> v(new float[nv]);
        fill(v.get());
        fb.val32.alloc(nv);
        fb.val32.upload(v.get(), nv, s);
        hip_check(hipStreamSynchronize(s), "field-block upload");
    } else {
        std::unique_ptr<double[]> v(new double[nv]);
        fill(v.get());
        fb.val64.alloc(nv);
        fb.val64.upload(v.get(), nv, s);
        hip_check(hipStreamSynchronize(s), "field-block upload");
    }
}

}  // namespace

void amg_build(Amg &amg, const HostMesh &m, const std::vector<double> &p0_vals, const std::vector<double> &near_null,
               const knp_amg_opts &o, hipStream_t s) {
    amg.clear();
    amg.fp32 = o.precision == 1;
    amg.degree = std::max(1, o.cheb_degree);
    amg.pre_degree = std::max(0, o.cheb_pre_degree);
    amg.coarse_pre = std::max(0, o.coarse_pre_degree);
    amg.coarse_post = std::max(1, o.coarse_post_degree);
    amg.ratio = o.cheb_ratio;
    amg.field_split = o.field_split == 1;
    amg.coarse_graph = o.coarse_graph == 1;
    // P_0 in CSR, in the solver's order (DOF off_r + 4 j + f): per region the scalar
    // pattern of the region for each field.  p0_vals and near_null come in ABI order
    // (block by block: region r, field f, then the pattern row by row).
    Csr A;
    A.nrows = A.ncols = m.N;
    A.rowptr.assign(m.N + 1, 0);
    for (int r = 0; r < 2; ++r)
        for (int64_t j = 0; j < m.Nr[r]; ++j)
            for (int f = 0; f < 4; ++f) A.rowptr[m.off[r] + 4 * j + f + 1] = m.prow[r][j + 1] - m.prow[r][j];
    for (int64_t i = 0; i < m.N; ++i) A.rowptr[i + 1] += A.rowptr[i];
    A.col.resize(A.rowptr[m.N]);
    A.val.resize(A.rowptr[m.N]);
    std::vector<double> B(m.N);
    {
        const int64_t nnz0 = m.prow[0][m.Nr[0]], nnz1 = m.prow[1][m.Nr[1]];
        const int64_t pbase[2] = {0, 4 * nnz0}, nnzr[2] = {nnz0, nnz1};
        for (int r = 0; r < 2; ++r) {
#pragma omp parallel for schedule(static)
            for (int64_t j = 0; j < m.Nr[r]; ++j)
                for (int f = 0; f < 4; ++f) {
                    const int64_t i = m.off[r] + 4 * j + f;
                    int64_t o2 = A.rowptr[i];
                    for (int64_t k = m.prow[r][j]; k < m.prow[r][j + 1]; ++k, ++o2) {
                        A.col[o2] = int32_t(m.off[r] + 4 * int64_t(m.pcol[r][k]) + f);
                        A.val[o2] = p0_vals[pbase[r] + f * nnzr[r] + k];
                    }
                    B[i] = near_null[m.off[r] + f * m.Nr[r] + j];
                }
        }
    }

    std::vector<HostLevel> H;
    // block of each row, carried to the coarser levels (aggregates never leave a block)
    std::vector<int8_t> RB(m.N);
    for (int64_t i = 0; i < m.N; ++i) RB[i] = int8_t((i >= m.off[1] ? 4 : 0) + (i & 3));
    const int max_levels = std::max(1, o.max_levels);
    const int64_t coarse_max = std::max<int32_t>(1, o.coarse_max);
    while (true) {
        HostLevel L;
        L.A = std::move(A);
        const int64_t n = L.A.nrows;
        if (n <= coarse_max || int(H.size()) + 1 >= max_levels) {
            L.blk = RB;
            H.push_back(std::move(L));
            break;
        }
        std::vector<int64_t> srow;
        std::vector<int32_t> scol;
        strength(L.A, o.strength, srow, scol);
        std::vector<int32_t> agg;
        int64_t nc = aggregate(n, srow, scol, agg);
        if (H.empty() && o.shared_ion_aggregates == 1) {
            // the Na+ and Cl- blocks of each region take the aggregates of its K+ block
            // (the three ion blocks share their pattern and differ by tau_k only); the
            // aggregates they had are dropped and the rest renumbered in order
            std::vector<int64_t> id(size_t(3) * size_t(nc), -1);
            for (int r = 0; r < 2; ++r)
                for (int64_t j = 0; j < m.Nr[r]; ++j) {
                    const int64_t base = m.off[r] + 4 * j;
                    agg[base + 0] = int32_t(agg[base + 1] + nc);
                    agg[base + 2] = int32_t(agg[base + 1] + 2 * nc);
                }
            int64_t c = 0;
            for (int64_t i = 0; i < n; ++i) {
                int64_t &t = id[size_t(agg[i])];
                if (t < 0) t = c++;
            }
            for (int64_t i = 0; i < n; ++i) agg[i] = int32_t(id[size_t(agg[i])]);
            nc = c;
        }
        if (double(nc) > 0.85 * double(n)) {   // coarsening stalled: make this the coarsest
            L.blk = RB;
            H.push_back(std::move(L));
            break;
        }
        if (H.empty()) {
            // Level 0 is in the solver's order (fields side by side), but P_0 couples no
            // two fields, so each aggregate lies in one (region, field) block.  Number
            // the aggregates block by block, keeping their order within a block, so
            // that every coarser level has each field's unknowns contiguous.
            std::vector<int32_t> blk_of(nc, 0);
            for (int64_t i = 0; i < n; ++i) blk_of[agg[i]] = int32_t((i >= m.off[1] ? 4 : 0) + (i & 3));
            std::vector<int64_t> start(9, 0);
            for (int64_t c = 0; c < nc; ++c) start[blk_of[c] + 1]++;
            for (int q = 0; q < 8; ++q) start[q + 1] += start[q];
            std::vector<int32_t> renum(nc);
            for (int64_t c = 0; c < nc; ++c) renum[c] = int32_t(start[blk_of[c]]++);
            for (int64_t i = 0; i < n; ++i) agg[i] = renum[agg[i]];
        }
        // tentative prolongator from B
        std::vector<double> bn(nc, 0.0);
        for (int64_t i = 0; i < n; ++i) bn[agg[i]] += B[i] * B[i];
        for (int64_t c = 0; c < nc; ++c) bn[c] = std::sqrt(bn[c]);
        Csr T;
        T.nrows = n;
        T.ncols = nc;
        T.rowptr.resize(n + 1);
        T.col.resize(n);
        T.val.resize(n);
        for (int64_t i = 0; i < n; ++i) {
            T.rowptr[i] = i;
            T.col[i] = agg[i];
            T.val[i] = bn[agg[i]] > 0.0 ? B[i] / bn[agg[i]] : 1.0;
        }
        T.rowptr[n] = n;
        // filtered operator: diagonal + strong couplings, weak couplings lumped (B-weighted)
        Csr AF;
        AF.nrows = AF.ncols = n;
        AF.rowptr.assign(n + 1, 0);
        for (int64_t i = 0; i < n; ++i) AF.rowptr[i + 1] = AF.rowptr[i] + 1 + (srow[i + 1] - srow[i]);
        AF.col.resize(AF.rowptr[n]);
        AF.val.resize(AF.rowptr[n]);
#pragma omp parallel
        {
        std::vector<std::pair<int32_t, double>> e;
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double diag = 0.0, lump = 0.0;
            int64_t ks = srow[i];
            e.clear();
            for (int64_t k = L.A.rowptr[i]; k < L.A.rowptr[i + 1]; ++k) {
                const int32_t j = L.A.col[k];
                if (j == i) {
                    diag = L.A.val[k];
                } else if (ks < srow[i + 1] && scol[ks] == j) {
                    e.push_back({j, L.A.val[k]});
                    ++ks;
                } else if (B[i] != 0.0) {
                    lump += L.A.val[k] * B[j] / B[i];
                }
            }
            double dF = diag + lump;
            if (!(dF > 0.0)) dF = diag;
            e.push_back({int32_t(i), dF});
            std::sort(e.begin(), e.end());
            int64_t oo = AF.rowptr[i];
            for (auto &pr : e) {
                AF.col[oo] = pr.first;
                AF.val[oo] = pr.second;
                ++oo;
            }
        }
        }
        // omega / rho(D_F^{-1} A_F) with a Gershgorin bound
        double rho = 0.0;
#pragma omp parallel for reduction(max : rho)
        for (int64_t i = 0; i < n; ++i) {
            double d = 0.0, sabs = 0.0;
            for (int64_t k = AF.rowptr[i]; k < AF.rowptr[i + 1]; ++k) {
                sabs += std::fabs(AF.val[k]);
                if (AF.col[k] == i) d = AF.val[k];
            }
            if (d > 0.0) rho = std::max(rho, sabs / d);
        }
        const double omega = rho > 0.0 ? 4.0 / (3.0 * rho) : 0.0;
        // P = (I - omega D_F^{-1} A_F) T
        Csr DA = AF;
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; ++i) {
            double d = 1.0;
            for (int64_t k = AF.rowptr[i]; k < AF.rowptr[i + 1]; ++k)
                if (AF.col[k] == i) d = AF.val[k];
            for (int64_t k = DA.rowptr[i]; k < DA.rowptr[i + 1]; ++k) {
                DA.val[k] = -omega * AF.val[k] / d;
                if (DA.col[k] == i) DA.val[k] += 1.0;
            }
        }
        Csr P = spgemm(DA, T);
        // release each intermediate once consumed (at ~1e8 unknowns each is 10-70 GB)
        AF = Csr();
        DA = Csr();
        T = Csr();
        std::vector<int64_t>().swap(srow);
        std::vector<int32_t>().swap(scol);
        Csr R = transpose(P);
        Csr Ac;
        {
            Csr AP = spgemm(L.A, P);
            Ac = spgemm(R, AP);
        }
        if (o.coarse_drop > 0.0) sparsify(Ac, bn, o.coarse_drop);
        // unit diagonal on the coarse level, absorbed into P and R
        std::vector<double> dc(nc, 1.0);
        for (int64_t c = 0; c < nc; ++c)
            for (int64_t k = Ac.rowptr[c]; k < Ac.rowptr[c + 1]; ++k)
                if (Ac.col[k] == c) dc[c] = Ac.val[k] > 0.0 ? 1.0 / std::sqrt(Ac.val[k]) : 1.0;
#pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < nc; ++c)
            for (int64_t k = Ac.rowptr[c]; k < Ac.rowptr[c + 1]; ++k) Ac.val[k] *= dc[c] * dc[Ac.col[k]];
        for (int64_t k = 0; k < P.nnz(); ++k) P.val[k] *= dc[P.col[k]];
        for (int64_t c = 0; c < nc; ++c)
            for (int64_t k = R.rowptr[c]; k < R.rowptr[c + 1]; ++k) R.val[k] *= dc[c];
        std::vector<double> Bc(nc);
        for (int64_t c = 0; c < nc; ++c) Bc[c] = bn[c] / dc[c];
        L.P = std::move(P);
        L.R = std::move(R);
        {
            std::vector<int8_t> RBc(nc, 0);
            for (int64_t i = 0; i < n; ++i) RBc[agg[i]] = RB[i];
            L.blk.swap(RB);
            RB.swap(RBc);
        }
        H.push_back(std::move(L));
        A = std::move(Ac);
        B.swap(Bc);
    }

    // spectral bounds for Chebyshev: on the finest level a power estimate (x1.1,
    // capped by Gershgorin); on the coarser levels the Gershgorin bound itself,
    // since there 20 power steps undershot the top of the spectrum and the
    // smoother then amplified the modes above its interval (one GMRES iteration
    // per step more on the 132^3 lattice)
    for (size_t l = 0; l < H.size(); ++l) {
        HostLevel &L = H[l];
        const double g = gershgorin(L.A);
        if (l > 0) {
            L.lmax = g;
            continue;
        }
        const double pw = L.A.nrows > 1 ? 1.1 * power_lmax(L.A, 20) : g;
        L.lmax = std::min(g, std::max(pw, 1e-12));
    }

    // coarsest level: connected components, dense inverses
    const Csr &C = H.back().A;
    const int64_t nC = C.nrows;
    std::vector<int32_t> comp(nC, -1);
    std::vector<int64_t> order;
    order.reserve(nC);
    std::vector<int64_t> cstart;
    int32_t ncomp = 0;
    for (int64_t i = 0; i < nC; ++i) {
        if (comp[i] >= 0) continue;
        cstart.push_back(int64_t(order.size()));
        size_t head = order.size();
        comp[i] = ncomp;
        order.push_back(i);
        while (head < order.size()) {
            const int64_t v = order[head++];
            for (int64_t k = C.rowptr[v]; k < C.rowptr[v + 1]; ++k) {
                const int32_t w = C.col[k];
                if (comp[w] < 0) {
                    comp[w] = ncomp;
                    order.push_back(w);
                }
            }
        }
        ++ncomp;
    }
    cstart.push_back(nC);
    // component members in ascending row order; position of each row inside its component
    for (int32_t c = 0; c < ncomp; ++c) std::sort(order.begin() + cstart[c], order.begin() + cstart[c + 1]);
    std::vector<int32_t> cloc(nC), cmem(nC);
    for (int32_t c = 0; c < ncomp; ++c)
        for (int64_t p = cstart[c]; p < cstart[c + 1]; ++p) {
            cmem[p] = int32_t(order[p]);
            cloc[order[p]] = int32_t(p - cstart[c]);
        }
    std::vector<int64_t> boff(ncomp);
    int64_t tot = 0;
    for (int32_t c = 0; c < ncomp; ++c) {
        const int64_t nb = cstart[c + 1] - cstart[c];
        if (nb > 4096) throw Error{KNP_E_NOMEM, "coarsest-level component too large for a dense inverse"};
        boff[c] = tot;
        tot += nb * nb;
    }
    std::vector<double> inv(std::max<int64_t>(1, tot), 0.0);
    // no exception may leave the parallel region: failures are flagged per component
    std::vector<char> singular(ncomp, 0);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < ncomp; ++c) {
        const int64_t s0 = cstart[c], nb = cstart[c + 1] - s0;
        std::vector<double> a(size_t(nb) * nb, 0.0);
        for (int64_t p = 0; p < nb; ++p) {
            const int64_t v = order[s0 + p];
            for (int64_t k = C.rowptr[v]; k < C.rowptr[v + 1]; ++k) a[size_t(p) * nb + cloc[C.col[k]]] = C.val[k];
        }
        if (!invert_dense(int(nb), a)) {
            singular[c] = 1;
            continue;
        }
        std::copy(a.begin(), a.end(), inv.begin() + boff[c]);
    }
    for (int32_t c = 0; c < ncomp; ++c)
        if (singular[c])
            throw Error{KNP_E_NUMERIC, "singular coarsest-level block (component " + std::to_string(c) + " of " +
                                           std::to_string(ncomp) + ", " +
                                           std::to_string(cstart[c + 1] - cstart[c]) + " rows)"};

    // upload
    const bool f32 = amg.fp32;
    for (size_t l = 0; l < H.size(); ++l) {
        Level *L = new Level();
        amg.levels.push_back(L);
        L->n = H[l].A.nrows;
        L->lmax = H[l].lmax;
        amg.level_n.push_back(L->n);
        amg.level_nnz.push_back(H[l].A.nnz());
        const bool last = l + 1 == H.size();
        if (!last) {
            if (l == 0) {
                upload_field_blocks(L->fb, m, p0_vals, f32, s);
                // level 0's residual reaches the restriction field-major
                for (auto &cidx : H[0].R.col) {
                    const int64_t i = cidx;
                    const int r = i >= m.off[1] ? 1 : 0;
                    const int64_t q = i - m.off[r];
                    cidx = int32_t(m.off[r] + (q & 3) * m.Nr[r] + (q >> 2));
                }
            } else {
                L->A.upload(H[l].A, f32, s);
                // field split: block row ranges (contiguous on the coarser levels, since
                // level 1 numbers its aggregates block by block and aggregation keeps the
                // order) and a Gershgorin bound per block
                const std::vector<int8_t> &rb = H[l].blk;
                const int64_t nl = H[l].A.nrows;
                bool ok = int64_t(rb.size()) == nl && nl < (int64_t(1) << 31);
                for (int64_t i = 1; ok && i < nl; ++i) ok = rb[i] >= rb[i - 1];
                if (ok) {
                    L->nblocks = CHEB_BLOCKS;
                    for (int q = 0; q <= CHEB_BLOCKS; ++q)
                        L->bstart[q] = int32_t(std::lower_bound(rb.begin(), rb.end(), int8_t(q)) - rb.begin());
                    for (int q = 0; q < CHEB_BLOCKS; ++q) {
                        double g = 0.0;
                        for (int64_t i = L->bstart[q]; i < L->bstart[q + 1]; ++i) {
                            double sabs = 0.0;
                            for (int64_t k = H[l].A.rowptr[i]; k < H[l].A.rowptr[i + 1]; ++k)
                                sabs += std::fabs(H[l].A.val[k]);
                            g = std::max(g, sabs);
                        }
                        L->blmax[q] = g > 0.0 ? g : H[l].lmax;
                    }
                }
            }
            L->P.upload(H[l].P, f32, s);
            L->R.upload(H[l].R, f32, s);
        }
        const size_t n = size_t(std::max<int64_t>(1, L->n));
        if (f32) {
            L->b32.alloc(n);
            L->x32.alloc(n);
            L->t32.alloc(n);
            L->d32.alloc(n);
            L->x2_32.alloc(n);
        } else {
            L->b64.alloc(n);
            L->x64.alloc(n);
            L->t64.alloc(n);
            L->d64.alloc(n);
            L->x2_64.alloc(n);
        }
    }
    amg.n_coarse = nC;
    amg.n_blocks = ncomp;
    amg.ccomp.alloc(std::max<int64_t>(1, nC));
    amg.ccomp.upload(comp, s);
    amg.cloc.alloc(std::max<int64_t>(1, nC));
    amg.cloc.upload(cloc, s);
    amg.cmem.alloc(std::max<int64_t>(1, nC));
    amg.cmem.upload(cmem, s);
    amg.cstart.alloc(cstart.size());
    amg.cstart.upload(cstart, s);
    amg.coff.alloc(std::max<size_t>(1, boff.size()));
    amg.coff.upload(boff, s);
    amg.cinv.alloc(inv.size());
    amg.cinv.upload(inv, s);
    amg.cb64.alloc(std::max<int64_t>(1, nC));
    amg.cx64.alloc(std::max<int64_t>(1, nC));
    hip_check(hipStreamSynchronize(s), "amg upload");
    // algorithmic bytes of one V-cycle: every matrix and vector each of its kernels
    // touches, once per kernel
    {
        const double vb = amg.fp32 ? 4.0 : 8.0;
        auto csr = [&](const DevCsr &M) { return double(M.nnz) * (vb + 4.0) + 8.0 * double(M.nrows + 1); };
        double bytes = amg.fp32 ? 12.0 * double(amg.levels[0]->n) : 0.0;   // FP64 input to FP32
        for (size_t l = 0; l + 1 < amg.levels.size(); ++l) {
            const Level *L = amg.levels[l];
            const double n = double(L->n), nc = double(amg.levels[l + 1]->n);
            const double mat = l == 0 ? double(L->fb.nnz) * (4.0 * vb + 4.0) + 8.0 * double(L->fb.nv + 1) : csr(L->A);
            const int dpre = l == 0 ? amg.pre_degree : amg.coarse_pre;
            const int dpost = l == 0 ? amg.degree : amg.coarse_post;
            if (dpre > 0) {
                bytes += 2.0 * vb * n;                                      // first step from x = 0
                for (int k = 1; k < dpre; ++k) bytes += mat + 4.0 * vb * n;
                bytes += mat + 3.0 * vb * n;                                // residual
            } else if (l == 0) {
                bytes += 2.0 * vb * n;                                      // b to field-major order
            }
            bytes += csr(L->R) + vb * (n + nc);                             // restriction
            bytes += csr(L->P) + vb * (nc + n) + (dpre > 0 ? vb * n : 0.0); // prolongation (+ x read)
            bytes += mat + 3.0 * vb * n;                                    // post-smoothing, c1 = 0
            for (int k = 1; k < dpost; ++k) bytes += mat + 4.0 * vb * n;
        }
        const double ncst = double(nC);
        bytes += 8.0 * double(tot) + 16.0 * ncst;                           // dense coarsest solve
        if (amg.fp32) bytes += 24.0 * ncst;                                 // its FP32 <-> FP64 copies
        amg.vcycle_bytes = bytes;
    }
    amg.ready = true;
}

namespace {

// Chebyshev coefficients (c1, c2) of the three-term recurrence for the interval
// [lmax/ratio, lmax]:  x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 (b - A x_k); c1 = 0 in
// the first step.
void cheb_coeffs(double lmax, double ratio, int degree, std::vector<std::pair<double, double>> &out) {
    const double a = lmax / ratio, b = lmax;
    const double theta = 0.5 * (b + a), delta = 0.5 * (b - a), sigma = theta / delta;
    double rho = 1.0 / sigma;
    out.clear();
    out.push_back({0.0, 1.0 / theta});
    for (int k = 1; k < degree; ++k) {
        const double rn = 1.0 / (2.0 * sigma - rho);
        out.push_back({rn * rho, 2.0 * rn / delta});
        rho = rn;
    }
}

template <typename T>
struct LV;
template <>
struct LV<double> {
    static double *b(Level *L) { return L->b64.p; }
    static double *x(Level *L) { return L->x64.p; }
    static double *x2(Level *L) { return L->x2_64.p; }
    static double *t(Level *L) { return L->t64.p; }
    static double *d(Level *L) { return L->d64.p; }
    static const double *A(Level *L) { return L->A.val64.p; }
    static const double *FB(Level *L) { return L->fb.val64.p; }
    static const double *P(Level *L) { return L->P.val64.p; }
    static const double *R(Level *L) { return L->R.val64.p; }
};
template <>
struct LV<float> {
    static float *b(Level *L) { return L->b32.p; }
    static float *x(Level *L) { return L->x32.p; }
    static float *x2(Level *L) { return L->x2_32.p; }
    static float *t(Level *L) { return L->t32.p; }
    static float *d(Level *L) { return L->d32.p; }
    static const float *A(Level *L) { return L->A.val32.p; }
    static const float *FB(Level *L) { return L->fb.val32.p; }
    static const float *P(Level *L) { return L->P.val32.p; }
    static const float *R(Level *L) { return L->R.val32.p; }
};

template <typename T>
T *vcycle_level(Amg &amg, size_t l, const T *b, hipStream_t s, Timers *tm, T *out = nullptr);

// The levels below the finest, from level 1's right-hand side bc (a level-1 buffer):
// launched one by one, or as the HIP graph of those launches (captured on the first call
// after a setup).  No timer event is recorded below the finest level, and these levels
// issue kernels only, so the capture holds the same work.
template <typename T>
T *coarse_cycle(Amg &amg, const T *bc, hipStream_t s, Timers *tm) {
    if (!amg.coarse_graph) return vcycle_level<T>(amg, 1, bc, s, tm);
    if (!amg.coarse_exec) {
        if (!amg.capture_stream)
            hip_check(hipStreamCreateWithFlags(&amg.capture_stream, hipStreamNonBlocking), "capture stream");
        hipStream_t cs = amg.capture_stream;
        hip_check(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "begin capture");
        T *xc = nullptr;
        hipGraph_t g = nullptr;
        try {
            xc = vcycle_level<T>(amg, 1, bc, cs, nullptr);
        } catch (...) {
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            throw;
        }
        hip_check(hipStreamEndCapture(cs, &g), "end capture");
        const hipError_t e = hipGraphInstantiate(&amg.coarse_exec, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        hip_check(e, "instantiate the coarse-level graph");
        amg.coarse_out = xc;
    }
    hip_check(hipGraphLaunch(amg.coarse_exec, s), "coarse-level graph");
    return static_cast<T *>(amg.coarse_out);
}

// V-cycle on level l: solves approximately A_l x = b, with b and the result in
// the level's own buffers; returns the buffer holding x.
template <typename T>
T *vcycle_level(Amg &amg, size_t l, const T *b, hipStream_t s, Timers *tm, T *out) {
    Level *L = amg.levels[l];
    if (l + 1 == amg.levels.size()) {
        T *x = LV<T>::x(L);
        if constexpr (std::is_same<T, double>::value) {
            launch::coarse_solve(amg.n_coarse, amg.ccomp.p, amg.cloc.p, amg.cmem.p, amg.cstart.p, amg.coff.p, amg.cinv.p, b, x, s);
        } else {
            launch::convert<float, double>(amg.n_coarse, b, amg.cb64.p, s);
            launch::coarse_solve(amg.n_coarse, amg.ccomp.p, amg.cloc.p, amg.cmem.p, amg.cstart.p, amg.coff.p,
                                 amg.cinv.p, amg.cb64.p, amg.cx64.p, s);
            launch::convert<double, float>(amg.n_coarse, amg.cx64.p, x, s);
        }
        return x;
    }
    // smoothing degrees: the finest level pre/post, the coarser levels their own
    const int dpre = l == 0 ? amg.pre_degree : amg.coarse_pre;
    const int dpost = l == 0 ? amg.degree : amg.coarse_post;
    std::vector<std::pair<double, double>> cpre, cc;
    if (dpre > 0) cheb_coeffs(L->lmax, amg.ratio, dpre, cpre);
    cheb_coeffs(L->lmax, amg.ratio, dpost, cc);
    // field split: the same recurrences on each block's own interval
    const bool fs = amg.field_split && l > 0 && L->nblocks == CHEB_BLOCKS;
    std::vector<std::pair<double, double>> bpre[CHEB_BLOCKS], bcc[CHEB_BLOCKS];
    if (fs)
        for (int q = 0; q < CHEB_BLOCKS; ++q) {
            if (dpre > 0) cheb_coeffs(L->blmax[q], amg.ratio, dpre, bpre[q]);
            cheb_coeffs(L->blmax[q], amg.ratio, dpost, bcc[q]);
        }
    auto blocks_at = [&](const std::vector<std::pair<double, double>> (&tab)[CHEB_BLOCKS], size_t k) {
        launch::ChebBlocks cb{};
        cb.nb = CHEB_BLOCKS;
        for (int q = 0; q <= CHEB_BLOCKS; ++q) cb.start[q] = L->bstart[q];
        for (int q = 0; q < CHEB_BLOCKS; ++q) {
            cb.c1[q] = tab[q][k].first;
            cb.c2[q] = tab[q][k].second;
        }
        return cb;
    };
    const int64_t n = L->n;
    const bool fbl = l == 0;     // level 0 is P_0 in the field-block layout
    const T *av = fbl ? LV<T>::FB(L) : LV<T>::A(L);
    T *t = LV<T>::t(L);
    // the Chebyshev recurrence in x alone (x_{k+1} from x_k and x_{k-1}) rotates three
    // buffers; cur = x_k and prev = x_{k-1}, null standing for the zero vector
    T *const buf[3] = {LV<T>::x(L), LV<T>::x2(L), LV<T>::d(L)};
    T *cur = nullptr, *prev = nullptr;
    auto spare = [&]() -> T * {
        for (T *p : buf)
            if (p != cur && p != prev) return p;
        return nullptr;   // unreachable: three buffers, two in use
    };
    // algorithmic bytes: values + column indices once, row pointers, each vector once
    const double vb = double(sizeof(T));
    const double mat = fbl ? double(L->fb.nnz) * (4.0 * vb + 4.0) + 8.0 * double(L->fb.nv + 1)
                           : double(L->A.nnz) * (vb + 4.0) + 8.0 * double(n + 1);
    Timers *t0 = (l == 0) ? tm : nullptr;
    // the finest level's timer class holds the steps that apply the operator (the
    // first step from x = 0 is a plain vector update)
    auto cheb = [&](T *xout, double c1, double c2, const launch::ChebBlocks *cbk = nullptr) {
        Timers *tc = cur ? t0 : nullptr;
        hipEvent_t e = tc ? tc->begin(KNP_TIMER_CHEB_L0, s) : nullptr;
        if (fbl)
            launch::fb_cheb_step<T>(L->fb.view(), av, cur, b, prev, xout, c1, c2, s);
        else if (cbk)
            launch::cheb_step_blocks<T>(L->A.view(), av, cur, b, prev, xout, *cbk, s);
        else
            launch::cheb_step<T>(L->A.view(), av, cur, b, prev, xout, c1, c2, s);
        // b, x_k (gathered and own rows), x_{k-1} when c1 != 0, x_{k+1}
        if (tc) tc->end(KNP_TIMER_CHEB_L0, e, mat + vb * double(n) * (c1 != 0.0 ? 4.0 : 3.0), s);
        prev = cur;
        cur = xout;
    };
    Level *Lc = amg.levels[l + 1];
    T *bc = LV<T>::b(Lc);
    if (dpre > 0) {
        // pre-smoothing from x = 0, residual, restriction
        for (size_t k = 0; k < cpre.size(); ++k) {
            const launch::ChebBlocks cb = fs ? blocks_at(bpre, k) : launch::ChebBlocks{};
            cheb(spare(), cpre[k].first, cpre[k].second, fs ? &cb : nullptr);
        }
        hipEvent_t e = t0 ? t0->begin(KNP_TIMER_RESID_L0, s) : nullptr;
        if (fbl)
            launch::fb_residual<T>(L->fb.view(), av, cur, b, t, s);
        else
            launch::residual<T>(L->A.view(), av, cur, b, t, s);
        if (t0) t0->end(KNP_TIMER_RESID_L0, e, mat + 3.0 * vb * double(n), s);
        launch::spmv<T, T, T>(L->R.view(), LV<T>::R(L), t, bc, s);
    } else {
        // no pre-smoothing: x = 0, so the residual is b itself (on level 0 taken to
        // field-major order, the restriction's column order there)
        if (fbl) {
            launch::to_field_major<T>(L->fb.view(), b, t, s);
            launch::spmv<T, T, T>(L->R.view(), LV<T>::R(L), t, bc, s);
        } else {
            launch::spmv<T, T, T>(L->R.view(), LV<T>::R(L), b, bc, s);
        }
    }
    T *xc = l == 0 ? coarse_cycle<T>(amg, bc, s, tm) : vcycle_level<T>(amg, l + 1, bc, s, tm);
    if (dpre > 0) {
        launch::prolong_add<T>(L->P.view(), LV<T>::P(L), xc, cur, s);
    } else {
        cur = spare();
        launch::spmv<T, T, T>(L->P.view(), LV<T>::P(L), xc, cur, s);   // x = P xc
    }
    // post-smoothing, a recurrence of its own (its first step has c1 = 0); the last
    // step writes to `out` when given
    prev = nullptr;
    for (size_t k = 0; k < cc.size(); ++k) {
        const launch::ChebBlocks cb = fs ? blocks_at(bcc, k) : launch::ChebBlocks{};
        cheb((out && k + 1 == cc.size()) ? out : spare(), cc[k].first, cc[k].second, fs ? &cb : nullptr);
    }
    return cur;
}

}  // namespace

void amg_vcycle(Amg &amg, const double *v, void *z, hipStream_t s, Timers *tm) {
    Level *L0 = amg.levels[0];
    const int64_t n = L0->n;
    hipEvent_t e = tm ? tm->begin(KNP_TIMER_VCYCLE, s) : nullptr;
    if (amg.fp32) {
        launch::convert<double, float>(n, v, L0->b32.p, s);
        float *zf = static_cast<float *>(z);
        float *x = vcycle_level<float>(amg, 0, L0->b32.p, s, tm, zf);
        if (x != zf) hip_check(hipMemcpyAsync(z, x, size_t(n) * sizeof(float), hipMemcpyDeviceToDevice, s), "copy");
    } else {
        double *zd = static_cast<double *>(z);
        double *x = vcycle_level<double>(amg, 0, v, s, tm, zd);
        if (x != zd) hip_check(hipMemcpyAsync(z, x, size_t(n) * sizeof(double), hipMemcpyDeviceToDevice, s), "copy");
    }
    if (tm) tm->end(KNP_TIMER_VCYCLE, e, amg.vcycle_bytes, s);
}

}  // namespace knp
