// Flexible GMRES(m) with classical Gram-Schmidt for A_{n-1} u_n = f_n and for
// the adjoint system, preconditioned on the right by one AMG V-cycle on P_0
// (Sec. "Solution and preconditioning strategy"; restart 30 and the previous
// step as initial guess, Sec. "Solver configurations").
//
// The iteration runs on the symmetrically scaled system (S A S) y = S b,
// x = S y, S = diag(P_0)^{-1/2}; its stopping test is ||S(b - A x)|| <= rtol ||S b||.
// Right preconditioning keeps the true residual available and lets the
// preconditioner vary between iterations, so the same recurrence serves the
// FP64 and the FP32 V-cycle.  Arnoldi, the Hessenberg least-squares problem,
// the solution update and the true-residual recomputation are FP64.
// One device-to-host copy of the new Hessenberg column per iteration.
//
// With gauge 1 the system carries no point condition and keeps the constant
// potential as its null vector (consistent right-hand side); the forward solve
// then applies, at the start of every cycle, the per-cell coarse correction of
// nullspace.hip to the iterate and its residual, so that the stopping test sees the
// corrected residual, and at return shifts every potential so that the reference
// extracellular DOF is zero: the solution of the point-condition system.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "ctx.h"

namespace knp {

namespace {

void ensure_pinned(knp_ctx *c, size_t count) {
    if (c->hbuf.n < count) c->hbuf.alloc(std::max<size_t>(count, 256));
}

void ensure_workspace(knp_ctx *c, int m, bool z32) {
    const int64_t N = c->hm.N;
    if (c->m_alloc >= m && c->z32 == z32) return;
    c->V.release();
    c->Z64.release();
    c->Z32.release();
    c->V.alloc(size_t(m + 1) * N);
    if (z32)
        c->Z32.alloc(size_t(m) * N);
    else
        c->Z64.alloc(size_t(m) * N);
    c->dscal.release();
    c->dscal.alloc(2 * size_t(m) + 64);
    ensure_pinned(c, 2 * size_t(m) + 8);
    c->m_alloc = m;
    c->z32 = z32;
}

// gauge 1: 1/S on each cell's intracellular potential DOFs (once; S is fixed at the
// first assembly), then W = S A S u and E for the current system (after every assembly)
void gauge_refresh(knp_ctx *c) {
    const int64_t N = c->hm.N;
    hipStream_t s = c->stream;
    if (!c->ns_basis) {
        const int64_t nidx = int64_t(c->d_ns_idx.n);
        c->d_ns_zs.alloc(size_t(nidx));
        c->d_ns_u.alloc(size_t(N));
        c->d_ns_w.alloc(size_t(N));
        c->d_ns_e.alloc(size_t(c->ns_ncell));
        c->d_ns_sum.alloc(size_t(c->ns_ncell));
        c->d_ns_part.alloc(size_t(c->ns_ncell) * launch::CELL_SPLIT);
        launch::cell_basis(N, nidx, c->d_ns_idx.p, c->d_int2ext.p, c->d_sc.p, c->d_ns_zs.p, c->d_ns_u.p, s);
        launch::fill_zero(N, c->d_ns_w.p, s);
        c->ns_basis = true;
        c->ns_stale = true;
    }
    if (c->ns_stale) {
        // W on the membrane rows, from their intracellular potential columns (u is 0 on the
        // others); the rest of W stays 0 (A z_k vanishes there)
        launch::rows_sub_spmv(c->ns_nrows, c->d_ns_rows.p, c->d_ns_wptr.p, c->d_ns_woff.p, c->d_rowptr_s.p,
                              c->d_colidx.p, c->d_vals.p, c->d_ns_u.p, c->d_ns_w.p, s);
        launch::cell_dot(c->ns_ncell, c->d_ns_ptr.p, c->d_ns_idx.p, c->d_ns_zs.p, c->d_ns_w.p, c->d_ns_part.p,
                         c->d_ns_e.p, s);
        c->ns_stale = false;
    }
}

}  // namespace

void gauge_build(knp_ctx *c) {
    const HostMesh &h = c->hm;
    const int64_t N = h.N, Ni = h.Nr[0], Ne = h.Nr[1];
    const int K = h.n_cells;
    if (K < 1) throw Error{KNP_E_ARG, "gauge 1 needs at least one cell"};
    // the cells' intracellular DOFs must not couple: every region neighbour of an
    // intracellular node and every membrane neighbour of a membrane node lies in its cell
    for (int64_t l = 0; l < Ni; ++l) {
        const int32_t cl = h.vcell[h.verts[0][l]];
        for (int64_t q = h.prow[0][l]; q < h.prow[0][l + 1]; ++q)
            if (h.vcell[h.verts[0][h.pcol[0][q]]] != cl)
                throw Error{KNP_E_ARG, "gauge 1 needs cells whose intracellular nodes do not neighbour each other"};
    }
    for (size_t g = 0; g < h.gamma.size(); ++g) {
        const int32_t cl = h.vcell[h.gamma[g]];
        for (int64_t q = h.grow[g]; q < h.grow[g + 1]; ++q)
            if (h.vcell[h.gcol[q]] != cl)
                throw Error{KNP_E_ARG, "gauge 1 needs cells whose membranes do not neighbour each other"};
    }
    // owner of each storage DOF: the cell of its intracellular node, or of its
    // extracellular node when that node is on the membrane; -1 otherwise
    std::vector<int32_t> owner(N, -1);
    std::vector<int64_t> ptr(size_t(K) + 1, 0);
    for (int64_t i = 0; i < N; ++i) {
        const int64_t e = c->int2ext[i];
        int32_t cell;
        if (e < 4 * Ni) {
            cell = h.vcell[h.verts[0][e % Ni]];
        } else {
            const int32_t v = h.verts[1][(e - 4 * Ni) % Ne];
            cell = h.gidx[v] >= 0 ? h.vcell[v] : 0;
        }
        if (cell < 0 || cell > K) throw Error{KNP_E_ARG, "internal: cell id out of range"};
        owner[i] = cell - 1;
        if (e >= 3 * Ni && e < 4 * Ni) ++ptr[cell];
    }
    for (int k = 0; k < K; ++k) ptr[k + 1] += ptr[k];
    // the rows of membrane nodes (both regions): elsewhere every term of a row that
    // meets z_k is a divergence form, so (A z_k)_i is 0 up to rounding and W_i is kept 0
    // and per such row the in-row positions of its intracellular potential columns (a
    // storage row keeps its ABI row's entry order)
    std::vector<int32_t> rows;
    std::vector<int64_t> wptr{0};
    std::vector<uint16_t> woff;
    for (int64_t i = 0; i < N; ++i) {
        const int64_t e = c->int2ext[i];
        const int32_t v = e < 4 * Ni ? h.verts[0][e % Ni] : h.verts[1][(e - 4 * Ni) % Ne];
        if (owner[i] < 0 || h.gidx[v] < 0) continue;
        rows.push_back(int32_t(i));
        const int64_t a = h.rowptr[e], len = h.rowptr[e + 1] - a;
        if (len > 65535) throw Error{KNP_E_ARG, "gauge 1: a membrane row holds more than 65535 entries"};
        for (int64_t q = 0; q < len; ++q) {
            const int64_t ce = h.colidx[a + q];
            if (ce >= 3 * Ni && ce < 4 * Ni) woff.push_back(uint16_t(q));
        }
        wptr.push_back(int64_t(woff.size()));
    }
    std::vector<int32_t> idx(size_t(ptr[K]));
    {
        std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
        for (int64_t i = 0; i < N; ++i) {
            const int64_t e = c->int2ext[i];
            if (e >= 3 * Ni && e < 4 * Ni) idx[size_t(fill[owner[i]]++)] = int32_t(i);
        }
    }
    hipStream_t s = c->stream;
    c->d_ns_owner.alloc(size_t(N));
    c->d_ns_owner.upload(owner, s);
    c->d_ns_ptr.alloc(ptr.size());
    c->d_ns_ptr.upload(ptr, s);
    c->d_ns_idx.alloc(idx.size());
    c->d_ns_idx.upload(idx, s);
    c->d_ns_rows.alloc(rows.size());
    c->d_ns_rows.upload(rows, s);
    c->ns_nrows = int64_t(rows.size());
    c->d_ns_wptr.alloc(wptr.size());
    c->d_ns_wptr.upload(wptr, s);
    c->d_ns_woff.alloc(woff.size());
    c->d_ns_woff.upload(woff, s);
    c->ns_ncell = K;
    c->ns_basis = false;
    c->ns_stale = true;
}

// y = b - (S A S) x, FP64: the product timed as the solver's true residual, then the
// subtraction (folding it into the product's epilogue measured slower: b is read after
// the row sums, its latency exposed)
void residual(knp_ctx *c, bool transpose, const double *x, const double *b, double *y) {
    apply_operator(c, transpose, x, y, KNP_TIMER_RESID_A);
    launch::sub(c->hm.N, b, y, y, c->stream);
}

void apply_operator(knp_ctx *c, bool transpose, const double *x, double *y, int timer) {
    const int64_t N = c->hm.N;
    hipEvent_t t0 = c->tm.begin(timer, c->stream);
    if (transpose) {
        launch::spmv<double, double, double>(c->viewT(), c->d_valsT.p, x, y, c->stream);
    } else if (c->vtx) {
        launch::spmv_vtx<double>(c->viewV(), c->d_vals.p, x, y, c->stream);
        c->tm.end(timer, t0, c->vtx_bytes(8.0), c->stream);
        return;
    } else {
        launch::spmv<double, double, double>(c->viewA(), c->d_vals.p, x, y, c->stream);
    }
    c->tm.end(timer, t0, 12.0 * double(c->hm.nnz) + 32.0 * double(N) + 8.0, c->stream);
}

knp_status krylov_solve(knp_ctx *c, bool transpose, const double *b, double *x, const knp_solve_opts &o,
                        knp_solve_info *info) {
    const int64_t N = c->hm.N;
    hipStream_t s = c->stream;
    const bool use_amg = o.precond == 1;
    if (use_amg && !c->amg.ready) throw Error{KNP_E_STATE, "knp_amg_setup has not been called"};
    const int m = o.restart;
    const bool z32 = use_amg && c->amg.fp32;
    ensure_workspace(c, m, z32);
    if (transpose) ensure_transpose(c);
    double *bh = c->bh.p, *yh = c->yh.p, *w = c->w.p;
    // into the solver's order and scaling: bh = S b, yh = S^{-1} x
    launch::to_internal(N, c->d_int2ext.p, b, c->d_sc.p, bh, 0, s);
    launch::to_internal(N, c->d_int2ext.p, x, c->d_sc.p, yh, 1, s);
    // ||S b||^2 goes to dscal[1] and reaches the host with the first residual's norm
    // (one synchronisation for both; the Arnoldi process overwrites the slot later)
    launch::multi_dot(N, bh, N, 1, bh, c->dscal.p + 1, c->partial.p, c->nblk, s);
    double bnorm = -1.0;   // not yet read
    knp_solve_info inf{};
    const bool gauge = c->gauge == 1 && !transpose;
    if (gauge) gauge_refresh(c);
    std::vector<double> H(size_t(m + 1) * m), H0(size_t(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hc = [&](int i, int j) -> double & { return H[size_t(j) * (m + 1) + i]; };
    auto H0c = [&](int i, int j) -> double & { return H0[size_t(j) * (m + 1) + i]; };   // before the rotations
    // At rtol >= UPDATED_MIN_RTOL, a cycle whose recurrence estimate meets rtol is tested on
    // the residual of its updated iterate formed from the Arnoldi relation,
    // r0 - (S A S) Z y = V (beta e_1 - H y), instead of a product with the operator: the two
    // differ by rounding in that relation, of the order of the unit roundoff times
    // G = sqrt(j + 1) sum_k |y_k| ||H e_k|| (the sizes of the products (S A S) z_k y_k it
    // sums), and the form is used only while UPDATED_EPS G stays below a hundredth of the
    // tolerance.  Below UPDATED_MIN_RTOL, and whenever that residual misses rtol, the
    // residual comes from a product, and the iterate is then exactly as without the test.
    constexpr double UPDATED_MIN_RTOL = 1e-10;
    constexpr double UPDATED_EPS = 1e-12;
    bool try_updated = false;
    int upd_j = 0;          // the cycle's last basis index: c = [c_0, ..., c_upd_j]
    double upd_c0 = 0.0;    // c_0 (host); c_1 ... in dscal[upd_j + 1 ...]
    std::vector<double> coef(size_t(m) + 1);
    int its = 0, restarts = 0;
    double est = 1.0;
    bool converged = false;
    // Attainable-accuracy floor: a cycle that ends on a converged recurrence
    // estimate while the recomputed residual stays above rtol has met the rounding
    // floor of ||S b - S A S y||.  After STALL_WINDOW such restarts in a row over
    // which the recomputed residual has not halved, the solve stops (KNP_E_NOCONV).
    constexpr int STALL_WINDOW = 50;
    int stall = 0;
    bool cycle_est_converged = false;
    double window_beta = 0.0;
    double true_rel = 1.0;   // residual of the current iterate
    // every exit below happens right after the residual of the current iterate is formed
    // (by a product, or from the Arnoldi relation), so that residual is the one reported
    while (true) {
        const bool updated = try_updated;
        try_updated = false;
        if (updated) {   // w = V c = c_0 v_0 + sum_{i >= 1} c_i v_i
            launch::axpby(N, upd_c0, c->V.p, 0.0, w, s);
            launch::multi_axpy<double>(N, c->V.p + N, N, upd_j, c->dscal.p + upd_j + 1, w, s);
        } else {
            residual(c, transpose, yh, bh, w);
        }
        if (gauge) {   // yh += sum_k c_k S^{-1} z_k, S r -= sum_k c_k S A z_k (yh only once
                       // an updated residual has passed the test)
            launch::cell_dot(c->ns_ncell, c->d_ns_ptr.p, c->d_ns_idx.p, c->d_ns_zs.p, w, c->d_ns_part.p,
                             c->d_ns_sum.p, s);
            launch::cell_correct(N, c->d_ns_owner.p, c->d_ns_w.p, c->d_ns_u.p, c->d_ns_sum.p, c->d_ns_e.p, w,
                                 updated ? nullptr : yh, s);
        }
        launch::multi_dot(N, w, N, 1, w, c->dscal.p, c->partial.p, c->nblk, s);
        const int nread = bnorm < 0.0 ? 2 : 1;
        hip_check(hipMemcpyAsync(c->hbuf.p, c->dscal.p, sizeof(double) * nread, hipMemcpyDeviceToHost, s),
                  "norm copy");
        hip_check(hipStreamSynchronize(s), "norm sync");
        if (bnorm < 0.0) {
            bnorm = std::sqrt(c->hbuf.p[1]);
            if (!std::isfinite(bnorm)) throw Error{KNP_E_NUMERIC, "NaN or Inf in the right-hand side"};
            if (bnorm == 0.0) {
                hip_check(hipMemsetAsync(x, 0, size_t(N) * sizeof(double), s), "zero x");
                hip_check(hipStreamSynchronize(s), "sync");
                c->tm.harvest();
                if (info) *info = inf;
                return KNP_OK;
            }
        }
        const double beta = std::sqrt(c->hbuf.p[0]);
        if (!std::isfinite(beta)) throw Error{KNP_E_NUMERIC, "NaN or Inf in the residual"};
        est = beta / bnorm;
        true_rel = est;
        if (est <= o.rtol) {
            if (updated && gauge)
                launch::cell_correct(N, c->d_ns_owner.p, c->d_ns_w.p, c->d_ns_u.p, c->d_ns_sum.p, c->d_ns_e.p,
                                     nullptr, yh, s);
            converged = true;
            break;
        }
        if (updated) continue;   // missed rtol: the residual from a product decides
        if (its >= o.max_it) break;
        if (restarts > 0 && cycle_est_converged && beta > 0.5 * window_beta) {
            if (++stall >= STALL_WINDOW) break;
        } else {
            stall = 0;
            window_beta = beta;
        }
        ++restarts;
        double *V = c->V.p;
        launch::axpby(N, 1.0 / beta, w, 0.0, V, s);
        std::fill(g.begin(), g.end(), 0.0);
        g[0] = beta;
        int jend = 0;
        for (int j = 0; j < m; ++j) {
            const double *vj = V + size_t(j) * N;
            double *wj = V + size_t(j + 1) * N;
            if (use_amg) {
                if (z32) {
                    float *zj = c->Z32.p + size_t(j) * N;
                    amg_vcycle(c->amg, vj, zj, s, &c->tm);
                    hipEvent_t t0 = c->tm.begin(KNP_TIMER_SPMV_A, s);
                    if (!transpose && c->vtx) {
                        launch::spmv_vtx<float>(c->viewV(), c->d_vals.p, zj, wj, s);
                        c->tm.end(KNP_TIMER_SPMV_A, t0, c->vtx_bytes(4.0), s);
                    } else {
                        launch::spmv<double, float, double>(transpose ? c->viewT() : c->viewA(),
                                                            transpose ? c->d_valsT.p : c->d_vals.p, zj, wj, s);
                        c->tm.end(KNP_TIMER_SPMV_A, t0, 12.0 * double(c->hm.nnz) + 28.0 * double(N) + 8.0, s);
                    }
                } else {
                    double *zj = c->Z64.p + size_t(j) * N;
                    amg_vcycle(c->amg, vj, zj, s, &c->tm);
                    apply_operator(c, transpose, zj, wj);
                }
            } else {
                apply_operator(c, transpose, vj, wj);
            }
            // classical Gram-Schmidt (optionally twice); the coefficients and the new
            // norm (dh[m + 1]) reach the host in one copy into pinned memory, the
            // first pass's coefficients in a copy of their own when there are two
            double *dh = c->dscal.p;
            double *hp = c->hbuf.p;   // [0, m + 2): last pass; [m + 2, 2m + 4): first of two
            launch::multi_dot(N, V, N, j + 1, wj, dh, c->partial.p, c->nblk, s);
            launch::gs_update(N, V, N, j + 1, dh, wj, c->partial.p, c->nblk, s);
            if (o.reorth) {
                hip_check(hipMemcpyAsync(hp + m + 2, dh, sizeof(double) * (j + 1), hipMemcpyDeviceToHost, s), "h");
                launch::multi_dot(N, V, N, j + 1, wj, dh, c->partial.p, c->nblk, s);
                launch::gs_update(N, V, N, j + 1, dh, wj, c->partial.p, c->nblk, s);
            }
            launch::reduce_partials(1, c->nblk, c->partial.p, dh + m + 1, s);
            hip_check(hipMemcpyAsync(hp, dh, sizeof(double) * (m + 2), hipMemcpyDeviceToHost, s), "h");
            hip_check(hipStreamSynchronize(s), "gs sync");
            const double hn = std::sqrt(hp[m + 1]);
            if (!std::isfinite(hn)) throw Error{KNP_E_NUMERIC, "NaN or Inf in the Arnoldi process"};
            for (int i = 0; i <= j; ++i) Hc(i, j) = H0c(i, j) = o.reorth ? hp[m + 2 + i] + hp[i] : hp[i];
            Hc(j + 1, j) = H0c(j + 1, j) = hn;
            if (hn > 0.0) launch::scale_by_inv_norm(N, wj, dh + m + 1, wj, s);
            // Givens rotations
            for (int i = 0; i < j; ++i) {
                const double t = cs[i] * Hc(i, j) + sn[i] * Hc(i + 1, j);
                Hc(i + 1, j) = -sn[i] * Hc(i, j) + cs[i] * Hc(i + 1, j);
                Hc(i, j) = t;
            }
            const double den = std::hypot(Hc(j, j), Hc(j + 1, j));
            cs[j] = den > 0.0 ? Hc(j, j) / den : 1.0;
            sn[j] = den > 0.0 ? Hc(j + 1, j) / den : 0.0;
            Hc(j, j) = den;
            Hc(j + 1, j) = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            ++its;
            jend = j + 1;
            est = std::fabs(g[j + 1]) / bnorm;
            if (est <= o.rtol || its >= o.max_it || hn == 0.0) break;
        }
        cycle_est_converged = est <= o.rtol;
        // y = H^{-1} g (upper triangular), x += Z y
        for (int i = jend - 1; i >= 0; --i) {
            double t = g[i];
            for (int k = i + 1; k < jend; ++k) t -= Hc(i, k) * y[k];
            y[i] = Hc(i, i) != 0.0 ? t / Hc(i, i) : 0.0;
        }
        // the updated iterate's residual coefficients, c = beta e_1 - H y (H as the Arnoldi
        // process built it, before the rotations)
        int ncopy = jend;
        double G = 0.0;
        for (int k = 0; k < jend && cycle_est_converged; ++k) {
            double cn = 0.0;
            for (int i = 0; i <= k + 1; ++i) cn += H0c(i, k) * H0c(i, k);
            G += std::fabs(y[k]) * std::sqrt(cn);
        }
        G *= std::sqrt(double(jend + 1));
        if (cycle_est_converged && o.rtol >= UPDATED_MIN_RTOL && UPDATED_EPS * (G + beta) <= 0.01 * o.rtol * bnorm) {
            for (int i = 0; i <= jend; ++i) {
                double t = i == 0 ? beta : 0.0;
                for (int k = std::max(0, i - 1); k < jend; ++k) t -= H0c(i, k) * y[k];
                coef[i] = t;
            }
            try_updated = true;
            upd_j = jend;
            upd_c0 = coef[0];
            ncopy = 2 * jend + 1;   // dscal[0, jend): y; dscal[jend, 2 jend + 1): c
        }
        // through pinned memory: the host writes it next only after the next cycle's
        // synchronisations, and the device-to-host copies into it are stream-ordered
        // after this copy
        std::memcpy(c->hbuf.p, y.data(), sizeof(double) * jend);
        if (try_updated) std::memcpy(c->hbuf.p + jend, coef.data(), sizeof(double) * (jend + 1));
        hip_check(hipMemcpyAsync(c->dscal.p, c->hbuf.p, sizeof(double) * ncopy, hipMemcpyHostToDevice, s), "y");
        if (!use_amg)
            launch::multi_axpy<double>(N, c->V.p, N, jend, c->dscal.p, yh, s);
        else if (z32)
            launch::multi_axpy<float>(N, c->Z32.p, N, jend, c->dscal.p, yh, s);
        else
            launch::multi_axpy<double>(N, c->Z64.p, N, jend, c->dscal.p, yh, s);
        inf.rel_res_est = est;
    }
    inf.rel_res = true_rel;
    if (its == 0) inf.rel_res_est = true_rel;   // no iteration: the estimate is the residual
    inf.its = its;
    inf.restarts = restarts;
    launch::to_external(N, c->d_int2ext.p, yh, c->d_sc.p, x, 0, s);   // x = S yh
    if (gauge) {   // every potential minus the reference DOF's value
        const int64_t Ni = c->hm.Nr[0], Ne = c->hm.Nr[1];
        hip_check(hipMemcpyAsync(c->d_ns_sum.p, x + c->hm.pin_dof, sizeof(double), hipMemcpyDeviceToDevice, s),
                  "reference potential");
        launch::shift_potentials(3 * Ni, 4 * Ni, 4 * Ni + 3 * Ne, 4 * Ni + 4 * Ne, c->d_ns_sum.p, x, s);
    }
    hip_check(hipStreamSynchronize(s), "solve sync");
    c->tm.harvest();
    if (info) *info = inf;
    if (!converged && !(inf.rel_res <= o.rtol)) return KNP_E_NOCONV;
    return KNP_OK;
}

void ensure_transpose(knp_ctx *c) {
    const HostMesh &m = c->hm;
    hipStream_t s = c->stream;
    if (!c->have_T) {
        // transpose of the stored (solver-order) pattern; perm[p] is the storage
        // position of the entry that lands at position p of the transpose
        std::vector<int64_t> rpT(m.N + 1, 0), perm(m.nnz);
        std::vector<int32_t> colT(m.nnz);
        for (int64_t k = 0; k < m.nnz; ++k) rpT[c->ext2int[m.colidx[k]] + 1]++;
        for (int64_t i = 0; i < m.N; ++i) rpT[i + 1] += rpT[i];
        std::vector<int64_t> fill(rpT.begin(), rpT.end() - 1);
        for (int64_t i = 0; i < m.N; ++i) {
            const int64_t R = c->int2ext[i], a = m.rowptr[R], len = m.rowptr[R + 1] - a;
            for (int64_t q = 0; q < len; ++q) {
                const int64_t p = fill[c->ext2int[m.colidx[a + q]]]++;
                colT[p] = int32_t(i);
                perm[p] = c->rowptr_s[i] + q;
            }
        }
        c->d_rowptrT.alloc(m.N + 1);
        c->d_rowptrT.upload(rpT, s);
        c->d_colT.alloc(m.nnz);
        c->d_colT.upload(colT, s);
        c->d_permT.alloc(m.nnz);
        c->d_permT.upload(perm, s);
        {
            std::vector<int32_t> b = row_blocks(rpT.data(), m.N);
            c->nblkT = int64_t(b.size()) - 1;
            c->d_blkT.alloc(b.size());
            c->d_blkT.upload(b, s);
        }
        c->d_valsT.alloc(m.nnz);
        hip_check(hipStreamSynchronize(s), "transpose upload");
        c->have_T = true;
        c->T_current = false;
    }
    if (!c->T_current) {
        launch::gather(m.nnz, c->d_vals.p, c->d_permT.p, c->d_valsT.p, s);
        c->T_current = true;
    }
}

}  // namespace knp
