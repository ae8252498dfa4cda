// Vector-Jacobian products of one step's residual R_n = A(u_{n-1}, theta) u_n
// - f(u_{n-1}, theta) (eq. ``lin_sys``) for the discrete adjoint: given lambda_n,
//   u_prev_bar += (dR_n/du_{n-1})^T lambda_n,   theta_bar += (dR_n/dtheta)^T lambda_n.
//
// u_{n-1} enters A through the concentration-weighted stiffness A_r^{k,n-1}
// (c_r^k rows: tilde-tau_k A_r^k in the phi_r columns; phi_r rows:
// sum_k z_k tilde-tau_k A_r^k) and through the membrane coefficient C_r^k; it
// enters f through M_r c^{k,n-1} and the membrane terms g_r^k, h_r (short-hands
// after eq. ``weak_disc`` and eq. ``weak_disc2``).  theta (per-cell factor on
// the leak conductances) enters only through the channel currents in g and h.
// Passive-leak membranes (with the optional stimulus); Hodgkin-Huxley gates are
// not differentiated.
//
// Deterministic gathers as in the assembly: one thread per region vertex walks
// its incident elements; one thread per membrane vertex walks its facets and
// applies the chain rule through the nodal membrane functions; one thread per
// cell sums the per-vertex theta contributions in a fixed order.
#include <hip/hip_runtime.h>

#include "fem_device.h"
#include "knp_internal.h"

namespace knp {
namespace launch {

namespace {

using namespace knp::fem;

// A_r^k[a,b] = sum_T mean_T(c^k) |T| grad(l_a).grad(l_b), so for a vertex v of T
//   d(sum_rows lambda_row R_row)/d c^k_v = (1/(D+1)) sum_{a,b in T} w^k_a K_T[a,b] phi_b,
//   w^k_a = tilde-tau_k (lambda(c_r^k, a) + z_k lambda(phi_r, a));
// and the right-hand side -M_r c^k contributes -(M_r lambda(c_r^k))_v.
template <int D>
__global__ void __launch_bounds__(64) k_vjp_bulk(RegionArgs ra, MeshArgs ma, PhysArgs p,
                                                 const double *__restrict__ u, const double *__restrict__ lam,
                                                 double *__restrict__ ubar, int64_t pin_dof) {
    const int64_t j = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (j >= ra.Nr) return;
    const int32_t *loc = ra.r == 0 ? ma.loc_i : ma.loc_e;
    const int64_t Nr = ra.Nr, off = ra.off, phib = ra.off + 3 * Nr;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int64_t t = ra.irow[j]; t < ra.irow[j + 1]; ++t) {
        const int32_t e = ra.ielem[t];
        const int slot = ra.ipos[t] & 3u;
        int32_t vg[D + 1];
        double x[D + 1][D], g[D + 1][D];
        load_simplex<D>(ma, e, vg, x);
        const double vol = simplex_grads<D>(x, g);
        double lc[3][D + 1], lp[D + 1], ph[D + 1];
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            const int64_t l = loc[vg[a]];
#pragma unroll
            for (int k = 0; k < 3; ++k) lc[k][a] = lam[off + k * Nr + l];
            const int64_t dphi = phib + l;
            // the pinned row keeps only its diagonal and the pinned column is zero
            lp[a] = dphi == pin_dof ? 0.0 : lam[dphi];
            ph[a] = dphi == pin_dof ? 0.0 : u[dphi];
        }
        double kph[D + 1];
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b <= D; ++b) {
                double dot = 0.0;
#pragma unroll
                for (int d = 0; d < D; ++d) dot += g[a][d] * g[b][d];
                s += vol * dot * ph[b];
            }
            kph[a] = s;
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double s = 0.0, m = 0.0;
#pragma unroll
            for (int a = 0; a <= D; ++a) {
                s += p.ttau[k] * (lc[k][a] + p.z[k] * lp[a]) * kph[a];
                m += vol * mass_moment<D>(a == slot) * lc[k][a];
            }
            acc[k] += s / double(D + 1) - m;
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) ubar[off + k * Nr + j] += acc[k];
}

// One thread per membrane vertex c.  Adjoints of the nodal membrane fields at c
// (sgn_r = +1 ICS, -1 ECS, F a facet containing c at slot sc):
//   Chat_r^k(c) = sgn_r sum_F sum_{a,b} lambda(c_r^k, a) |F| m3(a, b, sc) phi_M^n(b)
//   ghat_r^k(c) = sum_F sum_a lambda(c_r^k, a) |F| m2(a, sc)
//   hhat_r(c)   = sum_F sum_a lambda(phi_r, a) |F| m2(a, sc)
// then the chain rule through C, g, h -> alpha, I, E, phi_M^{n-1}, theta.
template <int D>
__global__ void k_vjp_membrane(GammaArgs g, MeshArgs ma, PhysArgs p, int64_t Ni, int64_t Ne,
                               const double *__restrict__ up, const double *__restrict__ un,
                               const double *__restrict__ lam, const double *__restrict__ theta,
                               double *__restrict__ ubar, double *__restrict__ thv) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= g.n_gamma) return;
    const int64_t off[2] = {0, 4 * Ni};
    const int64_t Nr[2] = {Ni, Ne};
    double Ch[2][3], gh[2][3], hh[2];
    for (int r = 0; r < 2; ++r) {
        const double sgn = r == 0 ? 1.0 : -1.0;
        const int32_t *loc = r == 0 ? ma.loc_i : ma.loc_e;
        const uint32_t *fpos = r == 0 ? g.fpos_i : g.fpos_e;
        for (int k = 0; k < 3; ++k) Ch[r][k] = gh[r][k] = 0.0;
        hh[r] = 0.0;
        for (int64_t t = g.frow[c]; t < g.frow[c + 1]; ++t) {
            const int32_t *fv = g.facets + int64_t(g.ffacet[t]) * D;
            const int sc = fpos[t] & 3u;
            const double meas = facet_measure<D>(ma, fv);
            double lc[3][D], lp[D], pm[D];
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const int64_t l = loc[fv[a]];
#pragma unroll
                for (int k = 0; k < 3; ++k) lc[k][a] = lam[off[r] + k * Nr[r] + l];
                lp[a] = lam[off[r] + 3 * Nr[r] + l];
                pm[a] = un[3 * Ni + ma.loc_i[fv[a]]] - un[4 * Ni + 3 * Ne + ma.loc_e[fv[a]]];
            }
#pragma unroll
            for (int a = 0; a < D; ++a) {
                const double m2 = meas * fmom2<D>(a, sc);
                hh[r] += lp[a] * m2;
                double w = 0.0;
#pragma unroll
                for (int b = 0; b < D; ++b) w += fmom3<D>(a, b, sc) * pm[b];
                w *= meas;
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    gh[r][k] += lc[k][a] * m2;
                    Ch[r][k] += sgn * lc[k][a] * w;
                }
            }
        }
    }
    // nodal quantities at c from u_{n-1}
    const int64_t li = g.gloc_i[c], le = g.gloc_e[c];
    const int cell = g.gcell[c] - 1;
    double cr[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cr[0][k] = up[k * Ni + li];
        cr[1][k] = up[4 * Ni + k * Ne + le];
    }
    const double phiM = up[3 * Ni + li] - up[4 * Ni + 3 * Ne + le];
    const double th = theta ? theta[cell] : 1.0;
    double gk[3], E[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        gk[k] = th * p.g_leak[k];
        E[k] = p.psi / p.z[k] * log(cr[1][k] / cr[0][k]);
    }
    if (g.cell_stim[cell]) gk[0] += p.g_stim_bar * exp(-fmod(p.t, p.stim_tau) / p.stim_a);
    double Ibar[3] = {0.0, 0.0, 0.0}, phibar = 0.0;
    double cbar[2][3];
    for (int r = 0; r < 2; ++r) {
        const double sgn = r == 0 ? 1.0 : -1.0;
        double w[3], ws = 0.0, alpha[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            w[k] = p.D[k] * p.z[k] * p.z[k];
            ws += w[k] * cr[r][k];
        }
        double abar[3], sa = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            alpha[k] = w[k] * cr[r][k] / ws;
            const double fz = p.F * p.z[k];
            Ibar[k] += gh[r][k] * sgn * p.dt / fz + hh[r] * sgn * p.dt / p.F;
            abar[k] = Ch[r][k] * p.C_m / fz - gh[r][k] * sgn * p.C_m * phiM / fz;
            phibar += -gh[r][k] * sgn * alpha[k] * p.C_m / fz;
            sa += abar[k] * alpha[k];
        }
        phibar += -hh[r] * sgn * p.C_m / p.F;
        // d alpha_k / d c_l = (delta_kl w_k - alpha_k w_l) / ws
#pragma unroll
        for (int l = 0; l < 3; ++l) cbar[r][l] = w[l] * (abar[l] - sa) / ws;
    }
    double thbar = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        phibar += Ibar[k] * gk[k];
        const double Ebar = -Ibar[k] * gk[k];
        cbar[1][k] += Ebar * p.psi / (p.z[k] * cr[1][k]);
        cbar[0][k] -= Ebar * p.psi / (p.z[k] * cr[0][k]);
        thbar += Ibar[k] * p.g_leak[k] * (phiM - E[k]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ubar[k * Ni + li] += cbar[0][k];
        ubar[4 * Ni + k * Ne + le] += cbar[1][k];
    }
    ubar[3 * Ni + li] += phibar;
    ubar[4 * Ni + 3 * Ne + le] -= phibar;
    thv[c] = thbar;
}

__global__ void k_reduce_theta(int n_cells, const int64_t *__restrict__ row, const int32_t *__restrict__ col,
                               const double *__restrict__ thv, double *__restrict__ out) {
    const int c = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= n_cells) return;
    double s = 0.0;
    for (int64_t t = row[c]; t < row[c + 1]; ++t) s += thv[col[t]];
    out[c] += s;
}

inline unsigned nblk(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

void vjp_bulk(const RegionArgs &ra, const MeshArgs &ma, const PhysArgs &p, const double *u_n, const double *lam,
              double *u_prev_bar, int64_t pin_dof, hipStream_t s) {
    if (ra.Nr == 0) return;
    if (ma.dim == 2)
        hipLaunchKernelGGL(k_vjp_bulk<2>, dim3(nblk(ra.Nr, 64)), dim3(64), 0, s, ra, ma, p, u_n, lam, u_prev_bar,
                           pin_dof);
    else
        hipLaunchKernelGGL(k_vjp_bulk<3>, dim3(nblk(ra.Nr, 64)), dim3(64), 0, s, ra, ma, p, u_n, lam, u_prev_bar,
                           pin_dof);
}

void vjp_membrane(const GammaArgs &g, const MeshArgs &ma, const PhysArgs &p, int64_t Ni, int64_t Ne,
                  const int64_t *prow_i, const int64_t *prow_e, const double *u_prev, const double *u_n,
                  const double *lam, const double *theta, double *u_prev_bar, double *theta_vertex, hipStream_t s) {
    (void)prow_i;
    (void)prow_e;
    if (g.n_gamma == 0) return;
    if (ma.dim == 2)
        hipLaunchKernelGGL(k_vjp_membrane<2>, dim3(nblk(g.n_gamma, 64)), dim3(64), 0, s, g, ma, p, Ni, Ne, u_prev,
                           u_n, lam, theta, u_prev_bar, theta_vertex);
    else
        hipLaunchKernelGGL(k_vjp_membrane<3>, dim3(nblk(g.n_gamma, 64)), dim3(64), 0, s, g, ma, p, Ni, Ne, u_prev,
                           u_n, lam, theta, u_prev_bar, theta_vertex);
}

void reduce_theta(int n_cells, const int64_t *cg_row, const int32_t *cg_col, const double *theta_vertex,
                  double *theta_bar, hipStream_t s) {
    if (n_cells == 0) return;
    hipLaunchKernelGGL(k_reduce_theta, dim3(nblk(n_cells, 64)), dim3(64), 0, s, n_cells, cg_row, cg_col, theta_vertex,
                       theta_bar);
}

}  // namespace launch
}  // namespace knp
