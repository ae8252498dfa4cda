// Assembly kernels for the IMEX-linearised KNP-EMI step (eq. ``lin_sys``): the
// membrane coefficients, the dt-dependent static blocks, and helpers.  The per-step bulk
// values of an order-1 mesh are in assemble_rows.hip, the membrane blocks and the
// order-2 path in assemble_p2.hip.
//
// The static kernel is a deterministic gather: one thread owns one region vertex (one
// scalar row, i.e. four global rows) and walks the elements incident to it in a fixed
// order, accumulating into LDS slots indexed by the row's column positions.  No
// floating-point atomics are used, so two runs are bitwise identical.
//
// Integrals are exact for P1: on a simplex of dimension m with measure |T|,
//   int prod lambda_a^{p_a} = m! |T| prod p_a! / (m + sum p_a)!.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "fem_device.h"
#include "knp_internal.h"

// Scratch of the allocation-free assembly entry point: the NaN counter in the first
// 256 bytes, then the per-membrane-vertex coefficient record.  Every device holds its
// own copy until the process ends.  Host code never passes this symbol to a kernel: it
// uses the device address that noalloc_scratch() obtains for the current device.
static __device__ __align__(256) double scratch[knp::NOALLOC_HEAD + knp::NOALLOC_MAX_GAMMA * knp::GC_STRIDE];

namespace knp {
namespace launch {

namespace {

using namespace knp::fem;

constexpr int BLK = 64;   // one wavefront per block; LDS slots are [..][pos][thread]

// ------------------------------------------------------------------ membrane coefficients
// Hodgkin-Huxley 1952 rates in 1/s; V in mV relative to rest.
__device__ inline double hh_ratio(double x) {   // x / (exp(x/10) - 1), limit 10
    return x == 0.0 ? 10.0 : x / expm1(x / 10.0);
}

__device__ inline void hh_rates(double V, double (&a)[3], double (&b)[3]) {
    a[0] = 0.01 * hh_ratio(10.0 - V) * 1000.0;
    b[0] = 0.125 * exp(-V / 80.0) * 1000.0;
    a[1] = 0.1 * hh_ratio(25.0 - V) * 1000.0;
    b[1] = 4.0 * exp(-V / 18.0) * 1000.0;
    a[2] = 0.07 * exp(-V / 20.0) * 1000.0;
    b[2] = 1.0 / (exp((30.0 - V) / 10.0) + 1.0) * 1000.0;
}

// One thread per membrane vertex: channel currents I_ch^k at u_{n-1} for the cell's model
// (0 passive leak, 1 Hodgkin-Huxley after the gating update, 2 Kir-Na/K, Sec. "Passive
// dynamics: Kir--Na/K"), then the coefficients C_r^k, g_r^k, h_r of both regions.
__global__ void k_membrane_coef(GammaArgs g, PhysArgs p, int64_t Ni, int64_t Ne, const double *__restrict__ u,
                                double *__restrict__ gates, const double *__restrict__ theta,
                                double *__restrict__ gc) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= g.n_gamma) return;
    const int64_t li = g.gloc_i[i], le = g.gloc_e[i];
    const int cell = g.gcell[i] - 1;
    const int64_t offe = 4 * Ni;
    double ci[3], ce[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        ci[k] = u[k * Ni + li];
        ce[k] = u[offe + k * Ne + le];
    }
    const double phiM = u[3 * Ni + li] - u[offe + 3 * Ne + le];
    const int model = g.cell_model[cell];
    const int stim = g.cell_stim[cell];
    const double th = theta ? theta[cell] : 1.0;

    double gk[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) gk[k] = th * p.g_leak[k];
    if (stim) gk[0] += p.g_stim_bar * exp(-fmod(p.t, p.stim_tau) / p.stim_a);
    if (model == 1) {
        // n_ode Rush-Larsen sub-steps of the gating ODE with phi_M frozen at phi_M^{n-1}
        double w[3] = {gates[3 * i + 0], gates[3 * i + 1], gates[3 * i + 2]};
        double a[3], b[3];
        hh_rates(1000.0 * (phiM - p.phi_rest), a, b);
        const double hs = p.dt / p.n_ode;
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const double tinv = a[q] + b[q];
            const double winf = a[q] / tinv;
            const double decay = exp(-tinv * hs);
            for (int s = 0; s < p.n_ode; ++s) w[q] = winf + (w[q] - winf) * decay;
            gates[3 * i + q] = w[q];
        }
        gk[0] += p.gbar_Na * w[1] * w[1] * w[1] * w[2];
        gk[1] += p.gbar_K * w[0] * w[0] * w[0] * w[0];
    }
    double I[3], E[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        E[k] = p.psi / p.z[k] * log(ce[k] / ci[k]);
        I[k] = gk[k] * (phiM - E[k]);
    }
    if (model == 2) {
        // Kir-Na/K: K+ leak times the inward-rectifier factor, and the Na/K pump, which
        // carries 3 Na+ out and 2 K+ in per cycle
        const double A = 1.0 + exp(0.433);
        const double B = 1.0 + exp(-(0.1186 + p.E_K0) / 0.0441);
        const double C = 1.0 + exp((phiM - E[1] + 0.0185) / 0.0425);
        const double D = 1.0 + exp(-(0.1186 + phiM) / 0.0441);
        const double fkir = A * B / (C * D) * sqrt(ce[1] / p.K_e0);
        const double na = ci[0] * sqrt(ci[0]);
        const double pna = p.P_Na * sqrt(p.P_Na);
        const double jp = p.rho_pump * na / (na + pna) * ce[1] / (ce[1] + p.P_K);
        I[0] += 3.0 * p.F * p.z[0] * jp;
        I[1] = I[1] * fkir - 2.0 * p.F * p.z[1] * jp;
    }
    const double Itot = I[0] + I[1] + I[2];
    double *o = gc + i * GC_STRIDE;
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const double *c = r == 0 ? ci : ce;
        const double sgn = r == 0 ? 1.0 : -1.0;
        double wsum = 0.0, wk[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            wk[k] = p.D[k] * p.z[k] * p.z[k] * c[k];
            wsum += wk[k];
        }
        double *orr = o + r * GC_REGION;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double alpha = wk[k] / wsum;
            orr[GC_C + k] = alpha * p.C_m / (p.F * p.z[k]);
            orr[GC_G + k] = sgn * (p.dt * I[k] - alpha * p.C_m * phiM) / (p.F * p.z[k]);
        }
        orr[GC_H] = sgn * (p.dt * Itot - p.C_m * phiM) / p.F;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) o[GC_I + k] = I[k];
}

// ------------------------------------------------------------------ bulk, static part
// c_r^k rows, own block: M + tau_k A;  phi_r row, c_r^k blocks: z_k tau_k A.
template <int D>
__global__ void __launch_bounds__(BLK) k_static(RegionArgs ra, MeshArgs ma, PhysArgs p,
                                                const int64_t *__restrict__ rowptr,
                                                const int64_t *__restrict__ rstart, double *__restrict__ vals,
                                                const double *__restrict__ sc, int64_t pin_dof) {
    __shared__ double sA[MAXN][BLK];
    __shared__ double sM[MAXN][BLK];
    const int tid = threadIdx.x;
    const int64_t j = int64_t(blockIdx.x) * BLK + tid;
    if (j >= ra.Nr) return;
    const int64_t p0 = ra.prow[j];
    const int n = int(ra.prow[j + 1] - p0);
    for (int q = 0; q < n; ++q) {
        sA[q][tid] = 0.0;
        sM[q][tid] = 0.0;
    }
    const int32_t *loc = ra.r == 0 ? ma.loc_i : ma.loc_e;
    for (int64_t t = ra.irow[j]; t < ra.irow[j + 1]; ++t) {
        const int32_t e = ra.ielem[t];
        const uint32_t pk = ra.ipos[t];
        const int slot = pk & 3u;
        int32_t vg[D + 1];
        double x[D + 1][D], g[D + 1][D];
        load_simplex<D>(ma, e, vg, x);
        const double vol = simplex_grads<D>(x, g);
#pragma unroll
        for (int a = 0; a <= D; ++a) {
            const int q = (pk >> (2 + 5 * a)) & 31u;
            double dot = 0.0;
#pragma unroll
            for (int d = 0; d < D; ++d) dot += g[slot][d] * g[a][d];
            sA[q][tid] += vol * dot;
            sM[q][tid] += vol * mass_moment<D>(a == slot);
        }
    }
    (void)loc;
    const int64_t Nr = ra.Nr;
    const int32_t *pc = ra.pcol + p0;
    for (int k = 0; k < 3; ++k) {
        const int64_t row = ra.off + k * Nr + j;
        const int64_t rp = rstart[row];
        const int gq = int(rowptr[row + 1] - rowptr[row]) - 2 * n;
        const int64_t seg = rp + (ra.r == 0 ? 0 : gq);
        const double sr = sc[row];
        for (int q = 0; q < n; ++q) {
            const int64_t col = ra.off + k * Nr + pc[q];
            vals[seg + q] = (sM[q][tid] + p.tau[k] * sA[q][tid]) * sr * sc[col];
        }
    }
    const int64_t row = ra.off + 3 * Nr + j;
    const int64_t rp = rstart[row];
    const int gq = int(rowptr[row + 1] - rowptr[row]) - 4 * n;
    const int64_t seg0 = rp + (ra.r == 0 ? 0 : gq);
    const double sr = sc[row];
    const bool pinrow = row == pin_dof;
    for (int k = 0; k < 3; ++k)
        for (int q = 0; q < n; ++q) {
            const int64_t col = ra.off + k * Nr + pc[q];
            vals[seg0 + k * n + q] = pinrow ? 0.0 : p.z[k] * p.tau[k] * sA[q][tid] * sr * sc[col];
        }
}

// ------------------------------------------------------------------ helpers
__global__ void k_check_finite(const double *__restrict__ u, int64_t n, int *flag) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        if (!isfinite(u[i])) *flag = 1;
}

__global__ void k_clear_flag(int *flag) { *flag = 0; }

__global__ void k_scaling_from_diag(int64_t N, const double *__restrict__ vals, const int64_t *__restrict__ dpos,
                                    double *__restrict__ sc) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double d = fabs(vals[dpos[i]]);
    sc[i] = d > 0.0 ? 1.0 / sqrt(d) : 1.0;
}

__global__ void k_gather(int64_t n, const double *__restrict__ src, const int64_t *__restrict__ map,
                         double *__restrict__ dst) {
    const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[map[i]];
}

// Solver order <-> ABI order.  The matrix and every solver vector are stored by
// vertex with the four fields side by side (internal DOF off_r + 4 j + f); the
// ABI and the assembly use off_r + f N_r + j.  int2ext maps the first to the
// second.  mode 0: times sc, 1: divided by sc, 2: plain copy (sc ignored).
__global__ void k_to_internal(int64_t n, const int32_t *__restrict__ int2ext, const double *__restrict__ x,
                              const double *__restrict__ sc, double *__restrict__ y, int mode) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t e = int2ext[i];
        y[i] = mode == 0 ? x[e] * sc[e] : (mode == 1 ? x[e] / sc[e] : x[e]);
    }
}

__global__ void k_to_external(int64_t n, const int32_t *__restrict__ int2ext, const double *__restrict__ y,
                              const double *__restrict__ sc, double *__restrict__ x, int mode) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t e = int2ext[i];
        x[e] = mode == 0 ? y[i] * sc[e] : (mode == 1 ? y[i] / sc[e] : y[i]);
    }
}

// values of each ABI-order row from their storage position
__global__ void k_rows_to_external(int64_t N, const int64_t *__restrict__ rowptr, const int64_t *__restrict__ rstart,
                                   const double *__restrict__ src, double *__restrict__ dst) {
    for (int64_t r = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; r < N; r += int64_t(gridDim.x) * blockDim.x) {
        const int64_t a = rowptr[r], len = rowptr[r + 1] - a, b = rstart[r];
        for (int64_t q = 0; q < len; ++q) dst[a + q] = src[b + q];
    }
}

inline unsigned nblocks(int64_t n, int b) { return unsigned((n + b - 1) / b); }

}  // namespace

void check_finite(const double *u, int64_t n, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_check_finite, dim3(1024), dim3(256), 0, s, u, n, flag);
}

void clear_flag(int *flag, hipStream_t s) { hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, s, flag); }

double *noalloc_scratch(int device) {
    static std::mutex mu;
    static std::vector<double *> addr;
    std::lock_guard<std::mutex> lock(mu);
    if (device < 0) throw Error{KNP_E_ARG, "no device for the static scratch"};
    if (size_t(device) >= addr.size()) addr.resize(size_t(device) + 1, nullptr);
    if (!addr[device]) {
        void *p = nullptr;
        hip_check(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
        addr[device] = static_cast<double *>(p);
    }
    return addr[device];
}

void membrane_coefficients(const GammaArgs &g, const PhysArgs &p, int64_t Ni, int64_t Ne, const double *u_prev,
                           double *gates, const double *theta, double *gcoef, hipStream_t s) {
    if (g.n_gamma == 0) return;
    hipLaunchKernelGGL(k_membrane_coef, dim3(nblocks(g.n_gamma, 128)), dim3(128), 0, s, g, p, Ni, Ne, u_prev,
                       gates, theta, gcoef);
}

void assemble_static(const RegionArgs &ra, const MeshArgs &ma, const PhysArgs &p, const int64_t *rowptr,
                     const int64_t *rstart, double *vals, const double *sc, int64_t pin_dof, hipStream_t s) {
    if (ra.Nr == 0) return;
    if (ma.dim == 2)
        hipLaunchKernelGGL(k_static<2>, dim3(nblocks(ra.Nr, BLK)), dim3(BLK), 0, s, ra, ma, p, rowptr, rstart, vals,
                           sc, pin_dof);
    else
        hipLaunchKernelGGL(k_static<3>, dim3(nblocks(ra.Nr, BLK)), dim3(BLK), 0, s, ra, ma, p, rowptr, rstart, vals,
                           sc, pin_dof);
}

void scaling_from_diag(int64_t N, const double *vals, const int64_t *diag_pos, double *sc, hipStream_t s) {
    hipLaunchKernelGGL(k_scaling_from_diag, dim3(nblocks(N, 256)), dim3(256), 0, s, N, vals, diag_pos, sc);
}

void gather(int64_t n, const double *src, const int64_t *map, double *dst, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_gather, dim3(nblocks(n, 256)), dim3(256), 0, s, n, src, map, dst);
}

void to_internal(int64_t n, const int32_t *int2ext, const double *x, const double *sc, double *y, int mode,
                 hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_to_internal, dim3(std::min<int64_t>(nblocks(n, 256), 8192)), dim3(256), 0, s, n, int2ext, x,
                       sc, y, mode);
}

void to_external(int64_t n, const int32_t *int2ext, const double *y, const double *sc, double *x, int mode,
                 hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_to_external, dim3(std::min<int64_t>(nblocks(n, 256), 8192)), dim3(256), 0, s, n, int2ext, y,
                       sc, x, mode);
}

void rows_to_external(int64_t N, const int64_t *rowptr, const int64_t *rstart, const double *src, double *dst,
                      hipStream_t s) {
    if (N == 0) return;
    hipLaunchKernelGGL(k_rows_to_external, dim3(std::min<int64_t>(nblocks(N, 256), 8192)), dim3(256), 0, s, N, rowptr,
                       rstart, src, dst);
}

}  // namespace launch
}  // namespace knp
