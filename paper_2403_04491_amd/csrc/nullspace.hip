// Kernels of the constant-potential gauge handled inside the solver (gauge 1; the
// third way of removing the nullspace that the Remark on the nullspace names: the
// system keeps its one-dimensional nullspace, the constant potential, and the Krylov
// solve deals with it).
//
// Besides the exact null vector, the operator has one near-null vector per cell: a
// constant intracellular potential on cell k, z_k.  Every bulk term of a potential or
// concentration row is a divergence form, so A z_k (and z_k^T A) reduce to the
// membrane terms of cell k, the capacitive weight C_m/F times the membrane mass (and
// the ions' shares of it in the concentration rows); an error along z_k shows in the
// residual only at that weight.  The solver
// therefore corrects its iterate along the z_k at the start of every cycle (a
// Galerkin coarse correction, E = Z^T A Z diagonal because the cells' intracellular
// DOFs do not couple), and at return shifts all potentials so that the reference
// extracellular DOF is zero, which gives the point-condition system's solution.
//
// All work here is a few streaming passes; the per-cell sums are deterministic
// (one workgroup per cell, fixed summation order).
#include <hip/hip_runtime.h>

#include <cmath>

#include "knp_internal.h"

namespace knp {
namespace launch {

namespace {

constexpr int TPB = 256;

// part[k * CELL_SPLIT + c] = sum over chunk c of [ptr[k], ptr[k+1]) of zs[q] * v[idx[q]]
// (CELL_SPLIT workgroups per cell, each a fixed-order tree over its chunk)
__global__ void __launch_bounds__(TPB) k_cell_dot_part(const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                                                       const double *__restrict__ zs, const double *__restrict__ v,
                                                       double *__restrict__ part) {
    __shared__ double red[TPB];
    const int k = int(blockIdx.x) / CELL_SPLIT, c = int(blockIdx.x) % CELL_SPLIT;
    const int64_t a0 = ptr[k], b0 = ptr[k + 1];
    const int64_t chunk = (b0 - a0 + CELL_SPLIT - 1) / CELL_SPLIT;
    const int64_t a = a0 + c * chunk, b = a + chunk < b0 ? a + chunk : b0;
    double s = 0.0;
    for (int64_t q = a + int64_t(threadIdx.x); q < b; q += TPB) s += zs[q] * v[idx[q]];
    red[threadIdx.x] = s;
    __syncthreads();
#pragma unroll
    for (int h = TPB / 2; h > 0; h >>= 1) {
        if (int(threadIdx.x) < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// out[k] = the cell's CELL_SPLIT partial sums added in order
__global__ void k_cell_dot_sum(int ncell, const double *__restrict__ part, double *__restrict__ out) {
    const int k = int(blockIdx.x) * blockDim.x + threadIdx.x;
    if (k >= ncell) return;
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < CELL_SPLIT; ++c) s += part[k * CELL_SPLIT + c];
    out[k] = s;
}

// zs[q] = 1 / S of storage DOF idx[q] (S in ABI order), and u[idx[q]] = zs[q]
__global__ void k_cell_basis(int64_t n, const int32_t *__restrict__ idx, const int32_t *__restrict__ int2ext,
                             const double *__restrict__ sc, double *__restrict__ zs, double *__restrict__ u) {
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += int64_t(gridDim.x) * blockDim.x) {
        const int32_t i = idx[q];
        const double z = 1.0 / sc[int2ext[i]];
        zs[q] = z;
        u[i] = z;
    }
}

__global__ void k_fill(int64_t n, double *__restrict__ y) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        y[i] = 0.0;
}

// With c_k = sum[k] / E[k] (0 if E[k] is 0 or not finite): r[i] -= c_k W[i] and
// y[i] += c_k u[i] for every storage DOF i whose rows couple to cell k (owner k >= 0);
// a null r or y skips that update
__global__ void k_cell_correct(int64_t n, const int32_t *__restrict__ owner, const double *__restrict__ W,
                               const double *__restrict__ u, const double *__restrict__ sum,
                               const double *__restrict__ E, double *__restrict__ r, double *__restrict__ y) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const int32_t k = owner[i];
        if (k < 0) continue;
        const double e = E[k];
        const double c = (e != 0.0 && isfinite(e)) ? sum[k] / e : 0.0;
        if (r) r[i] -= c * W[i];
        if (y) y[i] += c * u[i];
    }
}

// x[j] -= ref for j in [a0, a1) and [b0, b1), ref = the value of x at the reference DOF,
// copied to *ref before this kernel runs
__global__ void k_shift(int64_t a0, int64_t a1, int64_t b0, int64_t b1, const double *__restrict__ ref,
                        double *__restrict__ x) {
    const double d = ref[0];
    const int64_t na = a1 - a0, n = na + (b1 - b0);
    for (int64_t t = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; t < n; t += int64_t(gridDim.x) * blockDim.x) {
        const int64_t j = t < na ? a0 + t : b0 + (t - na);
        x[j] -= d;
    }
}

// y[rows[t]] = the listed entries of row rows[t] times x: the entries at storage positions
// rowptr[rows[t]] + off[e] for e in [wptr[t], wptr[t+1]); 16 lanes per listed row, fixed
// order (lane-strided partial sums, then a butterfly)
constexpr int RL = 16;
__global__ void __launch_bounds__(TPB) k_rows_sub_spmv(int64_t n, const int32_t *__restrict__ rows,
                                                       const int64_t *__restrict__ wptr,
                                                       const uint16_t *__restrict__ off,
                                                       const int64_t *__restrict__ rowptr,
                                                       const int32_t *__restrict__ col,
                                                       const double *__restrict__ val, const double *__restrict__ x,
                                                       double *__restrict__ y) {
    const int64_t t = (int64_t(blockIdx.x) * TPB + threadIdx.x) / RL;
    const int lane = int(threadIdx.x % RL);
    double s = 0.0;
    int32_t r = -1;
    if (t < n) {
        r = rows[t];
        const int64_t base = rowptr[r];
        for (int64_t e = wptr[t] + lane; e < wptr[t + 1]; e += RL) {
            const int64_t q = base + off[e];
            s += val[q] * x[col[q]];
        }
    }
#pragma unroll
    for (int o = RL / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, RL);
    if (lane == 0 && r >= 0) y[r] = s;
}

inline unsigned grid(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return unsigned(g);
}

}  // namespace

void cell_dot(int ncell, const int64_t *ptr, const int32_t *idx, const double *zs, const double *v, double *part,
              double *out, hipStream_t s) {
    if (ncell <= 0) return;
    hipLaunchKernelGGL(k_cell_dot_part, dim3(unsigned(ncell * CELL_SPLIT)), dim3(TPB), 0, s, ptr, idx, zs, v, part);
    hipLaunchKernelGGL(k_cell_dot_sum, dim3(unsigned((ncell + TPB - 1) / TPB)), dim3(TPB), 0, s, ncell, part, out);
}

void cell_basis(int64_t n, int64_t nidx, const int32_t *idx, const int32_t *int2ext, const double *sc, double *zs,
                double *u, hipStream_t s) {
    hipLaunchKernelGGL(k_fill, dim3(grid(n)), dim3(TPB), 0, s, n, u);
    if (nidx > 0) hipLaunchKernelGGL(k_cell_basis, dim3(grid(nidx)), dim3(TPB), 0, s, nidx, idx, int2ext, sc, zs, u);
}

void rows_sub_spmv(int64_t n, const int32_t *rows, const int64_t *wptr, const uint16_t *off, const int64_t *rowptr,
                   const int32_t *col, const double *val, const double *x, double *y, hipStream_t s) {
    if (n <= 0) return;
    const int64_t nb = (n * RL + TPB - 1) / TPB;
    hipLaunchKernelGGL(k_rows_sub_spmv, dim3(unsigned(nb)), dim3(TPB), 0, s, n, rows, wptr, off, rowptr, col, val, x,
                       y);
}

void fill_zero(int64_t n, double *y, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_fill, dim3(grid(n)), dim3(TPB), 0, s, n, y);
}

void cell_correct(int64_t n, const int32_t *owner, const double *W, const double *u, const double *sum,
                  const double *E, double *r, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_cell_correct, dim3(grid(n)), dim3(TPB), 0, s, n, owner, W, u, sum, E, r, y);
}

void shift_potentials(int64_t a0, int64_t a1, int64_t b0, int64_t b1, const double *ref, double *x, hipStream_t s) {
    const int64_t n = (a1 - a0) + (b1 - b0);
    if (n <= 0) return;
    hipLaunchKernelGGL(k_shift, dim3(grid(n)), dim3(TPB), 0, s, a0, a1, b0, b1, ref, x);
}

}  // namespace launch
}  // namespace knp
