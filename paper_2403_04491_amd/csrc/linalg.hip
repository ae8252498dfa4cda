// Sparse and dense linear-algebra kernels of the solver: the system matrix
// streamed by vertex (k_spmv_vtx), the finest AMG level in its field-block layout
// (stream_field_blocks), block-streamed CSR with fused epilogues (residual,
// Chebyshev step, prolongation-add) for the coarser levels and the transpose, the
// coarsest-level dense solve, and the Krylov vector kernels with deterministic
// two-stage reductions (classical Gram-Schmidt multi-dot and update, norms, axpys).
//
// All work is HBM-bound; nothing here is a dense contraction, so no matrix-core
// instructions are involved.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "knp_internal.h"

namespace knp {
namespace launch {

namespace {

constexpr int TPB = 256;

template <typename T>
struct Acc {
    using type = double;
};
template <>
struct Acc<float> {
    using type = float;   // FP32 levels accumulate in FP32
};

template <int G, typename A>
__device__ inline A group_sum(A v) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

typedef int32_t i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- block-streamed CSR
// Block b owns rows blk[b]..blk[b+1]-1, whose entries (at most STREAM_CAP) are
// contiguous in col/val.  Phase 1: the 256 threads stream the block's column
// indices and values with unit-stride loads (8 per thread, all issued before
// any x gather so the gathers overlap), multiply by the gathered x and stage
// the products in LDS.  Phase 2: each row is summed from LDS in a fixed order
// by one thread and handed to the epilogue (plain store, residual, Chebyshev
// update, prolongation add).  Deterministic: no atomics, fixed summation order.
//
// FP32 matrices (the AMG levels) stream 16 bytes of indices and 16 bytes of
// values per lane: each lane takes 4 consecutive entries from the block's
// start rounded down to a multiple of 4, skipping entries outside the block (the
// arrays carry STREAM_PAD zeroed entries, so the rounded loads stay in bounds).
// The products and their summation order are the same as the scalar stream's.
template <typename TM, typename TX, typename A, class Epi>
__device__ inline void stream_rows(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                   const TM *__restrict__ val, const TX *__restrict__ x,
                                   const int32_t *__restrict__ blk, int nblk, Epi &epi) {
    __shared__ A prod[STREAM_CAP];
    // blocks in launch order (a per-XCD contiguous remapping measured slower)
    const int lb = int(blockIdx.x);
    if (lb >= nblk) return;
    const int32_t r0 = blk[lb], r1 = blk[lb + 1];
    const int64_t k0 = rowptr[r0];
    const int n = int(rowptr[r1] - k0);
    if constexpr (std::is_same<TM, float>::value) {
        static_assert(STREAM_PAD >= 3, "the 4-wide stream reads up to 3 entries past a block");
        constexpr int UNITS = STREAM_CAP / (4 * TPB) + 1;
        const int64_t ka = k0 & ~int64_t(3);
        const int lead = int(k0 - ka);
        i32x4 c[UNITS];
        f32x4 v[UNITS];
#pragma unroll
        for (int u = 0; u < UNITS; ++u) {
            const int off = u * 4 * TPB + 4 * int(threadIdx.x);   // from ka
            if (off < lead + n) {
                c[u] = __builtin_nontemporal_load(reinterpret_cast<const i32x4 *>(col + ka + off));
                v[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(val + ka + off));
            }
        }
#pragma unroll
        for (int u = 0; u < UNITS; ++u) {
            const int off = u * 4 * TPB + 4 * int(threadIdx.x);
            if (off < lead + n) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int i = off + q - lead;
                    if (i >= 0 && i < n) prod[i] = A(v[u][q]) * A(x[c[u][q]]);
                }
            }
        }
    } else {
        constexpr int PER = STREAM_CAP / TPB;
        int32_t c[PER];
        TM v[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TPB;
            if (i < n) {
                c[u] = __builtin_nontemporal_load(col + k0 + i);
                v[u] = __builtin_nontemporal_load(val + k0 + i);
            }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * TPB;
            if (i < n) prod[i] = A(v[u]) * A(x[c[u]]);
        }
    }
    __syncthreads();
    for (int32_t row = r0 + int32_t(threadIdx.x); row < r1; row += TPB) {
        const int a = int(rowptr[row] - k0), b = int(rowptr[row + 1] - k0);
        A sum = A(0);
        for (int k = a; k < b; ++k) sum += prod[k];
        epi(row, sum);
    }
}

template <typename TY, typename A>
struct EpiStore {
    TY *y;
    __device__ void operator()(int32_t row, A s) const { y[row] = TY(s); }
};

template <typename T, typename A>
struct EpiResidual {
    const T *b;
    T *y;
    __device__ void operator()(int32_t row, A s) const { y[row] = T(A(b[row]) - s); }
};

// Chebyshev step in x alone: x_out = x_in + c1 (x_in - x_prev) + c2 (b - A x_in), where
// x_in - x_prev is the previous step's update; x_prev is read only when c1 != 0, and a
// null x_prev is the zero vector
template <typename T, typename A>
struct EpiCheb {
    const T *xin, *xprev, *b;
    T *xout;
    A c1, c2;
    bool use_prev;
    __device__ void operator()(int32_t row, A s) const {
        const A xi = A(xin[row]);
        const A r = A(b[row]) - s;
        const A dn = (use_prev ? c1 * (xi - (xprev ? A(xprev[row]) : A(0))) : A(0)) + c2 * r;
        xout[row] = T(xi + dn);
    }
};

// the Chebyshev step with the coefficients of the row's block
template <typename T, typename A>
struct EpiChebBlocks {
    const T *xin, *xprev, *b;
    T *xout;
    ChebBlocks cb;
    __device__ void coef(int32_t row, A &c1, A &c2) const {
        int q = 0;
#pragma unroll
        for (int k = 1; k < CHEB_BLOCKS; ++k) q += (k < cb.nb && row >= cb.start[k]) ? 1 : 0;
        c1 = A(cb.c1[0]);
        c2 = A(cb.c2[0]);
#pragma unroll
        for (int k = 1; k < CHEB_BLOCKS; ++k)
            if (q == k) {
                c1 = A(cb.c1[k]);
                c2 = A(cb.c2[k]);
            }
    }
    __device__ void operator()(int32_t row, A s) const {
        A c1, c2;
        coef(row, c1, c2);
        const A xi = A(xin[row]);
        const A r = A(b[row]) - s;
        const A dn = (c1 != A(0) ? c1 * (xi - (xprev ? A(xprev[row]) : A(0))) : A(0)) + c2 * r;
        xout[row] = T(xi + dn);
    }
};

template <typename T, typename A>
struct EpiAdd {
    T *x;
    __device__ void operator()(int32_t row, A s) const { x[row] = T(A(x[row]) + s); }
};

template <typename TM, typename TX, typename TY>
__global__ void __launch_bounds__(TPB) k_spmv(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                              const TM *__restrict__ val, const TX *__restrict__ x,
                                              const int32_t *__restrict__ blk, int nblk, TY *__restrict__ y) {
    using A = typename Acc<TM>::type;
    EpiStore<TY, A> e{y};
    stream_rows<TM, TX, A>(rowptr, col, val, x, blk, nblk, e);
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_residual(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ col, const T *__restrict__ val,
                                                  const T *__restrict__ x, const int32_t *__restrict__ blk,
                                                  int nblk, const T *__restrict__ b, T *__restrict__ y) {
    using A = typename Acc<T>::type;
    EpiResidual<T, A> e{b, y};
    stream_rows<T, T, A>(rowptr, col, val, x, blk, nblk, e);
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_cheb(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                                              const T *__restrict__ val, const T *__restrict__ xin,
                                              const int32_t *__restrict__ blk, int nblk, const T *__restrict__ b,
                                              const T *__restrict__ xprev, T *__restrict__ xout, double c1,
                                              double c2) {
    using A = typename Acc<T>::type;
    EpiCheb<T, A> e{xin, xprev, b, xout, A(c1), A(c2), c1 != 0.0};
    stream_rows<T, T, A>(rowptr, col, val, xin, blk, nblk, e);
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_cheb_blocks(const int64_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col, const T *__restrict__ val,
                                                     const T *__restrict__ xin, const int32_t *__restrict__ blk,
                                                     int nblk, const T *__restrict__ b, const T *__restrict__ xprev,
                                                     T *__restrict__ xout, ChebBlocks cb) {
    using A = typename Acc<T>::type;
    EpiChebBlocks<T, A> e{xin, xprev, b, xout, cb};
    stream_rows<T, T, A>(rowptr, col, val, xin, blk, nblk, e);
}

// first field-split step from x = 0: x = c2 b with the row's block coefficient
template <typename T>
__global__ void k_cheb_first_blocks(int64_t n, const T *__restrict__ b, T *__restrict__ xout, ChebBlocks cb) {
    using A = typename Acc<T>::type;
    EpiChebBlocks<T, A> e{nullptr, nullptr, b, xout, cb};
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        A c1, c2;
        e.coef(int32_t(i), c1, c2);
        xout[i] = T(c2 * A(b[i]));
    }
}

// first Chebyshev step from x = 0: x = c2 b (no operator application)
template <typename T>
__global__ void k_cheb_first(int64_t n, const T *__restrict__ b, T *__restrict__ xout, double c2) {
    using A = typename Acc<T>::type;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        xout[i] = T(A(c2) * A(b[i]));
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_prolong_add(const int64_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col, const T *__restrict__ val,
                                                     const T *__restrict__ xc, const int32_t *__restrict__ blk,
                                                     int nblk, T *__restrict__ x) {
    using A = typename Acc<T>::type;
    EpiAdd<T, A> e{x};
    stream_rows<T, T, A>(rowptr, col, val, xc, blk, nblk, e);
}

// ---------------------------------------------------------------- field-block stream (level 0)
// Level 0 keeps its vectors interleaved by field: the value of field f at vertex j
// of region r sits at off_r + 4 j + f, so one vertex's four fields are one 16- (or
// 32-) byte word.  Block b owns the block rows (region vertices) blk[b]..blk[b+1]-1
// of one region, whose entries (at most FB_CAP) are contiguous.  Phase 1: each
// thread takes entries tid + u*TPB, loads the column once, the four field values
// side by side and the four x values of that vertex as one vector gather, and
// stages the four products in LDS.  Phase 2: four threads per block row, one per
// field, sum the row's products in entry order (the scalar stream's order, so the
// sums match it bit for bit) and hand them to the epilogue with the DOF in the
// solver's order (off_r + 4 j + f) and in field-major order (off_r + f N_r + j).
typedef double f64x2 __attribute__((ext_vector_type(2)));

template <typename T>
__device__ inline void load4(const T *__restrict__ p, T (&v)[4], bool streaming) {
    if constexpr (std::is_same<T, float>::value) {
        const f32x4 w = streaming ? __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p))
                                  : *reinterpret_cast<const f32x4 *>(p);
        v[0] = w.x; v[1] = w.y; v[2] = w.z; v[3] = w.w;
    } else {
        const f64x2 w0 = streaming ? __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p))
                                   : *reinterpret_cast<const f64x2 *>(p);
        const f64x2 w1 = streaming ? __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p) + 1)
                                   : *(reinterpret_cast<const f64x2 *>(p) + 1);
        v[0] = w0.x; v[1] = w0.y; v[2] = w1.x; v[3] = w1.y;
    }
}

template <typename T, typename A, class Epi>
__device__ inline void stream_field_blocks(const FieldBlockView &fb, const T *__restrict__ val,
                                           const T *__restrict__ x, Epi &epi) {
    constexpr int PER = FB_CAP / TPB;
    __shared__ A prod[4][FB_CAP];
    const int lb = int(blockIdx.x);
    if (lb >= fb.nblk) return;
    const int32_t v0 = fb.blk[lb], v1 = fb.blk[lb + 1];
    const bool ext = v0 >= fb.Ni;                    // blocks never straddle the regions
    const int64_t Nr = ext ? fb.Ne : fb.Ni;
    const int64_t base = ext ? 4 * fb.Ni : 0;        // first DOF of the region
    const int32_t vfirst = ext ? int32_t(fb.Ni) : 0; // first block row of the region
    const int64_t k0 = fb.rowptr[v0];
    const int n = int(fb.rowptr[v1] - k0);
    const T *xr = x + base;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * TPB;
        if (i < n) {
            const int32_t c = __builtin_nontemporal_load(fb.col + k0 + i);
            T v[4], xv[4];
            load4<T>(val + 4 * (k0 + i), v, true);
            load4<T>(xr + 4 * int64_t(c), xv, false);
#pragma unroll
            for (int f = 0; f < 4; ++f) prod[f][i] = A(v[f]) * A(xv[f]);
        }
    }
    __syncthreads();
    const int f = int(threadIdx.x) & 3;
    for (int32_t row = v0 + int32_t(threadIdx.x >> 2); row < v1; row += TPB / 4) {
        const int a = int(fb.rowptr[row] - k0), b = int(fb.rowptr[row + 1] - k0);
        A sum = A(0);
        for (int k = a; k < b; ++k) sum += prod[f][k];
        const int64_t j = row - vfirst;
        epi(int32_t(base + 4 * j + f), int32_t(base + f * Nr + j), sum);
    }
}

// the residual goes out field-major: its only reader is the restriction, each of
// whose rows lies in one field
template <typename T, typename A>
struct FbResidualFM {
    const T *b;
    T *y;
    __device__ void operator()(int32_t i, int32_t ifm, A s) const { y[ifm] = T(A(b[i]) - s); }
};

template <typename T, typename A>
struct FbCheb {
    EpiCheb<T, A> e;
    __device__ void operator()(int32_t i, int32_t, A s) const { e(i, s); }
};

template <typename T>
__global__ void __launch_bounds__(TPB) k_fb_residual(FieldBlockView fb, const T *__restrict__ val,
                                                     const T *__restrict__ x, const T *__restrict__ b,
                                                     T *__restrict__ y) {
    using A = typename Acc<T>::type;
    FbResidualFM<T, A> e{b, y};
    stream_field_blocks<T, A>(fb, val, x, e);
}

template <typename T>
__global__ void __launch_bounds__(TPB) k_fb_cheb(FieldBlockView fb, const T *__restrict__ val,
                                                 const T *__restrict__ xin, const T *__restrict__ b,
                                                 const T *__restrict__ xprev, T *__restrict__ xout, double c1,
                                                 double c2) {
    using A = typename Acc<T>::type;
    FbCheb<T, A> e{EpiCheb<T, A>{xin, xprev, b, xout, A(c1), A(c2), c1 != 0.0}};
    stream_field_blocks<T, A>(fb, val, xin, e);
}

// ---------------------------------------------------------------- A by vertex
// The system matrix streamed by vertex (VtxView).  Phase 1: the block's values go
// to LDS with unit-stride non-temporal loads (8 per thread), and each neighbour's
// four x values are gathered once, as one 16- or 32-byte load, into LDS (a pair
// owns at least 4 entries, so a block has at most VTX_CAP / 4 pairs), beside the
// entry and pair starts of the block's vertices.  Phase 2: a row's entries are
// runs of consecutive pairs against one field (a concentration row: its own field,
// phi, the partners; the phi row: fields 0-3, the partners); one thread sums each
// run in entry order.  Phase 3: each row adds its run sums in order.  The result
// is deterministic (fixed order, no atomics); the association differs from the
// CSR stream's single chain, so the two agree to rounding.
template <typename TX>
__global__ void __launch_bounds__(TPB) k_spmv_vtx(VtxView A, const double *__restrict__ val,
                                                  const TX *__restrict__ x, double *__restrict__ y) {
    static_assert(VTX_CAP % TPB == 0, "whole entries per thread");
    constexpr int PER = VTX_CAP / TPB;
    constexpr int PPER = (VTX_CAP / 4 + TPB - 1) / TPB;
    __shared__ double vs[VTX_CAP];
    __shared__ TX xs[VTX_CAP];
    const int lb = int(blockIdx.x);
    if (lb >= A.nblk) return;
    const int32_t v0 = A.blk[lb], v1 = A.blk[lb + 1];
    const int64_t k0 = A.kblk[lb];
    const int n = int(A.kblk[lb + 1] - k0);
    const int32_t p0 = A.pblk[lb];
    const int np = A.pblk[lb + 1] - p0;
    __shared__ int vo[VTX_VMAX + 1], vp[VTX_VMAX + 1];   // entry and pair starts of the block's vertices
    __shared__ double part[VTX_RUNS * VTX_VMAX];        // run sums
    const int nvb = v1 - v0;
    for (int t = int(threadIdx.x); t <= nvb; t += TPB) {
        vo[t] = int(A.vptr[v0 + t] - k0);
        vp[t] = A.nptr[v0 + t] - p0;
    }
    double v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * TPB;
        if (i < n) v[u] = __builtin_nontemporal_load(val + k0 + i);
    }
    TX xv[PPER][4];
#pragma unroll
    for (int u = 0; u < PPER; ++u) {
        const int q = threadIdx.x + u * TPB;
        if (q < np) load4<TX>(x + 4 * int64_t(__builtin_nontemporal_load(A.nbr + p0 + q)), xv[u], false);
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * TPB;
        if (i < n) vs[i] = v[u];
    }
#pragma unroll
    for (int u = 0; u < PPER; ++u) {
        const int q = threadIdx.x + u * TPB;
        if (q < np)
#pragma unroll
            for (int g = 0; g < 4; ++g) xs[4 * q + g] = xv[u][g];
    }
    __syncthreads();
    // phase 2: one thread per run (14 per vertex: rows 0-2 have 3, row 3 has 5)
    for (int r = int(threadIdx.x); r < VTX_RUNS * nvb; r += TPB) {
        const int t = r / VTX_RUNS, k = r - t * VTX_RUNS;
        const int f = k < 9 ? k / 3 : 3, j = k < 9 ? k - 3 * f : k - 9;   // row, run within the row
        const int o0 = vo[t], len = vo[t + 1] - o0;
        const int pb = vp[t], npv = vp[t + 1] - pb;
        const int m = (len - 4 * npv) / 6;
        const int p = npv - m;
        const bool cf = v0 + t >= A.nv_i;   // partners first (region e)
        const int nsame = f < 3 ? 2 : 4;   // same-region runs in this row
        int o = o0 + (f < 3 ? f : 3) * (2 * m + p), base, cnt, g;
        const int js = cf ? j - 1 : j;      // index among the same-region runs
        if (cf ? j == 0 : j == nsame) {
            o += cf ? 0 : nsame * m;
            base = pb + (cf ? 0 : m);
            cnt = p;
            g = 3;
        } else {
            o += (cf ? p : 0) + js * m;
            base = pb + (cf ? p : 0);
            cnt = m;
            g = f < 3 ? (js == 0 ? f : 3) : js;
        }
        double sum = 0.0;
#pragma unroll 8
        for (int e = 0; e < cnt; ++e) sum += vs[o + e] * double(xs[4 * (base + e) + g]);
        part[r] = sum;
    }
    __syncthreads();
    // phase 3: each row adds its runs in order
    for (int r = int(threadIdx.x); r < 4 * nvb; r += TPB) {
        const int t = r >> 2, f = r & 3;
        const double *q = part + t * VTX_RUNS + (f < 3 ? 3 * f : 9);
        double sum = q[0] + q[1];
        sum += q[2];
        if (f == 3) {
            sum += q[3];
            sum += q[4];
        }
        y[4 * int64_t(v0 + t) + f] = sum;
    }
}

// level-0 vector from the solver's order (off_r + 4 j + f) to field-major order
// (off_r + f N_r + j), the order of the restriction's columns on level 0
template <typename T>
__global__ void k_to_field_major(int64_t Ni, int64_t Ne, const T *__restrict__ src, T *__restrict__ dst) {
    const int64_t n = 4 * (Ni + Ne);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        const bool ext = i >= 4 * Ni;
        const int64_t base = ext ? 4 * Ni : 0, li = i - base;
        dst[base + (li & 3) * (ext ? Ne : Ni) + (li >> 2)] = src[i];
    }
}

template <typename TA, typename TB>
__global__ void k_convert(int64_t n, const TA *__restrict__ a, TB *__restrict__ b) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        b[i] = TB(a[i]);
}

// coarsest level: x = A_c^{-1} b with one dense inverse per connected component
__global__ void __launch_bounds__(TPB) k_coarse(int64_t n, const int32_t *__restrict__ comp,
                                                const int32_t *__restrict__ cloc, const int32_t *__restrict__ cmem,
                                                const int64_t *__restrict__ cstart, const int64_t *__restrict__ coff,
                                                const double *__restrict__ inv, const double *__restrict__ b,
                                                double *__restrict__ x) {
    const int64_t row = (int64_t(blockIdx.x) * TPB + threadIdx.x) / 64;
    const int lane = threadIdx.x % 64;
    if (row >= n) return;
    const int32_t c = comp[row];
    const int64_t s0 = cstart[c];
    const int64_t nb = cstart[c + 1] - s0;
    const double *ir = inv + coff[c] + int64_t(cloc[row]) * nb;
    double s = 0.0;
    for (int64_t p = lane; p < nb; p += 64) s += ir[p] * b[cmem[s0 + p]];
    s = group_sum<64>(s);
    if (lane == 0) x[row] = s;
}

// ---------------------------------------------------------------- reductions
constexpr int KMAX = 16;

__device__ inline double wave_sum(double v) { return group_sum<64>(v); }

template <int K>
__device__ inline void block_store_sums(double (&acc)[K], int k, double *__restrict__ out) {
    __shared__ double sh[TPB / 64][K];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        if (q < k) {
            const double v = wave_sum(acc[q]);
            if (lane == 0) sh[wave][q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < k) {
        double s = 0.0;
#pragma unroll
        for (int w = 0; w < TPB / 64; ++w) s += sh[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

__global__ void __launch_bounds__(TPB) k_multi_dot(int64_t n, const double *__restrict__ V, int64_t ldv, int k,
                                                   const double *__restrict__ w, double *__restrict__ partial) {
    double acc[KMAX];
#pragma unroll
    for (int q = 0; q < KMAX; ++q) acc[q] = 0.0;
    for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
        const double wi = w[i];
#pragma unroll
        for (int q = 0; q < KMAX; ++q)
            if (q < k) acc[q] += V[q * ldv + i] * wi;
    }
    block_store_sums<KMAX>(acc, k, partial + int64_t(blockIdx.x) * KMAX);
}

__global__ void __launch_bounds__(TPB) k_gs_update(int64_t n, const double *__restrict__ V, int64_t ldv, int k,
                                                   const double *__restrict__ h, double *__restrict__ w,
                                                   double *__restrict__ partial) {
    extern __shared__ double sh_h[];
    for (int q = threadIdx.x; q < k; q += TPB) sh_h[q] = h[q];
    __syncthreads();
    double acc[1] = {0.0};
    for (int64_t i = int64_t(blockIdx.x) * TPB + threadIdx.x; i < n; i += int64_t(gridDim.x) * TPB) {
        double v = w[i];
        for (int q = 0; q < k; ++q) v -= sh_h[q] * V[q * ldv + i];
        w[i] = v;
        acc[0] += v * v;
    }
    block_store_sums<1>(acc, 1, partial + int64_t(blockIdx.x) * KMAX);
}

__global__ void __launch_bounds__(TPB) k_reduce_partials(int nblk, const double *__restrict__ partial,
                                                         double *__restrict__ out) {
    const int q = blockIdx.x;
    double acc[1] = {0.0};
    for (int b = threadIdx.x; b < nblk; b += TPB) acc[0] += partial[int64_t(b) * KMAX + q];
    block_store_sums<1>(acc, 1, out + q);
}

// w and v may alias (in-place normalisation)
__global__ void k_scale_inv_norm(int64_t n, const double *w, const double *__restrict__ nrm2, double *v) {
    const double s = 1.0 / sqrt(nrm2[0]);
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        v[i] = w[i] * s;
}

template <typename TZ>
__global__ void k_multi_axpy(int64_t n, const TZ *__restrict__ Z, int64_t ldz, int k, const double *__restrict__ c,
                             double *__restrict__ x) {
    extern __shared__ double sh_c[];
    for (int q = threadIdx.x; q < k; q += blockDim.x) sh_c[q] = c[q];
    __syncthreads();
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double s = x[i];
        for (int q = 0; q < k; ++q) s += sh_c[q] * double(Z[q * ldz + i]);
        x[i] = s;
    }
}

__global__ void k_axpby(int64_t n, double a, const double *x, double b, double *y) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        y[i] = a * x[i] + (b == 0.0 ? 0.0 : b * y[i]);
}

// out = a x + b y; operands may alias the output (element-wise)
__global__ void k_lincomb(int64_t n, double a, const double *x, double b, const double *y, double *out) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        out[i] = a * x[i] + b * y[i];
}

// operands may alias the output (element-wise)
__global__ void k_sub(int64_t n, const double *a, const double *b, double *y) {
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
        y[i] = a[i] - b[i];
}

inline unsigned grid_for(int64_t n, int per_block) {
    int64_t g = (n + per_block - 1) / per_block;
    if (g < 1) g = 1;
    return unsigned(g);
}

// grid for the row-block kernels: one workgroup per row block
inline unsigned block_grid(int64_t nblk) { return unsigned(nblk); }

inline unsigned stream_grid(int64_t n) {
    int64_t g = (n + TPB - 1) / TPB;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return unsigned(g);
}

}  // namespace

int reduce_blocks(int64_t n) {
    int64_t b = (n + TPB * 8 - 1) / (TPB * 8);
    if (b > 1024) b = 1024;
    if (b < 1) b = 1;
    return int(b);
}

template <typename TM, typename TX, typename TY>
void spmv(const CsrView &A, const TM *val, const TX *x, TY *y, hipStream_t s) {
    if (A.nblk == 0) return;
    hipLaunchKernelGGL((k_spmv<TM, TX, TY>), dim3(block_grid(A.nblk)), dim3(TPB), 0, s, A.rowptr, A.col, val, x, A.blk,
                       int(A.nblk), y);
}

template <typename T>
void to_field_major(const FieldBlockView &A, const T *src, T *dst, hipStream_t s) {
    const int64_t n = 4 * (A.Ni + A.Ne);
    if (n == 0) return;
    hipLaunchKernelGGL((k_to_field_major<T>), dim3(stream_grid(n)), dim3(TPB), 0, s, A.Ni, A.Ne, src, dst);
}

template <typename TX>
void spmv_vtx(const VtxView &A, const double *val, const TX *x, double *y, hipStream_t s) {
    if (A.nblk == 0) return;
    hipLaunchKernelGGL((k_spmv_vtx<TX>), dim3(block_grid(A.nblk)), dim3(TPB), 0, s, A, val, x, y);
}

template <typename T>
void residual(const CsrView &A, const T *val, const T *x, const T *b, T *y, hipStream_t s) {
    if (A.nblk == 0) return;
    hipLaunchKernelGGL((k_residual<T>), dim3(block_grid(A.nblk)), dim3(TPB), 0, s, A.rowptr, A.col, val, x, A.blk,
                       int(A.nblk), b, y);
}

template <typename T>
void cheb_step(const CsrView &A, const T *val, const T *x_in, const T *b, const T *x_prev, T *x_out, double c1,
               double c2, hipStream_t s) {
    if (A.nrows == 0) return;
    if (!x_in) {
        hipLaunchKernelGGL((k_cheb_first<T>), dim3(stream_grid(A.nrows)), dim3(TPB), 0, s, A.nrows, b, x_out, c2);
        return;
    }
    hipLaunchKernelGGL((k_cheb<T>), dim3(block_grid(A.nblk)), dim3(TPB), 0, s, A.rowptr, A.col, val, x_in, A.blk,
                       int(A.nblk), b, x_prev, x_out, c1, c2);
}

template <typename T>
void cheb_step_blocks(const CsrView &A, const T *val, const T *x_in, const T *b, const T *x_prev, T *x_out,
                      const ChebBlocks &cb, hipStream_t s) {
    if (A.nrows == 0) return;
    if (!x_in) {
        hipLaunchKernelGGL((k_cheb_first_blocks<T>), dim3(stream_grid(A.nrows)), dim3(TPB), 0, s, A.nrows, b, x_out,
                           cb);
        return;
    }
    hipLaunchKernelGGL((k_cheb_blocks<T>), dim3(block_grid(A.nblk)), dim3(TPB), 0, s, A.rowptr, A.col, val, x_in,
                       A.blk, int(A.nblk), b, x_prev, x_out, cb);
}

template <typename T>
void fb_residual(const FieldBlockView &A, const T *val, const T *x, const T *b, T *y, hipStream_t s) {
    if (A.nblk == 0) return;
    hipLaunchKernelGGL((k_fb_residual<T>), dim3(block_grid(A.nblk)), dim3(TPB), 0, s, A, val, x, b, y);
}

template <typename T>
void fb_cheb_step(const FieldBlockView &A, const T *val, const T *x_in, const T *b, const T *x_prev, T *x_out,
                  double c1, double c2, hipStream_t s) {
    const int64_t n = 4 * (A.Ni + A.Ne);
    if (n == 0) return;
    if (!x_in) {
        hipLaunchKernelGGL((k_cheb_first<T>), dim3(stream_grid(n)), dim3(TPB), 0, s, n, b, x_out, c2);
        return;
    }
    hipLaunchKernelGGL((k_fb_cheb<T>), dim3(block_grid(A.nblk)), dim3(TPB), 0, s, A, val, x_in, b, x_prev, x_out,
                       c1, c2);
}

template <typename T>
void prolong_add(const CsrView &P, const T *val, const T *xc, T *x, hipStream_t s) {
    if (P.nblk == 0) return;
    hipLaunchKernelGGL((k_prolong_add<T>), dim3(block_grid(P.nblk)), dim3(TPB), 0, s, P.rowptr, P.col, val, xc, P.blk,
                       int(P.nblk), x);
}

template <typename TA, typename TB>
void convert(int64_t n, const TA *a, TB *b, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL((k_convert<TA, TB>), dim3(stream_grid(n)), dim3(TPB), 0, s, n, a, b);
}

void coarse_solve(int64_t n, const int32_t *comp, const int32_t *cloc, const int32_t *cmem, const int64_t *cstart,
                  const int64_t *coff, const double *inv, const double *b, double *x, hipStream_t s) {
    if (n == 0) return;
    hipLaunchKernelGGL(k_coarse, dim3(grid_for(n * 64, TPB)), dim3(TPB), 0, s, n, comp, cloc, cmem, cstart, coff, inv,
                       b, x);
}

void multi_dot(int64_t n, const double *V, int64_t ldv, int k, const double *w, double *out, double *partial,
               int nblk, hipStream_t s) {
    for (int q0 = 0; q0 < k; q0 += KMAX) {
        const int kk = std::min(KMAX, k - q0);
        hipLaunchKernelGGL(k_multi_dot, dim3(nblk), dim3(TPB), 0, s, n, V + q0 * ldv, ldv, kk, w, partial);
        hipLaunchKernelGGL(k_reduce_partials, dim3(kk), dim3(TPB), 0, s, nblk, partial, out + q0);
    }
}

void gs_update(int64_t n, const double *V, int64_t ldv, int k, const double *h, double *w, double *partial, int nblk,
               hipStream_t s) {
    hipLaunchKernelGGL(k_gs_update, dim3(nblk), dim3(TPB), size_t(k > 0 ? k : 1) * sizeof(double), s, n, V, ldv, k, h,
                       w, partial);
}

void reduce_partials(int k, int nblk, const double *partial, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_reduce_partials, dim3(k), dim3(TPB), 0, s, nblk, partial, out);
}

void scale_by_inv_norm(int64_t n, const double *w, const double *nrm2, double *v, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_inv_norm, dim3(stream_grid(n)), dim3(TPB), 0, s, n, w, nrm2, v);
}

template <typename TZ>
void multi_axpy(int64_t n, const TZ *Z, int64_t ldz, int k, const double *coef, double *x, hipStream_t s) {
    if (k == 0) return;
    hipLaunchKernelGGL((k_multi_axpy<TZ>), dim3(stream_grid(n)), dim3(TPB), size_t(k) * sizeof(double), s, n, Z, ldz,
                       k, coef, x);
}

void add_scaled(int64_t n, double a, const double *x, double *y, hipStream_t s) {
    // y += a x
    hipLaunchKernelGGL(k_axpby, dim3(stream_grid(n)), dim3(TPB), 0, s, n, a, x, 1.0, y);
}

void axpby(int64_t n, double a, const double *x, double b, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(stream_grid(n)), dim3(TPB), 0, s, n, a, x, b, y);
}

void lincomb(int64_t n, double a, const double *x, double b, const double *y, double *out, hipStream_t s) {
    if (n > 0) hipLaunchKernelGGL(k_lincomb, dim3(stream_grid(n)), dim3(TPB), 0, s, n, a, x, b, y, out);
}

void sub(int64_t n, const double *a, const double *b, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_sub, dim3(stream_grid(n)), dim3(TPB), 0, s, n, a, b, y);
}

// explicit instantiations
template void to_field_major<double>(const FieldBlockView &, const double *, double *, hipStream_t);
template void to_field_major<float>(const FieldBlockView &, const float *, float *, hipStream_t);
template void spmv_vtx<double>(const VtxView &, const double *, const double *, double *, hipStream_t);
template void spmv_vtx<float>(const VtxView &, const double *, const float *, double *, hipStream_t);
template void spmv<double, double, double>(const CsrView &, const double *, const double *, double *, hipStream_t);
template void spmv<double, float, double>(const CsrView &, const double *, const float *, double *, hipStream_t);
template void spmv<float, float, float>(const CsrView &, const float *, const float *, float *, hipStream_t);
template void residual<double>(const CsrView &, const double *, const double *, const double *, double *,
                               hipStream_t);
template void residual<float>(const CsrView &, const float *, const float *, const float *, float *, hipStream_t);
template void cheb_step<double>(const CsrView &, const double *, const double *, const double *, const double *,
                                double *, double, double, hipStream_t);
template void cheb_step<float>(const CsrView &, const float *, const float *, const float *, const float *, float *,
                               double, double, hipStream_t);
template void cheb_step_blocks<double>(const CsrView &, const double *, const double *, const double *,
                                       const double *, double *, const ChebBlocks &, hipStream_t);
template void cheb_step_blocks<float>(const CsrView &, const float *, const float *, const float *, const float *,
                                      float *, const ChebBlocks &, hipStream_t);
template void fb_residual<double>(const FieldBlockView &, const double *, const double *, const double *, double *,
                                  hipStream_t);
template void fb_residual<float>(const FieldBlockView &, const float *, const float *, const float *, float *,
                                 hipStream_t);
template void fb_cheb_step<double>(const FieldBlockView &, const double *, const double *, const double *,
                                   const double *, double *, double, double, hipStream_t);
template void fb_cheb_step<float>(const FieldBlockView &, const float *, const float *, const float *, const float *,
                                  float *, double, double, hipStream_t);
template void prolong_add<double>(const CsrView &, const double *, const double *, double *, hipStream_t);
template void prolong_add<float>(const CsrView &, const float *, const float *, float *, hipStream_t);
template void convert<double, float>(int64_t, const double *, float *, hipStream_t);
template void convert<float, double>(int64_t, const float *, double *, hipStream_t);
template void convert<double, double>(int64_t, const double *, double *, hipStream_t);
template void multi_axpy<double>(int64_t, const double *, int64_t, int, const double *, double *, hipStream_t);
template void multi_axpy<float>(int64_t, const float *, int64_t, int, const double *, double *, hipStream_t);

}  // namespace launch
}  // namespace knp
