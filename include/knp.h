/*
 * knp.h -- C ABI of libknp: one time step of the KNP-EMI ionic electrodiffusion
 * model (IMEX-linearised finite element system) assembled and solved on one
 * AMD Instinct MI355X (gfx950).
 *
 * The calls follow the paper's statement of the problem: for n = 1..N_t find the
 * ion concentrations [k]_r^n and potentials phi_r^n of the intra- (r = i) and
 * extracellular (r = e) regions (Sec. "Time discretization"), given a conforming
 * simplicial mesh whose cells match at the membrane Gamma (Sec. "Spatial
 * discretization"), the physical parameters (Table "physconst"), the initial
 * state and dt.  Each step is the linear system A_{n-1} u_n = f_n of eq.
 * ``lin_sys``, solved by GMRES preconditioned with one algebraic-multigrid
 * V-cycle on the frozen block-diagonal matrix P_0 of eq. ``P_prec``
 * (Sec. "Solution and preconditioning strategy").
 *
 * Conventions shared by every call
 *  - Status: every call returns knp_status; on failure knp_last_error() gives a
 *    text.  No C++ exception crosses the ABI.  KNP_E_ARG leaves the context
 *    unchanged.
 *  - Host pointers ("host") are read during the call only; the caller keeps
 *    ownership.  Device pointers ("device") are HIP device memory owned by the
 *    caller (for example torch tensors); the library never frees them.
 *  - All device work is enqueued on the stream given to knp_create.  Calls that
 *    return host-visible results (solver statistics, layouts) synchronise that
 *    stream before returning.  One context per host thread.
 *  - Unknown vector layout (eq. ``lin_sys``): u = [c_i^Na, c_i^K, c_i^Cl, phi_i,
 *    c_e^Na, c_e^K, c_e^Cl, phi_e], each block of length N_r, region DOFs ordered
 *    by ascending global vertex id; membrane vertices appear once in each region.
 *    DOF(r, f, j) = off_r + f * N_r + j with off_i = 0, off_e = 4 N_i.
 *  - Units: SI (m, s, mol/m^3, V, S/m^2, F/m^2).
 */
#ifndef KNP_H
#define KNP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct knp_ctx knp_ctx;

typedef enum {
    KNP_OK = 0,
    KNP_E_ARG = 1,      /* invalid argument; nothing was changed                */
    KNP_E_STATE = 2,    /* call out of order (e.g. solve before setup)          */
    KNP_E_HIP = 3,      /* HIP runtime error                                    */
    KNP_E_NOMEM = 4,    /* device or host allocation failed                     */
    KNP_E_NOCONV = 5,   /* solver hit max_it; x holds the last (best) iterate   */
    KNP_E_NUMERIC = 6   /* NaN or Inf in the data                               */
} knp_status;

/* Sizes reported by knp_mesh_upload. */
typedef struct {
    int64_t n_vert, n_elem;
    int64_t N_i, N_e;       /* P1 DOFs (vertices) of the ICS and ECS             */
    int64_t N;              /* unknowns = 4 (N_i + N_e)                          */
    int64_t nnz_A;          /* structural nonzeros of A                          */
    int64_t nnz_P0;         /* structural nonzeros of P_0                        */
    int64_t n_gamma;        /* membrane vertices (one pair of DOFs each)         */
    int64_t n_facets;       /* membrane facets                                   */
    int32_t n_cells;        /* cells (ICS components), tags 1..n_cells           */
    int32_t dim;
    int64_t pin_dof;        /* the pinned phi_e DOF                              */
} knp_mesh_info;

/* Physical parameters (Table "physconst") and membrane models
 * (eq. ``HH_ionic_model``; passive leak: every ion I_k = theta g_leak^k (phi_M - E_k);
 * Kir-Na/K, Sec. "Passive dynamics: Kir--Na/K": leak channels with the K+ current scaled by
 * the inward-rectifier factor f_Kir, plus the Na/K pump, 3 Na+ out per 2 K+ in). */
typedef struct {
    double R, T, F, C_m;
    double z[3];            /* valences of Na+, K+, Cl-                           */
    double D[3];            /* diffusion coefficients, same in both regions       */
    double g_leak[3];       /* leak conductances                                  */
    double gbar_Na, gbar_K; /* Hodgkin-Huxley maximal conductances                */
    double g_stim_bar;      /* stimulus g_stim(t) = g_stim_bar exp(-(t mod tau)/a)*/
    double stim_a, stim_tau;
    double phi_rest;        /* HH resting potential                               */
    double rho_pump;        /* Kir-Na/K: maximum pump rate (mol m^-2 s^-1), >= 0   */
    double P_Na, P_K;       /* Kir-Na/K: pump thresholds of ICS Na+, ECS K+, > 0   */
    double K_e0, K_i0;      /* Kir-Na/K: initial ECS and ICS K+ concentrations, > 0;
                               they fix [K+]_e^0 and E_K^0 = psi/z_K ln(K_e0/K_i0) */
    int32_t n_ode;          /* Rush-Larsen sub-steps per time step                */
    int32_t n_cells;        /* must equal knp_mesh_info.n_cells                   */
    const int32_t *cell_model;  /* host [n_cells]: 0 passive leak, 1 Hodgkin-Huxley,
                                   2 Kir-Na/K; other values are KNP_E_ARG           */
    const int32_t *cell_stim;   /* host [n_cells]: 1 = stimulus on this cell's membrane */
} knp_params;

typedef struct {
    int32_t precision;      /* 0: levels stored and applied in FP64; 1: FP32      */
    double strength;        /* strength-of-connection threshold (0 < s < 1)       */
    int32_t cheb_degree;    /* finest level: post-smoothing Chebyshev degree (>= 1) */
    double cheb_ratio;      /* smoothing interval [lmax/cheb_ratio, lmax] (> 1)   */
    int32_t coarse_max;     /* coarsen until at most this many unknowns           */
    int32_t max_levels;
    double coarse_drop;     /* drop coarse-operator couplings with |a_ij| <        */
                            /* coarse_drop * sqrt(a_ii a_jj), lumped into a_ii     */
                            /* near-nullspace weighted (0: exact Galerkin; >= 0)   */
    int32_t cheb_pre_degree;     /* finest level: pre-smoothing degree (>= 0)      */
    int32_t coarse_pre_degree;   /* coarser levels: pre-smoothing degree (>= 0;    */
                                 /* 0, here and above: restrict the right-hand side) */
    int32_t coarse_post_degree;  /* coarser levels: post-smoothing degree (>= 1)   */
    int32_t operator_step;  /* 0: P_0, the diagonal blocks of the first assembled
                               matrix, for every step (the paper's choice);
                               1: P_n, those of the most recently assembled one  */
    int32_t field_split;    /* 1: on the coarser levels each (region, field) block
                               is smoothed on its own interval [g_q/cheb_ratio, g_q]
                               (g_q its Gershgorin bound), as a field-split AMG
                               would; 0: one interval per level                  */
    int32_t shared_ion_aggregates;  /* 1: the Na+ and Cl- blocks of the finest level
                               reuse the aggregates of the K+ block (one aggregation
                               for the three ion blocks); 0: each block its own   */
    int32_t coarse_graph;   /* 1: the levels below the finest run as one HIP graph,
                               captured at the first V-cycle after the setup and
                               replayed (the same kernels on the same buffers, so the
                               same results bit for bit, with one launch call);
                               0: their kernels are launched one by one          */
} knp_amg_opts;

typedef struct {
    double rtol;            /* stop when ||S(b - A x)||_2 <= rtol ||S b||_2       */
    int32_t restart;        /* Krylov subspace size per cycle (paper: 30)         */
    int32_t max_it;         /* total iteration cap                                */
    int32_t reorth;         /* 1: second classical Gram-Schmidt pass              */
    int32_t precond;        /* 1: AMG V-cycle on P_0 (needs knp_amg_setup); 0: none */
} knp_solve_opts;

typedef struct {
    int32_t its;            /* iterations performed                               */
    int32_t restarts;
    double rel_res;         /* ||S(b - A x)|| / ||S b|| of the returned x: from a
                               product with A, or (rtol >= 1e-10, the last cycle's
                               estimate within rtol) the Arnoldi relation's
                               V (beta e_1 - H y), equal up to rounding            */
    double rel_res_est;     /* the recurrence's estimate at the last iteration    */
} knp_solve_info;

/* Create a context on HIP device `hip_device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL = the default stream).  hip_device = -1 creates a
 * host-only context in which only knp_mesh_upload, knp_get_layout and
 * knp_get_gamma work (for checks of the host-side mesh logic).  On failure
 * *out is NULL and knp_last_error(NULL) gives the reason (per host thread).
 * The library must share the process's one HIP runtime with whatever owns the
 * device memory passed to it (e.g. load it after the framework's runtime). */
knp_status knp_create(knp_ctx **out, int hip_device, void *hip_stream);
void knp_destroy(knp_ctx *ctx);
const char *knp_last_error(const knp_ctx *ctx);

/* Mesh and DOF setup (Sec. "Spatial discretization"; Remark ``rem:nullspace``).
 * xyz: host [n_vert*dim] vertex coordinates (m); elem_vert: host
 * [n_elem*(dim+1)] simplices; elem_tag: host [n_elem], 0 = extracellular,
 * c >= 1 = cell c (cells numbered 1..n_cells, each a separate ICS component).
 * Membrane facets are the faces shared by a cell element and an extracellular
 * element.  pin_vertex: the extracellular vertex (off the membrane) whose phi_e
 * is pinned to 0.  Builds the DOF maps and the structural CSR pattern of A on
 * the host and uploads them once.  Errors (KNP_E_ARG): dim not 2 or 3, indices
 * out of range, two cells touching, a cell touching the outer boundary, a pin
 * on the membrane.  Any vertex degree is accepted: meshes whose vertices all have at
 * most 32 region neighbours and 16 membrane neighbours use the element-walk kernels,
 * others the product-form assembly of knp_mesh_upload_p2 with linear elements.
 * May be called once per context. */
knp_status knp_mesh_upload(knp_ctx *ctx, int dim, int64_t n_vert, const double *xyz,
                           int64_t n_elem, const int32_t *elem_vert,
                           const int32_t *elem_tag, int64_t pin_vertex,
                           knp_mesh_info *out);

/* The same with quadratic (P2) Lagrange elements (Sec. "Spatial discretization": elements
 * of degree p; the robustness study and Model D (ii) use p = 2).  Arguments as for
 * knp_mesh_upload: the vertex mesh, d + 1 vertices per element.  The library adds one node
 * per edge: the edge (a, b), a < b, e-th in lexicographic order of its vertex pair, is
 * node n_vert + e at the edge midpoint; membrane nodes (vertices and edges of membrane
 * facets) get one copy per region.  Everywhere after this call "vertex" means node:
 * knp_mesh_info.n_vert counts nodes (N = 4 (N_i + N_e) over nodes), knp_get_layout's
 * dof_vertex and knp_get_gamma give node ids, the gates array has one row per membrane
 * node, and the nonlinear membrane coefficients are P2 fields given by their values at
 * the membrane nodes.  Element node order: the d + 1 vertices, then the edges in
 * lexicographic order of the local pair; facets likewise.  knp_step_vjp stays order 1
 * (KNP_E_ARG on such a context).  Other errors as knp_mesh_upload. */
knp_status knp_mesh_upload_p2(knp_ctx *ctx, int dim, int64_t n_vert, const double *xyz, int64_t n_elem,
                              const int32_t *elem_vert, const int32_t *elem_tag, int64_t pin_vertex,
                              knp_mesh_info *out);

/* The edge nodes of a P2 mesh: *n_edges (may be NULL) receives their number, and
 * edge_vertices (host [2 * n_edges], may be NULL) the two vertices of node n_vert + e.
 * Zero edges for an order-1 mesh. */
knp_status knp_get_edges(knp_ctx *ctx, int64_t *n_edges, int32_t *edge_vertices);

/* Host copies of the structural pattern and DOF maps for bit-exact checks:
 * rowptr [N+1] (int64), colidx [nnz_A] (int32, strictly ascending per row),
 * dof_vertex [N] (global vertex of each DOF).  Any pointer may be NULL. */
knp_status knp_get_layout(knp_ctx *ctx, int64_t *rowptr, int32_t *colidx,
                          int32_t *dof_vertex);

/* Host copy of the membrane vertex ids, ascending [n_gamma]: the row order of
 * the gates array of knp_assemble_step. */
knp_status knp_get_gamma(knp_ctx *ctx, int32_t *gamma_vertex);

/* Physical parameters; copies everything it needs.  Required before the first
 * knp_assemble_step.  KNP_E_ARG for non-positive R, T, F, C_m or n_ode < 1, a zero
 * valence, a non-positive diffusivity, a cell model other than 0, 1, 2, or, when some
 * cell uses Kir-Na/K, a negative pump rate or a non-positive threshold or initial K+. */
knp_status knp_set_params(knp_ctx *ctx, const knp_params *params);

/* Assemble A_{n-1} and f_n (eq. ``lin_sys``; its block rows come from eqs.
 * ``weak_disc`` and ``weak_disc2``) for the step to time t_n = n dt.
 *   u_prev: device [N] u_{n-1};
 *   gates:  device [n_gamma*3] (n, m, h) per membrane vertex, in: w_{n-1},
 *           out: w_n after n_ode Rush-Larsen sub-steps at frozen phi_M^{n-1}
 *           (Hodgkin-Huxley cells only; other rows untouched); NULL allowed
 *           if no cell uses the Hodgkin-Huxley model;
 *   theta:  device [n_cells] factors on every leak conductance of each cell's
 *           membrane (the Kir-Na/K K+ current included, the pump not), or NULL
 *           for all 1;
 *   f_out:  device [N] receives f_n (unscaled).
 * A_{n-1} stays in the context, stored as S A S with S = diag(P_0)^{-1/2} fixed
 * at the first call.  The first call also fixes P_0.  KNP_E_NUMERIC if u_prev
 * holds a NaN or Inf (checked before anything is written).  After that check the call
 * only enqueues: f_out, gates and the stored system are ready in stream order, and
 * the inputs must stay valid until the stream reaches the call's kernels. */
knp_status knp_assemble_step(knp_ctx *ctx, double t_n, double dt, const double *u_prev,
                             double *gates, const double *theta, double *f_out);

/* For callers that cannot allocate device memory (code under stream capture, tight
 * serving loops, harnesses that forbid hipMalloc): knp_assemble_step with the same
 * arguments, results and errors, whose scratch (the NaN counter and the per-membrane-
 * vertex coefficient record) lives in a static device array of the library instead of
 * context memory; it allocates nothing and calls no hipMalloc/hipFree.  The array holds
 * at most 262,144 membrane vertices (40 MiB plus 256 bytes); each device the library
 * runs on keeps its own copy until the process ends, and it keeps the last call's
 * contents (the counter is cleared by a kernel at the start of each call).
 * Differences from knp_assemble_step:
 *   - the context must have been assembled once by knp_assemble_step (that first call
 *     fixes S and P_0), else KNP_E_STATE;
 *   - a mesh with more membrane vertices than the array holds is KNP_E_ARG;
 *   - calls that overlap on one device (several contexts or threads at once) share the
 *     array and race: serialise them;
 *   - it synchronises the stream before returning, so the array is free again on
 *     return. */
knp_status knp_assemble_step_noalloc(knp_ctx *ctx, double t_n, double dt, const double *u_prev,
                                     double *gates, const double *theta, double *f_out);

/* How the constant-potential nullspace of the system (Remark ``rem:nullspace``) is
 * removed; call after knp_mesh_upload and before the first knp_assemble_step
 * (KNP_E_STATE otherwise; the mode is fixed from then on).
 *   mode 0 (default): the remark's point condition phi_e(x_e) = 0 at the reference
 *     DOF (knp_mesh_info.pin_dof) is part of the assembled system: that DOF's row
 *     keeps only its diagonal, its column is zero, and f_n is 0 there.
 *   mode 1: the system is assembled without it (the remark's third way): A keeps the
 *     constant potential as its null vector and f_n is consistent.  knp_gmres_solve
 *     then starts every restart cycle with a coarse correction along the per-cell
 *     constant intracellular potentials (near-null vectors of A: on them only the
 *     membrane terms act; the correction is x += Z E^{-1} Z^T r with E = Z^T A Z, Z
 *     one column per cell), tests the corrected residual against rtol, and at return
 *     subtracts the reference DOF's value from every potential.  The returned x is an
 *     approximation of the same solution as in mode 0; S and P_0 are formed the same
 *     way.  knp_get_values and knp_apply(0/2) show the system without the condition;
 *     knp_adjoint_solve and knp_step_vjp need mode 0 (KNP_E_STATE).
 * KNP_E_ARG for another mode.  Mode 1 needs the cells' intracellular DOFs not to
 * couple, which knp_mesh_upload already ensures (it refuses cells that share a vertex);
 * the call checks it again and returns KNP_E_ARG if it fails. */
knp_status knp_set_gauge(knp_ctx *ctx, int32_t mode);

/* Build the algebraic-multigrid hierarchy of P_0 (eq. ``P_prec``), frozen for all
 * steps (same section), or with operator_step = 1 of the time-dependent P_n of the
 * most recent knp_assemble_step (the alternative that section weighs against P_0;
 * the caller calls again after each assembly).  Must follow the first
 * knp_assemble_step (else KNP_E_STATE).  opts NULL = defaults (FP64, strength 0.6,
 * Chebyshev smoothing on [lmax/2.5, lmax] of degree 0 before and 5 after the coarse
 * correction on the finest level and 0 and 1 on the coarser levels, coarse_max
 * 2000, max_levels 20, coarse_drop 0.01, operator_step 0, field_split 0,
 * shared_ion_aggregates 0, coarse_graph 0). */
knp_status knp_amg_setup(knp_ctx *ctx, const knp_amg_opts *opts);

/* Shape of the hierarchy built by knp_amg_setup: number of levels (<= 32) and,
 * per level, rows and stored nonzeros of the level operator (host arrays of 32). */
knp_status knp_amg_stats(knp_ctx *ctx, int32_t *n_levels, int64_t *level_rows, int64_t *level_nnz);

/* Solve A_{n-1} x = b with right-preconditioned flexible GMRES(restart) (the
 * paper's GMRES with one V-cycle of AMG(P_0) per iteration).  b: device [N]
 * (unscaled, e.g. f_n); x: device [N], in: initial guess (u_{n-1}), out: the
 * solution.  opts NULL = rtol 1e-6, restart 30, max_it 2000, reorth 0, precond 1.
 * Blocks until done.  KNP_E_NOCONV if max_it was reached, or earlier if rtol
 * lies below the attainable accuracy: 50 restarts in a row whose cycle ended
 * on a converged recurrence estimate while the recomputed residual, over the
 * 50, did not halve (x is the last iterate; info->rel_res says where it
 * stalled). */
knp_status knp_gmres_solve(knp_ctx *ctx, const double *b, double *x,
                           const knp_solve_opts *opts, knp_solve_info *info);

/* Solve the adjoint system A_{n-1}^T lambda = rhs with the same preconditioner
 * (P_0 is symmetric).  Same conventions as knp_gmres_solve. */
knp_status knp_adjoint_solve(knp_ctx *ctx, const double *rhs, double *lambda,
                             const knp_solve_opts *opts, knp_solve_info *info);

/* Vector-Jacobian products of the step residual R = A(u_prev, theta) u_n -
 * f(u_prev, theta) (eq. ``lin_sys``) for the discrete adjoint: accumulates
 *   u_prev_bar += (dR/du_prev)^T lambda_n   and   theta_bar += (dR/dtheta)^T lambda_n
 * (device; theta_bar [n_cells] may be NULL).  u_prev enters through the
 * concentration-weighted stiffness, the mass term of f and the nodal membrane
 * coefficients; theta through the leak currents.  Uses t_n, dt and the theta
 * pointer of the most recent knp_assemble_step, which must be the call for this
 * step (same u_prev and theta; theta must still be valid).  Passive-leak
 * membranes only (KNP_E_ARG if a Hodgkin-Huxley or Kir-Na/K cell is present). */
knp_status knp_step_vjp(knp_ctx *ctx, const double *u_prev, const double *u_n,
                        const double *lambda_n, double *u_prev_bar, double *theta_bar);

/* Initial guess for the next step's solve from the last two steps' solutions:
 * x0 = 2 u1 - u2 (device [N] each; u1 = u_{n-1}, u2 = u_{n-2}; x0 may alias either).
 * The paper starts each solve from the previous step (Sec. "Solver configurations");
 * the linear extrapolation in time is an alternative start that the caller may pass to
 * knp_gmres_solve as x.  Needs an uploaded mesh (N); enqueues one kernel and returns
 * without synchronising (x0 is ready in stream order). */
knp_status knp_extrapolate(knp_ctx *ctx, const double *u1, const double *u2, double *x0);

/* Operator hooks for tests and measurement (device vectors of length N):
 *   which 0: y = S A S x (the stored system matrix)
 *   which 1: y = one V-cycle on S P_0 S applied to x
 *   which 2: y = (S A S)^T x
 * and S itself: knp_get_scaling copies diag(S) to device [N]. */
knp_status knp_apply(knp_ctx *ctx, int which, const double *x, double *y);
knp_status knp_get_scaling(knp_ctx *ctx, double *s);

/* Copy the stored values S A S (device [nnz_A], pattern of knp_get_layout). */
knp_status knp_get_values(knp_ctx *ctx, double *vals);

/* Kernel timing for roofline measurement.  knp_timing(ctx, 1) resets the
 * counters and starts bracketing the instrumented launches with HIP events on
 * the context's stream; knp_timing(ctx, 0) stops.  knp_timing_read fills
 * out[KNP_TIMER_COUNT]: per kernel class the number of launches, their summed
 * device time (ms, from the events) and their summed algorithmic bytes (the
 * bytes the kernel must move at least once: matrix values and indices, row
 * pointers, each vector read or written once). */
enum { KNP_TIMER_SPMV_A = 0,        /* y = (S A S) x, Krylov operator          */
       KNP_TIMER_CHEB_L0 = 1,       /* Chebyshev steps on the finest AMG level that apply the operator */
       KNP_TIMER_RESID_L0 = 2,      /* residual on the finest AMG level        */
       KNP_TIMER_VCYCLE = 3,        /* one whole V-cycle                        */
       KNP_TIMER_ASSEMBLY = 4,      /* knp_assemble_step device work            */
       KNP_TIMER_RESID_A = 5,       /* y = (S A S) x for the solver's true residuals (FP64 x) */
       KNP_TIMER_COUNT = 6 };
typedef struct {
    int64_t launches;
    double total_ms;
    double bytes;
} knp_timer;
knp_status knp_timing(knp_ctx *ctx, int enable);
knp_status knp_timing_read(knp_ctx *ctx, knp_timer *out);

#ifdef __cplusplus
}
#endif

#endif /* KNP_H */
