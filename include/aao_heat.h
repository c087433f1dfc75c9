/*
 * aao_heat.h -- C ABI of the MI355X all-at-once Radau IIA heat solver.
 *
 * Problem (paper Sec. 2, eq. (2.1)): u_t - div(kappa grad u) = f on the unit
 * square (dim = 2) or cube (dim = 3), homogeneous Dirichlet data, u(0) = u0.
 * Space: 5/7-point finite differences on n interior nodes per axis,
 * h = 1/(n+1), so the mass matrix is M = I and K = -div(kappa grad)_h.
 * Time: s-stage Radau IIA, nt steps of tau = T/nt.  Collecting the update
 * eq. (2.2) and the stage systems eq. (2.3) of every step gives the
 * all-at-once system eq. (2.4),  A x = [b; f].
 *
 * VECTOR LAYOUT (every double* vector argument below, length U):
 *   x = [v_0, ..., v_nt, V_{0,1}, ..., V_{0,s}, ..., V_{nt-1,s}]
 *   U = N (nt (s+1) + 1),  N = n^dim; each block is N contiguous FP64 values
 *   with x fastest: node (i, j[, k]) (0-based) at index i + n j (+ n^2 k),
 *   coordinates ((i+1)h, (j+1)h[, (k+1)h]).
 *
 * OWNERSHIP: vector arguments are caller-owned DEVICE pointers (HBM of the
 * current HIP device), never retained after the call returns.  The handle
 * owns host metadata only; its device memory is one caller-provided
 * workspace (aao_set_workspace), which must outlive the handle's use.
 * Host pointers are marked "host".
 *
 * STREAMS: all work is enqueued on the handle's stream (aao_set_stream;
 * default: the null stream).  aao_apply_* and aao_assemble_rhs return once
 * enqueued.  aao_solve / aao_solve_adjoint synchronise the stream once per
 * outer iteration and return when finished.
 *
 * ERRORS: every entry point returns an aao_status and never throws;
 * aao_last_error() gives a message for the last failure on a handle.
 * Calls on one handle must not overlap (one host thread at a time).
 */
#ifndef AAO_HEAT_H
#define AAO_HEAT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum aao_status {
  AAO_OK = 0,
  AAO_NOT_CONVERGED = 1,       /* maxit reached; x holds the last iterate     */
  AAO_INVALID_ARG = -1,        /* bad size, null pointer, unsupported option  */
  AAO_HIP_ERROR = -2,          /* a HIP runtime call failed                   */
  AAO_NONFINITE = -3,          /* NaN/Inf met in the Krylov recurrence        */
  AAO_WORKSPACE_TOO_SMALL = -4,
  AAO_NO_WORKSPACE = -5        /* a device call before aao_set_workspace      */
} aao_status;

/* Precision in which the preconditioner P-tilde is applied (Sec. 4;
 * approaches A1/A2/A4/A5 of Sec. 5).  The outer FGMRES is FP64 unless
 * opts.outer_precision says otherwise.  BF16/FP16 store the coarse
 * multigrid levels of the shifted-block solves in 16 bits with FP32
 * arithmetic; level 0, the inner GMRES, Rana coupling and S-tilde then run
 * in FP32 (approach A5: P-tilde single, P-tilde_int half).  FP16_ALL is
 * approach A4 (P-tilde and P-tilde_int in half precision): every vector
 * P-tilde stores is FP16 -- inner GMRES bases and results, Theta-tilde and
 * S-tilde results, all multigrid levels, the outer Z basis -- with FP32
 * arithmetic and no scaling.  A negative control. */
typedef enum aao_precision {
  AAO_PREC_FP64 = 0,
  AAO_PREC_FP32 = 1,
  AAO_PREC_BF16 = 2,
  AAO_PREC_FP16 = 3,
  AAO_PREC_FP16_ALL = 4
} aao_precision;

/* How S-tilde^{-1} of eq. (3.3) is applied inside P-tilde. */
typedef enum aao_schur {
  AAO_SCHUR_SWEEP = 0,     /* forward substitution in time, one step after the
                              other (the sequential form of Fig. 5.1)          */
  AAO_SCHUR_MGRIT = 1      /* two-level MGRIT in time (the parallel runs of
                              Sec. 5.2 replace the substitution by MGRIT):
                              F- or FCF-relaxation batched over the coarse
                              intervals, C-points every mgrit_cf steps, and a
                              coarse propagator that is the S-tilde step with
                              step size mgrit_cf tau                           */
} aao_schur;

/* Where P-tilde enters the outer FGMRES (Algorithm 1 of Sec. 4: P_L on the
 * left, P_R on the right). */
/* Precision of the outer solve (Algorithm 1's u and u_A). */
typedef enum aao_outer {
  AAO_OUTER_FP64 = 0,      /* the system solved in FP64 (approaches A1/A2/A5)  */
  AAO_OUTER_FP32 = 1       /* approach A3 of Sec. 5: the system solved in single
                              precision, simulated as the paper simulates its
                              lower precisions: the result of every outer step
                              (products with A, residuals, basis vectors, the
                              iterate) is rounded to FP32; stats.relres stays
                              the FP64 true residual.  A negative control: the
                              true residual stalls near FP32's unit roundoff
                              times the problem's conditioning               */
} aao_outer;

/* Orthogonalization of the inner GMRES (Algorithm 1 prints modified
 * Gram-Schmidt; both forms here are classical, batched over all instances). */
typedef enum aao_orth {
  AAO_ORTH_CGS2 = 0,       /* two classical passes (reorthogonalized)          */
  AAO_ORTH_CGS1 = 1,       /* one classical pass: the dots with the basis and
                              <w,w> together, h_{j+1,j} = sqrt(<w,w> - |h|^2);
                              a pass less per iteration, orthogonality as
                              classical Gram-Schmidt keeps it (inner only)     */
  AAO_ORTH_GRAM = 2        /* two classical passes with the second taken from
                              the Gram matrix of the basis: h = (2I - G) V^T w,
                              ||w - V h||^2 from <w,w>, h and G; one sweep
                              over the basis per iteration (outer only)        */
} aao_orth;

typedef enum aao_side {
  AAO_SIDE_RIGHT = 0,      /* P_L = I, P_R = P-tilde (the sequential runs)      */
  AAO_SIDE_LEFT = 1,       /* P_L = P-tilde, P_R = I (the parallel runs)        */
  AAO_SIDE_SPLIT = 2       /* P_L = P_R = P-tilde                              */
} aao_side;

/* Spatial discretisation. */
typedef enum aao_disc {
  AAO_DISC_FD = 0,         /* 5/7-point finite differences on the unit square
                              or cube, M = I                                   */
  AAO_DISC_Q1 = 1,         /* bilinear finite elements (Sec. 2 and Sec. 5 use
                              Q1/Q2) on the square [0, length]^2, uniform grid,
                              with their mass matrix M: Phi and Psi1 carry M,
                              Theta_hat = I_s (x) M + tau A (x) K, the
                              multigrid solves M + a K, and S-tilde applies
                              M^{-1} by 20 steps of Chebyshev semi-iteration
                              with the Jacobi splitting (Sec. 5; D^{-1} M has
                              its spectrum in [1/4, 9/4]).  2D, kappa = NULL,
                              nu1, nu2 <= 3; the transposed solve and the
                              kappa gradient are not available                */
  AAO_DISC_Q2 = 2          /* biquadratic finite elements (Sec. 5, Tables 1-4)
                              under the same conditions as AAO_DISC_Q1: n odd
                              and >= 3 (n interior nodes per axis, (n + 1) / 2
                              elements of side 2 length / (n + 1)), nodes
                              ordered x fastest like every grid here; the
                              Chebyshev mass solve uses the Q2 interval
                              [1/4, 25/16]; the multigrid's first coarse level
                              holds the element vertices                       */
} aao_disc;

/* Problem description (Sec. 2).  kappa: host pointer to N nodal
 * diffusivities (> 0), copied at creation, or NULL for kappa = 1.  A face
 * between two interior nodes carries their harmonic mean, a face to the
 * boundary the interior node's value. */
typedef struct aao_desc {
  int dim;                 /* 2 or 3                                          */
  int n;                   /* interior nodes per axis, >= 2                   */
  int s;                   /* Radau IIA stages, 1..3                          */
  int nt;                  /* time steps, >= 1                                */
  double T;                /* final time, > 0                                 */
  const double* kappa;     /* host, N values, or NULL                          */
  int disc;                /* aao_disc                                         */
  double length;           /* side of the square for AAO_DISC_Q1/Q2 (0 = 1); the
                              finite-difference domain is the unit square or
                              cube (0 or 1 only)                               */
} aao_desc;

/* Solver options.  Fill with aao_default_opts, then override. */
typedef struct aao_opts {
  int restart;             /* outer FGMRES restart length (Algorithm 1)       */
  int maxit;               /* maximum outer iterations                        */
  double tol;              /* stop when ||rhs - A x|| <= tol ||rhs|| (FP64)    */
  int inner_k;             /* GMRES iterations per Theta-tilde application    */
  int cycles;              /* V-cycles per shifted-block solve                 */
  int nu1, nu2;            /* Jacobi sweeps before / after coarse correction  */
  double omega;            /* Jacobi weight; 0 = 0.8 (2D) or 6/7 (3D)         */
  int precision;           /* aao_precision of P-tilde                         */
  int use_graph;           /* 1: replay P-tilde as a captured HIP graph        */
  int mg_tail_max;         /* largest multigrid level (nodes) solved inside one
                              workgroup's LDS (2D); 0 = 1024, extended to one
                              more level of at most 64 x 64 when the
                              register-resident tail takes it (FP32, BF16,
                              FP16 arithmetic); capped by LDS                  */
  int coarse_max;          /* coarsening stops at a level of at most this many
                              nodes, solved exactly; 0 = 256.  Up to 1024 for
                              2D constant kappa (fast diagonalization), up to
                              256 otherwise (dense inverse)                    */
  double inner_tol;        /* an inner GMRES solve (Theta-tilde and every
                              S-tilde step) stops early once its residual
                              estimate is <= inner_tol times its initial
                              residual (Sec. 5.2 runs 1e-3 / 1e-6); 0 = always
                              inner_k iterations                               */
  int schur;               /* aao_schur                                        */
  int mgrit_cf;            /* MGRIT coarsening factor in time, 2..64 (0 = 8)   */
  int mgrit_iters;         /* MGRIT iterations, 1..nt (0 = 1); with
                              ceil(nt / mgrit_cf) - 1 of them the result is the
                              forward substitution's                           */
  int mgrit_fcf;           /* 1: FCF-relaxation, 0: F-relaxation               */
  int side;                /* aao_side.  RIGHT stops on the true residual
                              ||rhs - A x|| <= tol ||rhs||.  LEFT and SPLIT
                              follow Algorithm 1: the solve ends when the
                              least-squares residual of the preconditioned
                              system is <= tol times the first cycle's
                              ||P_L^{-1} rhs - P_L^{-1} A x0|| (or, at a
                              restart, when the preconditioned residual of x
                              is); stats.relres reports the true residual,
                              which P-tilde's nonlinearity (inner GMRES) can
                              leave larger                                     */
  int outer_precision;     /* aao_outer                                        */
  int mg_low_from;         /* BF16/FP16 preconditioners: the first multigrid
                              level stored in 16 bits; the levels above it stay
                              FP32 (per-level decreasing precision, Sec. 4).
                              0 = 1, every coarse level; a value beyond the last
                              level keeps them all in FP32                     */
  int mg_coarse_fp32;      /* 1: the coarse solve (2D: the one-workgroup tail
                              and its exact coarsest solve; 3D: the exactly
                              solved coarsest level) stays FP32 where
                              mg_low_from puts the levels above it in 16 bits
                              -- a coarse-solve precision apart from the
                              smoother's (Sec. 4); 0 = no                      */
  int relax_matvec;        /* 1: iteration-dependent precision of the products
                              with A inside an FGMRES cycle (Sec. 4 names this
                              relaxation, after Simoncini and Szyld, as future
                              work): the product of iteration k may carry a
                              relative error up to eta = tol beta0 / rho, rho
                              the least-squares residual after iteration k-1
                              (beta at a cycle's first) and beta0 the first
                              cycle's; it is rounded to BF16 when eta >= 10 *
                              2^-8, else to FP32 when eta >= 10 * 2^-24
                              (simulated, as the paper simulates its lower
                              precisions); products that start a cycle stay
                              FP64.  stats.relaxed_* count them.  0 = off      */
  int mgrit_coarse_k;      /* inner GMRES iterations of MGRIT's coarse
                              propagator (the S-tilde step of mgrit_cf tau);
                              the fine propagator keeps inner_k.  A cheaper
                              coarse propagator shortens the sequential
                              coarse sweep; with one MGRIT iteration S-tilde
                              stays an approximation either way.  0 = inner_k */
  int schur_k;             /* inner GMRES iterations of the Theta-tilde solves
                              inside S-tilde's steps (the substitution's, and
                              MGRIT's fine propagator); Theta-tilde's own
                              block solve keeps inner_k.  0 = inner_k          */
  int inner_orth;          /* aao_orth: orthogonalization of the inner GMRES
                              (CGS2 or CGS1)                                   */
  int outer_orth;          /* aao_orth: orthogonalization of the outer FGMRES
                              (CGS2 or GRAM)                                   */
} aao_opts;

/* Solve statistics (host struct filled by aao_solve*). */
typedef struct aao_stats {
  int outer_iterations;    /* total FGMRES iterations (preconditioner calls)  */
  int restarts;            /* restart cycles begun                            */
  double relres;           /* final true relative residual, FP64              */
  double time_ms;          /* wall time of the solve (device work included)   */
  double precond_ms;       /* time inside P-tilde applications                */
  double history[128];     /* relative residual estimate per iteration        */
  int history_len;
  int inner_solves;        /* inner GMRES solves run (one per time step of each
                              Theta-tilde application, one per S-tilde step)   */
  long long inner_iterations;  /* inner GMRES iterations over all those solves;
                              inner_iterations / inner_solves is the mean
                              count per solve (inner_k unless inner_tol stops
                              solves early)                                    */
  double theta_ms;         /* time in the Theta-tilde phase of P-tilde
                              (eq. (3.2): the batched block-diagonal solve)    */
  double schur_ms;         /* time in the S-tilde phase (eq. (3.3): the
                              sweep in time)                                   */
  int relaxed_fp32;        /* products with A rounded to FP32 (relax_matvec)  */
  int relaxed_bf16;        /* products with A rounded to BF16 (relax_matvec)  */
} aao_stats;

typedef struct aao_problem aao_problem;   /* opaque handle */

/* Defaults: restart 30, maxit 100, tol 1e-8, inner_k 3, cycles 1,
 * nu1 = nu2 = 2, omega 0, precision FP64, use_graph 1, mg_tail_max 0,
 * coarse_max 0, inner_tol 0, schur AAO_SCHUR_SWEEP, mgrit_cf 8,
 * mgrit_iters 1, mgrit_fcf 0, side RIGHT, outer_precision FP64,
 * mg_low_from 0, relax_matvec 0, mg_coarse_fp32 0, mgrit_coarse_k 0, schur_k 0, inner_orth and
 * outer_orth CGS2.  With use_graph the
 * first application of P-tilde for a given (inner_k, cycles, transpose) is
 * captured into a HIP graph on a private stream and later applications
 * replay it on the handle's stream (inputs and outputs pass through fixed
 * workspace buffers); results are bitwise identical to direct launches. */
void aao_default_opts(aao_opts* o);

/* Build a handle: Radau IIA tableau by collocation, Crout factor of A_RK
 * (Rana's stage preconditioner), multigrid hierarchy of the shifted blocks
 * I + tau L_ii K.  Host-only work; no device memory is touched.
 * Returns AAO_INVALID_ARG for unsupported sizes or options. */
int aao_create_problem(const aao_desc* d, const aao_opts* o, aao_problem** out);

/* Bytes of device workspace needed by every call on this handle. */
int aao_workspace_size(const aao_problem* h, size_t* bytes);

/* Hand over a device workspace of at least aao_workspace_size bytes
 * (alignment 256).  Uploads the handle's constant tables into it, on the
 * handle's stream.  The workspace stays caller-owned. */
int aao_set_workspace(aao_problem* h, void* dev_ptr, size_t bytes);

/* Replace the diffusivity of a handle created with variable kappa (Sec. 2,
 * eq. (2.1)): values is a DEVICE pointer to N nodal values, kappa itself
 * (is_log = 0) or theta = log kappa (is_log = 1; the library takes exp).
 * Rebuilds the face coefficients, the coarse Galerkin stencils and the
 * coarsest-level inverses on the host and copies them into the workspace in
 * place, so the captured P-tilde graphs stay valid (synchronises the
 * handle's stream).  AAO_INVALID_ARG for a constant-kappa handle or values
 * that are not finite and > 0; the handle is unchanged on error. */
int aao_set_kappa(aao_problem* h, const double* values, int is_log);

/* Stream for all later work (a hipStream_t; NULL = default stream). */
int aao_set_stream(aao_problem* h, void* stream);

/* Release host metadata and pinned host buffers.  The workspace is not freed. */
int aao_destroy(aao_problem* h);

/* Host copies of the tableau: A (s*s, row-major), b (s), c (s).  Any of the
 * pointers may be NULL. */
int aao_get_tableau(const aao_problem* h, double* A, double* b, double* c);

/* N = n^dim and U = N (nt (s+1) + 1). */
int aao_sizes(const aao_problem* h, int64_t* N, int64_t* U);

/* y = A x, eq. (2.4), matrix-free in FP64.  x, y: device, U values, must
 * not overlap. */
int aao_apply_A(aao_problem* h, const double* x, double* y);

/* y = A^T x (the transposed blocks of eq. (2.4)).  Same conventions. */
int aao_apply_AT(aao_problem* h, const double* x, double* y);

/* z = P-tilde^{-1} r, eqs. (3.2)-(3.3): Theta-tilde (inner GMRES with Rana's
 * preconditioner and multigrid block solves) for all steps at once, the
 * Psi1 coupling, then the S-tilde forward sweep in time.  Computed in the
 * handle's precision; r and z are FP64 at the boundary.  The map is
 * nonlinear in r (inner GMRES).  r, z: device, U values, must not overlap. */
int aao_apply_P(aao_problem* h, const double* r, double* z);

/* aao_apply_P with the inner settings overridden for this call: inner_k
 * GMRES iterations per Theta-tilde application (1 <= inner_k <= the
 * handle's opts.inner_k, which sizes the workspace) and `cycles` V-cycles
 * per shifted-block solve (>= 1).  As they grow, P-tilde tends to the
 * ideal P of eq. (3.1), for which A P^{-1} - I is nilpotent of degree two
 * (Sec. 3). */
int aao_apply_P_with(aao_problem* h, const double* r, double* z, int inner_k, int cycles);

/* z_b = (`cycles` geometric multigrid V-cycles from zero) applied to
 * (I + a K) z_b = r_b for the blocks b = 0 .. count-1: the shifted-block
 * solve inside Rana's preconditioner (Sec. 4), with a = tau L_ii, L the
 * lower Crout factor of the Radau IIA matrix A (transpose = 0) or of A^T
 * (transpose = 1, the adjoint preconditioner), i = `stage`.
 * The hierarchy, smoother and coarse solve are the handle's (opts.nu1,
 * nu2, omega; coarsening to at most 256 nodes, solved exactly).
 * r, z: device, count * N values each, block b at offset b * N, in the
 * preconditioner's working type: double for AAO_PREC_FP64, float for
 * FP32, BF16 and FP16 (the 16-bit formats are the coarse levels' storage),
 * FP16 (IEEE binary16) for FP16_ALL.
 * 1 <= count <= nt, 0 <= stage < s, 1 <= cycles <= 64; r and z must not
 * overlap.  Asynchronous on the handle's stream. */
int aao_apply_mg(aao_problem* h, int transpose, int stage, int count, int cycles, const void* r, void* z);

/* The multigrid hierarchy: *levels levels, level l with nodes[l] grid
 * nodes (written for l < cap; nodes may be NULL when cap == 0).  Level
 * l+1 keeps every second node of level l along each axis; the last level
 * has at most 256 nodes and is solved exactly.  Levels >= *tail_level
 * run inside one workgroup's LDS (2D; *tail_level = *levels when none
 * do); that split depends on the device, so it needs the workspace set
 * (AAO_NO_WORKSPACE otherwise, with *levels and nodes still filled).
 * Host-only. */
int aao_mg_levels(const aao_problem* h, int cap, int64_t* nodes, int* levels, int* tail_level);

/* rhs = [b; f] of eq. (2.4): b_0 = u0, b_{n>=1} = 0, then f.
 * f: device, nt*s*N values in (step, stage, node) order, f_{n,i} sampled
 * at t_n + c_i tau; u0: device, N values; rhs: device, U values. */
int aao_assemble_rhs(aao_problem* h, const double* f, const double* u0, double* rhs);

/* Solve A x = rhs by restarted FGMRES (Algorithm 1; P-tilde on the side
 * opts.side, right by default) in FP64 with P-tilde applied in the handle's
 * precision.
 * x: device, U values, initial guess on entry, solution on exit.
 * st: host, may be NULL.  Returns AAO_OK or AAO_NOT_CONVERGED (x holds the
 * last iterate, st filled) or an error. */
int aao_solve(aao_problem* h, const double* rhs, double* x, aao_stats* st);

/* aao_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * The handle's workspace is placed in a static device array of
 * AAO_NO_ALLOC_SCRATCH_BYTES that the library holds on every device it runs
 * on until the process ends; problems whose aao_workspace_size exceeds it
 * are rejected with AAO_WORKSPACE_TOO_SMALL.  No device memory is allocated
 * or freed, no graph is captured and no event is created (theta_ms and
 * schur_ms stay 0).  The handle needs no aao_set_workspace; if it has one,
 * that workspace is left untouched.  The array is shared by all calls on a
 * device and is re-initialised by each call: calls that overlap in time on
 * one device race and must be serialised by the caller.  Synchronous on the
 * handle's stream.  Results equal aao_solve's. */
#define AAO_NO_ALLOC_SCRATCH_BYTES (64u << 20)
int aao_solve_no_alloc(aao_problem* h, const double* rhs, double* x, aao_stats* st);

/* Solve A^T lam = g the same way with the transposed preconditioner.
 * g, lam: device, U values; lam holds the initial guess on entry. */
int aao_solve_adjoint(aao_problem* h, const double* g, double* lam, aao_stats* st);

/* Gradient of a loss with respect to theta = log kappa at the nodes, given
 * the forward solution x and the adjoint lam = A^{-T} dL/dx:
 * g_p = - sum_{n,i} lam_{V,n,i}^T (dK/dtheta_p) w_{n,i},
 * w_{n,i} = v_n + tau sum_j a_ij V_{n,j}.  x, lam: device, U values;
 * g: device, N values (overwritten). */
int aao_grad_logkappa(aao_problem* h, const double* x, const double* lam, double* g);

/* Launch timing of the shifted-block solve: one V-cycle from zero on
 * `count` blocks (1..nt) of stage `stage`, timed two ways over `reps`
 * (1..1000) repetitions on the handle's stream.  In situ: the cycle runs with
 * a HIP event after every kernel launch, so a launch's time is the interval
 * since the previous event -- the kernel as it runs inside a solve (inputs
 * just written by the launch before it, cold caches) plus the dispatch gap
 * after an event.  Alone: the cycle is captured as a graph and every launch
 * is replayed by itself, `reps` copies back to back, so its time is the warm
 * kernel plus the short gap between graph nodes.  Writes the number of
 * launches per cycle to *nlaunch, their mean in-situ / alone microseconds to
 * us / us_alone [0..min(cap, *nlaunch)-1] (either may be NULL), their labels
 * ("kernel@level", one per line, NUL-terminated, truncated to labels_cap) to
 * labels (may be NULL), and the mean time of the whole cycle replayed as a
 * graph to *total_us.  Uses the handle's inner-GMRES buffers as scratch
 * (their contents are overwritten).  Synchronous. */
int aao_profile_vcycle(aao_problem* h, int stage, int count, int reps, char* labels, size_t labels_cap, double* us,
                       double* us_alone, int cap, int* nlaunch, double* total_us);

/* Launch shapes of the multigrid kernels, chosen by aao_autotune.  The
 * tiled level kernels run short tiles or tall ones (and level 0 as row
 * marches) from tall_min_b blocks per launch on; in 3D, level 0 runs as
 * z-marches from tall_min_b blocks on; the register tail takes a 64 x 64
 * level too when tail_extend.  None of them changes the cycle's
 * arithmetic. */
typedef struct aao_tune {
  int tall_min_b;          /* chosen threshold (1, 8 or 2^30 = never)         */
  int tail_extend;         /* chosen: 1 or 0                                   */
  int from_cache;          /* 1: read from the cache file, nothing timed       */
  int blocks[3];           /* block counts timed: one S-tilde step, one MGRIT
                              relaxation batch, the Theta-tilde batch          */
  double weight[3];        /* V-cycles per P-tilde application at each         */
  double us[6][3];         /* mean V-cycle microseconds of candidate c
                              (tall_min_b = {1, 8, 2^30}[c % 3], tail_extend =
                              c < 3) at each block count (0: not timed)        */
} aao_tune;

/* Time the candidate launch shapes (`reps` V-cycles each, on stage 0) at
 * the block counts P-tilde uses and keep the one with the least V-cycle time
 * per application (weighted by the counts above).  With cache_path (host
 * string, may be NULL), a line for this device architecture and problem
 * shape is read from that text file if present -- then nothing is timed --
 * or appended after timing.  Drops captured graphs when the shapes change.
 * out: host, may be NULL.  Needs the workspace; synchronous. */
int aao_autotune(aao_problem* h, int reps, const char* cache_path, aao_tune* out);

/* Set the launch shapes directly (a choice made earlier by aao_autotune):
 * tall_min_b >= 1, tail_extend 0 or 1.  Drops captured graphs when they
 * change. */
int aao_set_launch_shapes(aao_problem* h, int tall_min_b, int tail_extend);

/* Message of the last failure on h (or of the last failed creation if h is
 * NULL).  Valid until the next call on h. */
const char* aao_last_error(const aao_problem* h);

/* ------------------------------------------------------------------------
 * Batches of independent problems
 *
 * Many all-at-once problems (each with its own grid, stages, steps and
 * diffusivity; the same options) are handled as one batch: batch vectors
 * are single device buffers holding the problems' vectors back to back, at
 * the offsets reported by aao_batch_offsets.  A batch call runs the
 * problems on `streams` HIP streams driven by host threads, largest problem
 * first, so that independent solves overlap on the device (Sec. 5: the
 * method's time-parallel phase is one batch dimension; separate problems
 * are another).  Batch calls start after the work already queued on the
 * batch's stream (aao_batch_set_stream; default: the null stream), return
 * once every problem is done, and leave that stream waiting for them.
 * ------------------------------------------------------------------------ */
typedef struct aao_batch aao_batch;   /* opaque */

/* Streams a batch may use: the device runs the work of one process on four
 * hardware queues, so more streams would only contend for them. */
#define AAO_BATCH_MAX_STREAMS 4

/* Create a batch of `count` problems described by descs[0..count-1], all
 * with the options *opts (NULL: defaults), to be run on `streams` streams
 * (1..AAO_BATCH_MAX_STREAMS).  Errors as aao_create_problem, with the failing problem named in
 * aao_batch_last_error(NULL). */
int aao_create_batch(const aao_desc* descs, int count, const aao_opts* opts, int streams, aao_batch** out);

/* Number of problems in the batch (0 for NULL). */
int aao_batch_count(const aao_batch* b);

/* Prefix offsets (count + 1 values each, any pointer may be NULL): problem
 * i's unknowns occupy [unknowns[i], unknowns[i+1]) of a batch vector (U_i
 * values), its nodes [nodes[i], nodes[i+1]) of a batch node field (u0,
 * log-kappa gradients; N_i values) and its forcing values [forcing[i],
 * forcing[i+1]) of a batch forcing buffer (nt_i s_i N_i values). */
int aao_batch_offsets(const aao_batch* b, int64_t* unknowns, int64_t* nodes, int64_t* forcing);

/* Device bytes of the batch workspace (the problems' workspaces back to
 * back), and attaching it (256-byte aligned, caller-owned, device current
 * at this call is the batch's device).  Creates the batch's streams. */
int aao_batch_workspace_size(const aao_batch* b, size_t* bytes);
int aao_batch_set_workspace(aao_batch* b, void* dev_ptr, size_t bytes);

/* Stream the batch calls are ordered after (and that waits for them). */
int aao_batch_set_stream(aao_batch* b, void* stream);

/* Borrow problem i's handle (owned by the batch; valid until
 * aao_batch_destroy), e.g. for its tableau or single-problem calls. */
int aao_batch_problem(aao_batch* b, int i, aao_problem** h);

/* aao_assemble_rhs for every problem: f, u0, rhs are batch buffers laid out
 * by the forcing, node and unknown offsets. */
int aao_batch_assemble_rhs(aao_batch* b, const double* f, const double* u0, double* rhs);

/* aao_solve / aao_solve_adjoint for every problem; rhs and x (g and lam) are
 * batch vectors; stats: NULL or count entries in problem order.  Returns
 * AAO_OK when every problem converged, AAO_NOT_CONVERGED when some did not,
 * else the first error (aao_batch_last_error names the problem). */
int aao_batch_solve(aao_batch* b, const double* rhs, double* x, aao_stats* stats);
int aao_batch_solve_adjoint(aao_batch* b, const double* g, double* lam, aao_stats* stats);

/* aao_grad_logkappa for every problem: x, lam batch vectors; grad a batch
 * node field. */
int aao_batch_grad_logkappa(aao_batch* b, const double* x, const double* lam, double* grad);

/* Message of the last failure on b (or of the last failed batch creation if
 * b is NULL). */
const char* aao_batch_last_error(const aao_batch* b);

/* Free the batch and its problems (not the caller's workspace). */
int aao_batch_destroy(aao_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* AAO_HEAT_H */
