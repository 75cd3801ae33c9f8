/*
 * mgm.h -- C ABI of the MI355X (gfx950) implementation of the solve phase of
 * MGM, the meshfree geometric multilevel method of Wright, Jones & Shankar
 * (arXiv 2204.06154), for the RBF-FD / GFD surface-Laplacian systems
 * L_h u = f defined on point-cloud surfaces.
 *
 * Conventions for every call:
 *  - Every function returns an mgm_status: 0 = MGM_OK, > 0 a warning, < 0 an
 *    error. After an error, outputs are unspecified; the handle stays usable
 *    unless the error was MGM_E_HIP. mgm_last_error() returns a thread-local
 *    human-readable detail string for the last failing call of this thread.
 *  - Host pointers ("h_" or documented as host) are borrowed for the duration
 *    of the call and copied as needed. Device pointers ("d_") are borrowed,
 *    caller-owned, contiguous FP64 arrays on the handle's device. The handle
 *    owns all internal host and device memory until mgm_destroy().
 *  - Calls that take a stream are ordered on that HIP stream (a hipStream_t
 *    passed as void*; NULL = the legacy default stream). Inputs must be ready
 *    on that stream; outputs are ready when the stream reaches the call's end.
 *  - Vectors are in the caller's point order. Internal reorderings (colouring)
 *    are applied and undone inside the library.
 *  - Calls on one handle must not overlap (one stream at a time per handle).
 */
#ifndef MGM_H
#define MGM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct mgm_ctx *mgm_handle;

typedef enum {
  MGM_OK = 0,
  MGM_NOT_CONVERGED = 1,       /* solve hit maxit; best iterate returned */
  MGM_E_ARG = -1,              /* invalid argument or parameter */
  MGM_E_ALLOC = -2,            /* host or device allocation failed */
  MGM_E_HIP = -3,              /* HIP runtime error (handle no longer usable) */
  MGM_E_STENCIL_SINGULAR = -4, /* a local weight system is singular (pivot ~0) */
  MGM_E_DUP_POINTS = -5,       /* two input points coincide */
  MGM_E_ZERO_DIAG = -6,        /* a level operator has a zero diagonal entry */
  MGM_E_COARSE_SINGULAR = -7,  /* coarsest-level LU hit a zero pivot */
  MGM_E_BREAKDOWN = -8,        /* Krylov breakdown */
  MGM_E_NONFINITE = -9,        /* NaN/Inf in an input or an iterate */
  MGM_E_SYNC = -10             /* a one-launch smoother sweep (gs_flow) gave up
                                  waiting for a coupled patch: the results of
                                  the calls since the last check are invalid;
                                  the sweeps are resynchronised (mgm_check) */
} mgm_status;

/* Discretisation of the Laplace-Beltrami operator (Sec. 2). */
enum { MGM_RBFFD = 0, MGM_GFD = 1 };
/* Problem (Sec. 1.1, eq. discrete_system): POISSON: L_h = D_h, solved as the
 * bordered system [L b^T; b 0][u; lambda] = [f; 0] with b = 1^T (Sec. 4.4,
 * eq. saddle_point); SCREENED: L_h = I - mu D_h. With mu < 0 this is the
 * shifted operator of shift-invert eigensolves (Sec. 6.1), L_h = -mu (D_h - sigma I)
 * with sigma = 1/mu: mu = -1 gives D_h + I (sigma = -1), which is indefinite. */
enum { MGM_SCREENED = 0, MGM_POISSON = 1 };
/* V-cycle arithmetic: FP64; FP32 values and vectors; FP16 operator values with
 * one FP32 scale per row, FP32 vectors. Outer Krylov and coarsest LU: FP64. */
enum { MGM_FP64 = 0, MGM_FP32 = 1, MGM_FP16 = 2 };
/* Smoother sweeps (Sec. 4.3: forward or backward Gauss-Seidel). */
enum { MGM_GS_FWD = 0, MGM_GS_BWD = 1 };
/* Cycle (Alg. 3 is the V-cycle; Sec. 4.5 names F- and W-cycles as options):
 * the coarse problem of a level is solved by one V-cycle of the next level,
 * by two W-cycles, or by an F-cycle followed by a V-cycle. A second visit
 * continues from the first visit's iterate (pre-smoothing with the current
 * multiplier, residual f - L e - b mu and constraint residual rho - b.e). */
enum { MGM_CYCLE_V = 0, MGM_CYCLE_W = 1, MGM_CYCLE_F = 2 };
/* Outer iteration (Sec. 4.6): right-preconditioned FGMRES(restart) or
 * BiCGSTAB, or the stationary V-cycle iteration u <- u + M(f - A u). */
enum { MGM_FGMRES = 0, MGM_BICGSTAB = 1, MGM_STATIONARY = 2 };

typedef struct {
  int32_t disc;           /* MGM_RBFFD | MGM_GFD */
  int32_t phs_order;      /* k of the PHS kernel r^(2k+1) (RBF-FD only), 1..8
                             (its Laplacian at the stencil centre is finite
                             only for k >= 1) */
  int32_t poly_degree;    /* l, degree of the bivariate polynomials, 0..8 */
  int32_t stencil_size;   /* n, stencil size, centre included, > L = (l+1)(l+2)/2 */
  double  gfd_alpha;      /* alpha of the GFD Gaussian weight (Sec. 2.3) */
  int32_t problem;        /* MGM_SCREENED | MGM_POISSON */
  double  mu;             /* screened: L = I - mu D, mu finite and non-zero */
  int32_t interp_size;    /* m, coarse stencil of the interpolation (Sec. 3); 3 */
  int32_t coarsen_factor; /* N_{j+1} = floor(N_j / factor) (Sec. 4.1); 4 */
  int32_t n_min;          /* > 0: p = floor(log(N_1/N_min)/log 4) + 1 (Alg. 2);
                             setup rejects p < 2 (MGM_E_ARG): the cycle needs
                             one smoothed level above the coarsest */
  int32_t n_coarse_max;   /* used when n_min == 0: coarsen while N_j > this */
  int32_t nu1, nu2;       /* pre/post smoothing sweeps (Alg. 3) */
  int32_t pre_smoother;   /* MGM_GS_FWD | MGM_GS_BWD */
  int32_t post_smoother;  /* MGM_GS_FWD | MGM_GS_BWD */
  int32_t precision;      /* MGM_FP64 | MGM_FP32 | MGM_FP16 (V-cycle only) */
  int32_t use_graph;      /* 1: replay the V-cycle as a captured HIP graph */
  int32_t device_weights; /* 1: stencil weights by the batched device solver */
  int32_t gs_block;       /* smoother blocking: 0 = plain multicolour GS (Jones-
                             Plassmann colours); B in 1..256 = patch-blocked
                             multicolour GS: patches of B points by recursive
                             coordinate bisection, patch graph coloured by
                             recursive largest first, in-patch graphs by DSATUR,
                             one workgroup per patch; levels
                             with rows longer than gs_max_width entries stay
                             plain */
  int32_t cycle;          /* MGM_CYCLE_V | MGM_CYCLE_W | MGM_CYCLE_F */
  int32_t device_setup;   /* 1: kNN searches (k <= 128) and the Galerkin sparse
                             products on the device; results identical to the
                             host path */
  int32_t gs_flow;        /* 1 (default): each patch-blocked sweep is one
                             launch in which a patch starts once the coupled
                             patches before it in the sweep order are done
                             (the same GS order and bit-identical results as
                             0: one launch per patch colour); each patch
                             loads the distinct rows outside it that its
                             entries reference once, into LDS (levels whose
                             patches reference at most 1024 such rows, and
                             with 32-bit vectors only levels of at most 512
                             patches; the others load per entry). 2: one
                             launch per sweep with loads per entry on every
                             level. A wait is
                             bounded; if one gives up, the next mgm_solve,
                             mgm_level_op or mgm_check returns MGM_E_SYNC */
  int32_t gs_max_width;   /* part of the smoother ordering: a level is
                             patch-blocked (gs_block > 0) only if none of its
                             rows has more than this many entries; 1..96 (the
                             widest row the patch kernels hold), default 96 */
} mgm_params;

/* Paper defaults (Table 1): RBF-FD, k = l = 3, n = 20, forward GS, nu = 1,
 * m = 3, factor 4, N_min = 250, screened with mu = 1; FP64 V-cycle, graphs
 * on, device weights and device setup on, gs_block = 256, V-cycle,
 * one-launch sweeps (gs_flow = 1), gs_max_width = 96. */
void mgm_default_params(mgm_params *p);

/* Preprocessing phase (Alg. 2): kNN stencils (Sec. 2), tangent-plane weights
 * (Sec. 2.1-2.3), L_1 (eq. discrete_system), then for each level: weighted
 * sample elimination (Sec. 4.1), PHS interpolation (Sec. 3, eq. rbf_fd_interp),
 * R = P^T, Galerkin L_{j+1} = R L_j P (eq. galerkin; bordered:
 * eq. gco_saddle_point), multicolour ordering, and the coarsest LU.
 *   h_xyz, h_normals: host, n x 3 row-major FP64 (normals need not be unit).
 *   device: HIP device ordinal that all later calls use; -1 builds a host-only
 *   handle (no GPU needed) that supports mgm_export and mgm_destroy only.
 *   stream: stream for the uploads.
 * Errors: MGM_E_ARG (bad sizes/params, too few points for one coarse level),
 * MGM_E_DUP_POINTS, MGM_E_STENCIL_SINGULAR, MGM_E_ZERO_DIAG,
 * MGM_E_COARSE_SINGULAR, MGM_E_NONFINITE, MGM_E_ALLOC, MGM_E_HIP. */
mgm_status mgm_setup(const double *h_xyz, const double *h_normals, int64_t n,
                     const mgm_params *params, int32_t device, void *stream,
                     mgm_handle *out);

/* Change the V-cycle precision (MGM_FP64/FP32/FP16) of an existing hierarchy;
 * reduced-precision operator copies are built on first use. */
mgm_status mgm_set_precision(mgm_handle h, int32_t precision);

/* One V(nu1,nu2)-cycle (Alg. 3) with zero initial guess: d_z = M d_r.
 * Length n (screened) or n+1 (Poisson: the last entry is the constraint
 * residual on input and the multiplier correction on output). d_r and d_z
 * may not alias. MGM_E_NONFINITE is not checked here (no host sync). */
mgm_status mgm_vcycle(mgm_handle h, const double *d_r, double *d_z, void *stream);

/* Apply the fine-level system operator (eq. discrete_system; bordered for
 * Poisson): d_y = A d_x, lengths as for mgm_vcycle. */
mgm_status mgm_apply(mgm_handle h, const double *d_x, double *d_y, void *stream);

typedef struct {
  int32_t krylov;   /* MGM_FGMRES | MGM_BICGSTAB | MGM_STATIONARY */
  int32_t restart;  /* FGMRES restart length m (1..200) */
  int32_t maxit;    /* maximum preconditioner applications */
  double  rtol;     /* stop when |f - A u|_2 <= rtol |f|_2 (true FP64 residual) */
  int32_t use_x0;   /* 1: d_u holds the initial guess; 0: start from zero */
} mgm_solve_opts;

typedef struct {
  int32_t iters;          /* preconditioner applications (Sec. 5 counting) */
  int32_t restarts;
  double  rel_res_est;    /* last Krylov estimate of the relative residual */
  double  rel_res_true;   /* |f - A u|_2 / |f|_2 recomputed in FP64 at the end */
  double  lambda;         /* Poisson: the Lagrange multiplier; else 0 */
} mgm_solve_info;

/* MGM-preconditioned solve (Sec. 4.6): right-preconditioned FGMRES(m) with
 * CGS2 or BiCGSTAB, entirely on device in FP64 around the V-cycle.
 *   d_f: right-hand side, length n (Poisson: n+1 with last entry 0).
 *   d_u: solution (and initial guess if use_x0), same length.
 *   h_res_hist: nullable host array of maxit+1 doubles receiving the relative
 *   residual estimate after each preconditioner application (entry 0 = 1).
 * Synchronises the stream once per outer iteration. Returns MGM_OK or
 * MGM_NOT_CONVERGED (best iterate in d_u), MGM_E_BREAKDOWN, MGM_E_NONFINITE. */
mgm_status mgm_solve(mgm_handle h, const double *d_f, double *d_u,
                     const mgm_solve_opts *opts, mgm_solve_info *info,
                     double *h_res_hist, void *stream);

/* Synchronises the stream and reports whether a one-launch smoother sweep
 * (gs_flow = 1) gave up waiting for a coupled patch since the last check:
 * MGM_E_SYNC if so (the results of the calls since then are invalid; the
 * sweeps' ticket counters and flags have been reset, so later calls are
 * valid again), else MGM_OK. mgm_solve and mgm_level_op make the same check
 * before returning; mgm_vcycle does not synchronise and leaves it to them or
 * to this call. */
mgm_status mgm_check(mgm_handle h, void *stream);

/* For tests of the give-up path: bound of each wait of the one-launch
 * sweeps, in ticks of the GPU's constant-rate real-time counter (100 MHz on
 * MI355X); ticks < 0 restores the default 2^24 (~0.17 s). With a bound too
 * small for the waits to succeed, sweeps give up (every kernel still ends)
 * and the next check returns MGM_E_SYNC. Waits for the device first. */
mgm_status mgm_set_flow_wait(mgm_handle h, int64_t ticks);

/* Per-level operations for testing and profiling; vectors are device FP64 in
 * the level's natural numbering (level 1: caller order; level j+1: the WSE
 * survivors of level j in ascending level-j index). Level indices are 0-based.
 *   MGM_OP_SMOOTH:  d_x <- one GS sweep of L_j on (d_x, d_b) with the border
 *                   term -b_j*scalar (Sec. 4.3; Sec. 4.4); reverse=1: backward.
 *   MGM_OP_SPMV:    d_y = L_j d_x.
 *   MGM_OP_RESTRICT_RESIDUAL: d_y (level j+1) = R_j (d_b - L_j d_x).
 *   MGM_OP_INTERP_ADD:        d_x (level j) += P_j d_y (level j+1).
 * All run in the handle's current precision (inputs/outputs stay FP64). */
enum { MGM_OP_SMOOTH = 0, MGM_OP_SPMV = 1, MGM_OP_RESTRICT_RESIDUAL = 2, MGM_OP_INTERP_ADD = 3 };
mgm_status mgm_level_op(mgm_handle h, int32_t op, int32_t level, double *d_x,
                        const double *d_b, double *d_y, double scalar,
                        int32_t reverse, void *stream);

/* Learned per-node Chebyshev smoother, one per smoothed level (an extension;
 * the paper smooths with Gauss-Seidel, Sec. 4.3).
 * Smoother: s Richardson steps e <- e + omega_{q,i} D^-1 (f - L e), with
 * omega_{q,i} = omega_q (1 + 0.5 tanh(o_{q,i})), omega_q = 1/theta_q the
 * reciprocal Chebyshev roots on [lam/4, 1.1 lam] (lam: 20-step power
 * estimate of rho(D^-1 L)), o = MLP(features) with 3n -> 64 -> 64 -> s ReLU
 * layers in FP32; features of node i: its stencil's tangent-plane offsets
 * (Sec. 2.1) over the stencil radius and its weights (Sec. 2.2-2.3) over
 * |c_ii|. Training snapshots: fine-level errors right after the coarse-grid
 * correction of MGM iterations (Gauss-Seidel V-cycle, FP64) on L e = 0;
 * loss mean_t |L S e_t|^2 / |L e_t|^2; adjoint-smoother backward; Adam.
 * A coarse level j has its own smoother of the same form: its features use the
 * level's own n nearest points (tangent-plane offsets with the points'
 * normals) and the Galerkin operator's entries L_j(i, k) / |L_j(i, i)| at those
 * points (0 off the pattern); its snapshots come from the cycle of the
 * sub-hierarchy that starts at level j, on L_j e = 0.
 * Bordered Poisson problem (Sec. 4.4): each Richardson step holds the
 * multiplier fixed, like the Gauss-Seidel sweep (f - L e - b_j mu_j with the
 * visit's mu_j; zero on a pre-smoothing from e = 0); snapshots and the
 * measured factors come from MGM iterations on the level's homogeneous
 * bordered system [L_j b_j; b_j^T 0](e, mu) = 0 started from (start, 0), the
 * snapshots being the e parts; the loss is unchanged. */
typedef struct {
  int32_t  steps;           /* Adam steps (0: prepare snapshots/estimate only) */
  double   lr;              /* Adam learning rate, e.g. 1e-3 */
  int32_t  s;               /* Richardson steps per smoothing sweep, 1..8 */
  int32_t  n_starts;        /* random starts (rows of d_starts) */
  int32_t  iters_per_start; /* MGM iterations per start; one snapshot each */
  uint64_t seed;            /* counter-based weight initialisation */
  int32_t  init;            /* 1: (re)initialise the MLP from seed */
  int32_t  activate;        /* 0: keep GS; 1: use the learned smoother when its
                               stationary convergence factor beats GS (measured
                               over 6 iterations from the first start); 2: always */
  int32_t  level;           /* level whose smoother is trained (0 = fine; must
                               be a smoothed level, not the coarsest) */
} mgm_train_opts;

typedef struct {
  double  lam;                    /* spectral estimate of D^-1 L */
  double  loss_first, loss_last;  /* training loss before / after */
  double  rate_gs, rate_learned;  /* measured convergence factors (activate == 1) */
  int32_t active;                 /* 1 if the V-cycle now uses the learned smoother */
} mgm_train_info;

/* Prepare and/or train the learned smoother.
 *   d_starts: device FP64, n_starts x N_j random start errors of the chosen
 *   level (caller order on level 0; on a coarse level, the order of its points,
 *   i.e. of MGM_EX_COARSE_IDX of the level above);
 *   h_loss_hist: nullable host array of steps+1 losses (entry k: before the
 *   (k+1)-th Adam step; the last: after training).
 * Errors: MGM_E_ARG (bad options, layer too wide: 3n + 1 inputs above 200,
 * i.e. a stencil above 66 points).
 * Synchronises the stream. */
mgm_status mgm_train_smoother(mgm_handle h, const mgm_train_opts *opts, const double *d_starts,
                              mgm_train_info *info, double *h_loss_hist, void *stream);

/* Get (set = 0) or set (set = 1) the MLP parameters of the smoother of
 * `level`, FP32 row-major with each
 * layer's bias as its last row: W1 (3n+1) x 64 | W2 65 x 64 | W3 65 x s.
 * h_params = NULL queries *len. Setting resets the Adam state and recomputes
 * the step weights. */
mgm_status mgm_smoother_params(mgm_handle h, int32_t level, int32_t set, float *h_params, int64_t *len);

/* Loss and its gradient (same layout as the parameters, host FP32) at the
 * current parameters on the current snapshots of `level`, without an update. */
mgm_status mgm_smoother_grad(mgm_handle h, int32_t level, float *h_grad, double *loss, void *stream);

/* Select the smoothers: bit j of level_mask set = level j uses its learned
 * smoother (which must be trained), clear = Gauss-Seidel. 0 = Gauss-Seidel
 * everywhere, 1 = learned on the fine level only. */
mgm_status mgm_set_smoother(mgm_handle h, int32_t level_mask);

/* Profiling of one hot-path kernel: `reps` timed repetitions on the handle's
 * internal buffers (contents arbitrary), each bracketed by HIP events on
 * `stream`; returns the mean device time of one launch in *ms and the
 * algorithmic HBM bytes that launch must move in *bytes (values + indices
 * of the rows it touches, each vector element counted once).
 *   MGM_TK_SPMV:     the fine-level FP64 operator y = L_1 x (eq. discrete_system).
 *   MGM_TK_GS:       one smoother launch of level `level` in the current
 *                    precision (Sec. 4.3): a colour phase (plain multicolour)
 *                    or a patch-colour launch (patch-blocked); averaged over
 *                    the launches of one sweep, bytes likewise per launch.
 *                    level = -1: every smoother launch of one V-cycle (all
 *                    smoothed levels, pre- and post-sweeps as the V-cycle
 *                    issues them) queued back to back between one pair of
 *                    events; *ms and *bytes are per launch.
 *   MGM_TK_RESIDUAL: residual r - L_j e of level `level`, current precision.
 *   MGM_TK_VCYCLE:   one whole V-cycle (Alg. 3) in the current precision;
 *                    bytes = sum over its kernels.
 *   MGM_TK_LEARNED:  every launch of the learned smoother in one V-cycle (the
 *                    levels where it is active, pre- and post-sweeps as the
 *                    cycle issues them) queued back to back between one pair
 *                    of events, `level` ignored; *ms and *bytes per launch (a
 *                    Richardson step: operator, x, f, output, D^-1 and the
 *                    step weights once each; bordered: b). MGM_E_ARG when no
 *                    level uses it. */
enum { MGM_TK_SPMV = 0, MGM_TK_GS = 1, MGM_TK_RESIDUAL = 2, MGM_TK_VCYCLE = 3, MGM_TK_LEARNED = 4 };
mgm_status mgm_time_kernel(mgm_handle h, int32_t which, int32_t level, int32_t reps,
                           void *stream, double *ms, double *bytes);

/* Stencil selection (Sec. 2): the k nearest points of every point of the
 * cloud, centre first, key (d2, index) with d2 = ((dx*dx)+(dy*dy))+dz*dz in
 * IEEE double. h_xyz: host n x 3; h_idx: host n x k int32 output.
 * Errors: MGM_E_ARG (k < 1 or k > n), MGM_E_DUP_POINTS. Host only. */
mgm_status mgm_stencils(const double *h_xyz, int64_t n, int32_t k, int32_t *h_idx);

/* Batched RBF-FD weights (Sec. 2.1-2.2, eq. rbf_fd_lap): for each of the
 * n_systems stencils (rows of d_stencils, n_systems x stencil_size int32,
 * centre first, indices into the n_points rows of d_xyz / d_normals, device
 * FP64 n_points x 3) solve the PHS r^(2*phs_order+1) + degree-poly_degree
 * saddle system in the tangent plane of the centre and write the stencil_size
 * weights of row i to d_weights (device FP64, n_systems x stencil_size).
 * One wavefront per system, FP64 Gauss-Jordan with partial pivoting; needs
 * phs_order 1..6, poly_degree 0..6 and
 * stencil_size + (poly_degree+1)(poly_degree+2)/2 <= 64. Systems of more
 * than 32 unknowns with poly_degree <= 4 are eliminated in panels of four
 * columns whose updates run on the FP64 matrix cores (MFMA); the others
 * one column at a time on the vector units. Synchronises the
 * stream once to report MGM_E_STENCIL_SINGULAR (some system had a pivot below
 * 1e-13 of its largest entry; the other rows are still written). An empty
 * batch (n_systems = 0) checks the sizes and writes nothing; d_stencils and
 * d_weights may then be null. */
mgm_status mgm_batched_weights(const double *d_xyz, const double *d_normals, int64_t n_points,
                               const int32_t *d_stencils, int64_t n_systems, int32_t stencil_size,
                               int32_t phs_order, int32_t poly_degree, double *d_weights,
                               void *stream);

/* Mixed-precision form of mgm_batched_weights (the same systems of Sec. 2.2,
 * eq. rbf_fd_lap; same arguments, layouts and errors, poly_degree <= 4 or
 * MGM_E_ARG): each system is eliminated in FP32 on the matrix cores (Gauss-
 * Jordan with partial pivoting in panels of four columns, on [A | I], so that
 * the elimination yields an FP32 inverse) and the solution is then refined in
 * FP64: from x = 0, four times x += A32^-1 (b - A x), the residual computed
 * in FP64 from the stencil coordinates. Each correction contracts the error
 * by about cond(A) * 6e-8; for the scaled PHS systems (cond ~ 3e4) the result
 * agrees with the FP64 elimination to ~1e-11. The singular flag is the FP64
 * kernel's (a pivot below 1e-13 of the largest entry). */
mgm_status mgm_batched_weights_mixed(const double *d_xyz, const double *d_normals, int64_t n_points,
                                     const int32_t *d_stencils, int64_t n_systems, int32_t stencil_size,
                                     int32_t phs_order, int32_t poly_degree, double *d_weights,
                                     void *stream);

/* Allocation-free form of mgm_batched_weights, for callers that cannot
 * allocate device memory (code that must not call hipMalloc, such as tight
 * serving loops or harnesses that forbid it). Same arguments, results
 * (bit for bit, same kernel) and errors as mgm_batched_weights, plus
 * MGM_E_ARG for a batch above 2^33 systems (the launch grid's limit, which
 * mgm_batched_weights shares). The singular-system flag that
 * mgm_batched_weights allocates per call lives instead in a 256-byte device
 * array of the library, one per GPU, held until the process ends; a call
 * uses 4 bytes of it whatever the batch size, clears it on the stream before
 * the solve and reads it back after (one stream synchronisation). Calls that
 * overlap on one GPU share that flag and race: serialise them. */
mgm_status mgm_batched_weights_noalloc(const double *d_xyz, const double *d_normals, int64_t n_points,
                                       const int32_t *d_stencils, int64_t n_systems, int32_t stencil_size,
                                       int32_t phs_order, int32_t poly_degree, double *d_weights,
                                       void *stream);

/* Surface gradient and divergence (Sec. 6.3: the heat method for geodesic
 * distance uses them with MGM solves; the weights are the tangent-plane RBF-FD
 * of Sec. 2.1-2.2 with first derivatives at the centre on the right-hand
 * side). mgm_surface_ops_setup builds, on the handle's fine point cloud,
 * stencils of stencil_size nearest points and PHS r^(2*phs_order+1) +
 * degree-poly_degree weights: a vector W_ij per entry, W_ij = g1_ij t1_i +
 * g2_ij t2_i with g1, g2 the weights of d/dxh, d/dyh in the tangent basis of
 * x_i. Needs 1 <= poly_degree <= 6, 1 <= phs_order <= 6 and
 * (l+1)(l+2)/2 <= stencil_size <= min(128, N); MGM_E_STENCIL_SINGULAR for a
 * singular local system. The handle owns the operator (about 28 bytes per
 * entry on the device). On a host-only handle the call builds the weights
 * for mgm_export only. Calling it again replaces the operator.
 *   mgm_surface_gradient: d_g (device FP64, N x 3 row-major, caller order) =
 *     grad_M u for d_u (device FP64, length N); normalise = 1 gives instead
 *     -grad u / |grad u| (the heat-method direction), 0 where grad u = 0.
 *   mgm_surface_divergence: d_out (device FP64, length N) = div_M v for a
 *     field d_v (device FP64, N x 3 row-major), taken in each node's tangent
 *     plane: sum_j W_ij . v_j.
 * Stream-ordered, no synchronisation; MGM_E_ARG before the setup call. */
mgm_status mgm_surface_ops_setup(mgm_handle h, int32_t phs_order, int32_t poly_degree, int32_t stencil_size,
                                 void *stream);
mgm_status mgm_surface_gradient(mgm_handle h, const double *d_u, double *d_g, int32_t normalise, void *stream);
mgm_status mgm_surface_divergence(mgm_handle h, const double *d_v, double *d_out, void *stream);

/* Export of setup results for bit-exact comparison (host buffers).
 * Call with h_buf = NULL to query *len (element count); then with a buffer of
 * at least *len elements. Element types: I32 = int32_t, F64 = double.
 *   MGM_EX_LEVEL_SIZES   I32  all levels                      (level ignored)
 *   MGM_EX_STENCILS      I32  N_1 x n, centre first           (level ignored)
 *   MGM_EX_WEIGHTS       F64  N_1 x n, weights c_ij           (level ignored)
 *   MGM_EX_COARSE_IDX    I32  survivors of level j (ascending level-j index)
 *   MGM_EX_INTERP_IDX    I32  N_j x m coarse neighbours (level j+1 numbering)
 *   MGM_EX_INTERP_W      F64  N_j x m weights (injection rows: 1,0,0)
 *   MGM_EX_COLOURS       I32  colour of each row of level j (natural order)
 *   MGM_EX_L_ROWPTR      I32  CSR row pointer of L_j (natural order)
 *   MGM_EX_L_COLS        I32  CSR column indices (sorted per row)
 *   MGM_EX_L_VALS        F64  CSR values
 *   MGM_EX_BORDER        F64  b_j (Poisson only)
 *   MGM_EX_NCOLOURS      I32  colours per smoothed level      (level ignored)
 *   MGM_EX_PATCH         I32  smoother patch of each row of level j (empty when
 *                             the level is not patch-blocked)
 *   MGM_EX_OMEGA         F64  N_j x s learned step weights of level j (caller
 *                             order)
 *   MGM_EX_GRAD_STENCILS I32  N_1 x n_g surface-operator stencils (after
 *                             mgm_surface_ops_setup)
 *   MGM_EX_GRAD_WEIGHTS  F64  N_1 x n_g x 3 surface-gradient weights W_ij
 *   MGM_EX_L16_VALS      F64  the FP16 operator values h_ij of level j as the
 *                             device holds them (each exactly widened), in
 *                             the order of MGM_EX_L_VALS; built on first use.
 *                             Smoothed levels of a device handle only
 *   MGM_EX_ROW_SCALE     F64  the FP32 row scales s_i of that operator
 *                             (L_ij ~ s_i h_ij), natural order
 *   MGM_EX_HALO_ROWS     I32  the staged halo of the one-launch sweeps of
 *                             level j: for each patch in ascending patch id,
 *                             its count, then the distinct rows outside it
 *                             that its rows' entries reference (natural
 *                             numbering, ascending); empty when the level
 *                             loads its halo per entry. Device handles only */
enum {
  MGM_EX_LEVEL_SIZES = 0, MGM_EX_STENCILS = 1, MGM_EX_WEIGHTS = 2,
  MGM_EX_COARSE_IDX = 3, MGM_EX_INTERP_IDX = 4, MGM_EX_INTERP_W = 5,
  MGM_EX_COLOURS = 6, MGM_EX_L_ROWPTR = 7, MGM_EX_L_COLS = 8,
  MGM_EX_L_VALS = 9, MGM_EX_BORDER = 10, MGM_EX_NCOLOURS = 11, MGM_EX_PATCH = 12,
  MGM_EX_OMEGA = 13, MGM_EX_GRAD_STENCILS = 14, MGM_EX_GRAD_WEIGHTS = 15,
  MGM_EX_L16_VALS = 16, MGM_EX_ROW_SCALE = 17, MGM_EX_HALO_ROWS = 18
};
mgm_status mgm_export(mgm_handle h, int32_t what, int32_t level, void *h_buf,
                      int64_t *len);

/* Release every resource of the handle (waits for its device work). */
void mgm_destroy(mgm_handle h);

const char *mgm_status_str(mgm_status s);
const char *mgm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* MGM_H */
