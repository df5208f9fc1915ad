/*
 * camg: classical algebraic multigrid preconditioned conjugate gradients
 * for sparse SPD systems on one AMD Instinct MI355X (gfx950).
 *
 * The method follows Isotton, Frigo, Spiezia, Janna, "Chronos: a general
 * purpose classical AMG solver for High Performance Computing"
 * (arXiv 2102.07417):
 *   - the problem A x = b with A sparse SPD in CSR (Section 1, eq. linSys;
 *     Section 3, CSRMAT storage);
 *   - hierarchy set-up, Alg. "AMG Set-up": Jacobi smoother (eq. smoother),
 *     classical strength of connection with a threshold (Section 2,
 *     Strength of Connection, eq. cla), PMIS C/F splitting, interpolation
 *     P = [W; I] (eq. prolOperator), Galerkin coarse operator
 *     A_c = P^T A P (eq. AcDef), dense Cholesky on the last level;
 *   - preconditioner application, Alg. "AMG application in a V-cycle";
 *   - PCG from x0 = 0, stopped when ||r|| < rtol ||b|| on the recursively
 *     updated residual (Section 4, set-up of the experiments).
 *
 * Every call returns a camg_status.  No exception or abort crosses this
 * interface.  The last error message of the calling thread is available
 * from camg_last_error().
 *
 * Pointer conventions: functions named *_dev take device pointers (memory
 * of the device the handle was created on, e.g. torch tensors) and run on
 * the given HIP stream (NULL = the default stream); the other functions take
 * host pointers and synchronise before returning.  Input arrays are borrowed
 * for the duration of the call; outputs are caller-allocated unless stated.
 * All indices are 0-based int32; values are IEEE double unless stated.
 */
#ifndef CAMG_H
#define CAMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CAMG_ABI_VERSION 8

typedef struct camg_hier *camg_handle;

typedef enum {
    CAMG_OK = 0,
    CAMG_E_MAXIT = 1,       /* warning: max_iter reached; outputs hold the last iterate */
    CAMG_E_ACCURACY = 2,    /* warning (mixed precision, rtol > 0): the recursive residual met the test but
                               the true residual ||b - A x|| / ||b|| is still >= rtol after the two restarts
                               from it; outputs hold the last iterate and its true residual */
    CAMG_E_ARG = -1,        /* bad argument (null pointer, n < 1, bad parameter) */
    CAMG_E_CSR = -2,        /* malformed CSR, non-finite value, missing diagonal, asymmetry */
    CAMG_E_NOT_SPD = -3,    /* non-positive diagonal or non-positive Cholesky pivot */
    CAMG_E_BREAKDOWN = -4,  /* CG breakdown: p.Ap <= 0 or r.z <= 0 (matrix or M not SPD) */
    CAMG_E_COARSE = -5,     /* coarsening stalled with more than 8192 unknowns on the last level */
    CAMG_E_NOMEM = -6,      /* device or host allocation failed */
    CAMG_E_DEVICE = -7,     /* HIP runtime error */
    CAMG_E_BUSY = -8        /* the handle is in use by another call */
} camg_status;

enum { CAMG_FP64 = 0, CAMG_MIXED_FP32 = 1 };
/* Smoother (Section 2, eq. smoother): Jacobi (M = D, the default) or the
 * factorised sparse approximate inverse M^{-1} = G^T G (eq. smo; here the
 * static factor on the pattern of the lower triangle of A; every row of it
 * must have at most 192 entries, CAMG_E_ARG otherwise).  FSAI_JACOBI: FSAI
 * on each level whose rows have at most 192 entries on or below the
 * diagonal and Jacobi on the others (e.g. the dense coarse levels of BAMG).
 * AFSAI: the adaptive factor, the paper's default smoother (eq. smo, with
 * the pattern search of the FSAI package it cites): row i of G minimises
 * psi_i(g) = g^T A g (g_i = 1) on a pattern grown from {i}; each step adds
 * the afsai_step columns j < i, taken from the rows of A indexed by the
 * pattern, with the largest |(A g)_j| (the Kaporin gradient; the smaller j
 * on ties), for at most afsai_steps steps, and a row stops early once psi_i
 * falls by no more than afsai_eps of its previous value in a step; the row
 * is scaled so that G A G^T has a unit diagonal.  A level where a row's
 * candidate set exceeds CAMG_AFSAI_MAXCAND columns uses Jacobi. */
enum { CAMG_SMOOTH_JACOBI = 0, CAMG_SMOOTH_FSAI = 1, CAMG_SMOOTH_FSAI_JACOBI = 2, CAMG_SMOOTH_AFSAI = 3 };
#define CAMG_AFSAI_MAXM 32        /* afsai_steps * afsai_step + 1 is at most this */
#define CAMG_AFSAI_MAXCAND 2048
/* Interpolation (Section 2, Interpolation).  DIRECT: distance-one direct
 * formula over C_i^S (the default).  CLASSICAL: eq. clasInt with the
 * correction for strong F neighbours that share no C point (they are
 * lumped into the diagonal), keeping the direct coupling a_ij in the
 * numerator.  EXTI: extended+i, eq. extpiInt, over C_i^S plus the strong C
 * neighbours of the strong F neighbours.  HYBRID: the same formula over the
 * smaller set of Alg. extintset (C_i^S plus, greedily, the C points that
 * cover the most strong F neighbours without a C point in the set; the
 * smallest index on ties).  Rows have at most 2048 candidate C points
 * (CAMG_E_ARG otherwise). */
enum { CAMG_INTERP_DIRECT = 0, CAMG_INTERP_CLASSICAL = 1, CAMG_INTERP_EXTI = 2, CAMG_INTERP_HYBRID = 3,
       CAMG_INTERP_BAMG = 4 };
/* CAMG_INTERP_BAMG (eq. minBAMG, Alg. BAMG; set up with camg_setup_tv): the
 * weights of F point i least-squares fit its row of the test space from
 * the rows of a basis of C points chosen greedily (largest residual norm,
 * smallest index on ties; at most nt points) among the C points within
 * strength-graph distance l; l grows from bamg_lmin while the relative
 * residual exceeds bamg_eps or ||w|| exceeds bamg_mu, up to bamg_lmax (at
 * most 2 here).  The test space is made orthonormal on level 0 and taken at
 * the C points on coarser levels.  Rows have at most 128 candidates
 * (CAMG_E_ARG otherwise). */
/* SRQM refinement (Section 2, the passage on unveiling the near kernel, eq.
 * eigP), camg_params.srqm_iters > 0, BAMG only: after the level-0 smoother is
 * built, each step takes the orthonormal test space V, the residual
 * R = A V - V (V^T A V) and W = M^{-1} R (M^{-1} = D^{-1} for Jacobi, G^T G for
 * FSAI), and replaces V by the nt Ritz vectors of A with the smallest Ritz
 * values on span[V, W] (columns of W that add no direction, pivot <= 1e-12 of
 * the largest Gram diagonal, are left out; a step where all are left out ends
 * the refinement).  The result is made orthonormal again.  The small dense
 * eigenproblem (at most 16 x 16) is solved on the device by cyclic Jacobi. */

/* Hierarchy and solver parameters. */
typedef struct {
    double   theta;       /* strength threshold; default 0.25 */
    uint64_t seed;        /* PMIS random seed; level l, point i uses splitmix64 draw (l << 40) + i */
    int32_t  nu_pre;      /* smoothing steps before the coarse correction; default 1 */
    int32_t  nu_post;     /* smoothing steps after it; default 1 (equal values keep M symmetric) */
    double   omega;       /* <= 0: per level, Jacobi (4/3) / max_i(sum_j |a_ij| / a_ii), FSAI (4/3) / rho_hat
                             with rho_hat the Rayleigh quotient of G A G^T after 15 power steps from a vector
                             drawn with seed + 1 (G, A, G^T applied in turn); > 0: fixed */
    int32_t  max_levels;  /* default 25 */
    int32_t  max_coarse;  /* a level with at most this many unknowns is solved directly; default 256 */
    int32_t  precision;   /* CAMG_FP64 or CAMG_MIXED_FP32 (FP32 V-cycle inside FP64 PCG) */
    int32_t  max_iter;    /* PCG iteration limit; default 1000 */
    int32_t  smoother;    /* CAMG_SMOOTH_JACOBI (default), _FSAI, _FSAI_JACOBI or _AFSAI; static FSAI needs at
                             most 192 entries on or below the diagonal per row; the FSAI smoothers run on the
                             single-system path only */
    int32_t  interp;      /* CAMG_INTERP_DIRECT (default), _CLASSICAL, _EXTI or _HYBRID */
    int64_t  rap_chunk;   /* Galerkin product R (A P): when A P has more products than this, it is formed in
                             windows of coarse rows of at most this many products (bounds the set-up's scratch
                             memory and keeps A P under 2^31 entries); 0: 2^30.  Results are bitwise the same */
    int32_t  bamg_lmin;   /* BAMG: first interpolation distance tried; default 1 */
    int32_t  bamg_lmax;   /* BAMG: last one (<= 2); default 2 */
    double   bamg_eps;    /* BAMG: accept when the relative residual of the fit is <= eps (default 1e-3) */
    double   bamg_mu;     /*       and the weights' 2-norm is <= mu (default 10) */
    int32_t  psmooth;     /* 1: smooth P by one Jacobi step, P - omega D^{-1} A P (omega: the level's Jacobi
                             weight); default 0 */
    double   pfilter;     /* < 1: filter P (Section 2, Filtering): per row keep the largest |p| up to this
                             fraction of the row's absolute sum and move the dropped entries' action on the
                             coarse test space (a unit vector without one) onto the kept entries by a
                             minimum-norm correction; default 1 (off) */
    int32_t  srqm_iters;  /* BAMG: steps of simultaneous Rayleigh quotient minimisation refining the level-0
                             test space before it is used (0 to 100; default 0); see camg_setup_tv */
    int32_t  afsai_steps; /* CAMG_SMOOTH_AFSAI: growth steps per row (default 10) */
    int32_t  afsai_step;  /*   columns added per step (default 2); afsai_steps * afsai_step + 1 <= 32 */
    double   afsai_eps;   /*   a row stops once psi_i falls by no more than this fraction in a step (>= 0;
                               default 0.01) */
} camg_params;

#define CAMG_MAX_LEVELS 32

typedef struct {
    int32_t levels;                       /* number of levels; the last one is solved directly */
    int32_t n[CAMG_MAX_LEVELS];           /* unknowns per level */
    int64_t nnz[CAMG_MAX_LEVELS];         /* nonzeros of A_l */
    int64_t nnz_p[CAMG_MAX_LEVELS];       /* nonzeros of P_l (0 on the last level) */
    int32_t pmis_rounds[CAMG_MAX_LEVELS]; /* PMIS rounds per level */
    double  omega[CAMG_MAX_LEVELS];       /* Jacobi weight per level */
    double  grid_complexity;              /* sum_l n_l / n_0 */
    double  operator_complexity;          /* sum_l nnz(A_l) / nnz(A_0) */
    int64_t device_bytes;                 /* device memory held by the handle */
    double  setup_ms;                     /* wall time of the set-up call */
    int32_t precision;
    double  setup_phase_ms[8];            /* set-up wall time by phase, summed over levels: input copy and
                                             checks, smoother weights, strength + PMIS + coarse numbering,
                                             interpolation, R = P^T, Galerkin product, last-level factorisation,
                                             launch shapes and solve buffers */
    int32_t compact_cols;                 /* bit 5 l + k set when matrix k of level l (A, P, R, G, G^T) has
                                             16-bit column differences for the row kernels (levels 0..5) */
} camg_info_t;

int32_t     camg_abi_version(void);
const char *camg_status_str(camg_status s);
const char *camg_last_error(void);
void        camg_params_default(camg_params *p);

/*
 * Build the hierarchy of A on the current HIP device (Alg. AMG Set-up).
 * n: order of A.  row_ptr[n+1], col_idx[nnz], val[nnz] with nnz = row_ptr[n]:
 * 0-based CSR, columns strictly increasing in each row, both triangles
 * stored, structurally symmetric with |a_ij - a_ji| <= 1e-12 max|a|, every
 * diagonal entry present and positive, all values finite.  Violations give
 * CAMG_E_CSR (CAMG_E_NOT_SPD for a non-positive diagonal) before any
 * hierarchy is built.  params may be NULL (defaults).  The handle owns
 * copies of everything it needs; release it with camg_destroy.
 * camg_setup takes host arrays; camg_setup_dev device arrays.
 */
camg_status camg_setup(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val,
                       const camg_params *params, camg_handle *out);
camg_status camg_setup_dev(int32_t n, const int32_t *d_row_ptr, const int32_t *d_col_idx, const double *d_val,
                           const camg_params *params, void *hip_stream, camg_handle *out);
/*
 * The same with a test space for BAMG interpolation (Section 2, Unveiling
 * the operator near kernel; eq. minBAMG): V is n x nt, row-major (row k =
 * the test-space values at unknown k), 1 <= nt <= 8, linearly independent
 * columns (CAMG_E_ARG otherwise), e.g. the rigid body modes of an
 * elasticity problem.  V is borrowed for the call (host memory for
 * camg_setup_tv, device memory for camg_setup_tv_dev).  With
 * params->interp != CAMG_INTERP_BAMG, V is ignored.
 */
camg_status camg_setup_tv(int32_t n, const int32_t *row_ptr, const int32_t *col_idx, const double *val, int32_t nt,
                          const double *V, const camg_params *params, camg_handle *out);
camg_status camg_setup_tv_dev(int32_t n, const int32_t *d_row_ptr, const int32_t *d_col_idx, const double *d_val,
                              int32_t nt, const double *d_V, const camg_params *params, void *hip_stream,
                              camg_handle *out);

/*
 * Solve A x = b by PCG preconditioned with one V-cycle per iteration
 * (Alg. AMG application in a V-cycle), from x0 = 0, until
 * ||r_k|| < rtol ||b|| on the recursively updated residual, or max_iter
 * iterations.  rtol <= 0 runs exactly max_iter iterations.
 * b, x: n doubles.  iters (may be NULL): iterations done.  hist (host, may be
 * NULL): hist[k] = ||r_k|| for k = 0..iters, truncated to hist_cap entries.
 * true_relres (may be NULL): ||b - A x|| / ||b|| in FP64 at exit.
 * b = 0 gives x = 0 after 0 iterations.  Returns CAMG_E_MAXIT (x valid) or
 * CAMG_E_BREAKDOWN (x = last iterate) when the loop did not converge.  In
 * mixed precision the true residual must pass the test too: when the
 * recursive one passes and the true one does not, PCG restarts from
 * r = b - A x (at most twice) and returns CAMG_E_ACCURACY if the true
 * residual still fails (in FP64 the test is the recursive residual's alone,
 * as in the paper; true_relres reports the other).
 * camg_solve: host b and x.  camg_solve_dev: device b and x, asynchronous
 * with respect to the host except for the convergence polling; it returns
 * after the solve has finished on `hip_stream`.
 */
camg_status camg_solve(camg_handle h, const double *b, double rtol, double *x, int32_t *iters,
                       double *hist, int32_t hist_cap, double *true_relres);
camg_status camg_solve_dev(camg_handle h, const double *d_b, double rtol, double *d_x, int32_t *iters,
                           double *hist, int32_t hist_cap, double *true_relres, void *hip_stream);

/*
 * k right-hand sides at once: d_B and d_X are n-by-k row-major device
 * blocks.  The columns run k independent PCG recurrences that share every
 * matrix pass (sparse matrix times row-major block, K = the next power of
 * two >= k columns, at most 64 per pass); a column stops updating once it
 * has converged.  Each column's result does not depend on the other columns
 * (bitwise, for a given K) and agrees with a single-vector solve to
 * rounding.  iters[k], true_relres[k] (host, may be NULL); hist (host, may
 * be NULL) is k-by-hist_cap row-major.  Returns the worst status over the
 * columns (breakdown before max_iter before accuracy before ok; accuracy as
 * for camg_solve_dev, per column).
 */
camg_status camg_solve_multi_dev(camg_handle h, int32_t k, const double *d_B, double rtol, double *d_X,
                                 int32_t *iters, double *hist, int32_t hist_cap, double *true_relres,
                                 void *hip_stream);

/*
 * Slot engine (continuous batching).  An engine holds `slots` columns (a
 * power of two, at most 64) of row-major n-by-slots work blocks on the
 * handle's hierarchy and runs one PCG recurrence per busy column, all
 * columns sharing every matrix pass.  Columns can be started while others
 * run; a finished column stops updating.  A column's iterates do not depend
 * on the other columns or on its slot (bitwise), for a given slot count.
 * The handle must outlive its engines; one engine is driven by one host
 * thread; engines of one handle may run concurrently on different streams.
 *   camg_engine_footprint: device bytes an engine of `slots` columns needs.
 *   camg_engine_create: allocate it (hist_cap entries of residual history per column).
 *   camg_engine_start: start columns [slot0, slot0+m) from the device block
 *     d_B (n-by-m row-major, row stride ldb), x0 = 0, rtol, max_iter.
 *   camg_engine_step: run up to max_steps iterations (fewer once no column is
 *     running); *running receives the number of columns still running.
 *   camg_engine_state: host arrays of `slots` entries: iterations done, done
 *     flag (1 done, 0 running, -1 free), status (camg_status of the column).
 *   camg_engine_finish: copy columns [slot0, slot0+m) of x into d_X (n-by-m
 *     row-major, row stride ldx), true relative residuals into true_relres
 *     (host, may be NULL), and free the slots.
 */
typedef struct camg_engine *camg_engine_t;
camg_status camg_engine_footprint(camg_handle h, int32_t slots, int64_t *bytes);
camg_status camg_engine_create(camg_handle h, int32_t slots, int32_t hist_cap, void *hip_stream, camg_engine_t *out);
camg_status camg_engine_start(camg_engine_t e, int32_t slot0, int32_t m, const double *d_B, int32_t ldb, double rtol,
                              int32_t max_iter);
camg_status camg_engine_step(camg_engine_t e, int32_t max_steps, int32_t *running);
camg_status camg_engine_state(camg_engine_t e, int32_t *iters, int32_t *done, int32_t *status);
camg_status camg_engine_finish(camg_engine_t e, int32_t slot0, int32_t m, double *d_X, int32_t ldx,
                               double *true_relres);
camg_status camg_engine_destroy(camg_engine_t e);

/*
 * Many small systems at once: count systems (handles of one precision, one
 * smoothing step each way, on one device, each listed once) are solved in
 * one kernel launch, one workgroup per system running that system's whole
 * PCG solve (every iteration and V-cycle level) with the same recurrence
 * and stopping test as camg_solve_dev, x0 = 0, rtol shared.  d_b[k], d_x[k]
 * are device vectors of system k; iters, true_relres and status are host
 * arrays of count entries (each may be NULL); per-system outcomes are in
 * status (CAMG_OK, CAMG_E_MAXIT, CAMG_E_BREAKDOWN, and CAMG_E_ACCURACY in
 * mixed precision as for camg_solve_dev) while the call returns
 * CAMG_OK.  Meant for systems up to ~1e5 unknowns (one compute unit works
 * through each system); larger ones are correct but slow.
 */
camg_status camg_solve_batch_dev(int32_t count, const camg_handle *hs, const double *const *d_b, double *const *d_x,
                                 double rtol, int32_t *iters, double *true_relres, int32_t *status,
                                 void *hip_stream);

/*
 * The same solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * identical arguments, kernels, results and per-system outcomes as
 * camg_solve_batch_dev, but the per-call device buffers (the systems'
 * descriptors and their results) sit in a static device array of
 * CAMG_NOALLOC_MAX_SYSTEMS entries (about 4.8 MB) that each GPU the library
 * runs on holds until the process ends, instead of two allocations per
 * call.  The call makes no device allocation and frees nothing; it still
 * stages the descriptors through ordinary host memory and waits for the
 * stream, like camg_solve_batch_dev.  count > CAMG_NOALLOC_MAX_SYSTEMS
 * returns CAMG_E_ARG.  Every call on one GPU shares that GPU's array (the
 * next call overwrites it; nothing in it needs clearing), so calls that
 * overlap on one GPU (other host threads, other streams) race: serialise
 * them.
 */
#define CAMG_NOALLOC_MAX_SYSTEMS 1024
camg_status camg_solve_batch_noalloc_dev(int32_t count, const camg_handle *hs, const double *const *d_b,
                                         double *const *d_x, double rtol, int32_t *iters, double *true_relres,
                                         int32_t *status, void *hip_stream);

/*
 * Server: resident hierarchies answering solve requests (the paper reuses
 * one hierarchy for many solves; here every system added keeps its
 * hierarchy and a slot engine on a stream of its own, so the systems' work
 * overlaps on the device).
 *   camg_server_create: a server whose device memory (engines plus request
 *     arena) stays within budget_bytes.
 *   camg_server_add: add the system of handle h with an engine of `slots`
 *     columns (power of two, at most 64) and iters_per_batch iterations per
 *     batch (0: chosen from n); *system receives its index.  CAMG_E_NOMEM if
 *     the engine does not fit the budget; CAMG_E_BUSY after the first
 *     request.  The handle must outlive the server.
 *   camg_server_submit: queue a request of k right-hand sides of one system:
 *     B (n-by-k row-major, row stride ldb) and X (solutions, row stride ldx)
 *     are host or device pointers (pinned host memory keeps the copies
 *     asynchronous) that stay valid until the request completes; x0 = 0.
 *     A request is admitted, in arrival order per system, when k slots are
 *     free and its n*k*8-byte staging block fits in the arena (the budget
 *     left after the engines).  CAMG_E_NOMEM if it can never fit.
 *   camg_server_poll: advance every system without waiting for the device
 *     (retire finished batches, check true residuals, copy results out,
 *     admit, launch); completed requests are appended to `out` (at most
 *     cap, the rest stay for the next call) and *n_out receives their
 *     number.  Each completion has the worst column status (CAMG_E_ACCURACY
 *     as for camg_solve_dev on a mixed-precision system), the largest
 *     iteration count and true relative residual of the request, the time
 *     from submission to admission and to completion (ms).
 *   camg_server_stats: arena bytes in use and its size, requests waiting,
 *     slots busy (any pointer may be NULL).
 *   camg_server_destroy: wait for the device and release everything; the
 *     outcome of requests not yet completed is undefined.
 * One host thread drives a server.  A request's solutions are bitwise the
 * same whatever else runs beside it (per-column arithmetic, slot count
 * fixed per system).
 */
typedef struct camg_server *camg_server_t;
typedef struct {
    int64_t tag;
    int32_t status;
    int32_t iters;
    double true_relres;
    double queue_ms;
    double latency_ms;
} camg_completion;
camg_status camg_server_create(int64_t budget_bytes, camg_server_t *out);
camg_status camg_server_add(camg_server_t s, camg_handle h, int32_t slots, int32_t iters_per_batch, int32_t *system);
camg_status camg_server_submit(camg_server_t s, int32_t system, int32_t k, const double *B, int32_t ldb, double *X,
                               int32_t ldx, double rtol, int32_t max_iter, int64_t tag);
camg_status camg_server_poll(camg_server_t s, camg_completion *out, int32_t cap, int32_t *n_out);
camg_status camg_server_stats(camg_server_t s, int64_t *arena_used, int64_t *arena_size, int32_t *queued,
                              int32_t *busy_slots);
camg_status camg_server_destroy(camg_server_t s);

/* z = M y: one V-cycle (device vectors of length n). */
camg_status camg_vcycle_dev(camg_handle h, const double *d_y, double *d_z, void *hip_stream);

/* Hierarchy statistics (host struct). */
camg_status camg_info(camg_handle h, camg_info_t *info);

/* Sizes of level l: n_l, nnz(A_l), nnz(P_l), n_{l+1} (the last two are 0 on the last level). */
camg_status camg_level_sizes(camg_handle h, int32_t l, int32_t *n, int64_t *nnz_a, int64_t *nnz_p, int32_t *nc);

/*
 * Copy part of level l to host buffers sized from camg_level_sizes:
 *   CAMG_X_A, CAMG_X_P, CAMG_X_R: a = row_ptr (int32), b = col_idx (int32), c = values (double);
 *   CAMG_X_CF: a = int8[n] (1 = C, -1 = F);   CAMG_X_STRONG: a = uint8[nnz(A_l)];
 *   CAMG_X_DINV: a = double[n] (1 / a_ii);    CAMG_X_OMEGA: a = double[1];
 *   CAMG_X_STCNT: a = int32[n] (|S_i^T|);      CAMG_X_COARSE_INV: a = double[n*n] (last level:
 *   the dense inverse applied by the coarse solve, row-major);
 *   CAMG_X_G (a level smoothed by FSAI or aFSAI): the factor G as CSR like CAMG_X_A; its nonzero
 *   count is a[n] (export with b = c = NULL first to size them).
 */
enum { CAMG_X_A = 0, CAMG_X_P = 1, CAMG_X_R = 2, CAMG_X_CF = 3, CAMG_X_STRONG = 4, CAMG_X_DINV = 5,
       CAMG_X_OMEGA = 6, CAMG_X_COARSE_INV = 7, CAMG_X_STCNT = 8, CAMG_X_G = 9 };
camg_status camg_export_level(camg_handle h, int32_t l, int32_t what, void *a, void *b, void *c);

/*
 * Galerkin product A_c = P^T (A P) (eq. AcDef) of caller-provided host CSR
 * matrices, computed on the current device by the same kernels the set-up
 * uses.  A: n-by-n, P: n-by-nc.  The result arrays are allocated by the
 * library (release each with camg_free_host); *nnz_out receives nnz(A_c).
 * The pattern is the full symbolic product (no dropping), rows sorted.
 */
camg_status camg_galerkin(int32_t n, const int32_t *a_rp, const int32_t *a_ci, const double *a_val,
                          int32_t nc, const int32_t *p_rp, const int32_t *p_ci, const double *p_val,
                          int32_t **c_rp, int32_t **c_ci, double **c_val, int64_t *nnz_out);
void camg_free_host(void *p);

/*
 * Kernel timing for benchmarks: while enabled, every solve on the handle
 * brackets the level-0 post-smoothing kernel (the fine-level Jacobi step
 * z = s + omega D^{-1} (y - A s) fused with the r.z partial sums) with HIP
 * events on the solve's stream, on every enable-th PCG iteration (the last
 * of each group of enable iterations), and accumulates the durations of the
 * timed launches that did work.  The multi-RHS engines of the handle
 * (camg_solve_multi_dev, camg_engine_step) time their level-0 block
 * post-smoothing kernel the same way, on every enable-th iteration they
 * issue (those iterations run without the engine's graph).  Each call
 * returns (and resets) the totals gathered since the previous call, then
 * sets timing: enable = 0 off, enable = n >= 1 on, every n-th iteration.
 * total_ms and launches may be NULL.
 */
camg_status camg_profile(camg_handle h, int32_t enable, double *total_ms, int64_t *launches);

/*
 * Options of a handle.  CAMG_OPT_GRAPH (default 1): run each PCG iteration
 * as a captured HIP graph (0: launch the kernels one by one; the results
 * are bitwise the same).  CAMG_OPT_AUTOTUNE (default 0): multi-RHS engines
 * created on the handle afterwards (camg_solve_multi_dev, camg_engine_create,
 * camg_server_add) time the candidate schedules of their row kernels on
 * every matrix of the hierarchy (entries per unrolled step, LDS chunk, grid)
 * and keep the fastest, cached per matrix signature for the process; the
 * results are bitwise the same as untuned.  CAMG_OPT_COMPACT_COLS (default
 * 1): the single-system row kernels read each tiled matrix's columns as
 * 16-bit words (the difference to the tile's smallest column when the tile
 * spans fewer than 65536 columns, else a window of 8192 columns out of at
 * most eight per tile and the offset in it) where every tile can be encoded
 * (10 bytes per FP64 nonzero instead of 12); 0 reads the int32 columns; the
 * results are bitwise the same.
 */
enum { CAMG_OPT_GRAPH = 1, CAMG_OPT_AUTOTUNE = 2, CAMG_OPT_COMPACT_COLS = 3 };
camg_status camg_set_option(camg_handle h, int32_t option, int64_t value);

/* Release the hierarchy and all its device memory.  NULL is ignored. */
camg_status camg_destroy(camg_handle h);

#ifdef __cplusplus
}
#endif
#endif /* CAMG_H */
