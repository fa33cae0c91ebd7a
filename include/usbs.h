/*
 * usbs.h -- C ABI of the MI355X (gfx950) implementation of Unified Spectral
 * Bundling with Sketching (USBS), Angell & McCallum, arXiv 2312.11801.
 *
 * The library solves the SDP pair (P)/(D) of Sec. 2.1:
 *     (P)  maximise <C, X>  s.t.  A_I' X = b_I',  A_I X <= b_I,  X PSD
 *     (D)  minimise <b, y>  s.t.  C - A^* y NSD,  y_I >= 0
 * by the proximal bundle iteration of Alg. 1 on the penalized dual
 *     f(y) = alpha [lambda_max(C - A^* y)]_+ + <b, y>,  y_I >= 0   (Sec. 3, eq. pen-D)
 * with the spectral bundle model of Sec. 3.1, the candidate of Sec. 3.2
 * (eq. dual_update), the master QP of App. B.2 and the Nystrom sketch of
 * Sec. 4 / App. C.  Every step runs on one GPU in hand-written HIP kernels.
 *
 * Conventions for every entry point:
 *   * Return value: 0 on success, USBS_NOT_CONVERGED (> 0) when a solve
 *     stopped at its iteration or time limit (outputs are still filled), a
 *     negative USBS_E_* code on error.  usbs_last_error() gives the message.
 *   * Pointers are host pointers unless the name ends in _dev (device
 *     memory of the GPU current at usbs_create, allocated by the caller).
 *   * usbs_create deep-copies the problem; the caller may free its arrays
 *     when it returns.  The handle owns all device memory it allocates and
 *     usbs_free releases it.  A handle is used by one host thread at a time.
 *   * Matrices handed over the boundary are row-major.
 *   * All quantities of the step-level entry points (usbs_op_*, usbs_step_*)
 *     are in the scaled units of App. E (eq. std_scaling): C_s = C/||C||_F,
 *     b_s = b/trace, y_s = y/||C||_F; usbs_solve reports both unit systems.
 */
#ifndef USBS_H
#define USBS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define USBS_OK 0
#define USBS_NOT_CONVERGED 1
#define USBS_E_INVALID (-1) /* malformed problem or parameters              */
#define USBS_E_NOMEM (-2)   /* device allocation failed (HBM budget)        */
#define USBS_E_DEVICE (-3)  /* HIP runtime error                            */
#define USBS_E_NUMERIC (-4) /* NaN/Inf in data or a failed inner solve      */
#define USBS_E_STATE (-5)   /* call out of order (e.g. warm start on NULL)  */

/* arithmetic of the sparse products and the sketch (Lanczos
 * re-orthogonalisation, Ritz problems and the master QP are always FP64) */
#define USBS_PREC_F64 0
#define USBS_PREC_F32 1
#define USBS_PREC_BF16 2

/* units of the stopping metrics */
#define USBS_UNITS_SCALED 0   /* the scaled problem of App. E (the paper's setting) */
#define USBS_UNITS_ORIGINAL 1 /* the problem as handed in                           */

typedef struct usbs_handle usbs_handle;

/* The SDP instance (Sec. 2.1).
 *   C: symmetric, CSR with both triangles and the diagonal (rowptr[n+1],
 *      col[nnz], val[nnz]); columns within a row in any order.
 *   A: triplets (a_row[t], a_i[t], a_j[t], a_v[t]) with a_i <= a_j, meaning
 *      <A_k, X> = sum over the triplets of row k of v * X_ij.  A pair (i,j) may
 *      appear in several rows (and several times in one row: the values add).
 *   b[m], is_ineq[m] (1 = row belongs to I, i.e. <A_k, X> <= b_k).
 *   trace: tr(X*) (or the value the constraints fix, e.g. n for MaxCut),
 *      used by the scaling of App. E.
 *   psi:  n x r row-major Gaussian test matrix of the Nystrom sketch (Sec. 4),
 *      or NULL: then the sketch runs with a test matrix generated on the device when
 *      usbs_params.psi_from_seed is set, else without the sketch. */
typedef struct usbs_problem {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *col;
    const double *val;
    int64_t m;
    int64_t n_triplets;
    const int32_t *a_row;
    const int32_t *a_i;
    const int32_t *a_j;
    const double *a_v;
    const double *b;
    const uint8_t *is_ineq;
    double trace;
    const float *psi;
} usbs_problem;

/* Parameters (defaults from usbs_default_params: the MaxCut settings of
 * App. E.1: alpha 2, rho 0.01, beta 0.25, k_c 10, k_p 1, r 10). */
typedef struct usbs_params {
    double alpha, rho, beta;
    int32_t k_c, k_p, r;
    double eps_gap, eps_infeas; /* stop when both relative errors <= eps   */
    int32_t units;              /* USBS_UNITS_*                            */
    int32_t max_iters;
    double time_limit;          /* seconds, <= 0 for none                  */
    int32_t lanczos_steps;      /* block steps per restart cycle (block 8; default 8, i.e.
                                   64 new Krylov vectors per cycle)          */
    int32_t lanczos_max_restarts; /* restart cycles of the in-iteration eigen-solve (default 10,
                                     the paper's; the certifying solves use at least 30)     */
    double lanczos_tol;         /* residual / spectral-radius estimate inside the iteration */
    double lanczos_tol_final;   /* same, for f(y0) and the certified f(y_T) at convergence  */
    int32_t precision;          /* USBS_PREC_*                             */
    uint64_t seed;              /* start block of the cold Lanczos solve   */
    void *stream;               /* hipStream_t, NULL = default stream       */
    int32_t verbose;
    int32_t autotune;           /* launch-shape tuning at usbs_create, cached per
                                   (device, n bucket, nonzeros per row, precision):
                                   0 = built-in shapes; 1 (default) = shapes that
                                   leave every result bitwise unchanged (SpMM columns
                                   per lane, grid of the MFMA updates); 2 = also the
                                   partition of the matrix-core reductions (faster,
                                   but rounding then depends on the choice)          */
    double lanczos_tol_rest;    /* residual tolerance of Ritz pairs 2..k_c inside the iteration
                                   (pair 1 uses lanczos_tol); <= 0: sqrt(lanczos_tol)          */
    uint64_t psi_seed;          /* seed of the device-generated test matrix                    */
    int32_t psi_from_seed;      /* != 0 and usbs_problem.psi == NULL: the n x r test matrix of
                                   the sketch (Sec. 4, i.i.d. N(0, 1)) is generated on the
                                   device: entry (i, c) from the Philox4x32-10 block (Salmon et
                                   al., SC'11) with counter (i mod 2^32, i div 2^32, c div 2, 0)
                                   and key (seed mod 2^32, seed div 2^32), words w0..w3,
                                   u1 = ((w1 w0 >> 11) + 1) 2^-53, u2 = (w3 w2 >> 11) 2^-53, and
                                   the Box-Muller pair sqrt(-2 ln u1) (cos, sin)(2 pi u2) for the
                                   even and odd column; stored as float32.  Row i depends only
                                   on (seed, i), so a warm start keeps the old rows.  0: the
                                   caller passes psi (or NULL for no sketch).                  */
} usbs_params;

typedef struct usbs_result {
    double primal_obj;        /* <C, X_T>, original units                         */
    double dual_bound;        /* f(y_T), original units (>= p* when alpha >= 2 tr X*) */
    double primal_obj_scaled; /* <C_s, X_T>                                       */
    double f_scaled;          /* f(y_T) in scaled units                           */
    double rel_gap;           /* |f - <C,X>| / (1 + |<C,X>|), units per params    */
    double rel_infeas;        /* dist(A X, K) / (1 + ||b||), units per params     */
    double lambda_max;        /* largest Ritz value of C_s - A^* y at the last candidate */
    double sketch_primal_obj; /* <C, Xhat> of the Nystrom reconstruction (original units) */
    double sketch_rel_infeas; /* dist(A Xhat, K)/(1+||b||) (units per params)     */
    double rel_gap_scaled, rel_infeas_scaled;     /* the paper's metric on the scaled problem */
    double rel_gap_original, rel_infeas_original; /* the same formulas in original units     */
    double seconds;
    int64_t lanczos_matvecs;  /* columns multiplied by C - A^* y                  */
    int32_t iters, descents, ipm_iters, status;
    int32_t lanczos_unconverged; /* in-iteration eigen-solves that hit the restart limit */
    int32_t stall_recoveries;    /* re-evaluations of f at the centre with the tight
                                    eigen-solve after 25 consecutive null steps           */
} usbs_result;

int usbs_default_params(usbs_params *prm);

/* Validate, scale (App. E) and upload the problem; cold start of Alg. 1
 * (y0 = 0, V0 = top-k eigenvectors of C_s, Xbar0 = 0). */
int usbs_create(const usbs_problem *prob, const usbs_params *prm, usbs_handle **out);

/* Run Alg. 1 until both relative errors are <= eps or a limit is hit.
 * y_out[m] (original units), U_out[n*r], lam_out[r] (rank-r Nystrom factors
 * of Xbar, App. C.1, original units) may each be NULL. */
int usbs_solve(usbs_handle *h, usbs_result *res, double *y_out, double *U_out, double *lam_out);

/* Warm start (Sec. 5.1): replace the problem by a grown one whose first
 * n_old vertices, first m_old constraint rows and their data are unchanged
 * (appended vertices/rows only).  y, Xbar's tracked quantities and the
 * sketch are padded with zeros and rescaled to the new scaling; V is padded
 * with zero rows and re-orthonormalised.  The next usbs_solve continues. */
int usbs_warm_start(usbs_handle *h, const usbs_problem *grown);

void usbs_free(usbs_handle *h); /* NULL-safe */
/* The message of the handle's last error; with h = NULL, that of the calling thread's
 * last failed handle-free call (usbs_sketch_update_noalloc), else "NULL handle". */
const char *usbs_last_error(const usbs_handle *h);

/* Packed solve of several instances in persistent launches (Sec. 3-4, Alg. 1, on
 * one workgroup per instance).  Each launch of the packed kernel runs, for every
 * listed handle that has not finished, up to iters_per_launch iterations of Alg. 1
 * with the same steps as usbs_solve: operator shift, block Lanczos with restarts,
 * master QP (App. B.2), model and sketch update (Sec. 3.1, Sec. 4), the stopping
 * test of Sec. 5 and the certifying eigen-solve; every decision (restart test,
 * alternating maximisation, stall recovery, stopping test) is taken on the device.
 * Launches repeat until every instance has converged or hit max_iters; time_limit
 * is checked between launches.  One workgroup of 256 threads per instance, so up to
 * one instance per compute unit runs at once; instances with small n gain the most.
 *   hs[count]: distinct ready handles of the current device (n >= 48 each).  Each
 *      handle's own stream is synchronised first; the launches run on 'stream'
 *      (hipStream_t, NULL = default stream).
 *   res[count] (may be NULL), status[count] (may be NULL): per-instance results and
 *      statuses as usbs_solve reports them.  The final y of a handle is read afterwards
 *      with usbs_get_dual (original units) and X_{t+1} with usbs_get_primal; the state
 *      stays in the handle, so a later
 *      usbs_solve, usbs_warm_start or usbs_round_maxcut continues from it.
 * Returns USBS_OK when all converged, USBS_NOT_CONVERGED if any stopped at a limit,
 * else the first negative status.  Results do not depend on which other handles
 * share the launch (each workgroup reads only its own instance). */
int usbs_solve_packed(usbs_handle *const *hs, int32_t count, int32_t iters_per_launch, void *stream,
                      usbs_result *res, int32_t *status);

/* Device time of the handle's packed launches per phase, from the GPU's wall clock
 * (milliseconds, accumulated since the handle was created or last reset; every
 * instance of a launch counts its own time).  ms_out[USBS_PACK_PHASES] in this order:
 * operator products; matrix-core reductions A^T B; matrix-core updates [A A2] H;
 * Rayleigh-Ritz eigenproblems; master-QP interior point method; constraint side (QP
 * Gram sums, A on low-rank factors, dot products); small dense steps (Gram-Schmidt
 * Cholesky, restart block, model update, f^); operator shift and bound; the whole
 * launch (the rest is copies, fills and scalar steps).  reset != 0 clears the counters
 * after reading. */
#define USBS_PACK_PHASES 9
int usbs_packed_profile(usbs_handle *h, int32_t reset, double *ms_out);

/* ---------------------------------------------------------------------
 * Step-level entry points: each runs one row of the hot path on device
 * arrays, for parity testing and for callers that drive the iteration.
 * ------------------------------------------------------------------- */

/* Y_dev = (C_s - A^* y) X_dev for an n x nb block (nb in 1..16), row-major
 * with leading dimensions ldx, ldy; y_dev (length m) sets the shift
 * (Sec. 3, the operator whose lambda_max defines f). */
int usbs_op_apply(usbs_handle *h, const double *y_dev, const double *X_dev, int32_t ldx,
                  double *Y_dev, int32_t ldy, int32_t nb);

/* Top eigenpairs of C_s - A^* y (the eigen step behind f(y), Sec. 3, by
 * block Lanczos).  w (host, k values, descending), U_dev (n x 16 row-major,
 * first k columns = eigenvectors), res (host, k residual norms) may be NULL;
 * start_dev (n x 16) optional warm start.  Returns restarts used in *cycles. */
int usbs_op_eigs(usbs_handle *h, const double *y_dev, int32_t k, const double *start_dev,
                 double *w, double *U_dev, double *res, int32_t *cycles);

/* (A(W diag(lam) W^T))_k for all rows k (App. C): out_dev[m];
 * W_dev is n x q row-major (q <= 16), lam host [q]. */
int usbs_op_lowrank_A(usbs_handle *h, const double *W_dev, int32_t q, const double *lam,
                      double *out_dev);

/* Sketch update of Sec. 4: P_dev <- g P_dev + W diag(lam) (W^T Psi), with
 * W_dev n x q (q <= 16), P_dev n x r (FP64 here), the handle's Psi. */
int usbs_op_sketch_update(usbs_handle *h, double g, const double *W_dev, int32_t q,
                          const double *lam, double *P_dev);

/* Master QP data (App. B.2, eq. compressed_subprob_2) for orthonormal
 * V_dev (n x k, k <= 16), duals y_dev, w_dev = b - nu (m), zbar_dev (m),
 * scalars tau, cbar.  Outputs (host): Q11 [d*d], q12 [d], q22, h1 [d], h2,
 * d = k(k+1)/2, svec ordering of App. B (column-wise lower triangle). */
int usbs_op_qp_data(usbs_handle *h, const double *V_dev, int32_t k, const double *y_dev,
                    const double *w_dev, const double *zbar_dev, double tau, double cbar,
                    double *Q11, double *q12, double *q22, double *h1, double *h2);

/* Interior point solve of the master QP (App. B.2) on the device from host
 * data (same layout as usbs_op_qp_data).  Outputs S [k*k], eta, and the
 * Newton iteration count. */
int usbs_op_ipm(usbs_handle *h, int32_t k, const double *Q11, const double *q12, double q22,
                const double *h1, double h2, double *S, double *eta, int32_t *iters);

/* Nystrom reconstruction (App. C.1, stable fixed-rank PSD method) of the
 * sketch P_dev (n x r, FP64) with the handle's Psi: U_dev (n x r), lam (host r). */
int usbs_op_nystrom(usbs_handle *h, const double *P_dev, double *U_dev, double *lam);

/* Run t iterations of Alg. 1 (no stopping test) and copy out the state in
 * scaled units: y (m), V (n x 16, first k columns), zbar (m), Pbar (n x r),
 * scal[8] = {f, tau, cbar, primal, rel_gap, rel_infeas, lambda1, descents}.
 * Any output may be NULL. */
int usbs_step_iterate(usbs_handle *h, int32_t t, double *y, double *V, double *zbar,
                      double *Pbar, double *scal);

/* The handle's n x r test matrix Psi of the sketch (Sec. 4; the caller's or the one
 * generated from usbs_params.psi_seed): psi_out[n*r] (host, float32, row-major).
 * USBS_E_INVALID without a sketch. */
int usbs_get_test_matrix(usbs_handle *h, float *psi_out);

/* The current centre y_t of Alg. 1 in original units (y = ||C||_F y_s, App. E):
 * y_out[m] (host).  Reads the state a usbs_solve_packed run leaves in the handle. */
int usbs_get_dual(usbs_handle *h, double *y_out);

/* The primal iterate of the last iteration of Alg. 1 (the one the stopping test of
 * Sec. 5, eq. relative_error_tol, judged), so that another program can re-evaluate
 * the certificate.  In scaled units (App. E):
 *     X_{t+1} = alpha ((eta / tau_t) Xbar_t + V_t S V_t^T)        (App. B.2 variables)
 *   ax_out[m]     A X_{t+1}, the constraint values whose distance to K is the
 *                 infeasibility;
 *   cx_out        <C_s, X_{t+1}>, the primal objective of the relative gap;
 *   V_out[n*k]    the bundle V_t the QP solution refers to (row-major, k = k_c + k_p);
 *   S_out[k*k]    the master-QP solution S (row-major, symmetric PSD);
 *   eta_out       its eta;  g_out = alpha eta / tau_t (0 while tau_t = 0).
 * With zbar (A Xbar_{t+1}), tau and cbar from usbs_step_iterate(h, 0, ...), the model
 * update of Sec. 3.1 gives A X_{t+1} = zbar + A(V_t (alpha S - K_c) V_t^T), where
 * K_c = Q_c Lam_c Q_c^T keeps all but the top k_p eigenpairs of alpha S.
 * Valid after usbs_solve, usbs_step_iterate with t >= 1 or usbs_solve_packed, until the
 * next usbs_warm_start; before any iteration of the current problem: USBS_E_STATE.
 * Any output may be NULL. */
int usbs_get_primal(usbs_handle *h, double *ax_out, double *cx_out, double *V_out, double *S_out,
                    double *eta_out, double *g_out);

/* Live kernel timing (HIP events on the handle's stream) for one category at a time:
 * flushes the pending events, returns the accumulated milliseconds and launch count of
 * the category being timed (optionally resetting them), then times 'category' from now
 * on (-1 = none).  Used by the benchmark for the roofline of the dominant kernel. */
#define USBS_PROF_SPMM 0   /* (C - A^* y) X block products                    */
#define USBS_PROF_REORTH 1 /* first stage of the first-pass [Q W]^T W reduction of the Krylov block
                              re-orthogonalisation (kernel k_tn_mfma<1, UNR, true>; the
                              finisher is not included)                                      */
#define USBS_PROF_RITZ 2   /* projected (Rayleigh-Ritz) eigenproblem          */
#define USBS_PROF_IPM 3    /* master-QP interior point solve                  */
#define USBS_PROF_UPDATE 4 /* first Gram-Schmidt update of a Krylov block fused with the second
                              pass's [Q W]^T W reduction (kernel k_nn_tn_mfma)               */
#define USBS_PROF_COUNT 5
int usbs_profile(usbs_handle *h, int32_t category, int32_t reset, double *ms_total, int64_t *launches);

/* Rounding of a MaxCut relaxation (App. E.1): the r cuts x_c = sign(U[:, c]) (ties to
 * +1) given by the columns of the Nystrom factor of the current sketch are evaluated as
 * x_c^T C x_c in FP64 (original units; for C = L/4 this is the cut weight) and the largest
 * is returned: x_out[n] (host, +1/-1, may be NULL), *cut_out, *column_out (the column of U,
 * first of equal values) and cuts_out[r] (every column's value); each output may be NULL.
 * Needs a sketch (r > 0); the handle state is unchanged.  Defined for any problem, it is a
 * cut only for the MaxCut form. */
int usbs_round_maxcut(usbs_handle *h, int8_t *x_out, double *cut_out, int32_t *column_out,
                      double *cuts_out);

/* Launch shapes chosen for this handle: out[5] = {SpMM variant for 8 columns, for 16
 * columns (0/1/2 = 1/2/4 columns per lane), grid cap of the MFMA update, workgroup cap
 * and rows in flight of the matrix-core reductions}; 0 = built-in default. */
int usbs_get_tuning(const usbs_handle *h, int32_t *out);

/* Scaling factors of the handle's problem: sigma = ||C||_F, trace. */
int usbs_get_scaling(const usbs_handle *h, double *sigma, double *trace);

/* Upper bound of the device memory (bytes) that usbs_create allocates for this
 * problem and these parameters (used by the server's admission test); < 0 on
 * malformed input. */
int64_t usbs_footprint_bytes(const usbs_problem *prob, const usbs_params *prm);

/* ------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP stream capture,
 * serving loops or harnesses that forbid hipMalloc): the sketch update of
 * usbs_op_sketch_update without a handle and without any allocation,
 *     P_dev <- g P_dev + W_dev diag(lam) (W_dev^T psi_dev).
 *   n        rows, 0 <= n < 2^31 (n = 0 does nothing);
 *   W_dev    n x q FP64, row-major, leading dimension q, 1 <= q <= USBS_NOALLOC_MAX_Q;
 *   lam      host array [q];
 *   psi_dev  n x r FP32 test matrix, row-major, leading dimension r,
 *            1 <= r <= USBS_NOALLOC_MAX_R;
 *   P_dev    n x r FP64 sketch, row-major, leading dimension r, updated in place;
 *   stream   hipStream_t (NULL = the default stream); the call only enqueues work.
 * The device arrays belong to the caller and live on the current device.  The
 * temporaries (the reduction partials of W^T psi and the q x r product) go to one fixed
 * array of USBS_NOALLOC_SCRATCH_BYTES that each GPU the library runs on holds until the
 * process ends; its address is looked up on the first call on each device.  All calls on
 * one GPU share that array.  Each call writes all of it that it reads before reading
 * it, so nothing carries over between calls; calls that overlap on one GPU (several
 * host threads, or streams not ordered with each other) race.  The result equals
 * usbs_op_sketch_update's bit for bit.  Returns USBS_OK, USBS_E_INVALID (size out of
 * range or NULL pointer) or USBS_E_DEVICE; usbs_last_error(NULL) then gives the calling
 * thread's message. */
#define USBS_NOALLOC_MAX_Q 16
#define USBS_NOALLOC_MAX_R 16
#define USBS_NOALLOC_SCRATCH_BYTES ((512 * 16 * 16 + 16 * 16) * 8)
int usbs_sketch_update_noalloc(int64_t n, int32_t q, int32_t r, double g, const double *W_dev,
                               const double *lam, const float *psi_dev, double *P_dev, void *stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching on one GPU.
 *
 * A request is one SDP instance, optionally with a grown version of it (more
 * vertices / rows appended, as in the incremental setting of Sec. 5.1) that is
 * warm-started (usbs_warm_start) from the first solve's resident state.  A free
 * slot admits the first queued request (arrival order) whose
 * usbs_footprint_bytes fits in the remaining HBM budget, so new arrivals join as
 * slots and memory free up.  In USBS_SERVE_STREAMS mode the server owns `slots`
 * worker threads, each with its own non-blocking HIP stream of default priority,
 * and the work of several instances overlaps on the device.  In USBS_SERVE_PACKED
 * mode one scheduler thread runs every admitted instance as a workgroup of the
 * packed launches (see usbs_solve_packed): between two launches it retires
 * finished solves, prepares warm restarts of grown instances (whose f(y0) is then
 * evaluated inside the next launch) and admits queued requests, whose cold start
 * also runs inside the launch.  Results do not depend on the mix: each request's
 * computation reads only its own data and every kernel is deterministic.
 * Times are seconds since usbs_server_create.
 * ------------------------------------------------------------------------ */
typedef struct usbs_server usbs_server;

#define USBS_SERVE_STREAMS 0 /* one worker thread and stream per slot, usbs_solve per request */
#define USBS_SERVE_PACKED 1  /* one scheduler thread; every admitted instance is a workgroup of
                                the packed launches (usbs_solve_packed); arrivals join and
                                finished requests leave between launches                     */

typedef struct usbs_server_config {
    int32_t slots;            /* instances on the device at once: 1..64 (streams), 1..1024
                                 (packed)                                              */
    int64_t hbm_budget_bytes; /* admission limit on summed footprints; <= 0: 90% of the
                                 free device memory at creation                      */
    usbs_params params;       /* parameters of every solve (the stream field is ignored) */
    int32_t mode;             /* USBS_SERVE_STREAMS or USBS_SERVE_PACKED              */
    int32_t iters_per_launch; /* packed mode: iterations per launch (<= 0: 8)         */
    int64_t packed_max_n;     /* packed mode: requests whose larger instance has more
                                 vertices go to per-instance workers (usbs_solve on
                                 their own streams, the whole chip per launch) that run
                                 beside the packed launches; <= 0: 20000            */
    int32_t large_slots;      /* packed mode: number of those workers, 0..16 (< 0: 2) */
} usbs_server_config;

typedef struct usbs_served_result {
    usbs_result base;         /* the solve of the submitted instance                 */
    usbs_result grown;        /* the warm-started solve of the grown instance         */
    int32_t status_base, status_grown, has_grown;
    int32_t slot;             /* streams mode: the worker; packed mode: -1 inside the packed
                                 launches, else the per-instance worker (>= 0)          */
    int64_t footprint_bytes;
    double t_submit, t_admit, t_base_done, t_done;
} usbs_served_result;

typedef struct usbs_server_stats {
    int64_t queued, running, peak_running, completed;
    int64_t budget_bytes, used_bytes, peak_used_bytes;
    double seconds;
} usbs_server_stats;

/* Start the worker threads on the current device. */
int usbs_server_create(const usbs_server_config *cfg, usbs_server **out);
/* Queue a request (deep copy of both problems; grown may be NULL).  Returns
 * USBS_E_NOMEM if its footprint exceeds the whole budget. */
int usbs_server_submit(usbs_server *sv, const usbs_problem *prob, const usbs_problem *grown,
                       int64_t *request_id);
/* Block until the request is done and return its results (once per request).
 * The return value is the first negative status of its solves, else USBS_OK
 * (per-solve statuses, including USBS_NOT_CONVERGED, are in *out). */
int usbs_server_wait(usbs_server *sv, int64_t request_id, usbs_served_result *out);
int usbs_server_get_stats(usbs_server *sv, usbs_server_stats *out);
const char *usbs_server_last_error(const usbs_server *sv);
/* Finish every queued and running request, stop the workers, release the server. */
void usbs_server_free(usbs_server *sv);

#ifdef __cplusplus
}
#endif
#endif /* USBS_H */
