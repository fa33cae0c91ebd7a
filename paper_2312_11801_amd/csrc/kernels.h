// Launchers for the gfx950 kernels of the USBS hot path.  Every launcher
// enqueues on the given stream and returns immediately; shapes are checked by
// the caller (usbs.hip) before any launch.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace usbs {

constexpr int kWG = 256;          // threads of every workgroup
constexpr int kMaxK = 12;         // bundle width k = k_c + k_p handled by the device IPM
constexpr int kMaxSvec = kMaxK * (kMaxK + 1) / 2;
constexpr int kRitz = 16;         // Ritz vectors kept per Lanczos restart
constexpr int kBlk = 8;           // Lanczos block width
constexpr int kMaxSteps = 8;      // block steps per restart cycle
constexpr int kMaxBasis = kRitz + kBlk * kMaxSteps;   // 80
constexpr int kMaxRank = 16;      // sketch rank r

// Scratch of the two-stage reductions: one partial result per workgroup of the
// first stage; a second kernel sums them in a fixed order (deterministic).
constexpr int kRedMaxBlocks = 512;
struct RedScratch {
    double *partials;   // kRedMaxBlocks * max_elems
    int max_blocks;
    int max_elems;      // doubles per partial
    unsigned *counter;  // zero between launches: workgroups of a fused finish count in here
};

// Launch-shape choices made by the autotuner (usbs.hip).  spmm8 / spmm16: 0 = one column
// per lane, 1 = two, 2 = four (bitwise identical results); nn_cap: grid cap of the MFMA
// update (identical results); red_cap / red_unr: workgroups and rows in flight of the
// matrix-core reductions (these change the partition of the sum, hence rounding).
// 0 everywhere means the built-in defaults.
struct Tuning {
    int spmm8 = 0, spmm16 = 0, nn_cap = 0, red_cap = 0, red_unr = 0;
};
// the tuning used by the launchers called from this host thread (nullptr: defaults)
void set_tuning(const Tuning *t);

// ---- sparse operator --------------------------------------------------
// Y[i, c] = diag[i] * X[i, c] + scale * sum_e val[e] * X[col[e], c],  c < nb
void spmm(hipStream_t s, int prec, int n, const int *rowptr, const int *col, const void *val,
          double scale, const double *diag, const double *X, int ldx, double *Y, int ldy, int nb);
// d[i] = cdiag[i] - sum over the diagonal triplets of vertex i of v * y[k]
void diag_shift(hipStream_t s, int n, const int *dptr, const int *dk, const double *dv,
                const double *cdiag, const double *y, double *d);
// val[slot[u]] = (cbase[slot[u]] - sum_{t in [ptr[u], ptr[u+1])} hv[t] * y[k[t]]) / scale for the
// ns constrained off-diagonal slots (a slot may belong to several constraint rows)
void offdiag_refresh(hipStream_t s, int prec, int ns, const int *slot, const int *ptr, const int *k,
                     const double *hv, const double *cbase, const double *y, double inv_scale,
                     void *val);
// Gershgorin bound max_i (|d_i| + scale sum_e |val_e|) of the shifted operator into *out
void op_bound(hipStream_t s, const RedScratch &rs, int prec, int n, const int *rowptr, const void *val, double scale,
              const double *d, double *out);
// copy base values into the compute-precision value array
void convert_values(hipStream_t s, int prec, int nnz, const double *src, double inv_scale, void *dst);

// ---- tall-skinny dense --------------------------------------------------
// H[a*ldh + c] = beta*H + alpha * sum_i A[i*lda + a] * B[i*ldb + c]   (a < ca <= 80, c < cb <= 32,
// ca * cb <= 1280)
// post: 0 = store; 1 = Cholesky-QR factor (H must be square; writes R^{-1} into H and
//       deflation flags into flags[0..ca) with the column offset flag_off)
void tn_reduce(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca,
               const double *B, int ldb, int cb, double *H, int ldh, double alpha, double beta,
               int post = 0, int *flags = nullptr, const double *floor_ref = nullptr);
// the same product for the Krylov re-orthogonalisation, split into its first stage
// (per-workgroup partials; returns the number of partials) and the finisher.  With
// both events given, they record the first stage's own start and end (timing).
int reorth_partials(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca, const double *B,
                    int ldb, int cb, hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// (the first stage computes [A B]^T B: A^T B followed by the Gram matrix B^T B; the
// finisher writes those (ca + cb) x cb values to H)
void reorth_finish(hipStream_t s, const RedScratch &rs, int blocks, int ca, int cb, double *H, int ldh);
// one pass of block Gram-Schmidt with Pythagorean inner products from Hg = [Q W]^T W
// ((cols + 8) x 8): coef ((cols + 8) x 8) = [-H R^{-1}; R^{-1}] with Omega = G - H^T H = R^T R
// (deflated columns flagged in flags[0..8) if not null, floor 1e-10 * *floor_ref if not
// null); pass 0 writes T (cols x 8, ldt) = H and saves R; pass 1 adds H * R_saved to T.
void pip_chol(hipStream_t s, const double *Hg, int cols, int pass, double *Rsave, double *T, int ldt,
              double *coef, int *flags, const double *floor_ref);
// reorth_finish and pip_chol in one launch: the workgroups of the finish sum their outputs
// into Hg, and the last one to finish (rs.counter) runs the pass's Cholesky step on Hg
// (pass 0 with skip: *skip = 1 when the second pass may be left out, see kPass2Skip)
void finish_pip(hipStream_t s, const RedScratch &rs, int blocks, int cols, double *Hg, int pass, double *Rsave,
                double *T, int ldt, double *coef, int *flags, const double *floor_ref, int *skip = nullptr);
// out[o] = sum over g < G of part[g * nout + o] (fixed order), o < nout
void sum_partials(hipStream_t s, const double *part, int G, int nout, double *out);
void tn_reduce_f(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca,
                 const float *B, int ldb, int cb, double *H, int ldh, double alpha);
// C[i*ldc + c] = beta*C + alpha * sum_a A[i*lda + a] * H[a*ldh + c]   (c < cc <= 16, ca <= 80)
void nn_update(hipStream_t s, int n, const double *A, int lda, int ca, const double *H, int ldh,
               int cc, double *C, int ldc, double alpha, double beta);
// the same with alpha = 1 and beta read from device memory (*beta_dev) by the kernel
void nn_update_beta_dev(hipStream_t s, int n, const double *A, int lda, int ca, const double *H, int ldh, int cc,
                        double *C, int ldc, const double *beta_dev);
// C (n x cc, ldc) = [A A2] H with a second source A2 (n x ca2, ca2 <= 8) whose rows
// follow A's in H (H is (ca + ca2) x cc).  C must not overlap A; it may be A2 itself (every
// row group is read into LDS before its outputs are written).  Nothing is done when skip is
// given and *skip is set.
void nn_update2(hipStream_t s, int n, const double *A, int lda, int ca, const double *A2, int lda2, int ca2,
                const double *H, int ldh, int cc, double *C, int ldc, const int *skip = nullptr);
// the first Gram-Schmidt update of a Lanczos block fused with the second pass's reduction:
// C (n x 8, ldc) = [A A2] H (A n x ca, A2 n x 8, H (ca + 8) x 8) and one partial of
// [A C]^T C ((ca + 8) x 8) per workgroup in rs.partials; returns the workgroup count
// (reorth_finish sums the partials).  Events, if given, time this dispatch.
int nn_update2_reorth(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca, const double *A2,
                      int lda2, const double *H, int ldh, double *C, int ldc, hipEvent_t ev_start = nullptr,
                      hipEvent_t ev_stop = nullptr);
// the n x r Gaussian test matrix of the sketch from a seed (Philox4x32-10 + Box-Muller, row i
// depends only on (seed, i)), float32, row-major
void psi_from_seed(hipStream_t s, long n, int r, uint64_t seed, float *psi);
// same with a float32 destination (sketch storage)
void nn_update_f(hipStream_t s, int n, const double *A, int lda, int ca, const double *H, int ldh,
                 int cc, float *C, int ldc, double alpha, double beta);
// C (n x cc, ldc) = A (n x cc, lda) (+ copy of float)
void copy_cols(hipStream_t s, int n, const double *A, int lda, int cc, double *C, int ldc);
void fill(hipStream_t s, size_t count, double v, double *p);
// deterministic pseudo-random start block (counter hash, uniform in [-1, 1])
void random_block(hipStream_t s, int n, int cc, uint64_t seed, double *C, int ldc);
// the same columns with C[:, cc..ldc) = 0 (the whole n x ldc block is written)
void random_block_pad(hipStream_t s, int n, int cc, uint64_t seed, double *C, int ldc);

// ---- small dense problems (one workgroup) --------------------------------
// top eigenpairs of the symmetric N x N matrix A (upper triangle read, ld lda, N <= kMaxBasis):
// w[0..min(N,16)) descending, Y (N x ny, ldy) = first ny <= 16 eigenvectors; entries of
// 'dead' (length N, may be null) mark columns to push to the bottom.
void small_eig(hipStream_t s, int N, const double *A, int lda, double *w, double *Y, int ldy,
               int ny, const int *dead);

// ---- Lanczos helpers ----------------------------------------------------
// from R^T R (16 x 16) and Ritz values theta: residual norms res, convergence
// flag (res_i <= tol * scale for i < kc), and Z (16 x 8) = top-8 right singular
// directions scaled by 1/sigma, so that R Z has orthonormal columns.
// convergence: residual of Ritz pair 0 <= tol * scale and of pairs 1..kc-1 <= tol_rest * scale
void lanczos_restart_prep(hipStream_t s, const double *RtR, const double *theta, int kc, double tol,
                          double tol_rest, double *res, int *flag, double *Z, double *scale_est);
// T (ld) := 0 with diag(theta) in the leading 16 x 16 block; dead flags cleared
void lanczos_reset_T(hipStream_t s, double *T, int ldt, int N, const double *theta, int *dead);
// theta = diag(TUU), Y = I (N x N)
void diag_theta(hipStream_t s, const double *TUU, int N, double *theta, double *Y);
// H = -diag(theta) (16 x 16)
void neg_diag(hipStream_t s, const double *theta, int N, double *H);
// decoupled rows (no off-diagonal entry in C - A^*(y) for any y): each carries the
// exact eigenpair (d_i, e_i).  mask_rows zeroes rows idx[0..count) of X (nc columns);
// iso_merge (one workgroup) merges the 16 largest d over those rows into the descending
// coupled Ritz values theta / residuals res (both length 16, in place; have_coupled = 0
// means there are none) and writes plan[q] = coupled column, -(row + 1) or 16 (empty);
// gather_ritz builds U (n x 16) from the coupled Ritz vectors Uc (n x 16) and plan.
void mask_rows(hipStream_t s, int count, const int *idx, double *X, int ldx, int nc);
void iso_merge(hipStream_t s, int count, const int *idx, const double *d, int have_coupled, double *theta,
               double *res, int *plan);
void gather_ritz(hipStream_t s, int n, const double *Uc, const int *plan, double *U);

// ---- USBS small steps ----------------------------------------------------
// Q11 sums and the G^T w products of the master QP (App. B.2), g_k = svec(V^T A_k V).
// out layout (d = k(k+1)/2): if do_q11, the upper triangle of sum_k g_k g_k^T row by row
// (entry (P,Q), P <= Q, at P d - P(P-1)/2 + Q - P, d(d+1)/2 values); then G^T w_j, j < nw.
void qp_gram(hipStream_t s, const RedScratch &rs, int m, const int *kptr, const int *ti,
             const int *tj, const double *tv, const double *V, int ldv, int k, const double *const *w,
             int nw, double *out, int do_q11);
// Rayleigh-Ritz update of a Lanczos restart cycle in one sweep: B (ldb) = U Y, R = MU Y -
// B diag(theta) (R may alias U), RtR (16 x 16) = R^T R; U, MU, R are n x 16 row-major, Y and
// theta on the device
void rr_update(hipStream_t s, const RedScratch &rs, int n, const double *U, const double *MU, const double *Y,
               const double *theta, double *B, int ldb, double *R, double *RtR);
// G^T w_j (layout of qp_gram's weight part, out[j d + p], nw <= 4) for constraint sets whose
// every triplet is diagonal: svec(V^T diag(a_j) V), a_j = diag(A^* w_j) from the per-vertex
// triplet lists (dptr, dk, dv) -- one sweep over the n rows of V instead of the m rows of A
void wgram(hipStream_t s, const RedScratch &rs, int n, const double *V, int ldv, int k, const int *dptr,
           const int *dk, const double *dv, const double *const *w, int nw, double *out);
// z[k] = beta*z[k] + gamma*zb[k] + alpha * sum_t v_t V_i^T K V_j  (K k x k symmetric, device)
void lowrank_A(hipStream_t s, int m, const int *kptr, const int *ti, const int *tj, const double *tv,
               const double *V, int ldv, int k, const double *K, double alpha, const double *zb,
               const double *gamma_dev, double gamma_host, double *z, double beta);
// dot products / norms with a deterministic two-stage reduction:
// out[j] = sum_i a_j[i] * b_j[i] for the given pairs (<= 8)
void dots(hipStream_t s, const RedScratch &rs, int m, const double *const *a, const double *const *b,
          int np, double *out);

struct IpmArgs {
    int k;
    double tol_mu, tol_res;
    int max_iter;
    int warm;          // start from the state in 'state' instead of the default point
};
// interior point method of App. B.2 on one workgroup.  qp = [Q11 (d*d) | q12 (d) | q22 | h1 (d) | h2]
// state = [S (k*k) | T (k*k) | eta | zeta | omega | iters | status]
void ipm(hipStream_t s, const IpmArgs &a, const double *qp, double *state);

}  // namespace usbs
