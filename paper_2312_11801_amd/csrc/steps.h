// Launchers of the USBS-specific small kernels and the slots of the
// device-resident scalar array of one solver instance.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"

namespace usbs {

enum ScalarSlot {
    SC_F = 0,       // f(y_t)
    SC_TAU,         // tr Xbar
    SC_CBAR,        // <C_s, Xbar>
    SC_ETA,         // eta of the last QP
    SC_G,           // alpha eta / tau
    SC_CX,          // <C_s, X_{t+1}>
    SC_FCAND,       // f(y~)
    SC_FHAT,        // f^_t(y~)
    SC_THETA1,      // largest Ritz value at y~
    SC_BY,          // <b, y~>
    SC_YZ,          // <y~, zbar>
    SC_DIST2,       // dist(A X_{t+1}, K)^2
    SC_GAP,         // relative suboptimality
    SC_INF,         // relative infeasibility
    SC_DESC,        // descent step taken
    SC_NDESC,       // number of descent steps
    SC_ZZ,          // <zbar, zbar>
    SC_YZBAR,       // <y_t, zbar>
    SC_BZ,          // <b, zbar>
    SC_LAMV,        // lambda_max(V^T (C - A^* y~) V)
    SC_NUZ,         // <nu, zbar>
    SC_DNU,         // ||nu_new - nu||^2
    SC_BNORM,       // ||b_s||
    SC_SIGMA,       // ||C||_F
    SC_TRACE,       // tr X* of the original problem
    SC_ALPHA,
    SC_RHO,
    SC_BETA,
    SC_UNITS,
    SC_IPMIT,       // accumulated IPM iterations
    SC_IPMSTATUS,   // nonzero if an IPM failed
    SC_SCALE,       // running spectral-radius estimate of the shifted operator
    SC_BYT,         // <b, y_t>
    SC_COUNT = 40
};

void qp_finalize(hipStream_t s, int k, const double *raw, const double *VCV, const double *sc, int has_nu,
                 double *qp);
void post_ipm(hipStream_t s, int k, const double *st, const double *VCV, double *sc);
void nu_update(hipStream_t s, int m, const double *b, const double *AX, const double *y, const double *ineq,
               double rho, double *nu, double *dnu);
void candidate(hipStream_t s, int m, const double *b, const double *AX, const double *y, const double *ineq,
               double rho, double *yc, double *e);
void fhat_prep(hipStream_t s, int k, const double *VCV, const double *Gy, double *sc);
void decide(hipStream_t s, const double *theta, double *sc);
void recompute_f(hipStream_t s, const double *theta, const double *y, const double *b, int m, const RedScratch &rs,
                 double *sc, int keep_max);
void cond_copy(hipStream_t s, int m, const double *flag, const double *src, double *dst);
void model_update(hipStream_t s, int k, int kp, int r, const double *st, const double *VCV, const double *VtPsi,
                  double *sc, double *Kc, double *Qp, double *Hsk);
void fix_dead(hipStream_t s, int n, const int *flags, int kc, int kp, const double *U, int ldu, double *Vn,
              int ldv);
void add_small(hipStream_t s, int rows, int cols, const double *H, int ldh, double *T, int ldt);
// P (rows x ldp) = H (rows x cols, ld ldh) with columns cols..ldp-1 zero
void pad_small(hipStream_t s, int rows, int cols, const double *H, int ldh, double *P, int ldp);
void set_int(hipStream_t s, int *p, int count, int v);
void nystrom_core(hipStream_t s, int n, int r, const double *Gm, double *H, double *lam, int *status);
void interleave(hipStream_t s, int n, int r, const double *P, const float *Psi, double *out);
// MaxCut rounding (App. E.1): S (n x 16) = sign of the first r columns of U (ties +1);
// out[c] = S[:, c]^T C_s S[:, c] in FP64 (off-diagonal CSR values val, diagonal diag)
int quad_forms(hipStream_t s, const RedScratch &rs, int n, int r, const int *rowptr, const int *col,
               const double *val, const double *diag, const double *U, int ldu, double *S, double *out);
void psi_to_double(hipStream_t s, long count, const float *a, double *b);

}  // namespace usbs
