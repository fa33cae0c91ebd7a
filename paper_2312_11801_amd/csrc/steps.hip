// Small USBS-specific kernels: assembling the master QP from its reduced
// pieces, the candidate iterate, the descent test, the model update and the
// Nystrom core.  Each is a single workgroup or an elementwise map; scalars of
// the iteration live in a device array so that consecutive kernels chain
// without host round trips.
#include "steps.h"
#include "small_dense.h"
#include "syev.h"
#include "wg_steps.h"

namespace usbs {

static inline int cdiv_(long a, long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// master QP coefficients (App. B.2, eq. compressed_subprob_2, normalised form)
//   raw = [upper triangle of sum g g^T | G^T zbar | G^T y | G^T b | G^T nu]
// ---------------------------------------------------------------------------
__global__ void k_qp_finalize(int k, const double *__restrict__ raw, const double *__restrict__ VCV,
                              const double *__restrict__ sc, int has_nu, double *__restrict__ qp) {
    wg_qp_finalize(k, raw, VCV, sc, has_nu, qp);
}

void qp_finalize(hipStream_t s, int k, const double *raw, const double *VCV, const double *sc, int has_nu,
                 double *qp) {
    hipLaunchKernelGGL(k_qp_finalize, dim3(1), dim3(kWG), 0, s, k, raw, VCV, sc, has_nu, qp);
}

// g = alpha eta / tau, <C, X_{t+1}> = g cbar + alpha <V^T C V, S>
__global__ void k_post_ipm(int k, const double *__restrict__ st, const double *__restrict__ VCV, double *sc) {
    if (threadIdx.x == 0) post_ipm_scalar(k, st, VCV, sc);
}
void post_ipm(hipStream_t s, int k, const double *st, const double *VCV, double *sc) {
    hipLaunchKernelGGL(k_post_ipm, dim3(1), dim3(64), 0, s, k, st, VCV, sc);
}

// alternating maximisation (eq. dual_slack_update): nu = proj_N(b - AX - rho y)
__global__ void k_nu_update(int m, const double *__restrict__ b, const double *__restrict__ AX,
                            const double *__restrict__ y, const double *__restrict__ ineq, double rho,
                            double *__restrict__ nu, double *__restrict__ dnu) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) nu_update_elem(k, b, AX, y, ineq, rho, nu, dnu);
}
void nu_update(hipStream_t s, int m, const double *b, const double *AX, const double *y, const double *ineq,
               double rho, double *nu, double *dnu) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_nu_update, dim3(cdiv_(m, kWG)), dim3(kWG), 0, s, m, b, AX, y, ineq, rho, nu, dnu);
}

// candidate (eq. dual_update, feasible form of Sec. 3.2) and the infeasibility vector
__global__ void k_candidate(int m, const double *__restrict__ b, const double *__restrict__ AX,
                            const double *__restrict__ y, const double *__restrict__ ineq, double rho,
                            double *__restrict__ yc, double *__restrict__ e) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < m) candidate_elem(k, b, AX, y, ineq, rho, yc, e);
}
void candidate(hipStream_t s, int m, const double *b, const double *AX, const double *y, const double *ineq,
               double rho, double *yc, double *e) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_candidate, dim3(cdiv_(m, kWG)), dim3(kWG), 0, s, m, b, AX, y, ineq, rho, yc, e);
}

// lambda_max(V^T (C - A^* y~) V) with V^T A^* y~ V = smat(G^T y~)
__global__ __launch_bounds__(kWG) void k_fhat_prep(int k, const double *__restrict__ VCV,
                                                   const double *__restrict__ Gy, double *sc) {
    __shared__ FhatWork w;
    wg_fhat_prep(k, VCV, Gy, sc, &w);
}
void fhat_prep(hipStream_t s, int k, const double *VCV, const double *Gy, double *sc) {
    hipLaunchKernelGGL(k_fhat_prep, dim3(1), dim3(kWG), 0, s, k, VCV, Gy, sc);
}

// descent test (Alg. 1), f, f^ and the relative errors
__global__ void k_decide(const double *__restrict__ theta, double *sc) {
    if (threadIdx.x == 0) decide_scalar(theta, sc);
}
void decide(hipStream_t s, const double *theta, double *sc) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(64), 0, s, theta, sc);
}

// f(y_t) = alpha [theta_1]_+ + <b, y_t> from an accurate Ritz value (SC_BYT holds <b, y_t>).
// A Ritz value never exceeds lambda_max, so both the stored f and the new one are lower
// bounds of f(y_t) when y_t is unchanged: keep_max then keeps the larger.
__global__ void k_refresh_f(const double *__restrict__ theta, double *sc, int keep_max) {
    if (threadIdx.x == 0) refresh_f_scalar(theta, sc, keep_max);
}
void recompute_f(hipStream_t s, const double *theta, const double *y, const double *b, int m, const RedScratch &rs,
                 double *sc, int keep_max) {
    const double *a[1] = {b}, *bb[1] = {y};
    dots(s, rs, m, a, bb, 1, sc + SC_BYT);
    hipLaunchKernelGGL(k_refresh_f, dim3(1), dim3(64), 0, s, theta, sc, keep_max);
}

__global__ void k_cond_copy(int m, const double *__restrict__ flag, const double *__restrict__ src,
                            double *__restrict__ dst) {
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m || *flag == 0.0) return;
    dst[k] = src[k];
}
void cond_copy(hipStream_t s, int m, const double *flag, const double *src, double *dst) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_cond_copy, dim3(cdiv_(m, kWG)), dim3(kWG), 0, s, m, flag, src, dst);
}

// model update (eqs. model_update_eigendecomposition, x_bar_def; App. C tracking):
// alpha S = Q diag(lam) Q^T (descending), Q_p = first k_p columns, Q_c = rest,
// Kc = Q_c Lam_c Q_c^T, tau <- g tau + tr Lam_c, cbar <- g cbar + <Kc, V^T C V>,
// Hsk = Kc (V^T Psi) (k x r) for the sketch.
__global__ __launch_bounds__(kWG) void k_model_update(int k, int kp, int r, const double *__restrict__ st,
                                                      const double *__restrict__ VCV,
                                                      const double *__restrict__ VtPsi, double *sc,
                                                      double *__restrict__ Kc, double *__restrict__ Qp,
                                                      double *__restrict__ Hsk) {
    __shared__ ModelWork w;
    wg_model_update(k, kp, r, st, VCV, VtPsi, sc, Kc, Qp, Hsk, &w);
}
void model_update(hipStream_t s, int k, int kp, int r, const double *st, const double *VCV, const double *VtPsi,
                  double *sc, double *Kc, double *Qp, double *Hsk) {
    hipLaunchKernelGGL(k_model_update, dim3(1), dim3(kWG), 0, s, k, kp, r, st, VCV, VtPsi, sc, Kc, Qp, Hsk);
}

// Vnew[:, kc + j] = Uritz[:, kc + j] where the orthogonalised V Q_p column died
__global__ void k_fix_dead(int n, const int *__restrict__ flags, int kc, int kp, const double *__restrict__ U,
                           int ldu, double *__restrict__ Vn, int ldv) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * kp) return;
    const long i = e / kp;
    const int j = (int)(e - i * kp);
    if (flags[j]) Vn[i * ldv + kc + j] = U[i * ldu + kc + j];
}
void fix_dead(hipStream_t s, int n, const int *flags, int kc, int kp, const double *U, int ldu, double *Vn,
              int ldv) {
    if (n <= 0 || kp <= 0) return;
    hipLaunchKernelGGL(k_fix_dead, dim3(cdiv_((long)n * kp, kWG)), dim3(kWG), 0, s, n, flags, kc, kp, U, ldu, Vn,
                       ldv);
}

__global__ void k_add_small(int rows, int cols, const double *__restrict__ H, int ldh, double *__restrict__ T,
                            int ldt) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * cols) return;
    const int a = e / cols, c = e - a * cols;
    T[a * ldt + c] += H[a * ldh + c];
}
__global__ void k_pad_small(int rows, int cols, const double *__restrict__ H, int ldh, double *__restrict__ P,
                            int ldp) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= rows * ldp) return;
    const int a = e / ldp, c = e - a * ldp;
    P[e] = (c < cols) ? H[a * ldh + c] : 0.0;
}
void pad_small(hipStream_t s, int rows, int cols, const double *H, int ldh, double *P, int ldp) {
    hipLaunchKernelGGL(k_pad_small, dim3(cdiv_(rows * ldp, kWG)), dim3(kWG), 0, s, rows, cols, H, ldh, P, ldp);
}
void add_small(hipStream_t s, int rows, int cols, const double *H, int ldh, double *T, int ldt) {
    hipLaunchKernelGGL(k_add_small, dim3(cdiv_(rows * cols, kWG)), dim3(kWG), 0, s, rows, cols, H, ldh, T, ldt);
}

__global__ void k_set_int(int *p, int count, int v) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = v;
}
void set_int(hipStream_t s, int *p, int count, int v) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_set_int, dim3(cdiv_(count, kWG)), dim3(kWG), 0, s, p, count, v);
}

// ---------------------------------------------------------------------------
// Nystrom core (App. C.1; fixed-rank PSD approximation of Tropp, Yurtsever,
// Udell & Cevher 2017): from the Gram of [P | Psi] (2r x 2r) compute
//   nu = sqrt(n) eps(||P||_2), B = Psi^T (P + nu Psi) = L L^T,
//   F = (P + nu Psi) L^{-T},  F^T F = Z Sigma^2 Z^T,  U = F Z Sigma^{-1},
//   lam = max(Sigma^2 - nu, 0).
// Output H (2r x r) with U = [P | Psi] H, and lam (r).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_nystrom_core(int n, int r, const double *__restrict__ Gm,
                                                      double *__restrict__ H, double *__restrict__ lamo,
                                                      int *status) {
    __shared__ SyevWork ws;
    __shared__ double G[2 * kMaxRank * 2 * kMaxRank];
    __shared__ double B[kMaxRank * kMaxRank], Li[kMaxRank * kMaxRank], PP[kMaxRank * kMaxRank];
    __shared__ double FF[kMaxRank * kMaxRank], Z[kMaxRank * kMaxRank], w[kMaxRank + 1], tmp[kMaxRank * kMaxRank];
    __shared__ double nu_s;
    __shared__ int bad;
    const int tid = threadIdx.x;
    const int r2 = 2 * r;
    for (int e = tid; e < r2 * r2; e += kWG) G[e] = Gm[e];
    __syncthreads();
    // ||P||_2^2 = lambda_max(P^T P)
    for (int e = tid; e < r * r; e += kWG) PP[e] = G[(e / r) * r2 + (e % r)];
    __syncthreads();
    wg_syev_load(r, PP, r, nullptr, &ws);
    wg_syev_top(r, 1, 0, &ws, w, nullptr, 0);
    if (tid == 0) {
        const double nrm = sqrt(fmax(w[0], 0.0));
        int ex;
        frexp(nrm, &ex);                                 // nrm = f 2^ex, f in [0.5, 1)
        const double eps = (nrm > 0.0) ? ldexp(1.0, ex - 53) : 0.0;   // spacing of doubles at nrm
        nu_s = sqrt((double)n) * eps;
        bad = 0;
    }
    __syncthreads();
    const double nu = nu_s;
    // PsiP = Psi^T P: rows r.. of G, cols 0..r ; PsiPsi = Psi^T Psi ; PP = P^T P
    // B = Psi^T P + nu Psi^T Psi (symmetrised)
    for (int e = tid; e < r * r; e += kWG) {
        const int i = e / r, j = e - i * r;
        const double bij = G[(r + i) * r2 + j] + nu * G[(r + i) * r2 + r + j];
        const double bji = G[(r + j) * r2 + i] + nu * G[(r + j) * r2 + r + i];
        B[i * kMaxRank + j] = 0.5 * (bij + bji);
    }
    __syncthreads();
    if ((tid >> 6) == 0) {
        const bool ok = wave_chol(r, B, kMaxRank);
        if ((tid & 63) == 0 && !ok) bad = 1;
        wave_tri_inv(r, B, kMaxRank, Li, kMaxRank);   // Li = L^{-1}
    }
    __syncthreads();
    // Pn^T Pn = PP + nu (Psi^T P + P^T Psi) + nu^2 Psi^T Psi ; FF = Li (Pn^T Pn) Li^T
    for (int e = tid; e < r * r; e += kWG) {
        const int i = e / r, j = e - i * r;
        tmp[e] = G[i * r2 + j] + nu * (G[(r + i) * r2 + j] + G[i * r2 + r + j]) + nu * nu * G[(r + i) * r2 + r + j];
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += kWG) {
        const int i = e / r, j = e - i * r;
        double v = 0.0;
        for (int a = 0; a < r; ++a) v += Li[i * kMaxRank + a] * tmp[a * r + j];
        PP[e] = v;
    }
    __syncthreads();
    for (int e = tid; e < r * r; e += kWG) {
        const int i = e / r, j = e - i * r;
        double v = 0.0;
        for (int a = 0; a < r; ++a) v += PP[i * r + a] * Li[j * kMaxRank + a];
        FF[e] = v;
    }
    __syncthreads();
    wg_syev_load(r, FF, r, nullptr, &ws);
    wg_syev_top(r, r, r, &ws, w, Z, r);
    __syncthreads();
    // U = Pn Li^T Z Sigma^{-1}; Pn = [P | Psi] [I ; nu I]
    // E = Li^T Z diag(1/sigma) (r x r)
    for (int e = tid; e < r * r; e += kWG) {
        const int i = e / r, c = e - i * r;
        const double sg = sqrt(fmax(w[c], 0.0));
        double v = 0.0;
        for (int a = 0; a < r; ++a) v += Li[a * kMaxRank + i] * Z[a * r + c];
        tmp[e] = (sg > 0.0) ? v / sg : 0.0;
    }
    __syncthreads();
    for (int e = tid; e < r2 * r; e += kWG) {
        const int a = e / r, c = e - a * r;
        H[e] = (a < r) ? tmp[a * r + c] : nu * tmp[(a - r) * r + c];
    }
    for (int c = tid; c < r; c += kWG) lamo[c] = fmax(w[c] - nu, 0.0);
    if (tid == 0 && status) *status = bad;
}
void nystrom_core(hipStream_t s, int n, int r, const double *Gm, double *H, double *lam, int *status) {
    hipLaunchKernelGGL(k_nystrom_core, dim3(1), dim3(kWG), 0, s, n, r, Gm, H, lam, status);
}

__global__ void k_interleave(int n, int r, const double *__restrict__ P, const float *__restrict__ Psi,
                             double *__restrict__ out) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * 2 * r) return;
    const long i = e / (2 * r);
    const int c = (int)(e - i * 2 * r);
    out[e] = (c < r) ? P[i * r + c] : (double)Psi[i * r + (c - r)];
}
void interleave(hipStream_t s, int n, int r, const double *P, const float *Psi, double *out) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_interleave, dim3(cdiv_((long)n * 2 * r, kWG)), dim3(kWG), 0, s, n, r, P, Psi, out);
}

__global__ void k_psi_to_double(long count, const float *__restrict__ a, double *__restrict__ b) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) b[e] = (double)a[e];
}
void psi_to_double(hipStream_t s, long count, const float *a, double *b) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_psi_to_double, dim3(cdiv_(count, kWG)), dim3(kWG), 0, s, count, a, b);
}

}  // namespace usbs

namespace usbs {
// ---------------------------------------------------------------------------
// MaxCut rounding (App. E.1): x_c = sign(U[:, c]) (ties to +1) for the r columns of the
// Nystrom factor, and the quadratic forms x_c^T C_s x_c = sum_i c_ii + sum_{e in row i}
// c_e x_ic x_{col(e)c} in FP64 from the FP64 copy of the off-diagonal values.  16 lanes
// per row (lane = column); one partial sum per workgroup and column.
// ---------------------------------------------------------------------------
__global__ void k_sign_cols(int n, int r, const double *__restrict__ U, int ldu, double *__restrict__ S) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (long)n * 16) {
        const long i = e >> 4;
        const int c = (int)(e & 15);
        S[e] = (c < r) ? ((U[i * ldu + c] >= 0.0) ? 1.0 : -1.0) : 0.0;
    }
}
__global__ __launch_bounds__(kWG) void k_quad_partials(int n, int r, const int *__restrict__ rowptr,
                                                       const int *__restrict__ col, const double *__restrict__ val,
                                                       const double *__restrict__ diag, const double *__restrict__ S,
                                                       double *__restrict__ part) {
    __shared__ double red[kWG];
    const int c = threadIdx.x & 15;
    double acc = 0.0;
    for (long i = (long)blockIdx.x * (kWG / 16) + (threadIdx.x >> 4); i < n; i += (long)gridDim.x * (kWG / 16)) {
        const double xi = S[i * 16 + c];
        double s = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) s += val[e] * S[(long)col[e] * 16 + c];
        acc += diag[i] * xi * xi + xi * s;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    if (threadIdx.x < 16) {
        double t = 0.0;
        for (int g = 0; g < kWG / 16; ++g) t += red[g * 16 + threadIdx.x];
        if (threadIdx.x < r) part[(size_t)blockIdx.x * r + threadIdx.x] = t;
    }
}
int quad_forms(hipStream_t s, const RedScratch &rs, int n, int r, const int *rowptr, const int *col,
               const double *val, const double *diag, const double *U, int ldu, double *S, double *out) {
    if (n <= 0 || r <= 0) return 0;
    hipLaunchKernelGGL(k_sign_cols, dim3(cdiv_((long)n * 16, kWG)), dim3(kWG), 0, s, n, r, U, ldu, S);
    int blocks = cdiv_(n, kWG / 16 * 4);
    if (blocks > rs.max_blocks) blocks = rs.max_blocks;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_quad_partials, dim3(blocks), dim3(kWG), 0, s, n, r, rowptr, col, val, diag, S, rs.partials);
    sum_partials(s, rs.partials, blocks, r, out);
    return blocks;
}
}  // namespace usbs
