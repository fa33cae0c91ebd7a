// Top eigenpairs of a small symmetric FP64 matrix (N <= kMaxBasis) on one
// workgroup of 256 threads, for the Rayleigh-Ritz problems of the block
// Lanczos solver and the other small eigenproblems of the iteration
// (eigen-split of S, lambda_max(V^T M V), the Nystrom core).
//
//   1. Householder reduction to tridiagonal form, A = Q T Q^T, with the matrix
//      in registers (a 16 x 16 thread grid, 5 x 5 entries per thread) and the
//      reflectors stored as the rows of ws->A (two barriers per column);
//   2. eigenvalues of T by 16-section: 16 lanes share one eigenvalue and
//      evaluate Sturm counts at 15 interior points of its bracket, which
//      shrinks 16x per step (16 steps from the Gershgorin interval);
//   3. eigenvectors of T by inverse iteration (one lane per eigenvector,
//      Gaussian elimination with partial pivoting on T - lambda I);
//   4. Cholesky-QR twice on the eigenvectors (vectors of a cluster become an
//      orthonormal basis of its invariant subspace), the Gram matrix and the
//      triangular solve on the FP64 matrix cores;
//   5. back-transformation by the reflectors (16 lanes per vector, the vector in
//      registers, sums across the lanes by DPP).
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"
#include "small_dense.h"

namespace usbs {

constexpr int kSyevMaxN = kMaxBasis;
constexpr int kSyevMaxV = 16;
constexpr int kSyR = kSyevMaxN / 16;   // entries per thread and dimension in the register grid
static_assert(kSyevMaxN % 16 == 0, "the register grid tiles the matrix by 16");

struct SyevWork {
    double A[kSyevMaxN][kSyevMaxN + 1];
    double d[kSyevMaxN], e[kSyevMaxN], e2[kSyevMaxN], beta[kSyevMaxN];
    double p[2][kSyevMaxN];   // p = b A v of the current column (two buffers: columns alternate)
    double vp[2][4];          // per-wavefront shares of v^T p
    double lam[kSyevMaxV];
    double X[kSyevMaxV][kSyevMaxN + 1];
    double G[kSyevMaxV][kSyevMaxV + 1];    // Gram matrix of the eigenvectors (Cholesky-QR)
    double Li[kSyevMaxV][kSyevMaxV + 1];   // inverse of its Cholesky factor
    double U0[kSyevMaxV][kSyevMaxN], U1[kSyevMaxV][kSyevMaxN], U2[kSyevMaxV][kSyevMaxN];
    double red[8];
    double gl, gh;
};

__device__ __forceinline__ double group16_sum(double v) { return row16_sum(v); }

// number of eigenvalues of the tridiagonal (d, e) strictly below x
__device__ __forceinline__ int sturm_count(int N, const double *d, const double *e2, double x, double pivmin) {
    int c = 0;
    double q = d[0] - x;
    if (fabs(q) < pivmin) q = -pivmin;
    c += (q < 0.0);
#pragma unroll 8
    for (int i = 1; i < N; ++i) {
        q = __builtin_fma(-e2[i - 1], rcp_nr(q), d[i] - x);
        if (fabs(q) < pivmin) q = -pivmin;
        c += (q < 0.0);
    }
    return c;
}

// A: the N x N matrix already in ws->A (symmetric, full).  Outputs the nv largest
// eigenvalues (descending) into lam_out[0..nv) and the first ny <= nv eigenvectors
// into Y[r * ldy + c] (r < N).  nv, ny <= 16.  All 256 threads must call.
__device__ __forceinline__ void wg_syev_top(int N, int nv, int ny, SyevWork *ws, double *lam_out, double *Y, int ldy) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    // ---- 1. tridiagonalisation ----
    // Thread (tr, tc) = (tid >> 4, tid & 15) keeps A[tr + 16 i][tc + 16 q], i, q < kSyR, in
    // registers.  Row j (= column j) lives in the 16 lanes of row group j & 15, one DPP row of
    // one wavefront: they form the reflector H = I - b v v^T that zeroes A[j + 2:, j] from
    // their own registers and store v (zero at indices <= j and >= N) as row j of ws->A.
    // After a barrier every thread forms its share of p = b A v over its columns and sums it
    // across its row group; five lanes of each group publish p at the group's rows, and every
    // wavefront its share of v^T p.  After a second barrier every thread applies
    // A -= v w^T + w v^T, w = p - (b/2)(p^T v) v, to its registers.  Rows and columns <= j
    // are left alone (v and p vanish there).
    {
        const int tr = tid >> 4, tc = tid & 15;
        double a[kSyR][kSyR];
#pragma unroll
        for (int i = 0; i < kSyR; ++i)
#pragma unroll
            for (int q = 0; q < kSyR; ++q) {
                const int r = tr + 16 * i, c = tc + 16 * q;
                a[i][q] = (r < N && c < N) ? ws->A[r][c] : 0.0;
            }
        __syncthreads();   // ws->A now receives the reflectors
#pragma unroll
        for (int jb = 0; jb < kSyR; ++jb) {
            for (int jj = 0; jj < 16; ++jj) {
                const int j = 16 * jb + jj;
                if (j + 2 >= N) break;
                const int par = j & 1;
                if (tr == jj) {
                    // row j: a[jb][q] = A[j][tc + 16 q]
                    double nx2 = 0.0, xf = 0.0;
#pragma unroll
                    for (int q = 0; q < kSyR; ++q) {
                        const int c = tc + 16 * q;
                        const double x = a[jb][q];
                        nx2 += (c > j) ? x * x : 0.0;
                        xf += (c == j + 1) ? x : 0.0;
                    }
                    nx2 = row16_sum(nx2);
                    xf = row16_sum(xf);   // one nonzero term: exact
                    const double nx = sqrt(nx2);
                    double alpha = (xf >= 0.0) ? -nx : nx;
                    const double vn2 = nx2 - xf * xf + (xf - alpha) * (xf - alpha);
                    const double b = (nx2 > 0.0 && vn2 > 0.0) ? 2.0 / vn2 : 0.0;
                    if (b == 0.0) alpha = xf;
#pragma unroll
                    for (int q = 0; q < kSyR; ++q) {
                        const int c = tc + 16 * q;
                        ws->A[j][c] = (c == j + 1) ? xf - alpha : ((c > j + 1 && c < N) ? a[jb][q] : 0.0);
                    }
                    if (tc == 0) {
                        ws->beta[j] = b;
                        ws->e[j] = alpha;
                    }
                    if (tc == jj) ws->d[j] = a[jb][jb];
                }
                __syncthreads();
                const double b = ws->beta[j];
                if (b == 0.0) continue;   // uniform: no reflection, nothing to update
                double vr[kSyR], vc[kSyR], pr[kSyR];
#pragma unroll
                for (int i = 0; i < kSyR; ++i) {
                    vr[i] = ws->A[j][tr + 16 * i];
                    vc[i] = ws->A[j][tc + 16 * i];
                }
                double vp = 0.0;
#pragma unroll
                for (int i = 0; i < kSyR; ++i) {
                    double sdot = 0.0;
#pragma unroll
                    for (int q = 0; q < kSyR; ++q) sdot += a[i][q] * vc[q];
                    sdot = row16_sum(sdot);
                    const int r = tr + 16 * i;
                    pr[i] = (r > j && r < N) ? b * sdot : 0.0;
                    if (tc == i) {
                        ws->p[par][r] = pr[i];
                        vp = vr[i] * pr[i];
                    }
                }
                vp = wave_allsum(vp);
                if (lane == 0) ws->vp[par][wave] = vp;
                __syncthreads();
                const double K = 0.5 * b * ((ws->vp[par][0] + ws->vp[par][1]) + (ws->vp[par][2] + ws->vp[par][3]));
                double wc[kSyR];
#pragma unroll
                for (int q = 0; q < kSyR; ++q) wc[q] = ws->p[par][tc + 16 * q] - K * vc[q];
#pragma unroll
                for (int i = 0; i < kSyR; ++i) {
                    const double wr = pr[i] - K * vr[i];
#pragma unroll
                    for (int q = 0; q < kSyR; ++q) a[i][q] -= vr[i] * wc[q] + wr * vc[q];
                }
            }
        }
        // the last two diagonal entries and the last off-diagonal one
#pragma unroll
        for (int i = 0; i < kSyR; ++i)
#pragma unroll
            for (int q = 0; q < kSyR; ++q) {
                const int r = tr + 16 * i, c = tc + 16 * q;
                if (r == c && r >= N - 2 && r < N) ws->d[r] = a[i][q];
                if (r == N - 1 && c == N - 2) ws->e[N - 2] = a[i][q];
            }
        if (tid == 0 && N >= 3) ws->beta[N - 2] = 0.0;
    }
    __syncthreads();
    // Gershgorin bracket of T on wavefront 0
    if (wave == 0) {
        double gl = 1e300, gh = -1e300;
        for (int i = lane; i < N; i += 64) {
            const double r = (i > 0 ? fabs(ws->e[i - 1]) : 0.0) + (i + 1 < N ? fabs(ws->e[i]) : 0.0);
            gl = fmin(gl, ws->d[i] - r);
            gh = fmax(gh, ws->d[i] + r);
            if (i + 1 < N) ws->e2[i] = ws->e[i] * ws->e[i];
        }
        gl = wave_min(gl);
        gh = wave_max(gh);
        if (lane == 0) {
            const double tn = fmax(fabs(gl), fabs(gh));
            // widen slightly so that the bracket certainly contains every eigenvalue
            ws->gl = gl - 4e-16 * tn - 1e-300;
            ws->gh = gh + 4e-16 * tn + 1e-300;
            ws->red[0] = tn;
        }
    }
    __syncthreads();
    // ---- 2. eigenvalues by 16-section ----
    {
        const double tn = ws->red[0];
        const double pivmin = fmax(1e-290, 1e-300 * tn * tn);
        const int g = tid >> 4, l = tid & 15;   // group g handles the g-th largest eigenvalue
        if (g < nv) {
            const int kidx = N - 1 - g;        // ascending index of the target
            double lo = ws->gl, hi = ws->gh;
            for (int it = 0; it < 18; ++it) {
                const double x = lo + (hi - lo) * (double)l * (1.0 / 16.0);
                const int cnt = (l == 0) ? -1 : sturm_count(N, ws->d, ws->e2, x, pivmin);
                // lanes with count <= kidx bound the eigenvalue from below, the others from above
                double cand_lo = (l > 0 && cnt <= kidx) ? x : -1e308;
                double cand_hi = (l > 0 && cnt > kidx) ? x : 1e308;
                cand_lo = row16_max(cand_lo);
                cand_hi = row16_min(cand_hi);
                if (cand_lo > -1e308) lo = cand_lo;
                if (cand_hi < 1e308) hi = cand_hi;
                if (hi - lo <= 1e-15 * tn) break;   // absolute accuracy eps * ||T||, as a stable solver
            }
            if (l == 0) ws->lam[g] = 0.5 * (lo + hi);
        }
    }
    __syncthreads();
    // ---- 3. inverse iteration: lane c < ny of each wave handles vector c (wave = c / 16 spread) ----
    // The running right-hand side entries are carried in registers; LDS holds the
    // final entries and the rows of U only (no store-to-load chains).
    {
        const int c = (tid & 3) * 4 + (tid >> 6);   // spread vectors over the 4 waves
        const bool act = (tid & 63) < 4 && c < ny;
        if (act) {
            const double lam = ws->lam[c];
            const double tn = ws->red[0];
            const double tiny = fmax(1e-300, 2.2e-16 * tn);
            double *x = ws->X[c];
            uint32_t st = 0x9E3779B9u * (uint32_t)(c + 1);
            for (int i = 0; i < N; ++i) {
                st = st * 1664525u + 1013904223u;
                x[i] = ((double)(st >> 8) * (1.0 / 16777216.0)) - 0.5;
            }
            // one solve: with lambda accurate to ~1e-15 ||T|| the target component grows by
            // ~gap / 1e-15 against the others (vectors of a cluster span its invariant
            // subspace and are orthonormalised below)
            for (int rep = 0; rep < 1; ++rep) {
                // eliminate T - lambda I with partial pivoting; rows of U in U0/U1/U2.
                // Branch-free (the four lanes of a wave follow different vectors) with the
                // next row's entries loaded one step ahead.
                double c0 = ws->d[0] - lam, c1 = (N > 1) ? ws->e[0] : 0.0;
                double xc = x[0];
                double ei = (N > 1) ? ws->e[0] : 0.0, dn = (N > 1) ? ws->d[1] : 0.0;
                double en = (N > 2) ? ws->e[1] : 0.0, xn = (N > 1) ? x[1] : 0.0;
                for (int i = 0; i + 1 < N; ++i) {
                    // prefetch row i + 2
                    const double ei2 = (i + 2 < N) ? ws->e[i + 1] : 0.0;
                    const double dn2 = (i + 2 < N) ? ws->d[i + 2] : 0.0;
                    const double en2 = (i + 3 < N) ? ws->e[i + 2] : 0.0;
                    const double xn2 = (i + 2 < N) ? x[i + 2] : 0.0;
                    const double an = dn - lam;
                    const bool keep = fabs(c0) >= fabs(ei);
                    const double piv = (c0 == 0.0) ? tiny : c0;
                    const double mlt = keep ? ei * rcp_nr(piv) : c0 * rcp_nr(ei);
                    ws->U0[c][i] = keep ? piv : ei;
                    ws->U1[c][i] = keep ? c1 : an;
                    ws->U2[c][i] = keep ? 0.0 : en;
                    x[i] = keep ? xc : xn;
                    const double xnew = keep ? xn - mlt * xc : xc - mlt * xn;
                    const double c0n = keep ? an - mlt * c1 : c1 - mlt * an;
                    const double c1n = keep ? en : -mlt * en;
                    xc = xnew;
                    c0 = c0n;
                    c1 = c1n;
                    ei = ei2;
                    dn = dn2;
                    en = en2;
                    xn = xn2;
                }
                x[N - 1] = xc;
                ws->U0[c][N - 1] = (fabs(c0) < tiny) ? (c0 < 0.0 ? -tiny : tiny) : c0;
                // back substitution with x_{i+1}, x_{i+2} carried; track max |x_i|
                double x1 = 0.0, x2 = 0.0, mx = 0.0;
                for (int i = N - 1; i >= 0; --i) {
                    double v = x[i];
                    if (i + 1 < N) v -= ws->U1[c][i] * x1;
                    if (i + 2 < N) v -= ws->U2[c][i] * x2;
                    const double u = ws->U0[c][i];
                    const double u0 = (fabs(u) < tiny) ? (u < 0.0 ? -tiny : tiny) : u;
                    const double xi = v * rcp_nr(u0);   // the reciprocal is off the chain through x
                    x[i] = xi;
                    mx = fmax(mx, fabs(xi));
                    x2 = x1;
                    x1 = xi;
                }
                const double inv = (mx > 0.0) ? 1.0 / mx : 1.0;
                double s = 0.0;
                for (int i = 0; i < N; ++i) {
                    const double t = x[i] * inv;
                    s += t * t;
                }
                const double sc = inv / sqrt(s);
                for (int i = 0; i < N; ++i) x[i] *= sc;
            }
        }
    }
    __syncthreads();
    // ---- 4. orthonormalise the ny vectors: Cholesky-QR twice ----
    // Wavefront 0 forms G = X X^T on the FP64 matrix cores (both operands are entry
    // (m, 4q + kq) of X) and its Cholesky factor in registers; a pivot at or below 1e-28
    // zeroes its vector.  Then X <- L^{-1} X on the matrix cores, 16 positions per tile,
    // the tiles spread over the four wavefronts.
    for (int pass = 0; pass < 2 && ny > 1; ++pass) {
        const int m = lane & 15, kq = lane >> 4;
        if (wave == 0) {
            dv4 g = {0.0, 0.0, 0.0, 0.0};
            for (int q = 0; 4 * q < N; ++q) {
                const int i = 4 * q + kq;
                const double x = (m < ny && i < N) ? ws->X[m][i] : 0.0;
                g = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, g, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) ws->G[kq + 4 * v][m] = g[v];
            wave_lds_order();
            double a[16], li[16], myd;
            wave_chol_rows(ny, &ws->G[0][0], kSyevMaxV + 1, 1e-28, a, li, myd);
            if (lane < 16)
#pragma unroll
                for (int c = 0; c < 16; ++c) ws->Li[lane][c] = li[c];
        }
        __syncthreads();
        for (int t = wave; 16 * t < N; t += 4) {
            const int pos = 16 * t + m;
            dv4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int l = 4 * q + kq;
                const double x = ws->Li[m][l];
                const double y = (l < ny && pos < N) ? ws->X[l][pos] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc, 0, 0, 0);
            }
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b2 = kq + 4 * v;
                if (b2 < ny && pos < N) ws->X[b2][pos] = acc[v];
            }
        }
        __syncthreads();
    }
    // ---- 5. back-transformation x <- H_0 ... H_{N-3} x, 16 lanes per vector ----
    // Lane l of the group keeps x[l + 16 t], t < kSyR; reflector j is row j of ws->A
    // (zero outside j + 1 .. N - 1), so no index masks are needed.
    {
        const int c = tid >> 4, l = tid & 15;
        if (c < ny) {
            double xr[kSyR];
#pragma unroll
            for (int t = 0; t < kSyR; ++t) xr[t] = (l + 16 * t < N) ? ws->X[c][l + 16 * t] : 0.0;
            for (int j = N - 3; j >= 0; --j) {
                const double b = ws->beta[j];
                if (b == 0.0) continue;
                double sdot = 0.0;
#pragma unroll
                for (int t = 0; t < kSyR; ++t) sdot += ws->A[j][l + 16 * t] * xr[t];
                sdot = b * group16_sum(sdot);
#pragma unroll
                for (int t = 0; t < kSyR; ++t) xr[t] -= sdot * ws->A[j][l + 16 * t];
            }
#pragma unroll
            for (int t = 0; t < kSyR; ++t)
                if (l + 16 * t < N) ws->X[c][l + 16 * t] = xr[t];
        }
    }
    __syncthreads();
    for (int c = tid; c < nv; c += kWG) lam_out[c] = ws->lam[c];
    if (Y)
        for (int q = tid; q < N * ny; q += kWG) {
            const int r = q / ny, c = q - r * ny;
            Y[r * ldy + c] = ws->X[c][r];
        }
    __syncthreads();
}

// Load the upper triangle of the global N x N matrix (ld lda) as a full symmetric
// matrix into ws->A; rows/columns flagged in dead become decoupled with a diagonal
// below every eigenvalue (-(2 ||A||_F + 1)).
__device__ __forceinline__ void wg_syev_load(int N, const double *A, int lda, const int *dead, SyevWork *ws) {
    const int tid = threadIdx.x;
    double s = 0.0;
    for (int q = tid; q < N * N; q += kWG) {
        const int r = q / N, c = q - r * N;
        const int lo = r < c ? r : c, hi = r < c ? c : r;
        double v = A[lo * lda + hi];
        if (dead && (dead[r] || dead[c])) v = 0.0;
        ws->A[r][c] = v;
        s += v * v;
    }
    s = wave_allsum(s);
    if ((tid & 63) == 0) ws->red[1 + (tid >> 6)] = s;
    __syncthreads();
    if (dead) {
        const double fro = sqrt(ws->red[1] + ws->red[2] + ws->red[3] + ws->red[4]);
        for (int r = tid; r < N; r += kWG)
            if (dead[r]) ws->A[r][r] = -(2.0 * fro + 1.0);
    }
    __syncthreads();
}

}  // namespace usbs
