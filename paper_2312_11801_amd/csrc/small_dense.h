// Small dense linear algebra for one workgroup (256 threads) or one wavefront
// (64 lanes) of gfx950, FP64, operating on LDS arrays:
//   * parallel cyclic Jacobi (round-robin pairing) for symmetric eigenproblems
//     up to kMaxBasis (the Rayleigh-Ritz problems of block Lanczos, the
//     eigen-split of S in Sec. 3.1, the Nystrom core of App. C.1);
//   * Cholesky factors for Cholesky-QR and the Newton systems of the master QP;
//   * the interior point method of App. B.2 for the master QP.
#pragma once
#include <hip/hip_runtime.h>
#include "kernels.h"

namespace usbs {

typedef double dv4 __attribute__((ext_vector_type(4)));   // one lane's FP64 MFMA accumulator

// ---------------------------------------------------------------------------
// wavefront reductions on DPP lane permutations (VALU, no LDS round trip).
// Within a row of 16 lanes: quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror; each step combines two lanes symmetrically, so
// every lane of a row ends with the bitwise-identical result.  The four row
// results of a wavefront are read with readlane and combined in a fixed order.
// All lanes of the rows involved must be active.
// ---------------------------------------------------------------------------
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, CTRL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
__device__ __forceinline__ double lane_read(double v, int l) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double quad_sum(double v) {
    v += dpp_f64<0xB1>(v);
    v += dpp_f64<0x4E>(v);
    return v;
}
__device__ __forceinline__ double row16_sum(double v) {
    v = quad_sum(v);
    v += dpp_f64<0x141>(v);
    v += dpp_f64<0x140>(v);
    return v;
}
__device__ __forceinline__ double row16_max(double v) {
    v = fmax(v, dpp_f64<0xB1>(v));
    v = fmax(v, dpp_f64<0x4E>(v));
    v = fmax(v, dpp_f64<0x141>(v));
    v = fmax(v, dpp_f64<0x140>(v));
    return v;
}
__device__ __forceinline__ double row16_min(double v) {
    v = fmin(v, dpp_f64<0xB1>(v));
    v = fmin(v, dpp_f64<0x4E>(v));
    v = fmin(v, dpp_f64<0x141>(v));
    v = fmin(v, dpp_f64<0x140>(v));
    return v;
}
// sum over the 64 lanes; every lane receives the same value
__device__ __forceinline__ double wave_allsum(double v) {
    v = row16_sum(v);
    return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// 1/q to double precision without the IEEE division sequence, for dependent chains: the
// hardware reciprocal approximation refined by two Newton steps (each squares the
// relative error), as the compiler's fast double division does
__device__ __forceinline__ double rcp_nr(double q) {
    double r = __builtin_amdgcn_rcp(q);
    r = __builtin_fma(r, __builtin_fma(-q, r, 1.0), r);
    r = __builtin_fma(r, __builtin_fma(-q, r, 1.0), r);
    return r;
}

// 1/sqrt(x) to double precision for dependent chains: the hardware approximation refined by
// two Newton steps y <- y (3 - x y^2) / 2 (x > 0)
__device__ __forceinline__ double rsq_nr(double x) {
    double y = __builtin_amdgcn_rsq(x);
    const double h = 0.5 * x;
    y = y * __builtin_fma(-h * y, y, 1.5);
    y = y * __builtin_fma(-h * y, y, 1.5);
    return y;
}

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}
// orders this wavefront's own LDS accesses (they execute in order) without waiting for its
// outstanding memory operations
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

template <int TEAM>
__device__ __forceinline__ void team_sync() {
    if constexpr (TEAM == kWG) __syncthreads();
    else wave_sync();
}

template <int TEAM, int MAXN>
struct JacobiWork {
    int p[MAXN / 2];
    int q[MAXN / 2];
    double c[MAXN / 2];
    double s[MAXN / 2];
    double red[TEAM];
    double fro;
    double off;
    int rank[MAXN];
    int rotated;
};
using JacobiScratch = JacobiWork<kWG, kMaxBasis>;

// team-wide sum (tree in LDS); every lane gets the result
template <int TEAM, int MAXN>
__device__ __forceinline__ double team_sum(double v, JacobiWork<TEAM, MAXN> *js, int lane) {
    js->red[lane] = v;
    team_sync<TEAM>();
    for (int st = TEAM / 2; st > 0; st >>= 1) {
        if (lane < st) js->red[lane] += js->red[lane + st];
        team_sync<TEAM>();
    }
    const double r = js->red[0];
    team_sync<TEAM>();
    return r;
}

// In-place Jacobi on the symmetric Np x Np LDS matrix A (Np even); V receives
// the eigenvectors (columns) when WANTV.  On exit diag(A) holds the eigenvalues.
template <int TEAM, int MAXN, bool WANTV>
__device__ __forceinline__ void jacobi_core(int Np, double *A, double *V, int ld, JacobiWork<TEAM, MAXN> *js, int lane,
                            int max_sweeps, double tol) {
    if (WANTV)
        for (int e = lane; e < Np * Np; e += TEAM) {
            const int r = e / Np, c = e - r * Np;
            V[r * ld + c] = (r == c) ? 1.0 : 0.0;
        }
    double s = 0.0;
    for (int e = lane; e < Np * Np; e += TEAM) {
        const int r = e / Np, c = e - r * Np;
        s += A[r * ld + c] * A[r * ld + c];
    }
    const double fro = sqrt(team_sum<TEAM, MAXN>(s, js, lane));
    const int half = Np / 2;
    // a rotation is skipped when |a_pq| is below rounding of both diagonal entries (or of
    // ||A||_F for zero diagonals); a sweep without any rotation ends the iteration
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        if (lane == 0) js->rotated = 0;
        team_sync<TEAM>();
        for (int rd = 0; rd < Np - 1; ++rd) {
            if (lane < half) {
                const int ia = lane, ib = Np - 1 - lane;
                const int pa = (ia == 0) ? 0 : ((ia - 1 + rd) % (Np - 1)) + 1;
                const int pb = ((ib - 1 + rd) % (Np - 1)) + 1;
                const int p = pa < pb ? pa : pb, q = pa < pb ? pb : pa;
                const double apq = A[p * ld + q], app = A[p * ld + p], aqq = A[q * ld + q];
                double cc = 1.0, ss = 0.0;
                const double thr = fmax(tol * fmax(fabs(app), fabs(aqq)), 1e-17 * fro);
                if (fabs(apq) > thr && fabs(apq) > 1e-300) {
                    const double th = (aqq - app) / (2.0 * apq);
                    double t = 1.0 / (fabs(th) + sqrt(th * th + 1.0));
                    if (th < 0.0) t = -t;
                    cc = 1.0 / sqrt(t * t + 1.0);
                    ss = t * cc;
                    js->rotated = 1;
                }
                js->p[lane] = p;
                js->q[lane] = q;
                js->c[lane] = cc;
                js->s[lane] = ss;
            }
            team_sync<TEAM>();
            for (int e = lane; e < half * Np; e += TEAM) {
                const int pi = e / Np, k = e - pi * Np;
                const double ss = js->s[pi];
                if (ss == 0.0) continue;
                const int p = js->p[pi], q = js->q[pi];
                const double cc = js->c[pi];
                const double ap = A[p * ld + k], aq = A[q * ld + k];
                A[p * ld + k] = cc * ap - ss * aq;
                A[q * ld + k] = ss * ap + cc * aq;
            }
            team_sync<TEAM>();
            for (int e = lane; e < half * Np; e += TEAM) {
                const int pi = e / Np, k = e - pi * Np;
                const double ss = js->s[pi];
                if (ss == 0.0) continue;
                const int p = js->p[pi], q = js->q[pi];
                const double cc = js->c[pi];
                const double ap = A[k * ld + p], aq = A[k * ld + q];
                A[k * ld + p] = cc * ap - ss * aq;
                A[k * ld + q] = ss * ap + cc * aq;
                if (WANTV) {
                    const double vp = V[k * ld + p], vq = V[k * ld + q];
                    V[k * ld + p] = cc * vp - ss * vq;
                    V[k * ld + q] = ss * vp + cc * vq;
                }
            }
            team_sync<TEAM>();
        }
        const int any = js->rotated;
        team_sync<TEAM>();
        if (!any) break;
    }
}

// Load the upper triangle of the N x N global matrix A (ld lda) as a symmetric
// matrix into LDS, pad to an even size; rows flagged in 'dead' and the pad row
// become decoupled with a diagonal below every eigenvalue.  Returns Np.
__device__ __forceinline__ int wg_load_sym(int N, const double *A, int lda, const int *dead, double *sA, int ld) {
    const int tid = threadIdx.x;
    const int Np = N + (N & 1);
    __shared__ double red[kWG];
    __shared__ double fro2;
    double s = 0.0;
    for (int e = tid; e < Np * Np; e += kWG) {
        const int r = e / Np, c = e - r * Np;
        double v = 0.0;
        if (r < N && c < N) {
            const int lo = r < c ? r : c, hi = r < c ? c : r;
            v = A[lo * lda + hi];
            if (dead && (dead[r] || dead[c])) v = 0.0;
        }
        sA[r * ld + c] = v;
        s += v * v;
    }
    red[tid] = s;
    __syncthreads();
    if (tid == 0) {
        double t = 0.0;
        for (int i = 0; i < kWG; ++i) t += red[i];
        fro2 = t;
    }
    __syncthreads();
    const double sentinel = -(2.0 * sqrt(fro2) + 1.0);
    for (int r = tid; r < Np; r += kWG) {
        const bool isdead = (r >= N) || (dead && dead[r]);
        if (isdead) sA[r * ld + r] = sentinel;
    }
    __syncthreads();
    return Np;
}

__device__ __forceinline__ void wg_jacobi(int N, double *sA, double *sV, int ld, JacobiScratch *js) {
    const int Np = N + (N & 1);
    jacobi_core<kWG, kMaxBasis, true>(Np, sA, sV, ld, js, threadIdx.x, 30, 2e-16);
}

// sort descending (stable by index), w[0..N), Y[r*ldy + c] for r < N, c < ny
__device__ __forceinline__ void wg_sort_store(int N, const double *sA, const double *sV, int ld, double *w,
                                              double *Y, int ldy, int ny, JacobiScratch *js) {
    const int tid = threadIdx.x;
    const int Np = N + (N & 1);
    for (int t = tid; t < Np; t += kWG) {
        const double wt = sA[t * ld + t];
        int rk = 0;
        for (int j = 0; j < Np; ++j) {
            const double wj = sA[j * ld + j];
            rk += (wj > wt) || (wj == wt && j < t);
        }
        js->rank[t] = rk;
    }
    __syncthreads();
    for (int t = tid; t < Np; t += kWG) {
        const int rk = js->rank[t];
        if (rk < N && w) w[rk] = sA[t * ld + t];
    }
    if (Y)
        for (int e = tid; e < Np * N; e += kWG) {
            const int t = e / N, r = e - t * N;
            const int rk = js->rank[t];
            if (rk < ny) Y[r * ldy + rk] = sV[r * ld + t];
        }
    __syncthreads();
}

// ---------------------------------------------------------------------------
// Cholesky with semidefinite deflation of the nc x nc LDS matrix G (nc <= 16) on one
// wavefront, in registers: lane r keeps row r of G, then of L, then of L^{-1}, and reads
// other rows' entries by readlane (uniform lane index).  A pivot at or below thr marks its
// column dead: the pivot counts as 1 and the column of L below it as zero.  On return
// a[c] = L[r][c] (c < r), myd = L[r][r], li[c] = L^{-1}[r][c] with the rows of dead pivots
// zero; the result is the mask of dead pivots (the same in every lane).
// ---------------------------------------------------------------------------
__device__ __forceinline__ unsigned wave_chol_rows(int nc, const double *G, int ld, double thr, double (&a)[16],
                                                   double (&li)[16], double &myd) {
    const int r = threadIdx.x & 63;
#pragma unroll
    for (int c = 0; c < 16; ++c) a[c] = (r < nc && c < nc) ? G[r * ld + c] : 0.0;
    unsigned dead = 0;
    myd = 1.0;
    // right-looking: after step j, a[j] = L[r][j] at lanes r > j
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j < nc) {
            const double piv = lane_read(a[j], j);
            const bool dj = !(piv > thr);
            if (dj) dead |= 1u << j;
            const double inv = dj ? 1.0 : rsq_nr(piv), dd = dj ? 1.0 : piv * inv;
            const double lj = (r > j && !dj) ? a[j] * inv : 0.0;
            a[j] = lj;
            if (r == j) myd = dd;
#pragma unroll
            for (int c = j + 1; c < 16; ++c)
                if (c < nc) a[c] -= lj * lane_read(lj, c);
        }
    }
    // L^{-1} by rows: li holds e_r - sum_{l < j} L[r][l] Li[l][:]; at step j row j is final
    // (li_j / L[j][j], read from lane j) and the rows below subtract L[r][j] times it
    const double myinv = 1.0 / myd;
#pragma unroll
    for (int c = 0; c < 16; ++c) li[c] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        if (j < nc) {
            const double lrj = a[j];
#pragma unroll
            for (int c = 0; c <= j; ++c) {
                const double lic = lane_read(li[c] * myinv, j);
                if (r > j) li[c] -= lrj * lic;
            }
        }
    }
    const bool dr = r < 16 && ((dead >> r) & 1u);
#pragma unroll
    for (int c = 0; c < 16; ++c) li[c] = dr ? 0.0 : li[c] * myinv;
    return dead;
}

// Cholesky-QR factor (one thread-team = wavefront 0 of the calling workgroup).
// G (nc x nc, LDS, ld, nc <= 16) = W^T W.  A pivot at or below max(1e-24 * max diag,
// floor2) marks the column dead and zeroes it.  Writes the factor L back into G's lower
// triangle and R^{-1} = L^{-T} to H (ldh), dead columns zero.  Returns the mask of dead
// columns.
__device__ __forceinline__ unsigned wave_cholqr(int nc, double *G, int ld, double *H, int ldh, int *flags,
                                                double floor2) {
    const int r = threadIdx.x & 63;
    double md = 0.0;
    for (int i = 0; i < nc; ++i) md = fmax(md, G[i * ld + i]);
    double a[16], li[16], myd;
    const unsigned dead = wave_chol_rows(nc, G, ld, fmax(1e-24 * md, floor2), a, li, myd);
    wave_sync();   // every lane has read G
    if (r < nc) {
#pragma unroll
        for (int c = 0; c < 16; ++c)
            if (c < nc) {
                if (c < r) G[r * ld + c] = a[c];
                if (c == r) G[r * ld + c] = myd;
                H[c * ldh + r] = li[c];   // R^{-1}[c][r] = L^{-1}[r][c]
            }
        if (flags && ((dead >> r) & 1u)) flags[r] = 1;
    }
    wave_sync();
    return dead;
}

// ---------------------------------------------------------------------------
// wavefront-level helpers for the k x k matrices of the IPM (k <= 12)
// ---------------------------------------------------------------------------
// lower Cholesky in place (A = L L^T); returns false if not positive definite
__device__ __forceinline__ bool wave_chol(int k, double *A, int ld) {
    const int lane = threadIdx.x & 63;
    __shared__ int bad[4];
    const int w = (threadIdx.x >> 6) & 3;
    if (lane == 0) bad[w] = 0;
    wave_sync();
    for (int j = 0; j < k; ++j) {
        if (lane == 0) {
            const double piv = A[j * ld + j];
            if (!(piv > 0.0)) {
                bad[w] = 1;
                A[j * ld + j] = 1.0;
            } else {
                A[j * ld + j] = sqrt(piv);
            }
        }
        wave_sync();
        const double ljj = A[j * ld + j];
        for (int i = j + 1 + lane; i < k; i += 64) A[i * ld + j] /= ljj;
        wave_sync();
        const int m = k - j - 1;
        for (int e = lane; e < m * m; e += 64) {
            const int i = j + 1 + e / m, l = j + 1 + e % m;
            if (l <= i) A[i * ld + l] -= A[i * ld + j] * A[l * ld + j];
        }
        wave_sync();
    }
    // clear the strict upper triangle
    for (int e = lane; e < k * k; e += 64) {
        const int i = e / k, l = e - i * k;
        if (l > i) A[i * ld + l] = 0.0;
    }
    wave_sync();
    return bad[w] == 0;
}

// Li = L^{-1} (lower), lane c solves for column c
__device__ __forceinline__ void wave_tri_inv(int k, const double *L, int ld, double *Li, int ldi) {
    const int lane = threadIdx.x & 63;
    if (lane < k) {
        const int c = lane;
        double x[kMaxK];
        for (int i = 0; i < kMaxK; ++i) x[i] = 0.0;
        for (int i = c; i < k; ++i) {
            double v = (i == c) ? 1.0 : 0.0;
            for (int l = c; l < i; ++l) v -= L[i * ld + l] * x[l];
            x[i] = v / L[i * ld + i];
        }
        for (int i = 0; i < k; ++i) Li[i * ldi + c] = x[i];
    }
    wave_sync();
}

// For the symmetric positive definite k x k LDS matrix X (k <= kMaxK), on one wavefront:
// Li = L^{-1} for its lower Cholesky factor L (LDS, ld ldi, k x k) and, if Xi is not null,
// X^{-1} = Li^T Li (LDS, ld ldxi).  Lane r < k keeps row r of X, then of L, then of L^{-1}
// in registers and reads other rows' entries with readlane (uniform lane index): neither the
// factorisation nor the inversion makes an LDS round trip.  X^{-1} is one 16 x 16 x 16 FP64
// MFMA product.  Returns false if a pivot is not positive (it is replaced by 1; the results
// are then not to be used).  All 64 lanes must call.
__device__ __forceinline__ bool wave_chol_inv(int k, const double *X, int ldx, double *Li, int ldi, double *Xi,
                                              int ldxi) {
    const int r = threadIdx.x & 63;
    double a[kMaxK];
#pragma unroll
    for (int c = 0; c < kMaxK; ++c) a[c] = (r < k && c < k) ? X[r * ldx + c] : 0.0;
    bool ok = true;
    double myd = 1.0;   // L[r][r]
    // right-looking Cholesky: after step j, a[j] = L[r][j] at lanes r > j
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        if (j < k) {
            double piv = lane_read(a[j], j);
            if (!(piv > 0.0)) {
                ok = false;
                piv = 1.0;
            }
            const double inv = rsq_nr(piv), dd = piv * inv;
            const double lj = (r > j) ? a[j] * inv : 0.0;
            a[j] = lj;
            if (r == j) myd = dd;
#pragma unroll
            for (int c = j + 1; c < kMaxK; ++c)
                if (c < k) a[c] -= lj * lane_read(lj, c);
        }
    }
    // L^{-1} by rows: z holds e_r - sum_{l < j} L[r][l] Li[l][:]; at step j row j is final
    // (z_j / L[j][j], read from lane j) and the rows below subtract L[r][j] times it
    const double myinv = 1.0 / myd;
    double z[kMaxK];
#pragma unroll
    for (int c = 0; c < kMaxK; ++c) z[c] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        if (j < k) {
            const double lrj = a[j];
#pragma unroll
            for (int c = 0; c <= j; ++c) {
                const double lic = lane_read(z[c] * myinv, j);
                if (r > j) z[c] -= lrj * lic;
            }
        }
    }
    if (r < k)
#pragma unroll
        for (int c = 0; c < kMaxK; ++c)
            if (c < k) Li[r * ldi + c] = z[c] * myinv;
    wave_sync();
    if (Xi) {
        // X^{-1}[i][j] = sum_l Li[l][i] Li[l][j]: operand entry (l, i) of both MFMA inputs
        const int m = r & 15, kq = r >> 4;
        dv4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int l = 4 * q + kq;
            const double x = (l < k && m < k) ? Li[l * ldi + m] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int i = kq + 4 * v;
            if (i < k && m < k) Xi[i * ldxi + m] = acc[v];
        }
        wave_sync();
    }
    return ok;
}

// X = Li D Li^T (D symmetric), via Y = Li D
__device__ __forceinline__ void wave_congruence(int k, const double *Li, int ldi, const double *D, int ldd,
                                                double *Y, double *X, int ldx) {
    const int lane = threadIdx.x & 63;
    for (int e = lane; e < k * k; e += 64) {
        const int r = e / k, c = e - r * k;
        double s = 0.0;
        for (int a = 0; a <= r; ++a) s += Li[r * ldi + a] * D[a * ldd + c];
        Y[r * ldx + c] = s;
    }
    wave_sync();
    for (int e = lane; e < k * k; e += 64) {
        const int r = e / k, c = e - r * k;
        double s = 0.0;
        for (int b = 0; b <= c; ++b) s += Y[r * ldx + b] * Li[c * ldi + b];
        X[r * ldx + c] = s;
    }
    wave_sync();
}

// smallest eigenvalue of the symmetric k x k LDS matrix X (destroyed)
__device__ __forceinline__ double wave_max(double v) {
    v = row16_max(v);
    return fmax(fmax(lane_read(v, 0), lane_read(v, 16)), fmax(lane_read(v, 32), lane_read(v, 48)));
}
__device__ __forceinline__ double wave_min(double v) {
    v = row16_min(v);
    return fmin(fmin(lane_read(v, 0), lane_read(v, 16)), fmin(lane_read(v, 32), lane_read(v, 48)));
}

// Lower bound (tight to ~1e-13 relative) of the smallest eigenvalue of the symmetric
// k x k LDS matrix X (k <= 16, full storage, overwritten) on one wavefront: Householder
// reduction to tridiagonal form (lane r owns row r), then 64-section on Sturm counts.
// js->red (64 doubles) is the wave's scratch.
__device__ __forceinline__ double wave_min_eig(int k, double *X, int ldx, JacobiWork<64, 16> *js) {
    const int lane = threadIdx.x & 63;
    double *vv = js->red, *ww = js->red + 16, *dd = js->red + 32, *ee = js->red + 48;
    for (int j = 0; j + 2 < k; ++j) {
        const int m = k - j - 1;
        const double x = (lane < m) ? X[(j + 1 + lane) * ldx + j] : 0.0;
        const double nx2 = wave_allsum(x * x);
        const double xf = X[(j + 1) * ldx + j];
        const double nx = sqrt(nx2);
        double alpha = (xf >= 0.0) ? -nx : nx;
        const double vn2 = nx2 - xf * xf + (xf - alpha) * (xf - alpha);
        const double b = (nx2 > 0.0 && vn2 > 0.0) ? 2.0 / vn2 : 0.0;
        if (b == 0.0) alpha = xf;
        const double djj = X[j * ldx + j];
        wave_sync();
        if (lane < m) vv[lane] = (lane == 0) ? xf - alpha : x;
        if (lane == 0) {
            dd[j] = djj;
            ee[j] = alpha;
        }
        wave_sync();
        if (b != 0.0) {
            double p = 0.0;
            if (lane < m) {
                for (int q = 0; q < m; ++q) p += X[(j + 1 + lane) * ldx + j + 1 + q] * vv[q];
                p *= b;
            }
            const double K = 0.5 * b * wave_allsum((lane < m) ? p * vv[lane] : 0.0);
            if (lane < m) ww[lane] = p - K * vv[lane];
            wave_sync();
            if (lane < m) {
                const double vr = vv[lane], wr = ww[lane];
                for (int q = 0; q < m; ++q) X[(j + 1 + lane) * ldx + j + 1 + q] -= vr * ww[q] + wr * vv[q];
            }
            wave_sync();
        }
    }
    if (lane == 0) {
        if (k >= 2) {
            dd[k - 2] = X[(k - 2) * ldx + (k - 2)];
            ee[k - 2] = X[(k - 1) * ldx + (k - 2)];
        }
        dd[k - 1] = X[(k - 1) * ldx + (k - 1)];
    }
    wave_sync();
    // Gershgorin interval (every lane computes the same values)
    double lo = 1e300, hi = -1e300;
    for (int i = 0; i < k; ++i) {
        const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < k ? fabs(ee[i]) : 0.0);
        lo = fmin(lo, dd[i] - r);
        hi = fmax(hi, dd[i] + r);
    }
    const double tn = fmax(fmax(fabs(lo), fabs(hi)), 1e-300);
    lo -= 4e-16 * tn;
    hi += 4e-16 * tn;
    const double pivmin = fmax(1e-290, 1e-300 * tn * tn);
    for (int it = 0; it < 12; ++it) {
        const double x = lo + (hi - lo) * (double)lane * (1.0 / 64.0);
        int cnt = 0;
        if (lane > 0) {
            double q = dd[0] - x;
            if (fabs(q) < pivmin) q = -pivmin;
            cnt += (q < 0.0);
            for (int i = 1; i < k; ++i) {
                q = dd[i] - x - ee[i - 1] * ee[i - 1] / q;
                if (fabs(q) < pivmin) q = -pivmin;
                cnt += (q < 0.0);
            }
        }
        // lambda_min < x  iff  cnt >= 1
        const double nlo = wave_max((cnt == 0) ? x : -1e308);
        const double nhi = wave_min((cnt >= 1) ? x : 1e308);
        lo = nlo;
        if (nhi < 1e308) hi = nhi;
        if (hi - lo <= 1e-13 * fmax(fabs(lo), fabs(hi)) + 1e-16 * tn) break;
    }
    return lo;
}

// Lower bound of the smallest eigenvalue of X = Li D Li^T (Li lower triangular, D symmetric,
// k x k in LDS, k <= kMaxK) on one wavefront, to a relative 1e-8 (the IPM's step length
// takes 0.95 of the distance to the boundary and needs no more):
//  * X from two 16 x 16 x 16 FP64 MFMA products: the accumulators of D Li^T are the entries
//    (Li D)[m][kq + 4v], which is exactly the left operand of (Li D) Li^T; X is staged once
//    through Xs (16 x 16 LDS) to give lane r its row r;
//  * Householder reduction to tridiagonal form with row r in lane r's registers and the
//    entries of v and w read from their lanes by readlane (no LDS round trip);
//  * 64-section on Sturm counts of the tridiagonal matrix, whose entries every lane holds.
// All 64 lanes must call.
__device__ __forceinline__ double wave_congruence_min_eig(int k, const double *Li, int ldi, const double *D, int ldd,
                                                          double *Xs) {
    const int lane = threadIdx.x & 63;
    const int m = lane & 15, kq = lane >> 4;
    dv4 z = {0.0, 0.0, 0.0, 0.0};
    double lt[4];   // Li[m][4q + kq]: the right operand of both products
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int c = 4 * q + kq;
        const double x = (m < k && c < k) ? D[m * ldd + c] : 0.0;
        lt[q] = (m < k && c < k) ? Li[m * ldi + c] : 0.0;
        z = __builtin_amdgcn_mfma_f64_16x16x4f64(x, lt[q], z, 0, 0, 0);
    }
    dv4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < 4; ++q) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(z[q], lt[q], acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) Xs[(kq + 4 * v) * 16 + m] = acc[v];
    wave_lds_order();
    double a[kMaxK];
#pragma unroll
    for (int c = 0; c < kMaxK; ++c) a[c] = (lane < k && c < k) ? Xs[lane * 16 + c] : 0.0;
    wave_lds_order();   // Xs may be rewritten by the caller
    double dd[kMaxK], ee[kMaxK];
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        dd[j] = 0.0;
        ee[j] = 0.0;
    }
#pragma unroll
    for (int j = 0; j < kMaxK; ++j) {
        if (j + 2 < k) {
            const double x = (lane > j) ? a[j] : 0.0;
            const double nx2 = wave_allsum(x * x);
            const double xf = lane_read(a[j], j + 1);
            const double nx = sqrt(nx2);
            double alpha = (xf >= 0.0) ? -nx : nx;
            const double vn2 = nx2 - xf * xf + (xf - alpha) * (xf - alpha);
            const double b = (nx2 > 0.0 && vn2 > 0.0) ? 2.0 / vn2 : 0.0;
            if (b == 0.0) alpha = xf;
            dd[j] = lane_read(a[j], j);
            ee[j] = alpha;
            const double v = (lane == j + 1) ? xf - alpha : ((lane > j + 1) ? a[j] : 0.0);
            if (b != 0.0) {
                double p = 0.0;
#pragma unroll
                for (int c = j + 1; c < kMaxK; ++c)
                    if (c < k) p += a[c] * lane_read(v, c);
                p = (lane > j) ? b * p : 0.0;
                const double K = 0.5 * b * wave_allsum(p * v);
                const double w = p - K * v;
#pragma unroll
                for (int c = j + 1; c < kMaxK; ++c)
                    if (c < k) a[c] -= v * lane_read(w, c) + w * lane_read(v, c);
            }
        } else if (j + 2 == k) {
            dd[j] = lane_read(a[j], j);
            ee[j] = lane_read(a[j], j + 1);
        } else if (j + 1 == k) {
            dd[j] = lane_read(a[j], j);
        }
    }
    // Gershgorin interval
    double lo = 1e300, hi = -1e300;
#pragma unroll
    for (int i = 0; i < kMaxK; ++i)
        if (i < k) {
            const double r = (i > 0 ? fabs(ee[i - 1]) : 0.0) + (i + 1 < k ? fabs(ee[i]) : 0.0);
            lo = fmin(lo, dd[i] - r);
            hi = fmax(hi, dd[i] + r);
        }
    const double tn = fmax(fmax(fabs(lo), fabs(hi)), 1e-300);
    lo -= 4e-16 * tn;
    hi += 4e-16 * tn;
    const double pivmin = fmax(1e-290, 1e-300 * tn * tn);
    double e2[kMaxK];
#pragma unroll
    for (int i = 0; i < kMaxK; ++i) e2[i] = ee[i] * ee[i];
    for (int it = 0; it < 12; ++it) {
        const double x = lo + (hi - lo) * (double)lane * (1.0 / 64.0);
        int cnt = 0;
        double q = dd[0] - x;
        if (fabs(q) < pivmin) q = -pivmin;
        cnt += (q < 0.0);
#pragma unroll
        for (int i = 1; i < kMaxK; ++i)
            if (i < k) {
                q = __builtin_fma(-e2[i - 1], rcp_nr(q), dd[i] - x);
                if (fabs(q) < pivmin) q = -pivmin;
                cnt += (q < 0.0);
            }
        if (lane == 0) cnt = -1;   // lane 0 evaluates lo itself: no information
        // lambda_min < x  iff  cnt >= 1
        const double nlo = wave_max((cnt == 0) ? x : -1e308);
        const double nhi = wave_min((cnt >= 1) ? x : 1e308);
        if (nlo > -1e308) lo = nlo;
        if (nhi < 1e308) hi = nhi;
        if (hi - lo <= 1e-8 * fmax(fabs(lo), fabs(hi)) + 1e-16 * tn) break;
    }
    return lo;
}

// ---------------------------------------------------------------------------
// Master QP (App. B.2, eq. compressed_subprob_2):
//   min 1/2 s'Q11 s + eta q12's + 1/2 q22 eta^2 + h1's + h2 eta
//   s.t. eta >= 0, S PSD, 1 - tr S - eta >= 0,      s = svec(S)
// Primal-dual path following as in App. B.1/B.2: mu estimate with the factor
// 1/2, step delta = min(1, 0.95 delta_max), mu <- min(mu, gamma * estimate),
// stop when mu < tol_mu and the residuals F1, F2 are below tol_res.
// Newton direction: Delta t, Delta zeta, Delta omega are eliminated, leaving
// the symmetric positive definite bordered system in (Delta s, Delta eta)
//   [Q11 + T(x)_s S^-1 + vv'/k1 ,  q12 + v/k1          ] [ds  ]   [-F1 + r4 - v r3/k1]
//   [(q12 + v/k1)'             ,  q22 + zeta/eta + 1/k1] [deta] = [-F2 + r5 - r3/k1  ]
// with k1 = (1 - tr S - eta)/omega, r3 = mu/omega + tr S + eta - 1,
// r4 = mu svec(S^-1) - t, r5 = mu/eta - zeta, v = svec(I); eliminating deta as
// well gives the paper's eq. delta_S_linear_system2 -- the same direction.
// ---------------------------------------------------------------------------
constexpr int kMaxD = kMaxSvec + 1;
// the Newton matrix bordered by its right-hand side, (D + 1) x (D + 1), in registers: a 16 x 16
// thread grid with kIpmR x kIpmR entries per thread
constexpr int kIpmR = (kMaxD + 1 + 15) / 16;
// row stride of the Newton matrix and of the factor's rows (odd: lanes reading one column
// of the factor fall on different banks)
constexpr int kIpmLd = 16 * kIpmR + 7;

struct IpmShared {
    double M[kMaxD * kIpmLd];   // the Newton matrix (lower triangle), then the rows of its factor
    double Q11[kMaxSvec * kMaxSvec];   // staged once per solve
    double S[kMaxK * kMaxK], T[kMaxK * kMaxK], Si[kMaxK * kMaxK];
    double LSi[kMaxK * kMaxK], LTi[kMaxK * kMaxK];
    double dS[kMaxK * kMaxK], dT[kMaxK * kMaxK];
    double Y0[16 * 16], X0[16 * 16], Y1[16 * 16], X1[16 * 16];
    double s[kMaxSvec], t[kMaxSvec], F1[kMaxSvec], q12[kMaxSvec], h1[kMaxSvec], svSi[kMaxSvec];
    double rhs[kMaxD], dt[kMaxSvec];
    double ldiag[kMaxD];   // diagonal of the factor
    int pi[kMaxSvec], pj[kMaxSvec];
    double red[kWG];
    JacobiWork<64, 16> js0, js1;
    double eta, zeta, om, mu, slack, F2, maxres, kap1, r3, r5, q22, h2, dmaxS, dmaxT, deta, dzeta, dom, delta;
    int okS, okT, okM, stop;
};

// workgroup-wide sum / max: DPP within each wavefront, then the four wave results in a
// fixed order (every thread receives the same value; all 256 threads must call)
__device__ __forceinline__ double wg_reduce_sum(double v, IpmShared *sh) {
    const int tid = threadIdx.x;
    v = wave_allsum(v);
    if ((tid & 63) == 0) sh->red[tid >> 6] = v;
    __syncthreads();
    const double r = (sh->red[0] + sh->red[1]) + (sh->red[2] + sh->red[3]);
    __syncthreads();
    return r;
}
__device__ __forceinline__ double wg_reduce_max(double v, IpmShared *sh) {
    const int tid = threadIdx.x;
    v = row16_max(v);
    v = fmax(fmax(lane_read(v, 0), lane_read(v, 16)), fmax(lane_read(v, 32), lane_read(v, 48)));
    if ((tid & 63) == 0) sh->red[tid >> 6] = v;
    __syncthreads();
    const double r = fmax(fmax(sh->red[0], sh->red[1]), fmax(sh->red[2], sh->red[3]));
    __syncthreads();
    return r;
}

// symmetric Kronecker product entry (G (x)_s H)_{PQ}, P=(i,j), Q=(k,l), i>=j, k>=l:
// 1/2 s_P c_Q (H_ik G_jl + H_il G_jk + G_ik H_jl + G_il H_jk),
// s_P = sqrt2 (i != j) or 1, c_Q = 1/sqrt2 (k != l) or 1/2.
__device__ __forceinline__ double skron_entry(int i, int j, int k, int l, const double *G, const double *H, int ld) {
    const double sP = (i != j) ? 1.4142135623730951 : 1.0;
    const double cQ = (k != l) ? 0.7071067811865476 : 0.5;
    return 0.5 * sP * cQ *
           (H[i * ld + k] * G[j * ld + l] + H[i * ld + l] * G[j * ld + k] + G[i * ld + k] * H[j * ld + l] +
            G[i * ld + l] * H[j * ld + k]);
}

__device__ __forceinline__ void wg_ipm(const IpmArgs a, const double *__restrict__ qp, double *state, IpmShared *sh) {
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int k = a.k, d = k * (k + 1) / 2, D = d + 1, ldm = kIpmLd;
    for (int e = tid; e < d * d; e += kWG) sh->Q11[e] = qp[e];
    const double *Q11 = sh->Q11;
    const double r2 = 1.4142135623730951;
    // svec index tables and data
    if (tid == 0) {
        int p = 0;
        for (int j = 0; j < k; ++j)
            for (int i = j; i < k; ++i) {
                sh->pi[p] = i;
                sh->pj[p] = j;
                ++p;
            }
    }
    for (int p = tid; p < d; p += kWG) {
        sh->q12[p] = qp[d * d + p];
        sh->h1[p] = qp[d * d + d + 1 + p];
    }
    if (tid == 0) {
        sh->q22 = qp[d * d + d];
        sh->h2 = qp[d * d + d + 1 + d];
    }
    for (int e = tid; e < k * k; e += kWG) {
        const int i = e / k, j = e - i * k;
        if (a.warm) {
            // previous solution pulled 10% towards the default interior point
            sh->S[i * kMaxK + j] = 0.9 * state[e] + ((i == j) ? 0.1 / (2.0 * k) : 0.0);
            sh->T[i * kMaxK + j] = 0.9 * state[k * k + e] + ((i == j) ? 0.1 : 0.0);
        } else {
            sh->S[i * kMaxK + j] = (i == j) ? 1.0 / (2.0 * k) : 0.0;
            sh->T[i * kMaxK + j] = (i == j) ? 1.0 : 0.0;
        }
    }
    if (tid == 0) {
        if (a.warm) {
            sh->eta = 0.9 * state[2 * k * k] + 0.1 * 0.25;
            sh->zeta = 0.9 * state[2 * k * k + 1] + 0.1;
            sh->om = 0.9 * state[2 * k * k + 2] + 0.1;
        } else {
            sh->eta = 0.25;
            sh->zeta = 1.0;
            sh->om = 1.0;
        }
        sh->stop = 0;
    }
    __syncthreads();
    // initial mu = (<S,T> + eta zeta + omega slack) / (2(k+2))
    {
        double v = 0.0;
        for (int e = tid; e < k * k; e += kWG) {
            const int i = e / k, j = e - i * k;
            v += sh->S[i * kMaxK + j] * sh->T[i * kMaxK + j];
        }
        const double st = wg_reduce_sum(v, sh);
        if (tid == 0) {
            double tr = 0.0;
            for (int i = 0; i < k; ++i) tr += sh->S[i * kMaxK + i];
            sh->slack = 1.0 - tr - sh->eta;
            sh->mu = (st + sh->eta * sh->zeta + sh->om * sh->slack) / (2.0 * (k + 2));
        }
        __syncthreads();
    }
    int it = 0, status = 0;
    for (;;) {
        // s, t
        for (int p = tid; p < d; p += kWG) {
            const int i = sh->pi[p], j = sh->pj[p];
            const double f = (i == j) ? 1.0 : r2;
            sh->s[p] = f * sh->S[i * kMaxK + j];
            sh->t[p] = f * sh->T[i * kMaxK + j];
        }
        __syncthreads();
        // residuals F1 (d) and F2: 4 lanes per row of Q11
        double f2part = 0.0, mres = 0.0;
        {
            const int q4 = tid & 3;
            for (int p = tid >> 2; p < ((d + 63) & ~63); p += kWG / 4) {
                double v = 0.0;
                if (p < d) {
                    const double *row = Q11 + (size_t)p * d;
                    for (int q = q4; q < d; q += 4) v += row[q] * sh->s[q];
                }
                v = quad_sum(v);
                if (p < d && q4 == 0) {
                    const double vI = (sh->pi[p] == sh->pj[p]) ? 1.0 : 0.0;
                    v += sh->eta * sh->q12[p] + sh->h1[p] - sh->t[p] + sh->om * vI;
                    sh->F1[p] = v;
                    mres = fmax(mres, fabs(v));
                    f2part += sh->q12[p] * sh->s[p];
                }
            }
        }
        const double qs = wg_reduce_sum(f2part, sh);
        const double m1 = wg_reduce_max(mres, sh);
        if (tid == 0) {
            sh->F2 = qs + sh->eta * sh->q22 + sh->h2 - sh->zeta + sh->om;
            sh->maxres = fmax(m1, fabs(sh->F2));
            sh->stop = (sh->mu < a.tol_mu && sh->maxres < a.tol_res) || it >= a.max_iter;
            if (!(sh->mu == sh->mu) || !(sh->maxres == sh->maxres)) sh->stop = 2;
        }
        __syncthreads();
        if (sh->stop) {
            if (sh->stop == 2) status = 2;
            else if (it >= a.max_iter && !(sh->mu < a.tol_mu && sh->maxres < a.tol_res)) status = 1;
            break;
        }
        // L_S^{-1} and S^{-1} (wave 0), L_T^{-1} (wave 1)
        if (wave == 0) {
            const bool ok = wave_chol_inv(k, sh->S, kMaxK, sh->LSi, kMaxK, sh->Si, kMaxK);
            if (lane == 0) sh->okS = ok;
        } else if (wave == 1) {
            const bool ok = wave_chol_inv(k, sh->T, kMaxK, sh->LTi, kMaxK, nullptr, 0);
            if (lane == 0) sh->okT = ok;
        }
        __syncthreads();
        if (!sh->okS || !sh->okT) {
            status = 2;
            break;
        }
        for (int p = tid; p < d; p += kWG) {
            const int i = sh->pi[p], j = sh->pj[p];
            sh->svSi[p] = ((i == j) ? 1.0 : r2) * sh->Si[i * kMaxK + j];
        }
        if (tid == 0) {
            double tr = 0.0;
            for (int i = 0; i < k; ++i) tr += sh->S[i * kMaxK + i];
            sh->slack = 1.0 - tr - sh->eta;
            sh->kap1 = sh->slack / sh->om;
            sh->r3 = sh->mu / sh->om + tr + sh->eta - 1.0;
            sh->r5 = sh->mu / sh->eta - sh->zeta;
        }
        __syncthreads();
        // bordered Newton matrix and right-hand side
        const double ik1 = 1.0 / sh->kap1;
        for (int e = tid; e < D * D; e += kWG) {
            const int P = e / D, Q = e - P * D;
            if (Q > P) continue;   // lower triangle only
            double v;
            if (P < d && Q < d) {
                const int i = sh->pi[P], j = sh->pj[P], kk = sh->pi[Q], l = sh->pj[Q];
                const double vP = (i == j) ? 1.0 : 0.0, vQ = (kk == l) ? 1.0 : 0.0;
                v = Q11[(size_t)P * d + Q] + skron_entry(i, j, kk, l, sh->T, sh->Si, kMaxK) + vP * vQ * ik1;
            } else if (P == d && Q < d) {
                const double vQ = (sh->pi[Q] == sh->pj[Q]) ? 1.0 : 0.0;
                v = sh->q12[Q] + vQ * ik1;
            } else {
                v = sh->q22 + sh->zeta / sh->eta + ik1;
            }
            sh->M[P * ldm + Q] = v;
        }
        for (int p = tid; p < D; p += kWG) {
            if (p < d) {
                const double vP = (sh->pi[p] == sh->pj[p]) ? 1.0 : 0.0;
                const double r4 = sh->mu * sh->svSi[p] - sh->t[p];
                sh->rhs[p] = -sh->F1[p] + r4 - vP * sh->r3 * ik1;
            } else {
                sh->rhs[p] = -sh->F2 + sh->r5 - sh->r3 * ik1;
            }
        }
        if (tid == 0) sh->okM = 1;
        __syncthreads();
        // Cholesky of the bordered matrix [M rhs; rhs^T 0] = L L^T, right-looking, column by
        // column: its last row is y = L_M^{-1} rhs, so the forward solve comes with the
        // factorisation.  Thread (tr, tc) = (tid >> 4, tid & 15) keeps entries
        // [tr + 16 i][tc + 16 q] of the full symmetric matrix in registers.  Row j (= column
        // j) lives in the 16 lanes of row group j & 15: they scale it by the pivot's square
        // root into row j of the factor's storage (column j of L, zero at indices <= j);
        // after one barrier every thread subtracts the outer product of that column from its
        // entries (entries in finished rows or columns meet a zero factor).  One workgroup
        // barrier per column, no matrix traffic through LDS.
        {
            const int tr = tid >> 4, tc = tid & 15, D1 = D + 1;
            double am[kIpmR][kIpmR];
#pragma unroll
            for (int i = 0; i < kIpmR; ++i)
#pragma unroll
                for (int q = 0; q < kIpmR; ++q) {
                    const int r = tr + 16 * i, c = tc + 16 * q;
                    double v = 0.0;
                    if (r < D && c < D) v = (r >= c) ? sh->M[r * ldm + c] : sh->M[c * ldm + r];
                    else if (r == D && c < D) v = sh->rhs[c];
                    else if (c == D && r < D) v = sh->rhs[r];
                    am[i][q] = v;
                }
            __syncthreads();   // sh->M now receives the factor's columns as rows
#pragma unroll
            for (int jb = 0; jb < kIpmR; ++jb) {
                for (int jj = 0; jj < 16; ++jj) {
                    const int j = 16 * jb + jj;
                    if (j >= D) break;
                    if (tr == jj) {
                        double piv = row16_sum((tc == jj) ? am[jb][jb] : 0.0);   // one nonzero term
                        if (!(piv > 0.0)) {
                            if (tc == 0) sh->okM = 0;
                            piv = 1.0;
                        }
                        const double inv = rsq_nr(piv), dd = piv * inv;
#pragma unroll
                        for (int q = 0; q < kIpmR; ++q) {
                            const int c = tc + 16 * q;
                            sh->M[j * ldm + c] = (c > j && c < D1) ? am[jb][q] * inv : 0.0;
                        }
                        if (tc == 0) sh->ldiag[j] = dd;
                    }
                    __syncthreads();
                    double lr[kIpmR], lc[kIpmR];
#pragma unroll
                    for (int i = 0; i < kIpmR; ++i) {
                        lr[i] = sh->M[j * ldm + tr + 16 * i];
                        lc[i] = sh->M[j * ldm + tc + 16 * i];
                    }
#pragma unroll
                    for (int i = 0; i < kIpmR; ++i)
#pragma unroll
                        for (int q = 0; q < kIpmR; ++q) am[i][q] -= lr[i] * lc[q];
                }
            }
        }
        __syncthreads();
        if (!sh->okM) {
            status = 2;
            break;
        }
        // back substitution L^T x = y on wavefront 0: lane l keeps rows l and l + 64 in
        // registers; each solved component is broadcast from its lane and the pivots'
        // reciprocals are formed first (no LDS round trip or divide on the dependent chain).
        // L[j][i] (i < j) is entry j of the factor's row i; y_i is its entry D.
        if (wave == 0) {
            const int i0 = lane, i1 = lane + 64;
            double r0 = (i0 < D) ? sh->M[i0 * ldm + D] : 0.0, r1 = (i1 < D) ? sh->M[i1 * ldm + D] : 0.0;
            const double v0 = (i0 < D) ? 1.0 / sh->ldiag[i0] : 0.0;
            const double v1 = (i1 < D) ? 1.0 / sh->ldiag[i1] : 0.0;
            // columns in blocks of 16, from the last: a block's factor entries are loaded
            // together (sixteen loads in flight) before its sixteen dependent steps
            for (int jb = (D - 1) >> 4; jb >= 0; --jb) {
                double m0[16], m1[16];
#pragma unroll
                for (int t = 0; t < 16; ++t) {
                    const int j = 16 * jb + t;
                    m0[t] = (i0 < j && j < D) ? sh->M[i0 * ldm + j] : 0.0;
                    m1[t] = (i1 < j && j < D) ? sh->M[i1 * ldm + j] : 0.0;
                }
#pragma unroll
                for (int t = 15; t >= 0; --t) {
                    const int j = 16 * jb + t;
                    if (j < D) {
                        const double xj = (j < 64) ? lane_read(r0 * v0, j) : lane_read(r1 * v1, j - 64);
                        if (i0 == j) r0 = xj;
                        if (i1 == j) r1 = xj;
                        r0 -= m0[t] * xj;
                        r1 -= m1[t] * xj;
                    }
                }
            }
            if (i0 < D) sh->rhs[i0] = r0;
            if (i1 < D) sh->rhs[i1] = r1;
        }
        __syncthreads();
        // back substitution of the eliminated unknowns: dt = mu svec(S^{-1}) - t - (T (x)_s S^{-1}) ds,
        // where (G (x)_s H) svec(X) = svec((H X G^T + G X H^T) / 2) for the symmetric Kronecker
        // product: with W = S^{-1} dS T the product is svec((W + W^T) / 2), two k x k products
        for (int e = tid; e < k * k; e += kWG) {
            const int i = e / k, j = e - i * k;
            const int lo = i > j ? j : i, hi = i > j ? i : j;
            const int p = lo * k - lo * (lo - 1) / 2 + (hi - lo);
            const double f = (i == j) ? 1.0 : (1.0 / r2);
            sh->dS[i * kMaxK + j] = f * sh->rhs[p];
        }
        __syncthreads();
        for (int e = tid; e < k * k; e += kWG) {   // Y0 = S^{-1} dS
            const int i = e / k, j = e - i * k;
            double v = 0.0;
            for (int l = 0; l < k; ++l) v += sh->Si[i * kMaxK + l] * sh->dS[l * kMaxK + j];
            sh->Y0[i * 16 + j] = v;
        }
        __syncthreads();
        for (int e = tid; e < k * k; e += kWG) {   // X0 = S^{-1} dS T
            const int i = e / k, j = e - i * k;
            double v = 0.0;
            for (int l = 0; l < k; ++l) v += sh->Y0[i * 16 + l] * sh->T[l * kMaxK + j];
            sh->X0[i * 16 + j] = v;
        }
        __syncthreads();
        for (int p = tid; p < d; p += kWG) {
            const int i = sh->pi[p], j = sh->pj[p];
            const double v = ((i == j) ? 1.0 : r2) * 0.5 * (sh->X0[i * 16 + j] + sh->X0[j * 16 + i]);
            sh->dt[p] = sh->mu * sh->svSi[p] - sh->t[p] - v;
        }
        __syncthreads();
        for (int e = tid; e < k * k; e += kWG) {
            const int i = e / k, j = e - i * k;
            const int lo = i > j ? j : i, hi = i > j ? i : j;
            const int p = lo * k - lo * (lo - 1) / 2 + (hi - lo);
            const double f = (i == j) ? 1.0 : (1.0 / r2);
            sh->dT[i * kMaxK + j] = f * sh->dt[p];
        }
        if (tid == 0) {
            double trd = 0.0;
            for (int i = 0; i < k; ++i) trd += sh->rhs[(i * k - i * (i - 1) / 2)];
            sh->deta = sh->rhs[d];
            sh->dzeta = sh->r5 - (sh->zeta / sh->eta) * sh->deta;
            sh->dom = (sh->r3 + trd + sh->deta) / sh->kap1;
        }
        __syncthreads();
        // step lengths: lambda_min(L_S^{-1} dS L_S^{-T}) on wave 0, same for T on wave 1
        if (wave == 0) {
            const double lm = wave_congruence_min_eig(k, sh->LSi, kMaxK, sh->dS, kMaxK, sh->X0);
            if (lane == 0) sh->dmaxS = (lm < 0.0) ? -1.0 / lm : 1e300;
        } else if (wave == 1) {
            const double lm = wave_congruence_min_eig(k, sh->LTi, kMaxK, sh->dT, kMaxK, sh->X1);
            if (lane == 0) sh->dmaxT = (lm < 0.0) ? -1.0 / lm : 1e300;
        }
        __syncthreads();
        if (tid == 0) {
            double dm = fmin(sh->dmaxS, sh->dmaxT);
            if (sh->deta < 0.0) dm = fmin(dm, -sh->eta / sh->deta);
            if (sh->dzeta < 0.0) dm = fmin(dm, -sh->zeta / sh->dzeta);
            if (sh->dom < 0.0) dm = fmin(dm, -sh->om / sh->dom);
            double trd = 0.0;
            for (int i = 0; i < k; ++i) trd += sh->dS[i * kMaxK + i];
            const double dsl = -trd - sh->deta;
            if (dsl < 0.0) dm = fmin(dm, -sh->slack / dsl);
            sh->delta = fmin(1.0, 0.95 * dm);
        }
        __syncthreads();
        const double dl = sh->delta;
        for (int e = tid; e < k * k; e += kWG) {
            const int i = e / k, j = e - i * k;
            if (j < i) continue;
            const double sv = sh->S[i * kMaxK + j] + dl * 0.5 * (sh->dS[i * kMaxK + j] + sh->dS[j * kMaxK + i]);
            const double tv = sh->T[i * kMaxK + j] + dl * 0.5 * (sh->dT[i * kMaxK + j] + sh->dT[j * kMaxK + i]);
            sh->S[i * kMaxK + j] = sv;
            sh->S[j * kMaxK + i] = sv;
            sh->T[i * kMaxK + j] = tv;
            sh->T[j * kMaxK + i] = tv;
        }
        __syncthreads();
        {
            double v = 0.0;
            for (int e = tid; e < k * k; e += kWG) {
                const int i = e / k, j = e - i * k;
                v += sh->S[i * kMaxK + j] * sh->T[i * kMaxK + j];
            }
            const double st = wg_reduce_sum(v, sh);
            if (tid == 0) {
                sh->eta += dl * sh->deta;
                sh->zeta += dl * sh->dzeta;
                sh->om += dl * sh->dom;
                double tr = 0.0;
                for (int i = 0; i < k; ++i) tr += sh->S[i * kMaxK + i];
                sh->slack = 1.0 - tr - sh->eta;
                const double gam = (dl <= 0.2) ? 1.0 : 0.5 - 0.4 * dl * dl;
                const double est = (st + sh->eta * sh->zeta + sh->om * sh->slack) / (2.0 * (k + 2));
                sh->mu = fmin(sh->mu, gam * est);
            }
            __syncthreads();
        }
        ++it;
    }
    __syncthreads();
    for (int e = tid; e < k * k; e += kWG) {
        const int i = e / k, j = e - i * k;
        state[e] = sh->S[i * kMaxK + j];
        state[k * k + e] = sh->T[i * kMaxK + j];
    }
    if (tid == 0) {
        state[2 * k * k] = sh->eta;
        state[2 * k * k + 1] = sh->zeta;
        state[2 * k * k + 2] = sh->om;
        state[2 * k * k + 3] = (double)it;
        state[2 * k * k + 4] = (double)status;
    }
}

}  // namespace usbs
