// Packed solver: one workgroup per USBS instance, many instances per launch.
//
// Each workgroup runs the iteration of Alg. 1 for its own instance exactly as the
// per-instance driver (usbs.hip) issues it as separate kernels: the same steps in the
// same order, the same step bodies (wg_steps.h, syev.h, small_dense.h), with each
// grid-wide reduction done by the one workgroup (so reductions sum in a different,
// still fixed, order).  The host decisions of the per-instance driver (Lanczos
// restart test, end of the alternating maximisation, stall recovery, stopping test)
// are taken on the device from the same scalars.  Instances never share data, so a
// result does not depend on which other instances share the launch.
//
// LDS: the workspaces of the steps overlay each other (steps run one after another,
// separated by workgroup barriers); the largest is the master-QP interior point
// method's.  One workgroup of 256 threads per compute unit.
#include "packed.h"

#include "kernels.h"
#include "small_dense.h"
#include "steps.h"
#include "syev.h"
#include "wg_steps.h"

namespace usbs {

namespace {

struct PackShared {
    union {
        SyevWork syev;
        IpmShared ipm;
        TnWork tn;
        NnWork nn;
        NnTnWork nt;
        QpGramWork qg;
        PipWork pip;
        RestartWork rp;
        IsoWork iso;
        FhatWork fh;
        ModelWork mu;
        double red[8][kWG];
    } u;
    double G16[16 * 17];   // Gram matrix of a Cholesky-QR (written after the reduction's LDS use)
    double sK[16 * 16];    // K of the low-rank constraint map
};

// The workgroup's LDS workspace.  Named directly by every helper (never passed as a
// pointer across a call), so that the compiler sees its address space and emits LDS
// instructions for it even in functions it does not inline.
__shared__ PackShared g_sh;

// instance context: descriptor and counters
struct Ctx {
    const PackDesc *D;
    PackState st;
    double *V, *Vn;        // current bundle and its successor (exchanged every iteration)
    bool last_conv;
};

constexpr int kPackUnr = 8;   // row groups in flight per wavefront in the reductions
// expansion cycles every tight eigen-solve runs before its convergence test counts (as in
// the per-instance driver)
constexpr int kCertifyMinCycles = 2;

// adds the device wall-clock time of its scope to one phase (every thread keeps the same
// counters; thread 0 writes them back)
struct Tick {
    unsigned long long *acc;
    unsigned long long t0;
    __device__ Tick(unsigned long long *a) : acc(a), t0(wall_clock64()) {}
    __device__ ~Tick() { *acc += wall_clock64() - t0; }
};
#define PK_TICK(c, ph) Tick tick_##ph(&(c).st.ticks[ph])

__device__ __forceinline__ void sync() { __syncthreads(); }

// ---------------------------------------------------------------------------
// elementwise helpers (all threads of the workgroup call; barrier at the end)
// ---------------------------------------------------------------------------
__device__ void pk_fill(double *p, long count, double v) {
    for (long e = threadIdx.x; e < count; e += kWG) p[e] = v;
    sync();
}
__device__ void pk_set_int(int *p, int count, int v) {
    for (int e = threadIdx.x; e < count; e += kWG) p[e] = v;
    sync();
}
__device__ void pk_copy_cols(int n, const double *A, int lda, int cc, double *C, int ldc) {
    const long tot = (long)n * cc;
    for (long e = threadIdx.x; e < tot; e += kWG) {
        const long i = e / cc;
        const int c = (int)(e - i * cc);
        C[i * ldc + c] = A[i * lda + c];
    }
    sync();
}
__device__ void pk_random_block(int n, int cc, uint64_t seed, double *C, int ldc) {
    const long tot = (long)n * cc;
    for (long e = threadIdx.x; e < tot; e += kWG) {
        const long i = e / cc;
        const int c = (int)(e - i * cc);
        C[i * ldc + c] = hash_uniform(seed, (uint64_t)e);
    }
    sync();
}

// ---------------------------------------------------------------------------
// operator: shift by A^* y, Gershgorin bound, products
// ---------------------------------------------------------------------------
template <typename VT>
__device__ void pk_offdiag_refresh_t(const PackDesc &D, const double *y, VT *val) {
    const double inv_scale = 1.0 / D.val_scale;
    for (int u = threadIdx.x; u < D.n_offt; u += kWG) {
        const int sl = D.off_slot[u];
        double v = D.cbase[sl];
        for (int t = D.off_ptr[u]; t < D.off_ptr[u + 1]; ++t) v -= D.off_hv[t] * y[D.off_k[t]];
        v *= inv_scale;
        if constexpr (sizeof(VT) == 2) val[sl] = f32_to_bf16((float)v);
        else val[sl] = (VT)v;
    }
}
template <typename VT>
__device__ double pk_row_abs(const PackDesc &D, const VT *val, int i) {
    double s = 0.0;
    for (int e = D.rowptr[i]; e < D.rowptr[i + 1]; ++e) {
        if constexpr (sizeof(VT) == 2) s += fabs((double)bf16_to_f32(val[e]));
        else s += fabs((double)val[e]);
    }
    return s;
}
// d = diag(C_s) - diag(A^* y), refreshed constrained off-diagonal values, and the
// Gershgorin bound of C_s - A^* y into sc[SC_SCALE]
__device__ void pk_shift_operator(Ctx &c, const double *y) {
    PK_TICK(c, PH_OTHER);
    const PackDesc &D = *uni(c.D);
    for (int i = threadIdx.x; i < D.n; i += kWG) {
        double v = D.cdiag[i];
        for (int e = D.dptr[i]; e < D.dptr[i + 1]; ++e) v -= D.dv[e] * y[D.dk[e]];
        D.dshift[i] = v;
    }
    if (D.n_offt > 0) {
        if (D.prec == 0) pk_offdiag_refresh_t<double>(D, y, (double *)D.val_cur);
        else if (D.prec == 1) pk_offdiag_refresh_t<float>(D, y, (float *)D.val_cur);
        else pk_offdiag_refresh_t<uint16_t>(D, y, (uint16_t *)D.val_cur);
    }
    sync();
    double mx = 0.0;
    for (int i = threadIdx.x; i < D.n; i += kWG) {
        double s;
        if (D.prec == 0) s = pk_row_abs<double>(D, (const double *)D.val_cur, i);
        else if (D.prec == 1) s = pk_row_abs<float>(D, (const float *)D.val_cur, i);
        else s = pk_row_abs<uint16_t>(D, (const uint16_t *)D.val_cur, i);
        mx = fmax(mx, fabs(D.dshift[i]) + fabs(D.val_scale) * s);
    }
    double *red = g_sh.u.red[0];
    red[threadIdx.x] = mx;
    sync();
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        sync();
    }
    if (threadIdx.x == 0) D.sc[SC_SCALE] = red[0];
    sync();
}

// Y = (off-diagonal part of val) X + diag X, nb <= 16 columns; rows two at a time per
// lane group (lanes own columns)
template <typename VT, typename ACC>
__device__ void pk_spmm_t(int n, const int *rowptr, const int *col, const VT *val, ACC scale, const double *diag,
                          const double *X, int ldx, double *Y, int ldy, int nb) {
    n = uni(n), ldx = uni(ldx), ldy = uni(ldy), nb = uni(nb);
    rowptr = uni(rowptr), col = uni(col), val = uni(val), diag = uni(diag), X = uni(X), Y = uni(Y);
    const int L = nb <= 8 ? 8 : 16;
    const int R = kWG / L;
    const int c = threadIdx.x % L, r0 = threadIdx.x / L;
    const bool act = c < nb;
    const int cc = act ? c : 0;
    for (int base = 0; base < n; base += 2 * R) {
        const int i0 = base + r0, i1 = base + R + r0;
        double v0 = 0.0, v1 = 0.0;
        if (i0 < n) v0 = spmm_row<VT, ACC>(i0, cc, rowptr, col, val, scale, diag, X, ldx);
        if (i1 < n) v1 = spmm_row<VT, ACC>(i1, cc, rowptr, col, val, scale, diag, X, ldx);
        if (act && i0 < n) Y[(size_t)i0 * ldy + c] = v0;
        if (act && i1 < n) Y[(size_t)i1 * ldy + c] = v1;
    }
    sync();
}
__device__ void pk_spmm(const PackDesc &D, const void *val, const double *diag, const double *X, int ldx, double *Y,
                        int ldy, int nb) {
    if (D.prec == 0)
        pk_spmm_t<double, double>(D.n, D.rowptr, D.col, (const double *)val, D.val_scale, diag, X, ldx, Y, ldy, nb);
    else if (D.prec == 1)
        pk_spmm_t<float, float>(D.n, D.rowptr, D.col, (const float *)val, (float)D.val_scale, diag, X, ldx, Y, ldy,
                                nb);
    else
        pk_spmm_t<uint16_t, float>(D.n, D.rowptr, D.col, (const uint16_t *)val, (float)D.val_scale, diag, X, ldx, Y,
                                   ldy, nb);
}
// (C_s - A^* y) X with the current shift
__device__ void pk_apply_op(Ctx &c, const double *X, int ldx, double *Y, int ldy, int nb) {
    PK_TICK(c, PH_SPMM);
    pk_spmm(*c.D, uni(c.D)->val_cur, uni(c.D)->dshift, X, ldx, Y, ldy, nb);
    c.st.matvecs += nb;
}
// C_s X
__device__ void pk_apply_C(Ctx &c, const double *X, int ldx, double *Y, int ldy, int nb) {
    PK_TICK(c, PH_SPMM);
    pk_spmm(*c.D, uni(c.D)->val_c, uni(c.D)->cdiag, X, ldx, Y, ldy, nb);
}

// ---------------------------------------------------------------------------
// tall-skinny products on the matrix cores (one workgroup)
// ---------------------------------------------------------------------------
// H (ca x cb, ldh) = alpha A^T B + beta H
template <typename TB>
__device__ void pk_tn(Ctx &c, const double *A, int lda, int ca, const TB *B, int ldb, int cb, double *H, int ldh,
                      double alpha, double beta) {
    PK_TICK(c, PH_TN);
    wg_tn_mfma<TB, kPackUnr, false>(uni(c.D)->n, A, lda, ca, B, ldb, cb, 0, 1, H, ldh, alpha, beta, &g_sh.u.tn);
    sync();
}
// Hg ((ca + 8) x 8) = [A B]^T B for an 8-column B
__device__ void pk_tn_gram(Ctx &c, const double *A, int lda, int ca, const double *B, int ldb, double *Hg) {
    PK_TICK(c, PH_TN);
    wg_tn_mfma<double, kPackUnr, true>(uni(c.D)->n, A, lda, ca, B, ldb, kBlk, 0, 1, Hg, kBlk, 1.0, 0.0, &g_sh.u.tn);
    sync();
}
// C = beta C + alpha [A A2] H
__device__ void pk_nn2(Ctx &c, const double *A, int lda, int ca, const double *A2, int lda2, int ca2, const double *H,
                       int ldh, int cc, double *C, int ldc, double alpha, double beta) {
    PK_TICK(c, PH_NN);
    const int n = uni(c.D)->n;
    with_tile_loads(ca + ca2, [&](auto nl) {
        wg_nn_mfma<decltype(nl)::value, FlatTile>(n, A, lda, ca, A2, lda2, ca2, H, ldh, cc, C, ldc, alpha, beta, 0,
                                                  1, &g_sh.u.nn);
    });
    sync();
}
// Wt = [A A2] H (pass-0 update of a Lanczos block) and Hg = [A Wt]^T Wt (pass-1 reduction)
// in one sweep over the rows of A (wg_nn_tn_mfma)
__device__ void pk_nn_tn(Ctx &c, const double *A, int lda, int ca, const double *A2, int lda2, const double *H,
                         int ldh, double *Wt, int ldw, double *Hg) {
    PK_TICK(c, PH_NN);
    const int n = uni(c.D)->n;
    with_tile_loads(ca + kBlk, [&](auto nl) {
        wg_nn_tn_mfma<decltype(nl)::value, FlatTile>(n, A, lda, ca, A2, lda2, H, ldh, Wt, ldw, 0, 1, Hg, &g_sh.u.nt);
    });
    sync();
}
__device__ void pk_nn(Ctx &c, const double *A, int lda, int ca, const double *H, int ldh, int cc, double *C, int ldc,
                      double alpha, double beta) {
    pk_nn2(c, A, lda, ca, nullptr, 0, 0, H, ldh, cc, C, ldc, alpha, beta);
}

// Cholesky-QR factor of the n x nc block src: Rinv = R^{-1} of src^T src = R^T R with
// deflation flags (floor 1e-10 * *floor_ref when given)
__device__ void pk_cholqr_factor(Ctx &c, const double *src, int lds, int nc, int *flags, const double *floor_ref) {
    pk_tn<double>(c, src, lds, nc, src, lds, nc, g_sh.G16, 17, 1.0, 0.0);
    PK_TICK(c, PH_SMALL);
    double f2 = 0.0;
    if (floor_ref) {
        const double rf = 1e-10 * (*floor_ref);
        f2 = rf * rf;
    }
    if (threadIdx.x < 64) wave_cholqr(nc, g_sh.G16, 17, uni(c.D)->Rinv, nc, flags, f2);
    sync();
}
// Cholesky-QR twice of src (n x nc) into dst; deflated columns are zero and flagged
__device__ void pk_cholqr2(Ctx &c, const double *src, int lds, int nc, double *tmp, int ldt, double *dst, int ldd,
                           int *flags) {
    pk_cholqr_factor(c, src, lds, nc, flags, uni(c.D)->sc + SC_SCALE);
    pk_nn(c, src, lds, nc, uni(c.D)->Rinv, nc, nc, tmp, ldt, 1.0, 0.0);
    pk_cholqr_factor(c, tmp, ldt, nc, flags, nullptr);
    pk_nn(c, tmp, ldt, nc, uni(c.D)->Rinv, nc, nc, dst, ldd, 1.0, 0.0);
}

// top eigenpairs of the symmetric N x N matrix A (upper triangle read)
__device__ void pk_small_eig(Ctx &c, int N, const double *A, int lda, double *w, double *Y, int ldy, int ny,
                             const int *dead) {
    PK_TICK(c, PH_RITZ);
    N = uni(N), lda = uni(lda), ldy = uni(ldy), ny = uni(ny);
    A = uni(A), w = uni(w), Y = uni(Y), dead = uni(dead);
    wg_syev_load(N, A, lda, dead, &g_sh.u.syev);
    const int nv = N < kSyevMaxV ? N : kSyevMaxV;
    wg_syev_top(N, nv, ny < nv ? ny : nv, &g_sh.u.syev, w, Y, ldy);
    sync();
}

// ---------------------------------------------------------------------------
// block Lanczos with Rayleigh-Ritz restarts (same steps as the per-instance
// eigen-solver): start block of 16 vectors, block width 8, 'steps' blocks per
// cycle, two passes of block Gram-Schmidt with Pythagorean inner products per
// block, Cholesky-QR2 for each new block; Uritz / theta hold the result.
// Returns the number of restart cycles; c.last_conv tells whether the test passed.
// ---------------------------------------------------------------------------
__device__ int pk_lanczos(Ctx &c, const double *start, int kc, double tol, double tol_rest, int maxr, bool orth_start,
                          int min_cyc) {
    const PackDesc &D = *uni(c.D);
    const int n = D.n, ldb = D.ldb, steps = D.steps;
    if (start != D.Ubuf) pk_copy_cols(n, start, 16, 16, D.Ubuf, 16);
    if (D.n_iso > 0) {
        for (long e = threadIdx.x; e < (long)D.n_iso * 16; e += kWG)
            D.Ubuf[(size_t)D.iso_idx[e >> 4] * 16 + (e & 15)] = 0.0;
        sync();
        orth_start = true;
        if (D.n_iso == n) {   // a diagonal operator: every eigenpair is exact
            wg_iso_merge(D.n_iso, D.iso_idx, D.dshift, 0, D.theta, D.res, D.plan, &g_sh.u.iso);
            sync();
            for (long e = threadIdx.x; e < (long)n * kRitz; e += kWG) {
                const int i = (int)(e / kRitz), q = (int)(e - (long)i * kRitz);
                const int p = D.plan[q];
                double v = 0.0;
                if (p >= 0 && p < kRitz) v = D.Ucpl[(size_t)i * kRitz + p];
                else if (p < 0) v = (i == -p - 1) ? 1.0 : 0.0;
                D.Uritz[e] = v;
            }
            sync();
            c.last_conv = true;
            return 0;
        }
    }
    if (orth_start) {
        pk_set_int(D.flag, 16, 0);
        pk_cholqr2(c, D.Ubuf, 16, 16, D.W2, 16, D.Ubuf, 16, D.flag);
    }
    int cyc = 0;
    for (cyc = 0; cyc <= maxr; ++cyc) {
        // explicit Rayleigh-Ritz on span(U) and residuals
        pk_apply_op(c, D.Ubuf, 16, D.W2, 16, 16);
        pk_tn<double>(c, D.Ubuf, 16, 16, D.W2, 16, 16, D.TUU, 16, 1.0, 0.0);
        if (cyc == 0 || tol < 1e-7) {
            pk_small_eig(c, 16, D.TUU, 16, D.theta, D.Ysm, 16, 16, (cyc == 0 && orth_start) ? D.flag : nullptr);
        } else {   // U holds the previous cycle's Ritz vectors: the projection is diagonal
            for (int e = threadIdx.x; e < 16 * 16; e += kWG) D.Ysm[e] = (e / 16 == e % 16) ? 1.0 : 0.0;
            if (threadIdx.x < 16) D.theta[threadIdx.x] = D.TUU[threadIdx.x * 17];
            sync();
        }
        pk_nn(c, D.Ubuf, 16, 16, D.Ysm, 16, 16, D.Bm, ldb, 1.0, 0.0);
        pk_nn(c, D.W2, 16, 16, D.Ysm, 16, 16, D.Ubuf, 16, 1.0, 0.0);
        for (int e = threadIdx.x; e < 16 * 16; e += kWG) D.Hd[e] = (e / 16 == e % 16) ? -D.theta[e / 16] : 0.0;
        sync();
        pk_nn(c, D.Bm, ldb, 16, D.Hd, 16, 16, D.Ubuf, 16, 1.0, 1.0);
        pk_tn<double>(c, D.Ubuf, 16, 16, D.Ubuf, 16, 16, D.RtR, 16, 1.0, 0.0);
        {
            PK_TICK(c, PH_SMALL);
            wg_restart_prep(D.RtR, D.theta, kc, tol, tol_rest, D.res, D.flag, D.Zc, D.sc + SC_SCALE, &g_sh.u.rp);
            sync();
        }
        const int conv = D.flag[0];
        sync();   // every thread has read the flag before it is reused
        c.last_conv = conv != 0;
        if ((conv && cyc >= min_cyc) || cyc == maxr) break;
        // Krylov expansion from the dominant residual directions
        for (int e = threadIdx.x; e < ldb * ldb; e += kWG) {
            const int a = e / ldb, q = e - a * ldb;
            D.Tm[e] = (a == q && a < kRitz) ? D.theta[a] : 0.0;
        }
        for (int e = threadIdx.x; e < ldb; e += kWG) D.dead[e] = 0;
        sync();
        pk_nn(c, D.Ubuf, 16, 16, D.Zc, 8, 8, D.W, 8, 1.0, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
            pk_tn<double>(c, D.Bm, ldb, 16, D.W, 8, 8, D.Hred, 8, 1.0, 0.0);
            pk_nn(c, D.Bm, ldb, 16, D.Hred, 8, 8, D.W, 8, -1.0, 1.0);
        }
        pk_cholqr2(c, D.W, 8, 8, D.Wt, 8, D.Bm + 16, ldb, D.dead + 16);
        for (int j = 0; j < steps; ++j) {
            const int c0 = 16 + 8 * j, cols = c0 + 8;
            const bool last = j == steps - 1;
            pk_apply_op(c, D.Bm + c0, ldb, D.W, 8, 8);
            for (int pass = 0; pass < 2; ++pass) {
                if (pass == 0) pk_tn_gram(c, D.Bm, ldb, cols, D.W, 8, D.Hg);
                else pk_nn_tn(c, D.Bm, ldb, cols, D.W, 8, D.coef, 8, D.Wt, 8, D.Hg);   // update of pass 0 too
                {
                    PK_TICK(c, PH_SMALL);
                    wg_pip_chol(D.Hg, cols, pass, D.Rsv, D.Tm + c0, ldb, D.coef,
                                (pass == 1 && !last) ? D.dead + cols : nullptr, pass == 0 ? D.sc + SC_SCALE : nullptr,
                                &g_sh.u.pip);
                    sync();
                }
                if (pass == 1 && !last) pk_nn2(c, D.Bm, ldb, cols, D.Wt, 8, 8, D.coef, 8, 8, D.Bm + cols, ldb, 1.0, 0.0);
            }
        }
        pk_small_eig(c, ldb, D.Tm, ldb, D.theta, D.Ysm, 16, 16, D.dead);
        pk_nn(c, D.Bm, ldb, ldb, D.Ysm, 16, 16, D.Ubuf, 16, 1.0, 0.0);
    }
    pk_copy_cols(n, D.Bm, ldb, 16, D.Ucpl, 16);
    if (D.n_iso > 0) {
        wg_iso_merge(D.n_iso, D.iso_idx, D.dshift, 1, D.theta, D.res, D.plan, &g_sh.u.iso);
        sync();
        for (long e = threadIdx.x; e < (long)n * kRitz; e += kWG) {
            const int i = (int)(e / kRitz), q = (int)(e - (long)i * kRitz);
            const int p = D.plan[q];
            double v = 0.0;
            if (p >= 0 && p < kRitz) v = D.Ucpl[(size_t)i * kRitz + p];
            else if (p < 0) v = (i == -p - 1) ? 1.0 : 0.0;
            D.Uritz[e] = v;
        }
        sync();
    }
    return cyc;
}

// ---------------------------------------------------------------------------
// constraint-side steps
// ---------------------------------------------------------------------------
// out[j] = sum_i a_j[i] b_j[i] (np <= 3), fixed-order workgroup reduction
__device__ void pk_dots(Ctx &c, int m, const double *a0, const double *b0, const double *a1, const double *b1,
                        const double *a2, const double *b2, int np, double *out) {
    PK_TICK(c, PH_CONSTR);
    m = uni(m), np = uni(np);
    a0 = uni(a0), b0 = uni(b0), a1 = uni(a1), b1 = uni(b1), a2 = uni(a2), b2 = uni(b2), out = uni(out);
    double acc[3] = {0.0, 0.0, 0.0};
    const double *as[3] = {a0, a1, a2}, *bs[3] = {b0, b1, b2};
    for (int i = threadIdx.x; i < m; i += kWG)
        for (int j = 0; j < np; ++j) acc[j] += as[j][i] * bs[j][i];
    double(*red)[kWG] = g_sh.u.red;
    for (int j = 0; j < np; ++j) red[j][threadIdx.x] = acc[j];
    sync();
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st)
            for (int j = 0; j < np; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + st];
        sync();
    }
    if (threadIdx.x < np) out[threadIdx.x] = red[threadIdx.x][0];
    sync();
}
__device__ void pk_qp_gram(Ctx &c, const double *V, const double *w0, const double *w1, const double *w2, int nw,
                           double *out, int do_q11) {
    PK_TICK(c, PH_CONSTR);
    const PackDesc &D = *uni(c.D);
    wg_qp_gram(D.m, D.kptr, D.ti, D.tj, D.tv, V, 16, D.k, do_q11, w0, w1, w2, nullptr, nw, 0, 1, out, &g_sh.u.qg);
    sync();
}
// z = beta z + gamma zb + alpha A(V K V^T) (K k x k, gamma from the device scalar when given)
__device__ void pk_lowrank_A(Ctx &c, const double *V, int kd, const double *K, double alpha, const double *zb,
                             const double *gamma_dev, double *z) {
    PK_TICK(c, PH_CONSTR);
    const PackDesc &D = *uni(c.D);
    double *sK = g_sh.sK;
    for (int e = threadIdx.x; e < 256; e += kWG) {
        const int a = e >> 4, b = e & 15;
        sK[e] = (a < kd && b < kd) ? K[a * kd + b] : 0.0;
    }
    sync();
    const double gam = gamma_dev ? *gamma_dev : 0.0;
    for (long k = threadIdx.x; k < D.m; k += kWG) {
        const double acc = lowrank_row(k, D.kptr, D.ti, D.tj, D.tv, V, 16, kd, sK);
        double v = alpha * acc;
        if (zb) v += gam * zb[k];
        z[k] = v;
    }
    sync();
}

// accurate f(y_t): tight eigen-solve on C_s - A^* y_t from the current Ritz vectors;
// f and the relative errors are recomputed from it (keep_max: the larger of the two
// lower bounds of the same f(y_t))
__device__ void pk_polish(Ctx &c, int keep_max) {
    const PackDesc &D = *uni(c.D);
    pk_shift_operator(c, D.y);
    pk_copy_cols(D.n, D.Ucpl, 16, 12, D.Ubuf, 16);
    pk_random_block(D.n, 4, D.seed + 1000003ull * (uint64_t)(c.st.iters + 1), D.W, 8);
    pk_copy_cols(D.n, D.W, 8, 4, D.Ubuf + 12, 16);
    pk_lanczos(c, D.Ubuf, 1, D.tol_final, D.tol_final, 30, true, kCertifyMinCycles);
    pk_dots(c, D.m, D.b, D.y, nullptr, nullptr, nullptr, nullptr, 1, D.sc + SC_BYT);
    if (threadIdx.x == 0) refresh_f_scalar(D.theta, D.sc, keep_max);
    sync();
}

// cold start: y0 = 0, V0 = top-k eigenvectors of C_s (tight tolerance), f(y0)
__device__ void pk_cold_start(Ctx &c) {
    const PackDesc &D = *uni(c.D);
    pk_fill(D.y, D.m, 0.0);
    pk_fill(D.zbar, D.m, 0.0);
    if (D.sketch) pk_fill(D.P, (long)D.n * D.r, 0.0);
    pk_random_block(D.n, 16, D.seed, D.Ubuf, 16);
    pk_shift_operator(c, D.y);
    pk_lanczos(c, D.Ubuf, D.k, D.tol_final, sqrt(D.tol_final), D.max_restarts > 30 ? D.max_restarts : 30, true,
               kCertifyMinCycles);
    pk_fill(c.V, (long)D.n * 16, 0.0);
    pk_copy_cols(D.n, D.Uritz, 16, D.k, c.V, 16);
    if (threadIdx.x == 0) D.sc[SC_F] = D.alpha * fmax(D.theta[0], 0.0);
    sync();
}

// f(y0) of a warm-started instance (its padded state is in place)
__device__ void pk_warm_f(Ctx &c) {
    const PackDesc &D = *uni(c.D);
    pk_shift_operator(c, D.y);
    pk_lanczos(c, D.Uritz, D.k, D.tol_final, sqrt(D.tol_final), D.max_restarts > 30 ? D.max_restarts : 30, false,
               kCertifyMinCycles);
    pk_dots(c, D.m, D.b, D.y, nullptr, nullptr, nullptr, nullptr, 1, D.sc + SC_BYT);
    if (threadIdx.x == 0) refresh_f_scalar(D.theta, D.sc, 0);
    sync();
}

constexpr int kStallWindow = 25;   // consecutive null steps before f at the centre is re-evaluated

// one iteration of Alg. 1 (same steps as the per-instance driver)
__device__ void pk_iterate(Ctx &c) {
    const PackDesc &D = *uni(c.D);
    const int n = D.n, m = D.m, k = D.k, kc = D.kc, kp = D.kp, r = D.r;
    const int d = k * (k + 1) / 2;
    double *sc = D.sc;
    // V^T C V
    pk_apply_C(c, c.V, 16, D.CV, 16, 16);
    pk_tn<double>(c, c.V, 16, k, D.CV, 16, k, D.VCV, k, 1.0, 0.0);
    // reductions of the master QP: sum g g^T, G^T zbar, G^T y, G^T b
    pk_qp_gram(c, c.V, D.zbar, D.y, D.b, 3, D.raw, 1);
    pk_dots(c, m, D.zbar, D.zbar, D.y, D.zbar, D.b, D.zbar, 3, sc + SC_ZZ);
    // alternating maximisation over (X, nu) (eqs. small_quad_sdp, dual_slack_update)
    pk_fill(D.nu, m, 0.0);
    IpmArgs ia{k, 1e-7, 1e-7, 100, 0};
    for (int pass = 0; pass < 50; ++pass) {
        if (pass > 0) {
            pk_qp_gram(c, c.V, D.nu, nullptr, nullptr, 1, D.Gy, 0);
            for (int p = threadIdx.x; p < d; p += kWG) D.raw[d * (d + 1) / 2 + 3 * d + p] = D.Gy[p];
            sync();
            pk_dots(c, m, D.nu, D.zbar, nullptr, nullptr, nullptr, nullptr, 1, sc + SC_NUZ);
        }
        wg_qp_finalize(k, D.raw, D.VCV, sc, pass > 0, D.qp);
        sync();
        ia.warm = pass > 0;
        {
            PK_TICK(c, PH_IPM);
            wg_ipm(ia, D.qp, D.ipm, &g_sh.u.ipm);
            sync();
        }
        if (threadIdx.x == 0) post_ipm_scalar(k, D.ipm, D.VCV, sc);
        sync();
        // A X_{t+1} = g zbar + alpha A(V S V^T)
        pk_lowrank_A(c, c.V, k, D.ipm, D.alpha, D.zbar, sc + SC_G, D.AX);
        if (!D.has_ineq) break;
        for (long q = threadIdx.x; q < m; q += kWG) nu_update_elem(q, D.b, D.AX, D.y, D.ineq, D.rho, D.nu, D.dnu);
        sync();
        pk_dots(c, m, D.dnu, D.dnu, nullptr, nullptr, nullptr, nullptr, 1, sc + SC_DNU);
        const double dn = sc[SC_DNU];
        sync();
        if (sqrt(dn) <= 1e-9) break;
    }
    // candidate (eq. dual_update) and primal infeasibility of X_{t+1}
    for (long q = threadIdx.x; q < m; q += kWG) candidate_elem(q, D.b, D.AX, D.y, D.ineq, D.rho, D.yc, D.evec);
    sync();
    pk_dots(c, m, D.b, D.yc, D.yc, D.zbar, D.evec, D.evec, 3, sc + SC_BY);   // SC_BY, SC_YZ, SC_DIST2
    pk_qp_gram(c, c.V, D.yc, nullptr, nullptr, 1, D.Gy, 0);
    {
        PK_TICK(c, PH_SMALL);
        wg_fhat_prep(k, D.VCV, D.Gy, sc, &g_sh.u.fh);
        sync();
    }
    // eigen step at the candidate: the previous Ritz block with its last two columns
    // replaced by fresh random directions
    pk_shift_operator(c, D.yc);
    pk_copy_cols(n, D.Ucpl, 16, 14, D.Ubuf, 16);
    pk_random_block(n, 2, D.seed + 7919ull * (uint64_t)(c.st.iters + 1), D.W, 8);
    pk_copy_cols(n, D.W, 8, 2, D.Ubuf + 14, 16);
    const int cyc = pk_lanczos(c, D.Ubuf, kc, D.tol, D.tol_rest, D.max_restarts, true, 0);
    if (cyc >= D.max_restarts && !c.last_conv) c.st.lz_unconverged++;
    if (threadIdx.x == 0) decide_scalar(D.theta, sc);
    sync();
    if (sc[SC_DESC] != 0.0)
        for (long q = threadIdx.x; q < m; q += kWG) D.y[q] = D.yc[q];
    sync();
    // model update
    if (D.sketch) pk_tn<float>(c, c.V, 16, k, D.psi, r, r, D.VtPsi, r, 1.0, 0.0);
    {
        PK_TICK(c, PH_SMALL);
        wg_model_update(k, kp, r, D.ipm, D.VCV, D.VtPsi, sc, D.Kc, D.Qp, D.sketch ? D.Hsk : nullptr, &g_sh.u.mu);
        sync();
    }
    pk_lowrank_A(c, c.V, k, D.Kc, 1.0, D.zbar, sc + SC_G, D.zbar);
    if (D.sketch) {   // P <- g P + V (Kc V^T Psi)
        const double g = sc[SC_G];
        for (long e = threadIdx.x; e < (long)n * r; e += kWG) D.P[e] *= g;
        sync();
        pk_nn(c, c.V, 16, k, D.Hsk, r, r, D.P, r, 1.0, 1.0);
    }
    // V_{t+1} = orth([V Q_p, v_1..v_kc]) (eq. v_next_def)
    pk_copy_cols(n, D.Uritz, 16, kc, c.Vn, 16);
    if (kp > 0) {
        pk_nn(c, c.V, 16, k, D.Qp, kp, kp, D.Zp, 16, 1.0, 0.0);
        for (int pass = 0; pass < 2; ++pass) {
            pk_tn<double>(c, D.Uritz, 16, kc, D.Zp, 16, kp, D.hz, kp, 1.0, 0.0);
            pk_nn(c, D.Uritz, 16, kc, D.hz, kp, kp, D.Zp, 16, -1.0, 1.0);
        }
        pk_set_int(D.zdead, 16, 0);
        pk_cholqr2(c, D.Zp, 16, kp, D.W2, 16, c.Vn + kc, 16, D.zdead);
        for (long e = threadIdx.x; e < (long)n * kp; e += kWG) {
            const long i = e / kp;
            const int j = (int)(e - i * kp);
            if (D.zdead[j]) c.Vn[i * 16 + kc + j] = D.Uritz[i * 16 + kc + j];
        }
        sync();
    }
    double *t = c.V;
    c.V = c.Vn;
    c.Vn = t;
    c.st.swapped ^= 1;
    c.st.iters++;
    c.st.solve_iters++;
    const bool desc = sc[SC_DESC] != 0.0;
    sync();
    c.st.null_run = desc ? 0 : c.st.null_run + 1;
    if (c.st.null_run >= kStallWindow) {
        pk_polish(c, 1);
        c.st.null_run = 0;
        c.st.recoveries++;
    }
}

__global__ __launch_bounds__(kWG) void k_packed(const PackDesc *__restrict__ descs, PackState *states, int iters) {
    const PackDesc *D = descs + blockIdx.x;
    Ctx c;
    c.D = D;
    c.st = states[blockIdx.x];
    c.V = D->V;
    c.Vn = D->Vn;
    c.last_conv = false;
    c.st.swapped = 0;
    const unsigned long long t_start = wall_clock64();
    if (c.st.init == PACK_INIT_COLD) pk_cold_start(c);
    else if (c.st.init == PACK_INIT_WARM) pk_warm_f(c);
    c.st.init = PACK_INIT_NONE;
    for (int t = 0; t < iters && c.st.done == PACK_RUNNING; ++t) {
        if (c.st.stop || c.st.solve_iters >= D->max_iters) {
            // stopped by a limit: certify f(y_T) with the tight eigen-solve
            pk_polish(c, 1);
            c.st.done = PACK_LIMIT;
            break;
        }
        pk_iterate(c);
        const double *sc = D->sc;
        const double f = sc[SC_F], cx = sc[SC_CX], ipst = sc[SC_IPMSTATUS];
        const double gap = sc[SC_GAP], inf = sc[SC_INF];
        sync();
        if (!isfinite(f) || !isfinite(cx) || ipst == 2.0) {
            c.st.done = PACK_FAILED;
            break;
        }
        if (gap <= D->eps_gap && inf <= D->eps_inf) {
            // certify: recompute lambda_max(C - A^* y_T) with a tight residual tolerance
            pk_polish(c, 1);
            const double gap2 = sc[SC_GAP], inf2 = sc[SC_INF];
            sync();
            if (gap2 <= D->eps_gap && inf2 <= D->eps_inf) c.st.done = PACK_CONVERGED;
        }
    }
    c.st.ticks[PH_ALL] += wall_clock64() - t_start;
    if (threadIdx.x == 0) states[blockIdx.x] = c.st;
}

}  // namespace

size_t packed_lds_bytes() { return sizeof(PackShared); }

void packed_launch(hipStream_t s, const PackDesc *desc_dev, PackState *state_dev, int count, int iters) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_packed, dim3(count), dim3(kWG), 0, s, desc_dev, state_dev, iters);
}

}  // namespace usbs
