// gfx950 kernels of the USBS hot path: sparse shifted operator, tall-skinny
// dense products for block Lanczos / sketch / low-rank constraint
// evaluation, and one-workgroup solvers for the small dense problems
// (Ritz eigenproblems, Cholesky-QR factors, the master-QP interior point method).
//
// Layout conventions: every n x c block is row-major (row i = c contiguous
// values), so a gathered row of an 8-column block is one 64-byte segment and
// a column slice of the Lanczos basis is addressed by (pointer + offset, ld).
#include "kernels.h"
#include "small_dense.h"
#include "syev.h"
#include "wg_steps.h"

#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

namespace usbs {

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// ---------------------------------------------------------------------------
// Second stage of every grid-wide reduction.  Stage-1 kernels write one partial
// per workgroup (part[b * nout + o]) and exit; no workgroup waits for another,
// so no device-scope fence (an L2 write-back/invalidate on this GPU) is issued
// per workgroup.  This kernel sums the G partials of each output in block order
// (deterministic): 4 waves split the partials, LDS combines them in fixed order.
//   out[(o / cb) * ldo + (o % cb)] = alpha * sum_b part[b][o] (+ beta * old)
// ---------------------------------------------------------------------------
// 16 outputs per workgroup: lane o % 16 of each 16-lane group, the G partials split over the
// sixteen groups (sixteen independent loads in flight per lane), then the group sums added in
// a fixed order (deterministic)
__device__ __forceinline__ double finish16(const double *__restrict__ part, int G, int nout, int o,
                                           double (*s16)[16]) {
    const int l16 = threadIdx.x & 15, sl = threadIdx.x >> 4;
    const int per = (G + 15) / 16;
    const int b0 = sl * per, b1 = min(G, b0 + per);
    double sum = 0.0;
    if (o < nout) {
        for (int bb = b0; bb < b1; bb += 16) {
            double v[16];
#pragma unroll
            for (int q = 0; q < 16; ++q) v[q] = (bb + q < b1) ? part[(size_t)(bb + q) * nout + o] : 0.0;
#pragma unroll
            for (int q = 0; q < 16; ++q) sum += v[q];
        }
    }
    s16[sl][l16] = sum;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x < 16)
#pragma unroll
        for (int q = 0; q < 16; ++q) t += s16[q][threadIdx.x];
    return t;   // meaningful in threads 0..15
}
__global__ __launch_bounds__(kWG) void k_red_finish(const double *__restrict__ part, int G, int nout,
                                                    double *out, int cb, int ldo, double alpha, double beta) {
    __shared__ double s16[16][16];
    const int o = blockIdx.x * 16 + (threadIdx.x & 15);
    const double t = alpha * finish16(part, G, nout, o, s16);
    if (threadIdx.x < 16 && o < nout) {
        const int r = o / cb, c = o - r * cb;
        double *dst = out + (size_t)r * ldo + c;
        *dst = (beta != 0.0) ? t + beta * (*dst) : t;
    }
}

static void red_finish(hipStream_t s, const double *part, int G, int nout, double *out, int cb, int ldo,
                       double alpha, double beta) {
    hipLaunchKernelGGL(k_red_finish, dim3(cdiv(nout, 16)), dim3(kWG), 0, s, part, G, nout, out, cb, ldo, alpha,
                       beta);
}

// Cholesky-QR factor from the partial Gram matrices (one workgroup): G = sum of the
// partials (nc x nc), then R^{-1} (upper) with deflation flags, see wave_cholqr.
__global__ __launch_bounds__(kWG) void k_cholqr_finish(const double *__restrict__ part, int G, int nc,
                                                       double *H, int ldh, int *flags, const double *floor_ref) {
    __shared__ double sR[16 * 17];
    __shared__ double sp[kWG];
    const int tid = threadIdx.x;
    const int nout = nc * nc;
    // thread (sl, o) sums partials sl, sl + S, ... of output o; sixteen loads in flight
    // per thread, then the S slices are added in a fixed order (deterministic)
    const int S = nout >= kWG ? 1 : kWG / nout;
    for (int o0 = 0; o0 < nout; o0 += kWG / S) {
        const int o = o0 + tid % (kWG / S), sl = tid / (kWG / S);
        double acc = 0.0;
        if (o < nout && sl < S) {
            for (int b0 = sl; b0 < G; b0 += 16 * S) {
                double v[16];
#pragma unroll
                for (int q = 0; q < 16; ++q) {
                    const int b = b0 + q * S;
                    v[q] = (b < G) ? part[(size_t)b * nout + o] : 0.0;
                }
#pragma unroll
                for (int q = 0; q < 16; ++q) acc += v[q];
            }
        }
        sp[tid] = acc;
        __syncthreads();
        if (tid < kWG / S) {
            const int oo = o0 + tid;
            if (oo < nout) {
                double t = 0.0;
                for (int q = 0; q < S; ++q) t += sp[q * (kWG / S) + tid];
                const int a = oo / nc, c = oo - a * nc;
                sR[a * 17 + c] = t;
            }
        }
        __syncthreads();
    }
    __syncthreads();
    double f2 = 0.0;
    if (floor_ref) {
        const double rf = 1e-10 * (*floor_ref);
        f2 = rf * rf;
    }
    if (tid < 64) wave_cholqr(nc, sR, 17, H, ldh, flags, f2);
}

// ---------------------------------------------------------------------------
// SpMM with the shifted diagonal: L lanes per row, lane c owns column c.
// The column index / value of a nonzero is read once per row group and
// broadcast; the gathered X row segment is contiguous.
// ---------------------------------------------------------------------------
template <typename VT, typename ACC, int L>
__global__ __launch_bounds__(kWG) void k_spmm(int n, const int *__restrict__ rowptr,
                                              const int *__restrict__ col,
                                              const VT *__restrict__ val, ACC scale,
                                              const double *__restrict__ diag,
                                              const double *__restrict__ X, int ldx,
                                              double *__restrict__ Y, int ldy, int nb) {
    const int i = blockIdx.x * (kWG / L) + threadIdx.x / L;
    const int c = threadIdx.x % L;
    if (i >= n) return;
    const bool act = c < nb;
    const double v = spmm_row<VT, ACC>(i, act ? c : 0, rowptr, col, val, scale, diag, X, ldx);
    if (act) Y[(size_t)i * ldy + c] = v;
}

// Variant with P consecutive columns per lane (one P-wide load per gathered row
// segment), L lanes per row.  Every (row, column) output accumulates the same products
// in the same order as k_spmm (even and odd nonzeros in two partial sums), so the
// variants give bitwise identical results and the choice is a pure launch-shape tuning.
template <typename VT, typename ACC, int L, int P>
__global__ __launch_bounds__(kWG) void k_spmm_p(int n, const int *__restrict__ rowptr,
                                                const int *__restrict__ col,
                                                const VT *__restrict__ val, ACC scale,
                                                const double *__restrict__ diag,
                                                const double *__restrict__ X, int ldx,
                                                double *__restrict__ Y, int ldy, int nb) {
    const int i = blockIdx.x * (kWG / L) + threadIdx.x / L;
    const int c0 = (threadIdx.x % L) * P;
    if (i >= n) return;
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    const int cc = (c0 + P <= nb) ? c0 : 0;   // lanes past nb read column block 0 and store nothing
    ACC acc0[P], acc1[P];
#pragma unroll
    for (int p = 0; p < P; ++p) acc0[p] = acc1[p] = 0;
    int e = e0;
    for (; e + 1 < e1; e += 2) {
        const int j0 = col[e], j1 = col[e + 1];
        ACC v0, v1;
        if constexpr (sizeof(VT) == 2) {
            v0 = (ACC)bf16_to_f32(val[e]);
            v1 = (ACC)bf16_to_f32(val[e + 1]);
        } else {
            v0 = (ACC)val[e];
            v1 = (ACC)val[e + 1];
        }
        const double *x0 = X + (size_t)j0 * ldx + cc;
        const double *x1 = X + (size_t)j1 * ldx + cc;
#pragma unroll
        for (int p = 0; p < P; ++p) {
            acc0[p] += v0 * (ACC)x0[p];
            acc1[p] += v1 * (ACC)x1[p];
        }
    }
    if (e < e1) {
        const int j0 = col[e];
        ACC v0;
        if constexpr (sizeof(VT) == 2) v0 = (ACC)bf16_to_f32(val[e]);
        else v0 = (ACC)val[e];
        const double *x0 = X + (size_t)j0 * ldx + cc;
#pragma unroll
        for (int p = 0; p < P; ++p) acc0[p] += v0 * (ACC)x0[p];
    }
    if (c0 + P <= nb) {
#pragma unroll
        for (int p = 0; p < P; ++p) {
            const double xi = X[(size_t)i * ldx + c0 + p];
            Y[(size_t)i * ldy + c0 + p] = diag[i] * xi + (double)(scale * (acc0[p] + acc1[p]));
        }
    }
}

// launch-shape choices of the tuned kernels (per handle; see usbs.hip for the tuner)
static thread_local const Tuning *g_tune = nullptr;
void set_tuning(const Tuning *t) { g_tune = t; }

template <typename VT, typename ACC>
static void spmm_t(hipStream_t s, int n, const int *rowptr, const int *col, const VT *val, ACC scale,
                   const double *diag, const double *X, int ldx, double *Y, int ldy, int nb) {
    if (n <= 0) return;
    // P columns per lane needs nb to be a multiple of P (every column owned by one lane)
    const int var = g_tune ? (nb <= 8 ? g_tune->spmm8 : g_tune->spmm16) : 0;
    if (var == 1 && nb % 2 == 0) {
        if (nb <= 8)
            hipLaunchKernelGGL((k_spmm_p<VT, ACC, 4, 2>), dim3(cdiv(n, kWG / 4)), dim3(kWG), 0, s, n, rowptr, col,
                               val, scale, diag, X, ldx, Y, ldy, nb);
        else
            hipLaunchKernelGGL((k_spmm_p<VT, ACC, 8, 2>), dim3(cdiv(n, kWG / 8)), dim3(kWG), 0, s, n, rowptr, col,
                               val, scale, diag, X, ldx, Y, ldy, nb);
        return;
    }
    if (var == 2 && nb % 4 == 0) {
        if (nb <= 8)
            hipLaunchKernelGGL((k_spmm_p<VT, ACC, 2, 4>), dim3(cdiv(n, kWG / 2)), dim3(kWG), 0, s, n, rowptr, col,
                               val, scale, diag, X, ldx, Y, ldy, nb);
        else
            hipLaunchKernelGGL((k_spmm_p<VT, ACC, 4, 4>), dim3(cdiv(n, kWG / 4)), dim3(kWG), 0, s, n, rowptr, col,
                               val, scale, diag, X, ldx, Y, ldy, nb);
        return;
    }
    if (nb <= 8) {
        hipLaunchKernelGGL((k_spmm<VT, ACC, 8>), dim3(cdiv(n, kWG / 8)), dim3(kWG), 0, s, n, rowptr, col,
                           val, scale, diag, X, ldx, Y, ldy, nb);
    } else {
        hipLaunchKernelGGL((k_spmm<VT, ACC, 16>), dim3(cdiv(n, kWG / 16)), dim3(kWG), 0, s, n, rowptr,
                           col, val, scale, diag, X, ldx, Y, ldy, nb);
    }
}

void spmm(hipStream_t s, int prec, int n, const int *rowptr, const int *col, const void *val,
          double scale, const double *diag, const double *X, int ldx, double *Y, int ldy, int nb) {
    if (prec == 0)
        spmm_t<double, double>(s, n, rowptr, col, (const double *)val, scale, diag, X, ldx, Y, ldy, nb);
    else if (prec == 1)
        spmm_t<float, float>(s, n, rowptr, col, (const float *)val, (float)scale, diag, X, ldx, Y, ldy, nb);
    else
        spmm_t<uint16_t, float>(s, n, rowptr, col, (const uint16_t *)val, (float)scale, diag, X, ldx, Y,
                                ldy, nb);
}

// ---------------------------------------------------------------------------
// shift of the operator by A^* y
// ---------------------------------------------------------------------------
__global__ void k_diag_shift(int n, const int *__restrict__ dptr, const int *__restrict__ dk,
                             const double *__restrict__ dv, const double *__restrict__ cdiag,
                             const double *__restrict__ y, double *__restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double v = cdiag[i];
    for (int e = dptr[i]; e < dptr[i + 1]; ++e) v -= dv[e] * y[dk[e]];
    d[i] = v;
}

// Gershgorin bound of the shifted operator: out = max_i (|d_i| + scale * sum_e |val_e|)
template <typename VT>
__global__ __launch_bounds__(kWG) void k_op_bound(int n, const int *__restrict__ rowptr,
                                                  const VT *__restrict__ val, double scale,
                                                  const double *__restrict__ d, double *__restrict__ part) {
    __shared__ double red[kWG];
    double mx = 0.0;
    for (long i = (long)blockIdx.x * kWG + threadIdx.x; i < n; i += (long)gridDim.x * kWG) {
        double s = 0.0;
        for (int e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if constexpr (sizeof(VT) == 2) s += fabs((double)bf16_to_f32(val[e]));
            else s += fabs((double)val[e]);
        }
        mx = fmax(mx, fabs(d[i]) + fabs(scale) * s);
    }
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}
__global__ void k_max_finish(const double *__restrict__ part, int G, double *out) {
    __shared__ double red[kWG];
    double mx = 0.0;
    for (int b = threadIdx.x; b < G; b += kWG) mx = fmax(mx, part[b]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (threadIdx.x < st) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + st]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0];
}
void op_bound(hipStream_t s, const RedScratch &rs, int prec, int n, const int *rowptr, const void *val, double scale,
              const double *d, double *out) {
    int blocks = cdiv(n, 4 * kWG);
    if (blocks > 256) blocks = 256;
    if (blocks < 1) blocks = 1;
    if (prec == 0)
        hipLaunchKernelGGL(k_op_bound<double>, dim3(blocks), dim3(kWG), 0, s, n, rowptr, (const double *)val, scale, d,
                           rs.partials);
    else if (prec == 1)
        hipLaunchKernelGGL(k_op_bound<float>, dim3(blocks), dim3(kWG), 0, s, n, rowptr, (const float *)val, scale, d,
                           rs.partials);
    else
        hipLaunchKernelGGL(k_op_bound<uint16_t>, dim3(blocks), dim3(kWG), 0, s, n, rowptr, (const uint16_t *)val,
                           scale, d, rs.partials);
    hipLaunchKernelGGL(k_max_finish, dim3(1), dim3(kWG), 0, s, rs.partials, blocks, out);
}

void diag_shift(hipStream_t s, int n, const int *dptr, const int *dk, const double *dv,
                const double *cdiag, const double *y, double *d) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_diag_shift, dim3(cdiv(n, kWG)), dim3(kWG), 0, s, n, dptr, dk, dv, cdiag, y, d);
}

template <typename VT>
__global__ void k_offdiag_refresh(int ns, const int *__restrict__ slot, const int *__restrict__ ptr,
                                  const int *__restrict__ kk, const double *__restrict__ hv,
                                  const double *__restrict__ cbase, const double *__restrict__ y, double inv_scale,
                                  VT *__restrict__ val) {
    const int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= ns) return;
    const int sl = slot[u];
    double v = cbase[sl];
    for (int t = ptr[u]; t < ptr[u + 1]; ++t) v -= hv[t] * y[kk[t]];
    v *= inv_scale;
    if constexpr (sizeof(VT) == 2) val[sl] = f32_to_bf16((float)v);
    else val[sl] = (VT)v;
}

void offdiag_refresh(hipStream_t s, int prec, int ns, const int *slot, const int *ptr, const int *k,
                     const double *hv, const double *cbase, const double *y, double inv_scale, void *val) {
    if (ns <= 0) return;
    dim3 g(cdiv(ns, kWG));
    if (prec == 0)
        hipLaunchKernelGGL(k_offdiag_refresh<double>, g, dim3(kWG), 0, s, ns, slot, ptr, k, hv, cbase, y,
                           inv_scale, (double *)val);
    else if (prec == 1)
        hipLaunchKernelGGL(k_offdiag_refresh<float>, g, dim3(kWG), 0, s, ns, slot, ptr, k, hv, cbase, y,
                           inv_scale, (float *)val);
    else
        hipLaunchKernelGGL(k_offdiag_refresh<uint16_t>, g, dim3(kWG), 0, s, ns, slot, ptr, k, hv, cbase, y,
                           inv_scale, (uint16_t *)val);
}

template <typename VT>
__global__ void k_convert(int nnz, const double *__restrict__ src, double inv_scale, VT *__restrict__ dst) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nnz) return;
    const double v = src[e] * inv_scale;
    if constexpr (sizeof(VT) == 2) dst[e] = f32_to_bf16((float)v);
    else dst[e] = (VT)v;
}

void convert_values(hipStream_t s, int prec, int nnz, const double *src, double inv_scale, void *dst) {
    if (nnz <= 0) return;
    dim3 g(cdiv(nnz, kWG));
    if (prec == 0)
        hipLaunchKernelGGL(k_convert<double>, g, dim3(kWG), 0, s, nnz, src, inv_scale, (double *)dst);
    else if (prec == 1)
        hipLaunchKernelGGL(k_convert<float>, g, dim3(kWG), 0, s, nnz, src, inv_scale, (float *)dst);
    else
        hipLaunchKernelGGL(k_convert<uint16_t>, g, dim3(kWG), 0, s, nnz, src, inv_scale, (uint16_t *)dst);
}

// ---------------------------------------------------------------------------
// H = beta*H + alpha*A^T B : two-stage deterministic reduction over rows.
// Stage 1: each workgroup streams 32-row tiles of A and B through LDS and
// accumulates its share of the (ca x cb) outputs in registers.
// Stage 2: the last workgroup to finish sums the partials in block order.
// ---------------------------------------------------------------------------
constexpr int kTile = 32;
constexpr int kMaxCB = 32;
constexpr int kMaxOut = kMaxBasis * 16;          // 1280 outputs (also >= 32 x 32)
constexpr int kOutPerThread = (kMaxOut + kWG - 1) / kWG;

// TAG only names the instantiation: 1 = the Krylov re-orthogonalisation (its own
// symbol, so that profilers report those launches separately).  GRAM: the outputs are
// [A B]^T B ((ca + cb) x cb), i.e. A^T B followed by the Gram matrix B^T B.
template <typename TB, int TAG, bool GRAM>
__global__ __launch_bounds__(kWG) void k_tn_reduce(int n, const double *__restrict__ A, int lda, int ca,
                                                   const TB *__restrict__ B, int ldb, int cb,
                                                   double *__restrict__ partials) {
    __shared__ double sA[kTile][kMaxBasis + kBlk + 1];
    __shared__ double sB[kTile][kMaxCB + 1];
    const int tid = threadIdx.x;
    const int rows_out = GRAM ? ca + cb : ca;
    const int nout = rows_out * cb;
    double acc[kOutPerThread];
#pragma unroll
    for (int q = 0; q < kOutPerThread; ++q) acc[q] = 0.0;

    for (long row0 = (long)blockIdx.x * kTile; row0 < n; row0 += (long)gridDim.x * kTile) {
        for (int e = tid; e < kTile * ca; e += kWG) {
            const int r = e / ca, a = e - r * ca;
            const long i = row0 + r;
            sA[r][a] = (i < n) ? A[i * lda + a] : 0.0;
        }
        for (int e = tid; e < kTile * cb; e += kWG) {
            const int r = e / cb, c = e - r * cb;
            const long i = row0 + r;
            const double v = (i < n) ? (double)B[i * ldb + c] : 0.0;
            sB[r][c] = v;
            if (GRAM) sA[r][ca + c] = v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kOutPerThread; ++q) {
            const int o = tid + q * kWG;
            if (o < nout) {
                const int a = o / cb, c = o - a * cb;
                double s = 0.0;
#pragma unroll 8
                for (int r = 0; r < kTile; ++r) s += sA[r][a] * sB[r][c];
                acc[q] += s;
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < kOutPerThread; ++q) {
        const int o = tid + q * kWG;
        if (o < nout) partials[(size_t)blockIdx.x * nout + o] = acc[q];
    }
}

static int tn_blocks(const RedScratch &rs, int n) {
    int blocks = cdiv(n, 4 * kTile);
    if (blocks > rs.max_blocks) blocks = rs.max_blocks;
    if (blocks < 1) blocks = 1;
    return blocks;
}

// ---------------------------------------------------------------------------
// [A B]^T B for an 8-column B (the Krylov re-orthogonalisation) on the FP64 matrix
// cores: V_MFMA_F64_16X16X4F64 accumulates X (16 x 4) Y (4 x 16) with X[m][k] in lane
// m + 16 k, Y[k][j] in lane j + 16 k, and D[m][j] in lane j + 16 (m % 4), element m / 4.
// A wavefront takes 4 rows at a time: X = 16 columns of A of those rows (one double
// per lane, 128 contiguous bytes per row), Y = the 8 columns of B (lanes j >= 8 hold 0),
// so every element of A is loaded once and no lane replicates another's data.  The
// Gram block B^T B uses Y as X.  UNR row groups are in flight per wavefront; the four
// wavefronts of a workgroup are summed in LDS in a fixed order into one partial per
// workgroup (layout as k_tn_reduce: (ca + 8) x 8).
// ---------------------------------------------------------------------------
template <int TAG, int UNR, bool GRAM>
__global__ __launch_bounds__(kWG) void k_tn_mfma(int n, const double *__restrict__ A, int lda, int ca,
                                                 const double *__restrict__ B, int ldb, int cb,
                                                 double *__restrict__ partials) {
    __shared__ TnWork w;
    const int rows_out = GRAM ? ca + cb : ca;
    wg_tn_mfma<double, UNR, GRAM>(n, A, lda, ca, B, ldb, cb, blockIdx.x, gridDim.x,
                                  partials + (size_t)blockIdx.x * rows_out * cb, cb, 1.0, 0.0, &w);
}

static int mfma_blocks(const RedScratch &rs, int n) {
    int blocks = cdiv(n, 64);   // at least 16 rows per wavefront
    if (g_tune && g_tune->red_cap > 0 && blocks > g_tune->red_cap) blocks = g_tune->red_cap;
    if (blocks > rs.max_blocks) blocks = rs.max_blocks;
    if (blocks < 1) blocks = 1;
    return blocks;
}

int reorth_partials(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca, const double *B,
                    int ldb, int cb, hipEvent_t ev_start, hipEvent_t ev_stop) {
    (void)cb;   // always 8 (one Lanczos block)
    const int blocks = mfma_blocks(rs, n);
    const bool u2 = g_tune && g_tune->red_unr == 2;
    if (ev_start && ev_stop) {   // events carry this dispatch's own start / end time
        if (u2)
            hipExtLaunchKernelGGL((k_tn_mfma<1, 2, true>), dim3(blocks), dim3(kWG), 0, s, ev_start, ev_stop, 0, n, A,
                                  lda, ca, B, ldb, kBlk, rs.partials);
        else
            hipExtLaunchKernelGGL((k_tn_mfma<1, 4, true>), dim3(blocks), dim3(kWG), 0, s, ev_start, ev_stop, 0, n, A,
                                  lda, ca, B, ldb, kBlk, rs.partials);
    } else if (u2) {
        hipLaunchKernelGGL((k_tn_mfma<1, 2, true>), dim3(blocks), dim3(kWG), 0, s, n, A, lda, ca, B, ldb, kBlk,
                           rs.partials);
    } else {
        hipLaunchKernelGGL((k_tn_mfma<1, 4, true>), dim3(blocks), dim3(kWG), 0, s, n, A, lda, ca, B, ldb, kBlk,
                           rs.partials);
    }
    return blocks;
}
void tn_reduce(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca, const double *B,
               int ldb, int cb, double *H, int ldh, double alpha, double beta, int post, int *flags,
               const double *floor_ref) {
    int blocks;
    if (cb <= 16 && ca <= kMaxBasis) {
        blocks = mfma_blocks(rs, n);
        hipLaunchKernelGGL((k_tn_mfma<0, 4, false>), dim3(blocks), dim3(kWG), 0, s, n, A, lda, ca, B, ldb, cb,
                           rs.partials);
    } else {
        blocks = tn_blocks(rs, n);
        hipLaunchKernelGGL((k_tn_reduce<double, 0, false>), dim3(blocks), dim3(kWG), 0, s, n, A, lda, ca, B, ldb, cb,
                           rs.partials);
    }
    if (post == 0) red_finish(s, rs.partials, blocks, ca * cb, H, cb, ldh, alpha, beta);
    else hipLaunchKernelGGL(k_cholqr_finish, dim3(1), dim3(kWG), 0, s, rs.partials, blocks, ca, H, ldh, flags, floor_ref);
}

void sum_partials(hipStream_t s, const double *part, int G, int nout, double *out) {
    red_finish(s, part, G, nout, out, nout, nout, 1.0, 0.0);
}

void reorth_finish(hipStream_t s, const RedScratch &rs, int blocks, int ca, int cb, double *H, int ldh) {
    red_finish(s, rs.partials, blocks, (ca + cb) * cb, H, cb, ldh, 1.0, 0.0);
}

// ---------------------------------------------------------------------------
// One pass of block Gram-Schmidt with Pythagorean inner products (one
// workgroup), from Hg = [Q W]^T W: rows 0..cols-1 hold H = Q^T W, rows
// cols..cols+7 hold G = W^T W.  With Q^T Q = I,
//   Omega = G - H^T H = (W - Q H)^T (W - Q H) = R^T R   (Cholesky, deflation)
//   coef  = [-H R^{-1}; R^{-1}]  so that  [Q W] coef = (W - Q H) R^{-1}.
// The projections of the block that entered the first pass are H1 + H2 R1
// (W0 = Q H1 + W1 R1, W1 = Q H2 + W2 R2): pass 0 stores H into T and keeps R;
// pass 1 adds H R_saved.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_pip_chol(const double *__restrict__ Hg, int cols, int pass,
                                                  double *__restrict__ Rsave, double *__restrict__ T, int ldt,
                                                  double *__restrict__ coef, int *flags,
                                                  const double *__restrict__ floor_ref) {
    __shared__ PipWork w;
    wg_pip_chol(Hg, cols, pass, Rsave, T, ldt, coef, flags, floor_ref, &w);
}
// k_red_finish's sums (alpha 1, beta 0, contiguous output) into Hg, then the pass's pip_chol on
// the last workgroup to finish.  Each workgroup's stores are released at device scope before
// it counts itself in; the last one acquires them before reading Hg and resets the counter
// for the next launch on the stream.  No workgroup waits for another.
__global__ __launch_bounds__(kWG) void k_finish_pip(const double *__restrict__ part, int G, int cols, double *Hg,
                                                    unsigned *counter, int pass, double *Rsave, double *T, int ldt,
                                                    double *coef, int *flags, const double *floor_ref, int *skip) {
    __shared__ PipWork w;
    __shared__ double s16[16][16];
    __shared__ unsigned arrived;
    const int nout = (cols + kBlk) * kBlk;
    const int o = blockIdx.x * 16 + (threadIdx.x & 15);
    const double t = finish16(part, G, nout, o, s16);
    if (threadIdx.x < 16 && o < nout) Hg[o] = t;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) arrived = atomicAdd(counter, 1u);
    __syncthreads();
    if (arrived != gridDim.x - 1) return;
    __threadfence();
    if (threadIdx.x == 0) *counter = 0u;
    wg_pip_chol(Hg, cols, pass, Rsave, T, ldt, coef, flags, floor_ref, &w, skip);
}
void finish_pip(hipStream_t s, const RedScratch &rs, int blocks, int cols, double *Hg, int pass, double *Rsave,
                double *T, int ldt, double *coef, int *flags, const double *floor_ref, int *skip) {
    const int nout = (cols + kBlk) * kBlk;
    hipLaunchKernelGGL(k_finish_pip, dim3(cdiv(nout, 16)), dim3(kWG), 0, s, rs.partials, blocks, cols, Hg, rs.counter,
                       pass, Rsave, T, ldt, coef, flags, floor_ref, skip);
}

void pip_chol(hipStream_t s, const double *Hg, int cols, int pass, double *Rsave, double *T, int ldt,
              double *coef, int *flags, const double *floor_ref) {
    hipLaunchKernelGGL(k_pip_chol, dim3(1), dim3(kWG), 0, s, Hg, cols, pass, Rsave, T, ldt, coef, flags,
                       floor_ref);
}

// the same reduction with an FP32 B (the sketch's test matrix), widened on load
__global__ __launch_bounds__(kWG) void k_tn_mfma_f(int n, const double *__restrict__ A, int lda, int ca,
                                                   const float *__restrict__ B, int ldb, int cb,
                                                   double *__restrict__ partials) {
    __shared__ TnWork w;
    wg_tn_mfma<float, 4, false>(n, A, lda, ca, B, ldb, cb, blockIdx.x, gridDim.x,
                                partials + (size_t)blockIdx.x * ca * cb, cb, 1.0, 0.0, &w);
}
void tn_reduce_f(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca, const float *B,
                 int ldb, int cb, double *H, int ldh, double alpha) {
    int blocks;
    if (cb <= 16 && ca <= kMaxBasis) {
        blocks = mfma_blocks(rs, n);
        hipLaunchKernelGGL(k_tn_mfma_f, dim3(blocks), dim3(kWG), 0, s, n, A, lda, ca, B, ldb, cb, rs.partials);
    } else {
        blocks = tn_blocks(rs, n);
        hipLaunchKernelGGL((k_tn_reduce<float, 0, false>), dim3(blocks), dim3(kWG), 0, s, n, A, lda, ca, B, ldb, cb,
                           rs.partials);
    }
    red_finish(s, rs.partials, blocks, ca * cb, H, cb, ldh, alpha, 0.0);
}

// ---------------------------------------------------------------------------
// C = beta*C + alpha*A H : rows of A staged through LDS, H (ca x cc) in LDS,
// L lanes per output row.
// ---------------------------------------------------------------------------
// C = beta*C + alpha*[A A2] H with an optional second source A2 (n x ca2, ca2 <= 8):
// the rows of both are staged side by side in LDS.
template <typename TC, int L>
__global__ __launch_bounds__(kWG) void k_nn_update(int n, const double *__restrict__ A, int lda, int ca,
                                                   const double *__restrict__ A2, int lda2, int ca2,
                                                   const double *__restrict__ H, int ldh, int cc,
                                                   TC *__restrict__ C, int ldc, double alpha, double beta,
                                                   const int *skip, const double *beta_dev) {
    constexpr int R = kWG / L;  // rows per workgroup
    if (skip && *skip) return;
    if (beta_dev) beta = *beta_dev;
    __shared__ double sH[(kMaxBasis + kBlk) * 16];
    __shared__ double sA[R][kMaxBasis + kBlk + 1];
    const int tid = threadIdx.x;
    const int ct = ca + ca2;
    for (int e = tid; e < ct * cc; e += kWG) {
        const int a = e / cc, c = e - a * cc;
        sH[e] = H[a * ldh + c];
    }
    const long row0 = (long)blockIdx.x * R;
    for (int e = tid; e < R * ca; e += kWG) {
        const int r = e / ca, a = e - r * ca;
        const long i = row0 + r;
        sA[r][a] = (i < n) ? A[i * lda + a] : 0.0;
    }
    for (int e = tid; e < R * ca2; e += kWG) {
        const int r = e / ca2, a = e - r * ca2;
        const long i = row0 + r;
        sA[r][ca + a] = (i < n) ? A2[i * lda2 + a] : 0.0;
    }
    __syncthreads();
    const int r = tid / L, c = tid % L;
    const long i = row0 + r;
    if (i >= n || c >= cc) return;
    double s = 0.0;
    for (int a = 0; a < ct; ++a) s += sA[r][a] * sH[a * cc + c];
    double v = alpha * s;
    if (beta != 0.0) v += beta * (double)C[i * ldc + c];
    C[i * ldc + c] = (TC)v;
}

// ---------------------------------------------------------------------------
// C = beta*C + alpha*[A A2] H on the FP64 matrix cores: a wavefront takes 16 rows at a
// time, loads them with row-contiguous loads into its own LDS tile, then runs
// V_MFMA_F64_16X16X4F64 over the (ca + ca2) columns four at a time:
// X[m][k] = tile[m][4 q + k], Y[k][j] = H[4 q + k][j] (held in registers for the whole
// launch), D[m][j] = output row row0 + m, column j.  Each element of A is read from
// memory once per launch.
// ---------------------------------------------------------------------------
template <int NL>
__global__ __launch_bounds__(kWG) void k_nn_mfma(int n, const double *__restrict__ A, int lda, int ca,
                                                 const double *__restrict__ A2, int lda2, int ca2,
                                                 const double *__restrict__ H, int ldh, int cc,
                                                 double *__restrict__ C, int ldc, double alpha, double beta,
                                                 const int *skip, const double *beta_dev) {
    __shared__ NnWork w;
    if (skip && *skip) return;
    if (beta_dev) beta = *beta_dev;
    wg_nn_mfma<NL>(n, A, lda, ca, A2, lda2, ca2, H, ldh, cc, C, ldc, alpha, beta, blockIdx.x, gridDim.x, &w);
}

// pass-0 update of a Lanczos block fused with the pass-1 reduction (wg_nn_tn_mfma)
template <int NL>
__global__ __launch_bounds__(kWG) void k_nn_tn_mfma(int n, const double *__restrict__ A, int lda, int ca,
                                                    const double *__restrict__ A2, int lda2,
                                                    const double *__restrict__ H, int ldh, double *__restrict__ C,
                                                    int ldc, double *__restrict__ partials) {
    __shared__ NnTnWork w;
    wg_nn_tn_mfma<NL>(n, A, lda, ca, A2, lda2, H, ldh, C, ldc, blockIdx.x, gridDim.x,
                      partials + (size_t)blockIdx.x * (ca + kBlk) * kBlk, &w);
}

template <int NL>
static void launch_nn_tn(hipStream_t s, int blocks, hipEvent_t e0, hipEvent_t e1, int n, const double *A, int lda,
                         int ca, const double *A2, int lda2, const double *H, int ldh, double *C, int ldc,
                         double *partials) {
    if (e0 && e1)
        hipExtLaunchKernelGGL(k_nn_tn_mfma<NL>, dim3(blocks), dim3(kWG), 0, s, e0, e1, 0, n, A, lda, ca, A2, lda2, H,
                              ldh, C, ldc, partials);
    else
        hipLaunchKernelGGL(k_nn_tn_mfma<NL>, dim3(blocks), dim3(kWG), 0, s, n, A, lda, ca, A2, lda2, H, ldh, C, ldc,
                           partials);
}

int nn_update2_reorth(hipStream_t s, const RedScratch &rs, int n, const double *A, int lda, int ca, const double *A2,
                      int lda2, const double *H, int ldh, double *C, int ldc, hipEvent_t ev_start,
                      hipEvent_t ev_stop) {
    const int blocks = mfma_blocks(rs, n);
    with_tile_loads(ca, [&](auto nl) {   // buffer loads per lane of one 16-row group
        launch_nn_tn<decltype(nl)::value>(s, blocks, ev_start, ev_stop, n, A, lda, ca, A2, lda2, H, ldh, C, ldc,
                                          rs.partials);
    });
    return blocks;
}

// the matrix-core update takes at most 16 output columns and 8 columns of A2
static bool use_nn_mfma(int n, int cc, int ca2) { return n > 0 && cc <= 16 && ca2 <= kBlk; }
static int nn_mfma_blocks(int n) {
    // one row group per wavefront up to the tuned cap (4096 workgroups by default); the
    // grid size does not change any output value
    const int cap = (g_tune && g_tune->nn_cap > 0) ? g_tune->nn_cap : 4096;
    int b = cdiv(((long)n + 15) / 16, 4);
    return b < 1 ? 1 : (b > cap ? cap : b);
}

template <typename TC>
static void nn_update_t(hipStream_t s, int n, const double *A, int lda, int ca, const double *A2, int lda2,
                        int ca2, const double *H, int ldh, int cc, TC *C, int ldc, double alpha, double beta,
                        const int *skip = nullptr, const double *beta_dev = nullptr) {
    if (n <= 0 || cc <= 0) return;
    if constexpr (sizeof(TC) == 8) {
        if (use_nn_mfma(n, cc, ca2)) {
            const dim3 grid(nn_mfma_blocks(n));
            with_tile_loads(ca, [&](auto nl) {
                hipLaunchKernelGGL(k_nn_mfma<decltype(nl)::value>, grid, dim3(kWG), 0, s, n, A, lda, ca, A2, lda2,
                                   ca2, H, ldh, cc, (double *)C, ldc, alpha, beta, skip, beta_dev);
            });
            return;
        }
    }
    if (cc <= 4)
        hipLaunchKernelGGL((k_nn_update<TC, 4>), dim3(cdiv(n, kWG / 4)), dim3(kWG), 0, s, n, A, lda, ca, A2, lda2,
                           ca2, H, ldh, cc, C, ldc, alpha, beta, skip, beta_dev);
    else if (cc <= 8)
        hipLaunchKernelGGL((k_nn_update<TC, 8>), dim3(cdiv(n, kWG / 8)), dim3(kWG), 0, s, n, A, lda, ca, A2, lda2,
                           ca2, H, ldh, cc, C, ldc, alpha, beta, skip, beta_dev);
    else
        hipLaunchKernelGGL((k_nn_update<TC, 16>), dim3(cdiv(n, kWG / 16)), dim3(kWG), 0, s, n, A, lda, ca, A2,
                           lda2, ca2, H, ldh, cc, C, ldc, alpha, beta, skip, beta_dev);
}

void nn_update2(hipStream_t s, int n, const double *A, int lda, int ca, const double *A2, int lda2, int ca2,
                const double *H, int ldh, int cc, double *C, int ldc, const int *skip) {
    nn_update_t<double>(s, n, A, lda, ca, A2, lda2, ca2, H, ldh, cc, C, ldc, 1.0, 0.0, skip);
}

void nn_update(hipStream_t s, int n, const double *A, int lda, int ca, const double *H, int ldh, int cc,
               double *C, int ldc, double alpha, double beta) {
    nn_update_t<double>(s, n, A, lda, ca, nullptr, 0, 0, H, ldh, cc, C, ldc, alpha, beta);
}
void nn_update_beta_dev(hipStream_t s, int n, const double *A, int lda, int ca, const double *H, int ldh, int cc,
                        double *C, int ldc, const double *beta_dev) {
    nn_update_t<double>(s, n, A, lda, ca, nullptr, 0, 0, H, ldh, cc, C, ldc, 1.0, 1.0, nullptr, beta_dev);
}
void nn_update_f(hipStream_t s, int n, const double *A, int lda, int ca, const double *H, int ldh, int cc,
                 float *C, int ldc, double alpha, double beta) {
    nn_update_t<float>(s, n, A, lda, ca, nullptr, 0, 0, H, ldh, cc, C, ldc, alpha, beta);
}

// ---------------------------------------------------------------------------
// Gaussian test matrix of the sketch generated on the device (Sec. 4: Psi has i.i.d.
// N(0, 1) entries).  Element (i, c) comes from one Philox4x32-10 block (Salmon, Moraes,
// Dror and Shaw, SC'11) with counter (i mod 2^32, i div 2^32, c div 2, 0) and key (seed mod
// 2^32, seed div 2^32): u1 = ((w1 w0 >> 11) + 1) 2^-53 in (0, 1], u2 = (w3 w2 >> 11) 2^-53
// in [0, 1), and the Box-Muller pair sqrt(-2 ln u1) (cos 2 pi u2, sin 2 pi u2) gives the
// even and the odd column.  Stored as float32.  A row depends only on (seed, row), so the
// rows of a grown problem's first vertices are unchanged.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1) {
    for (int rnd = 0; rnd < 10; ++rnd) {
        if (rnd > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint64_t p0 = (uint64_t)0xD2511F53u * c[0];
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c[2];
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c[0] = hi1 ^ c[1] ^ k0;
        c[1] = lo1;
        c[2] = hi0 ^ c[3] ^ k1;
        c[3] = lo0;
    }
}
__global__ void k_psi_from_seed(long n, int r, uint64_t seed, float *__restrict__ psi) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n * r) return;
    const long i = e / r;
    const int col = (int)(e - i * r);
    uint32_t c[4] = {(uint32_t)i, (uint32_t)((uint64_t)i >> 32), (uint32_t)(col >> 1), 0u};
    philox4x32_10(c, (uint32_t)seed, (uint32_t)(seed >> 32));
    const uint64_t a = ((uint64_t)c[1] << 32) | c[0];
    const uint64_t b = ((uint64_t)c[3] << 32) | c[2];
    const double u1 = (double)((a >> 11) + 1) * 0x1.0p-53;
    const double u2 = (double)(b >> 11) * 0x1.0p-53;
    const double rad = sqrt(-2.0 * log(u1));
    const double ang = 6.283185307179586 * u2;   // 2 pi u2
    psi[e] = (float)((col & 1) ? rad * sin(ang) : rad * cos(ang));
}
void psi_from_seed(hipStream_t s, long n, int r, uint64_t seed, float *psi) {
    if (n <= 0 || r <= 0) return;
    hipLaunchKernelGGL(k_psi_from_seed, dim3(cdiv(n * r, kWG)), dim3(kWG), 0, s, n, r, seed, psi);
}

__global__ void k_copy_cols(int n, const double *__restrict__ A, int lda, int cc, double *__restrict__ C,
                            int ldc) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * cc) return;
    const long i = e / cc;
    const int c = (int)(e - i * cc);
    C[i * ldc + c] = A[i * lda + c];
}
void copy_cols(hipStream_t s, int n, const double *A, int lda, int cc, double *C, int ldc) {
    if (n <= 0 || cc <= 0) return;
    hipLaunchKernelGGL(k_copy_cols, dim3(cdiv((long)n * cc, kWG)), dim3(kWG), 0, s, n, A, lda, cc, C, ldc);
}

__global__ void k_fill(size_t count, double v, double *p) {
    const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < count) p[e] = v;
}
void fill(hipStream_t s, size_t count, double v, double *p) {
    if (count == 0) return;
    hipLaunchKernelGGL(k_fill, dim3(cdiv((long)count, kWG)), dim3(kWG), 0, s, count, v, p);
}

__global__ void k_random_block(int n, int cc, uint64_t seed, double *C, int ldc) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * cc) return;
    const long i = e / cc;
    const int c = (int)(e - i * cc);
    C[i * ldc + c] = hash_uniform(seed, (uint64_t)e);
}
void random_block(hipStream_t s, int n, int cc, uint64_t seed, double *C, int ldc) {
    if (n <= 0 || cc <= 0) return;
    hipLaunchKernelGGL(k_random_block, dim3(cdiv((long)n * cc, kWG)), dim3(kWG), 0, s, n, cc, seed, C, ldc);
}
// the same cc random columns (the same values) with columns cc..ldc-1 set to zero
__global__ void k_random_block_pad(int n, int cc, int ldc, uint64_t seed, double *C) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (long)n * ldc) return;
    const long i = e / ldc;
    const int c = (int)(e - i * ldc);
    C[e] = (c < cc) ? hash_uniform(seed, (uint64_t)(i * cc + c)) : 0.0;
}
void random_block_pad(hipStream_t s, int n, int cc, uint64_t seed, double *C, int ldc) {
    if (n <= 0 || ldc <= 0) return;
    hipLaunchKernelGGL(k_random_block_pad, dim3(cdiv((long)n * ldc, kWG)), dim3(kWG), 0, s, n, cc, ldc, seed, C);
}

// ---------------------------------------------------------------------------
// small symmetric eigenproblem on one workgroup (parallel cyclic Jacobi)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_small_eig(int N, const double *__restrict__ A, int lda,
                                                   double *__restrict__ w, double *__restrict__ Y, int ldy,
                                                   int ny, const int *__restrict__ dead) {
    __shared__ SyevWork ws;
    wg_syev_load(N, A, lda, dead, &ws);
    const int nv = N < kSyevMaxV ? N : kSyevMaxV;
    wg_syev_top(N, nv, ny < nv ? ny : nv, &ws, w, Y, ldy);
}

void small_eig(hipStream_t s, int N, const double *A, int lda, double *w, double *Y, int ldy, int ny,
               const int *dead) {
    hipLaunchKernelGGL(k_small_eig, dim3(1), dim3(kWG), 0, s, N, A, lda, w, Y, ldy, ny, dead);
}

// ---------------------------------------------------------------------------
// Lanczos restart: residual norms, convergence test and the compression of
// the 16 Ritz residuals to the 8 dominant directions (next block).
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_restart_prep(const double *__restrict__ RtR,
                                                      const double *__restrict__ theta, int kc, double tol,
                                                      double tol_rest, double *__restrict__ res,
                                                      int *__restrict__ flag, double *__restrict__ Z,
                                                      const double *__restrict__ scale_est) {
    __shared__ RestartWork w;
    wg_restart_prep(RtR, theta, kc, tol, tol_rest, res, flag, Z, scale_est, &w);
}

void lanczos_restart_prep(hipStream_t s, const double *RtR, const double *theta, int kc, double tol,
                          double tol_rest, double *res, int *flag, double *Z, double *scale_est) {
    hipLaunchKernelGGL(k_restart_prep, dim3(1), dim3(kWG), 0, s, RtR, theta, kc, tol, tol_rest, res, flag, Z,
                       scale_est);
}

__global__ void k_reset_T(double *T, int ldt, int N, const double *theta, int *dead) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < N * ldt) {
        const int a = e / ldt, c = e - a * ldt;
        T[e] = (a == c && a < kRitz) ? theta[a] : 0.0;
    }
    if (e < N) dead[e] = 0;
}
void lanczos_reset_T(hipStream_t s, double *T, int ldt, int N, const double *theta, int *dead) {
    hipLaunchKernelGGL(k_reset_T, dim3(cdiv((long)N * ldt, kWG)), dim3(kWG), 0, s, T, ldt, N, theta, dead);
}

// Rayleigh quotient that is already diagonal (U = Ritz vectors of the previous cycle):
// theta = diag(TUU), Y = I
__global__ void k_diag_theta(const double *TUU, int N, double *theta, double *Y) {
    const int e = threadIdx.x;
    if (e < N * N) Y[e] = (e / N == e % N) ? 1.0 : 0.0;
    if (e < N) theta[e] = TUU[e * N + e];
}
void diag_theta(hipStream_t s, const double *TUU, int N, double *theta, double *Y) {
    hipLaunchKernelGGL(k_diag_theta, dim3(1), dim3(kWG), 0, s, TUU, N, theta, Y);
}

__global__ void k_neg_diag(const double *theta, int N, double *H) {
    const int e = threadIdx.x;
    if (e < N * N) H[e] = (e / N == e % N) ? -theta[e / N] : 0.0;
}
void neg_diag(hipStream_t s, const double *theta, int N, double *H) {
    hipLaunchKernelGGL(k_neg_diag, dim3(1), dim3(kWG), 0, s, theta, N, H);
}

// ---------------------------------------------------------------------------
// constraint-side kernels of the bundle (App. B.2 and App. C)
// ---------------------------------------------------------------------------
// Q11 raw sum and G^T w_j: one partial per workgroup (wg_qp_gram)
__global__ __launch_bounds__(kWG) void k_qp_gram(int m, const int *__restrict__ kptr, const int *__restrict__ ti,
                                                 const int *__restrict__ tj, const double *__restrict__ tv,
                                                 const double *__restrict__ V, int ldv, int kd, int do_q11,
                                                 const double *w0, const double *w1, const double *w2,
                                                 const double *w3, int nw, double *partials) {
    __shared__ QpGramWork w;
    const int d = kd * (kd + 1) / 2;
    const int nout = (do_q11 ? d * (d + 1) / 2 : 0) + nw * d;
    wg_qp_gram(m, kptr, ti, tj, tv, V, ldv, kd, do_q11, w0, w1, w2, w3, nw, blockIdx.x, gridDim.x,
               partials + (size_t)blockIdx.x * nout, &w);
}

void qp_gram(hipStream_t s, const RedScratch &rs, int m, const int *kptr, const int *ti, const int *tj,
             const double *tv, const double *V, int ldv, int k, const double *const *w, int nw, double *out,
             int do_q11) {
    int blocks = cdiv(m, 2 * kQB);
    if (blocks > rs.max_blocks) blocks = rs.max_blocks;
    if (blocks < 1) blocks = 1;
    const int d = k * (k + 1) / 2;
    const int nout = (do_q11 ? d * (d + 1) / 2 : 0) + nw * d;
    hipLaunchKernelGGL(k_qp_gram, dim3(blocks), dim3(kWG), 0, s, m, kptr, ti, tj, tv, V, ldv, k, do_q11,
                       nw > 0 ? w[0] : nullptr, nw > 1 ? w[1] : nullptr, nw > 2 ? w[2] : nullptr,
                       nw > 3 ? w[3] : nullptr, nw, rs.partials);
    red_finish(s, rs.partials, blocks, nout, out, nout, nout, 1.0, 0.0);
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz update of a restart cycle in one sweep over the rows (block Lanczos with
// explicit restarts, App. E): with U (n x 16) the current block, MU = (C_s - A^* y) U and
// (Y, theta) the eigenpairs of U^T M U,
//   B = U Y            (the Ritz vectors, into the first 16 columns of the basis)
//   R = MU Y - B diag(theta)   (their residuals, over U: R may alias U)
//   R^T R              (per-workgroup partials, summed by red_finish)
// A wavefront stages 16 rows of U and of MU in LDS (BufferTile), forms both 16 x 16
// products on the FP64 matrix cores (Y in registers), R from the two accumulators, and
// R^T R from an LDS copy of R (four rows per product).  Reads 2 x 16 and writes 2 x 16
// doubles per row: half the traffic of three updates and a reduction.
// ---------------------------------------------------------------------------
constexpr int kRrLd = 17;
struct RrWork {
    double u[4][16][kRrLd], mu[4][16][kRrLd], r[4][16][kRrLd];
    double sred[3][4][64];
};
__global__ __launch_bounds__(kWG) void k_rr_update(int n, const double *U, const double *__restrict__ MU,
                                                   const double *__restrict__ Y, const double *__restrict__ theta,
                                                   double *__restrict__ B, int ldb, double *R,
                                                   double *__restrict__ partials) {
    __shared__ RrWork w;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kk = lane >> 4, j = lane & 15;
    double yv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) yv[q] = Y[(4 * q + kk) * 16 + j];
    const double th = theta[j];
    double(*Tu)[kRrLd] = w.u[wave];
    double(*Tm)[kRrLd] = w.mu[wave];
    double(*Tr)[kRrLd] = w.r[wave];
    BufferTile<4, kRrLd> tile;
    tile.prepare(16, 16, 0, 0);
    v4d racc = {0.0, 0.0, 0.0, 0.0};
    const long ngroups = ((long)n + 15) >> 4;
    const long gstride = (long)gridDim.x * 4;
    for (long g = (long)blockIdx.x * 4 + wave; g < ngroups; g += gstride) {
        const long row0 = 16 * g;
        const int rows = (int)min(16L, (long)n - row0);
        tile.load(row0, rows, U, 16, 16, nullptr, 0, 0, Tu);
        tile.load(row0, rows, MU, 16, 16, nullptr, 0, 0, Tm);
        wave_lds_sync();
        v4d ab = {0.0, 0.0, 0.0, 0.0}, am = {0.0, 0.0, 0.0, 0.0};
        double xu[4], xm[4];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            xu[q] = Tu[m][4 * q + kk];
            xm[q] = Tm[m][4 * q + kk];
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) ab = __builtin_amdgcn_mfma_f64_16x16x4f64(xu[q], yv[q], ab, 0, 0, 0);
#pragma unroll
        for (int q = 0; q < 4; ++q) am = __builtin_amdgcn_mfma_f64_16x16x4f64(xm[q], yv[q], am, 0, 0, 0);
        wave_lds_sync();   // U's tile is read; R may overwrite U's rows
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
            const int r = kk + 4 * vv;
            const double b = ab[vv];
            const double rr = __dsub_rn(am[vv], __dmul_rn(b, th));
            Tr[r][j] = rr;
            if (r < rows) {
                B[(row0 + r) * ldb + j] = b;
                R[(row0 + r) * 16 + j] = rr;
            }
        }
        wave_lds_sync();
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const double x = Tr[4 * s4 + kk][m];
            racc = __builtin_amdgcn_mfma_f64_16x16x4f64(x, x, racc, 0, 0, 0);
        }
        wave_lds_sync();   // the tiles are reloaded for the next row group
    }
    if (wave > 0)
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) w.sred[wave - 1][vv][lane] = racc[vv];
    __syncthreads();
    if (wave == 0) {
        double *dst = partials + (size_t)blockIdx.x * 256;
#pragma unroll
        for (int vv = 0; vv < 4; ++vv) {
            const double t = ((racc[vv] + w.sred[0][vv][lane]) + w.sred[1][vv][lane]) + w.sred[2][vv][lane];
            dst[(kk + 4 * vv) * 16 + j] = t;
        }
    }
}
void rr_update(hipStream_t s, const RedScratch &rs, int n, const double *U, const double *MU, const double *Y,
               const double *theta, double *B, int ldb, double *R, double *RtR) {
    const int blocks = mfma_blocks(rs, n);
    hipLaunchKernelGGL(k_rr_update, dim3(blocks), dim3(kWG), 0, s, n, U, MU, Y, theta, B, ldb, R, rs.partials);
    red_finish(s, rs.partials, blocks, 256, RtR, 16, 16, 1.0, 0.0);
}

// ---------------------------------------------------------------------------
// G^T w_j = svec(V^T A^*(w_j) V) (App. B.2, g_k = svec(V^T A_k V), by linearity) when every
// constraint triplet is diagonal (the MaxCut SDP of Sec. 5): A^*(w) is then the diagonal
// matrix with a_i = sum of v w_k over vertex i's triplets (k, i, i, v), and V^T diag(a) V is
// a weighted Gram matrix of the rows of V.  FP64 MFMA with the operand layout of
// wg_tn_mfma: a wavefront takes 4 rows per product, X[m][kk] = V[row kk][m] and
// Y[kk][j] = a_row V[row kk][j] from the same lane, one 16 x 16 accumulator per weight
// vector (NW <= 4 in one sweep over the rows); a is formed per row from (dptr, dk, dv).
// Each workgroup writes its NW k x k partials; k_wgram_finish sums them in a fixed order
// and writes the svec entries.
// ---------------------------------------------------------------------------
constexpr int kWgMaxW = 4;
constexpr int kWgUnr = 4;   // row groups in flight per wavefront
struct WeightPtrs {
    const double *w[kWgMaxW];
};
template <int NW>
__global__ __launch_bounds__(kWG) void k_wgram(int n, const double *__restrict__ V, int ldv, int k,
                                               const int *__restrict__ dptr, const int *__restrict__ dk,
                                               const double *__restrict__ dv, WeightPtrs ws,
                                               double *__restrict__ partials) {
    __shared__ double sred[3][NW][4][64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kk = lane >> 4;
    v4d acc[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[j] = (v4d){0.0, 0.0, 0.0, 0.0};
    const long ngroups = ((long)n + 3) >> 2;
    const long gstride = (long)gridDim.x * 4;
    for (long g0 = (long)blockIdx.x * 4 + wave; g0 < ngroups; g0 += kWgUnr * gstride) {
        double x[kWgUnr], a[kWgUnr][NW];
#pragma unroll
        for (int u = 0; u < kWgUnr; ++u) {
            const long row = 4 * (g0 + u * gstride) + kk;
            const bool ok = row < n;
            x[u] = (ok && m < k) ? V[row * ldv + m] : 0.0;
#pragma unroll
            for (int j = 0; j < NW; ++j) a[u][j] = 0.0;
            if (ok)
                for (int e = dptr[row]; e < dptr[row + 1]; ++e) {
                    const double v = dv[e];
                    const int kr = dk[e];
#pragma unroll
                    for (int j = 0; j < NW; ++j) a[u][j] += v * ws.w[j][kr];
                }
        }
#pragma unroll
        for (int u = 0; u < kWgUnr; ++u)
#pragma unroll
            for (int j = 0; j < NW; ++j) acc[j] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], a[u][j] * x[u], acc[j], 0, 0, 0);
    }
    if (wave > 0)
#pragma unroll
        for (int j = 0; j < NW; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) sred[wave - 1][j][v][lane] = acc[j][v];
    __syncthreads();
    if (wave == 0) {
        double *out = partials + (size_t)blockIdx.x * NW * k * k;
#pragma unroll
        for (int j = 0; j < NW; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double t = ((acc[j][v] + sred[0][j][v][lane]) + sred[1][j][v][lane]) + sred[2][j][v][lane];
                const int r = kk + 4 * v, c = m;   // D[r][c]
                if (r < k && c < k) out[(size_t)j * k * k + r * k + c] = t;
            }
    }
}
// out[j d + p] = f_p sum over the G partials of entry (j, a, b), p = (a, b) of the
// column-wise lower triangle (b outer, a = b..k-1), f_p = 1 on the diagonal, sqrt 2 off it.
// One workgroup per output: thread t sums partials t, t + 256, ... and the 256 sums are
// added in a fixed tree order.
__global__ __launch_bounds__(kWG) void k_wgram_finish(const double *__restrict__ part, int G, int k, int nw,
                                                      double *__restrict__ out) {
    __shared__ double red[kWG];
    const int d = k * (k + 1) / 2;
    const int o = blockIdx.x;
    const int j = o / d;
    int p = o - j * d, b = 0;
    while (p >= k - b) p -= k - b, ++b;
    const int a = b + p;
    const size_t src = (size_t)j * k * k + a * k + b, stride = (size_t)nw * k * k;
    double s = 0.0;
    for (int g = threadIdx.x; g < G; g += kWG) s += part[g * stride + src];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int h = kWG / 2; h > 0; h >>= 1) {
        if (threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[o] = (a == b) ? red[0] : 1.4142135623730951 * red[0];
}
void wgram(hipStream_t s, const RedScratch &rs, int n, const double *V, int ldv, int k, const int *dptr,
           const int *dk, const double *dv, const double *const *w, int nw, double *out) {
    if (nw <= 0) return;
    // each row costs a chain of dependent loads (triplet range, row index, weight), so the
    // grid is as large as the partials' space allows (nw k^2 doubles per workgroup), up to
    // 4096 workgroups, to keep many chains in flight
    const long room = (long)rs.max_blocks * rs.max_elems / ((long)nw * k * k);
    int blocks = cdiv(n, 64);
    if (blocks > 4096) blocks = 4096;
    if (blocks > room) blocks = (int)room;
    if (blocks < 1) blocks = 1;
    WeightPtrs ws{};
    for (int j = 0; j < nw && j < kWgMaxW; ++j) ws.w[j] = w[j];
    switch (nw) {
    case 1: hipLaunchKernelGGL(k_wgram<1>, dim3(blocks), dim3(kWG), 0, s, n, V, ldv, k, dptr, dk, dv, ws, rs.partials); break;
    case 2: hipLaunchKernelGGL(k_wgram<2>, dim3(blocks), dim3(kWG), 0, s, n, V, ldv, k, dptr, dk, dv, ws, rs.partials); break;
    case 3: hipLaunchKernelGGL(k_wgram<3>, dim3(blocks), dim3(kWG), 0, s, n, V, ldv, k, dptr, dk, dv, ws, rs.partials); break;
    default: hipLaunchKernelGGL(k_wgram<4>, dim3(blocks), dim3(kWG), 0, s, n, V, ldv, k, dptr, dk, dv, ws, rs.partials);
    }
    const int d = k * (k + 1) / 2;
    hipLaunchKernelGGL(k_wgram_finish, dim3(nw * d), dim3(kWG), 0, s, rs.partials, blocks, k, nw, out);
}

__global__ __launch_bounds__(kWG) void k_lowrank_A(int m, const int *__restrict__ kptr, const int *__restrict__ ti,
                                                   const int *__restrict__ tj, const double *__restrict__ tv,
                                                   const double *__restrict__ V, int ldv, int kd,
                                                   const double *__restrict__ K, double alpha, const double *zb,
                                                   const double *gamma_dev, double gamma_host, double *z,
                                                   double beta) {
    // zb and z may be the same array: each thread reads its entry before writing it
    __shared__ double sK[16 * 16];
    for (int e = threadIdx.x; e < 256; e += blockDim.x) {
        const int a = e >> 4, b = e & 15;
        sK[e] = (a < kd && b < kd) ? K[a * kd + b] : 0.0;
    }
    __syncthreads();
    const long k = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= m) return;
    const double acc = lowrank_row(k, kptr, ti, tj, tv, V, ldv, kd, sK);
    double v = alpha * acc;
    if (zb) v += (gamma_dev ? *gamma_dev : gamma_host) * zb[k];
    if (beta != 0.0) v += beta * z[k];
    z[k] = v;
}

void lowrank_A(hipStream_t s, int m, const int *kptr, const int *ti, const int *tj, const double *tv,
               const double *V, int ldv, int k, const double *K, double alpha, const double *zb,
               const double *gamma_dev, double gamma_host, double *z, double beta) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_lowrank_A, dim3(cdiv(m, kWG)), dim3(kWG), 0, s, m, kptr, ti, tj, tv, V, ldv, k, K, alpha,
                       zb, gamma_dev, gamma_host, z, beta);
}

constexpr int kMaxDots = 8;
__global__ __launch_bounds__(kWG) void k_dots(int m, const double *a0, const double *a1, const double *a2,
                                              const double *a3, const double *a4, const double *a5,
                                              const double *a6, const double *a7, const double *b0,
                                              const double *b1, const double *b2, const double *b3,
                                              const double *b4, const double *b5, const double *b6,
                                              const double *b7, int np, double *partials) {
    const double *as[kMaxDots] = {a0, a1, a2, a3, a4, a5, a6, a7};
    const double *bs[kMaxDots] = {b0, b1, b2, b3, b4, b5, b6, b7};
    __shared__ double red[kMaxDots][kWG];
    const int tid = threadIdx.x;
    double acc[kMaxDots];
    for (int j = 0; j < kMaxDots; ++j) acc[j] = 0.0;
    for (long i = (long)blockIdx.x * kWG + tid; i < m; i += (long)gridDim.x * kWG)
        for (int j = 0; j < np; ++j) acc[j] += as[j][i] * bs[j][i];
    for (int j = 0; j < np; ++j) red[j][tid] = acc[j];
    __syncthreads();
    for (int st = kWG / 2; st > 0; st >>= 1) {
        if (tid < st)
            for (int j = 0; j < np; ++j) red[j][tid] += red[j][tid + st];
        __syncthreads();
    }
    if (tid < np) partials[(size_t)blockIdx.x * np + tid] = red[tid][0];
}

void dots(hipStream_t s, const RedScratch &rs, int m, const double *const *a, const double *const *b, int np,
          double *out) {
    int blocks = cdiv(m, 4 * kWG);
    if (blocks > 256) blocks = 256;
    if (blocks > rs.max_blocks) blocks = rs.max_blocks;
    if (blocks < 1) blocks = 1;
    const double *A[kMaxDots] = {}, *B[kMaxDots] = {};
    for (int j = 0; j < np && j < kMaxDots; ++j) {
        A[j] = a[j];
        B[j] = b[j];
    }
    hipLaunchKernelGGL(k_dots, dim3(blocks), dim3(kWG), 0, s, m, A[0], A[1], A[2], A[3], A[4], A[5], A[6], A[7],
                       B[0], B[1], B[2], B[3], B[4], B[5], B[6], B[7], np, rs.partials);
    red_finish(s, rs.partials, blocks, np, out, np, np, 1.0, 0.0);
}

// ---------------------------------------------------------------------------
// interior point method for the master QP (App. B.2), one workgroup
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kWG) void k_ipm(IpmArgs a, const double *__restrict__ qp, double *state) {
    __shared__ IpmShared sh;
    wg_ipm(a, qp, state, &sh);
}

void ipm(hipStream_t s, const IpmArgs &a, const double *qp, double *state) {
    hipLaunchKernelGGL(k_ipm, dim3(1), dim3(kWG), 0, s, a, qp, state);
}

}  // namespace usbs

namespace usbs {
// ---------------------------------------------------------------------------
// decoupled rows: C - A^*(y) restricted to them is diagonal for every y, so
// each such row i carries the exact eigenpair (d_i, e_i).  The Krylov solver
// works on the complementary (coupled) rows only; these kernels remove the
// decoupled rows from a block and merge their eigenpairs into the Ritz set.
// ---------------------------------------------------------------------------
__global__ void k_mask_rows(int count, const int *__restrict__ idx, double *__restrict__ X, int ldx, int nc) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (long)count * nc) {
        const int q = (int)(e / nc), c = (int)(e - (long)q * nc);
        X[(size_t)idx[q] * ldx + c] = 0.0;
    }
}
void mask_rows(hipStream_t s, int count, const int *idx, double *X, int ldx, int nc) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_mask_rows, dim3((unsigned)cdiv((long)count * nc, kWG)), dim3(kWG), 0, s, count, idx, X,
                       ldx, nc);
}

// one workgroup: the 16 largest d_i over the decoupled rows, merged with the coupled
// Ritz values (wg_iso_merge)
__global__ __launch_bounds__(kWG) void k_iso_merge(int count, const int *__restrict__ idx,
                                                   const double *__restrict__ d, int have_coupled,
                                                   double *__restrict__ theta, double *__restrict__ res,
                                                   int *__restrict__ plan) {
    __shared__ IsoWork w;
    wg_iso_merge(count, idx, d, have_coupled, theta, res, plan, &w);
}
void iso_merge(hipStream_t s, int count, const int *idx, const double *d, int have_coupled, double *theta,
               double *res, int *plan) {
    hipLaunchKernelGGL(k_iso_merge, dim3(1), dim3(kWG), 0, s, count, idx, d, have_coupled, theta, res, plan);
}

// U[i, q] = Uc[i, plan[q]] (coupled Ritz vector), e_{-plan[q]-1} (decoupled row) or 0
__global__ void k_gather_ritz(int n, const double *__restrict__ Uc, const int *__restrict__ plan,
                              double *__restrict__ U) {
    const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < (long)n * kRitz) {
        const int i = (int)(e / kRitz), q = (int)(e - (long)i * kRitz);
        const int p = plan[q];
        double v = 0.0;
        if (p >= 0 && p < kRitz) v = Uc[(size_t)i * kRitz + p];
        else if (p < 0) v = (i == -p - 1) ? 1.0 : 0.0;
        U[e] = v;
    }
}
void gather_ritz(hipStream_t s, int n, const double *Uc, const int *plan, double *U) {
    hipLaunchKernelGGL(k_gather_ritz, dim3((unsigned)cdiv((long)n * kRitz, kWG)), dim3(kWG), 0, s, n, Uc, plan, U);
}
}  // namespace usbs
