// Device-side bodies of the hot-path steps, shared by the per-instance kernels
// (kernels.hip, steps.hip: one launch per step, possibly many workgroups) and
// the packed solver (packed.hip: one workgroup runs every step of one
// instance).  A body that reduces over rows takes its workgroup's share of the
// rows as (blk, nblk): the per-instance kernels pass (blockIdx.x, gridDim.x)
// and write a partial result per workgroup; the packed solver passes (0, 1) and
// writes the final value.  Bodies that need LDS take it as a pointer to a
// workspace struct, so the packed kernel can overlay the workspaces of steps
// that never run at the same time.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

#include "kernels.h"
#include "small_dense.h"
#include "steps.h"
#include "syev.h"

namespace usbs {

typedef double v4d __attribute__((ext_vector_type(4)));   // one lane's MFMA FP64 accumulator

__device__ __forceinline__ float bf16_to_f32(uint16_t h) {
    return __uint_as_float(((uint32_t)h) << 16);
}
__host__ __device__ inline uint16_t f32_to_bf16(float f) {
    // round to nearest even
    uint32_t u;
#if defined(__HIP_DEVICE_COMPILE__)
    u = __float_as_uint(f);
#else
    memcpy(&u, &f, 4);
#endif
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);   // inf / nan
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

// Values that are the same on every lane, re-read from the first lane: inside a function
// the compiler does not inline, its arguments arrive in vector registers; this moves
// sizes and pointers back to scalar registers (uniform loop control, scalar address
// arithmetic).  A no-op where the compiler already knows the value is uniform.
__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ long uni(long v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (long)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ double uni(double v) { return __longlong_as_double(uni((long)__double_as_longlong(v))); }
template <typename T>
__device__ __forceinline__ T *uni(T *p) {
    return (T *)uni((long)(uintptr_t)p);
}

// splitmix64 finaliser; the start blocks of the eigen-solver are uniform in [-1, 1]
// from the hash of (seed, element index)
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}
__device__ __forceinline__ double hash_uniform(uint64_t seed, uint64_t e) {
    const uint64_t h = mix64(seed * 0x100000001B3ull + e);
    return (double)(h >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// ---------------------------------------------------------------------------
// one output row of the shifted operator: sum over the row's off-diagonal
// nonzeros in two partial sums (even / odd position), then the diagonal term
//   Y[i, c] = diag[i] X[i, c] + scale * sum_e val[e] X[col[e], c]
// ---------------------------------------------------------------------------
template <typename VT, typename ACC>
__device__ __forceinline__ ACC spmm_value(const VT *__restrict__ val, int e) {
    if constexpr (sizeof(VT) == 2) return (ACC)bf16_to_f32(val[e]);
    else return (ACC)val[e];
}
template <typename VT, typename ACC>
__device__ __forceinline__ double spmm_row(int i, int cc, const int *__restrict__ rowptr, const int *__restrict__ col,
                                           const VT *__restrict__ val, ACC scale, const double *__restrict__ diag,
                                           const double *__restrict__ X, int ldx) {
    const int e0 = rowptr[i], e1 = rowptr[i + 1];
    ACC acc0 = 0, acc1 = 0;
    int e = e0;
    for (; e + 1 < e1; e += 2) {
        const int j0 = col[e], j1 = col[e + 1];
        const ACC v0 = spmm_value<VT, ACC>(val, e), v1 = spmm_value<VT, ACC>(val, e + 1);
        const ACC x0 = (ACC)X[(size_t)j0 * ldx + cc];
        const ACC x1 = (ACC)X[(size_t)j1 * ldx + cc];
        acc0 += v0 * x0;
        acc1 += v1 * x1;
    }
    if (e < e1) acc0 += spmm_value<VT, ACC>(val, e) * (ACC)X[(size_t)col[e] * ldx + cc];
    return diag[i] * X[(size_t)i * ldx + cc] + (double)(scale * (acc0 + acc1));
}

// ---------------------------------------------------------------------------
// H = A^T B (and with GRAM also B^T B below it) for cb <= 16 on the FP64 matrix
// cores: V_MFMA_F64_16X16X4F64 accumulates X (16 x 4) Y (4 x 16) with X[m][k] in
// lane m + 16 k, Y[k][j] in lane j + 16 k, and D[m][j] in lane j + 16 (m % 4),
// element m / 4.  A wavefront takes 4 rows at a time: X = 16 columns of A of those
// rows (one double per lane, 128 contiguous bytes per row), Y = the columns of B
// (lanes j >= cb hold 0), so every element of A is loaded once.  The Gram block
// B^T B uses Y as X.  UNR row groups are in flight per wavefront; the four
// wavefronts are summed in LDS in a fixed order and wavefront 0 writes
//   dst[a * ldd + j] = alpha * sum (+ beta * dst),  a < ca (+ cb with GRAM), j < cb.
// Row groups of this workgroup: g = 4 blk + wave + u * 4 nblk.
// ---------------------------------------------------------------------------
constexpr int kMfmaMaxCh = kMaxBasis / 16;   // 16-column chunks of A (ca <= 80)
struct TnWork {
    double sred[3][kMfmaMaxCh + 1][4][64];
};
template <typename TB, int UNR, bool GRAM>
__device__ __forceinline__ void wg_tn_mfma(int n, const double *__restrict__ A, int lda, int ca,
                                           const TB *__restrict__ B, int ldb, int cb, int blk, int nblk,
                                           double *dst, int ldd, double alpha, double beta, TnWork *w) {
    n = uni(n), lda = uni(lda), ca = uni(ca), ldb = uni(ldb), cb = uni(cb), blk = uni(blk), nblk = uni(nblk);
    A = uni(A), B = uni(B), dst = uni(dst), ldd = uni(ldd), alpha = uni(alpha), beta = uni(beta);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kk = lane >> 4;
    const int nch = (ca + 15) >> 4;
    v4d acc[kMfmaMaxCh + 1];
#pragma unroll
    for (int q = 0; q <= kMfmaMaxCh; ++q) acc[q] = (v4d){0.0, 0.0, 0.0, 0.0};
    const long ngroups = ((long)n + 3) >> 2;
    const long gstride = (long)nblk * 4;
    for (long g0 = (long)blk * 4 + wave; g0 < ngroups; g0 += UNR * gstride) {
        double yv[UNR], xv[UNR][kMfmaMaxCh];
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
            const long row = 4 * (g0 + u * gstride) + kk;
            const bool ok = (g0 + u * gstride < ngroups) && row < n;
            yv[u] = (ok && m < cb) ? (double)B[row * ldb + m] : 0.0;
#pragma unroll
            for (int q = 0; q < kMfmaMaxCh; ++q) {
                const int c = 16 * q + m;
                xv[u][q] = (ok && q < nch && c < ca) ? A[row * lda + c] : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < UNR; ++u) {
#pragma unroll
            for (int q = 0; q < kMfmaMaxCh; ++q)
                if (q < nch) acc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(xv[u][q], yv[u], acc[q], 0, 0, 0);
            if (GRAM) acc[kMfmaMaxCh] = __builtin_amdgcn_mfma_f64_16x16x4f64(yv[u], yv[u], acc[kMfmaMaxCh], 0, 0, 0);
        }
    }
    if (wave > 0)
#pragma unroll
        for (int q = 0; q <= kMfmaMaxCh; ++q)
#pragma unroll
            for (int v = 0; v < 4; ++v) w->sred[wave - 1][q][v][lane] = acc[q][v];
    __syncthreads();
    if (wave == 0) {
        const int j = lane & 15;
#pragma unroll
        for (int q = 0; q <= kMfmaMaxCh; ++q) {
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const double t =
                    ((acc[q][v] + w->sred[0][q][v][lane]) + w->sred[1][q][v][lane]) + w->sred[2][q][v][lane];
                const int mm = (lane >> 4) + 4 * v;   // row of D held in this element
                const int a = (q < kMfmaMaxCh) ? 16 * q + mm : ca + mm;
                const bool valid = (q < kMfmaMaxCh) ? (q < nch && a < ca) : (GRAM && mm < cb);
                if (valid && j < cb) {
                    double *p = dst + (size_t)a * ldd + j;
                    *p = (beta != 0.0) ? alpha * t + beta * (*p) : alpha * t;
                }
            }
        }
    }
}

// orders this wavefront's LDS accesses (a wavefront's LDS operations execute in order):
// a compiler barrier that, unlike a workgroup-scope fence, does not wait for the
// wavefront's outstanding global loads and stores
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Rows row0 .. row0 + rows - 1 (rows <= 16) of [A A2] into the wavefront's LDS tile T
// (rows 0..15, columns 0..ca+ca2-1; rows >= rows are zero) with raw buffer loads.  The
// buffer resource of a row group (scalar registers) starts at its first row and ends after
// its last valid row; a lane's byte offset inside the group is the same for every group, so
// it is computed once (TileLanes), and the hardware range check returns zero for rows past
// the end and for lanes past the tile (their offset is out of range), with no per-row
// address arithmetic, clamps or predicated loads.  A's 16 ca elements form one flat
// sequence, element e = lane + 64 t being (row e / ca, column e % ca), so every lane is busy
// and each row is read contiguously (NL >= 16 ca / 64 loads per lane); A2 (ca2 <= 8 columns)
// takes two more loads per lane, element e = lane + 64 h being (row e / 8, column e % 8).
// Column LD - 1 of the tile is padding (ca + ca2 < LD): lanes past the tile store their
// zero there, so the stores need no branch either.
constexpr int kBufOutOfRange = 0x7ffffff8;   // a byte offset past every row group
constexpr int kBufDword3 = 0x00020000;       // buffer resource word 3 on CDNA (raw, 32-bit data)
template <int NL>
struct TileLanes {
    int boff[NL], loff[NL];   // A: byte offset in the row group, element offset in the tile
    int boff2[2], loff2[2];   // A2
};
template <int NL, int LD>
__device__ __forceinline__ void tile_lanes(int ca, int lda, int ca2, int lda2, TileLanes<NL> &tl) {
    const int lane = threadIdx.x & 63;
    const int nel = 16 * ca;
    // element e -> (row, column) with a float reciprocal and one correction step
    // (e < 64 NL <= 1408, far inside float precision)
    const float inv = 1.0f / (float)max(ca, 1);
#pragma unroll
    for (int t = 0; t < NL; ++t) {
        const int e = lane + 64 * t;
        int r = (int)((float)e * inv);
        int c = e - r * ca;
        if (c >= ca) c -= ca, ++r;
        if (c < 0) c += ca, --r;
        const bool in = e < nel;
        tl.boff[t] = in ? (r * lda + c) * 8 : kBufOutOfRange;
        tl.loff[t] = in ? r * LD + c : LD - 1;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int e = lane + 64 * h, r = e >> 3, c = e & 7;
        const bool in = c < ca2;
        tl.boff2[h] = in ? (r * lda2 + c) * 8 : kBufOutOfRange;
        tl.loff2[h] = in ? r * LD + ca + c : LD - 1;
    }
}
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_group_rsrc(const double *M, int ld, long row0, int rows) {
    return __builtin_amdgcn_make_buffer_rsrc((void *)uni(M + row0 * ld), (short)0, uni(rows * ld * 8), kBufDword3);
}
template <int NL, int LD>
__device__ __forceinline__ void wave_load_tile(long row0, int rows, const double *__restrict__ A, int lda,
                                               const double *__restrict__ A2, int lda2, int ca2,
                                               const TileLanes<NL> &tl, double (*T)[LD]) {
    const __amdgpu_buffer_rsrc_t ra = row_group_rsrc(A, lda, row0, rows);
    double v[NL];
#pragma unroll
    for (int t = 0; t < NL; ++t)
        v[t] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(ra, tl.boff[t], 0, 0));
    double v2[2] = {0.0, 0.0};
    if (ca2 > 0) {
        const __amdgpu_buffer_rsrc_t rb = row_group_rsrc(A2, lda2, row0, rows);
#pragma unroll
        for (int h = 0; h < 2; ++h)
            v2[h] = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rb, tl.boff2[h], 0, 0));
    }
    double *Tf = &T[0][0];
#pragma unroll
    for (int t = 0; t < NL; ++t) Tf[tl.loff[t]] = v[t];
    if (ca2 > 0)
#pragma unroll
        for (int h = 0; h < 2; ++h) Tf[tl.loff2[h]] = v2[h];
}
// Row-group loaders of the update kernels (template argument Tile of wg_nn_mfma and
// wg_nn_tn_mfma).  BufferTile: raw buffer loads as above, NL >= 16 ca / 64 (A2 separate).
// FlatTile: generic loads over the flat sequence of all 16 (ca + ca2) elements of [A A2]
// (element e = lane + 64 t is (row e / ct, column e % ct)), NL >= 16 (ca + ca2) / 64; every
// load comes from a valid (clamped) address and is masked by a product (the data are
// finite), so no load waits inside a branch.  The persistent packed kernel keeps FlatTile:
// with BufferTile its solves left the trajectory of FlatTile (the two forms computed side
// by side in that kernel agreed bit for bit), so the per-instance kernels alone use
// BufferTile.
template <int NL, int LD>
struct BufferTile {
    TileLanes<NL> tl;
    __device__ __forceinline__ void prepare(int ca, int lda, int ca2, int lda2) {
        tile_lanes<NL, LD>(ca, lda, ca2, lda2, tl);
    }
    __device__ __forceinline__ void load(long row0, int rows, const double *__restrict__ A, int lda, int,
                                         const double *__restrict__ A2, int lda2, int ca2, double (*T)[LD]) const {
        wave_load_tile<NL, LD>(row0, rows, A, lda, A2, lda2, ca2, tl, T);
    }
};
template <int NL, int LD>
struct FlatTile {
    __device__ __forceinline__ void prepare(int, int, int, int) {}
    __device__ __forceinline__ void load(long row0, int rows, const double *__restrict__ A, int lda, int ca,
                                         const double *__restrict__ A2, int lda2, int ca2, double (*T)[LD]) const {
        const int lane = threadIdx.x & 63;
        const int ct = ca + ca2, nel = 16 * ct;
        const float inv = 1.0f / (float)ct;
        double v[NL];
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int e = lane + 64 * t;
            int r = (int)((float)e * inv);
            int c = e - r * ct;
            if (c >= ct) c -= ct, ++r;
            if (c < 0) c += ct, --r;
            const long rc = row0 + min(r, rows - 1);
            const double *pa = A + rc * lda + min(c, ca - 1);
            const double *pb = (ca2 > 0) ? A2 + rc * lda2 + max(c - ca, 0) : pa;
            const double val = *((c < ca) ? pa : pb);
            v[t] = val * ((e < nel && r < rows) ? 1.0 : 0.0);
        }
#pragma unroll
        for (int t = 0; t < NL; ++t) {
            const int e = lane + 64 * t;
            int r = (int)((float)e * inv);
            int c = e - r * ct;
            if (c >= ct) c -= ct, ++r;
            if (c < 0) c += ct, --r;
            const bool in = e < nel;
            T[in ? r : 0][in ? c : LD - 1] = v[t];
        }
    }
};

// loads per lane for a 16-row group of c elements per row (c <= 88: ca for BufferTile,
// ca + ca2 for FlatTile), rounded up to an instantiated size, and a call of f with that
// size as a compile-time constant
__host__ __device__ constexpr int tile_loads(int ca) {
    return ca <= 16 ? 4 : ca <= 32 ? 8 : ca <= 48 ? 12 : ca <= 64 ? 16 : ca <= 80 ? 20 : 22;
}
template <int N>
struct TileLoadsC {
    static constexpr int value = N;
};
template <typename F>
__host__ __device__ __forceinline__ void with_tile_loads(int ca, F &&f) {
    switch (tile_loads(ca)) {
    case 4: f(TileLoadsC<4>{}); break;
    case 8: f(TileLoadsC<8>{}); break;
    case 12: f(TileLoadsC<12>{}); break;
    case 16: f(TileLoadsC<16>{}); break;
    case 20: f(TileLoadsC<20>{}); break;
    default: f(TileLoadsC<22>{});
    }
}

// ---------------------------------------------------------------------------
// C = beta*C + alpha*[A A2] H on the FP64 matrix cores: a wavefront takes 16 rows at a
// time, loads them into its own LDS tile (wave_load_tile), then runs
// V_MFMA_F64_16X16X4F64 over the (ca + ca2) columns four at a time:
// X[m][k] = tile[m][4 q + k], Y[k][j] = H[4 q + k][j] (held in registers), D[m][j] =
// output row row0 + m, column j.  Each element of A is read once.  C must not alias
// A or A2.  Row groups of this workgroup: g = 4 blk + wave + t * 4 nblk.
// ---------------------------------------------------------------------------
constexpr int kNnMaxQ = (kMaxBasis + kBlk) / 4;   // 22 four-column steps
constexpr int kNnLd = kMaxBasis + kBlk + 1;
struct NnWork {
    double tile[4][16][kNnLd];
};
template <int NL, template <int, int> class Tile = BufferTile>
__device__ __forceinline__ void wg_nn_mfma(int n, const double *__restrict__ A, int lda, int ca,
                                           const double *__restrict__ A2, int lda2, int ca2,
                                           const double *__restrict__ H, int ldh, int cc, double *__restrict__ C,
                                           int ldc, double alpha, double beta, int blk, int nblk, NnWork *w) {
    n = uni(n), lda = uni(lda), ca = uni(ca), lda2 = uni(lda2), ca2 = uni(ca2), ldh = uni(ldh), cc = uni(cc);
    ldc = uni(ldc), blk = uni(blk), nblk = uni(nblk), alpha = uni(alpha), beta = uni(beta);
    A = uni(A), A2 = uni(A2), H = uni(H), C = uni(C);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int m = lane & 15, kk = lane >> 4, j = lane & 15;
    const int ct = ca + ca2;
    const int nq = (ct + 3) >> 2;
    // H in registers (unconditional loads from clamped indices, masked): Y[k][j] = H[4 q + k][j]
    double yv[kNnMaxQ];
#pragma unroll
    for (int q = 0; q < kNnMaxQ; ++q) {
        const int a = 4 * q + kk;
        const double h = H[min(a, ct - 1) * ldh + min(j, cc - 1)];
        yv[q] = h * ((a < ct && j < cc) ? 1.0 : 0.0);
    }
    double(*T)[kNnLd] = w->tile[wave];
    // columns ct .. kNnLd - 1 of the tile are never loaded; the products of a four-step
    // chunk past ct read them (times yv = 0), so they are zeroed once
    for (int e = lane; e < 16 * kNnLd; e += 64)
        if (e % kNnLd >= ct) T[e / kNnLd][e % kNnLd] = 0.0;
    Tile<NL, kNnLd> tile;
    tile.prepare(ca, lda, ca2, lda2);
    const long ngroups = ((long)n + 15) >> 4;
    const long gstride = (long)nblk * 4;
    for (long g = (long)blk * 4 + wave; g < ngroups; g += gstride) {
        const long row0 = 16 * g;
        const int rows = (int)min(16L, (long)n - row0);
        tile.load(row0, rows, A, lda, ca, A2, lda2, ca2, T);
        wave_lds_sync();
        // four products at a time, their tile operands read first (one LDS wait per four)
        v4d acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int q0 = 0; q0 < kNnMaxQ; q0 += 4)
            if (q0 < nq) {
                double x[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = (q0 + u < kNnMaxQ) ? T[m][4 * (q0 + u) + kk] : 0.0;
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (q0 + u < kNnMaxQ) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], yv[q0 + u], acc, 0, 0, 0);
            }
        wave_lds_sync();   // the tile is reloaded for the next row group
        if (j < cc) {
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                const int r = kk + 4 * vv;
                if (r < rows) {
                    double o = alpha * acc[vv];
                    if (beta != 0.0) o += beta * C[(row0 + r) * ldc + j];
                    C[(row0 + r) * ldc + j] = o;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// The first Gram-Schmidt update of a Lanczos block fused with the second pass's
// reduction: C = [A A2] H (A2 and C of kBlk columns) as in wg_nn_mfma, then over the
// same 16 rows the partial [A C]^T C ((ca + kBlk) x kBlk, layout as wg_tn_mfma with
// GRAM): the rows of A are already in the wavefront's LDS tile, so the basis is read
// from memory once for both.  A wavefront loads its 16 rows of [A A2] as one flat
// sequence of 16 (ca + kBlk) elements (every lane busy, rows contiguous in memory);
// H sits in LDS.  Row groups of this workgroup: g = 4 blk + wave + t * 4 nblk.  The four
// wavefronts are summed in LDS in a fixed order into dst.
// ---------------------------------------------------------------------------
constexpr int kNtLd = kMaxBasis + 2 * kBlk + 1;
struct NnTnWork {
    union {
        double tile[4][16][kNtLd];   // [A | A2 | C] of 16 rows per wavefront
        double sred[3][kMfmaMaxCh + 1][4][64];
    } u;
    double sH[kMaxBasis + kBlk][kBlk];
};
template <int NL, template <int, int> class Tile = BufferTile>   // NL: loads per lane (see Tile)
__device__ __forceinline__ void wg_nn_tn_mfma(int n, const double *__restrict__ A, int lda, int ca,
                                              const double *__restrict__ A2, int lda2, const double *__restrict__ H,
                                              int ldh, double *__restrict__ C, int ldc, int blk, int nblk,
                                              double *__restrict__ dst, NnTnWork *w) {
    n = uni(n), lda = uni(lda), ca = uni(ca), lda2 = uni(lda2), ldh = uni(ldh), ldc = uni(ldc);
    blk = uni(blk), nblk = uni(nblk);
    A = uni(A), A2 = uni(A2), H = uni(H), C = uni(C), dst = uni(dst);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = lane & 15, kk = lane >> 4, j = lane & 15;
    const int ct = ca + kBlk;        // columns of [A A2]
    const int nq = (ct + 3) >> 2;
    const int nch = (ca + 15) >> 4;
    // H rows past ct and tile columns past ct are zero, read (as products with zero) by the
    // last four-step chunk of the update
    for (int e = tid; e < kNnMaxQ * 4 * kBlk; e += kWG)
        w->sH[e / kBlk][e % kBlk] = (e < ct * kBlk) ? H[(e / kBlk) * ldh + e % kBlk] : 0.0;
    double(*T)[kNtLd] = w->u.tile[wave];
    for (int e = lane; e < 16 * kNtLd; e += 64)
        if (e % kNtLd >= ct) T[e / kNtLd][e % kNtLd] = 0.0;
    Tile<NL, kNtLd> tile;
    tile.prepare(ca, lda, kBlk, lda2);
    __syncthreads();
    v4d racc[kMfmaMaxCh + 1];
#pragma unroll
    for (int q = 0; q <= kMfmaMaxCh; ++q) racc[q] = (v4d){0.0, 0.0, 0.0, 0.0};
    const long ngroups = ((long)n + 15) >> 4;
    const long gstride = (long)nblk * 4;
    for (long g = (long)blk * 4 + wave; g < ngroups; g += gstride) {
        const long row0 = 16 * g;
        const int rows = (int)min(16L, (long)n - row0);
        // ---- [A A2] rows into the tile ----
        tile.load(row0, rows, A, lda, ca, A2, lda2, kBlk, T);
        wave_lds_sync();
        // ---- C rows: D[m][j] = sum_a T[m][a] H[a][j]; ct is a multiple of 4, so every a < ct ----
        v4d acc = {0.0, 0.0, 0.0, 0.0};
        const double hmask = (j < kBlk) ? 1.0 : 0.0;
#pragma unroll
        for (int q0 = 0; q0 < kNnMaxQ; q0 += 4)
            if (q0 < nq) {
                // operands of four products read first (one LDS wait per four)
                double x[4], y[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int a = 4 * (q0 + u) + kk;
                    x[u] = (q0 + u < kNnMaxQ) ? T[m][a] : 0.0;
                    y[u] = (q0 + u < kNnMaxQ) ? w->sH[a][j & 7] * hmask : 0.0;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (q0 + u < kNnMaxQ) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(x[u], y[u], acc, 0, 0, 0);
            }
        if (j < kBlk) {
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                const int r = kk + 4 * vv;
                T[r][ct + j] = acc[vv];
                if (r < rows) C[(row0 + r) * ldc + j] = acc[vv];
            }
        }
        wave_lds_sync();
        // ---- [A C]^T C over these rows, four rows per product: X = 16 columns of A, Y = C.
        // Columns 16 q + m >= ca of X read the A2 / C part of the tile: they only feed rows
        // of the partial that are never written ----
        const double ymask = (m < kBlk) ? 1.0 : 0.0;
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
            const int row = 4 * s4 + kk;
            const double y = T[row][ct + (m & 7)] * ymask;
            double x[kMfmaMaxCh];
#pragma unroll
            for (int q = 0; q < kMfmaMaxCh; ++q) x[q] = T[row][16 * q + m];
#pragma unroll
            for (int q = 0; q < kMfmaMaxCh; ++q)
                if (q < nch) racc[q] = __builtin_amdgcn_mfma_f64_16x16x4f64(x[q], y, racc[q], 0, 0, 0);
            racc[kMfmaMaxCh] = __builtin_amdgcn_mfma_f64_16x16x4f64(y, y, racc[kMfmaMaxCh], 0, 0, 0);
        }
        wave_lds_sync();   // the tile is rewritten for the next row group
    }
    __syncthreads();   // the summation space overlays the tiles
    if (wave > 0)
#pragma unroll
        for (int q = 0; q <= kMfmaMaxCh; ++q)
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) w->u.sred[wave - 1][q][vv][lane] = racc[q][vv];
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int q = 0; q <= kMfmaMaxCh; ++q) {
#pragma unroll
            for (int vv = 0; vv < 4; ++vv) {
                const double t = ((racc[q][vv] + w->u.sred[0][q][vv][lane]) + w->u.sred[1][q][vv][lane]) +
                                 w->u.sred[2][q][vv][lane];
                const int mm = kk + 4 * vv;
                const int a = (q < kMfmaMaxCh) ? 16 * q + mm : ca + mm;
                const bool valid = (q < kMfmaMaxCh) ? (q < nch && a < ca) : (mm < kBlk);
                if (valid && j < kBlk) dst[(size_t)a * kBlk + j] = t;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// constraint-side bodies (App. B.2 and App. C)
// ---------------------------------------------------------------------------
// g_k = svec(V^T A_k V) for one constraint row k into g[0..d) (g may live in LDS)
__device__ __forceinline__ void svec_constraint(int k, const int *__restrict__ kptr, const int *__restrict__ ti,
                                                const int *__restrict__ tj, const double *__restrict__ tv,
                                                const double *__restrict__ V, int ldv, int kd, double *g) {
    const double r2 = 1.4142135623730951;
    int d = kd * (kd + 1) / 2;
    for (int p = 0; p < d; ++p) g[p] = 0.0;
    for (int t = kptr[k]; t < kptr[k + 1]; ++t) {
        const double *vi = V + (size_t)ti[t] * ldv;
        const double *vj = V + (size_t)tj[t] * ldv;
        const double v = tv[t];
        int p = 0;
        for (int b = 0; b < kd; ++b) {
            const double vib = vi[b], vjb = vj[b];
            for (int a = b; a < kd; ++a) {
                if (a == b) g[p] += v * vi[a] * vjb;
                else g[p] += v * r2 * 0.5 * (vi[a] * vjb + vib * vj[a]);
                ++p;
            }
        }
    }
}

// Q11 raw sum and G^T w_j over the constraint rows of this workgroup on the FP64 matrix
// cores.  G' = [G | w_0 .. w_{nw-1}] (row k: g_k = svec(V^T A_k V), then the weights
// w_j[k]) is built 64 rows at a time in LDS by all threads (four threads per row, each
// owning the svec columns b = part mod 4); the needed 16 x 16 tiles of G'^T G' (the
// upper triangle of G^T G when do_q11, and G^T w) are spread over the four wavefronts,
// each accumulated by V_MFMA_F64_16X16X4F64 over four rows per instruction (operand
// layout as wg_tn_mfma).  Every output is owned by one lane, so no cross-wave sum.
// out layout (d = kd(kd+1)/2): if do_q11, the upper triangle of sum_k g_k g_k^T row by
// row; then G^T w_j, j < nw.
constexpr int kQB = 64;
constexpr int kQgCh = (kMaxSvec + 15) / 16;                         // 16-column chunks of G
constexpr int kQgLd = 16 * (kQgCh + 1) + 1;                         // G chunks, weight chunk, pad
constexpr int kQgMaxTiles = kQgCh * (kQgCh + 1) / 2 + kQgCh;
constexpr int kQgPerWave = (kQgMaxTiles + 3) / 4;
struct QpGramWork {
    double sg[kQB][kQgLd];
};
__device__ __forceinline__ void wg_qp_gram(int m, const int *__restrict__ kptr, const int *__restrict__ ti,
                                           const int *__restrict__ tj, const double *__restrict__ tv,
                                           const double *__restrict__ V, int ldv, int kd, int do_q11,
                                           const double *w0, const double *w1, const double *w2, const double *w3,
                                           int nw, int blk, int nblk, double *out, QpGramWork *w) {
    m = uni(m), kd = uni(kd), do_q11 = uni(do_q11), nw = uni(nw), blk = uni(blk), nblk = uni(nblk), ldv = uni(ldv);
    kptr = uni(kptr), ti = uni(ti), tj = uni(tj), tv = uni(tv), V = uni(V), out = uni(out);
    w0 = uni(w0), w1 = uni(w1), w2 = uni(w2), w3 = uni(w3);
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m16 = lane & 15, kk = lane >> 4;
    const int d = kd * (kd + 1) / 2;
    const int nch = (d + 15) >> 4;
    const int nupper = do_q11 ? d * (d + 1) / 2 : 0;
    const int ntri = do_q11 ? nch * (nch + 1) / 2 : 0;
    const int ntiles = ntri + (nw > 0 ? nch : 0);
    int tP[kQgPerWave], tQ[kQgPerWave];
#pragma unroll
    for (int u = 0; u < kQgPerWave; ++u) {
        const int t = wave + 4 * u;
        tP[u] = -1;
        tQ[u] = -1;
        if (t < ntri) {   // (P, Q), P <= Q, in row order of the chunk grid
            int P = 0, rem = t;
            while (rem >= nch - P) {
                rem -= nch - P;
                ++P;
            }
            tP[u] = P;
            tQ[u] = P + rem;
        } else if (t < ntiles) {
            tP[u] = t - ntri;
            tQ[u] = kQgCh;   // the weight chunk
        }
    }
    v4d acc[kQgPerWave];
#pragma unroll
    for (int u = 0; u < kQgPerWave; ++u) acc[u] = (v4d){0.0, 0.0, 0.0, 0.0};
    const double *ws[4] = {w0, w1, w2, w3};
    const double r2 = 1.4142135623730951;
    const int brow = tid >> 2, part = tid & 3;
    for (long k0 = (long)blk * kQB; k0 < m; k0 += (long)nblk * kQB) {
        // ---- build 64 rows of G' (this thread: row brow, svec columns b = part mod 4) ----
        {
            const long k = k0 + brow;
            double *g = &w->sg[brow][0];
            for (int b = part; b < kd; b += 4) {
                const int off = b * kd - b * (b - 1) / 2;
                for (int a = b; a < kd; ++a) g[off + a - b] = 0.0;
            }
            if (k < m) {
                for (int t = kptr[k]; t < kptr[k + 1]; ++t) {
                    const double *vi = V + (size_t)ti[t] * ldv;
                    const double *vj = V + (size_t)tj[t] * ldv;
                    const double v = tv[t];
                    for (int b = part; b < kd; b += 4) {
                        const int off = b * kd - b * (b - 1) / 2;
                        const double vib = vi[b], vjb = vj[b];
                        for (int a = b; a < kd; ++a) {
                            if (a == b) g[off] += v * vi[a] * vjb;
                            else g[off + a - b] += v * r2 * 0.5 * (vi[a] * vjb + vib * vj[a]);
                        }
                    }
                }
            }
            if (part == 0)
                for (int j = 0; j < nw; ++j) g[16 * kQgCh + j] = (k < m) ? ws[j][k] : 0.0;
        }
        __syncthreads();
        // ---- G'^T G' tiles of this wavefront over the 64 rows ----
#pragma unroll
        for (int u = 0; u < kQgPerWave; ++u) {
            const int P = tP[u], Q = tQ[u];
            if (P < 0) continue;
            const int cx = 16 * P + m16;
            const bool wq = Q == kQgCh;
            const int cy = wq ? 16 * kQgCh + m16 : 16 * Q + m16;
            const bool okx = cx < d, oky = wq ? (m16 < nw) : (cy < d);
#pragma unroll 4
            for (int s4 = 0; s4 < kQB / 4; ++s4) {
                const int row = 4 * s4 + kk;
                const double x = okx ? w->sg[row][cx] : 0.0;
                const double y = oky ? w->sg[row][cy] : 0.0;
                acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, acc[u], 0, 0, 0);
            }
        }
        __syncthreads();
    }
    // ---- lane j + 16 (p % 4), element p / 4 holds D[p][j] of each tile ----
#pragma unroll
    for (int u = 0; u < kQgPerWave; ++u) {
        const int P = tP[u], Q = tQ[u];
        if (P < 0) continue;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int p = 16 * P + kk + 4 * v;
            if (p >= d) continue;
            if (Q < kQgCh) {
                const int q = 16 * Q + m16;
                if (q < d && p <= q) out[p * d - p * (p - 1) / 2 + (q - p)] = acc[u][v];
            } else if (m16 < nw) {
                out[nupper + m16 * d + p] = acc[u][v];
            }
        }
    }
}

// (A(V K V^T))_k for one constraint row: sum_t v_t V_i^T K V_j, K (16 x 16 padded) in LDS
__device__ __forceinline__ double lowrank_row(long k, const int *__restrict__ kptr, const int *__restrict__ ti,
                                              const int *__restrict__ tj, const double *__restrict__ tv,
                                              const double *__restrict__ V, int ldv, int kd, const double *sK) {
    double acc = 0.0;
    for (int t = kptr[k]; t < kptr[k + 1]; ++t) {
        const double *vi = V + (size_t)ti[t] * ldv;
        const double *vj = V + (size_t)tj[t] * ldv;
        double xj[16];
#pragma unroll
        for (int b = 0; b < 16; ++b) xj[b] = (b < kd) ? vj[b] : 0.0;
        double q = 0.0;
#pragma unroll 1
        for (int a = 0; a < kd; ++a) {
            double s = 0.0;
#pragma unroll
            for (int b = 0; b < 16; ++b) s += sK[a * 16 + b] * xj[b];
            q += vi[a] * s;
        }
        acc += tv[t] * q;
    }
    return acc;
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
struct PipWork {
    double sH[kMaxBasis][kBlk];
    double sOm[kBlk * 17];
    double sRi[kBlk * kBlk];
    double sR[kBlk][kBlk];
};
// A second pass adds nothing when the first lost little: with Pythagorean inner products the
// block after pass 0 is orthogonal to Q, and orthonormal, to about eps / p, where p is the
// smallest ratio L_cc^2 / ||W_c||^2 of the pass's Cholesky pivots to the column norms.
// With p >= kPass2Skip (error below 100 eps) and no deflated column, pass 0 sets *skip and
// the caller may take the pass-0 block as it stands (the pass-1 update is then skipped).
constexpr double kPass2Skip = 1e-2;
__device__ __forceinline__ void wg_pip_chol(const double *__restrict__ Hg, int cols, int pass,
                                            double *__restrict__ Rsave, double *__restrict__ T, int ldt,
                                            double *__restrict__ coef, int *flags,
                                            const double *__restrict__ floor_ref, PipWork *w, int *skip = nullptr) {
    const int tid = threadIdx.x;
    for (int e = tid; e < cols * kBlk; e += kWG) w->sH[e / kBlk][e % kBlk] = Hg[e];
    if (tid < kBlk * kBlk) w->sR[tid / kBlk][tid % kBlk] = (pass == 1) ? Rsave[tid] : 0.0;
    __syncthreads();
    {
        // Omega = G - H^T H: four lanes (one DPP quad) per entry
        static_assert(kBlk * kBlk * 4 == kWG, "one quad of lanes per entry of Omega");
        const int e = tid >> 2, q4 = tid & 3, i = e / kBlk, j = e % kBlk;
        double sacc = 0.0;
        for (int a = q4; a < cols; a += 4) sacc += w->sH[a][i] * w->sH[a][j];
        sacc = quad_sum(sacc);
        if (q4 == 0) w->sOm[i * 17 + j] = Hg[(cols + i) * kBlk + j] - sacc;
    }
    // projections of the original block into T
    for (int e = tid; e < cols * kBlk; e += kWG) {
        const int a = e / kBlk, c = e % kBlk;
        if (pass == 0) {
            T[a * ldt + c] = w->sH[a][c];
        } else {
            double v = 0.0;
            for (int k = 0; k <= c; ++k) v += w->sH[a][k] * w->sR[k][c];
            T[a * ldt + c] += v;
        }
    }
    __syncthreads();
    double f2 = 0.0;
    if (floor_ref) {
        const double rf = 1e-10 * (*floor_ref);
        f2 = rf * rf;
    }
    if (tid < 64) {
        const unsigned dead = wave_cholqr(kBlk, w->sOm, 17, w->sRi, kBlk, flags, f2);
        if (skip && pass == 0 && tid == 0) {
            bool ok = dead == 0;
            for (int c = 0; c < kBlk; ++c) {
                const double l = w->sOm[c * 17 + c];
                ok = ok && l * l >= kPass2Skip * Hg[(cols + c) * kBlk + c];
            }
            *skip = ok ? 1 : 0;
        }
    }
    __syncthreads();
    // R = L^T (upper) of this pass, kept for the correction of the next pass
    if (pass == 0 && tid < kBlk * kBlk) {
        const int i = tid / kBlk, j = tid % kBlk;
        Rsave[tid] = (j >= i) ? w->sOm[j * 17 + i] : 0.0;
    }
    for (int e = tid; e < (cols + kBlk) * kBlk; e += kWG) {
        const int a = e / kBlk, c = e % kBlk;
        double v;
        if (a < cols) {
            v = 0.0;
            for (int k = 0; k < kBlk; ++k) v -= w->sH[a][k] * w->sRi[k * kBlk + c];
        } else {
            v = w->sRi[(a - cols) * kBlk + c];
        }
        coef[e] = v;
    }
}

// ---------------------------------------------------------------------------
// Lanczos restart: residual norms, convergence test and the next block.  The next
// block is spanned by 8 of the 16 Ritz residuals, each scaled by 1 / ||r_p|| (the block
// is orthonormalised afterwards, with deflation), taken in this order: the wanted pairs
// (p < kc) that have not met their tolerance, from the top; then the unwanted pairs
// (p >= kc) from the top; then the converged wanted pairs.  For Ritz vectors of a block
// Krylov space all residuals lie in the span of the next Krylov block, so this is the
// thick restart; where the residuals of the kept vectors span more than 8 directions it
// keeps the ones that improve the pairs still to converge.
// convergence: residual of Ritz pair 0 <= tol * scale and of pairs 1..kc-1 <= tol_rest * scale
// ---------------------------------------------------------------------------
struct RestartWork {
    int sel[kBlk];
};
__device__ __forceinline__ void wg_restart_prep(const double *__restrict__ RtR, const double *__restrict__ theta,
                                                int kc, double tol, double tol_rest, double *__restrict__ res,
                                                int *__restrict__ flag, double *__restrict__ Z,
                                                const double *__restrict__ scale_est, RestartWork *w) {
    const int tid = threadIdx.x;
    (void)w;
    if (tid < kRitz) res[tid] = sqrt(fmax(RtR[tid * kRitz + tid], 0.0));
    if (tid == 0) {
        // tolerances are relative to a Gershgorin bound of the current operator
        double sc = fmax(fabs(theta[0]), fabs(theta[kRitz - 1]));
        if (scale_est) sc = fmax(sc, *scale_est);
        double r[kRitz], dmax = 0.0;
        bool conv[kRitz];
        for (int p = 0; p < kRitz; ++p) {
            r[p] = sqrt(fmax(RtR[p * kRitz + p], 0.0));
            dmax = fmax(dmax, r[p]);
            // the top Ritz pair sets f(y): tight tolerance; the others only shape the bundle
            conv[p] = r[p] <= ((p == 0) ? tol : tol_rest) * sc;
        }
        int ok = 1;
        for (int p = 0; p < kc && p < kRitz; ++p)
            if (!conv[p]) ok = 0;
        int sel[kBlk], ns = 0;
        for (int p = 0; p < kc && p < kRitz && ns < kBlk; ++p)
            if (!conv[p]) sel[ns++] = p;
        for (int p = kc; p < kRitz && ns < kBlk; ++p) sel[ns++] = p;
        for (int p = 0; p < kc && p < kRitz && ns < kBlk; ++p)
            if (conv[p]) sel[ns++] = p;
        for (int e = 0; e < kRitz * kBlk; ++e) Z[e] = 0.0;
        for (int t = 0; t < ns; ++t) {
            const int p = sel[t];
            if (r[p] > 1e-150 * dmax) Z[p * kBlk + t] = 1.0 / r[p];
        }
        *flag = ok;
    }
}

// ---------------------------------------------------------------------------
// decoupled rows (no off-diagonal entry in C - A^*(y) for any y): the 16 largest d
// over those rows (ties by row index) by repeated arg-max, then a merge with the 16
// descending coupled Ritz values; plan[q] = coupled column, -(row + 1) or 16 (empty).
// ---------------------------------------------------------------------------
struct IsoWork {
    double bv[kWG];
    int bq[kWG];
    double iv[kRitz];
    int ii[kRitz];
};
__device__ __forceinline__ void wg_iso_merge(int count, const int *__restrict__ idx, const double *__restrict__ d,
                                             int have_coupled, double *__restrict__ theta, double *__restrict__ res,
                                             int *__restrict__ plan, IsoWork *w) {
    const int tid = threadIdx.x;
    const int want = count < kRitz ? count : kRitz;
    for (int t = 0; t < want; ++t) {
        double best = -INFINITY;
        int bestq = -1;
        for (int q = tid; q < count; q += kWG) {
            bool taken = false;
            for (int u = 0; u < t; ++u) taken |= (w->ii[u] == q);
            const double v = d[idx[q]];
            if (!taken && (bestq < 0 || v > best)) {
                best = v;
                bestq = q;
            }
        }
        w->bv[tid] = best;
        w->bq[tid] = bestq;
        __syncthreads();
        for (int o = kWG / 2; o > 0; o >>= 1) {
            if (tid < o) {
                const double v2 = w->bv[tid + o];
                const int q2 = w->bq[tid + o];
                if (q2 >= 0 && (w->bq[tid] < 0 || v2 > w->bv[tid] || (v2 == w->bv[tid] && q2 < w->bq[tid]))) {
                    w->bv[tid] = v2;
                    w->bq[tid] = q2;
                }
            }
            __syncthreads();
        }
        if (tid == 0) {
            w->iv[t] = w->bv[0];
            w->ii[t] = w->bq[0];
        }
        __syncthreads();
    }
    if (tid == 0) {
        double th[kRitz], rr[kRitz];
        int pl[kRitz];
        int a = 0, b = 0;
        const int nc = have_coupled ? kRitz : 0;
        for (int q = 0; q < kRitz; ++q) {
            const bool take_c = a < nc && (b >= want || theta[a] >= w->iv[b]);
            if (take_c) {
                th[q] = theta[a];
                rr[q] = res[a];
                pl[q] = a++;
            } else if (b < want) {
                th[q] = w->iv[b];
                rr[q] = 0.0;
                pl[q] = -(idx[w->ii[b]] + 1);
                ++b;
            } else {   // fewer than 16 eigenpairs in total: pad with empty columns
                th[q] = -1e300;
                rr[q] = 0.0;
                pl[q] = kRitz;
            }
        }
        for (int q = 0; q < kRitz; ++q) {
            theta[q] = th[q];
            res[q] = rr[q];
            plan[q] = pl[q];
        }
    }
}

// ---------------------------------------------------------------------------
// small steps of the iteration on the device scalar array sc
// ---------------------------------------------------------------------------
// relative errors of eq. relative_error_tol (suboptimality through the upper bound of eq.
// objective_subopt_upper_bound) in the units selected by SC_UNITS
__device__ __forceinline__ void set_metrics(double *sc, double fn) {
    const double cx = sc[SC_CX];
    const double dist = sqrt(fmax(sc[SC_DIST2], 0.0));
    if (sc[SC_UNITS] != 0.0) {
        const double s = sc[SC_SIGMA] * sc[SC_TRACE];
        const double fo = s * fn, co = s * cx;
        sc[SC_GAP] = fabs(fo - co) / (1.0 + fabs(co));
        sc[SC_INF] = sc[SC_TRACE] * dist / (1.0 + sc[SC_TRACE] * sc[SC_BNORM]);
    } else {
        sc[SC_GAP] = fabs(fn - cx) / (1.0 + fabs(cx));
        sc[SC_INF] = dist / (1.0 + sc[SC_BNORM]);
    }
}

// master QP coefficients (App. B.2, eq. compressed_subprob_2, normalised form)
//   raw = [upper triangle of sum g g^T | G^T zbar | G^T y | G^T b | G^T nu]
__device__ __forceinline__ void wg_qp_finalize(int k, const double *__restrict__ raw, const double *__restrict__ VCV,
                                               const double *__restrict__ sc, int has_nu, double *__restrict__ qp) {
    const int d = k * (k + 1) / 2, nup = d * (d + 1) / 2;
    const double alpha = sc[SC_ALPHA], rho = sc[SC_RHO], tau = sc[SC_TAU];
    const double a2r = alpha * alpha / rho;
    const double *Gz = raw + nup, *Gy = Gz + d, *Gb = Gy + d, *Gn = Gb + d;
    for (int e = threadIdx.x; e < d * d; e += kWG) {
        const int P = e / d, Q = e - P * d;
        const int lo = P < Q ? P : Q, hi = P < Q ? Q : P;
        qp[e] = a2r * raw[lo * d - lo * (lo - 1) / 2 + (hi - lo)];
    }
    for (int p = threadIdx.x; p < d; p += kWG) {
        // p -> (i, j), i >= j, column-wise lower triangle
        int j = 0, rem = p;
        while (rem >= k - j) {
            rem -= k - j;
            ++j;
        }
        const int i = j + rem;
        const double sv = (i == j ? 1.0 : 1.4142135623730951) * VCV[i * k + j];
        const double gw = Gb[p] - (has_nu ? Gn[p] : 0.0);
        qp[d * d + p] = (tau > 0.0) ? a2r / tau * Gz[p] : 0.0;               // q12
        qp[d * d + d + 1 + p] = alpha * (Gy[p] - gw / rho - sv);             // h1
    }
    if (threadIdx.x == 0) {
        const double zz = sc[SC_ZZ], yz = sc[SC_YZBAR], bz = sc[SC_BZ], nz = has_nu ? sc[SC_NUZ] : 0.0;
        qp[d * d + d] = (tau > 0.0) ? a2r * zz / (tau * tau) : 0.0;                                        // q22
        qp[d * d + 2 * d + 1] = (tau > 0.0) ? alpha / tau * (yz - (bz - nz) / rho - sc[SC_CBAR]) : 0.0;   // h2
    }
}

// g = alpha eta / tau, <C, X_{t+1}> = g cbar + alpha <V^T C V, S>  (thread 0)
__device__ __forceinline__ void post_ipm_scalar(int k, const double *__restrict__ st, const double *__restrict__ VCV,
                                                double *sc) {
    const double alpha = sc[SC_ALPHA], tau = sc[SC_TAU];
    const double eta = st[2 * k * k];
    const double g = (tau > 0.0) ? alpha * eta / tau : 0.0;
    double vs = 0.0;
    for (int e = 0; e < k * k; ++e) vs += VCV[e] * st[e];
    sc[SC_ETA] = eta;
    sc[SC_G] = g;
    sc[SC_CX] = g * sc[SC_CBAR] + alpha * vs;
    sc[SC_IPMIT] += st[2 * k * k + 3];
    if (st[2 * k * k + 4] != 0.0) sc[SC_IPMSTATUS] = st[2 * k * k + 4];
}

// descent test (Alg. 1), f, f^ and the relative errors  (thread 0)
__device__ __forceinline__ void decide_scalar(const double *__restrict__ theta, double *sc) {
    const double alpha = sc[SC_ALPHA], beta = sc[SC_BETA], tau = sc[SC_TAU];
    const double by = sc[SC_BY];
    const double lam1 = theta[0];
    const double fc = alpha * fmax(lam1, 0.0) + by;
    double best = fmax(0.0, sc[SC_LAMV]);
    if (tau > 0.0) best = fmax(best, (sc[SC_CBAR] - sc[SC_YZ]) / tau);
    const double fhat = alpha * best + by;
    const double f = sc[SC_F];
    const int desc = (beta * (f - fhat) <= f - fc) ? 1 : 0;
    const double fn = desc ? fc : f;
    sc[SC_FCAND] = fc;
    sc[SC_FHAT] = fhat;
    sc[SC_THETA1] = lam1;
    sc[SC_DESC] = desc;
    sc[SC_NDESC] += desc;
    sc[SC_F] = fn;
    set_metrics(sc, fn);
}

// f(y_t) = alpha [theta_1]_+ + <b, y_t> from an accurate Ritz value (SC_BYT holds <b, y_t>).
// A Ritz value never exceeds lambda_max, so both the stored f and the new one are lower
// bounds of f(y_t) when y_t is unchanged: keep_max then keeps the larger.  (thread 0)
__device__ __forceinline__ void refresh_f_scalar(const double *__restrict__ theta, double *sc, int keep_max) {
    double fn = sc[SC_ALPHA] * fmax(theta[0], 0.0) + sc[SC_BYT];
    if (keep_max) fn = fmax(fn, sc[SC_F]);
    sc[SC_F] = fn;
    sc[SC_THETA1] = theta[0];
    set_metrics(sc, fn);
}

// alternating maximisation (eq. dual_slack_update): nu = proj_N(b - AX - rho y), one row
__device__ __forceinline__ void nu_update_elem(long k, const double *__restrict__ b, const double *__restrict__ AX,
                                              const double *__restrict__ y, const double *__restrict__ ineq,
                                              double rho, double *__restrict__ nu, double *__restrict__ dnu) {
    const double v = (ineq[k] != 0.0) ? fmax(b[k] - AX[k] - rho * y[k], 0.0) : 0.0;
    dnu[k] = v - nu[k];
    nu[k] = v;
}

// candidate (eq. dual_update, feasible form of Sec. 3.2) and the infeasibility vector, one row
__device__ __forceinline__ void candidate_elem(long k, const double *__restrict__ b, const double *__restrict__ AX,
                                              const double *__restrict__ y, const double *__restrict__ ineq,
                                              double rho, double *__restrict__ yc, double *__restrict__ e) {
    const double r = b[k] - AX[k];
    double v = y[k] - r / rho;
    if (ineq[k] != 0.0) {
        v = fmax(v, 0.0);
        e[k] = fmax(-r, 0.0);
    } else {
        e[k] = -r;
    }
    yc[k] = v;
}

// lambda_max(V^T (C - A^* y~) V) with V^T A^* y~ V = smat(G^T y~)
struct FhatWork {
    SyevWork ws;
    double Mv[kMaxK * kMaxK];
    double w[kMaxK + 1];
};
__device__ __forceinline__ void wg_fhat_prep(int k, const double *__restrict__ VCV, const double *__restrict__ Gy,
                                             double *sc, FhatWork *f) {
    const double r2 = 1.4142135623730951;
    for (int e = threadIdx.x; e < k * k; e += kWG) {
        const int i = e / k, j = e - i * k;
        const int lo = i > j ? j : i, hi = i > j ? i : j;
        const int p = lo * k - lo * (lo - 1) / 2 + (hi - lo);
        f->Mv[e] = VCV[e] - ((i == j) ? Gy[p] : Gy[p] / r2);
    }
    __syncthreads();
    wg_syev_load(k, f->Mv, k, nullptr, &f->ws);
    wg_syev_top(k, 1, 0, &f->ws, f->w, nullptr, 0);
    if (threadIdx.x == 0) sc[SC_LAMV] = f->w[0];
}

// model update (eqs. model_update_eigendecomposition, x_bar_def; App. C tracking):
// alpha S = Q diag(lam) Q^T (descending), Q_p = first k_p columns, Q_c = rest,
// Kc = Q_c Lam_c Q_c^T, tau <- g tau + tr Lam_c, cbar <- g cbar + <Kc, V^T C V>,
// Hsk = Kc (V^T Psi) (k x r) for the sketch.
struct ModelWork {
    SyevWork ws;
    double aS[kMaxK * kMaxK];
    double lam[kMaxK + 1];
    double Q[kMaxK * kMaxK];
    double sK[kMaxK * kMaxK];
};
__device__ __forceinline__ void wg_model_update(int k, int kp, int r, const double *__restrict__ st,
                                                const double *__restrict__ VCV, const double *__restrict__ VtPsi,
                                                double *sc, double *__restrict__ Kc, double *__restrict__ Qp,
                                                double *__restrict__ Hsk, ModelWork *w) {
    const double alpha = sc[SC_ALPHA];
    for (int e = threadIdx.x; e < k * k; e += kWG) w->aS[e] = alpha * st[e];
    __syncthreads();
    wg_syev_load(k, w->aS, k, nullptr, &w->ws);
    wg_syev_top(k, k, k, &w->ws, w->lam, w->Q, k);
    __syncthreads();
    for (int e = threadIdx.x; e < k * k; e += kWG) {
        const int i = e / k, j = e - i * k;
        double v = 0.0;
        for (int c = kp; c < k; ++c) v += w->Q[i * k + c] * w->lam[c] * w->Q[j * k + c];
        w->sK[e] = v;
        Kc[e] = v;
    }
    for (int e = threadIdx.x; e < k * kp; e += kWG) {
        const int i = e / kp, c = e - i * kp;
        Qp[e] = w->Q[i * k + c];
    }
    __syncthreads();
    if (Hsk)
        for (int e = threadIdx.x; e < k * r; e += kWG) {
            const int i = e / r, c = e - i * r;
            double v = 0.0;
            for (int a = 0; a < k; ++a) v += w->sK[i * k + a] * VtPsi[a * r + c];
            Hsk[e] = v;
        }
    if (threadIdx.x == 0) {
        const double g = sc[SC_G];
        double trc = 0.0, kv = 0.0;
        for (int c = kp; c < k; ++c) trc += w->lam[c];
        for (int e = 0; e < k * k; ++e) kv += w->sK[e] * VCV[e];
        sc[SC_TAU] = g * sc[SC_TAU] + trc;
        sc[SC_CBAR] = g * sc[SC_CBAR] + kv;
    }
}

}  // namespace usbs
