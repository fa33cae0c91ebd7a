// Packed execution of many USBS instances in one persistent launch: one
// workgroup per instance runs whole iterations of Alg. 1 (operator shift,
// block Lanczos with restarts, master QP, model and sketch update, stopping
// test) with every decision taken on the device, so a launch of G workgroups
// advances G independent solves with no host round trip.  The instances'
// data and state stay in the buffers their handles own; the descriptor table
// only carries sizes, parameters and pointers.
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>
#include "kernels.h"

namespace usbs {

struct PackDesc {
    // sizes and parameters
    int n, m, k, kc, kp, r, steps, ldb, prec;
    int n_iso, n_offt, has_ineq, sketch;
    int max_restarts, max_iters;
    double val_scale, tol, tol_rest, tol_final, alpha, rho, eps_gap, eps_inf;
    uint64_t seed;
    // operator: off-diagonal CSR (values in the compute precision), diagonal apart
    const int *rowptr, *col;
    void *val_cur;
    const void *val_c;
    const double *cbase, *cdiag;
    double *dshift;
    const int *dptr, *dk;
    const double *dv;
    const int *off_slot, *off_ptr, *off_k;
    const double *off_hv;
    // constraint rows (CSR over triplets), b, inequality mask, test matrix
    const int *kptr, *ti, *tj;
    const double *tv, *b, *ineq;
    const float *psi;
    // iteration state and work arrays (layouts as in the per-instance path)
    double *y, *yc, *nu, *dnu, *zbar, *AX, *evec;
    double *V, *Vn, *CV, *Uritz, *P, *Ucpl;
    const int *iso_idx;
    int *plan;
    double *Bm, *W, *Wt, *W2, *Ubuf, *Zp;
    double *Tm, *theta, *Ysm, *TUU, *RtR, *Zc, *Hred, *Hg, *coef, *Rsv, *Rinv, *res, *Hd;
    int *dead, *flag, *zdead;
    double *raw, *qp, *ipm, *VCV, *Gy, *Kc, *Qp, *Hsk, *VtPsi, *hz, *sc;
};

// what a launch does first for an instance
enum PackInit {
    PACK_INIT_NONE = 0,
    PACK_INIT_COLD = 1,   // cold start: y0 = 0, V0 = top-k eigenvectors of C_s, f(y0)
    PACK_INIT_WARM = 2,   // f(y0) of a warm-started instance (state already padded)
};
// how an instance's solve ended
enum PackDone {
    PACK_RUNNING = 0,
    PACK_CONVERGED = 1,   // both relative errors <= eps after the certifying eigen-solve
    PACK_LIMIT = 2,       // iteration limit or host stop request
    PACK_FAILED = -1,     // non-finite iterate or failed interior point solve
};

// phases of the packed kernel timed with the device wall clock (usbs_packed_profile)
enum PackPhase {
    PH_SPMM = 0,     // products with the shifted operator / with C
    PH_TN,           // tall-skinny reductions A^T B on the matrix cores
    PH_NN,           // tall-skinny updates C = [A A2] H on the matrix cores
    PH_RITZ,         // projected (Rayleigh-Ritz) eigenproblems
    PH_IPM,          // master-QP interior point method
    PH_CONSTR,       // constraint side: QP Gram sums, A on low-rank factors, dot products, candidate
    PH_SMALL,        // small dense steps: Gram-Schmidt Cholesky, restart block, model update, f^
    PH_OTHER,        // operator shift and Gershgorin bound
    PH_ALL,          // the whole launch (the rest: copies, fills, random directions, scalars)
    kPackPhases
};

// counters carried across launches (host <-> device), one per instance
struct PackState {
    int iters;            // iterations of Alg. 1 over the handle's life (seeds random directions)
    int solve_iters;      // iterations of the current solve
    int null_run;         // consecutive null steps
    int lz_unconverged;   // in-iteration eigen-solves that hit the restart limit
    int recoveries;       // stall re-evaluations of f at the centre
    int done;             // PackDone
    int swapped;          // V and Vn exchanged an odd number of times in the last launch
    int init;             // PackInit, cleared by the launch
    int stop;             // host request: certify f at the centre and stop
    int pad;
    long long matvecs;    // columns multiplied by the shifted operator
    unsigned long long ticks[kPackPhases];   // device wall-clock ticks spent per PackPhase
};

// Largest LDS footprint of the packed kernel (bytes), for the launch check.
size_t packed_lds_bytes();
// One launch: every instance of desc_dev[0..count) runs its pending init step and
// then up to 'iters' iterations (fewer once it is done).  desc_dev and state_dev are
// device arrays.
void packed_launch(hipStream_t s, const PackDesc *desc_dev, PackState *state_dev, int count, int iters);

}  // namespace usbs
