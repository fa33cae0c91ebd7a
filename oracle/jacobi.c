/*
 * Oracle (test infrastructure only): cyclic Jacobi eigendecomposition of a
 * dense real symmetric matrix in FP64.
 *
 * Used by the CPU oracle of Unified Spectral Bundling with Sketching for every
 * eigenproblem the method poses: lambda_max(C - A^* y) with its top
 * eigenvectors in the penalized dual f(y) (Sec. 3, eq. pen-D), the
 * eigen-split of S (Sec. 3.1, eq. model_update_eigendecomposition) and the
 * small matrices of the Nystrom reconstruction (App. C.1).
 *
 * Method: the classical cyclic-by-row Jacobi iteration.  For each off-diagonal
 * pair (p,q) a plane rotation J = [[c, s], [-s, c]] (in rows/columns p,q) is
 * chosen so that (J^T A J)_pq = 0:
 *     theta = (a_qq - a_pp) / (2 a_pq),
 *     t = sign(theta) / (|theta| + sqrt(theta^2 + 1)),   c = 1/sqrt(1+t^2), s = t c,
 * the smaller of the two roots of t^2 + 2 theta t - 1 = 0, which keeps the
 * rotation angle at most pi/4.  Sweeps repeat until the off-diagonal
 * Frobenius norm is below tol * ||A||_F.  The product of the rotations
 * accumulates the eigenvectors.
 *
 * Only tests, the smoke check and the CPU-baseline leg of the benchmark run
 * this code; the GPU path never links it.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* a:  n*n row-major symmetric input, overwritten (diagonal = eigenvalues).
 * w:  n eigenvalues, sorted in descending order on return.
 * vt: n*n row-major, row i = unit eigenvector for w[i].
 * Returns the number of sweeps used, or -1 if max_sweeps was reached. */
int oracle_jacobi_eigh(int n, double *a, double *w, double *vt, int max_sweeps, double tol)
{
    if (n <= 0) return 0;
    double *v = (double *)malloc(sizeof(double) * (size_t)n * n); /* row i = eigvec i */
    memset(v, 0, sizeof(double) * (size_t)n * n);
    for (int i = 0; i < n; ++i) v[(size_t)i * n + i] = 1.0;

    double fro2 = 0.0;
    for (size_t i = 0; i < (size_t)n * n; ++i) fro2 += a[i] * a[i];
    const double fro = sqrt(fro2);
    int sweeps = 0, converged = 0;

    while (sweeps < max_sweeps) {
        double off2 = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) off2 += a[(size_t)p * n + q] * a[(size_t)p * n + q];
        if (fro == 0.0 || sqrt(2.0 * off2) <= tol * fro) { converged = 1; break; }
        ++sweeps;
        for (int p = 0; p < n - 1; ++p) {
            for (int q = p + 1; q < n; ++q) {
                double *rp = a + (size_t)p * n, *rq = a + (size_t)q * n;
                const double apq = rp[q];
                if (apq == 0.0) continue;
                const double app = rp[p], aqq = rq[q];
                /* a rotation smaller than rounding of both diagonal entries
                 * changes nothing: drop the element instead. */
                if (fabs(apq) < 1e-300 ||
                    (fabs(app) + 100.0 * fabs(apq) == fabs(app) &&
                     fabs(aqq) + 100.0 * fabs(apq) == fabs(aqq))) {
                    rp[q] = 0.0; rq[p] = 0.0;
                    continue;
                }
                const double theta = (aqq - app) / (2.0 * apq);
                double t = 1.0 / (fabs(theta) + sqrt(theta * theta + 1.0));
                if (theta < 0.0) t = -t;
                const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
                /* rows p and q of A J (then mirrored to keep A symmetric) */
                for (int k = 0; k < n; ++k) {
                    if (k == p || k == q) continue;
                    const double akp = rp[k], akq = rq[k];
                    const double nkp = c * akp - s * akq;
                    const double nkq = s * akp + c * akq;
                    rp[k] = nkp; rq[k] = nkq;
                    a[(size_t)k * n + p] = nkp;
                    a[(size_t)k * n + q] = nkq;
                }
                rp[p] = app - t * apq;
                rq[q] = aqq + t * apq;
                rp[q] = 0.0; rq[p] = 0.0;
                /* V <- V J; the rows of v are the columns of V */
                double *vp = v + (size_t)p * n, *vq = v + (size_t)q * n;
                for (int k = 0; k < n; ++k) {
                    const double x = vp[k], y = vq[k];
                    vp[k] = c * x - s * y;
                    vq[k] = s * x + c * y;
                }
            }
        }
    }

    /* sort descending, ties kept in index order */
    int *idx = (int *)malloc(sizeof(int) * n);
    for (int i = 0; i < n; ++i) idx[i] = i;
    for (int i = 1; i < n; ++i) {            /* insertion sort: stable */
        int key = idx[i];
        double kv = a[(size_t)key * n + key];
        int j = i - 1;
        while (j >= 0 && a[(size_t)idx[j] * n + idx[j]] < kv) { idx[j + 1] = idx[j]; --j; }
        idx[j + 1] = key;
    }
    for (int i = 0; i < n; ++i) {
        w[i] = a[(size_t)idx[i] * n + idx[i]];
        memcpy(vt + (size_t)i * n, v + (size_t)idx[i] * n, sizeof(double) * n);
    }
    free(idx);
    free(v);
    return converged ? sweeps : -1;
}
