/*
 * Oracle (test infrastructure only): sparse and dense linear-algebra basics.
 *
 * - y = alpha A x + beta y, the first basic operation listed in Section 3.3;
 * - dense LU with partial pivoting (textbook Gaussian elimination);
 * - quasi-IMPES decoupling of Section 3.2.  The printed operator combines
 *   the pressure row with the secondary rows through D_ps D_ss^{-1}, where D_ps
 *   and D_ss are diagonals of A_ps and A_ss; the effective row operation is
 *   p-row minus D_ps D_ss^{-1} times the s-rows.  Two forms are offered: the
 *   pointwise diagonals of the cell's block (the literal operator), and the
 *   cell's full 2x2 saturation block (which zeroes the decoupled pressure
 *   row's saturation coefficients exactly).  The oil equation is the pressure
 *   row.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "bo_oracle.h"
#include "or_internal.h"

void or_bsr_spmv(int n, int bs, const int32_t *rowptr, const int32_t *colind, const double *val,
                 double alpha, const double *x, double beta, double *y)
{
    int b2 = bs * bs;
    for (int i = 0; i < n; i++) {
        for (int r = 0; r < bs; r++) {
            double s = 0.0;
            for (int e = rowptr[i]; e < rowptr[i + 1]; e++) {
                const double *blk = val + (size_t)b2 * e;
                const double *xj = x + (size_t)bs * colind[e];
                for (int c = 0; c < bs; c++) s += blk[bs * r + c] * xj[c];
            }
            double yi = beta == 0.0 ? 0.0 : beta * y[(size_t)bs * i + r];
            y[(size_t)bs * i + r] = alpha * s + yi;
        }
    }
}

int or_dense_solve(int n, double *A, double *b)
{
    for (int k = 0; k < n; k++) {
        int piv = k;
        double best = fabs(A[(size_t)k * n + k]);
        for (int r = k + 1; r < n; r++) {
            double v = fabs(A[(size_t)r * n + k]);
            if (v > best) { best = v; piv = r; }
        }
        if (best == 0.0) return OR_ERR_SINGULAR_BLOCK;
        if (piv != k) {
            for (int c = 0; c < n; c++) {
                double t = A[(size_t)k * n + c];
                A[(size_t)k * n + c] = A[(size_t)piv * n + c];
                A[(size_t)piv * n + c] = t;
            }
            double t = b[k]; b[k] = b[piv]; b[piv] = t;
        }
        for (int r = k + 1; r < n; r++) {
            double f = A[(size_t)r * n + k] / A[(size_t)k * n + k];
            if (f == 0.0) continue;
            for (int c = k; c < n; c++) A[(size_t)r * n + c] -= f * A[(size_t)k * n + c];
            b[r] -= f * b[k];
        }
    }
    for (int k = n - 1; k >= 0; k--) {
        double s = b[k];
        for (int c = k + 1; c < n; c++) s -= A[(size_t)k * n + c] * b[c];
        b[k] = s / A[(size_t)k * n + k];
    }
    return OR_OK;
}

/* Inverse of a 3x3 block by Gauss-Jordan elimination with partial pivoting.
 * Returns OR_ERR_SINGULAR_BLOCK when a pivot is (numerically) zero relative to
 * the block's largest entry. */
int or_inv3(const double *A, double *Ainv)
{
    double M[3][6];
    double amax = 0.0;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            M[r][c] = A[3 * r + c];
            M[r][3 + c] = (r == c) ? 1.0 : 0.0;
            if (fabs(A[3 * r + c]) > amax) amax = fabs(A[3 * r + c]);
        }
    if (!(amax > 0.0) || !isfinite(amax)) return OR_ERR_SINGULAR_BLOCK;
    for (int k = 0; k < 3; k++) {
        int piv = k;
        for (int r = k + 1; r < 3; r++)
            if (fabs(M[r][k]) > fabs(M[piv][k])) piv = r;
        if (fabs(M[piv][k]) <= 1e-300 * amax) return OR_ERR_SINGULAR_BLOCK;
        if (piv != k)
            for (int c = 0; c < 6; c++) { double t = M[k][c]; M[k][c] = M[piv][c]; M[piv][c] = t; }
        double d = M[k][k];
        for (int c = 0; c < 6; c++) M[k][c] /= d;
        for (int r = 0; r < 3; r++) {
            if (r == k) continue;
            double f = M[r][k];
            for (int c = 0; c < 6; c++) M[r][c] -= f * M[k][c];
        }
    }
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) Ainv[3 * r + c] = M[r][3 + c];
    return OR_OK;
}

/* C = A * B for 3x3 blocks */
/* Smallest |pivot| of LU with partial pivoting relative to the largest
 * |a_ij| (A row-major n x n, not modified); 0 for a zero matrix. */
double or_dense_min_pivot_ratio(int n, const double *A)
{
    double *M = malloc(sizeof(double) * (size_t)n * n);
    memcpy(M, A, sizeof(double) * (size_t)n * n);
    double amax = 0.0, pmin = INFINITY;
    for (size_t e = 0; e < (size_t)n * n; e++) if (fabs(M[e]) > amax) amax = fabs(M[e]);
    for (int k = 0; k < n; k++) {
        int p = k;
        for (int r = k + 1; r < n; r++) if (fabs(M[(size_t)r * n + k]) > fabs(M[(size_t)p * n + k])) p = r;
        double pv = fabs(M[(size_t)p * n + k]);
        if (pv < pmin) pmin = pv;
        if (pv == 0.0) break;
        if (p != k)
            for (int c = 0; c < n; c++) { double t = M[(size_t)k * n + c]; M[(size_t)k * n + c] = M[(size_t)p * n + c]; M[(size_t)p * n + c] = t; }
        for (int r = k + 1; r < n; r++) {
            double f = M[(size_t)r * n + k] / M[(size_t)k * n + k];
            for (int c = k; c < n; c++) M[(size_t)r * n + c] -= f * M[(size_t)k * n + c];
        }
    }
    free(M);
    return amax > 0.0 ? pmin / amax : 0.0;
}

void or_mul3(const double *A, const double *B, double *C)
{
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s += A[3 * r + k] * B[3 * k + c];
            C[3 * r + c] = s;
        }
}

/* y = A x for a 3x3 block */
void or_mv3(const double *A, const double *x, double *y)
{
    for (int r = 0; r < 3; r++) y[r] = A[3 * r] * x[0] + A[3 * r + 1] * x[1] + A[3 * r + 2] * x[2];
}

int or_qi_decouple(int n, const int32_t *rowptr, const int32_t *colind, const double *val,
                   int mode, double *cw, double *app)
{
    for (int i = 0; i < n; i++) {
        const double *B = NULL;
        for (int e = rowptr[i]; e < rowptr[i + 1]; e++)
            if (colind[e] == i) B = val + 9 * (size_t)e;
        if (!B) return OR_ERR_ARG;
        double a = B[4], b = B[5], c = B[7], d = B[8];
        double p0 = B[1], p1 = B[2];
        double w0, w1;
        if (mode == OR_QI_DIAG) {
            /* pointwise diagonals: w_i = D_ps D_ss^{-1} */
            if (a == 0.0 || d == 0.0) return OR_ERR_SINGULAR_BLOCK;
            w0 = p0 / a;
            w1 = p1 / d;
        } else {
            /* w_i solves w_i a_ss = a_ps with a_ps = B[0,1:3], a_ss = B[1:3,1:3] */
            double det = a * d - b * c;
            if (det == 0.0 || !isfinite(det)) return OR_ERR_SINGULAR_BLOCK;
            w0 = (p0 * d - p1 * c) / det;
            w1 = (p1 * a - p0 * b) / det;
        }
        /* c_i = s (1, -w0, -w1); a decoupled row may be scaled by -1, and s keeps
         * the decoupled pressure diagonal c_i . A_ii[:,0] positive */
        double dpp = B[0] - w0 * B[3] - w1 * B[6];
        double sg = dpp < 0.0 ? -1.0 : 1.0;
        cw[3 * i] = sg;
        cw[3 * i + 1] = -sg * w0;
        cw[3 * i + 2] = -sg * w1;
        for (int e = rowptr[i]; e < rowptr[i + 1]; e++) {
            const double *A = val + 9 * (size_t)e;
            app[e] = cw[3 * i] * A[0] + cw[3 * i + 1] * A[3] + cw[3 * i + 2] * A[6];
        }
    }
    return OR_OK;
}
