/* Oracle (test infrastructure only): exact elimination of the matrix cells of
 * a dual-porosity system.
 *
 * In the fractured-reservoir model of Section 2.1 every grid location holds a
 * fracture cell and a matrix cell, and the matrix cell exchanges fluid with
 * its own fracture cell only.  Block row N+g of the Jacobian (the matrix cell
 * of location g) therefore holds two blocks, A_mf at column g and A_mm at
 * column N+g, and fracture row g holds one block A_fm at column N+g besides
 * its stencil and well blocks.  Block Gaussian elimination of every matrix
 * unknown is exact and local:
 *   S_gg = A_ff,gg - A_fm A_mm^{-1} A_mf        (only the diagonal block changes)
 *   b'_g = b_g - A_fm A_mm^{-1} b_m
 *   x_m  = A_mm^{-1} (b_m - A_mf x_g)           (back-substitution)
 * The reduced system, rows = N fracture cells then the fixed-rate well rows,
 * has the single-porosity pattern (7-point stencil plus wells).  Its column
 * indices: fracture cells keep theirs, well row 2N + w becomes N + w.
 *
 * Every 3x3 product below sums in ascending inner index (or_mul3, or_mv3);
 * no operation is fused. */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "bo_oracle.h"
#include "or_internal.h"

/* column of the full system -> column of the reduced one (-1: a matrix cell) */
static int red_col(int N, int c)
{
    if (c < N) return c;
    if (c < 2 * N) return -1;
    return c - N;
}

int or_condense_pattern(int N, int nw, const int32_t *rp, const int32_t *ci, int32_t *srp, int32_t *sci)
{
    int nr = N + nw, cnt = 0;
    if (srp) srp[0] = 0;
    for (int r = 0; r < nr; r++) {
        int i = r < N ? r : N + r;   /* full row of reduced row r */
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            int c = red_col(N, ci[e]);
            if (c < 0) {
                if (r >= N || ci[e] != N + r) return -1;   /* only a fracture row's own matrix cell */
                continue;
            }
            if (sci) sci[cnt] = c;
            cnt++;
        }
        if (srp) srp[r + 1] = cnt;
    }
    return cnt;
}

int or_condense_values(int N, int nw, const int32_t *rp, const int32_t *ci, const double *val,
                       double *sval, double *minv, double *amf, double *wfm)
{
    int nr = N + nw, cnt = 0;
    for (int r = 0; r < nr; r++) {
        int i = r < N ? r : N + r;
        const double *afm = NULL;
        int diag = -1;
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            int c = red_col(N, ci[e]);
            if (c < 0) { afm = val + 9 * (size_t)e; continue; }
            if (c == r) diag = cnt;
            memcpy(sval + 9 * (size_t)cnt, val + 9 * (size_t)e, 9 * sizeof(double));
            cnt++;
        }
        if (r >= N) continue;
        /* matrix row m = N + r: blocks (m, r) and (m, m), in that column order */
        int m = N + r;
        if (!afm || diag < 0 || rp[m + 1] - rp[m] != 2 || ci[rp[m]] != r || ci[rp[m] + 1] != m) return OR_ERR_ARG;
        const double *Amf = val + 9 * (size_t)rp[m], *Amm = val + 9 * (size_t)(rp[m] + 1);
        double *Mi = minv + 9 * (size_t)r, *W = wfm + 9 * (size_t)r, T[9];
        if (or_inv3(Amm, Mi)) return OR_ERR_SINGULAR_BLOCK;
        memcpy(amf + 9 * (size_t)r, Amf, 9 * sizeof(double));
        or_mul3(afm, Mi, W);          /* W = A_fm A_mm^{-1} */
        or_mul3(W, Amf, T);           /* T = W A_mf */
        double *S = sval + 9 * (size_t)diag;
        for (int z = 0; z < 9; z++) S[z] = S[z] - T[z];
    }
    return OR_OK;
}

void or_condense_rhs(int N, int nw, const double *b, const double *wfm, double *br)
{
    for (int r = 0; r < N; r++) {
        double t[3];
        or_mv3(wfm + 9 * (size_t)r, b + 3 * (size_t)(N + r), t);
        for (int q = 0; q < 3; q++) br[3 * (size_t)r + q] = b[3 * (size_t)r + q] - t[q];
    }
    for (int w = 0; w < nw; w++)
        for (int q = 0; q < 3; q++) br[3 * (size_t)(N + w) + q] = b[3 * (size_t)(2 * N + w) + q];
}

void or_condense_back(int N, int nw, const double *b, const double *xr, const double *minv, const double *amf,
                      double *x)
{
    for (int r = 0; r < N; r++) {
        double t[3], u[3];
        for (int q = 0; q < 3; q++) x[3 * (size_t)r + q] = xr[3 * (size_t)r + q];
        or_mv3(amf + 9 * (size_t)r, xr + 3 * (size_t)r, t);
        for (int q = 0; q < 3; q++) u[q] = b[3 * (size_t)(N + r) + q] - t[q];
        or_mv3(minv + 9 * (size_t)r, u, x + 3 * (size_t)(N + r));
    }
    for (int w = 0; w < nw; w++)
        for (int q = 0; q < 3; q++) x[3 * (size_t)(2 * N + w) + q] = xr[3 * (size_t)(N + w) + q];
}
