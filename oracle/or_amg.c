/*
 * Oracle (test infrastructure only): aggregation AMG for the decoupled
 * pressure block.
 *
 * The paper applies BoomerAMG to A_pp inside CPR (Section 3.2).  The stand-in
 * here is smoothed aggregation with a deterministic distance-2 maximal
 * independent set, chosen so that a parallel implementation reaches exactly the
 * same aggregates:
 *   strength     |a_ij|^2 >= theta^2 |a_ii a_jj| in either direction (symmetric)
 *   priorities   (fmix32(i ^ 0x9E3779B9 (l+1)), i), compared lexicographically
 *   MIS-2        synchronous rounds: a node joins when it holds the largest
 *                undecided priority within distance 2; nodes within distance 2
 *                of a new member leave the undecided set
 *   aggregates   roots numbered in index order; neighbours of a root join it;
 *                remaining nodes join the aggregate of their strongest
 *                already-assigned strong neighbour (ties: smaller aggregate id);
 *                nodes without strong neighbours stay unaggregated
 *   prolongator  P = (I - omega D_F^{-1} A_F) P_tent with the weak entries of A
 *                lumped into the diagonal of A_F and omega = (4/3) / rho, rho the
 *                Gershgorin bound of D_F^{-1} A_F
 *   coarse op    A_c = P^T (A P), sums in ascending inner index
 *   cycle        V(s,s) from a zero guess.  Level 0 of a grid: red-black
 *                Gauss-Seidel by (i+j+k) mod 2, red then black before the
 *                coarse correction and black then red after it (or damped
 *                Jacobi); coarser levels: l1-Jacobi, x += (b - A x) / sum_j
 *                |a_ij| (the l1 smoother of hypre's BoomerAMG, the AMG the
 *                paper uses), or damped Jacobi with omega = 2/3; coarsest
 *                level by dense LU with partial pivoting.
 * fmix32 is the public MurmurHash3 finaliser.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "bo_oracle.h"
#include "or_internal.h"
#include "or_amg.h"

void or_csr_free(or_csr *a)
{
    free(a->rp); free(a->ci); free(a->v);
    memset(a, 0, sizeof *a);
}

static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16; h *= 0x85ebca6bu;
    h ^= h >> 13; h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* priority key, never 0 (0 means "none") */
static uint64_t prio(int i, int level)
{
    uint32_t h = fmix32((uint32_t)i ^ (0x9E3779B9u * (uint32_t)(level + 1)));
    return ((((uint64_t)h) << 32) | (uint32_t)i) + 1u;
}

static double entry(const or_csr *A, int i, int j)
{
    for (int e = A->rp[i]; e < A->rp[i + 1]; e++)
        if (A->ci[e] == j) return A->v[e];
    return 0.0;
}

/* per-entry symmetric strength flags (diagonal entries are never strong) */
static void strength(const or_csr *A, double theta, uint8_t *sf)
{
    double t2 = theta * theta;
    for (int i = 0; i < A->n; i++) {
        double aii = entry(A, i, i);
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            int j = A->ci[e];
            if (j == i) { sf[e] = 0; continue; }
            double ajj = entry(A, j, j);
            double aij = A->v[e], aji = entry(A, j, i);
            double thr = t2 * fabs(aii * ajj);
            sf[e] = (aij * aij >= thr) || (aji * aji >= thr);
        }
    }
}

enum { UND = 0, IN = 1, OUT = 2, ISO = 3 };

static void mis2(const or_csr *A, const uint8_t *sf, int level, uint8_t *state)
{
    int n = A->n;
    uint64_t *m1 = malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t *m2 = malloc(sizeof(uint64_t) * (size_t)n);
    uint8_t *nw = malloc((size_t)n), *d1 = malloc((size_t)n);
    for (int i = 0; i < n; i++) {
        int deg = 0;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) deg += sf[e];
        state[i] = deg ? UND : ISO;
    }
    for (;;) {
        int any = 0;
        for (int i = 0; i < n; i++) any |= state[i] == UND;
        if (!any) break;
        for (int i = 0; i < n; i++) {
            uint64_t m = state[i] == UND ? prio(i, level) : 0;
            for (int e = A->rp[i]; e < A->rp[i + 1]; e++)
                if (sf[e] && state[A->ci[e]] == UND) {
                    uint64_t q = prio(A->ci[e], level);
                    if (q > m) m = q;
                }
            m1[i] = m;
        }
        for (int i = 0; i < n; i++) {
            uint64_t m = m1[i];
            for (int e = A->rp[i]; e < A->rp[i + 1]; e++)
                if (sf[e] && m1[A->ci[e]] > m) m = m1[A->ci[e]];
            m2[i] = m;
        }
        for (int i = 0; i < n; i++) nw[i] = state[i] == UND && m2[i] == prio(i, level);
        for (int i = 0; i < n; i++) {
            uint8_t d = nw[i];
            for (int e = A->rp[i]; e < A->rp[i + 1]; e++) if (sf[e]) d |= nw[A->ci[e]];
            d1[i] = d;
        }
        for (int i = 0; i < n; i++) {
            uint8_t d = d1[i];
            for (int e = A->rp[i]; e < A->rp[i + 1]; e++) if (sf[e]) d |= d1[A->ci[e]];
            if (nw[i]) state[i] = IN;
            else if (state[i] == UND && d) state[i] = OUT;
        }
    }
    free(m1); free(m2); free(nw); free(d1);
}

/* returns the number of aggregates */
static int aggregate(const or_csr *A, const uint8_t *sf, const uint8_t *state, int32_t *agg)
{
    int n = A->n, nc = 0;
    int32_t *a1 = malloc(sizeof(int32_t) * (size_t)n);
    for (int i = 0; i < n; i++) a1[i] = -1;
    for (int i = 0; i < n; i++) if (state[i] == IN) a1[i] = nc++;
    for (int i = 0; i < n; i++)
        if (state[i] == IN)
            for (int e = A->rp[i]; e < A->rp[i + 1]; e++) if (sf[e]) a1[A->ci[e]] = a1[i];
    for (int i = 0; i < n; i++) {
        agg[i] = a1[i];
        if (a1[i] >= 0 || state[i] == ISO) continue;
        int best = -1; double bv = -1.0;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            int j = A->ci[e];
            if (!sf[e] || a1[j] < 0) continue;
            double v = fabs(A->v[e]);
            if (v > bv || (v == bv && a1[j] < best)) { bv = v; best = a1[j]; }
        }
        agg[i] = best;
    }
    free(a1);
    return nc;
}

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Gustavson product C = A B, accumulation in ascending inner index, output
 * columns sorted. */
static int spgemm(const or_csr *A, const or_csr *B, or_csr *C)
{
    int n = A->n, m = B->m;
    double *acc = calloc((size_t)m, sizeof(double));
    int32_t *mark = malloc(sizeof(int32_t) * (size_t)m);
    int32_t *cols = malloc(sizeof(int32_t) * (size_t)m);
    if (!acc || !mark || !cols) return OR_ERR_ALLOC;
    for (int j = 0; j < m; j++) mark[j] = -1;
    size_t cap = (size_t)A->nnz + 16, nnz = 0;
    C->n = n; C->m = m;
    C->rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    C->ci = malloc(sizeof(int32_t) * cap);
    C->v = malloc(sizeof(double) * cap);
    C->rp[0] = 0;
    for (int i = 0; i < n; i++) {
        int cnt = 0;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            int k = A->ci[e];
            double a = A->v[e];
            for (int f = B->rp[k]; f < B->rp[k + 1]; f++) {
                int j = B->ci[f];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; cols[cnt++] = j; }
                acc[j] += a * B->v[f];
            }
        }
        qsort(cols, (size_t)cnt, sizeof(int32_t), cmp_i32);
        if (nnz + (size_t)cnt > cap) {
            while (nnz + (size_t)cnt > cap) cap *= 2;
            C->ci = realloc(C->ci, sizeof(int32_t) * cap);
            C->v = realloc(C->v, sizeof(double) * cap);
        }
        for (int t = 0; t < cnt; t++) { C->ci[nnz] = cols[t]; C->v[nnz] = acc[cols[t]]; nnz++; }
        C->rp[i + 1] = (int32_t)nnz;
    }
    C->nnz = (int)nnz;
    free(acc); free(mark); free(cols);
    return OR_OK;
}

static void transpose(const or_csr *A, or_csr *T)
{
    T->n = A->m; T->m = A->n; T->nnz = A->nnz;
    T->rp = calloc((size_t)T->n + 1, sizeof(int32_t));
    T->ci = malloc(sizeof(int32_t) * (size_t)(A->nnz > 0 ? A->nnz : 1));
    T->v = malloc(sizeof(double) * (size_t)(A->nnz > 0 ? A->nnz : 1));
    for (int e = 0; e < A->nnz; e++) T->rp[A->ci[e] + 1]++;
    for (int r = 0; r < T->n; r++) T->rp[r + 1] += T->rp[r];
    int32_t *pos = malloc(sizeof(int32_t) * (size_t)(T->n + 1));
    memcpy(pos, T->rp, sizeof(int32_t) * (size_t)(T->n + 1));
    for (int i = 0; i < A->n; i++)
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            int d = pos[A->ci[e]]++;
            T->ci[d] = i; T->v[d] = A->v[e];
        }
    free(pos);
}

/* smoothed prolongator; returns omega through *omega */
static void prolongator(const or_csr *A, const uint8_t *sf, const int32_t *agg, int nc,
                        or_csr *P, double *omega)
{
    int n = A->n;
    double *aF = malloc(sizeof(double) * (size_t)n);
    double rho = 0.0;
    for (int i = 0; i < n; i++) {
        double d = entry(A, i, i);
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++)
            if (A->ci[e] != i && !sf[e]) d += A->v[e];
        if (d == 0.0) d = entry(A, i, i);
        aF[i] = d;
        double rs = 0.0;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            if (A->ci[e] == i) rs += fabs(d);
            else if (sf[e]) rs += fabs(A->v[e]);
        }
        double ratio = rs / fabs(d);
        if (ratio > rho) rho = ratio;
    }
    double om = (4.0 / 3.0) / rho;
    *omega = om;
    double *s = calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    int32_t *mark = malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    int32_t *cols = malloc(sizeof(int32_t) * (size_t)(nc > 0 ? nc : 1));
    for (int J = 0; J < nc; J++) mark[J] = -1;
    size_t cap = (size_t)A->nnz + 16, nnz = 0;
    P->n = n; P->m = nc;
    P->rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    P->ci = malloc(sizeof(int32_t) * cap);
    P->v = malloc(sizeof(double) * cap);
    P->rp[0] = 0;
    for (int i = 0; i < n; i++) {
        int cnt = 0;
        double d = om / aF[i];
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            int j = A->ci[e];
            if (!(j == i || sf[e]) || agg[j] < 0) continue;
            int J = agg[j];
            double a = (j == i) ? aF[i] : A->v[e];
            if (mark[J] != i) { mark[J] = i; s[J] = 0.0; cols[cnt++] = J; }
            s[J] += a;
        }
        qsort(cols, (size_t)cnt, sizeof(int32_t), cmp_i32);
        for (int t = 0; t < cnt; t++) {
            int J = cols[t];
            P->ci[nnz] = J;
            P->v[nnz] = (agg[i] == J ? 1.0 : 0.0) - d * s[J];
            nnz++;
        }
        P->rp[i + 1] = (int32_t)nnz;
    }
    P->nnz = (int)nnz;
    free(aF); free(s); free(mark); free(cols);
}

/* ---- the setup rules on a caller-given matrix (pins) ----------------------- */
void or_amg_strength_flags(const or_csr *A, double theta, uint8_t *sf) { strength(A, theta, sf); }

/* Aggregates from caller-chosen roots (1 = root): phase 1 and phase 2 of the
 * aggregation with the strength flags of theta; nodes without a strong
 * neighbour stay unaggregated (-1).  Returns the number of aggregates. */
int or_amg_aggregate_roots(const or_csr *A, double theta, const uint8_t *root, int32_t *agg)
{
    int n = A->n;
    uint8_t *sf = malloc((size_t)(A->nnz > 0 ? A->nnz : 1)), *state = malloc((size_t)(n > 0 ? n : 1));
    strength(A, theta, sf);
    for (int i = 0; i < n; i++) {
        int deg = 0;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) deg += sf[e];
        state[i] = root[i] ? IN : (deg ? OUT : ISO);
    }
    int nc = aggregate(A, sf, state, agg);
    free(sf); free(state);
    return nc;
}

void or_amg_free(or_amg *h)
{
    for (int l = 0; l < OR_MAXLEV; l++) {
        or_csr_free(&h->A[l]); or_csr_free(&h->P[l]); or_csr_free(&h->R[l]);
        free(h->agg[l]); free(h->sf[l]); free(h->color[l]); free(h->root[l]);
        free(h->dl1[l]); free(h->dl132[l]);
    }
    for (int l = 0; l < OR_MAXLEV; l++) { free(h->A32[l]); free(h->P32[l]); free(h->R32[l]); }
    free(h->cinv32);
    free(h->dense);
    memset(h, 0, sizeof *h);
}

int or_amg_setup(or_amg *h, const or_csr *A0, int nx, int ny, int nz, double theta,
                 int coarse_max, int max_levels, int smoother, int sweeps, int csmoother)
{
    memset(h, 0, sizeof *h);
    h->smoother = smoother; h->sweeps = sweeps; h->csmoother = csmoother;
    if (max_levels > OR_MAXLEV) max_levels = OR_MAXLEV;
    if (max_levels < 1) max_levels = 1;
    or_csr *A = &h->A[0];
    A->n = A0->n; A->m = A0->m; A->nnz = A0->nnz;
    A->rp = malloc(sizeof(int32_t) * (size_t)(A0->n + 1));
    A->ci = malloc(sizeof(int32_t) * (size_t)A0->nnz);
    A->v = malloc(sizeof(double) * (size_t)A0->nnz);
    memcpy(A->rp, A0->rp, sizeof(int32_t) * (size_t)(A0->n + 1));
    memcpy(A->ci, A0->ci, sizeof(int32_t) * (size_t)A0->nnz);
    memcpy(A->v, A0->v, sizeof(double) * (size_t)A0->nnz);
    int l = 0;
    for (;; l++) {
        or_csr *Al = &h->A[l];
        int n = Al->n;
        h->sf[l] = malloc((size_t)(Al->nnz > 0 ? Al->nnz : 1));
        strength(Al, theta, h->sf[l]);
        if (n <= coarse_max || l + 1 >= max_levels) break;
        uint8_t *state = malloc((size_t)n);
        mis2(Al, h->sf[l], l, state);
        h->agg[l] = malloc(sizeof(int32_t) * (size_t)n);
        int nc = aggregate(Al, h->sf[l], state, h->agg[l]);
        h->root[l] = malloc((size_t)n);
        for (int i = 0; i < n; i++) h->root[l][i] = state[i] == IN;
        free(state);
        if (nc == 0 || (double)nc > 0.8 * (double)n) {
            free(h->agg[l]); h->agg[l] = NULL; free(h->root[l]); h->root[l] = NULL;
            break;
        }
        prolongator(Al, h->sf[l], h->agg[l], nc, &h->P[l], &h->omega[l]);
        transpose(&h->P[l], &h->R[l]);
        or_csr AP;
        int st = spgemm(Al, &h->P[l], &AP);
        if (st) return st;
        st = spgemm(&h->R[l], &AP, &h->A[l + 1]);
        or_csr_free(&AP);
        if (st) return st;
    }
    h->nlev = l + 1;
    /* l1 row norms, ascending column order */
    for (int q = 0; q < h->nlev; q++) {
        const or_csr *Aq = &h->A[q];
        h->dl1[q] = malloc(sizeof(double) * (size_t)(Aq->n > 0 ? Aq->n : 1));
        for (int i = 0; i < Aq->n; i++) {
            double s = 0.0;
            for (int e = Aq->rp[i]; e < Aq->rp[i + 1]; e++) s += fabs(Aq->v[e]);
            h->dl1[q][i] = s;
        }
    }
    /* Gauss-Seidel colours exist only for level 0 of a grid: red-black */
    if (smoother == OR_SMOOTH_GS && nx > 0 && nx * ny * nz == h->A[0].n) {
        int n = h->A[0].n;
        h->color[0] = malloc(sizeof(int32_t) * (size_t)n);
        for (int g = 0; g < n; g++) {
            int i = g % nx, j = (g / nx) % ny, k = g / (nx * ny);
            h->color[0][g] = (i + j + k) & 1;
        }
        h->ncolor[0] = n > 1 ? 2 : 1;
    } else if (smoother == OR_SMOOTH_GS) {
        return OR_ERR_ARG;
    }
    /* coarsest: dense LU when small enough, else smoothing only */
    int nc = h->A[h->nlev - 1].n;
    h->coarse_direct = nc <= OR_DENSE_MAX;
    if (h->coarse_direct) {
        const or_csr *C = &h->A[h->nlev - 1];
        h->dense = calloc((size_t)nc * nc, sizeof(double));
        for (int i = 0; i < nc; i++)
            for (int e = C->rp[i]; e < C->rp[i + 1]; e++) h->dense[(size_t)i * nc + C->ci[e]] = C->v[e];
        /* singular to working precision: a pivot (partial pivoting) at or
         * below 1e-12 of the largest entry (a pure-Neumann pressure block
         * gives about 1e-16 of it) */
        if (!(or_dense_min_pivot_ratio(nc, h->dense) > 1e-12)) return OR_ERR_SINGULAR_COARSE;
    }
    return OR_OK;
}

/* ---- cycle ------------------------------------------------------------- */

static void gs_colour(const or_csr *A, const int32_t *color, int c, const double *b, double *x)
{
    for (int i = 0; i < A->n; i++) {
        if (color[i] != c) continue;
        double s = b[i], d = 0.0;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            int j = A->ci[e];
            if (j == i) d = A->v[e];
            else s -= A->v[e] * x[j];
        }
        x[i] = s / d;
    }
}

static void smooth(const or_amg *h, int l, const double *b, double *x, int forward)
{
    const or_csr *A = &h->A[l];
    int n = A->n;
    int kind = l == 0 ? h->smoother : OR_SMOOTH_JACOBI;
    int l1 = (l > 0 && h->csmoother == OR_CSMOOTH_L1) || (l == 0 && h->smoother == OR_SMOOTH_L1);
    for (int sw = 0; sw < h->sweeps; sw++) {
        if (l1) {
            double *t = malloc(sizeof(double) * (size_t)n);
            for (int i = 0; i < n; i++) {
                double s = 0.0;
                for (int e = A->rp[i]; e < A->rp[i + 1]; e++) s += A->v[e] * x[A->ci[e]];
                t[i] = x[i] + (b[i] - s) / h->dl1[l][i];
            }
            memcpy(x, t, sizeof(double) * (size_t)n);
            free(t);
        } else if (kind == OR_SMOOTH_JACOBI) {
            double *t = malloc(sizeof(double) * (size_t)n);
            for (int i = 0; i < n; i++) {
                double s = 0.0, d = 0.0;
                for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
                    s += A->v[e] * x[A->ci[e]];
                    if (A->ci[e] == i) d = A->v[e];
                }
                t[i] = x[i] + (2.0 / 3.0) * ((b[i] - s) / d);
            }
            memcpy(x, t, sizeof(double) * (size_t)n);
            free(t);
        } else if (forward) {
            for (int c = 0; c < h->ncolor[l]; c++) gs_colour(A, h->color[l], c, b, x);
        } else {
            for (int c = h->ncolor[l] - 1; c >= 0; c--) gs_colour(A, h->color[l], c, b, x);
        }
    }
}

static void csr_mv(const or_csr *A, const double *x, double *y)
{
    for (int i = 0; i < A->n; i++) {
        double s = 0.0;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) s += A->v[e] * x[A->ci[e]];
        y[i] = s;
    }
}

static void vcycle(const or_amg *h, int l, const double *b, double *x)
{
    const or_csr *A = &h->A[l];
    int n = A->n;
    if (l == h->nlev - 1) {
        if (h->coarse_direct) {
            double *M = malloc(sizeof(double) * (size_t)n * n);
            memcpy(M, h->dense, sizeof(double) * (size_t)n * n);
            memcpy(x, b, sizeof(double) * (size_t)n);
            or_dense_solve(n, M, x);
            free(M);
        } else {
            memset(x, 0, sizeof(double) * (size_t)n);
            smooth(h, l, b, x, 1);
            smooth(h, l, b, x, 0);
        }
        return;
    }
    memset(x, 0, sizeof(double) * (size_t)n);
    smooth(h, l, b, x, 1);
    double *r = malloc(sizeof(double) * (size_t)n);
    csr_mv(A, x, r);
    for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
    int nc = h->A[l + 1].n;
    double *bc = malloc(sizeof(double) * (size_t)nc), *xc = malloc(sizeof(double) * (size_t)nc);
    csr_mv(&h->R[l], r, bc);
    vcycle(h, l + 1, bc, xc);
    double *px = malloc(sizeof(double) * (size_t)n);
    csr_mv(&h->P[l], xc, px);
    for (int i = 0; i < n; i++) x[i] = x[i] + px[i];
    smooth(h, l, b, x, 0);
    free(r); free(bc); free(xc); free(px);
}

void or_amg_vcycle(const or_amg *h, const double *b, double *x)
{
    vcycle(h, 0, b, x);
}

/* ---- mixed-precision emulation ------------------------------------------
 * The hierarchy built above (FP64) is stored rounded to FP32 (C's double to
 * float conversion rounds to nearest even); the cycle then runs the same
 * steps as vcycle() with float arithmetic and float vectors.  The coarsest
 * level is solved with the FP32-rounded inverse of the FP64 coarsest matrix
 * (columns of the inverse by dense LU), applied as a float product. */

static float *round_f32(const double *a, size_t n)
{
    float *b = malloc(sizeof(float) * (n ? n : 1));
    for (size_t i = 0; i < n; i++) b[i] = (float)a[i];
    return b;
}

int or_amg_make_f32(or_amg *h)
{
    for (int l = 0; l < h->nlev; l++) {
        h->A32[l] = round_f32(h->A[l].v, (size_t)h->A[l].nnz);
        h->dl132[l] = round_f32(h->dl1[l], (size_t)h->A[l].n);
        if (l < h->nlev - 1) {
            h->P32[l] = round_f32(h->P[l].v, (size_t)h->P[l].nnz);
            h->R32[l] = round_f32(h->R[l].v, (size_t)h->R[l].nnz);
        }
    }
    const or_csr *C = &h->A[h->nlev - 1];
    int n = C->n;
    double *M = malloc(sizeof(double) * (size_t)n * n), *col = malloc(sizeof(double) * (size_t)n);
    h->cinv32 = malloc(sizeof(float) * (size_t)n * n);
    for (int j = 0; j < n; j++) {
        memset(M, 0, sizeof(double) * (size_t)n * n);
        for (int i = 0; i < n; i++)
            for (int e = C->rp[i]; e < C->rp[i + 1]; e++) M[(size_t)i * n + C->ci[e]] = C->v[e];
        memset(col, 0, sizeof(double) * (size_t)n);
        col[j] = 1.0;
        if (or_dense_solve(n, M, col)) { free(M); free(col); return OR_ERR_SINGULAR_COARSE; }
        for (int i = 0; i < n; i++) h->cinv32[(size_t)i * n + j] = (float)col[i];
    }
    free(M); free(col);
    return OR_OK;
}

static void gs_colour_f32(const or_csr *A, const float *v, const int32_t *color, int c, const float *b, float *x)
{
    for (int i = 0; i < A->n; i++) {
        if (color[i] != c) continue;
        float s = b[i], d = 0.0f;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
            int j = A->ci[e];
            if (j == i) d = v[e];
            else s -= v[e] * x[j];
        }
        x[i] = s / d;
    }
}

static void smooth_f32(const or_amg *h, int l, const float *b, float *x, int forward)
{
    const or_csr *A = &h->A[l];
    const float *v = h->A32[l];
    int n = A->n;
    int kind = l == 0 ? h->smoother : OR_SMOOTH_JACOBI;
    int l1 = (l > 0 && h->csmoother == OR_CSMOOTH_L1) || (l == 0 && h->smoother == OR_SMOOTH_L1);
    const float w = (float)(2.0 / 3.0);
    for (int sw = 0; sw < h->sweeps; sw++) {
        if (l1) {
            float *t = malloc(sizeof(float) * (size_t)n);
            for (int i = 0; i < n; i++) {
                float s = 0.0f;
                for (int e = A->rp[i]; e < A->rp[i + 1]; e++) s += v[e] * x[A->ci[e]];
                t[i] = x[i] + (b[i] - s) / h->dl132[l][i];
            }
            memcpy(x, t, sizeof(float) * (size_t)n);
            free(t);
        } else if (kind == OR_SMOOTH_JACOBI) {
            float *t = malloc(sizeof(float) * (size_t)n);
            for (int i = 0; i < n; i++) {
                float s = 0.0f, d = 0.0f;
                for (int e = A->rp[i]; e < A->rp[i + 1]; e++) {
                    s += v[e] * x[A->ci[e]];
                    if (A->ci[e] == i) d = v[e];
                }
                t[i] = x[i] + w * ((b[i] - s) / d);
            }
            memcpy(x, t, sizeof(float) * (size_t)n);
            free(t);
        } else if (forward) {
            for (int c = 0; c < h->ncolor[l]; c++) gs_colour_f32(A, v, h->color[l], c, b, x);
        } else {
            for (int c = h->ncolor[l] - 1; c >= 0; c--) gs_colour_f32(A, v, h->color[l], c, b, x);
        }
    }
}

static void csr_mv_f32(const or_csr *A, const float *v, const float *x, float *y)
{
    for (int i = 0; i < A->n; i++) {
        float s = 0.0f;
        for (int e = A->rp[i]; e < A->rp[i + 1]; e++) s += v[e] * x[A->ci[e]];
        y[i] = s;
    }
}

static void vcycle_f32(const or_amg *h, int l, const float *b, float *x)
{
    const or_csr *A = &h->A[l];
    int n = A->n;
    if (l == h->nlev - 1) {
        for (int i = 0; i < n; i++) {
            float s = 0.0f;
            for (int j = 0; j < n; j++) s += h->cinv32[(size_t)i * n + j] * b[j];
            x[i] = s;
        }
        return;
    }
    memset(x, 0, sizeof(float) * (size_t)n);
    smooth_f32(h, l, b, x, 1);
    float *r = malloc(sizeof(float) * (size_t)n);
    csr_mv_f32(A, h->A32[l], x, r);
    for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
    int nc = h->A[l + 1].n;
    float *bc = malloc(sizeof(float) * (size_t)nc), *xc = malloc(sizeof(float) * (size_t)nc);
    csr_mv_f32(&h->R[l], h->R32[l], r, bc);
    vcycle_f32(h, l + 1, bc, xc);
    float *px = malloc(sizeof(float) * (size_t)n);
    csr_mv_f32(&h->P[l], h->P32[l], xc, px);
    for (int i = 0; i < n; i++) x[i] = x[i] + px[i];
    smooth_f32(h, l, b, x, 0);
    free(r); free(bc); free(xc); free(px);
}

void or_amg_vcycle_f32(const or_amg *h, const float *b, float *x)
{
    vcycle_f32(h, 0, b, x);
}
