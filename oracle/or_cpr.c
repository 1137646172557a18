/*
 * Oracle (test infrastructure only): CPR preconditioner and flexible GMRES.
 *
 * F stage (Section 3.2): the paper's RAS with an ILU(0) local solver; on one
 * device this is block ILU(0) of the whole matrix in a chosen ordering
 * (natural, red-black by (i+j+k) mod 2, or tiles of tx x ty columns with the
 * couplings between tiles dropped, i.e. non-overlapping subdomains), or block
 * Jacobi.  Block ILU(0) is written here in its general IKJ form on the block
 * pattern; it runs on the original matrix A because block ILU(0) commutes with
 * left block-diagonal scaling, so applying it to D^{-1}A and D^{-1}r gives the
 * same result.
 *
 * P stage: quasi-IMPES restriction r_p = c_i . (r_o, r_w, r_g), one V-cycle on
 * the decoupled pressure block, prolongation into the pressure slot.
 *
 * Two-stage PF: x1 = Pi_p V(Pi_r v); x = x1 + F(v - A x1).
 * Algorithm CPR-FPF: x = F(v); x += Pi_p V(Pi_r (v - A x)); x += F(v - A x).
 *
 * FGMRES(m) (Saad's flexible variant, right preconditioning) runs on the
 * original system, so its implicit residual is the true residual of A x = b;
 * Givens rotations c = h_jj / hypot, s = h_j+1,j / hypot; the iteration count
 * is the number of preconditioner applications.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "bo_oracle.h"
#include "or_internal.h"
#include "or_amg.h"

struct or_cpr {
    int n;                       /* block rows (cells) */
    or_cpr_opts o;
    int32_t *rp, *ci;            /* copy of A's pattern */
    double *Aval;                /* copy of A's values */
    double *cw;                  /* decoupling rows c_i, 3N */
    or_amg amg;
    int has_amg;
    /* F stage */
    double *LU;                  /* ILU factors on the pattern (nnzb*9) */
    double *inv;                 /* N*9: inverse pivots (ILU) or diagonal blocks (BJ) */
    int32_t *rank, *order;       /* ILU ordering */
    uint8_t *drop;               /* per entry: coupling dropped by tiling */
    int32_t *diag;               /* entry index of the diagonal block per row */
    int npr;                     /* rows of the pressure system */
    /* mixed-precision emulation */
    float *inv32;                /* N*9: rounded pivots (ILU) or diagonal inverses (BJ) */
    float *A32;                  /* nnzb*9: rounded blocks of A (ILU, dropped ones zero) */
};

float or_bf16_round(float f)
{
    if (f == 0.0f || !isfinite(f)) return f;
    int e;
    float fr = frexpf(f, &e);                     /* f = fr 2^e, 0.5 <= |fr| < 1 */
    return ldexpf(rintf(ldexpf(fr, 8)), e - 8);   /* 8 significant bits, ties to even */
}

static float store_round(const or_cpr *c, double v, int bf16_ok)
{
    float f = (float)v;
    return (bf16_ok && c->o.precision == OR_PREC_FP32_BF16) ? or_bf16_round(f) : f;
}

/* rounded copies of the F stage's factors (and of the AMG hierarchy) */
static int mixed_setup(or_cpr *c)
{
    int n = c->n, nnzb = c->rp[n];
    c->inv32 = malloc(sizeof(float) * 9 * (size_t)n);
    for (size_t e = 0; e < 9 * (size_t)n; e++) c->inv32[e] = store_round(c, c->inv[e], 1);
    if (c->o.ftype != OR_F_BJ) {
        c->A32 = malloc(sizeof(float) * 9 * (size_t)(nnzb > 0 ? nnzb : 1));
        for (int e = 0; e < nnzb; e++)
            for (int z = 0; z < 9; z++)
                c->A32[9 * (size_t)e + z] = c->drop[e] ? 0.0f : store_round(c, c->Aval[9 * (size_t)e + z], 1);
    }
    if (c->has_amg) {
        if (!c->amg.coarse_direct) return OR_ERR_ARG;
        return or_amg_make_f32(&c->amg);
    }
    return OR_OK;
}

static void mv3f(const float *A, const float *x, float *y)
{
    y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    y[1] = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    y[2] = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
}

/* F stage in float: x = F(r).  Block Jacobi: x_i = E_i^{-1} r_i.  Block
 * ILU(0) in its diagonal form: w_i = E_i^{-1}(r_i - sum_{k in L(i)} A_ik w_k)
 * in order, then x_i = w_i - E_i^{-1} sum_{j in U(i)} A_ij x_j in reverse
 * order, neighbours in ascending column order. */
static void fstage_f32(const or_cpr *c, const float *r, float *x)
{
    int n = c->n;
    if (c->o.ftype == OR_F_BJ) {
        for (int i = 0; i < n; i++) mv3f(c->inv32 + 9 * (size_t)i, r + 3 * (size_t)i, x + 3 * (size_t)i);
        return;
    }
    float *w = malloc(sizeof(float) * 3 * (size_t)n);
    for (int ps = 0; ps < n; ps++) {
        int i = c->order[ps];
        float v[3] = { r[3 * i], r[3 * i + 1], r[3 * i + 2] }, t[3];
        for (int e = c->rp[i]; e < c->rp[i + 1]; e++) {
            int k = c->ci[e];
            if (c->drop[e] || c->rank[k] >= c->rank[i]) continue;
            mv3f(c->A32 + 9 * (size_t)e, w + 3 * (size_t)k, t);
            for (int q = 0; q < 3; q++) v[q] = v[q] - t[q];
        }
        mv3f(c->inv32 + 9 * (size_t)i, v, w + 3 * (size_t)i);
    }
    for (int ps = n - 1; ps >= 0; ps--) {
        int i = c->order[ps];
        float acc[3] = { 0.0f, 0.0f, 0.0f }, t[3];
        for (int e = c->rp[i]; e < c->rp[i + 1]; e++) {
            int j = c->ci[e];
            if (c->drop[e] || c->rank[j] <= c->rank[i]) continue;
            mv3f(c->A32 + 9 * (size_t)e, x + 3 * (size_t)j, t);
            for (int q = 0; q < 3; q++) acc[q] = acc[q] + t[q];
        }
        mv3f(c->inv32 + 9 * (size_t)i, acc, t);
        for (int q = 0; q < 3; q++) x[3 * i + q] = w[3 * i + q] - t[q];
    }
    free(w);
}

/* F stage at the mixed form's boundary: FP64 r in, rounded, FP64 out */
static void fstage_mixed(const or_cpr *c, const double *r, double *x)
{
    size_t len = 3 * (size_t)c->n;
    float *rf = malloc(sizeof(float) * len), *xf = malloc(sizeof(float) * len);
    for (size_t e = 0; e < len; e++) rf[e] = (float)r[e];
    fstage_f32(c, rf, xf);
    for (size_t e = 0; e < len; e++) x[e] = (double)xf[e];
    free(rf); free(xf);
}

static int grid_cell(const or_problem *p, int g, int *i, int *j, int *k)
{
    *i = g % p->nx; *j = (g / p->nx) % p->ny; *k = g / (p->nx * p->ny);
    return 0;
}

static int ilu_setup(or_cpr *c, const or_problem *p)
{
    int n = c->n, nnzb = c->rp[n];
    c->rank = malloc(sizeof(int32_t) * (size_t)n);
    c->order = malloc(sizeof(int32_t) * (size_t)n);
    c->drop = calloc((size_t)nnzb, 1);
    c->LU = malloc(sizeof(double) * 9 * (size_t)nnzb);
    c->inv = malloc(sizeof(double) * 9 * (size_t)n);
    /* a grid's cells, or (dual porosity / fixed-rate wells) the fracture cells
     * 0..N-1, matrix cells N..2N-1 paired with fracture cell g - N, and well
     * rows after the cells */
    int N = p ? p->nx * p->ny * p->nz : 0;
    int ncell = 0, rows = p ? or_rows(p, &ncell) : 0;
    int grid = p && (N == n || (rows == n && ncell >= N));
    if (c->o.ftype != OR_F_ILU_NATURAL && !grid) return OR_ERR_ARG;
    /* ordering key: (class, g) with class = colour or tile; a matrix cell takes
     * its fracture cell's class (so it follows the tile's fracture cells), the
     * well rows form one class of their own after every tile */
    int32_t *cls = calloc((size_t)n, sizeof(int32_t));
    int ntiles = 0;
    if (grid && c->o.ftype == OR_F_ILU_TILED)
        ntiles = ((p->nx + c->o.tile_x - 1) / c->o.tile_x) * ((p->ny + c->o.tile_y - 1) / c->o.tile_y);
    for (int g = 0; g < n; g++) {
        int i, j, k;
        if (!grid) { cls[g] = 0; continue; }
        if (g >= (ncell > N ? ncell : N)) { cls[g] = c->o.ftype == OR_F_ILU_TILED ? ntiles : 2; continue; }
        int gg = g < N ? g : g - N;
        grid_cell(p, gg, &i, &j, &k);
        if (c->o.ftype == OR_F_ILU_RB) cls[g] = (i + j + k) & 1;
        else if (c->o.ftype == OR_F_ILU_TILED) {
            int ntx = (p->nx + c->o.tile_x - 1) / c->o.tile_x;
            cls[g] = i / c->o.tile_x + ntx * (j / c->o.tile_y);
        } else cls[g] = 0;
    }
    int ncls = 0;
    for (int g = 0; g < n; g++) if (cls[g] + 1 > ncls) ncls = cls[g] + 1;
    int pos = 0;
    for (int q = 0; q < ncls; q++)
        for (int g = 0; g < n; g++)
            if (cls[g] == q) { c->order[pos] = g; c->rank[g] = pos; pos++; }
    if (c->o.ftype == OR_F_ILU_TILED)
        for (int i = 0; i < n; i++)
            for (int e = c->rp[i]; e < c->rp[i + 1]; e++) c->drop[e] = cls[i] != cls[c->ci[e]];
    free(cls);
    memcpy(c->LU, c->Aval, sizeof(double) * 9 * (size_t)nnzb);
    for (int e = 0; e < nnzb; e++)
        if (c->drop[e]) memset(c->LU + 9 * (size_t)e, 0, 9 * sizeof(double));
    /* IKJ block ILU(0) in rank order */
    int maxrow = 1;
    for (int i = 0; i < n; i++) if (c->rp[i + 1] - c->rp[i] > maxrow) maxrow = c->rp[i + 1] - c->rp[i];
    int32_t *low = malloc(sizeof(int32_t) * (size_t)maxrow);
    for (int ps = 0; ps < n; ps++) {
        int i = c->order[ps];
        int nl = 0;
        for (int e = c->rp[i]; e < c->rp[i + 1]; e++)
            if (!c->drop[e] && c->rank[c->ci[e]] < c->rank[i]) low[nl++] = e;
        /* ascending rank of the column */
        for (int a = 1; a < nl; a++) {
            int t = low[a], b = a - 1;
            while (b >= 0 && c->rank[c->ci[low[b]]] > c->rank[c->ci[t]]) { low[b + 1] = low[b]; b--; }
            low[b + 1] = t;
        }
        for (int q = 0; q < nl; q++) {
            int ek = low[q], k = c->ci[ek];
            double L[9];
            or_mul3(c->LU + 9 * (size_t)ek, c->inv + 9 * (size_t)k, L);
            memcpy(c->LU + 9 * (size_t)ek, L, sizeof L);
            for (int ej = c->rp[i]; ej < c->rp[i + 1]; ej++) {
                int j = c->ci[ej];
                if (c->drop[ej] || c->rank[j] <= c->rank[k]) continue;
                for (int f = c->rp[k]; f < c->rp[k + 1]; f++) {
                    if (c->ci[f] != j || c->drop[f]) continue;
                    double t[9];
                    or_mul3(L, c->LU + 9 * (size_t)f, t);
                    for (int z = 0; z < 9; z++) c->LU[9 * (size_t)ej + z] -= t[z];
                }
            }
        }
        if (or_inv3(c->LU + 9 * (size_t)c->diag[i], c->inv + 9 * (size_t)i)) {
            free(low);
            return OR_ERR_SINGULAR_BLOCK;
        }
    }
    free(low);
    return OR_OK;
}

int or_cpr_fstage(or_cpr *c, const double *r, double *x)
{
    int n = c->n;
    if (c->o.precision != OR_PREC_FP64) {
        fstage_mixed(c, r, x);
        return OR_OK;
    }
    if (c->o.ftype == OR_F_BJ) {
        for (int i = 0; i < n; i++) or_mv3(c->inv + 9 * (size_t)i, r + 3 * (size_t)i, x + 3 * (size_t)i);
        return OR_OK;
    }
    double *y = malloc(sizeof(double) * 3 * (size_t)n);
    for (int ps = 0; ps < n; ps++) {
        int i = c->order[ps];
        double s[3] = { r[3 * i], r[3 * i + 1], r[3 * i + 2] };
        for (int e = c->rp[i]; e < c->rp[i + 1]; e++) {
            int k = c->ci[e];
            if (c->drop[e] || c->rank[k] >= c->rank[i]) continue;
            double t[3];
            or_mv3(c->LU + 9 * (size_t)e, y + 3 * (size_t)k, t);
            for (int q = 0; q < 3; q++) s[q] -= t[q];
        }
        memcpy(y + 3 * (size_t)i, s, sizeof s);
    }
    for (int ps = n - 1; ps >= 0; ps--) {
        int i = c->order[ps];
        double s[3] = { y[3 * i], y[3 * i + 1], y[3 * i + 2] };
        for (int e = c->rp[i]; e < c->rp[i + 1]; e++) {
            int j = c->ci[e];
            if (c->drop[e] || c->rank[j] <= c->rank[i]) continue;
            double t[3];
            or_mv3(c->LU + 9 * (size_t)e, x + 3 * (size_t)j, t);
            for (int q = 0; q < 3; q++) s[q] -= t[q];
        }
        or_mv3(c->inv + 9 * (size_t)i, s, x + 3 * (size_t)i);
    }
    free(y);
    return OR_OK;
}

int or_cpr_setup(const or_problem *p, int n, const int32_t *rowptr, const int32_t *colind,
                 const double *val, const or_cpr_opts *o, or_cpr **out)
{
    *out = NULL;
    if (n <= 0 || !rowptr || !colind || !val || !o) return OR_ERR_ARG;
    or_cpr *c = calloc(1, sizeof *c);
    if (!c) return OR_ERR_ALLOC;
    c->n = n; c->o = *o;
    int nnzb = rowptr[n];
    c->rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    c->ci = malloc(sizeof(int32_t) * (size_t)(nnzb > 0 ? nnzb : 1));
    memcpy(c->rp, rowptr, sizeof(int32_t) * (size_t)(n + 1));
    memcpy(c->ci, colind, sizeof(int32_t) * (size_t)nnzb);
    c->Aval = malloc(sizeof(double) * 9 * (size_t)nnzb);
    memcpy(c->Aval, val, sizeof(double) * 9 * (size_t)nnzb);
    for (size_t e = 0; e < 9 * (size_t)nnzb; e++)
        if (!isfinite(val[e])) { or_cpr_free(c); return OR_ERR_NONFINITE; }
    c->diag = malloc(sizeof(int32_t) * (size_t)n);
    for (int i = 0; i < n; i++) {
        c->diag[i] = -1;
        for (int e = rowptr[i]; e < rowptr[i + 1]; e++) if (colind[e] == i) c->diag[i] = e;
        if (c->diag[i] < 0) { or_cpr_free(c); return OR_ERR_ARG; }
    }
    c->cw = malloc(sizeof(double) * 3 * (size_t)n);
    double *app = malloc(sizeof(double) * (size_t)nnzb);
    int st = or_qi_decouple(n, rowptr, colind, val, o->qi_mode, c->cw, app);
    if (st) { free(app); or_cpr_free(c); return st; }
    int npr = o->npr > 0 && o->npr < n ? o->npr : n;
    c->npr = npr;
    if (o->use_amg) {
        /* A_pp: the first npr rows and columns of the decoupled pressure block */
        int32_t *prp = malloc(sizeof(int32_t) * (size_t)(npr + 1)), *pci = malloc(sizeof(int32_t) * (size_t)nnzb);
        double *pv = malloc(sizeof(double) * (size_t)nnzb);
        int cnt = 0;
        prp[0] = 0;
        for (int i = 0; i < npr; i++) {
            for (int e = rowptr[i]; e < rowptr[i + 1]; e++)
                if (colind[e] < npr) { pci[cnt] = colind[e]; pv[cnt] = app[e]; cnt++; }
            prp[i + 1] = cnt;
        }
        or_csr A0 = { npr, npr, cnt, prp, pci, pv };
        int grid = p && p->nx * p->ny * p->nz == npr;
        int nx = grid ? p->nx : 0, ny = grid ? p->ny : 0, nz = grid ? p->nz : 0;
        st = or_amg_setup(&c->amg, &A0, nx, ny, nz, o->theta, o->coarse_max, o->max_levels,
                          o->smoother, o->sweeps, o->csmoother);
        free(prp); free(pci); free(pv);
        c->has_amg = 1;
        if (st) { free(app); or_cpr_free(c); return st; }
    }
    free(app);
    if (o->ftype == OR_F_BJ) {
        c->inv = malloc(sizeof(double) * 9 * (size_t)n);
        for (int i = 0; i < n; i++)
            if (or_inv3(val + 9 * (size_t)c->diag[i], c->inv + 9 * (size_t)i)) {
                or_cpr_free(c);
                return OR_ERR_SINGULAR_BLOCK;
            }
    } else {
        st = ilu_setup(c, p);
        if (st) { or_cpr_free(c); return st; }
    }
    if (o->precision != OR_PREC_FP64) {
        if (o->precision != OR_PREC_FP32 && o->precision != OR_PREC_FP32_BF16) { or_cpr_free(c); return OR_ERR_ARG; }
        st = mixed_setup(c);
        if (st) { or_cpr_free(c); return st; }
    }
    *out = c;
    return OR_OK;
}

/* A handle holding only the AMG hierarchy of a caller-given scalar CSR
 * matrix (l1-Jacobi smoothing, no grid): the hierarchy getters and
 * or_cpr_vcycle work on it. */
int or_amg_only(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double theta,
                int coarse_max, int max_levels, int keep_singular, or_cpr **out)
{
    *out = NULL;
    or_cpr *c = calloc(1, sizeof *c);
    if (!c) return OR_ERR_ALLOC;
    c->n = n;
    c->npr = n;
    c->o.precision = OR_PREC_FP64;
    or_csr A0 = { n, n, rowptr[n], (int32_t *)rowptr, (int32_t *)colind, (double *)val };
    int st = or_amg_setup(&c->amg, &A0, 0, 0, 0, theta, coarse_max, max_levels, OR_SMOOTH_L1, 1, OR_CSMOOTH_L1);
    c->has_amg = 1;
    /* the hierarchy is complete when only the coarsest matrix is singular */
    if (st && !(keep_singular && st == OR_ERR_SINGULAR_COARSE)) { or_cpr_free(c); return st; }
    *out = c;
    return st;
}

int or_amg_strength(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double theta,
                    uint8_t *sf)
{
    or_csr A = { n, n, rowptr[n], (int32_t *)rowptr, (int32_t *)colind, (double *)val };
    or_amg_strength_flags(&A, theta, sf);
    return OR_OK;
}

int or_amg_aggregate(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double theta,
                     const uint8_t *root, int32_t *agg)
{
    or_csr A = { n, n, rowptr[n], (int32_t *)rowptr, (int32_t *)colind, (double *)val };
    return or_amg_aggregate_roots(&A, theta, root, agg);
}

void or_cpr_free(or_cpr *c)
{
    if (!c) return;
    if (c->has_amg) or_amg_free(&c->amg);
    free(c->Aval); free(c->cw); free(c->LU); free(c->inv); free(c->rank); free(c->order);
    free(c->drop); free(c->diag); free(c->rp); free(c->ci);
    free(c->inv32); free(c->A32);
    free(c);
}

int or_cpr_restrict(or_cpr *c, const double *v, double *rp)
{
    for (int i = 0; i < c->npr; i++)
        rp[i] = c->cw[3 * i] * v[3 * i] + c->cw[3 * i + 1] * v[3 * i + 1] + c->cw[3 * i + 2] * v[3 * i + 2];
    return OR_OK;
}

/* one V-cycle; in the mixed form b is rounded to float on entry and the
 * float result is returned exactly */
static void vcycle_any(or_cpr *c, const double *b, double *x)
{
    int n = c->npr;
    if (c->o.precision == OR_PREC_FP64) {
        or_amg_vcycle(&c->amg, b, x);
        return;
    }
    float *bf = calloc((size_t)n, sizeof(float)), *xf = calloc((size_t)n, sizeof(float));
    for (int i = 0; i < n; i++) bf[i] = (float)b[i];
    or_amg_vcycle_f32(&c->amg, bf, xf);
    for (int i = 0; i < n; i++) x[i] = (double)xf[i];
    free(bf); free(xf);
}

int or_cpr_vcycle(or_cpr *c, const double *b, double *x)
{
    if (!c->has_amg) return OR_ERR_ARG;
    vcycle_any(c, b, x);
    return OR_OK;
}

/* x += Pi_p V(Pi_r r) */
static void pressure_stage(or_cpr *c, const double *r, double *x)
{
    int n = c->npr;
    double *rp = malloc(sizeof(double) * (size_t)n), *dp = malloc(sizeof(double) * (size_t)n);
    or_cpr_restrict(c, r, rp);
    vcycle_any(c, rp, dp);
    for (int i = 0; i < n; i++) x[3 * i] += dp[i];
    free(rp); free(dp);
}

/* r = v - A x */
static void residual(or_cpr *c, const double *v, const double *x, double *r)
{
    int n = c->n;
    memcpy(r, v, sizeof(double) * 3 * (size_t)n);
    or_bsr_spmv(n, 3, c->rp, c->ci, c->Aval, -1.0, x, 1.0, r);
}

int or_cpr_apply(or_cpr *c, const double *v, double *z)
{
    int n = c->n;
    size_t len = 3 * (size_t)n;
    double *r = malloc(sizeof(double) * len), *t = malloc(sizeof(double) * len);
    memset(z, 0, sizeof(double) * len);
    if (c->o.fpf) {
        or_cpr_fstage(c, v, z);
        if (c->has_amg) {
            residual(c, v, z, r);
            pressure_stage(c, r, z);
        }
    } else if (c->has_amg) {
        pressure_stage(c, v, z);
    }
    residual(c, v, z, r);
    or_cpr_fstage(c, r, t);
    for (size_t e = 0; e < len; e++) z[e] += t[e];
    free(r); free(t);
    return OR_OK;
}

int or_amg_nlevels(or_cpr *c) { return c->has_amg ? c->amg.nlev : 0; }

void or_amg_level_info(or_cpr *c, int l, int *n, int *nnz, int *pnnz, int *ncolors, double *omega)
{
    const or_amg *h = &c->amg;
    *n = h->A[l].n; *nnz = h->A[l].nnz;
    *pnnz = (l < h->nlev - 1) ? h->P[l].nnz : 0;
    *ncolors = h->ncolor[l];
    *omega = (l < h->nlev - 1) ? h->omega[l] : 0.0;
}

void or_amg_level_get(or_cpr *c, int l, int32_t *rowptr, int32_t *colind, double *val,
                      int32_t *agg, int32_t *color, int32_t *prowptr, int32_t *pcolind, double *pval,
                      int32_t *srp, int32_t *sci)
{
    const or_amg *h = &c->amg;
    const or_csr *A = &h->A[l];
    if (rowptr) memcpy(rowptr, A->rp, sizeof(int32_t) * (size_t)(A->n + 1));
    if (colind) memcpy(colind, A->ci, sizeof(int32_t) * (size_t)A->nnz);
    if (val) memcpy(val, A->v, sizeof(double) * (size_t)A->nnz);
    if (agg && h->agg[l]) memcpy(agg, h->agg[l], sizeof(int32_t) * (size_t)A->n);
    if (color && h->color[l]) memcpy(color, h->color[l], sizeof(int32_t) * (size_t)A->n);
    if (l < h->nlev - 1) {
        const or_csr *P = &h->P[l];
        if (prowptr) memcpy(prowptr, P->rp, sizeof(int32_t) * (size_t)(P->n + 1));
        if (pcolind) memcpy(pcolind, P->ci, sizeof(int32_t) * (size_t)P->nnz);
        if (pval) memcpy(pval, P->v, sizeof(double) * (size_t)P->nnz);
    }
    if (srp && sci) {
        int cnt = 0;
        srp[0] = 0;
        for (int i = 0; i < A->n; i++) {
            for (int e = A->rp[i]; e < A->rp[i + 1]; e++)
                if (h->sf[l][e]) sci[cnt++] = A->ci[e];
            srp[i + 1] = cnt;
        }
    }
}

void or_amg_level_roots(or_cpr *c, int l, uint8_t *root)
{
    if (c->amg.root[l]) memcpy(root, c->amg.root[l], (size_t)c->amg.A[l].n);
}

void or_cpr_get(or_cpr *c, double *cw, double *fpiv_inv)
{
    if (cw) memcpy(cw, c->cw, sizeof(double) * 3 * (size_t)c->n);
    if (fpiv_inv) memcpy(fpiv_inv, c->inv, sizeof(double) * 9 * (size_t)c->n);
}

/* ---- FGMRES ------------------------------------------------------------ */

static double dot(size_t len, const double *a, const double *b)
{
    double s = 0.0;
    for (size_t e = 0; e < len; e++) s += a[e] * b[e];
    return s;
}

/* w <- w - sum_i h_i v_i over i < k; h written into hcol */
static void orthogonalise(size_t len, int k, const double *V, double *w, double *hcol, int orth)
{
    if (orth == 0) {
        for (int i = 0; i < k; i++) {
            double h = dot(len, w, V + (size_t)i * len);
            hcol[i] = h;
            for (size_t e = 0; e < len; e++) w[e] -= h * V[(size_t)i * len + e];
        }
        return;
    }
    double *t = malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    for (int i = 0; i < k; i++) hcol[i] = 0.0;
    for (int pass = 0; pass < 2; pass++) {
        for (int i = 0; i < k; i++) t[i] = dot(len, w, V + (size_t)i * len);
        for (int i = 0; i < k; i++) {
            for (size_t e = 0; e < len; e++) w[e] -= t[i] * V[(size_t)i * len + e];
            hcol[i] += t[i];
        }
    }
    free(t);
}

static void precond(or_cpr *pc, size_t len, const double *v, double *z)
{
    if (pc) or_cpr_apply(pc, v, z);
    else memcpy(z, v, sizeof(double) * len);
}

int or_fgmres(int n, const int32_t *rowptr, const int32_t *colind, const double *val,
              or_cpr *pc, const double *b, double *x, const or_fgmres_opts *o,
              or_fgmres_stats *st, double *hist)
{
    int m = o->m;
    size_t len = 3 * (size_t)n;
    memset(st, 0, sizeof *st);
    if (m < 1 || m > 64 || o->maxit < 0) return OR_ERR_ARG;
    double *V = malloc(sizeof(double) * len * (size_t)(m + 1));
    double *Z = malloc(sizeof(double) * len * (size_t)m);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double));
    double *cs = malloc(sizeof(double) * (size_t)m), *sn = malloc(sizeof(double) * (size_t)m);
    double *g = malloc(sizeof(double) * (size_t)(m + 1)), *y = malloc(sizeof(double) * (size_t)m);
    double *r = malloc(sizeof(double) * len);
    if (!V || !Z || !H || !r) return OR_ERR_ALLOC;
    double bnorm = sqrt(dot(len, b, b));
    int status = OR_NOT_CONVERGED;
    if (!isfinite(bnorm)) { status = OR_ERR_NONFINITE; goto done; }
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * len);
        st->converged = 1; status = OR_OK;
        goto done;
    }
    double tol = o->rtol * bnorm;
    int its = 0;
    if (hist) hist[0] = 1.0;
    for (;;) {
        memcpy(r, b, sizeof(double) * len);
        or_bsr_spmv(n, 3, rowptr, colind, val, -1.0, x, 1.0, r);
        double beta = sqrt(dot(len, r, r));
        st->rel_residual = beta / bnorm;
        if (!isfinite(beta)) { status = OR_ERR_NONFINITE; break; }
        if (beta <= tol) { st->converged = 1; status = OR_OK; break; }
        if (its >= o->maxit) break;
        if (its > 0) st->restarts++;
        for (size_t e = 0; e < len; e++) V[e] = r[e] / beta;
        memset(g, 0, sizeof(double) * (size_t)(m + 1));
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; j++) {
            double *zj = Z + (size_t)j * len, *w = V + (size_t)(j + 1) * len;
            precond(pc, len, V + (size_t)j * len, zj);
            its++;
            or_bsr_spmv(n, 3, rowptr, colind, val, 1.0, zj, 0.0, w);
            double hcol[64 + 1];
            orthogonalise(len, j + 1, V, w, hcol, o->orth);
            double hn = sqrt(dot(len, w, w));
            for (int i = 0; i <= j; i++) H[(size_t)i * m + j] = hcol[i];
            H[(size_t)(j + 1) * m + j] = hn;
            int breakdown = !(hn > 1e-300);
            if (!breakdown)
                for (size_t e = 0; e < len; e++) w[e] = w[e] / hn;
            for (int i = 0; i < j; i++) {
                double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            double den = hypot(a, bb);
            cs[j] = a / den; sn[j] = bb / den;
            H[(size_t)j * m + j] = cs[j] * a + sn[j] * bb;
            H[(size_t)(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            k = j + 1;
            st->est_residual = fabs(g[j + 1]) / bnorm;
            if (hist && its <= o->maxit) hist[its] = st->est_residual;
            if (fabs(g[j + 1]) <= tol || its >= o->maxit || breakdown) break;
        }
        for (int i = k - 1; i >= 0; i--) {
            double s = g[i];
            for (int q = i + 1; q < k; q++) s -= H[(size_t)i * m + q] * y[q];
            y[i] = s / H[(size_t)i * m + i];
        }
        for (int i = 0; i < k; i++)
            for (size_t e = 0; e < len; e++) x[e] += y[i] * Z[(size_t)i * len + e];
    }
    st->iterations = its;
done:
    free(V); free(Z); free(H); free(cs); free(sn); free(g); free(y); free(r);
    return status;
}

int or_arnoldi(int n, const int32_t *rowptr, const int32_t *colind, const double *val,
               or_cpr *pc, const double *b, int k, int orth, double *Z, double *V, double *H)
{
    size_t len = 3 * (size_t)n;
    double beta = sqrt(dot(len, b, b));
    if (!(beta > 0.0) || k < 1 || k > 64) return OR_ERR_ARG;
    memset(H, 0, sizeof(double) * (size_t)(k + 1) * k);
    for (size_t e = 0; e < len; e++) V[e] = b[e] / beta;
    for (int j = 0; j < k; j++) {
        double *zj = Z + (size_t)j * len, *w = V + (size_t)(j + 1) * len;
        precond(pc, len, V + (size_t)j * len, zj);
        or_bsr_spmv(n, 3, rowptr, colind, val, 1.0, zj, 0.0, w);
        double hcol[64 + 1];
        orthogonalise(len, j + 1, V, w, hcol, orth);
        double hn = sqrt(dot(len, w, w));
        for (int i = 0; i <= j; i++) H[(size_t)i * k + j] = hcol[i];
        H[(size_t)(j + 1) * k + j] = hn;
        for (size_t e = 0; e < len; e++) w[e] = w[e] / hn;
    }
    return OR_OK;
}
