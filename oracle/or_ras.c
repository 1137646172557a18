/*
 * Oracle (test infrastructure only): the restricted additive Schwarz (RAS)
 * preconditioner with ILU(0) subdomain solves on a scalar 7-point system,
 * the preconditioner of the paper's pressure-system run (Section 3.2 names
 * RAS with an ILU(0) local solver; Section 4.2 times GMRES(30) with it).
 *
 * Subdomains: tiles of tx x ty grid columns (all layers); with overlap d each
 * tile is extended by d columns on every side inside the grid.  A subdomain's
 * matrix is A restricted to the extended tile's cells (couplings to cells
 * outside dropped), numbered naturally (x fastest, then y, then z), and
 * factored by ILU(0) in its general IKJ form on that pattern.  The
 * preconditioner sums, over the tiles, the local solution restricted to the
 * tile's own (non-extended) cells:  z = sum_t R~_t^T (L_t U_t)^{-1} R_t r.
 *
 * Matrix input: coef[s * N + g], slot s of row g in the order -z, -y, -x,
 * diagonal, +x, +y, +z (0 where the neighbour is outside the grid).
 */
#include <stdlib.h>
#include <string.h>
#include "bo_oracle.h"

typedef struct {
    int n;             /* cells of the extended tile */
    int32_t *cell;     /* global cell of each local index */
    uint8_t *own;      /* 1 where the cell belongs to the tile itself */
    int32_t *rp, *ci;  /* local CSR pattern, ascending columns */
    double *lu;        /* ILU(0) factors on the pattern: unit L below, U on and above */
    int32_t *diag;     /* position of the diagonal in each row */
} ras_tile;

struct or_ras {
    int nx, ny, nz, ntiles;
    ras_tile *t;
};

static const int slot_di[7] = { 0, 0, -1, 0, 1, 0, 0 };
static const int slot_dj[7] = { 0, -1, 0, 0, 0, 1, 0 };
static const int slot_dk[7] = { -1, 0, 0, 0, 0, 0, 1 };

static int tile_setup(ras_tile *T, int nx, int ny, int nz, const double *coef, int i0, int i1, int j0, int j1,
                      int e0, int e1, int f0, int f1)
{
    /* interior columns [i0, i1) x [j0, j1); extended [e0, e1) x [f0, f1) */
    int wx = e1 - e0, wy = f1 - f0;
    int n = wx * wy * nz;
    long long N = (long long)nx * ny * nz;
    T->n = n;
    T->cell = malloc(sizeof(int32_t) * (size_t)n);
    T->own = malloc((size_t)n);
    T->rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    T->ci = malloc(sizeof(int32_t) * (size_t)n * 7);
    T->lu = malloc(sizeof(double) * (size_t)n * 7);
    T->diag = malloc(sizeof(int32_t) * (size_t)n);
    if (!T->cell || !T->own || !T->rp || !T->ci || !T->lu || !T->diag) return OR_ERR_ALLOC;
    int nnz = 0;
    for (int k = 0; k < nz; k++)
        for (int j = f0; j < f1; j++)
            for (int i = e0; i < e1; i++) {
                int loc = (i - e0) + wx * ((j - f0) + wy * k);
                int g = i + nx * (j + ny * k);
                T->cell[loc] = g;
                T->own[loc] = i >= i0 && i < i1 && j >= j0 && j < j1;
                T->rp[loc] = nnz;
                /* slots in ascending column order */
                for (int s = 0; s < 7; s++) {
                    int a = i + slot_di[s], b = j + slot_dj[s], c = k + slot_dk[s];
                    if (a < e0 || a >= e1 || b < f0 || b >= f1 || c < 0 || c >= nz) continue;
                    int l2 = (a - e0) + wx * ((b - f0) + wy * c);
                    if (s == 3) T->diag[loc] = nnz;
                    T->ci[nnz] = l2;
                    T->lu[nnz] = coef[(long long)s * N + g];
                    nnz++;
                }
            }
    T->rp[n] = nnz;
    /* IKJ ILU(0): for each row i, for each k < i in its pattern (ascending):
     * a_ik /= a_kk; then a_ij -= a_ik a_kj for j > k in both patterns */
    for (int i = 0; i < n; i++) {
        for (int e = T->rp[i]; e < T->rp[i + 1]; e++) {
            int k = T->ci[e];
            if (k >= i) break;
            double piv = T->lu[T->diag[k]];
            if (piv == 0.0) return OR_ERR_SINGULAR_BLOCK;
            T->lu[e] = T->lu[e] / piv;
            for (int f = e + 1; f < T->rp[i + 1]; f++) {
                int j = T->ci[f];
                for (int q = T->rp[k]; q < T->rp[k + 1]; q++)
                    if (T->ci[q] == j) { T->lu[f] -= T->lu[e] * T->lu[q]; break; }
            }
        }
        if (T->lu[T->diag[i]] == 0.0) return OR_ERR_SINGULAR_BLOCK;
    }
    return OR_OK;
}

void or_ras_free(or_ras *h)
{
    if (!h) return;
    for (int t = 0; t < h->ntiles; t++) {
        free(h->t[t].cell); free(h->t[t].own); free(h->t[t].rp); free(h->t[t].ci);
        free(h->t[t].lu); free(h->t[t].diag);
    }
    free(h->t);
    free(h);
}

int or_ras_setup(int nx, int ny, int nz, const double *coef, int tx, int ty, int overlap, or_ras **out)
{
    *out = NULL;
    if (nx < 1 || ny < 1 || nz < 1 || tx < 1 || ty < 1 || overlap < 0 || !coef) return OR_ERR_ARG;
    or_ras *h = calloc(1, sizeof *h);
    if (!h) return OR_ERR_ALLOC;
    h->nx = nx; h->ny = ny; h->nz = nz;
    int ntx = (nx + tx - 1) / tx, nty = (ny + ty - 1) / ty;
    h->ntiles = ntx * nty;
    h->t = calloc((size_t)h->ntiles, sizeof(ras_tile));
    if (!h->t) { free(h); return OR_ERR_ALLOC; }
    for (int b = 0; b < nty; b++)
        for (int a = 0; a < ntx; a++) {
            int i0 = a * tx, i1 = i0 + tx < nx ? i0 + tx : nx;
            int j0 = b * ty, j1 = j0 + ty < ny ? j0 + ty : ny;
            int e0 = i0 - overlap > 0 ? i0 - overlap : 0, e1 = i1 + overlap < nx ? i1 + overlap : nx;
            int f0 = j0 - overlap > 0 ? j0 - overlap : 0, f1 = j1 + overlap < ny ? j1 + overlap : ny;
            int st = tile_setup(&h->t[a + ntx * b], nx, ny, nz, coef, i0, i1, j0, j1, e0, e1, f0, f1);
            if (st) { or_ras_free(h); return st; }
        }
    *out = h;
    return OR_OK;
}

int or_ras_apply(const or_ras *h, const double *r, double *z)
{
    for (int t = 0; t < h->ntiles; t++) {
        const ras_tile *T = &h->t[t];
        double *y = malloc(sizeof(double) * (size_t)T->n);
        if (!y) return OR_ERR_ALLOC;
        /* L y = r (unit lower), then U y = y */
        for (int i = 0; i < T->n; i++) {
            double s = r[T->cell[i]];
            for (int e = T->rp[i]; e < T->diag[i]; e++) s -= T->lu[e] * y[T->ci[e]];
            y[i] = s;
        }
        for (int i = T->n - 1; i >= 0; i--) {
            double s = y[i];
            for (int e = T->diag[i] + 1; e < T->rp[i + 1]; e++) s -= T->lu[e] * y[T->ci[e]];
            y[i] = s / T->lu[T->diag[i]];
        }
        for (int i = 0; i < T->n; i++)
            if (T->own[i]) z[T->cell[i]] = y[i];
        free(y);
    }
    return OR_OK;
}

int or_ras_tiles(const or_ras *h) { return h->ntiles; }

/* Tile t's local system: cells (global index), own flags, CSR pattern and the
 * ILU(0) factors on it.  Any output may be NULL; returns the cell count. */
int or_ras_tile(const or_ras *h, int t, int32_t *cell, uint8_t *own, int32_t *rp, int32_t *ci, double *lu)
{
    const ras_tile *T = &h->t[t];
    if (cell) memcpy(cell, T->cell, sizeof(int32_t) * (size_t)T->n);
    if (own) memcpy(own, T->own, (size_t)T->n);
    if (rp) memcpy(rp, T->rp, sizeof(int32_t) * (size_t)(T->n + 1));
    if (ci) memcpy(ci, T->ci, sizeof(int32_t) * (size_t)T->rp[T->n]);
    if (lu) memcpy(lu, T->lu, sizeof(double) * (size_t)T->rp[T->n]);
    return T->n;
}

int or_ras_tile_nnz(const or_ras *h, int t) { return h->t[t].rp[h->t[t].n]; }
