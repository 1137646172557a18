/*
 * Oracle (test infrastructure only): black-oil properties, residual and
 * analytic Jacobian.  Plain FP64, one face at a time.
 *
 * Model: Section 2.1 (three-component black oil, Darcy's law, constraints on
 * potentials and saturations, no-flow outer boundary, Stone II oil relative
 * permeability; for fractured reservoirs a dual-porosity model in which each
 * location holds a fracture cell and a matrix cell joined by a transfer
 * term), Section 2.3 (Peaceman well model with fixed bottom-hole pressure or
 * fixed water / liquid rate, the latter adding the bottom-hole pressure as an
 * unknown and the rate constraint as an equation), Section 3 (finite
 * differences on a structured hexahedral grid).
 *
 * Dual porosity (the paper names the model without its transfer function):
 * Kazemi's shape factor, T_mf = tcoef sigma k_m V_b with sigma = 4 (1/Lx^2 +
 * 1/Ly^2 + 1/Lz^2), upstream-weighted like a face between two cells at the
 * same depth; matrix cells have no matrix-matrix faces and no wells.
 *
 * Readings where the paper is silent: the equations are written per unit of
 * surface volume (oil and water in STB/day, gas in Mscf/day); capillary
 * pressure is zero; potentials use depth positive downward,
 * Phi = p - rho * g * depth; fluxes take the upstream cell of each phase
 * potential with ties going to the lower cell index and the arithmetic mean of
 * the two cells' densities; water injectors use the cell's total mobility.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "bo_oracle.h"

/* -------- fluid properties ----------------------------------------- */

/* b = 1/B for a formation volume factor linear in p: B = B0 (1 - c (p - p_ref)). */
static void recip_fvf(double B0, double c, double pref, double pr, double *b, double *db)
{
    double B = B0 * (1.0 - c * (pr - pref));
    double dB = -B0 * c;
    *b = 1.0 / B;
    *db = -dB / (B * B);
}

static double ipow(double x, int n)
{
    double r = 1.0;
    for (int k = 0; k < n; k++) r = r * x;
    return r;
}

/* Corey curve kr = clamp((s - lo) / span, 0, 1)^n and dkr/ds. */
static void corey(double s, double lo, double span, int n, double *kr, double *dkr)
{
    double sn = (s - lo) / span;
    if (sn <= 0.0) { *kr = 0.0; *dkr = 0.0; return; }
    if (sn >= 1.0) { *kr = 1.0; *dkr = 0.0; return; }
    *kr = ipow(sn, n);
    *dkr = (double)n * ipow(sn, n - 1) / span;
}

void or_relperm(const or_problem *p, double sw, double sg, double *out)
{
    double krw, dkrw, krow, dkrow, krg, dkrg, krog, dkrog;
    double spw = 1.0 - p->swc - p->sor;
    double spg = 1.0 - p->swc - p->sorg - p->sgc;
    corey(sw, p->swc, spw, p->nw, &krw, &dkrw);
    /* oil in water-oil: normalised by the movable oil 1 - Sw - Sor */
    corey(1.0 - sw, p->sor, spw, p->no, &krow, &dkrow);
    dkrow = -dkrow;
    corey(sg, p->sgc, spg, p->ng, &krg, &dkrg);
    /* oil in gas-oil with connate water: 1 - Swc - Sorg - Sg */
    corey(1.0 - sg - p->swc, p->sorg, spg, p->no, &krog, &dkrog);
    dkrog = -dkrog;
    /* Stone II with krocw = krow(Swc) = 1 */
    double krocw = 1.0;
    double a = krow / krocw + krw, da_w = dkrow / krocw + dkrw;
    double b = krog / krocw + krg, db_g = dkrog / krocw + dkrg;
    double kro = krocw * (a * b - krw - krg);
    double dkro_w = krocw * (da_w * b - dkrw);
    double dkro_g = krocw * (a * db_g - dkrg);
    if (kro <= 0.0) { kro = 0.0; dkro_w = 0.0; dkro_g = 0.0; }
    out[0] = krw; out[1] = krow; out[2] = krg; out[3] = krog; out[4] = kro;
    out[5] = dkro_w; out[6] = dkro_g;
    out[7] = dkrw; out[8] = dkrg;
}

typedef struct {
    double p, sw, sg, so;
    double bw, dbw, bo, dbo, bg, dbg, rs, drs, phi, dphi;
    double rw, drw, ro, dro, rg, drg;        /* reservoir densities and d/dp */
    double lw, lw_w;                          /* water mobility and d/dSw */
    double lo, lo_w, lo_g;                    /* oil mobility and d/dSw, d/dSg */
    double lg, lg_g;                          /* gas mobility and d/dSg */
} props;

static int ncells(const or_problem *p) { return p->nx * p->ny * p->nz; }

/* porosity at p_ref of cell row g: fracture (or single-porosity) cells use
 * phi0, matrix cells (rows N..2N-1) phim */
static double phi_ref(const or_problem *p, int g)
{
    int n = ncells(p);
    return g < n ? p->phi0[g] : p->phim[g - n];
}

static void cell_props(const or_problem *p, int g, const double *x, props *c)
{
    double pr = x[3 * g], sw = x[3 * g + 1], sg = x[3 * g + 2];
    c->p = pr; c->sw = sw; c->sg = sg; c->so = 1.0 - sw - sg;
    recip_fvf(p->Bw0, p->cw, p->p_ref, pr, &c->bw, &c->dbw);
    recip_fvf(p->Bo0, p->co, p->p_ref, pr, &c->bo, &c->dbo);
    recip_fvf(p->Bg0, p->cg, p->p_ref, pr, &c->bg, &c->dbg);
    c->rs = p->Rs0 * (1.0 + p->crs * (pr - p->p_ref));
    c->drs = p->Rs0 * p->crs;
    c->phi = phi_ref(p, g) * (1.0 + p->c_r * (pr - p->p_ref));
    c->dphi = phi_ref(p, g) * p->c_r;
    /* densities (lbm/ft3): surface densities carried by b; 1000 scf per Mscf */
    double gas_per_stb = 1000.0 * p->rho_gsc / p->rb_ft3;
    c->rw = p->rho_wsc * c->bw;
    c->drw = p->rho_wsc * c->dbw;
    c->ro = (p->rho_osc + gas_per_stb * c->rs) * c->bo;
    c->dro = gas_per_stb * c->drs * c->bo + (p->rho_osc + gas_per_stb * c->rs) * c->dbo;
    c->rg = gas_per_stb * c->bg;
    c->drg = gas_per_stb * c->dbg;
    double kr[9];
    or_relperm(p, sw, sg, kr);
    c->lw = kr[0] / p->mu_w;  c->lw_w = kr[7] / p->mu_w;
    c->lo = kr[4] / p->mu_o;  c->lo_w = kr[5] / p->mu_o;  c->lo_g = kr[6] / p->mu_o;
    c->lg = kr[2] / p->mu_g;  c->lg_g = kr[8] / p->mu_g;
}

/* -------- geometry --------------------------------------------------- */

static double depth_of(const or_problem *p, int g)
{
    int k = g / (p->nx * p->ny);
    return p->top_depth + ((double)k + 0.5) * p->dz;
}

double or_transmissibility(const or_problem *p, int a, int b)
{
    int d = abs(b - a);
    double area, len, ka, kb;
    if (d == 1) { area = p->dy * p->dz; len = p->dx; ka = p->kx[a]; kb = p->kx[b]; }
    else if (d == p->nx) { area = p->dx * p->dz; len = p->dy; ka = p->ky[a]; kb = p->ky[b]; }
    else { area = p->dx * p->dy; len = p->dz; ka = p->kz[a]; kb = p->kz[b]; }
    /* harmonic average of the two half-cell conductances */
    return p->tcoef * area / (len / (2.0 * ka) + len / (2.0 * kb));
}

double or_pore_volume(const or_problem *p, int g, double pr)
{
    double vb = p->dx * p->dy * p->dz;
    return p->phi0[g] * (1.0 + p->c_r * (pr - p->p_ref)) * vb / p->rb_ft3;
}

double or_well_index(const or_problem *p, int g, double rw, double skin)
{
    double kx = p->kx[g], ky = p->ky[g];
    double ryx = sqrt(ky / kx), rxy = sqrt(kx / ky);
    double ro = 0.28 * sqrt(ryx * p->dx * p->dx + rxy * p->dy * p->dy)
                / (pow(ky / kx, 0.25) + pow(kx / ky, 0.25));
    return p->tcoef * 2.0 * M_PI * sqrt(kx * ky) * p->dz / (log(ro / rw) + skin);
}

/* -------- BSR pattern ------------------------------------------------ */

int or_rows(const or_problem *p, int *ncell)
{
    int nc = ncells(p) * (p->dual ? 2 : 1), rows = nc;
    for (int w = 0; w < p->nwells; w++)
        if (p->w_ctrl[w] != OR_CTRL_BHP) rows++;
    if (ncell) *ncell = nc;
    return rows;
}

/* block row of fixed-rate well w (-1 for a fixed-BHP well) */
static int well_row(const or_problem *p, int w)
{
    int nc, r = 0;
    or_rows(p, &nc);
    if (p->w_ctrl[w] == OR_CTRL_BHP) return -1;
    for (int q = 0; q < w; q++)
        if (p->w_ctrl[q] != OR_CTRL_BHP) r++;
    return nc + r;
}

static int perforates(const or_problem *p, int w, int g)
{
    int nx = p->nx, nxy = p->nx * p->ny;
    int i = g % nx, j = (g / nx) % p->ny, k = g / nxy;
    return i == p->w_i[w] && j == p->w_j[w] && k >= p->w_ktop[w] && k <= p->w_kbot[w];
}

int or_pattern(const or_problem *p, int32_t *rowptr, int32_t *colind)
{
    int nx = p->nx, ny = p->ny, nz = p->nz, nxy = nx * ny, n = nx * ny * nz;
    int nc, rows = or_rows(p, &nc);
    int cnt = 0;
    if (rowptr) rowptr[0] = 0;
    for (int g = 0; g < n; g++) {
        int i = g % nx, j = (g / nx) % ny, k = g / nxy;
        int cand[7] = { k > 0 ? g - nxy : -1, j > 0 ? g - nx : -1, i > 0 ? g - 1 : -1, g,
                        i < nx - 1 ? g + 1 : -1, j < ny - 1 ? g + nx : -1, k < nz - 1 ? g + nxy : -1 };
        for (int s = 0; s < 7; s++) {
            if (cand[s] < 0) continue;
            if (colind) colind[cnt] = cand[s];
            cnt++;
        }
        if (p->dual) {
            if (colind) colind[cnt] = n + g;
            cnt++;
        }
        for (int w = 0; w < p->nwells; w++) {
            int wr = well_row(p, w);
            if (wr < 0 || !perforates(p, w, g)) continue;
            if (colind) colind[cnt] = wr;
            cnt++;
        }
        if (rowptr) rowptr[g + 1] = cnt;
    }
    if (p->dual)
        for (int g = 0; g < n; g++) {
            if (colind) { colind[cnt] = g; colind[cnt + 1] = n + g; }
            cnt += 2;
            if (rowptr) rowptr[n + g + 1] = cnt;
        }
    for (int w = 0; w < p->nwells; w++) {
        int wr = well_row(p, w);
        if (wr < 0) continue;
        for (int k = p->w_ktop[w]; k <= p->w_kbot[w]; k++) {
            if (colind) colind[cnt] = p->w_i[w] + nx * (p->w_j[w] + ny * k);
            cnt++;
        }
        if (colind) colind[cnt] = wr;
        cnt++;
        if (rowptr) rowptr[wr + 1] = cnt;
    }
    (void)rows;
    return cnt;
}

static double *block_at(const int32_t *rowptr, const int32_t *colind, double *val, int r, int c)
{
    for (int e = rowptr[r]; e < rowptr[r + 1]; e++)
        if (colind[e] == c) return val + 9 * (size_t)e;
    return NULL;
}

/* -------- residual and Jacobian ------------------------------------- */

/* Component mass per unit pore volume factor: m = phi * (surface volume per rb)
 * for (oil, water, gas); derivatives with respect to (p, Sw, Sg). */
static void masses(const props *c, double m[3], double dm[3][3])
{
    double so = c->so;
    m[0] = c->phi * so * c->bo;
    m[1] = c->phi * c->sw * c->bw;
    m[2] = c->phi * (c->sg * c->bg + c->rs * so * c->bo);
    if (!dm) return;
    dm[0][0] = c->dphi * so * c->bo + c->phi * so * c->dbo;
    dm[0][1] = -c->phi * c->bo;
    dm[0][2] = -c->phi * c->bo;
    dm[1][0] = c->dphi * c->sw * c->bw + c->phi * c->sw * c->dbw;
    dm[1][1] = c->phi * c->bw;
    dm[1][2] = 0.0;
    dm[2][0] = c->dphi * (c->sg * c->bg + c->rs * so * c->bo)
             + c->phi * (c->sg * c->dbg + c->drs * so * c->bo + c->rs * so * c->dbo);
    dm[2][1] = -c->phi * c->rs * c->bo;
    dm[2][2] = c->phi * (c->bg - c->rs * c->bo);
}

/* Upwinded quantity M of one flowing stream and its derivatives with respect to
 * the cell's own (p, Sw, Sg).  kind: 0 oil (lambda_o b_o), 1 water, 2 free gas,
 * 3 dissolved gas (R_s lambda_o b_o, carried by the oil phase). */
static void stream(const props *c, int kind, double *M, double dM[3])
{
    switch (kind) {
    case 0:
        *M = c->lo * c->bo;
        dM[0] = c->lo * c->dbo; dM[1] = c->lo_w * c->bo; dM[2] = c->lo_g * c->bo;
        break;
    case 1:
        *M = c->lw * c->bw;
        dM[0] = c->lw * c->dbw; dM[1] = c->lw_w * c->bw; dM[2] = 0.0;
        break;
    case 2:
        *M = c->lg * c->bg;
        dM[0] = c->lg * c->dbg; dM[1] = 0.0; dM[2] = c->lg_g * c->bg;
        break;
    default:
        *M = c->rs * c->lo * c->bo;
        dM[0] = c->lo * (c->drs * c->bo + c->rs * c->dbo);
        dM[1] = c->rs * c->lo_w * c->bo; dM[2] = c->rs * c->lo_g * c->bo;
        break;
    }
}

static void phase_density(const props *c, int phase, double *rho, double *drho)
{
    if (phase == 0) { *rho = c->ro; *drho = c->dro; }
    else if (phase == 1) { *rho = c->rw; *drho = c->drw; }
    else { *rho = c->rg; *drho = c->drg; }
}

/* Adds the flux terms of the connection (l, h), l < h, with transmissibility T
 * and depth difference ddep = depth(l) - depth(h), to R and (optionally) the
 * Jacobian: a face between two cells, or the fracture-matrix transfer. */
static void flux_terms(const or_problem *p, int l, int h, double T, double ddep, const props *cl,
                       const props *ch, double *R, const int32_t *rowptr, const int32_t *colind, double *val)
{
    double g = p->gravity ? p->grav : 0.0;
    /* component row, stream kind, phase whose potential drives it */
    static const int row_of[4] = { 0, 1, 2, 2 };
    static const int phase_of[4] = { 0, 1, 2, 0 };
    double *Jll = NULL, *Jlh = NULL, *Jhl = NULL, *Jhh = NULL;
    if (val) {
        Jll = block_at(rowptr, colind, val, l, l);
        Jlh = block_at(rowptr, colind, val, l, h);
        Jhl = block_at(rowptr, colind, val, h, l);
        Jhh = block_at(rowptr, colind, val, h, h);
    }
    for (int s = 0; s < 4; s++) {
        int ph = phase_of[s], row = row_of[s];
        double rl, drl, rh, drh;
        phase_density(cl, ph, &rl, &drl);
        phase_density(ch, ph, &rh, &drh);
        double rbar = 0.5 * (rl + rh);
        double dphi = (cl->p - ch->p) - rbar * g * ddep;
        double dphi_pl = 1.0 - 0.5 * drl * g * ddep;
        double dphi_ph = -1.0 - 0.5 * drh * g * ddep;
        int up_is_l = dphi >= 0.0;
        double M, dM[3];
        stream(up_is_l ? cl : ch, s, &M, dM);
        double F = T * M * dphi;
        R[3 * l + row] += F;
        R[3 * h + row] -= F;
        if (!val) continue;
        double dFl[3], dFh[3];
        dFl[0] = T * M * dphi_pl;
        dFh[0] = T * M * dphi_ph;
        dFl[1] = dFl[2] = dFh[1] = dFh[2] = 0.0;
        double *dFu = up_is_l ? dFl : dFh;
        for (int q = 0; q < 3; q++) dFu[q] += T * dM[q] * dphi;
        for (int q = 0; q < 3; q++) {
            Jll[3 * row + q] += dFl[q];
            Jlh[3 * row + q] += dFh[q];
            Jhl[3 * row + q] -= dFl[q];
            Jhh[3 * row + q] -= dFh[q];
        }
    }
}

static void face_terms(const or_problem *p, int l, int h, const props *cl, const props *ch,
                       double *R, const int32_t *rowptr, const int32_t *colind, double *val)
{
    flux_terms(p, l, h, or_transmissibility(p, l, h), depth_of(p, l) - depth_of(p, h), cl, ch, R, rowptr,
               colind, val);
}

double or_transfer(const or_problem *p, int g)
{
    return p->tcoef * p->sigma * p->km[g] * p->dx * p->dy * p->dz;
}

/* faces between (fracture) cells, then the fracture-matrix transfers */
static void for_each_face(const or_problem *p, const props *c, double *R, const int32_t *rowptr,
                          const int32_t *colind, double *val)
{
    int nx = p->nx, ny = p->ny, nz = p->nz, nxy = nx * ny;
    for (int k = 0; k < nz; k++)
        for (int j = 0; j < ny; j++)
            for (int i = 0; i < nx; i++) {
                int g = i + nx * (j + ny * k);
                if (i < nx - 1) face_terms(p, g, g + 1, &c[g], &c[g + 1], R, rowptr, colind, val);
                if (j < ny - 1) face_terms(p, g, g + nx, &c[g], &c[g + nx], R, rowptr, colind, val);
                if (k < nz - 1) face_terms(p, g, g + nxy, &c[g], &c[g + nxy], R, rowptr, colind, val);
            }
    if (p->dual) {
        int n = nx * ny * nz;
        for (int g = 0; g < n; g++)
            flux_terms(p, g, n + g, or_transfer(p, g), 0.0, &c[g], &c[n + g], R, rowptr, colind, val);
    }
}

/* Peaceman well terms (Section 2.3): q = WI * lambda * b * (p_h - p - rho g (z_h - z)).
 * The residual subtracts the source, so R -= q and J -= dq.  For a fixed-rate
 * well p_h is the unknown of its well row: the cell rows also get dq/dp_h in
 * column 0 of their block in the well's column, and the well row collects the
 * rate constraint. */
static int well_terms(const or_problem *p, const props *c, const double *x, double *R, const int32_t *rowptr,
                      const int32_t *colind, double *val)
{
    double g = p->gravity ? p->grav : 0.0;
    for (int w = 0; w < p->nwells; w++) {
        int ctrl = p->w_ctrl[w];
        if (ctrl != OR_CTRL_BHP && ctrl != OR_CTRL_WRATE && ctrl != OR_CTRL_LRATE) return OR_ERR_ARG;
        if (ctrl == OR_CTRL_WRATE && !p->w_inj[w]) return OR_ERR_ARG;
        if (ctrl == OR_CTRL_LRATE && p->w_inj[w]) return OR_ERR_ARG;
        int wr = well_row(p, w);
        double ph = wr < 0 ? p->w_target[w] : x[3 * wr];
        int top = p->w_i[w] + p->nx * (p->w_j[w] + p->ny * p->w_ktop[w]);
        double zh = depth_of(p, top);
        double *Jww = (val && wr >= 0) ? block_at(rowptr, colind, val, wr, wr) : NULL;
        for (int k = p->w_ktop[w]; k <= p->w_kbot[w]; k++) {
            int cell = p->w_i[w] + p->nx * (p->w_j[w] + p->ny * k);
            const props *cc = &c[cell];
            double WI = or_well_index(p, cell, p->w_rw[w], p->w_skin[w]);
            double dz = zh - depth_of(p, cell);
            double q[3] = { 0, 0, 0 }, dq[3][3], dqh[3] = { 0, 0, 0 };
            memset(dq, 0, sizeof dq);
            if (p->w_inj[w]) {
                double lt = cc->lo + cc->lw + cc->lg;
                double lt_w = cc->lo_w + cc->lw_w, lt_g = cc->lo_g + cc->lg_g;
                if (!p->inj_total_mobility) { lt = cc->lw; lt_w = cc->lw_w; lt_g = 0.0; }
                double dw = ph - cc->p - cc->rw * g * dz;
                double dw_p = -1.0 - cc->drw * g * dz;
                q[1] = WI * lt * cc->bw * dw;
                dq[1][0] = WI * lt * (cc->dbw * dw + cc->bw * dw_p);
                dq[1][1] = WI * lt_w * cc->bw * dw;
                dq[1][2] = WI * lt_g * cc->bw * dw;
                dqh[1] = WI * lt * cc->bw;
            } else {
                double d_o = ph - cc->p - cc->ro * g * dz;
                double d_w = ph - cc->p - cc->rw * g * dz;
                double d_g = ph - cc->p - cc->rg * g * dz;
                double do_p = -1.0 - cc->dro * g * dz;
                double dw_p = -1.0 - cc->drw * g * dz;
                double dg_p = -1.0 - cc->drg * g * dz;
                q[0] = WI * cc->lo * cc->bo * d_o;
                dq[0][0] = WI * cc->lo * (cc->dbo * d_o + cc->bo * do_p);
                dq[0][1] = WI * cc->lo_w * cc->bo * d_o;
                dq[0][2] = WI * cc->lo_g * cc->bo * d_o;
                q[1] = WI * cc->lw * cc->bw * d_w;
                dq[1][0] = WI * cc->lw * (cc->dbw * d_w + cc->bw * dw_p);
                dq[1][1] = WI * cc->lw_w * cc->bw * d_w;
                double qgf = WI * cc->lg * cc->bg * d_g;
                q[2] = qgf + cc->rs * q[0];
                dq[2][0] = WI * cc->lg * (cc->dbg * d_g + cc->bg * dg_p) + cc->drs * q[0] + cc->rs * dq[0][0];
                dq[2][1] = cc->rs * dq[0][1];
                dq[2][2] = WI * cc->lg_g * cc->bg * d_g + cc->rs * dq[0][2];
                dqh[0] = WI * cc->lo * cc->bo;
                dqh[1] = WI * cc->lw * cc->bw;
                dqh[2] = WI * cc->lg * cc->bg + cc->rs * dqh[0];
            }
            for (int r = 0; r < 3; r++) R[3 * cell + r] -= q[r];
            if (val) {
                double *J = block_at(rowptr, colind, val, cell, cell);
                for (int r = 0; r < 3; r++)
                    for (int s = 0; s < 3; s++) J[3 * r + s] -= dq[r][s];
            }
            if (wr < 0) continue;
            /* rate constraint: injected water, or produced oil + water */
            double sgn = p->w_inj[w] ? 1.0 : -1.0;
            double qc = p->w_inj[w] ? q[1] : q[0] + q[1];
            double dqc[3], dqch = p->w_inj[w] ? dqh[1] : dqh[0] + dqh[1];
            for (int s = 0; s < 3; s++) dqc[s] = p->w_inj[w] ? dq[1][s] : dq[0][s] + dq[1][s];
            R[3 * wr] += sgn * qc;
            if (val) {
                double *Jcw = block_at(rowptr, colind, val, cell, wr);
                double *Jwc = block_at(rowptr, colind, val, wr, cell);
                for (int r = 0; r < 3; r++) Jcw[3 * r] -= dqh[r];
                for (int s = 0; s < 3; s++) Jwc[s] += sgn * dqc[s];
                Jww[0] += sgn * dqch;
            }
        }
        if (wr >= 0) {
            R[3 * wr] -= p->w_target[w];
            R[3 * wr + 1] = x[3 * wr + 1];
            R[3 * wr + 2] = x[3 * wr + 2];
            if (Jww) { Jww[4] = 1.0; Jww[8] = 1.0; }
        }
    }
    return OR_OK;
}

int or_assemble(const or_problem *p, const double *x_old, const double *x_new, double dt,
                double *R, const int32_t *rowptr, const int32_t *colind, double *val)
{
    int nc, rows = or_rows(p, &nc);
    if (ncells(p) <= 0 || dt <= 0.0) return OR_ERR_ARG;
    if (p->dual && (!p->km || !p->phim || !(p->sigma > 0.0))) return OR_ERR_ARG;
    props *cn = malloc(sizeof(props) * (size_t)nc);
    if (!cn) return OR_ERR_ALLOC;
    for (int g = 0; g < nc; g++) cell_props(p, g, x_new, &cn[g]);
    memset(R, 0, sizeof(double) * 3 * (size_t)rows);
    if (val) memset(val, 0, sizeof(double) * 9 * (size_t)rowptr[rows]);
    /* accumulation: V_b / (5.615 dt) * (m(x_new) - m(x_old)) */
    double acc = p->dx * p->dy * p->dz / (p->rb_ft3 * dt);
    for (int g = 0; g < nc; g++) {
        props co;
        cell_props(p, g, x_old, &co);
        double m1[3], dm1[3][3], m0[3];
        masses(&cn[g], m1, dm1);
        masses(&co, m0, NULL);
        for (int r = 0; r < 3; r++) R[3 * g + r] += acc * (m1[r] - m0[r]);
        if (val) {
            double *J = block_at(rowptr, colind, val, g, g);
            for (int r = 0; r < 3; r++)
                for (int s = 0; s < 3; s++) J[3 * r + s] += acc * dm1[r][s];
        }
    }
    for_each_face(p, cn, R, rowptr, colind, val);
    int st = well_terms(p, cn, x_new, R, rowptr, colind, val);
    free(cn);
    if (st != OR_OK) return st;
    for (int e = 0; e < 3 * rows; e++)
        if (!isfinite(R[e])) return OR_ERR_NONFINITE;
    return OR_OK;
}

int or_flux_residual(const or_problem *p, const double *x, double *R)
{
    int nc;
    or_rows(p, &nc);
    props *c = malloc(sizeof(props) * (size_t)nc);
    if (!c) return OR_ERR_ALLOC;
    for (int g = 0; g < nc; g++) cell_props(p, g, x, &c[g]);
    memset(R, 0, sizeof(double) * 3 * (size_t)nc);
    for_each_face(p, c, R, NULL, NULL, NULL);
    free(c);
    return OR_OK;
}
