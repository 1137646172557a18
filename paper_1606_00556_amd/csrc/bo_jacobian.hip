// Jacobian and residual of the fully implicit black-oil equations.
//
// Model: Section 2.1 (three components; Darcy fluxes; Phi = p - rho g depth;
// S_o = 1 - S_w - S_g; zero capillary pressure; no-flow outer boundary; Stone
// II oil relative permeability from Corey two-phase curves), Section 2.3
// (Peaceman wells at fixed bottom-hole pressure), Section 3 (7-point finite
// differences).  Equations are per unit surface volume (STB/day, Mscf/day);
// the upstream cell of each phase potential carries the mobility, ties going
// to the lower cell index; face densities are the mean of the two cells.
//
// Dual porosity (fractured reservoirs): each location also holds a matrix
// cell (rows N..2N-1) coupled only to its fracture cell by a transfer term
// T_mf = tcoef sigma k_m V_b, upstream-weighted like a face at zero depth
// difference (Kazemi's shape factor; the paper names the model, not its
// transfer function).  Fixed-rate wells (Section 2.3) add their bottom-hole
// pressure as an unknown and the rate constraint as a block row.
//
// Layout: one thread per cell gathers its own accumulation and its six faces
// (in the order -z, -y, -x, +x, +y, +z), then the transfer, and writes its
// whole block row, so no atomics are needed and every face flux is evaluated
// identically from both sides (lower cell first).  A second kernel writes the
// matrix rows, a third the well terms (one thread per well; perforated cells
// are distinct), including the well rows and the well columns of the
// perforated cells (the last block of their rows).
#include <mutex>
#include "bo_common.hpp"

namespace bo {
namespace {

struct Fl {
    double p_ref, Bw0, cw, Bo0, co, Bg0, cg, Rs0, crs, mu_w, mu_o, mu_g, c_r;
    double rho_wsc, rho_osc, rho_gsc, swc, sor, sorg, sgc;
    int nw, no, ng;
    double tcoef, rb_ft3, grav;
    int gravity, inj_total_mobility;
};

struct GridG {
    int nx, ny, nz;
    double dx, dy, dz, top;
    const double *kx, *ky, *kz, *phi0;
    int dual;
    const double *km, *phim;
    double sigma;
};

struct Props {
    double p, sw, sg, so;
    double bw, dbw, bo, dbo, bg, dbg, rs, drs, phi, dphi;
    double rw, drw, ro, dro, rg, drg;
    double lw, lw_w;
    double lo, lo_w, lo_g;
    double lg, lg_g;
};

__device__ inline void recip_fvf(double B0, double c, double pref, double pr, double &b, double &db) {
    double B = B0 * (1.0 - c * (pr - pref));
    double dB = -B0 * c;
    b = 1.0 / B;
    db = -dB / (B * B);
}

__device__ inline double ipow(double x, int n) {
    double r = 1.0;
    for (int k = 0; k < n; k++) r = r * x;
    return r;
}

// Corey: kr = clamp((s - lo)/span, 0, 1)^n
__device__ inline void corey(double s, double lo, double span, int n, double &kr, double &dkr) {
    double sn = (s - lo) / span;
    if (sn <= 0.0) { kr = 0.0; dkr = 0.0; return; }
    if (sn >= 1.0) { kr = 1.0; dkr = 0.0; return; }
    kr = ipow(sn, n);
    dkr = (double)n * ipow(sn, n - 1) / span;
}

__device__ inline void relperm(const Fl &f, double sw, double sg, double kr[9]) {
    double krw, dkrw, krow, dkrow, krg, dkrg, krog, dkrog;
    double spw = 1.0 - f.swc - f.sor;
    double spg = 1.0 - f.swc - f.sorg - f.sgc;
    corey(sw, f.swc, spw, f.nw, krw, dkrw);
    corey(1.0 - sw, f.sor, spw, f.no, krow, dkrow);
    dkrow = -dkrow;
    corey(sg, f.sgc, spg, f.ng, krg, dkrg);
    corey(1.0 - sg - f.swc, f.sorg, spg, f.no, krog, dkrog);
    dkrog = -dkrog;
    double krocw = 1.0;
    double a = krow / krocw + krw, da_w = dkrow / krocw + dkrw;
    double b = krog / krocw + krg, db_g = dkrog / krocw + dkrg;
    double kro = krocw * (a * b - krw - krg);
    double dkro_w = krocw * (da_w * b - dkrw);
    double dkro_g = krocw * (a * db_g - dkrg);
    if (kro <= 0.0) { kro = 0.0; dkro_w = 0.0; dkro_g = 0.0; }
    kr[0] = krw; kr[1] = krow; kr[2] = krg; kr[3] = krog; kr[4] = kro;
    kr[5] = dkro_w; kr[6] = dkro_g; kr[7] = dkrw; kr[8] = dkrg;
}

__device__ inline void props_of(const Fl &f, double phi0, const double *x, Props &c) {
    double pr = x[0], sw = x[1], sg = x[2];
    c.p = pr; c.sw = sw; c.sg = sg; c.so = 1.0 - sw - sg;
    recip_fvf(f.Bw0, f.cw, f.p_ref, pr, c.bw, c.dbw);
    recip_fvf(f.Bo0, f.co, f.p_ref, pr, c.bo, c.dbo);
    recip_fvf(f.Bg0, f.cg, f.p_ref, pr, c.bg, c.dbg);
    c.rs = f.Rs0 * (1.0 + f.crs * (pr - f.p_ref));
    c.drs = f.Rs0 * f.crs;
    c.phi = phi0 * (1.0 + f.c_r * (pr - f.p_ref));
    c.dphi = phi0 * f.c_r;
    double gps = 1000.0 * f.rho_gsc / f.rb_ft3;
    c.rw = f.rho_wsc * c.bw;
    c.drw = f.rho_wsc * c.dbw;
    c.ro = (f.rho_osc + gps * c.rs) * c.bo;
    c.dro = gps * c.drs * c.bo + (f.rho_osc + gps * c.rs) * c.dbo;
    c.rg = gps * c.bg;
    c.drg = gps * c.dbg;
    double kr[9];
    relperm(f, sw, sg, kr);
    c.lw = kr[0] / f.mu_w; c.lw_w = kr[7] / f.mu_w;
    c.lo = kr[4] / f.mu_o; c.lo_w = kr[5] / f.mu_o; c.lo_g = kr[6] / f.mu_o;
    c.lg = kr[2] / f.mu_g; c.lg_g = kr[8] / f.mu_g;
}

__device__ inline void masses(const Props &c, double m[3], double dm[3][3], bool deriv) {
    double so = c.so;
    m[0] = c.phi * so * c.bo;
    m[1] = c.phi * c.sw * c.bw;
    m[2] = c.phi * (c.sg * c.bg + c.rs * so * c.bo);
    if (!deriv) return;
    dm[0][0] = c.dphi * so * c.bo + c.phi * so * c.dbo;
    dm[0][1] = -c.phi * c.bo;
    dm[0][2] = -c.phi * c.bo;
    dm[1][0] = c.dphi * c.sw * c.bw + c.phi * c.sw * c.dbw;
    dm[1][1] = c.phi * c.bw;
    dm[1][2] = 0.0;
    dm[2][0] = c.dphi * (c.sg * c.bg + c.rs * so * c.bo) +
               c.phi * (c.sg * c.dbg + c.drs * so * c.bo + c.rs * so * c.dbo);
    dm[2][1] = -c.phi * c.rs * c.bo;
    dm[2][2] = c.phi * (c.bg - c.rs * c.bo);
}

// upwinded stream quantity: 0 oil, 1 water, 2 free gas, 3 dissolved gas
__device__ inline void stream_q(const Props &c, int kind, double &M, double dM[3]) {
    switch (kind) {
    case 0:
        M = c.lo * c.bo;
        dM[0] = c.lo * c.dbo; dM[1] = c.lo_w * c.bo; dM[2] = c.lo_g * c.bo;
        break;
    case 1:
        M = c.lw * c.bw;
        dM[0] = c.lw * c.dbw; dM[1] = c.lw_w * c.bw; dM[2] = 0.0;
        break;
    case 2:
        M = c.lg * c.bg;
        dM[0] = c.lg * c.dbg; dM[1] = 0.0; dM[2] = c.lg_g * c.bg;
        break;
    default:
        M = c.rs * c.lo * c.bo;
        dM[0] = c.lo * (c.drs * c.bo + c.rs * c.dbo);
        dM[1] = c.rs * c.lo_w * c.bo; dM[2] = c.rs * c.lo_g * c.bo;
        break;
    }
}

__device__ inline void density(const Props &c, int ph, double &rho, double &drho) {
    if (ph == 0) { rho = c.ro; drho = c.dro; }
    else if (ph == 1) { rho = c.rw; drho = c.drw; }
    else { rho = c.rg; drho = c.drg; }
}

__device__ inline double depth_of(const GridG &g, int cell) {
    int k = cell / (g.nx * g.ny);
    return g.top + ((double)k + 0.5) * g.dz;
}

// face transmissibility between adjacent cells a < b through slot direction
__device__ inline double trans(const GridG &g, const Fl &f, int a, int b) {
    int d = b - a;
    double area, len, ka, kb;
    if (d == 1) { area = g.dy * g.dz; len = g.dx; ka = g.kx[a]; kb = g.kx[b]; }
    else if (d == g.nx) { area = g.dx * g.dz; len = g.dy; ka = g.ky[a]; kb = g.ky[b]; }
    else { area = g.dx * g.dy; len = g.dz; ka = g.kz[a]; kb = g.kz[b]; }
    return f.tcoef * area / (len / (2.0 * ka) + len / (2.0 * kb));
}

// blocks per row: stencil (+1 for the matrix cell) on fracture rows, 2 on
// matrix rows; the well columns and well rows are added by k_well_counts
__global__ void k_row_counts(int nx, int ny, int nz, int dual, int32_t *cnt) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (g >= n) return;
    int c = 0;
    for (int s = 0; s < NSLOT; s++) c += nbr_of(g, s, nx, ny, nz) >= 0;
    cnt[g] = c + (dual ? 1 : 0);
    if (dual) cnt[n + g] = 2;
}

__global__ void __launch_bounds__(kBlock) k_jac_cells(GridG G, Fl f, const double *__restrict__ xo,
                                                       const double *__restrict__ xn, double acc,
                                                       const int32_t *__restrict__ rowptr,
                                                       int32_t *__restrict__ colind, double *__restrict__ val,
                                                       double *__restrict__ b) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int n = G.nx * G.ny * G.nz;
    if (g >= n) return;
    Props c;
    props_of(f, G.phi0[g], xn + 3 * (size_t)g, c);
    double R[3], Jd[9];
    {
        Props co;
        props_of(f, G.phi0[g], xo + 3 * (size_t)g, co);
        double m1[3], dm1[3][3], m0[3], dd[3][3];
        masses(c, m1, dm1, true);
        masses(co, m0, dd, false);
        for (int r = 0; r < 3; r++) R[r] = acc * (m1[r] - m0[r]);
        for (int r = 0; r < 3; r++)
            for (int s = 0; s < 3; s++) Jd[3 * r + s] = acc * dm1[r][s];
    }
    const double gg = f.gravity ? f.grav : 0.0;
    const int row_of[4] = {0, 1, 2, 2};
    const int phase_of[4] = {0, 1, 2, 0};
    // Faces in ascending column order (-z -y -x, then +x +y +z); each face's
    // off-diagonal block is written as soon as it is complete, the diagonal
    // (which every face adds to) at the end.  The loops unroll fully, so no
    // block is indexed at run time and nothing spills to scratch memory.
    const int order[6] = {S_MZ, S_MY, S_MX, S_PX, S_PY, S_PZ};
    const int e0 = rowptr[g];
    int nlow = 0;
#pragma unroll
    for (int q = 0; q < 3; q++) nlow += nbr_of(g, order[q], G.nx, G.ny, G.nz) >= 0;
    const int ediag = e0 + nlow;
    int elo = e0, ehi = ediag + 1;
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const int s = order[q];
        const int nb = nbr_of(g, s, G.nx, G.ny, G.nz);
        if (nb < 0) continue;
        double Joff[9];
#pragma unroll
        for (int z = 0; z < 9; z++) Joff[z] = 0.0;
        Props cn;
        props_of(f, G.phi0[nb], xn + 3 * (size_t)nb, cn);
        bool g_low = g < nb;
        int l = g_low ? g : nb, h = g_low ? nb : g;
        const Props &cl = g_low ? c : cn;
        const Props &ch = g_low ? cn : c;
        double T = trans(G, f, l, h);
        double ddep = depth_of(G, l) - depth_of(G, h);
#pragma unroll
        for (int st = 0; st < 4; st++) {
            const int ph = phase_of[st], row = row_of[st];
            double rl, drl, rh, drh;
            density(cl, ph, rl, drl);
            density(ch, ph, rh, drh);
            double rbar = 0.5 * (rl + rh);
            double dphi = (cl.p - ch.p) - rbar * gg * ddep;
            double dphi_pl = 1.0 - 0.5 * drl * gg * ddep;
            double dphi_ph = -1.0 - 0.5 * drh * gg * ddep;
            bool up_l = dphi >= 0.0;
            double M, dM[3];
            stream_q(up_l ? cl : ch, st, M, dM);
            double F = T * M * dphi;
            double dFl[3], dFh[3];
            dFl[0] = T * M * dphi_pl;
            dFh[0] = T * M * dphi_ph;
            dFl[1] = dFl[2] = dFh[1] = dFh[2] = 0.0;
            if (up_l) { for (int k = 0; k < 3; k++) dFl[k] = dFl[k] + T * dM[k] * dphi; }
            else      { for (int k = 0; k < 3; k++) dFh[k] = dFh[k] + T * dM[k] * dphi; }
            if (g_low) {
                R[row] = R[row] + F;
                for (int k = 0; k < 3; k++) {
                    Jd[3 * row + k] = Jd[3 * row + k] + dFl[k];
                    Joff[3 * row + k] = Joff[3 * row + k] + dFh[k];
                }
            } else {
                R[row] = R[row] - F;
                for (int k = 0; k < 3; k++) {
                    Joff[3 * row + k] = Joff[3 * row + k] - dFl[k];
                    Jd[3 * row + k] = Jd[3 * row + k] - dFh[k];
                }
            }
        }
        const int e = q < 3 ? elo++ : ehi++;
        colind[e] = nb;
#pragma unroll
        for (int z = 0; z < 9; z++) val[9 * (size_t)e + z] = Joff[z];
    }
    // fracture-matrix transfer (this cell is the lower index)
    double Jm[9];
    if (G.dual) {
        Props cm;
        props_of(f, G.phim[g], xn + 3 * ((size_t)n + g), cm);
        double T = f.tcoef * G.sigma * G.km[g] * G.dx * G.dy * G.dz;
        for (int z = 0; z < 9; z++) Jm[z] = 0.0;
        for (int st = 0; st < 4; st++) {
            int row = row_of[st];
            double dphi = c.p - cm.p;
            bool up_l = dphi >= 0.0;
            double M, dM[3];
            stream_q(up_l ? c : cm, st, M, dM);
            double F = T * M * dphi;
            double dFl[3], dFh[3];
            dFl[0] = T * M * 1.0;
            dFh[0] = T * M * -1.0;
            dFl[1] = dFl[2] = dFh[1] = dFh[2] = 0.0;
            if (up_l) { for (int k = 0; k < 3; k++) dFl[k] = dFl[k] + T * dM[k] * dphi; }
            else      { for (int k = 0; k < 3; k++) dFh[k] = dFh[k] + T * dM[k] * dphi; }
            R[row] = R[row] + F;
            for (int k = 0; k < 3; k++) {
                Jd[3 * row + k] = Jd[3 * row + k] + dFl[k];
                Jm[3 * row + k] = Jm[3 * row + k] + dFh[k];
            }
        }
    }
    // the diagonal block between the lower and upper faces, then (matrix
    // cell) (well) after the upper faces
    colind[ediag] = g;
    for (int z = 0; z < 9; z++) val[9 * (size_t)ediag + z] = Jd[z];
    const int e = ehi;
    if (G.dual) {
        colind[e] = n + g;
        for (int z = 0; z < 9; z++) val[9 * (size_t)e + z] = Jm[z];
    }
    for (int r = 0; r < 3; r++) b[3 * (size_t)g + r] = -R[r];
}

// matrix rows N + g: accumulation with the matrix porosity and minus the
// fracture-matrix transfer; blocks (fracture g, matrix N + g)
__global__ void __launch_bounds__(kBlock) k_jac_matrix(GridG G, Fl f, const double *__restrict__ xo,
                                                        const double *__restrict__ xn, double acc,
                                                        const int32_t *__restrict__ rowptr,
                                                        int32_t *__restrict__ colind, double *__restrict__ val,
                                                        double *__restrict__ b) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    int n = G.nx * G.ny * G.nz;
    if (g >= n) return;
    size_t m = (size_t)n + g;
    Props cm, cf;
    props_of(f, G.phim[g], xn + 3 * m, cm);
    props_of(f, G.phi0[g], xn + 3 * (size_t)g, cf);
    double R[3], Jd[9], Jf[9];
    {
        Props co;
        props_of(f, G.phim[g], xo + 3 * m, co);
        double m1[3], dm1[3][3], m0[3], dd[3][3];
        masses(cm, m1, dm1, true);
        masses(co, m0, dd, false);
        for (int r = 0; r < 3; r++) R[r] = acc * (m1[r] - m0[r]);
        for (int r = 0; r < 3; r++)
            for (int s = 0; s < 3; s++) Jd[3 * r + s] = acc * dm1[r][s];
    }
    for (int z = 0; z < 9; z++) Jf[z] = 0.0;
    const int row_of[4] = {0, 1, 2, 2};
    double T = f.tcoef * G.sigma * G.km[g] * G.dx * G.dy * G.dz;
    for (int st = 0; st < 4; st++) {
        int row = row_of[st];
        double dphi = cf.p - cm.p;
        bool up_l = dphi >= 0.0;
        double M, dM[3];
        stream_q(up_l ? cf : cm, st, M, dM);
        double F = T * M * dphi;
        double dFl[3], dFh[3];
        dFl[0] = T * M * 1.0;
        dFh[0] = T * M * -1.0;
        dFl[1] = dFl[2] = dFh[1] = dFh[2] = 0.0;
        if (up_l) { for (int k = 0; k < 3; k++) dFl[k] = dFl[k] + T * dM[k] * dphi; }
        else      { for (int k = 0; k < 3; k++) dFh[k] = dFh[k] + T * dM[k] * dphi; }
        R[row] = R[row] - F;
        for (int k = 0; k < 3; k++) {
            Jf[3 * row + k] = Jf[3 * row + k] - dFl[k];
            Jd[3 * row + k] = Jd[3 * row + k] - dFh[k];
        }
    }
    int e = rowptr[m];
    colind[e] = g;
    colind[e + 1] = (int32_t)m;
    for (int z = 0; z < 9; z++) {
        val[9 * (size_t)e + z] = Jf[z];
        val[9 * (size_t)(e + 1) + z] = Jd[z];
    }
    for (int r = 0; r < 3; r++) b[3 * m + r] = -R[r];
}

// Peaceman well index of a perforated cell (Section 2.3)
__device__ inline double well_index(const GridG &G, const Fl &f, int cell, double rw, double skin) {
    double kx = G.kx[cell], ky = G.ky[cell];
    double ryx = sqrt(ky / kx), rxy = sqrt(kx / ky);
    double ro = 0.28 * sqrt(ryx * G.dx * G.dx + rxy * G.dy * G.dy) / (pow(ky / kx, 0.25) + pow(kx / ky, 0.25));
    return f.tcoef * 2.0 * M_PI * sqrt(kx * ky) * G.dz / (log(ro / rw) + skin);
}

constexpr int kWellChunk = 64;
struct WellChunk {
    bo_well w[kWellChunk];
    int32_t row[kWellChunk];  // block row of a fixed-rate well, -1 for fixed BHP
};

// pattern counts of the fixed-rate wells: one more block in each perforated
// cell row (the well column), and nperf + 1 blocks in the well row
__global__ void k_well_counts(int nx, int ny, int nwells, WellChunk wells, int32_t *cnt) {
    int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwells || wells.row[w] < 0) return;
    bo_well W = wells.w[w];
    for (int k = W.k_top; k <= W.k_bot; k++) cnt[W.i + nx * (W.j + ny * k)] += 1;
    cnt[wells.row[w]] = W.k_bot - W.k_top + 2;
}

// One thread per well (a chunk of up to 64 wells passed by value): subtract
// the source from R (b += q) and dq from the diagonal block of each
// perforated cell; for a fixed-rate well also write dq/dp_h into column 0 of
// the perforated rows' well block (their last block), and the well row: the
// rate constraint and its derivatives, then the identity rows.
__global__ void k_jac_wells(GridG G, Fl f, const double *__restrict__ xn, int nwells, WellChunk wells,
                            const int32_t *__restrict__ rowptr, int32_t *__restrict__ colind,
                            double *__restrict__ val, double *__restrict__ b) {
    // one wavefront per well, a lane per perforated layer (64 at a time); the
    // well row's sums run in layer order over the lanes' terms
    const int w = blockIdx.x, lane = threadIdx.x;
    if (w >= nwells) return;
    bo_well W = wells.w[w];
    const int wr = wells.row[w];
    double gg = f.gravity ? f.grav : 0.0;
    int top = W.i + G.nx * (W.j + G.ny * W.k_top);
    double zh = depth_of(G, top);
    const double ph = wr < 0 ? W.target : xn[3 * (size_t)wr];
    double Rw = 0.0, Jww = 0.0;
    const int ew0 = wr >= 0 ? rowptr[wr] : 0;  // the well row's first block
    const double sgn = W.injector ? 1.0 : -1.0;
    for (int k0 = W.k_top; k0 <= W.k_bot; k0 += 64) {
        const int k = k0 + lane, cnt = min(64, W.k_bot - k0 + 1);
        double tq = 0.0, th = 0.0;  // this layer's terms of Rw and Jww
        if (k <= W.k_bot) {
            int cell = W.i + G.nx * (W.j + G.ny * k);
            const int ew = ew0 + (k - W.k_top);
            Props c;
            props_of(f, G.phi0[cell], xn + 3 * (size_t)cell, c);
            double WI = well_index(G, f, cell, W.rw, W.skin);
            double dz = zh - depth_of(G, cell);
            double q[3] = {0.0, 0.0, 0.0}, dq[3][3], dqh[3] = {0.0, 0.0, 0.0};
            for (int r = 0; r < 3; r++)
                for (int s = 0; s < 3; s++) dq[r][s] = 0.0;
            if (W.injector) {
                double lt = c.lo + c.lw + c.lg;
                double lt_w = c.lo_w + c.lw_w, lt_g = c.lo_g + c.lg_g;
                if (!f.inj_total_mobility) { lt = c.lw; lt_w = c.lw_w; lt_g = 0.0; }
                double dw = ph - c.p - c.rw * gg * dz;
                double dw_p = -1.0 - c.drw * gg * dz;
                q[1] = WI * lt * c.bw * dw;
                dq[1][0] = WI * lt * (c.dbw * dw + c.bw * dw_p);
                dq[1][1] = WI * lt_w * c.bw * dw;
                dq[1][2] = WI * lt_g * c.bw * dw;
                dqh[1] = WI * lt * c.bw;
            } else {
                double d_o = ph - c.p - c.ro * gg * dz;
                double d_w = ph - c.p - c.rw * gg * dz;
                double d_g = ph - c.p - c.rg * gg * dz;
                double do_p = -1.0 - c.dro * gg * dz;
                double dw_p = -1.0 - c.drw * gg * dz;
                double dg_p = -1.0 - c.drg * gg * dz;
                q[0] = WI * c.lo * c.bo * d_o;
                dq[0][0] = WI * c.lo * (c.dbo * d_o + c.bo * do_p);
                dq[0][1] = WI * c.lo_w * c.bo * d_o;
                dq[0][2] = WI * c.lo_g * c.bo * d_o;
                q[1] = WI * c.lw * c.bw * d_w;
                dq[1][0] = WI * c.lw * (c.dbw * d_w + c.bw * dw_p);
                dq[1][1] = WI * c.lw_w * c.bw * d_w;
                double qgf = WI * c.lg * c.bg * d_g;
                q[2] = qgf + c.rs * q[0];
                dq[2][0] = WI * c.lg * (c.dbg * d_g + c.bg * dg_p) + c.drs * q[0] + c.rs * dq[0][0];
                dq[2][1] = c.rs * dq[0][1];
                dq[2][2] = WI * c.lg_g * c.bg * d_g + c.rs * dq[0][2];
                dqh[0] = WI * c.lo * c.bo;
                dqh[1] = WI * c.lw * c.bw;
                dqh[2] = WI * c.lg * c.bg + c.rs * dqh[0];
            }
            int dpos = rowptr[cell];
            while (colind[dpos] != cell) dpos++;  // the diagonal is in the row by construction
            double *J = val + 9 * (size_t)dpos;
            for (int r = 0; r < 3; r++) {
                b[3 * (size_t)cell + r] = b[3 * (size_t)cell + r] + q[r];
                for (int s = 0; s < 3; s++) J[3 * r + s] = J[3 * r + s] - dq[r][s];
            }
            if (wr >= 0) {
                // the cell row's well block (its last block)
                int ec = rowptr[cell + 1] - 1;
                colind[ec] = wr;
                double *Jc = val + 9 * (size_t)ec;
                for (int r = 0; r < 3; r++) {
                    Jc[3 * r] = 0.0 - dqh[r];
                    Jc[3 * r + 1] = 0.0;
                    Jc[3 * r + 2] = 0.0;
                }
                // the well row: rate constraint (injected water / produced oil + water)
                double qc = W.injector ? q[1] : q[0] + q[1];
                double dqch = W.injector ? dqh[1] : dqh[0] + dqh[1];
                tq = sgn * qc;
                colind[ew] = cell;
                double *Jw = val + 9 * (size_t)ew;
                for (int z = 0; z < 9; z++) Jw[z] = 0.0;
                for (int s2 = 0; s2 < 3; s2++) Jw[s2] = 0.0 + sgn * (W.injector ? dq[1][s2] : dq[0][s2] + dq[1][s2]);
                th = sgn * dqch;
            }
        }
        for (int u = 0; u < cnt; u++) {
            Rw = Rw + __shfl(tq, u, 64);
            Jww = Jww + __shfl(th, u, 64);
        }
    }
    if (wr >= 0 && lane == 0) {
        const int ew = ew0 + (W.k_bot - W.k_top + 1);
        Rw = Rw - W.target;
        colind[ew] = wr;
        double *Jw = val + 9 * (size_t)ew;
        for (int z = 0; z < 9; z++) Jw[z] = 0.0;
        Jw[0] = Jww;
        Jw[4] = 1.0;
        Jw[8] = 1.0;
        b[3 * (size_t)wr] = -Rw;
        b[3 * (size_t)wr + 1] = -xn[3 * (size_t)wr + 1];
        b[3 * (size_t)wr + 2] = -xn[3 * (size_t)wr + 2];
    }
}

}  // namespace
}  // namespace bo

using namespace bo;

namespace {
// pattern sizes of a problem (host); fixed-rate well w's block row is
// cells + (the number of fixed-rate wells before w)
struct Layout {
    long long n = 0, cells = 0, rows = 0, nnz = 0;
};

bo_status layout_of(const bo_problem *p, Layout &L) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(BO_ERR_INVALID_ARG, "grid dimensions must be >= 1");
    if (p->nwells < 0 || (p->nwells > 0 && !p->wells)) return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr: wells");
    long long n = (long long)p->nx * p->ny * p->nz;
    long long faces = (long long)(p->nx - 1) * p->ny * p->nz + (long long)p->nx * (p->ny - 1) * p->nz +
                      (long long)p->nx * p->ny * (p->nz - 1);
    L.n = n;
    L.cells = n * (p->dual ? 2 : 1);
    L.nnz = n + 2 * faces + (p->dual ? 3 * n : 0);
    L.rows = L.cells;
    for (int w = 0; w < p->nwells; w++) {
        const bo_well &W = p->wells[w];
        if (W.control == BO_CTRL_BHP) continue;
        if (W.control != BO_CTRL_WRATE && W.control != BO_CTRL_LRATE)
            return fail(BO_ERR_INVALID_ARG, "well " + std::to_string(w) + ": unknown control");
        if ((W.control == BO_CTRL_WRATE) != (W.injector != 0))
            return fail(BO_ERR_INVALID_ARG, "well " + std::to_string(w) +
                                                ": water rate needs an injector, liquid rate a producer");
        long long nperf = (long long)W.k_bot - W.k_top + 1;
        L.rows++;
        L.nnz += 2 * nperf + 1;
    }
    if (L.rows >= (1LL << 31) / 8 || L.nnz >= (1LL << 31))
        return fail(BO_ERR_INVALID_ARG, "grid too large for 32-bit block indices");
    return BO_OK;
}

// Argument and well checks shared by both entry points (no heap use: wells
// are vertical, so two of them share a cell exactly when they sit in the
// same column and their layer ranges overlap).
bo_status check_args(const bo_problem *p, const double *x_old, const double *x_new, double dt, const bo_bsr *J,
                     const double *b) {
    if (!x_old || !x_new || !J || !b || !J->rowptr || !J->colind || !J->val)
        return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr: NULL pointer");
    if (!(dt > 0.0)) return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr: dt must be > 0");
    if (!p->kx || !p->ky || !p->kz || !p->phi0) return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr: NULL field");
    if (p->dual && (!p->km || !p->phim || !(p->sigma > 0.0)))
        return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr: dual porosity needs km, phim and sigma > 0");
    if (p->fluid.nw < 1 || p->fluid.no < 1 || p->fluid.ng < 1)
        return fail(BO_ERR_INVALID_ARG, "Corey exponents must be >= 1");
    for (int w = 0; w < p->nwells; w++) {
        const bo_well &W = p->wells[w];
        if (W.i < 0 || W.i >= p->nx || W.j < 0 || W.j >= p->ny || W.k_top < 0 || W.k_bot >= p->nz ||
            W.k_top > W.k_bot || !(W.rw > 0.0))
            return fail(BO_ERR_INVALID_ARG, "well " + std::to_string(w) + " is outside the grid or malformed");
        for (int v = 0; v < w; v++) {
            const bo_well &U = p->wells[v];
            if (U.i == W.i && U.j == W.j && U.k_top <= W.k_bot && W.k_top <= U.k_bot)
                return fail(BO_ERR_INVALID_ARG, "two perforations share a cell");
        }
    }
    return BO_OK;
}

// Fills chunk ch with wells w0.. (at most kWellChunk) and their block rows
// (next_row: the row of the next fixed-rate well, advanced here).
int chunk_of(const bo_problem *p, int w0, long long &next_row, WellChunk &ch) {
    int c = std::min(kWellChunk, p->nwells - w0);
    for (int q = 0; q < c; q++) {
        ch.w[q] = p->wells[w0 + q];
        ch.row[q] = ch.w[q].control == BO_CTRL_BHP ? -1 : (int32_t)next_row++;
    }
    return c;
}

// Row counts of the pattern into cnt (rows entries).
bo_status launch_counts(const bo_problem *p, const Layout &Ly, int32_t *cnt, hipStream_t s) {
    k_row_counts<<<grid_for(Ly.n), kBlock, 0, s>>>(p->nx, p->ny, p->nz, p->dual, cnt);
    long long next_row = Ly.cells;
    for (int w0 = 0; w0 < p->nwells; w0 += kWellChunk) {
        WellChunk ch{};
        int c = chunk_of(p, w0, next_row, ch);
        k_well_counts<<<1, kWellChunk, 0, s>>>(p->nx, p->ny, c, ch, cnt);
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// Blocks and right-hand side, once J->rowptr holds the pattern's row pointers.
bo_status launch_values(const bo_problem *p, const Layout &Ly, const double *x_old, const double *x_new, double dt,
                        bo_bsr *J, double *b, hipStream_t s) {
    GridG G{p->nx, p->ny, p->nz, p->dx, p->dy, p->dz, p->top_depth, p->kx, p->ky, p->kz, p->phi0,
            p->dual, p->km, p->phim, p->sigma};
    const bo_fluid &q = p->fluid;
    Fl f{q.p_ref, q.Bw0, q.cw, q.Bo0, q.co, q.Bg0, q.cg, q.Rs0, q.crs, q.mu_w, q.mu_o, q.mu_g, q.c_r,
         q.rho_wsc, q.rho_osc, q.rho_gsc, q.swc, q.sor, q.sorg, q.sgc, q.nw, q.no, q.ng,
         q.tcoef, q.rb_ft3, q.grav, q.gravity, q.inj_total_mobility};
    double acc = p->dx * p->dy * p->dz / (q.rb_ft3 * dt);
    k_jac_cells<<<grid_for(Ly.n), kBlock, 0, s>>>(G, f, x_old, x_new, acc, J->rowptr, J->colind, J->val, b);
    if (p->dual)
        k_jac_matrix<<<grid_for(Ly.n), kBlock, 0, s>>>(G, f, x_old, x_new, acc, J->rowptr, J->colind, J->val, b);
    BO_HIP(hipGetLastError());
    long long next_row = Ly.cells;
    for (int w0 = 0; w0 < p->nwells; w0 += kWellChunk) {
        WellChunk ch{};
        int c = chunk_of(p, w0, next_row, ch);
        k_jac_wells<<<c, 64, 0, s>>>(G, f, x_new, c, ch, J->rowptr, J->colind, J->val, b);
        BO_HIP(hipGetLastError());
    }
    return BO_OK;
}
}  // namespace

extern "C" bo_status bo_jacobian_bsr_size(const bo_problem *p, int32_t *nbrows, int32_t *nnzb) {
    if (!p || !nbrows || !nnzb) return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr_size: NULL argument");
    Layout L;
    BO_TRY(layout_of(p, L));
    *nbrows = (int32_t)L.rows;
    *nnzb = (int32_t)L.nnz;
    return BO_OK;
}

extern "C" bo_status bo_jacobian_bsr(const bo_problem *p, const double *x_old, const double *x_new, double dt,
                                     bo_bsr *J, double *b, void *stream) {
    if (!p) return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr: NULL problem");
    Layout Ly;
    BO_TRY(layout_of(p, Ly));
    BO_TRY(check_args(p, x_old, x_new, dt, J, b));
    const int32_t rows = (int32_t)Ly.rows, nnz = (int32_t)Ly.nnz;
    hipStream_t s = (hipStream_t)stream;
    J->nbrows = rows;
    J->nnzb = nnz;
    int32_t *cnt = nullptr;
    BO_TRY(scratch_get(SC_JAC_CNT, sizeof(int32_t) * (size_t)rows, (void **)&cnt));
    BO_TRY(launch_counts(p, Ly, cnt, s));
    int32_t total = 0;
    BO_TRY(scan_counts(cnt, J->rowptr, rows, &total, s));
    if (total != nnz) return fail(BO_ERR_HIP, "row count scan disagrees with the pattern size");
    return launch_values(p, Ly, x_old, x_new, dt, J, b, s);
}

// ---- the variant that allocates nothing ------------------------------------------
// Its only scratch is the row-pointer scan's block sums, one word per 1024
// block rows, in this array.  Each GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the array's name as an
// address: the device address comes from hipGetSymbolAddress, once per device.
static constexpr int kNoAllocScanWords = 1 << 16;
static __device__ __align__(256) int32_t scratch[kNoAllocScanWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t *g_scratch_ptr[kMaxDevices] = {};

// the current device's address of `scratch` (looked up on the first call on
// that device, with that device current)
bo_status scratch_address(int32_t **out) {
    int dev = -1;
    BO_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(BO_ERR_UNSUPPORTED, "bo_jacobian_bsr_noalloc: device index");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(BO_ERR_HIP, std::string("bo_jacobian_bsr_noalloc: hipGetSymbolAddress: ") +
                                        hipGetErrorString(e));
        g_scratch_ptr[dev] = (int32_t *)ptr;
    }
    *out = g_scratch_ptr[dev];
    return BO_OK;
}
}  // namespace

extern "C" int32_t bo_jacobian_bsr_noalloc_max_rows(void) { return kNoAllocScanWords * 1024; }

extern "C" bo_status bo_jacobian_bsr_noalloc(const bo_problem *p, const double *x_old, const double *x_new,
                                             double dt, bo_bsr *J, double *b, void *stream) {
    if (!p) return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr_noalloc: NULL problem");
    Layout Ly;
    BO_TRY(layout_of(p, Ly));
    BO_TRY(check_args(p, x_old, x_new, dt, J, b));
    if (Ly.rows > (long long)bo_jacobian_bsr_noalloc_max_rows())
        return fail(BO_ERR_INVALID_ARG, "bo_jacobian_bsr_noalloc: " + std::to_string(Ly.rows) +
                                            " block rows exceed the maximum of " +
                                            std::to_string(bo_jacobian_bsr_noalloc_max_rows()));
    int32_t *sums = nullptr;
    BO_TRY(scratch_address(&sums));
    const int32_t rows = (int32_t)Ly.rows;
    hipStream_t s = (hipStream_t)stream;
    J->nbrows = rows;
    J->nnzb = (int32_t)Ly.nnz;
    // the row counts go into J->colind (nnzb >= rows: every row holds its
    // diagonal block), which the value kernels overwrite after the scan
    BO_TRY(launch_counts(p, Ly, J->colind, s));
    BO_TRY(scan_counts_async(J->colind, J->rowptr, rows, sums, s));
    return launch_values(p, Ly, x_old, x_new, dt, J, b, s);
}
