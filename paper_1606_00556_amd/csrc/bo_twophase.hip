// Two-phase oil-water model (Section 2.2): Jacobian and residual with 2x2
// blocks, and the 2x2-block BSR SpMV.
//
// The model is the black-oil model without the gas phase: oil and water mass
// balances (per unit of surface volume, STB/day), S_o + S_w = 1, unknowns
// (p_o, S_w) per cell, zero capillary pressure (p_w = p_o), dead oil (the
// oil's density and formation volume factor carry no dissolved gas), Corey
// relative permeabilities k_rw(S_w) and k_ro(1 - S_w) over the movable range
// [S_wc, 1 - S_or].  Fluxes and wells are those of the black-oil path
// restricted to two phases: Darcy fluxes through harmonic-mean face
// transmissibilities, the upstream cell of each phase potential carrying the
// mobility (ties to the lower cell index), face densities the mean of the two
// cells; Peaceman wells at fixed bottom-hole pressure (Section 2.3), water
// injectors with the cell's total mobility.
//
// Block rows are (oil, water), block columns (p_o, S_w), row-major.  Layout:
// one thread per cell gathers its accumulation and six faces and writes its
// block row (same schedule as the black-oil kernel); one wavefront per well,
// a lane per perforated layer, adds the well terms to the diagonal blocks.
#include "bo_common.hpp"

namespace bo {
namespace {

struct Fl2 {
    double p_ref, Bw0, cw, Bo0, co, mu_w, mu_o, c_r, rho_wsc, rho_osc, swc, sor;
    int nw, no;
    double tcoef, rb_ft3, grav;
    int gravity, inj_total_mobility;
};

struct Grid2 {
    int nx, ny, nz;
    double dx, dy, dz, top;
    const double *kx, *ky, *kz, *phi0;
};

struct Props2 {
    double p, sw, so;
    double bw, dbw, bo, dbo, phi, dphi;
    double rw, drw, ro, dro;
    double lw, lw_w, lo, lo_w;
};

__device__ inline void recip_fvf2(double B0, double c, double pref, double pr, double &b, double &db) {
    double B = B0 * (1.0 - c * (pr - pref));
    double dB = -B0 * c;
    b = 1.0 / B;
    db = -dB / (B * B);
}

// Corey curve kr = clamp((s - lo) / span, 0, 1)^n and dkr/ds
__device__ inline void corey2(double s, double lo, double span, int n, double &kr, double &dkr) {
    double sn = (s - lo) / span;
    if (sn <= 0.0) { kr = 0.0; dkr = 0.0; return; }
    if (sn >= 1.0) { kr = 1.0; dkr = 0.0; return; }
    double r = 1.0, r1 = 1.0;
    for (int k = 0; k < n; k++) r = r * sn;
    for (int k = 0; k < n - 1; k++) r1 = r1 * sn;
    kr = r;
    dkr = (double)n * r1 / span;
}

__device__ inline void props2(const Fl2 &f, double phi0, const double *x, Props2 &c) {
    double pr = x[0], sw = x[1];
    c.p = pr; c.sw = sw; c.so = 1.0 - sw;
    recip_fvf2(f.Bw0, f.cw, f.p_ref, pr, c.bw, c.dbw);
    recip_fvf2(f.Bo0, f.co, f.p_ref, pr, c.bo, c.dbo);
    c.phi = phi0 * (1.0 + f.c_r * (pr - f.p_ref));
    c.dphi = phi0 * f.c_r;
    c.rw = f.rho_wsc * c.bw;
    c.drw = f.rho_wsc * c.dbw;
    c.ro = f.rho_osc * c.bo;
    c.dro = f.rho_osc * c.dbo;
    double span = 1.0 - f.swc - f.sor;
    double krw, dkrw, kro, dkro;
    corey2(sw, f.swc, span, f.nw, krw, dkrw);
    corey2(1.0 - sw, f.sor, span, f.no, kro, dkro);
    c.lw = krw / f.mu_w; c.lw_w = dkrw / f.mu_w;
    c.lo = kro / f.mu_o; c.lo_w = -dkro / f.mu_o;
}

__device__ inline double depth2(const Grid2 &g, int cell) {
    int k = cell / (g.nx * g.ny);
    return g.top + ((double)k + 0.5) * g.dz;
}

__device__ inline double trans2(const Grid2 &g, const Fl2 &f, int a, int b) {
    int d = b - a;
    double area, len, ka, kb;
    if (d == 1) { area = g.dy * g.dz; len = g.dx; ka = g.kx[a]; kb = g.kx[b]; }
    else if (d == g.nx) { area = g.dx * g.dz; len = g.dy; ka = g.ky[a]; kb = g.ky[b]; }
    else { area = g.dx * g.dy; len = g.dz; ka = g.kz[a]; kb = g.kz[b]; }
    return f.tcoef * area / (len / (2.0 * ka) + len / (2.0 * kb));
}

__global__ void k_row_counts2(int nx, int ny, int nz, int32_t *cnt) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= nx * ny * nz) return;
    int c = 0;
    for (int s = 0; s < NSLOT; s++) c += nbr_of(g, s, nx, ny, nz) >= 0;
    cnt[g] = c;
}

__global__ void __launch_bounds__(kBlock) k_jac2_cells(Grid2 G, Fl2 f, const double *__restrict__ xo,
                                                        const double *__restrict__ xn, double acc,
                                                        const int32_t *__restrict__ rowptr,
                                                        int32_t *__restrict__ colind, double *__restrict__ val,
                                                        double *__restrict__ b) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G.nx * G.ny * G.nz) return;
    Props2 c, co;
    props2(f, G.phi0[g], xn + 2 * (size_t)g, c);
    props2(f, G.phi0[g], xo + 2 * (size_t)g, co);
    // accumulation: m_o = phi S_o b_o, m_w = phi S_w b_w
    double R[2], Jd[4];
    R[0] = acc * (c.phi * c.so * c.bo - co.phi * co.so * co.bo);
    R[1] = acc * (c.phi * c.sw * c.bw - co.phi * co.sw * co.bw);
    Jd[0] = acc * (c.dphi * c.so * c.bo + c.phi * c.so * c.dbo);
    Jd[1] = acc * (-c.phi * c.bo);
    Jd[2] = acc * (c.dphi * c.sw * c.bw + c.phi * c.sw * c.dbw);
    Jd[3] = acc * (c.phi * c.bw);
    const double gg = f.gravity ? f.grav : 0.0;
    const int order[6] = {S_MZ, S_MY, S_MX, S_PX, S_PY, S_PZ};
    const int e0 = rowptr[g];
    int nlow = 0;
#pragma unroll
    for (int q = 0; q < 3; q++) nlow += nbr_of(g, order[q], G.nx, G.ny, G.nz) >= 0;
    const int ediag = e0 + nlow;
    int elo = e0, ehi = ediag + 1;
#pragma unroll
    for (int q = 0; q < 6; q++) {
        const int nb = nbr_of(g, order[q], G.nx, G.ny, G.nz);
        if (nb < 0) continue;
        double Joff[4] = {0.0, 0.0, 0.0, 0.0};
        Props2 cn;
        props2(f, G.phi0[nb], xn + 2 * (size_t)nb, cn);
        const bool g_low = g < nb;
        const int l = g_low ? g : nb, h = g_low ? nb : g;
        const Props2 &cl = g_low ? c : cn;
        const Props2 &ch = g_low ? cn : c;
        const double T = trans2(G, f, l, h);
        const double ddep = depth2(G, l) - depth2(G, h);
#pragma unroll
        for (int ph = 0; ph < 2; ph++) {  // row 0 oil, row 1 water
            const double rl = ph == 0 ? cl.ro : cl.rw, drl = ph == 0 ? cl.dro : cl.drw;
            const double rh = ph == 0 ? ch.ro : ch.rw, drh = ph == 0 ? ch.dro : ch.drw;
            const double rbar = 0.5 * (rl + rh);
            const double dphi = (cl.p - ch.p) - rbar * gg * ddep;
            const double dphi_pl = 1.0 - 0.5 * drl * gg * ddep;
            const double dphi_ph = -1.0 - 0.5 * drh * gg * ddep;
            const bool up_l = dphi >= 0.0;
            const Props2 &u = up_l ? cl : ch;
            // upstream stream quantity lambda b and its derivatives
            const double M = ph == 0 ? u.lo * u.bo : u.lw * u.bw;
            const double dM0 = ph == 0 ? u.lo * u.dbo : u.lw * u.dbw;
            const double dM1 = ph == 0 ? u.lo_w * u.bo : u.lw_w * u.bw;
            const double F = T * M * dphi;
            double dFl0 = T * M * dphi_pl, dFh0 = T * M * dphi_ph, dFl1 = 0.0, dFh1 = 0.0;
            if (up_l) { dFl0 = dFl0 + T * dM0 * dphi; dFl1 = dFl1 + T * dM1 * dphi; }
            else      { dFh0 = dFh0 + T * dM0 * dphi; dFh1 = dFh1 + T * dM1 * dphi; }
            if (g_low) {
                R[ph] = R[ph] + F;
                Jd[2 * ph] = Jd[2 * ph] + dFl0;
                Jd[2 * ph + 1] = Jd[2 * ph + 1] + dFl1;
                Joff[2 * ph] = Joff[2 * ph] + dFh0;
                Joff[2 * ph + 1] = Joff[2 * ph + 1] + dFh1;
            } else {
                R[ph] = R[ph] - F;
                Joff[2 * ph] = Joff[2 * ph] - dFl0;
                Joff[2 * ph + 1] = Joff[2 * ph + 1] - dFl1;
                Jd[2 * ph] = Jd[2 * ph] - dFh0;
                Jd[2 * ph + 1] = Jd[2 * ph + 1] - dFh1;
            }
        }
        const int e = q < 3 ? elo++ : ehi++;
        colind[e] = nb;
#pragma unroll
        for (int z = 0; z < 4; z++) val[4 * (size_t)e + z] = Joff[z];
    }
    colind[ediag] = g;
#pragma unroll
    for (int z = 0; z < 4; z++) val[4 * (size_t)ediag + z] = Jd[z];
    b[2 * (size_t)g] = -R[0];
    b[2 * (size_t)g + 1] = -R[1];
}

__device__ inline double well_index2(const Grid2 &G, const Fl2 &f, int cell, double rw, double skin) {
    double kx = G.kx[cell], ky = G.ky[cell];
    double ryx = sqrt(ky / kx), rxy = sqrt(kx / ky);
    double ro = 0.28 * sqrt(ryx * G.dx * G.dx + rxy * G.dy * G.dy) / (pow(ky / kx, 0.25) + pow(kx / ky, 0.25));
    return f.tcoef * 2.0 * M_PI * sqrt(kx * ky) * G.dz / (log(ro / rw) + skin);
}

constexpr int kWellChunk2 = 64;
struct WellChunk2 {
    bo_well w[kWellChunk2];
};

// One wavefront per fixed-BHP well, a lane per perforated layer (64 at a
// time; perforated cells are distinct): b += q, diagonal block -= dq/dx.
__global__ void k_jac2_wells(Grid2 G, Fl2 f, const double *__restrict__ xn, int nwells, WellChunk2 wells,
                             const int32_t *__restrict__ rowptr, const int32_t *__restrict__ colind,
                             double *__restrict__ val, double *__restrict__ b) {
    const int w = blockIdx.x, lane = threadIdx.x;
    if (w >= nwells) return;
    const bo_well W = wells.w[w];
    const double gg = f.gravity ? f.grav : 0.0;
    const double zh = depth2(G, W.i + G.nx * (W.j + G.ny * W.k_top));
    const double ph = W.target;
    for (int k = W.k_top + lane; k <= W.k_bot; k += 64) {
        const int cell = W.i + G.nx * (W.j + G.ny * k);
        Props2 c;
        props2(f, G.phi0[cell], xn + 2 * (size_t)cell, c);
        const double WI = well_index2(G, f, cell, W.rw, W.skin);
        const double dz = zh - depth2(G, cell);
        double q[2] = {0.0, 0.0}, dq[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
        if (W.injector) {
            double lt = c.lo + c.lw, lt_w = c.lo_w + c.lw_w;
            if (!f.inj_total_mobility) { lt = c.lw; lt_w = c.lw_w; }
            const double dw = ph - c.p - c.rw * gg * dz;
            const double dw_p = -1.0 - c.drw * gg * dz;
            q[1] = WI * lt * c.bw * dw;
            dq[1][0] = WI * lt * (c.dbw * dw + c.bw * dw_p);
            dq[1][1] = WI * lt_w * c.bw * dw;
        } else {
            const double d_o = ph - c.p - c.ro * gg * dz, d_w = ph - c.p - c.rw * gg * dz;
            const double do_p = -1.0 - c.dro * gg * dz, dw_p = -1.0 - c.drw * gg * dz;
            q[0] = WI * c.lo * c.bo * d_o;
            dq[0][0] = WI * c.lo * (c.dbo * d_o + c.bo * do_p);
            dq[0][1] = WI * c.lo_w * c.bo * d_o;
            q[1] = WI * c.lw * c.bw * d_w;
            dq[1][0] = WI * c.lw * (c.dbw * d_w + c.bw * dw_p);
            dq[1][1] = WI * c.lw_w * c.bw * d_w;
        }
        int dpos = rowptr[cell];
        while (colind[dpos] != cell) dpos++;  // the diagonal is in the row by construction
        double *J = val + 4 * (size_t)dpos;
        for (int r = 0; r < 2; r++) {
            b[2 * (size_t)cell + r] = b[2 * (size_t)cell + r] + q[r];
            for (int s = 0; s < 2; s++) J[2 * r + s] = J[2 * r + s] - dq[r][s];
        }
    }
}

// y = alpha A x + beta y, one thread per block row, blocks in stored order
__global__ void __launch_bounds__(kBlock) k_bsr2_spmv(int n, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const double *__restrict__ v, double alpha,
                                                       const double *__restrict__ x, double beta,
                                                       double *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s0 = 0.0, s1 = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
        const double *a = v + 4 * (size_t)e;
        const int j = ci[e];
        const double x0 = x[2 * (size_t)j], x1 = x[2 * (size_t)j + 1];
        s0 = s0 + a[0] * x0; s0 = s0 + a[1] * x1;
        s1 = s1 + a[2] * x0; s1 = s1 + a[3] * x1;
    }
    double *yi = y + 2 * (size_t)i;
    if (beta == 0.0) {
        yi[0] = alpha * s0 + 0.0;
        yi[1] = alpha * s1 + 0.0;
    } else {
        yi[0] = alpha * s0 + beta * yi[0];
        yi[1] = alpha * s1 + beta * yi[1];
    }
}

bo_status layout2(const bo_problem *p, long long &n, long long &nnz) {
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return fail(BO_ERR_INVALID_ARG, "grid dimensions must be >= 1");
    if (p->dual) return fail(BO_ERR_UNSUPPORTED, "bo_jacobian2_bsr: the two-phase path has no dual porosity");
    if (p->nwells < 0 || (p->nwells > 0 && !p->wells)) return fail(BO_ERR_INVALID_ARG, "bo_jacobian2_bsr: wells");
    for (int w = 0; w < p->nwells; w++)
        if (p->wells[w].control != BO_CTRL_BHP)
            return fail(BO_ERR_UNSUPPORTED, "bo_jacobian2_bsr: well " + std::to_string(w) +
                                                ": the two-phase path takes fixed-BHP wells only");
    n = (long long)p->nx * p->ny * p->nz;
    long long faces = (long long)(p->nx - 1) * p->ny * p->nz + (long long)p->nx * (p->ny - 1) * p->nz +
                      (long long)p->nx * p->ny * (p->nz - 1);
    nnz = n + 2 * faces;
    if (n >= (1LL << 31) / 8 || nnz >= (1LL << 31))
        return fail(BO_ERR_INVALID_ARG, "grid too large for 32-bit block indices");
    return BO_OK;
}

bo_status check2(const bo_problem *p, const double *x_old, const double *x_new, double dt, const bo_bsr2 *J,
                 const double *b) {
    if (!x_old || !x_new || !J || !b || !J->rowptr || !J->colind || !J->val)
        return fail(BO_ERR_INVALID_ARG, "bo_jacobian2_bsr: NULL pointer");
    if (!(dt > 0.0)) return fail(BO_ERR_INVALID_ARG, "bo_jacobian2_bsr: dt must be > 0");
    if (!p->kx || !p->ky || !p->kz || !p->phi0) return fail(BO_ERR_INVALID_ARG, "bo_jacobian2_bsr: NULL field");
    if (p->fluid.nw < 1 || p->fluid.no < 1) return fail(BO_ERR_INVALID_ARG, "Corey exponents must be >= 1");
    if (!(p->fluid.swc + p->fluid.sor < 1.0))
        return fail(BO_ERR_INVALID_ARG, "bo_jacobian2_bsr: needs S_wc + S_or < 1");
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

}  // namespace
}  // namespace bo

using namespace bo;

extern "C" bo_status bo_jacobian2_bsr_size(const bo_problem *p, int32_t *nbrows, int32_t *nnzb) {
    if (!p || !nbrows || !nnzb) return fail(BO_ERR_INVALID_ARG, "bo_jacobian2_bsr_size: NULL argument");
    long long n = 0, nnz = 0;
    BO_TRY(layout2(p, n, nnz));
    *nbrows = (int32_t)n;
    *nnzb = (int32_t)nnz;
    return BO_OK;
}

extern "C" bo_status bo_jacobian2_bsr(const bo_problem *p, const double *x_old, const double *x_new, double dt,
                                      bo_bsr2 *J, double *b, void *stream) {
    if (!p) return fail(BO_ERR_INVALID_ARG, "bo_jacobian2_bsr: NULL problem");
    long long n = 0, nnz = 0;
    BO_TRY(layout2(p, n, nnz));
    BO_TRY(check2(p, x_old, x_new, dt, J, b));
    hipStream_t s = (hipStream_t)stream;
    J->nbrows = (int32_t)n;
    J->nnzb = (int32_t)nnz;
    int32_t *cnt = nullptr;
    BO_TRY(scratch_get(SC_JAC_CNT, sizeof(int32_t) * (size_t)n, (void **)&cnt));
    k_row_counts2<<<grid_for(n), kBlock, 0, s>>>(p->nx, p->ny, p->nz, cnt);
    BO_HIP(hipGetLastError());
    int32_t total = 0;
    BO_TRY(scan_counts(cnt, J->rowptr, (int)n, &total, s));
    if (total != nnz) return fail(BO_ERR_HIP, "row count scan disagrees with the pattern size");
    Grid2 G{p->nx, p->ny, p->nz, p->dx, p->dy, p->dz, p->top_depth, p->kx, p->ky, p->kz, p->phi0};
    const bo_fluid &q = p->fluid;
    Fl2 f{q.p_ref, q.Bw0, q.cw, q.Bo0, q.co, q.mu_w, q.mu_o, q.c_r, q.rho_wsc, q.rho_osc, q.swc, q.sor,
          q.nw, q.no, q.tcoef, q.rb_ft3, q.grav, q.gravity, q.inj_total_mobility};
    const double acc = p->dx * p->dy * p->dz / (q.rb_ft3 * dt);
    k_jac2_cells<<<grid_for(n), kBlock, 0, s>>>(G, f, x_old, x_new, acc, J->rowptr, J->colind, J->val, b);
    BO_HIP(hipGetLastError());
    for (int w0 = 0; w0 < p->nwells; w0 += kWellChunk2) {
        WellChunk2 ch{};
        const int c = std::min(kWellChunk2, p->nwells - w0);
        for (int k = 0; k < c; k++) ch.w[k] = p->wells[w0 + k];
        k_jac2_wells<<<c, 64, 0, s>>>(G, f, x_new, c, ch, J->rowptr, J->colind, J->val, b);
        BO_HIP(hipGetLastError());
    }
    return BO_OK;
}

extern "C" bo_status bo_bsr2_spmv(const bo_bsr2 *A, double alpha, const double *x, double beta, double *y,
                                  void *stream) {
    if (!A || !x || !y || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, "bo_bsr2_spmv: NULL argument");
    if (A->nbrows < 0) return fail(BO_ERR_INVALID_ARG, "bo_bsr2_spmv: negative size");
    if (A->nbrows == 0) return BO_OK;
    k_bsr2_spmv<<<grid_for(A->nbrows), kBlock, 0, (hipStream_t)stream>>>(A->nbrows, A->rowptr, A->colind, A->val,
                                                                         alpha, x, beta, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}
