// Restricted additive Schwarz with ILU(0) subdomain solves on a scalar
// 7-point system: the preconditioner of the paper's pressure-system run
// (Section 3.2 names RAS with an ILU(0) local solver; Section 4.2 times
// GMRES(30) with it for a fixed 90 iterations on one pressure system).
//
// Subdomains are tiles of tile_x x tile_y grid columns (all nz layers),
// extended by `overlap` columns on every side inside the grid.  Each extended
// tile is one wavefront, lane t = a + ex b owning column (i0 - d + a,
// j0 - d + b) and handling layer k = s - a - b at step s (ex = tile_x + 2d,
// ey = tile_y + 2d, ex ey <= 64): a cell's -x, -y and -z neighbours in the
// tile were handled one step earlier.  The subdomain matrix drops the
// couplings that leave the extended tile; its ILU(0) in natural order
// changes only the diagonal on the 7-point graph (no triangles):
//   d_i = a_ii - sum_{k<i} (a_ik / d_k) a_ki     (-z, -y, -x in that order),
//   forward  y_i = r_i - sum_{k<i} (a_ik / d_k) y_k,
//   backward x_i = (y_i - sum_{j>i} a_ij x_j) / d_i   (+x, +y, +z),
// and each tile writes x for its own (non-extended) cells only.
//
// Factors per slot (tile, step, lane): forward [l_-z, l_-y, l_-x, 0] with
// l = a_ik / d_k, backward [d, a_+x, a_+y, a_+z], two double2 each (one
// wavefront load of a double2 reads 1 KB); y in the same order.  The sweeps
// keep the next step's loads in flight while the current step waits for the
// neighbours' values (two shuffles).
//
// The handle is a bo_cpr with block size 1: bo_cpr_apply applies RAS,
// bo_cpr_spmv multiplies by the handle's copy of the coefficients, and
// bo_scalar_solve runs GMRES(m) (or FGMRES) with it.
#include <cmath>
#include "bo_cpr.hpp"

namespace bo {
namespace {

struct RasGeom {
    int nx, ny, nz, tx, ty, ov, ex, ey, ntx, nty, ns;
};

__device__ __forceinline__ size_t ras_pk(const RasGeom &T, int tile, int s, int pair, int lane) {
    return (((size_t)tile * T.ns + s) * 2 + pair) * 64 + lane;
}
__device__ __forceinline__ size_t ras_slot(const RasGeom &T, int tile, int s, int lane) {
    return ((size_t)tile * T.ns + s) * 64 + lane;
}

struct Lane {
    int a, b, i, j;
    bool active, own, has_mx, has_my, has_px, has_py;
};

__device__ __forceinline__ Lane lane_of(const RasGeom &T, int tile, int t) {
    Lane L;
    L.a = t % T.ex;
    L.b = t / T.ex;
    const int ti = tile % T.ntx, tj = tile / T.ntx;
    const int i0 = ti * T.tx, j0 = tj * T.ty;
    L.i = i0 - T.ov + L.a;
    L.j = j0 - T.ov + L.b;
    L.active = t < T.ex * T.ey && L.i >= 0 && L.i < T.nx && L.j >= 0 && L.j < T.ny;
    L.own = L.active && L.i >= i0 && L.i < i0 + T.tx && L.j >= j0 && L.j < j0 + T.ty;
    L.has_mx = L.a > 0 && L.i > 0;
    L.has_my = L.b > 0 && L.j > 0;
    L.has_px = L.a + 1 < T.ex && L.i + 1 < T.nx;
    L.has_py = L.b + 1 < T.ey && L.j + 1 < T.ny;
    return L;
}

// y = alpha A x + beta y, slots in ascending column order
__global__ void __launch_bounds__(kBlock) k_scalar_spmv(int nx, int ny, int nz, const double *__restrict__ A,
                                                        double alpha, const double *__restrict__ x, double beta,
                                                        double *__restrict__ y) {
    const int n = nx * ny * nz;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t N = (size_t)n;
    const int nxy = nx * ny;
    const int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        const int j = nb[q];
        if (j < 0) continue;
        s = s + __builtin_nontemporal_load(A + (size_t)q * N + i) * x[j];
    }
    y[i] = beta == 0.0 ? alpha * s + 0.0 : alpha * s + beta * y[i];
}

// Factorisation, one wavefront per extended tile.
__global__ void __launch_bounds__(64) k_ras_factor(RasGeom T, const double *__restrict__ A,
                                                   double2 *__restrict__ Ff, double2 *__restrict__ Fb,
                                                   int32_t *__restrict__ bad) {
    const int t = threadIdx.x, tile = blockIdx.x;
    const Lane L = lane_of(T, tile, t);
    const size_t N = (size_t)T.nx * T.ny * T.nz;
    double dp = 1.0, uxp = 0.0, uyp = 0.0, uzp = 0.0;  // this lane's d and upper couplings, previous step
    for (int s = 0; s < T.ns; s++) {
        const double dx = __shfl(dp, L.has_mx ? t - 1 : t, 64), ux = __shfl(uxp, L.has_mx ? t - 1 : t, 64);
        const double dy = __shfl(dp, L.has_my ? t - T.ex : t, 64), uy = __shfl(uyp, L.has_my ? t - T.ex : t, 64);
        const int k = s - L.a - L.b;
        if (!(L.active && k >= 0 && k < T.nz)) continue;
        const size_t g = (size_t)L.i + (size_t)T.nx * ((size_t)L.j + (size_t)T.ny * k);
        double d = A[(size_t)S_D * N + g];
        double lz = 0.0, ly = 0.0, lx = 0.0;
        if (k > 0) { lz = A[(size_t)S_MZ * N + g] / dp; d = d - lz * uzp; }
        if (L.has_my) { ly = A[(size_t)S_MY * N + g] / dy; d = d - ly * uy; }
        if (L.has_mx) { lx = A[(size_t)S_MX * N + g] / dx; d = d - lx * ux; }
        if (!(d != 0.0) || !isfinite(d)) *bad = 1;
        dp = d;
        uxp = L.has_px ? A[(size_t)S_PX * N + g] : 0.0;
        uyp = L.has_py ? A[(size_t)S_PY * N + g] : 0.0;
        uzp = k + 1 < T.nz ? A[(size_t)S_PZ * N + g] : 0.0;
        Ff[ras_pk(T, tile, s, 0, t)] = make_double2(lz, ly);
        Ff[ras_pk(T, tile, s, 1, t)] = make_double2(lx, 0.0);
        Fb[ras_pk(T, tile, s, 0, t)] = make_double2(d, uxp);
        Fb[ras_pk(T, tile, s, 1, t)] = make_double2(uyp, uzp);
    }
}

struct RasStep {
    double2 f0, f1;
    double v;
};

// forward sweep: y (slot order) from r (cell order)
__global__ void __launch_bounds__(64) k_ras_forward(RasGeom T, const double2 *__restrict__ Ff,
                                                    const double *__restrict__ r, double *__restrict__ Y) {
    const int t = threadIdx.x, tile = blockIdx.x;
    const Lane L = lane_of(T, tile, t);
    double yp = 0.0;  // this lane's y of the previous step (the -z neighbour)
    auto fetch = [&](int s, RasStep &F) {
        const int sc = min(s, T.ns - 1);
        const int k = sc - L.a - L.b;
        const bool act = L.active && k >= 0 && k < T.nz;
        const int tl = act ? t : 0;
        F.f0 = Ff[ras_pk(T, tile, sc, 0, tl)];
        F.f1 = Ff[ras_pk(T, tile, sc, 1, tl)];
        const size_t g = act ? (size_t)L.i + (size_t)T.nx * ((size_t)L.j + (size_t)T.ny * k) : 0;
        F.v = r[g];
    };
    auto step = [&](int s, const RasStep &F) {
        const double yx = __shfl(yp, L.has_mx ? t - 1 : t, 64);
        const double yy = __shfl(yp, L.has_my ? t - T.ex : t, 64);
        const int k = s - L.a - L.b;
        if (!(L.active && k >= 0 && k < T.nz)) return;
        double y = F.v;
        if (k > 0) y = y - F.f0.x * yp;
        if (L.has_my) y = y - F.f0.y * yy;
        if (L.has_mx) y = y - F.f1.x * yx;
        yp = y;
        Y[ras_slot(T, tile, s, t)] = y;
    };
    RasStep R0, R1;
    fetch(0, R0);
    int s0 = 0;
    for (; s0 + 2 <= T.ns; s0 += 2) {
        fetch(s0 + 1, R1);
        step(s0, R0);
        fetch(s0 + 2, R0);
        step(s0 + 1, R1);
    }
    if (s0 < T.ns) step(s0, R0);
}

// backward sweep: x (cell order, the tile's own cells) from y (slot order)
__global__ void __launch_bounds__(64) k_ras_backward(RasGeom T, const double2 *__restrict__ Fb,
                                                     const double *__restrict__ Y, double *__restrict__ x) {
    const int t = threadIdx.x, tile = blockIdx.x;
    const Lane L = lane_of(T, tile, t);
    double xp = 0.0;  // this lane's x of the later step (the +z neighbour)
    auto fetch = [&](int s, RasStep &F) {
        const int sc = max(s, 0);
        const int k = sc - L.a - L.b;
        const bool act = L.active && k >= 0 && k < T.nz;
        const int tl = act ? t : 0;
        F.f0 = Fb[ras_pk(T, tile, sc, 0, tl)];
        F.f1 = Fb[ras_pk(T, tile, sc, 1, tl)];
        F.v = Y[ras_slot(T, tile, sc, tl)];
    };
    auto step = [&](int s, const RasStep &F) {
        const double xx = __shfl(xp, L.has_px ? t + 1 : t, 64);
        const double xy = __shfl(xp, L.has_py ? t + T.ex : t, 64);
        const int k = s - L.a - L.b;
        if (!(L.active && k >= 0 && k < T.nz)) return;
        double v = F.v;
        if (L.has_px) v = v - F.f0.y * xx;
        if (L.has_py) v = v - F.f1.x * xy;
        if (k + 1 < T.nz) v = v - F.f1.y * xp;
        xp = v / F.f0.x;
        if (L.own) x[(size_t)L.i + (size_t)T.nx * ((size_t)L.j + (size_t)T.ny * k)] = xp;
    };
    RasStep R0, R1;
    fetch(T.ns - 1, R0);
    int s0 = T.ns - 1;
    for (; s0 - 2 >= -1; s0 -= 2) {
        fetch(s0 - 1, R1);
        step(s0, R0);
        fetch(s0 - 2, R0);
        step(s0 - 1, R1);
    }
    if (s0 >= 0) step(s0, R0);
}

__global__ void k_check_finite1(long long n, const double *__restrict__ v, int32_t *__restrict__ bad) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(v[i])) *bad = 1;
}

RasGeom ras_geom(const bo_cpr *pc) {
    RasGeom T{};
    T.nx = pc->g.nx; T.ny = pc->g.ny; T.nz = pc->g.nz;
    T.tx = pc->o.tile_x; T.ty = pc->o.tile_y; T.ov = pc->ras_overlap;
    T.ex = T.tx + 2 * T.ov;
    T.ey = T.ty + 2 * T.ov;
    T.ntx = (T.nx + T.tx - 1) / T.tx;
    T.nty = (T.ny + T.ty - 1) / T.ty;
    T.ns = T.nz + T.ex + T.ey - 2;
    return T;
}

}  // namespace

bo_status scalar_spmv(const Grid &g, const double *A, double alpha, const double *x, double beta, double *y,
                      hipStream_t s) {
    k_scalar_spmv<<<grid_for(g.n()), kBlock, 0, s>>>(g.nx, g.ny, g.nz, A, alpha, x, beta, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status ras_apply(bo_cpr *pc, const double *r, double *z, hipStream_t s) {
    const RasGeom T = ras_geom(pc);
    const int tiles = T.ntx * T.nty;
    k_ras_forward<<<tiles, 64, 0, s>>>(T, pc->ilu_f.p, r, pc->ilu_w.p);
    BO_HIP(hipGetLastError());
    k_ras_backward<<<tiles, 64, 0, s>>>(T, pc->ilu_b.p, pc->ilu_w.p, z);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

static bo_status ras_setup_impl(const bo_grid *grid, const double *coef, const bo_ras_opts *o, bo_cpr *pc,
                                hipStream_t s) {
    pc->bs = 1;
    pc->has_grid = true;
    pc->general = false;
    pc->g = Grid{grid->nx, grid->ny, grid->nz};
    pc->n = (int)pc->g.n();
    pc->ncell = pc->n;
    pc->npr = pc->n;
    pc->nnzb = 0;
    bo_cpr_default_opts(&pc->o);
    pc->o.use_amg = 0;
    pc->o.tile_x = o->tile_x;
    pc->o.tile_y = o->tile_y;
    pc->ras_overlap = o->overlap;
    const long long n = pc->n;
    BO_TRY(pc->flag.alloc(1));
    BO_TRY(pc->A.alloc(7 * n));
    BO_HIP(hipMemsetAsync(pc->flag.p, 0, sizeof(int32_t), s));
    k_check_finite1<<<grid_for(7 * n), kBlock, 0, s>>>(7 * n, coef, pc->flag.p);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    HostRead rd{pc->flag.p, sizeof bad, &bad};
    BO_TRY(host_reads(&rd, 1, s));
    if (bad) return fail(BO_ERR_NONFINITE, "bo_ras_setup: the coefficients hold NaN or Inf");
    BO_HIP(hipMemcpyAsync(pc->A.p, coef, sizeof(double) * 7 * n, hipMemcpyDeviceToDevice, s));
    const RasGeom T = ras_geom(pc);
    const size_t slots = (size_t)T.ntx * T.nty * T.ns * 64;
    BO_TRY(pc->ilu_f.alloc(2 * slots));
    BO_TRY(pc->ilu_b.alloc(2 * slots));
    BO_TRY(pc->ilu_w.alloc(slots));
    k_ras_factor<<<T.ntx * T.nty, 64, 0, s>>>(T, pc->A.p, pc->ilu_f.p, pc->ilu_b.p, pc->flag.p);
    BO_HIP(hipGetLastError());
    BO_TRY(host_reads(&rd, 1, s));
    if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "bo_ras_setup: a zero or non-finite ILU(0) pivot");
    BO_TRY(pc->t3a.alloc(n));
    BO_TRY(pc->red.init());
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}

}  // namespace bo

using namespace bo;

extern "C" void bo_ras_default_opts(bo_ras_opts *o) {
    if (!o) return;
    o->tile_x = 6;
    o->tile_y = 6;
    o->overlap = 1;
}

extern "C" bo_status bo_scalar_spmv(const bo_grid *grid, const double *coef, double alpha, const double *x,
                                    double beta, double *y, void *stream) {
    if (!grid || !coef || !x || !y) return fail(BO_ERR_INVALID_ARG, "bo_scalar_spmv: NULL argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || (long long)grid->nx * grid->ny * grid->nz >= (1LL << 31))
        return fail(BO_ERR_INVALID_ARG, "bo_scalar_spmv: grid dimensions out of range");
    return scalar_spmv(Grid{grid->nx, grid->ny, grid->nz}, coef, alpha, x, beta, y, (hipStream_t)stream);
}

extern "C" bo_status bo_ras_setup(const bo_grid *grid, const double *coef, const bo_ras_opts *opts,
                                  const bo_allocator *alloc, bo_cpr **out, void *stream) {
    if (!out) return fail(BO_ERR_INVALID_ARG, "bo_ras_setup: out is NULL");
    *out = nullptr;
    if (!grid || !coef || !opts) return fail(BO_ERR_INVALID_ARG, "bo_ras_setup: NULL argument");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || grid->dual)
        return fail(BO_ERR_INVALID_ARG, "bo_ras_setup: grid dimensions out of range");
    if ((long long)grid->nx * grid->ny * grid->nz >= (1LL << 31))
        return fail(BO_ERR_INVALID_ARG, "bo_ras_setup: grid too large for 32-bit cell indices");
    if (opts->tile_x < 1 || opts->tile_y < 1 || opts->overlap < 0 ||
        (opts->tile_x + 2 * opts->overlap) * (opts->tile_y + 2 * opts->overlap) > 64)
        return fail(BO_ERR_INVALID_ARG, "bo_ras_setup: extended tiles need (tile_x + 2 overlap)(tile_y + 2 overlap) <= 64");
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(BO_ERR_INVALID_ARG, "bo_ras_setup: an allocator needs both alloc and free");
    bo_cpr *pc = new (std::nothrow) bo_cpr();
    if (!pc) return fail(BO_ERR_ALLOC, "bo_ras_setup: out of host memory");
    if (alloc) {
        pc->has_alloc = true;
        pc->alloc = *alloc;
    }
    AllocScope scope(pc->allocator(), stream);
    bo_status st = ras_setup_impl(grid, coef, opts, pc, (hipStream_t)stream);
    if (st != BO_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        bo_cpr_destroy(pc);
        return st;
    }
    *out = pc;
    return BO_OK;
}

extern "C" bo_status bo_ras_update(bo_cpr *pc, const double *coef, void *stream) {
    if (!pc || !coef) return fail(BO_ERR_INVALID_ARG, "bo_ras_update: NULL argument");
    if (pc->bs != 1) return fail(BO_ERR_INVALID_ARG, "bo_ras_update: not a bo_ras_setup handle");
    AllocScope scope(pc->allocator(), stream);
    const bo_grid g{pc->g.nx, pc->g.ny, pc->g.nz, 0};
    const bo_ras_opts o{pc->o.tile_x, pc->o.tile_y, pc->ras_overlap};
    bo_status st = ras_setup_impl(&g, coef, &o, pc, (hipStream_t)stream);
    if (st != BO_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        pc->broken = true;
    } else {
        pc->broken = false;
    }
    return st;
}

extern "C" bo_status bo_scalar_solve(bo_cpr *pc, const double *coef, const double *b, double *x,
                                     const bo_fgmres_opts *opts, bo_solve_stats *stats, void *stream) {
    if (!pc || !coef || !b || !x || !opts) return fail(BO_ERR_INVALID_ARG, "bo_scalar_solve: NULL argument");
    if (pc->bs != 1) return fail(BO_ERR_INVALID_ARG, "bo_scalar_solve: not a bo_ras_setup handle");
    if (pc->broken) return fail(BO_ERR_INVALID_ARG, "bo_scalar_solve: the last bo_ras_update failed");
    if (opts->m < 1 || opts->m > 64 || opts->maxit < 0 || !(opts->rtol > 0.0) || opts->orth < 0 ||
        opts->orth > 2 || (opts->timing != 0 && opts->timing != 1) || (opts->graph != 0 && opts->graph != 1) ||
        (opts->flexible != 0 && opts->flexible != 1))
        return fail(BO_ERR_INVALID_ARG, "bo_scalar_solve: options out of range");
    AllocScope scope(pc->allocator(), stream);
    return fgmres_core(pc, UserA{nullptr, nullptr, coef}, b, x, opts, stats, (hipStream_t)stream);
}
