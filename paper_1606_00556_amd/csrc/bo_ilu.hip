// F stage of CPR (Section 3.2): the paper's restricted additive Schwarz with
// ILU(0) subdomain solves, mapped onto the GPU as non-overlapping subdomains
// of tile_x x tile_y grid columns (all nz layers), one wavefront per tile.
//
// On the 7-point stencil the grid graph has no triangles, so block ILU(0)
// only modifies the diagonal blocks: E_i = A_ii - sum_{k<i} A_ik E_k^{-1} A_ki
// over the lower neighbours k inside the tile (natural order: -z, -y, -x).
// The solve is w_i = E_i^{-1}(r_i - sum_{k<i} A_ik w_k) followed by
// x_i = w_i - E_i^{-1} sum_{j>i} A_ij x_j.
//
// Schedule: lane t = a + tile_x*b of the tile's wavefront owns grid column
// (i0+a, j0+b) and at step s handles layer k = s - a - b, so its -x, -y and
// -z neighbours were handled one step earlier by lanes t-1, t-tile_x and t
// itself; their values arrive through cross-lane shuffles (no LDS, no
// barriers).  The factors are stored in the same (tile, step, lane) order,
// packed in pairs, so each step reads its 36 doubles with 18 contiguous 1 KB
// wavefront loads, and the fields of the next two steps are loaded before the
// current step is computed.  Block Jacobi (x_i = A_ii^{-1} r_i) is the alternative F
// stage.
#include "bo_cpr.hpp"

namespace bo {
namespace {

struct TileGeom {
    int nx, ny, nz, tx, ty, ntx, nty, ns;
    __host__ __device__ long long slots() const { return (long long)ntx * nty * ns * 64; }
};

// The factors of one slot for one sweep are 36 doubles: E^{-1} and the three
// lower blocks (-z, -y, -x) for the forward sweep, E^{-1} and the three upper
// blocks (+x, +y, +z) for the backward sweep.  They are packed as 18 double2
// per slot in (tile, step, pair, lane) order, so one wavefront load of a
// pair reads 1 KB contiguously and a step needs 18 load instructions.
constexpr int kPairs = 18;
__device__ __forceinline__ size_t pk_index(int tile, int ns, int s, int pair, int lane) {
    return (((size_t)tile * ns + s) * kPairs + pair) * 64 + lane;
}

__device__ __forceinline__ void load_blk(const double *__restrict__ A, int slot, size_t N, int g, double *o) {
    const double *p = A + (size_t)slot * 9 * N + g;
#pragma unroll
    for (int z = 0; z < 9; z++) o[z] = p[(size_t)z * N];
}

__device__ __forceinline__ void mv3(const double *A, const double *x, double *y) {
    y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    y[1] = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    y[2] = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
}

template <int K>
__device__ __forceinline__ void shfl_arr(const double *src, double *dst, int lane) {
#pragma unroll
    for (int z = 0; z < K; z++) dst[z] = __shfl(src[z], lane, 64);
}

// Factorisation: writes E^{-1}, the lower blocks (-z,-y,-x) and upper blocks
// (+x,+y,+z) of each cell (zero where the neighbour lies outside the tile or
// grid) into the (tile, step, lane) layout, and the cell index of each slot
// (-1 for idle slots).  E^{-1} by Gauss-Jordan with partial pivoting.
__global__ void __launch_bounds__(64) k_ilu_factor(TileGeom T, const double *__restrict__ A,
                                                   double2 *__restrict__ Ff, double2 *__restrict__ Fb,
                                                   int32_t *__restrict__ cell, int32_t *__restrict__ slot_of,
                                                   int32_t *__restrict__ bad) {
    int t = threadIdx.x;
    int a = t % T.tx, b = t / T.tx;
    int tile = blockIdx.x;
    int ti = tile % T.ntx, tj = tile / T.ntx;
    int i = ti * T.tx + a, j = tj * T.ty + b;
    bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    bool has_mx = a > 0, has_my = b > 0;
    bool has_px = a + 1 < T.tx && i + 1 < T.nx, has_py = b + 1 < T.ty && j + 1 < T.ny;
    size_t N = (size_t)T.nx * T.ny * T.nz;
    double Ep[9], Uxp[9], Uyp[9], Uzp[9];  // this lane's values from the previous step
    for (int z = 0; z < 9; z++) Ep[z] = Uxp[z] = Uyp[z] = Uzp[z] = 0.0;
    for (int s = 0; s < T.ns; s++) {
        // neighbours' previous-step values (every lane takes part in the shuffles)
        double Ex[9], Ey[9], Ux[9], Uy[9];
        shfl_arr<9>(Ep, Ex, has_mx ? t - 1 : t);
        shfl_arr<9>(Uxp, Ux, has_mx ? t - 1 : t);
        shfl_arr<9>(Ep, Ey, has_my ? t - T.tx : t);
        shfl_arr<9>(Uyp, Uy, has_my ? t - T.tx : t);
        int k = s - a - b;
        size_t q = ((size_t)tile * T.ns + s) * 64 + t;
        if (active && k >= 0 && k < T.nz) {
            int g = i + T.nx * (j + T.ny * k);
            double E[9], L[9], Lk[9], tmp[9];
            double fw[36], bw[36];  // packed slot data: [E^{-1} | Lz Ly Lx] and [E^{-1} | Ux Uy Uz]
            for (int z = 0; z < 36; z++) fw[z] = bw[z] = 0.0;
            load_blk(A, S_D, N, g, E);
            // -z, -y, -x in ascending order
            if (k > 0) {
                load_blk(A, S_MZ, N, g, L);
                mul3(L, Ep, Lk); mul3(Lk, Uzp, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
                for (int z = 0; z < 9; z++) fw[9 + z] = L[z];
            }
            if (has_my) {
                load_blk(A, S_MY, N, g, L);
                mul3(L, Ey, Lk); mul3(Lk, Uy, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
                for (int z = 0; z < 9; z++) fw[18 + z] = L[z];
            }
            if (has_mx) {
                load_blk(A, S_MX, N, g, L);
                mul3(L, Ex, Lk); mul3(Lk, Ux, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
                for (int z = 0; z < 9; z++) fw[27 + z] = L[z];
            }
            double Ei[9];
            if (!inv3_gj(E, Ei)) {
                *bad = 1;
                for (int z = 0; z < 9; z++) Ei[z] = 0.0;
            }
            for (int z = 0; z < 9; z++) { fw[z] = Ei[z]; bw[z] = Ei[z]; Ep[z] = Ei[z]; }
            // upper blocks: this row's +x, +y, +z (zero outside the tile)
            if (has_px) load_blk(A, S_PX, N, g, Uxp); else for (int z = 0; z < 9; z++) Uxp[z] = 0.0;
            if (has_py) load_blk(A, S_PY, N, g, Uyp); else for (int z = 0; z < 9; z++) Uyp[z] = 0.0;
            if (k + 1 < T.nz) load_blk(A, S_PZ, N, g, Uzp); else for (int z = 0; z < 9; z++) Uzp[z] = 0.0;
            for (int z = 0; z < 9; z++) { bw[9 + z] = Uxp[z]; bw[18 + z] = Uyp[z]; bw[27 + z] = Uzp[z]; }
            for (int p2 = 0; p2 < kPairs; p2++) {
                Ff[pk_index(tile, T.ns, s, p2, t)] = make_double2(fw[2 * p2], fw[2 * p2 + 1]);
                Fb[pk_index(tile, T.ns, s, p2, t)] = make_double2(bw[2 * p2], bw[2 * p2 + 1]);
            }
            cell[q] = g;
            slot_of[g] = (int32_t)q;
        } else {
            cell[q] = -1;
        }
    }
}

struct Pack {
    double v[36];
    double w[3];   // the sweep's vector operand at this slot
    int g;
};

__device__ __forceinline__ void load_pack(const double2 *__restrict__ F, const int32_t *__restrict__ cell,
                                          const double *__restrict__ vec, size_t S, int tile, int ns, int s, int t,
                                          Pack &p) {
    size_t q = ((size_t)tile * ns + s) * 64 + t;
    p.g = cell[q];
#pragma unroll
    for (int p2 = 0; p2 < kPairs; p2++) {
        double2 d = F[pk_index(tile, ns, s, p2, t)];
        p.v[2 * p2] = d.x;
        p.v[2 * p2 + 1] = d.y;
    }
    p.w[0] = vec[q]; p.w[1] = vec[S + q]; p.w[2] = vec[2 * S + q];
}

// scatter a natural-order 3N vector into (tile, step, lane) order
__global__ void k_to_slots(long long n, const int32_t *__restrict__ slot_of, size_t S, const double *__restrict__ r,
                           double *__restrict__ rq) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t q = (size_t)slot_of[g];
    rq[q] = r[3 * g]; rq[S + q] = r[3 * g + 1]; rq[2 * S + q] = r[3 * g + 2];
}

// forward sweep: w = E^{-1}(r - L w_lower); r and w in (tile, step, lane) order
__global__ void __launch_bounds__(64) k_ilu_forward(TileGeom T, const double2 *__restrict__ F,
                                                    const int32_t *__restrict__ cell, const double *__restrict__ rq,
                                                    double *__restrict__ wq) {
    int t = threadIdx.x;
    int a = t % T.tx, b = t / T.tx;
    int tile = blockIdx.x;
    size_t S = (size_t)T.slots();
    int lx = a > 0 ? t - 1 : t, ly = b > 0 ? t - T.tx : t;
    double wp[3] = {0.0, 0.0, 0.0};
    // two steps of operands in flight ahead of the one being computed
    Pack cur, n1, n2;
    load_pack(F, cell, rq, S, tile, T.ns, 0, t, n1);
    if (T.ns > 1) load_pack(F, cell, rq, S, tile, T.ns, 1, t, n2);
    for (int s = 0; s < T.ns; s++) {
        cur = n1;
        n1 = n2;
        if (s + 2 < T.ns) load_pack(F, cell, rq, S, tile, T.ns, s + 2, t, n2);
        double wy[3], wx[3];
        for (int c = 0; c < 3; c++) { wx[c] = __shfl(wp[c], lx, 64); wy[c] = __shfl(wp[c], ly, 64); }
        if (cur.g >= 0) {
            double v[3] = {cur.w[0], cur.w[1], cur.w[2]};
            double y[3];
            // zero blocks stand for missing neighbours
            mv3(cur.v + 9, wp, y); v[0] = v[0] - y[0]; v[1] = v[1] - y[1]; v[2] = v[2] - y[2];
            mv3(cur.v + 18, wy, y); v[0] = v[0] - y[0]; v[1] = v[1] - y[1]; v[2] = v[2] - y[2];
            mv3(cur.v + 27, wx, y); v[0] = v[0] - y[0]; v[1] = v[1] - y[1]; v[2] = v[2] - y[2];
            mv3(cur.v, v, wp);
            size_t q = ((size_t)tile * T.ns + s) * 64 + t;
            wq[q] = wp[0]; wq[S + q] = wp[1]; wq[2 * S + q] = wp[2];
        } else {
            wp[0] = wp[1] = wp[2] = 0.0;
        }
    }
}

// backward sweep: x_i = w_i - E_i^{-1} sum_{upper} A_ij x_j, written in
// natural order as out = x + (dp, 0, 0) (dp may be NULL)
__global__ void __launch_bounds__(64) k_ilu_backward(TileGeom T, const double2 *__restrict__ F,
                                                     const int32_t *__restrict__ cell, const double *__restrict__ wq,
                                                     const double *__restrict__ dp, double *__restrict__ out) {
    int t = threadIdx.x;
    int a = t % T.tx, b = t / T.tx;
    int tile = blockIdx.x;
    size_t S = (size_t)T.slots();
    int px = a + 1 < T.tx && t + 1 < 64 ? t + 1 : t;
    int py = b + 1 < T.ty && t + T.tx < 64 ? t + T.tx : t;
    double xp[3] = {0.0, 0.0, 0.0};
    Pack cur, n1, n2;
    load_pack(F, cell, wq, S, tile, T.ns, T.ns - 1, t, n1);
    if (T.ns > 1) load_pack(F, cell, wq, S, tile, T.ns, T.ns - 2, t, n2);
    for (int s = T.ns - 1; s >= 0; s--) {
        cur = n1;
        n1 = n2;
        if (s >= 2) load_pack(F, cell, wq, S, tile, T.ns, s - 2, t, n2);
        double xx[3], xy[3];
        for (int c = 0; c < 3; c++) { xx[c] = __shfl(xp[c], px, 64); xy[c] = __shfl(xp[c], py, 64); }
        if (cur.g >= 0) {
            double acc[3], y[3];
            mv3(cur.v + 9, xx, acc);
            mv3(cur.v + 18, xy, y); acc[0] = acc[0] + y[0]; acc[1] = acc[1] + y[1]; acc[2] = acc[2] + y[2];
            mv3(cur.v + 27, xp, y); acc[0] = acc[0] + y[0]; acc[1] = acc[1] + y[1]; acc[2] = acc[2] + y[2];
            mv3(cur.v, acc, y);
            xp[0] = cur.w[0] - y[0]; xp[1] = cur.w[1] - y[1]; xp[2] = cur.w[2] - y[2];
            size_t g = (size_t)cur.g;
            out[3 * g] = dp ? dp[g] + xp[0] : xp[0];
            out[3 * g + 1] = xp[1];
            out[3 * g + 2] = xp[2];
        } else {
            xp[0] = xp[1] = xp[2] = 0.0;
        }
    }
}

__global__ void k_bj_setup(long long n, const double *__restrict__ A, double *__restrict__ einv,
                           int32_t *__restrict__ bad) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t N = (size_t)n;
    double E[9], Ei[9];
    load_blk(A, S_D, N, (int)g, E);
    if (!inv3_gj(E, Ei)) {
        *bad = 1;
        for (int z = 0; z < 9; z++) Ei[z] = 0.0;
    }
    for (int z = 0; z < 9; z++) einv[(size_t)z * N + g] = Ei[z];
}

__global__ void k_bj_apply(long long n, const double *__restrict__ einv, const double *__restrict__ r,
                           const double *__restrict__ dp, double *__restrict__ out) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t N = (size_t)n;
    double Ei[9], v[3] = {r[3 * g], r[3 * g + 1], r[3 * g + 2]}, o[3];
    for (int z = 0; z < 9; z++) Ei[z] = einv[(size_t)z * N + g];
    mv3(Ei, v, o);
    out[3 * g] = dp ? dp[g] + o[0] : o[0];
    out[3 * g + 1] = o[1];
    out[3 * g + 2] = o[2];
}

TileGeom geom(const bo_cpr *pc) {
    TileGeom T;
    T.nx = pc->g.nx; T.ny = pc->g.ny; T.nz = pc->g.nz;
    T.tx = pc->o.tile_x; T.ty = pc->o.tile_y;
    T.ntx = (T.nx + T.tx - 1) / T.tx;
    T.nty = (T.ny + T.ty - 1) / T.ty;
    T.ns = (T.tx - 1) + (T.ty - 1) + T.nz;
    return T;
}

}  // namespace

bo_status fstage_setup(bo_cpr *pc, hipStream_t s) {
    long long n = pc->n;
    BO_HIP(hipMemsetAsync(pc->flag.p, 0, sizeof(int32_t), s));
    if (pc->o.ftype == BO_F_BJ) {
        BO_TRY(pc->einv.alloc(9 * n));
        k_bj_setup<<<grid_for(n), kBlock, 0, s>>>(n, pc->A.p, pc->einv.p, pc->flag.p);
    } else {
        TileGeom T = geom(pc);
        size_t S = (size_t)T.slots();
        BO_TRY(pc->ilu_f.alloc(S * kPairs));
        BO_TRY(pc->ilu_b.alloc(S * kPairs));
        BO_TRY(pc->ilu_cell.alloc(S));
        BO_TRY(pc->ilu_slot.alloc(n));
        BO_TRY(pc->ilu_w.alloc(3 * S));
        BO_TRY(pc->ilu_r.alloc(3 * S));
        // idle slots keep zero factors
        BO_HIP(hipMemsetAsync(pc->ilu_f.p, 0, sizeof(double2) * S * kPairs, s));
        BO_HIP(hipMemsetAsync(pc->ilu_b.p, 0, sizeof(double2) * S * kPairs, s));
        k_ilu_factor<<<T.ntx * T.nty, 64, 0, s>>>(T, pc->A.p, pc->ilu_f.p, pc->ilu_b.p, pc->ilu_cell.p,
                                                   pc->ilu_slot.p, pc->flag.p);
    }
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    BO_HIP(hipMemcpyAsync(&bad, pc->flag.p, sizeof bad, hipMemcpyDeviceToHost, s));
    BO_HIP(hipStreamSynchronize(s));
    if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "F stage: singular 3x3 pivot block");
    return BO_OK;
}

// out = F(r) (+ Pi_p dp when dp != NULL).  With r_in_slots the residual is
// already in the F stage's slot order (pc->ilu_r, written by the caller).
bo_status fstage_apply(bo_cpr *pc, const double *r, const double *dp, double *out, bool r_in_slots, hipStream_t s) {
    long long n = pc->n;
    if (pc->o.ftype == BO_F_BJ) {
        k_bj_apply<<<grid_for(n), kBlock, 0, s>>>(n, pc->einv.p, r, dp, out);
    } else {
        TileGeom T = geom(pc);
        size_t S = (size_t)T.slots();
        if (!r_in_slots) k_to_slots<<<grid_for(n), kBlock, 0, s>>>(n, pc->ilu_slot.p, S, r, pc->ilu_r.p);
        k_ilu_forward<<<T.ntx * T.nty, 64, 0, s>>>(T, pc->ilu_f.p, pc->ilu_cell.p, pc->ilu_r.p, pc->ilu_w.p);
        k_ilu_backward<<<T.ntx * T.nty, 64, 0, s>>>(T, pc->ilu_b.p, pc->ilu_cell.p, pc->ilu_w.p, dp, out);
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

size_t fstage_slots(const bo_cpr *pc) { return (size_t)geom(pc).slots(); }

}  // namespace bo
