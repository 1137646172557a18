// F stage of CPR (Section 3.2): the paper's restricted additive Schwarz with
// ILU(0) subdomain solves, mapped onto the GPU as non-overlapping subdomains
// of tile_x x tile_y grid columns (all nz layers), one wavefront per tile.
//
// On the 7-point stencil the grid graph has no triangles, so block ILU(0)
// only modifies the diagonal blocks: E_i = A_ii - sum_{k<i} A_ik E_k^{-1} A_ki
// over the lower neighbours k inside the tile (natural order: -z, -y, -x).
// The solve is w_i = E_i^{-1}(r_i - sum_{k<i} A_ik w_k) followed by
// x_i = w_i - E_i^{-1} sum_{j>i} A_ij x_j.  Inside a tile thread (a,b) owns
// column (i0+a, j0+b) and at step s handles layer k = s - a - b, so each cell's
// lower (upper) neighbours were finished one step earlier (later); their
// values pass through a double-buffered LDS array.  The inverse pivots E^{-1}
// are stored SoA (9 x N).  Block Jacobi (x_i = A_ii^{-1} r_i) is the
// alternative F stage.
#include "bo_cpr.hpp"

namespace bo {
namespace {

constexpr int kTileThreads = 64;

struct TileGeom {
    int nx, ny, nz, tx, ty, ntx;
};

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

__global__ void __launch_bounds__(kTileThreads) k_ilu_factor(TileGeom T, const double *__restrict__ A,
                                                             double *__restrict__ einv, int32_t *__restrict__ bad) {
    __shared__ double Es[2][kTileThreads][9];
    int t = threadIdx.x;
    int a = t % T.tx, b = t / T.tx;
    int ti = blockIdx.x % T.ntx, tj = blockIdx.x / T.ntx;
    int i = ti * T.tx + a, j = tj * T.ty + b;
    bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    size_t N = (size_t)T.nx * T.ny * T.nz;
    int nxy = T.nx * T.ny;
    int steps = (T.tx - 1) + (T.ty - 1) + T.nz;
    for (int s = 0; s < steps; s++) {
        int k = s - a - b;
        int cur = s & 1, prv = cur ^ 1;
        if (active && k >= 0 && k < T.nz) {
            int g = i + T.nx * (j + T.ny * k);
            double E[9], L[9], U[9], Lk[9], tmp[9];
            load_blk(A, S_D, N, g, E);
            // lower neighbours in ascending order: -z, -y, -x
            if (k > 0) {
                load_blk(A, S_MZ, N, g, L);
                load_blk(A, S_PZ, N, g - nxy, U);
                mul3(L, Es[prv][t], Lk);
                mul3(Lk, U, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
            }
            if (b > 0) {
                load_blk(A, S_MY, N, g, L);
                load_blk(A, S_PY, N, g - T.nx, U);
                mul3(L, Es[prv][t - T.tx], Lk);
                mul3(Lk, U, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
            }
            if (a > 0) {
                load_blk(A, S_MX, N, g, L);
                load_blk(A, S_PX, N, g - 1, U);
                mul3(L, Es[prv][t - 1], Lk);
                mul3(Lk, U, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
            }
            double Ei[9];
            if (!inv3_gj(E, Ei)) {
                *bad = 1;
                for (int z = 0; z < 9; z++) Ei[z] = 0.0;
            }
            for (int z = 0; z < 9; z++) {
                Es[cur][t][z] = Ei[z];
                einv[(size_t)z * N + g] = Ei[z];
            }
        }
        __syncthreads();
    }
}

// forward sweep: w = (E + A_L)^{-1}-type solve, stored in w (3N)
__global__ void __launch_bounds__(kTileThreads) k_ilu_forward(TileGeom T, const double *__restrict__ A,
                                                              const double *__restrict__ einv,
                                                              const double *__restrict__ r, double *__restrict__ w) {
    __shared__ double Ws[2][kTileThreads][3];
    int t = threadIdx.x;
    int a = t % T.tx, b = t / T.tx;
    int ti = blockIdx.x % T.ntx, tj = blockIdx.x / T.ntx;
    int i = ti * T.tx + a, j = tj * T.ty + b;
    bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    size_t N = (size_t)T.nx * T.ny * T.nz;
    int steps = (T.tx - 1) + (T.ty - 1) + T.nz;
    for (int s = 0; s < steps; s++) {
        int k = s - a - b;
        int cur = s & 1, prv = cur ^ 1;
        if (active && k >= 0 && k < T.nz) {
            int g = i + T.nx * (j + T.ny * k);
            double v[3] = {r[3 * (size_t)g], r[3 * (size_t)g + 1], r[3 * (size_t)g + 2]};
            double L[9], y[3];
            if (k > 0) {
                load_blk(A, S_MZ, N, g, L);
                mv3(L, Ws[prv][t], y);
                v[0] = v[0] - y[0]; v[1] = v[1] - y[1]; v[2] = v[2] - y[2];
            }
            if (b > 0) {
                load_blk(A, S_MY, N, g, L);
                mv3(L, Ws[prv][t - T.tx], y);
                v[0] = v[0] - y[0]; v[1] = v[1] - y[1]; v[2] = v[2] - y[2];
            }
            if (a > 0) {
                load_blk(A, S_MX, N, g, L);
                mv3(L, Ws[prv][t - 1], y);
                v[0] = v[0] - y[0]; v[1] = v[1] - y[1]; v[2] = v[2] - y[2];
            }
            double Ei[9], o[3];
            for (int z = 0; z < 9; z++) Ei[z] = einv[(size_t)z * N + g];
            mv3(Ei, v, o);
            for (int c = 0; c < 3; c++) {
                Ws[cur][t][c] = o[c];
                w[3 * (size_t)g + c] = o[c];
            }
        }
        __syncthreads();
    }
}

// backward sweep: x_i = w_i - E_i^{-1} sum_{upper} A_ij x_j; writes
// out = x + (dp, 0, 0) when dp != NULL, else out = x.
__global__ void __launch_bounds__(kTileThreads) k_ilu_backward(TileGeom T, const double *__restrict__ A,
                                                               const double *__restrict__ einv,
                                                               const double *__restrict__ w,
                                                               const double *__restrict__ dp,
                                                               double *__restrict__ out) {
    __shared__ double Xs[2][kTileThreads][3];
    int t = threadIdx.x;
    int a = t % T.tx, b = t / T.tx;
    int ti = blockIdx.x % T.ntx, tj = blockIdx.x / T.ntx;
    int i = ti * T.tx + a, j = tj * T.ty + b;
    bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    bool has_px = a + 1 < T.tx && i + 1 < T.nx;
    bool has_py = b + 1 < T.ty && j + 1 < T.ny;
    size_t N = (size_t)T.nx * T.ny * T.nz;
    int steps = (T.tx - 1) + (T.ty - 1) + T.nz;
    for (int s = steps - 1; s >= 0; s--) {
        int k = s - a - b;
        int cur = s & 1, nxt = cur ^ 1;
        if (active && k >= 0 && k < T.nz) {
            int g = i + T.nx * (j + T.ny * k);
            double acc[3] = {0.0, 0.0, 0.0};
            double U[9], y[3];
            if (has_px) {
                load_blk(A, S_PX, N, g, U);
                mv3(U, Xs[nxt][t + 1], y);
                acc[0] = acc[0] + y[0]; acc[1] = acc[1] + y[1]; acc[2] = acc[2] + y[2];
            }
            if (has_py) {
                load_blk(A, S_PY, N, g, U);
                mv3(U, Xs[nxt][t + T.tx], y);
                acc[0] = acc[0] + y[0]; acc[1] = acc[1] + y[1]; acc[2] = acc[2] + y[2];
            }
            if (k + 1 < T.nz) {
                load_blk(A, S_PZ, N, g, U);
                mv3(U, Xs[nxt][t], y);
                acc[0] = acc[0] + y[0]; acc[1] = acc[1] + y[1]; acc[2] = acc[2] + y[2];
            }
            double Ei[9], c3[3];
            for (int z = 0; z < 9; z++) Ei[z] = einv[(size_t)z * N + g];
            mv3(Ei, acc, c3);
            double x0 = w[3 * (size_t)g] - c3[0];
            double x1 = w[3 * (size_t)g + 1] - c3[1];
            double x2 = w[3 * (size_t)g + 2] - c3[2];
            Xs[cur][t][0] = x0; Xs[cur][t][1] = x1; Xs[cur][t][2] = x2;
            out[3 * (size_t)g] = dp ? dp[g] + x0 : x0;
            out[3 * (size_t)g + 1] = x1;
            out[3 * (size_t)g + 2] = x2;
        }
        __syncthreads();
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
    return T;
}

}  // namespace

bo_status fstage_setup(bo_cpr *pc, hipStream_t s) {
    long long n = pc->n;
    BO_TRY(pc->einv.alloc(9 * n));
    BO_HIP(hipMemsetAsync(pc->flag.p, 0, sizeof(int32_t), s));
    if (pc->o.ftype == BO_F_BJ) {
        k_bj_setup<<<grid_for(n), kBlock, 0, s>>>(n, pc->A.p, pc->einv.p, pc->flag.p);
    } else {
        TileGeom T = geom(pc);
        int nty = (T.ny + T.ty - 1) / T.ty;
        k_ilu_factor<<<T.ntx * nty, kTileThreads, 0, s>>>(T, pc->A.p, pc->einv.p, pc->flag.p);
    }
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    BO_HIP(hipMemcpyAsync(&bad, pc->flag.p, sizeof bad, hipMemcpyDeviceToHost, s));
    BO_HIP(hipStreamSynchronize(s));
    if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "F stage: singular 3x3 pivot block");
    return BO_OK;
}

// out = F(r) (+ Pi_p dp when dp != NULL); wbuf is 3N scratch
bo_status fstage_apply(bo_cpr *pc, const double *r, const double *dp, double *out, double *wbuf, hipStream_t s) {
    long long n = pc->n;
    if (pc->o.ftype == BO_F_BJ) {
        k_bj_apply<<<grid_for(n), kBlock, 0, s>>>(n, pc->einv.p, r, dp, out);
    } else {
        TileGeom T = geom(pc);
        int nty = (T.ny + T.ty - 1) / T.ty;
        k_ilu_forward<<<T.ntx * nty, kTileThreads, 0, s>>>(T, pc->A.p, pc->einv.p, r, wbuf);
        k_ilu_backward<<<T.ntx * nty, kTileThreads, 0, s>>>(T, pc->A.p, pc->einv.p, wbuf, dp, out);
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

}  // namespace bo
