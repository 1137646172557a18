// CPR for the two-phase oil-water model's 2x2-block Jacobians (Section 3.2's
// preconditioner on the system of Section 2.2), on a grid's 7-point pattern.
//
// The operator is kept in a slot layout of 28 arrays of N doubles: entry z
// (row-major) of the block of slot s (-z, -y, -x, diag, +x, +y, +z) of cell g
// at A[(4 s + z) N + g], zero where the neighbour is outside the grid.
//
// Pressure stage: quasi-IMPES weights c_i = sign (1, -w_i) with w_i = d_01 /
// d_11 from the diagonal block D_i (so that c_i^T D_i has no saturation
// entry; the sign makes the decoupled diagonal positive), the decoupled
// pressure block A_pp (7 slot arrays) and the library's SA-AMG hierarchy on
// it, shared with the black-oil path.
//
// F stage: block Jacobi, or the tiled block ILU(0) of the black-oil path with
// 2x2 blocks: non-overlapping subdomains of tile_x x tile_y grid columns (all
// nz layers), one wavefront per tile, lane t = a + tile_x b owning column
// (i0 + a, j0 + b) and handling layer k = s - a - b at step s, so that its
// -x, -y and -z neighbours were handled one step earlier.  On the 7-point
// graph (no triangles) ILU(0) changes only the diagonal blocks:
//   E_i = A_ii - sum_{k<i} A_ik E_k^{-1} A_ki   (-z, -y, -x in that order),
//   forward  u_i = E_i^{-1} (r_i - sum_{k<i} A_ik u_k),
//   backward x_i = u_i - E_i^{-1} sum_{j>i} A_ij x_j.
// The factors are packed per slot (tile, step, lane): forward [E^{-1} | A_-z
// A_-y A_-x], backward [E^{-1} | A_+z A_+x A_+y], 16 doubles each, as 8
// double2 of which one wavefront load reads 1 KB contiguously; u is kept in
// the same order.
//
// Two-stage PF: x1 = Pi_p V(Pi_r v), x = x1 + F(v - A x1);
// CPR-FPF: x = F(v); x += Pi_p V(Pi_r (v - A x)); x += F(v - A x).
// FP64 throughout.
#include <cmath>
#include <functional>
#include "bo_cpr.hpp"

namespace bo {
bo_status amg_setup(bo_cpr *pc, hipStream_t s, const std::function<bo_status()> &after_l0);
bo_status amg_vcycle_ptr(bo_cpr *pc, const double *b, const double **res, hipStream_t s);

namespace {

struct Tile2 {
    int nx, ny, nz, tx, ty, ntx, nty, ns;
};

constexpr int kPk2 = 8;  // double2 per slot and sweep
__device__ __forceinline__ size_t pk2(const Tile2 &T, int tile, int s, int pair, int lane) {
    return (((size_t)tile * T.ns + s) * kPk2 + pair) * 64 + lane;
}
__device__ __forceinline__ size_t slot2(const Tile2 &T, int tile, int s, int lane) {
    return ((size_t)tile * T.ns + s) * 64 + lane;
}

// 2x2 helpers (row-major), sums from 0 in ascending inner index
__device__ __forceinline__ void mul2(const double *A, const double *B, double *C) {
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) {
            double s = 0.0;
            s = s + A[2 * r] * B[c];
            s = s + A[2 * r + 1] * B[2 + c];
            C[2 * r + c] = s;
        }
}
__device__ __forceinline__ void mv2(const double *A, const double *x, double *y) {
    double y0 = 0.0, y1 = 0.0;
    y0 = y0 + A[0] * x[0]; y0 = y0 + A[1] * x[1];
    y1 = y1 + A[2] * x[0]; y1 = y1 + A[3] * x[1];
    y[0] = y0;
    y[1] = y1;
}

// Inverse by Gauss-Jordan elimination with partial pivoting; false for a
// pivot that is zero relative to the block's largest entry.
__device__ __forceinline__ bool inv2_gj(const double *A, double *Ai) {
    double M[2][4] = {{A[0], A[1], 1.0, 0.0}, {A[2], A[3], 0.0, 1.0}};
    double amax = fmax(fmax(fabs(A[0]), fabs(A[1])), fmax(fabs(A[2]), fabs(A[3])));
    if (!(amax > 0.0) || !(amax < INFINITY)) return false;
#pragma unroll
    for (int k = 0; k < 2; k++) {
        if (k == 0) {
            const bool sw = fabs(M[1][0]) > fabs(M[0][0]);
#pragma unroll
            for (int c = 0; c < 4; c++) {
                double t = M[0][c];
                M[0][c] = sw ? M[1][c] : t;
                M[1][c] = sw ? t : M[1][c];
            }
        }
        if (fabs(M[k][k]) <= 1e-300 * amax) return false;
        const double d = M[k][k];
#pragma unroll
        for (int c = 0; c < 4; c++) M[k][c] = M[k][c] / d;
        const int r = 1 - k;
        const double f = M[r][k];
#pragma unroll
        for (int c = 0; c < 4; c++) M[r][c] = M[r][c] - f * M[k][c];
    }
    Ai[0] = M[0][2]; Ai[1] = M[0][3]; Ai[2] = M[1][2]; Ai[3] = M[1][3];
    return true;
}

__global__ void k_check_finite2(long long n, const double *__restrict__ v, int32_t *__restrict__ bad) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(v[i])) *bad = 1;
}

__global__ void k_bsr2_to_slots(int nx, int ny, int nz, const int32_t *__restrict__ rp,
                                const int32_t *__restrict__ ci, const double *__restrict__ v,
                                double *__restrict__ slots, int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (i >= n) return;
    size_t N = (size_t)n;
    int e = rp[i], end = rp[i + 1];
    for (int s = 0; s < NSLOT; s++) {
        int nb = nbr_of(i, s, nx, ny, nz);
        bool have = nb >= 0 && e < end && ci[e] == nb;
        for (int z = 0; z < 4; z++) slots[((size_t)s * 4 + z) * N + i] = have ? v[4 * (size_t)e + z] : 0.0;
        if (have) e++;
        else if (nb >= 0) *bad = 1;  // a stencil neighbour is missing from the pattern
    }
    if (e != end) *bad = 1;          // entries outside the 7-point stencil
}

// y = alpha A x + beta y on the slot layout; blocks in ascending column order
// (coefficients streamed past the caches, as in the black-oil SpMV)
__global__ void __launch_bounds__(kBlock) k_slot2_spmv(int nx, int ny, int nz, const double *__restrict__ A,
                                                       double alpha, const double *__restrict__ x, double beta,
                                                       double *__restrict__ y) {
    int n = nx * ny * nz;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
        int j = nb[s];
        if (j < 0) continue;
        const double *a = A + (size_t)s * 4 * N + i;
        const double x0 = x[2 * (size_t)j], x1 = x[2 * (size_t)j + 1];
        double e[4];
#pragma unroll
        for (int z = 0; z < 4; z++) e[z] = __builtin_nontemporal_load(a + z * N);
        s0 = s0 + e[0] * x0; s0 = s0 + e[1] * x1;
        s1 = s1 + e[2] * x0; s1 = s1 + e[3] * x1;
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

// r = v - A (Pi_p dp): column 0 of each block only
__global__ void __launch_bounds__(kBlock) k_slot2_col0_residual(int nx, int ny, int nz, const double *__restrict__ A,
                                                                const double *__restrict__ v,
                                                                const double *__restrict__ dp,
                                                                double *__restrict__ r) {
    int n = nx * ny * nz;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s0 = 0.0, s1 = 0.0;
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
        int j = nb[s];
        if (j < 0) continue;
        const double *a = A + (size_t)s * 4 * N + i;
        double p = dp[j];
        s0 = s0 + a[0] * p;
        s1 = s1 + a[2 * N] * p;
    }
    r[2 * (size_t)i] = v[2 * (size_t)i] - s0;
    r[2 * (size_t)i + 1] = v[2 * (size_t)i + 1] - s1;
}

// quasi-IMPES weights and the decoupled pressure block in slot form
__global__ void k_qi2_decouple(int nx, int ny, int nz, const double *__restrict__ A, double *__restrict__ cw,
                               double *__restrict__ app, int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (i >= n) return;
    size_t N = (size_t)n;
    const double *D = A + (size_t)S_D * 4 * N + i;
    double d11 = D[3 * N], d01 = D[1 * N];
    double w = 0.0;
    if (d11 == 0.0 || !isfinite(d11)) *bad = 1;
    else w = d01 / d11;
    double dpp = D[0] - w * D[2 * N];
    double sg = dpp < 0.0 ? -1.0 : 1.0;
    double c0 = sg, c1 = -sg * w;
    cw[2 * (size_t)i] = c0;
    cw[2 * (size_t)i + 1] = c1;
    for (int s = 0; s < NSLOT; s++) {
        const double *As = A + (size_t)s * 4 * N + i;
        app[(size_t)s * N + i] = c0 * As[0] + c1 * As[2 * N];
    }
}

__global__ void k_qi2_restrict(long long n, const double *__restrict__ cw, const double *__restrict__ v,
                               double *__restrict__ rp) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) rp[i] = cw[2 * i] * v[2 * i] + cw[2 * i + 1] * v[2 * i + 1];
}

__global__ void k_add_p2(long long n, const double *__restrict__ dp, double *__restrict__ z) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[2 * i] = z[2 * i] + dp[i];
}

// block Jacobi: inverses of the diagonal blocks (SoA 4 x N)
__global__ void k_bj2_setup(long long n, const double *__restrict__ A, double *__restrict__ einv,
                            int32_t *__restrict__ bad) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double *D = A + (size_t)S_D * 4 * n + i;
    double B[4] = {D[0], D[n], D[2 * n], D[3 * n]}, Bi[4];
    if (!inv2_gj(B, Bi)) {
        *bad = 1;
        Bi[0] = Bi[1] = Bi[2] = Bi[3] = 0.0;
    }
    for (int z = 0; z < 4; z++) einv[(size_t)z * n + i] = Bi[z];
}

// x = E^{-1} r (+ Pi_p dp)
__global__ void k_bj2_apply(long long n, const double *__restrict__ einv, const double *__restrict__ r,
                            const double *__restrict__ dp, double *__restrict__ x) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double E[4] = {einv[i], einv[n + i], einv[2 * n + i], einv[3 * n + i]};
    double ri[2] = {r[2 * i], r[2 * i + 1]}, xi[2];
    mv2(E, ri, xi);
    if (dp) xi[0] = xi[0] + dp[i];
    x[2 * i] = xi[0];
    x[2 * i + 1] = xi[1];
}

__device__ __forceinline__ void load_slot_blk(const double *__restrict__ A, int slot, size_t N, int g, double *o) {
    const double *p = A + (size_t)slot * 4 * N + g;
#pragma unroll
    for (int z = 0; z < 4; z++) o[z] = p[(size_t)z * N];
}

template <int K>
__device__ __forceinline__ void shfl_k(const double *src, double *dst, int lane) {
#pragma unroll
    for (int z = 0; z < K; z++) dst[z] = __shfl(src[z], lane, 64);
}

// Factorisation, one wavefront per tile: E_i and the packed slot data.
__global__ void __launch_bounds__(64) k_ilu2_factor(Tile2 T, const double *__restrict__ A,
                                                    double2 *__restrict__ Ff, double2 *__restrict__ Fb,
                                                    int32_t *__restrict__ bad) {
    const int t = threadIdx.x;
    const int a = t % T.tx, b = t / T.tx;
    const int tile = blockIdx.x;
    const int ti = tile % T.ntx, tj = tile / T.ntx;
    const int i = ti * T.tx + a, j = tj * T.ty + b;
    const bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    const bool has_mx = a > 0, has_my = b > 0;
    const bool has_px = a + 1 < T.tx && i + 1 < T.nx, has_py = b + 1 < T.ty && j + 1 < T.ny;
    const size_t N = (size_t)T.nx * T.ny * T.nz;
    double Ep[4] = {0, 0, 0, 0}, Uxp[4] = {0, 0, 0, 0}, Uyp[4] = {0, 0, 0, 0}, Uzp[4] = {0, 0, 0, 0};
    for (int s = 0; s < T.ns; s++) {
        double Ex[4], Ey[4], Ux[4], Uy[4];
        shfl_k<4>(Ep, Ex, has_mx ? t - 1 : t);
        shfl_k<4>(Uxp, Ux, has_mx ? t - 1 : t);
        shfl_k<4>(Ep, Ey, has_my ? t - T.tx : t);
        shfl_k<4>(Uyp, Uy, has_my ? t - T.tx : t);
        const int k = s - a - b;
        if (!(active && k >= 0 && k < T.nz)) continue;
        const int g = i + T.nx * (j + T.ny * k);
        double E[4], L[4], Lk[4], tmp[4];
        double fw[16], bw[16];
#pragma unroll
        for (int z = 0; z < 16; z++) fw[z] = bw[z] = 0.0;
        load_slot_blk(A, S_D, N, g, E);
        if (k > 0) {
            load_slot_blk(A, S_MZ, N, g, L);
            mul2(L, Ep, Lk); mul2(Lk, Uzp, tmp);
            for (int z = 0; z < 4; z++) { E[z] = E[z] - tmp[z]; fw[4 + z] = L[z]; }
        }
        if (has_my) {
            load_slot_blk(A, S_MY, N, g, L);
            mul2(L, Ey, Lk); mul2(Lk, Uy, tmp);
            for (int z = 0; z < 4; z++) { E[z] = E[z] - tmp[z]; fw[8 + z] = L[z]; }
        }
        if (has_mx) {
            load_slot_blk(A, S_MX, N, g, L);
            mul2(L, Ex, Lk); mul2(Lk, Ux, tmp);
            for (int z = 0; z < 4; z++) { E[z] = E[z] - tmp[z]; fw[12 + z] = L[z]; }
        }
        double Ei[4];
        if (!inv2_gj(E, Ei)) {
            *bad = 1;
            Ei[0] = Ei[1] = Ei[2] = Ei[3] = 0.0;
        }
        for (int z = 0; z < 4; z++) { fw[z] = Ei[z]; bw[z] = Ei[z]; Ep[z] = Ei[z]; }
        // this cell's upper blocks (zero outside the tile or grid)
        if (has_px) load_slot_blk(A, S_PX, N, g, Uxp); else for (int z = 0; z < 4; z++) Uxp[z] = 0.0;
        if (has_py) load_slot_blk(A, S_PY, N, g, Uyp); else for (int z = 0; z < 4; z++) Uyp[z] = 0.0;
        if (k + 1 < T.nz) load_slot_blk(A, S_PZ, N, g, Uzp); else for (int z = 0; z < 4; z++) Uzp[z] = 0.0;
        for (int z = 0; z < 4; z++) { bw[4 + z] = Uzp[z]; bw[8 + z] = Uxp[z]; bw[12 + z] = Uyp[z]; }
#pragma unroll
        for (int p2 = 0; p2 < kPk2; p2++) {
            Ff[pk2(T, tile, s, p2, t)] = make_double2(fw[2 * p2], fw[2 * p2 + 1]);
            Fb[pk2(T, tile, s, p2, t)] = make_double2(bw[2 * p2], bw[2 * p2 + 1]);
        }
    }
}

// The sweeps walk the steps with the next step's loads in flight: its
// factors (1 KB per load instruction), and its r (forward) or u and dp
// (backward), are fetched into the second of two register buffers before the
// current step's arithmetic, which waits only for the shuffled neighbour
// values of the previous step.  Lanes idle at a step load slot 0 of the tile
// and cell 0 (all in bounds) so that no load is skipped on some paths.
struct Step2 {
    double f[16];
    double v0, v1, d;
};

// forward sweep: u (slot order) from r (cell order)
__global__ void __launch_bounds__(64) k_ilu2_forward(Tile2 T, const double2 *__restrict__ Ff,
                                                     const double *__restrict__ r, double2 *__restrict__ U) {
    const int t = threadIdx.x;
    const int a = t % T.tx, b = t / T.tx;
    const int tile = blockIdx.x;
    const int ti = tile % T.ntx, tj = tile / T.ntx;
    const int i = ti * T.tx + a, j = tj * T.ty + b;
    const bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    const bool has_mx = a > 0, has_my = b > 0;
    double up[2] = {0.0, 0.0};  // this lane's u of the previous step (the -z neighbour)
    auto fetch = [&](int s, Step2 &F) {
        const int sc = min(s, T.ns - 1);
        const int k = sc - a - b;
        const bool act = active && k >= 0 && k < T.nz;
        const int tl = act ? t : 0;
#pragma unroll
        for (int p2 = 0; p2 < kPk2; p2++) {
            const double2 d = Ff[pk2(T, tile, sc, p2, tl)];
            F.f[2 * p2] = d.x;
            F.f[2 * p2 + 1] = d.y;
        }
        const size_t g = act ? (size_t)i + (size_t)T.nx * ((size_t)j + (size_t)T.ny * k) : 0;
        F.v0 = r[2 * g];
        F.v1 = r[2 * g + 1];
    };
    auto step = [&](int s, const Step2 &F) {
        double ux[2], uy[2];
        shfl_k<2>(up, ux, has_mx ? t - 1 : t);
        shfl_k<2>(up, uy, has_my ? t - T.tx : t);
        const int k = s - a - b;
        if (!(active && k >= 0 && k < T.nz)) return;
        const double *f = F.f;
        double y0 = F.v0, y1 = F.v1, tmp[2];
        if (k > 0) { mv2(f + 4, up, tmp); y0 = y0 - tmp[0]; y1 = y1 - tmp[1]; }
        if (has_my) { mv2(f + 8, uy, tmp); y0 = y0 - tmp[0]; y1 = y1 - tmp[1]; }
        if (has_mx) { mv2(f + 12, ux, tmp); y0 = y0 - tmp[0]; y1 = y1 - tmp[1]; }
        const double yv[2] = {y0, y1};
        mv2(f, yv, up);
        U[slot2(T, tile, s, t)] = make_double2(up[0], up[1]);
    };
    Step2 R0, R1;
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

// backward sweep: x (cell order) from u (slot order), + Pi_p dp when given
__global__ void __launch_bounds__(64) k_ilu2_backward(Tile2 T, const double2 *__restrict__ Fb,
                                                      const double2 *__restrict__ U,
                                                      const double *__restrict__ dp, double *__restrict__ x) {
    const int t = threadIdx.x;
    const int a = t % T.tx, b = t / T.tx;
    const int tile = blockIdx.x;
    const int ti = tile % T.ntx, tj = tile / T.ntx;
    const int i = ti * T.tx + a, j = tj * T.ty + b;
    const bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    const bool has_px = a + 1 < T.tx && i + 1 < T.nx, has_py = b + 1 < T.ty && j + 1 < T.ny;
    double xp[2] = {0.0, 0.0};  // this lane's x of the previous (later) step: the +z neighbour
    auto fetch = [&](int s, Step2 &F) {
        const int sc = max(s, 0);
        const int k = sc - a - b;
        const bool act = active && k >= 0 && k < T.nz;
        const int tl = act ? t : 0;
#pragma unroll
        for (int p2 = 0; p2 < kPk2; p2++) {
            const double2 d = Fb[pk2(T, tile, sc, p2, tl)];
            F.f[2 * p2] = d.x;
            F.f[2 * p2 + 1] = d.y;
        }
        const double2 u = U[slot2(T, tile, sc, tl)];
        F.v0 = u.x;
        F.v1 = u.y;
        const size_t g = act ? (size_t)i + (size_t)T.nx * ((size_t)j + (size_t)T.ny * k) : 0;
        F.d = dp ? dp[g] : 0.0;
    };
    auto step = [&](int s, const Step2 &F) {
        double xx[2], xy[2];
        shfl_k<2>(xp, xx, has_px ? t + 1 : t);
        shfl_k<2>(xp, xy, has_py ? t + T.tx : t);
        const int k = s - a - b;
        if (!(active && k >= 0 && k < T.nz)) return;
        const double *f = F.f;
        // sum_{j>i} A_ij x_j in ascending column order: +x, +y, +z
        double s0 = 0.0, s1 = 0.0, tmp[2];
        if (has_px) { mv2(f + 8, xx, tmp); s0 = s0 + tmp[0]; s1 = s1 + tmp[1]; }
        if (has_py) { mv2(f + 12, xy, tmp); s0 = s0 + tmp[0]; s1 = s1 + tmp[1]; }
        if (k + 1 < T.nz) { mv2(f + 4, xp, tmp); s0 = s0 + tmp[0]; s1 = s1 + tmp[1]; }
        const double sv[2] = {s0, s1};
        double c[2];
        mv2(f, sv, c);
        xp[0] = F.v0 - c[0];
        xp[1] = F.v1 - c[1];
        const size_t g = (size_t)i + (size_t)T.nx * ((size_t)j + (size_t)T.ny * k);
        x[2 * g] = dp ? xp[0] + F.d : xp[0];
        x[2 * g + 1] = xp[1];
    };
    Step2 R0, R1;
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

Tile2 tile_geom(const bo_cpr *pc) {
    Tile2 T{};
    T.nx = pc->g.nx; T.ny = pc->g.ny; T.nz = pc->g.nz;
    T.tx = pc->o.tile_x; T.ty = pc->o.tile_y;
    T.ntx = (T.nx + T.tx - 1) / T.tx;
    T.nty = (T.ny + T.ty - 1) / T.ty;
    T.ns = T.nz + T.tx + T.ty - 2;
    return T;
}

bo_status read_flag(bo_cpr *pc, hipStream_t s, int32_t *out) {
    HostRead rd{pc->flag.p, sizeof(int32_t), out};
    return host_reads(&rd, 1, s);
}

}  // namespace

bo_status slot2_spmv(bo_cpr *pc, double alpha, const double *x, double beta, double *y, hipStream_t s) {
    k_slot2_spmv<<<grid_for(pc->n), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, pc->A.p, alpha, x, beta, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status qi2_restrict(bo_cpr *pc, const double *v, double *rp, hipStream_t s) {
    k_qi2_restrict<<<grid_for(pc->n), kBlock, 0, s>>>(pc->n, pc->cw.p, v, rp);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// out = F(r) (+ Pi_p dp when dp is given)
bo_status fstage2_apply(bo_cpr *pc, const double *r, const double *dp, double *out, hipStream_t s) {
    if (pc->o.ftype == BO_F_BJ) {
        k_bj2_apply<<<grid_for(pc->n), kBlock, 0, s>>>(pc->n, pc->einv.p, r, dp, out);
        BO_HIP(hipGetLastError());
        return BO_OK;
    }
    const Tile2 T = tile_geom(pc);
    const int tiles = T.ntx * T.nty;
    k_ilu2_forward<<<tiles, 64, 0, s>>>(T, pc->ilu_f.p, r, (double2 *)pc->ilu_w.p);
    BO_HIP(hipGetLastError());
    k_ilu2_backward<<<tiles, 64, 0, s>>>(T, pc->ilu_b.p, (const double2 *)pc->ilu_w.p, dp, out);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status cpr2_apply(bo_cpr *pc, const double *v, double *z, hipStream_t s) {
    const long long n = pc->n;
    const Grid &g = pc->g;
    if (!pc->o.fpf) {
        if (!pc->o.use_amg) return fstage2_apply(pc, v, nullptr, z, s);
        BO_TRY(qi2_restrict(pc, v, pc->rp_.p, s));
        const double *dp;
        BO_TRY(amg_vcycle_ptr(pc, pc->rp_.p, &dp, s));
        k_slot2_col0_residual<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, pc->A.p, v, dp, pc->t3a.p);
        BO_HIP(hipGetLastError());
        return fstage2_apply(pc, pc->t3a.p, dp, z, s);
    }
    BO_TRY(fstage2_apply(pc, v, nullptr, z, s));
    if (pc->o.use_amg) {
        BO_HIP(hipMemcpyAsync(pc->t3a.p, v, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, s));
        BO_TRY(slot2_spmv(pc, -1.0, z, 1.0, pc->t3a.p, s));
        BO_TRY(qi2_restrict(pc, pc->t3a.p, pc->rp_.p, s));
        const double *dp;
        BO_TRY(amg_vcycle_ptr(pc, pc->rp_.p, &dp, s));
        k_add_p2<<<grid_for(n), kBlock, 0, s>>>(n, dp, z);
        BO_HIP(hipGetLastError());
    }
    BO_HIP(hipMemcpyAsync(pc->t3a.p, v, sizeof(double) * 2 * n, hipMemcpyDeviceToDevice, s));
    BO_TRY(slot2_spmv(pc, -1.0, z, 1.0, pc->t3a.p, s));
    BO_TRY(fstage2_apply(pc, pc->t3a.p, nullptr, pc->t3b.p, s));
    return axpby(2 * n, 1.0, pc->t3b.p, 1.0, z, s);
}

// Checks and setup of a 2x2-block handle (bo_cpr2_setup, bo_cpr2_update).
static bo_status cpr2_check(const bo_bsr2 *A, const bo_grid *grid, const bo_cpr_opts *o) {
    if (!grid) return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: the two-phase path needs the grid");
    if (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || grid->dual ||
        (long long)grid->nx * grid->ny * grid->nz != A->nbrows)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: the matrix must have one block row per grid cell");
    if ((long long)A->nbrows * 7 >= (1LL << 31)) return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: matrix too large");
    if (o->condense) return fail(BO_ERR_UNSUPPORTED, "bo_cpr2_setup: no condensed form for two phases");
    if (o->precision != BO_PREC_FP64) return fail(BO_ERR_UNSUPPORTED, "bo_cpr2_setup: FP64 only");
    if (o->ftype != BO_F_BJ && o->ftype != BO_F_ILU_TILED)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr2_setup: F stage must be BO_F_BJ or BO_F_ILU_TILED");
    if (o->ftype == BO_F_ILU_TILED && (o->tile_x < 1 || o->tile_y < 1 || o->tile_x * o->tile_y > 64))
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: tiles need 1 <= tile_x*tile_y <= 64");
    if (o->smoother != BO_SMOOTH_GS && o->smoother != BO_SMOOTH_JACOBI)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr2_setup: level-0 smoother must be BO_SMOOTH_GS or BO_SMOOTH_JACOBI");
    if (o->use_amg && (o->coarse_max < 1 || o->coarse_max > kCoarseMaxLimit || !(o->theta >= 0.0) ||
                       o->sweeps < 1 || o->sweeps > 8 || o->max_levels < 1))
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: AMG options out of range");
    if (o->csmoother != BO_CSMOOTH_JACOBI && o->csmoother != BO_CSMOOTH_L1)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: unknown coarse-level smoother");
    if (o->npr != 0 && o->npr != A->nbrows)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: on a grid every row is a pressure row");
    if (o->sell_rows < 0) return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: sell_rows out of range");
    return BO_OK;
}

static bo_status cpr2_setup_impl(const bo_bsr2 *A, const bo_grid *grid, const bo_cpr_opts *opts, bo_cpr *pc,
                                 hipStream_t s) {
    if (pc->gexec) {
        (void)hipGraphExecDestroy(pc->gexec);
        pc->gexec = nullptr;
    }
    pc->bs = 2;
    pc->has_grid = true;
    pc->g = Grid{grid->nx, grid->ny, grid->nz};
    pc->general = false;
    pc->n = A->nbrows;
    pc->ncell = A->nbrows;
    pc->nnzb = A->nnzb;
    pc->o = *opts;
    pc->npr = pc->n;
    const long long n = pc->n;
    BO_TRY(pc->flag.alloc(1));
    BO_TRY(pc->A.alloc(28 * n));
    BO_HIP(hipMemsetAsync(pc->flag.p, 0, sizeof(int32_t), s));
    k_check_finite2<<<grid_for(4LL * A->nnzb), kBlock, 0, s>>>(4LL * A->nnzb, A->val, pc->flag.p);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    BO_TRY(read_flag(pc, s, &bad));
    if (bad) return fail(BO_ERR_NONFINITE, "bo_cpr2_setup: the matrix holds NaN or Inf");
    k_bsr2_to_slots<<<grid_for(n), kBlock, 0, s>>>(grid->nx, grid->ny, grid->nz, A->rowptr, A->colind, A->val,
                                                   pc->A.p, pc->flag.p);
    BO_HIP(hipGetLastError());
    BO_TRY(read_flag(pc, s, &bad));
    if (bad) return fail(BO_ERR_UNSUPPORTED, "bo_cpr2_setup: the pattern is not the grid's 7-point stencil");
    BO_TRY(pc->cw.alloc(2 * n));
    BO_TRY(pc->app.alloc(7 * n));
    k_qi2_decouple<<<grid_for(n), kBlock, 0, s>>>(grid->nx, grid->ny, grid->nz, pc->A.p, pc->cw.p, pc->app.p,
                                                  pc->flag.p);
    BO_HIP(hipGetLastError());
    BO_TRY(read_flag(pc, s, &bad));
    if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "bo_cpr2_setup: a zero saturation diagonal entry (no decoupling)");
    if (pc->o.ftype == BO_F_BJ) {
        BO_TRY(pc->einv.alloc(4 * n));
        k_bj2_setup<<<grid_for(n), kBlock, 0, s>>>(n, pc->A.p, pc->einv.p, pc->flag.p);
    } else {
        const Tile2 T = tile_geom(pc);
        const size_t slots = (size_t)T.ntx * T.nty * T.ns * 64;
        BO_TRY(pc->ilu_f.alloc(slots * kPk2));
        BO_TRY(pc->ilu_b.alloc(slots * kPk2));
        BO_TRY(pc->ilu_w.alloc(2 * slots));
        k_ilu2_factor<<<T.ntx * T.nty, 64, 0, s>>>(T, pc->A.p, pc->ilu_f.p, pc->ilu_b.p, pc->flag.p);
    }
    BO_HIP(hipGetLastError());
    BO_TRY(read_flag(pc, s, &bad));
    if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "bo_cpr2_setup: a singular 2x2 pivot block in the F stage");
    if (pc->o.use_amg) BO_TRY(amg_setup(pc, s, nullptr));
    BO_TRY(pc->rp_.alloc(n));
    BO_TRY(pc->dp_.alloc(n));
    BO_TRY(pc->t3a.alloc(2 * n));
    BO_TRY(pc->t3b.alloc(2 * n));
    BO_TRY(pc->t3c.alloc(2 * n));
    BO_TRY(pc->wf.alloc(2 * n));
    BO_TRY(pc->red.init());
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}

bo_status user_spmv(bo_cpr *pc, const UserA &A, double alpha, const double *x, double beta, double *y,
                    hipStream_t s) {
    if (A.a3) return bo_bsr_spmv(A.a3, alpha, x, beta, y, s);
    if (A.a2) return bo_bsr2_spmv(A.a2, alpha, x, beta, y, s);
    if (A.c1) return scalar_spmv(pc->g, A.c1, alpha, x, beta, y, s);
    return op_spmv(pc, alpha, x, beta, y, s);
}

}  // namespace bo

using namespace bo;

extern "C" bo_status bo_cpr2_setup(const bo_bsr2 *A, const bo_grid *grid, const bo_cpr_opts *opts,
                                   const bo_allocator *alloc, bo_cpr **out, void *stream) {
    if (!out) return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: out is NULL");
    *out = nullptr;
    if (!A || !opts || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: NULL argument");
    if (A->nbrows < 1 || A->nnzb < A->nbrows) return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: empty matrix");
    BO_TRY(cpr2_check(A, grid, opts));
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_setup: an allocator needs both alloc and free");
    bo_cpr *pc = new (std::nothrow) bo_cpr();
    if (!pc) return fail(BO_ERR_ALLOC, "bo_cpr2_setup: out of host memory");
    if (alloc) {
        pc->has_alloc = true;
        pc->alloc = *alloc;
    }
    AllocScope scope(pc->allocator(), stream);
    bo_status st = cpr2_setup_impl(A, grid, opts, pc, (hipStream_t)stream);
    if (st != BO_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        bo_cpr_destroy(pc);
        return st;
    }
    *out = pc;
    return BO_OK;
}

extern "C" bo_status bo_cpr2_update(bo_cpr *pc, const bo_bsr2 *A, void *stream) {
    if (!pc || !A || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_update: NULL argument");
    if (pc->bs != 2) return fail(BO_ERR_INVALID_ARG, "bo_cpr2_update: not a 2x2-block handle (bo_cpr_update)");
    if (A->nbrows != pc->n || A->nnzb != pc->nnzb)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr2_update: matrix size differs from the setup");
    AllocScope scope(pc->allocator(), stream);
    bo_grid g{pc->g.nx, pc->g.ny, pc->g.nz, 0};
    bo_cpr_opts o = pc->o;
    bo_status st = cpr2_setup_impl(A, &g, &o, pc, (hipStream_t)stream);
    if (st != BO_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        pc->nlev = 0;
        pc->broken = true;
    } else {
        pc->broken = false;
    }
    return st;
}

static bo_status solve2_check(const char *who, bo_cpr *pc, const bo_bsr2 *A, const double *b, double *x,
                              const bo_fgmres_opts *opts) {
    if (!pc || !A || !b || !x || !opts || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, std::string(who) + ": NULL argument");
    if (pc->bs != 2) return fail(BO_ERR_INVALID_ARG, std::string(who) + ": not a 2x2-block handle");
    if (pc->broken) return fail(BO_ERR_INVALID_ARG, std::string(who) + ": the last bo_cpr2_update failed");
    if (A->nbrows != pc->n || A->nnzb != pc->nnzb)
        return fail(BO_ERR_INVALID_ARG, std::string(who) + ": A is not the matrix of the last setup or update");
    return BO_OK;
}

extern "C" bo_status bo_fgmres_solve2(bo_cpr *pc, const bo_bsr2 *A, const double *b, double *x,
                                      const bo_fgmres_opts *opts, bo_solve_stats *stats, void *stream) {
    BO_TRY(solve2_check("bo_fgmres_solve2", pc, A, b, x, opts));
    if (opts->m < 1 || opts->m > 64 || opts->maxit < 0 || !(opts->rtol > 0.0) || opts->orth < 0 ||
        opts->orth > 2 || (opts->timing != 0 && opts->timing != 1) || (opts->graph != 0 && opts->graph != 1) ||
        (opts->flexible != 0 && opts->flexible != 1))
        return fail(BO_ERR_INVALID_ARG, "bo_fgmres_solve2: options out of range");
    AllocScope scope(pc->allocator(), stream);
    return fgmres_core(pc, UserA{nullptr, A, nullptr}, b, x, opts, stats, (hipStream_t)stream);
}

extern "C" bo_status bo_bicgstab_solve2(bo_cpr *pc, const bo_bsr2 *A, const double *b, double *x,
                                        const bo_fgmres_opts *opts, bo_solve_stats *stats, void *stream) {
    BO_TRY(solve2_check("bo_bicgstab_solve2", pc, A, b, x, opts));
    if (opts->maxit < 0 || !(opts->rtol > 0.0))
        return fail(BO_ERR_INVALID_ARG, "bo_bicgstab_solve2: options out of range");
    AllocScope scope(pc->allocator(), stream);
    return bicgstab_core(pc, UserA{nullptr, A, nullptr}, b, x, opts, stats, (hipStream_t)stream);
}
