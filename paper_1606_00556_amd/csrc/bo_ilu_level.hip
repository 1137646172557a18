// F stage of CPR (Section 3.2) with block ILU(0) in natural order over the
// whole system, applied by level scheduling: the comparison point of the
// tiled form (which drops the couplings between tiles to run one wavefront
// per tile without grid-wide waits).
//
// Block ILU(0) by its IKJ definition, rows in index order: for each lower
// entry k of row i in ascending column order, L_ik = A_ik E_k^{-1} (with A_ik
// as updated so far), then A_ij -= L_ik A_kj for every later entry j of row i
// that row k also holds; E_i is the updated diagonal block.  Solve: y_i = r_i
// - sum_{k<i} L_ik y_k, then x_i = E_i^{-1} (y_i - sum_{j>i} A_ij x_j) with
// the updated upper blocks.
//
// Schedule: in natural order (x fastest, then y, then z) a grid cell's lower
// entries are its -x, -y and -z neighbours, all on the hyperplane i+j+k-1, so
// the cells of one hyperplane depend only on earlier hyperplanes.  The
// factorisation and each sweep take the nx+ny+nz-2 hyperplanes one launch at
// a time, one thread per cell.  Rows after the grid's cells (fixed-rate
// wells) come after every cell in natural order and may couple to each
// other: one thread takes them in order after the last hyperplane (before
// the first one in the backward sweep).  Each thread reads its own row's
// blocks (72 contiguous bytes each) and writes its own row only.
#include "bo_cpr.hpp"

namespace bo {
namespace {

// cells (i, j, k) of the grid with i + j + k = l in layer k
__host__ __device__ inline int nat_layer_count(int l, int k, int nx, int ny) {
    const int t = l - k;  // i + j
    if (t < 0) return 0;
    const int jlo = t - (nx - 1) > 0 ? t - (nx - 1) : 0;
    const int jhi = t < ny - 1 ? t : ny - 1;
    return jhi >= jlo ? jhi - jlo + 1 : 0;
}

// the pattern: bit 2 for a cell row whose lower entries are not among its
// -x, -y, -z neighbours, bit 1 for a row without its diagonal block
__global__ void k_nat_check(int n, int N, int nx, int ny, const int32_t *__restrict__ rp,
                            const int32_t *__restrict__ ci, int32_t *bad) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int i = r % nx, j = (r / nx) % ny, k = r / (nx * ny);
    bool diag = false, ok = true;
    for (int e = rp[r]; e < rp[r + 1]; e++) {
        const int c = ci[e];
        if (c == r) diag = true;
        else if (c < r && r < N)
            ok = ok && ((i > 0 && c == r - 1) || (j > 0 && c == r - nx) || (k > 0 && c == r - nx * ny));
    }
    if (!ok) atomicOr(bad, 2);
    if (!diag) atomicOr(bad, 1);
}

// perm[lptr[l] + q] = the q-th cell of hyperplane l, by layer and then by j
__global__ void k_nat_perm(int nx, int ny, int nz, const int32_t *__restrict__ lptr, int32_t *__restrict__ perm) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nx * ny * nz) return;
    const int i = c % nx, j = (c / nx) % ny, k = c / (nx * ny);
    const int l = i + j + k;
    int pos = lptr[l];
    for (int q = 0; q < k; q++) pos += nat_layer_count(l, q, nx, ny);
    const int t = l - k;
    pos += j - (t - (nx - 1) > 0 ? t - (nx - 1) : 0);
    perm[pos] = c;
}

__device__ __forceinline__ void ld9(const double *p, double *a) {
#pragma unroll
    for (int z = 0; z < 9; z++) a[z] = p[z];
}

__device__ __forceinline__ void mv3d(const double *A, const double *x, double *y) {
    y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    y[1] = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    y[2] = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
}

// IKJ elimination of row r over finished rows; false for a missing or
// singular pivot
__device__ bool nat_factor_row(int r, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, double *lu,
                               double *inv) {
    const int e0 = rp[r], e1 = rp[r + 1];
    int ed = -1;
    for (int e = e0; e < e1; e++) {
        const int k = ci[e];
        if (k == r) ed = e;
        if (k >= r) continue;
        double A[9], Ek[9], L[9];
        ld9(lu + 9 * (size_t)e, A);
        ld9(inv + 9 * (size_t)k, Ek);
        mul3(A, Ek, L);
#pragma unroll
        for (int z = 0; z < 9; z++) lu[9 * (size_t)e + z] = L[z];
        const int f0 = rp[k], f1 = rp[k + 1];
        for (int ej = e + 1; ej < e1; ej++) {
            const int j = ci[ej];
            for (int f = f0; f < f1; f++) {
                const int cf = ci[f];
                if (cf > j) break;
                if (cf != j) continue;
                double U[9], t[9];
                ld9(lu + 9 * (size_t)f, U);
                mul3(L, U, t);
#pragma unroll
                for (int z = 0; z < 9; z++) lu[9 * (size_t)ej + z] = lu[9 * (size_t)ej + z] - t[z];
                break;
            }
        }
    }
    double E[9], Ei[9];
    bool ok = ed >= 0;
    if (ok) {
        ld9(lu + 9 * (size_t)ed, E);
        ok = inv3_gj(E, Ei);
    }
    if (!ok)
        for (int z = 0; z < 9; z++) Ei[z] = 0.0;
#pragma unroll
    for (int z = 0; z < 9; z++) inv[9 * (size_t)r + z] = Ei[z];
    return ok;
}

// one hyperplane of the factorisation (rows perm[0..cnt))
__global__ void k_nat_factor(int cnt, const int32_t *__restrict__ perm, const int32_t *__restrict__ rp,
                             const int32_t *__restrict__ ci, double *lu, double *inv, int32_t *bad) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    if (!nat_factor_row(perm[t], rp, ci, lu, inv)) atomicOr(bad, 1);
}

// rows [r0, r1) one after the other (one thread)
__global__ void k_nat_factor_seq(int r0, int r1, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 double *lu, double *inv, int32_t *bad) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int r = r0; r < r1; r++)
        if (!nat_factor_row(r, rp, ci, lu, inv)) atomicOr(bad, 1);
}

// y_r = r_r - sum_{k<r} L_rk y_k (entries in ascending column order)
__device__ __forceinline__ void nat_forward_row(int r, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                                const double *__restrict__ lu, const double *__restrict__ rhs,
                                                double *y) {
    double s[3] = {rhs[3 * (size_t)r], rhs[3 * (size_t)r + 1], rhs[3 * (size_t)r + 2]};
    for (int e = rp[r]; e < rp[r + 1]; e++) {
        const int k = ci[e];
        if (k >= r) break;
        double L[9], yk[3] = {y[3 * (size_t)k], y[3 * (size_t)k + 1], y[3 * (size_t)k + 2]}, t[3];
        ld9(lu + 9 * (size_t)e, L);
        mv3d(L, yk, t);
        for (int q = 0; q < 3; q++) s[q] = s[q] - t[q];
    }
    for (int q = 0; q < 3; q++) y[3 * (size_t)r + q] = s[q];
}

// x_r = E_r^{-1} (y_r - sum_{j>r} U_rj x_j)
__device__ __forceinline__ void nat_backward_row(int r, const int32_t *__restrict__ rp,
                                                 const int32_t *__restrict__ ci, const double *__restrict__ lu,
                                                 const double *__restrict__ inv, const double *__restrict__ y,
                                                 double *x) {
    double s[3] = {y[3 * (size_t)r], y[3 * (size_t)r + 1], y[3 * (size_t)r + 2]};
    for (int e = rp[r]; e < rp[r + 1]; e++) {
        const int j = ci[e];
        if (j <= r) continue;
        double U[9], xj[3] = {x[3 * (size_t)j], x[3 * (size_t)j + 1], x[3 * (size_t)j + 2]}, t[3];
        ld9(lu + 9 * (size_t)e, U);
        mv3d(U, xj, t);
        for (int q = 0; q < 3; q++) s[q] = s[q] - t[q];
    }
    double Ei[9], o[3];
    ld9(inv + 9 * (size_t)r, Ei);
    mv3d(Ei, s, o);
    for (int q = 0; q < 3; q++) x[3 * (size_t)r + q] = o[q];
}

__global__ void k_nat_forward(int cnt, const int32_t *__restrict__ perm, const int32_t *__restrict__ rp,
                              const int32_t *__restrict__ ci, const double *__restrict__ lu,
                              const double *__restrict__ rhs, double *y) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) nat_forward_row(perm[t], rp, ci, lu, rhs, y);
}

__global__ void k_nat_forward_seq(int r0, int r1, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                  const double *__restrict__ lu, const double *__restrict__ rhs, double *y) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int r = r0; r < r1; r++) nat_forward_row(r, rp, ci, lu, rhs, y);
}

__global__ void k_nat_backward(int cnt, const int32_t *__restrict__ perm, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ ci, const double *__restrict__ lu,
                               const double *__restrict__ inv, const double *__restrict__ y, double *x) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < cnt) nat_backward_row(perm[t], rp, ci, lu, inv, y, x);
}

// rows r1-1 down to r0 (one thread)
__global__ void k_nat_backward_seq(int r0, int r1, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                   const double *__restrict__ lu, const double *__restrict__ inv,
                                   const double *__restrict__ y, double *x) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    for (int r = r1 - 1; r >= r0; r--) nat_backward_row(r, rp, ci, lu, inv, y, x);
}

// out_r += (dp_r, 0, 0) for the pressure rows
__global__ void k_nat_add_p(int npr, const double *__restrict__ dp, double *out) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r < npr) out[3 * (size_t)r] = dp[r] + out[3 * (size_t)r];
}

}  // namespace

// Factorisation on stream s over the handle's BSR copy (Arp, Aci, Aval); it
// reads nothing back: the flag pc->fflag (bit 1: a missing or singular
// pivot, bit 2: a cell row with lower entries off its grid neighbours) is
// read by fstage_check.
bo_status nat_launch(bo_cpr *pc, hipStream_t s) {
    const Grid &g = pc->g;
    const int n = pc->n, N = (int)g.n();
    if (!pc->has_grid || pc->ncell != N || n < N)
        return fail(BO_ERR_UNSUPPORTED, "F stage: the natural-order ILU needs a grid without matrix cells");
    const int nl = g.nx + g.ny + g.nz - 2;
    pc->nat_lptr.assign(nl + 1, 0);
    for (int l = 0; l < nl; l++) {
        int c = 0;
        for (int k = 0; k < g.nz; k++) c += nat_layer_count(l, k, g.nx, g.ny);
        pc->nat_lptr[l + 1] = pc->nat_lptr[l] + c;
    }
    if (pc->nat_lptr[nl] != N) return fail(BO_ERR_INVALID_ARG, "F stage: hyperplane count mismatch");
    const size_t nnzb = (size_t)pc->nnzb;
    BO_TRY(pc->nat_lu.alloc(9 * nnzb));
    BO_TRY(pc->nat_inv.alloc(9 * (size_t)n));
    BO_TRY(pc->nat_y.alloc(3 * (size_t)n));
    BO_TRY(pc->nat_perm.alloc(N));
    BO_TRY(pc->nat_lptr_d.alloc(nl + 1));
    int32_t *ff = pc->fflag.p;
    const int32_t *rp = pc->Arp.p, *ci = pc->Aci.p;
    BO_HIP(hipMemcpyAsync(pc->nat_lptr_d.p, pc->nat_lptr.data(), sizeof(int32_t) * (nl + 1),
                          hipMemcpyHostToDevice, s));
    BO_HIP(hipMemcpyAsync(pc->nat_lu.p, pc->Aval.p, sizeof(double) * 9 * nnzb, hipMemcpyDeviceToDevice, s));
    k_nat_check<<<grid_for(n), kBlock, 0, s>>>(n, N, g.nx, g.ny, rp, ci, ff);
    k_nat_perm<<<grid_for(N), kBlock, 0, s>>>(g.nx, g.ny, g.nz, pc->nat_lptr_d.p, pc->nat_perm.p);
    BO_HIP(hipGetLastError());
    for (int l = 0; l < nl; l++) {
        const int a = pc->nat_lptr[l], cnt = pc->nat_lptr[l + 1] - a;
        k_nat_factor<<<grid_for(cnt), kBlock, 0, s>>>(cnt, pc->nat_perm.p + a, rp, ci, pc->nat_lu.p, pc->nat_inv.p,
                                                      ff);
    }
    if (n > N) k_nat_factor_seq<<<1, 64, 0, s>>>(N, n, rp, ci, pc->nat_lu.p, pc->nat_inv.p, ff);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// out = F(r) (+ (dp, 0, 0) on the pressure rows when dp != NULL); out may be r
bo_status nat_apply(bo_cpr *pc, const double *r, const double *dp, double *out, hipStream_t s) {
    const int n = pc->n, N = (int)pc->g.n();
    const int nl = (int)pc->nat_lptr.size() - 1;
    const int32_t *rp = pc->Arp.p, *ci = pc->Aci.p, *perm = pc->nat_perm.p;
    const double *lu = pc->nat_lu.p, *inv = pc->nat_inv.p;
    double *y = pc->nat_y.p;
    for (int l = 0; l < nl; l++) {
        const int a = pc->nat_lptr[l], cnt = pc->nat_lptr[l + 1] - a;
        k_nat_forward<<<grid_for(cnt), kBlock, 0, s>>>(cnt, perm + a, rp, ci, lu, r, y);
    }
    if (n > N) {
        k_nat_forward_seq<<<1, 64, 0, s>>>(N, n, rp, ci, lu, r, y);
        k_nat_backward_seq<<<1, 64, 0, s>>>(N, n, rp, ci, lu, inv, y, out);
    }
    for (int l = nl - 1; l >= 0; l--) {
        const int a = pc->nat_lptr[l], cnt = pc->nat_lptr[l + 1] - a;
        k_nat_backward<<<grid_for(cnt), kBlock, 0, s>>>(cnt, perm + a, rp, ci, lu, inv, y, out);
    }
    if (dp) k_nat_add_p<<<grid_for(pc->npr), kBlock, 0, s>>>(pc->npr, dp, out);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

}  // namespace bo
