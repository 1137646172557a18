// Exact elimination of the matrix cells of a dual-porosity system.
//
// In the fractured-reservoir model (Section 2.1) every grid location holds a
// fracture cell and a matrix cell, and the matrix cell exchanges fluid with
// its own fracture cell only.  Block row N+g (matrix cell of location g)
// therefore holds exactly two blocks, A_mf at column g and A_mm at column
// N+g, and fracture row g holds one block A_fm at column N+g.  Block Gaussian
// elimination of every matrix unknown is exact and local:
//     S_gg = A_ff,gg - A_fm A_mm^{-1} A_mf       (only the diagonal changes)
//     b'_g = b_g - A_fm A_mm^{-1} b_m
//     x_m  = A_mm^{-1} (b_m - A_mf x_g)          (back-substitution)
// The reduced system (N fracture rows, then the fixed-rate well rows, whose
// row and column 2N+w become N+w) has the single-porosity pattern, and its
// CPR preconditioner is the ordinary one of a grid with wells (the extended
// grid form without matrix cells, or the plain grid form when there are no
// fixed-rate wells).  The Krylov solver runs on the reduced system, half the
// length of the full one, and the true residual is taken on the full system.
//
// Layout: W = A_fm A_mm^{-1}, A_mm^{-1} and A_mf per location as 9 arrays of
// N doubles (entry-major), so the per-location kernels read them coalesced.
// Every 3x3 product sums in ascending inner index, as the oracle's does.
#include <cmath>
#include "bo_cpr.hpp"

namespace bo {

struct Condensed {
    int N = 0, nw = 0, nr = 0;       // locations, fixed-rate wells, reduced rows (N + nw)
    long long nfull = 0;             // block rows of the full system (2N + nw)
    int nnz = 0;                     // blocks of the reduced system
    DBuf<int32_t> src;               // the full block each reduced block copies
    DBuf<double> W, minv, amf;       // 9 x N each
    DBuf<double> rb, rx, rfull;      // reduced right-hand side and solution, full residual
    DBuf<int32_t> flag;
    DBuf<double> nrm;                // a squared norm on its way to the host
    bo_cpr *inner = nullptr;
    ~Condensed() {
        if (inner) bo_cpr_destroy(inner);
    }
};

namespace {

__device__ __forceinline__ int full_row(int N, int r) { return r < N ? r : N + r; }

// reduced row counts: a fracture row loses its matrix block, a well row keeps all
__global__ void k_cond_counts(int N, int nr, const int32_t *__restrict__ rp, int32_t *__restrict__ cnt) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    int i = full_row(N, r);
    cnt[r] = rp[i + 1] - rp[i] - (r < N ? 1 : 0);
}

// reduced column indices and the source block of each reduced block; a
// pattern that is not a dual-porosity one raises the flag
__global__ void k_cond_pattern(int N, int nr, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const int32_t *__restrict__ srp, int32_t *__restrict__ sci,
                               int32_t *__restrict__ src, int32_t *__restrict__ bad) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    int i = full_row(N, r);
    int q = srp[r];
    int skipped = 0;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
        int c = ci[e];
        if (c >= N && c < 2 * N) {
            if (r >= N || c != N + r) *bad = 1;
            skipped++;
            continue;
        }
        sci[q] = c < N ? c : c - N;
        src[q] = e;
        q++;
    }
    if (q != srp[r + 1] || (r < N && skipped != 1)) *bad = 1;
    if (r < N) {
        int m = N + r;
        if (rp[m + 1] - rp[m] != 2 || ci[rp[m]] != r || ci[rp[m] + 1] != m) *bad = 1;
    }
}

// copies every block (one thread per double: coalesced reads and writes)
__global__ void k_cond_copy(long long nvals, const int32_t *__restrict__ src, const double *__restrict__ val,
                            double *__restrict__ sval) {
    long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nvals) return;
    long long e = t / 9;
    int z = (int)(t - 9 * e);
    sval[t] = val[9 * (size_t)src[e] + z];
}

// per location: A_mm^{-1}, W = A_fm A_mm^{-1}, the diagonal of the reduced
// fracture row S = A_ff - W A_mf (overwriting the copied A_ff)
__global__ void k_cond_pivots(int N, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              const double *__restrict__ val, const int32_t *__restrict__ srp,
                              const int32_t *__restrict__ sci, double *__restrict__ sval, double *__restrict__ W,
                              double *__restrict__ minv, double *__restrict__ amf, int32_t *__restrict__ bad) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= N) return;
    int em = -1;  // the fracture row's matrix block
    for (int e = rp[g]; e < rp[g + 1]; e++)
        if (ci[e] == N + g) em = e;
    int ed = -1;  // the reduced row's diagonal
    for (int e = srp[g]; e < srp[g + 1]; e++)
        if (sci[e] == g) ed = e;
    if (em < 0 || ed < 0) {
        *bad = 1;
        return;
    }
    const int m = N + g;
    double Afm[9], Amf[9], Amm[9], Mi[9], Wg[9], T[9];
    bool fin = true;
    for (int z = 0; z < 9; z++) {
        Afm[z] = val[9 * (size_t)em + z];
        Amf[z] = val[9 * (size_t)rp[m] + z];
        Amm[z] = val[9 * (size_t)(rp[m] + 1) + z];
        fin = fin && isfinite(Afm[z]) && isfinite(Amf[z]) && isfinite(Amm[z]);
    }
    // (the blocks the reduced system copies are checked by its own setup)
    if (!fin) {
        *bad = 3;
        return;
    }
    if (!inv3_gj(Amm, Mi)) {
        *bad = 2;
        return;
    }
    mul3(Afm, Mi, Wg);
    mul3(Wg, Amf, T);
    double *S = sval + 9 * (size_t)ed;
    for (int z = 0; z < 9; z++) {
        S[z] = S[z] - T[z];
        W[(size_t)z * N + g] = Wg[z];
        minv[(size_t)z * N + g] = Mi[z];
        amf[(size_t)z * N + g] = Amf[z];
    }
}

// b' = (b_f - W b_m, b_w)
__global__ void k_cond_reduce(int N, int nr, const double *__restrict__ b, const double *__restrict__ W,
                              double *__restrict__ br) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    if (r >= N) {
        for (int q = 0; q < 3; q++) br[3 * (size_t)r + q] = b[3 * (size_t)(N + r) + q];
        return;
    }
    const double *bm = b + 3 * (size_t)(N + r);
    double m0 = bm[0], m1 = bm[1], m2 = bm[2];
    for (int q = 0; q < 3; q++) {
        double t = W[(size_t)(3 * q) * N + r] * m0 + W[(size_t)(3 * q + 1) * N + r] * m1 +
                   W[(size_t)(3 * q + 2) * N + r] * m2;
        br[3 * (size_t)r + q] = b[3 * (size_t)r + q] - t;
    }
}

// x = (x'_f, A_mm^{-1} (b_m - A_mf x'_f), x'_w), or x += that vector (add)
__global__ void k_cond_back(int N, int nr, const double *__restrict__ b, const double *__restrict__ xr,
                            const double *__restrict__ minv, const double *__restrict__ amf, int add,
                            double *__restrict__ x) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= nr) return;
    double d[3];
    const double *xf = xr + 3 * (size_t)r;
    d[0] = xf[0];
    d[1] = xf[1];
    d[2] = xf[2];
    double *xo = x + 3 * (size_t)full_row(N, r);
    for (int q = 0; q < 3; q++) xo[q] = add ? xo[q] + d[q] : d[q];
    if (r >= N) return;
    const double *bm = b + 3 * (size_t)(N + r);
    double u[3];
    for (int q = 0; q < 3; q++) {
        double t = amf[(size_t)(3 * q) * N + r] * d[0] + amf[(size_t)(3 * q + 1) * N + r] * d[1] +
                   amf[(size_t)(3 * q + 2) * N + r] * d[2];
        u[q] = bm[q] - t;
    }
    double *xm = x + 3 * (size_t)(N + r);
    for (int q = 0; q < 3; q++) {
        double v = minv[(size_t)(3 * q) * N + r] * u[0] + minv[(size_t)(3 * q + 1) * N + r] * u[1] +
                   minv[(size_t)(3 * q + 2) * N + r] * u[2];
        xm[q] = add ? xm[q] + v : v;
    }
}

}  // namespace

bo_cpr *cond_inner(bo_cpr *pc) { return pc && pc->cond ? pc->cond->inner : pc; }

void cond_destroy(bo_cpr *pc) {
    if (pc && pc->cond) {
        delete pc->cond;
        pc->cond = nullptr;
    }
}

// Builds (or, for an existing handle, rebuilds in its memory) the reduced
// system of A and the CPR of the reduced system with the caller's options.
bo_status cond_setup(bo_cpr *pc, const bo_bsr *A, const bo_grid *grid, const bo_cpr_opts *opts, hipStream_t s) {
    const long long N = (long long)grid->nx * grid->ny * grid->nz;
    if (A->nbrows < 2 * N || A->nnzb < 2 * A->nbrows - N)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: condense needs a dual-porosity matrix of the grid");
    // the reduced system: a grid with wells (the extended grid form without
    // matrix cells), or the plain grid form without fixed-rate wells; the
    // level-0 smoother follows the form (red-black Gauss-Seidel needs the
    // plain grid, l1-Jacobi the extended one)
    const int nw = (int)(A->nbrows - 2 * N);
    const int nr = (int)N + nw;
    bo_grid g0{grid->nx, grid->ny, grid->nz, 0};
    bo_cpr_opts io = *opts;
    io.condense = 0;
    if (io.npr >= nr) io.npr = 0;
    if (nw > 0 && io.smoother == BO_SMOOTH_GS) io.smoother = BO_SMOOTH_L1;
    if (nw == 0 && io.smoother == BO_SMOOTH_L1) io.smoother = BO_SMOOTH_GS;
    BO_TRY(cpr_check(nr, &g0, &io));
    if (!pc->cond) {
        pc->cond = new (std::nothrow) Condensed();
        if (!pc->cond) return fail(BO_ERR_ALLOC, "bo_cpr_setup: out of host memory");
    }
    Condensed &C = *pc->cond;
    pc->o = *opts;
    pc->n = A->nbrows;
    pc->nnzb = A->nnzb;
    pc->g = Grid{grid->nx, grid->ny, grid->nz};
    pc->has_grid = true;
    pc->general = true;
    pc->ncell = (int)(2 * N);
    pc->npr = 0;
    C.N = (int)N;
    C.nw = nw;
    C.nr = nr;
    C.nfull = A->nbrows;
    C.nnz = A->nnzb - (int)(3 * N);
    if (!C.inner) {
        C.inner = new (std::nothrow) bo_cpr();
        if (!C.inner) return fail(BO_ERR_ALLOC, "bo_cpr_setup: out of host memory");
    }
    // the reduced BSR matrix is built in the inner handle's own operator
    // buffers (its setup then takes it without a copy)
    bo_cpr *in = C.inner;
    BO_TRY(in->Arp.alloc((size_t)nr + 1));
    BO_TRY(in->Aci.alloc(C.nnz));
    BO_TRY(in->Aval.alloc(9 * (size_t)C.nnz));
    int32_t *const srp = in->Arp.p, *const sci = in->Aci.p;
    double *const sval = in->Aval.p;
    BO_TRY(C.src.alloc(C.nnz));
    BO_TRY(C.W.alloc(9 * (size_t)N));
    BO_TRY(C.minv.alloc(9 * (size_t)N));
    BO_TRY(C.amf.alloc(9 * (size_t)N));
    BO_TRY(C.rb.alloc(3 * (size_t)nr));
    BO_TRY(C.rx.alloc(3 * (size_t)nr));
    BO_TRY(C.rfull.alloc(3 * (size_t)C.nfull));
    BO_TRY(C.flag.alloc(1));
    BO_TRY(C.nrm.alloc(1));
    // pattern (its counts staged in sci before the column indices overwrite them)
    k_cond_counts<<<grid_for(nr), kBlock, 0, s>>>(C.N, nr, A->rowptr, sci);
    BO_HIP(hipGetLastError());
    int32_t total = 0;
    BO_TRY(scan_counts(sci, srp, nr, &total, s));
    if (total != C.nnz) return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: not a dual-porosity pattern (block count)");
    BO_HIP(hipMemsetAsync(C.flag.p, 0, sizeof(int32_t), s));
    k_cond_pattern<<<grid_for(nr), kBlock, 0, s>>>(C.N, nr, A->rowptr, A->colind, srp, sci, C.src.p, C.flag.p);
    k_cond_copy<<<grid_for(9LL * C.nnz), kBlock, 0, s>>>(9LL * C.nnz, C.src.p, A->val, sval);
    k_cond_pivots<<<grid_for(N), kBlock, 0, s>>>(C.N, A->rowptr, A->colind, A->val, srp, sci, sval, C.W.p,
                                                 C.minv.p, C.amf.p, C.flag.p);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    HostRead rd{C.flag.p, sizeof bad, &bad};
    BO_TRY(host_reads(&rd, 1, s));
    if (bad == 1) return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: not a dual-porosity pattern");
    if (bad == 2) return fail(BO_ERR_SINGULAR_BLOCK, "bo_cpr_setup: a matrix cell's diagonal block is singular");
    if (bad == 3) return fail(BO_ERR_NONFINITE, "bo_cpr_setup: the matrix holds NaN or Inf");
    bo_bsr S{nr, C.nnz, srp, sci, sval};
    bo_status st = cpr_setup_impl(&S, &g0, &io, C.inner, s);
    C.inner->broken = st != BO_OK;
    return st;
}

bo_status cond_apply(bo_cpr *pc, const double *v, double *z, hipStream_t s) {
    Condensed &C = *pc->cond;
    k_cond_reduce<<<grid_for(C.nr), kBlock, 0, s>>>(C.N, C.nr, v, C.W.p, C.rb.p);
    BO_HIP(hipGetLastError());
    BO_TRY(cpr_apply(C.inner, C.rb.p, C.rx.p, s));
    k_cond_back<<<grid_for(C.nr), kBlock, 0, s>>>(C.N, C.nr, v, C.rx.p, C.minv.p, C.amf.p, 0, z);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// The full system through the reduced one: r = b - A x (caller's A); the
// Krylov solver (FGMRES or BiCGSTAB) on S d' = reduce(r) to ||reduce(r) -
// S d'|| <= rtol ||b||; x += back(r, d').
// After the back-substitution the matrix rows hold exactly (up to rounding),
// so the full residual is the reduced one; a further pass runs only if the
// full residual still exceeds the tolerance.
bo_status cond_solve(bo_cpr *pc, const bo_bsr *A, const double *b, double *x, const bo_fgmres_opts *opts,
                     bo_solve_stats *stats, hipStream_t s, KrylovCore core) {
    Condensed &C = *pc->cond;
    const long long len = 3 * C.nfull;
    bo_cpr *in = C.inner;
    bo_solve_stats st{};
    // norms through the inner handle's deterministic reducer, read back
    auto norm = [&](long long n, const double *v, double *out) -> bo_status {
        BO_TRY(in->red.dot(n, v, v, C.nrm.p, s));
        HostRead rd{C.nrm.p, sizeof(double), out};
        BO_TRY(host_reads(&rd, 1, s));
        *out = std::sqrt(*out);
        return BO_OK;
    };
    double bnorm = 0.0;
    BO_TRY(norm(len, b, &bnorm));
    if (!std::isfinite(bnorm)) {
        if (stats) *stats = st;
        return fail(BO_ERR_NONFINITE, "bo_fgmres_solve: right-hand side holds NaN or Inf");
    }
    if (bnorm == 0.0) {
        BO_TRY(fill(len, 0.0, x, s));
        BO_HIP(hipStreamSynchronize(s));
        st.converged = 1;
        if (stats) *stats = st;
        return BO_OK;
    }
    const double tol = opts->rtol * bnorm;
    // a zero initial guess leaves r = b: the first pass then takes b itself
    // (no product with the full matrix, no copy, its norm known)
    double xn = 0.0;
    BO_TRY(norm(len, x, &xn));
    bo_status status = BO_NOT_CONVERGED;
    for (int pass = 0; pass < 4; pass++) {
        const double *rf = C.rfull.p;
        double rn = 0.0;
        if (pass == 0 && xn == 0.0) {
            rf = b;
            rn = bnorm;
        } else {
            BO_HIP(hipMemcpyAsync(C.rfull.p, b, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
            BO_TRY(bo_bsr_spmv(A, -1.0, x, 1.0, C.rfull.p, s));
            BO_TRY(norm(len, C.rfull.p, &rn));
        }
        st.rel_residual = rn / bnorm;
        if (!std::isfinite(rn)) {
            status = fail(BO_ERR_NONFINITE, "bo_fgmres_solve: residual is not finite");
            break;
        }
        if (rn <= tol) {
            st.converged = 1;
            status = BO_OK;
            break;
        }
        if (st.iterations >= opts->maxit) break;
        k_cond_reduce<<<grid_for(C.nr), kBlock, 0, s>>>(C.N, C.nr, rf, C.W.p, C.rb.p);
        BO_HIP(hipGetLastError());
        double rbn = 0.0;
        BO_TRY(norm(3LL * C.nr, C.rb.p, &rbn));
        if (!(rbn > 0.0)) break;
        BO_TRY(fill(3LL * C.nr, 0.0, C.rx.p, s));
        bo_fgmres_opts io = *opts;
        io.rtol = tol / rbn;
        io.maxit = opts->maxit - st.iterations;
        bo_solve_stats ist{};
        bo_status rc = core(in, UserA{nullptr, nullptr, nullptr}, C.rb.p, C.rx.p, &io, &ist, s);
        st.iterations += ist.iterations;
        st.restarts += ist.restarts;
        st.spmv_ms += ist.spmv_ms;
        st.spmv_calls += ist.spmv_calls;
        st.est_residual = ist.est_residual * rbn / bnorm;
        if (rc != BO_OK && rc != BO_NOT_CONVERGED) {
            status = rc;
            break;
        }
        k_cond_back<<<grid_for(C.nr), kBlock, 0, s>>>(C.N, C.nr, rf, C.rx.p, C.minv.p, C.amf.p, 1, x);
        BO_HIP(hipGetLastError());
    }
    BO_HIP(hipStreamSynchronize(s));
    if (stats) *stats = st;
    return status;
}

}  // namespace bo
