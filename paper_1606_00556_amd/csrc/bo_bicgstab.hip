// BiCGSTAB, the Krylov solver of the paper's scaling runs (Section 3.3 lists
// it beside GMRES and Orthomin; Section 4.2's black-oil and oil-water runs use
// it), right-preconditioned by CPR (a fixed linear operator between
// iterations):
//   r = b - A x, rhat = r, rho = alpha = omega = 1, p = v = 0
//   repeat: rho' = <rhat, r>; beta = (rho' / rho)(alpha / omega)
//           p = r + beta (p - omega v); phat = M^{-1} p; v = A phat
//           alpha = rho' / <rhat, v>; s = r - alpha v
//           shat = M^{-1} s; t = A shat; omega = <t, s> / <t, t>
//           x += alpha phat + omega shat; r = s - omega t
// until ||r|| <= rtol ||b||; then the true residual b - A x is checked with
// the caller's A and the iteration restarts from it if needed.  Iterations
// count preconditioner applications (two per step), as for FGMRES; an odd
// cap ends on the half step's iterate x + alpha phat.  A zero
// <rhat, r>, <rhat, v> or <t, t> (breakdown of the recurrences) restarts
// from the current true residual once, then ends the solve with
// BO_ERR_BREAKDOWN.  Scalars are reduced on the device (fixed order) and read
// back each half step; every vector update is one kernel.
#include <cmath>
#include "bo_cpr.hpp"

namespace bo {
bo_status cpr_apply(bo_cpr *pc, const double *v, double *z, hipStream_t s);

namespace {

// p = r + beta (p - omega v)
__global__ void k_bicg_p(long long n, const double *__restrict__ r, const double *__restrict__ v, double beta,
                         double omega, double *__restrict__ p) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

// x += alpha phat + omega shat; r = s - omega t (s is in r on entry)
__global__ void k_bicg_update(long long n, double alpha, const double *__restrict__ phat, double omega,
                              const double *__restrict__ shat, const double *__restrict__ t, double *__restrict__ x,
                              double *__restrict__ r) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x[i] = x[i] + alpha * phat[i] + omega * shat[i];
    r[i] = r[i] - omega * t[i];
}

}  // namespace

bo_status bicgstab_core(bo_cpr *pc, UserA A, const double *b, double *x, const bo_fgmres_opts *opts,
                        bo_solve_stats *stats, hipStream_t s) {
    const long long len = (long long)pc->bs * pc->n;
    bo_solve_stats st{};
    BO_TRY(pc->bicg.alloc(7 * (size_t)len));
    BO_TRY(pc->bicg_sc.alloc(4));
    double *r = pc->bicg.p, *rh = r + len, *p = rh + len, *v = p + len, *ph = v + len, *sh = ph + len,
           *t = sh + len;
    double *sc = pc->bicg_sc.p;
    auto dot = [&](const double *a, const double *c, double *out) -> bo_status {
        BO_TRY(pc->red.dot(len, a, c, sc, s));
        HostRead rd{sc, sizeof(double), out};
        return host_reads(&rd, 1, s);
    };
    auto true_residual = [&](double *out_norm) -> bo_status {
        BO_HIP(hipMemcpyAsync(r, b, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
        BO_TRY(user_spmv(pc, A, -1.0, x, 1.0, r, s));
        double q = 0.0;
        BO_TRY(dot(r, r, &q));
        *out_norm = std::sqrt(q);
        return BO_OK;
    };
    double bb = 0.0;
    BO_TRY(dot(b, b, &bb));
    const double bnorm = std::sqrt(bb);
    if (!std::isfinite(bnorm)) return fail(BO_ERR_NONFINITE, "bo_bicgstab_solve: right-hand side holds NaN or Inf");
    if (bnorm == 0.0) {
        BO_TRY(fill(len, 0.0, x, s));
        BO_HIP(hipStreamSynchronize(s));
        st.converged = 1;
        if (stats) *stats = st;
        return BO_OK;
    }
    const double tol = opts->rtol * bnorm;
    bo_status status = BO_NOT_CONVERGED;
    int its = 0, restarts_left = 1;
    double rn = 0.0;
    BO_TRY(true_residual(&rn));
    for (;;) {
        st.rel_residual = rn / bnorm;
        if (!std::isfinite(rn)) { status = fail(BO_ERR_NONFINITE, "bo_bicgstab_solve: residual is not finite"); break; }
        if (rn <= tol) { st.converged = 1; status = BO_OK; break; }
        if (its >= opts->maxit) break;
        // (re)start the recurrences from the current residual
        BO_HIP(hipMemcpyAsync(rh, r, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
        BO_TRY(fill(len, 0.0, p, s));
        BO_TRY(fill(len, 0.0, v, s));
        double rho = 1.0, alpha = 1.0, omega = 1.0;
        bool breakdown = false;
        while (its < opts->maxit) {
            double rho1 = 0.0;
            BO_TRY(dot(rh, r, &rho1));
            if (!(std::fabs(rho1) > 0.0) || !std::isfinite(rho1)) { breakdown = true; break; }
            const double beta = (rho1 / rho) * (alpha / omega);
            k_bicg_p<<<grid_for(len), kBlock, 0, s>>>(len, r, v, beta, omega, p);
            BO_HIP(hipGetLastError());
            BO_TRY(cpr_apply(pc, p, ph, s));
            its++;
            BO_TRY(op_spmv(pc, 1.0, ph, 0.0, v, s));
            double rv = 0.0;
            BO_TRY(dot(rh, v, &rv));
            if (!(std::fabs(rv) > 0.0) || !std::isfinite(rv)) { breakdown = true; break; }
            alpha = rho1 / rv;
            // s = r - alpha v, in r
            BO_TRY(axpby(len, -alpha, v, 1.0, r, s));
            double ss = 0.0;
            BO_TRY(dot(r, r, &ss));
            if (std::sqrt(ss) <= tol || its >= opts->maxit) {  // converged, or the cap, at the half step
                BO_TRY(axpby(len, alpha, ph, 1.0, x, s));
                st.est_residual = std::sqrt(ss) / bnorm;
                break;
            }
            BO_TRY(cpr_apply(pc, r, sh, s));
            its++;
            BO_TRY(op_spmv(pc, 1.0, sh, 0.0, t, s));
            double ts = 0.0, tt = 0.0;
            BO_TRY(dot(t, r, &ts));
            BO_TRY(dot(t, t, &tt));
            if (!(tt > 0.0) || !std::isfinite(tt)) {
                BO_TRY(axpby(len, alpha, ph, 1.0, x, s));
                breakdown = true;
                break;
            }
            omega = ts / tt;
            k_bicg_update<<<grid_for(len), kBlock, 0, s>>>(len, alpha, ph, omega, sh, t, x, r);
            BO_HIP(hipGetLastError());
            double rr = 0.0;
            BO_TRY(dot(r, r, &rr));
            st.est_residual = std::sqrt(rr) / bnorm;
            rho = rho1;
            if (std::sqrt(rr) <= tol) break;
            if (!(std::fabs(omega) > 0.0)) { breakdown = true; break; }
        }
        BO_TRY(true_residual(&rn));
        if (breakdown) {
            if (rn <= tol) continue;
            if (restarts_left-- <= 0) {
                st.rel_residual = rn / bnorm;
                status = fail(BO_ERR_BREAKDOWN, "bo_bicgstab_solve: breakdown of the BiCGSTAB recurrences");
                break;
            }
        }
        if (its < opts->maxit && rn > tol) st.restarts++;
    }
    st.iterations = its;
    BO_HIP(hipStreamSynchronize(s));
    if (stats) *stats = st;
    return status;
}

}  // namespace bo

using namespace bo;

extern "C" bo_status bo_bicgstab_solve(bo_cpr *pc, const bo_bsr *A, const double *b, double *x,
                                       const bo_fgmres_opts *opts, bo_solve_stats *stats, void *stream) {
    if (!pc || !A || !b || !x || !opts || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, "bo_bicgstab_solve: NULL argument");
    if (pc->bs != 3) return fail(BO_ERR_INVALID_ARG, "bo_bicgstab_solve: a 2x2-block handle (bo_bicgstab_solve2)");
    if (pc->broken) return fail(BO_ERR_INVALID_ARG, "bo_bicgstab_solve: the last bo_cpr_update failed");
    if (A->nbrows != pc->n || A->nnzb != pc->nnzb)
        return fail(BO_ERR_INVALID_ARG, "bo_bicgstab_solve: A is not the matrix of the last setup or update");
    if (opts->maxit < 0 || !(opts->rtol > 0.0)) return fail(BO_ERR_INVALID_ARG, "bo_bicgstab_solve: options out of range");
    if (pc->nn) return fail(BO_ERR_UNSUPPORTED, "bo_bicgstab_solve: needs a linear preconditioner (no network)");
    AllocScope scope(pc->allocator(), stream);
    if (pc->cond) return cond_solve(pc, A, b, x, opts, stats, (hipStream_t)stream, bicgstab_core);
    return bicgstab_core(pc, UserA{A, nullptr, nullptr}, b, x, opts, stats, (hipStream_t)stream);
}
