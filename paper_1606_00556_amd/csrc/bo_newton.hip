// Inexact Newton (Section 3.1, Algorithm "inexact Newton") and a time-step
// loop on top of the Jacobian assembly and CPR-FGMRES.
//
// Iteration l: b(x^l) = -R(x^l) and J(x^l) from one assembly; the Newton
// system J dx = b is solved by FGMRES with CPR to ||b - J dx|| <= theta_l ||b||;
// the step is x^{l+1} = x^l + omega dx with omega = min(1, ds_max / max |dS|)
// (saturation chopping).  Forcing terms, with r^{l-1} = b(x^{l-1}) -
// J_{l-1} omega dx the linear model's residual of the step taken:
//   choice 1: ||b(x^l) - r^{l-1}|| / ||b(x^{l-1})||
//   choice 2: | ||b(x^l)|| - ||r^{l-1}|| | / ||b(x^{l-1})||
//   choice 3: gamma (||b(x^l)|| / ||b(x^{l-1})||)^beta
// or a fixed theta; theta_0 = theta0 and every theta clipped to [theta_min,
// theta_max].  Stop when ||b(x^l)|| <= max(atol, rtol ||b(x^0)||).
//
// The time-step loop repeats a step whose Newton loop fails with half the
// step, and grows the next step by `growth` after a step that needed at most
// `easy` Newton iterations.
#include <cmath>
#include <cstring>
#include "bo_cpr.hpp"

namespace bo {
namespace {

// largest |dS| over the saturation unknowns of the cell rows: the bits of a
// non-negative double order like the value, so an integer atomic max works
__global__ void k_max_dsat(long long ncell, const double *__restrict__ dx, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long red[256];
    unsigned long long m = 0;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < ncell;
         i += (long long)gridDim.x * blockDim.x) {
        double a = fmax(fabs(dx[3 * i + 1]), fabs(dx[3 * i + 2]));
        unsigned long long u = (unsigned long long)__double_as_longlong(a);
        m = u > m ? u : m;
    }
    red[threadIdx.x] = m;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] = red[threadIdx.x] > red[threadIdx.x + o] ? red[threadIdx.x]
                                                                                          : red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, red[0]);
}

}  // namespace
}  // namespace bo

using namespace bo;

struct bo_newton {
    bo_problem p{};
    std::vector<bo_well> wells;     // the problem's wells (copied: the struct points here)
    bo_grid grid{};
    bo_cpr_opts copts{};
    int32_t n = 0, nnzb = 0, ncell = 0;
    DBuf<int32_t> rp, ci;
    DBuf<double> val, b, dx, rprev, tmp, xold;
    DBuf<unsigned long long> dsmax;
    DBuf<double> nrm;
    Reducer red;
    bo_cpr *pc = nullptr;
    ~bo_newton() {
        if (pc) bo_cpr_destroy(pc);
    }
    bo_bsr J() { return bo_bsr{n, nnzb, rp.p, ci.p, val.p}; }
};

extern "C" void bo_newton_default_opts(bo_newton_opts *o) {
    if (!o) return;
    o->forcing = BO_FORCING_EW1;
    o->theta0 = 1e-2;
    o->theta_fixed = 1e-7;
    o->gamma = 0.9;
    o->beta = 2.0;
    o->theta_min = 1e-8;
    o->theta_max = 0.1;
    o->rtol = 1e-6;
    o->atol = 0.0;
    o->max_newton = 20;
    o->ds_max = 0.2;
}

extern "C" bo_status bo_newton_create(const bo_problem *p, const bo_grid *grid, const bo_cpr_opts *copts,
                                      bo_newton **out, void *stream) {
    if (!out) return fail(BO_ERR_INVALID_ARG, "bo_newton_create: out is NULL");
    *out = nullptr;
    if (!p || !grid || !copts) return fail(BO_ERR_INVALID_ARG, "bo_newton_create: NULL argument");
    int32_t n = 0, nnzb = 0;
    BO_TRY(bo_jacobian_bsr_size(p, &n, &nnzb));
    bo_newton *h = new (std::nothrow) bo_newton();
    if (!h) return fail(BO_ERR_ALLOC, "bo_newton_create: out of host memory");
    h->p = *p;
    h->wells.assign(p->wells, p->wells + p->nwells);
    h->p.wells = h->wells.empty() ? nullptr : h->wells.data();
    h->grid = *grid;
    h->copts = *copts;
    h->n = n;
    h->nnzb = nnzb;
    h->ncell = (int32_t)((long long)p->nx * p->ny * p->nz * (p->dual ? 2 : 1));
    bo_status st = BO_OK;
    if ((st = h->rp.alloc((size_t)n + 1)) || (st = h->ci.alloc(nnzb)) || (st = h->val.alloc(9 * (size_t)nnzb)) ||
        (st = h->b.alloc(3 * (size_t)n)) || (st = h->dx.alloc(3 * (size_t)n)) ||
        (st = h->rprev.alloc(3 * (size_t)n)) || (st = h->tmp.alloc(3 * (size_t)n)) ||
        (st = h->xold.alloc(3 * (size_t)n)) || (st = h->dsmax.alloc(1)) || (st = h->nrm.alloc(1)) ||
        (st = h->red.init())) {
        delete h;
        return st;
    }
    (void)stream;
    *out = h;
    return BO_OK;
}

extern "C" void bo_newton_destroy(bo_newton *h) {
    if (!h) return;
    (void)hipDeviceSynchronize();
    delete h;
}

namespace {

bo_status norm2(bo_newton *h, long long len, const double *v, double *out, hipStream_t s) {
    BO_TRY(h->red.dot(len, v, v, h->nrm.p, s));
    HostRead rd{h->nrm.p, sizeof(double), out};
    BO_TRY(host_reads(&rd, 1, s));
    *out = std::sqrt(*out);
    return BO_OK;
}

double forcing(const bo_newton_opts &o, int l, double bn, double bn_prev, double diff, double rn) {
    double t;
    if (o.forcing == BO_FORCING_FIXED) t = o.theta_fixed;
    else if (l == 0) t = o.theta0;
    else if (o.forcing == BO_FORCING_EW1) t = diff / bn_prev;
    else if (o.forcing == BO_FORCING_EW2) t = std::fabs(bn - rn) / bn_prev;
    else t = o.gamma * std::pow(bn / bn_prev, o.beta);
    return std::min(std::max(t, o.theta_min), o.theta_max);
}

}  // namespace

extern "C" bo_status bo_newton_solve(bo_newton *h, const double *x_old, double *x, double dt,
                                     const bo_newton_opts *o, const bo_fgmres_opts *fo, bo_newton_stats *st,
                                     void *stream) {
    if (!h || !x_old || !x || !o || !fo || !st) return fail(BO_ERR_INVALID_ARG, "bo_newton_solve: NULL argument");
    if (!(dt > 0.0)) return fail(BO_ERR_INVALID_ARG, "bo_newton_solve: dt must be > 0");
    if (o->forcing < BO_FORCING_FIXED || o->forcing > BO_FORCING_EW3 || o->max_newton < 0 ||
        o->max_newton > BO_NEWTON_HIST || !(o->theta_min > 0.0) || !(o->theta_max >= o->theta_min) ||
        !(o->ds_max > 0.0) || !(o->rtol >= 0.0) || !(o->atol >= 0.0))
        return fail(BO_ERR_INVALID_ARG, "bo_newton_solve: options out of range");
    hipStream_t s = (hipStream_t)stream;
    *st = bo_newton_stats{};
    const long long len = 3LL * h->n;
    bo_bsr J = h->J();
    BO_TRY(bo_jacobian_bsr(&h->p, x_old, x, dt, &J, h->b.p, stream));
    double bn = 0.0;
    BO_TRY(norm2(h, len, h->b.p, &bn, s));
    if (!std::isfinite(bn)) return fail(BO_ERR_NONFINITE, "bo_newton_solve: the residual is not finite");
    st->res0 = bn;
    st->res_hist[0] = bn;
    const double stop = std::max(o->atol, o->rtol * bn);
    double bn_prev = bn, diff = 0.0, rn = 0.0;
    bool have_prev = false;
    for (int l = 0;; l++) {
        st->res = bn;
        if (bn <= stop) {
            st->converged = 1;
            break;
        }
        if (l >= o->max_newton) break;
        if (have_prev) {
            // ||b(x^l) - r^{l-1}|| and ||r^{l-1}||
            BO_TRY(axpby(len, 1.0, h->b.p, 0.0, h->tmp.p, s));
            BO_TRY(axpby(len, -1.0, h->rprev.p, 1.0, h->tmp.p, s));
            BO_TRY(norm2(h, len, h->tmp.p, &diff, s));
            BO_TRY(norm2(h, len, h->rprev.p, &rn, s));
        }
        const double theta = forcing(*o, l, bn, bn_prev, diff, rn);
        if (!h->pc) BO_TRY(bo_cpr_setup(&J, &h->grid, &h->copts, nullptr, &h->pc, stream));
        else BO_TRY(bo_cpr_update(h->pc, &J, stream));
        BO_TRY(fill(len, 0.0, h->dx.p, s));
        bo_fgmres_opts lo = *fo;
        lo.rtol = theta;
        bo_solve_stats ls{};
        bo_status rc = bo_fgmres_solve(h->pc, &J, h->b.p, h->dx.p, &lo, &ls, stream);
        if (rc != BO_OK && rc != BO_NOT_CONVERGED) return rc;
        // omega from the largest saturation change
        BO_HIP(hipMemsetAsync(h->dsmax.p, 0, sizeof(unsigned long long), s));
        k_max_dsat<<<256, 256, 0, s>>>(h->ncell, h->dx.p, h->dsmax.p);
        BO_HIP(hipGetLastError());
        unsigned long long bits = 0;
        HostRead rd{h->dsmax.p, sizeof bits, &bits};
        BO_TRY(host_reads(&rd, 1, s));
        double dsm;
        std::memcpy(&dsm, &bits, sizeof dsm);
        const double omega = dsm <= o->ds_max ? 1.0 : o->ds_max / dsm;
        // r^l = b - J (omega dx) with this iterate's J; then x += omega dx
        BO_TRY(axpby(len, 1.0, h->b.p, 0.0, h->rprev.p, s));
        BO_TRY(bo_bsr_spmv(&J, -omega, h->dx.p, 1.0, h->rprev.p, stream));
        BO_TRY(axpby(len, omega, h->dx.p, 1.0, x, s));
        have_prev = true;
        st->theta_hist[l] = theta;
        st->omega_hist[l] = omega;
        st->lin_hist[l] = ls.iterations;
        st->linear_iterations += ls.iterations;
        st->iterations = l + 1;
        bn_prev = bn;
        BO_TRY(bo_jacobian_bsr(&h->p, x_old, x, dt, &J, h->b.p, stream));
        BO_TRY(norm2(h, len, h->b.p, &bn, s));
        st->res_hist[l + 1] = bn;
        if (!std::isfinite(bn)) return fail(BO_ERR_NONFINITE, "bo_newton_solve: the residual is not finite");
    }
    BO_HIP(hipStreamSynchronize(s));
    return st->converged ? BO_OK : BO_NOT_CONVERGED;
}

extern "C" bo_status bo_newton_run(bo_newton *h, double *x, double t_end, double dt0, double dt_max, double dt_min,
                                   double growth, int32_t easy, const bo_newton_opts *o, const bo_fgmres_opts *fo,
                                   bo_run_stats *rs, void *stream) {
    if (!h || !x || !o || !fo || !rs) return fail(BO_ERR_INVALID_ARG, "bo_newton_run: NULL argument");
    if (!(t_end > 0.0) || !(dt0 > 0.0) || !(dt_max >= dt0) || !(dt_min > 0.0) || !(growth >= 1.0) || easy < 0)
        return fail(BO_ERR_INVALID_ARG, "bo_newton_run: time-step options out of range");
    hipStream_t s = (hipStream_t)stream;
    *rs = bo_run_stats{};
    const long long len = 3LL * h->n;
    double t = 0.0, dt = dt0;
    while (t < t_end * (1.0 - 1e-12)) {
        dt = std::min(dt, t_end - t);
        // x_old = x; the Newton loop starts from the previous state
        BO_TRY(axpby(len, 1.0, x, 0.0, h->xold.p, s));
        bo_newton_stats ns{};
        bo_status rc = bo_newton_solve(h, h->xold.p, x, dt, o, fo, &ns, stream);
        if (rc != BO_OK && rc != BO_NOT_CONVERGED) return rc;
        rs->linear_iterations += ns.linear_iterations;
        rs->newton_iterations += ns.iterations;
        if (rc == BO_NOT_CONVERGED) {
            rs->cuts++;
            BO_TRY(axpby(len, 1.0, h->xold.p, 0.0, x, s));
            dt *= 0.5;
            if (dt < dt_min) {
                BO_HIP(hipStreamSynchronize(s));
                return fail(BO_NOT_CONVERGED, "bo_newton_run: the time step fell below dt_min");
            }
            continue;
        }
        if (rs->steps < BO_RUN_HIST) {
            rs->dt_hist[rs->steps] = dt;
            rs->newton_hist[rs->steps] = ns.iterations;
        }
        rs->steps++;
        t += dt;
        if (ns.iterations <= easy) dt = std::min(dt * growth, dt_max);
    }
    rs->t = t;
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}
