// The learned correction inside CPR's pressure stage, and the collection of
// its training pairs.
//
// Pressure stage with a network attached: dp = V(r_p) (one AMG V-cycle), then
// c = s N([r_p / s, z]) with s = RMS(r_p) and z the standardised
// log-permeability, and the judge uses dp + alpha c with alpha = <u, A_pp c>
// / ||A_pp c||^2, u = r_p - A_pp dp (the multiple of c that minimises
// ||r_p - A_pp x||) when alpha > 0; otherwise dp is used as it is.
// Everything, the decision included, stays on the device: no host round trip
// per application.
//
// Training pairs: the first pressure-stage inputs r_p of a CPR-FGMRES solve
// are recorded; for each, e = A_pp^{-1} r_p - V(r_p), with A_pp^{-1} r_p from
// restarted GMRES on A_pp preconditioned by the V-cycle.
#include <cmath>
#include "bo_cpr.hpp"
#include "bo_nn.hpp"

namespace bo {
bo_status nn_input_cpr(bo_nn *nn, const Grid &g, const void *rp, bool fp32, const double *s2, const float *z,
                       hipStream_t s);
bo_status amg_vcycle(bo_cpr *pc, const double *b, double *x, hipStream_t s);

namespace {

constexpr int kRB = 1024;  // fixed reduction grid

__device__ __forceinline__ double block_sum256(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    double r = red[0];
    __syncthreads();
    return r;
}

// partial sums of x and x^2 (q = 2 outputs per block)
template <typename T>
__global__ void __launch_bounds__(256) k_sums(long long n, const T *__restrict__ x, double *__restrict__ part) {
    __shared__ double red[256];
    double s1 = 0.0, s2 = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long long)gridDim.x * 256) {
        double v = (double)x[i];
        s1 += v;
        s2 += v * v;
    }
    s1 = block_sum256(s1, red);
    s2 = block_sum256(s2, red);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = s1; part[2 * blockIdx.x + 1] = s2; }
}

// out[0] = sum of part[2p] / n, out[1] = sum of part[2p+1] / n
__global__ void k_sums_final(int np, const double *__restrict__ part, double inv_n, double *__restrict__ out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int p = 0; p < np; p++) { a += part[2 * p]; b += part[2 * p + 1]; }
    out[0] = a * inv_n;
    out[1] = b * inv_n;
}

// z = (x - mean) / std, FP32 (std of zero: 1)
__global__ void k_standardise(long long n, const double *__restrict__ x, const double *__restrict__ mom,
                              float *__restrict__ z) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double mean = mom[0], var = mom[1] - mom[0] * mom[0];
    double sd = var > 0.0 ? sqrt(var) : 1.0;
    z[i] = (float)((x[i] - mean) / sd);
}

// judge partials: r0 = r_p - A dp, r1 = r0 - s A y per row (slot form A)
template <typename T>
__global__ void __launch_bounds__(256) k_judge(int nx, int ny, int nz, const T *__restrict__ A,
                                               const T *__restrict__ rp, const T *__restrict__ dp,
                                               const float *__restrict__ y, const double *__restrict__ mom,
                                               double *__restrict__ part) {
    __shared__ double red[256];
    long long n = (long long)nx * ny * nz;
    double s = sqrt(mom[1]);
    double q0 = 0.0, q1 = 0.0;
    int nxy = nx * ny;
    for (long long ii = (long long)blockIdx.x * 256 + threadIdx.x; ii < n; ii += (long long)gridDim.x * 256) {
        int i = (int)ii;
        int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
        const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                           ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
        double ad = 0.0, ay = 0.0;
        for (int q = 0; q < NSLOT; q++) {
            int j = nb[q];
            if (j < 0) continue;
            double a = (double)A[(size_t)q * n + i];
            ad += a * (double)dp[j];
            ay += a * (double)y[j];
        }
        double u = (double)rp[i] - ad;  // residual of the V-cycle result
        double w = s * ay;              // A_pp c
        q0 += u * w;
        q1 += w * w;
    }
    q0 = block_sum256(q0, red);
    q1 = block_sum256(q1, red);
    if (threadIdx.x == 0) { part[2 * blockIdx.x] = q0; part[2 * blockIdx.x + 1] = q1; }
}

// alpha = <u, A c> / ||A c||^2 (the multiple of c that minimises the
// pressure residual), kept when positive
__global__ void k_judge_final(int np, const double *__restrict__ part, double *__restrict__ alpha,
                              int32_t *__restrict__ used) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double p = 0.0, q = 0.0;
    for (int k = 0; k < np; k++) { p += part[2 * k]; q += part[2 * k + 1]; }
    const double a = (q > 0.0 && p > 0.0) ? p / q : 0.0;
    *alpha = a;
    if (a > 0.0) *used += 1;
}

// out = dp + alpha s y where the judge kept the correction, else dp
template <typename T>
__global__ void k_nn_apply(long long n, const T *__restrict__ dp, const float *__restrict__ y,
                           const double *__restrict__ mom, const double *__restrict__ alpha, T *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double a = *alpha;
    if (a > 0.0) out[i] = dp[i] + (T)(a * sqrt(mom[1]) * (double)y[i]);
    else out[i] = dp[i];
}

template <typename T>
__global__ void k_to_float(long long n, const T *__restrict__ a, float *__restrict__ b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

__global__ void k_float_to_double(long long n, const float *__restrict__ a, double *__restrict__ b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

__global__ void k_sub_to_float(long long n, const double *__restrict__ a, const double *__restrict__ b,
                               float *__restrict__ out) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = (float)(a[i] - b[i]);
}

// y = A x on the level-0 pressure matrix (slot form, FP64)
__global__ void __launch_bounds__(256) k_app_mv(int nx, int ny, int nz, const double *__restrict__ A,
                                                const double *__restrict__ x, double *__restrict__ y) {
    long long n = (long long)nx * ny * nz;
    long long ii = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (ii >= n) return;
    int i = (int)ii, nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s = 0.0;
    for (int q = 0; q < NSLOT; q++) {
        int j = nb[q];
        if (j < 0) continue;
        s = s + A[(size_t)q * n + i] * x[j];
    }
    y[i] = s;
}

// r = b - A x on the level-0 pressure matrix (slot form, FP64)
__global__ void __launch_bounds__(256) k_app_resid(int nx, int ny, int nz, const double *__restrict__ A,
                                                   const double *__restrict__ b, const double *__restrict__ x,
                                                   double *__restrict__ r) {
    long long n = (long long)nx * ny * nz;
    long long ii = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (ii >= n) return;
    int i = (int)ii, nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s = 0.0;
    for (int q = 0; q < NSLOT; q++) {
        int j = nb[q];
        if (j < 0) continue;
        s = s + A[(size_t)q * n + i] * x[j];
    }
    r[i] = b[i] - s;
}

}  // namespace

// dp <- judged V-cycle result with the network's correction (see the header)
template <typename T>
bo_status nn_correct(bo_cpr *pc, const T *rp, const T *dp, const T **out, hipStream_t s) {
    long long n = pc->n;
    const bool fp32 = sizeof(T) == 4;
    BO_TRY(pc->nn_part.alloc(2 * kRB));
    BO_TRY(pc->nn_mom.alloc(2));
    BO_TRY(pc->nn_alpha.alloc(1));
    k_sums<T><<<kRB, 256, 0, s>>>(n, rp, pc->nn_part.p);
    k_sums_final<<<1, 64, 0, s>>>(kRB, pc->nn_part.p, 1.0 / (double)n, pc->nn_mom.p);
    BO_HIP(hipGetLastError());
    // mom[1] = mean of r_p^2 = s^2
    BO_TRY(nn_input_cpr(pc->nn, pc->g, rp, fp32, pc->nn_mom.p + 1, pc->nn_z.p, s));
    const T *A = fp32 ? (const T *)pc->app32.p : (const T *)pc->app.p;
    k_judge<T><<<kRB, 256, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, A, rp, dp, pc->nn->y.p, pc->nn_mom.p,
                                   pc->nn_part.p);
    k_judge_final<<<1, 64, 0, s>>>(kRB, pc->nn_part.p, pc->nn_alpha.p, pc->nn_used.p);
    T *o;
    if (fp32) {
        BO_TRY(pc->nn_dp32.alloc(n));
        o = (T *)pc->nn_dp32.p;
    } else {
        BO_TRY(pc->nn_dp.alloc(n));
        o = (T *)pc->nn_dp.p;
    }
    k_nn_apply<T><<<grid_for(n), kBlock, 0, s>>>(n, dp, pc->nn->y.p, pc->nn_mom.p, pc->nn_alpha.p, o);
    BO_HIP(hipGetLastError());
    *out = o;
    return BO_OK;
}
template bo_status nn_correct<double>(bo_cpr *, const double *, const double *, const double **, hipStream_t);
template bo_status nn_correct<float>(bo_cpr *, const float *, const float *, const float **, hipStream_t);

// record the pressure-stage input for the pairs being collected
template <typename T>
bo_status nn_record(bo_cpr *pc, const T *rp, hipStream_t s) {
    if (!pc->rec_out || pc->rec_n >= pc->rec_max) return BO_OK;
    long long n = pc->n;
    k_to_float<T><<<grid_for(n), kBlock, 0, s>>>(n, rp, pc->rec_out + (size_t)pc->rec_n * n);
    BO_HIP(hipGetLastError());
    pc->rec_n++;
    return BO_OK;
}
template bo_status nn_record<double>(bo_cpr *, const double *, hipStream_t);
template bo_status nn_record<float>(bo_cpr *, const float *, hipStream_t);

// x = A_pp^{-1} r by right-preconditioned GMRES(m) with the V-cycle, from x = 0
static bo_status pressure_gmres(bo_cpr *pc, const double *r, double *x, double rtol, int maxit, int *its,
                                hipStream_t s) {
    const int m = 30;
    long long n = pc->n;
    const Grid &g = pc->g;
    BO_TRY(pc->pg_V.alloc((size_t)(m + 1) * n));
    BO_TRY(pc->pg_Z.alloc((size_t)m * n));
    BO_TRY(pc->pg_h.alloc(2 * (m + 1) + 1 + m));  // Arnoldi scalars, then the update coefficients
    std::vector<const double *> vp(m + 1), zp(m);
    for (int i = 0; i <= m; i++) vp[i] = pc->pg_V.p + (size_t)i * n;
    for (int i = 0; i < m; i++) zp[i] = pc->pg_Z.p + (size_t)i * n;
    double *hd = pc->pg_h.p;
    std::vector<double> hh(2 * (m + 1) + 1), H((size_t)(m + 1) * m), cs(m), sn(m), gv(m + 1), y(m);
    auto fetch = [&](int cnt) -> bo_status {
        BO_HIP(hipMemcpyAsync(hh.data(), hd, sizeof(double) * cnt, hipMemcpyDeviceToHost, s));
        BO_HIP(hipStreamSynchronize(s));
        return BO_OK;
    };
    BO_TRY(fill(n, 0.0, x, s));
    BO_TRY(pc->red.dot(n, r, r, hd, s));
    BO_TRY(fetch(1));
    double bnorm = std::sqrt(hh[0]);
    *its = 0;
    if (!(bnorm > 0.0)) return BO_OK;
    double* V = pc->pg_V.p;
    for (;;) {
        k_app_resid<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, pc->app.p, r, x, V);
        BO_HIP(hipGetLastError());
        BO_TRY(pc->red.dot(n, V, V, hd, s));
        BO_TRY(fetch(1));
        double beta = std::sqrt(hh[0]);
        if (beta <= rtol * bnorm || *its >= maxit) break;
        BO_TRY(axpby(n, 1.0 / beta, V, 0.0, V, s));
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int k = 0;
        for (int j = 0; j < m; j++) {
            double *vj = V + (size_t)j * n, *zj = pc->pg_Z.p + (size_t)j * n, *w = V + (size_t)(j + 1) * n;
            BO_TRY(amg_vcycle(pc, vj, zj, s));
            (*its)++;
            k_app_mv<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, pc->app.p, zj, w);
            BO_HIP(hipGetLastError());
            int nv = j + 1;
            BO_TRY(pc->red.cgs_pass(n, w, vp.data(), nv, nullptr, true, hd, s));
            BO_TRY(pc->red.cgs_pass(n, w, vp.data(), nv, hd, true, hd + (m + 1), s));
            BO_TRY(pc->red.cgs_pass(n, w, vp.data(), nv, hd + (m + 1), false, hd + 2 * (m + 1), s));
            BO_TRY(fetch(2 * (m + 1) + 1));
            double hn = std::sqrt(hh[2 * (m + 1)]);
            for (int i = 0; i <= j; i++) H[(size_t)i * m + j] = hh[i] + hh[m + 1 + i];
            H[(size_t)(j + 1) * m + j] = hn;
            bool breakdown = !(hn > 1e-300);
            if (!breakdown) BO_TRY(axpby(n, 1.0 / hn, w, 0.0, w, s));
            for (int i = 0; i < j; i++) {
                double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            double den = std::hypot(a, bb);
            cs[j] = a / den;
            sn[j] = bb / den;
            H[(size_t)j * m + j] = den;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            k = j + 1;
            if (std::fabs(gv[j + 1]) <= rtol * bnorm || *its >= maxit || breakdown) break;
        }
        for (int i = k - 1; i >= 0; i--) {
            double sum = gv[i];
            for (int q = i + 1; q < k; q++) sum -= H[(size_t)i * m + q] * y[q];
            y[i] = sum / H[(size_t)i * m + i];
        }
        BO_HIP(hipMemcpyAsync(hd + 2 * (m + 1) + 1, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        BO_TRY(multiaxpy(n, zp.data(), k, hd + 2 * (m + 1) + 1, 1.0, x, s));
        BO_HIP(hipStreamSynchronize(s));
    }
    return BO_OK;
}

}  // namespace bo

using namespace bo;

extern "C" bo_status bo_cpr_attach_nn(bo_cpr *pc, bo_nn *nn, const double *logk, void *stream) {
    if (!pc) return fail(BO_ERR_INVALID_ARG, "bo_cpr_attach_nn: NULL handle");
    if (!nn) {
        pc->nn = nullptr;
        return BO_OK;
    }
    if (!logk) return fail(BO_ERR_INVALID_ARG, "bo_cpr_attach_nn: logk is NULL");
    AllocScope scope(pc->allocator(), stream);
    if (!pc->o.use_amg) return fail(BO_ERR_INVALID_ARG, "bo_cpr_attach_nn: the handle has no pressure stage");
    if (pc->general || pc->cond || pc->bs != 3)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr_attach_nn: the network needs the black-oil grid form");
    hipStream_t s = (hipStream_t)stream;
    long long n = pc->n;
    BO_TRY(pc->nn_z.alloc(n));
    BO_TRY(pc->nn_part.alloc(2 * kRB));
    BO_TRY(pc->nn_mom.alloc(2));
    BO_TRY(pc->nn_used.alloc(1));
    k_sums<double><<<kRB, 256, 0, s>>>(n, logk, pc->nn_part.p);
    k_sums_final<<<1, 64, 0, s>>>(kRB, pc->nn_part.p, 1.0 / (double)n, pc->nn_mom.p);
    k_standardise<<<grid_for(n), kBlock, 0, s>>>(n, logk, pc->nn_mom.p, pc->nn_z.p);
    BO_HIP(hipGetLastError());
    BO_HIP(hipMemsetAsync(pc->nn_used.p, 0, sizeof(int32_t), s));
    BO_HIP(hipStreamSynchronize(s));
    pc->nn = nn;
    return BO_OK;
}

// level-0 pressure matrix in slot order as FP32 [7][N]
__global__ void k_app_to_f32(long long n, const double *__restrict__ app, float *__restrict__ out) {
    long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < 7 * n) out[e] = (float)app[e];
}

extern "C" bo_status bo_cpr_pressure_stencil(bo_cpr *pc, float *coef, void *stream) {
    if (!pc || !coef) return fail(BO_ERR_INVALID_ARG, "bo_cpr_pressure_stencil: NULL argument");
    if (pc->general || pc->cond || !pc->o.use_amg)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr_pressure_stencil: needs the plain grid form with a pressure stage");
    if (pc->broken) return fail(BO_ERR_INVALID_ARG, "bo_cpr_pressure_stencil: the last bo_cpr_update failed");
    long long n = pc->n;
    k_app_to_f32<<<grid_for(7 * n), kBlock, 0, (hipStream_t)stream>>>(n, pc->app.p, coef);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

extern "C" bo_status bo_cpr_collect_pairs(bo_cpr *pc, const double *b, int32_t ncalls, double rtol_inner,
                                          float *rp_out, float *e_out, int32_t *got, void *stream) {
    if (!pc || !b || !rp_out || !e_out || !got) return fail(BO_ERR_INVALID_ARG, "bo_cpr_collect_pairs: NULL argument");
    if (ncalls < 1 || !(rtol_inner > 0.0)) return fail(BO_ERR_INVALID_ARG, "bo_cpr_collect_pairs: bad arguments");
    if (!pc->o.use_amg) return fail(BO_ERR_INVALID_ARG, "bo_cpr_collect_pairs: the handle has no pressure stage");
    if (pc->general || pc->cond || pc->bs != 3)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr_collect_pairs: pairs need the black-oil grid form");
    AllocScope scope(pc->allocator(), stream);
    hipStream_t s = (hipStream_t)stream;
    long long n = pc->n;
    *got = 0;
    bo_nn *keep_nn = pc->nn;
    pc->nn = nullptr;  // pairs describe the plain V-cycle
    BO_TRY(pc->pg_x.alloc(3 * n));
    BO_TRY(fill(3 * n, 0.0, pc->pg_x.p, s));
    pc->rec_out = rp_out;
    pc->rec_max = ncalls;
    pc->rec_n = 0;
    bo_fgmres_opts o;
    bo_fgmres_default_opts(&o);
    o.maxit = ncalls;  // only the first ncalls applications are needed
    bo_solve_stats st;
    bo_status rc = fgmres_core(pc, UserA{nullptr, nullptr, nullptr}, b, pc->pg_x.p, &o, &st, s);
    int rec = pc->rec_n;
    pc->rec_out = nullptr;
    pc->rec_max = pc->rec_n = 0;
    pc->nn = keep_nn;
    if (rc != BO_OK && rc != BO_NOT_CONVERGED) return rc;
    BO_TRY(pc->pg_r.alloc(n));
    BO_TRY(pc->pg_v.alloc(n));
    BO_TRY(pc->pg_xs.alloc(n));
    for (int q = 0; q < rec; q++) {
        k_float_to_double<<<grid_for(n), kBlock, 0, s>>>(n, rp_out + (size_t)q * n, pc->pg_r.p);
        BO_HIP(hipGetLastError());
        BO_TRY(amg_vcycle(pc, pc->pg_r.p, pc->pg_v.p, s));
        int its = 0;
        BO_TRY(pressure_gmres(pc, pc->pg_r.p, pc->pg_xs.p, rtol_inner, 3000, &its, s));
        k_sub_to_float<<<grid_for(n), kBlock, 0, s>>>(n, pc->pg_xs.p, pc->pg_v.p, e_out + (size_t)q * n);
        BO_HIP(hipGetLastError());
    }
    BO_HIP(hipStreamSynchronize(s));
    *got = rec;
    return BO_OK;
}
