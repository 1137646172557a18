// CPR preconditioner assembly and application, and flexible GMRES.
//
// CPR (Section 3.2): the two-stage form applies the pressure stage and then
// the F stage to the remaining residual,
//     x1 = Pi_p AMG(A_pp)^{-1} Pi_r v,   x = x1 + F(v - A x1);
// Algorithm CPR-FPF adds an F stage in front:
//     x = F(v); x += Pi_p AMG^{-1} Pi_r (v - A x); x += F(v - A x).
// Pi_r is the quasi-IMPES restriction (c_i . v_i), Pi_p puts a pressure value
// in the Po slot.  In the two-stage form v - A x1 needs only column 0 of each
// block.
//
// FGMRES(m) (Krylov solver of Section 3.3, flexible variant so that the
// preconditioner may change between iterations) runs on the original system,
// right-preconditioned, so its implicit residual is the true residual.  The
// Hessenberg column is formed on the device (deterministic reductions), read
// back once per iteration, and the Givens rotations and the small triangular
// solve run on the host.
#include <cmath>
#include <cstring>
#include <functional>
#include "bo_cpr.hpp"

namespace bo {
bo_status qi_decouple(bo_cpr *pc, hipStream_t s);
bo_status qi_restrict(bo_cpr *pc, const double *v, double *rp, hipStream_t s);
bo_status amg_setup(bo_cpr *pc, hipStream_t s, const std::function<bo_status()> &after_l0);
bo_status amg_vcycle(bo_cpr *pc, const double *b, double *x, hipStream_t s);
bo_status amg_vcycle_ptr(bo_cpr *pc, const double *b, const double **res, hipStream_t s);
bo_status amg_vcycle_ptr_f32(bo_cpr *pc, const float *b, const float **res, hipStream_t s);
bo_status amg_make_f32(bo_cpr *pc, hipStream_t s);
bo_status qi_restrict_f32(bo_cpr *pc, const double *v, float *rp, hipStream_t s);
bo_status fstage_launch(bo_cpr *pc, hipStream_t s);
bo_status fstage_check(bo_cpr *pc, hipStream_t s);
bo_status fstage_apply(bo_cpr *pc, const double *r, const double *dp, double *out, hipStream_t s);
bo_status fstage_apply_f32dp(bo_cpr *pc, const double *r, const float *dp, double *out, hipStream_t s);
bool fstage_acc_ok(const bo_cpr *pc);
template <typename TD>
bo_status fstage_apply_acc(bo_cpr *pc, const double *r, const TD *dp, double *z, hipStream_t s);
template <typename T>
bo_status nn_correct(bo_cpr *pc, const T *rp, const T *dp, const T **out, hipStream_t s);
template <typename T>
bo_status nn_record(bo_cpr *pc, const T *rp, hipStream_t s);

// y = alpha A x + beta y with the handle's copy of A (slot or BSR form)
bo_status op_spmv(bo_cpr *pc, double alpha, const double *x, double beta, double *y, hipStream_t s) {
    if (pc->bs == 2) return slot2_spmv(pc, alpha, x, beta, y, s);
    if (pc->bs == 1) return scalar_spmv(pc->g, pc->A.p, alpha, x, beta, y, s);
    if (!pc->general) return slot_spmv(pc->g, pc->A.p, alpha, x, beta, y, s);
    return sell_spmv(pc->n, pc->Asoff.p, pc->Asci.p, pc->Asv.p, pc->Asg, alpha, x, beta, y, s);
}

// y = v - A x (3x3-block handles): the sliced form reads v in place of y,
// the others copy v into y first
static bo_status op_residual(bo_cpr *pc, const double *v, const double *x, double *y, hipStream_t s) {
    if (pc->bs == 3 && pc->general)
        return sell_spmv(pc->n, pc->Asoff.p, pc->Asci.p, pc->Asv.p, pc->Asg, -1.0, x, 1.0, y, s, v);
    BO_HIP(hipMemcpyAsync(y, v, sizeof(double) * pc->bs * pc->n, hipMemcpyDeviceToDevice, s));
    return op_spmv(pc, -1.0, x, 1.0, y, s);
}

namespace {

__global__ void k_check_finite(long long n, const double *__restrict__ v, int32_t *__restrict__ bad) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && !isfinite(v[i])) *bad = 1;
}

template <typename TD>
__global__ void k_add_p(long long n, const TD *__restrict__ dp, double *__restrict__ z) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[3 * i] = z[3 * i] + (double)dp[i];
}

}  // namespace

// the pressure stage: Pi_r v -> one V-cycle; *dp points at the result in the
// hierarchy's precision (FP64, or FP32 in the mixed form)
// With a network attached the V-cycle result is replaced by the judged
// corrected one (see bo_nn_cpr.hip).
static bo_status pressure_stage(bo_cpr *pc, const double *v, const void **dp, hipStream_t s) {
    if (pc->o.precision == BO_PREC_FP64) {
        BO_TRY(qi_restrict(pc, v, pc->rp_.p, s));
        BO_TRY(nn_record<double>(pc, pc->rp_.p, s));
        const double *d;
        BO_TRY(amg_vcycle_ptr(pc, pc->rp_.p, &d, s));
        if (pc->nn) BO_TRY(nn_correct<double>(pc, pc->rp_.p, d, &d, s));
        *dp = d;
        return BO_OK;
    }
    float *b32 = pc->lv[0].b32.p;
    BO_TRY(qi_restrict_f32(pc, v, b32, s));
    BO_TRY(nn_record<float>(pc, b32, s));
    const float *d;
    BO_TRY(amg_vcycle_ptr_f32(pc, b32, &d, s));
    if (pc->nn) BO_TRY(nn_correct<float>(pc, b32, d, &d, s));
    *dp = d;
    return BO_OK;
}

bo_status cpr_apply(bo_cpr *pc, const double *v, double *z, hipStream_t s) {
    if (pc->bs == 2) return cpr2_apply(pc, v, z, s);
    if (pc->bs == 1) return ras_apply(pc, v, z, s);
    long long n = pc->n, npr = pc->npr;
    const Grid &g = pc->g;
    const bool mixed = pc->o.precision != BO_PREC_FP64;
    if (!pc->o.fpf && pc->general) {
        // x1 = Pi_p V(Pi_r v); z = x1 + F(v - A x1) with the BSR operator
        if (!pc->o.use_amg) return fstage_apply(pc, v, nullptr, z, s);
        const void *dp;
        BO_TRY(pressure_stage(pc, v, &dp, s));
        BO_TRY(fill(3 * n, 0.0, pc->t3b.p, s));
        if (mixed) k_add_p<float><<<grid_for(npr), kBlock, 0, s>>>(npr, (const float *)dp, pc->t3b.p);
        else k_add_p<double><<<grid_for(npr), kBlock, 0, s>>>(npr, (const double *)dp, pc->t3b.p);
        BO_HIP(hipGetLastError());
        BO_TRY(op_residual(pc, v, pc->t3b.p, pc->t3a.p, s));
        BO_TRY(fstage_apply(pc, pc->t3a.p, nullptr, z, s));
        if (mixed) k_add_p<float><<<grid_for(npr), kBlock, 0, s>>>(npr, (const float *)dp, z);
        else k_add_p<double><<<grid_for(npr), kBlock, 0, s>>>(npr, (const double *)dp, z);
        BO_HIP(hipGetLastError());
        return BO_OK;
    }
    if (!pc->o.fpf) {
        if (!pc->o.use_amg) return fstage_apply(pc, v, nullptr, z, s);
        const void *dp;
        BO_TRY(pressure_stage(pc, v, &dp, s));
        if (mixed) {
            BO_TRY(slot_col0_residual(g, pc->A.p, v, (const float *)dp, pc->t3a.p, s));
            return fstage_apply_f32dp(pc, pc->t3a.p, (const float *)dp, z, s);
        }
        BO_TRY(slot_col0_residual(g, pc->A.p, v, (const double *)dp, pc->t3a.p, s));
        return fstage_apply(pc, pc->t3a.p, (const double *)dp, z, s);
    }
    // FPF
    BO_TRY(fstage_apply(pc, v, nullptr, z, s));
    BO_TRY(op_residual(pc, v, z, pc->t3a.p, s));
    // where the F stage has an accumulating form, Pi_p dp and the last F
    // stage go into z in one pass at the end
    const bool acc = fstage_acc_ok(pc);
    const void *dp = nullptr;
    if (pc->o.use_amg) {
        BO_TRY(pressure_stage(pc, pc->t3a.p, &dp, s));
        if (!acc) {
            if (mixed) k_add_p<float><<<grid_for(npr), kBlock, 0, s>>>(npr, (const float *)dp, z);
            else k_add_p<double><<<grid_for(npr), kBlock, 0, s>>>(npr, (const double *)dp, z);
        }
        BO_HIP(hipGetLastError());
        // v - A z for the updated z: the residual above minus A Pi_p dp (column
        // 0 of each block only, a third of the SpMV's coefficient bytes)
        if (pc->general) {
            if (mixed) BO_TRY(sell_col0_update(n, npr, pc->Asoff.p, pc->Asci.p, pc->Asv.p, pc->Asg,
                                               (const float *)dp, pc->t3a.p, s));
            else BO_TRY(sell_col0_update(n, npr, pc->Asoff.p, pc->Asci.p, pc->Asv.p, pc->Asg, (const double *)dp,
                                         pc->t3a.p, s));
        } else {
            if (mixed) BO_TRY(slot_col0_update(g, pc->A.p, (const float *)dp, pc->t3a.p, s));
            else BO_TRY(slot_col0_update(g, pc->A.p, (const double *)dp, pc->t3a.p, s));
        }
    }
    if (acc) {
        if (mixed) return fstage_apply_acc<float>(pc, pc->t3a.p, (const float *)dp, z, s);
        return fstage_apply_acc<double>(pc, pc->t3a.p, (const double *)dp, z, s);
    }
    BO_TRY(fstage_apply(pc, pc->t3a.p, nullptr, pc->t3b.p, s));
    return axpby(3 * n, 1.0, pc->t3b.p, 1.0, z, s);
}

// z = M^{-1} v through a HIP graph of cpr_apply captured once per setup on a
// private stream (input and output go through fixed buffers of the handle)
bo_status cpr_apply_graph(bo_cpr *pc, const double *v, double *z, hipStream_t s) {
    size_t len = (size_t)pc->bs * pc->n;
    if (!pc->gexec) {
        BO_TRY(pc->g_in.alloc(len));
        BO_TRY(pc->g_out.alloc(len));
        if (!pc->cap_stream) BO_HIP(hipStreamCreateWithFlags(&pc->cap_stream, hipStreamNonBlocking));
        BO_HIP(hipStreamBeginCapture(pc->cap_stream, hipStreamCaptureModeThreadLocal));
        bo_status st = cpr_apply(pc, pc->g_in.p, pc->g_out.p, pc->cap_stream);
        hipGraph_t graph = nullptr;
        hipError_t e = hipStreamEndCapture(pc->cap_stream, &graph);
        if (st != BO_OK || e != hipSuccess) {
            if (graph) (void)hipGraphDestroy(graph);
            return st != BO_OK ? st : fail(BO_ERR_HIP, std::string("graph capture: ") + hipGetErrorString(e));
        }
        e = hipGraphInstantiate(&pc->gexec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) {
            pc->gexec = nullptr;
            return fail(BO_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
        }
    }
    BO_HIP(hipMemcpyAsync(pc->g_in.p, v, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
    BO_HIP(hipGraphLaunch(pc->gexec, s));
    BO_HIP(hipMemcpyAsync(z, pc->g_out.p, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
    return BO_OK;
}

}  // namespace bo

using namespace bo;

extern "C" void bo_cpr_default_opts(bo_cpr_opts *o) {
    if (!o) return;
    o->fpf = 0;
    o->ftype = BO_F_ILU_TILED;
    o->tile_x = 8;
    o->tile_y = 8;
    o->theta = 0.08;
    o->coarse_max = 192;
    o->max_levels = 12;
    o->smoother = BO_SMOOTH_GS;
    o->sweeps = 1;
    o->use_amg = 1;
    o->qi_mode = BO_QI_BLOCK;
    o->precision = BO_PREC_FP64;
    o->csmoother = BO_CSMOOTH_L1;
    o->npr = 0;
    o->sell_rows = 0;
    o->condense = 0;
}

extern "C" void bo_fgmres_default_opts(bo_fgmres_opts *o) {
    if (!o) return;
    o->m = 30;
    o->maxit = 1500;
    o->rtol = 1e-6;
    // CGS2 with the second projection delayed one step: the same iterations
    // as CGS2 with two passes over the basis per step instead of three
    o->orth = 2;
    o->timing = 0;
    // direct launches: the host enqueues one Arnoldi step ahead, and the
    // replayed graph's copies in and out cost more than the launches it saves
    o->graph = 0;
    o->flexible = 1;
}

// grid == NULL: the general form (A kept as BSR; block-Jacobi F stage; the
// pressure system over the first opts->npr rows)
bo_status bo::cpr_setup_impl(const bo_bsr *A, const bo_grid *grid, const bo_cpr_opts *opts, bo_cpr *pc,
                             hipStream_t s) {
    if (pc->gexec) {  // buffers and levels may change: capture again on the next solve
        (void)hipGraphExecDestroy(pc->gexec);
        pc->gexec = nullptr;
    }
    pc->has_grid = grid != nullptr;
    pc->g = grid ? Grid{grid->nx, grid->ny, grid->nz} : Grid{A->nbrows, 1, 1};
    pc->general = grid == nullptr || pc->g.n() != A->nbrows;
    pc->n = A->nbrows;
    pc->ncell = grid ? (int)(pc->g.n() * (grid->dual ? 2 : 1)) : A->nbrows;
    pc->nnzb = A->nnzb;
    pc->o = *opts;
    pc->npr = (opts->npr > 0 && opts->npr < pc->n) ? opts->npr : pc->n;
    long long n = pc->n;
    BO_TRY(pc->flag.alloc(1));
    if (!pc->general) BO_TRY(pc->A.alloc(63 * n));
    // inputs must be finite
    BO_HIP(hipMemsetAsync(pc->flag.p, 0, sizeof(int32_t), s));
    k_check_finite<<<grid_for(9LL * A->nnzb), kBlock, 0, s>>>(9LL * A->nnzb, A->val, pc->flag.p);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    HostRead rd{pc->flag.p, sizeof bad, &bad};
    BO_TRY(host_reads(&rd, 1, s));
    if (bad) return fail(BO_ERR_NONFINITE, "bo_cpr_setup: the matrix holds NaN or Inf");
    // the BSR copy: the general form's operator, and the natural-order ILU's pattern
    if (pc->general || pc->o.ftype == BO_F_ILU_NATURAL) {
        BO_TRY(pc->Arp.alloc(n + 1));
        BO_TRY(pc->Aci.alloc(A->nnzb));
        BO_TRY(pc->Aval.alloc(9 * (size_t)A->nnzb));
        // (a matrix already in these buffers, the condensed form's reduced
        // system, is not copied)
        if (A->rowptr != pc->Arp.p)
            BO_HIP(hipMemcpyAsync(pc->Arp.p, A->rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToDevice, s));
        if (A->colind != pc->Aci.p)
            BO_HIP(hipMemcpyAsync(pc->Aci.p, A->colind, sizeof(int32_t) * A->nnzb, hipMemcpyDeviceToDevice, s));
        if (A->val != pc->Aval.p)
            BO_HIP(hipMemcpyAsync(pc->Aval.p, A->val, sizeof(double) * 9 * (size_t)A->nnzb, hipMemcpyDeviceToDevice,
                                  s));
    }
    if (pc->general) {
        // a grid's cell rows (the first N rows) keep their stencil blocks at
        // implicit columns
        pc->Asg = grid && pc->g.n() <= n ? SellGrid{(int)pc->g.n(), pc->g.nx, pc->g.ny, pc->g.nz} : SellGrid{};
        BO_TRY(sell_build(n, pc->Arp.p, pc->Aci.p, pc->Aval.p, pc->Asg, pc->Asoff, pc->Asci, pc->Asv, s));
    } else {
        BO_TRY(bsr_to_slots(pc->g, A->rowptr, A->colind, A->val, pc->A.p, s));
    }
    BO_TRY(qi_decouple(pc, s));
    // The F stage's factors depend on A alone: they are built on a second
    // stream, forked from s and joined back below, while the AMG setup (many
    // small launches and a few host reads) runs on s.  The fork waits for
    // level 0's aggregates: the factorisation's HBM traffic would otherwise
    // slow level 0's strength and MIS-2 passes, and the Galerkin products that
    // follow are bound by LDS hashing rather than HBM.
    if (!pc->side) BO_HIP(hipStreamCreateWithFlags(&pc->side, hipStreamNonBlocking));
    for (hipEvent_t &e : pc->evs)
        if (!e) BO_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    bool forked = false;
    bo_status fst = BO_OK;
    auto fork = [&]() -> bo_status {
        forked = true;
        BO_HIP(hipEventRecord(pc->evs[0], s));
        BO_HIP(hipStreamWaitEvent(pc->side, pc->evs[0], 0));
        fst = fstage_launch(pc, pc->side);
        return fst;
    };
    bo_status ast = BO_OK;
    if (pc->o.use_amg) {
        ast = amg_setup(pc, s, fork);
        if (ast == BO_OK && pc->o.precision != BO_PREC_FP64) ast = amg_make_f32(pc, s);
    }
    if (!forked) {
        const bo_status e = fork();
        if (ast == BO_OK && e != BO_OK && fst == BO_OK) fst = e;
    }
    // join on every path: nothing may still run on the side stream when this returns
    BO_HIP(hipEventRecord(pc->evs[1], pc->side));
    BO_HIP(hipStreamWaitEvent(s, pc->evs[1], 0));
    if (fst != BO_OK || ast != BO_OK) {
        (void)hipStreamSynchronize(s);
        return fst != BO_OK ? fst : ast;
    }
    BO_TRY(fstage_check(pc, s));
    BO_TRY(pc->rp_.alloc(n));
    BO_TRY(pc->dp_.alloc(n));
    BO_TRY(pc->t3a.alloc(3 * n));
    BO_TRY(pc->t3b.alloc(3 * n));
    BO_TRY(pc->t3c.alloc(3 * n));
    BO_TRY(pc->wf.alloc(3 * n));
    BO_TRY(pc->red.init());
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}

// Option and size checks of bo_cpr_setup for a matrix of nbrows block rows
// (also applied to the reduced system of the condensed form).
bo_status bo::cpr_check(int32_t nbrows, const bo_grid *grid, const bo_cpr_opts *opts) {
    const long long gn = grid ? (long long)grid->nx * grid->ny * grid->nz : 0;
    if (grid && (grid->nx < 1 || grid->ny < 1 || grid->nz < 1 || gn * (grid->dual ? 2 : 1) > nbrows ||
                 (grid->dual && gn * 2 > nbrows)))
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: grid does not match the matrix size");
    const bool general = !grid || gn != nbrows;
    if (!grid && opts->ftype != BO_F_BJ)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr_setup: without a grid the F stage must be BO_F_BJ");
    if (general && opts->ftype == BO_F_ILU_TILED && opts->precision != BO_PREC_FP64 && (!grid || grid->dual))
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr_setup: with matrix cells the extended grid form's tiled ILU is "
                                        "FP64 only");
    if (general && opts->use_amg && opts->smoother == BO_SMOOTH_GS)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: red-black Gauss-Seidel needs the plain grid form");
    if (!general && opts->smoother == BO_SMOOTH_L1)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr_setup: the l1 level-0 smoother is for the general form");
    if (opts->npr < 0 || opts->npr > nbrows) return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: npr out of range");
    if (opts->sell_rows < 0) return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: sell_rows out of range");
    if (!general && opts->npr != 0 && opts->npr != nbrows)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: on a grid every row is a pressure row");
    if ((long long)nbrows * 7 >= (1LL << 31)) return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: matrix too large");
    const bo_cpr_opts &o = *opts;
    if (o.ftype != BO_F_BJ && o.ftype != BO_F_ILU_TILED && o.ftype != BO_F_ILU_NATURAL)
        return fail(BO_ERR_UNSUPPORTED, "bo_cpr_setup: F stage must be BO_F_BJ, BO_F_ILU_TILED or BO_F_ILU_NATURAL");
    if (o.ftype == BO_F_ILU_NATURAL) {
        if (o.precision != BO_PREC_FP64)
            return fail(BO_ERR_UNSUPPORTED, "bo_cpr_setup: the natural-order ILU is FP64 only");
        if (grid->dual)
            return fail(BO_ERR_UNSUPPORTED, "bo_cpr_setup: the natural-order ILU needs a grid without matrix cells "
                                            "(the plain or the condensed form)");
        if (nbrows - gn > kNatExtraRows)
            return fail(BO_ERR_UNSUPPORTED, "bo_cpr_setup: the natural-order ILU takes at most 4096 rows after the "
                                            "grid's cells");
    }
    if (o.ftype == BO_F_ILU_TILED && (o.tile_x < 1 || o.tile_y < 1 || o.tile_x * o.tile_y > 64))
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: tiles need 1 <= tile_x*tile_y <= 64");
    if (o.use_amg && (o.coarse_max < 1 || o.coarse_max > kCoarseMaxLimit || !(o.theta >= 0.0) ||
                      o.sweeps < 1 || o.sweeps > 8 || o.max_levels < 1))
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: AMG options out of range");
    if (o.smoother != BO_SMOOTH_GS && o.smoother != BO_SMOOTH_JACOBI && o.smoother != BO_SMOOTH_L1)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: unknown smoother");
    if (o.csmoother != BO_CSMOOTH_JACOBI && o.csmoother != BO_CSMOOTH_L1)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: unknown coarse-level smoother");
    if (o.qi_mode != BO_QI_DIAG && o.qi_mode != BO_QI_BLOCK)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: unknown quasi-IMPES mode");
    if (o.precision != BO_PREC_FP64 && o.precision != BO_PREC_FP32 && o.precision != BO_PREC_FP32_BF16)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: unknown precision");
    return BO_OK;
}

extern "C" bo_status bo_cpr_setup(const bo_bsr *A, const bo_grid *grid, const bo_cpr_opts *opts,
                                  const bo_allocator *alloc, bo_cpr **out, void *stream) {
    if (!out) return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: out is NULL");
    *out = nullptr;
    if (!A || !opts || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: NULL argument");
    if (A->nbrows < 1 || A->nnzb < A->nbrows) return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: empty matrix");
    if (opts->condense != 0 && opts->condense != 1)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: condense must be 0 or 1");
    if (opts->condense) {
        if (!grid || !grid->dual)
            return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: condense needs the dual-porosity extended grid form");
    } else {
        BO_TRY(cpr_check(A->nbrows, grid, opts));
    }
    if (alloc && (!alloc->alloc || !alloc->free))
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_setup: an allocator needs both alloc and free");
    bo_cpr *pc = new (std::nothrow) bo_cpr();
    if (!pc) return fail(BO_ERR_ALLOC, "bo_cpr_setup: out of host memory");
    if (alloc) {
        pc->has_alloc = true;
        pc->alloc = *alloc;
    }
    AllocScope scope(pc->allocator(), stream);
    bo_status st = opts->condense ? cond_setup(pc, A, grid, opts, (hipStream_t)stream)
                                   : cpr_setup_impl(A, grid, opts, pc, (hipStream_t)stream);
    if (st != BO_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        bo_cpr_destroy(pc);
        return st;
    }
    *out = pc;
    return BO_OK;
}

extern "C" bo_status bo_cpr_update(bo_cpr *pc, const bo_bsr *A, void *stream) {
    if (!pc || !A || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, "bo_cpr_update: NULL argument");
    if (pc->bs != 3) return fail(BO_ERR_INVALID_ARG, "bo_cpr_update: a 2x2-block handle (bo_cpr2_update)");
    if (A->nbrows != pc->n) return fail(BO_ERR_INVALID_ARG, "bo_cpr_update: matrix size differs from the setup");
    if (A->nnzb != pc->nnzb) return fail(BO_ERR_INVALID_ARG, "bo_cpr_update: block count differs from the setup");
    AllocScope scope(pc->allocator(), stream);
    bo_grid g{pc->g.nx, pc->g.ny, pc->g.nz, pc->ncell > pc->g.n() ? 1 : 0};
    bo_cpr_opts o = pc->o;
    bo_status st = pc->cond ? cond_setup(pc, A, &g, &o, (hipStream_t)stream)
                            : cpr_setup_impl(A, pc->has_grid ? &g : nullptr, &o, pc, (hipStream_t)stream);
    if (st != BO_OK) {
        (void)hipStreamSynchronize((hipStream_t)stream);
        pc->nlev = 0;
        pc->broken = true;
    } else {
        pc->broken = false;
    }
    return st;
}

extern "C" void bo_cpr_destroy(bo_cpr *pc) {
    if (!pc) return;
    (void)hipDeviceSynchronize();
    AllocScope scope(pc->allocator(), nullptr);
    cond_destroy(pc);
    for (hipEvent_t &e : pc->ev)
        if (e) (void)hipEventDestroy(e);
    for (hipEvent_t &e : pc->evf)
        if (e) (void)hipEventDestroy(e);
    if (pc->gexec) (void)hipGraphExecDestroy(pc->gexec);
    if (pc->cap_stream) (void)hipStreamDestroy(pc->cap_stream);
    for (hipEvent_t &e : pc->evs)
        if (e) (void)hipEventDestroy(e);
    if (pc->side) (void)hipStreamDestroy(pc->side);
    delete pc;
}

extern "C" bo_status bo_cpr_apply(bo_cpr *pc, const double *v, double *z, void *stream) {
    if (!pc || !v || !z) return fail(BO_ERR_INVALID_ARG, "bo_cpr_apply: NULL argument");
    if (pc->broken) return fail(BO_ERR_INVALID_ARG, "bo_cpr_apply: the last bo_cpr_update failed");
    if (pc->cond) return cond_apply(pc, v, z, (hipStream_t)stream);
    return cpr_apply(pc, v, z, (hipStream_t)stream);
}

extern "C" bo_status bo_cpr_spmv(bo_cpr *pc, double alpha, const double *x, double beta, double *y, void *stream) {
    pc = cond_inner(pc);
    if (!pc || !x || !y) return fail(BO_ERR_INVALID_ARG, "bo_cpr_spmv: NULL argument");
    return op_spmv(pc, alpha, x, beta, y, (hipStream_t)stream);
}

extern "C" bo_status bo_cpr_restrict(bo_cpr *pc, const double *v, double *rp, void *stream) {
    pc = cond_inner(pc);
    if (!pc || !v || !rp) return fail(BO_ERR_INVALID_ARG, "bo_cpr_restrict: NULL argument");
    if (pc->bs == 2) return qi2_restrict(pc, v, rp, (hipStream_t)stream);
    return qi_restrict(pc, v, rp, (hipStream_t)stream);
}

extern "C" bo_status bo_cpr_vcycle(bo_cpr *pc, const double *b, double *x, void *stream) {
    pc = cond_inner(pc);
    if (!pc || !b || !x) return fail(BO_ERR_INVALID_ARG, "bo_cpr_vcycle: NULL argument");
    if (!pc->o.use_amg) return fail(BO_ERR_INVALID_ARG, "bo_cpr_vcycle: built without AMG");
    return amg_vcycle(pc, b, x, (hipStream_t)stream);
}

extern "C" bo_status bo_cpr_fstage(bo_cpr *pc, const double *r, double *x, void *stream) {
    pc = cond_inner(pc);
    if (!pc || !r || !x) return fail(BO_ERR_INVALID_ARG, "bo_cpr_fstage: NULL argument");
    if (pc->bs == 2) return fstage2_apply(pc, r, nullptr, x, (hipStream_t)stream);
    return fstage_apply(pc, r, nullptr, x, (hipStream_t)stream);
}

extern "C" bo_status bo_cpr_levels(bo_cpr *pc, int32_t *nlevels) {
    pc = cond_inner(pc);
    if (!pc || !nlevels) return fail(BO_ERR_INVALID_ARG, "bo_cpr_levels: NULL argument");
    *nlevels = pc->o.use_amg ? pc->nlev : 0;
    return BO_OK;
}

extern "C" bo_status bo_cpr_level_info(bo_cpr *pc, int32_t l, int32_t *n, int32_t *nnz, int32_t *pnnz,
                                       double *omega) {
    pc = cond_inner(pc);
    if (!pc || l < 0 || l >= pc->nlev) return fail(BO_ERR_INVALID_ARG, "bo_cpr_level_info: bad level");
    const Level &L = pc->lv[l];
    bool last = l == pc->nlev - 1;
    if (n) *n = L.n;
    if (nnz) *nnz = L.nnz;
    if (pnnz) *pnnz = last ? 0 : L.pnnz;
    if (omega) *omega = last ? 0.0 : L.omega;
    return BO_OK;
}

extern "C" bo_status bo_cpr_level_copy(bo_cpr *pc, int32_t l, int32_t *rowptr, int32_t *colind, double *val,
                                       int32_t *agg, uint8_t *root, int32_t *prowptr, int32_t *pcolind,
                                       double *pval) {
    pc = cond_inner(pc);
    if (!pc || l < 0 || l >= pc->nlev) return fail(BO_ERR_INVALID_ARG, "bo_cpr_level_copy: bad level");
    const Level &L = pc->lv[l];
    bool last = l == pc->nlev - 1;
    BO_HIP(hipDeviceSynchronize());
    if (rowptr) BO_HIP(hipMemcpy(rowptr, L.rp.p, sizeof(int32_t) * (L.n + 1), hipMemcpyDeviceToHost));
    if (colind) BO_HIP(hipMemcpy(colind, L.ci.p, sizeof(int32_t) * L.nnz, hipMemcpyDeviceToHost));
    if (val) BO_HIP(hipMemcpy(val, L.v.p, sizeof(double) * L.nnz, hipMemcpyDeviceToHost));
    if (!last) {
        if (agg) BO_HIP(hipMemcpy(agg, L.agg.p, sizeof(int32_t) * L.n, hipMemcpyDeviceToHost));
        if (root) BO_HIP(hipMemcpy(root, L.root.p, L.n, hipMemcpyDeviceToHost));
        if (prowptr) BO_HIP(hipMemcpy(prowptr, L.prp.p, sizeof(int32_t) * (L.n + 1), hipMemcpyDeviceToHost));
        if (pcolind) BO_HIP(hipMemcpy(pcolind, L.pci.p, sizeof(int32_t) * L.pnnz, hipMemcpyDeviceToHost));
        if (pval) BO_HIP(hipMemcpy(pval, L.pv.p, sizeof(double) * L.pnnz, hipMemcpyDeviceToHost));
    }
    return BO_OK;
}

extern "C" bo_status bo_cpr_copy_weights(bo_cpr *pc, double *c) {
    pc = cond_inner(pc);
    if (!pc || !c) return fail(BO_ERR_INVALID_ARG, "bo_cpr_copy_weights: NULL argument");
    BO_HIP(hipDeviceSynchronize());
    BO_HIP(hipMemcpy(c, pc->cw.p, sizeof(double) * pc->bs * pc->n, hipMemcpyDeviceToHost));
    return BO_OK;
}

// ---- FGMRES ---------------------------------------------------------------------
namespace {

// Z holds the m preconditioned basis vectors of the flexible form, or the one
// work vector of the standard form (flexible 0).
bo_status krylov_alloc(bo_cpr *pc, int m, bool flexible) {
    Krylov &K = pc->kr;
    long long len = (long long)pc->bs * pc->n;
    const int nz = flexible ? m : 1;
    if (K.m == m && K.len == len && K.nz == nz) return BO_OK;
    K.m = 0;
    BO_TRY(K.V.alloc((size_t)(m + 1) * len));
    BO_TRY(K.Z.alloc((size_t)nz * len));
    BO_TRY(K.h.alloc(2 * (2 * (m + 1) + 1)));
    BO_TRY(K.y.alloc(m + 1));
    if (K.host) (void)hipHostFree(K.host);
    K.host = nullptr;
    K.host_dev = nullptr;
    // coherent and mapped: the delayed Gram-Schmidt kernels write their
    // scalars here directly (through host_dev)
    BO_HIP(hipHostMalloc((void **)&K.host, sizeof(double) * (2 * (2 * m + 3) + m + 1),
                         hipHostMallocCoherent | hipHostMallocMapped));
    BO_HIP(hipHostGetDevicePointer((void **)&K.host_dev, K.host, 0));
    K.vptr.resize(m + 1);
    K.zptr.resize(nz);
    for (int i = 0; i <= m; i++) K.vptr[i] = K.V.p + (size_t)i * len;
    for (int i = 0; i < nz; i++) K.zptr[i] = K.Z.p + (size_t)i * len;
    K.m = m;
    K.nz = nz;
    K.len = len;
    return BO_OK;
}

}  // namespace

namespace bo {

// FGMRES(m) on pc's operator.  The residual at each restart and at exit (the
// true residual) is b - A x with the caller's matrix A, or with the handle's
// own copy when A names none (internal callers).  With opts->flexible 0 it is
// the standard right-preconditioned GMRES(m) for a fixed linear
// preconditioner: M^{-1} v_j goes to one work vector, and each cycle ends with
// x += M^{-1} (V_k y) (one more application, not counted as an iteration).
// In the delayed form the preconditioner acts on the pending vectors
// u_j = S_jj v_j + sum_{i<j} S_ij v_i, so the update is M^{-1} (V_k (S y)) with
// the upper triangular S of the re-orthogonalisation coefficients.
bo_status fgmres_core(bo_cpr *pc, UserA A, const double *b, double *x, const bo_fgmres_opts *opts,
                      bo_solve_stats *stats, hipStream_t s) {
    int m = opts->m;
    bo_solve_stats st{};
    const bool timed = opts->timing == 1;
    // graph replay of the preconditioner (not with a network attached, whose
    // buffers may grow during an application, nor while pairs are recorded,
    // which counts applications on the host)
    const bool use_graph = opts->graph == 1 && !pc->nn && !pc->rec_out;
    // steps enqueued ahead (not with a network, whose stage synchronises, nor
    // while pairs are recorded, which would record a discarded step)
    const bool allow_ahead = !pc->nn && !pc->rec_out;
    if (pc->nn) BO_HIP(hipMemsetAsync(pc->nn_used.p, 0, sizeof(int32_t), s));
    if (timed)
        for (hipEvent_t &e : pc->ev)
            if (!e) BO_HIP(hipEventCreate(&e));
    for (hipEvent_t &e : pc->evf)
        if (!e) BO_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    const bool flexible = opts->flexible != 0;
    BO_TRY(krylov_alloc(pc, m, flexible));
    Krylov &K = pc->kr;
    const long long len = K.len;
    // the delayed form needs at most 32 vectors per pass and 32-bit offsets,
    // and a preconditioner that is linear (the network's correction is not
    // applied to an unnormalised vector); otherwise CGS2
    const int orth = opts->orth == 2 && (m > 31 || len >= (1ll << 29) || pc->nn) ? 1 : opts->orth;
    const Grid &g = pc->g;
    double *V = K.V.p, *Z = K.Z.p;
    // scalars of an Arnoldi step, two sets (steps j and j+1 may be in flight):
    // [0, m+1): h1, [m+1, 2m+2): h2, [2m+2]: |w|^2
    const int hs = 2 * m + 3;
    double *hd = K.h.p;                 // device
    double *hh = K.host;                // pinned copies
    double *yh = K.host + 2 * hs;       // pinned update coefficients
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1);
    std::vector<double> Hr(orth == 2 ? (size_t)(m + 1) * m : 0, 0.0);  // delayed form: unrotated H
    // standard form with the delayed re-orthogonalisation: pending vectors U = V S
    std::vector<double> S(orth == 2 && !flexible ? (size_t)m * m : 0, 0.0);
    auto fetch = [&](int count) -> bo_status {
        BO_HIP(hipMemcpyAsync(hh, hd, sizeof(double) * count, hipMemcpyDeviceToHost, s));
        BO_HIP(hipStreamSynchronize(s));
        return BO_OK;
    };
    // ||b||
    BO_TRY(pc->red.dot(len, b, b, hd, s));
    BO_TRY(fetch(1));
    double bnorm = std::sqrt(hh[0]);
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
    double tol = opts->rtol * bnorm;
    int its = 0;
    bo_status status = BO_NOT_CONVERGED;
    for (;;) {
        // r = b - A x into V[0]
        BO_HIP(hipMemcpyAsync(V, b, sizeof(double) * len, hipMemcpyDeviceToDevice, s));
        BO_TRY(user_spmv(pc, A, -1.0, x, 1.0, V, s));
        BO_TRY(pc->red.dot(len, V, V, hd, s));
        BO_TRY(fetch(1));
        double beta = std::sqrt(hh[0]);
        st.rel_residual = beta / bnorm;
        if (!std::isfinite(beta)) { status = fail(BO_ERR_NONFINITE, "bo_fgmres_solve: residual is not finite"); break; }
        if (beta <= tol) { st.converged = 1; status = BO_OK; break; }
        if (its >= opts->maxit) break;
        if (its > 0) st.restarts++;
        BO_TRY(axpby(len, 1.0 / beta, V, 0.0, V, s));
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        if (orth == 2) std::fill(Hr.begin(), Hr.end(), 0.0);
        std::fill(S.begin(), S.end(), 0.0);
        double g0 = beta;  // delayed form: |r| in the rescaled first basis vector
        int k = 0;
        // One Arnoldi step is enqueued as: preconditioner, SpMV, orthogonalisation
        // (scalars into set p = j % 2), normalisation of w on the device, an
        // asynchronous copy of the scalars and an event.  While the estimate is
        // far from the tolerance the next step is enqueued before the host waits
        // for this one's scalars, so the GPU does not idle during the Givens
        // update; a step enqueued past convergence is discarded.
        auto enqueue_step = [&](int j) -> bo_status {
            double *vj = V + (size_t)j * len, *zj = flexible ? Z + (size_t)j * len : Z;
            double *w = V + (size_t)(j + 1) * len;
            const int p = j & 1;
            double *hdp = hd + p * hs;
            if (use_graph) BO_TRY(cpr_apply_graph(pc, vj, zj, s));
            else BO_TRY(cpr_apply(pc, vj, zj, s));
            if (timed) BO_HIP(hipEventRecord(pc->ev[2 * p], s));
            BO_TRY(op_spmv(pc, 1.0, zj, 0.0, w, s));
            if (timed) BO_HIP(hipEventRecord(pc->ev[2 * p + 1], s));
            int nv = j + 1;
            if (orth == 2) {
                // V[j] is pending: dots of [V[0..j), V[j]] with V[j] and w, then
                // V[j] final, w after its first projection pending in V[j+1]
                // (walked backwards: the dots pass left its end in cache)
                // the kernels also write their results into the pinned set p
                // (no copy kernel between this step and the next)
                double *hq = K.host_dev + p * hs;
                BO_TRY(pc->red.dcgs_dots(len, K.vptr.data(), nv, w, hdp, s, hq));
                BO_TRY(pc->red.dcgs_update(len, K.vptr.data(), j, hdp, hdp + 2 * m, hdp + 2 * m + 2, s, true,
                                           hq + 2 * m, hq + 2 * m + 2));
                BO_HIP(hipEventRecord(pc->evf[p], s));
                return BO_OK;
            }
            if (orth == 1) {
                // h1 = V^T w; w -= V h1 with h2 = V^T w; w -= V h2 with |w|^2
                // (the middle pass walks backwards: each pass starts on the
                // part of the basis the previous one left in cache)
                BO_TRY(pc->red.cgs_pass(len, w, K.vptr.data(), nv, nullptr, true, hdp, s));
                BO_TRY(pc->red.cgs_pass(len, w, K.vptr.data(), nv, hdp, true, hdp + (m + 1), s, true));
                BO_TRY(pc->red.cgs_pass(len, w, K.vptr.data(), nv, hdp + (m + 1), false, hdp + 2 * (m + 1), s));
            } else {
                for (int i = 0; i < nv; i++) {
                    BO_TRY(pc->red.multidot(len, w, K.vptr.data() + i, 1, hdp + i, s));
                    BO_TRY(multiaxpy(len, K.vptr.data() + i, 1, hdp + i, -1.0, w, s));
                }
                BO_TRY(pc->red.dot(len, w, w, hdp + 2 * (m + 1), s));
            }
            BO_TRY(normalize(len, hdp + 2 * (m + 1), w, s));
            BO_HIP(hipMemcpyAsync(hh + p * hs, hdp, sizeof(double) * hs, hipMemcpyDeviceToHost, s));
            BO_HIP(hipEventRecord(pc->evf[p], s));
            return BO_OK;
        };
        BO_TRY(enqueue_step(0));
        bool next_enqueued = true;  // step j is in the stream
        for (int j = 0; j < m; j++) {
            if (!next_enqueued) BO_TRY(enqueue_step(j));
            const bool ahead = allow_ahead && j + 1 < m && its + 1 < opts->maxit && std::fabs(gv[j]) > 8.0 * tol;
            if (ahead) BO_TRY(enqueue_step(j + 1));
            next_enqueued = ahead;
            const int p = j & 1;
            const double *hq = hh + p * hs;
            BO_HIP(hipEventSynchronize(pc->evf[p]));
            its++;
            if (timed) {  // both events precede the scalars' copy, so they are complete
                float ms = 0.f;
                BO_HIP(hipEventElapsedTime(&ms, pc->ev[2 * p], pc->ev[2 * p + 1]));
                st.spmv_ms += ms;
                st.spmv_calls++;
            }
            if (orth == 2) {
                // dots [s (j), <u,u>, p (j), <u,w>], beta and r at 2m, the new
                // pending vector's |.|^2 at 2m+2
                const int nv = j + 1;
                const double beta_u = hq[2 * m], r = hq[2 * m + 1], hn = std::sqrt(hq[2 * m + 2]);
                if (!std::isfinite(beta_u) || !std::isfinite(r) || !std::isfinite(hn)) {
                    status = fail(BO_ERR_NONFINITE, "bo_fgmres_solve: NaN in the iteration");
                    goto done;
                }
                if (!(beta_u > 0.0)) {
                    // the pending vector lies in the span of the basis: the space
                    // was invariant one step earlier
                    k = j;
                    break;
                }
                if (!flexible) {
                    S[(size_t)j * m + j] = beta_u;
                    for (int i = 0; i < j; i++) S[(size_t)i * m + j] = hq[i];
                }
                if (j == 0) {
                    g0 = beta * beta_u;  // V[0] was rescaled by 1 / beta_u
                } else {
                    // the pending vector u = beta_u v_j + V s: column j-1 completed
                    for (int i = 0; i < j; i++) Hr[(size_t)i * m + j - 1] += hq[i];
                    Hr[(size_t)j * m + j - 1] = beta_u;
                }
                for (int i = 0; i < j; i++) Hr[(size_t)i * m + j] = hq[nv + i];
                Hr[(size_t)j * m + j] = r;
                Hr[(size_t)(j + 1) * m + j] = hn;
                // Givens QR of columns 0..j from the start (column j-1 changed)
                std::fill(gv.begin(), gv.end(), 0.0);
                gv[0] = g0;
                for (int c = 0; c <= j; c++) {
                    for (int i = 0; i <= c + 1; i++) H[(size_t)i * m + c] = Hr[(size_t)i * m + c];
                    for (int i = 0; i < c; i++) {
                        double a = H[(size_t)i * m + c], bb = H[(size_t)(i + 1) * m + c];
                        H[(size_t)i * m + c] = cs[i] * a + sn[i] * bb;
                        H[(size_t)(i + 1) * m + c] = -sn[i] * a + cs[i] * bb;
                    }
                    double a = H[(size_t)c * m + c], bb = H[(size_t)(c + 1) * m + c];
                    double den = std::hypot(a, bb);
                    if (!(den > 0.0)) {
                        status = fail(BO_ERR_BREAKDOWN, "bo_fgmres_solve: Arnoldi breakdown with a singular "
                                                        "Hessenberg matrix (A maps a preconditioned basis "
                                                        "vector into the span of the basis: singular or "
                                                        "inconsistent system)");
                        goto done;
                    }
                    cs[c] = a / den;
                    sn[c] = bb / den;
                    H[(size_t)c * m + c] = cs[c] * a + sn[c] * bb;
                    H[(size_t)(c + 1) * m + c] = 0.0;
                    gv[c + 1] = -sn[c] * gv[c];
                    gv[c] = cs[c] * gv[c];
                }
                k = j + 1;
                st.est_residual = std::fabs(gv[j + 1]) / bnorm;
                if (std::fabs(gv[j + 1]) <= tol || its >= opts->maxit || !(hn > 1e-300)) break;
                continue;
            }
            double hn = std::sqrt(hq[2 * (m + 1)]);
            for (int i = 0; i <= j; i++)
                H[(size_t)i * m + j] = orth == 1 ? hq[i] + hq[m + 1 + i] : hq[i];
            H[(size_t)(j + 1) * m + j] = hn;
            bool breakdown = !(hn > 1e-300);
            if (!std::isfinite(hn)) { status = fail(BO_ERR_NONFINITE, "bo_fgmres_solve: NaN in the iteration"); goto done; }
            for (int i = 0; i < j; i++) {
                double a = H[(size_t)i * m + j], bb = H[(size_t)(i + 1) * m + j];
                H[(size_t)i * m + j] = cs[i] * a + sn[i] * bb;
                H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * bb;
            }
            double a = H[(size_t)j * m + j], bb = H[(size_t)(j + 1) * m + j];
            double den = std::hypot(a, bb);
            if (!(den > 0.0)) {
                status = fail(BO_ERR_BREAKDOWN, "bo_fgmres_solve: Arnoldi breakdown with a singular Hessenberg "
                                                "matrix (A maps a preconditioned basis vector into the span "
                                                "of the basis: singular or inconsistent system)");
                goto done;
            }
            cs[j] = a / den;
            sn[j] = bb / den;
            H[(size_t)j * m + j] = cs[j] * a + sn[j] * bb;
            H[(size_t)(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            k = j + 1;
            st.est_residual = std::fabs(gv[j + 1]) / bnorm;
            if (std::fabs(gv[j + 1]) <= tol || its >= opts->maxit || breakdown) break;
        }
        for (int i = k - 1; i >= 0; i--) {
            double sum = gv[i];
            for (int q = i + 1; q < k; q++) sum -= H[(size_t)i * m + q] * yh[q];
            yh[i] = sum / H[(size_t)i * m + i];
        }
        if (!flexible && orth == 2)
            for (int i = 0; i < k; i++) {  // S y, row by row (row i uses y[i..k))
                double t = 0.0;
                for (int q = i; q < k; q++) t += S[(size_t)i * m + q] * yh[q];
                yh[i] = t;
            }
        BO_HIP(hipMemcpyAsync(K.y.p, yh, sizeof(double) * k, hipMemcpyHostToDevice, s));
        if (flexible) {
            BO_TRY(multiaxpy(len, K.zptr.data(), k, K.y.p, 1.0, x, s));
        } else {
            // u = V_k y in Z, M^{-1} u in V[k] (no longer needed), x += it
            BO_TRY(fill(len, 0.0, Z, s));
            BO_TRY(multiaxpy(len, K.vptr.data(), k, K.y.p, 1.0, Z, s));
            double *mu = V + (size_t)k * len;
            if (use_graph) BO_TRY(cpr_apply_graph(pc, Z, mu, s));
            else BO_TRY(cpr_apply(pc, Z, mu, s));
            BO_TRY(axpby(len, 1.0, mu, 1.0, x, s));
        }
    }
done:
    st.iterations = its;
    if (pc->nn) BO_HIP(hipMemcpyAsync(&st.nn_used, pc->nn_used.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BO_HIP(hipStreamSynchronize(s));
    // converged with a network attached whose every correction was rejected
    if (status == BO_OK && pc->nn && st.nn_used == 0 && its > 0) status = BO_NN_FALLBACK;
    if (stats) *stats = st;
    return status;
}

}  // namespace bo

extern "C" bo_status bo_fgmres_solve(bo_cpr *pc, const bo_bsr *A, const double *b, double *x,
                                     const bo_fgmres_opts *opts, bo_solve_stats *stats, void *stream) {
    if (!pc || !A || !b || !x || !opts || !A->rowptr || !A->colind || !A->val)
        return fail(BO_ERR_INVALID_ARG, "bo_fgmres_solve: NULL argument");
    if (pc->bs != 3) return fail(BO_ERR_INVALID_ARG, "bo_fgmres_solve: a 2x2-block handle (bo_fgmres_solve2)");
    if (pc->broken) return fail(BO_ERR_INVALID_ARG, "bo_fgmres_solve: the last bo_cpr_update failed");
    if (A->nbrows != pc->n || A->nnzb != pc->nnzb)
        return fail(BO_ERR_INVALID_ARG, "bo_fgmres_solve: A is not the matrix of the last setup or update");
    if (opts->m < 1 || opts->m > 64 || opts->maxit < 0 || !(opts->rtol > 0.0) || opts->orth < 0 ||
        opts->orth > 2 || (opts->timing != 0 && opts->timing != 1) || (opts->graph != 0 && opts->graph != 1) ||
        (opts->flexible != 0 && opts->flexible != 1) || (opts->flexible == 0 && pc->nn))
        return fail(BO_ERR_INVALID_ARG, "bo_fgmres_solve: options out of range (the standard form needs a linear "
                                        "preconditioner)");
    AllocScope scope(pc->allocator(), stream);
    if (pc->cond) return cond_solve(pc, A, b, x, opts, stats, (hipStream_t)stream, fgmres_core);
    return fgmres_core(pc, UserA{A, nullptr, nullptr}, b, x, opts, stats, (hipStream_t)stream);
}
