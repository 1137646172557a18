// The CPR preconditioner handle (internal).
#pragma once
#include "bo_common.hpp"
#include "bo_linalg.hpp"

namespace bo {

constexpr int kMaxLevels = 16;
constexpr int kCoarseMaxLimit = 1024;
// rows after a grid's cells that the natural-order ILU takes (one thread, in order)
constexpr int kNatExtraRows = 4096;

// One level of the aggregation hierarchy: CSR operator (ascending columns),
// and for every level but the coarsest the transfer operators to the next.
// A CSR matrix of many rows also kept sliced (SELL-C): slices of c rows,
// each entry position of a slice stored for its c rows together (column
// indices and values), rows shorter than the slice's longest padded with
// (their first column, 0).  off[S] is slice S's first element (c x the widths of
// the slices before it).  c = 64 (one wavefront per slice) for level 0 of a
// grid, whose stencil slices keep implicit columns; c = 16 for the others,
// whose rows vary in length (aggregates), so that a slice pads to the longest
// of 16 rows rather than of 64 (a wavefront then reads four slices, each
// position as four runs of 16 consecutive values).
struct SellMat {
    bool on = false;
    int c = 64;                   // rows per slice
    long long len = 0;            // stored elements (padding included)
    SellGrid grid{};              // level 0 of a grid: stencil slices with implicit columns
    DBuf<int32_t> off, col;
    DBuf<double> val;
    DBuf<float> val32;
};

struct Level {
    int n = 0, nnz = 0;
    DBuf<int32_t> rp, ci;
    DBuf<double> v;
    DBuf<int32_t> diagpos;
    DBuf<double> dl1;             // l1 row norms sum_j |a_ij|
    // transfer to level + 1
    int nc = 0, pnnz = 0;
    DBuf<int32_t> prp, pci, rrp, rci;
    DBuf<double> pv, rv;
    DBuf<int32_t> agg;
    DBuf<uint8_t> root, sf;
    double omega = 0.0;
    // cycle work vectors
    DBuf<double> x, b, r, t;
    // single-precision copies (mixed form)
    DBuf<float> v32, pv32, rv32, x32, b32, r32, t32, dl132;
    // sliced copies of A, P and R for levels of many rows (see SellMat)
    SellMat sA, sP, sR;
};

// setup temporaries kept with the handle, reused (grow-only) by later setups
struct SetupWork {
    DBuf<uint8_t> state, nw, d1;
    DBuf<uint64_t> m1;
    DBuf<int32_t> cnt, id, a1, rc, gcnt;
    DBuf<double> aF;
    DBuf<unsigned long long> rho;
    DBuf<int32_t> dfl;            // deferred setup flags, read once at the end (see amg_setup)
    DBuf<double> omg;             // smoother weight of each level
    DBuf<int32_t> aprp, apci;
    DBuf<double> apv, dense;
    DBuf<int32_t> sg_prod, sg_rows, sg_stat;  // sparse product: products per row, long rows, reduction words
    DBuf<int32_t> sg_rows2, sg_key;           // rows of few products but many distinct columns, launch keys
    DBuf<int32_t> plong;          // prolongator rows longer than the register path: [count, rows...]
    DBuf<int32_t> misw;           // change words of the MIS-2 rounds, one per round
    DBuf<int32_t> scan_sums;      // block sums of the prefix sums that read nothing back
};

struct Krylov {
    int m = 0;
    int nz = 0;                   // vectors in Z (m, or 1 for the standard form)
    long long len = 0;
    DBuf<double> V, Z;            // (m+1) x len, nz x len
    std::vector<const double *> vptr, zptr;   // host lists of the basis vectors
    DBuf<double> h;               // device scalars of two Arnoldi steps, 2m+3 each
    DBuf<double> y;               // m coefficients for the update
    double *host = nullptr;       // pinned: two sets of 2m+3 fetched scalars, then m+1 coefficients
    double *host_dev = nullptr;   // the same memory as the device addresses it
    ~Krylov() { if (host) (void)hipHostFree(host); }
};

struct Condensed;                 // exact elimination of dual-porosity matrix cells (bo_condense.hip)

}  // namespace bo

struct bo_cpr {
    // the caller's allocator of this handle's device memory (copied at
    // setup; has_alloc false: hipMalloc / hipFree)
    bool has_alloc = false;
    bo_allocator alloc{};
    const bo_allocator *allocator() const { return has_alloc ? &alloc : nullptr; }
    bool broken = false;          // a failed bo_cpr_update leaves the handle unusable
    // condensed dual-porosity form: the matrix cells eliminated exactly, the
    // CPR of the reduced system in cond->inner (every other member unused)
    bo::Condensed *cond = nullptr;
    int bs = 3;                   // block size: 3 (black oil), 2 (two-phase oil-water, bo_cpr2_setup) or
                                  // 1 (a scalar system with the RAS preconditioner, bo_ras_setup)
    int ras_overlap = 0;          // bs 1: columns by which each RAS tile is extended
    bo::Grid g{};
    int n = 0;                    // block rows (the cells of a grid)
    int npr = 0;                  // rows of the pressure system (the first npr block rows)
    bool general = false;         // A kept in BSR form (Arp, Aci, Aval): no grid, or a grid
                                  // with extra rows (dual porosity, wells)
    int nnzb = 0;
    bool has_grid = false;        // set up with a grid (plain or extended form)
    int ncell = 0;                // cell rows (N, or 2N with dual porosity); later rows are wells
    // extended grid form's F stage: natural-order fracture pivots, matrix
    // pivots and couplings, well-row inverses (SoA 9 x count)
    bo::DBuf<double> x_einv_f, x_einv_m, x_amf, x_afm, x_einv_w;
    bo::DBuf<int32_t> Arp, Aci;
    bo::DBuf<double> Aval;
    bo::DBuf<int32_t> Asoff, Asci;  // sliced copy of A for the solver's SpMV (general form)
    bo::DBuf<double> Asv;
    bo::SellGrid Asg{};           // its grid rows (stencil slices with implicit columns)
    bo_cpr_opts o{};
    // operator (copy of A) in slot layout, 7 bs^2 N (63 N, or 28 N for 2x2 blocks)
    bo::DBuf<double> A;
    // decoupling rows, bs N
    bo::DBuf<double> cw;
    // level-0 pressure matrix in slot layout (7 * N) and the hierarchy
    bo::DBuf<double> app;
    bo::DBuf<float> app32;
    // the same split by colour for the red-black sweeps (2 x 7 x ceil(N/2))
    bo::DBuf<double> appc;
    bo::DBuf<float> appc32;
    int nlev = 0;
    bo::Level lv[bo::kMaxLevels];
    int coarse_n = 0;
    bo::DBuf<double> cinv;        // dense inverse of the coarsest matrix
    bo::DBuf<float> cinv32;
    // F stage: block-Jacobi inverses (SoA 9 * N), or the tiled ILU factors in
    // (tile, step, lane) order with the cell index of each slot and the
    // forward-sweep result in the same order; in the mixed form the same
    // buffers hold FP32 or BF16 values
    bo::DBuf<double> einv;
    bo::DBuf<double2> ilu_f, ilu_b;
    bo::DBuf<double2> ilu_pf, ilu_pb;  // mixed form: the FP64 packed blocks its factorisation reads
    bo::DBuf<double> ilu_w;
    bo::DBuf<float> ilu_w32;           // mixed form
    bo::DBuf<int32_t> ilu_slot;
    // natural-order block ILU(0) (BO_F_ILU_NATURAL): the factors over the
    // pattern of Arp / Aci (unit-lower blocks L_ik at the lower entries, the
    // updated blocks at the others), the pivots' inverses (9 per row), the
    // grid's cells by hyperplane with the hyperplanes' offsets (host and
    // device copies), the forward sweep's result
    bo::DBuf<double> nat_lu, nat_inv, nat_y;
    bo::DBuf<int32_t> nat_perm, nat_lptr_d;
    std::vector<int32_t> nat_lptr;
    // work vectors
    bo::DBuf<double> rp_, dp_, t3a, t3b, t3c, wf;
    bo::DBuf<int32_t> flag;
    bo::DBuf<int32_t> fflag;      // the F stage's singular-pivot flag (its own: it runs beside the AMG setup)
    hipStream_t side = nullptr;   // second stream of the setup: the F stage's factorisation
    hipEvent_t evs[2] = {};       // fork to and join from that stream
    bo::SetupWork sw;
    bo::Reducer red;
    bo::Krylov kr;
    bo::DBuf<double> bicg;        // BiCGSTAB work vectors: 7 x bs N (r, rhat, p, v, phat, shat, t)
    bo::DBuf<double> bicg_sc;     // its device scalars
    hipEvent_t ev[4] = {};        // SpMV timing in bo_fgmres_solve (two Arnoldi steps in flight)
    hipEvent_t evf[2] = {};       // completion of an Arnoldi step's scalars
    // the preconditioner as a HIP graph (captured once per setup)
    hipGraphExec_t gexec = nullptr;
    hipStream_t cap_stream = nullptr;
    bo::DBuf<double> g_in, g_out;
    // learned pressure-stage correction (not owned) and its work arrays
    bo_nn *nn = nullptr;
    bo::DBuf<float> nn_z;                 // standardised log-permeability
    bo::DBuf<double> nn_part, nn_mom, nn_dp;
    bo::DBuf<float> nn_dp32;
    bo::DBuf<int32_t> nn_used;
    bo::DBuf<double> nn_alpha;            // the judge's multiple of the correction (0: not used)
    // pair collection: recorded pressure-stage inputs (caller's buffer)
    float *rec_out = nullptr;
    int rec_max = 0, rec_n = 0;
    bo::DBuf<double> pg_V, pg_Z, pg_h, pg_x, pg_r, pg_v, pg_xs;
};

namespace bo {
// setup of a handle (plain grid, extended grid or general form), see bo_cpr_setup
bo_status cpr_setup_impl(const bo_bsr *A, const bo_grid *grid, const bo_cpr_opts *opts, bo_cpr *pc, hipStream_t s);
bo_status cpr_check(int32_t nbrows, const bo_grid *grid, const bo_cpr_opts *opts);
bo_status cpr_apply(bo_cpr *pc, const double *v, double *z, hipStream_t s);
// natural-order block ILU(0) by level scheduling (BO_F_ILU_NATURAL)
bo_status nat_launch(bo_cpr *pc, hipStream_t s);
bo_status nat_apply(bo_cpr *pc, const double *r, const double *dp, double *out, hipStream_t s);
// The caller's matrix of a solve, for its true residual: a 3x3-block or a
// 2x2-block BSR matrix, or the slot coefficients of a scalar system on the
// handle's grid (at most one of the three), or none: the handle's own copy
// of the operator.
struct UserA {
    const bo_bsr *a3;
    const bo_bsr2 *a2;
    const double *c1;
};
bo_status user_spmv(bo_cpr *pc, const UserA &A, double alpha, const double *x, double beta, double *y,
                    hipStream_t s);
bo_status fgmres_core(bo_cpr *pc, UserA A, const double *b, double *x, const bo_fgmres_opts *opts,
                      bo_solve_stats *stats, hipStream_t s);
// condensed form (bo_condense.hip)
bo_status cond_setup(bo_cpr *pc, const bo_bsr *A, const bo_grid *grid, const bo_cpr_opts *opts, hipStream_t s);
bo_status cond_apply(bo_cpr *pc, const double *v, double *z, hipStream_t s);
// a Krylov solver on pc's operator
typedef bo_status (*KrylovCore)(bo_cpr *pc, UserA A, const double *b, double *x, const bo_fgmres_opts *opts,
                                bo_solve_stats *stats, hipStream_t s);
bo_status bicgstab_core(bo_cpr *pc, UserA A, const double *b, double *x, const bo_fgmres_opts *opts,
                        bo_solve_stats *stats, hipStream_t s);
bo_status op_spmv(bo_cpr *pc, double alpha, const double *x, double beta, double *y, hipStream_t s);
bo_status cond_solve(bo_cpr *pc, const bo_bsr *A, const double *b, double *x, const bo_fgmres_opts *opts,
                     bo_solve_stats *stats, hipStream_t s, KrylovCore core);
void cond_destroy(bo_cpr *pc);
// the handle whose stages and hierarchy the entry points act on: the reduced
// system's CPR for a condensed handle, pc itself otherwise (NULL stays NULL)
bo_cpr *cond_inner(bo_cpr *pc);
// 2x2-block handles (bo_cpr2.hip)
bo_status cpr2_apply(bo_cpr *pc, const double *v, double *z, hipStream_t s);
bo_status slot2_spmv(bo_cpr *pc, double alpha, const double *x, double beta, double *y, hipStream_t s);
bo_status qi2_restrict(bo_cpr *pc, const double *v, double *rp, hipStream_t s);
bo_status fstage2_apply(bo_cpr *pc, const double *r, const double *dp, double *out, hipStream_t s);
// scalar systems (bo_ras.hip)
bo_status scalar_spmv(const Grid &g, const double *A, double alpha, const double *x, double beta, double *y,
                      hipStream_t s);
bo_status ras_apply(bo_cpr *pc, const double *r, double *z, hipStream_t s);
}  // namespace bo
