/*
 * bo: fully implicit black-oil Jacobian assembly and CPR-preconditioned
 * flexible GMRES on one AMD Instinct MI355X (gfx950).
 *
 * Method (Liu, Shen, Wang, Yang, Chen, "Numerical Simulation of Multi-phase
 * Flow in Porous Media on Parallel Computers"):
 *   - Section 2.1: three-phase, three-component black-oil model (Darcy's law,
 *     saturation and potential constraints, no-flow boundary, Stone II oil
 *     relative permeability) with unknowns (Po, Sw, Sg) per cell;
 *   - Section 2.2: the two-phase oil-water model, unknowns (Po, Sw), with
 *     2x2-block Jacobians (the bo_*2 entry points);
 *   - Section 2.3: Peaceman wells, fixed bottom-hole pressure control;
 *   - Section 3: finite differences on a structured hexahedral grid (7-point);
 *   - Section 3.2: block structure of the Jacobian, quasi-IMPES decoupling, and
 *     the CPR-FPF preconditioner (RAS with ILU(0) subdomain solves, AMG on the
 *     pressure block);
 *   - Section 3.3 (data structures and algorithms): y = alpha A x + beta y,
 *     dot products and norms, and the Krylov solvers (GMRES).
 *
 * Conventions shared by every entry point
 *   - Cells are numbered g = i + nx*(j + ny*k), i fastest.
 *   - Vectors have 3N doubles interleaving (Po, Sw, Sg) per cell.
 *   - A BSR matrix has 3x3 blocks stored row-major (block row = equation
 *     (oil, water, gas), block column = unknown (Po, Sw, Sg)); column indices
 *     ascend within each block row.
 *   - Every pointer is a DEVICE pointer unless its comment says [host].
 *   - `stream` is a hipStream_t (NULL: the default stream); all device work is
 *     enqueued on it.  Functions return after enqueueing unless stated.
 *   - Every function returns a bo_status.  On an error nothing is guaranteed
 *     about outputs, and bo_last_error() (per thread) describes the failure.
 *   - The library never takes ownership of caller buffers.  Handles own their
 *     device memory and release it in the matching destroy call.
 *   - A handle is not thread-safe; distinct handles may be used concurrently
 *     on distinct streams.
 */
#ifndef BO_H
#define BO_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BO_OK = 0,
    BO_NOT_CONVERGED = 1,         /* solver reached maxit; x holds the last iterate */
    BO_NN_FALLBACK = 2,           /* information, not an error: the solve converged with a
                                     network attached, and the judge kept none of its
                                     corrections (every pressure stage was the plain V-cycle) */
    BO_ERR_INVALID_ARG = -1,
    BO_ERR_HIP = -2,              /* a HIP runtime call failed */
    BO_ERR_ALLOC = -3,
    BO_ERR_NONFINITE = -4,        /* NaN/Inf in an input or during the iteration */
    BO_ERR_SINGULAR_BLOCK = -5,   /* a 3x3 pivot block is singular */
    BO_ERR_SINGULAR_COARSE = -6,  /* the coarsest AMG matrix is singular */
    BO_ERR_BREAKDOWN = -7,        /* Arnoldi breakdown with a singular Hessenberg matrix: the
                                     Krylov space holds no better iterate (a singular or
                                     inconsistent system); x keeps the last restart's iterate */
    BO_ERR_UNSUPPORTED = -8       /* e.g. a matrix pattern that is not the grid's 7-point stencil */
} bo_status;

/* Thread-local description of the last error (never NULL). */
const char *bo_last_error(void);
/* Library version string. */
const char *bo_version(void);

/* Block sparse row matrix with 3x3 blocks. */
typedef struct {
    int32_t nbrows;     /* block rows (= cells) */
    int32_t nnzb;       /* stored blocks */
    int32_t *rowptr;    /* nbrows+1 */
    int32_t *colind;    /* nnzb, ascending within each row */
    double *val;        /* 9*nnzb, row-major blocks */
} bo_bsr;

/* Block sparse row matrix with 2x2 blocks (the two-phase oil-water model,
 * Section 2.2): block row = equation (oil, water), block column = unknown
 * (Po, Sw), row-major; vectors interleave (Po, Sw) per cell (2N doubles). */
typedef struct {
    int32_t nbrows;     /* block rows (= cells) */
    int32_t nnzb;       /* stored blocks */
    int32_t *rowptr;    /* nbrows+1 */
    int32_t *colind;    /* nnzb, ascending within each row */
    double *val;        /* 4*nnzb, row-major blocks */
} bo_bsr2;

/* Fluid and rock description (field units: psi, ft, mD, cP, days). */
typedef struct {
    double p_ref;                   /* reference pressure */
    double Bw0, cw, Bo0, co, Bg0, cg;   /* B_a(p) = B_a0 (1 - c_a (p - p_ref)) */
    double Rs0, crs;                /* R_s(p) = Rs0 (1 + crs (p - p_ref)), Mscf/STB */
    double mu_w, mu_o, mu_g;        /* viscosities */
    double c_r;                     /* rock compressibility, phi = phi0 (1 + c_r (p - p_ref)) */
    double rho_wsc, rho_osc, rho_gsc;   /* surface densities, lbm/ft3 (gas: lbm/scf) */
    double swc, sor, sorg, sgc;     /* Corey end points */
    int32_t nw, no, ng;             /* Corey exponents (integers >= 1) */
    double tcoef;                   /* Darcy unit constant (0.001127) */
    double rb_ft3;                  /* ft3 per reservoir barrel (5.615) */
    double grav;                    /* psi per (lbm/ft3 * ft) (1/144) */
    int32_t gravity;                /* 0: potentials without the density term */
    int32_t inj_total_mobility;     /* 1: water injectors use the cell's total mobility */
} bo_fluid;

/* A vertical well through cells (i, j, k_top..k_bot), 0-based. */
typedef struct {
    int32_t i, j, k_top, k_bot;
    int32_t injector;   /* 1: water injector, 0: producer */
    int32_t control;    /* BO_CTRL_* (Section 2.3) */
    double target;      /* BO_CTRL_BHP: bottom-hole pressure at the top perforation's
                           depth, psi; rate controls: rate in STB/day (> 0 for
                           injection and production alike) */
    double rw, skin;    /* wellbore radius (ft) and skin */
} bo_well;

/* Well controls (Section 2.3).  A fixed-rate well adds one block row after the
 * cell rows, in well order, with unknowns (p_h, 0, 0): row 0 is the rate
 * constraint sum_m q_m - target (injected water for BO_CTRL_WRATE, which
 * needs an injector; produced oil + water for BO_CTRL_LRATE, which needs a
 * producer), rows 1 and 2 the identity. */
enum { BO_CTRL_BHP = 0, BO_CTRL_WRATE = 1, BO_CTRL_LRATE = 2 };

typedef struct {
    int32_t nx, ny, nz;
    double dx, dy, dz;          /* cell sizes, ft */
    double top_depth;           /* depth of the grid top, ft (positive down) */
    const double *kx, *ky, *kz; /* N permeabilities, mD */
    const double *phi0;         /* N porosities at p_ref */
    bo_fluid fluid;
    int32_t nwells;
    const bo_well *wells;       /* [host] nwells entries; no two perforations may share a cell */
    /* dual porosity (fractured reservoirs, Section 2.1): with dual != 0 each
     * location g also holds a matrix cell, block row N + g, exchanging fluid
     * only with its fracture cell g through T_mf = tcoef sigma km V_b (upstream
     * weighted, same depth); kx, ky, kz and phi0 then describe the fractures,
     * wells perforate fracture cells */
    int32_t dual;
    const double *km;           /* N matrix permeabilities, mD (dual only) */
    const double *phim;         /* N matrix porosities at p_ref (dual only) */
    double sigma;               /* shape factor, ft^-2 (dual only) */
} bo_problem;

/* ---- a1: Jacobian and right-hand side -------------------------------- */

/* [host only] Sizes of the Jacobian of `p`: nbrows = N cell rows (2N with
 * dual porosity) plus one per fixed-rate well; nnzb = blocks of the 7-point
 * pattern, plus the fracture-matrix pairs (3 per location), plus 2 per
 * perforation of a fixed-rate well and 1 per such well.  Fails with
 * BO_ERR_INVALID_ARG when indices would overflow int32. */
bo_status bo_jacobian_bsr_size(const bo_problem *p, int32_t *nbrows, int32_t *nnzb);

/* Residual R of the discrete black-oil equations (Sections 2.1, 2.3, 3) at the
 * Newton iterate x_new with old state x_old (3 nbrows each; a fixed-rate
 * well's entries are (p_h, 0, 0)) and time step dt (days), and its analytic
 * Jacobian dR/dx_new.  Writes J's pattern and values into the caller-allocated
 * J (rowptr nbrows+1, colind nnzb, val 9*nnzb from bo_jacobian_bsr_size) and
 * b = -R, so that J dx = b is the Newton system.  Row order: fracture (or
 * single-porosity) cells, matrix cells, fixed-rate wells; columns ascending
 * (stencil, then the matrix cell, then the well).  Residual rows are per unit
 * surface volume (STB/day for oil and water, Mscf/day for gas). */
bo_status bo_jacobian_bsr(const bo_problem *p, const double *x_old, const double *x_new, double dt,
                          bo_bsr *J, double *b, void *stream);

/* For callers that cannot allocate memory (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc): the same Jacobian and
 * right-hand side as bo_jacobian_bsr, bit for bit, from the same kernels,
 * without any allocation (no hipMalloc / hipFree, no pinned host memory, no
 * host synchronisation, no memset).  Its only scratch memory, the block sums
 * of the row-pointer scan, is a fixed device array of the library (one
 * 32-bit word per 1024 block rows, at most 65536 words = 256 KiB per GPU,
 * held until the process ends); the row counts are staged in J->colind
 * before the value kernels overwrite it.  Fails with BO_ERR_INVALID_ARG for
 * more than bo_jacobian_bsr_noalloc_max_rows() block rows.  Calls on one GPU
 * share that array: calls that overlap in time on one GPU (on different
 * streams, or from different host threads) race and must be serialised by
 * the caller.  Unlike bo_jacobian_bsr it does not read the pattern size back
 * to check it. */
bo_status bo_jacobian_bsr_noalloc(const bo_problem *p, const double *x_old, const double *x_new, double dt,
                                  bo_bsr *J, double *b, void *stream);
/* Largest nbrows bo_jacobian_bsr_noalloc accepts (2^26). */
int32_t bo_jacobian_bsr_noalloc_max_rows(void);

/* ---- Two-phase oil-water model (Section 2.2) ----------------------------
 * The black-oil model without the gas phase: oil and water mass balances,
 * S_o + S_w = 1, unknowns (Po, Sw) per cell, zero capillary pressure, dead
 * oil (fluid.Rs0, crs and the gas properties are not read), Corey relative
 * permeabilities k_rw(S_w) and k_ro(1 - S_w) on [swc, 1 - sor] with
 * exponents nw and no.  Fluxes, gravity, units and the Peaceman wells are
 * those of bo_jacobian_bsr; only fixed-BHP wells and single porosity
 * (dual == 0; otherwise BO_ERR_UNSUPPORTED).  The pattern is the grid's
 * 7-point stencil, one block row per cell. */

/* [host] sizes of the two-phase Jacobian of p. */
bo_status bo_jacobian2_bsr_size(const bo_problem *p, int32_t *nbrows, int32_t *nnzb);

/* J (2x2 blocks; rowptr, colind and val preallocated by the caller for the
 * sizes above) and b = -R(x_new) of one implicit step from x_old to x_new
 * (2N doubles each), dt in days.  Errors as for bo_jacobian_bsr. */
bo_status bo_jacobian2_bsr(const bo_problem *p, const double *x_old, const double *x_new, double dt,
                           bo_bsr2 *J, double *b, void *stream);

/* y = alpha*A*x + beta*y on a 2x2-block BSR matrix (beta == 0: y is not read). */
bo_status bo_bsr2_spmv(const bo_bsr2 *A, double alpha, const double *x, double beta, double *y, void *stream);

/* ---- Basic operations (Section 3.3) ---------------------------------- */

/* y = alpha*A*x + beta*y on the BSR layout (beta == 0: y is not read). */
bo_status bo_bsr_spmv(const bo_bsr *A, double alpha, const double *x, double beta, double *y,
                      void *stream);

/* ---- a2-a6: CPR preconditioner --------------------------------------- */

/* F stage: block Jacobi; block ILU(0) of the whole system in natural order
 * (Section 3.2's ILU(0), no coupling dropped), applied by level scheduling
 * over the grid's hyperplanes i+j+k = const with the rows after the cells
 * taken in order: FP64 only, on the plain grid form or on a grid with at
 * most 4096 rows after its cells (fixed-rate wells; the condensed
 * dual-porosity form's reduced system), nx+ny+nz-2 dependent launches per
 * sweep; tiled block ILU(0) (couplings between tiles dropped, one wavefront
 * per tile). */
enum { BO_F_BJ = 0, BO_F_ILU_NATURAL = 1, BO_F_ILU_TILED = 3 };
/* level-0 smoother: red-black Gauss-Seidel (needs the grid), damped Jacobi,
 * or l1-Jacobi (for the general form without a grid) */
enum { BO_SMOOTH_GS = 0, BO_SMOOTH_JACOBI = 1, BO_SMOOTH_L1 = 2 };
/* smoother of the levels between the finest and the coarsest: l1-Jacobi,
 * x += (b - A x) / sum_j |a_ij| (hypre's l1 smoother, robust where Galerkin
 * products of a high-contrast pressure matrix lose diagonal dominance), or
 * damped Jacobi, x += (2/3)(b - A x) / a_ii */
enum { BO_CSMOOTH_JACOBI = 0, BO_CSMOOTH_L1 = 1 };
enum { BO_QI_DIAG = 0, BO_QI_BLOCK = 1 };          /* quasi-IMPES weights */
/* Precision of the preconditioner's inner stages.  BO_PREC_FP64: everything
 * FP64.  BO_PREC_FP32: the AMG hierarchy (level operators, P, R, coarsest
 * inverse) and the F stage's factors are built in FP64 and stored rounded to
 * FP32; the V-cycle and the ILU / block-Jacobi sweeps run in FP32 arithmetic
 * on FP32 vectors.  BO_PREC_FP32_BF16: as FP32, with the F stage's factors
 * stored in BF16 (rounded to nearest even from the FP32 value).  In every form
 * the decoupling, the restriction Pi_r v, the residual v - A x1 and the sum
 * x1 + F(r) are FP64; values cross into FP32 by round-to-nearest at the entry
 * of the V-cycle and of the F stage and leave it exactly. */
enum { BO_PREC_FP64 = 0, BO_PREC_FP32 = 1, BO_PREC_FP32_BF16 = 2 };

typedef struct {
    int32_t fpf;            /* 0: two-stage P then F; 1: Algorithm CPR-FPF */
    int32_t ftype;          /* BO_F_* */
    int32_t tile_x, tile_y; /* ILU tiles: tile_x*tile_y columns of nz cells, tile_x*tile_y <= 64 */
    double theta;           /* AMG strength threshold */
    int32_t coarse_max;     /* coarsest level size bound (<= 1024) */
    int32_t max_levels;     /* <= 16 */
    int32_t smoother;       /* level 0: BO_SMOOTH_GS (red-black) or BO_SMOOTH_JACOBI */
    int32_t sweeps;         /* pre- and post-smoothing sweeps */
    int32_t use_amg;        /* 0: no pressure stage */
    int32_t qi_mode;        /* BO_QI_* */
    int32_t precision;      /* BO_PREC_*: storage/arithmetic of the AMG hierarchy and ILU factors */
    int32_t csmoother;      /* BO_CSMOOTH_*: levels between the finest and the coarsest */
    int32_t npr;            /* general form: the pressure system is the first npr block
                               rows (cells; later rows, e.g. fixed-rate wells, stay out
                               of A_pp and are only smoothed by the F stage); 0: all */
    int32_t sell_rows;      /* AMG matrices (level operators in CSR form, P, R) of at
                               least this many rows are also kept sliced (SELL-64, one
                               thread per row in the cycle); 0: 2^20.  Same results up
                               to the order of each row's sum. */
    int32_t condense;       /* 1 (dual-porosity extended grid form only): eliminate every
                               matrix cell exactly (block Gaussian elimination of the
                               fracture-matrix pairs of Section 2.1's model) and build the
                               CPR of the reduced system over the fracture cells and the
                               fixed-rate wells, with the other options of this struct
                               (npr counts reduced rows, 0: all of them; the level-0
                               smoother becomes l1-Jacobi when the reduced system has
                               well rows and red-black Gauss-Seidel when it has none).
                               bo_cpr_apply then applies elimination, reduced CPR and
                               back-substitution to full-length vectors; bo_fgmres_solve
                               runs FGMRES on the reduced system and checks the true
                               residual of the full one; bo_cpr_spmv, the stage calls
                               and the hierarchy introspection act on the reduced
                               system (vectors of 3 (N + wells)). */
} bo_cpr_opts;

/* Fills `o` [host] with the defaults: PF, tiled ILU0 8x8, theta 0.08,
 * coarse_max 192, 12 levels, red-black GS, 1 sweep, AMG on, block QI, FP64,
 * l1-Jacobi on the coarse levels, no condensation. */
void bo_cpr_default_opts(bo_cpr_opts *o);

typedef struct bo_cpr bo_cpr;

/* A caller-supplied device allocator for a CPR handle's memory (hierarchy,
 * factors, copies of the operator, Krylov basis, work vectors).  alloc
 * returns `bytes` of device memory usable on the stream passed (NULL on
 * failure); free releases a pointer alloc returned (stream: that of the
 * entry point releasing it, NULL from bo_cpr_destroy, which synchronises the
 * device first).  ctx is passed through.  The functions may be called from
 * bo_cpr_setup, bo_cpr_update, bo_fgmres_solve, bo_bicgstab_solve, bo_cpr_attach_nn,
 * bo_cpr_collect_pairs and bo_cpr_destroy of the handle, on the calling
 * thread.  Library-wide scratch (a few small grow-only buffers per host
 * thread) and pinned host staging buffers are not taken from it. */
typedef struct {
    void *(*alloc)(size_t bytes, void *ctx, void *stream);
    void (*free)(void *ptr, void *ctx, void *stream);
    void *ctx;
} bo_allocator;

/* [host] grid of the matrix: the F stage tiles and the level-0 colours use it.
 * With nbrows == nx*ny*nz A's pattern must be the 7-point stencil of the grid.
 * Otherwise (the extended grid form) the first nx*ny*nz rows are the grid's
 * (fracture) cells, followed by nx*ny*nz matrix cells when dual != 0, then
 * other rows (fixed-rate wells), as bo_jacobian_bsr writes them. */
typedef struct { int32_t nx, ny, nz, dual; } bo_grid;

/* Builds the CPR preconditioner of A (Section 3.2): quasi-IMPES weights and the
 * decoupled pressure block, the AMG hierarchy on it, and the F-stage factors.
 * Keeps a private copy of A's values in its own layout; A may be freed after
 * return.  alloc [host, may be NULL: hipMalloc / hipFree] supplies the
 * handle's device memory for its whole life (the struct is copied).
 * Synchronises `stream` (the hierarchy sizes are decided on the host).
 * The F-stage factors are built on a second stream of the handle, forked from
 * `stream` and joined back before return, beside the AMG setup.
 * The general form, for a block pattern other than a grid's 7-point stencil,
 * keeps A in BSR form and takes the pressure system over the first opts->npr
 * rows; its level-0 smoother must be Jacobi or l1-Jacobi.  With grid == NULL
 * its F stage must be block Jacobi; with the extended grid form (see bo_grid)
 * it may also be the tiled block ILU(0) (FP64 precision only), ordered tile by
 * tile: the tile's fracture cells, their matrix cells, and the remaining rows
 * as one block-Jacobi class of their own.  BO_F_ILU_NATURAL takes a grid
 * without matrix cells (the plain form, or at most 4096 rows after the cells,
 * such as fixed-rate wells) and FP64 precision; BO_ERR_UNSUPPORTED otherwise,
 * or when a cell row has a lower block other than its -x, -y, -z
 * neighbours. */
bo_status bo_cpr_setup(const bo_bsr *A, const bo_grid *grid, const bo_cpr_opts *opts,
                       const bo_allocator *alloc, bo_cpr **out, void *stream);
/* Rebuilds pc for new values of a matrix with the same grid, pattern and
 * options (a new Newton iterate): decoupling, AMG hierarchy and F-stage
 * factors are recomputed from scratch; device memory of pc is reused when
 * large enough.  On failure pc is unusable until a later update succeeds.
 * Synchronises `stream`. */
bo_status bo_cpr_update(bo_cpr *pc, const bo_bsr *A, void *stream);
void bo_cpr_destroy(bo_cpr *pc);

/* z = M^{-1} v (3N each): PF or FPF as configured. */
bo_status bo_cpr_apply(bo_cpr *pc, const double *v, double *z, void *stream);
/* y = alpha*A*x + beta*y with the copy of A held by pc (the solver's SpMV). */
bo_status bo_cpr_spmv(bo_cpr *pc, double alpha, const double *x, double beta, double *y, void *stream);
/* Stages, for parity checks: rp (N) = Pi_r v; x (N) = one V-cycle on the
 * pressure block for right-hand side b (N); x (3N) = F(r). */
bo_status bo_cpr_restrict(bo_cpr *pc, const double *v, double *rp, void *stream);
bo_status bo_cpr_vcycle(bo_cpr *pc, const double *b, double *x, void *stream);
bo_status bo_cpr_fstage(bo_cpr *pc, const double *r, double *x, void *stream);

/* [host] Hierarchy introspection.  Copies are synchronous; any output may be NULL.
 * Level l holds n rows and nnz entries (CSR, ascending columns). */
bo_status bo_cpr_levels(bo_cpr *pc, int32_t *nlevels);
bo_status bo_cpr_level_info(bo_cpr *pc, int32_t l, int32_t *n, int32_t *nnz, int32_t *pnnz, double *omega);
bo_status bo_cpr_level_copy(bo_cpr *pc, int32_t l, int32_t *rowptr, int32_t *colind, double *val,
                            int32_t *agg, uint8_t *root, int32_t *prowptr, int32_t *pcolind, double *pval);
/* [host] decoupling rows c (3N) */
bo_status bo_cpr_copy_weights(bo_cpr *pc, double *c);

/* ---- a7: flexible GMRES ---------------------------------------------- */

typedef struct {
    int32_t m;          /* restart length (1..64) */
    int32_t maxit;      /* preconditioner applications allowed */
    double rtol;        /* stop when ||b - A x|| <= rtol ||b|| (true residual) */
    int32_t orth;       /* 0: modified Gram-Schmidt, 1: classical GS twice (CGS2),
                           2: CGS2 with the second projection of each vector
                           delayed to the next step (two passes over the basis
                           per step instead of three; m <= 31; falls back to 1
                           with a network attached or 2^29+ unknowns) */
    int32_t timing;     /* 1: time every Arnoldi SpMV with HIP events on the
                           solve's stream (stats.spmv_ms / spmv_calls) */
    int32_t graph;      /* 1: replay the preconditioner as a HIP graph captured once per
                           setup (same kernels, same results; fewer host launches, but
                           two copies through the graph's fixed buffers per
                           application); 0: launch the kernels directly */
    int32_t flexible;   /* 1: flexible GMRES (the preconditioned basis is kept, m more
                           vectors); 0: standard right-preconditioned GMRES for a fixed
                           linear preconditioner (one work vector; each restart cycle
                           ends with x += M^{-1} (V_k y), one more application that is
                           not counted as an iteration; not with a network attached) */
} bo_fgmres_opts;

void bo_fgmres_default_opts(bo_fgmres_opts *o);   /* m 30, maxit 1500, rtol 1e-6, delayed CGS2 (orth 2), no timing, direct launches (graph 0), flexible 1 */

typedef struct {
    int32_t iterations;     /* preconditioner applications */
    int32_t restarts;
    int32_t converged;
    double rel_residual;    /* true ||b - A x|| / ||b|| at exit */
    double est_residual;    /* last Arnoldi estimate |g_{j+1}| / ||b|| */
    double spmv_ms;         /* with opts.timing: summed duration of the timed SpMVs */
    int32_t spmv_calls;     /* with opts.timing: their number (one per iteration) */
    int32_t nn_used;        /* with a network attached: applications whose correction was kept */
} bo_solve_stats;

/* Right-preconditioned FGMRES(m) (Section 3.3's Krylov solver, flexible
 * form) on A x = b with the preconditioner of pc.  A must be the matrix of
 * pc's last setup or update (same pattern and values, not modified since):
 * the Arnoldi steps use pc's own layout of it, and the residual at every
 * restart and at exit (the true residual ||b - A x||) is computed from A
 * itself.  x holds the initial guess on entry and the solution on exit.
 * Synchronous: it reads one Arnoldi scalar column per iteration.  Returns
 * BO_OK, BO_NOT_CONVERGED, BO_NN_FALLBACK (converged; see bo_status),
 * BO_ERR_BREAKDOWN or another error. */
bo_status bo_fgmres_solve(bo_cpr *pc, const bo_bsr *A, const double *b, double *x, const bo_fgmres_opts *opts,
                          bo_solve_stats *stats, void *stream);

/* ---- CPR on 2x2-block (two-phase) Jacobians (Section 3.2) -------------
 * bo_cpr2_setup builds the CPR preconditioner of a 2x2-block matrix on the
 * grid's 7-point pattern (grid required, nbrows = nx*ny*nz, dual = 0):
 * quasi-IMPES weights c_i = +-(1, -d_01/d_11) from the diagonal block (sign:
 * a positive decoupled diagonal), the decoupled pressure block and the same
 * SA-AMG hierarchy as the black-oil path, and an F stage of block Jacobi or
 * the tiled block ILU(0) with 2x2 blocks; PF or FPF.  Options as for
 * bo_cpr_setup, restricted to: precision BO_PREC_FP64, level-0 smoother
 * BO_SMOOTH_GS or BO_SMOOTH_JACOBI, condense 0, npr 0 (BO_ERR_UNSUPPORTED or
 * BO_ERR_INVALID_ARG otherwise).  The handle works with bo_cpr_apply,
 * bo_cpr_spmv, bo_cpr_restrict, bo_cpr_vcycle, bo_cpr_fstage, the hierarchy
 * introspection, bo_cpr_copy_weights (2N values) and bo_cpr_destroy, on
 * vectors of 2N doubles; not with bo_cpr_update, bo_fgmres_solve,
 * bo_bicgstab_solve or a network (BO_ERR_INVALID_ARG / BO_ERR_UNSUPPORTED).
 * Synchronises `stream`. */
bo_status bo_cpr2_setup(const bo_bsr2 *A, const bo_grid *grid, const bo_cpr_opts *opts, const bo_allocator *alloc,
                        bo_cpr **pc, void *stream);
/* Rebuilds a 2x2-block handle for new values of the same pattern (as bo_cpr_update). */
bo_status bo_cpr2_update(bo_cpr *pc, const bo_bsr2 *A, void *stream);
/* FGMRES(m) and BiCGSTAB with a 2x2-block handle: as bo_fgmres_solve and
 * bo_bicgstab_solve, A the 2x2-block matrix of the last setup or update,
 * vectors of 2N doubles. */
bo_status bo_fgmres_solve2(bo_cpr *pc, const bo_bsr2 *A, const double *b, double *x, const bo_fgmres_opts *opts,
                           bo_solve_stats *stats, void *stream);
bo_status bo_bicgstab_solve2(bo_cpr *pc, const bo_bsr2 *A, const double *b, double *x, const bo_fgmres_opts *opts,
                             bo_solve_stats *stats, void *stream);

/* Right-preconditioned BiCGSTAB (Section 3.3 names it among the Krylov
 * solvers; the scaling runs of Section 4.2 use it) on A x = b with the
 * preconditioner of pc, which must be linear (no network attached:
 * BO_ERR_UNSUPPORTED).  A and x as for bo_fgmres_solve; of opts only maxit
 * (a cap on preconditioner applications, two per BiCGSTAB step) and rtol are
 * read.  The recurrence residual stops the iteration; the true residual
 * ||b - A x|| is then computed from A and the iteration restarts from it
 * while it is above rtol ||b||.  A breakdown (a zero <rhat, r>, <rhat, v> or
 * <t, t>) restarts once from the true residual; a second one returns
 * BO_ERR_BREAKDOWN with x the last iterate.  With a condensed handle the
 * reduced system is solved as for bo_fgmres_solve.  Synchronous (reads five
 * scalars per step).  stats: iterations, restarts, converged, rel_residual
 * (true, at exit) and est_residual (recurrence); the timing fields stay 0.
 * Returns BO_OK, BO_NOT_CONVERGED, BO_ERR_BREAKDOWN or another error. */
bo_status bo_bicgstab_solve(bo_cpr *pc, const bo_bsr *A, const double *b, double *x, const bo_fgmres_opts *opts,
                            bo_solve_stats *stats, void *stream);

/* ---- Scalar pressure systems: GMRES with RAS (Sections 3.2, 4.2) --------
 * A scalar system on an nx x ny x nz grid's 7-point stencil is given by its
 * slot coefficients coef[s * N + g] (7N doubles, N = nx*ny*nz): row g's
 * coefficient on its neighbour through slot s in the order -z, -y, -x,
 * diagonal, +x, +y, +z, zero where the neighbour lies outside the grid.
 * The preconditioner is restricted additive Schwarz with ILU(0) subdomain
 * solves (the paper's RAS): tiles of tile_x x tile_y grid columns over all
 * layers, each extended by `overlap` columns on every side inside the grid;
 * each extended tile's matrix (couplings leaving it dropped) is factored by
 * ILU(0) in natural order, and each tile's solve writes its own cells only. */
typedef struct {
    int32_t tile_x, tile_y;   /* (tile_x + 2 overlap)(tile_y + 2 overlap) <= 64 */
    int32_t overlap;          /* >= 0 */
} bo_ras_opts;
void bo_ras_default_opts(bo_ras_opts *o);   /* 6x6 tiles, overlap 1 */

/* y = alpha A x + beta y for the slot coefficients coef on grid (beta == 0:
 * y is not read). */
bo_status bo_scalar_spmv(const bo_grid *grid, const double *coef, double alpha, const double *x, double beta,
                         double *y, void *stream);

/* Builds the RAS preconditioner of the scalar system coef on grid (dual 0):
 * a handle of block size 1 that keeps a copy of coef.  It works with
 * bo_cpr_apply (z = M^{-1} r, N doubles), bo_cpr_spmv (the copy),
 * bo_scalar_solve and bo_cpr_destroy.  BO_ERR_SINGULAR_BLOCK for a zero
 * ILU(0) pivot.  Synchronises `stream`. */
bo_status bo_ras_setup(const bo_grid *grid, const double *coef, const bo_ras_opts *opts, const bo_allocator *alloc,
                       bo_cpr **pc, void *stream);

/* Rebuilds the factors of a RAS handle for new coefficients on the same
 * grid and options, in the handle's memory. */
bo_status bo_ras_update(bo_cpr *pc, const double *coef, void *stream);

/* GMRES(m) with the RAS handle pc on the system coef x = b (coef: the
 * matrix of the setup; the true residual is computed from it).  opts as for
 * bo_fgmres_solve; flexible 0 gives the standard right-preconditioned
 * GMRES(m) of the paper's run, and a fixed number of iterations is maxit
 * with an rtol too small to be met. */
bo_status bo_scalar_solve(bo_cpr *pc, const double *coef, const double *b, double *x, const bo_fgmres_opts *opts,
                          bo_solve_stats *stats, void *stream);

/* ---- Inexact Newton and time steps (Section 3.1) ----------------------
 * One time step solves R(x; x_old, dt) = 0 by the inexact Newton method of
 * Section 3.1: iteration l assembles b(x^l) = -R(x^l) and its Jacobian
 * (bo_jacobian_bsr), solves J dx = b with CPR-FGMRES to ||b - J dx|| <=
 * theta_l ||b||, and steps x^{l+1} = x^l + omega dx with omega = min(1,
 * ds_max / max |dS|) over the saturations of the cell rows (chopping).
 * Forcing terms theta_l (r^{l-1} = b(x^{l-1}) - J_{l-1} omega dx, the linear
 * model's residual of the step taken): BO_FORCING_EW1 ||b(x^l) - r^{l-1}|| /
 * ||b(x^{l-1})||, BO_FORCING_EW2 | ||b(x^l)|| - ||r^{l-1}|| | / ||b(x^{l-1})||,
 * BO_FORCING_EW3 gamma (||b(x^l)|| / ||b(x^{l-1})||)^beta, BO_FORCING_FIXED
 * theta_fixed (the standard Newton method); theta_0 = theta0, every theta
 * clipped to [theta_min, theta_max].  The loop stops when ||b(x^l)|| <=
 * max(atol, rtol ||b(x^0)||) (2-norms). */
enum { BO_FORCING_FIXED = 0, BO_FORCING_EW1 = 1, BO_FORCING_EW2 = 2, BO_FORCING_EW3 = 3 };
#define BO_NEWTON_HIST 64
#define BO_RUN_HIST 256

typedef struct {
    int32_t forcing;                    /* BO_FORCING_* */
    double theta0, theta_fixed, gamma, beta, theta_min, theta_max;
    double rtol, atol;                  /* nonlinear stopping test */
    int32_t max_newton;                 /* <= BO_NEWTON_HIST */
    double ds_max;                      /* largest saturation change per iteration */
} bo_newton_opts;

/* Defaults: EW1, theta0 1e-2, theta_fixed 1e-7, gamma 0.9, beta 2, theta in
 * [1e-8, 0.1], rtol 1e-6, atol 0, 20 iterations, ds_max 0.2. */
void bo_newton_default_opts(bo_newton_opts *o);

typedef struct {
    int32_t iterations;                 /* Newton iterations (linear solves) */
    int32_t linear_iterations;          /* preconditioner applications, summed */
    int32_t converged;
    double res0, res;                   /* ||b(x^0)||, ||b(x^final)|| */
    double res_hist[BO_NEWTON_HIST + 1];/* ||b(x^l)||, l = 0..iterations */
    double theta_hist[BO_NEWTON_HIST];  /* theta_l */
    double omega_hist[BO_NEWTON_HIST];  /* step lengths */
    int32_t lin_hist[BO_NEWTON_HIST];   /* linear iterations of each solve */
} bo_newton_stats;

typedef struct {
    int32_t steps, cuts;                /* accepted steps, halved steps */
    int32_t newton_iterations, linear_iterations;   /* over every attempt */
    double t;                           /* time reached, days */
    double dt_hist[BO_RUN_HIST];        /* accepted step sizes (the first BO_RUN_HIST) */
    int32_t newton_hist[BO_RUN_HIST];   /* their Newton iterations */
} bo_run_stats;

typedef struct bo_newton bo_newton;

/* [host] A Newton driver for problem p (copied, wells included; the field
 * pointers must stay valid): it owns the Jacobian, right-hand side and work
 * vectors, and the CPR handle of its systems (set up with grid and copts on
 * the first solve, updated for every later Jacobian). */
bo_status bo_newton_create(const bo_problem *p, const bo_grid *grid, const bo_cpr_opts *copts, bo_newton **out,
                           void *stream);
void bo_newton_destroy(bo_newton *h);
/* One time step: x (3 nbrows) holds the initial iterate on entry and the
 * last iterate on exit; x_old the previous time level; dt in days; fo the
 * linear solver's options (its rtol is replaced by theta_l).  Synchronous.
 * Returns BO_OK (converged), BO_NOT_CONVERGED (max_newton reached) or an
 * error. */
bo_status bo_newton_solve(bo_newton *h, const double *x_old, double *x, double dt, const bo_newton_opts *o,
                          const bo_fgmres_opts *fo, bo_newton_stats *st, void *stream);
/* Time steps over [0, t_end] from the state x (updated in place): each step
 * is bo_newton_solve from the previous state; a step that does not converge
 * is repeated with half the step (BO_NOT_CONVERGED once it falls below
 * dt_min); after a step of at most `easy` Newton iterations the next step is
 * growth times longer, capped at dt_max and the remaining time. */
bo_status bo_newton_run(bo_newton *h, double *x, double t_end, double dt0, double dt_max, double dt_min,
                        double growth, int32_t easy, const bo_newton_opts *o, const bo_fgmres_opts *fo,
                        bo_run_stats *rs, void *stream);

/* ---- a9: learned pressure-stage correction ----------------------------
 * Not part of the paper, which stops at AMG for the pressure block (Section
 * 3.2); this stage adds to the V-cycle result a correction predicted by a
 * small 3-D convolutional network and keeps it only where it lowers the
 * pressure residual, so the plain V-cycle is always the fallback.
 *
 * Network: four zero-padded 3x3x3 convolutions, channels 2 -> 16 -> 16 -> 16
 * -> 1, biases, ReLU after the first three.  Input channels: r_p / s and the
 * standardised log-permeability, s = RMS(r_p); output: the correction / s.
 * Weights are FP32 masters; the passes use BF16 operands with FP32
 * accumulation on the matrix cores.  Parameters, flat FP32: per layer
 * W[t][c_in][c_out] (tap t = 9(dz+1) + 3(dy+1) + (dx+1)) then b[c_out];
 * bo_nn_num_params() values in total.  Tensors are channel-last,
 * [nb][nz][ny][nx][channels].  A handle is not thread-safe. */
typedef struct bo_nn bo_nn;

bo_status bo_nn_create(bo_nn **out);            /* [host] out; parameters zero */
void bo_nn_destroy(bo_nn *nn);
int32_t bo_nn_num_params(void);
/* [host] params: bo_nn_num_params() floats; resets the Adam state */
bo_status bo_nn_set_params(bo_nn *nn, const float *params, void *stream);
/* [host] params / grads (either may be NULL): the current parameters and the
 * gradients of the last bo_nn_backward */
bo_status bo_nn_get_params(bo_nn *nn, float *params, float *grads, void *stream);
/* out = N(in): in [nb][nz][ny][nx][2] FP32, out [nb][nz][ny][nx] FP32.  Keeps
 * the activations for bo_nn_backward. */
bo_status bo_nn_forward(bo_nn *nn, const float *in, float *out, int32_t nb, int32_t nz, int32_t ny, int32_t nx,
                        void *stream);
/* Gradients of the mean squared error between the last bo_nn_forward output
 * and target ([nb][nz][ny][nx] FP32); loss [host, may be NULL] receives the
 * loss.  Synchronous.  Fails after a forward pass made inside CPR. */
bo_status bo_nn_backward(bo_nn *nn, const float *target, double *loss, void *stream);
/* Gradients of the A_pp-weighted error instead: the mean, over the voxels
 * whose six neighbours lie in the volume, of (A (y - target))^2 with A the
 * 7-point pressure stencil given per voxel in coef ([7][nb][nz][ny][nx] FP32,
 * slots -z, -y, -x, self, +x, +y, +z, as bo_cpr_pressure_stencil writes it):
 * the pressure residual the correction y would leave if the error were
 * target, the quantity the judge of the pressure stage measures.  Fails if
 * a side of the volume is below 3.  Synchronous. */
bo_status bo_nn_backward_weighted(bo_nn *nn, const float *coef, const float *target, double *loss, void *stream);
/* Adam (beta 0.9 / 0.999, eps 1e-8, bias-corrected) with learning rate lr on
 * the gradients of the last bo_nn_backward or bo_nn_backward_weighted. */
bo_status bo_nn_adam_step(bo_nn *nn, float lr, void *stream);

/* Attaches nn (not owned; NULL detaches) to the pressure stage of pc; logk:
 * N FP64 values of ln k, standardised here.  With a network attached, each
 * pressure stage computes dp = V(r_p) and c = s N([r_p / s, z]) and uses
 * dp + alpha c with alpha = <u, A_pp c> / ||A_pp c||^2, u = r_p - A_pp dp
 * (the multiple of c that minimises ||r_p - A_pp x||) when alpha > 0, else
 * dp (bo_solve_stats.nn_used counts the kept corrections). */
bo_status bo_cpr_attach_nn(bo_cpr *pc, bo_nn *nn, const double *logk, void *stream);
/* [device] coef ([7][N] FP32): the decoupled level-0 pressure matrix A_pp of
 * pc (plain grid form) in slot order -z, -y, -x, self, +x, +y, +z, zero where
 * the neighbour is outside the grid: the stencil bo_nn_backward_weighted
 * takes (cropped like the pairs). */
bo_status bo_cpr_pressure_stencil(bo_cpr *pc, float *coef, void *stream);
/* Training pairs from a solve of A x = b (A of the last setup/update): runs
 * FGMRES with pc for at most ncalls preconditioner applications, recording the
 * pressure-stage inputs r_p of the first ncalls of them in rp_out
 * ([ncalls][N] FP32, caller-allocated), and writes e = A_pp^{-1} r_p - V(r_p)
 * to e_out ([ncalls][N] FP32), with A_pp^{-1} r_p from GMRES on A_pp
 * preconditioned by the V-cycle to relative residual rtol_inner.  *got [host]
 * receives the number of pairs.  The attached network is not used. */
bo_status bo_cpr_collect_pairs(bo_cpr *pc, const double *b, int32_t ncalls, double rtol_inner, float *rp_out,
                               float *e_out, int32_t *got, void *stream);

#ifdef __cplusplus
}
#endif
#endif
