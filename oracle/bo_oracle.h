/*
 * FP64 CPU oracle for the fully implicit black-oil Jacobian solve.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the plain, slow reference that
 * the GPU library is checked against.  Only the tests, the smoke check and the
 * CPU-baseline leg of the benchmark load it; the product path never does.  It
 * shares no code, header or table with the GPU library.
 *
 * What it computes (Liu, Shen, Wang, Yang, Chen, "Numerical Simulation of
 * Multi-phase Flow in Porous Media on Parallel Computers"):
 *   - the black-oil residual of Section 2.1 (three components, Darcy fluxes,
 *     Peaceman wells of Section 2.3 with fixed bottom-hole pressure), discretised
 *     by the 7-point finite-difference scheme of Section 3, and its analytic
 *     Jacobian as 3x3 blocks;
 *   - the quasi-IMPES decoupling operator of Section 3.2 and the pressure block;
 *   - an aggregation AMG standing in for BoomerAMG on the pressure block;
 *   - block ILU(0) (the RAS local solver of Section 3.2) and block Jacobi;
 *   - the CPR two-stage preconditioner (PF) and Algorithm "CPR-FPF";
 *   - restarted flexible GMRES (the Krylov method named in Section 3.3);
 *   - dense LU with partial pivoting for exact solutions of tiny systems.
 *
 * Parity status per function is documented beside it.
 *
 * Conventions: cells are numbered g = i + nx*(j + ny*k); vectors are 3N long
 * and interleave (Po, Sw, Sg) per cell; residual rows are ordered (oil, water,
 * gas); 3x3 blocks are row-major (row = equation, column = unknown); BSR rows
 * hold ascending column indices.  All arithmetic is IEEE double without
 * contraction (built with -ffp-contract=off).
 */
#ifndef BO_ORACLE_H
#define BO_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { OR_OK = 0, OR_NOT_CONVERGED = 1, OR_ERR_ARG = -1, OR_ERR_ALLOC = -3,
       OR_ERR_NONFINITE = -4, OR_ERR_SINGULAR_BLOCK = -5, OR_ERR_SINGULAR_COARSE = -6 };

typedef struct {
    int nx, ny, nz;
    double dx, dy, dz, top_depth;
    const double *kx, *ky, *kz, *phi0;      /* N each */
    /* fluid and rock */
    double p_ref, Bw0, cw, Bo0, co, Bg0, cg, Rs0, crs;
    double mu_w, mu_o, mu_g, c_r;
    double rho_wsc, rho_osc, rho_gsc;
    double swc, sor, sorg, sgc;
    int nw, no, ng;
    double tcoef, rb_ft3, grav;
    int gravity;               /* 0: potentials without the density term */
    int inj_total_mobility;    /* 1: water injectors use the cell's total mobility */
    /* wells: nwells entries each; ctrl OR_CTRL_*; target: BHP (psi) or rate
     * (STB/day, positive for injection and for production alike) */
    int nwells;
    const int32_t *w_i, *w_j, *w_ktop, *w_kbot, *w_inj, *w_ctrl;
    const double *w_target, *w_rw, *w_skin;
    /* dual porosity (fractured reservoirs, Section 2.1): with dual != 0 every
     * grid cell g also holds a matrix cell, block row N + g, that exchanges
     * fluid only with its fracture cell g through T_mf = tcoef sigma km V_b;
     * kx, ky, kz and phi0 then describe the fractures */
    int dual;
    const double *km, *phim;
    double sigma;
} or_problem;

/* Well controls (Section 2.3).  A fixed-rate well adds one block row after the
 * cell rows (in well order) whose unknowns are (p_h, 0, 0): row 0 is the rate
 * constraint sum_m q_m - target (water rate of an injector, oil + water rate
 * of a producer, in STB/day), rows 1 and 2 are the identity. */
enum { OR_CTRL_BHP = 0, OR_CTRL_WRATE = 1, OR_CTRL_LRATE = 2 };

/* Block rows of the system: cells (N, or 2N with dual porosity) then one per
 * fixed-rate well; *ncell receives the number of cell rows. */
int or_rows(const or_problem *p, int *ncell);

/* Relative permeabilities (Section 2.1; Stone II for oil).  out[0..5] =
 * krw, krow, krg, krog, kro, and out[5] = dkro/dSw, out[6] = dkro/dSg. */
void or_relperm(const or_problem *p, double sw, double sg, double *out);

/* Geometry: transmissibility of the face between cells a and b (adjacent),
 * pore volume of cell g at pressure pr, Peaceman well index of cell g. */
double or_transmissibility(const or_problem *p, int a, int b);
double or_pore_volume(const or_problem *p, int g, double pr);
double or_well_index(const or_problem *p, int g, double rw, double skin);
/* fracture-matrix transfer coefficient of location g (dual porosity) */
double or_transfer(const or_problem *p, int g);

/* BSR pattern: the 7-point stencil between (fracture) cells, the fracture-
 * matrix pair of each location, and the couplings of each fixed-rate well row
 * with its perforated cells; ascending columns.  Returns nnzb; fills rowptr
 * (rows + 1) and colind (nnzb) when they are not NULL. */
int or_pattern(const or_problem *p, int32_t *rowptr, int32_t *colind);

/* Residual R (3 rows) of the discrete black-oil equations at x_new with old
 * state x_old (both 3 rows long; a fixed-rate well's entries are (p_h, 0, 0));
 * when val != NULL also the analytic Jacobian dR/dx_new into the BSR values on
 * the pattern of or_pattern.  Returns OR_OK or an error code. */
int or_assemble(const or_problem *p, const double *x_old, const double *x_new, double dt,
                double *R, const int32_t *rowptr, const int32_t *colind, double *val);

/* Flux-only residual (faces and fracture-matrix transfer; no accumulation, no
 * wells) over the cell rows: used for conservation pins. */
int or_flux_residual(const or_problem *p, const double *x, double *R);

/* y = alpha*A*x + beta*y for a BSR matrix with bs x bs blocks (beta == 0 ignores y). */
void or_bsr_spmv(int n, int bs, const int32_t *rowptr, const int32_t *colind, const double *val,
                 double alpha, const double *x, double beta, double *y);

/* Dense LU with partial pivoting: solves A x = b in place (A row-major n x n,
 * b overwritten by x).  Returns OR_ERR_SINGULAR_BLOCK for a zero pivot. */
int or_dense_solve(int n, double *A, double *b);

/* Quasi-IMPES decoupling (Section 3.2).  Per cell the decoupled pressure row
 * is c_i . (oil, water, gas rows) with c_i = s_i (1, -w_i), s_i = +-1 chosen so
 * that the decoupled pressure diagonal is positive.  Outputs c (3N) and the
 * pressure block App (values on the BSR pattern, nnzb doubles).
 * mode OR_QI_DIAG: D_ps and D_ss are the pointwise diagonals of the cell's
 *   blocks, w_i = (a_o,Sw / a_w,Sw, a_o,Sg / a_g,Sg);
 * mode OR_QI_BLOCK: D_ss is the cell's 2x2 saturation block, w_i = a_ps a_ss^{-1}. */
enum { OR_QI_DIAG = 0, OR_QI_BLOCK = 1 };
int or_qi_decouple(int n, const int32_t *rowptr, const int32_t *colind, const double *val,
                   int mode, double *c, double *app);

/* ---- CPR preconditioner and FGMRES ---------------------------------- */
enum { OR_F_BJ = 0, OR_F_ILU_NATURAL = 1, OR_F_ILU_RB = 2, OR_F_ILU_TILED = 3 };
/* level-0 smoother: red-black Gauss-Seidel (needs the grid), damped Jacobi,
 * or l1-Jacobi (any graph) */
enum { OR_SMOOTH_GS = 0, OR_SMOOTH_JACOBI = 1, OR_SMOOTH_L1 = 2 };

typedef struct {
    int fpf;              /* 0: two-stage PF, 1: Algorithm CPR-FPF */
    int ftype;            /* OR_F_* */
    int tile_x, tile_y;   /* tiled ILU0 */
    double theta;         /* strength threshold */
    int coarse_max, max_levels;
    int smoother;         /* OR_SMOOTH_* on level 0 */
    int sweeps;           /* pre = post sweeps */
    int use_amg;          /* 0: pressure stage skipped (F only) */
    int qi_mode;          /* OR_QI_DIAG or OR_QI_BLOCK */
    int precision;        /* OR_PREC_*: mixed-precision emulation of the inner stages */
    int csmoother;        /* OR_CSMOOTH_* on levels >= 1 */
    int npr;              /* pressure rows: the first npr block rows (cells); later rows
                             (fixed-rate wells) stay out of A_pp.  0: all rows */
} or_cpr_opts;
enum { OR_CSMOOTH_JACOBI = 0, OR_CSMOOTH_L1 = 1 };

/* Mixed precision (emulated): OR_PREC_FP32 stores the AMG hierarchy and the F
 * stage's factors rounded to FP32 and runs the V-cycle and the F-stage sweeps
 * in float arithmetic; OR_PREC_FP32_BF16 stores the F stage's factors in BF16
 * (round to nearest even from the FP32 value).  Decoupling, restriction,
 * residuals and the final sums stay FP64; values enter the FP32 stages by
 * rounding and leave them exactly.  The tiled / natural / red-black F stages
 * use the diagonal form of block ILU(0) (valid on the 7-point pattern, whose
 * graph has no triangles), storing E^{-1} and the blocks of A. */
enum { OR_PREC_FP64 = 0, OR_PREC_FP32 = 1, OR_PREC_FP32_BF16 = 2 };
/* FP32 -> BF16 (8 significant bits), round to nearest even */
float or_bf16_round(float f);

typedef struct or_cpr or_cpr;

/* Builds decoupling weights, the AMG hierarchy and the F-stage factors.  nx,ny,nz
 * describe the grid (needed for red-black and tiled orderings, and for the
 * level-0 smoother colouring). */
int or_cpr_setup(const or_problem *p, int n, const int32_t *rowptr, const int32_t *colind,
                 const double *val, const or_cpr_opts *o, or_cpr **out);
void or_cpr_free(or_cpr *c);
/* z = M^{-1} v (3N). */
int or_cpr_apply(or_cpr *c, const double *v, double *z);
/* Individual stages for parity tests. */
int or_cpr_restrict(or_cpr *c, const double *v, double *rp);        /* rp_i = c_i . v_i (N) */
int or_cpr_vcycle(or_cpr *c, const double *b, double *x);           /* one V-cycle, level 0 */
int or_cpr_fstage(or_cpr *c, const double *r, double *x);           /* F(r) (3N) */

/* Hierarchy introspection. */
int or_amg_nlevels(or_cpr *c);
/* n, nnz of level l matrix; nnz of P_l (0 for the coarsest); number of colours. */
void or_amg_level_info(or_cpr *c, int l, int *n, int *nnz, int *pnnz, int *ncolors, double *omega);
/* Copies level-l data out (any pointer may be NULL). */
void or_amg_level_get(or_cpr *c, int l, int32_t *rowptr, int32_t *colind, double *val,
                      int32_t *agg, int32_t *color, int32_t *prowptr, int32_t *pcolind, double *pval,
                      int32_t *strong_rowptr, int32_t *strong_colind);
/* MIS-2 members of level l (1 = aggregate root), n bytes. */
void or_amg_level_roots(or_cpr *c, int l, uint8_t *root);
/* Decoupling rows c (3N) and F-stage pivot inverses (N*9, for ILU: inverses of U_ii). */
void or_cpr_get(or_cpr *c, double *cw, double *fpiv_inv);

typedef struct {
    int m, maxit;
    double rtol;
    int orth;             /* 0: modified Gram-Schmidt, 1: classical GS with one re-orthogonalisation */
} or_fgmres_opts;

typedef struct {
    int iterations, restarts, converged;
    double rel_residual;      /* true ||b - A x|| / ||b|| */
    double est_residual;      /* last |g_{j+1}| / ||b|| */
} or_fgmres_stats;

/* Right-preconditioned flexible GMRES(m) on the BSR system (x in: x0, out: x).
 * pc may be NULL (no preconditioner).  hist (optional, maxit+1) receives the
 * estimated relative residual after each iteration. */
int or_fgmres(int n, const int32_t *rowptr, const int32_t *colind, const double *val,
              or_cpr *pc, const double *b, double *x, const or_fgmres_opts *o,
              or_fgmres_stats *st, double *hist);

/* FGMRES returning the Arnoldi quantities of its first cycle (for the
 * Arnoldi-relation pin): Z (m x 3N), V ((m+1) x 3N), H ((m+1) x m, row-major,
 * before rotations).  Runs exactly k <= m steps without restart. */
int or_arnoldi(int n, const int32_t *rowptr, const int32_t *colind, const double *val,
               or_cpr *pc, const double *b, int k, int orth, double *Z, double *V, double *H);

/* The AMG setup rules on a caller-given scalar CSR matrix (for pins):
 * or_amg_only builds the hierarchy alone (l1-Jacobi, no grid) into a handle
 * that the level getters and or_cpr_vcycle accept (keep_singular: a singular
 * coarsest matrix still returns the handle, with OR_ERR_SINGULAR_COARSE); or_amg_strength writes the
 * symmetrised strength flag of every entry; or_amg_aggregate runs phase 1 and
 * phase 2 of the aggregation from caller-chosen roots (root[i] = 1) and
 * returns the number of aggregates. */
int or_amg_only(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double theta,
                int coarse_max, int max_levels, int keep_singular, or_cpr **out);
int or_amg_strength(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double theta,
                    uint8_t *sf);
int or_amg_aggregate(int n, const int32_t *rowptr, const int32_t *colind, const double *val, double theta,
                     const uint8_t *root, int32_t *agg);

/* ---- Exact elimination of the matrix cells (dual porosity) ------------- */
/* For a dual-porosity system (rows: N fracture cells, N matrix cells, nw
 * fixed-rate well rows) the reduced system over the fracture cells and the
 * wells: S_gg = A_ff,gg - A_fm A_mm^-1 A_mf on each fracture row's diagonal,
 * every other block copied; well row 2N+w and well column 2N+w become N+w.
 * or_condense_pattern returns the reduced block count (srp / sci may be NULL)
 * or -1 for a pattern that is not a dual-porosity one; or_condense_values
 * fills sval on that pattern and, per location, A_mm^-1 (minv), A_mf (amf)
 * and W = A_fm A_mm^-1 (wfm), 9 doubles each. */
int or_condense_pattern(int N, int nw, const int32_t *rp, const int32_t *ci, int32_t *srp, int32_t *sci);
int or_condense_values(int N, int nw, const int32_t *rp, const int32_t *ci, const double *val,
                       double *sval, double *minv, double *amf, double *wfm);
/* b' = (b_f - W b_m, b_w) (3(N+nw)) */
void or_condense_rhs(int N, int nw, const double *b, const double *wfm, double *br);
/* x = (x'_f, A_mm^-1 (b_m - A_mf x'_f), x'_w) (3(2N+nw)) */
void or_condense_back(int N, int nw, const double *b, const double *xr, const double *minv, const double *amf,
                      double *x);

/* Restricted additive Schwarz with ILU(0) subdomain solves on a scalar
 * 7-point system (or_ras.c): tiles of tx x ty columns extended by `overlap`
 * columns; coef[s * N + g] in slot order -z, -y, -x, diagonal, +x, +y, +z. */
typedef struct or_ras or_ras;
int or_ras_setup(int nx, int ny, int nz, const double *coef, int tx, int ty, int overlap, or_ras **out);
int or_ras_apply(const or_ras *h, const double *r, double *z);
void or_ras_free(or_ras *h);
int or_ras_tiles(const or_ras *h);
int or_ras_tile_nnz(const or_ras *h, int t);
int or_ras_tile(const or_ras *h, int t, int32_t *cell, uint8_t *own, int32_t *rp, int32_t *ci, double *lu);

#ifdef __cplusplus
}
#endif
#endif
