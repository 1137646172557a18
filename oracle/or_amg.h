/* Oracle (test infrastructure only): aggregation AMG hierarchy. */
#ifndef OR_AMG_H
#define OR_AMG_H
#include <stdint.h>
#include "or_internal.h"

#define OR_MAXLEV 16
#define OR_DENSE_MAX 2000

typedef struct {
    int nlev;
    or_csr A[OR_MAXLEV];        /* level operators */
    or_csr P[OR_MAXLEV];        /* prolongation level l+1 -> l */
    or_csr R[OR_MAXLEV];        /* restriction P^T */
    int32_t *agg[OR_MAXLEV];    /* aggregate of each node (-1: unaggregated) */
    uint8_t *sf[OR_MAXLEV];     /* strength flag per entry of A[l] */
    uint8_t *root[OR_MAXLEV];   /* MIS-2 members (aggregate roots) */
    int32_t *color[OR_MAXLEV];  /* red-black colours, level 0 only */
    int ncolor[OR_MAXLEV];
    double omega[OR_MAXLEV];
    double *dense;              /* coarsest matrix, row-major, when solved directly */
    int coarse_direct;
    int smoother, sweeps;
    int csmoother;              /* levels >= 1: OR_CSMOOTH_* */
    double *dl1[OR_MAXLEV];     /* l1 row norms sum_j |a_ij| of each level */
    float *dl132[OR_MAXLEV];    /* their FP32 roundings (mixed form) */
    /* mixed-precision emulation: FP32 copies of the level operators, P, R and
     * the coarsest inverse (NULL until or_amg_make_f32) */
    float *A32[OR_MAXLEV], *P32[OR_MAXLEV], *R32[OR_MAXLEV];
    float *cinv32;
} or_amg;

int or_amg_setup(or_amg *h, const or_csr *A0, int nx, int ny, int nz, double theta,
                 int coarse_max, int max_levels, int smoother, int sweeps, int csmoother);
void or_amg_vcycle(const or_amg *h, const double *b, double *x);
void or_amg_free(or_amg *h);
int or_amg_make_f32(or_amg *h);
void or_amg_strength_flags(const or_csr *A, double theta, uint8_t *sf);
int or_amg_aggregate_roots(const or_csr *A, double theta, const uint8_t *root, int32_t *agg);
void or_amg_vcycle_f32(const or_amg *h, const float *b, float *x);
#endif
