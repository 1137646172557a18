/* Oracle (test infrastructure only): helpers shared by the oracle's own files. */
#ifndef OR_INTERNAL_H
#define OR_INTERNAL_H
#include <stdint.h>

int or_inv3(const double *A, double *Ainv);
void or_mul3(const double *A, const double *B, double *C);
void or_mv3(const double *A, const double *x, double *y);
/* smallest |pivot| of partially pivoted LU over the largest |a_ij| */
double or_dense_min_pivot_ratio(int n, const double *A);

typedef struct {
    int n, m, nnz;              /* rows, columns, entries */
    int32_t *rp, *ci;
    double *v;
} or_csr;

void or_csr_free(or_csr *a);
#endif
