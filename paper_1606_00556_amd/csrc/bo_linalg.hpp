// Host wrappers of the basic GPU operations (internal).
#pragma once
#include "bo_common.hpp"

namespace bo {

bo_status slot_spmv(const Grid &g, const double *A, double alpha, const double *x, double beta, double *y,
                    hipStream_t s);
// r = v - A (Pi_p dp) (FP64 arithmetic; dp FP64 or FP32, r stored as TO)
template <typename TD, typename TO>
bo_status slot_col0_residual(const Grid &g, const double *A, const double *v, const TD *dp, TO *r, hipStream_t s);
// Sliced layout of a BSR matrix for the solver's SpMV: slices of 64 rows; a
// slice of width K stores, for k < K, the k-th block of each of its rows as 9
// arrays of 64 doubles and one array of 64 column indices (zero blocks on the
// row's own column past the end of a row).  soff[S] = sum of the widths of
// slices < S.  With a grid (G.rows > 0) the slices of cell rows keep the
// stencil blocks at positions 0..6 with implicit columns (see SellGrid).
bo_status sell_build(int n, const int32_t *rp, const int32_t *ci, const double *v, const SellGrid &G,
                     DBuf<int32_t> &soff, DBuf<int32_t> &sci, DBuf<double> &sv, hipStream_t s);
// (yin != NULL: y = alpha A x + beta yin, yin read instead of y)
bo_status sell_spmv(int n, const int32_t *soff, const int32_t *sci, const double *sv, const SellGrid &G,
                    double alpha, const double *x, double beta, double *y, hipStream_t s,
                    const double *yin = nullptr);
bo_status bsr_to_slots(const Grid &g, const int32_t *rp, const int32_t *ci, const double *v, double *slots,
                       hipStream_t s);
// r -= A Pi_p dp in place (column 0 of each block; dp FP64 or FP32), on the
// sliced layout (dp on the block columns below npr) and on the slot layout
template <typename TD>
bo_status sell_col0_update(int n, int npr, const int32_t *soff, const int32_t *sci, const double *sv,
                           const SellGrid &G, const TD *dp, double *r, hipStream_t s);
template <typename TD>
bo_status slot_col0_update(const Grid &g, const double *A, const TD *dp, double *r, hipStream_t s);
bo_status axpby(long long n, double a, const double *x, double b, double *y, hipStream_t s);
bo_status fill(long long n, double v, double *y, hipStream_t s);
// w /= sqrt(*nrm2) on the device (left unchanged when that is <= 1e-300)
bo_status normalize(long long n, const double *nrm2, double *w, hipStream_t s);
constexpr int kMaxVecList = 64;
// A list of device vectors passed to a kernel by value.
struct VecList {
    const double *p[kMaxVecList];
};

// y += sign * sum_q h[q] V[q]; Vhost: host array of nv device pointers, h on the device
bo_status multiaxpy(long long n, const double *const *Vhost, int nv, const double *h, double sign, double *y,
                    hipStream_t s);
bo_status scale_copy(long long n, const double *inv, const double *x, double *y, hipStream_t s);

constexpr int kRedBlocks = 1024;  // fixed reduction grid (determinism)

// Deterministic dot products; results land in device memory.
struct Reducer {
    DBuf<double> partial;
    bo_status init();
    // out[q] = <x, V[q]>, q < nv; Vhost is a host array of device pointers
    bo_status multidot(long long n, const double *x, const double *const *Vhost, int nv, double *out,
                       hipStream_t s);
    bo_status dot(long long n, const double *x, const double *y, double *out, hipStream_t s);
    // one classical Gram-Schmidt pass (see k_cgs_pass); results land in out.
    // reverse: walk the elements from the end (a pass that starts where the
    // previous one ended finds that part of the vectors still in cache)
    bo_status cgs_pass(long long n, double *w, const double *const *Vhost, int nv, const double *h, bool dots,
                       double *out, hipStream_t s, bool reverse = false);
    // delayed re-orthogonalisation (k_dcgs_dots / k_dcgs_update): dots of
    // [V[0..nv-1)] and the pending V[nv-1] with itself and w into out[0..2nv);
    // the update of step j over Vhost[0..j+2) (final basis, pending vector,
    // w) from those dots, beta and r into sc[0..1], |new pending|^2 into norm2
    // (mirror arguments: pinned host memory that also receives the results,
    // written by the kernels themselves)
    bo_status dcgs_dots(long long n, const double *const *Vhost, int nv, const double *w, double *out,
                        hipStream_t s, double *mirror = nullptr);
    bo_status dcgs_update(long long n, const double *const *Vhost, int j, const double *red, double *sc,
                          double *norm2, hipStream_t s, bool reverse, double *sc_mirror = nullptr,
                          double *norm2_mirror = nullptr);
};

}  // namespace bo
