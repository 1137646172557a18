// Quasi-IMPES decoupling and the aggregation AMG on the decoupled pressure
// block (the P stage of CPR, Section 3.2; the paper uses BoomerAMG here).
//
// Decoupling: per cell c_i = s (1, -w_i) with w_i = a_ps a_ss^{-1} from the
// cell's diagonal block (or the pointwise-diagonal form), s = +-1 keeping the
// decoupled pressure diagonal positive; A_pp(i,j) = c_i . A_ij[:,0].
//
// Setup, per level, every step a pure function of the previous one so the
// hierarchy does not depend on thread timing:
//   strength      |a_ij|^2 >= theta^2 |a_ii a_jj| in either direction
//   MIS-2         synchronous rounds with hashed priorities (fmix32 of the
//                 index, salted by the level; ties broken by the index)
//   aggregation   roots numbered in index order; strong neighbours of a root
//                 join it; the rest join their strongest assigned neighbour
//   prolongator   Jacobi-smoothed tentative prolongator, omega = (4/3)/rho
//   Galerkin      A_c = P^T (A P) by a row-wise product: one wavefront per
//                 output row, an LDS hash for the column set, then per output
//                 entry a sum over the left row in ascending order
//   coarsest      dense inverse by Gauss-Jordan with partial pivoting
// Cycle: V(s,s) from a zero guess; level 0 red-black Gauss-Seidel on the
// grid (or damped Jacobi), coarser levels damped Jacobi (omega 2/3), coarsest
// level by the dense inverse.
#include <cstring>
#include <functional>
#include "bo_cpr.hpp"

namespace bo {
namespace {

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
    h ^= h >> 16; h *= 0x85ebca6bu;
    h ^= h >> 13; h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

__device__ __forceinline__ uint64_t prio(int i, int level) {
    uint32_t h = fmix32((uint32_t)i ^ (0x9E3779B9u * (uint32_t)(level + 1)));
    return ((((uint64_t)h) << 32) | (uint32_t)i) + 1ull;
}

// ---- decoupling ---------------------------------------------------------------
__global__ void k_qi_decouple(int nx, int ny, int nz, const double *__restrict__ A, int mode,
                              double *__restrict__ cw, double *__restrict__ app,
                              int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (i >= n) return;
    size_t N = (size_t)n;
    const double *B = A + (size_t)S_D * 9 * N + i;
    double a = B[4 * N], b = B[5 * N], c = B[7 * N], d = B[8 * N];
    double p0 = B[1 * N], p1 = B[2 * N];
    double w0, w1;
    if (mode == BO_QI_DIAG) {
        if (a == 0.0 || d == 0.0) { *bad = 1; w0 = w1 = 0.0; }
        else { w0 = p0 / a; w1 = p1 / d; }
    } else {
        double det = a * d - b * c;
        if (det == 0.0 || !isfinite(det)) { *bad = 1; w0 = w1 = 0.0; }
        else {
            w0 = (p0 * d - p1 * c) / det;
            w1 = (p1 * a - p0 * b) / det;
        }
    }
    double dpp = B[0] - w0 * B[3 * N] - w1 * B[6 * N];
    double sg = dpp < 0.0 ? -1.0 : 1.0;
    double c0 = sg, c1 = -sg * w0, c2 = -sg * w1;
    cw[3 * (size_t)i] = c0;
    cw[3 * (size_t)i + 1] = c1;
    cw[3 * (size_t)i + 2] = c2;
    for (int s = 0; s < NSLOT; s++) {
        const double *As = A + (size_t)s * 9 * N + i;
        app[(size_t)s * N + i] = c0 * As[0] + c1 * As[3 * N] + c2 * As[6 * N];
    }
}

// General BSR form (no grid): the weights c_i of every block row from its
// diagonal block (a fixed-rate well row has zero saturation couplings, so its
// weights are (+-1, 0, 0), i.e. no decoupling)
__global__ void k_qi_weights_bsr(int nrows, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ val, int mode, double *__restrict__ cw,
                                 int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nrows) return;
    int e = rp[i];
    while (e < rp[i + 1] && ci[e] != i) e++;
    if (e == rp[i + 1]) { *bad = 1; cw[3 * (size_t)i] = 1.0; cw[3 * (size_t)i + 1] = cw[3 * (size_t)i + 2] = 0.0; return; }
    const double *B = val + 9 * (size_t)e;
    double a = B[4], b = B[5], c = B[7], d = B[8];
    double p0 = B[1], p1 = B[2];
    double w0, w1;
    if (mode == BO_QI_DIAG) {
        if (a == 0.0 || d == 0.0) { *bad = 1; w0 = w1 = 0.0; }
        else { w0 = p0 / a; w1 = p1 / d; }
    } else {
        double det = a * d - b * c;
        if (det == 0.0 || !isfinite(det)) { *bad = 1; w0 = w1 = 0.0; }
        else {
            w0 = (p0 * d - p1 * c) / det;
            w1 = (p1 * a - p0 * b) / det;
        }
    }
    double dpp = B[0] - w0 * B[3] - w1 * B[6];
    double sg = dpp < 0.0 ? -1.0 : 1.0;
    cw[3 * (size_t)i] = sg;
    cw[3 * (size_t)i + 1] = -sg * w0;
    cw[3 * (size_t)i + 2] = -sg * w1;
}

// A_pp of the general form: the first npr rows and columns of c_i . A_ij[:, 0]
__global__ void k_app_counts(int npr, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             int32_t *__restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npr) return;
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; e++) c += ci[e] < npr;
    cnt[i] = c;
}

__global__ void k_app_fill(int npr, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ val, const double *__restrict__ cw,
                           const int32_t *__restrict__ prp, int32_t *__restrict__ pci, double *__restrict__ pv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= npr) return;
    double c0 = cw[3 * (size_t)i], c1 = cw[3 * (size_t)i + 1], c2 = cw[3 * (size_t)i + 2];
    int o = prp[i];
    // batches of kB blocks, all loads of a batch issued together
    constexpr int kB = 8;
    const int b0 = rp[i], b1 = rp[i + 1];
    for (int e0 = b0; e0 < b1; e0 += kB) {
        int cc[kB];
        double a0[kB], a3[kB], a6[kB];
#pragma unroll
        for (int k = 0; k < kB; k++) {
            const int e = min(e0 + k, b1 - 1);
            const double *A = val + 9 * (size_t)e;
            cc[k] = ci[e];
            a0[k] = A[0]; a3[k] = A[3]; a6[k] = A[6];
        }
#pragma unroll
        for (int k = 0; k < kB; k++)
            if (e0 + k < b1 && cc[k] < npr) {
                pci[o] = cc[k];
                pv[o] = c0 * a0[k] + c1 * a3[k] + c2 * a6[k];
                o++;
            }
    }
}

// level-0 CSR from the slot form (pattern = the 7-point stencil)
__global__ void k_slots_to_csr(int nx, int ny, int nz, const double *__restrict__ app,
                               const int32_t *__restrict__ rp, int32_t *__restrict__ ci, double *__restrict__ v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (i >= n) return;
    int e = rp[i];
    for (int s = 0; s < NSLOT; s++) {
        int j = nbr_of(i, s, nx, ny, nz);
        if (j < 0) continue;
        ci[e] = j;
        v[e] = app[(size_t)s * n + i];
        e++;
    }
}

__global__ void k_stencil_counts(int nx, int ny, int nz, int32_t *cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (i >= n) return;
    int c = 0;
    for (int s = 0; s < NSLOT; s++) c += nbr_of(i, s, nx, ny, nz) >= 0;
    cnt[i] = c;
}

// restriction of a 3N residual: rp_i = c_i . v_i
// r_p = c_i . v_i in FP64, stored as T (FP32 at the mixed form's boundary)
template <typename T>
__global__ void k_qi_restrict(long long n, const double *__restrict__ cw, const double *__restrict__ v,
                              T *__restrict__ rp) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rp[i] = (T)(cw[3 * i] * v[3 * i] + cw[3 * i + 1] * v[3 * i + 1] + cw[3 * i + 2] * v[3 * i + 2]);
}

// ---- CSR utilities ---------------------------------------------------------------
__device__ __forceinline__ int find_col(const int32_t *ci, int lo, int hi, int col) {
    // binary search in ci[lo, hi) (ascending); -1 if absent
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        int c = ci[mid];
        if (c == col) return mid;
        if (c < col) lo = mid + 1; else hi = mid;
    }
    return -1;
}

// diagonal position and l1 row norm sum_j |a_ij| (ascending columns) of each row
__global__ void k_diag(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const double *__restrict__ v, int32_t *__restrict__ dpos, double *__restrict__ dl1,
                       int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = find_col(ci, rp[i], rp[i + 1], i);
    dpos[i] = p;
    double d = p >= 0 ? v[p] : 0.0;
    if (d == 0.0 || !isfinite(d)) *bad = 1;
    // l1 row sum in entry order, the loads of kB entries issued together
    constexpr int kB = 8;
    const int b = rp[i], e1 = rp[i + 1];
    double s = 0.0;
    for (int e0 = b; e0 < e1; e0 += kB) {
        double vv[kB];
#pragma unroll
        for (int k = 0; k < kB; k++) vv[k] = v[min(e0 + k, e1 - 1)];
#pragma unroll
        for (int k = 0; k < kB; k++)
            if (e0 + k < e1) s = s + fabs(vv[k]);
    }
    dl1[i] = s;
}

// G lanes per row, each entry on its own
template <int G>
__global__ void k_strength(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, const int32_t *__restrict__ dpos, double t2,
                           uint8_t *__restrict__ sf) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    int i = gid / G, sub = gid % G;
    if (i >= n) return;
    double aii = dpos[i] >= 0 ? v[dpos[i]] : 0.0;
    for (int e = rp[i] + sub; e < rp[i + 1]; e += G) {
        int j = ci[e];
        if (j == i) { sf[e] = 0; continue; }
        double ajj = dpos[j] >= 0 ? v[dpos[j]] : 0.0;
        int q = find_col(ci, rp[j], rp[j + 1], i);
        double aij = v[e], aji = q >= 0 ? v[q] : 0.0;
        double thr = t2 * fabs(aii * ajj);
        sf[e] = (aij * aij >= thr) || (aji * aji >= thr);
    }
}

// level-0 strength straight from the stencil layout: the transposed entry of
// slot s of row i is slot 6-s of row j
__global__ void k_strength_slots(int nx, int ny, int nz, const double *__restrict__ app,
                                 const int32_t *__restrict__ rp, double t2, uint8_t *__restrict__ sf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (i >= n) return;
    size_t N = (size_t)n;
    double aii = app[(size_t)S_D * N + i];
    int e = rp[i];
    for (int s = 0; s < NSLOT; s++) {
        int j = nbr_of(i, s, nx, ny, nz);
        if (j < 0) continue;
        if (s == S_D) { sf[e++] = 0; continue; }
        double ajj = app[(size_t)S_D * N + j];
        double aij = app[(size_t)s * N + i], aji = app[(size_t)(NSLOT - 1 - s) * N + j];
        double thr = t2 * fabs(aii * ajj);
        sf[e++] = (aij * aij >= thr) || (aji * aji >= thr);
    }
}

enum { UND = 0, IN = 1, OUT = 2, ISO = 3 };

// (also clears the change words of the level's MIS rounds, kMisWords of them)
constexpr int kMisWords = 64;
__global__ void k_mis_init(int n, const int32_t *__restrict__ rp, const uint8_t *__restrict__ sf,
                           uint8_t *__restrict__ state, int32_t *__restrict__ words) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < kMisWords) words[i] = 0;
    if (i >= n) return;
    int deg = 0;
    constexpr int kB = 8;
    const int b0 = rp[i], b1 = rp[i + 1];
    for (int e0 = b0; e0 < b1; e0 += kB) {
        uint8_t f[kB];
#pragma unroll
        for (int k = 0; k < kB; k++) f[k] = sf[min(e0 + k, b1 - 1)];
#pragma unroll
        for (int k = 0; k < kB; k++)
            if (e0 + k < b1) deg += f[k];
    }
    state[i] = deg ? UND : ISO;
}

// The MIS-2 round kernels take G lanes per row (G a power of two dividing
// 64): the lanes stride the row's entries and combine their maxima or flags
// with cross-lane shuffles.  Maxima and ORs do not depend on the order, so
// every G gives the same round.
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int off, int width) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = (uint32_t)__shfl_xor((int)lo, off, width);
    hi = (uint32_t)__shfl_xor((int)hi, off, width);
    return ((uint64_t)hi << 32) | lo;
}
template <int G>
__device__ __forceinline__ uint64_t group_max(uint64_t m) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) {
        uint64_t o = shfl_xor_u64(m, off, G);
        if (o > m) m = o;
    }
    return m;
}
template <int G>
__device__ __forceinline__ int group_or(int d) {
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) d |= __shfl_xor(d, off, G);
    return d;
}

template <int G>
__global__ void k_mis_m1(int n, int level, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const uint8_t *__restrict__ sf, const uint8_t *__restrict__ state,
                         uint64_t *__restrict__ m1) {
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i = (int)(gid / G), sub = (int)(gid % G);
    if (i >= n) return;  // whole groups leave together
    uint64_t m = sub == 0 && state[i] == UND ? prio(i, level) : 0ull;
    for (int e = rp[i] + sub; e < rp[i + 1]; e += G)
        if (sf[e] && state[ci[e]] == UND) {
            uint64_t q = prio(ci[e], level);
            if (q > m) m = q;
        }
    m = group_max<G>(m);
    if (sub == 0) m1[i] = m;
}

template <int G>
__global__ void k_mis_m2(int n, int level, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const uint8_t *__restrict__ sf, const uint8_t *__restrict__ state,
                         const uint64_t *__restrict__ m1, uint8_t *__restrict__ nw) {
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i = (int)(gid / G), sub = (int)(gid % G);
    if (i >= n) return;
    uint64_t m = sub == 0 ? m1[i] : 0ull;
    for (int e = rp[i] + sub; e < rp[i + 1]; e += G)
        if (sf[e] && m1[ci[e]] > m) m = m1[ci[e]];
    m = group_max<G>(m);
    if (sub == 0) nw[i] = state[i] == UND && m == prio(i, level);
}

template <int G>
__global__ void k_mis_spread(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const uint8_t *__restrict__ sf, const uint8_t *__restrict__ in,
                             uint8_t *__restrict__ out) {
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i = (int)(gid / G), sub = (int)(gid % G);
    if (i >= n) return;
    int d = sub == 0 ? in[i] : 0;
    for (int e = rp[i] + sub; e < rp[i + 1]; e += G)
        if (sf[e]) d |= in[ci[e]];
    d = group_or<G>(d);
    if (sub == 0) out[i] = (uint8_t)d;
}

template <int G>
__global__ void k_mis_update(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const uint8_t *__restrict__ sf, const uint8_t *__restrict__ nw,
                             const uint8_t *__restrict__ d1, uint8_t *__restrict__ state,
                             int32_t *__restrict__ any) {
    long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    int i = (int)(gid / G), sub = (int)(gid % G);
    if (i >= n) return;
    int d = sub == 0 ? d1[i] : 0;
    for (int e = rp[i] + sub; e < rp[i + 1]; e += G)
        if (sf[e]) d |= d1[ci[e]];
    d = group_or<G>(d);
    if (sub != 0) return;
    uint8_t st = state[i];
    if (nw[i]) st = IN;
    else if (st == UND && d) st = OUT;
    state[i] = st;
    if (st == UND) *any = 1;
}

__global__ void k_is_root(int n, const uint8_t *__restrict__ state, int32_t *__restrict__ cnt,
                          uint8_t *__restrict__ root) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cnt[i] = state[i] == IN;
    root[i] = state[i] == IN;
}

// phase 1: a root and its strong neighbours form an aggregate
__global__ void k_agg1(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const uint8_t *__restrict__ sf, const uint8_t *__restrict__ state,
                       const int32_t *__restrict__ id, int32_t *__restrict__ a1) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = -1;
    if (state[i] == IN) {
        a = id[i];
    } else {
        // entry order (the last strong root neighbour wins), kB entries'
        // loads at a time
        constexpr int kB = 8;
        const int b = rp[i], e1 = rp[i + 1];
        for (int e0 = b; e0 < e1; e0 += kB) {
            int cc[kB], ss[kB], st[kB], idv[kB];
#pragma unroll
            for (int k = 0; k < kB; k++) {
                const int e = min(e0 + k, e1 - 1);
                cc[k] = ci[e];
                ss[k] = sf[e];
            }
#pragma unroll
            for (int k = 0; k < kB; k++) { st[k] = state[cc[k]]; idv[k] = id[cc[k]]; }
#pragma unroll
            for (int k = 0; k < kB; k++)
                if (e0 + k < e1 && ss[k] && st[k] == IN) a = idv[k];
        }
    }
    a1[i] = a;
}

// phase 2: join the strongest assigned strong neighbour (ties: smaller id)
__global__ void k_agg2(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const double *__restrict__ v, const uint8_t *__restrict__ sf,
                       const uint8_t *__restrict__ state, const int32_t *__restrict__ a1,
                       int32_t *__restrict__ agg, int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = a1[i];
    if (a < 0 && state[i] != ISO) {
        int best = -1;
        double bv = -1.0;
        constexpr int kB = 8;
        const int b = rp[i], e1 = rp[i + 1];
        for (int e0 = b; e0 < e1; e0 += kB) {
            int ss[kB], aj[kB];
            double vv[kB];
#pragma unroll
            for (int k = 0; k < kB; k++) {
                const int e = min(e0 + k, e1 - 1);
                ss[k] = sf[e];
                aj[k] = a1[ci[e]];
                vv[k] = v[e];
            }
#pragma unroll
            for (int k = 0; k < kB; k++) {
                if (e0 + k >= e1 || !ss[k] || aj[k] < 0) continue;
                double x = fabs(vv[k]);
                if (x > bv || (x == bv && aj[k] < best)) { bv = x; best = aj[k]; }
            }
        }
        a = best;
        if (a < 0) *bad = 1;
    }
    agg[i] = a;
}

// filtered diagonal and the Gershgorin ratio of D_F^{-1} A_F (max via the
// order-preserving bit pattern of non-negative doubles)
// Reductions of one value over a launch (a maximum or a count) go through
// kRedSlots words: one atomic per workgroup, on word blockIdx % kRedSlots.
// Atomics on one word from every wavefront of a large launch serialise (about
// 12 ns each on the device), which made such a reduction cost more than the
// kernel's own work; the reader combines the words.
constexpr int kRedSlots = 64;
__device__ __forceinline__ void block_max_to_slots(uint64_t v, unsigned long long *slots) {
    __shared__ uint64_t wm[kBlock / 64];
    v = group_max<64>(v);
    if (threadIdx.x % 64 == 0) wm[threadIdx.x / 64] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint64_t m = wm[0];
        for (int w = 1; w < (int)(blockDim.x / 64); w++) m = wm[w] > m ? wm[w] : m;
        if (m > 0) atomicMax(&slots[blockIdx.x % kRedSlots], (unsigned long long)m);
    }
}

__global__ void __launch_bounds__(kBlock) k_filter(int n, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                   const int32_t *__restrict__ dpos, const uint8_t *__restrict__ sf,
                                                   double *__restrict__ aF, unsigned long long *__restrict__ rho_bits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t bits = 0;
    if (i < n) {
        // the row in batches of kB entries: every load of a batch is issued
        // before the sums, which still run in entry order; the row's values
        // stay in registers for the second sum only as one batch, so it
        // reloads them (cache hits)
        constexpr int kB = 8;
        const int b = rp[i], e1 = rp[i + 1];
        double aii = v[dpos[i]];
        double d = aii;
        for (int e0 = b; e0 < e1; e0 += kB) {
            int cc[kB], ss[kB];
            double vv[kB];
#pragma unroll
            for (int k = 0; k < kB; k++) {
                const int e = min(e0 + k, e1 - 1);  // rows are never empty (diagonal)
                cc[k] = ci[e]; ss[k] = sf[e]; vv[k] = v[e];
            }
#pragma unroll
            for (int k = 0; k < kB; k++)
                if (e0 + k < e1 && cc[k] != i && !ss[k]) d = d + vv[k];
        }
        if (d == 0.0) d = aii;
        aF[i] = d;
        double rs = 0.0;
        for (int e0 = b; e0 < e1; e0 += kB) {
            int cc[kB], ss[kB];
            double vv[kB];
#pragma unroll
            for (int k = 0; k < kB; k++) {
                const int e = min(e0 + k, e1 - 1);
                cc[k] = ci[e]; ss[k] = sf[e]; vv[k] = v[e];
            }
#pragma unroll
            for (int k = 0; k < kB; k++) {
                if (e0 + k >= e1) continue;
                if (cc[k] == i) rs = rs + fabs(d);
                else if (ss[k]) rs = rs + fabs(vv[k]);
            }
        }
        double ratio = rs / fabs(d);
        bits = (uint64_t)__double_as_longlong(ratio);
    }
    // the ratios are >= 0, so their bit patterns order as the values
    block_max_to_slots(bits, rho_bits);
}

__device__ __forceinline__ bool p_takes(int e, int i, const int32_t *ci, const uint8_t *sf, const int32_t *agg) {
    int j = ci[e];
    return (j == i || sf[e]) && agg[j] >= 0;
}

// Row data of the prolongator: the aggregate J of each entry that takes part
// ({i} and the strong neighbours, aggregated) or -1, and its filtered value.
// Register fast path for rows of up to KP entries (8 on levels of at most 8
// entries a row on average, else 16: the fully unrolled first-appearance
// and rank loops grow with the cube of KP); longer rows go to k_p_long,
// which forms the same sums in the same order.
template <int KP>
__global__ void k_p_count(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const uint8_t *__restrict__ sf, const int32_t *__restrict__ agg,
                          int32_t *__restrict__ cnt, int32_t *__restrict__ plong) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int len = i < n ? rp[i + 1] - rp[i] : 0;
    // rows longer than KP go to plong[1..] (count in plong[0]) for k_p_long /
    // k_p_vlong: one atomic per wavefront, each lane at its rank among them
    const bool lng = len > KP;
    const uint64_t m = __ballot(lng);
    if (m) {
        const int lane = threadIdx.x % 64;
        int base = 0;
        if (lane == __ffsll((unsigned long long)m) - 1) base = atomicAdd(plong, __popcll(m));
        base = __shfl(base, __ffsll((unsigned long long)m) - 1, 64);
        if (lng) plong[1 + base + __popcll(m & ((1ull << lane) - 1))] = i;
    }
    if (i >= n || lng) return;
    int c = 0;
    {
        int J[KP];
#pragma unroll
        for (int q = 0; q < KP; q++) {
            J[q] = -1;
            if (q < len) {
                int e = rp[i] + q;
                if (p_takes(e, i, ci, sf, agg)) J[q] = agg[ci[e]];
            }
        }
#pragma unroll
        for (int q = 0; q < KP; q++) {
            bool first = J[q] >= 0;
#pragma unroll
            for (int u = 0; u < q; u++) first = first && J[u] != J[q];
            c += first;
        }
    }
    cnt[i] = c;
}

// P row i: for each distinct aggregate J among {i} and its strong neighbours,
// (agg(i)==J) - omega/aF_ii * sum_{agg(j)=J} aF_ij (sums in ascending j),
// stored in ascending J.
template <int KP>
__global__ void k_p_fill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ v, const uint8_t *__restrict__ sf,
                         const int32_t *__restrict__ agg, const double *__restrict__ aF,
                         const double *__restrict__ omega, const int32_t *__restrict__ prp,
                         int32_t *__restrict__ pci, double *__restrict__ pv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = omega[0] / aF[i];
    int len = rp[i + 1] - rp[i];
    int ai = agg[i];
    if (len > KP) return;  // long rows: k_p_long
    {
        int J[KP];
        double a[KP];
#pragma unroll
        for (int q = 0; q < KP; q++) {
            J[q] = -1;
            a[q] = 0.0;
            if (q < len) {
                int e = rp[i] + q;
                if (p_takes(e, i, ci, sf, agg)) {
                    J[q] = agg[ci[e]];
                    a[q] = ci[e] == i ? aF[i] : v[e];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < KP; q++) {
            bool first = J[q] >= 0;
#pragma unroll
            for (int u = 0; u < q; u++) first = first && J[u] != J[q];
            if (!first) continue;
            double sum = 0.0;
            int rank = 0;
#pragma unroll
            for (int u = 0; u < KP; u++) {
                if (u >= q && J[u] == J[q]) sum = sum + a[u];
                // distinct aggregates below J[q]: count first appearances
                bool fu = J[u] >= 0 && J[u] < J[q];
#pragma unroll
                for (int w = 0; w < u; w++) fu = fu && J[w] != J[u];
                rank += fu;
            }
            pci[prp[i] + rank] = J[q];
            pv[prp[i] + rank] = (ai == J[q] ? 1.0 : 0.0) - d * sum;
        }
    }
}

// Long rows of the prolongator (more than KP entries): one wavefront per row.
// The row's (aggregate, filtered value) pairs are staged in LDS; an entry is
// the first appearance of its aggregate if no earlier entry has it; the
// entry's lane then sums the aggregate's values in ascending order and writes
// the result at the aggregate's rank among the row's distinct aggregates.
constexpr int KW = 512;
constexpr int kPWaves = 4;

__global__ void __launch_bounds__(64 * kPWaves) k_p_long(int n, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci, const double *__restrict__ v,
                                                          const uint8_t *__restrict__ sf,
                                                          const int32_t *__restrict__ agg,
                                                          const double *__restrict__ aF, const double *__restrict__ omega,
                                                          const int32_t *__restrict__ prp, int32_t *__restrict__ pci,
                                                          double *__restrict__ pv, int32_t *__restrict__ cnt,
                                                          int32_t *__restrict__ bad,
                                                          const int32_t *__restrict__ plong) {
    __shared__ int J[kPWaves][KW];
    __shared__ double A[kPWaves][KW];
    __shared__ uint8_t first[kPWaves][KW];
    int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    // the rows k_p_count listed, a wavefront each, over a fixed grid
    const int nl = plong[0];
    for (int idx = blockIdx.x * kPWaves + wave; idx < nl; idx += gridDim.x * kPWaves) {
    const int i = plong[1 + idx];
    int b = rp[i], len = rp[i + 1] - b;
    if (len > KW) continue;  // handled by k_p_vlong
    // the previous row's LDS reads are done before this row's writes
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    for (int q = lane; q < len; q += 64) {
        int e = b + q;
        bool take = p_takes(e, i, ci, sf, agg);
        J[wave][q] = take ? agg[ci[e]] : -1;
        A[wave][q] = take ? (ci[e] == i ? aF[i] : v[e]) : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    int mycount = 0;
    for (int q = lane; q < len; q += 64) {
        int Jq = J[wave][q];
        bool f = Jq >= 0;
        for (int u = 0; u < q && f; u++) f = J[wave][u] != Jq;
        first[wave][q] = f;
        mycount += f;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    if (cnt) {
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mycount += __shfl_xor(mycount, off, 64);
        if (lane == 0) cnt[i] = mycount;
        continue;
    }
    double d = omega[0] / aF[i];
    int ai = agg[i];
    for (int q = lane; q < len; q += 64) {
        if (!first[wave][q]) continue;
        int Jq = J[wave][q];
        double sum = 0.0;
        int rank = 0;
        for (int u = 0; u < len; u++) {
            int Ju = J[wave][u];
            if (u >= q && Ju == Jq) sum = sum + A[wave][u];
            rank += first[wave][u] && Ju < Jq;
        }
        pci[prp[i] + rank] = Jq;
        pv[prp[i] + rank] = (ai == Jq ? 1.0 : 0.0) - d * sum;
    }
    }
}

// The same for the rare rows longer than the LDS staging (a well row and its
// aggregates on coarse levels): one wavefront per row, the row's aggregate
// ids and values re-read from global memory, quadratic in the row length.
__global__ void __launch_bounds__(64 * kPWaves) k_p_vlong(int n, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const double *__restrict__ v,
                                                           const uint8_t *__restrict__ sf,
                                                           const int32_t *__restrict__ agg,
                                                           const double *__restrict__ aF, const double *__restrict__ omega,
                                                           const int32_t *__restrict__ prp, int32_t *__restrict__ pci,
                                                           double *__restrict__ pv, int32_t *__restrict__ cnt,
                                                           const int32_t *__restrict__ plong) {
    int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int nl = plong[0];
    for (int idx = blockIdx.x * kPWaves + wave; idx < nl; idx += gridDim.x * kPWaves) {
    const int i = plong[1 + idx];
    int b = rp[i], len = rp[i + 1] - b;
    if (len <= KW) continue;
    auto jof = [&](int q) -> int { int e = b + q; return p_takes(e, i, ci, sf, agg) ? agg[ci[e]] : -1; };
    auto aof = [&](int q) -> double {
        int e = b + q;
        return p_takes(e, i, ci, sf, agg) ? (ci[e] == i ? aF[i] : v[e]) : 0.0;
    };
    auto is_first = [&](int q, int Jq) -> bool {
        if (Jq < 0) return false;
        for (int u = 0; u < q; u++)
            if (jof(u) == Jq) return false;
        return true;
    };
    if (cnt) {
        int mycount = 0;
        for (int q = lane; q < len; q += 64) mycount += is_first(q, jof(q));
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) mycount += __shfl_xor(mycount, off, 64);
        if (lane == 0) cnt[i] = mycount;
        continue;
    }
    double d = omega[0] / aF[i];
    int ai = agg[i];
    for (int q = lane; q < len; q += 64) {
        int Jq = jof(q);
        if (!is_first(q, Jq)) continue;
        double sum = 0.0;
        int rank = 0;
        for (int u = 0; u < len; u++) {
            int Ju = jof(u);
            if (u >= q && Ju == Jq) sum = sum + aof(u);
            rank += Ju >= 0 && Ju < Jq && is_first(u, Ju);
        }
        pci[prp[i] + rank] = Jq;
        pv[prp[i] + rank] = (ai == Jq ? 1.0 : 0.0) - d * sum;
    }
    }
}

// transpose helpers
__global__ void k_col_counts(int nnz, const int32_t *__restrict__ ci, int32_t *__restrict__ cnt) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e < nnz) atomicAdd(&cnt[ci[e]], 1);
}

__global__ void k_transpose_fill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ v, const int32_t *__restrict__ trp,
                                 int32_t *__restrict__ fillpos, int32_t *__restrict__ tci, double *__restrict__ tv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
        int J = ci[e];
        int p = trp[J] + atomicAdd(&fillpos[J], 1);
        tci[p] = i;
        tv[p] = v[e];
    }
}

// sorts every row by column: one wavefront per row; rows of up to 64 entries
// are ranked across lanes (columns within a row are distinct)
__global__ void __launch_bounds__(kBlock) k_sort_rows(int n, const int32_t *__restrict__ rp,
                                                      int32_t *__restrict__ ci, double *__restrict__ v) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    int row = gid / 64, lane = gid % 64;
    if (row >= n) return;
    int b = rp[row], len = rp[row + 1] - b;
    if (len <= 64) {
        int c = lane < len ? ci[b + lane] : 0x7fffffff;
        double x = lane < len ? v[b + lane] : 0.0;
        int rank = 0;
        for (int u = 0; u < 64; u++) {
            int cu = __shfl(c, u, 64);
            rank += cu < c;
        }
        __builtin_amdgcn_wave_barrier();
        if (lane < len) { ci[b + rank] = c; v[b + rank] = x; }
        return;
    }
    if (lane != 0) return;
    for (int a = b + 1; a < b + len; a++) {
        int c = ci[a];
        double x = v[a];
        int q = a - 1;
        while (q >= b && ci[q] > c) { ci[q + 1] = ci[q]; v[q + 1] = v[q]; q--; }
        ci[q + 1] = c;
        v[q + 1] = x;
    }
}

// ---- row-wise sparse product C = A B ----------------------------------------------
// G lanes own one output row and an LDS hash of H slots (keys and values).
// The row of A is walked in ascending order; for one entry a_ik the lanes
// take the entries of row k of B in parallel.  Those have distinct columns,
// so no two lanes touch one slot at the same time, and each output value is
// accumulated in ascending k exactly as in a row-by-row Gustavson product.
// The distinct columns are then compacted, ranked (sorted) and written.

// products of each row (sum of the B row lengths it touches) and seven
// reductions over the rows, kRedSlots words each (one atomic per workgroup):
// [0] the largest product count, [1] rows above kLongProducts, [2] rows above
// kVeryLongProducts, [3] the largest count at or below kLongProducts, [4] the
// largest count at or below kVeryLongProducts, [5] rows above
// kShortProducts, [6] the largest count at or below kShortProducts, [7] rows
// above kMidProducts, [8] the largest count at or below kMidProducts
constexpr int kShortProducts = 32;
constexpr int kLongProducts = 128;
constexpr int kMidProducts = 256;
constexpr int kVeryLongProducts = 512;
constexpr int kBoundWords = 9;
__global__ void __launch_bounds__(kBlock) k_spgemm_bound(int n, const int32_t *__restrict__ arp,
                                                         const int32_t *__restrict__ aci,
                                                         const int32_t *__restrict__ brp, int32_t *__restrict__ prod,
                                                         int32_t *__restrict__ stat) {
    __shared__ int wred[kBoundWords][kBlock / 64];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int c = 0;
    if (i < n) {
        // batches of kB entries, all loads of a batch issued together
        constexpr int kB = 8;
        const int a0 = arp[i], a1 = arp[i + 1];
        for (int e0 = a0; e0 < a1; e0 += kB) {
            int kk[kB];
#pragma unroll
            for (int k = 0; k < kB; k++) kk[k] = aci[min(e0 + k, a1 - 1)];
            int lo[kB], hi[kB];
#pragma unroll
            for (int k = 0; k < kB; k++) { lo[k] = brp[kk[k]]; hi[k] = brp[kk[k] + 1]; }
#pragma unroll
            for (int k = 0; k < kB; k++)
                if (e0 + k < a1) c += hi[k] - lo[k];
        }
        prod[i] = c;
    }
    int r[kBoundWords] = {c, c > kLongProducts ? 1 : 0, c > kVeryLongProducts ? 1 : 0,
                          c <= kLongProducts ? c : 0, c <= kVeryLongProducts ? c : 0,
                          c > kShortProducts ? 1 : 0, c <= kShortProducts ? c : 0,
                          c > kMidProducts ? 1 : 0, c <= kMidProducts ? c : 0};
    for (int off = 32; off > 0; off >>= 1) {
        r[0] = max(r[0], __shfl_xor(r[0], off, 64));
        r[1] += __shfl_xor(r[1], off, 64);
        r[2] += __shfl_xor(r[2], off, 64);
        r[3] = max(r[3], __shfl_xor(r[3], off, 64));
        r[4] = max(r[4], __shfl_xor(r[4], off, 64));
        r[5] += __shfl_xor(r[5], off, 64);
        r[6] = max(r[6], __shfl_xor(r[6], off, 64));
        r[7] += __shfl_xor(r[7], off, 64);
        r[8] = max(r[8], __shfl_xor(r[8], off, 64));
    }
    if (threadIdx.x % 64 == 0)
        for (int q = 0; q < kBoundWords; q++) wred[q][threadIdx.x / 64] = r[q];
    __syncthreads();
    if (threadIdx.x == 0) {
        int m[kBoundWords] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int w = 0; w < (int)(blockDim.x / 64); w++) {
            m[0] = max(m[0], wred[0][w]);
            m[1] += wred[1][w];
            m[2] += wred[2][w];
            m[3] = max(m[3], wred[3][w]);
            m[4] = max(m[4], wred[4][w]);
            m[5] += wred[5][w];
            m[6] = max(m[6], wred[6][w]);
            m[7] += wred[7][w];
            m[8] = max(m[8], wred[8][w]);
        }
        const int slot = blockIdx.x % kRedSlots;
        if (m[0] > 0) atomicMax(&stat[slot], m[0]);
        if (m[1] > 0) atomicAdd(&stat[kRedSlots + slot], m[1]);
        if (m[2] > 0) atomicAdd(&stat[2 * kRedSlots + slot], m[2]);
        if (m[3] > 0) atomicMax(&stat[3 * kRedSlots + slot], m[3]);
        if (m[4] > 0) atomicMax(&stat[4 * kRedSlots + slot], m[4]);
        if (m[5] > 0) atomicAdd(&stat[5 * kRedSlots + slot], m[5]);
        if (m[6] > 0) atomicMax(&stat[6 * kRedSlots + slot], m[6]);
        if (m[7] > 0) atomicAdd(&stat[7 * kRedSlots + slot], m[7]);
        if (m[8] > 0) atomicMax(&stat[8 * kRedSlots + slot], m[8]);
    }
}

// the rows with val[i] > limit, in any order (each is computed on its own);
// one atomic per wavefront, each lane at its rank among the wavefront's rows
__global__ void k_spgemm_long_rows(int n, const int32_t *__restrict__ val, int limit, int32_t *__restrict__ rows,
                                   int32_t *__restrict__ pos) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool take = i < n && val[i] > limit;
    const uint64_t m = __ballot(take);
    if (!m) return;
    const int lane = threadIdx.x % 64, lead = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == lead) base = atomicAdd(pos, __popcll(m));
    base = __shfl(base, lead, 64);
    if (take) rows[base + __popcll(m & ((1ull << lane) - 1))] = i;
}

// After a split counting pass: key[i] = 1 for the rows the launch over all
// rows leaves out (more than plimit products, or more than dlimit distinct
// columns), and the rows of at most plimit products but more than dlimit
// distinct columns listed (one atomic per wavefront)
__global__ void k_spgemm_classify(int n, const int32_t *__restrict__ prod, int plimit,
                                  const int32_t *__restrict__ cnt, int dlimit, int32_t *__restrict__ key,
                                  int32_t *__restrict__ rows, int32_t *__restrict__ pos) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    const bool longp = i < n && prod[i] > plimit;
    const bool many = i < n && !longp && cnt[i] > dlimit;
    if (i < n) key[i] = longp || many ? 1 : 0;
    const uint64_t m = __ballot(many);
    if (!m) return;
    const int lane = threadIdx.x % 64, lead = __ffsll((unsigned long long)m) - 1;
    int base = 0;
    if (lane == lead) base = atomicAdd(pos, __popcll(m));
    base = __shfl(base, lead, 64);
    if (many) rows[base + __popcll(m & ((1ull << lane) - 1))] = i;
}

// Rows: with rows != NULL the kernel takes rows[0..n) (listed rows); with
// prod != NULL it takes rows 0..n-1 except those with prod[i] > plimit (the
// long rows by products, or in the numeric pass the rows of many distinct
// columns).
// The counting pass sizes its hash for the row's products and records the
// largest distinct count in *maxl; the numeric pass then takes a hash of at
// least twice that.
template <int G, int H, bool NUM>
__global__ void __launch_bounds__(256) k_spgemm(int n, const int32_t *__restrict__ arp,
                                               const int32_t *__restrict__ aci, const double *__restrict__ av,
                                               const int32_t *__restrict__ brp, const int32_t *__restrict__ bci,
                                               const double *__restrict__ bv, int32_t *__restrict__ cnt,
                                               const int32_t *__restrict__ crp, int32_t *__restrict__ cci,
                                               double *__restrict__ cv, int32_t *__restrict__ bad,
                                               const int32_t *__restrict__ rows, const int32_t *__restrict__ prod,
                                               int32_t *__restrict__ maxl, int plimit) {
    static_assert(H >= G && H % G == 0, "hash slots per lane");
    constexpr int R = 256 / G;
    constexpr int HV = NUM ? H : 1;  // the counting pass keeps no values
    __shared__ int key[R][H];
    __shared__ double val[R][HV];
    __shared__ int nl[R];
    int grp = threadIdx.x / G, sub = threadIdx.x % G;
    int idx = blockIdx.x * R + grp;
    for (int t = sub; t < H; t += G) key[grp][t] = -1;
    if (NUM)
        for (int t = sub; t < HV; t += G) val[grp][t] = 0.0;
    if (sub == 0) nl[grp] = 0;
    __syncthreads();
    if (idx >= n) return;
    const int i = rows ? rows[idx] : idx;
    if (prod && prod[i] > plimit) return;  // left to the launch over the listed rows
    constexpr bool numeric = NUM;
    // one product: the column's slot (linear probing), then its sum
    auto insert = [&](int c, double prod) {
        unsigned h = ((unsigned)c * 2654435761u) & (H - 1);
        int slot = -1;
        for (int probe = 0; probe < H; probe++) {
            int old = atomicCAS(&key[grp][h], -1, c);
            if (old == -1 || old == c) { slot = (int)h; break; }
            h = (h + 1) & (H - 1);
        }
        if (slot < 0) { *bad = 1; return; }
        if (numeric) val[grp][slot % HV] = val[grp][slot % HV] + prod;
    };
    // The row of A goes in chunks of G entries: lane u of the group holds
    // entry u of the chunk with the bounds of its row of B.  The first G
    // entries of the next kP rows of B are loaded together before they are
    // hashed, so the loads' latency is paid once per kP entries of A.
    constexpr int kP = 8;
    const int a0 = arp[i], a1 = arp[i + 1];
    for (int c0 = a0; c0 < a1; c0 += G) {
        const int m = min(G, a1 - c0);
        int lk_s = 0, lk_e = 0;
        double lk_a = 0.0;
        if (sub < m) {
            int k = aci[c0 + sub];
            lk_s = brp[k];
            lk_e = brp[k + 1];
            lk_a = numeric ? av[c0 + sub] : 0.0;
        }
        for (int u0 = 0; u0 < m; u0 += kP) {
            int cc[kP], fs[kP], fe[kP];
            double bb[kP], aq[kP];
#pragma unroll
            for (int q = 0; q < kP; q++) {
                cc[q] = -1; bb[q] = 0.0; aq[q] = 0.0; fs[q] = 0; fe[q] = 0;
                if (u0 + q < m) {
                    fs[q] = __shfl(lk_s, u0 + q, G);
                    fe[q] = __shfl(lk_e, u0 + q, G);
                    aq[q] = __shfl(lk_a, u0 + q, G);
                    int f = fs[q] + sub;
                    if (f < fe[q]) {
                        cc[q] = bci[f];
                        if (numeric) bb[q] = bv[f];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < kP; q++) {
                if (u0 + q < m) {
                    if (cc[q] >= 0) insert(cc[q], aq[q] * bb[q]);
                    for (int f = fs[q] + sub + G; f < fe[q]; f += G) insert(bci[f], numeric ? aq[q] * bv[f] : 0.0);
                }
                // the next entry of A may add to the same columns
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
                __builtin_amdgcn_wave_barrier();
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    // compact the occupied slots into a dense list at the front of key/val:
    // every lane first takes its slots into registers
    constexpr int PER = H / G;
    int kk[PER];
    double vv[PER];
#pragma unroll
    for (int u = 0; u < PER; u++) {
        kk[u] = key[grp][sub + u * G];
        vv[u] = numeric ? val[grp][(sub + u * G) % HV] : 0.0;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int u = 0; u < PER; u++)
        if (kk[u] >= 0) {
            int p = atomicAdd(&nl[grp], 1);
            key[grp][p] = kk[u];
            if (numeric) val[grp][p % HV] = vv[u];
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_wave_barrier();
    int L = nl[grp];
    if constexpr (!numeric) {
        if (sub == 0) {
            cnt[i] = L;
            if (L > H / 2) *bad = 1;
            // rows rarely raise the maximum: read it before the atomic
            if (L > __hip_atomic_load(maxl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) atomicMax(maxl, L);
        }
    } else {
        // each distinct column goes to its rank among the row's columns
        int base = crp[i];
        for (int t = sub; t < L; t += G) {
            int c = key[grp][t];
            int rank = 0;
            for (int u = 0; u < L; u++) rank += key[grp][u] < c;
            cci[base + rank] = c;
            cv[base + rank] = val[grp][t];
        }
    }
}

// ---- coarsest level: dense inverse ---------------------------------------------------
__global__ void k_dense_from_csr(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ v, double *__restrict__ M) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < 2 * n; c++) M[(size_t)i * 2 * n + c] = (c == n + i) ? 1.0 : 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) M[(size_t)i * 2 * n + ci[e]] = v[e];
}

// Relative pivot bound of the coarsest level's elimination: a matrix whose
// pivot (under partial pivoting) falls to 1e-12 of its largest entry is
// singular to working precision (a pure-Neumann pressure block gives pivots
// near 1e-16 of it; the workloads' coarsest matrices 1e-3 and more).
constexpr double kCoarsePivotTol = 1e-12;

// Gauss-Jordan with partial pivoting on [A | I] (n x 2n, row-major, n <=
// 1024), one workgroup of 1024 threads; leaves A^{-1} in the right half.
// Per column: pivot = largest |a_rk| (ties: smallest row), swap, scale the
// pivot row, then every thread owns columns c (coalesced across threads) and
// eliminates them in all other rows with the multipliers cached in LDS.
__global__ void __launch_bounds__(1024) k_gauss_jordan(int n, double *__restrict__ M, int32_t *__restrict__ bad) {
    __shared__ double f[1024];
    __shared__ double wv[16];
    __shared__ int wi[16];
    __shared__ int piv;
    __shared__ double thr;
    int t = threadIdx.x, lane = t % 64, wave = t / 64;
    int w = 2 * n;
    // a pivot at or below kCoarsePivotTol x max |a_ij| marks the matrix singular
    {
        double m = 0.0;
        for (long long e = t; e < (long long)n * n; e += blockDim.x) m = fmax(m, fabs(M[(e / n) * w + e % n]));
        for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
        if (lane == 0) wv[wave] = m;
        __syncthreads();
        if (t == 0) {
            double mm = wv[0];
            for (int q = 1; q < 16; q++) mm = fmax(mm, wv[q]);
            thr = kCoarsePivotTol * mm;
        }
        __syncthreads();
    }
    for (int k = 0; k < n; k++) {
        int r = k + t;
        double bv = r < n ? fabs(M[(size_t)r * w + k]) : -1.0;
        int bi = r < n ? r : n;
        for (int off = 32; off > 0; off >>= 1) {
            double ov = __shfl_xor(bv, off, 64);
            int oi = __shfl_xor(bi, off, 64);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (lane == 0) { wv[wave] = bv; wi[wave] = bi; }
        __syncthreads();
        if (t == 0) {
            double best = wv[0];
            int bidx = wi[0];
            for (int q = 1; q < 16; q++)
                if (wv[q] > best || (wv[q] == best && wi[q] < bidx)) { best = wv[q]; bidx = wi[q]; }
            piv = bidx;
            if (!(best > thr)) *bad = 1;
        }
        __syncthreads();
        int p = piv;
        if (p != k && p < n)
            for (int c = t; c < w; c += blockDim.x) {
                double x = M[(size_t)k * w + c];
                M[(size_t)k * w + c] = M[(size_t)p * w + c];
                M[(size_t)p * w + c] = x;
            }
        __syncthreads();
        double d = M[(size_t)k * w + k];
        __syncthreads();
        for (int c = k + t; c < w; c += blockDim.x) M[(size_t)k * w + c] = M[(size_t)k * w + c] / d;
        for (int rr = t; rr < n; rr += blockDim.x) f[rr] = rr == k ? 0.0 : M[(size_t)rr * w + k];
        __syncthreads();
        // (row, column) pairs in a 2-D walk: columns fastest, no divisions
        int ncol = w - (k + 1);
        int rows_per = (int)blockDim.x / ncol;
        if (rows_per >= 1) {
            // f[k] = 0 leaves the pivot row unchanged; rows go in batches of
            // four independent updates
            int rr0 = t / ncol, c = k + 1 + t % ncol;
            if (rr0 < rows_per) {
                double pk = M[k * w + c];
                int rr = rr0;
                for (; rr + 3 * rows_per < n; rr += 4 * rows_per) {
                    int r1 = rr + rows_per, r2 = rr + 2 * rows_per, r3 = rr + 3 * rows_per;
                    double m0 = M[rr * w + c], m1 = M[r1 * w + c], m2 = M[r2 * w + c], m3 = M[r3 * w + c];
                    M[rr * w + c] = m0 - f[rr] * pk;
                    M[r1 * w + c] = m1 - f[r1] * pk;
                    M[r2 * w + c] = m2 - f[r2] * pk;
                    M[r3 * w + c] = m3 - f[r3] * pk;
                }
                for (; rr < n; rr += rows_per) M[rr * w + c] = M[rr * w + c] - f[rr] * pk;
            }
        } else {
            for (int c = k + 1 + t; c < w; c += blockDim.x) {
                double pk = M[k * w + c];
                for (int rr = 0; rr < n; rr++)
                    if (rr != k) M[rr * w + c] = M[rr * w + c] - f[rr] * pk;
            }
        }
        for (int rr = t; rr < n; rr += blockDim.x)
            if (rr != k) M[(size_t)rr * w + k] = 0.0;
        __syncthreads();
    }
}

// The same Gauss-Jordan elimination for n <= 32 G (G <= 6) with the matrix
// held in registers: thread t = 32 tc + tr owns rows tr + 32 i and columns
// tc + 32 j (i, j < G).  The inverse is formed in place: after step k, column
// k of the working matrix is column orig[k] of A^{-1}, where orig[] follows
// the row swaps.  On every entry that is not structurally zero this performs
// the same operations, in the same order, as the [A | I] form above (the unit
// column n + orig[k] of the right half is 0 in every row but k when step k
// begins), so both forms give the same inverse.  The row and column of the
// step pass through LDS, double-buffered by the parity of k: two barriers per
// pivot.  The pivot loop is split by k / 32 so that the register row and
// column of the pivot are compile-time indices; the swapped-in row, the pivot
// row and the pivot column are patched around one uniform update of all
// entries.
constexpr int kGjRegMax = 192;
template <int G>
__global__ void __launch_bounds__(1024) k_gj_regs(int n, const double *__restrict__ M, double *__restrict__ inv,
                                                  int32_t *__restrict__ bad) {
    __shared__ double rowk[2][32 * G];  // the pivot row after the swap, unscaled
    __shared__ double rowo[2][32 * G];  // row k before the swap (it becomes row p)
    __shared__ double colk[2][32 * G];  // column k before the step, rows before the swap
    __shared__ int piv[2];
    __shared__ int orig[32 * G];
    __shared__ double wmax[16];
    __shared__ double thr;
    int t = threadIdx.x, tr = t % 32, tc = t / 32;
    int w = 2 * n;
    double a[G][G];
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < G; i++)
#pragma unroll
        for (int j = 0; j < G; j++) {
            int r = tr + 32 * i, c = tc + 32 * j;
            a[i][j] = (r < n && c < n) ? M[(size_t)r * w + c] : 0.0;
            m = fmax(m, fabs(a[i][j]));
        }
    // a pivot at or below kCoarsePivotTol x max |a_ij| marks the matrix singular
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if (t % 64 == 0) wmax[t / 64] = m;
    __syncthreads();
    if (t == 0) {
        double mm = wmax[0];
        for (int q = 1; q < 16; q++) mm = fmax(mm, wmax[q]);
        thr = kCoarsePivotTol * mm;
    }
    __syncthreads();
    for (int q = t; q < n; q += blockDim.x) orig[q] = q;
#pragma unroll
    for (int kg = 0; kg < G; kg++) {
        for (int kr = 0; kr < 32; kr++) {
            int k = 32 * kg + kr;
            if (k >= n) break;
            int h = k & 1;
            // column k: its owners (tc == kr) are the 32 lanes of one half wavefront
            if (tc == kr) {
                double bv = -1.0;
                int bi = n;
                bool nan = false;
#pragma unroll
                for (int i = 0; i < G; i++) {
                    int r = tr + 32 * i;
                    double v = a[i][kg];
                    if (r < n) colk[h][r] = v;
                    if (r >= k && r < n) {
                        double av = fabs(v);
                        nan = nan || av != av;
                        if (av > bv) { bv = av; bi = r; }
                    }
                }
                for (int off = 16; off > 0; off >>= 1) {
                    double ov = __shfl_xor(bv, off, 64);
                    int oi = __shfl_xor(bi, off, 64);
                    if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
                }
                if (nan) *bad = 1;
                if (tr == 0) {
                    piv[h] = bi;
                    if (!(bv > thr)) *bad = 1;
                }
            }
            __syncthreads();
            int p = piv[h];
            if (p >= n) p = k;  // no finite candidate: flagged above, no swap
            int pi = p / 32, pr = p % 32;
            if (tr == kr)
#pragma unroll
                for (int j = 0; j < G; j++) {
                    int c = tc + 32 * j;
                    if (c < n) rowo[h][c] = a[kg][j];
                }
#pragma unroll
            for (int i = 0; i < G; i++)
                if (i == pi && tr == pr)
#pragma unroll
                    for (int j = 0; j < G; j++) {
                        int c = tc + 32 * j;
                        if (c < n) rowk[h][c] = a[i][j];
                    }
            if (t == 0 && p != k) {
                int o = orig[k];
                orig[k] = orig[p];
                orig[p] = o;
            }
            __syncthreads();
            double d = rowk[h][k];
            double pk[G];
#pragma unroll
            for (int j = 0; j < G; j++) {
                int c = tc + 32 * j;
                pk[j] = c < n ? (c == k ? 1.0 / d : rowk[h][c] / d) : 0.0;
            }
            double fk = colk[h][k];
            double f[G];
#pragma unroll
            for (int i = 0; i < G; i++) {
                int r = tr + 32 * i;
                f[i] = r == p ? fk : (r < n ? colk[h][r] : 0.0);
            }
            // row p now holds the old row k
#pragma unroll
            for (int i = 0; i < G; i++)
                if (i == pi && tr == pr)
#pragma unroll
                    for (int j = 0; j < G; j++) {
                        int c = tc + 32 * j;
                        a[i][j] = c < n ? rowo[h][c] : 0.0;
                    }
#pragma unroll
            for (int i = 0; i < G; i++)
#pragma unroll
                for (int j = 0; j < G; j++) a[i][j] = a[i][j] - f[i] * pk[j];
            // the unit column n + orig[k] of the [A | I] form, and the pivot row
            if (tc == kr)
#pragma unroll
                for (int i = 0; i < G; i++) a[i][kg] = 0.0 - f[i] * pk[kg];
            if (tr == kr)
#pragma unroll
                for (int j = 0; j < G; j++) a[kg][j] = pk[j];
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < G; i++)
#pragma unroll
        for (int j = 0; j < G; j++) {
            int r = tr + 32 * i, c = tc + 32 * j;
            if (r < n && c < n) inv[(size_t)r * n + orig[c]] = a[i][j];
        }
}

__global__ void k_extract_inverse(int n, const double *__restrict__ M, double *__restrict__ inv) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int r = idx / n, c = idx % n;
    inv[idx] = M[(size_t)r * 2 * n + n + c];
}

// ---- cycle kernels -------------------------------------------------------------------
// Every cycle kernel is instantiated for double (FP64 form) and float (mixed
// form: hierarchy stored in FP32, FP32 arithmetic and accumulation).
template <typename T> __device__ __forceinline__ T two_thirds() { return (T)(2.0 / 3.0); }

// Level 0 on the grid, red-black Gauss-Seidel, on a copy of the slot arrays
// split by colour.  Cells 2h and 2h+1 always differ in the parity of i+j+k
// (a step along x flips it, and a row or layer boundary that falls inside a
// pair does too, since nx, or nx and ny, are then odd), so pair h holds one
// cell of each colour, and out[(c*7 + q)*H + h] (H = ceil(n/2)) is slot q of
// pair h's colour-c cell (0 where an odd n leaves the pair one cell).  A
// colour's sweep then reads half of the coefficients, contiguously.
__device__ __forceinline__ int cell_colour(int g, int nx, int nxy) { return ((g % nx) + (g % nxy) / nx + g / nxy) & 1; }
template <typename T>
__global__ void __launch_bounds__(kBlock) k_split_colours(int nx, int ny, int nz, const T *__restrict__ A,
                                                          T *__restrict__ out, int32_t *__restrict__ bad) {
    const int n = nx * ny * nz, nxy = nx * ny, H = (n + 1) / 2;
    int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= H) return;
    const size_t N = (size_t)n, HH = (size_t)H;
    const int g0 = 2 * h, c0 = cell_colour(g0, nx, nxy);
    const bool two = g0 + 1 < n;
    if (two && cell_colour(g0 + 1, nx, nxy) == c0) *bad = 1;  // cannot happen (see above)
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        out[((size_t)c0 * NSLOT + q) * HH + h] = A[(size_t)q * N + g0];
        out[((size_t)(1 - c0) * NSLOT + q) * HH + h] = two ? A[(size_t)q * N + g0 + 1] : (T)0;
    }
}

// colour c of the sweep; with zero set the other colour is taken as 0 and x
// is not read (b - 0 is b exactly, so this equals the sweep over a zeroed x).
// Same operations in the same order as the sweep over the slot arrays.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_gs_split(int nx, int ny, int nz, const T *__restrict__ Ac,
                                                     const T *__restrict__ b, T *__restrict__ x, int colour,
                                                     int zero) {
    const int n = nx * ny * nz, nxy = nx * ny, H = (n + 1) / 2;
    int h = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (h >= H) return;
    const int g0 = 2 * h;
    const int i = cell_colour(g0, nx, nxy) == colour ? g0 : g0 + 1;
    if (i >= n) return;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    const size_t HH = (size_t)H;
    const T *Aq = Ac + (size_t)colour * NSLOT * HH;
    T s = b[i], d = Aq[(size_t)S_D * HH + h];
    if (!zero) {
#pragma unroll
        for (int q = 0; q < NSLOT; q++) {
            int j = nb[q];
            if (j < 0 || q == S_D) continue;
            s = s - Aq[(size_t)q * HH + h] * x[j];
        }
    }
    x[i] = s / d;
}

// level 0 damped Jacobi sweep (slot form): xo = xi + (2/3) (b - A xi) / a_ii
template <typename T>
__global__ void __launch_bounds__(kBlock) k_jacobi_slots(int nx, int ny, int nz, const T *__restrict__ A,
                                                         const T *__restrict__ b, const T *__restrict__ xi,
                                                         T *__restrict__ xo) {
    int n = nx * ny * nz;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    size_t N = (size_t)n;
    T s = 0, d = 0;
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        int j = nb[q];
        if (j < 0) continue;
        T a = A[(size_t)q * N + i];
        s = s + a * xi[j];
        if (q == S_D) d = a;
    }
    xo[i] = xi[i] + two_thirds<T>() * ((b[i] - s) / d);
}

// r = b - A x (slot form)
template <typename T>
__global__ void __launch_bounds__(kBlock) k_resid_slots(int nx, int ny, int nz, const T *__restrict__ A,
                                                        const T *__restrict__ b, const T *__restrict__ x,
                                                        T *__restrict__ r) {
    int n = nx * ny * nz;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    size_t N = (size_t)n;
    T s = 0;
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        int j = nb[q];
        if (j < 0) continue;
        s = s + A[(size_t)q * N + i] * x[j];
    }
    r[i] = b[i] - s;
}

// CSR row operations on coarse levels: G lanes per row (G a power of two
// dividing 64) sum the row's products in strides of G and combine them with
// cross-lane shuffles.
// OP_JACOBI: damped Jacobi sweep, y = x + (2/3)(b - A x) / a_ii; OP_L1: l1-Jacobi
// sweep, y = x + (b - A x) / sum_j |a_ij|; the *0 forms start from x = 0.
enum { OP_MV = 0, OP_RESID = 1, OP_ADD = 2, OP_JACOBI = 3, OP_JACOBI0 = 4, OP_L1 = 5, OP_L10 = 6 };

template <int G, typename T>
__global__ void __launch_bounds__(kBlock) k_csr_rowop(int n, const int32_t *__restrict__ rp,
                                                      const int32_t *__restrict__ ci, const T *__restrict__ v,
                                                      const T *__restrict__ x, int op, const T *__restrict__ b,
                                                      const int32_t *__restrict__ dpos, const T *__restrict__ dl1,
                                                      T *__restrict__ y) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    int row = gid / G, sub = gid % G;
    if (row >= n) return;  // whole groups leave together
    if (op == OP_JACOBI0) {
        // one damped Jacobi sweep from a zero guess
        if (sub == 0) y[row] = two_thirds<T>() * (b[row] / v[dpos[row]]);
        return;
    }
    if (op == OP_L10) {
        if (sub == 0) y[row] = b[row] / dl1[row];
        return;
    }
    T s = 0;
#pragma unroll 4
    for (int e = rp[row] + sub; e < rp[row + 1]; e += G) s = s + v[e] * x[ci[e]];
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s = s + __shfl_xor(s, off, G);
    if (sub != 0) return;
    switch (op) {
    case OP_MV: y[row] = s; break;
    case OP_RESID: y[row] = b[row] - s; break;
    case OP_ADD: y[row] = y[row] + s; break;
    case OP_L1: y[row] = x[row] + (b[row] - s) / dl1[row]; break;
    default: {
        T d = v[dpos[row]];
        y[row] = x[row] + two_thirds<T>() * ((b[row] - s) / d);
    }
    }
}

// the zero-guess l1-Jacobi sweep and the residual in one pass: x = b / d_l1
// and r = b - A x, the neighbours' x_j formed from b_j and d_j as the sweep
// forms them (same values, same summation as the two passes)
template <int G, typename T>
__global__ void __launch_bounds__(kBlock) k_csr_l1_resid(int n, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci, const T *__restrict__ v,
                                                         const T *__restrict__ b, const T *__restrict__ dl1,
                                                         T *__restrict__ x, T *__restrict__ r) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    int row = gid / G, sub = gid % G;
    if (row >= n) return;  // whole groups leave together
    T s = 0;
#pragma unroll 4
    for (int e = rp[row] + sub; e < rp[row + 1]; e += G) {
        int j = ci[e];
        s = s + v[e] * (b[j] / dl1[j]);
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) s = s + __shfl_xor(s, off, G);
    if (sub != 0) return;
    T bi = b[row];
    x[row] = bi / dl1[row];
    r[row] = bi - s;
}

// ---- sliced copies of large CSR matrices --------------------------------------------
// Matrices of at least kSellRows rows (bo_cpr_opts.sell_rows) are also kept
// in SELL-C form (C = 64 or 16 rows per slice, see SellMat): one thread per
// row then reads its entries with every load of a wavefront on runs of C
// consecutive words, where the lanes-per-row form reads short runs of a row
// each (a level of 11M rows with 40 entries a row streamed at about 2 TB/s).
// The row sums run in entry order.
constexpr int kSellRows = 1 << 20;
// the width of each slice (times C): its longest row, or in a stencil slice
// (a grid's cell rows, see SellGrid; C = 64) 7 + the most entries a row has
// beyond its stencil neighbours (one lane per row, the maximum by shuffles
// over the slice's C lanes)
template <int C>
__global__ void k_csr_slice_width(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                  SellGrid G, int32_t *__restrict__ w64) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x, S = r / C;
    int len = 0;
    if (r < n) {
        len = rp[r + 1] - rp[r];
        if (C == 64 && sell_stencil_slice(G, S)) {
            int nb[NSLOT], extra = 0;
            sell_stencil_nbrs(G, r, nb);
            for (int e = rp[r]; e < rp[r + 1]; e++) extra += sell_slot_in(nb, ci[e]) < 0;
            len = NSLOT + extra;
        }
    }
    for (int off = C / 2; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, C));
    if (threadIdx.x % C == 0 && C * S < n) w64[S] = C * len;
}
template <int C>
__global__ void k_csr_sell_fill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                const double *__restrict__ v, const int32_t *__restrict__ off, SellGrid G,
                                int32_t *__restrict__ col, double *__restrict__ val) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int S = r / C, lane = r % C;
    const int base = off[S] + lane, w = (off[S + 1] - off[S]) / C;
    const int b = rp[r], len = rp[r + 1] - b;
    if (C == 64 && sell_stencil_slice(G, S)) {
        // stencil positions (zero where the row lacks the entry) on their
        // implicit columns, then the other entries; padding on the row's own
        // column
        for (int p = 0; p < w; p++) {
            col[base + C * p] = p < NSLOT ? sell_stencil_col(G, r, p, n) : r;
            val[base + C * p] = 0.0;
        }
        int nb[NSLOT];
        sell_stencil_nbrs(G, r, nb);
        int next = NSLOT;
        for (int q = 0; q < len; q++) {
            const int c = ci[b + q];
            int p = sell_slot_in(nb, c);
            if (p < 0) p = next++;
            col[base + C * p] = c;
            val[base + C * p] = v[b + q];
        }
        return;
    }
    // padding: the row's first column (a valid index of x for rectangular
    // P and R too; column 0 for an empty row) with value 0
    const int pad = len > 0 ? ci[b] : 0;
    for (int p = 0; p < w; p++) {
        col[base + C * p] = p < len ? ci[b + p] : pad;
        val[base + C * p] = p < len ? v[b + p] : 0.0;
    }
}
// y = op(A x) as k_csr_rowop, for OP_MV, OP_RESID, OP_ADD and OP_L1
template <typename T, int C>
__global__ void __launch_bounds__(kBlock) k_sell_rowop(int n, const int32_t *__restrict__ off,
                                                       const int32_t *__restrict__ col, const T *__restrict__ val,
                                                       SellGrid G, const T *__restrict__ x, int op,
                                                       const T *__restrict__ b, const T *__restrict__ dl1,
                                                       T *__restrict__ y) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int S = r / C, lane = r % C;
    const int base = off[S] + lane, w = (off[S + 1] - off[S]) / C;
    T s = 0;
    int p0 = 0;
    if (C == 64 && sell_stencil_slice(G, S)) {
        // the stencil positions: columns from the row index, loads issued together
        T a[NSLOT], xv[NSLOT];
#pragma unroll
        for (int p = 0; p < NSLOT; p++) a[p] = val[base + C * p];
#pragma unroll
        for (int p = 0; p < NSLOT; p++) xv[p] = x[sell_stencil_col(G, r, p, n)];
#pragma unroll
        for (int p = 0; p < NSLOT; p++) s = s + a[p] * xv[p];
        p0 = NSLOT;
    }
#pragma unroll 4
    for (int p = p0; p < w; p++) s = s + val[base + C * p] * x[col[base + C * p]];
    switch (op) {
    case OP_MV: y[r] = s; break;
    case OP_RESID: y[r] = b[r] - s; break;
    case OP_ADD: y[r] = y[r] + s; break;
    default: y[r] = x[r] + (b[r] - s) / dl1[r]; break;  // OP_L1
    }
}

// dense y = M x, one wavefront per row
template <typename T>
__global__ void __launch_bounds__(kBlock) k_dense_mv(int n, const T *__restrict__ M, const T *__restrict__ x,
                                                     T *__restrict__ y) {
    int gid = blockIdx.x * blockDim.x + threadIdx.x;
    int row = gid / 64, lane = gid % 64;
    if (row >= n) return;
    T s = 0;
    for (int c = lane; c < n; c += 64) s = s + M[(size_t)row * n + c] * x[c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = s + __shfl_xor(s, off, 64);
    if (lane == 0) y[row] = s;
}

// round an FP64 array to FP32 (round to nearest even)
__global__ void k_to_f32(long long n, const double *__restrict__ a, float *__restrict__ b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

template <typename T>
__global__ void k_zero(long long n, T *__restrict__ x) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (T)0;
}

__global__ void k_f32_to_f64(long long n, const float *__restrict__ a, double *__restrict__ b) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (double)a[i];
}

bo_status read_flag(int32_t *dflag, hipStream_t s, int32_t *out) {
    HostRead r{dflag, sizeof(int32_t), out};
    return host_reads(&r, 1, s);
}

}  // namespace

// the sliced copy of a CSR matrix of n rows (M.on stays false below min_rows)
static bo_status sell_from_csr(SellMat &M, int n, const int32_t *rp, const int32_t *ci, const double *v,
                               int min_rows, DBuf<int32_t> &work, hipStream_t s, const SellGrid &G = SellGrid{}) {
    M.on = false;
    M.grid = G;
    M.c = G.rows > 0 ? 64 : 16;
    if (n < 1 || n < min_rows) return BO_OK;
    const int nsl = (n + M.c - 1) / M.c;
    BO_TRY(work.alloc(nsl));
    BO_TRY(M.off.alloc(nsl + 1));
    if (M.c == 64) k_csr_slice_width<64><<<grid_for(64LL * nsl), kBlock, 0, s>>>(n, rp, ci, G, work.p);
    else k_csr_slice_width<16><<<grid_for(16LL * nsl), kBlock, 0, s>>>(n, rp, ci, G, work.p);
    // the padded size in 64 bits first: the prefix sum is 32-bit
    std::vector<int32_t> w(nsl);
    BO_HIP(hipMemcpyAsync(w.data(), work.p, sizeof(int32_t) * nsl, hipMemcpyDeviceToHost, s));
    BO_HIP(hipStreamSynchronize(s));
    long long padded = 0;
    for (int32_t x : w) padded += x;
    if (padded > (1ll << 30)) return BO_OK;  // keep the CSR form
    int32_t total = 0;
    BO_TRY(scan_counts(work.p, M.off.p, nsl, &total, s));
    BO_TRY(M.col.alloc(total));
    BO_TRY(M.val.alloc(total));
    if (M.c == 64) k_csr_sell_fill<64><<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, M.off.p, G, M.col.p, M.val.p);
    else k_csr_sell_fill<16><<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, M.off.p, G, M.col.p, M.val.p);
    BO_HIP(hipGetLastError());
    M.len = total;
    M.on = true;
    return BO_OK;
}

template <typename T> static const T *sell_val(const SellMat &M);
template <> const double *sell_val<double>(const SellMat &M) { return M.val.p; }
template <> const float *sell_val<float>(const SellMat &M) { return M.val32.p; }

// y = op(A x) for a CSR matrix with nnz entries over n rows (see k_csr_rowop)
template <typename T>
static bo_status csr_rowop(int n, int nnz, const int32_t *rp, const int32_t *ci, const T *v, const T *x, int op,
                           const T *b, const int32_t *dpos, T *y, hipStream_t s, const T *dl1 = nullptr,
                           const SellMat *sm = nullptr) {
    if (sm && sm->on && (op == OP_MV || op == OP_RESID || op == OP_ADD || op == OP_L1)) {
        if (sm->c == 64)
            k_sell_rowop<T, 64><<<grid_for(n), kBlock, 0, s>>>(n, sm->off.p, sm->col.p, sell_val<T>(*sm), sm->grid,
                                                               x, op, b, dl1, y);
        else
            k_sell_rowop<T, 16><<<grid_for(n), kBlock, 0, s>>>(n, sm->off.p, sm->col.p, sell_val<T>(*sm), sm->grid,
                                                               x, op, b, dl1, y);
        BO_HIP(hipGetLastError());
        return BO_OK;
    }
    double avg = n > 0 ? (double)nnz / n : 1.0;
    long long threads;
#define BO_ROWOP(G)                                                                                  \
    threads = (long long)n * G;                                                                      \
    k_csr_rowop<G, T><<<grid_for(threads), kBlock, 0, s>>>(n, rp, ci, v, x, op, b, dpos, dl1, y)
    // two to four entries per lane: a wavefront then covers several rows per
    // round trip to memory
    if (avg <= 8.0) { BO_ROWOP(4); }
    else if (avg <= 16.0) { BO_ROWOP(8); }
    else if (avg <= 64.0) { BO_ROWOP(16); }
    else if (avg <= 128.0) { BO_ROWOP(32); }
    else { BO_ROWOP(64); }
#undef BO_ROWOP
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// x = b / d_l1 and r = b - A x (k_csr_l1_resid), lanes per row as csr_rowop
template <typename T>
static bo_status csr_l1_resid(int n, int nnz, const int32_t *rp, const int32_t *ci, const T *v, const T *b,
                              const T *dl1, T *x, T *r, hipStream_t s) {
    double avg = n > 0 ? (double)nnz / n : 1.0;
    long long threads;
#define BO_L1R(G)                                                                                    \
    threads = (long long)n * G;                                                                      \
    k_csr_l1_resid<G, T><<<grid_for(threads), kBlock, 0, s>>>(n, rp, ci, v, b, dl1, x, r)
    if (avg <= 8.0) { BO_L1R(4); }
    else if (avg <= 16.0) { BO_L1R(8); }
    else if (avg <= 64.0) { BO_L1R(16); }
    else if (avg <= 128.0) { BO_L1R(32); }
    else { BO_L1R(64); }
#undef BO_L1R
    BO_HIP(hipGetLastError());
    return BO_OK;
}

static bo_status to_f32(long long n, const double *a, float *b, hipStream_t s) {
    if (n <= 0) return BO_OK;
    k_to_f32<<<grid_for(n), kBlock, 0, s>>>(n, a, b);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// ---- host: decoupling -------------------------------------------------------------
bo_status qi_decouple(bo_cpr *pc, hipStream_t s) {
    long long n = pc->n;
    if (pc->general) {
        // weights of every row, then A_pp in CSR as level 0 of the hierarchy
        BO_TRY(pc->cw.alloc(3 * n));
        BO_HIP(hipMemsetAsync(pc->flag.p, 0, sizeof(int32_t), s));
        k_qi_weights_bsr<<<grid_for(n), kBlock, 0, s>>>((int)n, pc->Arp.p, pc->Aci.p, pc->Aval.p, pc->o.qi_mode,
                                                        pc->cw.p, pc->flag.p);
        BO_HIP(hipGetLastError());
        int32_t bad = 0;
        BO_TRY(read_flag(pc->flag.p, s, &bad));
        if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "quasi-IMPES: singular saturation block or missing diagonal");
        Level &L0 = pc->lv[0];
        int npr = pc->npr;
        L0.n = npr;
        BO_TRY(pc->sw.cnt.alloc(npr));
        BO_TRY(L0.rp.alloc(npr + 1));
        k_app_counts<<<grid_for(npr), kBlock, 0, s>>>(npr, pc->Arp.p, pc->Aci.p, pc->sw.cnt.p);
        int32_t total = 0;
        BO_TRY(scan_counts(pc->sw.cnt.p, L0.rp.p, npr, &total, s));
        L0.nnz = total;
        BO_TRY(L0.ci.alloc(total));
        BO_TRY(L0.v.alloc(total));
        k_app_fill<<<grid_for(npr), kBlock, 0, s>>>(npr, pc->Arp.p, pc->Aci.p, pc->Aval.p, pc->cw.p, L0.rp.p,
                                                    L0.ci.p, L0.v.p);
        BO_HIP(hipGetLastError());
        return BO_OK;
    }
    BO_TRY(pc->cw.alloc(3 * n));
    BO_TRY(pc->app.alloc(7 * n));
    BO_HIP(hipMemsetAsync(pc->flag.p, 0, sizeof(int32_t), s));
    k_qi_decouple<<<grid_for(n), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, pc->A.p, pc->o.qi_mode,
                                                 pc->cw.p, pc->app.p, pc->flag.p);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    BO_TRY(read_flag(pc->flag.p, s, &bad));
    if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "quasi-IMPES: singular saturation block");
    return BO_OK;
}

bo_status qi_restrict(bo_cpr *pc, const double *v, double *rp, hipStream_t s) {
    long long n = pc->npr;
    k_qi_restrict<double><<<grid_for(n), kBlock, 0, s>>>(n, pc->cw.p, v, rp);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status qi_restrict_f32(bo_cpr *pc, const double *v, float *rp, hipStream_t s) {
    long long n = pc->npr;
    k_qi_restrict<float><<<grid_for(n), kBlock, 0, s>>>(n, pc->cw.p, v, rp);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// ---- host: hierarchy ---------------------------------------------------------------
// dflag: a deferred flag (checked at the end of the setup; a zero diagonal
// only makes values non-finite, every index stays valid)
static bo_status level_diag(Level &L, int32_t *dflag, hipStream_t s) {
    BO_TRY(L.diagpos.alloc(L.n));
    BO_TRY(L.dl1.alloc(L.n));
    k_diag<<<grid_for(L.n), kBlock, 0, s>>>(L.n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p, L.dl1.p, dflag);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// smoother weight of the prolongator, (4/3)/rho, on the device
__global__ void k_omega(const unsigned long long *__restrict__ rho_bits, double *__restrict__ omega,
                        int32_t *__restrict__ bad, int32_t *__restrict__ plong) {
    plong[0] = 0;  // the long-row list of the prolongator, filled next
    unsigned long long rb = 0;
    for (int q = 0; q < kRedSlots; q++) rb = rho_bits[q] > rb ? rho_bits[q] : rb;
    double rho = __longlong_as_double((long long)rb);
    if (!(rho > 0.0) || !(rho < INFINITY)) {
        *bad = 1;
        *omega = 0.0;
    } else {
        *omega = (4.0 / 3.0) / rho;
    }
}

// C = A B, counting pass, prefix sum, numeric pass.  The counting hash of a
// row must hold twice its products: rows are sized by the longest row unless
// a few rows (under 1 %: a well through many layers, the aggregates next to
// it) have more than 512 or more than 128 products; then the others take a
// hash sized for the longest of them and the long rows a launch of their
// own.  Each launch's numeric pass sizes its hash from the largest distinct
// count its own rows had.
static bo_status spgemm(int n, const int32_t *arp, const int32_t *aci, const double *av, const int32_t *brp,
                        const int32_t *bci, const double *bv, DBuf<int32_t> &crp, DBuf<int32_t> &cci,
                        DBuf<double> &cv, int *cnnz, SetupWork &W, hipStream_t s, double bavg) {
    // rows of many products whose B rows are short (at most 32 entries on
    // average) take 32 lanes, not 64, so that fewer lanes idle per B row
    const bool g32 = bavg <= 32.0;
    DBuf<int32_t> &cnt = W.gcnt;
    BO_TRY(cnt.alloc(n));
    BO_TRY(crp.alloc(n + 1));
    BO_TRY(W.sg_prod.alloc(n));
    // [0, kBoundWords kRedSlots): reduction words of k_spgemm_bound, then
    // the long-row list position, the largest distinct counts of the rows
    // launched together and of the long rows, and the hash-capacity flag
    // (one clear for all of them)
    constexpr int kPos = kBoundWords * kRedSlots, kMaxl = kPos + 1, kMaxlLong = kPos + 2, kBad = kPos + 3;
    BO_TRY(W.sg_stat.alloc(kBad + 1));
    BO_HIP(hipMemsetAsync(W.sg_stat.p, 0, sizeof(int32_t) * (kBad + 1), s));
    int32_t *const bflag = W.sg_stat.p + kBad;
    k_spgemm_bound<<<grid_for(n), kBlock, 0, s>>>(n, arp, aci, brp, W.sg_prod.p, W.sg_stat.p);
    int32_t stat[kBoundWords * kRedSlots] = {};
    HostRead rd{W.sg_stat.p, sizeof stat, stat};
    BO_TRY(host_reads(&rd, 1, s));
    int red[kBoundWords] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = 0; q < kRedSlots; q++) {
        red[0] = std::max(red[0], stat[q]);
        red[1] += stat[kRedSlots + q];
        red[2] += stat[2 * kRedSlots + q];
        red[3] = std::max(red[3], stat[3 * kRedSlots + q]);
        red[4] = std::max(red[4], stat[4 * kRedSlots + q]);
        red[5] += stat[5 * kRedSlots + q];
        red[6] = std::max(red[6], stat[6 * kRedSlots + q]);
        red[7] += stat[7 * kRedSlots + q];
        red[8] = std::max(red[8], stat[8 * kRedSlots + q]);
    }
    const int bound = red[0];
    // counting pass: lanes per row and hash slots from the row's products
    auto pick = [](int b) { return b <= 32 ? 0 : b <= 64 ? 4 : b <= 128 ? 1 : b <= 256 ? 5 : b <= 512 ? 2 : 3; };
    auto count_slots = [](int sel) {
        return sel == 0 ? 64 : sel == 4 ? 128 : sel == 1 ? 256 : sel == 5 ? 512 : sel == 2 ? 1024 : 2048;
    };
    // split when the long rows are few (below 1 %): at 32 products if the
    // longest row would otherwise take more than 8 lanes (a grid's level 0
    // next to long well rows: 8 lanes and a 64-slot hash for the others),
    // else at 128, else at 256, else at 512
    int limit = 0, nlong = 0, bound_rest = bound;
    if (bound > 2 * kShortProducts && (long long)red[5] * 100 < n) {
        limit = kShortProducts; nlong = red[5]; bound_rest = red[6];
    } else if (bound > kLongProducts && (long long)red[1] * 100 < n) {
        limit = kLongProducts; nlong = red[1]; bound_rest = red[3];
    } else if (bound > kMidProducts && (long long)red[7] * 100 < n) {
        limit = kMidProducts; nlong = red[7]; bound_rest = red[8];
    } else if (bound > kVeryLongProducts && (long long)red[2] * 100 < n) {
        limit = kVeryLongProducts; nlong = red[2]; bound_rest = red[4];
    }
    const bool split = limit > 0;
    const int sel_all = pick(bound_rest), sel_long = pick(bound);
    const int32_t *prod = split ? W.sg_prod.p : nullptr;
    if (split) {
        BO_TRY(W.sg_rows.alloc(nlong));
        k_spgemm_long_rows<<<grid_for(n), kBlock, 0, s>>>(n, W.sg_prod.p, limit, W.sg_rows.p, W.sg_stat.p + kPos);
    }
    auto count = [&](int sel, int rn, const int32_t *rows, const int32_t *pr, int32_t *maxl) {
        if (rn <= 0) return;
#define BO_SPGEMM_COUNT(G, H)                                                                                 \
    k_spgemm<G, H, false><<<grid_for((long long)rn * G), 256, 0, s>>>(rn, arp, aci, av, brp, bci, bv, cnt.p, \
                                                                      nullptr, nullptr, nullptr, bflag, rows, \
                                                                      pr, maxl, limit)
        switch (sel) {
        case 0: BO_SPGEMM_COUNT(8, 64); break;
        case 4: BO_SPGEMM_COUNT(8, 128); break;
        case 1: BO_SPGEMM_COUNT(16, 256); break;
        case 5: BO_SPGEMM_COUNT(32, 512); break;
        case 2: if (g32) BO_SPGEMM_COUNT(32, 1024); else BO_SPGEMM_COUNT(64, 1024); break;
        default: if (g32) BO_SPGEMM_COUNT(32, 2048); else BO_SPGEMM_COUNT(64, 2048); break;
        }
#undef BO_SPGEMM_COUNT
    };
    count(sel_all, n, nullptr, prod, W.sg_stat.p + kMaxl);
    if (split) count(sel_long, nlong, W.sg_rows.p, nullptr, W.sg_stat.p + kMaxlLong);
    BO_HIP(hipGetLastError());
    int32_t bad = 0, total = 0, lmax = 0, lmax_long = 0;
    HostRead ex[3] = {{bflag, sizeof bad, &bad}, {W.sg_stat.p + kMaxl, sizeof lmax, &lmax},
                      {W.sg_stat.p + kMaxlLong, sizeof lmax_long, &lmax_long}};
    BO_TRY(scan_counts(cnt.p, crp.p, n, &total, s, ex, 3));
    if (bad) return fail(BO_ERR_UNSUPPORTED, "AMG: Galerkin product row exceeds the LDS hash capacity");
    BO_TRY(cci.alloc(total));
    BO_TRY(cv.alloc(total));
    // numeric pass: the same lanes per row, a hash of at least twice the
    // largest distinct count of the rows it takes (never more than the
    // counting pass had), so no insertion can fail and the LDS left over
    // keeps more rows resident
    auto numeric = [&](int sel, int rn, const int32_t *rows, const int32_t *pr, int plimit, int dmax) {
        if (rn <= 0) return;
        int h = 64;
        while (h < 2 * dmax && h < count_slots(sel)) h *= 2;
        // (32 lanes hold at most a 1024-slot numeric hash within the LDS)
        const int G = sel == 0 || sel == 4 ? 8 : sel == 1 ? 16 : (g32 && h <= 1024 ? 32 : 64);
#define BO_SPGEMM_NUM(GG, H)                                                                                    \
    k_spgemm<GG, H, true><<<grid_for((long long)rn * GG), 256, 0, s>>>(rn, arp, aci, av, brp, bci, bv, nullptr, \
                                                                       crp.p, cci.p, cv.p, bflag, rows, pr,    \
                                                                       W.sg_stat.p + kMaxl, plimit)
        if (G == 8) {
            if (h <= 64) BO_SPGEMM_NUM(8, 64); else BO_SPGEMM_NUM(8, 128);
        } else if (G == 16) {
            if (h <= 64) BO_SPGEMM_NUM(16, 64); else if (h <= 128) BO_SPGEMM_NUM(16, 128); else BO_SPGEMM_NUM(16, 256);
        } else if (G == 32) {
            switch (h) {
            case 64: BO_SPGEMM_NUM(32, 64); break;
            case 128: BO_SPGEMM_NUM(32, 128); break;
            case 256: BO_SPGEMM_NUM(32, 256); break;
            case 512: BO_SPGEMM_NUM(32, 512); break;
            default: BO_SPGEMM_NUM(32, 1024); break;
            }
        } else {
            switch (h) {
            case 64: BO_SPGEMM_NUM(64, 64); break;
            case 128: BO_SPGEMM_NUM(64, 128); break;
            case 256: BO_SPGEMM_NUM(64, 256); break;
            case 512: BO_SPGEMM_NUM(64, 512); break;
            case 1024: BO_SPGEMM_NUM(64, 1024); break;
            default: BO_SPGEMM_NUM(64, 2048); break;
            }
        }
#undef BO_SPGEMM_NUM
    };
    // A few rows of many distinct columns (a well's) would size every row's
    // hash: below 10 % of the rows they are listed and take a launch of their
    // own, the others a hash for kFewDistinct columns.
    // Without a split by products the threshold is 64 distinct columns, or,
    // on products of 2^17 rows and more, 128 where more than 10 % of the rows
    // have over 64 (a coarse level's Galerkin product: a 256-slot hash for
    // the others instead of one sized by the longest row; on fewer rows the
    // extra list and read cost more than they save).
    constexpr int kFewDistinct = 64;
    int nbig = 0, dlim = kFewDistinct;
    if (!split && lmax > kFewDistinct) {
        int32_t *pos = W.sg_stat.p + kPos;  // unused without the products split
        BO_TRY(W.sg_rows.alloc(n));
        const int dmaxl = n >= (1 << 17) ? 2 * kFewDistinct : kFewDistinct;
        for (int dl = kFewDistinct; dl <= dmaxl && lmax > dl; dl *= 2) {
            BO_HIP(hipMemsetAsync(pos, 0, sizeof(int32_t), s));
            k_spgemm_long_rows<<<grid_for(n), kBlock, 0, s>>>(n, cnt.p, dl, W.sg_rows.p, pos);
            HostRead rb{pos, sizeof nbig, &nbig};
            BO_TRY(host_reads(&rb, 1, s));
            dlim = dl;
            if ((long long)nbig * 10 < n) break;
        }
    }
    // The same after a split by products: the rows of few products whose
    // distinct columns are many (next to a long row) take a launch of their
    // own too.
    int nbig2 = 0;
    if (split && lmax > kFewDistinct) {
        int32_t *pos = W.sg_stat.p + kPos;  // the long-row list is complete: its position word is free again
        BO_TRY(W.sg_rows2.alloc(n));
        BO_TRY(W.sg_key.alloc(n));
        BO_HIP(hipMemsetAsync(pos, 0, sizeof(int32_t), s));
        // (the products per row stay: the launch below may still need them)
        k_spgemm_classify<<<grid_for(n), kBlock, 0, s>>>(n, W.sg_prod.p, limit, cnt.p, kFewDistinct, W.sg_key.p,
                                                          W.sg_rows2.p, pos);
        HostRead rb{pos, sizeof nbig2, &nbig2};
        BO_TRY(host_reads(&rb, 1, s));
    }
    if (nbig > 0 && (long long)nbig * 10 < n) {
        numeric(sel_all, n, nullptr, cnt.p, dlim, dlim);
        numeric(sel_all, nbig, W.sg_rows.p, nullptr, 0, lmax);
    } else if (nbig2 > 0 && (long long)nbig2 * 10 < n) {
        numeric(sel_all, n, nullptr, W.sg_key.p, 0, kFewDistinct);
        numeric(sel_all, nbig2, W.sg_rows2.p, nullptr, 0, lmax);
        numeric(sel_long, nlong, W.sg_rows.p, nullptr, 0, lmax_long);
    } else {
        numeric(sel_all, n, nullptr, prod, limit, lmax);
        if (split) numeric(sel_long, nlong, W.sg_rows.p, nullptr, 0, lmax_long);
    }
    BO_HIP(hipGetLastError());
    *cnnz = total;
    return BO_OK;
}

// after_l0 (may be NULL) is called once on the host when level 0's
// aggregates have been enqueued (or when the hierarchy stops at level 0):
// work that competes for HBM with level 0's strength and MIS-2 passes can be
// started then, beside the products that follow.
bo_status amg_setup(bo_cpr *pc, hipStream_t s, const std::function<bo_status()> &after_l0) {
    bool forked = false;
    auto fork = [&]() -> bo_status {
        if (forked || !after_l0) return BO_OK;
        forked = true;
        return after_l0();
    };
    const bo_cpr_opts &o = pc->o;
    int32_t *flag = pc->flag.p;
    // level 0: CSR with the stencil pattern (the general form built it with
    // the decoupling)
    Level &L0 = pc->lv[0];
    SetupWork &W = pc->sw;
    if (!pc->general) {
        L0.n = pc->n;
        DBuf<int32_t> &cnt = W.cnt;
        BO_TRY(cnt.alloc(L0.n));
        BO_TRY(L0.rp.alloc(L0.n + 1));
        k_stencil_counts<<<grid_for(L0.n), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, cnt.p);
        int32_t total = 0;
        BO_TRY(scan_counts(cnt.p, L0.rp.p, L0.n, &total, s));
        L0.nnz = total;
        BO_TRY(L0.ci.alloc(total));
        BO_TRY(L0.v.alloc(total));
        k_slots_to_csr<<<grid_for(L0.n), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, pc->app.p, L0.rp.p,
                                                          L0.ci.p, L0.v.p);
        BO_HIP(hipGetLastError());
    }
    int max_levels = std::min(std::max(o.max_levels, 1), kMaxLevels);
    double t2 = o.theta * o.theta;
    // flags whose failure leaves every index valid are checked once, at the
    // end: [0] zero diagonal, [1] unaggregated node, [2] smoother bound,
    // [3] a colour pair of the split level-0 copy
    BO_TRY(W.dfl.alloc(4));
    BO_TRY(W.omg.alloc(kMaxLevels));
    BO_HIP(hipMemsetAsync(W.dfl.p, 0, sizeof(int32_t) * 4, s));
    if (!pc->general && o.smoother == BO_SMOOTH_GS) {
        // the colour-split copy the red-black sweeps read (k_gs_split)
        const long long H = ((long long)L0.n + 1) / 2;
        BO_TRY(pc->appc.alloc(2 * NSLOT * (size_t)H));
        k_split_colours<double><<<grid_for(H), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, pc->app.p, pc->appc.p,
                                                               W.dfl.p + 3);
        BO_HIP(hipGetLastError());
    }
    int l = 0;
    for (;; l++) {
        Level &L = pc->lv[l];
        BO_TRY(level_diag(L, W.dfl.p, s));
        BO_TRY(L.x.alloc(L.n));
        BO_TRY(L.b.alloc(L.n));
        BO_TRY(L.r.alloc(L.n));
        BO_TRY(L.t.alloc(L.n));
        if (L.n <= o.coarse_max || l + 1 >= max_levels) break;
        int n = L.n;
        BO_TRY(L.sf.alloc(L.nnz));
        if (l == 0 && !pc->general)
            k_strength_slots<<<grid_for(n), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, pc->app.p, L.rp.p, t2,
                                                             L.sf.p);
        else if ((double)L.nnz / n <= 12.0)
            k_strength<4><<<grid_for((long long)n * 4), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p, t2,
                                                                        L.sf.p);
        else
            k_strength<32><<<grid_for((long long)n * 32), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p,
                                                                          t2, L.sf.p);
        // MIS-2
        DBuf<uint8_t> &state = W.state, &nw = W.nw, &d1 = W.d1;
        DBuf<uint64_t> &m1 = W.m1;
        BO_TRY(state.alloc(n)); BO_TRY(nw.alloc(n)); BO_TRY(d1.alloc(n)); BO_TRY(m1.alloc(n));
        // each round reports a change in a word of its own (cleared by
        // k_mis_init, kMisWords of them, cleared again when they run out), so
        // no round needs a memset before it
        BO_TRY(W.misw.alloc(kMisWords));
        k_mis_init<<<grid_for(std::max(n, kMisWords)), kBlock, 0, s>>>(n, L.rp.p, L.sf.p, state.p, W.misw.p);
        int word = 0;
        // rounds are checked for completion after the fourth and then every
        // second round: a round on a graph with no undecided node changes
        // nothing
        for (int round = 0;; round += 2) {
            if (round > 10000) return fail(BO_ERR_HIP, "AMG: MIS-2 did not terminate");
            int32_t *rflag = nullptr;
            for (int rep = 0; rep < (round == 0 ? 4 : 2); rep++) {
                if (word == kMisWords) {
                    BO_HIP(hipMemsetAsync(W.misw.p, 0, sizeof(int32_t) * kMisWords, s));
                    word = 0;
                }
                rflag = W.misw.p + word++;
                // lanes per row: about two to four entries per lane
#define BO_MIS_ROUND(G)                                                                                       \
    do {                                                                                                      \
        unsigned gb = grid_for((long long)n * G);                                                            \
        k_mis_m1<G><<<gb, kBlock, 0, s>>>(n, l, L.rp.p, L.ci.p, L.sf.p, state.p, m1.p);                      \
        k_mis_m2<G><<<gb, kBlock, 0, s>>>(n, l, L.rp.p, L.ci.p, L.sf.p, state.p, m1.p, nw.p);                \
        k_mis_spread<G><<<gb, kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, nw.p, d1.p);                        \
        k_mis_update<G><<<gb, kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, nw.p, d1.p, state.p, rflag);        \
    } while (0)
                double avg = (double)L.nnz / n;
                if (avg <= 10.0) BO_MIS_ROUND(1);
                else if (avg <= 20.0) BO_MIS_ROUND(4);
                else if (avg <= 40.0) BO_MIS_ROUND(8);
                else BO_MIS_ROUND(16);
#undef BO_MIS_ROUND
            }
            BO_HIP(hipGetLastError());
            int32_t any = 0;
            BO_TRY(read_flag(rflag, s, &any));  // the last round's word
            if (!any) break;
        }
        // aggregates
        DBuf<int32_t> &cnt = W.cnt, &id = W.id, &a1 = W.a1;
        BO_TRY(cnt.alloc(n)); BO_TRY(id.alloc(n + 1)); BO_TRY(a1.alloc(n));
        BO_TRY(L.root.alloc(n));
        BO_TRY(L.agg.alloc(n));
        k_is_root<<<grid_for(n), kBlock, 0, s>>>(n, state.p, cnt.p, L.root.p);
        int32_t nc = 0;
        BO_TRY(scan_counts(cnt.p, id.p, n, &nc, s));
        if (nc == 0 || (double)nc > 0.8 * (double)n) break;
        k_agg1<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, state.p, id.p, a1.p);
        k_agg2<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, state.p, a1.p, L.agg.p,
                                              W.dfl.p + 1);
        BO_HIP(hipGetLastError());
        L.nc = nc;
        if (l == 0) BO_TRY(fork());
        // prolongator
        DBuf<double> &aF = W.aF;
        DBuf<unsigned long long> &rho = W.rho;
        BO_TRY(aF.alloc(n)); BO_TRY(rho.alloc(kRedSlots));
        BO_HIP(hipMemsetAsync(rho.p, 0, sizeof(unsigned long long) * kRedSlots, s));
        k_filter<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p, L.sf.p, aF.p, rho.p);
        const double *omega = W.omg.p + l;
        BO_TRY(W.plong.alloc(n + 1));
        k_omega<<<1, 1, 0, s>>>(rho.p, W.omg.p + l, W.dfl.p + 2, W.plong.p);
        const bool kp8 = L.nnz <= 8LL * n;
        if (kp8) k_p_count<8><<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, L.agg.p, cnt.p, W.plong.p);
        else k_p_count<16><<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, L.agg.p, cnt.p, W.plong.p);
        // the listed long rows, a wavefront each up to 65536 of them
        const unsigned pgrid = (unsigned)std::min<long long>((n + kPWaves - 1) / kPWaves, 16384);
        k_p_long<<<pgrid, 64 * kPWaves, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, L.agg.p, aF.p, omega, nullptr,
                                                nullptr, nullptr, cnt.p, flag, W.plong.p);
        k_p_vlong<<<pgrid, 64 * kPWaves, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, L.agg.p, aF.p, omega, nullptr,
                                                 nullptr, nullptr, cnt.p, W.plong.p);
        BO_TRY(L.prp.alloc(n + 1));
        int32_t pnnz = 0;
        BO_TRY(scan_counts(cnt.p, L.prp.p, n, &pnnz, s));
        L.pnnz = pnnz;
        BO_TRY(L.pci.alloc(pnnz)); BO_TRY(L.pv.alloc(pnnz));
        if (kp8)
            k_p_fill<8><<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, L.agg.p, aF.p, omega,
                                                       L.prp.p, L.pci.p, L.pv.p);
        else
            k_p_fill<16><<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, L.agg.p, aF.p, omega,
                                                        L.prp.p, L.pci.p, L.pv.p);
        k_p_long<<<pgrid, 64 * kPWaves, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, L.agg.p, aF.p, omega, L.prp.p,
                                                L.pci.p, L.pv.p, nullptr, flag, W.plong.p);
        k_p_vlong<<<pgrid, 64 * kPWaves, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, L.agg.p, aF.p, omega, L.prp.p,
                                                 L.pci.p, L.pv.p, nullptr, W.plong.p);
        BO_HIP(hipGetLastError());
        // R = P^T
        // column counts and fill positions in one buffer (one clear); R has
        // P's nnz, so its row pointers need no read back
        DBuf<int32_t> &rc = W.rc;
        BO_TRY(rc.alloc(2 * (size_t)nc));
        int32_t *const rcnt = rc.p, *const fp = rc.p + nc;
        BO_HIP(hipMemsetAsync(rc.p, 0, sizeof(int32_t) * 2 * nc, s));
        k_col_counts<<<grid_for(pnnz), kBlock, 0, s>>>(pnnz, L.pci.p, rcnt);
        BO_TRY(L.rrp.alloc(nc + 1));
        BO_TRY(W.scan_sums.alloc(scan_sum_words(nc)));
        BO_TRY(scan_counts_async(rcnt, L.rrp.p, nc, W.scan_sums.p, s));
        BO_TRY(L.rci.alloc(pnnz)); BO_TRY(L.rv.alloc(pnnz));
        k_transpose_fill<<<grid_for(n), kBlock, 0, s>>>(n, L.prp.p, L.pci.p, L.pv.p, L.rrp.p, fp, L.rci.p, L.rv.p);
        k_sort_rows<<<grid_for((long long)nc * 64), kBlock, 0, s>>>(nc, L.rrp.p, L.rci.p, L.rv.p);
        BO_HIP(hipGetLastError());
        // A_c = R (A P)
        DBuf<int32_t> &aprp = W.aprp, &apci = W.apci;
        DBuf<double> &apv = W.apv;
        int apnnz = 0;
        BO_TRY(spgemm(n, L.rp.p, L.ci.p, L.v.p, L.prp.p, L.pci.p, L.pv.p, aprp, apci, apv, &apnnz, W, s,
                      (double)L.pnnz / n));
        Level &C = pc->lv[l + 1];
        C.n = nc;
        BO_TRY(spgemm(nc, L.rrp.p, L.rci.p, L.rv.p, aprp.p, apci.p, apv.p, C.rp, C.ci, C.v, &C.nnz, W, s,
                      (double)apnnz / n));
    }
    pc->nlev = l + 1;
    BO_TRY(fork());
    // sliced copies of the large matrices the cycle applies row by row
    const int sell_min = o.sell_rows > 0 ? o.sell_rows : kSellRows;
    for (int q = 0; q + 1 < pc->nlev; q++) {
        Level &L = pc->lv[q], &C = pc->lv[q + 1];
        // level 0 of a grid with extra rows: the cells' stencil entries with
        // implicit columns
        SellGrid sg{};
        if (q == 0 && pc->has_grid && pc->g.n() <= L.n) sg = SellGrid{(int)pc->g.n(), pc->g.nx, pc->g.ny, pc->g.nz};
        if (q > 0 || pc->general) BO_TRY(sell_from_csr(L.sA, L.n, L.rp.p, L.ci.p, L.v.p, sell_min, W.cnt, s, sg));
        else L.sA.on = false;
        BO_TRY(sell_from_csr(L.sP, L.n, L.prp.p, L.pci.p, L.pv.p, sell_min, W.cnt, s));
        BO_TRY(sell_from_csr(L.sR, C.n, L.rrp.p, L.rci.p, L.rv.p, sell_min, W.cnt, s));
    }
    // coarsest: dense inverse
    Level &Lc = pc->lv[l];
    int nc = Lc.n;
    if (nc > kCoarseMaxLimit)
        return fail(BO_ERR_UNSUPPORTED, "AMG: coarsening stalled above the dense coarse-solve limit (" +
                                            std::to_string(nc) + " rows)");
    pc->coarse_n = nc;
    DBuf<double> &M = W.dense;
    BO_TRY(M.alloc((size_t)nc * 2 * nc));
    BO_TRY(pc->cinv.alloc((size_t)nc * nc));
    k_dense_from_csr<<<grid_for(nc), kBlock, 0, s>>>(nc, Lc.rp.p, Lc.ci.p, Lc.v.p, M.p);
    BO_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    if (nc <= 128) {
        k_gj_regs<4><<<1, 1024, 0, s>>>(nc, M.p, pc->cinv.p, flag);
    } else if (nc <= 160) {
        k_gj_regs<5><<<1, 1024, 0, s>>>(nc, M.p, pc->cinv.p, flag);
    } else if (nc <= kGjRegMax) {
        k_gj_regs<6><<<1, 1024, 0, s>>>(nc, M.p, pc->cinv.p, flag);
    } else {
        k_gauss_jordan<<<1, 1024, 0, s>>>(nc, M.p, flag);
        k_extract_inverse<<<grid_for((long long)nc * nc), kBlock, 0, s>>>(nc, M.p, pc->cinv.p);
    }
    BO_HIP(hipGetLastError());
    int32_t bad = 0, dfl[4] = {0, 0, 0, 0};
    double omg[kMaxLevels] = {};
    HostRead rd[3] = {{flag, sizeof bad, &bad}, {W.dfl.p, sizeof dfl, dfl}, {W.omg.p, sizeof(double) * kMaxLevels, omg}};
    BO_TRY(host_reads(rd, pc->nlev > 1 ? 3 : 2, s));
    if (dfl[0]) return fail(BO_ERR_SINGULAR_COARSE, "AMG: zero or non-finite diagonal in the pressure hierarchy");
    if (dfl[1]) return fail(BO_ERR_HIP, "AMG: a node could not be aggregated");
    if (dfl[2]) return fail(BO_ERR_SINGULAR_COARSE, "AMG: bad smoother bound");
    if (dfl[3]) return fail(BO_ERR_HIP, "AMG: colour pairs of the level-0 sweep");
    if (bad) return fail(BO_ERR_SINGULAR_COARSE, "AMG: the coarsest matrix is singular");
    for (int q = 0; q + 1 < pc->nlev; q++) pc->lv[q].omega = omg[q];
    return BO_OK;
}

// ---- host: V-cycle -------------------------------------------------------------------
// the arrays a cycle in precision T works on
template <typename T> struct Prec;
template <> struct Prec<double> {
    static const double *v(const Level &L) { return L.v.p; }
    static const double *pv(const Level &L) { return L.pv.p; }
    static const double *rv(const Level &L) { return L.rv.p; }
    static double *x(Level &L) { return L.x.p; }
    static double *b(Level &L) { return L.b.p; }
    static double *r(Level &L) { return L.r.p; }
    static double *t(Level &L) { return L.t.p; }
    static const double *dl1(const Level &L) { return L.dl1.p; }
    static const double *app(const bo_cpr *pc) { return pc->app.p; }
    static const double *appc(const bo_cpr *pc) { return pc->appc.p; }
    static const double *cinv(const bo_cpr *pc) { return pc->cinv.p; }
};
template <> struct Prec<float> {
    static const float *v(const Level &L) { return L.v32.p; }
    static const float *pv(const Level &L) { return L.pv32.p; }
    static const float *rv(const Level &L) { return L.rv32.p; }
    static float *x(Level &L) { return L.x32.p; }
    static float *b(Level &L) { return L.b32.p; }
    static float *r(Level &L) { return L.r32.p; }
    static float *t(Level &L) { return L.t32.p; }
    static const float *dl1(const Level &L) { return L.dl132.p; }
    static const float *app(const bo_cpr *pc) { return pc->app32.p; }
    static const float *appc(const bo_cpr *pc) { return pc->appc32.p; }
    static const float *cinv(const bo_cpr *pc) { return pc->cinv32.p; }
};

// zero: x holds no guess (the cycle's pre-smoother); the Gauss-Seidel form
// then skips the neighbour reads of its first colour, the Jacobi form starts
// from a zeroed x
template <typename T>
static bo_status smooth0(bo_cpr *pc, const T *b, T *x, bool forward, bool zero, hipStream_t s) {
    const Grid &g = pc->g;
    long long n = pc->n;
    Level &L = pc->lv[0];
    const T *A = Prec<T>::app(pc);
    if (zero && pc->o.smoother != BO_SMOOTH_GS) k_zero<T><<<grid_for(n), kBlock, 0, s>>>(n, x);
    for (int sw = 0; sw < pc->o.sweeps; sw++) {
        if (pc->o.smoother == BO_SMOOTH_GS) {
            int c0 = forward ? 0 : 1;
            const T *Ac = Prec<T>::appc(pc);
            const long long H = (n + 1) / 2;
            k_gs_split<T><<<grid_for(H), kBlock, 0, s>>>(g.nx, g.ny, g.nz, Ac, b, x, c0, zero && sw == 0 ? 1 : 0);
            k_gs_split<T><<<grid_for(H), kBlock, 0, s>>>(g.nx, g.ny, g.nz, Ac, b, x, 1 - c0, 0);
        } else {
            T *t = Prec<T>::r(L);
            k_jacobi_slots<T><<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, A, b, x, t);
            BO_HIP(hipMemcpyAsync(x, t, sizeof(T) * n, hipMemcpyDeviceToDevice, s));
        }
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// coarse-level l1-Jacobi or damped Jacobi; `x` holds the guess (NULL: zero)
// and the result is returned in one of x / t
template <typename T>
static bo_status smooth_c(Level &L, int sweeps, bool l1, const T *b, T *x, T **res, hipStream_t s) {
    // a sweep reads its input at the neighbours, so it never writes in place:
    // the two level buffers alternate, starting from the one x is not
    T *cur = x, *oth = x == Prec<T>::t(L) ? Prec<T>::x(L) : Prec<T>::t(L);
    const T *d = Prec<T>::dl1(L);
    int first = 0;
    if (!x) {
        BO_TRY(csr_rowop<T>(L.n, L.nnz, L.rp.p, L.ci.p, Prec<T>::v(L), nullptr, l1 ? OP_L10 : OP_JACOBI0, b,
                            L.diagpos.p, Prec<T>::x(L), s, d));
        cur = Prec<T>::x(L);
        first = 1;
    }
    for (int sw = first; sw < sweeps; sw++) {
        BO_TRY(csr_rowop<T>(L.n, L.nnz, L.rp.p, L.ci.p, Prec<T>::v(L), cur, l1 ? OP_L1 : OP_JACOBI, b, L.diagpos.p,
                            oth, s, d, &L.sA));
        std::swap(cur, oth);
    }
    *res = cur;
    return BO_OK;
}

// levels up to this many rows take the fused zero-guess sweep and residual
constexpr int kFuseRows = 1 << 20;

// one V-cycle on level l for right-hand side b; returns the result pointer
template <typename T>
static bo_status vcycle_rec(bo_cpr *pc, int l, const T *b, T **res, hipStream_t s) {
    Level &L = pc->lv[l];
    if (l == pc->nlev - 1) {
        k_dense_mv<T><<<grid_for((long long)L.n * 64), kBlock, 0, s>>>(L.n, Prec<T>::cinv(pc), b, Prec<T>::x(L));
        BO_HIP(hipGetLastError());
        *res = Prec<T>::x(L);
        return BO_OK;
    }
    T *x;
    const bool slots0 = l == 0 && !pc->general;
    const bool l1 = l == 0 ? pc->o.smoother == BO_SMOOTH_L1 : pc->o.csmoother == BO_CSMOOTH_L1;
    if (slots0) {
        x = Prec<T>::x(L);
        BO_TRY(smooth0<T>(pc, b, x, true, true, s));
        k_resid_slots<T><<<grid_for(L.n), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, Prec<T>::app(pc), b, x,
                                                           Prec<T>::r(L));
    } else if (l1 && pc->o.sweeps == 1 && L.n <= kFuseRows) {
        // the one zero-guess sweep fused with the residual (on small levels,
        // where the launch it saves costs more than gathering b and d_l1
        // instead of x)
        x = Prec<T>::x(L);
        BO_TRY(csr_l1_resid<T>(L.n, L.nnz, L.rp.p, L.ci.p, Prec<T>::v(L), b, Prec<T>::dl1(L), x, Prec<T>::r(L), s));
    } else {
        BO_TRY(smooth_c<T>(L, pc->o.sweeps, l1, b, nullptr, &x, s));
        BO_TRY(csr_rowop<T>(L.n, L.nnz, L.rp.p, L.ci.p, Prec<T>::v(L), x, OP_RESID, b, nullptr, Prec<T>::r(L), s,
                            nullptr, &L.sA));
    }
    Level &C = pc->lv[l + 1];
    BO_TRY(csr_rowop<T>(C.n, L.pnnz, L.rrp.p, L.rci.p, Prec<T>::rv(L), Prec<T>::r(L), OP_MV, nullptr, nullptr,
                        Prec<T>::b(C), s, nullptr, &L.sR));
    T *xc;
    BO_TRY(vcycle_rec<T>(pc, l + 1, Prec<T>::b(C), &xc, s));
    BO_TRY(csr_rowop<T>(L.n, L.pnnz, L.prp.p, L.pci.p, Prec<T>::pv(L), xc, OP_ADD, nullptr, nullptr, x, s, nullptr,
                        &L.sP));
    if (slots0) {
        BO_TRY(smooth0<T>(pc, b, x, false, false, s));
        *res = x;
    } else {
        BO_TRY(smooth_c<T>(L, pc->o.sweeps, l1, b, x, res, s));
    }
    return BO_OK;
}

// one V-cycle for b; *res points at the result (a buffer of the hierarchy,
// valid until the next cycle)
bo_status amg_vcycle_ptr(bo_cpr *pc, const double *b, const double **res, hipStream_t s) {
    double *r;
    BO_TRY(vcycle_rec<double>(pc, 0, b, &r, s));
    *res = r;
    return BO_OK;
}

// mixed form: b is the FP32 right-hand side, the cycle runs in FP32
bo_status amg_vcycle_ptr_f32(bo_cpr *pc, const float *b, const float **res, hipStream_t s) {
    float *r;
    BO_TRY(vcycle_rec<float>(pc, 0, b, &r, s));
    *res = r;
    return BO_OK;
}

bo_status amg_vcycle(bo_cpr *pc, const double *b, double *x, hipStream_t s) {
    if (pc->o.precision != BO_PREC_FP64) {
        // FP64 in and out, FP32 inside: the stage boundaries of the mixed form
        Level &L0 = pc->lv[0];
        BO_TRY(to_f32(pc->npr, b, L0.b32.p, s));
        const float *res;
        BO_TRY(amg_vcycle_ptr_f32(pc, L0.b32.p, &res, s));
        k_f32_to_f64<<<grid_for(pc->npr), kBlock, 0, s>>>(pc->npr, res, x);
        BO_HIP(hipGetLastError());
        return BO_OK;
    }
    const double *res;
    BO_TRY(amg_vcycle_ptr(pc, b, &res, s));
    if (res != x) BO_HIP(hipMemcpyAsync(x, res, sizeof(double) * pc->npr, hipMemcpyDeviceToDevice, s));
    return BO_OK;
}

// FP32 copies of the hierarchy for the mixed form (the setup itself is FP64)
bo_status amg_make_f32(bo_cpr *pc, hipStream_t s) {
    if (!pc->general) {
        BO_TRY(pc->app32.alloc(7 * (size_t)pc->n));
        BO_TRY(to_f32(7 * (long long)pc->n, pc->app.p, pc->app32.p, s));
        if (pc->o.smoother == BO_SMOOTH_GS) {
            const long long words = 2 * NSLOT * (((long long)pc->n + 1) / 2);
            BO_TRY(pc->appc32.alloc(words));
            BO_TRY(to_f32(words, pc->appc.p, pc->appc32.p, s));
        }
    }
    for (int l = 0; l < pc->nlev; l++) {
        Level &L = pc->lv[l];
        const bool csr = l > 0 || pc->general;
        BO_TRY(L.x32.alloc(L.n)); BO_TRY(L.b32.alloc(L.n)); BO_TRY(L.r32.alloc(L.n)); BO_TRY(L.t32.alloc(L.n));
        if (csr) {
            BO_TRY(L.v32.alloc(L.nnz));
            BO_TRY(to_f32(L.nnz, L.v.p, L.v32.p, s));
        }
        if (csr && l + 1 < pc->nlev) {
            BO_TRY(L.dl132.alloc(L.n));
            BO_TRY(to_f32(L.n, L.dl1.p, L.dl132.p, s));
        }
        for (SellMat *M : {&L.sA, &L.sP, &L.sR})
            if (M->on) {
                BO_TRY(M->val32.alloc(M->len));
                BO_TRY(to_f32(M->len, M->val.p, M->val32.p, s));
            }
        if (l + 1 < pc->nlev) {
            BO_TRY(L.pv32.alloc(L.pnnz)); BO_TRY(L.rv32.alloc(L.pnnz));
            BO_TRY(to_f32(L.pnnz, L.pv.p, L.pv32.p, s));
            BO_TRY(to_f32(L.pnnz, L.rv.p, L.rv32.p, s));
        }
    }
    BO_TRY(pc->cinv32.alloc((size_t)pc->coarse_n * pc->coarse_n));
    BO_TRY(to_f32((long long)pc->coarse_n * pc->coarse_n, pc->cinv.p, pc->cinv32.p, s));
    return BO_OK;
}

}  // namespace bo
