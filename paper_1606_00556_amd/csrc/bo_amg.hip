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
__global__ void k_qi_restrict(long long n, const double *__restrict__ cw, const double *__restrict__ v,
                              double *__restrict__ rp) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    rp[i] = cw[3 * i] * v[3 * i] + cw[3 * i + 1] * v[3 * i + 1] + cw[3 * i + 2] * v[3 * i + 2];
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

__global__ void k_diag(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                       const double *__restrict__ v, int32_t *__restrict__ dpos, double *__restrict__ dinv,
                       int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int p = find_col(ci, rp[i], rp[i + 1], i);
    dpos[i] = p;
    double d = p >= 0 ? v[p] : 0.0;
    if (d == 0.0 || !isfinite(d)) *bad = 1;
    dinv[i] = d != 0.0 ? 1.0 / d : 0.0;
}

__global__ void k_strength(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, const int32_t *__restrict__ dpos, double t2,
                           uint8_t *__restrict__ sf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double aii = dpos[i] >= 0 ? v[dpos[i]] : 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
        int j = ci[e];
        if (j == i) { sf[e] = 0; continue; }
        double ajj = dpos[j] >= 0 ? v[dpos[j]] : 0.0;
        int q = find_col(ci, rp[j], rp[j + 1], i);
        double aij = v[e], aji = q >= 0 ? v[q] : 0.0;
        double thr = t2 * fabs(aii * ajj);
        sf[e] = (aij * aij >= thr) || (aji * aji >= thr);
    }
}

enum { UND = 0, IN = 1, OUT = 2, ISO = 3 };

__global__ void k_mis_init(int n, const int32_t *__restrict__ rp, const uint8_t *__restrict__ sf,
                           uint8_t *__restrict__ state) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int deg = 0;
    for (int e = rp[i]; e < rp[i + 1]; e++) deg += sf[e];
    state[i] = deg ? UND : ISO;
}

__global__ void k_mis_m1(int n, int level, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const uint8_t *__restrict__ sf, const uint8_t *__restrict__ state,
                         uint64_t *__restrict__ m1) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t m = state[i] == UND ? prio(i, level) : 0ull;
    for (int e = rp[i]; e < rp[i + 1]; e++)
        if (sf[e] && state[ci[e]] == UND) {
            uint64_t q = prio(ci[e], level);
            if (q > m) m = q;
        }
    m1[i] = m;
}

__global__ void k_mis_m2(int n, int level, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const uint8_t *__restrict__ sf, const uint8_t *__restrict__ state,
                         const uint64_t *__restrict__ m1, uint8_t *__restrict__ nw) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t m = m1[i];
    for (int e = rp[i]; e < rp[i + 1]; e++)
        if (sf[e] && m1[ci[e]] > m) m = m1[ci[e]];
    nw[i] = state[i] == UND && m == prio(i, level);
}

__global__ void k_mis_spread(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const uint8_t *__restrict__ sf, const uint8_t *__restrict__ in,
                             uint8_t *__restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint8_t d = in[i];
    for (int e = rp[i]; e < rp[i + 1]; e++)
        if (sf[e]) d |= in[ci[e]];
    out[i] = d;
}

__global__ void k_mis_update(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const uint8_t *__restrict__ sf, const uint8_t *__restrict__ nw,
                             const uint8_t *__restrict__ d1, uint8_t *__restrict__ state,
                             int32_t *__restrict__ any) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint8_t d = d1[i];
    for (int e = rp[i]; e < rp[i + 1]; e++)
        if (sf[e]) d |= d1[ci[e]];
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
    if (state[i] == IN) a = id[i];
    else
        for (int e = rp[i]; e < rp[i + 1]; e++)
            if (sf[e] && state[ci[e]] == IN) a = id[ci[e]];
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
        for (int e = rp[i]; e < rp[i + 1]; e++) {
            int j = ci[e];
            if (!sf[e] || a1[j] < 0) continue;
            double x = fabs(v[e]);
            if (x > bv || (x == bv && a1[j] < best)) { bv = x; best = a1[j]; }
        }
        a = best;
        if (a < 0) *bad = 1;
    }
    agg[i] = a;
}

// filtered diagonal and the Gershgorin ratio of D_F^{-1} A_F (max via the
// order-preserving bit pattern of non-negative doubles)
__global__ void k_filter(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ v, const int32_t *__restrict__ dpos,
                         const uint8_t *__restrict__ sf, double *__restrict__ aF,
                         unsigned long long *__restrict__ rho_bits) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double aii = v[dpos[i]];
    double d = aii;
    for (int e = rp[i]; e < rp[i + 1]; e++)
        if (ci[e] != i && !sf[e]) d = d + v[e];
    if (d == 0.0) d = aii;
    aF[i] = d;
    double rs = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
        if (ci[e] == i) rs = rs + fabs(d);
        else if (sf[e]) rs = rs + fabs(v[e]);
    }
    double ratio = rs / fabs(d);
    atomicMax(rho_bits, (unsigned long long)__double_as_longlong(ratio));
}

__device__ __forceinline__ bool p_takes(int e, int i, const int32_t *ci, const uint8_t *sf, const int32_t *agg) {
    int j = ci[e];
    return (j == i || sf[e]) && agg[j] >= 0;
}

__global__ void k_p_count(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                          const uint8_t *__restrict__ sf, const int32_t *__restrict__ agg,
                          int32_t *__restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int e = rp[i]; e < rp[i + 1]; e++) {
        if (!p_takes(e, i, ci, sf, agg)) continue;
        int J = agg[ci[e]];
        bool first = true;
        for (int f = rp[i]; f < e; f++)
            if (p_takes(f, i, ci, sf, agg) && agg[ci[f]] == J) { first = false; break; }
        c += first;
    }
    cnt[i] = c;
}

// P row i: entries for each distinct aggregate J among {i} and its strong
// neighbours, (agg(i)==J) - omega/aF_ii * sum_{agg(j)=J} aF_ij (sums in
// ascending j), then sorted by J.
__global__ void k_p_fill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ v, const uint8_t *__restrict__ sf,
                         const int32_t *__restrict__ agg, const double *__restrict__ aF, double omega,
                         const int32_t *__restrict__ prp, int32_t *__restrict__ pci, double *__restrict__ pv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = omega / aF[i];
    int pos = prp[i];
    for (int e = rp[i]; e < rp[i + 1]; e++) {
        if (!p_takes(e, i, ci, sf, agg)) continue;
        int J = agg[ci[e]];
        bool first = true;
        for (int f = rp[i]; f < e; f++)
            if (p_takes(f, i, ci, sf, agg) && agg[ci[f]] == J) { first = false; break; }
        if (!first) continue;
        double s = 0.0;
        for (int f = e; f < rp[i + 1]; f++)
            if (p_takes(f, i, ci, sf, agg) && agg[ci[f]] == J) s = s + (ci[f] == i ? aF[i] : v[f]);
        pci[pos] = J;
        pv[pos] = (agg[i] == J ? 1.0 : 0.0) - d * s;
        pos++;
    }
    // insertion sort of the row by column
    int b = prp[i], end = prp[i + 1];
    for (int a = b + 1; a < end; a++) {
        int c = pci[a];
        double x = pv[a];
        int q = a - 1;
        while (q >= b && pci[q] > c) { pci[q + 1] = pci[q]; pv[q + 1] = pv[q]; q--; }
        pci[q + 1] = c;
        pv[q + 1] = x;
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

__global__ void k_sort_rows(int n, const int32_t *__restrict__ rp, int32_t *__restrict__ ci, double *__restrict__ v) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int b = rp[i], end = rp[i + 1];
    for (int a = b + 1; a < end; a++) {
        int c = ci[a];
        double x = v[a];
        int q = a - 1;
        while (q >= b && ci[q] > c) { ci[q + 1] = ci[q]; v[q + 1] = v[q]; q--; }
        ci[q + 1] = c;
        v[q + 1] = x;
    }
}

// ---- row-wise sparse product C = A B ----------------------------------------------
constexpr int kHash = 2048;            // LDS hash slots per wavefront
constexpr int kWavesPerGroup = 4;

__device__ __forceinline__ unsigned hash_col(int c) { return ((unsigned)c * 2654435761u) & (kHash - 1); }

// inserts the column set of row i of A*B into the wave's hash; returns the count
__device__ int gather_cols(int i, const int32_t *arp, const int32_t *aci, const int32_t *brp, const int32_t *bci,
                           int *tab, int *count, int lane) {
    for (int e = arp[i]; e < arp[i + 1]; e++) {
        int k = aci[e];
        for (int f = brp[k] + lane; f < brp[k + 1]; f += 64) {
            int c = bci[f];
            unsigned h = hash_col(c);
            for (int probe = 0; probe < kHash; probe++) {
                int old = atomicCAS(&tab[h], -1, c);
                if (old == -1) { atomicAdd(count, 1); break; }
                if (old == c) break;
                h = (h + 1) & (kHash - 1);
            }
        }
    }
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    return *count;
}

__global__ void __launch_bounds__(64 * kWavesPerGroup) k_spgemm_count(int n, const int32_t *__restrict__ arp,
                                                                       const int32_t *__restrict__ aci,
                                                                       const int32_t *__restrict__ brp,
                                                                       const int32_t *__restrict__ bci,
                                                                       int32_t *__restrict__ cnt,
                                                                       int32_t *__restrict__ bad) {
    __shared__ int tab[kWavesPerGroup][kHash];
    __shared__ int count[kWavesPerGroup];
    int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    int i = blockIdx.x * kWavesPerGroup + wave;
    for (int t = lane; t < kHash; t += 64) tab[wave][t] = -1;
    if (lane == 0) count[wave] = 0;
    __syncthreads();
    if (i < n) {
        int c = gather_cols(i, arp, aci, brp, bci, tab[wave], &count[wave], lane);
        if (lane == 0) {
            cnt[i] = c;
            if (c > kHash / 2) *bad = 1;
        }
    }
}

__global__ void __launch_bounds__(64 * kWavesPerGroup) k_spgemm_fill(int n, const int32_t *__restrict__ arp,
                                                                      const int32_t *__restrict__ aci,
                                                                      const double *__restrict__ av,
                                                                      const int32_t *__restrict__ brp,
                                                                      const int32_t *__restrict__ bci,
                                                                      const double *__restrict__ bv,
                                                                      const int32_t *__restrict__ crp,
                                                                      int32_t *__restrict__ cci,
                                                                      double *__restrict__ cv) {
    __shared__ int tab[kWavesPerGroup][kHash];
    __shared__ int count[kWavesPerGroup];
    int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    int i = blockIdx.x * kWavesPerGroup + wave;
    for (int t = lane; t < kHash; t += 64) tab[wave][t] = -1;
    if (lane == 0) count[wave] = 0;
    __syncthreads();
    if (i >= n) return;
    int total = gather_cols(i, arp, aci, brp, bci, tab[wave], &count[wave], lane);
    int base = crp[i];
    // rank of each distinct column = number of distinct columns below it
    for (int t = lane; t < kHash; t += 64) {
        int c = tab[wave][t];
        if (c < 0) continue;
        int rank = 0;
        for (int u = 0; u < kHash; u++) {
            int d = tab[wave][u];
            rank += (d >= 0 && d < c);
        }
        // value: sum over the row of A in ascending order
        double s = 0.0;
        for (int e = arp[i]; e < arp[i + 1]; e++) {
            int k = aci[e];
            int q = find_col(bci, brp[k], brp[k + 1], c);
            if (q >= 0) s = s + av[e] * bv[q];
        }
        cci[base + rank] = c;
        cv[base + rank] = s;
    }
    (void)total;
}

// ---- coarsest level: dense inverse ---------------------------------------------------
__global__ void k_dense_from_csr(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                 const double *__restrict__ v, double *__restrict__ M) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int c = 0; c < 2 * n; c++) M[(size_t)i * 2 * n + c] = (c == n + i) ? 1.0 : 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) M[(size_t)i * 2 * n + ci[e]] = v[e];
}

// Gauss-Jordan with partial pivoting on [A | I] (n x 2n, row-major), one
// workgroup; leaves A^{-1} in the right half.
__global__ void __launch_bounds__(1024) k_gauss_jordan(int n, double *__restrict__ M, int32_t *__restrict__ bad) {
    __shared__ double bestv[1024];
    __shared__ int besti[1024];
    __shared__ int piv;
    __shared__ double pivval;
    int t = threadIdx.x, w = 2 * n;
    for (int k = 0; k < n; k++) {
        double bv = -1.0;
        int bi = n;
        for (int r = k + t; r < n; r += blockDim.x) {
            double a = fabs(M[(size_t)r * w + k]);
            if (a > bv || (a == bv && r < bi)) { bv = a; bi = r; }
        }
        bestv[t] = bv;
        besti[t] = bi;
        __syncthreads();
        for (int s = blockDim.x / 2; s > 0; s >>= 1) {
            if (t < s) {
                double o = bestv[t + s];
                int oi = besti[t + s];
                if (o > bestv[t] || (o == bestv[t] && oi < besti[t])) { bestv[t] = o; besti[t] = oi; }
            }
            __syncthreads();
        }
        if (t == 0) {
            piv = besti[0];
            if (!(bestv[0] > 0.0)) *bad = 1;
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
        if (t == 0) pivval = M[(size_t)k * w + k];
        __syncthreads();
        double d = pivval;
        for (int c = t; c < w; c += blockDim.x) M[(size_t)k * w + c] = M[(size_t)k * w + c] / d;
        __syncthreads();
        for (int idx = t; idx < n * w; idx += blockDim.x) {
            int r = idx / w, c = idx % w;
            if (r == k) continue;
            double f = M[(size_t)r * w + k];
            if (c == k) continue;
            M[(size_t)idx] = M[(size_t)idx] - f * M[(size_t)k * w + c];
        }
        __syncthreads();
        for (int r = t; r < n; r += blockDim.x)
            if (r != k) M[(size_t)r * w + k] = 0.0;
        __syncthreads();
    }
}

__global__ void k_extract_inverse(int n, const double *__restrict__ M, double *__restrict__ inv) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= n * n) return;
    int r = idx / n, c = idx % n;
    inv[idx] = M[(size_t)r * 2 * n + n + c];
}

// ---- cycle kernels -------------------------------------------------------------------
// level 0 on the grid (slot form), colour c of red-black Gauss-Seidel
__global__ void __launch_bounds__(kBlock) k_gs_slots(int nx, int ny, int nz, const double *__restrict__ A,
                                                     const double *__restrict__ b, double *__restrict__ x, int colour) {
    int n = nx * ny * nz;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    if (((ix + iy + iz) & 1) != colour) return;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    size_t N = (size_t)n;
    double s = b[i], d = 0.0;
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        int j = nb[q];
        if (j < 0) continue;
        double a = A[(size_t)q * N + i];
        if (q == S_D) d = a;
        else s = s - a * x[j];
    }
    x[i] = s / d;
}

// level 0 damped Jacobi sweep (slot form): xo = xi + (2/3) (b - A xi) / a_ii
__global__ void __launch_bounds__(kBlock) k_jacobi_slots(int nx, int ny, int nz, const double *__restrict__ A,
                                                         const double *__restrict__ b, const double *__restrict__ xi,
                                                         double *__restrict__ xo) {
    int n = nx * ny * nz;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    size_t N = (size_t)n;
    double s = 0.0, d = 0.0;
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        int j = nb[q];
        if (j < 0) continue;
        double a = A[(size_t)q * N + i];
        s = s + a * xi[j];
        if (q == S_D) d = a;
    }
    xo[i] = xi[i] + (2.0 / 3.0) * ((b[i] - s) / d);
}

// r = b - A x (slot form)
__global__ void __launch_bounds__(kBlock) k_resid_slots(int nx, int ny, int nz, const double *__restrict__ A,
                                                        const double *__restrict__ b, const double *__restrict__ x,
                                                        double *__restrict__ r) {
    int n = nx * ny * nz;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    size_t N = (size_t)n;
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        int j = nb[q];
        if (j < 0) continue;
        s = s + A[(size_t)q * N + i] * x[j];
    }
    r[i] = b[i] - s;
}

// CSR: damped Jacobi sweep xo = xi + (2/3) (b - A xi) / a_ii
__global__ void k_jacobi_csr(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                             const double *__restrict__ v, const int32_t *__restrict__ dpos,
                             const double *__restrict__ b, const double *__restrict__ xi, double *__restrict__ xo) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) s = s + v[e] * xi[ci[e]];
    double d = v[dpos[i]];
    xo[i] = xi[i] + (2.0 / 3.0) * ((b[i] - s) / d);
}

// CSR: r = b - A x
__global__ void k_resid_csr(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            const double *__restrict__ v, const double *__restrict__ b,
                            const double *__restrict__ x, double *__restrict__ r) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) s = s + v[e] * x[ci[e]];
    r[i] = b[i] - s;
}

// CSR: y = A x
__global__ void k_mv_csr(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                         const double *__restrict__ v, const double *__restrict__ x, double *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) s = s + v[e] * x[ci[e]];
    y[i] = s;
}

// CSR: x = x + P xc
__global__ void k_prolong_add(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              const double *__restrict__ v, const double *__restrict__ xc, double *__restrict__ x) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int e = rp[i]; e < rp[i + 1]; e++) s = s + v[e] * xc[ci[e]];
    x[i] = x[i] + s;
}

// dense y = M x (n <= 1024), one row per thread
__global__ void k_dense_mv(int n, const double *__restrict__ M, const double *__restrict__ x, double *__restrict__ y) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int c = 0; c < n; c++) s = s + M[(size_t)i * n + c] * x[c];
    y[i] = s;
}

bo_status read_flag(int32_t *dflag, hipStream_t s, int32_t *out) {
    BO_HIP(hipMemcpyAsync(out, dflag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}

}  // namespace

// ---- host: decoupling -------------------------------------------------------------
bo_status qi_decouple(bo_cpr *pc, hipStream_t s) {
    long long n = pc->n;
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
    long long n = pc->n;
    k_qi_restrict<<<grid_for(n), kBlock, 0, s>>>(n, pc->cw.p, v, rp);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// ---- host: hierarchy ---------------------------------------------------------------
static bo_status level_diag(Level &L, int32_t *flag, hipStream_t s) {
    BO_TRY(L.diagpos.alloc(L.n));
    BO_TRY(L.dinv.alloc(L.n));
    BO_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    k_diag<<<grid_for(L.n), kBlock, 0, s>>>(L.n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p, L.dinv.p, flag);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    BO_TRY(read_flag(flag, s, &bad));
    if (bad) return fail(BO_ERR_SINGULAR_COARSE, "AMG: zero or non-finite diagonal in the pressure hierarchy");
    return BO_OK;
}

static bo_status spgemm(int n, const int32_t *arp, const int32_t *aci, const double *av, const int32_t *brp,
                        const int32_t *bci, const double *bv, DBuf<int32_t> &crp, DBuf<int32_t> &cci,
                        DBuf<double> &cv, int *cnnz, int32_t *flag, hipStream_t s) {
    DBuf<int32_t> cnt;
    BO_TRY(cnt.alloc(n));
    BO_TRY(crp.alloc(n + 1));
    BO_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    unsigned groups = (unsigned)((n + kWavesPerGroup - 1) / kWavesPerGroup);
    k_spgemm_count<<<groups, 64 * kWavesPerGroup, 0, s>>>(n, arp, aci, brp, bci, cnt.p, flag);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    BO_TRY(read_flag(flag, s, &bad));
    if (bad) return fail(BO_ERR_UNSUPPORTED, "AMG: Galerkin product row exceeds the LDS hash capacity");
    int32_t total = 0;
    BO_TRY(scan_counts(cnt.p, crp.p, n, &total, s));
    BO_TRY(cci.alloc(total));
    BO_TRY(cv.alloc(total));
    k_spgemm_fill<<<groups, 64 * kWavesPerGroup, 0, s>>>(n, arp, aci, av, brp, bci, bv, crp.p, cci.p, cv.p);
    BO_HIP(hipGetLastError());
    BO_HIP(hipStreamSynchronize(s));
    *cnnz = total;
    return BO_OK;
}

bo_status amg_setup(bo_cpr *pc, hipStream_t s) {
    const bo_cpr_opts &o = pc->o;
    int32_t *flag = pc->flag.p;
    // level 0: CSR with the stencil pattern
    Level &L0 = pc->lv[0];
    L0.n = pc->n;
    {
        DBuf<int32_t> cnt;
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
    int l = 0;
    for (;; l++) {
        Level &L = pc->lv[l];
        BO_TRY(level_diag(L, flag, s));
        BO_TRY(L.x.alloc(L.n));
        BO_TRY(L.b.alloc(L.n));
        BO_TRY(L.r.alloc(L.n));
        if (L.n <= o.coarse_max || l + 1 >= max_levels) break;
        int n = L.n;
        BO_TRY(L.sf.alloc(L.nnz));
        k_strength<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p, t2, L.sf.p);
        // MIS-2
        DBuf<uint8_t> state, nw, d1;
        DBuf<uint64_t> m1;
        BO_TRY(state.alloc(n)); BO_TRY(nw.alloc(n)); BO_TRY(d1.alloc(n)); BO_TRY(m1.alloc(n));
        k_mis_init<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.sf.p, state.p);
        for (int round = 0;; round++) {
            if (round > 10000) return fail(BO_ERR_HIP, "AMG: MIS-2 did not terminate");
            BO_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
            k_mis_m1<<<grid_for(n), kBlock, 0, s>>>(n, l, L.rp.p, L.ci.p, L.sf.p, state.p, m1.p);
            k_mis_m2<<<grid_for(n), kBlock, 0, s>>>(n, l, L.rp.p, L.ci.p, L.sf.p, state.p, m1.p, nw.p);
            k_mis_spread<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, nw.p, d1.p);
            k_mis_update<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, nw.p, d1.p, state.p, flag);
            BO_HIP(hipGetLastError());
            int32_t any = 0;
            BO_TRY(read_flag(flag, s, &any));
            if (!any) break;
        }
        // aggregates
        DBuf<int32_t> cnt, id, a1;
        BO_TRY(cnt.alloc(n)); BO_TRY(id.alloc(n + 1)); BO_TRY(a1.alloc(n));
        BO_TRY(L.root.alloc(n));
        BO_TRY(L.agg.alloc(n));
        k_is_root<<<grid_for(n), kBlock, 0, s>>>(n, state.p, cnt.p, L.root.p);
        int32_t nc = 0;
        BO_TRY(scan_counts(cnt.p, id.p, n, &nc, s));
        if (nc == 0 || (double)nc > 0.8 * (double)n) break;
        k_agg1<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, state.p, id.p, a1.p);
        BO_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
        k_agg2<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, state.p, a1.p, L.agg.p, flag);
        BO_HIP(hipGetLastError());
        int32_t bad = 0;
        BO_TRY(read_flag(flag, s, &bad));
        if (bad) return fail(BO_ERR_HIP, "AMG: a node could not be aggregated");
        L.nc = nc;
        // prolongator
        DBuf<double> aF;
        DBuf<unsigned long long> rho;
        BO_TRY(aF.alloc(n)); BO_TRY(rho.alloc(1));
        BO_HIP(hipMemsetAsync(rho.p, 0, sizeof(unsigned long long), s));
        k_filter<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p, L.sf.p, aF.p, rho.p);
        unsigned long long rb = 0;
        BO_HIP(hipMemcpyAsync(&rb, rho.p, sizeof rb, hipMemcpyDeviceToHost, s));
        BO_HIP(hipStreamSynchronize(s));
        double rhov;
        std::memcpy(&rhov, &rb, sizeof rhov);
        if (!(rhov > 0.0) || !(rhov < INFINITY)) return fail(BO_ERR_SINGULAR_COARSE, "AMG: bad smoother bound");
        L.omega = (4.0 / 3.0) / rhov;
        k_p_count<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.sf.p, L.agg.p, cnt.p);
        BO_TRY(L.prp.alloc(n + 1));
        int32_t pnnz = 0;
        BO_TRY(scan_counts(cnt.p, L.prp.p, n, &pnnz, s));
        L.pnnz = pnnz;
        BO_TRY(L.pci.alloc(pnnz)); BO_TRY(L.pv.alloc(pnnz));
        k_p_fill<<<grid_for(n), kBlock, 0, s>>>(n, L.rp.p, L.ci.p, L.v.p, L.sf.p, L.agg.p, aF.p, L.omega,
                                                L.prp.p, L.pci.p, L.pv.p);
        BO_HIP(hipGetLastError());
        // R = P^T
        DBuf<int32_t> rc, fp;
        BO_TRY(rc.alloc(nc)); BO_TRY(fp.alloc(nc));
        BO_HIP(hipMemsetAsync(rc.p, 0, sizeof(int32_t) * nc, s));
        BO_HIP(hipMemsetAsync(fp.p, 0, sizeof(int32_t) * nc, s));
        k_col_counts<<<grid_for(pnnz), kBlock, 0, s>>>(pnnz, L.pci.p, rc.p);
        BO_TRY(L.rrp.alloc(nc + 1));
        int32_t rn = 0;
        BO_TRY(scan_counts(rc.p, L.rrp.p, nc, &rn, s));
        BO_TRY(L.rci.alloc(pnnz)); BO_TRY(L.rv.alloc(pnnz));
        k_transpose_fill<<<grid_for(n), kBlock, 0, s>>>(n, L.prp.p, L.pci.p, L.pv.p, L.rrp.p, fp.p, L.rci.p, L.rv.p);
        k_sort_rows<<<grid_for(nc), kBlock, 0, s>>>(nc, L.rrp.p, L.rci.p, L.rv.p);
        BO_HIP(hipGetLastError());
        // A_c = R (A P)
        DBuf<int32_t> aprp, apci;
        DBuf<double> apv;
        int apnnz = 0;
        BO_TRY(spgemm(n, L.rp.p, L.ci.p, L.v.p, L.prp.p, L.pci.p, L.pv.p, aprp, apci, apv, &apnnz, flag, s));
        Level &C = pc->lv[l + 1];
        C.n = nc;
        BO_TRY(spgemm(nc, L.rrp.p, L.rci.p, L.rv.p, aprp.p, apci.p, apv.p, C.rp, C.ci, C.v, &C.nnz, flag, s));
        BO_HIP(hipStreamSynchronize(s));
    }
    pc->nlev = l + 1;
    // coarsest: dense inverse
    Level &Lc = pc->lv[l];
    int nc = Lc.n;
    if (nc > kCoarseMaxLimit)
        return fail(BO_ERR_UNSUPPORTED, "AMG: coarsening stalled above the dense coarse-solve limit (" +
                                            std::to_string(nc) + " rows)");
    pc->coarse_n = nc;
    DBuf<double> M;
    BO_TRY(M.alloc((size_t)nc * 2 * nc));
    BO_TRY(pc->cinv.alloc((size_t)nc * nc));
    k_dense_from_csr<<<grid_for(nc), kBlock, 0, s>>>(nc, Lc.rp.p, Lc.ci.p, Lc.v.p, M.p);
    BO_HIP(hipMemsetAsync(flag, 0, sizeof(int32_t), s));
    k_gauss_jordan<<<1, 1024, 0, s>>>(nc, M.p, flag);
    k_extract_inverse<<<grid_for((long long)nc * nc), kBlock, 0, s>>>(nc, M.p, pc->cinv.p);
    BO_HIP(hipGetLastError());
    int32_t bad = 0;
    BO_TRY(read_flag(flag, s, &bad));
    if (bad) return fail(BO_ERR_SINGULAR_COARSE, "AMG: the coarsest matrix is singular");
    return BO_OK;
}

// ---- host: V-cycle -------------------------------------------------------------------
static bo_status smooth0(bo_cpr *pc, const double *b, double *x, bool forward, hipStream_t s) {
    const Grid &g = pc->g;
    long long n = pc->n;
    Level &L = pc->lv[0];
    for (int sw = 0; sw < pc->o.sweeps; sw++) {
        if (pc->o.smoother == BO_SMOOTH_GS) {
            int c0 = forward ? 0 : 1;
            k_gs_slots<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, pc->app.p, b, x, c0);
            k_gs_slots<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, pc->app.p, b, x, 1 - c0);
        } else {
            k_jacobi_slots<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, pc->app.p, b, x, L.r.p);
            BO_HIP(hipMemcpyAsync(x, L.r.p, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        }
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

static bo_status smooth_c(Level &L, int sweeps, const double *b, double *x, hipStream_t s) {
    for (int sw = 0; sw < sweeps; sw++) {
        k_jacobi_csr<<<grid_for(L.n), kBlock, 0, s>>>(L.n, L.rp.p, L.ci.p, L.v.p, L.diagpos.p, b, x, L.r.p);
        BO_HIP(hipMemcpyAsync(x, L.r.p, sizeof(double) * L.n, hipMemcpyDeviceToDevice, s));
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

static bo_status vcycle_rec(bo_cpr *pc, int l, const double *b, double *x, hipStream_t s) {
    Level &L = pc->lv[l];
    if (l == pc->nlev - 1) {
        k_dense_mv<<<grid_for(L.n), kBlock, 0, s>>>(L.n, pc->cinv.p, b, x);
        BO_HIP(hipGetLastError());
        return BO_OK;
    }
    BO_TRY(fill(L.n, 0.0, x, s));
    if (l == 0) BO_TRY(smooth0(pc, b, x, true, s));
    else BO_TRY(smooth_c(L, pc->o.sweeps, b, x, s));
    if (l == 0)
        k_resid_slots<<<grid_for(L.n), kBlock, 0, s>>>(pc->g.nx, pc->g.ny, pc->g.nz, pc->app.p, b, x, L.r.p);
    else
        k_resid_csr<<<grid_for(L.n), kBlock, 0, s>>>(L.n, L.rp.p, L.ci.p, L.v.p, b, x, L.r.p);
    Level &C = pc->lv[l + 1];
    k_mv_csr<<<grid_for(C.n), kBlock, 0, s>>>(C.n, L.rrp.p, L.rci.p, L.rv.p, L.r.p, C.b.p);
    BO_HIP(hipGetLastError());
    BO_TRY(vcycle_rec(pc, l + 1, C.b.p, C.x.p, s));
    k_prolong_add<<<grid_for(L.n), kBlock, 0, s>>>(L.n, L.prp.p, L.pci.p, L.pv.p, C.x.p, x);
    BO_HIP(hipGetLastError());
    if (l == 0) BO_TRY(smooth0(pc, b, x, false, s));
    else BO_TRY(smooth_c(L, pc->o.sweeps, b, x, s));
    return BO_OK;
}

bo_status amg_vcycle(bo_cpr *pc, const double *b, double *x, hipStream_t s) {
    return vcycle_rec(pc, 0, b, x, s);
}

}  // namespace bo
