// Basic operations of Section 3.3 (data structures and algorithms) on the GPU: y = alpha A x + beta y (BSR and
// the library's slot layout), y = alpha x + beta y, dot products and norms,
// plus the prefix sums the setup phases need.
//
// Slot layout of a 7-point 3x3-block matrix: val[(s*9 + e)*N + i] holds entry
// e (row-major in the block) of the block of row i in slot s (-z,-y,-x,diag,
// +x,+y,+z).  Consecutive threads own consecutive rows, so every one of the 63
// value streams is read fully coalesced; blocks outside the grid are zero and
// are skipped.
//
// Reductions are deterministic: a fixed grid of workgroups writes per-group
// partial sums in a fixed tree order, and a second one-workgroup kernel adds
// the partials in a fixed order (no device-scope fences in the hot loop).
#include <algorithm>
#include "bo_common.hpp"
#include <cstring>
#include "bo_linalg.hpp"

namespace bo {

static thread_local std::string g_err = "no error";
thread_local const bo_allocator *t_alloc = nullptr;
thread_local void *t_alloc_stream = nullptr;

void set_error(const std::string &msg) { g_err = msg; }
bo_status fail(bo_status st, const std::string &msg) {
    g_err = msg;
    return st;
}

bo_status scratch_get(int slot, size_t bytes, void **ptr) {
    static thread_local void *buf[SC_COUNT] = {};
    static thread_local size_t cap[SC_COUNT] = {};
    if (slot < 0 || slot >= SC_COUNT) return fail(BO_ERR_INVALID_ARG, "scratch slot");
    if (bytes > cap[slot]) {
        if (buf[slot]) (void)hipFree(buf[slot]);
        buf[slot] = nullptr;
        cap[slot] = 0;
        size_t want = std::max<size_t>(bytes, 4096);
        hipError_t e = hipMalloc(&buf[slot], want);
        if (e != hipSuccess)
            return fail(BO_ERR_ALLOC, std::string("scratch hipMalloc failed: ") + hipGetErrorString(e));
        cap[slot] = want;
    }
    *ptr = buf[slot];
    return BO_OK;
}

bo_status host_reads(const HostRead *r, int count, hipStream_t s) {
    constexpr size_t kMail = 4096;
    static thread_local char *mail = nullptr;
    if (!mail) {
        hipError_t e = hipHostMalloc((void **)&mail, kMail, hipHostMallocDefault);
        if (e != hipSuccess) {
            mail = nullptr;
            return fail(BO_ERR_ALLOC, std::string("hipHostMalloc of the read buffer failed: ") + hipGetErrorString(e));
        }
    }
    size_t off = 0;
    for (int q = 0; q < count; q++) {
        if (off + r[q].bytes > kMail) return fail(BO_ERR_INVALID_ARG, "host_reads: more than 4 KB");
        BO_HIP(hipMemcpyAsync(mail + off, r[q].src, r[q].bytes, hipMemcpyDeviceToHost, s));
        off += (r[q].bytes + 15) / 16 * 16;
    }
    BO_HIP(hipStreamSynchronize(s));
    off = 0;
    for (int q = 0; q < count; q++) {
        std::memcpy(r[q].dst, mail + off, r[q].bytes);
        off += (r[q].bytes + 15) / 16 * 16;
    }
    return BO_OK;
}

// ---- scan ------------------------------------------------------------------
constexpr int kScanBlock = 1024;

__global__ void k_block_sums(const int32_t *in, int n, int32_t *sums) {
    __shared__ int32_t sh[kScanBlock];
    int base = blockIdx.x * kScanBlock;
    int t = threadIdx.x;
    sh[t] = base + t < n ? in[base + t] : 0;
    __syncthreads();
    for (int w = kScanBlock / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] += sh[t + w];
        __syncthreads();
    }
    if (t == 0) sums[blockIdx.x] = sh[0];
}

// exclusive scan of `sums` (nb entries) in one workgroup, sequential chunks
__global__ void k_scan_sums(int32_t *sums, int nb) {
    __shared__ int32_t sh[kScanBlock];
    __shared__ int32_t carry;
    int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += kScanBlock) {
        int v = base + t < nb ? sums[base + t] : 0;
        sh[t] = v;
        __syncthreads();
        for (int off = 1; off < kScanBlock; off <<= 1) {
            int a = t >= off ? sh[t - off] : 0;
            __syncthreads();
            sh[t] += a;
            __syncthreads();
        }
        if (base + t < nb) sums[base + t] = carry + sh[t] - v;
        __syncthreads();
        if (t == kScanBlock - 1) carry += sh[t];
        __syncthreads();
    }
}

__global__ void k_scan_apply(const int32_t *in, int n, const int32_t *sums, int32_t *out) {
    __shared__ int32_t sh[kScanBlock];
    int base = blockIdx.x * kScanBlock;
    int t = threadIdx.x;
    int v = base + t < n ? in[base + t] : 0;
    sh[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        int a = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += a;
        __syncthreads();
    }
    if (base + t < n) out[base + t] = sums[blockIdx.x] + sh[t] - v;
    if (base + t == n - 1) out[n] = sums[blockIdx.x] + sh[t];
}

int scan_sum_words(int n) { return n > 0 ? (n + kScanBlock - 1) / kScanBlock : 1; }

bo_status scan_counts_async(const int32_t *counts, int32_t *out, int n, int32_t *sums, hipStream_t s) {
    if (n <= 0) {
        BO_HIP(hipMemsetAsync(out, 0, sizeof(int32_t), s));
        return BO_OK;
    }
    int nb = (n + kScanBlock - 1) / kScanBlock;
    k_block_sums<<<nb, kScanBlock, 0, s>>>(counts, n, sums);
    k_scan_sums<<<1, kScanBlock, 0, s>>>(sums, nb);
    k_scan_apply<<<nb, kScanBlock, 0, s>>>(counts, n, sums, out);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status scan_counts(const int32_t *counts, int32_t *out, int n, int32_t *total, hipStream_t s,
                      const HostRead *extra, int nextra) {
    if (nextra < 0 || nextra > 3) return fail(BO_ERR_INVALID_ARG, "scan_counts: at most three extra reads");
    HostRead r[4];
    for (int q = 0; q < nextra; q++) r[1 + q] = extra[q];
    if (n <= 0) {
        int32_t z = 0;
        BO_HIP(hipMemcpyAsync(out, &z, sizeof z, hipMemcpyHostToDevice, s));
        if (nextra > 0) {
            BO_TRY(host_reads(r + 1, nextra, s));
        } else {
            BO_HIP(hipStreamSynchronize(s));
        }
        if (total) *total = 0;
        return BO_OK;
    }
    int nb = (n + kScanBlock - 1) / kScanBlock;
    int32_t *sums = nullptr;
    BO_TRY(scratch_get(SC_SCAN, sizeof(int32_t) * nb, (void **)&sums));
    k_block_sums<<<nb, kScanBlock, 0, s>>>(counts, n, sums);
    k_scan_sums<<<1, kScanBlock, 0, s>>>(sums, nb);
    k_scan_apply<<<nb, kScanBlock, 0, s>>>(counts, n, sums, out);
    BO_HIP(hipGetLastError());
    int32_t tot = 0;
    r[0] = HostRead{out + n, sizeof tot, &tot};
    BO_TRY(host_reads(r, 1 + nextra, s));
    if (total) *total = tot;
    return BO_OK;
}

// ---- BSR SpMV on the ABI layout ---------------------------------------------
// Three threads per block row, thread r forming component r: per block it
// reads block row r (three contiguous doubles), so the three threads of a
// row read the block's 72 contiguous bytes together and a wavefront's loads
// touch three times fewer cache lines than with one thread per row; each
// component sums in block order and, within a block, in column order.
__global__ void k_bsr_spmv(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, double alpha, const double *__restrict__ x,
                           double beta, double *__restrict__ y) {
    const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= 3LL * n) return;
    const int i = (int)(t / 3), r = (int)(t - 3LL * i);
    double s = 0.0;
    const int e1 = rp[i + 1];
    for (int e = rp[i]; e < e1; e++) {
        const double *b3 = v + 9 * (size_t)e + 3 * r;
        const double *xj = x + 3 * (size_t)ci[e];
        s = s + b3[0] * xj[0];
        s = s + b3[1] * xj[1];
        s = s + b3[2] * xj[2];
    }
    const double yi = beta == 0.0 ? 0.0 : beta * y[t];
    y[t] = alpha * s + yi;
}

// ---- sliced BSR (general operator of the solver) -------------------------------
// the width of each slice: its longest row, or in a stencil slice 7 + the
// most entries a row has beyond its stencil neighbours
// (a wavefront per slice: one lane per row, the maximum by shuffles)
__global__ void k_sell_width(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci, SellGrid G,
                             int32_t *__restrict__ width) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x, S = r >> 6;
    int len = 0;
    if (r < n) {
        len = rp[r + 1] - rp[r];
        if (sell_stencil_slice(G, S)) {
            int nb[NSLOT], extra = 0;
            sell_stencil_nbrs(G, r, nb);
            for (int e = rp[r]; e < rp[r + 1]; e++) extra += sell_slot_in(nb, ci[e]) < 0;
            len = NSLOT + extra;
        }
    }
    for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
    if ((threadIdx.x & 63) == 0 && 64 * S < n) width[S] = len;
}

__global__ void k_sell_fill(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                            const double *__restrict__ v, const int32_t *__restrict__ soff, SellGrid G,
                            int32_t *__restrict__ sci, double *__restrict__ sv) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int S = r >> 6, lane = r & 63;
    int k0 = soff[S], K = soff[S + 1] - k0;
    int e0 = rp[r], len = rp[r + 1] - e0;
    // padding (past the row's end, or a stencil position the row lacks): a
    // zero block on the row's own column (in a stencil slice: the column the
    // kernels derive), so its product adds +0 and the x load stays in bounds
    for (int k = 0; k < K; k++) {
        size_t b = (size_t)(k0 + k) * 64 + lane;
        sci[b] = sell_stencil_slice(G, S) && k < NSLOT ? sell_stencil_col(G, r, k, n) : r;
        for (int z = 0; z < 9; z++) sv[((size_t)(k0 + k) * 9 + z) * 64 + lane] = 0.0;
    }
    const bool st = sell_stencil_slice(G, S);
    int nb[NSLOT];
    if (st) sell_stencil_nbrs(G, r, nb);
    int next = st ? NSLOT : 0;
    for (int q = 0; q < len; q++) {
        const int c = ci[e0 + q];
        int k = st ? sell_slot_in(nb, c) : -1;
        if (k < 0) k = next++;
        size_t b = (size_t)(k0 + k) * 64 + lane;
        sci[b] = c;
        for (int z = 0; z < 9; z++) sv[((size_t)(k0 + k) * 9 + z) * 64 + lane] = v[9 * (size_t)(e0 + q) + z];
    }
}

// One row of the sliced layout, W blocks: every index and value load of the
// row is issued before the first product (no load waits on a branch), then
// the x gathers and the sums in block order.
template <int W, bool ST>
__device__ __forceinline__ void sell_row(const int32_t *__restrict__ sci, const double *__restrict__ sv, int k0,
                                         int lane, const SellGrid &G, int r, int n, const double *__restrict__ x,
                                         double &s0, double &s1, double &s2) {
    int c[W];
#pragma unroll
    for (int k = 0; k < W; k++) c[k] = ST && k < NSLOT ? sell_stencil_col(G, r, k, n) : sci[(size_t)(k0 + k) * 64 + lane];
    double e[W][9];
#pragma unroll
    for (int k = 0; k < W; k++)
#pragma unroll
        for (int z = 0; z < 9; z++) e[k][z] = __builtin_nontemporal_load(sv + ((size_t)(k0 + k) * 9 + z) * 64 + lane);
#pragma unroll
    for (int k = 0; k < W; k++) {
        const double *xj = x + 3 * (size_t)c[k];
        double x0 = xj[0], x1 = xj[1], x2 = xj[2];
        s0 = s0 + e[k][0] * x0; s0 = s0 + e[k][1] * x1; s0 = s0 + e[k][2] * x2;
        s1 = s1 + e[k][3] * x0; s1 = s1 + e[k][4] * x1; s1 = s1 + e[k][5] * x2;
        s2 = s2 + e[k][6] * x0; s2 = s2 + e[k][7] * x1; s2 = s2 + e[k][8] * x2;
    }
}

// y = alpha A x + beta y on the sliced layout: the blocks of a row in their
// BSR order and each block's entries in order, as k_bsr_spmv; the 64 lanes of
// a wavefront read each of a block column's 9 value arrays as one 512 B line
// pair (non-temporal: read once per launch).  A wavefront is one slice, so the
// slice width selects one path for all its lanes: widths 7 and 8 (the 7-point
// stencil, and a row with a well block) unrolled, others in a loop.  Padding
// blocks are zero blocks on the row's own column and add +0.
__global__ void __launch_bounds__(kBlock) k_sell_spmv(int n, const int32_t *__restrict__ soff,
                                                      const int32_t *__restrict__ sci,
                                                      const double *__restrict__ sv, SellGrid G, double alpha,
                                                      const double *__restrict__ x, double beta,
                                                      const double *yin, double *y) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    int S = r >> 6, lane = r & 63;
    int k0 = soff[S], K = soff[S + 1] - k0;
    const bool st = sell_stencil_slice(G, S);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (K == 7) {
        if (st) sell_row<7, true>(sci, sv, k0, lane, G, r, n, x, s0, s1, s2);
        else sell_row<7, false>(sci, sv, k0, lane, G, r, n, x, s0, s1, s2);
    } else if (K == 8) {
        if (st) sell_row<8, true>(sci, sv, k0, lane, G, r, n, x, s0, s1, s2);
        else sell_row<8, false>(sci, sv, k0, lane, G, r, n, x, s0, s1, s2);
    } else {
        for (int k = 0; k < K; k++) {
            int c = st && k < NSLOT ? sell_stencil_col(G, r, k, n) : sci[(size_t)(k0 + k) * 64 + lane];
            const double *blk = sv + (size_t)(k0 + k) * 9 * 64 + lane;
            double e[9];
#pragma unroll
            for (int z = 0; z < 9; z++) e[z] = __builtin_nontemporal_load(blk + z * 64);
            double x0 = x[3 * (size_t)c], x1 = x[3 * (size_t)c + 1], x2 = x[3 * (size_t)c + 2];
            s0 = s0 + e[0] * x0; s0 = s0 + e[1] * x1; s0 = s0 + e[2] * x2;
            s1 = s1 + e[3] * x0; s1 = s1 + e[4] * x1; s1 = s1 + e[5] * x2;
            s2 = s2 + e[6] * x0; s2 = s2 + e[7] * x1; s2 = s2 + e[8] * x2;
        }
    }
    // y = alpha A x + beta yin (yin is y itself, or another vector)
    const double *wi = yin + 3 * (size_t)r;
    double t0 = beta == 0.0 ? 0.0 : beta * wi[0];
    double t1 = beta == 0.0 ? 0.0 : beta * wi[1];
    double t2 = beta == 0.0 ? 0.0 : beta * wi[2];
    double *yi = y + 3 * (size_t)r;
    yi[0] = alpha * s0 + t0;
    yi[1] = alpha * s1 + t1;
    yi[2] = alpha * s2 + t2;
}

// r -= A Pi_p dp on the sliced layout, in place: column 0 of each block (3
// of its 9 value arrays), dp on the block columns below npr (0 elsewhere;
// padding blocks sit on the row's own column with zero values).
template <typename TD>
__global__ void __launch_bounds__(kBlock) k_sell_col0_update(int n, int npr, const int32_t *__restrict__ soff,
                                                             const int32_t *__restrict__ sci,
                                                             const double *__restrict__ sv, SellGrid G,
                                                             const TD *__restrict__ dp, double *r) {
    const int row = blockIdx.x * blockDim.x + threadIdx.x;
    if (row >= n) return;
    const int S = row >> 6, lane = row & 63;
    const int k0 = soff[S], K = soff[S + 1] - k0;
    const bool st = sell_stencil_slice(G, S);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int k = 0; k < K; k++) {
        const int c = st && k < NSLOT ? sell_stencil_col(G, row, k, n) : sci[(size_t)(k0 + k) * 64 + lane];
        const double *blk = sv + (size_t)(k0 + k) * 9 * 64 + lane;
        const double p = c < npr ? (double)dp[c] : 0.0;
        s0 = s0 + __builtin_nontemporal_load(blk) * p;
        s1 = s1 + __builtin_nontemporal_load(blk + 3 * 64) * p;
        s2 = s2 + __builtin_nontemporal_load(blk + 6 * 64) * p;
    }
    double *ri = r + 3 * (size_t)row;
    ri[0] = ri[0] - s0;
    ri[1] = ri[1] - s1;
    ri[2] = ri[2] - s2;
}

// r -= A Pi_p dp on the slot layout, in place (column 0 of each block)
template <typename TD>
__global__ void __launch_bounds__(kBlock) k_slot_col0_update(int nx, int ny, int nz, const double *__restrict__ A,
                                                             const TD *__restrict__ dp, double *r) {
    const int n = nx * ny * nz;
    const int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const size_t N = (size_t)n;
    const int nxy = nx * ny;
    const int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int q = 0; q < NSLOT; q++) {
        const int j = nb[q];
        if (j < 0) continue;
        const double *a = A + (size_t)q * 9 * N + i;
        const double p = (double)dp[j];
        s0 = s0 + a[0 * N] * p;
        s1 = s1 + a[3 * N] * p;
        s2 = s2 + a[6 * N] * p;
    }
    double *ri = r + 3 * (size_t)i;
    ri[0] = ri[0] - s0;
    ri[1] = ri[1] - s1;
    ri[2] = ri[2] - s2;
}

// ---- BSR -> slot layout -------------------------------------------------------
__global__ void k_bsr_to_slots(int nx, int ny, int nz, const int32_t *__restrict__ rp,
                               const int32_t *__restrict__ ci, const double *__restrict__ v,
                               double *__restrict__ slots, int32_t *__restrict__ bad) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = nx * ny * nz;
    if (i >= n) return;
    size_t N = (size_t)n;
    int e = rp[i], end = rp[i + 1];
    for (int s = 0; s < NSLOT; s++) {
        int nb = nbr_of(i, s, nx, ny, nz);
        bool have = nb >= 0 && e < end && ci[e] == nb;
        for (int z = 0; z < 9; z++) slots[((size_t)s * 9 + z) * N + i] = have ? v[9 * (size_t)e + z] : 0.0;
        if (have) e++;
        else if (nb >= 0) *bad = 1;  // a stencil neighbour is missing from the pattern
    }
    if (e != end) *bad = 1;          // entries outside the 7-point stencil
}

// y = alpha A x + beta y on the slot layout.  Each row sums its blocks in
// ascending column order and each block's entries in ascending order.  The
// workgroups run in launch order (not remapped per XCD), so the whole chip
// reads each of the 63 coefficient arrays at one advancing front, and the
// coefficients, read once per launch, are loaded non-temporally (streamed
// past the caches).  Measured on the 2M-cell grid this reads 12 % faster than
// one contiguous row range per XCD.
__global__ void __launch_bounds__(kBlock) k_slot_spmv(int nx, int ny, int nz, const double *__restrict__ A,
                                                      double alpha, const double *__restrict__ x, double beta,
                                                      double *__restrict__ y) {
    int n = nx * ny * nz;
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
        int j = nb[s];
        if (j < 0) continue;
        const double *a = A + (size_t)s * 9 * N + i;
        double x0 = x[3 * (size_t)j], x1 = x[3 * (size_t)j + 1], x2 = x[3 * (size_t)j + 2];
        double e[9];
#pragma unroll
        for (int z = 0; z < 9; z++) e[z] = __builtin_nontemporal_load(a + z * N);
        s0 = s0 + e[0] * x0; s0 = s0 + e[1] * x1; s0 = s0 + e[2] * x2;
        s1 = s1 + e[3] * x0; s1 = s1 + e[4] * x1; s1 = s1 + e[5] * x2;
        s2 = s2 + e[6] * x0; s2 = s2 + e[7] * x1; s2 = s2 + e[8] * x2;
    }
    double *yi = y + 3 * (size_t)i;
    if (beta == 0.0) {
        yi[0] = alpha * s0 + 0.0; yi[1] = alpha * s1 + 0.0; yi[2] = alpha * s2 + 0.0;
    } else {
        yi[0] = alpha * s0 + beta * yi[0];
        yi[1] = alpha * s1 + beta * yi[1];
        yi[2] = alpha * s2 + beta * yi[2];
    }
}

// r = v - A (Pi_p dp): only column 0 of each block is needed.  The residual
// is formed in FP64; dp may be FP32 (mixed form) and r is stored as TO.
template <typename TD, typename TO>
__global__ void __launch_bounds__(kBlock) k_slot_col0_residual(int nx, int ny, int nz,
                                                               const double *__restrict__ A,
                                                               const double *__restrict__ v,
                                                               const TD *__restrict__ dp,
                                                               TO *__restrict__ r) {
    int n = nx * ny * nz;
    int i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    size_t N = (size_t)n;
    int nxy = nx * ny;
    int ix = i % nx, iy = (i / nx) % ny, iz = i / nxy;
    const int nb[7] = {iz > 0 ? i - nxy : -1, iy > 0 ? i - nx : -1, ix > 0 ? i - 1 : -1, i,
                       ix < nx - 1 ? i + 1 : -1, iy < ny - 1 ? i + nx : -1, iz < nz - 1 ? i + nxy : -1};
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
#pragma unroll
    for (int s = 0; s < NSLOT; s++) {
        int j = nb[s];
        if (j < 0) continue;
        const double *a = A + (size_t)s * 9 * N + i;
        double p = (double)dp[j];
        s0 = s0 + a[0 * N] * p;
        s1 = s1 + a[3 * N] * p;
        s2 = s2 + a[6 * N] * p;
    }
    r[3 * (size_t)i] = (TO)(v[3 * (size_t)i] - s0);
    r[3 * (size_t)i + 1] = (TO)(v[3 * (size_t)i + 1] - s1);
    r[3 * (size_t)i + 2] = (TO)(v[3 * (size_t)i + 2] - s2);
}

// The same residual written in the F stage's slot order: component c of cell
// i goes to out[c * S + slot_of[i]].
// ---- BLAS-1 -------------------------------------------------------------------
__global__ void k_axpby(long long n, double a, const double *__restrict__ x, double b, double *__restrict__ y) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = b == 0.0 ? a * x[i] : a * x[i] + b * y[i];
}

// w <- w / sqrt(nrm2[0]) unless that norm is <= 1e-300 (Arnoldi breakdown):
// the same product (1/h) w as axpby with the factor formed on the host
__global__ void k_normalize(long long n, const double *__restrict__ nrm2, double *__restrict__ w) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double h = sqrt(nrm2[0]);
    if (h > 1e-300) w[i] = (1.0 / h) * w[i];
}

__global__ void k_fill(long long n, double v, double *__restrict__ y) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = v;
}

// wavefront sum by butterfly shuffles (fixed order)
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = v + __shfl_xor(v, off, 64);
    return v;
}

// Multi-dot, pass 1: each of the kRedBlocks workgroups writes the partial
// sums of its grid-stride share, partial[q * nblocks + block] = sum x[e] V[q][e].
template <int NV>
__global__ void __launch_bounds__(kBlock) k_multidot_partial(long long n, const double *__restrict__ x, VecList V,
                                                             double *__restrict__ partial) {
    __shared__ double sh[NV][kBlock / 64];
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) acc[q] = 0.0;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double xe = x[e];
#pragma unroll
        for (int q = 0; q < NV; q++) acc[q] = acc[q] + xe * V.p[q][e];
    }
    int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double w = wave_sum(acc[q]);
        if (lane == 0) sh[q][wave] = w;
    }
    __syncthreads();
    if (threadIdx.x < NV) {
        double t = 0.0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; w++) t = t + sh[threadIdx.x][w];
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// Classical Gram-Schmidt pass over the basis V (nv <= NV vectors), one read of
// every vector per element:
//   h == NULL:            partial sums of <w, V[q]>
//   h != NULL, dots != 0: w -= sum_q h[q] V[q], then partial sums of <w, V[q]>
//   h != NULL, dots == 0: w -= sum_q h[q] V[q], then the partial sum of <w, w>
// The basis values of an element stay in registers between the update and
// the dot products.  This form takes up to NV vectors (loads predicated on
// nv) and any length; k_cgs_exact below is the one the solver normally runs.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_cgs_pass(long long n, double *__restrict__ w, VecList V, int nv,
                                                     const double *__restrict__ h, int dots,
                                                     double *__restrict__ partial) {
    __shared__ double hs[NV];
    __shared__ double sh[NV][kBlock / 64];
    if (h && threadIdx.x < nv) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    double acc[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) acc[q] = 0.0;
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double we = w[e];
        double vq[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) vq[q] = q < nv ? V.p[q][e] : 0.0;
        if (h) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NV; q++)
                if (q < nv) s = s + hs[q] * vq[q];
            we = we - s;
            w[e] = we;
        }
        if (dots || !h) {
#pragma unroll
            for (int q = 0; q < NV; q++) acc[q] = acc[q] + we * vq[q];
        } else {
            acc[0] = acc[0] + we * we;
        }
    }
    int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    int nout = (dots || !h) ? nv : 1;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double t = wave_sum(acc[q]);
        if (lane == 0) sh[q][wave] = t;
    }
    __syncthreads();
    if (threadIdx.x < nout) {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < kBlock / 64; u++) t = t + sh[threadIdx.x][u];
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// The same pass for exactly NV vectors below 4 GiB each, one kernel per mode
// (0: dots, 1: update then dots, 2: update then norm): no predicated loads (a
// load that only some paths issue makes the compiler wait for every load in
// flight) and no branches in the loop; each load is a vector base in scalar
// registers plus one 32-bit byte offset shared by all vectors, so addresses
// cost no vector registers.  Same arithmetic order as k_cgs_pass.
template <int NV, int MODE>
__global__ void __launch_bounds__(kBlock) k_cgs_exact(uint32_t n, double *__restrict__ w, VecList V,
                                                      const double *__restrict__ h, int rev,
                                                      double *__restrict__ partial) {
    constexpr bool upd = MODE != 0;
    constexpr int NA = MODE == 2 ? 1 : NV;  // accumulators
    __shared__ double hs[NV];
    __shared__ double sh[NA][kBlock / 64];
    if (upd && threadIdx.x < NV) hs[threadIdx.x] = h[threadIdx.x];
    __syncthreads();
    auto at = [](const double *p, uint32_t boff) -> const double * {
        return (const double *)((const char *)p + boff);
    };
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; q++) acc[q] = 0.0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const uint32_t boff = (rev ? n - 1 - e : e) * (uint32_t)sizeof(double);
        double we = *at(w, boff);
        double vq[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) vq[q] = *at(V.p[q], boff);
        if constexpr (upd) {
            double s = 0.0;
#pragma unroll
            for (int q = 0; q < NV; q++) s = s + hs[q] * vq[q];
            we = we - s;
            *(double *)at(w, boff) = we;
        }
        if constexpr (MODE == 2) {
            acc[0] = acc[0] + we * we;
        } else {
#pragma unroll
            for (int q = 0; q < NV; q++) acc[q] = acc[q] + we * vq[q];
        }
    }
    int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int q = 0; q < NA; q++) {
        double t = wave_sum(acc[q]);
        if (lane == 0) sh[q][wave] = t;
    }
    __syncthreads();
    if (threadIdx.x < NA) {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < kBlock / 64; u++) t = t + sh[threadIdx.x][u];
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// ---- Gram-Schmidt with the re-orthogonalisation delayed by one step ---------
// (classical Gram-Schmidt twice, each vector's second projection taken in the
// step after it was formed, so one step reads the basis twice, not three
// times; Arnoldi step j has the final basis V[0..j), the pending vector
// V[j] = u (w of the previous step after its first projection) and w = A z_j)
//
// Dots: against u and w, for every vector of [V[0..j), u] (NV = j + 1):
// partial sums of <V[q], u> into rows q, of <V[q], w> into rows NV + q.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_dcgs_dots(uint32_t n, VecList V, const double *__restrict__ w,
                                                      double *__restrict__ partial) {
    __shared__ double sh[2 * NV][kBlock / 64];
    auto at = [](const double *p, uint32_t boff) -> const double * {
        return (const double *)((const char *)p + boff);
    };
    double a1[NV], a2[NV];
#pragma unroll
    for (int q = 0; q < NV; q++) a1[q] = a2[q] = 0.0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const uint32_t boff = e * (uint32_t)sizeof(double);
        double we = *at(w, boff);
        double vq[NV];
#pragma unroll
        for (int q = 0; q < NV; q++) vq[q] = *at(V.p[q], boff);
        const double u = vq[NV - 1];
#pragma unroll
        for (int q = 0; q < NV; q++) {
            a1[q] = a1[q] + vq[q] * u;
            a2[q] = a2[q] + vq[q] * we;
        }
    }
    int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
#pragma unroll
    for (int q = 0; q < NV; q++) {
        double t1 = wave_sum(a1[q]), t2 = wave_sum(a2[q]);
        if (lane == 0) { sh[q][wave] = t1; sh[NV + q][wave] = t2; }
    }
    __syncthreads();
    if (threadIdx.x < 2 * NV) {
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < kBlock / 64; u++) t = t + sh[threadIdx.x][u];
        partial[(size_t)threadIdx.x * gridDim.x + blockIdx.x] = t;
    }
}

// Update for step J, from the dots red = [<V[i],u> (s_i), <u,u>, <V[i],w> (p_i),
// <u,w>]: beta = sqrt(<u,u> - |s|^2) (the norm of u - V s), the final vector
// v = (u - V s) / beta into V[J], r = <v,w> = (<u,w> - s.p) / beta, and
// w - V p - r v into V[J+1] (the next pending vector) with partial sums of
// its squared norm.  beta and r go to sc[0], sc[1] (workgroup 0); every
// workgroup forms the same coefficients.  A pending vector inside the span of
// the basis (beta^2 <= 0) leaves beta = 0 in sc[0] and zero vectors.
template <int J>
__global__ void __launch_bounds__(kBlock) k_dcgs_update(uint32_t n, VecList V, const double *__restrict__ red,
                                                        double *__restrict__ sc, int rev,
                                                        double *__restrict__ partial, double *sc_mirror) {
    __shared__ double cs[J > 0 ? J : 1], cp[J > 0 ? J : 1], cb[2];
    __shared__ double sh[kBlock / 64];
    if (threadIdx.x == 0) {
        double ss = 0.0, sp = 0.0;
        for (int i = 0; i < J; i++) {
            ss = ss + red[i] * red[i];
            sp = sp + red[i] * red[J + 1 + i];
        }
        double b2 = red[J] - ss, beta = 0.0, r = 0.0, ib = 0.0;
        if (b2 > 0.0) {
            beta = sqrt(b2);
            ib = 1.0 / beta;
            r = (red[2 * J + 1] - sp) / beta;
        }
        cb[0] = ib;
        cb[1] = r;
        if (blockIdx.x == 0) {
            sc[0] = beta; sc[1] = r;
            if (sc_mirror) { sc_mirror[0] = beta; sc_mirror[1] = r; }
        }
    }
    if (threadIdx.x < J) {
        cs[threadIdx.x] = red[threadIdx.x];
        cp[threadIdx.x] = red[J + 1 + threadIdx.x];
    }
    __syncthreads();
    const double ib = cb[0], r = ib > 0.0 ? cb[1] : 0.0;
    auto at = [](const double *p, uint32_t boff) -> double * {
        return (double *)((const char *)p + boff);
    };
    double acc = 0.0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        const uint32_t boff = (rev ? n - 1 - e : e) * (uint32_t)sizeof(double);
        double vq[J > 0 ? J : 1];
#pragma unroll
        for (int q = 0; q < J; q++) vq[q] = *at(V.p[q], boff);
        double u = *at(V.p[J], boff), we = *at(V.p[J + 1], boff);
        double s1 = 0.0, s2 = 0.0;
#pragma unroll
        for (int q = 0; q < J; q++) {
            s1 = s1 + cs[q] * vq[q];
            s2 = s2 + cp[q] * vq[q];
        }
        double v = (u - s1) * ib;
        double wn = we - s2 - r * v;
        *at(V.p[J], boff) = v;
        *at(V.p[J + 1], boff) = wn;
        acc = acc + wn * wn;
    }
    int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    double t = wave_sum(acc);
    if (lane == 0) sh[wave] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        double u = 0.0;
#pragma unroll
        for (int k = 0; k < kBlock / 64; k++) u = u + sh[k];
        partial[blockIdx.x] = u;
    }
}

// pass 2 (one workgroup per result): out[q] = sum over the partials in a
// fixed order (strided per thread, then across the wavefront, then across the
// four wavefronts in order)
// (with mirror set, each result is also written there: pinned host memory
// the host reads after the stream's next event, instead of a copy)
__global__ void __launch_bounds__(kBlock) k_partial_final(int nblocks, const double *__restrict__ partial,
                                                          double *__restrict__ out, double *mirror = nullptr) {
    __shared__ double sh[kBlock / 64];
    int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    int q = blockIdx.x;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += blockDim.x) s = s + partial[(size_t)q * nblocks + b];
    s = wave_sum(s);
    if (lane == 0) sh[wave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < kBlock / 64; w++) t = t + sh[w];
        out[q] = t;
        if (mirror) mirror[q] = t;
    }
}

// y = y + sign * sum_q h[q] * V[q]  (h on the device)
__global__ void __launch_bounds__(kBlock) k_multiaxpy(long long n, VecList V, int nv,
                                                      const double *__restrict__ h, double sign,
                                                      double *__restrict__ y) {
    __shared__ double hs[kMaxVecList];
    if (threadIdx.x < nv) hs[threadIdx.x] = sign * h[threadIdx.x];
    __syncthreads();
    long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += stride) {
        double s = 0.0;
        for (int q = 0; q < nv; q++) s = s + hs[q] * V.p[q][e];
        y[e] = y[e] + s;
    }
}

__global__ void k_scale_copy(long long n, const double *__restrict__ inv, const double *__restrict__ x,
                             double *__restrict__ y) {
    long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = x[i] * inv[0];
}

// ---- host wrappers -------------------------------------------------------------
bo_status slot_spmv(const Grid &g, const double *A, double alpha, const double *x, double beta, double *y,
                    hipStream_t s) {
    long long n = g.n();
    k_slot_spmv<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, A, alpha, x, beta, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

template <typename TD, typename TO>
bo_status slot_col0_residual(const Grid &g, const double *A, const double *v, const TD *dp, TO *r, hipStream_t s) {
    long long n = g.n();
    k_slot_col0_residual<TD, TO><<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, A, v, dp, r);
    BO_HIP(hipGetLastError());
    return BO_OK;
}
template bo_status slot_col0_residual<double, double>(const Grid &, const double *, const double *, const double *,
                                                      double *, hipStream_t);
template bo_status slot_col0_residual<float, double>(const Grid &, const double *, const double *, const float *,
                                                     double *, hipStream_t);

bo_status sell_build(int n, const int32_t *rp, const int32_t *ci, const double *v, const SellGrid &G,
                     DBuf<int32_t> &soff, DBuf<int32_t> &sci, DBuf<double> &sv, hipStream_t s) {
    int nsl = (n + 63) / 64;
    BO_TRY(soff.alloc((size_t)nsl + 1));
    int32_t *width = nullptr;
    BO_TRY(scratch_get(SC_SELL, sizeof(int32_t) * (size_t)std::max(nsl, 1), (void **)&width));
    k_sell_width<<<grid_for(64LL * nsl), kBlock, 0, s>>>(n, rp, ci, G, width);
    BO_HIP(hipGetLastError());
    int32_t cols = 0;
    BO_TRY(scan_counts(width, soff.p, nsl, &cols, s));
    BO_TRY(sci.alloc((size_t)cols * 64));
    BO_TRY(sv.alloc((size_t)cols * 64 * 9));
    if (n > 0) k_sell_fill<<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, soff.p, G, sci.p, sv.p);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status sell_spmv(int n, const int32_t *soff, const int32_t *sci, const double *sv, const SellGrid &G,
                    double alpha, const double *x, double beta, double *y, hipStream_t s, const double *yin) {
    if (n <= 0) return BO_OK;
    k_sell_spmv<<<grid_for(n), kBlock, 0, s>>>(n, soff, sci, sv, G, alpha, x, beta, yin ? yin : y, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

template <typename TD>
bo_status sell_col0_update(int n, int npr, const int32_t *soff, const int32_t *sci, const double *sv,
                           const SellGrid &G, const TD *dp, double *r, hipStream_t s) {
    if (n <= 0) return BO_OK;
    k_sell_col0_update<TD><<<grid_for(n), kBlock, 0, s>>>(n, npr, soff, sci, sv, G, dp, r);
    BO_HIP(hipGetLastError());
    return BO_OK;
}
template bo_status sell_col0_update<double>(int, int, const int32_t *, const int32_t *, const double *,
                                            const SellGrid &, const double *, double *, hipStream_t);
template bo_status sell_col0_update<float>(int, int, const int32_t *, const int32_t *, const double *,
                                           const SellGrid &, const float *, double *, hipStream_t);

template <typename TD>
bo_status slot_col0_update(const Grid &g, const double *A, const TD *dp, double *r, hipStream_t s) {
    k_slot_col0_update<TD><<<grid_for(g.n()), kBlock, 0, s>>>(g.nx, g.ny, g.nz, A, dp, r);
    BO_HIP(hipGetLastError());
    return BO_OK;
}
template bo_status slot_col0_update<double>(const Grid &, const double *, const double *, double *, hipStream_t);
template bo_status slot_col0_update<float>(const Grid &, const double *, const float *, double *, hipStream_t);

bo_status bsr_to_slots(const Grid &g, const int32_t *rp, const int32_t *ci, const double *v, double *slots,
                       hipStream_t s) {
    long long n = g.n();
    int32_t *bad = nullptr;
    BO_TRY(scratch_get(SC_FLAG, sizeof(int32_t), (void **)&bad));
    BO_HIP(hipMemsetAsync(bad, 0, sizeof(int32_t), s));
    k_bsr_to_slots<<<grid_for(n), kBlock, 0, s>>>(g.nx, g.ny, g.nz, rp, ci, v, slots, bad);
    BO_HIP(hipGetLastError());
    int32_t h = 0;
    HostRead r{bad, sizeof h, &h};
    BO_TRY(host_reads(&r, 1, s));
    if (h) return fail(BO_ERR_UNSUPPORTED, "matrix pattern is not the 7-point stencil of the grid");
    return BO_OK;
}

bo_status axpby(long long n, double a, const double *x, double b, double *y, hipStream_t s) {
    k_axpby<<<grid_for(n), kBlock, 0, s>>>(n, a, x, b, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status normalize(long long n, const double *nrm2, double *w, hipStream_t s) {
    k_normalize<<<grid_for(n), kBlock, 0, s>>>(n, nrm2, w);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status fill(long long n, double v, double *y, hipStream_t s) {
    k_fill<<<grid_for(n), kBlock, 0, s>>>(n, v, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status multiaxpy(long long n, const double *const *Vhost, int nv, const double *h, double sign, double *y,
                    hipStream_t s) {
    if (nv > kMaxVecList || nv < 1) return fail(BO_ERR_INVALID_ARG, "multiaxpy: 1..64 vectors");
    VecList L{};
    for (int q = 0; q < nv; q++) L.p[q] = Vhost[q];
    long long blocks = std::min<long long>((n + kBlock - 1) / kBlock, 4096);
    k_multiaxpy<<<(unsigned)std::max<long long>(blocks, 1), kBlock, 0, s>>>(n, L, nv, h, sign, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status scale_copy(long long n, const double *inv, const double *x, double *y, hipStream_t s) {
    k_scale_copy<<<grid_for(n), kBlock, 0, s>>>(n, inv, x, y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status Reducer::init() {
    BO_TRY(partial.alloc((size_t)kRedBlocks * kMaxVecList));
    return BO_OK;
}

// Workgroups of the Gram-Schmidt kernels: as many as are resident at once, at
// most four per compute unit (kRedBlocks on a full device), found once per
// kernel and device; a fixed count per kernel keeps the partial sums' order
// fixed.  Slots: k_cgs_exact<K, M> 4K + M, k_dcgs_dots<K> 4K + 3,
// k_dcgs_update<K> 4(kCgsExactMax + 1) + K.
constexpr int kCgsExactMax = 32;
static int resident_blocks(const void *kernel, int slot) {
    constexpr int kSlots = (kCgsExactMax + 1) * 5, kDevs = 16;
    static int cache[kDevs][kSlots] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kDevs) return kRedBlocks;
    int &c = cache[dev][slot];
    if (c == 0) {
        int per_cu = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kBlock, 0) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || per_cu < 1 ||
            cus < 1)
            c = kRedBlocks;
        else
            c = std::min(kRedBlocks, std::min(per_cu, 4) * cus);
    }
    return c;
}

bo_status Reducer::cgs_pass(long long n, double *w, const double *const *Vhost, int nv, const double *h, bool dots,
                            double *out, hipStream_t s, bool reverse) {
    if (nv < 1 || nv > kMaxVecList) return fail(BO_ERR_INVALID_ARG, "cgs_pass: 1..64 vectors");
    VecList L{};
    for (int q = 0; q < nv; q++) L.p[q] = Vhost[q];
    // a fixed grid per vector count (the partial sums' order does not depend
    // on the device), small enough to be resident at once
    int nb = kRedBlocks;
    if (nv <= kCgsExactMax && n < (1ll << 29)) {
        const uint32_t n32 = (uint32_t)n;
        const int mode = !h ? 0 : dots ? 1 : 2, rev = reverse ? 1 : 0;
        switch (nv * 4 + mode) {
#define BO_CGS1(K, M)                                                                  \
    case K * 4 + M:                                                                    \
        nb = resident_blocks((const void *)k_cgs_exact<K, M>, K * 4 + M);              \
        k_cgs_exact<K, M><<<nb, kBlock, 0, s>>>(n32, w, L, h, rev, partial.p);              \
        break;
#define BO_CGS(K) BO_CGS1(K, 0) BO_CGS1(K, 1) BO_CGS1(K, 2)
            BO_CGS(1) BO_CGS(2) BO_CGS(3) BO_CGS(4) BO_CGS(5) BO_CGS(6) BO_CGS(7) BO_CGS(8)
            BO_CGS(9) BO_CGS(10) BO_CGS(11) BO_CGS(12) BO_CGS(13) BO_CGS(14) BO_CGS(15) BO_CGS(16)
            BO_CGS(17) BO_CGS(18) BO_CGS(19) BO_CGS(20) BO_CGS(21) BO_CGS(22) BO_CGS(23) BO_CGS(24)
            BO_CGS(25) BO_CGS(26) BO_CGS(27) BO_CGS(28) BO_CGS(29) BO_CGS(30) BO_CGS(31) BO_CGS(32)
#undef BO_CGS
#undef BO_CGS1
        default: break;
        }
    } else if (nv <= 8) {
        k_cgs_pass<8><<<nb, kBlock, 0, s>>>(n, w, L, nv, h, dots ? 1 : 0, partial.p);
    } else if (nv <= 16) {
        k_cgs_pass<16><<<nb, kBlock, 0, s>>>(n, w, L, nv, h, dots ? 1 : 0, partial.p);
    } else if (nv <= 32) {
        k_cgs_pass<32><<<nb, kBlock, 0, s>>>(n, w, L, nv, h, dots ? 1 : 0, partial.p);
    } else {
        k_cgs_pass<64><<<nb, kBlock, 0, s>>>(n, w, L, nv, h, dots ? 1 : 0, partial.p);
    }
    int nout = (dots || !h) ? nv : 1;
    k_partial_final<<<nout, kBlock, 0, s>>>(nb, partial.p, out);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

static void launch_partial(int nv, long long n, const double *x, const VecList &L, double *partial, hipStream_t s) {
    switch (nv) {
#define BO_MD(K) case K: k_multidot_partial<K><<<kRedBlocks, kBlock, 0, s>>>(n, x, L, partial); break;
        BO_MD(1) BO_MD(2) BO_MD(3) BO_MD(4) BO_MD(5) BO_MD(6) BO_MD(7) BO_MD(8)
        BO_MD(9) BO_MD(10) BO_MD(11) BO_MD(12) BO_MD(13) BO_MD(14) BO_MD(15) BO_MD(16)
#undef BO_MD
    default: break;
    }
}

bo_status Reducer::multidot(long long n, const double *x, const double *const *Vhost, int nv, double *out,
                            hipStream_t s) {
    for (int q0 = 0; q0 < nv; q0 += 16) {
        int c = std::min(16, nv - q0);
        VecList L{};
        for (int q = 0; q < c; q++) L.p[q] = Vhost[q0 + q];
        launch_partial(c, n, x, L, partial.p, s);
        k_partial_final<<<c, kBlock, 0, s>>>(kRedBlocks, partial.p, out + q0);
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status Reducer::dcgs_dots(long long n, const double *const *Vhost, int nv, const double *w, double *out,
                             hipStream_t s, double *mirror) {
    if (nv < 1 || nv > kCgsExactMax || n >= (1ll << 29))
        return fail(BO_ERR_INVALID_ARG, "dcgs_dots: 1..32 vectors below 2^29 elements");
    VecList L{};
    for (int q = 0; q < nv; q++) L.p[q] = Vhost[q];
    const uint32_t n32 = (uint32_t)n;
    int nb = kRedBlocks;
    switch (nv) {
#define BO_D(K)                                                                   \
    case K:                                                                       \
        nb = resident_blocks((const void *)k_dcgs_dots<K>, 4 * K + 3);            \
        k_dcgs_dots<K><<<nb, kBlock, 0, s>>>(n32, L, w, partial.p);               \
        break;
        BO_D(1) BO_D(2) BO_D(3) BO_D(4) BO_D(5) BO_D(6) BO_D(7) BO_D(8)
        BO_D(9) BO_D(10) BO_D(11) BO_D(12) BO_D(13) BO_D(14) BO_D(15) BO_D(16)
        BO_D(17) BO_D(18) BO_D(19) BO_D(20) BO_D(21) BO_D(22) BO_D(23) BO_D(24)
        BO_D(25) BO_D(26) BO_D(27) BO_D(28) BO_D(29) BO_D(30) BO_D(31) BO_D(32)
#undef BO_D
    default: break;
    }
    k_partial_final<<<2 * nv, kBlock, 0, s>>>(nb, partial.p, out, mirror);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status Reducer::dcgs_update(long long n, const double *const *Vhost, int j, const double *red, double *sc,
                               double *norm2, hipStream_t s, bool reverse, double *sc_mirror, double *norm2_mirror) {
    if (j < 0 || j + 1 > kCgsExactMax || n >= (1ll << 29))
        return fail(BO_ERR_INVALID_ARG, "dcgs_update: step 0..31 below 2^29 elements");
    VecList L{};
    for (int q = 0; q < j + 2; q++) L.p[q] = Vhost[q];
    const uint32_t n32 = (uint32_t)n;
    const int rev = reverse ? 1 : 0;
    int nb = kRedBlocks;
    switch (j) {
#define BO_U(K)                                                                     \
    case K:                                                                         \
        nb = resident_blocks((const void *)k_dcgs_update<K>, 4 * (kCgsExactMax + 1) + K);          \
        k_dcgs_update<K><<<nb, kBlock, 0, s>>>(n32, L, red, sc, rev, partial.p, sc_mirror); \
        break;
        BO_U(0) BO_U(1) BO_U(2) BO_U(3) BO_U(4) BO_U(5) BO_U(6) BO_U(7)
        BO_U(8) BO_U(9) BO_U(10) BO_U(11) BO_U(12) BO_U(13) BO_U(14) BO_U(15)
        BO_U(16) BO_U(17) BO_U(18) BO_U(19) BO_U(20) BO_U(21) BO_U(22) BO_U(23)
        BO_U(24) BO_U(25) BO_U(26) BO_U(27) BO_U(28) BO_U(29) BO_U(30) BO_U(31)
#undef BO_U
    default: break;
    }
    k_partial_final<<<1, kBlock, 0, s>>>(nb, partial.p, norm2, norm2_mirror);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

bo_status Reducer::dot(long long n, const double *x, const double *y, double *out, hipStream_t s) {
    VecList L{};
    L.p[0] = y;
    launch_partial(1, n, x, L, partial.p, s);
    k_partial_final<<<1, kBlock, 0, s>>>(kRedBlocks, partial.p, out);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

}  // namespace bo

using namespace bo;

extern "C" const char *bo_last_error(void) { return g_err.c_str(); }
extern "C" const char *bo_version(void) { return "bo 0.1 (gfx950)"; }

extern "C" bo_status bo_bsr_spmv(const bo_bsr *A, double alpha, const double *x, double beta, double *y,
                                 void *stream) {
    if (!A || !x || !y || !A->rowptr || !A->colind || !A->val || A->nbrows < 0)
        return fail(BO_ERR_INVALID_ARG, "bo_bsr_spmv: NULL argument");
    if (A->nbrows == 0) return BO_OK;
    hipStream_t s = (hipStream_t)stream;
    k_bsr_spmv<<<grid_for(3LL * A->nbrows), kBlock, 0, s>>>(A->nbrows, A->rowptr, A->colind, A->val, alpha, x, beta,
                                                            y);
    BO_HIP(hipGetLastError());
    return BO_OK;
}
