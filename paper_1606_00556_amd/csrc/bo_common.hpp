// Internal helpers of the bo HIP library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <algorithm>
#include <string>
#include <vector>
#include "../../include/bo.h"

namespace bo {

// ---- errors -----------------------------------------------------------------
void set_error(const std::string &msg);
bo_status fail(bo_status st, const std::string &msg);

#define BO_HIP(call)                                                                 \
    do {                                                                             \
        hipError_t e_ = (call);                                                      \
        if (e_ != hipSuccess)                                                        \
            return ::bo::fail(BO_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

#define BO_TRY(expr)                       \
    do {                                   \
        bo_status s_ = (expr);             \
        if (s_ != BO_OK) return s_;        \
    } while (0)

// ---- device memory ----------------------------------------------------------
// The caller's allocator of the handle an entry point is working on (set for
// the duration of that entry point by AllocScope; NULL: hipMalloc / hipFree),
// and the stream of that entry point.
extern thread_local const bo_allocator *t_alloc;
extern thread_local void *t_alloc_stream;
struct AllocScope {
    const bo_allocator *prev_a;
    void *prev_s;
    AllocScope(const bo_allocator *a, void *stream) : prev_a(t_alloc), prev_s(t_alloc_stream) {
        t_alloc = a;
        t_alloc_stream = stream;
    }
    ~AllocScope() {
        t_alloc = prev_a;
        t_alloc_stream = prev_s;
    }
};

// Owned device buffer (freed in the destructor).  Memory comes from the
// allocator in scope when it is allocated and goes back to the same one.
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    void (*ufree)(void *, void *, void *) = nullptr;  // caller's free, or NULL for hipFree
    void *uctx = nullptr;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n), ufree(o.ufree), uctx(o.uctx) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; n = o.n; ufree = o.ufree; uctx = o.uctx;
            o.p = nullptr; o.n = 0;
        }
        return *this;
    }
    ~DBuf() { release(); }
    void release() {
        if (p) {
            if (ufree) ufree(p, uctx, t_alloc_stream);
            else (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
        ufree = nullptr;
        uctx = nullptr;
    }
    // Grows only: a buffer that has to grow again (a rebuild for a system
    // with larger coarse levels) takes a quarter more than asked, so that a
    // sequence of similar systems stops reallocating (hipFree / hipMalloc
    // synchronise the device).
    bo_status alloc(size_t count) {
        if (count <= n && p) return BO_OK;
        bool regrow = p != nullptr;
        release();
        if (regrow) count = std::max(count, count + count / 4);
        size_t bytes = (count ? count : 1) * sizeof(T);
        if (t_alloc && t_alloc->alloc) {
            p = (T *)t_alloc->alloc(bytes, t_alloc->ctx, t_alloc_stream);
            if (!p) return fail(BO_ERR_ALLOC, "the caller's allocator returned NULL for " + std::to_string(bytes) +
                                                  " bytes");
            ufree = t_alloc->free;
            uctx = t_alloc->ctx;
            n = count;
            return BO_OK;
        }
        hipError_t e = hipMalloc((void **)&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            return fail(BO_ERR_ALLOC, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                          hipGetErrorString(e));
        }
        n = count;
        return BO_OK;
    }
};

// ---- launch geometry --------------------------------------------------------
constexpr int kBlock = 256;
inline unsigned grid_for(long long n, int block = kBlock) {
    long long g = (n + block - 1) / block;
    return (unsigned)(g > 0 ? g : 1);
}

// MI355X has 8 XCDs, each with its own L2; consecutive workgroups are dealt
// round-robin to the XCDs.  Remapping the workgroup index so that each XCD
// owns one contiguous range of rows keeps a row's stencil neighbours (rows +-
// nx*ny away) in the same L2.
__device__ __forceinline__ unsigned xcd_block(unsigned b, unsigned nblocks) {
    const unsigned nx = 8;
    unsigned per = nblocks / nx, rem = nblocks % nx;
    unsigned x = b % nx, q = b / nx;
    // XCD x receives per (+1 if x < rem) blocks; its range starts at base(x)
    unsigned base = x * per + (x < rem ? x : rem);
    return base + q;
}

// ---- structured 7-point stencil ----------------------------------------------
// Slot order = ascending column order of a block row: -z, -y, -x, diag, +x, +y, +z.
enum { S_MZ = 0, S_MY = 1, S_MX = 2, S_D = 3, S_PX = 4, S_PY = 5, S_PZ = 6, NSLOT = 7 };

struct Grid {
    int nx, ny, nz;
    long long n() const { return (long long)nx * ny * nz; }
};

// neighbour of cell g through slot s, or -1 outside the grid
__device__ __forceinline__ int nbr_of(int g, int s, int nx, int ny, int nz) {
    int nxy = nx * ny;
    int i = g % nx, j = (g / nx) % ny, k = g / nxy;
    switch (s) {
    case S_MZ: return k > 0 ? g - nxy : -1;
    case S_MY: return j > 0 ? g - nx : -1;
    case S_MX: return i > 0 ? g - 1 : -1;
    case S_D: return g;
    case S_PX: return i < nx - 1 ? g + 1 : -1;
    case S_PY: return j < ny - 1 ? g + nx : -1;
    default: return k < nz - 1 ? g + nxy : -1;
    }
}

// ---- sliced layouts over a grid's cells -----------------------------------------
// A sliced (SELL-64) matrix whose first `rows` rows are the cells of an
// nx x ny x nz grid: a slice of 64 rows all below `rows` keeps each row's
// stencil entries at positions 0..6 in slot order (ascending column order;
// zero values where the row has no such entry) and the row's other entries
// (columns of extra rows: matrix cells, wells) from position 7 on.  Kernels
// take the columns of positions 0..6 from the row index instead of reading
// them; every other slice (and every matrix without a grid, rows == 0) keeps
// explicit columns.  The same entries in the same order as the CSR row, with
// +0 products where a neighbour is missing, so the same sums.
struct SellGrid {
    int rows = 0;
    int nx = 0, ny = 0, nz = 0;
};
__host__ __device__ inline bool sell_stencil_slice(const SellGrid &G, int S) {
    return 64LL * (S + 1) <= (long long)G.rows;
}
// the column of stencil position k of row r: its neighbour through slot k,
// or r itself where that offset leaves 0..n-1 (the value there is zero)
__device__ __forceinline__ int sell_stencil_col(const SellGrid &G, int r, int k, int n) {
    const int nxy = G.nx * G.ny;
    const int d = k == S_MZ ? -nxy : k == S_MY ? -G.nx : k == S_MX ? -1 : k == S_D ? 0 : k == S_PX ? 1
                : k == S_PY ? G.nx : nxy;
    const int c = r + d;
    return c < 0 || c >= n ? r : c;
}
// the stencil neighbours of cell r in slot order (-1 outside the grid)
__device__ __forceinline__ void sell_stencil_nbrs(const SellGrid &G, int r, int *nb) {
    const int nxy = G.nx * G.ny;
    const int i = r % G.nx, j = (r / G.nx) % G.ny, k = r / nxy;
    nb[S_MZ] = k > 0 ? r - nxy : -1;
    nb[S_MY] = j > 0 ? r - G.nx : -1;
    nb[S_MX] = i > 0 ? r - 1 : -1;
    nb[S_D] = r;
    nb[S_PX] = i < G.nx - 1 ? r + 1 : -1;
    nb[S_PY] = j < G.ny - 1 ? r + G.nx : -1;
    nb[S_PZ] = k < G.nz - 1 ? r + nxy : -1;
}
// the slot of column c among the neighbours nb, or -1 (not a stencil neighbour)
__device__ __forceinline__ int sell_slot_in(const int *nb, int c) {
    int slot = -1;
#pragma unroll
    for (int k = 0; k < NSLOT; k++) slot = nb[k] == c ? k : slot;
    return slot;
}

// ---- small dense blocks ------------------------------------------------------
// Inverse of a 3x3 block by Gauss-Jordan elimination with partial pivoting;
// returns false for a pivot that is zero relative to the block's largest entry.
__host__ __device__ inline bool inv3_gj(const double *A, double *Ainv) {
    double M[3][6];
    double amax = 0.0;
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            M[r][c] = A[3 * r + c];
            M[r][3 + c] = (r == c) ? 1.0 : 0.0;
            double a = fabs(A[3 * r + c]);
            if (a > amax) amax = a;
        }
    if (!(amax > 0.0) || !(amax < INFINITY)) return false;
    // every index below is a compile-time constant once the loops unroll (the
    // pivot row is chosen by selects, not by indexing), so M stays in
    // registers on the GPU
#pragma unroll
    for (int k = 0; k < 3; k++) {
        int piv = k;
        double best = fabs(M[k][k]);
#pragma unroll
        for (int r = k + 1; r < 3; r++) {
            double a = fabs(M[r][k]);
            if (a > best) { best = a; piv = r; }
        }
        if (best <= 1e-300 * amax) return false;
#pragma unroll
        for (int r = k + 1; r < 3; r++) {
            const bool sw = piv == r;
#pragma unroll
            for (int c = 0; c < 6; c++) {
                double t = M[k][c];
                M[k][c] = sw ? M[r][c] : t;
                M[r][c] = sw ? t : M[r][c];
            }
        }
        double d = M[k][k];
        for (int c = 0; c < 6; c++) M[k][c] = M[k][c] / d;
        for (int r = 0; r < 3; r++) {
            if (r == k) continue;
            double f = M[r][k];
            for (int c = 0; c < 6; c++) M[r][c] = M[r][c] - f * M[k][c];
        }
    }
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) Ainv[3 * r + c] = M[r][3 + c];
    return true;
}

// C = A B (3x3), sums from 0 in ascending inner index
__host__ __device__ inline void mul3(const double *A, const double *B, double *C) {
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0.0;
            for (int k = 0; k < 3; k++) s = s + A[3 * r + k] * B[3 * k + c];
            C[3 * r + c] = s;
        }
}

// ---- deterministic reductions ------------------------------------------------
// Sum of a double over a workgroup of kBlock threads in a fixed tree order.
__device__ inline double block_sum(double v, double *sh) {
    int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
        if (t < w) sh[t] = sh[t] + sh[t + w];
        __syncthreads();
    }
    double r = sh[0];
    __syncthreads();
    return r;
}

// ---- process-lifetime scratch ------------------------------------------------------
// Grow-only device buffers for temporaries of host wrappers that synchronise
// the stream before returning (so a buffer is idle whenever a call starts);
// steady-state calls then do not allocate, and hipFree does not synchronise
// the device.  One set per host thread; never freed.
enum ScratchSlot { SC_SCAN = 0, SC_FLAG, SC_JAC_CNT, SC_SELL, SC_COUNT };
bo_status scratch_get(int slot, size_t bytes, void **ptr);

// ---- small device-to-host reads ----------------------------------------------------
// Each read goes through a pinned host buffer (one per host thread, 4 KB,
// never freed), so the copy is a direct DMA; one stream synchronisation
// serves all the reads of a call.
struct HostRead {
    const void *src;  // device
    size_t bytes;
    void *dst;        // host
};
bo_status host_reads(const HostRead *r, int count, hipStream_t s);

// ---- host-side scan / reductions (declared in bo_linalg.hip) -------------------
// Exclusive prefix sum of n int32 counts into out (n+1 entries, out[n] = total);
// returns the total on the host (synchronises the stream).  The nextra reads
// in extra (device words the caller wants) are served in the same
// synchronisation (at most three).
bo_status scan_counts(const int32_t *counts, int32_t *out, int n, int32_t *total, hipStream_t s,
                      const HostRead *extra = nullptr, int nextra = 0);
// The same prefix sum enqueued without reading anything back (no
// synchronisation), for callers that know the total; sums is the caller's
// work buffer of scan_sum_words(n) words, in use until the stream reaches it.
int scan_sum_words(int n);
bo_status scan_counts_async(const int32_t *counts, int32_t *out, int n, int32_t *sums, hipStream_t s);

}  // namespace bo
