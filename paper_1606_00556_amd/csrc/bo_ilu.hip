// F stage of CPR (Section 3.2): the paper's restricted additive Schwarz with
// ILU(0) subdomain solves, mapped onto the GPU as non-overlapping subdomains
// of tile_x x tile_y grid columns (all nz layers), one wavefront per tile.
//
// On the 7-point stencil the grid graph has no triangles, so block ILU(0)
// only modifies the diagonal blocks: E_i = A_ii - sum_{k<i} A_ik E_k^{-1} A_ki
// over the lower neighbours k inside the tile (natural order: -z, -y, -x).
// The FP64 solve takes the unit-lower factors L_ik = A_ik E_k^{-1}:
// y_i = r_i - sum_{k<i} L_ik y_k, then x_i = E_i^{-1}(y_i - sum_{j>i} A_ij x_j)
// (27 factor values per cell forward, 36 backward).  The FP32 / BF16 forms
// keep the blocks of A: w_i = E_i^{-1}(r_i - sum_{k<i} A_ik w_k), then
// x_i = w_i - E_i^{-1} sum_{j>i} A_ij x_j.
//
// Schedule: lane t = a + tile_x*b of the tile owns grid column (i0+a, j0+b)
// and at step s handles layer k = s - a - b, so its -x, -y and -z neighbours
// were handled one step earlier by lanes t-1, t-tile_x and t itself.  The
// factors are stored in the same (tile, step, lane) order, packed in pairs, so
// each step reads its doubles with contiguous 1 KB loads (14 or 18 of them).  Two
// wavefronts share a tile, each loading half of the factors several steps
// ahead and exchanging partial products through LDS (see the sweeps below).
// Block Jacobi (x_i = A_ii^{-1} r_i) is the alternative F stage.
//
// Mixed form: the factors (E^{-1} and the blocks of A) are computed in FP64
// and stored rounded to FP32 (9 float4 per slot and sweep) or to BF16 (9 uint2
// per slot and sweep, round to nearest even from the FP32 value); the sweeps
// run in FP32 on FP32 vectors.
#include <type_traits>
#include "bo_cpr.hpp"

namespace bo {
namespace {

struct TileGeom {
    int nx, ny, nz, tx, ty, ntx, nty, ns;
    __host__ __device__ long long slots() const { return (long long)ntx * nty * ns * 64; }
};

// The factors of one slot for one sweep are 36 doubles: E^{-1} and the three
// lower blocks (-z, -y, -x) for the forward sweep, E^{-1} and the three upper
// blocks (+z, +x, +y) for the backward sweep.  They are packed as 18 double2
// per slot in (tile, step, pair, lane) order, so one wavefront load of a
// pair reads 1 KB contiguously and a step needs 18 load instructions.  In the
// FP64 form the forward slot holds the unit-lower factors in place of the
// lower blocks and its sweep reads pairs 4..17 only (values 8..35).
constexpr int kPairs = 18;
__device__ __forceinline__ size_t pk_index(int tile, int ns, int s, int pair, int lane) {
    return (((size_t)tile * ns + s) * kPairs + pair) * 64 + lane;
}

enum { ST_F64 = 0, ST_F32 = 1, ST_BF16 = 2 };
constexpr int kQuads = 9;  // 36 values as 9 groups of four (FP32 / BF16 forms)
__device__ __forceinline__ size_t pq_index(int tile, int ns, int s, int quad, int lane) {
    return (((size_t)tile * ns + s) * kQuads + quad) * 64 + lane;
}

// FP32 -> BF16, round to nearest even (inputs are finite)
__device__ __forceinline__ uint32_t bf16_bits(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ __forceinline__ float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

// store one slot's 36 FP64 values in the chosen format
template <int St>
__device__ __forceinline__ void store_pack(void *F, int tile, int ns, int s, int t, const double *v) {
    if constexpr (St == ST_F64) {
        double2 *D = (double2 *)F;
        for (int p2 = 0; p2 < kPairs; p2++) D[pk_index(tile, ns, s, p2, t)] = make_double2(v[2 * p2], v[2 * p2 + 1]);
    } else if constexpr (St == ST_F32) {
        float4 *D = (float4 *)F;
        for (int qd = 0; qd < kQuads; qd++)
            D[pq_index(tile, ns, s, qd, t)] = make_float4((float)v[4 * qd], (float)v[4 * qd + 1],
                                                          (float)v[4 * qd + 2], (float)v[4 * qd + 3]);
    } else {
        uint2 *D = (uint2 *)F;
        for (int qd = 0; qd < kQuads; qd++) {
            uint32_t h0 = bf16_bits((float)v[4 * qd]), h1 = bf16_bits((float)v[4 * qd + 1]);
            uint32_t h2 = bf16_bits((float)v[4 * qd + 2]), h3 = bf16_bits((float)v[4 * qd + 3]);
            D[pq_index(tile, ns, s, qd, t)] = make_uint2(h0 | (h1 << 16), h2 | (h3 << 16));
        }
    }
}

__device__ __forceinline__ void load_blk(const double *__restrict__ A, int slot, size_t N, int g, double *o) {
    const double *p = A + (size_t)slot * 9 * N + g;
#pragma unroll
    for (int z = 0; z < 9; z++) o[z] = p[(size_t)z * N];
}

template <typename T>
__device__ __forceinline__ void mv3(const T *A, const T *x, T *y) {
    y[0] = A[0] * x[0] + A[1] * x[1] + A[2] * x[2];
    y[1] = A[3] * x[0] + A[4] * x[1] + A[5] * x[2];
    y[2] = A[6] * x[0] + A[7] * x[1] + A[8] * x[2];
}

template <int K>
__device__ __forceinline__ void shfl_arr(const double *src, double *dst, int lane) {
#pragma unroll
    for (int z = 0; z < K; z++) dst[z] = __shfl(src[z], lane, 64);
}

// Factorisation in two passes, in FP64 for every storage format.  Pack: one
// thread per slot (tile, step, lane), all slots at once, gathers its cell's
// blocks into the FP64 packed layout (forward slot: [A_ii | Az Ay Ax] with
// the lower blocks -z, -y, -x; backward slot: [- | Uz Ux Uy] with the upper
// blocks +z, +x, +y; zero where the neighbour lies outside the tile or grid)
// and records the slot of each cell.  Chain: one wavefront per tile walks the
// steps; lane t = a + tile_x*b at step s handles layer k = s - a - b and forms
// E_i = A_ii - sum over -z, -y, -x of (A_ik E_k^{-1}) U_ki from the values its
// neighbours held one step earlier (shuffled), reading each step's blocks
// from the packed layout (1 KB per load instruction), and E_i^{-1} by
// Gauss-Jordan with partial pivoting.
__global__ void __launch_bounds__(kBlock) k_ilu_pack(TileGeom T, const double *__restrict__ A,
                                                     double2 *__restrict__ Ff, double2 *__restrict__ Fb,
                                                     int32_t *__restrict__ slot_of) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T.slots()) return;
    const int t = (int)(q % 64);
    const long long ts = q / 64;
    const int s = (int)(ts % T.ns), tile = (int)(ts / T.ns);
    const int a = t % T.tx, b = t / T.tx;
    const int ti = tile % T.ntx, tj = tile / T.ntx;
    const int i = ti * T.tx + a, j = tj * T.ty + b, k = s - a - b;
    if (!(t < T.tx * T.ty && i < T.nx && j < T.ny && k >= 0 && k < T.nz)) return;  // idle slot
    const bool has_mx = a > 0, has_my = b > 0;
    const bool has_px = a + 1 < T.tx && i + 1 < T.nx, has_py = b + 1 < T.ty && j + 1 < T.ny;
    const size_t N = (size_t)T.nx * T.ny * T.nz;
    const int g = i + T.nx * (j + T.ny * k);
    double fw[36], bw[36];
#pragma unroll
    for (int z = 0; z < 36; z++) fw[z] = bw[z] = 0.0;
    load_blk(A, S_D, N, g, fw);
    if (k > 0) load_blk(A, S_MZ, N, g, fw + 9);
    if (has_my) load_blk(A, S_MY, N, g, fw + 18);
    if (has_mx) load_blk(A, S_MX, N, g, fw + 27);
    if (k + 1 < T.nz) load_blk(A, S_PZ, N, g, bw + 9);
    if (has_px) load_blk(A, S_PX, N, g, bw + 18);
    if (has_py) load_blk(A, S_PY, N, g, bw + 27);
#pragma unroll
    for (int p2 = 0; p2 < kPairs; p2++) {
        Ff[pk_index(tile, T.ns, s, p2, t)] = make_double2(fw[2 * p2], fw[2 * p2 + 1]);
        if (p2 >= 4) Fb[pk_index(tile, T.ns, s, p2, t)] = make_double2(bw[2 * p2], bw[2 * p2 + 1]);
    }
    slot_of[g] = (int32_t)q;
}

// The same pack straight from a BSR matrix whose first N block rows are the
// grid's cells, each row's stencil blocks first in ascending column order
// (the extended grid form; later columns, matrix cells or wells, follow):
// the thread reads its cell's row (contiguous blocks) instead of 63 slot
// planes.  A stencil neighbour missing from the row raises *bad.
__global__ void __launch_bounds__(kBlock) k_ilu_pack_bsr(TileGeom T, const int32_t *__restrict__ rp,
                                                         const int32_t *__restrict__ ci,
                                                         const double *__restrict__ v, double2 *__restrict__ Ff,
                                                         double2 *__restrict__ Fb, int32_t *__restrict__ slot_of,
                                                         int32_t *__restrict__ bad) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= T.slots()) return;
    const int t = (int)(q % 64);
    const long long ts = q / 64;
    const int s = (int)(ts % T.ns), tile = (int)(ts / T.ns);
    const int a = t % T.tx, b = t / T.tx;
    const int ti = tile % T.ntx, tj = tile / T.ntx;
    const int i = ti * T.tx + a, j = tj * T.ty + b, k = s - a - b;
    if (!(t < T.tx * T.ty && i < T.nx && j < T.ny && k >= 0 && k < T.nz)) return;  // idle slot
    const int g = i + T.nx * (j + T.ny * k);
    // grid neighbours present (slot order) and the blocks the tile keeps
    const unsigned have = (k > 0 ? 1u << S_MZ : 0u) | (j > 0 ? 1u << S_MY : 0u) | (i > 0 ? 1u << S_MX : 0u) |
                          (1u << S_D) | (i + 1 < T.nx ? 1u << S_PX : 0u) | (j + 1 < T.ny ? 1u << S_PY : 0u) |
                          (k + 1 < T.nz ? 1u << S_PZ : 0u);
    const unsigned keep = (k > 0 ? 1u << S_MZ : 0u) | (b > 0 ? 1u << S_MY : 0u) | (a > 0 ? 1u << S_MX : 0u) |
                          (1u << S_D) | (a + 1 < T.tx && i + 1 < T.nx ? 1u << S_PX : 0u) |
                          (b + 1 < T.ty && j + 1 < T.ny ? 1u << S_PY : 0u) | (k + 1 < T.nz ? 1u << S_PZ : 0u);
    const int e0 = rp[g], e1 = rp[g + 1];
    const int nxy = T.nx * T.ny;
    const int nb[NSLOT] = {g - nxy, g - T.nx, g - 1, g, g + 1, g + T.nx, g + nxy};
    int pos[NSLOT];
    int c[NSLOT];
#pragma unroll
    for (int sl = 0; sl < NSLOT; sl++) {
        pos[sl] = e0 + __popc(have & ((1u << sl) - 1u));
        c[sl] = (have >> sl) & 1u ? ci[min(pos[sl], e1 - 1)] : -1;
    }
    bool ok = true;
#pragma unroll
    for (int sl = 0; sl < NSLOT; sl++)
        if ((have >> sl) & 1u) ok = ok && pos[sl] < e1 && c[sl] == nb[sl];
    if (!ok) {
        *bad = 1;
        return;
    }
    // fw = [A_ii | -z | -y | -x], bw[9..35] = [+z | +x | +y]; zero blocks outside the tile
    const int fsl[4] = {S_D, S_MZ, S_MY, S_MX}, bsl[3] = {S_PZ, S_PX, S_PY};
    double fw[36], bw[27];
#pragma unroll
    for (int u = 0; u < 4; u++) {
        const bool k_ = (keep >> fsl[u]) & 1u;
        const double *src = v + 9 * (size_t)(k_ ? pos[fsl[u]] : e0);
#pragma unroll
        for (int z = 0; z < 9; z++) fw[9 * u + z] = k_ ? src[z] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 3; u++) {
        const bool k_ = (keep >> bsl[u]) & 1u;
        const double *src = v + 9 * (size_t)(k_ ? pos[bsl[u]] : e0);
#pragma unroll
        for (int z = 0; z < 9; z++) bw[9 * u + z] = k_ ? src[z] : 0.0;
    }
#pragma unroll
    for (int p2 = 0; p2 < kPairs; p2++) {
        Ff[pk_index(tile, T.ns, s, p2, t)] = make_double2(fw[2 * p2], fw[2 * p2 + 1]);
        if (p2 >= 5) Fb[pk_index(tile, T.ns, s, p2, t)] = make_double2(bw[2 * p2 - 9], bw[2 * p2 - 8]);
    }
    // pair 4 of the backward slot: (E^{-1}[8], +z[0]); the chain writes E^{-1}
    Fb[pk_index(tile, T.ns, s, 4, t)] = make_double2(0.0, bw[0]);
    slot_of[g] = (int32_t)q;
}

// one slot of the FP32 / BF16 forms: values 0..8 from e, 9..35 from r (the
// three blocks of A), rounded to nearest
template <int St>
__device__ __forceinline__ void store_mixed(void *F, int tile, int ns, int s, int t, const double *e,
                                            const double *r) {
#pragma unroll
    for (int qd = 0; qd < kQuads; qd++) {
        float f[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int z = 4 * qd + u;
            f[u] = (float)(z < 9 ? e[z] : r[z - 9]);
        }
        if constexpr (St == ST_F32) {
            ((float4 *)F)[pq_index(tile, ns, s, qd, t)] = make_float4(f[0], f[1], f[2], f[3]);
        } else {
            ((uint2 *)F)[pq_index(tile, ns, s, qd, t)] =
                make_uint2(bf16_bits(f[0]) | (bf16_bits(f[1]) << 16), bf16_bits(f[2]) | (bf16_bits(f[3]) << 16));
        }
    }
}

// FP64 form: E^{-1} and the unit-lower factors over the packed input (Ff,
// Fb).  FP32 / BF16 forms: the packed input is left as it is and each slot
// is stored rounded into Of ([E^{-1} | Az Ay Ax]) and Ob ([E^{-1} | Uz Ux
// Uy]), the blocks of A as the sweeps of those forms take them.
template <int St>
__global__ void __launch_bounds__(64) k_ilu_chain(TileGeom T, double2 *__restrict__ Ff, double2 *__restrict__ Fb,
                                                  int32_t *__restrict__ bad, double *__restrict__ einv_nat,
                                                  void *__restrict__ Of, void *__restrict__ Ob) {
    int t = threadIdx.x;
    int a = t % T.tx, b = t / T.tx;
    int tile = blockIdx.x;
    int ti = tile % T.ntx, tj = tile / T.ntx;
    int i = ti * T.tx + a, j = tj * T.ty + b;
    bool active = t < T.tx * T.ty && i < T.nx && j < T.ny;
    bool has_mx = a > 0, has_my = b > 0;
    size_t N = (size_t)T.nx * T.ny * T.nz;
    double Ep[9], Uxp[9], Uyp[9], Uzp[9];  // this lane's values from the previous step
    for (int z = 0; z < 9; z++) Ep[z] = Uxp[z] = Uyp[z] = Uzp[z] = 0.0;
    // a step's 63 values, loaded one step ahead into a ring of two buffers
    // (the loop is unrolled by two so that no buffer is copied: a copy of
    // registers with loads in flight makes the compiler wait for all of them)
    struct Slot {
        double fw[36], uw[27];
    };
    auto fetch = [&](int s, Slot &S) {
        const int sc = min(s, T.ns - 1);
        const int k = sc - a - b;
        // every lane loads (idle lanes read lane 0's slot) so that no load
        // is skipped on some paths
        const int tl = active && k >= 0 && k < T.nz ? t : 0;
#pragma unroll
        for (int p2 = 0; p2 < kPairs; p2++) {
            double2 d = Ff[pk_index(tile, T.ns, sc, p2, tl)];
            S.fw[2 * p2] = d.x;
            S.fw[2 * p2 + 1] = d.y;
        }
        double2 d = Fb[pk_index(tile, T.ns, sc, 4, tl)];
        S.uw[0] = d.y;
#pragma unroll
        for (int p2 = 5; p2 < kPairs; p2++) {
            double2 e = Fb[pk_index(tile, T.ns, sc, p2, tl)];
            S.uw[2 * p2 - 9] = e.x;
            S.uw[2 * p2 - 8] = e.y;
        }
    };
    auto step = [&](int s, const Slot &S) {
        double Ex[9], Ey[9], Ux[9], Uy[9];
        shfl_arr<9>(Ep, Ex, has_mx ? t - 1 : t);
        shfl_arr<9>(Uxp, Ux, has_mx ? t - 1 : t);
        shfl_arr<9>(Ep, Ey, has_my ? t - T.tx : t);
        shfl_arr<9>(Uyp, Uy, has_my ? t - T.tx : t);
        int k = s - a - b;
        const bool act = active && k >= 0 && k < T.nz;
        const double *fw = S.fw, *uw = S.uw;
        if (act) {
            // lw: E^{-1}[8] and the unit-lower factors L_ik = A_ik E_k^{-1}
            // (-z, -y, -x) as values 8..35 of the forward slot
            double E[9], lw[28], tmp[9];
            for (int z = 0; z < 28; z++) lw[z] = 0.0;
            for (int z = 0; z < 9; z++) E[z] = fw[z];
            // -z, -y, -x in ascending order (zero blocks where missing)
            if (k > 0) {
                mul3(fw + 9, Ep, lw + 1); mul3(lw + 1, Uzp, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
            }
            if (has_my) {
                mul3(fw + 18, Ey, lw + 10); mul3(lw + 10, Uy, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
            }
            if (has_mx) {
                mul3(fw + 27, Ex, lw + 19); mul3(lw + 19, Ux, tmp);
                for (int z = 0; z < 9; z++) E[z] = E[z] - tmp[z];
            }
            double Ei[9];
            if (!inv3_gj(E, Ei)) {
                *bad = 1;
                for (int z = 0; z < 9; z++) Ei[z] = 0.0;
            }
            for (int z = 0; z < 9; z++) Ep[z] = Ei[z];
            if (einv_nat) {
                const int g = i + T.nx * (j + T.ny * k);
                for (int z = 0; z < 9; z++) einv_nat[(size_t)z * N + g] = Ei[z];
            }
            if constexpr (St != ST_F64) {
                store_mixed<St>(Of, tile, T.ns, s, t, Ei, fw + 9);
                store_mixed<St>(Ob, tile, T.ns, s, t, Ei, uw);
                for (int z = 0; z < 9; z++) { Uzp[z] = uw[z]; Uxp[z] = uw[9 + z]; Uyp[z] = uw[18 + z]; }
                return;
            }
            // E^{-1} into values 0..8 of the backward slot, the lower factors
            // over the forward slot's blocks of A (its values 0..7, A_ii, are
            // not read again)
#pragma unroll
            for (int p2 = 0; p2 < 4; p2++)
                Fb[pk_index(tile, T.ns, s, p2, t)] = make_double2(Ei[2 * p2], Ei[2 * p2 + 1]);
            ((double *)&Fb[pk_index(tile, T.ns, s, 4, t)])[0] = Ei[8];
            lw[0] = Ei[8];
#pragma unroll
            for (int p2 = 4; p2 < kPairs; p2++)
                Ff[pk_index(tile, T.ns, s, p2, t)] = make_double2(lw[2 * p2 - 8], lw[2 * p2 - 7]);
            // this cell's upper blocks for the next step's neighbours
            for (int z = 0; z < 9; z++) { Uzp[z] = uw[z]; Uxp[z] = uw[9 + z]; Uyp[z] = uw[18 + z]; }
        }
    };
    Slot R0, R1;
    fetch(0, R0);
    int s0 = 0;
    for (; s0 + 2 <= T.ns; s0 += 2) {
        fetch(s0 + 1, R1);
        step(s0, R0);
        fetch(s0 + 2, R0);
        step(s0 + 1, R1);
    }
    if (s0 < T.ns) step(s0, R0);
}

// One half of a slot's 36 factor values: half 0 = values 0..17 (E^{-1} and
// the first block), half 1 = values 18..35 (the other two blocks).  In the
// FP32 / BF16 forms the quad holding values 16..19 is read by both halves.
template <typename T>
struct Half {
    T v[18];
};
template <int St, typename T, int H>
__device__ __forceinline__ void load_half(const void *__restrict__ F, int tile, int ns, int s, int t, Half<T> &p) {
    // (callers pass lane 0 for idle slots: all idle lanes of a load then hit
    // one cache line)
    if constexpr (St == ST_F64) {
        const double2 *D = (const double2 *)F;
#pragma unroll
        for (int i = 0; i < 9; i++) {
            double2 d = D[pk_index(tile, ns, s, 9 * H + i, t)];
            p.v[2 * i] = d.x;
            p.v[2 * i + 1] = d.y;
        }
    } else {
        T u[20];
#pragma unroll
        for (int i = 0; i < 5; i++) {
            int qd = 4 * H + i;
            if constexpr (St == ST_F32) {
                float4 f = ((const float4 *)F)[pq_index(tile, ns, s, qd, t)];
                u[4 * i] = f.x; u[4 * i + 1] = f.y; u[4 * i + 2] = f.z; u[4 * i + 3] = f.w;
            } else {
                uint2 b = ((const uint2 *)F)[pq_index(tile, ns, s, qd, t)];
                u[4 * i] = bf16_value(b.x & 0xFFFFu); u[4 * i + 1] = bf16_value(b.x >> 16);
                u[4 * i + 2] = bf16_value(b.y & 0xFFFFu); u[4 * i + 3] = bf16_value(b.y >> 16);
            }
        }
        // half 0: values 0..17 = u[0..17]; half 1: values 18..35 = u[2..19]
#pragma unroll
        for (int i = 0; i < 18; i++) p.v[i] = u[i + 2 * H];
    }
}

// the FP64 forward slot's -z factor (values 9..17, with value 8) into
// p.v[8..17]: pairs 4..8 only
__device__ __forceinline__ void load_lz(const void *__restrict__ F, int tile, int ns, int s, int t,
                                        Half<double> &p) {
    const double2 *D = (const double2 *)F;
#pragma unroll
    for (int i = 4; i < 9; i++) {
        double2 d = D[pk_index(tile, ns, s, i, t)];
        p.v[2 * i] = d.x;
        p.v[2 * i + 1] = d.y;
    }
}

// the sweep's vector operand at one slot (three arrays S apart)
template <typename T>
__device__ __forceinline__ void load_vec(const T *__restrict__ vec, size_t S, size_t q, T *w) {
    w[0] = vec[q]; w[1] = vec[S + q]; w[2] = vec[2 * S + q];
}

// Sweeps: two wavefronts per tile.  Wavefront 0 loads the first half of each
// slot's factors (E^{-1} and the -z block forward, only the -z factor in the
// FP64 form; E^{-1} and the +z block backward) with the vector operand,
// wavefront 1 the second half (the -y and
// -x blocks; the +x and +y blocks), so each keeps its own steps of loads in
// flight.  Per step, wavefront 1 multiplies its
// blocks with the neighbours' values of the previous step (read from LDS) and
// hands the products to wavefront 0 through LDS; wavefront 0 completes the
// step and hands the new values back.  The products are combined in the
// order of the one-wavefront formula, so the results do not change.  Idle
// slots (column outside the tile or grid, layer outside 0..nz-1) load
// nothing.
struct SweepLane {
    int t, a, b;
    bool col_ok;
    __device__ SweepLane(const TileGeom &G, int tile, int lane) : t(lane) {
        a = lane % G.tx;
        b = lane / G.tx;
        int ti = tile % G.ntx, tj = tile / G.ntx;
        col_ok = lane < G.tx * G.ty && ti * G.tx + a < G.nx && tj * G.ty + b < G.ny;
    }
    __device__ bool active(const TileGeom &G, int s) const {
        int k = s - a - b;
        return col_ok && k >= 0 && k < G.nz;
    }
    // the grid cell of an active slot (the factorisation's cell index)
    __device__ size_t cell(const TileGeom &G, int tile, int s) const {
        int i = (tile % G.ntx) * G.tx + a, j = (tile / G.ntx) * G.ty + b, k = s - a - b;
        return (size_t)i + (size_t)G.nx * ((size_t)j + (size_t)G.ny * k);
    }
};

// Each wavefront keeps a ring of register buffers, one per step in flight;
// the step loop is unrolled by the ring length, so a buffer is refilled in
// place once its step is done and no register holding a load in flight is
// ever copied (a copy would have to wait for the load).  Every lane loads at
// every step (idle slots and steps past the end read lane 0's data of a
// valid step of the tile and ignore it, so the idle lanes of a load share one
// cache line): loads that some paths skip would make the compiler wait for
// all outstanding loads before using any of them.
// Two steps ahead in both wavefronts: the sweeps then take about 140
// registers and three tiles' wavefronts share a SIMD (with rings of four and
// six steps, 248 registers and two), and the extra tiles in flight hide the
// latency better than longer rings (measured on the 32M-cell workload, same
// on the 500k- and 2M-cell ones).  A ring of one step (64 and 78 registers,
// every tile of a 400x400 grid resident at once) measured the same as two.
constexpr int kAhead0 = 2;  // wavefront 0: its factor and vector loads per step
constexpr int kAhead1 = 2;  // wavefront 1: 9 factor loads per step

// forward sweep: FP64: y = r - sum_lower L y_lower with the unit-lower
// factors L_ik = A_ik E_k^{-1}; FP32 / BF16: w = E^{-1}(r - sum_lower A w_lower)
// (w = E^{-1} y).  r (FP64) in natural order, read at the slot's cell and
// rounded to T; the result in (tile, step, lane) order
template <int St, typename T>
__global__ void __launch_bounds__(128) k_ilu_forward(TileGeom G, const void *__restrict__ F,
                                                     const double *__restrict__ r,
                                                     T *__restrict__ wq) {
    __shared__ T wsh[2][3][64];  // w of a step, by step parity
    __shared__ T ysh[2][6][64];  // wavefront 1's products L_y w_y and L_x w_x
    const int wv = threadIdx.x / 64;
    const int tile = blockIdx.x;
    const SweepLane L(G, tile, threadIdx.x % 64);
    const int t = L.t;
    const size_t S = (size_t)G.slots();
    const int ns = G.ns;
    if (wv == 1) {
        const int lx = L.a > 0 ? t - 1 : t, ly = L.b > 0 ? t - G.tx : t;
        Half<T> buf[kAhead1];
        auto fetch = [&](int s, Half<T> &h) {
            const int sc = min(s, ns - 1);
            load_half<St, T, 1>(F, tile, ns, sc, L.active(G, sc) ? t : 0, h);
        };
        auto step = [&](int s, Half<T> &h) {
            T wy[3] = {0, 0, 0}, wx[3] = {0, 0, 0};
            if (s > 0) {
                const int p = (s - 1) & 1;
                for (int c = 0; c < 3; c++) { wy[c] = wsh[p][c][ly]; wx[c] = wsh[p][c][lx]; }
            }
            T ya[3] = {0, 0, 0}, yb[3] = {0, 0, 0};
            if (L.active(G, s)) {
                mv3(h.v, wy, ya);
                mv3(h.v + 9, wx, yb);
            }
            fetch(s + kAhead1, h);
            for (int c = 0; c < 3; c++) { ysh[s & 1][c][t] = ya[c]; ysh[s & 1][3 + c][t] = yb[c]; }
            __syncthreads();  // products of step s published
            __syncthreads();  // w of step s published
        };
#pragma unroll
        for (int u = 0; u < kAhead1; u++) fetch(u, buf[u]);
        int s0 = 0;
        for (; s0 + kAhead1 <= ns; s0 += kAhead1) {
#pragma unroll
            for (int u = 0; u < kAhead1; u++) step(s0 + u, buf[u]);
        }
#pragma unroll
        for (int u = 0; u < kAhead1; u++)
            if (s0 + u < ns) step(s0 + u, buf[u]);
    } else {
        T wp[3] = {0, 0, 0};
        Half<T> buf[kAhead0];
        T vec[kAhead0][3];
        auto fetch = [&](int s, Half<T> &h, T *w) {
            const int sc = min(s, ns - 1);
            const bool act = L.active(G, sc);
            if constexpr (St == ST_F64) load_lz(F, tile, ns, sc, act ? t : 0, h);
            else load_half<St, T, 0>(F, tile, ns, sc, act ? t : 0, h);
            const double *rg = r + 3 * (act ? L.cell(G, tile, sc) : 0);
            w[0] = (T)rg[0]; w[1] = (T)rg[1]; w[2] = (T)rg[2];
        };
        auto step = [&](int s, Half<T> &h, T *w) {
            __syncthreads();  // products of step s published
            if (L.active(G, s)) {
                T v[3] = {w[0], w[1], w[2]};
                T y[3];
                // zero blocks stand for missing neighbours
                mv3(h.v + 9, wp, y); v[0] = v[0] - y[0]; v[1] = v[1] - y[1]; v[2] = v[2] - y[2];
                v[0] = v[0] - ysh[s & 1][0][t]; v[1] = v[1] - ysh[s & 1][1][t]; v[2] = v[2] - ysh[s & 1][2][t];
                v[0] = v[0] - ysh[s & 1][3][t]; v[1] = v[1] - ysh[s & 1][4][t]; v[2] = v[2] - ysh[s & 1][5][t];
                if constexpr (St == ST_F64) {
                    wp[0] = v[0]; wp[1] = v[1]; wp[2] = v[2];
                } else {
                    mv3(h.v, v, wp);
                }
            } else {
                wp[0] = wp[1] = wp[2] = 0;
            }
            for (int c = 0; c < 3; c++) wsh[s & 1][c][t] = wp[c];
            {  // idle slots store 0
                size_t q = ((size_t)tile * ns + s) * 64 + t;
                wq[q] = wp[0]; wq[S + q] = wp[1]; wq[2 * S + q] = wp[2];
            }
            fetch(s + kAhead0, h, w);
            __syncthreads();  // w of step s published
        };
#pragma unroll
        for (int u = 0; u < kAhead0; u++) fetch(u, buf[u], vec[u]);
        int s0 = 0;
        for (; s0 + kAhead0 <= ns; s0 += kAhead0) {
#pragma unroll
            for (int u = 0; u < kAhead0; u++) step(s0 + u, buf[u], vec[u]);
        }
#pragma unroll
        for (int u = 0; u < kAhead0; u++)
            if (s0 + u < ns) step(s0 + u, buf[u], vec[u]);
    }
}

// backward sweep: FP64: x_i = E_i^{-1}(y_i - sum_{upper} A_ij x_j); FP32 /
// BF16: x_i = w_i - E_i^{-1} sum_{upper} A_ij x_j; written in natural order as
// out = x + (dp, 0, 0) in FP64 (dp may be NULL).
// Output staging (D > 0, D = tile_x + tile_y - 1 layers of 64 x 3 doubles in
// dynamic LDS): lane (a, b) finishes layer k at step k + a + b, so the layers
// in flight at step s are s .. s + D - 1 and layer s is complete once step s
// is.  Wavefront 0 puts each result into the layer's ring slot (k mod D);
// wavefront 1, at the start of step s - 1 (after step s's last barrier),
// writes layer s of the tile to HBM as tile_y rows of 3 tile_x contiguous
// doubles, and layer 0 after the last step.  A slot is next written at step
// s - 1 after that step's first barrier, which orders it after the write-out.
// Without staging (D == 0) every lane writes its 24 bytes at its cell, and the
// partial lines cost HBM writes of more than twice the output's size.
// With zin != NULL the result is added to it: out = zin + (x + (dp, 0, 0))
// (zin may be out itself: each cell is read and written by one thread).
template <int St, typename T, typename TD>
__global__ void __launch_bounds__(128) k_ilu_backward(TileGeom G, const void *__restrict__ F,
                                                      const T *__restrict__ wq,
                                                      const TD *__restrict__ dp, double *out,
                                                      int D, const double *zin) {
    __shared__ T xsh[2][3][64];  // x of a step, by step parity
    __shared__ T ash[2][3][64];  // wavefront 1's U_x x_x + U_y x_y
    extern __shared__ double obuf[];  // D slots of [lane][3]
    const int wv = threadIdx.x / 64;
    const int tile = blockIdx.x;
    const SweepLane L(G, tile, threadIdx.x % 64);
    const int t = L.t;
    const size_t S = (size_t)G.slots();
    const int ns = G.ns, e = G.ns - 1;
    if (wv == 1) {
        const int px = L.a + 1 < G.tx && t + 1 < 64 ? t + 1 : t;
        const int py = L.b + 1 < G.ty && t + G.tx < 64 ? t + G.tx : t;
        Half<T> buf[kAhead1];
        auto fetch = [&](int s, Half<T> &h) {
            const int sc = max(s, 0);
            load_half<St, T, 1>(F, tile, ns, sc, L.active(G, sc) ? t : 0, h);
        };
        // layer k of the tile from its ring slot to HBM
        const int i0 = (tile % G.ntx) * G.tx, j0 = (tile / G.ntx) * G.ty;
        const int rowlen = 3 * G.tx, tot = rowlen * G.ty;
        auto flush = [&](int k) {
            if (D == 0 || k >= G.nz) return;
            const double *ob = obuf + (size_t)(k % D) * 192;
            for (int q = t; q < tot; q += 64) {
                const int b = q / rowlen, rem = q - b * rowlen, a = rem / 3;
                if (i0 + a < G.nx && j0 + b < G.ny) {
                    const size_t g0 = (size_t)i0 + (size_t)G.nx * ((size_t)(j0 + b) + (size_t)G.ny * k);
                    const double o = ob[3 * (a + G.tx * b) + (rem - 3 * a)];
                    out[3 * g0 + rem] = zin ? zin[3 * g0 + rem] + o : o;
                }
            }
        };
        auto step = [&](int s, Half<T> &h) {
            flush(s + 1);
            T xx[3] = {0, 0, 0}, xy[3] = {0, 0, 0};
            if (s < e) {
                const int p = (s + 1) & 1;
                for (int c = 0; c < 3; c++) { xx[c] = xsh[p][c][px]; xy[c] = xsh[p][c][py]; }
            }
            T acc[3] = {0, 0, 0};
            if (L.active(G, s)) {
                T y[3];
                mv3(h.v, xx, acc);
                mv3(h.v + 9, xy, y); acc[0] = acc[0] + y[0]; acc[1] = acc[1] + y[1]; acc[2] = acc[2] + y[2];
            }
            fetch(s - kAhead1, h);
            for (int c = 0; c < 3; c++) ash[s & 1][c][t] = acc[c];
            __syncthreads();  // products of step s published
            __syncthreads();  // x of step s published
        };
#pragma unroll
        for (int u = 0; u < kAhead1; u++) fetch(e - u, buf[u]);
        int s0 = e;
        for (; s0 - kAhead1 + 1 >= 0; s0 -= kAhead1) {
#pragma unroll
            for (int u = 0; u < kAhead1; u++) step(s0 - u, buf[u]);
        }
#pragma unroll
        for (int u = 0; u < kAhead1; u++)
            if (s0 - u >= 0) step(s0 - u, buf[u]);
        flush(0);
    } else {
        T xp[3] = {0, 0, 0};
        Half<T> buf[kAhead0];
        T vec[kAhead0][3];
        TD dpv[kAhead0];
        // dp of the slot's cell is loaded with the slot (a load waited for
        // inside the step would wait for every load in flight)
        auto fetch = [&](int s, Half<T> &h, T *w, TD &d) {
            const int sc = max(s, 0);
            const bool act = L.active(G, sc);
            const int tl = act ? t : 0;
            load_half<St, T, 0>(F, tile, ns, sc, tl, h);
            load_vec(wq, S, ((size_t)tile * ns + sc) * 64 + tl, w);
            if (dp) d = dp[act ? L.cell(G, tile, sc) : 0];
        };
        auto step = [&](int s, Half<T> &h, T *w, TD &d) {
            __syncthreads();  // products of step s published
            if (L.active(G, s)) {
                T acc[3], y[3];
                acc[0] = ash[s & 1][0][t]; acc[1] = ash[s & 1][1][t]; acc[2] = ash[s & 1][2][t];
                mv3(h.v + 9, xp, y); acc[0] = acc[0] + y[0]; acc[1] = acc[1] + y[1]; acc[2] = acc[2] + y[2];
                if constexpr (St == ST_F64) {
                    y[0] = w[0] - acc[0]; y[1] = w[1] - acc[1]; y[2] = w[2] - acc[2];
                    mv3(h.v, y, xp);
                } else {
                    mv3(h.v, acc, y);
                    xp[0] = w[0] - y[0]; xp[1] = w[1] - y[1]; xp[2] = w[2] - y[2];
                }
            } else {
                xp[0] = xp[1] = xp[2] = 0;
            }
            for (int c = 0; c < 3; c++) xsh[s & 1][c][t] = xp[c];
            if (L.active(G, s)) {
                const double o0 = dp ? (double)d + (double)xp[0] : (double)xp[0];
                if (D > 0) {
                    double *ob = obuf + (size_t)((s - L.a - L.b) % D) * 192 + 3 * t;
                    ob[0] = o0;
                    ob[1] = (double)xp[1];
                    ob[2] = (double)xp[2];
                } else {
                    size_t g = L.cell(G, tile, s);
                    if (zin) {
                        out[3 * g] = zin[3 * g] + o0;
                        out[3 * g + 1] = zin[3 * g + 1] + (double)xp[1];
                        out[3 * g + 2] = zin[3 * g + 2] + (double)xp[2];
                    } else {
                        out[3 * g] = o0;
                        out[3 * g + 1] = (double)xp[1];
                        out[3 * g + 2] = (double)xp[2];
                    }
                }
            }
            fetch(s - kAhead0, h, w, d);
            __syncthreads();  // x of step s published
        };
#pragma unroll
        for (int u = 0; u < kAhead0; u++) fetch(e - u, buf[u], vec[u], dpv[u]);
        int s0 = e;
        for (; s0 - kAhead0 + 1 >= 0; s0 -= kAhead0) {
#pragma unroll
            for (int u = 0; u < kAhead0; u++) step(s0 - u, buf[u], vec[u], dpv[u]);
        }
#pragma unroll
        for (int u = 0; u < kAhead0; u++)
            if (s0 - u >= 0) step(s0 - u, buf[u], vec[u], dpv[u]);
    }
}

template <int St>
__global__ void k_bj_setup(long long n, const double *__restrict__ A, void *__restrict__ einv,
                           int32_t *__restrict__ bad) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t N = (size_t)n;
    double E[9], Ei[9];
    load_blk(A, S_D, N, (int)g, E);
    if (!inv3_gj(E, Ei)) {
        *bad = 1;
        for (int z = 0; z < 9; z++) Ei[z] = 0.0;
    }
    for (int z = 0; z < 9; z++) {
        if constexpr (St == ST_F64) ((double *)einv)[(size_t)z * N + g] = Ei[z];
        else if constexpr (St == ST_F32) ((float *)einv)[(size_t)z * N + g] = (float)Ei[z];
        else ((uint16_t *)einv)[(size_t)z * N + g] = (uint16_t)bf16_bits((float)Ei[z]);
    }
}

// the same from a general BSR matrix (diagonal block located in each row)
template <int St>
__global__ void k_bj_setup_bsr(long long n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                               const double *__restrict__ val, void *__restrict__ einv, int32_t *__restrict__ bad) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t N = (size_t)n;
    int e = rp[g];
    while (e < rp[g + 1] && ci[e] != (int)g) e++;
    double E[9], Ei[9];
    if (e == rp[g + 1]) {
        *bad = 1;
        for (int z = 0; z < 9; z++) Ei[z] = 0.0;
    } else {
        for (int z = 0; z < 9; z++) E[z] = val[9 * (size_t)e + z];
        if (!inv3_gj(E, Ei)) {
            *bad = 1;
            for (int z = 0; z < 9; z++) Ei[z] = 0.0;
        }
    }
    for (int z = 0; z < 9; z++) {
        if constexpr (St == ST_F64) ((double *)einv)[(size_t)z * N + g] = Ei[z];
        else if constexpr (St == ST_F32) ((float *)einv)[(size_t)z * N + g] = (float)Ei[z];
        else ((uint16_t *)einv)[(size_t)z * N + g] = (uint16_t)bf16_bits((float)Ei[z]);
    }
}

template <int St, typename T, typename TD>
__global__ void k_bj_apply(long long n, const void *__restrict__ einv, const double *__restrict__ r,
                           const TD *__restrict__ dp, double *__restrict__ out) {
    long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t N = (size_t)n;
    T Ei[9], v[3] = {(T)r[3 * g], (T)r[3 * g + 1], (T)r[3 * g + 2]}, o[3];
    for (int z = 0; z < 9; z++) {
        if constexpr (St == ST_F64) Ei[z] = ((const double *)einv)[(size_t)z * N + g];
        else if constexpr (St == ST_F32) Ei[z] = ((const float *)einv)[(size_t)z * N + g];
        else Ei[z] = bf16_value(((const uint16_t *)einv)[(size_t)z * N + g]);
    }
    mv3(Ei, v, o);
    out[3 * g] = dp ? (double)dp[g] + (double)o[0] : (double)o[0];
    out[3 * g + 1] = (double)o[1];
    out[3 * g + 2] = (double)o[2];
}

int store_of(const bo_cpr *pc) {
    return pc->o.precision == BO_PREC_FP64 ? ST_F64 : pc->o.precision == BO_PREC_FP32 ? ST_F32 : ST_BF16;
}

// ---- the extended grid form: dual porosity and well rows -----------------------
// Block ILU(0) of the whole system ordered tile by tile: a tile's fracture
// cells (wavefront order as above), then their matrix cells, and the well rows
// as one class of their own after every tile (their couplings to the cells
// dropped, like the couplings between tiles).  A matrix cell's only lower
// neighbour is its fracture cell, so its pivot is E_m = A_mm - (A_mf E_f^{-1})
// A_fm, and a fracture cell's only extra upper neighbour is its matrix cell
// (matrix cells exist in the FP64 form only):
//   forward   y_f (tiles),  y_m = r_m - (A_mf E_f^{-1}) y_f
//   backward  x_m = E_m^{-1} y_m,  x_f = E_f^{-1} (y_f - A_fm x_m - sum_stencil A x)
// The term A_fm x_m is taken out of y_f before the tile's backward sweep.

// matrix pivots E_m^{-1} and the coupling blocks A_mf (row N+g, col g) and
// A_fm (row g, col N+g), SoA 9 x N
__global__ void k_dual_pivots(int n, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                              const double *__restrict__ v, const double *__restrict__ einv_f,
                              double *__restrict__ einv_m, double *__restrict__ amf, double *__restrict__ afm,
                              int32_t *__restrict__ bad) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t N = (size_t)n;
    int ef = rp[g];
    while (ef < rp[g + 1] && ci[ef] != n + g) ef++;
    int em = rp[n + g];  // row N+g holds (g, N+g)
    if (ef == rp[g + 1] || rp[n + g + 1] - em != 2 || ci[em] != g || ci[em + 1] != n + g) {
        *bad = 1;
        return;
    }
    double Af[9], Am[9], Amm[9], Ef[9], L[9], t[9], E[9], Ei[9];
    for (int z = 0; z < 9; z++) {
        Af[z] = v[9 * (size_t)ef + z];
        Am[z] = v[9 * (size_t)em + z];
        Amm[z] = v[9 * (size_t)(em + 1) + z];
        Ef[z] = einv_f[(size_t)z * N + g];
    }
    mul3(Am, Ef, L);
    mul3(L, Af, t);
    for (int z = 0; z < 9; z++) E[z] = Amm[z] - t[z];
    if (!inv3_gj(E, Ei)) {
        *bad = 1;
        for (int z = 0; z < 9; z++) Ei[z] = 0.0;
    }
    for (int z = 0; z < 9; z++) {
        einv_m[(size_t)z * N + g] = Ei[z];
        amf[(size_t)z * N + g] = Am[z];
        afm[(size_t)z * N + g] = Af[z];
    }
}

// inverses of the diagonal blocks of rows [r0, r0 + cnt) (the well rows), 9 x cnt
__global__ void k_rows_inv(int r0, int cnt, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                           const double *__restrict__ v, double *__restrict__ out, int32_t *__restrict__ bad) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cnt) return;
    int r = r0 + q;
    int e = rp[r];
    while (e < rp[r + 1] && ci[e] != r) e++;
    double E[9], Ei[9];
    if (e == rp[r + 1]) {
        *bad = 1;
        for (int z = 0; z < 9; z++) Ei[z] = 0.0;
    } else {
        for (int z = 0; z < 9; z++) E[z] = v[9 * (size_t)e + z];
        if (!inv3_gj(E, Ei)) {
            *bad = 1;
            for (int z = 0; z < 9; z++) Ei[z] = 0.0;
        }
    }
    for (int z = 0; z < 9; z++) out[(size_t)z * cnt + q] = Ei[z];
}

// forward step of the matrix cells and the fracture adjustment, on the FP64
// forward result y_f (slot order): x_m = E_m^{-1}(r_m - A_mf E_f^{-1} y_f)
// into out (the matrix cell's lower factor is A_mf E_f^{-1} and it has no
// upper neighbour), then y_f -= A_fm x_m (the fracture cell's coupling to its
// matrix cell, taken out before the tile's backward sweep)
__global__ void k_dual_forward(int n, const int32_t *__restrict__ slot_of, size_t S, const double *__restrict__ r,
                               const double *__restrict__ einv_m, const double *__restrict__ amf,
                               const double *__restrict__ afm, const double *__restrict__ einv_f,
                               double *__restrict__ wq, double *__restrict__ out) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    size_t N = (size_t)n;
    size_t q = (size_t)slot_of[g];
    double yf[3] = {wq[q], wq[S + q], wq[2 * S + q]};
    double B[9], wf[3], y[3], v3[3], xm[3];
    for (int z = 0; z < 9; z++) B[z] = einv_f[(size_t)z * N + g];
    mv3(B, yf, wf);
    for (int z = 0; z < 9; z++) B[z] = amf[(size_t)z * N + g];
    mv3(B, wf, y);
    for (int c = 0; c < 3; c++) v3[c] = r[3 * (N + g) + c] - y[c];
    for (int z = 0; z < 9; z++) B[z] = einv_m[(size_t)z * N + g];
    mv3(B, v3, xm);
    for (int c = 0; c < 3; c++) out[3 * (N + g) + c] = xm[c];
    for (int z = 0; z < 9; z++) B[z] = afm[(size_t)z * N + g];
    mv3(B, xm, y);
    wq[q] = yf[0] - y[0];
    wq[S + q] = yf[1] - y[1];
    wq[2 * S + q] = yf[2] - y[2];
}

// well rows: x_r = E_r^{-1} r_r; with zin != NULL out = zin + (x + (dp, 0, 0))
// (dp on the row's own index; zin may be out)
template <typename TD>
__global__ void k_rows_apply(int r0, int cnt, const double *__restrict__ inv, const double *__restrict__ r,
                             double *out, const TD *__restrict__ dp, const double *zin) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= cnt) return;
    size_t R = (size_t)(r0 + q);
    double B[9], v3[3] = {r[3 * R], r[3 * R + 1], r[3 * R + 2]}, o[3];
    for (int z = 0; z < 9; z++) B[z] = inv[(size_t)z * cnt + q];
    mv3(B, v3, o);
    if (dp) o[0] = (double)dp[R] + o[0];
    for (int c = 0; c < 3; c++) out[3 * R + c] = zin ? zin[3 * R + c] + o[c] : o[c];
}

// the backward sweep's output staging: tile_x + tile_y - 1 layers of 64
// cells x 3 doubles when they fit in 32 KB of LDS (tiles of 16x4, 8x8 and
// smaller), else direct writes
constexpr int kStageBytes = 64 * 3 * (int)sizeof(double);
inline int stage_layers(const TileGeom &G) {
    const int D = G.tx + G.ty - 1;
    return D * kStageBytes <= 32768 ? D : 0;
}

TileGeom geom(const bo_cpr *pc) {
    TileGeom T;
    T.nx = pc->g.nx; T.ny = pc->g.ny; T.nz = pc->g.nz;
    T.tx = pc->o.tile_x; T.ty = pc->o.tile_y;
    T.ntx = (T.nx + T.tx - 1) / T.tx;
    T.nty = (T.ny + T.ty - 1) / T.ty;
    T.ns = (T.tx - 1) + (T.ty - 1) + T.nz;
    return T;
}

}  // namespace

// Launches the F stage's factorisation on stream s and reads nothing back:
// its singular-pivot flag (pc->fflag) is read by fstage_check, so the
// factorisation can run on a stream of its own beside the AMG setup.
bo_status fstage_launch(bo_cpr *pc, hipStream_t s) {
    long long n = pc->n;
    int st = store_of(pc);
    BO_TRY(pc->fflag.alloc(1));
    int32_t *ff = pc->fflag.p;
    BO_HIP(hipMemsetAsync(ff, 0, sizeof(int32_t), s));
    if (pc->o.ftype == BO_F_ILU_NATURAL) return nat_launch(pc, s);
    if (pc->o.ftype == BO_F_BJ) {
        BO_TRY(pc->einv.alloc(9 * n));  // FP64 size: large enough for every format
        void *E = pc->einv.p;
        if (pc->general) {
            const int32_t *rp = pc->Arp.p, *ci = pc->Aci.p;
            const double *v = pc->Aval.p;
            if (st == ST_F64) k_bj_setup_bsr<ST_F64><<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, E, ff);
            else if (st == ST_F32) k_bj_setup_bsr<ST_F32><<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, E, ff);
            else k_bj_setup_bsr<ST_BF16><<<grid_for(n), kBlock, 0, s>>>(n, rp, ci, v, E, ff);
        } else if (st == ST_F64) k_bj_setup<ST_F64><<<grid_for(n), kBlock, 0, s>>>(n, pc->A.p, E, ff);
        else if (st == ST_F32) k_bj_setup<ST_F32><<<grid_for(n), kBlock, 0, s>>>(n, pc->A.p, E, ff);
        else k_bj_setup<ST_BF16><<<grid_for(n), kBlock, 0, s>>>(n, pc->A.p, E, ff);
    } else {
        TileGeom T = geom(pc);
        size_t S = (size_t)T.slots();
        const long long N = pc->g.n();
        const bool ext = pc->general;  // the extended grid form (extra matrix / well rows)
        if (ext) {
            // FP32 / BF16 factors: only without matrix cells (the tiles and the
            // well rows; a matrix cell's pivot needs its fracture cell's E^-1 in
            // natural order, which the FP64 chain writes)
            if (st != ST_F64 && pc->ncell > N)
                return fail(BO_ERR_UNSUPPORTED, "F stage: with matrix cells the extended form's ILU is FP64 only");
            if (st == ST_F64) BO_TRY(pc->x_einv_f.alloc(9 * N));
        }
        // factor buffers: FP64 packed (the FP64 form factors in place), or
        // the FP32 / BF16 layout (a float4 or uint2 per quad; sized for
        // float4) beside an FP64 packed copy that the factorisation reads
        const bool f64 = st == ST_F64;
        BO_TRY(pc->ilu_f.alloc(f64 ? S * kPairs : S * kQuads));
        BO_TRY(pc->ilu_b.alloc(f64 ? S * kPairs : S * kQuads));
        if (!f64) {
            BO_TRY(pc->ilu_pf.alloc(S * kPairs));
            BO_TRY(pc->ilu_pb.alloc(S * kPairs));
        }
        double2 *Pf = f64 ? pc->ilu_f.p : pc->ilu_pf.p, *Pb = f64 ? pc->ilu_b.p : pc->ilu_pb.p;
        BO_TRY(pc->ilu_slot.alloc(n));
        if (f64) BO_TRY(pc->ilu_w.alloc(3 * S));
        else BO_TRY(pc->ilu_w32.alloc(3 * S));
        // idle slots are never read by the sweeps: their factors stay unset
        int nb = T.ntx * T.nty;
        if (ext)
            k_ilu_pack_bsr<<<grid_for(T.slots()), kBlock, 0, s>>>(T, pc->Arp.p, pc->Aci.p, pc->Aval.p, Pf, Pb,
                                                                  pc->ilu_slot.p, ff);
        else
            k_ilu_pack<<<grid_for(T.slots()), kBlock, 0, s>>>(T, pc->A.p, Pf, Pb, pc->ilu_slot.p);
        if (f64)
            k_ilu_chain<ST_F64><<<nb, 64, 0, s>>>(T, Pf, Pb, ff, ext ? pc->x_einv_f.p : nullptr, nullptr, nullptr);
        else if (st == ST_F32)
            k_ilu_chain<ST_F32><<<nb, 64, 0, s>>>(T, Pf, Pb, ff, nullptr, pc->ilu_f.p, pc->ilu_b.p);
        else
            k_ilu_chain<ST_BF16><<<nb, 64, 0, s>>>(T, Pf, Pb, ff, nullptr, pc->ilu_f.p, pc->ilu_b.p);
        if (ext && pc->ncell > N) {
            BO_TRY(pc->x_einv_m.alloc(9 * N));
            BO_TRY(pc->x_amf.alloc(9 * N));
            BO_TRY(pc->x_afm.alloc(9 * N));
            k_dual_pivots<<<grid_for(N), kBlock, 0, s>>>((int)N, pc->Arp.p, pc->Aci.p, pc->Aval.p, pc->x_einv_f.p,
                                                         pc->x_einv_m.p, pc->x_amf.p, pc->x_afm.p, ff);
        }
        if (ext && pc->n > pc->ncell) {
            int cnt = pc->n - pc->ncell;
            BO_TRY(pc->x_einv_w.alloc(9 * (size_t)cnt));
            k_rows_inv<<<grid_for(cnt), kBlock, 0, s>>>(pc->ncell, cnt, pc->Arp.p, pc->Aci.p, pc->Aval.p,
                                                        pc->x_einv_w.p, ff);
        }
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// The F stage's flag, once the work fstage_launch queued is ordered before s.
bo_status fstage_check(bo_cpr *pc, hipStream_t s) {
    int32_t bad = 0;
    HostRead rd{pc->fflag.p, sizeof bad, &bad};
    BO_TRY(host_reads(&rd, 1, s));
    if (bad & 2)
        return fail(BO_ERR_UNSUPPORTED, "F stage: a cell row's lower blocks are not its -x, -y, -z neighbours");
    if (bad) return fail(BO_ERR_SINGULAR_BLOCK, "F stage: singular 3x3 pivot block");
    return BO_OK;
}

namespace {
template <int St, typename T, typename TD>
bo_status fstage_run(bo_cpr *pc, const double *r, const TD *dp, double *out, T *wq, hipStream_t s,
                     const double *zin = nullptr) {
    long long n = pc->n;
    if (pc->o.ftype == BO_F_BJ) {
        if (zin) return fail(BO_ERR_UNSUPPORTED, "F stage: no accumulating block-Jacobi form");
        k_bj_apply<St, T, TD><<<grid_for(n), kBlock, 0, s>>>(n, pc->einv.p, r, dp, out);
    } else {
        TileGeom G = geom(pc);
        k_ilu_forward<St, T><<<G.ntx * G.nty, 128, 0, s>>>(G, pc->ilu_f.p, r, wq);
        const int D = stage_layers(G);
        k_ilu_backward<St, T, TD><<<G.ntx * G.nty, 128, D * kStageBytes, s>>>(G, pc->ilu_b.p, wq, dp, out, D,
                                                                                 zin);
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}
}  // namespace

// out = F(r) (+ Pi_p dp when dp != NULL); r in natural order
bo_status fstage_apply(bo_cpr *pc, const double *r, const double *dp, double *out, hipStream_t s) {
    if (pc->o.ftype == BO_F_ILU_NATURAL) return nat_apply(pc, r, dp, out, s);
    if (pc->general && pc->o.ftype == BO_F_ILU_TILED) {
        // the extended grid form: tiles of fracture cells, then matrix cells,
        // then well rows (FP64, or FP32 / BF16 tile factors without matrix
        // cells; the well rows' inverses stay FP64)
        if (dp) return fail(BO_ERR_INVALID_ARG, "F stage: extended form takes no pressure correction");
        TileGeom G = geom(pc);
        size_t S = (size_t)G.slots();
        const long long N = pc->g.n();
        const int st = store_of(pc);
        if (st != ST_F64) {
            if (st == ST_F32) k_ilu_forward<ST_F32, float><<<G.ntx * G.nty, 128, 0, s>>>(G, pc->ilu_f.p, r,
                                                                                          pc->ilu_w32.p);
            else k_ilu_forward<ST_BF16, float><<<G.ntx * G.nty, 128, 0, s>>>(G, pc->ilu_f.p, r, pc->ilu_w32.p);
            if (pc->n > pc->ncell) {
                int cnt = pc->n - pc->ncell;
                k_rows_apply<double><<<grid_for(cnt), kBlock, 0, s>>>(pc->ncell, cnt, pc->x_einv_w.p, r, out, nullptr,
                                                                      nullptr);
            }
            const int D = stage_layers(G);
            if (st == ST_F32)
                k_ilu_backward<ST_F32, float, double><<<G.ntx * G.nty, 128, D * kStageBytes, s>>>(
                    G, pc->ilu_b.p, pc->ilu_w32.p, nullptr, out, D, nullptr);
            else
                k_ilu_backward<ST_BF16, float, double><<<G.ntx * G.nty, 128, D * kStageBytes, s>>>(
                    G, pc->ilu_b.p, pc->ilu_w32.p, nullptr, out, D, nullptr);
            BO_HIP(hipGetLastError());
            return BO_OK;
        }
        k_ilu_forward<ST_F64, double><<<G.ntx * G.nty, 128, 0, s>>>(G, pc->ilu_f.p, r, pc->ilu_w.p);
        if (pc->ncell > N)
            k_dual_forward<<<grid_for(N), kBlock, 0, s>>>((int)N, pc->ilu_slot.p, S, r, pc->x_einv_m.p, pc->x_amf.p,
                                                          pc->x_afm.p, pc->x_einv_f.p, pc->ilu_w.p, out);
        if (pc->n > pc->ncell) {
            int cnt = pc->n - pc->ncell;
            k_rows_apply<double><<<grid_for(cnt), kBlock, 0, s>>>(pc->ncell, cnt, pc->x_einv_w.p, r, out, nullptr,
                                                                  nullptr);
        }
        const int D = stage_layers(G);
        k_ilu_backward<ST_F64, double, double><<<G.ntx * G.nty, 128, D * kStageBytes, s>>>(
            G, pc->ilu_b.p, pc->ilu_w.p, nullptr, out, D, nullptr);
        BO_HIP(hipGetLastError());
        return BO_OK;
    }
    switch (store_of(pc)) {
    case ST_F64: return fstage_run<ST_F64, double, double>(pc, r, dp, out, pc->ilu_w.p, s);
    case ST_F32: return fstage_run<ST_F32, float, double>(pc, r, dp, out, pc->ilu_w32.p, s);
    default: return fstage_run<ST_BF16, float, double>(pc, r, dp, out, pc->ilu_w32.p, s);
    }
}

// z += F(r) + Pi_p dp in one pass over z (dp may be NULL; FP64 dp with the
// FP64 factors, FP32 dp with the FP32 / BF16 ones), for the tiled ILU of a
// grid and of the extended form without matrix cells with the pressure system
// over all rows; BO_ERR_UNSUPPORTED for the other forms (the caller then adds
// the terms one by one)
bool fstage_acc_ok(const bo_cpr *pc) {
    if (pc->o.ftype != BO_F_ILU_TILED) return false;
    if (!pc->general) return true;
    return pc->has_grid && pc->ncell == pc->g.n() && pc->npr == pc->n;
}
template <typename TD>
bo_status fstage_apply_acc(bo_cpr *pc, const double *r, const TD *dp, double *z, hipStream_t s) {
    if (!fstage_acc_ok(pc)) return fail(BO_ERR_UNSUPPORTED, "F stage: no accumulating form here");
    const int st = store_of(pc);
    if ((st == ST_F64) != std::is_same<TD, double>::value)
        return fail(BO_ERR_INVALID_ARG, "F stage: pressure correction precision does not match the factors");
    TileGeom G = geom(pc);
    if (pc->general && pc->n > pc->ncell) {
        // the well rows first: they read r and write their own rows of z only
        const int cnt = pc->n - pc->ncell;
        k_rows_apply<TD><<<grid_for(cnt), kBlock, 0, s>>>(pc->ncell, cnt, pc->x_einv_w.p, r, z, dp, z);
        BO_HIP(hipGetLastError());
    }
    if (st == ST_F64)
        return fstage_run<ST_F64, double, TD>(pc, r, dp, z, pc->ilu_w.p, s, z);
    if (st == ST_F32) return fstage_run<ST_F32, float, TD>(pc, r, dp, z, pc->ilu_w32.p, s, z);
    return fstage_run<ST_BF16, float, TD>(pc, r, dp, z, pc->ilu_w32.p, s, z);
}
template bo_status fstage_apply_acc<double>(bo_cpr *, const double *, const double *, double *, hipStream_t);
template bo_status fstage_apply_acc<float>(bo_cpr *, const double *, const float *, double *, hipStream_t);

// mixed form with the FP32 pressure correction of the V-cycle
bo_status fstage_apply_f32dp(bo_cpr *pc, const double *r, const float *dp, double *out, hipStream_t s) {
    switch (store_of(pc)) {
    case ST_F32: return fstage_run<ST_F32, float, float>(pc, r, dp, out, pc->ilu_w32.p, s);
    case ST_BF16: return fstage_run<ST_BF16, float, float>(pc, r, dp, out, pc->ilu_w32.p, s);
    default: return fail(BO_ERR_INVALID_ARG, "F stage: FP32 pressure correction in the FP64 form");
    }
}


}  // namespace bo
