// Learned pressure-stage correction: a 3-D convolutional network (four
// zero-padded 3x3x3 convolutions, channels 2 -> 16 -> 16 -> 16 -> 1, biases,
// ReLU after the first three) trained on pairs of pressure residual and the
// error one AMG V-cycle leaves.  Forward and backward passes run on the
// matrix cores: BF16 operands, FP32 accumulation (v_mfma_f32_16x16x32_bf16,
// lane l holding A[l % 16][8 (l / 16) + j], B[8 (l / 16) + j][l % 16] for
// j < 8, and receiving C[4 (l / 16) + j][l % 16] for j < 4).
//
// Convolution as an implicit GEMM.  A workgroup owns an output tile of
// 16 (x) by 4 (y) by 4 (z) voxels = 16 rows of 16 voxels; its four wavefronts
// take four rows each.  The input halo (18 x 6 x 6 voxels, channel-last BF16)
// and the layer's weights are staged in LDS.  For one row and one tap the
// product is D[n][i] = sum_k W[t][n][k] X[i + off(t)][k] with n the output
// channel, i the voxel of the row and k the input channel, with the weights
// as the A operand and the shifted row as the B operand, so that lane l ends
// with output channels 4(l/16)..4(l/16)+3 of voxel l%16 and stores them as one
// 8-byte write.  One 16x16x32 MFMA covers two taps of 16 input channels (lane
// groups 0-1 the first tap, 2-3 the second; 27 taps padded to 28 with a zero
// one): 14 per row.  The first layer has 2 input channels (padded to 4): one
// MFMA covers eight taps, each lane group two of them (27 taps padded to 32).
//
// Backward: the input gradient of a layer is the same convolution with the
// kernel flipped and transposed (dX[u][c] = sum_t sum_o dZ[u - off(t)][o]
// W[t][c][o]), masked by the ReLU of the layer below; the weight gradient
// dW[t][c][o] = sum_v X[v + off(t)][c] dZ[v][o] is an MFMA reduction over the
// voxels of each tile (32 voxels, two rows, per MFMA), combined across
// workgroups in a fixed order.
#include "bo_nn.hpp"
#include "bo_cpr.hpp"

namespace bo {
namespace {

typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v4f __attribute__((ext_vector_type(4)));

// eight BF16 values (16 bytes) as an MFMA operand
__device__ __forceinline__ v8bf bf8(uint4 u) { return __builtin_bit_cast(v8bf, u); }
__device__ __forceinline__ v8bf lds8(const uint16_t *p) { return bf8(*(const uint4 *)p); }

constexpr int TX = 16, TY = 4, TZ = 4;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int HV = HX * HY * HZ;      // halo voxels of a tile
constexpr int TV = TX * TY * TZ;      // voxels of a tile
enum { MODE_ACT = 0, MODE_OUT = 1, MODE_GRAD = 2 };

// FP32 -> BF16 (round to nearest even; values are finite) and back
__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint32_t h) { return __uint_as_float(h << 16); }

struct TileXY {
    int b, z0, y0, x0;
};
__device__ __forceinline__ TileXY tile_of(const Vol &V, int tile) {
    int ntx = (V.nx + TX - 1) / TX, nty = (V.ny + TY - 1) / TY, ntz = (V.nz + TZ - 1) / TZ;
    TileXY T;
    T.x0 = (tile % ntx) * TX;
    tile /= ntx;
    T.y0 = (tile % nty) * TY;
    tile /= nty;
    T.z0 = (tile % ntz) * TZ;
    T.b = tile / ntz;
    return T;
}
inline long long tiles_of(const Vol &V) {
    return (long long)((V.nx + TX - 1) / TX) * ((V.ny + TY - 1) / TY) * ((V.nz + TZ - 1) / TZ) * V.nb;
}
__device__ __forceinline__ long long voxel(const Vol &V, int b, int z, int y, int x) {
    return (((long long)b * V.nz + z) * V.ny + y) * V.nx + x;
}

// halo of a C-channel BF16 tensor into LDS (zero outside the volume)
template <int C>
__device__ __forceinline__ void load_halo(const uint16_t *__restrict__ act, const Vol &V, const TileXY &T,
                                          uint16_t *lds) {
    constexpr int CH = C / 4;
    for (int q = threadIdx.x; q < HV * CH; q += blockDim.x) {
        int hv = q / CH, c4 = q % CH;
        int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
        int x = T.x0 + hx - 1, y = T.y0 + hy - 1, z = T.z0 + hz - 1;
        uint2 val = make_uint2(0u, 0u);
        if (x >= 0 && x < V.nx && y >= 0 && y < V.ny && z >= 0 && z < V.nz)
            val = *(const uint2 *)(act + voxel(V, T.b, z, y, x) * C + 4 * c4);
        *(uint2 *)(lds + hv * C + 4 * c4) = val;
    }
}

__device__ __forceinline__ int halo_index(int z, int y, int x) { return (z * HY + y) * HX + x; }

// Convolution of a CIN-channel input to 16 output channels.  W: [taps][16][CIN]
// BF16 (27 taps and zero ones up to 28 (CIN = 16) or 32 (CIN = 4)).
//   MODE_ACT:  out = BF16(ReLU(acc + bias))              -> act_out [v][16]
//   MODE_OUT:  y = acc[channel 0] + bias[0]              -> y_out [v] (FP32)
//   MODE_GRAD: out = BF16(acc) where mask[v][n] > 0, else 0 -> act_out [v][16]
template <int CIN, int MODE>
__global__ void __launch_bounds__(256) k_nn_conv(Vol V, const uint16_t *__restrict__ in,
                                                 const uint16_t *__restrict__ W, const float *__restrict__ bias,
                                                 const uint16_t *__restrict__ mask, uint16_t *__restrict__ act_out,
                                                 float *__restrict__ y_out) {
    constexpr int NT = CIN == 4 ? 32 : 28;
    __shared__ __align__(16) uint16_t xs[HV * CIN];
    __shared__ __align__(16) uint16_t ws[NT * 16 * CIN];
    const TileXY T = tile_of(V, blockIdx.x);
    load_halo<CIN>(in, V, T, xs);
    for (int q = threadIdx.x; q < NT * 16 * CIN / 4; q += blockDim.x)
        *(uint2 *)(ws + 4 * q) = *(const uint2 *)(W + 4 * q);
    __syncthreads();
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int i = lane % 16, g = lane / 16;
    float bv[4] = {0.f, 0.f, 0.f, 0.f};
    if (MODE != MODE_GRAD)
        for (int j = 0; j < 4; j++) bv[j] = (MODE == MODE_OUT && 4 * g + j > 0) ? 0.f : bias[4 * g + j];
    for (int rr = 0; rr < 4; rr++) {
        const int r = wave * 4 + rr;
        const int ry = r % TY, rz = r / TY;
        v4f acc = {0.f, 0.f, 0.f, 0.f};
        if (CIN == 16) {
            // k = 8g + j: tap 2 tp + g / 2, input channel 8 (g % 2) + j
            const int ko = 8 * (g & 1);
#pragma unroll 2
            for (int tp = 0; tp < 14; tp++) {
                const int t = 2 * tp + (g >> 1);
                const int tt = t < 27 ? t : 26;        // tap 27 has zero weights
                const int dz = tt / 9 - 1, dy = (tt / 3) % 3 - 1, dx = tt % 3 - 1;
                v8bf a = lds8(ws + (t * 16 + i) * 16 + ko);
                v8bf b = lds8(xs + halo_index(rz + 1 + dz, ry + 1 + dy, i + 1 + dx) * 16 + ko);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
        } else {
            // k = 8g + 4h + j: tap 8q + 2g + h, input channel j
#pragma unroll
            for (int q = 0; q < 4; q++) {
                uint2 wa[2], xb[2];
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const int t = 8 * q + 2 * g + h;
                    const int tt = t < 27 ? t : 26;    // taps 27..31 have zero weights
                    const int dz = tt / 9 - 1, dy = (tt / 3) % 3 - 1, dx = tt % 3 - 1;
                    wa[h] = *(const uint2 *)(ws + (t * 16 + i) * 4);
                    xb[h] = *(const uint2 *)(xs + halo_index(rz + 1 + dz, ry + 1 + dy, i + 1 + dx) * 4);
                }
                v8bf a = bf8(make_uint4(wa[0].x, wa[0].y, wa[1].x, wa[1].y));
                v8bf b = bf8(make_uint4(xb[0].x, xb[0].y, xb[1].x, xb[1].y));
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
        }
        const int x = T.x0 + i, y = T.y0 + ry, z = T.z0 + rz;
        if (x >= V.nx || y >= V.ny || z >= V.nz) continue;
        const long long v = voxel(V, T.b, z, y, x);
        if (MODE == MODE_OUT) {
            if (g == 0) y_out[v] = acc[0] + bv[0];
        } else {
            uint16_t o[4];
            if (MODE == MODE_ACT) {
                for (int j = 0; j < 4; j++) o[j] = to_bf16(fmaxf(acc[j] + bv[j], 0.f));
            } else {
                uint2 mk = *(const uint2 *)(mask + v * 16 + 4 * g);
                uint32_t mw[4] = {mk.x & 0xFFFFu, mk.x >> 16, mk.y & 0xFFFFu, mk.y >> 16};
                for (int j = 0; j < 4; j++) o[j] = (mw[j] & 0x7FFFu) ? to_bf16(acc[j]) : (uint16_t)0;
            }
            *(uint2 *)(act_out + v * 16 + 4 * g) =
                make_uint2((uint32_t)o[0] | ((uint32_t)o[1] << 16), (uint32_t)o[2] | ((uint32_t)o[3] << 16));
        }
    }
}

// Weight and bias gradients of one layer: dW[t][c][o] = sum_v X[v+off(t)][c]
// dZ[v][o], db[o] = sum_v dZ[v][o], with X the layer's CIN-channel input and
// dZ its COUT-channel (4 or 16, zero padded) output gradient.  Each wavefront
// accumulates 27 16x16 tiles D_t[o][c] over its rows of every tile it visits
// and writes them to part[(block*4 + wave)][27*256 + 16].
template <int CIN, int COUT>
__global__ void __launch_bounds__(256) k_nn_wgrad(Vol V, long long ntiles, const uint16_t *__restrict__ X,
                                                  const uint16_t *__restrict__ dZ, float *__restrict__ part) {
    __shared__ __align__(16) uint16_t xs[HV * CIN];
    __shared__ __align__(16) uint16_t ds[TV * COUT];
    const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
    const int c = lane % 16, g = lane / 16;   // A: output channel o = c; B: input channel = c
    v4f acc[27];
#pragma unroll
    for (int t = 0; t < 27; t++) acc[t] = (v4f){0.f, 0.f, 0.f, 0.f};
    float db = 0.f;
    for (long long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const TileXY T = tile_of(V, (int)tile);
        __syncthreads();  // LDS reuse
        load_halo<CIN>(X, V, T, xs);
        for (int q = threadIdx.x; q < TV * COUT / 4; q += blockDim.x) {
            int tv = q / (COUT / 4), c4 = q % (COUT / 4);
            int tx = tv % TX, ty = (tv / TX) % TY, tz = tv / (TX * TY);
            int x = T.x0 + tx, y = T.y0 + ty, z = T.z0 + tz;
            uint2 val = make_uint2(0u, 0u);
            if (x < V.nx && y < V.ny && z < V.nz) val = *(const uint2 *)(dZ + voxel(V, T.b, z, y, x) * COUT + 4 * c4);
            *(uint2 *)(ds + tv * COUT + 4 * c4) = val;
        }
        __syncthreads();
        // two rows of 16 voxels per MFMA: k = 8g + j is voxel 8 (g % 2) + j of
        // row r0 + g / 2
        for (int rp = 0; rp < 2; rp++) {
            const int r = wave * 4 + 2 * rp + (g >> 1);
            const int ry = r % TY, rz = r / TY;
            const int vo = 8 * (g & 1);
            // A[o = c][k]
            uint16_t ha[8];
#pragma unroll
            for (int j = 0; j < 8; j++) {
                uint16_t h = c < COUT ? ds[(r * TX + vo + j) * COUT + c] : (uint16_t)0;
                ha[j] = h;
                db += from_bf16(h);
            }
            const v8bf a = bf8(make_uint4(ha[0] | ((uint32_t)ha[1] << 16), ha[2] | ((uint32_t)ha[3] << 16),
                                          ha[4] | ((uint32_t)ha[5] << 16), ha[6] | ((uint32_t)ha[7] << 16)));
            // fully unrolled: the 27 accumulators stay in registers
#pragma unroll
            for (int t = 0; t < 27; t++) {
                const int dz = t / 9 - 1, dy = (t / 3) % 3 - 1, dx = t % 3 - 1;
                uint16_t hb[8];
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    int hv = halo_index(rz + 1 + dz, ry + 1 + dy, vo + j + 1 + dx);
                    hb[j] = c < CIN ? xs[hv * CIN + c] : (uint16_t)0;
                }
                const v8bf b = bf8(make_uint4(hb[0] | ((uint32_t)hb[1] << 16), hb[2] | ((uint32_t)hb[3] << 16),
                                              hb[4] | ((uint32_t)hb[5] << 16), hb[6] | ((uint32_t)hb[7] << 16)));
                acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[t], 0, 0, 0);
            }
        }
    }
    // D_t[o = 4g+j][c]
    float *out = part + (size_t)(blockIdx.x * 4 + wave) * (27 * 256 + 16);
#pragma unroll
    for (int t = 0; t < 27; t++)
        for (int j = 0; j < 4; j++) out[t * 256 + (4 * g + j) * 16 + c] = acc[t][j];
    // bias: lanes with the same c hold partial sums over different voxels
    db += __shfl_xor(db, 16, 64);
    db += __shfl_xor(db, 32, 64);
    if (g == 0) out[27 * 256 + c] = db;
}

// sum the partials in a fixed order into the flat gradient of one layer
__global__ void k_nn_wgrad_reduce(int nparts, const float *__restrict__ part, int cin, int cout,
                                  float *__restrict__ gW, float *__restrict__ gb) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int nw = 27 * cin * cout;
    if (e >= nw + cout) return;
    int src;
    if (e < nw) {
        int t = e / (cin * cout), ci = (e / cout) % cin, co = e % cout;
        src = t * 256 + co * 16 + ci;
    } else {
        src = 27 * 256 + (e - nw);
    }
    float s = 0.f;
    for (int p = 0; p < nparts; p++) s += part[(size_t)p * (27 * 256 + 16) + src];
    if (e < nw) gW[e] = s;
    else gb[e - nw] = s;
}

// network input from FP32 pairs of channels [v][2] -> BF16 [v][4]
__global__ void k_nn_input(long long nv, const float *__restrict__ in, uint16_t *__restrict__ x) {
    long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nv) return;
    uint32_t h0 = to_bf16(in[2 * v]), h1 = to_bf16(in[2 * v + 1]);
    *(uint2 *)(x + 4 * v) = make_uint2(h0 | (h1 << 16), 0u);
}

// output gradient of the mean squared error: dZ4 = BF16(2 (y - t) / M) in a
// 4-channel tensor; partial sums of (y - t)^2 per block
__global__ void __launch_bounds__(256) k_nn_loss(long long nv, const float *__restrict__ y,
                                                 const float *__restrict__ tgt, float scale,
                                                 uint16_t *__restrict__ dz, double *__restrict__ lpart) {
    __shared__ double red[256];
    long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (v < nv) {
        float d = y[v] - tgt[v];
        sq = (double)d * d;
        *(uint2 *)(dz + 4 * v) = make_uint2((uint32_t)to_bf16(d * scale), 0u);
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

__global__ void k_nn_loss_final(int nparts, const double *__restrict__ lpart, double inv_m, double *__restrict__ loss) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double s = 0.0;
    for (int p = 0; p < nparts; p++) s += lpart[p];
    *loss = s * inv_m;
}

// A_pp-weighted loss: R = A (y - t) on the voxels whose six neighbours lie in
// the volume (0 elsewhere), coef [7][voxels] in slot order (-z, -y, -x, self,
// +x, +y, +z); partial sums of R^2 per block
__global__ void __launch_bounds__(256) k_nn_wres(Vol V, const float *__restrict__ coef, const float *__restrict__ y,
                                                 const float *__restrict__ tgt, float *__restrict__ R,
                                                 double *__restrict__ lpart) {
    __shared__ double red[256];
    const long long nv = V.voxels();
    const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double sq = 0.0;
    if (v < nv) {
        const int x = (int)(v % V.nx), yy = (int)((v / V.nx) % V.ny), z = (int)((v / ((long long)V.nx * V.ny)) % V.nz);
        float r = 0.f;
        if (x > 0 && x < V.nx - 1 && yy > 0 && yy < V.ny - 1 && z > 0 && z < V.nz - 1) {
            const long long sx = 1, sy = V.nx, sz = (long long)V.nx * V.ny;
            const long long nb[7] = {v - sz, v - sy, v - sx, v, v + sx, v + sy, v + sz};
            double acc = 0.0;
            for (int q = 0; q < 7; q++)
                acc += (double)coef[(size_t)q * nv + v] * (double)(y[nb[q]] - tgt[nb[q]]);
            r = (float)acc;
        }
        R[v] = r;
        sq = (double)r * r;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) lpart[blockIdx.x] = red[0];
}

// output gradient of the weighted loss: dZ4 = BF16(scale (A^T R)) in a
// 4-channel tensor, (A^T R)_j = sum over the cells i whose slot q couples to
// j of coef[q][i] R_i
__global__ void k_nn_wout(Vol V, const float *__restrict__ coef, const float *__restrict__ R, float scale,
                          uint16_t *__restrict__ dz) {
    const long long nv = V.voxels();
    const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nv) return;
    const int x = (int)(j % V.nx), yy = (int)((j / V.nx) % V.ny), z = (int)((j / ((long long)V.nx * V.ny)) % V.nz);
    const long long sx = 1, sy = V.nx, sz = (long long)V.nx * V.ny;
    // cell i = j - off(q): slot q of i points at j
    const bool in[7] = {z < V.nz - 1, yy < V.ny - 1, x < V.nx - 1, true, x > 0, yy > 0, z > 0};
    const long long src[7] = {j + sz, j + sy, j + sx, j, j - sx, j - sy, j - sz};
    double g = 0.0;
    for (int q = 0; q < 7; q++)
        if (in[q]) g += (double)coef[(size_t)q * nv + src[q]] * (double)R[src[q]];
    *(uint2 *)(dz + 4 * j) = make_uint2((uint32_t)to_bf16((float)(scale * g)), 0u);
}

__global__ void k_nn_adam(int n, float *__restrict__ w, const float *__restrict__ g, float *__restrict__ m,
                          float *__restrict__ v, float lr, float b1, float b2, float eps, float c1, float c2) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float gi = g[e];
    float mi = b1 * m[e] + (1.f - b1) * gi;
    float vi = b2 * v[e] + (1.f - b2) * gi * gi;
    m[e] = mi;
    v[e] = vi;
    w[e] = w[e] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// BF16 weight layouts from the FP32 master W[t][ci][co] of one layer:
//   forward  wf[t][n][k]  = W[t][k][n]          (k < kpad, n < 16; zero padded)
//   backward wb[t][n][k]  = W[26 - t][n][k]     (n = ci < 16, k = co < kpad)
__global__ void k_nn_pack(const float *__restrict__ W, int ci, int co, int kf, int ntf, uint16_t *__restrict__ wf,
                          int kb, int ntb, uint16_t *__restrict__ wb) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    int nf = ntf * 16 * kf;
    if (e < nf) {
        int t = e / (16 * kf), n = (e / kf) % 16, k = e % kf;
        float val = (t < 27 && n < co && k < ci) ? W[(t * ci + k) * co + n] : 0.f;
        wf[e] = to_bf16(val);
    }
    if (wb) {
        int nb = ntb * 16 * kb;
        if (e < nb) {
            int t = e / (16 * kb), n = (e / kb) % 16, k = e % kb;
            float val = (t < 27 && n < ci && k < co) ? W[((26 - t) * ci + n) * co + k] : 0.f;
            wb[e] = to_bf16(val);
        }
    }
}

int layer_off(int l) {
    int off = 0;
    for (int q = 0; q < l; q++) off += 27 * kNnChan[q] * kNnChan[q + 1] + kNnChan[q + 1];
    return off;
}

}  // namespace

// ---- host ----------------------------------------------------------------------
bo_status nn_pack(bo_nn *nn, hipStream_t s) {
    for (int l = 0; l < kNnLayers; l++) {
        int ci = kNnChan[l], co = kNnChan[l + 1];
        int kf = l == 0 ? 4 : 16, ntf = l == 0 ? 32 : 28;
        BO_TRY(nn->wf[l].alloc((size_t)ntf * 16 * kf));
        uint16_t *wb = nullptr;
        int kb = 16, ntb = 28;
        if (l > 0) {
            kb = l == kNnLayers - 1 ? 4 : 16;
            ntb = kb == 4 ? 32 : 28;
            BO_TRY(nn->wb[l].alloc((size_t)ntb * 16 * kb));
            wb = nn->wb[l].p;
        }
        int n = std::max(ntf * 16 * kf, ntb * 16 * kb);
        k_nn_pack<<<grid_for(n), kBlock, 0, s>>>(nn->w.p + layer_off(l), ci, co, kf, ntf, nn->wf[l].p, kb, ntb, wb);
    }
    BO_HIP(hipGetLastError());
    return BO_OK;
}

static bo_status nn_buffers(bo_nn *nn, const Vol &V) {
    size_t nv = (size_t)V.voxels();
    BO_TRY(nn->x1.alloc(4 * nv));
    BO_TRY(nn->a1.alloc(16 * nv));
    BO_TRY(nn->a2.alloc(16 * nv));
    BO_TRY(nn->a3.alloc(16 * nv));
    BO_TRY(nn->y.alloc(nv));
    nn->vol = V;
    return BO_OK;
}

// forward pass of the network on x1 (already filled); the output lands in nn->y
bo_status nn_forward_x1(bo_nn *nn, const Vol &V, hipStream_t s) {
    long long nt = tiles_of(V);
    if (nt <= 0) return BO_OK;
    const float *w = nn->w.p;
    k_nn_conv<4, MODE_ACT><<<(unsigned)nt, 256, 0, s>>>(V, nn->x1.p, nn->wf[0].p, w + layer_off(0) + 27 * 2 * 16,
                                                        nullptr, nn->a1.p, nullptr);
    k_nn_conv<16, MODE_ACT><<<(unsigned)nt, 256, 0, s>>>(V, nn->a1.p, nn->wf[1].p, w + layer_off(1) + 27 * 16 * 16,
                                                         nullptr, nn->a2.p, nullptr);
    k_nn_conv<16, MODE_ACT><<<(unsigned)nt, 256, 0, s>>>(V, nn->a2.p, nn->wf[2].p, w + layer_off(2) + 27 * 16 * 16,
                                                         nullptr, nn->a3.p, nullptr);
    k_nn_conv<16, MODE_OUT><<<(unsigned)nt, 256, 0, s>>>(V, nn->a3.p, nn->wf[3].p, w + layer_off(3) + 27 * 16,
                                                         nullptr, nullptr, nn->y.p);
    BO_HIP(hipGetLastError());
    return BO_OK;
}

// BF16 network input for CPR: channel 0 = r_p / s, channel 1 = standardised
// log-permeability (FP32, per cell)
template <typename T>
__global__ void k_nn_input_cpr(long long n, const T *__restrict__ rp, const double *__restrict__ s2,
                               const float *__restrict__ z, uint16_t *__restrict__ x) {
    long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    double s = sqrt(*s2);
    float r = (float)((double)rp[v] / (s > 0.0 ? s : 1.0));
    uint32_t h0 = to_bf16(r), h1 = to_bf16(z[v]);
    *(uint2 *)(x + 4 * v) = make_uint2(h0 | (h1 << 16), 0u);
}
template __global__ void k_nn_input_cpr<double>(long long, const double *, const double *, const float *, uint16_t *);
template __global__ void k_nn_input_cpr<float>(long long, const float *, const double *, const float *, uint16_t *);

bo_status nn_input_cpr(bo_nn *nn, const Grid &g, const void *rp, bool fp32, const double *s2, const float *z,
                       hipStream_t s) {
    Vol V;
    V.nb = 1; V.nz = g.nz; V.ny = g.ny; V.nx = g.nx;
    BO_TRY(nn_buffers(nn, V));
    nn->last_from_cpr = true;
    long long n = V.voxels();
    if (fp32) k_nn_input_cpr<float><<<grid_for(n), kBlock, 0, s>>>(n, (const float *)rp, s2, z, nn->x1.p);
    else k_nn_input_cpr<double><<<grid_for(n), kBlock, 0, s>>>(n, (const double *)rp, s2, z, nn->x1.p);
    BO_HIP(hipGetLastError());
    return nn_forward_x1(nn, V, s);
}

}  // namespace bo

using namespace bo;

extern "C" bo_status bo_nn_create(bo_nn **out) {
    if (!out) return fail(BO_ERR_INVALID_ARG, "bo_nn_create: out is NULL");
    *out = nullptr;
    bo_nn *nn = new (std::nothrow) bo_nn();
    if (!nn) return fail(BO_ERR_ALLOC, "bo_nn_create: out of host memory");
    bo_status st = BO_OK;
    if ((st = nn->w.alloc(kNnParams)) || (st = nn->g.alloc(kNnParams)) || (st = nn->m.alloc(kNnParams)) ||
        (st = nn->v.alloc(kNnParams)) || (st = nn->lpart.alloc(1)) || (st = nn->loss.alloc(1))) {
        delete nn;
        return st;
    }
    if (hipMemset(nn->w.p, 0, sizeof(float) * kNnParams) != hipSuccess ||
        hipMemset(nn->g.p, 0, sizeof(float) * kNnParams) != hipSuccess ||
        hipMemset(nn->m.p, 0, sizeof(float) * kNnParams) != hipSuccess ||
        hipMemset(nn->v.p, 0, sizeof(float) * kNnParams) != hipSuccess) {
        delete nn;
        return fail(BO_ERR_HIP, "bo_nn_create: hipMemset failed");
    }
    if ((st = nn_pack(nn, nullptr)) != BO_OK || hipDeviceSynchronize() != hipSuccess) {
        delete nn;
        return st != BO_OK ? st : fail(BO_ERR_HIP, "bo_nn_create: packing the weights failed");
    }
    *out = nn;
    return BO_OK;
}

extern "C" void bo_nn_destroy(bo_nn *nn) {
    if (!nn) return;
    (void)hipDeviceSynchronize();
    delete nn;
}

extern "C" int32_t bo_nn_num_params(void) { return kNnParams; }

extern "C" bo_status bo_nn_set_params(bo_nn *nn, const float *params, void *stream) {
    if (!nn || !params) return fail(BO_ERR_INVALID_ARG, "bo_nn_set_params: NULL argument");
    hipStream_t s = (hipStream_t)stream;
    BO_HIP(hipMemcpyAsync(nn->w.p, params, sizeof(float) * kNnParams, hipMemcpyHostToDevice, s));
    BO_HIP(hipMemsetAsync(nn->m.p, 0, sizeof(float) * kNnParams, s));
    BO_HIP(hipMemsetAsync(nn->v.p, 0, sizeof(float) * kNnParams, s));
    nn->step = 0;
    BO_TRY(nn_pack(nn, s));
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}

extern "C" bo_status bo_nn_get_params(bo_nn *nn, float *params, float *grads, void *stream) {
    if (!nn) return fail(BO_ERR_INVALID_ARG, "bo_nn_get_params: NULL handle");
    hipStream_t s = (hipStream_t)stream;
    if (params) BO_HIP(hipMemcpyAsync(params, nn->w.p, sizeof(float) * kNnParams, hipMemcpyDeviceToHost, s));
    if (grads) BO_HIP(hipMemcpyAsync(grads, nn->g.p, sizeof(float) * kNnParams, hipMemcpyDeviceToHost, s));
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}

extern "C" bo_status bo_nn_forward(bo_nn *nn, const float *in, float *out, int32_t nb, int32_t nz, int32_t ny,
                                   int32_t nx, void *stream) {
    if (!nn || !in || !out) return fail(BO_ERR_INVALID_ARG, "bo_nn_forward: NULL argument");
    if (nb < 1 || nz < 1 || ny < 1 || nx < 1) return fail(BO_ERR_INVALID_ARG, "bo_nn_forward: empty volume");
    Vol V;
    V.nb = nb; V.nz = nz; V.ny = ny; V.nx = nx;
    if (tiles_of(V) >= (1LL << 31)) return fail(BO_ERR_INVALID_ARG, "bo_nn_forward: volume too large");
    hipStream_t s = (hipStream_t)stream;
    BO_TRY(nn_buffers(nn, V));
    nn->last_from_cpr = false;
    long long nv = V.voxels();
    k_nn_input<<<grid_for(nv), kBlock, 0, s>>>(nv, in, nn->x1.p);
    BO_HIP(hipGetLastError());
    BO_TRY(nn_forward_x1(nn, V, s));
    BO_HIP(hipMemcpyAsync(out, nn->y.p, sizeof(float) * nv, hipMemcpyDeviceToDevice, s));
    return BO_OK;
}

namespace {
// gradients of every layer from the output gradient in nn->dz4; the loss in
// nn->loss is copied to *loss (may be NULL); synchronises the stream
bo_status nn_backprop(bo_nn *nn, const Vol &V, double *loss, hipStream_t s) {
    long long nt = tiles_of(V);
    int wblocks = (int)std::min<long long>(nt, kNnWgradBlocks);
    BO_TRY(nn->part.alloc((size_t)wblocks * 4 * (27 * 256 + 16)));
    float *gw = nn->g.p;
    auto reduce = [&](int l) {
        int ci = kNnChan[l], co = kNnChan[l + 1];
        int n = 27 * ci * co + co;
        k_nn_wgrad_reduce<<<grid_for(n), kBlock, 0, s>>>(wblocks * 4, nn->part.p, ci, co, gw + layer_off(l),
                                                          gw + layer_off(l) + 27 * ci * co);
    };
    // layer 4 (A3 -> y)
    k_nn_wgrad<16, 4><<<wblocks, 256, 0, s>>>(V, nt, nn->a3.p, nn->dz4.p, nn->part.p);
    reduce(3);
    k_nn_conv<4, MODE_GRAD><<<(unsigned)nt, 256, 0, s>>>(V, nn->dz4.p, nn->wb[3].p, nullptr, nn->a3.p, nn->dz.p,
                                                         nullptr);
    // layer 3 (A2 -> A3)
    k_nn_wgrad<16, 16><<<wblocks, 256, 0, s>>>(V, nt, nn->a2.p, nn->dz.p, nn->part.p);
    reduce(2);
    k_nn_conv<16, MODE_GRAD><<<(unsigned)nt, 256, 0, s>>>(V, nn->dz.p, nn->wb[2].p, nullptr, nn->a2.p, nn->dzb.p,
                                                          nullptr);
    // layer 2 (A1 -> A2)
    k_nn_wgrad<16, 16><<<wblocks, 256, 0, s>>>(V, nt, nn->a1.p, nn->dzb.p, nn->part.p);
    reduce(1);
    k_nn_conv<16, MODE_GRAD><<<(unsigned)nt, 256, 0, s>>>(V, nn->dzb.p, nn->wb[1].p, nullptr, nn->a1.p, nn->dz.p,
                                                          nullptr);
    // layer 1 (X1 -> A1)
    k_nn_wgrad<4, 16><<<wblocks, 256, 0, s>>>(V, nt, nn->x1.p, nn->dz.p, nn->part.p);
    reduce(0);
    BO_HIP(hipGetLastError());
    if (loss) BO_HIP(hipMemcpyAsync(loss, nn->loss.p, sizeof(double), hipMemcpyDeviceToHost, s));
    BO_HIP(hipStreamSynchronize(s));
    return BO_OK;
}

bo_status nn_backward_check(bo_nn *nn, const char *who) {
    long long nv = nn->vol.voxels();
    if (nv <= 0 || nn->last_from_cpr)
        return fail(BO_ERR_INVALID_ARG, std::string(who) + ": the last forward pass was not a bo_nn_forward call");
    BO_TRY(nn->dz4.alloc(4 * (size_t)nv));
    BO_TRY(nn->dz.alloc(16 * (size_t)nv));
    BO_TRY(nn->dzb.alloc(16 * (size_t)nv));
    BO_TRY(nn->lpart.alloc(grid_for(nv)));
    return BO_OK;
}
}  // namespace

extern "C" bo_status bo_nn_backward(bo_nn *nn, const float *target, double *loss, void *stream) {
    if (!nn || !target) return fail(BO_ERR_INVALID_ARG, "bo_nn_backward: NULL argument");
    BO_TRY(nn_backward_check(nn, "bo_nn_backward"));
    const Vol V = nn->vol;
    long long nv = V.voxels();
    hipStream_t s = (hipStream_t)stream;
    unsigned nlb = grid_for(nv);
    k_nn_loss<<<nlb, 256, 0, s>>>(nv, nn->y.p, target, (float)(2.0 / (double)nv), nn->dz4.p, nn->lpart.p);
    k_nn_loss_final<<<1, 64, 0, s>>>((int)nlb, nn->lpart.p, 1.0 / (double)nv, nn->loss.p);
    return nn_backprop(nn, V, loss, s);
}

extern "C" bo_status bo_nn_backward_weighted(bo_nn *nn, const float *coef, const float *target, double *loss,
                                             void *stream) {
    if (!nn || !coef || !target) return fail(BO_ERR_INVALID_ARG, "bo_nn_backward_weighted: NULL argument");
    BO_TRY(nn_backward_check(nn, "bo_nn_backward_weighted"));
    const Vol V = nn->vol;
    long long nv = V.voxels();
    long long interior = (long long)V.nb * std::max(V.nz - 2, 0) * std::max(V.ny - 2, 0) * std::max(V.nx - 2, 0);
    if (interior <= 0)
        return fail(BO_ERR_INVALID_ARG, "bo_nn_backward_weighted: the volume has no interior voxel (a side below 3)");
    hipStream_t s = (hipStream_t)stream;
    unsigned nlb = grid_for(nv);
    BO_TRY(nn->wres.alloc((size_t)nv));
    k_nn_wres<<<nlb, 256, 0, s>>>(V, coef, nn->y.p, target, nn->wres.p, nn->lpart.p);
    k_nn_loss_final<<<1, 64, 0, s>>>((int)nlb, nn->lpart.p, 1.0 / (double)interior, nn->loss.p);
    k_nn_wout<<<nlb, kBlock, 0, s>>>(V, coef, nn->wres.p, (float)(2.0 / (double)interior), nn->dz4.p);
    return nn_backprop(nn, V, loss, s);
}

extern "C" bo_status bo_nn_adam_step(bo_nn *nn, float lr, void *stream) {
    if (!nn) return fail(BO_ERR_INVALID_ARG, "bo_nn_adam_step: NULL handle");
    if (!(lr > 0.f)) return fail(BO_ERR_INVALID_ARG, "bo_nn_adam_step: lr must be positive");
    hipStream_t s = (hipStream_t)stream;
    nn->step++;
    const float b1 = 0.9f, b2 = 0.999f;
    float c1 = (float)(1.0 - std::pow(0.9, (double)nn->step));
    float c2 = (float)(1.0 - std::pow(0.999, (double)nn->step));
    k_nn_adam<<<grid_for(kNnParams), kBlock, 0, s>>>(kNnParams, nn->w.p, nn->g.p, nn->m.p, nn->v.p, lr, b1, b2,
                                                     1e-8f, c1, c2);
    BO_HIP(hipGetLastError());
    return nn_pack(nn, s);
}
