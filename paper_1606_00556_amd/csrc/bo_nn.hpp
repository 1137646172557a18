// The learned pressure-stage network (internal).
#pragma once
#include "bo_common.hpp"

namespace bo {

// a batch of nb volumes of nz x ny x nx voxels, channel-last tensors
struct Vol {
    int nb = 0, nz = 0, ny = 0, nx = 0;
    __host__ __device__ long long voxels() const { return (long long)nb * nz * ny * nx; }
};

constexpr int kNnLayers = 4;
constexpr int kNnChan[kNnLayers + 1] = {2, 16, 16, 16, 1};
constexpr int kNnParams = 15169;  // sum over layers of 27 c_in c_out + c_out
constexpr int kNnWgradBlocks = 256;

}  // namespace bo

struct bo_nn {
    // FP32 master parameters, gradients and Adam moments, flat: per layer
    // W[t][c_in][c_out] then b[c_out]
    bo::DBuf<float> w, g, m, v;
    long long step = 0;
    // BF16 weights in the layouts the kernels read: forward [taps][16][k]
    // (k = 4 for the first layer, 16 otherwise) and, for layers 1-3, the
    // flipped transposes used for input gradients
    bo::DBuf<uint16_t> wf[bo::kNnLayers], wb[bo::kNnLayers];
    // activations of the last forward pass (BF16, channel-last)
    bo::Vol vol;
    bool last_from_cpr = false;                   // the last forward pass ran inside a CPR application
    bo::DBuf<uint16_t> x1, a1, a2, a3, dz4, dz;  // dz: [voxels][16] scratch for input gradients
    bo::DBuf<uint16_t> dzb;                       // second [voxels][16] scratch
    bo::DBuf<float> y;                            // output of the last forward pass
    bo::DBuf<float> part;                         // weight-gradient partial sums
    bo::DBuf<double> lpart;                       // loss partial sums
    bo::DBuf<double> loss;                        // last loss (device)
    bo::DBuf<float> wres;                         // weighted loss: the residual A (y - t) per voxel
};
