// MLP closure on the device: 13 -> 128 -> 128 -> 128 -> 9 with SiLU,
// BF16 matrix-core products with FP32 accumulation, FP32 master weights.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

struct dsmc_mlp_s;

namespace dsmcx {

constexpr int kMlpIn = 13, kMlpHid = 128, kMlpOut = 9;
constexpr int kMlpW1 = 0;                               // W1[13][128]
constexpr int kMlpB1 = kMlpW1 + kMlpIn * kMlpHid;       // b1[128]
constexpr int kMlpW2 = kMlpB1 + kMlpHid;                // W2[128][128]
constexpr int kMlpB2 = kMlpW2 + kMlpHid * kMlpHid;
constexpr int kMlpW3 = kMlpB2 + kMlpHid;
constexpr int kMlpB3 = kMlpW3 + kMlpHid * kMlpHid;
constexpr int kMlpW4 = kMlpB3 + kMlpHid;                // W4[128][9]
constexpr int kMlpB4 = kMlpW4 + kMlpHid * kMlpOut;
constexpr int kMlpParams = kMlpB4 + kMlpOut;            // 35977
constexpr int kMlpTile = 32;                            // rows per workgroup (two waves of 16)

// BF16 operand copies of the weights, padded for the 16x16x32 products:
// "f" copies are output-major (forward products), "b" copies input-major
// (products with the transposed weights in the backward pass).
struct MlpDev {
    const uint16_t* wf1;  // [128][32]
    const uint16_t* wf2;  // [128][128]
    const uint16_t* wf3;  // [128][128]
    const uint16_t* wf4;  // [16][128]
    const uint16_t* wb2;  // [128][128]
    const uint16_t* wb3;  // [128][128]
    const uint16_t* wb4;  // [128][32]
    const float* params;  // FP32 master (biases read from here)
};

constexpr int kMlpPackTotal = 128 * 32 + 128 * 128 * 2 + 16 * 128 + 128 * 128 * 2 + 128 * 32;

void launch_mlp_pack(hipStream_t s, const float* params, uint16_t* packed);
MlpDev mlp_dev_view(const float* params, const uint16_t* packed);
MlpDev mlp_handle_view(dsmc_mlp_s* net);
// Forward on n rows of x[n][13] (FP32) -> y[n][9]; rows may be gathered by idx.
void launch_mlp_forward(hipStream_t s, const MlpDev& m, const float* x, const int32_t* idx, int64_t n, float* y);
// Forward + backward of the mean squared error over the n rows; per-block
// gradient partials [blocks][kMlpParams] and loss partials [blocks].
int64_t mlp_blocks(int64_t n);
void launch_mlp_grad(hipStream_t s, const MlpDev& m, const float* x, const float* t, const int32_t* idx, int64_t n,
                     float* partial, float* loss_partial);
// grad = sum of the block partials; *loss = (sum of the loss partials) / denom
void launch_mlp_reduce(hipStream_t s, const float* partial, const float* loss_partial, int64_t nblk, float* grad,
                       double* loss, double denom = 1.0);
void launch_mlp_adam(hipStream_t s, float* params, const float* grad, float* m, float* v, int step, float lr,
                     float b1, float b2, float eps);
void launch_mlp_init(hipStream_t s, float* params, RngKey key);
void launch_mlp_batch(hipStream_t s, RngKey key, uint32_t step, int64_t n, int64_t batch, int32_t* idx);

}  // namespace dsmcx
