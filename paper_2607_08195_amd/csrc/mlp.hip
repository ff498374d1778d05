// MLP closure kernels: fused forward (and backward) of a 32-row tile per
// workgroup on the 16x16x32 BF16 matrix cores with FP32 accumulation.
//
// Precision contract: inputs, weights, hidden activations fed to the next
// layer and pre-activation gradients fed to a product are bfloat16 (round
// to nearest even); products accumulate in FP32; biases, pre-activations,
// SiLU, bias gradients and the optimiser run in FP32.
//
// Tile layout (two waves, wave w owns rows 16w..16w+15 of the tile):
//   forward    H_l = silu(H_{l-1} W_l + b_l)       rows x 128, K = 32 or 128
//   backward   dW_l^T = dZ_l^T H_{l-1}              contraction over the 32 rows
//              dH_{l-1} = dZ_l W_l^T                contraction over the outputs
// Row-major activations feed the forward products; transposed copies of
// H_l and dZ_l (feature-major, rows contiguous) feed the weight-gradient
// products, so every matrix-core operand is one 16-byte LDS read.
#include <cmath>

#include "mlp.h"

namespace dsmcx {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kSA = 136;  // row stride (elements) of row-major tiles [32][128 + 8]
constexpr int kST = 40;   // row stride of transposed tiles [features][32 + 8]
constexpr int kThreads = 128;

constexpr int kOffWf1 = 0, kOffWf2 = kOffWf1 + 128 * 32, kOffWf3 = kOffWf2 + 128 * 128, kOffWf4 = kOffWf3 + 128 * 128,
              kOffWb2 = kOffWf4 + 16 * 128, kOffWb3 = kOffWb2 + 128 * 128, kOffWb4 = kOffWb3 + 128 * 128;

__device__ __forceinline__ uint16_t to_bf16(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7FFFFFFFu) > 0x7F800000u) return 0x7FC0;
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ f32x4 mfma(uint4 a, uint4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

__device__ __forceinline__ float sigmoidf(float z) { return 1.0f / (1.0f + expf(-z)); }

// acc[t] (16 x 16 block t) = sum over KS steps of A[row0.., k] * Bt[col0 + 16 t.., k]
// A: row-major, lda elements per row; Bt: one row per output column.
template <int KS, int NT>
__device__ __forceinline__ void mm(const uint16_t* A, int lda, int row0, const uint16_t* Bt, int ldb, int col0,
                                   f32x4* acc) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
        const uint4 a = *(const uint4*)(A + (size_t)(row0 + r) * lda + ks * 32 + 8 * g);
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const uint4 b = *(const uint4*)(Bt + (size_t)(col0 + 16 * t + r) * ldb + ks * 32 + 8 * g);
            acc[t] = mfma(a, b, acc[t]);
        }
    }
}

// Hidden-layer epilogue: z = acc + b, h = silu(z) (bf16) into the next
// row-major tile and (training) the transposed tile; z kept for the backward.
template <bool TRAIN>
__device__ __forceinline__ void hidden_out(const f32x4* acc, const float* bias, int row0, uint16_t* Hn, uint16_t* Ht,
                                           f32x4* zkeep) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int col = 16 * t + r;
        const float b = bias[col];
        uint16_t hb[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float z = acc[t][i] + b;
            if (TRAIN) zkeep[t][i] = z;
            hb[i] = to_bf16(z * sigmoidf(z));
            Hn[(row0 + 4 * g + i) * kSA + col] = hb[i];
        }
        if (TRAIN) {
            uint2 pk;
            pk.x = (uint32_t)hb[0] | ((uint32_t)hb[1] << 16);
            pk.y = (uint32_t)hb[2] | ((uint32_t)hb[3] << 16);
            *(uint2*)(Ht + col * kST + row0 + 4 * g) = pk;
        }
    }
}

// dZ = dH * silu'(z) (FP32), stored bf16 row-major and transposed; the
// FP32 column sums over the wave's rows go to bsum[wave][col].
__device__ __forceinline__ void grad_out(const f32x4* dh, const f32x4* z, int row0, uint16_t* D, uint16_t* Dt,
                                         float* bsum) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4, w = threadIdx.x >> 6;
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        const int col = 16 * t + r;
        uint16_t db[4];
        float s = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const float sg = sigmoidf(z[t][i]);
            const float d = dh[t][i] * (sg * (1.0f + z[t][i] * (1.0f - sg)));
            s += d;
            db[i] = to_bf16(d);
            D[(row0 + 4 * g + i) * kSA + col] = db[i];
        }
        uint2 pk;
        pk.x = (uint32_t)db[0] | ((uint32_t)db[1] << 16);
        pk.y = (uint32_t)db[2] | ((uint32_t)db[3] << 16);
        *(uint2*)(Dt + col * kST + row0 + 4 * g) = pk;
        s += __shfl_xor(s, 16, 64);
        s += __shfl_xor(s, 32, 64);
        if (g == 0) bsum[w * 128 + col] = s;
    }
}

// Weight gradient W[k][n] (flat, in-major) += sum_r dZ[r][n] H[r][k] for the
// 16-column output tiles mt of this wave: rows n of dZt, rows k of Ht.
template <int NKT>
__device__ __forceinline__ void weight_grad(const uint16_t* Dt, const uint16_t* Ht, int mt0, int nmt, int kvalid,
                                            int nout, float* out) {
    const int l = threadIdx.x & 63, r = l & 15, g = l >> 4;
    for (int mt = mt0; mt < mt0 + nmt; ++mt) {
        f32x4 acc[NKT];
        mm<1, NKT>(Dt, kST, 16 * mt, Ht, kST, 0, acc);
#pragma unroll
        for (int t = 0; t < NKT; ++t) {
            const int k = 16 * t + r;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int n = 16 * mt + 4 * g + i;
                if (k < kvalid && n < nout) out[(size_t)k * nout + n] = acc[t][i];
            }
        }
    }
}

template <bool TRAIN>
__global__ __launch_bounds__(kThreads) void k_mlp_tile(MlpDev m, const float* x, const float* tgt, const int32_t* idx,
                                                       int64_t n, float scale, float* y, float* partial,
                                                       float* loss_partial) {
    __shared__ __attribute__((aligned(16))) uint16_t HA[kMlpTile * kSA];
    __shared__ __attribute__((aligned(16))) uint16_t HB[kMlpTile * kSA];
    __shared__ __attribute__((aligned(16))) uint16_t Ht0[32 * kST];
    __shared__ __attribute__((aligned(16))) uint16_t Ht1[128 * kST];
    __shared__ __attribute__((aligned(16))) uint16_t Ht2[128 * kST];
    __shared__ __attribute__((aligned(16))) uint16_t Ht3[128 * kST];
    __shared__ __attribute__((aligned(16))) uint16_t Dt[128 * kST];
    __shared__ float bsum[2 * 128];
    __shared__ float lsum[2];

    const int tid = threadIdx.x, w = tid >> 6, l = tid & 63, r = l & 15, g = l >> 4;
    const int row0 = 16 * w;
    const int64_t base = (int64_t)blockIdx.x * kMlpTile;

    // inputs: rows of the tile (gathered through idx), 13 features padded to 32
    for (int e = tid; e < kMlpTile * 32; e += kThreads) {
        const int rr = e >> 5, f = e & 31;
        const int64_t row = base + rr;
        float v = 0.f;
        if (row < n && f < kMlpIn) {
            const int64_t src = idx ? (int64_t)idx[row] : row;
            v = x[src * kMlpIn + f];
        }
        const uint16_t b = to_bf16(v);
        HA[rr * kSA + f] = b;
        if (TRAIN) Ht0[f * kST + rr] = b;
    }
    __syncthreads();

    f32x4 acc[8], z1[8], z2[8], z3[8];
    mm<1, 8>(HA, kSA, row0, m.wf1, 32, 0, acc);
    hidden_out<TRAIN>(acc, m.params + kMlpB1, row0, HB, Ht1, z1);
    __syncthreads();
    mm<4, 8>(HB, kSA, row0, m.wf2, 128, 0, acc);
    hidden_out<TRAIN>(acc, m.params + kMlpB2, row0, HA, Ht2, z2);
    __syncthreads();
    mm<4, 8>(HA, kSA, row0, m.wf3, 128, 0, acc);
    hidden_out<TRAIN>(acc, m.params + kMlpB3, row0, HB, Ht3, z3);
    __syncthreads();
    f32x4 out;
    mm<4, 1>(HB, kSA, row0, m.wf4, 128, 0, &out);
    const int col = r;
    const float b4 = col < kMlpOut ? m.params[kMlpB4 + col] : 0.f;
    if (!TRAIN) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t row = base + row0 + 4 * g + i;
            if (row < n && col < kMlpOut) y[row * kMlpOut + col] = out[i] + b4;
        }
        return;
    }

    // ---- backward ------------------------------------------------------
    // dY = scale (y - t); bf16 copies: row-major [32][32] in HA (columns
    // >= 9 zero), transposed [16][32] in Dt.
    __syncthreads();  // all reads of HA as the layer-3 input are done
    float dz4[4], loss = 0.f, s4 = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int64_t row = base + row0 + 4 * g + i;
        float d = 0.f;
        if (row < n && col < kMlpOut) {
            const int64_t src = idx ? (int64_t)idx[row] : row;
            const float e = (out[i] + b4) - tgt[src * kMlpOut + col];
            loss += e * e;
            d = scale * e;
        }
        dz4[i] = d;
        s4 += d;
    }
    for (int e = tid; e < kMlpTile * 32; e += kThreads) HA[(e >> 5) * kSA + (e & 31)] = 0;
    __syncthreads();
    {
        uint16_t db[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            db[i] = to_bf16(dz4[i]);
            HA[(row0 + 4 * g + i) * kSA + col] = db[i];
        }
        uint2 pk;
        pk.x = (uint32_t)db[0] | ((uint32_t)db[1] << 16);
        pk.y = (uint32_t)db[2] | ((uint32_t)db[3] << 16);
        *(uint2*)(Dt + col * kST + row0 + 4 * g) = pk;
        s4 += __shfl_xor(s4, 16, 64);
        s4 += __shfl_xor(s4, 32, 64);
        if (g == 0) bsum[w * 128 + col] = s4;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) loss += __shfl_xor(loss, o, 64);
    if (l == 0) lsum[w] = loss;
    __syncthreads();
    float* P = partial + (size_t)blockIdx.x * kMlpParams;
    if (tid < kMlpOut) P[kMlpB4 + tid] = bsum[tid] + bsum[128 + tid];
    if (tid == 0) loss_partial[blockIdx.x] = lsum[0] + lsum[1];
    // dW4 (16 output rows of which 9 are real) x 128 inputs: wave w takes input tiles 4w..4w+3
    {
        f32x4 a4[4];
        mm<1, 4>(Dt, kST, 0, Ht3, kST, 64 * w, a4);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 64 * w + 16 * t + r;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int j = 4 * g + i;
                if (j < kMlpOut) P[kMlpW4 + k * kMlpOut + j] = a4[t][i];
            }
        }
    }
    // dH3 = dZ4 W4^T (contraction over the 9 outputs padded to 32)
    mm<1, 8>(HA, kSA, row0, m.wb4, 32, 0, acc);
    __syncthreads();  // Dt and HA (dZ4) fully read
    grad_out(acc, z3, row0, HB, Dt, bsum);
    __syncthreads();
    if (tid < 128) P[kMlpB3 + tid] = bsum[tid] + bsum[128 + tid];
    weight_grad<8>(Dt, Ht2, 4 * w, 4, 128, 128, P + kMlpW3);
    mm<4, 8>(HB, kSA, row0, m.wb3, 128, 0, acc);
    __syncthreads();
    grad_out(acc, z2, row0, HA, Dt, bsum);
    __syncthreads();
    if (tid < 128) P[kMlpB2 + tid] = bsum[tid] + bsum[128 + tid];
    weight_grad<8>(Dt, Ht1, 4 * w, 4, 128, 128, P + kMlpW2);
    mm<4, 8>(HA, kSA, row0, m.wb2, 128, 0, acc);
    __syncthreads();
    grad_out(acc, z1, row0, HB, Dt, bsum);
    __syncthreads();
    if (tid < 128) P[kMlpB1 + tid] = bsum[tid] + bsum[128 + tid];
    weight_grad<2>(Dt, Ht0, 4 * w, 4, kMlpIn, 128, P + kMlpW1);
}

// grad[p] = sum over blocks of the partials (fixed order); loss likewise.
__global__ void k_mlp_reduce(const float* partial, const float* loss_partial, int64_t nblk, float* grad,
                             double* loss, double denom) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < kMlpParams) {
        float s = 0.f;
        for (int64_t b = 0; b < nblk; ++b) s += partial[(size_t)b * kMlpParams + p];
        grad[p] = s;
    }
    if (p == 0) {
        double s = 0.0;
        for (int64_t b = 0; b < nblk; ++b) s += (double)loss_partial[b];
        *loss = s / denom;
    }
}

__global__ void k_mlp_adam(float* params, const float* grad, float* m, float* v, float lr, float b1, float b2,
                           float eps, float c1, float c2) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    const float g = grad[p];
    const float mm_ = b1 * m[p] + (1.0f - b1) * g;
    const float vv = b2 * v[p] + (1.0f - b2) * g * g;
    m[p] = mm_;
    v[p] = vv;
    params[p] -= lr * (mm_ / c1) / (sqrtf(vv / c2) + eps);
}

// bf16 operand copies of the FP32 weights (zero padding).
__global__ void k_mlp_pack(const float* P, uint16_t* out) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= kMlpPackTotal) return;
    float v = 0.f;
    if (e < kOffWf2) {  // wf1[n][k], k < 32
        const int q = e - kOffWf1, nn = q >> 5, k = q & 31;
        if (k < kMlpIn) v = P[kMlpW1 + k * 128 + nn];
    } else if (e < kOffWf3) {
        const int q = e - kOffWf2, nn = q >> 7, k = q & 127;
        v = P[kMlpW2 + k * 128 + nn];
    } else if (e < kOffWf4) {
        const int q = e - kOffWf3, nn = q >> 7, k = q & 127;
        v = P[kMlpW3 + k * 128 + nn];
    } else if (e < kOffWb2) {  // wf4[j][k], j < 16
        const int q = e - kOffWf4, j = q >> 7, k = q & 127;
        if (j < kMlpOut) v = P[kMlpW4 + k * kMlpOut + j];
    } else if (e < kOffWb3) {  // wb2[k][n]
        v = P[kMlpW2 + (e - kOffWb2)];
    } else if (e < kOffWb4) {
        v = P[kMlpW3 + (e - kOffWb3)];
    } else {  // wb4[k][j], j < 32
        const int q = e - kOffWb4, k = q >> 5, j = q & 31;
        if (j < kMlpOut) v = P[kMlpW4 + k * kMlpOut + j];
    }
    out[e] = to_bf16(v);
}

// Initial weights uniform in (-1, 1)/sqrt(fan_in) (purpose 8, block 1,
// subject = parameter index), biases zero.
__global__ void k_mlp_init(float* P, RngKey key) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams) return;
    int fan = 0;
    if (p < kMlpB1) fan = kMlpIn;
    else if (p >= kMlpW2 && p < kMlpB2) fan = kMlpHid;
    else if (p >= kMlpW3 && p < kMlpB3) fan = kMlpHid;
    else if (p >= kMlpW4 && p < kMlpB4) fan = kMlpHid;
    if (!fan) {
        P[p] = 0.f;
        return;
    }
    const Rand4 r = draw(key, (uint32_t)p, 0u, kPurposeMlp, 1);
    P[p] = (float)((2.0 * u01(r.w[0], r.w[1]) - 1.0) / sqrt((double)fan));
}

// Minibatch of indices in [0, n), drawn with replacement (purpose 8).
__global__ void k_mlp_batch(RngKey key, uint32_t step, int64_t n, int64_t batch, int32_t* idx) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= batch) return;
    const Rand4 r = draw(key, (uint32_t)(i & 0xFFFFFFFF), step, kPurposeMlp, 0);
    idx[i] = (int32_t)pick(r.w[0], (uint32_t)n);
}

}  // namespace

MlpDev mlp_dev_view(const float* params, const uint16_t* packed) {
    MlpDev d;
    d.wf1 = packed + kOffWf1;
    d.wf2 = packed + kOffWf2;
    d.wf3 = packed + kOffWf3;
    d.wf4 = packed + kOffWf4;
    d.wb2 = packed + kOffWb2;
    d.wb3 = packed + kOffWb3;
    d.wb4 = packed + kOffWb4;
    d.params = params;
    return d;
}

void launch_mlp_pack(hipStream_t s, const float* params, uint16_t* packed) {
    hipLaunchKernelGGL(k_mlp_pack, dim3((kMlpPackTotal + 255) / 256), dim3(256), 0, s, params, packed);
}

int64_t mlp_blocks(int64_t n) { return (n + kMlpTile - 1) / kMlpTile; }

void launch_mlp_forward(hipStream_t s, const MlpDev& m, const float* x, const int32_t* idx, int64_t n, float* y) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_mlp_tile<false>, dim3((unsigned)mlp_blocks(n)), dim3(kThreads), 0, s, m, x,
                       (const float*)nullptr, idx, n, 0.f, y, (float*)nullptr, (float*)nullptr);
}

void launch_mlp_grad(hipStream_t s, const MlpDev& m, const float* x, const float* t, const int32_t* idx, int64_t n,
                     float* partial, float* loss_partial) {
    if (n <= 0) return;
    const float scale = (float)(2.0 / ((double)n * kMlpOut));
    hipLaunchKernelGGL(k_mlp_tile<true>, dim3((unsigned)mlp_blocks(n)), dim3(kThreads), 0, s, m, x, t, idx, n, scale,
                       (float*)nullptr, partial, loss_partial);
}

void launch_mlp_reduce(hipStream_t s, const float* partial, const float* loss_partial, int64_t nblk, float* grad,
                       double* loss, double denom) {
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, partial, loss_partial, nblk,
                       grad, loss, denom);
}

void launch_mlp_adam(hipStream_t s, float* params, const float* grad, float* m, float* v, int step, float lr,
                     float b1, float b2, float eps) {
    const float c1 = (float)(1.0 - std::pow((double)b1, step));
    const float c2 = (float)(1.0 - std::pow((double)b2, step));
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params, grad, m, v, lr, b1, b2,
                       eps, c1, c2);
}

void launch_mlp_init(hipStream_t s, float* params, RngKey key) {
    hipLaunchKernelGGL(k_mlp_init, dim3((kMlpParams + 255) / 256), dim3(256), 0, s, params, key);
}

void launch_mlp_batch(hipStream_t s, RngKey key, uint32_t step, int64_t n, int64_t batch, int32_t* idx) {
    hipLaunchKernelGGL(k_mlp_batch, dim3((unsigned)((batch + 255) / 256)), dim3(256), 0, s, key, step, n, batch, idx);
}

}  // namespace dsmcx
