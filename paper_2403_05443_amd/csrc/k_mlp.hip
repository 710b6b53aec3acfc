// k_mlp.hip - the warm-start surrogate: an 8 -> 64 -> 64 -> 6 tanh MLP whose
// forward and backward passes run on the gfx950 matrix cores (bfloat16
// operands, FP32 accumulation), plus the gradient reduction and the Adam
// update (Kingma & Ba 2015).
//
// Work split: a wave owns a tile of 16 samples and carries it through all
// three layers (and back); a work-group of four waves shares one bfloat16 copy
// of the weights in LDS.  Products over the 64 hidden units (forward layers 2
// and 3, the error back-propagated into layer 1) are sums of 16 x 16 x 32
// tiles (v_mfma_f32_16x16x32_bf16); products over 16 (the padded inputs and
// outputs, and the weight gradients over the tile's 16 samples) take the
// 16 x 16 x 16 shape (v_mfma_f32_16x16x16_bf16).
// Rounding points (mirrored by the FP64 reference): inputs, weights, hidden
// activations and back-propagated errors are rounded to bfloat16 where they
// enter a product; biases, tanh, error terms and all sums stay FP32.  Each
// tile writes its own partial gradient, and one thread per parameter sums the
// tiles in a fixed order, so results do not depend on scheduling.
#include "lbell_dev.h"
#include "lbell_launch.h"

namespace lbd {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MLP_WAVES = 4;  // tiles of 16 samples per work-group

__device__ __forceinline__ uint16_t to_bf16(float v) {  // round to nearest even (finite inputs)
    uint32_t u = __float_as_uint(v);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// acc += A * B for 16 x 16 tiles given by element accessors A(m, k), B(k, n)
// returning bfloat16 bits.  Lane l supplies A[l % 16][4 (l / 16) + j] and
// B[4 (l / 16) + j][l % 16], j = 0..3, and receives D[4 (l / 16) + j][l % 16].
template <class FA, class FB>
__device__ __forceinline__ f32x4 mma16(FA A, FB B, f32x4 acc, int lane) {
    const int r = lane & 15, g = lane >> 4;
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        a[j] = (short)A(r, 4 * g + j);
        b[j] = (short)B(4 * g + j, r);
    }
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
}

// The same for a K = 32 slice: lane l supplies A[l % 16][8 (l / 16) + j] and
// B[8 (l / 16) + j][l % 16], j = 0..7; D as above.  A and B take the same K
// order, so the sum pairs A[m][k] with B[k][n] whatever K order the unit uses.
template <class FA, class FB>
__device__ __forceinline__ f32x4 mma32(FA A, FB B, f32x4 acc, int lane) {
    const int r = lane & 15, g = lane >> 4;
    bf16x8 a, b;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        a[j] = __builtin_bit_cast(__bf16, (uint16_t)A(r, 8 * g + j));
        b[j] = __builtin_bit_cast(__bf16, (uint16_t)B(8 * g + j, r));
    }
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
}

struct MlpShm {
    uint16_t w1[MLP_H][16];   // W1 with the 8 inputs padded to 16
    uint16_t w2[MLP_H][MLP_H];
    uint16_t w3[16][MLP_H];   // W3 with the 6 outputs padded to 16
    struct Wave {
        uint16_t x[16][16];
        uint16_t h1[16][MLP_H], h2[16][MLP_H];
        uint16_t d3[16][16], d2[16][MLP_H], d1[16][MLP_H];
        float e[16][MLP_H];   // FP32 error terms of the current layer (bias gradients)
    } w[MLP_WAVES];
};

// mode 0: outputs for n samples -> out (n x 6).  mode 1: loss and gradient of
// the mean squared error against Y, scaled so that the tiles' partial
// gradients sum to the gradient of L = scale / 2 * sum (y - Y)^2; partial of
// tile t at G + t * MLP_NP, its sum of squared errors at Lpart[t].
__global__ __launch_bounds__(64 * MLP_WAVES) void k_mlp(MlpArgs a) {
    __shared__ MlpShm sh;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const float* P = a.P;
    for (int k = tid; k < MLP_H * 16; k += blockDim.x) {
        const int o = k >> 4, i = k & 15;
        sh.w1[o][i] = i < MLP_IN ? to_bf16(P[MLP_OW1 + o * MLP_IN + i]) : 0;
    }
    for (int k = tid; k < MLP_H * MLP_H; k += blockDim.x) sh.w2[k >> 6][k & 63] = to_bf16(P[MLP_OW2 + k]);
    for (int k = tid; k < 16 * MLP_H; k += blockDim.x) {
        const int o = k >> 6;
        sh.w3[o][k & 63] = o < MLP_OUT ? to_bf16(P[MLP_OW3 + k]) : 0;
    }
    MlpShm::Wave& W = sh.w[wv];
    const int tile = blockIdx.x * MLP_WAVES + wv;
    const int base = tile * 16;
    for (int k = lane; k < 256; k += 64) {
        const int m = k >> 4, i = k & 15;
        W.x[m][i] = (i < MLP_IN && base + m < a.n) ? to_bf16(a.X[(long long)(base + m) * MLP_IN + i]) : 0;
    }
    __syncthreads();
    // every wave runs every phase (a tile past the end computes on zeros and
    // writes nothing), so the work-group barriers below are reached by all
    const bool live = base < a.n;
    const int r = lane & 15, g = lane >> 4;

    // forward
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        f32x4 acc = {0, 0, 0, 0};
        acc = mma16([&](int m, int k) { return W.x[m][k]; }, [&](int k, int n) { return sh.w1[16 * ot + n][k]; },
                    acc, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            W.h1[4 * g + j][16 * ot + r] = to_bf16(tanhf(acc[j] + P[MLP_OB1 + 16 * ot + r]));
    }
    __syncthreads();
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        f32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int kt = 0; kt < 2; ++kt)
            acc = mma32([&](int m, int k) { return W.h1[m][32 * kt + k]; },
                        [&](int k, int n) { return sh.w2[16 * ot + n][32 * kt + k]; }, acc, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            W.h2[4 * g + j][16 * ot + r] = to_bf16(tanhf(acc[j] + P[MLP_OB2 + 16 * ot + r]));
    }
    __syncthreads();
    f32x4 y = {0, 0, 0, 0};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt)
        y = mma32([&](int m, int k) { return W.h2[m][32 * kt + k]; },
                  [&](int k, int n) { return sh.w3[n][32 * kt + k]; }, y, lane);
    if (a.mode == 0) {
        if (r < MLP_OUT)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int m = 4 * g + j;
                if (live && base + m < a.n) a.out[(long long)(base + m) * MLP_OUT + r] = y[j] + P[MLP_OB3 + r];
            }
        return;
    }

    // backward: e3 = dL/dy.  Tiles past the end write nothing (G is only
    // valid for tiles that hold samples)
    float* G = live ? a.G + (long long)tile * MLP_NP : nullptr;
    float sq = 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int m = 4 * g + j;
        float e = 0.f;
        if (r < MLP_OUT && base + m < a.n) {
            const float d = y[j] + P[MLP_OB3 + r] - a.Y[(long long)(base + m) * MLP_OUT + r];
            sq += d * d;
            e = a.scale * d;
        }
        W.e[m][r] = e;
        W.d3[m][r] = to_bf16(e);
    }
    __syncthreads();
    // squared error of the tile (lanes hold disjoint entries)
    for (int off = 32; off > 0; off >>= 1) sq += __shfl_xor(sq, off);
    if (live && lane == 0) a.Lpart[tile] = sq;
    if (live && lane < MLP_OUT) {
        float s = 0.f;
        for (int m = 0; m < 16; ++m) s += W.e[m][lane];
        G[MLP_OB3 + lane] = s;
    }
    // dW3[n][k] = sum_m e3[m][n] h2[m][k]
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        f32x4 acc = {0, 0, 0, 0};
        acc = mma16([&](int n, int m) { return W.d3[m][n]; }, [&](int m, int k) { return W.h2[m][16 * kt + k]; },
                    acc, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (live && 4 * g + j < MLP_OUT) G[MLP_OW3 + (4 * g + j) * MLP_H + 16 * kt + r] = acc[j];
    }
    // e2 = (e3 W3) * (1 - h2^2)
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        f32x4 acc = {0, 0, 0, 0};
        acc = mma16([&](int m, int n) { return W.d3[m][n]; }, [&](int n, int k) { return sh.w3[n][16 * kt + k]; },
                    acc, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 4 * g + j, k = 16 * kt + r;
            const float h = from_bf16(W.h2[m][k]);
            const float e = acc[j] * (1.f - h * h);
            W.e[m][k] = e;
            W.d2[m][k] = to_bf16(e);
        }
    }
    __syncthreads();
    if (live) {
        float s = 0.f;
        for (int m = 0; m < 16; ++m) s += W.e[m][lane];
        G[MLP_OB2 + lane] = s;
    }
    // dW2[o][k] = sum_m e2[m][o] h1[m][k]
#pragma unroll
    for (int ot = 0; ot < 4; ++ot)
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            f32x4 acc = {0, 0, 0, 0};
            acc = mma16([&](int o, int m) { return W.d2[m][16 * ot + o]; },
                        [&](int m, int k) { return W.h1[m][16 * kt + k]; }, acc, lane);
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (live) G[MLP_OW2 + (16 * ot + 4 * g + j) * MLP_H + 16 * kt + r] = acc[j];
        }
    // e1 = (e2 W2) * (1 - h1^2)
    __syncthreads();
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        f32x4 acc = {0, 0, 0, 0};
#pragma unroll
        for (int ot = 0; ot < 2; ++ot)
            acc = mma32([&](int m, int o) { return W.d2[m][32 * ot + o]; },
                        [&](int o, int k) { return sh.w2[32 * ot + o][16 * kt + k]; }, acc, lane);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int m = 4 * g + j, k = 16 * kt + r;
            const float h = from_bf16(W.h1[m][k]);
            const float e = acc[j] * (1.f - h * h);
            W.e[m][k] = e;
            W.d1[m][k] = to_bf16(e);
        }
    }
    __syncthreads();
    if (live) {
        float s = 0.f;
        for (int m = 0; m < 16; ++m) s += W.e[m][lane];
        G[MLP_OB1 + lane] = s;
    }
    // dW1[o][i] = sum_m e1[m][o] x[m][i]
#pragma unroll
    for (int ot = 0; ot < 4; ++ot) {
        f32x4 acc = {0, 0, 0, 0};
        acc = mma16([&](int o, int m) { return W.d1[m][16 * ot + o]; }, [&](int m, int i) { return W.x[m][i]; },
                    acc, lane);
        if (live && r < MLP_IN)
#pragma unroll
            for (int j = 0; j < 4; ++j) G[MLP_OW1 + (16 * ot + 4 * g + j) * MLP_IN + r] = acc[j];
    }
}

// One thread per parameter: sum of the tiles' partial gradients in tile
// order; mode 0 applies Adam (c1 = 1 / (1 - beta1^t), c2 = 1 / (1 - beta2^t)),
// mode 1 writes the sum to gsum.  Thread 0 also adds the tiles' squared
// errors to *loss_acc, or writes their sum over loss_div to *loss_out.
__global__ __launch_bounds__(256) void k_mlp_reduce(MlpReduceArgs a) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0 && (a.loss_acc || a.loss_out)) {
        double s = 0.0;
        for (int t = 0; t < a.ntiles; ++t) s += (double)a.Lpart[t];
        if (a.loss_acc) *a.loss_acc += s;
        if (a.loss_out) *a.loss_out = (float)(s / a.loss_div);
    }
    if (p >= MLP_NP) return;
    float gsum = 0.f;
    for (int t = 0; t < a.ntiles; ++t) gsum += a.G[(long long)t * MLP_NP + p];
    if (a.mode == 1) {
        a.gsum[p] = gsum;
        return;
    }
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float m = b1 * a.M[p] + (1.f - b1) * gsum;
    const float v = b2 * a.V[p] + (1.f - b2) * gsum * gsum;
    a.M[p] = m;
    a.V[p] = v;
    a.P[p] -= a.lr * (m * a.c1) / (sqrtf(v * a.c2) + eps);
}

hipError_t launch_mlp(const MlpArgs& a, hipStream_t st) {
    if (a.n <= 0) return hipSuccess;
    const int tiles = (a.n + 15) / 16;
    const int blocks = (tiles + MLP_WAVES - 1) / MLP_WAVES;
    hipLaunchKernelGGL(k_mlp, dim3(blocks), dim3(64 * MLP_WAVES), 0, st, a);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(const MlpReduceArgs& a, hipStream_t st) {
    hipLaunchKernelGGL(k_mlp_reduce, dim3((MLP_NP + 255) / 256), dim3(256), 0, st, a);
    return hipGetLastError();
}

}  // namespace lbd
