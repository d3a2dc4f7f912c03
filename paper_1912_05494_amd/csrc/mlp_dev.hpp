// mlp_dev.hpp -- device code of the surrogate network shared by the training
// kernels and the render: matrix-core fragments, the BF16 weight layout
// staged in LDS, and the forward pass of one 16-sample tile per wave.
#pragma once
#include <hip/hip_runtime.h>

#include "sdm_dev.hpp"

namespace sdm {

// ---------------------------------------------------------------------------
// MFMA fragments (gfx950).  For a lane l, g = l / 16, c = l % 16:
//   v_mfma_f32_16x16x32_bf16:  A[c][8g .. 8g+7], B[8g .. 8g+7][c], D[4g .. 4g+3][c]
//   v_mfma_f32_16x16x16_bf16:  A[c][4g .. 4g+3], B[4g .. 4g+3][c], D[4g .. 4g+3][c]
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f32x4 mfma16(s16x4 a, s16x4 b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ short bits(__bf16 x) { return __builtin_bit_cast(short, x); }

// ---------------------------------------------------------------------------
// Surrogate network
// ---------------------------------------------------------------------------
// Kernel weight layout (BF16): W1p[64][32] (inputs 12..31 zero), W2[64][64],
// W3[64][64], W4p[16][64] (outputs 3..15 zero); biases FP32 b1[64] b2[64]
// b3[64] b4p[16].  Canonical FP32 parameter vector: W1[64][12] b1 W2 b2 W3 b3
// W4[3][64] b4 E[n_panes][8].
constexpr int kNetParams = 64 * 12 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 3 * 64 + 3;   // 9347
constexpr int kOffW1 = 0, kOffB1 = 768, kOffW2 = 832, kOffB2 = 4928, kOffW3 = 4992, kOffB3 = 9088,
              kOffW4 = 9152, kOffB4 = 9344, kOffE = 9347;
constexpr int kWb = 64 * 32 + 64 * 64 + 64 * 64 + 16 * 64;   // 11264 BF16
constexpr int kBb = 64 + 64 + 64 + 16;                       // 208 FP32

// LDS row strides (BF16 elements) of the staged weights and the per-wave
// activations: rows padded by 8, so consecutive rows start 16 bytes apart
// modulo the 128-byte bank cycle (80 and 144 bytes; 48 for the 16-wide
// output gradients) and a column read by 16 lanes does not fall in one bank.
constexpr int kLd32 = 40, kLd64 = 72, kLd16 = 24;

struct alignas(16) NetLds {
    __bf16 W1[64 * kLd32], W2[64 * kLd64], W3[64 * kLd64], W4[16 * kLd64];
    float b1[64], b2[64], b3[64], b4[16];
};

struct alignas(16) WaveBuf {   // per wave, 16 samples
    __bf16 X0[16 * kLd32], H1[16 * kLd64], H2[16 * kLd64], H3[16 * kLd64], Z0[16 * kLd64], Z1[16 * kLd64],
        dO[16 * kLd16];
    float O[16 * 16];
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Stages the weights (rows of 8-value chunks into the padded rows) and the
// biases in LDS with 16-byte copies; the device copies are allocation-aligned.
static_assert(kWb * 2 % 16 == 0 && kBb * 4 % 16 == 0, "16-byte staging");
__device__ __forceinline__ void load_net(NetLds &net, const __bf16 *wb, const float *bb)
{
    const uint4 *src = reinterpret_cast<const uint4 *>(wb);
    for (int q = threadIdx.x; q < kWb * 2 / 16; q += blockDim.x) {
        __bf16 *d;
        if (q < 256) d = net.W1 + (q / 4) * kLd32 + 8 * (q % 4);                       // W1p [64][32]
        else if (q < 768) d = net.W2 + ((q - 256) / 8) * kLd64 + 8 * ((q - 256) % 8);  // W2 [64][64]
        else if (q < 1280) d = net.W3 + ((q - 768) / 8) * kLd64 + 8 * ((q - 768) % 8); // W3 [64][64]
        else d = net.W4 + ((q - 1280) / 8) * kLd64 + 8 * ((q - 1280) % 8);             // W4p [16][64]
        *reinterpret_cast<uint4 *>(d) = src[q];
    }
    const uint4 *bs = reinterpret_cast<const uint4 *>(bb);
    uint4 *bd = reinterpret_cast<uint4 *>(net.b1);
    for (int i = threadIdx.x; i < kBb * 4 / 16; i += blockDim.x) bd[i] = bs[i];
    __syncthreads();
}

// Inputs of one sample: cos, (lambda - 580) / 200, (d - 3.5) / 1.5,
// rho_b / 34, then the pane's 8 embedding values.
__device__ __forceinline__ void features(float cosv, float lam, float d, float rho, const float *E, __bf16 *row)
{
    row[0] = (__bf16)cosv;
    row[1] = (__bf16)((lam - 580.0f) / 200.0f);
    row[2] = (__bf16)((d - 3.5f) / 1.5f);
    row[3] = (__bf16)(rho / 34.0f);
    for (int e = 0; e < 8; ++e) row[4 + e] = (__bf16)E[e];
    for (int e = 12; e < 32; ++e) row[e] = (__bf16)0.0f;
}

// Y[16][64] = relu(X[16][K] W[64][K]^T + b), K = 32 * ksteps, stored BF16
// with row stride ldy.
__device__ __forceinline__ void dense_relu(const __bf16 *X, int ldx, const __bf16 *W, int ldw, const float *b,
                                           int ksteps, __bf16 *Y, int ldy)
{
    const int l = lane_id(), g = l / 16, c = l % 16;
    for (int t = 0; t < 4; ++t) {
        f32x4 acc = {0, 0, 0, 0};
        for (int ks = 0; ks < ksteps; ++ks) {
            const bf16x8 a = *reinterpret_cast<const bf16x8 *>(X + c * ldx + 32 * ks + 8 * g);
            const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(W + (16 * t + c) * ldw + 32 * ks + 8 * g);
            acc = mfma32(a, bv, acc);
        }
        for (int r = 0; r < 4; ++r) {
            const float z = acc[r] + b[16 * t + c];
            Y[(4 * g + r) * ldy + 16 * t + c] = (__bf16)(z > 0.0f ? z : 0.0f);
        }
    }
}

__device__ __forceinline__ void forward_tile(const NetLds &net, WaveBuf &wb)
{
    dense_relu(wb.X0, kLd32, net.W1, kLd32, net.b1, 1, wb.H1, kLd64);
    wave_sync();
    dense_relu(wb.H1, kLd64, net.W2, kLd64, net.b2, 2, wb.H2, kLd64);
    wave_sync();
    dense_relu(wb.H2, kLd64, net.W3, kLd64, net.b3, 2, wb.H3, kLd64);
    wave_sync();
    const int l = lane_id(), g = l / 16, c = l % 16;
    f32x4 acc = {0, 0, 0, 0};
    for (int ks = 0; ks < 2; ++ks) {
        const bf16x8 a = *reinterpret_cast<const bf16x8 *>(wb.H3 + c * kLd64 + 32 * ks + 8 * g);
        const bf16x8 bv = *reinterpret_cast<const bf16x8 *>(net.W4 + c * kLd64 + 32 * ks + 8 * g);
        acc = mfma32(a, bv, acc);
    }
    for (int r = 0; r < 4; ++r) wb.O[(4 * g + r) * 16 + c] = acc[r] + net.b4[c];
    wave_sync();
}

__device__ __forceinline__ void heads(float o0, float o1, float o2, float &R, float &T, float &w)
{
    const float m = fmaxf(fmaxf(o0, o1), 0.0f);
    const float a = expf(o0 - m), b = expf(o1 - m), c = expf(-m);
    const float s = a + b + c;
    R = a / s;
    T = b / s;
    w = o2 > 30.0f ? o2 : log1pf(expf(o2));
}

}  // namespace sdm
