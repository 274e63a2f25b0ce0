// mlp_common.hpp -- the learned Newton initial guess: parameter layout, the
// model object, input features and bfloat16-weight inference (shared by the
// training kernels and the temperature solve of the AP step).
//
// Network (5 -> 64 -> 64 -> 1, exact gelu x Phi(x)):
//   x  = (f - mu_f) / sd_f,  f = log10(rho*, T^n, sigma0 (T^n)^-m, eps, dt)
//   h1 = gelu(W1 x + b1),  h2 = gelu(W2 h1 + b2),  y = W3 . h2 + b3
//   T0 = T^n exp(mu_t + sd_t y)          (y predicts log(T^{n+1} / T^n))
// Flat parameter vector: W1 (64x5 row-major), b1, W2 (64x64, row = output
// unit), b2, W3, b3 -- 4609 values; normalisation: mu_f(5) sd_f(5) mu_t sd_t.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

struct grte_mlp {
    float *theta = nullptr;       // FP32 master parameters
    uint16_t *wbf = nullptr;      // bfloat16 copy used for inference
    float *am = nullptr, *av = nullptr;   // Adam moments
    float *norm = nullptr;        // 12 normalisation values
    float *gpart = nullptr;       // per-block partial gradients of the training kernel
    float *lpart = nullptr;       // per-block partial losses
    float *lhist = nullptr;       // device loss history of one training call
    int gcap = 0;                 // blocks gpart can hold
    int hcap = 0;                 // entries lhist can hold
    int adam_k = 0;               // Adam steps taken
    hipStream_t stream = nullptr;
};

namespace {

constexpr int MLP_IN = 5, MLP_H = 64;
constexpr int MLP_OW1 = 0, MLP_OB1 = 320, MLP_OW2 = 384, MLP_OB2 = 4480, MLP_OW3 = 4544, MLP_OB3 = 4608;
constexpr int MLP_NPARAM = 4609;
constexpr int MLP_NNORM = 12;

__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float((unsigned)h << 16); }

// binary32 -> bfloat16, round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ uint16_t f_to_bf16(float x)
{
    unsigned u = __float_as_uint(x);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

__device__ __forceinline__ float gelu_prime_f(float x)
{
    return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * expf(-0.5f * x * x) * 0.39894228040143268f;
}

// log10 inputs, computed in binary64 and rounded to binary32
__device__ __forceinline__ void mlp_features(double rho, double Tn, double s0, int m, double eps, double dt,
                                             float (&f)[MLP_IN])
{
    const double seff = (m == 0) ? s0 : s0 / (Tn * Tn * Tn);
    f[0] = (float)log10(fmax(fabs(rho), 1e-300));
    f[1] = (float)log10(Tn);
    f[2] = (float)log10(seff);
    f[3] = (float)log10(eps);
    f[4] = (float)log10(dt);
}

// network output for raw features f; weights in bfloat16 (W, any address
// space the caller passes), normalisation and accumulation in binary32
__device__ __forceinline__ float mlp_eval(const uint16_t *W, const float *norm, const float (&f)[MLP_IN])
{
    float x[MLP_IN];
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) x[q] = (f[q] - norm[q]) / norm[MLP_IN + q];
    float h1[MLP_H];
#pragma unroll
    for (int i = 0; i < MLP_H; ++i) {
        float z = bf16_to_f(W[MLP_OB1 + i]);
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) z += bf16_to_f(W[MLP_OW1 + MLP_IN * i + q]) * x[q];
        h1[i] = gelu_f(z);
    }
    float y = bf16_to_f(W[MLP_OB3]);
    for (int i = 0; i < MLP_H; ++i) {
        float z = bf16_to_f(W[MLP_OB2 + i]);
#pragma unroll
        for (int j = 0; j < MLP_H; ++j) z += bf16_to_f(W[MLP_OW2 + MLP_H * i + j]) * h1[j];
        y += bf16_to_f(W[MLP_OW3 + i]) * gelu_f(z);
    }
    return y;
}

// The same network output, its second layer accumulated input by input: the
// 64 second-layer sums stay in registers while each first-layer unit is formed
// once and used at once (the 64 first-layer values are never all live), so a
// kernel doing nothing else keeps it in registers.  The sums run over the
// inputs in increasing order from the bias, as in mlp_eval.
__device__ __forceinline__ float mlp_eval_streamed(const uint16_t *W, const float *norm, const float (&f)[MLP_IN])
{
    float x[MLP_IN];
#pragma unroll
    for (int q = 0; q < MLP_IN; ++q) x[q] = (f[q] - norm[q]) / norm[MLP_IN + q];
    float z2[MLP_H];
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) z2[k] = bf16_to_f(W[MLP_OB2 + k]);
#pragma unroll 1
    for (int i = 0; i < MLP_H; ++i) {
        float z = bf16_to_f(W[MLP_OB1 + i]);
#pragma unroll
        for (int q = 0; q < MLP_IN; ++q) z += bf16_to_f(W[MLP_OW1 + MLP_IN * i + q]) * x[q];
        const float h = gelu_f(z);
#pragma unroll
        for (int k = 0; k < MLP_H; ++k) z2[k] += bf16_to_f(W[MLP_OW2 + MLP_H * k + i]) * h;
    }
    float y = bf16_to_f(W[MLP_OB3]);
#pragma unroll
    for (int k = 0; k < MLP_H; ++k) y += bf16_to_f(W[MLP_OW3 + k]) * gelu_f(z2[k]);
    return y;
}

}  // namespace
