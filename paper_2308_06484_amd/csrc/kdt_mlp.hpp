// Repair-or-rebuild selector: block features, a small FP32 multilayer
// perceptron (16 -> 32 -> 32 -> 2, ReLU) with forward, backward and SGD
// kernels, and the threshold rule it falls back to.
//
// The paper's trade-off (Sec. I and the abstract): points that move far are
// better handled by rebuilding the triangulation than by updating it.  The
// network predicts, per block and time step, the log2 cost (device clock
// ticks) of repairing the block's moves one by one (output 0) and of
// rebuilding the block from scratch (output 1); the cheaper branch runs.
// Either branch ends in the same triangulation (DT* is unique), so the
// choice changes only the time taken.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace kdt {

constexpr int MLP_IN = 16, MLP_H = 32, MLP_OUT = 2;
// parameter layout: W1[H][IN], b1[H], W2[H][H], b2[H], W3[OUT][H], b3[OUT]
constexpr int MLP_W1 = 0;
constexpr int MLP_B1 = MLP_W1 + MLP_H * MLP_IN;
constexpr int MLP_W2 = MLP_B1 + MLP_H;
constexpr int MLP_B2 = MLP_W2 + MLP_H * MLP_H;
constexpr int MLP_W3 = MLP_B2 + MLP_H;
constexpr int MLP_B3 = MLP_W3 + MLP_OUT * MLP_H;
constexpr int MLP_NPARAM = MLP_B3 + MLP_OUT;  // 1666

constexpr int LOG_FIELDS = 20;  // 16 features, branch, cost (ticks), moves, 0

// One sample's forward pass (one thread); h1, h2 keep the hidden activations
// for the backward pass.
__device__ __forceinline__ void mlp_forward1(const float* W, const float* x, float* h1, float* h2,
                                             float* out) {
#pragma unroll 4
    for (int j = 0; j < MLP_H; ++j) {
        float a = W[MLP_B1 + j];
        for (int i = 0; i < MLP_IN; ++i) a += W[MLP_W1 + j * MLP_IN + i] * x[i];
        h1[j] = a > 0.f ? a : 0.f;
    }
#pragma unroll 4
    for (int j = 0; j < MLP_H; ++j) {
        float a = W[MLP_B2 + j];
        for (int i = 0; i < MLP_H; ++i) a += W[MLP_W2 + j * MLP_H + i] * h1[i];
        h2[j] = a > 0.f ? a : 0.f;
    }
    for (int o = 0; o < MLP_OUT; ++o) {
        float a = W[MLP_B3 + o];
        for (int i = 0; i < MLP_H; ++i) a += W[MLP_W3 + o * MLP_H + i] * h2[i];
        out[o] = a;
    }
}

// Gradient of 0.5 * sum_o (out_o - y_o)^2 for one sample, added into g
// (shared-memory accumulator, float atomics).  Returns the sample's loss.
__device__ __forceinline__ float mlp_backward1(const float* W, const float* x, const float* y,
                                               float* g) {
    float h1[MLP_H], h2[MLP_H], out[MLP_OUT], d2[MLP_H], d1[MLP_H];
    mlp_forward1(W, x, h1, h2, out);
    float loss = 0.f, dout[MLP_OUT];
    for (int o = 0; o < MLP_OUT; ++o) {
        dout[o] = out[o] - y[o];
        loss += 0.5f * dout[o] * dout[o];
        atomicAdd(&g[MLP_B3 + o], dout[o]);
        for (int i = 0; i < MLP_H; ++i) atomicAdd(&g[MLP_W3 + o * MLP_H + i], dout[o] * h2[i]);
    }
    for (int i = 0; i < MLP_H; ++i) {
        float a = 0.f;
        for (int o = 0; o < MLP_OUT; ++o) a += W[MLP_W3 + o * MLP_H + i] * dout[o];
        d2[i] = h2[i] > 0.f ? a : 0.f;
    }
    for (int j = 0; j < MLP_H; ++j) {
        atomicAdd(&g[MLP_B2 + j], d2[j]);
        for (int i = 0; i < MLP_H; ++i) atomicAdd(&g[MLP_W2 + j * MLP_H + i], d2[j] * h1[i]);
    }
    for (int i = 0; i < MLP_H; ++i) {
        float a = 0.f;
        for (int j = 0; j < MLP_H; ++j) a += W[MLP_W2 + j * MLP_H + i] * d2[j];
        d1[i] = h1[i] > 0.f ? a : 0.f;
    }
    for (int j = 0; j < MLP_H; ++j) {
        atomicAdd(&g[MLP_B1 + j], d1[j]);
        for (int i = 0; i < MLP_IN; ++i) atomicAdd(&g[MLP_W1 + j * MLP_IN + i], d1[j] * x[i]);
    }
    return loss;
}

}  // namespace kdt
