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

// ---- gradient over many samples, in a fixed order (no atomics)
//
// The samples are taken in chunks of MLP_CHUNK.  A workgroup of
// MLP_THREADS threads computes a chunk layer by layer in LDS (activations,
// then the output error and the back-propagated errors), then every thread
// sums, for the parameters it owns, the chunk's per-sample terms in sample
// order.  A workgroup that takes several chunks adds their sums in chunk
// order.  So the gradient of samples [0, n) is
//   ((0 + G_0) + G_1) + ... ,  G_c = sum over the chunk's samples in order,
// whether one workgroup runs every chunk or each chunk has its own
// workgroup whose sums are added afterwards in chunk order: both give the
// same floats.
constexpr int MLP_CHUNK = 64;
constexpr int MLP_THREADS = 256;
constexpr int MLP_GRAD_N = MLP_NPARAM + 1;  // the gradient, then the loss
constexpr int MLP_OWN = (MLP_GRAD_N + MLP_THREADS - 1) / MLP_THREADS;  // entries per thread

struct MlpChunkLDS {
    float w[MLP_NPARAM];
    float x[MLP_CHUNK][MLP_IN];
    float h1[MLP_CHUNK][MLP_H];
    float h2[MLP_CHUNK][MLP_H];
    float d1[MLP_CHUNK][MLP_H];
    float d2[MLP_CHUNK][MLP_H];
    float d3[MLP_CHUNK][MLP_OUT];
    float y[MLP_CHUNK][MLP_OUT];
};

// The chunk starting at sample c0: per-sample activations and errors in L.
// Samples past n contribute nothing (their errors are zero).
__device__ __forceinline__ void mlp_chunk_pass(MlpChunkLDS& L, const float* __restrict__ X,
                                               const float* __restrict__ Y, long long n, long long c0) {
#pragma clang fp contract(off)
    const int t = threadIdx.x;
    for (int e = t; e < MLP_CHUNK * MLP_IN; e += MLP_THREADS) {
        const long long s = c0 + e / MLP_IN;
        L.x[e / MLP_IN][e % MLP_IN] = s < n ? X[s * MLP_IN + e % MLP_IN] : 0.f;
    }
    for (int e = t; e < MLP_CHUNK * MLP_OUT; e += MLP_THREADS) {
        const long long s = c0 + e / MLP_OUT;
        L.y[e / MLP_OUT][e % MLP_OUT] = s < n ? Y[s * MLP_OUT + e % MLP_OUT] : 0.f;
    }
    __syncthreads();
    for (int e = t; e < MLP_CHUNK * MLP_H; e += MLP_THREADS) {
        const int s = e / MLP_H, j = e % MLP_H;
        float a = L.w[MLP_B1 + j];
        for (int i = 0; i < MLP_IN; ++i) a = fmaf(L.w[MLP_W1 + j * MLP_IN + i], L.x[s][i], a);
        L.h1[s][j] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int e = t; e < MLP_CHUNK * MLP_H; e += MLP_THREADS) {
        const int s = e / MLP_H, j = e % MLP_H;
        float a = L.w[MLP_B2 + j];
        for (int i = 0; i < MLP_H; ++i) a = fmaf(L.w[MLP_W2 + j * MLP_H + i], L.h1[s][i], a);
        L.h2[s][j] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int e = t; e < MLP_CHUNK * MLP_OUT; e += MLP_THREADS) {
        const int s = e / MLP_OUT, o = e % MLP_OUT;
        float a = L.w[MLP_B3 + o];
        for (int i = 0; i < MLP_H; ++i) a = fmaf(L.w[MLP_W3 + o * MLP_H + i], L.h2[s][i], a);
        L.d3[s][o] = c0 + s < n ? a - L.y[s][o] : 0.f;
    }
    __syncthreads();
    for (int e = t; e < MLP_CHUNK * MLP_H; e += MLP_THREADS) {
        const int s = e / MLP_H, i = e % MLP_H;
        float a = 0.f;
        for (int o = 0; o < MLP_OUT; ++o) a = fmaf(L.w[MLP_W3 + o * MLP_H + i], L.d3[s][o], a);
        L.d2[s][i] = L.h2[s][i] > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int e = t; e < MLP_CHUNK * MLP_H; e += MLP_THREADS) {
        const int s = e / MLP_H, i = e % MLP_H;
        float a = 0.f;
        for (int j = 0; j < MLP_H; ++j) a = fmaf(L.w[MLP_W2 + j * MLP_H + i], L.d2[s][j], a);
        L.d1[s][i] = L.h1[s][i] > 0.f ? a : 0.f;
    }
    __syncthreads();
}

// Sum over the chunk's samples (in order) of the term of gradient entry p
// (p == MLP_NPARAM: the loss 0.5 |out - y|^2).
__device__ __forceinline__ float mlp_chunk_term(const MlpChunkLDS& L, int p) {
#pragma clang fp contract(off)
    float a = 0.f;
    if (p < MLP_B1) {
        const int j = p / MLP_IN, i = p % MLP_IN;
        for (int s = 0; s < MLP_CHUNK; ++s) a = fmaf(L.d1[s][j], L.x[s][i], a);
    } else if (p < MLP_W2) {
        for (int s = 0; s < MLP_CHUNK; ++s) a += L.d1[s][p - MLP_B1];
    } else if (p < MLP_B2) {
        const int j = (p - MLP_W2) / MLP_H, i = (p - MLP_W2) % MLP_H;
        for (int s = 0; s < MLP_CHUNK; ++s) a = fmaf(L.d2[s][j], L.h1[s][i], a);
    } else if (p < MLP_W3) {
        for (int s = 0; s < MLP_CHUNK; ++s) a += L.d2[s][p - MLP_B2];
    } else if (p < MLP_B3) {
        const int o = (p - MLP_W3) / MLP_H, i = (p - MLP_W3) % MLP_H;
        for (int s = 0; s < MLP_CHUNK; ++s) a = fmaf(L.d3[s][o], L.h2[s][i], a);
    } else if (p < MLP_NPARAM) {
        for (int s = 0; s < MLP_CHUNK; ++s) a += L.d3[s][p - MLP_B3];
    } else {
        for (int s = 0; s < MLP_CHUNK; ++s)
            for (int o = 0; o < MLP_OUT; ++o) a = fmaf(0.5f * L.d3[s][o], L.d3[s][o], a);
    }
    return a;
}

}  // namespace kdt
