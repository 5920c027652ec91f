// Per-phase selector: features of the phase-start state and the FP32 forward
// pass evaluated inside the solver (one workgroup). Shared by phased.hip and mlp.hip.
//
// Features: twelve ratios of exact integers, each evaluated in double
// precision in the order written and rounded to float once:
//   x0 = F/n              x1 = S/n                 x2 = Fp ? Sp/Fp : 0
//   x3 = min(k,4096)/4096 x4 = t inf ? 1 : min((t-a)/Wm, 64)/64
//   x5 = min(max((SD/F - a)/Wm, 0), 256)/256       x6 = min((DG/F)/(m/n), 8)/8
//   x7 = Fp ? Ip/Fp : 0   x8 = Fp ? Op/Fp : 0      x9 = Fp ? min(F/Fp, 4)/4 : 0
//   x10 = (n-R)/n         x11 = min(a/Wm, 4096)/4096
// with F = |F|, S = settled, R = reached, a = minD, t = OUT-STATIC threshold,
// SD / DG = sum over F of d / out-degree, Fp = previous |F|, Sp = previous
// |S'|, Ip / Op = previous-phase queued vertices passing IN-STATIC /
// OUT-STATIC, k = phase index, Wm = (sum of weights)/m. For Delta-stepping
// (bucket starts) x4..x9 are 0.
// Network: W1[64][12] b1[64] W2[64][64] b2[64] W3[6][64] b3[6]; each neuron is
// its bias followed by fmaf over its inputs in index order; ReLU on the two
// hidden layers. Outputs 0..2 choose the phase criterion (IN-STATIC|OUT-STATIC,
// IN-SIMPLE|OUT-SIMPLE, IN|OUT), outputs 3..5 the bucket width 2^12, 2^14, 2^16;
// the argmax takes the lowest index on ties.
#pragma once

#include "common.h"

constexpr int kMlpIn = 12, kMlpH = 64, kMlpOut = 6;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpOut * kMlpH + kMlpOut;

struct FeatIn {
    unsigned long long n, m, F, S, R, a, t, SD, DG, Fp, Sp, Ip, Op, k;
    double Wm;
    int delta_mode;
};

__device__ __forceinline__ double fdmin(double x, double y) { return x < y ? x : y; }
__device__ __forceinline__ double fdmax(double x, double y) { return x > y ? x : y; }

__device__ __noinline__ void features_dev(const FeatIn &q, float *x) {
#pragma clang fp contract(off)
    const double n = (double)q.n, m = (double)q.m, F = (double)q.F, Fp = (double)q.Fp;
    x[0] = (float)(F / n);
    x[1] = (float)((double)q.S / n);
    x[2] = (float)(q.Fp ? (double)q.Sp / Fp : 0.0);
    x[3] = (float)(fdmin((double)q.k, 4096.0) / 4096.0);
    x[10] = (float)((n - (double)q.R) / n);
    x[11] = (float)(fdmin((double)q.a / q.Wm, 4096.0) / 4096.0);
    if (q.delta_mode) {
        for (int i = 4; i < 10; ++i) x[i] = 0.0f;
        return;
    }
    x[4] = (float)(q.t == INF64 ? 1.0 : fdmin((double)(q.t - q.a) / q.Wm, 64.0) / 64.0);
    x[5] = (float)(fdmin(fdmax(((double)q.SD / F - (double)q.a) / q.Wm, 0.0), 256.0) / 256.0);
    x[6] = (float)(fdmin(((double)q.DG / F) / (m / n), 8.0) / 8.0);
    x[7] = (float)(q.Fp ? (double)q.Ip / Fp : 0.0);
    x[8] = (float)(q.Fp ? (double)q.Op / Fp : 0.0);
    x[9] = (float)(q.Fp ? fdmin(F / Fp, 4.0) / 4.0 : 0.0);
}

struct MlpLds {
    float x[kMlpIn];
    float h1[kMlpH];
    float h2[kMlpH];
    float z[kMlpOut];
    int choice;
};

// Called by every thread of one workgroup (>= 64 threads) after thread 0 has
// written L.x; returns the argmax of outputs [lo, lo+3) to every thread.
__device__ __forceinline__ int mlp_choice_block(const float *__restrict__ w, MlpLds &L, int lo) {
    const float *W1 = w, *b1 = W1 + kMlpH * kMlpIn, *W2 = b1 + kMlpH, *b2 = W2 + kMlpH * kMlpH;
    const float *W3 = b2 + kMlpH, *b3 = W3 + kMlpOut * kMlpH;
    const int j = threadIdx.x;
    __syncthreads();
    if (j < kMlpH) {
        float acc = b1[j];
        for (int i = 0; i < kMlpIn; ++i) acc = fmaf(W1[j * kMlpIn + i], L.x[i], acc);
        L.h1[j] = acc > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    if (j < kMlpH) {
        float acc = b2[j];
        for (int i = 0; i < kMlpH; ++i) acc = fmaf(W2[j * kMlpH + i], L.h1[i], acc);
        L.h2[j] = acc > 0.0f ? acc : 0.0f;
    }
    __syncthreads();
    if (j < kMlpOut) {
        float acc = b3[j];
        for (int i = 0; i < kMlpH; ++i) acc = fmaf(W3[j * kMlpH + i], L.h2[i], acc);
        L.z[j] = acc;
    }
    __syncthreads();
    if (j == 0) {
        int best = lo;
        for (int c = lo + 1; c < lo + 3; ++c)
            if (L.z[c] > L.z[best]) best = c;
        L.choice = best;
    }
    __syncthreads();
    return L.choice;
}

struct sssp_selector;
const float *selector_device_weights(const sssp_selector *s);
