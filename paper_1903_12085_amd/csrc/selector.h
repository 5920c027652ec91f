// Per-phase selector: features of a solver snapshot and the FP32 forward pass
// evaluated inside the solver by one wavefront. Shared by phased.hip and mlp.hip.
//
// Features: twelve ratios of exact integers, each evaluated in double
// precision in the order written and rounded to float once:
//   x0 = F/n              x1 = S/n                 x2 = D ? Sp/D : 0
//   x3 = min(F/2^22,4)/4  x4 = t inf ? 1 : min((t-a)/Wm, 64)/64
//   x5 = min(max((SD/F - a)/Wm, 0), 256)/256       x6 = min((DG/F)/(m/n), 8)/8
//   x7 = D ? Ip/D : 0     x8 = D ? Op/D : 0        x9 = Fp ? min(F/Fp, 4)/4 : 0
//   x10 = (n-R)/n         x11 = min(a/Wm, 4096)/4096
// with F = |F|, S = settled, R = reached, a = minD, t = OUT-STATIC threshold,
// SD / DG = sum over F of d / out-degree (all at the snapshot), Fp = |F| at
// the previous snapshot, D = queued vertices the last criterion evaluation
// ran over, Sp / Ip / Op = how many of them it settled / pass IN-STATIC /
// pass OUT-STATIC, k = index of the phase (bucket) the choice is for,
// Wm = (sum of weights)/m. Phase 0's choice uses the state {s} with nothing
// evaluated (D = Sp = Ip = Op = Fp = 0); phase k+1's uses phase k's snapshot
// and phase k's own outcome (D = |F_k|, Sp = |S'_k|, Fp = |F_{k-1}|), so it
// is made while S'_k relaxes. For Delta-stepping (bucket starts, delta_mode 1)
// D = |F| at the previous bucket start, Sp = what that bucket settled, and
// x4..x9 are 0. Checkpoint mode (delta_mode 2; a choice after every 16th phase
// of a plain static solve): the snapshot of the checkpoint phase k and its
// outcome as above, Fp = |F| at the previous checkpoint, x5 = floor(log2 n)/32,
// x6 = min(m/n, 64)/64 (the graph's size and mean degree) and x7 = x8 = 0.
// Network: W1[64][12] b1[64] W2[64][64] b2[64] W3[6][64] b3[6]; each neuron is
// its bias followed by fmaf over its inputs in index order; ReLU on the two
// hidden layers. Outputs 0..2 choose the phase criterion (IN-STATIC|OUT-STATIC,
// IN-SIMPLE|OUT-SIMPLE, IN-SIMPLE|OUT-STATIC), outputs 3..5 the bucket width 2^12, 2^14, 2^16;
// the argmax takes the lowest index on ties.
#pragma once

#include "common.h"

constexpr int kMlpIn = 12, kMlpH = 64, kMlpOut = 6;
constexpr int kMlpParams = kMlpH * kMlpIn + kMlpH + kMlpH * kMlpH + kMlpH + kMlpOut * kMlpH + kMlpOut;

struct FeatIn {
    unsigned long long n, m, F, S, R, a, t, SD, DG, Fp, D, Sp, Ip, Op, k;
    double Wm;
    int delta_mode;
};

__device__ __forceinline__ double fdmin(double x, double y) { return x < y ? x : y; }
__device__ __forceinline__ double fdmax(double x, double y) { return x > y ? x : y; }

__device__ __forceinline__ void features_dev(const FeatIn &q, float *x) {
#pragma clang fp contract(off)
    const double n = (double)q.n, m = (double)q.m, F = (double)q.F, Fp = (double)q.Fp, D = (double)q.D;
    x[0] = (float)(F / n);
    x[1] = (float)((double)q.S / n);
    x[2] = (float)(q.D ? (double)q.Sp / D : 0.0);
    x[3] = (float)(fdmin(F / 4194304.0, 4.0) / 4.0);
    x[10] = (float)((n - (double)q.R) / n);
    x[11] = (float)(fdmin((double)q.a / q.Wm, 4096.0) / 4096.0);
    if (q.delta_mode == 1) {
        for (int i = 4; i < 10; ++i) x[i] = 0.0f;
        return;
    }
    x[4] = (float)(q.t == INF64 ? 1.0 : fdmin((double)(q.t - q.a) / q.Wm, 64.0) / 64.0);
    x[5] = (float)(fdmin(fdmax(((double)q.SD / F - (double)q.a) / q.Wm, 0.0), 256.0) / 256.0);
    x[6] = (float)(fdmin(((double)q.DG / F) / (m / n), 8.0) / 8.0);
    x[7] = (float)(q.D ? (double)q.Ip / D : 0.0);
    x[8] = (float)(q.D ? (double)q.Op / D : 0.0);
    x[9] = (float)(q.Fp ? fdmin(F / Fp, 4.0) / 4.0 : 0.0);
    if (q.delta_mode == 2) {  // checkpoint mode: the plain kernels fold no SD, DG, Ip, Op
        x[5] = (float)((double)(63 - __clzll(q.n)) / 32.0);
        x[6] = (float)(fdmin(m / n, 64.0) / 64.0);
        x[7] = x[8] = 0.0f;
    }
}

// One wavefront evaluates the network. Lane j loads row j of W1 and W2 and
// row min(j,5) of W3 with 16-byte loads, all issued before any arithmetic,
// and hidden activations reach every lane through readlane, so there is no
// LDS traffic and no barrier. x must be the same in every lane. Returns the
// argmax of outputs [lo, lo+3) in every lane.
constexpr int kOffB1 = kMlpH * kMlpIn, kOffW2 = kOffB1 + kMlpH, kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH, kOffB3 = kOffW3 + kMlpOut * kMlpH;
static_assert(kOffW2 % 4 == 0 && kOffW3 % 4 == 0 && kMlpIn % 4 == 0, "16-byte aligned weight rows");

__device__ __forceinline__ float bcast(float v, int lane) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

struct MlpRegs {
    float4 w1[kMlpIn / 4], w2[kMlpH / 4], w3[kMlpH / 4];
    float c1, c2, c3;
};

// Issues every weight load of this lane (no waits): call it before other
// loads so that all of them are in flight together.
__device__ __forceinline__ void mlp_load(const float *__restrict__ w, MlpRegs &R) {
    const int j = threadIdx.x & 63;
    const int o = j < kMlpOut ? j : kMlpOut - 1;
    const float4 *r1 = reinterpret_cast<const float4 *>(w + j * kMlpIn);
    const float4 *r2 = reinterpret_cast<const float4 *>(w + kOffW2 + j * kMlpH);
    const float4 *r3 = reinterpret_cast<const float4 *>(w + kOffW3 + o * kMlpH);
#pragma unroll
    for (int i = 0; i < kMlpIn / 4; ++i) R.w1[i] = r1[i];
#pragma unroll
    for (int i = 0; i < kMlpH / 4; ++i) R.w2[i] = r2[i];
#pragma unroll
    for (int i = 0; i < kMlpH / 4; ++i) R.w3[i] = r3[i];
    R.c1 = w[kOffB1 + j];
    R.c2 = w[kOffB2 + j];
    R.c3 = w[kOffB3 + o];
}

__device__ __forceinline__ int mlp_eval(const MlpRegs &R, const float *x, int lo) {
    float acc = R.c1;
#pragma unroll
    for (int i = 0; i < kMlpIn / 4; ++i) {
        acc = fmaf(R.w1[i].x, x[4 * i], acc);
        acc = fmaf(R.w1[i].y, x[4 * i + 1], acc);
        acc = fmaf(R.w1[i].z, x[4 * i + 2], acc);
        acc = fmaf(R.w1[i].w, x[4 * i + 3], acc);
    }
    const float h1 = acc > 0.0f ? acc : 0.0f;
    acc = R.c2;
#pragma unroll
    for (int i = 0; i < kMlpH / 4; ++i) {
        acc = fmaf(R.w2[i].x, bcast(h1, 4 * i), acc);
        acc = fmaf(R.w2[i].y, bcast(h1, 4 * i + 1), acc);
        acc = fmaf(R.w2[i].z, bcast(h1, 4 * i + 2), acc);
        acc = fmaf(R.w2[i].w, bcast(h1, 4 * i + 3), acc);
    }
    const float h2 = acc > 0.0f ? acc : 0.0f;
    acc = R.c3;  // lane o < 6: output o
#pragma unroll
    for (int i = 0; i < kMlpH / 4; ++i) {
        acc = fmaf(R.w3[i].x, bcast(h2, 4 * i), acc);
        acc = fmaf(R.w3[i].y, bcast(h2, 4 * i + 1), acc);
        acc = fmaf(R.w3[i].z, bcast(h2, 4 * i + 2), acc);
        acc = fmaf(R.w3[i].w, bcast(h2, 4 * i + 3), acc);
    }
    float z[kMlpOut];
#pragma unroll
    for (int c = 0; c < kMlpOut; ++c) z[c] = bcast(acc, c);
    int best = lo;
    for (int c = lo + 1; c < lo + 3; ++c)
        if (z[c] > z[best]) best = c;
    return best;
}

struct sssp_selector;
const float *selector_device_weights(const sssp_selector *s);
