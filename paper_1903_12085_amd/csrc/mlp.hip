// Per-phase selector network: 12 -> 64 (ReLU) -> 64 (ReLU) -> 6, FP32.
//
// Training kernels (deterministic: every sum runs in a fixed order in one
// thread, no atomics): dense layer forward, softmax cross-entropy, weight and
// input gradients of a dense layer, Adam. The in-solver forward pass
// (mlp_eval, selector.h) uses the same sequential fmaf order as the
// batch forward here, so a decision depends only on the weights and the
// features.
#include <algorithm>
#include <string.h>
#include <vector>

#include "common.h"
#include "graph.h"
#include "selector.h"

struct sssp_selector {
    float *w = nullptr;     // device, kMlpParams
    float *m = nullptr;     // Adam first moment
    float *v = nullptr;     // Adam second moment
    uint64_t steps = 0;
    int device = 0;
};

// out[r][j] = act(b[j] + sum_i in[r][i] * W[j][i]), i in order (fmaf chain).
__global__ void k_dense_fwd(const float *__restrict__ in, int nin, const float *__restrict__ W,
                            const float *__restrict__ b, int nout, int rows, int relu, float *__restrict__ pre,
                            float *__restrict__ out) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * nout) return;
    const int r = t / nout, j = t % nout;
    float acc = b[j];
    for (int i = 0; i < nin; ++i) acc = fmaf(W[j * nin + i], in[r * nin + i], acc);
    if (pre) pre[t] = acc;
    out[t] = relu ? (acc > 0.0f ? acc : 0.0f) : acc;
}

// Softmax cross-entropy per row; dz = (softmax - onehot) / rows; loss[r] per row.
__global__ void k_softmax_ce(const float *__restrict__ z, const int *__restrict__ y, int rows,
                             float *__restrict__ dz, float *__restrict__ loss) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float mx = z[r * kMlpOut];
    for (int j = 1; j < kMlpOut; ++j) mx = fmaxf(mx, z[r * kMlpOut + j]);
    float e[kMlpOut], s = 0.0f;
    for (int j = 0; j < kMlpOut; ++j) {
        e[j] = expf(z[r * kMlpOut + j] - mx);
        s += e[j];
    }
    const int yr = y[r];
    for (int j = 0; j < kMlpOut; ++j) dz[r * kMlpOut + j] = (e[j] / s - (j == yr ? 1.0f : 0.0f)) / (float)rows;
    loss[r] = logf(s) - (z[r * kMlpOut + yr] - mx);
}

// dW[j][i] = sum_r da[r][j] * in[r][i]; db[j] = sum_r da[r][j] (threads j*nin+i, and j for db).
__global__ void k_dense_bwd_w(const float *__restrict__ da, const float *__restrict__ in, int rows, int nin,
                              int nout, float *__restrict__ dW, float *__restrict__ db) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nout * nin) {
        const int j = t / nin, i = t % nin;
        float acc = 0.0f;
        for (int r = 0; r < rows; ++r) acc = fmaf(da[r * nout + j], in[r * nin + i], acc);
        dW[t] = acc;
    } else if (t < nout * nin + nout) {
        const int j = t - nout * nin;
        float acc = 0.0f;
        for (int r = 0; r < rows; ++r) acc += da[r * nout + j];
        db[j] = acc;
    }
}

// dprev[r][i] = (sum_j da[r][j] * W[j][i]) * (pre_prev[r][i] > 0).
__global__ void k_dense_bwd_x(const float *__restrict__ da, const float *__restrict__ W, const float *__restrict__ pre_prev,
                              int rows, int nin, int nout, float *__restrict__ dprev) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * nin) return;
    const int r = t / nin, i = t % nin;
    float acc = 0.0f;
    for (int j = 0; j < nout; ++j) acc = fmaf(da[r * nout + j], W[j * nin + i], acc);
    dprev[t] = pre_prev[t] > 0.0f ? acc : 0.0f;
}

__global__ void k_adam(float *__restrict__ w, float *__restrict__ m, float *__restrict__ v, const float *__restrict__ g,
                       int n, float lr, float bc1, float bc2) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = 0.9f * m[i] + 0.1f * gi;
    const float vi = 0.999f * v[i] + 0.001f * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + 1e-8f);
}

__global__ void k_gather_rows(const float *__restrict__ X, const int *__restrict__ Y, const uint32_t *__restrict__ idx,
                              int rows, float *__restrict__ Xb, int *__restrict__ Yb) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= rows * kMlpIn) return;
    const int r = t / kMlpIn, i = t % kMlpIn;
    Xb[t] = X[(uint64_t)idx[r] * kMlpIn + i];
    if (i == 0) Yb[r] = Y[idx[r]];
}

static inline int nb(int items) { return (items + 255) / 256; }

// Work buffers for a batch of up to `cap` rows.
struct MlpWork {
    float *a1 = nullptr, *h1 = nullptr, *a2 = nullptr, *h2 = nullptr, *z = nullptr;
    float *dz = nullptr, *d2 = nullptr, *d1 = nullptr, *loss = nullptr, *grad = nullptr;
    int cap = 0;
    int alloc(int rows) {
        cap = rows;
        HIP_OK(hipMalloc(&a1, rows * kMlpH * 4)); HIP_OK(hipMalloc(&h1, rows * kMlpH * 4));
        HIP_OK(hipMalloc(&a2, rows * kMlpH * 4)); HIP_OK(hipMalloc(&h2, rows * kMlpH * 4));
        HIP_OK(hipMalloc(&z, rows * kMlpOut * 4)); HIP_OK(hipMalloc(&dz, rows * kMlpOut * 4));
        HIP_OK(hipMalloc(&d2, rows * kMlpH * 4)); HIP_OK(hipMalloc(&d1, rows * kMlpH * 4));
        HIP_OK(hipMalloc(&loss, rows * 4)); HIP_OK(hipMalloc(&grad, kMlpParams * 4));
        return SSSP_OK;
    }
    ~MlpWork() {
        sssp_free(a1); sssp_free(h1); sssp_free(a2); sssp_free(h2); sssp_free(z);
        sssp_free(dz); sssp_free(d2); sssp_free(d1); sssp_free(loss); sssp_free(grad);
    }
};

static void forward(const float *w, const float *X, int rows, MlpWork &k, hipStream_t s) {
    const float *W1 = w, *b1 = W1 + kMlpH * kMlpIn, *W2 = b1 + kMlpH, *b2 = W2 + kMlpH * kMlpH;
    const float *W3 = b2 + kMlpH, *b3 = W3 + kMlpOut * kMlpH;
    hipLaunchKernelGGL(k_dense_fwd, dim3(nb(rows * kMlpH)), dim3(256), 0, s, X, kMlpIn, W1, b1, kMlpH, rows, 1, k.a1, k.h1);
    hipLaunchKernelGGL(k_dense_fwd, dim3(nb(rows * kMlpH)), dim3(256), 0, s, k.h1, kMlpH, W2, b2, kMlpH, rows, 1, k.a2, k.h2);
    hipLaunchKernelGGL(k_dense_fwd, dim3(nb(rows * kMlpOut)), dim3(256), 0, s, k.h2, kMlpH, W3, b3, kMlpOut, rows, 0,
                       (float *)nullptr, k.z);
}

// Loss per row in k.loss and the mean-loss gradient (flat layout) in k.grad.
static void backward(const float *w, const float *X, const int *Y, int rows, MlpWork &k, hipStream_t s) {
    const float *W2 = w + kMlpH * kMlpIn + kMlpH, *W3 = W2 + kMlpH * kMlpH + kMlpH;
    float *gW1 = k.grad, *gb1 = gW1 + kMlpH * kMlpIn, *gW2 = gb1 + kMlpH, *gb2 = gW2 + kMlpH * kMlpH;
    float *gW3 = gb2 + kMlpH, *gb3 = gW3 + kMlpOut * kMlpH;
    hipLaunchKernelGGL(k_softmax_ce, dim3(nb(rows)), dim3(256), 0, s, k.z, Y, rows, k.dz, k.loss);
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb(kMlpOut * kMlpH + kMlpOut)), dim3(256), 0, s, k.dz, k.h2, rows, kMlpH, kMlpOut, gW3, gb3);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(nb(rows * kMlpH)), dim3(256), 0, s, k.dz, W3, k.a2, rows, kMlpH, kMlpOut, k.d2);
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb(kMlpH * kMlpH + kMlpH)), dim3(256), 0, s, k.d2, k.h1, rows, kMlpH, kMlpH, gW2, gb2);
    hipLaunchKernelGGL(k_dense_bwd_x, dim3(nb(rows * kMlpH)), dim3(256), 0, s, k.d2, W2, k.a1, rows, kMlpH, kMlpH, k.d1);
    hipLaunchKernelGGL(k_dense_bwd_w, dim3(nb(kMlpH * kMlpIn + kMlpH)), dim3(256), 0, s, k.d1, X, rows, kMlpIn, kMlpH, gW1, gb1);
}

extern "C" int sssp_selector_create(const float *weights, sssp_selector **out) {
    if (!out) return sssp_set_error(SSSP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    sssp_selector *s = new (std::nothrow) sssp_selector();
    if (!s) return sssp_set_error(SSSP_ERR_OOM, "host allocation failed");
    if (hipGetDevice(&s->device) != hipSuccess || hipMalloc(&s->w, kMlpParams * 4) != hipSuccess ||
        hipMalloc(&s->m, kMlpParams * 4) != hipSuccess || hipMalloc(&s->v, kMlpParams * 4) != hipSuccess) {
        sssp_selector_destroy(s);
        return sssp_set_error(SSSP_ERR_OOM, "selector allocation failed");
    }
    hipError_t e = weights ? hipMemcpy(s->w, weights, kMlpParams * 4, hipMemcpyHostToDevice)
                           : hipMemset(s->w, 0, kMlpParams * 4);
    if (e == hipSuccess) e = hipMemset(s->m, 0, kMlpParams * 4);
    if (e == hipSuccess) e = hipMemset(s->v, 0, kMlpParams * 4);
    if (e != hipSuccess) {
        sssp_selector_destroy(s);
        return sssp_set_error(SSSP_ERR_DEVICE, "selector init: %s", hipGetErrorString(e));
    }
    *out = s;
    return SSSP_OK;
}

extern "C" int sssp_selector_destroy(sssp_selector *s) {
    if (!s) return SSSP_OK;
    sssp_free(s->w); sssp_free(s->m); sssp_free(s->v);
    delete s;
    return SSSP_OK;
}

extern "C" int sssp_selector_get_weights(const sssp_selector *s, float *host_out) {
    if (!s || !host_out) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    HIP_OK(hipMemcpy(host_out, s->w, kMlpParams * 4, hipMemcpyDeviceToHost));
    return SSSP_OK;
}

extern "C" int sssp_selector_set_weights(sssp_selector *s, const float *host_in) {
    if (!s || !host_in) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    HIP_OK(hipMemcpy(s->w, host_in, kMlpParams * 4, hipMemcpyHostToDevice));
    HIP_OK(hipMemset(s->m, 0, kMlpParams * 4));
    HIP_OK(hipMemset(s->v, 0, kMlpParams * 4));
    s->steps = 0;
    return SSSP_OK;
}

const float *selector_device_weights(const sssp_selector *s) { return s ? s->w : nullptr; }

static int upload_xy(const float *x, const int32_t *y, uint32_t n, float **dx, int **dy) {
    HIP_OK(hipMalloc(dx, (uint64_t)n * kMlpIn * 4));
    HIP_OK(hipMemcpy(*dx, x, (uint64_t)n * kMlpIn * 4, hipMemcpyHostToDevice));
    if (y) {
        for (uint32_t i = 0; i < n; ++i)
            if (y[i] < 0 || y[i] >= kMlpOut) return sssp_set_error(SSSP_ERR_INVALID, "label %d out of range", y[i]);
        HIP_OK(hipMalloc(dy, (uint64_t)n * 4));
        HIP_OK(hipMemcpy(*dy, y, (uint64_t)n * 4, hipMemcpyHostToDevice));
    }
    return SSSP_OK;
}

extern "C" int sssp_selector_forward(const sssp_selector *s, const float *x, uint32_t n, float *logits_out) {
    if (!s || !x || !logits_out || n == 0 || n > (1u << 24)) return sssp_set_error(SSSP_ERR_INVALID, "bad argument");
    float *dx = nullptr;
    int *dy = nullptr;
    int rc = upload_xy(x, nullptr, n, &dx, &dy);
    MlpWork k;
    if (!rc) rc = k.alloc((int)n);
    if (!rc) {
        forward(s->w, dx, (int)n, k, nullptr);
        if (hipMemcpy(logits_out, k.z, (uint64_t)n * kMlpOut * 4, hipMemcpyDeviceToHost) != hipSuccess)
            rc = sssp_set_error(SSSP_ERR_DEVICE, "logits copy");
    }
    sssp_free(dx);
    return rc;
}

extern "C" int sssp_selector_grad(const sssp_selector *s, const float *x, const int32_t *y, uint32_t n,
                                  float *loss_out, float *grad_out) {
    if (!s || !x || !y || n == 0 || n > (1u << 24)) return sssp_set_error(SSSP_ERR_INVALID, "bad argument");
    float *dx = nullptr;
    int *dy = nullptr;
    int rc = upload_xy(x, y, n, &dx, &dy);
    MlpWork k;
    if (!rc) rc = k.alloc((int)n);
    if (!rc) {
        forward(s->w, dx, (int)n, k, nullptr);
        backward(s->w, dx, dy, (int)n, k, nullptr);
        std::vector<float> l(n);
        if (hipMemcpy(l.data(), k.loss, (uint64_t)n * 4, hipMemcpyDeviceToHost) != hipSuccess ||
            (grad_out && hipMemcpy(grad_out, k.grad, kMlpParams * 4, hipMemcpyDeviceToHost) != hipSuccess)) {
            rc = sssp_set_error(SSSP_ERR_DEVICE, "gradient copy");
        } else if (loss_out) {
            double t = 0;
            for (float v : l) t += v;
            *loss_out = (float)(t / n);
        }
    }
    sssp_free(dx);
    sssp_free(dy);
    return rc;
}

// SplitMix64 step for the shuffle (host side).
static uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

extern "C" int sssp_selector_train(sssp_selector *s, const float *x, const int32_t *y, uint32_t n, uint32_t epochs,
                                   uint32_t batch, float lr, uint64_t seed, float *final_loss) {
    if (!s || !x || !y || n == 0 || batch == 0 || n > (1u << 24) || batch > 65536 || !(lr > 0.0f))
        return sssp_set_error(SSSP_ERR_INVALID, "bad argument");
    float *dx = nullptr, *xb = nullptr;
    int *dy = nullptr, *yb = nullptr;
    uint32_t *didx = nullptr;
    int rc = upload_xy(x, y, n, &dx, &dy);
    MlpWork k;
    const uint32_t B = batch < n ? batch : n;
    if (!rc) rc = k.alloc((int)B);
    if (!rc && (hipMalloc(&xb, (uint64_t)B * kMlpIn * 4) != hipSuccess || hipMalloc(&yb, B * 4) != hipSuccess ||
                hipMalloc(&didx, (uint64_t)n * 4) != hipSuccess))
        rc = sssp_set_error(SSSP_ERR_OOM, "training buffers");
    std::vector<uint32_t> perm(n);
    double last = 0;
    for (uint32_t ep = 0; !rc && ep < epochs; ++ep) {
        for (uint32_t i = 0; i < n; ++i) perm[i] = i;
        for (uint32_t i = n - 1; i > 0; --i) {  // Fisher-Yates from a counter-based stream
            const uint64_t r = mix64(seed * 0x9E3779B97F4A7C15ULL + ((uint64_t)ep << 32) + i);
            std::swap(perm[i], perm[(uint32_t)(r % (i + 1))]);
        }
        if (hipMemcpy(didx, perm.data(), (uint64_t)n * 4, hipMemcpyHostToDevice) != hipSuccess) {
            rc = sssp_set_error(SSSP_ERR_DEVICE, "index upload");
            break;
        }
        double tot = 0;
        for (uint32_t b0 = 0; b0 + B <= n; b0 += B) {  // full batches only
            hipLaunchKernelGGL(k_gather_rows, dim3(nb(B * kMlpIn)), dim3(256), 0, 0, dx, dy, didx + b0, (int)B, xb, yb);
            forward(s->w, xb, (int)B, k, nullptr);
            backward(s->w, xb, yb, (int)B, k, nullptr);
            s->steps++;
            const float bc1 = 1.0f - powf(0.9f, (float)s->steps), bc2 = 1.0f - powf(0.999f, (float)s->steps);
            hipLaunchKernelGGL(k_adam, dim3(nb(kMlpParams)), dim3(256), 0, 0, s->w, s->m, s->v, k.grad, kMlpParams, lr,
                               bc1, bc2);
            if (b0 + 2 * B > n) {  // last batch of the epoch: its mean loss
                std::vector<float> l(B);
                if (hipMemcpy(l.data(), k.loss, B * 4, hipMemcpyDeviceToHost) != hipSuccess) {
                    rc = sssp_set_error(SSSP_ERR_DEVICE, "loss copy");
                    break;
                }
                tot = 0;
                for (float v : l) tot += v;
                last = tot / B;
            }
        }
    }
    if (!rc && hipDeviceSynchronize() != hipSuccess) rc = sssp_set_error(SSSP_ERR_DEVICE, "training failed");
    if (!rc && final_loss) *final_loss = (float)last;
    sssp_free(dx); sssp_free(dy); sssp_free(xb); sssp_free(yb); sssp_free(didx);
    return rc;
}
