// Device graph: CSR upload and validation, static minima
// (equations crit:instatic / crit:outstatic need min in- and out-edge weight
// per vertex, computed once in O(m), Section 3; the implementation section
// computes the minimum in-edge weight with an atomic minimum per edge), and
// the per-row weight sort and the reverse adjacency (CSC), both built lazily
// for the dynamic criteria.
#include <chrono>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <rocprim/rocprim.hpp>

#include "common.h"
#include "graph.h"

// ---------------------------------------------------------------------------
// error reporting

static thread_local char g_err[512] = "";

int sssp_set_error(int code, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
    return code;
}

extern "C" const char *sssp_last_error(void) { return g_err; }

// ---------------------------------------------------------------------------
// kernels

// Checks row_ptr[0] == 0, monotone rows, row_ptr[n] == m and col < n.
__global__ void k_validate(uint32_t n, uint64_t m, const uint64_t *__restrict__ rp,
                           const uint32_t *__restrict__ col, unsigned int *__restrict__ bad) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t v = t0; v < n; v += stride)
        if (rp[v + 1] < rp[v]) atomicOr(bad, 1u);
    if (t0 == 0 && (rp[0] != 0 || rp[n] != m)) atomicOr(bad, 2u);
    for (uint64_t e = t0; e < m; e += stride)
        if (col[e] >= n) atomicOr(bad, 4u);
}

__global__ void k_rp32(uint32_t n, const uint64_t *__restrict__ rp64, uint32_t *__restrict__ rp) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n;
         v += (uint64_t)gridDim.x * blockDim.x)
        rp[v] = (uint32_t)rp64[v];
}

// key = (target << 32) | weight for the reverse adjacency; payload = source.
__global__ void k_col_keys(uint64_t m, const uint2 *__restrict__ edges, const uint32_t *__restrict__ rp,
                           uint32_t n, unsigned long long *__restrict__ key, uint32_t *__restrict__ src) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo + 1) / 2;
            if (rp[mid] <= e) lo = mid; else hi = mid - 1;
        }
        uint2 ed = edges[e];
        key[e] = ((unsigned long long)ed.x << 32) | ed.y;
        src[e] = lo;
    }
}

__global__ void k_pack_edges(uint64_t m, const unsigned long long *__restrict__ key,
                             const uint32_t *__restrict__ val, uint2 *__restrict__ out) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x)
        out[e] = make_uint2(val[e], (uint32_t)(key[e] & 0xFFFFFFFFull));
}

// minOut = the lightest edge of each row (rows in input order); minIn reset to INF.
// A wavefront takes 64 consecutive rows, whose edges are contiguous: it reads
// them 64 at a time (coalesced), finds each edge's row among the 64 by a
// binary search over the row starts held one per lane, and folds the weight
// into that row's minimum in LDS.
__global__ __launch_bounds__(256) void k_min_out(uint32_t n, const uint32_t *__restrict__ rp,
                                                 const uint2 *__restrict__ edges, uint2 *__restrict__ vmin) {
    __shared__ uint32_t smin[256];
    const uint32_t lane = threadIdx.x & 63;
    uint32_t *wmin = smin + (threadIdx.x & ~63u);
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t base = (uint64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~63u); base < n; base += stride) {
        const uint64_t v = base + lane;  // base is wavefront-uniform
        const uint32_t rs = v < n ? rp[v] : rp[n];  // this lane's row start (rows past n are empty)
        const uint32_t e0 = (uint32_t)__shfl((int)rs, 0, 64);
        const uint32_t e1 = rp[base + 64 < n ? base + 64 : n];
        wmin[lane] = INF32;
        __builtin_amdgcn_wave_barrier();
        for (uint32_t k = e0 + lane; __ballot(k < e1); k += 64) {  // wavefront-uniform
            const bool in = k < e1;
            const uint32_t w = in ? edges[k].y : INF32;
            int lo = 0;  // last row of the window whose start is <= k (every lane shuffles)
#pragma unroll
            for (int st = 32; st > 0; st >>= 1) {
                const uint32_t r = (uint32_t)__shfl((int)rs, lo + st, 64);
                if (r <= k) lo += st;
            }
            if (in) atomicMin(&wmin[lo], w);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        if (v < n) vmin[v] = make_uint2(INF32, wmin[lane]);
        __builtin_amdgcn_wave_barrier();
    }
}

// The input's edges as (target, weight), rows in input order.
__global__ void k_pack_cw(uint64_t m, const uint32_t *__restrict__ col, const uint32_t *__restrict__ w,
                          uint2 *__restrict__ out) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        out[e] = make_uint2(col[e], w[e]);
}

// key = (row << 32) | weight and payload = target of every edge, for the row
// sort; the row by binary search in row_ptr.
__global__ void k_row_keys_e(uint32_t n, uint64_t m, const uint32_t *__restrict__ rp, const uint2 *__restrict__ edges,
                             unsigned long long *__restrict__ key, uint32_t *__restrict__ val) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo + 1) / 2;
            if (rp[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const uint2 ed = edges[e];
        key[e] = ((unsigned long long)lo << 32) | ed.y;
        val[e] = ed.x;
    }
}

// minIn[v] = min over in-edges (u, v) of c(u, v), by one atomic minimum per edge.
__global__ void k_min_in(uint64_t m, const uint2 *__restrict__ edges, uint2 *__restrict__ vmin) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint2 ed = edges[e];
        uint32_t *slot = &vmin[ed.x].x;
        if (ed.y < *slot) atomicMin(slot, ed.y);
    }
}

// emin[e] = minOut of edge e's target: relax folds the next OUT-STATIC threshold
// from the edge's own row position, with no load that waits for the atomic.
__global__ void k_emin(uint64_t m, const uint2 *__restrict__ edges, const uint2 *__restrict__ vmin,
                       uint32_t *__restrict__ emin) {
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x)
        emin[e] = vmin[edges[e].x].y;
}

// Exact sum of all edge weights (one block-level sum and one atomic per block);
// out[1] counts the edges of weight 2^32 - 1.
__global__ void k_sum_w(uint64_t m, const uint2 *__restrict__ edges, unsigned long long *__restrict__ out) {
    __shared__ unsigned long long sh[4], shx[4];
    unsigned long long t = 0, x = 0;
    for (uint64_t e = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t w = edges[e].y;
        t += w;
        x += w == INF32 ? 1u : 0u;
    }
    for (int o = 32; o > 0; o >>= 1) {
        t += __shfl_xor(t, o, 64);
        x += __shfl_xor(x, o, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = t;
        shx[threadIdx.x >> 6] = x;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicAdd(out, sh[0] + sh[1] + sh[2] + sh[3]);
        const unsigned long long nx = shx[0] + shx[1] + shx[2] + shx[3];
        if (nx) atomicAdd(out + 1, nx);
    }
}

// in_ptr[v] = first index whose sorted key has target >= v.
__global__ void k_in_ptr(uint32_t n, uint64_t m, const unsigned long long *__restrict__ key,
                         uint32_t *__restrict__ ip) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        unsigned long long target = (unsigned long long)v << 32;
        uint64_t lo = 0, hi = m;
        while (lo < hi) {
            uint64_t mid = (lo + hi) / 2;
            if (key[mid] < target) lo = mid + 1; else hi = mid;
        }
        ip[v] = (uint32_t)lo;
    }
}

static inline int grid_for(uint64_t items, int block = 256, int cap = 8192) {
    uint64_t g = (items + block - 1) / block;
    if (g < 1) g = 1;
    if (g > (uint64_t)cap) g = cap;
    return (int)g;
}

static int bits_for(uint32_t n) {
    int b = 1;
    while (b < 32 && (1ull << b) < n) ++b;
    return b;
}

// Sort (key, value) pairs with rocPRIM's device radix sort, in place via a
// second buffer pair; `end_bit` bounds the key width.
static int radix_sort(unsigned long long *&k0, unsigned long long *&k1, uint32_t *&v0, uint32_t *&v1,
                      uint64_t m, int end_bit, hipStream_t s) {
    size_t tmp_bytes = 0;
    if (rocprim::radix_sort_pairs(nullptr, tmp_bytes, k0, k1, v0, v1, (size_t)m, 0, end_bit, s) != hipSuccess)
        return sssp_set_error(SSSP_ERR_DEVICE, "radix_sort_pairs size query failed");
    void *tmp = nullptr;
    HIP_OK(hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 1));
    hipError_t e = rocprim::radix_sort_pairs(tmp, tmp_bytes, k0, k1, v0, v1, (size_t)m, 0, end_bit, s);
    hipError_t e2 = hipStreamSynchronize(s);
    sssp_free(tmp);
    if (e != hipSuccess || e2 != hipSuccess)
        return sssp_set_error(SSSP_ERR_DEVICE, "radix_sort_pairs failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
    unsigned long long *tk = k0; k0 = k1; k1 = tk;  // sorted data now in k0 / v0
    uint32_t *tv = v0; v0 = v1; v1 = tv;
    return SSSP_OK;
}

// ---------------------------------------------------------------------------
// host API

static int create_impl(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                       const uint32_t *weight, int device_ptrs, hipStream_t s, sssp_graph *g) {
    // 1. stage the CSR on the device
    uint64_t *rp64 = nullptr;
    uint32_t *dcol = nullptr, *dw = nullptr;
    unsigned int *bad = nullptr;
    int rc = SSSP_OK;
#define TRY(call) do { hipError_t _e = (call); if (_e != hipSuccess) { \
        rc = sssp_set_error(_e == hipErrorOutOfMemory ? SSSP_ERR_OOM : SSSP_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(_e)); goto done; } } while (0)
    TRY(hipMalloc(&g->rp, (n + 1) * sizeof(uint32_t)));
    TRY(hipMalloc(&g->vmin, (uint64_t)n * sizeof(uint2)));
    TRY(hipMalloc(&g->edges, (m ? m : 1) * sizeof(uint2)));
    TRY(hipMalloc(&g->emin, (m ? m : 1) * sizeof(uint32_t)));
    TRY(hipMalloc(&bad, sizeof(unsigned int)));
    TRY(hipMemsetAsync(bad, 0, sizeof(unsigned int), s));
    if (device_ptrs) {
        rp64 = (uint64_t *)row_ptr;
        dcol = (uint32_t *)col;
        dw = (uint32_t *)weight;
    } else {
        TRY(hipMalloc(&rp64, (n + 1) * sizeof(uint64_t)));
        TRY(hipMemcpyAsync(rp64, row_ptr, (n + 1) * sizeof(uint64_t), hipMemcpyHostToDevice, s));
        if (m) {
            TRY(hipMalloc(&dcol, m * sizeof(uint32_t)));
            TRY(hipMalloc(&dw, m * sizeof(uint32_t)));
            TRY(hipMemcpyAsync(dcol, col, m * sizeof(uint32_t), hipMemcpyHostToDevice, s));
            TRY(hipMemcpyAsync(dw, weight, m * sizeof(uint32_t), hipMemcpyHostToDevice, s));
        }
    }
    {
        hipLaunchKernelGGL(k_validate, dim3(grid_for(m > n ? m : n)), dim3(256), 0, s, n, m, rp64, dcol, bad);
        unsigned int hbad = 0;
        TRY(hipMemcpyAsync(&hbad, bad, sizeof hbad, hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        if (hbad) { rc = sssp_set_error(SSSP_ERR_INVALID, "malformed CSR (code %u)", hbad); goto done; }
    }
    {
        hipEvent_t e0, e1;
        TRY(hipEventCreate(&e0));
        TRY(hipEventCreate(&e1));
        TRY(hipEventRecord(e0, s));
        hipLaunchKernelGGL(k_rp32, dim3(grid_for(n + 1)), dim3(256), 0, s, n, rp64, g->rp);
        // 2. the edges in input order; rows are sorted by weight only when a solve first needs the
        // cursors of the dynamic criteria (graph_ensure_sorted)
        if (m) hipLaunchKernelGGL(k_pack_cw, dim3(grid_for(m)), dim3(256), 0, s, m, dcol, dw, g->edges);
        // 3. static minima
        hipLaunchKernelGGL(k_min_out, dim3(grid_for(n)), dim3(256), 0, s, n, g->rp, g->edges, g->vmin);
        if (m) hipLaunchKernelGGL(k_min_in, dim3(grid_for(m)), dim3(256), 0, s, m, g->edges, g->vmin);
        if (m) hipLaunchKernelGGL(k_emin, dim3(grid_for(m)), dim3(256), 0, s, m, g->edges, g->vmin, g->emin);
        TRY(hipEventRecord(e1, s));
        TRY(hipEventSynchronize(e1));
        if (m) {  // weight sum for the selector's feature scale and the 2^32 - 1 flag (not timed)
            unsigned long long *dsum = nullptr;
            TRY(hipMalloc(&dsum, 2 * sizeof(unsigned long long)));
            TRY(hipMemsetAsync(dsum, 0, 2 * sizeof(unsigned long long), s));
            hipLaunchKernelGGL(k_sum_w, dim3(grid_for(m, 256, 1024)), dim3(256), 0, s, m, g->edges, dsum);
            unsigned long long hs[2] = {0, 0};
            TRY(hipMemcpyAsync(hs, dsum, sizeof hs, hipMemcpyDeviceToHost, s));
            TRY(hipStreamSynchronize(s));
            sssp_free(dsum);
            g->sum_w = hs[0];
            g->wmax = hs[1] != 0;
        }
        float ms = 0;
        TRY(hipEventElapsedTime(&ms, e0, e1));
        g->precompute_ns = (uint64_t)(ms * 1e6);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        TRY(hipGetLastError());
    }
done:
#undef TRY
    if (!device_ptrs) { sssp_free(rp64); sssp_free(dcol); sssp_free(dw); }
    sssp_free(bad);
    return rc;
}

extern "C" int sssp_graph_create(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                                 const uint32_t *weight, int device_ptrs, void *hip_stream,
                                 sssp_graph **out) {
    if (!out) return sssp_set_error(SSSP_ERR_INVALID, "out is NULL");
    *out = nullptr;
    if (n == 0) return sssp_set_error(SSSP_ERR_INVALID, "n must be >= 1");
    if (!row_ptr || (m && (!col || !weight))) return sssp_set_error(SSSP_ERR_INVALID, "NULL CSR array");
    if (n >= (1u << 26) || m >= (1ull << 32))
        return sssp_set_error(SSSP_ERR_UNSUPPORTED, "graph too large (n=%u, m=%llu): need n < 2^26, m < 2^32",
                              n, (unsigned long long)m);
    if (!device_ptrs) {  // host-side validation
        if (row_ptr[0] != 0 || row_ptr[n] != m)
            return sssp_set_error(SSSP_ERR_INVALID, "row_ptr[0] must be 0 and row_ptr[n] must equal m");
        for (uint32_t v = 0; v < n; ++v)
            if (row_ptr[v + 1] < row_ptr[v]) return sssp_set_error(SSSP_ERR_INVALID, "row_ptr not monotone at %u", v);
        for (uint64_t e = 0; e < m; ++e)
            if (col[e] >= n) return sssp_set_error(SSSP_ERR_INVALID, "col[%llu] = %u >= n", (unsigned long long)e, col[e]);
    }
    sssp_graph *g = new (std::nothrow) sssp_graph();
    if (!g) return sssp_set_error(SSSP_ERR_OOM, "host allocation failed");
    g->n = n;
    g->m = m;
    g->stream = (hipStream_t)hip_stream;
    if (hipGetDevice(&g->device) != hipSuccess) { delete g; return sssp_set_error(SSSP_ERR_DEVICE, "no HIP device"); }
    int rc = create_impl(n, m, row_ptr, col, weight, device_ptrs, g->stream, g);
    if (rc != SSSP_OK) { sssp_graph_destroy(g); return rc; }
    graph_default_cfg(g);
    *out = g;
    return SSSP_OK;
}

extern "C" int sssp_graph_destroy(sssp_graph *g) {
    if (!g) return SSSP_OK;
    sssp_free(g->rp); sssp_free(g->edges); sssp_free(g->vmin); sssp_free(g->emin);
    sssp_free(g->ip); sssp_free(g->in_edges);
    sssp_free(g->one_fm);  // the one-workgroup scratch's other buffers go with solve_bufs_free
    solve_bufs_free(g);
    delete g;
    return SSSP_OK;
}

extern "C" int sssp_set_stream(sssp_graph *g, void *hip_stream) {
    if (!g) return sssp_set_error(SSSP_ERR_INVALID, "graph is NULL");
    g->stream = (hipStream_t)hip_stream;
    return SSSP_OK;
}

__global__ void k_split_minima(uint32_t n, const uint2 *__restrict__ vmin, uint32_t *mi, uint32_t *mo) {
    for (uint64_t v = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        uint2 x = vmin[v];
        if (mi) mi[v] = x.x;
        if (mo) mo[v] = x.y;
    }
}

extern "C" int sssp_graph_minima(sssp_graph *g, uint32_t *min_in, uint32_t *min_out) {
    if (!g) return sssp_set_error(SSSP_ERR_INVALID, "graph is NULL");
    hipLaunchKernelGGL(k_split_minima, dim3(grid_for(g->n)), dim3(256), 0, g->stream, g->n, g->vmin, min_in, min_out);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(g->stream));
    return SSSP_OK;
}

// Sorts each row of the CSR by weight, in place (the cursors of the dynamic
// criteria walk rows lightest first); emin follows the edges. Once per graph.
int graph_ensure_sorted(sssp_graph *g) {
    if (g->rows_sorted || g->m == 0) {
        g->rows_sorted = true;
        return SSSP_OK;
    }
    const uint64_t m = g->m;
    hipStream_t s = g->stream;
    unsigned long long *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    int rc = SSSP_OK;
#define TRY(call) do { hipError_t _e = (call); if (_e != hipSuccess) { \
        rc = sssp_set_error(_e == hipErrorOutOfMemory ? SSSP_ERR_OOM : SSSP_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(_e)); goto done; } } while (0)
    TRY(hipMalloc(&k0, m * sizeof(unsigned long long)));
    TRY(hipMalloc(&k1, m * sizeof(unsigned long long)));
    TRY(hipMalloc(&v0, m * sizeof(uint32_t)));
    TRY(hipMalloc(&v1, m * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_row_keys_e, dim3(grid_for(m)), dim3(256), 0, s, g->n, m, g->rp, g->edges, k0, v0);
    rc = radix_sort(k0, k1, v0, v1, m, 32 + bits_for(g->n), s);
    if (rc != SSSP_OK) goto done;
    hipLaunchKernelGGL(k_pack_edges, dim3(grid_for(m)), dim3(256), 0, s, m, k0, v0, g->edges);
    hipLaunchKernelGGL(k_emin, dim3(grid_for(m)), dim3(256), 0, s, m, g->edges, g->vmin, g->emin);
    TRY(hipGetLastError());
    TRY(hipStreamSynchronize(s));
    g->rows_sorted = true;
done:
#undef TRY
    sssp_free(k0); sssp_free(k1); sssp_free(v0); sssp_free(v1);
    return rc;
}

// Reverse adjacency with rows sorted by weight (for the dynamic IN terms).
int graph_ensure_csc(sssp_graph *g) {
    if (g->ip || g->m == 0) {
        if (!g->ip) {  // edgeless graph: all-zero in_ptr
            HIP_OK(hipMalloc(&g->ip, (g->n + 1) * sizeof(uint32_t)));
            HIP_OK(hipMemsetAsync(g->ip, 0, (g->n + 1) * sizeof(uint32_t), g->stream));
            HIP_OK(hipMalloc(&g->in_edges, sizeof(uint2)));
        }
        return SSSP_OK;
    }
    const uint64_t m = g->m;
    hipStream_t s = g->stream;
    unsigned long long *k0 = nullptr, *k1 = nullptr;
    uint32_t *v0 = nullptr, *v1 = nullptr;
    int rc = SSSP_OK;
    if (hipMalloc(&k0, m * 8) != hipSuccess || hipMalloc(&k1, m * 8) != hipSuccess ||
        hipMalloc(&v0, m * 4) != hipSuccess || hipMalloc(&v1, m * 4) != hipSuccess ||
        hipMalloc(&g->ip, (g->n + 1) * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&g->in_edges, m * sizeof(uint2)) != hipSuccess) {
        rc = sssp_set_error(SSSP_ERR_OOM, "CSC allocation failed");
    } else {
        hipLaunchKernelGGL(k_col_keys, dim3(grid_for(m)), dim3(256), 0, s, m, g->edges, g->rp, g->n, k0, v0);
        rc = radix_sort(k0, k1, v0, v1, m, 32 + bits_for(g->n), s);
        if (rc == SSSP_OK) {
            hipLaunchKernelGGL(k_pack_edges, dim3(grid_for(m)), dim3(256), 0, s, m, k0, v0, g->in_edges);
            hipLaunchKernelGGL(k_in_ptr, dim3(grid_for(g->n + 1)), dim3(256), 0, s, g->n, m, k0, g->ip);
            if (hipStreamSynchronize(s) != hipSuccess) rc = sssp_set_error(SSSP_ERR_DEVICE, "CSC build failed");
        }
    }
    sssp_free(k0); sssp_free(k1); sssp_free(v0); sssp_free(v1);
    if (rc != SSSP_OK) {
        sssp_free(g->ip); sssp_free(g->in_edges);
        g->ip = nullptr; g->in_edges = nullptr;
    }
    return rc;
}
