// Autotuners: time candidate launch shapes with HIP events on the graph's
// stream and keep the fastest. Results never depend on the shape, only time.
#include <algorithm>
#include <vector>

#include "common.h"
#include "graph.h"

static int device_cus() {
    int dev = 0, cus = 256;
    hipDeviceProp_t p;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
    return cus > 0 ? cus : 256;
}

// Median of `reps` timed calls of fn (after one untimed call).
template <class F>
static int time_call(hipStream_t s, int reps, F fn, float *ms_out) {
    hipEvent_t e0, e1;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    int rc = fn();
    std::vector<float> t;
    for (int r = 0; rc == SSSP_OK && r < reps; ++r) {
        float ms = 0;
        if (hipEventRecord(e0, s) != hipSuccess) { rc = sssp_set_error(SSSP_ERR_DEVICE, "event record"); break; }
        rc = fn();
        if (rc) break;
        if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            rc = sssp_set_error(SSSP_ERR_DEVICE, "event timing");
            break;
        }
        t.push_back(ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc == SSSP_OK) {
        std::sort(t.begin(), t.end());
        *ms_out = t[t.size() / 2];
    }
    return rc;
}

extern "C" int sssp_autotune(sssp_graph *g, uint32_t source, uint32_t criterion, sssp_launch_cfg *best,
                             float *best_ms) {
    if (!g) return sssp_set_error(SSSP_ERR_INVALID, "graph is NULL");
    if (source >= g->n) return sssp_set_error(SSSP_ERR_INVALID, "source %u >= n", source);
    uint64_t *dist = nullptr;
    HIP_OK(hipMalloc(&dist, (uint64_t)g->n * sizeof(uint64_t)));
    const int cus = device_cus();
    const uint64_t quads = ((uint64_t)g->n + 3) / 4;
    int in = IN_NONE, out = OUT_NONE;
    crit_modes(criterion, &in, &out);
    const uint32_t queue_max = static_modes(in, out) ? 2u : 1u;  // 2 = keyed, static criteria only
    std::vector<sssp_launch_cfg> cands;
    for (int sb_mul : {1, 2, 4, 8})
        for (int rb_mul : {2, 4, 8})
            for (uint32_t ch : {256u, 512u})
                for (uint32_t ug : {0u, 1u})
                    for (uint32_t qu = 0; qu <= queue_max; ++qu) {
                        uint64_t sb = (uint64_t)cus * sb_mul;
                        const uint64_t need = (quads + kBlock - 1) / kBlock;
                        if (sb > need) sb = need ? need : 1;
                        uint64_t rb = (uint64_t)cus * rb_mul;
                        const uint64_t rneed = (g->m + ch - 1) / ch;
                        if (rb > rneed) rb = rneed ? rneed : 1;
                        sssp_launch_cfg c = {(uint32_t)sb, (uint32_t)rb, ch, ug, qu, 0};
                        bool dup = false;
                        for (auto &o : cands) dup |= o.scan_blocks == c.scan_blocks && o.relax_blocks == c.relax_blocks &&
                                                    o.chunk == c.chunk && o.use_graph == c.use_graph && o.queue == c.queue;
                        if (!dup) cands.push_back(c);
                    }
    sssp_launch_cfg keep;
    sssp_get_launch(g, &keep);
    sssp_launch_cfg win = keep;
    float win_ms = 1e30f;
    int rc = SSSP_OK;
    if (static_modes(in, out)) {
        // one workgroup for the whole solve: a candidate only when phases settle few vertices
        // on average (a workgroup would take too long over a large F)
        sssp_launch_cfg c = keep;
        c.single = 0;
        sssp_stats st{};
        rc = sssp_set_launch(g, &c);
        if (rc == SSSP_OK) rc = sssp_solve_ex(g, source, criterion, dist, &st, nullptr, nullptr, 0);
        if (rc) { sssp_free(dist); sssp_set_launch(g, &keep); return rc; }
        if (st.phases && st.n_reach <= 4096ull * st.phases) {
            c.single = 1;
            cands.push_back(c);
        }
    }
    for (const auto &c : cands) {
        rc = sssp_set_launch(g, &c);
        if (rc) break;
        float ms = 0;
        rc = time_call(g->stream, 3, [&] { return sssp_solve(g, source, criterion, dist, nullptr); }, &ms);
        if (rc) break;
        if (ms < win_ms) { win_ms = ms; win = c; }
    }
    sssp_free(dist);
    if (rc) { sssp_set_launch(g, &keep); return rc; }
    sssp_set_launch(g, &win);
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return SSSP_OK;
}

extern "C" int sssp_autotune_batch(sssp_graph *const *graphs, const uint32_t *sources, uint32_t nq,
                                   uint32_t criterion, uint64_t *const *dist_outs, sssp_batch_cfg *best,
                                   float *best_ms) {
    if (nq == 0 || !graphs || !graphs[0]) return sssp_set_error(SSSP_ERR_INVALID, "empty batch");
    const int cus = device_cus();
    sssp_batch_cfg win = {0, 0, 0, 0, 0};
    float win_ms = 1e30f;
    for (uint32_t bs : {256u, 512u, 1024u})
        for (uint32_t split : {16u, 64u, 256u})
            for (uint32_t per_cu : {1u, 2u, 4u})
                for (uint32_t team_edges : {UINT32_MAX, 1u << 20, 1u << 22})
                    for (uint32_t team_size : {0u, 2u}) {  // automatic, or pairs (large teams lose under load)
                        if (bs == 1024 && per_cu > 2) continue;
                        if (team_edges == UINT32_MAX && team_size) continue;
                        sssp_batch_cfg c = {bs, split, (uint32_t)cus * per_cu, team_edges, team_size};
                        float ms = 0;
                        int rc = time_call(graphs[0]->stream, 2, [&] {
                            return sssp_solve_batch_ex(graphs, sources, nq, criterion, dist_outs, nullptr, &c);
                        }, &ms);
                        if (rc) return rc;
                        if (ms < win_ms) { win_ms = ms; win = c; }
                    }
    sssp_batch_set_config(&win);
    if (best) *best = win;
    if (best_ms) *best_ms = win_ms;
    return SSSP_OK;
}

// Throughput of returning 64-bit atomicMin (the relax kernel's update): every
// thread issues `iters` atomics on slots drawn from its own xorshift sequence
// (slots is a power of two; slots = 1 is one contended address). Eight per
// thread are in flight at a time; the returned values are summed so the
// atomics stay returning.
__global__ __launch_bounds__(256) void k_atomic_min_bench(unsigned long long *buf, uint64_t mask, uint32_t iters) {
    uint64_t x = 0x9E3779B97F4A7C15ull * ((uint64_t)blockIdx.x * 256u + threadIdx.x + 1u);
    unsigned long long acc = 0;
#pragma unroll 8
    for (uint32_t i = 0; i < iters; ++i) {
        x ^= x << 13;
        x ^= x >> 7;
        x ^= x << 17;
        acc += atomicMin(&buf[(x >> 11) & mask], x >> 1);
    }
    if (acc == 0x5A5A5A5A5A5A5A5Aull) buf[0] = acc;  // practically never: keeps the sum live
}

extern "C" int sssp_measure_atomic_min(uint64_t *buf, uint64_t slots, uint32_t blocks, uint32_t iters,
                                       void *hip_stream, float *ms_out) {
    if (!buf || !ms_out) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    if (slots == 0 || (slots & (slots - 1)) != 0) return sssp_set_error(SSSP_ERR_INVALID, "slots must be a power of two");
    if (blocks == 0 || blocks > (1u << 20) || iters == 0 || iters > (1u << 16))
        return sssp_set_error(SSSP_ERR_INVALID, "blocks in [1, 2^20] and iters in [1, 2^16]");
    hipStream_t s = (hipStream_t)hip_stream;
    return time_call(s, 3, [&] {
        hipLaunchKernelGGL(k_atomic_min_bench, dim3(blocks), dim3(256), 0, s, (unsigned long long *)buf, slots - 1,
                           iters);
        HIP_OK(hipGetLastError());
        return (int)SSSP_OK;
    }, ms_out);
}
