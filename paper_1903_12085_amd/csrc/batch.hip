// Batched phased SSSP: many (graph, source) queries in one persistent launch.
//
// Each workgroup takes whole queries from a device work queue (largest first)
// and runs the generic phased algorithm of Section 3 for that query with
// workgroup barriers only, so a batch needs no grid synchronisation and no
// launch per phase:
//   identify  over the query's fringe list: a vertex the criterion certifies
//             (phase-start minD / OUT-STATIC threshold) goes to the settled
//             list, the others to the next fringe list and fold next minima
//             (wavefront ballot + one LDS atomic per wavefront).
//   relax     over the settled list: rows up to `split` edges by their own
//             lane, longer rows are queued in LDS and expanded by the whole
//             workgroup (degree split). 64-bit atomicMin on the query's
//             distance array; the atomic that replaces infinity appends the
//             target to the next fringe. Improving candidates fold into next
//             minD / threshold.
// Distances and states written in one phase are read in the next with
// L1-bypassing atomic loads (device-scope atomics update L2, not the CU's L1).
//
// Criteria: DIJK, IN-STATIC, OUT-STATIC and their disjunctions (the static
// criteria need no per-phase term pass).
#include <algorithm>
#include <string.h>
#include <vector>

#include "common.h"
#include "graph.h"

struct BatchQuery {
    const uint32_t *rp;
    const uint2 *edges;
    const uint2 *vmin;
    const uint32_t *emin;  // per edge: minOut of its target
    unsigned long long *dist;
    uint8_t *st;
    uint32_t *fl;      // 3 * n entries: fringe list A, fringe list B, settled list
    uint32_t n;
    uint32_t src;
    uint32_t wmax;     // the graph has an edge of weight 2^32 - 1 (see min_out64)
};

struct BatchCtl {
    unsigned int next;    // work-queue head
    unsigned int error;   // set if a query exceeds its phase bound
};

constexpr uint8_t ST_NEW = 3;  // settled in the current phase, out-edges not yet relaxed
constexpr int kHubCap = 256;

// Values written by other wavefronts of the workgroup in an earlier phase are
// read with L1-bypassing loads (device-scope atomics update L2, not the CU's L1,
// and list buffers are reused every other phase).
__device__ __forceinline__ unsigned long long ld_dist(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint8_t ld_st(const uint8_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Workgroup minima of a and b in one LDS round with one barrier. The caller
// writes sh again only after at least one more barrier (the next phase's),
// so no second barrier is needed to protect it.
template <int BS>
__device__ __forceinline__ void bmin2(unsigned long long &a, unsigned long long &b, unsigned long long *sh) {
    a = wave_min64(a);
    b = wave_min64(b);
    if ((threadIdx.x & 63) == 0) {
        sh[threadIdx.x >> 6] = a;
        sh[BS / 64 + (threadIdx.x >> 6)] = b;
    }
    __syncthreads();
    unsigned long long ra = INF64, rb = INF64;
    for (int i = 0; i < BS / 64; ++i) {
        ra = umin64(ra, sh[i]);
        rb = umin64(rb, sh[BS / 64 + i]);
    }
    a = ra;
    b = rb;
}

// Wavefront-aggregated append of v to a list whose length is the LDS counter
// *cnt: one LDS atomic by the lowest taking lane, which is always active.
__device__ __forceinline__ void wave_append(bool take, uint32_t v, uint32_t *list, uint32_t *cnt) {
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (take) list[base + __popcll(mask & ((1ull << lane) - 1ull))] = v;
}

// Relaxes the edges ed[j] (bit j of have) from a vertex at distance du: the
// state and distance loads of all of them are issued together, then the
// atomics. Returns the mask of edges whose atomic replaced infinity (the
// target was discovered; exactly one atomic can do that).
template <int U, bool OUT>
__device__ __forceinline__ uint32_t relax_edges(const BatchQuery &q, unsigned long long du, const uint2 *ed,
                                                const uint32_t *em, uint32_t have, unsigned long long &cmin,
                                                unsigned long long &ctst) {
    uint8_t sv[U];
    unsigned long long cur[U], cand[U], old[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        sv[j] = ST_S;
        cur[j] = 0;
        if ((have >> j) & 1u) {
            sv[j] = ld_st(&q.st[ed[j].x]);
            cur[j] = ld_dist(&q.dist[ed[j].x]);
        }
    }
    uint32_t issued = 0;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        cand[j] = old[j] = INF64;
        if (sv[j] == ST_S || sv[j] == ST_NEW) continue;
        cand[j] = du + ed[j].y;
        if (cand[j] < cur[j]) {
            old[j] = atomicMin(&q.dist[ed[j].x], cand[j]);
            issued |= 1u << j;
        }
    }
    uint32_t disc = 0;
#pragma unroll
    for (int j = 0; j < U; ++j) {
        if (!((issued >> j) & 1u) || !(cand[j] < old[j])) continue;
        cmin = umin64(cmin, cand[j]);
        if (OUT) ctst = umin64(ctst, sadd64(cand[j], min_out64(em[j], q.wmax, q.rp, ed[j].x)));
        if (old[j] == INF64) {
            q.st[ed[j].x] = ST_F;
            disc |= 1u << j;
        }
    }
    return disc;
}

constexpr int kBatchU = 4;  // fringe entries / edges a lane handles per step

// IN: IN_NONE, IN_DIJK or IN_STATIC_M; OUT: OUT-STATIC on/off.
template <int BS, int IN, bool OUT>
__global__ __launch_bounds__(BS) void k_batch(const BatchQuery *__restrict__ queries, const uint32_t *__restrict__ order,
                                              uint32_t nq, BatchCtl *ctl, uint32_t *__restrict__ phases_out,
                                              uint32_t split) {
    __shared__ unsigned long long sh[2 * (BS / 64)];
    __shared__ uint32_t s_q;
    __shared__ uint32_t hub_v[kHubCap];
    __shared__ unsigned long long hub_du[kHubCap];
    // list counters by phase parity: phase p appends with set p & 1 while the
    // other set, last read at the end of phase p - 1, is cleared for phase p + 1
    __shared__ uint32_t hub_n[2], s_nset[2], s_nnext[2];
    for (;;) {
        if (threadIdx.x == 0) s_q = atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const uint32_t qi = s_q;
        __syncthreads();
        if (qi >= nq) return;
        const BatchQuery q = queries[order[qi]];
        const uint32_t n = q.n;
        for (uint32_t v = threadIdx.x; v < n; v += BS) {
            q.dist[v] = v == q.src ? 0ull : INF64;
            q.st[v] = v == q.src ? ST_F : ST_U;
        }
        if (threadIdx.x == 0) {
            q.fl[0] = q.src;
            for (int k = 0; k < 2; ++k) hub_n[k] = s_nset[k] = s_nnext[k] = 0;
        }
        uint32_t nF = 1, cur = 0, phases = 0;
        unsigned long long minD = 0, T = min_out64(q.vmin[q.src].y, q.wmax, q.rp, q.src);
        __syncthreads();
        while (nF > 0) {
            uint32_t *F = q.fl + (uint64_t)cur * n;
            uint32_t *Fn = q.fl + (uint64_t)(cur ^ 1) * n;
            uint32_t *Sp = q.fl + 2ull * n;
            const int pp = (int)(phases & 1u);
            // identify over the fringe list
            unsigned long long fmin = INF64, ftst = INF64;
            // kBatchU fringe entries per thread and step, their loads issued together
            for (uint32_t base = 0; base < nF; base += BS * kBatchU) {
                uint32_t v[kBatchU];
                unsigned long long dv[kBatchU];
                uint2 mm[kBatchU];
                uint32_t have = 0;
#pragma unroll
                for (int j = 0; j < kBatchU; ++j) {
                    const uint32_t i = base + j * BS + threadIdx.x;
                    v[j] = 0;
                    if (i < nF) {
                        v[j] = ld_u32(&F[i]);
                        have |= 1u << j;
                    }
                }
#pragma unroll
                for (int j = 0; j < kBatchU; ++j) {
                    dv[j] = INF64;
                    mm[j] = make_uint2(INF32, INF32);
                    if ((have >> j) & 1u) {
                        dv[j] = ld_dist(&q.dist[v[j]]);
                        mm[j] = q.vmin[v[j]];
                    }
                }
#pragma unroll
                for (int j = 0; j < kBatchU; ++j) {
                    bool set = false, keep = false;
                    if ((have >> j) & 1u) {
                        bool ok = false;
                        if (IN == IN_DIJK) ok = dv[j] == minD;
                        else if (IN == IN_STATIC_M) ok = dv[j] <= sadd64(minD, min_in_test(mm[j].x));
                        if (OUT) ok = ok || dv[j] <= T;
                        set = ok;
                        keep = !ok;
                        if (keep) {
                            fmin = umin64(fmin, dv[j]);
                            if (OUT) ftst = umin64(ftst, sadd64(dv[j], min_out64(mm[j].y, q.wmax, q.rp, v[j])));
                        } else {
                            q.st[v[j]] = ST_NEW;
                        }
                    }
                    wave_append(set, v[j], Sp, &s_nset[pp]);
                    wave_append(keep, v[j], Fn, &s_nnext[pp]);
                }
            }
            __syncthreads();
            // every wavefront is past the previous phase's last counter reads
            if (threadIdx.x == 0) hub_n[pp ^ 1] = s_nset[pp ^ 1] = s_nnext[pp ^ 1] = 0;
            const uint32_t nS = s_nset[pp];
            ++phases;
            if (nS == 0 || phases > n + 1) {  // a non-empty fringe always certifies its minimum
                if (threadIdx.x == 0) atomicOr(&ctl->error, 1u);
                break;
            }
            // relax: short rows by their own lane, long rows by the whole workgroup
            unsigned long long cmin = INF64, ctst = INF64;
            for (uint32_t base = 0; base < nS; base += BS) {
                const uint32_t i = base + threadIdx.x;
                uint32_t b = 0, e = 0;
                unsigned long long du = 0;
                if (i < nS) {
                    const uint32_t v = ld_u32(&Sp[i]);
                    q.st[v] = ST_S;
                    b = q.rp[v];
                    e = q.rp[v + 1];
                    du = ld_dist(&q.dist[v]);
                    if (e - b > split) {
                        const uint32_t slot = atomicAdd(&hub_n[pp], 1u);
                        if (slot < kHubCap) {
                            hub_v[slot] = v;
                            hub_du[slot] = du;
                            e = b;  // expanded below by the whole workgroup
                        }
                    }
                }
                // lanes walk their rows in lock step so discoveries can be appended per wavefront
                uint32_t len = e - b;
                uint32_t mx = len;
                for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
                for (uint32_t k = 0; k < mx; k += kBatchU) {
                    uint2 ed[kBatchU];
                    uint32_t em[kBatchU];
                    uint32_t have = 0;
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j) {
                        ed[j] = make_uint2(0u, 0u);
                        em[j] = INF32;
                        if (k + j < len) {
                            ed[j] = q.edges[b + k + j];
                            if (OUT) em[j] = q.emin[b + k + j];
                            have |= 1u << j;
                        }
                    }
                    const uint32_t disc = relax_edges<kBatchU, OUT>(q, du, ed, em, have, cmin, ctst);
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j)  // every lane of the wavefront takes part
                        wave_append((disc >> j) & 1u, ed[j].x, Fn, &s_nnext[pp]);
                }
            }
            __syncthreads();
            const uint32_t nh = min(hub_n[pp], (uint32_t)kHubCap);
            for (uint32_t h = 0; h < nh; ++h) {
                const uint32_t v = hub_v[h];
                const uint32_t b = q.rp[v], e = q.rp[v + 1];
                for (uint64_t kb = b; kb < e; kb += BS * kBatchU) {
                    uint2 ed[kBatchU];
                    uint32_t em[kBatchU];
                    uint32_t have = 0;
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j) {
                        const uint64_t k = kb + (uint64_t)j * BS + threadIdx.x;
                        ed[j] = make_uint2(0u, 0u);
                        em[j] = INF32;
                        if (k < e) {
                            ed[j] = q.edges[k];
                            if (OUT) em[j] = q.emin[k];
                            have |= 1u << j;
                        }
                    }
                    const uint32_t disc = relax_edges<kBatchU, OUT>(q, hub_du[h], ed, em, have, cmin, ctst);
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j) wave_append((disc >> j) & 1u, ed[j].x, Fn, &s_nnext[pp]);
                }
            }
            unsigned long long a = umin64(fmin, cmin), t = umin64(ftst, ctst);
            bmin2<BS>(a, t, sh);  // its barrier also completes every append of this phase
            minD = a;
            if (OUT) T = t;
            nF = s_nnext[pp];
            cur ^= 1;
        }
        if (threadIdx.x == 0) phases_out[order[qi]] = phases;
        __syncthreads();
    }
}

typedef void (*bfn)(const BatchQuery *, const uint32_t *, uint32_t, BatchCtl *, uint32_t *, uint32_t);

template <int BS>
static bfn pick_batch_bs(int in, bool out) {
    if (in == IN_DIJK) return out ? k_batch<BS, IN_DIJK, true> : k_batch<BS, IN_DIJK, false>;
    if (in == IN_STATIC_M) return out ? k_batch<BS, IN_STATIC_M, true> : k_batch<BS, IN_STATIC_M, false>;
    return out ? k_batch<BS, IN_NONE, true> : k_batch<BS, IN_NONE, false>;
}

static bfn pick_batch(int bs, int in, bool out) {
    switch (bs) {
    case 256: return pick_batch_bs<256>(in, out);
    case 1024: return pick_batch_bs<1024>(in, out);
    default: return pick_batch_bs<512>(in, out);
    }
}

static sssp_batch_cfg g_batch_cfg = {0, 0, 0};  // process-wide default shape

// One query on one workgroup of 512 threads (measured on 128^2 to 2048^2 grids:
// 512 beats 1024 by 3-15 % and 256 on all but the smallest): sssp_solve's path
// under the launch option `single`, for graphs whose phases settle few vertices
// each (the grid-wide kernels would spend most of a phase on their two launches).
// The scratch stays on the graph; the host record lives until the final sync.
int batch_solve_one(sssp_graph *g, uint32_t source, int in, bool out_static, uint64_t *dist_out,
                    uint32_t *phases_out) {
    struct OneAux {
        BatchQuery q;
        uint32_t order, phases;
        BatchCtl ctl;
    };
    hipStream_t s = g->stream;
    if (!g->one_aux) {
        HIP_OK(hipMalloc(&g->one_st, ((uint64_t)g->n + 255) & ~255ull));
        HIP_OK(hipMalloc(&g->one_fl, 3ull * g->n * sizeof(uint32_t)));
        HIP_OK(hipMalloc(&g->one_aux, sizeof(OneAux)));
    }
    OneAux h;
    memset(&h, 0, sizeof h);
    h.q = BatchQuery{g->rp, g->edges, g->vmin, g->emin, (unsigned long long *)dist_out, g->one_st, g->one_fl, g->n,
                     source, g->wmax};
    OneAux *d = (OneAux *)g->one_aux;
    HIP_OK(hipMemcpyAsync(d, &h, sizeof h, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(pick_batch(512, in, out_static), dim3(1), dim3(512), 0, s, &d->q, &d->order, 1u, &d->ctl,
                       &d->phases, 64u);
    HIP_OK(hipGetLastError());
    OneAux r;
    HIP_OK(hipMemcpyAsync(&r, d, sizeof r, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (r.ctl.error) return sssp_set_error(SSSP_ERR_INTERNAL, "the query exceeded its phase bound");
    if (phases_out) *phases_out = r.phases;
    return SSSP_OK;
}

extern "C" int sssp_batch_set_config(const sssp_batch_cfg *cfg) {
    if (!cfg) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    if (cfg->block != 0 && cfg->block != 256 && cfg->block != 512 && cfg->block != 1024)
        return sssp_set_error(SSSP_ERR_INVALID, "block size must be 256, 512 or 1024");
    g_batch_cfg = *cfg;
    return SSSP_OK;
}

extern "C" int sssp_batch_get_config(sssp_batch_cfg *cfg) {
    if (!cfg) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    *cfg = g_batch_cfg;
    return SSSP_OK;
}

extern "C" int sssp_solve_batch(sssp_graph *const *graphs, const uint32_t *sources, uint32_t nq,
                                uint32_t criterion, uint64_t *const *dist_outs, uint32_t *phases_out) {
    return sssp_solve_batch_ex(graphs, sources, nq, criterion, dist_outs, phases_out, nullptr);
}

extern "C" int sssp_solve_batch_ex(sssp_graph *const *graphs, const uint32_t *sources, uint32_t nq,
                                   uint32_t criterion, uint64_t *const *dist_outs, uint32_t *phases_out,
                                   const sssp_batch_cfg *cfg_in) {
    const sssp_batch_cfg cfg = cfg_in ? *cfg_in : g_batch_cfg;
    if (cfg.block != 0 && cfg.block != 256 && cfg.block != 512 && cfg.block != 1024)
        return sssp_set_error(SSSP_ERR_INVALID, "block size must be 256, 512 or 1024");
    if (nq == 0 || !graphs || !sources || !dist_outs)
        return sssp_set_error(SSSP_ERR_INVALID, "empty batch or NULL array");
    if (criterion == 0 || (criterion & ~SSSP_CRIT_ALL))
        return sssp_set_error(SSSP_ERR_INVALID, "criterion 0x%x is empty or has unknown bits", criterion);
    int in = IN_NONE, out = OUT_NONE;
    crit_modes(criterion, &in, &out);
    if (in > IN_STATIC_M || out > OUT_STATIC_M)
        return sssp_set_error(SSSP_ERR_UNSUPPORTED, "the batched solver evaluates DIJK, IN-STATIC and OUT-STATIC");
    std::vector<BatchQuery> hq(nq);
    std::vector<uint64_t> st_off(nq), fl_off(nq);
    uint64_t st_total = 0, fl_total = 0;
    for (uint32_t i = 0; i < nq; ++i) {
        const sssp_graph *g = graphs[i];
        if (!g || !dist_outs[i]) return sssp_set_error(SSSP_ERR_INVALID, "query %u: NULL graph or output", i);
        if (sources[i] >= g->n) return sssp_set_error(SSSP_ERR_INVALID, "query %u: source %u >= n", i, sources[i]);
        hq[i].rp = g->rp;
        hq[i].edges = g->edges;
        hq[i].vmin = g->vmin;
        hq[i].emin = g->emin;
        hq[i].dist = (unsigned long long *)dist_outs[i];
        hq[i].n = g->n;
        hq[i].src = sources[i];
        hq[i].wmax = g->wmax;
        st_off[i] = st_total;
        st_total += (g->n + 255) & ~255ull;
        fl_off[i] = fl_total;
        fl_total += 3ull * g->n;
    }
    // longest-processing-time order: most edges first
    std::vector<uint32_t> order(nq);
    for (uint32_t i = 0; i < nq; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return graphs[x]->m + graphs[x]->n > graphs[y]->m + graphs[y]->n;
    });
    hipStream_t s = graphs[0]->stream;
    HIP_OK(hipSetDevice(graphs[0]->device));
    uint8_t *st = nullptr;
    uint32_t *fl = nullptr;
    BatchQuery *dq = nullptr;
    uint32_t *dorder = nullptr, *dph = nullptr;
    BatchCtl *dctl = nullptr;
    int rc = SSSP_OK;
#define TRY(call) do { hipError_t _e = (call); if (_e != hipSuccess) { \
        rc = sssp_set_error(_e == hipErrorOutOfMemory ? SSSP_ERR_OOM : SSSP_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(_e)); goto done; } } while (0)
    TRY(hipMalloc(&st, st_total));
    TRY(hipMalloc(&fl, fl_total * sizeof(uint32_t)));
    for (uint32_t i = 0; i < nq; ++i) {
        hq[i].st = st + st_off[i];
        hq[i].fl = fl + fl_off[i];
    }
    TRY(hipMalloc(&dq, nq * sizeof(BatchQuery)));
    TRY(hipMalloc(&dorder, nq * sizeof(uint32_t)));
    TRY(hipMalloc(&dph, nq * sizeof(uint32_t)));
    TRY(hipMalloc(&dctl, sizeof(BatchCtl)));
    TRY(hipMemcpyAsync(dq, hq.data(), nq * sizeof(BatchQuery), hipMemcpyHostToDevice, s));
    TRY(hipMemcpyAsync(dorder, order.data(), nq * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    TRY(hipMemsetAsync(dctl, 0, sizeof(BatchCtl), s));
    {
        int dev = 0, cus = 256;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        const int bs = cfg.block ? (int)cfg.block : 512;
        const uint32_t split = cfg.split ? cfg.split : 64;
        uint32_t grid = cfg.blocks ? cfg.blocks : (uint32_t)cus * (bs >= 1024 ? 2 : 4);
        if (grid > nq) grid = nq;
        bfn k = pick_batch(bs, in, out == OUT_STATIC_M);
        hipLaunchKernelGGL(k, dim3(grid), dim3(bs), 0, s, dq, dorder, nq, dctl, dph, split);
        TRY(hipGetLastError());
        BatchCtl hctl;
        TRY(hipMemcpyAsync(&hctl, dctl, sizeof hctl, hipMemcpyDeviceToHost, s));
        if (phases_out) TRY(hipMemcpyAsync(phases_out, dph, nq * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        if (hctl.error) rc = sssp_set_error(SSSP_ERR_INTERNAL, "a batched query exceeded its phase bound");
    }
done:
#undef TRY
    sssp_free(st); sssp_free(fl); sssp_free(dq); sssp_free(dorder); sssp_free(dph); sssp_free(dctl);
    return rc;
}
