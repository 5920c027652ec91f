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
    uint2 *fm;         // 2 * n entries: (minIn, minOut) of each fringe list entry
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
__device__ __forceinline__ uint2 ld_u2(const uint2 *p) {
    const unsigned long long x =
        __hip_atomic_load(reinterpret_cast<const unsigned long long *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
}
// Stores of values another workgroup of a team reads (team launch only): device-scope
// atomic stores, which do not stay in one die's L2, so that a team barrier only has to
// wait for its own stores to complete (no cache write-back).
template <typename T>
__device__ __forceinline__ void st_dev(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
template <bool TEAM = false>
__device__ __forceinline__ void wave_append(bool take, uint32_t v, uint32_t *list, uint32_t *cnt) {
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (!take) return;
    uint32_t *slot = &list[base + __popcll(mask & ((1ull << lane) - 1ull))];
    if (TEAM) st_dev(slot, v);
    else *slot = v;
}

// Relaxes the edges ed[j] (bit j of have) from a vertex at distance du: the
// state and distance loads of all of them are issued together, then the
// atomics. Returns the mask of edges whose atomic replaced infinity (the
// target was discovered; exactly one atomic can do that). MM: also loads each
// target's static minima into tm (with the state and distance), for the
// fringe entry of a discovered target.
template <int U, bool OUT, bool TEAM = false, bool MM = false>
__device__ __forceinline__ uint32_t relax_edges(const BatchQuery &q, unsigned long long du, const uint2 *ed,
                                                const uint32_t *em, uint32_t have, unsigned long long &cmin,
                                                unsigned long long &ctst, uint2 *tm = nullptr) {
    uint8_t sv[U];
    unsigned long long cur[U], cand[U], old[U];
#pragma unroll
    for (int j = 0; j < U; ++j) {
        sv[j] = ST_S;
        cur[j] = 0;
        if (MM) tm[j] = make_uint2(INF32, INF32);
        if ((have >> j) & 1u) {
            sv[j] = ld_st(&q.st[ed[j].x]);
            cur[j] = ld_dist(&q.dist[ed[j].x]);
            if (MM) tm[j] = q.vmin[ed[j].x];
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
            if (TEAM) st_dev(&q.st[ed[j].x], (uint8_t)ST_F);
            else q.st[ed[j].x] = ST_F;
            disc |= 1u << j;
        }
    }
    return disc;
}

constexpr int kBatchU = 4;  // fringe entries / edges a lane handles per step

// Wavefront-aggregated append of a fringe entry: vertex v to list, its static
// minima mm to mlist at the same index (a phase then reads a fringe vertex's
// minima from its entry, coalesced, instead of gathering them). TEAM: other
// members read the entry, so it is written with device-scope atomic stores.
template <bool TEAM = false>
__device__ __forceinline__ void wave_append_fm(bool take, uint32_t v, uint2 mm, uint32_t *list, uint2 *mlist,
                                               uint32_t *cnt) {
    const int lane = threadIdx.x & 63;
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(cnt, (uint32_t)__popcll(mask));
    base = __shfl(base, leader, 64);
    if (!take) return;
    const uint32_t i = base + (uint32_t)__popcll(mask & ((1ull << lane) - 1ull));
    if (TEAM) {
        st_dev(&list[i], v);
        st_dev(reinterpret_cast<unsigned long long *>(&mlist[i]), ((unsigned long long)mm.y << 32) | mm.x);
    } else {
        list[i] = v;
        mlist[i] = mm;
    }
}

// One workgroup per query, queries taken from order[0 .. nq) through ctl->next.
// IN: IN_NONE, IN_DIJK or IN_STATIC_M; OUT: OUT-STATIC on/off.
template <int BS, int IN, bool OUT>
__device__ __forceinline__ void batch_single(const BatchQuery *__restrict__ queries, const uint32_t *__restrict__ order,
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
            q.fm[0] = q.vmin[q.src];
            for (int k = 0; k < 2; ++k) hub_n[k] = s_nset[k] = s_nnext[k] = 0;
        }
        uint32_t nF = 1, cur = 0, phases = 0;
        unsigned long long minD = 0, T = min_out64(q.vmin[q.src].y, q.wmax, q.rp, q.src);
        __syncthreads();
        while (nF > 0) {
            uint32_t *F = q.fl + (uint64_t)cur * n;
            uint32_t *Fn = q.fl + (uint64_t)(cur ^ 1) * n;
            uint32_t *Sp = q.fl + 2ull * n;
            const uint2 *Fm = q.fm + (uint64_t)cur * n;
            uint2 *Fnm = q.fm + (uint64_t)(cur ^ 1) * n;
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
                        mm[j] = ld_u2(&Fm[base + j * BS + threadIdx.x]);  // the entry's minima (coalesced)
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
                    wave_append_fm(keep, v[j], mm[j], Fn, Fnm, &s_nnext[pp]);
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
                    uint2 tm[kBatchU];
                    const uint32_t disc = relax_edges<kBatchU, OUT, false, true>(q, du, ed, em, have, cmin, ctst, tm);
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j)  // every lane of the wavefront takes part
                        wave_append_fm((disc >> j) & 1u, ed[j].x, tm[j], Fn, Fnm, &s_nnext[pp]);
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
                    uint2 tm[kBatchU];
                    const uint32_t disc =
                        relax_edges<kBatchU, OUT, false, true>(q, hub_du[h], ed, em, have, cmin, ctst, tm);
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j)
                        wave_append_fm((disc >> j) & 1u, ed[j].x, tm[j], Fn, Fnm, &s_nnext[pp]);
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

// ---------------------------------------------------------------------------
// Large queries: a team of W workgroups per query (one cooperative launch, so
// that every member is resident while the others wait for it).
//
// The team runs the same phase loop with the query's lists shared: member m
// takes the fringe entries and settled vertices m, m + W, ... (in steps of a
// workgroup's width), appends to the shared lists through the team's global
// counters (one atomic per wavefront) and folds its minima into the team's
// slots, and the team meets at a barrier after identify and after relax. Lists
// and counters are double-buffered by phase parity as in the one-workgroup
// kernel: the slots of phase p + 1 are cleared by member 0 after phase p's first
// barrier, when every member has read them for the last time.
// Every value one member writes and another reads (distances, states, list
// entries, counters, minima) is written with device-scope atomics (st_dev,
// atomicAdd, atomicMin) and read with device-scope loads (ld_*), so the
// barrier needs no cache write-back or invalidation: each thread waits for its
// own memory operations to complete, then the member's thread 0 adds one to
// the team's arrival counter and waits until it reaches W times the barrier's
// index. The wait is bounded: past kTeamSpin polls, or once another member has
// failed, the member sets the error and leaves, so a kernel whose members could
// not all run ends instead of hanging.

struct TeamCtl {
    unsigned int bar;                   // arrivals (monotone over the launch)
    unsigned int pad;
    unsigned int nset[2], nnext[2];     // S' and next-fringe lengths by phase parity
    unsigned long long fmin[2], ftst[2];// next minD / OUT-STATIC threshold by phase parity
};

constexpr unsigned long long kTeamSpin = 1ull << 22;

// All threads of the member; false if the team failed (the caller leaves).
__device__ __forceinline__ bool team_barrier(TeamCtl *tc, uint32_t W, uint32_t &arrivals, BatchCtl *ctl,
                                             int *s_ok) {
    __builtin_amdgcn_s_waitcnt(0);  // this thread's stores and atomics have completed
    __syncthreads();
    arrivals += W;
    if (threadIdx.x == 0) {
        int ok = 1;
        atomicAdd(&tc->bar, 1u);
        unsigned long long spins = 0;
        while (__hip_atomic_load(&tc->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < arrivals) {
            if (++spins > kTeamSpin || __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (!ok) atomicOr(&ctl->error, 2u);
        *s_ok = ok;
    }
    __syncthreads();
    return *s_ok != 0;
}

// Workgroups [0, nteams * W) form the teams of the large queries; the others
// take the remaining queries one per workgroup (batch_single) at the same time.
template <int BS, int IN, bool OUT>
__global__ __launch_bounds__(BS) void k_batch_team(const BatchQuery *__restrict__ queries,
                                                   const uint32_t *__restrict__ large, uint32_t nlarge, uint32_t W,
                                                   uint32_t nteams, TeamCtl *teams,
                                                   const uint32_t *__restrict__ small, uint32_t nsmall, BatchCtl *ctl,
                                                   uint32_t *__restrict__ phases_out, uint32_t split) {
    __shared__ unsigned long long sh[2 * (BS / 64)];
    __shared__ uint32_t hub_v[kHubCap];
    __shared__ unsigned long long hub_du[kHubCap];
    __shared__ uint32_t hub_n;
    __shared__ int s_ok;
    if (blockIdx.x >= nteams * W) {
        batch_single<BS, IN, OUT>(queries, small, nsmall, ctl, phases_out, split);
        return;
    }
    const uint32_t t = blockIdx.x / W, m = blockIdx.x % W;
    TeamCtl *tc = teams + t;
    uint32_t arrivals = 0;
    for (uint32_t qi = t; qi < nlarge; qi += nteams) {
        const BatchQuery q = queries[large[qi]];
        const uint32_t n = q.n;
        for (uint32_t v = m * BS + threadIdx.x; v < n; v += W * BS) {
            st_dev(&q.dist[v], v == q.src ? 0ull : INF64);
            st_dev(&q.st[v], (uint8_t)(v == q.src ? ST_F : ST_U));
        }
        if (m == 0 && threadIdx.x == 0) {
            st_dev(&q.fl[0], q.src);
            const uint2 m0 = q.vmin[q.src];
            st_dev(reinterpret_cast<unsigned long long *>(&q.fm[0]), ((unsigned long long)m0.y << 32) | m0.x);
            for (int k = 0; k < 2; ++k) {
                st_dev(&tc->nset[k], 0u);
                st_dev(&tc->nnext[k], 0u);
                st_dev(&tc->fmin[k], INF64);
                st_dev(&tc->ftst[k], INF64);
            }
        }
        if (!team_barrier(tc, W, arrivals, ctl, &s_ok)) return;
        uint32_t nF = 1, cur = 0, phases = 0;
        unsigned long long minD = 0, T = min_out64(q.vmin[q.src].y, q.wmax, q.rp, q.src);
        while (nF > 0) {  // team-uniform: every member reads the same counters after a barrier
            uint32_t *F = q.fl + (uint64_t)cur * n;
            uint32_t *Fn = q.fl + (uint64_t)(cur ^ 1) * n;
            uint32_t *Sp = q.fl + 2ull * n;
            const uint2 *Fm = q.fm + (uint64_t)cur * n;
            uint2 *Fnm = q.fm + (uint64_t)(cur ^ 1) * n;
            const int pp = (int)(phases & 1u);
            unsigned long long fmin = INF64, ftst = INF64;
            for (uint32_t base = m * BS * kBatchU; base < nF; base += W * BS * kBatchU) {
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
                        mm[j] = ld_u2(&Fm[base + j * BS + threadIdx.x]);  // the entry's minima (coalesced)
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
                            st_dev(&q.st[v[j]], (uint8_t)ST_NEW);
                        }
                    }
                    wave_append<true>(set, v[j], Sp, &tc->nset[pp]);
                    wave_append_fm<true>(keep, v[j], mm[j], Fn, Fnm, &tc->nnext[pp]);
                }
            }
            if (!team_barrier(tc, W, arrivals, ctl, &s_ok)) return;
            const uint32_t nS = ld_u32(&tc->nset[pp]);
            if (m == 0 && threadIdx.x == 0) {  // every member read phase p - 1's slots before this barrier
                st_dev(&tc->nset[pp ^ 1], 0u);
                st_dev(&tc->nnext[pp ^ 1], 0u);
                st_dev(&tc->fmin[pp ^ 1], INF64);
                st_dev(&tc->ftst[pp ^ 1], INF64);
            }
            if (threadIdx.x == 0) hub_n = 0;
            ++phases;
            if (nS == 0 || phases > n + 1) {  // a non-empty fringe always certifies its minimum
                if (threadIdx.x == 0) atomicOr(&ctl->error, 1u);
                return;
            }
            __syncthreads();  // hub_n cleared
            unsigned long long cmin = INF64, ctst = INF64;
            for (uint32_t base = m * BS; base < nS; base += W * BS) {
                const uint32_t i = base + threadIdx.x;
                uint32_t b = 0, e = 0;
                unsigned long long du = 0;
                if (i < nS) {
                    const uint32_t v = ld_u32(&Sp[i]);
                    st_dev(&q.st[v], (uint8_t)ST_S);
                    b = q.rp[v];
                    e = q.rp[v + 1];
                    du = ld_dist(&q.dist[v]);
                    if (e - b > split) {
                        const uint32_t slot = atomicAdd(&hub_n, 1u);
                        if (slot < kHubCap) {
                            hub_v[slot] = v;
                            hub_du[slot] = du;
                            e = b;  // expanded below by the whole workgroup
                        }
                    }
                }
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
                    uint2 tm[kBatchU];
                    const uint32_t disc = relax_edges<kBatchU, OUT, true, true>(q, du, ed, em, have, cmin, ctst, tm);
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j)
                        wave_append_fm<true>((disc >> j) & 1u, ed[j].x, tm[j], Fn, Fnm, &tc->nnext[pp]);
                }
            }
            __syncthreads();
            const uint32_t nh = min(hub_n, (uint32_t)kHubCap);
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
                    uint2 tm[kBatchU];
                    const uint32_t disc =
                        relax_edges<kBatchU, OUT, true, true>(q, hub_du[h], ed, em, have, cmin, ctst, tm);
#pragma unroll
                    for (int j = 0; j < kBatchU; ++j)
                        wave_append_fm<true>((disc >> j) & 1u, ed[j].x, tm[j], Fn, Fnm, &tc->nnext[pp]);
                }
            }
            unsigned long long a = umin64(fmin, cmin), tt = umin64(ftst, ctst);
            bmin2<BS>(a, tt, sh);
            if (threadIdx.x == 0) {
                if (a != INF64) atomicMin(&tc->fmin[pp], a);
                if (OUT && tt != INF64) atomicMin(&tc->ftst[pp], tt);
            }
            if (!team_barrier(tc, W, arrivals, ctl, &s_ok)) return;
            nF = ld_u32(&tc->nnext[pp]);
            minD = __hip_atomic_load(&tc->fmin[pp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (OUT) T = __hip_atomic_load(&tc->ftst[pp], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            cur ^= 1;
        }
        if (m == 0 && threadIdx.x == 0) phases_out[large[qi]] = phases;
        // every member has read the last phase's counters before member 0 clears them for the next query
        if (!team_barrier(tc, W, arrivals, ctl, &s_ok)) return;
    }
}

typedef void (*tfn)(const BatchQuery *, const uint32_t *, uint32_t, uint32_t, uint32_t, TeamCtl *, const uint32_t *,
                    uint32_t, BatchCtl *, uint32_t *, uint32_t);

template <int BS>
static tfn pick_team_bs(int in, bool out) {
    if (in == IN_DIJK) return out ? k_batch_team<BS, IN_DIJK, true> : k_batch_team<BS, IN_DIJK, false>;
    if (in == IN_STATIC_M) return out ? k_batch_team<BS, IN_STATIC_M, true> : k_batch_team<BS, IN_STATIC_M, false>;
    return out ? k_batch_team<BS, IN_NONE, true> : k_batch_team<BS, IN_NONE, false>;
}

static tfn pick_team(int bs, int in, bool out) {
    switch (bs) {
    case 256: return pick_team_bs<256>(in, out);
    case 1024: return pick_team_bs<1024>(in, out);
    default: return pick_team_bs<512>(in, out);
    }
}

template <int BS, int IN, bool OUT>
__global__ __launch_bounds__(BS) void k_batch(const BatchQuery *__restrict__ queries, const uint32_t *__restrict__ order,
                                              uint32_t nq, BatchCtl *ctl, uint32_t *__restrict__ phases_out,
                                              uint32_t split) {
    batch_single<BS, IN, OUT>(queries, order, nq, ctl, phases_out, split);
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

static sssp_batch_cfg g_batch_cfg = {0, 0, 0, 0, 0};  // process-wide default shape

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
    if (!(g->one_aux && g->one_st && g->one_fl && g->one_fm)) {  // all or none (a failed call may leave some)
        sssp_free(g->one_st); sssp_free(g->one_fl); sssp_free(g->one_fm); sssp_free(g->one_aux);
        g->one_st = nullptr;
        g->one_fl = nullptr;
        g->one_fm = nullptr;
        g->one_aux = nullptr;
        HIP_OK(hipMalloc(&g->one_st, ((uint64_t)g->n + 255) & ~255ull));
        HIP_OK(hipMalloc(&g->one_fl, 3ull * g->n * sizeof(uint32_t)));
        HIP_OK(hipMalloc(&g->one_fm, 2ull * g->n * sizeof(uint2)));
        HIP_OK(hipMalloc(&g->one_aux, sizeof(OneAux)));
    }
    OneAux h;
    memset(&h, 0, sizeof h);
    h.q = BatchQuery{g->rp,   g->edges,  g->vmin, g->emin, (unsigned long long *)dist_out, g->one_st, g->one_fl,
                     g->one_fm, g->n, source, g->wmax};
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
    std::vector<uint64_t> st_off(nq), fl_off(nq), fm_off(nq);
    uint64_t st_total = 0, fl_total = 0, fm_total = 0;
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
        fm_off[i] = fm_total;
        fm_total += 2ull * g->n;
    }
    // longest-processing-time order: most edges first; queries on graphs with at least
    // team_edges edges go to the team launch
    std::vector<uint32_t> order(nq);
    for (uint32_t i = 0; i < nq; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t x, uint32_t y) {
        return graphs[x]->m + graphs[x]->n > graphs[y]->m + graphs[y]->n;
    });
    const uint64_t team_edges = cfg.team_edges ? cfg.team_edges : (1u << 20);
    if (cfg.team_size == 1 || cfg.team_size > 64)
        return sssp_set_error(SSSP_ERR_INVALID, "team size must be 2 .. 64 (0: automatic)");
    std::vector<uint32_t> large, small;
    for (uint32_t i : order) (cfg.team_edges != UINT32_MAX && graphs[i]->m >= team_edges ? large : small).push_back(i);
    hipStream_t s = graphs[0]->stream;
    HIP_OK(hipSetDevice(graphs[0]->device));
    uint8_t *st = nullptr;
    uint32_t *fl = nullptr;
    uint2 *fm = nullptr;
    BatchQuery *dq = nullptr;
    uint32_t *dorder = nullptr, *dph = nullptr, *dlarge = nullptr;
    BatchCtl *dctl = nullptr;
    TeamCtl *dteams = nullptr;
    int rc = SSSP_OK;
#define TRY(call) do { hipError_t _e = (call); if (_e != hipSuccess) { \
        rc = sssp_set_error(_e == hipErrorOutOfMemory ? SSSP_ERR_OOM : SSSP_ERR_DEVICE, "%s: %s", #call, hipGetErrorString(_e)); goto done; } } while (0)
    TRY(hipMalloc(&st, st_total));
    TRY(hipMalloc(&fl, fl_total * sizeof(uint32_t)));
    TRY(hipMalloc(&fm, fm_total * sizeof(uint2)));
    for (uint32_t i = 0; i < nq; ++i) {
        hq[i].st = st + st_off[i];
        hq[i].fl = fl + fl_off[i];
        hq[i].fm = fm + fm_off[i];
    }
    TRY(hipMalloc(&dq, nq * sizeof(BatchQuery)));
    TRY(hipMalloc(&dorder, nq * sizeof(uint32_t)));
    TRY(hipMalloc(&dph, nq * sizeof(uint32_t)));
    TRY(hipMalloc(&dctl, sizeof(BatchCtl)));
    TRY(hipMemcpyAsync(dq, hq.data(), nq * sizeof(BatchQuery), hipMemcpyHostToDevice, s));
    TRY(hipMemsetAsync(dctl, 0, sizeof(BatchCtl), s));
    {
        int dev = 0, cus = 256;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess) cus = p.multiProcessorCount;
        const int bs = cfg.block ? (int)cfg.block : 512;
        uint32_t split = cfg.split ? cfg.split : 64;
        bool teamed = false;
        if (!large.empty()) {
            // one cooperative launch: teams of W workgroups for the large queries, the other
            // resident workgroups for the rest, all at once
            tfn tk = pick_team(bs, in, out == OUT_STATIC_M);
            int per_cu = 0;
            TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)tk, bs, 0));
            const uint64_t resident = (uint64_t)(per_cu > 0 ? per_cu : 0) * cus;
            uint32_t nlarge = (uint32_t)large.size();
            uint32_t W = cfg.team_size;
            if (!W) {  // at most half of the resident workgroups in teams
                W = 16;
                while (W > 2 && (uint64_t)W * nlarge * 2 > resident) W /= 2;
            }
            const uint32_t nteams = (uint32_t)std::min<uint64_t>(nlarge, resident / W / 2 ? resident / W / 2 : 1);
            const uint64_t team_blocks = (uint64_t)nteams * W;
            if (team_blocks < resident) {
                uint32_t nsmall = (uint32_t)small.size();
                uint64_t single_blocks = cfg.blocks ? cfg.blocks : (uint64_t)cus * (bs >= 1024 ? 2 : 4);
                if (single_blocks > nsmall) single_blocks = nsmall;
                if (team_blocks + single_blocks > resident) single_blocks = resident - team_blocks;
                uint32_t grid = (uint32_t)(team_blocks + single_blocks);
                TRY(hipMalloc(&dlarge, nlarge * sizeof(uint32_t)));
                TRY(hipMalloc(&dteams, nteams * sizeof(TeamCtl)));
                TRY(hipMemcpyAsync(dlarge, large.data(), nlarge * sizeof(uint32_t), hipMemcpyHostToDevice, s));
                TRY(hipMemsetAsync(dteams, 0, nteams * sizeof(TeamCtl), s));
                if (nsmall) TRY(hipMemcpyAsync(dorder, small.data(), nsmall * sizeof(uint32_t), hipMemcpyHostToDevice, s));
                uint32_t nt = nteams;
                void *args[] = {&dq, &dlarge, &nlarge, &W, &nt, &dteams, &dorder, &nsmall, &dctl, &dph, &split};
                TRY(hipLaunchCooperativeKernel((const void *)tk, dim3(grid), dim3(bs), args, 0, s));
                teamed = true;
            } else {
                small.insert(small.begin(), large.begin(), large.end());  // no room for a team
            }
        }
        const uint32_t nsmall = (uint32_t)small.size();
        if (!teamed && nsmall) {
            TRY(hipMemcpyAsync(dorder, small.data(), nsmall * sizeof(uint32_t), hipMemcpyHostToDevice, s));
            uint32_t grid = cfg.blocks ? cfg.blocks : (uint32_t)cus * (bs >= 1024 ? 2 : 4);
            if (grid > nsmall) grid = nsmall;
            bfn k = pick_batch(bs, in, out == OUT_STATIC_M);
            hipLaunchKernelGGL(k, dim3(grid), dim3(bs), 0, s, dq, dorder, nsmall, dctl, dph, split);
            TRY(hipGetLastError());
        }
        BatchCtl hctl;
        TRY(hipMemcpyAsync(&hctl, dctl, sizeof hctl, hipMemcpyDeviceToHost, s));
        if (phases_out) TRY(hipMemcpyAsync(phases_out, dph, nq * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TRY(hipStreamSynchronize(s));
        if (hctl.error & 2u) rc = sssp_set_error(SSSP_ERR_INTERNAL, "a team of the batched launch timed out at a barrier");
        else if (hctl.error) rc = sssp_set_error(SSSP_ERR_INTERNAL, "a batched query exceeded its phase bound");
    }
done:
#undef TRY
    sssp_free(st); sssp_free(fl); sssp_free(fm); sssp_free(dq); sssp_free(dorder); sssp_free(dph); sssp_free(dctl);
    sssp_free(dlarge); sssp_free(dteams);
    return rc;
}
