// Phased SSSP (Section 3) and Delta-stepping (Section 5) on one set of kernels.
//
// One phase = [term pass] -> identify -> relax, all launched back to back on
// the graph's stream with no host round trip:
//   term pass  (dynamic criteria only) per queued vertex v: the IN-family
//              minimum over in-edges of its equation, and the OUT-family
//              minimum over out-edges; the IN test result is stored as a flag
//              bit, the OUT right-hand side min_{u in F} d[u] + term(u) is
//              reduced to one threshold.
//   identify   dense, coalesced scan of the 1-byte vertex state array; every
//              queued vertex is tested against the phase-start thresholds.
//              Certified vertices are settled and compacted into S' with a
//              wavefront ballot + prefix sum and one packed (count, edges)
//              atomic per wavefront on the block's shard, which also assigns
//              each entry its shard-local offset in the phase's edge space.
//              Vertices that stay queued contribute to next phase's minD and
//              OUT-STATIC threshold.
//   relax      each shard's edge space is cut into equal chunks; a block
//              stages a chunk's S' entries (start edge, snapshot distance) in
//              LDS and each lane finds its edge's owner by binary search
//              (merge path), so rows of any degree split evenly. Each edge does
//              a plain-load filter and a 64-bit atomicMin; the atomic that
//              replaces infinity discovers the target (U -> F). Improving
//              candidates fold into next phase's minD / OUT-STATIC threshold
//              (d only decreases, so the minimum over final values equals the
//              minimum over kept values and improving candidates).
// Control state lives in device memory slots indexed by phase parity, so
// phases can be queued many at a time and empty phases exit at once; values
// combined by many blocks are sharded (see Sharded in common.h).
#include <string.h>

#include <mutex>
#include <vector>

#include "common.h"
#include "graph.h"
#include "selector.h"

static_assert(sizeof(PhaseRec) == sizeof(sssp_phase_rec), "trace record layout");

struct KArgs {
    DevGraph g;
    SolveBufs b;
    uint32_t crit;
    uint32_t approx_k;   // approximate criteria: recompute after this many counted changes (0: never)
    const float *mlp_w;  // learned mode: selector weights (device)
    double wm;           // learned mode: mean edge weight (feature scale)
    const unsigned long long *ref;  // ORACLE mode: dist(s, .) of this source (device)
    uint32_t mark;       // stored full terms: identify and relax flag state changes (ST_CHG)
    uint32_t fresh_at;   // stored full terms: the phase at which every queued vertex computes them
};

// The selector's three criteria: IN-STATIC|OUT-STATIC, IN-SIMPLE|OUT-SIMPLE, IN-SIMPLE|OUT-STATIC.
static __device__ const uint32_t kChoiceCrit[3] = {SSSP_IN_STATIC | SSSP_OUT_STATIC, SSSP_IN_SIMPLE | SSSP_OUT_SIMPLE,
                                                  SSSP_IN_SIMPLE | SSSP_OUT_STATIC};

// Host side of kChoiceCrit (same order).
static uint32_t choice_criterion(unsigned int c) {
    return c == 0 ? (SSSP_IN_STATIC | SSSP_OUT_STATIC) : c == 1 ? (SSSP_IN_SIMPLE | SSSP_OUT_SIMPLE)
                                                                : (SSSP_IN_SIMPLE | SSSP_OUT_STATIC);
}

__device__ __forceinline__ unsigned long long *slot_of(Sharded &s, int i) { return &s.v[i * kPad]; }
__device__ __forceinline__ int my_shard() { return (int)(blockIdx.x % kShards); }

// Slot `lane` of a sharded value (or `idle` for lanes past the last shard);
// wave_sum64 / wave_min64 of it combines the value in every lane. A kernel
// loads every slot it needs before the first combine, so that all those loads
// are in flight together.
__device__ __forceinline__ unsigned long long lane_slot(const Sharded &s, unsigned long long idle) {
    const int i = threadIdx.x & 63;
    return i < kShards ? s.v[i * kPad] : idle;
}
// Block 0, threads < kShards: reset every slot.
__device__ __forceinline__ void shard_fill(Sharded &s, unsigned long long x) {
    if (threadIdx.x < kShards) s.v[threadIdx.x * kPad] = x;
}

// ---------------------------------------------------------------------------
// initialisation

// Fill two u32 arrays of n entries with x (either may be null).
__global__ void k_fill_u32(uint32_t n, uint32_t *__restrict__ p, uint32_t *__restrict__ q, uint32_t x) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        if (p) p[v] = x;
        if (q) q[v] = x;
    }
}

// End of a solve: drop the settled bit from every distance word.
__global__ void k_clear_settled(uint32_t n, unsigned long long *__restrict__ d) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        const unsigned long long x = d[v];
        if (dist_settled(x)) d[v] = x & ~kSettledBit;
    }
}

__global__ void k_init_state(uint32_t n, uint32_t src, unsigned long long *__restrict__ d,
                             uint8_t *__restrict__ st, uint32_t *__restrict__ phase_of,
                             uint32_t *__restrict__ out_cur, const uint32_t *__restrict__ rp,
                             uint32_t *__restrict__ in_cur, const uint32_t *__restrict__ ip,
                             uint32_t *__restrict__ stamp, uint2 *__restrict__ out_head,
                             const uint2 *__restrict__ edges, uint2 *__restrict__ in_head,
                             const uint2 *__restrict__ in_edges) {
    const uint2 none = make_uint2(INF32, INF32);
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v < n; v += gridDim.x * blockDim.x) {
        d[v] = v == src ? 0ull : INF64;
        st[v] = v == src ? ST_F : ST_U;
        if (phase_of) phase_of[v] = 0;
        if (out_cur) {  // cursors at each row's first (lightest) edge, nothing settled yet
            const uint32_t b = rp[v];
            out_cur[v] = b;
            out_head[v] = b < rp[v + 1] ? edges[b] : none;
        }
        if (in_cur) {
            const uint32_t b = ip[v];
            in_cur[v] = b;
            in_head[v] = b < ip[v + 1] ? in_edges[b] : none;
        }
        if (stamp) stamp[v] = 0;
    }
}

// One block of 64 threads.
__global__ void k_init_ctl(Ctl *ctl, const uint2 *__restrict__ vmin, const uint32_t *__restrict__ rp, uint32_t wmax,
                           uint32_t src, uint32_t n_deltas, unsigned long long qdelta0) {
    const int i = threadIdx.x;
    if (i == 0) {
        CtlHead h;
        memset(&h, 0, sizeof h);
        h.n_deltas = n_deltas;
        h.qdelta[0] = qdelta0;  // keyed queue arrays: split margin of the first rebuild
        ctl->h = h;
    }
    if (i < kShards) {
        const int o = i * kPad;
        ctl->reached.v[o] = i == 0 ? 1ull : 0ull;
        ctl->relax_edges.v[o] = ctl->improving.v[o] = 0;
        for (int k = 0; k < 2; ++k) {
            ctl->spack[k].v[o] = ctl->szero[k].v[o] = 0;
            ctl->win_improved[k].v[o] = 0;
        }
        for (int k = 0; k < 3; ++k) ctl->minD[k].v[o] = ctl->tst[k].v[o] = ctl->tdyn[k].v[o] = INF64;
        ctl->minD[0].v[o] = i == 0 ? 0ull : INF64;
        ctl->tst[0].v[o] = i == 0 ? min_out64(vmin[src].y, wmax, rp, src) : INF64;  // 0 + minOut[s]
        ctl->nextmin[0].v[o] = i == 0 ? 0ull : INF64;
        ctl->nextmin[1].v[o] = INF64;
        for (int k = 0; k < 3; ++k) ctl->sumd[k].v[o] = 0;  // sum over F = {s} of d is 0
        ctl->degsum.v[o] = 0;
        for (int k = 0; k < 2; ++k) {
            ctl->nin[k].v[o] = ctl->nout[k].v[o] = 0;
        }
        for (int k = 0; k < 6; ++k) ctl->cnt_cf[k].v[o] = 0;
    }
}

// Learned mode: the degree sum of the queued set starts with the source, and
// the first phase's (or bucket's) choice comes from the features of {s}.
// One wavefront.
__global__ __launch_bounds__(64) void k_init_choice(KArgs a, uint32_t src, int delta_mode) {
    Ctl *ctl = a.b.ctl;
    const unsigned long long deg = a.g.rp[src + 1] - a.g.rp[src];
    FeatIn q;
    q.n = a.g.n;
    q.m = a.g.m;
    q.F = 1;
    q.S = 0;
    q.R = 1;
    q.a = 0;
    q.t = min_out64(a.g.vmin[src].y, a.g.wmax, a.g.rp, src);
    q.SD = 0;
    q.DG = deg;
    q.Fp = q.D = q.Sp = q.Ip = q.Op = 0;
    q.k = 0;
    q.Wm = a.wm;
    q.delta_mode = delta_mode;
    float x[kMlpIn];
    features_dev(q, x);
    MlpRegs W;
    mlp_load(a.mlp_w, W);
    const int c = mlp_eval(W, x, delta_mode ? 3 : 0);
    if (threadIdx.x == 0) {
        ctl->degsum.v[0] = deg;
        if (delta_mode) ctl->h.next_delta = 1ull << (12 + 2 * (c - 3));
        else ctl->h.choice[0] = (unsigned int)c;
        if (a.b.trace_feat && a.b.trace_cap)
            for (int i = 0; i < kMlpIn; ++i) a.b.trace_feat[i] = x[i];
    }
}

// ---------------------------------------------------------------------------
// S' append. Settled vertices are first collected per block in LDS (one LDS
// atomic per wavefront); at the end of the scan the block takes one packed
// (count, edges) atomic on its shard, which gives consecutive shard slots and
// consecutive shard-local edge offsets, and writes the entries out.
// chunk_start records the entry owning edge c*CH of the shard. If the LDS
// buffer fills, a wavefront appends straight to its shard instead.

constexpr int kAppendBuf = 512;
constexpr int kInOracle = 4;  // identify template value of the ORACLE criterion

struct AppendLds {
    uint32_t row[kAppendBuf];
    uint32_t deg[kAppendBuf];
    unsigned long long du[kAppendBuf];
    uint32_t cnt;     // slots reserved (may run past kAppendBuf)
    uint32_t filled;  // slots written: wavefronts whose reservation fit, which tile [0, filled)
    uint32_t zero;
    uint32_t wsum[kWaves];
    unsigned long long base;
};

template <int CH>
__device__ __forceinline__ void write_entry(const KArgs &a, int sh, uint32_t j, uint64_t off, uint32_t row,
                                            uint32_t deg, unsigned long long du) {
    const uint64_t g = (uint64_t)sh * a.b.shard_cap + j;
    a.b.srow[g] = row;
    a.b.soff[g] = (uint32_t)off;
    a.b.sdu[g] = du;
    uint32_t *cs = a.b.chunk_start + (uint64_t)sh * a.b.chunk_cap;
    for (uint64_t c = (off + CH - 1) / CH; c * CH < off + deg; ++c) cs[c] = j;
}

// Wavefront-uniform call: every lane of the wavefront takes part.
template <int CH>
__device__ __forceinline__ void append_settled(const KArgs &a, Ctl *ctl, int p2, AppendLds &L, bool set,
                                               uint32_t row, uint32_t deg, unsigned long long du) {
    const int lane = threadIdx.x & 63;
    const unsigned long long lt = (1ull << lane) - 1ull;
    const bool app = set && deg > 0;
    const unsigned long long mask = __ballot(app);
    if (mask) {
        const uint32_t cntw = (uint32_t)__popcll(mask);
        uint32_t pos = 0;
        if (lane == 0) pos = atomicAdd(&L.cnt, cntw);
        pos = __shfl(pos, 0, 64);
        if (pos + cntw <= kAppendBuf) {
            if (app) {
                const uint32_t r = pos + (uint32_t)__popcll(mask & lt);
                L.row[r] = row;
                L.deg[r] = deg;
                L.du[r] = du;
            }
            if (lane == 0) atomicAdd(&L.filled, cntw);
        } else {  // buffer full: direct append for this wavefront (its reserved slots stay unused)
            const uint32_t x = app ? deg : 0u;
            const uint32_t incl = wave_incl_scan(x);
            const uint32_t tot = __shfl(incl, 63, 64);
            unsigned long long base = 0;
            if (lane == 0) base = atomicAdd(slot_of(ctl->spack[p2], my_shard()), ((unsigned long long)cntw << 32) | tot);
            base = __shfl(base, 0, 64);
            if (app)
                write_entry<CH>(a, my_shard(), (uint32_t)(base >> 32) + (uint32_t)__popcll(mask & lt),
                                (uint32_t)base + incl - x, row, deg, du);
        }
    }
    const unsigned long long zm = __ballot(set && deg == 0);
    if (zm && lane == 0) atomicAdd(&L.zero, (uint32_t)__popcll(zm));
}

// Wavefront-uniform call: each lane appends its up to N settled vertices
// (bit i of sm) that have out-edges, with row start row[i], out-degree deg[i]
// and snapshot distance dv[i]; one LDS reservation for the whole wavefront.
template <int CH, int N>
__device__ __forceinline__ void append_settled_n(const KArgs &a, Ctl *ctl, int p2, AppendLds &L, uint32_t sm,
                                                 const uint32_t *row, const uint32_t *deg,
                                                 const unsigned long long *dv) {
    const int lane = threadIdx.x & 63;
    uint32_t k = 0, dtot = 0, z = 0;
#pragma unroll
    for (int i = 0; i < N; ++i)
        if ((sm >> i) & 1u) {
            if (deg[i]) { ++k; dtot += deg[i]; }
            else ++z;
        }
    if (__ballot(z != 0)) {
        const uint32_t zw = wave_sum32(z);
        if (lane == 0) atomicAdd(&L.zero, zw);
    }
    if (!__ballot(k != 0)) return;  // wavefront-uniform
    const uint32_t kin = wave_incl_scan(k);
    const uint32_t K = (uint32_t)__builtin_amdgcn_readlane((int)kin, 63);
    uint32_t pos = 0;
    if (lane == 0) pos = atomicAdd(&L.cnt, K);
    pos = (uint32_t)__builtin_amdgcn_readlane((int)pos, 0);
    if (pos + K <= kAppendBuf) {
        uint32_t r = pos + kin - k;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (((sm >> i) & 1u) && deg[i]) {
                L.row[r] = row[i];
                L.deg[r] = deg[i];
                L.du[r] = dv[i];
                ++r;
            }
        if (lane == 0) atomicAdd(&L.filled, K);
    } else {  // buffer full: direct append for this wavefront (its reserved slots stay unused)
        const uint32_t din = wave_incl_scan(dtot);
        const uint32_t D = (uint32_t)__builtin_amdgcn_readlane((int)din, 63);
        unsigned long long b = 0;
        if (lane == 0) b = atomicAdd(slot_of(ctl->spack[p2], my_shard()), ((unsigned long long)K << 32) | D);
        b = readlane64(b, 0);
        uint32_t j = (uint32_t)(b >> 32) + kin - k;
        uint64_t off = (uint64_t)(uint32_t)b + din - dtot;
#pragma unroll
        for (int i = 0; i < N; ++i)
            if (((sm >> i) & 1u) && deg[i]) {
                write_entry<CH>(a, my_shard(), j, off, row[i], deg[i], dv[i]);
                ++j;
                off += deg[i];
            }
    }
}

// Block-wide flush of the LDS buffer (all threads call it once, after the scan).
template <int CH>
__device__ __forceinline__ void append_flush(const KArgs &a, Ctl *ctl, int p2, AppendLds &L) {
    __syncthreads();
    // Reservations are handed out in increasing order, so every wavefront that
    // fit reserved before the first one that did not: the written slots are
    // exactly [0, filled). Slots reserved by overflowing wavefronts are never read.
    const uint32_t cnt = L.filled;
    if (cnt == 0) {  // block-uniform
        if (threadIdx.x == 0 && L.zero) atomicAdd(slot_of(ctl->szero[p2], my_shard()), (unsigned long long)L.zero);
        return;
    }
    constexpr int PER = kAppendBuf / kBlock;
    uint32_t loc[PER];
    uint32_t tsum = 0;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t t = threadIdx.x * PER + q;
        loc[q] = tsum;
        tsum += t < cnt ? L.deg[t] : 0u;
    }
    const uint32_t incl = wave_incl_scan(tsum);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) L.wsum[w] = incl;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
    for (int i = 0; i < kWaves; ++i) {
        wbase += i < w ? L.wsum[i] : 0u;
        total += L.wsum[i];
    }
    const uint32_t excl = wbase + incl - tsum;
    if (threadIdx.x == 0) {
        const int sh = my_shard();
        L.base = atomicAdd(slot_of(ctl->spack[p2], sh), ((unsigned long long)cnt << 32) | total);
        if (L.zero) atomicAdd(slot_of(ctl->szero[p2], sh), (unsigned long long)L.zero);
    }
    __syncthreads();
    const unsigned long long base = L.base;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const uint32_t t = threadIdx.x * PER + q;
        if (t < cnt)
            write_entry<CH>(a, my_shard(), (uint32_t)(base >> 32) + t, (uint64_t)(uint32_t)base + excl + loc[q],
                            L.row[t], L.deg[t], L.du[t]);
    }
}

// Four consecutive state bytes starting at 4q (bytes past n read as unexplored).
__device__ __forceinline__ uint32_t load_st4(const uint8_t *st, uint32_t q, uint32_t n) {
    const uint32_t v0 = 4 * q;
    if (v0 + 3 < n) return *reinterpret_cast<const uint32_t *>(st + v0);
    uint32_t s4 = 0;
    for (uint32_t i = 0; i < 4 && v0 + i < n; ++i) s4 |= (uint32_t)st[v0 + i] << (8 * i);
    return s4;
}

// ---------------------------------------------------------------------------
// term pass (dynamic criteria)

// Consecutive vertices in one window: a queue-array scan block owns such windows
// (one per grid step), the term and dirty-set passes take one per block.
constexpr uint32_t kOwnSpan = 16 * kBlock;

// Minimum weight of an out-edge of an unexplored x towards a non-settled vertex
// (the inner minimum of eq. crit:out), from x's weight-sorted row and x's
// monotone cursor out_cur (settled stays settled, so the cursor only moves past
// settled ends; the OUT criteria that use it have no OUT-SIMPLE cursor of their
// own). Threads evaluating neighbours of the same x in one pass may advance its
// cursor together: each starts at or before the first edge to a non-settled
// vertex, finds that same edge, and publishes it with atomicMax.
__device__ __forceinline__ unsigned long long ns_cursor(const KArgs &a, uint32_t x) {
    const uint32_t end = a.g.rp[x + 1];
    const uint32_t c0 = a.b.out_cur[x];
    uint32_t c = c0;
    unsigned long long w = INF64;
    for (; c < end; ++c) {
        const uint2 ed = a.g.edges[c];
        if ((a.b.st[ed.x] & ST_SET) != ST_S) {
            w = ed.y;
            break;
        }
    }
    if (c != c0) atomicMax(&a.b.out_cur[x], c);
    return w;
}

// SIMPLE terms (eq. crit:insimple, crit:outsimple): the weight of the lightest
// edge of v's weight-sorted row whose other end is not settled. The cursor
// only moves forward (settled stays settled); head caches the edge at the
// cursor, so while its end is not settled the term costs one state load. A
// settled end moves cursor and cache past every settled end.
__device__ __forceinline__ unsigned long long cursor_term(uint32_t *__restrict__ curs, uint2 *__restrict__ head,
                                                          const uint2 *__restrict__ row_edges,
                                                          const uint32_t *__restrict__ row_ptr, uint32_t v,
                                                          const uint8_t *__restrict__ st) {
    uint2 h = head[v];
    if (h.x != INF32 && (st[h.x] & ST_SET) == ST_S) {
        uint32_t cur = curs[v] + 1;
        const uint32_t end = row_ptr[v + 1];
        h = make_uint2(INF32, INF32);
        for (; cur < end; ++cur) {
            const uint2 e = row_edges[cur];
            if ((st[e.x] & ST_SET) != ST_S) {
                h = e;
                break;
            }
        }
        curs[v] = cur;
        head[v] = h;
    }
    return h.x != INF32 ? (unsigned long long)h.y : INF64;
}

// The dynamic IN term of a queued vertex v (INF64 when none): eq. crit:insimple
// from the cursor, or eq. crit:in by a scan of v's in-edges.
template <int IN>
__device__ __forceinline__ unsigned long long in_term(const KArgs &a, uint32_t v) {
    if (IN == IN_SIMPLE_M) {
        // eq. crit:insimple: lightest in-edge from a non-settled vertex; sorted row + cursor
        return cursor_term(a.b.in_cur, a.b.in_head, a.g.in_edges, a.g.ip, v, a.b.st);
    }
    // eq. crit:in: in-edges from F, or from w in U plus w's own lightest in-edge
    // (every in-neighbour of an unexplored w is queued or unexplored)
    unsigned long long term = INF64;
    const uint32_t end = a.g.ip[v + 1];
    for (uint32_t e = a.g.ip[v]; e < end; ++e) {
        const uint2 ie = a.g.in_edges[e];
        const uint8_t sw = a.b.st[ie.x] & ST_SET;
        if (sw == ST_F) term = umin64(term, ie.y);
        else if (sw == ST_U) term = umin64(term, sadd64(ie.y, min_in_u64(a.g.vmin[ie.x].x, a.g.wmax, a.g.ip, ie.x)));
    }
    return term;
}

// The dynamic OUT term of a queued vertex u (INF64 when none): eq. crit:outsimple
// from the cursor, eq. crit:outweak or eq. crit:out by a scan of u's out-edges.
template <int OUT>
__device__ __forceinline__ unsigned long long out_term(const KArgs &a, uint32_t u) {
    if (OUT == OUT_SIMPLE_M) {
        // eq. crit:outsimple (u in F, w in F u U): lightest out-edge to a non-settled vertex
        return cursor_term(a.b.out_cur, a.b.out_head, a.g.edges, a.g.rp, u, a.b.st);
    }
    unsigned long long term = INF64;
    const uint32_t end = a.g.rp[u + 1];
    for (uint32_t e = a.g.rp[u]; e < end; ++e) {
        const uint2 ed = a.g.edges[e];
        const uint8_t sx = a.b.st[ed.x] & ST_SET;
        if (sx == ST_F) {
            term = umin64(term, ed.y);
        } else if (sx == ST_U) {
            // eq. crit:outweak: second edge over all of V; eq. crit:out: into F u U
            const unsigned long long second =
                OUT == OUT_WEAK_M ? min_out64(a.g.vmin[ed.x].y, a.g.wmax, a.g.rp, ed.x) : ns_cursor(a, ed.x);
            term = umin64(term, sadd64(ed.y, second));
        }
    }
    return term;
}

// Dynamic terms of one queued vertex v (distance dv at phase start): the IN
// result as a flag, and d + the OUT term for the phase threshold (INF64
// without a dynamic OUT).
template <int IN, int OUT>
__device__ __forceinline__ bool vertex_terms(const KArgs &a, uint32_t v, unsigned long long dv,
                                             unsigned long long minD, unsigned long long &tval) {
    const bool ok = IN != IN_NONE && dv <= sadd64(minD, in_term<IN>(a, v));
    tval = OUT != OUT_NONE ? sadd64(dv, out_term<OUT>(a, v)) : INF64;
    return ok;
}

// Dirty-set maintenance of the stored IN (full), OUTWEAK and OUT (full) terms
// (Section 3 keeps these minima per vertex and updates them as neighbours
// change state). A vertex whose state changed in the last phase carries ST_CHG:
//  - discovered w (U -> F; relax also flagged w ST_TDIRTY, so its own terms are
//    computed in full): the candidate of w in an out-neighbour v's IN term was
//    c(w,v) + minIn(w) and is now c(w,v), so tin[v] = min(tin[v], c(w,v)); the
//    candidate of w in an in-neighbour u's OUT term (c(u,w) plus w's static
//    lightest out-edge, or plus its lightest out-edge to a non-settled vertex)
//    is now c(u,w), so tout[u] = min(tout[u], c(u,w));
//  - settled w (F -> S): its candidate c leaves the IN term of each out-neighbour
//    and the OUT term of each in-neighbour; where the stored term equals c it may
//    rise, and that vertex is flagged ST_TDIRTY (computed in full by the term
//    pass); elsewhere the minimum is unchanged;
//  - OUT (full) only: a settled w may also raise, for an unexplored in-neighbour
//    x, the lightest out-edge of x to a non-settled vertex (ns_cursor), which
//    enters the OUT term of every in-neighbour z of x as c(z, x) + that weight:
//    when x's cursor points at an edge to w, each z whose stored term equals its
//    candidate through x is flagged. Every stored OUT term that used x's value
//    was computed with the cursor at that edge, and the cursor cannot move on
//    before w settles, so the check sees it there.
// Stored values of vertices that are not queued are never read (a vertex is
// computed in full in the phase it is first queued, after this pass), so updates
// that land on them are harmless. The changed vertices of a window go to an LDS
// list whose rows the block walks together (below); all state writes here are
// atomic.

// Flattened row walk of a block's list of selected vertices (dirty-set and term
// passes): entry j holds a vertex, a flag byte, its first in-edge (CSC) and
// first out-edge (CSR) and how many of its in-edges are walked (n1) before its
// out-edges; off[j] holds its edge count until row_list_scan turns the counts
// into exclusive offsets (off[cnt] = total). Each thread then takes an equal
// contiguous range of the total, so one long row is shared by the whole block
// and many short ones do not leave threads idle.
constexpr uint32_t kListCap = 512;

struct RowList {
    uint32_t v[kListCap], a0[kListCap], b0[kListCap], n1[kListCap], off[kListCap + 1];
    uint8_t f[kListCap];
    uint32_t cnt;
    uint32_t wsum[kWaves];
};

// All threads; cnt <= kListCap entries with their counts in off[0 .. cnt).
__device__ __forceinline__ void row_list_scan(RowList &L, uint32_t cnt) {
    const uint32_t j0 = 2 * threadIdx.x;
    const uint32_t l0 = j0 < cnt ? L.off[j0] : 0u, l1 = j0 + 1 < cnt ? L.off[j0 + 1] : 0u;
    const uint32_t sum = l0 + l1;
    const uint32_t incl = wave_incl_scan(sum);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) L.wsum[w] = incl;
    __syncthreads();
    uint32_t base = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kWaves; ++i) {
        base += i < w ? L.wsum[i] : 0u;
        tot += L.wsum[i];
    }
    const uint32_t ex = base + incl - sum;
    if (j0 < cnt) L.off[j0] = ex;
    if (j0 + 1 < cnt) L.off[j0 + 1] = ex + l0;
    if (threadIdx.x == 0) L.off[cnt] = tot;
    __syncthreads();
}

// This thread's contiguous range [e, end) of the list's edges and the entry j
// holding edge e (the last entry whose offset is <= e).
__device__ __forceinline__ void row_list_range(const RowList &L, uint32_t cnt, uint32_t &e, uint32_t &end,
                                               uint32_t &j) {
    const uint32_t T = L.off[cnt];
    const uint32_t chunk = (T + kBlock - 1) / kBlock;
    e = threadIdx.x * chunk;
    end = e + chunk < T ? e + chunk : T;
    uint32_t lo = 0, hi = cnt;  // off[lo] <= e < off[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (L.off[mid] <= e) lo = mid;
        else hi = mid;
    }
    j = lo;
}

__device__ __forceinline__ void flag_state(uint8_t *st, uint32_t v, uint32_t f) {
    atomicOr(reinterpret_cast<uint32_t *>(st + (v & ~3u)), f << (8 * (v & 3u)));
}

// Dirty-set updates along one out-edge (w, v) of a changed vertex w: the IN term of v.
__device__ __forceinline__ void mark_out_edge(const KArgs &a, uint2 ed, bool settled) {
    if (!settled) atomicMin(&a.b.tin[ed.x], (unsigned long long)ed.y);
    else if (a.b.tin[ed.x] == ed.y) flag_state(a.b.st, ed.x, ST_TDIRTY);
}

// Dirty-set updates along one in-edge (u, w) of a changed vertex w: the OUT term of u.
// OUT (full): for an unexplored u whose cursor points at an edge (u, w) to the settled
// w, the candidate c(z, u) + c(u, w) of each in-neighbour z may rise: z is flagged
// where its stored OUT term equals that candidate. The in-row of u goes to the
// block's second list L2 (walked together after the first), or is walked here when
// L2 is full.
template <int OUT_M>
__device__ __forceinline__ void mark_in_edge(const KArgs &a, uint2 ie, bool settled, uint32_t w, RowList *L2) {
    if (!settled) {
        atomicMin(&a.b.tout[ie.x], (unsigned long long)ie.y);
        return;
    }
    if (a.b.tout[ie.x] == ie.y) flag_state(a.b.st, ie.x, ST_TDIRTY);
    if (OUT_M == OUT_FULL_M && (a.b.st[ie.x] & ST_SET) == ST_U) {
        // the lightest non-settled out-edge of the unexplored in-neighbour x rises only if
        // x's cursor points at an edge to w; then every in-neighbour of x is flagged
        const uint32_t c = a.b.out_cur[ie.x];
        if (c < a.g.rp[ie.x + 1]) {
            const uint2 ce = a.g.edges[c];
            if (ce.x != w) return;
            const uint32_t b = a.g.ip[ie.x], end = a.g.ip[ie.x + 1];
            if (b == end) return;
            const uint32_t j = atomicAdd(&L2->cnt, 1u);
            if (j < kListCap) {
                L2->a0[j] = b;
                L2->b0[j] = ce.y;
                L2->off[j] = end - b;
                return;
            }
            for (uint32_t f = b; f < end; ++f) {
                const uint2 ze = a.g.in_edges[f];
                if (a.b.tout[ze.x] == (unsigned long long)ze.y + ce.y) flag_state(a.b.st, ze.x, ST_TDIRTY);
            }
        }
    }
}

template <bool IN_ON, int OUT_M>
__global__ __launch_bounds__(kBlock) void k_mark(KArgs a, int par) {
    __shared__ uint4 s_st[kOwnSpan / 16];
    __shared__ RowList L;
    __shared__ RowList L2[1];  // OUT (full): in-rows to flag
    Ctl *ctl = a.b.ctl;
    const unsigned long long r0 = lane_slot(ctl->reached, 0ull);
    const unsigned long long settled_cnt = ctl->h.settled;
    const uint32_t n = a.g.n;
    const unsigned long long reached = wave_sum64(r0);
    if (reached == settled_cnt) return;
    const uint8_t *sw = reinterpret_cast<const uint8_t *>(s_st);
    for (uint64_t vb = (uint64_t)blockIdx.x * kOwnSpan; vb < n; vb += (uint64_t)gridDim.x * kOwnSpan) {
        const uint64_t v0 = vb + 16u * threadIdx.x;
        uint4 x = make_uint4(0u, 0u, 0u, 0u);
        if (v0 + 16 <= n) {
            x = *reinterpret_cast<const uint4 *>(a.b.st + v0);
        } else if (v0 < n) {
            uint32_t q[4] = {0u, 0u, 0u, 0u};
            for (uint32_t j = 0; v0 + j < n; ++j) q[j >> 2] |= (uint32_t)a.b.st[v0 + j] << (8 * (j & 3));
            x = make_uint4(q[0], q[1], q[2], q[3]);
        }
        const bool any = ((x.x | x.y | x.z | x.w) & 0x80808080u) != 0;
        __syncthreads();  // the previous window's LDS reads are done
        s_st[threadIdx.x] = x;
        if (threadIdx.x == 0) {
            L.cnt = 0;
            if (OUT_M == OUT_FULL_M) L2[0].cnt = 0;
        }
        if (!__syncthreads_or(any)) continue;  // block-uniform
        for (uint32_t r = 0; r < kOwnSpan / kBlock; ++r) {
            const uint32_t i = r * kBlock + threadIdx.x;
            const uint32_t sb = sw[i];
            if (!(sb & ST_CHG)) continue;
            const uint32_t w = (uint32_t)vb + i;
            atomicAnd(reinterpret_cast<uint32_t *>(a.b.st + (w & ~3u)), ~((uint32_t)ST_CHG << (8 * (w & 3u))));
            const bool sett = (sb & ST_SET) == ST_S;
            const uint32_t ob = IN_ON ? a.g.rp[w] : 0u, oe = IN_ON ? a.g.rp[w + 1] : 0u;
            const uint32_t ib = OUT_M ? a.g.ip[w] : 0u, ie = OUT_M ? a.g.ip[w + 1] : 0u;
            const uint32_t len = (oe - ob) + (ie - ib);
            if (len == 0) continue;
            const uint32_t j = atomicAdd(&L.cnt, 1u);
            if (j < kListCap) {
                L.v[j] = w;
                L.f[j] = sett ? 1 : 0;
                L.a0[j] = ib;
                L.b0[j] = ob;
                L.n1[j] = oe - ob;  // the out-edges first
                L.off[j] = len;
                continue;
            }
            for (uint32_t e = ob; e < oe; ++e) mark_out_edge(a, a.g.edges[e], sett);  // list full
            for (uint32_t e = ib; e < ie; ++e) mark_in_edge<OUT_M>(a, a.g.in_edges[e], sett, w, &L2[0]);
        }
        __syncthreads();
        const uint32_t cnt = L.cnt < kListCap ? L.cnt : kListCap;
        if (cnt) {  // block-uniform
            row_list_scan(L, cnt);
            uint32_t e, end, j;
            row_list_range(L, cnt, e, end, j);
            for (; e < end; e += 4) {  // four edges at a time, their loads issued together
                uint32_t jq[4];
                bool outq[4];
                uint2 eq[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    jq[q] = kListCap;
                    outq[q] = false;
                    eq[q] = make_uint2(0u, 0u);
                    if (e + q < end) {
                        while (e + q >= L.off[j + 1]) ++j;
                        const uint32_t k = e + q - L.off[j];
                        jq[q] = j;
                        outq[q] = k < L.n1[j];
                        eq[q] = outq[q] ? a.g.edges[L.b0[j] + k] : a.g.in_edges[L.a0[j] + (k - L.n1[j])];
                    }
                }
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (jq[q] == kListCap) continue;
                    const bool sett = L.f[jq[q]] != 0;
                    if (outq[q]) mark_out_edge(a, eq[q], sett);
                    else mark_in_edge<OUT_M>(a, eq[q], sett, L.v[jq[q]], &L2[0]);
                }
            }
        }
        if (OUT_M == OUT_FULL_M) {  // the in-rows collected in L2, walked together
            __syncthreads();
            const uint32_t cnt2 = L2[0].cnt < kListCap ? L2[0].cnt : kListCap;
            if (cnt2) {  // block-uniform
                row_list_scan(L2[0], cnt2);
                uint32_t e, end, j;
                row_list_range(L2[0], cnt2, e, end, j);
                for (; e < end; ++e) {
                    while (e >= L2[0].off[j + 1]) ++j;
                    const uint2 ze = a.g.in_edges[L2[0].a0[j] + (e - L2[0].off[j])];
                    if (a.b.tout[ze.x] == (unsigned long long)ze.y + L2[0].b0[j]) flag_state(a.b.st, ze.x, ST_TDIRTY);
                }
            }
        }
    }
}

// Dynamic terms over every vertex, one per thread in a grid-stride loop (the
// per-phase learned mode, whose criterion changes from phase to phase).
template <int IN, int OUT>
__device__ __forceinline__ void terms_body(const KArgs &a, int par, unsigned long long *sh) {
    Ctl *ctl = a.b.ctl;
    const int p3 = par % 3;
    __shared__ unsigned long long s_reached, s_minD;
    if (threadIdx.x < 64) {
        const unsigned long long r0 = lane_slot(ctl->reached, 0ull), m0 = lane_slot(ctl->minD[p3], INF64);
        const unsigned long long r = wave_sum64(r0);
        const unsigned long long md = wave_min64(m0);
        if (threadIdx.x == 0) { s_reached = r; s_minD = md; }
    }
    __syncthreads();
    if (s_reached == ctl->h.settled) return;
    const unsigned long long minD = s_minD;
    unsigned long long tmin = INF64;
    const uint32_t n = a.g.n;
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const uint8_t s = a.b.st[v];
        if ((s & ST_SET) != ST_F) continue;
        unsigned long long tv;
        const bool ok = vertex_terms<IN, OUT>(a, v, a.b.dist[v], minD, tv);
        if (IN != IN_NONE) a.b.st[v] = ok ? (uint8_t)(ST_F | ST_INOK) : (uint8_t)ST_F;
        tmin = umin64(tmin, tv);
    }
    if (OUT != OUT_NONE) {
        block_reduce<kWaves, 1u, 1u>(&tmin, sh);
        if (threadIdx.x == 0 && tmin != INF64) atomicMin(slot_of(ctl->tdyn[p3], my_shard()), tmin);
    }
}

// Trace mode: the dynamic terms of the selector's criteria on the same
// snapshot: the IN-SIMPLE result goes to state bit 2, OUT-SIMPLE's threshold
// to tdyn (IN-SIMPLE|OUT-STATIC reuses both halves).
__global__ __launch_bounds__(kBlock) void k_terms_trace(KArgs a, int par) {
    __shared__ unsigned long long sh[8 * kWaves];
    Ctl *ctl = a.b.ctl;
    const int p3 = par % 3;
    const unsigned long long r0 = lane_slot(ctl->reached, 0ull), m0 = lane_slot(ctl->minD[p3], INF64);
    const unsigned long long settled = ctl->h.settled;
    const unsigned long long reached = wave_sum64(r0);
    if (reached == settled) return;
    const unsigned long long minD = wave_min64(m0);
    unsigned long long ts = INF64;
    const uint32_t n = a.g.n;
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const uint8_t s = a.b.st[v];
        if ((s & ST_SET) != ST_F) continue;
        const unsigned long long dv = a.b.dist[v];
        const unsigned long long ins = cursor_term(a.b.in_cur, a.b.in_head, a.g.in_edges, a.g.ip, v, a.b.st);
        const unsigned long long outs = cursor_term(a.b.out_cur, a.b.out_head, a.g.edges, a.g.rp, v, a.b.st);
        a.b.st[v] = (uint8_t)(ST_F | (dv <= sadd64(minD, ins) ? ST_INOK : 0));
        ts = umin64(ts, sadd64(dv, outs));
    }
    block_reduce<kWaves, 1u, 1u>(&ts, sh);
    if (threadIdx.x == 0 && ts != INF64) atomicMin(slot_of(ctl->tdyn[p3], my_shard()), ts);
}

// Approximate criteria (Section 3, closing paragraphs): per queued vertex the
// IN value (minimum over in-edges (w,v): c for w queued, c + minIn(w) for w
// unexplored) and the OUTWEAK value (out-edges (v,w): c for w queued, c +
// minOut(w) for w unexplored), maintained conservatively: a neighbour's move
// U -> F lowers the value at once, a move F -> S only counts as a change, and a
// vertex evaluated with k or more counted changes recomputes from this phase's
// state (k = 0: never). Evaluated here in closed form from the settle phase of
// each neighbour: the kept value equals the exact one except that neighbours
// settled after the vertex's last recomputation (phase index L) still count as
// queued, and the counted changes are exactly those edges. One pass over the row
// gives both the exact minimum and the stale terms; a recomputation sets L to
// this phase's index (every settled vertex settled in a phase <= it).
template <bool IN_ON, bool OUT_ON>
__global__ __launch_bounds__(kBlock) void k_terms_approx(KArgs a, int par) {
    __shared__ unsigned long long sh[8 * kWaves];
    Ctl *ctl = a.b.ctl;
    const int p2 = par & 1, p3 = par % 3;
    __shared__ unsigned long long s_reached, s_minD;
    const unsigned int P = ctl->h.pnum[p2];
    if (threadIdx.x < 64) {
        const unsigned long long r0 = lane_slot(ctl->reached, 0ull), m0 = lane_slot(ctl->minD[p3], INF64);
        const unsigned long long r = wave_sum64(r0);
        const unsigned long long md = wave_min64(m0);
        if (threadIdx.x == 0) { s_reached = r; s_minD = md; }
    }
    __syncthreads();
    if (s_reached == ctl->h.settled) return;
    const unsigned long long minD = s_minD;
    const uint32_t k = a.approx_k;
    unsigned long long tmin = INF64;
    const uint32_t n = a.g.n;
    for (uint32_t v = blockIdx.x * kBlock + threadIdx.x; v < n; v += gridDim.x * kBlock) {
        const uint8_t s = a.b.st[v];
        if ((s & ST_SET) != ST_F) continue;
        const unsigned long long dv = a.b.dist[v];
        if (IN_ON) {
            const uint32_t L = a.b.apx_lin[v];
            unsigned long long exact = INF64, stale = INF64;
            uint32_t changes = 0;
            const uint32_t end = a.g.ip[v + 1];
            for (uint32_t e = a.g.ip[v]; e < end; ++e) {
                const uint2 ie = a.g.in_edges[e];
                const uint8_t sw = a.b.st[ie.x] & ST_SET;
                if (sw == ST_F) exact = umin64(exact, ie.y);
                else if (sw == ST_U) exact = umin64(exact, sadd64(ie.y, min_in_u64(a.g.vmin[ie.x].x, a.g.wmax, a.g.ip, ie.x)));
                else if (a.b.apx_sp[ie.x] > L) { stale = umin64(stale, ie.y); ++changes; }
            }
            const bool recompute = k && changes >= k;
            if (recompute) a.b.apx_lin[v] = P;
            const unsigned long long term = recompute ? exact : umin64(exact, stale);
            a.b.st[v] = dv <= sadd64(minD, term) ? (uint8_t)(ST_F | ST_INOK) : (uint8_t)ST_F;
        }
        if (OUT_ON) {
            const uint32_t L = a.b.apx_lout[v];
            unsigned long long exact = INF64, stale = INF64;
            uint32_t changes = 0;
            const uint32_t end = a.g.rp[v + 1];
            for (uint32_t e = a.g.rp[v]; e < end; ++e) {
                const uint2 ed = a.g.edges[e];
                const uint8_t sx = a.b.st[ed.x] & ST_SET;
                if (sx == ST_F) exact = umin64(exact, ed.y);
                else if (sx == ST_U) exact = umin64(exact, sadd64(ed.y, min_out64(a.g.vmin[ed.x].y, a.g.wmax, a.g.rp, ed.x)));
                else if (a.b.apx_sp[ed.x] > L) { stale = umin64(stale, ed.y); ++changes; }
            }
            const bool recompute = k && changes >= k;
            if (recompute) a.b.apx_lout[v] = P;
            tmin = umin64(tmin, sadd64(dv, recompute ? exact : umin64(exact, stale)));
        }
    }
    if (OUT_ON) {
        block_reduce<kWaves, 1u, 1u>(&tmin, sh);
        if (threadIdx.x == 0 && tmin != INF64) atomicMin(slot_of(ctl->tdyn[p3], my_shard()), tmin);
    }
}

// Learned mode: the term pass of the criterion the selector chose for this phase.
__global__ __launch_bounds__(kBlock) void k_terms_learned(KArgs a, int par) {
    __shared__ unsigned long long sh[8 * kWaves];
    const unsigned int c = a.b.ctl->h.choice[par & 1];
    if (c == 1) terms_body<IN_SIMPLE_M, OUT_SIMPLE_M>(a, par, sh);
    else if (c == 2) terms_body<IN_SIMPLE_M, OUT_NONE>(a, par, sh);
}

// ---------------------------------------------------------------------------
// identify (phased)

// Start of an identify pass, every block: with F empty (reached == settled)
// block 0 marks the solve done, and the caller returns.
__device__ __forceinline__ bool phase_done(Ctl *ctl, int p2, unsigned int P, unsigned long long reached,
                                           unsigned long long settled) {
    if (reached != settled) return false;
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            ctl->h.done = 1;
            ctl->h.pnum[p2 ^ 1] = P;
        }
        shard_fill(ctl->spack[p2 ^ 1], 0);
        shard_fill(ctl->szero[p2 ^ 1], 0);
    }
    return true;
}

// Start of a non-empty phase, block 0 only: header counters, the trace record
// and the control slots that the next phases fill.
template <bool LEARN, bool TRACE>
__device__ __forceinline__ void phase_open(const KArgs &a, Ctl *ctl, int p2, int p3, unsigned int P,
                                           unsigned long long reached, unsigned long long settled,
                                           unsigned long long minD, unsigned long long dgall) {
    if (threadIdx.x == 0) {
        ctl->h.pnum[p2 ^ 1] = P + 1;
        ctl->h.phases = P + 1;
        ctl->h.sum_f += reached - settled;
        if (LEARN) {
            ctl->h.fprev = ctl->h.fk;
            ctl->h.dgk = dgall - ctl->h.m_reach;
        }
        ctl->h.fk = reached - settled;
        ctl->h.s_k = settled;
        ctl->h.m_k = ctl->h.m_reach;
        if (P < a.b.trace_cap) {
            PhaseRec r;
            r.min_d = minD;
            r.fringe = (unsigned int)(reached - settled);
            r.settled = 0;
            r.criterion = LEARN ? kChoiceCrit[ctl->h.choice[p2]] : a.crit;
            r.edges = 0;
            a.b.trace[P] = r;
        }
    }
    shard_fill(ctl->spack[p2 ^ 1], 0);
    shard_fill(ctl->szero[p2 ^ 1], 0);
    shard_fill(ctl->minD[(p3 + 2) % 3], INF64);
    shard_fill(ctl->tst[(p3 + 2) % 3], INF64);
    shard_fill(ctl->tdyn[(p3 + 1) % 3], INF64);
    if (LEARN) {
        shard_fill(ctl->sumd[(p3 + 2) % 3], 0);
        shard_fill(ctl->nin[p2 ^ 1], 0);
        shard_fill(ctl->nout[p2 ^ 1], 0);
    }
    if (TRACE) {
        for (int c = 0; c < 3; ++c) shard_fill(ctl->cnt_cf[(p2 ^ 1) * 3 + c], 0);
    }
}

// IN: IN_NONE, IN_DIJK, IN_STATIC_M, 3 = "flag from the term pass", or
// kInOracle = the clairvoyant criterion d[v] = dist(s, v) against a reference.
// OUT: 0 none, 1 static threshold, 2 threshold from the term pass.
// Each lane owns four consecutive vertices per step: one 32-bit state load,
// then the distance / minima loads of all its queued vertices in flight at once.
// LEARN: also count the queued vertices passing each static test, fold the
// sum of kept distances and always fold the OUT-STATIC threshold (features).
// TRACE: evaluate all three criteria (flags / thresholds from k_terms_trace),
// count what each certifies, settle what the phase's chosen one certifies.
template <int IN, int OUT, int CH, bool LEARN, bool TRACE = false>
__device__ __forceinline__ void identify_body(const KArgs &a, int par, unsigned long long *sh, AppendLds &L) {
    Ctl *ctl = a.b.ctl;
    const int p2 = par & 1, p3 = par % 3;
    if (threadIdx.x == 0) { L.cnt = 0; L.filled = 0; L.zero = 0; }
    // every wavefront combines the sharded phase-start values itself (no block barrier)
    const unsigned long long r0 = lane_slot(ctl->reached, 0ull), m0 = lane_slot(ctl->minD[p3], INF64);
    const unsigned long long t0 = OUT == 1 ? lane_slot(ctl->tst[p3], INF64) : OUT == 2 ? lane_slot(ctl->tdyn[p3], INF64) : 0ull;
    const unsigned long long st0 = LEARN ? lane_slot(ctl->tst[p3], INF64) : 0ull;
    const unsigned long long dg0 = LEARN && blockIdx.x == 0 ? lane_slot(ctl->degsum, 0ull) : 0ull;
    const unsigned long long si0 = TRACE ? lane_slot(ctl->tdyn[p3], INF64) : 0ull;
    const unsigned long long settled = ctl->h.settled;
    const unsigned int P = ctl->h.pnum[p2];
    const unsigned int choice = TRACE ? ctl->h.choice[p2] : 0u;
    const unsigned long long reached = wave_sum64(r0);
    const unsigned long long minD = wave_min64(m0);
    const unsigned long long T = OUT ? wave_min64(t0) : 0ull;
    if (phase_done(ctl, p2, P, reached, settled)) return;
    if (blockIdx.x == 0) {
        // learned mode: sum over F of out-degrees = degrees of all ever queued minus those settled
        const unsigned long long dgall = LEARN ? wave_sum64(dg0) : 0ull;
        phase_open<LEARN, TRACE>(a, ctl, p2, p3, P, reached, settled, minD, dgall);
    }
    __syncthreads();  // LDS counters initialised
    unsigned long long fmin = INF64, ftst = INF64, fsum = 0, cin = 0, cout = 0, cc[3] = {0, 0, 0};
    const unsigned long long Tst = LEARN ? wave_min64(st0) : 0ull;
    const unsigned long long Tsi = TRACE ? wave_min64(si0) : 0ull;
    const uint32_t n = a.g.n;
    const uint32_t nq = (n + 3) / 4;  // lane q takes vertices 4q .. 4q+3
    constexpr bool kMinima = LEARN || IN == IN_STATIC_M || OUT == 1;
    // With at least a quarter of the vertices queued nearly every line of d and
    // (minIn, minOut) holds a queued vertex and is fetched anyway: then a lane
    // loads its four words of each with 16-byte loads issued together with the
    // state word, instead of after it.
    const bool dense = (reached - settled) * 4 >= (unsigned long long)n &&
                       (reinterpret_cast<uintptr_t>(a.b.dist) & 15) == 0;
    for (uint32_t base = blockIdx.x * kBlock; base < nq; base += gridDim.x * kBlock) {
        const uint32_t q = base + threadIdx.x;
        const uint32_t v0 = 4 * q;
        const uint32_t s4 = q < nq ? load_st4(a.b.st, q, n) : 0u;
        unsigned long long dv[4];
        uint2 mm[4];
        if (dense && v0 + 4 <= n) {
            const ulonglong2 *dp = reinterpret_cast<const ulonglong2 *>(a.b.dist + v0);
            const ulonglong2 d01 = dp[0], d23 = dp[1];
            dv[0] = d01.x; dv[1] = d01.y; dv[2] = d23.x; dv[3] = d23.y;
            if (kMinima) {
                const uint4 *mp = reinterpret_cast<const uint4 *>(a.g.vmin + v0);
                const uint4 m01 = mp[0], m23 = mp[1];
                mm[0] = make_uint2(m01.x, m01.y); mm[1] = make_uint2(m01.z, m01.w);
                mm[2] = make_uint2(m23.x, m23.y); mm[3] = make_uint2(m23.z, m23.w);
            }
        } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                dv[i] = INF64;
                mm[i] = make_uint2(INF32, INF32);
                if (((s4 >> (8 * i)) & ST_SET) == ST_F) {
                    dv[i] = a.b.dist[v0 + i];
                    if (kMinima) mm[i] = a.g.vmin[v0 + i];
                }
            }
        }
        uint32_t sm = 0;  // settled now, bit i = vertex v0 + i
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint8_t s = (uint8_t)(s4 >> (8 * i));
            if ((s & ST_SET) != ST_F) continue;
            if (LEARN) {
                cin += dv[i] <= sadd64(minD, min_in_test(mm[i].x)) ? 1 : 0;
                cout += dv[i] <= Tst ? 1 : 0;
            }
            bool ok = false;
            if (TRACE) {
                const bool c0 = dv[i] <= sadd64(minD, min_in_test(mm[i].x)) || dv[i] <= Tst;
                const bool c1 = (s & ST_INOK) != 0 || dv[i] <= Tsi;
                const bool c2 = (s & ST_INOK) != 0 || dv[i] <= Tst;
                cc[0] += c0;
                cc[1] += c1;
                cc[2] += c2;
                ok = choice == 0 ? c0 : choice == 1 ? c1 : c2;
            } else {
                if (IN == IN_DIJK) ok = dv[i] == minD;
                else if (IN == IN_STATIC_M) ok = dv[i] <= sadd64(minD, min_in_test(mm[i].x));
                else if (IN == 3) ok = (s & ST_INOK) != 0;
                else if (IN == kInOracle) ok = dv[i] == a.ref[v0 + i];  // Section 3: ORACLE(v)
                if (OUT != 0) ok = ok || dv[i] <= T;
            }
            if (ok) {
                sm |= 1u << i;
            } else {
                fmin = umin64(fmin, dv[i]);
                if (LEARN || OUT == 1) ftst = umin64(ftst, sadd64(dv[i], min_out64(mm[i].y, a.g.wmax, a.g.rp, v0 + i)));
                if (LEARN) fsum += dv[i];
            }
        }
        uint32_t row[4], deg[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) row[i] = deg[i] = 0;
        if (sm) {  // row pointers of the four vertices in one batch
            if (v0 + 4 <= n) {
                const uint4 r = *reinterpret_cast<const uint4 *>(a.g.rp + v0);
                const uint32_t r4 = a.g.rp[v0 + 4];
                row[0] = r.x; row[1] = r.y; row[2] = r.z; row[3] = r.w;
                deg[0] = r.y - r.x; deg[1] = r.z - r.y; deg[2] = r.w - r.z; deg[3] = r4 - r.w;
            } else {
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (v0 + i < n) {
                        row[i] = a.g.rp[v0 + i];
                        deg[i] = a.g.rp[v0 + i + 1] - row[i];
                    }
            }
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if ((sm >> i) & 1u) {
                    a.b.st[v0 + i] = (uint8_t)(ST_S | (a.mark ? ST_CHG : 0));
                    a.b.dist[v0 + i] = dv[i] | kSettledBit;
                    if (a.b.phase_of) a.b.phase_of[v0 + i] = P + 1;
                }
        }
        append_settled_n<CH, 4>(a, ctl, p2, L, sm, row, deg, dv);
    }
    append_flush<CH>(a, ctl, p2, L);
    // [0] fmin, [1] ftst, [2] fsum, [3] cin, [4] cout, [5..7] per-criterion counts
    unsigned long long v[8] = {fmin, ftst, fsum, cin, cout, cc[0], cc[1], cc[2]};
    constexpr unsigned kAct = TRACE ? 0xffu : LEARN ? 0x1fu : OUT == 1 ? 0x3u : 0x1u;
    block_reduce<kWaves, kAct, 0x3u, 0xf8u>(v, sh);
    fmin = v[0];
    ftst = v[1];
    fsum = v[2];
    cin = v[3];
    cout = v[4];
    if (TRACE && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c)
            if (v[5 + c]) atomicAdd(slot_of(ctl->cnt_cf[p2 * 3 + c], my_shard()), v[5 + c]);
    if (threadIdx.x == 0) {
        if (fmin != INF64) atomicMin(slot_of(ctl->minD[(p3 + 1) % 3], my_shard()), fmin);
        if (ftst != INF64) atomicMin(slot_of(ctl->tst[(p3 + 1) % 3], my_shard()), ftst);
        if (LEARN) {
            if (fsum) atomicAdd(slot_of(ctl->sumd[(p3 + 1) % 3], my_shard()), fsum);
            if (cin) atomicAdd(slot_of(ctl->nin[p2], my_shard()), cin);
            if (cout) atomicAdd(slot_of(ctl->nout[p2], my_shard()), cout);
        }
    }
}

template <int IN, int OUT, int CH>
__global__ __launch_bounds__(kBlock) void k_identify(KArgs a, int par) {
    __shared__ unsigned long long sh[8 * kWaves];
    __shared__ AppendLds L;
    identify_body<IN, OUT, CH, false>(a, par, sh, L);
}

template <int CH>
__global__ __launch_bounds__(kBlock) void k_identify_trace(KArgs a, int par) {
    __shared__ unsigned long long sh[8 * kWaves];
    __shared__ AppendLds L;
    identify_body<IN_STATIC_M, 1, CH, true, true>(a, par, sh, L);
}

// Learned mode: identify with the criterion the selector chose for this phase.
template <int CH>
__global__ __launch_bounds__(kBlock) void k_identify_learned(KArgs a, int par) {
    __shared__ unsigned long long sh[8 * kWaves];
    __shared__ AppendLds L;
    if (a.b.ctl->h.choice[par & 1] == 0) identify_body<IN_STATIC_M, 1, CH, true>(a, par, sh, L);
    else if (a.b.ctl->h.choice[par & 1] == 1) identify_body<3, 2, CH, true>(a, par, sh, L);
    else identify_body<3, 1, CH, true>(a, par, sh, L);  // IN-SIMPLE flag or the OUT-STATIC threshold
}

// ---------------------------------------------------------------------------
// identify over queue arrays (static criteria)

constexpr unsigned long long kTomb = INF64;  // queue entry whose vertex has settled
constexpr uint32_t kQWin = 4 * kOwnSpan;     // most vertices a scan block may own (state window in LDS)

// Queue-array identify (IN: IN_NONE, IN_DIJK, IN_STATIC_M, or 3 = the dynamic
// IN flag in the state byte; OUT: 0, 1 = OUT-STATIC threshold, 2 = the dynamic
// OUT threshold). With a dynamic criterion, k_terms_win has evaluated the
// phase's terms over the same entries before this launch.
// Scan block b owns the vertices kOwnSpan * (k * G + b) + [0, kOwnSpan),
// k = 0, 1, ... (G blocks), and keeps an entry (d, v, minIn, minOut, row start,
// out-degree) for each of them that is queued, in slots [b * qspan, (b + 1) *
// qspan): a phase reads those entries, 28 bytes per queued vertex, and the state
// bytes of the block's vertices, instead of the distance and minima of every
// vertex; settling an entry's vertex reads no row pointers. Relax flags a
// vertex it discovers ST_QNEW and one whose distance it lowers ST_QDIRTY; the
// owner gathers a new vertex's distance and minima once and gives it an entry
// if it stays queued, and reloads a dirty entry's distance, so an entry holds
// its vertex's distance at phase start. The new vertices' loads are issued before
// the entries' (the two are independent), so that a phase waits for one round of
// loads for both. A settled entry becomes a tombstone; a
// block whose slots hold more than a quarter of tombstones moves its live
// entries down over them. Each vertex gets at most one entry, so a block's
// slots never overflow.
// With 3/8 or more of the vertices queued the entries cost about as much as
// the dense scan (measured on random graphs), so such phases run the dense scan
// (identify_body) and leave the arrays stale; the next queue phase rebuilds
// them from the state bytes, as the first phase of a solve does. The switch
// back waits until F is below 3/10 of the vertices, so that F sizes near the
// threshold do not rebuild every other phase. Every block takes the same
// decision from the phase-start counters.
//
// KEYED (launch option queue = 2; the paper's keyed queues of Section 5 in one
// partition): a block's entries hold only the queued vertices whose IN-STATIC
// key d - minIn is at most a grid-wide split; the others carry ST_QFAR in their
// state byte and are not read. Every vertex the criteria certify has key <= X,
// X = the OUT-STATIC threshold T when OUT-STATIC is on (d <= T gives key <= T,
// and minD <= T), else minD; the vertices attaining minD and T have key <= X as
// well. So while the split is >= X, the entries alone certify the phase and fold
// the next thresholds exactly: a far vertex has d >= key > split >= X. Relax
// flags the far vertices it lowers; their owner moves those whose key fell to
// the split into its entries. When the folded threshold of a launch exceeds the
// split, that launch is a rebuild and not a phase: every block gathers all its
// queued vertices, enters those with key <= X + margin (the new split), marks
// the rest far, and folds the exact minD and T over all of them; relax skips
// it and the next launch runs the phase. The margin is kSplitPhases times the
// threshold's advance per phase since the previous rebuild.
constexpr unsigned long long kSplitPhases = 20;

template <int IN, int OUT, int CH, bool KEYED = false>
__global__ __launch_bounds__(kBlock) void k_identify_queue(KArgs a, int par) {
    static_assert(!KEYED || (IN <= IN_STATIC_M && OUT <= 1), "keyed queue arrays take static criteria only");
    __shared__ unsigned long long sh[8 * kWaves];
    __shared__ AppendLds L;
    __shared__ uint32_t s_wk[kWaves];  // compaction: entries each wavefront keeps in one step
    __shared__ uint32_t s_app;         // entries appended to this block's slots in this pass
    __shared__ uint4 s_st[kQWin / 16]; // state bytes of the block's vertices
    __shared__ uint16_t s_need[kBlock * 16];  // per wavefront: its window vertices that need an entry
    Ctl *ctl = a.b.ctl;
    const int p2 = par & 1, p3 = par % 3;
    const unsigned long long r0 = lane_slot(ctl->reached, 0ull), m0 = lane_slot(ctl->minD[p3], INF64);
    const unsigned long long t0 = OUT == 1 ? lane_slot(ctl->tst[p3], INF64) : OUT == 2 ? lane_slot(ctl->tdyn[p3], INF64) : 0ull;
    const unsigned long long settled = ctl->h.settled;
    const unsigned int live = ctl->h.qlive[p2];
    const unsigned int P = ctl->h.pnum[p2];
    const uint32_t n = a.g.n, b = blockIdx.x, G = gridDim.x;
    const uint32_t cnt_l = a.b.qcnt[2 * b], tomb_l = a.b.qcnt[2 * b + 1];
    const unsigned long long ksplit = KEYED ? ctl->h.qsplit[p2] : 0ull, kdelta = KEYED ? ctl->h.qdelta[p2] : 0ull;
    const unsigned long long kxrep = KEYED ? ctl->h.qxrep[p2] : 0ull;
    const unsigned int kprep = KEYED ? ctl->h.qprep[p2] : 0u;
    // the block's state bytes (window w = its w-th grid step, at most four) are loaded
    // now, with the control slots, and written to LDS once the phase is known to run
    const uint32_t span = a.b.qspan;
    const uint64_t rb = (uint64_t)b * span;
    unsigned long long *qd = a.b.qd + rb;
    uint32_t *qv = a.b.qv + rb;
    uint2 *qm = a.b.qm + rb;
    uint2 *qr = a.b.qr + rb;
    uint4 win[kQWin / kOwnSpan];
#pragma unroll
    for (uint32_t w = 0; w < kQWin / kOwnSpan; ++w) {
        win[w] = make_uint4(0u, 0u, 0u, 0u);
        if (w * kOwnSpan >= span) continue;
        const uint64_t v0 = (uint64_t)kOwnSpan * ((uint64_t)w * G + b) + 16u * threadIdx.x;
        if (v0 + 16 <= n) {
            win[w] = *reinterpret_cast<const uint4 *>(a.b.st + v0);
        } else if (v0 < n) {
            uint32_t q[4] = {0u, 0u, 0u, 0u};
            for (uint32_t j = 0; v0 + j < n; ++j) q[j >> 2] |= (uint32_t)a.b.st[v0 + j] << (8 * (j & 3));
            win[w] = make_uint4(q[0], q[1], q[2], q[3]);
        }
    }
    const unsigned long long reached = wave_sum64(r0);
    const unsigned long long nf = reached - settled;
    const bool dense = !KEYED && (live ? nf * 8 >= 3ull * n : nf * 10 >= 3ull * n);  // grid-uniform
    if (dense) {
        if (b == 0 && threadIdx.x == 0 && nf) ctl->h.qlive[p2 ^ 1] = 0;
        identify_body<IN, OUT, CH, false>(a, par, sh, L);
        return;
    }
    if (threadIdx.x == 0) { L.cnt = 0; L.filled = 0; L.zero = 0; s_app = 0; }
    const unsigned long long minD = wave_min64(m0);
    const unsigned long long T = OUT ? wave_min64(t0) : 0ull;
    if (phase_done(ctl, p2, P, reached, settled)) return;
    // keyed: a rebuild when the entries are not current or the threshold passed the split
    const unsigned long long X = OUT == 1 ? T : minD;
    const bool rebuild = KEYED && (!live || X > ksplit);  // grid-uniform
    unsigned long long split = ksplit;
    if (rebuild) {
        unsigned long long margin = kdelta;
        if (live && P > kprep && X > kxrep) {
            const unsigned long long rate = (X - kxrep) / (P - kprep);
            margin = rate > INF64 / kSplitPhases ? INF64 : rate * kSplitPhases;
            if (margin < 1) margin = 1;
        }
        split = sadd64(X, margin);
        if (b == 0) {
            if (threadIdx.x == 0) {
                ctl->h.repart[p2] = 1;
                ctl->h.qrebuilds += 1;
                ctl->h.pnum[p2 ^ 1] = P;  // the next launch runs phase P
                ctl->h.qsplit[p2 ^ 1] = split;
                ctl->h.qdelta[p2 ^ 1] = margin;
                ctl->h.qxrep[p2 ^ 1] = X;
                ctl->h.qprep[p2 ^ 1] = P;
                ctl->h.qlive[p2 ^ 1] = 1;
            }
            // the slots the next launch (phase P) clears in a phase: its S' counters and the
            // fold slots of the phase after it (this launch folds phase P's exact thresholds)
            shard_fill(ctl->spack[p2 ^ 1], 0);
            shard_fill(ctl->szero[p2 ^ 1], 0);
            shard_fill(ctl->minD[(p3 + 2) % 3], INF64);
            shard_fill(ctl->tst[(p3 + 2) % 3], INF64);
        }
    } else if (b == 0) {
        phase_open<false, false>(a, ctl, p2, p3, P, reached, settled, minD, 0ull);
        if (threadIdx.x == 0) {
            ctl->h.qlive[p2 ^ 1] = 1;
            if (KEYED) {
                ctl->h.repart[p2] = 0;
                ctl->h.qsplit[p2 ^ 1] = ksplit;
                ctl->h.qdelta[p2 ^ 1] = kdelta;
                ctl->h.qxrep[p2 ^ 1] = kxrep;
                ctl->h.qprep[p2 ^ 1] = kprep;
            }
        }
    }
    const uint32_t cnt0 = live && !rebuild ? cnt_l : 0u, tomb0 = live && !rebuild ? tomb_l : 0u;
    // state bytes of the block's vertices into LDS
#pragma unroll
    for (uint32_t w = 0; w < kQWin / kOwnSpan; ++w)
        if (w * kOwnSpan < span) s_st[w * kBlock + threadIdx.x] = win[w];
    __syncthreads();  // LDS counters and state window ready
    const uint8_t *sw = reinterpret_cast<const uint8_t *>(s_st);
    auto win_of = [&](uint32_t v) {  // LDS index of an owned vertex's state byte
        const uint32_t step = ((v / kOwnSpan) - b) / G;
        return step * kOwnSpan + (v % kOwnSpan);
    };
    unsigned long long fmin = INF64, ftst = INF64, ntomb = 0;
    auto certified = [&](unsigned long long d, uint2 mm, uint32_t sb) {
        bool ok = false;
        if (IN == IN_DIJK) ok = d == minD;
        else if (IN == IN_STATIC_M) ok = d <= sadd64(minD, min_in_test(mm.x));  // eq. crit:instatic
        else if (IN == 3) ok = (sb & ST_INOK) != 0;                     // the term pass's IN result
        if (OUT != 0) ok = ok || d <= T;                                // eq. crit:outstatic, or dynamic
        return ok;
    };
    auto settle = [&](uint32_t v, unsigned long long d) {
        a.b.st[v] = (uint8_t)(ST_S | (a.mark ? ST_CHG : 0));
        a.b.dist[v] = d | kSettledBit;
        if (a.b.phase_of) a.b.phase_of[v] = P + 1;
    };
    // 2a. vertices that need an entry: new ones, or (rebuild) every queued one, read from
    // the LDS state window (sixteen per lane). Keyed: also far vertices whose distance
    // dropped; a vertex stays far (no entry, no fold) while its key exceeds the split,
    // except in a rebuild, which folds every queued vertex and certifies none. A
    // wavefront lists its window's such vertices in LDS, so that each round gives every
    // lane one of them, and issues the loads of its first round now, before the entries:
    // they are independent of them (no entry holds a vertex that needs one).
    const int lane = threadIdx.x & 63;
    const bool gather_all = KEYED ? rebuild : !live;
    auto in_key = [&](unsigned long long d, uint2 mm) {  // d - minIn, floored at 0 (eq. crit:instatic)
        const unsigned long long mi = min_in_test(mm.x);
        return d > mi ? d - mi : 0ull;
    };
    constexpr uint32_t kWin = kQWin / kOwnSpan;
    const uint32_t wo = 1024u * (threadIdx.x >> 6);  // the wavefront's first vertex in a window
    uint16_t *need = s_need + wo;
    auto need_mask = [&](uint32_t w) {  // bit j: vertex 16 * threadIdx.x + j of window w
        const uint4 x = s_st[w * kBlock + threadIdx.x];
        const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
        uint32_t nm = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const uint32_t sb = (xs[q] >> (8 * j)) & 0xffu;
                const bool nd = gather_all ? (sb & ST_SET) == ST_F
                                : KEYED ? (sb & ST_QNEW) != 0 || (sb & (ST_QDIRTY | ST_QFAR)) == (ST_QDIRTY | ST_QFAR)
                                        : (sb & ST_QNEW) != 0;
                if (nd) nm |= 1u << (4 * q + j);
            }
        return nm;
    };
    auto list_need = [&](uint32_t nm) {  // wavefront-uniform; returns the list's length
        const uint32_t c = (uint32_t)__popc(nm);
        const uint32_t incl = wave_incl_scan(c);
        const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
        if (tot != 0) {
            __builtin_amdgcn_wave_barrier();  // earlier reads of the list come first
            for (uint32_t o = incl - c, bits = nm; bits; bits &= bits - 1)
                need[o++] = (uint16_t)(16 * lane + __ffs(bits) - 1);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        return tot;
    };
    struct Gathered {
        uint32_t v, row, deg;
        unsigned long long d;
        uint2 mm;
    };
    auto gather = [&](uint64_t wv0, uint32_t off) {
        Gathered g;
        g.v = (uint32_t)(wv0 + off);
        g.d = a.b.dist[g.v];
        g.mm = a.g.vmin[g.v];
        g.row = a.g.rp[g.v];
        g.deg = a.g.rp[g.v + 1] - g.row;
        return g;
    };
    uint32_t nmw[kWin], totw[kWin], offw[kWin];
    Gathered gw[kWin];
#pragma unroll
    for (uint32_t w = 0; w < kWin; ++w) {
        nmw[w] = totw[w] = offw[w] = 0;
        gw[w] = Gathered{0u, 0u, 0u, INF64, make_uint2(INF32, INF32)};
        const uint64_t wv0 = (uint64_t)kOwnSpan * ((uint64_t)w * G + b) + wo;
        if (w * kOwnSpan >= span || wv0 >= n) continue;  // wavefront-uniform
        nmw[w] = need_mask(w);
        totw[w] = list_need(nmw[w]);
        if ((uint32_t)lane < totw[w]) {
            offw[w] = need[lane];
            gw[w] = gather(wv0, offw[w]);
        }
    }
    // 1. the block's entries, four consecutive ones per lane
    const bool compact = tomb0 * 4u > cnt0;  // block-uniform
    uint32_t kept = 0;                       // compaction: entries kept so far
    for (uint32_t i0 = 0; i0 < cnt0; i0 += 4 * kBlock) {
        const uint32_t i = i0 + 4 * threadIdx.x;
        unsigned long long d[4];
        uint32_t v[4];
        uint2 mm[4], rr[4];  // rr: (row start, out-degree)
        if (i + 4 <= cnt0) {
            const ulonglong2 *dp = reinterpret_cast<const ulonglong2 *>(qd + i);
            const uint4 *mp = reinterpret_cast<const uint4 *>(qm + i);
            const uint4 *rp4 = reinterpret_cast<const uint4 *>(qr + i);
            const ulonglong2 d01 = dp[0], d23 = dp[1];
            const uint4 vv = *reinterpret_cast<const uint4 *>(qv + i);
            const uint4 m01 = mp[0], m23 = mp[1], r01 = rp4[0], r23 = rp4[1];
            d[0] = d01.x; d[1] = d01.y; d[2] = d23.x; d[3] = d23.y;
            v[0] = vv.x; v[1] = vv.y; v[2] = vv.z; v[3] = vv.w;
            mm[0] = make_uint2(m01.x, m01.y); mm[1] = make_uint2(m01.z, m01.w);
            mm[2] = make_uint2(m23.x, m23.y); mm[3] = make_uint2(m23.z, m23.w);
            rr[0] = make_uint2(r01.x, r01.y); rr[1] = make_uint2(r01.z, r01.w);
            rr[2] = make_uint2(r23.x, r23.y); rr[3] = make_uint2(r23.z, r23.w);
        } else {
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                d[j] = kTomb;
                v[j] = 0;
                mm[j] = rr[j] = make_uint2(INF32, 0u);
                if (i + j < cnt0) {
                    d[j] = qd[i + j];
                    v[j] = qv[i + j];
                    mm[j] = qm[i + j];
                    rr[j] = qr[i + j];
                }
            }
        }
        // entries whose distance a relax lowered: reload it, clear the flag
        uint32_t sbj[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            sbj[j] = d[j] != kTomb ? sw[win_of(v[j])] : 0u;
            if (sbj[j] & ST_QDIRTY) {
                d[j] = a.b.dist[v[j]];
                if (!compact) qd[i + j] = d[j];
                a.b.st[v[j]] = ST_F;
            }
        }
        uint32_t sm = 0, keep = 0;
        uint32_t row[4], deg[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            row[j] = deg[j] = 0;
            if (d[j] == kTomb) continue;
            row[j] = rr[j].x;
            deg[j] = rr[j].y;
            if (certified(d[j], mm[j], sbj[j])) {
                sm |= 1u << j;
            } else {
                keep |= 1u << j;
                fmin = umin64(fmin, d[j]);
                if (OUT == 1) ftst = umin64(ftst, sadd64(d[j], min_out64(mm[j].y, a.g.wmax, a.g.rp, v[j])));
            }
        }
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if ((sm >> j) & 1u) settle(v[j], d[j]);
        append_settled_n<CH, 4>(a, ctl, p2, L, sm, row, deg, d);
        if (!compact) {
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((sm >> j) & 1u) qd[i + j] = kTomb;
            ntomb += (unsigned long long)__popc(sm);
        } else {
            // kept entries move down to [kept, kept + this step's count): below every slot a
            // later step reads; this step's loads have all returned before the first barrier
            const uint32_t kc = (uint32_t)__popc(keep);
            const uint32_t incl = wave_incl_scan(kc);
            const int w = threadIdx.x >> 6;
            if ((threadIdx.x & 63) == 63) s_wk[w] = incl;
            __builtin_amdgcn_s_waitcnt(0);
            __syncthreads();
            uint32_t wb = 0, tot = 0;
#pragma unroll
            for (int x = 0; x < kWaves; ++x) {
                wb += x < w ? s_wk[x] : 0u;
                tot += s_wk[x];
            }
            __syncthreads();  // s_wk is rewritten by the next step
            uint32_t o = kept + wb + incl - kc;
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if ((keep >> j) & 1u) {
                    qd[o] = d[j];
                    qv[o] = v[j];
                    qm[o] = mm[j];
                    qr[o] = rr[j];
                    ++o;
                }
            kept += tot;
        }
    }
    const uint32_t cnt = compact ? kept : cnt0;  // block-uniform
    // 2b. the vertices listed in 2a: certify, settle, or give an entry. Lists longer than one
    // round (a rebuild gathers every queued vertex) are taken kR rounds at a time, the loads of
    // all of them issued together.
    auto process = [&](bool has, uint32_t w, uint32_t off, const Gathered &g) {  // wavefront-uniform
        const uint32_t v = g.v, row = g.row, deg = g.deg;
        const unsigned long long d = g.d;
        const uint2 mm = g.mm;
        const uint32_t sb = has ? sw[w * kOwnSpan + wo + off] : 0u;
        const bool ok = has && !rebuild && certified(d, mm, sb);
        if (ok) settle(v, d);
        append_settled<CH>(a, ctl, p2, L, ok, row, deg, d);
        const bool far = KEYED && has && !ok && in_key(d, mm) > split;
        const bool app = has && !ok && !far;
        if (app || (rebuild && far)) {
            fmin = umin64(fmin, d);
            if (OUT == 1) ftst = umin64(ftst, sadd64(d, min_out64(mm.y, a.g.wmax, a.g.rp, v)));
        }
        if (far) a.b.st[v] = ST_F | ST_QFAR;
        const unsigned long long am = __ballot(app);
        if (am) {
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(&s_app, (uint32_t)__popcll(am));
            base = (uint32_t)__builtin_amdgcn_readlane((int)base, 0);
            if (app) {
                const uint32_t o = cnt + base + (uint32_t)__popcll(am & ((1ull << lane) - 1ull));
                qd[o] = d;
                qv[o] = v;
                qm[o] = mm;
                qr[o] = make_uint2(row, deg);
                a.b.st[v] = ST_F;
            }
        }
    };
    constexpr uint32_t kR = 4;
#pragma unroll
    for (uint32_t w = 0; w < kWin; ++w) {
        if (totw[w] == 0) continue;  // wavefront-uniform
        const uint64_t wv0 = (uint64_t)kOwnSpan * ((uint64_t)w * G + b) + wo;
        if (totw[w] <= 64) {  // one round, its loads issued in 2a
            process((uint32_t)lane < totw[w], w, offw[w], gw[w]);
            continue;
        }
        list_need(nmw[w]);  // the LDS list was overwritten by later windows
        for (uint32_t k0 = 0; k0 < totw[w]; k0 += 64 * kR) {  // wavefront-uniform
            uint32_t oq[kR];
            Gathered gq[kR];
#pragma unroll
            for (uint32_t r = 0; r < kR; ++r) {
                const uint32_t k = k0 + 64 * r + (uint32_t)lane;
                oq[r] = 0;
                gq[r] = Gathered{0u, 0u, 0u, INF64, make_uint2(INF32, INF32)};
                if (k0 == 0 && r == 0) {
                    oq[r] = offw[w];
                    gq[r] = gw[w];
                } else if (k < totw[w]) {
                    oq[r] = need[k];
                    gq[r] = gather(wv0, oq[r]);
                }
            }
#pragma unroll
            for (uint32_t r = 0; r < kR; ++r)
                if (k0 + 64 * r < totw[w]) process(k0 + 64 * r + (uint32_t)lane < totw[w], w, oq[r], gq[r]);
        }
    }
    append_flush<CH>(a, ctl, p2, L);  // starts with a barrier: s_app is final after it
    // [0] fmin, [1] ftst, [2] entries settled (tombstones made)
    unsigned long long r[8] = {fmin, ftst, ntomb, 0, 0, 0, 0, 0};
    block_reduce<kWaves, OUT == 1 ? 0x7u : 0x5u, 0x3u, 0x4u>(r, sh);
    if (threadIdx.x == 0) {
        a.b.qcnt[2 * b] = cnt + s_app;
        a.b.qcnt[2 * b + 1] = compact ? 0u : tomb0 + (uint32_t)r[2];
        if (r[0] != INF64) atomicMin(slot_of(ctl->minD[(p3 + 1) % 3], my_shard()), r[0]);
        if (OUT == 1 && r[1] != INF64) atomicMin(slot_of(ctl->tst[(p3 + 1) % 3], my_shard()), r[1]);
    }
}

// Term pass of the plain solvers (dynamic criteria): block b evaluates the
// terms of the queued vertices among kOwnSpan consecutive vertices (b + k G) *
// kOwnSpan + [0, kOwnSpan), k = 0, 1, ...; the host launches enough blocks for
// one window each, independent of the scan grid, so that the dependent loads of
// the cursor walks are spread over as many threads as the device holds. A
// window's state bytes are loaded with one 16-byte load per thread, issued with
// the control-slot loads for the first window, and staged in LDS; a window
// without a queued vertex is skipped, and the queued vertices are taken one per
// thread in vertex order, so that a wavefront's distance, cursor and cache loads
// are coalesced. The IN result goes to the vertex's ST_INOK bit (its other flag
// bits are kept for the queue-array identify), the OUT threshold is folded into
// this phase's tdyn slots. IN (full), OUTWEAK and OUT (full) terms are stored
// per vertex (tin, tout) and kept by k_mark: a vertex recomputes them from its
// rows only when flagged ST_TDIRTY, or in the phase a.fresh_at (every queued
// vertex: the first phase of the criterion).
template <int IN, int OUT>
__global__ __launch_bounds__(kBlock) void k_terms_win(KArgs a, int par) {
    constexpr bool kStoreIn = IN == IN_FULL_M, kStoreOut = OUT == OUT_WEAK_M || OUT == OUT_FULL_M;
    constexpr bool kStore = kStoreIn || kStoreOut;
    __shared__ unsigned long long sh[8 * kWaves];
    __shared__ uint4 s_st[kOwnSpan / 16];
    // stored terms: the vertices computed in full in this window, and their minima
    __shared__ RowList L;
    __shared__ unsigned long long s_ti[kStore ? kListCap : 1], s_to[kStore ? kListCap : 1];
    Ctl *ctl = a.b.ctl;
    const int p3 = par % 3;
    const unsigned long long r0 = lane_slot(ctl->reached, 0ull), m0 = lane_slot(ctl->minD[p3], INF64);
    const unsigned long long settled = ctl->h.settled;
    const bool fresh_all = kStore && ctl->h.pnum[par & 1] == a.fresh_at;
    const uint32_t n = a.g.n;
    auto load16 = [&](uint64_t v0) {
        if (v0 + 16 <= n) return *reinterpret_cast<const uint4 *>(a.b.st + v0);
        uint32_t q[4] = {0u, 0u, 0u, 0u};
        for (uint32_t j = 0; v0 + j < n; ++j) q[j >> 2] |= (uint32_t)a.b.st[v0 + j] << (8 * (j & 3));
        return make_uint4(q[0], q[1], q[2], q[3]);
    };
    const uint64_t step = (uint64_t)gridDim.x * kOwnSpan;
    uint64_t vb = (uint64_t)blockIdx.x * kOwnSpan;
    uint4 x = vb < n ? load16(vb + 16u * threadIdx.x) : make_uint4(0u, 0u, 0u, 0u);
    const unsigned long long reached = wave_sum64(r0);
    if (reached == settled) return;
    const unsigned long long minD = wave_min64(m0);
    const uint8_t *sw = reinterpret_cast<const uint8_t *>(s_st);
    unsigned long long tmin = INF64;
    // the phase's result for v from its terms ti / to: the IN flag, the OUT fold, the state byte
    auto finish = [&](uint32_t v, uint32_t sb, unsigned long long dv, unsigned long long ti, unsigned long long to) {
        bool ok = false;
        if (IN != IN_NONE) ok = dv <= sadd64(minD, ti);
        if (OUT != OUT_NONE) tmin = umin64(tmin, sadd64(dv, to));
        if (IN != IN_NONE || (sb & ST_TDIRTY))
            a.b.st[v] = (uint8_t)((sb & ~(uint32_t)(ST_INOK | ST_TDIRTY)) | (ok ? ST_INOK : 0u));
    };
    for (; vb < n; vb += step) {  // block-uniform
        bool any = false;
        const uint32_t xs[4] = {x.x, x.y, x.z, x.w};
#pragma unroll
        for (int j = 0; j < 16; ++j) any |= ((xs[j >> 2] >> (8 * (j & 3))) & ST_SET) == ST_F;
        __syncthreads();  // the previous window's LDS reads are done
        s_st[threadIdx.x] = x;
        if (kStore && threadIdx.x == 0) L.cnt = 0;
        if (__syncthreads_or(any)) {  // block-uniform
#pragma unroll 2
            for (uint32_t r = 0; r < kOwnSpan / kBlock; ++r) {
                const uint32_t i = r * kBlock + threadIdx.x;
                const uint32_t sb = sw[i];
                if ((sb & ST_SET) != ST_F) continue;
                const uint32_t v = (uint32_t)vb + i;
                const bool full = fresh_all || (sb & ST_TDIRTY) != 0;
                if (kStore && full) {
                    // computed in full by the block's flattened walk below, unless the list is full
                    const uint32_t ib = kStoreIn ? a.g.ip[v] : 0u, ie = kStoreIn ? a.g.ip[v + 1] : 0u;
                    const uint32_t ob = kStoreOut ? a.g.rp[v] : 0u, oe = kStoreOut ? a.g.rp[v + 1] : 0u;
                    const uint32_t j = atomicAdd(&L.cnt, 1u);
                    if (j < kListCap) {
                        L.v[j] = v;
                        L.f[j] = (uint8_t)sb;
                        L.a0[j] = ib;
                        L.b0[j] = ob;
                        L.n1[j] = ie - ib;  // the in-edges first
                        L.off[j] = (ie - ib) + (oe - ob);
                        s_ti[j] = INF64;
                        s_to[j] = INF64;
                        continue;
                    }
                }
                const unsigned long long dv = a.b.dist[v];
                unsigned long long ti = 0, to = 0;
                if (IN != IN_NONE) {
                    if (kStoreIn && !full) {
                        ti = a.b.tin[v];
                    } else {
                        ti = in_term<IN>(a, v);
                        if (kStoreIn) a.b.tin[v] = ti;
                    }
                }
                if (OUT != OUT_NONE) {
                    if (kStoreOut && !full) {
                        to = a.b.tout[v];
                    } else {
                        to = out_term<OUT>(a, v);
                        if (kStoreOut) a.b.tout[v] = to;
                    }
                }
                finish(v, sb, dv, ti, to);
            }
        }
        if (kStore) {
            __syncthreads();  // the list is complete
            const uint32_t cnt = L.cnt < kListCap ? L.cnt : kListCap;
            if (cnt) {  // block-uniform
                row_list_scan(L, cnt);
                uint32_t e, end, j;
                row_list_range(L, cnt, e, end, j);
                // four edges at a time: their loads are issued together (the walk is a chain of
                // dependent loads per edge: edge, end's state, end's minimum or cursor)
                for (; e < end; e += 4) {
                    uint32_t jq[4];
                    bool inq[4];
                    uint2 eq[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        jq[q] = kListCap;
                        inq[q] = false;
                        eq[q] = make_uint2(0u, 0u);
                        if (e + q < end) {
                            while (e + q >= L.off[j + 1]) ++j;
                            const uint32_t k = e + q - L.off[j];
                            jq[q] = j;
                            inq[q] = kStoreIn && k < L.n1[j];
                            eq[q] = inq[q] ? a.g.in_edges[L.a0[j] + k] : a.g.edges[L.b0[j] + (k - L.n1[j])];
                        }
                    }
                    uint32_t sq[4];
#pragma unroll
                    for (int q = 0; q < 4; ++q) sq[q] = jq[q] < kListCap ? (a.b.st[eq[q].x] & ST_SET) : (uint32_t)ST_S;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (sq[q] == ST_S) continue;  // settled end (or no edge): no candidate
                        unsigned long long c = eq[q].y;
                        if (inq[q]) {
                            // eq. crit:in: in-edges from F, or from w in U plus w's lightest in-edge
                            if (sq[q] == ST_U) c = sadd64(c, min_in_u64(a.g.vmin[eq[q].x].x, a.g.wmax, a.g.ip, eq[q].x));
                            atomicMin(&s_ti[jq[q]], c);
                        } else if (kStoreOut) {
                            // eq. crit:outweak / crit:out: out-edges into F, or into w in U plus w's second edge
                            if (sq[q] == ST_U)
                                c = sadd64(c, OUT == OUT_WEAK_M ? min_out64(a.g.vmin[eq[q].x].y, a.g.wmax, a.g.rp, eq[q].x)
                                                                : ns_cursor(a, eq[q].x));
                            atomicMin(&s_to[jq[q]], c);
                        }
                    }
                }
                __syncthreads();  // the minima are complete
                for (uint32_t q = threadIdx.x; q < cnt; q += kBlock) {
                    const uint32_t v = L.v[q];
                    unsigned long long ti = s_ti[q], to = s_to[q];
                    // the other side of a mixed criterion (a SIMPLE cursor) by this thread
                    if (IN != IN_NONE && !kStoreIn) ti = in_term<IN>(a, v);
                    if (OUT != OUT_NONE && !kStoreOut) to = out_term<OUT>(a, v);
                    if (kStoreIn) a.b.tin[v] = ti;
                    if (kStoreOut) a.b.tout[v] = to;
                    finish(v, L.f[q], a.b.dist[v], ti, to);
                }
            }
        }
        if (vb + step < n) x = load16(vb + step + 16u * threadIdx.x);
    }
    if (OUT != OUT_NONE) {
        block_reduce<kWaves, 1u, 1u>(&tmin, sh);
        if (threadIdx.x == 0 && tmin != INF64) atomicMin(slot_of(ctl->tdyn[p3], my_shard()), tmin);
    }
}

// ---------------------------------------------------------------------------
// identify (Delta-stepping round)

// Round kinds: 0 = first light round of a bucket (every queued vertex inside
// the window), 1 = later light round (vertices improved inside the window in
// the previous round), 2 = heavy round (everything the bucket removed).
template <int CH, bool LEARN>
__global__ __launch_bounds__(kBlock) void k_identify_delta(KArgs a, int par) {
    Ctl *ctl = a.b.ctl;
    const int p2 = par & 1;
    __shared__ unsigned long long sh[8 * kWaves];
    __shared__ AppendLds L;
    if (threadIdx.x == 0) { L.cnt = 0; L.filled = 0; L.zero = 0; }
    const unsigned int P = ctl->h.pnum[p2];
    const unsigned int b_now = ctl->h.buckets;
    const unsigned long long r0 = lane_slot(ctl->reached, 0ull), i0 = lane_slot(ctl->win_improved[p2 ^ 1], 0ull);
    const unsigned long long n0 = lane_slot(ctl->nextmin[b_now & 1], INF64);
    const unsigned long long settled = ctl->h.settled;
    const unsigned long long reached = wave_sum64(r0);
    const unsigned long long improved = wave_sum64(i0);
    const unsigned long long next = wave_min64(n0);
    int kind = 0;
    if (P > 0) {
        const unsigned int prev = ctl->h.rmode[p2 ^ 1];
        kind = prev == 2 ? 0 : (improved > 0 ? 1 : 2);
    }
    if (kind == 0 && reached == settled) {
        if (blockIdx.x == 0) {
            if (threadIdx.x == 0) {
                ctl->h.done = 1;
                ctl->h.pnum[p2 ^ 1] = P;
                ctl->h.rmode[p2] = 2;  // later empty rounds stay "after heavy"
            }
            shard_fill(ctl->spack[p2 ^ 1], 0);
            shard_fill(ctl->szero[p2 ^ 1], 0);
        }
        return;
    }
    const unsigned int b = kind == 0 ? b_now : ctl->h.win_bucket;
    unsigned long long lo, hi, delta;
    if (kind == 0) {
        delta = LEARN ? ctl->h.next_delta : a.b.deltas[b < ctl->h.n_deltas ? b : ctl->h.n_deltas - 1];
        lo = (next / delta) * delta;
        hi = sadd64(lo, delta);
    } else {
        lo = ctl->h.win_lo;
        hi = ctl->h.win_hi;
        delta = ctl->h.win_delta;
    }
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) {
            ctl->h.pnum[p2 ^ 1] = P + 1;
            ctl->h.phases = P + 1;
            ctl->h.rmode[p2] = kind;
            ctl->h.s_k = settled;
            if (kind == 2) ctl->h.buckets = b + 1;
            if (kind == 0) {
                ctl->h.fbucket = reached - settled;
                ctl->h.win_bucket = b;
                ctl->h.win_lo = lo;
                ctl->h.win_hi = hi;
                ctl->h.win_delta = delta;
                ctl->h.sum_f += reached - settled;
            }
            if (P < a.b.trace_cap) {
                PhaseRec r;
                r.min_d = lo;
                r.fringe = (unsigned int)(reached - settled);
                r.settled = 0;
                r.criterion = kind;
                r.edges = 0;
                a.b.trace[P] = r;
            }
        }
        shard_fill(ctl->win_improved[p2], 0);
        shard_fill(ctl->spack[p2 ^ 1], 0);
        shard_fill(ctl->szero[p2 ^ 1], 0);
        if (kind == 0) shard_fill(ctl->nextmin[(b + 1) & 1], INF64);
    }
    __syncthreads();  // LDS counters initialised
    unsigned long long fmin = INF64;
    const uint32_t n = a.g.n;
    const uint32_t nq = (n + 3) / 4;
    for (uint32_t base = blockIdx.x * kBlock; base < nq; base += gridDim.x * kBlock) {
        const uint32_t q = base + threadIdx.x;
        const uint32_t s4 = q < nq ? load_st4(a.b.st, q, n) : 0u;
        unsigned long long dv[4];
        uint32_t stp[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint8_t s = (s4 >> (8 * i)) & ST_SET;
            dv[i] = INF64;
            stp[i] = 0;
            const bool need = kind == 0 ? s == ST_F : kind == 1 ? (s == ST_F || s == ST_R) : (s == ST_F || s == ST_R);
            if (need) {
                dv[i] = a.b.dist[4 * q + i];
                if (kind == 1) stp[i] = a.b.stamp[4 * q + i];
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t v = 4 * q + i;
            const uint8_t s = (s4 >> (8 * i)) & ST_SET;
            bool set = false;
            if (kind == 0) set = s == ST_F && dv[i] < hi;
            else if (kind == 1) set = (s == ST_F || s == ST_R) && stp[i] == P;
            else {
                set = s == ST_R;
                if (s == ST_F) fmin = umin64(fmin, dv[i]);  // exact: nothing leaves F until the next bucket
            }
            uint32_t row = 0, deg = 0;
            if (set) {
                row = a.g.rp[v];
                deg = a.g.rp[v + 1] - row;
                a.b.st[v] = kind == 2 ? ST_S : ST_R;
                if (kind == 2) {
                    a.b.dist[v] = dv[i] | kSettledBit;
                    if (a.b.phase_of) a.b.phase_of[v] = P + 1;
                }
            }
            append_settled<CH>(a, ctl, p2, L, set, row, deg, dv[i]);
        }
    }
    append_flush<CH>(a, ctl, p2, L);
    if (kind == 2) {
        block_reduce<kWaves, 1u, 1u>(&fmin, sh);
        if (threadIdx.x == 0 && fmin != INF64) atomicMin(slot_of(ctl->nextmin[(b + 1) & 1], my_shard()), fmin);
    }
}

// ---------------------------------------------------------------------------
// relax

__device__ __forceinline__ unsigned long long aload(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long shard_sum_all(const Sharded &s) {
    unsigned long long t = 0;
    for (int i = 0; i < kShards; ++i) t += aload(&s.v[i * kPad]);
    return t;
}
__device__ __forceinline__ unsigned long long shard_min_all(const Sharded &s) {
    unsigned long long t = INF64;
    for (int i = 0; i < kShards; ++i) t = umin64(t, aload(&s.v[i * kPad]));
    return t;
}

// FOLDT: also fold the OUT-STATIC threshold (needed when OUT-STATIC is the
// OUT member of the phase's criterion).
// Learned mode, block 0 of relax(k): phase k+1's criterion from phase k's
// snapshot and outcome. Everything read here was final when relax(k) started
// and no block of relax(k) writes it. To stay within the relax kernel's
// register budget, lane j of wavefront w holds inputs [16w, 16w+16) of row j
// of W2 and of row min(j,5) of W3 (loaded once the features are done), and
// each neuron's fmaf chain passes from wavefront 0 to 3 through LDS, in the
// same sequential order as the one-wave evaluation.
__device__ __forceinline__ void select_next_phase(const KArgs &a, int p2, int p3, unsigned int P,
                                                  unsigned long long nS) {
    static_assert(kWaves * 16 == kMlpH, "four wavefronts of sixteen inputs");
    __shared__ float s_h1[kMlpH], s_acc[kMlpH], s_h2[kMlpH], s_z[kMlpOut];
    Ctl *ctl = a.b.ctl;
    const float *w = a.mlp_w;
    const int wv = threadIdx.x >> 6, j = threadIdx.x & 63, o = j < kMlpOut ? j : kMlpOut - 1;
    float4 w2[4], w3[4];
    const float4 *r2 = reinterpret_cast<const float4 *>(w + kOffW2 + j * kMlpH + 16 * wv);
    const float4 *r3 = reinterpret_cast<const float4 *>(w + kOffW3 + o * kMlpH + 16 * wv);
    if (wv == 0) {
        const float4 *r1 = reinterpret_cast<const float4 *>(w + j * kMlpIn);
        float4 w1[kMlpIn / 4];
#pragma unroll
        for (int i = 0; i < kMlpIn / 4; ++i) w1[i] = r1[i];
        const float c1 = w[kOffB1 + j], c2 = w[kOffB2 + j], c3 = w[kOffB3 + o];
        const unsigned long long F = ctl->h.fk, S = ctl->h.s_k, Fp = ctl->h.fprev, DG = ctl->h.dgk;
        const unsigned long long a0 = lane_slot(ctl->minD[p3], INF64), t0 = lane_slot(ctl->tst[p3], INF64);
        const unsigned long long sd0 = lane_slot(ctl->sumd[p3], 0ull);
        const unsigned long long in0 = lane_slot(ctl->nin[p2], 0ull), out0 = lane_slot(ctl->nout[p2], 0ull);
        FeatIn q;
        q.n = a.g.n;
        q.m = a.g.m;
        q.F = F;
        q.S = S;
        q.R = F + S;
        q.a = wave_min64(a0);
        q.t = wave_min64(t0);
        q.SD = wave_sum64(sd0);
        q.DG = DG;
        q.Fp = Fp;
        q.D = F;
        q.Sp = nS;
        q.Ip = wave_sum64(in0);
        q.Op = wave_sum64(out0);
        q.k = P + 1ull;
        q.Wm = a.wm;
        q.delta_mode = 0;
        float x[kMlpIn];
        features_dev(q, x);
        float acc = c1;
#pragma unroll
        for (int i = 0; i < kMlpIn / 4; ++i) {
            acc = fmaf(w1[i].x, x[4 * i], acc);
            acc = fmaf(w1[i].y, x[4 * i + 1], acc);
            acc = fmaf(w1[i].z, x[4 * i + 2], acc);
            acc = fmaf(w1[i].w, x[4 * i + 3], acc);
        }
        s_h1[j] = acc > 0.0f ? acc : 0.0f;
        s_acc[j] = c2;
        if (j < kMlpOut) s_z[j] = c3;
        if (a.b.trace_feat && q.k < a.b.trace_cap && j < kMlpIn) a.b.trace_feat[q.k * kMlpIn + j] = x[j];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // W3 stays in flight during layer 2
        w2[i] = r2[i];
        w3[i] = r3[i];
    }
    for (int step = 0; step < kWaves; ++step) {  // layer 2, inputs [16 step, 16 step + 16)
        if (wv == step) {
            float acc = s_acc[j];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc = fmaf(w2[i].x, s_h1[16 * step + 4 * i], acc);
                acc = fmaf(w2[i].y, s_h1[16 * step + 4 * i + 1], acc);
                acc = fmaf(w2[i].z, s_h1[16 * step + 4 * i + 2], acc);
                acc = fmaf(w2[i].w, s_h1[16 * step + 4 * i + 3], acc);
            }
            if (step == kWaves - 1) s_h2[j] = acc > 0.0f ? acc : 0.0f;
            else s_acc[j] = acc;
        }
        __syncthreads();
    }
    for (int step = 0; step < kWaves; ++step) {  // layer 3, lanes 0..5
        if (wv == step && j < kMlpOut) {
            float acc = s_z[j];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                acc = fmaf(w3[i].x, s_h2[16 * step + 4 * i], acc);
                acc = fmaf(w3[i].y, s_h2[16 * step + 4 * i + 1], acc);
                acc = fmaf(w3[i].z, s_h2[16 * step + 4 * i + 2], acc);
                acc = fmaf(w3[i].w, s_h2[16 * step + 4 * i + 3], acc);
            }
            s_z[j] = acc;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        int best = 0;
        for (int c = 1; c < 3; ++c)
            if (s_z[c] > s_z[best]) best = c;
        ctl->h.choice[p2 ^ 1] = (unsigned int)best;
    }
}

// LEARN: also fold the selector's feature sums (sum of d and of out-degrees
// over the queued set) for the next phase; in the phased solver block 0 only
// evaluates the selector for phase k+1 and the other blocks take its share of
// the edges.
// Q: queue arrays are in use (static criteria): a discovered vertex is marked
// ST_F | ST_QNEW and a vertex whose distance drops ST_QDIRTY, for its owner's
// identify.
template <int CH, bool DELTA, bool FOLDT, bool LEARN, bool Q = false>
__global__ __launch_bounds__(kBlock) void k_relax(KArgs a, int par) {
    Ctl *ctl = a.b.ctl;
    const int p2 = par & 1, p3 = par % 3;
    __shared__ uint32_t s_pos[CH + 1];
    __shared__ uint32_t s_start[CH + 1];
    __shared__ unsigned long long s_du[CH + 1];
    __shared__ unsigned long long sh[8 * kWaves];
    __shared__ uint32_t s_ns[kShards], s_E[kShards], s_nch[kShards];
    __shared__ uint32_t s_cmax, s_ctot;
    __shared__ uint32_t s_cpre[kShards];  // exclusive prefix of the shards' chunk counts
    __shared__ unsigned long long s_tot_settled, s_tot_edges;
    // Chunks are interleaved over the shards: chunk c is chunk c / kShards of shard
    // c % kShards, so a block knows its first chunk before it has read the shard
    // counters and loads that chunk's entry bounds with them (guarded to stay inside
    // the chunk_start rows; the values count only if the chunk exists).
    constexpr bool kSel = LEARN && !DELTA;
    const bool split = kSel && gridDim.x > 1;  // block 0 selects, blocks 1.. relax
    const uint32_t cfirst = split ? blockIdx.x - 1 : blockIdx.x, cstep = split ? gridDim.x - 1 : gridDim.x;
    const uint32_t lc0 = cfirst / kShards;
    const int sd0 = (int)(cfirst % kShards);
    uint32_t spec0 = 0, spec1 = 0;
    const bool spec = lc0 + 1 < a.b.chunk_cap;
    if (spec) {
        const uint32_t *cs = a.b.chunk_start + (uint64_t)sd0 * a.b.chunk_cap;
        spec0 = cs[lc0];
        spec1 = cs[lc0 + 1];
    }
    // header fields, loaded with the shard slots (before the barrier)
    const unsigned int done = ctl->h.done, P = ctl->h.pnum[p2];
    const unsigned int rebuilt = Q ? ctl->h.repart[p2] : 0u;  // keyed: a rebuild launch, not a phase
    const unsigned int rmode = DELTA ? ctl->h.rmode[p2] : 0u;
    const unsigned long long win_hi = DELTA ? ctl->h.win_hi : INF64, win_delta = DELTA ? ctl->h.win_delta : 0ull;
    if (threadIdx.x < 64) {
        // per-shard S' sizes, edge totals and an exclusive prefix of their chunk counts
        const int i = threadIdx.x;
        const unsigned long long pk = i < kShards ? ctl->spack[p2].v[i * kPad] : 0ull;
        const unsigned long long nz = i < kShards ? ctl->szero[p2].v[i * kPad] : 0ull;
        const uint32_t ns = (uint32_t)(pk >> 32), E = (uint32_t)pk;
        const uint32_t nch = (uint32_t)(((uint64_t)E + CH - 1) / CH);
        uint32_t mx = nch;  // most chunks in one shard: chunks c < kShards * mx may exist
        for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o, 64));
        const uint32_t cin = wave_incl_scan(i < kShards ? nch : 0u);
        if (i < kShards) {
            s_ns[i] = ns;
            s_E[i] = E;
            s_nch[i] = nch;
            s_cpre[i] = cin - nch;
        }
        if (i == kShards - 1) s_ctot = cin;
        const unsigned long long tset = wave_sum64((unsigned long long)ns + nz);
        const unsigned long long tedge = wave_sum64(E);
        if (i == 0) { s_tot_settled = tset; s_tot_edges = tedge; s_cmax = kShards * mx; }
    }
    __syncthreads();
    if (rebuilt) return;  // it settled nothing (its S' counters are zero) and relaxes nothing
    if (!DELTA && s_tot_settled == 0 && !done && blockIdx.x == 0 && threadIdx.x == 0) {
        // F is non-empty but nothing was certified: only an ORACLE reference that is not
        // dist(s, .) gets here (every other criterion certifies the queue minimum)
        ctl->h.stalled = 1;
        ctl->h.done = 1;
    }
    if (s_tot_settled == 0 || done) return;
    int kind = 0;
    unsigned long long hi = INF64, delta = 0;
    if (DELTA) {
        kind = rmode == 2 ? 2 : 1;
        hi = win_hi;
        delta = win_delta;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!DELTA || kind == 2) {
            ctl->h.settled += s_tot_settled;
            ctl->h.m_reach += s_tot_edges;
        }
        ctl->h.last_settled = s_tot_settled;  // |S'| of this phase (selector feature)
        if (P < a.b.trace_cap) {
            a.b.trace[P].settled = (unsigned int)s_tot_settled;
            a.b.trace[P].edges = (unsigned int)s_tot_edges;
            if (a.b.trace_cf && !DELTA)
                for (int c = 0; c < 3; ++c) a.b.trace_cf[3 * P + c] = (uint32_t)shard_sum_all(ctl->cnt_cf[p2 * 3 + c]);
        }
    }
    if (kSel && blockIdx.x == 0) {
        select_next_phase(a, p2, p3, P, s_tot_settled);
        if (split) return;
    }
    unsigned long long cmin = INF64, ctst = INF64, tried = 0, improv = 0, disc = 0, winimp = 0, dsum = 0, ddeg = 0;
    // Chunk c is chunk c / kShards of shard c % kShards while that leaves every block
    // at most one chunk index (then the first chunk's bounds were loaded above);
    // otherwise some shard holds many more edges than the others (a high-degree row
    // settled), and the chunks are numbered shard by shard, so that the blocks take
    // equal numbers of them.
    const bool ilv = s_cmax <= cstep;  // block-uniform
    const uint32_t cmax = ilv ? s_cmax : s_ctot;
    // Chunk c's shard, shard-local index and first / last S' entry (ok = the chunk
    // exists); the entry bounds of the block's next chunk are loaded while this one
    // is processed.
    struct ChunkRef {
        int sd;
        uint32_t lc, j0, jend;
        bool ok;
    };
    auto chunk_ref = [&](uint32_t c, bool use_spec) {
        ChunkRef r;
        if (ilv) {
            r.sd = (int)(c % kShards);
            r.lc = c / kShards;
        } else {
            int lo = 0;  // last shard whose first chunk number is <= c
#pragma unroll
            for (int st = kShards / 2; st > 0; st >>= 1)
                if (s_cpre[lo + st] <= c) lo += st;
            r.sd = lo;
            r.lc = c - s_cpre[lo];
            use_spec = false;
        }
        r.ok = r.lc < s_nch[r.sd];
        r.j0 = r.jend = 0;
        if (r.ok) {
            const bool last = (uint64_t)r.lc * CH + CH >= s_E[r.sd];
            if (use_spec) {
                r.j0 = spec0;
                r.jend = last ? s_ns[r.sd] - 1 : spec1;
            } else {
                const uint32_t *cs = a.b.chunk_start + (uint64_t)r.sd * a.b.chunk_cap;
                r.j0 = cs[r.lc];
                r.jend = last ? s_ns[r.sd] - 1 : cs[r.lc + 1];
            }
        }
        return r;
    };
    ChunkRef nxt{};
    if (cfirst < cmax) nxt = chunk_ref(cfirst, spec);
    for (uint32_t c = cfirst; c < cmax; c += cstep) {
        const ChunkRef ck = nxt;
        if (c + cstep < cmax) nxt = chunk_ref(c + cstep, false);
        if (!ck.ok) continue;  // block-uniform
        const int sd = ck.sd;
        const uint32_t lc = ck.lc;
        const uint32_t Es = s_E[sd];
        const uint32_t e0 = lc * CH;
        const uint32_t len = min(Es - e0, (uint32_t)CH);
        const uint32_t j0 = ck.j0;
        const uint32_t jend = ck.jend;
        const uint32_t cnt = jend - j0 + 1;
        const uint64_t gbase = (uint64_t)sd * a.b.shard_cap;
        __syncthreads();
        for (uint32_t t = threadIdx.x; t < cnt; t += kBlock) {
            const uint64_t j = gbase + j0 + t;
            const uint32_t off = a.b.soff[j];
            s_pos[t] = off > e0 ? off - e0 : 0u;
            s_start[t] = a.b.srow[j] + (off > e0 ? 0u : e0 - off);
            s_du[t] = a.b.sdu[j];
        }
        __syncthreads();
        // Each thread takes edges threadIdx.x + k * kBlock (k < E) of the chunk, every stage's
        // loads and atomics for its E edges issued together.
        constexpr int E = CH / kBlock;
        constexpr int kSteps = CH >= 1024 ? 11 : CH >= 512 ? 10 : 9;  // > log2(CH + 1)
        uint32_t lo[E], hi2[E];
#pragma unroll
        for (int k = 0; k < E; ++k) {
            lo[k] = 0;  // last entry whose first chunk position is <= i
            hi2[k] = cnt - 1;
        }
#pragma unroll
        for (int it = 0; it < kSteps; ++it)
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const uint32_t i = threadIdx.x + k * kBlock;
                if (lo[k] < hi2[k]) {
                    const uint32_t mid = (lo[k] + hi2[k] + 1) >> 1;
                    if (s_pos[mid] <= i) lo[k] = mid; else hi2[k] = mid - 1;
                }
            }
        uint2 ed[E];
        uint32_t em[E];  // FOLDT: minOut of each edge's target, loaded beside the edge
        unsigned long long cur[E], cand[E], old[E];
        uint32_t live = 0, issued = 0;
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t i = threadIdx.x + k * kBlock;
            ed[k] = make_uint2(0u, 0u);
            em[k] = INF32;
            if (i < len) {
                const uint32_t e = s_start[lo[k]] + (i - s_pos[lo[k]]);
                ed[k] = a.g.edges[e];
                if (FOLDT) em[k] = a.g.emin[e];
                live |= 1u << k;
            }
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            cur[k] = 0;
            if (DELTA && ((live >> k) & 1u)) {
                if (kind == 1 && ed[k].y >= delta) live &= ~(1u << k);  // light: c < delta
                if (kind == 2 && ed[k].y < delta) live &= ~(1u << k);   // heavy: c >= delta
            }
            if ((live >> k) & 1u) cur[k] = a.b.dist[ed[k].x];
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            cand[k] = old[k] = INF64;
            if (!((live >> k) & 1u) || dist_settled(cur[k])) continue;
            ++tried;
            cand[k] = s_du[lo[k]] + ed[k].y;
            if (cand[k] < cur[k]) {
                old[k] = atomicMin(&a.b.dist[ed[k].x], cand[k]);
                issued |= 1u << k;
            }
        }
#pragma unroll
        for (int k = 0; k < E; ++k) {
            if (!((issued >> k) & 1u) || !(cand[k] < old[k])) continue;
            const uint32_t v = ed[k].x;
            ++improv;
            if (!DELTA) {
                cmin = umin64(cmin, cand[k]);
                if (FOLDT) ctst = umin64(ctst, sadd64(cand[k], min_out64(em[k], a.g.wmax, a.g.rp, v)));
            } else if (kind == 2) {
                cmin = umin64(cmin, cand[k]);
            } else if (cand[k] < hi) {
                const unsigned int prev = atomicExch(&a.b.stamp[v], P + 1);
                if (prev != P + 1) ++winimp;
            }
            if (LEARN && !DELTA) dsum += old[k] == INF64 ? cand[k] : cand[k] - old[k];  // mod 2^64: sum over F of d
            if (Q) {
                // flag for the owner's identify: word-wide OR, as other lanes flag the same word
                uint32_t *w = reinterpret_cast<uint32_t *>(a.b.st + (v & ~3u));
                const uint32_t f = old[k] == INF64 ? (uint32_t)(ST_F | ST_QNEW | (a.mark ? ST_CHG | ST_TDIRTY : 0))
                                                   : (uint32_t)ST_QDIRTY;
                atomicOr(w, f << (8 * (v & 3u)));
            }
            if (old[k] == INF64) {
                if (!Q) a.b.st[v] = (uint8_t)(ST_F | (a.mark ? ST_CHG | ST_TDIRTY : 0));
                ++disc;
                if (LEARN && !DELTA) ddeg += a.g.rp[v + 1] - a.g.rp[v];
            }
        }
    }
    // [0] cmin, [1] ctst, [2] tried, [3] improv, [4] disc, [5] winimp, [6] dsum, [7] ddeg
    unsigned long long v[8] = {cmin, ctst, tried, improv, disc, winimp, dsum, ddeg};
    constexpr unsigned kAct = 0x1du | (FOLDT ? 0x2u : 0u) | (DELTA ? 0x20u : 0u) | (kSel ? 0xc0u : 0u);
    block_reduce<kWaves, kAct, 0x3u, 0xbcu>(v, sh);
    cmin = v[0];
    ctst = v[1];
    tried = v[2];
    improv = v[3];
    disc = v[4];
    winimp = v[5];
    dsum = v[6];
    ddeg = v[7];
    if (threadIdx.x == 0) {
        const int s = my_shard();
        if (LEARN && !DELTA) {
            if (dsum) atomicAdd(slot_of(ctl->sumd[(p3 + 1) % 3], s), dsum);
            if (ddeg) atomicAdd(slot_of(ctl->degsum, s), ddeg);
        }
        if (cmin != INF64) {
            if (!DELTA) atomicMin(slot_of(ctl->minD[(p3 + 1) % 3], s), cmin);
            else atomicMin(slot_of(ctl->nextmin[(ctl->h.win_bucket + 1) & 1], s), cmin);
        }
        if (FOLDT && ctst != INF64) atomicMin(slot_of(ctl->tst[(p3 + 1) % 3], s), ctst);
        if (tried) atomicAdd(slot_of(ctl->relax_edges, s), tried);
        if (improv) atomicAdd(slot_of(ctl->improving, s), improv);
        if (disc) atomicAdd(slot_of(ctl->reached, s), disc);
        if (winimp) atomicAdd(slot_of(ctl->win_improved[p2], s), winimp);
    }
}

// ---------------------------------------------------------------------------
// learned mode: the selector between phases

// Learned Delta-stepping, one wavefront after every round: after a heavy
// round, the next bucket's width from the state at the next bucket start.
__global__ __launch_bounds__(64) void k_select_delta(KArgs a, int par) {
    Ctl *ctl = a.b.ctl;
    const int p2 = par & 1;
    MlpRegs W;
    mlp_load(a.mlp_w, W);
    const unsigned int done = ctl->h.done, rmode = ctl->h.rmode[p2], wb = ctl->h.win_bucket;
    const unsigned long long S = ctl->h.settled, Sp = ctl->h.last_settled, Fb = ctl->h.fbucket;
    const unsigned long long r0 = lane_slot(ctl->reached, 0ull);
    const unsigned long long a0 = lane_slot(ctl->nextmin[(wb + 1) & 1], INF64);
    if (done || rmode != 2) return;  // only after a heavy round
    const unsigned long long R = wave_sum64(r0);
    FeatIn q;
    q.n = a.g.n;
    q.m = a.g.m;
    q.F = R - S;
    q.S = S;
    q.R = R;
    q.a = wave_min64(a0);
    q.t = INF64;
    q.SD = q.DG = q.Ip = q.Op = q.Fp = 0;
    q.D = Fb;
    q.Sp = Sp;
    q.k = wb + 1ull;
    q.Wm = a.wm;
    q.delta_mode = 1;
    if (q.F == 0) return;  // F is empty: no next bucket
    float x[kMlpIn];
    features_dev(q, x);
    const int c = mlp_eval(W, x, 3);
    if (threadIdx.x == 0) {
        ctl->h.next_delta = 1ull << (12 + 2 * (c - 3));
        if (a.b.trace_feat && q.k < a.b.trace_cap)
            for (int i = 0; i < kMlpIn; ++i) a.b.trace_feat[q.k * kMlpIn + i] = x[i];
    }
}

// Learned checkpoint mode, one wavefront after the last phase k of every batch
// of kSwitchBatch phases of a plain static solve: the selector looks at phase
// k's snapshot and outcome (F, S, minD and the OUT-STATIC threshold of phase k,
// what it settled, |F| at the previous checkpoint; checkpoint features) and
// writes its choice: 0 = keep the static criterion, 1 = IN-SIMPLE|OUT-SIMPLE,
// 2 = IN-SIMPLE|OUT-STATIC from now on. Everything read was final when relax(k)
// ended; identify(k+1) clears phase k's slots only after this kernel.
__global__ __launch_bounds__(64) void k_select_checkpoint(KArgs a, int par) {
    Ctl *ctl = a.b.ctl;
    const int p2 = par & 1, p3 = par % 3;
    MlpRegs W;
    mlp_load(a.mlp_w, W);
    const unsigned int done = ctl->h.done, P = ctl->h.pnum[p2];
    const unsigned long long F = ctl->h.fk, S = ctl->h.s_k, Sp = ctl->h.last_settled, Fp = ctl->h.cp_fprev;
    const unsigned long long a0 = lane_slot(ctl->minD[p3], INF64), t0 = lane_slot(ctl->tst[p3], INF64);
    if (done) return;
    FeatIn q;
    q.n = a.g.n;
    q.m = a.g.m;
    q.F = F;
    q.S = S;
    q.R = F + S;
    q.a = wave_min64(a0);
    q.t = wave_min64(t0);
    q.SD = q.DG = q.Ip = q.Op = 0;
    q.Fp = Fp;
    q.D = F;
    q.Sp = Sp;
    q.k = P + 1ull;
    q.Wm = a.wm;
    q.delta_mode = 2;
    float x[kMlpIn];
    features_dev(q, x);
    const int c = mlp_eval(W, x, 0);
    if (threadIdx.x == 0) {
        ctl->h.cp_choice = (unsigned int)c;
        ctl->h.cp_fprev = F;
        const unsigned int j = P / 16;  // checkpoint index (phases 16 j .. 16 j + 15 before it)
        if (a.b.trace_feat && j < a.b.trace_cap)
            for (int i = 0; i < kMlpIn; ++i) a.b.trace_feat[j * kMlpIn + i] = x[i];
    }
}

// ---------------------------------------------------------------------------
// host side

DevGraph dev_view(const sssp_graph *g) {
    DevGraph d;
    d.n = g->n;
    d.m = g->m;
    d.rp = g->rp;
    d.edges = g->edges;
    d.vmin = g->vmin;
    d.ip = g->ip;
    d.in_edges = g->in_edges;
    d.emin = g->emin;
    d.wmax = g->wmax;
    return d;
}

static int num_cus() {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            cus = p.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

void graph_default_cfg(sssp_graph *g) {
    const int cus = num_cus();
    // scan: 4 vertices per lane, about 4 blocks per compute unit on large graphs
    uint64_t sb = ((uint64_t)g->n + 4 * kBlock - 1) / (4 * kBlock);
    if (sb < 1) sb = 1;
    if (sb > (uint64_t)cus * 4) sb = (uint64_t)cus * 4;
    g->cfg.scan_blocks = (int)sb;
    g->cfg.chunk = 256;
    uint64_t rb = (g->m + g->cfg.chunk - 1) / g->cfg.chunk;
    if (rb < 1) rb = 1;
    if (rb > (uint64_t)cus * 4) rb = (uint64_t)cus * 4;
    g->cfg.relax_blocks = (int)rb;
    g->cfg.use_graph = 0;
    g->cfg.queue = 1;
}

void solve_bufs_free(sssp_graph *g) {
    SolveBufs &b = g->b;
    sssp_free(b.ctl); sssp_free(b.st); sssp_free(b.srow); sssp_free(b.soff); sssp_free(b.sdu);
    sssp_free(b.chunk_start); sssp_free(b.in_cur); sssp_free(b.out_cur); sssp_free(b.stamp); sssp_free(b.deltas);
    sssp_free(b.in_head); sssp_free(b.out_head);
    sssp_free(b.qd); sssp_free(b.qv); sssp_free(b.qm); sssp_free(b.qr); sssp_free(b.qcnt);
    sssp_free(b.apx_lin); sssp_free(b.apx_lout); sssp_free(b.apx_sp);
    sssp_free(b.tin); sssp_free(b.tout);
    sssp_free(g->one_st); sssp_free(g->one_fl); sssp_free(g->one_aux);
    g->one_st = nullptr;
    g->one_fl = nullptr;
    g->one_aux = nullptr;
    if (g->h_ctl) sssp_host_free(g->h_ctl);
    for (uint32_t i = 0; i < g->pev_cap; ++i) (void)hipEventDestroy(g->pev[i]);
    delete[] g->pev;
    g->pev = nullptr;
    g->pev_cap = 0;
    for (int i = 0; i < 2; ++i) if (g->ev[i]) (void)hipEventDestroy(g->ev[i]);
    if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
    g->graph_exec = nullptr;
    g->graph = nullptr;
    g->cap_stream = nullptr;
    g->graph_key_len = 0;
    memset(&b, 0, sizeof b);
    g->h_ctl = nullptr;
    g->ev[0] = g->ev[1] = nullptr;
    g->bufs_ready = false;
    g->bufs_scan_blocks = 0;
    g->delta_cap = 0;  // b.deltas was released with the rest
}

// Vertices a shard can settle in one phase: block b of the dense scan owns
// the vertex quads q = b*kBlock + i + k*G*kBlock (vertices 4q..4q+3); with
// queue arrays it owns kOwnSpan = 16 * kBlock consecutive vertices per grid
// step. Shard = b % kShards, so a shard owns at most ceil(G / kShards) blocks
// of at most scan_span(n, G, vpl) = vpl * kBlock * ceil(ceil(n / vpl) / (G * kBlock))
// vertices each (vpl = 4 or 16 vertices per lane).
static uint64_t scan_span(uint32_t n, int G, uint64_t vpl) {
    const uint64_t nv = ((uint64_t)n + vpl - 1) / vpl;
    const uint64_t iters = (nv + (uint64_t)G * kBlock - 1) / ((uint64_t)G * kBlock);
    return vpl * kBlock * iters;
}
static uint32_t shard_capacity(uint32_t n, int G) {
    const uint64_t blocks = ((uint64_t)G + kShards - 1) / kShards;
    const uint64_t a = scan_span(n, G, 4), b = scan_span(n, G, 16);
    return (uint32_t)(blocks * (a > b ? a : b));
}

// Allocates every buffer of a group or none: on a failure the buffers already
// taken are released and every pointer of the group is null again, so a later
// call starts the group afresh.
static int alloc_group(void **const *ptr, const uint64_t *bytes, int k) {
    for (int i = 0; i < k; ++i) {
        const hipError_t e = hipMalloc(ptr[i], bytes[i] ? bytes[i] : 1);
        if (e != hipSuccess) {
            for (int j = 0; j < k; ++j) {
                sssp_free(*ptr[j]);
                *ptr[j] = nullptr;
            }
            return sssp_set_error(e == hipErrorOutOfMemory ? SSSP_ERR_OOM : SSSP_ERR_DEVICE,
                                  "scratch allocation of %llu bytes failed: %s", (unsigned long long)bytes[i],
                                  hipGetErrorString(e));
        }
    }
    return SSSP_OK;
}

int solve_bufs_ensure(sssp_graph *g, bool cursors, bool stamps, bool queue, bool approx, bool store) {
    SolveBufs &b = g->b;
    const uint64_t n = g->n;
    if (g->bufs_ready && g->bufs_scan_blocks != (uint32_t)g->cfg.scan_blocks) {
        // the S' shard layout depends on the scan grid: rebuild the scratch
        solve_bufs_free(g);
    }
    if (!g->bufs_ready) {
        solve_bufs_free(g);  // whatever a failed earlier call left behind
        b.shard_cap = shard_capacity(g->n, g->cfg.scan_blocks);
        b.chunk_cap = (uint32_t)(g->m / 256 + 2);  // every chunk size is >= 256 edges
        const uint64_t sent = (uint64_t)kShards * b.shard_cap;
        void **const p[] = {(void **)&b.ctl, (void **)&b.st, (void **)&b.srow, (void **)&b.soff, (void **)&b.sdu,
                            (void **)&b.chunk_start};
        // st in whole words: relax ORs flags into 32-bit words
        const uint64_t z[] = {sizeof(Ctl), (n + 15) & ~15ull, sent * 4, sent * 4, sent * 8,
                              (uint64_t)kShards * b.chunk_cap * 4};
        int rc = alloc_group(p, z, 6);
        if (rc) return rc;
        HIP_OK(hipHostMalloc((void **)&g->h_ctl, 2 * sizeof(CtlHead), hipHostMallocDefault));
        HIP_OK(hipEventCreateWithFlags(&g->ev[0], hipEventDisableTiming));
        HIP_OK(hipEventCreateWithFlags(&g->ev[1], hipEventDisableTiming));
        g->bufs_ready = true;
        g->bufs_scan_blocks = (uint32_t)g->cfg.scan_blocks;
    }
    if (cursors && !(b.in_cur && b.out_cur && b.in_head && b.out_head)) {
        void **const p[] = {(void **)&b.in_cur, (void **)&b.out_cur, (void **)&b.in_head, (void **)&b.out_head};
        const uint64_t z[] = {n * 4, n * 4, n * 8, n * 8};
        int rc = alloc_group(p, z, 4);
        if (rc) return rc;
    }
    if (stamps && !b.stamp) HIP_OK(hipMalloc(&b.stamp, n * 4));
    if (queue && !(b.qd && b.qv && b.qm && b.qr && b.qcnt)) {
        const uint64_t G = (uint64_t)g->cfg.scan_blocks;
        const uint64_t span = scan_span(g->n, g->cfg.scan_blocks, 16);
        if (G * span >= INF32) return sssp_set_error(SSSP_ERR_UNSUPPORTED, "queue arrays: too many slots");
        b.qspan = (uint32_t)span;
        void **const p[] = {(void **)&b.qd, (void **)&b.qv, (void **)&b.qm, (void **)&b.qr, (void **)&b.qcnt};
        const uint64_t z[] = {G * span * 8, G * span * 4, G * span * 8, G * span * 8, G * 8};
        int rc = alloc_group(p, z, 5);
        if (rc) return rc;
    }
    if (approx && !(b.apx_lin && b.apx_lout && b.apx_sp)) {
        void **const p[] = {(void **)&b.apx_lin, (void **)&b.apx_lout, (void **)&b.apx_sp};
        const uint64_t z[] = {n * 4, n * 4, n * 4};
        int rc = alloc_group(p, z, 3);
        if (rc) return rc;
    }
    if (store && !(b.tin && b.tout)) {
        void **const p[] = {(void **)&b.tin, (void **)&b.tout};
        const uint64_t z[] = {n * 8, n * 8};
        int rc = alloc_group(p, z, 2);
        if (rc) return rc;
    }
    return SSSP_OK;
}

typedef void (*kfn)(KArgs, int);

template <int CH>
static kfn pick_identify(int in, int out) {
    // in: IN_NONE, IN_DIJK, IN_STATIC_M, >= IN_SIMPLE_M -> flag (3)
    // out: OUT_NONE, OUT_STATIC_M, dynamic -> 2
    const int i = in >= IN_SIMPLE_M ? 3 : in;
    const int o = out >= OUT_SIMPLE_M ? 2 : out;
    static const kfn tab[4][3] = {
        {k_identify<0, 0, CH>, k_identify<0, 1, CH>, k_identify<0, 2, CH>},
        {k_identify<1, 0, CH>, k_identify<1, 1, CH>, k_identify<1, 2, CH>},
        {k_identify<2, 0, CH>, k_identify<2, 1, CH>, k_identify<2, 2, CH>},
        {k_identify<3, 0, CH>, k_identify<3, 1, CH>, k_identify<3, 2, CH>}};
    return tab[i][o];
}

static kfn pick_terms(int in, int out) {
    const int i = in == IN_SIMPLE_M ? 1 : in == IN_FULL_M ? 2 : 0;
    const int o = out == OUT_SIMPLE_M ? 1 : out == OUT_WEAK_M ? 2 : out == OUT_FULL_M ? 3 : 0;
    static const kfn tab[3][4] = {
        {nullptr, k_terms_win<0, OUT_SIMPLE_M>, k_terms_win<0, OUT_WEAK_M>, k_terms_win<0, OUT_FULL_M>},
        {k_terms_win<IN_SIMPLE_M, 0>, k_terms_win<IN_SIMPLE_M, OUT_SIMPLE_M>, k_terms_win<IN_SIMPLE_M, OUT_WEAK_M>,
         k_terms_win<IN_SIMPLE_M, OUT_FULL_M>},
        {k_terms_win<IN_FULL_M, 0>, k_terms_win<IN_FULL_M, OUT_SIMPLE_M>, k_terms_win<IN_FULL_M, OUT_WEAK_M>,
         k_terms_win<IN_FULL_M, OUT_FULL_M>}};
    return tab[i][o];
}

// The dirty-set pass of the stored full terms (nullptr when the criterion has none).
static kfn pick_mark(int in, int out) {
    const bool i = in == IN_FULL_M;
    const int o = out == OUT_WEAK_M ? 1 : out == OUT_FULL_M ? 2 : 0;
    static const kfn tab[2][3] = {{nullptr, k_mark<false, OUT_WEAK_M>, k_mark<false, OUT_FULL_M>},
                                  {k_mark<true, 0>, k_mark<true, OUT_WEAK_M>, k_mark<true, OUT_FULL_M>}};
    return tab[i][o];
}

// Grid of the term pass: one block per kOwnSpan vertices, independent of the
// scan grid (the term kernels loop over further windows if the grid is capped).
static uint32_t terms_grid(uint32_t n) {
    const uint64_t b = ((uint64_t)n + kOwnSpan - 1) / kOwnSpan;
    return (uint32_t)(b < 1 ? 1 : b > 65535 ? 65535 : b);
}

struct PhaseKernels {
    kfn mark = nullptr, terms = nullptr, identify = nullptr, relax = nullptr, select = nullptr;
    int keyed = 0;  // keyed queue arrays: a launch may rebuild instead of running a phase
};


// Queue-array kernels for any criterion: the term pass over the entries when a
// criterion is dynamic, then identify with the static tests, the IN flag (3)
// and / or the dynamic OUT threshold (2). Keyed arrays: static criteria only.
template <int CH>
static PhaseKernels pick_queue(int in, int out, bool keyed) {
    const int i = in >= IN_SIMPLE_M ? 3 : in;
    const int o = out >= OUT_SIMPLE_M ? 2 : out;
    static const kfn tab[4][3] = {
        {nullptr, k_identify_queue<IN_NONE, 1, CH>, k_identify_queue<IN_NONE, 2, CH>},
        {k_identify_queue<IN_DIJK, 0, CH>, k_identify_queue<IN_DIJK, 1, CH>, k_identify_queue<IN_DIJK, 2, CH>},
        {k_identify_queue<IN_STATIC_M, 0, CH>, k_identify_queue<IN_STATIC_M, 1, CH>,
         k_identify_queue<IN_STATIC_M, 2, CH>},
        {k_identify_queue<3, 0, CH>, k_identify_queue<3, 1, CH>, k_identify_queue<3, 2, CH>}};
    static const kfn tabk[3][2] = {
        {nullptr, k_identify_queue<IN_NONE, 1, CH, true>},
        {k_identify_queue<IN_DIJK, 0, CH, true>, k_identify_queue<IN_DIJK, 1, CH, true>},
        {k_identify_queue<IN_STATIC_M, 0, CH, true>, k_identify_queue<IN_STATIC_M, 1, CH, true>}};
    PhaseKernels k;
    keyed = keyed && i < 3 && o < 2;
    k.identify = keyed ? tabk[i][o] : tab[i][o];
    k.terms = pick_terms(in, out);
    k.mark = pick_mark(in, out);
    k.keyed = keyed;
    k.relax = out == OUT_STATIC_M ? k_relax<CH, false, true, false, true> : k_relax<CH, false, false, false, true>;
    return k;
}

template <int CH>
static PhaseKernels pick_phase_ch(int in, int out, bool delta, bool learn, bool trace = false) {
    PhaseKernels k;
    if (trace && !delta) {
        k.terms = k_terms_trace;
        k.identify = k_identify_trace<CH>;
        k.relax = k_relax<CH, false, true, true>;
        return k;
    }
    if (delta) {
        k.identify = learn ? k_identify_delta<CH, true> : k_identify_delta<CH, false>;
        k.relax = learn ? k_relax<CH, true, false, true> : k_relax<CH, true, false, false>;
        if (learn) k.select = k_select_delta;
        return k;
    }
    if (learn) {
        k.terms = k_terms_learned;
        k.identify = k_identify_learned<CH>;
        k.relax = k_relax<CH, false, true, true>;
        return k;
    }
    k.terms = pick_terms(in, out);
    k.mark = pick_mark(in, out);
    k.identify = pick_identify<CH>(in, out);
    k.relax = out == OUT_STATIC_M ? k_relax<CH, false, true, false> : k_relax<CH, false, false, false>;
    return k;
}

static PhaseKernels pick_phase(int chunk, int in, int out, bool delta, bool learn, bool trace, bool queue = false,
                               bool keyed = false) {
    if (queue) {
        switch (chunk) {
        case 256: return pick_queue<256>(in, out, keyed);
        case 1024: return pick_queue<1024>(in, out, keyed);
        default: return pick_queue<512>(in, out, keyed);
        }
    }
    switch (chunk) {
    case 256: return pick_phase_ch<256>(in, out, delta, learn, trace);
    case 1024: return pick_phase_ch<1024>(in, out, delta, learn, trace);
    default: return pick_phase_ch<512>(in, out, delta, learn, trace);
    }
}

// Approximate criteria: their term pass, then identify with the IN flag (3) and/or the
// dynamic OUT threshold (2), DIJK otherwise implied (it implies both criteria).
template <int CH>
static PhaseKernels pick_approx_ch(uint32_t crit) {
    const bool in = crit & SSSP_IN_APPROX, out = crit & SSSP_OUT_APPROX;
    PhaseKernels k;
    k.terms = in ? (out ? k_terms_approx<true, true> : k_terms_approx<true, false>)
                 : (out ? k_terms_approx<false, true> : nullptr);
    k.identify = in ? (out ? k_identify<3, 2, CH> : k_identify<3, 0, CH>)
                    : (out ? k_identify<1, 2, CH> : k_identify<1, 0, CH>);
    if (in && !out && !(crit & SSSP_DIJK)) k.identify = k_identify<3, 0, CH>;
    if (!in && out && !(crit & SSSP_DIJK)) k.identify = k_identify<0, 2, CH>;
    k.relax = k_relax<CH, false, false, false>;
    return k;
}

static PhaseKernels pick_approx(int chunk, uint32_t crit) {
    switch (chunk) {
    case 256: return pick_approx_ch<256>(crit);
    case 1024: return pick_approx_ch<1024>(crit);
    default: return pick_approx_ch<512>(crit);
    }
}

static PhaseKernels pick_oracle(int chunk) {
    PhaseKernels k;
    switch (chunk) {
    case 256: k.identify = k_identify<kInOracle, 0, 256>; k.relax = k_relax<256, false, false, false>; break;
    case 1024: k.identify = k_identify<kInOracle, 0, 1024>; k.relax = k_relax<1024, false, false, false>; break;
    default: k.identify = k_identify<kInOracle, 0, 512>; k.relax = k_relax<512, false, false, false>; break;
    }
    return k;
}

static int valid_chunk(int c) { return c == 256 || c == 512 || c == 1024; }

// Phase loop with an event before and after every kernel (profiling): one
// batch at a time, durations summed over the non-empty phases. Phases k0 ..
// k_stop - 1 at most; a run that starts at k0 > 0 adds to the previous run's
// figures. On stopping at k_stop, *head gets the control header it left.
static int run_loop_profiled(sssp_graph *g, const KArgs &a, const PhaseKernels &K, uint64_t max_phases,
                             uint64_t k0, uint64_t k_stop, CtlHead *head) {
    constexpr uint32_t kBatch = 64;
    hipStream_t s = g->stream;
    if (g->pev_cap < 4 * kBatch) {
        g->pev = new (std::nothrow) hipEvent_t[4 * kBatch];
        if (!g->pev) return sssp_set_error(SSSP_ERR_OOM, "event pool");
        for (uint32_t i = 0; i < 4 * kBatch; ++i) HIP_OK(hipEventCreate(&g->pev[i]));
        g->pev_cap = 4 * kBatch;
    }
    sssp_kernel_profile pr{};
    if (k0) pr = g->last_prof;
    else g->phase_ms.clear();
    const dim3 blk(kBlock), gs(g->cfg.scan_blocks), gr(g->cfg.relax_blocks), gt(terms_grid(g->n));
    uint64_t k = k0;
    for (;;) {
        const uint64_t kb = k;
        for (uint32_t i = 0; i < kBatch && k < k_stop; ++i, ++k) {
            const int par = (int)(k % 6);
            hipEvent_t *e = &g->pev[4 * i];
            HIP_OK(hipEventRecord(e[0], s));
            if (K.mark) hipLaunchKernelGGL(K.mark, gt, blk, 0, s, a, par);
            if (K.terms) hipLaunchKernelGGL(K.terms, gt, blk, 0, s, a, par);
            HIP_OK(hipEventRecord(e[1], s));
            hipLaunchKernelGGL(K.identify, gs, blk, 0, s, a, par);
            HIP_OK(hipEventRecord(e[2], s));
            hipLaunchKernelGGL(K.relax, gr, blk, 0, s, a, par);
            if (K.select) hipLaunchKernelGGL(K.select, dim3(1), dim3(64), 0, s, a, par);
            HIP_OK(hipEventRecord(e[3], s));
        }
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(&g->h_ctl[0], a.b.ctl, sizeof(CtlHead), hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        const uint64_t real = g->h_ctl[0].phases + g->h_ctl[0].qrebuilds;  // launches that did work
        for (uint32_t i = 0; kb + i < k && kb + i < real; ++i) {
            float t0 = 0, t1 = 0, t2 = 0;
            hipEvent_t *e = &g->pev[4 * i];
            HIP_OK(hipEventElapsedTime(&t0, e[0], e[1]));
            HIP_OK(hipEventElapsedTime(&t1, e[1], e[2]));
            HIP_OK(hipEventElapsedTime(&t2, e[2], e[3]));
            pr.term_ms += K.terms ? t0 : 0.f;
            pr.identify_ms += t1;
            pr.relax_ms += t2;
            pr.phases++;
            g->phase_ms.push_back((K.terms ? t0 : 0.f) + t1 + t2);
        }
        if (g->h_ctl[0].done) {
            if (head) *head = g->h_ctl[0];  // F emptied before k_stop
            break;
        }
        if (k >= k_stop) {
            if (head) *head = g->h_ctl[0];
            break;
        }
        if (k > (K.keyed ? 2 : 1) * max_phases + 2 * kBatch)
            return sssp_set_error(SSSP_ERR_INTERNAL, "phase loop did not terminate after %llu phases",
                                  (unsigned long long)k);
    }
    g->last_prof = pr;
    return SSSP_OK;
}

// Six consecutive phases (every parity of the control slots) captured once
// into a HIP graph; re-captured only when the kernel arguments change.
constexpr int kGraphPhases = 6;

struct GraphKey {
    KArgs a;
    PhaseKernels K;
    LaunchCfg cfg;
};

static int ensure_phase_graph(sssp_graph *g, const KArgs &a, const PhaseKernels &K) {
    GraphKey key;
    memset(&key, 0, sizeof key);
    key.a = a;
    key.K = K;
    key.cfg = g->cfg;
    static_assert(sizeof(GraphKey) <= sizeof(g->graph_key), "graph key size");
    if (g->graph_exec && g->graph_key_len == sizeof key && memcmp(g->graph_key, &key, sizeof key) == 0)
        return SSSP_OK;
    if (g->graph_exec) (void)hipGraphExecDestroy(g->graph_exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    g->graph_exec = nullptr;
    g->graph = nullptr;
    g->graph_key_len = 0;
    if (!g->cap_stream) HIP_OK(hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking));
    hipStream_t cs = g->cap_stream;
    const dim3 blk(kBlock), gs(g->cfg.scan_blocks), gr(g->cfg.relax_blocks), gt(terms_grid(g->n));
    HIP_OK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    for (int par = 0; par < kGraphPhases; ++par) {
        if (K.mark) hipLaunchKernelGGL(K.mark, gt, blk, 0, cs, a, par);
        if (K.terms) hipLaunchKernelGGL(K.terms, gt, blk, 0, cs, a, par);
        hipLaunchKernelGGL(K.identify, gs, blk, 0, cs, a, par);
        hipLaunchKernelGGL(K.relax, gr, blk, 0, cs, a, par);
        if (K.select) hipLaunchKernelGGL(K.select, dim3(1), dim3(64), 0, cs, a, par);
    }
    hipError_t e = hipStreamEndCapture(cs, &g->graph);
    if (e != hipSuccess) return sssp_set_error(SSSP_ERR_DEVICE, "graph capture failed: %s", hipGetErrorString(e));
    HIP_OK(hipGraphInstantiate(&g->graph_exec, g->graph, nullptr, nullptr, 0));
    memcpy(g->graph_key, &key, sizeof key);
    g->graph_key_len = sizeof key;
    return SSSP_OK;
}

// Runs the phase loop: queues phases in growing batches, keeps one batch in
// flight while the host inspects the previous batch's copy of the control
// block, and stops once a batch ends with F empty. Phases k0 .. k_stop - 1 at
// most (a run may continue another one's phases); phases whose index is a
// multiple of six start a captured six-phase graph when graphs are enabled.
// On stopping at k_stop, *head gets the control header the last phase left.
static int run_loop(sssp_graph *g, const KArgs &a, const PhaseKernels &K, uint64_t max_phases, uint64_t k0 = 0,
                    uint64_t k_stop = UINT64_MAX, CtlHead *head = nullptr) {
    if (g->prof) return run_loop_profiled(g, a, K, max_phases, k0, k_stop, head);
    const bool graphs = g->cfg.use_graph;
    if (graphs) {
        int rc = ensure_phase_graph(g, a, K);
        if (rc) return rc;
    }
    hipStream_t s = g->stream;
    const dim3 blk(kBlock);
    const dim3 gs(g->cfg.scan_blocks), gr(g->cfg.relax_blocks), gt(terms_grid(g->n));
    uint64_t k = k0;
    uint32_t batch = graphs ? kGraphPhases : 4;
    int slot = 0;
    bool have_prev = false;
    for (;;) {
        for (uint32_t i = 0; i < batch && k < k_stop;) {
            if (graphs && k % kGraphPhases == 0 && k + kGraphPhases <= k_stop) {
                HIP_OK(hipGraphLaunch(g->graph_exec, s));
                i += kGraphPhases;
                k += kGraphPhases;
                continue;
            }
            const int par = (int)(k % 6);
            if (K.mark) hipLaunchKernelGGL(K.mark, gt, blk, 0, s, a, par);
            if (K.terms) hipLaunchKernelGGL(K.terms, gt, blk, 0, s, a, par);
            hipLaunchKernelGGL(K.identify, gs, blk, 0, s, a, par);
            hipLaunchKernelGGL(K.relax, gr, blk, 0, s, a, par);
            if (K.select) hipLaunchKernelGGL(K.select, dim3(1), dim3(64), 0, s, a, par);
            ++i;
            ++k;
        }
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(&g->h_ctl[slot], a.b.ctl, sizeof(CtlHead), hipMemcpyDeviceToHost, s));
        HIP_OK(hipEventRecord(g->ev[slot], s));
        if (k >= k_stop) {
            HIP_OK(hipEventSynchronize(g->ev[slot]));
            if (head) *head = g->h_ctl[slot];
            break;
        }
        if (have_prev) {
            HIP_OK(hipEventSynchronize(g->ev[slot ^ 1]));
            if (g->h_ctl[slot ^ 1].done) {
                if (head) *head = g->h_ctl[slot ^ 1];  // F emptied before k_stop
                break;
            }
        }
        have_prev = true;
        slot ^= 1;
        if (batch < 16) batch *= 2;
        if (k > (K.keyed ? 2 : 1) * max_phases + 2 * 64 + 8)  // keyed: at most one rebuild per phase
            return sssp_set_error(SSSP_ERR_INTERNAL, "phase loop did not terminate after %llu phases",
                                  (unsigned long long)k);
    }
    HIP_OK(hipStreamSynchronize(s));
    return SSSP_OK;
}

// First stage of a switched solve (sssp_solve_switch): plain launches in
// fixed batches of kSwitchBatch phases from phase k0 (0, or the end of a
// committed learned prefix). After queuing batch j the host reads
// the header copy of batch j - 1; once |F| there (at the start of that batch's
// last phase) is at most num/den of the largest |F| seen at an earlier check,
// and below it, batch j is the last one of this stage. The switch phase is
// therefore kSwitchBatch * (j + 1) whatever the timing. *k_next gets the index
// of the first phase not queued, *head the header after it (done set when the
// solve ended in this stage).
constexpr uint32_t kSwitchBatch = 16;

// Learned checkpoint mode (checkpoint = true): instead of the |F| rule, the
// k_select_checkpoint kernel runs after each batch's last phase and the first
// batch whose choice is not 0 (keep static) ends the stage in the same way.
static int run_until_drop(sssp_graph *g, const KArgs &a, const PhaseKernels &K, uint64_t max_phases, uint32_t num,
                          uint32_t den, uint64_t *k_next, CtlHead *head, uint64_t k0 = 0, bool checkpoint = false,
                          unsigned int *choice = nullptr) {
    hipStream_t s = g->stream;
    const dim3 blk(kBlock), gs(g->cfg.scan_blocks), gr(g->cfg.relax_blocks), gt(terms_grid(g->n));
    uint64_t k = k0;
    int slot = 0;
    bool have_prev = false;
    unsigned long long peak = 0;
    for (;;) {
        for (uint32_t i = 0; i < kSwitchBatch; ++i, ++k) {
            const int par = (int)(k % 6);
            if (K.mark) hipLaunchKernelGGL(K.mark, gt, blk, 0, s, a, par);
            if (K.terms) hipLaunchKernelGGL(K.terms, gt, blk, 0, s, a, par);
            hipLaunchKernelGGL(K.identify, gs, blk, 0, s, a, par);
            hipLaunchKernelGGL(K.relax, gr, blk, 0, s, a, par);
        }
        if (checkpoint) hipLaunchKernelGGL(k_select_checkpoint, dim3(1), dim3(64), 0, s, a, (int)((k - 1) % 6));
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(&g->h_ctl[slot], a.b.ctl, sizeof(CtlHead), hipMemcpyDeviceToHost, s));
        HIP_OK(hipEventRecord(g->ev[slot], s));
        if (have_prev) {
            HIP_OK(hipEventSynchronize(g->ev[slot ^ 1]));
            const CtlHead &h = g->h_ctl[slot ^ 1];
            const unsigned long long f = h.fk;
            const bool decide = checkpoint ? h.cp_choice != 0
                                           : peak && f < peak && (unsigned __int128)f * den <= (unsigned __int128)peak * num;
            if (h.done || decide) {
                if (choice) *choice = h.cp_choice;  // the deciding checkpoint's choice
                HIP_OK(hipEventSynchronize(g->ev[slot]));
                *head = g->h_ctl[slot];
                *k_next = k;
                return SSSP_OK;
            }
            if (f > peak) peak = f;
        }
        have_prev = true;
        slot ^= 1;
        if (k > max_phases + 2 * kSwitchBatch)
            return sssp_set_error(SSSP_ERR_INTERNAL, "phase loop did not terminate after %llu phases",
                                  (unsigned long long)k);
    }
}

static unsigned long long shard_sum(const Sharded &x) {
    unsigned long long t = 0;
    for (int i = 0; i < kShards; ++i) t += x.v[i * kPad];
    return t;
}

// Copies the whole control block once at the end of a solve and checks the
// end state: F empty, and every vertex ever queued settled.
// The control block's header and its first three sharded sums, the part a finished
// solve reports (laid out first in Ctl, so one short copy fetches them).
struct CtlPrefix {
    CtlHead h;
    Sharded reached, relax_edges, improving;
};
static_assert(offsetof(Ctl, reached) == offsetof(CtlPrefix, reached) &&
                  offsetof(Ctl, improving) == offsetof(CtlPrefix, improving) &&
                  sizeof(CtlPrefix) <= offsetof(Ctl, spack) + 0,
              "finish_stats copies a prefix of Ctl");

static int finish_stats(const sssp_graph *g, const Ctl *dctl, sssp_stats *st, uint32_t *phases) {
    CtlPrefix pre;
    const CtlPrefix *c = &pre;
    // on the solve's stream: the copy waits for this solve only, not for other streams' work
    hipError_t e = hipMemcpyAsync(&pre, dctl, sizeof(CtlPrefix), hipMemcpyDeviceToHost, g->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->stream);
    if (e != hipSuccess) return sssp_set_error(SSSP_ERR_DEVICE, "control block copy: %s", hipGetErrorString(e));
    const unsigned long long reached = shard_sum(c->reached);
    int rc = SSSP_OK;
    if (c->h.stalled)
        rc = sssp_set_error(SSSP_ERR_INVALID, "a phase certified no vertex although F was not empty: the ORACLE "
                                              "reference is not dist(source, .) of this graph");
    else if (!c->h.done || reached != c->h.settled)
        rc = sssp_set_error(SSSP_ERR_INTERNAL, "solve ended in an inconsistent state (done=%u reached=%llu settled=%llu)",
                            c->h.done, reached, c->h.settled);
    if (phases) *phases = c->h.phases;
    if (st) {
        st->phases = c->h.phases;
        st->buckets = c->h.buckets;
        st->sum_f = c->h.sum_f;
        st->n_reach = c->h.settled;
        st->m_reach = c->h.m_reach;
        st->relax_edges = shard_sum(c->relax_edges);
        st->improving = shard_sum(c->improving);
        st->precompute_ns = g->precompute_ns;
    }
    return rc;
}

// A switched solve's second criterion and the fraction of the peak |F| at
// which it takes over.
// mode 0: the |F| rule (num/den of the peak); mode 1: at phase `at` (a fixed
// schedule); mode 2: when the selector's checkpoint choice is not static, to
// the criterion it chose (learned checkpoint mode; crit_then names the
// strongest criterion that may follow, for buffer set-up).
struct SwitchReq {
    uint32_t crit_then, num, den;
    uint32_t at = 0;
    int mode = 0;
};

static int solve_common(sssp_graph *g, uint32_t source, bool delta_mode, uint32_t crit,
                        const uint64_t *deltas, uint32_t n_deltas, uint64_t *dist_out,
                        sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace,
                        uint32_t trace_cap, const sssp_selector *sel = nullptr, float *feat_host = nullptr,
                        uint32_t *cf_host = nullptr, const uint64_t *oracle_ref = nullptr, uint32_t commit = 0,
                        const SwitchReq *sw = nullptr, const uint32_t *apx = nullptr) {
    const bool ckpt = sw && sw->mode == 2;  // the selector only chooses at checkpoints
    const bool learn = sel != nullptr && !ckpt;
    const bool oracle = oracle_ref != nullptr;
    const bool trace_mode = learn && !delta_mode && cf_host != nullptr;
    if (!g) return sssp_set_error(SSSP_ERR_INVALID, "graph is NULL");
    if (!dist_out) return sssp_set_error(SSSP_ERR_INVALID, "dist_out is NULL");
    if (source >= g->n) return sssp_set_error(SSSP_ERR_INVALID, "source %u >= n = %u", source, g->n);
    if (trace_cap && !trace) return sssp_set_error(SSSP_ERR_INVALID, "trace is NULL but trace_cap > 0");
    if (commit && (!learn || delta_mode || trace_mode))
        return sssp_set_error(SSSP_ERR_INVALID, "commit applies to the learned phased solver only");
    int in = IN_NONE, out = OUT_NONE;
    if (learn && !delta_mode) {
        in = IN_SIMPLE_M;  // any of the three criteria may be chosen: CSC and cursors are needed
        out = OUT_SIMPLE_M;
    } else if (learn) {
        // bucket widths come from the selector
    } else if (oracle) {
        // ORACLE: no term pass, no thresholds
    } else if (apx) {
        // approximate criteria: their own term pass (pick_approx)
        if (crit == 0 || (crit & ~(SSSP_DIJK | SSSP_IN_APPROX | SSSP_OUT_APPROX)))
            return sssp_set_error(SSSP_ERR_INVALID, "criterion 0x%x: the approximate solve takes DIJK, IN_APPROX "
                                                    "and OUT_APPROX", crit);
    } else if (!delta_mode) {
        if (crit == 0 || (crit & ~SSSP_CRIT_ALL))
            return sssp_set_error(SSSP_ERR_INVALID, "criterion 0x%x is empty or has unknown bits", crit);
        crit_modes(crit, &in, &out);
    } else {
        if (!deltas || n_deltas == 0) return sssp_set_error(SSSP_ERR_INVALID, "no bucket width given");
        for (uint32_t i = 0; i < n_deltas; ++i)
            if (deltas[i] == 0) return sssp_set_error(SSSP_ERR_INVALID, "bucket width must be >= 1");
    }
    int in2 = IN_NONE, out2 = OUT_NONE;  // switched solves: the second stage's modes
    if (sw) {
        // plain: crit is the first stage's criterion; learned: the committed choice, if static
        if (learn ? (delta_mode || trace_mode || !commit) : (oracle || delta_mode || !static_modes(in, out)))
            return sssp_set_error(SSSP_ERR_INVALID, "the first criterion of a switched solve must be made of "
                                                    "DIJK, IN_STATIC and OUT_STATIC");
        if (sw->crit_then == 0 || (sw->crit_then & ~SSSP_CRIT_ALL))
            return sssp_set_error(SSSP_ERR_INVALID, "criterion 0x%x is empty or has unknown bits", sw->crit_then);
        if (sw->mode == 0 && (sw->num == 0 || sw->den < sw->num))
            return sssp_set_error(SSSP_ERR_INVALID, "drop fraction %u/%u is not in (0, 1]", sw->num, sw->den);
        if (ckpt && !sel) return sssp_set_error(SSSP_ERR_INVALID, "selector is NULL");
        crit_modes(sw->crit_then, &in2, &out2);
        if (out2 == OUT_STATIC_M && out != OUT_STATIC_M && !learn)
            return sssp_set_error(SSSP_ERR_INVALID, "OUT_STATIC after the switch needs OUT_STATIC before it");
    }
    if (!valid_chunk(g->cfg.chunk)) return sssp_set_error(SSSP_ERR_INTERNAL, "bad chunk size");
    HIP_OK(hipSetDevice(g->device));
    const int in_all = in > in2 ? in : in2, out_all = out > out2 ? out : out2;  // both stages' needs
    const bool dyn = in_all >= IN_SIMPLE_M || out_all >= OUT_SIMPLE_M;
    // queue arrays: plain static criteria, or the plain static phases after a committed prefix
    // (a scan block's state window must fit in LDS: at most kQWin vertices per block)
    const bool queue_fits = g->cfg.queue && scan_span(g->n, g->cfg.scan_blocks, 16) <= kQWin;
    const bool queue_now = queue_fits && !learn && !oracle && !apx && !delta_mode;
    const bool queue_later = queue_fits && (commit != 0 || sw);
    // stored full terms (dirty-set pass) for IN (full), OUTWEAK and OUT (full) in the plain kernels;
    // the pass walks in-edges for the OUT terms
    auto stores = [](int i, int o) { return i == IN_FULL_M || o == OUT_WEAK_M || o == OUT_FULL_M; };
    const bool store = !learn && !trace_mode && !oracle && !apx && !delta_mode && (stores(in, out) || stores(in2, out2));
    if (in_all >= IN_SIMPLE_M || (apx && (crit & SSSP_IN_APPROX)) || store) {
        int rc = graph_ensure_csc(g);
        if (rc) return rc;
    }
    if (dyn) {  // the cursors walk each row lightest edge first
        int rc = graph_ensure_sorted(g);
        if (rc) return rc;
    }
    int rc = solve_bufs_ensure(g, dyn, delta_mode, queue_now || queue_later, apx != nullptr, store);
    if (rc) return rc;
    if (learn) n_deltas = 0;
    if (delta_mode && g->delta_cap < n_deltas) {
        sssp_free(g->b.deltas);
        g->b.deltas = nullptr;
        HIP_OK(hipMalloc(&g->b.deltas, n_deltas * sizeof(unsigned long long)));
        g->delta_cap = n_deltas;
    }
    hipStream_t s = g->stream;
    if (delta_mode && n_deltas)
        HIP_OK(hipMemcpyAsync(g->b.deltas, deltas, n_deltas * sizeof(uint64_t), hipMemcpyHostToDevice, s));
    KArgs a;
    a.g = dev_view(g);
    a.b = g->b;
    a.b.dist = (unsigned long long *)dist_out;
    a.b.phase_of = phase_of;
    if (apx) {  // the approximate term pass reads every vertex's settle phase
        if (!phase_of) a.b.phase_of = a.b.apx_sp;
        a.b.apx_sp = a.b.phase_of;
    }
    a.b.trace = nullptr;
    a.b.trace_cap = 0;
    a.crit = crit;
    a.approx_k = apx ? *apx : 0u;
    a.mark = !learn && !trace_mode && !oracle && !apx && !delta_mode && stores(in, out);
    a.fresh_at = 0;
    a.mlp_w = sel ? selector_device_weights(sel) : nullptr;
    a.wm = g->m ? (double)g->sum_w / (double)g->m : 1.0;
    a.ref = (const unsigned long long *)oracle_ref;
    a.b.trace_feat = nullptr;
    a.b.trace_cf = nullptr;
    CallBuffer trace_buf, feat_buf, cf_buf;  // freed on every return below
    if (trace_cap) {
        HIP_OK(hipMalloc(&trace_buf.p, (uint64_t)trace_cap * sizeof(PhaseRec)));
        a.b.trace = (PhaseRec *)trace_buf.p;
        a.b.trace_cap = trace_cap;
        if (feat_host) HIP_OK(hipMalloc(&feat_buf.p, (uint64_t)trace_cap * kMlpIn * sizeof(float)));
        if (cf_host) HIP_OK(hipMalloc(&cf_buf.p, (uint64_t)trace_cap * 3 * sizeof(uint32_t)));
        a.b.trace_feat = (float *)feat_buf.p;
        a.b.trace_cf = (uint32_t *)cf_buf.p;
    }
    const int ib = (int)(((uint64_t)g->n + 255) / 256 > 8192 ? 8192 : ((uint64_t)g->n + 255) / 256);
    hipLaunchKernelGGL(k_init_state, dim3(ib), dim3(256), 0, s, g->n, source, a.b.dist, a.b.st, a.b.phase_of,
                       dyn ? a.b.out_cur : nullptr, g->rp, (in_all >= IN_SIMPLE_M) ? a.b.in_cur : nullptr,
                       g->ip, delta_mode ? a.b.stamp : nullptr, a.b.out_head, g->edges, a.b.in_head, g->in_edges);
    // keyed queue arrays: the first split lies a sixteenth of the mean weight above T (or minD)
    const unsigned long long qdelta0 = g->m ? (g->sum_w / g->m) / 16 + 1 : 1;
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, a.b.ctl, g->vmin, g->rp, g->wmax, source, n_deltas,
                       qdelta0);
    if (learn) hipLaunchKernelGGL(k_init_choice, dim3(1), dim3(64), 0, s, a, source, (int)delta_mode);
    if (apx) hipLaunchKernelGGL(k_fill_u32, dim3(ib), dim3(256), 0, s, g->n, a.b.apx_lin, a.b.apx_lout, 0u);
    const PhaseKernels K = oracle ? pick_oracle(g->cfg.chunk)
                         : apx ? pick_approx(g->cfg.chunk, crit)
                                  : pick_phase(g->cfg.chunk, in, out, delta_mode, learn, trace_mode, queue_now,
                                               // keyed: launches and phases differ, so not where the host
                                               // counts phases by launches (switched and committed solves)
                                               queue_now && g->cfg.queue == 2 && !sw && !commit &&
                                                   static_modes(in, out));
    // phases <= reachable vertices; Delta rounds <= 2 * n + light rounds bounded by n per bucket
    // Delta: light rounds per bucket <= window vertices + 1, one heavy round per bucket
    const uint64_t max_phases = delta_mode ? 4ull * g->n + 64 : (uint64_t)g->n + 2;
    uint32_t cp_rows = 0;  // checkpoint mode: feature rows written (one per checkpoint)
    if (commit) {
        // the selector chooses phases 0 .. commit - 1 one by one (queued without
        // graphs: they are few), then the rest run the plain kernels of the
        // criterion it chose for phase `commit`
        CtlHead h{};
        const bool graphs = g->cfg.use_graph;
        g->cfg.use_graph = false;
        rc = run_loop(g, a, K, max_phases, 0, commit, &h);
        g->cfg.use_graph = graphs;
        if (rc == SSSP_OK && !h.done) {
            KArgs a2 = a;
            a2.crit = choice_criterion(h.choice[commit & 1]);
            a2.mlp_w = nullptr;
            int ic = IN_NONE, oc = OUT_NONE;
            crit_modes(a2.crit, &ic, &oc);
            // the first queue-array phase rebuilds the arrays from the state bytes (qlive = 0)
            const bool q2 = queue_later;
            const PhaseKernels K2 = pick_phase(g->cfg.chunk, ic, oc, false, false, false, q2);
            if (sw && static_modes(ic, oc)) {
                // committed to the static criterion: switch to the second criterion once F has
                // fallen to the given fraction of its peak (batch boundaries counted from commit)
                CtlHead h2{};
                uint64_t k_next = commit;
                const bool prof = g->prof;
                g->prof = false;
                rc = run_until_drop(g, a2, K2, max_phases, sw->num, sw->den, &k_next, &h2, commit);
                if (rc == SSSP_OK && !h2.done) {
                    KArgs a3 = a2;
                    a3.crit = sw->crit_then;
                    a3.mark = stores(in2, out2);
                    a3.fresh_at = (uint32_t)k_next;
                    rc = run_loop(g, a3, pick_phase(g->cfg.chunk, in2, out2, false, false, false,
                                                    queue_fits),
                                  max_phases, k_next);
                }
                g->prof = prof;
            } else {
                rc = run_loop(g, a2, K2, max_phases, commit);
            }
        }
    } else if (sw) {
        // static phases until F has fallen to the given fraction of its peak (or until phase
        // sw->at, or until the selector chooses at a checkpoint), then the second criterion's
        // plain kernels (no per-kernel timing: both stages use plain launches)
        const bool prof = g->prof;
        g->prof = false;
        CtlHead h{};
        uint64_t k_next = 0;
        unsigned int choice = 0;
        if (sw->mode == 1) {
            const bool graphs = g->cfg.use_graph;
            g->cfg.use_graph = false;
            rc = sw->at ? run_loop(g, a, K, max_phases, 0, sw->at, &h) : SSSP_OK;
            g->cfg.use_graph = graphs;
            k_next = sw->at;
        } else {
            rc = run_until_drop(g, a, K, max_phases, sw->num, sw->den, &k_next, &h, 0, ckpt, &choice);
        }
        if (ckpt) cp_rows = (uint32_t)(k_next / kSwitchBatch);
        if (rc == SSSP_OK && !h.done) {
            KArgs a2 = a;
            a2.crit = ckpt ? choice_criterion(choice) : sw->crit_then;
            int i2 = in2, o2 = out2;
            if (ckpt) crit_modes(a2.crit, &i2, &o2);
            a2.mark = stores(i2, o2);
            a2.fresh_at = (uint32_t)k_next;
            const bool q2 = queue_later;
            rc = run_loop(g, a2, pick_phase(g->cfg.chunk, i2, o2, false, false, false, q2), max_phases, k_next);
        }
        g->prof = prof;
    } else {
        rc = run_loop(g, a, K, max_phases);
    }
    if (rc == SSSP_OK) {
        hipLaunchKernelGGL(k_clear_settled, dim3(ib), dim3(256), 0, s, g->n, a.b.dist);
        HIP_OK(hipGetLastError());
        HIP_OK(hipStreamSynchronize(s));
    }
    uint32_t phases = 0;
    if (rc == SSSP_OK) rc = finish_stats(g, a.b.ctl, stats, &phases);
    if (rc == SSSP_OK && trace_cap) {
        const uint32_t cnt = phases < trace_cap ? phases : trace_cap;
        const uint32_t fcnt = delta_mode ? (stats ? stats->buckets : 0) : ckpt ? (cp_rows < phases / kSwitchBatch ? cp_rows : phases / kSwitchBatch) : cnt;
        const uint32_t fc = fcnt < trace_cap ? fcnt : trace_cap;
        hipError_t e = hipSuccess;
        if (cnt) e = hipMemcpyAsync(trace, a.b.trace, cnt * sizeof(PhaseRec), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && feat_host && fc)
            e = hipMemcpyAsync(feat_host, a.b.trace_feat, (uint64_t)fc * kMlpIn * sizeof(float), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess && cf_host && cnt)
            e = hipMemcpyAsync(cf_host, a.b.trace_cf, (uint64_t)cnt * 3 * sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) rc = sssp_set_error(SSSP_ERR_DEVICE, "trace copy failed: %s", hipGetErrorString(e));
    }
    return rc;
}

extern "C" int sssp_solve(sssp_graph *g, uint32_t source, uint32_t criterion, uint64_t *dist_out,
                          uint32_t *phases_out) {
    if (g && g->cfg.single && criterion != 0 && !(criterion & ~SSSP_CRIT_ALL)) {
        int in = IN_NONE, out = OUT_NONE;
        crit_modes(criterion, &in, &out);
        if (static_modes(in, out)) {  // the whole solve in one workgroup (the batched kernel)
            if (!dist_out) return sssp_set_error(SSSP_ERR_INVALID, "dist_out is NULL");
            if (source >= g->n) return sssp_set_error(SSSP_ERR_INVALID, "source %u >= n = %u", source, g->n);
            HIP_OK(hipSetDevice(g->device));
            return batch_solve_one(g, source, in, out == OUT_STATIC_M, dist_out, phases_out);
        }
    }
    sssp_stats st;
    int rc = solve_common(g, source, false, criterion, nullptr, 0, dist_out, &st, nullptr, nullptr, 0);
    if (rc == SSSP_OK && phases_out) *phases_out = st.phases;
    return rc;
}

extern "C" int sssp_solve_ex(sssp_graph *g, uint32_t source, uint32_t criterion, uint64_t *dist_out,
                             sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace,
                             uint32_t trace_cap) {
    return solve_common(g, source, false, criterion, nullptr, 0, dist_out, stats, phase_of, trace, trace_cap);
}

extern "C" int sssp_delta_step(sssp_graph *g, uint32_t source, uint64_t delta, uint64_t *dist_out,
                               uint32_t *phases_out) {
    if (delta == 0) return sssp_set_error(SSSP_ERR_INVALID, "delta must be >= 1");
    sssp_stats st;
    int rc = solve_common(g, source, true, 0, &delta, 1, dist_out, &st, nullptr, nullptr, 0);
    if (rc == SSSP_OK && phases_out) *phases_out = st.phases;
    return rc;
}

extern "C" int sssp_delta_step_ex(sssp_graph *g, uint32_t source, const uint64_t *deltas, uint32_t n_deltas,
                                  uint64_t *dist_out, sssp_stats *stats, sssp_phase_rec *trace,
                                  uint32_t trace_cap) {
    return solve_common(g, source, true, 0, deltas, n_deltas, dist_out, stats, nullptr, trace, trace_cap);
}

extern "C" int sssp_solve_oracle(sssp_graph *g, uint32_t source, const uint64_t *dist_ref, uint64_t *dist_out,
                                 sssp_stats *stats, uint32_t *phase_of) {
    if (!dist_ref) return sssp_set_error(SSSP_ERR_INVALID, "dist_ref is NULL");
    return solve_common(g, source, false, 0, nullptr, 0, dist_out, stats, phase_of, nullptr, 0, nullptr, nullptr,
                        nullptr, dist_ref);
}

extern "C" int sssp_solve_approx(sssp_graph *g, uint32_t source, uint32_t criterion, uint32_t k,
                                 uint64_t *dist_out, sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace,
                                 uint32_t trace_cap) {
    return solve_common(g, source, false, criterion, nullptr, 0, dist_out, stats, phase_of, trace, trace_cap,
                        nullptr, nullptr, nullptr, nullptr, 0, nullptr, &k);
}

extern "C" int sssp_profile_enable(sssp_graph *g, int enable) {
    if (!g) return sssp_set_error(SSSP_ERR_INVALID, "graph is NULL");
    g->prof = enable != 0;
    return SSSP_OK;
}

extern "C" int sssp_profile_get(const sssp_graph *g, sssp_kernel_profile *out) {
    if (!g || !out) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    *out = g->last_prof;
    return SSSP_OK;
}

extern "C" int sssp_profile_phases(const sssp_graph *g, float *ms, uint32_t cap, uint32_t *count) {
    if (!g || !count || (cap && !ms)) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    const size_t k = g->phase_ms.size();
    *count = (uint32_t)k;
    for (size_t i = 0; i < k && i < cap; ++i) ms[i] = g->phase_ms[i];
    return SSSP_OK;
}

extern "C" int sssp_get_launch(const sssp_graph *g, sssp_launch_cfg *out) {
    if (!g || !out) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    out->scan_blocks = (uint32_t)g->cfg.scan_blocks;
    out->relax_blocks = (uint32_t)g->cfg.relax_blocks;
    out->chunk = (uint32_t)g->cfg.chunk;
    out->use_graph = (uint32_t)g->cfg.use_graph;
    out->queue = (uint32_t)g->cfg.queue;
    out->single = (uint32_t)g->cfg.single;
    return SSSP_OK;
}

extern "C" int sssp_set_launch(sssp_graph *g, const sssp_launch_cfg *cfg) {
    if (!g || !cfg) return sssp_set_error(SSSP_ERR_INVALID, "NULL argument");
    if (cfg->scan_blocks == 0 || cfg->relax_blocks == 0 || cfg->scan_blocks > (1u << 20) ||
        cfg->relax_blocks > (1u << 20) || !valid_chunk((int)cfg->chunk) || cfg->queue > 2)
        return sssp_set_error(SSSP_ERR_INVALID, "bad launch shape (%u, %u, %u)", cfg->scan_blocks,
                              cfg->relax_blocks, cfg->chunk);
    g->cfg.scan_blocks = (int)cfg->scan_blocks;
    g->cfg.relax_blocks = (int)cfg->relax_blocks;
    g->cfg.chunk = (int)cfg->chunk;
    g->cfg.use_graph = cfg->use_graph != 0;
    g->cfg.queue = (int)cfg->queue;
    g->cfg.single = cfg->single != 0;
    return SSSP_OK;
}

extern "C" int sssp_solve_learned(sssp_graph *g, uint32_t source, const sssp_selector *sel, uint64_t *dist_out,
                                  sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap) {
    if (!sel) return sssp_set_error(SSSP_ERR_INVALID, "selector is NULL");
    return solve_common(g, source, false, 0, nullptr, 0, dist_out, stats, phase_of, trace, trace_cap, sel);
}

extern "C" int sssp_solve_learned_commit(sssp_graph *g, uint32_t source, const sssp_selector *sel,
                                         uint32_t commit_phase, uint64_t *dist_out, sssp_stats *stats,
                                         uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap) {
    if (!sel) return sssp_set_error(SSSP_ERR_INVALID, "selector is NULL");
    if (commit_phase == 0) return sssp_set_error(SSSP_ERR_INVALID, "commit_phase must be >= 1");
    return solve_common(g, source, false, 0, nullptr, 0, dist_out, stats, phase_of, trace, trace_cap, sel, nullptr,
                        nullptr, nullptr, commit_phase);
}

extern "C" int sssp_solve_switch(sssp_graph *g, uint32_t source, uint32_t crit_first, uint32_t crit_then,
                                 uint32_t drop_num, uint32_t drop_den, uint64_t *dist_out, sssp_stats *stats,
                                 uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap) {
    const SwitchReq sw{crit_then, drop_num, drop_den};
    return solve_common(g, source, false, crit_first, nullptr, 0, dist_out, stats, phase_of, trace, trace_cap,
                        nullptr, nullptr, nullptr, nullptr, 0, &sw);
}

extern "C" int sssp_solve_learned_switch(sssp_graph *g, uint32_t source, const sssp_selector *sel,
                                         uint32_t commit_phase, uint32_t crit_then, uint32_t drop_num,
                                         uint32_t drop_den, uint64_t *dist_out, sssp_stats *stats, uint32_t *phase_of,
                                         sssp_phase_rec *trace, uint32_t trace_cap) {
    if (!sel) return sssp_set_error(SSSP_ERR_INVALID, "selector is NULL");
    if (commit_phase == 0) return sssp_set_error(SSSP_ERR_INVALID, "commit_phase must be >= 1");
    const SwitchReq sw{crit_then, drop_num, drop_den};
    return solve_common(g, source, false, 0, nullptr, 0, dist_out, stats, phase_of, trace, trace_cap, sel, nullptr,
                        nullptr, nullptr, commit_phase, &sw);
}

extern "C" int sssp_solve_schedule(sssp_graph *g, uint32_t source, uint32_t crit_first, uint32_t crit_then,
                                   uint32_t switch_phase, uint64_t *dist_out, sssp_stats *stats, uint32_t *phase_of,
                                   sssp_phase_rec *trace, uint32_t trace_cap) {
    SwitchReq sw{crit_then, 1, 1};
    sw.at = switch_phase;
    sw.mode = 1;
    return solve_common(g, source, false, crit_first, nullptr, 0, dist_out, stats, phase_of, trace, trace_cap,
                        nullptr, nullptr, nullptr, nullptr, 0, &sw);
}

extern "C" int sssp_solve_learned_checkpoint(sssp_graph *g, uint32_t source, const sssp_selector *sel,
                                             uint64_t *dist_out, sssp_stats *stats, uint32_t *phase_of,
                                             sssp_phase_rec *trace, uint32_t trace_cap, float *features_out) {
    if (!sel) return sssp_set_error(SSSP_ERR_INVALID, "selector is NULL");
    if (features_out && !trace_cap) return sssp_set_error(SSSP_ERR_INVALID, "features_out needs trace_cap > 0");
    SwitchReq sw{SSSP_IN_SIMPLE | SSSP_OUT_SIMPLE | SSSP_OUT_STATIC, 1, 1};
    sw.mode = 2;
    if (!trace && features_out) {
        // feature rows ride on the trace buffers: keep a host trace of trace_cap records here
        std::vector<sssp_phase_rec> tmp(trace_cap);
        return solve_common(g, source, false, SSSP_IN_STATIC | SSSP_OUT_STATIC, nullptr, 0, dist_out, stats,
                            phase_of, tmp.data(), trace_cap, sel, features_out, nullptr, nullptr, 0, &sw);
    }
    return solve_common(g, source, false, SSSP_IN_STATIC | SSSP_OUT_STATIC, nullptr, 0, dist_out, stats, phase_of,
                        trace, trace ? trace_cap : 0, sel, features_out, nullptr, nullptr, 0, &sw);
}

extern "C" int sssp_delta_step_learned(sssp_graph *g, uint32_t source, const sssp_selector *sel, uint64_t *dist_out,
                                       sssp_stats *stats, sssp_phase_rec *trace, uint32_t trace_cap) {
    if (!sel) return sssp_set_error(SSSP_ERR_INVALID, "selector is NULL");
    return solve_common(g, source, true, 0, nullptr, 0, dist_out, stats, nullptr, trace, trace_cap, sel);
}

extern "C" int sssp_trace_learned(sssp_graph *g, uint32_t source, const sssp_selector *sel, int delta_mode,
                                  uint64_t *dist_out, sssp_stats *stats, uint32_t trace_cap, sssp_phase_rec *trace,
                                  float *features_out, uint32_t *counts_out) {
    if (!sel) return sssp_set_error(SSSP_ERR_INVALID, "selector is NULL");
    if (!trace_cap || !trace || !features_out || (!delta_mode && !counts_out))
        return sssp_set_error(SSSP_ERR_INVALID, "trace buffers missing");
    sssp_stats st;
    int rc = solve_common(g, source, delta_mode != 0, 0, nullptr, 0, dist_out, &st, nullptr, trace, trace_cap, sel,
                          features_out, delta_mode ? nullptr : counts_out);
    if (stats) *stats = st;
    return rc;
}

// ---------------------------------------------------------------------------
// Allocation-free solve (sssp_solve_noalloc): the plain static-criterion phase
// loop (dense scan identify + relax, the kernels of sssp_solve) with its
// per-solve scratch -- control block, state bytes, S' shards, chunk starts --
// carved from one file-scope device array instead of graph-owned buffers.

constexpr uint64_t kNoAllocBytes = 64ull << 20;  // per device, held until the process ends
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

constexpr int kNoAllocMaxDev = 64;
static void *g_noalloc_ptr[kNoAllocMaxDev];     // device address of `scratch`, per device
static std::mutex g_noalloc_mu[kNoAllocMaxDev]; // calls on one device share its array

struct NoAllocLayout {
    uint64_t ctl, st, srow, soff, sdu, chunk, total;
    uint32_t shard_cap, chunk_cap;
};

static uint64_t align256(uint64_t x) { return (x + 255) & ~255ull; }

static NoAllocLayout noalloc_layout(uint32_t n, uint64_t m, int scan_blocks) {
    NoAllocLayout L;
    // dense scan only: a shard holds the S' entries of ceil(G / kShards) blocks of at most
    // scan_span(n, G, 4) vertices each
    L.shard_cap = (uint32_t)(((uint64_t)scan_blocks + kShards - 1) / kShards * scan_span(n, scan_blocks, 4));
    L.chunk_cap = (uint32_t)(m / 256 + 2);
    const uint64_t sent = (uint64_t)kShards * L.shard_cap;
    uint64_t o = 0;
    L.ctl = o;   o = align256(o + sizeof(Ctl));
    L.st = o;    o = align256(o + (((uint64_t)n + 15) & ~15ull));
    L.srow = o;  o = align256(o + sent * 4);
    L.soff = o;  o = align256(o + sent * 4);
    L.sdu = o;   o = align256(o + sent * 8);
    L.chunk = o; o = align256(o + (uint64_t)kShards * L.chunk_cap * 4);
    L.total = o;
    return L;
}

// Device address of `scratch` on device dev, looked up once per device with
// that device current (each device holds its own copy at its own address).
static int noalloc_scratch(int dev, unsigned char **out) {
    if (dev < 0 || dev >= kNoAllocMaxDev) return sssp_set_error(SSSP_ERR_UNSUPPORTED, "device %d out of range", dev);
    if (!g_noalloc_ptr[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return sssp_set_error(SSSP_ERR_DEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_noalloc_ptr[dev] = p;
    }
    *out = (unsigned char *)g_noalloc_ptr[dev];
    return SSSP_OK;
}

extern "C" int sssp_solve_noalloc(sssp_graph *g, uint32_t source, uint32_t criterion, uint64_t *dist_out,
                                  uint32_t *phases_out) {
    if (!g) return sssp_set_error(SSSP_ERR_INVALID, "graph is NULL");
    if (!dist_out) return sssp_set_error(SSSP_ERR_INVALID, "dist_out is NULL");
    if (source >= g->n) return sssp_set_error(SSSP_ERR_INVALID, "source %u >= n = %u", source, g->n);
    if (criterion == 0 || (criterion & ~SSSP_CRIT_ALL))
        return sssp_set_error(SSSP_ERR_INVALID, "criterion 0x%x is empty or has unknown bits", criterion);
    int in = IN_NONE, out = OUT_NONE;
    crit_modes(criterion, &in, &out);
    if (!static_modes(in, out))
        return sssp_set_error(SSSP_ERR_UNSUPPORTED, "sssp_solve_noalloc evaluates DIJK, IN_STATIC and OUT_STATIC");
    if (!valid_chunk(g->cfg.chunk)) return sssp_set_error(SSSP_ERR_INTERNAL, "bad chunk size");
    const NoAllocLayout L = noalloc_layout(g->n, g->m, g->cfg.scan_blocks);
    if (L.total > kNoAllocBytes)
        return sssp_set_error(SSSP_ERR_UNSUPPORTED,
                              "sssp_solve_noalloc: the graph needs %llu bytes of scratch, more than its %llu "
                              "(n = %u, m = %llu, %d scan blocks)", (unsigned long long)L.total,
                              (unsigned long long)kNoAllocBytes, g->n, (unsigned long long)g->m, g->cfg.scan_blocks);
    HIP_OK(hipSetDevice(g->device));
    if (g->device < 0 || g->device >= kNoAllocMaxDev)
        return sssp_set_error(SSSP_ERR_UNSUPPORTED, "device %d out of range", g->device);
    std::lock_guard<std::mutex> lock(g_noalloc_mu[g->device]);
    unsigned char *base = nullptr;
    int rc = noalloc_scratch(g->device, &base);
    if (rc) return rc;
    KArgs a;
    memset(&a, 0, sizeof a);
    a.g = dev_view(g);
    a.b.ctl = (Ctl *)(base + L.ctl);
    a.b.st = base + L.st;
    a.b.srow = (uint32_t *)(base + L.srow);
    a.b.soff = (uint32_t *)(base + L.soff);
    a.b.sdu = (unsigned long long *)(base + L.sdu);
    a.b.chunk_start = (uint32_t *)(base + L.chunk);
    a.b.shard_cap = L.shard_cap;
    a.b.chunk_cap = L.chunk_cap;
    a.b.dist = (unsigned long long *)dist_out;
    a.crit = criterion;
    hipStream_t s = g->stream;
    const int ib = (int)(((uint64_t)g->n + 255) / 256 > 8192 ? 8192 : ((uint64_t)g->n + 255) / 256);
    // every byte a solve reads before writing it is set here: state bytes, distances, control block
    hipLaunchKernelGGL(k_init_state, dim3(ib), dim3(256), 0, s, g->n, source, a.b.dist, a.b.st, nullptr, nullptr,
                       g->rp, nullptr, g->ip, nullptr, nullptr, g->edges, nullptr, g->in_edges);
    hipLaunchKernelGGL(k_init_ctl, dim3(1), dim3(64), 0, s, a.b.ctl, g->vmin, g->rp, g->wmax, source, 0u, 1ull);
    const PhaseKernels K = pick_phase(g->cfg.chunk, in, out, false, false, false, false);
    const dim3 blk(kBlock), gs(g->cfg.scan_blocks), gr(g->cfg.relax_blocks);
    const uint64_t max_phases = (uint64_t)g->n + 2;
    CtlHead h;
    uint64_t k = 0;
    for (;;) {  // batches of 16 phases; the header is read into host stack memory after each
        for (uint32_t i = 0; i < 16; ++i, ++k) {
            const int par = (int)(k % 6);
            hipLaunchKernelGGL(K.identify, gs, blk, 0, s, a, par);
            hipLaunchKernelGGL(K.relax, gr, blk, 0, s, a, par);
        }
        HIP_OK(hipGetLastError());
        HIP_OK(hipMemcpyAsync(&h, a.b.ctl, sizeof h, hipMemcpyDeviceToHost, s));
        HIP_OK(hipStreamSynchronize(s));
        if (h.done) break;
        if (k > max_phases + 32)
            return sssp_set_error(SSSP_ERR_INTERNAL, "phase loop did not terminate after %llu phases",
                                  (unsigned long long)k);
    }
    hipLaunchKernelGGL(k_clear_settled, dim3(ib), dim3(256), 0, s, g->n, a.b.dist);
    Sharded reached;
    HIP_OK(hipGetLastError());
    HIP_OK(hipMemcpyAsync(&reached, &a.b.ctl->reached, sizeof reached, hipMemcpyDeviceToHost, s));
    HIP_OK(hipStreamSynchronize(s));
    if (shard_sum(reached) != h.settled)
        return sssp_set_error(SSSP_ERR_INTERNAL, "solve ended in an inconsistent state (reached=%llu settled=%llu)",
                              shard_sum(reached), h.settled);
    if (phases_out) *phases_out = h.phases;
    return SSSP_OK;
}
