// Internal declarations shared by the HIP translation units of libsssp.
// Target: gfx950 (CDNA4), 64-wide wavefronts.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sssp.h"

#define INF64 0xFFFFFFFFFFFFFFFFull
#define INF32 0xFFFFFFFFu

// Vertex state byte: low two bits = set membership, bit 2 = "IN test passed"
// flag written by the dynamic-term pass for the current phase.
// Queue arrays only: bit 4 (ST_QNEW) = discovered by a relax since the vertex's
// scan block last looked, bit 5 (ST_QDIRTY) = distance lowered since then;
// keyed queue arrays: bit 6 (ST_QFAR) = queued vertex kept out of its block's
// entries because its IN-STATIC key d - minIn exceeded the split.
// Stored IN (full) / OUTWEAK / OUT (full) terms: bit 7 (ST_CHG) = the vertex
// changed state in the last phase (settled by identify, discovered by relax),
// bit 3 (ST_TDIRTY) = its stored terms must be computed in full.
enum : uint8_t { ST_U = 0, ST_F = 1, ST_S = 2, ST_R = 3, ST_SET = 3, ST_INOK = 4, ST_TDIRTY = 8, ST_QNEW = 16,
                 ST_QDIRTY = 32, ST_QFAR = 64, ST_CHG = 128 };

// A settled vertex carries this bit in its distance word while the solve runs
// (real distances stay below 2^58 and INF is all ones, so a word with the bit
// set is either INF or settled); relax then learns a target's settled status
// from the one load it needs anyway. Cleared before the solve returns.
constexpr unsigned long long kSettledBit = 1ull << 63;
__host__ __device__ __forceinline__ bool dist_settled(unsigned long long x) {
    return (x & kSettledBit) != 0 && x != 0xFFFFFFFFFFFFFFFFull;
}

// Which IN-family / OUT-family member a phase evaluates. Inside each family
// the members are ordered by strength (X-STATIC => X-SIMPLE => (OUTWEAK =>) X,
// Section 3), so a disjunction of members equals its strongest member, and
// DIJK implies every other criterion.
enum InMode : int { IN_NONE = 0, IN_DIJK = 1, IN_STATIC_M = 2, IN_SIMPLE_M = 3, IN_FULL_M = 4 };
enum OutMode : int { OUT_NONE = 0, OUT_STATIC_M = 1, OUT_SIMPLE_M = 2, OUT_WEAK_M = 3, OUT_FULL_M = 4 };

static inline void crit_modes(uint32_t c, int *in, int *out) {
    *in = (c & SSSP_IN_FULL) ? IN_FULL_M : (c & SSSP_IN_SIMPLE) ? IN_SIMPLE_M
        : (c & SSSP_IN_STATIC) ? IN_STATIC_M : IN_NONE;
    *out = (c & SSSP_OUT_FULL) ? OUT_FULL_M : (c & SSSP_OUT_WEAK) ? OUT_WEAK_M
         : (c & SSSP_OUT_SIMPLE) ? OUT_SIMPLE_M : (c & SSSP_OUT_STATIC) ? OUT_STATIC_M : OUT_NONE;
    if (*in == IN_NONE && *out == OUT_NONE && (c & SSSP_DIJK)) *in = IN_DIJK;
}

// Criteria made of DIJK, IN-STATIC and OUT-STATIC only (the queue-array kernels).
static inline bool static_modes(int in, int out) { return in <= IN_STATIC_M && out <= OUT_STATIC_M; }

// Same-address device-scope atomics serialise (about 12 ns each on MI355X),
// so every value that many blocks combine is spread over kShards slots, each
// on its own 128-byte line; block b uses slot b % kShards and readers combine
// the kShards slots with one wavefront.
constexpr int kShards = 32;
constexpr int kPad = 16;  // 16 x 8 B = 128 B between slots
struct alignas(128) Sharded {
    unsigned long long v[kShards * kPad];
};

// Scalar part of the control block: single writers only (block 0 of a
// kernel); the host copies just this header between batches of phases.
struct alignas(128) CtlHead {
    unsigned long long settled;     // vertices settled
    unsigned long long sum_f;       // sum of |F| at phase start
    unsigned long long m_reach;     // out-edges of settled vertices
    unsigned int pnum[2];           // 0-based index of the phase running with this parity
    unsigned int phases;            // phases executed so far
    unsigned int done;              // set once F is empty
    // Delta-stepping
    unsigned int rmode[2];          // round kind by parity: 0 bucket start, 1 light, 2 heavy
    unsigned int buckets;           // buckets finished (written by the heavy round's identify)
    unsigned int win_bucket;        // index of the bucket in progress
    unsigned int n_deltas;
    unsigned int choice[2];         // learned mode: choice index of the phase with this parity
    unsigned long long win_lo, win_hi, win_delta;
    unsigned long long fk;          // |F| at the start of the phase in progress (feature input)
    unsigned long long fprev;       // learned mode: |F| at the start of the previous phase
    unsigned long long dgk;         // learned mode: sum over F of out-degrees at the phase start
    unsigned long long s_k;         // settled count at the start of the phase (round) in progress
    unsigned long long m_k;         // m_reach at the start of the phase in progress
    unsigned long long fbucket;     // |F| at the start of the bucket in progress (feature input)
    unsigned long long next_delta;  // learned Delta-stepping: width of the next bucket
    unsigned long long last_settled;// |S'| of the last phase (selector feature input)
    unsigned int stalled;           // a phase with F non-empty certified nothing (bad ORACLE reference)
    unsigned int qlive[2];          // queue arrays: the phase with this parity left them current
    // keyed queue arrays, by launch parity: the launch with parity p reads [p] and writes [p ^ 1]
    unsigned int repart[2];         // the launch with this parity rebuilt the entries (not a phase)
    unsigned int qprep[2];          // phase index of the last rebuild
    unsigned long long qsplit[2];   // split: entries hold the queued vertices with d - minIn <= split
    unsigned long long qdelta[2];   // split margin above the threshold at the last rebuild
    unsigned long long qxrep[2];    // threshold at the last rebuild
    unsigned int qrebuilds;         // rebuild launches so far (launches = phases + rebuilds)
    // learned checkpoint mode: the selector's choice at the last checkpoint (0 = stay static)
    // and |F| at that checkpoint's phase
    unsigned int cp_choice;
    unsigned long long cp_fprev;
};

// Device control block of one solve. Slots indexed by phase parity (mod 2 or
// mod 3) let phase k fold values for phase k+1 while k's are still read,
// with no host round trip between phases.
struct Ctl {
    CtlHead h;
    Sharded reached;                // sum: vertices ever queued (source included)
    Sharded relax_edges;            // sum: relaxations towards non-settled targets
    Sharded improving;              // sum: relaxations that lowered d
    Sharded spack[2];               // per shard: S' (count << 32) | edge total
    Sharded szero[2];               // per shard: S' vertices without out-edges
    Sharded minD[3];                // min: min_{v in F} d[v] for the phase
    Sharded tst[3];                 // min: OUT-STATIC threshold min_{u in F} d[u] + minOut[u]
    Sharded tdyn[3];                // min: dynamic OUT threshold from the term pass
    Sharded nextmin[2];             // min: Delta-stepping, min d over F for the next bucket
    Sharded win_improved[2];        // sum: Delta-stepping, vertices improved inside the window
    // learned mode (selector features)
    Sharded sumd[3];                // sum over F of d (mod 2^64 while folding), by phase mod 3
    Sharded degsum;                 // sum of out-degrees of every vertex ever queued
    Sharded nin[2], nout[2];        // queued vertices passing IN-STATIC / OUT-STATIC, by phase parity
    // trace mode (training data): every criterion evaluated on every snapshot
    Sharded cnt_cf[6];              // sum: vertices each of the three criteria certifies, [parity*3 + c]
};

// Per-phase device trace record (mirrors sssp_phase_rec).
struct PhaseRec {
    unsigned long long min_d;
    unsigned int fringe, settled, criterion, edges;
};

// Device-resident graph plus the per-solve scratch kept between solves.
struct sssp_graph_impl;

struct DevGraph {
    uint32_t n;
    uint64_t m;
    const uint32_t *rp;     // row_ptr (u32, n+1)
    const uint2 *edges;     // (target, weight), each row sorted by weight
    const uint2 *vmin;      // (minIn, minOut) per vertex
    const uint32_t *ip;     // CSC in_ptr (n+1) or null
    const uint2 *in_edges;  // CSC (source, weight), rows sorted by weight, or null
    const uint32_t *emin;   // per edge (CSR order): minOut of its target (vmin[target].y)
    uint32_t wmax;          // nonzero if some edge weighs 2^32 - 1 (see min_out64)
};

// Scratch used by a solve.
struct SolveBufs {
    Ctl *ctl;
    uint32_t shard_cap;     // S' entries per shard (srow/soff/sdu hold kShards * shard_cap)
    uint32_t chunk_cap;     // chunk_start entries per shard
    uint8_t *st;
    uint32_t *srow;         // S' first out-edge index (row start) of each settled vertex with out-edges
    uint32_t *soff;         // S' exclusive edge offsets
    unsigned long long *sdu;// S' snapshot distances
    uint32_t *chunk_start;  // first S' entry (shard-local) of each shard-local edge chunk
    uint32_t *in_cur;       // IN-SIMPLE cursors (absolute CSC index)
    uint32_t *out_cur;      // OUT-SIMPLE cursors (absolute CSR index)
    uint2 *in_head;         // (source, weight) of the in-edge at each IN-SIMPLE cursor; x = INF32 at the row end
    uint2 *out_head;        // (target, weight) of the out-edge at each OUT-SIMPLE cursor; likewise
    uint32_t *stamp;        // Delta-stepping improvement stamps
    unsigned long long *deltas; // Delta-stepping widths per bucket
    PhaseRec *trace;
    uint32_t trace_cap;
    float *trace_feat;      // trace mode: selector features of each phase (bucket), [cap][12]
    uint32_t *trace_cf;     // trace mode: vertices each criterion certifies per phase, [cap][3]
    uint32_t *phase_of;
    unsigned long long *dist;
    // Queue arrays (static criteria, launch option `queue`): scan block b keeps
    // an entry for each queued vertex it owns in slots [b * qspan, (b+1) * qspan).
    unsigned long long *qd; // distance of the entry's vertex (kTomb once it settled)
    uint32_t *qv;           // the entry's vertex
    uint2 *qm;              // its (minIn, minOut)
    uint2 *qr;              // its row start and out-degree (settling reads no row pointers)
    uint32_t *qcnt;         // per scan block: slots in use, then tombstones among them
    uint32_t qspan;         // slots per scan block (vertices it owns)
    // approximate criteria: phase index of each vertex's last IN / OUT recomputation, and the
    // 1-based settle phase of each vertex (the caller's phase_of when given)
    uint32_t *apx_lin, *apx_lout, *apx_sp;
    // stored terms of the queued vertices: IN (full) and OUTWEAK / OUT (full), kept
    // by the dirty-set pass (k_mark) and recomputed in full only where flagged
    unsigned long long *tin, *tout;
};

int sssp_set_error(int code, const char *fmt, ...);

// Release helpers for clean-up paths, where a failure has nothing left to undo.
static inline void sssp_free(void *p) {
    if (p) (void)hipFree(p);
}
static inline void sssp_host_free(void *p) {
    if (p) (void)hipHostFree(p);
}

// Owner of a device allocation made inside one call: freed on every return path.
struct CallBuffer {
    void *p = nullptr;
    CallBuffer() = default;
    CallBuffer(const CallBuffer &) = delete;
    CallBuffer &operator=(const CallBuffer &) = delete;
    ~CallBuffer() { sssp_free(p); }
};

#define HIP_OK(call)                                                                      \
    do {                                                                                  \
        hipError_t _e = (call);                                                           \
        if (_e != hipSuccess)                                                             \
            return sssp_set_error(_e == hipErrorOutOfMemory ? SSSP_ERR_OOM : SSSP_ERR_DEVICE, \
                                  "%s failed: %s (%s:%d)", #call, hipGetErrorString(_e),  \
                                  __FILE__, __LINE__);                                    \
    } while (0)

// ---------------------------------------------------------------------------
// Device helpers

__device__ __forceinline__ unsigned long long sadd64(unsigned long long a, unsigned long long b) {
    unsigned long long s = a + b;
    return s < a ? INF64 : s;
}
__device__ __forceinline__ unsigned long long umin64(unsigned long long a, unsigned long long b) {
    return a < b ? a : b;
}

// The static minima are stored as u32 with INF32 for an empty edge set, but
// 2^32 - 1 is also a legal weight. Only graphs holding such an edge (wmax) need
// the row length to tell the two apart; elsewhere INF32 always means empty.
//   minOut (eq. crit:outstatic, and the second edge of eq. crit:outweak): an
//   empty row makes the term infinite.
__device__ __forceinline__ unsigned long long min_out64(uint32_t x, uint32_t wmax, const uint32_t *rp, uint32_t v) {
    if (x != INF32) return x;
    if (!wmax) return INF64;
    return rp[v + 1] > rp[v] ? (unsigned long long)INF32 : INF64;
}
//   minIn in the unexplored-vertex term of eq. crit:in: an unexplored vertex
//   without in-edges contributes no two-edge path (needs the reverse adjacency).
__device__ __forceinline__ unsigned long long min_in_u64(uint32_t x, uint32_t wmax, const uint32_t *ip, uint32_t w) {
    if (x != INF32) return x;
    if (!wmax) return INF64;
    return ip[w + 1] > ip[w] ? (unsigned long long)INF32 : INF64;
}
//   minIn in the IN-STATIC test (eq. crit:instatic) is read as the number it
//   holds: a queued vertex other than the source was reached over an in-edge,
//   so its minimum is real; the source is queued alone in phase 1 and is the
//   queue minimum, certified by any threshold. Reading INF32 as 2^32 - 1
//   therefore never changes a test, while reading a real 2^32 - 1 as infinity
//   would certify every such vertex.
__device__ __forceinline__ unsigned long long min_in_test(uint32_t x) { return (unsigned long long)x; }

// Wavefront reductions with DPP lane moves inside each row of 16 lanes
// (quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror: after
// these four steps every lane holds its row's result), then the four row
// results are read with readlane. Every lane gets the wavefront's result.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}
template <int CTRL>
__device__ __forceinline__ unsigned long long dpp64(unsigned long long v) {
    return ((unsigned long long)dpp32<CTRL>((uint32_t)(v >> 32)) << 32) | dpp32<CTRL>((uint32_t)v);
}
__device__ __forceinline__ unsigned long long readlane64(unsigned long long v, int lane) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
    return ((unsigned long long)hi << 32) | lo;
}
constexpr int kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

__device__ __forceinline__ unsigned long long wave_min64(unsigned long long x) {
    x = umin64(x, dpp64<kDppQuadSwap1>(x));
    x = umin64(x, dpp64<kDppQuadSwap2>(x));
    x = umin64(x, dpp64<kDppHalfMirror>(x));
    x = umin64(x, dpp64<kDppMirror>(x));
    return umin64(umin64(readlane64(x, 0), readlane64(x, 16)), umin64(readlane64(x, 32), readlane64(x, 48)));
}
__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long x) {
    x += dpp64<kDppQuadSwap1>(x);
    x += dpp64<kDppQuadSwap2>(x);
    x += dpp64<kDppHalfMirror>(x);
    x += dpp64<kDppMirror>(x);
    return (readlane64(x, 0) + readlane64(x, 16)) + (readlane64(x, 32) + readlane64(x, 48));
}
// Inclusive prefix sum over the 64 lanes of a wavefront.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_sum32(uint32_t x) {
    x += dpp32<kDppQuadSwap1>(x);
    x += dpp32<kDppQuadSwap2>(x);
    x += dpp32<kDppHalfMirror>(x);
    x += dpp32<kDppMirror>(x);
    return ((uint32_t)__builtin_amdgcn_readlane((int)x, 0) + (uint32_t)__builtin_amdgcn_readlane((int)x, 16)) +
           ((uint32_t)__builtin_amdgcn_readlane((int)x, 32) + (uint32_t)__builtin_amdgcn_readlane((int)x, 48));
}

// Block-wide combine of the values v[i] whose bit i is set in ACT, all in one
// LDS round: bit i of MIN set means a minimum, else a sum; bit i of U32 set
// means the sum over one wavefront fits in 32 bits (cheaper shuffles).
// Results are valid in thread 0. One barrier and none after it: the caller
// writes sh (8 * NWAVES entries) no more in this kernel.
template <int NWAVES, unsigned ACT, unsigned MIN, unsigned U32 = 0u>
__device__ __forceinline__ void block_reduce(unsigned long long *v, unsigned long long *sh) {
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        if (!((ACT >> i) & 1u)) continue;
        if ((MIN >> i) & 1u) v[i] = wave_min64(v[i]);
        else if ((U32 >> i) & 1u) v[i] = wave_sum32((uint32_t)v[i]);
        else v[i] = wave_sum64(v[i]);
    }
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int i = 0; i < 8; ++i)
            if ((ACT >> i) & 1u) sh[i * NWAVES + w] = v[i];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            if (!((ACT >> i) & 1u)) continue;
            for (int k = 1; k < NWAVES; ++k) {
                const unsigned long long x = sh[i * NWAVES + k];
                v[i] = ((MIN >> i) & 1u) ? umin64(v[i], x) : v[i] + x;
            }
        }
}

constexpr int kBlock = 256;          // threads per block for the phase kernels
constexpr int kWaves = kBlock / 64;

// Launch shape chosen per graph (autotuned in tune.hip).
struct LaunchCfg {
    int scan_blocks;    // blocks of the dense vertex-scan kernels
    int relax_blocks;   // blocks of the relax kernel
    int chunk;          // edges per relax chunk (256, 512 or 1024)
    int use_graph;      // replay phases from a captured HIP graph
    int queue;          // static criteria: per-block queue arrays instead of the dense scan (2: keyed)
    int single;         // sssp_solve with static criteria: the whole solve in one workgroup
};
constexpr int kMaxChunk = 2048;
