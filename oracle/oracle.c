/*
 * CPU ORACLE for phased single-source shortest paths -- test infrastructure.
 *
 * Plain, slow, obviously correct reference implementations used only by the
 * tests, by the smoke check and by the benchmark's CPU-baseline leg. Nothing
 * in the GPU product path includes, links or calls this file.
 *
 * Paper: M. Kainer, J. L. Traff, "More Parallelism in Dijkstra's
 * Single-Source Shortest Path Algorithm" (arXiv 1903.12085).
 *
 * Conventions
 *   Graph: directed, CSR (row_ptr u64[n+1], col u32[m], w u32[m]); weights
 *   are non-negative by type (Section 2, "Preliminaries").
 *   Distances: u64, UINT64_MAX stands for infinity (unreachable, Section 2).
 *   a (+) b: saturating addition, so INF (+) x = INF. A test "d[v] - X <= minD"
 *   is evaluated as d[v] <= minD (+) X, which is the same inequality over the
 *   reals and cannot underflow.
 *
 * Contents
 *   orc_validate        -- CSR sanity checks.
 *   orc_dijkstra        -- binary-heap Dijkstra (Section 2), plus the fewest
 *                          number of edges among all minimum-cost paths
 *                          (hops), keyed lexicographically by (cost, hops).
 *   orc_bellman_ford    -- brute force by repeated relaxation of every edge.
 *   orc_phased          -- the generic phased algorithm (Section 3): per
 *                          phase, on a snapshot of (S, F, U, d), evaluate the
 *                          chosen criteria for every v in F by enumerating the
 *                          edge sets in their defining equations, settle every
 *                          vertex any of them certifies, relax all out-edges
 *                          of the settled vertices. Criteria: DIJK, IN,
 *                          OUT, OUTWEAK, IN-STATIC, OUT-STATIC, IN-SIMPLE,
 *                          OUT-SIMPLE (equations crit:in, crit:out,
 *                          crit:outweak, crit:instatic, crit:outstatic,
 *                          crit:insimple, crit:outsimple).
 *   orc_delta_step      -- Delta-stepping (Section 5, the comparison
 *                          algorithm of Meyer and Sanders), one bucket width
 *                          per bucket from a caller-given list.
 *
 * Readings of the paper taken here (see the design notes for the reasons):
 *   - OUT-SIMPLE is read with the vertex sets of its minimum swapped: u in F,
 *     w in F u U, i.e. min over edges (u, w) with u queued and w not settled
 *     of d[u] + c(u, w). Printed literally (u in F u U, w in V) it would be
 *     identical to OUT-STATIC because d[u] = infinity for u in U.
 *   - Thresholds are computed once per phase from the phase-start snapshot;
 *     every v in F that satisfies the criterion on that snapshot is settled.
 *   - DIJK settles every vertex of minimum tentative distance, not just one.
 *   - Self-loops and parallel edges take part in every minimum as written.
 *   - Delta-stepping: light edge <=> c < Delta, heavy <=> c >= Delta; bucket
 *     of the window [b*Delta, (b+1)*Delta) with b = floor(minD / Delta); light
 *     rounds are synchronous (every frontier vertex relaxes with its
 *     round-start distance), the next frontier is the set of vertices whose
 *     distance dropped in the round and lies inside the window; one heavy
 *     round per bucket from every vertex the bucket removed.
 *
 * Pins (the tests): Bellman-Ford and Dijkstra agree on random multigraphs;
 * closed forms (paths, stars, unit grids); hand-traced phase sets of small
 * graphs derived from the equations; invariants (every criterion certifies
 * the minimum-distance vertices, certified vertices are correct, the
 * strength chains DIJK => X-STATIC => X-SIMPLE => (OUTWEAK =>) X hold on
 * every snapshot, ORACLE lower bound <= phases <= reachable vertices).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define INF UINT64_MAX
#define U32INF UINT32_MAX

enum { ST_U = 0, ST_F = 1, ST_S = 2 };

/* Criterion bits; a set of bits means their disjunction (Section 3: a
 * disjunction of sound criteria is sound). */
enum {
    C_DIJK = 1u << 0, C_IN_STATIC = 1u << 1, C_OUT_STATIC = 1u << 2, C_IN_SIMPLE = 1u << 3,
    C_OUT_SIMPLE = 1u << 4, C_IN_FULL = 1u << 5, C_OUT_WEAK = 1u << 6, C_OUT_FULL = 1u << 7,
    C_ALL = 0xFFu,
    /* approximate criteria (Section 3, last paragraphs): see approx_t below */
    C_IN_APPROX = 1u << 8, C_OUT_APPROX = 1u << 9, C_APPROX = C_IN_APPROX | C_OUT_APPROX
};

enum { ORC_OK = 0, ORC_EINVAL = -1, ORC_ENOMEM = -2, ORC_EUNSOUND = -10, ORC_EINCOMPLETE = -11,
       ORC_ECHAIN = -12, ORC_EDIST = -13 };

static inline uint64_t sadd(uint64_t a, uint64_t b) {
    uint64_t s = a + b;
    return s < a ? INF : s;
}
static inline uint64_t min64(uint64_t a, uint64_t b) { return a < b ? a : b; }

int orc_validate(uint32_t n, const uint64_t *rp, const uint32_t *col) {
    if (n == 0 || !rp) return ORC_EINVAL;
    if (rp[0] != 0) return ORC_EINVAL;
    for (uint32_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v]) return ORC_EINVAL;
    uint64_t m = rp[n];
    if (m && !col) return ORC_EINVAL;
    for (uint64_t e = 0; e < m; ++e)
        if (col[e] >= n) return ORC_EINVAL;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Dijkstra with a binary heap and lazy deletion (Section 2).               */

typedef struct { uint64_t d; uint32_t h; uint32_t v; } hent;

static inline int hless(const hent *a, const hent *b) {
    if (a->d != b->d) return a->d < b->d;
    if (a->h != b->h) return a->h < b->h;
    return a->v < b->v;
}

typedef struct { hent *a; uint64_t len, cap; } heap_t;

static int hpush(heap_t *H, hent x) {
    if (H->len == H->cap) {
        uint64_t nc = H->cap ? H->cap * 2 : 1024;
        hent *na = (hent *)realloc(H->a, nc * sizeof(hent));
        if (!na) return -1;
        H->a = na; H->cap = nc;
    }
    uint64_t i = H->len++;
    while (i > 0) {
        uint64_t p = (i - 1) / 2;
        if (!hless(&x, &H->a[p])) break;
        H->a[i] = H->a[p];
        i = p;
    }
    H->a[i] = x;
    return 0;
}

static hent hpop(heap_t *H) {
    hent top = H->a[0];
    hent x = H->a[--H->len];
    uint64_t i = 0, n = H->len;
    for (;;) {
        uint64_t l = 2 * i + 1, r = l + 1, s = i;
        const hent *best = &x;
        if (l < n && hless(&H->a[l], best)) { s = l; best = &H->a[l]; }
        if (r < n && hless(&H->a[r], best)) { s = r; }
        if (s == i) break;
        H->a[i] = H->a[s];
        i = s;
    }
    if (n) H->a[i] = x;
    return top;
}

/* dist[v] = dist(s, v) or INF; hops[v] = fewest edges over minimum-cost
 * paths (U32INF if unreachable); hops may be NULL. Returns the number of
 * vertices settled (reachable), or a negative error. */
int64_t orc_dijkstra(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                     uint32_t src, uint64_t *dist, uint32_t *hops) {
    if (src >= n) return ORC_EINVAL;
    uint32_t *h = hops ? hops : (uint32_t *)malloc((uint64_t)n * sizeof(uint32_t));
    uint8_t *done = (uint8_t *)calloc(n, 1);
    heap_t H = {0, 0, 0};
    if (!h || !done) { if (!hops) free(h); free(done); return ORC_ENOMEM; }
    for (uint32_t v = 0; v < n; ++v) { dist[v] = INF; h[v] = U32INF; }
    dist[src] = 0; h[src] = 0;
    int64_t settled = 0;
    if (hpush(&H, (hent){0, 0, src})) goto oom;
    while (H.len) {
        hent t = hpop(&H);
        if (done[t.v] || t.d != dist[t.v] || t.h != h[t.v]) continue;
        done[t.v] = 1;
        ++settled;
        for (uint64_t e = rp[t.v]; e < rp[t.v + 1]; ++e) {
            uint32_t x = col[e];
            if (done[x]) continue;
            uint64_t nd = t.d + w[e];
            uint32_t nh = t.h + 1;
            if (nd < dist[x] || (nd == dist[x] && nh < h[x])) {
                dist[x] = nd; h[x] = nh;
                if (hpush(&H, (hent){nd, nh, x})) goto oom;
            }
        }
    }
    free(H.a); free(done); if (!hops) free(h);
    return settled;
oom:
    free(H.a); free(done); if (!hops) free(h);
    return ORC_ENOMEM;
}

/* Brute force: relax every edge until nothing changes (at most n-1 passes
 * are needed with non-negative weights). */
int orc_bellman_ford(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                     uint32_t src, uint64_t *dist) {
    if (src >= n) return ORC_EINVAL;
    for (uint32_t v = 0; v < n; ++v) dist[v] = INF;
    dist[src] = 0;
    for (uint32_t pass = 0; pass < n; ++pass) {
        int changed = 0;
        for (uint32_t u = 0; u < n; ++u) {
            if (dist[u] == INF) continue;
            for (uint64_t e = rp[u]; e < rp[u + 1]; ++e) {
                uint64_t c = dist[u] + w[e];
                if (c < dist[col[e]]) { dist[col[e]] = c; changed = 1; }
            }
        }
        if (!changed) break;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Generic phased algorithm (Section 3).                                     */

typedef struct {
    uint32_t phases;        /* loop iterations; phase 1 settles the source */
    uint32_t pad;
    uint64_t sum_f;         /* sum over phases of |F| at phase start */
    uint64_t n_reach;       /* vertices settled = reachable vertices */
    uint64_t m_reach;       /* out-edges of reachable vertices */
    uint64_t relax_edges;   /* edges relaxed (target not settled) */
    uint64_t improving;     /* relaxations that lowered a tentative distance */
} orc_stats;

typedef struct {
    uint64_t *ip;  /* in_ptr[n+1] */
    uint32_t *is;  /* in-edge sources */
    uint32_t *iw;  /* in-edge weights */
} csc_t;

static int build_csc(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, csc_t *c) {
    uint64_t m = rp[n];
    c->ip = (uint64_t *)calloc((uint64_t)n + 1, sizeof(uint64_t));
    c->is = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    c->iw = (uint32_t *)malloc((m ? m : 1) * sizeof(uint32_t));
    if (!c->ip || !c->is || !c->iw) return ORC_ENOMEM;
    for (uint64_t e = 0; e < m; ++e) c->ip[col[e] + 1]++;
    for (uint32_t v = 0; v < n; ++v) c->ip[v + 1] += c->ip[v];
    uint64_t *pos = (uint64_t *)malloc(((uint64_t)n + 1) * sizeof(uint64_t));
    if (!pos) return ORC_ENOMEM;
    memcpy(pos, c->ip, ((uint64_t)n + 1) * sizeof(uint64_t));
    for (uint32_t u = 0; u < n; ++u)
        for (uint64_t e = rp[u]; e < rp[u + 1]; ++e) {
            uint64_t p = pos[col[e]]++;
            c->is[p] = u;
            c->iw[p] = w[e];
        }
    free(pos);
    return ORC_OK;
}

static void free_csc(csc_t *c) { free(c->ip); free(c->is); free(c->iw); }

/* Static minima (equations crit:instatic and crit:outstatic): minimum
 * weight over all in-edges / all out-edges; U32INF when there are none.
 * Exported form only: a real minimum can also be 2^32 - 1. */
static void static_minima(uint32_t n, const uint64_t *rp, const uint32_t *w, const csc_t *c,
                          uint32_t *min_in, uint32_t *min_out) {
    for (uint32_t v = 0; v < n; ++v) {
        uint32_t mo = U32INF, mi = U32INF;
        for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) if (w[e] < mo) mo = w[e];
        for (uint64_t e = c->ip[v]; e < c->ip[v + 1]; ++e) if (c->iw[e] < mi) mi = c->iw[e];
        min_out[v] = mo; min_in[v] = mi;
    }
}

/* Exported for tests: the static per-vertex minima. */
int orc_static_minima(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                      uint32_t *min_in, uint32_t *min_out) {
    csc_t c = {0, 0, 0};
    if (build_csc(n, rp, col, w, &c)) { free_csc(&c); return ORC_ENOMEM; }
    static_minima(n, rp, w, &c, min_in, min_out);
    free_csc(&c);
    return ORC_OK;
}

/* The same minima in 64 bits, INF for an empty edge set. A real minimum may be
 * 2^32 - 1 (a legal weight), so the criteria never read the 32-bit form, whose
 * U32INF would stand for both. */
static void static_minima64(uint32_t n, const uint64_t *rp, const uint32_t *w, const csc_t *c,
                            uint64_t *min_in, uint64_t *min_out) {
    for (uint32_t v = 0; v < n; ++v) {
        uint64_t mo = INF, mi = INF;
        for (uint64_t e = rp[v]; e < rp[v + 1]; ++e) mo = min64(mo, w[e]);
        for (uint64_t e = c->ip[v]; e < c->ip[v + 1]; ++e) mi = min64(mi, c->iw[e]);
        min_out[v] = mo; min_in[v] = mi;
    }
}

/* Which criterion (single bit) holds for v on the snapshot. Thresholds that
 * do not depend on v (minD and the OUT-family right-hand sides) are passed
 * in; the IN-family left-hand minima are enumerated here from the edge sets
 * of their equations. */
typedef struct {
    uint64_t minD;
    uint64_t t_out_static, t_out_simple, t_out_weak, t_out_full;
} thresholds_t;

static uint64_t in_simple_term(uint32_t v, const csc_t *c, const uint8_t *st) {
    /* crit:insimple: min over (w, v) in E with w in F u U of c(w, v) */
    uint64_t t = INF;
    for (uint64_t e = c->ip[v]; e < c->ip[v + 1]; ++e)
        if (st[c->is[e]] != ST_S) t = min64(t, c->iw[e]);
    return t;
}

/* Per-phase memo of an inner minimum: val[x] is valid while stamp[x] equals the
 * phase's stamp (the snapshot does not change while a phase is evaluated). */
typedef struct { uint64_t *val; uint32_t *stamp; uint32_t now; } memo_t;

static uint64_t in_full_term(uint32_t v, const csc_t *c, const uint8_t *st, memo_t *M) {
    /* crit:in: min( min_{w in F, (w,v)} c(w,v),
     *               min_{w in U, w' in F u U, (w,v), (w',w)} c(w,v) + c(w',w) ) */
    uint64_t t = INF;
    for (uint64_t e = c->ip[v]; e < c->ip[v + 1]; ++e) {
        uint32_t wv = c->is[e];
        if (st[wv] == ST_F) {
            t = min64(t, c->iw[e]);
        } else if (st[wv] == ST_U) {
            if (M->stamp[wv] != M->now) {
                uint64_t inner = INF;
                for (uint64_t f = c->ip[wv]; f < c->ip[wv + 1]; ++f)
                    if (st[c->is[f]] != ST_S) inner = min64(inner, c->iw[f]);
                M->val[wv] = inner;
                M->stamp[wv] = M->now;
            }
            t = min64(t, sadd(c->iw[e], M->val[wv]));
        }
    }
    return t;
}

static uint32_t eval_bits(uint32_t v, uint32_t want, const thresholds_t *T, const uint64_t *d,
                          const uint8_t *st, const uint64_t *min_in, const csc_t *c, memo_t *M) {
    uint32_t b = 0;
    uint64_t dv = d[v];
    if ((want & C_DIJK) && dv == T->minD) b |= C_DIJK;
    if ((want & C_IN_STATIC) && dv <= sadd(T->minD, min_in[v])) b |= C_IN_STATIC;
    if ((want & C_IN_SIMPLE) && dv <= sadd(T->minD, in_simple_term(v, c, st))) b |= C_IN_SIMPLE;
    if ((want & C_IN_FULL) && dv <= sadd(T->minD, in_full_term(v, c, st, M))) b |= C_IN_FULL;
    if ((want & C_OUT_STATIC) && dv <= T->t_out_static) b |= C_OUT_STATIC;
    if ((want & C_OUT_SIMPLE) && dv <= T->t_out_simple) b |= C_OUT_SIMPLE;
    if ((want & C_OUT_WEAK) && dv <= T->t_out_weak) b |= C_OUT_WEAK;
    if ((want & C_OUT_FULL) && dv <= T->t_out_full) b |= C_OUT_FULL;
    return b;
}

/* OUT-family right-hand sides on the snapshot, each the minimum over the
 * edge sets of its equation. `inner_ns` memoises, per phase, the minimum
 * out-edge weight of a vertex w towards non-settled vertices (the c(w, w')
 * term of crit:out with w' in F u U); memo_stamp marks validity. */
static void out_thresholds(uint32_t want, const uint32_t *Flist, uint64_t nF, const uint64_t *rp,
                           const uint32_t *col, const uint32_t *w, const uint64_t *d, const uint8_t *st,
                           const uint64_t *min_out, uint64_t *inner_ns, uint32_t *memo_stamp,
                           uint32_t stamp, thresholds_t *T) {
    T->t_out_static = T->t_out_simple = T->t_out_weak = T->t_out_full = INF;
    const uint32_t dyn = want & (C_OUT_SIMPLE | C_OUT_WEAK | C_OUT_FULL);
    for (uint64_t i = 0; i < nF; ++i) {
        uint32_t u = Flist[i];
        uint64_t du = d[u];
        /* crit:outstatic: min over u in F and all out-edges (u, w) of d[u] + c(u, w)
         * = d[u] + minOut[u], the precomputed static minimum (Section 3) */
        if (want & C_OUT_STATIC) T->t_out_static = min64(T->t_out_static, sadd(du, min_out[u]));
        if (!dyn) continue;
        for (uint64_t e = rp[u]; e < rp[u + 1]; ++e) {
            uint32_t x = col[e];
            uint64_t c = w[e];
            if (st[x] == ST_S) continue;
            /* crit:outsimple (sets read as u in F, w in F u U) */
            if (want & C_OUT_SIMPLE) T->t_out_simple = min64(T->t_out_simple, sadd(du, c));
            if (st[x] == ST_F) {
                /* first line of crit:outweak / crit:out: u in F, w in F */
                if (want & C_OUT_WEAK) T->t_out_weak = min64(T->t_out_weak, sadd(du, c));
                if (want & C_OUT_FULL) T->t_out_full = min64(T->t_out_full, sadd(du, c));
            } else { /* x in U: second line */
                if (want & C_OUT_WEAK) /* w' in V */
                    T->t_out_weak = min64(T->t_out_weak, sadd(sadd(du, c), min_out[x]));
                if (want & C_OUT_FULL) { /* w' in F u U */
                    if (memo_stamp[x] != stamp) {
                        uint64_t inner = INF;
                        for (uint64_t f = rp[x]; f < rp[x + 1]; ++f)
                            if (st[col[f]] != ST_S) inner = min64(inner, w[f]);
                        inner_ns[x] = inner;
                        memo_stamp[x] = stamp;
                    }
                    T->t_out_full = min64(T->t_out_full, sadd(sadd(du, c), inner_ns[x]));
                }
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Learned per-phase selector: features and FP32 forward pass.               */
/*
 * Twelve features of a snapshot of the solver state and of the outcome of the
 * last criterion evaluation, each a ratio of exact integers evaluated in
 * double precision in the order written, then rounded to float:
 *   n, m          vertices, edges;  Wm = (sum of weights) / m (1 if m = 0)
 *   F, S, R       |F|, settled, reached (= F + S) at the snapshot
 *   a, t          minD and the OUT-STATIC threshold min_{u in F} d[u] (+) minOut[u]
 *   SD, DG        sum over F of d[u], sum over F of out-degree
 *   Fp            |F| at the previous snapshot
 *   D, Sp, Ip, Op queued vertices the last evaluation ran over, how many it
 *                 settled, and how many of them pass IN-STATIC / OUT-STATIC
 *   k             index of the phase (bucket) the choice is for
 * x0 = F/n; x1 = S/n; x2 = D ? Sp/D : 0; x3 = min(F/2^22, 4)/4;
 * x4 = t = INF ? 1 : min((t-a)/Wm, 64)/64;
 * x5 = min(max((SD/F - a)/Wm, 0), 256)/256; x6 = min((DG/F)/(m/n), 8)/8;
 * x7 = D ? Ip/D : 0; x8 = D ? Op/D : 0; x9 = Fp ? min(F/Fp, 4)/4 : 0;
 * x10 = (n-R)/n; x11 = min(a/Wm, 4096)/4096.
 * Phased solver: the criterion of phase 0 comes from the state {s} with no
 * evaluation yet (D = Sp = Ip = Op = Fp = 0); the criterion of phase k+1 comes
 * from phase k's snapshot together with phase k's own outcome (D = |F_k|,
 * Sp = |S'_k|, Fp = |F_{k-1}|), so it is known as soon as phase k has
 * identified S'_k and can be evaluated while S'_k relaxes.
 * Delta-stepping (delta_mode 1): the state is taken at a bucket start (a =
 * minD, D = |F| at the previous bucket start, Sp = the vertices that bucket
 * settled, Ip = Op = 0); x4..x9 are 0. Checkpoint mode (delta_mode 2): after
 * every 16th phase k of a static solve, phase k's snapshot and outcome as for
 * the phased solver, Fp = |F| at the previous checkpoint; x5 = floor(log2 n)/32,
 * x6 = min(m/n, 64)/64, x7 = x8 = 0.
 * MLP: 12 -> 64 (ReLU) -> 64 (ReLU) -> 6, FP32; each neuron is its bias
 * followed by fmaf over its inputs in index order. Weights, flat: W1[64][12],
 * b1[64], W2[64][64], b2[64], W3[6][64], b3[6] (5382 floats). The phased
 * solver takes the argmax of outputs 0..2 (ties: lowest index) as the phase's
 * criterion: 0 = IN-STATIC|OUT-STATIC, 1 = IN-SIMPLE|OUT-SIMPLE, 2 =
 * IN-SIMPLE|OUT-STATIC; Delta-stepping takes the argmax of outputs 3..5 as the bucket width
 * 2^12, 2^14, 2^16.
 */
#define MLP_IN 12
#define MLP_H 64
#define MLP_OUT 6
#define MLP_NPARAM (MLP_H * MLP_IN + MLP_H + MLP_H * MLP_H + MLP_H + MLP_OUT * MLP_H + MLP_OUT)

typedef struct {
    uint64_t n, m, F, S, R, a, t, SD, DG, Fp, D, Sp, Ip, Op, k;
    double Wm;
    int delta_mode;
} feat_in;

static double dmin(double x, double y) { return x < y ? x : y; }
static double dmax(double x, double y) { return x > y ? x : y; }

static void features(const feat_in *q, float *x) {
    const double n = (double)q->n, m = (double)q->m, F = (double)q->F, Fp = (double)q->Fp, D = (double)q->D;
    x[0] = (float)(F / n);
    x[1] = (float)((double)q->S / n);
    x[2] = (float)(q->D ? (double)q->Sp / D : 0.0);
    x[3] = (float)(dmin(F / 4194304.0, 4.0) / 4.0);
    x[10] = (float)((n - (double)q->R) / n);
    x[11] = (float)(dmin((double)q->a / q->Wm, 4096.0) / 4096.0);
    if (q->delta_mode == 1) {
        for (int i = 4; i < 10; ++i) x[i] = 0.0f;
        return;
    }
    x[4] = (float)(q->t == INF ? 1.0 : dmin((double)(q->t - q->a) / q->Wm, 64.0) / 64.0);
    x[5] = (float)(dmin(dmax(((double)q->SD / F - (double)q->a) / q->Wm, 0.0), 256.0) / 256.0);
    x[6] = (float)(dmin(((double)q->DG / F) / (m / n), 8.0) / 8.0);
    x[7] = (float)(q->D ? (double)q->Ip / D : 0.0);
    x[8] = (float)(q->D ? (double)q->Op / D : 0.0);
    x[9] = (float)(q->Fp ? dmin(F / Fp, 4.0) / 4.0 : 0.0);
    if (q->delta_mode == 2) {  /* checkpoint mode: the graph's size and mean degree */
        x[5] = (float)((double)(63 - __builtin_clzll(q->n)) / 32.0);
        x[6] = (float)(dmin(m / n, 64.0) / 64.0);
        x[7] = x[8] = 0.0f;
    }
}

/* FP32 forward pass; returns the argmax of outputs [lo, lo+3). */
static int mlp_choice(const float *w, const float *x, int lo, float *out_logits) {
    const float *W1 = w, *b1 = W1 + MLP_H * MLP_IN, *W2 = b1 + MLP_H, *b2 = W2 + MLP_H * MLP_H;
    const float *W3 = b2 + MLP_H, *b3 = W3 + MLP_OUT * MLP_H;
    float h1[MLP_H], h2[MLP_H], z[MLP_OUT];
    for (int j = 0; j < MLP_H; ++j) {
        float acc = b1[j];
        for (int i = 0; i < MLP_IN; ++i) acc = fmaf(W1[j * MLP_IN + i], x[i], acc);
        h1[j] = acc > 0.0f ? acc : 0.0f;
    }
    for (int j = 0; j < MLP_H; ++j) {
        float acc = b2[j];
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(W2[j * MLP_H + i], h1[i], acc);
        h2[j] = acc > 0.0f ? acc : 0.0f;
    }
    for (int j = 0; j < MLP_OUT; ++j) {
        float acc = b3[j];
        for (int i = 0; i < MLP_H; ++i) acc = fmaf(W3[j * MLP_H + i], h2[i], acc);
        z[j] = acc;
    }
    if (out_logits) memcpy(out_logits, z, sizeof z);
    int best = lo;
    for (int j = lo + 1; j < lo + 3; ++j)
        if (z[j] > z[best]) best = j;
    return best;
}

/* Exported for tests: features of one state and the forward pass. */
void orc_features(const uint64_t *ints /* n m F S R a t SD DG Fp D Sp Ip Op k */, double Wm, int delta_mode,
                  float *x) {
    feat_in q = {ints[0], ints[1], ints[2], ints[3], ints[4], ints[5], ints[6], ints[7], ints[8], ints[9],
                 ints[10], ints[11], ints[12], ints[13], ints[14], Wm, delta_mode};
    features(&q, x);
}

int orc_mlp_choice(const float *w, const float *x, int lo, float *logits) { return mlp_choice(w, x, lo, logits); }

static const uint32_t CHOICE_CRIT[3] = {C_IN_STATIC | C_OUT_STATIC, C_IN_SIMPLE | C_OUT_SIMPLE, C_IN_SIMPLE | C_OUT_STATIC};

static const uint32_t ALL_BITS[8] = {C_DIJK, C_IN_STATIC, C_OUT_STATIC, C_IN_SIMPLE,
                                     C_OUT_SIMPLE, C_IN_FULL, C_OUT_WEAK, C_OUT_FULL};

static int chain_ok(uint32_t b, uint32_t evaluated) {
    /* DIJK => every criterion; X-STATIC => X-SIMPLE => (OUTWEAK =>) X; and, when the approximate
     * criteria are evaluated, DIJK and X-STATIC => X-APPROX (an approximate minimum is never below the
     * static one: it is a minimum over a subset of the same edges, each term at least its weight) */
#define IMPL(a, c) (!(b & (a)) || (b & (c)))
    int ok = 1;
    for (int i = 1; i < 8; ++i) ok &= IMPL(C_DIJK, ALL_BITS[i]);
    ok &= IMPL(C_IN_STATIC, C_IN_SIMPLE) & IMPL(C_IN_SIMPLE, C_IN_FULL);
    ok &= IMPL(C_OUT_STATIC, C_OUT_SIMPLE) & IMPL(C_OUT_SIMPLE, C_OUT_WEAK) & IMPL(C_OUT_WEAK, C_OUT_FULL);
    if (evaluated & C_IN_APPROX) ok &= IMPL(C_DIJK, C_IN_APPROX) & IMPL(C_IN_STATIC, C_IN_APPROX);
    if (evaluated & C_OUT_APPROX) ok &= IMPL(C_DIJK, C_OUT_APPROX) & IMPL(C_OUT_STATIC, C_OUT_APPROX);
#undef IMPL
    return ok;
}

/*
 * Approximate criteria (Section 3, closing paragraphs). With each vertex v the
 * paper keeps four minima: min_{w in F} c(w,v) and min_{w in U} (c(w,v) + min_{w'
 * in V} c(w',w)) for IN, min_{w in F} c(v,w) and min_{w in U} (c(v,w) + min_{w' in
 * V} c(w,w')) for OUTWEAK; each criterion uses the smaller of its pair, so one
 * value per side is kept here: in[v] and out[v]. They are maintained
 * conservatively -- never above the exact value, which would be unsound:
 *   - a neighbour w moving U -> F turns its term c + minIn(w) (c + minOut(w)) into
 *     c, a decrease, applied at once: in[v] = min(in[v], c(w,v)) for every out-edge
 *     (w,v), out[u] = min(out[u], c(u,w)) for every in-edge (u,w);
 *   - a neighbour moving F -> S removes a term, which may raise the exact value: it
 *     is only counted (cin[v] per edge (w,v), cout[u] per edge (u,w)); the value is
 *     recomputed from the current state when the vertex is evaluated (queued, at a
 *     phase start) with at least k counted changes, and the count restarts;
 *     k = 0: never recomputed (minima computed once, then only lowered).
 * All values start exact for the state F = {s}. IN-APPROX(v): d[v] - in[v] <= minD;
 * OUT-APPROX(v): d[v] <= min_{u in F} d[u] + out[u]. Changes of a phase are applied
 * after its relaxation, so the next phase's evaluation sees them.
 */
typedef struct {
    uint32_t k;
    uint64_t *in, *out;
    uint32_t *cin, *cout;
} approx_t;

static uint64_t approx_in_exact(uint32_t v, const csc_t *c, const uint8_t *st, const uint64_t *min_in) {
    uint64_t t = INF;
    for (uint64_t e = c->ip[v]; e < c->ip[v + 1]; ++e) {
        uint32_t x = c->is[e];
        if (st[x] == ST_F) t = min64(t, c->iw[e]);
        else if (st[x] == ST_U) t = min64(t, sadd(c->iw[e], min_in[x]));
    }
    return t;
}

static uint64_t approx_out_exact(uint32_t u, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                                 const uint8_t *st, const uint64_t *min_out) {
    uint64_t t = INF;
    for (uint64_t e = rp[u]; e < rp[u + 1]; ++e) {
        uint32_t x = col[e];
        if (st[x] == ST_F) t = min64(t, w[e]);
        else if (st[x] == ST_U) t = min64(t, sadd(w[e], min_out[x]));
    }
    return t;
}

/*
 * The generic phased SSSP algorithm of Section 3 with S' = every v in F for
 * which the criterion (disjunction of `crit` bits) holds on the phase-start
 * snapshot.
 *
 *   crit_seq  optional per-phase criteria: phase k (0-based) uses
 *             crit_seq[min(k, seq_len-1)] instead of crit.
 *   check     evaluate all eight criteria on every snapshot and verify the
 *             strength chains and completeness (DIJK set inside S');
 *             dist_ref, if given, verifies soundness (settled d == dist).
 *   dist_out  final tentative distances = dist(s, .) (INF if unreachable).
 *   trace_*   per phase (up to trace_cap phases): |F| at phase start, |S'|,
 *             minD, and in check mode the number of F vertices each of the
 *             eight criteria certifies (trace_counts[8*k + i], bit order of
 *             ALL_BITS).
 *   phase_of  optional: 1-based phase in which each vertex was settled, 0 if
 *             never (unreachable).
 *   mlp_w     optional selector weights: each phase's criterion is the
 *             selector's choice (crit is ignored); with commit = K > 0 the
 *             choice made for phase K is kept for all later phases.
 */
int orc_phased(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t src,
               uint32_t crit, const uint32_t *crit_seq, uint32_t seq_len, int check,
               const uint64_t *dist_ref, uint64_t *dist_out, orc_stats *stats, uint32_t trace_cap,
               uint32_t *trace_f, uint32_t *trace_s, uint64_t *trace_mind, uint32_t *trace_counts,
               uint32_t *phase_of, const float *mlp_w, uint32_t *trace_crit, uint32_t *trace_union,
               float *trace_feat, uint32_t commit, uint32_t approx_k, uint32_t ckpt) {
    if (src >= n || (crit == 0 && !crit_seq && !mlp_w) || (crit & ~(C_ALL | C_APPROX))) return ORC_EINVAL;
    if ((crit & C_APPROX) && (crit_seq || mlp_w)) return ORC_EINVAL;
    if (ckpt && (!mlp_w || crit != (C_IN_STATIC | C_OUT_STATIC) || crit_seq || commit)) return ORC_EINVAL;
    int rc = ORC_OK;
    csc_t c = {0, 0, 0};
    uint64_t *min_in = (uint64_t *)malloc((uint64_t)n * 8), *min_out = (uint64_t *)malloc((uint64_t)n * 8);
    uint8_t *st = (uint8_t *)calloc(n, 1);
    uint32_t *Fl = (uint32_t *)malloc((uint64_t)n * 4), *Fn = (uint32_t *)malloc((uint64_t)n * 4);
    uint32_t *Sp = (uint32_t *)malloc((uint64_t)n * 4);
    uint64_t *inner = (uint64_t *)malloc((uint64_t)n * 8);
    uint32_t *stamp = (uint32_t *)calloc(n, 4);
    memo_t M = {(uint64_t *)malloc((uint64_t)n * 8), (uint32_t *)calloc(n, 4), 0};
    approx_t A = {approx_k, NULL, NULL, NULL, NULL};
    uint64_t *d = dist_out;
    orc_stats S;
    memset(&S, 0, sizeof S);
    if (!min_in || !min_out || !st || !Fl || !Fn || !Sp || !inner || !stamp || !M.val || !M.stamp ||
        build_csc(n, rp, col, w, &c)) {
        rc = ORC_ENOMEM; goto out;
    }
    static_minima64(n, rp, w, &c, min_in, min_out);
    for (uint32_t v = 0; v < n; ++v) d[v] = INF;
    if (phase_of) memset(phase_of, 0, (uint64_t)n * 4);
    d[src] = 0; st[src] = ST_F;
    if (crit & C_APPROX) {  /* exact approximate minima for the state F = {s} */
        A.in = (uint64_t *)malloc((uint64_t)n * 8);
        A.out = (uint64_t *)malloc((uint64_t)n * 8);
        A.cin = (uint32_t *)calloc(n, 4);
        A.cout = (uint32_t *)calloc(n, 4);
        if (!A.in || !A.out || !A.cin || !A.cout) { rc = ORC_ENOMEM; goto out; }
        for (uint32_t v = 0; v < n; ++v) {
            A.in[v] = approx_in_exact(v, &c, st, min_in);
            A.out[v] = approx_out_exact(v, rp, col, w, st, min_out);
        }
    }
    uint64_t nF = 1;
    Fl[0] = src;
    uint32_t k = 0;
    /* learned mode: |F| of the previous phase and the choice for the next phase */
    uint64_t prevF = 0, settled = 0;
    int choice = 0;
    /* checkpoint mode: the first checkpoint choosing c != 0 switches from phase cp_at on */
    int cp_decided = 0;
    uint32_t cp_at = 0, cp_crit = 0;
    uint64_t cp_fprev = 0;
    double Wm = 1.0;
    if (mlp_w && rp[n] > 0) {  /* exact integer weight sum, then one division */
        uint64_t sw = 0;
        for (uint64_t e = 0; e < rp[n]; ++e) sw += w[e];
        Wm = (double)sw / (double)rp[n];
    }
    if (mlp_w && !ckpt) {  /* phase 0: the state {s}, nothing evaluated yet */
        feat_in q = {n, rp[n], 1, 0, 1, 0, min_out[src], 0, rp[src + 1] - rp[src],
                     0, 0, 0, 0, 0, 0, Wm, 0};
        float x[MLP_IN];
        features(&q, x);
        if (trace_cap && trace_feat) memcpy(trace_feat, x, sizeof x);
        choice = mlp_choice(mlp_w, x, 0, NULL);
    }
    while (nF > 0) {
        uint32_t ck = crit_seq ? crit_seq[k < seq_len ? k : seq_len - 1] : crit;
        uint32_t want = check ? C_ALL | (ck & C_APPROX) : ck;
        thresholds_t T;
        T.minD = INF;
        for (uint64_t i = 0; i < nF; ++i) T.minD = min64(T.minD, d[Fl[i]]);
        if (mlp_w && !ckpt) {
            ck = CHOICE_CRIT[choice];
            want = (check ? C_ALL : ck) | C_IN_STATIC | C_OUT_STATIC;
        }
        if (ckpt && cp_decided && k >= cp_at) {
            ck = cp_crit;
            want = check ? C_ALL : ck;
        }
        if (ck == 0 || (ck & ~(C_ALL | C_APPROX))) { rc = ORC_EINVAL; goto out; }
        if (k < trace_cap && trace_crit) trace_crit[k] = ck;
        out_thresholds(want, Fl, nF, rp, col, w, d, st, min_out, inner, stamp, k + 1, &T);
        M.now = k + 1;
        uint64_t t_apx = INF;
        if (want & C_APPROX) {
            /* queued vertices with k or more counted changes recompute from this snapshot */
            for (uint64_t i = 0; i < nF; ++i) {
                uint32_t v = Fl[i];
                if (A.k && A.cin[v] >= A.k) { A.in[v] = approx_in_exact(v, &c, st, min_in); A.cin[v] = 0; }
                if (A.k && A.cout[v] >= A.k) { A.out[v] = approx_out_exact(v, rp, col, w, st, min_out); A.cout[v] = 0; }
            }
            for (uint64_t i = 0; i < nF; ++i) t_apx = min64(t_apx, sadd(d[Fl[i]], A.out[Fl[i]]));
        }
        uint32_t cnt[8] = {0}, uni[3] = {0, 0, 0};
        uint64_t nS = 0, nK = 0, nin = 0, nout = 0;
        for (uint64_t i = 0; i < nF; ++i) {
            uint32_t v = Fl[i];
            uint32_t b = eval_bits(v, want, &T, d, st, min_in, &c, &M);
            if ((want & C_IN_APPROX) && d[v] <= sadd(T.minD, A.in[v])) b |= C_IN_APPROX;
            if ((want & C_OUT_APPROX) && d[v] <= t_apx) b |= C_OUT_APPROX;
            nin += (b & C_IN_STATIC) ? 1 : 0;
            nout += (b & C_OUT_STATIC) ? 1 : 0;
            if (check) {
                for (int j = 0; j < 8; ++j) cnt[j] += (b & ALL_BITS[j]) ? 1 : 0;
                for (int j = 0; j < 3; ++j) uni[j] += (b & CHOICE_CRIT[j]) ? 1 : 0;
                if (!chain_ok(b, want)) { rc = ORC_ECHAIN; goto out; }
                if (d[v] == T.minD && !(b & C_DIJK)) { rc = ORC_EINCOMPLETE; goto out; }
            }
            if (b & ck) {
                if (dist_ref && d[v] != dist_ref[v]) { rc = ORC_EUNSOUND; goto out; }
                Sp[nS++] = v;
            } else {
                Fn[nK++] = v;
            }
        }
        if (nS == 0) { rc = ORC_EINCOMPLETE; goto out; }
        if (k < trace_cap) {
            if (trace_f) trace_f[k] = (uint32_t)nF;
            if (trace_s) trace_s[k] = (uint32_t)nS;
            if (trace_mind) trace_mind[k] = T.minD;
            if (trace_counts) memcpy(trace_counts + 8ull * k, cnt, sizeof cnt);
            if (trace_union) memcpy(trace_union + 3ull * k, uni, sizeof uni);
        }
        if (ckpt && !cp_decided && (k + 1) % 16 == 0) {
            /* checkpoint after the last phase of a batch of 16: phase k's snapshot and outcome,
             * |F| at the previous checkpoint; no SD, DG, Ip, Op (delta_mode 2) */
            feat_in q = {n, rp[n], nF, settled, nF + settled, T.minD, T.t_out_static, 0, 0, cp_fprev, nF, nS, 0, 0,
                         k + 1, Wm, 2};
            float x[MLP_IN];
            features(&q, x);
            uint32_t j = k / 16;
            if (j < trace_cap && trace_feat) memcpy(trace_feat + (uint64_t)MLP_IN * j, x, sizeof x);
            int c = mlp_choice(mlp_w, x, 0, NULL);
            cp_fprev = nF;
            if (c != 0) { cp_decided = 1; cp_at = k + 17; cp_crit = CHOICE_CRIT[c]; }
        }
        if (mlp_w && !ckpt && (!commit || k + 1 <= commit)) {
            /* the selector for phase k+1, on phase k's snapshot and outcome (with a commit phase
             * K > 0, phase K's choice is kept for every later phase) */
            uint64_t SD = 0, DG = 0;
            for (uint64_t i = 0; i < nF; ++i) { SD += d[Fl[i]]; DG += rp[Fl[i] + 1] - rp[Fl[i]]; }
            feat_in q = {n, rp[n], nF, settled, nF + settled, T.minD, T.t_out_static, SD, DG, prevF, nF, nS, nin,
                         nout, k + 1, Wm, 0};
            float x[MLP_IN];
            features(&q, x);
            if (k + 1 < trace_cap && trace_feat) memcpy(trace_feat + (uint64_t)MLP_IN * (k + 1), x, sizeof x);
            choice = mlp_choice(mlp_w, x, 0, NULL);
        }
        prevF = nF; settled += nS;
        S.sum_f += nF;
        /* settle all of S' (moved to S), then relax their out-edges */
        for (uint64_t i = 0; i < nS; ++i) st[Sp[i]] = ST_S;
        if (phase_of) for (uint64_t i = 0; i < nS; ++i) phase_of[Sp[i]] = k + 1;
        const uint64_t nK0 = nK;  /* Fn[nK0 ..] will hold the vertices this relaxation discovers */
        for (uint64_t i = 0; i < nS; ++i) {
            uint32_t u = Sp[i];
            S.m_reach += rp[u + 1] - rp[u];
            for (uint64_t e = rp[u]; e < rp[u + 1]; ++e) {
                uint32_t x = col[e];
                if (st[x] == ST_S) continue;
                S.relax_edges++;
                uint64_t cand = d[u] + w[e];
                if (cand < d[x]) {
                    d[x] = cand;
                    S.improving++;
                    if (st[x] == ST_U) { st[x] = ST_F; Fn[nK++] = x; }
                }
            }
        }
        S.n_reach += nS;
        if (crit & C_APPROX) {
            /* F -> S moves are counted on both sides of each edge of a settled vertex */
            for (uint64_t i = 0; i < nS; ++i) {
                uint32_t x = Sp[i];
                for (uint64_t e = rp[x]; e < rp[x + 1]; ++e) A.cin[col[e]]++;
                for (uint64_t e = c.ip[x]; e < c.ip[x + 1]; ++e) A.cout[c.is[e]]++;
            }
            /* U -> F moves lower the neighbours' minima at once */
            for (uint64_t i = nK0; i < nK; ++i) {
                uint32_t x = Fn[i];
                for (uint64_t e = rp[x]; e < rp[x + 1]; ++e) A.in[col[e]] = min64(A.in[col[e]], w[e]);
                for (uint64_t e = c.ip[x]; e < c.ip[x + 1]; ++e) A.out[c.is[e]] = min64(A.out[c.is[e]], c.iw[e]);
            }
        }
        uint32_t *t = Fl; Fl = Fn; Fn = t;
        nF = nK;
        ++k;
    }
    S.phases = k;
    if (dist_ref)
        for (uint32_t v = 0; v < n; ++v)
            if (d[v] != dist_ref[v]) { rc = ORC_EDIST; goto out; }
out:
    if (stats) *stats = S;
    free(min_in); free(min_out); free(st); free(Fl); free(Fn); free(Sp); free(inner); free(stamp);
    free(M.val); free(M.stamp);
    free(A.in); free(A.out); free(A.cin); free(A.cout);
    free_csc(&c);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Delta-stepping (Section 5), one bucket width per bucket.                  */

typedef struct {
    uint32_t rounds;       /* light rounds + heavy rounds (one per bucket) */
    uint32_t buckets;
    uint64_t light_relax;  /* light-edge relaxations (re-relaxations included) */
    uint64_t heavy_relax;
    uint64_t sum_frontier; /* sum of light-round frontier sizes */
} orc_dstats;

int orc_delta_step(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w,
                   uint32_t src, const uint64_t *deltas, uint32_t n_deltas, uint64_t *dist_out,
                   orc_dstats *stats, uint32_t trace_cap, uint64_t *trace_delta, const float *mlp_w) {
    if (src >= n || (n_deltas == 0 && !mlp_w)) return ORC_EINVAL;
    for (uint32_t i = 0; i < n_deltas; ++i) if (deltas[i] == 0) return ORC_EINVAL;
    double Wm = 1.0;
    if (mlp_w && rp[n] > 0) {  /* exact integer weight sum, then one division */
        uint64_t sw = 0;
        for (uint64_t e = 0; e < rp[n]; ++e) sw += w[e];
        Wm = (double)sw / (double)rp[n];
    }
    uint64_t Fp = 0, Sp = 0, settled = 0;
    int rc = ORC_OK;
    uint64_t *d = dist_out;
    uint8_t *st = (uint8_t *)calloc(n, 1);
    uint8_t *inR = (uint8_t *)calloc(n, 1);
    uint32_t *mark = (uint32_t *)calloc(n, 4);
    uint32_t *Fl = (uint32_t *)malloc((uint64_t)n * 4), *Fn = (uint32_t *)malloc((uint64_t)n * 4);
    uint32_t *X = (uint32_t *)malloc((uint64_t)n * 4), *Xn = (uint32_t *)malloc((uint64_t)n * 4);
    uint64_t *xd = (uint64_t *)malloc((uint64_t)n * 8);
    uint32_t *R = (uint32_t *)malloc((uint64_t)n * 4);
    orc_dstats D;
    memset(&D, 0, sizeof D);
    if (!st || !inR || !mark || !Fl || !Fn || !X || !Xn || !xd || !R) { rc = ORC_ENOMEM; goto out; }
    for (uint32_t v = 0; v < n; ++v) d[v] = INF;
    d[src] = 0; st[src] = ST_F;
    /* Fl holds every reached, unsettled vertex (plus, transiently, vertices
     * first reached during the current bucket, appended at the end). */
    uint64_t nF = 1;
    Fl[0] = src;
    uint32_t rstamp = 0;
    while (nF > 0) {
        uint64_t minD = INF;
        for (uint64_t i = 0; i < nF; ++i) minD = min64(minD, d[Fl[i]]);
        uint64_t delta;
        if (mlp_w) {
            feat_in q = {n, rp[n], nF, settled, nF + settled, minD, INF, 0, 0, 0, Fp, Sp, 0, 0, D.buckets, Wm, 1};
            float x[MLP_IN];
            features(&q, x);
            delta = 1ull << (12 + 2 * (mlp_choice(mlp_w, x, 3, NULL) - 3));
        } else {
            delta = deltas[D.buckets < n_deltas ? D.buckets : n_deltas - 1];
        }
        if (D.buckets < trace_cap && trace_delta) trace_delta[D.buckets] = delta;
        Fp = nF;
        uint64_t lo = (minD / delta) * delta;  /* bucket floor(minD / delta) */
        uint64_t hi = sadd(lo, delta);
        uint64_t nX = 0, nR = 0, nF0 = nF;
        for (uint64_t i = 0; i < nF; ++i) if (d[Fl[i]] < hi) X[nX++] = Fl[i];
        while (nX > 0) { /* light rounds */
            ++rstamp;
            D.rounds++;
            D.sum_frontier += nX;
            for (uint64_t i = 0; i < nX; ++i) {
                xd[i] = d[X[i]]; /* round-start distance */
                if (!inR[X[i]]) { inR[X[i]] = 1; R[nR++] = X[i]; }
            }
            uint64_t nXn = 0;
            for (uint64_t i = 0; i < nX; ++i) {
                uint32_t u = X[i];
                for (uint64_t e = rp[u]; e < rp[u + 1]; ++e) {
                    if ((uint64_t)w[e] >= delta) continue; /* light: c < delta */
                    uint32_t x = col[e];
                    if (st[x] == ST_S) continue;
                    D.light_relax++;
                    uint64_t cand = xd[i] + w[e];
                    if (cand < d[x]) {
                        d[x] = cand;
                        if (st[x] == ST_U) { st[x] = ST_F; Fl[nF++] = x; }
                        if (cand < hi && mark[x] != rstamp) { mark[x] = rstamp; Xn[nXn++] = x; }
                    }
                }
            }
            uint32_t *t = X; X = Xn; Xn = t;
            nX = nXn;
        }
        /* heavy round: everything the bucket removed is settled and relaxes
         * its heavy edges once */
        D.rounds++;
        Sp = nR;
        settled += nR;
        for (uint64_t i = 0; i < nR; ++i) { st[R[i]] = ST_S; inR[R[i]] = 0; }
        for (uint64_t i = 0; i < nR; ++i) {
            uint32_t u = R[i];
            for (uint64_t e = rp[u]; e < rp[u + 1]; ++e) {
                if ((uint64_t)w[e] < delta) continue; /* heavy: c >= delta */
                uint32_t x = col[e];
                if (st[x] == ST_S) continue;
                D.heavy_relax++;
                uint64_t cand = d[u] + w[e];
                if (cand < d[x]) {
                    d[x] = cand;
                    if (st[x] == ST_U) { st[x] = ST_F; Fl[nF++] = x; }
                }
            }
        }
        D.buckets++;
        (void)nF0;
        uint64_t k2 = 0;
        for (uint64_t i = 0; i < nF; ++i) if (st[Fl[i]] == ST_F) Fn[k2++] = Fl[i];
        uint32_t *t = Fl; Fl = Fn; Fn = t;
        nF = k2;
    }
out:
    if (stats) *stats = D;
    free(st); free(inR); free(mark); free(Fl); free(Fn); free(X); free(Xn); free(xd); free(R);
    return rc;
}
