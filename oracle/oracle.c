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
    C_ALL = 0xFFu
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
 * weight over all in-edges / all out-edges; U32INF when there are none. */
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

static inline uint64_t w64(uint32_t x) { return x == U32INF ? INF : (uint64_t)x; }

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

static uint64_t in_full_term(uint32_t v, const csc_t *c, const uint8_t *st) {
    /* crit:in: min( min_{w in F, (w,v)} c(w,v),
     *               min_{w in U, w' in F u U, (w,v), (w',w)} c(w,v) + c(w',w) ) */
    uint64_t t = INF;
    for (uint64_t e = c->ip[v]; e < c->ip[v + 1]; ++e) {
        uint32_t wv = c->is[e];
        if (st[wv] == ST_F) {
            t = min64(t, c->iw[e]);
        } else if (st[wv] == ST_U) {
            uint64_t inner = INF;
            for (uint64_t f = c->ip[wv]; f < c->ip[wv + 1]; ++f)
                if (st[c->is[f]] != ST_S) inner = min64(inner, c->iw[f]);
            t = min64(t, sadd(c->iw[e], inner));
        }
    }
    return t;
}

static uint32_t eval_bits(uint32_t v, uint32_t want, const thresholds_t *T, const uint64_t *d,
                          const uint8_t *st, const uint32_t *min_in, const csc_t *c) {
    uint32_t b = 0;
    uint64_t dv = d[v];
    if ((want & C_DIJK) && dv == T->minD) b |= C_DIJK;
    if ((want & C_IN_STATIC) && dv <= sadd(T->minD, w64(min_in[v]))) b |= C_IN_STATIC;
    if ((want & C_IN_SIMPLE) && dv <= sadd(T->minD, in_simple_term(v, c, st))) b |= C_IN_SIMPLE;
    if ((want & C_IN_FULL) && dv <= sadd(T->minD, in_full_term(v, c, st))) b |= C_IN_FULL;
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
                           const uint32_t *min_out, uint64_t *inner_ns, uint32_t *memo_stamp,
                           uint32_t stamp, thresholds_t *T) {
    T->t_out_static = T->t_out_simple = T->t_out_weak = T->t_out_full = INF;
    const uint32_t dyn = want & (C_OUT_SIMPLE | C_OUT_WEAK | C_OUT_FULL);
    for (uint64_t i = 0; i < nF; ++i) {
        uint32_t u = Flist[i];
        uint64_t du = d[u];
        /* crit:outstatic: min over u in F and all out-edges (u, w) of d[u] + c(u, w)
         * = d[u] + minOut[u], the precomputed static minimum (Section 3) */
        if (want & C_OUT_STATIC) T->t_out_static = min64(T->t_out_static, sadd(du, w64(min_out[u])));
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
                    T->t_out_weak = min64(T->t_out_weak, sadd(sadd(du, c), w64(min_out[x])));
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

static const uint32_t ALL_BITS[8] = {C_DIJK, C_IN_STATIC, C_OUT_STATIC, C_IN_SIMPLE,
                                     C_OUT_SIMPLE, C_IN_FULL, C_OUT_WEAK, C_OUT_FULL};

static int chain_ok(uint32_t b) {
    /* DIJK => every criterion; X-STATIC => X-SIMPLE => (OUTWEAK =>) X */
#define IMPL(a, c) (!(b & (a)) || (b & (c)))
    int ok = 1;
    for (int i = 1; i < 8; ++i) ok &= IMPL(C_DIJK, ALL_BITS[i]);
    ok &= IMPL(C_IN_STATIC, C_IN_SIMPLE) & IMPL(C_IN_SIMPLE, C_IN_FULL);
    ok &= IMPL(C_OUT_STATIC, C_OUT_SIMPLE) & IMPL(C_OUT_SIMPLE, C_OUT_WEAK) & IMPL(C_OUT_WEAK, C_OUT_FULL);
#undef IMPL
    return ok;
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
 */
int orc_phased(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t src,
               uint32_t crit, const uint32_t *crit_seq, uint32_t seq_len, int check,
               const uint64_t *dist_ref, uint64_t *dist_out, orc_stats *stats, uint32_t trace_cap,
               uint32_t *trace_f, uint32_t *trace_s, uint64_t *trace_mind, uint32_t *trace_counts,
               uint32_t *phase_of) {
    if (src >= n || (crit == 0 && !crit_seq) || (crit & ~C_ALL)) return ORC_EINVAL;
    int rc = ORC_OK;
    csc_t c = {0, 0, 0};
    uint32_t *min_in = (uint32_t *)malloc((uint64_t)n * 4), *min_out = (uint32_t *)malloc((uint64_t)n * 4);
    uint8_t *st = (uint8_t *)calloc(n, 1);
    uint32_t *Fl = (uint32_t *)malloc((uint64_t)n * 4), *Fn = (uint32_t *)malloc((uint64_t)n * 4);
    uint32_t *Sp = (uint32_t *)malloc((uint64_t)n * 4);
    uint64_t *inner = (uint64_t *)malloc((uint64_t)n * 8);
    uint32_t *stamp = (uint32_t *)calloc(n, 4);
    uint64_t *d = dist_out;
    orc_stats S;
    memset(&S, 0, sizeof S);
    if (!min_in || !min_out || !st || !Fl || !Fn || !Sp || !inner || !stamp || build_csc(n, rp, col, w, &c)) {
        rc = ORC_ENOMEM; goto out;
    }
    static_minima(n, rp, w, &c, min_in, min_out);
    for (uint32_t v = 0; v < n; ++v) d[v] = INF;
    if (phase_of) memset(phase_of, 0, (uint64_t)n * 4);
    d[src] = 0; st[src] = ST_F;
    uint64_t nF = 1;
    Fl[0] = src;
    uint32_t k = 0;
    while (nF > 0) {
        uint32_t ck = crit_seq ? crit_seq[k < seq_len ? k : seq_len - 1] : crit;
        if (ck == 0 || (ck & ~C_ALL)) { rc = ORC_EINVAL; goto out; }
        uint32_t want = check ? C_ALL : ck;
        thresholds_t T;
        T.minD = INF;
        for (uint64_t i = 0; i < nF; ++i) T.minD = min64(T.minD, d[Fl[i]]);
        out_thresholds(want, Fl, nF, rp, col, w, d, st, min_out, inner, stamp, k + 1, &T);
        uint32_t cnt[8] = {0};
        uint64_t nS = 0, nK = 0;
        for (uint64_t i = 0; i < nF; ++i) {
            uint32_t v = Fl[i];
            uint32_t b = eval_bits(v, want, &T, d, st, min_in, &c);
            if (check) {
                for (int j = 0; j < 8; ++j) cnt[j] += (b & ALL_BITS[j]) ? 1 : 0;
                if (!chain_ok(b)) { rc = ORC_ECHAIN; goto out; }
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
        }
        S.sum_f += nF;
        /* settle all of S' (moved to S), then relax their out-edges */
        for (uint64_t i = 0; i < nS; ++i) st[Sp[i]] = ST_S;
        if (phase_of) for (uint64_t i = 0; i < nS; ++i) phase_of[Sp[i]] = k + 1;
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
                   orc_dstats *stats, uint32_t trace_cap, uint64_t *trace_delta) {
    if (src >= n || n_deltas == 0) return ORC_EINVAL;
    for (uint32_t i = 0; i < n_deltas; ++i) if (deltas[i] == 0) return ORC_EINVAL;
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
        uint64_t delta = deltas[D.buckets < n_deltas ? D.buckets : n_deltas - 1];
        if (D.buckets < trace_cap && trace_delta) trace_delta[D.buckets] = delta;
        uint64_t minD = INF;
        for (uint64_t i = 0; i < nF; ++i) minD = min64(minD, d[Fl[i]]);
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
