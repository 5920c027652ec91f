/*
 * Sanitizer driver for the CPU oracle and the input generators -- TEST INFRASTRUCTURE ONLY.
 *
 * Built by the tests with gcc -fsanitize=address,undefined together with
 * oracle.c and graphgen/gen.c, and fed on stdin; every result is printed so
 * that the test can compare it with the ordinary (-O2) build. Commands, one
 * per line:
 *   G n m src k d_1 .. d_k     followed by m lines "u v w" in row order: the
 *                              graph is checked (orc_validate), solved with
 *                              Dijkstra, Bellman-Ford (n <= 64), every
 *                              criterion of the list below in check mode
 *                              against Dijkstra, and Delta-stepping with each
 *                              width d_i.
 *   E n k wlo whi seed         generate a random graph (gg_er), then as G with
 *   R scale ef wlo whi seed    source gg_sources(.., 1, seed) and no widths;
 *   D W H wlo whi seed         R-MAT (gg_rmat) and grid (gg_grid) likewise.
 * Output per graph: "OK n m src hash(dist) n_reach" then, per criterion,
 * "phases sum_f", then per width "rounds buckets", all on one line; a
 * generated graph first prints "GEN hash(row_ptr, col, w)".
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint32_t phases, pad;
    uint64_t sum_f, n_reach, m_reach, relax_edges, improving;
} orc_stats;
typedef struct {
    uint32_t rounds, buckets;
    uint64_t light_relax, heavy_relax, sum_frontier;
} orc_dstats;

int orc_validate(uint32_t n, const uint64_t *rp, const uint32_t *col);
int64_t orc_dijkstra(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t src,
                     uint64_t *dist, uint32_t *hops);
int orc_bellman_ford(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t src,
                     uint64_t *dist);
int orc_static_minima(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t *min_in,
                      uint32_t *min_out);
int orc_phased(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t src, uint32_t crit,
               const uint32_t *crit_seq, uint32_t seq_len, int check, const uint64_t *dist_ref, uint64_t *dist_out,
               orc_stats *stats, uint32_t trace_cap, uint32_t *trace_f, uint32_t *trace_s, uint64_t *trace_mind,
               uint32_t *trace_counts, uint32_t *phase_of, const float *mlp_w, uint32_t *trace_crit,
               uint32_t *trace_union, float *trace_feat, uint32_t commit, uint32_t approx_k, uint32_t ckpt);
int orc_delta_step(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t src,
                   const uint64_t *deltas, uint32_t n_deltas, uint64_t *dist_out, orc_dstats *stats,
                   uint32_t trace_cap, uint64_t *trace_delta, const float *mlp_w);
int gg_er(uint32_t n, uint32_t k, uint32_t wlo, uint32_t whi, uint64_t seed, uint64_t *row_ptr, uint32_t *col,
          uint32_t *w);
int gg_rmat(uint32_t scale, uint32_t ef, uint32_t a16, uint32_t b16, uint32_t c16, uint32_t wlo, uint32_t whi,
            uint64_t seed, int permute, uint64_t *row_ptr, uint32_t *col, uint32_t *w, uint64_t *m_out);
int gg_grid(uint32_t W, uint32_t H, uint32_t wlo, uint32_t whi, uint64_t seed, uint64_t *row_ptr, uint32_t *col,
            uint32_t *w);
int gg_sources(uint32_t n, const uint64_t *row_ptr, uint32_t count, uint64_t seed, uint32_t *out);

/* the criteria, as bit sets: each single bit, the three disjunctions, IN_FULL|OUT_WEAK, and the
 * approximate pair with DIJK (recomputed every second change) */
static const uint32_t CRITS[] = {1, 2, 4, 8, 16, 32, 64, 128, 6, 24, 160, 96, 769};
#define NCRIT (sizeof CRITS / sizeof CRITS[0])

static uint64_t fnv(uint64_t h, const void *p, size_t len) {
    const unsigned char *b = (const unsigned char *)p;
    for (size_t i = 0; i < len; ++i) h = (h ^ b[i]) * 1099511628211ull;
    return h;
}

static int solve_all(uint32_t n, const uint64_t *rp, const uint32_t *col, const uint32_t *w, uint32_t src,
                     const uint64_t *deltas, uint32_t k) {
    if (orc_validate(n, rp, col) != 0) { printf("INVALID\n"); return 0; }
    uint64_t *d = malloc((n ? n : 1) * 8), *bf = malloc((n ? n : 1) * 8), *x = malloc((n ? n : 1) * 8);
    uint32_t *hops = malloc((n ? n : 1) * 4), *mi = malloc((n ? n : 1) * 4), *mo = malloc((n ? n : 1) * 4);
    int rc = 0;
    int64_t nr = orc_dijkstra(n, rp, col, w, src, d, hops);
    if (nr < 0) { rc = 1; goto out; }
    if (n <= 64) {
        if (orc_bellman_ford(n, rp, col, w, src, bf) != 0 || memcmp(bf, d, (size_t)n * 8)) { rc = 2; goto out; }
    }
    if (orc_static_minima(n, rp, col, w, mi, mo) != 0) { rc = 3; goto out; }
    printf("OK %u %llu %u %llu %lld", n, (unsigned long long)rp[n], src,
           (unsigned long long)fnv(14695981039346656037ull, d, (size_t)n * 8), (long long)nr);
    for (size_t c = 0; c < NCRIT; ++c) {
        orc_stats st;
        int r = orc_phased(n, rp, col, w, src, CRITS[c], NULL, 0, 1, d, x, &st, 0, NULL, NULL, NULL, NULL, NULL,
                           NULL, NULL, NULL, NULL, 0, 2, 0);
        if (r != 0 || memcmp(x, d, (size_t)n * 8)) { rc = 4; goto out; }
        printf(" %u %llu", st.phases, (unsigned long long)st.sum_f);
    }
    for (uint32_t i = 0; i < k; ++i) {
        orc_dstats ds;
        if (orc_delta_step(n, rp, col, w, src, deltas + i, 1, x, &ds, 0, NULL, NULL) != 0 ||
            memcmp(x, d, (size_t)n * 8)) { rc = 5; goto out; }
        printf(" %u %u", ds.rounds, ds.buckets);
    }
    printf("\n");
out:
    free(d); free(bf); free(x); free(hops); free(mi); free(mo);
    return rc;
}

int main(void) {
    char cmd[4];
    while (scanf("%3s", cmd) == 1) {
        int rc = 0;
        if (cmd[0] == 'G') {
            uint32_t n, src, k;
            unsigned long long m;
            if (scanf("%u %llu %u %u", &n, &m, &src, &k) != 4) return 10;
            uint64_t *deltas = malloc((k ? k : 1) * 8);
            for (uint32_t i = 0; i < k; ++i) {
                unsigned long long t;
                if (scanf("%llu", &t) != 1) return 11;
                deltas[i] = t;
            }
            uint64_t *rp = calloc((size_t)n + 1, 8);
            uint32_t *col = malloc((m ? m : 1) * 4), *w = malloc((m ? m : 1) * 4);
            for (unsigned long long e = 0; e < m; ++e) {
                unsigned u, v, c;
                if (scanf("%u %u %u", &u, &v, &c) != 3 || u >= n) return 12;
                rp[u + 1]++;
                col[e] = v;
                w[e] = c;
            }
            for (uint32_t v = 0; v < n; ++v) rp[v + 1] += rp[v];
            rc = solve_all(n, rp, col, w, src, deltas, k);
            free(deltas); free(rp); free(col); free(w);
        } else if (cmd[0] == 'E' || cmd[0] == 'R' || cmd[0] == 'D') {
            unsigned a, b, wlo, whi;
            unsigned long long seed;
            if (scanf("%u %u %u %u %llu", &a, &b, &wlo, &whi, &seed) != 5) return 13;
            uint32_t n = cmd[0] == 'E' ? a : cmd[0] == 'R' ? (1u << a) : a * b;
            uint64_t mcap = cmd[0] == 'E' ? (uint64_t)a * b : cmd[0] == 'R' ? ((uint64_t)b << a) : 4ull * a * b;
            uint64_t *rp = calloc((size_t)n + 1, 8);
            uint32_t *col = malloc(mcap * 4), *w = malloc(mcap * 4);
            uint64_t m = mcap;
            int g = cmd[0] == 'E' ? gg_er(n, b, wlo, whi, seed, rp, col, w)
                  : cmd[0] == 'R' ? gg_rmat(a, b, 37356, 12452, 12452, wlo, whi, seed, 1, rp, col, w, &m)
                                  : gg_grid(a, b, wlo, whi, seed, rp, col, w);
            if (g != 0) return 14;
            m = rp[n];
            uint64_t h = fnv(14695981039346656037ull, rp, ((size_t)n + 1) * 8);
            h = fnv(h, col, m * 4);
            h = fnv(h, w, m * 4);
            uint32_t src = 0;
            if (gg_sources(n, rp, 1, seed, &src) != 0) return 15;
            printf("GEN %llu\n", (unsigned long long)h);
            rc = solve_all(n, rp, col, w, src, NULL, 0);
            free(rp); free(col); free(w);
        } else {
            return 16;
        }
        if (rc) { printf("FAIL %d\n", rc); return rc; }
        fflush(stdout);
    }
    return 0;
}
