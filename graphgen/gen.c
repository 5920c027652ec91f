/*
 * Seeded synthetic graph generators (input construction only).
 *
 * This file builds the directed, non-negatively weighted graphs that both the
 * CPU oracle and the GPU solver consume. It holds none of the shortest-path
 * method's arithmetic: it only draws random numbers and lays edges out in
 * compressed sparse row (CSR) form, sorted by (source, target).
 *
 * Random numbers come from SplitMix64 used as a counter-based generator: the
 * i-th output of a SplitMix64 stream with state `key` is mix(key + (i+1)*G),
 * G = 0x9E3779B97F4A7C15, mix = the published SplitMix64 finaliser
 * (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014). Every draw is addressed by (stream key, counter), so output is
 * independent of thread count and call order.
 *
 * Families (the workloads of the paper's simulation and benchmark sections):
 *   - Erdos-Renyi style, fixed out-degree: each vertex gets exactly k distinct
 *     uniform targets other than itself.
 *   - R-MAT / Kronecker with initiator (a, b, c, d): recursive quadrant
 *     choice per edge, self-loops dropped, duplicate (u, v) pairs merged,
 *     vertex ids scrambled by a seeded permutation.
 *   - W x H 4-neighbour grid, every directed edge with its own weight (the
 *     paper's road-network treatment gives each direction an independent
 *     weight).
 * Weights are uniform integers in [wlo, whi] drawn per CSR edge slot.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* i-th output of the SplitMix64 stream whose state starts at `key`. */
static inline uint64_t sm_at(uint64_t key, uint64_t i) { return sm_mix(key + (i + 1) * GOLDEN); }

/* Stream key for (seed, purpose tag). */
static inline uint64_t stream_key(uint64_t seed, uint64_t tag) {
    return sm_mix(seed * 0xD1B54A32D192ED03ULL + tag * GOLDEN + 0x632BE59BD9B4E019ULL);
}

/* Uniform integer in [0, r) from the high 32 bits (multiply-shift). r <= 2^32. */
static inline uint64_t below(uint64_t x, uint64_t r) { return ((x >> 32) * r) >> 32; }

/* Uniform in [0, r) for r up to 2^64 using 128-bit multiply-high. */
static inline uint64_t below64(uint64_t x, uint64_t r) {
    return (uint64_t)(((unsigned __int128)x * (unsigned __int128)r) >> 64);
}

enum { TAG_ER_TGT = 1, TAG_W = 2, TAG_RMAT = 3, TAG_PERM = 4, TAG_SRC = 5, TAG_U64 = 6 };

static void fill_weights(uint64_t seed, uint64_t m, uint32_t wlo, uint32_t whi, uint32_t *w) {
    uint64_t key = stream_key(seed, TAG_W);
    uint64_t span = (uint64_t)whi - (uint64_t)wlo + 1;
    for (uint64_t e = 0; e < m; ++e) w[e] = wlo + (uint32_t)below64(sm_at(key, e), span);
}

static int cmp_u32(const void *a, const void *b) {
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return (x > y) - (x < y);
}

/* Fixed out-degree random digraph: n vertices, k distinct targets != v each.
 * row_ptr: n+1, col: n*k, w: n*k. Returns 0, or -1 if k >= n. */
int gg_er(uint32_t n, uint32_t k, uint32_t wlo, uint32_t whi, uint64_t seed,
          uint64_t *row_ptr, uint32_t *col, uint32_t *w) {
    if (n < 2 || k >= n) return -1;
    uint64_t key = stream_key(seed, TAG_ER_TGT);
    for (uint32_t v = 0; v < n; ++v) {
        uint32_t *row = col + (uint64_t)v * k;
        uint64_t attempt = 0;
        for (uint32_t j = 0; j < k;) {
            uint64_t x = sm_at(key, ((uint64_t)v << 24) + attempt++);
            uint32_t t = (uint32_t)below(x, n - 1);
            if (t >= v) ++t; /* skip the self-loop */
            int dup = 0;
            for (uint32_t q = 0; q < j; ++q) dup |= (row[q] == t);
            if (!dup) row[j++] = t;
        }
        qsort(row, k, sizeof(uint32_t), cmp_u32);
        row_ptr[v] = (uint64_t)v * k;
    }
    row_ptr[n] = (uint64_t)n * k;
    fill_weights(seed, (uint64_t)n * k, wlo, whi, w);
    return 0;
}

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* LSD radix sort of 64-bit keys (8 passes of 8 bits); tmp has room for cnt keys. */
static void radix_u64(uint64_t *keys, uint64_t *tmp, uint64_t cnt) {
    uint64_t *src = keys, *dst = tmp;
    for (int pass = 0; pass < 8; ++pass) {
        uint64_t hist[256] = {0};
        int sh = pass * 8;
        for (uint64_t i = 0; i < cnt; ++i) hist[(src[i] >> sh) & 255]++;
        uint64_t s = 0;
        for (int b = 0; b < 256; ++b) { uint64_t c = hist[b]; hist[b] = s; s += c; }
        for (uint64_t i = 0; i < cnt; ++i) dst[hist[(src[i] >> sh) & 255]++] = src[i];
        uint64_t *t = src; src = dst; dst = t;
    }
    /* 8 passes: result is back in keys */
}

/* Seeded permutation of [0, n) (Fisher-Yates driven by the counter stream). */
static void seeded_perm(uint64_t seed, uint32_t n, uint32_t *perm) {
    uint64_t key = stream_key(seed, TAG_PERM);
    for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    for (uint32_t i = n - 1; i > 0; --i) {
        uint32_t j = (uint32_t)below64(sm_at(key, i), (uint64_t)i + 1);
        uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
}

/* R-MAT. Samples ef * 2^scale edges with quadrant probabilities (a, b, c,
 * 1-a-b-c) given in units of 1/65536, drops self-loops, merges duplicates,
 * permutes ids (permute != 0). col and w must hold ef * 2^scale entries;
 * *m_out receives the final edge count. scale <= 30. */
int gg_rmat(uint32_t scale, uint32_t ef, uint32_t a16, uint32_t b16, uint32_t c16,
            uint32_t wlo, uint32_t whi, uint64_t seed, int permute,
            uint64_t *row_ptr, uint32_t *col, uint32_t *w, uint64_t *m_out) {
    if (scale < 1 || scale > 30 || a16 + b16 + c16 > 65536) return -1;
    uint32_t n = 1u << scale;
    uint64_t ms = (uint64_t)ef << scale;
    uint64_t *keys = (uint64_t *)malloc(ms * sizeof(uint64_t));
    uint64_t *tmp = (uint64_t *)malloc(ms * sizeof(uint64_t));
    uint32_t *perm = (uint32_t *)malloc((uint64_t)n * sizeof(uint32_t));
    if (!keys || !tmp || !perm) { free(keys); free(tmp); free(perm); return -2; }
    if (permute) seeded_perm(seed, n, perm);
    else for (uint32_t i = 0; i < n; ++i) perm[i] = i;
    uint64_t key = stream_key(seed, TAG_RMAT);
    uint32_t tab = a16, tabb = a16 + b16, tabbc = a16 + b16 + c16;
    uint32_t draws = (scale + 3) / 4; /* four 16-bit quadrant draws per 64-bit output */
    uint64_t cnt = 0;
    for (uint64_t e = 0; e < ms; ++e) {
        uint32_t u = 0, v = 0;
        for (uint32_t d = 0; d < draws; ++d) {
            uint64_t x = sm_at(key, e * draws + d);
            for (uint32_t q = 0; q < 4; ++q) {
                uint32_t lvl = d * 4 + q;
                if (lvl >= scale) break;
                uint32_t r = (uint32_t)((x >> (16 * q)) & 0xFFFF);
                uint32_t bit = 1u << (scale - 1 - lvl);
                if (r < tab) { /* top-left */ }
                else if (r < tabb) v |= bit;
                else if (r < tabbc) u |= bit;
                else { u |= bit; v |= bit; }
            }
        }
        u = perm[u]; v = perm[v];
        if (u == v) continue;
        keys[cnt++] = ((uint64_t)u << 32) | v;
    }
    radix_u64(keys, tmp, cnt);
    uint64_t m = 0;
    for (uint64_t i = 0; i < cnt; ++i)
        if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
    memset(row_ptr, 0, ((uint64_t)n + 1) * sizeof(uint64_t));
    for (uint64_t i = 0; i < m; ++i) {
        row_ptr[(keys[i] >> 32) + 1]++;
        col[i] = (uint32_t)(keys[i] & 0xFFFFFFFFu);
    }
    for (uint32_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    fill_weights(seed, m, wlo, whi, w);
    *m_out = m;
    free(keys); free(tmp); free(perm);
    return 0;
}

/* W x H grid, vertex id y*W + x, out-edges to the (up to) four axis
 * neighbours in increasing id order. col/w need 2*(2WH - W - H) entries. */
int gg_grid(uint32_t W, uint32_t H, uint32_t wlo, uint32_t whi, uint64_t seed,
            uint64_t *row_ptr, uint32_t *col, uint32_t *w) {
    if (W == 0 || H == 0) return -1;
    uint64_t e = 0;
    for (uint32_t y = 0; y < H; ++y)
        for (uint32_t x = 0; x < W; ++x) {
            uint64_t v = (uint64_t)y * W + x;
            row_ptr[v] = e;
            if (y > 0) col[e++] = (uint32_t)(v - W);
            if (x > 0) col[e++] = (uint32_t)(v - 1);
            if (x + 1 < W) col[e++] = (uint32_t)(v + 1);
            if (y + 1 < H) col[e++] = (uint32_t)(v + W);
        }
    row_ptr[(uint64_t)W * H] = e;
    fill_weights(seed, e, wlo, whi, w);
    return 0;
}

/* `count` source vertices drawn uniformly among vertices with out-degree >= 1
 * (with replacement across draws). Returns -1 if no vertex has an out-edge. */
int gg_sources(uint32_t n, const uint64_t *row_ptr, uint32_t count, uint64_t seed, uint32_t *out) {
    uint64_t cand = 0;
    for (uint32_t v = 0; v < n; ++v) cand += (row_ptr[v + 1] > row_ptr[v]);
    if (cand == 0) return -1;
    uint64_t key = stream_key(seed, TAG_SRC);
    for (uint32_t i = 0; i < count; ++i) {
        uint64_t r = below64(sm_at(key, i), cand);
        for (uint32_t v = 0; v < n; ++v)
            if (row_ptr[v + 1] > row_ptr[v]) { if (r == 0) { out[i] = v; break; } --r; }
    }
    return 0;
}

/* Raw counter-stream outputs (for seeded feature / weight tensors elsewhere). */
void gg_u64(uint64_t seed, uint64_t tag, uint64_t start, uint64_t count, uint64_t *out) {
    uint64_t key = stream_key(seed, TAG_U64 + (tag << 8));
    for (uint64_t i = 0; i < count; ++i) out[i] = sm_at(key, start + i);
}

/* Sort helper kept for callers that want canonical (source, target) order. */
void gg_sort_u64(uint64_t *keys, uint64_t cnt) { qsort(keys, cnt, sizeof(uint64_t), cmp_u64); }
