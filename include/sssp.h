/*
 * sssp.h -- C ABI of the MI355X (gfx950) phased single-source shortest path library.
 *
 * Method: M. Kainer, J. L. Traff, "More Parallelism in Dijkstra's Single-Source
 * Shortest Path Algorithm", arXiv 1903.12085.
 *
 * Problem (Section 2): a directed graph G = (V, E), non-negative edge costs
 * c(u, v), a source s; compute dist(s, v) for every v, infinity if v is not
 * reachable. Costs are uint32 (non-negative by type); distances are uint64,
 * with UINT64_MAX standing for infinity.
 *
 * Method (Section 3): the generic phased algorithm. Vertices are settled (S),
 * queued (F) or unexplored (U). Each phase evaluates a correctness criterion
 * on every queued vertex against the phase-start state, settles every vertex
 * it certifies and relaxes all their out-edges in parallel, until F is empty.
 * A criterion is a bit set; several bits mean their disjunction, which is
 * sound because each disjunct is (Section 3).
 *
 * Conventions for every entry point:
 *   - Graph data is given in CSR form (row_ptr[n+1], col[m], weight[m]) with
 *     row_ptr[0] = 0, row_ptr non-decreasing, row_ptr[n] = m, col[e] < n.
 *     Self-loops and parallel edges are allowed and enter every minimum.
 *   - Output distance arrays are DEVICE pointers with room for n uint64 and
 *     are owned by the caller; the library never frees caller memory.
 *   - Every call is synchronous: when it returns, outputs are complete.
 *     Work runs on the graph's HIP stream (sssp_set_stream).
 *   - Return value: SSSP_OK (0) or a negative sssp_status. On error, output
 *     buffers hold unspecified data; sssp_last_error() describes the failure
 *     (thread-local string, valid until the next call on that thread).
 *   - A graph handle may be used by one host thread at a time.
 *   - Limits: 1 <= n < 2^26, m < 2^32; otherwise SSSP_ERR_UNSUPPORTED.
 */
#ifndef SSSP_H
#define SSSP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sssp_graph sssp_graph;

typedef enum {
    SSSP_OK = 0,
    SSSP_ERR_INVALID = -1,     /* bad argument or malformed CSR */
    SSSP_ERR_OOM = -2,         /* device or host allocation failed */
    SSSP_ERR_DEVICE = -3,      /* a HIP runtime call failed */
    SSSP_ERR_UNSUPPORTED = -4, /* size beyond the documented limits */
    SSSP_ERR_INTERNAL = -5     /* invariant violated (e.g. phase count above n) */
} sssp_status;

/* Criterion bits (Section 3). The phase settles v in F when any set bit holds:
 *   SSSP_DIJK        d[v] = min_{u in F} d[u]
 *   SSSP_IN_STATIC   d[v] - min over all in-edges (w,v) of c(w,v) <= minD      (eq. crit:instatic)
 *   SSSP_OUT_STATIC  d[v] <= min_{u in F} d[u] + min over all out-edges of u   (eq. crit:outstatic)
 *   SSSP_IN_SIMPLE   as IN_STATIC, in-edges from non-settled w only            (eq. crit:insimple)
 *   SSSP_OUT_SIMPLE  as OUT_STATIC, out-edges (u,w) to non-settled w only      (eq. crit:outsimple,
 *                    read with u in F and w in F u U)
 *   SSSP_IN_FULL     IN: in-edges from F, or two-edge paths through U          (eq. crit:in)
 *   SSSP_OUT_WEAK    OUT with the second edge minimised over all of V          (eq. crit:outweak)
 *   SSSP_OUT_FULL    OUT: edges into F, or two-edge paths into U then F u U    (eq. crit:out)
 * minD = min_{u in F} d[u]; all terms use the phase-start snapshot. */
enum {
    SSSP_DIJK = 1u << 0,
    SSSP_IN_STATIC = 1u << 1,
    SSSP_OUT_STATIC = 1u << 2,
    SSSP_IN_SIMPLE = 1u << 3,
    SSSP_OUT_SIMPLE = 1u << 4,
    SSSP_IN_FULL = 1u << 5,
    SSSP_OUT_WEAK = 1u << 6,
    SSSP_OUT_FULL = 1u << 7,
    SSSP_CRIT_ALL = 0xFFu,
    /* approximate criteria (Section 3, closing paragraphs), sssp_solve_approx only */
    SSSP_IN_APPROX = 1u << 8,
    SSSP_OUT_APPROX = 1u << 9
};

/* Per-solve statistics (Section 4 measures phases and the summed fringe sizes). */
typedef struct {
    uint32_t phases;       /* phases (phased solver) or rounds (Delta-stepping) */
    uint32_t buckets;      /* Delta-stepping buckets processed; 0 for the phased solver */
    uint64_t sum_f;        /* sum over phases of |F| at phase start */
    uint64_t n_reach;      /* vertices settled = vertices reachable from the source */
    uint64_t m_reach;      /* out-edges of reachable vertices (the GTEPS numerator) */
    uint64_t relax_edges;  /* edge relaxations attempted towards non-settled targets */
    uint64_t improving;    /* relaxations that lowered a tentative distance */
    uint64_t precompute_ns;/* one-time per-graph preprocessing time, nanoseconds */
} sssp_stats;

/* One record per phase (Section 4 plots vertices settled per phase). */
typedef struct {
    uint64_t min_d;        /* minD at phase start (or the bucket floor for Delta-stepping) */
    uint32_t fringe;       /* |F| at phase start */
    uint32_t settled;      /* |S'| settled in this phase (frontier size for a light round) */
    uint32_t criterion;    /* criterion bits evaluated in this phase (learned solves vary it) */
    uint32_t edges;        /* out-edges expanded in this phase */
} sssp_phase_rec;

/*
 * Create a device graph from CSR arrays (Section 5 uses an adjacency array of
 * out-edges). device_ptrs = 0: row_ptr/col/weight are host pointers;
 * device_ptrs = 1: they are device pointers. The library copies the data into
 * buffers it owns, so the caller may free its arrays after the call. It
 * precomputes the static minima minIn/minOut (equations crit:instatic and
 * crit:outstatic, computed once in O(m), Section 3). Rows keep the input's
 * edge order; the first solve with a SIMPLE or full criterion sorts every row
 * by weight in place, once. hip_stream: a hipStream_t or NULL for the null stream.
 * Errors: SSSP_ERR_INVALID for n = 0, a malformed CSR (checked on the device
 * when device_ptrs = 1) or out == NULL; SSSP_ERR_OOM; SSSP_ERR_UNSUPPORTED.
 */
int sssp_graph_create(uint32_t n, uint64_t m, const uint64_t *row_ptr, const uint32_t *col,
                      const uint32_t *weight, int device_ptrs, void *hip_stream, sssp_graph **out);

/* Release every device buffer the graph owns. NULL is accepted. */
int sssp_graph_destroy(sssp_graph *g);

/* Change the HIP stream used by later calls on g. */
int sssp_set_stream(sssp_graph *g, void *hip_stream);

/* Copy the static minima to caller DEVICE buffers of n uint32 each
 * (UINT32_MAX where a vertex has no in- / out-edge). Either may be NULL. */
int sssp_graph_minima(sssp_graph *g, uint32_t *min_in, uint32_t *min_out);

/*
 * Phased SSSP (Section 3) with the given criterion bits.
 *   dist_out   DEVICE, n uint64: dist(s, v), UINT64_MAX if unreachable.
 *   phases_out HOST, may be NULL: number of phases (phase 1 settles s).
 * Errors: SSSP_ERR_INVALID for source >= n, criterion 0 or unknown bits,
 * dist_out NULL.
 */
int sssp_solve(sssp_graph *g, uint32_t source, uint32_t criterion, uint64_t *dist_out,
               uint32_t *phases_out);

/*
 * sssp_solve with observability.
 *   stats      HOST, may be NULL.
 *   phase_of   DEVICE, n uint32, may be NULL: the 1-based phase in which each
 *              vertex was settled, 0 if never.
 *   trace      HOST, trace_cap records, may be NULL: one record per phase for
 *              the first trace_cap phases.
 */
int sssp_solve_ex(sssp_graph *g, uint32_t source, uint32_t criterion, uint64_t *dist_out,
                  sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap);

/*
 * Delta-stepping (Section 5, the comparison algorithm), run on the same
 * kernels. Bucket b is the window [b*delta, (b+1)*delta) holding the smallest
 * queued distance; light edges (c < delta) are relaxed in synchronous rounds
 * until no vertex inside the window improves, then one round relaxes the
 * heavy edges (c >= delta) of everything the bucket removed.
 *   phases_out HOST, may be NULL: light rounds + heavy rounds.
 * Errors: SSSP_ERR_INVALID for delta = 0, source >= n, dist_out NULL.
 */
int sssp_delta_step(sssp_graph *g, uint32_t source, uint64_t delta, uint64_t *dist_out,
                    uint32_t *phases_out);

/* Delta-stepping with a per-bucket width: bucket b uses deltas[min(b, n_deltas-1)]
 * (HOST array, every entry >= 1). stats/trace as for sssp_solve_ex. */
int sssp_delta_step_ex(sssp_graph *g, uint32_t source, const uint64_t *deltas, uint32_t n_deltas,
                       uint64_t *dist_out, sssp_stats *stats, sssp_phase_rec *trace,
                       uint32_t trace_cap);

/*
 * Batched phased SSSP: nq independent queries (graphs[i], sources[i]) in one
 * persistent launch; each workgroup runs whole queries, largest first, with
 * the phase loop of Section 3 inside the kernel. Graph handles may repeat.
 * Every query uses `criterion`, a disjunction of SSSP_DIJK, SSSP_IN_STATIC
 * and SSSP_OUT_STATIC (the static criteria, eq. crit:instatic / crit:outstatic).
 *   dist_outs  HOST array of nq DEVICE pointers, each with room for
 *              graphs[i]->n uint64; the buffers must not overlap.
 *   phases_out HOST, nq entries, may be NULL.
 * Runs on graphs[0]'s stream. The call allocates about 29 bytes of device
 * scratch per vertex of each query (a state byte, two fringe lists holding each
 * entry's vertex and static minima, a settled list) and frees it before
 * returning. Errors: SSSP_ERR_INVALID for nq = 0, a NULL pointer, a bad source
 * or criterion; SSSP_ERR_UNSUPPORTED for the dynamic criteria; SSSP_ERR_OOM
 * when the scratch does not fit.
 */
int sssp_solve_batch(sssp_graph *const *graphs, const uint32_t *sources, uint32_t nq,
                     uint32_t criterion, uint64_t *const *dist_outs, uint32_t *phases_out);

/* Launch shape of the batched solver. A zero field means the default.
 * Queries on graphs with at least team_edges edges each run on a team of
 * team_size workgroups that share its fringe and settled lists and meet at a
 * barrier twice per phase, while the other resident workgroups take the other
 * queries one per workgroup, all in one cooperative launch (so every member is
 * resident; a member that waits longer than a bounded spin sets the error and
 * the call returns SSSP_ERR_INTERNAL). */
typedef struct {
    uint32_t block;      /* threads per workgroup: 256, 512 or 1024 (default 512) */
    uint32_t split;      /* rows with more out-edges than this are expanded by the whole
                            workgroup instead of one lane (default 64) */
    uint32_t blocks;     /* workgroups of the persistent launch (default 4 per compute unit) */
    uint32_t team_edges; /* edge count from which a query gets a team (default 2^20;
                            UINT32_MAX: no teams) */
    uint32_t team_size;  /* workgroups per team: 2 .. 64 (default: the largest power of two
                            <= 16 that keeps the teams within half of the resident
                            workgroups; more large queries than teams are taken in turn) */
} sssp_batch_cfg;

/* sssp_solve_batch with an explicit launch shape (cfg may be NULL: defaults). */
int sssp_solve_batch_ex(sssp_graph *const *graphs, const uint32_t *sources, uint32_t nq,
                        uint32_t criterion, uint64_t *const *dist_outs, uint32_t *phases_out,
                        const sssp_batch_cfg *cfg);

/* Process-wide default shape used by sssp_solve_batch (set by the autotuner). */
int sssp_batch_set_config(const sssp_batch_cfg *cfg);
int sssp_batch_get_config(sssp_batch_cfg *cfg);



/* Per-kernel device time of the last solve on g, measured with HIP events on
 * the graph's stream around every kernel launch (observability; enabling it
 * adds one host synchronisation per batch of queued phases). */
typedef struct {
    uint32_t phases;       /* non-empty phases (or rounds) that were timed; with keyed queue
                              arrays also the rebuild launches */
    float term_ms;         /* total time of the dynamic-term pass kernels */
    float identify_ms;     /* total time of the identify kernels */
    float relax_ms;        /* total time of the relax kernels (learned mode: plus the selector) */
} sssp_kernel_profile;

/* Phased solve with the clairvoyant ORACLE criterion of Section 3: a queued
 * vertex is settled as soon as d[v] = dist(source, v). It needs the answer in
 * advance, so it measures the fewest phases the generic algorithm can take on
 * this graph (each v is settled in phase 1 + the fewest edges over its
 * minimum-cost paths), the bound every sound criterion is compared with.
 *   dist_ref  device pointer, n words: dist(source, .) of this graph (UINT64_MAX
 *             for unreachable vertices), e.g. from an earlier sssp_solve; read only.
 *   dist_out, stats, phase_of  as in sssp_solve_ex (phase_of may be NULL).
 * Returns SSSP_ERR_INVALID if dist_ref is NULL or turns out not to be
 * dist(source, .): a phase that certifies nothing while F is not empty stops
 * the solve. */
int sssp_solve_oracle(sssp_graph *g, uint32_t source, const uint64_t *dist_ref, uint64_t *dist_out,
                      sssp_stats *stats, uint32_t *phase_of);

/*
 * Phased SSSP with the approximate criteria of Section 3 (closing paragraphs).
 * With each vertex v one IN value is kept, the minimum over in-edges (w,v) of
 * c(w,v) for w in F and c(w,v) + min over all in-edges of w for w in U (the
 * two IN minima of the paper), and one OUTWEAK value, the same over out-edges
 * (v,w) with the minimum out-edge of w. They are kept conservatively, never
 * above their exact value: a neighbour moving U -> F lowers them at once; a
 * neighbour moving F -> S, which may raise the exact value, is only counted
 * (per edge), and a queued vertex evaluated with at least k counted changes
 * recomputes its values from the phase-start state (k = 0: never, the minima
 * computed once and only lowered afterwards). Criteria: SSSP_IN_APPROX holds if
 * d[v] - in[v] <= minD, SSSP_OUT_APPROX if d[v] <= min_{u in F} d[u] + out[u];
 * criterion is a non-empty disjunction of SSSP_DIJK, SSSP_IN_APPROX and
 * SSSP_OUT_APPROX (the paper combines the approximate criteria with DIJK;
 * with non-negative weights DIJK implies both). k = 1 gives the exact IN
 * (eq. crit:in) and OUTWEAK (eq. crit:outweak) criteria. Arguments otherwise as
 * sssp_solve_ex; SSSP_ERR_INVALID for other criterion bits.
 */
int sssp_solve_approx(sssp_graph *g, uint32_t source, uint32_t criterion, uint32_t k, uint64_t *dist_out,
                      sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap);

/* Turn per-kernel event timing on (enable != 0) or off for later solves on g. */
int sssp_profile_enable(sssp_graph *g, int enable);

/* Read the per-kernel times of the last solve run with timing on. */
int sssp_profile_get(const sssp_graph *g, sssp_kernel_profile *out);

/* Per-phase kernel time (term pass + identify + relax, milliseconds, launch
 * order; a keyed rebuild launch, see sssp_launch_cfg.queue, has an entry of
 * its own) of the last phased solve run with timing on: *count receives the
 * number of entries, and the first min(*count, cap) times are written to ms
 * (host memory, caller-owned). Returns SSSP_ERR_INVALID for a NULL g or count,
 * or a NULL ms with cap > 0. */
int sssp_profile_phases(const sssp_graph *g, float *ms, uint32_t cap, uint32_t *count);

/* Launch shape of the phase kernels of a graph (tuning; results never depend
 * on it). Defaults are chosen from n, m and the device's compute-unit count. */
typedef struct {
    uint32_t scan_blocks;   /* blocks of the per-vertex scan kernels (identify, term pass) */
    uint32_t relax_blocks;  /* blocks of the relax kernel */
    uint32_t chunk;         /* edges per relax chunk: 256, 512 or 1024 */
    uint32_t use_graph;     /* 1: replay phases from a captured HIP graph; 0: plain launches */
    uint32_t queue;         /* criteria made of DIJK, IN_STATIC and OUT_STATIC only: 1 keeps the
                               queued vertices with their distance and static minima in per-block
                               queue arrays, so identify reads F itself instead of scanning the
                               distance and minima arrays of all vertices (phases with 3/8 or more
                               of the vertices queued still use that dense scan); 0: the dense
                               scan always; 2: keyed queue arrays (the keyed priority queues of
                               Section 5, partitioned by the IN-STATIC key d - minIn): a block's
                               entries hold only the queued vertices whose key is at most a split
                               kept above the phase's threshold (OUT-STATIC's T, else minD), which
                               contain every vertex the phase certifies and the vertices attaining
                               the next thresholds; the others are not read until the threshold
                               passes the split, when one extra launch rebuilds the entries (it
                               settles nothing and is not counted as a phase). sssp_solve and
                               sssp_solve_ex only; switched and committed solves use 1. Applies
                               when each scan block owns at most 16384 vertices (n <= 4096 *
                               scan_blocks * 4), else the dense scan runs. Ignored by every other
                               criterion and solver. Values above 2: SSSP_ERR_INVALID. */
    uint32_t single;        /* 1: sssp_solve with a criterion made of DIJK, IN_STATIC and OUT_STATIC
                               runs the whole solve in one workgroup of the batched kernel
                               (sssp_solve_batch with one query): no kernel launch per phase, for
                               graphs whose phases settle few vertices each (grids). Same
                               distances and phase count; no per-kernel timing is recorded
                               (sssp_profile_get keeps the previous figures). sssp_solve_ex and
                               every other solver ignore it. */
} sssp_launch_cfg;

/* Read the launch shape used by later solves on g. */
int sssp_get_launch(const sssp_graph *g, sssp_launch_cfg *out);

/* Set the launch shape for later solves on g. Errors: SSSP_ERR_INVALID for a
 * zero block count or an unsupported chunk size. */
int sssp_set_launch(sssp_graph *g, const sssp_launch_cfg *cfg);

/*
 * Autotuner for the plain solver: times sssp_solve(g, source, criterion) with
 * HIP events for a set of launch shapes (scan grid, relax grid, chunk size,
 * graph replay, the dense scan or queue arrays; for static criteria also keyed
 * queue arrays and the one-workgroup option), keeps the fastest on g and
 * returns it in best (may be NULL)
 * with its time in best_ms (may be NULL). Distances are never affected.
 */
int sssp_autotune(sssp_graph *g, uint32_t source, uint32_t criterion, sssp_launch_cfg *best,
                  float *best_ms);

/*
 * Autotuner for the batched solver: times the batch for workgroup sizes,
 * degree-split thresholds, workgroup counts and team thresholds (no teams,
 * 2^20 or 2^22 edges; automatic team size or teams of two), makes the fastest
 * the process-wide default and returns it. dist_outs are overwritten with the
 * batch's distances.
 */
int sssp_autotune_batch(sssp_graph *const *graphs, const uint32_t *sources, uint32_t nq,
                        uint32_t criterion, uint64_t *const *dist_outs, sssp_batch_cfg *best,
                        float *best_ms);

/*
 * Learned per-phase selector: an MLP 12 -> 64 (ReLU) -> 64 (ReLU) -> 6 in FP32
 * that looks at the phase-start state and picks, per phase, which criterion
 * the phased solver evaluates (outputs 0..2: IN-STATIC|OUT-STATIC,
 * IN-SIMPLE|OUT-SIMPLE, IN-SIMPLE|OUT-STATIC) or, per bucket, Delta-stepping's width
 * (outputs 3..5: 2^12, 2^14, 2^16). Every criterion is sound (Section 3), so a
 * choice changes work and phase count, never a distance.
 * Features (12 floats, each a ratio of exact integers computed in double and
 * rounded once): F/n, S/n, Sp/Fp, min(F/2^22,4)/4, min((t-a)/Wm,64)/64,
 * min(max((SD/F-a)/Wm,0),256)/256, min((DG/F)/(m/n),8)/8, Ip/Fp, Op/Fp,
 * min(F/Fp,4)/4, (n-R)/n, min(a/Wm,4096)/4096 -- F, S, R: queued, settled,
 * reached; a: minD; t: OUT-STATIC threshold; SD, DG: sums over F of d and of
 * out-degree; Fp, Sp, Ip, Op: previous |F|, |S'|, and previous queued vertices
 * passing IN-STATIC / OUT-STATIC; Wm: mean weight. For
 * Delta-stepping (at bucket starts) the 5th to 10th features are 0.
 * Weights: 5382 floats, W1[64][12] b1[64] W2[64][64] b2[64] W3[6][64] b3[6].
 */
typedef struct sssp_selector sssp_selector;

#define SSSP_SELECTOR_PARAMS 5382

/* Create a selector with the given HOST weights (NULL: all zeros). */
int sssp_selector_create(const float *weights, sssp_selector **out);
int sssp_selector_destroy(sssp_selector *s);
int sssp_selector_get_weights(const sssp_selector *s, float *host_out);
/* Replace the weights (HOST array) and reset the optimiser state. */
int sssp_selector_set_weights(sssp_selector *s, const float *host_in);

/* Logits for n feature rows (HOST x[n][12] -> HOST logits[n][6]). */
int sssp_selector_forward(const sssp_selector *s, const float *x, uint32_t n, float *logits_out);

/* Mean softmax cross-entropy of n rows with labels y (0..5) and its gradient
 * with respect to the weights (HOST, 5382 floats, same layout). */
int sssp_selector_grad(const sssp_selector *s, const float *x, const int32_t *y, uint32_t n, float *loss_out,
                       float *grad_out);

/* Adam training on the GPU: `epochs` passes over n rows in shuffled batches
 * of `batch` (shuffle seeded by `seed`); final_loss: mean loss of the last
 * batch (may be NULL). */
int sssp_selector_train(sssp_selector *s, const float *x, const int32_t *y, uint32_t n, uint32_t epochs,
                        uint32_t batch, float lr, uint64_t seed, float *final_loss);

/* Phased SSSP whose criterion is chosen per phase by the selector (trace
 * records carry each phase's criterion bits). Arguments as sssp_solve_ex. */
int sssp_solve_learned(sssp_graph *g, uint32_t source, const sssp_selector *sel, uint64_t *dist_out,
                       sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap);

/*
 * Learned phased SSSP with the choice committed after a prefix: the selector
 * chooses the criteria of phases 0 .. commit_phase - 1 one by one, exactly as
 * sssp_solve_learned does, and every later phase uses the criterion it chose
 * for phase commit_phase, run by that criterion's plain kernels (no per-phase
 * features or network after the prefix). This trades the selector's per-phase
 * cost against adapting late in the solve, the accuracy-versus-overhead
 * question that the paper's concluding remarks (Section 7) leave open. commit_phase >= 1
 * (SSSP_ERR_INVALID otherwise). The host reads the control block once, after
 * the prefix. Distances are those of every other solver; other arguments as
 * sssp_solve_ex.
 */
int sssp_solve_learned_commit(sssp_graph *g, uint32_t source, const sssp_selector *sel, uint32_t commit_phase,
                              uint64_t *dist_out, sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace,
                              uint32_t trace_cap);

/*
 * Switched phased solve: phases evaluate crit_first, a criterion made of DIJK,
 * IN_STATIC and OUT_STATIC (the cheap static tests of Section 3), until |F| has
 * fallen to drop_num/drop_den of its peak, then crit_then (any criterion, e.g.
 * IN_SIMPLE | OUT_STATIC) for every later phase. The stronger criteria of
 * Section 3 certify most of the remaining queue in a few phases once most
 * vertices are settled, where a static criterion needs many short phases. Every
 * criterion is sound, so distances equal every other solver's. The switch is
 * taken at a batch boundary: phases run in batches of 16, the host checks |F|
 * at the start of the last phase of each batch one batch behind, and the first
 * check at or below the fraction of the largest |F| seen at an earlier check
 * (and below it) makes the phase two batch boundaries later the first with
 * crit_then; the phase is therefore independent of timing. Trace records carry
 * each phase's criterion. Errors: SSSP_ERR_INVALID for a crit_first that is not
 * static, an empty or unknown crit_then, drop_num = 0 or drop_num > drop_den,
 * or a crit_then with OUT_STATIC after a crit_first without it (no threshold
 * is carried over). No per-kernel timing is recorded. Other arguments as
 * sssp_solve_ex.
 */
int sssp_solve_switch(sssp_graph *g, uint32_t source, uint32_t crit_first, uint32_t crit_then, uint32_t drop_num,
                      uint32_t drop_den, uint64_t *dist_out, sssp_stats *stats, uint32_t *phase_of,
                      sssp_phase_rec *trace, uint32_t trace_cap);

/*
 * sssp_solve_learned_commit followed, when the committed choice is the static
 * criterion (IN_STATIC | OUT_STATIC), by the switch of sssp_solve_switch: from
 * phase commit_phase on, the static criterion runs until |F| has fallen to
 * drop_num/drop_den of its peak (batches of 16 counted from commit_phase), then
 * crit_then. A committed choice of a stronger criterion runs to the end as in
 * sssp_solve_learned_commit. Errors as for both; other arguments as
 * sssp_solve_ex.
 */
int sssp_solve_learned_switch(sssp_graph *g, uint32_t source, const sssp_selector *sel, uint32_t commit_phase,
                              uint32_t crit_then, uint32_t drop_num, uint32_t drop_den, uint64_t *dist_out,
                              sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap);

/*
 * Fixed two-stage schedule: phases 0 .. switch_phase - 1 evaluate crit_first, a
 * criterion made of DIJK, IN_STATIC and OUT_STATIC, every later phase crit_then
 * (any criterion; OUT_STATIC in crit_then needs OUT_STATIC in crit_first).
 * switch_phase = 0 runs crit_then throughout. Every criterion is sound
 * (Section 3), so distances equal every other solver's. Errors and other
 * arguments as sssp_solve_switch.
 */
int sssp_solve_schedule(sssp_graph *g, uint32_t source, uint32_t crit_first, uint32_t crit_then, uint32_t switch_phase,
                        uint64_t *dist_out, sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace,
                        uint32_t trace_cap);

/*
 * Learned checkpoint solve: IN_STATIC | OUT_STATIC on the plain kernels, and
 * after every 16th phase (the last phase k of each batch of 16) one wavefront
 * runs the selector on phase k's snapshot and outcome with the checkpoint
 * features (delta_mode 2: F, S, minD and the OUT-STATIC threshold of phase k,
 * |S'| of phase k, |F| at the previous checkpoint, the graph's size and mean
 * degree as x5 = floor(log2 n)/32 and x6 = min(m/n, 64)/64; x7 = x8 = 0). Its output 0
 * keeps the static criterion; the first checkpoint j that chooses 1
 * (IN_SIMPLE | OUT_SIMPLE) or 2 (IN_SIMPLE | OUT_STATIC) switches every phase
 * from 16 (j + 2) on to that criterion (the host reads each checkpoint one
 * batch behind, so the switch phase does not depend on timing). The network
 * alone decides; its cost is one small launch per 16 phases. Distances equal
 * every other solver's.
 *   features_out HOST, may be NULL: row j (12 floats) = checkpoint j's features,
 *                for j < min(checkpoints, trace_cap); needs trace_cap > 0.
 * Other arguments as sssp_solve_ex; trace records carry each phase's criterion.
 */
int sssp_solve_learned_checkpoint(sssp_graph *g, uint32_t source, const sssp_selector *sel, uint64_t *dist_out,
                                  sssp_stats *stats, uint32_t *phase_of, sssp_phase_rec *trace, uint32_t trace_cap,
                                  float *features_out);

/* Delta-stepping whose bucket width is chosen per bucket by the selector. */
int sssp_delta_step_learned(sssp_graph *g, uint32_t source, const sssp_selector *sel, uint64_t *dist_out,
                            sssp_stats *stats, sssp_phase_rec *trace, uint32_t trace_cap);

/*
 * Training traces from the solver itself. delta_mode = 0: a learned phased
 * solve that, on every phase's snapshot, also evaluates all three criteria
 * and records how many queued vertices each certifies (counts_out[k][3],
 * HOST) next to the phase's features (features_out[k][12], HOST); the phase
 * still settles what the selector's choice certifies. delta_mode = 1: a
 * learned Delta-stepping solve recording the features of every bucket start
 * (counts_out unused). trace_cap records at most; trace as for sssp_solve_ex.
 */
int sssp_trace_learned(sssp_graph *g, uint32_t source, const sssp_selector *sel, int delta_mode,
                       uint64_t *dist_out, sssp_stats *stats, uint32_t trace_cap, sssp_phase_rec *trace,
                       float *features_out, uint32_t *counts_out);

/*
 * Measurement helper: throughput of the returning 64-bit atomicMin that relax
 * uses to lower distances, the second ceiling of the phase loop beside HBM
 * bandwidth. blocks x 256 threads each issue iters atomics on slots of buf
 * drawn from a per-thread pseudo-random sequence (slots = 1: one contended
 * address). buf: DEVICE, slots uint64 entries, caller-owned, overwritten with
 * smaller values. slots a power of two, blocks in [1, 2^20], iters in
 * [1, 2^16], else SSSP_ERR_INVALID. hip_stream: a hipStream_t or NULL.
 * *ms_out (HOST): median of three timed launches after one untimed one.
 */
int sssp_measure_atomic_min(uint64_t *buf, uint64_t slots, uint32_t blocks, uint32_t iters, void *hip_stream,
                            float *ms_out);

/*
 * sssp_solve for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same phased solve with a static criterion (a disjunction of SSSP_DIJK,
 * SSSP_IN_STATIC and SSSP_OUT_STATIC), the same kernels (dense-scan identify
 * and relax) and the same distances and phase count, with every per-solve
 * scratch buffer (control block, state bytes, settled-vertex lists) carved
 * from one device array of 64 MiB that the library holds on each device it
 * runs on until the process ends. The call makes no device or pinned host
 * allocation; the graph handle must already exist (sssp_graph_create
 * allocates) and the caller owns dist_out.
 *   dist_out   DEVICE, n uint64: dist(s, v), UINT64_MAX if unreachable.
 *   phases_out HOST, may be NULL: number of phases.
 * Scratch needed: about 17 bytes per vertex plus 2 bytes per edge (the exact
 * figure depends on the graph's scan grid); a graph needing more than the
 * array holds is rejected with SSSP_ERR_UNSUPPORTED before any device work.
 * All calls on one device share its array and each call overwrites it, so
 * calls on one device are serialised by a per-device lock inside the library;
 * without it, overlapping calls would race. Errors: SSSP_ERR_INVALID for a
 * NULL graph or dist_out, source >= n, an empty or unknown criterion;
 * SSSP_ERR_UNSUPPORTED for a dynamic criterion or an oversized graph.
 */
int sssp_solve_noalloc(sssp_graph *g, uint32_t source, uint32_t criterion, uint64_t *dist_out,
                       uint32_t *phases_out);

/* Human-readable description of the last error on the calling thread. */
const char *sssp_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SSSP_H */
