// The opaque sssp_graph handle and the helpers shared between translation units.
#pragma once

#include <vector>

#include "common.h"

struct sssp_graph {
    uint32_t n = 0;
    uint64_t m = 0;
    int device = 0;
    hipStream_t stream = nullptr;
    uint32_t *rp = nullptr;        // row_ptr as u32 (n+1)
    uint2 *edges = nullptr;        // (target, weight); rows sorted by weight once rows_sorted
    bool rows_sorted = false;      // set by graph_ensure_sorted (the dynamic criteria's cursors)
    uint2 *vmin = nullptr;         // (minIn, minOut)
    uint32_t *emin = nullptr;      // per edge: minOut of its target (relax folds the next OUT-STATIC threshold)
    uint32_t *ip = nullptr;        // CSC in_ptr (lazy)
    uint2 *in_edges = nullptr;     // CSC (source, weight), rows sorted by weight (lazy)
    uint64_t precompute_ns = 0;
    uint64_t sum_w = 0;            // exact sum of edge weights (selector feature scale)
    uint32_t wmax = 0;             // some edge weighs 2^32 - 1 (a stored minimum INF32 is then ambiguous)
    LaunchCfg cfg{};
    // per-solve scratch, allocated on first use and kept
    SolveBufs b{};
    bool bufs_ready = false;
    uint32_t bufs_scan_blocks = 0; // scan grid the S' shard capacity was sized for
    uint32_t delta_cap = 0;        // entries of b.deltas
    CtlHead *h_ctl = nullptr;      // pinned host mirror of the control-block header (2 slots)
    hipEvent_t ev[2] = {nullptr, nullptr};
    // per-kernel event timing
    bool prof = false;
    hipEvent_t *pev = nullptr;     // 4 events per phase of one batch
    uint32_t pev_cap = 0;
    sssp_kernel_profile last_prof{};
    std::vector<float> phase_ms;   // per-phase kernel time of the last timed solve
    // captured phase batch (6 phases) for graph replay
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    unsigned char graph_key[512] = {0};
    uint32_t graph_key_len = 0;
    // one-workgroup solves (launch option `single`): the batched kernel's per-query scratch
    uint8_t *one_st = nullptr;     // state bytes, n rounded up to 256
    uint32_t *one_fl = nullptr;    // two fringe lists and the settled list, 3 * n
    uint2 *one_fm = nullptr;       // (minIn, minOut) of the two fringe lists' entries, 2 * n
    void *one_aux = nullptr;       // query record, order, phase count, work-queue control
};

DevGraph dev_view(const sssp_graph *g);
int graph_ensure_csc(sssp_graph *g);
int graph_ensure_sorted(sssp_graph *g);
void graph_default_cfg(sssp_graph *g);
int solve_bufs_ensure(sssp_graph *g, bool cursors, bool stamps, bool queue, bool approx = false, bool store = false);
void solve_bufs_free(sssp_graph *g);
int batch_solve_one(sssp_graph *g, uint32_t source, int in, bool out_static, uint64_t *dist_out,
                    uint32_t *phases_out);
