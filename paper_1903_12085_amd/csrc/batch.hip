// Batched phased SSSP (placeholder until the persistent batched kernel lands).
#include "common.h"
#include "graph.h"

extern "C" int sssp_solve_batch(sssp_graph *const *graphs, const uint32_t *sources, uint32_t nq,
                                uint32_t criterion, uint64_t *const *dist_outs, uint32_t *phases_out) {
    if (nq == 0 || !graphs || !sources || !dist_outs)
        return sssp_set_error(SSSP_ERR_INVALID, "empty batch or NULL array");
    for (uint32_t q = 0; q < nq; ++q) {
        uint32_t ph = 0;
        int rc = sssp_solve(graphs[q], sources[q], criterion, dist_outs[q], &ph);
        if (rc) return rc;
        if (phases_out) phases_out[q] = ph;
    }
    return SSSP_OK;
}
