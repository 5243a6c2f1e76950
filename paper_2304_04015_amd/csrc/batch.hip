// Batched single-source queries over several graphs.
//
// Each query's result is exactly the one simrank_single_source_ex returns for
// it alone: results depend only on (graph, query).
#include <algorithm>
#include <vector>

#include "common.hpp"

using namespace srk;

extern "C" int simrank_batch(simrank_graph *const *graphs, int32_t ngraphs,
                             const simrank_query *qs, int32_t nq, double *const *outs,
                             uint32_t *const *counts_opt, simrank_stats *st_opt) {
    clear_error();
    if (ngraphs < 0 || nq < 0) return fail(SIMRANK_EINVAL, "negative count");
    if (nq > 0 && (!graphs || !qs)) return fail(SIMRANK_EINVAL, "NULL argument");
    std::vector<simrank_params> ps(nq);
    std::vector<int> modes(nq);
    int32_t maxR = 1, maxL = 1;
    for (int32_t i = 0; i < nq; ++i) {
        const simrank_query &q = qs[i];
        if (q.graph < 0 || q.graph >= ngraphs || !graphs[q.graph])
            return fail(SIMRANK_EINVAL, "query " + std::to_string(i) + ": bad graph index");
        const simrank_graph *g = graphs[q.graph];
        int rc = query_params(&q, g->n, &ps[i], &modes[i]);
        if (rc) return fail(rc, "query " + std::to_string(i) + ": " + simrank_last_error());
        if (q.s < 0 || q.s >= g->n)
            return fail(SIMRANK_EINVAL, "query " + std::to_string(i) + ": source out of range");
        if (modes[i] == SIMRANK_MODE_STITCHED && (!g->index || g->index->T != ps[i].T))
            return fail(SIMRANK_ESTATE, "query " + std::to_string(i) + ": no matching index");
        maxR = std::max(maxR, ps[i].R);
        maxL = std::max(maxL, ps[i].L);
    }
    if (nq == 0) {
        if (st_opt) *st_opt = simrank_stats{};
        return SIMRANK_OK;
    }
    const int device = graphs[qs[0].graph]->device;
    SRK_HIP(hipSetDevice(device));
    int32_t maxN = 1;
    for (int32_t i = 0; i < nq; ++i) maxN = std::max(maxN, graphs[qs[i].graph]->n);
    Workspace ws;
    double *out_dev = nullptr;
    uint32_t *cnt_dev = nullptr;
    hipStream_t st = nullptr;
    int rc = workspace_init(graphs[qs[0].graph], maxR, maxL, &ws);
    if (!rc) rc = device_alloc((void **)&out_dev, 8 * (size_t)maxN, nullptr);
    if (!rc) rc = device_alloc((void **)&cnt_dev, 4 * (size_t)maxN, nullptr);
    if (!rc) {
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    simrank_stats tot{};
    for (int32_t i = 0; i < nq && !rc; ++i) {
        const simrank_graph *g = graphs[qs[i].graph];
        rc = enqueue_query(g, &qs[i], ps[i], modes[i], &ws, out_dev, cnt_dev, st);
        if (!rc) {
            hipError_t e = hipEventSynchronize(ws.ev1);
            unsigned long long c[8];
            if (e == hipSuccess) e = hipMemcpy(c, ws.counters, sizeof(c), hipMemcpyDeviceToHost);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, ws.ev0, ws.ev1);
            if (e == hipSuccess && outs && outs[i])
                e = hipMemcpy(outs[i], out_dev, 8 * (size_t)g->n, hipMemcpyDeviceToHost);
            if (e == hipSuccess && counts_opt && counts_opt[i])
                e = hipMemcpy(counts_opt[i], cnt_dev, 4 * (size_t)g->n, hipMemcpyDeviceToHost);
            if (e != hipSuccess) {
                rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
                break;
            }
            tot.pairs += (uint64_t)(g->n - 1) * (uint64_t)ps[i].R;
            tot.pairs_walked += c[C_PAIRS];
            tot.moves += c[C_MOVES];
            tot.draws += c[C_DRAWS];
            tot.meets += c[C_MEETS];
            tot.tail_steps += c[C_TAIL];
            tot.source_moves += c[C_SRC_MOVES];
            tot.ms += ms;
        }
    }
    if (st) (void)hipStreamDestroy(st);
    device_free(out_dev);
    device_free(cnt_dev);
    workspace_release(&ws);
    if (!rc && st_opt) *st_opt = tot;
    return rc;
}
