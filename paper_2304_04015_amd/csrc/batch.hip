// Batched single-source queries over several graphs, and the unit-size tuner.
//
// A plan holds the device buffers of a set of queries (carved from one
// allocation) and a hipGraph of the whole launch sequence: init, source walks
// of every query, compaction, work-unit offsets, one persistent meet launch
// whose work units span all queries (per kind: plain, stitched, stratified),
// estimate.
// Queries on graphs of very different sizes share the launch and its tail.
// Queries of one kind on one graph with the same seed and walk parameters form
// groups that walk each pair (v, j) once for all members (group.hip).
// Each query's result is exactly the one a lone simrank_single_source_ex call
// returns: results depend only on (graph, query).
#include <algorithm>
#include <cstring>
#include <map>
#include <tuple>
#include <vector>

#include "common.hpp"

namespace srk {
namespace {

constexpr size_t ARENA_ALIGN = 256;

size_t align_up(size_t x) { return (x + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1); }

// A group's walks (GroupDesc::wk) for queries of a mode.
int32_t walk_kind(int mode) {
    return mode == SIMRANK_MODE_STITCHED ? 1 : mode == SIMRANK_MODE_STRATIFIED ? 2 : 0;
}

// Groups of queries of one kind that share (graph, seed, continue threshold,
// cap; stratified: z, N and phi): each such set of two or more queries is
// split into ceil(size / GROUP_MAX) groups of nearly equal size, in query
// order.
std::vector<std::vector<int32_t>> form_groups(simrank_graph *const *graphs, const simrank_query *qs,
                                              int32_t nq, const std::vector<simrank_params> &ps,
                                              const std::vector<int> &modes) {
    using Key = std::tuple<const Graph *, int, uint64_t, uint32_t, int32_t, int32_t, uint64_t>;
    std::map<Key, std::vector<int32_t>> by;
    for (int32_t i = 0; i < nq; ++i) {
        const Graph *g = graphs[qs[i].graph];
        uint64_t zbits = 0;
        if (modes[i] == SIMRANK_MODE_STRATIFIED) {
            StratParams sp;
            if (strat_params(&qs[i], g->n, &sp, nullptr)) continue;
            std::memcpy(&zbits, &sp.z, sizeof(zbits));
        }
        by[Key(g, modes[i], qs[i].seed, ps[i].T, ps[i].L, ps[i].R * (modes[i] == SIMRANK_MODE_STRATIFIED),
               zbits)]
            .push_back(i);
    }
    std::vector<std::vector<int32_t>> out;
    for (auto &kv : by) {
        const std::vector<int32_t> &v = kv.second;
        const int32_t sz = (int32_t)v.size();
        if (sz < 2) continue;
        const int32_t ngr = (sz + GROUP_MAX - 1) / GROUP_MAX;
        int32_t at = 0;
        for (int32_t k = 0; k < ngr; ++k) {
            const int32_t take = sz / ngr + (k < sz % ngr ? 1 : 0);
            out.emplace_back(v.begin() + at, v.begin() + at + take);
            at += take;
        }
    }
    return out;
}

}  // namespace
}  // namespace srk

using namespace srk;

struct simrank_batch_plan {
    int device = 0;
    int32_t nq = 0;
    std::vector<QueryDesc> desc;       // host copies (buffer addresses)
    std::vector<GroupDesc> gdesc;
    std::vector<simrank_params> params;
    std::vector<const Graph *> graphs;
    std::vector<uint64_t> index_gen;   // per stitched query: its graph's index generation
    char *arena = nullptr;
    QueryDesc *desc_dev = nullptr;
    uint32_t *units = nullptr;
    GroupDesc *gdesc_dev = nullptr;
    uint32_t *gunits = nullptr;
    unsigned long long *counters = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipStream_t last_stream = nullptr;
    bool ran = false;
    int64_t bytes = 0;
};

static void plan_release(simrank_batch_plan *p) {
    if (!p) return;
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    device_free(p->arena);
    device_free(p->desc_dev);
    device_free(p->units);
    device_free(p->gdesc_dev);
    device_free(p->gunits);
    device_free(p->counters);
    if (p->ev0) (void)hipEventDestroy(p->ev0);
    if (p->ev1) (void)hipEventDestroy(p->ev1);
    delete p;
}

static int check_queries(simrank_graph *const *graphs, int32_t ngraphs, const simrank_query *qs,
                         int32_t nq, std::vector<simrank_params> &ps, std::vector<int> &modes) {
    if (ngraphs < 0 || nq < 0) return fail(SIMRANK_EINVAL, "negative count");
    if (nq > 0 && (!graphs || !qs)) return fail(SIMRANK_EINVAL, "NULL argument");
    ps.resize(nq);
    modes.resize(nq);
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
        if (g->device != graphs[qs[0].graph]->device)
            return fail(SIMRANK_EINVAL, "all graphs of a batch must live on one device");
        const int64_t ub = (int64_t)max_tiles_for(ps[i].R, ps[i].L) *
                           ((g->n_active + default_unit_nodes(g) - 1) / default_unit_nodes(g));
        if (ub >= (int64_t)0x7fffffff)
            return fail(SIMRANK_EINVAL, "query " + std::to_string(i) + ": too many work units");
    }
    return SIMRANK_OK;
}

extern "C" int simrank_batch_plan_create_ex(simrank_graph *const *graphs, int32_t ngraphs,
                                            const simrank_query *qs, int32_t nq, uint32_t flags,
                                            simrank_batch_plan **plan_out, int32_t *n_groups_out) {
    clear_error();
    if (!plan_out) return fail(SIMRANK_EINVAL, "plan is NULL");
    *plan_out = nullptr;
    if (n_groups_out) *n_groups_out = 0;
    if (nq < 1) return fail(SIMRANK_EINVAL, "a plan needs at least one query");
    if (flags & ~SIMRANK_PLAN_GROUPS) return fail(SIMRANK_EINVAL, "unknown plan flags");
    std::vector<simrank_params> ps;
    std::vector<int> modes;
    int rc = check_queries(graphs, ngraphs, qs, nq, ps, modes);
    if (rc) return rc;
    std::vector<std::vector<int32_t>> groups;
    if (flags & SIMRANK_PLAN_GROUPS) groups = form_groups(graphs, qs, nq, ps, modes);
    // a group's work units are counted in 32 bits, as are a kind's
    std::vector<int32_t> group_of(nq, -1);
    std::vector<int64_t> g_Rmax, g_RL;
    {
        std::vector<std::vector<int32_t>> kept;
        int64_t units = 0;
        for (auto &m : groups) {
            int64_t Rmax = 0, RL = 0;
            for (int32_t i : m) {
                Rmax = std::max<int64_t>(Rmax, ps[i].R);
                RL += (int64_t)ps[i].R * ps[i].L;
            }
            const Graph *g = graphs[qs[m[0]].graph];
            const int64_t vb = group_unit_nodes(g->n_active, (int32_t)m.size(),
                                                walk_kind(modes[m[0]]));   // as describe_group sets it
            const int64_t ub = (int64_t)group_max_tiles(Rmax, RL, ps[m[0]].L, (int32_t)m.size(),
                                                        walk_kind(modes[m[0]])) *
                               ((g->n_active + vb - 1) / vb);
            // packed positions are addressed in 32 bits
            if (group_pos_words(Rmax, RL, ps[m[0]].L) >= (int64_t)0xffff0000)
                continue;                                       // these queries run alone
            if (units + ub >= (int64_t)0x7fffffff) continue;
            units += ub;
            for (int32_t i : m) group_of[i] = (int32_t)kept.size();
            kept.push_back(m);
            g_Rmax.push_back(Rmax);
            g_RL.push_back(RL);
        }
        groups.swap(kept);
    }
    const int32_t ngr = (int32_t)groups.size();
    // Each kind's meet launch numbers the work units of all its queries in 32
    // bits (unit offsets and the persistent cursor, which the grid's blocks
    // advance past the end once each): refuse a plan whose units could wrap.
    {
        int64_t kind_units[N_KINDS] = {0, 0, 0};
        for (int32_t i = 0; i < nq; ++i) {
            if (group_of[i] >= 0) continue;
            const Graph *g = graphs[qs[i].graph];
            const int64_t vb = default_unit_nodes(g);
            const int kind = modes[i] == SIMRANK_MODE_STITCHED ? K_STITCHED
                             : modes[i] == SIMRANK_MODE_STRATIFIED ? K_STRAT : K_PLAIN;
            kind_units[kind] += (int64_t)max_tiles_for(ps[i].R, ps[i].L) * ((g->n_active + vb - 1) / vb);
        }
        for (int k = 0; k < N_KINDS; ++k)
            if (kind_units[k] >= (int64_t)0xffffffffu - (1 << 20))
                return fail(SIMRANK_EINVAL, "the batch's queries of one kind have " +
                                                std::to_string(kind_units[k]) +
                                                " work units, beyond 2^32: split the batch");
    }
    simrank_batch_plan *p = new simrank_batch_plan();
    p->device = graphs[qs[0].graph]->device;
    p->nq = nq;
    p->params = ps;
    auto bail = [&](int code) {
        plan_release(p);
        return code;
    };
    hipError_t e = hipSetDevice(p->device);
    if (e != hipSuccess) return bail(fail(SIMRANK_EDEVICE, hipGetErrorString(e)));
    size_t total = 0;
    for (int32_t i = 0; i < nq; ++i) total += request_bytes(ps[i], modes[i], graphs[qs[i].graph]->n);
    for (int32_t k = 0; k < ngr; ++k) {
        GroupDesc gd{};
        gd.Rmax = (int32_t)g_Rmax[k];
        gd.L = ps[groups[k][0]].L;
        gd.G = (int32_t)groups[k].size();
        gd.gw = (gd.G + 3) / 4;
        gd.wk = walk_kind(modes[groups[k][0]]);
        total += group_buffers(&gd, g_RL[k], nullptr);
    }
    size_t free_b = 0, tot_b = 0;
    if (hipMemGetInfo(&free_b, &tot_b) == hipSuccess && total > free_b)
        return bail(fail(SIMRANK_ENOMEM, "batch needs " + std::to_string(total) +
                                             " device bytes, " + std::to_string(free_b) + " free"));
    if ((rc = device_alloc((void **)&p->arena, total, &p->bytes))) return bail(rc);
    if ((rc = device_alloc((void **)&p->desc_dev, sizeof(QueryDesc) * nq, &p->bytes))) return bail(rc);
    if ((rc = device_alloc((void **)&p->units, 4 * units_words(nq), &p->bytes)))
        return bail(rc);
    if ((rc = device_alloc((void **)&p->counters, 8 * 8, &p->bytes))) return bail(rc);
    if (ngr > 0) {
        if ((rc = device_alloc((void **)&p->gdesc_dev, sizeof(GroupDesc) * ngr, &p->bytes)))
            return bail(rc);
        if ((rc = device_alloc((void **)&p->gunits, 4 * group_units_words(ngr), &p->bytes)))
            return bail(rc);
    }
    QuerySet set;
    set.nq = nq;
    char *cur = p->arena;
    auto take = [&](size_t b) {
        char *r = cur;
        cur += align_up(b);
        return r;
    };
    p->desc.resize(nq);
    p->graphs.resize(nq);
    p->index_gen.assign(nq, ~0ull);
    for (int32_t i = 0; i < nq; ++i) {
        const simrank_graph *g = graphs[qs[i].graph];
        const simrank_params &pp = ps[i];
        QueryDesc &d = p->desc[i];
        describe_query(g, &qs[i], pp, modes[i], default_unit_nodes(g), &d);
        carve_request(pp, modes[i], g->n, take(request_bytes(pp, modes[i], g->n)), &d);
        if (modes[i] == SIMRANK_MODE_STRATIFIED) {
            StratParams sp;
            StratTab tab{};
            if ((rc = strat_params(&qs[i], g->n, &sp, &tab))) return bail(rc);
            d.z = sp.z;
            d.sa = sp.sa;
            d.sb = sp.sb;
            e = hipMemcpy((void *)d.tab, &tab, sizeof(StratTab), hipMemcpyHostToDevice);
            if (e != hipSuccess) return bail(fail(SIMRANK_EDEVICE, hipGetErrorString(e)));
        }
        p->graphs[i] = g;
        if (modes[i] == SIMRANK_MODE_STITCHED) p->index_gen[i] = g->index_gen;
        set.max_R = std::max(set.max_R, pp.R);
        set.max_n = std::max(set.max_n, g->n);
        if (group_of[i] >= 0) {
            d.kind = d.kind == K_STITCHED ? K_GROUPED_STITCHED   // walked with its group
                     : d.kind == K_STRAT  ? K_GROUPED_STRAT : K_GROUPED;
        } else {
            const int64_t ub = (int64_t)max_tiles_for(pp.R, pp.L) * d.n_chunks;
            set.units_bound[d.kind] += ub;
        }
    }
    GroupSet gset;
    p->gdesc.resize(ngr);
    for (int32_t k = 0; k < ngr; ++k) {
        const std::vector<int32_t> &m = groups[k];
        std::vector<const QueryDesc *> mem;
        for (int32_t i : m) mem.push_back(&p->desc[i]);
        GroupDesc &gd = p->gdesc[k];
        describe_group(mem.data(), (int32_t)m.size(), &gd);
        const int32_t mt = group_max_tiles(gd.Rmax, g_RL[k], gd.L, gd.G, gd.wk);
        (void)take(group_buffers(&gd, g_RL[k], cur));   // carved at cur, which it advances
        gset.units_bound[group_list(gd.G, gd.wk)] += (int64_t)mt * gd.n_chunks;
    }
    if (ngr > 0) {
        e = hipMemcpy(p->gdesc_dev, p->gdesc.data(), sizeof(GroupDesc) * ngr, hipMemcpyHostToDevice);
        if (e != hipSuccess) return bail(fail(SIMRANK_EDEVICE, hipGetErrorString(e)));
        gset.desc = p->gdesc_dev;
        gset.ng = ngr;
        gset.units = p->gunits;
        set.groups = &gset;
    }
    e = hipMemcpy(p->desc_dev, p->desc.data(), sizeof(QueryDesc) * nq, hipMemcpyHostToDevice);
    if (e != hipSuccess) return bail(fail(SIMRANK_EDEVICE, hipGetErrorString(e)));
    set.desc = p->desc_dev;
    set.units = p->units;
    set.counters = p->counters;
    // capture the launch sequence into a graph
    hipStream_t cs = nullptr;
    e = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
    if (e != hipSuccess) return bail(fail(SIMRANK_EDEVICE, hipGetErrorString(e)));
    e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        rc = launch_query_set(set, cs, nullptr, nullptr);
        hipGraph_t gr = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &gr);
        p->graph = gr;
        if (!rc && e2 != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e2));
        if (!rc) {
            e2 = hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0);
            if (e2 != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e2));
        }
    } else {
        rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    (void)hipStreamDestroy(cs);
    if (rc) return bail(rc);
    e = hipEventCreate(&p->ev0);
    if (e == hipSuccess) e = hipEventCreate(&p->ev1);
    if (e != hipSuccess) return bail(fail(SIMRANK_EDEVICE, hipGetErrorString(e)));
    *plan_out = p;
    if (n_groups_out) *n_groups_out = ngr;
    return SIMRANK_OK;
}

extern "C" int simrank_batch_plan_create(simrank_graph *const *graphs, int32_t ngraphs,
                                         const simrank_query *qs, int32_t nq,
                                         simrank_batch_plan **plan_out) {
    return simrank_batch_plan_create_ex(graphs, ngraphs, qs, nq, SIMRANK_PLAN_GROUPS, plan_out,
                                        nullptr);
}

extern "C" int simrank_batch_plan_run(simrank_batch_plan *p, void *stream) {
    clear_error();
    if (!p) return fail(SIMRANK_EINVAL, "plan is NULL");
    // a stitched query's descriptor holds the addresses of the index it was
    // planned with
    for (int32_t i = 0; i < p->nq; ++i)
        if (p->index_gen[i] != ~0ull && p->graphs[i]->index_gen != p->index_gen[i])
            return fail(SIMRANK_ESTATE, "query " + std::to_string(i) +
                                            ": its graph's index was rebuilt after the plan was made");
    SRK_HIP(hipSetDevice(p->device));
    hipStream_t st = (hipStream_t)stream;
    SRK_HIP(hipEventRecord(p->ev0, st));
    SRK_HIP(hipGraphLaunch(p->exec, st));
    SRK_HIP(hipEventRecord(p->ev1, st));
    p->last_stream = st;
    p->ran = true;
    return SIMRANK_OK;
}

extern "C" int simrank_batch_plan_wait(simrank_batch_plan *p, simrank_stats *st) {
    clear_error();
    if (!p) return fail(SIMRANK_EINVAL, "plan is NULL");
    if (!p->ran) return fail(SIMRANK_ESTATE, "plan has not run");
    SRK_HIP(hipEventSynchronize(p->ev1));
    if (st) {
        unsigned long long c[8];
        SRK_HIP(hipMemcpy(c, p->counters, sizeof(c), hipMemcpyDeviceToHost));
        float ms = 0.f;
        SRK_HIP(hipEventElapsedTime(&ms, p->ev0, p->ev1));
        *st = simrank_stats{};
        for (int32_t i = 0; i < p->nq; ++i)
            st->pairs += (uint64_t)(p->graphs[i]->n - 1) * (uint64_t)p->params[i].R;
        st->pairs_walked = c[C_PAIRS];
        st->moves = c[C_MOVES];
        st->draws = c[C_DRAWS];
        st->meets = c[C_MEETS];
        st->tail_steps = c[C_TAIL];
        st->source_moves = c[C_SRC_MOVES];
        st->ms = ms;
        st->meet_ms = ms;
    }
    return SIMRANK_OK;
}

extern "C" int simrank_batch_plan_read(simrank_batch_plan *p, int32_t i, double *out_host,
                                       uint32_t *counts_host) {
    clear_error();
    if (!p) return fail(SIMRANK_EINVAL, "plan is NULL");
    if (i < 0 || i >= p->nq) return fail(SIMRANK_EINVAL, "query index out of range");
    if (!p->ran) return fail(SIMRANK_ESTATE, "plan has not run");
    SRK_HIP(hipSetDevice(p->device));
    SRK_HIP(hipEventSynchronize(p->ev1));
    const size_t n = (size_t)p->graphs[i]->n;
    if (counts_host && strat_kind(p->desc[i].kind))
        return fail(SIMRANK_EINVAL, "a stratified query has weighted sums, not counts: "
                                    "use simrank_batch_plan_read_stratified");
    if (out_host) SRK_HIP(hipMemcpy(out_host, p->desc[i].out, 8 * n, hipMemcpyDeviceToHost));
    if (counts_host) SRK_HIP(hipMemcpy(counts_host, p->desc[i].cnt, 4 * n, hipMemcpyDeviceToHost));
    return SIMRANK_OK;
}

extern "C" int simrank_batch_plan_read_stratified(simrank_batch_plan *p, int32_t i,
                                                  double *out_host, double *out_n_host,
                                                  uint64_t *wsum_host) {
    clear_error();
    if (!p) return fail(SIMRANK_EINVAL, "plan is NULL");
    if (i < 0 || i >= p->nq) return fail(SIMRANK_EINVAL, "query index out of range");
    if (!strat_kind(p->desc[i].kind)) return fail(SIMRANK_EINVAL, "not a stratified query");
    if (!p->ran) return fail(SIMRANK_ESTATE, "plan has not run");
    SRK_HIP(hipSetDevice(p->device));
    SRK_HIP(hipEventSynchronize(p->ev1));
    const size_t n = (size_t)p->graphs[i]->n;
    if (out_host) SRK_HIP(hipMemcpy(out_host, p->desc[i].out, 8 * n, hipMemcpyDeviceToHost));
    if (out_n_host) SRK_HIP(hipMemcpy(out_n_host, p->desc[i].out_n, 8 * n, hipMemcpyDeviceToHost));
    if (wsum_host) SRK_HIP(hipMemcpy(wsum_host, p->desc[i].wsum, 8 * n, hipMemcpyDeviceToHost));
    return SIMRANK_OK;
}

// Waits for the plan's last run and frees it (leaves the error message alone).
static void plan_finish(simrank_batch_plan *p) {
    (void)hipSetDevice(p->device);
    if (p->ran) (void)hipEventSynchronize(p->ev1);
    plan_release(p);
}

extern "C" int simrank_batch_plan_free(simrank_batch_plan *p) {
    clear_error();
    if (p) plan_finish(p);
    return SIMRANK_OK;
}

extern "C" int simrank_batch(simrank_graph *const *graphs, int32_t ngraphs,
                             const simrank_query *qs, int32_t nq, double *const *outs,
                             uint32_t *const *counts_opt, simrank_stats *st_opt) {
    clear_error();
    std::vector<simrank_params> ps;
    std::vector<int> modes;
    int rc = check_queries(graphs, ngraphs, qs, nq, ps, modes);
    if (rc) return rc;
    simrank_stats tot{};
    if (nq == 0) {
        if (st_opt) *st_opt = tot;
        return SIMRANK_OK;
    }
    SRK_HIP(hipSetDevice(graphs[qs[0].graph]->device));
    // Admission by device memory: consecutive queries are grouped into plans
    // that fit half of the free memory at the time each plan is made.
    int32_t i0 = 0;
    while (i0 < nq && !rc) {
        size_t free_b = 0, tot_b = 0;
        SRK_HIP(hipMemGetInfo(&free_b, &tot_b));
        const size_t budget = free_b / 2;
        size_t used = 0;
        int32_t i1 = i0;
        while (i1 < nq) {
            const size_t b = request_bytes(ps[i1], modes[i1], graphs[qs[i1].graph]->n) +
                             sizeof(QueryDesc) + 64 +
                             4 * (size_t)ps[i1].R * ps[i1].L + 16 * (size_t)ps[i1].R +
                             1024;   // its share of a group's buffers
            if (i1 > i0 && used + b > budget) break;
            used += b;
            ++i1;
        }
        simrank_batch_plan *p = nullptr;
        rc = simrank_batch_plan_create(graphs, ngraphs, qs + i0, i1 - i0, &p);
        if (rc) break;
        hipStream_t st = nullptr;
        hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
        simrank_stats s1{};
        if (!rc) rc = simrank_batch_plan_run(p, st);
        if (!rc) rc = simrank_batch_plan_wait(p, &s1);
        for (int32_t i = i0; i < i1 && !rc; ++i)   // stratified queries have no counts
            rc = simrank_batch_plan_read(p, i - i0, outs ? outs[i] : nullptr,
                                         counts_opt && modes[i] != SIMRANK_MODE_STRATIFIED
                                             ? counts_opt[i] : nullptr);
        if (st) {
            (void)hipStreamSynchronize(st);   // whatever was enqueued has ended
            (void)hipStreamDestroy(st);
        }
        plan_finish(p);
        tot.pairs += s1.pairs;
        tot.pairs_walked += s1.pairs_walked;
        tot.moves += s1.moves;
        tot.draws += s1.draws;
        tot.meets += s1.meets;
        tot.tail_steps += s1.tail_steps;
        tot.source_moves += s1.source_moves;
        tot.ms += s1.ms;
        tot.meet_ms += s1.meet_ms;
        i0 = i1;
    }
    if (!rc && st_opt) *st_opt = tot;
    return rc;
}

// ------------------------------------------------------------------ tuner

// One measurement: the meet kernel's time of q's second run (the first warms
// the caches) with the graph's current tuning.
static int time_meet(simrank_graph *g, const simrank_query *q, const simrank_params &p, int mode,
                     Workspace *ws, uint32_t *cnt, float *ms_out) {
    float ms = 0.f;
    for (int rep = 0; rep < 2; ++rep) {
        int rc = enqueue_query(g, q, p, mode, ws, nullptr, cnt, g->stream);
        if (rc) return rc;
        SRK_HIP(hipEventSynchronize(ws->ev1));
        SRK_HIP(hipEventElapsedTime(&ms, ws->evm0, ws->evm1));
    }
    *ms_out = ms;
    return SIMRANK_OK;
}

extern "C" int simrank_tune_ex(simrank_graph *g, const simrank_query *q, simrank_tuning *out) {
    clear_error();
    if (!g || !q) return fail(SIMRANK_EINVAL, "NULL argument");
    simrank_params p;
    int mode;
    int rc = query_params(q, g->n, &p, &mode);
    if (rc) return rc;
    if (q->s < 0 || q->s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
    if (mode == SIMRANK_MODE_STRATIFIED) return fail(SIMRANK_EINVAL, "the tuner takes plain or stitched queries");
    if (mode == SIMRANK_MODE_STITCHED && (!g->index || g->index->T != p.T))
        return fail(SIMRANK_ESTATE, "stitched query without a matching index");
    SRK_HIP(hipSetDevice(g->device));
    const int kind = mode == SIMRANK_MODE_STITCHED ? K_STITCHED : K_PLAIN;
    Workspace ws;
    uint32_t *cnt = nullptr;
    rc = workspace_init(g, p.R, p.L, &ws);
    if (!rc) rc = device_alloc((void **)&cnt, 4 * (size_t)g->n, nullptr);
    const int32_t saved_vb = g->tuned_vb, saved_tj = g->tuned_tile_j[kind];
    int32_t best_vb = 0, best_tj = 0;
    float best_ms = 0.f;
    // walks per tile: the kind's tile and each halving down to MIN_TILE_J;
    // nodes per unit: 32 .. MEET_VB while the units still fill a GPU
    for (int32_t tj = tile_j_of(kind); tj >= MIN_TILE_J && !rc; tj /= 2) {
        for (int32_t vb = 32; vb <= MEET_VB && !rc; vb *= 2) {
            if (vb > 32 && (g->n_active + vb - 1) / vb < 64) break;
            g->tuned_vb = vb;
            g->tuned_tile_j[kind] = tj;
            float ms = 0.f;
            rc = time_meet(g, q, p, mode, &ws, cnt, &ms);
            if (!rc && (best_vb == 0 || ms < best_ms)) {
                best_vb = vb;
                best_tj = tj;
                best_ms = ms;
            }
        }
    }
    g->tuned_vb = rc ? saved_vb : best_vb;
    g->tuned_tile_j[kind] = rc ? saved_tj : best_tj;
    device_free(cnt);
    workspace_release(&ws);
    if (!rc && out) {
        *out = simrank_tuning{};
        out->unit_nodes = best_vb;
        out->tile_walks = best_tj;
        out->seg_log2 = g->index ? g->index->seg_log2 : -1;
        out->meet_ms = best_ms;
        out->build_ms = g->index ? g->index->build_ms : 0.0;
    }
    return rc;
}

extern "C" int simrank_tune(simrank_graph *g, const simrank_query *q, int32_t *vb_out) {
    simrank_tuning t;
    const int rc = simrank_tune_ex(g, q, &t);
    if (!rc && vb_out) *vb_out = t.unit_nodes;
    return rc;
}

extern "C" int simrank_set_tuning(simrank_graph *g, int32_t unit_nodes, int32_t tile_walks) {
    clear_error();
    if (!g) return fail(SIMRANK_EINVAL, "graph is NULL");
    if (unit_nodes < 0 || unit_nodes > MEET_VB)
        return fail(SIMRANK_EINVAL, "unit_nodes must lie in [0, " + std::to_string(MEET_VB) + "]");
    if (tile_walks != 0 && (tile_walks < MIN_TILE_J || tile_walks > tile_j_of(K_PLAIN)))
        return fail(SIMRANK_EINVAL, "tile_walks must be 0 or lie in [" + std::to_string(MIN_TILE_J) +
                                        ", " + std::to_string(tile_j_of(K_PLAIN)) + "]");
    g->tuned_vb = unit_nodes;
    for (int k = 0; k < N_KINDS; ++k) g->tuned_tile_j[k] = tile_walks;
    return SIMRANK_OK;
}

extern "C" int simrank_tune_index(simrank_graph *g, const simrank_query *q,
                                  const simrank_index_params *base, const int32_t *seg_log2,
                                  int32_t count, simrank_tuning *out, double *ms_each) {
    clear_error();
    if (!g || !q || !base || !seg_log2) return fail(SIMRANK_EINVAL, "NULL argument");
    if (count < 1 || count > 7) return fail(SIMRANK_EINVAL, "count must lie in [1, 7]");
    if (q->mode != SIMRANK_MODE_STITCHED) return fail(SIMRANK_EINVAL, "the index tuner takes a stitched query");
    for (int32_t i = 0; i < count; ++i)
        if (seg_log2[i] < 0 || seg_log2[i] > 6) return fail(SIMRANK_EINVAL, "seg_log2 must lie in [0, 6]");
    simrank_params p;
    int mode;
    int rc = query_params(q, g->n, &p, &mode);
    if (rc) return rc;
    if (q->s < 0 || q->s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
    if (continue_threshold(base->c) != p.T)
        return fail(SIMRANK_EINVAL, "the query's c differs from the index's c");
    SRK_HIP(hipSetDevice(g->device));
    Workspace ws;
    uint32_t *cnt = nullptr;
    rc = workspace_init(g, p.R, p.L, &ws);
    if (!rc) rc = device_alloc((void **)&cnt, 4 * (size_t)g->n, nullptr);
    int32_t best = -1, built = -1;
    float best_ms = 0.f;
    for (int32_t i = 0; i < count && !rc; ++i) {
        simrank_index_params ip = *base;
        ip.seg_log2 = seg_log2[i];
        rc = simrank_build_index(g, &ip);
        if (rc) break;
        built = seg_log2[i];
        float ms = 0.f;
        rc = time_meet(g, q, p, mode, &ws, cnt, &ms);
        if (rc) break;
        if (ms_each) ms_each[i] = ms;
        if (best < 0 || ms < best_ms) {
            best = seg_log2[i];
            best_ms = ms;
        }
    }
    device_free(cnt);
    workspace_release(&ws);
    if (!rc && built != best) {
        simrank_index_params ip = *base;
        ip.seg_log2 = best;
        rc = simrank_build_index(g, &ip);
    }
    if (!rc && out) {
        *out = simrank_tuning{};
        out->unit_nodes = default_unit_nodes(g);
        out->tile_walks = g->tuned_tile_j[K_STITCHED] > 0 ? g->tuned_tile_j[K_STITCHED]
                                                          : tile_j_of(K_STITCHED);
        out->seg_log2 = best;
        out->meet_ms = best_ms;
        out->build_ms = g->index->build_ms;
    }
    return rc;
}
