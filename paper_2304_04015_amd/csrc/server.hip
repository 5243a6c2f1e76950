// Serving: a request loop over one device-resident graph (and its index).
//
// Requests are queued by simrank_server_submit and admitted by a worker thread
// into slots as slots free up.  A slot is a workspace, device buffers for the
// estimate and the counts, pinned host buffers and its own stream; the number
// of slots is what the device-memory budget admits.  An admitted request is
// enqueued whole on its slot's stream (query kernels, then the copy of its
// results to the slot's pinned buffers, then an event), so requests that arrive
// while others run are started as soon as a slot is free and their kernels
// overlap on the device.  With group_max >= 2, plain or stitched requests that
// share (mode, seed, c, cap) and are waiting together are admitted as one
// query group (group.hip) into as many slots: one launch on the first slot's
// stream walks each (v, j) once for all of them.  While a group runs, the
// requests that arrive wait and form the next group.  Each result equals the
// lone query's.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "common.hpp"

namespace srk {
namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct Request {
    uint64_t ticket = 0;
    simrank_query q{};
    simrank_params p{};
    int mode = 0;
    int state = 0;          // 0 queued, 1 running, 2 done, 3 failed
    int rc = 0;
    std::string err;
    double t_submit = 0, t_start = 0, t_done = 0;
    std::vector<double> out;
    std::vector<uint32_t> cnt;
    simrank_stats st{};
};

struct Slot {
    bool grouped = false;           // its request runs in the server's group
    int32_t group_size = 1;
    Workspace ws;
    double *out_dev = nullptr;
    uint32_t *cnt_dev = nullptr;
    double *out_host = nullptr;     // pinned
    uint32_t *cnt_host = nullptr;   // pinned
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Request *req = nullptr;
};

// The one group in flight: descriptors of its members and of the group
// (pinned staging copies and device arrays), the unit tables and counters of
// its launch, and the group's compaction buffers, sized for group_max members
// of (max_R, max_L).
struct GroupRun {
    QueryDesc *desc_host = nullptr, *desc_dev = nullptr;
    GroupDesc *gdesc_host = nullptr, *gdesc_dev = nullptr;
    uint32_t *units = nullptr, *gunits = nullptr;
    unsigned long long *counters = nullptr;
    char *buffers = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around the group's kernels
    bool busy = false;
    int32_t lead = -1;                         // slot whose stream runs it
};

// Requests of one group share the walks from every node.
bool same_walks(const Request *a, const Request *b) {
    return a->mode == b->mode && a->q.seed == b->q.seed && a->p.T == b->p.T && a->p.L == b->p.L;
}

}  // namespace
}  // namespace srk

using namespace srk;

struct simrank_server {
    simrank_graph *g = nullptr;
    simrank_server_params prm{};
    std::vector<Slot> slots;
    int64_t slot_bytes = 0;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    uint64_t n_done = 0, n_failed = 0;
    GroupRun grp;
    int32_t gmax = 0;          // largest group the server forms (its buffers' size)
    uint64_t n_groups = 0, n_grouped = 0;
};

// Attaches a slot's workspace and result buffers to a descriptor.
static void slot_buffers(Slot &sl, QueryDesc *d) {
    d->sw = sl.ws.sw;
    d->slen = sl.ws.slen;
    d->jj = sl.ws.jj;
    d->joff = sl.ws.joff;
    d->swc = sl.ws.swc;
    d->tiles = sl.ws.tiles;
    d->meta = sl.ws.meta;
    d->cnt = sl.cnt_dev;
    d->out = sl.out_dev;
}

// Enqueues the group of requests rs (2..group_max, equal walks) into the free
// slots idx on the first slot's stream: descriptors, the query set with its
// group, result copies, each slot's completion event.
static int launch_group(simrank_server *S, const std::vector<Request *> &rs,
                        const std::vector<int32_t> &idx) {
    GroupRun &gr = S->grp;
    const Graph *g = S->g;
    const int32_t G = (int32_t)rs.size();
    hipStream_t st = S->slots[idx[0]].stream;
    const int32_t vb = default_unit_nodes(g);
    std::vector<const QueryDesc *> mem(G);
    int64_t sum_RL = 0;
    for (int32_t i = 0; i < G; ++i) {
        QueryDesc &d = gr.desc_host[i];
        describe_query(g, &rs[i]->q, rs[i]->p, rs[i]->mode, vb, &d);
        slot_buffers(S->slots[idx[i]], &d);
        d.kind = d.kind == K_STITCHED ? K_GROUPED_STITCHED : K_GROUPED;
        mem[i] = &d;
        sum_RL += (int64_t)d.R * d.L;
    }
    GroupDesc *gd = gr.gdesc_host;
    describe_group(mem.data(), G, gd);
    (void)group_buffers(gd, sum_RL, gr.buffers);
    const int64_t units = (int64_t)group_max_tiles(gd->Rmax, sum_RL, gd->L, G, gd->wk) * gd->n_chunks;
    if (units >= (int64_t)0x7fffffff) return fail(SIMRANK_EINVAL, "group has too many work units");
    GroupSet gs;
    gs.desc = gr.gdesc_dev;
    gs.ng = 1;
    gs.units_bound[group_list(G, gd->wk)] = units;
    gs.units = gr.gunits;
    QuerySet qs;
    qs.desc = gr.desc_dev;
    qs.nq = G;
    qs.max_R = gd->Rmax;
    qs.max_n = g->n;
    qs.units = gr.units;
    qs.counters = gr.counters;
    qs.groups = &gs;
    SRK_HIP(hipMemcpyAsync(gr.desc_dev, gr.desc_host, sizeof(QueryDesc) * G, hipMemcpyHostToDevice, st));
    SRK_HIP(hipMemcpyAsync(gr.gdesc_dev, gr.gdesc_host, sizeof(GroupDesc), hipMemcpyHostToDevice, st));
    SRK_HIP(hipEventRecord(gr.ev0, st));
    int rc = launch_query_set(qs, st, nullptr, nullptr);
    if (rc) return rc;
    SRK_HIP(hipEventRecord(gr.ev1, st));
    const size_t n = (size_t)g->n;
    for (int32_t i = 0; i < G; ++i) {
        Slot &sl = S->slots[idx[i]];
        SRK_HIP(hipMemcpyAsync(sl.out_host, sl.out_dev, 8 * n, hipMemcpyDeviceToHost, st));
        SRK_HIP(hipMemcpyAsync(sl.cnt_host, sl.cnt_dev, 4 * n, hipMemcpyDeviceToHost, st));
        SRK_HIP(hipEventRecord(sl.done, st));
    }
    gr.busy = true;
    gr.lead = idx[0];
    return SIMRANK_OK;
}

// Copies a finished slot's results and work counters into its request.
static void collect_results(simrank_server *S, Slot &sl, Request *r) {
    const size_t n = (size_t)S->g->n;
    r->out.assign(sl.out_host, sl.out_host + n);
    r->cnt.assign(sl.cnt_host, sl.cnt_host + n);
    // a grouped request reports its share (1/G) of its group's work and the
    // group's device time
    unsigned long long c[8];
    hipError_t e = hipMemcpy(c, sl.grouped ? S->grp.counters : sl.ws.counters, sizeof(c),
                             hipMemcpyDeviceToHost);
    if (sl.grouped)
        for (unsigned long long &x : c) x /= (unsigned long long)sl.group_size;
    float ms = 0.f, mms = 0.f;
    if (sl.grouped) {
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, S->grp.ev0, S->grp.ev1);
        mms = ms;
    } else {
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, sl.ws.ev0, sl.ws.ev1);
        if (e == hipSuccess) e = hipEventElapsedTime(&mms, sl.ws.evm0, sl.ws.evm1);
    }
    if (e != hipSuccess) {
        (void)hipGetLastError();
        r->rc = SIMRANK_EDEVICE;
        r->err = hipGetErrorString(e);
        return;
    }
    r->st.pairs = (uint64_t)(S->g->n - 1) * (uint64_t)r->p.R;
    r->st.pairs_walked = c[C_PAIRS];
    r->st.moves = c[C_MOVES];
    r->st.draws = c[C_DRAWS];
    r->st.meets = c[C_MEETS];
    r->st.tail_steps = c[C_TAIL];
    r->st.source_moves = c[C_SRC_MOVES];
    r->st.ms = ms;
    r->st.meet_ms = mms;
    r->st.R = r->p.R;
    r->st.L = r->p.L;
    r->st.T = r->p.T;
    r->rc = SIMRANK_OK;
}

// Enqueues request r alone on slot sl: its kernels, the copies of its results
// to the slot's pinned buffers, the slot's completion event.
static int launch_single(simrank_server *S, Slot &sl, Request *r) {
    const size_t n = (size_t)S->g->n;
    int rc = enqueue_query(S->g, &r->q, r->p, r->mode, &sl.ws, sl.out_dev, sl.cnt_dev, sl.stream);
    if (rc) return rc;
    SRK_HIP(hipMemcpyAsync(sl.out_host, sl.out_dev, 8 * n, hipMemcpyDeviceToHost, sl.stream));
    SRK_HIP(hipMemcpyAsync(sl.cnt_host, sl.cnt_dev, 4 * n, hipMemcpyDeviceToHost, sl.stream));
    SRK_HIP(hipEventRecord(sl.done, sl.stream));
    return SIMRANK_OK;
}

// The worker.  It alone touches the slots and the group's buffers, and it
// alone writes a running request's results; the mutex guards the queue, the
// requests' states and the counters.  A waiter reads a request's results only
// after its state, set under the mutex, says it ended, so results are copied
// and kernels enqueued without holding the mutex, and submitters and waiters
// are never held up by device calls.
static void server_loop(simrank_server *S) {
    (void)hipSetDevice(S->g->device);
    std::vector<Request *> ended, admitted;
    std::vector<int32_t> idx;
    for (;;) {
        bool progressed = false;
        uint64_t inflight = 0;
        // completions
        ended.clear();
        for (Slot &sl : S->slots) {
            if (!sl.req) continue;
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipErrorNotReady) {
                ++inflight;
                continue;
            }
            Request *r = sl.req;
            if (e == hipSuccess) {
                collect_results(S, sl, r);
            } else {
                (void)hipGetLastError();
                r->rc = SIMRANK_EDEVICE;
                r->err = hipGetErrorString(e);
            }
            r->t_done = now_s();
            ended.push_back(r);
            sl.req = nullptr;
            sl.grouped = false;
        }
        // the group is done once none of its slots holds a request
        if (S->grp.busy) {
            bool running = false;
            for (Slot &sl : S->slots) running |= sl.grouped;
            if (!running) S->grp.busy = false;
        }
        idx.clear();
        for (int32_t i = 0; i < (int32_t)S->slots.size(); ++i)
            if (!S->slots[i].req) idx.push_back(i);
        // admission: requests leave the queue under the mutex
        admitted.clear();
        bool group = false;
        const int32_t gmax = S->gmax;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            for (Request *r : ended) {
                r->state = r->rc ? 3 : 2;
                ++(r->rc ? S->n_failed : S->n_done);
            }
            if (!ended.empty()) {
                progressed = true;
                S->cv_done.notify_all();
            }
            // Groups (group_max >= 2): one launch in flight at a time.  Once
            // the device is free, the requests waiting with the same walks as
            // the first one (up to group_max and the free slots) start as one
            // group; a request with no partner starts alone.
            if (gmax >= 2 && !S->queue.empty() && inflight == 0) {
                Request *head = S->queue.front();
                const size_t cap = (size_t)std::min<int32_t>(gmax, (int32_t)idx.size());
                for (Request *r : S->queue)
                    if (admitted.size() < cap && same_walks(head, r)) admitted.push_back(r);
                if (admitted.size() >= 2) {
                    group = true;
                    for (Request *r : admitted)
                        S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
                } else {
                    admitted.clear();
                }
            }
            if (!group) {
                // one request per free slot; with groups, one alone and only
                // when nothing runs
                const size_t cap = gmax >= 2 ? (inflight == 0 ? 1 : 0) : idx.size();
                while (admitted.size() < std::min(cap, idx.size()) && !S->queue.empty()) {
                    admitted.push_back(S->queue.front());
                    S->queue.pop_front();
                }
            }
            for (Request *r : admitted) r->state = 1;
            if (admitted.empty()) {
                if (S->stop && S->queue.empty() && inflight == 0) break;
                if (!progressed) {
                    if (inflight == 0 && S->queue.empty())
                        S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
                    else
                        S->cv_work.wait_for(lk, std::chrono::microseconds(50));
                }
                continue;
            }
        }
        // enqueue on the device, without the mutex
        const double t = now_s();
        for (Request *r : admitted) r->t_start = t;
        if (group) {
            idx.resize(admitted.size());
            const int rc = launch_group(S, admitted, idx);
            for (size_t i = 0; i < admitted.size(); ++i) {
                Request *r = admitted[i];
                if (rc) {
                    r->rc = rc;
                    r->err = simrank_last_error();
                    r->t_done = now_s();
                } else {
                    Slot &sl = S->slots[idx[i]];
                    sl.req = r;
                    sl.grouped = true;
                    sl.group_size = (int32_t)admitted.size();
                }
            }
            if (rc) {
                // copies of the staged descriptors may have been enqueued:
                // let them finish before the staging buffers are reused
                (void)hipStreamSynchronize(S->slots[idx[0]].stream);
                S->grp.busy = false;
            }
        } else {
            for (size_t i = 0; i < admitted.size(); ++i) {
                Request *r = admitted[i];
                Slot &sl = S->slots[idx[i]];
                const int rc = launch_single(S, sl, r);
                if (rc) {
                    r->rc = rc;
                    r->err = simrank_last_error();
                    r->t_done = now_s();
                } else {
                    sl.req = r;
                }
            }
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            bool failed = false;
            for (Request *r : admitted)
                if (r->rc) {
                    r->state = 3;
                    ++S->n_failed;
                    failed = true;
                }
            if (group && !failed) {
                ++S->n_groups;
                S->n_grouped += admitted.size();
            }
            if (failed) S->cv_done.notify_all();
        }
    }
}

static void server_release(simrank_server *S) {
    GroupRun &gr = S->grp;
    if (gr.lead >= 0 && S->slots[gr.lead].stream) (void)hipStreamSynchronize(S->slots[gr.lead].stream);
    if (gr.desc_host) (void)hipHostFree(gr.desc_host);
    if (gr.gdesc_host) (void)hipHostFree(gr.gdesc_host);
    device_free(gr.desc_dev);
    device_free(gr.gdesc_dev);
    device_free(gr.units);
    device_free(gr.gunits);
    device_free(gr.counters);
    device_free(gr.buffers);
    if (gr.ev0) (void)hipEventDestroy(gr.ev0);
    if (gr.ev1) (void)hipEventDestroy(gr.ev1);
    for (Slot &sl : S->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        workspace_release(&sl.ws);
        device_free(sl.out_dev);
        device_free(sl.cnt_dev);
        if (sl.out_host) (void)hipHostFree(sl.out_host);
        if (sl.cnt_host) (void)hipHostFree(sl.cnt_host);
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    for (auto &kv : S->all) delete kv.second;
    delete S;
}

extern "C" int simrank_server_create(simrank_graph *g, const simrank_server_params *p,
                                     simrank_server **out) {
    clear_error();
    if (!g || !p || !out) return fail(SIMRANK_EINVAL, "NULL argument");
    *out = nullptr;
    if (p->max_slots < 1 || p->max_slots > 64) return fail(SIMRANK_EINVAL, "max_slots must lie in [1, 64]");
    if (p->max_R < 1 || p->max_R > MAX_R) return fail(SIMRANK_EINVAL, "max_R must lie in [1, 2^24]");
    if (p->max_L < 1 || p->max_L > MAX_CAP) return fail(SIMRANK_EINVAL, "max_L must lie in [1, 255]");
    if (p->group_max < 0 || p->group_max > GROUP_MAX)
        return fail(SIMRANK_EINVAL, "group_max must lie in [0, 32]");
    SRK_HIP(hipSetDevice(g->device));
    simrank_server *S = new simrank_server();
    S->g = g;
    S->prm = *p;
    const size_t RL = (size_t)p->max_R * (size_t)p->max_L;
    S->slot_bytes = (int64_t)(8 * RL + 13 * (size_t)p->max_R + 4 * (size_t)max_tiles_for(p->max_R, p->max_L) +
                              12 * (size_t)g->n + 4096);
    size_t free_b = 0, tot_b = 0;
    SRK_HIP(hipMemGetInfo(&free_b, &tot_b));
    int64_t budget = p->hbm_budget > 0 ? std::min<int64_t>(p->hbm_budget, (int64_t)free_b)
                                       : (int64_t)(free_b / 2);
    const int64_t fit = budget / std::max<int64_t>(S->slot_bytes, 1);
    const int32_t nslots = (int32_t)std::min<int64_t>(p->max_slots, fit);
    if (nslots < 1) {
        delete S;
        return fail(SIMRANK_ENOMEM, "device-memory budget admits no slot of " +
                                        std::to_string(S->slot_bytes) + " bytes");
    }
    S->slots.resize(nslots);
    int rc = SIMRANK_OK;
    for (Slot &sl : S->slots) {
        rc = workspace_init(g, p->max_R, p->max_L, &sl.ws);
        if (!rc) rc = device_alloc((void **)&sl.out_dev, 8 * (size_t)g->n, nullptr);
        if (!rc) rc = device_alloc((void **)&sl.cnt_dev, 4 * (size_t)g->n, nullptr);
        hipError_t e = hipSuccess;
        if (!rc) e = hipHostMalloc((void **)&sl.out_host, 8 * (size_t)g->n, hipHostMallocDefault);
        if (!rc && e == hipSuccess) e = hipHostMalloc((void **)&sl.cnt_host, 4 * (size_t)g->n, hipHostMallocDefault);
        if (!rc && e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (!rc && e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (!rc && e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
        if (rc) break;
    }
    int32_t gmax = std::min<int32_t>(p->group_max, nslots);
    // a group's packed positions are addressed in 32 bits
    while (gmax >= 2 &&
           group_pos_words(p->max_R, (int64_t)gmax * p->max_R * p->max_L, p->max_L) >= (int64_t)0xffff0000)
        --gmax;
    S->gmax = gmax;
    if (!rc && gmax >= 2) {   // the group's own buffers
        GroupRun &gr = S->grp;
        GroupDesc gd{};
        gd.Rmax = p->max_R;
        gd.L = p->max_L;
        gd.G = gmax;
        gd.gw = (gmax + 3) / 4;
        const int64_t sum_RL = (int64_t)gmax * p->max_R * p->max_L;
        const size_t gb = group_buffers(&gd, sum_RL, nullptr);
        rc = device_alloc((void **)&gr.buffers, gb, nullptr);
        if (!rc) rc = device_alloc((void **)&gr.desc_dev, sizeof(QueryDesc) * gmax, nullptr);
        if (!rc) rc = device_alloc((void **)&gr.gdesc_dev, sizeof(GroupDesc), nullptr);
        if (!rc) rc = device_alloc((void **)&gr.units, 4 * units_words(gmax), nullptr);
        if (!rc) rc = device_alloc((void **)&gr.gunits, 4 * group_units_words(1), nullptr);
        if (!rc) rc = device_alloc((void **)&gr.counters, 8 * 8, nullptr);
        hipError_t e = hipSuccess;
        if (!rc) e = hipHostMalloc((void **)&gr.desc_host, sizeof(QueryDesc) * gmax, hipHostMallocDefault);
        if (!rc && e == hipSuccess) e = hipHostMalloc((void **)&gr.gdesc_host, sizeof(GroupDesc), hipHostMallocDefault);
        if (!rc && e == hipSuccess) e = hipEventCreate(&gr.ev0);
        if (!rc && e == hipSuccess) e = hipEventCreate(&gr.ev1);
        if (!rc && e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    if (rc) {
        server_release(S);
        return rc;
    }
    S->worker = std::thread(server_loop, S);
    *out = S;
    return SIMRANK_OK;
}

extern "C" int simrank_server_info(const simrank_server *S, int32_t *slots, int64_t *slot_bytes) {
    clear_error();
    if (!S) return fail(SIMRANK_EINVAL, "server is NULL");
    if (slots) *slots = (int32_t)S->slots.size();
    if (slot_bytes) *slot_bytes = S->slot_bytes;
    return SIMRANK_OK;
}

extern "C" int simrank_server_counts(simrank_server *S, uint64_t *done, uint64_t *failed,
                                     uint64_t *groups, uint64_t *grouped) {
    clear_error();
    if (!S) return fail(SIMRANK_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    if (done) *done = S->n_done;
    if (failed) *failed = S->n_failed;
    if (groups) *groups = S->n_groups;
    if (grouped) *grouped = S->n_grouped;
    return SIMRANK_OK;
}

extern "C" int simrank_server_submit(simrank_server *S, const simrank_query *q, uint64_t *ticket) {
    clear_error();
    if (!S || !q || !ticket) return fail(SIMRANK_EINVAL, "NULL argument");
    Request *r = new Request();
    r->q = *q;
    int rc = query_params(q, S->g->n, &r->p, &r->mode);
    if (!rc && (q->s < 0 || q->s >= S->g->n)) rc = fail(SIMRANK_EINVAL, "source out of range");
    if (!rc && r->mode == SIMRANK_MODE_STRATIFIED)
        rc = fail(SIMRANK_EINVAL, "stratified queries are not served");
    if (!rc && (r->p.R > S->prm.max_R || r->p.L > S->prm.max_L))
        rc = fail(SIMRANK_EINVAL, "query needs R or L beyond the server's slots");
    if (!rc && r->mode == SIMRANK_MODE_STITCHED && (!S->g->index || S->g->index->T != r->p.T))
        rc = fail(SIMRANK_ESTATE, "stitched query without a matching index");
    if (rc) {
        delete r;
        return rc;
    }
    r->t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->stop) {
            delete r;
            return fail(SIMRANK_ESTATE, "server is stopping");
        }
        r->ticket = S->next_ticket++;
        S->all[r->ticket] = r;
        S->queue.push_back(r);
    }
    S->cv_work.notify_one();
    *ticket = r->ticket;
    return SIMRANK_OK;
}

extern "C" int simrank_server_wait(simrank_server *S, uint64_t ticket, double timeout_s,
                                   double *out_host, uint32_t *counts_host,
                                   simrank_request_info *info) {
    clear_error();
    if (!S) return fail(SIMRANK_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    if (S->all.find(ticket) == S->all.end()) return fail(SIMRANK_EINVAL, "unknown ticket");
    // looked up afresh at every wake-up: another wait on the same ticket may
    // have retired it meanwhile
    auto finished = [&] {
        auto it = S->all.find(ticket);
        return it == S->all.end() || it->second->state >= 2;
    };
    if (timeout_s < 0) {
        S->cv_done.wait(lk, finished);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
        return fail(SIMRANK_ESTATE, "request not finished");
    }
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(SIMRANK_EINVAL, "ticket retired by another wait");
    Request *r = it->second;
    S->all.erase(it);
    lk.unlock();
    int rc = SIMRANK_OK;
    if (r->state == 3) {
        rc = fail(r->rc, r->err);
    } else {
        const size_t n = (size_t)S->g->n;
        if (out_host) std::copy(r->out.begin(), r->out.begin() + n, out_host);
        if (counts_host) std::copy(r->cnt.begin(), r->cnt.begin() + n, counts_host);
        if (info) {
            info->queue_s = r->t_start - r->t_submit;
            info->latency_s = r->t_done - r->t_submit;
            info->stats = r->st;
        }
    }
    delete r;
    return rc;
}

extern "C" int simrank_server_destroy(simrank_server *S) {
    clear_error();
    if (!S) return SIMRANK_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    if (S->worker.joinable()) S->worker.join();
    server_release(S);
    return SIMRANK_OK;
}
