// Serving: continuous batching of single-source requests over one
// device-resident graph (and its stitched index).
//
// Requests are queued by simrank_server_submit and admitted by a worker
// thread, oldest first, as soon as a ring entry and the request's own device
// memory are free: each request takes request_bytes(R, L, n) from the
// server's device pool (admission by memory, sized per request).  An admitted
// request is prepared on the preparation stream (descriptor, source walks,
// compaction) and published into the ring (common.hpp); persistent meet
// kernels, one launch per kind after each round of admissions, alternating
// between two streams, take work units from every published entry of their
// kind, oldest first, and exit when no unit is left.  Requests that arrive
// while others run are therefore admitted while the GPU works, and their
// units join the running kernel's stream of units: their work overlaps the
// running requests' on the device, and one request's last units overlap the
// next one's first.  The block that finishes a request's last unit writes its
// estimate and raises its flag in pinned host memory; the worker then copies
// the results to the host (staging buffers, copy stream) and retires the
// request.  Plain, stitched and stratified requests are served.
//
// With group_max >= 2, plain or stitched requests that share (mode, seed, c,
// cap) wait while a request with the same walks runs, and those that then
// wait together are admitted as one query group (group.hip), which walks each
// (v, j) once for all of them; a group is one launch on a worker stream (one
// group in flight at a time).  Every result equals the lone query's.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
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

// First-fit allocator over the server's device pool (offsets, 256-byte
// granules); free blocks are merged with their neighbours.
class PoolAlloc {
  public:
    explicit PoolAlloc(size_t bytes = 0) {
        if (bytes) free_[0] = bytes;
        total_ = bytes;
    }
    bool alloc(size_t bytes, size_t *off) {
        bytes = (bytes + 255) & ~(size_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            *off = it->first;
            const size_t rest = it->second - bytes;
            const size_t at = it->first + bytes;
            free_.erase(it);
            if (rest) free_[at] = rest;
            used_ += bytes;
            peak_ = std::max(peak_, used_);
            return true;
        }
        return false;
    }
    void release(size_t off, size_t bytes) {
        bytes = (bytes + 255) & ~(size_t)255;
        used_ -= bytes;
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    size_t peak() const { return peak_; }
    size_t total() const { return total_; }

  private:
    std::map<size_t, size_t> free_;
    size_t total_ = 0, used_ = 0, peak_ = 0;
};

struct Request {
    uint64_t ticket = 0;
    simrank_query q{};
    simrank_params p{};
    int mode = 0;
    int state = 0;          // 0 queued, 1 running, 2 done, 3 failed
    int rc = 0;
    std::string err;
    double t_submit = 0, t_start = 0, t_done = 0;
    std::vector<double> out, out_n;
    std::vector<uint32_t> cnt;
    std::vector<unsigned long long> wsum;
    simrank_stats st{};
    // worker-side
    int32_t slot = -1;      // ring entry (lone requests)
    uint32_t seq = 0;
    size_t mem_off = 0, mem_bytes = 0;
    QueryDesc d{};
    int phase = 0;          // 1 on the device, 2 results being copied
    int stage = -1;         // staging set while copying
    bool grouped = false;
    int32_t group_size = 1;
    int32_t group_pos = 0;
    uint64_t zbits = 0;     // stratified: the bits of Algorithm 2's z (part of its walks)
};

// Pinned host buffers for one request's results, with the copy's event.
struct Staging {
    double *out = nullptr, *out_n = nullptr;
    uint32_t *cnt = nullptr;
    unsigned long long *wsum = nullptr;
    unsigned long long *ctr = nullptr;   // [8]
    hipEvent_t ev = nullptr;
    bool busy = false;
};

// The one group in flight: descriptors of its members and of the group
// (pinned staging copies and device arrays), unit tables, counters and the
// group's compaction buffers, sized for gmax members of (max_R, max_L).
struct GroupRun {
    QueryDesc *desc_host = nullptr, *desc_dev = nullptr;
    GroupDesc *gdesc_host = nullptr, *gdesc_dev = nullptr;
    uint32_t *units = nullptr, *gunits = nullptr;
    unsigned long long *counters = nullptr;
    char *buffers = nullptr;
    StratTab *tabs_host = nullptr;       // pinned [GROUP_MAX] class tables of stratified members
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    std::vector<Request *> members;
    bool busy = false;
};

// Requests whose walks are the same (a group walks them once for all): mode,
// seed, continue threshold and cap; stratified also N and z, which fix the
// length classes.
bool same_walks(const Request *a, const Request *b) {
    return a->mode == b->mode && a->q.seed == b->q.seed && a->p.T == b->p.T && a->p.L == b->p.L &&
           (a->mode != SIMRANK_MODE_STRATIFIED || (a->p.R == b->p.R && a->zbits == b->zbits));
}

int kind_of(int mode) {
    return mode == SIMRANK_MODE_STITCHED ? K_STITCHED : mode == SIMRANK_MODE_STRATIFIED ? K_STRAT
                                                                                           : K_PLAIN;
}

constexpr int N_STAGING = 4;

}  // namespace
}  // namespace srk

using namespace srk;

struct simrank_server {
    simrank_graph *g = nullptr;
    simrank_server_params prm{};
    int32_t entries = 0;                 // ring entries (requests in flight), <= RING_MAX
    int64_t slot_bytes = 0;              // bytes of a (max_R, max_L) plain request
    // device pool and ring
    char *pool = nullptr;
    PoolAlloc alloc;
    StreamRing ring{};
    uint32_t *flags_host = nullptr;      // pinned, written by the device
    StratTab *tabs_host = nullptr;       // pinned [RING_MAX] class tables of stratified requests
    std::vector<Request *> slot_req;     // request in each ring entry
    uint32_t next_seq = 1;
    hipStream_t prep = nullptr, copy = nullptr, work[2] = {nullptr, nullptr};
    int next_work = 0;
    hipEvent_t ev_prep = nullptr;
    Staging stage[N_STAGING];
    GroupRun grp;
    int32_t gmax = 0;
    // host-side queue (mutex)
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Request *> queue;
    std::unordered_map<uint64_t, Request *> all;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::thread worker;
    uint64_t n_done = 0, n_failed = 0, n_groups = 0, n_grouped = 0, n_launches = 0;
    int32_t inflight_peak = 0;
    int32_t inflight = 0;                // worker-only
};

// Enqueues the copies of a finished request's results to staging set k.
static int start_copy(simrank_server *S, Request *r, int k) {
    Staging &sg = S->stage[k];
    const size_t n = (size_t)S->g->n;
    hipStream_t st = S->copy;
    const QueryDesc &d = r->d;
    SRK_HIP(hipMemcpyAsync(sg.out, d.out, 8 * n, hipMemcpyDeviceToHost, st));
    if (r->mode == SIMRANK_MODE_STRATIFIED) {
        SRK_HIP(hipMemcpyAsync(sg.out_n, d.out_n, 8 * n, hipMemcpyDeviceToHost, st));
        SRK_HIP(hipMemcpyAsync(sg.wsum, d.wsum, 8 * n, hipMemcpyDeviceToHost, st));
    } else {
        SRK_HIP(hipMemcpyAsync(sg.cnt, d.cnt, 4 * n, hipMemcpyDeviceToHost, st));
    }
    const unsigned long long *ctr = r->grouped ? S->grp.counters : S->ring.counters + (size_t)r->slot * 8;
    SRK_HIP(hipMemcpyAsync(sg.ctr, ctr, 64, hipMemcpyDeviceToHost, st));
    SRK_HIP(hipEventRecord(sg.ev, st));
    sg.busy = true;
    r->stage = k;
    r->phase = 2;
    return SIMRANK_OK;
}

// Moves a copied request's results from its staging set into the request.
static void finish_copy(simrank_server *S, Request *r) {
    Staging &sg = S->stage[r->stage];
    const size_t n = (size_t)S->g->n;
    r->out.assign(sg.out, sg.out + n);
    if (r->mode == SIMRANK_MODE_STRATIFIED) {
        r->out_n.assign(sg.out_n, sg.out_n + n);
        r->wsum.assign(sg.wsum, sg.wsum + n);
    } else {
        r->cnt.assign(sg.cnt, sg.cnt + n);
    }
    unsigned long long c[8];
    std::memcpy(c, sg.ctr, sizeof(c));
    if (r->grouped)   // a grouped request reports its share of its group's work
        for (unsigned long long &x : c) x /= (unsigned long long)r->group_size;
    r->st = simrank_stats{};
    r->st.pairs = (uint64_t)(S->g->n - 1) * (uint64_t)r->p.R;
    r->st.pairs_walked = c[C_PAIRS];
    r->st.moves = c[C_MOVES];
    r->st.draws = c[C_DRAWS];
    r->st.meets = c[C_MEETS];
    r->st.tail_steps = c[C_TAIL];
    r->st.source_moves = c[C_SRC_MOVES];
    if (r->grouped) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, S->grp.ev0, S->grp.ev1) != hipSuccess) (void)hipGetLastError();
        r->st.ms = r->st.meet_ms = ms;
    } else {
        // the request shares persistent kernels with others: its span from
        // the start of its preparation to its completion, on the host clock
        r->st.ms = r->st.meet_ms = 1e3 * (now_s() - r->t_start);
    }
    r->st.R = r->p.R;
    r->st.L = r->p.L;
    r->st.T = r->p.T;
    r->rc = SIMRANK_OK;
    sg.busy = false;
    r->stage = -1;
}

// Returns a retired request's device resources.
static void release_request(simrank_server *S, Request *r) {
    if (r->mem_bytes) S->alloc.release(r->mem_off, r->mem_bytes);
    r->mem_bytes = 0;
    if (r->slot >= 0) S->slot_req[r->slot] = nullptr;
    r->slot = -1;
    --S->inflight;
}

// Reserves a ring entry (lone requests) and device memory; fills the
// request's descriptor.  false if either is not available now.
static bool reserve(simrank_server *S, Request *r, bool lone) {
    int32_t slot = -1;
    if (lone) {
        for (int32_t i = 0; i < S->entries; ++i)
            if (!S->slot_req[i]) {
                slot = i;
                break;
            }
        if (slot < 0) return false;
    }
    const size_t bytes = request_bytes(r->p, r->mode, S->g->n);
    size_t off = 0;
    if (!S->alloc.alloc(bytes, &off)) return false;
    r->mem_off = off;
    r->mem_bytes = bytes;
    r->slot = slot;
    if (lone) S->slot_req[slot] = r;
    describe_query(S->g, &r->q, r->p, r->mode, default_unit_nodes(S->g), &r->d);
    carve_request(r->p, r->mode, S->g->n, S->pool + off, &r->d);
    ++S->inflight;
    S->inflight_peak = std::max(S->inflight_peak, S->inflight);
    return true;
}

// Enqueues a lone request's preparation and publication into its ring entry.
static int prepare(simrank_server *S, Request *r) {
    r->seq = S->next_seq;
    S->next_seq = S->next_seq + 1 < RING_SEQ_LIMIT ? S->next_seq + 1 : 1u;
    if (r->mode == SIMRANK_MODE_STRATIFIED) {
        StratParams sp;
        StratTab *tab = S->tabs_host + r->slot;
        int rc = strat_params(&r->q, S->g->n, &sp, tab);
        if (rc) return rc;
        r->d.z = sp.z;
        r->d.sa = sp.sa;
        r->d.sb = sp.sb;
        SRK_HIP(hipMemcpyAsync((void *)r->d.tab, tab, sizeof(StratTab), hipMemcpyHostToDevice, S->prep));
    }
    return enqueue_ring_request(r->d, S->ring, r->slot, r->seq, S->prep);
}

// Enqueues the group rs (2..gmax members with equal walks, memory reserved)
// on a worker stream: descriptors, the group's launch sequence, its events.
static int launch_group(simrank_server *S, const std::vector<Request *> &rs, hipStream_t st) {
    GroupRun &gr = S->grp;
    const Graph *g = S->g;
    const int32_t G = (int32_t)rs.size();
    std::vector<const QueryDesc *> mem(G);
    int64_t sum_RL = 0;
    for (int32_t i = 0; i < G; ++i) {
        QueryDesc &d = gr.desc_host[i];
        d = rs[i]->d;
        d.kind = d.kind == K_STITCHED ? K_GROUPED_STITCHED
                 : d.kind == K_STRAT  ? K_GROUPED_STRAT
                                      : K_GROUPED;
        if (rs[i]->mode == SIMRANK_MODE_STRATIFIED) {
            // the member's class table, staged in pinned memory that the next
            // group rewrites only after this one has finished
            StratParams sp;
            const int rc = strat_params(&rs[i]->q, g->n, &sp, gr.tabs_host + i);
            if (rc) return rc;
            d.z = sp.z;
            d.sa = sp.sa;
            d.sb = sp.sb;
            SRK_HIP(hipMemcpyAsync((void *)d.tab, gr.tabs_host + i, sizeof(StratTab),
                                   hipMemcpyHostToDevice, st));
        }
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
    gr.members = rs;
    gr.busy = true;
    for (int32_t i = 0; i < G; ++i) {
        rs[i]->grouped = true;
        rs[i]->group_size = G;
        rs[i]->group_pos = i;
    }
    return SIMRANK_OK;
}

// The worker.  It alone touches the device, the pool, the ring and the
// staging buffers, and it alone writes a running request's results; the
// mutex guards the queue, the requests' states and the counters.  A waiter
// reads a request's results only after its state, set under the mutex, says
// it ended.
static void server_loop(simrank_server *S) {
    (void)hipSetDevice(S->g->device);
    std::vector<Request *> running;          // admitted, not yet retired
    std::vector<Request *> ended, admitted;
    for (;;) {
        bool progressed = false;
        ended.clear();
        // 1. completions: a lone request's flag, the group's event
        for (Request *r : running) {
            if (r->phase != 1) continue;
            bool finished = false;
            if (r->grouped) {
                const hipError_t e = hipEventQuery(S->grp.ev1);
                if (e == hipSuccess) finished = true;
                else if (e != hipErrorNotReady) {
                    (void)hipGetLastError();
                    r->rc = SIMRANK_EDEVICE;
                    r->err = hipGetErrorString(e);
                    r->phase = 3;
                }
            } else {
                finished = __atomic_load_n(&S->flags_host[r->slot], __ATOMIC_ACQUIRE) == r->seq;
            }
            if (!finished) continue;
            int k = -1;
            for (int i = 0; i < N_STAGING; ++i)
                if (!S->stage[i].busy) {
                    k = i;
                    break;
                }
            if (k < 0) break;                     // all staging sets are copying
            const int rc = start_copy(S, r, k);
            if (rc) {
                r->rc = rc;
                r->err = simrank_last_error();
                r->phase = 3;
            }
            progressed = true;
        }
        // 2. copies done
        for (Request *r : running) {
            if (r->phase == 2) {
                const hipError_t e = hipEventQuery(S->stage[r->stage].ev);
                if (e == hipErrorNotReady) continue;
                if (e == hipSuccess) {
                    finish_copy(S, r);
                } else {
                    (void)hipGetLastError();
                    r->rc = SIMRANK_EDEVICE;
                    r->err = hipGetErrorString(e);
                    S->stage[r->stage].busy = false;
                }
                r->phase = 3;
            }
            if (r->phase == 3) {
                r->t_done = now_s();
                release_request(S, r);
                ended.push_back(r);
            }
        }
        if (!ended.empty()) {
            running.erase(std::remove_if(running.begin(), running.end(),
                                         [](Request *r) { return r->phase == 3; }),
                          running.end());
            if (S->grp.busy) {
                bool any = false;
                for (Request *r : running) any |= r->grouped;
                if (!any) S->grp.busy = false;
            }
        }
        // 3. admission, oldest first, while a ring entry and memory are free
        admitted.clear();
        std::vector<Request *> group;
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
            // With groups, requests that share their walks with a running
            // request wait until it has finished; those that then wait
            // together start as one group (or alone, if only one waits), so
            // that under load the arrivals gather into groups while the
            // device works on the previous ones.
            auto walks_running = [&](const Request *r) {
                for (const Request *o : running)
                    if (same_walks(o, r)) return true;
                return false;
            };
            // set when a group could not get the memory of two members: the
            // requests then go alone, so that a pool too small for two of
            // them cannot keep them waiting for each other for ever
            bool no_room = false;
            if (S->gmax >= 2 && !S->grp.busy) {
                for (Request *head : S->queue) {
                    if (walks_running(head)) continue;
                    for (Request *r : S->queue)
                        if ((int32_t)group.size() < S->gmax && same_walks(head, r)) group.push_back(r);
                    if (group.size() < 2) {
                        group.clear();
                        continue;
                    }
                    size_t kept = 0;
                    for (Request *r : group) {
                        if (!reserve(S, r, false)) break;
                        ++kept;
                    }
                    if (kept < 2) {
                        for (size_t i = 0; i < kept; ++i) {
                            S->alloc.release(group[i]->mem_off, group[i]->mem_bytes);
                            group[i]->mem_bytes = 0;
                            --S->inflight;
                        }
                        group.clear();
                        no_room = true;
                    } else {
                        group.resize(kept);
                        for (Request *r : group)
                            S->queue.erase(std::find(S->queue.begin(), S->queue.end(), r));
                    }
                    break;   // one group in flight at a time
                }
            }
            // lone admission, oldest first; with groups, a request whose walks
            // a running request or a group just formed shares, or that has a
            // partner waiting (unless a group found no room), waits
            for (auto it = S->queue.begin(); it != S->queue.end();) {
                Request *r = *it;
                bool wait = false;
                if (S->gmax >= 2) {
                    wait = walks_running(r);
                    for (const Request *o : group) wait |= same_walks(o, r);
                    if (!no_room)
                        for (const Request *o : S->queue)
                            if (o != r && same_walks(o, r)) {
                                wait = true;
                                break;
                            }
                }
                if (wait) {
                    ++it;
                    continue;
                }
                if (!reserve(S, r, true)) break;
                it = S->queue.erase(it);
                admitted.push_back(r);
            }
            for (Request *r : admitted) r->state = 1;
            for (Request *r : group) r->state = 1;
            if (admitted.empty() && group.empty()) {
                if (S->stop && S->queue.empty() && running.empty()) break;
                if (!progressed) {
                    if (running.empty() && S->queue.empty())
                        S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
                    else
                        S->cv_work.wait_for(lk, std::chrono::microseconds(50));
                }
                continue;
            }
        }
        // 4. enqueue on the device, without the mutex
        const double t = now_s();
        bool kinds[N_KINDS] = {false, false, false};
        std::vector<Request *> failed;
        for (Request *r : admitted) {
            r->t_start = t;
            const int rc = prepare(S, r);
            if (rc) {
                r->rc = rc;
                r->err = simrank_last_error();
                failed.push_back(r);
                continue;
            }
            r->phase = 1;
            kinds[kind_of(r->mode)] = true;
            running.push_back(r);
        }
        int rc_launch = SIMRANK_OK;
        if (!admitted.empty() && (kinds[0] || kinds[1] || kinds[2])) {
            // one persistent meet kernel per kind admitted, after the
            // preparations, on the next worker stream
            hipStream_t ws = S->work[S->next_work];
            S->next_work ^= 1;
            hipError_t e = hipEventRecord(S->ev_prep, S->prep);
            if (e == hipSuccess) e = hipStreamWaitEvent(ws, S->ev_prep, 0);
            if (e != hipSuccess) rc_launch = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
            for (int k = 0; k < N_KINDS && !rc_launch; ++k)
                if (kinds[k]) {
                    rc_launch = launch_ring_meet(k, S->ring, ws);
                    ++S->n_launches;
                }
        }
        if (!group.empty()) {
            for (Request *r : group) r->t_start = t;
            hipStream_t ws = S->work[S->next_work];
            S->next_work ^= 1;
            const int rc = launch_group(S, group, ws);
            if (rc) {
                (void)hipStreamSynchronize(ws);
                for (Request *r : group) {
                    r->rc = rc;
                    r->err = simrank_last_error();
                    failed.push_back(r);
                }
            } else {
                for (Request *r : group) {
                    r->phase = 1;
                    running.push_back(r);
                }
                ++S->n_launches;
            }
        }
        if (rc_launch) {
            // a launch failed: the published requests of this round cannot
            // be relied on; fail them after their preparation has finished
            (void)hipStreamSynchronize(S->prep);
            for (Request *r : admitted)
                if (r->phase == 1) {
                    r->rc = rc_launch;
                    r->err = simrank_last_error();
                    r->phase = 3;
                }
        }
        for (Request *r : failed) {
            r->t_done = now_s();
            release_request(S, r);
        }
        {
            std::lock_guard<std::mutex> lk(S->mu);
            for (Request *r : failed) {
                r->state = 3;
                ++S->n_failed;
            }
            if (!group.empty() && failed.empty()) {
                ++S->n_groups;
                S->n_grouped += group.size();
            }
            if (!failed.empty()) S->cv_done.notify_all();
        }
    }
}

static void server_release(simrank_server *S) {
    if (S->prep) (void)hipStreamSynchronize(S->prep);
    for (hipStream_t w : S->work)
        if (w) (void)hipStreamSynchronize(w);
    if (S->copy) (void)hipStreamSynchronize(S->copy);
    GroupRun &gr = S->grp;
    if (gr.desc_host) (void)hipHostFree(gr.desc_host);
    if (gr.tabs_host) (void)hipHostFree(gr.tabs_host);
    if (gr.gdesc_host) (void)hipHostFree(gr.gdesc_host);
    device_free(gr.desc_dev);
    device_free(gr.gdesc_dev);
    device_free(gr.units);
    device_free(gr.gunits);
    device_free(gr.counters);
    device_free(gr.buffers);
    if (gr.ev0) (void)hipEventDestroy(gr.ev0);
    if (gr.ev1) (void)hipEventDestroy(gr.ev1);
    for (Staging &sg : S->stage) {
        if (sg.out) (void)hipHostFree(sg.out);
        if (sg.out_n) (void)hipHostFree(sg.out_n);
        if (sg.cnt) (void)hipHostFree(sg.cnt);
        if (sg.wsum) (void)hipHostFree(sg.wsum);
        if (sg.ctr) (void)hipHostFree(sg.ctr);
        if (sg.ev) (void)hipEventDestroy(sg.ev);
    }
    device_free(S->pool);
    device_free(S->ring.desc);
    device_free(S->ring.ctl);
    device_free(S->ring.counters);
    if (S->flags_host) (void)hipHostFree(S->flags_host);
    if (S->tabs_host) (void)hipHostFree(S->tabs_host);
    if (S->ev_prep) (void)hipEventDestroy(S->ev_prep);
    for (hipStream_t st : {S->prep, S->copy, S->work[0], S->work[1]})
        if (st) (void)hipStreamDestroy(st);
    for (auto &kv : S->all) delete kv.second;
    delete S;
}

extern "C" int simrank_server_create(simrank_graph *g, const simrank_server_params *p,
                                     simrank_server **out) {
    clear_error();
    if (!g || !p || !out) return fail(SIMRANK_EINVAL, "NULL argument");
    *out = nullptr;
    if (p->max_slots < 1 || p->max_slots > RING_MAX)
        return fail(SIMRANK_EINVAL, "max_slots must lie in [1, 64]");
    if (p->max_R < 1 || p->max_R > MAX_R) return fail(SIMRANK_EINVAL, "max_R must lie in [1, 2^24]");
    if (p->max_L < 1 || p->max_L > MAX_CAP) return fail(SIMRANK_EINVAL, "max_L must lie in [1, 255]");
    if (p->group_max < 0 || p->group_max > GROUP_MAX)
        return fail(SIMRANK_EINVAL, "group_max must lie in [0, 32]");
    SRK_HIP(hipSetDevice(g->device));
    simrank_server *S = new simrank_server();
    S->g = g;
    S->prm = *p;
    simrank_params big{p->max_R, p->max_L, 0u, 0};
    S->slot_bytes = (int64_t)request_bytes(big, SIMRANK_MODE_PLAIN, g->n);
    size_t free_b = 0, tot_b = 0;
    SRK_HIP(hipMemGetInfo(&free_b, &tot_b));
    const int64_t budget = p->hbm_budget > 0 ? std::min<int64_t>(p->hbm_budget, (int64_t)free_b)
                                             : (int64_t)(free_b / 2);
    if (budget < S->slot_bytes) {
        delete S;
        return fail(SIMRANK_ENOMEM, "device-memory budget admits no request of " +
                                        std::to_string(S->slot_bytes) + " bytes");
    }
    const int64_t pool_bytes = std::min<int64_t>(budget, (int64_t)p->max_slots * S->slot_bytes);
    S->entries = p->max_slots;
    S->slot_req.assign(S->entries, nullptr);
    int rc = SIMRANK_OK;
    auto hip = [&](hipError_t e) {
        if (!rc && e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    };
    rc = device_alloc((void **)&S->pool, (size_t)pool_bytes, nullptr);
    if (!rc) S->alloc = PoolAlloc((size_t)pool_bytes);
    if (!rc) rc = device_alloc((void **)&S->ring.desc, sizeof(QueryDesc) * RING_MAX, nullptr);
    if (!rc) rc = device_alloc((void **)&S->ring.ctl, sizeof(RingCtl) * RING_MAX, nullptr);
    if (!rc) rc = device_alloc((void **)&S->ring.counters, 64 * RING_MAX, nullptr);
    if (!rc) hip(hipMemset(S->ring.ctl, 0, sizeof(RingCtl) * RING_MAX));
    if (!rc) hip(hipHostMalloc((void **)&S->flags_host, 4 * RING_MAX, hipHostMallocCoherent));
    if (!rc) std::memset(S->flags_host, 0, 4 * RING_MAX);
    if (!rc) hip(hipHostMalloc((void **)&S->tabs_host, sizeof(StratTab) * RING_MAX, hipHostMallocDefault));
    S->ring.flags = S->flags_host;
    S->ring.entries = S->entries;
    for (hipStream_t *st : {&S->prep, &S->copy, &S->work[0], &S->work[1]})
        hip(hipStreamCreateWithFlags(st, hipStreamNonBlocking));
    hip(hipEventCreateWithFlags(&S->ev_prep, hipEventDisableTiming));
    const size_t n = (size_t)g->n;
    for (Staging &sg : S->stage) {
        hip(hipHostMalloc((void **)&sg.out, 8 * n, hipHostMallocDefault));
        hip(hipHostMalloc((void **)&sg.out_n, 8 * n, hipHostMallocDefault));
        hip(hipHostMalloc((void **)&sg.cnt, 4 * n, hipHostMallocDefault));
        hip(hipHostMalloc((void **)&sg.wsum, 8 * n, hipHostMallocDefault));
        hip(hipHostMalloc((void **)&sg.ctr, 64, hipHostMallocDefault));
        hip(hipEventCreateWithFlags(&sg.ev, hipEventDisableTiming));
    }
    int32_t gmax = std::min<int32_t>(p->group_max, p->max_slots);
    // a group's packed positions are addressed in 32 bits
    while (gmax >= 2 &&
           group_pos_words(p->max_R, (int64_t)gmax * p->max_R * p->max_L, p->max_L) >= (int64_t)0xffff0000)
        --gmax;
    S->gmax = gmax;
    if (!rc && gmax >= 2) {   // the group's own buffers
        GroupRun &gr = S->grp;
        // the buffers of the largest group of any walks and size (stratified
        // groups have the smaller tiles, so the most of them)
        size_t gb = 0;
        for (int32_t wk = 0; wk < 3; ++wk)
            for (int32_t G = 2; G <= gmax; ++G) {
                GroupDesc gd{};
                gd.Rmax = p->max_R;
                gd.L = p->max_L;
                gd.G = G;
                gd.gw = (G + 3) / 4;
                gd.wk = wk;
                gb = std::max(gb, group_buffers(&gd, (int64_t)G * p->max_R * p->max_L, nullptr));
            }
        rc = device_alloc((void **)&gr.buffers, gb, nullptr);
        if (!rc) rc = device_alloc((void **)&gr.desc_dev, sizeof(QueryDesc) * gmax, nullptr);
        if (!rc) rc = device_alloc((void **)&gr.gdesc_dev, sizeof(GroupDesc), nullptr);
        if (!rc) rc = device_alloc((void **)&gr.units, 4 * units_words(gmax), nullptr);
        if (!rc) rc = device_alloc((void **)&gr.gunits, 4 * group_units_words(1), nullptr);
        if (!rc) rc = device_alloc((void **)&gr.counters, 8 * 8, nullptr);
        hip(hipHostMalloc((void **)&gr.desc_host, sizeof(QueryDesc) * gmax, hipHostMallocDefault));
        hip(hipHostMalloc((void **)&gr.gdesc_host, sizeof(GroupDesc), hipHostMallocDefault));
        hip(hipHostMalloc((void **)&gr.tabs_host, sizeof(StratTab) * gmax, hipHostMallocDefault));
        hip(hipEventCreate(&gr.ev0));
        hip(hipEventCreate(&gr.ev1));
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
    if (slots)
        *slots = (int32_t)std::min<int64_t>(S->entries, (int64_t)S->alloc.total() / S->slot_bytes);
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

extern "C" int simrank_server_load(simrank_server *S, int32_t *inflight_peak, int64_t *pool_bytes,
                                   int64_t *pool_peak, uint64_t *launches) {
    clear_error();
    if (!S) return fail(SIMRANK_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(S->mu);
    if (inflight_peak) *inflight_peak = S->inflight_peak;
    if (pool_bytes) *pool_bytes = (int64_t)S->alloc.total();
    if (pool_peak) *pool_peak = (int64_t)S->alloc.peak();
    if (launches) *launches = S->n_launches;
    return SIMRANK_OK;
}

extern "C" int simrank_server_submit(simrank_server *S, const simrank_query *q, uint64_t *ticket) {
    clear_error();
    if (!S || !q || !ticket) return fail(SIMRANK_EINVAL, "NULL argument");
    Request *r = new Request();
    r->q = *q;
    int rc = query_params(q, S->g->n, &r->p, &r->mode);
    if (!rc && (q->s < 0 || q->s >= S->g->n)) rc = fail(SIMRANK_EINVAL, "source out of range");
    if (!rc && (r->p.R > S->prm.max_R || r->p.L > S->prm.max_L))
        rc = fail(SIMRANK_EINVAL, "query needs R or L beyond the server's maximum");
    if (!rc && r->mode == SIMRANK_MODE_STRATIFIED) {
        StratParams sp;
        rc = strat_params(q, S->g->n, &sp, nullptr);
        if (!rc) std::memcpy(&r->zbits, &sp.z, sizeof(r->zbits));
    }
    if (!rc && r->mode == SIMRANK_MODE_STITCHED && (!S->g->index || S->g->index->T != r->p.T))
        rc = fail(SIMRANK_ESTATE, "stitched query without a matching index");
    if (!rc) {
        const int64_t units = (int64_t)max_tiles_for(r->p.R, r->p.L) *
                              ((S->g->n_active + default_unit_nodes(S->g) - 1) / default_unit_nodes(S->g));
        if (units >= (int64_t)0x7fffffff) rc = fail(SIMRANK_EINVAL, "R * L * n too large for one request");
    }
    if (!rc && (int64_t)request_bytes(r->p, r->mode, S->g->n) > (int64_t)S->alloc.total())
        rc = fail(SIMRANK_ENOMEM, "the request needs more device memory than the server's budget");
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

extern "C" int simrank_server_poll(simrank_server *S, uint64_t ticket, int32_t *state) {
    clear_error();
    if (!S || !state) return fail(SIMRANK_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(SIMRANK_EINVAL, "unknown ticket");
    *state = std::min(it->second->state, 2);
    return SIMRANK_OK;
}

// Waits for the request and retires its ticket; the results stay with the
// returned request, which the caller deletes.
static int wait_request(simrank_server *S, uint64_t ticket, double timeout_s, bool stratified,
                        Request **out) {
    std::unique_lock<std::mutex> lk(S->mu);
    auto it0 = S->all.find(ticket);
    if (it0 == S->all.end()) return fail(SIMRANK_EINVAL, "unknown ticket");
    if ((it0->second->mode == SIMRANK_MODE_STRATIFIED) != stratified)
        return fail(SIMRANK_EINVAL, stratified ? "not a stratified request: use simrank_server_wait"
                                               : "stratified request: use simrank_server_wait_stratified");
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
    *out = it->second;
    S->all.erase(it);
    return SIMRANK_OK;
}

static void fill_info(const Request *r, simrank_request_info *info) {
    if (!info) return;
    info->queue_s = r->t_start - r->t_submit;
    info->latency_s = r->t_done - r->t_submit;
    info->stats = r->st;
}

extern "C" int simrank_server_wait(simrank_server *S, uint64_t ticket, double timeout_s,
                                   double *out_host, uint32_t *counts_host,
                                   simrank_request_info *info) {
    clear_error();
    if (!S) return fail(SIMRANK_EINVAL, "server is NULL");
    Request *r = nullptr;
    int rc = wait_request(S, ticket, timeout_s, false, &r);
    if (rc) return rc;
    if (r->state == 3) {
        rc = fail(r->rc, r->err);
    } else {
        const size_t n = (size_t)S->g->n;
        if (out_host) std::copy(r->out.begin(), r->out.begin() + n, out_host);
        if (counts_host) std::copy(r->cnt.begin(), r->cnt.begin() + n, counts_host);
        fill_info(r, info);
    }
    delete r;
    return rc;
}

extern "C" int simrank_server_wait_stratified(simrank_server *S, uint64_t ticket, double timeout_s,
                                              double *out_host, double *out_n_host,
                                              uint64_t *wsum_host, simrank_request_info *info) {
    clear_error();
    if (!S) return fail(SIMRANK_EINVAL, "server is NULL");
    Request *r = nullptr;
    int rc = wait_request(S, ticket, timeout_s, true, &r);
    if (rc) return rc;
    if (r->state == 3) {
        rc = fail(r->rc, r->err);
    } else {
        const size_t n = (size_t)S->g->n;
        if (out_host) std::copy(r->out.begin(), r->out.begin() + n, out_host);
        if (out_n_host) std::copy(r->out_n.begin(), r->out_n.begin() + n, out_n_host);
        if (wsum_host) std::copy(r->wsum.begin(), r->wsum.begin() + n, wsum_host);
        fill_info(r, info);
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
