// Serving: a request loop over one device-resident graph (and its index).
//
// Requests are queued by simrank_server_submit and admitted by a worker thread
// into slots as slots free up.  A slot is a workspace, device buffers for the
// estimate and the counts, pinned host buffers and its own stream; the number
// of slots is what the device-memory budget admits.  An admitted request is
// enqueued whole on its slot's stream (query kernels, then the copy of its
// results to the slot's pinned buffers, then an event), so requests that arrive
// while others run are started as soon as a slot is free and their kernels
// overlap on the device.  Each result equals the lone query's.
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
    Workspace ws;
    double *out_dev = nullptr;
    uint32_t *cnt_dev = nullptr;
    double *out_host = nullptr;     // pinned
    uint32_t *cnt_host = nullptr;   // pinned
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Request *req = nullptr;
};

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
    uint64_t n_done = 0, n_failed = 0, max_inflight = 0;
};

static void server_loop(simrank_server *S) {
    (void)hipSetDevice(S->g->device);
    std::unique_lock<std::mutex> lk(S->mu);
    while (true) {
        bool progressed = false;
        // completions
        uint64_t inflight = 0;
        for (Slot &sl : S->slots) {
            if (!sl.req) continue;
            const hipError_t e = hipEventQuery(sl.done);
            if (e == hipErrorNotReady) {
                ++inflight;
                continue;
            }
            Request *r = sl.req;
            r->t_done = now_s();
            if (e == hipSuccess) {
                const size_t n = (size_t)S->g->n;
                r->out.assign(sl.out_host, sl.out_host + n);
                r->cnt.assign(sl.cnt_host, sl.cnt_host + n);
                unsigned long long c[8];
                hipError_t e2 = hipMemcpy(c, sl.ws.counters, sizeof(c), hipMemcpyDeviceToHost);
                float ms = 0.f, mms = 0.f;
                if (e2 == hipSuccess) e2 = hipEventElapsedTime(&ms, sl.ws.ev0, sl.ws.ev1);
                if (e2 == hipSuccess) e2 = hipEventElapsedTime(&mms, sl.ws.evm0, sl.ws.evm1);
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
                r->state = 2;
                ++S->n_done;
            } else {
                (void)hipGetLastError();
                r->state = 3;
                r->rc = SIMRANK_EDEVICE;
                r->err = hipGetErrorString(e);
                ++S->n_failed;
            }
            sl.req = nullptr;
            progressed = true;
        }
        if (progressed) S->cv_done.notify_all();
        // admissions
        for (Slot &sl : S->slots) {
            if (S->queue.empty()) break;
            if (sl.req) continue;
            Request *r = S->queue.front();
            S->queue.pop_front();
            r->t_start = now_s();
            int rc = enqueue_query(S->g, &r->q, r->p, r->mode, &sl.ws, sl.out_dev, sl.cnt_dev,
                                   sl.stream);
            const size_t n = (size_t)S->g->n;
            hipError_t e = hipSuccess;
            if (!rc) e = hipMemcpyAsync(sl.out_host, sl.out_dev, 8 * n, hipMemcpyDeviceToHost,
                                        sl.stream);
            if (!rc && e == hipSuccess)
                e = hipMemcpyAsync(sl.cnt_host, sl.cnt_dev, 4 * n, hipMemcpyDeviceToHost, sl.stream);
            if (!rc && e == hipSuccess) e = hipEventRecord(sl.done, sl.stream);
            if (rc || e != hipSuccess) {
                r->state = 3;
                r->rc = rc ? rc : SIMRANK_EDEVICE;
                r->err = rc ? simrank_last_error() : hipGetErrorString(e);
                r->t_done = now_s();
                ++S->n_failed;
                S->cv_done.notify_all();
                continue;
            }
            r->state = 1;
            sl.req = r;
            ++inflight;
            progressed = true;
        }
        if (inflight > S->max_inflight) S->max_inflight = inflight;
        if (S->stop && S->queue.empty() && inflight == 0) break;
        if (!progressed) {
            if (inflight == 0 && S->queue.empty())
                S->cv_work.wait(lk, [&] { return S->stop || !S->queue.empty(); });
            else
                S->cv_work.wait_for(lk, std::chrono::microseconds(50));
        }
    }
}

static void server_release(simrank_server *S) {
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
    auto it = S->all.find(ticket);
    if (it == S->all.end()) return fail(SIMRANK_EINVAL, "unknown ticket");
    Request *r = it->second;
    auto finished = [&] { return r->state >= 2; };
    if (timeout_s < 0) {
        S->cv_done.wait(lk, finished);
    } else if (!S->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), finished)) {
        return fail(SIMRANK_ESTATE, "request not finished");
    }
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
