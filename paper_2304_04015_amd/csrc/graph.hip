// Graph ingest: the in-edge CSR of G (the reversed graph the walks run on,
// Algorithm 1 "reverse the edges") becomes the library's gather layout.
//
//   nodes[v] = (o(v), deg(v)),  o(v) = sum_{u < v} max(deg(u), 1)
//   E[o(v) + k] = nodes[in_src[in_off[v] + k]]      for k < deg(v)
//   node_of[o(v)] = v
//   E[o(v)] = (NIL, NIL) for a node without in-neighbours (never read by a walk)
//
// A walk at (o, d) picks k < d and reads E[o + k]: one 8-byte gather gives
// the next node's identity o and its degree, so a move never needs a second,
// dependent gather of a row array.  Edge order inside a row is preserved, so
// the k-th in-neighbour is the same as in the caller's CSR.
#include <vector>

#include "common.hpp"

namespace srk {
namespace {

__global__ void k_slot_counts(const int32_t *__restrict__ off, int32_t n,
                              uint32_t *__restrict__ slots, uint32_t *__restrict__ has_in) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t d = off[v + 1] - off[v];
    slots[v] = d > 0 ? (uint32_t)d : 1u;
    has_in[v] = d > 0 ? 1u : 0u;
}

__global__ void k_nodes(const int32_t *__restrict__ off, const int64_t *__restrict__ o, int32_t n,
                        const int64_t *__restrict__ act_pos, uint2 *__restrict__ nodes,
                        uint32_t *__restrict__ node_of, int32_t *__restrict__ active) {
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= n) return;
    const int32_t d = off[v + 1] - off[v];
    nodes[v] = make_uint2((uint32_t)o[v], (uint32_t)d);
    node_of[o[v]] = (uint32_t)v;
    if (d > 0) active[act_pos[v]] = (int32_t)v;
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t n, uint32_t val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

// One thread per edge; the owning row is found by binary search over in_off.
// dbar[u] counts the rows that list u (the pool sizes of the stitched index
// follow it).
__global__ void k_edges(const int32_t *__restrict__ off, const int32_t *__restrict__ src,
                        int32_t n, int64_t m, const uint2 *__restrict__ nodes,
                        uint2 *__restrict__ E, uint32_t *__restrict__ dbar) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= m) return;
    int32_t lo = 0, hi = n;  // find v with off[v] <= e < off[v+1]
    while (hi - lo > 1) {
        const int32_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)off[mid] <= e) lo = mid; else hi = mid;
    }
    // the largest v with off[v] <= e is the row holding e (empty rows before it
    // share its offset and lose the search)
    const int32_t v = lo;
    const uint2 row = nodes[v];
    const int32_t u = src[e];
    E[(int64_t)row.x + (e - off[v])] = nodes[u];
    atomicAdd(&dbar[u], 1u);
}

}  // namespace

int device_alloc(void **p, size_t bytes, int64_t *acct) {
    *p = nullptr;
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(SIMRANK_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                        hipGetErrorString(e));
    }
    if (acct) *acct += (int64_t)bytes;
    return SIMRANK_OK;
}

void device_free(void *p) {
    if (p) (void)hipFree(p);
}

static void graph_release(simrank_graph *g) {
    if (!g) return;
    if (g->index) {
        index_free(g->index);
        delete g->index;
        g->index = nullptr;
    }
    device_free(g->nodes);
    device_free(g->E);
    device_free(g->node_of);
    device_free(g->active);
    device_free(g->dbar);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

}  // namespace srk

using namespace srk;


extern "C" int simrank_load_graph(int32_t n, int64_t m, const int32_t *in_off,
                                  const int32_t *in_src, simrank_graph **g_out) {
    clear_error();
    if (!g_out) return fail(SIMRANK_EINVAL, "g_out is NULL");
    *g_out = nullptr;
    if (!in_off || (m > 0 && !in_src)) return fail(SIMRANK_EINVAL, "NULL CSR array");
    if (n < 1) return fail(SIMRANK_EINVAL, "n must be >= 1");
    if (m < 0 || m + (int64_t)n >= (int64_t)0x7fffffff)
        return fail(SIMRANK_EINVAL, "need 0 <= m and m + n < 2^31");
    // Host-side validation of the CSR (the copy below trusts it).
    if (in_off[0] != 0) return fail(SIMRANK_EINVAL, "in_off[0] must be 0");
    int32_t max_deg = 0;
    int32_t n_active = 0;
    for (int32_t v = 0; v < n; ++v) {
        const int64_t d = (int64_t)in_off[v + 1] - in_off[v];
        if (d < 0) return fail(SIMRANK_EINVAL, "in_off decreases at row " + std::to_string(v));
        if (d > max_deg) max_deg = (int32_t)d;
        n_active += d > 0;
    }
    if ((int64_t)in_off[n] != m) return fail(SIMRANK_EINVAL, "in_off[n] != m");
    for (int64_t e = 0; e < m; ++e)
        if (in_src[e] < 0 || in_src[e] >= n)
            return fail(SIMRANK_EINVAL, "in_src[" + std::to_string(e) + "] out of range");

    simrank_graph *g = new simrank_graph();
    g->n = n;
    g->m = m;
    g->max_deg = max_deg;
    g->n_active = n_active;
    g->m_slots = m + (int64_t)(n - n_active);
    int rc;
    int32_t *d_off = nullptr, *d_src = nullptr;
    uint32_t *d_slots = nullptr, *d_has = nullptr;
    int64_t *d_o = nullptr, *d_apos = nullptr, *d_tot = nullptr;
#define SRK_TRY(x)                     \
    do {                               \
        rc = (x);                      \
        if (rc != SIMRANK_OK) goto bad; \
    } while (0)
#define SRK_TRYHIP(x)                                                            \
    do {                                                                         \
        hipError_t e_ = (x);                                                     \
        if (e_ != hipSuccess) {                                                  \
            rc = fail(SIMRANK_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
            goto bad;                                                            \
        }                                                                        \
    } while (0)
    {
        SRK_TRYHIP(hipGetDevice(&g->device));
        SRK_TRYHIP(hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking));
        hipStream_t st = g->stream;
        SRK_TRY(device_alloc((void **)&g->nodes, sizeof(uint2) * (size_t)n, &g->bytes));
        SRK_TRY(device_alloc((void **)&g->E, sizeof(uint2) * (size_t)g->m_slots, &g->bytes));
        SRK_TRY(device_alloc((void **)&g->node_of, sizeof(uint32_t) * (size_t)g->m_slots,
                             &g->bytes));
        SRK_TRY(device_alloc((void **)&g->active, sizeof(int32_t) * (size_t)(n_active ? n_active : 1),
                             &g->bytes));
        SRK_TRY(device_alloc((void **)&g->dbar, sizeof(uint32_t) * (size_t)n, &g->bytes));
        SRK_TRY(device_alloc((void **)&d_off, sizeof(int32_t) * (size_t)(n + 1), nullptr));
        SRK_TRY(device_alloc((void **)&d_src, sizeof(int32_t) * (size_t)(m ? m : 1), nullptr));
        SRK_TRY(device_alloc((void **)&d_slots, sizeof(uint32_t) * (size_t)n, nullptr));
        SRK_TRY(device_alloc((void **)&d_has, sizeof(uint32_t) * (size_t)n, nullptr));
        SRK_TRY(device_alloc((void **)&d_o, sizeof(int64_t) * (size_t)n, nullptr));
        SRK_TRY(device_alloc((void **)&d_apos, sizeof(int64_t) * (size_t)n, nullptr));
        SRK_TRY(device_alloc((void **)&d_tot, sizeof(int64_t) * 2, nullptr));
        SRK_TRYHIP(hipMemcpyAsync(d_off, in_off, sizeof(int32_t) * (size_t)(n + 1),
                                  hipMemcpyHostToDevice, st));
        if (m) SRK_TRYHIP(hipMemcpyAsync(d_src, in_src, sizeof(int32_t) * (size_t)m,
                                         hipMemcpyHostToDevice, st));
        k_slot_counts<<<grid_for(n, 256), 256, 0, st>>>(d_off, n, d_slots, d_has);
        SRK_TRY(scan_exclusive_u32_to_i64(d_slots, n, d_o, d_tot, st));
        SRK_TRY(scan_exclusive_u32_to_i64(d_has, n, d_apos, d_tot + 1, st));
        k_fill_u32<<<1024, 256, 0, st>>>(g->node_of, g->m_slots, NIL);
        k_fill_u32<<<1024, 256, 0, st>>>((uint32_t *)g->E, 2 * g->m_slots, NIL);
        k_fill_u32<<<1024, 256, 0, st>>>(g->dbar, n, 0u);
        k_nodes<<<grid_for(n, 256), 256, 0, st>>>(d_off, d_o, n, d_apos, g->nodes, g->node_of,
                                                   g->active);
        if (m) k_edges<<<grid_for(m, 256), 256, 0, st>>>(d_off, d_src, n, m, g->nodes, g->E,
                                                        g->dbar);
        SRK_TRYHIP(hipGetLastError());
        int64_t tot[2];
        SRK_TRYHIP(hipMemcpyAsync(tot, d_tot, sizeof(tot), hipMemcpyDeviceToHost, st));
        SRK_TRYHIP(hipStreamSynchronize(st));
        if (tot[0] != g->m_slots || tot[1] != n_active) {
            rc = fail(SIMRANK_EDEVICE, "ingest totals disagree with the host count");
            goto bad;
        }
    }
    device_free(d_off); device_free(d_src); device_free(d_slots); device_free(d_has);
    device_free(d_o); device_free(d_apos); device_free(d_tot);
    *g_out = g;
    return SIMRANK_OK;
bad:
    device_free(d_off); device_free(d_src); device_free(d_slots); device_free(d_has);
    device_free(d_o); device_free(d_apos); device_free(d_tot);
    graph_release(g);
    return rc;
#undef SRK_TRY
#undef SRK_TRYHIP
}

extern "C" int simrank_free_graph(simrank_graph *g) {
    clear_error();
    if (!g) return SIMRANK_OK;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    graph_release(g);
    return SIMRANK_OK;
}

extern "C" int simrank_graph_info(const simrank_graph *g, int32_t *n, int64_t *m,
                                  int32_t *n_active, int64_t *device_bytes) {
    clear_error();
    if (!g) return fail(SIMRANK_EINVAL, "graph is NULL");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (n_active) *n_active = g->n_active;
    if (device_bytes) *device_bytes = g->bytes + (g->index ? g->index->bytes : 0);
    return SIMRANK_OK;
}
