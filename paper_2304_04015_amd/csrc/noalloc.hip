// A single-source query that allocates nothing: simrank_single_source_noalloc.
//
// It runs the same launch sequence as simrank_single_source_async (source
// walks, compaction, the fused walk + meet + count kernel, the estimate), but
// its per-query scratch (source walks and their compacted copy, tile table,
// descriptor, unit table, counters) lives in `scratch`, a file-scope device
// array of fixed size that every GPU the library runs on holds until the
// process ends.  The caller passes the graph, the query, device outputs and a
// stream; the call makes no hipMalloc, hipFree or other allocation, so it can
// be used where allocation is not allowed.
//
// In host code the array's name is only a host-side stand-in for the symbol;
// the device address of each GPU's copy comes from hipGetSymbolAddress, taken
// once per device on the entry point's first call there (with that device
// current) and kept in `scratch_dev`.  Only that address is ever handed to
// kernels.  Every call on one GPU shares its copy: the kernels clear what must
// start at zero (counters, unit cursors) and write every other piece before
// reading it, and calls that overlap on one GPU race.
#include <mutex>

#include "common.hpp"

namespace srk {
namespace {

// Largest query the scratch holds.
constexpr int64_t NOALLOC_MAX_R = 1 << 16;     // walks per node
constexpr int64_t NOALLOC_MAX_RL = 1 << 20;    // R * L source-walk positions

constexpr size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Tiles of any query within the limits, at most (the bound of max_tiles_for
// with the smallest tile: 2048 walks, 8192 - L positions, L <= 255).
constexpr int64_t NOALLOC_MAX_TILES =
    2 + NOALLOC_MAX_R / MIN_TILE_J + NOALLOC_MAX_RL / (8192 - MAX_CAP) + 1;

// The pieces, in carving order.
struct Carve {
    uint32_t *sw, *swc, *jj, *joff, *tiles, *meta, *units;
    uint8_t *slen;
    unsigned long long *counters;
    QueryDesc *desc;
};

constexpr size_t NOALLOC_BYTES =
    align256(4 * NOALLOC_MAX_RL) +                      // sw
    align256(4 * NOALLOC_MAX_RL) +                      // swc
    align256(4 * NOALLOC_MAX_R) +                       // jj
    align256(4 * (NOALLOC_MAX_R + 1)) +                 // joff
    align256(4 * (NOALLOC_MAX_TILES + 1)) +             // tiles
    align256(4 * 8) +                                   // meta
    align256(4 * (N_KINDS * 2 + N_KINDS)) +             // units (units_words(1))
    align256(NOALLOC_MAX_R) +                           // slen
    align256(8 * 8) +                                   // counters
    align256(sizeof(QueryDesc));                        // desc

Carve carve(char *base) {
    Carve c{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        char *p = base + off;
        off += align256(bytes);
        return p;
    };
    c.sw = (uint32_t *)take(4 * NOALLOC_MAX_RL);
    c.swc = (uint32_t *)take(4 * NOALLOC_MAX_RL);
    c.jj = (uint32_t *)take(4 * NOALLOC_MAX_R);
    c.joff = (uint32_t *)take(4 * (NOALLOC_MAX_R + 1));
    c.tiles = (uint32_t *)take(4 * (NOALLOC_MAX_TILES + 1));
    c.meta = (uint32_t *)take(4 * 8);
    c.units = (uint32_t *)take(4 * units_words(1));
    c.slen = (uint8_t *)take(NOALLOC_MAX_R);
    c.counters = (unsigned long long *)take(8 * 8);
    c.desc = (QueryDesc *)take(sizeof(QueryDesc));
    return c;
}

__global__ void k_put_desc(QueryDesc *dst, QueryDesc d) { *dst = d; }

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
char *scratch_dev[MAX_DEVICES] = {};

}  // namespace

// The allocation-free call's scratch, one copy per GPU (see the top of the file).
static __device__ __align__(256) unsigned char scratch[NOALLOC_BYTES];

namespace {

// Device address of the current device's scratch (looked up once per device).
int scratch_of(int dev, char **out) {
    if (dev < 0 || dev >= MAX_DEVICES) return fail(SIMRANK_EDEVICE, "device ordinal beyond 63");
    std::lock_guard<std::mutex> lk(scratch_mu);
    if (!scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(SIMRANK_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                             hipGetErrorString(e));
        scratch_dev[dev] = (char *)p;
    }
    *out = scratch_dev[dev];
    return SIMRANK_OK;
}

}  // namespace
}  // namespace srk

using namespace srk;

extern "C" int simrank_single_source_noalloc(const simrank_graph *g, const simrank_query *q,
                                             double *out_dev, uint32_t *counts_dev, void *stream) {
    clear_error();
    if (!g || !q) return fail(SIMRANK_EINVAL, "NULL argument");
    if (!counts_dev) return fail(SIMRANK_EINVAL, "counts buffer is NULL");
    simrank_params p;
    int mode;
    int rc = query_params(q, g->n, &p, &mode);
    if (rc) return rc;
    if (q->s < 0 || q->s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
    if (mode == SIMRANK_MODE_STRATIFIED)
        return fail(SIMRANK_EINVAL, "stratified queries are not taken by the allocation-free call");
    if (p.R > NOALLOC_MAX_R)
        return fail(SIMRANK_EINVAL, "R = " + std::to_string(p.R) + " exceeds the allocation-free "
                                    "call's limit of 65536 walks per node");
    if ((int64_t)p.R * p.L > NOALLOC_MAX_RL)
        return fail(SIMRANK_EINVAL, "R * L = " + std::to_string((int64_t)p.R * p.L) +
                                        " exceeds the allocation-free call's limit of 2^20");
    const bool stitched = mode == SIMRANK_MODE_STITCHED;
    if (stitched && !g->index) return fail(SIMRANK_ESTATE, "stitched query without an index");
    if (stitched && g->index->T != p.T)
        return fail(SIMRANK_EINVAL, "stitched query's c differs from the index's c");
    SRK_HIP(hipSetDevice(g->device));
    char *base = nullptr;
    if ((rc = scratch_of(g->device, &base))) return rc;
    const Carve c = carve(base);

    QueryDesc d;
    describe_query(g, q, p, mode, default_unit_nodes(g), &d);
    d.sw = c.sw;
    d.slen = c.slen;
    d.jj = c.jj;
    d.joff = c.joff;
    d.swc = c.swc;
    d.tiles = c.tiles;
    d.meta = c.meta;
    d.cnt = counts_dev;
    d.out = out_dev;
    // the meet kernel counts work units (tile x node chunk) in 32 bits
    const int64_t units_bound = (int64_t)max_tiles_for(d.R, d.L) * d.n_chunks;
    if (units_bound >= (int64_t)0xffffffffu - (1 << 20))
        return fail(SIMRANK_EINVAL, "R * L * n too large for one launch");
    QuerySet qs;
    qs.desc = c.desc;
    qs.nq = 1;
    qs.max_R = d.R;
    qs.max_n = g->n;
    qs.units_bound[d.kind] = units_bound;
    qs.units = c.units;
    qs.counters = c.counters;
    hipStream_t st = (hipStream_t)stream;
    k_put_desc<<<1, 1, 0, st>>>(c.desc, d);
    SRK_HIP(hipGetLastError());
    return launch_query_set(qs, st, nullptr, nullptr);
}
