// Algorithm 2's tuple form of meet detection, for up to 32 sources at once.
//
// Section 3.2 and Algorithm 2: every walk is decomposed into one tuple per
// step after its start, (j, i, node, start); the tuples are sorted on
// (j, i, node) with the sources' tuples first among equal keys; each other
// tuple is linked to the closest source tuple before it (PREDECESSOR), and an
// equal (j, i, node) is a meet of walk j of that source and walk j of the
// tuple's start node, counted once per pair.
//
// On one GPU the tuples of all walks do not fit at once (3.3e10 at the medium
// size), so the nodes are cut into chunks whose tuples fit a buffer, and each
// chunk's tuples are sorted together with the sources' own.  A chunk:
//   1. lengths of its walks (and the sources'), an exclusive scan of them;
//   2. the walks again, writing 64-bit keys j | i | o | flag and a 32-bit
//      payload (walk id, or source number), flag 0 for a source tuple;
//   3. an LSD radix sort of the keys, 8 bits per pass, stable;
//   4. PREDECESSOR as an inclusive running maximum of (position + 1) over the
//      source tuples; each other tuple walks back over the source tuples of its
//      key and sets one bit per meeting source in its walk's mask;
//   5. per node, the masks are reduced to counts (plain walks) or Lemma 5's
//      weighted sums (stratified walks).
// Walks are the same as the fused kernel's (same keys, same steps), but are
// followed to their full length rather than to the first meet, so the counts
// must agree with the fused path: an independent cross-check of it, and the
// paper's own form for several sources that share their walks' key.
#include <algorithm>
#include <string>
#include <vector>

#include "common.hpp"
#include "device_common.hpp"
#include "philox.hpp"

namespace srk {
namespace {

constexpr int MAX_TUPLE_SOURCES = 32;
constexpr int RS_BLOCK = 256;                     // threads of the sort kernels
#ifndef SRK_RS_ROUNDS
#define SRK_RS_ROUNDS 8
#endif
constexpr int RS_ROUNDS = SRK_RS_ROUNDS;          // 64-key rounds per wave and tile
constexpr int RS_TILE = RS_BLOCK * RS_ROUNDS;     // 2048 keys per tile
constexpr int32_t MAX_GRID_Y = 65535;

struct TupleArgs {
    const uint2 *nodes;
    const uint2 *E;
    const int32_t *active;       // chunk node vl is active[a0 + vl]
    int32_t a0, V;               // first active index of the chunk, its nodes
    int32_t N, L;                // walks per node; cap (stratified: phi)
    PhiloxKey key;
    uint32_t T;                  // plain: continue threshold
    int32_t strat;
    const StratTab *tab;         // stratified: class table
    uint32_t sa, sb;             // stratified: shuffle grid
    const int32_t *src;          // [k] source nodes
    int32_t k;
    uint32_t ib, nb;             // key fields: bits of the step, of the o-value
};

// Walk (v, j) of the query's kind, followed to its end; f(i, o) for every
// position i >= 1 (o-value of the node).  *cls_out: the stratified class.
template <typename F>
__device__ __forceinline__ uint32_t tuple_walk(const TupleArgs &a, uint32_t v, uint32_t j,
                                               uint32_t *cls_out, F f) {
    uint2 cur = a.nodes[v];
    uint32_t len = 0;
    if (a.strat) {
        const uint4 fk = philox4x32_10(v, 0u, 0u, DOM_SHUFFLE, a.key);
        const uint32_t r = shuffle_slot(j, (uint32_t)a.N, a.sa, a.sb, fk);
        const uint32_t cls = slot_class(r, a.tab->ccum, a.L);
        *cls_out = cls;
        WalkDraws w = walk_draws_begin(v, r, a.key, DOM_STRAT);
        for (uint32_t t = 1; t <= cls; ++t) {
            if (cur.y == 0) break;
            const uint2 x = walk_draw_next(w, a.key);
            cur = a.E[cur.x + pick32(x.y, cur.y)];
            f(t, cur.x);
            len = t;
        }
    } else {
        *cls_out = 0;
        WalkDraws w = walk_draws_begin(v, j, a.key);
        for (uint32_t t = 1; t <= (uint32_t)a.L; ++t) {
            const uint2 x = walk_draw_next(w, a.key);
            if (x.x >= a.T || cur.y == 0) break;
            cur = a.E[cur.x + pick32(x.y, cur.y)];
            f(t, cur.x);
            len = t;
        }
    }
    return len;
}

__device__ __forceinline__ uint32_t row_node(const TupleArgs &a, int32_t row) {
    return row < a.V ? (uint32_t)a.active[a.a0 + row] : (uint32_t)a.src[row - a.V];
}

// Walk lengths.  Rows 0..V-1 are the chunk's nodes, rows V..rows-1 the
// sources; grid (x over j, y over rows, strided).  lens[row N + j] (may be
// NULL); row_sum[row] += the row's tuples (may be NULL); cls_src[q N + j] the
// class of the sources' walks (stratified).
__global__ __launch_bounds__(256) void k_tw_len(TupleArgs a, int32_t rows, uint32_t *lens,
                                                unsigned long long *row_sum, uint8_t *cls_src) {
    __shared__ unsigned long long part[4];
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
        uint32_t len = 0;
        if (j < a.N) {
            uint32_t cls;
            len = tuple_walk(a, row_node(a, row), (uint32_t)j, &cls, [](uint32_t, uint32_t) {});
            if (lens) lens[(size_t)row * a.N + j] = len;
            if (cls_src && row >= a.V) cls_src[(size_t)(row - a.V) * a.N + j] = (uint8_t)cls;
        }
        if (row_sum) {
            unsigned long long s = len;
            for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
            if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
            __syncthreads();
            if (threadIdx.x == 0) {
                const unsigned long long t = part[0] + part[1] + part[2] + part[3];
                if (t) atomicAdd(&row_sum[row], t);
            }
            __syncthreads();
        }
    }
}

// The tuples of every walk at its scanned offset.
__global__ __launch_bounds__(256) void k_tw_emit(TupleArgs a, int32_t rows,
                                                 const int64_t *__restrict__ offs,
                                                 uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ vals) {
    const int32_t j = blockIdx.x * 256 + threadIdx.x;
    if (j >= a.N) return;
    for (int32_t row = blockIdx.y; row < rows; row += gridDim.y) {
        const bool is_src = row >= a.V;
        const uint64_t flag = is_src ? 0ull : 1ull;
        const uint32_t val = is_src ? (uint32_t)(row - a.V) : (uint32_t)(row * a.N + j);
        const uint64_t hj = (uint64_t)j << (a.ib + a.nb + 1);
        int64_t p = offs[(size_t)row * a.N + j];
        uint32_t cls;
        tuple_walk(a, row_node(a, row), (uint32_t)j, &cls, [&](uint32_t i, uint32_t o) {
            keys[p] = hj | ((uint64_t)i << (a.nb + 1)) | ((uint64_t)o << 1) | flag;
            vals[p] = val;
            ++p;
        });
    }
}

// ---------------------------------------------------------------- radix sort
// LSD, 8-bit digits, stable.  Tile = 2048 keys: 4 waves x 8 rounds x 64
// (against 4096 keys: 2.54 vs 2.99 s per 8-source call on the medium graph,
// with four blocks per CU instead of two).

__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid) {
    uint64_t m = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
        const uint64_t bb = __ballot((d >> b) & 1u);
        m &= ((d >> b) & 1u) ? bb : ~bb;
    }
    return m;
}

__global__ __launch_bounds__(RS_BLOCK) void k_rs_hist(const uint64_t *__restrict__ keys,
                                                      int64_t count, int shift,
                                                      uint32_t *__restrict__ hist, int64_t tiles) {
    __shared__ uint32_t h[256];
    const int64_t tile = blockIdx.x;
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t base = tile * RS_TILE;
    for (int it = 0; it < RS_ROUNDS; ++it) {
        const int64_t idx = base + (int64_t)it * RS_BLOCK + threadIdx.x;
        if (idx < count) atomicAdd(&h[(uint32_t)(keys[idx] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * tiles + tile] = h[threadIdx.x];
}

// offs[d * tiles + t]: exclusive scan of hist, i.e. where tile t's keys with
// digit d start.  Within a tile the keys are first put in digit order in LDS
// (earlier waves first, then rounds, then lanes: the input order, so the sort
// stays stable); then consecutive threads write consecutive keys, so each
// digit's run of a tile goes out as contiguous stores.
__global__ __launch_bounds__(RS_BLOCK) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                         const uint32_t *__restrict__ vin,
                                                         uint64_t *__restrict__ kout,
                                                         uint32_t *__restrict__ vout,
                                                         int64_t count, int shift,
                                                         const int64_t *__restrict__ offs,
                                                         int64_t tiles) {
    __shared__ uint64_t sk[RS_TILE];
    __shared__ uint32_t sv[RS_TILE];
    __shared__ uint32_t wtot[4][256];   // per wave and digit: count, then local start
    __shared__ uint32_t wrun[4][256];
    __shared__ uint32_t dstart[256];    // tile-local start of each digit
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t tile = blockIdx.x;
    const int64_t tbase = tile * RS_TILE;
    const int64_t base = tbase + (int64_t)wave * (RS_ROUNDS * 64);
    const int32_t n_tile = (int32_t)min((int64_t)RS_TILE, count - tbase);
    for (int i = threadIdx.x; i < 4 * 256; i += RS_BLOCK) {
        (&wtot[0][0])[i] = 0u;
        (&wrun[0][0])[i] = 0u;
    }
    __syncthreads();
    uint64_t key[RS_ROUNDS];   // the wave's keys of the tile, kept for the second pass
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < count;
        key[r] = valid ? kin[idx] : 0ull;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        const uint64_t m = match_digit(d, valid);
        if (valid && lane == __ffsll((long long)m) - 1) atomicAdd(&wtot[wave][d], (uint32_t)__popcll(m));
    }
    __syncthreads();
    {
        // digit dg: its count over the tile, then an exclusive scan over digits
        const int dg = threadIdx.x;   // RS_BLOCK == 256: one digit per thread
        uint32_t c = 0;
        for (int w = 0; w < 4; ++w) c += wtot[w][dg];
        uint32_t total;
        const uint32_t start = block_excl_sum(c, &total);
        dstart[dg] = start;
        uint32_t acc = start;
        for (int w = 0; w < 4; ++w) {
            const uint32_t x = wtot[w][dg];
            wtot[w][dg] = acc;
            acc += x;
        }
    }
    __syncthreads();
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t idx = base + r * 64 + lane;
        const bool valid = idx < count;
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        const uint64_t m = match_digit(d, valid);
        const int leader = valid ? __ffsll((long long)m) - 1 : lane;
        uint32_t old = 0;
        if (valid && lane == leader) old = atomicAdd(&wrun[wave][d], (uint32_t)__popcll(m));
        old = __shfl(old, leader, 64);
        if (valid) {
            const uint32_t lp = wtot[wave][d] + old + (uint32_t)__popcll(m & lt);
            sk[lp] = key[r];
            sv[lp] = vin[idx];
        }
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n_tile; i += RS_BLOCK) {
        const uint64_t k = sk[i];
        const uint32_t d = (uint32_t)(k >> shift) & 255u;
        const int64_t pos = offs[(int64_t)d * tiles + tile] + (i - (int32_t)dstart[d]);
        kout[pos] = k;
        vout[pos] = sv[i];
    }
}

// ------------------------------------------------------------- PREDECESSOR

__global__ void k_tw_last_init(const uint64_t *__restrict__ keys, int64_t count,
                               uint32_t *__restrict__ last) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count;
         p += (int64_t)gridDim.x * blockDim.x)
        last[p] = (keys[p] & 1ull) ? 0u : (uint32_t)(p + 1);
}

__global__ void k_fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_u64(unsigned long long *p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0ull;
}

// A tuple of a node's walk is linked to the closest source tuple before it; if
// that has the same (j, i, o), so do the source tuples just before it (the
// sources' tuples of one key are contiguous and come first): each is a meet.
__global__ void k_tw_link(const uint64_t *__restrict__ keys, const uint32_t *__restrict__ vals,
                          const uint32_t *__restrict__ last, int64_t count,
                          uint32_t *__restrict__ mask) {
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < count;
         p += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t kp = keys[p];
        if (!(kp & 1ull)) continue;
        uint32_t bits = 0;
        for (int64_t q = (int64_t)last[p] - 1; q >= 0 && (keys[q] >> 1) == (kp >> 1); --q)
            bits |= 1u << vals[q];
        if (bits) atomicOr(&mask[vals[p]], bits);
    }
}

// Per node of the chunk (one block each): counts or weighted sums per source.
__global__ __launch_bounds__(256) void k_tw_reduce(TupleArgs a, const uint32_t *__restrict__ mask,
                                                   const uint8_t *__restrict__ cls_src,
                                                   unsigned long long *__restrict__ out,
                                                   int32_t n,
                                                   unsigned long long *__restrict__ counters) {
    __shared__ unsigned long long acc[MAX_TUPLE_SOURCES];
    const int32_t vl = blockIdx.x;
    const uint32_t v = (uint32_t)a.active[a.a0 + vl];
    if (threadIdx.x < MAX_TUPLE_SOURCES) acc[threadIdx.x] = 0ull;
    __syncthreads();
    uint32_t meets = 0;
    uint4 fk = make_uint4(0, 0, 0, 0);
    if (a.strat) fk = philox4x32_10(v, 0u, 0u, DOM_SHUFFLE, a.key);
    for (int32_t j = threadIdx.x; j < a.N; j += blockDim.x) {
        uint32_t m = mask[(size_t)vl * a.N + j];
        if (!m) continue;
        uint32_t cv = 0;
        if (a.strat) cv = slot_class(shuffle_slot((uint32_t)j, (uint32_t)a.N, a.sa, a.sb, fk),
                                     a.tab->ccum, a.L);
        while (m) {
            const int q = __ffs(m) - 1;
            m &= m - 1;
            if ((uint32_t)a.src[q] == v) continue;
            const unsigned long long w =
                a.strat ? strat_weight(a.tab->a, cls_src[(size_t)q * a.N + j], cv) : 1ull;
            atomicAdd(&acc[q], w);
            ++meets;
        }
    }
    __syncthreads();
    if (threadIdx.x < a.k) out[(size_t)threadIdx.x * n + v] = acc[threadIdx.x];
    unsigned long long s = meets;
    for (int d = 32; d > 0; d >>= 1) s += __shfl_xor(s, d, 64);
    if ((threadIdx.x & 63) == 0 && s) atomicAdd(&counters[C_MEETS], s);
}

// A source's own entry: R (plain: every pair meets at step 0) or 0 (stratified).
__global__ void k_tw_sources(TupleArgs a, unsigned long long *out, int32_t n) {
    const int q = threadIdx.x;
    if (q < a.k) out[(size_t)q * n + a.src[q]] = a.strat ? 0ull : (unsigned long long)a.N;
}

int bits_for(uint64_t max_value) {
    int b = 1;
    while (b < 64 && (max_value >> b) != 0) ++b;
    return b;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { device_free(p); }
};

}  // namespace
}  // namespace srk

using namespace srk;

extern "C" int simrank_tuple_meets(const simrank_graph *g, const simrank_query *qs, int32_t k,
                                   uint64_t *sums, simrank_stats *st_opt) {
    clear_error();
    if (!g || !qs || !sums) return fail(SIMRANK_EINVAL, "NULL argument");
    if (k < 1 || k > MAX_TUPLE_SOURCES) return fail(SIMRANK_EINVAL, "k must lie in [1, 32]");
    simrank_params p0;
    int mode0;
    int rc = query_params(&qs[0], g->n, &p0, &mode0);
    if (rc) return rc;
    if (mode0 == SIMRANK_MODE_STITCHED)
        return fail(SIMRANK_EINVAL, "the tuple form takes plain or stratified queries");
    StratTab tab{};
    StratParams sp{};
    const bool strat = mode0 == SIMRANK_MODE_STRATIFIED;
    if (strat && (rc = strat_params(&qs[0], g->n, &sp, &tab))) return rc;
    std::vector<int32_t> srcs(k);
    for (int32_t q = 0; q < k; ++q) {
        simrank_params p;
        int mode;
        if ((rc = query_params(&qs[q], g->n, &p, &mode))) return rc;
        if (qs[q].s < 0 || qs[q].s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
        if (mode != mode0 || p.R != p0.R || p.L != p0.L || p.T != p0.T || qs[q].seed != qs[0].seed)
            return fail(SIMRANK_EINVAL, "the tuple form's queries must share mode, seed, c, R and L");
        if (strat) {
            StratParams s2;
            if ((rc = strat_params(&qs[q], g->n, &s2, nullptr))) return rc;
            if (s2.z != sp.z) return fail(SIMRANK_EINVAL, "stratified queries must share z");
        }
        srcs[q] = qs[q].s;
    }
    const int32_t N = p0.R, L = p0.L;
    SRK_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    // e0 / e1 around the call, s0 / s1 around each chunk's radix sort
    struct EvGuard {
        hipEvent_t e[4] = {nullptr, nullptr, nullptr, nullptr};
        ~EvGuard() {
            for (hipEvent_t x : e)
                if (x) (void)hipEventDestroy(x);
        }
    } evg;
    for (hipEvent_t &x : evg.e) SRK_HIP(hipEventCreate(&x));
    hipEvent_t e0 = evg.e[0], e1 = evg.e[1], s0 = evg.e[2], s1 = evg.e[3];
    double sort_ms = 0.0;
    uint64_t sort_bytes = 0;
    SRK_HIP(hipEventRecord(e0, st));

    const size_t n = (size_t)g->n;
    DevBuf d_src, d_tab, d_out, d_rowsum, d_cnt;
    if ((rc = device_alloc(&d_src.p, 4 * (size_t)k, nullptr))) return rc;
    if ((rc = device_alloc(&d_tab.p, sizeof(StratTab), nullptr))) return rc;
    if ((rc = device_alloc(&d_out.p, 8 * n * (size_t)k, nullptr))) return rc;
    if ((rc = device_alloc(&d_cnt.p, 8 * 8, nullptr))) return rc;
    SRK_HIP(hipMemcpyAsync(d_src.p, srcs.data(), 4 * (size_t)k, hipMemcpyHostToDevice, st));
    SRK_HIP(hipMemcpyAsync(d_tab.p, &tab, sizeof(StratTab), hipMemcpyHostToDevice, st));
    auto *out = (unsigned long long *)d_out.p;
    auto *counters = (unsigned long long *)d_cnt.p;
    k_fill_u64<<<grid_for((int64_t)(n * k), 256), 256, 0, st>>>(out, (int64_t)(n * k));
    k_fill_u64<<<1, 64, 0, st>>>(counters, 8);

    TupleArgs a{};
    a.nodes = g->nodes;
    a.E = g->E;
    a.active = g->active;
    a.N = N;
    a.L = L;
    a.key = make_key(qs[0].seed);
    a.T = p0.T;
    a.strat = strat ? 1 : 0;
    a.tab = (const StratTab *)d_tab.p;
    a.sa = (uint32_t)sp.sa;
    a.sb = (uint32_t)sp.sb;
    a.src = (const int32_t *)d_src.p;
    a.k = k;
    a.ib = (uint32_t)bits_for((uint64_t)L);
    a.nb = (uint32_t)bits_for((uint64_t)std::max<int64_t>(g->m_slots - 1, 1));
    const int jb = bits_for((uint64_t)std::max(N - 1, 1));
    const int key_bits = jb + (int)a.ib + (int)a.nb + 1;
    if (key_bits > 64) return fail(SIMRANK_EINVAL, "tuple keys exceed 64 bits");

    // tuples per node (all active nodes), to cut the chunks
    const int32_t na = g->n_active;
    std::vector<unsigned long long> row_sum(std::max(na, 1), 0ull);
    if (na > 0) {
        if ((rc = device_alloc(&d_rowsum.p, 8 * (size_t)na, nullptr))) return rc;
        k_fill_u64<<<grid_for(na, 256), 256, 0, st>>>((unsigned long long *)d_rowsum.p, na);
        TupleArgs all = a;
        all.a0 = 0;
        all.V = na;
        k_tw_len<<<dim3(grid_for(N, 256), std::min(na, MAX_GRID_Y)), 256, 0, st>>>(
            all, na, nullptr, (unsigned long long *)d_rowsum.p, nullptr);
        SRK_HIP(hipGetLastError());
        SRK_HIP(hipMemcpyAsync(row_sum.data(), d_rowsum.p, 8 * (size_t)na, hipMemcpyDeviceToHost, st));
        SRK_HIP(hipStreamSynchronize(st));
    }
    // chunk limits: tuples per chunk (keys and payloads twice, running maxima)
    // and walks per chunk (lengths, offsets, masks)
    const int64_t src_tuples_max = (int64_t)k * N * L;
    const int64_t cap_tuples = (int64_t)1 << 28, cap_walks = (int64_t)1 << 27;
    std::vector<std::pair<int32_t, int32_t>> chunks;   // (first active index, nodes)
    {
        int32_t c0 = 0;
        int64_t tup = 0;
        for (int32_t i = 0; i < na; ++i) {
            const int64_t t = (int64_t)row_sum[i];
            const bool full = i > c0 && (tup + t + src_tuples_max > cap_tuples ||
                                         (int64_t)(i - c0 + 1) * N > cap_walks ||
                                         i - c0 + 1 + k > MAX_GRID_Y);
            if (full) {
                chunks.push_back({c0, i - c0});
                c0 = i;
                tup = 0;
            }
            tup += t;
        }
        if (na > 0) chunks.push_back({c0, na - c0});
    }
    int64_t max_tuples = 0, max_walks = 0;
    for (auto &c : chunks) {
        int64_t t = src_tuples_max;
        for (int32_t i = c.first; i < c.first + c.second; ++i) t += (int64_t)row_sum[i];
        max_tuples = std::max(max_tuples, t);
        max_walks = std::max(max_walks, (int64_t)(c.second + k) * N);
    }
    if (max_tuples >= (int64_t)0xffffffffu)
        return fail(SIMRANK_EINVAL, "one node's walks exceed the tuple buffer");
    uint64_t total_moves = 0;
    if (!chunks.empty()) {
        const int64_t tiles_max = (max_tuples + RS_TILE - 1) / RS_TILE;
        DevBuf k0, k1, v0, v1, last, lens, offs, mask, hist, hoffs, tot, cls;
        if ((rc = device_alloc(&k0.p, 8 * (size_t)max_tuples, nullptr)) ||
            (rc = device_alloc(&k1.p, 8 * (size_t)max_tuples, nullptr)) ||
            (rc = device_alloc(&v0.p, 4 * (size_t)max_tuples, nullptr)) ||
            (rc = device_alloc(&v1.p, 4 * (size_t)max_tuples, nullptr)) ||
            (rc = device_alloc(&last.p, 4 * (size_t)max_tuples, nullptr)) ||
            (rc = device_alloc(&lens.p, 4 * (size_t)max_walks, nullptr)) ||
            (rc = device_alloc(&offs.p, 8 * (size_t)max_walks, nullptr)) ||
            (rc = device_alloc(&mask.p, 4 * (size_t)max_walks, nullptr)) ||
            (rc = device_alloc(&hist.p, 4 * 256 * (size_t)std::max<int64_t>(tiles_max, 1), nullptr)) ||
            (rc = device_alloc(&hoffs.p, 8 * 256 * (size_t)std::max<int64_t>(tiles_max, 1), nullptr)) ||
            (rc = device_alloc(&tot.p, 8, nullptr)) ||
            (rc = device_alloc(&cls.p, (size_t)k * N, nullptr)))
            return rc;
        for (auto &c : chunks) {
            TupleArgs ca = a;
            ca.a0 = c.first;
            ca.V = c.second;
            const int32_t rows = c.second + k;
            const dim3 grid(grid_for(N, 256), std::min(rows, MAX_GRID_Y));
            k_tw_len<<<grid, 256, 0, st>>>(ca, rows, (uint32_t *)lens.p, nullptr, (uint8_t *)cls.p);
            if ((rc = scan_exclusive_u32_to_i64((const uint32_t *)lens.p, (int64_t)rows * N,
                                                (int64_t *)offs.p, (int64_t *)tot.p, st)))
                return rc;
            int64_t count = 0;
            SRK_HIP(hipMemcpyAsync(&count, tot.p, 8, hipMemcpyDeviceToHost, st));
            SRK_HIP(hipStreamSynchronize(st));
            if (count > max_tuples) return fail(SIMRANK_EDEVICE, "tuple count beyond its bound");
            if (count == 0) continue;
            k_tw_emit<<<grid, 256, 0, st>>>(ca, rows, (const int64_t *)offs.p, (uint64_t *)k0.p,
                                           (uint32_t *)v0.p);
            SRK_HIP(hipGetLastError());
            // stable LSD radix sort on the key bits in use
            uint64_t *kin = (uint64_t *)k0.p, *kout = (uint64_t *)k1.p;
            uint32_t *vin = (uint32_t *)v0.p, *vout = (uint32_t *)v1.p;
            const int64_t tiles = (count + RS_TILE - 1) / RS_TILE;
            SRK_HIP(hipEventRecord(s0, st));
            int passes = 0;
            for (int shift = 0; shift < key_bits; shift += 8, ++passes) {
                k_rs_hist<<<(unsigned)tiles, RS_BLOCK, 0, st>>>(kin, count, shift, (uint32_t *)hist.p,
                                                               tiles);
                if ((rc = scan_exclusive_u32_to_i64((const uint32_t *)hist.p, 256 * tiles,
                                                    (int64_t *)hoffs.p, (int64_t *)tot.p, st)))
                    return rc;
                k_rs_scatter<<<(unsigned)tiles, RS_BLOCK, 0, st>>>(kin, vin, kout, vout, count, shift,
                                                                  (const int64_t *)hoffs.p, tiles);
                std::swap(kin, kout);
                std::swap(vin, vout);
            }
            SRK_HIP(hipEventRecord(s1, st));
            SRK_HIP(hipGetLastError());
            // a histogram pass reads each 8-byte key; a scatter pass reads and
            // writes each key and its 4-byte payload
            sort_bytes += (uint64_t)passes * (uint64_t)count * (8u + 24u);
            // PREDECESSOR: running maximum of (position + 1) over the sources' tuples
            k_tw_last_init<<<grid_for(count, 256), 256, 0, st>>>(kin, count, (uint32_t *)last.p);
            if ((rc = scan_inclusive_max_u32((uint32_t *)last.p, count, st))) return rc;
            k_fill_u32<<<grid_for((int64_t)c.second * N, 256), 256, 0, st>>>(
                (uint32_t *)mask.p, (int64_t)c.second * N, 0u);
            k_tw_link<<<std::min<unsigned>(grid_for(count, 256), 65536u), 256, 0, st>>>(
                kin, vin, (const uint32_t *)last.p, count, (uint32_t *)mask.p);
            k_tw_reduce<<<(unsigned)c.second, 256, 0, st>>>(ca, (const uint32_t *)mask.p,
                                                           (const uint8_t *)cls.p, out, g->n,
                                                           counters);
            SRK_HIP(hipGetLastError());
            int64_t src_count = 0;
            {
                // the sources' tuples: the scanned offset of row V is where they start
                int64_t first_src = 0;
                SRK_HIP(hipMemcpyAsync(&first_src, (int64_t *)offs.p + (size_t)c.second * N, 8,
                                       hipMemcpyDeviceToHost, st));
                SRK_HIP(hipStreamSynchronize(st));
                src_count = count - first_src;
                float sms = 0.f;
                SRK_HIP(hipEventElapsedTime(&sms, s0, s1));
                sort_ms += sms;
            }
            total_moves += (uint64_t)(count - src_count);
        }
    }
    k_tw_sources<<<1, 64, 0, st>>>(a, out, g->n);
    SRK_HIP(hipGetLastError());
    SRK_HIP(hipEventRecord(e1, st));
    SRK_HIP(hipMemcpyAsync(sums, out, 8 * n * (size_t)k, hipMemcpyDeviceToHost, st));
    unsigned long long c[8];
    SRK_HIP(hipMemcpyAsync(c, counters, sizeof(c), hipMemcpyDeviceToHost, st));
    SRK_HIP(hipStreamSynchronize(st));
    if (st_opt) {
        float ms = 0.f;
        SRK_HIP(hipEventElapsedTime(&ms, e0, e1));
        *st_opt = simrank_stats{};
        st_opt->pairs = (uint64_t)(g->n - 1) * (uint64_t)N * (uint64_t)k;
        st_opt->moves = total_moves;
        st_opt->draws = sort_bytes;        // bytes the sort passes move (see simrank.h)
        st_opt->meet_ms = sort_ms;
        st_opt->meets = c[C_MEETS];
        st_opt->ms = ms;
        st_opt->R = N;
        st_opt->L = L;
        st_opt->T = p0.T;
    }
    return SIMRANK_OK;
}
