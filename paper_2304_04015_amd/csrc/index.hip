// Stitched-walk index: per-node pools of short walk segments, joined into
// long walks by pointer doubling — the single-GPU counterpart of building
// long walks from short ones in few rounds (Theorem 2, Section 4.1).
//
//   P(y)      = ceil(kappa * dbar(y)), dbar(y) = number of in-edge rows that
//               list y (walks arrive at y along those edges; counted once at
//               graph ingest); pools are sampled with replacement, so they
//               never run out
//   slot sigma = pool_off[y] + i, i < P(y): a sqrt(c)-walk of at most 2^k
//               steps from y keyed (y, i, t, 1) under the index seed
//   succ(sigma) = pool_off[z] + pick(draw(y, i, 0, 3).x0, P(z)) if the
//               segment made all 2^k moves and ended at z, else none
//   chain[sigma][m] = succ^m(sigma) for m < width = 64 / 2^k, built in
//               log2(width) doubling rounds: round r copies the first 2^r
//               entries of chain[J_r(sigma)] behind those of sigma, with
//               J_0 = succ and J_{r+1} = J_r o J_r.
#include "common.hpp"
#include "philox.hpp"

// Segments in flight per lane and consecutive slots per wave of k_segments.
#ifndef SRK_SEG_SLOTS
#define SRK_SEG_SLOTS 2
#endif
#ifndef SRK_SEG_CHUNK
#define SRK_SEG_CHUNK 2048
#endif
// 1: rows of up to 16 positions are assembled in registers and written once.
#ifndef SRK_SEG_BUFFER
#define SRK_SEG_BUFFER 1
#endif

namespace srk {
namespace {

__global__ void k_fill_u32i(uint32_t *__restrict__ p, int64_t n, uint32_t val) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = val;
}

__global__ void k_pool_sizes(const uint32_t *__restrict__ dbar, int32_t n, double kappa,
                             int64_t *__restrict__ P, uint32_t *__restrict__ too_big) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    const double p = ceil(kappa * (double)dbar[y]);
    if (p >= 4294967295.0) {
        *too_big = 1u;
        P[y] = 0;
    } else {
        P[y] = (int64_t)p;
    }
}

__global__ void k_owner_scatter(const int64_t *__restrict__ pool_off, const int64_t *__restrict__ P,
                                int32_t n, uint32_t *__restrict__ owner) {
    const int64_t y = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (y >= n) return;
    if (P[y] > 0) owner[pool_off[y]] = (uint32_t)y;
}

struct SegArgs {
    const uint2 *nodes;
    const uint2 *E;
    const uint32_t *node_of;
    const int64_t *pool_off;
    const uint32_t *owner;
    uint32_t *seg;
    uint8_t *seg_lens;
    uint32_t *succ;
    uint32_t *chain;
    unsigned long long *moves;
    PhiloxKey key;
    uint32_t T;
    int32_t seg_len, width;
    int64_t segments;
    int64_t chunk;       // consecutive slots per wave
};

// One segment being built on a lane.  LB > 0: the segment's positions are
// kept in registers (LB = 2^k words) and its row is written once, whole, when
// the segment ends.
template <int LB>
struct SegSlot {
    uint32_t sig;        // its slot
    uint32_t y;          // the node whose pool holds it
    uint32_t o, d;       // current position (slot offset in E, in-degree)
    uint32_t t;          // moves made
    uint32_t ph;         // SEG_*: what the slot waits for
    WalkDraws w;         // the segment's draws (walk index = i, its rank in y's pool)
    uint32_t pos[LB > 0 ? LB : 1];   // positions 1..t, NIL after (LB > 0)
};

// Position t + 1 of a buffered segment (selects, so that the array stays in
// registers).
template <int LB>
__device__ __forceinline__ void seg_put(SegSlot<LB> &s, uint32_t o) {
#pragma unroll
    for (int k = 0; k < LB; ++k) s.pos[k] = (s.t == (uint32_t)k) ? o : s.pos[k];
}

// A buffered segment's whole row, in 16-byte pieces where it has four words
// or more.
template <int LB>
__device__ __forceinline__ void seg_write_row(const SegSlot<LB> &s, uint32_t *seg) {
    uint32_t *row = seg + (size_t)s.sig * LB;
    if constexpr (LB >= 4) {
#pragma unroll
        for (int k = 0; k < LB; k += 4)
            *(uint4 *)(row + k) = make_uint4(s.pos[k], s.pos[k + 1], s.pos[k + 2], s.pos[k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < LB; ++k) row[k] = s.pos[k];
    }
}

// Phases of a segment slot.  Every phase but IDLE issues one load per
// iteration, so a lane keeps NS independent loads in flight.
enum : uint32_t {
    SEG_IDLE = 0,
    SEG_OWNER = 1,   // read owner[sig]                    -> y
    SEG_START = 2,   // read pool_off[y] and nodes[y]       -> i, first position
    SEG_WALK = 3,    // one step: draw, then read E[o + pick] -> next position
    SEG_END = 4,     // the segment made all 2^k moves: read node_of[o] -> z
    SEG_SUCC = 5     // read pool_off[z], pool_off[z + 1]  -> successor slot
};

// Segments of the index.  Each wave builds a chunk of consecutive slots; every
// lane keeps NS segments in flight and takes the next slot of the chunk as soon
// as one of its segments is finished (ballot + rank), so lanes do not idle while
// the longest segment of a wave is still walking, and every lane has NS
// independent loads outstanding per iteration.  Consecutive slots belong to the
// same node y, so the first steps of a chunk share rows in the CU's L1.  A
// segment's row is first filled with NIL and then receives one position per
// move.  succ(sigma) is picked from the pool of the node where an open segment
// ends.
template <int NS, int LB>
__global__ __launch_bounds__(256) void k_segments(SegArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int64_t c0 = wave * a.chunk;
    if (c0 >= a.segments) return;
    const int64_t c1 = min(c0 + a.chunk, a.segments);
    int64_t cursor = c0;
    const uint32_t L = (uint32_t)a.seg_len;
    uint32_t moves = 0;
    SegSlot<LB> sl[NS];
#pragma unroll
    for (int q = 0; q < NS; ++q) sl[q].ph = SEG_IDLE;

    for (;;) {
        // refill idle slots from the wave's chunk
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            const uint64_t need = __ballot(sl[q].ph == SEG_IDLE);
            const int64_t left = c1 - cursor;
            if (need == 0ull || left <= 0) continue;
            const uint32_t want = (uint32_t)__popcll(need);
            const uint32_t take = left < (int64_t)want ? (uint32_t)left : want;
            const uint32_t rank = __builtin_amdgcn_mbcnt_hi(
                (uint32_t)(need >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)need, 0u));
            if (((need >> lane) & 1ull) && rank < take) {
                sl[q].sig = (uint32_t)(cursor + rank);
                sl[q].ph = SEG_OWNER;
            }
            cursor += take;
        }
        bool any = false;
#pragma unroll
        for (int q = 0; q < NS; ++q) any |= sl[q].ph != SEG_IDLE;
        if (__ballot(any) == 0ull) break;   // the chunk is done

        // issue: one load per busy slot
        uint2 e[NS];
        uint32_t u[NS];
        int64_t b0[NS], b1[NS];
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            SegSlot<LB> &s = sl[q];
            switch (s.ph) {
            case SEG_OWNER: u[q] = a.owner[s.sig]; break;
            case SEG_START: b0[q] = a.pool_off[s.y]; e[q] = a.nodes[s.y]; break;
            case SEG_WALK: {
                const uint2 x = walk_draw_next(s.w, a.key);   // step t + 1
                if (x.x >= a.T || s.d == 0u) {
                    s.ph = SEG_IDLE;                           // closed before 2^k moves
                    if constexpr (LB > 0) seg_write_row(s, a.seg);
                    a.seg_lens[s.sig] = (uint8_t)s.t;
                    a.succ[s.sig] = NIL;
                    if (a.width == 1) a.chain[s.sig] = s.sig;
                } else {
                    e[q] = a.E[s.o + pick32(x.y, s.d)];
                }
                break;
            }
            case SEG_END: u[q] = a.node_of[s.o]; break;
            case SEG_SUCC: b0[q] = a.pool_off[s.y]; b1[q] = a.pool_off[s.y + 1]; break;
            default: break;
            }
        }
        // consume
#pragma unroll
        for (int q = 0; q < NS; ++q) {
            SegSlot<LB> &s = sl[q];
            switch (s.ph) {
            case SEG_OWNER:
                s.y = u[q];
                s.ph = SEG_START;
                break;
            case SEG_START: {
                const uint32_t i = (uint32_t)((int64_t)s.sig - b0[q]);
                s.w = walk_draws_begin(s.y, i, a.key, DOM_SEGMENT);
                s.o = e[q].x;
                s.d = e[q].y;
                s.t = 0;
                if constexpr (LB > 0) {
#pragma unroll
                    for (int k = 0; k < LB; ++k) s.pos[k] = NIL;
                } else {
                    uint32_t *row = a.seg + (size_t)s.sig * L;
                    if (L >= 4) {
                        for (uint32_t k = 0; k < L; k += 4)
                            *(uint4 *)(row + k) = make_uint4(NIL, NIL, NIL, NIL);
                    } else {
                        for (uint32_t k = 0; k < L; ++k) row[k] = NIL;
                    }
                }
                s.ph = SEG_WALK;
                break;
            }
            case SEG_WALK:
                s.o = e[q].x;
                s.d = e[q].y;
                if constexpr (LB > 0) seg_put(s, s.o);
                else a.seg[(size_t)s.sig * L + s.t] = s.o;
                ++s.t;
                ++moves;
                if (s.t == L) {
                    if constexpr (LB > 0) seg_write_row(s, a.seg);
                    s.ph = SEG_END;
                }
                break;
            case SEG_END:
                // keep the walk index for the successor draw; y becomes z
                s.o = s.y;      // the segment's own node, for the draw below
                s.y = u[q];
                s.ph = SEG_SUCC;
                break;
            case SEG_SUCC: {
                const uint32_t i = s.w.j;
                const uint4 x = philox4x32_10(s.o, i, 0u, DOM_SUCC, a.key);
                const uint32_t nx = (uint32_t)(b0[q] + (int64_t)pick64(x.x, (uint64_t)(b1[q] - b0[q])));
                a.seg_lens[s.sig] = (uint8_t)L;
                a.succ[s.sig] = nx;
                if (a.width == 1) a.chain[s.sig] = s.sig;
                s.ph = SEG_IDLE;
                break;
            }
            default: break;
            }
        }
    }
    unsigned long long m = moves;
    for (int d = 32; d > 0; d >>= 1) m += __shfl_xor(m, d, 64);
    if (lane == 0 && m) atomicAdd(a.moves, m);
}

// Round r of pointer doubling: chain[s][h + i] = chain[J[s]][i] for i < h = 2^r,
// Jn[s] = J[J[s]].  Reads touch columns < h and writes columns >= h, so the
// round can update chain in place.  Round 0 writes columns 0 and 1 together:
// chain[s][0] = s and chain[s][1] = J[s] = succ(s) (column 0 of any row is the
// row's own slot), without reading another row.  Columns move in 8- or 16-byte
// pieces.
__global__ __launch_bounds__(256) void k_double(uint32_t *__restrict__ chain,
                                                const uint32_t *__restrict__ J,
                                                uint32_t *__restrict__ Jn, int64_t segments,
                                                int32_t width, int32_t h) {
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= segments) return;
    const uint32_t a = J[s];
    uint32_t *row = chain + (size_t)s * width;
    if (Jn) Jn[s] = (a == NIL) ? NIL : J[a];
    if (h == 1) {
        *(uint2 *)row = make_uint2((uint32_t)s, a);
        return;
    }
    uint32_t *dst = row + h;
    const uint32_t *src = chain + (size_t)a * width;
    if (h == 2) {
        *(uint2 *)dst = (a == NIL) ? make_uint2(NIL, NIL) : *(const uint2 *)src;
        return;
    }
    for (int32_t k = 0; k < h; k += 4)
        *(uint4 *)(dst + k) = (a == NIL) ? make_uint4(NIL, NIL, NIL, NIL) : *(const uint4 *)(src + k);
}

struct ReadArgs {
    const Index *ix;
    const uint32_t *node_of;
    const int64_t *sigma;
    int64_t count;
    int32_t *nodes;
    int32_t *lens;
    int64_t *succ;
    int64_t *chain;
};

__global__ void k_index_read(const uint32_t *__restrict__ node_of, const uint32_t *__restrict__ seg,
                             const uint8_t *__restrict__ seg_lens, const uint32_t *__restrict__ succ,
                             const uint32_t *__restrict__ chain, int32_t seg_len, int32_t width,
                             const int64_t *__restrict__ sig, int64_t count,
                             int32_t *__restrict__ out_nodes, int32_t *__restrict__ out_lens,
                             int64_t *__restrict__ out_succ, int64_t *__restrict__ out_chain) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const int64_t s = sig[i];
    const int32_t l = seg_lens[s];
    out_lens[i] = l;
    for (int32_t t = 0; t < seg_len; ++t)
        out_nodes[i * seg_len + t] = t < l ? (int32_t)node_of[seg[s * seg_len + t]] : -1;
    const uint32_t nx = succ[s];
    out_succ[i] = nx == NIL ? -1 : (int64_t)nx;
    if (out_chain)
        for (int32_t m = 0; m < width; ++m) {
            const uint32_t c = chain[s * width + m];
            out_chain[i * width + m] = c == NIL ? -1 : (int64_t)c;
        }
}

}  // namespace

void index_free(Index *ix) {
    if (!ix) return;
    device_free(ix->pool_off);
    device_free(ix->seg);
    device_free(ix->seg_lens);
    device_free(ix->succ);
    device_free(ix->chain);
    *ix = Index{};
}

}  // namespace srk

using namespace srk;


extern "C" int simrank_build_index(simrank_graph *g, const simrank_index_params *p) {
    clear_error();
    if (!g || !p) return fail(SIMRANK_EINVAL, "NULL argument");
    if (p->seg_log2 < 0 || p->seg_log2 > 6) return fail(SIMRANK_EINVAL, "seg_log2 must lie in [0, 6]");
    if (!(p->kappa > 0.0) || !(p->kappa < 1e6)) return fail(SIMRANK_EINVAL, "kappa must lie in (0, 1e6)");
    if (!(p->c > 0.0 && p->c < 1.0)) return fail(SIMRANK_EINVAL, "c must lie in (0, 1)");
    SRK_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    SRK_HIP(hipStreamSynchronize(st));
    ++g->index_gen;   // plans made with the old index must not run on the new one
    if (g->index) {
        index_free(g->index);
        delete g->index;
        g->index = nullptr;
    }
    Index *ix = new Index();
    ix->seg_log2 = p->seg_log2;
    ix->seg_len = 1 << p->seg_log2;
    ix->width = MAX_STITCH_CAP / ix->seg_len;
    ix->levels = 0;
    while ((1 << ix->levels) < ix->width) ++ix->levels;
    ix->kappa = p->kappa;
    ix->c = p->c;
    ix->T = continue_threshold(p->c);
    ix->seed = p->seed;
    const int32_t n = g->n;
    int rc = SIMRANK_OK;
    uint32_t *owner = nullptr, *Ja = nullptr, *Jb = nullptr, *flag = nullptr;
    int64_t *P = nullptr, *tot = nullptr;
    unsigned long long *moves = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr, es0 = nullptr, es1 = nullptr;
    auto cleanup = [&]() {
        device_free(owner); device_free(Ja); device_free(Jb);
        device_free(flag); device_free(P); device_free(tot); device_free(moves);
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (es0) (void)hipEventDestroy(es0);
        if (es1) (void)hipEventDestroy(es1);
    };
    auto bail = [&](int code) {
        cleanup();
        index_free(ix);
        delete ix;
        return code;
    };
#define IX_TRY(x)                         \
    do {                                  \
        rc = (x);                         \
        if (rc != SIMRANK_OK) return bail(rc); \
    } while (0)
#define IX_HIP(x)                                                                         \
    do {                                                                                  \
        hipError_t e_ = (x);                                                              \
        if (e_ != hipSuccess)                                                             \
            return bail(fail(SIMRANK_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_))); \
    } while (0)

    IX_HIP(hipEventCreate(&e0));
    IX_HIP(hipEventCreate(&e1));
    IX_HIP(hipEventCreate(&es0));
    IX_HIP(hipEventCreate(&es1));
    IX_TRY(device_alloc((void **)&P, 8 * (size_t)n, nullptr));
    IX_TRY(device_alloc((void **)&tot, 8 * 2, nullptr));
    IX_TRY(device_alloc((void **)&flag, 4, nullptr));
    IX_TRY(device_alloc((void **)&moves, 8, nullptr));
    IX_TRY(device_alloc((void **)&ix->pool_off, 8 * ((size_t)n + 1), &ix->bytes));
    IX_HIP(hipEventRecord(e0, st));
    k_fill_u32i<<<1, 64, 0, st>>>(flag, 1, 0u);
    k_fill_u32i<<<1, 64, 0, st>>>((uint32_t *)moves, 2, 0u);
    k_pool_sizes<<<grid_for(n, 256), 256, 0, st>>>(g->dbar, n, p->kappa, P, flag);
    IX_TRY(scan_exclusive_i64(P, n, ix->pool_off, tot, st));
    IX_HIP(hipMemcpyAsync(ix->pool_off + n, tot, 8, hipMemcpyDeviceToDevice, st));
    int64_t total = 0;
    uint32_t too_big = 0;
    IX_HIP(hipMemcpyAsync(&total, tot, 8, hipMemcpyDeviceToHost, st));
    IX_HIP(hipMemcpyAsync(&too_big, flag, 4, hipMemcpyDeviceToHost, st));
    IX_HIP(hipStreamSynchronize(st));
    if (too_big || total >= (int64_t)NIL)
        return bail(fail(SIMRANK_EINVAL, "pool sizes exceed 2^32 - 1 segments"));
    ix->segments = total;
    const int64_t S = total > 0 ? total : 1;
    IX_TRY(device_alloc((void **)&ix->seg, 4 * (size_t)S * ix->seg_len, &ix->bytes));
    IX_TRY(device_alloc((void **)&ix->seg_lens, (size_t)S, &ix->bytes));
    IX_TRY(device_alloc((void **)&ix->succ, 4 * (size_t)S, &ix->bytes));
    IX_TRY(device_alloc((void **)&ix->chain, 4 * (size_t)S * ix->width, &ix->bytes));
    IX_TRY(device_alloc((void **)&owner, 4 * (size_t)S, nullptr));
    if (ix->levels > 1) {
        IX_TRY(device_alloc((void **)&Ja, 4 * (size_t)S, nullptr));
        IX_TRY(device_alloc((void **)&Jb, 4 * (size_t)S, nullptr));
    }
    if (total > 0) {
        k_fill_u32i<<<2048, 256, 0, st>>>(owner, total, 0u);
        k_owner_scatter<<<grid_for(n, 256), 256, 0, st>>>(ix->pool_off, P, n, owner);
        IX_TRY(scan_inclusive_max_u32(owner, total, st));
        SegArgs sa{g->nodes, g->E, g->node_of, ix->pool_off, owner, ix->seg, ix->seg_lens,
                   ix->succ, ix->chain, moves, make_key(p->seed), ix->T, ix->seg_len, ix->width,
                   total, SRK_SEG_CHUNK};
        const int64_t waves = (total + SRK_SEG_CHUNK - 1) / SRK_SEG_CHUNK;
        IX_HIP(hipEventRecord(es0, st));
        // rows of up to 16 positions are assembled in registers and written
        // once; longer ones are written position by position
        const unsigned gs = grid_for(waves * 64, 256);
        switch (SRK_SEG_BUFFER ? ix->seg_len : 0) {
        case 1: k_segments<SRK_SEG_SLOTS, 1><<<gs, 256, 0, st>>>(sa); break;
        case 2: k_segments<SRK_SEG_SLOTS, 2><<<gs, 256, 0, st>>>(sa); break;
        case 4: k_segments<SRK_SEG_SLOTS, 4><<<gs, 256, 0, st>>>(sa); break;
        case 8: k_segments<SRK_SEG_SLOTS, 8><<<gs, 256, 0, st>>>(sa); break;
        case 16: k_segments<SRK_SEG_SLOTS, 16><<<gs, 256, 0, st>>>(sa); break;
        default: k_segments<SRK_SEG_SLOTS, 0><<<gs, 256, 0, st>>>(sa); break;
        }
        IX_HIP(hipEventRecord(es1, st));
        const uint32_t *J = ix->succ;
        for (int32_t r = 0; r < ix->levels; ++r) {
            uint32_t *Jn = (r + 1 < ix->levels) ? ((r & 1) ? Jb : Ja) : nullptr;
            k_double<<<grid_for(total, 256), 256, 0, st>>>(ix->chain, J, Jn, total, ix->width,
                                                           1 << r);
            J = Jn;
        }
        IX_HIP(hipGetLastError());
    }
    IX_HIP(hipEventRecord(e1, st));
    unsigned long long mv = 0;
    IX_HIP(hipMemcpyAsync(&mv, moves, 8, hipMemcpyDeviceToHost, st));
    IX_HIP(hipStreamSynchronize(st));
    float ms = 0.f, sms = 0.f, dms = 0.f;
    IX_HIP(hipEventElapsedTime(&ms, e0, e1));
    if (total > 0) {
        IX_HIP(hipEventElapsedTime(&sms, es0, es1));
        IX_HIP(hipEventElapsedTime(&dms, es1, e1));
    }
    ix->build_ms = ms;
    ix->segments_ms = sms;
    ix->doubling_ms = dms;
    ix->build_moves = mv;
    cleanup();
    g->index = ix;
    return SIMRANK_OK;
#undef IX_TRY
#undef IX_HIP
}

extern "C" int simrank_index_info(const simrank_graph *g, simrank_index_summary *out) {
    clear_error();
    if (!g || !out) return fail(SIMRANK_EINVAL, "NULL argument");
    if (!g->index) return fail(SIMRANK_ESTATE, "no index built");
    const Index *ix = g->index;
    out->segments = ix->segments;
    out->bytes = ix->bytes;
    out->seg_log2 = ix->seg_log2;
    out->levels = ix->levels;
    out->build_ms = ix->build_ms;
    out->build_moves = ix->build_moves;
    out->segments_ms = ix->segments_ms;
    out->doubling_ms = ix->doubling_ms;
    return SIMRANK_OK;
}

extern "C" int simrank_index_read(const simrank_graph *g, const int64_t *sigma, int64_t count,
                                  int32_t *nodes, int32_t *lens, int64_t *succ,
                                  int64_t *chain_opt) {
    clear_error();
    if (!g || (count > 0 && (!sigma || !nodes || !lens || !succ)))
        return fail(SIMRANK_EINVAL, "NULL argument");
    if (!g->index) return fail(SIMRANK_ESTATE, "no index built");
    const Index *ix = g->index;
    for (int64_t i = 0; i < count; ++i)
        if (sigma[i] < 0 || sigma[i] >= ix->segments)
            return fail(SIMRANK_EINVAL, "slot out of range");
    if (count <= 0) return SIMRANK_OK;
    SRK_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    int64_t *dsig = nullptr, *dsucc = nullptr, *dchain = nullptr;
    int32_t *dnodes = nullptr, *dlens = nullptr;
    int rc = device_alloc((void **)&dsig, 8 * (size_t)count, nullptr);
    if (!rc) rc = device_alloc((void **)&dsucc, 8 * (size_t)count, nullptr);
    if (!rc) rc = device_alloc((void **)&dnodes, 4 * (size_t)count * ix->seg_len, nullptr);
    if (!rc) rc = device_alloc((void **)&dlens, 4 * (size_t)count, nullptr);
    if (!rc && chain_opt) rc = device_alloc((void **)&dchain, 8 * (size_t)count * ix->width, nullptr);
    if (!rc) {
        hipError_t e = hipMemcpyAsync(dsig, sigma, 8 * (size_t)count, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            k_index_read<<<grid_for(count, 256), 256, 0, st>>>(
                g->node_of, ix->seg, ix->seg_lens, ix->succ, ix->chain, ix->seg_len, ix->width,
                dsig, count, dnodes, dlens, dsucc, dchain);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(nodes, dnodes, 4 * (size_t)count * ix->seg_len,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(lens, dlens, 4 * (size_t)count, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipMemcpyAsync(succ, dsucc, 8 * (size_t)count, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess && chain_opt)
            e = hipMemcpyAsync(chain_opt, dchain, 8 * (size_t)count * ix->width,
                               hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    device_free(dsig); device_free(dsucc); device_free(dnodes); device_free(dlens);
    device_free(dchain);
    return rc;
}
