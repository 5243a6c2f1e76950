// Single-source query: source walks, their compaction into LDS tiles, the
// fused walk + meet + count kernel, and the estimate.
//
// Method (Section 2.2; Lemma 2; Section 3.2 pairing): walk j of the source s
// is paired with walk j of every node v, j < R; the pair meets if the two
// walks are on the same node at the same step; s_hat(s, v) = meets / R.
//
// The meet kernel generates walk (v, j) only as far as it can still meet walk
// (s, j): it stops at the first meeting step (a pair counts once, Section 4.4),
// when walk (v, j) stops, and when walk (s, j) has no later position.  This
// reads exactly the positions the meet test compares, so the counts equal
// those of full walks, while a pair costs about sum_t c^t = c / (1 - c) moves.
#include <math.h>

#include <algorithm>

#include "common.hpp"
#include "device_common.hpp"
#include "philox.hpp"

namespace srk {
namespace {

// ------------------------------------------------------------ small kernels

__global__ void k_set_desc(QueryDesc *dst, QueryDesc d) { *dst = d; }

// grid (x over nodes, y = query)
__global__ void k_init(const QueryDesc *__restrict__ qd, unsigned long long *__restrict__ counters) {
    const QueryDesc &d = qd[blockIdx.y];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (blockIdx.x == 0 && threadIdx.x < 8) {
        d.meta[threadIdx.x] = 0u;
        if (blockIdx.y == 0) counters[threadIdx.x] = 0ull;
    }
    if (strat_kind(d.kind)) {
        for (int64_t v = i; v < d.n; v += (int64_t)gridDim.x * blockDim.x) d.wsum[v] = 0ull;
    } else {
        for (int64_t v = i; v < d.n; v += (int64_t)gridDim.x * blockDim.x) d.cnt[v] = 0u;
    }
}

// s_hat(s, v) = cnt[v] / R; the pair (s, s) meets at step 0 for every j.
// Stratified (Algorithm 2): s~(s, v) = wsum[v] 2^-40 / z, and the variant
// normalised by the N pairs, s~(s, v) N / z; both are 1 at v = s.
__device__ __forceinline__ void estimate_one(const QueryDesc &d, int64_t v) {
    if (strat_kind(d.kind)) {
        const double x = (double)d.wsum[v] * 9.094947017729282379150390625e-13;   // 2^-40
        const double e = x / d.z;
        if (d.out) d.out[v] = (v == d.s) ? 1.0 : e;
        if (d.out_n) d.out_n[v] = (v == d.s) ? 1.0 : e * ((double)d.R / d.z);
        return;
    }
    if (v == d.s) d.cnt[v] = (uint32_t)d.R;
    if (d.out) d.out[v] = (v == d.s) ? 1.0 : (double)d.cnt[v] / (double)d.R;
}

// grid (x over nodes, y = query)
__global__ void k_estimate(const QueryDesc *__restrict__ qd) {
    const QueryDesc &d = qd[blockIdx.y];
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < d.n;
         v += (int64_t)gridDim.x * blockDim.x)
        estimate_one(d, v);
}

// ------------------------------------------------------------ source walks
// Walk (s, j) for j < R: positions 1..len as o() values.  Stratified: walk j
// of s is the fixed-length walk generated in slot pi_s(j); its class goes to
// scls[j].  grid (x over j, y = query)
__global__ __launch_bounds__(256) void k_source_walks(const QueryDesc *__restrict__ qd,
                                                      unsigned long long *__restrict__ counters) {
    const QueryDesc &d = qd[blockIdx.y];
    const int32_t j = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t steps = 0;
    if (j < d.R) {
        const PhiloxKey key{d.k0, d.k1};
        uint32_t *row = d.sw + (size_t)j * d.L;
        uint2 cur = d.nodes[d.s];
        int32_t len = 0;
        if (strat_kind(d.kind)) {
            const uint4 fk = philox4x32_10((uint32_t)d.s, 0u, 0u, DOM_SHUFFLE, key);
            const uint32_t r = shuffle_slot((uint32_t)j, (uint32_t)d.R, (uint32_t)d.sa, (uint32_t)d.sb, fk);
            const uint32_t cls = slot_class(r, d.tab->ccum, d.L);
            for (int32_t t = 1; t <= (int32_t)cls; ++t) {
                if (cur.y == 0) break;
                const uint4 x = philox4x32_10((uint32_t)d.s, r, (uint32_t)t, DOM_STRAT, key);
                cur = d.E[cur.x + pick32(x.y, cur.y)];
                row[t - 1] = cur.x;
                len = t;
            }
            d.scls[j] = (uint8_t)cls;
        } else {
            const bool stitched = d.kind == K_STITCHED || d.kind == K_GROUPED_STITCHED;
            const int32_t head = stitched ? min(d.ix.seg_len, d.L) : d.L;
            for (int32_t t = 1; t <= head; ++t) {
                const uint4 x = philox4x32_10((uint32_t)d.s, (uint32_t)j, (uint32_t)t, DOM_WALK, key);
                if (x.x >= d.T || cur.y == 0) break;
                cur = d.E[cur.x + pick32(x.y, cur.y)];
                row[t - 1] = cur.x;
                len = t;
            }
            if (stitched && len == d.ix.seg_len && len < d.L) {
                const uint32_t y = d.ix.node_of[cur.x];
                const uint32_t sigma = entry_slot(d.ix, key, (uint32_t)d.s, (uint32_t)j, y);
                for (int32_t mm = 0; mm < d.ix.width && len < d.L; ++mm) {
                    const uint32_t sg = d.ix.chain[(size_t)sigma * d.ix.width + mm];
                    if (sg == NIL) break;
                    const int32_t sl = d.ix.seg_lens[sg];
                    for (int32_t u = 0; u < sl && len < d.L; ++u) {
                        row[len] = d.ix.seg[(size_t)sg * d.ix.seg_len + u];
                        ++len;
                    }
                    if (sl < d.ix.seg_len) break;
                }
            }
        }
        d.slen[j] = (uint8_t)len;
        steps = (uint32_t)len;
    }
    unsigned long long m64 = steps;
    for (int dd = 32; dd > 0; dd >>= 1) m64 += __shfl_xor(m64, dd, 64);
    if ((threadIdx.x & 63) == 0 && m64) atomicAdd(&counters[C_SRC_MOVES], m64);
}

// ------------------------------------------------------------ compaction
// One block per query.  Keeps the walks with at least one step (a walk of
// length 0 can only meet at step 0, i.e. only the source itself), packs their
// positions back to back (swc), and cuts the packed list into tiles that fit
// the meet kernel's LDS: with the kind's shape (TJ walks, TN positions), each
// tile is the longest run of walks from the previous one's end that holds at
// most TJ walks and TN positions (cut_tiles).
__global__ __launch_bounds__(1024) void k_compact(const QueryDesc *__restrict__ qd) {
    const QueryDesc &d = qd[blockIdx.x];
    if (d.kind >= K_GROUPED) return;   // compacted with its group
    const int32_t R = d.R, L = d.L;
    const uint32_t TJ = (uint32_t)d.tile_j;
    const uint32_t TN = (uint32_t)tile_nodes_of(d.kind);
    const int32_t per = (R + blockDim.x - 1) / blockDim.x;
    const int32_t j0 = min(R, (int32_t)threadIdx.x * per), j1 = min(R, j0 + per);
    uint32_t cnt = 0, nodes = 0;
    for (int32_t j = j0; j < j1; ++j) {
        const uint32_t l = d.slen[j];
        cnt += l > 0;
        nodes += l;
    }
    uint32_t R1, total;
    const uint32_t kb = block_excl_sum(cnt, &R1);
    const uint32_t nb = block_excl_sum(nodes, &total);
    uint32_t k = kb, off = nb;
    for (int32_t j = j0; j < j1; ++j) {
        const uint32_t l = d.slen[j];
        if (!l) continue;
        d.jj[k] = (uint32_t)j;
        d.joff[k] = off;
        const uint32_t *src = d.sw + (size_t)j * L;
        for (uint32_t t = 0; t < l; ++t) d.swc[off + t] = src[t];
        ++k;
        off += l;
    }
    if (threadIdx.x == 0) d.joff[R1] = total;
    __syncthreads();
    if (threadIdx.x < 64) {
        const uint32_t n_tiles = cut_tiles(d.joff, R1, TJ, TN, d.tiles, (int)threadIdx.x);
        if (threadIdx.x == 0) {
            d.tiles[n_tiles] = R1;
            d.meta[0] = R1;
            d.meta[1] = total;
            d.meta[2] = n_tiles;
        }
    }
}

// Work-unit offsets of the queries (one block): one list of nq + 1 offsets per
// kind (a query of another kind has no units in a list), then one cursor per
// kind.
__global__ __launch_bounds__(1024) void k_unit_offsets(const QueryDesc *__restrict__ qd, int32_t nq,
                                                       uint32_t *__restrict__ units) {
    const int32_t per = (nq + blockDim.x - 1) / blockDim.x;
    const int32_t q0 = min(nq, (int32_t)threadIdx.x * per), q1 = min(nq, q0 + per);
    for (int list = 0; list < N_KINDS; ++list) {
        uint32_t sum = 0;
        for (int32_t q = q0; q < q1; ++q)
            if (qd[q].kind == list) sum += qd[q].meta[2] * (uint32_t)qd[q].n_chunks;
        uint32_t total;
        uint32_t run = block_excl_sum(sum, &total);
        uint32_t *u = units + list * (nq + 1);
        for (int32_t q = q0; q < q1; ++q) {
            u[q] = run;
            if (qd[q].kind == list) run += qd[q].meta[2] * (uint32_t)qd[q].n_chunks;
        }
        if (threadIdx.x == 0) {
            u[nq] = total;
            units[N_KINDS * (nq + 1) + list] = 0u;
        }
    }
}

// ------------------------------------------------------------ meet kernel
//
// Persistent blocks take work units from a device cursor.  A unit is (query,
// tile of its source walks, chunk of vb of its nodes with in-edges); the units
// of all queries of a launch form one list, so queries on graphs of any size
// share the launch and its tail.  A block stages its tile (walk ids, packed
// positions) in LDS once and keeps it while consecutive units share it, and
// stages the chunk's nodes (id, row) per unit.
//
// Inside a unit the pairs (v, k), v-major, are handed out from one block-wide
// cursor in chunks of 64 to the waves, so all waves of a block work on the same
// one or two nodes v at a time: the rows a walk reads at its first two steps
// (v's own row and those of its in-neighbours) are then shared by the whole
// block and stay in the CU's L1.  Each lane runs NS independent pairs (slots)
// so that NS gathers per lane are in flight at once; a slot whose pair ended
// (stop, meet, or end of walk (s, j)) is refilled before the next step.
// A step: one Philox draw, a multiply-high neighbour pick, one 8-byte gather
// of E, one LDS compare.  Meets go to an LDS counter per node, flushed to the
// global counts once per unit.
//
// KIND selects the walks: K_PLAIN (sqrt(c)-walks), K_STITCHED (private head,
// then a tail read from the segment index) or K_STRAT (the stratified
// estimator's fixed-length walks: walk j of v has the class of slot pi_v(j),
// takes no stop draw, and a meet adds Lemma 5's weight of the two classes).
//
// Stitched walks run their private heads (the first 2^k steps, the plain
// walk's own draws) exactly as plain walks do.  A pair whose head made all its
// moves with both walks alive and apart is not continued on its slot: it goes
// to the wave's tail queue in LDS (unit-local node, tile entry, position) and
// the slot takes a new pair.  Whenever the queue holds a wave's worth of
// pairs, and once more when the unit's pairs are done, the wave follows 64
// queued tails at once through the index (the end node's pool slot drawn with
// (v, j, 0, 2), then the chain of segments), comparing with the tile in LDS.
// Heads thus keep the plain kernel's shape and rate, and the rarer tails do
// not hold slots of their own.

// Serving (STREAM): wave 0 of a block claims the next units from the ring:
// among published entries of the kernel's kind with unclaimed units, the
// oldest (smallest seq), all read from the entries' claim words alone; the
// claim is a compare-and-swap (acquire) that counts down up to RING_RUN
// consecutive units (consecutive node chunks of one tile).  A failed swap
// means another block took them, or the entry was republished: look again.
// The block fences only when it moves to a request it has not worked on
// (below), so its caches keep the graph's rows from unit to unit.
// *o_slot = RING_MAX when no entry has units left.
constexpr uint32_t RING_RUN = 4;
template <int KIND>
__device__ void ring_claim(const StreamRing &ring, int lane, uint32_t *o_slot, uint32_t *o_unit,
                           uint32_t *o_count, uint32_t *o_seq) {
    for (;;) {
        unsigned long long key = ~0ull, c = 0ull;
        if (lane < ring.entries) {
            c = __hip_atomic_load(&ring.ctl[lane].claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t tag = (uint32_t)(c >> 32), left = (uint32_t)c;
            if (tag != 0u && (tag & 3u) == (uint32_t)KIND && left > 0u)
                key = ((unsigned long long)(tag >> 2) << 32) | (uint32_t)lane;
        }
        for (int off = 32; off > 0; off >>= 1) {
            const unsigned long long o = __shfl_xor(key, off, 64);
            key = o < key ? o : key;
        }
        if (key == ~0ull) {
            if (lane == 0) *o_slot = RING_MAX;
            return;
        }
        const int best = (int)(uint32_t)key;
        const unsigned long long cb = __shfl(c, best, 64);
        const uint32_t left = (uint32_t)cb;
        const uint32_t take = min(RING_RUN, left);
        bool won = false;
        if (lane == 0) {
            unsigned long long expect = cb;
            won = __hip_atomic_compare_exchange_strong(&ring.ctl[best].claim, &expect, cb - take,
                                                       __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                       __HIP_MEMORY_SCOPE_AGENT);
            if (won) {
                const uint32_t nu = __hip_atomic_load(&ring.ctl[best].n_units, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
                *o_slot = (uint32_t)best;
                *o_unit = nu - left;
                *o_count = take;
                *o_seq = (uint32_t)(cb >> 34);
            }
        }
        if (__shfl((int)won, 0, 64)) return;
    }
}

// Serving: a block reports `units` finished units of ring entry `slot`
// (request `tag`) and the work it did on them (the lanes' counters, which it
// then clears); the block whose report completes the entry writes the
// request's estimate and then its flag in host memory.  Block-wide.
__device__ void ring_report(const StreamRing &ring, const QueryDesc &d, uint32_t slot,
                            uint32_t tag, uint32_t units, int lane, uint32_t &st_moves,
                            uint32_t &st_draws, uint32_t &st_meets, uint32_t &st_tail,
                            uint32_t &st_pairs, uint32_t *s_last) {
    unsigned long long w0 = st_moves, w1 = st_draws, w2 = st_meets, w3 = st_tail, w4 = st_pairs;
    for (int dd = 32; dd > 0; dd >>= 1) {
        w0 += __shfl_xor(w0, dd, 64);
        w1 += __shfl_xor(w1, dd, 64);
        w2 += __shfl_xor(w2, dd, 64);
        w3 += __shfl_xor(w3, dd, 64);
        w4 += __shfl_xor(w4, dd, 64);
    }
    unsigned long long *ec = ring.counters + (size_t)slot * 8;
    if (lane == 0) {
        if (w0) atomicAdd(&ec[C_MOVES], w0);
        if (w1) atomicAdd(&ec[C_DRAWS], w1);
        if (w2) atomicAdd(&ec[C_MEETS], w2);
        if (w3) atomicAdd(&ec[C_TAIL], w3);
        if (w4) atomicAdd(&ec[C_PAIRS], w4);
    }
    st_moves = st_draws = st_meets = st_tail = st_pairs = 0;
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) {
        // the size is read coherently: a plain load could return the size of
        // an earlier request in this entry from a cache and miss the last unit
        const uint32_t old = atomicAdd(&ring.ctl[slot].done, units);
        const uint32_t nu =
            __hip_atomic_load(&ring.ctl[slot].n_units, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *s_last = (old + units == nu) ? 1u : 0u;
    }
    __syncthreads();
    if (*s_last) {
        __threadfence();
        for (int64_t v = threadIdx.x; v < d.n; v += blockDim.x) estimate_one(d, v);
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_store(&ring.flags[slot], tag, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
    __syncthreads();
}

template <int KIND, int NS, bool STREAM>
__global__ __launch_bounds__(meet_block_of(KIND)) void k_meet(const QueryDesc *__restrict__ qd, int32_t nq,
                                                     const uint32_t *__restrict__ ustart,
                                                     uint32_t *__restrict__ cursor,
                                                     unsigned long long *__restrict__ counters,
                                                     StreamRing ring) {
    constexpr bool STITCHED = KIND == K_STITCHED;
    constexpr bool STRAT = KIND == K_STRAT;
    constexpr int TJ = tile_j_of(KIND), TN = tile_nodes_of(KIND);
    __shared__ uint32_t s_nodes[TN];
    __shared__ uint32_t s_j[TJ];
    __shared__ uint16_t s_off[TJ + 1];
    __shared__ uint32_t s_cnt[STRAT ? 1 : MEET_VB];
    __shared__ uint32_t s_vid[MEET_VB];
    __shared__ uint2 s_vrow[MEET_VB];
    __shared__ uint32_t s_unit, s_item, s_slot, s_seq, s_last, s_run;
    // stratified: classes of the tile's source walks, class starts, the
    // shuffle keys of the unit's nodes, weighted sums
    __shared__ uint8_t s_cls[STRAT ? TJ : 1];
    __shared__ uint32_t s_ccum[STRAT ? MAX_CAP + 2 : 1];
    __shared__ uint4 s_fk[STRAT ? MEET_VB : 1];
    __shared__ unsigned long long s_w[STRAT ? MEET_VB : 1];
    __shared__ uint2 s_q[STRAT ? meet_block_of(KIND) : 1];   // 64 prepared pairs per wave
    // stitched: per-wave ring of pairs waiting for their tails, (vl << 16 | k, o)
    __shared__ uint2 s_tq[STITCHED ? (meet_block_of(KIND) / 64) * TAIL_Q : 1];

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const uint32_t n_units = STREAM ? 0u : ustart[nq];
    uint32_t tq_head = 0, tq_tail = 0;   // stitched: the wave's tail ring (wave-uniform)
    // serving: the request whose finished units this block has not reported yet
    uint32_t acc_slot = 0, acc_tag = 0, acc_units = 0;
    uint32_t run_next = 0, run_left = 0;   // serving: claimed units not yet taken
    uint32_t cur_q = 0xffffffffu, cur_tile = 0xffffffffu;
    uint32_t K = 0;
    uint32_t st_moves = 0, st_draws = 0, st_meets = 0, st_tail = 0, st_pairs = 0;

    for (;;) {
        uint32_t unit = 0, tag_s = 0;
        if constexpr (STREAM) {
            if (run_left == 0u) {
                if (threadIdx.x < 64) ring_claim<KIND>(ring, lane, &s_slot, &s_unit, &s_run, &s_seq);
                __syncthreads();
                run_next = s_unit;
                run_left = s_slot < (uint32_t)RING_MAX ? s_run : 0u;
            }
            const uint32_t nslot = s_slot, nseq = s_seq;
            unit = run_next++;
            if (run_left) --run_left;
            // the block reports the units it finished of a request, and their
            // work, once: when it moves on to another request or runs out
            if (acc_units && (nslot >= (uint32_t)RING_MAX || nseq != acc_tag)) {
                ring_report(ring, qd[acc_slot], acc_slot, acc_tag, acc_units, lane,
                            st_moves, st_draws, st_meets, st_tail, st_pairs, &s_last);
                acc_units = 0;
            }
            if (nslot >= (uint32_t)RING_MAX) break;
            tag_s = nseq;
            // a request this block has not worked on: see its descriptor and
            // buffers as its publication left them
            if (tag_s != cur_q) __threadfence();
        } else {
            if (threadIdx.x == 0) s_unit = atomicAdd(cursor, 1u);
            __syncthreads();
            unit = s_unit;
            if (unit >= n_units) break;
        }
        int32_t lo = 0;
        if constexpr (STREAM) {
            lo = (int32_t)s_slot;
        } else {
            // query of the unit: the last q with ustart[q] <= unit
            int32_t hi = nq;
            while (hi - lo > 1) {
                const int32_t mid = (lo + hi) >> 1;
                if (ustart[mid] <= unit) lo = mid; else hi = mid;
            }
        }
        const int32_t q = lo;
        const uint32_t local = STREAM ? unit : unit - ustart[q];
        const uint32_t tag = STREAM ? tag_s : (uint32_t)q;
        const QueryDesc &d = qd[q];
        const int32_t n_chunks = (int32_t)uni((uint32_t)d.n_chunks);
        const int32_t vb = (int32_t)uni((uint32_t)d.vb);
        const uint32_t tile = local / (uint32_t)n_chunks;
        const uint32_t chunk = local - tile * (uint32_t)n_chunks;
        const PhiloxKey key{uni(d.k0), uni(d.k1)};
        const uint32_t T = uni(d.T);
        const int32_t src = (int32_t)uni((uint32_t)d.s);
        const uint32_t NN = uni((uint32_t)d.R), sa = uni((uint32_t)d.sa), sb = uni((uint32_t)d.sb);
        const int32_t phi = (int32_t)uni((uint32_t)d.L);
        if (tag != cur_q || tile != cur_tile) {
            const uint32_t k0 = d.tiles[tile], k1 = d.tiles[tile + 1];
            const uint32_t nb = d.joff[k0], ne = d.joff[k1];
            K = k1 - k0;
            for (uint32_t i = threadIdx.x; i < K; i += blockDim.x) {
                const uint32_t jw = d.jj[k0 + i];
                s_j[i] = jw;
                s_off[i] = (uint16_t)(d.joff[k0 + i] - nb);
                if (STRAT) s_cls[i] = d.scls[jw];
            }
            if (threadIdx.x == 0) s_off[K] = (uint16_t)(ne - nb);
            for (uint32_t i = threadIdx.x; i < ne - nb; i += blockDim.x) s_nodes[i] = d.swc[nb + i];
            if (STRAT)
                for (uint32_t i = threadIdx.x; i < (uint32_t)phi + 2; i += blockDim.x)
                    s_ccum[i] = d.tab->ccum[i];
            cur_q = tag;
            cur_tile = tile;
        }
        const int32_t vbase = (int32_t)chunk * vb;
        const uint32_t nv = (uint32_t)min(vb, d.n_active - vbase);
        for (uint32_t i = threadIdx.x; i < MEET_VB; i += blockDim.x) {
            if (STRAT) s_w[i] = 0ull; else s_cnt[i] = 0u;
            if (i < nv) {
                const uint32_t id = (uint32_t)d.active[vbase + (int32_t)i];
                s_vid[i] = id;
                s_vrow[i] = d.nodes[id];
                if (STRAT) s_fk[i] = philox4x32_10(id, 0u, 0u, DOM_SHUFFLE, key);
            }
        }
        if (threadIdx.x == 0) s_item = 0u;
        __syncthreads();

        // Pairs of the unit: item i = vl * K + k for node vl < nv and walk k < K.
        const uint32_t total = nv * K;
        // wave-uniform chunk of items [ci, ce) and the (node, walk) of item ci
        uint32_t ci = 0, ce = 0, cvl = 0, ck = 0;
        bool drained = false;
        uint32_t qh = 0, qn = 0;   // stratified: the wave's queue of prepared pairs [qh, qn)

        Slot sl[NS];
#pragma unroll
        for (int qq = 0; qq < NS; ++qq) sl[qq].busy = false;

        // Stitched: follow the tails of the first `c` queued pairs (one per
        // lane) through the index; meets go to the unit's LDS counters.
        auto drain_tails = [&](uint32_t c) {
            if (lane < (int)c) {
                const uint2 r = s_tq[wave * TAIL_Q + ((tq_head + (uint32_t)lane) & (TAIL_Q - 1))];
                const uint32_t vl = r.x >> 16, k = r.x & 0xffffu;
                const uint32_t base = s_off[k];
                const uint32_t len = (uint32_t)s_off[k + 1] - base;
                const uint32_t seg_len = (uint32_t)d.ix.seg_len, width = (uint32_t)d.ix.width;
                const uint32_t y = d.ix.node_of[r.y];
                const int64_t pb = d.ix.pool_off[y];
                const int64_t pe = d.ix.pool_off[y + 1];
                const uint4 x = philox4x32_10(s_vid[vl], s_j[k], 0u, DOM_ENTRY, key);
                const uint32_t sigma = (uint32_t)(pb + (int64_t)pick64(x.x, (uint64_t)(pe - pb)));
                const uint32_t *crow = d.ix.chain + (size_t)sigma * width;
                uint32_t t = seg_len;
                bool done = false;
                for (uint32_t mm = 0; mm < width && !done; ++mm) {
                    const uint32_t sg = crow[mm];
                    if (sg == NIL) break;
                    const uint32_t sln = d.ix.seg_lens[sg];
                    const uint32_t *srow = d.ix.seg + (size_t)sg * seg_len;
                    for (uint32_t u = 0; u < sln; ++u) {
                        ++t;
                        ++st_tail;
                        if (srow[u] == s_nodes[base + t - 1]) {
                            atomicAdd(&s_cnt[vl], 1u);
                            ++st_meets;
                            done = true;
                            break;
                        }
                        if (t == len) {
                            done = true;
                            break;
                        }
                    }
                    if (sln < seg_len) break;
                }
            }
            tq_head += c;
        };

        for (;;) {
            // ---- refill idle slots from the block's cursor; a lane whose item
            // has nothing to walk (the source's own pair, or a stratified walk
            // of length 0) takes the next item
            if constexpr (STRAT) {
                // A pair's shuffle and class search cost about a hundred
                // instructions: they are done for 64 items at once by all
                // lanes of the wave, and the pairs with steps to walk wait in
                // the wave's queue in LDS until slots free up.
#pragma unroll
                for (int qq = 0; qq < NS; ++qq) {
                    uint64_t need = __ballot(!sl[qq].busy);
                    while (need != 0ull) {
                        if (qh == qn) {
                            if (drained) break;
                            uint32_t x = 0;
                            if (lane == 0) x = atomicAdd(&s_item, ITEM_CHUNK);
                            x = __builtin_amdgcn_readfirstlane(x);
                            if (x >= total) {
                                drained = true;
                                break;
                            }
                            const uint32_t item = x + (uint32_t)lane;
                            bool ok = item < total;
                            uint32_t vl = 0, k = 0, r = 0, cv = 0;
                            if (ok) {
                                vl = item / K;
                                k = item - vl * K;
                                ok = (int32_t)s_vid[vl] != src;
                            }
                            if (ok) {
                                r = shuffle_slot(s_j[k], NN, sa, sb, s_fk[vl]);
                                cv = slot_class(r, s_ccum, phi);
                                ok = cv > 0u;
                            }
                            const uint64_t m = __ballot(ok);
                            if (ok) s_q[wave * 64 + lane_rank(m)] = make_uint2((vl << 24) | (k << 8) | cv, r);
                            qn = (uint32_t)__popcll(m);
                            qh = 0;
                            continue;
                        }
                        const uint32_t want = (uint32_t)__popcll(need);
                        const uint32_t avail = qn - qh;
                        const uint32_t take = avail < want ? avail : want;
                        const uint32_t rank = lane_rank(need);
                        const bool mine = ((need >> lane) & 1ull) && rank < take;
                        if (mine) {
                            const uint2 e = s_q[wave * 64 + qh + rank];
                            const uint32_t vl = e.x >> 24, k = (e.x >> 8) & 0xffffu, cv = e.x & 0xffu;
                            const uint32_t base = s_off[k];
                            const uint32_t len = min((uint32_t)s_off[k + 1] - base, cv);
                            const uint2 row = s_vrow[vl];
                            sl[qq].aux = ((uint32_t)s_cls[k] << 8) | cv;
                            sl[qq].rng = walk_draws_begin(s_vid[vl], e.y, key, DOM_STRAT);
                            sl[qq].pos = base | (len << 16) | (vl << 24);
                            sl[qq].t = 0;
                            sl[qq].o = row.x;
                            sl[qq].d = row.y;
                            sl[qq].busy = true;
                            ++st_pairs;
                        }
                        need &= ~__ballot(mine);
                        qh += take;
                    }
                }
            } else {
#pragma unroll
                for (int qq = 0; qq < NS; ++qq) {
                    uint64_t need = __ballot(!sl[qq].busy);
                    while (need != 0ull) {
                        if (ci == ce) {
                            if (drained) break;
                            uint32_t x = 0;
                            if (lane == 0) x = atomicAdd(&s_item, ITEM_CHUNK);
                            x = __builtin_amdgcn_readfirstlane(x);
                            if (x >= total) {
                                drained = true;
                                break;
                            }
                            ci = x;
                            ce = min(x + ITEM_CHUNK, total);
                            cvl = x / K;
                            ck = x - cvl * K;
                        }
                        const uint32_t want = (uint32_t)__popcll(need);
                        const uint32_t avail = ce - ci;
                        const uint32_t take = avail < want ? avail : want;
                        const uint32_t rank = lane_rank(need);
                        const bool mine = ((need >> lane) & 1ull) && rank < take;
                        bool filled = false;
                        if (mine) {
                            uint32_t k = ck + rank, vl = cvl;
                            while (k >= K) {
                                k -= K;
                                ++vl;
                            }
                            const uint32_t id = s_vid[vl];
                            if ((int32_t)id != src) {   // the source's own pairs are not walked
                                const uint32_t base = s_off[k];
                                const uint32_t len = (uint32_t)s_off[k + 1] - base;
                                const uint2 row = s_vrow[vl];
                                sl[qq].rng = walk_draws_begin(id, s_j[k], key);
                                sl[qq].pos = base | (len << 16) | (vl << 24);
                                sl[qq].t = 0;
                                sl[qq].o = row.x;
                                sl[qq].d = row.y;
                                sl[qq].busy = true;
                                if (STITCHED) sl[qq].aux = k;
                                filled = true;
                                ++st_pairs;
                            }
                        }
                        need &= ~__ballot(filled);
                        ci += take;
                        ck += take;
                        while (ck >= K && K > 0) {
                            ck -= K;
                            ++cvl;
                        }
                    }
                }
            }
            bool any = false;
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) any |= sl[qq].busy;
            // A refill round can hand out only pairs with nothing to walk: a
            // wave leaves only once the block's cursor is drained.
            if (__ballot(any) == 0ull) {
                if (drained && qh == qn) {
                    if constexpr (STITCHED) {
                        while (tq_tail != tq_head) drain_tails(min(64u, tq_tail - tq_head));
                    }
                    break;
                }
                continue;
            }

            // ---- head steps: draws, then all gathers, then the compares
            bool go[NS];
            uint32_t at[NS];
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) {
                go[qq] = false;
                at[qq] = 0;
                if (sl[qq].busy) {
                    ++sl[qq].t;
                    const uint2 x = walk_draw_next(sl[qq].rng, key);
                    ++st_draws;
                    if (!STRAT && x.x >= T) {
                        sl[qq].busy = false;
                    } else {
                        go[qq] = true;
                        at[qq] = sl[qq].o + pick32(x.y, sl[qq].d);
                    }
                }
            }
            // all gathers of the lane's slots, then the compares
            uint2 e[NS];
#pragma unroll
            for (int qq = 0; qq < NS; ++qq)
                if (go[qq]) e[qq] = load_edge(d.E + at[qq]);
            bool tails[NS];
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) tails[qq] = false;
#pragma unroll
            for (int qq = 0; qq < NS; ++qq) {
                if (!go[qq]) continue;
                ++st_moves;
                Slot &w = sl[qq];
                w.o = e[qq].x;
                w.d = e[qq].y;
                const uint32_t base = w.pos & 0xffffu, len = (w.pos >> 16) & 0xffu;
                if (w.o == s_nodes[base + w.t - 1]) {
                    if (STRAT)
                        atomicAdd(&s_w[w.pos >> 24], strat_weight(d.tab->a, w.aux >> 8, w.aux & 0xffu));
                    else
                        atomicAdd(&s_cnt[w.pos >> 24], 1u);
                    ++st_meets;
                    w.busy = false;
                } else if (w.t == len || w.d == 0u) {
                    w.busy = false;
                } else if (STITCHED && w.t == (uint32_t)d.ix.seg_len) {
                    w.busy = false;   // the head made all its moves: its tail is queued
                    tails[qq] = true;
                }
            }
            if constexpr (STITCHED) {
                // queue the pairs whose heads ended open (tails[qq]), then
                // follow queued tails while a wave's worth is waiting
                bool any_tail = false;
#pragma unroll
                for (int qq = 0; qq < NS; ++qq) any_tail |= tails[qq];
                if (__ballot(any_tail) != 0ull) {
#pragma unroll
                    for (int qq = 0; qq < NS; ++qq) {
                        const uint64_t m = __ballot(tails[qq]);
                        if (tails[qq])
                            s_tq[wave * TAIL_Q + ((tq_tail + lane_rank(m)) & (TAIL_Q - 1))] =
                                make_uint2(((sl[qq].pos >> 24) << 16) | sl[qq].aux, sl[qq].o);
                        tq_tail += (uint32_t)__popcll(m);
                        if (tq_tail - tq_head >= 64u) drain_tails(64u);
                    }
                }
            }
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < nv; i += blockDim.x) {
            if (STRAT) {
                const unsigned long long c = s_w[i];
                if (c) atomicAdd(&d.wsum[s_vid[i]], c);
            } else {
                const uint32_t c = s_cnt[i];
                if (c) atomicAdd(&d.cnt[s_vid[i]], c);
            }
        }
        if constexpr (STREAM) {
            ++acc_units;
            acc_slot = (uint32_t)q;
            acc_tag = tag;
        }
    }
    if constexpr (STREAM) return;

    unsigned long long v0 = st_moves, v1 = st_draws, v2 = st_meets, v3 = st_tail, v4 = st_pairs;
    for (int dd = 32; dd > 0; dd >>= 1) {
        v0 += __shfl_xor(v0, dd, 64);
        v1 += __shfl_xor(v1, dd, 64);
        v2 += __shfl_xor(v2, dd, 64);
        v3 += __shfl_xor(v3, dd, 64);
        v4 += __shfl_xor(v4, dd, 64);
    }
    if (lane == 0) {
        atomicAdd(&counters[C_MOVES], v0);
        atomicAdd(&counters[C_DRAWS], v1);
        atomicAdd(&counters[C_MEETS], v2);
        atomicAdd(&counters[C_TAIL], v3);
        atomicAdd(&counters[C_PAIRS], v4);
    }
}

// ------------------------------------------------------ walk materialisation

struct WalkArgs {
    const uint2 *nodes;
    const uint2 *E;
    IndexView ix;
    const int32_t *vs;
    const uint32_t *js;
    int64_t count;
    int32_t *paths;   // [count][L+1]
    int32_t *lens;
    PhiloxKey key;
    uint32_t T;
    int32_t L;
};

template <bool STITCHED>
__global__ __launch_bounds__(256) void k_walks(WalkArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    int32_t *row = a.paths + (size_t)i * (a.L + 1);
    const uint32_t v = (uint32_t)a.vs[i], j = a.js[i];
    row[0] = (int32_t)v;
    uint2 cur = a.nodes[v];
    const int32_t head = STITCHED ? min(a.ix.seg_len, a.L) : a.L;
    int32_t len = 0;
    for (int32_t t = 1; t <= head; ++t) {
        const uint4 x = philox4x32_10(v, j, (uint32_t)t, DOM_WALK, a.key);
        if (x.x >= a.T || cur.y == 0) break;
        cur = a.E[cur.x + pick32(x.y, cur.y)];
        row[t] = (int32_t)a.ix.node_of[cur.x];
        len = t;
    }
    if (STITCHED && len == a.ix.seg_len && len < a.L) {
        const uint32_t sigma = entry_slot(a.ix, a.key, v, j, (uint32_t)row[len]);
        for (int32_t mm = 0; mm < a.ix.width && len < a.L; ++mm) {
            const uint32_t sg = a.ix.chain[(size_t)sigma * a.ix.width + mm];
            if (sg == NIL) break;
            const int32_t sl = a.ix.seg_lens[sg];
            for (int32_t u = 0; u < sl && len < a.L; ++u) {
                ++len;
                row[len] = (int32_t)a.ix.node_of[a.ix.seg[(size_t)sg * a.ix.seg_len + u]];
            }
            if (sl < a.ix.seg_len) break;
        }
    }
    for (int32_t t = len + 1; t <= a.L; ++t) row[t] = -1;
    a.lens[i] = len;
}

// Stratified: walk j of v after the shuffle (the fixed-length walk of slot
// pi_v(j)); paths hold node ids, row[0] = v.
struct StratWalkArgs {
    const uint2 *nodes;
    const uint2 *E;
    const uint32_t *node_of;
    const StratTab *tab;
    const int32_t *vs;
    const uint32_t *js;
    int64_t count;
    int32_t *paths;   // [count][phi+1] or NULL
    int32_t *lens;    // or NULL
    uint32_t *slots;  // or NULL
    int32_t *classes; // or NULL
    PhiloxKey key;
    uint32_t N, sa, sb;
    int32_t phi;
};

__global__ __launch_bounds__(256) void k_walks_strat(StratWalkArgs a) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.count) return;
    const uint32_t v = (uint32_t)a.vs[i], j = a.js[i];
    const uint4 fk = philox4x32_10(v, 0u, 0u, DOM_SHUFFLE, a.key);
    const uint32_t r = shuffle_slot(j, a.N, a.sa, a.sb, fk);
    const uint32_t cls = slot_class(r, a.tab->ccum, a.phi);
    if (a.slots) a.slots[i] = r;
    if (a.classes) a.classes[i] = (int32_t)cls;
    if (!a.paths) return;
    int32_t *row = a.paths + (size_t)i * (a.phi + 1);
    row[0] = (int32_t)v;
    uint2 cur = a.nodes[v];
    int32_t len = 0;
    for (int32_t t = 1; t <= (int32_t)cls; ++t) {
        if (cur.y == 0) break;
        const uint4 x = philox4x32_10(v, r, (uint32_t)t, DOM_STRAT, a.key);
        cur = a.E[cur.x + pick32(x.y, cur.y)];
        row[t] = (int32_t)a.node_of[cur.x];
        len = t;
    }
    for (int32_t t = len + 1; t <= a.phi; ++t) row[t] = -1;
    a.lens[i] = len;
}

#ifndef SRK_MEET_SLOTS
#define SRK_MEET_SLOTS 2
#endif
#ifndef SRK_MEET_SLOTS_STITCHED
#define SRK_MEET_SLOTS_STITCHED 2
#endif

#ifndef SRK_MEET_SLOTS_STRAT
#define SRK_MEET_SLOTS_STRAT 2
#endif

// Resident blocks of a meet-kernel instance on the whole device (computed
// once per process; a function-local static is initialised thread-safely).
template <int KIND, int NS, bool STREAM>
int meet_grid_blocks() {
    static const int blocks = [] {
        int dev = 0, cus = 0, per = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_meet<KIND, NS, STREAM>,
                                                           meet_block_of(KIND), 0);
        if (cus <= 0) cus = 256;
        if (per <= 0) per = 1;
        return cus * per;
    }();
    return blocks;
}

template <int KIND, int NS>
void launch_meet(const QuerySet &qs, hipStream_t st) {
    const int blocks = (int)std::min<int64_t>(qs.units_bound[KIND], meet_grid_blocks<KIND, NS, false>());
    const uint32_t *ustart = qs.units + (size_t)KIND * (qs.nq + 1);
    uint32_t *cursor = qs.units + (size_t)N_KINDS * (qs.nq + 1) + KIND;
    k_meet<KIND, NS, false><<<blocks, meet_block_of(KIND), 0, st>>>(qs.desc, qs.nq, ustart, cursor,
                                                                    qs.counters, StreamRing{});
}

template <int KIND, int NS>
void launch_meet_ring(const StreamRing &ring, hipStream_t st) {
    k_meet<KIND, NS, true><<<meet_grid_blocks<KIND, NS, true>(), meet_block_of(KIND), 0, st>>>(
        ring.desc, ring.entries, nullptr, nullptr, ring.counters, ring);
}

// Publication of a ring entry, the last kernel of its request's preparation:
// the entry's unit count (tiles x node chunks, from the compaction), then its
// (seq, 0) claim word.  A request with nothing to walk is finished here:
// estimate, then its flag.  One block.
__global__ __launch_bounds__(256) void k_publish(StreamRing ring, int32_t slot, uint32_t seq) {
    const QueryDesc &d = ring.desc[slot];
    const uint32_t nu = d.meta[2] * (uint32_t)d.n_chunks;
    if (nu > 0u) {
        if (threadIdx.x == 0) {
            RingCtl &c = ring.ctl[slot];
            c.n_units = nu;
            c.done = 0u;
            c.kind = d.kind;
            c.seq = seq;
            __threadfence();
            const unsigned long long tag = ((unsigned long long)seq << 2) | (uint32_t)d.kind;
            __hip_atomic_store(&c.claim, (tag << 32) | nu, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
        return;
    }
    for (int64_t v = threadIdx.x; v < d.n; v += blockDim.x) estimate_one(d, v);
    __threadfence_system();
    __syncthreads();
    if (threadIdx.x == 0)
        __hip_atomic_store(&ring.flags[slot], seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

}  // namespace

IndexView index_view(const Graph *g) {
    IndexView v{};
    v.node_of = g->node_of;
    if (g->index) {
        v.pool_off = g->index->pool_off;
        v.seg = g->index->seg;
        v.seg_lens = g->index->seg_lens;
        v.chain = g->index->chain;
        v.seg_len = g->index->seg_len;
        v.width = g->index->width;
    }
    return v;
}

// Tiles of R walks of cap L, at most, for any kind and any tile a query may be
// given (the smallest shape).
int32_t max_tiles_for(int32_t R, int32_t L) {
    const int64_t TJ =
        std::min({MIN_TILE_J, tile_j_of(K_PLAIN), tile_j_of(K_STITCHED), tile_j_of(K_STRAT)});
    const int64_t NW =
        std::min({tile_nodes_of(K_PLAIN), tile_nodes_of(K_STITCHED), tile_nodes_of(K_STRAT)}) - L;
    return (int32_t)(2 + R / TJ + ((int64_t)R * L) / NW);
}

// Nodes per work unit: small graphs use small chunks so that their units
// still spread over all CUs; simrank_tune replaces this by a measured choice.
int32_t default_unit_nodes(const Graph *g) {
    if (g->tuned_vb > 0) return g->tuned_vb;
    if (g->n_active >= (1 << 19)) return 256;
    if (g->n_active >= (1 << 17)) return 128;
    if (g->n_active >= (1 << 15)) return 64;
    return 32;
}

void describe_query(const Graph *g, const simrank_query *q, const simrank_params &p, int mode,
                    int32_t vb, QueryDesc *d) {
    *d = QueryDesc{};
    d->nodes = g->nodes;
    d->E = g->E;
    d->active = g->active;
    d->ix = index_view(g);
    const PhiloxKey key = make_key(q->seed);
    d->k0 = key.k0;
    d->k1 = key.k1;
    d->T = p.T;
    d->n = g->n;
    d->n_active = g->n_active;
    d->s = q->s;
    d->R = p.R;
    d->L = p.L;
    d->vb = vb;
    d->n_chunks = (g->n_active + vb - 1) / vb;
    d->kind = mode == SIMRANK_MODE_STITCHED ? K_STITCHED
              : mode == SIMRANK_MODE_STRATIFIED ? K_STRAT : K_PLAIN;
    const int32_t tj = g->tuned_tile_j[d->kind];
    d->tile_j = tj > 0 ? std::min<int32_t>(tj, tile_j_of(d->kind)) : tile_j_of(d->kind);
}

int launch_query_set(const QuerySet &qs, hipStream_t st, hipEvent_t ev_meet0, hipEvent_t ev_meet1) {
    if (qs.nq <= 0) return SIMRANK_OK;
    const unsigned nq = (unsigned)qs.nq;
    const unsigned gx_n = std::min<unsigned>(grid_for(std::max(qs.max_n, 1), 256), 1024u);
    k_init<<<dim3(gx_n, nq), 256, 0, st>>>(qs.desc, qs.counters);
    k_source_walks<<<dim3(grid_for(qs.max_R, 256), nq), 256, 0, st>>>(qs.desc, qs.counters);
    k_compact<<<nq, 1024, 0, st>>>(qs.desc);
    k_unit_offsets<<<1, 1024, 0, st>>>(qs.desc, qs.nq, qs.units);
    if (ev_meet0) SRK_HIP(hipEventRecord(ev_meet0, st));
    if (qs.units_bound[K_PLAIN] > 0) launch_meet<K_PLAIN, SRK_MEET_SLOTS>(qs, st);
    if (qs.units_bound[K_STITCHED] > 0) launch_meet<K_STITCHED, SRK_MEET_SLOTS_STITCHED>(qs, st);
    if (qs.units_bound[K_STRAT] > 0) launch_meet<K_STRAT, SRK_MEET_SLOTS_STRAT>(qs, st);
    if (qs.groups && qs.groups->ng > 0) {
        const int rc = launch_groups(*qs.groups, qs.counters, st);
        if (rc) return rc;
    }
    if (ev_meet1) SRK_HIP(hipEventRecord(ev_meet1, st));
    k_estimate<<<dim3(gx_n, nq), 256, 0, st>>>(qs.desc);
    SRK_HIP(hipGetLastError());
    return SIMRANK_OK;
}

// Preparation of a served request in ring entry `slot`.  Every kernel is
// small (one wave per SIMD at most) so that it fits beside a running
// persistent meet kernel on the same CUs.
int enqueue_ring_request(const QueryDesc &d, const StreamRing &ring, int32_t slot, uint32_t seq,
                         hipStream_t st) {
    QueryDesc *qd = ring.desc + slot;
    unsigned long long *ctr = ring.counters + (size_t)slot * 8;
    const unsigned gx_n = std::min<unsigned>(grid_for(std::max(d.n, 1), 256), 1024u);
    k_set_desc<<<1, 1, 0, st>>>(qd, d);
    k_init<<<dim3(gx_n, 1), 256, 0, st>>>(qd, ctr);
    k_source_walks<<<dim3(grid_for(d.R, 256), 1), 256, 0, st>>>(qd, ctr);
    k_compact<<<1, 256, 0, st>>>(qd);
    k_publish<<<1, 256, 0, st>>>(ring, slot, seq);
    SRK_HIP(hipGetLastError());
    return SIMRANK_OK;
}

int launch_ring_meet(int kind, const StreamRing &ring, hipStream_t st) {
    if (kind == K_PLAIN) launch_meet_ring<K_PLAIN, SRK_MEET_SLOTS>(ring, st);
    else if (kind == K_STITCHED) launch_meet_ring<K_STITCHED, SRK_MEET_SLOTS_STITCHED>(ring, st);
    else launch_meet_ring<K_STRAT, SRK_MEET_SLOTS_STRAT>(ring, st);
    SRK_HIP(hipGetLastError());
    return SIMRANK_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device bytes of one query's buffers (stratified queries: class table, walk
// classes, weighted sums and the second estimate instead of counts).
size_t request_bytes(const simrank_params &p, int mode, int32_t n) {
    const size_t RL = (size_t)p.R * (size_t)p.L;
    size_t b = align256(4 * RL) + align256((size_t)p.R) + align256(4 * (size_t)p.R) +
               align256(4 * ((size_t)p.R + 1)) + align256(4 * RL) +
               align256(4 * ((size_t)max_tiles_for(p.R, p.L) + 1)) + align256(32) +
               align256(8 * (size_t)n);
    if (mode == SIMRANK_MODE_STRATIFIED)
        b += align256(sizeof(StratTab)) + align256((size_t)p.R) + 2 * align256(8 * (size_t)n);
    else
        b += align256(4 * (size_t)n);
    return b;
}

void carve_request(const simrank_params &p, int mode, int32_t n, char *base, QueryDesc *d) {
    char *cur = base;
    auto take = [&](size_t b) {
        char *r = cur;
        cur += align256(b);
        return r;
    };
    const size_t RL = (size_t)p.R * (size_t)p.L;
    d->sw = (uint32_t *)take(4 * RL);
    d->slen = (uint8_t *)take((size_t)p.R);
    d->jj = (uint32_t *)take(4 * (size_t)p.R);
    d->joff = (uint32_t *)take(4 * ((size_t)p.R + 1));
    d->swc = (uint32_t *)take(4 * RL);
    d->tiles = (uint32_t *)take(4 * ((size_t)max_tiles_for(p.R, p.L) + 1));
    d->meta = (uint32_t *)take(32);
    d->out = (double *)take(8 * (size_t)n);
    if (mode == SIMRANK_MODE_STRATIFIED) {
        d->tab = (const StratTab *)take(sizeof(StratTab));
        d->scls = (uint8_t *)take((size_t)p.R);
        d->wsum = (unsigned long long *)take(8 * (size_t)n);
        d->out_n = (double *)take(8 * (size_t)n);
        d->cnt = nullptr;
    } else {
        d->cnt = (uint32_t *)take(4 * (size_t)n);
    }
}

// ---------------------------------------------------------------- host side

int query_params(const simrank_query *q, int32_t n, simrank_params *out, int *mode) {
    if (!q) return fail(SIMRANK_EINVAL, "query is NULL");
    if (!(q->c > 0.0 && q->c < 1.0)) return fail(SIMRANK_EINVAL, "c must lie in (0, 1)");
    if (!(q->delta > 0.0 && q->delta < 1.0)) return fail(SIMRANK_EINVAL, "delta must lie in (0, 1)");
    if (!(q->eps > 0.0 && q->eps < 1.0)) return fail(SIMRANK_EINVAL, "eps must lie in (0, 1)");
    if (q->mode != SIMRANK_MODE_PLAIN && q->mode != SIMRANK_MODE_STITCHED &&
        q->mode != SIMRANK_MODE_STRATIFIED)
        return fail(SIMRANK_EINVAL, "unknown mode");
    if (q->R_override < 0) return fail(SIMRANK_EINVAL, "R_override must be >= 0");
    if (q->mode == SIMRANK_MODE_STRATIFIED) {
        StratParams sp;
        const int rc = strat_params(q, n, &sp, nullptr);
        if (rc) return rc;
        out->R = sp.N;
        out->L = sp.phi;
        out->T = 0;
        out->reserved = 0;
        if (mode) *mode = q->mode;
        return SIMRANK_OK;
    }
    const int32_t L = q->walk_cap == 0 ? 64 : q->walk_cap;
    if (L < 1 || L > MAX_CAP) return fail(SIMRANK_EINVAL, "walk_cap must lie in [1, 255]");
    if (q->mode == SIMRANK_MODE_STITCHED && L > MAX_STITCH_CAP)
        return fail(SIMRANK_EINVAL, "stitched walks are capped at 64 steps");
    int64_t R;
    if (q->R_override > 0) {
        R = q->R_override;
    } else {
        // Hoeffding: 2 exp(-2 R lambda^2) <= delta (per node) or delta / n
        // (union over n nodes); lambda = eps minus the truncation bias c^(L+1).
        const double lam = q->eps - pow(q->c, (double)(L + 1));
        if (!(lam > 0.0)) return fail(SIMRANK_EINVAL, "eps must exceed c^(L+1)");
        const double num = q->union_bound ? log(2.0 * (double)n / q->delta) : log(2.0 / q->delta);
        const double r = ceil(num / (2.0 * lam * lam));
        if (!(r <= (double)MAX_R)) return fail(SIMRANK_EINVAL, "R exceeds 2^24");
        R = (int64_t)r;
    }
    if (R > MAX_R) return fail(SIMRANK_EINVAL, "R exceeds 2^24");
    out->R = (int32_t)R;
    out->L = L;
    out->T = continue_threshold(q->c);
    out->reserved = 0;
    if (mode) *mode = q->mode;
    return SIMRANK_OK;
}

// Algorithm 1 caps walks at phi = log_{1/sqrt c} n steps (floor) and draws
// N_l = ceil(Z_l) walks of length l from every node, Z_l = z sqrt(c)^l
// (1 - sqrt(c)), with Algorithm 2's z = ln(2n) / (2 (eps - 3/n)^2).  A query
// may fix phi (walk_cap > 0, the longer cap of the error-threshold extension)
// and z (R_override > 0).  sqrt(c)^l is formed by repeated multiplication.
int strat_params(const simrank_query *q, int32_t n, StratParams *sp, StratTab *tab) {
    if (n < 1) return fail(SIMRANK_EINVAL, "n must be >= 1");
    double z;
    if (q->R_override > 0) {
        z = (double)q->R_override;
    } else {
        const double gap = q->eps - 3.0 / (double)n;
        if (!(gap > 0.0)) return fail(SIMRANK_EINVAL, "stratified estimator needs eps > 3/n");
        z = log(2.0 * (double)n) / (2.0 * gap * gap);
    }
    const double r = sqrt(q->c);
    int32_t phi;
    if (q->walk_cap > 0) {
        phi = q->walk_cap;
    } else {
        const double f = floor(log((double)n) / log(1.0 / r));
        if (!(f >= 0.0 && f <= (double)MAX_CAP)) return fail(SIMRANK_EINVAL, "phi beyond 255");
        phi = (int32_t)f;
    }
    if (phi < 1 || phi > MAX_CAP) return fail(SIMRANK_EINVAL, "walk cap phi must lie in [1, 255]");
    double g = 1.0;
    double N = 0.0;
    for (int32_t l = 0; l <= phi; ++l) {
        const double Zl = (z * g) * (1.0 - r);
        const double Zh = ceil(Zl);
        if (tab) {
            tab->ccum[l] = (uint32_t)N;
            tab->a[l] = Zl / Zh;
        }
        N += Zh;
        if (!(N <= (double)MAX_STRAT_N))
            return fail(SIMRANK_EINVAL, "stratified estimator needs fewer than 2^24 walks per node");
        g = g * r;
    }
    if (tab) tab->ccum[phi + 1] = (uint32_t)N;
    sp->z = z;
    sp->N = (int32_t)N;
    sp->phi = phi;
    int32_t bits = 0;
    while ((1 << bits) < sp->N) ++bits;
    sp->sb = (bits + 1) / 2;
    sp->sa = (sp->N + (1 << sp->sb) - 1) >> sp->sb;
    return SIMRANK_OK;
}

int workspace_init(const Graph *g, int32_t max_R, int32_t max_L, Workspace *ws) {
    if (max_R < 1 || max_R > MAX_R) return fail(SIMRANK_EINVAL, "max_R must lie in [1, 2^24]");
    if (max_L < 1 || max_L > MAX_CAP) return fail(SIMRANK_EINVAL, "max_L must lie in [1, 255]");
    ws->g = g;
    ws->max_R = max_R;
    ws->max_L = max_L;
    ws->max_tiles = max_tiles_for(max_R, max_L);
    const size_t RL = (size_t)max_R * (size_t)max_L;
    int rc;
    if ((rc = device_alloc((void **)&ws->sw, 4 * RL, nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->slen, (size_t)max_R, nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->jj, 4 * (size_t)max_R, nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->joff, 4 * ((size_t)max_R + 1), nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->swc, 4 * RL, nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->tiles, 4 * ((size_t)ws->max_tiles + 1), nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->meta, 4 * 8, nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->counters, 8 * 8, nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->desc, sizeof(QueryDesc), nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->units, 4 * units_words(1), nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->scls, (size_t)max_R, nullptr))) return rc;
    if ((rc = device_alloc((void **)&ws->tab, sizeof(StratTab), nullptr))) return rc;
    SRK_HIP(hipHostMalloc((void **)&ws->tab_host, sizeof(StratTab), hipHostMallocDefault));
    SRK_HIP(hipEventCreate(&ws->ev_tab));
    SRK_HIP(hipEventCreate(&ws->ev0));
    SRK_HIP(hipEventCreate(&ws->ev1));
    SRK_HIP(hipEventCreate(&ws->evm0));
    SRK_HIP(hipEventCreate(&ws->evm1));
    return SIMRANK_OK;
}

void workspace_release(Workspace *ws) {
    if (!ws) return;
    device_free(ws->sw);
    device_free(ws->slen);
    device_free(ws->jj);
    device_free(ws->joff);
    device_free(ws->swc);
    device_free(ws->tiles);
    device_free(ws->meta);
    device_free(ws->counters);
    device_free(ws->desc);
    device_free(ws->units);
    device_free(ws->scls);
    device_free(ws->tab);
    if (ws->tab_host) (void)hipHostFree(ws->tab_host);
    if (ws->ev_tab) (void)hipEventDestroy(ws->ev_tab);
    if (ws->ev0) (void)hipEventDestroy(ws->ev0);
    if (ws->ev1) (void)hipEventDestroy(ws->ev1);
    if (ws->evm0) (void)hipEventDestroy(ws->evm0);
    if (ws->evm1) (void)hipEventDestroy(ws->evm1);
    *ws = Workspace{};
}

// One query on a workspace: its descriptor, then the whole launch sequence.
static int launch_single(const Graph *g, Workspace *ws, const QueryDesc &d, hipStream_t st) {
    // the meet kernel counts work units (tile x node chunk) in 32 bits
    const int64_t units_bound = (int64_t)max_tiles_for(d.R, d.L) * d.n_chunks;
    if (units_bound >= (int64_t)0xffffffffu - (1 << 20))
        return fail(SIMRANK_EINVAL, "R * L * n too large for one launch");
    QuerySet qs;
    qs.desc = ws->desc;
    qs.nq = 1;
    qs.max_R = d.R;
    qs.max_n = g->n;
    qs.units_bound[d.kind] = units_bound;
    qs.units = ws->units;
    qs.counters = ws->counters;
    SRK_HIP(hipEventRecord(ws->ev0, st));
    k_set_desc<<<1, 1, 0, st>>>(ws->desc, d);
    int rc = launch_query_set(qs, st, ws->evm0, ws->evm1);
    if (rc) return rc;
    SRK_HIP(hipEventRecord(ws->ev1, st));
    ws->last_stream = st;
    ws->last_params.R = d.R;
    ws->last_params.L = d.L;
    ws->last_params.T = d.T;
    ws->last_params.reserved = 0;
    ws->last_n = g->n;
    ws->pending = true;
    return SIMRANK_OK;
}

static void attach_buffers(Workspace *ws, QueryDesc *d) {
    d->sw = ws->sw;
    d->slen = ws->slen;
    d->jj = ws->jj;
    d->joff = ws->joff;
    d->swc = ws->swc;
    d->tiles = ws->tiles;
    d->meta = ws->meta;
    d->scls = ws->scls;
    d->tab = ws->tab;
}

int enqueue_query(const Graph *g, const simrank_query *q, const simrank_params &p, int mode,
                  Workspace *ws, double *out_dev, uint32_t *counts_dev, hipStream_t st) {
    if (q->s < 0 || q->s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
    if (mode == SIMRANK_MODE_STRATIFIED)
        return fail(SIMRANK_EINVAL, "stratified queries return weighted sums: use the stratified calls");
    if (p.R > ws->max_R || p.L > ws->max_L)
        return fail(SIMRANK_EINVAL, "query needs R or L beyond the workspace's size");
    if (!counts_dev) return fail(SIMRANK_EINVAL, "counts buffer is NULL");
    const bool stitched = mode == SIMRANK_MODE_STITCHED;
    if (stitched && !g->index) return fail(SIMRANK_ESTATE, "stitched query without an index");
    if (stitched && g->index->T != p.T)
        return fail(SIMRANK_EINVAL, "stitched query's c differs from the index's c");
    QueryDesc d;
    describe_query(g, q, p, mode, default_unit_nodes(g), &d);
    attach_buffers(ws, &d);
    d.cnt = counts_dev;
    d.out = out_dev;
    return launch_single(g, ws, d, st);
}

int enqueue_stratified(const Graph *g, const simrank_query *q, Workspace *ws, double *out_dev,
                       double *out_n_dev, unsigned long long *wsum_dev, hipStream_t st) {
    if (q->s < 0 || q->s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
    if (q->mode != SIMRANK_MODE_STRATIFIED) return fail(SIMRANK_EINVAL, "not a stratified query");
    if (!wsum_dev) return fail(SIMRANK_EINVAL, "weighted-sum buffer is NULL");
    // the staging copy of the class table may still be read by the previous call
    if (ws->pending) SRK_HIP(hipEventSynchronize(ws->ev_tab));
    StratParams sp;
    int rc = strat_params(q, g->n, &sp, ws->tab_host);
    if (rc) return rc;
    if (sp.N > ws->max_R || sp.phi > ws->max_L)
        return fail(SIMRANK_EINVAL, "query needs N or phi beyond the workspace's size");
    simrank_params p{sp.N, sp.phi, 0u, 0};
    QueryDesc d;
    describe_query(g, q, p, SIMRANK_MODE_STRATIFIED, default_unit_nodes(g), &d);
    attach_buffers(ws, &d);
    d.wsum = wsum_dev;
    d.out = out_dev;
    d.out_n = out_n_dev;
    d.z = sp.z;
    d.sa = sp.sa;
    d.sb = sp.sb;
    SRK_HIP(hipMemcpyAsync(ws->tab, ws->tab_host, sizeof(StratTab), hipMemcpyHostToDevice, st));
    SRK_HIP(hipEventRecord(ws->ev_tab, st));
    return launch_single(g, ws, d, st);
}

static int read_stats(Workspace *ws, simrank_stats *st) {
    SRK_HIP(hipEventSynchronize(ws->ev1));
    unsigned long long c[8];
    SRK_HIP(hipMemcpy(c, ws->counters, sizeof(c), hipMemcpyDeviceToHost));
    float ms = 0.f, mms = 0.f;
    SRK_HIP(hipEventElapsedTime(&ms, ws->ev0, ws->ev1));
    SRK_HIP(hipEventElapsedTime(&mms, ws->evm0, ws->evm1));
    if (st) {
        *st = simrank_stats{};
        st->pairs = (uint64_t)(ws->last_n - 1) * (uint64_t)ws->last_params.R;
        st->pairs_walked = c[C_PAIRS];
        st->moves = c[C_MOVES];
        st->draws = c[C_DRAWS];
        st->meets = c[C_MEETS];
        st->tail_steps = c[C_TAIL];
        st->source_moves = c[C_SRC_MOVES];
        st->ms = ms;
        st->meet_ms = mms;
        st->R = ws->last_params.R;
        st->L = ws->last_params.L;
        st->T = ws->last_params.T;
    }
    ws->pending = false;
    return SIMRANK_OK;
}

}  // namespace srk

using namespace srk;


extern "C" int simrank_derive_params(const simrank_query *q, int32_t n, simrank_params *out) {
    clear_error();
    if (!out) return fail(SIMRANK_EINVAL, "out is NULL");
    if (n < 1) return fail(SIMRANK_EINVAL, "n must be >= 1");
    simrank_params p;
    const int rc = query_params(q, n, &p, nullptr);
    if (rc == SIMRANK_OK) *out = p;
    return rc;
}

extern "C" int simrank_workspace_create(const simrank_graph *g, int32_t max_R, int32_t max_L,
                                        simrank_workspace **ws_out) {
    clear_error();
    if (!g || !ws_out) return fail(SIMRANK_EINVAL, "NULL argument");
    *ws_out = nullptr;
    SRK_HIP(hipSetDevice(g->device));
    simrank_workspace *ws = new simrank_workspace();
    const int rc = workspace_init(g, max_R, max_L, ws);
    if (rc != SIMRANK_OK) {
        workspace_release(ws);
        delete ws;
        return rc;
    }
    *ws_out = ws;
    return SIMRANK_OK;
}

extern "C" int simrank_workspace_free(simrank_workspace *ws) {
    clear_error();
    if (!ws) return SIMRANK_OK;
    if (ws->pending && ws->last_stream) (void)hipStreamSynchronize(ws->last_stream);
    workspace_release(ws);
    delete ws;
    return SIMRANK_OK;
}

extern "C" int simrank_single_source_async(const simrank_graph *g, const simrank_query *q,
                                           simrank_workspace *ws, double *out_dev,
                                           uint32_t *counts_dev, void *stream) {
    clear_error();
    if (!g || !q || !ws) return fail(SIMRANK_EINVAL, "NULL argument");
    if (ws->g != g) return fail(SIMRANK_EINVAL, "workspace belongs to another graph");
    simrank_params p;
    int mode;
    int rc = query_params(q, g->n, &p, &mode);
    if (rc) return rc;
    SRK_HIP(hipSetDevice(g->device));
    return enqueue_query(g, q, p, mode, ws, out_dev, counts_dev, (hipStream_t)stream);
}

extern "C" int simrank_workspace_stats(simrank_workspace *ws, simrank_stats *st) {
    clear_error();
    if (!ws) return fail(SIMRANK_EINVAL, "workspace is NULL");
    if (!ws->pending) return fail(SIMRANK_ESTATE, "no call recorded on this workspace");
    return read_stats(ws, st);
}

extern "C" int simrank_single_source_ex(const simrank_graph *g, const simrank_query *q,
                                        double *out_host, uint32_t *counts_host,
                                        simrank_stats *st_opt) {
    clear_error();
    if (!g || !q) return fail(SIMRANK_EINVAL, "NULL argument");
    simrank_params p;
    int mode;
    int rc = query_params(q, g->n, &p, &mode);
    if (rc) return rc;
    if (q->s < 0 || q->s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
    if (mode == SIMRANK_MODE_STRATIFIED)
        return fail(SIMRANK_EINVAL, "stratified queries: use simrank_single_source_stratified");
    if (mode == SIMRANK_MODE_STITCHED && !g->index)
        return fail(SIMRANK_ESTATE, "stitched query without an index");
    if (mode == SIMRANK_MODE_STITCHED && g->index->T != p.T)
        return fail(SIMRANK_EINVAL, "stitched query's c differs from the index's c");
    SRK_HIP(hipSetDevice(g->device));
    Workspace ws;
    double *out_dev = nullptr;
    uint32_t *cnt_dev = nullptr;
    rc = workspace_init(g, p.R, p.L, &ws);
    if (!rc) rc = device_alloc((void **)&cnt_dev, 4 * (size_t)g->n, nullptr);
    if (!rc && out_host) rc = device_alloc((void **)&out_dev, 8 * (size_t)g->n, nullptr);
    if (!rc) rc = enqueue_query(g, q, p, mode, &ws, out_dev, cnt_dev, g->stream);
    if (!rc) rc = read_stats(&ws, st_opt);
    if (!rc && out_host) {
        hipError_t e = hipMemcpy(out_host, out_dev, 8 * (size_t)g->n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    if (!rc && counts_host) {
        hipError_t e = hipMemcpy(counts_host, cnt_dev, 4 * (size_t)g->n, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    device_free(out_dev);
    device_free(cnt_dev);
    workspace_release(&ws);
    return rc;
}

extern "C" int simrank_single_source(const simrank_graph *g, int32_t s, double c, double eps,
                                     double delta, double *out) {
    if (!out) {
        clear_error();
        return fail(SIMRANK_EINVAL, "out is NULL");
    }
    simrank_query q{};
    q.s = s;
    q.c = c;
    q.eps = eps;
    q.delta = delta;
    q.seed = 0;
    q.walk_cap = 64;
    q.mode = SIMRANK_MODE_PLAIN;
    return simrank_single_source_ex(g, &q, out, nullptr, nullptr);
}

extern "C" int simrank_walks(const simrank_graph *g, const simrank_query *q, const int32_t *v,
                             const uint32_t *j, int64_t count, int32_t *paths, int32_t *lens) {
    clear_error();
    if (!g || !q || (count > 0 && (!v || !j || !paths || !lens)))
        return fail(SIMRANK_EINVAL, "NULL argument");
    if (count < 0) return fail(SIMRANK_EINVAL, "count < 0");
    simrank_params p;
    int mode;
    int rc = query_params(q, g->n, &p, &mode);
    if (rc) return rc;
    if (mode == SIMRANK_MODE_STRATIFIED)
        return fail(SIMRANK_EINVAL, "stratified walks: use simrank_stratified_walks");
    for (int64_t i = 0; i < count; ++i)
        if (v[i] < 0 || v[i] >= g->n) return fail(SIMRANK_EINVAL, "walk start out of range");
    const bool stitched = mode == SIMRANK_MODE_STITCHED;
    if (stitched && !g->index) return fail(SIMRANK_ESTATE, "stitched walks without an index");
    if (stitched && g->index->T != p.T)
        return fail(SIMRANK_EINVAL, "stitched walks' c differs from the index's c");
    if (count == 0) return SIMRANK_OK;
    SRK_HIP(hipSetDevice(g->device));
    int32_t *dv = nullptr, *dpaths = nullptr, *dlens = nullptr;
    uint32_t *dj = nullptr;
    const size_t rowb = 4 * (size_t)(p.L + 1);
    rc = device_alloc((void **)&dv, 4 * (size_t)count, nullptr);
    if (!rc) rc = device_alloc((void **)&dj, 4 * (size_t)count, nullptr);
    if (!rc) rc = device_alloc((void **)&dpaths, rowb * (size_t)count, nullptr);
    if (!rc) rc = device_alloc((void **)&dlens, 4 * (size_t)count, nullptr);
    hipStream_t st = g->stream;
    if (!rc) {
        hipError_t e = hipMemcpyAsync(dv, v, 4 * (size_t)count, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipMemcpyAsync(dj, j, 4 * (size_t)count, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) {
            WalkArgs wa{g->nodes, g->E, index_view(g), dv, dj, count, dpaths, dlens,
                        make_key(q->seed), p.T, p.L};
            if (stitched)
                k_walks<true><<<grid_for(count, 256), 256, 0, st>>>(wa);
            else
                k_walks<false><<<grid_for(count, 256), 256, 0, st>>>(wa);
            e = hipGetLastError();
        }
        if (e == hipSuccess)
            e = hipMemcpyAsync(paths, dpaths, rowb * (size_t)count, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(lens, dlens, 4 * (size_t)count, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    device_free(dv);
    device_free(dj);
    device_free(dpaths);
    device_free(dlens);
    return rc;
}

// ------------------------------------------------ length-stratified estimator

extern "C" int simrank_derive_stratified(const simrank_query *q, int32_t n,
                                         simrank_strat_params *out) {
    clear_error();
    if (!q || !out) return fail(SIMRANK_EINVAL, "NULL argument");
    simrank_query qq = *q;
    qq.mode = SIMRANK_MODE_STRATIFIED;
    simrank_params p;
    int rc = query_params(&qq, n, &p, nullptr);
    if (rc) return rc;
    StratParams sp;
    rc = strat_params(&qq, n, &sp, nullptr);
    if (rc) return rc;
    *out = simrank_strat_params{sp.z, sp.N, sp.phi, sp.sb, sp.sa};
    return SIMRANK_OK;
}

extern "C" int simrank_stratified_async(const simrank_graph *g, const simrank_query *q,
                                        simrank_workspace *ws, double *out_dev, double *out_n_dev,
                                        uint64_t *wsum_dev, void *stream) {
    clear_error();
    if (!g || !q || !ws) return fail(SIMRANK_EINVAL, "NULL argument");
    if (ws->g != g) return fail(SIMRANK_EINVAL, "workspace belongs to another graph");
    simrank_params p;
    int rc = query_params(q, g->n, &p, nullptr);
    if (rc) return rc;
    SRK_HIP(hipSetDevice(g->device));
    return enqueue_stratified(g, q, ws, out_dev, out_n_dev, (unsigned long long *)wsum_dev,
                              (hipStream_t)stream);
}

extern "C" int simrank_single_source_stratified(const simrank_graph *g, const simrank_query *q,
                                                double *out, double *out_n, uint64_t *wsum,
                                                simrank_stats *st_opt) {
    clear_error();
    if (!g || !q) return fail(SIMRANK_EINVAL, "NULL argument");
    if (q->mode != SIMRANK_MODE_STRATIFIED) return fail(SIMRANK_EINVAL, "not a stratified query");
    simrank_params p;
    int rc = query_params(q, g->n, &p, nullptr);
    if (rc) return rc;
    if (q->s < 0 || q->s >= g->n) return fail(SIMRANK_EINVAL, "source out of range");
    SRK_HIP(hipSetDevice(g->device));
    Workspace ws;
    double *out_dev = nullptr, *out_n_dev = nullptr;
    unsigned long long *w_dev = nullptr;
    const size_t n = (size_t)g->n;
    rc = workspace_init(g, p.R, p.L, &ws);
    if (!rc) rc = device_alloc((void **)&w_dev, 8 * n, nullptr);
    if (!rc && out) rc = device_alloc((void **)&out_dev, 8 * n, nullptr);
    if (!rc && out_n) rc = device_alloc((void **)&out_n_dev, 8 * n, nullptr);
    if (!rc) rc = enqueue_stratified(g, q, &ws, out_dev, out_n_dev, w_dev, g->stream);
    if (!rc) rc = read_stats(&ws, st_opt);
    hipError_t e = hipSuccess;
    if (!rc && out) e = hipMemcpy(out, out_dev, 8 * n, hipMemcpyDeviceToHost);
    if (!rc && e == hipSuccess && out_n) e = hipMemcpy(out_n, out_n_dev, 8 * n, hipMemcpyDeviceToHost);
    if (!rc && e == hipSuccess && wsum) e = hipMemcpy(wsum, w_dev, 8 * n, hipMemcpyDeviceToHost);
    if (!rc && e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    device_free(out_dev);
    device_free(out_n_dev);
    device_free(w_dev);
    workspace_release(&ws);
    return rc;
}

extern "C" int simrank_stratified_walks(const simrank_graph *g, const simrank_query *q,
                                        const int32_t *v, const uint32_t *j, int64_t count,
                                        uint32_t *slot, int32_t *cls, int32_t *paths,
                                        int32_t *lens) {
    clear_error();
    if (!g || !q || (count > 0 && (!v || !j || !slot || !cls)))
        return fail(SIMRANK_EINVAL, "NULL argument");
    if ((paths == nullptr) != (lens == nullptr))
        return fail(SIMRANK_EINVAL, "paths and lens go together");
    if (count < 0) return fail(SIMRANK_EINVAL, "count < 0");
    if (q->mode != SIMRANK_MODE_STRATIFIED) return fail(SIMRANK_EINVAL, "not a stratified query");
    simrank_params p;
    int rc = query_params(q, g->n, &p, nullptr);
    if (rc) return rc;
    StratTab tab;
    StratParams sp;
    rc = strat_params(q, g->n, &sp, &tab);
    if (rc) return rc;
    for (int64_t i = 0; i < count; ++i) {
        if (v[i] < 0 || v[i] >= g->n) return fail(SIMRANK_EINVAL, "walk start out of range");
        if (j[i] >= (uint32_t)sp.N) return fail(SIMRANK_EINVAL, "walk index beyond N");
    }
    if (count == 0) return SIMRANK_OK;
    SRK_HIP(hipSetDevice(g->device));
    int32_t *dv = nullptr, *dpaths = nullptr, *dlens = nullptr, *dcls = nullptr;
    uint32_t *dj = nullptr, *dslot = nullptr;
    StratTab *dtab = nullptr;
    const size_t rowb = 4 * (size_t)(sp.phi + 1), c4 = 4 * (size_t)count;
    rc = device_alloc((void **)&dv, c4, nullptr);
    if (!rc) rc = device_alloc((void **)&dj, c4, nullptr);
    if (!rc) rc = device_alloc((void **)&dslot, c4, nullptr);
    if (!rc) rc = device_alloc((void **)&dcls, c4, nullptr);
    if (!rc) rc = device_alloc((void **)&dtab, sizeof(StratTab), nullptr);
    if (!rc && paths) rc = device_alloc((void **)&dpaths, rowb * (size_t)count, nullptr);
    if (!rc && paths) rc = device_alloc((void **)&dlens, c4, nullptr);
    hipStream_t st = g->stream;
    if (!rc) {
        hipError_t e = hipMemcpy(dv, v, c4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dj, j, c4, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(dtab, &tab, sizeof(StratTab), hipMemcpyHostToDevice);
        if (e == hipSuccess) {
            StratWalkArgs wa{g->nodes, g->E, g->node_of, dtab, dv, dj, count, dpaths, dlens,
                             dslot, dcls, make_key(q->seed), (uint32_t)sp.N, (uint32_t)sp.sa,
                             (uint32_t)sp.sb, sp.phi};
            k_walks_strat<<<grid_for(count, 256), 256, 0, st>>>(wa);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e == hipSuccess) e = hipMemcpy(slot, dslot, c4, hipMemcpyDeviceToHost);
        if (e == hipSuccess) e = hipMemcpy(cls, dcls, c4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && paths) e = hipMemcpy(paths, dpaths, rowb * (size_t)count, hipMemcpyDeviceToHost);
        if (e == hipSuccess && paths) e = hipMemcpy(lens, dlens, c4, hipMemcpyDeviceToHost);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
    }
    device_free(dv);
    device_free(dj);
    device_free(dslot);
    device_free(dcls);
    device_free(dtab);
    device_free(dpaths);
    device_free(dlens);
    return rc;
}
