// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "simrank.h"

namespace srk {

// ------------------------------------------------------------------ errors
void set_error(const std::string &msg);
void clear_error();
int fail(int code, const std::string &msg);

#define SRK_HIP(expr)                                                                      \
    do {                                                                                   \
        hipError_t e_ = (expr);                                                            \
        if (e_ != hipSuccess)                                                              \
            return ::srk::fail(SIMRANK_EDEVICE, std::string(#expr) + ": " +                \
                                                    hipGetErrorString(e_));                \
    } while (0)

// --------------------------------------------------------------- constants
constexpr uint32_t NIL = 0xffffffffu;   // no successor / no segment
constexpr int MAX_CAP = 255;            // walk cap limit (lengths fit a byte)
constexpr int MAX_STITCH_CAP = 64;      // stitched walks: long walks span 64 steps
constexpr int64_t MAX_R = 1 << 24;
constexpr int64_t MAX_STRAT_N = (1 << 24) - 1;  // weighted sums stay below 2^64

// Query kinds (one meet-kernel instance each).
enum Kind : int32_t { K_PLAIN = 0, K_STITCHED = 1, K_STRAT = 2, N_KINDS = 3 };


// Meet-kernel tiling of the compacted source walks (see query.hip), per kind.
// The more walks of one node a block holds, the more of their early steps
// share rows in the CU's L1; LDS bounds the tile.  Measured per query:
//  - plain (medium graph, in the Infinity Cache): 1024-thread blocks, tiles of
//    up to 8192 walks / 24576 positions (148 KB of LDS, one block per CU):
//    50.5 ms, against 58.9 ms with 512 threads and 1024 / 4096;
//  - stratified (medium graph; its LDS also holds classes, shuffle keys and a
//    queue of prepared pairs): 1024 threads, 6144 / 20480: 99.6 ms, against
//    114.1 ms with 512 threads and 1024 / 4096;
//  - stitched: the plain kind's block and positions per tile (its private
//    heads are plain walks), with room in LDS for the waves' tail queues
//    (16 waves x 128 x 8 bytes): tiles of up to 6144 walks / 24576 positions.
#ifndef SRK_TILE_J
#define SRK_TILE_J 8192
#endif
#ifndef SRK_TILE_NODES
#define SRK_TILE_NODES 24576
#endif
#ifndef SRK_MEET_BLOCK
#define SRK_MEET_BLOCK 1024
#endif
#ifndef SRK_STITCH_TILE_J
#define SRK_STITCH_TILE_J 6144
#endif
#ifndef SRK_STITCH_TILE_NODES
#define SRK_STITCH_TILE_NODES 24576
#endif
#ifndef SRK_STITCH_MEET_BLOCK
#define SRK_STITCH_MEET_BLOCK 1024
#endif
#ifndef SRK_STRAT_TILE_J
#define SRK_STRAT_TILE_J 6144
#endif
#ifndef SRK_STRAT_TILE_NODES
#define SRK_STRAT_TILE_NODES 20480
#endif
#ifndef SRK_STRAT_MEET_BLOCK
#define SRK_STRAT_MEET_BLOCK 1024
#endif
constexpr int MEET_VB = 256;                // nodes v per work unit, at most
constexpr int MIN_TILE_J = 2048;            // smallest tile a query may be given (buffers are
                                            // sized for it: max_tiles_for)
__host__ __device__ constexpr int tile_j_of(int kind) {
    return kind == K_PLAIN ? SRK_TILE_J : kind == K_STITCHED ? SRK_STITCH_TILE_J : SRK_STRAT_TILE_J;
}
__host__ __device__ constexpr int tile_nodes_of(int kind) {   // < 2^16
    return kind == K_PLAIN ? SRK_TILE_NODES
           : kind == K_STITCHED ? SRK_STITCH_TILE_NODES : SRK_STRAT_TILE_NODES;
}
__host__ __device__ constexpr int meet_block_of(int kind) {
    return kind == K_PLAIN ? SRK_MEET_BLOCK
           : kind == K_STITCHED ? SRK_STITCH_MEET_BLOCK : SRK_STRAT_MEET_BLOCK;
}

// ------------------------------------------------------------ device graph
// Gather layout of the reversed graph.  Every node v owns the edge slots
// [o(v), o(v) + max(deg(v), 1)) of E; E[o(v) + k] describes the k-th
// in-neighbour u of v by (o(u), deg(u)), so one 8-byte gather moves a walk and
// already yields the row of the node it lands on.  o() is strictly increasing,
// so it identifies nodes; nodes without in-neighbours own one unused slot.
struct Index;

struct Graph {
    int device = 0;
    int32_t n = 0;
    int64_t m = 0;
    int64_t m_slots = 0;          // sum over v of max(deg(v), 1)
    int32_t n_active = 0;         // nodes with deg >= 1
    int32_t max_deg = 0;
    uint2 *nodes = nullptr;       // [n]     (o(v), deg(v))
    uint2 *E = nullptr;           // [m_slots]
    uint32_t *node_of = nullptr;  // [m_slots] node id owning slot o (valid at o(v))
    int32_t *active = nullptr;    // [n_active] nodes with deg >= 1, ascending
    uint32_t *dbar = nullptr;     // [n] rows of the CSR that list v (v's in-degree in the
                                  //     reversed graph), counted at ingest
    hipStream_t stream = nullptr; // stream of the synchronous calls
    Index *index = nullptr;
    uint64_t index_gen = 0;       // counts replacements of the index (plans check it)
    int32_t tuned_vb = 0;         // nodes per meet work unit chosen by simrank_tune (0: default)
    int32_t tuned_tile_j[N_KINDS] = {0, 0, 0};   // source walks per LDS tile, per kind (0: default)
    int64_t bytes = 0;
};

// Stitched-walk index (see index.hip).
struct Index {
    int32_t seg_log2 = 3;
    int32_t seg_len = 8;          // 2^k
    int32_t width = 8;            // long-walk width in segments: 64 / 2^k
    int32_t levels = 3;           // doubling rounds: log2(width)
    double kappa = 1.0;
    double c = 0.6;               // decay of the segments' walks
    uint32_t T = 0;               // their continue threshold
    uint64_t seed = 0;
    int64_t segments = 0;
    int64_t *pool_off = nullptr;  // [n+1]
    uint32_t *seg = nullptr;      // [segments][seg_len] o() of positions 1..len, NIL after
    uint8_t *seg_lens = nullptr;  // [segments]
    uint32_t *succ = nullptr;     // [segments] successor slot or NIL
    uint32_t *chain = nullptr;    // [segments][width] slots of the long walk from sigma
    int64_t bytes = 0;
    double build_ms = 0;
    double segments_ms = 0, doubling_ms = 0;   // parts of build_ms
    uint64_t build_moves = 0;
};

// Read-only view of a graph's stitched index, as the kernels see it.
struct IndexView {
    const uint32_t *node_of;
    const int64_t *pool_off;
    const uint32_t *seg;
    const uint8_t *seg_lens;
    const uint32_t *chain;
    int32_t seg_len, width;
};

// Length-stratified estimator: the first slot of each length class and
// Lemma 5's per-class ratio Z_l / Zhat_l (computed on the host).
struct StratTab {
    uint32_t ccum[MAX_CAP + 2];   // ccum[l] = Zhat_0 + ... + Zhat_{l-1}; ccum[phi+1] = N
    double a[MAX_CAP + 1];
};

struct StratParams {
    double z = 0;                 // Algorithm 2's normaliser
    int32_t N = 0;                // walks per node, sum of Zhat_l
    int32_t phi = 0;              // walk length cap
    int32_t sb = 0;               // shuffle grid [0, sa) x [0, 2^sb), sa 2^sb >= N
    int32_t sa = 1;
};

// One query as the device kernels see it (one entry per query of a launch).
struct QueryDesc {
    const uint2 *nodes;
    const uint2 *E;
    const int32_t *active;
    IndexView ix;
    uint32_t *sw;          // [R][L] source walk positions 1..L (o values)
    uint8_t *slen;         // [R]
    uint32_t *jj;          // [R] walk index of compact entry k
    uint32_t *joff;        // [R + 1] start of entry k in swc
    uint32_t *swc;         // [R * L] packed positions
    uint32_t *tiles;       // [max tiles + 1]
    uint32_t *meta;        // [8]: R1, packed positions, tiles
    uint32_t *cnt;         // [n] meet counts (caller's; plain and stitched)
    double *out;           // [n] estimate or NULL
    uint32_t k0, k1;       // Philox key of the query's walks
    uint32_t T;            // continue threshold
    int32_t n, n_active, s, R, L;
    int32_t vb;            // nodes per work unit (<= MEET_VB)
    int32_t n_chunks;      // ceil(n_active / vb)
    int32_t kind;          // Kind
    int32_t tile_j;        // source walks per LDS tile, MIN_TILE_J .. tile_j_of(kind)
    // stratified only (R = N walks per node, L = phi)
    const StratTab *tab;
    uint8_t *scls;         // [R] length class of walk (s, j)
    unsigned long long *wsum;  // [n] weighted meet sums, 2^40 = weight 1 (caller's)
    double *out_n;         // [n] estimate normalised by the N pairs, or NULL
    double z;
    int32_t sa, sb;        // shuffle grid
};

// A set of queries whose descriptors are already in device memory.
struct QuerySet {
    const QueryDesc *desc;        // device [nq]
    int32_t nq = 0;
    int32_t max_R = 0, max_n = 0;
    int64_t units_bound[N_KINDS] = {0, 0, 0};   // work units of each kind's queries, at most
    uint32_t *units = nullptr;    // device [units_words(nq)]: unit offsets per kind, then cursors
    unsigned long long *counters = nullptr;  // device [8]
    const struct GroupSet *groups = nullptr;  // grouped plain queries, if any
};

// Words of a query set's unit table: N_KINDS lists of nq + 1 offsets, then
// one cursor per kind.
inline size_t units_words(int32_t nq) { return (size_t)N_KINDS * ((size_t)nq + 1) + N_KINDS; }

// ------------------------------------------------------------ query groups
// In a batch, queries of one kind on one graph with the same walk key and walk
// parameters (c and cap; the stratified estimator's z and cap) have the same
// walk (v, j) from every node v: a group of up to GROUP_MAX such queries
// follows each walk once and tests it against every
// member's walk j of its own source (group.hip).  A member keeps its own
// descriptor (source walks, counts or weighted sums, estimate) with kind
// K_GROUPED, K_GROUPED_STITCHED or K_GROUPED_STRAT, which no per-kind unit list
// takes.
constexpr int GROUP_MAX = 32;
constexpr int32_t K_GROUPED = N_KINDS, K_GROUPED_STITCHED = N_KINDS + 1, K_GROUPED_STRAT = N_KINDS + 2;
// Groups of more than 8 stratified queries keep their 64-bit weighted sums for
// at most this many nodes per work unit (64 KB of LDS at 256 nodes; their tile
// is the smaller for it).
#ifndef SRK_GROUP_STRAT32_VB
#define SRK_GROUP_STRAT32_VB 256
#endif
constexpr int GROUP_STRAT32_VB = SRK_GROUP_STRAT32_VB;
// Kinds whose walks are the stratified estimator's (weighted sums, not counts).
__host__ __device__ inline bool strat_kind(int32_t kind) { return kind == K_STRAT || kind == K_GROUPED_STRAT; }

struct GroupDesc {
    const uint2 *nodes;
    const uint2 *E;
    const int32_t *active;
    int32_t n_active, vb, n_chunks;
    int32_t G, L, Rmax;
    int32_t gw;                          // words of member lengths per entry: ceil(G / 4)
    int32_t wk;                          // walks: 0 plain, 1 stitched (index tails), 2 stratified
    IndexView ix;
    // stratified: the class table, N = R of every member, the shuffle grid
    const StratTab *tab;
    int32_t sa, sb;
    uint32_t k0, k1, T;
    int32_t s[GROUP_MAX];                // members' sources
    int32_t R[GROUP_MAX];
    const uint32_t *sw[GROUP_MAX];       // members' source walks [R][L]
    const uint8_t *slen[GROUP_MAX];      // and their lengths [R]
    uint32_t *cnt[GROUP_MAX];            // members' meet counts [n] (plain, stitched)
    unsigned long long *wsum[GROUP_MAX]; // members' weighted sums [n] (stratified)
    const uint8_t *scls[GROUP_MAX];      // classes of the members' walks [R] (stratified)
    // Compacted walks: entry e is a walk index jj[e] for which at least one
    // member's walk has a step; from pos[joff[e]], one block per step t of its
    // longest member walk: a word with bit q set for each member q whose walk
    // j has a position at step t, then those positions in member order.
    // Member q's length is byte q of the entry's gw words glen[e gw ...].
    uint32_t *jj;                        // [Rmax]
    uint32_t *joff;                      // [Rmax + 1]
    uint32_t *glen;                      // [Rmax][gw]
    uint32_t *pos;                       // [group_pos_words]
    uint32_t *tiles;                     // [group_max_tiles + 1]
    uint32_t *meta;                      // [8]: entries, positions, tiles
};

// Kernel instance of a group: plain walks with up to 8 members (0) or more
// (1), stitched walks with up to 8 (2) or more (3), stratified walks with up
// to 8 (4) or more (5).
constexpr int GROUP_LISTS = 6;
__host__ __device__ inline int group_list(int32_t G, int32_t wk) { return 2 * wk + (G > 8 ? 1 : 0); }

struct GroupSet {
    const GroupDesc *desc = nullptr;     // device [ng]
    int32_t ng = 0;
    int64_t units_bound[GROUP_LISTS] = {};       // work units per kernel instance (group_list)
    uint32_t *units = nullptr;           // device [group_units_words(ng)]
};
// Unit offsets of a group set: one list of ng + 1 offsets per instance, then
// one cursor per list.
inline size_t group_units_words(int32_t ng) { return GROUP_LISTS * ((size_t)ng + 1) + GROUP_LISTS; }

// Words of a group's compacted walks, at most: every member position and one
// member word per step of each entry.
inline int64_t group_pos_words(int64_t Rmax, int64_t sum_RL, int32_t L) { return sum_RL + Rmax * L; }
// Tiles of a group's compacted walks, at most.
int32_t group_max_tiles(int64_t Rmax, int64_t sum_RL, int32_t L, int32_t G, int32_t wk);
// Nodes per work unit of a group of G members with walks wk on a graph with
// n_active nodes that have in-edges (the lone queries' tuning does not apply).
int32_t group_unit_nodes(int32_t n_active, int32_t G, int32_t wk);
// Fills a group's descriptor (all but its compaction buffers jj .. meta) from
// the descriptors of its G members (kinds K_GROUPED, K_GROUPED_STITCHED or
// K_GROUPED_STRAT, buffers attached).
void describe_group(const QueryDesc *const *members, int32_t G, GroupDesc *gd);
// Device bytes of a group's compaction buffers and their carving from `base`
// (256-byte aligned pieces); returns the bytes taken.
size_t group_buffers(GroupDesc *gd, int64_t sum_RL, char *base);
// Enqueues a query set's groups: compaction, unit offsets, the group meet
// kernel (after the members' source walks, before their estimates).
int launch_groups(const GroupSet &gs, unsigned long long *counters, hipStream_t st);

// ------------------------------------------------------------ serving ring
// The server's in-flight requests (server.hip) sit in a ring of entries that
// persistent meet kernels take work units from.  An entry's `claim` word holds
// everything a block needs to decide whether it may take units from it:
//   claim = (seq << 2 | kind) << 32 | units not yet claimed,
// so availability, kind and age come from one atomic read, never from fields
// that a reuse of the entry may be rewriting.  An entry is published by the
// last kernel of its request's preparation: the other fields first, then
// `claim` with all n_units units unclaimed (release).  A block takes up to a
// run of units by moving the count down with compare-and-swap (acquire), then
// reads n_units (the first unit it took is n_units minus the count it saw).
// A swap cannot succeed on an older request's word once the entry has been
// reused (seq differs), and a fully claimed word (count 0) is never a
// candidate.  The block that finishes the entry's last unit writes the
// estimate and then the entry's flag in host memory (the request's seq).
// seq is nonzero and below 2^30.
constexpr int RING_MAX = 64;
constexpr uint32_t RING_SEQ_LIMIT = 1u << 30;
struct RingCtl {
    unsigned long long claim;   // see above; 0 = never published
    uint32_t n_units;           // tiles x node chunks of the request
    uint32_t done;              // units finished
    int32_t kind;               // Kind of the meet kernel that takes it
    uint32_t seq;               // the request's sequence number
    uint32_t pad[2];
};
struct StreamRing {
    QueryDesc *desc;                 // device [RING_MAX]
    RingCtl *ctl;                    // device [RING_MAX]
    unsigned long long *counters;    // device [RING_MAX][8]: work counters per entry
    uint32_t *flags;                 // pinned host [RING_MAX], written by the device
    int32_t entries;                 // entries in use, <= RING_MAX
};
// Serving (query.hip): enqueue on `st` the preparation of ring entry `slot`
// for the request described by d (its buffers attached): descriptor, init,
// source walks, compaction, publication.  Launch a persistent meet kernel of
// `kind` that takes units from every published entry of that kind and exits
// when none is left.  Bytes of device memory a request needs for its buffers.
int enqueue_ring_request(const QueryDesc &d, const StreamRing &ring, int32_t slot, uint32_t seq,
                         hipStream_t st);
int launch_ring_meet(int kind, const StreamRing &ring, hipStream_t st);
size_t request_bytes(const simrank_params &p, int mode, int32_t n);
// Carves a request's buffers (request_bytes of them) from base into d.
void carve_request(const simrank_params &p, int mode, int32_t n, char *base, QueryDesc *d);

// Per-query scratch.
struct Workspace {
    const Graph *g = nullptr;
    int32_t max_R = 0, max_L = 0;
    uint32_t *sw = nullptr;        // [max_R][max_L] source walk positions 1..L (o values)
    uint8_t *slen = nullptr;       // [max_R]
    uint32_t *jj = nullptr;        // [max_R] walk index of compact entry k
    uint32_t *joff = nullptr;      // [max_R + 1] start of entry k in swc
    uint32_t *swc = nullptr;       // [max_R * max_L] compact positions
    uint32_t *tiles = nullptr;     // [max tiles + 1] first compact entry of each tile
    uint32_t *meta = nullptr;      // [8]: R1, total nodes, n_tiles, ...
    unsigned long long *counters = nullptr;  // [8] stats
    QueryDesc *desc = nullptr;     // device [1]
    uint32_t *units = nullptr;     // device [units_words(1)]
    uint8_t *scls = nullptr;       // [max_R] stratified: class of walk (s, j)
    StratTab *tab = nullptr;       // device table of the last stratified query
    StratTab *tab_host = nullptr;  // its pinned host staging copy
    hipEvent_t ev_tab = nullptr;   // after the copy of tab_host
    int32_t max_tiles = 0;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;     // around the whole query
    hipEvent_t evm0 = nullptr, evm1 = nullptr;   // around the meet kernel
    hipStream_t last_stream = nullptr;
    simrank_params last_params{};
    int32_t last_n = 0;
    bool pending = false;
};

enum Counter : int {
    C_MOVES = 0, C_DRAWS = 1, C_MEETS = 2, C_TAIL = 3, C_PAIRS = 4, C_SRC_MOVES = 5,
    C_UNITS = 6, C_SPARE = 7
};

// ----------------------------------------------------------------- helpers
int device_alloc(void **p, size_t bytes, int64_t *acct);
void device_free(void *p);

// Device-wide scans (scan.hip).  Exclusive sum of `in` (n values) into `out`
// (n values); returns the total in *total_dev (device scalar).  Temp storage
// is allocated and released by the call.
int scan_exclusive_u32_to_i64(const uint32_t *in, int64_t n, int64_t *out, int64_t *total_dev,
                              hipStream_t st);
int scan_exclusive_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *total_dev,
                       hipStream_t st);
// Inclusive running maximum of u32 values, in place.
int scan_inclusive_max_u32(uint32_t *data, int64_t n, hipStream_t st);

// Queries (query.hip).
int query_params(const simrank_query *q, int32_t n, simrank_params *out, int *mode);
// Stratified estimator: z, N, phi, shuffle width and (if tab) the class table.
int strat_params(const simrank_query *q, int32_t n, StratParams *sp, StratTab *tab);
int32_t max_tiles_for(int32_t R, int32_t L);
int32_t default_unit_nodes(const Graph *g);
IndexView index_view(const Graph *g);
// Fills everything but the buffers (sw .. out) of a descriptor.
void describe_query(const Graph *g, const simrank_query *q, const simrank_params &p, int mode,
                    int32_t vb, QueryDesc *d);
// Enqueues init, source walks, compaction, unit offsets, meet and estimate for
// every query of the set; records ev_meet0 / ev_meet1 (may be NULL) around the
// meet kernels.
int launch_query_set(const QuerySet &qs, hipStream_t st, hipEvent_t ev_meet0, hipEvent_t ev_meet1);
int enqueue_query(const Graph *g, const simrank_query *q, const simrank_params &p, int mode,
                  Workspace *ws, double *out_dev, uint32_t *counts_dev, hipStream_t st);
int enqueue_stratified(const Graph *g, const simrank_query *q, Workspace *ws, double *out_dev,
                       double *out_n_dev, unsigned long long *wsum_dev, hipStream_t st);
int workspace_init(const Graph *g, int32_t max_R, int32_t max_L, Workspace *ws);
void workspace_release(Workspace *ws);

// Index (index.hip).
void index_free(Index *ix);

inline unsigned grid_for(int64_t n, int block) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > 0x7fffffff) b = 0x7fffffff;
    return (unsigned)b;
}

uint32_t continue_threshold(double c);

}  // namespace srk

// The opaque handles of the C ABI are the internal objects.
struct simrank_graph : srk::Graph {};
struct simrank_workspace : srk::Workspace {};
