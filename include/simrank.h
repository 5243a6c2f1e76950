/*
 * simrank.h — C ABI of the MI355X (gfx950) single-source SimRank library.
 *
 * What it computes (Luo & Zhu, "Massively Parallel Single-Source SimRanks in
 * o(log n) Rounds", arXiv 2304.04015):
 *   - Problem (Section 2.2 and Algorithm 1's input/output): given a directed
 *     graph G, a source s, decay c, error eps and failure probability delta,
 *     return s_hat(s, u) for every node u with |s(s,u) - s_hat(s,u)| <= eps.
 *   - Estimator (Lemma 2 and the Monte Carlo paragraph of Section 2.2): pair
 *     the j-th sqrt(c)-walk from s with the j-th sqrt(c)-walk from u on the
 *     reversed graph, j < R; s_hat(s,u) = (number of pairs that meet) / R.
 *     Two walks meet when they are on the same node at the same step i >= 0;
 *     a pair counts once however often its walks coincide (Section 4.4).
 *   - Walks are truncated at L steps (Algorithm 1 truncates at log_{1/sqrt c} n;
 *     Appendix B.4 extends the cap); R follows from Hoeffding's inequality
 *     (Section 3; Appendix B.3/B.4).
 *   - Stitched mode: long walks are formed from short per-node walk segments
 *     joined by pointer doubling, the one-GPU counterpart of the few-round walk
 *     sampler of Theorem 2 / Section 4.1.
 *
 * Random numbers: Philox4x32-10 (Salmon et al., SC'11) with key = (seed low
 * word, seed high word) and counter = (node, walk, step, domain); domain 0 =
 * step of a walk, 1 = step of a pool segment, 2 = pool slot entered after the
 * private head, 3 = successor slot of a segment, 4 = step of a stratified
 * fixed-length walk (counter (node, slot, step, 4)), 5 = round keys of a
 * node's walk shuffle (counter (node, 0, 0, 5)).  At step t (1-based) a walk
 * draws x; it stops if x0 >= T = floor(sqrt(c) * 2^32) or its node has no
 * in-neighbour, else moves to in-neighbour number floor(x1 * deg / 2^32) of the
 * in-edge row (row order as passed to simrank_load_graph).  Results are a pure
 * function of (graph, query) and never depend on launch shape or timing.
 *
 * Conventions for every call:
 *   - Return 0 (SIMRANK_OK) or a SIMRANK_E* code; on error nothing is written
 *     to caller outputs and simrank_last_error() describes the failure.
 *   - "host" pointers are ordinary CPU memory, read or written synchronously;
 *     "device" pointers are HIP device memory on the graph's device.
 *   - A graph (and its index, once built) is immutable and may be queried from
 *     several threads at once; a workspace is used by one call at a time.
 *     The calls that change a graph (simrank_build_index,
 *     simrank_index_load, the tuners, simrank_set_tuning, simrank_free_graph)
 *     must not overlap other calls on it.
 */
#ifndef SIMRANK_H
#define SIMRANK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIMRANK_OK 0
#define SIMRANK_EINVAL 1   /* bad argument: NULL, range, malformed CSR, eps <= c^(L+1) ... */
#define SIMRANK_ENOMEM 2   /* device or host allocation failed, or admission refused */
#define SIMRANK_EDEVICE 3  /* a HIP call failed */
#define SIMRANK_ESTATE 4   /* call not valid in the object's state (e.g. no index built) */
#define SIMRANK_EIO 5      /* a file could not be opened, written or closed */

#define SIMRANK_MODE_PLAIN 0     /* every walk generated step by step */
#define SIMRANK_MODE_STITCHED 1  /* private head + tail read from the segment index */
#define SIMRANK_MODE_STRATIFIED 2 /* Algorithms 1-2: fixed-length walk classes, shuffled,
                                     meets weighted by Lemma 5; see the stratified calls */

typedef struct simrank_graph simrank_graph;         /* opaque; device resident */
typedef struct simrank_workspace simrank_workspace; /* opaque; per-call scratch */

/* One single-source query (Algorithm 1 input: G, s, c, delta, eps). */
typedef struct simrank_query {
    int32_t graph;       /* simrank_batch only: index into its graph array */
    int32_t s;           /* source node, 0 <= s < n */
    double c;            /* decay factor, 0 < c < 1 */
    double eps;          /* absolute error target, c^(L+1) < eps < 1 */
    double delta;        /* failure probability, 0 < delta < 1 */
    uint64_t seed;       /* Philox key of the query's walks */
    int32_t walk_cap;    /* L, the truncation length; 0 selects 64 (stratified mode:
                            0 selects phi = floor(log_{1/sqrt c} n)); at most 255 */
    int32_t R_override;  /* walks per node; 0 selects the Hoeffding count (stratified
                            mode: the value of z; 0 selects Algorithm 2's z) */
    int32_t mode;        /* SIMRANK_MODE_PLAIN, _STITCHED or _STRATIFIED */
    int32_t union_bound; /* 0: delta per node; 1: delta for all n nodes at once */
} simrank_query;

/* Derived per-query constants. */
typedef struct simrank_params {
    int32_t R;   /* walks per node: ceil(ln(2/delta) / (2 (eps - c^(L+1))^2)),
                    with 2n/delta in place of 2/delta when union_bound is set */
    int32_t L;   /* walk cap */
    uint32_t T;  /* continue threshold floor(sqrt(c) 2^32), at most 2^32 - 1 */
    int32_t reserved;
} simrank_params;

/* Work and timing of one call (filled by the synchronous calls). */
typedef struct simrank_stats {
    uint64_t pairs;        /* (v, j) pairs with v != s the query covers: (n - 1) * R */
    uint64_t pairs_walked; /* pairs whose walk had to be generated (v has in-edges,
                              the source walk j has at least one step) */
    uint64_t moves;        /* walk steps taken along in-edges by the meet kernel */
    uint64_t draws;        /* Philox draws made by the meet kernel */
    uint64_t meets;        /* pairs that met (sum of counts minus R for s) */
    uint64_t tail_steps;   /* stitched mode: steps read from the segment index */
    uint64_t source_moves; /* steps of the R source walks */
    double ms;             /* device time of the call, from HIP events */
    double meet_ms;        /* device time of the fused walk + meet kernel alone */
    int32_t R, L;
    uint32_t T;
    int32_t reserved;
} simrank_stats;

/* Length-stratified estimator constants (Algorithm 1 and Algorithm 2). */
typedef struct simrank_strat_params {
    double z;            /* ln(2n) / (2 (eps - 3/n)^2), the expected number of walks */
    int32_t N;           /* walks per node: sum over l of ceil(z sqrt(c)^l (1 - sqrt(c))) */
    int32_t phi;         /* walk length cap: floor(log_{1/sqrt c} n) */
    int32_t shuffle_b;   /* the shuffle permutes the grid [0, shuffle_A) x [0, 2^shuffle_b), */
    int32_t shuffle_A;   /* b = ceil(ceil(log2 N) / 2), A = ceil(N / 2^b) */
} simrank_strat_params;

/* Stitched-walk index parameters. */
typedef struct simrank_index_params {
    int32_t seg_log2;    /* k: segments have 2^k steps; 0 <= k <= 6; default 3 */
    int32_t reserved;
    double kappa;        /* pool size P(y) = ceil(kappa * dbar(y)), dbar(y) = number
                            of in-edge rows that list y; 0 < kappa < 1e6 */
    double c;            /* decay of the segments' walks; stitched queries must use it */
    uint64_t seed;       /* Philox key of the segments and successor picks */
} simrank_index_params;

typedef struct simrank_index_summary {
    int64_t segments;    /* sum over y of P(y) */
    int64_t bytes;       /* device bytes held by the index */
    int32_t seg_log2;
    int32_t levels;      /* doubling rounds run: log2(ceil(max cap / 2^k)) */
    double build_ms;     /* device time of the last build */
    uint64_t build_moves;/* steps taken while building the segments */
    double segments_ms;  /* of build_ms: the segment walks (one per slot, with successors) */
    double doubling_ms;  /* of build_ms: the pointer-doubling rounds */
} simrank_index_summary;

/* ---------------------------------------------------------------- graphs */

/* Copies the in-edge CSR of G to the current HIP device and builds the
 * library's gather layout.  Row v, in_src[in_off[v] .. in_off[v+1]), lists the
 * in-neighbours of v, I(v) (Eq. 1; Algorithm 1 "reverse the edges").
 * in_off: host int32[n+1], in_off[0] = 0, non-decreasing, in_off[n] = m.
 * in_src: host int32[m], each in [0, n).  Duplicates are allowed and then
 * weigh the neighbour pick.  1 <= n, 0 <= m < 2^31 - n.  The caller keeps
 * ownership of its arrays.  *g_out receives a handle owned by the library
 * until simrank_free_graph.  EINVAL on a malformed CSR. */
int simrank_load_graph(int32_t n, int64_t m, const int32_t *in_off, const int32_t *in_src,
                       simrank_graph **g_out);

/* Frees the graph, its index and its device memory.  NULL is a no-op. */
int simrank_free_graph(simrank_graph *g);

/* n, m, number of nodes with at least one in-neighbour, device bytes held. */
int simrank_graph_info(const simrank_graph *g, int32_t *n, int64_t *m, int32_t *n_active,
                       int64_t *device_bytes);

/* ------------------------------------------------------------ parameters */

/* Fills *out from q (walk cap default, R from Hoeffding, T).  EINVAL when an
 * argument is out of range, when eps <= c^(L+1) (the truncation bias
 * S - S_L <= c^(L+1) would use up the error budget), or when R > 2^24. */
int simrank_derive_params(const simrank_query *q, int32_t n, simrank_params *out);

/* --------------------------------------------------------------- queries */

/* Plain query with seed 0, cap 64, per-node delta.  out: host double[n],
 * out[u] = s_hat(s, u), out[s] = 1.  Synchronous. */
int simrank_single_source(const simrank_graph *g, int32_t s, double c, double eps, double delta,
                          double *out);

/* Full query.  out_host: host double[n] or NULL; counts_host: host uint32[n]
 * or NULL (counts[u] = meeting pairs, counts[s] = R); st_opt may be NULL.
 * Synchronous; allocates and frees its own workspace. */
int simrank_single_source_ex(const simrank_graph *g, const simrank_query *q, double *out_host,
                             uint32_t *counts_host, simrank_stats *st_opt);

/* Workspace for asynchronous queries on one graph: scratch for source walks
 * (R x L) and counters, sized for queries with R <= max_R and L <= max_L. */
int simrank_workspace_create(const simrank_graph *g, int32_t max_R, int32_t max_L,
                             simrank_workspace **ws_out);
int simrank_workspace_free(simrank_workspace *ws);

/* Enqueues a whole query on `stream` (a hipStream_t; NULL = default stream)
 * and returns without waiting.  out_dev: device double[n] or NULL;
 * counts_dev: device uint32[n], required (caller-owned, overwritten).  No
 * allocation, no host synchronisation.  The workspace must not be reused until
 * the stream has passed this call. */
int simrank_single_source_async(const simrank_graph *g, const simrank_query *q,
                                simrank_workspace *ws, double *out_dev, uint32_t *counts_dev,
                                void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the query of
 * simrank_single_source_async without a workspace and without any allocation.
 * Its scratch (source walks, tiles, descriptor, counters: about 9 MB) is a
 * fixed device array that each GPU the library runs on holds from the first
 * such call there until the process ends.  Plain and stitched queries with
 * R <= 65536 and R * L <= 2^20 (the medium workload's R = 9502, L = 64 fits);
 * EINVAL beyond that and for stratified queries.  out_dev: device double[n] or
 * NULL; counts_dev: device uint32[n], required; both caller-owned and
 * overwritten.  Enqueues on `stream` (hipStream_t; NULL = default stream) and
 * returns without waiting; results equal simrank_single_source_async's.  All
 * calls on one GPU share its scratch: a call must not overlap another on the
 * same GPU (calls on one stream are ordered; across streams or threads they
 * race).  No stats. */
int simrank_single_source_noalloc(const simrank_graph *g, const simrank_query *q,
                                  double *out_dev, uint32_t *counts_dev, void *stream);

/* Waits for the workspace's last call and fills *st (moves, draws, meets...;
 * ms = device time between the call's first and last kernel). */
int simrank_workspace_stats(simrank_workspace *ws, simrank_stats *st);

/* Materialises walks (v[i], j[i]) for i < count under query q (seed, c, cap,
 * mode): paths host int32[count][L+1] with -1 after the walk's end, lens host
 * int32[count] (moves made).  For parity checks and inspection. */
int simrank_walks(const simrank_graph *g, const simrank_query *q, const int32_t *v,
                  const uint32_t *j, int64_t count, int32_t *paths, int32_t *lens);

/* ------------------------------------------- length-stratified estimator */
/*
 * Algorithm 1 draws, from every node v, N_l = ceil(Z_l) walks of exactly l
 * steps for l = 0..phi, Z_l = z sqrt(c)^l (1 - sqrt(c)), and shuffles each
 * node's N = sum N_l walks; Algorithm 2 pairs walk j of s with walk j of u and
 * adds (Z_l1 Z_l2) / (N_l1 N_l2) / z to s~(s, u) for every pair that meets
 * (Lemma 5), counted once per pair.  Here: the walks of v are generated class
 * by class into slots 0..N-1 (slot r of class l walks l uniform steps keyed
 * (v, r, t, 4); a walk that reaches a node without in-neighbours ends there),
 * and the shuffle maps walk j to slot pi_v(j), a keyed permutation of [0, N)
 * (a four-round mixed-radix Feistel network on a grid of A 2^b >= N points
 * with round keys Philox(v, 0, 0, 5), cycle walked into [0, N)).  Weights are summed in fixed point, 2^40 per unit
 * weight, each weight truncated: the sums are exact and order independent.
 * Query fields used: s, c, eps (z, unless R_override > 0 gives z), walk_cap
 * (0: phi from n), seed; delta is checked but not used by the method.
 * EINVAL if eps <= 3/n, phi is outside [1, 255] or N >= 2^24.
 */
int simrank_derive_stratified(const simrank_query *q, int32_t n, simrank_strat_params *out);

/* One stratified query, synchronous.  Host outputs, each n entries, any may be
 * NULL: out = Algorithm 2's estimate (weighted meets / z), out_n = the estimate
 * normalised by the N pairs actually formed (out * N / z), wsum = the weighted
 * meet sums (2^40 = weight 1).  Entry s of out and out_n is 1, of wsum 0. */
int simrank_single_source_stratified(const simrank_graph *g, const simrank_query *q, double *out,
                                     double *out_n, uint64_t *wsum, simrank_stats *st_opt);

/* Enqueues a stratified query on `stream` using the workspace (max_R >= N,
 * max_L >= phi).  out_dev, out_n_dev: device double[n] or NULL; wsum_dev:
 * device uint64[n], required.  The caller owns the buffers and keeps them
 * until the stream has passed this call.  Stats via simrank_workspace_stats. */
int simrank_stratified_async(const simrank_graph *g, const simrank_query *q,
                             simrank_workspace *ws, double *out_dev, double *out_n_dev,
                             uint64_t *wsum_dev, void *stream);

/* The shuffle and walks of a stratified query for the listed (v[i], j[i]):
 * slot host uint32[count] = pi_v(j), cls host int32[count] = the slot's length
 * class, and (paths, lens may be NULL) paths host int32[count][phi+1] with the
 * walk's nodes (-1 after its end), lens host int32[count] its moves.  For
 * parity checks and inspection. */
int simrank_stratified_walks(const simrank_graph *g, const simrank_query *q, const int32_t *v,
                             const uint32_t *j, int64_t count, uint32_t *slot, int32_t *cls,
                             int32_t *paths, int32_t *lens);

/* ------------------------------------------------ Algorithm 2's tuple form */
/*
 * Meet detection in the paper's own form (Section 3.2; Algorithm 2) for k
 * queries (1 <= k <= 32) on one graph that share mode (plain or stratified),
 * seed, c, walk cap and walk count (R; or z, N and phi).  Every walk is
 * decomposed into one tuple (j, i, node, start) per step after its start; all
 * tuples are sorted with the sources' tuples first among equal (j, i, node);
 * each other tuple is linked to the closest source tuple before it
 * (PREDECESSOR); an equal key is a meet, counted once per pair.  Walks are the
 * fused path's walks followed to their full length.
 * sums: host uint64[k][n].  Plain queries: meet counts, sums[q][s_q] = R (equal
 * to simrank_single_source_ex's counts).  Stratified queries: weighted sums in
 * units of 2^-40, sums[q][s_q] = 0 (equal to simrank_single_source_stratified's
 * wsum).  Nodes are processed in chunks whose tuples fit a 2^28-entry buffer.
 * st_opt: moves = steps of the nodes' walks (= tuples), meets = meeting pairs,
 * ms = device time; for this call meet_ms is the device time of the radix
 * sort's passes (summed over the chunks) and draws the bytes they move (8 per
 * key a histogram pass reads, 24 per tuple a scatter pass reads and writes).  EINVAL for stitched queries, k outside [1, 32], queries
 * that differ in anything but s, or a source out of range.
 */
int simrank_tuple_meets(const simrank_graph *g, const simrank_query *qs, int32_t k,
                        uint64_t *sums, simrank_stats *st_opt);

/* ----------------------------------------------------------------- index */

/* Builds the stitched-walk index on the graph (replacing any earlier one):
 * per-node segment pools, one 2^k-step walk per slot keyed (y, i, t, 1),
 * successor picks keyed (y, i, 0, 3), and long walks of up to 64 steps by
 * pointer doubling.  Synchronous.  ENOMEM if it does not fit.  Not to be
 * called while other threads query g or a server serves it; a batch plan with
 * stitched queries made before the rebuild refuses to run (ESTATE). */
int simrank_build_index(simrank_graph *g, const simrank_index_params *p);
int simrank_index_info(const simrank_graph *g, simrank_index_summary *out);

/* Reads index entries for inspection.  For each slot sigma[i] (0 <= sigma[i] <
 * segments): nodes host int32[count][2^k] receives the segment's positions
 * 1..len as node ids (-1 padded), lens host int32[count] its number of moves,
 * succ host int64[count] its successor slot (-1 if none), and chain_opt (host
 * int64[count][64 / 2^k], may be NULL) the slots of the long walk that starts
 * at sigma[i]: sigma[i], succ(sigma[i]), succ^2(sigma[i]), ..., -1 padded. */
int simrank_index_read(const simrank_graph *g, const int64_t *sigma, int64_t count,
                       int32_t *nodes, int32_t *lens, int64_t *succ, int64_t *chain_opt);

/* Checkpoint and resume of the stitched-walk index (the index of Section
 * 4.1's segments and Theorem 2's doubled chains, as simrank_build_index
 * made it), so that a server can restart on the same graph without a
 * rebuild.  simrank_index_save writes the graph's index to the file at
 * `path` (a 128-byte header with the graph's fingerprint and a checksum of
 * every array, then the arrays; about the index's device bytes); ESTATE if no
 * index is built, EIO if the file cannot be written.  simrank_index_load
 * reads such a file into device memory and makes it the graph's index,
 * replacing any earlier one (batch plans made before refuse to run, as after
 * a rebuild); stitched queries then give the counts they gave with the saved
 * index.  EINVAL, with the graph's index unchanged, if the file was written
 * for another graph (n, m or the fingerprint of its gather layout differ), is
 * truncated or longer than its arrays, or its arrays do not match their
 * checksums; EIO if it cannot be opened.  Synchronous; the same threading
 * rule as simrank_build_index. */
int simrank_index_save(const simrank_graph *g, const char *path);
int simrank_index_load(simrank_graph *g, const char *path);

/* ----------------------------------------------------------------- batch */

/* Runs nq queries over ngraphs graphs (qs[i].graph selects the graph; all
 * graphs on one device).  Consecutive queries are grouped into plans that fit
 * half of the free device memory (admission by memory); each plan is one
 * captured launch sequence (below).  outs[i]: host double[n of its graph] or
 * NULL; counts_opt (may be NULL, or entries NULL): host uint32[n].  Each
 * query's result equals what simrank_single_source_ex returns for it alone.
 * Stratified queries may be mixed in: outs[i] receives Algorithm 2's estimate
 * (as simrank_single_source_stratified's out) and counts_opt[i] is not
 * written.  st_opt: totals over all queries; ms is device time. */
int simrank_batch(simrank_graph *const *graphs, int32_t ngraphs, const simrank_query *qs,
                  int32_t nq, double *const *outs, uint32_t *const *counts_opt,
                  simrank_stats *st_opt);

/* A batch plan owns the device buffers of nq queries and a hipGraph of their
 * whole launch sequence: source walks of every query, compaction, one
 * persistent meet launch per kind whose work units span all its queries,
 * estimates.  It can be run any number of times.  ENOMEM if its buffers
 * exceed free memory. */
typedef struct simrank_batch_plan simrank_batch_plan;
int simrank_batch_plan_create(simrank_graph *const *graphs, int32_t ngraphs,
                              const simrank_query *qs, int32_t nq, simrank_batch_plan **plan_out);
/* Flags of simrank_batch_plan_create_ex. */
#define SIMRANK_PLAN_GROUPS 1u
/* simrank_batch_plan_create with flags (simrank_batch_plan_create and
 * simrank_batch pass SIMRANK_PLAN_GROUPS).  SIMRANK_PLAN_GROUPS: queries of one
 * mode on one graph with equal seed and walk parameters (plain and stitched:
 * c and walk cap; stratified: z, N and phi) are run in groups of up to 32
 * that share the walks from every node (Section 3's
 * walk (v, j), and Algorithm 1's walk in slot pi_v(j), depend on the seed and
 * those parameters only, not on the source): each walk (v, j) is taken once
 * and compared with walk j of every member's source.  Results are bit for bit
 * those without the flag; the stats count a shared walk's steps once.
 * n_groups_out (may be NULL) receives the number of groups formed.  EINVAL
 * for unknown flags. */
int simrank_batch_plan_create_ex(simrank_graph *const *graphs, int32_t ngraphs,
                                 const simrank_query *qs, int32_t nq, uint32_t flags,
                                 simrank_batch_plan **plan_out, int32_t *n_groups_out);
/* Enqueues the plan's graph on `stream` (hipStream_t; NULL = default stream).
 * Every run writes the plan's own buffers: runs of one plan must not overlap,
 * so enqueue the next run on the same stream or after simrank_batch_plan_wait.
 * Plans are independent of each other. */
int simrank_batch_plan_run(simrank_batch_plan *plan, void *stream);
/* Waits for the last run; st (may be NULL) receives totals and its device time. */
int simrank_batch_plan_wait(simrank_batch_plan *plan, simrank_stats *st);
/* Copies query i's estimate (host double[n], may be NULL) and counts (host
 * uint32[n], may be NULL) after the last run.  EINVAL for counts of a
 * stratified query. */
int simrank_batch_plan_read(simrank_batch_plan *plan, int32_t i, double *out_host,
                            uint32_t *counts_host);
/* A stratified query's results after the last run, as
 * simrank_single_source_stratified returns them (each host pointer may be
 * NULL): out double[n], out_n double[n], wsum uint64[n]. */
int simrank_batch_plan_read_stratified(simrank_batch_plan *plan, int32_t i, double *out_host,
                                       double *out_n_host, uint64_t *wsum_host);
int simrank_batch_plan_free(simrank_batch_plan *plan);

/* ---------------------------------------------------------------- tuning */

/* A tuner's choice for a graph. */
typedef struct simrank_tuning {
    int32_t unit_nodes;   /* nodes v per meet work unit (walks per block: unit_nodes x tile) */
    int32_t tile_walks;   /* source walks j per LDS tile */
    int32_t seg_log2;     /* the index's segment length 2^k (-1: no index) */
    int32_t reserved;
    double meet_ms;       /* meet-kernel time of the tuning query at this choice */
    double build_ms;      /* device time of the index build at this choice */
} simrank_tuning;

/* Measures the meet kernel of query q (plain or stitched) on g for each tile
 * of source walks (the kind's largest tile, 8192 for plain walks, halved down
 * to 2048) and each work-unit size (nodes per unit 32, 64, 128, 256, as long
 * as the units still number 64 or more) and keeps the fastest pair for later
 * queries on g, batches and servers included (*out, may be NULL).  Results
 * never depend on the choice.  Not to be called while other threads query g. */
int simrank_tune_ex(simrank_graph *g, const simrank_query *q, simrank_tuning *out);
/* simrank_tune_ex, returning the nodes per unit only (*vb_out, may be NULL). */
int simrank_tune(simrank_graph *g, const simrank_query *q, int32_t *vb_out);
/* Fixes the tuning by hand: unit_nodes in [0, 256] (0: the library's default
 * by graph size), tile_walks 0 (each kind's largest tile) or in [2048, 8192]
 * (clamped to each kind's largest tile).  Results never depend on it.  Not to
 * be called while other threads query g. */
int simrank_set_tuning(simrank_graph *g, int32_t unit_nodes, int32_t tile_walks);
/* Segment-length tuner for the stitched index (Section 4's segments of 2^k
 * steps joined by pointer doubling): for each seg_log2[i] (count in [1, 7],
 * each in [0, 6]) builds the index from *base with that k, times stitched
 * query q's meet kernel (second run) into ms_each[i] (may be NULL), and leaves
 * the index of the fastest k built (*out, may be NULL).  Stitched walks depend
 * on k: a query's counts are those of the index it ran with.  EINVAL if q is
 * not stitched or its c differs from base->c.  Rebuilds the index: the same
 * rules as simrank_build_index apply. */
int simrank_tune_index(simrank_graph *g, const simrank_query *q, const simrank_index_params *base,
                       const int32_t *seg_log2, int32_t count, simrank_tuning *out,
                       double *ms_each);

/* --------------------------------------------------------------- serving */

/* A request loop over one device-resident graph (and its index) with
 * continuous batching.  simrank_server_submit queues a request; a worker
 * thread admits queued requests oldest first as soon as a ring entry (at most
 * max_slots requests in flight) and the request's own device memory (its R, L
 * and mode decide how much, taken from the server's pool of hbm_budget bytes)
 * are free.  An admitted request's source walks and compaction are prepared
 * on the device and its work units (tiles of source walks x chunks of nodes)
 * are published into a device ring; persistent meet kernels take units from
 * every published request of their kind, oldest first, and exit when none is
 * left, so requests that arrive while others run join the work on the device
 * without waiting for it to end.  The block that finishes a request's last
 * unit writes its estimate and flags the request in pinned host memory; the
 * worker copies the results to the host and retires it.  Plain, stitched and
 * stratified requests are served; each result equals what the lone call
 * returns for the same query (simrank_single_source_ex, or
 * simrank_single_source_stratified). */
typedef struct simrank_server simrank_server;

typedef struct simrank_server_params {
    int32_t max_slots;    /* 1..64 requests in flight at once */
    int32_t max_R;        /* largest R (stratified: N) a request may need */
    int32_t max_L;        /* largest walk cap (stratified: phi) a request may use */
    int32_t group_max;    /* 0 or 1: every request runs alone.  2..32: a
                             request waits while a request with the same walks
                             runs (mode, seed, c and cap; stratified also N and
                             z); those that then wait together are admitted as
                             one query group of up to group_max, which takes
                             each walk (v, j) once for all of them (Section 3's
                             walk (v, j) does not depend on the source); one
                             group runs at a time, beside the lone requests.
                             If the pool cannot hold two of them, they run one
                             after another.  A grouped request's stats are its
                             share (1/G) of its group's work and the group's
                             device time. */
    int64_t hbm_budget;   /* device bytes for the requests in flight (the pool);
                             0: half the free memory.  At most max_slots requests
                             of (max_R, max_L) are reserved for. */
} simrank_server_params;

typedef struct simrank_request_info {
    double queue_s;       /* submit -> admission (its preparation enqueued) */
    double latency_s;     /* submit -> results in host memory */
    simrank_stats stats;  /* work of the request; ms and meet_ms: admission ->
                             completion on the host clock (a lone request shares
                             its kernels with others), or its group's device time */
} simrank_request_info;

/* The graph must outlive the server.  ENOMEM when the budget admits no
 * request of (max_R, max_L); EINVAL for max_slots outside [1, 64] or
 * group_max outside [0, 32]. */
int simrank_server_create(simrank_graph *g, const simrank_server_params *p,
                          simrank_server **server_out);
/* Requests of (max_R, max_L) the pool holds at once (at most max_slots), and
 * device bytes one such plain request takes. */
int simrank_server_info(const simrank_server *server, int32_t *slots, int64_t *slot_bytes);
/* Requests finished and failed so far, query groups launched and the
 * requests they held (each pointer may be NULL). */
int simrank_server_counts(simrank_server *server, uint64_t *done, uint64_t *failed,
                          uint64_t *groups, uint64_t *grouped);
/* Most requests in flight at once so far, the pool's size and peak use in
 * bytes, and the kernel launches made (persistent meet kernels and groups);
 * each pointer may be NULL. */
int simrank_server_load(simrank_server *server, int32_t *inflight_peak, int64_t *pool_bytes,
                        int64_t *pool_peak, uint64_t *launches);
/* Validates and queues a query (q->graph ignored); returns at once with a
 * ticket.  EINVAL when it needs R or L beyond the server's maximum, ENOMEM
 * when its buffers exceed the whole pool. */
int simrank_server_submit(simrank_server *server, const simrank_query *q, uint64_t *ticket);
/* *state: 0 queued, 1 running, 2 finished (a wait returns at once); EINVAL
 * for an unknown or retired ticket. */
int simrank_server_poll(simrank_server *server, uint64_t ticket, int32_t *state);
/* Waits up to timeout_s seconds (< 0: no limit) for a plain or stitched
 * request, copies its estimate (host double[n], may be NULL) and counts (host
 * uint32[n], may be NULL) and fills info (may be NULL); the ticket is then
 * retired.  ESTATE on timeout (the ticket stays valid); EINVAL for an unknown
 * or retired ticket (of two waits on one ticket, one receives the result, the
 * other EINVAL) and for a stratified request (nothing retired).  Safe to call
 * from several threads at once. */
int simrank_server_wait(simrank_server *server, uint64_t ticket, double timeout_s,
                        double *out_host, uint32_t *counts_host, simrank_request_info *info);
/* simrank_server_wait for a stratified request: out, out_n and wsum as
 * simrank_single_source_stratified returns them (host arrays of n, each may
 * be NULL).  EINVAL for a plain or stitched request (nothing retired). */
int simrank_server_wait_stratified(simrank_server *server, uint64_t ticket, double timeout_s,
                                   double *out_host, double *out_n_host, uint64_t *wsum_host,
                                   simrank_request_info *info);
/* Finishes the queued and running requests, then frees the server.  No other
 * call on the server may run during or after it. */
int simrank_server_destroy(simrank_server *server);

/* ---------------------------------------------------------------- errors */

/* Message of the last error on the calling thread ("" if none). */
const char *simrank_last_error(void);

/* Library version string. */
const char *simrank_version(void);

#ifdef __cplusplus
}
#endif

#endif /* SIMRANK_H */
