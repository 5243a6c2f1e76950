/*
 * CPU oracle for Monte Carlo single-source SimRank with sqrt(c)-walks.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may load this file's
 * library: only the test suite, the smoke check and the benchmark's CPU-baseline
 * leg do.  It is single-threaded, slow on purpose and shares no code, header or
 * constant table with the GPU library.  Every function says which passage of
 * Luo & Zhu, "Massively Parallel Single-Source SimRanks in o(log n) Rounds"
 * (arXiv 2304.04015) it follows.
 *
 * Graph input everywhere: the in-edge CSR of G, i.e. the adjacency of the
 * reversed graph that the walks run on (Algorithm 1, "reverse the edges"):
 * I(v) = src[off[v] .. off[v+1]).
 *
 * Random numbers: Philox4x32-10, written from its published description
 * (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As Easy as 1, 2, 3",
 * SC'11).  Key = (seed low 32 bits, seed high 32 bits).  Counter =
 * (node, walk, step, domain) with domains
 *   0 = step of a plain walk, 1 = step of a pool segment,
 *   2 = pick of the pool slot a walk enters after its private head,
 *   3 = pick of the successor slot of a pool segment,
 *   4 = step of a fixed-length walk of the length-stratified estimator,
 *   5 = round keys of a node's walk shuffle.
 *
 * Readings of the paper that the oracle fixes:
 *  - a walk at step t first draws; it stops if x0 >= T, T = floor(sqrt(c)*2^32)
 *    (Section 2.2: stop with probability 1 - sqrt(c)); otherwise it stops at a
 *    node without in-neighbours (the paper is silent; a zero column of W), else
 *    it moves to in-neighbour number floor(x1 * deg / 2^32);
 *  - a stopped walk has no later positions (a length-l walk has l+1 nodes);
 *  - two walks meet when they hold the same node at the same index i >= 0
 *    (Lemma 2), counted once per pair however often they coincide
 *    (Section 4.4, "counted only once").
 *
 * Parity status: Philox, plain walks and plain meet counts are pinned by
 * published known-answer vectors, closed forms and distribution tests.  The
 * stitched-walk functions are pinned by their special cases (a segment at
 * least as long as the walk cap reduces them to plain walks, heads equal plain
 * prefixes, serial traversal) and, for the effect of shared pool slots, by the
 * exact meeting probability of two stitched walks on a six-node graph,
 * enumerated over every outcome of heads, entry picks and slot contents
 * (tests/test_oracle_stitched_exact.py).  The length-stratified
 * estimator is pinned by its expectation, computed exactly from first-meeting
 * probabilities (oracle/exact.py), by the permutation property of the shuffle
 * and by the class sizes.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (SC'11, Section 4.2: the Philox bijection with N=4, W=32,   */
/* ten rounds; multipliers and Weyl key increments as published there).      */
/* ------------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k[2] = {key_in[0], key_in[1]};
    for (int round = 0; round < 10; ++round) {
        if (round > 0) {              /* the key schedule advances between rounds */
            k[0] += 0x9E3779B9u;
            k[1] += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x[0];
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x[2];
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x[1] ^ k[0];
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x[3] ^ k[1];
        uint32_t y3 = lo0;
        x[0] = y0; x[1] = y1; x[2] = y2; x[3] = y3;
    }
    out[0] = x[0]; out[1] = x[1]; out[2] = x[2]; out[3] = x[3];
}

static void draw(uint64_t seed, uint32_t node, uint32_t walk, uint32_t step, uint32_t domain,
                 uint32_t out[4])
{
    uint32_t ctr[4] = {node, walk, step, domain};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    oracle_philox4x32_10(ctr, key, out);
}

/* Probability thresholds as integers: continue iff x0 < T; Pr = T / 2^32. */
uint32_t oracle_continue_threshold(double c)
{
    double t = floor(sqrt(c) * 4294967296.0);
    if (t >= 4294967295.0) return 0xffffffffu;
    if (t <= 0.0) return 0u;
    return (uint32_t)t;
}

/* Uniform pick in [0, k) from one 32-bit word: floor(x * k / 2^32). */
static uint64_t pick(uint32_t x, uint64_t k)
{
    return (uint64_t)(((unsigned __int128)x * k) >> 32);
}

/* ------------------------------------------------------------------------ */
/* Plain sqrt(c)-walk (Section 2.2; Lemma 2), truncated at L steps.          */
/* path[0..len] receives the visited nodes; returns len (number of moves).   */
/* ------------------------------------------------------------------------ */
int32_t oracle_walk_plain(const int32_t *off, const int32_t *src, uint64_t seed, uint32_t T,
                          int32_t L, int32_t v, uint32_t j, int32_t *path)
{
    int32_t cur = v;
    path[0] = v;
    int32_t t;
    for (t = 1; t <= L; ++t) {
        uint32_t x[4];
        draw(seed, (uint32_t)v, j, (uint32_t)t, 0u, x);
        if (x[0] >= T) break;                       /* stops with probability 1 - sqrt(c) */
        int32_t deg = off[cur + 1] - off[cur];
        if (deg == 0) break;                        /* no in-neighbour to move to */
        cur = src[off[cur] + (int32_t)pick(x[1], (uint64_t)deg)];
        path[t] = cur;
    }
    return t - 1;
}

/* Meet test between two complete walks (Lemma 2: same node at the same step,
 * any i >= 0 while both walks still exist; a pair counts once). */
static int walks_meet(const int32_t *a, int32_t la, const int32_t *b, int32_t lb, int32_t *first)
{
    int32_t lim = la < lb ? la : lb;
    for (int32_t i = 0; i <= lim; ++i)
        if (a[i] == b[i]) { if (first) *first = i; return 1; }
    if (first) *first = -1;
    return 0;
}

/*
 * Single-source meet counts (Section 2.2, Monte Carlo estimate H/N; the j-th
 * walk of s is paired with the j-th walk of v, Section 3.2).  For each listed
 * node vs[i]: cnt[i] = #{ j < R : walk (s,j) and walk (vs[i],j) meet }.
 *
 * work_opt (may be NULL), per listed node: the number of moves a walker needs
 * when it follows walk (v,j) only as far as the pair can still meet, i.e. up to
 * min(len_s, len_v, first meeting index), summed over j; for v == s it is 0
 * (the pair meets at index 0).  Used to state the work behind a throughput
 * figure; it does not enter the estimate.
 */
void oracle_meet_counts_plain(const int32_t *off, const int32_t *src, uint64_t seed, uint32_t T,
                              int32_t L, int32_t R, int32_t s, const int32_t *vs, int64_t nv,
                              uint32_t *cnt, uint64_t *work_opt)
{
    int32_t *sw = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * (size_t)(L + 1));
    int32_t *sl = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L + 1));
    for (int32_t j = 0; j < R; ++j)
        sl[j] = oracle_walk_plain(off, src, seed, T, L, s, (uint32_t)j, sw + (size_t)j * (L + 1));
    for (int64_t i = 0; i < nv; ++i) {
        uint32_t c = 0;
        uint64_t w = 0;
        for (int32_t j = 0; j < R; ++j) {
            int32_t lv = oracle_walk_plain(off, src, seed, T, L, vs[i], (uint32_t)j, pv);
            int32_t first;
            int met = walks_meet(sw + (size_t)j * (L + 1), sl[j], pv, lv, &first);
            c += (uint32_t)met;
            if (vs[i] != s) {
                int32_t lim = lv < sl[j] ? lv : sl[j];
                if (met && first < lim) lim = first;
                w += (uint64_t)lim;
            }
        }
        cnt[i] = c;
        if (work_opt) work_opt[i] = w;
    }
    free(sw); free(sl); free(pv);
}

/* Walk table: for the (v, j) pairs listed, path rows of L+1 int32 (-1 after the
 * walk ends) and lengths. */
void oracle_walk_table_plain(const int32_t *off, const int32_t *src, uint64_t seed, uint32_t T,
                             int32_t L, const int32_t *vs, const uint32_t *js, int64_t count,
                             int32_t *paths, int32_t *lens)
{
    for (int64_t i = 0; i < count; ++i) {
        int32_t *row = paths + (size_t)i * (L + 1);
        for (int32_t t = 0; t <= L; ++t) row[t] = -1;
        lens[i] = oracle_walk_plain(off, src, seed, T, L, vs[i], js[i], row);
    }
}

/* ------------------------------------------------------------------------ */
/* Stitched walks: per-node pools of short walk segments, joined end to      */
/* start, standing in for the few-round walk sampler the paper relies on     */
/* (Theorem 2 and Section 4.1: long walks from short ones by doubling).       */
/* ------------------------------------------------------------------------ */

/* Pool sizes: P(y) = ceil(kappa * dbar(y)), dbar(y) = number of occurrences of
 * y in src (its in-degree in the reversed graph, which is where walks arrive
 * from).  Written as plain counting. */
void oracle_pool_sizes(int32_t n, int64_t m, const int32_t *src, double kappa, int64_t *P)
{
    for (int32_t y = 0; y < n; ++y) P[y] = 0;
    for (int64_t e = 0; e < m; ++e) P[src[e]] += 1;
    for (int32_t y = 0; y < n; ++y) {
        double d = (double)P[y];
        P[y] = (int64_t)ceil(kappa * d);
    }
}

/* Segment (y, i): a walk from y of at most seglen steps keyed (y, i, t, 1) under
 * the index seed.  nodes[0..len) receive positions 1..len; returns len.  It is
 * open (has a successor) iff len == seglen. */
int32_t oracle_segment(const int32_t *off, const int32_t *src, uint64_t index_seed, uint32_t T,
                       int32_t seglen, int32_t y, uint32_t i, int32_t *nodes)
{
    int32_t cur = y;
    int32_t t;
    for (t = 1; t <= seglen; ++t) {
        uint32_t x[4];
        draw(index_seed, (uint32_t)y, i, (uint32_t)t, 1u, x);
        if (x[0] >= T) break;
        int32_t deg = off[cur + 1] - off[cur];
        if (deg == 0) break;
        cur = src[off[cur] + (int32_t)pick(x[1], (uint64_t)deg)];
        nodes[t - 1] = cur;
    }
    return t - 1;
}

/* Successor slot of an open segment (y, i) that ends at z. */
static uint32_t succ_slot(uint64_t index_seed, int32_t y, uint32_t i, const int64_t *P, int32_t z)
{
    uint32_t x[4];
    draw(index_seed, (uint32_t)y, i, 0u, 3u, x);
    return (uint32_t)pick(x[0], (uint64_t)P[z]);
}

/* Stitched walk (v, j): private head = the first min(seglen, L) steps of the
 * plain walk (v, j); if the head made all seglen moves and steps remain, the
 * walk enters slot (y, pick(draw(v,j,0,2).x0, P(y))) of the pool of its end
 * node y, and continues through segments, each regenerated from the CSR, until
 * one stops early or L steps are reached.  path[0..len]; returns len. */
int32_t oracle_walk_stitched(const int32_t *off, const int32_t *src, uint64_t seed,
                             uint64_t index_seed, uint32_t T, int32_t L, int32_t seglen,
                             const int64_t *P, int32_t v, uint32_t j, int32_t *path)
{
    int32_t head_cap = seglen < L ? seglen : L;
    int32_t len = oracle_walk_plain(off, src, seed, T, head_cap, v, j, path);
    if (len < seglen || len >= L) return len;
    int32_t y = path[len];
    uint32_t x[4];
    draw(seed, (uint32_t)v, j, 0u, 2u, x);
    uint32_t i = (uint32_t)pick(x[0], (uint64_t)P[y]);
    int32_t *seg = (int32_t *)malloc(sizeof(int32_t) * (size_t)seglen);
    for (;;) {
        int32_t sl = oracle_segment(off, src, index_seed, T, seglen, y, i, seg);
        for (int32_t t = 0; t < sl && len < L; ++t) path[++len] = seg[t];
        if (sl < seglen || len >= L) break;
        int32_t z = seg[seglen - 1];
        i = succ_slot(index_seed, y, i, P, z);
        y = z;
    }
    free(seg);
    return len;
}

void oracle_walk_table_stitched(const int32_t *off, const int32_t *src, uint64_t seed,
                                uint64_t index_seed, uint32_t T, int32_t L, int32_t seglen,
                                const int64_t *P, const int32_t *vs, const uint32_t *js,
                                int64_t count, int32_t *paths, int32_t *lens)
{
    for (int64_t i = 0; i < count; ++i) {
        int32_t *row = paths + (size_t)i * (L + 1);
        for (int32_t t = 0; t <= L; ++t) row[t] = -1;
        lens[i] = oracle_walk_stitched(off, src, seed, index_seed, T, L, seglen, P, vs[i], js[i], row);
    }
}

/* Meet counts over stitched walks (same pairing and meet rule as the plain
 * counts; both the source's and v's walks are stitched). */
void oracle_meet_counts_stitched(const int32_t *off, const int32_t *src, uint64_t seed,
                                 uint64_t index_seed, uint32_t T, int32_t L, int32_t seglen,
                                 const int64_t *P, int32_t R, int32_t s, const int32_t *vs,
                                 int64_t nv, uint32_t *cnt)
{
    int32_t *sw = (int32_t *)malloc(sizeof(int32_t) * (size_t)R * (size_t)(L + 1));
    int32_t *sl = (int32_t *)malloc(sizeof(int32_t) * (size_t)R);
    int32_t *pv = (int32_t *)malloc(sizeof(int32_t) * (size_t)(L + 1));
    for (int32_t j = 0; j < R; ++j)
        sl[j] = oracle_walk_stitched(off, src, seed, index_seed, T, L, seglen, P, s, (uint32_t)j,
                                     sw + (size_t)j * (L + 1));
    for (int64_t i = 0; i < nv; ++i) {
        uint32_t c = 0;
        for (int32_t j = 0; j < R; ++j) {
            int32_t lv = oracle_walk_stitched(off, src, seed, index_seed, T, L, seglen, P, vs[i],
                                              (uint32_t)j, pv);
            c += (uint32_t)walks_meet(sw + (size_t)j * (L + 1), sl[j], pv, lv, NULL);
        }
        cnt[i] = c;
    }
    free(sw); free(sl); free(pv);
}

/* Bulk draws for distribution tests: out[4i..4i+3] = Philox(ctr = (c0, c1, c2_first + i, c3)). */
void oracle_draw_block(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2_first, uint32_t c3,
                       int64_t count, uint32_t *out)
{
    for (int64_t i = 0; i < count; ++i)
        draw(seed, c0, c1, c2_first + (uint32_t)i, c3, out + 4 * i);
}

/* ------------------------------------------------------------------------ */
/* Length-stratified estimator (Algorithm 1: N_l walks of exact length l     */
/* from every node, l = 0..phi, then a shuffle of each node's walks;          */
/* Algorithm 2 with Lemma 5: the j-th walks of s and u are paired, and a      */
/* pair that meets adds (Z_l1 Z_l2) / (Zhat_l1 Zhat_l2) / z to s~(s,u)).       */
/* ------------------------------------------------------------------------ */

/* Parameters.  phi = floor(ln n / ln(1/sqrt c)) (Algorithm 1's walk length
 * cap), unless phi_override > 0 (the p-fold cap of the error-threshold
 * extension).  z = ln(2n) / (2 (eps - 3/n)^2) (Algorithm 2), unless
 * z_override > 0.  Z_l = z * sqrt(c)^l * (1 - sqrt(c)), the expected number of
 * length-l walks, and Zhat_l = ceil(Z_l) walks are generated (Section 5 on
 * rounding); N = sum of Zhat_l.  sqrt(c)^l is formed by repeated
 * multiplication.  Z and Zhat need phi + 1 entries (at most 256).
 * Returns 0, or -1 for an invalid request (eps <= 3/n, phi outside [0, 255]). */
int oracle_strat_params(int32_t n, double c, double eps, double z_override, int32_t phi_override,
                        double *z_out, int32_t *phi_out, int64_t *N_out, double *Z, int64_t *Zhat)
{
    double z;
    if (z_override > 0.0) {
        z = z_override;
    } else {
        double gap = eps - 3.0 / (double)n;
        if (!(gap > 0.0)) return -1;
        z = log(2.0 * (double)n) / (2.0 * gap * gap);
    }
    double r = sqrt(c);
    int32_t phi;
    if (phi_override > 0) {
        phi = phi_override;
    } else {
        double f = floor(log((double)n) / log(1.0 / r));
        if (!(f >= 0.0 && f <= 255.0)) return -1;
        phi = (int32_t)f;
    }
    if (phi > 255) return -1;
    double g = 1.0;                 /* sqrt(c)^l */
    int64_t N = 0;
    for (int32_t l = 0; l <= phi; ++l) {
        Z[l] = (z * g) * (1.0 - r);
        Zhat[l] = (int64_t)ceil(Z[l]);
        N += Zhat[l];
        g = g * r;
    }
    *z_out = z;
    *phi_out = phi;
    *N_out = N;
    return 0;
}

/* MurmurHash3's 32-bit finalizer (A. Appleby, public domain): the round
 * function of the shuffle's Feistel network. */
static uint32_t fmix32(uint32_t h)
{
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

/* A keyed bijection of the grid [0, A) x [0, B), B = 2^b: four rounds that
 * alternately add to the high coordinate, modulo A, a round-function value
 * scaled into [0, A), and XOR the low coordinate with the round-function
 * value's low b bits.  Each round is invertible when the other coordinate is
 * held, so the whole map is (a Feistel network over mixed radix, as in the
 * FF1 mode of NIST SP 800-38G).  The grid point (hi, lo) is the integer
 * hi * B + lo. */
static uint32_t feistel4(uint32_t x, uint32_t A, int b, const uint32_t k[4])
{
    uint32_t B = 1u << b;
    uint32_t hi = x >> b, lo = x & (B - 1u);
    hi = (uint32_t)(((uint64_t)hi + pick(fmix32(lo ^ k[0]), A)) % A);
    lo ^= fmix32(hi ^ k[1]) & (B - 1u);
    hi = (uint32_t)(((uint64_t)hi + pick(fmix32(lo ^ k[2]), A)) % A);
    lo ^= fmix32(hi ^ k[3]) & (B - 1u);
    return (hi << b) | lo;
}

/* Shuffle of node v's N walks (Section 4.2; the paper leaves the method
 * open): walk j after the shuffle is the walk generated in slot pi_v(j).
 * pi_v is the bijection above on the grid of A * B >= N points with
 * B = 2^ceil(ceil(log2 N) / 2) and A = ceil(N / B), restricted to [0, N) by
 * cycle walking (Black and Rogaway, "Ciphers with Arbitrary Finite Domains",
 * CT-RSA 2002): apply it again while the value is >= N.  Fewer than 2/sqrt(N)
 * of the grid's points lie beyond N.  Round keys: Philox(ctr = (v, 0, 0, 5)). */
uint32_t oracle_shuffle_slot(uint64_t seed, int32_t v, uint32_t j, int64_t N)
{
    int bits = 0;
    while (((int64_t)1 << bits) < N) ++bits;
    int b = (bits + 1) / 2;
    uint32_t A = (uint32_t)((N + ((int64_t)1 << b) - 1) >> b);
    uint32_t k[4];
    draw(seed, (uint32_t)v, 0u, 0u, 5u, k);
    uint32_t y = feistel4(j, A, b, k);
    while ((int64_t)y >= N) y = feistel4(y, A, b, k);
    return y;
}

/* Length class of generated slot r: the walks of node v are generated class
 * by class, Zhat_0 of length 0 first, then Zhat_1 of length 1, ... */
static int32_t slot_class(uint32_t r, const int64_t *Zhat, int32_t phi)
{
    int64_t start = 0;
    for (int32_t l = 0; l <= phi; ++l) {
        if ((int64_t)r < start + Zhat[l]) return l;
        start += Zhat[l];
    }
    return -1;   /* r >= N: not a slot */
}

/* The walk generated in slot r of node v: `length` uniform steps on the
 * reversed graph, step t picking in-neighbour floor(x1 * deg / 2^32) of
 * x = Philox(ctr = (v, r, t, 4)).  It ends early at a node without
 * in-neighbours (the paper does not say what a fixed-length walk does there).
 * path[0..len]; returns len. */
int32_t oracle_walk_strat(const int32_t *off, const int32_t *src, uint64_t seed, int32_t length,
                          int32_t v, uint32_t r, int32_t *path)
{
    int32_t cur = v;
    path[0] = v;
    int32_t t;
    for (t = 1; t <= length; ++t) {
        int32_t deg = off[cur + 1] - off[cur];
        if (deg == 0) break;
        uint32_t x[4];
        draw(seed, (uint32_t)v, r, (uint32_t)t, 4u, x);
        cur = src[off[cur] + (int32_t)pick(x[1], (uint64_t)deg)];
        path[t] = cur;
    }
    return t - 1;
}

/* Walk j of node v after the shuffle: its slot, class and path. */
int32_t oracle_walk_strat_j(const int32_t *off, const int32_t *src, uint64_t seed,
                            const int64_t *Zhat, int32_t phi, int64_t N, int32_t v, uint32_t j,
                            uint32_t *slot_out, int32_t *class_out, int32_t *path)
{
    uint32_t r = oracle_shuffle_slot(seed, v, j, N);
    int32_t l = slot_class(r, Zhat, phi);
    if (slot_out) *slot_out = r;
    if (class_out) *class_out = l;
    return oracle_walk_strat(off, src, seed, l, v, r, path);
}

void oracle_walk_table_strat(const int32_t *off, const int32_t *src, uint64_t seed,
                             const int64_t *Zhat, int32_t phi, int64_t N, const int32_t *vs,
                             const uint32_t *js, int64_t count, int32_t *paths, int32_t *lens,
                             uint32_t *slots, int32_t *classes)
{
    for (int64_t i = 0; i < count; ++i) {
        int32_t *row = paths + (size_t)i * (phi + 1);
        for (int32_t t = 0; t <= phi; ++t) row[t] = -1;
        lens[i] = oracle_walk_strat_j(off, src, seed, Zhat, phi, N, vs[i], js[i], slots + i,
                                      classes + i, row);
    }
}

/* Meet weight of a pair of classes (Lemma 5) in fixed point: the product
 * (Z_l1 / Zhat_l1) * (Z_l2 / Zhat_l2), scaled by 2^40 and truncated to an
 * integer, so that sums of weights are exact and independent of order. */
uint64_t oracle_strat_weight(const double *Z, const int64_t *Zhat, int32_t l1, int32_t l2)
{
    double a1 = Z[l1] / (double)Zhat[l1];
    double a2 = Z[l2] / (double)Zhat[l2];
    return (uint64_t)ldexp(a1 * a2, 40);
}

/*
 * Weighted meet sums of Algorithm 2 for the listed nodes u:
 *   wsum[i] = sum over j < N of [walks j of s and of u meet] * weight(l1, l2),
 * with l1, l2 the classes of the two walks and a meet = the same node at the
 * same step i >= 1 (the tuples of a walk are its steps 1..len, Section 4.3),
 * counted once per pair.  u == s has no pairs (its estimate is 1).
 * meets_opt: number of meeting pairs; work_opt: moves a walker needs to follow
 * walk j of u only as far as the pair can still meet (min(len_s, len_u, first
 * meeting step)), summed over j.
 */
void oracle_strat_sums(const int32_t *off, const int32_t *src, uint64_t seed, const double *Z,
                       const int64_t *Zhat, int32_t phi, int64_t N, int32_t s, const int32_t *vs,
                       int64_t nv, uint64_t *wsum, uint32_t *meets_opt, uint64_t *work_opt)
{
    int32_t *sw = (int32_t *)malloc(sizeof(int32_t) * (size_t)N * (size_t)(phi + 1));
    int32_t *sl = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *sc = (int32_t *)malloc(sizeof(int32_t) * (size_t)N);
    int32_t *pu = (int32_t *)malloc(sizeof(int32_t) * (size_t)(phi + 1));
    for (int64_t j = 0; j < N; ++j)
        sl[j] = oracle_walk_strat_j(off, src, seed, Zhat, phi, N, s, (uint32_t)j, NULL, sc + j,
                                    sw + (size_t)j * (phi + 1));
    for (int64_t i = 0; i < nv; ++i) {
        uint64_t acc = 0, work = 0;
        uint32_t meets = 0;
        if (vs[i] != s) {
            for (int64_t j = 0; j < N; ++j) {
                int32_t cu;
                int32_t lu = oracle_walk_strat_j(off, src, seed, Zhat, phi, N, vs[i], (uint32_t)j,
                                                 NULL, &cu, pu);
                const int32_t *ps = sw + (size_t)j * (phi + 1);
                int32_t lim = lu < sl[j] ? lu : sl[j];
                int32_t first = 0;
                for (int32_t t = 1; t <= lim; ++t)
                    if (ps[t] == pu[t]) { first = t; break; }
                if (first) {
                    acc += oracle_strat_weight(Z, Zhat, sc[j], cu);
                    meets += 1;
                    work += (uint64_t)first;
                } else {
                    work += (uint64_t)lim;
                }
            }
        }
        wsum[i] = acc;
        if (meets_opt) meets_opt[i] = meets;
        if (work_opt) work_opt[i] = work;
    }
    free(sw); free(sl); free(sc); free(pu);
}

/* Estimates from the weighted sums: Algorithm 2's s~(s,u) = wsum 2^-40 / z,
 * and the variant normalised by the N pairs actually formed,
 * s~(s,u) * N / z, whose expectation is the meeting probability of two
 * sqrt(c)-walks truncated at phi steps; both are 1 for u == s. */
void oracle_strat_estimates(const uint64_t *wsum, const int32_t *vs, int64_t nv, int32_t s,
                            double z, int64_t N, double *out, double *out_n)
{
    for (int64_t i = 0; i < nv; ++i) {
        if (vs[i] == s) {
            out[i] = 1.0;
            out_n[i] = 1.0;
            continue;
        }
        double x = ldexp((double)wsum[i], -40);
        out[i] = x / z;
        out_n[i] = (x / z) * ((double)N / z);
    }
}
