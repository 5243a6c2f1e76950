/*
 * A plain C99 client of the library's C ABI (include/simrank.h), with no
 * Python or torch in the process: it builds a seeded random in-edge CSR,
 * loads it, runs one single-source query through simrank_single_source_ex and
 * one through simrank_single_source (host buffers), and checks the meet counts
 * of every node against the CPU oracle's (oracle/liboracle.so, linked for this
 * test only), bit for bit, and the estimate against counts / R.
 *
 * Usage: c_abi_client [n] [R]; exit status 0 when everything agrees.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "simrank.h"

/* the oracle's entry points (oracle/simrank_oracle.c) */
uint32_t oracle_continue_threshold(double c);
void oracle_meet_counts_plain(const int32_t *off, const int32_t *src, uint64_t seed, uint32_t T,
                              int32_t L, int32_t R, int32_t s, const int32_t *vs, int64_t nv,
                              uint32_t *cnt, uint64_t *work_opt);

/* splitmix64: the test's own input generator */
static uint64_t next_u64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static int fail_with(const char *what, int rc) {
    fprintf(stderr, "c_abi_client: %s failed (%d): %s\n", what, rc, simrank_last_error());
    return 1;
}

int main(int argc, char **argv) {
    const int32_t n = argc > 1 ? (int32_t)atoi(argv[1]) : 3000;
    const int32_t R = argc > 2 ? (int32_t)atoi(argv[2]) : 1500;
    const int32_t L = 32;
    const double c = 0.6;
    const uint64_t seed = 0x2304040150000C01ull;
    if (n < 2 || R < 1) return 2;

    /* in-degrees 0..7 (about one node in eight without in-neighbours), sources uniform */
    uint64_t rng = 7;
    int32_t *off = malloc(sizeof(int32_t) * ((size_t)n + 1));
    off[0] = 0;
    for (int32_t v = 0; v < n; ++v) off[v + 1] = off[v] + (int32_t)(next_u64(&rng) % 8);
    const int64_t m = off[n];
    int32_t *src = malloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t e = 0; e < m; ++e) src[e] = (int32_t)(next_u64(&rng) % (uint64_t)n);
    int32_t s = 0;
    while (s < n && off[s + 1] == off[s]) ++s;   /* a source with in-neighbours */
    if (s == n) return 2;

    simrank_graph *g = NULL;
    int rc = simrank_load_graph(n, m, off, src, &g);
    if (rc) return fail_with("simrank_load_graph", rc);

    simrank_query q;
    memset(&q, 0, sizeof(q));
    q.s = s;
    q.c = c;
    q.eps = 0.05;
    q.delta = 1e-3;
    q.seed = seed;
    q.walk_cap = L;
    q.R_override = R;
    q.mode = SIMRANK_MODE_PLAIN;
    double *out = malloc(sizeof(double) * (size_t)n);
    uint32_t *cnt = malloc(sizeof(uint32_t) * (size_t)n);
    simrank_stats st;
    rc = simrank_single_source_ex(g, &q, out, cnt, &st);
    if (rc) return fail_with("simrank_single_source_ex", rc);

    int32_t *vs = malloc(sizeof(int32_t) * (size_t)n);
    for (int32_t v = 0; v < n; ++v) vs[v] = v;
    uint32_t *want = malloc(sizeof(uint32_t) * (size_t)n);
    oracle_meet_counts_plain(off, src, seed, oracle_continue_threshold(c), L, R, s, vs, n, want, NULL);
    int64_t bad = 0;
    for (int32_t v = 0; v < n; ++v) {
        if (cnt[v] != want[v]) ++bad;
        if (out[v] != (v == s ? 1.0 : (double)cnt[v] / (double)R)) ++bad;
    }
    if (bad) {
        fprintf(stderr, "c_abi_client: %lld entries differ from the oracle\n", (long long)bad);
        return 1;
    }

    /* the problem statement's entry point: seed 0, cap 64, R from (eps, delta) */
    rc = simrank_single_source(g, s, c, 0.05, 1e-3, out);
    if (rc) return fail_with("simrank_single_source", rc);
    for (int32_t v = 0; v < n; ++v)
        if (!(out[v] >= 0.0 && out[v] <= 1.0)) ++bad;
    if (bad || out[s] != 1.0) {
        fprintf(stderr, "c_abi_client: estimate outside [0, 1] or s(s, s) != 1\n");
        return 1;
    }
    /* errors come back as codes with a message, nothing written */
    out[0] = -7.0;
    rc = simrank_single_source(g, n, c, 0.05, 1e-3, out);
    if (rc != SIMRANK_EINVAL || out[0] != -7.0 || simrank_last_error()[0] == '\0') {
        fprintf(stderr, "c_abi_client: a source out of range was not rejected\n");
        return 1;
    }
    rc = simrank_free_graph(g);
    if (rc) return fail_with("simrank_free_graph", rc);
    printf("c_abi_client ok: n=%d m=%lld s=%d R=%d meets=%llu moves=%llu\n", n, (long long)m, s, R,
           (unsigned long long)st.meets, (unsigned long long)st.moves);
    free(off);
    free(src);
    free(out);
    free(cnt);
    free(vs);
    free(want);
    return 0;
}
