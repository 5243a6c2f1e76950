/*
 * Drives the C oracle (oracle/simrank_oracle.c, compiled into this program)
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer: reads an
 * in-edge CSR from a binary file, runs the plain meet counts with their work,
 * the pool sizes and stitched meet counts, the stratified parameters and
 * weighted sums, and walk tables, and prints every result as text so that
 * the test can compare them with the unsanitized library's.
 *
 * Input file: int32 n, int64 m, int32 off[n + 1], int32 src[m] (little endian).
 * Usage: oracle_sanitize_driver graph.bin s
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

uint32_t oracle_continue_threshold(double c);
void oracle_meet_counts_plain(const int32_t *off, const int32_t *src, uint64_t seed, uint32_t T,
                              int32_t L, int32_t R, int32_t s, const int32_t *vs, int64_t nv,
                              uint32_t *cnt, uint64_t *work_opt);
void oracle_walk_table_plain(const int32_t *off, const int32_t *src, uint64_t seed, uint32_t T,
                             int32_t L, const int32_t *vs, const uint32_t *js, int64_t count,
                             int32_t *paths, int32_t *lens);
void oracle_pool_sizes(int32_t n, int64_t m, const int32_t *src, double kappa, int64_t *P);
void oracle_meet_counts_stitched(const int32_t *off, const int32_t *src, uint64_t seed,
                                 uint64_t index_seed, uint32_t T, int32_t L, int32_t seglen,
                                 const int64_t *P, int32_t R, int32_t s, const int32_t *vs,
                                 int64_t nv, uint32_t *cnt);
int oracle_strat_params(int32_t n, double c, double eps, double z_override, int32_t phi_override,
                        double *z_out, int32_t *phi_out, int64_t *N_out, double *Z, int64_t *Zhat);
void oracle_strat_sums(const int32_t *off, const int32_t *src, uint64_t seed, const double *Z,
                       const int64_t *Zhat, int32_t phi, int64_t N, int32_t s, const int32_t *vs,
                       int64_t nv, uint64_t *wsum, uint32_t *meets_opt, uint64_t *work_opt);

static void *must(void *p) {
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(3);
    }
    return p;
}

int main(int argc, char **argv) {
    if (argc < 3) return 2;
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 2;
    int32_t n;
    int64_t m;
    if (fread(&n, 4, 1, f) != 1 || fread(&m, 8, 1, f) != 1 || n < 1 || m < 0) return 2;
    int32_t *off = must(malloc(4 * ((size_t)n + 1)));
    int32_t *src = must(malloc(4 * (size_t)(m > 0 ? m : 1)));
    if (fread(off, 4, (size_t)n + 1, f) != (size_t)n + 1) return 2;
    if (m > 0 && fread(src, 4, (size_t)m, f) != (size_t)m) return 2;
    fclose(f);
    const int32_t s = atoi(argv[2]);
    const double c = 0.6;
    const uint32_t T = oracle_continue_threshold(c);
    int32_t *vs = must(malloc(4 * (size_t)n));
    for (int32_t v = 0; v < n; ++v) vs[v] = v;

    uint32_t *cnt = must(malloc(4 * (size_t)n));
    uint64_t *work = must(malloc(8 * (size_t)n));
    oracle_meet_counts_plain(off, src, 0x51u, T, 32, 300, s, vs, n, cnt, work);
    printf("plain");
    for (int32_t v = 0; v < n; ++v) printf(" %u", cnt[v]);
    printf("\nwork");
    for (int32_t v = 0; v < n; ++v) printf(" %llu", (unsigned long long)work[v]);
    printf("\n");

    int64_t *P = must(malloc(8 * (size_t)n));
    oracle_pool_sizes(n, m, src, 1.0, P);
    oracle_meet_counts_stitched(off, src, 0x52u, 0x53u, T, 32, 4, P, 200, s, vs, n, cnt);
    printf("stitched");
    for (int32_t v = 0; v < n; ++v) printf(" %u", cnt[v]);
    printf("\n");

    double z, Z[256];
    int32_t phi;
    int64_t N, Zhat[256];
    if (oracle_strat_params(n, c, 0.1, 400.0, 8, &z, &phi, &N, Z, Zhat) != 0) return 4;
    uint64_t *wsum = must(malloc(8 * (size_t)n));
    oracle_strat_sums(off, src, 0x54u, Z, Zhat, phi, N, s, vs, n, wsum, NULL, NULL);
    printf("strat");
    for (int32_t v = 0; v < n; ++v) printf(" %llu", (unsigned long long)wsum[v]);
    printf("\n");

    const int64_t cntw = 64;
    int32_t *wv = must(malloc(4 * (size_t)cntw));
    uint32_t *wj = must(malloc(4 * (size_t)cntw));
    int32_t *paths = must(malloc(4 * (size_t)cntw * 33));
    int32_t *lens = must(malloc(4 * (size_t)cntw));
    for (int64_t i = 0; i < cntw; ++i) {
        wv[i] = (int32_t)((i * 7) % n);
        wj[i] = (uint32_t)i;
    }
    oracle_walk_table_plain(off, src, 0x55u, T, 32, wv, wj, cntw, paths, lens);
    printf("walks");
    for (int64_t i = 0; i < cntw * 33; ++i) printf(" %d", paths[i]);
    printf("\n");

    free(off); free(src); free(vs); free(cnt); free(work); free(P); free(wsum);
    free(wv); free(wj); free(paths); free(lens);
    return 0;
}
