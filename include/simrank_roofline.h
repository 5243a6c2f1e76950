/*
 * simrank_roofline.h — measured ceilings for the SimRank walk kernels on the
 * current HIP device (gfx950).
 *
 * The walk kernels of simrank.h are bound by random gathers (one edge slot per
 * walk step, Section 2.2's sqrt(c)-walk) and by Philox arithmetic (one draw per
 * step).  These calls measure the machine's own rates for those two patterns,
 * so a kernel can be stated as a fraction of what the hardware sustains:
 *   - random gathers of `entry_bytes` at uniform random addresses over a buffer
 *     of `footprint_bytes`, either independent (addresses from a hash) or as
 *     dependent chains (each address read from the previous load, like a walk);
 *   - Philox4x32-10 draws with no memory traffic;
 *   - a streaming device-to-device copy (HBM bandwidth).
 * Each call allocates and frees its own device buffers, runs one untimed and one
 * timed launch at full occupancy, and times the launch with HIP events.
 * Returns SIMRANK_OK or a SIMRANK_E* code (simrank.h); *out is unchanged on error.
 */
#ifndef SIMRANK_ROOFLINE_H
#define SIMRANK_ROOFLINE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct simrank_rate {
    double per_s;     /* operations (gathers, draws) or bytes per second */
    double ms;        /* duration of the timed launch */
    double count;     /* operations or bytes in the timed launch */
} simrank_rate;

/* Random gathers.  footprint_bytes: buffer size (>= 4096, rounded down to a
 * whole number of entries); entry_bytes: 4 or 8; dependent: 0 = independent
 * addresses, 1 = chains where each load supplies the next index. */
int simrank_roofline_gather(int64_t footprint_bytes, int32_t entry_bytes, int32_t dependent,
                            simrank_rate *out);

/* Independent random gathers as above, in a grid of `blocks` blocks of
 * `block_threads` threads (a multiple of 64 in [64, 1024]; blocks in
 * [1, 2^20]) instead of the full-occupancy grid; each lane keeps 4 gathers in
 * flight, and the launch makes at least as many gathers as the full grid's.
 * With fewer CUs or fewer waves per CU than the full grid it shows whether
 * the gather rate is set per CU or by the memory system as a whole. */
int simrank_roofline_gather_grid(int64_t footprint_bytes, int32_t entry_bytes, int32_t blocks,
                                 int32_t block_threads, simrank_rate *out);

/* Philox4x32-10 draws per second (counter (lane, i, 0, 0), all four words used). */
int simrank_roofline_philox(simrank_rate *out);

/* Streaming copy of `bytes` (>= 1 MiB): out->per_s is bytes moved (read +
 * write) per second. */
int simrank_roofline_copy(int64_t bytes, simrank_rate *out);

#ifdef __cplusplus
}
#endif

#endif /* SIMRANK_ROOFLINE_H */
