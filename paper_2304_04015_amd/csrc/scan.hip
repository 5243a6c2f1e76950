// Device-wide scans used by graph ingest (slot offsets, active-node list) and
// by the index build (pool offsets, slot owners).  Three passes: per-block
// partial reductions, one block scanning the partials, per-block scans that
// add the block's offset.  Each thread owns ITEMS consecutive values, so a
// wave touches 64 * ITEMS consecutive values per load.
#include "common.hpp"

namespace srk {
namespace {

constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

struct OpSum {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a + b; }
};
struct OpMax {
    template <typename T>
    __device__ T operator()(T a, T b) const { return a > b ? a : b; }
};

template <typename T, typename Op>
__device__ T wave_inclusive(T x, Op op) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x = op(x, y);
    }
    return x;
}

// Exclusive scan across the block; *block_total receives the reduction.
template <typename T, typename Op>
__device__ T block_exclusive(T x, Op op, T identity, T *block_total) {
    __shared__ T wave_tot[16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = (blockDim.x + 63) >> 6;
    T inc = wave_inclusive(x, op);
    if (lane == 63) wave_tot[wave] = inc;
    __syncthreads();
    T before = identity;
    T total = identity;
    for (int w = 0; w < nwaves; ++w) {
        if (w < wave) before = op(before, wave_tot[w]);
        total = op(total, wave_tot[w]);
    }
    __syncthreads();
    T excl = __shfl_up(inc, 1, 64);
    if (lane == 0) excl = identity;
    *block_total = total;
    return op(before, excl);
}

template <typename TIn, typename TAcc, typename Op>
__global__ __launch_bounds__(SCAN_BLOCK) void k_partials(const TIn *__restrict__ in, int64_t n,
                                                         TAcc *__restrict__ partial, Op op,
                                                         TAcc identity) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    TAcc acc = identity;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i)
        if (base + i < n) acc = op(acc, (TAcc)in[base + i]);
    TAcc tot;
    block_exclusive(acc, op, identity, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// One block: exclusive scan of nb partials in place; grand total to *total.
template <typename TAcc, typename Op>
__global__ __launch_bounds__(1024) void k_scan_partials(TAcc *__restrict__ partial, int64_t nb,
                                                        TAcc *__restrict__ total, Op op,
                                                        TAcc identity) {
    const int64_t per = (nb + blockDim.x - 1) / blockDim.x;
    const int64_t b0 = (int64_t)threadIdx.x * per;
    TAcc acc = identity;
    for (int64_t i = b0; i < b0 + per && i < nb; ++i) acc = op(acc, partial[i]);
    TAcc tot;
    TAcc run = block_exclusive(acc, op, identity, &tot);
    for (int64_t i = b0; i < b0 + per && i < nb; ++i) {
        TAcc v = partial[i];
        partial[i] = run;
        run = op(run, v);
    }
    if (threadIdx.x == 0 && total) *total = tot;
}

template <typename TIn, typename TAcc, typename Op, bool INCLUSIVE>
__global__ __launch_bounds__(SCAN_BLOCK) void k_apply(const TIn *__restrict__ in, int64_t n,
                                                      const TAcc *__restrict__ partial,
                                                      TAcc *__restrict__ out, Op op,
                                                      TAcc identity) {
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
    TAcc vals[SCAN_ITEMS];
    TAcc acc = identity;
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        vals[i] = (base + i < n) ? (TAcc)in[base + i] : identity;
        acc = op(acc, vals[i]);
    }
    TAcc tot;
    TAcc run = op(partial[blockIdx.x], block_exclusive(acc, op, identity, &tot));
#pragma unroll
    for (int i = 0; i < SCAN_ITEMS; ++i) {
        if (base + i < n) {
            if (INCLUSIVE) {
                run = op(run, vals[i]);
                out[base + i] = run;
            } else {
                out[base + i] = run;
                run = op(run, vals[i]);
            }
        }
    }
}

template <typename TIn, typename TAcc, typename Op, bool INCLUSIVE>
int scan_impl(const TIn *in, int64_t n, TAcc *out, TAcc *total_dev, Op op, TAcc identity,
              hipStream_t st) {
    if (n <= 0) return SIMRANK_OK;
    const int64_t nb = (n + SCAN_TILE - 1) / SCAN_TILE;
    TAcc *partial = nullptr;
    SRK_HIP(hipMallocAsync((void **)&partial, sizeof(TAcc) * (size_t)nb, st));
    k_partials<TIn, TAcc, Op><<<(unsigned)nb, SCAN_BLOCK, 0, st>>>(in, n, partial, op, identity);
    k_scan_partials<TAcc, Op><<<1, 1024, 0, st>>>(partial, nb, total_dev, op, identity);
    k_apply<TIn, TAcc, Op, INCLUSIVE>
        <<<(unsigned)nb, SCAN_BLOCK, 0, st>>>(in, n, partial, out, op, identity);
    SRK_HIP(hipGetLastError());
    SRK_HIP(hipFreeAsync(partial, st));
    return SIMRANK_OK;
}

}  // namespace

int scan_exclusive_u32_to_i64(const uint32_t *in, int64_t n, int64_t *out, int64_t *total_dev,
                              hipStream_t st) {
    return scan_impl<uint32_t, int64_t, OpSum, false>(in, n, out, total_dev, OpSum{}, (int64_t)0,
                                                      st);
}

int scan_exclusive_i64(const int64_t *in, int64_t n, int64_t *out, int64_t *total_dev,
                       hipStream_t st) {
    return scan_impl<int64_t, int64_t, OpSum, false>(in, n, out, total_dev, OpSum{}, (int64_t)0,
                                                     st);
}

int scan_inclusive_max_u32(uint32_t *data, int64_t n, hipStream_t st) {
    return scan_impl<uint32_t, uint32_t, OpMax, true>(data, n, data, (uint32_t *)nullptr, OpMax{},
                                                      0u, st);
}

}  // namespace srk
