// Measured ceilings: random gathers, Philox draws, streaming copy.
#include <algorithm>

#include "common.hpp"
#include "philox.hpp"
#include "simrank_roofline.h"

namespace srk {
namespace {

constexpr int RF_BLOCK = 256;

// 32-bit integer mixer (the finaliser of MurmurHash3).
__device__ __forceinline__ uint32_t mix32(uint32_t h) {
    h ^= h >> 16;
    h *= 0x85ebca6bu;
    h ^= h >> 13;
    h *= 0xc2b2ae35u;
    h ^= h >> 16;
    return h;
}

template <typename T>
__global__ __launch_bounds__(RF_BLOCK) void k_rf_fill(T *__restrict__ buf, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t next = (uint32_t)(((uint64_t)mix32((uint32_t)i ^ 0x9e3779b9u) * n) >> 32);
        buf[i] = (T)next;
    }
}

// Independent gathers: 4 loads in flight per lane per iteration.
template <typename T>
__global__ __launch_bounds__(RF_BLOCK) void k_rf_gather(const T *__restrict__ buf, uint64_t n,
                                                        int32_t iters, uint64_t *__restrict__ sink) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc = 0;
    uint32_t h = mix32(gid * 0x27d4eb2du + 1u);
    for (int32_t i = 0; i < iters; ++i) {
        uint64_t idx[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            h = mix32(h + 0x9e3779b9u);
            idx[u] = ((uint64_t)h * n) >> 32;
        }
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = buf[idx[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += (uint64_t)v[u];
    }
    if (acc == 0x5eed5eed5eedull) sink[0] = acc;   // keeps the loads
}

// The same independent gathers in a grid of the caller's shape (blocks of up
// to 1024 threads), to see whether the rate depends on the CUs or the waves
// that issue them.
template <typename T>
__global__ __launch_bounds__(1024) void k_rf_gather_grid(const T *__restrict__ buf, uint64_t n,
                                                         int32_t iters, uint64_t *__restrict__ sink) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc = 0;
    uint32_t h = mix32(gid * 0x27d4eb2du + 1u);
    for (int32_t i = 0; i < iters; ++i) {
        uint64_t idx[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            h = mix32(h + 0x9e3779b9u);
            idx[u] = ((uint64_t)h * n) >> 32;
        }
        T v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = buf[idx[u]];
#pragma unroll
        for (int u = 0; u < 4; ++u) acc += (uint64_t)v[u];
    }
    if (acc == 0x5eed5eed5eedull) sink[0] = acc;
}

// Dependent chains: each lane's next index is a hash of the value it just
// loaded and its own salt, so lanes never fall into shared paths (plain
// next = buf[cur] chains merge and then share cache lines).
template <typename T>
__global__ __launch_bounds__(RF_BLOCK) void k_rf_chase(const T *__restrict__ buf, uint64_t n,
                                                       int32_t iters, uint64_t *__restrict__ sink) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t salt = mix32(gid ^ 0xa5a5a5a5u);
    uint64_t cur = ((uint64_t)mix32(gid + 7u) * n) >> 32;
    for (int32_t i = 0; i < iters; ++i)
        cur = ((uint64_t)mix32((uint32_t)buf[cur] ^ salt ^ (uint32_t)i) * n) >> 32;
    if (cur == 0x5eed5eedull) sink[0] = cur;
}

__global__ __launch_bounds__(RF_BLOCK) void k_rf_philox(int32_t iters, PhiloxKey key,
                                                        uint64_t *__restrict__ sink) {
    const uint32_t gid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int32_t i = 0; i < iters; ++i) {
        const uint4 x = philox4x32_10(gid, (uint32_t)i, 0u, 0u, key);
        acc ^= x.x ^ x.y ^ x.z ^ x.w;
    }
    if (acc == 0x5eed5eedu) sink[0] = acc;
}

__global__ __launch_bounds__(RF_BLOCK) void k_rf_copy(const uint4 *__restrict__ src,
                                                      uint4 *__restrict__ dst, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

int full_grid() {
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    return std::max(cus, 1) * 8;   // 8 blocks x 4 waves = 32 waves per CU
}

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    hipStream_t st = nullptr;
    ~Timer() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
        if (st) (void)hipStreamDestroy(st);
    }
};

template <typename F>
int timed(F launch, double *ms_out) {
    Timer tm;
    SRK_HIP(hipStreamCreateWithFlags(&tm.st, hipStreamNonBlocking));
    SRK_HIP(hipEventCreate(&tm.a));
    SRK_HIP(hipEventCreate(&tm.b));
    launch(tm.st);                      // untimed
    SRK_HIP(hipGetLastError());
    SRK_HIP(hipEventRecord(tm.a, tm.st));
    launch(tm.st);
    SRK_HIP(hipEventRecord(tm.b, tm.st));
    SRK_HIP(hipGetLastError());
    SRK_HIP(hipEventSynchronize(tm.b));
    float ms = 0.f;
    SRK_HIP(hipEventElapsedTime(&ms, tm.a, tm.b));
    *ms_out = ms;
    return SIMRANK_OK;
}

template <typename T>
int gather_impl(int64_t footprint, int32_t dependent, simrank_rate *out, int32_t blocks = 0,
                int32_t threads = 0) {
    const uint64_t n = (uint64_t)footprint / sizeof(T);
    T *buf = nullptr;
    uint64_t *sink = nullptr;
    int rc = device_alloc((void **)&buf, sizeof(T) * n, nullptr);
    if (!rc) rc = device_alloc((void **)&sink, 8, nullptr);
    if (rc) {
        device_free(buf);
        device_free(sink);
        return rc;
    }
    const int grid = full_grid();
    k_rf_fill<T><<<grid, RF_BLOCK>>>(buf, n);
    const bool shaped = blocks > 0;
    const int64_t lanes = shaped ? (int64_t)blocks * threads : (int64_t)grid * RF_BLOCK;
    // about as many gathers as the full-grid launch, whatever the shape
    const int32_t iters = dependent ? 512
                          : shaped  ? (int32_t)std::max<int64_t>(256, (int64_t)grid * RF_BLOCK * 256 / lanes)
                                    : 256;
    double ms = 0;
    rc = timed(
        [&](hipStream_t st) {
            if (dependent)
                k_rf_chase<T><<<grid, RF_BLOCK, 0, st>>>(buf, n, iters, sink);
            else if (shaped)
                k_rf_gather_grid<T><<<blocks, threads, 0, st>>>(buf, n, iters, sink);
            else
                k_rf_gather<T><<<grid, RF_BLOCK, 0, st>>>(buf, n, iters, sink);
        },
        &ms);
    device_free(buf);
    device_free(sink);
    if (rc) return rc;
    const double count = (double)lanes * iters * (dependent ? 1 : 4);
    out->count = count;
    out->ms = ms;
    out->per_s = count / (ms * 1e-3);
    return SIMRANK_OK;
}

}  // namespace
}  // namespace srk

using namespace srk;

extern "C" int simrank_roofline_gather(int64_t footprint_bytes, int32_t entry_bytes,
                                       int32_t dependent, simrank_rate *out) {
    clear_error();
    if (!out) return fail(SIMRANK_EINVAL, "out is NULL");
    if (footprint_bytes < 4096) return fail(SIMRANK_EINVAL, "footprint below 4096 bytes");
    if (footprint_bytes / entry_bytes >= ((int64_t)1 << 32))
        return fail(SIMRANK_EINVAL, "footprint above 2^32 entries");
    if (entry_bytes == 4) return gather_impl<uint32_t>(footprint_bytes, dependent, out);
    if (entry_bytes == 8) return gather_impl<uint64_t>(footprint_bytes, dependent, out);
    return fail(SIMRANK_EINVAL, "entry_bytes must be 4 or 8");
}

extern "C" int simrank_roofline_gather_grid(int64_t footprint_bytes, int32_t entry_bytes,
                                            int32_t blocks, int32_t block_threads,
                                            simrank_rate *out) {
    clear_error();
    if (!out) return fail(SIMRANK_EINVAL, "out is NULL");
    if (footprint_bytes < 4096) return fail(SIMRANK_EINVAL, "footprint below 4096 bytes");
    if (footprint_bytes / entry_bytes >= ((int64_t)1 << 32))
        return fail(SIMRANK_EINVAL, "footprint above 2^32 entries");
    if (blocks < 1 || blocks > (1 << 20))
        return fail(SIMRANK_EINVAL, "blocks must be in [1, 2^20]");
    if (block_threads < 64 || block_threads > 1024 || block_threads % 64)
        return fail(SIMRANK_EINVAL, "block_threads must be a multiple of 64 in [64, 1024]");
    if (entry_bytes == 4) return gather_impl<uint32_t>(footprint_bytes, 0, out, blocks, block_threads);
    if (entry_bytes == 8) return gather_impl<uint64_t>(footprint_bytes, 0, out, blocks, block_threads);
    return fail(SIMRANK_EINVAL, "entry_bytes must be 4 or 8");
}

extern "C" int simrank_roofline_philox(simrank_rate *out) {
    clear_error();
    if (!out) return fail(SIMRANK_EINVAL, "out is NULL");
    uint64_t *sink = nullptr;
    int rc = device_alloc((void **)&sink, 8, nullptr);
    if (rc) return rc;
    const int grid = full_grid();
    const int32_t iters = 2048;
    double ms = 0;
    rc = timed([&](hipStream_t st) {
        k_rf_philox<<<grid, RF_BLOCK, 0, st>>>(iters, make_key(0x1234567887654321ull), sink);
    }, &ms);
    device_free(sink);
    if (rc) return rc;
    out->count = (double)grid * RF_BLOCK * iters;
    out->ms = ms;
    out->per_s = out->count / (ms * 1e-3);
    return SIMRANK_OK;
}

extern "C" int simrank_roofline_copy(int64_t bytes, simrank_rate *out) {
    clear_error();
    if (!out) return fail(SIMRANK_EINVAL, "out is NULL");
    if (bytes < (1 << 20)) return fail(SIMRANK_EINVAL, "copy size below 1 MiB");
    const uint64_t n = (uint64_t)bytes / 16;
    uint4 *a = nullptr, *b = nullptr;
    int rc = device_alloc((void **)&a, 16 * n, nullptr);
    if (!rc) rc = device_alloc((void **)&b, 16 * n, nullptr);
    if (rc) {
        device_free(a);
        device_free(b);
        return rc;
    }
    const int grid = full_grid() * 4;
    double ms = 0;
    rc = timed([&](hipStream_t st) { k_rf_copy<<<grid, RF_BLOCK, 0, st>>>(a, b, n); }, &ms);
    device_free(a);
    device_free(b);
    if (rc) return rc;
    out->count = 2.0 * 16.0 * (double)n;
    out->ms = ms;
    out->per_s = out->count / (ms * 1e-3);
    return SIMRANK_OK;
}
