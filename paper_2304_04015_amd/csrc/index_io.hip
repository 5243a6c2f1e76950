// Saving and loading a graph's stitched-walk index, so that a server can
// restart without rebuilding it (the index is a pure function of the graph,
// k, kappa, c and its seed; the file holds the arrays the build produced).
//
// File layout (little endian): a 128-byte header (IndexFileHeader below),
// then pool_off (int64[n + 1]), the segment rows (uint32[segments][2^k]),
// segment lengths (uint8[segments]), successors (uint32[segments]) and the
// doubled chains (uint32[segments][64 / 2^k]).  The header carries a
// fingerprint of the graph's gather layout and a checksum of every array;
// both are recomputed on the device at load, and a file that does not match
// them, the graph or its own sizes is refused (EINVAL) without touching the
// graph's current index.
#include <cstdio>
#include <cstring>
#include <string>

#include "common.hpp"

namespace srk {
namespace {

constexpr char INDEX_MAGIC[8] = {'S', 'R', 'K', 'I', 'N', 'D', 'E', 'X'};
constexpr uint32_t INDEX_FILE_VERSION = 1;

struct IndexFileHeader {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    int32_t n;
    int32_t seg_log2;
    int64_t m;
    int64_t segments;
    double kappa;
    double c;
    uint64_t seed;
    uint32_t T;
    int32_t width;
    uint64_t graph_fp;
    uint64_t cs[5];       // pool_off, rows, lengths, successors, chains
    uint64_t build_moves;
};
static_assert(sizeof(IndexFileHeader) == 128, "index file header is 128 bytes");

// SplitMix64's output function (Steele, Lea, Flood, "Fast splittable
// pseudorandom number generators", OOPSLA 2014), used as a mixer.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// Order-independent checksum of `bytes` bytes: the sum, modulo 2^64, of
// mix64 over (8-byte word i + i * golden ratio + salt), the last word zero
// padded.
__global__ void k_checksum(const uint8_t *__restrict__ p, int64_t bytes, uint64_t salt,
                           unsigned long long *__restrict__ out) {
    const int64_t words = bytes / 8;
    const uint64_t *w = (const uint64_t *)p;
    uint64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += mix64(w[i] + (uint64_t)i * 0x9e3779b97f4a7c15ull + salt);
    if (blockIdx.x == 0 && threadIdx.x == 0 && (bytes & 7)) {
        uint64_t last = 0;
        for (int64_t b = words * 8; b < bytes; ++b) last |= (uint64_t)p[b] << (8 * (b - words * 8));
        acc += mix64(last + (uint64_t)words * 0x9e3779b97f4a7c15ull + salt);
    }
    for (int d = 32; d > 0; d >>= 1) acc += __shfl_xor(acc, d, 64);
    if ((threadIdx.x & 63) == 0 && acc) atomicAdd(out, (unsigned long long)acc);
}

int device_checksum(const void *p, int64_t bytes, uint64_t salt, unsigned long long *scratch,
                    hipStream_t st, uint64_t *out) {
    SRK_HIP(hipMemsetAsync(scratch, 0, 8, st));
    if (bytes > 0) {
        const int64_t words = bytes / 8 + 1;
        const unsigned blocks = (unsigned)std::min<int64_t>((words + 255) / 256, 4096);
        k_checksum<<<blocks, 256, 0, st>>>((const uint8_t *)p, bytes, salt, scratch);
    }
    unsigned long long v = 0;
    SRK_HIP(hipMemcpyAsync(&v, scratch, 8, hipMemcpyDeviceToHost, st));
    SRK_HIP(hipStreamSynchronize(st));
    *out = (uint64_t)v;
    return SIMRANK_OK;
}

// Fingerprint of the graph as the library holds it: its node table and gather
// layout, which the CSR determines.
int graph_fingerprint(const Graph *g, unsigned long long *scratch, hipStream_t st, uint64_t *fp) {
    uint64_t a = 0, b = 0;
    int rc = device_checksum(g->nodes, 8 * (int64_t)g->n, 0x51ull, scratch, st, &a);
    if (!rc) rc = device_checksum(g->E, 8 * g->m_slots, 0x52ull, scratch, st, &b);
    *fp = a ^ ((b << 17) | (b >> 47)) ^ ((uint64_t)g->n << 32) ^ (uint64_t)g->m;
    return rc;
}

struct Arr {
    void *dev;
    int64_t bytes;
};

void index_arrays(const Index *ix, int32_t n, Arr a[5]) {
    const int64_t S = ix->segments;
    a[0] = {ix->pool_off, 8 * ((int64_t)n + 1)};
    a[1] = {ix->seg, 4 * S * ix->seg_len};
    a[2] = {ix->seg_lens, S};
    a[3] = {ix->succ, 4 * S};
    a[4] = {ix->chain, 4 * S * ix->width};
}

constexpr size_t IO_CHUNK = (size_t)64 << 20;   // bytes per pinned staging transfer

}  // namespace
}  // namespace srk

using namespace srk;

extern "C" int simrank_index_save(const simrank_graph *g, const char *path) {
    clear_error();
    if (!g || !path) return fail(SIMRANK_EINVAL, "NULL argument");
    if (!g->index) return fail(SIMRANK_ESTATE, "no index built");
    const Index *ix = g->index;
    SRK_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    SRK_HIP(hipStreamSynchronize(st));
    unsigned long long *scratch = nullptr;
    int rc = device_alloc((void **)&scratch, 8, nullptr);
    if (rc) return rc;
    IndexFileHeader h;
    std::memset(&h, 0, sizeof(h));
    std::memcpy(h.magic, INDEX_MAGIC, 8);
    h.version = INDEX_FILE_VERSION;
    h.header_bytes = sizeof(h);
    h.n = g->n;
    h.seg_log2 = ix->seg_log2;
    h.m = g->m;
    h.segments = ix->segments;
    h.kappa = ix->kappa;
    h.c = ix->c;
    h.seed = ix->seed;
    h.T = ix->T;
    h.width = ix->width;
    h.build_moves = ix->build_moves;
    Arr a[5];
    index_arrays(ix, g->n, a);
    rc = graph_fingerprint(g, scratch, st, &h.graph_fp);
    for (int i = 0; i < 5 && !rc; ++i)
        rc = device_checksum(a[i].dev, a[i].bytes, 0x100ull + i, scratch, st, &h.cs[i]);
    char *stage = nullptr;
    FILE *f = nullptr;
    if (!rc && hipHostMalloc((void **)&stage, IO_CHUNK) != hipSuccess) {
        (void)hipGetLastError();
        stage = nullptr;
        rc = fail(SIMRANK_ENOMEM, "pinned staging buffer");
    }
    if (!rc) {
        f = std::fopen(path, "wb");
        if (!f) rc = fail(SIMRANK_EIO, std::string("cannot open ") + path + " for writing");
    }
    if (!rc && std::fwrite(&h, sizeof(h), 1, f) != 1) rc = fail(SIMRANK_EIO, "write failed");
    for (int i = 0; i < 5 && !rc; ++i) {
        for (int64_t off = 0; off < a[i].bytes && !rc; off += (int64_t)IO_CHUNK) {
            const size_t len = (size_t)std::min<int64_t>((int64_t)IO_CHUNK, a[i].bytes - off);
            hipError_t e = hipMemcpyAsync(stage, (const char *)a[i].dev + off, len,
                                          hipMemcpyDeviceToHost, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
            else if (std::fwrite(stage, 1, len, f) != len) rc = fail(SIMRANK_EIO, "write failed");
        }
    }
    if (f && std::fclose(f) != 0 && !rc) rc = fail(SIMRANK_EIO, "close failed");
    if (stage) (void)hipHostFree(stage);
    device_free(scratch);
    return rc;
}

extern "C" int simrank_index_load(simrank_graph *g, const char *path) {
    clear_error();
    if (!g || !path) return fail(SIMRANK_EINVAL, "NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(SIMRANK_EIO, std::string("cannot open ") + path);
    IndexFileHeader h;
    if (std::fread(&h, sizeof(h), 1, f) != 1) {
        std::fclose(f);
        return fail(SIMRANK_EINVAL, "index file shorter than its header");
    }
    auto refuse = [&](const std::string &why) {
        std::fclose(f);
        return fail(SIMRANK_EINVAL, "index file refused: " + why);
    };
    if (std::memcmp(h.magic, INDEX_MAGIC, 8) != 0) return refuse("not an index file");
    if (h.version != INDEX_FILE_VERSION || h.header_bytes != sizeof(h))
        return refuse("unknown version");
    if (h.n != g->n || h.m != g->m) return refuse("built for another graph (n, m)");
    if (h.seg_log2 < 0 || h.seg_log2 > 6 || h.width != MAX_STITCH_CAP >> h.seg_log2)
        return refuse("segment length");
    if (!(h.c > 0.0 && h.c < 1.0) || h.T != continue_threshold(h.c) || !(h.kappa > 0.0))
        return refuse("decay or pool scale");
    if (h.segments < 0 || h.segments >= (int64_t)NIL) return refuse("segment count");
    {   // the file's size must be the header's arrays, checked before any allocation
        const int64_t S = h.segments, L = (int64_t)1 << h.seg_log2;
        const int64_t want = (int64_t)sizeof(h) + 8 * ((int64_t)h.n + 1) + 4 * S * L + S + 4 * S +
                             4 * S * h.width;
        if (std::fseek(f, 0, SEEK_END) != 0) return refuse("cannot seek");
        const long size = std::ftell(f);
        if (size < 0 || (int64_t)size != want) return refuse("size does not match its header");
        if (std::fseek(f, (long)sizeof(h), SEEK_SET) != 0) return refuse("cannot seek");
    }
    SRK_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    SRK_HIP(hipStreamSynchronize(st));
    unsigned long long *scratch = nullptr;
    int rc = device_alloc((void **)&scratch, 8, nullptr);
    uint64_t fp = 0;
    if (!rc) rc = graph_fingerprint(g, scratch, st, &fp);
    if (!rc && fp != h.graph_fp) rc = fail(SIMRANK_EINVAL, "index file refused: built for another graph");
    Index *ix = new Index();
    ix->seg_log2 = h.seg_log2;
    ix->seg_len = 1 << h.seg_log2;
    ix->width = h.width;
    ix->levels = 0;
    while ((1 << ix->levels) < ix->width) ++ix->levels;
    ix->kappa = h.kappa;
    ix->c = h.c;
    ix->T = h.T;
    ix->seed = h.seed;
    ix->segments = h.segments;
    ix->build_moves = h.build_moves;
    const int64_t S = h.segments > 0 ? h.segments : 1;
    if (!rc) rc = device_alloc((void **)&ix->pool_off, 8 * ((size_t)g->n + 1), &ix->bytes);
    if (!rc) rc = device_alloc((void **)&ix->seg, 4 * (size_t)S * ix->seg_len, &ix->bytes);
    if (!rc) rc = device_alloc((void **)&ix->seg_lens, (size_t)S, &ix->bytes);
    if (!rc) rc = device_alloc((void **)&ix->succ, 4 * (size_t)S, &ix->bytes);
    if (!rc) rc = device_alloc((void **)&ix->chain, 4 * (size_t)S * ix->width, &ix->bytes);
    char *stage = nullptr;
    if (!rc && hipHostMalloc((void **)&stage, IO_CHUNK) != hipSuccess) {
        (void)hipGetLastError();
        stage = nullptr;
        rc = fail(SIMRANK_ENOMEM, "pinned staging buffer");
    }
    Arr a[5];
    index_arrays(ix, g->n, a);
    for (int i = 0; i < 5 && !rc; ++i) {
        for (int64_t off = 0; off < a[i].bytes && !rc; off += (int64_t)IO_CHUNK) {
            const size_t len = (size_t)std::min<int64_t>((int64_t)IO_CHUNK, a[i].bytes - off);
            if (std::fread(stage, 1, len, f) != len) {
                rc = fail(SIMRANK_EINVAL, "index file refused: shorter than its arrays");
                break;
            }
            hipError_t e = hipMemcpyAsync((char *)a[i].dev + off, stage, len, hipMemcpyHostToDevice, st);
            if (e == hipSuccess) e = hipStreamSynchronize(st);
            if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
        }
    }
    if (!rc && std::fgetc(f) != EOF) rc = fail(SIMRANK_EINVAL, "index file refused: longer than its arrays");
    std::fclose(f);
    for (int i = 0; i < 5 && !rc; ++i) {
        uint64_t cs = 0;
        rc = device_checksum(a[i].dev, a[i].bytes, 0x100ull + i, scratch, st, &cs);
        if (!rc && cs != h.cs[i]) rc = fail(SIMRANK_EINVAL, "index file refused: checksum mismatch");
    }
    int64_t last = -1;
    if (!rc) {
        hipError_t e = hipMemcpyAsync(&last, ix->pool_off + g->n, 8, hipMemcpyDeviceToHost, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        if (e != hipSuccess) rc = fail(SIMRANK_EDEVICE, hipGetErrorString(e));
        else if (last != h.segments) rc = fail(SIMRANK_EINVAL, "index file refused: pool offsets");
    }
    if (stage) (void)hipHostFree(stage);
    device_free(scratch);
    if (rc) {
        index_free(ix);
        delete ix;
        return rc;
    }
    ++g->index_gen;   // plans made with the old index must not run on this one
    if (g->index) {
        index_free(g->index);
        delete g->index;
    }
    g->index = ix;
    return SIMRANK_OK;
}
