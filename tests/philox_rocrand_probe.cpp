// Evaluates rocRAND's Philox4x32-10 engine (its header-only implementation,
// compiled for the host) at given (counter, key) pairs, so that the oracle's
// Philox can be checked against an implementation it shares nothing with.
//
// rocRAND's engine with seed S and subsequence Q, advanced by 4B outputs,
// holds key (S mod 2^32, S >> 32) and counter (B mod 2^32, B >> 32,
// Q mod 2^32, Q >> 32); its next four outputs are one Philox4x32-10 block.
// B is added in steps below 2^60 blocks, since the offset counts outputs.
//
// stdin: lines "c0 c1 c2 c3 k0 k1" in hex; stdout: "x0 x1 x2 x3" in hex.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main() {
    unsigned c[4], k[2];
    while (std::scanf("%x %x %x %x %x %x", &c[0], &c[1], &c[2], &c[3], &k[0], &k[1]) == 6) {
        const unsigned long long seed = (static_cast<unsigned long long>(k[1]) << 32) | k[0];
        const unsigned long long sub = (static_cast<unsigned long long>(c[3]) << 32) | c[2];
        const unsigned long long blk = (static_cast<unsigned long long>(c[1]) << 32) | c[0];
        rocrand_device::philox4x32_10_engine e(seed, sub, 0);
        for (unsigned long long i = 0; i < (blk >> 60); ++i) e.discard(1ull << 62);
        e.discard(4ull * (blk & ((1ull << 60) - 1)));
        const uint4 x = e.next4();
        std::printf("%08x %08x %08x %08x\n", x.x, x.y, x.z, x.w);
    }
    return 0;
}
