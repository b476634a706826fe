// Host-side reference outputs of rocRAND's Philox4x32-10 engine, used to pin the oracle's own
// Philox implementation against an independent library.  Reads lines "k0 k1 c0 c1 c2 c3"
// (decimal uint32) from stdin and prints the first block the engine returns for that key and
// counter.  rocRAND maps seed -> key (low word, high word), subsequence -> counter words 2-3
// and (word offset) / 4 -> counter words 0-1.
#include <rocrand/rocrand_philox4x32_10.h>
#include <cstdio>
int main() {
    unsigned k0, k1, c0, c1, c2, c3;
    while (std::scanf("%u %u %u %u %u %u", &k0, &k1, &c0, &c1, &c2, &c3) == 6) {
        unsigned long long seed = ((unsigned long long)k1 << 32) | k0;
        unsigned long long subseq = ((unsigned long long)c3 << 32) | c2;
        unsigned long long blocks = ((unsigned long long)c1 << 32) | c0;
        rocrand_device::philox4x32_10_engine e(seed, subseq, 0ULL);
        // skip `blocks` blocks of 4 words without overflowing the 64-bit word offset
        unsigned long long q = blocks / 4ULL, rem = blocks % 4ULL;
        for (int i = 0; i < 4; ++i) e.discard(4ULL * q);
        e.discard(4ULL * rem);
        uint4 r = e.next4();
        std::printf("%u %u %u %u\n", r.x, r.y, r.z, r.w);
    }
    return 0;
}
