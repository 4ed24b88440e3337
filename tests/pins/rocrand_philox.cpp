// Library pin for the oracle's Philox4x32-10: evaluates rocRAND's own
// Philox4x32-10 engine (host side of rocrand_philox4x32_10.h) on the
// counter/key pairs read from stdin, one "c0 c1 c2 c3 k0 k1" (hex) per line,
// and prints the four output words in hex.
//
// rocRAND's engine(seed, subsequence, offset) starts at key = (seed_lo,
// seed_hi) and counter = (offset/4 as the low 64 bits, subsequence as the high
// 64 bits); its first four outputs are one Philox block of that counter.
#include <cstdio>
#include <rocrand/rocrand_philox4x32_10.h>

int main()
{
    unsigned c0, c1, c2, c3, k0, k1;
    while (std::scanf("%x %x %x %x %x %x", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
        unsigned long long seed = (unsigned long long)k0 | ((unsigned long long)k1 << 32);
        unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long block = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0ull);
        // advance the low 64 counter bits by `block` (discard counts words,
        // four per block, so step in chunks that cannot overflow)
        while (block > 0) {
            unsigned long long chunk = block < (1ull << 61) ? block : (1ull << 61);
            eng.discard(chunk * 4ull);
            block -= chunk;
        }
        unsigned w[4];
        for (int i = 0; i < 4; ++i) w[i] = eng();
        std::printf("%08x %08x %08x %08x\n", w[0], w[1], w[2], w[3]);
    }
    return 0;
}
