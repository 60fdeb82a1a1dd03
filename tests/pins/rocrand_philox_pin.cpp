// Independent Philox4x32-10 reference for the oracle's generator: rocRAND's
// open-source philox4x32_10 engine, run on the host. Reads lines
// "seed c0 c1 c2 c3" and prints the four output words of the block at that
// counter. rocRAND addresses a block by (subsequence, offset): the counter is
// (offset/4 low, offset/4 high, subsequence low, subsequence high).
#include <rocrand/rocrand_philox4x32_10.h>
#include <cinttypes>
#include <cstdio>

int main()
{
    unsigned long long seed;
    unsigned c0, c1, c2, c3;
    while (std::scanf("%llu %u %u %u %u", &seed, &c0, &c1, &c2, &c3) == 5) {
        unsigned long long subsequence = (unsigned long long)c2 | ((unsigned long long)c3 << 32);
        unsigned long long block = (unsigned long long)c0 | ((unsigned long long)c1 << 32);
        rocrand_device::philox4x32_10_engine eng(seed, subsequence, 0ull);
        // discard() counts single words; advance in pieces so 4 * block cannot overflow
        while (block != 0) {
            unsigned long long step = block < (1ull << 60) ? block : (1ull << 60);
            eng.discard(step * 4ull);
            block -= step;
        }
        unsigned a = eng.next(), b = eng.next(), c = eng.next(), d = eng.next();
        std::printf("%u %u %u %u\n", a, b, c, d);
    }
    return 0;
}
