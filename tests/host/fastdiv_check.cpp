// Host check of kbc::fdiv (the node-index division used by every kernel):
// exhaustive over small divisors and sampled over large node counts.
#include <cstdio>
#include <cstdint>
#include <random>

#include "kbc_device.h"

int main()
{
    std::mt19937_64 rng(12345);
    long bad = 0;
    for (uint32_t d = 1; d <= 2048; ++d) {
        const kbc::FastDiv f = kbc::make_fastdiv(d);
        for (uint32_t n = 0; n < 70000; ++n)
            if (kbc::fdiv(n, f) != n / d) ++bad;
        for (int k = 0; k < 20000; ++k) {
            const uint32_t n = (uint32_t)(rng() % 2147483648ull);
            if (kbc::fdiv(n, f) != n / d) ++bad;
        }
        const uint32_t edge[] = {2147483647u, 2147483646u, d * 1000u - 1u};
        for (uint32_t n : edge)
            if (n < 2147483648u && kbc::fdiv(n, f) != n / d) ++bad;
    }
    const uint32_t big[] = {65536u, 262144u, 1048576u, 16777216u, 1u << 30, 2147483647u};
    for (uint32_t d : big) {
        const kbc::FastDiv f = kbc::make_fastdiv(d);
        for (int k = 0; k < 200000; ++k) {
            const uint32_t n = (uint32_t)(rng() % 2147483648ull);
            if (kbc::fdiv(n, f) != n / d) ++bad;
        }
    }
    std::printf("mismatches %ld\n", bad);
    return bad == 0 ? 0 : 1;
}
