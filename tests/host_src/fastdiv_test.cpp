// Host check of the invariant-divisor division used by the copy kernels.
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2208_13707_amd/csrc/mpixs_dev.h"

int main() {
    using namespace mpixs;
    std::mt19937_64 g(12345);
    uint64_t checked = 0;
    auto check = [&](uint32_t n, uint32_t d, const FastDiv &f) {
        ++checked;
        if (fd_div(n, f) != n / d) {
            std::printf("FAIL n=%u d=%u got=%u want=%u\n", n, d, fd_div(n, f), n / d);
            return false;
        }
        return true;
    };
    std::vector<uint32_t> ds = {1, 2, 3, 5, 7, 12, 24, 96, 1000, 65535, 65536, 65537,
                                131070, 2147483647u, 2147483648u, 4294967295u};
    for (int i = 0; i < 2000; ++i) ds.push_back(uint32_t(g() % 4294967295u) + 1);
    for (int i = 0; i < 2000; ++i) ds.push_back(uint32_t(g() % 100000) + 1);
    for (uint32_t d : ds) {
        const FastDiv f = make_fastdiv(d);
        const uint32_t edge[] = {0, 1, d - 1, d, d + 1, 2 * d - 1, 2 * d, 4294967295u,
                                 4294967294u, 2147483648u, uint32_t(uint64_t(4294967295u) / d * d),
                                 uint32_t(uint64_t(4294967295u) / d * d - 1)};
        for (uint32_t n : edge)
            if (!check(n, d, f)) return 1;
        for (int k = 0; k < 2000; ++k)
            if (!check(uint32_t(g()), d, f)) return 1;
    }
    // every n for a few small divisors
    for (uint32_t d : {3u, 7u, 12u}) {
        const FastDiv f = make_fastdiv(d);
        for (uint64_t n = 0; n < (uint64_t(1) << 32); n += 9973)
            if (!check(uint32_t(n), d, f)) return 1;
    }
    std::printf("ok %llu\n", (unsigned long long)checked);
    return 0;
}
