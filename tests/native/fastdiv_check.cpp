// Host check of the library's division by a multiply and a shift (FastDiv in
// csrc/common.h) against integer division: every divisor up to 5000, powers
// of two and their neighbours, and random divisors up to 2^31 - 1, each at
// the numerators where an error would show first (around multiples of the
// divisor and at the top of the range) and at random ones.
#include <cstdio>
#include <cstdint>
#include <random>
#include <vector>

#include "common.h"

int main() {
    std::vector<uint32_t> divs;
    for (uint32_t d = 1; d <= 5000; ++d) divs.push_back(d);
    for (int k = 1; k < 31; ++k) {
        divs.push_back(1u << k);
        divs.push_back((1u << k) - 1);
        divs.push_back((1u << k) + 1);
    }
    divs.push_back(0x7fffffffu);
    std::mt19937 rng(12345);
    std::uniform_int_distribution<uint32_t> any(1, 0x7fffffffu);
    for (int k = 0; k < 20000; ++k) divs.push_back(any(rng));
    long long checks = 0;
    for (uint32_t d : divs) {
        const hub::FastDiv f = hub::make_fastdiv(d);
        std::vector<int64_t> ns = {0, 1, (int64_t)d - 1, d, (int64_t)d + 1, 0x7fffffff,
                                   0x7ffffffe};
        const int64_t top = 0x7fffffffLL / d * d;
        ns.push_back(top);
        ns.push_back(top - 1);
        if (top >= (int64_t)d) ns.push_back(top - d);
        for (int k = 0; k < 40; ++k) ns.push_back(any(rng) - 1);
        for (int64_t n : ns) {
            if (n < 0 || n > 0x7fffffff) continue;
            const int got = hub::fdiv((int)n, f);
            if (got != (int)(n / d)) {
                std::printf("FAIL d=%u n=%lld got %d want %lld\n", d, (long long)n, got,
                            (long long)(n / d));
                return 1;
            }
            ++checks;
        }
    }
    std::printf("ok %lld checks\n", checks);
    return 0;
}
