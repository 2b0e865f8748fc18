// Exhaustive-boundary check of the multiply-shift division used for node index decomposition.
#include "../../paper_1903_07715_amd/csrc/fastdiv.hpp"

#include <cstdio>
#include <random>

int main()
{
    std::mt19937_64 rng(20190318);
    long bad = 0;
    for (uint32_t d = 2; d <= 70000; d = d < 5000 ? d + 1 : d + 97) {
        hjr::FastDivParams p = hjr::fastdiv_params(d);
        const uint32_t xmax = 0x7fffffffu;
        // every quotient boundary near 0 and near 2^31, plus random values
        for (uint32_t k = 0; k < 64; ++k) {
            uint64_t lo = (uint64_t)k * d, hi = (uint64_t)(xmax / d - k) * d;
            for (int64_t o = -1; o <= 1; ++o) {
                for (uint64_t base : {lo, hi}) {
                    int64_t x = (int64_t)base + o;
                    if (x < 0 || x > (int64_t)xmax) continue;
                    if (hjr::fastdiv_host((uint32_t)x, p) != (uint32_t)x / d) ++bad;
                }
            }
        }
        for (int r = 0; r < 2000; ++r) {
            uint32_t x = (uint32_t)(rng() & xmax);
            if (hjr::fastdiv_host(x, p) != x / d) ++bad;
        }
        if (hjr::fastdiv_host(xmax, p) != xmax / d) ++bad;
    }
    std::printf("fastdiv mismatches: %ld\n", bad);
    return bad ? 1 : 0;
}
