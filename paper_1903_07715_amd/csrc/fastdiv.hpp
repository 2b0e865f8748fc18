// fastdiv.hpp -- multiply-shift replacement of 32-bit unsigned division by a runtime constant.
//
// For a divisor d >= 2 let s = ceil(log2 d) - 1 and mul = ceil(2^(32+s) / d) (< 2^32).  Then for
// every 0 <= x < 2^31, floor(x / d) = floor(x * mul / 2^(32+s)): writing mul = 2^(32+s)/d + e/d
// with 0 <= e < d <= 2^(s+1), the excess x e / (d 2^(32+s)) is below 1/d, which cannot carry
// the quotient past the next integer.
#pragma once

#include <stdint.h>

namespace hjr {

struct FastDivParams {
    uint32_t mul;
    uint32_t shift;
};

inline FastDivParams fastdiv_params(uint32_t d)
{
    uint32_t c = 0;  // ceil(log2 d)
    while ((1ull << c) < d) ++c;
    const uint32_t s = c - 1;
    const uint64_t num = 1ull << (32 + s);
    FastDivParams p;
    p.mul = (uint32_t)((num + d - 1) / d);
    p.shift = s;
    return p;
}

inline uint32_t fastdiv_host(uint32_t x, FastDivParams p)
{
    return (uint32_t)(((uint64_t)x * p.mul) >> 32) >> p.shift;
}

}  // namespace hjr
