// Morton (Z-order) codes of three coordinates, shared by the orderings of
// query rows (the reduced-precision screens' query order and the routed
// form's tiles).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace rsc {

// float bits mapped to unsigned integers of the same order
__device__ __forceinline__ uint32_t ordered_bits(float x) {
    const uint32_t b = __float_as_uint(x);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float from_ordered(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

// 10 bits spread to every third bit position
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

// Coordinate x quantised to 10 bits over [lo, lo + span] (0 when the span is
// empty or not finite; NaN maps to 0).
__device__ __forceinline__ uint32_t quantise10(float x, float lo, float scale) {
    float q = (x - lo) * scale;
    q = fminf(fmaxf(q, 0.f), 1023.f);
    return (uint32_t)q;
}
__device__ __forceinline__ float scale10(float lo, float hi) {
    const float span = hi - lo;
    return span > 0.f && isfinite(span) ? 1023.f / span : 0.f;
}

}  // namespace rsc
