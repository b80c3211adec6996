// Rounding of fp32 quantiser products to integers, shared by the kernels and
// by the host check that exports it.
#pragma once

#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

namespace adct {

// Round half away from zero of an fp32 value, as an integer: add the largest
// float below 1/2 (0x1.fffffep-2) with x's sign, in one round-to-nearest-even
// fp32 addition, then convert, which truncates.  If x has a fraction of at
// least 1/2 the sum reaches the next integer away from zero (a fraction of
// exactly 1/2 gives a tie between the integer and the float just below it,
// broken towards the integer); otherwise it stays below it.  Integers that
// need all 24 mantissa bits stay put, the addend being less than half their
// spacing.  So this equals (int32_t)roundf(x) for every x whose rounded value
// fits an int32, in three instructions instead of seven.
__host__ __device__ __forceinline__ int32_t round_away(float x) {
    // The addition is its own rounding step: it must not absorb a multiply
    // that produced x (a fused multiply-add would skip the rounding of the
    // fp32 product that the quantiser definition applies first).
#pragma clang fp contract(off)
    const float h = copysignf(0x1.fffffep-2f, x);
#ifdef __HIP_DEVICE_COMPILE__
    return (int32_t)(x + h);
#else
    volatile float s = x + h;  // one fp32 addition, not fused or widened
    return (int32_t)s;
#endif
}

// round_away(y) given h = copysign(0x1.fffffep-2f, x) for an x of y's sign,
// or any x when y is zero: a dequantised level y = level * dqs has the sign
// of the quantised value x it came from, so the quantiser's addend serves
// both roundings.
__device__ __forceinline__ int32_t round_away_h(float y, float h) {
#pragma clang fp contract(off)
    return (int32_t)(y + h);
}

}  // namespace adct
