// Fixed-point terms of the per-frame voxel sums of fusion (Eq. (1)-(3)).
//
// A term w x enters as (w 2^f) x: scaling by a power of two is exact, so
// this is (w x) 2^f rounded once.  The 64-bit integer is formed from two
// 32-bit conversions, hi = floor(w x 2^(f-32)) and lo = w x 2^f - hi 2^32
// (one instruction each, where a direct 64-bit conversion is a long
// sequence).  For w x >= 0, and for w x <= -2^(32-f) (whose float32 value
// is a multiple of 2^9 units), the remainder lo is exact and lies in
// [0, 2^32).  A negative term smaller than that in magnitude leaves a
// remainder 2^32 - |w x 2^f| that can need more than 24 bits; lo is then
// rounded to the nearest float, at most 2^7 units away, and may round up to
// exactly 2^32, where the conversion saturates to 2^32 - 1 (one unit below
// the carry it stands for, again within 2^7).  So a term is exact unless it
// is below 2^(23-f) or a negative one below 2^(32-f) in magnitude, which is
// rounded, deterministically, within 2^(7-f).  Integer sums are exact and
// the total is rounded once, to float.  ws = w 2^f, wh = w 2^(f-32).
//
// Everything here is plain arithmetic on host and device, so a host unit
// test exercises the same functions the fusion kernel calls.
#pragma once

#include <cmath>
#include <cstdint>

namespace gsdf {

// float in [0, 2^32] (never negative or NaN here) to uint32, saturating at
// 2^32 - 1.  On the device this is one v_cvt_u32_f32, which clamps to the
// unsigned range by definition of the instruction (a C++ cast of 2^32
// would be undefined); the host form states the same clamp explicitly.
__host__ __device__ inline uint32_t sat_u32(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
    uint32_t r;
    asm("v_cvt_u32_f32 %0, %1" : "=v"(r) : "v"(x));
    return r;
#else
    return x >= 4294967296.0f ? 0xffffffffu : (uint32_t)x;
#endif
}

__host__ __device__ inline unsigned long long fixed_term(float ws, float wh, float x) {
    const float s = ws * x;
    const float hs = floorf(wh * x);
    const float lo = fmaf(-hs, 4294967296.0f, s);
    return ((unsigned long long)(uint32_t)(int32_t)hs << 32) | (unsigned long long)sat_u32(lo);
}

__host__ __device__ inline float from_fixed(unsigned long long a, double inv) {
    return (float)((double)(long long)a * inv);
}

}  // namespace gsdf
