// records.h -- layouts of the predicted j-particle records in device memory.
//
// The predictor writes one record per particle; the force kernels read the
// j-particles of a loop step with wave-uniform addresses (scalar loads into
// SGPRs, used directly as VALU operands) and the active i-particles with
// per-lane vector loads.  Sizes are multiples of 16 bytes.
#pragma once

#include <stdint.h>

namespace nb {

// FP64 mode: positions, mass, velocities, and for order >= 6 accelerations,
// order 8 jerks, all double.
template <int P> struct RecF64;
template <> struct alignas(16) RecF64<4> { double x, y, z, m, vx, vy, vz, pad; };                       // 64 B
template <> struct alignas(16) RecF64<6> { double x, y, z, m, vx, vy, vz, ax, ay, az; };                // 80 B
template <> struct alignas(16) RecF64<8> { double x, y, z, m, vx, vy, vz, ax, ay, az, jx, jy, jz, pad; }; // 112 B

// MIXED and DS modes: double-single positions and velocities
// (hi = float(x), lo = float(x - hi)), FP32 mass, acceleration and jerk.
template <int P> struct RecDS;
template <> struct alignas(16) RecDS<4> {
    float xh, yh, zh, m, xl, yl, zl, vxh, vyh, vzh, vxl, vyl, vzl, p0, p1, p2;                             // 64 B
};
template <> struct alignas(16) RecDS<6> {
    float xh, yh, zh, m, xl, yl, zl, vxh, vyh, vzh, vxl, vyl, vzl, ax, ay, az;                             // 64 B
};
template <> struct alignas(16) RecDS<8> {
    float xh, yh, zh, m, xl, yl, zl, vxh, vyh, vzh, vxl, vyl, vzl, ax, ay, az, jx, jy, jz, p0;             // 80 B
};

static_assert(sizeof(RecF64<4>) == 64 && sizeof(RecF64<6>) == 80 && sizeof(RecF64<8>) == 112, "f64 rec");
static_assert(sizeof(RecDS<4>) == 64 && sizeof(RecDS<6>) == 64 && sizeof(RecDS<8>) == 80, "ds rec");

// Reciprocal square root in FP64: the hardware estimate (about 24 correct
// bits on gfx950) refined by one third-order Householder step,
// y <- y (1 + h/2 + 3h^2/8) with h = 1 - x y^2, which leaves an error far
// below one unit in the last place before the final rounding.
__device__ __forceinline__ double rsqrt64(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    const double h = __builtin_fma(-x, y * y, 1.0);
    return __builtin_fma(y * h, __builtin_fma(h, 0.375, 0.5), y);
}

}  // namespace nb
