// Device helpers shared by the tiled kernels and the resident solver.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.hpp"

namespace hms {

// tanh(x) carrying the rounding in its sign bit: set iff x does not round to
// true (x <= 0, -0.0 or NaN).
static __device__ __forceinline__ float signed_tanh(float x) {
    uint32_t b = __float_as_uint(tanhf(x)) & kIdx;
    if (!(x > 0.0f)) b |= kSign;
    return __uint_as_float(b);
}

// sech^2(x) = 4 e / (1 + e)^2 with e = exp(-2|x|): no cancellation for large |x|.
static __device__ __forceinline__ float sech2f(float x) {
    float e = expf(-2.0f * fabsf(x));
    float d = 1.0f + e;
    return (4.0f * e) / (d * d);
}

// SplitMix64 (Steele, Lea, Flood 2014): output k of the stream seeded `seed`.
static __device__ __forceinline__ uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Loads of plan data (read-only for the whole solve) through the constant
// address space: a wave-uniform address becomes a scalar load.
static __device__ __forceinline__ uint32_t ldc(const uint32_t* p) {
    return *(const __attribute__((address_space(4))) uint32_t*)p;
}
static __device__ __forceinline__ TileDesc ldtile(const TileDesc* p) {
    const uint32_t* w = reinterpret_cast<const uint32_t*>(p);
    return TileDesc{ldc(w), ldc(w + 1), ldc(w + 2), ldc(w + 3)};
}

// Gradient of one (variable, restart): g = sech^2(x) * G, rounded once from FP64.
static __device__ __forceinline__ float grad_of(float x, double G) { return (float)((double)sech2f(x) * G); }

// Scalars of Adam step number tt (1-based, PyTorch semantics): lr / (1 - b1^tt)
// and 1 / sqrt(1 - b2^tt), computed in FP64 and rounded once.
static __device__ __forceinline__ void adam_scalars(double tt, double lr, double b1, double b2, float& ss,
                                                    float& ib2) {
    const double bc1 = 1.0 - pow(b1, tt);
    const double bc2 = 1.0 - pow(b2, tt);
    ss = (float)(lr / bc1);
    ib2 = (float)(1.0 / sqrt(bc2));
}

struct AdamCoef {
    float b1, b2, eps, omb1, omb2;
};

// One Adam update of (x, m, v) with gradient g in FP32 (no contraction).
static __device__ __forceinline__ void adam_update(float& x, float& m, float& v, float g, float ss, float ib2,
                                                   const AdamCoef& k) {
    m = k.b1 * m + k.omb1 * g;
    v = k.b2 * v + k.omb2 * (g * g);
    const float denom = sqrtf(v) * ib2 + k.eps;
    x = x - (ss * m) / denom;
}

}  // namespace hms
