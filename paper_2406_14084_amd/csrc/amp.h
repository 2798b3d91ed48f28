// amp.h -- amplitude types and complex helpers for the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace qs {

// Interleaved complex amplitudes.  16 B (complex128) and 8 B (complex64)
// so that one lane moves one amplitude with one global or LDS access.
struct alignas(16) c128 { double x, y; };
struct alignas(8) c64 { float x, y; };

template <typename F> struct AmpOf;
template <> struct AmpOf<double> { using type = c128; };
template <> struct AmpOf<float> { using type = c64; };

__device__ __forceinline__ double qfma(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float qfma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// acc += (mr + i mi) * v, as four fused multiply-adds
template <typename F, typename V>
__device__ __forceinline__ void cmac(V &acc, F mr, F mi, const V &v)
{
    acc.x = qfma(mr, v.x, acc.x);
    acc.x = qfma(-mi, v.y, acc.x);
    acc.y = qfma(mr, v.y, acc.y);
    acc.y = qfma(mi, v.x, acc.y);
}

template <typename F, typename V>
__device__ __forceinline__ V cmul(F mr, F mi, const V &v)
{
    V r;
    r.x = mr * v.x;
    r.x = qfma(-mi, v.y, r.x);
    r.y = mr * v.y;
    r.y = qfma(mi, v.x, r.y);
    return r;
}

}  // namespace qs
