// Complex FP32 helpers shared by the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace mlfma {
namespace dev {

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cfma(float2 a, float2 b, float2 c)
{
    c.x = fmaf(a.x, b.x, c.x);
    c.x = fmaf(-a.y, b.y, c.x);
    c.y = fmaf(a.x, b.y, c.y);
    c.y = fmaf(a.y, b.x, c.y);
    return c;
}
// conj(a) * b + c
__device__ __forceinline__ float2 cfma_conj(float2 a, float2 b, float2 c)
{
    c.x = fmaf(a.x, b.x, c.x);
    c.x = fmaf(a.y, b.y, c.x);
    c.y = fmaf(a.x, b.y, c.y);
    c.y = fmaf(-a.y, b.x, c.y);
    return c;
}

}  // namespace dev
}  // namespace mlfma
