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

// 1 / |r| from r2 = |r|^2: the hardware reciprocal square root (without
// the rescaling rsqrtf applies to subnormal inputs; a positive r2 below the
// smallest normal float is taken as that float) and 0 for r2 == 0, the
// coincident point, which the Green's function sums leave out
__device__ __forceinline__ float rsq_or_zero(float r2)
{
    const float y = __builtin_amdgcn_rsqf(fmaxf(r2, 1.17549435e-38f));
    return r2 > 0.f ? y : 0.f;
}
// sin and cos of 2 pi t (t in turns) on the hardware sine / cosine units
__device__ __forceinline__ void sincos_turns(float t, float *s, float *c)
{
    *s = __builtin_amdgcn_sinf(t);
    *c = __builtin_amdgcn_cosf(t);
}

}  // namespace dev
}  // namespace mlfma
