// GELU of the time-conditioned U-Net's blocks (Materials and Methods, "U-Net
// with temporal conditioning"), shared by the normalisation kernels and the
// convolution that applies a normalisation as it loads its input, so that
// both evaluate it with the same instructions.
#pragma once
#include <hip/hip_runtime.h>

namespace pfu {

// GELU, tanh form: 0.5 a (1 + tanh(sqrt(2/pi) (a + 0.044715 a^3)))
constexpr float kGeluS = 0.7978845608028654f;
constexpr float kGeluA = 0.044715f;
// (1 + tanh u) / 2 = 1 / (1 + exp(-2u)): the logistic form, on the hardware
// base-2 exponential and reciprocal (exp2 of +-inf gives 0 or inf, so both
// tails saturate to 0 and 1)
__device__ __forceinline__ float gelu_s(float a)
{
    const float u = kGeluS * fmaf(kGeluA * a, a * a, a);
    return __builtin_amdgcn_rcpf(1.f + __builtin_amdgcn_exp2f(-2.f * 1.4426950408889634f * u));
}
__device__ __forceinline__ float gelu(float a) { return a * gelu_s(a); }
__device__ __forceinline__ float gelu_grad(float a)
{
    const float s = gelu_s(a);
    return s + 2.f * a * s * (1.f - s) * kGeluS * fmaf(3.f * kGeluA * a, a, 1.f);
}

}  // namespace pfu
