// Short-latency logistic functions for FP32 device code (logistic-regression
// evaluation and the sequential sampler).
#pragma once

#include <hip/hip_runtime.h>

namespace pmc {

// Short-latency forms built on the hardware exp2 / log2 / reciprocal (each
// accurate to about one ulp).  Relative errors stay within a few FP32 ulps:
//   sigmoid(z) = 1 / (1 + 2^(-z log2 e)); overflow of the exponential gives 0.
//   expm1(x): x q(x), q the Taylor polynomial through x^7 / 8!, for |x| < 1/2
//     (the first omitted term is below 2^-26 relative); exp(x) - 1 elsewhere,
//     where |expm1(x)| > 0.39 bounds the cancellation.
//   log1p(w): 2 atanh(r) with r = w / (2 + w), series through r^7 / 7, for
//     |w| < 1/4 (|r| < 1/7, omitted terms below 2^-25 relative); log(1 + w)
//     elsewhere, where |log1p(w)| > 0.22 bounds the effect of rounding 1 + w.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * kLn2; }

__device__ __forceinline__ float sigm(float z) { return frcp(1.f + fexp(-z)); }

__device__ __forceinline__ float expm1_s(float x)
{
    float q = fmaf(x, 1.f / 40320.f, 1.f / 5040.f);
    q = fmaf(x, q, 1.f / 720.f);
    q = fmaf(x, q, 1.f / 120.f);
    q = fmaf(x, q, 1.f / 24.f);
    q = fmaf(x, q, 1.f / 6.f);
    q = fmaf(x, q, 0.5f);
    q = fmaf(x, q, 1.f);
    const float big = fexp(x) - 1.f;
    return fabsf(x) < 0.5f ? x * q : big;
}

__device__ __forceinline__ float log1p_s(float w)
{
    const float r = w * frcp(2.f + w);
    const float r2 = r * r;
    float p = fmaf(r2, 1.f / 7.f, 1.f / 5.f);
    p = fmaf(r2, p, 1.f / 3.f);
    p = fmaf(r2, p, 1.f);
    const float big = flog(1.f + w);
    return fabsf(w) < 0.25f ? 2.f * r * p : big;
}

__device__ __forceinline__ float softplus(float x) { return fmaxf(x, 0.f) + log1p_s(fexp(-fabsf(x))); }

}  // namespace pmc
