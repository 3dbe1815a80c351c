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
//   log1p(w): log(a) + (w - (a - 1)) / a with a = fl(1 + w): the hardware
//     log2 is accurate to about one ulp relative to its result even next to
//     1, and the second term restores what rounding 1 + w dropped (a - 1 is
//     exact), so small w keep their relative accuracy.
constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

__device__ __forceinline__ float fexp(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ float flog(float x) { return __builtin_amdgcn_logf(x) * kLn2; }

__device__ __forceinline__ float sigm(float z) { return frcp(1.f + fexp(-z)); }

// The same function of u = z log2(e) (argument already scaled for exp2).
__device__ __forceinline__ float sigm2(float u) { return frcp(1.f + __builtin_amdgcn_exp2f(-u)); }

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

// log1p(w) given a = fl(1 + w) and ra = 1 / a
__device__ __forceinline__ float log1p_ar(float w, float a, float ra) { return fmaf(w - (a - 1.f), ra, flog(a)); }

__device__ __forceinline__ float log1p_s(float w)
{
    const float a = 1.f + w;
    return log1p_ar(w, a, frcp(a));
}

__device__ __forceinline__ float softplus(float x) { return fmaxf(x, 0.f) + log1p_s(fexp(-fabsf(x))); }

}  // namespace pmc
