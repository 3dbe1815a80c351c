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

// The same functions of u = z log2(e) (arguments already scaled for exp2).
__device__ __forceinline__ float sigm2(float u) { return frcp(1.f + __builtin_amdgcn_exp2f(-u)); }

// expm1(u ln 2): Taylor polynomial in u through (u ln 2)^8 / 8! for
// |u ln 2| < 1/2, exp2(u) - 1 elsewhere (as expm1 above).
__device__ __forceinline__ float expm1_2(float u)
{
    // coefficients (ln 2)^k / k!, k = 8 .. 1
    float q = fmaf(u, 1.32154868e-06f, 1.52527338e-05f);
    q = fmaf(u, q, 1.54035304e-04f);
    q = fmaf(u, q, 1.33335581e-03f);
    q = fmaf(u, q, 9.61812911e-03f);
    q = fmaf(u, q, 5.55041087e-02f);
    q = fmaf(u, q, 2.40226507e-01f);
    q = fmaf(u, q, 6.93147181e-01f);
    const float big = __builtin_amdgcn_exp2f(u) - 1.f;
    return fabsf(u) < 0.72134752f ? u * q : big;
}

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
