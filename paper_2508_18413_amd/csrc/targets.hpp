// Device-side targets for per-lane evaluation (one lane holds a whole state
// vector in registers).  Each target gives the gradient, the Hessian diagonal,
// Hessian entries, Hessian-vector products, and log p(x~) - log p(x) written
// in terms of the exact increment delta = x~ - x so that FP32 does not lose
// the difference of two large log-densities.  Padded coordinates (d >= D) hold
// zeros and must produce zero gradient entries.
#pragma once

#include <hip/hip_runtime.h>

namespace pmc {

template <typename R>
__device__ __forceinline__ R dexp(R x) { return exp(x); }
template <>
__device__ __forceinline__ float dexp<float>(float x) { return expf(x); }

// log p(x) = -x1^2/2 - (x2 - x1^2)^2/2
template <typename R>
struct Banana {
    static constexpr int DM = 2;
    int D;
    __device__ void grad(const R *x, R *g) const
    {
        const R a = x[1] - x[0] * x[0];
        g[0] = -x[0] + R(2) * x[0] * a;
        g[1] = -a;
    }
    __device__ R hess(const R *x, int i, int j) const
    {
        if (i == 0 && j == 0) return R(-1) + R(2) * (x[1] - x[0] * x[0]) - R(4) * x[0] * x[0];
        if (i == 1 && j == 1) return R(-1);
        return R(2) * x[0];
    }
    __device__ void hess_diag(const R *x, R *h) const
    {
        h[0] = hess(x, 0, 0);
        h[1] = R(-1);
    }
    __device__ void dgrad_dtheta(const R *, R *o) const { o[0] = o[1] = R(0); }
    __device__ void hvp(const R *x, const R *v, R *o) const
    {
        const R h00 = hess(x, 0, 0), h01 = R(2) * x[0];
        o[0] = h00 * v[0] + h01 * v[1];
        o[1] = h01 * v[0] - v[1];
    }
    // log p(xt) - log p(x) with dl = xt - x exact
    __device__ R logp_diff(const R *x, const R *xt, const R *dl, const R *, const R *) const
    {
        const R dq1 = dl[0] * (xt[0] + x[0]);  // xt1^2 - x1^2
        const R a = x[1] - x[0] * x[0];
        const R at = xt[1] - xt[0] * xt[0];
        const R da = dl[1] - dq1;              // at - a
        return -R(0.5) * dq1 - R(0.5) * da * (at + a);
    }
};

// log p(x) = -(x - mu)^T P (x - mu) / 2, P symmetric [D, D] in global memory
template <typename R, int DMax>
struct Gaussian {
    static constexpr int DM = DMax;
    // Widest per-lane instance: beyond D = 16 the evaluation kernels' private
    // arrays exceed 1 KiB per lane, the HIP runtime's default per-thread stack,
    // which the library keeps every kernel within.
    static constexpr int kMaxLaneDim = 16;
    int D;
    const R *mean, *prec;
    __device__ void grad(const R *x, R *g) const
    {
        R c[DM];
#pragma unroll
        for (int j = 0; j < DM; j++) c[j] = j < D ? x[j] - mean[j] : R(0);
#pragma unroll
        for (int i = 0; i < DM; i++) {
            R s = R(0);
            if (i < D) {
#pragma unroll
                for (int j = 0; j < DM; j++)
                    if (j < D) s = fma(prec[i * D + j], c[j], s);
            }
            g[i] = -s;
        }
    }
    __device__ R hess(const R *, int i, int j) const { return -prec[i * D + j]; }
    __device__ void dgrad_dtheta(const R *, R *o) const
    {
#pragma unroll
        for (int i = 0; i < DM; i++) o[i] = R(0);
    }
    __device__ void hess_diag(const R *, R *h) const
    {
#pragma unroll
        for (int i = 0; i < DM; i++) h[i] = i < D ? -prec[i * D + i] : R(0);
    }
    __device__ void hvp(const R *, const R *v, R *o) const
    {
#pragma unroll
        for (int i = 0; i < DM; i++) {
            R s = R(0);
            if (i < D) {
#pragma unroll
                for (int j = 0; j < DM; j++)
                    if (j < D) s = fma(prec[i * D + j], v[j], s);
            }
            o[i] = -s;
        }
    }
    // quadratic: log p(xt) - log p(x) = dl . (g + gt) / 2 exactly
    __device__ R logp_diff(const R *, const R *, const R *dl, const R *g, const R *gt) const
    {
        R s = R(0);
#pragma unroll
        for (int i = 0; i < DM; i++) s = fma(dl[i], g[i] + gt[i], s);
        return R(0.5) * s;
    }
};

// Funnel: x1 ~ N(0, e^{2 theta}), x_d | x1 ~ N(0, e^{x1}), d = 2..D
template <typename R, int DMax>
struct Funnel {
    static constexpr int DM = DMax;
    static constexpr int kMaxLaneDim = 32;
    int D;
    R theta;
    __device__ R tail_sq(const R *x) const
    {
        R q = R(0);
#pragma unroll
        for (int d = 1; d < DM; d++) q = fma(x[d], x[d], q);
        return q;
    }
    __device__ void grad(const R *x, R *g) const
    {
        const R e = dexp<R>(-x[0]), q = tail_sq(x);
        g[0] = -x[0] * dexp<R>(R(-2) * theta) + R(0.5) * e * q - R(0.5) * R(D - 1);
#pragma unroll
        for (int d = 1; d < DM; d++) g[d] = -e * x[d];
    }
    __device__ R hess(const R *x, int i, int j) const
    {
        const R e = dexp<R>(-x[0]);
        if (i == 0 && j == 0) return -dexp<R>(R(-2) * theta) - R(0.5) * e * tail_sq(x);
        if (i == 0) return e * x[j];
        if (j == 0) return e * x[i];
        return i == j ? -e : R(0);
    }
    // d/dtheta of grad log p: only the first coordinate depends on theta
    __device__ void dgrad_dtheta(const R *x, R *o) const
    {
        o[0] = R(2) * x[0] * dexp<R>(R(-2) * theta);
#pragma unroll
        for (int d = 1; d < DM; d++) o[d] = R(0);
    }
    __device__ void hess_diag(const R *x, R *h) const
    {
        const R e = dexp<R>(-x[0]);
        h[0] = -dexp<R>(R(-2) * theta) - R(0.5) * e * tail_sq(x);
#pragma unroll
        for (int d = 1; d < DM; d++) h[d] = d < D ? -e : R(0);
    }
    __device__ void hvp(const R *x, const R *v, R *o) const
    {
        const R e = dexp<R>(-x[0]);
        R s = (-dexp<R>(R(-2) * theta) - R(0.5) * e * tail_sq(x)) * v[0];
#pragma unroll
        for (int d = 1; d < DM; d++) {
            s = fma(e * x[d], v[d], s);
            o[d] = e * (x[d] * v[0] - v[d]);
        }
        o[0] = s;
    }
    // log p(xt) - log p(x) = -e^{-2 theta}(xt1^2 - x1^2)/2
    //   - e^{-x1} [expm1(-dl1) Qt + (Qt - Q)] / 2 - (D-1) dl1 / 2
    __device__ R logp_diff(const R *x, const R *xt, const R *dl, const R *, const R *) const
    {
        R qt = R(0), dq = R(0);
#pragma unroll
        for (int d = 1; d < DM; d++) {
            qt = fma(xt[d], xt[d], qt);
            dq = fma(dl[d], xt[d] + x[d], dq);
        }
        const R dq1 = dl[0] * (xt[0] + x[0]);
        return -R(0.5) * dexp<R>(R(-2) * theta) * dq1 -
               R(0.5) * dexp<R>(-x[0]) * (expm1(-dl[0]) * qt + dq) - R(0.5) * R(D - 1) * dl[0];
    }
};

}  // namespace pmc
