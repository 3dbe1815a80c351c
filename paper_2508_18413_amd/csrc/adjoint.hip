// Derivatives of a trajectory functional F(s_{1:T}) through a converged chain,
// by the adjoint (reverse) recursion over transposed step Jacobians:
//   lambda_T = dF/ds_T,  lambda_t = dF/ds_t + J_{t+1}^T lambda_{t+1},
//   dF/dp = sum_t lambda_t . df_t/dp,  p in {theta, eps},
// with the frozen-gate step derivatives (the accept decision a_t held fixed):
//   J_t = a_t (I + eps H(s_{t-1})) + (1 - a_t) I,
//   df_t/dtheta = a_t eps d(grad log p)/dtheta (s_{t-1}),
//   df_t/deps   = a_t (grad log p(s_{t-1}) + xi_t / sqrt(2 eps)).
// In reversed time tau = T - 1 - t the recursion is the forward affine
// recursion mu_tau = J_{T-tau}^T mu_{tau-1} + dF/ds_{T-1-tau}, solved by the
// FP32 matrix-core dense scan (one solve, so FP32 compositions, not BF16).
// H is symmetric, so J_t^T = J_t.  The two sums are accumulated in FP64 with a
// fixed reduction order.
#include <math.h>

#include <vector>

#include "pmc_internal.hpp"
#include "targets.hpp"

namespace pmc {
namespace {

struct AdjArgs {
    int64_t T;
    int D;
    float eps;
    const float *s0, *states, *noise, *dFds;
    const uint8_t *accept;
    float4 *Jrev;     // [T] F32 fragments, reversed time
    float *brev;      // [T, D] reversed dF/ds
    float *dth, *deps;// [T, D] step derivatives
};

template <class Tg>
__global__ void __launch_bounds__(256) k_adj_eval(AdjArgs a, Tg tg)
{
    constexpr int DM = Tg::DM;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= a.T) return;
    const int D = a.D;
    float x[DM], g[DM], dg[DM];
#pragma unroll
    for (int d = 0; d < DM; d++)
        x[d] = d < D ? (t == 0 ? a.s0[d] : a.states[(size_t)(t - 1) * D + d]) : 0.f;
    const int acc = a.accept[t] != 0;
    tg.grad(x, g);
    tg.dgrad_dtheta(x, dg);
    const float c = 1.f / sqrtf(2.f * a.eps);
#pragma unroll
    for (int d = 0; d < DM; d++) {
        if (d < D) {
            const float xi = a.noise[(size_t)t * D + d];
            a.dth[(size_t)t * D + d] = acc ? a.eps * dg[d] : 0.f;
            a.deps[(size_t)t * D + d] = acc ? g[d] + c * xi : 0.f;
            a.brev[(size_t)(a.T - 1 - t) * D + d] = a.dFds[(size_t)t * D + d];
        }
    }
    // J_t goes to reversed position T - t (t >= 1); position 0 holds zero
    const int64_t tau = t == 0 ? 0 : a.T - t;
    const float ea = (t == 0 || !acc) ? 0.f : a.eps;
    const bool zero = t == 0;
    float4 *o = a.Jrev + (size_t)tau * 256;
    for (int m4 = 0; m4 < 4; m4++)
        for (int hh = 0; hh < 2; hh++)
            for (int i = 0; i < 32; i++) {
                float v[4];
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const int k = 2 * (4 * m4 + q) + hh;
                    float e = 0.f;
                    if (!zero && i < D && k < D) e = (i == k ? 1.f : 0.f) + ea * tg.hess(x, i, k);
                    v[q] = e;
                }
                o[m4 * 64 + hh * 32 + i] = make_float4(v[0], v[1], v[2], v[3]);
            }
}

// Per-block FP64 partial sums of lambda_t . dth_t and lambda_t . deps_t,
// lambda_t = mu_{T-1-t}.
__global__ void __launch_bounds__(256)
k_adj_dot(const float *mu, const float *dth, const float *deps, int64_t T, int D, double *part)
{
    __shared__ double s0[256], s1[256];
    double a0 = 0, a1 = 0;
    for (int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x; k < T * D; k += (int64_t)gridDim.x * 256) {
        const int64_t t = k / D;
        const int d = (int)(k % D);
        const double l = mu[(size_t)(T - 1 - t) * D + d];
        a0 += l * dth[k];
        a1 += l * deps[k];
    }
    s0[threadIdx.x] = a0;
    s1[threadIdx.x] = a1;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            s0[threadIdx.x] += s0[threadIdx.x + h];
            s1[threadIdx.x] += s1[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s0[0];
        part[2 * blockIdx.x + 1] = s1[0];
    }
}

template <class Tg>
pmc_status adj_eval(pmc_context *ctx, const AdjArgs &a, const Tg &tg)
{
    hipLaunchKernelGGL((k_adj_eval<Tg>), dim3((unsigned)((a.T + 255) / 256)), dim3(256), 0, ctx->stream,
                       a, tg);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

}  // namespace
}  // namespace pmc

using namespace pmc;

extern "C" pmc_status pmc_adjoint(pmc_context *ctx, const pmc_problem *prob, const void *states,
                                  const uint8_t *accept, const void *dF_ds, double *dF_dtheta,
                                  double *dF_dstep)
{
    PMC_REQUIRE(ctx && prob && prob->target && dF_dtheta && dF_dstep, "pmc_adjoint: NULL argument");
    const DevTarget &t = prob->target->t;
    PMC_REQUIRE(prob->n_chains == 1, "pmc_adjoint: one chain per call");
    PMC_REQUIRE(prob->step_size > 0, "pmc_adjoint: step_size > 0");
    if (t.dtype != PMC_F32 || t.dim > 32 || t.kind == PMC_TARGET_LOGREG) {
        set_error("pmc_adjoint: built for F32 banana, Gaussian and funnel targets with D <= 32");
        return PMC_ERR_UNSUPPORTED;
    }
    const int64_t T = prob->n_steps;
    const int D = t.dim;
    *dF_dtheta = *dF_dstep = 0.0;
    if (T == 0) return PMC_OK;
    PMC_REQUIRE(is_device_ptr(states) && is_device_ptr(accept) && is_device_ptr(dF_ds) &&
                    is_device_ptr(prob->s0) && is_device_ptr(prob->noise),
                "pmc_adjoint: s0, noise, states, accept and dF_ds must be device pointers");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    const int nb = 512;
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align_up(off + b, 256);
        return o;
    };
    const size_t oJ = take((size_t)T * 4096), ob = take((size_t)T * D * 4), oth = take((size_t)T * D * 4),
                 oep = take((size_t)T * D * 4), omu = take((size_t)T * D * 4), opart = take(nb * 16),
                 ows = take(dense_mfma_ws_bytes(T));
    PMC_TRY(ensure_pool(ctx, off));
    char *ws = (char *)ctx->pool;
    AdjArgs a;
    a.T = T;
    a.D = D;
    a.eps = (float)prob->step_size;
    a.s0 = (const float *)prob->s0;
    a.states = (const float *)states;
    a.noise = (const float *)prob->noise;
    a.dFds = (const float *)dF_ds;
    a.accept = accept;
    a.Jrev = (float4 *)(ws + oJ);
    a.brev = (float *)(ws + ob);
    a.dth = (float *)(ws + oth);
    a.deps = (float *)(ws + oep);
    switch (t.kind) {
    case PMC_TARGET_BANANA: PMC_TRY(adj_eval(ctx, a, Banana<float>{2})); break;
    case PMC_TARGET_FUNNEL:
        if (D <= 8)
            PMC_TRY(adj_eval(ctx, a, Funnel<float, 8>{D, (float)t.theta}));
        else
            PMC_TRY(adj_eval(ctx, a, Funnel<float, 32>{D, (float)t.theta}));
        break;
    case PMC_TARGET_GAUSSIAN:
        if (D <= 8)
            PMC_TRY(adj_eval(ctx, a, Gaussian<float, 8>{D, (const float *)t.mean, (const float *)t.prec}));
        else
            PMC_TRY(adj_eval(ctx, a, Gaussian<float, 32>{D, (const float *)t.mean, (const float *)t.prec}));
        break;
    default: set_error("pmc_adjoint: target"); return PMC_ERR_UNSUPPORTED;
    }
    float *mu = (float *)(ws + omu);
    PMC_TRY(launch_linrec_dense_mfma_packed(ctx, 0, D, T, a.Jrev, a.brev, mu, ws + ows));
    double *part = (double *)(ws + opart);
    hipLaunchKernelGGL(k_adj_dot, dim3(nb), dim3(256), 0, ctx->stream, (const float *)mu, a.dth, a.deps, T,
                       D, part);
    PMC_TRY_HIP(hipGetLastError());
    std::vector<double> hp(2 * nb);
    PMC_TRY_HIP(hipMemcpyAsync(hp.data(), part, sizeof(double) * 2 * nb, hipMemcpyDeviceToHost,
                               ctx->stream));
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    double s0 = 0, s1 = 0;
    for (int b = 0; b < nb; b++) {
        s0 += hp[2 * b];
        s1 += hp[2 * b + 1];
    }
    *dF_dtheta = s0;
    *dF_dstep = s1;
    return PMC_OK;
}
