// HMC with parallel leapfrog integration (Appendix A.2 algorithm, Sec. 3.3).
//
// One persistent workgroup runs the proposals in order.  For proposal p:
// v0 = momenta[p]; H0 = |v0|^2/2 - log p(x0); half step v += eps/2 grad log p(x0);
// the L leapfrog steps s_t = f(s_{t-1}) on s = [x, v] (x' = x + eps v,
// v' = v + eps grad log p(x')) are solved by Newton sweeps entirely in LDS:
//   eval:  F_t = f(S_{t-1}) for all t at once, the L gradients computed as one
//          product of the precision with the L positions;
//   scan:  per coordinate d the 2x2 recursion of block quasi-DEER
//          (Appendix A.3) with J_t = [[1, eps], [eps h, 1 + eps^2 h]],
//          h = d^2 log p / dx_d^2 at x'_t (diagonal quasi-DEER keeps only the
//          diagonal [1, 1 + eps^2 h]; Picard uses J = 0), in the form
//          S_t <- F_t + J_t delta_{t-1} with delta_t = J_t delta_{t-1} + F_t - S_t;
//   test:  Algorithm 1's max |delta| / (atol + rtol |S|) <= 1.
// then the reverse half step, HL, and the Metropolis test log U < H0 - HL.
// The sequential mode integrates the same L steps one after another.
//
// Target: Gaussian N(mu, P^-1) with P in global memory (read through the
// caches; it is re-read every sweep), FP32.
#include <math.h>
#include <string.h>

#include <vector>

#include "pmc_internal.hpp"

namespace pmc {
namespace {

struct HMCArgs {
    int D, L, n_prop;
    float eps;
    const float *mean, *prec;
    const float *x0, *momenta, *unif;
    float *chain;
    uint8_t *accept;
    int32_t *sweeps;
    int parallel;
    int variant;  // PMC_QDEER_BLOCK2, PMC_QDEER_DIAG, PMC_PICARD
    float atol, rtol;
    int floor_stall;
    int max_sweeps;
};

constexpr int kNT = 1024;

__device__ float block_sum(float v, float *red)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    float s = 0.f;
    for (int i = 0; i < kNT / 64; i++) s += red[i];
    return s;
}

__device__ float block_max(float v, float *red)
{
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    __syncthreads();
    if (l == 0) red[w] = v;
    __syncthreads();
    float s = 0.f;
    for (int i = 0; i < kNT / 64; i++) s = fmaxf(s, red[i]);
    return s;
}

// g = -P (x - mu) for `cnt` vectors stored row-wise at xs (stride 2D in LDS,
// x part first); writes g to gs (stride gstride).
__device__ void gauss_grads(const HMCArgs &a, const float *xs, int xstride, float *gs, int gstride,
                            int cnt)
{
    const int D = a.D;
    for (int o = threadIdx.x; o < cnt * D; o += kNT) {
        const int t = o / D, i = o % D;
        const float *row = a.prec + (size_t)i * D;
        const float *x = xs + (size_t)t * xstride;
        float s = 0.f;
        for (int k = 0; k < D; k++) s = fmaf(row[k], x[k] - a.mean[k], s);
        gs[(size_t)t * gstride + i] = -s;
    }
}

__global__ void __launch_bounds__(kNT) k_hmc(HMCArgs a)
{
    extern __shared__ float sm[];
    const int D = a.D, L = a.L, S2 = 2 * D;
    float *S = sm;                          // [(L+1) * 2D]: row 0 = s_0, row t = s_t
    float *F = S + (size_t)(L + 1) * S2;    // [L * 2D]
    float *x = F + (size_t)L * S2;          // [D] current state
    float *g = x + D;                       // [D] gradient scratch
    float *red = g + D;                     // [16]
    __shared__ int s_flag;
    const int tid = threadIdx.x;
    const float eps = a.eps;

    for (int i = tid; i < D; i += kNT) {
        x[i] = a.x0[i];
        a.chain[i] = a.x0[i];
    }
    __syncthreads();
    for (int p = 0; p < a.n_prop; p++) {
        const float *v0 = a.momenta + (size_t)p * D;
        // H0 and the half step
        gauss_grads(a, x, 0, g, 0, 1);
        __syncthreads();
        float kin = 0.f, lp = 0.f;
        for (int i = tid; i < D; i += kNT) {
            const float v = v0[i];
            kin += v * v;
            lp += (x[i] - a.mean[i]) * g[i];  // log p = (x - mu).g / 2
            S[i] = x[i];
            S[D + i] = v + 0.5f * eps * g[i];
        }
        const float H0 = 0.5f * block_sum(kin, red) - 0.5f * block_sum(lp, red);
        __syncthreads();
        int nsw = 0;
        if (a.parallel) {
            // initial guess: every s_t = s_0
            for (int o = tid; o < L * S2; o += kNT) S[S2 + o] = S[o % S2];
            __syncthreads();
            float best = INFINITY;
            int stall = 0;
            for (;;) {
                // eval: F_t = f(S_{t-1}); positions first, then the L gradients
                for (int o = tid; o < L * D; o += kNT) {
                    const int t = o / D, i = o % D;
                    const float *sp = S + (size_t)t * S2;
                    F[(size_t)t * S2 + i] = sp[i] + eps * sp[D + i];
                }
                __syncthreads();
                gauss_grads(a, F, S2, F + D, S2, L);  // F_t[D + i] <- g(x'_t)
                __syncthreads();
                for (int o = tid; o < L * D; o += kNT) {
                    const int t = o / D, i = o % D;
                    F[(size_t)t * S2 + D + i] = S[(size_t)t * S2 + D + i] + eps * F[(size_t)t * S2 + D + i];
                }
                __syncthreads();
                // scan per coordinate
                float rmax = 0.f;
                for (int d = tid; d < D; d += kNT) {
                    const float h = -a.prec[(size_t)d * D + d];
                    float ja = 1.f, jb = eps, jc = eps * h, jd = 1.f + eps * eps * h;
                    if (a.variant == PMC_QDEER_DIAG) jb = jc = 0.f;
                    if (a.variant == PMC_PICARD) ja = jb = jc = jd = 0.f;
                    float dx = 0.f, dv = 0.f;
                    for (int t = 1; t <= L; t++) {
                        float *st = S + (size_t)t * S2;
                        const float *ft = F + (size_t)(t - 1) * S2;
                        const float fx = ft[d], fv = ft[D + d];
                        const float nx = fx + ja * dx + jb * dv;  // S_t <- F_t + J delta_{t-1}
                        const float nv = fv + jc * dx + jd * dv;
                        dx = nx - st[d];
                        dv = nv - st[D + d];
                        const float r = fmaxf(fabsf(dx) / (a.atol + a.rtol * fabsf(nx)),
                                              fabsf(dv) / (a.atol + a.rtol * fabsf(nv)));
                        rmax = (r == r) ? fmaxf(rmax, r) : INFINITY;
                        st[d] = nx;
                        st[D + d] = nv;
                    }
                }
                const float ratio = block_max(rmax, red);
                nsw++;
                if (ratio < 0.5f * best) {
                    best = ratio;
                    stall = 0;
                } else {
                    stall++;
                }
                if (ratio <= 1.f || nsw >= a.max_sweeps ||
                    (a.floor_stall > 0 && stall >= a.floor_stall && ratio <= 100.f))
                    break;
                __syncthreads();
            }
        } else {
            // sequential leapfrog on row 0 of S
            for (int t = 1; t <= L; t++) {
                for (int i = tid; i < D; i += kNT) S[i] += eps * S[D + i];
                __syncthreads();
                gauss_grads(a, S, 0, g, 0, 1);
                __syncthreads();
                for (int i = tid; i < D; i += kNT) S[D + i] += eps * g[i];
                __syncthreads();
            }
        }
        const float *sL = a.parallel ? S + (size_t)L * S2 : S;
        __syncthreads();
        // reverse half step, HL, Metropolis test
        gauss_grads(a, sL, 0, g, 0, 1);
        __syncthreads();
        kin = 0.f;
        lp = 0.f;
        for (int i = tid; i < D; i += kNT) {
            const float v = sL[D + i] - 0.5f * eps * g[i];
            kin += v * v;
            lp += (sL[i] - a.mean[i]) * g[i];
        }
        const float HL = 0.5f * block_sum(kin, red) - 0.5f * block_sum(lp, red);
        if (tid == 0) {
            const int acc = logf(a.unif[p]) < H0 - HL;
            s_flag = acc;
            if (a.accept) a.accept[p] = (uint8_t)acc;
            if (a.sweeps) a.sweeps[p] = nsw;
        }
        __syncthreads();
        const int acc = s_flag;
        for (int i = tid; i < D; i += kNT) {
            if (acc) x[i] = sL[i];
            a.chain[(size_t)(p + 1) * D + i] = x[i];
        }
        __syncthreads();
    }
}

}  // namespace
}  // namespace pmc

using namespace pmc;

extern "C" pmc_status pmc_hmc_sample(pmc_context *ctx, const pmc_target *target, double step_size,
                                     int L, int n_prop, const void *x0, const void *momenta,
                                     const void *unif, const pmc_options *opts,
                                     int parallel_leapfrog, void *out_chain, uint8_t *accept,
                                     int32_t *sweeps, pmc_result *res)
{
    PMC_REQUIRE(ctx && target && opts, "pmc_hmc_sample: NULL argument");
    const DevTarget &t = target->t;
    if (t.kind != PMC_TARGET_GAUSSIAN || t.dtype != PMC_F32) {
        set_error("pmc_hmc_sample: parallel leapfrog is built for F32 Gaussian targets");
        return PMC_ERR_UNSUPPORTED;
    }
    PMC_REQUIRE(L >= 1 && n_prop >= 0, "pmc_hmc_sample: L >= 1, n_prop >= 0");
    PMC_REQUIRE(step_size > 0 && isfinite(step_size), "pmc_hmc_sample: step_size > 0");
    if (parallel_leapfrog) {
        const int v = opts->variant;
        if (v != PMC_QDEER_BLOCK2 && v != PMC_QDEER_DIAG && v != PMC_PICARD) {
            set_error("pmc_hmc_sample: variant must be block2, diag or picard");
            return PMC_ERR_UNSUPPORTED;
        }
    }
    const int D = t.dim;
    const size_t lds = sizeof(float) * ((size_t)(2 * L + 1) * 2 * D + 2 * D + 16);
    if (lds > 160 * 1024) {
        set_error("pmc_hmc_sample: L = %d, D = %d needs %zu bytes of LDS (> 160 KiB)", L, D, lds);
        return PMC_ERR_UNSUPPORTED;
    }
    if (res) memset(res, 0, sizeof(*res));
    if (n_prop == 0) return PMC_OK;
    PMC_REQUIRE(is_device_ptr(x0) && is_device_ptr(momenta) && is_device_ptr(unif) &&
                    is_device_ptr(out_chain),
                "pmc_hmc_sample: x0, momenta, unif, out_chain must be device pointers");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    PMC_TRY(ensure_pool(ctx, sizeof(int32_t) * n_prop + n_prop));
    int32_t *d_sw = (int32_t *)ctx->pool;
    uint8_t *d_acc = accept ? accept : (uint8_t *)ctx->pool + sizeof(int32_t) * n_prop;
    HMCArgs a;
    a.D = D;
    a.L = L;
    a.n_prop = n_prop;
    a.eps = (float)step_size;
    a.mean = (const float *)t.mean;
    a.prec = (const float *)t.prec;
    a.x0 = (const float *)x0;
    a.momenta = (const float *)momenta;
    a.unif = (const float *)unif;
    a.chain = (float *)out_chain;
    a.accept = d_acc;
    a.sweeps = d_sw;
    a.parallel = parallel_leapfrog;
    a.variant = opts->variant;
    a.atol = (float)opts->atol;
    a.rtol = (float)opts->rtol;
    a.floor_stall = opts->floor_stall;
    a.max_sweeps = opts->max_iter > 0 ? opts->max_iter : L + 1;
    PMC_TRY_HIP(hipFuncSetAttribute((const void *)k_hmc, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds));
    PMC_TRY_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    hipLaunchKernelGGL(k_hmc, dim3(1), dim3(kNT), lds, ctx->stream, a);
    PMC_TRY_HIP(hipGetLastError());
    PMC_TRY_HIP(hipEventRecord(ctx->ev1, ctx->stream));
    std::vector<int32_t> hsw(n_prop);
    std::vector<uint8_t> hacc(n_prop);
    PMC_TRY_HIP(hipMemcpyAsync(hsw.data(), d_sw, sizeof(int32_t) * n_prop, hipMemcpyDeviceToHost,
                               ctx->stream));
    PMC_TRY_HIP(hipMemcpyAsync(hacc.data(), d_acc, n_prop, hipMemcpyDeviceToHost, ctx->stream));
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (sweeps)
        for (int p = 0; p < n_prop; p++) sweeps[p] = hsw[p];
    float ms = 0;
    PMC_TRY_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (res) {
        res->elapsed_ms = ms;
        int64_t na = 0;
        int mx = 0;
        for (int p = 0; p < n_prop; p++) {
            na += hacc[p];
            mx = hsw[p] > mx ? hsw[p] : mx;
        }
        res->n_accept = na;
        res->sweeps_total = mx;
        res->n_converged = 1;
    }
    return PMC_OK;
}
