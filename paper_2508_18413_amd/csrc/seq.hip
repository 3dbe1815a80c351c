// Same-GPU sequential samplers: s_t = f_t(s_{t-1}) evaluated step after step
// on the device (Sec. 2, the sequential evaluation the parallel Newton solve
// replaces).  They are the baseline of the chain-steps/s comparison, so they
// are written to be fast: the whole T-step loop runs inside one launch with
// no host round trips, the next step's noise is prefetched, and the
// transition reuses the gradient of the current state (computed once, when
// that state was proposed).
//
// Small targets: one lane per chain, state in registers.
// Logistic regression: one workgroup per chain; each thread owns data rows
// (X rows and the current linear predictor z_n in registers) and the
// per-step gradient is a workgroup reduction.
#include <math.h>

#include "logistic.hpp"
#include "pmc_internal.hpp"
#include "targets.hpp"

namespace pmc {
namespace {

// softplus(z + dz) - softplus(z) from s = sigma(z): log1p(s expm1(dz)), written
// out directly for large or very negative increments.
__device__ __forceinline__ float softplus_diff(float z, float dz, float s)
{
    if (dz > -8.f && dz < 30.f) return log1p_s(s * expm1_s(dz));
    return softplus(z + dz) - softplus(z);
}

// Workgroup barrier that orders LDS only: global loads issued before it stay
// in flight (the sampler prefetches the next step's noise across it).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <class Tg, typename R>
__global__ void __launch_bounds__(64) k_seq_small(SeqArgs a, Tg tg)
{
    constexpr int DM = Tg::DM;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    const int D = a.D;
    const int64_t t0 = a.offsets[c], t1 = a.offsets[c + 1];
    const R *noise = (const R *)a.noise, *unif = (const R *)a.unif;
    R *out = (R *)a.out;
    R x[DM], g[DM], xi[DM], xt[DM], gt[DM], dl[DM];
#pragma unroll
    for (int d = 0; d < DM; d++) x[d] = d < D ? ((const R *)a.s0)[(size_t)c * D + d] : R(0);
    tg.grad(x, g);
    const R eps = (R)a.eps, cc = sqrt(R(2) * eps), hq = sqrt(R(0.5) * eps);
    for (int64_t t = t0; t < t1; t++) {
#pragma unroll
        for (int d = 0; d < DM; d++) xi[d] = d < D ? noise[(size_t)t * D + d] : R(0);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            dl[d] = d < D ? fma(eps, g[d], cc * xi[d]) : R(0);
            xt[d] = x[d] + dl[d];
        }
        tg.grad(xt, gt);
        int acc = 1;
        R gate = R(INFINITY);
        if (!a.ula) {
            R sn = R(0), sx = R(0);
#pragma unroll
            for (int d = 0; d < DM; d++) {
                const R s = g[d] + gt[d];
                sn = fma(s, s, sn);
                sx = fma(xi[d], s, sx);
            }
            const R ell = tg.logp_diff(x, xt, dl, g, gt) - R(0.25) * eps * sn - hq * sx;
            const R la = ell < R(0) ? ell : R(0);
            gate = la - log(unif[t]);
            acc = gate > R(0);
            if (!(ell == ell)) acc = 0;
        }
        if (acc) {
#pragma unroll
            for (int d = 0; d < DM; d++) {
                x[d] = xt[d];
                g[d] = gt[d];
            }
        }
#pragma unroll
        for (int d = 0; d < DM; d++)
            if (d < D) out[(size_t)t * D + d] = x[d];
        if (a.accept) a.accept[t] = (uint8_t)acc;
        if (a.gtilde) a.gtilde[t] = (float)gate;
    }
}

// Workgroup-per-chain logistic regression sampler (F32).  The state and its
// gradient live in wave 0 (lane d holds coordinate d); every thread owns RPT
// data rows with their linear predictors.  Per step: wave 0 publishes the
// increment delta and the proposal through LDS, every thread recomputes its
// rows' predictors at the proposal from scratch (never by accumulating
// increments, so rounding does not build up over accepted steps) and its
// partial sums, the partials are summed through LDS in 8-way column groups,
// and wave 0 takes the accept decision.
template <int DM, int NT, int RPT>
__global__ void __launch_bounds__(NT)
k_seq_logreg(SeqArgs a, const float *__restrict__ X, const float *__restrict__ y, int N, float pp)
{
    constexpr int V = DM + 1;    // reduced values: gradient (DM) + log-likelihood difference
    constexpr int VS = V + 1;    // odd LDS row stride
    constexpr int GRP = (V * 8 <= NT) ? 8 : 4;  // threads summing one column
    static_assert(V * GRP <= NT, "reduction groups exceed the block");
    __shared__ float s_part[NT * VS];
    __shared__ float s_sum[V];
    __shared__ float s_dl[DM], s_xt[DM];
    __shared__ int s_acc;
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int D = a.D;
    const int64_t t0 = a.offsets[c], t1 = a.offsets[c + 1];
    const float eps = (float)a.eps, cc = sqrtf(2.f * eps), hq = sqrtf(0.5f * eps);
    const float *noise = (const float *)a.noise, *unif = (const float *)a.unif;
    float *out = (float *)a.out;
    const bool w0 = tid < 64;
    const bool own = w0 && lane < D;  // lanes 32..63 of wave 0 never own a coordinate (D <= 32)

    float xr[RPT][DM], yr[RPT], z[RPT], sz[RPT];
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int n = tid + k * NT;
        const bool ok = n < N;
#pragma unroll
        for (int d = 0; d < DM; d++) xr[k][d] = ok ? X[(size_t)n * DM + d] : 0.f;
        yr[k] = ok ? y[n] : 0.f;
    }
    // wave-0 state: x_d, g_d
    float x = own ? ((const float *)a.s0)[(size_t)c * D + lane] : 0.f;
    float g = 0.f;

    auto column_sum = [&](float (&v)[V]) {
#pragma unroll
        for (int i = 0; i < V; i++) s_part[tid * VS + i] = v[i];
        lds_barrier();
        if (tid < V * GRP) {
            const int i = tid / GRP, p = tid % GRP;
            float s = 0.f;
            for (int r = p; r < NT; r += GRP) s += s_part[r * VS + i];
#pragma unroll
            for (int m = 1; m < GRP; m <<= 1) s += __shfl_xor(s, m, 64);
            if (p == 0) s_sum[i] = s;
        }
        lds_barrier();
    };

    // initial gradient: publish x through s_dl, rows compute predictors
    if (w0 && lane < DM) s_dl[lane] = x;
    __syncthreads();
    {
        float v[V];
#pragma unroll
        for (int i = 0; i < V; i++) v[i] = 0.f;
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            float zz = 0.f;
#pragma unroll
            for (int d = 0; d < DM; d++) zz = fmaf(xr[k][d], s_dl[d], zz);
            z[k] = zz;
            sz[k] = sigm(zz);
            const float r = yr[k] - sz[k];
#pragma unroll
            for (int d = 0; d < DM; d++) v[d] = fmaf(r, xr[k][d], v[d]);
        }
        column_sum(v);
        if (w0 && lane < DM) g = s_sum[lane] - pp * x;
    }

    // wave 0 publishes the first increment; afterwards each step's epilogue
    // publishes the decision together with the next step's increment
    float xi = (own && t0 < t1) ? noise[(size_t)t0 * D + lane] : 0.f;
    float u = (t0 < t1 && unif) ? unif[t0] : 0.5f;
    float dl = 0.f;
    if (w0) {
        dl = own ? fmaf(eps, g, cc * xi) : 0.f;
        if (lane < DM) {
            s_dl[lane] = dl;
            s_xt[lane] = x + dl;
        }
        if (lane == 0) s_acc = 0;
    }
    __syncthreads();
    float zt[RPT], szt[RPT];
    for (int64_t t = t0; t < t1; t++) {
        // the next step's noise and uniform, loaded now and used at the end
        // of this step (LDS-only barriers keep the loads in flight)
        float xin = 0.f, un = 0.5f;
        if (w0 && t + 1 < t1) {
            xin = own ? noise[(size_t)(t + 1) * D + lane] : 0.f;
            if (unif) un = unif[t + 1];
        }
        // rows: predictors at the proposal, gradient and log-likelihood partials
        float v[V];
#pragma unroll
        for (int i = 0; i < V; i++) v[i] = 0.f;
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            float dz = 0.f, zz = 0.f;
#pragma unroll
            for (int d = 0; d < DM; d++) {
                dz = fmaf(xr[k][d], s_dl[d], dz);
                zz = fmaf(xr[k][d], s_xt[d], zz);
            }
            zt[k] = zz;
            szt[k] = sigm(zz);
            const float spd = softplus_diff(z[k], dz, sz[k]);
            const float r = yr[k] - szt[k];
#pragma unroll
            for (int d = 0; d < DM; d++) v[d] = fmaf(r, xr[k][d], v[d]);
            v[DM] += yr[k] * dz - spd;
        }
        column_sum(v);
        if (w0) {
            const float xt = x + dl;
            const float gt = own ? s_sum[lane] - pp * xt : 0.f;
            const float sg = g + gt;
            float sn = own ? sg * sg : 0.f, sx = own ? xi * sg : 0.f, dpr = own ? dl * (xt + x) : 0.f;
#pragma unroll
            for (int m = 16; m >= 1; m >>= 1) {  // D <= 32: lanes 0..31 hold the components
                sn += __shfl_xor(sn, m, 32);
                sx += __shfl_xor(sx, m, 32);
                dpr += __shfl_xor(dpr, m, 32);
            }
            int acc = 1;
            float gate = INFINITY;
            if (!a.ula) {
                const float ell = s_sum[DM] - 0.5f * pp * dpr - 0.25f * eps * sn - hq * sx;
                const float la = ell < 0.f ? ell : 0.f;
                gate = la - logf(u);
                acc = gate > 0.f;
                if (!(ell == ell)) acc = 0;
            }
            if (acc) {
                x = xt;
                g = gt;
            }
            if (own) out[(size_t)t * D + lane] = x;
            if (lane == 0) {
                if (a.accept) a.accept[t] = (uint8_t)acc;
                if (a.gtilde) a.gtilde[t] = gate;
            }
            // next step's increment
            if (t + 1 < t1) {
                xi = xin;
                u = un;
                dl = own ? fmaf(eps, g, cc * xi) : 0.f;
                if (lane < DM) {
                    s_dl[lane] = dl;
                    s_xt[lane] = x + dl;
                }
            }
            if (lane == 0) s_acc = acc;
        }
        lds_barrier();
        if (s_acc) {
#pragma unroll
            for (int k = 0; k < RPT; k++) {
                z[k] = zt[k];
                sz[k] = szt[k];
            }
        }
    }
}

template <class Tg, typename R>
pmc_status seq_small(pmc_context *ctx, const SeqArgs &a, const Tg &tg)
{
    hipLaunchKernelGGL((k_seq_small<Tg, R>), dim3((a.n_chains + 63) / 64), dim3(64), 0, ctx->stream, a, tg);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

template <typename R, template <typename, int> class TG, class... Extra>
pmc_status seq_dm(pmc_context *ctx, const SeqArgs &a, int D, Extra... ex)
{
    if (D <= 4) return seq_small<TG<R, 4>, R>(ctx, a, TG<R, 4>{D, ex...});
    if (D <= 8) return seq_small<TG<R, 8>, R>(ctx, a, TG<R, 8>{D, ex...});
    if (D <= 16) return seq_small<TG<R, 16>, R>(ctx, a, TG<R, 16>{D, ex...});
    if constexpr (TG<R, 32>::kMaxLaneDim >= 32) {
        if (D <= 32) return seq_small<TG<R, 32>, R>(ctx, a, TG<R, 32>{D, ex...});
    }
    set_error("per-lane evaluation of this target supports D <= %d (got %d)", TG<R, 32>::kMaxLaneDim, D);
    return PMC_ERR_UNSUPPORTED;
}

}  // namespace

pmc_status launch_sequential(pmc_context *ctx, const DevTarget &t, const SeqArgs &a)
{
    const int D = t.dim;
    switch (t.kind) {
    case PMC_TARGET_BANANA:
        if (t.dtype == PMC_F64) return seq_small<Banana<double>, double>(ctx, a, Banana<double>{2});
        return seq_small<Banana<float>, float>(ctx, a, Banana<float>{2});
    case PMC_TARGET_GAUSSIAN:
        if (t.dtype == PMC_F64)
            return seq_dm<double, Gaussian>(ctx, a, D, (const double *)t.mean, (const double *)t.prec);
        return seq_dm<float, Gaussian>(ctx, a, D, (const float *)t.mean, (const float *)t.prec);
    case PMC_TARGET_FUNNEL:
        if (t.dtype == PMC_F64) return seq_dm<double, Funnel>(ctx, a, D, (double)t.theta);
        return seq_dm<float, Funnel>(ctx, a, D, (float)t.theta);
    case PMC_TARGET_LOGREG: {
        if (t.dim >= kWideMinDim) return launch_sequential_logreg_wide(ctx, t, a);
        // 256 threads x 4 rows up to 1024 data points, 512 x 4 up to 2048
        if (t.n_data > 4 * 512) {
            set_error("sequential logreg sampler supports n_data <= 2048");
            return PMC_ERR_UNSUPPORTED;
        }
        const float pp = (float)(1.0 / t.prior_var);
        const float *X = (const float *)t.X, *y = (const float *)t.y;
        dim3 grid(a.n_chains);
        if (t.n_data <= 4 * 256) {
            dim3 block(256);
            switch (t.ldx) {
            case 4: hipLaunchKernelGGL((k_seq_logreg<4, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 8: hipLaunchKernelGGL((k_seq_logreg<8, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 16: hipLaunchKernelGGL((k_seq_logreg<16, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 25: hipLaunchKernelGGL((k_seq_logreg<25, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 32: hipLaunchKernelGGL((k_seq_logreg<32, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            default: set_error("logreg: unsupported padded dimension %d", t.ldx); return PMC_ERR_UNSUPPORTED;
            }
        } else {
            dim3 block(512);
            switch (t.ldx) {
            case 4: hipLaunchKernelGGL((k_seq_logreg<4, 512, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 8: hipLaunchKernelGGL((k_seq_logreg<8, 512, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 16: hipLaunchKernelGGL((k_seq_logreg<16, 512, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 25: hipLaunchKernelGGL((k_seq_logreg<25, 512, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            case 32: hipLaunchKernelGGL((k_seq_logreg<32, 512, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
            default: set_error("logreg: unsupported padded dimension %d", t.ldx); return PMC_ERR_UNSUPPORTED;
            }
        }
        PMC_TRY_HIP(hipGetLastError());
        return PMC_OK;
    }
    }
    set_error("unknown target kind");
    return PMC_ERR_INVALID;
}

}  // namespace pmc
