// Evaluation step of the parallel Newton sweep (Sec. 2 eq. 2): for every
// step t of the active window, at the current iterate s_{t-1}, compute
// F_t = f_t(s_{t-1}) -- the MALA transition of Sec. 3.2 (or ULA) -- and the
// Jacobian J_t = df_t/ds in the structure the Newton variant uses.
//
// MALA in a form that keeps FP32 accurate (the decision compares a log ratio
// with log u, so it must not be the difference of two large log-densities):
// with g = grad log p(x), x~ = x + delta, delta = eps g + sqrt(2 eps) xi,
// g~ = grad log p(x~):
//   log q(x~|x) = -|xi|^2/2 and
//   log q(x|x~) = -(eps/4)|g + g~|^2 - sqrt(eps/2) xi.(g + g~) - |xi|^2/2,
// so  l = [log p(x~) - log p(x)] - (eps/4)|g + g~|^2 - sqrt(eps/2) xi.(g + g~),
// with the log-density difference computed from delta by the target.  Then
// log alpha = min(0, l), g~ate = log alpha - log u, accept iff g~ate > 0; the
// forward pass selects x~ or x (no 0 * inf from a blend).
// Frozen-gate Jacobian: a (I + eps H(x)) + (1 - a) I.  Surrogate gate (the
// stop-gradient relaxation of Sec. 3.2) adds sigma'(g~ate) delta (dl/dx)^T
// where l < 0, with dl/dx = M g~ - g + (H(x) w + M H(x~) w)/2,
// M = I + eps H(x), w = -delta - eps g~.
#include <math.h>

#include "pmc_internal.hpp"
#include "targets.hpp"

namespace pmc {
namespace {

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);                                             // round to nearest even
    return (uint16_t)(u >> 16);
}

template <typename R>
__device__ __forceinline__ R clampj(R v, double damping, double clip, int clip_inf)
{
    v = (R)damping * v;
    if (clip > 0 && !clip_inf) v = fmin(fmax(v, (R)-clip), (R)clip);
    return v;
}

// ------------------------------------------------ per-lane eval (small D)
template <class Tg, typename R, int JM>
__global__ void __launch_bounds__(256) k_eval_small(EvalArgs a, Tg tg)
{
    constexpr int DM = Tg::DM;
    const SegTile tl = a.tiles[blockIdx.x];
    const ChainStatus &cs = a.chains[tl.chain];
    if (!cs.active) return;
    const int64_t t = tl.start + threadIdx.x;
    if ((int)threadIdx.x >= tl.len || t < cs.win_start || t >= cs.win_end) return;
    const int D = a.D;
    const int64_t ld = a.ld;
    const R *S = (const R *)a.S;
    const bool head = (t == a.offsets[tl.chain]);

    R x[DM], xi[DM], g[DM], dl[DM], xt[DM], gt[DM];
#pragma unroll
    for (int d = 0; d < DM; d++) {
        if (d < D) {
            x[d] = head ? ((const R *)a.s0)[(size_t)tl.chain * D + d] : S[(size_t)d * ld + t - 1];
            xi[d] = ((const R *)a.noise)[(size_t)t * D + d];
        } else {
            x[d] = R(0);
            xi[d] = R(0);
        }
    }
    // orthogonal reparameterisation (Sec. 3.4 eq. 11): the planes hold
    // z = Q^T s, so the previous state is s = Q z (the chain's s0 is in s)
    const R *Q = (const R *)a.basis;
    if (Q && !head) {
        R z[DM];
#pragma unroll
        for (int d = 0; d < DM; d++) z[d] = x[d];
#pragma unroll
        for (int d = 0; d < DM; d++) {
            R v = R(0);
            if (d < D)
                for (int k = 0; k < D; k++) v = fma(Q[(size_t)d * D + k], z[k], v);
            x[d] = v;
        }
    }
    const R eps = (R)a.eps;
    const R c = sqrt(R(2) * eps);
    tg.grad(x, g);
#pragma unroll
    for (int d = 0; d < DM; d++) {
        dl[d] = d < D ? fma(eps, g[d], c * xi[d]) : R(0);
        xt[d] = x[d] + dl[d];
    }
    int acc = 1;
    R gate = R(INFINITY), ell = R(0);
    if (!a.ula) {
        tg.grad(xt, gt);
        R sn = R(0), sx = R(0);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            const R s = g[d] + gt[d];
            sn = fma(s, s, sn);
            sx = fma(xi[d], s, sx);
        }
        ell = tg.logp_diff(x, xt, dl, g, gt) - R(0.25) * eps * sn - sqrt(R(0.5) * eps) * sx;
        const R la = ell < R(0) ? ell : R(0);
        const R u = ((const R *)a.unif)[t];
        gate = la - log(u);
        acc = gate > R(0);
        if (!(ell == ell)) acc = 0;
        acc = sticky_decision(a, cs, t, (double)gate, acc);
    }
    R *F = (R *)a.F;
    if (Q) {
        // F~ = Q^T f
#pragma unroll
        for (int k = 0; k < DM; k++) {
            if (k < D) {
                R v = R(0);
#pragma unroll
                for (int d = 0; d < DM; d++)
                    if (d < D) v = fma(Q[(size_t)d * D + k], acc ? xt[d] : x[d], v);
                F[(size_t)k * ld + t] = v;
            }
        }
    } else {
#pragma unroll
        for (int d = 0; d < DM; d++)
            if (d < D) F[(size_t)d * ld + t] = acc ? xt[d] : x[d];
    }
    if (a.accept) a.accept[t] = (uint8_t)acc;
    if (a.gtilde) a.gtilde[t] = (float)gate;
    if (JM == JM_NONE) return;

    // surrogate-gate rank-one factor: coef * delta (dl/dx)^T
    R dldx[DM];
    R coef = R(0);
    const bool surr = !a.ula && a.gate == PMC_GATE_SURROGATE && ell < R(0);
    if (surr) {
        const R sg = R(1) / (R(1) + exp(-gate));
        coef = sg * (R(1) - sg);
        R w[DM], hw[DM], htw[DM], mhtw[DM], hgt[DM];
#pragma unroll
        for (int d = 0; d < DM; d++) w[d] = -dl[d] - eps * gt[d];
        tg.hvp(x, w, hw);
        tg.hvp(xt, w, htw);
        tg.hvp(x, htw, mhtw);
        tg.hvp(x, gt, hgt);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            mhtw[d] = htw[d] + eps * mhtw[d];
            dldx[d] = gt[d] + eps * hgt[d] - g[d] + R(0.5) * hw[d] + R(0.5) * mhtw[d];
        }
    }
    const R ea = acc ? eps : R(0);

    if (JM == JM_DIAG) {
        R *J = (R *)a.J;
        if (Q) {
            // diag(Q^T J Q): 1 + eps a q_k^T H q_k (+ the surrogate's
            // coef (q_k . dl)(dl/dx . q_k)) for each column q_k of Q
            for (int k = 0; k < D; k++) {
                R q[DM], hq[DM];
#pragma unroll
                for (int d = 0; d < DM; d++) q[d] = d < D ? Q[(size_t)d * D + k] : R(0);
                tg.hvp(x, q, hq);
                R qhq = R(0), qdl = R(0), qg = R(0);
#pragma unroll
                for (int d = 0; d < DM; d++) {
                    qhq = fma(q[d], hq[d], qhq);
                    if (surr) {
                        qdl = fma(q[d], dl[d], qdl);
                        qg = fma(dldx[d], q[d], qg);
                    }
                }
                R j = fma(ea, qhq, R(1));
                if (surr) j = fma(coef * qdl, qg, j);
                J[(size_t)k * ld + t] = clampj(j, a.damping, a.clip, 0);
            }
            return;
        }
        if (a.probes) {
            // z o (J z) with J z = z + eps H z (+ the rank-one surrogate term)
            R z[DM], hz[DM];
            const uint64_t hs = probe_mix(probe_mix(a.probe_seed) ^ (uint64_t)(uint32_t)cs.sweeps);
#pragma unroll
            for (int d = 0; d < DM; d++)
                z[d] = d < D ? ((probe_mix(hs ^ (uint64_t)(1024 * t + d)) >> 63) ? R(-1) : R(1)) : R(0);
            tg.hvp(x, z, hz);
            R dz = R(0);
            if (surr)
#pragma unroll
                for (int d = 0; d < DM; d++) dz = fma(dldx[d], z[d], dz);
#pragma unroll
            for (int d = 0; d < DM; d++) {
                if (d < D) {
                    R jz = fma(ea, hz[d], z[d]);
                    if (surr) jz = fma(coef * dl[d], dz, jz);
                    J[(size_t)d * ld + t] = clampj(z[d] * jz, a.damping, a.clip, 0);
                }
            }
            return;
        }
        R h[DM];
        tg.hess_diag(x, h);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            if (d < D) {
                R j = fma(ea, h[d], R(1));
                if (surr) j = fma(coef * dl[d], dldx[d], j);
                J[(size_t)d * ld + t] = clampj(j, a.damping, a.clip, 0);
            }
        }
        return;
    }

    // dense outputs: entry (i, j)
    auto entry = [&](int i, int k) -> R {
        if (i >= D || k >= D) return R(0);
        R v = (i == k ? R(1) : R(0)) + ea * tg.hess(x, i, k);
        if (surr) v = fma(coef * dl[i], dldx[k], v);
        return v;
    };
    R scale = (R)a.damping;
    if (a.clip > 0 && a.clip_inf) {
        R nrm = R(0);
        for (int i = 0; i < D; i++) {
            R r = R(0);
            for (int k = 0; k < D; k++) r += fabs(entry(i, k));
            nrm = fmax(nrm, r);
        }
        nrm *= scale;
        if (nrm > (R)a.clip) scale *= (R)a.clip / nrm;
    }
    const bool eclip = a.clip > 0 && !a.clip_inf;
    auto fin = [&](R v) -> R {
        v *= scale;
        if (eclip) v = fmin(fmax(v, (R)-a.clip), (R)a.clip);
        return v;
    };
    if (JM == JM_DENSE_ROW) {
        R *J = (R *)a.J + (size_t)t * D * D;
        for (int i = 0; i < D; i++)
            for (int k = 0; k < D; k++) J[i * D + k] = fin(entry(i, k));
    } else if (JM == JM_DENSE_BF16) {
        // element (i, k): kk = k/16, h = (k%16)/8, lane = 32 h + i, j = k%8
        uint4 *J = (uint4 *)((uint16_t *)a.J + (size_t)t * 1024);
        for (int kk = 0; kk < 2; kk++)
            for (int hh = 0; hh < 2; hh++)
                for (int i = 0; i < 32; i++) {
                    uint32_t p[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int k0 = kk * 16 + hh * 8 + 2 * q;
                        p[q] = (uint32_t)f2bf((float)fin(entry(i, k0))) |
                               ((uint32_t)f2bf((float)fin(entry(i, k0 + 1))) << 16);
                    }
                    J[kk * 64 + hh * 32 + i] = make_uint4(p[0], p[1], p[2], p[3]);
                }
    } else if (JM == JM_DENSE_F32) {
        // element (i, k): m = k/2, h = k%2, lane = 32 h + i, m4 = m/4, j = m%4
        float4 *J = (float4 *)((float *)a.J + (size_t)t * 1024);
        for (int m4 = 0; m4 < 4; m4++)
            for (int hh = 0; hh < 2; hh++)
                for (int i = 0; i < 32; i++) {
                    float v[4];
#pragma unroll
                    for (int q = 0; q < 4; q++) v[q] = (float)fin(entry(i, 2 * (4 * m4 + q) + hh));
                    J[m4 * 64 + hh * 32 + i] = make_float4(v[0], v[1], v[2], v[3]);
                }
    }
}

template <class Tg, typename R>
pmc_status eval_small(pmc_context *ctx, const EvalArgs &a, const Tg &tg)
{
    dim3 grid(a.n_tiles), block(256);
    switch (a.jmode) {
    case JM_DIAG: hipLaunchKernelGGL((k_eval_small<Tg, R, JM_DIAG>), grid, block, 0, ctx->stream, a, tg); break;
    case JM_DENSE_ROW: hipLaunchKernelGGL((k_eval_small<Tg, R, JM_DENSE_ROW>), grid, block, 0, ctx->stream, a, tg); break;
    case JM_DENSE_BF16: hipLaunchKernelGGL((k_eval_small<Tg, R, JM_DENSE_BF16>), grid, block, 0, ctx->stream, a, tg); break;
    case JM_DENSE_F32: hipLaunchKernelGGL((k_eval_small<Tg, R, JM_DENSE_F32>), grid, block, 0, ctx->stream, a, tg); break;
    default: hipLaunchKernelGGL((k_eval_small<Tg, R, JM_NONE>), grid, block, 0, ctx->stream, a, tg); break;
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

template <typename R, template <typename, int> class TG, class... Extra>
pmc_status eval_dm(pmc_context *ctx, const EvalArgs &a, int D, Extra... ex)
{
    if (D <= 4) return eval_small<TG<R, 4>, R>(ctx, a, TG<R, 4>{D, ex...});
    if (D <= 8) return eval_small<TG<R, 8>, R>(ctx, a, TG<R, 8>{D, ex...});
    if (D <= 16) return eval_small<TG<R, 16>, R>(ctx, a, TG<R, 16>{D, ex...});
    if constexpr (TG<R, 32>::kMaxLaneDim >= 32) {
        if (D <= 32) return eval_small<TG<R, 32>, R>(ctx, a, TG<R, 32>{D, ex...});
    }
    set_error("per-lane evaluation of this target supports D <= %d (got %d)", TG<R, 32>::kMaxLaneDim, D);
    return PMC_ERR_UNSUPPORTED;
}

}  // namespace

int eval_tile_steps(const DevTarget &tg)
{
    if (tg.kind == PMC_TARGET_LOGREG) return tg.dim >= kWideMinDim ? wide_tile_steps() : 32;
    return 256;
}

pmc_status launch_eval(pmc_context *ctx, const DevTarget &t, const EvalArgs &a)
{
    if (a.n_tiles == 0) return PMC_OK;
    if (a.hmc_L > 0) return launch_eval_hmc(ctx, t, a);
    const int D = t.dim;
    switch (t.kind) {
    case PMC_TARGET_BANANA:
        if (t.dtype == PMC_F64) return eval_small<Banana<double>, double>(ctx, a, Banana<double>{2});
        return eval_small<Banana<float>, float>(ctx, a, Banana<float>{2});
    case PMC_TARGET_GAUSSIAN:
        if (t.dtype == PMC_F64)
            return eval_dm<double, Gaussian>(ctx, a, D, (const double *)t.mean, (const double *)t.prec);
        return eval_dm<float, Gaussian>(ctx, a, D, (const float *)t.mean, (const float *)t.prec);
    case PMC_TARGET_FUNNEL:
        if (t.dtype == PMC_F64) return eval_dm<double, Funnel>(ctx, a, D, (double)t.theta);
        return eval_dm<float, Funnel>(ctx, a, D, (float)t.theta);
    case PMC_TARGET_LOGREG:
        if (t.dtype != PMC_F32) {
            set_error("logistic regression runs in F32");
            return PMC_ERR_UNSUPPORTED;
        }
        if (t.dim >= kWideMinDim) {
            set_error("logistic regression with D > 32 is evaluated by the solve's GEMM path only");
            return PMC_ERR_UNSUPPORTED;
        }
        // dense modes: the kernel writes f_t and the decisions only; the
        // Jacobians come from launch_logreg_dense_jac
        if (a.gate == PMC_GATE_SURROGATE && !a.ula) {
            set_error("logistic regression eval supports the frozen gate only");
            return PMC_ERR_UNSUPPORTED;
        }
        return launch_eval_logreg(ctx, t, a);
    }
    set_error("unknown target kind %d", (int)t.kind);
    return PMC_ERR_INVALID;
}

}  // namespace pmc
