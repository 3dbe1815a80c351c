// HMC across the sequence (Sec. 3.3, "Parallel HMC with Sequential Leapfrog
// Integration"): the chain step f_t is one whole HMC transition, so the
// Newton sweep evaluates, for every step t of the active window at the
// current iterate x = s_{t-1}, the sequential leapfrog integrator and the
// accept gate, and the Jacobian dx_t/dx_{t-1} in the variant's structure.
//
// Transition (momentum draw xi_t ~ N(0, I), uniform u_t, diagonal mass
// matrix M = diag(m) given by its inverse, identity by default):
//   v0 = xi / sqrt(m);  v = v0 + eps/2 g(x0);
//   L times:  x <- x + eps M^-1 v,  v <- v + eps g(x);
//   v_f = v - eps/2 g(x_L);
//   H0 - HL = [v0.M^-1 v0 - v_f.M^-1 v_f] / 2 + log p(x_L) - log p(x0),
// the log-density difference taken from the exact increment x_L - x0 (the
// targets' difference forms), so FP32 does not subtract two large values;
// gate g~ = min(0, H0 - HL) - log u, accept iff g~ > 0 (select, no blend).
// Jacobian by forward-mode tangents through the integrator (the leapfrog
// Jacobian blocks of Sec. 3.3 applied to a direction d):
//   xd = d, vd = eps/2 H(x0) d;  per step xd += eps M^-1 vd, vd += eps H(x) xd;
//   J d = a xd_L + (1 - a) d, plus for the relaxed gate (Sec. 3.2's
//   stop-gradient construction) sigma'(g~) (x_L - x0) (dg~ . d) with
//   dg~ . d = 1(H0 - HL < 0) [-g(x0).d - (v_f.M^-1 vd_f - g(x_L).xd_L)],
//   vd_f = vd_L - eps/2 H(x_L) xd_L.
// Variants: exact diagonal (one tangent per coordinate), the one-probe
// diagonal z o (J z) (Sec. 3.4 eq. 10, one tangent), dense J for D <= 4
// (one tangent per column), Picard (no tangent).
//
// Per-lane targets run one step per lane with the state in registers.  The
// same-GPU sequential sampler for these targets is here too.
#include <math.h>

#include "pmc_internal.hpp"
#include "targets.hpp"

namespace pmc {
namespace {

template <typename R>
__device__ __forceinline__ R clampj_h(R v, double damping, double clip, int clip_inf)
{
    v = (R)damping * v;
    if (clip > 0 && !clip_inf) v = fmin(fmax(v, (R)-clip), (R)clip);
    return v;
}

// One HMC transition from x0 with momentum draw xi.  Outputs the end point
// x_L (and its increment dl = x_L - x0), the gradients at both ends, v0,
// v_f and the energy difference H0 - HL.
template <class Tg, typename R>
struct HmcLane {
    static constexpr int DM = Tg::DM;
    const Tg &tg;
    int D, L;
    R eps;
    const R *im;  // [D] or nullptr

    __device__ R imass(int d) const { return im ? im[d] : R(1); }

    __device__ R forward(const R *x0, const R *xi, R *v0, R *g0, R *xl, R *dl, R *gl, R *vf) const
    {
        R v[DM];
        tg.grad(x0, g0);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            v0[d] = d < D ? xi[d] / sqrt(imass(d)) : R(0);
            v[d] = fma(R(0.5) * eps, g0[d], v0[d]);
            dl[d] = R(0);
            xl[d] = x0[d];
            gl[d] = g0[d];
        }
        for (int l = 0; l < L; l++) {
#pragma unroll
            for (int d = 0; d < DM; d++) {
                if (d < D) dl[d] = fma(eps * imass(d), v[d], dl[d]);
                xl[d] = x0[d] + dl[d];
            }
            tg.grad(xl, gl);
#pragma unroll
            for (int d = 0; d < DM; d++) v[d] = fma(eps, gl[d], v[d]);
        }
        R kin = R(0);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            vf[d] = fma(R(-0.5) * eps, gl[d], v[d]);
            if (d < D) kin = fma(imass(d) * (v0[d] - vf[d]), v0[d] + vf[d], kin);
        }
        return R(0.5) * kin + tg.logp_diff(x0, xl, dl, g0, gl);
    }

    // J dir (without the (1 - a) part) and dg~ . dir: re-runs the integrator
    // carrying the tangent (xd, vd).  jd receives xd_L.
    __device__ R tangent(const R *x0, const R *v0, const R *g0, const R *dir, R *jd) const
    {
        R xl[DM], v[DM], g[DM], dl[DM], vd[DM], hv[DM];
        tg.hvp(x0, dir, hv);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            jd[d] = dir[d];
            vd[d] = R(0.5) * eps * hv[d];
            v[d] = fma(R(0.5) * eps, g0[d], v0[d]);
            dl[d] = R(0);
            xl[d] = x0[d];
            g[d] = g0[d];
        }
        for (int l = 0; l < L; l++) {
#pragma unroll
            for (int d = 0; d < DM; d++) {
                if (d < D) {
                    dl[d] = fma(eps * imass(d), v[d], dl[d]);
                    jd[d] = fma(eps * imass(d), vd[d], jd[d]);
                }
                xl[d] = x0[d] + dl[d];
            }
            tg.grad(xl, g);
            tg.hvp(xl, jd, hv);
#pragma unroll
            for (int d = 0; d < DM; d++) {
                v[d] = fma(eps, g[d], v[d]);
                vd[d] = fma(eps, hv[d], vd[d]);
            }
        }
        // dH/dx0 . dir, with H0 - HL
        tg.hvp(xl, jd, hv);
        R dhl = R(0), dh0 = R(0);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            const R vf = fma(R(-0.5) * eps, g[d], v[d]);
            const R vdf = fma(R(-0.5) * eps, hv[d], vd[d]);
            if (d < D) dhl = fma(imass(d) * vf, vdf, dhl);
            dhl = fma(-g[d], jd[d], dhl);
            dh0 = fma(-g0[d], dir[d], dh0);
        }
        return dh0 - dhl;
    }
};

template <class Tg, typename R, int JM>
__global__ void __launch_bounds__(256) k_eval_hmc_small(EvalArgs a, Tg tg)
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
    HmcLane<Tg, R> hl{tg, D, a.hmc_L, (R)a.eps, (const R *)a.inv_mass};

    R x0[DM], xi[DM], v0[DM], g0[DM], xl[DM], dl[DM], gl[DM], vf[DM];
#pragma unroll
    for (int d = 0; d < DM; d++) {
        if (d < D) {
            x0[d] = head ? ((const R *)a.s0)[(size_t)tl.chain * D + d] : S[(size_t)d * ld + t - 1];
            xi[d] = ((const R *)a.noise)[(size_t)t * D + d];
        } else {
            x0[d] = R(0);
            xi[d] = R(0);
        }
    }
    const R dh = hl.forward(x0, xi, v0, g0, xl, dl, gl, vf);
    const R la = dh < R(0) ? dh : R(0);
    const R gate = la - log(((const R *)a.unif)[t]);
    const int acc = sticky_decision(a, cs, t, (double)gate, (gate > R(0) && dh == dh) ? 1 : 0);
    R *F = (R *)a.F;
#pragma unroll
    for (int d = 0; d < DM; d++)
        if (d < D) F[(size_t)d * ld + t] = acc ? xl[d] : x0[d];
    if (a.accept) a.accept[t] = (uint8_t)acc;
    if (a.gtilde) a.gtilde[t] = (float)gate;
    if constexpr (JM == JM_NONE) return;

    const bool surr = a.gate == PMC_GATE_SURROGATE && dh < R(0);
    R coef = R(0);
    if (surr) {
        const R sg = R(1) / (R(1) + exp(-gate));
        coef = sg * (R(1) - sg);
    }
    R dir[DM], jd[DM];
    // J dir = a xd_L + (1 - a) dir + coef dl (dg~ . dir)
    auto jdir = [&](R *out) {
        const R dg = hl.tangent(x0, v0, g0, dir, jd);
#pragma unroll
        for (int d = 0; d < DM; d++) {
            R v = acc ? jd[d] : dir[d];
            if (surr) v = fma(coef * dl[d], dg, v);
            out[d] = v;
        }
    };
    if constexpr (JM == JM_DIAG) {
        R *J = (R *)a.J;
        R col[DM];
        if (a.probes) {
            const uint64_t hs = probe_mix(probe_mix(a.probe_seed) ^ (uint64_t)(uint32_t)cs.sweeps);
#pragma unroll
            for (int d = 0; d < DM; d++)
                dir[d] = d < D ? ((probe_mix(hs ^ (uint64_t)(1024 * t + d)) >> 63) ? R(-1) : R(1)) : R(0);
            jdir(col);
#pragma unroll
            for (int d = 0; d < DM; d++)
                if (d < D) J[(size_t)d * ld + t] = clampj_h(dir[d] * col[d], a.damping, a.clip, 0);
            return;
        }
        for (int k = 0; k < D; k++) {
#pragma unroll
            for (int d = 0; d < DM; d++) dir[d] = d == k ? R(1) : R(0);
            jdir(col);
            R jk = R(0);
#pragma unroll
            for (int d = 0; d < DM; d++)
                if (d == k) jk = col[d];
            J[(size_t)k * ld + t] = clampj_h(jk, a.damping, a.clip, 0);
        }
        return;
    }
    if constexpr (JM == JM_DENSE_ROW && DM <= 4) {
        R Jm[DM][DM], col[DM];
        for (int k = 0; k < D; k++) {
#pragma unroll
            for (int d = 0; d < DM; d++) dir[d] = d == k ? R(1) : R(0);
            jdir(col);
#pragma unroll
            for (int i = 0; i < DM; i++)
#pragma unroll
                for (int kk = 0; kk < DM; kk++)
                    if (kk == k) Jm[i][kk] = col[i];
        }
        R scale = (R)a.damping;
        if (a.clip > 0 && a.clip_inf) {
            R nrm = R(0);
            for (int i = 0; i < D; i++) {
                R r = R(0);
                for (int k = 0; k < D; k++) r += fabs(Jm[i][k]);
                nrm = fmax(nrm, r);
            }
            nrm *= scale;
            if (nrm > (R)a.clip) scale *= (R)a.clip / nrm;
        }
        R *J = (R *)a.J + (size_t)t * D * D;
        for (int i = 0; i < D; i++)
            for (int k = 0; k < D; k++) {
                R v = Jm[i][k] * scale;
                if (a.clip > 0 && !a.clip_inf) v = fmin(fmax(v, (R)-a.clip), (R)a.clip);
                J[i * D + k] = v;
            }
    }
}

template <class Tg, typename R>
__global__ void __launch_bounds__(64) k_seq_hmc_small(SeqArgs a, Tg tg)
{
    constexpr int DM = Tg::DM;
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= a.n_chains) return;
    const int D = a.D;
    const int64_t t0 = a.offsets[c], t1 = a.offsets[c + 1];
    const R *noise = (const R *)a.noise, *unif = (const R *)a.unif;
    R *out = (R *)a.out;
    HmcLane<Tg, R> hl{tg, D, a.hmc_L, (R)a.eps, (const R *)a.inv_mass};
    R x[DM], xi[DM], v0[DM], g0[DM], xl[DM], dl[DM], gl[DM], vf[DM];
#pragma unroll
    for (int d = 0; d < DM; d++) x[d] = d < D ? ((const R *)a.s0)[(size_t)c * D + d] : R(0);
    for (int64_t t = t0; t < t1; t++) {
#pragma unroll
        for (int d = 0; d < DM; d++) xi[d] = d < D ? noise[(size_t)t * D + d] : R(0);
        const R dh = hl.forward(x, xi, v0, g0, xl, dl, gl, vf);
        const R la = dh < R(0) ? dh : R(0);
        const R gate = la - log(unif[t]);
        const int acc = (gate > R(0) && dh == dh) ? 1 : 0;
        if (acc) {
#pragma unroll
            for (int d = 0; d < DM; d++) x[d] = xl[d];
        }
#pragma unroll
        for (int d = 0; d < DM; d++)
            if (d < D) out[(size_t)t * D + d] = x[d];
        if (a.accept) a.accept[t] = (uint8_t)acc;
        if (a.gtilde) a.gtilde[t] = (float)gate;
    }
}

template <class Tg, typename R>
pmc_status run(pmc_context *ctx, const EvalArgs &a, const Tg &tg)
{
    dim3 grid(a.n_tiles), block(256);
    switch (a.jmode) {
    case JM_DIAG: hipLaunchKernelGGL((k_eval_hmc_small<Tg, R, JM_DIAG>), grid, block, 0, ctx->stream, a, tg); break;
    case JM_DENSE_ROW:
        if (Tg::DM > 4) {
            set_error("HMC dense DEER on per-lane targets supports D <= 4");
            return PMC_ERR_UNSUPPORTED;
        }
        hipLaunchKernelGGL((k_eval_hmc_small<Tg, R, JM_DENSE_ROW>), grid, block, 0, ctx->stream, a, tg);
        break;
    case JM_NONE: hipLaunchKernelGGL((k_eval_hmc_small<Tg, R, JM_NONE>), grid, block, 0, ctx->stream, a, tg); break;
    default: set_error("HMC evaluation: unsupported Jacobian mode %d", a.jmode); return PMC_ERR_UNSUPPORTED;
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

template <class Tg, typename R>
pmc_status run(pmc_context *ctx, const SeqArgs &a, const Tg &tg)
{
    hipLaunchKernelGGL((k_seq_hmc_small<Tg, R>), dim3((a.n_chains + 63) / 64), dim3(64), 0, ctx->stream, a, tg);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

template <typename R, template <typename, int> class TG, class Args, class... Extra>
pmc_status by_dim(pmc_context *ctx, const Args &a, int D, Extra... ex)
{
    if (D <= 4) return run<TG<R, 4>, R>(ctx, a, TG<R, 4>{D, ex...});
    if (D <= 8) return run<TG<R, 8>, R>(ctx, a, TG<R, 8>{D, ex...});
    if (D <= 16) return run<TG<R, 16>, R>(ctx, a, TG<R, 16>{D, ex...});
    if constexpr (TG<R, 32>::kMaxLaneDim >= 32) {
        if (D <= 32) return run<TG<R, 32>, R>(ctx, a, TG<R, 32>{D, ex...});
    }
    set_error("per-lane evaluation of this target supports D <= %d (got %d)", TG<R, 32>::kMaxLaneDim, D);
    return PMC_ERR_UNSUPPORTED;
}

template <class Args>
pmc_status dispatch_small(pmc_context *ctx, const DevTarget &t, const Args &a)
{
    const int D = t.dim;
    switch (t.kind) {
    case PMC_TARGET_BANANA:
        if (t.dtype == PMC_F64) return run<Banana<double>, double>(ctx, a, Banana<double>{2});
        return run<Banana<float>, float>(ctx, a, Banana<float>{2});
    case PMC_TARGET_GAUSSIAN:
        if (t.dtype == PMC_F64)
            return by_dim<double, Gaussian>(ctx, a, D, (const double *)t.mean, (const double *)t.prec);
        return by_dim<float, Gaussian>(ctx, a, D, (const float *)t.mean, (const float *)t.prec);
    case PMC_TARGET_FUNNEL:
        if (t.dtype == PMC_F64) return by_dim<double, Funnel>(ctx, a, D, (double)t.theta);
        return by_dim<float, Funnel>(ctx, a, D, (float)t.theta);
    default: break;
    }
    set_error("HMC: unsupported per-lane target kind %d", (int)t.kind);
    return PMC_ERR_UNSUPPORTED;
}

}  // namespace

pmc_status launch_eval_hmc_logreg(pmc_context *ctx, const DevTarget &t, const EvalArgs &a);
pmc_status launch_seq_hmc_logreg(pmc_context *ctx, const DevTarget &t, const SeqArgs &a);

pmc_status launch_eval_hmc(pmc_context *ctx, const DevTarget &t, const EvalArgs &a)
{
    if (a.n_tiles == 0) return PMC_OK;
    if (t.kind == PMC_TARGET_LOGREG) return launch_eval_hmc_logreg(ctx, t, a);
    return dispatch_small(ctx, t, a);
}

pmc_status launch_sequential_hmc(pmc_context *ctx, const DevTarget &t, const SeqArgs &a)
{
    if (t.kind == PMC_TARGET_LOGREG) return launch_seq_hmc_logreg(ctx, t, a);
    return dispatch_small(ctx, t, a);
}

}  // namespace pmc
