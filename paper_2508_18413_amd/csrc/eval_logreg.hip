// Evaluation step for the Bayesian logistic-regression target on gfx950
// matrix cores.  For 32 consecutive steps (one wavefront) the per-step
// matrix-vector products of the MALA transition (Sec. 3.2) are batched into
// 32 x 32 x 2 FP32 matrix-core products over row tiles of 32 data points:
//   pass 1:  Z = X S            (linear predictors at s_{t-1}),
//            G = X^T (y - sigma(Z))              -> grad log-likelihood at s_{t-1}
//   pass 2:  Z, dZ = X Delta    (predictors at s_{t-1} and their increment),
//            G~ = X^T (y - sigma(Z + dZ))        -> grad at the proposal,
//            Hd = (X o X)^T (sigma(Z)(1 - sigma(Z)))  -> minus the Hessian diagonal,
//            sum_n [y dz - log1p(sigma(z) expm1(dz))]  -> log-likelihood difference,
// then one lane per step assembles the log Metropolis ratio in the
// cancellation-free form (the proposal-density terms through g + g~), the
// accept decision, f_t and the quasi-DEER Jacobian diagonal
// a (1 + eps H_dd) + (1 - a).
//
// Operands (lane l, i = l % 32, hh = l / 32; K = 2 per instruction):
//   A fragments are precomputed per row tile rt when the target is created:
//     xa[rt][m][l]   = X[32 rt + i][2 m + hh]          (A of Z = X S)
//     xta[rt][m][l]  = X[32 rt + 2 m + hh][i]          (A of G = X^T R)
//     x2ta[rt][m][l] = X[32 rt + 2 m + hh][i]^2
//   B operands: S_B[m] = s_{t-1}[2 m + hh] for step t = t0 + i; R in the
//   accumulator layout (register r holds row 8 (r / 4) + 4 hh + r % 4 of the
//   tile) is moved to the B layout (row 2 m + hh) by exchanging half of the
//   registers between lanes l and l ^ 32.
#include <math.h>

#include "pmc_internal.hpp"

namespace pmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kWaves = 4;

__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

__device__ __forceinline__ float sigm(float z)
{
    const float e = expf(-fabsf(z));
    const float r = 1.f / (1.f + e);
    return z >= 0.f ? r : e * r;
}

// With s = sigma(z) and m = expm1(dz): sigma(z + dz) = s (1 + m) / (1 + s m) and
// softplus(z + dz) - softplus(z) = log1p(s m); one exponential serves both.
// Large increments (dz >= 30) take the direct forms.
__device__ __forceinline__ void shifted(float z, float dz, float s, float &st, float &spd)
{
    if (dz < 30.f) {
        const float m = expm1f(dz);
        const float q = fmaf(s, m, 1.f);
        st = s * (1.f + m) / q;
        spd = log1pf(s * m);
    } else {
        const float zt = z + dz;
        st = sigm(zt);
        const float spt = zt > 0.f ? zt + log1pf(expf(-zt)) : log1pf(expf(zt));
        const float sp = z > 0.f ? z + log1pf(expf(-z)) : log1pf(expf(z));
        spd = spt - sp;
    }
}

// accumulator -> B operand (rows of parity hh)
__device__ __forceinline__ void acc_to_b(const f32x16 &c, float (&b)[16], int h)
{
    float rc[8];
#pragma unroll
    for (int q = 0; q < 8; q++) rc[q] = __shfl_xor(h ? c[2 * q] : c[2 * q + 1], 32, 64);
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const int g = m >> 2, w = m & 3;
        if (h == 0)
            b[m] = w < 2 ? c[4 * g + 2 * w] : rc[2 * g + (w - 2)];
        else
            b[m] = w < 2 ? rc[2 * g + w] : c[4 * g + 2 * (w - 2) + 1];
    }
}

struct Frags {
    const float *xa, *xta, *x2ta, *y;
    int nr;
    float pp;  // prior precision 1 / prior_var
};

template <int MK>
__global__ void __launch_bounds__(64 * kWaves, 2) k_eval_logreg(EvalArgs a, Frags f)
{
    __shared__ float s_t[kWaves][3][32 * 33];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, j = lane & 31, hh = lane >> 5;
    const int tix = blockIdx.x * kWaves + w;
    if (tix >= a.n_tiles) return;
    const SegTile tl = a.tiles[tix];
    const ChainStatus &cs = a.chains[tl.chain];
    if (!cs.active || tl.start + tl.len <= cs.win_start) return;
    const int64_t t = tl.start + j;
    const bool valid = j < tl.len && t >= cs.win_start;
    const int64_t tt = j < tl.len ? t : tl.start;
    const int D = a.D;
    const int64_t ld = a.ld;
    const bool head = (tt == a.offsets[tl.chain]);
    const float *S = (const float *)a.S, *s0 = (const float *)a.s0 + (size_t)tl.chain * D;
    const float *noise = (const float *)a.noise;
    const float eps = (float)a.eps, c = sqrtf(2.f * eps), pp = f.pp;
    float *sg = s_t[w][0], *sgt = s_t[w][1], *shd = s_t[w][2];

    float SB[MK];
#pragma unroll
    for (int m = 0; m < MK; m++) {
        const int d = 2 * m + hh;
        SB[m] = d < D ? (head ? s0[d] : S[(size_t)d * ld + tt - 1]) : 0.f;
    }
    const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    // ---- pass 1: gradient of the log-likelihood at s_{t-1}
    f32x16 G = zero;
    for (int rt = 0; rt < f.nr; rt++) {
        const float *xa = f.xa + (size_t)rt * MK * 64 + lane;
        const float *xta = f.xta + (size_t)rt * 16 * 64 + lane;
        f32x16 Z = zero;
#pragma unroll
        for (int m = 0; m < MK; m++) Z = __builtin_amdgcn_mfma_f32_32x32x2f32(xa[m * 64], SB[m], Z, 0, 0, 0);
        f32x16 R;
#pragma unroll
        for (int r = 0; r < 16; r++) R[r] = f.y[32 * rt + crow(r, hh)] - sigm(Z[r]);
        float RB[16];
        acc_to_b(R, RB, hh);
#pragma unroll
        for (int m = 0; m < 16; m++) G = __builtin_amdgcn_mfma_f32_32x32x2f32(xta[m * 64], RB[m], G, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 16; r++) sg[crow(r, hh) * 33 + j] = G[r];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // proposal increment Delta = eps g + sqrt(2 eps) xi in the B layout
    float DB[MK];
#pragma unroll
    for (int m = 0; m < MK; m++) {
        const int d = 2 * m + hh;
        DB[m] = 0.f;
        if (d < D) {
            const float g = sg[d * 33 + j] - pp * SB[m];
            DB[m] = fmaf(eps, g, c * noise[(size_t)tt * D + d]);
        }
    }

    // ---- pass 2: gradient at the proposal, Hessian diagonal, log-likelihood difference
    f32x16 Gt = zero, Hd = zero;
    float dll = 0.f;
    for (int rt = 0; rt < f.nr; rt++) {
        const float *xa = f.xa + (size_t)rt * MK * 64 + lane;
        const float *xta = f.xta + (size_t)rt * 16 * 64 + lane;
        const float *x2ta = f.x2ta + (size_t)rt * 16 * 64 + lane;
        f32x16 Z = zero, dZ = zero;
#pragma unroll
        for (int m = 0; m < MK; m++) {
            const float a1 = xa[m * 64];
            Z = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, SB[m], Z, 0, 0, 0);
            dZ = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, DB[m], dZ, 0, 0, 0);
        }
        f32x16 Rt, Wv;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float yv = f.y[32 * rt + crow(r, hh)];
            const float z = Z[r], dz = dZ[r];
            const float s = sigm(z);
            float st, spd;
            shifted(z, dz, s, st, spd);
            Rt[r] = yv - st;
            Wv[r] = s * (1.f - s);
            dll += yv * dz - spd;
        }
        {
            float RB[16];
            acc_to_b(Rt, RB, hh);
#pragma unroll
            for (int m = 0; m < 16; m++)
                Gt = __builtin_amdgcn_mfma_f32_32x32x2f32(xta[m * 64], RB[m], Gt, 0, 0, 0);
        }
        {
            float WB[16];
            acc_to_b(Wv, WB, hh);
#pragma unroll
            for (int m = 0; m < 16; m++)
                Hd = __builtin_amdgcn_mfma_f32_32x32x2f32(x2ta[m * 64], WB[m], Hd, 0, 0, 0);
        }
    }
#pragma unroll
    for (int r = 0; r < 16; r++) {
        sgt[crow(r, hh) * 33 + j] = Gt[r];
        shd[crow(r, hh) * 33 + j] = Hd[r];
    }
    dll += __shfl_xor(dll, 32, 64);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (hh != 0 || !valid) return;

    // ---- one lane per step: log ratio, decision, f_t, Jacobian diagonal
    float sn = 0.f, sx = 0.f, dpr = 0.f;
    for (int d = 0; d < D; d++) {
        const float x = head ? s0[d] : S[(size_t)d * ld + t - 1];
        const float xi = noise[(size_t)t * D + d];
        const float g = sg[d * 33 + j] - pp * x;
        const float dl = fmaf(eps, g, c * xi);
        const float xt = x + dl;
        const float gt = sgt[d * 33 + j] - pp * xt;
        const float s = g + gt;
        sn = fmaf(s, s, sn);
        sx = fmaf(xi, s, sx);
        dpr = fmaf(dl, xt + x, dpr);
    }
    int acc = 1;
    float gate = INFINITY;
    if (!a.ula) {
        const float ell = dll - 0.5f * pp * dpr - 0.25f * eps * sn - sqrtf(0.5f * eps) * sx;
        const float la = ell < 0.f ? ell : 0.f;
        gate = la - logf(((const float *)a.unif)[t]);
        acc = gate > 0.f;
        if (!(ell == ell)) acc = 0;
    }
    float *F = (float *)a.F;
    float *J = (float *)a.J;
    const float ea = acc ? eps : 0.f;
    for (int d = 0; d < D; d++) {
        const float x = head ? s0[d] : S[(size_t)d * ld + t - 1];
        const float g = sg[d * 33 + j] - pp * x;
        const float xt = x + fmaf(eps, g, c * noise[(size_t)t * D + d]);
        F[(size_t)d * ld + t] = acc ? xt : x;
        if (a.jmode == JM_DIAG) {
            const float hdd = -shd[d * 33 + j] - pp;
            float jv = (float)a.damping * fmaf(ea, hdd, 1.f);
            if (a.clip > 0) jv = fminf(fmaxf(jv, (float)-a.clip), (float)a.clip);
            J[(size_t)d * ld + t] = jv;
        }
    }
    if (a.accept) a.accept[t] = (uint8_t)acc;
    if (a.gtilde) a.gtilde[t] = gate;
}

// A-operand fragments of X, X^T and (X o X)^T per 32-row tile, and y padded.
__global__ void k_logreg_frags(const float *X, int ldx, const float *y, int N, int D, int MK, int nr,
                               float *xa, float *xta, float *x2ta, float *ypad)
{
    const int rt = blockIdx.x, lane = threadIdx.x, i = lane & 31, hh = lane >> 5;
    if (rt >= nr) return;
    for (int m = 0; m < MK; m++) {
        const int n = 32 * rt + i, d = 2 * m + hh;
        xa[((size_t)rt * MK + m) * 64 + lane] = (n < N && d < D) ? X[(size_t)n * ldx + d] : 0.f;
    }
    for (int m = 0; m < 16; m++) {
        const int n = 32 * rt + 2 * m + hh, d = i;
        const float v = (n < N && d < D) ? X[(size_t)n * ldx + d] : 0.f;
        xta[((size_t)rt * 16 + m) * 64 + lane] = v;
        x2ta[((size_t)rt * 16 + m) * 64 + lane] = v * v;
    }
    if (lane < 32) ypad[32 * rt + lane] = (32 * rt + lane < N) ? y[32 * rt + lane] : 0.f;
}

}  // namespace

pmc_status logreg_build_frags(pmc_context *ctx, DevTarget &t)
{
    const int nr = (t.n_data + 31) / 32, mk = (t.dim + 1) / 2;
    t.nr = nr;
    t.mk = mk <= 2 ? 2 : mk <= 4 ? 4 : mk <= 8 ? 8 : mk <= 13 ? 13 : 16;
    const size_t bxa = sizeof(float) * nr * t.mk * 64, bxt = sizeof(float) * nr * 16 * 64;
    PMC_TRY_HIP(hipMalloc(&t.xa, bxa));
    PMC_TRY_HIP(hipMalloc(&t.xta, bxt));
    PMC_TRY_HIP(hipMalloc(&t.x2ta, bxt));
    PMC_TRY_HIP(hipMalloc(&t.ypad, sizeof(float) * nr * 32));
    hipLaunchKernelGGL(k_logreg_frags, dim3(nr), dim3(64), 0, ctx->stream, (const float *)t.X, t.ldx,
                       (const float *)t.y, t.n_data, t.dim, t.mk, nr, (float *)t.xa, (float *)t.xta,
                       (float *)t.x2ta, (float *)t.ypad);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status launch_eval_logreg(pmc_context *ctx, const DevTarget &t, const EvalArgs &a)
{
    Frags f{(const float *)t.xa, (const float *)t.xta, (const float *)t.x2ta, (const float *)t.ypad,
            t.nr, (float)(1.0 / t.prior_var)};
    dim3 grid((a.n_tiles + kWaves - 1) / kWaves), block(64 * kWaves);
    switch (t.mk) {
    case 2: hipLaunchKernelGGL(k_eval_logreg<2>, grid, block, 0, ctx->stream, a, f); break;
    case 4: hipLaunchKernelGGL(k_eval_logreg<4>, grid, block, 0, ctx->stream, a, f); break;
    case 8: hipLaunchKernelGGL(k_eval_logreg<8>, grid, block, 0, ctx->stream, a, f); break;
    case 13: hipLaunchKernelGGL(k_eval_logreg<13>, grid, block, 0, ctx->stream, a, f); break;
    case 16: hipLaunchKernelGGL(k_eval_logreg<16>, grid, block, 0, ctx->stream, a, f); break;
    default: set_error("logreg eval: unsupported dimension"); return PMC_ERR_UNSUPPORTED;
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

}  // namespace pmc
