// Evaluation step for the Bayesian logistic-regression target on gfx950
// matrix cores.  For 32 consecutive steps (one wavefront) the per-step
// matrix-vector products of the MALA transition (Sec. 3.2) are batched into
// 32 x 32 x 2 FP32 matrix-core products over row tiles of 32 data points:
//   pass 1:  Z = X S            (linear predictors at s_{t-1}),
//            G = X^T (y - sigma(Z))              -> grad log-likelihood at s_{t-1}
//            Hd = (X o X)^T (sigma(Z)(1 - sigma(Z)))  -> minus the Hessian diagonal,
//   pass 2:  Z, dZ = X Delta    (predictors at s_{t-1} and their increment),
//            G~ = X^T (y - sigma(Z + dZ))        -> grad at the proposal,
//            sum_n log(1 + sigma(z) (e^dz - 1))  -> the softplus part of the
//            log-likelihood difference (its linear part is (X^T y) . Delta),
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

#include <algorithm>
#include <cmath>
#include <vector>

#include "logistic.hpp"
#include "pmc_internal.hpp"

namespace pmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
constexpr int kWaves = 4;

__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// With s = sigma(z), m = expm1(dz) and w = s m:
//   sigma(z + dz) = s (1 + m) / (1 + w),  softplus(z + dz) - softplus(z) = log1p(w);
// one exponential serves both.  Large increments (dz >= 30) take the direct forms.
__device__ __forceinline__ void shifted(float z, float dz, float s, float &st, float &spd)
{
    if (dz < 30.f) {
        const float m = expm1_s(dz);
        const float w = s * m;
        st = s * (1.f + m) * frcp(1.f + w);
        spd = log1p_s(w);
    } else {
        const float zt = z + dz;
        st = sigm(zt);
        spd = softplus(zt) - softplus(z);
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

// Same exchange with the gfx950 lane-half swap: the instruction exchanges
// the upper 32 lanes of its first operand with the lower 32 lanes of its
// second, which turns the pair (c[4g], c[4g+1]) into (b[4g], b[4g+2]) and
// (c[4g+2], c[4g+3]) into (b[4g+1], b[4g+3]).
__device__ __forceinline__ void acc_to_b_swap(const f32x16 &c, float (&b)[16])
{
#pragma unroll
    for (int g = 0; g < 4; g++) {
        const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[4 * g]),
                                                        __float_as_uint(c[4 * g + 1]), false, false);
        b[4 * g] = __uint_as_float(p[0]);
        b[4 * g + 2] = __uint_as_float(p[1]);
        const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[4 * g + 2]),
                                                        __float_as_uint(c[4 * g + 3]), false, false);
        b[4 * g + 1] = __uint_as_float(q[0]);
        b[4 * g + 3] = __uint_as_float(q[1]);
    }
}

// v(lane) + v(lane ^ 32), added in the same order in both halves.
__device__ __forceinline__ float half_sum(float v)
{
    const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(v), __float_as_uint(v), false, false);
    return __uint_as_float(p[0]) + __uint_as_float(p[1]);
}

// The FP64 form of half_sum (both 32-bit words exchanged).
__device__ __forceinline__ double half_sum_d(double v)
{
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const auto lo = __builtin_amdgcn_permlane32_swap((uint32_t)b, (uint32_t)b, false, false);
    const auto hi = __builtin_amdgcn_permlane32_swap((uint32_t)(b >> 32), (uint32_t)(b >> 32), false, false);
    const double a0 = __longlong_as_double((long long)(((uint64_t)hi[0] << 32) | lo[0]));
    const double a1 = __longlong_as_double((long long)(((uint64_t)hi[1] << 32) | lo[1]));
    return a0 + a1;
}

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// ------------------------------------------------ LDS-resident evaluation
// The data matrix (rows padded to 32, row stride kXS words, zero columns up
// to kXS) and y live in LDS, loaded once per workgroup; the workgroup's waves
// then take 32-step tiles round-robin until none is left.  A fragments are
// read from LDS in both layouts, so nothing but the iterate, the noise and
// the outputs touch global memory inside the loop.  The per-step epilogue
// works in the B layout (lane (i, hh) holds coordinates 2 m + hh of step i)
// and combines the two halves with lane swaps.  The Hessian diagonal, which
// only shapes the Jacobian approximation, is accumulated with BF16 matrix
// instructions whose contraction slots are assigned to the rows already held
// in the FP32 fragments (slot j of instruction kk, half hh <-> row
// 2 (8 kk + j) + hh).
constexpr int kXS = 33;
constexpr int kLdsWaves = 8;
constexpr int kLdsMaxRowTiles = 36;  // (36 * 32 * 34 + 32) * 4 bytes = 153 KiB

struct LdsArgs {
    const float *xl;  // [nr * 32 * kXS] padded X, [nr * 32] padded y, [32] X^T y
    int nr;
    float pp;
};

// Per-element work of pass 2 for increments |dz| < 8, free of branches:
// s = sigma(z), w = s (e^dz - 1), a = 1 + w gives
//   sigma(z + dz) = (s + w) / a,  softplus(z + dz) - softplus(z) = log(a),
// with one reciprocal of a serving the first; the callers multiply the a of
// four (FP32 products) or eight (split-FP16 products) elements, each within
// [e^-8, e^8], and take one logarithm of the product.  Everything downstream is an absolute-accuracy sum (the gradient
// X^T r and the log-likelihood difference), so e^dz - 1 is formed directly:
// its absolute error (one ulp of e^dz, carried through one fused
// multiply-add) is what the sums see either way.
// Arguments are u = z log2(e) and du = dz log2(e) (the LDS copy of X is
// scaled); returns y - sigma(z + dz) and a.
__device__ __forceinline__ float pass2_elem(float u, float du, float y, float &a)
{
    const float s = sigm2(u);
    const float w = fmaf(s, __builtin_amdgcn_exp2f(du), -s);  // s (e^dz - 1), one rounding
    a = 1.f + w;
    return fmaf(-(s + w), frcp(a), y);
}

// Per-step epilogue shared by the LDS-resident kernels (both lane halves hold
// the step; B layout, coordinate 2 m + hh in register m).  The log ratio is
// assembled in FP64: its terms (each up to ~10^2 on this posterior) cancel to
// O(1), and FP32 sums of them would add errors of ~10^-5 to a quantity
// compared against log u.  The linear part of the log-likelihood difference
// is (X^T y) . Delta; dll_s is the softplus part in log2 units; gsc[m] turns
// the accumulated proposal gradient into natural units.
template <int MK>
__device__ __forceinline__ void finish_step(const EvalArgs &a, const float *s_xty, const f32x16 &Gt, double dll_s,
                                            const float (&SB)[MK], const float (&DB)[MK], const float (&gB)[MK],
                                            const float (&gsc)[MK], float pp, int hh, int64_t ld, int64_t t,
                                            int64_t tt, bool valid, bool want_j, float damp, float clip,
                                            const ChainStatus &cs)
{
    const int D = a.D;
    const float *noise = (const float *)a.noise;
    float *F = (float *)a.F, *J = (float *)a.J;
    double dll_y = 0.0;
#pragma unroll
    for (int m = 0; m < MK; m++) dll_y = fma((double)s_xty[2 * m + hh], (double)DB[m], dll_y);
    const double dll = half_sum_d(fma(-dll_s, (double)kLn2, dll_y));

    float GtB[16];
    acc_to_b_swap(Gt, GtB);
    double sn = 0.0, sx = 0.0, dpr = 0.0;
#pragma unroll
    for (int m = 0; m < MK; m++) {
        const int d = 2 * m + hh;
        if (d < D) {
            const float x = SB[m], dl = DB[m], xt = x + dl;
            const float gt = fmaf(GtB[m], gsc[m], -pp * xt);
            const double sg = (double)gB[m] + (double)gt;
            sn = fma(sg, sg, sn);
            sx = fma((double)noise[(size_t)tt * D + d], sg, sx);
            dpr = fma((double)dl, (double)xt + (double)x, dpr);
        }
    }
    sn = half_sum_d(sn);
    sx = half_sum_d(sx);
    dpr = half_sum_d(dpr);
    if (!valid) return;
    int acc = 1;
    float gate = INFINITY;
    if (!a.ula) {
        const double ell = dll - 0.5 * (double)pp * dpr - 0.25 * a.eps * sn - sqrt(0.5 * a.eps) * sx;
        const double la = ell < 0.0 ? ell : 0.0;
        const double gd = la - log((double)((const float *)a.unif)[t]);
        gate = (float)gd;
        acc = gd > 0.0;
        if (!(ell == ell)) acc = 0;
        acc = sticky_decision(a, cs, t, gd, acc);
    }
    float jrej = damp;
    if (clip > 0) jrej = fminf(fmaxf(jrej, -clip), clip);
#pragma unroll
    for (int m = 0; m < MK; m++) {
        const int d = 2 * m + hh;
        if (d < D) {
            F[(size_t)d * ld + t] = acc ? SB[m] + DB[m] : SB[m];
            if (want_j && !acc) J[(size_t)d * ld + t] = jrej;
        }
    }
    if (hh == 0) {
        if (a.accept) a.accept[t] = (uint8_t)acc;
        if (a.gtilde) a.gtilde[t] = gate;
    }
}

template <int MK>
__device__ __forceinline__ f32x16 z_chain(const float *xr, int i, int hh, const float (&v)[MK])
{
    f32x16 Z = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int m = 0; m < MK; m++) Z = __builtin_amdgcn_mfma_f32_32x32x2f32(xr[i * kXS + 2 * m + hh], v[m], Z, 0, 0, 0);
    return Z;
}

template <int MK>
__global__ void __launch_bounds__(64 * kLdsWaves, 2) k_eval_logreg_lds(EvalArgs a, LdsArgs f)
{
    extern __shared__ float s_x[];
    if (a.glob && !eval_has_chains(a)) return;  // a sweep queued past the last active chain
    const int nrow = f.nr * 32;
    {
        const int nw = nrow * (kXS + 1) + 32;
        const float4 *src = (const float4 *)f.xl;
        float4 *dst = (float4 *)s_x;
        for (int k = threadIdx.x; k < nw / 4; k += blockDim.x) dst[k] = src[k];
    }
    __syncthreads();
    const float *s_y = s_x + nrow * kXS;
    const float *s_xty = s_y + nrow;
    const int lane = threadIdx.x & 63, i = lane & 31, hh = lane >> 5;
    const int D = a.D, nr = f.nr;
    const int64_t ld = a.ld;
    const float *S = (const float *)a.S, *noise = (const float *)a.noise;
    float *J = (float *)a.J;
    const float eps = (float)a.eps, c = sqrtf(2.f * eps), pp = f.pp;
    const float damp = (float)a.damping, clip = (float)a.clip;
    const bool want_j = a.jmode == JM_DIAG && !a.probes;  // probes: launch_logreg_probe_diag writes J
    const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};

    // tiles are dealt to waves round-robin (tile costs are uniform; the idle
    // prefix of a sliding window spreads over all waves)
    const int n_waves = gridDim.x * kLdsWaves;
    for (int tix = blockIdx.x * kLdsWaves + (threadIdx.x >> 6); tix < a.n_tiles; tix += n_waves) {
        const SegTile tl = a.tiles[tix];
        const ChainStatus &cs = a.chains[tl.chain];
        if (!cs.active || !eval_takes(a, cs) || tl.start + tl.len <= cs.win_start || tl.start >= cs.win_end)
            continue;
        const int64_t t = tl.start + i;
        const bool valid = i < tl.len && t >= cs.win_start && t < cs.win_end;
        const int64_t tt = i < tl.len ? t : tl.start;
        const bool head = (tt == a.offsets[tl.chain]);
        const float *s0 = (const float *)a.s0 + (size_t)tl.chain * D;

        float SB[MK];
#pragma unroll
        for (int m = 0; m < MK; m++) {
            const int d = 2 * m + hh;
            SB[m] = d < D ? (head ? s0[d] : S[(size_t)d * ld + tt - 1]) : 0.f;
        }

        // ---- pass 1: gradient and Hessian diagonal of the log-likelihood at
        // s_{t-1}.  Software-pipelined over row tiles: iteration rt issues the
        // predictors of tile rt + 1 and the gradient / Hessian products of
        // tile rt - 1 on the matrix cores while the vector units work on the
        // sigmoids of tile rt (the group barriers ask the scheduler to
        // interleave the two instruction streams).
        f32x16 G = zero, Hd = zero;
        f32x16 Zc = z_chain<MK>(s_x, i, hh, SB);
        float RBp[16], XTp[16];
        bf16x8 Wp[2];
#pragma unroll
        for (int m = 0; m < 16; m++) {
            RBp[m] = 0.f;
            XTp[m] = 0.f;
        }
#pragma unroll
        for (int j = 0; j < 8; j++) Wp[0][j] = Wp[1][j] = (__bf16)0.f;
        for (int rt = 0; rt < nr; rt++) {
            const int rn = rt + 1 < nr ? rt + 1 : rt;
            const f32x16 Zn = z_chain<MK>(s_x + (32 * rn) * kXS, i, hh, SB);
#pragma unroll
            for (int m = 0; m < 16; m++) G = __builtin_amdgcn_mfma_f32_32x32x2f32(XTp[m], RBp[m], G, 0, 0, 0);
#pragma unroll
            for (int kk = 0; kk < 2; kk++) {
                bf16x8 A;
#pragma unroll
                for (int j = 0; j < 8; j++) A[j] = (__bf16)(XTp[8 * kk + j] * XTp[8 * kk + j]);
                Hd = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Wp[kk], Hd, 0, 0, 0);
            }
            const float *xr = s_x + (32 * rt) * kXS;
            const float4 *y4 = (const float4 *)(s_y + 32 * rt + 4 * hh);
            f32x16 R, Wv;
#pragma unroll
            for (int g = 0; g < 4; g++) {
                const float4 y4v = y4[2 * g];
                const float yv[4] = {y4v.x, y4v.y, y4v.z, y4v.w};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const float sv = sigm2(Zc[4 * g + q]);
                    R[4 * g + q] = yv[q] - sv;
                    Wv[4 * g + q] = fmaf(-sv, sv, sv);
                }
            }
#pragma unroll
            for (int m = 0; m < 16; m++) XTp[m] = xr[(2 * m + hh) * kXS + i];
            acc_to_b_swap(R, RBp);
            {
                float WB[16];
                acc_to_b_swap(Wv, WB);
#pragma unroll
                for (int kk = 0; kk < 2; kk++)
#pragma unroll
                    for (int j = 0; j < 8; j++) Wp[kk][j] = (__bf16)WB[8 * kk + j];
            }
            Zc = Zn;
#pragma unroll
            for (int k = 0; k < MK + 18; k++) {
                __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);  // one matrix instruction
                __builtin_amdgcn_sched_group_barrier(0x002, 6, 0);  // then vector work
            }
        }
#pragma unroll
        for (int m = 0; m < 16; m++) G = __builtin_amdgcn_mfma_f32_32x32x2f32(XTp[m], RBp[m], G, 0, 0, 0);
#pragma unroll
        for (int kk = 0; kk < 2; kk++) {
            bf16x8 A;
#pragma unroll
            for (int j = 0; j < 8; j++) A[j] = (__bf16)(XTp[8 * kk + j] * XTp[8 * kk + j]);
            Hd = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, Wp[kk], Hd, 0, 0, 0);
        }
        // gradient at s_{t-1}, the proposal increment, and the Jacobian
        // diagonal for an accepted step (rejected steps rewrite it below)
        float gB[MK], DB[MK];
        {
            float GB[16], HB[16];
            acc_to_b_swap(G, GB);
            acc_to_b_swap(Hd, HB);
#pragma unroll
            for (int m = 0; m < MK; m++) {
                const int d = 2 * m + hh;
                gB[m] = fmaf(GB[m], kLn2, -pp * SB[m]);
                DB[m] = d < D ? fmaf(eps, gB[m], c * noise[(size_t)tt * D + d]) : 0.f;
                if (want_j && valid && d < D) {
                    float jv = damp * fmaf(eps, fmaf(-HB[m], kLn2 * kLn2, -pp), 1.f);
                    if (clip > 0) jv = fminf(fmaxf(jv, -clip), clip);
                    J[(size_t)d * ld + t] = jv;
                }
            }
        }

        // ---- pass 2: gradient at the proposal and log-likelihood difference.
        // Row tile rt is processed in four groups of four accumulator rows;
        // group g also issues the gradient products of tile rt - 1 that use
        // the B rows 4g..4g+3 (whose registers it then refills with tile
        // rt's values) and a share of the predictor chains of tile rt + 1,
        // so matrix and vector work interleave with few live registers.
        // A group holding an element with |dz| >= 8 is redone by a rare
        // direct path.  The softplus sums are kept in log2 units, one FP32
        // partial per row tile added into an FP64 total.
        f32x16 Gt = zero;
        double dll_s = 0.0;
        Zc = z_chain<MK>(s_x, i, hh, SB);
        f32x16 dZc = z_chain<MK>(s_x, i, hh, DB);
        float RtB[16];
#pragma unroll
        for (int m = 0; m < 16; m++) RtB[m] = 0.f;
        for (int rt = 0; rt < nr; rt++) {
            const int rn = rt + 1 < nr ? rt + 1 : rt;
            const float *xn = s_x + (32 * rn) * kXS;
            const float *xp = s_x + (32 * (rt > 0 ? rt - 1 : 0)) * kXS;
            const float *yr = s_y + 32 * rt + 4 * hh;
            f32x16 Zn = zero, dZn = zero;
            float tile_s = 0.f;
#pragma unroll
            for (int g = 0; g < 4; g++) {
#pragma unroll
                for (int m = 4 * g; m < 4 * g + 4; m++)
                    Gt = __builtin_amdgcn_mfma_f32_32x32x2f32(xp[(2 * m + hh) * kXS + i], RtB[m], Gt, 0, 0, 0);
                constexpr int per = (MK + 3) / 4;
#pragma unroll
                for (int m = per * g; m < per * (g + 1) && m < MK; m++) {
                    const float a1 = xn[i * kXS + 2 * m + hh];
                    Zn = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, SB[m], Zn, 0, 0, 0);
                    dZn = __builtin_amdgcn_mfma_f32_32x32x2f32(a1, DB[m], dZn, 0, 0, 0);
                }
                const float4 y4v = *(const float4 *)(yr + 8 * g);
                const float yv[4] = {y4v.x, y4v.y, y4v.z, y4v.w};
                float Rt[4], av[4];
                bool wide = false;
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const float du = dZc[4 * g + q];
                    Rt[q] = pass2_elem(Zc[4 * g + q], du, yv[q], av[q]);
                    wide |= !(fabsf(du) < 8.f * kLog2e);
                }
                float lg = __builtin_amdgcn_logf((av[0] * av[1]) * (av[2] * av[3]));
                if (__builtin_amdgcn_ballot_w64(wide)) {  // rare
                    if (wide) {
                        lg = 0.f;
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            const float u = Zc[4 * g + q], du = dZc[4 * g + q];
                            if (fabsf(du) < 8.f * kLog2e) {
                                lg += __builtin_amdgcn_logf(av[q]);
                            } else {
                                const float z = u * kLn2, zt = z + du * kLn2;
                                Rt[q] = yv[q] - sigm(zt);
                                lg += (softplus(zt) - softplus(z)) * kLog2e;
                            }
                        }
                    }
                }
                tile_s += lg;
                // accumulator rows 4g..4g+3 -> B rows 4g, 4g+2, 4g+1, 4g+3
                const auto p0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(Rt[0]), __float_as_uint(Rt[1]),
                                                                 false, false);
                const auto p1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(Rt[2]), __float_as_uint(Rt[3]),
                                                                 false, false);
                RtB[4 * g] = __uint_as_float(p0[0]);
                RtB[4 * g + 2] = __uint_as_float(p0[1]);
                RtB[4 * g + 1] = __uint_as_float(p1[0]);
                RtB[4 * g + 3] = __uint_as_float(p1[1]);
            }
            dll_s += (double)tile_s;
            Zc = Zn;
            dZc = dZn;
        }
        {
            const float *xp = s_x + (32 * (nr - 1)) * kXS;
#pragma unroll
            for (int m = 0; m < 16; m++)
                Gt = __builtin_amdgcn_mfma_f32_32x32x2f32(xp[(2 * m + hh) * kXS + i], RtB[m], Gt, 0, 0, 0);
        }
        float gsc[MK];
#pragma unroll
        for (int m = 0; m < MK; m++) gsc[m] = kLn2;
        finish_step<MK>(a, s_xty, Gt, dll_s, SB, DB, gB, gsc, pp, hh, ld, t, tt, valid, want_j, damp, clip, cs);
    }
}

// ------------------------------------------ split-FP16 matrix-core evaluation
// The same evaluation with every product formed on the FP16 matrix cores
// (32 x 32 x 16 per instruction, FP32 accumulation) from a two-term split of
// each operand: v = hi + lo with hi = fp16(v) and lo = fp16(v - hi), both
// rounded to nearest, and
//   A B ~ A_lo B_hi + A_hi B_lo + A_hi B_hi
// (the error-compensated half-precision product of Markidis et al. 2018 and
// Ootomo & Yokota 2022; the dropped A_lo B_lo and the rounding of lo leave
// about 2^-22 of each product, and each instruction adds 16 products before
// it rounds into the accumulator).  An FP16 instruction does 16x the work of
// an FP32 one in half the cycles, so the three terms cost about a sixth of
// the FP32 products.
//
// LDS image (written once per target, copied into LDS per workgroup): the hi
// and lo planes of X log2(e) as FP16, 32 entries per row, then y and X^T y in
// FP32.  Coordinates and rows are stored in the orders the two products read:
//   Z = X S:      lane (i, hh), slot j of contraction block kk reads row i,
//                 coordinate d = 16 kk + 2 j + hh, stored at column
//                 16 kk + 8 hh + j, so a lane's eight slots are one 16-byte read;
//                 the B operand is then s[2 m + hh] with m = 8 kk + j, which is
//                 the epilogue's register order.
//   G = X^T R:    lane (d = i, hh), slot j of block kk pairs with accumulator
//                 register 8 kk + j of R, that is row crow(8 kk + j, hh) of the
//                 tile, stored at position 16 kk + 2 j + hh, so R is an operand
//                 without any exchange between lanes, and the two lane halves
//                 read rows one position apart (distinct LDS banks).
// Operand ranges.  FP16 keeps 11 significant bits only down to 2^-14, so
// every operand is brought to a known range by exact power-of-two scalings
// before it is split: column d of X log2(e) is stored times 2^e_d with its
// largest entry in [4, 8) (the Hessian weights use hi^2 < 2^6), and the image
// carries c_d = 2^-e_d; the iterate and the increment enter as s_d c_d and
// Delta_d c_d, so X S and X Delta need no correction, and the gradients come
// out per coordinate times 2^e_d.  Per 32-step tile the scaled increment is
// taken to a maximum in [2^13, 2^14) and the scaled iterate, when its maximum
// lies outside [2^-3, 2^14), to the same range (both undone on the products).
// The residuals R lie in [-1, 1].  Entries far below their operand's maximum
// keep an absolute error of about 2^-25 of the scaled unit, far below the
// rounding of the largest terms.
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef float f32x2 __attribute__((ext_vector_type(2)));

constexpr int kHW = 32;               // FP16 entries per image row
constexpr int kHMaxRowTiles = 38;     // 38 * 4224 + 256 bytes = 157 KiB

// hi plane, lo plane, y (FP32), X^T y (32 FP32), c_d (32 FP32)
constexpr size_t kHImageBytes(int nr) { return (size_t)nr * 32 * (4 * kHW + 4) + 2 * 32 * 4; }

// storage column of coordinate d, storage position of tile row r
__host__ __device__ constexpr int h_col(int d) { return (d & 16) | ((d & 1) << 3) | ((d >> 1) & 7); }
__host__ __device__ constexpr int h_row(int r) { return (r & ~7) | ((r & 3) << 1) | ((r >> 2) & 1); }

struct HArgs {
    const void *img;  // kHImageBytes(nr) bytes, layout above
    int nr;
    float pp;
};

// x - hi for hi in the low or high half of a packed FP16 pair: one
// mixed-precision fused multiply-add (hi widened exactly; the difference is
// exact in FP32)
__device__ __forceinline__ float sub_f16_lo(uint32_t hp, float x)
{
    float r;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel_hi:[1,0,0]" : "=v"(r) : "v"(hp), "v"(x));
    return r;
}
__device__ __forceinline__ float sub_f16_hi(uint32_t hp, float x)
{
    float r;
    asm("v_fma_mix_f32 %0, %1, -1.0, %2 op_sel:[1,0,0] op_sel_hi:[1,0,0]" : "=v"(r) : "v"(hp), "v"(x));
    return r;
}

// v = hi + lo, both FP16 rounded to nearest
__device__ __forceinline__ void split8(const float (&v)[8], f16x8 &h, f16x8 &l)
{
#pragma unroll
    for (int j = 0; j < 8; j += 2) {
        const f32x2 x = {v[j], v[j + 1]};
        const f16x2 hp = __builtin_convertvector(x, f16x2);
        const uint32_t hb = __builtin_bit_cast(uint32_t, hp);
        const f32x2 r = {sub_f16_lo(hb, v[j]), sub_f16_hi(hb, v[j + 1])};
        const f16x2 lp = __builtin_convertvector(r, f16x2);
        h[j] = hp[0];
        h[j + 1] = hp[1];
        l[j] = lp[0];
        l[j + 1] = lp[1];
    }
}

__device__ __forceinline__ f32x16 mfma3(const f16x8 &ah, const f16x8 &al, const f16x8 &bh, const f16x8 &bl,
                                        f32x16 c)
{
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(al, bh, c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bl, c, 0, 0, 0);
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(ah, bh, c, 0, 0, 0);
}

// A operand of G = X^T R for block kk of a row tile: rows 16 kk + 2 j + hh
// (storage order), column h_col(d)
__device__ __forceinline__ f16x8 g_operand(const _Float16 *plane, int base)
{
    f16x8 v;
#pragma unroll
    for (int j = 0; j < 8; j++) v[j] = plane[base + 2 * kHW * j];
    return v;
}

__device__ __forceinline__ float wave_max(float v)
{
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}

// the MK entries of a B-layout vector (m = 8 kk + j), scaled by 2^e, as KB
// split operands
template <int MK, int KB>
__device__ __forceinline__ void split_b(const float (&v)[MK], int e, f16x8 (&h)[KB], f16x8 (&l)[KB])
{
#pragma unroll
    for (int kk = 0; kk < KB; kk++) {
        float w[8];
#pragma unroll
        for (int j = 0; j < 8; j++) w[j] = 8 * kk + j < MK ? ldexpf(v[8 * kk + j], e) : 0.f;
        split8(w, h[kk], l[kk]);
    }
}

template <int MK>
__global__ void __launch_bounds__(64 * kLdsWaves, 1) k_eval_logreg_h(EvalArgs a, HArgs f)
{
    constexpr int KB = MK > 8 ? 2 : 1;
    extern __shared__ float4 s_img[];
    if (a.glob && !eval_has_chains(a)) return;  // a sweep queued past the last active chain
    const int nrow = f.nr * 32;
    {
        const int n4 = (int)(kHImageBytes(f.nr) / 16);
        const float4 *src = (const float4 *)f.img;
        for (int k = threadIdx.x; k < n4; k += blockDim.x) s_img[k] = src[k];
    }
    __syncthreads();
    const _Float16 *s_hi = (const _Float16 *)s_img;
    const _Float16 *s_lo = s_hi + nrow * kHW;
    const float *s_y = (const float *)(s_lo + nrow * kHW);
    const float *s_xty = s_y + nrow;
    const int lane = threadIdx.x & 63, i = lane & 31, hh = lane >> 5;
    const int D = a.D, nr = f.nr;
    const int64_t ld = a.ld;
    const float *S = (const float *)a.S, *noise = (const float *)a.noise;
    float *J = (float *)a.J, *F = (float *)a.F;
    const float *s_csc = s_xty + 32;  // c_d
    const float eps = (float)a.eps, c = sqrtf(2.f * eps), pp = f.pp;
    const float damp = (float)a.damping, clip = (float)a.clip;
    const bool want_j = a.jmode == JM_DIAG && !a.probes;  // probes: launch_logreg_probe_diag writes J
    const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // per-lane offsets: the Z operand row (storage order) and the G operand column
    const int zoff = h_row(i) * kHW + 8 * hh;
    const int goff = hh * kHW + h_col(i);

    const int n_waves = gridDim.x * kLdsWaves;
    for (int tix = blockIdx.x * kLdsWaves + (threadIdx.x >> 6); tix < a.n_tiles; tix += n_waves) {
        const SegTile tl = a.tiles[tix];
        const ChainStatus &cs = a.chains[tl.chain];
        if (!cs.active || !eval_takes(a, cs) || tl.start + tl.len <= cs.win_start || tl.start >= cs.win_end)
            continue;
        const int64_t t = tl.start + i;
        const bool valid = i < tl.len && t >= cs.win_start && t < cs.win_end;
        const int64_t tt = i < tl.len ? t : tl.start;
        const bool head = (tt == a.offsets[tl.chain]);
        const float *s0 = (const float *)a.s0 + (size_t)tl.chain * D;

        // the iterate s_{t-1} in the B layout; loaded where it is used (after
        // pass 1 and in the epilogue) rather than held through both passes,
        // which keeps the kernel within its 256 registers
        auto sb = [&](int m) -> float {
            const int d = 2 * m + hh;
            return d < D ? (head ? s0[d] : S[(size_t)d * ld + tt - 1]) : 0.f;
        };
        float SC[MK];
        float smax = 0.f;
#pragma unroll
        for (int m = 0; m < MK; m++) {
            SC[m] = sb(m) * s_csc[2 * m + hh];
            smax = fmaxf(smax, fabsf(SC[m]));
        }
        // scaled iterate outside [2^-3, 2^14): taken to [2^13, 2^14) (Z undone by 2^-es)
        smax = wave_max(smax);
        const int es = __builtin_amdgcn_readfirstlane(
            (smax >= 16384.f || smax < 0.125f) && smax > 0.f && smax < INFINITY ? 13 - ilogbf(smax) : 0);
        f16x8 Sh[KB], Sl[KB];
        split_b<MK, KB>(SC, es, Sh, Sl);

        // ---- pass 1: gradient and Hessian diagonal at s_{t-1}; iteration rt
        // issues the predictors of tile rt + 1 and the products of tile rt - 1
        // around the sigmoids of tile rt.
        f32x16 G = zero, Hd = zero;
        f32x16 Zc = zero;
#pragma unroll
        for (int kk = 0; kk < KB; kk++)
            Zc = mfma3(*(const f16x8 *)(s_hi + zoff + 16 * kk), *(const f16x8 *)(s_lo + zoff + 16 * kk), Sh[kk],
                       Sl[kk], Zc);
        if (es)
#pragma unroll
            for (int r = 0; r < 16; r++) Zc[r] = ldexpf(Zc[r], -es);
        f16x8 Rh[2], Rl[2], Wh[2], Xh[2], Xl[2];
#pragma unroll
        for (int kk = 0; kk < 2; kk++)
#pragma unroll
            for (int j = 0; j < 8; j++) Rh[kk][j] = Rl[kk][j] = Wh[kk][j] = Xh[kk][j] = Xl[kk][j] = (_Float16)0.f;
        for (int rt = 0; rt < nr; rt++) {
            const int rn = rt + 1 < nr ? rt + 1 : rt;
            f32x16 Zn = zero;
#pragma unroll
            for (int kk = 0; kk < KB; kk++) {
                const int o = (32 * rn) * kHW + zoff + 16 * kk;
                Zn = mfma3(*(const f16x8 *)(s_hi + o), *(const f16x8 *)(s_lo + o), Sh[kk], Sl[kk], Zn);
            }
#pragma unroll
            for (int kk = 0; kk < 2; kk++) {
                G = mfma3(Xh[kk], Xl[kk], Rh[kk], Rl[kk], G);
                Hd = __builtin_amdgcn_mfma_f32_32x32x16_f16(Xh[kk] * Xh[kk], Wh[kk], Hd, 0, 0, 0);
            }
            const float4 *y4 = (const float4 *)(s_y + 32 * rt + 4 * hh);
            float Rv[16], Wv[16];
#pragma unroll
            for (int g = 0; g < 4; g++) {
                const float4 y4v = y4[2 * g];
                const float yv[4] = {y4v.x, y4v.y, y4v.z, y4v.w};
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    const float sv = sigm2(Zc[4 * g + q]);
                    Rv[4 * g + q] = yv[q] - sv;
                    Wv[4 * g + q] = fmaf(-sv, sv, sv);
                }
            }
#pragma unroll
            for (int kk = 0; kk < 2; kk++) {
                float r8[8], w8[8];
#pragma unroll
                for (int j = 0; j < 8; j++) {
                    r8[j] = Rv[8 * kk + j];
                    w8[j] = Wv[8 * kk + j];
                }
                split8(r8, Rh[kk], Rl[kk]);
#pragma unroll
                for (int j = 0; j < 8; j += 2) {
                    const f32x2 x = {w8[j], w8[j + 1]};
                    const f16x2 hp = __builtin_convertvector(x, f16x2);
                    Wh[kk][j] = hp[0];
                    Wh[kk][j + 1] = hp[1];
                }
                const int o = (32 * rt + 16 * kk) * kHW + goff;
                Xh[kk] = g_operand(s_hi, o);
                Xl[kk] = g_operand(s_lo, o);
            }
            if (es)
#pragma unroll
                for (int r = 0; r < 16; r++) Zn[r] = ldexpf(Zn[r], -es);
            Zc = Zn;
        }
#pragma unroll
        for (int kk = 0; kk < 2; kk++) {
            G = mfma3(Xh[kk], Xl[kk], Rh[kk], Rl[kk], G);
            Hd = __builtin_amdgcn_mfma_f32_32x32x16_f16(Xh[kk] * Xh[kk], Wh[kk], Hd, 0, 0, 0);
        }
        float gB[MK], DB[MK], DC[MK];
        float dmax = 0.f;
        {
            float GB[16], HB[16];
            acc_to_b_swap(G, GB);
            acc_to_b_swap(Hd, HB);
#pragma unroll
            for (int m = 0; m < MK; m++) {
                const int d = 2 * m + hh;
                const float cd = s_csc[2 * m + hh], gs = kLn2 * cd;
                gB[m] = fmaf(GB[m], gs, -pp * sb(m));
                DB[m] = d < D ? fmaf(eps, gB[m], c * noise[(size_t)tt * D + d]) : 0.f;
                // the gradient waits for the epilogue in this step's F slot
                // (written there at the end), not in registers through pass 2
                if (valid && d < D) F[(size_t)d * ld + t] = gB[m];
                DC[m] = DB[m] * cd;
                dmax = fmaxf(dmax, fabsf(DC[m]));
                if (want_j && valid && d < D) {
                    float jv = damp * fmaf(eps, fmaf(-HB[m], gs * gs, -pp), 1.f);
                    if (clip > 0) jv = fminf(fmaxf(jv, -clip), clip);
                    J[(size_t)d * ld + t] = jv;
                }
            }
        }
        // the increment is scaled to a maximum in [2^13, 2^14) before it is split
        dmax = wave_max(dmax);
        const int ed = __builtin_amdgcn_readfirstlane(dmax > 0.f && dmax < INFINITY ? 13 - ilogbf(dmax) : 0);
        const float dsc = ldexpf(1.f, -ed);
        f16x8 Dh[KB], Dl[KB];
        split_b<MK, KB>(DC, ed, Dh, Dl);

        // ---- pass 2: gradient at the proposal and the log-likelihood
        // difference.  Block kk of row tile rt issues the proposal-gradient
        // products of tile rt - 1 that use R~ registers 8 kk .. 8 kk + 7
        // (then refilled with tile rt's values) and block kk of the predictor
        // chains of tile rt + 1.
        f32x16 Gt = zero;
        double dll_s = 0.0;
        Zc = zero;
        f32x16 dZc = zero;
#pragma unroll
        for (int kk = 0; kk < KB; kk++) {
            const f16x8 ah = *(const f16x8 *)(s_hi + zoff + 16 * kk), al = *(const f16x8 *)(s_lo + zoff + 16 * kk);
            Zc = mfma3(ah, al, Sh[kk], Sl[kk], Zc);
            dZc = mfma3(ah, al, Dh[kk], Dl[kk], dZc);
        }
        if (es)
#pragma unroll
            for (int r = 0; r < 16; r++) Zc[r] = ldexpf(Zc[r], -es);
        f16x8 Th[2], Tl[2];
#pragma unroll
        for (int kk = 0; kk < 2; kk++)
#pragma unroll
            for (int j = 0; j < 8; j++) Th[kk][j] = Tl[kk][j] = (_Float16)0.f;
        for (int rt = 0; rt < nr; rt++) {
            const int rn = rt + 1 < nr ? rt + 1 : rt, rp = rt > 0 ? rt - 1 : 0;
            const float *yr = s_y + 32 * rt + 4 * hh;
            f32x16 Zn = zero, dZn = zero;
            float tile_s = 0.f;
#pragma unroll
            for (int kk = 0; kk < 2; kk++) {
                {
                    const int o = (32 * rp + 16 * kk) * kHW + goff;
                    Gt = mfma3(g_operand(s_hi, o), g_operand(s_lo, o), Th[kk], Tl[kk], Gt);
                }
                if (kk < KB) {
                    const int o = (32 * rn) * kHW + zoff + 16 * kk;
                    const f16x8 ah = *(const f16x8 *)(s_hi + o), al = *(const f16x8 *)(s_lo + o);
                    Zn = mfma3(ah, al, Sh[kk], Sl[kk], Zn);
                    dZn = mfma3(ah, al, Dh[kk], Dl[kk], dZn);
                }
                // accumulator registers 8 kk .. 8 kk + 7; the a of all eight
                // (each within [e^-8, e^8]) share one logarithm
                float r8[8], av[8];
                bool wide = false;
#pragma unroll
                for (int gg = 0; gg < 2; gg++) {
                    const float4 y4v = *(const float4 *)(yr + 8 * (2 * kk + gg));
                    const float yv[4] = {y4v.x, y4v.y, y4v.z, y4v.w};
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        const int r = 8 * kk + 4 * gg + q;
                        const float du = dZc[r] * dsc;
                        r8[4 * gg + q] = pass2_elem(Zc[r], du, yv[q], av[4 * gg + q]);
                        wide |= !(fabsf(du) < 8.f * kLog2e);
                    }
                }
                float lg = __builtin_amdgcn_logf(((av[0] * av[1]) * (av[2] * av[3])) *
                                                 ((av[4] * av[5]) * (av[6] * av[7])));
                if (__builtin_amdgcn_ballot_w64(wide)) {  // rare
                    if (wide) {
                        lg = 0.f;
#pragma unroll
                        for (int q = 0; q < 8; q++) {
                            const int r = 8 * kk + q;
                            const float u = Zc[r], du = dZc[r] * dsc;
                            if (fabsf(du) < 8.f * kLog2e) {
                                lg += __builtin_amdgcn_logf(av[q]);
                            } else {
                                const float yq = yr[8 * (2 * kk + (q >> 2)) + (q & 3)];
                                const float z = u * kLn2, zt = z + du * kLn2;
                                r8[q] = yq - sigm(zt);
                                lg += (softplus(zt) - softplus(z)) * kLog2e;
                            }
                        }
                    }
                }
                tile_s += lg;
                split8(r8, Th[kk], Tl[kk]);
            }
            dll_s += (double)tile_s;
            if (es)
#pragma unroll
                for (int r = 0; r < 16; r++) Zn[r] = ldexpf(Zn[r], -es);
            Zc = Zn;
            dZc = dZn;
        }
#pragma unroll
        for (int kk = 0; kk < 2; kk++) {
            const int o = (32 * (nr - 1) + 16 * kk) * kHW + goff;
            Gt = mfma3(g_operand(s_hi, o), g_operand(s_lo, o), Th[kk], Tl[kk], Gt);
        }
        // (the compiler must not carry the stashed gradient in registers
        // through pass 2: an empty asm statement that clobbers memory makes
        // the loads below real)
        asm volatile("" ::: "memory");
        float gsc[MK], SB[MK];
#pragma unroll
        for (int m = 0; m < MK; m++) {
            const int d = 2 * m + hh;
            gsc[m] = kLn2 * s_csc[2 * m + hh];
            SB[m] = sb(m);
            gB[m] = valid && d < D ? F[(size_t)d * ld + t] : 0.f;
            // the increment again, from the same operands (bit for bit)
            DB[m] = d < D ? fmaf(eps, gB[m], c * noise[(size_t)tt * D + d]) : 0.f;
        }
        finish_step<MK>(a, s_xty, Gt, dll_s, SB, DB, gB, gsc, pp, hh, ld, t, tt, valid, want_j, damp, clip, cs);
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
    if (!cs.active || tl.start + tl.len <= cs.win_start || tl.start >= cs.win_end) return;
    const int64_t t = tl.start + j;
    const bool valid = j < tl.len && t >= cs.win_start && t < cs.win_end;
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
    double dll = 0.0;  // FP32 partial per row tile, FP64 total
    for (int rt = 0; rt < f.nr; rt++) {
        float dtile = 0.f;
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
            dtile += yv * dz - spd;
        }
        dll += (double)dtile;
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
    dll += __shfl_xor(dll, 32, 64);  // the two halves in the same order on both
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (hh != 0 || !valid) return;

    // ---- one lane per step: log ratio (assembled in FP64 from the FP32
    // products, as in the LDS-resident kernel), decision, f_t, Jacobian diagonal
    double sn = 0.0, sx = 0.0, dpr = 0.0;
    for (int d = 0; d < D; d++) {
        const float x = head ? s0[d] : S[(size_t)d * ld + t - 1];
        const float xi = noise[(size_t)t * D + d];
        const float g = sg[d * 33 + j] - pp * x;
        const float dl = fmaf(eps, g, c * xi);
        const float xt = x + dl;
        const float gt = sgt[d * 33 + j] - pp * xt;
        const double s = (double)g + (double)gt;
        sn = fma(s, s, sn);
        sx = fma((double)xi, s, sx);
        dpr = fma((double)dl, (double)xt + (double)x, dpr);
    }
    int acc = 1;
    float gate = INFINITY;
    if (!a.ula) {
        const double ell = dll - 0.5 * (double)pp * dpr - 0.25 * a.eps * sn - sqrt(0.5 * a.eps) * sx;
        const double la = ell < 0.0 ? ell : 0.0;
        const double gd = la - log((double)((const float *)a.unif)[t]);
        gate = (float)gd;
        acc = gd > 0.0;
        if (!(ell == ell)) acc = 0;
        acc = sticky_decision(a, cs, t, gd, acc);
    }
    float *F = (float *)a.F;
    float *J = (float *)a.J;
    const float ea = acc ? eps : 0.f;
    for (int d = 0; d < D; d++) {
        const float x = head ? s0[d] : S[(size_t)d * ld + t - 1];
        const float g = sg[d * 33 + j] - pp * x;
        const float xt = x + fmaf(eps, g, c * noise[(size_t)t * D + d]);
        F[(size_t)d * ld + t] = acc ? xt : x;
        if (a.jmode == JM_DIAG && !a.probes) {
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


// LDS image: X log2(e) (predictor products then come out as arguments of
// exp2; the gradient and Hessian sums are rescaled by ln 2 and ln^2 2), rows
// padded to nr * 32, row stride kXS, zero columns beyond D, followed by y
// padded with zeros and by X^T y (32 entries, filled by k_logreg_xty).
__global__ void k_logreg_lds_image(const float *X, int ldx, const float *y, int N, int D, int nr, float *xl)
{
    const int nrow = nr * 32;
    const int64_t total = (int64_t)nrow * (kXS + 1);
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < total;
         k += (int64_t)gridDim.x * blockDim.x) {
        float v = 0.f;
        if (k < (int64_t)nrow * kXS) {
            const int n = (int)(k / kXS), d = (int)(k % kXS);
            if (n < N && d < D) v = X[(size_t)n * ldx + d] * kLog2e;
        } else {
            const int n = (int)(k - (int64_t)nrow * kXS);
            if (n < N) v = y[n];
        }
        xl[k] = v;
    }
}

// X^T y in FP64, rounded once: one workgroup per coordinate d < 32 (zero
// beyond D), strided partial sums folded in a fixed order.
__global__ void __launch_bounds__(256) k_logreg_xty(const float *X, int ldx, const float *y, int N, int D,
                                                   float *out)
{
    __shared__ double s_p[256];
    const int d = blockIdx.x, tid = threadIdx.x;
    double acc = 0.0;
    if (d < D)
        for (int n = tid; n < N; n += 256) acc += (double)X[(size_t)n * ldx + d] * (double)y[n];
    s_p[tid] = acc;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if (tid < h) s_p[tid] += s_p[tid + h];
        __syncthreads();
    }
    if (tid == 0) out[d] = (float)s_p[0];
}

constexpr int kLdsImageFloats(int nr) { return nr * 32 * (kXS + 1) + 32; }

// Per-column scalings of the split-FP16 image: X_nd log2(e) 2^e_d is stored,
// and c_d = 2^-e_d.
struct HScale {
    float mul[32], c[32];
};

// Split-FP16 image (layout at k_eval_logreg_h): hi and lo planes of the scaled
// X in storage order, then y padded with zeros; X^T y (k_logreg_xty) and c_d
// follow.
__global__ void k_logreg_h_image(const float *X, int ldx, const float *y, int N, int D, int nr, HScale sc,
                                 _Float16 *hi, float *yp)
{
    const int nrow = nr * 32;
    _Float16 *lo = hi + (size_t)nrow * kHW;
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nrow * kHW; k += gridDim.x * blockDim.x) {
        const int pos = k / kHW, p = k % kHW, q = pos & 31;
        const int r = (q & ~7) | ((q & 1) << 2) | ((q >> 1) & 3);  // h_row(r) = q
        const int d = (p & 16) | ((p & 7) << 1) | ((p >> 3) & 1);  // h_col(d) = p
        const int n = (pos & ~31) + r;
        const float v = (n < N && d < D) ? X[(size_t)n * ldx + d] * sc.mul[d] : 0.f;
        const _Float16 h = (_Float16)v;
        hi[k] = h;
        lo[k] = (_Float16)(v - (float)h);
    }
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < nrow; k += gridDim.x * blockDim.x)
        yp[k] = k < N ? y[k] : 0.f;
    if (blockIdx.x == 0 && threadIdx.x < 32) yp[nrow + 32 + threadIdx.x] = sc.c[threadIdx.x];
}

template <int MK>
hipError_t allow_lds()
{
    const hipError_t e = hipFuncSetAttribute((const void *)k_eval_logreg_lds<MK>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             kLdsImageFloats(kLdsMaxRowTiles) * (int)sizeof(float));
    if (e != hipSuccess) return e;
    return hipFuncSetAttribute((const void *)k_eval_logreg_h<MK>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kHImageBytes(kHMaxRowTiles));
}

}  // namespace

pmc_status logreg_build_frags(pmc_context *ctx, DevTarget &t)
{
    if (t.dim >= kWideMinDim) return logreg_wide_tables(ctx, t);
    const int nr = (t.n_data + 31) / 32, mk = (t.dim + 1) / 2;
    t.nr = nr;
    t.mk = mk <= 2 ? 2 : mk <= 4 ? 4 : mk <= 8 ? 8 : mk <= 13 ? 13 : 16;
    if (t.products == PMC_PRODUCTS_REFINE && nr > kLdsMaxRowTiles) {
        set_error("logreg target: refined products need n_data <= %d", 32 * kLdsMaxRowTiles);
        return PMC_ERR_UNSUPPORTED;
    }
    if (t.products != PMC_PRODUCTS_F32) {
        // split-FP16 products need the image in LDS
        if (nr <= kHMaxRowTiles) {
            // column scalings: largest |X_nd| log2(e) 2^e_d in [4, 8)
            std::vector<float> hx((size_t)t.n_data * t.ldx);
            PMC_TRY_HIP(hipMemcpyAsync(hx.data(), t.X, sizeof(float) * hx.size(), hipMemcpyDeviceToHost,
                                       ctx->stream));
            PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
            HScale sc;
            for (int d = 0; d < 32; d++) {
                float mx = 0.f;
                if (d < t.dim)
                    for (int n = 0; n < t.n_data; n++) mx = std::max(mx, std::fabs(hx[(size_t)n * t.ldx + d]));
                const float v = mx * kLog2e;
                const int e = (v > 0.f && std::isfinite(v)) ? 2 - std::ilogb(v) : 0;
                sc.mul[d] = std::ldexp(kLog2e, e);
                sc.c[d] = std::ldexp(1.f, -e);
            }
            PMC_TRY_HIP(hipMalloc(&t.xh, kHImageBytes(nr)));
            float *yp = (float *)((char *)t.xh + (size_t)nr * 32 * kHW * 2 * sizeof(_Float16));
            hipLaunchKernelGGL(k_logreg_h_image, dim3(64), dim3(256), 0, ctx->stream, (const float *)t.X, t.ldx,
                               (const float *)t.y, t.n_data, t.dim, nr, sc, (_Float16 *)t.xh, yp);
            PMC_TRY_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_logreg_xty, dim3(32), dim3(256), 0, ctx->stream, (const float *)t.X, t.ldx,
                               (const float *)t.y, t.n_data, t.dim, yp + (size_t)nr * 32);
            PMC_TRY_HIP(hipGetLastError());
        } else if (t.products == PMC_PRODUCTS_SPLIT16) {
            set_error("logreg target: split-FP16 products need n_data <= %d", 32 * kHMaxRowTiles);
            return PMC_ERR_UNSUPPORTED;
        }
    }
    if ((!t.xh || t.products == PMC_PRODUCTS_REFINE) && nr <= kLdsMaxRowTiles) {
        // LDS-resident path (FP32 products): one padded image of X and y
        const size_t bl = sizeof(float) * (size_t)kLdsImageFloats(nr);
        PMC_TRY_HIP(hipMalloc(&t.xl, bl));
        hipLaunchKernelGGL(k_logreg_lds_image, dim3(64), dim3(256), 0, ctx->stream, (const float *)t.X, t.ldx,
                           (const float *)t.y, t.n_data, t.dim, nr, (float *)t.xl);
        PMC_TRY_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_logreg_xty, dim3(32), dim3(256), 0, ctx->stream, (const float *)t.X, t.ldx,
                           (const float *)t.y, t.n_data, t.dim, (float *)t.xl + (size_t)nr * 32 * (kXS + 1));
        PMC_TRY_HIP(hipGetLastError());
    }
    if (t.xh || t.xl) {
        PMC_TRY_HIP(allow_lds<2>());
        PMC_TRY_HIP(allow_lds<4>());
        PMC_TRY_HIP(allow_lds<8>());
        PMC_TRY_HIP(allow_lds<13>());
        PMC_TRY_HIP(allow_lds<16>());
        return PMC_OK;
    }
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

pmc_status launch_eval_logreg(pmc_context *ctx, const DevTarget &t, const EvalArgs &a_in)
{
    if (a_in.n_tiles <= 0) return PMC_OK;
    EvalArgs a = a_in;
    if (t.xh && t.xl) {
        // refined products: the split-FP16 kernel takes the chains still in
        // their first phase, the FP32 kernel the others (each returns at
        // once when it has no chain)
        a.fine_sel = 0;
    }
    if (t.xh) {
        HArgs f{t.xh, t.nr, (float)(1.0 / t.prior_var)};
        const size_t lds = kHImageBytes(t.nr);
        const int want = (a.n_tiles + kLdsWaves - 1) / kLdsWaves;
        dim3 grid(std::max(1, std::min(want, ctx->n_cu > 0 ? ctx->n_cu : 256))), block(64 * kLdsWaves);
        switch (t.mk) {
        case 2: hipLaunchKernelGGL(k_eval_logreg_h<2>, grid, block, lds, ctx->stream, a, f); break;
        case 4: hipLaunchKernelGGL(k_eval_logreg_h<4>, grid, block, lds, ctx->stream, a, f); break;
        case 8: hipLaunchKernelGGL(k_eval_logreg_h<8>, grid, block, lds, ctx->stream, a, f); break;
        case 13: hipLaunchKernelGGL(k_eval_logreg_h<13>, grid, block, lds, ctx->stream, a, f); break;
        case 16: hipLaunchKernelGGL(k_eval_logreg_h<16>, grid, block, lds, ctx->stream, a, f); break;
        default: set_error("logreg eval: unsupported dimension"); return PMC_ERR_UNSUPPORTED;
        }
        PMC_TRY_HIP(hipGetLastError());
        if (!t.xl) return PMC_OK;
        a.fine_sel = 1;
    }
    if (t.xl) {
        LdsArgs f{(const float *)t.xl, t.nr, (float)(1.0 / t.prior_var)};
        const size_t lds = sizeof(float) * (size_t)kLdsImageFloats(t.nr);
        const int want = (a.n_tiles + kLdsWaves - 1) / kLdsWaves;
        dim3 grid(std::max(1, std::min(want, ctx->n_cu > 0 ? ctx->n_cu : 256))), block(64 * kLdsWaves);
        switch (t.mk) {
        case 2: hipLaunchKernelGGL(k_eval_logreg_lds<2>, grid, block, lds, ctx->stream, a, f); break;
        case 4: hipLaunchKernelGGL(k_eval_logreg_lds<4>, grid, block, lds, ctx->stream, a, f); break;
        case 8: hipLaunchKernelGGL(k_eval_logreg_lds<8>, grid, block, lds, ctx->stream, a, f); break;
        case 13: hipLaunchKernelGGL(k_eval_logreg_lds<13>, grid, block, lds, ctx->stream, a, f); break;
        case 16: hipLaunchKernelGGL(k_eval_logreg_lds<16>, grid, block, lds, ctx->stream, a, f); break;
        default: set_error("logreg eval: unsupported dimension"); return PMC_ERR_UNSUPPORTED;
        }
        PMC_TRY_HIP(hipGetLastError());
        return PMC_OK;
    }
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
