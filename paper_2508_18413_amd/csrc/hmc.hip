// HMC with parallel leapfrog integration (Appendix A.2 algorithm, Sec. 3.3).
//
// One persistent workgroup runs the proposals in order.  For proposal p:
// v0 = momenta[p]; H0 = |v0|^2/2 - log p(x0); half step v += eps/2 grad log p(x0);
// the L leapfrog steps s_t = f(s_{t-1}) on s = [x, v] (x' = x + eps v,
// v' = v + eps grad log p(x')), then the reverse half step, HL, and the
// Metropolis test log U < H0 - HL.
//
// Parallel mode: the L steps are solved by Newton sweeps entirely in LDS:
//   eval:  F_t = f(S_{t-1}) for all t at once; the L gradients are one
//          product of the precision P (D x D) with the L positions on FP32
//          matrix cores, P held in registers as A fragments for the whole
//          launch (one wave per 32 x 32 output tile);
//   scan:  per coordinate d, the 2x2 recursion of block quasi-DEER
//          (Appendix A.3) delta_t = J_t delta_{t-1} + (F_t - S_t) with
//          J_t = [[1, eps], [eps h, 1 + eps^2 h]], h = -P_dd (diagonal
//          quasi-DEER keeps [1, 1 + eps^2 h]; Picard uses J = 0), as an
//          inclusive scan of affine maps across the lanes of a wave (lane l
//          holds step l + 1), then S_t <- F_t + J_t delta_{t-1};
//   test:  Algorithm 1's max |delta| / (atol + rtol |S|) <= 1.
// Sequential mode integrates the same L steps one after another with P's
// rows held in registers (eight lanes per row).
//
// Target: Gaussian N(mu, P^-1), FP32, D <= 128; parallel mode L <= 64.
#include <math.h>
#include <string.h>

#include <vector>

#include "pmc_internal.hpp"

namespace pmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

struct HMCArgs {
    int D, L, n_prop;
    float eps;
    const float *mean, *prec;
    const float *x0, *momenta, *unif;
    float *chain;
    uint8_t *accept;
    float *logr;    // (H0 - HL) - log U per proposal, or nullptr
    int32_t *sweeps;
    int variant;  // PMC_QDEER_BLOCK2, PMC_QDEER_DIAG, PMC_PICARD
    float atol, rtol;
    int floor_stall;
    int max_sweeps;
    int probes;             // 1: h from one Hessian-vector product per step and sweep (App. A.3)
    uint64_t probe_seed;
};

constexpr int kNT = 1024;      // sequential kernel
constexpr int kNW = kNT / 64;
constexpr int kParNT = 512;    // parallel kernel: two waves per SIMD leave 256 registers per lane
constexpr int kParNW = kParNT / 64;
constexpr int kMaxD = 128;
constexpr int kMaxLPar = 64;

__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Sum / max over the workgroup; every thread gets the result.  `red` holds NW values.
template <int NW, typename T>
__device__ T block_sum(T v, T *red)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    T s = T(0);
#pragma unroll
    for (int i = 0; i < NW; i++) s += red[i];
    return s;
}

template <int NW>
__device__ float block_max(float v, float *red)
{
    for (int m = 32; m >= 1; m >>= 1) v = fmaxf(v, __shfl_xor(v, m, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < NW; i++) s = fmaxf(s, red[i]);
    return s;
}

// ------------------------------------------------------- sequential leapfrog
// Lane (row, c) = (tid / 8, tid % 8) holds P[row][c CW .. c CW + CW - 1]; a
// gradient entry is an 8-lane sum.  Lane c = 0 of each row owns x_row, v_row
// and g_row in registers; positions are published through a double-buffered
// LDS vector, so one barrier per leapfrog step suffices.
template <int CW>
__global__ void __launch_bounds__(kNT) k_hmc_seq(HMCArgs a)
{
    __shared__ float s_xb[2][kMaxD], s_mu[kMaxD];
    __shared__ double s_red[kNW];
    __shared__ int s_flag;
    const int tid = threadIdx.x, row = tid >> 3, c = tid & 7;
    const int D = a.D, L = a.L;
    const float eps = a.eps;
    const bool owner = c == 0 && row < D;
    float PR[CW];
#pragma unroll
    for (int k = 0; k < CW; k++) {
        const int col = c * CW + k;
        PR[k] = (row < D && col < D) ? a.prec[(size_t)row * D + col] : 0.f;
    }
    for (int d = tid; d < kMaxD; d += kNT) {
        s_mu[d] = d < D ? a.mean[d] : 0.f;
        s_xb[0][d] = d < D ? a.x0[d] : 0.f;
        s_xb[1][d] = 0.f;
    }
    float x = owner ? a.x0[row] : 0.f;
    if (owner) a.chain[row] = x;
    __syncthreads();
    // grad log p at the positions in buffer b: -(P (x - mu))_row, in all 8 lanes of a row
    auto grad = [&](int b) {
        float acc = 0.f;
#pragma unroll
        for (int k = 0; k < CW; k++) {
            const int col = c * CW + k;
            acc = fmaf(PR[k], s_xb[b][col] - s_mu[col], acc);
        }
        acc += __shfl_xor(acc, 1, 64);
        acc += __shfl_xor(acc, 2, 64);
        acc += __shfl_xor(acc, 4, 64);
        return -acc;
    };
    float g = grad(0);
    const float mu = owner ? s_mu[row] : 0.f;
    int b = 0;  // buffer holding the current state
    for (int p = 0; p < a.n_prop; p++) {
        const float v0 = owner ? a.momenta[(size_t)p * D + row] : 0.f;
        // energies: FP32 terms, FP64 sums (log p = -(x - mu).P(x - mu)/2 = (x - mu).g/2)
        const double H0 = block_sum<kNW>(owner ? 0.5 * ((double)v0 * v0 - (double)(x - mu) * g) : 0.0, s_red);
        float xl = x, v = fmaf(0.5f * eps, g, v0), gl = g;
        int bl = b;
        for (int t = 1; t <= L; t++) {
            bl ^= 1;
            xl = fmaf(eps, v, xl);
            if (owner) s_xb[bl][row] = xl;
            __syncthreads();
            gl = grad(bl);
            v = fmaf(eps, gl, v);
        }
        const float vf = fmaf(-0.5f * eps, gl, v);
        const double HL = block_sum<kNW>(owner ? 0.5 * ((double)vf * vf - (double)(xl - mu) * gl) : 0.0, s_red);
        if (tid == 0) {
            const double lr = (H0 - HL) - log((double)a.unif[p]);
            const int acc = lr > 0.0;
            s_flag = acc;
            if (a.accept) a.accept[p] = (uint8_t)acc;
            if (a.logr) a.logr[p] = (float)lr;
            if (a.sweeps) a.sweeps[p] = 0;
        }
        __syncthreads();
        if (s_flag) {
            x = xl;
            g = gl;
            b = bl;  // the proposal's last buffer holds x_L
        } else if (owner) {
            s_xb[b][row] = x;  // x's buffer may have been reused by the trajectory
        }
        if (owner) a.chain[(size_t)(p + 1) * D + row] = x;
        __syncthreads();
    }
}

// --------------------------------------------------------- parallel leapfrog
struct Aff2 {
    float a, b, c, d, e, f;  // [[a, b], [c, d]] and offset [e, f]
};

// later o earlier
__device__ __forceinline__ Aff2 compose2(const Aff2 &L, const Aff2 &E)
{
    Aff2 r;
    r.a = fmaf(L.a, E.a, L.b * E.c);
    r.b = fmaf(L.a, E.b, L.b * E.d);
    r.c = fmaf(L.c, E.a, L.d * E.c);
    r.d = fmaf(L.c, E.b, L.d * E.d);
    r.e = fmaf(L.a, E.e, fmaf(L.b, E.f, L.e));
    r.f = fmaf(L.c, E.e, fmaf(L.d, E.f, L.f));
    return r;
}

__device__ __forceinline__ Aff2 shfl_up2(const Aff2 &x, int o)
{
    Aff2 r;
    r.a = __shfl_up(x.a, o, 64);
    r.b = __shfl_up(x.b, o, 64);
    r.c = __shfl_up(x.c, o, 64);
    r.d = __shfl_up(x.d, o, 64);
    r.e = __shfl_up(x.e, o, 64);
    r.f = __shfl_up(x.f, o, 64);
    return r;
}

// MKP = K pairs of the precision's A fragments (ceil(D / 2) rounded up to 8).
template <int MKP>
__global__ void __launch_bounds__(kParNT) k_hmc_par(HMCArgs a)
{
    extern __shared__ float sm[];
    const int D = a.D, L = a.L, SP = 2 * D + 1;  // odd row stride
    float *S = sm;                                // [L + 1][SP]: row 0 = s_0, row t = s_t
    float *F = S + (size_t)(L + 1) * SP;          // [L][SP]: row t - 1 = F_t
    float *s_mu = F + (size_t)L * SP;             // [kMaxD]
    float *s_h = s_mu + kMaxD;                    // [kMaxD]: -P_dd
    float *s_x = s_h + kMaxD;                     // [kMaxD] current state
    float *s_g = s_x + kMaxD;                     // [kMaxD] gradient at the current state
    float *s_gl = s_g + kMaxD;                    // [kMaxD] gradient at x_L
    float *s_red = s_gl + kMaxD;                  // [kParNW]
    float *s_hp = s_red + kParNW;                 // [L][D] probed Hessian diagonal (probes)
    uint32_t *s_zb = (uint32_t *)(s_hp + (a.probes ? L * D : 0));  // [L][ceil(D / 32)] probe sign bits
    const int NZW = (D + 31) / 32;
    __shared__ double s_redd[kParNW];
    __shared__ int s_flag;
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 31, hh = lane >> 5;
    const float eps = a.eps;
    const int n_mt = (D + 31) / 32, n_nt = (L + 31) / 32;
    const bool mw = w < n_mt * n_nt;  // this wave owns a gradient output tile
    const int mb = w % n_mt, nb = w / n_mt;

    float PA[MKP];  // A fragments: P[32 mb + i][2 m + hh]
#pragma unroll
    for (int m = 0; m < MKP; m++) {
        const int r = 32 * mb + i, k = 2 * m + hh;
        PA[m] = (mw && r < D && k < D) ? a.prec[(size_t)r * D + k] : 0.f;
    }
    for (int d = tid; d < kMaxD; d += kParNT) {
        s_mu[d] = d < D ? a.mean[d] : 0.f;
        s_h[d] = d < D ? -a.prec[(size_t)d * D + d] : 0.f;
        s_x[d] = d < D ? a.x0[d] : 0.f;
        if (d < D) a.chain[d] = a.x0[d];
    }
    __syncthreads();

    // P (x_t - mu) for the positions x_t = X[t][0..D) (row stride SP), t < cnt;
    // calls emit(t, row, value) for every computed entry.  With probe set
    // the operand is instead the Rademacher probe z_t, -1 where bit k of
    // s_zb[t] is set.
    auto zsign = [&](int t, int k) { return ((s_zb[t * NZW + (k >> 5)] >> (k & 31)) & 1u) ? -1.f : 1.f; };
    auto pmul = [&](const float *X, int cnt, auto emit, bool probe = false) {
        if (!mw || 32 * nb >= cnt) return;
        const int t = 32 * nb + i;
        const bool tv = t < cnt;
        f32x16 acc = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < MKP; m++) {
            const int k = 2 * m + hh;
            float bv = 0.f;
            if (tv && k < D)
                bv = probe ? zsign(t, k) : X[(size_t)t * SP + k] - s_mu[k];
            acc = __builtin_amdgcn_mfma_f32_32x32x2f32(PA[m], bv, acc, 0, 0, 0);
        }
        if (tv) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int row = 32 * mb + crow(r, hh);
                if (row < D) emit(t, row, acc[r]);
            }
        }
    };

    // gradient at x0 (row 0 of S holds the position)
    for (int d = tid; d < D; d += kParNT) S[d] = s_x[d];
    __syncthreads();
    pmul(S, 1, [&](int, int row, float v) { s_g[row] = -v; });
    __syncthreads();

    for (int p = 0; p < a.n_prop; p++) {
        const float *v0 = a.momenta + (size_t)p * D;
        double h0 = 0.0;  // energies: FP32 terms, FP64 sums
        for (int d = tid; d < D; d += kParNT) {
            const float v = v0[d];
            h0 += 0.5 * ((double)v * v - (double)(s_x[d] - s_mu[d]) * s_g[d]);  // log p = (x - mu).g / 2
            S[d] = s_x[d];
            S[D + d] = fmaf(0.5f * eps, s_g[d], v);
        }
        const double H0 = block_sum<kParNW>(h0, s_redd);
        // initial guess: every s_t = s_0
        for (int o = tid; o < L * SP; o += kParNT) S[SP + o] = S[o % SP];
        __syncthreads();
        float best = INFINITY;
        int stall = 0, nsw = 0;
        for (;;) {
            // eval: positions, then the L gradients into the velocities
            for (int o = tid; o < L * D; o += kParNT) {
                const int t = o / D, d = o % D;
                F[(size_t)t * SP + d] = fmaf(eps, S[(size_t)t * SP + D + d], S[(size_t)t * SP + d]);
            }
            if (a.probes) {
                // one Rademacher probe per leapfrog step and sweep: sign bit d of
                // step l of proposal p from (seed, sweep, global step p L + l, d)
                const uint64_t hs = probe_mix(probe_mix(a.probe_seed) ^ (uint64_t)(uint32_t)nsw);
                for (int o = tid; o < L * NZW; o += kParNT) {
                    const int t = o / NZW, k0 = 32 * (o % NZW);
                    const uint64_t base = 1024 * ((uint64_t)p * L + t);
                    uint32_t bits = 0;
                    for (int b = 0; b < 32 && k0 + b < D; b++)
                        bits |= (uint32_t)(probe_mix(hs ^ (base + k0 + b)) >> 63) << b;
                    s_zb[o] = bits;
                }
            }
            __syncthreads();
            pmul(F, L, [&](int t, int row, float v) {
                F[(size_t)t * SP + D + row] = fmaf(-eps, v, S[(size_t)t * SP + D + row]);
            });
            if (a.probes)  // h_t ~ z_t o (H z_t) with H = -P
                pmul(F, L, [&](int t, int row, float v) { s_hp[t * D + row] = -zsign(t, row) * v; }, true);
            __syncthreads();
            // scan: lane l holds step l + 1 (F row l, S row l + 1)
            float rmax = 0.f;
            const bool lv = lane < L;
            for (int d = w; d < D; d += kParNW) {
                const float h = a.probes ? (lv ? s_hp[lane * D + d] : 0.f) : s_h[d];
                float ja = 1.f, jb = eps, jc = eps * h, jd = fmaf(eps * eps, h, 1.f);
                if (a.variant == PMC_QDEER_DIAG) jb = jc = 0.f;
                if (a.variant == PMC_PICARD) ja = jb = jc = jd = 0.f;
                const float fx = lv ? F[(size_t)lane * SP + d] : 0.f;
                const float fv = lv ? F[(size_t)lane * SP + D + d] : 0.f;
                const float sx = lv ? S[(size_t)(lane + 1) * SP + d] : 0.f;
                const float sv = lv ? S[(size_t)(lane + 1) * SP + D + d] : 0.f;
                Aff2 e;
                e.a = lv ? ja : 1.f;
                e.b = lv ? jb : 0.f;
                e.c = lv ? jc : 0.f;
                e.d = lv ? jd : 1.f;
                e.e = fx - sx;
                e.f = fv - sv;
#pragma unroll
                for (int o = 1; o < 64; o <<= 1) {
                    const Aff2 u = shfl_up2(e, o);
                    if (lane >= o) e = compose2(e, u);
                }
                // delta_{t-1}: the previous lane's inclusive offset (0 before step 1)
                float px = __shfl_up(e.e, 1, 64), pv = __shfl_up(e.f, 1, 64);
                if (lane == 0) px = pv = 0.f;
                if (lv) {
                    const float nx = fx + fmaf(ja, px, jb * pv);
                    const float nv = fv + fmaf(jc, px, jd * pv);
                    const float dx = nx - sx, dv = nv - sv;
                    const float r = fmaxf(fabsf(dx) / (a.atol + a.rtol * fabsf(nx)),
                                          fabsf(dv) / (a.atol + a.rtol * fabsf(nv)));
                    rmax = (r == r) ? fmaxf(rmax, r) : INFINITY;
                    S[(size_t)(lane + 1) * SP + d] = nx;
                    S[(size_t)(lane + 1) * SP + D + d] = nv;
                }
            }
            const float ratio = block_max<kParNW>(rmax, s_red);
            nsw++;
            if (ratio < 0.5f * best) {
                best = ratio;
                stall = 0;
            } else {
                stall++;
            }
            if (ratio <= 1.f || nsw >= a.max_sweeps ||
                (a.floor_stall > 0 && stall >= a.floor_stall && ratio <= 2.f))
                break;
        }
        // gradient at x_L, reverse half step, HL, Metropolis test
        const float *sL = S + (size_t)L * SP;
        pmul(sL, 1, [&](int, int row, float v) { s_gl[row] = -v; });
        __syncthreads();
        double hl = 0.0;
        for (int d = tid; d < D; d += kParNT) {
            const float v = fmaf(-0.5f * eps, s_gl[d], sL[D + d]);
            hl += 0.5 * ((double)v * v - (double)(sL[d] - s_mu[d]) * s_gl[d]);
        }
        const double HL = block_sum<kParNW>(hl, s_redd);
        if (tid == 0) {
            const double lr = (H0 - HL) - log((double)a.unif[p]);
            const int acc = lr > 0.0;
            s_flag = acc;
            if (a.accept) a.accept[p] = (uint8_t)acc;
            if (a.logr) a.logr[p] = (float)lr;
            if (a.sweeps) a.sweeps[p] = nsw;
        }
        __syncthreads();
        const int acc = s_flag;
        for (int d = tid; d < D; d += kParNT) {
            if (acc) {
                s_x[d] = sL[d];
                s_g[d] = s_gl[d];
            }
            a.chain[(size_t)(p + 1) * D + d] = s_x[d];
        }
        __syncthreads();
    }
}

template <int MKP>
void launch_par(const HMCArgs &a, size_t lds, hipStream_t st)
{
    (void)hipFuncSetAttribute((const void *)k_hmc_par<MKP>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k_hmc_par<MKP>, dim3(1), dim3(kParNT), lds, st, a);
}

template <int CW>
void launch_seq(const HMCArgs &a, hipStream_t st)
{
    hipLaunchKernelGGL(k_hmc_seq<CW>, dim3(1), dim3(kNT), 0, st, a);
}

}  // namespace
}  // namespace pmc

using namespace pmc;

extern "C" pmc_status pmc_hmc_sample(pmc_context *ctx, const pmc_target *target, double step_size,
                                     int L, int n_prop, const void *x0, const void *momenta,
                                     const void *unif, const pmc_options *opts,
                                     int parallel_leapfrog, void *out_chain, uint8_t *accept,
                                     float *logr, int32_t *sweeps, pmc_result *res)
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
    if (D > kMaxD) {
        set_error("pmc_hmc_sample: D = %d exceeds %d", D, kMaxD);
        return PMC_ERR_UNSUPPORTED;
    }
    if (parallel_leapfrog && L > kMaxLPar) {
        set_error("pmc_hmc_sample: parallel leapfrog supports L <= %d (got %d)", kMaxLPar, L);
        return PMC_ERR_UNSUPPORTED;
    }
    const bool probes = parallel_leapfrog && opts->jac_probes == 1;
    PMC_REQUIRE(opts->jac_probes == 0 || opts->jac_probes == 1, "pmc_hmc_sample: jac_probes is 0 or 1");
    if (probes && opts->variant != PMC_QDEER_BLOCK2 && opts->variant != PMC_QDEER_DIAG) {
        set_error("pmc_hmc_sample: jac_probes applies to the block and diagonal variants");
        return PMC_ERR_UNSUPPORTED;
    }
    const size_t lds = sizeof(float) * ((size_t)(2 * L + 1) * (2 * D + 1) + 5 * kMaxD + kParNW +
                                        (probes ? (size_t)L * D + (size_t)L * ((D + 31) / 32) : 0));
    if (parallel_leapfrog && lds > (size_t)160 * 1024) {
        set_error("pmc_hmc_sample: the parallel leapfrog of D = %d, L = %d%s needs %zu bytes of LDS (160 KiB)", D, L,
                  probes ? " with probes" : "", lds);
        return PMC_ERR_UNSUPPORTED;
    }
    if (res) memset(res, 0, sizeof(*res));
    if (n_prop == 0) return PMC_OK;
    PMC_REQUIRE(is_device_ptr(x0) && is_device_ptr(momenta) && is_device_ptr(unif) &&
                    is_device_ptr(out_chain),
                "pmc_hmc_sample: x0, momenta, unif, out_chain must be device pointers");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    {
        const InputCheck in[3] = {{x0, (int64_t)D, 0}, {momenta, (int64_t)n_prop * D, 0}, {unif, n_prop, 1}};
        PMC_TRY(check_inputs(ctx, PMC_F32, in, 3));
    }
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
    a.logr = logr;
    a.sweeps = d_sw;
    a.variant = opts->variant;
    a.atol = (float)opts->atol;
    a.rtol = (float)opts->rtol;
    a.floor_stall = opts->floor_stall;
    a.max_sweeps = opts->max_iter > 0 ? opts->max_iter : L + 1;
    a.probes = probes ? 1 : 0;
    a.probe_seed = opts->probe_seed;
    PMC_TRY_HIP(hipEventRecord(ctx->ev0, ctx->stream));
    if (parallel_leapfrog) {
        const int mkp = ((D + 1) / 2 + 7) / 8 * 8;
        switch (mkp) {
        case 8: launch_par<8>(a, lds, ctx->stream); break;
        case 16: launch_par<16>(a, lds, ctx->stream); break;
        case 24: launch_par<24>(a, lds, ctx->stream); break;
        case 32: launch_par<32>(a, lds, ctx->stream); break;
        case 40: launch_par<40>(a, lds, ctx->stream); break;
        case 48: launch_par<48>(a, lds, ctx->stream); break;
        case 56: launch_par<56>(a, lds, ctx->stream); break;
        default: launch_par<64>(a, lds, ctx->stream); break;
        }
    } else {
        const int cw = ((D + 7) / 8 + 3) / 4 * 4;
        switch (cw) {
        case 4: launch_seq<4>(a, ctx->stream); break;
        case 8: launch_seq<8>(a, ctx->stream); break;
        case 12: launch_seq<12>(a, ctx->stream); break;
        default: launch_seq<16>(a, ctx->stream); break;
        }
    }
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
