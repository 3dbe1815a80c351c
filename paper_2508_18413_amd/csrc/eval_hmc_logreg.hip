// HMC across the sequence (Sec. 3.3, "Parallel HMC with Sequential Leapfrog
// Integration") on the logistic-regression posterior, with the settings of
// App. B.4 in mind (L = 4 leapfrog steps, the one-probe "memory-efficient"
// diagonal of Sec. 3.4 eq. 10, damping and clipping of the diagonal).
//
// Evaluation (k_eval_hmc_logreg): a workgroup of 8 waves holds X and y in
// LDS and works through 32-step tiles.  For the 32 steps of a tile it runs
// the transitions' leapfrog integrators in lock step, each position update
// being one batched gradient of the 32 positions:
//   Z = X P (data x steps) on FP32 matrix cores (32x32x2), the residual
//   r = y - sigma(Z), and G = X^T r, again on matrix cores, where the
//   contraction slots of X^T r are the accumulator rows each lane already
//   holds (X^T's operand rows are permuted to match, so r never moves
//   between lanes);
// and, for the probe direction z, the Hessian-vector products
// H d = -X^T (w o X d) - d / prior_var with w = sigma(Z)(1 - sigma(Z)) in
// the same pass (forward-mode tangent of the integrator).  Each wave takes
// every 8th row tile; the partial sums meet in a fixed-order tree through
// LDS, so results are deterministic, and are broadcast back so that each
// wave keeps the transitions' state (position increment, momentum,
// tangents) of 4 of the 32 coordinates in registers (lane = step), in the
// matrix-core accumulator layout; per-step sums meet in LDS in fixed order.
// The energy difference is assembled in FP64 from FP32 terms, with the
// log-likelihood difference taken through the exact increment
// dl = x_L - x0: sum_n [y_n (X dl)_n - log(1 + sigma(z0_n) expm1((X dl)_n))].
//
// Sequential sampler (k_seq_hmc_logreg): one workgroup per chain, rows of X
// in registers, each gradient a workgroup reduction.
#include <math.h>

#include <algorithm>

#include "logistic.hpp"
#include "pmc_internal.hpp"

namespace pmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kW = 8;               // waves per workgroup
constexpr int kNT = 64 * kW;
constexpr int kPS = 33;             // row stride of the step x coordinate staging arrays
constexpr int kMaxRowsHmc = 1024;   // data points held in LDS
constexpr size_t kLdsLimit = 160 * 1024;  // LDS of a gfx950 compute unit

__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

// Workgroup barrier that orders LDS only.
__device__ __forceinline__ void lds_barrier_fn()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ float softplus_diff_h(float z, float dz, float s)
{
    if (dz > -8.f && dz < 30.f) return log1p_s(s * expm1_s(dz));
    return softplus(z + dz) - softplus(z);
}

struct HmcLogregArgs {
    const float *X;      // [n_data, ldx]
    const float *y;      // [n_data]
    int N, ldx, D;
    float pp;            // 1 / prior_var
};

// Dynamic LDS layout (floats): X rows [NR][ldx], y [NR], P and Pd [32][kPS],
// the tree-reduction buffer [4][2][16][64] and per-step FP64 partials
// [4][kW][32].
struct Lds {
    float *X, *y, *P, *Pd, *buf;
    double *red;  // [4][kW][32] per-step partial sums
};

__device__ __forceinline__ Lds lds_layout(float *sm, int NR, int ldx)
{
    Lds l;
    l.X = sm;
    l.y = l.X + (size_t)NR * ldx;
    l.P = l.y + NR;
    l.Pd = l.P + 32 * kPS;
    l.buf = l.Pd + 32 * kPS;
    l.red = (double *)(l.buf + 4 * 2 * 16 * 64);
    return l;
}

size_t lds_bytes(int NR, int ldx)
{
    return sizeof(float) * ((size_t)NR * ldx + NR + 2 * 32 * kPS + 4 * 2 * 16 * 64) + sizeof(double) * 4 * kW * 32;
}

// Z (+ Zd) = X_tile P (+ Pd) for one 32-row tile; lane (i, h): A slot m =
// X[32 rt + i][2 m + h], B slot m = P[step i][2 m + h]; accumulator register
// r = row crow(r, h), column = step i.
// With bft the tangent product is formed on BF16 matrix instructions (16 k
// per instruction, lane half h taking k = 16 kb + 8 h + j): for directions
// that only enter a Jacobian, never f.  The HMC transitions' probe tangents
// take it; the relaxed MALA gate keeps FP32 (its rank-one term is a small
// correction whose BF16 error would be a few per cent of it).
template <int MK>
__device__ __forceinline__ void fwd_dir_bf16(const float *xr, const float *dir, int D, int i, int h, f32x16 &Zd)
{
    constexpr int KB = (2 * MK + 15) / 16;
#pragma unroll
    for (int kb = 0; kb < KB; kb++) {
        bf16x8 A, B;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int k = 16 * kb + 8 * h + j;
            A[j] = (__bf16)(k < D ? xr[k] : 0.f);
            B[j] = (__bf16)dir[i * kPS + k];
        }
        Zd = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, Zd, 0, 0, 0);
    }
}

template <int MK, bool tangent, bool bft = false>
__device__ __forceinline__ void fwd_products(const Lds &l, int ldx, int D, int rt, int i, int h, f32x16 &Z,
                                             f32x16 &Zd)
{
    Z = f32x16{0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    Zd = Z;
    const float *xr = l.X + (size_t)(32 * rt + i) * ldx;
#pragma unroll
    for (int m = 0; m < MK; m++) {
        const int k = 2 * m + h;
        const float a = k < D ? xr[k] : 0.f;
        Z = __builtin_amdgcn_mfma_f32_32x32x2f32(a, l.P[i * kPS + k], Z, 0, 0, 0);
        if (tangent && !bft) Zd = __builtin_amdgcn_mfma_f32_32x32x2f32(a, l.Pd[i * kPS + k], Zd, 0, 0, 0);
    }
    if (tangent && bft) fwd_dir_bf16<MK>(xr, l.Pd, D, i, h, Zd);
}

// G (+ Gd) += X_tile^T R (+ Rd): lane (i = coordinate, h): A slot m =
// X[32 rt + crow(m, h)][i]; B slot m = accumulator register m of R.
// BF16 form of Gd += X_tile^T Rd: k slot (kb, h, j) is row crow(8 kb + j, h),
// so A is the lane's X column entries av[8 kb + j] and B its own accumulator
// registers Rd[8 kb + j].
__device__ __forceinline__ void bwd_dir_bf16(const float (&av)[16], const f32x16 &Rd, f32x16 &Gd)
{
#pragma unroll
    for (int kb = 0; kb < 2; kb++) {
        bf16x8 A, B;
#pragma unroll
        for (int j = 0; j < 8; j++) {
            A[j] = (__bf16)av[8 * kb + j];
            B[j] = (__bf16)Rd[8 * kb + j];
        }
        Gd = __builtin_amdgcn_mfma_f32_32x32x16_bf16(A, B, Gd, 0, 0, 0);
    }
}

template <bool tangent, bool grad = true, bool bft = false>
__device__ __forceinline__ void bwd_products(const Lds &l, int ldx, int D, int rt, int i, int h, const f32x16 &R,
                                             const f32x16 &Rd, f32x16 &G, f32x16 &Gd)
{
    const bool own = i < D;
    float av[16];
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const float a = own ? l.X[(size_t)(32 * rt + crow(m, h)) * ldx + i] : 0.f;
        av[m] = a;
        if (grad) G = __builtin_amdgcn_mfma_f32_32x32x2f32(a, R[m], G, 0, 0, 0);
        if (tangent && !bft) Gd = __builtin_amdgcn_mfma_f32_32x32x2f32(a, Rd[m], Gd, 0, 0, 0);
    }
    if (tangent && bft) bwd_dir_bf16(av, Rd, Gd);
}

// Fixed-order tree over the 8 waves, then a broadcast: every wave w receives
// the sums of G and Gd in registers r = 2w and 2w + 1 (coordinates
// crow(2w, h) and crow(2w + 1, h) of step i in lane (i, h)).
template <bool tangent>
__device__ __forceinline__ void tree_reduce(const Lds &l, int w, int lane, f32x16 &G, f32x16 &Gd, float (&gs)[2],
                                            float (&hs)[2])
{
#pragma unroll
    for (int half = kW / 2; half >= 1; half >>= 1) {
        if (w >= half && w < 2 * half) {
            float *b = l.buf + (size_t)(w - half) * 2 * 16 * 64;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                b[r * 64 + lane] = G[r];
                if (tangent) b[(16 + r) * 64 + lane] = Gd[r];
            }
        }
        __syncthreads();
        if (w < half) {
            const float *b = l.buf + (size_t)w * 2 * 16 * 64;
#pragma unroll
            for (int r = 0; r < 16; r++) {
                G[r] += b[r * 64 + lane];
                if (tangent) Gd[r] += b[(16 + r) * 64 + lane];
            }
        }
        __syncthreads();
    }
    if (w == 0) {
#pragma unroll
        for (int r = 0; r < 16; r++) {
            l.buf[r * 64 + lane] = G[r];
            l.buf[(16 + r) * 64 + lane] = tangent ? Gd[r] : 0.f;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; q++) {
        gs[q] = l.buf[(2 * w + q) * 64 + lane];
        hs[q] = l.buf[(16 + 2 * w + q) * 64 + lane];
    }
    __syncthreads();  // the buffer is free again
}

// One batched evaluation at the positions in l.P (and directions in l.Pd):
// G = X^T (y - sigma(X p)) and Gd = X^T (w o X d) per (coordinate, step);
// wave w receives the entries of its coordinates (tree_reduce).  Without
// grad only Gd is formed (gs returns zeros); with bft the direction's
// products run on BF16 matrix instructions (Jacobian directions only).
template <int MK, bool tangent, bool grad = true, bool bft = false>
__device__ __forceinline__ void evaluate(const Lds &l, const HmcLogregArgs &t, int NR, int w, int lane,
                                         float (&gs)[2], float (&hs)[2])
{
    const int i = lane & 31, h = lane >> 5;
    f32x16 G = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    f32x16 Gd = G;
    for (int rt = w; 32 * rt < NR; rt += kW) {
        f32x16 Z, Zd;
        fwd_products<MK, tangent, bft>(l, t.ldx, t.D, rt, i, h, Z, Zd);
        f32x16 R, Rd;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float s = sigm(Z[r]);
            R[r] = l.y[32 * rt + crow(r, h)] - s;
            Rd[r] = s * (1.f - s) * Zd[r];
        }
        bwd_products<tangent, grad, bft>(l, t.ldx, t.D, rt, i, h, R, Rd, G, Gd);
    }
    tree_reduce<tangent>(l, w, lane, G, Gd, gs, hs);
}

// Three Hessian-vector products at the positions in l.P, in one pass over
// the data: Gk = X^T (w o X dk) for the directions d1 = l.Pd, d2 and d3
// (step-major [32][kPS] like l.Pd; d2 and d3 may lie in l.buf, which is
// read here only before the reduction's first barrier).  Wave w receives the
// entries of its coordinates as evaluate does.
template <int MK>
__device__ __forceinline__ void evaluate_hvp3(const Lds &l, const HmcLogregArgs &t, int NR, int w, int lane,
                                              const float *d2, const float *d3, float (&h1)[2], float (&h2)[2],
                                              float (&h3)[2])
{
    const int i = lane & 31, h = lane >> 5;
    const f32x16 zero = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    f32x16 G1 = zero, G2 = zero, G3 = zero;
    for (int rt = w; 32 * rt < NR; rt += kW) {
        f32x16 Z, Z1, Z2 = zero, Z3 = zero;
        fwd_products<MK, true>(l, t.ldx, t.D, rt, i, h, Z, Z1);
        const float *xr = l.X + (size_t)(32 * rt + i) * t.ldx;
#pragma unroll
        for (int m = 0; m < MK; m++) {
            const int k = 2 * m + h;
            const float a = k < t.D ? xr[k] : 0.f;
            Z2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, d2[i * kPS + k], Z2, 0, 0, 0);
            Z3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, d3[i * kPS + k], Z3, 0, 0, 0);
        }
        f32x16 R1, R2, R3;
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float sv = sigm(Z[r]);
            const float sp = sv * (1.f - sv);
            R1[r] = sp * Z1[r];
            R2[r] = sp * Z2[r];
            R3[r] = sp * Z3[r];
        }
        const bool own = i < t.D;
#pragma unroll
        for (int m = 0; m < 16; m++) {
            const float a = own ? l.X[(size_t)(32 * rt + crow(m, h)) * t.ldx + i] : 0.f;
            G1 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, R1[m], G1, 0, 0, 0);
            G2 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, R2[m], G2, 0, 0, 0);
            G3 = __builtin_amdgcn_mfma_f32_32x32x2f32(a, R3[m], G3, 0, 0, 0);
        }
    }
    __syncthreads();  // every wave is done reading d2 and d3
    tree_reduce<true>(l, w, lane, G1, G2, h1, h2);
    f32x16 none = zero;
    float unused[2];
    tree_reduce<false>(l, w, lane, G3, none, h3, unused);
}

// Sum of the 16 registers and the two lane halves: a per-step total in every lane.
__device__ __forceinline__ double step_sum(double v)
{
    return v + __shfl_xor(v, 32, 64);
}

template <int MK, bool tangent>
__global__ void __launch_bounds__(kNT, 1) k_eval_hmc_logreg(EvalArgs a, HmcLogregArgs t)
{
    extern __shared__ float sm[];
    const int NR = (t.N + 31) / 32 * 32;
    const Lds l = lds_layout(sm, NR, t.ldx);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 31, h = lane >> 5;
    const int D = t.D, L = a.hmc_L;
    const float eps = (float)a.eps, pp = t.pp;
    if (a.glob && a.glob->n_active == 0) return;

    for (int k = tid; k < NR * t.ldx; k += kNT) l.X[k] = k < t.N * t.ldx ? t.X[k] : 0.f;
    for (int k = tid; k < NR; k += kNT) l.y[k] = k < t.N ? t.y[k] : 0.f;
    __syncthreads();

    // tangent: the probe direction of the one-probe diagonal (Picard needs none)
    const float *im = (const float *)a.inv_mass;
    // this wave's two coordinates of step i (register slice r = 2w, 2w + 1)
    int dq[2];
    bool oq[2];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        dq[q] = crow(2 * w + q, h);
        oq[q] = dq[q] < D;
    }
    for (int tix = blockIdx.x; tix < a.n_tiles; tix += gridDim.x) {
        const SegTile tl = a.tiles[tix];
        const ChainStatus &cs = a.chains[tl.chain];
        if (!cs.active || tl.start + tl.len <= cs.win_start || tl.start >= cs.win_end) continue;  // uniform
        const int64_t tstep = tl.start + i;
        const bool valid = i < tl.len && tstep >= cs.win_start && tstep < cs.win_end;
        const int64_t tt = i < tl.len ? tstep : tl.start;
        const bool head = tt == a.offsets[tl.chain];
        const float *s0 = (const float *)a.s0 + (size_t)tl.chain * D;
        const float *S = (const float *)a.S;
        const float *noise = (const float *)a.noise;
        const uint64_t hsd = probe_mix(probe_mix(a.probe_seed) ^ (uint64_t)(uint32_t)cs.sweeps);

        // the transitions' state for this wave's coordinates
        float x0[2], v0[2], v[2], dl[2], z[2], xd[2], vd[2], imv[2], g[2], hv[2];
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const int d = dq[q];
            x0[q] = oq[q] ? (head ? s0[d] : S[(size_t)d * a.ld + tt - 1]) : 0.f;
            imv[q] = oq[q] ? (im ? im[d] : 1.f) : 0.f;
            v0[q] = oq[q] ? noise[(size_t)tt * D + d] / sqrtf(im ? im[d] : 1.f) : 0.f;
            z[q] = oq[q] ? ((probe_mix(hsd ^ (uint64_t)(1024 * tt + d)) >> 63) ? -1.f : 1.f) : 0.f;
            l.P[i * kPS + d] = x0[q];
            l.Pd[i * kPS + d] = z[q];
            dl[q] = 0.f;
            xd[q] = z[q];
        }
        __syncthreads();
        float gs[2], hs[2];
        evaluate<MK, tangent, true, true>(l, t, NR, w, lane, gs, hs);
        double g0z = 0.0;  // g(x0) . z, for the relaxed gate's directional derivative
#pragma unroll
        for (int q = 0; q < 2; q++) {
            g[q] = gs[q] - pp * x0[q];
            hv[q] = -hs[q] - pp * z[q];
            v[q] = fmaf(0.5f * eps, g[q], v0[q]);
            vd[q] = 0.5f * eps * hv[q];
            g0z = fma((double)g[q], (double)z[q], g0z);
        }
        for (int s = 0; s < L; s++) {
#pragma unroll
            for (int q = 0; q < 2; q++) {
                dl[q] = fmaf(eps * imv[q], v[q], dl[q]);
                xd[q] = fmaf(eps * imv[q], vd[q], xd[q]);
                l.P[i * kPS + dq[q]] = x0[q] + dl[q];
                l.Pd[i * kPS + dq[q]] = xd[q];
            }
            __syncthreads();
            evaluate<MK, tangent, true, true>(l, t, NR, w, lane, gs, hs);
#pragma unroll
            for (int q = 0; q < 2; q++) {
                g[q] = gs[q] - pp * (x0[q] + dl[q]);
                hv[q] = -hs[q] - pp * xd[q];
                v[q] = fmaf(eps, g[q], v[q]);
                vd[q] = fmaf(eps, hv[q], vd[q]);
            }
        }
        // per-step partial sums over this wave's coordinates (FP64): kinetic and
        // prior parts of H0 - HL, and the relaxed gate's directional derivative
        double kin = 0.0, prior = 0.0, dgd = -g0z;
#pragma unroll
        for (int q = 0; q < 2; q++) {
            const float vf = fmaf(-0.5f * eps, g[q], v[q]);
            const float vdf = fmaf(-0.5f * eps, hv[q], vd[q]);
            const float xl = x0[q] + dl[q];
            kin = fma((double)imv[q] * (double)(v0[q] - vf), (double)(v0[q] + vf), kin);
            prior = fma((double)dl[q], (double)xl + (double)x0[q], prior);
            dgd += -(double)imv[q] * vf * vdf + (double)g[q] * xd[q];
            l.P[i * kPS + dq[q]] = x0[q];
            l.Pd[i * kPS + dq[q]] = dl[q];
        }
        kin = step_sum(kin);
        prior = step_sum(prior);
        dgd = step_sum(dgd);
        __syncthreads();
        // log-likelihood difference through the exact increment: Z0 = X x0, dZ = X dl
        double ll = 0.0;
        for (int rt = w; 32 * rt < NR; rt += kW) {
            f32x16 Z0, dZ;
            fwd_products<MK, true>(l, t.ldx, D, rt, i, h, Z0, dZ);
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const float yv = l.y[32 * rt + crow(r, h)];
                const float sg = sigm(Z0[r]);
                ll += (double)(yv * dZ[r]) - (double)softplus_diff_h(Z0[r], dZ[r], sg);
            }
        }
        ll = step_sum(ll);
        // per-step totals over the waves, in a fixed order: [4][kW][32] doubles
        double *rd = l.red;
        if (h == 0) {
            rd[(0 * kW + w) * 32 + i] = ll;
            rd[(1 * kW + w) * 32 + i] = kin;
            rd[(2 * kW + w) * 32 + i] = prior;
            rd[(3 * kW + w) * 32 + i] = dgd;
        }
        __syncthreads();
        double tot[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int k = 0; k < 4; k++)
#pragma unroll
            for (int ww = 0; ww < kW; ww++) tot[k] += rd[(k * kW + ww) * 32 + i];
        __syncthreads();  // the totals are read before the next tile rewrites them
        const double dh = 0.5 * tot[1] + tot[0] - 0.5 * (double)pp * tot[2];  // H0 - HL
        const double la = dh < 0.0 ? dh : 0.0;
        const double gd = valid ? la - log((double)((const float *)a.unif)[tt]) : 0.0;
        int acc = gd > 0.0 && dh == dh;
        if (valid) acc = sticky_decision(a, cs, tstep, gd, acc);
        if (valid) {
            const bool surr = a.gate == PMC_GATE_SURROGATE && dh < 0.0;
            float coef = 0.f;
            if (surr) {
                const float sg = 1.f / (1.f + expf(-(float)gd));
                coef = sg * (1.f - sg);
            }
            float *F = (float *)a.F, *J = (float *)a.J;
#pragma unroll
            for (int q = 0; q < 2; q++) {
                if (!oq[q]) continue;
                const int d = dq[q];
                F[(size_t)d * a.ld + tstep] = acc ? x0[q] + dl[q] : x0[q];
                if (tangent) {
                    float jz = acc ? xd[q] : z[q];
                    if (surr) jz = fmaf(coef * dl[q], (float)tot[3], jz);
                    float jv = (float)a.damping * (z[q] * jz);
                    if (a.clip > 0) jv = fminf(fmaxf(jv, (float)-a.clip), (float)a.clip);
                    J[(size_t)d * a.ld + tstep] = jv;
                }
            }
            if (w == 0 && h == 0) {
                if (a.accept) a.accept[tstep] = (uint8_t)acc;
                if (a.gtilde) a.gtilde[tstep] = (float)gd;
            }
        }
    }
}

// ------------------------------------------- relaxed MALA gate (Sec. 3.2)
// The stop-gradient gate's rank-one part of the MALA Jacobian on the
// logistic posterior, added to the diagonal the evaluation wrote (exact
// diagonal or the one-probe z o (J z)), which then receives the damping and
// the clip.  With x~ = x + delta, g = grad log p(x), g~ = grad log p(x~),
// w = -delta - eps g~ and M = I + eps H(x), the log ratio's gradient is
//   dl/dx = M g~ - g + (H(x) w + M H(x~) w) / 2,
// so the term is sigma'(g~ate) delta (dl/dx)^T where l < 0: its diagonal is
// sigma' delta_d (dl/dx)_d, its probe part sigma' z_d delta_d (dl/dx . z).
// The gradients and Hessian-vector products are the batched evaluations of
// the HMC kernel above (32 steps per tile, matrix cores).
template <int MK>
__global__ void __launch_bounds__(kNT, 1) k_logreg_surrogate(EvalArgs a, HmcLogregArgs t)
{
    extern __shared__ float sm[];
    const int NR = (t.N + 31) / 32 * 32;
    const Lds l = lds_layout(sm, NR, t.ldx);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63, i = lane & 31, h = lane >> 5;
    const int D = t.D;
    const float eps = (float)a.eps, pp = t.pp, c = sqrtf(2.f * eps);
    if (a.glob && a.glob->n_active == 0) return;
    for (int k = tid; k < NR * t.ldx; k += kNT) l.X[k] = k < t.N * t.ldx ? t.X[k] : 0.f;
    for (int k = tid; k < NR; k += kNT) l.y[k] = k < t.N ? t.y[k] : 0.f;
    __syncthreads();
    int dq[2];
    bool oq[2];
#pragma unroll
    for (int q = 0; q < 2; q++) {
        dq[q] = crow(2 * w + q, h);
        oq[q] = dq[q] < D;
    }
    for (int tix = blockIdx.x; tix < a.n_tiles; tix += gridDim.x) {
        const SegTile tl = a.tiles[tix];
        const ChainStatus &cs = a.chains[tl.chain];
        if (!cs.active || tl.start + tl.len <= cs.win_start || tl.start >= cs.win_end) continue;  // uniform
        const int64_t tstep = tl.start + i;
        const bool valid = i < tl.len && tstep >= cs.win_start && tstep < cs.win_end;
        const int64_t tt = i < tl.len ? tstep : tl.start;
        const bool head = tt == a.offsets[tl.chain];
        const float *s0 = (const float *)a.s0 + (size_t)tl.chain * D;
        const float *S = (const float *)a.S, *noise = (const float *)a.noise;
        float x[2], xi[2], g[2], dl[2], gt[2], wv[2], t1[2], dll[2], gs[2], hs[2];
        auto put = [&](const float (&p)[2], const float (&d)[2]) {
#pragma unroll
            for (int q = 0; q < 2; q++) {
                l.P[i * kPS + dq[q]] = p[q];
                l.Pd[i * kPS + dq[q]] = d[q];
            }
            __syncthreads();
        };
        const float zero[2] = {0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 2; q++) {
            x[q] = oq[q] ? (head ? s0[dq[q]] : S[(size_t)dq[q] * a.ld + tt - 1]) : 0.f;
            xi[q] = oq[q] ? noise[(size_t)tt * D + dq[q]] : 0.f;
        }
        put(x, zero);
        evaluate<MK, false>(l, t, NR, w, lane, gs, hs);
        float xt[2];
#pragma unroll
        for (int q = 0; q < 2; q++) {
            g[q] = gs[q] - pp * x[q];
            dl[q] = oq[q] ? fmaf(eps, g[q], c * xi[q]) : 0.f;
            xt[q] = x[q] + dl[q];
        }
        put(xt, zero);
        evaluate<MK, false>(l, t, NR, w, lane, gs, hs);
#pragma unroll
        for (int q = 0; q < 2; q++) {
            gt[q] = gs[q] - pp * xt[q];
            wv[q] = -dl[q] - eps * gt[q];
        }
        put(xt, wv);
        evaluate<MK, true, false>(l, t, NR, w, lane, gs, hs);  // the gradient at x~ is already in gt
#pragma unroll
        for (int q = 0; q < 2; q++) {
            t1[q] = -hs[q] - pp * wv[q];                     // H(x~) w
            dll[q] = gt[q] - g[q];
        }
        // H(x) applied to w, g~ and H(x~) w in one pass over the data (the
        // two later directions staged in the reduction buffer)
        {
            float *d2 = l.buf, *d3 = l.buf + 32 * kPS;
#pragma unroll
            for (int q = 0; q < 2; q++) {
                l.P[i * kPS + dq[q]] = x[q];
                l.Pd[i * kPS + dq[q]] = wv[q];
                d2[i * kPS + dq[q]] = gt[q];
                d3[i * kPS + dq[q]] = t1[q];
            }
            __syncthreads();
            float hw[2], hg[2], ht[2];
            evaluate_hvp3<MK>(l, t, NR, w, lane, d2, d3, hw, hg, ht);
#pragma unroll
            for (int q = 0; q < 2; q++) {
                dll[q] += 0.5f * (-hw[q] - pp * wv[q]);                           // H(x) w / 2
                dll[q] += eps * (-hg[q] - pp * gt[q]);                            // eps H(x) g~
                dll[q] += 0.5f * (t1[q] + eps * (-ht[q] - pp * t1[q]));           // M H(x~) w / 2
            }
        }
        // the probe part needs dl/dx . z per step: a fixed-order sum over the waves
        float zq[2] = {0.f, 0.f};
        double dz = 0.0;
        if (a.probes) {
            const uint64_t hsd = probe_mix(probe_mix(a.probe_seed) ^ (uint64_t)(uint32_t)cs.sweeps);
#pragma unroll
            for (int q = 0; q < 2; q++) {
                zq[q] = oq[q] ? ((probe_mix(hsd ^ (uint64_t)(1024 * tt + dq[q])) >> 63) ? -1.f : 1.f) : 0.f;
                dz = fma((double)dll[q], (double)zq[q], dz);
            }
            dz = step_sum(dz);
            if (h == 0) l.red[w * 32 + i] = dz;
            __syncthreads();
            dz = 0.0;
#pragma unroll
            for (int ww = 0; ww < kW; ww++) dz += l.red[ww * 32 + i];
            __syncthreads();
        }
        if (!valid) continue;
        const float u = ((const float *)a.unif)[tstep];
        const float gate = a.gtilde[tstep];
        // l < 0 (otherwise min(0, l) is the constant 0): the evaluation stored
        // g~ = (float)(min(0, l) - log u) with log u in FP64, so l >= 0 leaves
        // exactly (float)(-log u)
        const bool neg = gate < (float)(-log((double)u));
        const float sg = 1.f / (1.f + expf(-gate));
        const float coef = neg ? sg * (1.f - sg) : 0.f;
        float *J = (float *)a.J;
#pragma unroll
        for (int q = 0; q < 2; q++) {
            if (!oq[q]) continue;
            const size_t k = (size_t)dq[q] * a.ld + tstep;
            const float add = a.probes ? coef * zq[q] * dl[q] * (float)dz : coef * dl[q] * dll[q];
            float jv = (float)a.damping * (J[k] + add);
            if (a.clip > 0) jv = fminf(fmaxf(jv, (float)-a.clip), (float)a.clip);
            J[k] = jv;
        }
    }
}

// ------------------------------------------------------ sequential sampler
// One workgroup per chain; thread k owns data rows k, k + NT, ... (RPT of
// them) with their X rows in registers; wave 0 lanes d < D own coordinate d.
// Each gradient is a column sum through LDS in a fixed order.
template <int DM, int NT, int RPT>
__global__ void __launch_bounds__(NT) k_seq_hmc_logreg(SeqArgs a, const float *__restrict__ X,
                                                       const float *__restrict__ y, int N, float pp)
{
    constexpr int V = DM + 1;  // gradient components + one extra sum
    constexpr int VS = V + 1;
    constexpr int GRP = (V * 8 <= NT) ? 8 : 4;
    __shared__ float s_part[NT * VS];
    __shared__ double s_sumd[V];
    __shared__ float s_vec[DM], s_vec2[DM];
    __shared__ double s_w[NT / 64];
    __shared__ int s_acc;
    const int c = blockIdx.x, tid = threadIdx.x, lane = tid & 63;
    const int D = a.D, L = a.hmc_L;
    const int64_t t0 = a.offsets[c], t1 = a.offsets[c + 1];
    const float eps = (float)a.eps;
    const float *noise = (const float *)a.noise, *unif = (const float *)a.unif, *im = (const float *)a.inv_mass;
    float *out = (float *)a.out;
    const bool own = tid < 64 && lane < D;

    float xr[RPT][DM], yr[RPT], z0[RPT];
#pragma unroll
    for (int k = 0; k < RPT; k++) {
        const int n = tid + k * NT;
        const bool ok = n < N;
#pragma unroll
        for (int d = 0; d < DM; d++) xr[k][d] = ok ? X[(size_t)n * DM + d] : 0.f;
        yr[k] = ok ? y[n] : 0.f;
    }
    // column sums: v[0..DM) and v[DM] (the extra sum, FP64 across threads)
    auto column_sum = [&](float (&v)[V], double extra) {
#pragma unroll
        for (int q = 0; q < DM; q++) s_part[tid * VS + q] = v[q];
        lds_barrier_fn();
        if (tid < DM * GRP) {
            const int q = tid / GRP, p = tid % GRP;
            float s = 0.f;
            for (int r = p; r < NT; r += GRP) s += s_part[r * VS + q];
#pragma unroll
            for (int m = 1; m < GRP; m <<= 1) s += __shfl_xor(s, m, 64);
            if (p == 0) s_sumd[q] = s;
        }
        // the extra sum in FP64: wave partials, then wave 0
        double e = extra;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) e += __shfl_xor(e, m, 64);
        if (lane == 0) s_w[tid >> 6] = e;
        lds_barrier_fn();
        if (tid == 0) {
            double tot = 0.0;
            for (int k = 0; k < NT / 64; k++) tot += s_w[k];
            s_sumd[DM] = tot;
        }
        lds_barrier_fn();
    };
    // gradient of the log posterior at the position published in s_vec
    // (wave 0 lane d receives it); z_out receives the rows' predictors
    auto gradient = [&](float xpos, float (&zo)[RPT]) -> float {
        float v[V];
#pragma unroll
        for (int q = 0; q < V; q++) v[q] = 0.f;
#pragma unroll
        for (int k = 0; k < RPT; k++) {
            float zz = 0.f;
#pragma unroll
            for (int d = 0; d < DM; d++) zz = fmaf(xr[k][d], s_vec[d], zz);
            zo[k] = zz;
            const float r = yr[k] - sigm(zz);
#pragma unroll
            for (int d = 0; d < DM; d++) v[d] = fmaf(r, xr[k][d], v[d]);
        }
        column_sum(v, 0.0);
        return own ? (float)s_sumd[lane] - pp * xpos : 0.f;
    };

    float x = own ? ((const float *)a.s0)[(size_t)c * D + lane] : 0.f;
    const float imd = own && im ? im[lane] : 1.f;
    if (tid < DM) s_vec[tid] = tid < D ? ((const float *)a.s0)[(size_t)c * D + tid] : 0.f;
    __syncthreads();
    float g = gradient(x, z0);
    for (int64_t t = t0; t < t1; t++) {
        const float v0 = own ? noise[(size_t)t * D + lane] / sqrtf(imd) : 0.f;
        float v = fmaf(0.5f * eps, g, v0), dlv = 0.f, gl = g;
        float zl[RPT];
        for (int s = 0; s < L; s++) {
            if (tid < 64) {
                dlv = own ? fmaf(eps * imd, v, dlv) : 0.f;
                if (lane < DM) s_vec[lane] = x + dlv;
            }
            lds_barrier_fn();
            gl = gradient(x + dlv, zl);
            v = fmaf(eps, gl, v);
        }
        // H0 - HL: kinetic and prior parts in wave 0, log-likelihood through dl
        if (tid < 64 && lane < DM) s_vec2[lane] = own ? dlv : 0.f;
        lds_barrier_fn();
        double llp = 0.0;
        {
            float vz[V];
#pragma unroll
            for (int q = 0; q < V; q++) vz[q] = 0.f;
#pragma unroll
            for (int k = 0; k < RPT; k++) {
                float dz = 0.f;
#pragma unroll
                for (int d = 0; d < DM; d++) dz = fmaf(xr[k][d], s_vec2[d], dz);
                const float s = sigm(z0[k]);
                llp += (double)(yr[k] * dz) - (double)softplus_diff_h(z0[k], dz, s);
            }
            column_sum(vz, llp);
        }
        if (tid < 64) {
            const float vf = fmaf(-0.5f * eps, gl, v);
            const float xl = x + dlv;
            double kin = own ? (double)imd * (double)(v0 - vf) * (double)(v0 + vf) : 0.0;
            double pri = own ? (double)dlv * ((double)xl + (double)x) : 0.0;
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) {
                kin += __shfl_xor(kin, m, 64);
                pri += __shfl_xor(pri, m, 64);
            }
            const double dh = 0.5 * kin + s_sumd[DM] - 0.5 * (double)pp * pri;
            const double la = dh < 0.0 ? dh : 0.0;
            const double gd = la - log((double)unif[t]);
            const int acc = gd > 0.0 && dh == dh;
            if (acc) {
                x = xl;
                g = gl;
            }
            if (own) out[(size_t)t * D + lane] = x;
            if (lane == 0) {
                if (a.accept) a.accept[t] = (uint8_t)acc;
                if (a.gtilde) a.gtilde[t] = (float)gd;
                s_acc = acc;
            }
        }
        lds_barrier_fn();
        if (s_acc) {
#pragma unroll
            for (int k = 0; k < RPT; k++) z0[k] = zl[k];
        }
        // the next step starts from x with its gradient g and predictors z0
    }
}

}  // namespace

pmc_status launch_eval_hmc_logreg(pmc_context *ctx, const DevTarget &t, const EvalArgs &a)
{
    if (a.n_tiles == 0) return PMC_OK;
    const int NR0 = (t.n_data + 31) / 32 * 32;
    if (t.n_data > kMaxRowsHmc || t.dim > 32 || lds_bytes(NR0, t.ldx) > kLdsLimit) {
        set_error("HMC transitions on logistic regression hold X in LDS: n_data <= %d and %zu bytes <= %zu",
                  kMaxRowsHmc, lds_bytes(NR0, t.ldx), kLdsLimit);
        return PMC_ERR_UNSUPPORTED;
    }
    if (a.jmode != JM_DIAG && a.jmode != JM_NONE) {
        set_error("HMC transitions on logistic regression: one-probe diagonal or Picard only");
        return PMC_ERR_UNSUPPORTED;
    }
    const int NR = (t.n_data + 31) / 32 * 32;
    const size_t lds = lds_bytes(NR, t.ldx);
    HmcLogregArgs h{(const float *)t.X, (const float *)t.y, t.n_data, t.ldx, t.dim, (float)(1.0 / t.prior_var)};
    const int n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
    const unsigned grid = (unsigned)std::min<int64_t>(a.n_tiles, n_cu);
    auto go = [&](auto kern) -> pmc_status {
        PMC_TRY_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, ctx->stream, a, h);
        PMC_TRY_HIP(hipGetLastError());
        return PMC_OK;
    };
    const int mk = (t.dim + 1) / 2;
    const bool tg = a.jmode == JM_DIAG;
    if (mk <= 2) return tg ? go(k_eval_hmc_logreg<2, true>) : go(k_eval_hmc_logreg<2, false>);
    if (mk <= 4) return tg ? go(k_eval_hmc_logreg<4, true>) : go(k_eval_hmc_logreg<4, false>);
    if (mk <= 8) return tg ? go(k_eval_hmc_logreg<8, true>) : go(k_eval_hmc_logreg<8, false>);
    if (mk <= 13) return tg ? go(k_eval_hmc_logreg<13, true>) : go(k_eval_hmc_logreg<13, false>);
    return tg ? go(k_eval_hmc_logreg<16, true>) : go(k_eval_hmc_logreg<16, false>);
}

pmc_status launch_logreg_surrogate(pmc_context *ctx, const DevTarget &t, const EvalArgs &a)
{
    if (a.n_tiles == 0) return PMC_OK;
    const int NR = (t.n_data + 31) / 32 * 32;
    if (t.n_data > kMaxRowsHmc || t.dim > 32 || lds_bytes(NR, t.ldx) > kLdsLimit) {
        set_error("the relaxed gate on logistic regression holds X in LDS: n_data <= %d", kMaxRowsHmc);
        return PMC_ERR_UNSUPPORTED;
    }
    const size_t lds = lds_bytes(NR, t.ldx);
    HmcLogregArgs h{(const float *)t.X, (const float *)t.y, t.n_data, t.ldx, t.dim, (float)(1.0 / t.prior_var)};
    const int n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
    const unsigned grid = (unsigned)std::min<int64_t>(a.n_tiles, n_cu);
    auto go = [&](auto kern) -> pmc_status {
        PMC_TRY_HIP(hipFuncSetAttribute((const void *)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
        hipLaunchKernelGGL(kern, dim3(grid), dim3(kNT), lds, ctx->stream, a, h);
        PMC_TRY_HIP(hipGetLastError());
        return PMC_OK;
    };
    const int mk = (t.dim + 1) / 2;
    if (mk <= 2) return go(k_logreg_surrogate<2>);
    if (mk <= 4) return go(k_logreg_surrogate<4>);
    if (mk <= 8) return go(k_logreg_surrogate<8>);
    if (mk <= 13) return go(k_logreg_surrogate<13>);
    return go(k_logreg_surrogate<16>);
}

pmc_status launch_seq_hmc_logreg(pmc_context *ctx, const DevTarget &t, const SeqArgs &a)
{
    if (t.n_data > 4 * 256) {
        set_error("sequential HMC on logistic regression supports n_data <= 1024");
        return PMC_ERR_UNSUPPORTED;
    }
    const float pp = (float)(1.0 / t.prior_var);
    const float *X = (const float *)t.X, *y = (const float *)t.y;
    dim3 grid(a.n_chains), block(256);
    switch (t.ldx) {
    case 4: hipLaunchKernelGGL((k_seq_hmc_logreg<4, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
    case 8: hipLaunchKernelGGL((k_seq_hmc_logreg<8, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
    case 16: hipLaunchKernelGGL((k_seq_hmc_logreg<16, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
    case 25: hipLaunchKernelGGL((k_seq_hmc_logreg<25, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
    case 32: hipLaunchKernelGGL((k_seq_hmc_logreg<32, 256, 4>), grid, block, 0, ctx->stream, a, X, y, t.n_data, pp); break;
    default: set_error("logreg: unsupported padded dimension %d", t.ldx); return PMC_ERR_UNSUPPORTED;
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

}  // namespace pmc
