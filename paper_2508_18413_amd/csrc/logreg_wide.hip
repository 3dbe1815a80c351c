// Evaluation step of MALA on a Bayesian logistic-regression posterior of
// high dimension (32 < D <= 1024; the 768-dimensional embedding regression
// of Sec. 5.5), for every step of the active windows at once.
//
// With S the iterate (planes [D][ld], step t in column t) and X the design
// [N][D], one evaluation of the MALA transition (Sec. 3.2) for all steps t
// is five matrix products over the steps, each a tiled FP32 matrix-core
// GEMM with a fused epilogue (C[i][t] = sum_k P[i][k] Q[k][t]):
//   1. A  = X s_{t-1}              epilogue: R = y - sigma(A), W = sigma'(A)
//   2. G  = X^T R                  epilogue: g = G - s/v, Delta = eps g + sqrt(2 eps) xi
//   3. dA = X Delta                epilogue: R~ = y - sigma(A + dA); per step
//                                  sum_n y dA - (softplus(A + dA) - softplus(A))
//   4. G~ = X^T R~                 epilogue: per step |g + g~|^2, xi.(g + g~),
//                                  Delta.(s~ + s) (the proposal-density and
//                                  prior terms of the log Metropolis ratio)
//   5. decision per step (log ratio in FP64, gate, accept bit, g~)
//   6. H  = (X o X)^T W            epilogue: f_t = s + a Delta, and the
//                                  quasi-DEER diagonal a (1 + eps H_dd) + (1 - a)
//                                  with damping and clip
// The log-likelihood difference uses the increment dA = X Delta (exact to
// rounding of its own product), not the difference of two large predictors,
// and softplus(a + d) - softplus(a) = log(1 + sigma(a) (e^d - 1)).
//
// The GEMM: 256 threads (four waves as 2 x 2), a 128 x 128 output tile,
// K in steps of 32 through double-buffered LDS; each wave accumulates a
// 64 x 64 block as 2 x 2 v_mfma_f32_32x32x2f32 tiles.  Along the steps the
// tiles are the solver's evaluation tiles (one chain each, 128 steps), and
// a tile outside its chain's active window returns at once.
#include <math.h>

#include <algorithm>

#include "pmc_internal.hpp"

namespace pmc {
namespace {

typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kBI = 128, kBJ = 128, kBK = 32;
constexpr int kThreads = 256;
constexpr int kPS = kBK + 1;   // LDS row stride of the P tile (conflict-free column reads)
constexpr int kQS = kBJ + 32;  // LDS row stride of the Q tile (the two half-waves use disjoint banks)
constexpr int kStageFloats = kBI * kPS + kBK * kQS;

__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

enum WideMode { W_FWD = 0, W_GRAD = 1, W_DELTA = 2, W_GRADP = 3, W_HESS = 4, W_ROT = 5 };
// Q-operand forms: k-major planes Q[k][j]; the iterate shifted to s_{t-1}
// (s0 at a chain's first step); or a row-major matrix read transposed.
enum QForm { Q_PLANES = 0, Q_PREV = 1, Q_TRANS = 2 };

struct WideGemm {
    // C[i][j] = sum_k P[i][k] Q[k][j] for i < I, k < K
    const float *P;
    int64_t ldp;
    int I, K;
    const float *Q;
    int64_t ldq;
    int qform;
    // columns: evaluation tiles (one chain each) or, with tiles == nullptr,
    // the plain range [0, J)
    const SegTile *tiles;
    int64_t J;
    int64_t n_jtiles;
    const ChainStatus *chains;
    const int64_t *offsets;
    const float *s0;  // [n_chains][D] (Q_PREV and the epilogues' s_{t-1})
    const GlobalStatus *glob;
    // epilogue operands (per mode)
    float *out;       // W_ROT: row-major [I][ldo]
    int64_t ldo;
    int N, D;         // data points, coordinates (masks of the per-step sums and stores)
    int64_t ld;       // plane stride of every [rows][ld] buffer below
    const float *S;   // iterate planes [D][ld]
    const float *y;   // [Np] (zero past N)
    const float *xi;  // noise planes [D][ld]
    float *Abuf, *Rbuf, *Wbuf;  // [Np][ld]
    float *Gbuf, *Dbuf;         // [D][ld]
    double *part;     // per step and row tile: [n_itiles][parts][ld]
    float eps, c, pp; // step size, sqrt(2 eps), 1 / prior variance
    const uint8_t *accept;
    float *F, *Jd;    // planes [D][ld]
    float damp, clip;
    int want_j;
};

// Per-column context of a tile: global step, chain start, validity.
struct ColCtx {
    int64_t t;
    int valid;
    int head;
    int chain;
};

__device__ __forceinline__ float sigmoidf_(float a) { return 1.f / (1.f + __expf(-a)); }

// softplus(a + d) - softplus(a) = log(1 + sigma(a) (e^d - 1))
//                               = d + log(1 + sigma(-a) (e^-d - 1)),
// the first form for a <= 0 and the second for a > 0 (so that the sigmoid
// factor is at most 1/2 and the argument of log1p stays above -1/2 on the
// side where it is negative); accurate to the rounding of d itself when d is
// small.  Beyond |d| > 20 the direct difference.
__device__ __forceinline__ double softplus_inc(float a, float d)
{
    if (fabsf(d) > 20.f) {
        const float b = a + d;
        const double sb = (double)fmaxf(b, 0.f) + (double)log1pf(__expf(-fabsf(b)));
        const double sa = (double)fmaxf(a, 0.f) + (double)log1pf(__expf(-fabsf(a)));
        return sb - sa;
    }
    if (a <= 0.f) return (double)log1pf(sigmoidf_(a) * expm1f(d));
    return (double)d + (double)log1pf(sigmoidf_(-a) * expm1f(-d));
}

template <int MODE>
__device__ __forceinline__ constexpr int n_parts()
{
    return MODE == W_DELTA ? 1 : MODE == W_GRADP ? 3 : 0;
}

// s_{t-1}[d] for the step of column context cc
__device__ __forceinline__ float prev_state(const WideGemm &g, const ColCtx &cc, int d)
{
    return cc.head ? g.s0[(size_t)cc.chain * g.D + d] : g.S[(size_t)d * g.ld + cc.t - 1];
}

template <int MODE, int QF>
__global__ void __launch_bounds__(kThreads, 2) k_wide_gemm(WideGemm g)
{
    extern __shared__ float lds[];
    __shared__ ColCtx s_col[kBJ];
    if (g.glob && g.glob->n_active == 0) return;
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6, wi = w >> 1, wj = w & 1;
    const int jl = lane & 31, h = lane >> 5;
    // workgroup -> (row tile, column tile): consecutive workgroups go to the
    // eight XCDs in turn, so the row tiles of one column tile are given the
    // same XCD and share its L2 copy of the column panel
    const int n_it = (g.I + kBI - 1) / kBI;
    const int64_t slot = blockIdx.x >> 3;
    const int xcd = blockIdx.x & 7;
    const int it = (int)(slot % n_it);
    const int64_t jt = (slot / n_it) * 8 + xcd;
    if (jt >= g.n_jtiles) return;
    const int i0 = it * kBI;

    // ---- columns of this tile
    int64_t j0 = 0;
    int jlen = 0;
    if (g.tiles) {
        const SegTile tl = g.tiles[jt];
        const ChainStatus &cs = g.chains[tl.chain];
        if (!cs.active || tl.start + tl.len <= cs.win_start || tl.start >= cs.win_end) return;
        j0 = tl.start;
        jlen = tl.len;
        if (tid < kBJ) {
            ColCtx cc;
            cc.t = j0 + tid;
            cc.chain = tl.chain;
            cc.valid = tid < tl.len && cc.t >= cs.win_start && cc.t < cs.win_end;
            cc.head = tid < tl.len && cc.t == g.offsets[tl.chain];
            s_col[tid] = cc;
        }
    } else {
        j0 = jt * kBJ;
        jlen = (int)min<int64_t>(kBJ, g.J - j0);
        if (tid < kBJ) {
            ColCtx cc;
            cc.t = j0 + tid;
            cc.chain = 0;
            cc.valid = tid < jlen;
            cc.head = 0;
            s_col[tid] = cc;
        }
    }
    __syncthreads();

    // ---- operand staging.  P: in the evaluation (operands padded with zeros
    // to whole tiles) thread tid loads four float4 runs along k, rows
    // (tid >> 3) + 32 q; a rotation (unpadded rows) loads single elements,
    // rows pr0 + 8 q of column pk, masked.  Q: rows qr0 + 2 q of column qj,
    // from a per-thread base and stride (planes: the column's step, stride ld;
    // the iterate's previous step or s0 at a chain's first step; transposed:
    // a row, stride 1); a row past K or a column past the tile loads the
    // base and is replaced by zero when stored.
    constexpr bool kPadP = MODE != W_ROT;
    const int pk = tid & 31, pr0 = tid >> 5;
    const int pk4 = (tid & 7) * 4, pr4 = tid >> 3;
    const int qj = tid & 127, qr0 = tid >> 7;
    const ColCtx qcc = s_col[qj];
    const bool qval = qj < jlen;
    const float *qbase;
    int64_t qstride;
    if (QF == Q_PLANES) {
        qbase = g.Q + (qval ? qcc.t : j0);
        qstride = g.ldq;
    } else if (QF == Q_TRANS) {
        qbase = g.Q + (qval ? qcc.t : j0) * g.ldq;
        qstride = 1;
    } else {
        const bool hd = qval && qcc.head;
        qbase = hd ? g.s0 + (size_t)qcc.chain * g.D : g.Q + (qval ? qcc.t - 1 : 0);
        qstride = hd ? 1 : g.ldq;
    }
    const float *prow[16];
    if (kPadP) {
#pragma unroll
        for (int q = 0; q < 4; q++) prow[q] = g.P + (size_t)(i0 + pr4 + 32 * q) * g.ldp + pk4;
    } else {
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int i = min(i0 + pr0 + 8 * q, g.I - 1);
            prow[q] = g.P + (size_t)i * g.ldp;
        }
    }
    float pv[16], qv[16];
    auto load_stage = [&](int k0) {
        if (kPadP) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 v = *(const float4 *)(prow[q] + k0);
                pv[4 * q] = v.x;
                pv[4 * q + 1] = v.y;
                pv[4 * q + 2] = v.z;
                pv[4 * q + 3] = v.w;
            }
        } else {
            const int k = min(k0 + pk, g.K - 1);
#pragma unroll
            for (int q = 0; q < 16; q++) pv[q] = prow[q][k];
        }
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int kk = k0 + qr0 + 2 * q;
            qv[q] = qbase[(kk < g.K ? kk : 0) * qstride];
        }
    };
    auto store_stage = [&](int s, int k0) {
        float *Ps = lds + s * kStageFloats, *Qs = Ps + kBI * kPS;
        if (kPadP) {
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int e = 0; e < 4; e++) Ps[(pr4 + 32 * q) * kPS + pk4 + e] = pv[4 * q + e];
        } else {
            const bool kv = k0 + pk < g.K;
#pragma unroll
            for (int q = 0; q < 16; q++)
                Ps[(pr0 + 8 * q) * kPS + pk] = (kv && i0 + pr0 + 8 * q < g.I) ? pv[q] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 16; q++)
            Qs[(qr0 + 2 * q) * kQS + qj] = (qval && k0 + qr0 + 2 * q < g.K) ? qv[q] : 0.f;
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[a][b][r] = 0.f;

    const int nk = (g.K + kBK - 1) / kBK;
    load_stage(0);
    store_stage(0, 0);
    __syncthreads();
    for (int kt = 0; kt < nk; kt++) {
        const bool more = kt + 1 < nk;
        if (more) load_stage((kt + 1) * kBK);
        const float *Ps = lds + (kt & 1) * kStageFloats, *Qs = Ps + kBI * kPS;
#pragma unroll
        for (int kp = 0; kp < kBK / 2; kp++) {
            const int kk = 2 * kp + h;
            float af[2], bf[2];
#pragma unroll
            for (int a = 0; a < 2; a++) af[a] = Ps[(64 * wi + 32 * a + jl) * kPS + kk];
#pragma unroll
            for (int b = 0; b < 2; b++) bf[b] = Qs[kk * kQS + 64 * wj + 32 * b + jl];
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int b = 0; b < 2; b++)
                    acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x2f32(af[a], bf[b], acc[a][b], 0, 0, 0);
        }
        if (more) store_stage((kt + 1) & 1, (kt + 1) * kBK);
        __syncthreads();
    }

    // ---- epilogue: lane (jl, h) of block (a, b) holds C[i][jj] with
    // i = i0 + 64 wi + 32 a + crow(r, h), jj = 64 wj + 32 b + jl
    constexpr int NP = n_parts<MODE>();
    double psum[2][3];
#pragma unroll
    for (int b = 0; b < 2; b++)
#pragma unroll
        for (int p = 0; p < 3; p++) psum[b][p] = 0.0;
#pragma unroll
    for (int b = 0; b < 2; b++) {
        const int jj = 64 * wj + 32 * b + jl;
        const ColCtx cc = s_col[jj];
        if (!cc.valid) continue;
        const int64_t t = cc.t;
#pragma unroll
        for (int a = 0; a < 2; a++) {
#pragma unroll
            for (int r = 0; r < 16; r++) {
                const int i = i0 + 64 * wi + 32 * a + crow(r, h);
                const float v = acc[a][b][r];
                if (MODE == W_ROT) {
                    if (i < g.I) g.out[(size_t)i * g.ldo + t] = v;
                } else if (MODE == W_FWD) {
                    if (i < g.I) {
                        const float s = sigmoidf_(v);
                        g.Abuf[(size_t)i * g.ld + t] = v;
                        g.Rbuf[(size_t)i * g.ld + t] = g.y[i] - s;
                        g.Wbuf[(size_t)i * g.ld + t] = s * (1.f - s);
                    }
                } else if (MODE == W_GRAD) {
                    if (i < g.D) {
                        const float x = prev_state(g, cc, i);
                        const float gr = fmaf(-g.pp, x, v);
                        g.Gbuf[(size_t)i * g.ld + t] = gr;
                        g.Dbuf[(size_t)i * g.ld + t] = fmaf(g.eps, gr, g.c * g.xi[(size_t)i * g.ld + t]);
                    }
                } else if (MODE == W_DELTA) {
                    if (i < g.I) {
                        const float a0 = g.Abuf[(size_t)i * g.ld + t];
                        g.Rbuf[(size_t)i * g.ld + t] = g.y[i] - sigmoidf_(a0 + v);
                        if (i < g.N) psum[b][0] += (double)g.y[i] * (double)v - softplus_inc(a0, v);
                    }
                } else if (MODE == W_GRADP) {
                    if (i < g.D) {
                        const float x = prev_state(g, cc, i);
                        const float dl = g.Dbuf[(size_t)i * g.ld + t];
                        const float xt = x + dl;
                        const float gt = fmaf(-g.pp, xt, v);
                        const double sg = (double)g.Gbuf[(size_t)i * g.ld + t] + (double)gt;
                        psum[b][0] = fma(sg, sg, psum[b][0]);
                        psum[b][1] = fma((double)g.xi[(size_t)i * g.ld + t], sg, psum[b][1]);
                        psum[b][2] = fma((double)dl, (double)xt + (double)x, psum[b][2]);
                    }
                } else if (MODE == W_HESS) {
                    if (i < g.D) {
                        const float x = prev_state(g, cc, i);
                        const int ac = g.accept[t];
                        const float dl = g.Dbuf[(size_t)i * g.ld + t];
                        g.F[(size_t)i * g.ld + t] = ac ? x + dl : x;
                        if (g.want_j) {
                            float jv = ac ? g.damp * fmaf(g.eps, -v - g.pp, 1.f) : g.damp;
                            if (g.clip > 0.f) jv = fminf(fmaxf(jv, -g.clip), g.clip);
                            g.Jd[(size_t)i * g.ld + t] = jv;
                        }
                    }
                }
            }
        }
    }
    if (NP > 0) {
        // per step: the two half-waves, then the two waves along i, in a fixed order
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int p = 0; p < NP; p++) psum[b][p] += __shfl_xor(psum[b][p], 32, 64);
        // the operand stages are free after the main loop's last barrier
        double *s_red = (double *)lds;  // [NP][kBJ]
        if (wi == 1 && h == 0)
#pragma unroll
            for (int b = 0; b < 2; b++)
#pragma unroll
                for (int p = 0; p < NP; p++) s_red[p * kBJ + 64 * wj + 32 * b + jl] = psum[b][p];
        __syncthreads();
        if (wi == 0 && h == 0) {
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const int jj = 64 * wj + 32 * b + jl;
                const ColCtx cc = s_col[jj];
                if (!cc.valid) continue;
#pragma unroll
                for (int p = 0; p < NP; p++)
                    g.part[((size_t)it * NP + p) * g.ld + cc.t] = psum[b][p] + s_red[p * kBJ + jj];
            }
        }
    }
}

// Per step: the log Metropolis ratio from the row-tile sums, the gate, the
// decision (sticky within the tie band), the accept bit and g~.
struct DecideArgs {
    EvalArgs e;
    const double *part_dll;   // [n_it_n][ld]
    const double *part_q;     // [n_it_d][3][ld]
    int n_it_n, n_it_d;
    float pp;
};

__global__ void __launch_bounds__(kBJ) k_wide_decide(DecideArgs d)
{
    const EvalArgs &a = d.e;
    if (a.glob && a.glob->n_active == 0) return;
    const SegTile tl = a.tiles[blockIdx.x];
    const ChainStatus &cs = a.chains[tl.chain];
    const int64_t t = tl.start + threadIdx.x;
    if (!cs.active || (int)threadIdx.x >= tl.len || t < cs.win_start || t >= cs.win_end) return;
    int acc = 1;
    float gate = INFINITY;
    if (!a.ula) {
        double dll = 0.0, sn = 0.0, sx = 0.0, dpr = 0.0;
        for (int q = 0; q < d.n_it_n; q++) dll += d.part_dll[(size_t)q * a.ld + t];
        for (int q = 0; q < d.n_it_d; q++) {
            const double *p = d.part_q + (size_t)q * 3 * a.ld;
            sn += p[t];
            sx += p[a.ld + t];
            dpr += p[2 * a.ld + t];
        }
        const double ell = dll - 0.5 * (double)d.pp * dpr - 0.25 * a.eps * sn - sqrt(0.5 * a.eps) * sx;
        const double la = ell < 0.0 ? ell : 0.0;
        const double gd = la - log((double)((const float *)a.unif)[t]);
        gate = (float)gd;
        acc = gd > 0.0;
        if (!(ell == ell)) acc = 0;
        acc = sticky_decision(a, cs, t, gd, acc);
    }
    if (a.accept) a.accept[t] = (uint8_t)acc;
    if (a.gtilde) a.gtilde[t] = gate;
}

// Picard (no Jacobian): f_t = s_{t-1} + a_t Delta_t
__global__ void __launch_bounds__(kBJ) k_wide_f(EvalArgs a, const float *Dbuf)
{
    if (a.glob && a.glob->n_active == 0) return;
    const SegTile tl = a.tiles[blockIdx.x];
    const ChainStatus &cs = a.chains[tl.chain];
    const int64_t t = tl.start + threadIdx.x;
    if (!cs.active || (int)threadIdx.x >= tl.len || t < cs.win_start || t >= cs.win_end) return;
    const bool head = t == a.offsets[tl.chain];
    const float *S = (const float *)a.S, *s0 = (const float *)a.s0 + (size_t)tl.chain * a.D;
    float *F = (float *)a.F;
    const int ac = a.accept[t];
    for (int d = 0; d < a.D; d++) {
        const float x = head ? s0[d] : S[(size_t)d * a.ld + t - 1];
        F[(size_t)d * a.ld + t] = ac ? x + Dbuf[(size_t)d * a.ld + t] : x;
    }
}

// X^T and (X o X)^T from X [Np][Dp]
__global__ void k_wide_tables(const float *X, int Np, int Dp, float *XT, float *X2T)
{
    __shared__ float tile[32][33];
    const int n0 = blockIdx.x * 32, d0 = blockIdx.y * 32, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) tile[r][tx] = X[(size_t)(n0 + r) * Dp + d0 + tx];
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const float v = tile[tx][r];
        XT[(size_t)(d0 + r) * Np + n0 + tx] = v;
        X2T[(size_t)(d0 + r) * Np + n0 + tx] = v * v;
    }
}

// noise rows [n][D] -> planes [D][ld]
__global__ void k_rows_to_planes_f32(const float *in, int64_t n, int D, int64_t ld, float *out)
{
    __shared__ float tile[32][33];
    const int64_t t0 = (int64_t)blockIdx.x * 32;
    const int d0 = blockIdx.y * 32, tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
    for (int r = ty; r < 32; r += 8) {
        const int64_t t = t0 + r;
        tile[r][tx] = (t < n && d0 + tx < D) ? in[(size_t)t * D + d0 + tx] : 0.f;
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int d = d0 + r;
        const int64_t t = t0 + tx;
        if (d < D && t < n) out[(size_t)d * ld + t] = tile[tx][r];
    }
}

size_t gemm_lds() { return sizeof(float) * 2 * (size_t)kStageFloats; }

template <int MODE, int QF>
pmc_status launch_gemm(pmc_context *ctx, WideGemm g, int64_t n_jtiles)
{
    if (n_jtiles <= 0 || g.I <= 0) return PMC_OK;
    const int64_t n_it = (g.I + kBI - 1) / kBI;
    const int64_t blocks = (n_jtiles + 7) / 8 * 8 * n_it;
    PMC_REQUIRE(blocks <= 0x7fffffff, "wide logistic: %lld workgroups exceed the launch limit", (long long)blocks);
    g.n_jtiles = n_jtiles;
    PMC_TRY_HIP(hipFuncSetAttribute((const void *)k_wide_gemm<MODE, QF>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)gemm_lds()));
    hipLaunchKernelGGL((k_wide_gemm<MODE, QF>), dim3((unsigned)blocks), dim3(kThreads), gemm_lds(), ctx->stream, g);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

}  // namespace

int wide_pad(int n) { return (n + kBI - 1) / kBI * kBI; }
int wide_tile_steps() { return kBJ; }

namespace {
// workspace: A, R, W [Np][ld]; G, Delta, xi [D][ld]; row-tile sums
struct WideWs {
    float *A, *R, *W, *G, *Dl, *xi;
    double *part_dll, *part_q;
    size_t total;
};
WideWs wide_layout(void *base, const DevTarget &t, int64_t ld)
{
    const size_t np = (size_t)wide_pad(t.n_data), D = (size_t)t.dim;
    const size_t nid = (size_t)(wide_pad(t.dim) / kBI), nin = np / kBI;
    auto al = [](size_t b) { return align_up(b, 256); };
    char *p = (char *)base;
    size_t off = 0;
    auto take = [&](size_t b) {
        char *q = p ? p + off : nullptr;
        off += al(b);
        return q;
    };
    WideWs w;
    w.A = (float *)take(4 * np * ld);
    w.R = (float *)take(4 * np * ld);
    w.W = (float *)take(4 * np * ld);
    w.G = (float *)take(4 * D * ld);
    w.Dl = (float *)take(4 * D * ld);
    w.xi = (float *)take(4 * D * ld);
    w.part_dll = (double *)take(8 * nin * ld);
    w.part_q = (double *)take(8 * 3 * nid * ld);
    w.total = off;
    return w;
}
}  // namespace

size_t wide_workspace_bytes(const DevTarget &t, int64_t ld) { return wide_layout(nullptr, t, ld).total; }
float *wide_xi_planes(void *ws, const DevTarget &t, int64_t ld) { return wide_layout(ws, t, ld).xi; }

pmc_status logreg_wide_tables(pmc_context *ctx, DevTarget &t)
{
    const int Np = wide_pad(t.n_data), Dp = t.ldx;
    PMC_REQUIRE(Dp % kBI == 0 && Dp >= t.dim, "wide logistic: bad padded width %d", Dp);
    if (!t.xwt) PMC_TRY_HIP(hipMalloc(&t.xwt, sizeof(float) * (size_t)Np * Dp));
    if (!t.x2wt) PMC_TRY_HIP(hipMalloc(&t.x2wt, sizeof(float) * (size_t)Np * Dp));
    hipLaunchKernelGGL(k_wide_tables, dim3(Np / 32, Dp / 32), dim3(256), 0, ctx->stream, (const float *)t.X, Np, Dp,
                       (float *)t.xwt, (float *)t.x2wt);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status wide_rotate_rows(pmc_context *ctx, const float *in, int64_t rows, int64_t ld_in, const float *Q, int D,
                            bool transpose, float *out, int64_t ld_out)
{
    if (rows <= 0) return PMC_OK;
    // out[r][e] = sum_d in[r][d] Q[d][e]  (transpose: Q[e][d])
    WideGemm g{};
    g.P = in;
    g.ldp = ld_in;
    g.I = (int)std::min<int64_t>(rows, 0x7fffffff);
    PMC_REQUIRE(rows <= 0x7fffff80, "wide rotation: %lld rows", (long long)rows);
    g.K = D;
    g.Q = Q;
    g.ldq = D;
    g.J = D;
    g.out = out;
    g.ldo = ld_out;
    g.D = D;
    const int64_t nj = (D + kBJ - 1) / kBJ;
    // the epilogue stores C[i][t] at out[i * ldo + t] with t the column
    if (transpose) return launch_gemm<W_ROT, Q_TRANS>(ctx, g, nj);
    return launch_gemm<W_ROT, Q_PLANES>(ctx, g, nj);
}

pmc_status wide_rows_to_planes(pmc_context *ctx, const float *in, int64_t n, int D, int64_t ld, float *out)
{
    if (n <= 0) return PMC_OK;
    PMC_REQUIRE((n + 31) / 32 <= 0x7fffffff, "wide noise: %lld steps", (long long)n);
    hipLaunchKernelGGL(k_rows_to_planes_f32, dim3((unsigned)((n + 31) / 32), (unsigned)((D + 31) / 32)), dim3(256), 0,
                       ctx->stream, in, n, D, ld, out);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status launch_eval_logreg_wide(pmc_context *ctx, const DevTarget &t, const EvalArgs &a, void *ws)
{
    if (a.n_tiles == 0) return PMC_OK;
    PMC_REQUIRE(t.xwt && t.x2wt && t.ldx % kBI == 0, "wide logistic: target tables missing");
    const int Np = wide_pad(t.n_data), D = t.dim;
    const int64_t ld = a.ld;
    const WideWs w = wide_layout(ws, t, ld);
    float *Abuf = w.A, *Rbuf = w.R, *Wbuf = w.W, *Gbuf = w.G, *Dbuf = w.Dl;
    const float *xi_planes = w.xi;
    const int n_it_n = Np / kBI, n_it_d = t.ldx / kBI;
    double *part_dll = w.part_dll, *part_q = w.part_q;

    WideGemm g{};
    g.tiles = a.tiles;
    g.chains = a.chains;
    g.offsets = a.offsets;
    g.s0 = (const float *)a.s0;
    g.glob = a.glob;
    g.N = t.n_data;
    g.D = D;
    g.ld = ld;
    g.S = (const float *)a.S;
    g.y = (const float *)t.y;
    g.xi = xi_planes;
    g.Abuf = Abuf;
    g.Rbuf = Rbuf;
    g.Wbuf = Wbuf;
    g.Gbuf = Gbuf;
    g.Dbuf = Dbuf;
    g.eps = (float)a.eps;
    g.c = sqrtf(2.f * (float)a.eps);
    g.pp = (float)(1.0 / t.prior_var);
    g.accept = a.accept;
    g.F = (float *)a.F;
    g.Jd = (float *)a.J;
    g.damp = (float)a.damping;
    g.clip = (float)a.clip;
    g.want_j = a.jmode == JM_DIAG;
    const int64_t nj = a.n_tiles;

    // 1. predictors at s_{t-1}
    WideGemm g1 = g;
    g1.P = (const float *)t.X;
    g1.ldp = t.ldx;
    g1.I = Np;
    g1.K = D;
    g1.Q = (const float *)a.S;
    g1.ldq = ld;
    PMC_TRY((launch_gemm<W_FWD, Q_PREV>(ctx, g1, nj)));
    // 2. gradient at s_{t-1}, increment Delta
    WideGemm g2 = g;
    g2.P = (const float *)t.xwt;
    g2.ldp = Np;
    g2.I = D;
    g2.K = Np;
    g2.Q = Rbuf;
    g2.ldq = ld;
    PMC_TRY((launch_gemm<W_GRAD, Q_PLANES>(ctx, g2, nj)));
    if (!a.ula) {
        // 3. predictor increments and the log-likelihood difference
        WideGemm g3 = g;
        g3.P = (const float *)t.X;
        g3.ldp = t.ldx;
        g3.I = Np;
        g3.K = D;
        g3.Q = Dbuf;
        g3.ldq = ld;
        g3.part = part_dll;
        PMC_TRY((launch_gemm<W_DELTA, Q_PLANES>(ctx, g3, nj)));
        // 4. gradient at the proposal and the proposal-density terms
        WideGemm g4 = g2;
        g4.Q = Rbuf;
        g4.part = part_q;
        PMC_TRY((launch_gemm<W_GRADP, Q_PLANES>(ctx, g4, nj)));
    }
    // 5. decisions
    DecideArgs da;
    da.e = a;
    da.part_dll = part_dll;
    da.part_q = part_q;
    da.n_it_n = n_it_n;
    da.n_it_d = n_it_d;
    da.pp = g.pp;
    PMC_REQUIRE(nj <= 0x7fffffff, "wide logistic: too many tiles");
    hipLaunchKernelGGL(k_wide_decide, dim3((unsigned)nj), dim3(kBJ), 0, ctx->stream, da);
    PMC_TRY_HIP(hipGetLastError());
    // 6. f_t and the Jacobian diagonal
    if (a.jmode == JM_DIAG) {
        WideGemm g6 = g;
        g6.P = (const float *)t.x2wt;
        g6.ldp = Np;
        g6.I = D;
        g6.K = Np;
        g6.Q = Wbuf;
        g6.ldq = ld;
        PMC_TRY((launch_gemm<W_HESS, Q_PLANES>(ctx, g6, nj)));
    } else {
        hipLaunchKernelGGL(k_wide_f, dim3((unsigned)nj), dim3(kBJ), 0, ctx->stream, a, (const float *)Dbuf);
        PMC_TRY_HIP(hipGetLastError());
    }
    return PMC_OK;
}


// ------------------------------------------------------------------------
// The same-GPU sequential sampler for D > 32: the chain's steps in order,
// each step spread over the whole GPU.  nb workgroups (one cooperative
// launch, all resident) each own rpw data rows, whose slice of X stays in
// LDS.  Per step and chain, workgroup w computes for its rows the predictor
// increments dA = X Delta, the residuals at the proposal and its share of
// X^T R~ and of the log-likelihood difference, and publishes them; one grid
// barrier; then every workgroup sums all shares in the same fixed order, so
// each one takes the same decision and holds the same state (x, g, Delta)
// without a second barrier.  Partial sums are double-buffered by step
// parity.  Up to kSeqChains chains run in one launch.
namespace {

constexpr int kSeqThreads = 256, kSeqChains = 4;
constexpr size_t kSeqLdsLimit = 150 * 1024;

struct SeqWide {
    SeqArgs a;
    const float *X;     // [Np][ldx]
    const float *y;     // [Np]
    int N, ldx, D;
    float pp;
    int nb, rpw;        // workgroups, rows per workgroup
    int c0, nc;         // chains c0 .. c0 + nc - 1
    int64_t steps;      // longest chain of the group
    float *part;        // [2][kSeqChains][D + 1][nb]: workgroup w's share last
    uint32_t *ctr;      // grid barrier counter (zero at launch)
    uint32_t *abort_;   // set when a barrier wait times out
};

__device__ __forceinline__ double block_sum_d(double v, double *red)
{
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < kSeqThreads / 64; i++) s += red[i];
    return s;
}

// Grid barrier number b (1-based); false if it timed out or another
// workgroup gave up.
__device__ bool grid_barrier(const SeqWide &q, uint32_t b)
{
    __shared__ int s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __hip_atomic_fetch_add(q.ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t target = b * (uint32_t)q.nb;
        int ok = 1;
        for (uint32_t spin = 0;; spin++) {
            if (__hip_atomic_load(q.ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (__hip_atomic_load(q.abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u || spin > (1u << 24)) {
                __hip_atomic_store(q.abort_, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        s_ok = ok;
    }
    __syncthreads();
    return s_ok != 0;
}

__global__ void __launch_bounds__(kSeqThreads) k_seq_logreg_wide(SeqWide q)
{
    extern __shared__ float sm[];
    __shared__ double s_red[kSeqThreads / 64];
    __shared__ int s_acc[kSeqChains];
    const int D = q.D, ldx = q.ldx, rpw = q.rpw, nc = q.nc, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r0 = blockIdx.x * rpw;
    float *sX = sm;                                  // [rpw][ldx]
    float *sx = sX + (size_t)rpw * ldx;              // [nc][D] x
    float *sg = sx + (size_t)kSeqChains * D;         // [nc][D] gradient at x
    float *sdl = sg + (size_t)kSeqChains * D;        // [nc][D] Delta
    float *sgt = sdl + (size_t)kSeqChains * D;       // [nc][D] gradient at the proposal
    float *sa = sgt + (size_t)kSeqChains * D;        // [nc][rpw] predictors of own rows at x
    float *sat = sa + kSeqChains * rpw;              // [nc][rpw] at the proposal
    float *sr = sat + kSeqChains * rpw;              // [nc][rpw] residuals
    const float eps = (float)q.a.eps, cc = sqrtf(2.f * eps);
    const float *noise = (const float *)q.a.noise, *unif = (const float *)q.a.unif;
    const int64_t *offs = q.a.offsets;
    float *out = (float *)q.a.out;
    const int nb = q.nb;
    // share of workgroup w in value v (0..D-1: X^T r, D: log-likelihood difference) of chain c
    auto pidx = [&](int buf, int c, int v, int w) {
        return (((size_t)buf * kSeqChains + c) * ((size_t)D + 1) + v) * nb + w;
    };

    for (int o = tid; o < rpw * ldx; o += kSeqThreads) sX[o] = q.X[(size_t)r0 * ldx + o];
    for (int c = 0; c < nc; c++)
        for (int d = tid; d < D; d += kSeqThreads) sx[c * D + d] = ((const float *)q.a.s0)[(size_t)(q.c0 + c) * D + d];
    __syncthreads();

    // predictors of own rows for the rows' share of a product with X
    auto row_dots = [&](const float *vec, float *dst) {
        for (int pr = wv; pr < nc * rpw; pr += kSeqThreads / 64) {
            const int c = pr / rpw, r = pr % rpw;
            float acc = 0.f;
            for (int d = lane; d < D; d += 64) acc = fmaf(sX[(size_t)r * ldx + d], vec[c * D + d], acc);
            for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
            if (lane == 0) dst[c * rpw + r] = acc;
        }
    };
    // this workgroup's share of X^T r
    auto share_xtr = [&](int buf, const float *rr) {
        for (int c = 0; c < nc; c++)
            for (int d = tid; d < D; d += kSeqThreads) {
                float acc = 0.f;
                for (int r = 0; r < rpw; r++) acc = fmaf(sX[(size_t)r * ldx + d], rr[c * rpw + r], acc);
                q.part[pidx(buf, c, d, blockIdx.x)] = acc;
            }
    };
    // sum of all workgroups' shares of one value, in workgroup order
    // (nb is a multiple of 4: the shares are read as float4)
    auto gather = [&](int buf, int c, int v) {
        const float4 *pb = (const float4 *)(q.part + pidx(buf, c, v, 0));
        float s = 0.f;
        for (int w = 0; w < nb / 4; w++) {
            const float4 u = pb[w];
            s += u.x;
            s += u.y;
            s += u.z;
            s += u.w;
        }
        return s;
    };

    // ---- gradient at s0
    uint32_t bar = 0;
    row_dots(sx, sa);
    __syncthreads();
    for (int o = tid; o < nc * rpw; o += kSeqThreads) {
        const int r = o % rpw, n = r0 + r;
        sr[o] = n < q.N ? q.y[n] - 1.f / (1.f + __expf(-sa[o])) : 0.f;
    }
    __syncthreads();
    share_xtr(0, sr);
    if (!grid_barrier(q, ++bar)) return;
    for (int c = 0; c < nc; c++)
        for (int d = tid; d < D; d += kSeqThreads) sg[c * D + d] = fmaf(-q.pp, sx[c * D + d], gather(0, c, d));
    __syncthreads();

    for (int64_t k = 0; k < q.steps; k++) {
        const int buf = (int)((k + 1) & 1);
        // Delta for every chain that has step k
        for (int c = 0; c < nc; c++) {
            const int64_t t = offs[q.c0 + c] + k;
            const bool live = t < offs[q.c0 + c + 1];
            for (int d = tid; d < D; d += kSeqThreads)
                sdl[c * D + d] = live ? fmaf(eps, sg[c * D + d], cc * noise[(size_t)t * D + d]) : 0.f;
        }
        __syncthreads();
        row_dots(sdl, sat);  // dA of own rows
        __syncthreads();
        for (int c = 0; c < nc; c++) {
            double dl = 0.0;
            for (int r = tid; r < rpw; r += kSeqThreads) {
                const int n = r0 + r, o = c * rpw + r;
                const float a0 = sa[o], da = sat[o];
                if (n < q.N) {
                    sr[o] = q.y[n] - 1.f / (1.f + __expf(-(a0 + da)));
                    dl += (double)q.y[n] * (double)da - softplus_inc(a0, da);
                } else {
                    sr[o] = 0.f;
                }
                sat[o] = a0 + da;
            }
            dl = block_sum_d(dl, s_red);
            if (tid == 0) q.part[pidx(buf, c, D, blockIdx.x)] = (float)dl;
        }
        __syncthreads();
        share_xtr(buf, sr);
        if (!grid_barrier(q, ++bar)) return;
        // every workgroup: the ratio and decision of each chain, identically
        for (int c = 0; c < nc; c++) {
            const int64_t t = offs[q.c0 + c] + k;
            const bool live = t < offs[q.c0 + c + 1];
            double sn = 0.0, sxi = 0.0, dpr = 0.0;
            for (int d = tid; d < D; d += kSeqThreads) {
                const float x = sx[c * D + d], dl = sdl[c * D + d], xt = x + dl;
                const float gt = fmaf(-q.pp, xt, gather(buf, c, d));
                const double sgv = (double)sg[c * D + d] + (double)gt;
                sn = fma(sgv, sgv, sn);
                if (live) sxi = fma((double)noise[(size_t)t * D + d], sgv, sxi);
                dpr = fma((double)dl, (double)xt + (double)x, dpr);
                sgt[c * D + d] = gt;
            }
            sn = block_sum_d(sn, s_red);
            sxi = block_sum_d(sxi, s_red);
            dpr = block_sum_d(dpr, s_red);
            if (tid == 0) {
                double dll = 0.0;
                for (int w = 0; w < nb; w++) dll += (double)q.part[pidx(buf, c, D, w)];
                int acc = 1;
                float gate = INFINITY;
                if (!q.a.ula) {
                    const double ell = dll - 0.5 * (double)q.pp * dpr - 0.25 * q.a.eps * sn - sqrt(0.5 * q.a.eps) * sxi;
                    const double la = ell < 0.0 ? ell : 0.0;
                    const double gd = live ? la - log((double)unif[t]) : -1.0;
                    gate = (float)gd;
                    acc = gd > 0.0 && ell == ell;
                }
                if (!live) acc = 0;
                s_acc[c] = acc;
                if (live && blockIdx.x == 0) {
                    if (q.a.accept) q.a.accept[t] = (uint8_t)acc;
                    if (q.a.gtilde) q.a.gtilde[t] = gate;
                }
            }
            __syncthreads();
        }
        // state update (every workgroup) and the step's output (coordinates
        // spread over the workgroups)
        const int dpw = (D + q.nb - 1) / q.nb, d0 = blockIdx.x * dpw, d1 = min(D, d0 + dpw);
        for (int c = 0; c < nc; c++) {
            const int64_t t = offs[q.c0 + c] + k;
            const bool live = t < offs[q.c0 + c + 1];
            const int acc = s_acc[c];
            if (acc) {
                for (int d = tid; d < D; d += kSeqThreads) {
                    sx[c * D + d] = sx[c * D + d] + sdl[c * D + d];
                    sg[c * D + d] = sgt[c * D + d];
                }
                for (int r = tid; r < rpw; r += kSeqThreads) sa[c * rpw + r] = sat[c * rpw + r];
            }
            __syncthreads();
            if (live)
                for (int d = d0 + tid; d < d1; d += kSeqThreads) out[(size_t)t * D + d] = sx[c * D + d];
        }
        __syncthreads();
    }
}

struct SeqPlan {
    int rpw = 0, nb = 0;
    size_t lds = 0;
};

SeqPlan seq_plan(const DevTarget &t)
{
    SeqPlan p;
    const int Np = wide_pad(t.n_data);
    for (int r : {32, 16, 8, 4}) {
        const int nb = Np / r;
        const size_t lds = sizeof(float) * ((size_t)r * t.ldx + 4 * (size_t)kSeqChains * t.dim + 3 * kSeqChains * r);
        if (Np % r == 0 && nb % 4 == 0 && nb <= 256 && lds <= kSeqLdsLimit) {
            p.rpw = r;
            p.nb = nb;
            p.lds = lds;
            break;
        }
    }
    return p;
}

}  // namespace

size_t seq_scratch_bytes(const DevTarget &t, int n_chains)
{
    (void)n_chains;
    if (t.kind != PMC_TARGET_LOGREG || t.dim < kWideMinDim) return 0;
    const SeqPlan p = seq_plan(t);
    if (!p.nb) return 0;
    return 256 + sizeof(float) * 2 * kSeqChains * ((size_t)t.dim + 1) * p.nb;
}

pmc_status launch_sequential_logreg_wide(pmc_context *ctx, const DevTarget &t, const SeqArgs &a)
{
    const SeqPlan p = seq_plan(t);
    if (!p.nb) {
        set_error("sequential logistic sampler: N = %d, D = %d do not fit the per-workgroup data slices",
                  t.n_data, t.dim);
        return PMC_ERR_UNSUPPORTED;
    }
    PMC_REQUIRE(a.scratch && a.host_offsets, "sequential logistic sampler: scratch and host offsets required");
    int coop = 0;
    PMC_TRY_HIP(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, ctx->device));
    if (!coop) {
        set_error("sequential logistic sampler (D > 32) needs cooperative launches");
        return PMC_ERR_UNSUPPORTED;
    }
    uint32_t *ctr = (uint32_t *)a.scratch, *abort_ = ctr + 1;
    float *part = (float *)((char *)a.scratch + 256);
    PMC_TRY_HIP(hipFuncSetAttribute((const void *)k_seq_logreg_wide, hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)p.lds));
    PMC_TRY_HIP(hipMemsetAsync(abort_, 0, sizeof(uint32_t), ctx->stream));
    for (int c0 = 0; c0 < a.n_chains; c0 += kSeqChains) {
        SeqWide q;
        q.a = a;
        q.X = (const float *)t.X;
        q.y = (const float *)t.y;
        q.N = t.n_data;
        q.ldx = t.ldx;
        q.D = t.dim;
        q.pp = (float)(1.0 / t.prior_var);
        q.nb = p.nb;
        q.rpw = p.rpw;
        q.c0 = c0;
        q.nc = std::min(kSeqChains, a.n_chains - c0);
        q.steps = 0;
        for (int c = c0; c < c0 + q.nc; c++)
            q.steps = std::max<int64_t>(q.steps, a.host_offsets[c + 1] - a.host_offsets[c]);
        q.part = part;
        q.ctr = ctr;
        q.abort_ = abort_;
        if (q.steps == 0) continue;
        PMC_TRY_HIP(hipMemsetAsync(ctr, 0, sizeof(uint32_t), ctx->stream));
        void *args[] = {&q};
        PMC_TRY_HIP(hipLaunchCooperativeKernel((const void *)k_seq_logreg_wide, dim3(p.nb), dim3(kSeqThreads), args,
                                               (unsigned)p.lds, ctx->stream));
    }
    uint32_t h_abort = 0;
    PMC_TRY_HIP(hipMemcpyAsync(&h_abort, abort_, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (h_abort) {
        set_error("sequential logistic sampler: a grid barrier timed out");
        return PMC_ERR_HIP;
    }
    return PMC_OK;
}

}  // namespace pmc
