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
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

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
    // split K (narrow windows, where a launch has few output tiles): the
    // kernel's phase 1 computes slice blockIdx.y of ksplit slices of K into
    // kpart planes [ksplit][ipad][ldk], whose columns are the compact grid's
    // (column kBJ s + j of window tile slot s); phase 2 sums the slices in order and
    // runs the epilogue; phase 0 is the whole product in one launch
    int ksplit;
    int64_t ipad, ldk;
    float *kpart;
    // fixed-width windows: with win_tiles > 0 the grid covers only the
    // win_tiles evaluation tiles of each chain from the one holding its
    // window start (ctile0[c]: the chain's first tile, [n_chains + 1])
    const int32_t *ctile0;
    int win_tiles;
    int n_chains;
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

template <int MODE, int QF, int PH>
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
    int it;
    int64_t jt, kslot = 0;
    if (g.win_tiles > 0) {
        // compact grid: workgroup -> (row tile, chain, k-th tile of its window)
        it = (int)(blockIdx.x % n_it);
        const int64_t rest = blockIdx.x / n_it;
        kslot = rest;
        const int c = (int)(rest / g.win_tiles);
        const ChainStatus &cs = g.chains[c];
        if (!cs.active) return;
        jt = g.ctile0[c] + (cs.win_start / kBJ - g.offsets[c] / kBJ) + rest % g.win_tiles;
        if (jt >= g.ctile0[c + 1]) return;
    } else {
        const int64_t slot = blockIdx.x >> 3;
        it = (int)(slot % n_it);
        jt = (slot / n_it) * 8 + (blockIdx.x & 7);
        if (jt >= g.n_jtiles) return;
    }
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
    // two register sets: the loads of stage kt + 2 are issued before the
    // products of stage kt and stored to LDS after those of stage kt + 1
    float pv[2][16], qv[2][16];
    auto load_stage = [&](int r, int k0) {
        if (kPadP) {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float4 v = *(const float4 *)(prow[q] + k0);
                pv[r][4 * q] = v.x;
                pv[r][4 * q + 1] = v.y;
                pv[r][4 * q + 2] = v.z;
                pv[r][4 * q + 3] = v.w;
            }
        } else {
            const int k = min(k0 + pk, g.K - 1);
#pragma unroll
            for (int q = 0; q < 16; q++) pv[r][q] = prow[q][k];
        }
#pragma unroll
        for (int q = 0; q < 16; q++) {
            const int kk = k0 + qr0 + 2 * q;
            qv[r][q] = qbase[(kk < g.K ? kk : 0) * qstride];
        }
    };
    auto store_stage = [&](int r, int s, int k0) {
        float *Ps = lds + s * kStageFloats, *Qs = Ps + kBI * kPS;
        if (kPadP) {
#pragma unroll
            for (int q = 0; q < 4; q++)
#pragma unroll
                for (int e = 0; e < 4; e++) Ps[(pr4 + 32 * q) * kPS + pk4 + e] = pv[r][4 * q + e];
        } else {
            const bool kv = k0 + pk < g.K;
#pragma unroll
            for (int q = 0; q < 16; q++)
                Ps[(pr0 + 8 * q) * kPS + pk] = (kv && i0 + pr0 + 8 * q < g.I) ? pv[r][q] : 0.f;
        }
#pragma unroll
        for (int q = 0; q < 16; q++)
            Qs[(qr0 + 2 * q) * kQS + qj] = (qval && k0 + qr0 + 2 * q < g.K) ? qv[r][q] : 0.f;
    };

    f32x16 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++)
#pragma unroll
            for (int r = 0; r < 16; r++) acc[a][b][r] = 0.f;
    auto compute = [&](int s) {
        const float *Ps = lds + s * kStageFloats, *Qs = Ps + kBI * kPS;
        if constexpr (MODE == W_HESS) {
            // the Hessian diagonal only enters the Jacobian, which sets the
            // Newton step and not the fixed point: BF16 products with FP32
            // accumulation, 16 k per instruction (lane half h takes k 8h..8h+7
            // of both operands)
#pragma unroll
            for (int kk = 0; kk < kBK / 16; kk++) {
                const int k0 = 16 * kk + 8 * h;
                bf16x8 af[2], bf[2];
#pragma unroll
                for (int a = 0; a < 2; a++) {
                    const float *pr = Ps + (64 * wi + 32 * a + jl) * kPS + k0;
#pragma unroll
                    for (int j = 0; j < 8; j++) af[a][j] = (__bf16)pr[j];
                }
#pragma unroll
                for (int b = 0; b < 2; b++)
#pragma unroll
                    for (int j = 0; j < 8; j++) bf[b][j] = (__bf16)Qs[(k0 + j) * kQS + 64 * wj + 32 * b + jl];
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int b = 0; b < 2; b++)
                        acc[a][b] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(af[a], bf[b], acc[a][b], 0, 0, 0);
            }
            return;
        }
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
    };

    // K tiles [kb, kb + nk) of this launch: all of them, or one slice
    const int nk_all = (g.K + kBK - 1) / kBK;
    int kb = 0, nk = nk_all;
    if (PH == 1) {
        const int per = (nk_all + g.ksplit - 1) / g.ksplit;
        kb = min(nk_all, (int)blockIdx.y * per);
        nk = min(nk_all, kb + per) - kb;
    } else if (PH == 2) {
        nk = 0;
    }
    if (nk > 0) {
        load_stage(0, kb * kBK);
        store_stage(0, 0, kb * kBK);
        if (nk > 1) load_stage(1, (kb + 1) * kBK);
        __syncthreads();
    }
    // stage kt lives in LDS buffer kt & 1 and arrives through register set kt & 1
    for (int kt = 0; kt < nk; kt += 2) {
        if (kt + 2 < nk) load_stage(0, (kb + kt + 2) * kBK);
        compute(0);
        if (kt + 1 < nk) store_stage(1, 1, (kb + kt + 1) * kBK);
        __syncthreads();
        if (kt + 1 < nk) {
            if (kt + 3 < nk) load_stage(1, (kb + kt + 3) * kBK);
            compute(1);
            if (kt + 2 < nk) store_stage(0, 0, (kb + kt + 2) * kBK);
            __syncthreads();
        }
    }
    if (PH == 1) {
        // this slice's partial products, for the valid columns
#pragma unroll
        for (int b = 0; b < 2; b++) {
            const ColCtx cc = s_col[64 * wj + 32 * b + jl];
            if (!cc.valid) continue;
#pragma unroll
            for (int a = 0; a < 2; a++)
#pragma unroll
                for (int r = 0; r < 16; r++) {
                    const int i = i0 + 64 * wi + 32 * a + crow(r, h);
                    if (i < g.I)
                        g.kpart[((size_t)blockIdx.y * g.ipad + i) * g.ldk + kslot * kBJ + 64 * wj + 32 * b + jl] =
                            acc[a][b][r];
                }
        }
        return;
    }
    if (PH == 2) {
        // the slices summed in order.  Every lane loads all 64 of its
        // elements of a slice unconditionally (a masked column or row reads
        // an in-range element that is then dropped), so a slice's loads are
        // in flight together instead of one branch and one round trip each.
        // (rows past I lie inside the slice planes, which have ipad rows)
        for (int ks = 0; ks < g.ksplit; ks++) {
            const float *src = g.kpart + (size_t)ks * g.ipad * g.ldk;
#pragma unroll
            for (int b = 0; b < 2; b++) {
                const ColCtx cc = s_col[64 * wj + 32 * b + jl];
                const float *col = src + kslot * kBJ + 64 * wj + 32 * b + jl + (size_t)(i0 + 64 * wi + 4 * h) * g.ldk;
                float v[2][16];
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int r = 0; r < 16; r++) v[a][r] = col[(size_t)(32 * a + crow(r, 0)) * g.ldk];
#pragma unroll
                for (int a = 0; a < 2; a++)
#pragma unroll
                    for (int r = 0; r < 16; r++) {
                        const int i = i0 + 64 * wi + 32 * a + crow(r, h);
                        if (cc.valid && i < g.I) acc[a][b][r] += v[a][r];
                    }
                asm volatile("" ::: "memory");
            }
        }
    }

    // ---- epilogue: lane (jl, h) of block (a, b) holds C[i][jj] with
    // i = i0 + 64 wi + 32 a + crow(r, h), jj = 64 wj + 32 b + jl.  Per block
    // (a, b) the operands of all 16 elements are gathered first, with
    // in-range addresses for masked elements (column j0, row clamped), and
    // only then combined and stored: loads placed after a store to a buffer
    // the compiler cannot prove disjoint would each wait for the previous
    // element's round trip.
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
        const bool cv = cc.valid;
        const int64_t t = cv ? cc.t : j0;
        // s_{t-1}: the chain's s0 at its first step, else the previous column of S
        const bool hd = cv && cc.head;
        const float *xp = hd ? g.s0 + (size_t)cc.chain * g.D : g.S + (t > 0 ? t - 1 : 0);
        const int64_t xs = hd ? 1 : g.ld;
        const int ac = (MODE == W_HESS) ? g.accept[t] : 0;
        // elements per gather: fewer where the combine step is long (the
        // log-likelihood increments), so that its temporaries fit in registers
        constexpr int GS = MODE == W_DELTA || MODE == W_GRADP ? 8 : 16;
#pragma unroll
        for (int ag = 0; ag < 32 / GS; ag++) {
            const int a = ag * GS / 16, r0 = ag * GS % 16;
            const int ib = i0 + 64 * wi + 32 * a;
            float o0[16], o1[16], o2[16], o3[16];
            // gather
#pragma unroll
            for (int r = r0; r < r0 + GS; r++) {
                const int i = ib + crow(r, h);
                const int ii = min(i, g.I - 1);
                const int id = min(i, g.D - 1);
                if (MODE == W_FWD) {
                    o0[r] = g.y[ii];
                } else if (MODE == W_GRAD) {
                    o0[r] = xp[(size_t)id * xs];
                    o1[r] = g.xi[(size_t)id * g.ld + t];
                } else if (MODE == W_DELTA) {
                    o0[r] = g.Abuf[(size_t)ii * g.ld + t];
                    o1[r] = g.y[ii];
                } else if (MODE == W_GRADP) {
                    o0[r] = xp[(size_t)id * xs];
                    o1[r] = g.Dbuf[(size_t)id * g.ld + t];
                    o2[r] = g.Gbuf[(size_t)id * g.ld + t];
                    o3[r] = g.xi[(size_t)id * g.ld + t];
                } else if (MODE == W_HESS) {
                    o0[r] = xp[(size_t)id * xs];
                    o1[r] = g.Dbuf[(size_t)id * g.ld + t];
                }
            }
            if (!cv) continue;
            // combine and store
#pragma unroll
            for (int r = r0; r < r0 + GS; r++) {
                const int i = ib + crow(r, h);
                const float v = acc[a][b][r];
                if (MODE == W_ROT) {
                    if (i < g.I) g.out[(size_t)i * g.ldo + t] = v;
                } else if (MODE == W_FWD) {
                    if (i < g.I) {
                        const float sg = sigmoidf_(v);
                        g.Abuf[(size_t)i * g.ld + t] = v;
                        g.Rbuf[(size_t)i * g.ld + t] = o0[r] - sg;
                        g.Wbuf[(size_t)i * g.ld + t] = sg * (1.f - sg);
                    }
                } else if (MODE == W_GRAD) {
                    if (i < g.D) {
                        const float gr = fmaf(-g.pp, o0[r], v);
                        g.Gbuf[(size_t)i * g.ld + t] = gr;
                        g.Dbuf[(size_t)i * g.ld + t] = fmaf(g.eps, gr, g.c * o1[r]);
                    }
                } else if (MODE == W_DELTA) {
                    if (i < g.I) {
                        const float a0 = o0[r];
                        g.Rbuf[(size_t)i * g.ld + t] = o1[r] - sigmoidf_(a0 + v);
                        if (i < g.N) psum[b][0] += (double)o1[r] * (double)v - softplus_inc(a0, v);
                    }
                } else if (MODE == W_GRADP) {
                    if (i < g.D) {
                        const float x = o0[r];
                        const float dl = o1[r];
                        const float xt = x + dl;
                        const float gt = fmaf(-g.pp, xt, v);
                        const double sg = (double)o2[r] + (double)gt;
                        psum[b][0] = fma(sg, sg, psum[b][0]);
                        psum[b][1] = fma((double)o3[r], sg, psum[b][1]);
                        psum[b][2] = fma((double)dl, (double)xt + (double)x, psum[b][2]);
                    }
                } else if (MODE == W_HESS) {
                    if (i < g.D) {
                        const float x = o0[r];
                        const float dl = o1[r];
                        g.F[(size_t)i * g.ld + t] = ac ? x + dl : x;
                        if (g.want_j) {
                            float jv = ac ? g.damp * fmaf(g.eps, -v - g.pp, 1.f) : g.damp;
                            if (g.clip > 0.f) jv = fminf(fmaxf(jv, -g.clip), g.clip);
                            g.Jd[(size_t)i * g.ld + t] = jv;
                        }
                    }
                }
            }
            // the next block's gathers are not hoisted above these stores
            asm volatile("" ::: "memory");
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
    const int64_t blocks =
        g.win_tiles > 0 ? (int64_t)g.n_chains * g.win_tiles * n_it : (n_jtiles + 7) / 8 * 8 * n_it;
    PMC_REQUIRE(blocks <= 0x7fffffff, "wide logistic: %lld workgroups exceed the launch limit", (long long)blocks);
    g.n_jtiles = n_jtiles;
    if (g.ksplit > 1 && g.kpart && g.win_tiles > 0) {
        PMC_TRY_HIP(hipFuncSetAttribute((const void *)k_wide_gemm<MODE, QF, 1>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds()));
        PMC_TRY_HIP(hipFuncSetAttribute((const void *)k_wide_gemm<MODE, QF, 2>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds()));
        hipLaunchKernelGGL((k_wide_gemm<MODE, QF, 1>), dim3((unsigned)blocks, (unsigned)g.ksplit), dim3(kThreads),
                           gemm_lds(), ctx->stream, g);
        hipLaunchKernelGGL((k_wide_gemm<MODE, QF, 2>), dim3((unsigned)blocks), dim3(kThreads), gemm_lds(),
                           ctx->stream, g);
    } else {
        PMC_TRY_HIP(hipFuncSetAttribute((const void *)k_wide_gemm<MODE, QF, 0>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)gemm_lds()));
        hipLaunchKernelGGL((k_wide_gemm<MODE, QF, 0>), dim3((unsigned)blocks), dim3(kThreads), gemm_lds(),
                           ctx->stream, g);
    }
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
    float *kpart;  // split-K slices [ksplit][max(Np, Dp)][kcols], or nullptr
    size_t total;
};
WideWs wide_layout(void *base, const DevTarget &t, int64_t ld, int ksplit, int64_t kcols)
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
    w.kpart = ksplit > 1 && kcols > 0 ? (float *)take(4 * (size_t)ksplit * std::max(np, (size_t)t.ldx) * kcols)
                                      : nullptr;
    w.total = off;
    return w;
}
}  // namespace

// columns of the compact window grid: each chain's window tiles
int64_t wide_window_cols(int64_t window_width, int n_chains)
{
    return window_width > 0 ? (int64_t)n_chains * ((window_width + kBJ - 1) / kBJ + 1) * kBJ : 0;
}
size_t wide_workspace_bytes(const DevTarget &t, int64_t ld, int ksplit, int64_t window_width, int n_chains)
{
    return wide_layout(nullptr, t, ld, ksplit, wide_window_cols(window_width, n_chains)).total;
}
float *wide_xi_planes(void *ws, const DevTarget &t, int64_t ld, int ksplit, int64_t window_width, int n_chains)
{
    return wide_layout(ws, t, ld, ksplit, wide_window_cols(window_width, n_chains)).xi;
}

int wide_ksplit(const DevTarget &t, int64_t window_width, int n_chains)
{
    // enough workgroups (about kSplitTarget) for the chip's 256 CUs
    constexpr int64_t kSplitTarget = 512, kSplitMax = 8;
    if (window_width <= 0) return 1;
    // output tiles of a launch: row tiles x the chains' active column tiles
    // (a window may straddle one more tile than its width covers)
    const int64_t n_it = std::max(wide_pad(t.n_data), t.ldx) / kBI;
    const int64_t cols = (int64_t)n_chains * ((window_width + kBJ - 1) / kBJ + 1);
    const int64_t ks = kSplitTarget / std::max<int64_t>(1, n_it * cols);
    return (int)std::min<int64_t>(kSplitMax, std::max<int64_t>(1, ks));
}

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
    const WideWs w = wide_layout(ws, t, ld, a.ksplit, wide_window_cols(a.window_width, a.n_chains));
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
    g.ksplit = w.kpart ? a.ksplit : 1;
    g.kpart = w.kpart;
    g.ipad = std::max(Np, t.ldx);
    g.ldk = wide_window_cols(a.window_width, a.n_chains);
    if (a.window_width > 0 && a.chain_etile_begin) {
        g.ctile0 = a.chain_etile_begin;
        g.win_tiles = (int)((a.window_width + kBJ - 1) / kBJ + 1);
        g.n_chains = a.n_chains;
    }
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
// LDS, and a slice of the coordinates.  Every workgroup keeps the whole
// state (x, grad log p(x), Delta) of each chain; per step and chain:
//   A. all: Delta = eps g + sqrt(2 eps) xi, the predictor increments of own
//      rows, residuals at the proposal; publish own share of X^T r~ (every
//      coordinate) and of the log-likelihood difference;
//   B. coordinate owners: sum the shares of own coordinates -> g~ there,
//      and own slice's sums for the proposal-density and prior terms;
//      publish them;
//   C. all: read g~ and the slice sums, take the decision (the same values
//      in the same order everywhere, so every workgroup decides alike) and
//      update the state.
// Shared words carry the step's tag in their upper half (agent-scope
// atomic 64-bit stores and loads); a reader waits until the tag matches,
// so no grid barrier and no cache flush is needed.  Words are
// double-buffered by tag parity: a workgroup cannot publish step k + 2
// before every workgroup has consumed step k.  Up to kSeqChains chains run
// in one launch.
namespace {

constexpr int kSeqThreads = 512, kSeqChains = 4;
constexpr size_t kSeqLdsLimit = 150 * 1024;
constexpr int kSeqQ = 6;  // slice sums: |g + g~|^2, xi.(g + g~), Delta.(x~ + x), each as two words

struct SeqWide {
    SeqArgs a;
    const float *X;     // [Np][ldx]
    const float *y;     // [Np]
    int N, ldx, D;
    float pp;
    int nb, rpw, dpw;   // workgroups, rows and coordinates per workgroup
    int c0, nc;         // chains c0 .. c0 + nc - 1
    int64_t steps;      // longest chain of the group
    uint64_t *p1;       // [2][nb][kSeqChains][D + 1] shares of X^T r~ and of the log-likelihood difference
    uint64_t *p2;       // [2][kSeqChains][D] g~
    uint64_t *p3;       // [2][nb][kSeqChains][kSeqQ] slice sums
    uint32_t *abort_;   // set when a wait times out
};

__device__ __forceinline__ uint64_t tagw(uint32_t tag, uint32_t bits) { return ((uint64_t)tag << 32) | bits; }
__device__ __forceinline__ void put(uint64_t *w, uint32_t tag, float v)
{
    __hip_atomic_store(w, tagw(tag, __float_as_uint(v)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Loads n tagged words (n <= 16) into v once all carry `tag`; false on a
// timeout or when another workgroup gave up.
template <int NMAX>
__device__ bool take(const SeqWide &q, const uint64_t *const *w, int n, uint32_t tag, float *v)
{
    uint32_t ready = 0;
    const uint32_t all = n >= 32 ? 0xffffffffu : ((1u << n) - 1u);
    for (uint32_t spin = 0;; spin++) {
#pragma unroll
        for (int i = 0; i < NMAX; i++) {
            if (i < n && !(ready >> i & 1u)) {
                const uint64_t x = __hip_atomic_load(w[i], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                if ((uint32_t)(x >> 32) == tag) {
                    v[i] = __uint_as_float((uint32_t)x);
                    ready |= 1u << i;
                }
            }
        }
        if (ready == all) return true;
        if (spin > (1u << 22) || __hip_atomic_load(q.abort_, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
            __hip_atomic_store(q.abort_, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return false;
        }
        __builtin_amdgcn_s_sleep(1);
    }
}

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

// the workgroup-wide AND of per-thread flags
__device__ __forceinline__ bool block_all(bool ok)
{
    return __syncthreads_and(ok ? 1 : 0) != 0;
}

__device__ __forceinline__ void put_d(uint64_t *w, uint32_t tag, double v)
{
    const uint64_t u = (uint64_t)__double_as_longlong(v);
    __hip_atomic_store(w, tagw(tag, (uint32_t)u), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(w + 1, tagw(tag, (uint32_t)(u >> 32)), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void __launch_bounds__(kSeqThreads) k_seq_logreg_wide(SeqWide q)
{
    extern __shared__ float sm[];
    __shared__ double s_red[kSeqThreads / 64];
    __shared__ double s_sum[kSeqChains][4];
    __shared__ int s_acc[kSeqChains];
    __shared__ int64_t s_t0[kSeqChains], s_t1[kSeqChains];
    __shared__ float s_y[32];
    const int D = q.D, ldx = q.ldx, rpw = q.rpw, nc = q.nc, nb = q.nb, tid = threadIdx.x;
    const int lane = tid & 63, wv = tid >> 6;
    const int r0 = blockIdx.x * rpw;
    const int d0 = min(D, (int)blockIdx.x * q.dpw), d1 = min(D, d0 + q.dpw);
    float *sX = sm;                                  // [rpw][ldx]
    float *sx = sX + (size_t)rpw * ldx;              // [kSeqChains][D] x
    float *sg = sx + (size_t)kSeqChains * D;         // [kSeqChains][D] gradient at x
    float *sdl = sg + (size_t)kSeqChains * D;        // [kSeqChains][D] Delta
    float *sgt = sdl + (size_t)kSeqChains * D;       // [kSeqChains][D] gradient at the proposal
    float *sa = sgt + (size_t)kSeqChains * D;        // [kSeqChains][rpw] predictors of own rows at x
    float *sat = sa + kSeqChains * rpw;              // [kSeqChains][rpw] at the proposal
    float *sr = sat + kSeqChains * rpw;              // [kSeqChains][rpw] residuals
    const float eps = (float)q.a.eps, cc = sqrtf(2.f * eps);
    const float *noise = (const float *)q.a.noise, *unif = (const float *)q.a.unif;
    const int64_t *offs = q.a.offsets;
    float *out = (float *)q.a.out;
    // word addresses (32-bit index arithmetic: every buffer holds < 2^31 words)
    uint64_t *const p1 = q.p1, *const p2 = q.p2, *const p3 = q.p3;
    const uint32_t D1 = (uint32_t)D + 1, ud = (uint32_t)D, unb = (uint32_t)nb;
    auto P1 = [=](uint32_t tag, int w, int c, int v) {
        return p1 + ((((tag & 1u) * unb + (uint32_t)w) * kSeqChains + (uint32_t)c) * D1 + (uint32_t)v);
    };
    auto P2 = [=](uint32_t tag, int c, int d) { return p2 + (((tag & 1u) * kSeqChains + (uint32_t)c) * ud + (uint32_t)d); };
    auto P3 = [=](uint32_t tag, int w, int c) {
        return p3 + ((((tag & 1u) * unb + (uint32_t)w) * kSeqChains + (uint32_t)c) * kSeqQ);
    };

    for (int o = tid; o < rpw * ldx; o += kSeqThreads) sX[o] = q.X[(size_t)r0 * ldx + o];
    for (int c = 0; c < nc; c++)
        for (int d = tid; d < D; d += kSeqThreads) sx[c * D + d] = ((const float *)q.a.s0)[(size_t)(q.c0 + c) * D + d];
    if (tid < nc) {
        s_t0[tid] = offs[q.c0 + tid];
        s_t1[tid] = offs[q.c0 + tid + 1];
    }
    if (tid < rpw) s_y[tid] = r0 + tid < q.N ? q.y[r0 + tid] : 0.f;
    __syncthreads();
    // the noise of the next step, in registers: xin at coordinates tid + 256 j,
    // xown at the own coordinate d0 + tid; the uniform in thread c
    float xin[kSeqChains][4], xown[kSeqChains], un = 0.f;
    auto load_xi = [&](int64_t k) {
#pragma unroll
        for (int c = 0; c < kSeqChains; c++) {
            const int64_t t = s_t0[c < nc ? c : 0] + k;
            const bool live = c < nc && t < s_t1[c < nc ? c : 0];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int d = tid + kSeqThreads * j;
                xin[c][j] = (live && d < D) ? noise[(size_t)t * D + d] : 0.f;
            }
            xown[c] = (live && tid < 64 && d0 + tid < d1) ? noise[(size_t)t * D + d0 + tid] : 0.f;
            if (tid == c && live && !q.a.ula) un = unif[t];
        }
    };

    // dst[c][r] = X_r . vec_c for own rows r: each wave takes eight (chain,
    // row) pairs at a time, lanes over the coordinates, eight independent
    // accumulators
    auto row_dots = [&](const float *vec, float *dst) {
        const int npairs = nc * rpw;
        for (int p0 = wv * 8; p0 < npairs; p0 += (kSeqThreads / 64) * 8) {
            float acc[8];
            int pc[8], pr[8];
#pragma unroll
            for (int i = 0; i < 8; i++) {
                const int pi = min(p0 + i, npairs - 1);
                pc[i] = pi / rpw;
                pr[i] = pi % rpw;
                acc[i] = 0.f;
            }
#pragma unroll 4
            for (int d = lane; d < D; d += 64) {
#pragma unroll
                for (int i = 0; i < 8; i++) acc[i] = fmaf(sX[(size_t)pr[i] * ldx + d], vec[pc[i] * D + d], acc[i]);
            }
#pragma unroll
            for (int i = 0; i < 8; i++) {
                float v = acc[i];
                for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
                if (lane == 0 && p0 + i < npairs) dst[pc[i] * rpw + pr[i]] = v;
            }
        }
    };
    // A: publish this workgroup's share of X^T r (every coordinate): thread
    // tid sums over own rows for coordinates tid + 256 j and every chain
    auto publish_share = [&](uint32_t tag, const float *rr) {
        float acc[kSeqChains][4];
#pragma unroll
        for (int c = 0; c < kSeqChains; c++)
#pragma unroll
            for (int j = 0; j < 4; j++) acc[c][j] = 0.f;
        // branch-free: chains past nc and coordinates past D read valid
        // elements, and their sums are never stored
        int cofs[kSeqChains], dcl[4];
#pragma unroll
        for (int c = 0; c < kSeqChains; c++) cofs[c] = min(c, nc - 1) * rpw;
#pragma unroll
        for (int j = 0; j < 4; j++) dcl[j] = min(tid + kSeqThreads * j, D - 1);
#pragma unroll 4
        for (int r = 0; r < rpw; r++) {
            float rv[kSeqChains];
#pragma unroll
            for (int c = 0; c < kSeqChains; c++) rv[c] = rr[cofs[c] + r];
            const float *xr = sX + (size_t)r * ldx;
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const float xv = xr[dcl[j]];
#pragma unroll
                for (int c = 0; c < kSeqChains; c++) acc[c][j] = fmaf(xv, rv[c], acc[c][j]);
            }
        }
        uint64_t *const base = P1(tag, blockIdx.x, 0, 0);  // chain c at base + c (D + 1)
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int d = tid + kSeqThreads * j;
            if (d < D) {
                uint64_t *w = base + d;
#pragma unroll
                for (int c = 0; c < kSeqChains; c++) {
                    if (c < nc) put(w, tag, acc[c][j]);
                    w += D1;
                }
            }
        }
    };
    // B: sums of own coordinates' shares (in workgroup order) into sgt
    auto reduce_own = [&](uint32_t tag) -> bool {
        bool ok = true;
        const int n_own = (d1 - d0) * nc;
        for (int o = tid; o < n_own; o += kSeqThreads) {
            const int c = o / (d1 - d0), d = d0 + o % (d1 - d0);
            float s = 0.f;
            for (int w0 = 0; w0 < nb && ok; w0 += 16) {
                const int n = min(16, nb - w0);
                const uint64_t *ws[16];
                float v[16];
#pragma unroll
                for (int i = 0; i < 16; i++) ws[i] = P1(tag, w0 + (i < n ? i : 0), c, d);
                ok = take<16>(q, ws, n, tag, v);
#pragma unroll
                for (int i = 0; i < 16; i++)
                    if (i < n) s += v[i];
            }
            sgt[c * D + d] = s;
        }
        return block_all(ok);
    };
    // C: every coordinate's reduced value from its owner, into dst
    auto gather_all = [&](uint32_t tag, float *dst) -> bool {
        bool ok = true;
        for (int o0 = 0; o0 < nc * D && ok; o0 += 16 * kSeqThreads) {
            const uint64_t *ws[16];
            float v[16];
            int n = 0;
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int o = o0 + i * kSeqThreads + tid;
                ws[i] = o < nc * D ? P2(tag, o / D, o % D) : P2(tag, 0, 0);
                if (o < nc * D) n = i + 1;
            }
            ok = take<16>(q, ws, n, tag, v);
#pragma unroll
            for (int i = 0; i < 16; i++) {
                const int o = o0 + i * kSeqThreads + tid;
                if (i < n && o < nc * D) dst[o] = v[i];
            }
        }
        return block_all(ok);
    };

    // ---- gradient at s0 (tag 1)
    row_dots(sx, sa);
    __syncthreads();
    for (int o = tid; o < nc * rpw; o += kSeqThreads) {
        const int r = o % rpw, n = r0 + r;
        sr[o] = n < q.N ? q.y[n] - 1.f / (1.f + __expf(-sa[o])) : 0.f;
    }
    __syncthreads();
    publish_share(1, sr);
    if (!reduce_own(1)) return;
    for (int o = tid; o < (d1 - d0) * nc; o += kSeqThreads) {
        const int c = o / (d1 - d0), d = d0 + o % (d1 - d0);
        put(P2(1, c, d), 1, fmaf(-q.pp, sx[c * D + d], sgt[c * D + d]));
    }
    if (!gather_all(1, sg)) return;

    load_xi(0);
    for (int64_t k = 0; k < q.steps; k++) {
        const uint32_t tag = (uint32_t)(k + 2);
        // ---- A
        for (int c = 0; c < nc; c++) {
            const bool live = s_t0[c] + k < s_t1[c];
#pragma unroll
            for (int j = 0; j < 4; j++) {
                const int d = tid + kSeqThreads * j;
                if (d < D) sdl[c * D + d] = live ? fmaf(eps, sg[c * D + d], cc * xin[c][j]) : 0.f;
            }
        }
        __syncthreads();
        row_dots(sdl, sat);
        __syncthreads();
        if (wv == 0) {
            // own rows (rpw <= 32): lanes 0..31 take chain c, lanes 32..63 chain c + 1
            for (int c2 = 0; c2 < nc; c2 += 2) {
                const int c = c2 + (lane >> 5), r = lane & 31;
                double dl = 0.0;
                if (r < rpw && c < nc) {
                    const int n = r0 + r, o = c * rpw + r;
                    const float a0 = sa[o], da = sat[o];
                    if (n < q.N) {
                        sr[o] = s_y[r] - 1.f / (1.f + __expf(-(a0 + da)));
                        dl = (double)s_y[r] * (double)da - softplus_inc(a0, da);
                    } else {
                        sr[o] = 0.f;
                    }
                    sat[o] = a0 + da;
                }
                for (int m = 16; m >= 1; m >>= 1) dl += __shfl_xor(dl, m, 64);
                if (r == 0 && c < nc) put(P1(tag, blockIdx.x, c, D), tag, (float)dl);
            }
        }
        __syncthreads();
        publish_share(tag, sr);
        // ---- B
        if (!reduce_own(tag)) return;
        if (wv == 0) {
            // own coordinates (at most 64) in lanes of wave 0
            for (int c = 0; c < nc; c++) {
                double sn = 0.0, sxi = 0.0, dpr = 0.0;
                const int d = d0 + lane;
                if (d < d1) {
                    const float x = sx[c * D + d], dl = sdl[c * D + d], xt = x + dl;
                    const float gt = fmaf(-q.pp, xt, sgt[c * D + d]);
                    put(P2(tag, c, d), tag, gt);
                    const double sgv = (double)sg[c * D + d] + (double)gt;
                    sn = sgv * sgv;
                    sxi = (double)xown[c] * sgv;
                    dpr = (double)dl * ((double)xt + (double)x);
                }
                for (int m = 32; m >= 1; m >>= 1) {
                    sn += __shfl_xor(sn, m, 64);
                    sxi += __shfl_xor(sxi, m, 64);
                    dpr += __shfl_xor(dpr, m, 64);
                }
                if (lane == 0) {
                    uint64_t *w = P3(tag, blockIdx.x, c);
                    put_d(w, tag, sn);
                    put_d(w + 2, tag, sxi);
                    put_d(w + 4, tag, dpr);
                }
            }
        }
        // ---- C: g~ everywhere; the slice sums and the log-likelihood shares
        // of every workgroup, summed in the same order in each workgroup.
        // The uniform of this step is kept; the next step's noise loads
        // while this workgroup waits.
        const float u_now = un;
        load_xi(k + 1);
        if (!gather_all(tag, sgt)) return;
        bool ok = true;
        double tot[4] = {0.0, 0.0, 0.0, 0.0};
        if (wv < nc) {
            const int c = wv;
            for (int w0 = lane; w0 < nb && ok; w0 += 64) {
                const uint64_t *ws[7];
                float v[7];
#pragma unroll
                for (int i = 0; i < kSeqQ; i++) ws[i] = P3(tag, w0, c) + i;
                ws[6] = P1(tag, w0, c, D);
                ok = take<7>(q, ws, 7, tag, v);
                auto dbl = [&](int i) {
                    return __longlong_as_double((long long)((uint64_t)__float_as_uint(v[i]) |
                                                            ((uint64_t)__float_as_uint(v[i + 1]) << 32)));
                };
                tot[0] += dbl(0);
                tot[1] += dbl(2);
                tot[2] += dbl(4);
                tot[3] += (double)v[6];
            }
#pragma unroll
            for (int i = 0; i < 4; i++)
                for (int m = 32; m >= 1; m >>= 1) tot[i] += __shfl_xor(tot[i], m, 64);
            if (lane == 0)
#pragma unroll
                for (int i = 0; i < 4; i++) s_sum[c][i] = tot[i];
        }
        if (!block_all(ok)) return;
        if (tid < nc) {
            const int c = tid;
            const int64_t t = s_t0[c] + k;
            const bool live = t < s_t1[c];
            const double sn = s_sum[c][0], sxi = s_sum[c][1], dpr = s_sum[c][2], dll = s_sum[c][3];
            int acc = 1;
            float gate = INFINITY;
            if (!q.a.ula) {
                const double ell = dll - 0.5 * (double)q.pp * dpr - 0.25 * q.a.eps * sn - sqrt(0.5 * q.a.eps) * sxi;
                const double la = ell < 0.0 ? ell : 0.0;
                const double gd = live ? la - log((double)u_now) : -1.0;
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
        // state update (every workgroup) and the step's output (own coordinates)
        for (int c = 0; c < nc; c++) {
            if (!s_acc[c]) continue;
            for (int d = tid; d < D; d += kSeqThreads) {
                sx[c * D + d] = sx[c * D + d] + sdl[c * D + d];
                sg[c * D + d] = sgt[c * D + d];
            }
            for (int r = tid; r < rpw; r += kSeqThreads) sa[c * rpw + r] = sat[c * rpw + r];
        }
        __syncthreads();
        for (int c = 0; c < nc; c++) {
            const int64_t t = s_t0[c] + k;
            if (t < s_t1[c])
                for (int d = d0 + tid; d < d1; d += kSeqThreads) out[(size_t)t * D + d] = sx[c * D + d];
        }
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
        // own coordinates are handled by one wave: at most 64 per workgroup
        if (Np % r == 0 && nb % 4 == 0 && nb <= 256 && (t.dim + nb - 1) / nb <= 64 && lds <= kSeqLdsLimit) {
            p.rpw = r;
            p.nb = nb;
            p.lds = lds;
            break;
        }
    }
    return p;
}

size_t seq_words(const SeqPlan &p, int D)
{
    return 2 * (size_t)p.nb * kSeqChains * ((size_t)D + 1) + 2 * (size_t)kSeqChains * D +
           2 * (size_t)p.nb * kSeqChains * kSeqQ;
}

}  // namespace

size_t seq_scratch_bytes(const DevTarget &t, int n_chains)
{
    (void)n_chains;
    if (t.kind != PMC_TARGET_LOGREG || t.dim < kWideMinDim) return 0;
    const SeqPlan p = seq_plan(t);
    if (!p.nb) return 0;
    return 256 + sizeof(uint64_t) * seq_words(p, t.dim);
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
    uint32_t *abort_ = (uint32_t *)a.scratch;
    uint64_t *words = (uint64_t *)((char *)a.scratch + 256);
    const size_t nw = seq_words(p, t.dim);
    uint64_t *p1 = words, *p2 = p1 + 2 * (size_t)p.nb * kSeqChains * ((size_t)t.dim + 1);
    uint64_t *p3 = p2 + 2 * (size_t)kSeqChains * t.dim;
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
        q.dpw = (t.dim + p.nb - 1) / p.nb;
        q.c0 = c0;
        q.nc = std::min(kSeqChains, a.n_chains - c0);
        q.steps = 0;
        for (int c = c0; c < c0 + q.nc; c++)
            q.steps = std::max<int64_t>(q.steps, a.host_offsets[c + 1] - a.host_offsets[c]);
        q.p1 = p1;
        q.p2 = p2;
        q.p3 = p3;
        q.abort_ = abort_;
        if (q.steps == 0) continue;
        // tags restart at 1 in every launch: clear the words of the previous one
        PMC_TRY_HIP(hipMemsetAsync(words, 0, sizeof(uint64_t) * nw, ctx->stream));
        void *args[] = {&q};
        PMC_TRY_HIP(hipLaunchCooperativeKernel((const void *)k_seq_logreg_wide, dim3(p.nb), dim3(kSeqThreads), args,
                                               (unsigned)p.lds, ctx->stream));
    }
    uint32_t h_abort = 0;
    PMC_TRY_HIP(hipMemcpyAsync(&h_abort, abort_, sizeof(uint32_t), hipMemcpyDeviceToHost, ctx->stream));
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (h_abort) {
        set_error("sequential logistic sampler: a wait for another workgroup's words timed out");
        return PMC_ERR_HIP;
    }
    return PMC_OK;
}

}  // namespace pmc
