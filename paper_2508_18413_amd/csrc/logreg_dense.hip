// Full-DEER Jacobians of the MALA/ULA transition on the Bayesian
// logistic-regression posterior (Sec. 2 with the model of App. B.1):
//   J_t = I + a_t eps Hess log p(s_{t-1}),
//   Hess log p(x) = -X^T diag(w) X - I / prior_var,
//   w_n = sigma(m_n) (1 - sigma(m_n)),  m = X x,
// a_t the frozen accept decision of the current evaluation (1 under ULA).
// The evaluation kernel supplies f_t and a_t; the two kernels here supply J_t.
//
// k_logreg_dense_h: for 32 steps per wavefront, the data term as two chained
// BF16 matrix-core products with FP32 accumulation (v_mfma_f32_32x32x16_bf16):
//   M^T = X S^T     data points x steps, K = D (padded to 32),
//   Hp  = W P       steps x pairs,      K = data points,
// with P[n][p] = x_nd x_ne over the D (D + 1) / 2 pairs d <= e (row-major
// upper triangle), so the symmetric D x D sum is formed once per pair.  The
// accumulator of the first product holds, in lane (i, h), step i and the 16
// data points 32 nb + 8 (r / 4) + 4 h + r % 4, r = 0..15; once w is formed
// in place, registers 8 q .. 8 q + 7 are the A operand of the second
// product's K block q of that data tile, provided P's K slots follow the same
// order (the table pb is written that way), so nothing moves between lanes.
// The Jacobian only steers the Newton iteration (the residual f_t is exact
// FP32), so BF16 operands cost sweeps, not accuracy.
//
// k_logreg_dense_j: one wavefront per step forms J_t from the pair sums,
// applies the damping and the entrywise or infinity-norm clip exactly as the
// per-lane evaluation does, and writes the matrix-core A-operand image the
// dense scan reads (BF16, 2 KiB per step, or FP32, 4 KiB per step).
//
// k_logreg_probe_diag: quasi-DEER with the one-probe diagonal z o (J z) of
// Sec. 3.4 eq. 10.  For 32 steps per wavefront, M^T = X S^T and V^T = X Z^T
// (Z the probe signs), U = w o V in the accumulator, then X^T U, whose
// B operand is again the accumulator (the table xt orders X^T's K slots the
// same way), gives (X^T W X z)_d; the diagonal planes receive
// damping (1 + a_t eps z_d (H z)_d) with H z = -X^T W X z - z / prior_var.
//
// Register layouts (lane l, i = l % 32, h = l / 32), as in the dense scan:
//   A operand (32 x 16): A[i][8 h + j], j = 0..7;
//   B operand (16 x 32): B[8 h + j][i];
//   accumulator register r: C[8 (r / 4) + 4 h + r % 4][i].
#include <math.h>

#include "pmc_internal.hpp"

namespace pmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kDenseWaves = 4;  // 32-step tiles per workgroup
constexpr int kMaxPairCols = 32 * 33 / 2;  // D (D + 1) / 2 at D = 32
// pair tiles accumulated per pass over the data: each pass recomputes M^T
// and w, but 3 tiles (about 125 registers) leave room for 4 wavefronts per
// SIMD to hide the operand loads, which is faster than 4 tiles (3 per SIMD),
// 6 (2) or all 11 of D = 25 in one pass (1)
constexpr int kMaxGroup = 3;

__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

typedef float f32x8 __attribute__((ext_vector_type(8)));

// eight FP32 values to BF16, round to nearest even (v_cvt_pk_bf16_f32)
__device__ __forceinline__ bf16x8 pack8(const float *v)
{
    const f32x8 x = {v[0], v[1], v[2], v[3], v[4], v[5], v[6], v[7]};
    return __builtin_convertvector(x, bf16x8);
}

// pair index of (d, e), d <= e, in the row-major upper triangle of a D x D matrix
__host__ __device__ __forceinline__ int pair_index(int d, int e, int D) { return d * D - d * (d - 1) / 2 + (e - d); }

// Operand tables, one thread per 8-value fragment:
//   xa[nb][kd][l] = X[32 nb + i][16 kd + 8 h + j]                   (A of M^T)
//   pb[nb][q][pt][l] slot j = P[32 nb + 16 q + 8 (j / 4) + 4 h + j % 4][32 pt + i]
//   xt[nb][q][l]  slot j = X[32 nb + 16 q + 8 (j / 4) + 4 h + j % 4][i]  (A of X^T U)
// zero outside the data, the coordinates and the pairs.
__global__ void k_logreg_dense_tables(const float *X, int ldx, int N, int D, int nb_count, int npt,
                                      uint4 *xa, uint4 *pb, uint4 *xt)
{
    const int64_t n_xa = (int64_t)nb_count * 2 * 64, n_pb = (int64_t)nb_count * 2 * npt * 64;
    const int np = D * (D + 1) / 2;
    for (int64_t id = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; id < 2 * n_xa + n_pb;
         id += (int64_t)gridDim.x * blockDim.x) {
        float v[8];
        if (id >= n_xa + n_pb) {
            const int64_t k = id - n_xa - n_pb;
            const int l = (int)(k % 64), q = (int)((k / 64) % 2), nb = (int)(k / 128);
            const int d = l & 31, h = l >> 5;
            for (int j = 0; j < 8; j++) {
                const int n = 32 * nb + 16 * q + 8 * (j >> 2) + 4 * h + (j & 3);
                v[j] = (n < N && d < D) ? X[(size_t)n * ldx + d] : 0.f;
            }
            xt[k] = __builtin_bit_cast(uint4, pack8(v));
        } else if (id < n_xa) {
            const int l = (int)(id % 64), kd = (int)((id / 64) % 2), nb = (int)(id / 128);
            const int n = 32 * nb + (l & 31), h = l >> 5;
            for (int j = 0; j < 8; j++) {
                const int d = 16 * kd + 8 * h + j;
                v[j] = (n < N && d < D) ? X[(size_t)n * ldx + d] : 0.f;
            }
            xa[id] = __builtin_bit_cast(uint4, pack8(v));
        } else {
            const int64_t k = id - n_xa;
            const int l = (int)(k % 64), pt = (int)((k / 64) % npt);
            const int q = (int)((k / (64 * npt)) % 2), nb = (int)(k / (128 * npt));
            const int p = 32 * pt + (l & 31), h = l >> 5;
            int d = 0, e = 0;
            if (p < np) {
                while (pair_index(d, D - 1, D) < p) d++;
                e = d + (p - pair_index(d, d, D));
            }
            for (int j = 0; j < 8; j++) {
                const int n = 32 * nb + 16 * q + 8 * (j >> 2) + 4 * h + (j & 3);
                v[j] = (n < N && p < np) ? X[(size_t)n * ldx + d] * X[(size_t)n * ldx + e] : 0.f;
            }
            pb[k] = __builtin_bit_cast(uint4, pack8(v));
        }
    }
}

struct DenseHArgs {
    const uint4 *xa, *pb;
    int nb_count, npt;  // data tiles, pair tiles (a multiple of the group)
    const float *S;     // [D, ld]
    const float *s0;    // [n_chains, D]
    const int64_t *offsets;  // [n_chains + 1] first step of each chain
    int n_chains;
    int64_t ld, n;
    int D;
    float *H;           // [n, 32 npt] pair sums
    const GlobalStatus *glob;  // n_active == 0 at launch: nothing to do
};

// chain of global step t (offsets ascending, offsets[0] = 0 <= t < offsets[n_chains])
__device__ __forceinline__ int chain_of(const int64_t *offsets, int n_chains, int64_t t)
{
    int lo = 0, hi = n_chains - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (offsets[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// grid.x: 32-step tiles / kDenseWaves, grid.y: groups of G pair tiles
template <int G>
__global__ void __launch_bounds__(64 * kDenseWaves) k_logreg_dense_h(DenseHArgs a)
{
    const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t t0 = ((int64_t)blockIdx.x * kDenseWaves + (threadIdx.x >> 6)) * 32;
    if (t0 >= a.n) return;  // uniform per wavefront
    if (a.glob && a.glob->n_active == 0) return;
    const int pt0 = blockIdx.y * G;
    const int64_t t = t0 + i;
    // the state entering step t: s0 of its chain at the chain's first step
    int c = 0;
    bool head = t == 0;
    if (a.n_chains > 1 && t < a.n) {
        c = chain_of(a.offsets, a.n_chains, t);
        head = t == a.offsets[c];
    }

    // B operand of M^T = X S^T: lane (i, h) holds s_{t-1}[16 kd + 8 h + j]
    bf16x8 sb[2];
#pragma unroll
    for (int kd = 0; kd < 2; kd++) {
        float v[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int d = 16 * kd + 8 * h + j;
            float x = 0.f;
            if (t < a.n && d < a.D) x = head ? a.s0[(size_t)c * a.D + d] : a.S[(size_t)d * a.ld + t - 1];
            v[j] = x;
        }
        sb[kd] = pack8(v);
    }

    f32x16 acc[G];
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int r = 0; r < 16; r++) acc[g][r] = 0.f;

    // the next data tile's fragments are requested before this one is
    // multiplied (the last tile reloads itself, so every load is
    // unconditional); the compiler may still move them, and the occupancy
    // above is what hides their latency
    const size_t pstep = 2 * (size_t)a.npt * 64;
    const uint4 *xa = a.xa + lane;
    const uint4 *pb = a.pb + (size_t)pt0 * 64 + lane;
    uint4 nx[2], np[2 * G];
    nx[0] = xa[0];
    nx[1] = xa[64];
#pragma unroll
    for (int g = 0; g < G; g++) {
        np[g] = pb[g * 64];
        np[G + g] = pb[(a.npt + g) * 64];
    }
    for (int nb = 0; nb < a.nb_count; nb++) {
        uint4 cx[2] = {nx[0], nx[1]}, cp[2 * G];
#pragma unroll
        for (int k = 0; k < 2 * G; k++) cp[k] = np[k];
        const int nn = nb + 1 < a.nb_count ? nb + 1 : nb;
        nx[0] = xa[(size_t)nn * 128];
        nx[1] = xa[(size_t)nn * 128 + 64];
#pragma unroll
        for (int g = 0; g < G; g++) {
            np[g] = pb[nn * pstep + g * 64];
            np[G + g] = pb[nn * pstep + (a.npt + g) * 64];
        }
        f32x16 m;
#pragma unroll
        for (int r = 0; r < 16; r++) m[r] = 0.f;
        m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, cx[0]), sb[0], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, cx[1]), sb[1], m, 0, 0, 0);
        // w = sigma (1 - sigma) = e / (1 + e)^2 with e = exp(-|m|); the
        // hardware reciprocal is ample for a Jacobian rounded to BF16
        float w[16];
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float e = __expf(-fabsf(m[r]));
            const float s = 1.f + e;
            w[r] = e * __builtin_amdgcn_rcpf(s * s);
        }
        const bf16x8 w0 = pack8(w), w1 = pack8(w + 8);
#pragma unroll
        for (int g = 0; g < G; g++) {
            acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w0, __builtin_bit_cast(bf16x8, cp[g]), acc[g], 0, 0, 0);
            acc[g] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w1, __builtin_bit_cast(bf16x8, cp[G + g]), acc[g], 0, 0,
                                                            0);
        }
    }

    const int64_t hld = 32 * (int64_t)a.npt;
#pragma unroll
    for (int g = 0; g < G; g++)
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const int64_t tr = t0 + crow(r, h);
            if (tr < a.n) a.H[tr * hld + 32 * (pt0 + g) + i] = acc[g][r];
        }
}

struct DenseJArgs {
    const float *H;  // [n, hld]
    int64_t hld, n;
    const uint8_t *accept;
    float eps, pp;   // step size, 1 / prior_var
    int D;
    float damping, clip;
    int clip_inf, f32;
    void *J;
    const GlobalStatus *glob;
};

// one wavefront per step; lane (i, h) forms row i over the 16 columns the
// A-operand image gives it
__global__ void __launch_bounds__(256) k_logreg_dense_j(DenseJArgs a)
{
    const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= a.n) return;  // uniform per wavefront
    if (a.glob && a.glob->n_active == 0) return;
    const float ea = a.accept[t] ? a.eps : 0.f;
    // the step's pair sums, read coalesced into LDS, then gathered per entry
    __shared__ float s_h[4][kMaxPairCols];
    float *sh = s_h[threadIdx.x >> 6];
    const float *Ht = a.H + t * a.hld;
    const int np = a.D * (a.D + 1) / 2;
    for (int p = lane; p < np; p += 64) sh[p] = Ht[p];
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    float v[16];
    float rs = 0.f;
#pragma unroll
    for (int c = 0; c < 16; c++) {
        // BF16 image: column 16 (c / 8) + 8 h + c % 8; FP32 image: column 2 c + h
        const int k = a.f32 ? 2 * c + h : 16 * (c >> 3) + 8 * h + (c & 7);
        float x = 0.f;
        if (i < a.D && k < a.D) {
            const float hs = sh[i <= k ? pair_index(i, k, a.D) : pair_index(k, i, a.D)];
            x = i == k ? fmaf(-ea, hs + a.pp, 1.f) : -ea * hs;
        }
        v[c] = x;
        rs += fabsf(x);
    }
    float scale = a.damping;
    if (a.clip > 0.f && a.clip_inf) {
        float nrm = rs + __shfl_xor(rs, 32);
#pragma unroll
        for (int m = 16; m >= 1; m >>= 1) nrm = fmaxf(nrm, __shfl_xor(nrm, m));
        nrm *= scale;
        if (nrm > a.clip) scale *= a.clip / nrm;
    }
    const bool eclip = a.clip > 0.f && !a.clip_inf;
#pragma unroll
    for (int c = 0; c < 16; c++) {
        float x = v[c] * scale;
        if (eclip) x = fminf(fmaxf(x, -a.clip), a.clip);
        v[c] = x;
    }
    if (a.f32) {
        // [t][m / 4][lane][m % 4]
        float4 *J = (float4 *)((float *)a.J + (size_t)t * 1024);
#pragma unroll
        for (int m4 = 0; m4 < 4; m4++) J[m4 * 64 + lane] = make_float4(v[4 * m4], v[4 * m4 + 1], v[4 * m4 + 2], v[4 * m4 + 3]);
    } else {
        // [t][kk][lane][8]
        uint4 *J = (uint4 *)((uint16_t *)a.J + (size_t)t * 1024);
#pragma unroll
        for (int kk = 0; kk < 2; kk++) J[kk * 64 + lane] = __builtin_bit_cast(uint4, pack8(v + 8 * kk));
    }
}

struct ProbeArgs {
    const uint4 *xa, *xt;
    int nb_count;
    const float *S, *s0;  // [D, ld], [n_chains, D]
    int64_t ld, n;
    int D;
    const uint8_t *accept;
    float eps, pp, damping, clip;
    const int64_t *offsets;     // [n_chains + 1] first step of each chain
    int n_chains;
    const ChainStatus *chains;  // a chain's sweep counter selects its probe
    uint64_t seed;
    float *J;                   // [D, ld]
    const GlobalStatus *glob;
};


__device__ __forceinline__ float probe_sign(uint64_t hs, int64_t t, int d)
{
    return (probe_mix(hs ^ (uint64_t)(1024 * t + d)) >> 63) ? -1.f : 1.f;
}

__global__ void __launch_bounds__(64 * kDenseWaves) k_logreg_probe_diag(ProbeArgs a)
{
    const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t t0 = ((int64_t)blockIdx.x * kDenseWaves + (threadIdx.x >> 6)) * 32;
    if (t0 >= a.n) return;  // uniform per wavefront
    if (a.glob && a.glob->n_active == 0) return;
    const int64_t t = t0 + i;
    const bool live = t < a.n;
    // this step's chain: its first step takes s0 of the chain, its sweep
    // counter picks the probe
    const int c = live ? chain_of(a.offsets, a.n_chains, t) : 0;
    const bool head = live && t == a.offsets[c];
    const uint64_t hs = probe_mix(probe_mix(a.seed) ^ (uint64_t)(uint32_t)a.chains[c].sweeps);

    // B operands: s_{t-1} and the probe z_t, coordinates 16 kd + 8 h + j
    bf16x8 sb[2], zb[2];
#pragma unroll
    for (int kd = 0; kd < 2; kd++) {
        float v[8], z[8];
#pragma unroll
        for (int j = 0; j < 8; j++) {
            const int d = 16 * kd + 8 * h + j;
            const bool in = live && d < a.D;
            v[j] = in ? (head ? a.s0[(size_t)c * a.D + d] : a.S[(size_t)d * a.ld + t - 1]) : 0.f;
            z[j] = in ? probe_sign(hs, t, d) : 0.f;
        }
        sb[kd] = pack8(v);
        zb[kd] = pack8(z);
    }
    f32x16 P;
#pragma unroll
    for (int r = 0; r < 16; r++) P[r] = 0.f;
    for (int nb = 0; nb < a.nb_count; nb++) {
        const bf16x8 x0 = __builtin_bit_cast(bf16x8, a.xa[(size_t)nb * 128 + lane]);
        const bf16x8 x1 = __builtin_bit_cast(bf16x8, a.xa[(size_t)nb * 128 + 64 + lane]);
        f32x16 m, v;
#pragma unroll
        for (int r = 0; r < 16; r++) m[r] = v[r] = 0.f;
        m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, sb[0], m, 0, 0, 0);
        m = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, sb[1], m, 0, 0, 0);
        v = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x0, zb[0], v, 0, 0, 0);
        v = __builtin_amdgcn_mfma_f32_32x32x16_bf16(x1, zb[1], v, 0, 0, 0);
        float u[16];
#pragma unroll
        for (int r = 0; r < 16; r++) {
            const float e = __expf(-fabsf(m[r]));
            const float s = 1.f + e;
            u[r] = e * __builtin_amdgcn_rcpf(s * s) * v[r];
        }
        P = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a.xt[(size_t)nb * 128 + lane]),
                                                    pack8(u), P, 0, 0, 0);
        P = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a.xt[(size_t)nb * 128 + 64 + lane]),
                                                    pack8(u + 8), P, 0, 0, 0);
    }
    // register r: (X^T W X z)_d for d = 8 (r / 4) + 4 h + r % 4 at step t
    if (!live) return;
    const float ea = a.accept[t] ? a.eps : 0.f;
#pragma unroll
    for (int r = 0; r < 16; r++) {
        const int d = crow(r, h);
        if (d < a.D) {
            const float z = probe_sign(hs, t, d);
            const float hz = -P[r] - a.pp * z;
            float jv = a.damping * fmaf(ea, z * hz, 1.f);
            if (a.clip > 0.f) jv = fminf(fmaxf(jv, -a.clip), a.clip);
            a.J[(size_t)d * a.ld + t] = jv;
        }
    }
}

// pair tiles accumulated per pass: the fewest passes of at most kMaxGroup
// tiles, split evenly
int pair_group(int D)
{
    const int npt0 = (D * (D + 1) / 2 + 31) / 32, passes = (npt0 + kMaxGroup - 1) / kMaxGroup;
    return (npt0 + passes - 1) / passes;
}

}  // namespace

int logreg_dense_pair_cols(int D)
{
    // pair tiles padded with zero columns to a whole number of groups
    const int npt0 = (D * (D + 1) / 2 + 31) / 32, g = pair_group(D);
    return 32 * ((npt0 + g - 1) / g * g);
}

pmc_status logreg_dense_tables(pmc_context *ctx, DevTarget &t)
{
    if (t.dxa) return PMC_OK;
    if (t.dim > 32) {
        set_error("matrix-core Jacobians of logistic regression support D <= 32 (got %d)", t.dim);
        return PMC_ERR_UNSUPPORTED;
    }
    const int grp = pair_group(t.dim), nbc = (t.n_data + 31) / 32, npt = logreg_dense_pair_cols(t.dim) / 32;
    const size_t bxa = (size_t)nbc * 2 * 64 * 16, bpb = (size_t)nbc * 2 * npt * 64 * 16;
    void *xa = nullptr, *pb = nullptr, *xt = nullptr;
    PMC_TRY_HIP(hipMalloc(&xa, bxa));
    if (hipMalloc(&pb, bpb) != hipSuccess || hipMalloc(&xt, bxa) != hipSuccess) {
        (void)hipFree(xa);
        if (pb) (void)hipFree(pb);
        set_error("dense DEER tables: out of device memory (%zu bytes)", 2 * bxa + bpb);
        return PMC_ERR_OOM;
    }
    const int64_t work = (int64_t)(2 * bxa + bpb) / 16;
    const int blocks = (int)std::min<int64_t>((work + 255) / 256, 4096);
    hipLaunchKernelGGL(k_logreg_dense_tables, dim3(blocks), dim3(256), 0, ctx->stream, (const float *)t.X, t.ldx,
                       t.n_data, t.dim, nbc, npt, (uint4 *)xa, (uint4 *)pb, (uint4 *)xt);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) {
        (void)hipFree(xa);
        (void)hipFree(pb);
        (void)hipFree(xt);
        set_error("dense DEER tables: %s", hipGetErrorString(e));
        return PMC_ERR_HIP;
    }
    t.dxa = xa;
    t.dpb = pb;
    t.dxt = xt;
    t.dnb = nbc;
    t.dnpt = npt;
    t.dgrp = grp;
    return PMC_OK;
}

pmc_status launch_logreg_dense_jac(pmc_context *ctx, const DevTarget &t, const EvalArgs &a, int64_t n,
                                   int n_chains, float *H, bool f32)
{
    if (n <= 0) return PMC_OK;
    PMC_REQUIRE(t.dxa && t.dpb, "logreg dense Jacobian: tables not built");
    DenseHArgs ha{(const uint4 *)t.dxa, (const uint4 *)t.dpb, t.dnb, t.dnpt, (const float *)a.S,
                  (const float *)a.s0, a.offsets, n_chains, a.ld, n, t.dim, H, a.glob};
    const int g = t.dgrp;
    const int64_t tiles = (n + 31) / 32, gx = (tiles + kDenseWaves - 1) / kDenseWaves;
    PMC_REQUIRE(gx <= 0x7fffffff && g >= 1 && g <= kMaxGroup && t.dnpt % g == 0,
                "logreg dense Jacobian: bad launch shape");
    const dim3 grid((unsigned)gx, (unsigned)(t.dnpt / g)), block(64 * kDenseWaves);
    switch (g) {
#define PMC_DENSE_H_CASE(G)                                                                        \
    case G: hipLaunchKernelGGL(k_logreg_dense_h<G>, grid, block, 0, ctx->stream, ha); break;
        PMC_DENSE_H_CASE(1)
        PMC_DENSE_H_CASE(2)
        PMC_DENSE_H_CASE(3)
#undef PMC_DENSE_H_CASE
    default: set_error("logreg dense Jacobian: group %d", g); return PMC_ERR_UNSUPPORTED;
    }
    PMC_TRY_HIP(hipGetLastError());
    DenseJArgs ja{H, 32 * (int64_t)t.dnpt, n, a.accept, (float)a.eps, (float)(1.0 / t.prior_var), t.dim,
                  (float)a.damping, (float)a.clip, a.clip_inf, f32 ? 1 : 0, a.J, a.glob};
    PMC_REQUIRE((n + 3) / 4 <= 0x7fffffff, "logreg dense Jacobian: too many steps");
    hipLaunchKernelGGL(k_logreg_dense_j, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, ctx->stream, ja);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status launch_logreg_probe_diag(pmc_context *ctx, const DevTarget &t, const EvalArgs &a, int64_t n,
                                    int n_chains)
{
    if (n <= 0) return PMC_OK;
    PMC_REQUIRE(t.dxa && t.dxt, "logreg probed diagonal: tables not built");
    const int64_t gx = ((n + 31) / 32 + kDenseWaves - 1) / kDenseWaves;
    PMC_REQUIRE(gx <= 0x7fffffff, "logreg probed diagonal: too many steps");
    PMC_REQUIRE(n_chains >= 1, "logreg probed diagonal: no chains");
    ProbeArgs pa{(const uint4 *)t.dxa, (const uint4 *)t.dxt, t.dnb, (const float *)a.S, (const float *)a.s0,
                 a.ld, n, t.dim, a.accept, (float)a.eps, (float)(1.0 / t.prior_var), (float)a.damping,
                 (float)a.clip, a.offsets, n_chains, a.chains, a.probe_seed, (float *)a.J, a.glob};
    hipLaunchKernelGGL(k_logreg_probe_diag, dim3((unsigned)gx), dim3(64 * kDenseWaves), 0, ctx->stream, pa);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

}  // namespace pmc
