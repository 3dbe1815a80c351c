// Dense DEER scan on gfx950 matrix cores: delta_t = J_t delta_{t-1} + b_t with
// J_t a full D x D matrix (D <= 32, padded to 32), the linearised recursion of
// Sec. 2 eq. 3.
//
// Hierarchical reduce-then-scan over units of 32 elements, one wavefront per
// unit:
//   up:   each unit composes its 32 affine maps into one (P, B):
//         P = J_32 ... J_1 by matrix-core products with the running product in
//         the B-operand role (J_t streams in as the A operand straight from
//         memory; the accumulator returns to the B layout by a swap of half
//         its registers between lanes l and l + 32), B = the unit applied to a
//         zero carry, by FP32 matrix-vector products;
//         levels repeat on the (P, B) arrays until at most 32 maps remain;
//   down: from a zero carry at the top, each unit applies its maps in order to
//         produce the carries of the level below; at level 0 the apply is the
//         Newton update S_t <- F_t + J_t delta_{t-1} in FP32 with fused
//         convergence partials.
// Level-0 J is BF16 (v_mfma_f32_32x32x16_bf16, FP32 accumulation; the exact
// FP32 residual makes the Newton iteration a refinement, so BF16 products cost
// sweeps, not accuracy) or FP32 (v_mfma_f32_32x32x2_f32).  Levels >= 1 are FP32.
//
// Register layouts (lane l, i = l % 32, h = l / 32):
//   BF16 A operand of J (32 x 32): lane holds J[i][16 kk + 8 h + j], kk = 0, 1,
//     j = 0..7, stored as [t][kk][lane][8] bf16 (2 KiB per step);
//   F32 A operand: lane holds M[i][2 m + h], m = 0..15, stored as
//     [t][m / 4][lane][m % 4] (4 KiB per step);
//   accumulator (C/D) of a 32 x 32 product: register r holds
//     C[8 (r / 4) + 4 h + r % 4][i].
#include <math.h>

#include <vector>

#include "pmc_internal.hpp"

namespace pmc {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int kU = 32;  // elements per level-0 unit
constexpr int kU1 = 8;  // maps per unit at levels >= 1 (more, shorter chains)
constexpr int kWPB = 4; // waves (units) per block

__device__ __forceinline__ int crow(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// ---------------------------------------------------------------- A operands
struct FragB {  // BF16 J_t
    uint4 q[2];
    __device__ void load(const uint4 *J, int64_t t, int lane)
    {
        q[0] = J[(size_t)t * 128 + lane];
        q[1] = J[(size_t)t * 128 + 64 + lane];
    }
    __device__ void zero() { q[0] = q[1] = make_uint4(0, 0, 0, 0); }
    __device__ float at(int kk, int j) const  // J[i][16 kk + 8 h + j]
    {
        const uint4 v = q[kk];
        const uint32_t w = j < 2 ? v.x : j < 4 ? v.y : j < 6 ? v.z : v.w;
        return bf2f((uint16_t)((j & 1) ? (w >> 16) : (w & 0xffffu)));
    }
    // y_i partial: sum over this lane's 16 columns of J[i][k] v[k]
    __device__ float dot(const float *v, int h) const
    {
        float s = 0.f;
#pragma unroll
        for (int kk = 0; kk < 2; kk++)
#pragma unroll
            for (int j = 0; j < 8; j++) s = fmaf(at(kk, j), v[16 * kk + 8 * h + j], s);
        return s;
    }
};

struct FragF {  // F32 M
    float4 q[4];
    __device__ void load(const float4 *M, int64_t t, int lane)
    {
#pragma unroll
        for (int m4 = 0; m4 < 4; m4++) q[m4] = M[((size_t)t * 4 + m4) * 64 + lane];
    }
    __device__ void zero()
    {
#pragma unroll
        for (int m4 = 0; m4 < 4; m4++) q[m4] = make_float4(0.f, 0.f, 0.f, 0.f);
    }
    __device__ float at(int m) const
    {
        const float4 v = q[m >> 2];
        const int j = m & 3;
        return j == 0 ? v.x : j == 1 ? v.y : j == 2 ? v.z : v.w;
    }
    __device__ float dot(const float *v, int h) const
    {
        float s = 0.f;
#pragma unroll
        for (int m = 0; m < 16; m++) s = fmaf(at(m), v[2 * m + h], s);
        return s;
    }
};

// ------------------------------------------------ running product P <- A P
// P kept in the B-operand layout.  BF16 B operand: lane holds
// P[16 kk + 8 h + j][i]; F32 B operand: lane holds P[2 m + h][i].
struct ChainB {
    bf16x8 b[2];
    __device__ void identity(int i, int h)
    {
#pragma unroll
        for (int kk = 0; kk < 2; kk++)
#pragma unroll
            for (int j = 0; j < 8; j++) b[kk][j] = (__bf16)((16 * kk + 8 * h + j) == i ? 1.f : 0.f);
    }
    __device__ f32x16 mul(const FragB &A) const
    {
        bf16x8 a0, a1;
        __builtin_memcpy(&a0, &A.q[0], 16);
        __builtin_memcpy(&a1, &A.q[1], 16);
        f32x16 c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a0, b[0], c, 0, 0, 0);
        c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1, b[1], c, 0, 0, 0);
        return c;
    }
    // accumulator -> B layout: lane h = 0 needs rows 0-7 and 16-23, lane h = 1
    // rows 8-15 and 24-31.  The gfx950 lane-half swap (upper 32 lanes of its
    // first operand <-> lower 32 lanes of its second) applied to the register
    // pairs (c[q], c[4+q]) and (c[8+q], c[12+q]) leaves exactly those rows in
    // b[0][q], b[0][4+q], b[1][q], b[1][4+q] on both halves.
    __device__ void from_acc(const f32x16 &c, int)
    {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const auto p0 = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[q]), __float_as_uint(c[4 + q]),
                                                             false, false);
            const auto p1 = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[8 + q]),
                                                             __float_as_uint(c[12 + q]), false, false);
            b[0][q] = (__bf16)__uint_as_float(p0[0]);
            b[0][4 + q] = (__bf16)__uint_as_float(p0[1]);
            b[1][q] = (__bf16)__uint_as_float(p1[0]);
            b[1][4 + q] = (__bf16)__uint_as_float(p1[1]);
        }
    }
};

struct ChainF {
    float b[16];
    __device__ void identity(int i, int h)
    {
#pragma unroll
        for (int m = 0; m < 16; m++) b[m] = (2 * m + h) == i ? 1.f : 0.f;
    }
    __device__ f32x16 mul(const FragF &A) const
    {
        f32x16 c = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int m = 0; m < 16; m++) c = __builtin_amdgcn_mfma_f32_32x32x2f32(A.at(m), b[m], c, 0, 0, 0);
        return c;
    }
    // lane h needs rows of parity h (B row 2 m + h).  Register 4g + w holds row
    // 8g + 4h + w; the lane-half swap of the pairs (c[4g], c[4g+1]) and
    // (c[4g+2], c[4g+3]) gives (b[4g], b[4g+2]) and (b[4g+1], b[4g+3]).
    __device__ void from_acc(const f32x16 &c, int)
    {
#pragma unroll
        for (int g = 0; g < 4; g++) {
            const auto p = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[4 * g]), __float_as_uint(c[4 * g + 1]),
                                                            false, false);
            const auto q = __builtin_amdgcn_permlane32_swap(__float_as_uint(c[4 * g + 2]),
                                                            __float_as_uint(c[4 * g + 3]), false, false);
            b[4 * g] = __uint_as_float(p[0]);
            b[4 * g + 2] = __uint_as_float(p[1]);
            b[4 * g + 1] = __uint_as_float(q[0]);
            b[4 * g + 3] = __uint_as_float(q[1]);
        }
    }
};

// Store an accumulator (32 x 32) as an F32 A operand [m4][lane][4] via LDS.
__device__ void store_acc_as_fragf(const f32x16 &c, float *lds /*32*33*/, float4 *out, int lane)
{
    const int i = lane & 31, h = lane >> 5;
#pragma unroll
    for (int r = 0; r < 16; r++) lds[crow(r, h) * 33 + i] = c[r];
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int m4 = 0; m4 < 4; m4++) {
        float v[4];
#pragma unroll
        for (int j = 0; j < 4; j++) v[j] = lds[i * 33 + 2 * (4 * m4 + j) + h];
        out[m4 * 64 + lane] = make_float4(v[0], v[1], v[2], v[3]);
    }
}

// matrix-vector through LDS: vin (32 floats in LDS) -> returns y_i = (A v)_i in
// both lanes i and i + 32
template <class Frag>
__device__ __forceinline__ float matvec(const Frag &A, const float *vin, int h)
{
    float s = A.dot(vin, h);
    return s + __shfl_xor(s, 32, 64);
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ----------------------------------------------------------- level inputs
struct Lvl0In {  // Newton level 0: b_t = F_t - S_t from planes (FP32)
    const float *F, *S;
    int64_t ld;
    int D;
    const ChainStatus *chain;  // window start of the (single) chain, or nullptr
    __device__ int64_t first() const { return chain ? chain->win_start : 0; }
    __device__ int64_t last() const { return chain ? chain->win_end : INT64_MAX; }
    __device__ float b(int64_t t, int i) const
    {
        if (i >= D) return 0.f;
        const size_t k = (size_t)i * ld + t;
        return F[k] - S[k];
    }
};
struct RowIn {  // standalone level 0: b_t rows [T, D]
    const float *B;
    int D;
    __device__ int64_t first() const { return 0; }
    __device__ int64_t last() const { return INT64_MAX; }
    __device__ float b(int64_t t, int i) const { return i < D ? B[(size_t)t * D + i] : 0.f; }
};
struct MapIn {  // levels >= 1: B vectors [n, 32]
    const float *B;
    __device__ int64_t first() const { return 0; }
    __device__ int64_t last() const { return INT64_MAX; }
    __device__ float b(int64_t t, int i) const { return B[(size_t)t * 32 + i]; }
};

// ---------------------------------------------------------------- up pass
template <class Frag, class Chain, class In>
__global__ void __launch_bounds__(64 * kWPB)
k_up(const void *Jv, In in, int64_t n, int unit, float4 *Pout, float *Bout, const GlobalStatus *glob)
{
    if (glob && glob->n_active == 0) return;  // Newton: the chain has stopped
    __shared__ float s_t[kWPB][32 * 33];
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u * unit >= n) return;
    const int64_t t0 = u * unit;
    const int cnt = (int)min((int64_t)unit, n - t0);
    Chain P;
    P.identity(i, h);
    // steps before the sliding window are the identity map with b = 0: the
    // carry entering the window is exactly zero whatever their stale J holds
    f32x16 c;
#pragma unroll
    for (int r = 0; r < 16; r++) c[r] = crow(r, h) == i ? 1.f : 0.f;
    float *v = s_v[w];
    if (h == 0) v[i] = 0.f;
    wave_lds_sync();
    bool first = true;
    const int64_t ws = in.first(), we = in.last();
    const int e0 = ws > t0 ? (int)min((int64_t)cnt, ws - t0) : 0;
    const int e1 = we < t0 + cnt ? (int)max((int64_t)0, we - t0) : cnt;  // steps from the window's end on: identity
    for (int e = e0; e < e1; e++) {
        Frag A;
        if constexpr (sizeof(Frag) == sizeof(FragB))
            A.load((const uint4 *)Jv, t0 + e, lane);
        else
            A.load((const float4 *)Jv, t0 + e, lane);
        if (!first) P.from_acc(c, h);
        c = P.mul(A);
        first = false;
        const float y = matvec(A, v, h) + in.b(t0 + e, i);
        wave_lds_sync();
        if (h == 0) v[i] = y;
        wave_lds_sync();
    }
    store_acc_as_fragf(c, s_t[w], Pout + (size_t)u * 256, lane);
    if (h == 0) Bout[(size_t)u * 32 + i] = v[i];
}

// ------------------------------------------------------------- down pass
// Level >= 1: carries of the children.  carry_in == nullptr means zero.
__global__ void __launch_bounds__(64 * kWPB)
k_down_maps(const float4 *P, const float *B, int64_t n, int unit, const float *carry_in, float *carry_out,
            const GlobalStatus *glob)
{
    if (glob && glob->n_active == 0) return;
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u * unit >= n) return;
    const int64_t t0 = u * unit;
    const int cnt = (int)min((int64_t)unit, n - t0);
    float *v = s_v[w];
    if (h == 0) v[i] = carry_in ? carry_in[(size_t)u * 32 + i] : 0.f;
    wave_lds_sync();
    for (int e = 0; e < cnt; e++) {
        FragF A;
        A.load(P, t0 + e, lane);
        if (h == 0) carry_out[(size_t)(t0 + e) * 32 + i] = v[i];
        const float y = matvec(A, v, h) + B[(size_t)(t0 + e) * 32 + i];
        wave_lds_sync();
        if (h == 0) v[i] = y;
        wave_lds_sync();
    }
}

struct PartW {
    float ratio;
    uint32_t nonfinite;
    int64_t first_bad;
    double rsq, rinf;
};

// Level 0, Newton: S_t <- F_t + J_t delta_{t-1}, delta_t = J_t delta_{t-1} + b_t.
template <class Frag>
__global__ void __launch_bounds__(64 * kWPB)
k_down0_newton(const void *Jv, const float *F, float *S, int64_t ld, int D, int64_t n,
               const float *carry_in, TilePartial *partials, double atol, double rtol, float *trace,
               const GlobalStatus *glob, const ChainStatus *chain)
{
    // Once the status fold has stopped the chain, the sweeps still queued
    // behind it must leave S alone: F and J are no longer refreshed, and
    // re-applying S <- F + J delta with them need not stay bounded.
    if (glob && glob->n_active == 0) return;
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u * kU >= n) return;
    const int64_t t0 = u * kU;
    const int cnt = (int)min((int64_t)kU, n - t0);
    float *v = s_v[w];
    // steps before the chain's sliding window are frozen: S keeps its values,
    // delta stays zero and they add nothing to the convergence partials
    const int64_t ws = chain ? chain->win_start : 0, we = chain ? chain->win_end : INT64_MAX;
    const int e0 = ws > t0 ? (int)min((int64_t)cnt, ws - t0) : 0;
    const int e1 = we < t0 + cnt ? (int)max((int64_t)0, we - t0) : cnt;  // steps past the window: untouched
    if (h == 0) v[i] = (carry_in && e0 == 0) ? carry_in[(size_t)u * 32 + i] : 0.f;
    wave_lds_sync();
    PartW p{0.f, 0u, INT64_MAX, 0.0, 0.0};
    const bool own = h == 0 && i < D;
    for (int e = e0; e < e1; e++) {
        const int64_t t = t0 + e;
        Frag A;
        if constexpr (sizeof(Frag) == sizeof(FragB))
            A.load((const uint4 *)Jv, t, lane);
        else
            A.load((const float4 *)Jv, t, lane);
        const float jv = matvec(A, v, h);
        float y = 0.f;
        if (own) {
            const size_t k = (size_t)i * ld + t;
            const float f = F[k], so = S[k];
            const float b = f - so;
            y = jv + b;
            const float sn = f + jv;
            S[k] = sn;
            if (trace) trace[k] = sn;
            float r = (float)(fabs((double)y) / (atol + rtol * fabs((double)sn)));
            if (!(r == r)) r = INFINITY;
            if (!isfinite(sn)) p.nonfinite++;
            if (r > kFreezeRatio && t < p.first_bad) p.first_bad = t;
            p.ratio = fmaxf(p.ratio, r);
            p.rsq += (double)b * b;
            double ab = fabs((double)b);
            p.rinf = (ab == ab) ? fmax(p.rinf, ab) : INFINITY;
        }
        wave_lds_sync();
        if (h == 0) v[i] = y;
        wave_lds_sync();
    }
#pragma unroll
    for (int m = 1; m < 64; m <<= 1) {
        p.ratio = fmaxf(p.ratio, __shfl_xor(p.ratio, m, 64));
        p.nonfinite += __shfl_xor(p.nonfinite, m, 64);
        p.first_bad = min(p.first_bad, (int64_t)__shfl_xor((long long)p.first_bad, m, 64));
        p.rsq += __shfl_xor(p.rsq, m, 64);
        p.rinf = fmax(p.rinf, __shfl_xor(p.rinf, m, 64));
    }
    if (lane == 0) {
        TilePartial &tp = partials[u];
        tp.max_ratio = p.ratio;
        tp.nonfinite = p.nonfinite;
        tp.first_bad = p.first_bad;
        tp.resid_sq = p.rsq;
        tp.resid_inf = p.rinf;
    }
}

// Level 0, standalone recursion: out_t = delta_t, rows [T, D].
template <class Frag>
__global__ void __launch_bounds__(64 * kWPB)
k_down0_plain(const void *Jv, const float *Bv, float *out, int D, int64_t n, const float *carry_in)
{
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u * kU >= n) return;
    const int64_t t0 = u * kU;
    const int cnt = (int)min((int64_t)kU, n - t0);
    float *v = s_v[w];
    if (h == 0) v[i] = carry_in ? carry_in[(size_t)u * 32 + i] : 0.f;
    wave_lds_sync();
    for (int e = 0; e < cnt; e++) {
        const int64_t t = t0 + e;
        Frag A;
        if constexpr (sizeof(Frag) == sizeof(FragB))
            A.load((const uint4 *)Jv, t, lane);
        else
            A.load((const float4 *)Jv, t, lane);
        float y = matvec(A, v, h);
        if (h == 0 && i < D) {
            y += Bv[(size_t)t * D + i];
            out[(size_t)t * D + i] = y;
        }
        wave_lds_sync();
        if (h == 0) v[i] = i < D ? y : 0.f;
        wave_lds_sync();
    }
}

// Row-major [T, D, D] FP32 -> fragment layout (BF16 or F32), zero padded.
__global__ void k_pack(const float *A, int D, int64_t T, void *out, int bf16)
{
    const int64_t t = blockIdx.x;
    if (t >= T) return;
    const int lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const float *At = A + (size_t)t * D * D;
    auto get = [&](int r, int k) -> float { return (r < D && k < D) ? At[r * D + k] : 0.f; };
    if (bf16) {
        uint4 *o = (uint4 *)out;
        for (int kk = 0; kk < 2; kk++) {
            uint32_t p[4];
            for (int q = 0; q < 4; q++) {
                const int k0 = 16 * kk + 8 * h + 2 * q;
                p[q] = (uint32_t)f2bf(get(i, k0)) | ((uint32_t)f2bf(get(i, k0 + 1)) << 16);
            }
            o[(size_t)t * 128 + kk * 64 + lane] = make_uint4(p[0], p[1], p[2], p[3]);
        }
    } else {
        float4 *o = (float4 *)out;
        for (int m4 = 0; m4 < 4; m4++) {
            float v[4];
            for (int j = 0; j < 4; j++) v[j] = get(i, 2 * (4 * m4 + j) + h);
            o[((size_t)t * 4 + m4) * 64 + lane] = make_float4(v[0], v[1], v[2], v[3]);
        }
    }
}

inline unsigned blocks_for(int64_t n, int unit = kU) { return (unsigned)(((n + unit - 1) / unit + kWPB - 1) / kWPB); }

}  // namespace

// Workspace of the hierarchy for n level-0 elements.
size_t dense_mfma_ws_bytes(int64_t n)
{
    size_t b = 0;
    int64_t m = n;
    int unit = kU;
    while (m > unit) {
        const int64_t u = (m + unit - 1) / unit;
        b += align_up((size_t)u * 1024 * 4, 256) + 2 * align_up((size_t)u * 32 * 4, 256);
        m = u;
        unit = kU1;
    }
    return b + 256;
}

// Shared driver: runs the up levels, the top and the down levels >= 1, and
// returns the carries for the level-0 units (nullptr if T <= 32).
template <class Frag, class Chain, class In>
static pmc_status dense_hierarchy(pmc_context *ctx, const void *J, const In &in0, int64_t n, char *ws,
                                  const float **carry0, const GlobalStatus *glob = nullptr)
{
    struct Lv {
        int64_t n;      // elements of this level (maps of the level below)
        float4 *P;      // [n] maps (level >= 1)
        float *B;       // [n][32]
        float *carry;   // [n][32] carries entering each element
    };
    std::vector<Lv> lv;
    int64_t m = n;
    char *p = ws;
    int unit = kU;  // level 0 groups 32 steps, the levels above kU1 maps
    while (m > unit) {
        const int64_t u = (m + unit - 1) / unit;
        unit = kU1;
        Lv L;
        L.n = u;
        L.P = (float4 *)p;
        p += align_up((size_t)u * 1024 * 4, 256);
        L.B = (float *)p;
        p += align_up((size_t)u * 32 * 4, 256);
        L.carry = (float *)p;
        p += align_up((size_t)u * 32 * 4, 256);
        lv.push_back(L);
        m = u;
    }
    if (lv.empty()) {
        *carry0 = nullptr;
        return PMC_OK;
    }
    // up
    hipLaunchKernelGGL((k_up<Frag, Chain, In>), dim3(blocks_for(n)), dim3(64 * kWPB), 0, ctx->stream, J,
                       in0, n, kU, lv[0].P, lv[0].B, glob);
    for (size_t k = 1; k < lv.size(); k++)
        hipLaunchKernelGGL((k_up<FragF, ChainF, MapIn>), dim3(blocks_for(lv[k - 1].n, kU1)), dim3(64 * kWPB),
                           0, ctx->stream, (const void *)lv[k - 1].P, MapIn{lv[k - 1].B}, lv[k - 1].n, kU1,
                           lv[k].P, lv[k].B, glob);
    // top: the last level's maps (<= kU1) from a zero carry
    const Lv &top = lv.back();
    hipLaunchKernelGGL(k_down_maps, dim3(1), dim3(64 * kWPB), 0, ctx->stream, (const float4 *)top.P,
                       (const float *)top.B, top.n, kU1, (const float *)nullptr, top.carry, glob);
    for (int k = (int)lv.size() - 2; k >= 0; k--)
        hipLaunchKernelGGL(k_down_maps, dim3(blocks_for(lv[k].n, kU1)), dim3(64 * kWPB), 0, ctx->stream,
                           (const float4 *)lv[k].P, (const float *)lv[k].B, lv[k].n, kU1,
                           (const float *)lv[k + 1].carry, lv[k].carry, glob);
    PMC_TRY_HIP(hipGetLastError());
    *carry0 = lv[0].carry;
    return PMC_OK;
}

pmc_status launch_dense_mfma_newton(pmc_context *ctx, int bf16, const void *J, const float *F,
                                    float *S, int64_t ld, int D, int64_t n, TilePartial *partials,
                                    double atol, double rtol, float *trace, void *ws, const GlobalStatus *glob,
                                    const ChainStatus *chain)
{
    const float *c0 = nullptr;
    Lvl0In in{F, S, ld, D, chain};
    if (bf16) {
        PMC_TRY((dense_hierarchy<FragB, ChainB, Lvl0In>(ctx, J, in, n, (char *)ws, &c0, glob)));
        hipLaunchKernelGGL(k_down0_newton<FragB>, dim3(blocks_for(n)), dim3(64 * kWPB), 0, ctx->stream,
                           J, F, S, ld, D, n, c0, partials, atol, rtol, trace, glob, chain);
    } else {
        PMC_TRY((dense_hierarchy<FragF, ChainF, Lvl0In>(ctx, J, in, n, (char *)ws, &c0, glob)));
        hipLaunchKernelGGL(k_down0_newton<FragF>, dim3(blocks_for(n)), dim3(64 * kWPB), 0, ctx->stream,
                           J, F, S, ld, D, n, c0, partials, atol, rtol, trace, glob, chain);
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

int dense_mfma_unit() { return kU; }

pmc_status launch_linrec_dense_mfma_packed(pmc_context *ctx, int bf16, int D, int64_t T,
                                           const void *Jf, const float *b, float *out, void *ws)
{
    const float *c0 = nullptr;
    RowIn in{b, D};
    if (bf16) {
        PMC_TRY((dense_hierarchy<FragB, ChainB, RowIn>(ctx, Jf, in, T, (char *)ws, &c0)));
        hipLaunchKernelGGL(k_down0_plain<FragB>, dim3(blocks_for(T)), dim3(64 * kWPB), 0, ctx->stream,
                           Jf, b, out, D, T, c0);
    } else {
        PMC_TRY((dense_hierarchy<FragF, ChainF, RowIn>(ctx, Jf, in, T, (char *)ws, &c0)));
        hipLaunchKernelGGL(k_down0_plain<FragF>, dim3(blocks_for(T)), dim3(64 * kWPB), 0, ctx->stream,
                           Jf, b, out, D, T, c0);
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status launch_linrec_dense_mfma(pmc_context *ctx, int bf16, int D, int64_t T, const float *A,
                                    const float *b, float *out)
{
    const size_t jb = (size_t)T * (bf16 ? 2048 : 4096);
    const size_t need = align_up(jb, 256) + dense_mfma_ws_bytes(T);
    PMC_TRY(ensure_pool(ctx, need));
    char *ws = (char *)ctx->pool;
    void *Jf = ws;
    hipLaunchKernelGGL(k_pack, dim3((unsigned)T), dim3(64), 0, ctx->stream, A, D, T, Jf, bf16);
    PMC_TRY_HIP(hipGetLastError());
    const float *c0 = nullptr;
    RowIn in{b, D};
    char *hw = ws + align_up(jb, 256);
    if (bf16) {
        PMC_TRY((dense_hierarchy<FragB, ChainB, RowIn>(ctx, Jf, in, T, hw, &c0)));
        hipLaunchKernelGGL(k_down0_plain<FragB>, dim3(blocks_for(T)), dim3(64 * kWPB), 0, ctx->stream,
                           (const void *)Jf, b, out, D, T, c0);
    } else {
        PMC_TRY((dense_hierarchy<FragF, ChainF, RowIn>(ctx, Jf, in, T, hw, &c0)));
        hipLaunchKernelGGL(k_down0_plain<FragF>, dim3(blocks_for(T)), dim3(64 * kWPB), 0, ctx->stream,
                           (const void *)Jf, b, out, D, T, c0);
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

}  // namespace pmc
