// Dense DEER scan on gfx950 matrix cores: delta_t = J_t delta_{t-1} + b_t with
// J_t a full D x D matrix (D <= 32, padded to 32), the linearised recursion of
// Sec. 2 eq. 3.
//
// Hierarchical reduce-then-scan, one wavefront per unit, every chain of a
// batch with a hierarchy of its own (chains laid end to end; a chain's
// level-0 units are its scan tiles of at most 32 steps):
//   up:   each level-0 unit composes its steps' affine maps into one (P, B):
//         P = J_last ... J_first by matrix-core products with the running
//         product in the B-operand role (J_t streams in as the A operand
//         straight from memory; the accumulator returns to the B layout by a
//         swap of half its registers between lanes l and l + 32), B = the
//         unit applied to a zero carry, by FP32 matrix-vector products;
//         levels above compose groups of 8 maps the same way, until a chain
//         has at most 8 maps left (its top level);
//   down: from a zero carry at each chain's top, each group applies its maps
//         in order to produce the carries of the level below; at level 0 the
//         apply is the Newton update S_t <- F_t + J_t delta_{t-1} in FP32 with
//         fused convergence partials.
// One launch per level and direction covers every chain that has the level.
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
#include <string.h>

#include <algorithm>
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

// ----------------------------------------------------------- level-0 units
// A level-0 unit is one scan tile (at most 32 steps of one chain).  In the
// Newton update the tile map and the chains' windows give its steps; the
// standalone recursion cuts its one sequence every 32 steps.
struct Unit {
    int64_t t0;  // first step
    int cnt;     // steps
    int e0, e1;  // steps [e0, e1) of the unit lie in the chain's window
    int chain;
};

struct Lvl0In {  // Newton level 0: b_t = F_t - S_t from planes (FP32)
    const float *F, *S;
    int64_t ld;
    int D;
    const SegTile *tiles;
    const ChainStatus *chains;
    int64_t single_len;  // > 0: one chain of this many steps, cut every 32 (no tile load)
    // false if the unit's chain has stopped (nothing to do)
    __device__ bool unit(int64_t u, Unit &g) const
    {
        if (single_len > 0) {
            g.t0 = u * kU;
            g.cnt = (int)min((int64_t)kU, single_len - g.t0);
            g.chain = 0;
        } else {
            const SegTile st = tiles[u];
            g.t0 = st.start;
            g.cnt = st.len;
            g.chain = st.chain;
        }
        const ChainStatus &cs = chains[g.chain];
        if (!cs.active) return false;
        // steps before the window are the identity map with b = 0 (the carry
        // entering the window is exactly zero whatever their stale J holds);
        // steps from the window's end on are the identity too
        const int64_t ws = cs.win_start, we = cs.win_end;
        g.e0 = ws > g.t0 ? (int)min((int64_t)g.cnt, ws - g.t0) : 0;
        g.e1 = we < g.t0 + g.cnt ? (int)max((int64_t)0, we - g.t0) : g.cnt;
        return true;
    }
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
    int64_t n;
    __device__ bool unit(int64_t u, Unit &g) const
    {
        g.t0 = u * kU;
        g.cnt = (int)min((int64_t)kU, n - g.t0);
        g.e0 = 0;
        g.e1 = g.cnt;
        g.chain = 0;
        return true;
    }
    __device__ float b(int64_t t, int i) const { return i < D ? B[(size_t)t * D + i] : 0.f; }
};

// ---------------------------------------------------------- level-0 up pass
// Each unit composes its steps into one map (P, B): P = J_last ... J_first by
// matrix-core products, B = the unit applied to a zero carry.
template <class Frag, class Chain, class In>
__global__ void __launch_bounds__(64 * kWPB)
k_up0(const void *Jv, In in, int64_t n_units, float4 *Pout, float *Bout, const GlobalStatus *glob)
{
    if (glob && glob->n_active == 0) return;  // Newton: every chain has stopped
    __shared__ float s_t[kWPB][32 * 33];
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u >= n_units) return;
    Unit g;
    if (!in.unit(u, g)) return;
    Chain P;
    P.identity(i, h);
    f32x16 c;
#pragma unroll
    for (int r = 0; r < 16; r++) c[r] = crow(r, h) == i ? 1.f : 0.f;
    float *v = s_v[w];
    if (h == 0) v[i] = 0.f;
    wave_lds_sync();
    bool first = true;
    // J of the next step is requested before this step's products
    auto load_j = [&](int e, Frag &A) {
        if constexpr (sizeof(Frag) == sizeof(FragB))
            A.load((const uint4 *)Jv, g.t0 + e, lane);
        else
            A.load((const float4 *)Jv, g.t0 + e, lane);
    };
    Frag An;
    if (g.e0 < g.e1) load_j(g.e0, An);
    for (int e = g.e0; e < g.e1; e++) {
        const Frag A = An;
        if (e + 1 < g.e1) load_j(e + 1, An);
        if (!first) P.from_acc(c, h);
        c = P.mul(A);
        first = false;
        const float y = matvec(A, v, h) + in.b(g.t0 + e, i);
        wave_lds_sync();
        if (h == 0) v[i] = y;
        wave_lds_sync();
    }
    store_acc_as_fragf(c, s_t[w], Pout + (size_t)u * 256, lane);
    if (h == 0) Bout[(size_t)u * 32 + i] = v[i];
}

// ------------------------------------------------------------ upper levels
// Level k >= 1 holds, per chain, one map per group of 8 maps of level k - 1
// (its last group may be shorter), up to the chain's top level of at most 8
// maps.  One launch per level and direction, over the units of every chain
// that has that level: up, a unit composes its group into the level's map;
// down, a unit applies the maps of its group in order from the carry entering
// the group (zero for a chain's top level) and writes the carry entering each
// map.  Level-0 maps and carries are indexed by scan tile; the maps of levels
// >= 1 of all chains share one array (DenseChainGeom::ubase).
struct LevelArgs {
    int k;                       // level
    const int32_t *units;        // [n_units][2] (chain, group), or nullptr: one chain, group = unit
    int64_t n_units;
    const DenseChainGeom *geom;  // [n_chains]
    const float4 *P0;            // level-0 maps [n_tiles][256] float4 (F32 fragment layout)
    const float *B0;             // [n_tiles][32]
    float *C0;                   // carries entering each level-0 map [n_tiles][32]
    float4 *UP;                  // upper-level maps [n_up][256] float4
    float *UB, *UC;              // [n_up][32]
    const ChainStatus *chains;   // nullptr: standalone (the chain is active)
    const GlobalStatus *glob;
};

// Map e of a group at level k of chain G: level 0 by tile, levels >= 1 from
// the shared array.
struct MapSrc {
    const float4 *P;
    const float *B;
    __device__ void load(int64_t x, int lane, FragF &A, float &b) const
    {
        A.load(P, x, lane);
        b = B[(size_t)x * 32 + (lane & 31)];
    }
};

__device__ __forceinline__ bool level_unit(const LevelArgs &a, int64_t u, int &c, int64_t &grp)
{
    if (a.units) {
        c = a.units[2 * u];
        grp = a.units[2 * u + 1];
    } else {
        c = 0;
        grp = u;
    }
    return !a.chains || a.chains[c].active;
}

__global__ void __launch_bounds__(64 * kWPB) k_up_level(LevelArgs a)
{
    if (a.glob && a.glob->n_active == 0) return;
    __shared__ float s_t[kWPB][32 * 33];
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u >= a.n_units) return;
    int c;
    int64_t p;
    if (!level_unit(a, u, c, p)) return;
    const DenseChainGeom &G = a.geom[c];
    const int k = a.k;
    const int cnt = (int)min((int64_t)8, G.m[k - 1] - 8 * p);
    const int64_t x0 = (k == 1 ? G.tile0 : G.ubase[k - 1]) + 8 * p;
    const MapSrc src{k == 1 ? a.P0 : (const float4 *)a.UP, k == 1 ? a.B0 : (const float *)a.UB};
    float *v = s_v[w];
    ChainF P;
    P.identity(i, h);
    f32x16 acc;
    if (h == 0) v[i] = 0.f;
    wave_lds_sync();
    // the next map is requested before this one's products
    FragF An;
    float bn;
    src.load(x0, lane, An, bn);
    for (int e = 0; e < cnt; e++) {
        const FragF A = An;
        const float b = bn;
        if (e + 1 < cnt) src.load(x0 + e + 1, lane, An, bn);
        if (e > 0) P.from_acc(acc, h);
        acc = P.mul(A);
        const float y = matvec(A, v, h) + b;
        wave_lds_sync();
        if (h == 0) v[i] = y;
        wave_lds_sync();
    }
    const int64_t xo = G.ubase[k] + p;
    store_acc_as_fragf(acc, s_t[w], a.UP + (size_t)xo * 256, lane);
    if (h == 0) a.UB[(size_t)xo * 32 + i] = v[i];
}

__global__ void __launch_bounds__(64 * kWPB) k_down_level(LevelArgs a)
{
    if (a.glob && a.glob->n_active == 0) return;
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u >= a.n_units) return;
    int c;
    int64_t q;
    if (!level_unit(a, u, c, q)) return;
    const DenseChainGeom &G = a.geom[c];
    const int k = a.k;
    const bool top = k == G.L - 1;  // the top level starts from a zero carry
    const int64_t first = top ? 0 : 8 * q;
    const int cnt = top ? (int)G.m[k] : (int)min((int64_t)8, G.m[k] - first);
    const int64_t x0 = (k == 0 ? G.tile0 : G.ubase[k]) + first;
    const MapSrc src{k == 0 ? a.P0 : (const float4 *)a.UP, k == 0 ? a.B0 : (const float *)a.UB};
    float *out = k == 0 ? a.C0 : a.UC;
    float *v = s_v[w];
    if (h == 0) v[i] = top ? 0.f : a.UC[(size_t)(G.ubase[k + 1] + q) * 32 + i];
    wave_lds_sync();
    FragF An;
    float bn;
    src.load(x0, lane, An, bn);
    for (int e = 0; e < cnt; e++) {
        const FragF A = An;
        const float b = bn;
        if (e + 1 < cnt) src.load(x0 + e + 1, lane, An, bn);
        if (h == 0) out[(size_t)(x0 + e) * 32 + i] = v[i];
        const float y = matvec(A, v, h) + b;
        wave_lds_sync();
        if (h == 0) v[i] = y;
        wave_lds_sync();
    }
}

__global__ void k_store_geom(DenseChainGeom g, DenseChainGeom *out) { *out = g; }

// ------------------------------------------------------------- down pass
struct PartW {
    float ratio;
    uint32_t nonfinite;
    int64_t first_bad;
    double rsq, rinf;
};

// Level 0, Newton: S_t <- F_t + J_t delta_{t-1}, delta_t = J_t delta_{t-1} + b_t
// from the unit's carry, with the tile's convergence partials.
template <class Frag>
__global__ void __launch_bounds__(64 * kWPB)
k_down0_newton(const void *Jv, Lvl0In in, int64_t n_units, const float *carry, TilePartial *partials,
               double atol, double rtol, float *trace, const GlobalStatus *glob)
{
    // Once the status fold has stopped every chain, the sweeps still queued
    // behind it must leave S alone: F and J are no longer refreshed, and
    // re-applying S <- F + J delta with them need not stay bounded.
    if (glob && glob->n_active == 0) return;
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u >= n_units) return;
    PartW p{0.f, 0u, INT64_MAX, 0.0, 0.0};
    Unit g;
    if (in.unit(u, g)) {
        float *v = s_v[w];
        // steps before the chain's window are frozen: S keeps its values,
        // delta stays zero and they add nothing to the convergence partials
        if (h == 0) v[i] = g.e0 == 0 ? carry[(size_t)u * 32 + i] : 0.f;
        wave_lds_sync();
        const bool own = h == 0 && i < in.D;
        auto load_j = [&](int64_t t, Frag &A) {
            if constexpr (sizeof(Frag) == sizeof(FragB))
                A.load((const uint4 *)Jv, t, lane);
            else
                A.load((const float4 *)Jv, t, lane);
        };
        Frag An;
        if (g.e0 < g.e1) load_j(g.t0 + g.e0, An);
        for (int e = g.e0; e < g.e1; e++) {
            const int64_t t = g.t0 + e;
            const Frag A = An;
            if (e + 1 < g.e1) load_j(t + 1, An);
            const float jv = matvec(A, v, h);
            float y = 0.f;
            if (own) {
                const size_t k = (size_t)i * in.ld + t;
                const float f = in.F[k], so = in.S[k];
                const float b = f - so;
                y = jv + b;
                const float sn = f + jv;
                ((float *)in.S)[k] = sn;
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
k_down0_plain(const void *Jv, const float *Bv, float *out, int D, int64_t n, const float *carry)
{
    __shared__ float s_v[kWPB][32];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, i = lane & 31, h = lane >> 5;
    const int64_t u = (int64_t)blockIdx.x * kWPB + w;
    if (u * kU >= n) return;
    const int64_t t0 = u * kU;
    const int cnt = (int)min((int64_t)kU, n - t0);
    float *v = s_v[w];
    if (h == 0) v[i] = carry[(size_t)u * 32 + i];
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

inline unsigned blocks_for_units(int64_t n_units) { return (unsigned)((n_units + kWPB - 1) / kWPB); }

// Levels of one chain of m0 tile maps; returns the number of upper-level
// maps it adds (their first index is ubase0).
int64_t chain_geom(int64_t m0, int64_t tile0, int64_t ubase0, DenseChainGeom &g)
{
    memset(&g, 0, sizeof(g));
    g.tile0 = tile0;
    if (m0 <= 0) return 0;
    g.m[0] = m0;
    g.L = 1;
    while (g.m[g.L - 1] > 8) {
        g.m[g.L] = (g.m[g.L - 1] + 7) / 8;
        g.L++;
    }
    int64_t add = 0;
    for (int k = 1; k < g.L; k++) {
        g.ubase[k] = ubase0 + add;
        add += g.m[k];
    }
    return add;
}

void hier_layout(DenseHier &h)
{
    size_t off = 0;
    auto take = [&](size_t b) {
        const size_t o = off;
        off = align_up(off + std::max<size_t>(b, 1), 256);
        return o;
    };
    h.o_P0 = take((size_t)h.n_tiles * 4096);
    h.o_B0 = take((size_t)h.n_tiles * 128);
    h.o_C0 = take((size_t)h.n_tiles * 128);
    h.o_UP = take((size_t)h.n_up * 4096);
    h.o_UB = take((size_t)h.n_up * 128);
    h.o_UC = take((size_t)h.n_up * 128);
    h.o_geom = take(sizeof(DenseChainGeom) * std::max(h.n_chains, 1));
    h.o_units = take(sizeof(int32_t) * h.units.size());
    h.bytes = off;
}

LevelArgs level_args(const DenseHier &h, char *ws, int k, bool up, const ChainStatus *chains,
                     const GlobalStatus *glob)
{
    LevelArgs a;
    memset(&a, 0, sizeof(a));
    a.k = k;
    if (h.n_chains > 1) {
        const int64_t off = up ? h.up_off[k] : h.down_off[k];
        a.units = (const int32_t *)(ws + h.o_units) + 2 * off;
        a.n_units = up ? h.up_cnt[k] : h.down_cnt[k];
    } else {
        const DenseChainGeom &g = h.geom[0];
        a.units = nullptr;
        a.n_units = up ? g.m[k] : (k == g.L - 1 ? 1 : g.m[k + 1]);
    }
    a.geom = (const DenseChainGeom *)(ws + h.o_geom);
    a.P0 = (const float4 *)(ws + h.o_P0);
    a.B0 = (const float *)(ws + h.o_B0);
    a.C0 = (float *)(ws + h.o_C0);
    a.UP = (float4 *)(ws + h.o_UP);
    a.UB = (float *)(ws + h.o_UB);
    a.UC = (float *)(ws + h.o_UC);
    a.chains = chains;
    a.glob = glob;
    return a;
}

// The levels >= 1 (up, then down to the carries of the level-0 maps).
pmc_status run_levels(pmc_context *ctx, const DenseHier &h, char *ws, const ChainStatus *chains,
                      const GlobalStatus *glob)
{
    for (int k = 1; k < h.L_max; k++) {
        const LevelArgs a = level_args(h, ws, k, true, chains, glob);
        if (a.n_units > 0)
            hipLaunchKernelGGL(k_up_level, dim3(blocks_for_units(a.n_units)), dim3(64 * kWPB), 0, ctx->stream, a);
    }
    for (int k = h.L_max - 1; k >= 0; k--) {
        const LevelArgs a = level_args(h, ws, k, false, chains, glob);
        if (a.n_units > 0)
            hipLaunchKernelGGL(k_down_level, dim3(blocks_for_units(a.n_units)), dim3(64 * kWPB), 0, ctx->stream, a);
    }
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

}  // namespace

void dense_hier_plan(const std::vector<int32_t> &ctb, int n_chains, int64_t n_steps, DenseHier &h)
{
    h = DenseHier();
    h.n_chains = n_chains;
    h.single_len = n_chains == 1 ? n_steps : 0;
    h.n_tiles = n_chains > 0 ? ctb[n_chains] : 0;
    h.geom.resize(std::max(n_chains, 1));
    int64_t ub = 0;
    for (int c = 0; c < n_chains; c++) {
        ub += chain_geom(ctb[c + 1] - ctb[c], ctb[c], ub, h.geom[c]);
        h.L_max = std::max(h.L_max, h.geom[c].L);
    }
    h.n_up = ub;
    if (n_chains > 1) {
        // units per level: up level k composes groups of level k - 1 into
        // the chain's level-k maps; down level k applies groups of level k
        // (a chain's top level is one group)
        for (int k = 0; k < h.L_max; k++) {
            h.up_off[k] = (int64_t)h.units.size() / 2;
            for (int c = 0; c < n_chains && k >= 1; c++)
                for (int64_t p = 0; k < h.geom[c].L && p < h.geom[c].m[k]; p++) h.units.insert(h.units.end(), {c, (int32_t)p});
            h.up_cnt[k] = (int64_t)h.units.size() / 2 - h.up_off[k];
        }
        for (int k = 0; k < h.L_max; k++) {
            h.down_off[k] = (int64_t)h.units.size() / 2;
            for (int c = 0; c < n_chains; c++) {
                const DenseChainGeom &g = h.geom[c];
                if (k == g.L - 1)
                    h.units.insert(h.units.end(), {c, 0});
                else if (k < g.L - 1)
                    for (int64_t q = 0; q < g.m[k + 1]; q++) h.units.insert(h.units.end(), {c, (int32_t)q});
            }
            h.down_cnt[k] = (int64_t)h.units.size() / 2 - h.down_off[k];
        }
    }
    hier_layout(h);
}

pmc_status dense_hier_setup(pmc_context *ctx, const DenseHier &h, void *ws)
{
    char *p = (char *)ws;
    if (h.n_chains <= 1) {
        // one chain: its geometry travels as a kernel argument (the host
        // copy may be gone before an asynchronous copy would run)
        hipLaunchKernelGGL(k_store_geom, dim3(1), dim3(1), 0, ctx->stream, h.geom[0], (DenseChainGeom *)(p + h.o_geom));
        PMC_TRY_HIP(hipGetLastError());
    } else {
        PMC_TRY_HIP(hipMemcpyAsync(p + h.o_geom, h.geom.data(), sizeof(DenseChainGeom) * h.n_chains,
                                   hipMemcpyHostToDevice, ctx->stream));
        PMC_TRY_HIP(hipMemcpyAsync(p + h.o_units, h.units.data(), sizeof(int32_t) * h.units.size(),
                                   hipMemcpyHostToDevice, ctx->stream));
    }
    return PMC_OK;
}

// Workspace of the hierarchy of one sequence of n steps.
size_t dense_mfma_ws_bytes(int64_t n)
{
    DenseHier h;
    dense_hier_plan({0, (int32_t)((n + kU - 1) / kU)}, 1, n, h);
    return h.bytes;
}

int dense_mfma_unit() { return kU; }

pmc_status launch_dense_mfma_newton(pmc_context *ctx, int bf16, const void *J, const float *F,
                                    float *S, int64_t ld, int D, const SegTile *tiles,
                                    const ChainStatus *chains, TilePartial *partials, double atol,
                                    double rtol, float *trace, void *ws, const DenseHier &h,
                                    const GlobalStatus *glob)
{
    if (h.n_tiles == 0) return PMC_OK;
    char *p = (char *)ws;
    Lvl0In in{F, S, ld, D, tiles, chains, h.single_len};
    if (bf16)
        hipLaunchKernelGGL((k_up0<FragB, ChainB, Lvl0In>), dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0,
                           ctx->stream, J, in, h.n_tiles, (float4 *)(p + h.o_P0), (float *)(p + h.o_B0), glob);
    else
        hipLaunchKernelGGL((k_up0<FragF, ChainF, Lvl0In>), dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0,
                           ctx->stream, J, in, h.n_tiles, (float4 *)(p + h.o_P0), (float *)(p + h.o_B0), glob);
    PMC_TRY(run_levels(ctx, h, p, chains, glob));
    if (bf16)
        hipLaunchKernelGGL(k_down0_newton<FragB>, dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0,
                           ctx->stream, J, in, h.n_tiles, (const float *)(p + h.o_C0), partials, atol, rtol, trace,
                           glob);
    else
        hipLaunchKernelGGL(k_down0_newton<FragF>, dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0,
                           ctx->stream, J, in, h.n_tiles, (const float *)(p + h.o_C0), partials, atol, rtol, trace,
                           glob);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status launch_linrec_dense_mfma_packed(pmc_context *ctx, int bf16, int D, int64_t T,
                                           const void *Jf, const float *b, float *out, void *ws)
{
    if (T == 0) return PMC_OK;
    DenseHier h;
    dense_hier_plan({0, (int32_t)((T + kU - 1) / kU)}, 1, T, h);
    PMC_TRY(dense_hier_setup(ctx, h, ws));
    char *p = (char *)ws;
    RowIn in{b, D, T};
    if (bf16)
        hipLaunchKernelGGL((k_up0<FragB, ChainB, RowIn>), dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0,
                           ctx->stream, Jf, in, h.n_tiles, (float4 *)(p + h.o_P0), (float *)(p + h.o_B0), nullptr);
    else
        hipLaunchKernelGGL((k_up0<FragF, ChainF, RowIn>), dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0,
                           ctx->stream, Jf, in, h.n_tiles, (float4 *)(p + h.o_P0), (float *)(p + h.o_B0), nullptr);
    PMC_TRY(run_levels(ctx, h, p, nullptr, nullptr));
    if (bf16)
        hipLaunchKernelGGL(k_down0_plain<FragB>, dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0, ctx->stream,
                           Jf, b, out, D, T, (const float *)(p + h.o_C0));
    else
        hipLaunchKernelGGL(k_down0_plain<FragF>, dim3(blocks_for_units(h.n_tiles)), dim3(64 * kWPB), 0, ctx->stream,
                           Jf, b, out, D, T, (const float *)(p + h.o_C0));
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
    if (T > 0) {
        hipLaunchKernelGGL(k_pack, dim3((unsigned)T), dim3(64), 0, ctx->stream, A, D, T, Jf, bf16);
        PMC_TRY_HIP(hipGetLastError());
    }
    return launch_linrec_dense_mfma_packed(ctx, bf16, D, T, Jf, b, out, ws + align_up(jb, 256));
}

}  // namespace pmc
