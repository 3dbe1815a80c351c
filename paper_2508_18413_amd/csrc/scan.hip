// Single-pass scans of the linearised recursion of the Newton update
// (Sec. 2 eq. 2-4, Appendix A.3) for gfx950.
//
// The recursion delta_t = A_t delta_{t-1} + b_t is a composition of affine
// maps (A, b); compositions of affine maps are affine (Sec. 2), so a tile of C
// consecutive steps reduces to one map.  One kernel launch does the whole
// scan:
//   1. each thread composes ITEMS consecutive steps held in registers;
//   2. a wavefront inclusive scan of the thread aggregates (DPP lane moves);
//   3. wave aggregates combine through LDS into the tile aggregate;
//   4. decoupled look-back: the tile publishes its aggregate, then wave 0 reads
//      up to 64 predecessor descriptors at once and folds aggregates back to the
//      nearest published inclusive value;
//   5. every thread re-applies its steps from its exact carry and writes the
//      new iterate, fusing the convergence partials (Algorithm 1's Delta test,
//      residual norms in FP64, first unconverged step, non-finite count).
//
// Descriptor words are 64-bit (tag << 32 | 32-bit payload piece) written and
// read with agent-scope atomics, so every word validates itself and no memory
// fence is needed between payload and flag.  Tags carry a per-launch epoch
// that a one-thread kernel advances after each scan, or, inside a Newton
// solve, the status fold that follows the scan (descriptors never need
// clearing; captured graphs can replay the scan).  A tile's id is its
// workgroup index: workgroups are dispatched in index order on each XCD, so a
// tile's predecessors were scheduled before it, and no per-tile counter (a
// same-address atomic that serialises across XCDs) is needed.
#include <float.h>
#include <math.h>

#include "pmc_internal.hpp"
#include "wave.hpp"

namespace pmc {
namespace {

constexpr int kWave = 64;

// Workgroup barrier that orders LDS only: the tile's global loads and stores
// stay in flight across it (no thread reads another thread's global data).
__device__ __forceinline__ void lds_barrier()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// ------------------------------------------------------------- affine maps
template <typename R, int M>
struct Aff {
    R a[M][M];
    R b[M];
};

template <typename R, int M>
__device__ __forceinline__ Aff<R, M> aff_identity()
{
    Aff<R, M> e;
#pragma unroll
    for (int i = 0; i < M; i++) {
#pragma unroll
        for (int j = 0; j < M; j++) e.a[i][j] = (i == j) ? R(1) : R(0);
        e.b[i] = R(0);
    }
    return e;
}

// later o earlier: x -> L.a (E.a x + E.b) + L.b
template <typename R, int M>
__device__ __forceinline__ Aff<R, M> compose(const Aff<R, M> &L, const Aff<R, M> &E)
{
    Aff<R, M> c;
#pragma unroll
    for (int i = 0; i < M; i++) {
#pragma unroll
        for (int j = 0; j < M; j++) {
            R s = R(0);
#pragma unroll
            for (int k = 0; k < M; k++) s = fma(L.a[i][k], E.a[k][j], s);
            c.a[i][j] = s;
        }
        R s = L.b[i];
#pragma unroll
        for (int k = 0; k < M; k++) s = fma(L.a[i][k], E.b[k], s);
        c.b[i] = s;
    }
    return c;
}

template <typename R, int M>
__device__ __forceinline__ void apply(const Aff<R, M> &e, const R (&x)[M], R (&y)[M])
{
    R t[M];
#pragma unroll
    for (int i = 0; i < M; i++) {
        R s = e.b[i];
#pragma unroll
        for (int k = 0; k < M; k++) s = fma(e.a[i][k], x[k], s);
        t[i] = s;
    }
#pragma unroll
    for (int i = 0; i < M; i++) y[i] = t[i];
}

// Moves every register of a map with one DPP pattern (wave.hpp).
struct AffMover {
    template <int CTRL, int ROWS, typename R, int M>
    __device__ __forceinline__ Aff<R, M> move(const Aff<R, M> &old, const Aff<R, M> &v) const
    {
        Aff<R, M> o;
#pragma unroll
        for (int i = 0; i < M; i++) {
#pragma unroll
            for (int j = 0; j < M; j++) o.a[i][j] = wave::dpp<CTRL, ROWS>(old.a[i][j], v.a[i][j]);
            o.b[i] = wave::dpp<CTRL, ROWS>(old.b[i], v.b[i]);
        }
        return o;
    }
};

// Inclusive scan of the lanes' maps in lane order (lane 0 earliest): lane l
// ends with e_l o ... o e_0; `excl` gets e_{l-1} o ... o e_0 (identity in
// lane 0).  All 64 lanes must be active.
template <typename R, int M>
__device__ __forceinline__ Aff<R, M> wave_scan_aff(const Aff<R, M> &e, Aff<R, M> &excl)
{
    const Aff<R, M> id = aff_identity<R, M>();
    const Aff<R, M> inc = wave::scan_incl(e, id, AffMover{},
                                          [](const Aff<R, M> &L, const Aff<R, M> &E) { return compose(L, E); });
    excl = wave::shift_up1(inc, id, AffMover{});
    return inc;
}

// Map of lane l in every lane.
template <typename R, int M>
__device__ __forceinline__ Aff<R, M> aff_lane(const Aff<R, M> &e, int l)
{
    Aff<R, M> o;
#pragma unroll
    for (int i = 0; i < M; i++) {
#pragma unroll
        for (int j = 0; j < M; j++) o.a[i][j] = wave::lane_value(e.a[i][j], l);
        o.b[i] = wave::lane_value(e.b[i], l);
    }
    return o;
}

// ---------------------------------------------------- look-back descriptors
template <typename R>
struct Pieces;
template <>
struct Pieces<float> {
    static constexpr int n = 1;
    __device__ static void split(float v, uint32_t *p) { p[0] = __float_as_uint(v); }
    __device__ static float join(const uint32_t *p) { return __uint_as_float(p[0]); }
};
template <>
struct Pieces<double> {
    static constexpr int n = 2;
    __device__ static void split(double v, uint32_t *p)
    {
        uint64_t u = __double_as_longlong(v);
        p[0] = (uint32_t)u;
        p[1] = (uint32_t)(u >> 32);
    }
    __device__ static double join(const uint32_t *p)
    {
        return __longlong_as_double(((uint64_t)p[1] << 32) | p[0]);
    }
};

template <typename R, int M>
struct Desc {
    static constexpr int P = Pieces<R>::n;
    static constexpr int kInc = M * P;            // words of the inclusive value
    static constexpr int kAgg = (M * M + M) * P;  // words of the aggregate
    static constexpr int kWords = kInc + kAgg;
};

__device__ __forceinline__ void word_store(uint64_t *w, uint32_t tag, uint32_t v)
{
    __hip_atomic_store(w, ((uint64_t)tag << 32) | v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t word_load(const uint64_t *w)
{
    return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

constexpr uint32_t kAggState = 1, kIncState = 2;
__device__ __forceinline__ uint32_t make_tag(uint32_t epoch, uint32_t st) { return (epoch << 2) | st; }

template <typename R, int M>
__device__ void publish_agg(uint64_t *d, uint32_t epoch, const Aff<R, M> &e)
{
    using DS = Desc<R, M>;
    uint32_t tag = make_tag(epoch, kAggState);
    uint32_t p[Pieces<R>::n];
    int w = DS::kInc;
#pragma unroll
    for (int i = 0; i < M; i++) {
#pragma unroll
        for (int j = 0; j < M; j++) {
            Pieces<R>::split(e.a[i][j], p);
#pragma unroll
            for (int k = 0; k < Pieces<R>::n; k++) word_store(d + w++, tag, p[k]);
        }
        Pieces<R>::split(e.b[i], p);
#pragma unroll
        for (int k = 0; k < Pieces<R>::n; k++) word_store(d + w++, tag, p[k]);
    }
}

template <typename R, int M>
__device__ void publish_inc(uint64_t *d, uint32_t epoch, const R (&v)[M])
{
    uint32_t tag = make_tag(epoch, kIncState);
    uint32_t p[Pieces<R>::n];
    int w = 0;
#pragma unroll
    for (int i = 0; i < M; i++) {
        Pieces<R>::split(v[i], p);
#pragma unroll
        for (int k = 0; k < Pieces<R>::n; k++) word_store(d + w++, tag, p[k]);
    }
}

// Reads one descriptor (every word is loaded at once, so one round trip
// serves both forms).  Returns 2 with the inclusive value as a constant map
// (a = 0, b = value), 1 with the aggregate, or 0 if not yet published.
template <typename R, int M>
__device__ int read_desc(const uint64_t *d, uint32_t epoch, Aff<R, M> &out)
{
    using DS = Desc<R, M>;
    constexpr int P = Pieces<R>::n;
    const uint32_t ti = make_tag(epoch, kIncState), ta = make_tag(epoch, kAggState);
    uint64_t x[DS::kWords];
#pragma unroll
    for (int w = 0; w < DS::kWords; w++) x[w] = word_load(d + w);
    uint32_t p[P];
    bool inc = true, agg = true;
    int w = 0;
#pragma unroll
    for (int i = 0; i < M; i++) {
#pragma unroll
        for (int k = 0; k < P; k++, w++) {
            inc &= (uint32_t)(x[w] >> 32) == ti;
            p[k] = (uint32_t)x[w];
        }
        out.b[i] = Pieces<R>::join(p);
    }
    if (inc) {
#pragma unroll
        for (int i = 0; i < M; i++)
#pragma unroll
            for (int j = 0; j < M; j++) out.a[i][j] = R(0);
        return 2;
    }
#pragma unroll
    for (int i = 0; i < M; i++) {
#pragma unroll
        for (int j = 0; j < M; j++) {
#pragma unroll
            for (int k = 0; k < P; k++, w++) {
                agg &= (uint32_t)(x[w] >> 32) == ta;
                p[k] = (uint32_t)x[w];
            }
            out.a[i][j] = Pieces<R>::join(p);
        }
#pragma unroll
        for (int k = 0; k < P; k++, w++) {
            agg &= (uint32_t)(x[w] >> 32) == ta;
            p[k] = (uint32_t)x[w];
        }
        out.b[i] = Pieces<R>::join(p);
    }
    return agg ? 1 : 0;
}

// Wave-parallel look-back (wave 0 only).  `self` is this tile's descriptor id,
// `head` the id of the first tile of its sequence (which publishes an
// inclusive value without looking back).  Returns the carry entering the tile.
// A predecessor that never publishes is a bug; after kSpinLimit polls the
// look-back gives up, raises sync->pad and uses a zero carry, so the launch
// ends and the host reports the failure instead of hanging the device.
constexpr uint32_t kSpinLimit = 1u << 18;  // polls; with the naps, tens of ms to a fraction of a second

template <typename R, int M>
__device__ void lookback(uint64_t *desc, int64_t self, int64_t head, uint32_t epoch, R (&carry)[M],
                         ScanSync *sync)
{
    // Each round covers the 64 nearest unread predecessors.  While some are
    // unpublished, only those lanes poll again, after a sleep that doubles up
    // to about a memory round trip: polling every descriptor at full rate
    // floods the uncached path the tiles' own data also uses.
    using DS = Desc<R, M>;
    const int lid = threadIdx.x % kWave;
    Aff<R, M> acc = aff_identity<R, M>();
    int64_t p = self - 1;
    uint32_t spins = 0;
    for (;;) {
        const int64_t q = p - lid;
        Aff<R, M> m = aff_identity<R, M>();
        int st = q >= head ? 0 : 3;  // 0 unpublished, 1 aggregate, 2 inclusive, 3 beyond the head
        int nap = 1;
        for (;;) {
            if (st == 0) st = read_desc<R, M>(desc + (size_t)q * DS::kWords, epoch, m);
            const uint64_t incmask = __ballot(st == 2);
            const int first_inc = incmask ? __ffsll((unsigned long long)incmask) - 1 : kWave;
            const uint64_t waitmask = __ballot(st == 0 && lid <= first_inc);
            if (!waitmask) break;
            if (++spins >= kSpinLimit) {
                if (lid == 0) atomicOr(&sync->pad, 1u);
#pragma unroll
                for (int i = 0; i < M; i++) carry[i] = R(0);
                return;
            }
            for (int k = 0; k < nap; k++) __builtin_amdgcn_s_sleep(4);
            nap = nap < 8 ? 2 * nap : 8;
        }
        const uint64_t incmask = __ballot(st == 2);
        const int first_inc = incmask ? __ffsll((unsigned long long)incmask) - 1 : kWave;
        // ordered fold m_0 o m_1 o ... o m_first_inc (lane 0 is the nearest
        // tile, so a lower lane's map applies after a higher lane's); lane 63
        // ends with the whole fold
        if (lid > first_inc || st == 3) m = aff_identity<R, M>();
        m = wave::scan_incl(m, aff_identity<R, M>(), AffMover{},
                            [](const Aff<R, M> &higher, const Aff<R, M> &lower) { return compose(lower, higher); });
        m = aff_lane(m, kWave - 1);
        acc = compose(acc, m);
        if (first_inc < kWave) break;
        p -= kWave;
    }
#pragma unroll
    for (int i = 0; i < M; i++) carry[i] = acc.b[i];
}

// ------------------------------------------------------------ partials
struct Part {
    float ratio;
    uint32_t nonfinite;
    int64_t first_bad;
    double rsq;
    double rinf;
};

__device__ __forceinline__ Part part_neutral()
{
    Part p;
    p.ratio = 0.f;
    p.nonfinite = 0;
    p.first_bad = INT64_MAX;
    p.rsq = 0.0;
    p.rinf = 0.0;
    return p;
}

__device__ __forceinline__ void part_merge(Part &a, const Part &b)
{
    a.ratio = fmaxf(a.ratio, b.ratio);
    a.nonfinite += b.nonfinite;
    a.first_bad = min(a.first_bad, b.first_bad);
    a.rsq += b.rsq;
    a.rinf = fmax(a.rinf, b.rinf);
}

struct PartMover {
    template <int CTRL, int ROWS>
    __device__ __forceinline__ Part move(const Part &old, const Part &v) const
    {
        Part o;
        o.ratio = wave::dpp<CTRL, ROWS>(old.ratio, v.ratio);
        o.nonfinite = wave::dpp<CTRL, ROWS>(old.nonfinite, v.nonfinite);
        o.first_bad = wave::dpp<CTRL, ROWS>(old.first_bad, v.first_bad);
        o.rsq = wave::dpp<CTRL, ROWS>(old.rsq, v.rsq);
        o.rinf = wave::dpp<CTRL, ROWS>(old.rinf, v.rinf);
        return o;
    }
};

// The wave's partials folded into one, in every lane (all lanes active).
__device__ __forceinline__ Part wave_fold_part(const Part &p)
{
    Part f = wave::scan_incl(p, part_neutral(), PartMover{}, [](Part a, const Part &b) {
        part_merge(a, b);
        return a;
    });
    Part o;
    o.ratio = wave::lane_value(f.ratio, kWave - 1);
    o.nonfinite = wave::lane_value(f.nonfinite, kWave - 1);
    o.first_bad = wave::lane_value(f.first_bad, kWave - 1);
    o.rsq = wave::lane_value(f.rsq, kWave - 1);
    o.rinf = wave::lane_value(f.rinf, kWave - 1);
    return o;
}

template <typename R>
__device__ __forceinline__ float delta_ratio(R delta, R snew, double atol, double rtol)
{
    return (float)(fabs((double)delta) / (atol + rtol * fabs((double)snew)));
}
// FP32 states: the ratio in FP32 with the hardware reciprocal (one ulp); it
// only feeds the comparison with 1 and the reported maximum.
template <>
__device__ __forceinline__ float delta_ratio<float>(float delta, float snew, double atol, double rtol)
{
    return fabsf(delta) * __builtin_amdgcn_rcpf(fmaf((float)rtol, fabsf(snew), (float)atol));
}

template <typename R>
__device__ __forceinline__ void part_add(Part &p, int64_t t, R delta, R snew, R b, double atol,
                                         double rtol)
{
    float r = delta_ratio<R>(delta, snew, atol, rtol);
    if (!(r == r)) r = INFINITY;
    if (!isfinite(snew)) p.nonfinite++;
    if (r > kFreezeRatio && t < p.first_bad) p.first_bad = t;
    p.ratio = fmaxf(p.ratio, r);
    double bb = (double)b;
    p.rsq += bb * bb;
    double ab = fabs(bb);
    if (!(ab == ab)) ab = INFINITY;
    p.rinf = fmax(p.rinf, ab);
}

// ------------------------------------------------------------ IO policies
// Geometry shared by the Newton-update policies: tiles of one chain (or one
// sliding window of it) in a SegTile map.
struct SegGeom {
    const SegTile *tiles;
    int n_tiles;
    const int64_t *offsets;
    const ChainStatus *chains;
    const int32_t *chain_tile_begin;
    // > 0: the map holds one chain of this many steps from step 0, so tile ti
    // is [ti C, (ti + 1) C) and only the chain's status is loaded (one
    // dependent load before the tile's data instead of two)
    int64_t single_len;

    // [t0, t1) of the tile, its sequence head tile, false if the tile is idle.
    __device__ bool range(int ti, int C, int64_t &t0, int64_t &t1, int &head_ti) const
    {
        if (single_len > 0) {
            const ChainStatus &cs = chains[0];
            if (!cs.active) return false;
            const int64_t ws = cs.win_start > 0 ? cs.win_start : 0;
            t0 = (int64_t)ti * C;
            t1 = t0 + C < single_len ? t0 + C : single_len;
            if (cs.win_end < t1) t1 = cs.win_end;
            if (ws >= t1) return false;
            if (t0 < ws) t0 = ws;
            if (t0 >= t1) return false;
            head_ti = (int)(ws / C);
            return true;
        }
        const SegTile st = tiles[ti];
        const ChainStatus &cs = chains[st.chain];
        if (!cs.active) return false;
        const int64_t off = offsets[st.chain];
        const int64_t ws = cs.win_start > off ? cs.win_start : off;
        t1 = st.start + st.len;
        if (cs.win_end < t1) t1 = cs.win_end;
        if (ws >= t1) return false;
        t0 = st.start > ws ? st.start : ws;
        if (t0 >= t1) return false;
        // tile boundaries sit at absolute multiples of C (the first tile of a
        // chain runs from its offset to the next multiple)
        head_ti = chain_tile_begin[st.chain] + (int)(ws / C - off / C);
        return true;
    }
};

// Quasi-DEER (eq. 4) over dimension-major planes.
template <typename R>
struct DiagNewtonIO {
    using Real = R;
    static constexpr int M = 1;
    SegGeom g;
    int64_t ld;
    const R *J, *F;
    R *S;
    R *trace;
    double atol, rtol;
    struct Extra {
        R f[1];
    };
    __device__ void load(int lane, int64_t t, Aff<R, 1> &e, Extra &x) const
    {
        const size_t i = (size_t)lane * ld + t;
        const R f = F[i];
        e.a[0][0] = J[i];
        e.b[0] = f - S[i];
        x.f[0] = f;
    }
    __device__ void store(int lane, int64_t t, const Aff<R, 1> &e, const Extra &x, const R (&dp)[1],
                          const R (&dc)[1], Part &p) const
    {
        const size_t i = (size_t)lane * ld + t;
        const R s = fma(e.a[0][0], dp[0], x.f[0]);
        S[i] = s;
        if (trace) trace[i] = s;
        part_add<R>(p, t, dc[0], s, e.b[0], atol, rtol);
    }
    // Vector form (FP32): four consecutive steps from a 16-byte aligned index
    // (the planes' stride ld is a multiple of 64).
    static constexpr bool kVec = sizeof(R) == 4;
    __device__ bool vec_ok(int64_t t0) const { return (t0 & 3) == 0; }
    __device__ void load4(int lane, int64_t t, Aff<R, 1> *e, Extra *x) const
    {
        const size_t i = (size_t)lane * ld + t;
        const float4 j4 = *(const float4 *)(J + i), f4 = *(const float4 *)(F + i),
                     s4 = *(const float4 *)(S + i);
        const float jj[4] = {j4.x, j4.y, j4.z, j4.w}, ff[4] = {f4.x, f4.y, f4.z, f4.w},
                    ss[4] = {s4.x, s4.y, s4.z, s4.w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            e[q].a[0][0] = jj[q];
            e[q].b[0] = ff[q] - ss[q];
            x[q].f[0] = ff[q];
        }
    }
    // steps t .. t+nv-1 (nv <= 4) with the carry d entering step t; d leaves
    // as the carry after the last one
    __device__ void update4(int lane, int64_t t, int nv, const Aff<R, 1> *e, const Extra *x, R (&d)[1],
                            Part &p) const
    {
        const size_t i = (size_t)lane * ld + t;
        R sv[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (q < nv) {
                const R dp = d[0];
                d[0] = fma(e[q].a[0][0], dp, e[q].b[0]);
                sv[q] = fma(e[q].a[0][0], dp, x[q].f[0]);
                part_add<R>(p, t + q, d[0], sv[q], e[q].b[0], atol, rtol);
            }
        }
        if (nv == 4) {
            *(float4 *)(S + i) = make_float4(sv[0], sv[1], sv[2], sv[3]);
            if (trace) *(float4 *)(trace + i) = make_float4(sv[0], sv[1], sv[2], sv[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                if (q < nv) {
                    S[i + q] = sv[q];
                    if (trace) trace[i + q] = sv[q];
                }
            }
        }
    }
};

// Small dense DEER (eq. 3): J_t row-major [ld, M, M], states in planes.
template <typename R, int MM>
struct DenseNewtonIO {
    using Real = R;
    static constexpr int M = MM;
    SegGeom g;
    int64_t ld;
    const R *J, *F;
    R *S;
    R *trace;
    double atol, rtol;
    struct Extra {
        R f[MM];
    };
    __device__ void load(int lane, int64_t t, Aff<R, MM> &e, Extra &x) const
    {
        const R *Jt = J + (size_t)t * MM * MM;
#pragma unroll
        for (int i = 0; i < MM; i++) {
#pragma unroll
            for (int j = 0; j < MM; j++) e.a[i][j] = Jt[i * MM + j];
            const size_t k = (size_t)i * ld + t;
            x.f[i] = F[k];
            e.b[i] = x.f[i] - S[k];
        }
    }
    __device__ void store(int lane, int64_t t, const Aff<R, MM> &e, const Extra &x,
                          const R (&dp)[MM], const R (&dc)[MM], Part &p) const
    {
#pragma unroll
        for (int i = 0; i < MM; i++) {
            R s = x.f[i];
#pragma unroll
            for (int j = 0; j < MM; j++) s = fma(e.a[i][j], dp[j], s);
            const size_t k = (size_t)i * ld + t;
            S[k] = s;
            if (trace) trace[k] = s;
            part_add<R>(p, t, dc[i], s, e.b[i], atol, rtol);
        }
    }
};

// Standalone linear recursions: one sequence per lane, no chains.
struct LinGeom {
    int64_t T;
    int n_tiles;
    __device__ bool range(int ti, int C, int64_t &t0, int64_t &t1, int &head_ti) const
    {
        t0 = (int64_t)ti * C;
        t1 = t0 + C < T ? t0 + C : T;
        head_ti = 0;
        return t0 < T;
    }
};

template <typename R>
struct DiagLinIO {
    using Real = R;
    static constexpr int M = 1;
    LinGeom g;
    const R *a, *b;
    R *out;
    struct Extra {};
    __device__ void load(int lane, int64_t t, Aff<R, 1> &e, Extra &) const
    {
        const size_t i = (size_t)lane * g.T + t;
        e.a[0][0] = a[i];
        e.b[0] = b[i];
    }
    __device__ void store(int lane, int64_t t, const Aff<R, 1> &, const Extra &, const R (&)[1],
                          const R (&dc)[1], Part &) const
    {
        out[(size_t)lane * g.T + t] = dc[0];
    }
    // Vector form (FP32): needs 16-byte aligned plane offsets, so T % 4 == 0.
    static constexpr bool kVec = sizeof(R) == 4;
    __device__ bool vec_ok(int64_t t0) const { return (t0 & 3) == 0 && (g.T & 3) == 0; }
    __device__ void load4(int lane, int64_t t, Aff<R, 1> *e, Extra *) const
    {
        const size_t i = (size_t)lane * g.T + t;
        const float4 a4 = *(const float4 *)(a + i), b4 = *(const float4 *)(b + i);
        const float aa[4] = {a4.x, a4.y, a4.z, a4.w}, bb[4] = {b4.x, b4.y, b4.z, b4.w};
#pragma unroll
        for (int q = 0; q < 4; q++) {
            e[q].a[0][0] = aa[q];
            e[q].b[0] = bb[q];
        }
    }
    __device__ void update4(int lane, int64_t t, int nv, const Aff<R, 1> *e, const Extra *, R (&d)[1],
                            Part &) const
    {
        const size_t i = (size_t)lane * g.T + t;
        R v[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (q < nv) d[0] = fma(e[q].a[0][0], d[0], e[q].b[0]);
            v[q] = d[0];
        }
        if (nv == 4) {
            *(float4 *)(out + i) = make_float4(v[0], v[1], v[2], v[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (q < nv) out[i + q] = v[q];
        }
    }
    // Correction of a chunk scanned from a zero carry: v <- a v step by step
    // (v the carry's image), added to the stored values.
    __device__ void fix4(int lane, int64_t t, int nv, const Aff<R, 1> *e, R (&v)[1]) const
    {
        const size_t i = (size_t)lane * g.T + t;
        if (nv == 4) {
            float4 o = *(const float4 *)(out + i);
            float w[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                v[0] = e[q].a[0][0] * v[0];
                w[q] += v[0];
            }
            *(float4 *)(out + i) = make_float4(w[0], w[1], w[2], w[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (q < nv) {
                    v[0] = e[q].a[0][0] * v[0];
                    out[i + q] += v[0];
                }
        }
    }
};

struct Block2LinIO {
    using Real = float;
    static constexpr int M = 2;
    LinGeom g;
    int n_lanes;
    const float *coef, *rhs;
    float *out;
    struct Extra {};
    __device__ void load(int lane, int64_t t, Aff<float, 2> &e, Extra &) const
    {
        const size_t pl = (size_t)n_lanes * g.T;
        const size_t i = (size_t)lane * g.T + t;
        e.a[0][0] = coef[i];
        e.a[0][1] = coef[pl + i];
        e.a[1][0] = coef[2 * pl + i];
        e.a[1][1] = coef[3 * pl + i];
        e.b[0] = rhs[i];
        e.b[1] = rhs[pl + i];
    }
    __device__ void store(int lane, int64_t t, const Aff<float, 2> &, const Extra &,
                          const float (&)[2], const float (&dc)[2], Part &) const
    {
        const size_t pl = (size_t)n_lanes * g.T;
        const size_t i = (size_t)lane * g.T + t;
        out[i] = dc[0];
        out[pl + i] = dc[1];
    }
    // Vector form: needs 16-byte aligned plane offsets, so T % 4 == 0.
    static constexpr bool kVec = true;
    __device__ bool vec_ok(int64_t t0) const { return (t0 & 3) == 0 && (g.T & 3) == 0; }
    __device__ void load4(int lane, int64_t t, Aff<float, 2> *e, Extra *) const
    {
        const size_t pl = (size_t)n_lanes * g.T;
        const size_t i = (size_t)lane * g.T + t;
        float v[6][4];
        const float *src[6] = {coef + i, coef + pl + i, coef + 2 * pl + i, coef + 3 * pl + i, rhs + i, rhs + pl + i};
#pragma unroll
        for (int k = 0; k < 6; k++) {
            const float4 w = *(const float4 *)src[k];
            v[k][0] = w.x, v[k][1] = w.y, v[k][2] = w.z, v[k][3] = w.w;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            e[q].a[0][0] = v[0][q];
            e[q].a[0][1] = v[1][q];
            e[q].a[1][0] = v[2][q];
            e[q].a[1][1] = v[3][q];
            e[q].b[0] = v[4][q];
            e[q].b[1] = v[5][q];
        }
    }
    __device__ void update4(int lane, int64_t t, int nv, const Aff<float, 2> *e, const Extra *, float (&d)[2],
                            Part &) const
    {
        const size_t pl = (size_t)n_lanes * g.T;
        const size_t i = (size_t)lane * g.T + t;
        float p[4], q4[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if (q < nv) {
                float dp[2] = {d[0], d[1]};
                apply(e[q], dp, d);
            }
            p[q] = d[0];
            q4[q] = d[1];
        }
        if (nv == 4) {
            *(float4 *)(out + i) = make_float4(p[0], p[1], p[2], p[3]);
            *(float4 *)(out + pl + i) = make_float4(q4[0], q4[1], q4[2], q4[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++) {
                if (q < nv) {
                    out[i + q] = p[q];
                    out[pl + i + q] = q4[q];
                }
            }
        }
    }
    __device__ void fix4(int lane, int64_t t, int nv, const Aff<float, 2> *e, float (&v)[2]) const
    {
        const size_t pl = (size_t)n_lanes * g.T;
        const size_t i = (size_t)lane * g.T + t;
        if (nv == 4) {
            float4 o0 = *(const float4 *)(out + i), o1 = *(const float4 *)(out + pl + i);
            float w0[4] = {o0.x, o0.y, o0.z, o0.w}, w1[4] = {o1.x, o1.y, o1.z, o1.w};
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const float p = e[q].a[0][0] * v[0] + e[q].a[0][1] * v[1];
                const float r = e[q].a[1][0] * v[0] + e[q].a[1][1] * v[1];
                v[0] = p;
                v[1] = r;
                w0[q] += p;
                w1[q] += r;
            }
            *(float4 *)(out + i) = make_float4(w0[0], w0[1], w0[2], w0[3]);
            *(float4 *)(out + pl + i) = make_float4(w1[0], w1[1], w1[2], w1[3]);
        } else {
#pragma unroll
            for (int q = 0; q < 4; q++)
                if (q < nv) {
                    const float p = e[q].a[0][0] * v[0] + e[q].a[0][1] * v[1];
                    const float r = e[q].a[1][0] * v[0] + e[q].a[1][1] * v[1];
                    v[0] = p;
                    v[1] = r;
                    out[i + q] += p;
                    out[pl + i + q] += r;
                }
        }
    }
};

template <typename R, int MM>
struct DenseLinIO {
    using Real = R;
    static constexpr int M = MM;
    LinGeom g;
    const R *A, *b;
    R *out;
    struct Extra {};
    __device__ void load(int, int64_t t, Aff<R, MM> &e, Extra &) const
    {
#pragma unroll
        for (int i = 0; i < MM; i++) {
#pragma unroll
            for (int j = 0; j < MM; j++) e.a[i][j] = A[((size_t)t * MM + i) * MM + j];
            e.b[i] = b[(size_t)t * MM + i];
        }
    }
    __device__ void store(int, int64_t t, const Aff<R, MM> &, const Extra &, const R (&)[MM],
                          const R (&dc)[MM], Part &) const
    {
#pragma unroll
        for (int i = 0; i < MM; i++) out[(size_t)t * MM + i] = dc[i];
    }
};

template <class IO, class = void>
struct HasVec {
    static constexpr bool value = false;
};
template <class IO>
struct HasVec<IO, decltype(void(IO::kVec))> {
    static constexpr bool value = IO::kVec;
};

template <class IO>
struct HasPartials {
    static constexpr bool value = false;
};
template <typename R>
struct HasPartials<DiagNewtonIO<R>> {
    static constexpr bool value = true;
};
template <typename R, int MM>
struct HasPartials<DenseNewtonIO<R, MM>> {
    static constexpr bool value = true;
};

// ------------------------------------------------------------ the kernel
template <class IO, int BLOCK, int ITEMS>
__global__ void __launch_bounds__(BLOCK)
k_scan(IO io, ScanSync *sync, uint64_t *desc, int n_tiles, TilePartial *partials)
{
    using R = typename IO::Real;
    constexpr int M = IO::M;
    constexpr int NW = BLOCK / kWave;
    constexpr int C = BLOCK * ITEMS;
    using A = Aff<R, M>;
    using DS = Desc<R, M>;

    __shared__ A s_wagg[NW];
    __shared__ R s_carry[M];
    __shared__ Part s_part[NW];
    __shared__ uint32_t s_cnt;

    const int tid = threadIdx.x, wid = tid / kWave, lid = tid % kWave;
    if (tid == 0) s_cnt = 0;  // ordered before the waves' arrivals by the barriers below
    // only wave 0 publishes and looks back; its epoch load overlaps the data loads
    uint32_t epoch = 0;
    if (wid == 0) epoch = __hip_atomic_load(&sync->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // Consecutive workgroups take the same tile index of consecutive lanes
    // (planes), so the tiles in flight form n_lanes short look-back chains
    // instead of one long chain through a single plane.
    const uint32_t id = blockIdx.x;
    const int n_lanes = (int)(gridDim.x / (uint32_t)n_tiles);
    const int lane = (int)(id % (uint32_t)n_lanes), ti = (int)(id / (uint32_t)n_lanes);

    int64_t t0 = 0, t1 = 0;
    int head_ti = 0;
    const bool active = io.g.range(ti, C, t0, t1, head_ti);
    Part part = part_neutral();

    if (active) {
        A e[ITEMS];
        typename IO::Extra x[ITEMS];
        const int64_t base = t0 + (int64_t)tid * ITEMS;
        bool vec = false;
        // every item of this thread inside the tile: the vector loads and
        // updates run without per-item bounds (the common case)
        const bool whole = base + ITEMS <= t1;
        if constexpr (HasVec<IO>::value && ITEMS % 4 == 0) vec = io.vec_ok(t0);
        if constexpr (HasVec<IO>::value && ITEMS % 4 == 0) {
            if (vec && whole) {
#pragma unroll
                for (int i = 0; i < ITEMS; i += 4) io.load4(lane, base + i, &e[i], &x[i]);
            } else if (vec) {
#pragma unroll
                for (int i = 0; i < ITEMS; i += 4) {
                    if (base + i + 3 < t1) {
                        io.load4(lane, base + i, &e[i], &x[i]);
                    } else {
#pragma unroll
                        for (int q = 0; q < 4; q++) {
                            if (base + i + q < t1)
                                io.load(lane, base + i + q, e[i + q], x[i + q]);
                            else
                                e[i + q] = aff_identity<R, M>();
                        }
                    }
                }
            }
        }
        if (!vec) {
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (base + i < t1)
                    io.load(lane, base + i, e[i], x[i]);
                else
                    e[i] = aff_identity<R, M>();
            }
        }
        A agg = e[0];
#pragma unroll
        for (int i = 1; i < ITEMS; i++) agg = compose(e[i], agg);
        A excl;
        const A inc = wave_scan_aff(agg, excl);
        if (lid == kWave - 1) s_wagg[wid] = inc;
        lds_barrier();
        A wpre = aff_identity<R, M>();
        for (int w = 0; w < wid; w++) wpre = compose(s_wagg[w], wpre);
        if (wid == 0) {
            A total = s_wagg[0];
            for (int w = 1; w < NW; w++) total = compose(s_wagg[w], total);
            R carry[M];
#pragma unroll
            for (int i = 0; i < M; i++) carry[i] = R(0);
            const int64_t self = (int64_t)lane * n_tiles + ti;
            if (ti != head_ti) {
                if (lid == 0) publish_agg<R, M>(desc + (size_t)self * DS::kWords, epoch, total);
                lookback<R, M>(desc, self, (int64_t)lane * n_tiles + head_ti, epoch, carry, sync);
            }
            if (lid == 0) {
                R outv[M];
                apply(total, carry, outv);
                publish_inc<R, M>(desc + (size_t)self * DS::kWords, epoch, outv);
#pragma unroll
                for (int i = 0; i < M; i++) s_carry[i] = carry[i];
            }
        }
        lds_barrier();
        R d[M];
#pragma unroll
        for (int i = 0; i < M; i++) d[i] = s_carry[i];
        apply(wpre, d, d);
        apply(excl, d, d);
        if constexpr (HasVec<IO>::value && ITEMS % 4 == 0) {
            if (vec && whole) {
#pragma unroll
                for (int i = 0; i < ITEMS; i += 4) io.update4(lane, base + i, 4, &e[i], &x[i], d, part);
            } else if (vec) {
#pragma unroll
                for (int i = 0; i < ITEMS; i += 4) {
                    const int64_t left = t1 - (base + i);
                    const int nv = left >= 4 ? 4 : left > 0 ? (int)left : 0;
                    if (nv > 0) io.update4(lane, base + i, nv, &e[i], &x[i], d, part);
                }
            }
        }
        if (!vec) {
#pragma unroll
            for (int i = 0; i < ITEMS; i++) {
                if (base + i < t1) {
                    R dp[M];
#pragma unroll
                    for (int k = 0; k < M; k++) dp[k] = d[k];
                    apply(e[i], dp, d);
                    io.store(lane, base + i, e[i], x[i], dp, d, part);
                }
            }
        }
    }

    if constexpr (HasPartials<IO>::value) {
        // Each wave folds its partial and leaves it in LDS; the wave that
        // arrives last (LDS counter) folds the NW of them across its lanes
        // and writes the tile's partial, so no wave waits for the others.
        part = wave_fold_part(part);
        TilePartial &tp = partials[(size_t)lane * n_tiles + ti];
        bool write = false;
        if (!active) {
            write = wid == 0;  // every wave holds the neutral partial
        } else {
            uint32_t arrived = 0;
            if (lid == 0) {
                s_part[wid] = part;
                arrived = __hip_atomic_fetch_add(&s_cnt, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            arrived = wave::lane_value(arrived, 0);
            if (arrived == NW - 1) {
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
                part = wave_fold_part(lid < NW ? s_part[lid] : part_neutral());
                write = true;
            }
        }
        if (write && lid == 0) {
            tp.max_ratio = part.ratio;
            tp.nonfinite = part.nonfinite;
            tp.first_bad = part.first_bad;
            tp.resid_sq = part.rsq;
            tp.resid_inf = part.rinf;
        }
    }
}

// ---------------------------------------------- chunked scan (long recursions)
// For long standalone recursions each workgroup owns one contiguous chunk of
// a lane and streams it tile by tile: the next tile's loads are issued before
// the current tile is scanned, and the carry between tiles stays in
// registers, so the chunk is scanned as if its carry-in were zero without any
// wait on other workgroups.  Then one look-back per chunk (over the chunk
// aggregates, all published at about the same time) gives the true carry-in
// c, and the stored values get the correction v_t = A_t v_{t-1}, v = c at the
// chunk start (the exact difference between the two scans, by linearity).
// The correction stops after the first tile whose outgoing v is exactly zero
// in FP32, so the result is that of the full correction for any
// coefficients; when the products of the A_t decay (|a| < 1) that is the
// chunk's first tile or two.  Every workgroup of a launch is resident (at
// most one per compute unit, or a single chunk per lane), so the look-back
// always finds its predecessors running.  The streaming pass keeps DEPTH - 1
// tiles loading while it scans one (register buffers in an unrolled loop).
template <class IO, int BLOCK, int ITEMS, int DEPTH>
__global__ void __launch_bounds__(BLOCK)
k_scan_chunked(IO io, ScanSync *sync, uint64_t *desc, int n_chunks, int64_t chunk_len)
{
    using R = typename IO::Real;
    constexpr int M = IO::M;
    constexpr int NW = BLOCK / kWave;
    constexpr int C = BLOCK * ITEMS;
    using A = Aff<R, M>;
    using DS = Desc<R, M>;
    static_assert(ITEMS % 4 == 0, "vector tiles");
    static_assert(DEPTH == 2 || DEPTH == 3, "tiles in flight");

    __shared__ A s_wagg[2][NW];
    __shared__ R s_carry[M];

    const int tid = threadIdx.x, wid = tid / kWave, lid = tid % kWave;
    uint32_t epoch = 0;
    if (wid == 0) epoch = __hip_atomic_load(&sync->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int n_lanes = (int)(gridDim.x / (uint32_t)n_chunks);
    const int lane = (int)(blockIdx.x % (uint32_t)n_lanes), k = (int)(blockIdx.x / (uint32_t)n_lanes);
    // whole tiles only (the host launches this kernel when C divides T, and
    // chunk_len is a multiple of C): no load or store is conditional, so the
    // next tile's loads stay in flight while the current tile is scanned
    const int64_t c0 = (int64_t)k * chunk_len;
    const int64_t c1 = c0 + chunk_len < io.g.T ? c0 + chunk_len : io.g.T;
    const int n_t = (int)((c1 - c0) / C);
    typename IO::Extra xd[ITEMS];

    auto load_tile = [&](int j, A (&e)[ITEMS]) {
        const int64_t base = c0 + (int64_t)j * C + (int64_t)tid * ITEMS;
#pragma unroll
        for (int i = 0; i < ITEMS; i += 4) io.load4(lane, base + i, &e[i], &xd[i]);
    };
    // Tile scan: the map taking the tile's carry-in to this thread's carry-in,
    // and the tile's total map.
    auto scan_tile = [&](const A (&e)[ITEMS], int par, A &pre, A &total) {
        A agg = e[0];
#pragma unroll
        for (int i = 1; i < ITEMS; i++) agg = compose(e[i], agg);
        A excl;
        const A inc = wave_scan_aff(agg, excl);
        if (lid == kWave - 1) s_wagg[par][wid] = inc;
        lds_barrier();
        A wpre = aff_identity<R, M>();
        for (int w = 0; w < wid; w++) wpre = compose(s_wagg[par][w], wpre);
        total = wpre;
        for (int w = wid; w < NW; w++) total = compose(s_wagg[par][w], total);
        pre = compose(excl, wpre);
    };
    R d[M];
#pragma unroll
    for (int i = 0; i < M; i++) d[i] = R(0);
    A chunk = aff_identity<R, M>();
    Part part = part_neutral();
    auto zero_carry_tile = [&](const A (&e)[ITEMS], int j) {
        A pre, total;
        scan_tile(e, j & 1, pre, total);
        R dt[M];
        apply(pre, d, dt);
        const int64_t base = c0 + (int64_t)j * C + (int64_t)tid * ITEMS;
#pragma unroll
        for (int i = 0; i < ITEMS; i += 4) io.update4(lane, base + i, 4, &e[i], &xd[i], dt, part);
        apply(total, d, d);
        chunk = compose(total, chunk);
    };

    // ---- 1: the chunk from a zero carry.  DEPTH register buffers rotate
    // through an unrolled loop, so DEPTH - 1 tiles are loading while one is
    // scanned (a prefetch past the last tile reloads the last tile).
    auto tile_at = [&](int j) { return j < n_t ? j : n_t - 1; };
    A ea[ITEMS], eb[ITEMS];
    load_tile(0, ea);
    if constexpr (DEPTH == 2) {
        for (int j = 0; j < n_t; j += 2) {
            load_tile(tile_at(j + 1), eb);
            zero_carry_tile(ea, j);
            load_tile(tile_at(j + 2), ea);
            if (j + 1 < n_t) zero_carry_tile(eb, j + 1);
        }
    } else {
        A ec[ITEMS];
        load_tile(tile_at(1), eb);
        int j = 0;
        for (; j + 3 <= n_t; j += 3) {
            load_tile(tile_at(j + 2), ec);
            zero_carry_tile(ea, j);
            load_tile(tile_at(j + 3), ea);
            zero_carry_tile(eb, j + 1);
            load_tile(tile_at(j + 4), eb);
            zero_carry_tile(ec, j + 2);
        }
        if (j < n_t) zero_carry_tile(ea, j);
        if (j + 1 < n_t) zero_carry_tile(eb, j + 1);
    }

    // ---- 2: carry-in of the chunk
    if (wid == 0) {
        R carry[M];
#pragma unroll
        for (int i = 0; i < M; i++) carry[i] = R(0);
        const int64_t self = (int64_t)lane * n_chunks + k;
        if (k != 0) {
            if (lid == 0) publish_agg<R, M>(desc + (size_t)self * DS::kWords, epoch, chunk);
            lookback<R, M>(desc, self, (int64_t)lane * n_chunks, epoch, carry, sync);
        }
        if (lid == 0) {
            R outv[M];
            apply(chunk, carry, outv);
            publish_inc<R, M>(desc + (size_t)self * DS::kWords, epoch, outv);
#pragma unroll
            for (int i = 0; i < M; i++) s_carry[i] = carry[i];
        }
    }
    lds_barrier();

    // ---- 3: correction of the chunk's head
    R v[M];
    bool live = false;
#pragma unroll
    for (int i = 0; i < M; i++) {
        v[i] = s_carry[i];
        live |= v[i] != R(0);
    }
    for (int j = 0; j < n_t && live; j++) {
        load_tile(j, ea);
#pragma unroll
        for (int i = 0; i < ITEMS; i++)
#pragma unroll
            for (int r = 0; r < M; r++) ea[i].b[r] = R(0);
        A pre, total;
        scan_tile(ea, (n_t + j) & 1, pre, total);
        R vt[M];
        apply(pre, v, vt);
        const int64_t base = c0 + (int64_t)j * C + (int64_t)tid * ITEMS;
#pragma unroll
        for (int i = 0; i < ITEMS; i += 4) io.fix4(lane, base + i, 4, &ea[i], vt);
        apply(total, v, v);
        live = false;
#pragma unroll
        for (int i = 0; i < M; i++) live |= v[i] != R(0);
    }
}

// ------------------------------------------ chunked Newton scan (one chain)
// The quasi-DEER update of one long chain (eq. 4 applied to the residual of
// eq. 1): S_t <- F_t + J_t d_{t-1}, d_t = J_t d_{t-1} + F_t - S_t over the
// window [w, T) (before w the iterate is frozen: S kept, d = 0), with the
// chunked scheme of k_scan_chunked:
//  1. each workgroup scans its chunk of whole tiles from a zero carry, writes
//     the local iterate in place and each tile's convergence partial from the
//     local d; while the product of the chunk's J so far is non-zero it also
//     writes the local d into the F plane (F is not read again in the sweep);
//  2. one look-back per chunk gives the true carry c;
//  3. while that product is non-zero and v (v_t = J_t v_{t-1}, v = c at the
//     chunk start) is non-zero: d_t = d_t(local) + v_t, S_t += v_t, and the
//     tile's partial is recomputed from them (its residual fields, which do
//     not depend on the carry, are kept).
// Tiles before the window get neutral partials, as the tiled scan gives them.
struct NewtonChunkArgs {
    int n_tiles;               // T / C
    int64_t ld;                // plane stride
    const ChainStatus *chains; // chain 0
    const float *J;
    float *F, *S;
    TilePartial *partials;     // [n_lanes, n_tiles]
    double atol, rtol;
};

__device__ __forceinline__ void part_store(TilePartial &tp, const Part &p)
{
    tp.max_ratio = p.ratio;
    tp.nonfinite = p.nonfinite;
    tp.first_bad = p.first_bad;
    tp.resid_sq = p.rsq;
    tp.resid_inf = p.rinf;
}

template <int BLOCK, int ITEMS>
__global__ void __launch_bounds__(BLOCK, 1)
k_scan_newton_chunked(NewtonChunkArgs a, ScanSync *sync, uint64_t *desc, int n_chunks)
{
    constexpr int NW = BLOCK / kWave;
    constexpr int C = BLOCK * ITEMS;
    using A = Aff<float, 1>;
    using DS = Desc<float, 1>;
    static_assert(ITEMS % 4 == 0, "vector tiles");

    __shared__ A s_wagg[2][NW];
    __shared__ Part s_part[2][NW];
    __shared__ float s_carry;

    const ChainStatus &cs = a.chains[0];
    if (!cs.active) return;  // the status fold skips an inactive chain
    const int tid = threadIdx.x, wid = tid / kWave, lid = tid % kWave;
    uint32_t epoch = 0;
    if (wid == 0) epoch = __hip_atomic_load(&sync->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int n_lanes = (int)(gridDim.x / (uint32_t)n_chunks);
    const int lane = (int)(blockIdx.x % (uint32_t)n_lanes), k = (int)(blockIdx.x / (uint32_t)n_lanes);
    const int64_t ws = cs.win_start > 0 ? cs.win_start : 0;
    const int tw = (int)(ws / C);  // tile holding the window start
    TilePartial *parts = a.partials + (size_t)lane * a.n_tiles;
    for (int j = k * BLOCK + tid; j < tw; j += n_chunks * BLOCK) {
        Part p = part_neutral();
        part_store(parts[j], p);
    }
    const int tpc = (a.n_tiles - tw + n_chunks - 1) / n_chunks;
    const int j0 = tw + k * tpc;
    const int j1 = j0 + tpc < a.n_tiles ? j0 + tpc : a.n_tiles;
    if (j0 >= j1) return;  // an empty chunk is last in its lane: nothing waits for it
    const int n_t = j1 - j0;
    const size_t pl = (size_t)lane * a.ld;
    const float *Jp = a.J + pl;
    float *Fp = a.F + pl, *Sp = a.S + pl;
    const float atol = (float)a.atol, rtol = (float)a.rtol;

    // phase 1 items: J, F, S as loaded (nothing is computed from them before
    // the tile is scanned, so the loads of the next tiles stay in flight)
    struct Item {
        float j, f, s;
    };
    auto load_tile = [&](int jt, Item (&e)[ITEMS]) {
        const int64_t base = (int64_t)jt * C + (int64_t)tid * ITEMS;
#pragma unroll
        for (int i = 0; i < ITEMS; i += 4) {
            const float4 j4 = *(const float4 *)(Jp + base + i), f4 = *(const float4 *)(Fp + base + i),
                         s4 = *(const float4 *)(Sp + base + i);
            e[i] = Item{j4.x, f4.x, s4.x};
            e[i + 1] = Item{j4.y, f4.y, s4.y};
            e[i + 2] = Item{j4.z, f4.z, s4.z};
            e[i + 3] = Item{j4.w, f4.w, s4.w};
        }
    };
    // Tile scan over the items' maps: the map from the tile's carry-in to this
    // thread's, and the tile's total map.
    auto scan_tile = [&](auto map_of, int par, A &pre, A &total) {
        A agg = map_of(0);
#pragma unroll
        for (int i = 1; i < ITEMS; i++) agg = compose(map_of(i), agg);
        A excl;
        const A inc = wave_scan_aff(agg, excl);
        if (lid == kWave - 1) s_wagg[par][wid] = inc;
        lds_barrier();
        A wpre = aff_identity<float, 1>();
        for (int w = 0; w < wid; w++) wpre = compose(s_wagg[par][w], wpre);
        total = wpre;
        for (int w = wid; w < NW; w++) total = compose(s_wagg[par][w], total);
        pre = compose(excl, wpre);
    };
    // each wave leaves its folded partial in s_part[par]; after the next
    // barrier wave 0 folds the NW of them
    auto leave_part = [&](Part p, int par) {
        p = wave_fold_part(p);
        if (lid == 0) s_part[par][wid] = p;
    };
    auto fold_prev = [&](int par) {
        return wave_fold_part(lid < NW ? s_part[par][lid] : part_neutral());
    };

    // ---- 1: the chunk from a zero carry.  A step's map is (J, F - S) and
    // S_new = J d_{t-1} + F; an element before the window is (1, 0) with
    // S_new = S (the frozen iterate passes through).
    float d = 0.f;
    A chunk = aff_identity<float, 1>();
    auto zero_carry_tile = [&](const Item (&e)[ITEMS], int j) {
        const int jt = j0 + j;
        const int64_t base = (int64_t)jt * C + (int64_t)tid * ITEMS;
        A pre, total;
        scan_tile(
            [&](int i) {
                const bool frozen = base + i < ws;
                A m;
                m.a[0][0] = frozen ? 1.f : e[i].j;
                m.b[0] = frozen ? 0.f : e[i].f - e[i].s;
                return m;
            },
            j & 1, pre, total);
        if (wid == 0 && j > 0) {
            const Part p = fold_prev((j - 1) & 1);
            if (lid == 0) part_store(parts[jt - 1], p);
        }
        const bool keep_d = k != 0 && chunk.a[0][0] != 0.f;  // uniform
        float dt = fmaf(pre.a[0][0], d, pre.b[0]);
        Part p = part_neutral();
#pragma unroll
        for (int i = 0; i < ITEMS; i += 4) {
            float sv[4], dv[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                const Item &it = e[i + q];
                const bool frozen = base + i + q < ws;
                const float aa = frozen ? 1.f : it.j, bb = frozen ? 0.f : it.f - it.s;
                const float dp = dt;
                dt = fmaf(aa, dp, bb);
                sv[q] = fmaf(aa, dp, frozen ? it.s : it.f);
                dv[q] = dt;
                if (!frozen) part_add<float>(p, base + i + q, dt, sv[q], bb, a.atol, a.rtol);
            }
            *(float4 *)(Sp + base + i) = make_float4(sv[0], sv[1], sv[2], sv[3]);
            if (keep_d) *(float4 *)(Fp + base + i) = make_float4(dv[0], dv[1], dv[2], dv[3]);
        }
        leave_part(p, j & 1);
        d = fmaf(total.a[0][0], d, total.b[0]);
        chunk = compose(total, chunk);
    };
    {
        Item ea[ITEMS], eb[ITEMS];
        auto tile_at = [&](int j) { return j0 + (j < n_t ? j : n_t - 1); };
        load_tile(tile_at(0), ea);
        for (int j = 0; j < n_t; j += 2) {
            load_tile(tile_at(j + 1), eb);
            zero_carry_tile(ea, j);
            load_tile(tile_at(j + 2), ea);
            if (j + 1 < n_t) zero_carry_tile(eb, j + 1);
        }
    }
    lds_barrier();
    if (wid == 0) {
        const Part p = fold_prev((n_t - 1) & 1);
        if (lid == 0) part_store(parts[j1 - 1], p);
    }

    // ---- 2: carry-in of the chunk
    if (wid == 0) {
        float carry[1] = {0.f};
        const int64_t self = (int64_t)lane * n_chunks + k;
        if (k != 0) {
            if (lid == 0) publish_agg<float, 1>(desc + (size_t)self * DS::kWords, epoch, chunk);
            lookback<float, 1>(desc, self, (int64_t)lane * n_chunks, epoch, carry, sync);
        }
        if (lid == 0) {
            float outv[1];
            apply(chunk, carry, outv);
            publish_inc<float, 1>(desc + (size_t)self * DS::kWords, epoch, outv);
            s_carry = carry[0];
        }
    }
    __syncthreads();  // the carry, and this workgroup's partials for phase 3

    // ---- 3: correction of the chunk's head (chunks after the first, which
    // have no element before the window)
    float v = s_carry, P = 1.f;
    int j = 0;
    for (; j < n_t && v != 0.f && P != 0.f; j++) {
        const int jt = j0 + j;
        const int64_t base = (int64_t)jt * C + (int64_t)tid * ITEMS;
        float jv[ITEMS], dl[ITEMS], sl[ITEMS];  // J, the local d (in F), the local iterate (in S)
#pragma unroll
        for (int i = 0; i < ITEMS; i += 4) {
            const float4 j4 = *(const float4 *)(Jp + base + i), f4 = *(const float4 *)(Fp + base + i),
                         s4 = *(const float4 *)(Sp + base + i);
            jv[i] = j4.x, jv[i + 1] = j4.y, jv[i + 2] = j4.z, jv[i + 3] = j4.w;
            dl[i] = f4.x, dl[i + 1] = f4.y, dl[i + 2] = f4.z, dl[i + 3] = f4.w;
            sl[i] = s4.x, sl[i + 1] = s4.y, sl[i + 2] = s4.z, sl[i + 3] = s4.w;
        }
        A pre, total;
        scan_tile(
            [&](int i) {
                A m;
                m.a[0][0] = jv[i];
                m.b[0] = 0.f;
                return m;
            },
            (n_t + j) & 1, pre, total);
        if (wid == 0 && j > 0) {
            Part p = fold_prev((n_t + j - 1) & 1);
            if (lid == 0) {
                const TilePartial &old = parts[jt - 1];
                p.rsq = old.resid_sq;
                p.rinf = old.resid_inf;
                part_store(parts[jt - 1], p);
            }
        }
        float vt = pre.a[0][0] * v;
        Part p = part_neutral();
#pragma unroll
        for (int i = 0; i < ITEMS; i += 4) {
            float sv[4];
#pragma unroll
            for (int q = 0; q < 4; q++) {
                vt = jv[i + q] * vt;
                sv[q] = sl[i + q] + vt;
                part_add<float>(p, base + i + q, dl[i + q] + vt, sv[q], 0.f, a.atol, a.rtol);
            }
            *(float4 *)(Sp + base + i) = make_float4(sv[0], sv[1], sv[2], sv[3]);
        }
        leave_part(p, (n_t + j) & 1);
        v = total.a[0][0] * v;
        P *= total.a[0][0];
    }
    if (j > 0) {
        lds_barrier();
        if (wid == 0) {
            Part p = fold_prev((n_t + j - 1) & 1);
            if (lid == 0) {
                const TilePartial &old = parts[j0 + j - 1];
                p.rsq = old.resid_sq;
                p.rinf = old.resid_inf;
                part_store(parts[j0 + j - 1], p);
            }
        }
    }
}

// Advances the descriptor epoch after a scan, so the next launch (or graph
// replay) ignores every descriptor this one wrote.
__global__ void k_bump_epoch(ScanSync *sync)
{
    const uint32_t e = __hip_atomic_load(&sync->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&sync->epoch, (e + 1) & 0x3fffffffu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// With `timed`, the scan kernel (not the epoch advance) is bracketed by the
// context's events kev[0] and kev[1].
template <class IO, int BLOCK, int ITEMS>
pmc_status run_scan(pmc_context *ctx, const IO &io, int n_lanes, int n_tiles, TilePartial *partials,
                    bool bump = true, bool timed = false)
{
    using DS = Desc<typename IO::Real, IO::M>;
    const size_t n_desc = (size_t)n_lanes * n_tiles;
    if (n_desc == 0) return PMC_OK;
    if (n_desc > 0x7fffffffULL) {
        set_error("scan: %zu tiles exceed the launch limit", n_desc);
        return PMC_ERR_UNSUPPORTED;
    }
    PMC_TRY(ensure_lb_desc(ctx, n_desc * DS::kWords * sizeof(uint64_t)));
    if (timed) PMC_TRY_HIP(hipEventRecord(ctx->kev[0], ctx->stream));
    hipLaunchKernelGGL((k_scan<IO, BLOCK, ITEMS>), dim3((unsigned)n_desc), dim3(BLOCK), 0,
                       ctx->stream, io, ctx->sync, (uint64_t *)ctx->lb_desc, n_tiles, partials);
    PMC_TRY_HIP(hipGetLastError());
    if (timed) PMC_TRY_HIP(hipEventRecord(ctx->kev[1], ctx->stream));
    if (bump) {
        hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(1), 0, ctx->stream, ctx->sync);
        PMC_TRY_HIP(hipGetLastError());
    }
    return PMC_OK;
}

// Chunked scan of a long standalone recursion whose length is a multiple of
// the tile: one chunk per compute unit.
template <class IO, int BLOCK, int ITEMS, int DEPTH>
pmc_status run_scan_chunked(pmc_context *ctx, const IO &io, int n_lanes, int64_t T, bool timed)
{
    using DS = Desc<typename IO::Real, IO::M>;
    constexpr int C = BLOCK * ITEMS;
    const int n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
    int want = n_lanes >= n_cu ? 1 : n_cu / n_lanes;
    const int64_t tiles = T / C;
    if (want > tiles) want = (int)tiles;
    const int64_t chunk_len = (tiles + want - 1) / want * C;
    const int n_chunks = (int)((T + chunk_len - 1) / chunk_len);
    const size_t n_wg = (size_t)n_lanes * n_chunks;
    if (n_wg == 0) return PMC_OK;
    if (n_wg > 0x7fffffffULL) {
        set_error("scan: %zu chunks exceed the launch limit", n_wg);
        return PMC_ERR_UNSUPPORTED;
    }
    PMC_TRY(ensure_lb_desc(ctx, n_wg * DS::kWords * sizeof(uint64_t)));
    if (timed) PMC_TRY_HIP(hipEventRecord(ctx->kev[0], ctx->stream));
    hipLaunchKernelGGL((k_scan_chunked<IO, BLOCK, ITEMS, DEPTH>), dim3((unsigned)n_wg), dim3(BLOCK), 0, ctx->stream, io,
                       ctx->sync, (uint64_t *)ctx->lb_desc, n_chunks, chunk_len);
    PMC_TRY_HIP(hipGetLastError());
    if (timed) PMC_TRY_HIP(hipEventRecord(ctx->kev[1], ctx->stream));
    hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(1), 0, ctx->stream, ctx->sync);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

// ------------------------------------------------------- chain status fold
namespace {

constexpr int kStatusThreads = 256;

struct Fold {
    double q, qi;
    float r;
    uint32_t f;
    int64_t fb;
};

__device__ __forceinline__ void fold_merge(Fold &v, const Fold &o)
{
    v.q += o.q;
    v.qi = fmax(v.qi, o.qi);
    v.r = fmaxf(v.r, o.r);
    v.f += o.f;
    v.fb = o.fb < v.fb ? o.fb : v.fb;
}

struct FoldMover {
    template <int CTRL, int ROWS>
    __device__ __forceinline__ Fold move(const Fold &old, const Fold &v) const
    {
        Fold o;
        o.q = wave::dpp<CTRL, ROWS>(old.q, v.q);
        o.qi = wave::dpp<CTRL, ROWS>(old.qi, v.qi);
        o.r = wave::dpp<CTRL, ROWS>(old.r, v.r);
        o.f = wave::dpp<CTRL, ROWS>(old.f, v.f);
        o.fb = wave::dpp<CTRL, ROWS>(old.fb, v.fb);
        return o;
    }
};

// Block-wide fold of per-thread values; the result is valid in thread 0.
// Fixed tree order, so the FP64 sums are deterministic.
__device__ Fold block_fold(Fold v)
{
    __shared__ Fold s_w[kStatusThreads / 64];
    v = wave::scan_incl(v, Fold{0.0, 0.0, 0.f, 0u, INT64_MAX}, FoldMover{}, [](Fold a, const Fold &o) {
        fold_merge(a, o);
        return a;
    });
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) s_w[w] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        v = s_w[0];
        for (int i = 1; i < kStatusThreads / 64; i++) fold_merge(v, s_w[i]);
    }
    __syncthreads();
    return v;
}

}  // namespace

// One workgroup per chain folds that chain's tile partials (all lanes) and
// updates its Newton state; the last workgroup to finish folds every chain
// into the global status and re-arms the completion counter, so the kernel
// can be replayed inside a captured graph.
// One chain's Newton state after a sweep, from the fold of its tile partials
// (off and cend are the chain's first and one-past-last step).
__device__ void chain_update(ChainStatus &cs, const Fold &v, const StatusArgs &a, int64_t off, int64_t cend)
{
    const float r = v.r;
    const int64_t fb = v.fb;
    cs.sweeps += 1;
    cs.max_ratio = r;
    cs.first_bad = fb;
    cs.resid_sq = v.q;
    cs.resid_inf = v.qi;
    cs.nonfinite = v.f;
    // Plateau detection: progress is a 2x drop of the best ratio or an
    // advance of the converged front; rounding noise gives neither.
    const int64_t front = fb == INT64_MAX ? cs.win_end : fb;
    if (r < 0.5f * cs.best_ratio || front > cs.best_front) {
        cs.best_ratio = fminf(cs.best_ratio, r);
        cs.best_front = front > cs.best_front ? front : cs.best_front;
        cs.stall = 0;
    } else {
        cs.stall += 1;
    }
    // Refined products: the tolerance met (or the rounding floor reached)
    // with the split-FP16 evaluation starts the final phase instead of
    // stopping: FP32 products from the chain's first step, with the window
    // and the plateau detection started afresh, until the tolerance is met
    // again under them.
    const bool floor_hit = a.floor_stall > 0 && cs.stall >= a.floor_stall && r <= 2.f;
    if (!cs.fine && ((r <= 1.f && cs.win_end >= cend) || floor_hit)) {
        if (cs.sweeps >= a.max_iter) {  // no sweep left for the final phase
            cs.active = 0;
            return;
        }
        cs.fine = 1;
        cs.win_start = off;
        cs.fb_prev = off;
        cs.best_front = off;
        cs.best_ratio = INFINITY;
        cs.stall = 0;
        return;
    }
    if (r <= 1.f && cs.win_end >= cend) {
        cs.converged = 1;
        cs.active = 0;
    } else if (r <= 1.f) {
        // a fixed-width window whose steps all met the tolerance: the next
        // window starts where this one ended
        cs.win_start = cs.win_end;
        cs.win_end = cs.win_start + a.window_width < cend ? cs.win_start + a.window_width : cend;
        cs.fb_prev = cs.win_start;
    } else if (cs.sweeps >= a.max_iter) {
        cs.active = 0;
    } else if (floor_hit) {
        // rounding floor: no progress for floor_stall sweeps with the last change within
        // twice the tolerance (the state error of a change-based stop is a few times the
        // last change, so this keeps it near the converged chains' error)
        cs.at_floor = 1;
        cs.active = 0;
    } else if (a.skip_prefix && fb != INT64_MAX) {
        // the window starts at the first step that has not met the
        // tolerance in both of the last two sweeps (its frozen
        // residual is then the second, smaller change), rounded down
        // to a multiple of 4 (aligned vector loads)
        const int64_t f2 = fb < cs.fb_prev ? fb : cs.fb_prev;
        const int64_t w = f2 & ~(int64_t)3;
        cs.win_start = w > off ? w : off;
        if (a.window_width > 0) {
            const int64_t e = cs.win_start + a.window_width;
            cs.win_end = e < cend ? e : cend;
        }
    }
    if (!(r <= 1.f)) cs.fb_prev = fb;
}

__global__ void __launch_bounds__(kStatusThreads) k_status(StatusArgs a)
{
    const int c = blockIdx.x, tid = threadIdx.x;
    ChainStatus &cs = a.chains[c];
    if (cs.active && !a.fold_only) {  // uniform per block
        const int k0 = a.chain_tile_begin[c], ntc = a.chain_tile_begin[c + 1] - k0;
        const int64_t cnt = (int64_t)a.n_lanes * ntc;
        Fold v{0.0, 0.0, 0.f, 0u, INT64_MAX};
        for (int64_t i = tid; i < cnt; i += kStatusThreads) {
            const int l = (int)(i / ntc), k = k0 + (int)(i - (int64_t)l * ntc);
            const TilePartial &p = a.partials[(size_t)l * a.n_tiles + k];
            v.r = fmaxf(v.r, p.max_ratio);
            v.fb = p.first_bad < v.fb ? p.first_bad : v.fb;
            v.q += p.resid_sq;
            v.qi = fmax(v.qi, p.resid_inf);
            v.f += p.nonfinite;
        }
        v = block_fold(v);
        if (tid == 0) {
            ChainStatus x = cs;
            chain_update(x, v, a, a.offsets[c], a.offsets[c + 1]);
            cs = x;
        }
    }
    // completion count: the last workgroup sees every chain's update (a
    // single workgroup is its own last one and needs neither the device-scope
    // fences nor the counter)
    const bool single = gridDim.x == 1;
    __shared__ int s_last;
    if (!single) __threadfence();
    __syncthreads();
    if (tid == 0) s_last = single || atomicAdd(&a.global->fold_ctr, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last) return;
    if (!single) __threadfence();
    __shared__ int s_cnt[kStatusThreads / 64][5];
    Fold v{0.0, 0.0, 0.f, 0u, INT64_MAX};
    int nact = 0, nconv = 0, nfloor = 0, sweeps = 0, nfine = 0;
    int64_t nsteps = 0;
    for (int i = tid; i < a.n_chains; i += kStatusThreads) {
        const ChainStatus &o = a.chains[i];
        if (o.active) {
            const int64_t off = a.offsets[i];
            nsteps += o.win_end - (o.win_start > off ? o.win_start : off);
        }
        v.q += o.resid_sq;
        v.qi = fmax(v.qi, o.resid_inf);
        v.r = fmaxf(v.r, o.max_ratio);
        v.f += o.nonfinite;
        nact += o.active;
        nfine += o.active && o.fine;
        nconv += o.converged;
        nfloor += o.at_floor;
        sweeps = max(sweeps, o.sweeps);
    }
    nact = wave::reduce_sum(nact);
    nfine = wave::reduce_sum(nfine);
    nconv = wave::reduce_sum(nconv);
    nfloor = wave::reduce_sum(nfloor);
    sweeps = wave::reduce_max(sweeps, INT32_MIN);
    nsteps = wave::reduce_sum(nsteps);
    __shared__ int64_t s_steps[kStatusThreads / 64];
    if ((tid & 63) == 0) {
        s_cnt[tid >> 6][0] = nact;
        s_cnt[tid >> 6][1] = nconv;
        s_cnt[tid >> 6][2] = nfloor;
        s_cnt[tid >> 6][3] = sweeps;
        s_cnt[tid >> 6][4] = nfine;
        s_steps[tid >> 6] = nsteps;
    }
    v = block_fold(v);
    if (tid == 0) {
        for (int w = 1; w < kStatusThreads / 64; w++) {
            nact += s_cnt[w][0];
            nconv += s_cnt[w][1];
            nfloor += s_cnt[w][2];
            sweeps = max(sweeps, s_cnt[w][3]);
            nfine += s_cnt[w][4];
            nsteps += s_steps[w];
        }
        GlobalStatus *g = a.global;
        g->n_active = nact;
        g->n_fine = nfine;
        g->n_converged = nconv;
        g->n_floor = nfloor;
        g->sweeps = sweeps;
        g->resid_sq = v.q;
        g->resid_inf = v.qi;
        g->max_ratio = v.r;
        g->nonfinite = v.f;
        g->n_accept = 0;
        if (!a.fold_only) {
            g->eval_steps += g->next_steps;  // what this sweep evaluated
            g->next_steps = nsteps;
        }
        if (a.bump_epoch) {
            ScanSync *sy = a.bump_epoch;
            const uint32_t e = __hip_atomic_load(&sy->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&sy->epoch, (e + 1) & 0x3fffffffu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (!single) __hip_atomic_store(&g->fold_ctr, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The status fold of a problem with one chain, in one workgroup: every load
// the fold needs (the chain's state, its tile partials, which are all the
// map's tiles, the global counters and the scan epoch) is issued at the
// start, and the global status is written from the updated chain state held
// in registers, so the launch waits for one round of loads instead of a
// chain of dependent ones.  Same results as k_status with one workgroup.
__global__ void __launch_bounds__(kStatusThreads) k_status_one(StatusArgs a)
{
    const int tid = threadIdx.x;
    ChainStatus cs;
    int64_t cend = 0, eval_steps = 0, next_steps = 0;
    uint32_t epoch = 0;
    if (tid == 0) {
        cs = a.chains[0];
        cend = a.offsets[1];
        eval_steps = a.global->eval_steps;
        next_steps = a.global->next_steps;
        if (a.bump_epoch) epoch = __hip_atomic_load(&a.bump_epoch->epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    Fold v{0.0, 0.0, 0.f, 0u, INT64_MAX};
    const int64_t cnt = (int64_t)a.n_lanes * a.n_tiles;
    for (int64_t i = tid; i < cnt; i += kStatusThreads) {
        const TilePartial &p = a.partials[i];
        v.r = fmaxf(v.r, p.max_ratio);
        v.fb = p.first_bad < v.fb ? p.first_bad : v.fb;
        v.q += p.resid_sq;
        v.qi = fmax(v.qi, p.resid_inf);
        v.f += p.nonfinite;
    }
    v = block_fold(v);
    if (tid != 0) return;
    if (cs.active && !a.fold_only) {
        chain_update(cs, v, a, 0, cend);
        a.chains[0] = cs;
    }
    GlobalStatus *g = a.global;
    g->n_active = cs.active;
    g->n_fine = cs.active && cs.fine;
    g->n_converged = cs.converged;
    g->n_floor = cs.at_floor;
    g->sweeps = cs.sweeps;
    g->resid_sq = cs.resid_sq;
    g->resid_inf = cs.resid_inf;
    g->max_ratio = cs.max_ratio;
    g->nonfinite = cs.nonfinite;
    g->n_accept = 0;
    if (!a.fold_only) {
        g->eval_steps = eval_steps + next_steps;  // what this sweep evaluated
        g->next_steps = cs.active ? cs.win_end - (cs.win_start > 0 ? cs.win_start : 0) : 0;
    }
    if (a.bump_epoch)
        __hip_atomic_store(&a.bump_epoch->epoch, (epoch + 1) & 0x3fffffffu, __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

// Number of accepted proposals: a grid-stride byte count added into the
// global status (which the preceding status fold has set to zero).
__global__ void __launch_bounds__(256) k_count_accept(const uint8_t *__restrict__ acc, int64_t n,
                                                      GlobalStatus *g)
{
    uint32_t s = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        s += acc[i];
    s = wave::reduce_sum(s);
    __shared__ uint32_t s_w[4];
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0)
        atomicAdd((unsigned long long *)&g->n_accept,
                  (unsigned long long)(s_w[0] + s_w[1] + s_w[2] + s_w[3]));
}

}  // namespace

// ------------------------------------------------------------ launchers
namespace {
// The chunked Newton scan: one chain, whole 8192-step tiles (512 threads x 16
// steps: the tiled scan's tile, with the registers for two tiles in flight),
// no trace, large scans.
pmc_status newton_chunked(pmc_context *ctx, const NewtonScanArgs &a)
{
    constexpr int BLOCK = 512, ITEMS = 16;
    using DS = Desc<float, 1>;
    const int n_cu = ctx->n_cu > 0 ? ctx->n_cu : 256;
    int n_chunks = a.n_lanes >= n_cu ? 1 : n_cu / a.n_lanes;
    if (n_chunks > a.n_tiles) n_chunks = a.n_tiles;
    const size_t n_wg = (size_t)a.n_lanes * n_chunks;
    PMC_TRY(ensure_lb_desc(ctx, n_wg * DS::kWords * sizeof(uint64_t)));
    NewtonChunkArgs c{a.n_tiles, a.ld, a.chains, (const float *)a.J, (float *)a.F, (float *)a.S, a.partials,
                      a.atol, a.rtol};
    hipLaunchKernelGGL((k_scan_newton_chunked<BLOCK, ITEMS>), dim3((unsigned)n_wg), dim3(BLOCK), 0, ctx->stream, c,
                       ctx->sync, (uint64_t *)ctx->lb_desc, n_chunks);
    PMC_TRY_HIP(hipGetLastError());
    if (!a.defer_epoch) {
        hipLaunchKernelGGL(k_bump_epoch, dim3(1), dim3(1), 0, ctx->stream, ctx->sync);
        PMC_TRY_HIP(hipGetLastError());
    }
    return PMC_OK;
}

// Steps of the one chain of a tile map that holds a single chain cut at
// multiples of C (the chain starts at step 0), else 0.
int64_t single_chain_len(const NewtonScanArgs &a, int C)
{
    if (a.n_chains != 1 || a.n_steps <= 0 || a.n_tiles != (a.n_steps + C - 1) / C) return 0;
    return a.n_steps;
}

template <typename R, int BLOCK, int ITEMS>
pmc_status diag_newton(pmc_context *ctx, const NewtonScanArgs &a)
{
    if constexpr (sizeof(R) == 4 && BLOCK == 1024 && ITEMS == 8) {
        constexpr int C = BLOCK * ITEMS;
        if (a.n_chains == 1 && !a.trace && !a.fixed_window && a.n_steps % C == 0 && a.n_tiles == a.n_steps / C &&
            a.ld == a.n_steps && (int64_t)a.n_lanes * a.n_steps >= (int64_t(1) << 23))
            return newton_chunked(ctx, a);
    }
    SegGeom g{a.tiles, a.n_tiles, a.offsets, a.chains, a.chain_tile_begin, single_chain_len(a, BLOCK * ITEMS)};
    DiagNewtonIO<R> io{g, a.ld, (const R *)a.J, (const R *)a.F, (R *)a.S, (R *)a.trace, a.atol, a.rtol};
    return run_scan<DiagNewtonIO<R>, BLOCK, ITEMS>(ctx, io, a.n_lanes, a.n_tiles, a.partials, !a.defer_epoch);
}
template <typename R, int MM, int BLOCK, int ITEMS>
pmc_status dense_newton(pmc_context *ctx, const NewtonScanArgs &a)
{
    SegGeom g{a.tiles, a.n_tiles, a.offsets, a.chains, a.chain_tile_begin, single_chain_len(a, BLOCK * ITEMS)};
    DenseNewtonIO<R, MM> io{g, a.ld, (const R *)a.J, (const R *)a.F, (R *)a.S, (R *)a.trace, a.atol,
                            a.rtol};
    return run_scan<DenseNewtonIO<R, MM>, BLOCK, ITEMS>(ctx, io, 1, a.n_tiles, a.partials, !a.defer_epoch);
}
}  // namespace

int scan_tile_steps(pmc_dtype dt, int variant_m, int items, int block)
{
    if (variant_m > 1) return 256 * (variant_m == 2 ? 4 : 2);
    if (dt == PMC_F64) return 256 * (items >= 8 ? 8 : 4);
    if (block == 1024) return 1024 * (items >= 16 ? 16 : 8);
    if (block == 512) return 512 * (items >= 16 ? 16 : 8);
    return 256 * (items >= 16 ? 16 : (items >= 8 ? 8 : 4));
}

pmc_status launch_newton_scan_diag(pmc_context *ctx, pmc_dtype dt, const NewtonScanArgs &a,
                                   int items, int block)
{
    if (dt == PMC_F64) {
        if (items >= 8) return diag_newton<double, 256, 8>(ctx, a);
        return diag_newton<double, 256, 4>(ctx, a);
    }
    if (block == 1024) {
        if (items >= 16) return diag_newton<float, 1024, 16>(ctx, a);
        return diag_newton<float, 1024, 8>(ctx, a);
    }
    if (block == 512) {
        if (items >= 16) return diag_newton<float, 512, 16>(ctx, a);
        return diag_newton<float, 512, 8>(ctx, a);
    }
    if (items >= 16) return diag_newton<float, 256, 16>(ctx, a);
    if (items >= 8) return diag_newton<float, 256, 8>(ctx, a);
    return diag_newton<float, 256, 4>(ctx, a);
}

pmc_status launch_newton_scan_dense_small(pmc_context *ctx, pmc_dtype dt, int D,
                                          const NewtonScanArgs &a)
{
    if (dt == PMC_F64) {
        switch (D) {
        case 2: return dense_newton<double, 2, 256, 4>(ctx, a);
        case 3: return dense_newton<double, 3, 256, 2>(ctx, a);
        case 4: return dense_newton<double, 4, 256, 2>(ctx, a);
        }
    } else {
        switch (D) {
        case 2: return dense_newton<float, 2, 256, 4>(ctx, a);
        case 3: return dense_newton<float, 3, 256, 2>(ctx, a);
        case 4: return dense_newton<float, 4, 256, 2>(ctx, a);
        }
    }
    set_error("dense VALU scan supports D <= 4 (got %d)", D);
    return PMC_ERR_UNSUPPORTED;
}

pmc_status launch_linrec_diag(pmc_context *ctx, pmc_dtype dt, int n_lanes, int64_t T, const void *a,
                              const void *b, void *out)
{
    const bool timed = ctx->scan_timing != 0;
    if (dt == PMC_F64) {
        constexpr int C = 256 * 8;
        int nt = (int)((T + C - 1) / C);
        DiagLinIO<double> io{LinGeom{T, nt}, (const double *)a, (const double *)b, (double *)out};
        return run_scan<DiagLinIO<double>, 256, 8>(ctx, io, n_lanes, nt, nullptr, true, timed);
    }
    // long recursions: chunked scan (one chunk per compute unit)
    if ((int64_t)n_lanes * T >= (int64_t(1) << 23) && T % (1024 * 8) == 0) {
        DiagLinIO<float> io{LinGeom{T, 0}, (const float *)a, (const float *)b, (float *)out};
        return run_scan_chunked<DiagLinIO<float>, 1024, 8, 3>(ctx, io, n_lanes, T, timed);
    }
    // the Newton scan's rule: larger tiles (fewer look-back hops) for large scans
    if ((int64_t)n_lanes * T >= (int64_t(1) << 23)) {
        constexpr int C = 1024 * 8;
        int nt = (int)((T + C - 1) / C);
        DiagLinIO<float> io{LinGeom{T, nt}, (const float *)a, (const float *)b, (float *)out};
        return run_scan<DiagLinIO<float>, 1024, 8>(ctx, io, n_lanes, nt, nullptr, true, timed);
    }
    constexpr int C = 512 * 8;
    int nt = (int)((T + C - 1) / C);
    DiagLinIO<float> io{LinGeom{T, nt}, (const float *)a, (const float *)b, (float *)out};
    return run_scan<DiagLinIO<float>, 512, 8>(ctx, io, n_lanes, nt, nullptr, true, timed);
}

pmc_status launch_linrec_block2(pmc_context *ctx, int n_lanes, int64_t T, const void *coef,
                                const void *rhs, void *out)
{
    const bool timed = ctx->scan_timing != 0;
    if ((int64_t)n_lanes * T >= (int64_t(1) << 22) && T % (1024 * 4) == 0) {
        Block2LinIO io{LinGeom{T, 0}, n_lanes, (const float *)coef, (const float *)rhs, (float *)out};
        return run_scan_chunked<Block2LinIO, 1024, 4, 2>(ctx, io, n_lanes, T, timed);
    }
    if ((int64_t)n_lanes * T >= (int64_t(1) << 22)) {
        constexpr int C = 1024 * 4;
        int nt = (int)((T + C - 1) / C);
        Block2LinIO io{LinGeom{T, nt}, n_lanes, (const float *)coef, (const float *)rhs, (float *)out};
        return run_scan<Block2LinIO, 1024, 4>(ctx, io, n_lanes, nt, nullptr, true, timed);
    }
    constexpr int C = 256 * 4;
    int nt = (int)((T + C - 1) / C);
    Block2LinIO io{LinGeom{T, nt}, n_lanes, (const float *)coef, (const float *)rhs, (float *)out};
    return run_scan<Block2LinIO, 256, 4>(ctx, io, n_lanes, nt, nullptr, true, timed);
}

pmc_status launch_linrec_dense_small(pmc_context *ctx, int D, int64_t T, const double *A,
                                     const double *b, double *out)
{
    constexpr int C2 = 256 * 4, C4 = 256 * 2;
    switch (D) {
    case 1: return launch_linrec_diag(ctx, PMC_F64, 1, T, A, b, out);
    case 2: {
        int nt = (int)((T + C2 - 1) / C2);
        DenseLinIO<double, 2> io{LinGeom{T, nt}, A, b, out};
        return run_scan<DenseLinIO<double, 2>, 256, 4>(ctx, io, 1, nt, nullptr);
    }
    case 3: {
        int nt = (int)((T + C4 - 1) / C4);
        DenseLinIO<double, 3> io{LinGeom{T, nt}, A, b, out};
        return run_scan<DenseLinIO<double, 3>, 256, 2>(ctx, io, 1, nt, nullptr);
    }
    case 4: {
        int nt = (int)((T + C4 - 1) / C4);
        DenseLinIO<double, 4> io{LinGeom{T, nt}, A, b, out};
        return run_scan<DenseLinIO<double, 4>, 256, 2>(ctx, io, 1, nt, nullptr);
    }
    }
    set_error("dense FP64 scan supports D <= 4 (got %d)", D);
    return PMC_ERR_UNSUPPORTED;
}

pmc_status check_scan_health(pmc_context *ctx)
{
    ScanSync h;
    PMC_TRY_HIP(hipMemcpyAsync(&h, ctx->sync, sizeof(h), hipMemcpyDeviceToHost, ctx->stream));
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (h.pad) {
        set_error("scan look-back timed out (a predecessor tile never published)");
        return PMC_ERR_HIP;
    }
    return PMC_OK;
}

pmc_status launch_status(pmc_context *ctx, const StatusArgs &a)
{
    if (a.n_chains <= 0) return PMC_OK;
    if (a.n_chains == 1)
        hipLaunchKernelGGL(k_status_one, dim3(1), dim3(kStatusThreads), 0, ctx->stream, a);
    else
        hipLaunchKernelGGL(k_status, dim3(a.n_chains), dim3(kStatusThreads), 0, ctx->stream, a);
    PMC_TRY_HIP(hipGetLastError());
    if (a.accept && a.n_steps > 0) {
        const int64_t per = 256 * 16;
        const int blocks = (int)std::min<int64_t>(1024, (a.n_steps + per - 1) / per);
        hipLaunchKernelGGL(k_count_accept, dim3(blocks), dim3(256), 0, ctx->stream, a.accept,
                           a.n_steps, a.global);
        PMC_TRY_HIP(hipGetLastError());
    }
    return PMC_OK;
}

}  // namespace pmc
