// Cross-lane primitives for 64-lane wavefronts on gfx950 built on DPP
// (data-parallel primitives: a lane reads another lane's register inside a
// vector instruction), so scans and folds across a wave stay on the vector
// ALU instead of the LDS crossbar that ds_bpermute (and so __shfl_*) uses.
//
// GFX9 DPP controls used here:
//   row_shr:n    lane i reads lane i - n of its own 16-lane row;
//   row_bcast:15 rows 1, 2, 3 read the last lane of the previous row;
//   row_bcast:31 rows 2 and 3 read lane 31;
//   wave_shr:1   lane i reads lane i - 1 across the whole wave.
// A lane whose source lies outside the pattern, or whose row is masked off,
// keeps the `old` operand (bound_ctrl off).  Every helper must be called with
// all 64 lanes active.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pmc {
namespace wave {

constexpr int kRowShr = 0x110;  // + n, n = 1..15
constexpr int kWaveShr1 = 0x138;
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp32(uint32_t old, uint32_t v)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)v, CTRL, ROWS, 0xf, false);
}

template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ float dpp(float old, float v)
{
    return __uint_as_float(dpp32<CTRL, ROWS>(__float_as_uint(old), __float_as_uint(v)));
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint32_t dpp(uint32_t old, uint32_t v)
{
    return dpp32<CTRL, ROWS>(old, v);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int dpp(int old, int v)
{
    return (int)dpp32<CTRL, ROWS>((uint32_t)old, (uint32_t)v);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ uint64_t dpp(uint64_t old, uint64_t v)
{
    const uint32_t lo = dpp32<CTRL, ROWS>((uint32_t)old, (uint32_t)v);
    const uint32_t hi = dpp32<CTRL, ROWS>((uint32_t)(old >> 32), (uint32_t)(v >> 32));
    return ((uint64_t)hi << 32) | lo;
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ int64_t dpp(int64_t old, int64_t v)
{
    return (int64_t)dpp<CTRL, ROWS>((uint64_t)old, (uint64_t)v);
}
template <int CTRL, int ROWS = 0xf>
__device__ __forceinline__ double dpp(double old, double v)
{
    return __longlong_as_double(
        (long long)dpp<CTRL, ROWS>((uint64_t)__double_as_longlong(old), (uint64_t)__double_as_longlong(v)));
}

// Value of lane `l` (a compile-time or wave-uniform index) in every lane.
__device__ __forceinline__ float lane_value(float v, int l)
{
    return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)__float_as_uint(v), l));
}
__device__ __forceinline__ uint32_t lane_value(uint32_t v, int l)
{
    return (uint32_t)__builtin_amdgcn_readlane((int)v, l);
}
__device__ __forceinline__ int lane_value(int v, int l) { return __builtin_amdgcn_readlane(v, l); }
__device__ __forceinline__ uint64_t lane_value(uint64_t v, int l)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
    return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ int64_t lane_value(int64_t v, int l) { return (int64_t)lane_value((uint64_t)v, l); }
__device__ __forceinline__ double lane_value(double v, int l)
{
    return __longlong_as_double((long long)lane_value((uint64_t)__double_as_longlong(v), l));
}

// Inclusive scan across the wave in lane order with an associative operator
// `later_after(x_later, x_earlier)`: lane l ends with x_l . x_{l-1} ... x_0
// (the lower lane is the earlier operand).  The Mover's move<CTRL, ROWS>(old,
// v) moves every register of a T with one DPP pattern, so aggregates of
// several registers move as one.  A lane whose source is outside the pattern
// keeps its value (`ident` is only the DPP fallback operand), so the operator
// is never applied to the fallback.  Hillis-Steele steps of 1, 2, 4, 8 inside
// each 16-lane row, then the row totals through the two broadcasts.
template <class T, class Mover, class Op>
__device__ __forceinline__ T scan_incl(T v, const T &ident, Mover mv, Op later_after)
{
    const int l = (int)(threadIdx.x & 63), r = l & 15, row = l >> 4;
    T t;
    t = mv.template move<kRowShr + 1, 0xf>(ident, v);
    if (r >= 1) v = later_after(v, t);
    t = mv.template move<kRowShr + 2, 0xf>(ident, v);
    if (r >= 2) v = later_after(v, t);
    t = mv.template move<kRowShr + 4, 0xf>(ident, v);
    if (r >= 4) v = later_after(v, t);
    t = mv.template move<kRowShr + 8, 0xf>(ident, v);
    if (r >= 8) v = later_after(v, t);
    t = mv.template move<kRowBcast15, 0xa>(ident, v);
    if (row & 1) v = later_after(v, t);
    t = mv.template move<kRowBcast31, 0xc>(ident, v);
    if (row >= 2) v = later_after(v, t);
    return v;
}

// Shift by one lane across the wave: lane l gets lane l - 1, lane 0 `ident`.
template <class T, class Mover>
__device__ __forceinline__ T shift_up1(const T &v, const T &ident, Mover mv)
{
    return mv.template move<kWaveShr1, 0xf>(ident, v);
}

// Mover for a single scalar register value.
struct ScalarMover {
    template <int CTRL, int ROWS, class T>
    __device__ __forceinline__ T move(T old, T v) const
    {
        return dpp<CTRL, ROWS>(old, v);
    }
};

// Wave-wide sum / max / min of a scalar: the result is uniform across lanes.
template <class T>
__device__ __forceinline__ T reduce_sum(T v)
{
    v = scan_incl(v, T(0), ScalarMover{}, [](T a, T b) { return a + b; });
    return lane_value(v, 63);
}
template <class T>
__device__ __forceinline__ T reduce_max(T v, T lowest)
{
    v = scan_incl(v, lowest, ScalarMover{}, [](T a, T b) { return a > b ? a : b; });
    return lane_value(v, 63);
}
template <class T>
__device__ __forceinline__ T reduce_min(T v, T highest)
{
    v = scan_incl(v, highest, ScalarMover{}, [](T a, T b) { return a < b ? a : b; });
    return lane_value(v, 63);
}

}  // namespace wave
}  // namespace pmc
