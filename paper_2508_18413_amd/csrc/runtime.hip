// Context, targets, errors and small layout kernels of libpmcmc.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>

#include "pmc_internal.hpp"

namespace pmc {

static thread_local char g_err[1024] = "";

// ---------------------------------------------------- allocation-free scratch
// Device memory of pmc_solve_noalloc: one statically sized array per device,
// loaded with the library's code object and held until the process ends.
// Host code never uses the array's name as an address: its per-device
// address comes from hipGetSymbolAddress, taken once per device (with that
// device current) by pmc_create.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};
}  // namespace

pmc_status scratch_init(int device)
{
    PMC_REQUIRE(device >= 0 && device < kMaxDevices, "scratch: device %d out of range", device);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch[device]) return PMC_OK;
    void *ptr = nullptr;
    PMC_TRY_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    PMC_REQUIRE(ptr != nullptr, "scratch: no device address for device %d", device);
    g_scratch[device] = ptr;
    return PMC_OK;
}

void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch[device];
}

void set_error(const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
const char *last_error() { return g_err; }

pmc_status ensure_lb_desc(pmc_context *ctx, size_t bytes)
{
    if (bytes <= ctx->lb_desc_bytes) return PMC_OK;
    if (ctx->no_alloc) {
        set_error("pmc_solve_noalloc: %zu bytes of look-back descriptors exceed the %zu reserved in scratch", bytes,
                  ctx->lb_desc_bytes);
        return PMC_ERR_UNSUPPORTED;
    }
    size_t nb = align_up(bytes + bytes / 4, 1 << 20);
    if (ctx->lb_desc) {
        PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
        PMC_TRY_HIP(hipFree(ctx->lb_desc));
        ctx->lb_desc = nullptr;
        ctx->lb_desc_bytes = 0;
    }
    if (hipMalloc(&ctx->lb_desc, nb) != hipSuccess) {
        ctx->lb_desc = nullptr;
        set_error("out of device memory for %zu bytes of look-back descriptors", nb);
        return PMC_ERR_OOM;
    }
    PMC_TRY_HIP(hipMemsetAsync(ctx->lb_desc, 0, nb, ctx->stream));
    ctx->lb_desc_bytes = nb;
    return PMC_OK;
}

pmc_status ensure_pool(pmc_context *ctx, size_t bytes)
{
    if (bytes <= ctx->pool_bytes) return PMC_OK;
    if (ctx->no_alloc) {
        set_error("pmc_solve_noalloc: a %zu-byte workspace pool would have to be allocated", bytes);
        return PMC_ERR_UNSUPPORTED;
    }
    if (ctx->pool) {
        PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
        PMC_TRY_HIP(hipFree(ctx->pool));
        ctx->pool = nullptr;
        ctx->pool_bytes = 0;
    }
    size_t nb = align_up(bytes, 1 << 20);
    if (hipMalloc(&ctx->pool, nb) != hipSuccess) {
        ctx->pool = nullptr;
        set_error("out of device memory for a %zu-byte workspace", nb);
        return PMC_ERR_OOM;
    }
    ctx->pool_bytes = nb;
    return PMC_OK;
}

// ------------------------------------------------------------ layout kernels
namespace {
template <typename R>
__global__ void k_rows_to_planes(const R *rows, R *planes, int64_t n, int D, int64_t ld)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * D) return;
    const int64_t t = i / D;
    const int d = (int)(i % D);
    planes[(size_t)d * ld + t] = rows[i];
}
template <typename R>
__global__ void k_planes_to_rows(const R *planes, R *rows, int64_t n, int D, int64_t ld)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * D) return;
    const int64_t t = i / D;
    const int d = (int)(i % D);
    rows[i] = planes[(size_t)d * ld + t];
}
// planes[d][t] = s0[chain(t)][d]
template <typename R>
__global__ void k_broadcast_s0(const R *s0, const int64_t *offsets, int n_chains, R *planes,
                               int64_t n, int D, int64_t ld)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    int lo = 0, hi = n_chains - 1;
    while (lo < hi) {  // last chain with offsets[c] <= t
        const int mid = (lo + hi + 1) / 2;
        if (offsets[mid] <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    for (int d = 0; d < D; d++) planes[(size_t)d * ld + t] = s0[(size_t)lo * D + d];
}
// out[d][t] = sum_e M[d][e] in[e][t], M = Q or Q^T (Q row-major D x D, D <= 32)
template <typename R>
__global__ void k_rotate_planes(const R *Q, const R *in, R *out, int64_t n, int D, int64_t ld, int transpose)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    R v[32];
    for (int e = 0; e < D; e++) v[e] = in[(size_t)e * ld + t];
    for (int d = 0; d < D; d++) {
        R acc = R(0);
        for (int e = 0; e < D; e++) acc = fma(transpose ? Q[(size_t)e * D + d] : Q[(size_t)d * D + e], v[e], acc);
        out[(size_t)d * ld + t] = acc;
    }
}
}  // namespace

pmc_status rotate_planes(pmc_context *ctx, pmc_dtype dt, const void *Q, const void *in, void *out, int64_t n,
                         int D, int64_t ld, bool transpose)
{
    if (n == 0) return PMC_OK;
    PMC_REQUIRE(D >= 1 && D <= 32, "rotate_planes: D <= 32 (got %d)", D);
    dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (dt == PMC_F64)
        hipLaunchKernelGGL(k_rotate_planes<double>, g, b, 0, ctx->stream, (const double *)Q, (const double *)in,
                           (double *)out, n, D, ld, transpose ? 1 : 0);
    else
        hipLaunchKernelGGL(k_rotate_planes<float>, g, b, 0, ctx->stream, (const float *)Q, (const float *)in,
                           (float *)out, n, D, ld, transpose ? 1 : 0);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status rows_to_planes(pmc_context *ctx, pmc_dtype dt, const void *rows, void *planes, int64_t n,
                          int D, int64_t ld)
{
    const int64_t tot = n * D;
    if (tot == 0) return PMC_OK;
    dim3 g((unsigned)((tot + 255) / 256)), b(256);
    if (dt == PMC_F64)
        hipLaunchKernelGGL(k_rows_to_planes<double>, g, b, 0, ctx->stream, (const double *)rows,
                           (double *)planes, n, D, ld);
    else
        hipLaunchKernelGGL(k_rows_to_planes<float>, g, b, 0, ctx->stream, (const float *)rows,
                           (float *)planes, n, D, ld);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status planes_to_rows(pmc_context *ctx, pmc_dtype dt, const void *planes, void *rows, int64_t n,
                          int D, int64_t ld)
{
    const int64_t tot = n * D;
    if (tot == 0) return PMC_OK;
    dim3 g((unsigned)((tot + 255) / 256)), b(256);
    if (dt == PMC_F64)
        hipLaunchKernelGGL(k_planes_to_rows<double>, g, b, 0, ctx->stream, (const double *)planes,
                           (double *)rows, n, D, ld);
    else
        hipLaunchKernelGGL(k_planes_to_rows<float>, g, b, 0, ctx->stream, (const float *)planes,
                           (float *)rows, n, D, ld);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

pmc_status broadcast_s0(pmc_context *ctx, pmc_dtype dt, const void *s0, const int64_t *d_offsets,
                        int n_chains, void *planes, int64_t n, int D, int64_t ld)
{
    if (n == 0) return PMC_OK;
    dim3 g((unsigned)((n + 255) / 256)), b(256);
    if (dt == PMC_F64)
        hipLaunchKernelGGL(k_broadcast_s0<double>, g, b, 0, ctx->stream, (const double *)s0,
                           d_offsets, n_chains, (double *)planes, n, D, ld);
    else
        hipLaunchKernelGGL(k_broadcast_s0<float>, g, b, 0, ctx->stream, (const float *)s0,
                           d_offsets, n_chains, (float *)planes, n, D, ld);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

namespace {
// Counts the entries of up to four input arrays that are not finite (and, for
// arrays flagged `unit`, that lie outside the open interval (0, 1)).
struct BadScan {
    const void *p[5];
    int64_t n[5];
    int unit[5];  // 0: finite; 1: in (0, 1); 2: positive and finite
};
template <typename R>
__global__ void __launch_bounds__(256) k_count_bad(BadScan s, uint32_t *out)
{
    uint32_t c = 0;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
#pragma unroll
    for (int k = 0; k < 5; k++) {
        const R *a = (const R *)s.p[k];
        if (!a) continue;
        const int kind = s.unit[k];
        for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < s.n[k]; i += stride) {
            const R v = a[i];
            const bool bad = !isfinite(v) || (kind == 1 && !(v > R(0) && v < R(1))) || (kind == 2 && !(v > R(0)));
            c += bad ? 1u : 0u;
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) c += __shfl_xor(c, m);
    if ((threadIdx.x & 63) == 0 && c) atomicAdd(out, c);
}
}  // namespace

pmc_status check_inputs(pmc_context *ctx, pmc_dtype dt, const InputCheck *in, int n_in)
{
    PMC_REQUIRE(n_in >= 0 && n_in <= 5, "check_inputs: at most 5 arrays");
    BadScan s;
    int64_t most = 0;
    for (int k = 0; k < 5; k++) {
        s.p[k] = k < n_in && in[k].n > 0 ? in[k].p : nullptr;
        s.n[k] = k < n_in ? in[k].n : 0;
        s.unit[k] = k < n_in ? in[k].unit : 0;
        if (s.p[k]) most = std::max(most, s.n[k]);
    }
    if (most == 0) return PMC_OK;
    hipStream_t st = ctx->stream;
    *ctx->h_bad = 0;
    PMC_TRY_HIP(hipMemcpyAsync(ctx->d_bad, ctx->h_bad, sizeof(uint32_t), hipMemcpyHostToDevice, st));
    const unsigned blocks = (unsigned)std::min<int64_t>((most + 255) / 256, 2048);
    if (dt == PMC_F64)
        hipLaunchKernelGGL(k_count_bad<double>, dim3(blocks), dim3(256), 0, st, s, ctx->d_bad);
    else
        hipLaunchKernelGGL(k_count_bad<float>, dim3(blocks), dim3(256), 0, st, s, ctx->d_bad);
    PMC_TRY_HIP(hipGetLastError());
    PMC_TRY_HIP(hipMemcpyAsync(ctx->h_bad, ctx->d_bad, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    PMC_TRY_HIP(hipStreamSynchronize(st));
    if (*ctx->h_bad) {
        set_error("%u input values are not finite (or uniforms outside (0, 1), or inverse masses not positive)",
                  *ctx->h_bad);
        return PMC_ERR_NONFINITE;
    }
    return PMC_OK;
}

bool is_device_ptr(const void *p)
{
    if (!p) return false;
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

}  // namespace pmc

using namespace pmc;

extern "C" {

const char *pmc_last_error(void) { return pmc::last_error(); }
const char *pmc_version(void) { return "libpmcmc 0.1 (gfx950)"; }

pmc_status pmc_create(pmc_context **out, int device, void *hip_stream)
{
    if (!out) {
        set_error("pmc_create: out is NULL");
        return PMC_ERR_INVALID;
    }
    *out = nullptr;
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n == 0) {
        (void)hipGetLastError();
        set_error("pmc_create: no HIP device available (%s)", hipGetErrorString(e));
        return PMC_ERR_HIP;
    }
    if (device < 0 || device >= n) {
        set_error("pmc_create: device %d out of range [0, %d)", device, n);
        return PMC_ERR_INVALID;
    }
    PMC_TRY_HIP(hipSetDevice(device));
    hipDeviceProp_t prop;
    PMC_TRY_HIP(hipGetDeviceProperties(&prop, device));
    pmc_context *ctx = new pmc_context();
    ctx->device = device;
    ctx->stream = (hipStream_t)hip_stream;
    ctx->arch = prop.gcnArchName;
    ctx->n_cu = prop.multiProcessorCount;
    if (hipMalloc((void **)&ctx->sync, sizeof(ScanSync) * kMaxSyncSlots) != hipSuccess ||
        hipMemset(ctx->sync, 0, sizeof(ScanSync) * kMaxSyncSlots) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_status, sizeof(GlobalStatus)) != hipSuccess ||
        hipMalloc((void **)&ctx->d_bad, sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc((void **)&ctx->h_bad, sizeof(uint32_t)) != hipSuccess ||
        hipEventCreate(&ctx->ev0) != hipSuccess || hipEventCreate(&ctx->ev1) != hipSuccess) {
        set_error("pmc_create: device initialisation failed");
        pmc_destroy(ctx);
        return PMC_ERR_HIP;
    }
    // per-device address of the allocation-free entry point's scratch array
    if (scratch_init(device) != PMC_OK) {
        pmc_destroy(ctx);
        return PMC_ERR_HIP;
    }
    // timing-only events: no system-scope fence when they complete (the
    // solver reads them after synchronising the stream)
    for (hipEvent_t &e : ctx->kev) {
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) {
            set_error("pmc_create: event creation failed");
            pmc_destroy(ctx);
            return PMC_ERR_HIP;
        }
    }
    *out = ctx;
    return PMC_OK;
}

pmc_status pmc_destroy(pmc_context *ctx)
{
    if (!ctx) return PMC_OK;
    if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
    (void)hipDeviceSynchronize();
    if (ctx->sync) (void)hipFree(ctx->sync);
    if (ctx->lb_desc) (void)hipFree(ctx->lb_desc);
    if (ctx->pool) (void)hipFree(ctx->pool);
    if (ctx->h_status) (void)hipHostFree(ctx->h_status);
    if (ctx->d_bad) (void)hipFree(ctx->d_bad);
    if (ctx->h_bad) (void)hipHostFree(ctx->h_bad);
    if (ctx->ev0) (void)hipEventDestroy(ctx->ev0);
    if (ctx->ev1) (void)hipEventDestroy(ctx->ev1);
    for (hipEvent_t e : ctx->kev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return PMC_OK;
}

pmc_status pmc_set_stream(pmc_context *ctx, void *hip_stream)
{
    if (!ctx) {
        set_error("pmc_set_stream: ctx is NULL");
        return PMC_ERR_INVALID;
    }
    ctx->stream = (hipStream_t)hip_stream;
    return PMC_OK;
}

pmc_status pmc_target_create(pmc_context *ctx, const pmc_target_desc *d, pmc_target **out)
{
    PMC_REQUIRE(ctx && d && out, "pmc_target_create: NULL argument");
    *out = nullptr;
    PMC_REQUIRE(d->dim >= 1, "pmc_target_create: dim must be >= 1 (got %d)", d->dim);
    PMC_REQUIRE(d->dtype == PMC_F32 || d->dtype == PMC_F64, "pmc_target_create: bad dtype");
    const size_t es = d->dtype == PMC_F64 ? 8 : 4;
    DevTarget t;
    t.kind = d->kind;
    t.dtype = d->dtype;
    t.dim = d->dim;
    t.n_data = 0;
    t.ldx = 0;
    t.prior_var = d->prior_var;
    t.theta = d->theta;
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    switch (d->kind) {
    case PMC_TARGET_BANANA:
        PMC_REQUIRE(d->dim == 2, "banana target has dim 2 (got %d)", d->dim);
        break;
    case PMC_TARGET_FUNNEL:
        PMC_REQUIRE(d->dim >= 2 && d->dim <= 32, "funnel target: 2 <= dim <= 32 (got %d)", d->dim);
        break;
    case PMC_TARGET_GAUSSIAN: {
        PMC_REQUIRE(d->dim <= 1024, "gaussian target: dim <= 1024 (got %d)", d->dim);
        PMC_REQUIRE(is_device_ptr(d->mean) && is_device_ptr(d->prec),
                    "gaussian target: mean and prec must be device pointers");
        PMC_TRY_HIP(hipMalloc(&t.mean, es * d->dim));
        PMC_TRY_HIP(hipMalloc(&t.prec, es * d->dim * d->dim));
        PMC_TRY_HIP(hipMemcpyAsync(t.mean, d->mean, es * d->dim, hipMemcpyDeviceToDevice, ctx->stream));
        PMC_TRY_HIP(hipMemcpyAsync(t.prec, d->prec, es * d->dim * d->dim, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        break;
    }
    case PMC_TARGET_LOGREG: {
        PMC_REQUIRE(d->dtype == PMC_F32, "logreg target runs in F32");
        PMC_REQUIRE(d->n_data >= 1, "logreg target: n_data >= 1");
        PMC_REQUIRE(d->prior_var > 0, "logreg target: prior_var > 0");
        PMC_REQUIRE(is_device_ptr(d->X) && is_device_ptr(d->y),
                    "logreg target: X and y must be device pointers");
        int ldx = 0;
        for (int c : {4, 8, 16, 25, 32})
            if (d->dim <= c) {
                ldx = c;
                break;
            }
        const bool wide = d->dim >= kWideMinDim;
        if (wide) {
            // the matrix-core GEMM path: rows and columns padded to its tile
            if (d->dim > kWideMaxDim) {
                set_error("logreg target: dim <= %d (got %d)", kWideMaxDim, d->dim);
                return PMC_ERR_UNSUPPORTED;
            }
            PMC_REQUIRE(d->products != PMC_PRODUCTS_SPLIT16 && d->products != PMC_PRODUCTS_REFINE,
                        "logreg target: dim > 32 evaluates with FP32 matrix products only");
            PMC_REQUIRE(d->n_data <= (1 << 24), "logreg target: n_data <= 2^24 (got %d)", d->n_data);
            ldx = wide_pad(d->dim);
        }
        PMC_REQUIRE(d->products >= PMC_PRODUCTS_AUTO && d->products <= PMC_PRODUCTS_REFINE,
                    "logreg target: unknown products mode %d", (int)d->products);
        t.ldx = ldx;
        t.n_data = d->n_data;
        t.products = wide ? PMC_PRODUCTS_F32 : d->products;
        const size_t rows = wide ? (size_t)wide_pad(d->n_data) : (size_t)d->n_data;
        PMC_TRY_HIP(hipMalloc(&t.X, 4 * (size_t)ldx * rows));
        PMC_TRY_HIP(hipMalloc(&t.y, 4 * rows));
        PMC_TRY_HIP(hipMemsetAsync(t.X, 0, 4 * (size_t)ldx * rows, ctx->stream));
        PMC_TRY_HIP(hipMemsetAsync(t.y, 0, 4 * rows, ctx->stream));
        PMC_TRY_HIP(hipMemcpy2DAsync(t.X, 4 * ldx, d->X, 4 * d->dim, 4 * d->dim, d->n_data,
                                     hipMemcpyDeviceToDevice, ctx->stream));
        PMC_TRY_HIP(hipMemcpyAsync(t.y, d->y, 4 * (size_t)d->n_data, hipMemcpyDeviceToDevice,
                                   ctx->stream));
        PMC_TRY(logreg_build_frags(ctx, t));
        break;
    }
    default:
        set_error("pmc_target_create: unknown kind %d", (int)d->kind);
        return PMC_ERR_INVALID;
    }
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    pmc_target *o = new pmc_target();
    o->t = t;
    o->device = ctx->device;
    *out = o;
    return PMC_OK;
}

pmc_status pmc_target_destroy(pmc_target *tgt)
{
    if (!tgt) return PMC_OK;
    (void)hipDeviceSynchronize();
    if (tgt->t.mean) (void)hipFree(tgt->t.mean);
    if (tgt->t.prec) (void)hipFree(tgt->t.prec);
    if (tgt->t.X) (void)hipFree(tgt->t.X);
    if (tgt->t.y) (void)hipFree(tgt->t.y);
    for (void *q : {tgt->t.xa, tgt->t.xta, tgt->t.x2ta, tgt->t.ypad, tgt->t.xl, tgt->t.xh, tgt->t.dxa, tgt->t.dpb, tgt->t.dxt,
                    tgt->t.xwt, tgt->t.x2wt})
        if (q) (void)hipFree(q);
    delete tgt;
    return PMC_OK;
}

}  // extern "C"
