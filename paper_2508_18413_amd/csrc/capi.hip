// C entry points for the standalone linear recursions and the tuning table.
#include <string.h>

#include "pmc_internal.hpp"

using namespace pmc;

extern "C" {

pmc_status pmc_linrec_diag(pmc_context *ctx, pmc_dtype dtype, int n_lanes, int64_t T, const void *a,
                           const void *b, void *out)
{
    PMC_REQUIRE(ctx, "pmc_linrec_diag: ctx is NULL");
    PMC_REQUIRE(dtype == PMC_F32 || dtype == PMC_F64, "pmc_linrec_diag: bad dtype");
    PMC_REQUIRE(n_lanes >= 0 && T >= 0, "pmc_linrec_diag: negative size");
    if (n_lanes == 0 || T == 0) return PMC_OK;
    PMC_REQUIRE(is_device_ptr(a) && is_device_ptr(b) && is_device_ptr(out),
                "pmc_linrec_diag: a, b, out must be device pointers");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    PMC_TRY(launch_linrec_diag(ctx, dtype, n_lanes, T, a, b, out));
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->scan_timing) PMC_TRY_HIP(hipEventElapsedTime(&ctx->last_scan_ms, ctx->kev[0], ctx->kev[1]));
    return check_scan_health(ctx);
}

pmc_status pmc_linrec_block2(pmc_context *ctx, int n_lanes, int64_t T, const void *coef,
                             const void *rhs, void *out)
{
    PMC_REQUIRE(ctx, "pmc_linrec_block2: ctx is NULL");
    PMC_REQUIRE(n_lanes >= 0 && T >= 0, "pmc_linrec_block2: negative size");
    if (n_lanes == 0 || T == 0) return PMC_OK;
    PMC_REQUIRE(is_device_ptr(coef) && is_device_ptr(rhs) && is_device_ptr(out),
                "pmc_linrec_block2: coef, rhs, out must be device pointers");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    PMC_TRY(launch_linrec_block2(ctx, n_lanes, T, coef, rhs, out));
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    if (ctx->scan_timing) PMC_TRY_HIP(hipEventElapsedTime(&ctx->last_scan_ms, ctx->kev[0], ctx->kev[1]));
    return check_scan_health(ctx);
}

pmc_status pmc_linrec_dense(pmc_context *ctx, pmc_dtype dtype, pmc_jac_prec jac_prec, int D,
                            int64_t T, const void *A, const void *b, void *out)
{
    PMC_REQUIRE(ctx, "pmc_linrec_dense: ctx is NULL");
    PMC_REQUIRE(D >= 1 && T >= 0, "pmc_linrec_dense: D >= 1, T >= 0");
    if (T == 0) return PMC_OK;
    PMC_REQUIRE(is_device_ptr(A) && is_device_ptr(b) && is_device_ptr(out),
                "pmc_linrec_dense: A, b, out must be device pointers");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    if (dtype == PMC_F64) {
        PMC_TRY(launch_linrec_dense_small(ctx, D, T, (const double *)A, (const double *)b, (double *)out));
    } else if (dtype == PMC_F32) {
        if (D > 32) {
            set_error("pmc_linrec_dense: F32 matrix-core path supports D <= 32 (got %d)", D);
            return PMC_ERR_UNSUPPORTED;
        }
        PMC_TRY(launch_linrec_dense_mfma(ctx, jac_prec == PMC_JAC_BF16, D, T, (const float *)A,
                                         (const float *)b, (float *)out));
    } else {
        set_error("pmc_linrec_dense: bad dtype");
        return PMC_ERR_INVALID;
    }
    PMC_TRY_HIP(hipStreamSynchronize(ctx->stream));
    return check_scan_health(ctx);
}

pmc_status pmc_set_scan_timing(pmc_context *ctx, int on)
{
    PMC_REQUIRE(ctx, "pmc_set_scan_timing: ctx is NULL");
    ctx->scan_timing = on != 0;
    ctx->last_scan_ms = 0.f;
    return PMC_OK;
}

pmc_status pmc_last_scan_ms(pmc_context *ctx, float *ms)
{
    PMC_REQUIRE(ctx && ms, "pmc_last_scan_ms: ctx and ms must be non-NULL");
    *ms = ctx->last_scan_ms;
    return PMC_OK;
}

}  // extern "C"
