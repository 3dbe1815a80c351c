// Newton driver (Algorithm 1, Appendix A.1) and the sequential baseline entry.
//
// Per sweep, for every still-active chain (and, with the sliding window, only
// from its first unconverged step): eval kernel (F_t, J_t at s^{(i)}), scan
// kernel (the linearised recursion, Sec. 2 eq. 2-4, updating s in place and
// emitting convergence partials), status kernel (per-chain Delta test, sweep
// counts, window starts, global status).  The host either reads the status
// after each sweep or replays a captured HIP graph of `graph_sweeps` sweeps
// between reads; kernels of converged chains return immediately, so a replay
// past convergence changes nothing.
#include <math.h>
#include <string.h>

#include <stdio.h>
#include <stdlib.h>

#include <algorithm>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "pmc_internal.hpp"
#include "targets.hpp"

namespace pmc {
namespace {

struct Plan {
    const DevTarget *tg;
    pmc_dtype dt;
    size_t es;
    int D;
    int64_t n;
    int n_chains;
    int64_t ld;
    int64_t Tmax;
    int variant;
    int jmode;
    int n_lanes;
    int scan_items, scan_block, C_scan, C_eval;
    DenseHier dh;  // matrix-core dense scan: per-chain hierarchy and its workspace layout
    std::vector<int64_t> offs;
    std::vector<SegTile> etiles, stiles;
    std::vector<int32_t> ctb;
    size_t o_S, o_F, o_J, o_hier, o_acc, o_gt, o_etiles, o_stiles, o_ctb, o_offs, o_part, o_chains,
        o_global, total;
    int max_iter;
    bool logreg_dense = false;  // dense J of the logistic posterior (pair sums in o_hpair)
    bool logreg_probe = false;  // probed diagonal of the logistic posterior (MALA)
    bool hmc = false;           // f_t is a whole HMC transition (Sec. 3.3)
    bool logreg_surrogate = false;  // MALA relaxed gate on the logistic posterior (diagonal variants)
    const void *basis = nullptr;  // orthogonal reparameterisation (iterates z = Q^T s)
    size_t o_rot = 0;             // rotation scratch planes [D, ld]
    size_t o_hpair = 0;
    bool logreg_wide = false;     // logistic regression with D > 32 (matrix-core GEMM evaluation)
    int wide_ks = 1;              // K slices of its GEMMs (fixed-width windows)
    bool refine = false;          // split-FP16 products until convergence, then FP32 products
    size_t o_wide = 0;
    std::vector<int32_t> ectb;    // each chain's first eval tile (wide, fixed-width windows)
    size_t o_ectb = 0;
};

void build_tiles(const std::vector<int64_t> &offs, int C, std::vector<SegTile> &tiles,
                 std::vector<int32_t> *ctb)
{
    tiles.clear();
    const int nc = (int)offs.size() - 1;
    if (ctb) ctb->assign(nc + 1, 0);
    // tile boundaries at absolute multiples of C: interior tiles start
    // aligned; a chain's first tile runs from its offset to the next multiple
    for (int c = 0; c < nc; c++) {
        if (ctb) (*ctb)[c] = (int32_t)tiles.size();
        for (int64_t s = offs[c]; s < offs[c + 1];) {
            const int64_t e = std::min<int64_t>(offs[c + 1], (s / C + 1) * C);
            tiles.push_back(SegTile{s, (int32_t)(e - s), c});
            s = e;
        }
    }
    if (ctb) (*ctb)[nc] = (int32_t)tiles.size();
}

pmc_status make_plan(pmc_context *ctx, const pmc_problem *p, const pmc_options *o, Plan &pl)
{
    PMC_REQUIRE(ctx && p && o, "pmc_solve: NULL argument");
    PMC_REQUIRE(p->target, "pmc_solve: problem has no target");
    const DevTarget &t = p->target->t;
    pl.tg = &t;
    pl.dt = t.dtype;
    pl.es = t.dtype == PMC_F64 ? 8 : 4;
    pl.D = t.dim;
    PMC_REQUIRE(p->sampler == PMC_SAMPLER_MALA || p->sampler == PMC_SAMPLER_ULA || p->sampler == PMC_SAMPLER_HMC,
                "pmc_solve: sampler must be MALA, ULA or HMC");
    pl.hmc = p->sampler == PMC_SAMPLER_HMC;
    if (pl.hmc) PMC_REQUIRE(p->n_leapfrog >= 1 && p->n_leapfrog <= 1024, "pmc_solve: HMC needs 1 <= n_leapfrog <= 1024");
    PMC_REQUIRE(p->n_chains >= 1, "pmc_solve: n_chains >= 1 (got %d)", p->n_chains);
    PMC_REQUIRE(p->step_size > 0 && isfinite(p->step_size), "pmc_solve: step_size > 0");
    PMC_REQUIRE(o->atol >= 0 && o->rtol >= 0 && (o->atol > 0 || o->rtol > 0),
                "pmc_solve: tolerances must be >= 0 and not both 0");
    pl.n_chains = p->n_chains;
    pl.offs.assign(p->n_chains + 1, 0);
    if (p->offsets) {
        PMC_REQUIRE(p->offsets[0] == 0, "pmc_solve: offsets[0] must be 0");
        for (int c = 0; c < p->n_chains; c++) {
            PMC_REQUIRE(p->offsets[c + 1] >= p->offsets[c], "pmc_solve: offsets must be non-decreasing");
            pl.offs[c + 1] = p->offsets[c + 1];
        }
        PMC_REQUIRE(p->offsets[p->n_chains] == p->n_steps,
                    "pmc_solve: offsets[n_chains] (%lld) != n_steps (%lld)",
                    (long long)p->offsets[p->n_chains], (long long)p->n_steps);
    } else {
        PMC_REQUIRE(p->n_chains == 1, "pmc_solve: offsets required for n_chains > 1");
        pl.offs[1] = p->n_steps;
    }
    PMC_REQUIRE(p->n_steps >= 0, "pmc_solve: n_steps >= 0");
    pl.n = p->n_steps;
    pl.Tmax = 0;
    for (int c = 0; c < p->n_chains; c++) pl.Tmax = std::max(pl.Tmax, pl.offs[c + 1] - pl.offs[c]);
    if (pl.n > 0) {
        PMC_REQUIRE(is_device_ptr(p->s0), "pmc_solve: s0 must be a device pointer");
        PMC_REQUIRE(is_device_ptr(p->noise), "pmc_solve: noise must be a device pointer");
        PMC_REQUIRE(is_device_ptr(p->out_states), "pmc_solve: out_states must be a device pointer");
        if (p->sampler != PMC_SAMPLER_ULA)
            PMC_REQUIRE(is_device_ptr(p->uniforms), "pmc_solve: MALA and HMC need device uniforms");
        if (pl.hmc && p->inv_mass)
            PMC_REQUIRE(is_device_ptr(p->inv_mass), "pmc_solve: inv_mass must be a device pointer");
        if (p->init_guess)
            PMC_REQUIRE(is_device_ptr(p->init_guess), "pmc_solve: init_guess must be a device pointer");
    }
    if (t.kind == PMC_TARGET_GAUSSIAN && pl.D > Gaussian<float, 16>::kMaxLaneDim) {
        set_error("pmc_solve: per-step Gaussian evaluation supports D <= %d (got %d)",
                  Gaussian<float, 16>::kMaxLaneDim, pl.D);
        return PMC_ERR_UNSUPPORTED;
    }
    pl.logreg_wide = t.kind == PMC_TARGET_LOGREG && pl.D >= kWideMinDim;
    // refined products drive the per-step evaluation of MALA / ULA on the
    // logistic posterior; fixed-width windows start with the final products
    pl.refine = t.kind == PMC_TARGET_LOGREG && t.products == PMC_PRODUCTS_REFINE && !pl.logreg_wide &&
                !pl.hmc && o->window_width == 0;
    if (pl.logreg_wide &&
        (pl.hmc || (o->variant != PMC_QDEER_DIAG && o->variant != PMC_PICARD) || o->jac_probes ||
         (o->gate == PMC_GATE_SURROGATE && p->sampler == PMC_SAMPLER_MALA))) {
        set_error("pmc_solve: logistic regression with D > 32 runs MALA or ULA, frozen gate, with quasi-DEER "
                  "(exact diagonal) or Picard");
        return PMC_ERR_UNSUPPORTED;
    }
    pl.variant = o->variant;
    pl.n_lanes = pl.D;
    if (pl.hmc) {
        // HMC transitions (Sec. 3.3): dense J for D <= 4 on the vector scan;
        // the logistic posterior takes the one-probe diagonal (its exact
        // diagonal would need one tangent integration per coordinate)
        if (o->variant == PMC_DEER_DENSE && (t.kind == PMC_TARGET_LOGREG || pl.D > 4)) {
            set_error("pmc_solve: HMC with dense DEER supports per-lane targets with D <= 4");
            return PMC_ERR_UNSUPPORTED;
        }
        if (t.kind == PMC_TARGET_LOGREG && o->variant == PMC_QDEER_DIAG && o->jac_probes != 1) {
            set_error("pmc_solve: HMC on logistic regression takes the one-probe diagonal (jac_probes = 1)");
            return PMC_ERR_UNSUPPORTED;
        }
        if (o->basis) {
            set_error("pmc_solve: basis is not supported with HMC transitions");
            return PMC_ERR_UNSUPPORTED;
        }
    }
    switch (o->variant) {
    case PMC_QDEER_DIAG: pl.jmode = JM_DIAG; break;
    case PMC_PICARD: pl.jmode = JM_NONE; break;
    case PMC_DEER_DENSE:
        pl.n_lanes = 1;
        if (t.kind == PMC_TARGET_LOGREG) {
            // Jacobians from the pair-sum kernels, composed by the matrix-core scan
            if (pl.D > 32) {
                set_error("pmc_solve: dense DEER on logistic regression supports D <= 32 (got %d)", pl.D);
                return PMC_ERR_UNSUPPORTED;
            }
            pl.jmode = o->jac_prec == PMC_JAC_BF16 ? JM_DENSE_BF16 : JM_DENSE_F32;
            pl.logreg_dense = true;
            break;
        }
        if (pl.dt == PMC_F64 || (pl.D <= 4 && o->jac_prec == PMC_JAC_F32) || pl.hmc) {
            if (pl.D > 4) {
                set_error("pmc_solve: FP64 dense DEER supports D <= 4 (got %d)", pl.D);
                return PMC_ERR_UNSUPPORTED;
            }
            pl.jmode = JM_DENSE_ROW;
        } else {
            if (pl.D > 32) {
                set_error("pmc_solve: matrix-core dense DEER supports D <= 32 (got %d)", pl.D);
                return PMC_ERR_UNSUPPORTED;
            }
            pl.jmode = o->jac_prec == PMC_JAC_BF16 ? JM_DENSE_BF16 : JM_DENSE_F32;
        }
        break;
    case PMC_QDEER_BLOCK2:
        set_error("pmc_solve: block quasi-DEER applies to leapfrog integration (pmc_hmc_sample)");
        return PMC_ERR_UNSUPPORTED;
    default:
        set_error("pmc_solve: unknown variant %d", (int)o->variant);
        return PMC_ERR_INVALID;
    }
    PMC_REQUIRE(o->gate == PMC_GATE_FROZEN || o->gate == PMC_GATE_SURROGATE, "pmc_solve: bad gate");
    PMC_REQUIRE(o->damping > 0 && isfinite(o->damping), "pmc_solve: damping must be > 0");
    PMC_REQUIRE(o->tie_band >= 0 && isfinite(o->tie_band), "pmc_solve: tie_band must be >= 0");
    PMC_REQUIRE(o->window_width >= 0, "pmc_solve: window_width must be >= 0");
    PMC_REQUIRE(o->window_width == 0 || o->skip_converged_prefix,
                "pmc_solve: a fixed-width window needs skip_converged_prefix");
    if (t.kind == PMC_TARGET_LOGREG && o->gate == PMC_GATE_SURROGATE && p->sampler == PMC_SAMPLER_MALA) {
        // the relaxed gate's rank-one term is added to the diagonal (exact or probed)
        if (pl.jmode != JM_DIAG && pl.jmode != JM_NONE) {
            set_error("pmc_solve: the relaxed gate on logistic regression takes the diagonal variants");
            return PMC_ERR_UNSUPPORTED;
        }
        pl.logreg_surrogate = pl.jmode == JM_DIAG;
    }
    PMC_REQUIRE(!(o->graph_sweeps > 0 && o->trace_out), "pmc_solve: trace_out needs graph_sweeps = 0");
    PMC_REQUIRE(o->jac_probes == 0 || o->jac_probes == 1, "pmc_solve: jac_probes is 0 or 1");
    if (o->jac_probes) {
        PMC_REQUIRE(o->variant == PMC_QDEER_DIAG, "pmc_solve: jac_probes needs the diagonal variant");
        if (t.kind == PMC_TARGET_LOGREG && !pl.hmc) {
            // J z through the matrix-core kernel of logreg_dense.hip
            if (pl.D > 32) {
                set_error("pmc_solve: probed diagonals on logistic regression support D <= 32 (got %d)", pl.D);
                return PMC_ERR_UNSUPPORTED;
            }
            pl.logreg_probe = true;
        }
    }

    if (o->basis) {
        PMC_REQUIRE(is_device_ptr(o->basis), "pmc_solve: basis must be a device pointer");
        // the logistic posterior is solved as the rotated model (solve_logreg_rotated)
        if (t.kind != PMC_TARGET_LOGREG) {
            if (!(pl.jmode == JM_DIAG || pl.jmode == JM_NONE) || o->jac_probes) {
                set_error("pmc_solve: basis applies to quasi-DEER or Picard without probes");
                return PMC_ERR_UNSUPPORTED;
            }
            pl.basis = o->basis;
        }
    }
    if (pl.jmode == JM_DENSE_BF16 || pl.jmode == JM_DENSE_F32) {
        pl.scan_items = 1;
        pl.scan_block = 256;
        pl.C_scan = dense_mfma_unit();
    } else if (pl.jmode == JM_DENSE_ROW) {
        pl.scan_items = pl.D == 2 ? 4 : 2;
        pl.scan_block = 256;
        pl.C_scan = 256 * pl.scan_items;
    } else {
        // untuned default (FP32): 512 x 8 below 2^23 elements per scan, where
        // launch latency dominates and every configuration takes about the
        // same time; 1024 x 8 above, where its fewer look-back hops per
        // plane are worth 8-13 % (16 planes x 2^22 steps)
        pl.scan_items = ctx->diag_items ? ctx->diag_items : 8;
        const bool big = (int64_t)pl.n_lanes * pl.n >= (int64_t(1) << 23);
        pl.scan_block = ctx->diag_block ? ctx->diag_block : (pl.dt == PMC_F64 ? 256 : big ? 1024 : 512);
        // fixed-width windows of at most 1024 steps over many coordinates:
        // 1024-step tiles, so that a workgroup's tile holds little beyond the
        // window (768 coordinates, 4 chains, 128-step windows: 25 against 50 us)
        if (o->window_width > 0 && o->window_width <= 1024 && pl.n_lanes >= 128 && pl.dt == PMC_F32 &&
            !ctx->diag_block && !ctx->diag_items) {
            pl.scan_items = 4;
            pl.scan_block = 256;
        }
        pl.C_scan = scan_tile_steps(pl.dt, 1, pl.scan_items, pl.scan_block);
    }
    pl.C_eval = eval_tile_steps(t);
    build_tiles(pl.offs, pl.C_scan, pl.stiles, &pl.ctb);
    build_tiles(pl.offs, pl.C_eval, pl.etiles,
                pl.logreg_wide && o->window_width > 0 ? &pl.ectb : nullptr);

    pl.max_iter = o->max_iter;
    if (pl.max_iter <= 0)
        pl.max_iter = (int)std::min<int64_t>(pl.Tmax + 1, 50 + (int64_t)(5e-4 * (double)pl.Tmax));
    if (o->trace_out) {
        const size_t need = (size_t)pl.max_iter * pl.n * pl.D * pl.es;
        PMC_REQUIRE(o->trace_bytes >= need, "pmc_solve: trace_out needs %zu bytes", need);
    }

    pl.ld = (int64_t)align_up((size_t)std::max<int64_t>(pl.n, 1), 64);
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o2 = off;
        off = align_up(off + bytes, 256);
        return o2;
    };
    const size_t plane = (size_t)pl.ld * pl.es;
    pl.o_S = take(plane * pl.D);
    pl.o_F = take(plane * pl.D);
    size_t jb = 0;
    switch (pl.jmode) {
    case JM_DIAG:
    case JM_NONE: jb = plane * pl.D; break;
    case JM_DENSE_ROW: jb = (size_t)pl.n * pl.D * pl.D * pl.es; break;
    case JM_DENSE_BF16: jb = (size_t)pl.n * 2048; break;
    case JM_DENSE_F32: jb = (size_t)pl.n * 4096; break;
    default: jb = 0;
    }
    pl.o_J = take(std::max<size_t>(jb, 256));
    if (pl.jmode == JM_DENSE_BF16 || pl.jmode == JM_DENSE_F32) dense_hier_plan(pl.ctb, pl.n_chains, pl.n, pl.dh);
    pl.o_hier = take(pl.jmode == JM_DENSE_BF16 || pl.jmode == JM_DENSE_F32 ? pl.dh.bytes : 256);
    if (pl.logreg_dense) pl.o_hpair = take(sizeof(float) * (size_t)pl.n * logreg_dense_pair_cols(pl.D));
    if (pl.basis) pl.o_rot = take(plane * pl.D);
    if (pl.logreg_wide) {
        pl.wide_ks = wide_ksplit(t, o->window_width, pl.n_chains);
        pl.o_wide = take(wide_workspace_bytes(t, pl.ld, pl.wide_ks, o->window_width, pl.n_chains));
        if (!pl.ectb.empty()) pl.o_ectb = take(sizeof(int32_t) * pl.ectb.size());
    }
    pl.o_acc = take(std::max<int64_t>(pl.n, 1));
    pl.o_gt = take(4 * std::max<int64_t>(pl.n, 1));
    pl.o_etiles = take(sizeof(SegTile) * std::max<size_t>(pl.etiles.size(), 1));
    pl.o_stiles = take(sizeof(SegTile) * std::max<size_t>(pl.stiles.size(), 1));
    pl.o_ctb = take(sizeof(int32_t) * pl.ctb.size());
    pl.o_offs = take(sizeof(int64_t) * pl.offs.size());
    pl.o_part = take(sizeof(TilePartial) * std::max<size_t>((size_t)pl.n_lanes * pl.stiles.size(), 1));
    pl.o_chains = take(sizeof(ChainStatus) * pl.n_chains);
    pl.o_global = take(sizeof(GlobalStatus));
    pl.total = off;
    return PMC_OK;
}

struct Sweep {
    EvalArgs ea;
    NewtonScanArgs sa;
    StatusArgs st;
    void *hier;  // matrix-core scan hierarchy workspace
    float *hpair = nullptr;  // pair sums of the logistic Hessian (dense DEER)
    void *wide = nullptr;    // workspace of the D > 32 logistic evaluation
};

// One Newton sweep: evaluation, scan, status fold.  ev (optional) receives
// three events: before the evaluation, between evaluation and scan, after the scan.
pmc_status one_sweep(pmc_context *ctx, const Plan &pl, const Sweep &sw, hipEvent_t *ev = nullptr)
{
    if (ev) PMC_TRY_HIP(hipEventRecord(ev[0], ctx->stream));
    if (pl.logreg_surrogate) {
        // the evaluation (and probe) kernels write the frozen-gate diagonal
        // undamped and unclipped; the relaxed gate's term, the damping and the
        // clip follow
        EvalArgs e = sw.ea;
        e.gate = PMC_GATE_FROZEN;
        e.damping = 1.0;
        e.clip = 0.0;
        PMC_TRY(launch_eval(ctx, *pl.tg, e));
        if (pl.logreg_probe) PMC_TRY(launch_logreg_probe_diag(ctx, *pl.tg, e, pl.n, pl.n_chains));
        PMC_TRY(launch_logreg_surrogate(ctx, *pl.tg, sw.ea));
    } else if (pl.logreg_wide) {
        PMC_TRY(launch_eval_logreg_wide(ctx, *pl.tg, sw.ea, sw.wide));
    } else {
        PMC_TRY(launch_eval(ctx, *pl.tg, sw.ea));
        if (pl.logreg_dense)
            PMC_TRY(launch_logreg_dense_jac(ctx, *pl.tg, sw.ea, pl.n, pl.n_chains, sw.hpair,
                                            pl.jmode == JM_DENSE_F32));
        if (pl.logreg_probe) PMC_TRY(launch_logreg_probe_diag(ctx, *pl.tg, sw.ea, pl.n, pl.n_chains));
    }
    if (ev) PMC_TRY_HIP(hipEventRecord(ev[1], ctx->stream));
    if (pl.jmode == JM_DENSE_BF16 || pl.jmode == JM_DENSE_F32)
        PMC_TRY(launch_dense_mfma_newton(ctx, pl.jmode == JM_DENSE_BF16, sw.sa.J, (const float *)sw.sa.F,
                                         (float *)sw.sa.S, sw.sa.ld, pl.D, sw.sa.tiles, sw.sa.chains,
                                         sw.sa.partials, sw.sa.atol, sw.sa.rtol, nullptr, sw.hier, pl.dh,
                                         sw.ea.glob));
    else if (pl.jmode == JM_DENSE_ROW)
        PMC_TRY(launch_newton_scan_dense_small(ctx, pl.dt, pl.D, sw.sa));
    else
        PMC_TRY(launch_newton_scan_diag(ctx, pl.dt, sw.sa, pl.scan_items, pl.scan_block));
    if (ev) PMC_TRY_HIP(hipEventRecord(ev[2], ctx->stream));
    PMC_TRY(launch_status(ctx, sw.st));
    return PMC_OK;
}

// out[r][k] = sum_d in[r][d] M[d][k] with M = Q, or Q^T when transpose (FP32, D <= 32)
__global__ void k_rotate_rows(const float *in, int64_t rows, int ld_in, const float *Q, int D, int transpose,
                              float *out, int ld_out)
{
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= rows) return;
    float v[32];
    for (int d = 0; d < D; d++) v[d] = in[(size_t)r * ld_in + d];
    for (int k = 0; k < D; k++) {
        float acc = 0.f;
        for (int d = 0; d < D; d++) acc = fmaf(v[d], transpose ? Q[(size_t)k * D + d] : Q[(size_t)d * D + k], acc);
        out[(size_t)r * ld_out + k] = acc;
    }
}

pmc_status rotate_rows(pmc_context *ctx, const void *in, int64_t rows, int ld_in, const void *Q, int D,
                       bool transpose, void *out, int ld_out)
{
    if (rows <= 0) return PMC_OK;
    if (D >= kWideMinDim)
        return wide_rotate_rows(ctx, (const float *)in, rows, ld_in, (const float *)Q, D, transpose, (float *)out,
                                ld_out);
    PMC_REQUIRE(D >= 1 && D <= 32 && (rows + 255) / 256 <= 0x7fffffff, "rotate_rows: bad shape");
    hipLaunchKernelGGL(k_rotate_rows, dim3((unsigned)((rows + 255) / 256)), dim3(256), 0, ctx->stream,
                       (const float *)in, rows, ld_in, (const float *)Q, D, transpose ? 1 : 0, (float *)out, ld_out);
    PMC_TRY_HIP(hipGetLastError());
    return PMC_OK;
}

// The logistic posterior in the coordinates z = Q^T s (Sec. 3.4 eq. 11) is the
// same model with design X Q (the prior N(0, prior_var I) is unchanged by a
// rotation) and MALA noise Q^T xi, so quasi-DEER's diag(Q^T J Q) is the
// rotated model's exact Jacobian diagonal.  The rotated target, noise, s0
// and initial guess are formed on the device, the rotated problem is solved
// with every variant the target supports, and the states and trace are
// rotated back.  Allocates the rotated copies for the duration of the call.
pmc_status solve_logreg_rotated(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts, void *workspace,
                                size_t ws_bytes, pmc_result *res)
{
    const DevTarget &t = prob->target->t;
    const int D = t.dim, nc = prob->n_chains;
    const int64_t n = prob->n_steps;
    PMC_REQUIRE(is_device_ptr(opts->basis), "pmc_solve: basis must be a device pointer");
    PMC_REQUIRE(nc >= 1 && n >= 0 && D <= kWideMaxDim, "pmc_solve: bad rotated logistic problem");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    pmc_target rt;
    rt.device = prob->target->device;
    rt.t.kind = t.kind;
    rt.t.dtype = t.dtype;
    rt.t.dim = D;
    rt.t.n_data = t.n_data;
    rt.t.ldx = t.ldx;
    rt.t.prior_var = t.prior_var;
    rt.t.theta = t.theta;
    rt.t.products = t.products;
    rt.t.y = t.y;  // shared, not freed here
    float *xi = nullptr, *s0 = nullptr, *guess = nullptr, *zout = nullptr, *ztrace = nullptr;
    auto release = [&]() {
        (void)hipStreamSynchronize(ctx->stream);
        for (void *q : {(void *)rt.t.X, rt.t.xa, rt.t.xta, rt.t.x2ta, rt.t.ypad, rt.t.xl, rt.t.xh, rt.t.dxa,
                        rt.t.dpb, rt.t.dxt, rt.t.xwt, rt.t.x2wt, (void *)xi, (void *)s0, (void *)guess, (void *)zout,
                        (void *)ztrace})
            if (q) (void)hipFree(q);
    };
    pmc_status st = PMC_OK;
    auto run = [&]() -> pmc_status {
        const size_t xrows = D >= kWideMinDim ? (size_t)wide_pad(t.n_data) : (size_t)t.n_data;
        const size_t xb = 4 * (size_t)t.ldx * xrows, rb = 4 * (size_t)std::max<int64_t>(n, 1) * D;
        PMC_TRY_HIP(hipMalloc(&rt.t.X, xb));
        PMC_TRY_HIP(hipMemsetAsync(rt.t.X, 0, xb, ctx->stream));
        PMC_TRY(rotate_rows(ctx, t.X, t.n_data, t.ldx, opts->basis, D, false, rt.t.X, t.ldx));  // X Q
        PMC_TRY(logreg_build_frags(ctx, rt.t));
        PMC_TRY_HIP(hipMalloc(&xi, rb));
        PMC_TRY_HIP(hipMalloc(&s0, 4 * (size_t)nc * D));
        PMC_TRY_HIP(hipMalloc(&zout, rb));
        PMC_TRY(rotate_rows(ctx, prob->noise, n, D, opts->basis, D, false, xi, D));  // rows (Q^T xi)^T
        PMC_TRY(rotate_rows(ctx, prob->s0, nc, D, opts->basis, D, false, s0, D));
        pmc_problem p2 = *prob;
        pmc_options o2 = *opts;
        o2.basis = nullptr;
        p2.target = &rt;
        p2.noise = xi;
        p2.s0 = s0;
        p2.out_states = zout;
        if (prob->init_guess) {
            PMC_TRY_HIP(hipMalloc(&guess, rb));
            PMC_TRY(rotate_rows(ctx, prob->init_guess, n, D, opts->basis, D, false, guess, D));
            p2.init_guess = guess;
        }
        if (opts->trace_out) {
            // rows of sweeps that do not run come back as the caller left them
            PMC_TRY_HIP(hipMalloc(&ztrace, opts->trace_bytes));
            PMC_TRY_HIP(hipMemcpyAsync(ztrace, opts->trace_out, opts->trace_bytes, hipMemcpyDeviceToDevice,
                                       ctx->stream));
            PMC_TRY(rotate_rows(ctx, opts->trace_out, (int64_t)(opts->trace_bytes / (4 * (size_t)D)), D, opts->basis,
                                D, false, ztrace, D));
            o2.trace_out = ztrace;
        }
        st = pmc_solve(ctx, &p2, &o2, workspace, ws_bytes, res);
        if (st != PMC_OK && st != PMC_NOT_CONVERGED) return st;
        PMC_TRY(rotate_rows(ctx, zout, n, D, opts->basis, D, true, prob->out_states, D));  // s = Q z
        if (opts->trace_out)
            PMC_TRY(rotate_rows(ctx, ztrace, (int64_t)(opts->trace_bytes / (4 * (size_t)D)), D, opts->basis, D, true,
                                opts->trace_out, D));
        return st;
    };
    const pmc_status r = run();
    release();
    return r;
}

}  // namespace
}  // namespace pmc

using namespace pmc;

extern "C" {

pmc_status pmc_default_options(pmc_options *o, pmc_dtype dtype)
{
    PMC_REQUIRE(o, "pmc_default_options: NULL");
    memset(o, 0, sizeof(*o));
    o->variant = PMC_QDEER_DIAG;
    o->jac_prec = PMC_JAC_F32;
    o->gate = PMC_GATE_FROZEN;
    // FP32: 5e-7 keeps the state error of a converged chain within half of a
    // 1e-5 relative bound against an exact sequential run (a change-based
    // stop leaves an error a few times the last change)
    o->atol = o->rtol = dtype == PMC_F64 ? 1e-12 : 5e-7;
    o->max_iter = 0;
    o->damping = 1.0;
    o->clip = 0.0;
    o->skip_converged_prefix = 1;
    o->floor_stall = 16;
    o->tie_band = dtype == PMC_F64 ? 0.0 : 2e-5;
    return PMC_OK;
}

pmc_status pmc_workspace_size(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                              size_t *bytes)
{
    PMC_REQUIRE(bytes, "pmc_workspace_size: bytes is NULL");
    Plan pl;
    PMC_TRY(make_plan(ctx, prob, opts, pl));
    *bytes = pl.total;
    return PMC_OK;
}

}  // extern "C"

namespace pmc {
namespace {
// pmc_solve's body.  scratch_ws: the workspace is the static scratch array
// (its address is not a runtime allocation, so it is not checked as one).
pmc_status solve_impl(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts, void *workspace,
                      size_t ws_bytes, pmc_result *res, bool scratch_ws)
{
    Plan pl;
    PMC_TRY(make_plan(ctx, prob, opts, pl));
    if (opts->basis && prob->target->t.kind == PMC_TARGET_LOGREG)
        return solve_logreg_rotated(ctx, prob, opts, workspace, ws_bytes, res);
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    if (res) {
        int32_t *spc = res->sweeps_per_chain;
        int8_t *cst = res->chain_state;
        memset(res, 0, sizeof(*res));
        res->sweeps_per_chain = spc;
        res->chain_state = cst;
    }
    if (pl.n == 0) {
        if (res) {
            res->n_converged = pl.n_chains;
            if (res->sweeps_per_chain) memset(res->sweeps_per_chain, 0, 4 * pl.n_chains);
            if (res->chain_state) memset(res->chain_state, 0, pl.n_chains);
        }
        return PMC_OK;
    }
    {
        const InputCheck in[5] = {{prob->s0, (int64_t)pl.n_chains * pl.D, 0},
                                  {prob->noise, pl.n * pl.D, 0},
                                  {prob->sampler != PMC_SAMPLER_ULA ? prob->uniforms : nullptr, pl.n, 1},
                                  {prob->init_guess, prob->init_guess ? pl.n * pl.D : 0, 0},
                                  {pl.hmc ? prob->inv_mass : nullptr, pl.D, 2}};
        PMC_TRY(check_inputs(ctx, pl.dt, in, 5));
    }
    char *ws;
    if (workspace) {
        PMC_REQUIRE(ws_bytes >= pl.total, "pmc_solve: workspace of %zu bytes < %zu needed", ws_bytes,
                    pl.total);
        PMC_REQUIRE(scratch_ws || is_device_ptr(workspace), "pmc_solve: workspace must be a device pointer");
        ws = (char *)workspace;
    } else {
        PMC_TRY(ensure_pool(ctx, pl.total));
        ws = (char *)ctx->pool;
    }
    hipStream_t st = ctx->stream;
    void *S = ws + pl.o_S, *F = ws + pl.o_F, *J = ws + pl.o_J;
    uint8_t *acc = prob->out_accept ? prob->out_accept : (uint8_t *)(ws + pl.o_acc);
    float *gt = prob->out_gtilde ? prob->out_gtilde : (float *)(ws + pl.o_gt);
    SegTile *d_et = (SegTile *)(ws + pl.o_etiles), *d_st = (SegTile *)(ws + pl.o_stiles);
    int32_t *d_ctb = (int32_t *)(ws + pl.o_ctb);
    int64_t *d_offs = (int64_t *)(ws + pl.o_offs);
    TilePartial *d_part = (TilePartial *)(ws + pl.o_part);
    ChainStatus *d_chains = (ChainStatus *)(ws + pl.o_chains);
    GlobalStatus *d_glob = (GlobalStatus *)(ws + pl.o_global);

    std::vector<ChainStatus> hc(pl.n_chains);
    for (int c = 0; c < pl.n_chains; c++) {
        ChainStatus &cs = hc[c];
        memset(&cs, 0, sizeof(cs));
        cs.win_start = pl.offs[c];
        cs.win_end = opts->window_width > 0 ? std::min<int64_t>(pl.offs[c + 1], pl.offs[c] + opts->window_width)
                                            : pl.offs[c + 1];
        cs.first_bad = INT64_MAX;
        const bool nonempty = pl.offs[c + 1] > pl.offs[c];
        cs.active = nonempty;
        cs.converged = !nonempty;
        cs.best_ratio = INFINITY;
        cs.best_front = pl.offs[c];
        cs.fb_prev = pl.offs[c];
        cs.fine = !pl.refine;
    }
    PMC_TRY_HIP(hipMemcpyAsync(d_et, pl.etiles.data(), sizeof(SegTile) * pl.etiles.size(),
                               hipMemcpyHostToDevice, st));
    PMC_TRY_HIP(hipMemcpyAsync(d_st, pl.stiles.data(), sizeof(SegTile) * pl.stiles.size(),
                               hipMemcpyHostToDevice, st));
    PMC_TRY_HIP(hipMemcpyAsync(d_ctb, pl.ctb.data(), sizeof(int32_t) * pl.ctb.size(),
                               hipMemcpyHostToDevice, st));
    PMC_TRY_HIP(hipMemcpyAsync(d_offs, pl.offs.data(), sizeof(int64_t) * pl.offs.size(),
                               hipMemcpyHostToDevice, st));
    PMC_TRY_HIP(hipMemcpyAsync(d_chains, hc.data(), sizeof(ChainStatus) * hc.size(),
                               hipMemcpyHostToDevice, st));
    {
        // the first sweep evaluates every step of every non-empty chain
        GlobalStatus *g0 = ctx->h_status;
        memset(g0, 0, sizeof(*g0));
        for (int c = 0; c < pl.n_chains; c++) {
            g0->n_active += hc[c].active;
            g0->n_fine += hc[c].active && hc[c].fine;
            g0->n_converged += hc[c].converged;
        }
        g0->next_steps = 0;
        for (int c = 0; c < pl.n_chains; c++) g0->next_steps += hc[c].win_end - hc[c].win_start;
        PMC_TRY_HIP(hipMemcpyAsync(d_glob, g0, sizeof(GlobalStatus), hipMemcpyHostToDevice, st));
    }
    if (pl.jmode == JM_NONE)  // Picard: J = 0 through the diagonal scan
        PMC_TRY_HIP(hipMemsetAsync(J, 0, (size_t)pl.ld * pl.es * pl.D, st));

    PMC_TRY_HIP(hipEventRecord(ctx->ev0, st));
    if (prob->init_guess)
        PMC_TRY(rows_to_planes(ctx, pl.dt, prob->init_guess, S, pl.n, pl.D, pl.ld));
    else
        PMC_TRY(broadcast_s0(ctx, pl.dt, prob->s0, d_offs, pl.n_chains, S, pl.n, pl.D, pl.ld));
    void *rot = pl.basis ? ws + pl.o_rot : nullptr;
    if (pl.basis) {
        // the iteration runs on z = Q^T s
        PMC_TRY(rotate_planes(ctx, pl.dt, pl.basis, S, rot, pl.n, pl.D, pl.ld, true));
        PMC_TRY_HIP(hipMemcpyAsync(S, rot, (size_t)pl.ld * pl.es * pl.D, hipMemcpyDeviceToDevice, st));
    }

    Sweep sw;
    sw.hier = ws + pl.o_hier;
    if (pl.jmode == JM_DENSE_BF16 || pl.jmode == JM_DENSE_F32) PMC_TRY(dense_hier_setup(ctx, pl.dh, sw.hier));
    if (pl.logreg_wide) {
        // the noise as planes, once per solve
        sw.wide = ws + pl.o_wide;
        PMC_TRY(wide_rows_to_planes(ctx, (const float *)prob->noise, pl.n, pl.D, pl.ld,
                                    wide_xi_planes(sw.wide, *pl.tg, pl.ld, pl.wide_ks, opts->window_width,
                                                   pl.n_chains)));
    }
    if (pl.logreg_dense || pl.logreg_probe) {
        // operand tables: derived data of the target, built by its first
        // dense or probed solve
        PMC_TRY(logreg_dense_tables(ctx, const_cast<DevTarget &>(*pl.tg)));
        if (pl.logreg_dense) sw.hpair = (float *)(ws + pl.o_hpair);
    }
    EvalArgs &ea = sw.ea;
    ea.tiles = d_et;
    ea.n_tiles = (int)pl.etiles.size();
    ea.offsets = d_offs;
    ea.chains = d_chains;
    ea.D = pl.D;
    ea.ld = pl.ld;
    ea.s0 = prob->s0;
    ea.S = S;
    ea.noise = prob->noise;
    ea.unif = prob->uniforms;
    ea.F = F;
    ea.J = J;
    ea.accept = acc;
    ea.gtilde = gt;
    ea.eps = prob->step_size;
    ea.ula = prob->sampler == PMC_SAMPLER_ULA;
    ea.hmc_L = pl.hmc ? prob->n_leapfrog : 0;
    ea.inv_mass = pl.hmc ? prob->inv_mass : nullptr;
    ea.gate = opts->gate;
    ea.damping = opts->damping;
    ea.clip = opts->clip;
    ea.clip_inf = opts->clip_inf_norm;
    ea.jmode = pl.jmode == JM_NONE ? JM_NONE : pl.jmode;
    ea.probes = opts->jac_probes;
    ea.basis = pl.basis;
    ea.probe_seed = opts->probe_seed;
    ea.tie_band = (float)opts->tie_band;
    ea.tg = pl.tg;
    ea.glob = d_glob;
    ea.ksplit = pl.wide_ks;
    if (!pl.ectb.empty()) {
        int32_t *d_ectb = (int32_t *)(ws + pl.o_ectb);
        PMC_TRY_HIP(hipMemcpyAsync(d_ectb, pl.ectb.data(), sizeof(int32_t) * pl.ectb.size(), hipMemcpyHostToDevice,
                                   st));
        ea.chain_etile_begin = d_ectb;
        ea.window_width = opts->window_width;
        ea.n_chains = pl.n_chains;
    }
    NewtonScanArgs &sa = sw.sa;
    sa.n_lanes = pl.n_lanes;
    sa.ld = pl.ld;
    sa.tiles = d_st;
    sa.n_tiles = (int)pl.stiles.size();
    sa.offsets = d_offs;
    sa.chains = d_chains;
    sa.chain_tile_begin = d_ctb;
    sa.J = J;
    sa.F = F;
    sa.S = S;
    sa.partials = d_part;
    sa.atol = opts->atol;
    sa.rtol = opts->rtol;
    sa.eps = prob->step_size;
    sa.trace = nullptr;
    sa.n_chains = pl.n_chains;
    sa.n_steps = pl.n;
    sa.fixed_window = opts->window_width > 0;
    // the look-back scans leave the epoch advance to the status fold that follows
    sa.defer_epoch = pl.jmode == JM_DIAG || pl.jmode == JM_NONE || pl.jmode == JM_DENSE_ROW;
    StatusArgs &sta = sw.st;
    sta.n_chains = pl.n_chains;
    sta.n_lanes = pl.n_lanes;
    sta.tiles = d_st;
    sta.n_tiles = (int)pl.stiles.size();
    sta.chain_tile_begin = d_ctb;
    sta.partials = d_part;
    sta.chains = d_chains;
    sta.global = d_glob;
    sta.accept = nullptr;
    sta.offsets = d_offs;
    sta.max_iter = pl.max_iter;
    sta.skip_prefix = opts->skip_converged_prefix;
    sta.floor_stall = opts->floor_stall;
    sta.window_width = opts->window_width;
    sta.n_steps = pl.n;
    sta.bump_epoch = sa.defer_epoch ? ctx->sync : nullptr;

    GlobalStatus *hs = ctx->h_status;
    int sweeps_done = 0;
    float prof_eval_ms = 0, prof_scan_ms = 0;
    PMC_REQUIRE(!(opts->profile_kernels && opts->graph_sweeps > 0),
                "pmc_solve: profile_kernels needs graph_sweeps = 0");
    if (opts->graph_sweeps > 0) {
        const int m = opts->graph_sweeps;
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
        PMC_TRY_HIP(hipStreamSynchronize(st));
        hipStream_t cap = st;
        bool own_stream = false;
        if (!cap) {  // the legacy default stream cannot be captured
            PMC_TRY_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
            own_stream = true;
        }
        // descriptors and pool must not grow inside the capture
        PMC_TRY(ensure_lb_desc(ctx, (size_t)48 * 8 * pl.n_lanes * pl.stiles.size()));
        hipStream_t saved = ctx->stream;
        ctx->stream = cap;
        pmc_status rc = PMC_OK;
        hipError_t he = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
        if (he == hipSuccess) {
            for (int i = 0; i < m && rc == PMC_OK; i++) rc = one_sweep(ctx, pl, sw);
            if (rc == PMC_OK)
                he = hipMemcpyAsync(hs, d_glob, sizeof(GlobalStatus), hipMemcpyDeviceToHost, cap);
            hipError_t he2 = hipStreamEndCapture(cap, &graph);
            if (he == hipSuccess) he = he2;
        }
        if (rc == PMC_OK && he == hipSuccess) he = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        for (; rc == PMC_OK && he == hipSuccess && sweeps_done < pl.max_iter;) {
            he = hipGraphLaunch(exec, cap);
            if (he == hipSuccess) he = hipStreamSynchronize(cap);
            sweeps_done = hs->sweeps;
            if (hs->n_active == 0) break;
        }
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        ctx->stream = saved;
        if (own_stream) (void)hipStreamDestroy(cap);
        if (rc != PMC_OK) return rc;
        PMC_TRY_HIP(he);
    } else {
        // Sweeps are enqueued in batches between reads of the global status;
        // sweeps past the last active chain return at once.  A trace keeps one
        // sweep per batch so that its rows after convergence stay untouched.
        const bool prof = opts->profile_kernels != 0;
        const int batch = opts->trace_out ? 1 : kSweepBatch;
        for (int it = 0; it < pl.max_iter;) {
            const int nb = std::min(batch, pl.max_iter - it);
            for (int j = 0; j < nb; j++) {
                PMC_TRY(one_sweep(ctx, pl, sw, prof ? &ctx->kev[3 * j] : nullptr));
                if (opts->trace_out) {
                    const void *src = S;
                    if (pl.basis) {
                        PMC_TRY(rotate_planes(ctx, pl.dt, pl.basis, S, rot, pl.n, pl.D, pl.ld, false));
                        src = rot;
                    }
                    PMC_TRY(planes_to_rows(ctx, pl.dt, src,
                                           (char *)opts->trace_out + (size_t)(it + j) * pl.n * pl.D * pl.es,
                                           pl.n, pl.D, pl.ld));
                }
            }
            PMC_TRY_HIP(hipMemcpyAsync(hs, d_glob, sizeof(GlobalStatus), hipMemcpyDeviceToHost, st));
            PMC_TRY_HIP(hipStreamSynchronize(st));
            if (prof) {
                // only sweeps in which some chain was still active
                for (int j = 0; j < nb && it + j < hs->sweeps; j++) {
                    float me = 0, msc = 0;
                    PMC_TRY_HIP(hipEventElapsedTime(&me, ctx->kev[3 * j], ctx->kev[3 * j + 1]));
                    PMC_TRY_HIP(hipEventElapsedTime(&msc, ctx->kev[3 * j + 1], ctx->kev[3 * j + 2]));
                    prof_eval_ms += me;
                    prof_scan_ms += msc;
                }
            }
            it += nb;
            sweeps_done = hs->sweeps;
            if (hs->n_active == 0) break;
        }
    }
    if (pl.basis) {
        PMC_TRY(rotate_planes(ctx, pl.dt, pl.basis, S, rot, pl.n, pl.D, pl.ld, false));  // s = Q z
        PMC_TRY(planes_to_rows(ctx, pl.dt, rot, prob->out_states, pl.n, pl.D, pl.ld));
    } else {
        PMC_TRY(planes_to_rows(ctx, pl.dt, S, prob->out_states, pl.n, pl.D, pl.ld));
    }
    PMC_TRY_HIP(hipEventRecord(ctx->ev1, st));
    // final accept count
    sta.accept = acc;
    sta.fold_only = 1;  // the totals and the accept count only: no chain is updated again
    PMC_TRY(launch_status(ctx, sta));
    PMC_TRY_HIP(hipMemcpyAsync(hs, d_glob, sizeof(GlobalStatus), hipMemcpyDeviceToHost, st));
    PMC_TRY_HIP(hipMemcpyAsync(hc.data(), d_chains, sizeof(ChainStatus) * hc.size(),
                               hipMemcpyDeviceToHost, st));
    PMC_TRY_HIP(hipStreamSynchronize(st));
    PMC_TRY(check_scan_health(ctx));
    float ms = 0;
    PMC_TRY_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (res) {
        res->n_converged = hs->n_converged;
        res->sweeps_total = hs->sweeps;
        res->n_accept = prob->sampler == PMC_SAMPLER_ULA ? pl.n : hs->n_accept;
        res->resid_inf = hs->resid_inf;
        res->resid_l2 = sqrt(hs->resid_sq);
        res->max_ratio = hs->max_ratio;
        res->nonfinite = hs->nonfinite;
        res->elapsed_ms = ms;
        res->eval_ms = prof_eval_ms;
        res->scan_ms = prof_scan_ms;
        res->eval_steps = opts->profile_kernels ? hs->eval_steps : 0;
        if (res->sweeps_per_chain)
            for (int c = 0; c < pl.n_chains; c++) res->sweeps_per_chain[c] = hc[c].sweeps;
        if (res->chain_state)
            for (int c = 0; c < pl.n_chains; c++)
                res->chain_state[c] = (int8_t)(hc[c].converged ? 0 : hc[c].at_floor ? 1 : 2);
    }
    if (res) res->n_floor = hs->n_floor;
    // a chain stopped at its rounding floor has not met the tolerance: its
    // outputs are valid but the call reports the soft status
    if (hs->n_converged < pl.n_chains) {
        set_error("pmc_solve: %d of %d chains not converged after %d sweeps (%d stopped at their rounding "
                  "floor; max ratio %g)",
                  pl.n_chains - hs->n_converged, pl.n_chains, hs->sweeps, hs->n_floor, (double)hs->max_ratio);
        return PMC_NOT_CONVERGED;
    }
    return PMC_OK;
}

__global__ void k_zero_words(uint64_t *p, size_t n)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}
}  // namespace
}  // namespace pmc

extern "C" {

pmc_status pmc_solve(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                     void *workspace, size_t ws_bytes, pmc_result *res)
{
    return solve_impl(ctx, prob, opts, workspace, ws_bytes, res, false);
}

// The workspace and the look-back descriptors of the scans come from the
// per-device static scratch array: look-back descriptors first (cleared by a
// fill kernel at every call), then the solve's workspace.  Rejects what would
// allocate: graph capture, the rotated logistic model, and the logistic
// posterior's dense or probed Jacobians before their operand tables exist.
pmc_status pmc_solve_noalloc(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                             pmc_result *res)
{
    Plan pl;
    PMC_TRY(make_plan(ctx, prob, opts, pl));
    const DevTarget &t = *pl.tg;
    if (opts->graph_sweeps > 0) {
        set_error("pmc_solve_noalloc: graph_sweeps must be 0 (graph instantiation allocates)");
        return PMC_ERR_UNSUPPORTED;
    }
    if (opts->basis && t.kind == PMC_TARGET_LOGREG) {
        set_error("pmc_solve_noalloc: the rotated logistic model allocates its rotated copies");
        return PMC_ERR_UNSUPPORTED;
    }
    if ((pl.logreg_dense || pl.logreg_probe) && !t.dxa) {
        set_error("pmc_solve_noalloc: this target's dense/probe operand tables are not built yet "
                  "(one pmc_solve with this variant builds them)");
        return PMC_ERR_UNSUPPORTED;
    }
    char *base = (char *)scratch_ptr(ctx->device);
    if (!base) {
        set_error("pmc_solve_noalloc: no scratch address for device %d", ctx->device);
        return PMC_ERR_HIP;
    }
    // one descriptor of at most 48 words per lane and scan tile (every scan of the solve fits)
    const size_t desc = align_up((size_t)48 * 8 * pl.n_lanes * std::max<size_t>(pl.stiles.size(), 1), 256);
    if (desc + pl.total > kScratchBytes) {
        set_error("pmc_solve_noalloc: problem needs %zu bytes of scratch, more than its %zu", desc + pl.total,
                  kScratchBytes);
        return PMC_ERR_INVALID;
    }
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    hipLaunchKernelGGL(k_zero_words, dim3((unsigned)std::min<size_t>((desc / 8 + 255) / 256, 1024)), dim3(256), 0,
                       ctx->stream, (uint64_t *)base, desc / 8);
    PMC_TRY_HIP(hipGetLastError());
    void *saved = ctx->lb_desc;
    const size_t saved_bytes = ctx->lb_desc_bytes;
    ctx->lb_desc = base;
    ctx->lb_desc_bytes = desc;
    ctx->no_alloc = true;
    const pmc_status st = solve_impl(ctx, prob, opts, base + desc, pl.total, res, true);
    ctx->no_alloc = false;
    ctx->lb_desc = saved;
    ctx->lb_desc_bytes = saved_bytes;
    return st;
}

pmc_status pmc_sample_sequential(pmc_context *ctx, const pmc_problem *p, pmc_result *res)
{
    PMC_REQUIRE(ctx && p && p->target, "pmc_sample_sequential: NULL argument");
    const DevTarget &t = p->target->t;
    PMC_REQUIRE(p->sampler == PMC_SAMPLER_MALA || p->sampler == PMC_SAMPLER_ULA || p->sampler == PMC_SAMPLER_HMC,
                "pmc_sample_sequential: sampler must be MALA, ULA or HMC");
    const bool hmc = p->sampler == PMC_SAMPLER_HMC;
    if (hmc)
        PMC_REQUIRE(p->n_leapfrog >= 1 && p->n_leapfrog <= 1024,
                    "pmc_sample_sequential: HMC needs 1 <= n_leapfrog <= 1024");
    PMC_REQUIRE(p->n_chains >= 1, "pmc_sample_sequential: n_chains >= 1");
    std::vector<int64_t> offs(p->n_chains + 1, 0);
    if (p->offsets) {
        PMC_REQUIRE(p->offsets[0] == 0, "pmc_sample_sequential: offsets[0] must be 0");
        for (int c = 0; c < p->n_chains; c++) {
            PMC_REQUIRE(p->offsets[c + 1] >= p->offsets[c], "offsets must be non-decreasing");
            offs[c + 1] = p->offsets[c + 1];
        }
        PMC_REQUIRE(offs[p->n_chains] == p->n_steps, "offsets[n_chains] != n_steps");
    } else {
        PMC_REQUIRE(p->n_chains == 1, "pmc_sample_sequential: offsets required for n_chains > 1");
        offs[1] = p->n_steps;
    }
    if (res) {
        int32_t *spc = res->sweeps_per_chain;
        int8_t *cst = res->chain_state;
        memset(res, 0, sizeof(*res));
        res->sweeps_per_chain = spc;
        res->chain_state = cst;
    }
    if (p->n_steps == 0) return PMC_OK;
    PMC_REQUIRE(is_device_ptr(p->s0) && is_device_ptr(p->noise) && is_device_ptr(p->out_states),
                "pmc_sample_sequential: s0, noise and out_states must be device pointers");
    if (p->sampler != PMC_SAMPLER_ULA)
        PMC_REQUIRE(is_device_ptr(p->uniforms), "pmc_sample_sequential: MALA and HMC need device uniforms");
    if (hmc && p->inv_mass)
        PMC_REQUIRE(is_device_ptr(p->inv_mass), "pmc_sample_sequential: inv_mass must be a device pointer");
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    {
        const InputCheck in[4] = {{p->s0, (int64_t)p->n_chains * t.dim, 0},
                                  {p->noise, p->n_steps * t.dim, 0},
                                  {p->sampler != PMC_SAMPLER_ULA ? p->uniforms : nullptr, p->n_steps, 1},
                                  {hmc ? p->inv_mass : nullptr, t.dim, 2}};
        PMC_TRY(check_inputs(ctx, t.dtype, in, 4));
    }
    const size_t offs_bytes = align_up(sizeof(int64_t) * offs.size(), 256);
    PMC_TRY(ensure_pool(ctx, offs_bytes + (hmc ? 0 : seq_scratch_bytes(t, p->n_chains))));
    int64_t *d_offs = (int64_t *)ctx->pool;
    hipStream_t st = ctx->stream;
    PMC_TRY_HIP(hipMemcpyAsync(d_offs, offs.data(), sizeof(int64_t) * offs.size(),
                               hipMemcpyHostToDevice, st));
    SeqArgs a;
    a.n_chains = p->n_chains;
    a.offsets = d_offs;
    a.D = t.dim;
    a.s0 = p->s0;
    a.noise = p->noise;
    a.unif = p->sampler != PMC_SAMPLER_ULA ? p->uniforms : nullptr;
    a.out = p->out_states;
    a.accept = p->out_accept;
    a.gtilde = p->out_gtilde;
    a.eps = p->step_size;
    a.ula = p->sampler == PMC_SAMPLER_ULA;
    a.hmc_L = hmc ? p->n_leapfrog : 0;
    a.inv_mass = hmc ? p->inv_mass : nullptr;
    a.scratch = (char *)ctx->pool + offs_bytes;
    a.host_offsets = offs.data();
    PMC_TRY_HIP(hipEventRecord(ctx->ev0, st));
    if (hmc)
        PMC_TRY(launch_sequential_hmc(ctx, t, a));
    else
        PMC_TRY(launch_sequential(ctx, t, a));
    PMC_TRY_HIP(hipEventRecord(ctx->ev1, st));
    PMC_TRY_HIP(hipStreamSynchronize(st));
    float ms = 0;
    PMC_TRY_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
    if (res) {
        res->elapsed_ms = ms;
        res->n_converged = p->n_chains;
    }
    return PMC_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ tuning
// Times the diagonal-scan tile configurations (items per thread x block) on
// this problem's shape and keeps the fastest in the context.  Cache file:
// one JSON object, one entry per line, keyed "<gcnArchName>|<shape key>".
namespace {
struct Cand {
    int items, block;
};

std::string tune_key(pmc_context *ctx, const Plan &pl)
{
    int ln = 0, lc = 0;
    while ((int64_t(1) << (ln + 1)) <= pl.n) ln++;
    while ((1 << (lc + 1)) <= pl.n_chains) lc++;
    char buf[256];
    snprintf(buf, sizeof(buf), "%s|diag-%s-d%d-n2^%d-c2^%d", ctx->arch.c_str(),
             pl.dt == PMC_F64 ? "f64" : "f32", pl.D, ln, lc);
    return buf;
}

bool cache_lookup(const char *path, const std::string &key, Cand &c)
{
    std::ifstream f(path);
    std::string line;
    const std::string q = "\"" + key + "\"";
    while (std::getline(f, line)) {
        const size_t p = line.find(q);
        if (p == std::string::npos) continue;
        int it = 0, bl = 0;
        const size_t a = line.find("\"items\":", p), b = line.find("\"block\":", p);
        if (a == std::string::npos || b == std::string::npos) continue;
        if (sscanf(line.c_str() + a + 8, "%d", &it) == 1 && sscanf(line.c_str() + b + 8, "%d", &bl) == 1) {
            c = Cand{it, bl};
            return true;
        }
    }
    return false;
}

void cache_store(const char *path, const std::string &key, const Cand &c, float ms)
{
    std::vector<std::string> lines;
    {
        std::ifstream f(path);
        std::string line;
        while (std::getline(f, line))
            if (line.find("\"items\"") != std::string::npos && line.find("\"" + key + "\"") == std::string::npos)
                lines.push_back(line);
    }
    char buf[512];
    snprintf(buf, sizeof(buf), "  \"%s\": {\"items\": %d, \"block\": %d, \"ms\": %.5f}", key.c_str(),
             c.items, c.block, ms);
    lines.push_back(buf);
    std::ofstream o(path);
    o << "{\n";
    for (size_t i = 0; i < lines.size(); i++) {
        std::string l = lines[i];
        while (!l.empty() && (l.back() == ',' || l.back() == ' ')) l.pop_back();
        o << l << (i + 1 < lines.size() ? ",\n" : "\n");
    }
    o << "}\n";
}
}  // namespace

extern "C" pmc_status pmc_autotune(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                                   const char *cache_path)
{
    Plan base;
    PMC_TRY(make_plan(ctx, prob, opts, base));
    if (base.jmode != JM_DIAG && base.jmode != JM_NONE) return PMC_OK;  // only the diagonal scan is tuned
    if (base.n == 0) return PMC_OK;
    const std::string key = tune_key(ctx, base);
    Cand best{0, 0};
    if (cache_path && cache_lookup(cache_path, key, best)) {
        ctx->diag_items = best.items;
        ctx->diag_block = best.block;
        return PMC_OK;
    }
    std::vector<Cand> cands;
    if (base.dt == PMC_F64)
        cands = {{4, 256}, {8, 256}};
    else
        cands = {{4, 256}, {8, 256}, {16, 256}, {8, 512}, {16, 512}, {8, 1024}, {16, 1024}};
    PMC_TRY_HIP(hipSetDevice(ctx->device));
    // workspace: planes J, F, S (zero), per-tile partials for the smallest tile, tiles, chains
    const size_t plane = (size_t)base.ld * base.es * base.D;
    int minC = 1 << 30;
    for (auto &c : cands) minC = std::min(minC, scan_tile_steps(base.dt, 1, c.items, c.block));
    std::vector<SegTile> tiles;
    std::vector<int32_t> ctb;
    build_tiles(base.offs, minC, tiles, &ctb);
    size_t off = 0;
    auto take = [&](size_t b) {
        size_t o = off;
        off = align_up(off + b, 256);
        return o;
    };
    const size_t oJ = take(plane), oF = take(plane), oS = take(plane),
                 oP = take(sizeof(TilePartial) * base.D * tiles.size()), oT = take(sizeof(SegTile) * tiles.size()),
                 oC = take(sizeof(int32_t) * ctb.size()), oO = take(sizeof(int64_t) * base.offs.size()),
                 oCh = take(sizeof(ChainStatus) * base.n_chains);
    PMC_TRY(ensure_pool(ctx, off));
    char *ws = (char *)ctx->pool;
    hipStream_t st = ctx->stream;
    PMC_TRY_HIP(hipMemsetAsync(ws, 0, 3 * plane, st));
    std::vector<ChainStatus> hc(base.n_chains);
    for (int c = 0; c < base.n_chains; c++) {
        memset(&hc[c], 0, sizeof(ChainStatus));
        hc[c].win_start = base.offs[c];
        hc[c].win_end = base.offs[c + 1];
        hc[c].active = base.offs[c + 1] > base.offs[c];
    }
    PMC_TRY_HIP(hipMemcpyAsync(ws + oCh, hc.data(), sizeof(ChainStatus) * hc.size(), hipMemcpyHostToDevice, st));
    PMC_TRY_HIP(hipMemcpyAsync(ws + oO, base.offs.data(), sizeof(int64_t) * base.offs.size(),
                               hipMemcpyHostToDevice, st));
    float best_ms = 1e30f;
    for (auto &c : cands) {
        const int C = scan_tile_steps(base.dt, 1, c.items, c.block);
        build_tiles(base.offs, C, tiles, &ctb);
        PMC_TRY_HIP(hipMemcpyAsync(ws + oT, tiles.data(), sizeof(SegTile) * tiles.size(), hipMemcpyHostToDevice, st));
        PMC_TRY_HIP(hipMemcpyAsync(ws + oC, ctb.data(), sizeof(int32_t) * ctb.size(), hipMemcpyHostToDevice, st));
        NewtonScanArgs sa;
        memset(&sa, 0, sizeof(sa));
        sa.n_lanes = base.D;
        sa.ld = base.ld;
        sa.tiles = (const SegTile *)(ws + oT);
        sa.n_tiles = (int)tiles.size();
        sa.offsets = (const int64_t *)(ws + oO);
        sa.chains = (const ChainStatus *)(ws + oCh);
        sa.chain_tile_begin = (const int32_t *)(ws + oC);
        sa.J = ws + oJ;
        sa.F = ws + oF;
        sa.S = ws + oS;
        sa.partials = (TilePartial *)(ws + oP);
        sa.atol = sa.rtol = 1e-6;
        PMC_TRY(launch_newton_scan_diag(ctx, base.dt, sa, c.items, c.block));  // warm-up
        PMC_TRY_HIP(hipEventRecord(ctx->ev0, st));
        for (int r = 0; r < 5; r++) PMC_TRY(launch_newton_scan_diag(ctx, base.dt, sa, c.items, c.block));
        PMC_TRY_HIP(hipEventRecord(ctx->ev1, st));
        PMC_TRY_HIP(hipEventSynchronize(ctx->ev1));
        float ms = 0;
        PMC_TRY_HIP(hipEventElapsedTime(&ms, ctx->ev0, ctx->ev1));
        ms /= 5;
        if (getenv("PMC_AUTOTUNE_VERBOSE"))
            fprintf(stderr, "pmc_autotune %s: items %d block %d: %.4f ms\n", key.c_str(), c.items, c.block, ms);
        if (ms < best_ms) {
            best_ms = ms;
            best = c;
        }
    }
    PMC_TRY(check_scan_health(ctx));
    ctx->diag_items = best.items;
    ctx->diag_block = best.block;
    if (cache_path) cache_store(cache_path, key, best, best_ms);
    return PMC_OK;
}
