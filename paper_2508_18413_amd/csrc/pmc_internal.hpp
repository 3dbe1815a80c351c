// Internal declarations of libpmcmc (HIP, gfx950).  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "pmcmc.h"

namespace pmc {

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);
const char *last_error();

#define PMC_TRY_HIP(call)                                                                  \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess) {                                                            \
            pmc::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                           __LINE__);                                                      \
            return PMC_ERR_HIP;                                                            \
        }                                                                                  \
    } while (0)

#define PMC_TRY(call)                       \
    do {                                    \
        pmc_status s_ = (call);             \
        if (s_ != PMC_OK) return s_;        \
    } while (0)

#define PMC_REQUIRE(cond, ...)              \
    do {                                    \
        if (!(cond)) {                      \
            pmc::set_error(__VA_ARGS__);    \
            return PMC_ERR_INVALID;         \
        }                                   \
    } while (0)

// ------------------------------------------------------------ tiling
// A contiguous run of one chain's steps handled by one workgroup.
struct SegTile {
    int64_t start;  // global step index of the first step
    int32_t len;    // number of steps (>= 1)
    int32_t chain;  // owning chain
};

// Per-tile convergence partials, written by every scan tile (neutral when the
// tile does no work) and folded per chain by the status kernel.
// A step counts as unsettled (it starts the next sweep's sliding window) when
// its last change exceeds this fraction of the tolerance.
constexpr float kFreezeRatio = 1.0f;

struct TilePartial {
    float max_ratio;     // max |delta| / (atol + rtol |s_new|)
    uint32_t nonfinite;  // count of non-finite new iterate elements
    int64_t first_bad;   // smallest global step index with ratio > kFreezeRatio (INT64_MAX if none)
    double resid_sq;     // sum of squared residuals b_t = f_t(s_{t-1}) - s_t, FP64
    double resid_inf;    // max |b_t|
};

// Per-chain Newton state, device resident.
struct ChainStatus {
    int64_t win_start;   // first step of the active window (sliding window)
    int64_t first_bad;   // first step of the last sweep not yet settled (ratio > kFreezeRatio)
    double resid_sq;
    double resid_inf;
    float max_ratio;
    int32_t sweeps;      // sweeps run on this chain
    int32_t active;      // 1 while the chain iterates
    int32_t converged;   // 1 once the tolerance is met
    int32_t stall;       // sweeps without progress (floor guard)
    float best_ratio;
    uint32_t nonfinite;
    int32_t at_floor;    // 1 if stopped at the rounding floor
    int32_t fine;        // 1 once the evaluation uses the final arithmetic (refined products:
                         // 0 while the split-FP16 products drive the iteration)
    int64_t best_front;  // furthest converged front seen
    int64_t fb_prev;     // first_bad of the sweep before (the window starts at the earlier of
                         // the two: a step is frozen once it met the tolerance twice in a row)
    int64_t win_end;     // end (exclusive) of the active window: the chain's end, or
                         // win_start + window_width for a fixed-width window
};

// Whole-problem status, read by the host after each sweep or graph replay.
struct GlobalStatus {
    int32_t n_active;
    int32_t n_converged;
    int32_t sweeps;      // sweeps executed
    int32_t n_floor;     // chains stopped at the rounding floor
    double resid_sq;
    double resid_inf;
    float max_ratio;
    uint32_t nonfinite;
    int64_t n_accept;
    int64_t next_steps;  // steps the next sweep evaluates (active chains, from their windows)
    int64_t eval_steps;  // steps evaluated by all sweeps so far
    uint32_t fold_ctr;   // status-fold completion counter; zero between launches
    int32_t n_fine;      // active chains with fine = 1
};

// Synchronisation words of the single-pass scans.  A one-thread kernel after
// each scan advances the epoch that tags every look-back descriptor, so
// descriptors never need clearing and captured graphs can replay the scan.
// pad is raised when a look-back gives up.
struct ScanSync {
    uint32_t spare0;
    uint32_t spare1;
    uint32_t epoch;
    uint32_t pad;
};
// Slots of pmc_context::sync: 0 = single-pass scans (the others are spare).
constexpr int kScanSyncSlot = 0;
constexpr int kMaxSyncSlots = 4;

// Sweeps a solve enqueues between two reads of the global status.  Sweeps
// queued after the last chain has stopped find n_active == 0 and return at
// once (each costs a few microseconds of launches).
constexpr int kSweepBatch = 8;


// ------------------------------------------------------------ targets
struct DevTarget {
    pmc_target_kind kind;
    pmc_dtype dtype;
    int dim;
    int n_data;
    int ldx;           // padded row stride of X (logreg)
    double prior_var;
    double theta;
    void *mean = nullptr;  // [D]
    void *prec = nullptr;  // [D*D]
    void *X = nullptr;     // [n_data * ldx], zero padded
    void *y = nullptr;     // [n_data]
    // logreg matrix-core fragments (per 32-row tile)
    int nr = 0, mk = 0;
    void *xa = nullptr, *xta = nullptr, *x2ta = nullptr, *ypad = nullptr;
    void *xl = nullptr;    // LDS image of X and y (small data sets)
    void *xh = nullptr;    // split-FP16 LDS image of X, with y and X^T y
    int products = 0;      // pmc_products
    // full-DEER operand tables (built on the first dense solve): X and the
    // pair products x_d x_e in BF16 matrix-core order
    void *dxa = nullptr, *dpb = nullptr, *dxt = nullptr;
    int dnb = 0, dnpt = 0, dgrp = 0;
    // logistic regression with D > 32: X is [Np][ldx] (both padded to 128,
    // zero filled, y zero past n_data), with X^T and (X o X)^T [ldx][Np]
    void *xwt = nullptr, *x2wt = nullptr;
};

}  // namespace pmc

struct pmc_target {
    pmc::DevTarget t;
    int device;
};

struct pmc_context {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string arch;
    int n_cu = 0;
    // persistent device state
    pmc::ScanSync *sync = nullptr;   // [kMaxSyncSlots]
    void *lb_desc = nullptr;         // look-back descriptors
    size_t lb_desc_bytes = 0;
    void *pool = nullptr;            // workspace pool
    size_t pool_bytes = 0;
    bool no_alloc = false;           // inside pmc_solve_noalloc: growing lb_desc or pool is an error
    pmc::GlobalStatus *h_status = nullptr;  // pinned host mirror
    uint32_t *d_bad = nullptr;       // count of invalid input values (device word)
    uint32_t *h_bad = nullptr;       // its pinned host mirror
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    hipEvent_t kev[3 * pmc::kSweepBatch] = {};  // per-kernel timing of one batch of sweeps
    // tuning: items per thread of the diagonal scan (0 = default)
    int diag_items = 0;
    int diag_block = 0;
    // kernel timing of the standalone recursions (events kev[0], kev[1])
    int scan_timing = 0;
    float last_scan_ms = 0.f;
};

namespace pmc {

// bytes helper
inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Allocation-free entry point: size of the per-device static scratch array,
// its one-time address lookup (pmc_create, with the device current) and the
// address for a device (nullptr before scratch_init on that device).
constexpr size_t kScratchBytes = size_t(64) << 20;
pmc_status scratch_init(int device);
void *scratch_ptr(int device);

// Layout helpers: row-major [n, D] <-> dimension-major planes [D, ld].
pmc_status rows_to_planes(pmc_context *ctx, pmc_dtype dt, const void *rows, void *planes, int64_t n,
                          int D, int64_t ld);
// out planes = Q in (or Q^T in when transpose), Q row-major [D, D], D <= 32
pmc_status rotate_planes(pmc_context *ctx, pmc_dtype dt, const void *Q, const void *in, void *out, int64_t n,
                         int D, int64_t ld, bool transpose);
pmc_status planes_to_rows(pmc_context *ctx, pmc_dtype dt, const void *planes, void *rows, int64_t n,
                          int D, int64_t ld);
// planes[d][t] = s0[chain(t)][d] (d_offsets: device [n_chains+1])
pmc_status broadcast_s0(pmc_context *ctx, pmc_dtype dt, const void *s0, const int64_t *d_offsets,
                        int n_chains, void *planes, int64_t n, int D, int64_t ld);
bool is_device_ptr(const void *p);

// One input array for check_inputs: n elements of the call's dtype; unit = 1
// also requires every value to lie in (0, 1) (the accept uniforms), unit = 2
// to be positive (inverse masses).
struct InputCheck {
    const void *p;
    int64_t n;
    int unit;
};
// PMC_ERR_NONFINITE if any listed array holds a non-finite value (or a
// uniform outside (0, 1)); synchronises the context's stream.
pmc_status check_inputs(pmc_context *ctx, pmc_dtype dt, const InputCheck *in, int n_in);  // n_in <= 5

// Ensures ctx->lb_desc holds at least `bytes` (zero filled on growth).
pmc_status ensure_lb_desc(pmc_context *ctx, size_t bytes);
pmc_status ensure_pool(pmc_context *ctx, size_t bytes);

// ------------------------------------------------------ scan launchers
// Newton-update scans over dimension-major planes of length ld (stride between
// planes).  For every active tile: b_t = F_t - S_t; delta_t = J_t delta_{t-1} + b_t
// (delta = 0 before a chain's or window's first step); S_t <- F_t + J_t delta_{t-1};
// partials[lane * n_tiles + tile] receives the convergence partials.
struct NewtonScanArgs {
    int n_lanes;            // planes (D for diag, D for block2 with x/v pairs)
    int64_t ld;             // plane stride
    const SegTile *tiles;   // [n_tiles]
    int n_tiles;
    const int64_t *offsets; // [n_chains+1] device
    const ChainStatus *chains;
    const int32_t *chain_tile_begin;  // [n_chains+1] first scan tile of each chain
    const void *J;          // diag: [n_lanes, ld]; block2 (leapfrog): h [n_lanes, ld]
    const void *F;          // [n_lanes, ld] (block2: [2*n_lanes, ld], x planes then v planes)
    void *S;                // [n_lanes, ld] in/out (block2: [2*n_lanes, ld])
    TilePartial *partials;  // [n_lanes * n_tiles]
    double atol, rtol;
    double eps;             // leapfrog step (block2)
    void *trace;            // optional copy of S after the update, or nullptr
    int defer_epoch;        // 1: the status fold that follows advances the scan epoch
    int n_chains;           // chains in the tile map (0: unknown)
    int64_t n_steps;        // steps over all chains
    int fixed_window = 0;   // 1: windows of fixed width (the one-chain chunked form is not used)
};

// Steps per scan tile for a configuration (the host builds its tile map with it).
int scan_tile_steps(pmc_dtype dt, int variant_m, int items, int block);
pmc_status launch_newton_scan_diag(pmc_context *ctx, pmc_dtype dt, const NewtonScanArgs &a,
                                   int items, int block);
pmc_status launch_linrec_diag(pmc_context *ctx, pmc_dtype dt, int n_lanes, int64_t T, const void *a,
                              const void *b, void *out);
pmc_status launch_linrec_block2(pmc_context *ctx, int n_lanes, int64_t T, const void *coef,
                                const void *rhs, void *out);
pmc_status launch_linrec_dense_small(pmc_context *ctx, int D, int64_t T, const double *A,
                                     const double *b, double *out);

// Dense Newton scan (small D, VALU, F64 or F32): J as [ld, D, D] row-major per step.
pmc_status launch_newton_scan_dense_small(pmc_context *ctx, pmc_dtype dt, int D,
                                          const NewtonScanArgs &a);

// ------------------------------------------------------ evaluation
// Jacobian output formats of the eval kernels.
enum JacMode {
    JM_DIAG = 0,       // diag(J_t) in planes [D, ld]
    JM_DENSE_ROW = 1,  // J_t row-major [n_steps, D, D] in the state dtype (VALU dense scan)
    JM_DENSE_BF16 = 2, // J_t padded to 32x32, bf16, matrix-core A-operand order, 2 KB per step
    JM_DENSE_F32 = 3,  // J_t padded to 32x32, f32, matrix-core A-operand order, 4 KB per step
    JM_NONE = 4        // Picard: J_t = 0, nothing written
};

struct EvalArgs {
    const SegTile *tiles;     // eval tile map (tile length <= block size)
    int n_tiles;
    const int64_t *offsets;   // [n_chains+1]
    const ChainStatus *chains;
    int D;
    int64_t ld;               // plane stride of S and F (and diag J)
    const void *s0;           // [n_chains, D]
    const void *S;            // [D, ld] current iterate
    const void *noise;        // [n_steps, D]
    const void *unif;         // [n_steps]
    void *F;                  // [D, ld] f_t(s_{t-1})
    void *J;                  // per JacMode
    uint8_t *accept;          // [n_steps]
    float *gtilde;            // [n_steps]
    double eps;
    int ula;
    int gate;                 // pmc_gate
    double damping;
    double clip;
    int clip_inf;
    int jmode;
    const pmc::DevTarget *tg; // host copy of the target description (fields passed by value)
    const GlobalStatus *glob = nullptr;  // n_active == 0 at launch: nothing left to evaluate
    int probes = 0;           // 1: probed diagonal z o (J z) instead of diag(J) (JM_DIAG)
    const void *basis = nullptr;  // [D, D] orthogonal Q: iterates are z = Q^T s (per-lane targets)
    uint64_t probe_seed = 0;
    float tie_band = 0.f;         // |g~| below this (from a chain's second sweep on): keep the
                                  // previous sweep's decision, read from accept[t]
    int hmc_L = 0;                // > 0: f_t is a whole HMC step with this many leapfrog steps
    const void *inv_mass = nullptr;  // HMC: [D] diagonal of M^-1, or nullptr = identity
    int ksplit = 1;               // logistic D > 32: K slices of the GEMMs (wide_ksplit)
    int fine_sel = -1;            // evaluate only chains with ChainStatus::fine == fine_sel (-1: all)
    // fixed-width windows (logistic D > 32): the width, the chain count and
    // each chain's first eval tile [n_chains + 1]
    int64_t window_width = 0;
    int n_chains = 0;
    const int32_t *chain_etile_begin = nullptr;
};

// Whether an evaluation launch has chains to take (from the global status
// the last status fold wrote), and whether it takes chain cs.
__device__ __forceinline__ bool eval_has_chains(const EvalArgs &a)
{
    const int n = a.glob->n_active, nf = a.glob->n_fine;
    return a.fine_sel < 0 ? n > 0 : a.fine_sel ? nf > 0 : n > nf;
}
__device__ __forceinline__ bool eval_takes(const EvalArgs &a, const ChainStatus &cs)
{
    return a.fine_sel < 0 || cs.fine == a.fine_sel;
}
pmc_status launch_eval(pmc_context *ctx, const DevTarget &tg, const EvalArgs &a);

// A decision whose gate lies within the tie band keeps the previous sweep's
// value (stored in accept[t]) once the chain has run a sweep.
__device__ __forceinline__ int sticky_decision(const EvalArgs &a, const ChainStatus &cs, int64_t t, double gate,
                                               int acc)
{
    if (a.tie_band > 0.f && cs.sweeps >= 1 && fabs(gate) < (double)a.tie_band && a.accept) return a.accept[t];
    return acc;
}

// SplitMix64 (Steele, Lea & Flood 2014): the output function applied to
// x + 0x9E3779B97F4A7C15, modulo 2^64.  The probe sign of coordinate d at
// global step t in a chain's sweep i is the top bit of
// m(m(m(seed) ^ i) ^ (1024 t + d)) (1: -1, 0: +1).
__device__ __forceinline__ uint64_t probe_mix(uint64_t x)
{
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
pmc_status launch_eval_logreg(pmc_context *ctx, const DevTarget &t, const EvalArgs &a);
pmc_status logreg_build_frags(pmc_context *ctx, DevTarget &t);
// Logistic regression with 32 < D <= 1024 (logreg_wide.hip): the MALA
// evaluation as five FP32 matrix-core GEMMs over the steps of the active
// windows, with fused epilogues.  Workspace per solve (wide_workspace_bytes)
// holds the predictor and residual planes, the gradient and increment
// planes, the noise in planes (filled once per solve by wide_rows_to_planes
// at wide_xi_planes) and the per-step row-tile sums.
constexpr int kWideMinDim = 33, kWideMaxDim = 1024;
int wide_pad(int n);          // rows and columns padded to the GEMM tile (128)
int wide_tile_steps();        // evaluation tile (steps)
size_t wide_workspace_bytes(const DevTarget &t, int64_t ld, int ksplit, int64_t window_width, int n_chains);
// K slices of the wide GEMMs for fixed-width windows of this width (1: none)
int wide_ksplit(const DevTarget &t, int64_t window_width, int n_chains);
float *wide_xi_planes(void *ws, const DevTarget &t, int64_t ld, int ksplit, int64_t window_width, int n_chains);
pmc_status logreg_wide_tables(pmc_context *ctx, DevTarget &t);
pmc_status wide_rotate_rows(pmc_context *ctx, const float *in, int64_t rows, int64_t ld_in, const float *Q, int D,
                            bool transpose, float *out, int64_t ld_out);
pmc_status wide_rows_to_planes(pmc_context *ctx, const float *in, int64_t n, int D, int64_t ld, float *out);
pmc_status launch_eval_logreg_wide(pmc_context *ctx, const DevTarget &t, const EvalArgs &a, void *ws);
// Full-DEER Jacobians on the logistic posterior: operand tables (once per
// target), then per sweep the pair sums H [n, 32 dnpt] and the dense J image
// (BF16 or FP32) from the evaluation's accept decisions.
pmc_status logreg_dense_tables(pmc_context *ctx, DevTarget &t);
int logreg_dense_pair_cols(int D);  // row stride of H (D <= 32)
// One-probe diagonal z o (J z) on the logistic posterior (Sec. 3.4 eq. 10):
// J z through X^T (w o X z) on BF16 matrix cores; writes the diagonal planes.
pmc_status launch_logreg_probe_diag(pmc_context *ctx, const DevTarget &t, const EvalArgs &a, int64_t n,
                                    int n_chains);
pmc_status launch_logreg_dense_jac(pmc_context *ctx, const DevTarget &t, const EvalArgs &a, int64_t n,
                                   int n_chains, float *H, bool f32);
// Tile length the eval kernel for this target expects.
int eval_tile_steps(const DevTarget &tg);

// Same-GPU sequential sampler: one workgroup (or lane) per chain, T-step loop
// on the device.  Writes out_states [n_steps, D], accept, gtilde.
struct SeqArgs {
    int n_chains;
    const int64_t *offsets;
    int D;
    const void *s0, *noise, *unif;
    void *out;
    uint8_t *accept;
    float *gtilde;
    double eps;
    int ula;
    int hmc_L = 0;                   // > 0: HMC transitions with this many leapfrog steps
    const void *inv_mass = nullptr;  // HMC: [D] diagonal of M^-1, or nullptr
    void *scratch = nullptr;         // device scratch of seq_scratch_bytes bytes
    const int64_t *host_offsets = nullptr;  // [n_chains + 1], host copy of offsets
};
pmc_status launch_sequential(pmc_context *ctx, const DevTarget &tg, const SeqArgs &a);
// Device scratch the sequential sampler needs for this target (the D > 32
// logistic sampler's grid-barrier words and partial sums), else 0.
size_t seq_scratch_bytes(const DevTarget &tg, int n_chains);
// The same-GPU sequential MALA sampler for logistic regression with D > 32:
// one cooperative launch per group of up to four chains (logreg_wide.hip).
pmc_status launch_sequential_logreg_wide(pmc_context *ctx, const DevTarget &t, const SeqArgs &a);
// HMC transitions as chain steps (Sec. 3.3): evaluation (per-lane targets and
// the logistic posterior) and the same-GPU sequential sampler.
pmc_status launch_eval_hmc(pmc_context *ctx, const DevTarget &t, const EvalArgs &a);
// The relaxed MALA gate's rank-one diagonal term on the logistic posterior
// (Sec. 3.2), added to the undamped diagonal the evaluation wrote, followed
// by the damping and the clip.
pmc_status launch_logreg_surrogate(pmc_context *ctx, const DevTarget &t, const EvalArgs &a);
pmc_status launch_sequential_hmc(pmc_context *ctx, const DevTarget &t, const SeqArgs &a);

// Dense DEER scan on matrix cores (D <= 32, F32 states; J in the BF16 or F32
// fragment layout written by the eval kernels).
//
// Every chain has a hierarchy of its own: level 0 holds one affine map per
// scan tile of the chain (at most 32 steps), each level above composes
// groups of 8 maps of the level below, up to a top level of at most 8 maps.
constexpr int kDenseMaxLev = 11;  // 2^31 steps: 2^26 tiles, then / 8 per level
struct DenseChainGeom {
    int32_t L;                    // levels (0: empty chain; 1: its <= 8 tile maps are the top)
    int32_t pad;
    int64_t tile0;                // first scan tile of the chain (index of its level-0 maps)
    int64_t m[kDenseMaxLev];      // maps per level (m[0]: the chain's tiles)
    int64_t ubase[kDenseMaxLev];  // k >= 1: index of the level's first map among all upper-level maps
};
struct DenseHier {
    int n_chains = 0;
    int L_max = 0;
    int64_t n_tiles = 0, n_up = 0;
    int64_t single_len = 0;            // one chain: its steps (its tiles are then every 32 steps)
    std::vector<DenseChainGeom> geom;  // per chain
    // several chains: (chain, group) pairs of each level's up and down launch
    std::vector<int32_t> units;
    int64_t up_off[kDenseMaxLev] = {}, up_cnt[kDenseMaxLev] = {};
    int64_t down_off[kDenseMaxLev] = {}, down_cnt[kDenseMaxLev] = {};
    size_t o_P0 = 0, o_B0 = 0, o_C0 = 0, o_UP = 0, o_UB = 0, o_UC = 0, o_geom = 0, o_units = 0,
           bytes = 0;                  // workspace layout
};
// Hierarchy of the chains whose scan tiles are [ctb[c], ctb[c + 1]) (n_steps
// steps in all, cut into tiles at multiples of 32).
void dense_hier_plan(const std::vector<int32_t> &ctb, int n_chains, int64_t n_steps, DenseHier &h);
// Copies the chain tables into the workspace (once per solve, before the
// first sweep).
pmc_status dense_hier_setup(pmc_context *ctx, const DenseHier &h, void *ws);
// Workspace of the hierarchy of one sequence of n steps.
size_t dense_mfma_ws_bytes(int64_t n);
int dense_mfma_unit();
// One Newton update of every active chain: the scan tiles are the level-0
// units; chains[c].active == 0 leaves chain c untouched; glob->n_active == 0
// at launch makes the whole call a no-op.
pmc_status launch_dense_mfma_newton(pmc_context *ctx, int bf16, const void *J, const float *F,
                                    float *S, int64_t ld, int D, const SegTile *tiles,
                                    const ChainStatus *chains, TilePartial *partials, double atol,
                                    double rtol, float *trace, void *ws, const DenseHier &h,
                                    const GlobalStatus *glob);
pmc_status launch_linrec_dense_mfma(pmc_context *ctx, int bf16, int D, int64_t T, const float *A,
                                    const float *b, float *out);
// Same on J already in the fragment layout; ws: dense_mfma_ws_bytes(T) bytes.
pmc_status launch_linrec_dense_mfma_packed(pmc_context *ctx, int bf16, int D, int64_t T,
                                           const void *Jf, const float *b, float *out, void *ws);

// Chain status fold (one launch per sweep).
struct StatusArgs {
    int n_chains;
    int n_lanes;
    const SegTile *tiles;
    int n_tiles;
    const int32_t *chain_tile_begin;  // [n_chains+1] scan-tile ranges per chain
    const TilePartial *partials;
    ChainStatus *chains;
    GlobalStatus *global;
    const uint8_t *accept;            // [n_steps] or nullptr
    const int64_t *offsets;
    int max_iter;
    int skip_prefix;
    int floor_stall;                  // > 0: stop a chain whose ratio has not improved for this
                                      // many sweeps while within twice the tolerance
    int64_t window_width;             // > 0: fixed-width sliding window (steps per chain and sweep)
    int64_t n_steps;
    ScanSync *bump_epoch;             // non-null: the last workgroup advances this scan epoch
    int fold_only = 0;                // 1: re-fold the totals without updating any chain (after the last sweep)
};
pmc_status launch_status(pmc_context *ctx, const StatusArgs &a);
// PMC_ERR_HIP if any scan's look-back gave up since the context was created.
pmc_status check_scan_health(pmc_context *ctx);

}  // namespace pmc
