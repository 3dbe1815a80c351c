/*
 * pmcmc.h -- C ABI of libpmcmc: parallel-in-sequence MCMC on AMD Instinct MI355X (gfx950).
 *
 * The library evaluates an MCMC chain s_t = f_t(s_{t-1}), t = 1..T, from s_0 as
 * the solution of the fixed-point problem r(s_{1:T}) = 0 (Sec. 2 eq. 1) by the
 * parallel Newton iteration of Sec. 2 eq. 2-3 (DEER), its diagonal quasi-Newton
 * form eq. 4 (quasi-DEER), the block quasi-Newton form for leapfrog
 * integration (Sec. 3.3, Appendix A.3), or Picard iteration (J = 0), looping as
 * Algorithm 1 (Appendix A.1) does until successive iterates agree.  f_t is a
 * built-in sampler transition (MALA or ULA, Sec. 3.2; leapfrog, Sec. 3.3) on a
 * built-in target, chosen by enum: arbitrary device code cannot cross a C ABI.
 *
 * Conventions (all entry points):
 *  - Pointers documented DEVICE point to device memory owned by the caller;
 *    pointers documented HOST point to host memory owned by the caller.  The
 *    library never frees caller memory.  Arrays are C-contiguous, row-major.
 *  - All GPU work is enqueued on the context's stream.  Every entry point
 *    returns only after its outputs (device and host) are complete.
 *  - Each call returns a pmc_status and, on failure, sets a thread-local
 *    message readable with pmc_last_error().  PMC_NOT_CONVERGED is a soft
 *    status: all outputs are written and valid (the last Newton iterate).
 *    pmc_solve returns PMC_OK only when every chain met the tolerance; a
 *    chain stopped early at its rounding floor (floor_stall) counts as not
 *    converged (pmc_result.n_floor counts such chains).
 *  - Floating-point types: PMC_F32 arrays are float, PMC_F64 arrays double.
 *  - Calls on one context are not thread-safe; use one context per thread.
 */
#ifndef PMCMC_H
#define PMCMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    PMC_OK = 0,
    PMC_ERR_INVALID = 1,     /* bad argument (null pointer, size, enum, layout)      */
    PMC_ERR_UNSUPPORTED = 2, /* valid request that the library does not implement   */
    PMC_ERR_OOM = 3,         /* device allocation failed or workspace too small      */
    PMC_ERR_HIP = 4,         /* HIP runtime error (no device, launch failure, ...)   */
    PMC_NOT_CONVERGED = 5,   /* soft: some chain did not meet the tolerance; outputs
                                hold the last iterate                                 */
    PMC_ERR_NONFINITE = 6    /* a non-finite value in an input array (initial states,
                                noise, momenta, initial guess) or a uniform outside
                                (0, 1); checked on the device before any sweep        */
} pmc_status;

typedef enum { PMC_F32 = 0, PMC_F64 = 1 } pmc_dtype;

/* Transition f_t.  MALA: the MALA function of Sec. 3.2 with noise xi_t and
 * uniform u_t; ULA: the same proposal, always kept.  HMC: one whole HMC step
 * (Sec. 3.3, parallel HMC across the sequence): momentum v0 = xi_t / sqrt(m)
 * for the diagonal mass matrix diag(m) (identity by default), a half step,
 * n_leapfrog sequential leapfrog steps of size step_size, the reverse half
 * step, and the accept gate g~ = min(0, H0 - HL) - log u_t with
 * H = v.M^-1 v / 2 - log p(x); its relaxed form (PMC_GATE_SURROGATE) enters
 * the Jacobian as for MALA. */
typedef enum { PMC_SAMPLER_MALA = 0, PMC_SAMPLER_ULA = 1, PMC_SAMPLER_HMC = 2 } pmc_sampler;

typedef enum {
    PMC_TARGET_GAUSSIAN = 0, /* log p = -(x-mu)^T P (x-mu) / 2                          */
    PMC_TARGET_BANANA = 1,   /* D = 2: log p = -x1^2/2 - (x2 - x1^2)^2/2                */
    PMC_TARGET_LOGREG = 2,   /* sum_n [y_n z_n - log(1+e^{z_n})] - |x|^2/(2 prior_var), z = X x */
    PMC_TARGET_FUNNEL = 3    /* x1 ~ N(0, e^{2 theta}), x_d | x1 ~ N(0, e^{x1}), d >= 2 */
} pmc_target_kind;

/* Jacobian structure of the Newton update. */
typedef enum {
    PMC_DEER_DENSE = 0,   /* full D x D J_t (Sec. 2 eq. 2-3)                         */
    PMC_QDEER_DIAG = 1,   /* diag(J_t) (Sec. 2 eq. 4)                                 */
    PMC_QDEER_BLOCK2 = 2, /* diagonal of each D x D block (leapfrog only, App. A.3)   */
    PMC_PICARD = 3        /* J_t = 0                                                  */
} pmc_variant;

/* Storage/compute precision of dense Jacobian compositions (PMC_DEER_DENSE). */
typedef enum { PMC_JAC_F32 = 0, PMC_JAC_BF16 = 1 } pmc_jac_prec;

/* How the accept gate enters the Jacobian: FROZEN treats the decision as a
 * constant; SURROGATE is the stop-gradient relaxation of Sec. 3.2, adding
 * sigma'(g~) (x~ - x) (d g~/dx)^T. */
typedef enum { PMC_GATE_FROZEN = 0, PMC_GATE_SURROGATE = 1 } pmc_gate;

/* How the logistic-regression evaluation forms its matrix products (FP32
 * targets, D <= 32 for SPLIT16 and REFINE).  SPLIT16 writes each operand as hi + lo, two FP16 numbers, and sums
 * lo*hi + hi*lo + hi*hi on the FP16 matrix cores with FP32 accumulation (the
 * error-compensated half-precision product of Markidis et al. 2018 and Ootomo
 * & Yokota 2022: about 2^-22 of each product is dropped, against 2^-24 for
 * FP32; operands are brought to FP16's range by exact power-of-two scalings);
 * it needs n_data <= 1216.  AUTO takes SPLIT16 where that holds and FP32
 * matrix instructions elsewhere; SPLIT16 requested for more data points is
 * PMC_ERR_UNSUPPORTED at pmc_target_create.  REFINE keeps both: in pmc_solve
 * (MALA or ULA, no fixed-width window) each chain's Newton iteration runs on
 * SPLIT16 products until it meets the tolerance (or its rounding floor), then
 * restarts its window at its first step and runs on FP32 products until it
 * meets the tolerance again, so the result is the FP32-product iteration's
 * fixed point (Alg. 1 with a cheaper f in its early sweeps; the paper's
 * convergence test applies unchanged to the final sweeps).  It needs
 * n_data <= 1152 (PMC_ERR_UNSUPPORTED at pmc_target_create otherwise); with
 * a fixed-width window, and for HMC, chains use FP32 products throughout. */
typedef enum { PMC_PRODUCTS_AUTO = 0, PMC_PRODUCTS_F32 = 1, PMC_PRODUCTS_SPLIT16 = 2, PMC_PRODUCTS_REFINE = 3 } pmc_products;

typedef struct pmc_context pmc_context; /* opaque: device, stream, workspace pool, tuning table */
typedef struct pmc_target pmc_target;   /* opaque: device copy of a target's parameters        */

/* Target description.  All pointers DEVICE, read only during pmc_target_create,
 * in the dtype given (the library copies them). */
typedef struct {
    pmc_target_kind kind;
    int dim;             /* D */
    pmc_dtype dtype;
    const void *mean;    /* GAUSSIAN: [D]                          */
    const void *prec;    /* GAUSSIAN: [D, D] symmetric precision   */
    const void *X;       /* LOGREG:   [n_data, D] design           */
    const void *y;       /* LOGREG:   [n_data] labels in {0, 1}    */
    int n_data;          /* LOGREG                                 */
    double prior_var;    /* LOGREG:   prior N(0, prior_var I)      */
    double theta;        /* FUNNEL:   neck log-scale               */
    pmc_products products; /* LOGREG: matrix-product arithmetic (0 = AUTO) */
} pmc_target_desc;

/* One or more independent chains on one target, concatenated along time.
 * Chain c owns global steps offsets[c] .. offsets[c+1]-1 (CSR form). */
typedef struct {
    pmc_sampler sampler;
    const pmc_target *target;
    double step_size;         /* eps */
    int n_chains;             /* >= 1 */
    const int64_t *offsets;   /* HOST [n_chains+1], offsets[0] = 0, non-decreasing; NULL => one
                                 chain of length n_steps */
    int64_t n_steps;          /* sum of chain lengths (= offsets[n_chains] when offsets given) */
    const void *s0;           /* DEVICE [n_chains, D] initial states                        */
    const void *noise;        /* DEVICE [n_steps, D]  xi_t                                  */
    const void *uniforms;     /* DEVICE [n_steps]     u_t in (0, 1) (MALA only; may be NULL for ULA) */
    const void *init_guess;   /* DEVICE [n_steps, D] initial Newton guess, or NULL => each chain's
                                 s0 broadcast over its steps (the paper's choice)            */
    void *out_states;         /* DEVICE [n_steps, D] written: the trajectory                */
    uint8_t *out_accept;      /* DEVICE [n_steps] or NULL: accept decision of each step     */
    float *out_gtilde;        /* DEVICE [n_steps] or NULL: g~ = log alpha - log u (MALA, HMC) */
    int n_leapfrog;           /* HMC: leapfrog steps L per transition (1..1024)              */
    const void *inv_mass;     /* HMC: DEVICE [D] diagonal of M^-1 (positive), or NULL = identity */
} pmc_problem;

typedef struct {
    pmc_variant variant;
    pmc_jac_prec jac_prec;    /* PMC_DEER_DENSE only                                          */
    pmc_gate gate;
    double atol, rtol;        /* stop when max_{t,d} |s^{i+1} - s^i| / (atol + rtol |s^{i+1}|) <= 1 */
    int max_iter;             /* <= 0: min(T + 1, 50 + 5e-4 T), T the longest chain          */
    double damping;           /* J <- damping * J before clipping (1 = none)                  */
    double clip;              /* > 0: clip entries of J to [-clip, clip] (clip_inf_norm = 0), or
                                 rescale J so that |J|_inf <= clip (clip_inf_norm = 1)        */
    int clip_inf_norm;
    int skip_converged_prefix;/* sliding window (default 1): each sweep starts at the chain's
                                 first unconverged step, so the converged prefix is frozen;
                                 without it, rounding-level changes of that prefix can keep
                                 flipping a near-tie accept decision further on              */
    int graph_sweeps;         /* > 0: replay a captured HIP graph of this many sweeps between
                                 host convergence checks; 0: enqueue sweeps 8 at a time
                                 between checks (one at a time with trace_out).  Sweeps
                                 queued after every chain has stopped return at once and
                                 are not counted                                            */
    void *trace_out;          /* DEVICE or NULL: iterate after every sweep, [max_iter, n_steps, D] */
    size_t trace_bytes;       /* size of trace_out                                           */
    int floor_stall;          /* > 0: stop a chain at its rounding floor after this many sweeps
                                 without progress (no 2x drop of its best ratio and no advance
                                 of its converged front) while its ratio is <= 2 (the last
                                 change within twice the tolerance); 0: never                */
    int profile_kernels;      /* != 0 (graph_sweeps = 0 only): time every eval and scan launch
                                 with HIP events on the context's stream (pmc_result.*_ms)    */
    int jac_probes;           /* PMC_QDEER_DIAG.  0 (default): the exact diagonal of J_t.
                                 1: the stochastic estimate z o (J_t z) (Sec. 3.4 eq. 10; its
                                 mean over Rademacher z is diag J_t), one probe per step and
                                 sweep; the fixed point is unchanged, the sweep count is not.
                                 LOGREG forms J_t z on BF16 matrix cores (D <= 32)            */
    uint64_t probe_seed;      /* sign of coordinate d at global step t in sweep i (counted from
                                 0 per chain): -1 if the top bit of m(m(m(probe_seed) ^ i) ^
                                 (1024 t + d)) is set, else +1, where m(x) is SplitMix64 (the
                                 output function of x + 0x9E3779B97F4A7C15)                   */
    const void *basis;        /* NULL (default), or DEVICE [D, D] row-major orthogonal Q in the
                                 state dtype: quasi-DEER (or Picard) iterates z = Q^T s and
                                 takes diag(Q^T J_t Q) (Sec. 3.4 eq. 11); the states, trace and
                                 initial guess stay in s.  Per-step targets: no probes.
                                 LOGREG: solved as the rotated model (design X Q, noise
                                 Q^T xi) with any variant it supports, allocating the rotated
                                 copies for the call.  Q must outlive the call              */
    int window_width;         /* > 0 (needs skip_converged_prefix): the sliding window of Sec. 3.4
                                 with a fixed width -- each sweep updates at most this many
                                 steps of a chain, from its first unconverged step; the window
                                 moves on once its steps meet the tolerance.  0: the window
                                 runs to the chain's end                                      */
    double tie_band;          /* >= 0: an accept decision whose gate |g~| is below this keeps the
                                 decision of the chain's previous sweep (from its second sweep
                                 on), so that rounding-level changes of the iterate cannot flip
                                 a decision the arithmetic cannot resolve back and forth between
                                 sweeps; 0 disables.  Default 2e-5 for F32 (the FP32 error
                                 bound of g~ on the logistic posterior), 0 for F64            */
} pmc_options;

typedef struct {
    int32_t *sweeps_per_chain;/* HOST [n_chains] or NULL: sweeps (Alg. 1 count) per chain   */
    int n_converged;          /* chains that met the tolerance                               */
    int sweeps_total;         /* sweeps executed (max over chains)                           */
    int n_floor;              /* chains stopped at their rounding floor (see floor_stall)      */
    int64_t n_accept;         /* accepted steps (MALA), from the last sweep's decisions      */
    double resid_inf;         /* max |s_t - f_t(s_{t-1})| at the last linearisation point      */
    double resid_l2;          /* its Euclidean norm, accumulated in FP64                      */
    double max_ratio;         /* final Delta-ratio (<= 1 means converged)                     */
    int64_t nonfinite;        /* count of non-finite iterate elements seen in the last sweep  */
    float elapsed_ms;         /* device time of the call, HIP events                          */
    float eval_ms;            /* with profile_kernels: summed duration of the eval launches   */
    float scan_ms;            /* with profile_kernels: summed duration of the scan launches   */
    int64_t eval_steps;       /* with profile_kernels: steps evaluated over all sweeps        */
    int8_t *chain_state;      /* HOST [n_chains] or NULL: per chain 0 = met the tolerance,
                                 1 = stopped at its rounding floor, 2 = reached max_iter     */
} pmc_result;

/* ---- context ------------------------------------------------------------ */
/* Creates a context on HIP device `device`, enqueueing on `hip_stream`
 * (a hipStream_t, or NULL for the default stream).  Fails with PMC_ERR_HIP
 * when no usable device exists. */
pmc_status pmc_create(pmc_context **out, int device, void *hip_stream);
pmc_status pmc_destroy(pmc_context *ctx);
pmc_status pmc_set_stream(pmc_context *ctx, void *hip_stream);

/* ---- targets ------------------------------------------------------------ */
/* Copies the target's parameters to library-owned device memory. */
pmc_status pmc_target_create(pmc_context *ctx, const pmc_target_desc *desc, pmc_target **out);
pmc_status pmc_target_destroy(pmc_target *tgt);

/* ---- parallel Newton solve (Algorithm 1) --------------------------------- */
/* Device workspace pmc_solve needs for this problem and options. */
pmc_status pmc_workspace_size(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                              size_t *bytes);
/* Fills *opts with the defaults: quasi-DEER diagonal, frozen gate,
 * atol = rtol = 5e-7 (1e-12 for F64), max_iter auto, no damping or clipping,
 * floor_stall 16. */
pmc_status pmc_default_options(pmc_options *opts, pmc_dtype dtype);
/* Solves every chain of `prob` by parallel Newton iterations.  `workspace`
 * is DEVICE memory of at least pmc_workspace_size bytes, or NULL to use the
 * context's pool.  res (HOST) may be NULL.
 * PMC_DEER_DENSE: F32 states with D <= 32 use the matrix-core scan (one chain
 * per call; jac_prec F32 with D <= 4, or F64 states, the vector scan).  On
 * the logistic posterior the Jacobians I + a_t eps Hess log p(s_{t-1}) are
 * formed from BF16 matrix-core pair sums of X^T diag(w) X (Sec. 2 with the
 * model of App. B.1); the first dense solve on a target allocates its
 * operand tables (about 1 KiB per 32 data points and 32 variable pairs,
 * kept until pmc_target_destroy), so concurrent first dense solves on one
 * target are not allowed.  Undamped full DEER on that posterior takes large
 * excursions; clip_inf_norm with clip = 1 keeps it stable. */
pmc_status pmc_solve(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                     void *workspace, size_t ws_bytes, pmc_result *res);

/* ---- allocation-free solve -------------------------------------------------- */
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): pmc_solve
 * with its workspace and the scans' look-back descriptors taken from a
 * per-device static scratch array of 64 MiB (PMC_SCRATCH_BYTES), loaded with
 * the library and held until the process ends.  Calls no hipMalloc, hipFree
 * or allocating library routine.  The caller passes inputs and outputs as
 * for pmc_solve.  A problem whose workspace plus descriptors exceed the
 * scratch is PMC_ERR_INVALID (quasi-DEER F32 fits up to about 5e6 steps x
 * coordinates); graph_sweeps > 0, the rotated logistic model (basis on
 * LOGREG) and the logistic posterior's dense or probed Jacobians before one
 * pmc_solve has built the target's operand tables are PMC_ERR_UNSUPPORTED.
 * Every call on a device shares that device's scratch and leaves its
 * contents behind (the descriptors are cleared at each call, the workspace
 * is fully rewritten), so calls that overlap on one device -- from several
 * threads, contexts or streams -- race. */
#define PMC_SCRATCH_BYTES (64u << 20)
pmc_status pmc_solve_noalloc(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                             pmc_result *res);

/* ---- same-GPU sequential sampler ------------------------------------------ */
/* Evaluates s_t = f_t(s_{t-1}) step by step on the device (one workgroup per
 * chain): the baseline the parallel solve is measured against (Sec. 2). */
pmc_status pmc_sample_sequential(pmc_context *ctx, const pmc_problem *prob, pmc_result *res);

/* ---- HMC with parallel leapfrog (Appendix A.2 algorithm) ------------------ */
/* n_prop sequential HMC proposals with L leapfrog steps of size step_size on
 * `target` (F32 only).  Each proposal draws momentum momenta[p] (DEVICE
 * [n_prop, D]), half-steps it, integrates, reverse half-steps and accepts iff
 * log unif[p] < H0 - HL (DEVICE [n_prop]).  parallel_leapfrog != 0 solves the
 * L-step leapfrog recursion on s = [x, v] in R^{2D} by Newton iterations with
 * opts->variant (PMC_QDEER_BLOCK2, PMC_QDEER_DIAG or PMC_PICARD) and tolerance;
 * 0 integrates sequentially.  out_chain: DEVICE [n_prop+1, D] (row 0 = x0);
 * accept: DEVICE [n_prop] or NULL; logr: DEVICE [n_prop] or NULL, the test's
 * margin (H0 - HL) - log U, assembled in FP64 from FP32 terms and rounded to
 * float (accept iff > 0); sweeps: HOST [n_prop] or NULL (Newton sweeps per
 * proposal). */
pmc_status pmc_hmc_sample(pmc_context *ctx, const pmc_target *target, double step_size, int L,
                          int n_prop, const void *x0, const void *momenta, const void *unif,
                          const pmc_options *opts, int parallel_leapfrog, void *out_chain,
                          uint8_t *accept, float *logr, int32_t *sweeps, pmc_result *res);

/* ---- derivatives through a converged chain ---------------------------------- */
/* Reverse (adjoint) scan lambda_t = dF/ds_t + J_{t+1}^T lambda_{t+1} over the
 * transposed step Jacobians at the trajectory `states` (DEVICE [T, D], the
 * converged output of pmc_solve with accept decisions `accept`, DEVICE [T]),
 * then dF/dtheta = sum_t lambda_t . df_t/dtheta and dF/deps likewise, FP64
 * sums.  dF_ds: DEVICE [T, D].  Single chain, F32, frozen gate.  Results are
 * written to the HOST scalars. */
pmc_status pmc_adjoint(pmc_context *ctx, const pmc_problem *prob, const void *states,
                       const uint8_t *accept, const void *dF_ds, double *dF_dtheta,
                       double *dF_dstep);

/* ---- linear recursions on their own (the scans of the Newton update) ------- */
/* delta_t = a_t * delta_{t-1} + b_t, delta_0 = 0, for n_lanes independent
 * lanes.  a, b, out: DEVICE [n_lanes, T] (each lane's sequence contiguous).
 * Quasi-DEER's recursion (Sec. 2 eq. 4). */
pmc_status pmc_linrec_diag(pmc_context *ctx, pmc_dtype dtype, int n_lanes, int64_t T,
                           const void *a, const void *b, void *out);
/* Block form of Appendix A.3: per lane [p; q]_t = [[a, b], [c, d]]_t [p; q]_{t-1}
 * + [e; f]_t.  coef: DEVICE [4, n_lanes, T] (planes a, b, c, d); rhs: DEVICE
 * [2, n_lanes, T] (planes e, f); out: DEVICE [2, n_lanes, T] (planes p, q). F32. */
pmc_status pmc_linrec_block2(pmc_context *ctx, int n_lanes, int64_t T, const void *coef,
                             const void *rhs, void *out);
/* Dense form (Sec. 2 eq. 3): delta_t = A_t delta_{t-1} + b_t.  A: DEVICE
 * [T, D, D]; b, out: DEVICE [T, D].  F64 for D <= 4 (VALU); F32 with
 * jac_prec BF16 or F32 for D <= 32 (matrix cores). */
pmc_status pmc_linrec_dense(pmc_context *ctx, pmc_dtype dtype, pmc_jac_prec jac_prec, int D,
                            int64_t T, const void *A, const void *b, void *out);

/* Kernel timing of the two recursions above.  With on != 0, pmc_linrec_diag
 * and pmc_linrec_block2 record HIP events around their scan kernel on the
 * context's stream (the calls still synchronise before returning);
 * pmc_last_scan_ms writes that kernel's duration in milliseconds for the
 * most recent such call to the HOST float *ms (0 before any).  Off by
 * default. */
pmc_status pmc_set_scan_timing(pmc_context *ctx, int on);
pmc_status pmc_last_scan_ms(pmc_context *ctx, float *ms);

/* ---- tuning --------------------------------------------------------------- */
/* Times the scan tile configurations for this problem's shape on the device
 * and stores the fastest in the context (and, if cache_path != NULL, in a
 * JSON file keyed by the device's architecture name).  If the file exists
 * and holds an entry for this shape, it is loaded instead of timing. */
pmc_status pmc_autotune(pmc_context *ctx, const pmc_problem *prob, const pmc_options *opts,
                        const char *cache_path);

/* Thread-local description of the last failure on this thread. */
const char *pmc_last_error(void);
const char *pmc_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PMCMC_H */
