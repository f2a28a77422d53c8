/*
 * pcls - parallel continuous local search for symmetric pseudo-Boolean SAT.
 *
 * C ABI of the MI355X (gfx950) library libpcls.so.
 *
 * The library evaluates, for many restarts at once, the Walsh-Fourier relaxed
 * objective F(x) = sum_c w_c FE_c(x) of a formula of symmetric constraints on
 * the hypercube [-1,1]^n and its gradient, and takes projected gradient steps
 * x <- clip(x - lr * grad F, -1, 1) (paper: Background, "Satisfaction as
 * Optimisation"; the FE of one constraint is eq. wft with the coefficients of
 * eq. wfcoef, Background, "Walsh-Fourier Transformation").
 *
 * Conventions.
 *  - Boolean True is -1 and False is +1.  A literal over variable v has value
 *    y = s * x_v, s = +1 for a positive literal and -1 for a negated one; a
 *    positive literal is true at x_v = -1.
 *  - A symmetric constraint's value at a corner is -1 when it holds and +1
 *    when it is violated; a corner satisfies the formula iff sum_c FE_c = -m.
 *  - Restart state X is float32, laid out [n][R_pad] (restart index
 *    contiguous), R_pad = round_up(R, 64).  Columns r >= R are padding: the
 *    library may read and write them and their content is unspecified.
 *  - Gradients are accumulated in exact fixed point, so they (and hence the
 *    iterates) are bitwise reproducible and independent of the launch shape;
 *    objectives are FP32 sums over fixed work chunks added in exact fixed point,
 *    bitwise reproducible for a given launch shape.  The fixed-point scales are
 *    chosen per problem (see pcls_info) so that no sum overflows.
 *  - All device pointers are caller-owned (hipMalloc'd or torch tensors).
 *    Every device operation is enqueued asynchronously on the given HIP
 *    stream (hipStream_t passed as void*; NULL = the null stream); the host
 *    pointers passed to pcls_plan are borrowed only for the call.
 *  - Every function returns a status code and never throws or aborts across
 *    the ABI; pcls_last_error() describes the last failure on this thread.
 *  - A planned problem is read-only after pcls_upload: concurrent evaluate /
 *    step / extract calls on different streams with different X are safe.
 */
#ifndef PCLS_H
#define PCLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pcls_problem pcls_problem;

enum {
  PCLS_OK = 0,
  PCLS_E_INVALID = 1,      /* malformed input (bad CSR, literal, type, parameter, pointer) */
  PCLS_E_UNSUPPORTED = 2,  /* constraint longer than 256 literals, or problem too large */
  PCLS_E_DUPVAR = 3,       /* a variable occurs twice in one constraint */
  PCLS_E_WORKSPACE = 4,    /* workspace missing or smaller than reported */
  PCLS_E_HIP = 5           /* a HIP runtime call failed (message holds the HIP error string) */
};

/* Constraint types (paper: Table 2 and Appendix A). */
enum {
  PCLS_OR = 0,      /* at least one literal true                                  */
  PCLS_XOR = 1,     /* number of true literals = param (mod 2); param 1 = odd parity */
  PCLS_CARD_GE = 2, /* at least param literals true, 0 <= param <= k               */
  PCLS_NAE = 3,     /* not all equal: 0 < #true < k                                */
  PCLS_EO = 4,      /* exactly one true                                            */
  PCLS_AMO = 5,     /* at most one true                                            */
  PCLS_EK = 6       /* exactly param true, 0 <= param <= k                         */
};

/* Planning options (pcls_plan_ex).  Zero-initialised = defaults. */
typedef struct pcls_plan_options {
  int32_t force_generic;    /* 1: evaluate every constraint through the K-node DFT path
                               (no one- or two-node product forms); for testing */
  int32_t accumulator_bits; /* gradient accumulator: 0 = automatic, 32 or 64.  Automatic
                               takes 32-bit fixed point when its quantum is at most 2^-24
                               (grad_scale_log2_32 >= 24: no coarser than FP32 rounding at
                               unit scale), else 64-bit when the state fits on chip, else
                               32-bit */
  int32_t bucket_table;     /* length buckets the constraints are padded to: 0 = every
                               compiled length (1..8, 12, 16, 24, 32, 48, 64, 96, 128, 192,
                               256), 1 = 1..8 and the powers of two above (fewer segments,
                               more padding); chosen by the autotuners */
  int32_t reserved[5];
} pcls_plan_options;

typedef struct pcls_info {
  int32_t n_vars, n_cons;
  int64_t n_lits;            /* L = sum of constraint lengths */
  int32_t max_len;
  int32_t n_classes;         /* distinct (type, length, param) */
  int32_t n_segments;
  int32_t accumulator_bits;  /* requested gradient accumulator width (0 = automatic) */
  int32_t grad_scale_log2_64; /* fixed-point scales 2^S of the 64-bit and 32-bit gradient */
  int32_t grad_scale_log2_32; /* accumulators and of the objective accumulator            */
  int32_t obj_scale_log2;
  int32_t tile_restarts;     /* restarts per workgroup of the resident engine (0 = auto) */
  int32_t block_threads;     /* threads per workgroup of the resident engine (0 = auto) */
  size_t workspace_bytes;
  size_t lds_bytes_per_restart; /* on-chip bytes one restart's state needs */
  int32_t cons_by_kind[5];   /* constraints per evaluation path: one-node product, two-node
                                product, K-node DFT, truncated count distribution (k <= 48,
                                window of at most 4 counts for k <= 8, at most half the
                                length bucket above), constant */
  int32_t bucket_table;      /* length-bucket table of the plan (pcls_plan_options) */
} pcls_info;

/*
 * Validate a formula and plan its evaluation on the host.
 *   n_vars, n_cons   : n >= 1 variables, m >= 0 constraints.
 *   row_ptr[m+1]     : host; row_ptr[0] = 0, non-decreasing; constraint c owns
 *                      lit[row_ptr[c] .. row_ptr[c+1]); every length k >= 1.
 *   lit[L]           : host; +v / -v, 1 <= v <= n_vars; no variable twice in
 *                      one constraint (PCLS_E_DUPVAR); k <= 256 (PCLS_E_UNSUPPORTED).
 *   type[m]          : host; PCLS_OR .. PCLS_EK.
 *   param[m]         : host; XOR parity in {0,1}; CARD_GE / EK kappa in [0,k];
 *                      ignored for other types; NULL = all zero.
 *   weight[m]        : host; finite constraint weights; NULL = all 1.0.
 * On success *out receives a host plan (free with pcls_destroy) and
 * *workspace_bytes the size of the device workspace pcls_upload needs.
 * Computes, per distinct (type, k, param), the spectrum sp_t (eq. wfcoef) and
 * either its one/two-node product form or the FP64 inverse-DFT weights
 * chat_m = (1/K) sum_t sp_t omega^-tm, K = k + 1, rounded once to float32.
 */
int32_t pcls_plan(int32_t n_vars, int32_t n_cons, const int32_t* row_ptr, const int32_t* lit,
                  const int8_t* type, const int32_t* param, const float* weight, pcls_problem** out,
                  size_t* workspace_bytes);
int32_t pcls_plan_ex(int32_t n_vars, int32_t n_cons, const int32_t* row_ptr, const int32_t* lit,
                     const int8_t* type, const int32_t* param, const float* weight,
                     const pcls_plan_options* options, pcls_problem** out, size_t* workspace_bytes);

/* Sizes and launch settings of a plan. */
int32_t pcls_problem_info(const pcls_problem* p, pcls_info* info);

/*
 * Copy the plan into caller-owned device memory d_workspace (>= workspace_bytes,
 * 256-byte aligned), asynchronously on stream, and bind it to the plan.  The
 * image holds what the evaluation of every constraint needs (paper: Background,
 * "Walsh-Fourier Transformation", eq. wfcoef and the DFT evaluation named in
 * "Satisfaction as Optimisation"): the spectra sp_i, the inverse-DFT node
 * weights and node factors planned from them, and the constraints' literals in
 * segment order.  The workspace must stay allocated while the plan is used;
 * the library never frees it.  Errors: PCLS_E_INVALID for a NULL plan;
 * PCLS_E_WORKSPACE for a NULL or not 256-byte aligned workspace or when
 * bytes < workspace_bytes; PCLS_E_HIP when the copy cannot be enqueued.
 */
int32_t pcls_upload(pcls_problem* p, void* d_workspace, size_t bytes, void* hip_stream);

/*
 * Restart initialisation x[v][r] ~ U[-1,1) (paper: "starting assignments",
 * Case Studies, "Costas Arrays"; the distribution is this library's choice).
 * Philox4x32-10 (Salmon et al., SC'11) with counter (r, v, 0, 0) and key
 * (seed low word, seed high word); the top 24 bits i of the first output word
 * give x = (i - 2^23) / 2^23.  Padding columns r in [R, R_pad) are set to 0.
 * d_x: device [n][R_pad] float32.
 */
int32_t pcls_init_restarts(const pcls_problem* p, int32_t R, uint64_t seed, float* d_x, void* hip_stream);

/*
 * Fresh starting points for selected restarts only: every restart r < R with
 * d_mask[r] != 0 gets exactly the column pcls_init_restarts would write for
 * this seed; all other columns of d_x (padding included) are left as they are.
 * This is how converged restarts are recycled while the others keep running
 * (in lockstep, restarts that have converged would otherwise idle until the
 * slowest finishes: Case Studies, "Costas Arrays: Convergence Profile
 * Analysis").  d_mask: device uint8 [R], read only; NULL is PCLS_E_INVALID.
 */
int32_t pcls_init_restarts_masked(const pcls_problem* p, int32_t R, uint64_t seed, const uint8_t* d_mask,
                                  float* d_x, void* hip_stream);

/*
 * Objective and gradient at X (Background, "Satisfaction as Optimisation").
 *   d_x    : device [n][R_pad] float32, read only.
 *   d_obj  : device [R] float32, F_r = sum_c w_c FE_c(x_r).
 *   d_grad : device [n][R_pad] float32 (padding columns written too) or NULL.
 */
int32_t pcls_evaluate(const pcls_problem* p, int32_t R, const float* d_x, float* d_obj, float* d_grad,
                      void* hip_stream);

/*
 * n_steps >= 0 projected gradient steps x <- min(1, max(-1, x - lr * grad F(x)))
 * in place on d_x ([n][R_pad] float32).  If d_obj_trace is not NULL it receives
 * [n_steps][R] float32: entry (s, r) is F at x_s, before step s.
 */
int32_t pcls_step(const pcls_problem* p, int32_t R, float* d_x, float lr, int32_t n_steps,
                  float* d_obj_trace, void* hip_stream);

/*
 * Options of pcls_step_ex (zero-initialised = plain pcls_step).
 *  d_fixed : device int8 [n] or NULL.  0 = free; -1 / +1 = variable held at
 *            True / False in every restart (its x is set on entry and after
 *            every step): completion of a partial assignment (paper: Case
 *            Studies, "Hard Random 3-SAT: Partial Assignment Completion").
 *  tol     : > 0 enables the convergence test max_v |x_{s+1} - x_s| < tol per
 *            restart.  A workgroup's restarts stop stepping once all of them
 *            have converged (converged restarts stop costing compute: Case
 *            Studies, "Costas Arrays"); trace entries after that repeat the
 *            last evaluated objective.  0 = no test.
 *  d_iters : device int32 [R] or NULL: 1-based step at which the restart first
 *            passed the test, n_steps if it never did (requires tol > 0).
 */
typedef struct pcls_step_options {
  const int8_t* d_fixed;
  float tol;
  int32_t* d_iters;
  int32_t reserved[4];
} pcls_step_options;

int32_t pcls_step_ex(const pcls_problem* p, int32_t R, float* d_x, float lr, int32_t n_steps, float* d_obj_trace,
                     const pcls_step_options* options, void* hip_stream);

/*
 * Round X to corners and count violated constraints exactly (paper: Background,
 * "Satisfaction as Optimisation": a corner sign(X) satisfies the formula iff
 * sum_c FE_c(sign X) = -m, i.e. iff every constraint's spectrum entry sp_i at
 * its number i of true literals is -1, eq. wfcoef).
 *   d_assign : device [R][n] int8 or NULL; -1 (True) where x < 0, else +1
 *              (False; -0.0 and +0.0 both give False).
 *   d_unsat  : device [R] int32, number of constraints violated by the corner.
 *   d_best   : device [1] int32 or NULL: restart with the fewest violations,
 *              ties to the lowest index.
 */
int32_t pcls_extract(const pcls_problem* p, int32_t R, const float* d_x, int8_t* d_assign,
                     int32_t* d_unsat, int32_t* d_best, void* hip_stream);

/*
 * Launch settings of the resident engine: restarts per workgroup (power of
 * two, 1..64) and threads per workgroup (256, 512 or 1024); 0 = automatic.
 * PCLS_E_UNSUPPORTED if the setting does not fit the device's on-chip memory.
 */
int32_t pcls_set_launch(pcls_problem* p, int32_t tile_restarts, int32_t block_threads);

/*
 * The resident-engine launch the library will use for R restarts on the current
 * device: restarts per workgroup, threads per workgroup, gradient accumulator
 * width (32 or 64), its fixed-point scale log2 (a gradient sum is exact in units
 * of 2^-S; each term is rounded to the nearest unit) and LDS bytes per
 * workgroup.  Any output pointer may be NULL.  Queries the device (no launch).
 */
int32_t pcls_launch_info(const pcls_problem* p, int32_t R, int32_t* tile_restarts, int32_t* block_threads,
                         int32_t* accumulator_bits, int32_t* grad_scale_log2, size_t* lds_bytes);

/* ------------------------------------------------------------------ batches
 * Many uploaded problems (instances of uneven size) and their restarts run in
 * one persistent launch: work items (instance, restart tile) are claimed from a
 * device counter in order of decreasing cost, and each workgroup runs all steps
 * of its tile on chip.  Restarts are independent, so no cross-workgroup
 * synchronisation is needed.  A configuration (threads per workgroup and the
 * LDS budget the tiles are sized for) can be chosen by pcls_batch_autotune.
 */
typedef struct pcls_batch pcls_batch;

typedef struct pcls_batch_config {
  int32_t block_threads;    /* 256, 512 or 1024 (0 = 1024) */
  int32_t lds_budget;       /* LDS bytes per workgroup the tiles are sized for (0 = device max) */
  int32_t wgs_per_cu;       /* cap on persistent workgroups per CU (0 = as many as fit); reports the value used */
  int32_t accumulator_bits; /* 0 = automatic, 32 or 64; reports the width used.  One width
                               serves the whole batch: automatic takes 64 bits if any
                               instance asks for them or needs them by the rule of
                               pcls_plan_options and every instance fits with them */
} pcls_batch_config;

/*
 * problems[count]: uploaded plans (borrowed; must outlive the batch);
 * restarts[count]: R_i >= 1.  *workspace_bytes: device workspace to pass to
 * pcls_batch_bind (256-byte aligned, caller-owned).
 */
int32_t pcls_batch_create(const pcls_problem* const* problems, int32_t count, const int32_t* restarts,
                          pcls_batch** out, size_t* workspace_bytes);
/*
 * Bind device memory: d_x[i] is instance i's state [n_i][round_up(R_i, 64)]
 * float32; d_trace[i] (or d_trace NULL / entries NULL) receives
 * [n_steps][R_i] objective values on each pcls_batch_step.  Host arrays are
 * borrowed for the call.  Applies the current configuration (default on first
 * bind) and synchronises the stream.  Invalidates a captured graph.
 */
int32_t pcls_batch_bind(pcls_batch* b, void* d_workspace, size_t bytes, float* const* d_x, float* const* d_trace,
                        void* hip_stream);
int32_t pcls_batch_set_config(pcls_batch* b, const pcls_batch_config* cfg, void* hip_stream);
int32_t pcls_batch_get_config(const pcls_batch* b, pcls_batch_config* cfg, int32_t* n_items, int32_t* grid);
/* n_steps projected gradient steps of every instance: one fused launch (plus a counter reset). */
int32_t pcls_batch_step(pcls_batch* b, float lr, int32_t n_steps, void* hip_stream);
/*
 * Capture one pcls_batch_step(lr, n_steps) into a HIP graph (on a private
 * stream, after synchronising hip_stream); pcls_batch_replay launches it on a
 * stream.  The graph holds the bound pointers and configuration.
 */
int32_t pcls_batch_capture(pcls_batch* b, float lr, int32_t n_steps, void* hip_stream);
int32_t pcls_batch_replay(pcls_batch* b, void* hip_stream);
/*
 * Time every feasible configuration (threads per workgroup x LDS budget) on
 * probe_steps real steps of the bound states (which advance), keep the fastest.
 */
int32_t pcls_batch_autotune(pcls_batch* b, float lr, int32_t probe_steps, void* hip_stream, pcls_batch_config* best,
                            float* best_ms);
/* Free the batch (and its graph); never frees caller memory or the problems. */
int32_t pcls_batch_destroy(pcls_batch* b);

/* Free the host plan; never frees caller memory. */
int32_t pcls_destroy(pcls_problem* p);

/*
 * Per-constraint gradient statistic for adaptive weighting (Case Studies,
 * "Redundant Constraint Effect", and Conclusions: weights informed by
 * per-constraint gradient magnitudes).  For every constraint c,
 *   d_out[c] = sum over restarts r < R of sum over literals i of c of
 *              (dFE_c/dy_i at x_r)^2,
 * unweighted (y_i the literal value), in the caller's constraint order.
 *   d_x   : device [n_vars][R_pad] state, as for pcls_evaluate.
 *   d_acc : device scratch of n_cons 64-bit words (caller-owned, overwritten).
 *   d_out : device float[n_cons].
 * Sums are exact 64-bit fixed point at scale 2^s, s = min(40, 60 - ceil(log2(R
 * max_len + 1))), so the result is deterministic; constant constraints report
 * 0.  Asynchronous on `stream`.  PCLS_E_INVALID for R < 1 or a NULL pointer
 * (n_cons > 0); PCLS_E_UNSUPPORTED when one restart's state does not fit in LDS.
 */
int32_t pcls_constraint_grad_stats(const pcls_problem* p, int32_t R, const float* d_x, uint64_t* d_acc,
                                   float* d_out, void* stream);

/*
 * pcls_constraint_grad_stats without the caller's accumulator, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the accumulator is a static device array
 * of the library (2 MiB per device, held until the process ends), and the call
 * allocates nothing.  Same arguments otherwise, same results bit for bit.
 * PCLS_E_UNSUPPORTED when n_cons exceeds 262144 (the array's 64-bit words).
 * Every call on one device shares that device's array and clears it first:
 * calls that overlap on one device (concurrent streams, threads) race, so
 * serialise them.
 */
int32_t pcls_constraint_grad_stats_noalloc(const pcls_problem* p, int32_t R, const float* d_x, float* d_out,
                                           void* hip_stream);

/* Thread-local description of the last error; valid until the next call. */
const char* pcls_last_error(void);


#ifdef __cplusplus
}
#endif
#endif /* PCLS_H */
