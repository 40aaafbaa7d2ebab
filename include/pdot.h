/*
 * pdot.h -- C ABI of the MI355X (gfx950) restarted-PDHG optimal-transport library.
 *
 * The library solves the discrete Kantorovich problem (Lu & Yang, "PDOT", arXiv
 * 2407.19689, Section 1, eq. ot)
 *
 *     min <C, X>   s.t.   X 1_n = f,   X^T 1_m = g,   X >= 0
 *
 * with restarted PDHG in the matrix-free form of Algorithm 2 (alg:rpd): per iteration a
 * projected primal step X+ = max(0, X - tau (C - p 1^T - 1 q^T)), the row and column sums
 * of 2X+ - X, the dual steps p+ = p + sigma (f - (2X+ - X) 1), q+ = q + sigma (g -
 * (2X+ - X)^T 1), and a running average.  Control follows Section 5: restart to the
 * candidate of lower relative KKT error with the three restart conditions, the adaptive
 * step size eta with tau = eta/omega and sigma = eta*omega, the primal-weight update at
 * restarts, and termination on relative KKT error (Section 5.1, "Termination criteria").
 * The KKT error is the stacked 2-norm of Section 3.1 (display after Algorithm 2); the
 * relative form and the other readings of the text are listed with ot_params below.
 *
 * Every iteration runs on the GPU in hand-written HIP kernels; the host only launches
 * graphs of iteration slots and reads a status word between them.
 *
 * Conventions for every entry point:
 *   - Matrices are row-major.  X_ij is transported mass from source i to target j.
 *   - Input pointers may be host or device pointers (unified addressing); they are read
 *     during the call only.  The caller owns every buffer it passes; the library never
 *     frees or retains caller memory.
 *   - The library allocates its own device workspace for the duration of a call unless
 *     a workspace of at least ot_workspace_size() bytes is passed.
 *   - Calls are ordered on the HIP stream passed as `stream` (hipStream_t, may be NULL
 *     for an internal stream) and are synchronous: they return when results are in the
 *     output buffers.
 *   - Return value: OT_OK, or an error code; ot_last_error() then holds a message
 *     (per thread).  OT_NOT_CONVERGED still fills every output with the returned iterate.
 */
#ifndef PDOT_H
#define PDOT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    OT_OK = 0,
    OT_ERR_INVALID = 1,    /* bad sizes, pointers, non-finite data, sum f != sum g, tol <= 0 */
    OT_ERR_OOM = 2,        /* device allocation failed or workspace too small             */
    OT_ERR_DEVICE = 3,     /* a HIP runtime call failed                                    */
    OT_NOT_CONVERGED = 4,  /* iteration, pass or time limit reached, or the returned arrays
                              failed the final verification verify_retries + 1 times;
                              outputs are filled                                        */
    OT_ERR_NUMERIC = 5,    /* a KKT or step-size scalar became NaN/Inf                     */
    OT_ERR_BUSY = 6        /* server queue full or request over its memory budget          */
} ot_status;

/* Working precision of the iterates and of the cost stream.  OT_PREC_FP64 is the paper's
 * own precision (8-byte cost entries, Section 5.1 Table stats).  OT_PREC_FP32 streams X,
 * the average and C in FP32 while p, q, all row/column sums, KKT pieces, the duality gap
 * and every control scalar stay in FP64 (the primal step is evaluated in FP64 and rounded
 * once to FP32). */
typedef enum { OT_PREC_FP64 = 0, OT_PREC_FP32 = 1 } ot_precision;

/* Cost description (eq. ot; the pixel-grid costs of Section 5.1).
 *   OT_COST_DENSE            C: m x n FP64, row stride ldc (>= n) elements.
 *   OT_COST_POINTS_SQEUCLID  C_ij = sum_k (x_ik - y_jk)^2, x: m x dim, y: n x dim FP64.
 *   OT_COST_POINTS_EUCLID    C_ij = sqrt(sum_k (x_ik - y_jk)^2).
 *   OT_COST_GRID_SQEUCLID    m = n = side^2 pixels of an side x side image, pixel
 *                            i = (i / side, i % side); C_ij = scale * squared pixel distance.
 *   OT_COST_GRID_L1, OT_COST_GRID_L2, OT_COST_GRID_LINF
 *                            the same pixels with the l1, l2 and l-infinity distances (the
 *                            C^1, C^2, C^inf costs of Section 5.1) times scale.
 * For the coordinate kinds `store` = 0 regenerates C_ij inside the iteration kernel from
 * the coordinates (no cost bytes streamed); `store` = 1 materialises C once in device
 * memory.  Both produce bit-identical cost values in the working precision. */
typedef enum {
    OT_COST_DENSE = 0,
    OT_COST_POINTS_SQEUCLID = 1,
    OT_COST_POINTS_EUCLID = 2,
    OT_COST_GRID_SQEUCLID = 3,
    OT_COST_GRID_L1 = 4,
    OT_COST_GRID_L2 = 5,
    OT_COST_GRID_LINF = 6
} ot_cost_kind;

typedef struct {
    int32_t kind;       /* ot_cost_kind                                  */
    int32_t dim;        /* points kinds: coordinate dimension, 1..3      */
    int32_t side;       /* grid kind: image side                         */
    int32_t store;      /* coordinate kinds: 0 regenerate, 1 materialise */
    int64_t ldc;        /* dense kind: row stride of C in elements       */
    const double *C;    /* dense kind                                    */
    const double *x;    /* points kinds: m x dim, row-major              */
    const double *y;    /* points kinds: n x dim, row-major              */
    double scale;       /* grid kind: multiplier of the squared distance */
} ot_cost;

/* One record of the solver's control sequence (Section 5): a rejected step trial, or an
 * accepted iteration with the relative KKT errors of the current iterate and of the
 * average, the restart candidate and the restart decision.  The same fields as the FP64
 * oracle's trace, so the two can be compared decision by decision. */
typedef struct {
    int64_t pass;        /* step trials evaluated so far, this one included              */
    int64_t iter;        /* accepted iterations so far (this one included if accepted)   */
    int32_t accepted;    /* 1: the trial met the step-size bound                         */
    int32_t restart;     /* 0 none; 1, 2, 3: restart conditions (i), (ii), (iii) fired   */
    int32_t cand_avg;    /* restart candidate is the average                             */
    int32_t pad;
    double eta_used;     /* step size of the trial                                       */
    double eta_bar;      /* its step-size bound (+inf for a constant step)               */
    double k_cur, k_avg; /* relative KKT of the current iterate and of the average       */
    double omega;        /* primal weight in use                                         */
} ot_trace_rec;

/* One OT instance with its outputs. */
typedef struct {
    ot_cost cost;
    int64_t m, n;        /* m >= 1 sources, n >= 1 targets                           */
    const double *f;     /* m, >= 0, finite                                          */
    const double *g;     /* n, >= 0, finite, |sum f - sum g| <= 1e-12 max(sum f, sum g) */
    double tol;          /* > 0 overrides ot_params.tol for this instance            */
    void *X_out;         /* nullable; m x n contiguous, FP64 or FP32 per precision   */
    double *u_out;       /* nullable; m, the row duals p of the returned iterate      */
    double *v_out;       /* nullable; n, the column duals q                          */
    int32_t tile_vec;    /* > 0 overrides ot_params.tile_vec for this instance       */
    int32_t tile_rows;   /* > 0 overrides ot_params.tile_rows for this instance      */
    ot_trace_rec *trace; /* nullable; host or device, trace_cap records: the first
                            trace_cap control records of the solve (ot_result.trace_len
                            gives how many were written)                             */
    int64_t trace_cap;
} ot_problem;

/* Solver parameters.  Defaults (ot_params_default) are the paper's constants:
 * beta_sufficient 0.1, beta_necessary 0.9, beta_artificial 0.36 (Section 5, adaptive
 * restart), theta 0.5 and omega0 1 (Section 5, primal weight), tol 1e-4 (Section 5.1).
 * Readings where the paper is silent:
 *   kkt_mode 0: relative KKT = sqrt(rel_P^2 + rel_D^2 + rel_G^2) with
 *     rel_P = ||[X1-f; X^T1-g]|| / ||[f;g]||, rel_D = ||[p1^T+1q^T-C]^+||_F / ||C||_F,
 *     rel_G = |<C,X> - f^T p - g^T q| / (|<C,X>| + |f^T p + g^T q|);
 *   kkt_mode 1: denominators 1+||[f;g]||, 1+||C||_F, 1+|<C,X>|+|f^T p+g^T q|.
 *   eta0 <= 0 selects 1/sqrt(m+n) = 1/||A||_2 (Proposition prop:norm-sharp).
 *   step_rule 0: accept eta when eta <= omega||dX||^2 + ||dy||^2/omega over
 *     2|dp^T dX 1 + dq^T dX^T 1| (squared weighted norm), else retry from the same point;
 *     either way eta <- min((1-(T+1)^-a) eta_bar, (1+(T+1)^-b) eta), a = 0.3, b = 0.6.
 *   avg_weighting 0: average weighted by the step eta used; 1: uniform (Algorithm 2).
 *   restart_rule 0: Section 5 adaptive restart to the candidate; 1: Algorithm 2's rule
 *     KKT(average) <= beta_basic KKT(restart point), restart to the average; 2: never.
 *   output 0: return the restart candidate that met the tolerance; 1: the current iterate.
 */
typedef struct {
    double tol;
    int64_t max_iters;        /* accepted iterations                          */
    int64_t max_passes;       /* step trials (accepted + rejected)            */
    double time_limit_s;      /* <= 0: none (checked between graph launches)  */
    int32_t precision;        /* ot_precision                                 */
    int32_t kkt_mode;
    int32_t step_rule;        /* 0 adaptive, 1 constant eta                   */
    int32_t restart_rule;
    int32_t avg_weighting;
    int32_t primal_weight_update;  /* 1 on, 0 keep omega0                    */
    int32_t output;
    int32_t graph_slots;      /* iteration slots per graph launch, 0 = auto   */
    double beta_sufficient, beta_necessary, beta_artificial, beta_basic;
    double theta, omega0, eta0, eps_zero;
    double step_reduction_exp, step_growth_exp;
    int32_t tile_vec;         /* columns per lane (1, 2, 4); 0: the library's choice
                                 (the widest lane that still gives about 1024 tiles
                                 of 16 rows)                                     */
    int32_t tile_rows;        /* rows per tile (multiple of 16); 0: the library's
                                 choice (about four tiles per compute unit).  The
                                 Python helper tiles_for() returns the shapes that
                                 the autotuner measured best on gfx950           */
    int32_t profile;          /* 1: launch blocks of 16 slots back to back without a
                                 graph, every launch stamping its own HIP events
                                 (ot_result.pass_ms, combine_ms)                     */
    int32_t engine;           /* 0 auto: instances of at most OT_RESIDENT_MAX_ELEMS plan
                                 entries run resident (one work-group runs the whole
                                 instance for many iterations per launch), larger ones on
                                 the whole GPU one iteration per launch; 1 always the
                                 whole GPU; 2 resident up to OT_RESIDENT_HARD_MAX_ELEMS.
                                 One work-group handles about one plan entry per cycle, so
                                 the resident path only pays below a few thousand entries.
                                 The choice depends on the instance only, so an instance
                                 takes the same path solo, in a batch or in the server.  */
    int32_t verify_retries;   /* final verifications that may fail (the returned arrays
                                 above tol although the running estimate met it) before
                                 the solve returns OT_NOT_CONVERGED; after a failure the
                                 internal threshold is tightened and iteration continues.
                                 Default 8.                                           */
    int32_t pad0;
} ot_params;

#define OT_RESIDENT_MAX_ELEMS 4096
#define OT_RESIDENT_HARD_MAX_ELEMS (1 << 22)

typedef struct {
    int32_t status;            /* ot_status of this instance                       */
    int32_t returned_average;  /* 1 if the returned iterate is the running average */
    int64_t iterations;        /* accepted PDHG iterations                         */
    int64_t passes;            /* step trials evaluated (accepted + rejected)      */
    int64_t restarts;
    int64_t kernel_passes;     /* streaming passes launched (incl. speculative)    */
    double objective;          /* <C, X> of the returned X                         */
    double dual_objective;     /* f^T u + g^T v                                    */
    double rel_primal, rel_dual, rel_gap, rel_kkt;   /* of the returned triple     */
    double eta, omega;         /* final step size and primal weight                */
    double seconds;            /* wall time of the call                            */
    int64_t mode_passes[7];    /* streaming passes by kind: 0 unused, 1 start-point KKT,
                                  2 step trial, 3 KKT + trial, 4 restart distance,
                                  5 final verification, 6 fold of the current iterate into
                                  the stored average (before a restart to the average or
                                  before returning it)                                 */
    double pass_bytes;         /* algorithmic HBM bytes of those passes (plan, average
                                  and cost streams; partial sums excluded)            */
    double pass_ms;            /* profile mode: summed duration of the pass launches   */
    double combine_ms;         /* profile mode: summed duration of the combine launches*/
    int64_t verify_retries;    /* final verifications that found the returned arrays above
                                  tol (the threshold was tightened and iteration resumed)  */
    double kkt_estimate;       /* running relative-KKT estimate of the returned candidate
                                  when the solver stopped (the verified value is rel_kkt) */
    double estimate_parts[3];  /* its rel_primal, rel_dual, rel_gap                        */
    double estimate_objective; /* its <C, X> (before the plan's storage rounding)          */
    int64_t avg_fold_passes;   /* kinds 2 and 3 that also folded their start iterate and
                                  their trial into the stored running average (the average
                                  is read and written every other pass)                  */
    int64_t trace_len;         /* control records written to ot_problem.trace           */
} ot_result;

/* Fill *prm with the defaults described above (precision OT_PREC_FP32). */
void ot_params_default(ot_params *prm);

/* Device bytes ot_solve needs for this problem when the caller provides the workspace.
 * Returns 0 and sets ot_last_error() for an invalid problem. */
size_t ot_workspace_size(const ot_problem *prob, const ot_params *prm);

/* Solve one instance (Algorithm 2 with the Section 5 enhancements) on the current HIP
 * device.  workspace: nullable device pointer of workspace_bytes >= ot_workspace_size(),
 * 256-byte aligned.  res: nullable.  Returns the instance status. */
ot_status ot_solve(const ot_problem *prob, const ot_params *prm, ot_result *res,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Solve `count` independent instances together: every iteration slot is one launch of the
 * streaming kernel over the tiles of all running instances and one launch of the combine
 * kernel, so instances of uneven m x n share the GPU.  Each instance follows exactly the
 * arithmetic of a solo ot_solve with the same parameters and tile shape (results are
 * bit-identical).  res: array of count results.  Returns OT_OK when every instance
 * converged, otherwise the first non-OK instance status. */
ot_status ot_solve_batch(const ot_problem *probs, int32_t count, const ot_params *prm,
                         ot_result *res, void *stream);

/* ---- solving without allocation ------------------------------------------------------
 *
 * For callers that cannot allocate (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): ot_solve with its whole workspace -- plan buffers,
 * cost, coordinates, vectors, partial sums, control block and the launch tables -- in a
 * static device array of OT_NOALLOC_MAX_BYTES that the library holds on every GPU it runs
 * on until the process ends.  The call allocates nothing (no device, pinned or heap memory,
 * no stream, event or graph): it launches the same kernels as ot_solve directly on
 * `stream` (NULL: the null stream) and returns when the results are in the outputs, which
 * equal ot_solve's for the same problem and parameters bit for bit.  Every call on a GPU
 * uses that GPU's one array, so calls that overlap on one GPU race: serialise them per
 * device.  The array keeps the last call's contents; a call clears what it uses first.
 * ot_params.profile is ignored.  OT_ERR_OOM (with the size in ot_last_error()) when the
 * problem needs more than OT_NOALLOC_MAX_BYTES; otherwise the statuses of ot_solve. */
#define OT_NOALLOC_MAX_BYTES ((size_t)128 << 20)
ot_status ot_solve_noalloc(const ot_problem *prob, const ot_params *prm, ot_result *res,
                           void *stream);

/* ---- rounding to a feasible plan and the certified bracket ---------------------------
 *
 * Algorithm 3 (Section 3.2; Altschuler et al.'s rounding) maps an approximately feasible
 * plan X to an exactly feasible X_feas: rows scaled by min(f_i/(X1)_i, 1), then columns by
 * min(g_j/(X^T 1)_j, 1), then the rank-one correction err_r err_c^T / ||err_r||_1; Lemma
 * lem:round bounds ||X_feas - X||_1 by 2 (||f - X1||_1 + ||g - X^T 1||_1).  The paper
 * reports every result on the rounded plan (Section 5.1).  With any duals u, the
 * c-transform v_j = min_i (C_ij - u_i) makes (u, v) dual feasible, so
 *     lower = f^T u + g^T v  <=  OPT  <=  upper = <C, X_feas>   (weak duality).
 * Everything is computed in FP64 with the FP64 cost (stored or regenerated). */
typedef struct {
    double upper;            /* <C, X_feas>, the cost of a feasible plan (>= OPT)        */
    double lower;            /* f^T u + g^T v with v the c-transform of u (<= OPT)       */
    double l1_change;        /* ||X_feas - X||_1                                         */
    double marginal_l1;      /* ||f - X1||_1 + ||g - X^T 1||_1 of the input plan          */
    double feas_violation;   /* max_i |(X_feas 1)_i - f_i|, max_j |(X_feas^T 1)_j - g_j|  */
} ot_bracket;

/* Round the plan X of `prob` (m x n, row stride n, FP32 when precision is OT_PREC_FP32,
 * else FP64; host or device) and bound the optimal value with the duals u (length m, FP64,
 * host or device).  X_feas: nullable m x n FP64 output (host or device).  Uses its own
 * device workspace (about five FP64 m x n buffers), released before returning;
 * synchronous on `stream` (nullable).  OT_ERR_INVALID for a null argument, an unknown
 * precision or an invalid problem. */
ot_status ot_round(const ot_problem *prob, int32_t precision, const void *X, const double *u,
                   double *X_feas, ot_bracket *out, void *stream);

/* ---- serving: continuous batching of arriving solves --------------------------------
 *
 * A server owns one device arena of hbm_budget_bytes and a scheduler thread.  Submitted
 * problems wait in a FIFO queue; the scheduler admits the head of the queue whenever it
 * has a free slot (at most max_active instances) and its workspace fits in the arena, so
 * requests that arrive while others run join the running set between graph launches of
 * iteration slots.  Every slot of a launch advances all running instances together (one
 * streaming-pass launch per kernel variant and one combine launch), and each instance's
 * arithmetic is exactly that of a solo ot_solve with the same parameters and tile shape,
 * so its result does not depend on the mix.  Iterates stay in device memory from
 * admission to completion; finished instances release their slot and arena space.
 *
 * Callers: one server per device.  ot_server_submit copies the inputs (f, g, costs or
 * coordinates; host or device pointers) before it returns; the output pointers of the
 * problem must stay valid until its completion has been returned by ot_server_poll.
 */
typedef struct ot_server ot_server;

typedef struct {
    size_t hbm_budget_bytes;   /* arena size; a request larger than it is rejected (BUSY) */
    int32_t max_active;        /* running instances at most (>= 1)                       */
    int32_t max_queue;         /* queued requests at most, 0 = unbounded                 */
    double block_ms;           /* target duration of one graph launch, 0 = 2 ms          */
    ot_params params;          /* solver parameters shared by all requests               */
} ot_server_cfg;

typedef struct {
    uint64_t ticket;
    ot_result result;          /* result.status is the request's status                  */
    double t_submit, t_admit, t_done;   /* seconds since the server was created          */
} ot_completion;

/* Create a server on the current HIP device; starts its scheduler thread. */
ot_status ot_server_create(const ot_server_cfg *cfg, ot_server **out);

/* Queue a problem; *ticket identifies its completion.  OT_ERR_BUSY if the queue is full or
 * the problem can never fit in the arena; OT_ERR_INVALID for an invalid problem. */
ot_status ot_server_submit(ot_server *srv, const ot_problem *prob, uint64_t *ticket);

/* Move up to max finished requests into out (completion order); *n_out is the count. */
ot_status ot_server_poll(ot_server *srv, ot_completion *out, int32_t max, int32_t *n_out);

/* Block until every submitted request has completed or timeout_s elapsed (<= 0: no
 * limit); OT_NOT_CONVERGED on timeout. */
ot_status ot_server_drain(ot_server *srv, double timeout_s);

/* Counters: submitted, admitted, completed, currently running, queued, arena bytes in use,
 * graph launches, and the largest number of instances that ran together. */
typedef struct {
    int64_t submitted, admitted, completed, running, queued;
    int64_t arena_used, arena_peak, launches, max_running;
} ot_server_stats;
ot_status ot_server_get_stats(ot_server *srv, ot_server_stats *out);

/* Stop the scheduler (running and queued requests are abandoned) and free everything. */
ot_status ot_server_destroy(ot_server *srv);

/* Message for the last failing call on this thread ("" if none). */
const char *ot_last_error(void);

/* Library version string. */
const char *ot_version(void);

#ifdef __cplusplus
}
#endif

#endif /* PDOT_H */
