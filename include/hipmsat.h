/*
 * hipmsat.h -- C ABI of the MI355X (gfx950) solve loop for the gradient-based
 * MaxSAT method of Hosny & Reda, "torchmSAT: A GPU-Accelerated Approximation To
 * The Maximum Satisfiability Problem" (arXiv 2402.03640).
 *
 * The method (Section 4): each Boolean variable is relaxed to a real x_i; the
 * clause scores are f = tanh(x) W with W[i][j] = +1 / -1 when x_i / not-x_i is
 * a literal of clause j; a clause is unsatisfied when every literal is false
 * under the rounding a_i = [x_i > 0]; the loss is the mean over all m clauses
 * of f_j^2 taken over the unsatisfied clauses; its gradient is
 * back-propagated to x and an optimizer step follows.  Algorithm 1 repeats
 * this while tracking the assignment with the fewest unsatisfied clauses.
 *
 * Conventions
 *  - Every function returns hms_status: HMS_OK (0) or a negative error code;
 *    hms_last_error() then holds a message (thread-local, valid until the next
 *    call on the same thread).  No C++ exception crosses this boundary.
 *  - "HOST" pointers are ordinary CPU memory; "DEVICE" pointers are HIP device
 *    memory on the current device.  Relaxed values are FP32, laid out [n][R]:
 *    variable-major with the restart index innermost, in the caller's original
 *    (0-based) variable order.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued on
 *    it; functions that return host results synchronise it before returning.
 *  - An hms_cnf handle is immutable after loading; several solves may use one
 *    handle at once (each call allocates its own state).  No call keeps a
 *    caller pointer after it returns.
 *  - Calls may run on several host threads at once, each on its own stream;
 *    their results are the same as when run one after the other.
 */
#ifndef HIPMSAT_H
#define HIPMSAT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t hms_status;

#define HMS_OK 0
#define HMS_ERR_ARG (-1)           /* invalid argument (null pointer, bad size, bad enum) */
#define HMS_ERR_PARSE (-2)         /* malformed CNF: last clause not 0-terminated, bad DIMACS */
#define HMS_ERR_LITERAL_RANGE (-3) /* literal |l| > n_vars */
#define HMS_ERR_DEVICE (-4)        /* no usable gfx950 device or a HIP runtime error */
#define HMS_ERR_NOMEM (-5)         /* host or device allocation failed */
#define HMS_ERR_NONFINITE (-6)     /* a relaxed value or the loss became NaN/Inf */
#define HMS_ERR_CANCELLED (-7)     /* the caller's cancel flag stopped the solve (result filled) */
#define HMS_ERR_IO (-8)            /* file could not be read */
#define HMS_ERR_TOO_LARGE (-9)     /* instance exceeds the 31-bit index space */

#define HMS_ADAM 0       /* Adam, PyTorch 1.10 semantics (Section 5 "Setup": Adam, lr 1e-4) */
#define HMS_SGD 1        /* x <- x - lr g (the Section 4 worked example, lr 0.1) */

#define HMS_LOSS_UNSAT 0 /* loss over the unsatisfied clauses (Section 4, Algorithm 1) */
#define HMS_LOSS_ALL 1   /* loss over every clause (reproduces the worked example's step) */

typedef struct hms_cnf hms_cnf; /* opaque: canonical instance, host plan and device structure */

typedef struct {
    int32_t n_vars;         /* variables as declared */
    int32_t n_clauses;      /* clauses as given, m (the loss divides by m) */
    int64_t n_lits;         /* nonzero literals as given */
    int64_t nnz;            /* nonzero entries of W after canonicalisation */
    int32_t n_empty;        /* empty clauses (always unsatisfied) */
    int32_t n_taut;         /* clauses with a complementary pair (always satisfied) */
    int32_t n_active;       /* variables with a nonzero W entry */
    int32_t n_heavy;        /* variables whose transposed row is split into segments */
    int64_t struct_bytes;   /* device bytes held by the handle */
    int64_t state_bytes_r1; /* device bytes of solver state per restart */
    int32_t weighted;       /* 1 if the clauses carry weights */
    int64_t total_weight;   /* total clause weight (n_clauses without weights) */
    int32_t plan_threads;   /* host threads the plan build used: the host's hardware threads (at most
                               16) shared by the loads running at once, at most one per 2^16 literals,
                               or the count the HIPMSAT_PLAN_THREADS variable sets (shared the same
                               way); the plan does not depend on it */
    int64_t slot_bytes;     /* device bytes a one-restart solve under a slot schedule holds beside
                               its state (one FP32 per variable-side entry; 0: no slot schedule) */
} hms_cnf_info;

/*
 * Load a CNF given DIMACS-style: `lits` (HOST, n_lits int32) holds the clauses
 * one after the other, literals as signed 1-based variable indices, each clause
 * ended by 0 (Section 2, CNF of equation 1; Section 4 builds W from it).
 * Repeated literals count once; a clause holding v and not-v is always
 * satisfied and its pair contributes 0 to the score; an empty clause is always
 * unsatisfied.  n_vars = 0 with no clauses is valid.
 * Errors: HMS_ERR_PARSE (last clause not terminated), HMS_ERR_LITERAL_RANGE
 * (|l| > n_vars), HMS_ERR_ARG, HMS_ERR_DEVICE, HMS_ERR_NOMEM.
 * On success *out owns host and device memory until hms_free_cnf.  The upload
 * is ordered on `stream` and complete when the call returns.
 */
hms_status hms_load_cnf(int32_t n_vars, const int32_t* lits, int64_t n_lits, void* stream,
                        hms_cnf** out);

/*
 * Weighted MaxSAT (weighted partial CNF is defined in Section 2; Section 6
 * leaves weights to future work, so the loss is our reading):
 * clause j has weight weights[j] > 0 (HOST, one per clause, at most 2^53,
 * total below 2^63).  The cost of an assignment is the total weight of its
 * unsatisfied clauses, the loss is (1/m) sum_j mu_j w_j f_j^2, and the best
 * cost starts at the total weight.  Hard clauses (partial MaxSAT) are clauses
 * whose weight exceeds the total soft weight.  With weights all 1 every
 * result equals the unweighted one bit for bit.  Otherwise as hms_load_cnf;
 * HMS_ERR_ARG for a weight out of range.
 */
hms_status hms_load_wcnf(int32_t n_vars, const int32_t* lits, int64_t n_lits, const int64_t* weights, void* stream,
                         hms_cnf** out);

/*
 * Same, from a DIMACS file (the CNF of Section 2, equation 1: a conjunction
 * of clauses, each a disjunction of literals x_i or not x_i; weighted
 * partial CNF as defined in Section 2).  "c" lines are comments.  Accepted
 * forms: "p cnf n m" (unweighted); "p wcnf n m top" (each clause led by its
 * weight, kept as given); no header, each clause led by its weight or by "h"
 * (hard: weight 1 + the total soft weight).  Clauses end with 0 and may span
 * lines.  `path` is a HOST string read once; nothing is kept after the call.
 * Errors: HMS_ERR_IO (unreadable file), HMS_ERR_PARSE (bad token, header or
 * an unterminated clause), HMS_ERR_LITERAL_RANGE, HMS_ERR_TOO_LARGE,
 * HMS_ERR_ARG, HMS_ERR_DEVICE, HMS_ERR_NOMEM.  On success *out is as for
 * hms_load_cnf.
 */
hms_status hms_load_cnf_dimacs(const char* path, void* stream, hms_cnf** out);

/* Sizes of a loaded instance. */
hms_status hms_cnf_info_get(const hms_cnf* cnf, hms_cnf_info* out);

/* Release a handle (NULL is allowed).  Not while a call on it is running. */
void hms_free_cnf(hms_cnf* cnf);

/*
 * The state Algorithm 1 carries from one iteration to the next (Section 4,
 * "The Solving Process"): the relaxed values, the Adam moments, the number of
 * iterations taken, and the best rounded iterate so far with its cost and
 * step (the "save and output" of each improvement).  A solve can start from
 * one (hms_solve_params.resume) and hand one back (hms_solve_result.state), so
 * a long solve can be cut into pieces: T1 steps, then T2 more from the state
 * they left, equal T1 + T2 steps bit for bit when T1 is a multiple of
 * eval_every (otherwise the extra count of the T1-th iterate can only lower
 * the best).  All arrays are caller-owned; n and R are the instance's and the
 * solve's.
 */
typedef struct {
    float* x;                 /* DEVICE [n][R] relaxed values (caller variable order) */
    float* m;                 /* DEVICE [n][R] Adam first moments (ignored with HMS_SGD) */
    float* v;                 /* DEVICE [n][R] Adam second moments (ignored with HMS_SGD) */
    uint8_t* best_assignment; /* DEVICE [R][n] each restart's best rounded iterate (0/1 bytes) */
    int64_t* best;            /* HOST [R] each restart's best cost */
    int32_t* best_step;       /* HOST [R] the iteration of that iterate (-1: the start, not beaten) */
    int32_t step;             /* iterations taken (the Adam step count; >= 0) */
    int32_t pad;
} hms_solve_state;

typedef struct {
    int32_t steps;       /* optimizer steps T (>= 0) */
    int32_t restarts;    /* R independent relaxed points solved together (>= 1) */
    int32_t eval_every;  /* K: round and count every K steps, and at x_T (>= 1) */
    int32_t optimizer;   /* HMS_ADAM or HMS_SGD */
    uint64_t seed;       /* restart r starts from the SplitMix64 stream seeded seed + r */
    float lr, beta1, beta2, eps; /* Adam: PyTorch defaults 0.9 / 0.999 / 1e-8 */
    int32_t loss_mode;   /* HMS_LOSS_UNSAT or HMS_LOSS_ALL */
    int32_t schedule;    /* 0 = automatic; else table index | rows-per-unit << 8
                            | backward rows-per-unit << 16 (0 = the same; see hms_tune) */
    int32_t use_graph;   /* 1 = replay the step body as a HIP graph, 0 = direct launches */
    int32_t autotune;    /* 1 = with schedule 0, time the candidate schedules once per handle,
                            restart count, optimizer and loss mode, and keep the fastest
                            (small instances skip the timing); 0 = take the resident solver
                            (255) when the state fits it and nnz <= 2^15 (2^16 with K = 1),
                            else a fixed tiled schedule for R */
    double time_limit_s; /* > 0: stop at a K-step boundary once exceeded (not reproducible) */
    const float* x0;     /* DEVICE [n][R] initial values, or NULL for SplitMix64 U(-1,1) */
    void* stream;        /* hipStream_t */
    const volatile int32_t* cancel; /* HOST flag or NULL: once nonzero (set by another thread), the
                            solve stops at the next K-step boundary, fills the result with the
                            best so far and returns HMS_ERR_CANCELLED */
    const hms_solve_state* resume; /* NULL: start from x0 or the seed; else continue from this
                            state (x0 must then be NULL): iteration numbers, the counting
                            period and the Adam step count go on from resume->step, and the
                            best so far is kept unless strictly beaten.  Read only. */
} hms_solve_params;

/* One counted iterate of one restart (the trajectory of hms_solve_result). */
typedef struct {
    int32_t step;             /* iteration t of the iterate */
    int32_t pad;
    int64_t cost;             /* unsatisfied clauses (their total weight) of its rounding */
    double loss;              /* the loss at it */
} hms_trace_point;

typedef struct {
    int64_t best_cost;        /* fewest unsatisfied clauses seen over all restarts */
    int32_t best_restart;     /* restart that found it (lowest index on ties) */
    int32_t best_step;        /* step at which it was found (-1: the initial point never beaten) */
    int32_t steps_done;       /* steps taken (< steps only with a time limit or a cancel) */
    int32_t schedule;         /* kernel schedule that ran */
    double final_loss;        /* loss at x_T of best_restart */
    uint8_t* best_assignment; /* caller HOST buffer of n bytes (0/1), or NULL */
    int64_t* restart_best;    /* caller HOST [R] per-restart best cost, or NULL */
    int32_t* restart_step;    /* caller HOST [R] per-restart best step, or NULL */
    double* restart_loss;     /* caller HOST [R] loss at x_T, or NULL */
    float* x_final;           /* caller DEVICE [n][R] receives x_T, or NULL */
    double device_ms;         /* device time of the step loop (HIP events) */
    hms_solve_state* state;   /* NULL, or a state whose arrays receive the state after the last
                                 step taken (also on HMS_ERR_CANCELLED and with a time limit), to
                                 pass as a later solve's resume; m and v are written with Adam */
    hms_trace_point* trace;   /* NULL, or a caller HOST [trace_cap][R] array: the trajectory of the
                                 solve, one row of R points per counted iterate (t a multiple of K,
                                 and the last), kept on the device in a ring of trace_cap rows and
                                 read at the end; it receives the last trace_cap rows, oldest first */
    int32_t trace_cap;        /* rows of trace (>= 1 when trace is given) */
    int32_t trace_len;        /* out: rows written (the counts taken, at most trace_cap) */
} hms_solve_result;

/* Fill *p with the defaults: T = 1000, R = 1, K = 1, Adam lr 1e-4, UNSAT loss,
 * automatic schedule with autotuning, graphs on, no time limit, seed 0, null
 * stream. */
void hms_solve_params_default(hms_solve_params* p);

/*
 * Algorithm 1 (Section 4 "The Solving Process"), R restarts at once.
 * Initial best cost = m (all clauses); x^0 from `x0` or SplitMix64 U(-1,1).
 * For t = 0..T-1: when t % K == 0 the rounded iterate is counted and kept if
 * strictly better; the loss gradient at x_t (mask from the same iterate) takes
 * one optimizer step.  x_T is counted too.  Synchronous: returns when `result`
 * is filled.  Results are bitwise reproducible for equal inputs and do not
 * depend on the schedule or on R (restart r of a solve with seed s equals the
 * single-restart solve with seed s + r), except `final_loss` rounding.
 * With params->resume the loop continues from that state instead: t runs
 * from resume->step to resume->step + T, counting when t % K == 0 and at the
 * last iterate, Adam step t + 1, best_step in that numbering.  With
 * result->state the state after the last step taken is written there; with
 * result->trace the (step, cost, loss) of every counted iterate.
 * Errors: HMS_ERR_ARG (also a null array of a given state, x0 beside
 * resume, or resume->step + steps past 2^31 - 1), HMS_ERR_DEVICE,
 * HMS_ERR_NOMEM; HMS_ERR_NONFINITE when the final loss is not finite (the
 * result is still filled).
 */
hms_status hms_solve(const hms_cnf* cnf, const hms_solve_params* params, hms_solve_result* result);

/*
 * Measurement helper for the benchmark: initialises a solve exactly as
 * hms_solve does with `params` (steps and eval_every ignored), then times on
 * params->stream with HIP events `iters` back-to-back launches of the forward
 * kernel (scores, mask, adjoint), then of the backward kernels (transposed sums
 * and fused optimizer step), then of whole steps.  Outputs are the average
 * milliseconds per launch (any may be NULL).  The relaxed state keeps moving
 * during the measurement; nothing is returned from it.
 */
hms_status hms_time_kernels(const hms_cnf* cnf, const hms_solve_params* params, int32_t iters,
                            double* fwd_ms, double* bwd_ms, double* step_ms);

/*
 * Batched solve of `count` instances (Algorithm 1 for each, as hms_solve):
 * cnfs[i] with params[i] into results[i] (statuses[i], may be NULL, receives each
 * instance's status).  Instances that request the resident solver, or leave
 * the schedule automatic and fit it with at most 2^15 nonzeros (2^16 when
 * eval_every is 1), share launches, one workgroup per (instance, restart).  The others are grouped by restarts,
 * steps, eval_every, optimizer, loss mode and requested schedule: each step of
 * a group is one launch per kernel over all its instances (a work queue of
 * (instance, work unit) items, replayed as a HIP graph), with the schedule of
 * its largest instance.  A group of one, a solve with a time limit or a
 * cancel flag, and a solve that resumes, returns its state or records its
 * trajectory run as hms_solve.  All work goes on params[0].stream.  Each result is bitwise the
 * one hms_solve gives for that instance alone (restart_loss and final_loss may
 * differ in the last bits when the schedule does).  Returns the first error.
 */
hms_status hms_solve_batch(const hms_cnf* const* cnfs, const hms_solve_params* params, int32_t count,
                           hms_solve_result* results, hms_status* statuses);

/*
 * Schedule autotuner: for every kernel schedule that can run
 * params->restarts restarts, times the forward and the backward pass at each
 * rows-per-unit value (`iters` launches each, HIP events on params->stream)
 * and pairs the fastest of each; then times whole steps of those pairs and
 * of the resident solver, and records the fastest for this handle (and its
 * size class); later solves with schedule 0 use it.  The choice changes speed only: results are bitwise the same under
 * every schedule.  Outputs the chosen schedule id and its time per step.
 */
hms_status hms_tune(const hms_cnf* cnf, const hms_solve_params* params, int32_t iters, int32_t* schedule,
                    double* step_ms);

/*
 * The schedule ids hms_tune times for `restarts` restarts and `loss_mode`
 * (host only, no device needed): up to `cap` ids into `codes` (HOST), the
 * number of candidates into *count (also when it exceeds cap).  The resident
 * schedule (255), tried as well when an instance fits it, is not listed.
 */
hms_status hms_tune_candidates(int32_t restarts, int32_t loss_mode, int32_t* codes, int32_t cap, int32_t* count);

/*
 * Number of kernel table entries (host only): schedule table indices run
 * from 1 to this count.  Every entry computes the same values; they differ
 * in how lanes, restarts and rows map onto wavefronts, in how many columns
 * of a row one load batch takes and, for the unsat-masked loss, in whether
 * a bitset lets the backward pass skip the adjoints of satisfied clauses or,
 * at one restart, whether the forward pass stores each occurrence's adjoint
 * where the backward pass reads its terms in order (the slot entries, which
 * run their unmasked twin with several restarts or the unmasked loss).
 */
int32_t hms_schedule_count(void);

/*
 * Count the clauses an assignment leaves unsatisfied (Section 4 "Unsatisfiable
 * Cores", with the rounding a_i in {0,1}).  `assignment`: HOST n bytes, nonzero
 * = true.  *unsat receives the count.  Synchronises `stream`.
 */
hms_status hms_evaluate(const hms_cnf* cnf, const uint8_t* assignment, int64_t* unsat, void* stream);

/*
 * One evaluation of the relaxed objective at R points (the parity entry
 * point): the forward pass, loss and backpropagation of one iteration of
 * Algorithm 1, without the optimizer step.  For each restart r:
 *   - scores f = tanh(x_r) W (Section 4, display equation for f);
 *   - unsatisfied clauses of the rounding x_r > 0 (Section 4, "Unsatisfiable
 *     Cores"; Algorithm 1 forward step), counted into unsat[r] (their total
 *     weight for a weighted instance);
 *   - loss[r] = (1/m) sum_j mu_j w_j f_j^2 with mu_j = 1 for the unsatisfied
 *     clauses (HMS_LOSS_UNSAT, Algorithm 1 loss step) or for every clause
 *     (HMS_LOSS_ALL, the Section 4 worked example's loss);
 *   - grad = dL/dx with mu held constant (Algorithm 1 backpropagation step).
 * x: DEVICE [n][R] FP32, caller order, read only.  loss: HOST [R] doubles,
 * unsat: HOST [R] int64, grad: DEVICE [n][R] FP32 (caller-owned; each may be
 * NULL).  The call allocates its own device workspace and releases it in
 * stream order.  Synchronises `stream` when a host output is requested.
 * Errors: HMS_ERR_ARG (null instance or x, R < 1, bad loss mode),
 * HMS_ERR_DEVICE, HMS_ERR_NOMEM, HMS_ERR_TOO_LARGE.
 */
hms_status hms_eval_relaxed(const hms_cnf* cnf, const float* x, int32_t restarts, int32_t loss_mode,
                            double* loss, float* grad, int64_t* unsat, void* stream);

/*
 * For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, hosts that forbid allocation.  The same
 * evaluation as hms_eval_relaxed (bitwise the same loss, gradient and
 * counts), with no allocation and no wait: its workspace is a fixed array of
 * 64 MiB inside the library, one per GPU, which each GPU the library runs on
 * holds until the process ends; loss (DEVICE [R] doubles) and unsat (DEVICE
 * [R] int64) are device outputs like grad (DEVICE [n][R]); each may be NULL.
 * All work is enqueued on `stream`; the outputs are ready when it reaches
 * them.  Every call on one GPU uses that GPU's one array, which keeps the last
 * call's contents (nothing in it needs clearing: each call writes what it
 * reads): calls that overlap on one GPU race, so order them (one stream, or
 * events).  Errors: HMS_ERR_TOO_LARGE when the instance and R need more than
 * the 64 MiB (hms_eval_relaxed has no such limit), and as hms_eval_relaxed.
 */
hms_status hms_eval_relaxed_noalloc(const hms_cnf* cnf, const float* x, int32_t restarts, int32_t loss_mode,
                                    double* loss, float* grad, int64_t* unsat, void* stream);

/*
 * Differentiable pieces of the loss, for autograd frameworks (Section 4: the
 * loss is differentiated through the network by backpropagation).
 * hms_forward: loss[R] (DEVICE doubles) at x (DEVICE [n][R]) and optionally the
 * unsat counts (DEVICE int64 [R]); when `adjoint` is non-NULL it receives the
 * score adjoint dL/df (DEVICE workspace of hms_adjoint_bytes bytes, opaque
 * layout) for a later hms_backward.  The unsat mask is held constant under
 * differentiation (it depends on the rounding only).
 * hms_backward: grad_x (DEVICE [n][R]) = grad_loss[r] * dL_r/dx (grad_loss DEVICE
 * floats [R], or NULL for 1).  With `adjoint` NULL the scores are recomputed
 * from x (checkpoint mode); the gradient is bitwise the same either way.
 * Both are asynchronous on `stream`.
 */
hms_status hms_adjoint_bytes(const hms_cnf* cnf, int32_t restarts, int64_t* bytes);
hms_status hms_forward(const hms_cnf* cnf, const float* x, int32_t restarts, int32_t loss_mode, double* loss,
                       int64_t* unsat, void* adjoint, void* stream);
hms_status hms_backward(const hms_cnf* cnf, const float* x, int32_t restarts, int32_t loss_mode,
                        const void* adjoint, const float* grad_loss, float* grad_x, void* stream);

/* Message of the last failed call on this thread ("" if none). */
const char* hms_last_error(void);

/* Library version string. */
const char* hms_version(void);

/*
 * Host-only view of an instance plan, for tests of the layouts (no device
 * needed).  Builds the plan of the CNF as hms_load_cnf would and copies out
 * the counters and arrays.  The arrays are owned by the view and released by
 * hms_plan_view_free.
 */
typedef struct {
    int32_t n, m, mk, c_tiles, n_act, n_heavy, seg_rows, seg_tiles, v_tiles, n_empty, n_taut;
    int32_t tile_rows, seg_len;      /* rows per tile (64), entries per segment */
    int32_t split_len;               /* longest variable row kept whole; longer ones are split into
                                        ceil(degree / seg_len) interleaved segments */
    int64_t nnz, c_ent_len, v_ent_len;
    const uint32_t* c_tile;          /* [c_tiles][4]: base, len, nreal, flags */
    const uint32_t* c_ent;           /* [c_ent_len] new variable | sign << 31 */
    const int32_t* c_row_orig;       /* [c_tiles * 64] original clause or -1 */
    const uint32_t* v_tile;          /* [v_tiles][4] */
    const uint32_t* v_ent;           /* [v_ent_len] clause row | sign << 31 */
    const int32_t* seg_first;        /* [n_heavy + 1] */
    const int32_t* seg_row;          /* [seg_rows] row of each segment; the identity, since a heavy
                                        variable's segments are consecutive rows in segment order */
    const int32_t* var_old;          /* [n] new -> original */
    const uint32_t* c_slot;          /* [c_ent_len] v_ent index of the same occurrence | sign << 31, or
                                        0xffffffff for padding; entry (c, row) of a tile at
                                        base + row * len + c (row by row); NULL when v_ent_len >= 2^31 */
    void* priv;
} hms_plan_view;

hms_status hms_plan_view_build(int32_t n_vars, const int32_t* lits, int64_t n_lits, hms_plan_view* out);
void hms_plan_view_free(hms_plan_view* view);

/*
 * The occurrence map a loaded instance holds on its device (built there at
 * load, for the slot schedules), copied to `out`: a caller-owned HOST array
 * of `cap` >= c_ent_len entries laid out as hms_plan_view.c_slot (the
 * variable-side entry of each clause-side entry | sign << 31, 0xffffffff for
 * padding), for tests of the layouts.  *len receives c_ent_len, or 0 when the
 * instance has no map (no entries, or 2^31 variable-side entries or more);
 * with out = NULL only *len is set.  Synchronises the instance's device.
 * Errors: HMS_ERR_ARG (null instance or len, cap too small), HMS_ERR_DEVICE.
 */
hms_status hms_cnf_slot_map(const hms_cnf* cnf, uint32_t* out, int64_t cap, int64_t* len);

#ifdef __cplusplus
}
#endif

#endif /* HIPMSAT_H */
