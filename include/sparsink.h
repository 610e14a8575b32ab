/*
 * sparsink.h -- C ABI of the MI355X (gfx950) Spar-Sink library.
 *
 * Spar-Sink (Li, Yu, Li & Meng, "Importance Sparsification for Sinkhorn
 * Algorithm", JMLR 24, 2023) approximates entropic OT (eq. (rot)) and entropic
 * UOT (eq. (ruot)) by running the Sinkhorn scaling loop (Alg. 1 / Alg. 2) on a
 * Poisson-sparsified kernel K~ (eq. (pois)) drawn with the importance
 * probabilities of eq. (pij-ot) / eq. (pij-uot), then reporting the estimate of
 * Alg. 3 / Alg. 4.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Pointers documented "device" must point to memory the current HIP device
 *   can read (hipMalloc'd or torch CUDA tensors).  Pointers documented "host"
 *   are ordinary process memory.  The library never allocates or frees caller
 *   memory: every scratch byte comes from the caller's workspace `ws`, whose
 *   size is given by ss_workspace_size() for the same problem and options.
 * - All device work is enqueued on `stream` (a hipStream_t; NULL is the null
 *   stream).  Calls that fill a host ss_result synchronise that stream before
 *   returning.  Calls with disjoint workspaces may run concurrently from
 *   different host threads.
 * - Return value: 0 = success; > 0 = warning, outputs valid; < 0 = error,
 *   outputs undefined.  No C++ exception crosses this boundary.
 *   ss_status_string() names every code; ss_last_error() returns a text
 *   description of the most recent error on the calling thread.
 * - Inputs are FP64 in every precision mode, so for a given seed the sampled
 *   sparsity pattern is the same in every precision.
 */
#ifndef SPARSINK_H
#define SPARSINK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- codes */
enum {
    SS_OK = 0,
    SS_NOT_CONVERGED = 1,     /* max_iter reached with err > tol; result valid     */
    SS_E_INVALID_ARG = -1,    /* bad size, parameter, or a null required pointer   */
    SS_E_HIP = -2,            /* a HIP runtime call failed                         */
    SS_E_WORKSPACE = -3,      /* ws is NULL, misaligned (256 B) or too small       */
    SS_E_NONFINITE = -4,      /* NaN/Inf appeared in the scalings                  */
    SS_E_EMPTY = -5,          /* empty row/column with empty_policy = FAIL         */
    SS_E_CAPACITY = -6        /* sampled nnz exceeded the workspace capacity       */
};

enum { SS_F64 = 0, SS_F32 = 1, SS_F32_LOG = 2 };                 /* ss_options.precision */
enum { SS_COST_SQEUCLID_MAXNORM = 0, SS_COST_SQEUCLID = 1, SS_COST_WFR = 2,
       SS_COST_EUCLID = 3 }; /* ss_options.cost */
enum { SS_STOP_MARGINAL_L1 = 0, SS_STOP_SCALING_DELTA_L1 = 1 };   /* ss_options.stop_rule */
enum { SS_EMPTY_AUTO = 0, SS_EMPTY_RENORMALIZE = 1, SS_EMPTY_ZERO = 2, SS_EMPTY_FAIL = 3 };

/* ---------------------------------------------------------------- types */

/* One transport problem between mu = sum_i a_i delta_{x_i} and
 * nu = sum_j b_j delta_{y_j} (Sec. 2 notation).  All arrays are device
 * pointers to FP64 data: x is n*d row-major, y is m*d row-major, a has n and
 * b has m non-negative finite entries.  problem_index selects an independent
 * random stream for the Poisson mask (third word of the hash counter). */
typedef struct ss_problem {
    int64_t n, m;
    int32_t d;
    uint32_t problem_index;
    const double *x, *y, *a, *b;
} ss_problem;

/* Solver options.
 * eps    > 0   entropic regularisation (eq. (rot) / eq. (ruot)).
 * lambda > 0   KL relaxation weight of eq. (ruot); +INFINITY selects OT.
 * s      > 0   subsample budget of eq. (pois): p*_ij = min(1, s p_ij).
 * tol   >= 0   stop at the first iterate t with err(t) <= tol.
 * seed         64-bit key of the counter-based hash (Philox4x32-10).
 * max_iter >= 1 cap on Sinkhorn iterations.
 * precision    SS_F64: FP64 values and scalings.
 *              SS_F32: FP32 values, FP32 scalings, FP32 accumulation in the
 *                      sparse products; residual, stop test and estimate FP64.
 *              SS_F32_LOG: log-domain iteration (appendix, proof of Thm. 3):
 *                      FP32 log-values log K~_ij, FP64 potentials, stabilised
 *                      log-sum-exp with FP32 exponentials.
 * cost         SS_COST_SQEUCLID_MAXNORM: C = |x-y|^2 / max |x-y|^2.
 *              SS_COST_SQEUCLID:         C = |x-y|^2.
 *              SS_COST_EUCLID:           C = |x-y| (the Euclidean distance the
 *                      generative-modelling section names between samples);
 *                      OT sampling only (lambda = +INFINITY): spar_sink_ot,
 *                      spar_sink_ot_noalloc, ss_sample and the divergence.
 *              SS_COST_WFR: the Wasserstein-Fisher-Rao cost of the UOT
 *                      background section, C = -log cos_+^2(|x-y| / (2 eta)),
 *                      evaluated as -2 log cos(|x-y| * (1 / (2 eta))) and
 *                      +infinity (K = 0, never sampled) where that argument
 *                      is >= pi/2.  Sparse solvers need finite lambda (the
 *                      UOT probability vanishes with K) and shrink = 0;
 *                      batches and spar_ibp reject it.
 * stop_rule    SS_STOP_MARGINAL_L1: err(t) = L1 marginal error of (u^t, v^t) on
 *              the iterated kernel (for UOT the fixed-point residual
 *              sum|u^(1/th) K~v - a| + sum|v^(1/th) K~'u - b|, th = lam/(lam+eps)).
 *              SS_STOP_SCALING_DELTA_L1: |u^t-u^(t-1)|_1 + |v^t-v^(t-1)|_1 (Alg. 1/2).
 * empty_policy rows/columns of K~ with no entry: AUTO = RENORMALIZE for OT
 *              (a, b rescaled to mass 1 on the non-empty support), ZERO for UOT
 *              (u_i = 0, the sparse UOT optimum); FAIL returns SS_E_EMPTY.
 * block_threads  sparse-product schedule: threads per block of the iteration
 *              kernel (each block owns block_threads/4 lines and sweeps the
 *              gathered vector through LDS in 128 KB (1024) or 32 KB (256)
 *              slices); 0 = automatic, else 256 or 1024.
 * graph_iters  iterations per captured HIP graph; 0 = automatic, < 0 = plain
 *              launches.
 * init_log_u, init_log_v  optional device FP64 warm start (log u^0, log v^0).
 * u_out, v_out optional device FP64 outputs: the returned scalings u^t, v^t.
 * err_hist     optional device FP64 array of max_iter entries: err(t) for
 *              t = 1..iters (entries past iters untouched).
 * eta          > 0, the WFR cost's length scale (ignored by the other costs).
 * shrink       g in [0, 1]: shrinkage toward uniform sampling (Sec. 4),
 *              p_ij = (1 - g) p_ij + g / (nm) in place of eq. (pij-ot) /
 *              eq. (pij-uot); 0 is Spar-Sink, 1 is Rand-Sink (Sec. 5, uniform
 *              probabilities s / (nm)).  Only the sampling changes: the
 *              sketch's values stay K_ij / p*_ij.  Batches need 0. */
typedef struct ss_options {
    double eps, lambda, s, tol;
    uint64_t seed;
    int32_t max_iter, precision, cost, stop_rule, empty_policy;
    int32_t block_threads, graph_iters, reserved0;
    const double *init_log_u, *init_log_v;
    double *u_out, *v_out, *err_hist;
    double shrink, eta;
} ss_options;

/* Result of a solve (host struct).
 * estimate    Alg. 3: <T~,C> - eps H(T~);  Alg. 4 adds lam KL(T~1|a) + lam KL(T~'1|b).
 * transport   <T~, C>.       neg_entropy  sum T~ (log T~ - 1) = -H(T~).
 * kl_a, kl_b  KL terms (UOT; 0 for OT).
 * sparse_objective  the sparse problem's own value <T~, C~> - eps H(T~) (+ KLs),
 *             C~ = -eps log K~ (appendix, proof of Thm. 3).
 * marginal_err err(iters) under the chosen stop rule.
 * cmax        max_ij |x_i - y_j|^2.   z_norm  UOT normaliser sum q_ij (0 for OT).
 * dropped_mass_a/b  mass of a / b on empty rows / columns.
 * nnz, empty_rows, empty_cols  size of K~ and its empty lines (with a_i>0 / b_j>0).
 * iters       t of the returned iterate.   status  same as the return value.
 * t_*_ms      stage times measured with HIP events on `stream`.
 * warm_start  the start given by init_log_u / init_log_v: -1 none given;
 *             1 used; 0 (spar_sink_batched only) judged worse than the plain
 *             start u = v = 1 and replaced by it (see spar_sink_batched). */
typedef struct ss_result {
    double estimate, transport, neg_entropy, kl_a, kl_b, sparse_objective;
    double marginal_err, cmax, z_norm, dropped_mass_a, dropped_mass_b;
    int64_t nnz, empty_rows, empty_cols;
    int32_t iters, status;
    float t_prep_ms, t_sample_ms, t_iter_ms, t_obj_ms;
    int32_t warm_start, reserved;
} ss_result;

/* Caller-allocated device arrays receiving the sparse sketch (ss_sample).
 * Any pointer may be NULL to skip that output.  `capacity` is the number of
 * entries available in col_idx/val/row_idx/val_t.  Value arrays hold FP64
 * (SS_F64), FP32 (SS_F32) or FP32 log K~ (SS_F32_LOG) entries.
 * mask:   n * ceil(m/64) words, bit (j & 63) of word j >> 6 of row i set iff
 *         entry (i, j) is kept.
 * row_ptr (n+1), col_idx (ascending within a row), val        -- CSR of K~.
 * col_ptr (m+1), row_idx (ascending within a column), val_t   -- CSC of K~.
 * row_fac (n), col_fac (m): OT: alpha_i = s sqrt(a_i) / (S_a S_b) and sqrt(b_j),
 *         so p*_ij = min(1, alpha_i * col_fac_j); UOT: th_u log a_i, th_u log b_j.
 * z_in (host, input): UOT only; 0 = the library computes the normaliser
 *         Z = sum_ij q_ij of eq. (pij-uot) itself; > 0 = this value is used as Z
 *         (the parity surface: given the same Z, every keep decision and
 *         stored value is a fixed sequence of IEEE operations, so an
 *         independent implementation of the same definitions reproduces the
 *         mask, CSR and CSC bit for bit).  Ignored for OT.
 * On return nnz, cmax and z_norm are filled (host fields). */
typedef struct ss_sparse {
    uint64_t *mask;
    int64_t *row_ptr;
    int32_t *col_idx;
    void *val;
    int64_t *col_ptr;
    int32_t *row_idx;
    void *val_t;
    double *row_fac, *col_fac;
    int64_t capacity;
    int64_t nnz;
    double cmax, z_norm;
    double z_in;
} ss_sparse;

/* ---------------------------------------------------------------- calls */

/* Workspace bytes needed by every call below for this problem and options
 * (the maximum over them).  Host-only; touches no device memory. */
int ss_workspace_size(const ss_problem *problem, const ss_options *opts, size_t *bytes);

/* Steps 1 of Alg. 3/4: sampling probabilities (eq. (pij-ot) or (pij-uot)),
 * Poisson mask (eq. (pois)) from the counter hash, CSR and CSC of K~ = K/p*.
 * Copies the requested pieces into `out` and synchronises `stream`. */
int ss_sample(const ss_problem *problem, const ss_options *opts, ss_sparse *out,
              void *ws, size_t ws_bytes, void *stream);

/* Alg. 3 (Spar-Sink for OT).  Requires lambda = +INFINITY. */
int spar_sink_ot(const ss_problem *problem, const ss_options *opts, void *ws,
                 size_t ws_bytes, void *stream, ss_result *result);

/* Alg. 4 (Spar-Sink for UOT).  Requires finite lambda > 0. */
int spar_sink_uot(const ss_problem *problem, const ss_options *opts, void *ws,
                  size_t ws_bytes, void *stream, ss_result *result);

/* Bytes of the static scratch array behind spar_sink_ot_noalloc (per GPU). */
#define SS_NOALLOC_SCRATCH_BYTES (32u << 20)

/* spar_sink_ot without allocation, for callers that cannot allocate device
 * memory (code under stream capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as spar_sink_ot,
 * minus the workspace: scratch is a static device array of
 * SS_NOALLOC_SCRATCH_BYTES that each GPU holds from the first call there
 * until the process ends.  The call allocates no device or pinned host
 * memory and creates no stream, event or graph: the loop runs as plain
 * launches on `stream` (which must belong to the current device) and the
 * t_*_ms fields read 0.  A problem whose ss_workspace_size exceeds
 * SS_NOALLOC_SCRATCH_BYTES is rejected with SS_E_WORKSPACE (n = m = 4096 at
 * s = 8 n ln n in FP64 fits).  Every call on one GPU shares that GPU's
 * array and leaves its contents behind; calls that overlap on one GPU
 * (other threads, other streams) race and must be serialised by the
 * caller. */
int spar_sink_ot_noalloc(const ss_problem *problem, const ss_options *opts, void *stream,
                         ss_result *result);

/* Alg. 1 (lambda = +INFINITY) or Alg. 2 on the full kernel K = exp(-C/eps),
 * recomputed from the coordinates in every half-step (never stored).  Same
 * options, stop rules and estimate as the sparse solvers (nnz = n*m). */
int dense_sinkhorn(const ss_problem *problem, const ss_options *opts, void *ws,
                   size_t ws_bytes, void *stream, ss_result *result);

/* Measurement hook for the memory-bound iteration kernel.  Samples K~ like
 * the matching solver (OT if lambda = +INFINITY, else UOT), then runs exactly
 * `iters` Sinkhorn iterations (even, >= 2; tol ignored, every launch does
 * work) as one captured HIP graph: one warm-up replay, one replay between two
 * HIP events on `stream`.  *ms_per_launch (host) receives the mean duration of
 * one iteration-kernel launch (two launches per iteration: the K~ v product
 * with the u-update, then the K~' u product with the v-update). */
int ss_time_iterations(const ss_problem *problem, const ss_options *opts, void *ws,
                       size_t ws_bytes, void *stream, int32_t iters, double *ms_per_launch);

/* ------------------------------------------------------------------------
 * Batches of independent OT problems (Alg. 3 applied to each problem, with
 * the probabilities of Sec. 3.1 eq. (pij-ot) and the subsampling of eq.
 * (pois)).  All problems share d and the options; sizes and budgets differ.
 *
 * count          number of problems, >= 1.
 * d              point dimension, 1..64.
 * n, m           host arrays [count]: points of x and of y per problem,
 *                each in 1..SS_BATCH_MAX_SIDE.
 * s              host array [count]: subsample budget s_k > 0 per problem.
 * problem_index  host array [count] or NULL (then problem k uses k): third
 *                word of the hash counter, so problem k samples exactly the
 *                mask spar_sink_ot would sample with that problem_index.
 * x, y, a, b     device FP64 arrays, the problems concatenated in order:
 *                x is sum(n) x d row-major, y sum(m) x d, a sum(n), b sum(m).
 * Options: lambda must be +INFINITY; precision SS_F64 or SS_F32; stop rule
 * SS_STOP_MARGINAL_L1; empty_policy AUTO (= RENORMALIZE), RENORMALIZE or
 * ZERO (FAIL is rejected for batches); s, block_threads and graph_iters are
 * ignored;
 * init_log_u / init_log_v (warm start) and u_out / v_out are device FP64
 * arrays of sum(n) / sum(m) entries, concatenated like a and b; err_hist
 * must be NULL. */
#define SS_BATCH_MAX_SIDE 4096

typedef struct ss_batch {
    int32_t count;
    int32_t d;
    const int64_t *n, *m;
    const double *s;
    const uint32_t *problem_index;
    const double *x, *y, *a, *b;
} ss_batch;

/* Schedule of the batched iteration kernel: each line (row or column) of a
 * problem is reduced by `lanes_per_line` lanes (4, 8, 16 or 32) of a block of
 * `block_threads` threads (256, 512 or 1024); one block solves one problem at
 * a time, taking problems largest-first from a device queue. */
typedef struct ss_schedule {
    int32_t lanes_per_line;
    int32_t block_threads;
} ss_schedule;

/* Workspace bytes for spar_sink_batched / ss_autotune_batched. */
int ss_batch_workspace_size(const ss_batch *batch, const ss_options *opts, size_t *bytes);

/* Solves every problem of the batch on `stream`: one launch per sampling
 * stage over all problems, one persistent iteration launch in which every
 * problem runs Alg. 1 to its own tolerance, one objective launch; the device
 * part is captured in a hipGraph and replayed once.  With max_iter > 64 the
 * persistent launch first runs at most 64 iterations; if one or two problems
 * are then still above tol, each continues on the single-problem solver
 * (spar_sink_ot's path, the same sketch) from its iterate for the remaining
 * max_iter - 64 iterations (its outs[k] is then that solve's result with
 * iters counted from the start); with more such problems the persistent
 * launch is run again from the start to max_iter.  A warm start
 * (opts->init_log_u / init_log_v, e.g. from ss_warmstart_predict; zero-init
 * Sinkhorn is its fallback) is judged per problem in its first u-update
 * against the plain start u = v = 1: it is kept only when every start value
 * and its u^1 are finite and its L1 row marginal error sum |u0 (K~v0) - a| is
 * no larger than the plain start's sum |K~1 - a|; otherwise the problem
 * continues from the plain start and its iterates are those of a solve
 * without a warm start (outs[k].warm_start = 0).  `schedule` NULL uses 8
 * lanes per line and 1024 threads (the schedule ss_autotune_batched picks
 * on MI355X for batches of a few hundred problems); the library keeps no
 * tuning state, so a caller who wants tuning runs ss_autotune_batched once
 * and passes its result.  outs: host array [count]; each entry
 * is filled as by spar_sink_ot (z_norm 0; stage times are those of the whole
 * batch).  Returns SS_OK when every problem converged, SS_NOT_CONVERGED when
 * some did not (see outs[k].status), or an error code for the whole batch. */
int spar_sink_batched(const ss_batch *batch, const ss_options *opts, const ss_schedule *schedule,
                      void *ws, size_t ws_bytes, void *stream, ss_result *outs);

/* Project autotuner: samples the batch once, then times the iteration kernel
 * (16 iterations, every problem active) under each candidate schedule with
 * HIP events and returns the fastest in *best.  cand_ms (host, may be NULL)
 * receives up to *ncand times in the order lanes_per_line in {4, 8, 16, 32}
 * major, block_threads in {256, 512, 1024} minor; *ncand is set to the
 * number of candidates (12). */
int ss_autotune_batched(const ss_batch *batch, const ss_options *opts, void *ws, size_t ws_bytes,
                        void *stream, ss_schedule *best, float *cand_ms, int32_t *ncand);

/* ------------------------------------------------------------------------
 * Learned warm start: a DeepSets network (hidden width 256, d = 3) that
 * predicts log u^0 and log v^0 for every problem of a batch.  Points enter in
 * kernel units: centred on the mean of all points of their problem and
 * divided by sqrt(eps C_s), C_s = max |x_i - y_j|^2 for SS_COST_SQEUCLID_MAXNORM
 * and 1 for SS_COST_SQEUCLID (the Gibbs kernel of eq. (rot) becomes
 * exp(-|x' - y'|^2)).  For the side predicting the scalings of points z_i
 * with weights w_i given the opposite measure (o_j, q_j), j < m:
 *   phi_j = ReLU(P [o_j, m q_j] + p),  e = mean_j phi_j,  g = U e + c1,
 *   h1_i = ReLU(W1 z_i + g),  h2_i = ReLU(W2 h1_i + c2),  psi_i = w3 . h2_i + c3,
 *   log y0_i = log w_i + psi_i;
 * the u side uses (x, a) with opposite (y, b), the v side (y, b) with (x, a).
 * Training minimises the mean over sides of the centred squared error
 * mean_M (d - mean_M d)^2, d = psi - (log y* - log w), over the points with
 * a finite target: Alg. 1 reads only v^0 and a constant shift of log v^0
 * leaves its iterates' plans unchanged (eq. (rot-solu)).
 *
 * params   device FP32 [SS_MLP_PARAMS] master weights in the order
 *          P (256x4), p (256), W1 (256x3), U (256x256), c1 (256),
 *          W2 (256x256), c2 (256), w3 (256), c3 (1), matrices row-major.
 * bf16     device BF16 copy [SS_MLP_PARAMS] used by the kernels.
 * w2t      device BF16 [256 x 256]: W2 transposed.
 * adam_m, adam_v  device FP32 [SS_MLP_PARAMS] Adam moments (zero at start).
 * step     Adam steps taken (incremented by ss_warmstart_train_step).
 * All buffers are owned by the caller. */
#define SS_MLP_PARAMS 133889

typedef struct ss_mlp {
    float *params;
    void *bf16;
    void *w2t;
    float *adam_m, *adam_v;
    int32_t step;
    int32_t reserved;
} ss_mlp;

/* Refreshes bf16 and w2t from params (after the caller changed params). */
int ss_mlp_sync(ss_mlp *mlp, void *stream);

/* Workspace bytes for ss_warmstart_predict / ss_warmstart_train_step on this
 * batch (d must be 3; the problem sizes of ss_batch apply). */
int ss_warmstart_workspace_size(const ss_batch *batch, size_t *bytes);

/* log_u0 (device FP64, sum(n)) and log_v0 (device FP64, sum(m)) for every
 * problem; pass them as init_log_u / init_log_v to spar_sink_batched (or to
 * spar_sink_ot per problem).  eps and cost are those of the solve.  Either
 * output may be NULL. */
int ss_warmstart_predict(const ss_mlp *mlp, const ss_batch *batch, double eps, int32_t cost,
                         double *log_u0, double *log_v0, void *ws, size_t ws_bytes, void *stream);

/* Learned warm start for a batch: spar_sink_batched started from
 * the network's prediction (ss_warmstart_predict), with the
 * prediction on a second stream of the library (one per host thread and
 * device, default priority) that overlaps the sampling stage; the loop waits
 * for it.  The prediction is judged per problem against the plain start, as
 * in spar_sink_batched, and the results equal ss_warmstart_predict followed
 * by spar_sink_batched with its outputs as init_log_u / init_log_v.  opts
 * must not carry init_log_u / init_log_v; d = 3; cost maxnorm or plain.
 * ws: ss_batch_learned_workspace_size bytes (the batch's, the network's and
 * the two start vectors).  Returns as spar_sink_batched. */
int ss_batch_learned_workspace_size(const ss_batch *batch, const ss_options *opts, size_t *bytes);
int spar_sink_batched_learned(const ss_batch *batch, const ss_options *opts,
                              const ss_schedule *schedule, const ss_mlp *mlp, void *ws,
                              size_t ws_bytes, void *stream, ss_result *outs);

/* One Adam step (learning rate lr, betas 0.9 / 0.999, eps 1e-8) on the batch
 * loss against the solutions tgt_log_u (device FP64, sum(n)) and tgt_log_v
 * (sum(m)); entries that are not finite (empty lines) are left out.  *loss
 * (host) receives the batch loss before the step; grad_out (device FP32
 * [SS_MLP_PARAMS], may be NULL) receives its gradient.  lr = 0 computes the
 * loss and gradient without changing the weights or the step count. */
int ss_warmstart_train_step(ss_mlp *mlp, const ss_batch *batch, double eps, int32_t cost,
                            const double *tgt_log_u, const double *tgt_log_v, float lr, void *ws,
                            size_t ws_bytes, void *stream, float *loss, float *grad_out);

/* ------------------------------------------------------------------------
 * Spar-IBP: fixed-support Wasserstein barycenters (the paper's barycenter
 * section: eq. (wb), eq. (rwb), Alg. IBP, eq. (pois-k), Alg. Spar-IBP).
 *
 * `count` probability measures b_k on one support {x_i} (n points in R^d)
 * and weights w_k >= 0 summing to 1.  Every measure gets its own sketch
 * K~_k of K = exp(-C/eps) (C as selected by opts->cost, shared by all
 * measures), sampled with p*_{k,ij} = min(1, s sqrt(b_kj) / (n sum_j
 * sqrt(b_kj))) (the Spar-Sink probability with the barycenter replaced by its
 * uniform start), mixed with the uniform s/n^2 by opts->shrink (Sec. 4;
 * shrink = 1 is Rand-IBP), from hash stream k (problem index k of the
 * Spar-Sink mask).  The loop is Alg. IBP in the order of the Bregman
 * projections: for every k, v_k = b_k / K~_k' u_k; q = prod_k (K~_k v_k)^(w_k);
 * for every k, u_k = q / K~_k v_k; q^0 = 1/n, u_k^0 = 1; a quotient with a
 * zero denominator is 0.  It stops at the first t with |q^t - q^(t-1)|_1 <=
 * opts->tol, or at opts->max_iter.
 *
 * x: device FP64 n*d row-major; b: device FP64 count*n (measure k at b + k n);
 * w: host FP64 count entries.  1 <= count <= SS_IBP_MAX_MEASURES. */
#define SS_IBP_MAX_MEASURES 64

typedef struct ss_ibp_problem {
    int64_t n;
    int32_t d, count;
    const double *x, *b;
    const double *w;
} ss_ibp_problem;

/* Result of spar_ibp (host struct).
 * err         |q^t - q^(t-1)|_1 at the returned t.   iters  that t.
 * cmax        max_ij |x_i - x_j|^2.   nnz  entries over all sketches.
 * empty_rows, empty_cols  lines of the sketches with no entry (summed over k).
 * status      same as the return value.   t_*_ms  stage times on `stream`. */
typedef struct ss_ibp_result {
    double err, cmax;
    int64_t nnz, empty_rows, empty_cols;
    int32_t iters, status;
    float t_sample_ms, t_iter_ms;
} ss_ibp_result;

/* Workspace bytes for spar_ibp and ss_ibp_sample.  Host-only. */
int ss_ibp_workspace_size(const ss_ibp_problem *problem, const ss_options *opts, size_t *bytes);

/* Alg. Spar-IBP.  Options used: eps, s, tol, seed, max_iter, precision
 * (SS_F64, or SS_F32: FP32 stored K~ values, FP64 products, scalings and
 * barycenter), cost, shrink, graph_iters, err_hist (max_iter FP64 entries:
 * |q^t - q^(t-1)|_1), u_out and v_out (count*n FP64 each, measure-major: the
 * returned u_k, v_k).  lambda must be +INFINITY; init_log_u/v must be NULL.
 * q_out: device FP64, n entries, receives the returned q^t.
 * Returns SS_OK, SS_NOT_CONVERGED (max_iter reached; result valid),
 * SS_E_INVALID_ARG, SS_E_CAPACITY, SS_E_NONFINITE (q became NaN or Inf) or
 * SS_E_HIP. */
int spar_ibp(const ss_ibp_problem *problem, const ss_options *opts, double *q_out, void *ws,
             size_t ws_bytes, void *stream, ss_ibp_result *result);

/* The sketch of measure k alone (parity surface of eq. (pois-k)): mask,
 * CSR, CSC and factors as in ss_sample, with row_fac_i = c and col_fac_j =
 * sqrt(b_kj) such that p*_{k,ij} = min(1, c col_fac_j + s shrink / n^2).
 * Synchronises `stream`. */
int ss_ibp_sample(const ss_ibp_problem *problem, const ss_options *opts, int32_t k,
                  ss_sparse *out, void *ws, size_t ws_bytes, void *stream);

/* Measurement hook for the Spar-IBP loop: samples the sketches like
 * spar_ibp, then runs exactly `iters` (>= 1) steps with tol ignored as one
 * captured HIP graph: one warm-up replay, one replay between two HIP events on
 * `stream`.  *ms_per_iter (host) receives the mean duration of one step (its
 * column launch and its row launch); *nnz (host, may be NULL) the entries
 * over all sketches. */
int ss_ibp_time_iterations(const ss_ibp_problem *problem, const ss_options *opts, void *ws,
                           size_t ws_bytes, void *stream, int32_t iters, double *ms_per_iter,
                           int64_t *nnz);

/* ------------------------------------------------------------------------
 * Sinkhorn divergence (the generative-modelling section, eq. (sink-div)):
 * S(mu, nu) = OT_eps(mu, nu) - (OT_eps(mu, mu) + OT_eps(nu, nu)) / 2 with each
 * term the Spar-Sink estimate of Alg. 3, from three OT solves on hash streams
 * problem_index, problem_index + 1 and problem_index + 2.  The cost must be
 * SS_COST_SQEUCLID (one cost for all three terms) and lambda +INFINITY.
 * Gradients (optional, device FP64, grad_x n*d and grad_y m*d row-major, both
 * or neither): the derivatives of the sparse problems' values in the points
 * by the envelope theorem, sum_j T~_ij 2 (x_i - y_j) per term, with the mask
 * fixed (the OT probability depends on the masses only); the self terms
 * contribute through both of their arguments.  opts->u_out, v_out, err_hist,
 * init_log_u and init_log_v are ignored.  The workspace is the largest of
 * the three solves' (ss_divergence_workspace_size). */
typedef struct ss_divergence {
    double value;          /* S from the Alg. 3 estimates */
    double value_sparse;   /* S from the sparse problems' values */
    double ot_xy, ot_xx, ot_yy;
    double sparse_xy, sparse_xx, sparse_yy;
    int64_t nnz;           /* entries over the three sketches */
    int32_t iters_xy, iters_xx, iters_yy, status;
} ss_divergence;

int ss_divergence_workspace_size(const ss_problem *problem, const ss_options *opts,
                                 size_t *bytes);
int ss_sinkhorn_divergence(const ss_problem *problem, const ss_options *opts, double *grad_x,
                           double *grad_y, void *ws, size_t ws_bytes, void *stream,
                           ss_divergence *result);

const char *ss_status_string(int status);
const char *ss_last_error(void);
int ss_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPARSINK_H */
