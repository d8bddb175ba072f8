/*
 * svmhip.h -- C-ABI of libsvmhip.so, an SMO trainer for two-class soft-margin
 * RBF support vector machines on one AMD Instinct MI355X (gfx950).
 *
 * Method: the parallel SMO with adaptive shrinking of Narasimhan, Vishnu,
 * Holder and Hoisie ("Fast Support Vector Machines Using Parallel Adaptive
 * Shrinking on Distributed Systems").  The library solves the Wolfe dual
 * (eq:lagdual with the constraints of eq:eqconst):
 *
 *     max_alpha  sum_i alpha_i - 1/2 sum_ij alpha_i alpha_j y_i y_j K(x_i, x_j)
 *     s.t.       0 <= alpha_i <= C,  sum_i alpha_i y_i = 0
 *
 * with the Gaussian kernel K(x, z) = exp(-gamma * ||x - z||^2), gamma = 1/(2 sigma^2)
 * (Section "Datasets").  It maintains f_i = sum_j alpha_j y_j K_ij - y_i
 * (eq:fcache, the paper's gamma_i), selects the two worst violators b_up /
 * b_low (eq:bminmax) with the lowest sample index on ties, updates the pair
 * (eq:alphaup, eq:rho) and stops when b_low - b_up <= 2 eps (eq:kktterm).
 * Shrinking follows eq:shrink with the schedules of Table 3 and the driver of
 * Alg. 5 (single reconstruction) or its multi-reconstruction variant;
 * shrunk samples get their f back by gradient reconstruction (Alg. 6).
 *
 * Conventions for every entry point:
 *   - every array argument is a DEVICE pointer unless it is marked "host";
 *   - the caller owns every buffer; the library never frees caller memory;
 *   - `stream` is a hipStream_t (NULL = the default stream); calls are
 *     stream-ordered and return after the host-visible outputs are written;
 *   - return value: 0 = SVM_OK, > 0 = warning (the outputs are consistent),
 *     < 0 = error (outputs undefined); svm_strerror() gives the text.
 *   - calls are not re-entrant on one workspace; distinct workspaces may be
 *     used from distinct host threads.
 */
#ifndef SVMHIP_H
#define SVMHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes */
#define SVM_OK 0
#define SVM_NOT_CONVERGED 1      /* max_iter reached; alpha, f and the result are consistent */
#define SVM_EINVAL (-1)          /* bad argument: sizes, C/gamma/eps <= 0, labels not +-1, bad CSR */
#define SVM_EONECLASS (-2)       /* only one class present in y */
#define SVM_ENONFINITE (-3)      /* NaN or Inf in the sample values */
#define SVM_EWORKSPACE (-4)      /* workspace too small or misaligned */
#define SVM_EHIP (-5)            /* a HIP runtime call failed */
#define SVM_EUNSUPPORTED (-6)    /* shape outside what the library handles (e.g. CSR row too long) */
#define SVM_ENOMEM (-7)          /* an internal allocation failed (server budget exhausted, ...) */
#define SVM_EBUSY (-8)           /* serving: the ticket is still running */
#define SVM_EABORT (-9)          /* the device loop stopped on its watchdog (barrier wait timed out) */
#define SVM_ESCRATCH (-10)       /* svm_decision_noalloc: the problem needs more than its built-in scratch */

/* ---- sample layouts */
#define SVM_DENSE_ROW_MAJOR 0     /* x[i*ldx + k], ldx >= d */
#define SVM_DENSE_FEATURE_MAJOR 1 /* x[k*ldx + i], ldx >= n */
#define SVM_CSR 2                 /* row_ptr[n+1], col/val[nnz]; columns sorted, unique, in [0, d) */

/* ---- shrinking (Table 3): mode and schedule */
#define SVM_SHRINK_NONE 0         /* Alg. 2 "Original": no shrinking */
#define SVM_SHRINK_SINGLE 1       /* Alg. 5: shrink until 20 eps, reconstruct once, finish unshrunk */
#define SVM_SHRINK_MULTI 2        /* multi-reconstruction variant: reconstruct whenever the active set meets the tolerance */
#define SVM_KIND_FIXED 0          /* "random: k": shrink every k iterations (k = shrink_param) */
#define SVM_KIND_FRACTION 1       /* "numsamples": first shrink after ceil(shrink_param * n) iterations */

/* ---- kernel-value precision */
#define SVM_KERNEL_FP32 0         /* kernel values in FP32; f, alpha, thresholds, KKT test in FP64 */
#define SVM_KERNEL_FP64 1         /* everything in FP64 (follows the FP64 reference trajectory) */

/* ---- flags */
#define SVM_FLAG_WARM_START 1u         /* alpha and f are inputs: f must equal eq:fcache for alpha */
#define SVM_FLAG_NO_FINAL_RECOMPUTE 2u /* skip the closing FP64-accumulated recompute of f and KKT re-check */
#define SVM_FLAG_NO_LDS_PAYLOAD 4u     /* tuning/test: stream row payload from HBM even when it fits in LDS */
#define SVM_FLAG_NO_LDS_STATE 8u       /* tuning/test: keep per-row state in HBM as well */
#define SVM_FLAG_NO_BITSETS 16u        /* tuning/test: binary CSR rows as column ids, not bitsets */
#define SVM_FLAG_KERNEL_MATRIX 32u     /* svm_train, FP32 kernel values, CSR rows with the dense head (see
                                          head_cols): when cache_mb holds all n rows, the whole kernel matrix
                                          is computed into the cache on the matrix cores before the loop (the
                                          reconstruction's kernel sums, storing each value), and every
                                          iteration reads both kernel rows and K(up, low) from it.  Its values
                                          come from that kernel's arithmetic, not the loop's, so the FP32
                                          trajectory is not the one without the flag.  Ignored when the
                                          conditions do not hold (result.kernel_matrix says whether it ran) */

/* A labelled (or, for queries, unlabelled) sample set.  All pointers are device pointers. */
typedef struct {
    int32_t n;                /* samples, >= 1 (training: >= 2) */
    int32_t d;                /* features, >= 1 */
    int32_t layout;           /* SVM_DENSE_ROW_MAJOR | SVM_DENSE_FEATURE_MAJOR | SVM_CSR */
    int32_t reserved;
    const float* x;           /* dense values */
    int64_t ldx;              /* dense leading dimension (elements) */
    const int32_t* row_ptr;   /* CSR */
    const int32_t* col;       /* CSR */
    const float* val;         /* CSR; values read as given */
    const int8_t* y;          /* labels +1 / -1 (may be NULL for query sets) */
} svm_problem_t;

typedef struct {
    double C;                 /* box bound, > 0 */
    double gamma;             /* RBF width 1/(2 sigma^2), > 0 */
    double eps;               /* tolerance: stop when b_low - b_up <= 2 eps */
    int32_t shrink_mode;      /* SVM_SHRINK_* */
    int32_t shrink_kind;      /* SVM_KIND_* */
    double shrink_param;      /* k (fixed) or fraction of n */
    int64_t max_iter;         /* iteration cap (> 0); reaching it returns SVM_NOT_CONVERGED */
    int32_t kernel_precision; /* SVM_KERNEL_FP32 | SVM_KERNEL_FP64 */
    uint32_t flags;           /* SVM_FLAG_* */
    int32_t grid_blocks;      /* 0 = choose automatically (the shape svm_autotune recorded for the problem's
                                 class, else a built-in rule); else the number of workgroups of the step
                                 (svm_train; fewer where the device or the LDS cannot hold that many, the
                                 result's grid_blocks says how many) or of the problem's team (batch /
                                 server, at most 64) */
    int32_t lanes_per_row;    /* 0 = choose automatically; CSR lanes per row (1, 2, 4, 8, 16, 32, 64) */
    int32_t head_cols;        /* CSR with d > 12,288 and FP32 kernel values (svm_train): columns kept as dense
                                 rows for the matrix cores in the reconstruction and recompute sums (Alg. 6),
                                 the most frequent ones; 0 = automatic (128), 32, 64 or 128; -1 = none (every
                                 nonzero through the sparse path) */
    int32_t cache_mb;         /* svm_train: MiB of the workspace for a kernel-row cache (0 = none).  Used when
                                 the SMO loop streams rows from HBM (not for rows kept in LDS, not for binary
                                 bitset rows): a slot holds K(s, i) of one sample s for every sample i, slot
                                 s mod S for S = min(n, cache_mb MiB / (n * value bytes)) slots; an iteration
                                 whose two pair rows are both in the cache reads no row data.  The cached values
                                 are the ones the loop computes, so results are identical with and without it. */
} svm_params_t;

typedef struct {
    double beta;              /* threshold: mean f over I0, else (b_up + b_low)/2 */
    double b_up, b_low;       /* final thresholds over all samples */
    double dual_obj;          /* sum alpha - 1/2 sum alpha_i y_i (f_i + y_i) */
    int64_t iterations;       /* SMO pair updates */
    int32_t n_sv, n_bsv;      /* alpha > 0, alpha == C */
    int32_t n_recon;          /* gradient reconstructions (Alg. 6) */
    int32_t status;           /* SVM_OK or SVM_NOT_CONVERGED */
    int64_t shrink_passes;    /* iterations on which the shrink rule ran */
    int64_t shrunk_total;     /* samples removed over all shrink passes */
    int32_t n_launches;       /* persistent-loop launches (phases) */
    int32_t grid_blocks;      /* workgroups used by the step */
    double ms_total;          /* wall time of the call (host clock) */
    double ms_step;           /* time in the persistent SMO loop launches (HIP events on the call's stream) */
    double ms_recon;          /* time in reconstruction / recompute (host clock) */
    int64_t rows_streamed;    /* active rows visited by the SMO loop, summed over iterations */
    int64_t nnz_streamed;     /* CSR: nonzeros of those rows (0 for dense) */
    int32_t pattern_only;     /* CSR values were all 1.0 and were not read */
    int32_t lanes_per_row;    /* CSR lanes per row used by the step */
    int32_t ksum_mfma;        /* reconstruction sums on the matrix cores: 1 dense rows (FP32), 2 the dense head
                                 of wide CSR rows (FP32), 0 none */
    double ms_ksum;           /* time in the reconstruction / recompute kernel-sum launches (HIP events) */
    int64_t recon_pairs;      /* (row, support vector) pairs those launches evaluated */
    int32_t head_cols;        /* head columns of the wide-CSR kernel sums (0: not used) */
    int32_t cache_rows;       /* slots of the kernel-row cache (0: not used) */
    int64_t rows_read;        /* of rows_streamed, those whose row data was read (the rest came from the cache) */
    int64_t cache_values;     /* kernel values read from or written to the row cache */
    int64_t cache_both;       /* iterations whose two kernel rows both came from the cache */
    int32_t kernel_matrix;    /* 1: the whole kernel matrix was computed into the cache (SVM_FLAG_KERNEL_MATRIX) */
    int32_t reserved;
    double ms_kmatrix;        /* time of that computation (HIP events on the call's stream) */
} svm_result_t;

/* Bytes of device workspace svm_train needs for this problem (256-byte aligned). */
size_t svm_train_workspace_size(const svm_problem_t* prob, const svm_params_t* params);

/* Train on `prob` (labels required).  alpha: n doubles (output; input with
 * SVM_FLAG_WARM_START).  f: n doubles or NULL (output: f_i of eq:fcache).
 * out: host struct.  workspace/ws_bytes: device buffer of at least
 * svm_train_workspace_size() bytes, or NULL/0 to let the library allocate and
 * free one itself.  The inputs are validated on the device first
 * (SVM_EINVAL / SVM_EONECLASS / SVM_ENONFINITE). */
int svm_train(const svm_problem_t* prob, const svm_params_t* params, double* alpha, double* f,
              svm_result_t* out, void* workspace, size_t ws_bytes, void* stream);

/* Several training problems over one sample set, trained in lockstep: one-vs-rest labelings
 * of a dataset or a C / gamma grid (the problems the paper's sample distribution shares, Sec.
 * "Data Structure Organization").  Each SMO iteration (Alg. 2, eq:fup, eq:bminmax) advances
 * every unconverged problem and reads each row once for all of them, so the row bytes per
 * problem-iteration fall about k-fold.  x: the shared samples (its y is not used); y[p]: the
 * labels of problem p (device, n bytes); params[p]: its C, gamma, eps, max_iter and flags,
 * with shrink_mode SVM_SHRINK_NONE and one kernel_precision for all (SVM_EUNSUPPORTED
 * otherwise); alpha[p] / f[p] (f may be NULL) and out[p] as in svm_train.  1 <= k <= 8; rows
 * dense, or CSR whose values are all 1.0 with d <= 1024 (kept as bitsets); SVM_EUNSUPPORTED
 * for other CSR.  Every problem's arithmetic is its svm_train run's (same trajectory, same
 * closing recompute), so alpha and f equal those of svm_train with the same parameters bit for
 * bit.  workspace: at least svm_train_shared_workspace_size() bytes, or NULL/0 to let the
 * library allocate it.  out[p].ms_step and rows_streamed are those of the shared launches. */
size_t svm_train_shared_workspace_size(const svm_problem_t* x, int32_t k, const int8_t* const* y,
                                       const svm_params_t* params);
int svm_train_shared(const svm_problem_t* x, int32_t k, const int8_t* const* y, const svm_params_t* params,
                     double* const* alpha, double* const* f, svm_result_t* out, void* workspace, size_t ws_bytes,
                     void* stream);

/* Decision values out[q] = sum_j alpha_j y_j K(x_j, z_q) - beta (eq:classi
 * before the sign; the class is +1 when the value is >= 0).  train: the
 * training set (labels required); alpha: n doubles; queries: nq samples of
 * the same d and the same family of layout (dense or CSR; labels ignored);
 * out: nq doubles.  kernel_precision as in svm_params_t.  workspace/ws_bytes:
 * device scratch of at least svm_decision_workspace_size() bytes, 256-byte
 * aligned (SVM_EWORKSPACE otherwise), or NULL/0 to let the library allocate
 * and free it on `stream` (stream-ordered).  Binary CSR rows on both sides
 * (every value 1.0, d <= 1024) are summed through bitsets; CSR with
 * 12,288 < d <= 65,535 and FP32 kernel values through the dense head of the
 * 128 most frequent training columns on the matrix cores plus the sparse tail. */
size_t svm_decision_workspace_size(const svm_problem_t* train, const svm_problem_t* queries, int32_t kernel_precision);
int svm_decision(const svm_problem_t* train, const double* alpha, double beta, double gamma,
                 const svm_problem_t* queries, double* out, int32_t kernel_precision, void* workspace,
                 size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that forbid
 * hipMalloc): svm_decision with the same arguments minus the workspace, running on a 96 MiB
 * scratch array that the library keeps in each GPU's memory from the first call on that GPU
 * until the process ends.  It calls no allocator.  Like svm_decision it reads its validation
 * results back and synchronises `stream`, so it cannot be recorded into a HIP graph.  A problem
 * whose scratch (svm_decision_workspace_size) exceeds 96 MiB returns SVM_ESCRATCH.  Every call
 * on one GPU uses that GPU's array: calls that overlap in time on one GPU (from several host
 * threads, or on streams that run concurrently) race and their outputs are undefined. */
int svm_decision_noalloc(const svm_problem_t* train, const double* alpha, double beta, double gamma,
                         const svm_problem_t* queries, double* out, int32_t kernel_precision, void* stream);

/* Several independent problems in one persistent fused launch: problem p is
 * solved by its own team of workgroups (one to 64: the smallest team whose
 * members can each keep their share of the samples, with its rows, in LDS,
 * when that share is at least 512 samples; else about 1500 samples per
 * workgroup, whose rows stream from HBM while their f, status and active
 * list stay in LDS; a team size recorded by svm_autotune for the problem's class
 * replaces that rule, and params[p].grid_blocks overrides both), problems never synchronise
 * with each other.  Every problem runs the whole method of svm_train (SMO
 * loop, shrinking, reconstruction, closing recompute) inside its team; alpha
 * and f do not depend on the team size or on the other problems.  alpha[p]
 * (device, n_p doubles) and f[p] (device or NULL) receive the solution; out[p]
 * (host) the result (grid_blocks = team size, ms_step = device time of the
 * solve).  All problems share one kernel precision.  CSR rows may hold at
 * most 4096 nonzeros and d (dense: d rounded up to 4) at most about 1700
 * (SVM_EUNSUPPORTED beyond).  Lanes per row come from a built-in rule unless
 * params[p].lanes_per_row is set.  The call allocates the problems' solver
 * state on the device itself and frees it before returning.  Returns the first
 * non-OK status. */
int svm_train_batch(int32_t k, const svm_problem_t* probs, const svm_params_t* params, double* const* alpha,
                    double* const* f, svm_result_t* out, void* stream);

/* ---- serving: continuous batching of training problems */
/* Create a server with a device-memory budget (bytes of solver state it may
 * keep resident) and at most max_slots (1..1024) problems in flight.  The
 * server owns one persistent device loop whose workgroups validate and pack
 * each admitted problem, then solve it (a team per problem, as in
 * svm_train_batch) as slots and memory free up; a host thread admits waiting
 * problems as running ones complete and stops the loop after 2 s without
 * work (the next submit starts it again).  Prepared problems are handed to
 * the loop largest estimated work (n^2 x bytes per row) first, and only while
 * the loop is short of work, so a burst finishes longest-first; a problem
 * prepared more than 3 s ago goes ahead of newer ones, oldest first.  While
 * the loop runs it holds all but 8 compute units, so other device work of the
 * process (copies, kernels) runs on those 8.  FP32 kernel values only. */
int svm_server_create(size_t hbm_budget, int32_t max_slots, void** server);
/* Queue a problem (its arrays must stay valid until the ticket completes).
 * alpha: n doubles (device) that receive the solution.  Returns a ticket; a
 * problem that fails the loop's validation (SVM_EINVAL, SVM_ENONFINITE,
 * SVM_EONECLASS, SVM_EUNSUPPORTED) or needs more solver state than the whole
 * budget (SVM_ENOMEM) gets a ticket whose svm_server_poll returns that error. */
int svm_server_submit(void* server, const svm_problem_t* prob, const svm_params_t* params, double* alpha,
                      int64_t* ticket);
/* SVM_OK and *out filled when done, SVM_EBUSY while queued or running. */
int svm_server_poll(void* server, int64_t ticket, svm_result_t* out);
/* Block until every submitted problem has completed. */
int svm_server_drain(void* server);
/* Serving counters (host): admitted, deferred-for-memory, completed, in flight. */
int svm_server_stats(void* server, int64_t* admitted, int64_t* deferred, int64_t* completed, int64_t* in_flight);
int svm_server_destroy(void* server);

const char* svm_strerror(int code);
int svm_version(void);

/* ---- shape autotuner */
#define SVM_TUNE_GRID 0           /* workgroups of svm_train's SMO loop */
#define SVM_TUNE_TEAM 1           /* team size of a problem in svm_train_batch / the server */
typedef struct {
    int32_t target;               /* SVM_TUNE_GRID or SVM_TUNE_TEAM */
    int32_t chosen;               /* the shape now used for problems of this class */
    int32_t n_candidates;
    int32_t reserved;
    int32_t shape[8];             /* the candidates as launched */
    double us_per_iter[8];        /* measured device time per SMO iteration of each */
} svm_tune_t;
/* Times a few launch shapes on `prob` (trial solves of its first iterations, on the device)
 * and keeps one for every later problem of its class when params.grid_blocks is 0 -- for
 * SVM_TUNE_GRID the fastest (the problem has the GPU to itself), for SVM_TUNE_TEAM the one with
 * the fewest workgroup-microseconds per iteration among those within 1.5x of the fastest time
 * per iteration (a team shares the launch with other problems, so its cost is workgroups held
 * times time, with a bound on how much slower one problem may get): a
 * class is the row layout, kernel precision, whether all CSR values are 1.0, whether
 * shrinking is on, and n and d rounded up to powers of two.  The shapes only spread the work
 * differently (the selection of eq:bminmax is exact and f is updated row by row), so results
 * do not depend on them.  Allocates trial buffers; alpha of the problem is not touched.
 * svm_autotune_reset forgets every class (the built-in rules apply again). */
int svm_autotune(const svm_problem_t* prob, const svm_params_t* params, int32_t target, svm_tune_t* out,
                 void* stream);
int svm_autotune_reset(void);

/* ---- test hooks */
/* Two-threshold selection (eq:bminmax) over the samples listed in `active`
 * (n_active ids; order irrelevant), from f, alpha and y (device arrays of the
 * full problem) and C, with the same block/grid reduction as the training
 * loop split over `num_blocks` workgroups (0 = automatic).  Ties go to the
 * lowest sample id; an empty side yields +-inf and id -1.  Outputs are host.
 * Allocates a small device buffer on `stream` for the call. */
int svm_debug_select(int32_t n_active, const int32_t* active, const double* f, const double* alpha,
                     const int8_t* y, double C, int32_t num_blocks, double* b_up, int32_t* i_up, double* b_low,
                     int32_t* i_low, void* stream);

/* Per-iteration pair trace of the next svm_train call on this host thread:
 * up to `cap` records of (i_up, i_low) and (b_up, b_low) as selected before
 * each pair update (device arrays).  Pass cap = 0 to switch it off. */
int svm_debug_set_trace(int64_t cap, int32_t* i_up, int32_t* i_low, double* b_up, double* b_low);

/* Per-phase device timer of the SMO loop: when `slots` (device, 8 uint64) is
 * non-NULL, workgroup 0 of every later svm_train on this host thread adds the
 * wall-clock ticks (100 MHz) it spent in [0] pair staging and update, [1] the
 * f-update / selection / shrink pass, [2] its block reduction, [3] the grid
 * barrier wait, [4] the record merge, [5] the iteration count, [6] staging of
 * the segment at launch, [7] the write-back at exit.  Problems admitted to
 * svm_train_batch (or a server) from this thread while it is set add rank 0's
 * ticks instead: [0] pair staging and K(up, low), [1] the f-update / selection
 * / shrink pass, [2] block reduction, [3] team selection exchange, [4]
 * reconstruction and recompute, [5] iterations, [6] start-up to the first
 * selection, [7] summary and completion.  NULL switches it off. */
int svm_debug_set_profile(uint64_t* slots);

/* Residency mode (0 HBM, 1 per-row state in LDS, 2 state and rows in LDS),
 * workgroups and CSR lanes per row chosen by the last svm_train on this host
 * thread (host outputs, may be NULL). */
int svm_debug_step_info(int32_t* mode, int32_t* grid_blocks, int32_t* lanes_per_row);

#ifdef __cplusplus
}
#endif
#endif /* SVMHIP_H */
