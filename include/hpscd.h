/*
 * hpscd.h - C ABI of libhpscd, an MI355X (gfx950) implementation of the HPSCD
 * column-wise solver for X·a = y.
 *
 * The method (paper, Section 2, Algorithm 1; step derivation in Section 3):
 * start from a = a0 (zero unless given) and e = y - X·a, then repeat sweeps
 * over the columns j = 1..n in order:
 *     da = <X_j, e> / <X_j, X_j>;   e <- e - X_j·da;   a_j <- a_j + da.
 * Section 4 proves ||e|| never increases and tends to the least-squares
 * minimum; Section 5 counts O(m) work per column step, O(mn) per sweep.
 *
 * Conventions shared by every entry point:
 *  - X is column-major: column j starts at X + j*ldx.  Rows m..ldx-1 of a
 *    column are never read as data (they may hold anything, NaN included).
 *  - Array arguments named X*, y, a*, e*, *pool are DEVICE pointers owned by
 *    the caller; arguments named hist, info, sys, sweeps_done, converged,
 *    final_rel_resid, norm_out are HOST pointers owned by the caller.  The
 *    library owns only the workspace held by its context.
 *  - `stream` is a hipStream_t (NULL = the default stream).  Work is queued on
 *    it in order; every solve call returns after the solve has finished,
 *    because it fills host-side outputs.
 *  - Arguments are validated before any device work.  On HPSCD_EINVAL no
 *    output is written and hpscd_last_error() names the argument.
 *  - A context is not thread-safe: use one context per host thread.
 *  - No C++ exception crosses this interface.
 */
#ifndef HPSCD_H
#define HPSCD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HPSCD_VERSION 2

typedef struct hpscd_ctx hpscd_ctx;

typedef enum {
  HPSCD_OK = 0,
  HPSCD_EINVAL = 1,     /* bad argument (nothing was run) */
  HPSCD_ENOMEM = 2,     /* device workspace could not be allocated */
  HPSCD_EDEVICE = 3,    /* HIP runtime error, or no usable device */
  HPSCD_ENONFINITE = 4, /* X or y holds NaN/Inf (found before the first sweep), or the iteration overflowed */
  HPSCD_EABORTED = 5,   /* hpscd_abort() was called during the solve */
  HPSCD_ETIMEOUT = 6    /* a grid-wide reduction waited longer than the bound; results are invalid */
} hpscd_status;

/* Stopping rules.  Algorithm 1 runs a fixed number N of sweeps; Section 2
 * allows breaking once the error is under a threshold (max_tol in the
 * nomenclature) without defining the error.  hist[s] = ||e||_2 after sweep s. */
typedef enum {
  HPSCD_STOP_NONE = 0,       /* run exactly max_sweeps sweeps */
  HPSCD_STOP_REL_CHANGE = 1, /* stop after sweep s >= 1 when hist[s-1] - hist[s] < tol*hist[s] */
  HPSCD_STOP_REL_RESID = 2,  /* stop when ||e|| < tol*||y||: tested before the first sweep, after
                                every sweep, and every check_cols column steps if check_cols > 0 */
  HPSCD_STOP_REL_GRAD = 3    /* stop after sweep s when ||X^T e||_2 < tol*||X^T y||_2 (least-squares
                                systems, whose residual does not vanish).  X^T e is one more pass
                                over X after every sweep (FP64 sums of the single-precision e);
                                single-system FP32 solves only.  A zero residual or gradient stops. */
} hpscd_stop;

#define HPSCD_F_NO_FINAL_CHECK 1 /* skip the FP64 ||y - X·a|| pass (final_rel_resid = NaN) */
#define HPSCD_F_FORCE_GRID 2     /* single system: use a persistent grid of workgroups */
#define HPSCD_F_FORCE_WG 4       /* single system: use one workgroup */
#define HPSCD_F_NO_COOP 8        /* launch the grid without hipLaunchCooperativeKernel */

typedef struct {
  int32_t max_sweeps;   /* N >= 0 */
  int32_t stop;         /* hpscd_stop */
  double tol;           /* finite, >= 0; ignored by HPSCD_STOP_NONE */
  int64_t check_cols;   /* >= 0, see HPSCD_STOP_REL_RESID (rounded to the block size) */
  int64_t refresh_cols; /* e = y - X32·a (FP64 sums) every refresh_cols column steps (X32 = X for
                           hpscd_solve_f32); with HPSCD_STOP_REL_RESID a stop signalled by the running
                           residual then holds only if the refreshed one passes too; 0 = never */
  int32_t block;        /* columns per reduction round (1, 2, 4, 8; 16 with depth 8 or 9; 32 with depth 9
                           on bfloat16 columns); 0 = library choice */
  int32_t flags;        /* HPSCD_F_* */
  int32_t team_threads; /* threads per workgroup; 0 = library choice.  Batched calls: 256
                           (four waves, eight chunks per thread) or 512 (eight waves, four) */
  int32_t depth;        /* kernel kind; 0 = library choice.  2, 3: prefetch ring of 2 or 3 blocks;
                           4: a 4-block ring (one workgroup only);
                           5: grid kernel whose polling waves never wait behind column loads
                           (their rows arrive through LDS); 8: 16-column blocks through each
                           block's precomputed step matrix, no column loads in flight during the
                           exchange, the next block's first two columns requested right after it
                           (a grid, or one workgroup without exchange for at most 4096 rows); 9: the column chain of a short system (at most 2048 rows) on one
                           workgroup, 16 FP32 or 32 bfloat16 columns per block through its step
                           matrix, the next block's columns and step matrix in flight (the library
                           choice for such systems when the options allow it: block 0 or that
                           size, which divides check_cols, refresh_cols and then n; no thr, no
                           order, no HPSCD_F_FORCE_GRID) */
  /* Variants of the method (single-system FP32 solves, kernel kind 8 only; the block size is 16): */
  int32_t thr;          /* Section 7, Algorithm 2 (HPSCDP): every sweep takes the columns in consecutive
                           blocks of thr (the last block holds what remains); all columns of a block step
                           against the residual at the block's start, then e takes the whole block.
                           0 or 1 = Algorithm 1.  Not combined with `order`. */
  const int32_t* order; /* Section 2's randomly selected index: NULL = cyclic order, else a DEVICE array
                           [max_sweeps][n] whose row s-1 lists the columns visited in sweep s (each row a
                           permutation of 0..n-1, not checked: a repeated or missing index changes the
                           method, an index outside 0..n-1 is an error the caller must not make).  The
                           statistics of the sweep's 16-column blocks are recomputed before every sweep
                           (one more pass over X per sweep); X must be smaller than 4 GiB. */
  int32_t spin_timeout_us; /* bound on every wait of a grid's workgroups for one another (each grid
                              reduction), in microseconds; 0 = 10 s.  A wait past it ends the solve with
                              HPSCD_ETIMEOUT (a and the history are then invalid).  A bound under
                              2.4 us also shortens the pause before a reduction's first poll to half
                              the bound.  Must be >= 0. */
} hpscd_opts;

typedef struct {
  int32_t sweeps_done;     /* complete sweeps */
  int32_t converged;       /* 1 if a stop rule fired */
  int64_t cols_done;       /* column steps performed */
  int64_t zero_cols;       /* columns with <X_j, X_j> = 0, skipped (da = 0) */
  double final_norm;       /* ||e||_2 of the running single-precision residual at exit */
  double final_rel_resid;  /* ||y - X·a||_2 / ||y||_2 of the returned (FP32) a, FP64 sums (NaN if skipped) */
  double y_norm;           /* ||y||_2 */
  int32_t block_used;      /* B: columns per reduction round */
  int32_t team_wgs;        /* workgroups in the team (1 = one workgroup) */
  int32_t team_threads;    /* threads per workgroup */
  int32_t refreshes;       /* residual refreshes queued (bf16 form) */
  double sweep_ms;         /* device time of the sweep kernels (HIP events) */
  double total_ms;         /* device time of the whole call (HIP events) */
  int32_t kernel_kind;     /* sweep kernel used (the values of hpscd_opts.depth); 0 for batched calls */
  int32_t diverged;        /* 1 if ||e|| grew by more than 0.1 % over some sweep (Algorithm 2 with
                              strongly correlated columns in one block; never for Algorithm 1) */
  double rel_grad;         /* HPSCD_STOP_REL_GRAD: ||X^T e||/||X^T y|| at the last test; else NaN */
} hpscd_info;

/* Fill *o with defaults: max_sweeps 100, HPSCD_STOP_NONE, tol 0, no checks,
 * no refresh, block 0, flags 0, Algorithm 1 (thr 0), cyclic order. */
void hpscd_default_opts(hpscd_opts* o);

/* Create a context on HIP device `device` (owns the workspace).  Returns
 * HPSCD_EDEVICE when no such device exists. */
hpscd_status hpscd_create(int device, hpscd_ctx** out);
void hpscd_destroy(hpscd_ctx* ctx);

/* Check the arguments of hpscd_solve_f32 without touching a device (used by
 * the solve itself first).  Returns HPSCD_OK or HPSCD_EINVAL. */
hpscd_status hpscd_validate(int64_t m, int64_t n, const void* X, int64_t ldx, int elem_bytes, const void* y,
                            const hpscd_opts* opts, const void* a_out);

/* Solve X·a = y by Algorithm 1 in single precision (FP32 X, residual and
 * products; FP64 sums of the per-workgroup partials, FP64 accumulation of a).
 * X: m x n column-major FP32, 16-byte aligned, ldx >= m, ldx % 4 == 0.
 * y: m floats.  a0: n floats or NULL (zero start).  a_out: n floats.
 * hist: NULL or max_sweeps+1 doubles, hist[s] = ||e||_2 after sweep s for
 * s <= sweeps_done.  info: NULL or filled on return. */
hpscd_status hpscd_solve_f32(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx, const float* y,
                             const float* a0, const hpscd_opts* opts, float* a_out, double* hist,
                             hpscd_info* info, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): hpscd_solve_f32 with the
 * same arguments, results and kernels, allocating nothing.  Its whole device
 * workspace (control words, residual copies, column statistics, exchange
 * words, partial sums, history) lies in a fixed scratch area of
 * HPSCD_NOALLOC_SCRATCH_BYTES per device, which the library holds from the
 * loading of its code on that device until the process ends; host results
 * return through copies into the caller's memory (hist may be NULL; then
 * info->diverged stays 0).  A solve whose workspace does not fit (about
 * 8·m + 9 MB for a single-precision system; 4·m less without a0) returns
 * HPSCD_EINVAL before any device work, naming the size.  Every call on one
 * device shares that device's area, and it keeps the last call's contents:
 * calls that overlap on one GPU (two streams, two threads, two contexts)
 * race and must be serialised by the caller. */
#define HPSCD_NOALLOC_SCRATCH_BYTES (64u << 20)
hpscd_status hpscd_solve_f32_noalloc(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx,
                                     const float* y, const float* a0, const hpscd_opts* opts, float* a_out,
                                     double* hist, hpscd_info* info, void* stream);

/* Reduced-precision storage form: the sweeps read X rounded to bfloat16
 * (Xb, ldxb % 8 == 0) with FP32 products and residual; the starting residual,
 * every residual refresh (opts->refresh_cols) and the final check use the FP32
 * copy X32 with FP64 sums.  Other arguments as hpscd_solve_f32. */
hpscd_status hpscd_solve_bf16(hpscd_ctx* ctx, int64_t m, int64_t n, const uint16_t* Xb, int64_t ldxb,
                              const float* X32, int64_t ldx, const float* y, const float* a0,
                              const hpscd_opts* opts, float* a_out, double* hist, hpscd_info* info, void* stream);

/* dst = bfloat16(src), round to nearest, ties to even; rows x cols,
 * column-major, ldd % 8 == 0, dst 16-byte aligned.  Rows rows..ldd-1 are
 * written as zero. */
hpscd_status hpscd_convert_bf16(hpscd_ctx* ctx, int64_t rows, int64_t cols, const float* src, int64_t lds,
                                uint16_t* dst, int64_t ldd, void* stream);

/* r = y - X·a with FP64 sums (the check of Section 4's e = y - X·a).
 * e_out: NULL or m floats.  norm_out: NULL or host double, receives ||r||_2. */
hpscd_status hpscd_residual_f64(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx,
                                const float* y, const float* a, float* e_out, double* norm_out, void* stream);

/* Feature selection with HPSCD (Section 8, Algorithm 3, HPSCDF).  Starting
 * from a = a0 (zero if NULL) and e = y - X·a, F times: take the step
 * da_j = <X_j, e>/<X_j, X_j> of every column against the same e, choose the
 * column j^ not selected yet whose step leaves the smallest squared error
 * ||e - X_j da_j||^2 = ||e||^2 - <X_j,e>^2/<X_j,X_j> (the largest
 * <X_j,e>^2/<X_j,X_j>; ties to the lowest index; zero columns never), then
 * a_j^ += da_j^ and e -= X_j^ da_j^.  tol > 0 is the section's while-loop
 * variant: selection stops before a column whose step lowers ||e||^2 by less
 * than tol*||e||^2.  The residual and the inner products are FP64 (X is read
 * as FP32); every selection is one pass over X (HBM-bound).
 * X: m x n column-major FP32 as hpscd_solve_f32.  a0: NULL or n floats.
 * a_out: n floats (device).  J_out: host, F entries (the selected columns in
 * order; entries past *selected are -1).  da_out, hist: NULL or host arrays
 * of F and F+1 doubles (the steps taken; ||e||_2 before the first and after
 * each selection).  selected: host, receives the number of columns chosen. */
hpscd_status hpscd_select_f32(hpscd_ctx* ctx, int64_t m, int64_t n, const float* X, int64_t ldx, const float* y,
                              const float* a0, int32_t F, double tol, float* a_out, int32_t* J_out,
                              double* da_out, double* hist, int32_t* selected, void* stream);

/* Batched form: `count` independent systems in one persistent launch.
 * sys[i] gives system i's sizes and element offsets into the pools; every
 * system needs x_off % 4 == 0, ldx % 4 == 0, ldx >= m, 1 <= m <= 8192.
 * sys[i].tol > 0 replaces opts->tol for that system's stop rule (0: use
 * opts->tol); it must be finite and >= 0.
 * a0pool: NULL or initial guesses at a_off.  apool: results at a_off.
 * hist: NULL or count*(max_sweeps+1) doubles (row i for system i).
 * sweeps_done, converged, final_rel_resid: NULL or count entries (host). */
typedef struct {
  int64_t m, n, x_off, ldx, y_off, a_off;
  double tol;
} hpscd_sys;

hpscd_status hpscd_solve_batched_f32(hpscd_ctx* ctx, int32_t count, const hpscd_sys* sys, const float* Xpool,
                                     const float* ypool, const float* a0pool, const hpscd_opts* opts, float* apool,
                                     double* hist, int32_t* sweeps_done, int32_t* converged,
                                     double* final_rel_resid, hpscd_info* info, void* stream);

/* Time the batched kernel's variants on this batch (block size 1, 2 or 4;
 * systems that fit one wave packed as many to a workgroup as it has waves, or
 * one workgroup per system) and remember the fastest for batches of the same
 * shape (kept in the context), together with the sweeps each system took:
 * later solves and plans of such a batch hand out the systems in decreasing
 * order of (sweeps + 1) * blocks * the team's time per block, so the longest
 * column chains start first.  The order changes no result. */
hpscd_status hpscd_autotune_batched(hpscd_ctx* ctx, int32_t count, const hpscd_sys* sys, const float* Xpool,
                                    const float* ypool, const hpscd_opts* opts, float* apool, void* stream);

/* Recorded batched solve.  hpscd_batched_plan_create validates and plans the
 * batch once (block size and work split from hpscd_autotune_batched when it
 * was run on a batch of this shape), uploads the system table into the
 * plan's own device workspace, and records the whole solve (initial
 * residuals, column statistics, the persistent sweep kernel, the output of a
 * and the FP64 check) as a HIP graph.  The pools are bound by address: their
 * contents (X, y, a0) may change between launches, their addresses may not.
 * hpscd_batched_plan_launch queues one replay on `stream` and returns without
 * waiting; hpscd_batched_plan_results waits for `stream` and returns the
 * per-system results of the last replay (arguments as in
 * hpscd_solve_batched_f32; info->sweep_ms and total_ms are NaN).  A plan
 * belongs to its context (same thread rules); replays of one plan must not
 * overlap.  The host staging buffer of the context is used by results. */
typedef struct hpscd_batch_plan hpscd_batch_plan;

hpscd_status hpscd_batched_plan_create(hpscd_ctx* ctx, int32_t count, const hpscd_sys* sys, const float* Xpool,
                                       const float* ypool, const float* a0pool, const hpscd_opts* opts,
                                       float* apool, hpscd_batch_plan** plan);
hpscd_status hpscd_batched_plan_launch(hpscd_batch_plan* plan, void* stream);
hpscd_status hpscd_batched_plan_results(hpscd_batch_plan* plan, double* hist, int32_t* sweeps_done,
                                        int32_t* converged, double* final_rel_resid, hpscd_info* info, void* stream);
void hpscd_batched_plan_destroy(hpscd_batch_plan* plan);

/* Measured denominator of the bandwidth roofline: average device time of one
 * pass of 16-byte loads over `bytes` of the device buffer `buf` (16-byte
 * aligned, bytes a multiple of 16) over `passes` passes after one untimed
 * pass; the loaded data is summed and discarded.  Returns after the passes. */
hpscd_status hpscd_read_stream(hpscd_ctx* ctx, const void* buf, int64_t bytes, int32_t passes, double* ms_per_pass,
                               void* stream);

/* Ask a running solve on this context to stop at its next sweep boundary;
 * that solve returns HPSCD_EABORTED.  Safe to call from another thread.  The
 * request is a store to a word of pinned host memory that the kernels read at
 * sweep starts: it issues no GPU work, so it takes effect while a persistent
 * kernel occupies every CU.  A request made while no solve runs is dropped
 * when the next solve starts. */
hpscd_status hpscd_abort(hpscd_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Learned warm start: a multilayer perceptron in -> h1 -> h2 -> out with the
 * exact GELU (0.5 z (1 + erf(z / sqrt 2))) after both hidden layers and a
 * linear output, trained with Adam (beta1 0.9, beta2 0.999, eps 1e-8) on the
 * mean squared error L = sum_{b,k} (o_bk - t_bk)^2 / (batch * out).  It maps a
 * system's parameters to a predicted solution, used as the initial guess a0
 * of Algorithm 1 (the algorithm's first line allows any initial guess).
 * Parameter vector (FP32, device): W1[h1][in], b1[h1], W2[h2][h1], b2[h2],
 * W3[out][h2], b3[out] (row o of a W holds the weights of output unit o).
 * With an output scaling (below) the output and the loss are taken in
 * standardised units.
 * x, target, y, flat and grad_flat are device pointers; rows are row-major
 * ([batch][in], [batch][out]).  All work is queued on `stream`; calls that
 * fill loss_out (host) wait for it.
 * ------------------------------------------------------------------------- */
typedef struct hpscd_mlp hpscd_mlp;

/* A network on the context's device, its parameters drawn by the library:
 * the weights and biases of each layer uniform in [-1/sqrt(fan_in),
 * 1/sqrt(fan_in)) (fan_in: that layer's input width); parameter k of the
 * flat vector takes value k of the SplitMix64 stream started at `seed`
 * (Steele, Lea and Flood 2014), u = top 53 bits / 2^53, w = (2u - 1)·bound.
 * The Adam state starts at zero. */
hpscd_status hpscd_mlp_create(hpscd_ctx* ctx, int in, int h1, int h2, int out, uint64_t seed, hpscd_mlp** res);
void hpscd_mlp_destroy(hpscd_mlp* net);
int64_t hpscd_mlp_num_params(const hpscd_mlp* net);
/* Copy parameters in (and reset the Adam state) / out. */
hpscd_status hpscd_mlp_set_params(hpscd_mlp* net, const float* flat, void* stream);
hpscd_status hpscd_mlp_get_params(hpscd_mlp* net, float* flat, void* stream);
/* y[batch][out] = net(x[batch][in]). */
hpscd_status hpscd_mlp_forward(hpscd_mlp* net, int batch, const float* x, float* y, void* stream);
/* Gradient of L at the current parameters into grad_flat (NULL: kept inside). */
hpscd_status hpscd_mlp_grads(hpscd_mlp* net, int batch, const float* x, const float* target, float* grad_flat,
                             float* loss_out, void* stream);
/* One Adam step on L for this batch; loss_out (host, NULL ok) gets L before the step. */
hpscd_status hpscd_mlp_train_step(hpscd_mlp* net, int batch, const float* x, const float* target, float lr,
                                  float* loss_out, void* stream);

/* Output scaling (standardised targets).  hpscd_mlp_fit_output_scaling sets,
 * for every output k, mu_k and sd_k to the mean and the sample standard
 * deviation (FP64 sums; sd at least 1e-12, 1 for one row) of column k of
 * target[count][out] (device).  From then on the network's output is
 * y = sd ⊙ (W3 h2 + b3) + mu (hpscd_mlp_forward), and the loss of
 * hpscd_mlp_grads / hpscd_mlp_train_step compares W3 h2 + b3 with the
 * standardised target (t - mu) / sd.  A new network has mu = 0, sd = 1.
 * mu_sd: device, 2*out floats [mu..., sd...] (get: written; set: read). */
hpscd_status hpscd_mlp_fit_output_scaling(hpscd_mlp* net, int count, const float* target, void* stream);
hpscd_status hpscd_mlp_get_output_scaling(hpscd_mlp* net, float* mu_sd, void* stream);
hpscd_status hpscd_mlp_set_output_scaling(hpscd_mlp* net, const float* mu_sd, void* stream);

/* Message of the last failure on this host thread ("" if none). */
const char* hpscd_last_error(void);

int hpscd_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HPSCD_H */
