/*
 * sp2.h - C ABI of the SP2 density-matrix purification library (gfx950).
 *
 * The library computes the density matrix D of a symmetric matrix F with the
 * second-order spectral projection (SP2) recursion and the parameterless
 * stopping criterion of Kruchinina, Rudberg and Rubensson (2015), Alg. 2:
 *
 *   X_0  = (lambda_max I - F) / (lambda_max - lambda_min)        (Alg. 2)
 *   X_i  = X~_{i-1}^2           if the trace test picks x^2      (p_i = 1)
 *        = 2 X~_{i-1} - X~_{i-1}^2   otherwise                  (p_i = 0)
 *   X~_i = X_i + E_i,  E_i = removal of entries with |x| < tau (sec. 5)
 *   stop at step k >= 2 when p_k != p_{k-1} and
 *        log(v_k / C) / log(v_{k-2}) < 1.8,  C = (71 + 17 sqrt 17)/32,
 *   where v_k = ||X~_k - X~_k^2||_F (sec. 2, eq. eq:frobnorm) and the test
 *   is evaluated only when 0 < v_{k-2} < 1.
 *
 * Readings of the paper that this interface fixes:
 *   - n (n_iter) is the 0-based index of the returned iterate X~_n; n + 1
 *     matrix squares were computed (the paper's printed iteration counts
 *     equal n + 1).
 *   - The default polynomial choice takes x^2 iff the trace it produces is
 *     nearer to n_occ than the trace of 2x - x^2 (ties take 2x - x^2). This
 *     equals Alg. 2's "Tr X > n_occ" whenever Tr X^2 <= Tr X, i.e. for every
 *     spectrum inside [0,1]; the literal rule is SP2_BRANCH_LITERAL.
 *   - n_occ == 0 returns D = 0 and n_occ == n returns D = I, both with n = 0.
 *   - v_k == 0 exactly stops with n = k.
 *
 * Conventions for every entry point:
 *   - Every call returns an sp2_status; nothing throws across the ABI.
 *   - Pointers named *_dev are device pointers on the context's device;
 *     every other pointer is host memory. The caller owns all memory it
 *     passes; the context owns every workspace it allocates.
 *   - Matrices are dense, row-major, with a leading dimension (elements
 *     between the starts of consecutive rows) >= n. F must be symmetric;
 *     only the upper triangle of the iterates is computed and mirrored, so
 *     an asymmetric F is treated as given and not symmetrised.
 *   - A context is not thread-safe; separate contexts are independent.
 *   - Work is ordered on the context's HIP stream.
 */
#ifndef SP2_H
#define SP2_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Largest number of squares one run may compute. */
#define SP2_MAX_ITER_LIMIT 200

typedef struct sp2_ctx_s* sp2_ctx;

typedef enum {
  SP2_OK = 0,             /* success; for sp2_run: the stop criterion fired */
  SP2_INVALID_ARG = 1,    /* an argument failed validation; nothing was run */
  SP2_OUT_OF_MEMORY = 2,  /* a device or pinned-host allocation failed */
  SP2_HIP_ERROR = 3,      /* a HIP runtime call failed; see sp2_last_error */
  SP2_NOT_CONVERGED = 4,  /* max_iter squares computed, the stop never fired */
  SP2_DIVERGED = 5,       /* non-finite error or trace, or Tr X^2 > Tr X + n:
                             the bounds do not enclose the spectrum or F has
                             non-finite entries */
  SP2_BAD_STATE = 6       /* call out of order (e.g. sp2_run before init) */
} sp2_status;

/* Precision of the matrix squares and of the stored iterates. The affine
 * start X_0 is always formed in FP64 from the FP64 input and then rounded to
 * the storage precision; traces, the idempotency error and the stop test are
 * always accumulated and evaluated in FP64. */
typedef enum {
  SP2_FP64 = 0,    /* FP64 iterates, FP64 MFMA squares */
  SP2_FP32 = 1,    /* FP32 iterates, FP32 MFMA squares */
  SP2_BF16X3 = 2   /* FP32 iterates; each square as H H + H L + L H with
                      H = bf16(X), L = bf16(X - H) (round to nearest even),
                      BF16 MFMA products accumulated in FP32 */
} sp2_precision;

typedef enum {
  SP2_BRANCH_NEAREST = 0,  /* trace-nearest choice (default, see above) */
  SP2_BRANCH_LITERAL = 1   /* Alg. 2 as printed: x^2 iff Tr X > n_occ */
} sp2_branch;

/* Norm of X~_k - X~_k^2 that the stop test uses (sec. 2). */
typedef enum {
  SP2_NORM_FROBENIUS = 0,  /* v_k = ||.||_F (default) */
  SP2_NORM_MIXED = 1,      /* m_k = spectral norm of the matrix of Frobenius
                              norms of the 32 x 32 blocks (the block size of
                              sec. 6); spectral <= mixed <= Frobenius, and for
                              large n it stays below 1 where the Frobenius
                              norm does not. The spectral norm of the
                              block-norm matrix is its largest eigenvalue,
                              found by Lanczos (FP64, full
                              reorthogonalisation, at most 64 steps, until
                              the top Ritz value changes by < 1e-12
                              relative) */
  SP2_NORM_SPECTRAL = 2    /* e_k = ||X~_k - X~_k^2||_2, the error of Alg. 2
                              as printed (dense, batched and block-sparse
                              runs; block-sparse products walk the flagged
                              blocks of each block row). Found
                              by Lanczos on E = X~_k - X~_k^2 applied as
                              X~_k q - X~_k (X~_k q) to the stored iterate in
                              FP64 arithmetic (E is never formed): three-term
                              recurrence with exact inner products, at most
                              64 steps (two products with X~_k each), until
                              the estimate max(|top|, |bottom| Ritz value)
                              changes by < 1e-12 relative. The Ritz values
                              lie inside E's spectrum, so the estimate never
                              exceeds the norm; where E's top eigenvalues
                              cluster (the first steps) it may stay below it
                              by ~1e-4 relative. One cooperative launch per
                              step (every workgroup resident at once) runs
                              the Lanczos processes of all instances */
} sp2_norm;

/* How a run is driven. */
typedef enum {
  SP2_LAUNCH_AUTO = 0,       /* persistent for a batch of more than one
                                instance with the Frobenius norm (Alg. 2 or
                                SP2-ACC), otherwise a launch sequence per
                                step */
  SP2_LAUNCH_SEQUENCE = 1,   /* one sequence of kernel launches per step
                                (square kernels per configuration, then the
                                scalar step for all instances); the host
                                queues a few steps ahead of the last outcome
                                it has observed */
  SP2_LAUNCH_PERSISTENT = 2  /* one persistent kernel for the whole run,
                                captured with the affine start in a HIP graph
                                at the first run after an init and replayed
                                by every later run: its workgroups take
                                (instance, tile, step) items from a queue in
                                device memory, the workgroup that finishes an
                                instance's last tile of a step runs that
                                instance's stop and branch logic and queues
                                its next step, so every instance advances and
                                stops on its own. Every instance uses one
                                square-kernel configuration (kernel_config, or
                                the library's choice for the largest
                                instance) among the 64- and 128-tile ones;
                                Frobenius norm only; kernel_timing records
                                nothing */
} sp2_launch;

/* Block edge of SP2_NORM_MIXED. */
#define SP2_MIXED_BLOCK 32

typedef struct {
  int32_t precision;  /* sp2_precision */
  int32_t branch;     /* sp2_branch */
  double trunc_tau;   /* element-magnitude truncation threshold, 0 = off;
                         entries with |x| < tau are set to zero in X_0 and
                         after every polynomial step (sec. 5) */
  int32_t max_iter;   /* at most this many squares; 0 selects 100; must be
                         <= SP2_MAX_ITER_LIMIT */
  int32_t kernel_config; /* square-kernel configuration: 0 lets the library
                            choose; otherwise a 1-based id from
                            sp2_kernel_config_info whose precision matches */
  int32_t tail_split;  /* tiles of an incomplete last round of workgroups are
                          split along k into pieces summed by a second
                          kernel: 0 = automatic, 1 = never, k >= 2 = k pieces
                          (at most 64) */
  int32_t kernel_timing; /* nonzero: bracket every square launch with a pair
                            of HIP timing events (read back through
                            sp2_get_kernel_times); adds a few microseconds
                            per step */
  int32_t norm;       /* sp2_norm: the error of the stop test */
  int32_t launch;     /* sp2_launch: how a run is driven */
} sp2_options;

/* Fills *opt with the defaults: SP2_FP64, SP2_BRANCH_NEAREST, no truncation,
 * max_iter 100, automatic kernel configuration and tail split, no kernel
 * timing, Frobenius norm, automatic launch. */
void sp2_default_options(sp2_options* opt);

/* Creates a context on HIP device `device`; `hip_stream` is a hipStream_t
 * (NULL = the default stream) that every later call orders its work on.
 * *out receives the handle. Errors: SP2_INVALID_ARG (out NULL, bad device),
 * SP2_HIP_ERROR. */
sp2_status sp2_create(sp2_ctx* out, int device, void* hip_stream);

/* Releases every workspace of the context (after synchronising its stream)
 * and the handle itself. NULL is accepted and ignored. */
sp2_status sp2_destroy(sp2_ctx ctx);

/* Prepares a dense run (Alg. 2 input: F, lambda_min, lambda_max, n_occ).
 * F_dev: n x n FP64, row-major, leading dimension ldf >= n, symmetric.
 * lambda_min <= smallest and lambda_max >= largest eigenvalue of F
 * (sec. 3, bounds of the extremal eigenvalues); lambda_max > lambda_min.
 * 0 <= n_occ <= n. opt may be NULL (defaults). Allocates the context's
 * workspaces (two iterate buffers padded to the tile size, FP64 partial sums,
 * the history) on first use or when n grows; reads nothing from F yet: F
 * must stay valid until sp2_run returns.
 * Errors: SP2_INVALID_ARG, SP2_OUT_OF_MEMORY, SP2_HIP_ERROR. */
sp2_status sp2_init_dense(sp2_ctx ctx, const double* F_dev, int64_t n,
                          int64_t ldf, double lambda_min, double lambda_max,
                          int64_t n_occ, const sp2_options* opt);

/* Runs Alg. 2 to the stop: the affine start, then one fused symmetric square
 * per step (the kernel's epilogue applies the chosen polynomial, the
 * truncation, and accumulates Tr X, Tr X^2 and ||X - X^2||_F^2 in FP64), and
 * the FP64 stop test on the device. Returns once the stream has finished the
 * run. Returns SP2_OK when the stop fired (or v_k == 0, or n_occ is 0 or n),
 * SP2_NOT_CONVERGED after max_iter squares, SP2_DIVERGED, or an error.
 * sp2_get_* report the outcome in every one of these cases. */
sp2_status sp2_run(sp2_ctx ctx);

/* Copies the returned iterate X~_n (n x n) to D_dev with leading dimension
 * ldd >= n: as FP64 when as_fp64 != 0, else in the storage precision (FP64
 * for SP2_FP64, FP32 for SP2_FP32 and SP2_BF16X3). Ordered on the stream and
 * synchronised before returning. After SP2_NOT_CONVERGED the iterate is
 * X~_{max_iter}. Errors: SP2_BAD_STATE before a completed run,
 * SP2_INVALID_ARG, SP2_HIP_ERROR. */
sp2_status sp2_get_density(sp2_ctx ctx, void* D_dev, int64_t ldd,
                           int32_t as_fp64);

/* Outcome of the last run: n_iter = n (index of the returned iterate),
 * n_squares = number of matrix squares computed, run_ms = device time of
 * sp2_run from the first kernel to the last, measured with HIP events.
 * Any pointer may be NULL. Errors: SP2_BAD_STATE before a run. */
sp2_status sp2_get_info(sp2_ctx ctx, int32_t* n_iter, int32_t* n_squares,
                        double* run_ms);

/* Mixed-norm history of instance `index` of the last run (index 0 for a
 * dense or block-sparse context): m[k] = ||X~_k - X~_k^2||_M for
 * k = 0..n_squares-1, with the same conventions as v of sp2_get_history.
 * Errors: SP2_BAD_STATE before a run or when the run did not use
 * SP2_NORM_MIXED, SP2_INVALID_ARG. */
sp2_status sp2_get_mixed_history(sp2_ctx ctx, int32_t index, int32_t cap,
                                 int32_t* len, double* m);

/* History of the error the stop test read, for a run with the mixed or the
 * spectral norm: e[k] = ||X~_k - X~_k^2|| in that norm for
 * k = 0..n_squares-1 (sec. 2; Alg. 2 for the spectral norm), same
 * conventions as sp2_get_mixed_history; the Frobenius norms stay available
 * through sp2_get_history. krylov[k] receives the number of Lanczos steps
 * behind e[k] (each step of the spectral norm is two products with X~_k).
 * e and krylov are host arrays of capacity `cap` and may be NULL. Errors:
 * SP2_BAD_STATE before a run or after a Frobenius-norm run,
 * SP2_INVALID_ARG. */
sp2_status sp2_get_norm_history(sp2_ctx ctx, int32_t index, int32_t cap,
                                int32_t* len, double* e, int32_t* krylov);

/* Per-step history of the last run, host arrays of capacity `cap`:
 * v[k] = ||X~_k - X~_k^2||_F for k = 0..n_squares-1; t1[k] = Tr X~_k and
 * t2[k] = ||X~_k||_F^2 = Tr X~_k^2 for k = 0..n_squares (t1/t2 of the iterate
 * of the last square is included when it was formed); p[k] = polynomial of
 * step k (1 = x^2, 0 = 2x - x^2; p[0] = -1); r[k] = observed order
 * log(v_k/C)/log(v_{k-2}) or NaN where undefined. *len receives the number of
 * valid v entries (= n_squares); t1, t2 and p hold up to n_squares + 1
 * entries. Arrays shorter than needed are filled up to cap. Any array
 * pointer may be NULL. */
sp2_status sp2_get_history(sp2_ctx ctx, int32_t cap, int32_t* len, double* v,
                           double* t1, double* t2, int8_t* p, double* r);

/* Device durations (milliseconds, from HIP events on the context's stream)
 * of the square launches of the last run whose options set kernel_timing:
 * ms[i] covers every square kernel of step i + 1 (all instances), for the
 * steps of the longest instance. *len receives that step count. ms may be
 * NULL. Errors: SP2_BAD_STATE when the last run did not record timings. */
sp2_status sp2_get_kernel_times(sp2_ctx ctx, int32_t cap, int32_t* len,
                                float* ms);

/* Device durations (milliseconds, HIP events on the context's stream) of the
 * spectral-norm launches of the last run, which must have used
 * SP2_NORM_SPECTRAL and kernel_timing: ms[i] covers the Lanczos estimate of
 * e_i (all instances). *len receives the step count. ms may be NULL.
 * Errors: SP2_BAD_STATE otherwise. */
sp2_status sp2_get_norm_times(sp2_ctx ctx, int32_t cap, int32_t* len,
                                float* ms);

/* ---- Block-sparse purification: the iterates are kept in block-sparse
 * row (BSR) form with 32 x 32 FP32 blocks and truncated by element
 * magnitude after every step (sec. 5: removal of entries below tau keeps
 * the iterates of a matrix with decaying entries sparse). ---- */

/* Prepares a block-sparse run. n: dimension; block must be 32; the
 * nb = ceil(n / 32) block rows are given by row_ptr_dev (nb + 1 entries,
 * row_ptr[0] = 0, row_ptr[nb] = nnzb) and col_idx_dev (nnzb block columns,
 * strictly increasing within each row); blocks_dev holds nnzb blocks of
 * 32 x 32 FP64 values, each row-major. The pattern must be symmetric and
 * contain every diagonal block; the values must be exactly symmetric
 * (block (J,I) is the transpose of block (I,J)); entries of the last block
 * row and column beyond n are ignored. All three arrays are device memory
 * owned by the caller; blocks_dev must stay valid until sp2_run returns
 * (row_ptr/col_idx are copied during this call). opt->precision must be
 * SP2_FP32 (NULL opt: SP2_FP32 defaults); trunc_tau is the element
 * threshold; every norm applies (the spectral norm's Lanczos products read
 * the block-sparse iterate). The library keeps room for up to
 * min(nb^2, 16 nnzb + 64 nb)
 * blocks per iterate; sp2_run reports SP2_OUT_OF_MEMORY when the fill
 * exceeds it. Errors: SP2_INVALID_ARG (the message names the failed check),
 * SP2_OUT_OF_MEMORY, SP2_HIP_ERROR. After this call sp2_run, sp2_get_info,
 * sp2_get_history and sp2_get_density (dense n x n expansion) apply. */
sp2_status sp2_init_bsr(sp2_ctx ctx, int64_t n, int32_t block, int64_t nnzb,
                        const int32_t* row_ptr_dev, const int32_t* col_idx_dev,
                        const double* blocks_dev, double lambda_min,
                        double lambda_max, int64_t n_occ,
                        const sp2_options* opt);

/* Number of nonzero blocks of the returned block-sparse iterate. */
sp2_status sp2_get_bsr_nnzb(sp2_ctx ctx, int64_t* nnzb);

/* Copies the returned block-sparse iterate (its nonzero blocks only) to
 * caller device arrays: row_ptr_dev (nb + 1), col_idx_dev (nnzb, sorted per
 * row) and blocks_dev (nnzb blocks of 32 x 32, FP64 when as_fp64 != 0 else
 * FP32), nnzb as reported by sp2_get_bsr_nnzb. A block counts as nonzero
 * when its stored form is: where the step after the returned one was
 * scheduled with a stretch (SP2-ACC, Alg. 4), that form is a X~ + c I, so
 * a diagonal block of X~ that is all zero can be among the blocks. */
sp2_status sp2_get_bsr(sp2_ctx ctx, int32_t* row_ptr_dev, int32_t* col_idx_dev,
                       void* blocks_dev, int32_t as_fp64);

/* Work of the last block-sparse run, per step i + 1 (i = 0 .. len-1):
 * stored[i] = blocks of the pattern of X~_{i+1} (the symbolic product),
 * nonzero[i] = nonzero blocks of the stored X~_i (a X~_i + c I under a
 * stretch) that entered the product, products[i]
 * = 32 x 32 block products X_IK X_JK^T computed for the upper blocks.
 * *len receives the number of squares. Any array may be NULL. */
sp2_status sp2_get_bsr_stats(sp2_ctx ctx, int32_t cap, int32_t* len,
                             int64_t* stored, int64_t* nonzero,
                             int64_t* products);

/* ---- Batched purification: many independent matrices, one launch
 * sequence per step, each instance with its own polynomial choices and its
 * own stop (Alg. 2 applied to every instance). A dense run (sp2_init_dense)
 * is a batch of one. ---- */

/* Prepares `count` independent runs. F_dev, n, ldf, lambda_min, lambda_max
 * and n_occ are host arrays of length count; F_dev[b] is a device pointer to
 * instance b's n[b] x n[b] FP64 matrix (row-major, leading dimension
 * ldf[b]), which must stay valid until sp2_batch_run returns. Every instance
 * obeys the sp2_init_dense rules; the options apply to all instances
 * (kernel_config 0 lets the library pick a configuration per instance
 * size). Instances are padded to their tile size and share two iterate
 * pools. Errors: SP2_INVALID_ARG (the message names the instance),
 * SP2_OUT_OF_MEMORY, SP2_HIP_ERROR. */
sp2_status sp2_batch_init(sp2_ctx ctx, int32_t count,
                          const double* const* F_dev, const int64_t* n,
                          const int64_t* ldf, const double* lambda_min,
                          const double* lambda_max, const int64_t* n_occ,
                          const sp2_options* opt);

/* Runs every instance to its own stop; returns SP2_OK once all instances
 * have an outcome (each instance's status, including SP2_NOT_CONVERGED and
 * SP2_DIVERGED, is read with sp2_batch_get), or an error of the run. */
sp2_status sp2_batch_run(sp2_ctx ctx);

/* Outcome of instance idx of the last batch run: n_iter, n_squares and its
 * status (an sp2_status value); when D_dev is not NULL also copies its
 * returned iterate X~_n like sp2_get_density. Any output pointer may be
 * NULL. Errors: SP2_BAD_STATE before a run, SP2_INVALID_ARG. */
sp2_status sp2_batch_get(sp2_ctx ctx, int32_t idx, void* D_dev, int64_t ldd,
                         int32_t as_fp64, int32_t* n_iter, int32_t* n_squares,
                         int32_t* status);

/* History of instance idx, with the conventions of sp2_get_history. */
sp2_status sp2_batch_get_history(sp2_ctx ctx, int32_t idx, int32_t cap,
                                 int32_t* len, double* v, double* t1,
                                 double* t2, int8_t* p, double* r);

/* Device time of the last run (HIP events, first kernel to last) and the
 * number of steps of its longest instance. Either pointer may be NULL. */
sp2_status sp2_batch_get_run_time(sp2_ctx ctx, double* run_ms,
                                  int32_t* steps);

/* ---------------------------------------------------------------------
 * SP2-ACC: a polynomial schedule from homo/lumo bounds with scale-and-fold
 * acceleration (Alg. 3 and Alg. 4 of the paper, sec. 4).
 *
 * Given lambda_min <= homo_out <= homo_in < lumo_in <= lumo_out <=
 * lambda_max (homo_out/homo_in bound the highest occupied eigenvalue of F
 * from below/above, lumo_in/lumo_out the lowest unoccupied one), Alg. 3
 * fixes before the run, for every step i = 1..n_max, the polynomial p_i and
 * the stretch alpha_i >= 1:
 *   X_i = ((1 - alpha_i) I + alpha_i X~_{i-1})^2        (p_i = 1)
 *       = 2 alpha_i X~_{i-1} - (alpha_i X~_{i-1})^2     (p_i = 0)
 * The stretch is switched off (alpha = 1) once both outer-bound distances
 * are below 0.01; the stop test of Alg. 2 is evaluated from step n_min on
 * (instead of 2). Readings fixed here:
 *   - the loop of Alg. 3 runs while the bounds are not idempotent to the
 *     FP64 machine epsilon or the last two polynomials are equal (so the
 *     schedule ends on an alternation); it has at least two steps;
 *   - if the stop has not fired at step n_max, X~_{n_max} is returned with
 *     n = n_max and SP2_OK;
 *   - homo_in > lambda_min and lumo_in < lambda_max are required.
 * Each step computes one square, of the matrix the polynomial is applied
 * to: the epilogue of the previous step (the affine start for step 1)
 * stores Y_i = alpha_i X~_{i-1} + (1 - alpha_i) I for p_i = 1 and
 * Y_i = alpha_i X~_{i-1} for p_i = 0, the square kernel forms S = Y_i^2 and
 * X_i = S or 2 Y_i - S, and the error of X~_{i-1} is taken from Y_i and S
 * in FP64. The returned iterate is recovered from its stored matrix.
 * --------------------------------------------------------------------- */

/* Alg. 3 alone, on the host (no device, no context). accelerate = 0 uses
 * the lower bounds 0 (alpha_i = 1, the setting of Theorem 2). Writes n_min
 * and n_max, and p[i-1], alpha[i-1] for i = 1..n_max when the arrays are
 * given (host arrays of cap entries; either may be NULL; with both NULL cap
 * is ignored). Errors: SP2_INVALID_ARG for bounds that are not finite, out
 * of order or overlapping, for NULL n_min/n_max, or when the schedule needs
 * more than cap (or SP2_MAX_ITER_LIMIT) steps. */
sp2_status sp2_acc_schedule(double lambda_min, double lambda_max,
                            double homo_out, double homo_in, double lumo_in,
                            double lumo_out, int32_t accelerate, int32_t cap,
                            int32_t* n_min, int32_t* n_max, int8_t* p,
                            double* alpha);

/* Switches the instances of the last sp2_init_dense, sp2_init_bsr or
 * sp2_batch_init to SP2-ACC (Alg. 4) for the following runs: count must
 * equal the number of instances (1 for dense and block-sparse contexts);
 * the four host arrays give each instance's bounds, with the lambda_min and
 * lambda_max of its init. The schedule replaces opt->branch; opt->max_iter
 * still caps the squares (a schedule needs up to n_max + 1). A later init
 * returns the context to Alg. 2. Errors: SP2_BAD_STATE before an init,
 * SP2_INVALID_ARG (count mismatch, NULL arrays, or bounds of an instance
 * that sp2_acc_schedule rejects; the message names the instance),
 * SP2_OUT_OF_MEMORY, SP2_HIP_ERROR. */
sp2_status sp2_set_homo_lumo(sp2_ctx ctx, int32_t count,
                             const double* homo_out, const double* homo_in,
                             const double* lumo_in, const double* lumo_out,
                             int32_t accelerate);

/* ---------------------------------------------------------------------
 * McWeeny and McW-ACC (sec. 3 of the paper).
 *
 * X_0 = (mu I - F) / gamma + I / 2 with gamma = 2 max(lambda_max - mu,
 * mu - lambda_min); each step X_i = 3 X_s^2 - 2 X_s^3 with
 * X_s = alpha_i (X~_{i-1} - I/2) + I/2, truncation as in SP2, and the stop
 * at the first step k with log(e_k / 4) / log(e_{k-1}) < 1.8 (e = the
 * Frobenius, mixed or spectral norm of X~_k - X~_k^2, evaluated when
 * 0 < e_{k-1} < 1).
 * Regular McWeeny: alpha = 1. McW-ACC with gap estimate xi:
 * beta_0 = (1 - xi / gamma) / 2, alpha_i = 3 / sqrt(12 beta^2 - 18 beta + 9),
 * beta_i = p_mw(alpha_i (beta_{i-1} - 1/2) + 1/2); the stretch is switched
 * off (alpha = 1) once beta < 0.01 and the stop is tested from the step
 * after (the Frobenius estimate can stop too early while it is on); with
 * SP2_NORM_SPECTRAL the stretch stays on and the stop is tested from step 1
 * as printed.
 * Each step computes two products of the stretched matrix X_s (stored by
 * the previous step's epilogue), S = X_s^2 (which also gives e_{i-1}, from
 * X_s and S in FP64) and X_s S, and forms 3 S - 2 X_s S in the second
 * one's epilogue. The stretches come from the beta recursion, evaluated on
 * the host at this call.
 * --------------------------------------------------------------------- */

/* Switches the instances of the last sp2_init_dense or sp2_batch_init to
 * McWeeny for the following runs. mu (host array of count values) is the
 * chemical potential of each instance, inside [lambda_min, lambda_max]; xi
 * (host array, or NULL for the regular expansion) the McW-ACC gap
 * estimates, each in (0, gamma]. n_occ of the init still selects the
 * trivial cases 0 and n. sp2_get_info's n_squares counts steps (two
 * products each); the history's p entries are 1. A later init returns the
 * context to Alg. 2. Errors: SP2_BAD_STATE before an init, SP2_INVALID_ARG
 * (count mismatch, NULL mu, values out of range (the message names the
 * instance), block-sparse contexts, a context with an SP2-ACC schedule),
 * SP2_OUT_OF_MEMORY, SP2_HIP_ERROR. */
sp2_status sp2_set_mcweeny(sp2_ctx ctx, int32_t count, const double* mu,
                           const double* xi);

/* Installs a table that chooses the square-kernel configuration per
 * instance when opt->kernel_config is 0: for an instance of dimension n and
 * precision p, the first entry e (in the given order) with precision[e] == p
 * and n <= n_max[e] gives the 1-based configuration config_id[e]; instances
 * no entry covers use the library's built-in choice. count = 0 removes the
 * table. The table is copied; it applies to later sp2_init_dense and
 * sp2_batch_init calls on this context. Errors: SP2_INVALID_ARG (unknown
 * configuration id or one whose precision differs from the entry's). */
sp2_status sp2_set_kernel_table(sp2_ctx ctx, int32_t count,
                                const int32_t* precision, const int64_t* n_max,
                                const int32_t* config_id);

/* Number of compiled square-kernel configurations (ids 1..count). */
int32_t sp2_kernel_config_count(void);

/* Describes configuration `id` (1-based): its precision, macro-tile edge
 * (rows and columns of S per workgroup), waves along rows and columns, and
 * the K slice staged per LDS buffer. Any output pointer may be NULL.
 * Errors: SP2_INVALID_ARG for an unknown id. */
sp2_status sp2_kernel_config_info(int32_t id, int32_t* precision,
                                  int32_t* tile, int32_t* waves_m,
                                  int32_t* waves_n, int32_t* k_slice);

/* Name of configuration `id` (1-based): kernel family (F64, F32, B3 padded
 * LDS, B3S swizzled LDS, B3P pre-split operands), macro tile, waves and, where
 * it is not the family's default, the K slice, e.g. "B3P_256_2x4_32". A
 * static string; NULL for an unknown id. */
const char* sp2_kernel_config_name(int32_t id);

/* The square-kernel configuration (1-based id) that instance `index` of the
 * last sp2_init_dense / sp2_batch_init uses (index 0 for a dense context),
 * as chosen by options.kernel_config, the context's kernel table or the
 * built-in default, in that order. *config_id = 0 for an instance with
 * n_occ = 0 or n (no square is computed) and for block-sparse contexts.
 * Errors: SP2_BAD_STATE before an init, SP2_INVALID_ARG. */
sp2_status sp2_get_config(sp2_ctx ctx, int32_t index, int32_t* config_id);

/* ---------------------------------------------------------------------
 * Dense purification without any device allocation, for callers that
 * cannot allocate device memory (code that must not call hipMalloc: tight
 * serving loops, harnesses that forbid allocation). Equivalent to
 * sp2_create + sp2_init_dense + sp2_run + sp2_get_density + sp2_get_info on
 * the given device and stream (same kernels, same work plan, same results
 * bit for bit for the same options and kernel configuration, with
 * tail_split 1), except that every workspace is carved from the library's
 * static scratch array of 64 MiB per device (held until the process ends)
 * and no context, event or pinned host buffer is created.
 *
 * F_dev, n, ldf, lambda_min, lambda_max, n_occ and opt are those of
 * sp2_init_dense (opt may be NULL); the kernel table of a context does not
 * apply (kernel_config 0 picks the library's built-in choice). D_dev
 * receives X~_n like sp2_get_density (ldd >= n, FP64 when as_fp64 != 0).
 * v (host, cap entries, may be NULL when cap is 0) receives the history
 * v[k] = ||X~_k - X~_k^2||_F (NaN past n_squares); n_iter and n_squares
 * (may be NULL) as sp2_get_info. Returns the run outcome like sp2_run.
 *
 * Limits: opt->norm must be SP2_NORM_FROBENIUS, opt->kernel_timing 0 and
 * opt->tail_split 0 or 1 (tail tiles are never split); the run needs
 * about 2 P L w bytes (w = 8 for SP2_FP64, 4 for SP2_FP32) or 16 P L
 * bytes (SP2_BF16X3: FP32 iterates and their bf16 split), plus less than
 * 1 MiB, where P is n rounded up to the square kernel's tile (64 or 128)
 * and L the row stride (P, or P + 128 when P >= 2048 is a multiple of
 * 512): n <= 1920 fits in every precision. Larger inputs, and the options
 * above, return SP2_INVALID_ARG before any work is queued.
 *
 * The scratch array is shared by every call on a device and keeps the last
 * call's contents (each call clears what must start at zero); calls whose
 * work overlaps on one device (other threads or streams) race and must be
 * serialised by the caller. Errors: SP2_INVALID_ARG, SP2_HIP_ERROR. */
sp2_status sp2_run_dense_noalloc(int device, void* hip_stream,
                                 const double* F_dev, int64_t n, int64_t ldf,
                                 double lambda_min, double lambda_max,
                                 int64_t n_occ, const sp2_options* opt,
                                 void* D_dev, int64_t ldd, int32_t as_fp64,
                                 int32_t cap, double* v, int32_t* n_iter,
                                 int32_t* n_squares);

/* Static description of a status code. */
const char* sp2_status_string(sp2_status s);

/* Text of the last error recorded on the context (empty if none). The
 * pointer stays valid until the next call on the context. */
const char* sp2_last_error(sp2_ctx ctx);

#ifdef __cplusplus
}
#endif

#endif /* SP2_H */
