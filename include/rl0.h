/*
 * librl0 -- Robust-l0 decoding of expander sketches on AMD Instinct MI355X (gfx950).
 *
 * Method: Mendoza-Smith, Tanner, Wechsung, "A robust parallel algorithm for
 * combinatorial compressed sensing" (arXiv 1704.09012).  The decoder is Alg. 1
 * (Robust-l0) with the continuous scores of Table "scores"; with sigma = 0 it reduces
 * to Alg. 2 (Parallel-l0).
 *
 * Conventions shared by every entry point
 *   - Pointers without an _h suffix are DEVICE pointers owned by the caller; the
 *     library never frees them.  Pointers with an _h suffix are host pointers.
 *   - The expander A in {0,1}^{m x n} (Definition "Expander matrices": exactly d ones
 *     per column) is passed as A_cols: int32 [n][d], row-major, where A_cols[j*d + p]
 *     is the p-th row index of column j.  The d indices of a column must be distinct,
 *     ascending and in [0, m).
 *   - Vectors are float32: x has n entries, y has m entries.
 *   - `stream` is a hipStream_t (NULL = the default stream).  Calls are
 *     stream-ordered; a call that fills a host-side stats struct synchronises its
 *     stream before returning.
 *   - Return codes: RL0_OK, or a negative RL0_E* code; rl0_last_error() then returns
 *     a message (kept per calling thread).  Non-convergence of the decoder is not an
 *     error (stats.converged = 0).
 *   - Working memory is allocated by the library on first use and cached per
 *     (device, stream); it is released by rl0_release().
 */
#ifndef RL0_H
#define RL0_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RL0_OK 0
#define RL0_EINVAL (-1)     /* bad sizes or parameters, non-finite or out-of-range values */
#define RL0_EINDEX (-2)     /* A_cols: an index out of [0, m), repeated or not ascending */
#define RL0_ENOMEM (-3)     /* device allocation failed */
#define RL0_EHIP (-4)       /* a HIP runtime call failed */
#define RL0_ENOWEIGHTS (-5) /* learned posterior requested without weights */
#define RL0_ERANGE (-6)     /* a value left the 64-bit fixed-point range (|v| >= 2^22) */
#define RL0_EIO (-7)        /* a file could not be read or written, or is no valid checkpoint */

#define RL0_TABLE_N 4096    /* intervals of each score table */
/* floats of a set of score tables given by the caller (rl0_params.tables):
 * T_z [RL0_TABLE_N + 1], T_e [RL0_TABLE_N + 1], inv_h_z, inv_h_e */
#define RL0_TABLES_FLOATS (2 * (RL0_TABLE_N + 1) + 2)
/* laws of the signal entries and of the noise (rl0_params.signal_law / noise_law), each
 * symmetric about 0 and given by its standard deviation */
#define RL0_LAW_GAUSSIAN 0  /* N(0, s^2) */
#define RL0_LAW_LAPLACE 1   /* density exp(-|x|/b) / (2b), b = s / sqrt(2) */
#define RL0_MAX_D 16        /* largest supported column weight d */

/* Decoder parameters (Alg. 1 "KwData": alpha, mu, nu, c; variant flags of Table
 * "variants").  Fill with rl0_params_default() and override fields as needed. */
typedef struct rl0_params {
    int32_t k;              /* sparsity k used by H_k and by rho = k/m in the posteriors */
    float sigma;            /* noise std sigma_n of nu = N(0, sigma_n^2); 0 = noiseless
                               (Parallel-l0 indicator scores) */
    float sigma_signal;     /* signal std sigma_s of mu = N(0, sigma_s^2) (default 1) */
    float alpha;            /* consensus threshold, alpha in (1, d] (default 2) */
    float c;                /* decrement of t per iteration, in (0, 1); 0 selects the
                               paper's rule eq:finetune_c_cont */
    int32_t series_terms;   /* ell, explicit terms of eq:pz_approx/eq:pe_approx (default 4) */
    int32_t max_iters;      /* 0 = ceil(1/c) (t runs 1, 1-c, ... > 0) */
    int32_t l1_test;        /* 0 = column reading sum_{N(j)}|r-omega| <= sum_{N(j)}|r|,
                               1 = literal |r_i - omega| <= |r_i| */
    int32_t posterior;      /* 0 = analytic scores, 1 = learned network (mlp != NULL) */
    const void* mlp;        /* device pointer to the network's fp32 parameters
                               (posterior = 1; see rl0_mlp_num_params) */
    int32_t validate;       /* 1 = check A_cols on the device before decoding */
    int32_t variant;        /* scores of Table "scores": 0 = continuous, 1 = quantised
                               (indicators q_e = 1{p_breve_e >= t}, q_z = 1{p_breve_z >= 1 - t};
                               c = 0 then selects eq:finetune_c_quant) */
    int32_t adaptive_k;     /* 1 = Alg. 1's adaptive_k branch (rl0_decode, analytic scores,
                               sigma > 0): after every accepted iteration the posteriors'
                               sparsity becomes k_0 = max(k - sum_j (1 - p_breve_z(|x_hat_j|)),
                               floor(m/100), 1) and the score tables and outer-test thresholds
                               are rebuilt with rho = k_0/m (c, the t-sweep, H_k's k and the
                               stopping tolerance stay); the sum is taken in units of 2^-30,
                               sum_j rint(2^30 fl32(1 - Tz(|x_hat_j|))).  The host reads k_0
                               back after every iteration, so such a decode is launched
                               eagerly rather than replayed from a graph.  Ignored for
                               sigma = 0.  rl0_step, learned and batched decodes, other
                               laws than Gaussian or given tables: RL0_EINVAL */
    int32_t signal_law;     /* RL0_LAW_* of mu, standard deviation sigma_signal */
    int32_t noise_law;      /* RL0_LAW_* of nu, standard deviation sigma.  Both Gaussian
                               (the default): the tables of eq:pz_approx / eq:pe_approx.
                               Otherwise the posteriors of Thm "Probabilities for general
                               signal and noise distributions" (eq:pz_general,
                               eq:pe_general), the whole series, tabulated like the
                               Gaussian ones (range R = q sqrt(v0)/8, v0 = Var(nu) for z and
                               2 Var(nu) for e, first q >= 8 with p_breve < 2^-27; p_breve =
                               p / p(0); T[0] = 1); the stopping tolerance is m E|eta_i|
                               (m sigma / sqrt(2) for Laplace noise) */
    int32_t log;            /* 1 = record the per-iteration log of the decode (rl0_last_log;
                               a few stores per iteration), 0 (default) = none */
    const float* tables;    /* NULL, or host pointer to RL0_TABLES_FLOATS floats: score
                               tables to use instead of the library's (sigma > 0).  Each
                               table must be finite, start at 1, stay in [0, 1] and be
                               non-increasing; inv_h finite and > 0 (else RL0_EINVAL).
                               Read during the call only (the library keeps a copy, keyed
                               by a 64-bit hash of the floats) */
    int32_t wg_order;       /* 0 (default): the workgroups of the loop kernels take their
                               column and row tiles in launch order; 1: in the reverse
                               order.  The results are the same bits either way (a check
                               that nothing depends on the order in which the hardware
                               runs workgroups).  rl0_decode and rl0_step; batched decodes
                               vary their schedule through rl0_batch_schedule_set */
} rl0_params;

/* What a decode did.  l1 values are ||r_hat||_1; the fixed-point one is exact. */
typedef struct rl0_stats {
    int32_t iterations;     /* loop iterations executed (sweeps run) */
    int32_t accepted;       /* iterations whose ||r||_1 decreased */
    int32_t converged;      /* ||r_hat||_1 <= m sigma sqrt(2/pi) at exit */
    int32_t updates_total;  /* column updates proposed by the sweeps, summed */
    int64_t l1_final_fx;    /* sum_i rint(2^30 |r_hat_i|) */
    double l1_final;        /* l1_final_fx * 2^-30 */
    double l1_tol;          /* m sigma sqrt(2/pi) (Sec. 4 "Stopping conditions") */
    float t_final;          /* t of the last executed iteration */
    int32_t error_flags;    /* device-side flags; nonzero only with an error return */
    float ms_total;         /* device time of the call, from the first kernel of the decode to
                               the copy of x_hat (HIP events on the stream) */
    int32_t fx_inexact_y;   /* entries of y whose conversion to the 2^-40 fixed point rounds
                               (|y_i| < 2^-17 and not a multiple of 2^-40); r_hat <- y is not
                               exact on those rows */
    int32_t fx_inexact_x;   /* updated entries x'_j != 0 whose conversion rounds, summed over
                               the executed iterations (in a learned decode over its learned
                               and analytic sub-iterations) */
    double k_post;          /* the sparsity the posteriors assumed last: k, or with adaptive_k
                               the last k_0 */
} rl0_stats;

/* One executed loop iteration of the last decode (rl0_last_log), recorded on the device
 * by workgroup 0 of the iteration's row kernel and of the kernel that takes the decision
 * on it (the sweep carries no logging code).  The row kernel starts once the sweep has
 * ended, so the span between one record's rows_end and the next one's rows_start holds
 * the next sweep and two kernel boundaries. */
typedef struct rl0_iter_log {
    int64_t l1_trial_fx;    /* ||r||_1 of the iteration's trial iterate (units of 2^-30) */
    int64_t l1_hat_fx;      /* ||r_hat||_1 after the decision on it (Alg. 1's acceptance test) */
    int32_t accepted;       /* that decision */
    int32_t updates;        /* column updates its sweep proposed */
    float t;                /* its t */
    int32_t it;             /* its loop index (learned decodes: the sub-iteration, 2j learned,
                               2j + 1 the analytic retry at the same t) */
    uint64_t rows_start, rows_end;  /* device wall clock (100 MHz) when workgroup 0 of the
                                       iteration's row kernel began and ended */
} rl0_iter_log;

/* Host copy of the decoder's constants, for inspection and tests. */
typedef struct rl0_constants {
    int32_t n_iters;                 /* iterations the t-sweep allows */
    int32_t exact;                   /* 1 when sigma = 0 (indicator scores) */
    double c;                        /* decrement of t actually used */
    double tol;                      /* m sigma sqrt(2/pi) */
    double range_z, range_e;         /* table ranges R_z, R_e */
    float inv_h_z, inv_h_e;          /* fl32(N / R) */
    float table_z[RL0_TABLE_N + 1];  /* fl32(p_breve_z(i R_z / N)) */
    float table_e[RL0_TABLE_N + 1];  /* fl32(p_breve_e(i R_e / N)) */
} rl0_constants;

/* Fill *p with the paper's defaults for an instance of GM(n, m, k, d, N(0,1),
 * N(0, sigma^2)): alpha = 2, c = 0 (= the rule eq:finetune_c_cont: 0.01 if m/n <= 0.05,
 * else 0.025, taken as exact decimals), ell = 4, analytic posterior, validation on.
 * Returns RL0_EINVAL on bad sizes. */
int rl0_params_default(rl0_params* p_h, int32_t n, int32_t m, int32_t d, int32_t k, float sigma);

/* Host only, no device work.  Computes the posteriors p_breve_z, p_breve_e
 * (eq:pz_approx, eq:pe_approx normalised as in eq:breve) and their tables exactly as
 * rl0_decode uses them.  t_h, if not NULL, receives n_iters values t_it = fl32(1 - it c)
 * and tau_h the matching thresholds: row p of a column is a candidate of the outer test
 * 1 - p_breve_z(r_p) >= t (Alg. 1) iff |r_p| >= tau (both float32); each array must hold
 * at least max(ceil(1/c), max_iters) entries. */
int rl0_compute_constants(const rl0_params* p_h, int32_t n, int32_t m, int32_t d,
                          rl0_constants* out_h, float* t_h, float* tau_h);

/* y = A x (Sec. 1; the measurement map of Definition "Generating model").
 * y_i = fl32(2^-40 * sum_{j : i in N(j)} rint(2^40 x_j)), an order-independent integer
 * sum that equals the exactly rounded A x whenever every x_j is a multiple of 2^-40.
 * A_cols [n][d], x [n], y [m] on the device.  Every column of A_cols is validated on the
 * way (RL0_EINDEX, and y is left unwritten); RL0_ERANGE if some |x_j| >= 2^22 (y is then
 * left unwritten too).  Synchronises the stream. */
int rl0_sketch(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* x,
               float* y, void* stream);

/* For callers that cannot allocate device memory (tight serving loops, harnesses that
 * forbid hipMalloc): rl0_sketch with the same arguments, results and errors, whose
 * scratch memory (the 64-bit sums, 8 bytes per row, and the error flags) is a fixed array
 * of the library's, one per GPU, held until the process ends.  It calls no allocating
 * routine.  m must be <= RL0_SKETCH_STATIC_MAX_M (else RL0_EINVAL).  Calls on one GPU share
 * that array: the library serialises its own calls (each synchronises its stream before
 * returning), but two processes' arrays are their own, and calls that overlap on one GPU
 * from outside that order race.  Synchronises the stream. */
#define RL0_SKETCH_STATIC_MAX_M 2097152
int rl0_sketch_static(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* x,
                      float* y, void* stream);

/* Device-side check of A_cols: RL0_EINDEX if any index is outside [0, m) or a column
 * is not strictly ascending.  Synchronises the stream. */
int rl0_validate(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, void* stream);

/* The same check on a host copy of A_cols [n][d] (no device work).  RL0_EINVAL for bad
 * sizes or a NULL pointer. */
int rl0_validate_host(const int32_t* A_cols_h, int32_t n, int32_t m, int32_t d);

/* Bytes of the device workspace a decode of this size allocates (the library allocates
 * it at the first decode and keeps it per device and stream): the fixed-point and
 * rounded residuals, bitmasks, candidate segments, packed indices and loop state
 * described with Alg. 1's data.  0 for invalid sizes (d outside [1, 16] or d > m,
 * k outside [1, m)). */
size_t rl0_workspace_bytes(int32_t n, int32_t m, int32_t d, int32_t k);

/* Robust-l0 (Alg. 1): recover x_hat ~ x from y_hat = A x + eta.
 * A_cols [n][d] and y [m] on the device; x_out [n] (device) receives x_hat, the best
 * accepted iterate.  If st_h != NULL the stream is synchronised and *st_h filled.
 * RL0_EINVAL for d < 1 or d > min(m, RL0_MAX_D), k < 1 or k >= m, alpha outside (1, d],
 * c outside [0, 1), sigma < 0, sigma_signal <= 0; RL0_EINDEX when validate = 1 and
 * A_cols is malformed; RL0_ERANGE if y or an iterate leaves the fixed-point range. */
int rl0_decode(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* y,
               const rl0_params* p_h, float* x_out, rl0_stats* st_h, void* stream);

/* One iteration of Alg. 1's loop body from a caller-held state, for per-iteration
 * checks and resumption.  In: x_hat [n], r_hat [m] (device; r_hat must be the
 * residual of x_hat), *L_hat_h = sum_i rint(2^30 |r_hat_i|), it (t = fl32(1 - it c)).
 * Out: x_hat, r_hat, *L_hat_h updated in place if the iteration is accepted; *accepted_h
 * = 1/0.  Optional device outputs (NULL to skip), per column: updated [n] (int32 0/1),
 * omega [n] (float32, 0 where not updated), x_trial [n] (H_k(x') before acceptance),
 * and r_trial [m].  Synchronises the stream. */
int rl0_step(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* y,
             const rl0_params* p_h, int32_t it, float* x_hat, float* r_hat, int64_t* L_hat_h,
             int32_t* accepted_h, int32_t* updated, float* omega, float* x_trial,
             float* r_trial, void* stream);

/* ---------------------------------------------------------------- batched decoding
 *
 * Many independent Robust-l0 decodes (Alg. 1) of uneven n, m and k in one persistent
 * launch, replayed from a captured hipGraph.  Every workgroup takes the next instance
 * from a queue ordered largest first and decodes it alone; each instance's x_hat and
 * statistics are bit-identical to what rl0_decode returns for it. */

#define RL0_SIZE_CLASSES 12     /* schedule classes by n: class c holds n in [2^(10+c),
                                   2^(11+c)); class 0 also n < 2^10, class 11 n >= 2^21 */
#define RL0_BATCH_MAX_M 524288  /* rows per instance (its outer-test bitmask sits in LDS) */

/* One instance.  A_cols [n][d] (16-byte aligned), y [m] and x_out [n] are device
 * pointers; params as for rl0_decode (posterior = 0). */
typedef struct rl0_problem {
    const int32_t* A_cols;
    int32_t n, m, d;
    const float* y;
    rl0_params params;
    float* x_out;
} rl0_problem;

/* How a batch runs: the launch shape, and per size class the columns each thread takes
 * per tile of the column sweep and the number of workgroups that decode one instance
 * together.  Results do not depend on it. */
typedef struct rl0_batch_schedule {
    int32_t block;                      /* threads per workgroup: 256, 512 or 1024 */
    int32_t per_cu;                     /* resident workgroups per compute unit the
                                           persistent grid is sized for, 1..8 */
    int32_t cols[RL0_SIZE_CLASSES];     /* 1, 2 or 4 */
    int32_t group[RL0_SIZE_CLASSES];    /* 1, 2, 4, 8 or 16 workgroups per instance (a group
                                           splits each step's columns, rows and lists and
                                           meets at bounded barriers; capped by the grid) */
} rl0_batch_schedule;

/* Decode count instances (probs_h: host array).  Every instance is checked as in
 * rl0_decode before anything runs (RL0_EINVAL names the first bad one in
 * rl0_last_error); m must be <= RL0_BATCH_MAX_M, and posterior = 1 and adaptive_k = 1
 * are refused (RL0_EINVAL).  st_h (host, count entries, may be
 * NULL) receives each instance's statistics; the stream is synchronised.  When a
 * decode fails on the device (malformed A_cols with validate = 1, non-finite y,
 * fixed-point range), that instance's x_out and stats.error_flags say so, the others
 * are unaffected, and the call returns the first such error's code.  Uses the
 * calling device's current schedule. */
int rl0_decode_batched(const rl0_problem* probs_h, int32_t count, rl0_stats* st_h, void* stream);

/* Timeline of the last rl0_decode_batched (or autotuning run) on this device and stream,
 * for its first `count` instances (host arrays, count entries each, any may be NULL):
 * when each instance's decode began and ended on the device, in milliseconds after the
 * earliest start, and how many workgroups decoded it.  RL0_EINVAL if there was no such
 * call or count exceeds its instances. */
int rl0_batch_timeline(int32_t count, double* start_ms_h, double* end_ms_h, int32_t* group_h, void* stream);

/* The calling device's batch schedule (a default until set or tuned). */
int rl0_batch_schedule_get(rl0_batch_schedule* out_h);
/* Install a schedule for the calling device; RL0_EINVAL if a field is out of range. */
int rl0_batch_schedule_set(const rl0_batch_schedule* s_h);

/* Autotuner: decodes the given batch under candidate schedules, timing each persistent
 * launch with HIP events (median of `reps` runs): first the launch shape (block, per_cu)
 * over the feasible candidates, then for each size class present, largest first, the
 * columns per thread.  Installs the fastest schedule for the calling device and writes
 * it to best_h (may be NULL); ms_h (may be NULL) receives its median time.  The x_out
 * buffers hold valid decodes afterwards. */
int rl0_autotune_batched(const rl0_problem* probs_h, int32_t count, int32_t reps,
                         rl0_batch_schedule* best_h, double* ms_h, void* stream);

/* ---------------------------------------------------------------- learned decision
 *
 * Not in the paper: a network of a column's residual neighbourhood takes the place of
 * the analytic column test of Alg. 1 (the scores built from eq:pz_approx/eq:pe_approx);
 * H_k, the residual and the acceptance test are unchanged.  Features of column j: its d
 * residual entries sorted ascending, then sigma_n.  Network: d+1 -> 64 (GELU) -> 64
 * (GELU) -> 2 = (logit, value), GELU in its exact erf form.  Column j updates, by
 * x'_j = x_hat_j + value, iff logit >= log(t / (1 - t)).  Parameters: one fp32 device
 * vector of rl0_mlp_num_params(d) values, W1 [64][d+1], b1 [64], W2 [64][64], b2 [64],
 * W3 [2][64], b3 [2], owned by the caller.
 *
 * rl0_decode with params.posterior = 1 and params.mlp = that vector (d <= 15) runs, at
 * every t of the schedule, an iteration with the learned decision and, when it is not
 * accepted, one with the analytic decision at the same t (stats.iterations counts both);
 * inference runs on the matrix cores with bf16 operands and fp32 accumulation.
 * rl0_step with posterior = 1 runs one learned iteration. */

int32_t rl0_mlp_num_params(int32_t d);

/* w [rl0_mlp_num_params(d)] (device) <- weights uniform in +-sqrt(3 / fan_in), zero
 * biases, from a SplitMix64 stream seeded with `seed`.  Synchronises the stream. */
int rl0_mlp_init(float* w, int32_t d, uint64_t seed, void* stream);

/* feats [n][d+1] (device) <- the features of every column on the residual r [m]. */
int rl0_mlp_features(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* r, float sigma,
                     float* feats, void* stream);

/* Training targets for iterate x_hat of a signal x_true (both [n], device): labels
 * [n][2] <- (1 if x_true_j != 0 and |x_true_j - x_hat_j| > 3 sigma / sqrt(d) else 0,
 * x_true_j - x_hat_j). */
int rl0_mlp_labels(const float* x_true, const float* x_hat, int32_t n, int32_t d, float sigma, float* labels,
                   void* stream);

/* Loss over N samples (feats [N][d+1], labels [N][2]): the mean of
 * BCE(logit, y_acc) + lam * (value - y_val)^2.  grad [P] (device) <- its
 * gradient at w (fp32 backpropagation; the shares of the workgroups, which take tiles
 * of 16 samples, are added in a fixed order, so the result does not vary from run to
 * run); *loss_h <- the loss.  Synchronises. */
int rl0_mlp_grad(const float* feats, const float* labels, int32_t N, int32_t d, const float* w, float lam,
                 float* grad, float* loss_h, void* stream);

typedef struct rl0_train_cfg {
    float lr, beta1, beta2, eps;  /* Adam (defaults 1e-3, 0.9, 0.999, 1e-8) */
    float lam;                    /* weight of the value loss (default 1) */
    int32_t batch;                /* samples per step (default 4096) */
    int32_t steps;                /* Adam steps of this call */
    int32_t t0;                   /* steps already taken (Adam's bias correction; batch order) */
} rl0_train_cfg;

/* `steps` Adam steps on (feats, labels) [N] (device, already shuffled): step i takes the
 * (t0 + i) mod floor(N / batch)-th block of `batch` samples.  w, adam_m, adam_v [P]
 * (device) are updated in place (zero m and v before the first call).  *loss_h (may be
 * NULL) <- the mean loss of the last min(steps, 50) steps.  Synchronises. */
int rl0_mlp_train(const float* feats, const float* labels, int64_t N, int32_t d, float* w, float* adam_m,
                  float* adam_v, const rl0_train_cfg* cfg, float* loss_h, void* stream);

/* One Adam update (Kingma and Ba) of w at step t >= 1 with the gradient grad (all [P]
 * = rl0_mlp_num_params(d) values on the device, w, adam_m and adam_v updated in place):
 * m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
 * w <- w - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps), in float32 with the bias
 * corrections taken in double; cfg supplies lr, beta1, beta2 and eps (its other fields are
 * not used).  This is the update rl0_mlp_train applies after each gradient. */
int rl0_mlp_adam(float* w, const float* grad, float* adam_m, float* adam_v, int32_t d, int32_t t,
                 const rl0_train_cfg* cfg, void* stream);

/* packed_h [rl0_mlp_num_params(d)] <- the parameters w_h (host, fp32) as bf16 bit
 * patterns, rounded to nearest even: the weights the matrix-core inference multiplies
 * with (it keeps the biases in fp32; their entries here are the bf16 roundings).  The
 * decoder packs its device copy itself; this is the same rounding on the host. */
int rl0_mlp_pack_bf16(const float* w_h, int32_t d, uint16_t* packed_h);

/* out [N][2] (device) <- (logit, value) of the N samples: fp32 (bf16 = 0) or on the
 * matrix cores as the decoder runs it (bf16 = 1, d <= 15). */
int rl0_mlp_forward(const float* feats, int32_t N, int32_t d, const float* w, float* out, int32_t bf16,
                    void* stream);

/* Checkpoint of a training run of the learned column decision: the parameter vector w
 * and Adam's moments adam_m, adam_v, with what resuming needs.  rl0_mlp_train called with
 * the stored batch and hyper-parameters and t0 = step continues exactly (bit for bit) as
 * the uninterrupted run would have: its batch order and bias corrections depend only on
 * the step, and its gradient sum has a fixed order. */
typedef struct rl0_mlp_ckpt {
    int32_t d;          /* network input width d (features d + 1) */
    int32_t dtype;      /* element type of the arrays: 0 = float32, the only one */
    int64_t P;          /* entries of each array, rl0_mlp_num_params(d) */
    uint64_t seed;      /* seed of the rl0_mlp_init that began the run (kept, not used) */
    int64_t step;       /* Adam steps taken: the t0 of the next rl0_mlp_train */
    rl0_train_cfg cfg;  /* lr, beta1, beta2, eps, lam and batch of those steps; on load
                           steps = 0 and t0 = step (the file keeps neither) */
} rl0_mlp_ckpt;

/* File layout (little-endian, no padding; CRC-32 is that of IEEE 802.3 / zlib):
 *   bytes  0..7   "RL0MLPCK"
 *          8..11  format version, 1
 *         12..15  dtype (0)          16..19  d            20..23  batch
 *         24..31  P                  32..39  seed         40..47  step
 *         48..67  lr, beta1, beta2, eps, lam (float32)
 *         68..71  CRC-32 of the payload
 *         72..75  CRC-32 of bytes 0..71
 *         76..79  zero
 *   payload from byte 80: w, adam_m, adam_v, float32 [P] each (12 P bytes).
 *
 * Save: info_h gives d, seed, step and cfg (its dtype and P are ignored and written as 0
 * and rl0_mlp_num_params(d)); w, adam_m and adam_v are device arrays of that size, read
 * on `stream` (synchronises).  The file is written to "<path>.tmp" and then renamed over
 * path, so an interrupted save leaves any earlier checkpoint at path whole.  RL0_EINVAL
 * for bad arguments, RL0_EIO if the file cannot be written. */
int rl0_mlp_save(const char* path_h, const rl0_mlp_ckpt* info_h, const float* w, const float* adam_m,
                 const float* adam_v, void* stream);

/* Load: reads the whole file and checks it (magic, version, dtype, d in [1, 16],
 * P = rl0_mlp_num_params(d), the file's size, both CRCs, finite hyper-parameters and
 * step >= 0) before anything is written; RL0_EIO names the first check that failed, and
 * then nothing is written.  On success *info_h is filled (may be NULL) and each of w,
 * adam_m, adam_v that is not NULL (device arrays of P floats) receives its array on
 * `stream` (synchronises); with all three NULL only the header is read back, to size
 * the arrays. */
int rl0_mlp_load(const char* path_h, rl0_mlp_ckpt* info_h, float* w, float* adam_m, float* adam_v, void* stream);

/* The per-iteration log of the last rl0_decode (or rl0_step) on this stream, when it ran
 * with params.log = 1: the records of its executed iterations in order, at most cap of
 * them, into out_h (host); *count_h <- the number of executed iterations (0 if that call
 * did not log; records beyond 4096 are not kept).  Batched decodes keep no log.
 * Synchronises the stream. */
int rl0_last_log(rl0_iter_log* out_h, int32_t cap, int32_t* count_h, void* stream);

/* Device index checks.  The library also builds a checked copy of itself
 * (librl0_checked.so): there every data-dependent index of the loop kernels (rows read
 * from A_cols or its packed form, candidate-segment sizes and positions, the sweep's
 * queue, H_k's boundary bucket, columns decoded from keys and written by the copy-out;
 * in the batched kernel rows read from A_cols, queue, change-list and key-list slots, and
 * columns read back from those lists or decoded from keys; in the learned decision's
 * network and feature kernels rows read from A_cols, queue slots and queued columns) is tested against
 * its range before use; an index outside its range is replaced by 0, so that the kernel
 * stays inside its buffers and finishes, and the source line of the first failed check
 * is recorded.  *line_h <- that line since the last call (0: none; the records are then
 * cleared; a line of the batched kernel's source is reported as 100000 + line, one of the
 * network kernel's as 200000 + line, and a single-decode line first, then a batched one,
 * when several failed), or -1 in the normal library, which has no checks.  Synchronises
 * the stream in the checked library. */
int rl0_device_check(int32_t* line_h, void* stream);

/* Kernel timing.  While enabled, rl0_decode launches its kernels one by one (instead of
 * replaying its captured graph), each loop kernel with a pair of HIP events that take
 * the dispatch's own start and end times on the decode stream; once the decode has
 * synchronised the elapsed times are added to running totals.  A decode launches a
 * fixed number of loop iterations; those after the stopping condition held exit early
 * and are counted apart.  Enabling (or disabling) resets the totals. */
int rl0_profile_enable(int32_t enable);

/* Total sweep time in milliseconds and number of timed sweep launches (every launched
 * iteration) since the last rl0_profile_enable. */
int rl0_profile_read(double* sweep_ms_total_h, int64_t* sweep_launches_h);

/* Totals since the last rl0_profile_enable.  ms_total_h (4 doubles): [0] the column
 * sweep, [1] the row kernel (H_k, the trial residual, ||r||_1, the next outer-test
 * bitmasks; for m > 393216 plus the kernel that classifies H_k's candidates before it),
 * over every launched iteration; [2..3] the same over the iterations that ran
 * before the stopping condition.  counts_h (2 int64, may be NULL): the two iteration
 * counts. */
int rl0_profile_read_kernels(double* ms_total_h, int64_t* counts_h);

/* The learned column decision (the network on every column of the residual) as
 * rl0_step with posterior = 1 launches it: total milliseconds and launches since the last
 * rl0_profile_enable, each launch timed with a pair of HIP events on the step's stream. */
int rl0_profile_read_learned(double* ms_total_h, int64_t* launches_h);

/* Message for the last failing call on this thread ("" if none). */
const char* rl0_last_error(void);

/* Frees every cached device buffer of the calling process (all devices, streams). */
void rl0_release(void);

#ifdef __cplusplus
}
#endif

#endif /* RL0_H */
