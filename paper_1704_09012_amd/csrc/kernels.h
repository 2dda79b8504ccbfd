// Device kernels of the Robust-l0 decoder and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rl0 {

constexpr int kMaxD = 16;
constexpr int kFxShift = 40;   // residual / sketch fixed point: 40 fractional bits
constexpr int kL1Shift = 30;   // ||r||_1 fixed point: 30 fractional bits
constexpr int kHistBins = 2048;
constexpr int kHistCopies = 8;        // one per XCD: workgroup b adds into copy b % 8
constexpr int kTableStrideFloats = 4100;  // floats between the starts of the two score tables
constexpr int kSweepGridMax = 256;   // workgroups of the sweep (each owns a candidate segment)
constexpr int kRowGrid = 256;        // workgroups of the row kernels (each owns a partial sum)
constexpr int kPreRows = 393216;     // above this m, H_k classifies the candidates in a kernel of its own

enum ErrFlag : int {
    kErrRange = 1,      // a value left the fixed-point range
    kErrIndex = 2,      // A_cols malformed
    kErrNonFinite = 4,  // y holds NaN or Inf
    kErrTimeout = 8,    // a bounded wait between workgroups timed out (batched groups)
};

// Loop state after the decision of one iteration.  Iteration it decides iteration it-1
// at its start and writes slot[it & 1]; it reads slot[(it - 1) & 1], which nothing
// writes during iteration it, so no two kernels race on a slot.
struct Slot {
    long long L_hat;   // ||r_hat||_1 in units of 2^-30
    int cur;           // buffer index holding (x_hat, r_hat, S_hat)
    int done;          // no further iteration runs
    int pending;       // this iteration ran and awaits its decision
    int accepted;      // accepted iterations so far
    int iterations;    // executed iterations so far
    int accepted_last; // the last decision accepted
    int t_step;        // schedule step (index of t) of the last executed iteration
    int last_par;      // parity of the last sweep that ran: its segments hold x_hat
};

// Nothing here is updated by contended atomics: every workgroup writes its own entry
// (candidate segment length, proposed updates, partial ||r||_1) and readers add them up.
// One executed loop iteration, recorded on the device (the layout of rl0_iter_log).
constexpr int kLogCap = 4096;
struct IterLog {
    long long L_trial;     // ||r||_1 of the iteration's trial iterate, units of 2^-30
    long long L_hat;       // ||r_hat||_1 after the decision on the iteration
    int accepted;          // that decision
    int updates;           // column updates the iteration's sweep proposed
    float t;               // the iteration's t
    int it;                // its loop index (the sub-iteration index in a learned decode)
    unsigned long long rows_start, rows_end;     // wall clock (100 MHz) of workgroup 0 in the row kernel
};

struct DevState {
    Slot slot[2];
    unsigned long long kth_key[2];        // smallest key H_k keeps
    int updates_total;                    // column updates proposed, summed over iterations
    int err;                              // ErrFlag bits
    int inexact_y;                        // entries of y whose fixed-point conversion rounds
    int inexact_x;                        // updated x'_j != 0 whose conversion rounds (all sweeps)
    int peek_cur, peek_done;              // the coming decision, evaluated ahead (learned decode,
    int peek_acc;                         //   adaptive_k): buffer, stop, accepted
    long long adapt_sum;                  // sum_j rint(2^30 fl32(1 - Tz(|x_hat_j|))) (adaptive_k)
    int bucket_n[2];                      // entries of H_k's boundary bucket listed by k_hk_classify
    int seg_count[2][kSweepGridMax];      // candidates written by each sweep workgroup
    int seg_front[2][kSweepGridMax];      //   of which at the segment's front (tested columns)
    int seg_nz[2][kSweepGridMax];         //   of which with x' != 0
    int seg_updates[2][kSweepGridMax];    // updates proposed by each sweep workgroup
    long long L_part[2][kRowGrid];        // partial ||r||_1 of the trial residual
    unsigned flag_part[2][2][kRowGrid];   // rows passing the next outer test, per iteration parity,
                                          // bitmask buffer and row workgroup (selects the sweep's
                                          // dense mode)
    unsigned hk_hist[2][kHistCopies][kHistBins];   // nonzero candidates by the top 11 bits of
                                                   // |x'_j|, one copy per XCD (added up by H_k)
    IterLog log[kLogCap];                 // per executed iteration, by its ordinal (not cleared:
                                          // a decode writes the records of the iterations it runs)
};

struct DecodeDims {
    int n, m, d, k;
};

struct ScoreTables {
    const float* Tz;   // kTableN + 1 entries, 16-byte aligned
    const float* Te;   // Tz + kTableStrideFloats
    float inv_h_z, inv_h_e;
    int exact;         // indicator scores (sigma = 0)
    uint32_t e_zero_bits;   // |a| >= this (float bits)  =>  e-score 0
    // quantised scores of one iteration (Table "scores", middle column): q_e = 1 iff
    // |a| <= qe_bits (float bits), q_z = 1 iff |v| <= qz_bits
    int quant = 0;
    uint32_t qe_bits = 0, qz_bits = 0;
};

struct IterParams {
    float t;              // threshold of this iteration
    uint32_t tau_bits;    // |v| >= tau  <=>  fl32(1 - p_breve_z(v)) >= t
    uint32_t tau_next;    // the same for iteration it + 1 (bitmask for the next sweep)
    float alpha;
    int l1_test;
    int it;
    int n_iters;
    double tol_fx;        // tolerance in units of 2^-30 (negative: never converged)
    int step = 0;         // index of t in the schedule (= it, except in the learned decode)
    int retry = 0;        // 1: an analytic retry, skipped when the iteration before was accepted
    int quant = 0;        // quantised scores, with this iteration's thresholds:
    uint32_t qe_bits = 0; //   q_e(a) = 1 iff bits(|a|) <= qe_bits
    uint32_t qz_bits = 0; //   q_z(v) = 1 iff bits(|v|) <= qz_bits
    int log = 0;          // record the iteration in the per-iteration log
    int wg_rev = 0;       // the loop kernels' workgroups take their tiles in reverse order
};

// Double-buffered decoder state; index b in {0, 1} is selected by Slot::cur.  x_hat
// itself lives in the candidate segments (see the sweep kernel).
struct Workspace {
    long long* Sy;        // rint(2^40 y) [m]
    long long* S[2];      // fixed-point residual [m]
    long long* D;         // [m] change of the residual during an iteration (zero between iterations)
    float* r[2];          // float32 residual [m]
    uint32_t* bm[2];      // bit i: |r[b]_i| >= tau of the next sweep [ceil(m/32)]
    uint32_t* bs[2];      // bit g: some row of 8g .. 8g + 7 has its bit set in bm[b] [ceil(m/256)]
    int* cand_j[2];       // candidate list per iteration parity, one segment per sweep
    float* cand_x[2];     //   workgroup of seg_cap entries: column j, x'_j and
    float* cand_h[2];     //   x_hat_j (0 if j was not in the support)
    float* learned;       // [n] learned decisions of the current iteration (NaN: none)
    float* lcache;        // [2n] the network's (logit, value) per column at its last evaluation
    float* reval[2];      // [m] residuals the learned decisions were last evaluated on
    float* ystage;        // [m] y of a decode replayed on staging buffers
    float* xstage;        // [n] its x_hat before the copy out
    uint4* Apk;           // [n] A_cols packed into one 16-byte word per column
    unsigned long long* bkey[2];   // H_k's boundary bucket (key, x'_j) per iteration parity,
    float* bx[2];                  //   one entry per candidate at most (large m only, else null)
    int seg_cap;          // entries per segment
    int sweep_grid;       // sweep workgroups (= segments)
    DevState* st;
};

struct DebugOut {
    int* updated;        // [n] or nullptr (zeroed by the caller)
    float* omega;        // [n] or nullptr (zeroed by the caller)
};

// The source line of the first failed index check in the loop kernels since the last
// call (0: none), which is then cleared; -1 when the library was built without the checks.
hipError_t device_check_read(int* line, hipStream_t s);

size_t workspace_bytes(int n, int m);
void carve_workspace(void* base, int n, int m, Workspace* w);

hipError_t launch_validate(const int32_t* A, int n, int m, int d, int* err, hipStream_t s);
hipError_t launch_sketch(const int32_t* A, int n, int m, int d, const float* x, float* y,
                         long long* S, int* err, hipStream_t s);
hipError_t launch_clear_state(DevState* st, hipStream_t s);
hipError_t launch_zero_i32(int* p, long long count, hipStream_t s);
hipError_t launch_zero_f32(float* p, long long count, hipStream_t s);
hipError_t launch_copy_f32(const float* src, float* dst, long long count, hipStream_t s);

// Prepare a run that starts at iteration it0 from x_hat0 (nullptr: x = 0); x_zero, when
// given, is cleared on the way (the decode's output, written at its end).
// validate: check A_cols first (a malformed A stops the run before any sweep).
hipError_t launch_prepare(const DecodeDims& dm, const int32_t* A, bool validate, const float* y,
                          const float* x_hat0, const Workspace& w, const IterParams& ip0,
                          hipStream_t s, float* x_zero = nullptr);
// One loop iteration (the sweep, then H_k with the rows; for m > kPreRows H_k's
// classification kernel between them).  ev (optional, 6 events) gets the start and end of
// the sweep dispatch in ev[0..1], of the classification in ev[2..3] and of the row dispatch
// in ev[4..5].  With
// `learned` (per column: the update, NaN for none) the sweep takes those decisions in
// place of the analytic column test.
hipError_t launch_iteration(const DecodeDims& dm, const int32_t* A, const Workspace& w,
                            const ScoreTables& tb, const IterParams& ip, const DebugOut& dbg,
                            hipStream_t s, const hipEvent_t* ev = nullptr, const float* learned = nullptr);
// The decision the next sweep will take, written ahead to DevState::peek_cur/peek_done/
// peek_acc (ip.it = that sweep's iteration).
hipError_t launch_peek(const Workspace& w, const IterParams& ip, hipStream_t s);
// adaptive_k, after iteration it (ip.it = it + 1, whose decision launch_peek evaluated):
// DevState::adapt_sum <- sum over x_hat = H_k(x') of iteration it (were it accepted) of
// rint(2^30 fl32(1 - Tz(|x_hat_j|))), on the tables of tb.
hipError_t launch_adapt_sum(const Workspace& w, const ScoreTables& tb, int it, hipStream_t s);
// The outer-test bitmask (and, for large m, its summary and flagged-row counts) of the
// residual buffer `buf` redone for the threshold tau, after the posteriors changed
// (adaptive_k); it = the iteration that produced that residual.
hipError_t launch_rebuild_outer(const DecodeDims& dm, const Workspace& w, int buf, uint32_t tau, int it,
                                hipStream_t s);
// Decide the last iteration (ip_last.it = n_iters) and write x_out = x_hat (x_zeroed: x_out
// already holds zeros).
hipError_t launch_finish(const DecodeDims& dm, const Workspace& w, const IterParams& ip_last,
                         float* x_out, hipStream_t s, bool x_zeroed = false);
// After launch_finish: H_k(x') of the last executed iteration, zero elsewhere.
hipError_t launch_trial_out(const DecodeDims& dm, const Workspace& w, int it_end, float* x_trial,
                            hipStream_t s);

}  // namespace rl0
