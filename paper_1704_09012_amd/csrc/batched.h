// Batched decoding: many independent Robust-l0 decodes of uneven size in one persistent
// launch.  Each workgroup takes instances from a queue (largest first) and runs the
// whole of Alg. 1 for one instance on its own, so no instance waits on another and the
// launch needs no grid-wide synchronisation.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rl0 {

constexpr int kBatchMaxRows = 1 << 19;   // m of one instance: its outer-test bitmask sits in LDS

// One instance, as the persistent kernel reads it (device memory).
struct BatchProblem {
    const int32_t* A;        // [n][d] row indices, ascending per column, 16-byte aligned
    const float* y;          // [m]
    float* x;                // [n] output; holds x_hat during the decode
    long long* S;            // [m] workspace: fixed-point residual of x_hat (of x' mid-iteration)
    float* xp;               // [n] workspace: x' (equals x_hat between iterations)
    int* stamp;              // [n] workspace: last iteration that put the column on the change list
    int* chg;                // [n] workspace: change list of the current iteration
    unsigned long long* keys;  // [n] workspace: H_k keys of the nonzero entries of x' 
    const float* Tz;         // score tables, kTableN + 1 entries each
    const float* Te;
    const uint32_t* tau;     // [n_iters] outer-test threshold bits per iteration
    const uint32_t* qe;      // [n_iters] quantised-score thresholds per iteration (quant = 1)
    const uint32_t* qz;
    double tol_fx;           // stopping tolerance in units of 2^-30
    int n, m, d, k;
    float alpha, inv_h_z, inv_h_e;
    int exact, l1_test, validate, n_iters;
    int quant;               // quantised scores (Table "scores", middle column)
    int cols;                // columns per thread per tile: 1, 2 or 4 (the schedule)
    uint32_t e_zero_bits;    // |a| >= this (float bits)  =>  e-score 0
};

// What a decode did (device memory, one per instance).
struct BatchResult {
    long long L_hat;
    int iterations, accepted, updates_total, err;
};

// The launch-wide part of a schedule.
struct BatchLaunch {
    int block;        // threads per workgroup: 256, 512 or 1024
    int per_cu;       // resident workgroups per compute unit the grid is sized for
};

// Bytes rounded up to the 256-byte alignment every workspace array starts on.
inline size_t al_host(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

size_t batched_lds_bytes(int max_m);
// Workgroups of the batched kernel for column weight d and `block` threads that one
// compute unit holds at once with `lds_bytes` of dynamic LDS (0 if the shape is invalid).
int batched_max_resident(int d, int block, size_t lds_bytes);
// Raise every batched kernel's dynamic LDS limit to what kBatchMaxRows needs (once per
// device, before the first launch or capture).
hipError_t batched_set_lds_limits();
// Zero the queue counter, then the persistent decode of `count` instances taken in
// `order` (indices into probs).  All instances have the same d.
hipError_t launch_batched(int d, const BatchLaunch& L, int grid, size_t lds_bytes, const BatchProblem* probs,
                          const int* order, int count, BatchResult* res, int* counter, hipStream_t s,
                          hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);

}  // namespace rl0
