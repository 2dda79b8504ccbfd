// Batched decoding: many independent Robust-l0 decodes of uneven size in one persistent
// launch.  Each workgroup takes instances from a queue (largest first) and runs the
// whole of Alg. 1 for one instance on its own, so no instance waits on another and the
// launch needs no grid-wide synchronisation.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rl0 {

constexpr int kBatchMaxRows = 1 << 19;   // m of one instance: its outer-test bitmask sits in LDS

struct BatchCtl;

// One instance, as the persistent kernel reads it (device memory).
struct BatchProblem {
    const int32_t* A;        // [n][d] row indices, ascending per column, 16-byte aligned
    const float* y;          // [m]
    float* x;                // [n] output; holds x_hat during the decode
    long long* S;            // [m] workspace: fixed-point residual of x_hat (of x' mid-iteration)
    float* r;                // [m] workspace: fl32 of S, written with the outer-test bitmask at
                             // the start of each iteration (the sweep's residual snapshot)
    float* xp;               // [n] workspace: x' (equals x_hat between iterations)
    int* stamp;              // [n] workspace: last iteration that put the column on the change list
    int* chg;                // [n] workspace: change list of the current iteration
    int* chg2;               // [n] workspace: the second change list of a group (odd iterations)
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
    int group;               // workgroups that decode the instance together (1 = alone)
    BatchCtl* ctl;           // their shared state (group > 1)
    int cols;                // columns per thread per tile: 1, 2 or 4 (the schedule)
    uint32_t e_zero_bits;    // |a| >= this (float bits)  =>  e-score 0
};

// Shared state of the G workgroups that decode one instance together (device memory,
// zeroed before every launch).  Counters that live for one iteration come in two copies,
// by iteration parity: the copy of iteration it + 1 is cleared during iteration it.
struct BatchCtl {
    unsigned bar;            // barrier arrivals so far (all members)
    int abort;               // a member's bounded wait timed out: every member leaves
    int err;                 // ErrFlag bits of the instance
    int nchg[2], nupd[2], nzd[2], nkeys[2];
    long long L0;            // ||r||_1 of r = y, summed over the members
    long long dl[2];         // change of ||r||_1 by the iteration's residual change
    long long dsupp[2];      // change of |supp x'|
    int inexact_y;           // rounded conversions of y, summed over the members
    int inexact_x;           // rounded conversions of updated x'_j, over the iterations
    int pad[8];
};
static_assert(sizeof(BatchCtl) % 16 == 0, "BatchCtl keeps 16-byte alignment");

// A ticket of the queue: instance index and member (part) of its group.
constexpr int kTicketParts = 32;   // tickets are instance * kTicketParts + part
constexpr int kMaxGroup = 16;      // largest group of workgroups on one instance

// What a decode did (device memory, one per instance).
struct BatchResult {
    long long L_hat;
    int iterations, accepted, updates_total, err;
    unsigned long long t_start, t_end;   // wall clock (100 MHz) when the decode began and ended
    int inexact_y;   // entries of y whose 2^-40 fixed-point conversion rounds
    int inexact_x;   // updated x'_j != 0 whose conversion rounds, over the executed iterations
};

// The launch-wide part of a schedule.
struct BatchLaunch {
    int block;        // threads per workgroup: 256, 512 or 1024
    int per_cu;       // resident workgroups per compute unit the grid is sized for
    int r_off = 0;    // float offset in dynamic LDS of the residual snapshot's region
    int r_rows = 0;   // its rows: instances with m <= r_rows keep the snapshot in LDS
};

// Bytes rounded up to the 256-byte alignment every workspace array starts on.
inline size_t al_host(size_t b) { return (b + 255) & ~static_cast<size_t>(255); }

size_t batched_lds_bytes(int max_m);
// Workgroups of the batched kernel for column weight d and `block` threads that one
// compute unit holds at once with `lds_bytes` of dynamic LDS (0 if the shape is invalid).
int batched_max_resident(int d, int block, size_t lds_bytes);
// Static LDS of the batched kernel for column weight d and `block` threads (0 if invalid).
size_t batched_static_lds(int d, int block);
// The source line of the first failed index check in the batched kernel since the last
// call (0: none; the record is then cleared), or -1 where the checks are not compiled in.
hipError_t batched_check_read(int* line, hipStream_t s);
// Raise every batched kernel's dynamic LDS limit to all that the compute unit's LDS leaves
// beside its static LDS (once per device, before the first launch or capture).
hipError_t batched_set_lds_limits();
// Zero the queue counter, then the persistent decode of the `count` tickets in `order`
// (instance * kTicketParts + part; a group's tickets are consecutive).  All instances
// have the same d.  The caller zeroes the groups' BatchCtl blocks first (launch_zero_words).
hipError_t launch_batched(int d, const BatchLaunch& L, int grid, size_t lds_bytes, const BatchProblem* probs,
                          const int* order, int count, BatchResult* res, int* counter, hipStream_t s,
                          hipEvent_t ev_start = nullptr, hipEvent_t ev_stop = nullptr);
// words [count] <- 0 with a fill kernel (capturable).
hipError_t launch_zero_words(int* words, long long count, hipStream_t s);

}  // namespace rl0
