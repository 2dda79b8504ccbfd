// Device kernels of the Robust-l0 decoder and their host-side launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rl0 {

constexpr int kMaxD = 16;
constexpr int kFxShift = 40;   // residual / sketch fixed point: 40 fractional bits
constexpr int kL1Shift = 30;   // ||r||_1 fixed point: 30 fractional bits

enum ErrFlag : int {
    kErrRange = 1,      // a value left the fixed-point range
    kErrIndex = 2,      // A_cols malformed
    kErrNonFinite = 4,  // y holds NaN or Inf
};

// Device-resident state of one decode.  Two-slot fields are indexed by iteration
// parity so that iteration it can clear the slot of it+1 while its own is read.
struct DevState {
    long long L_hat;             // ||r_hat||_1 in units of 2^-30
    long long L_trial[2];        // ||r||_1 of the trial iterate
    int cand_count[2];           // entries in the candidate list
    int done;                    // converged, out of iterations, or failed
    int cur;                     // which residual buffer holds r_hat
    int executed_it;             // last iteration that ran (-1 before any)
    int accepted_flag;           // that iteration was accepted
    int iterations;
    int accepted;
    int updates_total;
    int err;                     // ErrFlag bits
    int n_kept;                  // |supp H_k(x')| of the last iteration
    unsigned long long kth_key;  // smallest key kept by H_k
};

struct DecodeDims {
    int n, m, d, k;
};

struct ScoreTables {
    const float* Tz;   // kTableN + 1 entries
    const float* Te;
    float inv_h_z, inv_h_e;
    int exact;         // indicator scores (sigma = 0)
};

struct IterParams {
    float t;           // threshold of this iteration
    uint32_t tau_bits; // |v| >= tau  <=>  fl32(1 - p_breve_z(v)) >= t
    float alpha;
    int l1_test;
    int it;
    int n_iters;
    double tol_fx;     // tolerance in units of 2^-30
};

struct Workspace {
    long long* Sy;       // rint(2^40 y) [m]
    long long* S;        // trial residual accumulator [m]
    float* r_buf[2];     // r_hat and trial residual [m]
    int* cand_j;         // candidate list (column) [n]
    float* cand_x;       // candidate list (x'_j) [n]
    DevState* st;
};

struct DebugOut {
    int* updated;        // [n] or nullptr
    float* omega;        // [n] or nullptr
    float* x_trial;      // [n] or nullptr
};

hipError_t launch_validate(const int32_t* A, int n, int m, int d, int* err, hipStream_t s);
hipError_t launch_sketch(const int32_t* A, int n, int m, int d, const float* x, float* y,
                         long long* S, int* err, hipStream_t s);
// reset the state, optionally validate A_cols, x_hat = 0, r_hat = y, L_hat = L(y)
hipError_t launch_init(const DecodeDims& dm, const int32_t* A, bool validate, const float* y,
                       float* x_hat, const Workspace& w, const IterParams& ip, hipStream_t s);
// One loop iteration.  ev_sweep[0], ev_sweep[1] (optional) are recorded on s right
// before and after the sweep kernel.
hipError_t launch_iteration(const DecodeDims& dm, const int32_t* A, const float* y,
                            float* x_hat, const Workspace& w, const ScoreTables& tb,
                            const IterParams& ip, const DebugOut& dbg, hipStream_t s,
                            hipEvent_t* ev_sweep = nullptr);
hipError_t launch_fix(const float* y, long long* Sy, int m, DevState* st, hipStream_t s);
hipError_t launch_reset_state(DevState* st, long long L_hat, hipStream_t s);

}  // namespace rl0
