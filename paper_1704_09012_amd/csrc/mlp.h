// The learned column decision: a 2-hidden-layer network of a column's residual
// neighbourhood, its training kernels (fp32 forward, backward, Adam) and its inference
// on the matrix cores (bf16 operands, fp32 accumulation).
//
// Parameters: one flat fp32 vector, W1 [64][d+1], b1 [64], W2 [64][64], b2 [64],
// W3 [2][64], b3 [2].  Features of column j: its d residual entries sorted ascending,
// then sigma_n.  Output: (logit, value); the column updates iff logit >= log(t/(1-t)),
// by x'_j = x_hat_j + value.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace rl0 {

constexpr int kHidden = 64;
constexpr int kMlpMaxFeatures = 16;   // d + 1 for the matrix-core inference (d <= 15)

inline int mlp_params(int d) {
    const int f = d + 1;
    return kHidden * f + kHidden + kHidden * kHidden + kHidden + 2 * kHidden + 2;
}

// feats [n][d+1]: sorted residual entries of each column's rows, then sigma.
hipError_t launch_mlp_features(const int32_t* A, int n, int m, int d, const float* r, float sigma, float* feats,
                               hipStream_t s);
// labels [n][2]: (1 if x_true_j != 0 and |x_true_j - x_hat_j| > thr else 0, x_true_j - x_hat_j).
hipError_t launch_mlp_labels(const float* x_true, const float* x_hat, int n, double thr, float* labels,
                             hipStream_t s);
// One Adam step: w, m, v in place; c1 = 1 - beta1^t and c2 = 1 - beta2^t.
struct AdamStep {
    float* w;
    float* m;
    float* v;
    float lr, b1, b2, eps, c1, c2;
};

// Workgroups of a gradient launch; each sums the gradient over its share of the samples.
constexpr int kGradMaxGroups = 512;
// Floats of the scratch `part` that launch_mlp_grad needs for column weight d.
size_t mlp_grad_scratch_floats(int d);
// grad [P] = d(mean loss)/dw over the N samples, loss[0] = the mean loss (both written,
// not accumulated).  part: scratch of mlp_grad_scratch_floats(d) floats, the
// workgroups' shares, added in a fixed order (the result is deterministic).  With adam
// the kernel that adds the shares also takes the Adam step on each parameter (that
// kernel starts after every share has been computed from the old weights).
hipError_t launch_mlp_grad(const float* feats, const float* labels, int N, int d, const float* w, float lam,
                           float* grad, float* loss, float* part, hipStream_t s, const AdamStep* adam = nullptr);
// One Adam step in place; c1 = 1 - beta1^t and c2 = 1 - beta2^t are the bias corrections.
hipError_t launch_mlp_adam(float* w, const float* grad, float* m, float* v, int P, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s);
hipError_t launch_zero_floats(float* p, long long count, hipStream_t s);
// out [N][2]: fp32 (bf16 = 0) or matrix-core bf16 (bf16 = 1) inference.
hipError_t launch_mlp_forward(const float* feats, int N, int d, const float* w, float* out, int bf16,
                              hipStream_t s);
// The learned decision of every column: value[j] = the network's value if its logit >=
// logit_t, else NaN (no update).  d <= 15.
struct LearnedCols {
    const int32_t* A;          // [n][d]
    int n, m, d;
    const float* r;            // residual [m]
    const float* r1;           // with pick: the residual if pick[0] != 0
    const int* pick;           // {use r1, stopped} on the device, or nullptr; nothing runs if stopped
    const float* reval_in;     // residual of the last evaluation (cache valid), or nullptr: evaluate all
    float* reval_out;          // <- the residual used, or nullptr
    float* cache;              // [2n] (logit, value) per column: read where unchanged, written where
                               // evaluated; nullptr only without reval_in
    float sigma, logit_t;
    const float* w;            // parameters (fp32)
    float* value;              // [n] out
};
hipError_t launch_learned_cols(const LearnedCols& lc, hipStream_t s);

// The source line of the first failed index check in the learned-decision kernel since
// the last call (0: none; the record is then cleared), or -1 where the checks are not
// compiled in.
hipError_t mlp_check_read(int* line, hipStream_t s);

}  // namespace rl0
