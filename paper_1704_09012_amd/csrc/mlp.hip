// Kernels of the learned column decision (see mlp.h for the network and its layout).
//
// Training runs in fp32: one workgroup takes 64 samples, keeps the weights and every
// activation of its samples in LDS, and adds its share of the gradient of the mean
// loss to a global buffer; Adam then updates the weights elementwise.
//
// Inference on the matrix cores: a wave evaluates the network for its 64 samples with
// v_mfma_f32_16x16x32_bf16.  The products are laid out transposed (hidden units along
// M, samples along N), so each layer's accumulators already sit in the lanes and
// registers that the next layer's B operand needs; the K order of a layer is permuted to
// match and the weights are read from LDS in that order.
#include "mlp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "column_math.h"

#pragma clang fp contract(off)

namespace rl0 {

namespace {

// Checked builds (compiled with RL0_DEVICE_CHECKS=1 into the second copy of the library):
// MCHK(i, n) tests a data-dependent index of the learned-decision kernels (a row read from
// A_cols, a slot of a wave's queue, a queued column) against [0, n).  Outside it, the
// source line of the first failed check is recorded in g_mlp_check_line (read back by
// mlp_check_read) and the index becomes 0, so that the access stays inside its buffer and
// the kernel runs to its end.  In normal builds MCHK(i, n) is i.
#if RL0_DEVICE_CHECKS
__device__ unsigned g_mlp_check_line;

template <class I>
__device__ __forceinline__ I mchk(I i, long long n, unsigned line) {
    const long long v = static_cast<long long>(i);
    if (v >= 0 && v < n) return i;
    atomicCAS(&g_mlp_check_line, 0u, line);
    return static_cast<I>(0);
}
#define MCHK(i, n) mchk((i), static_cast<long long>(n), __LINE__)
#else
#define MCHK(i, n) (i)
#endif

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kGradTile = 16;        // samples per tile of the training kernel
constexpr int kGradBlock = 256;
constexpr int kGradW1Per = (kHidden * (kMaxD + 1) + kGradBlock - 1) / kGradBlock;   // W1 entries per thread
constexpr float kInvSqrt2 = 0.70710678118654752f;
constexpr float kInvSqrt2Pi = 0.39894228040143268f;

__device__ __forceinline__ float gelu(float u) { return 0.5f * u * (1.0f + erff(u * kInvSqrt2)); }

// GELU for the matrix-core inference, whose activations are rounded to bf16 (8
// significant bits) right after: Phi from Abramowitz & Stegun 7.1.26,
//   erf(x) = 1 - (a1 t + a2 t^2 + a3 t^3 + a4 t^4 + a5 t^5) exp(-x^2),  t = 1 / (1 + p x),
// for x = |u| / sqrt(2) >= 0 (absolute error <= 1.5e-7), with the hardware's reciprocal
// and base-2 exponential.  With tail = 1 - Phi(|u|) = (t/2)(a1 + a2 t + ...) exp(-x^2),
// gelu(u) = u Phi(u) = max(u, 0) - |u| tail for either sign of u; 1/sqrt(2) is folded into
// p and 1/2 into the a's, so that a GELU is 11 full-rate and 2 transcendental instructions.
__device__ __forceinline__ float gelu_bf16(float u) {
    constexpr float p = 0.3275911f * kInvSqrt2;
    constexpr float a1 = 0.5f * 0.254829592f, a2 = 0.5f * -0.284496736f, a3 = 0.5f * 1.421413741f,
                    a4 = 0.5f * -1.453152027f, a5 = 0.5f * 1.061405429f;
    constexpr float kHalfLog2e = 0.72134752044448170f;   // log2(e) / 2
    const float a = fabsf(u);
    const float t = __builtin_amdgcn_rcpf(fmaf(p, a, 1.0f));
    float q = fmaf(t, a5, a4);
    q = fmaf(t, q, a3);
    q = fmaf(t, q, a2);
    q = fmaf(t, q, a1);
    const float e = __builtin_amdgcn_exp2f((u * u) * -kHalfLog2e);   // exp(-x^2)
    const float tail = (t * q) * e;
    return fmaf(-a, tail, fmaxf(u, 0.0f));
}

__device__ __forceinline__ float gelu_grad(float u) {
    return 0.5f * (1.0f + erff(u * kInvSqrt2)) + u * expf(-0.5f * u * u) * kInvSqrt2Pi;
}

// ------------------------------------------------------------------ features, labels

template <int D>
__global__ void k_mlp_features(const int32_t* __restrict__ A, int n, int m, const float* __restrict__ r, float sigma,
                               float* __restrict__ feats) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float v[D];
#pragma unroll
    for (int p = 0; p < D; ++p) v[p] = r[MCHK(A[static_cast<size_t>(j) * D + p], m)];
    // insertion sort, ascending
#pragma unroll
    for (int a = 1; a < D; ++a)
#pragma unroll
        for (int b = a; b > 0; --b) {
            const float lo = fminf(v[b - 1], v[b]), hi = fmaxf(v[b - 1], v[b]);
            v[b - 1] = lo;
            v[b] = hi;
        }
    float* out = feats + static_cast<size_t>(j) * (D + 1);
#pragma unroll
    for (int p = 0; p < D; ++p) out[p] = v[p];
    out[D] = sigma;
}

__global__ void k_mlp_labels(const float* __restrict__ x_true, const float* __restrict__ x_hat, int n, double thr,
                             float* __restrict__ labels) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float xt = x_true[j];
    const float diff = xt - x_hat[j];
    const bool acc = xt != 0.0f && static_cast<double>(fabsf(diff)) > thr;
    labels[2 * static_cast<size_t>(j)] = acc ? 1.0f : 0.0f;
    labels[2 * static_cast<size_t>(j) + 1] = diff;
}

// ------------------------------------------------------------------ training

// One workgroup takes the tiles blockIdx.x, blockIdx.x + gridDim.x, ... of kGradTile
// samples each and keeps the weights, the tile's features, labels, pre-activations and
// activations in LDS.  Its share of the gradient of the mean loss is summed over its
// tiles in registers and written to part[blockIdx.x][P], its share of the loss to
// part[gridDim.x * P + blockIdx.x]; k_mlp_grad_sum adds the shares in a fixed order, so
// the gradient does not depend on the order in which workgroups run.  Thread tid works
// on sample tid / 16 and hidden units 4 (tid % 16) .. + 3 of a tile's activations.
__global__ __launch_bounds__(kGradBlock) void k_mlp_grad(const float* __restrict__ feats,
                                                         const float* __restrict__ labels, int N, int F,
                                                         const float* __restrict__ w, float lam, float inv_n,
                                                         float* __restrict__ part) {
    extern __shared__ __attribute__((aligned(16))) float lds[];
    __shared__ float red[kGradBlock / 64];
    const int P = kHidden * F + kHidden + kHidden * kHidden + kHidden + 2 * kHidden + 2;
    constexpr int kAct = kGradTile * kHidden;
    float* W = lds;                          // the parameters, in the layout of mlp.h
    float* W2T = W + ((P + 3) & ~3);         // W2 transposed, [k][h] (16-byte aligned)
    float* Fs = W2T + kHidden * kHidden;     // [kGradTile][F]
    float* Z1 = Fs + kGradTile * F;          // [kGradTile][kHidden]; later dZ1
    float* H1 = Z1 + kAct;
    float* Z2 = H1 + kAct;                   // later dZ2
    float* H2 = Z2 + kAct;
    float* dO = H2 + kAct;                   // [kGradTile][2]
    float* Ys = dO + 2 * kGradTile;          // [kGradTile][2]
    const int oW1 = 0, ob1 = kHidden * F, oW2 = ob1 + kHidden, ob2 = oW2 + kHidden * kHidden,
              oW3 = ob2 + kHidden, ob3 = oW3 + 2 * kHidden;
    const float* W1 = W + oW1;
    const float* b1 = W + ob1;
    const float* W2 = W + oW2;
    const float* b2 = W + ob2;
    const float* W3 = W + oW3;
    const float* b3 = W + ob3;
    const int tid = threadIdx.x;
    const int sa = tid >> 4, hb = tid & 15;  // sample and unit group of the activation work
    for (int i = tid; i < P; i += kGradBlock) W[i] = w[i];
    for (int i = tid; i < kHidden * kHidden; i += kGradBlock) W2T[i] = w[oW2 + (i & 63) * kHidden + (i >> 6)];
    float gW2[16], gW1[kGradW1Per];
#pragma unroll
    for (int c = 0; c < 16; ++c) gW2[c] = 0.0f;
#pragma unroll
    for (int c = 0; c < kGradW1Per; ++c) gW1[c] = 0.0f;
    float gb1 = 0.0f, gb2 = 0.0f, gW3 = 0.0f, gb3 = 0.0f, lsum = 0.0f;
    __syncthreads();
    for (int tile = blockIdx.x; tile * kGradTile < N; tile += gridDim.x) {
        const int s0 = tile * kGradTile;
        const int ns = min(kGradTile, N - s0);
        for (int i = tid; i < kGradTile * F; i += kGradBlock)
            Fs[i] = i / F < ns ? feats[static_cast<size_t>(s0) * F + i] : 0.0f;
        if (tid < 2 * kGradTile) Ys[tid] = (tid >> 1) < ns ? labels[2 * static_cast<size_t>(s0) + tid] : 0.0f;
        __syncthreads();
        // layer 1
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int h = 4 * hb + i;
            float a = 0.0f;
            for (int k = 0; k < F; ++k) a = a + W1[h * F + k] * Fs[sa * F + k];
            a = a + b1[h];
            Z1[sa * kHidden + h] = a;
            H1[sa * kHidden + h] = gelu(a);
        }
        __syncthreads();
        // layer 2, from the transposed weights (a wave's 16 unit groups read 256
        // consecutive bytes)
        {
            float a0 = 0.0f, a1 = 0.0f, a2 = 0.0f, a3 = 0.0f;
            for (int k = 0; k < kHidden; ++k) {
                const float hv = H1[sa * kHidden + k];
                const float4 wv = *reinterpret_cast<const float4*>(&W2T[k * kHidden + 4 * hb]);
                a0 = a0 + wv.x * hv;
                a1 = a1 + wv.y * hv;
                a2 = a2 + wv.z * hv;
                a3 = a3 + wv.w * hv;
            }
            const float av[4] = {a0, a1, a2, a3};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int h = 4 * hb + i;
                const float z = av[i] + b2[h];
                Z2[sa * kHidden + h] = z;
                H2[sa * kHidden + h] = gelu(z);
            }
        }
        __syncthreads();
        // outputs, loss and the gradient at the outputs (one thread per sample)
        if (tid < kGradTile) {
            const int sm = tid;
            float o0 = 0.0f, o1 = 0.0f;
            for (int k = 0; k < kHidden; ++k) {
                o0 = o0 + W3[k] * H2[sm * kHidden + k];
                o1 = o1 + W3[kHidden + k] * H2[sm * kHidden + k];
            }
            o0 = o0 + b3[0];
            o1 = o1 + b3[1];
            float g0 = 0.0f, g1 = 0.0f;
            if (sm < ns) {
                const float ya = Ys[2 * sm], yv = Ys[2 * sm + 1];
                const float dv = o1 - yv;
                lsum = lsum + (fmaxf(o0, 0.0f) - ya * o0 + log1pf(expf(-fabsf(o0))) + lam * dv * dv);
                const float sig = 1.0f / (1.0f + expf(-o0));
                g0 = (sig - ya) * inv_n;
                g1 = 2.0f * lam * dv * inv_n;
            }
            dO[2 * sm] = g0;
            dO[2 * sm + 1] = g1;
        }
        __syncthreads();
        // dZ2 = (dO W3) * gelu'(Z2), in place of Z2; W3 and b3 from dO and H2
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int h = 4 * hb + i, e = sa * kHidden + h;
            const float g = dO[2 * sa] * W3[h] + dO[2 * sa + 1] * W3[kHidden + h];
            Z2[e] = g * gelu_grad(Z2[e]);
        }
        if (tid < 2 * kHidden) {
            const int o = tid >> 6, k = tid & 63;
            for (int sm = 0; sm < kGradTile; ++sm) gW3 = gW3 + dO[2 * sm + o] * H2[sm * kHidden + k];
        }
        if (tid < 2)
            for (int sm = 0; sm < kGradTile; ++sm) gb3 = gb3 + dO[2 * sm + tid];
        __syncthreads();
        // W2 [h][k] += sum_s dZ2[s][h] H1[s][k] (thread: h = tid / 4, 16 consecutive k); b2
        {
            const int h = tid >> 2, k0 = 16 * (tid & 3);
            for (int sm = 0; sm < kGradTile; ++sm) {
                const float dz = Z2[sm * kHidden + h];
#pragma unroll
                for (int c = 0; c < 16; c += 4) {
                    const float4 hv = *reinterpret_cast<const float4*>(&H1[sm * kHidden + k0 + c]);
                    gW2[c] = gW2[c] + dz * hv.x;
                    gW2[c + 1] = gW2[c + 1] + dz * hv.y;
                    gW2[c + 2] = gW2[c + 2] + dz * hv.z;
                    gW2[c + 3] = gW2[c + 3] + dz * hv.w;
                }
            }
        }
        if (tid < kHidden)
            for (int sm = 0; sm < kGradTile; ++sm) gb2 = gb2 + Z2[sm * kHidden + tid];
        // dZ1 = (dZ2 W2) * gelu'(Z1), in place of Z1 (nothing else reads Z1 now)
        {
            float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, g3 = 0.0f;
            for (int h = 0; h < kHidden; ++h) {
                const float dz = Z2[sa * kHidden + h];
                const float4 wv = *reinterpret_cast<const float4*>(&W2[h * kHidden + 4 * hb]);
                g0 = g0 + dz * wv.x;
                g1 = g1 + dz * wv.y;
                g2 = g2 + dz * wv.z;
                g3 = g3 + dz * wv.w;
            }
            const float gv[4] = {g0, g1, g2, g3};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int e = sa * kHidden + 4 * hb + i;
                Z1[e] = gv[i] * gelu_grad(Z1[e]);
            }
        }
        __syncthreads();
        // W1 [h][k] += sum_s dZ1[s][h] F[s][k]; b1
#pragma unroll
        for (int c = 0; c < kGradW1Per; ++c) {
            const int e = tid + c * kGradBlock;
            if (e < kHidden * F) {
                const int h = e / F, k = e % F;
                for (int sm = 0; sm < kGradTile; ++sm) gW1[c] = gW1[c] + Z1[sm * kHidden + h] * Fs[sm * F + k];
            }
        }
        if (tid < kHidden)
            for (int sm = 0; sm < kGradTile; ++sm) gb1 = gb1 + Z1[sm * kHidden + tid];
        __syncthreads();   // the next tile overwrites Fs, Ys and the activations
    }
    float* __restrict__ out = part + static_cast<size_t>(blockIdx.x) * P;
    {
        const int h = tid >> 2, k0 = 16 * (tid & 3);
#pragma unroll
        for (int c = 0; c < 16; ++c) out[oW2 + h * kHidden + k0 + c] = gW2[c];
    }
#pragma unroll
    for (int c = 0; c < kGradW1Per; ++c) {
        const int e = tid + c * kGradBlock;
        if (e < kHidden * F) out[oW1 + e] = gW1[c];
    }
    if (tid < kHidden) {
        out[ob1 + tid] = gb1;
        out[ob2 + tid] = gb2;
    }
    if (tid < 2 * kHidden) out[oW3 + tid] = gW3;
    if (tid < 2) out[ob3 + tid] = gb3;
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off);
    if ((tid & 63) == 0) red[tid >> 6] = lsum;
    __syncthreads();
    if (tid == 0) part[static_cast<size_t>(gridDim.x) * P + blockIdx.x] = (red[0] + red[1]) + (red[2] + red[3]);
}

// One Adam step of parameter i with gradient gi (c1 = 1 - beta1^t, c2 = 1 - beta2^t).
__device__ __forceinline__ void adam_update(const AdamStep& a, int i, float gi) {
    const float mi = a.b1 * a.m[i] + (1.0f - a.b1) * gi;
    const float vi = a.b2 * a.v[i] + (1.0f - a.b2) * gi * gi;
    a.m[i] = mi;
    a.v[i] = vi;
    a.w[i] = a.w[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
}

// grad[p] = the sum of the G shares part[g][p]: thread slice sl adds shares sl, sl + 16,
// ... (all loaded first; the missing ones add 0), then the 16 partial sums are added in
// a fixed order.  loss[0] = inv_n times the sum of the G loss shares.  With ADAM the
// step then updates parameter p.
constexpr int kSumSlices = 16;
constexpr int kSharesPerSlice = (kGradMaxGroups + kSumSlices - 1) / kSumSlices;
template <bool ADAM>
__global__ __launch_bounds__(64 * kSumSlices) void k_mlp_grad_sum(const float* __restrict__ part, int G, int P,
                                                                  float inv_n, float* __restrict__ grad,
                                                                  float* __restrict__ loss, AdamStep adam) {
    __shared__ float red[kSumSlices][64];
    const int c = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int p = blockIdx.x * 64 + c;
    float v[kSharesPerSlice];
#pragma unroll
    for (int q = 0; q < kSharesPerSlice; ++q) {
        const int g = sl + kSumSlices * q;
        v[q] = (p < P && g < G) ? part[static_cast<size_t>(g) * P + p] : 0.0f;
    }
    float a = 0.0f;
#pragma unroll
    for (int q = 0; q < kSharesPerSlice; ++q) a = a + v[q];
    red[sl][c] = a;
    __syncthreads();
    if (sl == 0 && p < P) {
        float t = 0.0f;
        for (int q = 0; q < kSumSlices; ++q) t = t + red[q][c];
        grad[p] = t;
        if (ADAM) adam_update(adam, p, t);
    }
    if (blockIdx.x == 0 && sl == 1) {
        float l = 0.0f;
        for (int g = c; g < G; g += 64) l = l + part[static_cast<size_t>(G) * P + g];
        for (int off = 32; off > 0; off >>= 1) l += __shfl_down(l, off);
        if (c == 0) loss[0] = l * inv_n;
    }
}

__global__ void k_mlp_adam(const float* __restrict__ g, int P, AdamStep a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < P) adam_update(a, i, g[i]);
}

__global__ void k_zero_floats(float* __restrict__ p, long long count) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0f;
}

// ------------------------------------------------------------------ fp32 inference

__global__ void k_mlp_forward_f32(const float* __restrict__ feats, int N, int F, const float* __restrict__ w,
                                  float* __restrict__ out) {
    extern __shared__ float W[];
    const int P = kHidden * F + kHidden + kHidden * kHidden + kHidden + 2 * kHidden + 2;
    for (int i = threadIdx.x; i < P; i += blockDim.x) W[i] = w[i];
    __syncthreads();
    const int sm = blockIdx.x * blockDim.x + threadIdx.x;
    if (sm >= N) return;
    const float* W1 = W;
    const float* b1 = W1 + kHidden * F;
    const float* W2 = b1 + kHidden;
    const float* b2 = W2 + kHidden * kHidden;
    const float* W3 = b2 + kHidden;
    const float* b3 = W3 + 2 * kHidden;
    float f[kMlpMaxFeatures + 1];
    for (int k = 0; k < F; ++k) f[k] = feats[static_cast<size_t>(sm) * F + k];
    float h1[kHidden];
    for (int h = 0; h < kHidden; ++h) {
        float a = 0.0f;
        for (int k = 0; k < F; ++k) a = a + W1[h * F + k] * f[k];
        h1[h] = gelu(a + b1[h]);
    }
    float o0 = 0.0f, o1 = 0.0f;
    for (int h = 0; h < kHidden; ++h) {
        float a = 0.0f;
        for (int k = 0; k < kHidden; ++k) a = a + W2[h * kHidden + k] * h1[k];
        const float h2 = gelu(a + b2[h]);
        o0 = o0 + W3[h] * h2;
        o1 = o1 + W3[kHidden + h] * h2;
    }
    out[2 * static_cast<size_t>(sm)] = o0 + b3[0];
    out[2 * static_cast<size_t>(sm) + 1] = o1 + b3[1];
}

// ------------------------------------------------------------------ matrix-core inference

constexpr int kInferBlock = 256;
constexpr int kInferWaves = kInferBlock / 64;
constexpr int kQueueCap = 128;   // per-wave queue of samples awaiting the network

// The network in LDS for the matrix cores: every lane's A operand of every product as
// one 16-byte word (bf16), the biases in fp32.  Lane l = 16 g + c of the wave holds
//   A1[mt][l]: W1[16 mt + c][8 g + 0..7] (inputs zero-padded to 16; zero for g >= 2),
//   A2[mt][kt][l]: W2[16 mt + c][32 kt + 4 g + 0..3, 32 kt + 16 + 4 g + 0..3],
//   A3[kt][l]: the same K order of W3 row c (zero for c >= 2).
// The permuted K order of A2 and A3 is the order in which the previous layer's
// activations sit in a lane's registers (see activations()).
struct MlpLds {
    bf16x8 A1[4][64];
    bf16x8 A2[4][2][64];
    bf16x8 A3[2][64];
    float b1[kHidden], b2[kHidden], b3[2];
};

__device__ void load_mlp_lds(MlpLds& L, const float* __restrict__ w, int F) {
    const float* W1 = w;
    const float* b1 = W1 + kHidden * F;
    const float* W2 = b1 + kHidden;
    const float* b2 = W2 + kHidden * kHidden;
    const float* W3 = b2 + kHidden;
    const float* b3 = W3 + 2 * kHidden;
    constexpr int kWords = 4 * 64 + 8 * 64 + 2 * 64;
    // every load reads an address inside w (a padding entry reads a clamped one and is
    // then replaced by 0), so no per-lane branch makes the loads wait for each other
    for (int e = threadIdx.x; e < kWords; e += blockDim.x) {
        const int l = e & 63, g = l >> 4, c = l & 15;
        bf16x8 v;
        if (e < 256) {
            const int mt = e >> 6;
            const float* __restrict__ wr = W1 + (16 * mt + c) * F;
            float t[8];
#pragma unroll
            for (int j = 0; j < 8; ++j) t[j] = wr[min(8 * g + j, F - 1)];
#pragma unroll
            for (int j = 0; j < 8; ++j) v[j] = static_cast<__bf16>(8 * g + j < F ? t[j] : 0.0f);
            L.A1[mt][l] = v;
        } else {
            const bool l2 = e < 768;
            const int q = l2 ? (e - 256) >> 6 : (e - 768) >> 6;
            const int kt = q & 1;
            const bool live = l2 || c < 2;
            const float* row = l2 ? W2 + (16 * (q >> 1) + c) * kHidden : W3 + (live ? c : 0) * kHidden;
            float t0[4], t1[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                t0[j] = row[32 * kt + 4 * g + j];
                t1[j] = row[32 * kt + 16 + 4 * g + j];
            }
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                v[j] = static_cast<__bf16>(live ? t0[j] : 0.0f);
                v[4 + j] = static_cast<__bf16>(live ? t1[j] : 0.0f);
            }
            if (l2)
                L.A2[q >> 1][kt][l] = v;
            else
                L.A3[kt][l] = v;
        }
    }
    for (int i = threadIdx.x; i < kHidden; i += blockDim.x) {
        L.b1[i] = b1[i];
        L.b2[i] = b2[i];
    }
    if (threadIdx.x < 2) L.b3[threadIdx.x] = b3[threadIdx.x];
}

__device__ __forceinline__ bf16x8 zero8() {
    bf16x8 z;
#pragma unroll
    for (int j = 0; j < 8; ++j) z[j] = static_cast<__bf16>(0.0f);
    return z;
}

// Half kt of the next layer's B operand from accumulators acc[2 kt], acc[2 kt + 1] (hidden
// unit 16 mt + 4 g + i of sample 16 nt + c in lane 16 g + c, bias included): GELU, bf16,
// in the permuted K order of A2 and A3 (hidden 32 kt + 4 g + i, then 32 kt + 16 + 4 g + i).
__device__ __forceinline__ void activations(const floatx4 (&acc)[2][4], bf16x8 (&b)[4]) {
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            b[nt][i] = static_cast<__bf16>(gelu_bf16(acc[0][nt][i]));
            b[nt][4 + i] = static_cast<__bf16>(gelu_bf16(acc[1][nt][i]));
        }
}

// The network for 64 samples of a wave: feat holds sample e's inputs in row e (16
// bf16, zero beyond F).  Returns the logit and value of sample `lane`.  The biases enter
// as the accumulators' initial values (fp32).  Each layer runs in two halves of 32
// hidden units, so that only half of its accumulators is live at a time.  Every lane
// must call.
__device__ void mlp_tile(const MlpLds& L, const __bf16* feat, float& logit, float& value) {
    const int lane = __lane_id();
    const int g = lane >> 4, c = lane & 15;
    bf16x8 h1[2][4];
    {
        bf16x8 bf[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
            bf[nt] = g < 2 ? *reinterpret_cast<const bf16x8*>(feat + (16 * nt + c) * kMlpMaxFeatures + 8 * g) : zero8();
#pragma unroll
        for (int kt = 0; kt < 2; ++kt) {
            floatx4 acc[2][4];
#pragma unroll
            for (int u = 0; u < 2; ++u) {
                const int mt = 2 * kt + u;
                const floatx4 bias = *reinterpret_cast<const floatx4*>(&L.b1[16 * mt + 4 * g]);
                const bf16x8 a = L.A1[mt][lane];
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) acc[u][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, bf[nt], bias, 0, 0, 0);
            }
            activations(acc, h1[kt]);
        }
    }
    const floatx4 z4 = {0.0f, 0.0f, 0.0f, 0.0f};
    floatx4 out[4] = {z4, z4, z4, z4};
#pragma unroll
    for (int kt = 0; kt < 2; ++kt) {
        floatx4 acc[2][4];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int mt = 2 * kt + u;
            const floatx4 bias = *reinterpret_cast<const floatx4*>(&L.b2[16 * mt + 4 * g]);
            const bf16x8 a0 = L.A2[mt][0][lane], a1 = L.A2[mt][1][lane];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                acc[u][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a0, h1[0][nt], bias, 0, 0, 0);
                acc[u][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1, h1[1][nt], acc[u][nt], 0, 0, 0);
            }
        }
        bf16x8 h2[4];
        activations(acc, h2);
        const bf16x8 a3 = L.A3[kt][lane];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) out[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a3, h2[nt], out[nt], 0, 0, 0);
    }
    // outputs of sample 16 nt + c sit in lane c (rows 0 and 1); bring them to lane 16 nt + c
    const int my_nt = lane >> 4, src = lane & 15;
    float lg = 0.0f, vl = 0.0f;
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const float t0 = __shfl(out[nt][0], src);
        const float t1 = __shfl(out[nt][1], src);
        if (nt == my_nt) {
            lg = t0;
            vl = t1;
        }
    }
    logit = lg + L.b3[0];
    value = vl + L.b3[1];
}

__global__ __launch_bounds__(kInferBlock) void k_mlp_forward_bf16(const float* __restrict__ feats, int N, int F,
                                                                  const float* __restrict__ w, float* __restrict__ out) {
    __shared__ MlpLds L;
    __shared__ __attribute__((aligned(16))) __bf16 stage[kInferWaves][64 * kMlpMaxFeatures];
    load_mlp_lds(L, w, F);
    const int sm = blockIdx.x * kInferBlock + threadIdx.x;
    __bf16* st = stage[threadIdx.x >> 6] + __lane_id() * kMlpMaxFeatures;
#pragma unroll
    for (int k = 0; k < kMlpMaxFeatures; ++k)
        st[k] = static_cast<__bf16>((sm < N && k < F) ? feats[static_cast<size_t>(sm) * F + k] : 0.0f);
    __syncthreads();
    float logit, value;
    mlp_tile(L, stage[threadIdx.x >> 6], logit, value);
    if (sm < N) {
        out[2 * static_cast<size_t>(sm)] = logit;
        out[2 * static_cast<size_t>(sm) + 1] = value;
    }
}

struct LearnedArgs {
    const int32_t* A;
    int n, m;
    const float* r0;
    const float* r1;
    const int* pick;          // {use r1, stopped} or nullptr (r0)
    const float* reval_in;    // residual the cached outputs were computed on, or nullptr
    float* reval_out;         // <- the residual used now, or nullptr
    float2* cache;            // [n] (logit, value) of the last evaluation, or nullptr
    float sigma, logit_t;
    const float* w;
    float* value;
};

// The learned decision of every column.  Each wave takes rounds of 64 consecutive
// columns, one per lane: a column whose d residual entries are bit-identical to those
// of the last evaluation takes its cached (logit, value); the others queue their
// sorted features in the wave's LDS queue, which is run through the network 64 at a time.
template <int D>
__global__ __launch_bounds__(kInferBlock, 4) void k_learned_cols(LearnedArgs a) {
    __shared__ MlpLds L;
    __shared__ __attribute__((aligned(16))) __bf16 qf[kInferWaves][kQueueCap * kMlpMaxFeatures];
    __shared__ int qj[kInferWaves][kQueueCap];
    if (a.pick && a.pick[1]) return;
    const float* __restrict__ r = (a.pick && a.pick[0]) ? a.r1 : a.r0;
    load_mlp_lds(L, a.w, D + 1);
    if (a.reval_out) {
        for (int i = blockIdx.x * kInferBlock + threadIdx.x; i < a.m; i += gridDim.x * kInferBlock)
            a.reval_out[i] = r[i];
    }
    __syncthreads();
    const int wave = threadIdx.x >> 6, lane = __lane_id();
    __bf16* __restrict__ myf = qf[wave];
    int* __restrict__ myj = qj[wave];
    const float nan = __builtin_nanf("");
    const int rounds = (a.n + 63) >> 6;
    const int nw = gridDim.x * kInferWaves;
    int qn = 0;
    for (int rd = blockIdx.x * kInferWaves + wave; rd < rounds; rd += nw) {
        const int j = rd * 64 + lane;
        bool need = false;
        float v[D];
        if (j < a.n) {
            int rows[D];
#pragma unroll
            for (int p = 0; p < D; ++p) rows[p] = MCHK(a.A[static_cast<size_t>(j) * D + p], a.m);
#pragma unroll
            for (int p = 0; p < D; ++p) v[p] = r[rows[p]];
            need = true;
            if (a.reval_in) {
                // all d earlier residuals are loaded before any comparison (a comparison
                // that could skip the next load makes every load wait for the one before)
                float rv[D];
#pragma unroll
                for (int p = 0; p < D; ++p) rv[p] = a.reval_in[rows[p]];
                bool same = true;
#pragma unroll
                for (int p = 0; p < D; ++p) same = same & (__float_as_uint(rv[p]) == __float_as_uint(v[p]));
                if (same) {
                    const float2 cc = a.cache[j];
                    a.value[j] = cc.x >= a.logit_t ? cc.y : nan;
                    need = false;
                }
            }
        }
        const unsigned long long bal = __ballot(need);
        if (need) {
#pragma unroll
            for (int x = 1; x < D; ++x)
#pragma unroll
                for (int y = x; y > 0; --y) {
                    const float lo = fminf(v[y - 1], v[y]), hi = fmaxf(v[y - 1], v[y]);
                    v[y - 1] = lo;
                    v[y] = hi;
                }
            const int slot = MCHK(qn + __popcll(bal & ((1ull << lane) - 1ull)), kQueueCap);
            bf16x8 f0, f1;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                f0[k] = static_cast<__bf16>(k < D ? v[k < D ? k : 0] : (k == D ? a.sigma : 0.0f));
                f1[k] = static_cast<__bf16>(k + 8 < D ? v[k + 8 < D ? k + 8 : 0] : (k + 8 == D ? a.sigma : 0.0f));
            }
            bf16x8* dst = reinterpret_cast<bf16x8*>(myf + slot * kMlpMaxFeatures);
            dst[0] = f0;
            dst[1] = f1;
            myj[slot] = j;
        }
        qn += __popcll(bal);
        if (qn >= 64) {
            __builtin_amdgcn_wave_barrier();
            float lg, vl;
            mlp_tile(L, myf, lg, vl);
            const int jj = MCHK(myj[lane], a.n);
            if (a.cache) a.cache[jj] = make_float2(lg, vl);
            a.value[jj] = lg >= a.logit_t ? vl : nan;
            // entries 64.. move to the front of the queue
            qn -= 64;
            if (lane < qn) {
                (void)MCHK(64 + lane, kQueueCap);
                const bf16x8* src = reinterpret_cast<const bf16x8*>(myf + (64 + lane) * kMlpMaxFeatures);
                bf16x8* dst = reinterpret_cast<bf16x8*>(myf + lane * kMlpMaxFeatures);
                const bf16x8 s0 = src[0], s1 = src[1];
                const int sj = myj[64 + lane];
                dst[0] = s0;
                dst[1] = s1;
                myj[lane] = sj;
            }
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (qn > 0) {
        // the rest; rows qn..63 of the tile hold stale samples whose outputs are unused
        __builtin_amdgcn_wave_barrier();
        float lg, vl;
        mlp_tile(L, myf, lg, vl);
        if (lane < qn) {
            const int jj = MCHK(myj[lane], a.n);
            if (a.cache) a.cache[jj] = make_float2(lg, vl);
            a.value[jj] = lg >= a.logit_t ? vl : nan;
        }
    }
}

int blocks_of(long long count, int block) { return static_cast<int>((count + block - 1) / block); }

}  // namespace

hipError_t mlp_check_read(int* line, hipStream_t s) {
#if RL0_DEVICE_CHECKS
    unsigned v = 0u;
    hipError_t e = hipMemcpyFromSymbolAsync(&v, HIP_SYMBOL(g_mlp_check_line), sizeof(v), 0, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && v != 0u) {
        const unsigned zero = 0u;
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_mlp_check_line), &zero, sizeof(zero), 0, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
    }
    *line = static_cast<int>(v);
    return e;
#else
    (void)s;
    *line = -1;
    return hipSuccess;
#endif
}

hipError_t launch_mlp_features(const int32_t* A, int n, int m, int d, const float* r, float sigma, float* feats,
                               hipStream_t s) {
    const int g = blocks_of(n, 256);
    switch (d) {
#define RL0_FEAT(D) \
    case D: k_mlp_features<D><<<g, 256, 0, s>>>(A, n, m, r, sigma, feats); break;
        RL0_FEAT(1) RL0_FEAT(2) RL0_FEAT(3) RL0_FEAT(4) RL0_FEAT(5) RL0_FEAT(6) RL0_FEAT(7) RL0_FEAT(8)
        RL0_FEAT(9) RL0_FEAT(10) RL0_FEAT(11) RL0_FEAT(12) RL0_FEAT(13) RL0_FEAT(14) RL0_FEAT(15) RL0_FEAT(16)
#undef RL0_FEAT
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_mlp_labels(const float* x_true, const float* x_hat, int n, double thr, float* labels,
                             hipStream_t s) {
    k_mlp_labels<<<blocks_of(n, 256), 256, 0, s>>>(x_true, x_hat, n, thr, labels);
    return hipGetLastError();
}

size_t mlp_grad_lds(int F) {
    const size_t P = static_cast<size_t>(mlp_params(F - 1));
    return sizeof(float) * (((P + 3) & ~static_cast<size_t>(3)) + kHidden * kHidden + kGradTile * F +
                            4 * kGradTile * kHidden + 4 * kGradTile);
}

int mlp_grad_groups(int N) { return std::max(1, std::min(blocks_of(N, kGradTile), kGradMaxGroups)); }

size_t mlp_grad_scratch_floats(int d) {
    return static_cast<size_t>(kGradMaxGroups) * (static_cast<size_t>(mlp_params(d)) + 1);
}

hipError_t launch_mlp_grad(const float* feats, const float* labels, int N, int d, const float* w, float lam,
                           float* grad, float* loss, float* part, hipStream_t s, const AdamStep* adam) {
    const int F = d + 1;
    const size_t lds = mlp_grad_lds(F);
    static bool attr = false;
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_mlp_grad),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 static_cast<int>(mlp_grad_lds(kMaxD + 1)));
        if (e != hipSuccess) return e;
        attr = true;
    }
    const int G = mlp_grad_groups(N), P = mlp_params(d);
    k_mlp_grad<<<G, kGradBlock, lds, s>>>(feats, labels, N, F, w, lam, 1.0f / static_cast<float>(N), part);
    if (adam)
        k_mlp_grad_sum<true><<<blocks_of(P, 64), 64 * kSumSlices, 0, s>>>(part, G, P, 1.0f / static_cast<float>(N),
                                                                         grad, loss, *adam);
    else
        k_mlp_grad_sum<false><<<blocks_of(P, 64), 64 * kSumSlices, 0, s>>>(part, G, P, 1.0f / static_cast<float>(N),
                                                                          grad, loss, AdamStep{});
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float* w, const float* grad, float* m, float* v, int P, float lr, float b1, float b2,
                           float eps, float c1, float c2, hipStream_t s) {
    const AdamStep a{w, m, v, lr, b1, b2, eps, c1, c2};
    k_mlp_adam<<<blocks_of(P, 256), 256, 0, s>>>(grad, P, a);
    return hipGetLastError();
}

hipError_t launch_zero_floats(float* p, long long count, hipStream_t s) {
    if (count > 0) k_zero_floats<<<blocks_of(count, 256), 256, 0, s>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float* feats, int N, int d, const float* w, float* out, int bf16,
                              hipStream_t s) {
    const int F = d + 1;
    if (bf16) {
        if (F > kMlpMaxFeatures) return hipErrorInvalidValue;
        k_mlp_forward_bf16<<<blocks_of(N, kInferBlock), kInferBlock, 0, s>>>(feats, N, F, w, out);
    } else {
        const size_t lds = sizeof(float) * mlp_params(d);
        k_mlp_forward_f32<<<blocks_of(N, 128), 128, lds, s>>>(feats, N, F, w, out);
    }
    return hipGetLastError();
}

hipError_t launch_learned_cols(const LearnedCols& lc, hipStream_t s) {
    LearnedArgs a;
    a.A = lc.A;
    a.n = lc.n;
    a.m = lc.m;
    a.r0 = lc.r;
    a.r1 = lc.r1;
    a.pick = lc.pick;
    a.reval_in = lc.reval_in;
    a.reval_out = lc.reval_out;
    a.cache = reinterpret_cast<float2*>(lc.cache);
    a.sigma = lc.sigma;
    a.logit_t = lc.logit_t;
    a.w = lc.w;
    a.value = lc.value;
    if (a.reval_in && !a.cache) return hipErrorInvalidValue;
    int cus = 256;
    {
        int dev = 0;
        if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    }
    const int rounds = blocks_of(lc.n, 64);
    const int g = std::max(1, std::min(blocks_of(rounds, kInferWaves), 4 * cus));
    switch (lc.d) {
#define RL0_LC(D) \
    case D: k_learned_cols<D><<<g, kInferBlock, 0, s>>>(a); break;
        RL0_LC(1) RL0_LC(2) RL0_LC(3) RL0_LC(4) RL0_LC(5) RL0_LC(6) RL0_LC(7) RL0_LC(8)
        RL0_LC(9) RL0_LC(10) RL0_LC(11) RL0_LC(12) RL0_LC(13) RL0_LC(14) RL0_LC(15)
#undef RL0_LC
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace rl0
