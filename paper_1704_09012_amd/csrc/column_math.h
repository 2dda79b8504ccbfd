// Arithmetic shared by the decoder's kernels: fixed-point conversions, the tabulated
// score functions and the column body of Alg. 1, all under the float32 contract
// (operations in the written order, no contraction, IEEE division); and two wave-level
// helpers for histograms and list appends.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "kernels.h"

#pragma clang fp contract(off)

namespace rl0 {

constexpr int kTableN = 4096;
constexpr double kTwo40 = 1099511627776.0;          // 2^40
constexpr double kTwoM40 = 1.0 / 1099511627776.0;   // 2^-40
constexpr double kTwo30 = 1073741824.0;             // 2^30
constexpr double kFxLimit = 4611686018427387904.0;  // 2^62


__device__ __forceinline__ long long to_fx(float v, int* err) {
    const double s = static_cast<double>(v) * kTwo40;
    if (!(fabs(s) < kFxLimit)) {
        atomicOr(err, kErrRange);
        return 0;
    }
    return __double2ll_rn(s);
}

// v is not a multiple of 2^-40, so rint(2^40 v) rounds (only possible for |v| < 2^-17)
__device__ __forceinline__ bool fx_inexact(float v) {
    const double s = static_cast<double>(v) * kTwo40;
    return s != rint(s);
}

__device__ __forceinline__ float from_fx(long long S) {
    return static_cast<float>(static_cast<double>(S) * kTwoM40);
}

__device__ __forceinline__ long long l1_term(float r) {
    return __double2ll_rn(static_cast<double>(fabsf(r)) * kTwo30);
}

__device__ __forceinline__ uint32_t abs_bits(float v) { return __float_as_uint(v) & 0x7FFFFFFFu; }

__device__ __forceinline__ float table_score(const float* __restrict__ T, float inv_h, float a) {
    const float u = a * inv_h;
    if (!(u < static_cast<float>(kTableN))) return 0.0f;
    const int i = static_cast<int>(u);
    const float f = u - static_cast<float>(i);
    const float t0 = T[i];
    const float t1 = T[i + 1];
    return t0 + f * (t1 - t0);
}

__device__ __forceinline__ float score(const float* __restrict__ T, float inv_h, int exact, float a) {
    if (exact) return a == 0.0f ? 1.0f : 0.0f;
    return table_score(T, inv_h, a);
}

__device__ __forceinline__ unsigned long long hk_key(int j, float x) {
    return (static_cast<unsigned long long>(abs_bits(x)) << 32) |
           static_cast<unsigned long long>(0xFFFFFFFFu - static_cast<unsigned int>(j));
}

// Column body of Alg. 1 on the snapshot r_hat, float32 contract.  cmask marks the rows
// that pass the outer test; they are visited in ascending row order, so the first row
// with the strictly largest n_e wins.  Returns whether the column proposes an update
// and its omega.  Each lane walks its own set bits, so the lanes of a wave stay busy
// whichever rows their columns flag.
template <int D>
__device__ __forceinline__ bool column_update(const float (&v)[D], unsigned int cmask,
                                                      const ScoreTables& tb, float alpha, int l1_test,
                                                      float* omega_out) {
    float n_z = 0.0f;
    float S1 = 0.0f;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        // quantised: the indicator 1{p_breve_z(v) >= 1 - t}, a threshold on |v|
        const float z = tb.quant ? (abs_bits(v[p]) <= tb.qz_bits ? 1.0f : 0.0f)
                                 : score(tb.Tz, tb.inv_h_z, tb.exact, fabsf(v[p]));
        n_z = n_z + z;
        S1 = S1 + fabsf(v[p]);
    }
    bool has = false;
    float best_ne = 0.0f, best_om = 0.0f;
    unsigned int rem = cmask;
    while (rem) {
        const int p = __builtin_ctz(rem);
        rem &= rem - 1u;
        float vp = v[0];
#pragma unroll
        for (int q = 1; q < D; ++q)
            if (p == q) vp = v[q];
        // every e-score is at most 1 and is 0 once |v_p - v_l| reaches the end of the
        // table, so n_e <= 1 + (rows closer than that); when even that bound fails the
        // test, the candidate fails it (fp32 sums and differences are monotone)
        // (quantised: near counts the rows with q_e = 1, so 1 + near is n_e itself)
        int near = 0;
        const uint32_t e_bound = tb.quant ? tb.qe_bits + 1u : tb.e_zero_bits;
#pragma unroll
        for (int l = 0; l < D; ++l) near += (l != p && abs_bits(vp - v[l]) < e_bound) ? 1 : 0;
        if (!((1.0f + static_cast<float>(near)) - n_z >= alpha)) continue;
        float n_e = 0.0f, s = 0.0f;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            float w;
            if (l == p)
                w = 1.0f;
            else if (tb.quant)
                w = abs_bits(vp - v[l]) <= tb.qe_bits ? 1.0f : 0.0f;   // 1{p_breve_e(a) >= t}
            else
                w = score(tb.Te, tb.inv_h_e, tb.exact, fabsf(vp - v[l]));
            n_e = n_e + w;
            s = s + v[l] * w;
        }
        const float om = s / n_e;
        bool l1_ok;
        if (l1_test == 0) {
            float Lp = 0.0f;
#pragma unroll
            for (int l = 0; l < D; ++l) Lp = Lp + fabsf(v[l] - om);
            l1_ok = Lp <= S1;
        } else {
            l1_ok = fabsf(vp - om) <= fabsf(vp);
        }
        const bool pass = ((n_e - n_z) >= alpha) && l1_ok;
        if (pass && (!has || n_e > best_ne)) {
            has = true;
            best_ne = n_e;
            best_om = om;
        }
    }
    *omega_out = best_om;
    return has;
}

// The column body of Alg. 1 (column_update) for a column most of whose rows pass the
// outer test: the e-score of each of its D (D - 1) / 2 row pairs is taken once, since a
// score depends on |v_p - v_l| alone and v_p - v_l = -(v_l - v_p) exactly in float32.
// Each candidate row then adds its row's scores in the order column_update adds them
// (l = 0 .. D - 1, 1 for l = p), and every candidate is evaluated in full: the bound
// by which column_update skips some can only skip candidates that fail the test.  The
// two functions return the same bits (beyond 8 rows this one calls column_update).
template <int D>
__device__ __forceinline__ bool column_update_pairs(const float (&v)[D], unsigned int cmask, const ScoreTables& tb,
                                                    float alpha, int l1_test, float* omega_out) {
    // beyond 8 rows the pairs would not fit the registers: the candidates one by one
    if constexpr (D > 8) return column_update<D>(v, cmask, tb, alpha, l1_test, omega_out);
    float n_z = 0.0f;
    float S1 = 0.0f;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const float z = tb.quant ? (abs_bits(v[p]) <= tb.qz_bits ? 1.0f : 0.0f)
                                 : score(tb.Tz, tb.inv_h_z, tb.exact, fabsf(v[p]));
        n_z = n_z + z;
        S1 = S1 + fabsf(v[p]);
    }
    float w[D][D];
#pragma unroll
    for (int p = 0; p < D; ++p) {
        w[p][p] = 1.0f;
#pragma unroll
        for (int l = p + 1; l < D; ++l) {
            const float a = v[p] - v[l];
            const float e = tb.quant ? (abs_bits(a) <= tb.qe_bits ? 1.0f : 0.0f)
                                     : score(tb.Te, tb.inv_h_e, tb.exact, fabsf(a));
            w[p][l] = e;
            w[l][p] = e;
        }
    }
    bool has = false;
    float best_ne = 0.0f, best_om = 0.0f;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        if (!((cmask >> p) & 1u)) continue;
        float n_e = 0.0f, s = 0.0f;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            n_e = n_e + w[p][l];
            s = s + v[l] * w[p][l];
        }
        const float om = s / n_e;
        bool l1_ok;
        if (l1_test == 0) {
            float Lp = 0.0f;
#pragma unroll
            for (int l = 0; l < D; ++l) Lp = Lp + fabsf(v[l] - om);
            l1_ok = Lp <= S1;
        } else {
            l1_ok = fabsf(v[p] - om) <= fabsf(v[p]);
        }
        const bool pass = ((n_e - n_z) >= alpha) && l1_ok;
        if (pass && (!has || n_e > best_ne)) {
            has = true;
            best_ne = n_e;
            best_om = om;
        }
    }
    *omega_out = best_om;
    return has;
}

// ---- wave-level helpers (all 64 lanes of the wave must call them)

// hist[bin] += 1 for every lane with valid set; lanes of a wave that hit the same bin
// add together (the magnitudes of a support cluster in a few bins).  Every lane of the
// wave must call.
__device__ __forceinline__ void hist_add(unsigned* hist, unsigned bin, bool valid) {
    unsigned long long active = __ballot(valid);
    const int lane = __lane_id();
    while (active) {
        const int leader = __ffsll(static_cast<long long>(active)) - 1;
        const unsigned b = __shfl(bin, leader);
        const unsigned long long same = __ballot(valid && bin == b);
        if (lane == leader) atomicAdd(&hist[b], static_cast<unsigned>(__popcll(same)));
        active &= ~same;
    }
}

// Append for every lane with pred: one atomic per wave reserves the slots; returns the
// lane's slot (meaningless where pred is false).
__device__ __forceinline__ int wave_append(int* counter, bool pred) {
    const unsigned long long b = __ballot(pred);
    const int lane = __lane_id();
    int base = 0;
    if (b) {
        const int leader = __ffsll(static_cast<long long>(b)) - 1;
        if (lane == leader) base = atomicAdd(counter, static_cast<int>(__popcll(b)));
        base = __shfl(base, leader);
    }
    return base + static_cast<int>(__popcll(b & ((1ull << lane) - 1ull)));
}

}  // namespace rl0
