// HIP kernels of the Robust-l0 decoder for gfx950 (MI355X).
//
// One decode iteration (the while-loop body of Alg. 1) is
//   sweep    every column j reads its d residual entries, runs the noisy consensus test
//            and proposes x'_j; columns in supp(x_hat) or updated join a candidate list
//   select   H_k: the k-th largest key (|x'_j| bits, then smaller j) over the list
//   residual r = y - A H_k(x') in 64-bit fixed point (exact integer atomics, so the
//            result does not depend on the order of the atomics), rounded to float32
//   accept   keep (x', r) if ||r||_1 (exact integer) decreased; advance t; stop test
//
// Floating point follows a fixed contract so that results are bitwise reproducible:
// float32 operations in the written order, no contraction (-ffp-contract=off and the
// pragma below), IEEE division.
#include "kernels.h"

#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace rl0 {

namespace {

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

__device__ __forceinline__ float from_fx(long long S) {
    return static_cast<float>(static_cast<double>(S) * kTwoM40);
}

__device__ __forceinline__ long long l1_term(float r) {
    return __double2ll_rn(static_cast<double>(fabsf(r)) * kTwo30);
}

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
    const unsigned int mag = __float_as_uint(x) & 0x7FFFFFFFu;
    return (static_cast<unsigned long long>(mag) << 32) |
           static_cast<unsigned long long>(0xFFFFFFFFu - static_cast<unsigned int>(j));
}

// Wave-aggregated slot reservation in an append list.  Every lane of the wave must call.
__device__ __forceinline__ int wave_append(bool pred, int* counter) {
    const unsigned long long mask = __ballot(pred);
    if (mask == 0ull) return -1;
    const int lane = __lane_id();
    const int leader = __ffsll(static_cast<long long>(mask)) - 1;
    int base = 0;
    if (lane == leader) base = atomicAdd(counter, __popcll(mask));
    base = __shfl(base, leader);
    const int rank = __popcll(mask & ((1ull << lane) - 1ull));
    return pred ? base + rank : -1;
}

template <int BLOCK>
__device__ __forceinline__ long long block_sum_ll(long long v, long long* sh) {
    // wave reduction then LDS across waves
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    long long tot = 0;
    if (threadIdx.x == 0) {
        for (int w = 0; w < BLOCK / 64; ++w) tot += sh[w];
    }
    return tot;  // valid in thread 0
}

// ------------------------------------------------------------------ validation, sketch

__global__ void k_validate(const int32_t* __restrict__ A, int n, int m, int d, int* err) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const int32_t* col = A + static_cast<size_t>(j) * d;
    int prev = -1;
    bool bad = false;
    for (int p = 0; p < d; ++p) {
        const int r = col[p];
        bad |= (r <= prev) | (r >= m);
        prev = r;
    }
    if (bad) atomicOr(err, kErrIndex);
}

__global__ void k_zero_ll(long long* __restrict__ S, int m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) S[i] = 0;
}

__global__ void k_zero_f32(float* __restrict__ x, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = 0.0f;
}

__global__ void k_sketch_scatter(const int32_t* __restrict__ A, int n, int d,
                                 const float* __restrict__ x, long long* __restrict__ S, int* err) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || *err) return;
    const float xj = x[j];
    if (xj == 0.0f) return;
    const long long fx = to_fx(xj, err);
    const int32_t* col = A + static_cast<size_t>(j) * d;
    for (int p = 0; p < d; ++p)
        atomicAdd(reinterpret_cast<unsigned long long*>(S + col[p]), static_cast<unsigned long long>(fx));
}

__global__ void k_sketch_finish(const long long* __restrict__ S, float* __restrict__ y, int m) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) y[i] = from_fx(S[i]);
}

// ------------------------------------------------------------------ decode: init

__global__ void k_reset_state(DevState* st, long long L_hat) {
    st->L_hat = L_hat;
    st->L_trial[0] = st->L_trial[1] = 0;
    st->cand_count[0] = st->cand_count[1] = 0;
    st->done = 0;
    st->cur = 0;
    st->executed_it = -1;
    st->accepted_flag = 0;
    st->iterations = 0;
    st->accepted = 0;
    st->updates_total = 0;
    st->err = 0;
    st->n_kept = 0;
    st->kth_key = 0ull;
}

// Sy = rint(2^40 y); r0 = fl32(2^-40 Sy) (the residual of x = 0); L_hat = L(r0)
__global__ __launch_bounds__(256) void k_init(const float* __restrict__ y, long long* __restrict__ Sy,
                                              float* __restrict__ r0, int m, DevState* st, int add_l1) {
    __shared__ long long sh[4];
    const int i = blockIdx.x * 256 + threadIdx.x;
    long long l = 0;
    if (i < m) {
        const float yi = y[i];
        if (!isfinite(yi)) atomicOr(&st->err, kErrNonFinite);
        const long long s = to_fx(yi, &st->err);
        Sy[i] = s;
        const float r = from_fx(s);
        if (r0) r0[i] = r;
        l = l1_term(r);
    }
    const long long tot = block_sum_ll<256>(l, sh);
    if (add_l1 && threadIdx.x == 0 && tot != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(&st->L_hat), static_cast<unsigned long long>(tot));
}

__global__ void k_init_done(DevState* st, int n_iters, double tol_fx) {
    if (st->err || n_iters <= 0 || static_cast<double>(st->L_hat) <= tol_fx) st->done = 1;
}

// ------------------------------------------------------------------ decode: sweep

struct SweepArgs {
    const int32_t* A;
    int n;
    const float* r_buf0;
    const float* r_buf1;
    const float* x_hat;
    ScoreTables tb;
    IterParams ip;
    int* cand_j;
    float* cand_x;
    DevState* st;
    DebugOut dbg;
};

// Column body of Alg. 1 on the snapshot r_hat, float32 contract.  Returns whether the
// column proposes an update and the chosen omega.
template <int D>
__device__ __forceinline__ bool column_update(const float (&v)[D], unsigned int cmask,
                                              const ScoreTables& tb, float alpha, int l1_test,
                                              float* omega_out) {
    float z[D];
    float n_z = 0.0f;
    float S1 = 0.0f;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        z[p] = score(tb.Tz, tb.inv_h_z, tb.exact, fabsf(v[p]));
        n_z = n_z + z[p];
        S1 = S1 + fabsf(v[p]);
    }
    bool has = false;
    float best_ne = 0.0f, best_om = 0.0f;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        if (!((cmask >> p) & 1u)) continue;
        float n_e = 0.0f, s = 0.0f;
#pragma unroll
        for (int l = 0; l < D; ++l) {
            const float w = (l == p) ? 1.0f : score(tb.Te, tb.inv_h_e, tb.exact, fabsf(v[p] - v[l]));
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

template <int D>
__global__ __launch_bounds__(256) void k_sweep(SweepArgs a) {
    DevState* st = a.st;
    if (st->done | st->err) return;
    const float* __restrict__ r = st->cur ? a.r_buf1 : a.r_buf0;
    const int j = blockIdx.x * 256 + threadIdx.x;
    bool emit = false, upd = false;
    float xp = 0.0f, om = 0.0f;
    if (j < a.n) {
        float v[D];
        const int32_t* __restrict__ col = a.A + static_cast<size_t>(j) * D;
        unsigned int cmask = 0u;
#pragma unroll
        for (int p = 0; p < D; ++p) {
            v[p] = r[col[p]];
            if ((__float_as_uint(v[p]) & 0x7FFFFFFFu) >= a.ip.tau_bits) cmask |= 1u << p;
        }
        const float xh = a.x_hat[j];
        if (cmask) upd = column_update<D>(v, cmask, a.tb, a.ip.alpha, a.ip.l1_test, &om);
        xp = upd ? xh + om : xh;
        emit = upd || (xh != 0.0f);
        if (a.dbg.updated) a.dbg.updated[j] = upd ? 1 : 0;
        if (a.dbg.omega) a.dbg.omega[j] = upd ? om : 0.0f;
    }
    const int slot = wave_append(emit, &st->cand_count[a.ip.it & 1]);
    if (slot >= 0) {
        a.cand_j[slot] = j;
        a.cand_x[slot] = xp;
    }
    const unsigned long long um = __ballot(upd);
    if (__lane_id() == 0 && um) atomicAdd(&st->updates_total, __popcll(um));
}

// ------------------------------------------------------------------ decode: H_k select

// One workgroup: the k-th largest key among nonzero candidates by 11-bit radix passes.
__global__ __launch_bounds__(1024) void k_select(const int* __restrict__ cand_j,
                                                 const float* __restrict__ cand_x, DevState* st,
                                                 int it, int k) {
    if (st->done | st->err) return;
    __shared__ unsigned int hist[2048];
    __shared__ unsigned int scan[1024];
    __shared__ unsigned long long prefix, pmask;
    __shared__ unsigned int remaining;
    __shared__ unsigned int nz_total;
    const int tid = threadIdx.x;
    const int count = st->cand_count[it & 1];
    if (tid == 0) nz_total = 0;
    __syncthreads();
    unsigned int nz = 0;
    for (int e = tid; e < count; e += 1024) nz += (cand_x[e] != 0.0f);
    atomicAdd(&nz_total, nz);
    __syncthreads();
    if (nz_total <= static_cast<unsigned int>(k)) {
        if (tid == 0) {
            st->kth_key = 1ull << 32;
            st->n_kept = static_cast<int>(nz_total);
        }
        return;
    }
    if (tid == 0) {
        prefix = 0ull;
        pmask = 0ull;
        remaining = static_cast<unsigned int>(k);
    }
    const int shifts[6] = {53, 42, 31, 20, 9, 0};
    const int widths[6] = {11, 11, 11, 11, 11, 9};
    for (int pass = 0; pass < 6; ++pass) {
        const int sh = shifts[pass];
        const unsigned int dmask = (1u << widths[pass]) - 1u;
        hist[tid] = 0u;
        hist[tid + 1024] = 0u;
        __syncthreads();
        const unsigned long long pf = prefix, pm = pmask;
        for (int e = tid; e < count; e += 1024) {
            const float x = cand_x[e];
            if (x == 0.0f) continue;
            const unsigned long long key = hk_key(cand_j[e], x);
            if ((key & pm) == pf) atomicAdd(&hist[(key >> sh) & dmask], 1u);
        }
        __syncthreads();
        // thread t owns bins 2047-2t and 2046-2t; inclusive scan over t (top bins first)
        const unsigned int hi = hist[2047 - 2 * tid], lo = hist[2046 - 2 * tid];
        scan[tid] = hi + lo;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            const unsigned int add = tid >= off ? scan[tid - off] : 0u;
            __syncthreads();
            scan[tid] += add;
            __syncthreads();
        }
        const unsigned int incl = scan[tid];
        const unsigned int before = incl - hi - lo;
        const unsigned int rem = remaining;
        __syncthreads();
        int digit = -1;
        unsigned int above = 0;
        if (before < rem && rem <= before + hi) {
            digit = 2047 - 2 * tid;
            above = before;
        } else if (before + hi < rem && rem <= incl) {
            digit = 2046 - 2 * tid;
            above = before + hi;
        }
        if (digit >= 0) {
            prefix = pf | (static_cast<unsigned long long>(digit) << sh);
            pmask = pm | (static_cast<unsigned long long>(dmask) << sh);
            remaining = rem - above;
        }
        __syncthreads();
    }
    if (tid == 0) {
        st->kth_key = prefix;
        st->n_kept = k;
    }
}

// ------------------------------------------------------------------ decode: residual

__global__ void k_copy_ll(const long long* __restrict__ src, long long* __restrict__ dst, int m,
                          const DevState* st) {
    if (st->done | st->err) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) dst[i] = src[i];
}

__global__ void k_res_scatter(const int32_t* __restrict__ A, int d, const int* __restrict__ cand_j,
                              const float* __restrict__ cand_x, long long* __restrict__ S,
                              DevState* st, int it) {
    if (st->done | st->err) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= st->cand_count[it & 1]) return;
    const float x = cand_x[e];
    if (x == 0.0f) return;
    const int j = cand_j[e];
    if (hk_key(j, x) < st->kth_key) return;
    const long long fx = to_fx(x, &st->err);
    const int32_t* col = A + static_cast<size_t>(j) * d;
    for (int p = 0; p < d; ++p)
        atomicAdd(reinterpret_cast<unsigned long long*>(S + col[p]), static_cast<unsigned long long>(-fx));
}

__global__ __launch_bounds__(256) void k_res_finish(const long long* __restrict__ S, float* r_buf0,
                                                    float* r_buf1, int m, DevState* st, int it) {
    if (st->done | st->err) return;
    __shared__ long long sh[4];
    float* __restrict__ r = st->cur ? r_buf0 : r_buf1;   // the trial buffer
    const int i = blockIdx.x * 256 + threadIdx.x;
    long long l = 0;
    if (i < m) {
        const float v = from_fx(S[i]);
        r[i] = v;
        l = l1_term(v);
    }
    const long long tot = block_sum_ll<256>(l, sh);
    if (threadIdx.x == 0 && tot != 0)
        atomicAdd(reinterpret_cast<unsigned long long*>(&st->L_trial[it & 1]), static_cast<unsigned long long>(tot));
}

// ------------------------------------------------------------------ decode: accept

__global__ void k_decide(DevState* st, int it, int n_iters, double tol_fx) {
    if (st->done) return;
    if (st->err) {
        st->done = 1;
        return;
    }
    const long long Lt = st->L_trial[it & 1];
    const int acc = (Lt < st->L_hat) && (st->err == 0);
    st->accepted_flag = acc;
    st->executed_it = it;
    st->iterations = it + 1;
    if (acc) {
        st->L_hat = Lt;
        st->accepted += 1;
        st->cur ^= 1;
    }
    // clear the other parity's slots for iteration it + 1
    st->L_trial[(it + 1) & 1] = 0;
    st->cand_count[(it + 1) & 1] = 0;
    if (st->err || it + 1 >= n_iters || static_cast<double>(st->L_hat) <= tol_fx) st->done = 1;
}

__global__ void k_commit(const int* __restrict__ cand_j, const float* __restrict__ cand_x,
                         float* __restrict__ x_hat, float* __restrict__ x_trial,
                         const DevState* st, int it) {
    if (st->executed_it != it) return;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= st->cand_count[it & 1]) return;
    const int j = cand_j[e];
    const float x = cand_x[e];
    const bool kept = (x != 0.0f) && (hk_key(j, x) >= st->kth_key);
    const float val = kept ? x : 0.0f;
    if (x_trial) x_trial[j] = val;
    if (st->accepted_flag) x_hat[j] = val;
}

inline int blocks(long long n, int b) { return static_cast<int>((n + b - 1) / b); }

template <int D>
hipError_t launch_sweep_d(const SweepArgs& a, hipStream_t s) {
    k_sweep<D><<<blocks(a.n, 256), 256, 0, s>>>(a);
    return hipGetLastError();
}

hipError_t launch_sweep(int d, const SweepArgs& a, hipStream_t s) {
    switch (d) {
        case 1: return launch_sweep_d<1>(a, s);
        case 2: return launch_sweep_d<2>(a, s);
        case 3: return launch_sweep_d<3>(a, s);
        case 4: return launch_sweep_d<4>(a, s);
        case 5: return launch_sweep_d<5>(a, s);
        case 6: return launch_sweep_d<6>(a, s);
        case 7: return launch_sweep_d<7>(a, s);
        case 8: return launch_sweep_d<8>(a, s);
        case 9: return launch_sweep_d<9>(a, s);
        case 10: return launch_sweep_d<10>(a, s);
        case 11: return launch_sweep_d<11>(a, s);
        case 12: return launch_sweep_d<12>(a, s);
        case 13: return launch_sweep_d<13>(a, s);
        case 14: return launch_sweep_d<14>(a, s);
        case 15: return launch_sweep_d<15>(a, s);
        case 16: return launch_sweep_d<16>(a, s);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

// ------------------------------------------------------------------ launchers

hipError_t launch_validate(const int32_t* A, int n, int m, int d, int* err, hipStream_t s) {
    if (n > 0) k_validate<<<blocks(n, 256), 256, 0, s>>>(A, n, m, d, err);
    return hipGetLastError();
}

hipError_t launch_sketch(const int32_t* A, int n, int m, int d, const float* x, float* y,
                         long long* S, int* err, hipStream_t s) {
    k_validate<<<blocks(n, 256), 256, 0, s>>>(A, n, m, d, err);
    k_zero_ll<<<blocks(m, 256), 256, 0, s>>>(S, m);
    if (n > 0) k_sketch_scatter<<<blocks(n, 256), 256, 0, s>>>(A, n, d, x, S, err);
    k_sketch_finish<<<blocks(m, 256), 256, 0, s>>>(S, y, m);
    return hipGetLastError();
}

hipError_t launch_reset_state(DevState* st, long long L_hat, hipStream_t s) {
    k_reset_state<<<1, 1, 0, s>>>(st, L_hat);
    return hipGetLastError();
}

hipError_t launch_fix(const float* y, long long* Sy, int m, DevState* st, hipStream_t s) {
    // Sy only; L_hat is left as set by the caller (the state is reset to L_hat first)
    k_init<<<blocks(m, 256), 256, 0, s>>>(y, Sy, nullptr, m, st, 0);
    return hipGetLastError();
}

hipError_t launch_init(const DecodeDims& dm, const int32_t* A, bool validate, const float* y,
                       float* x_hat, const Workspace& w, const IterParams& ip, hipStream_t s) {
    k_reset_state<<<1, 1, 0, s>>>(w.st, 0);
    if (validate) k_validate<<<blocks(dm.n, 256), 256, 0, s>>>(A, dm.n, dm.m, dm.d, &w.st->err);
    k_zero_f32<<<blocks(dm.n, 256), 256, 0, s>>>(x_hat, dm.n);
    k_init<<<blocks(dm.m, 256), 256, 0, s>>>(y, w.Sy, w.r_buf[0], dm.m, w.st, 1);
    k_init_done<<<1, 1, 0, s>>>(w.st, ip.n_iters, ip.tol_fx);
    return hipGetLastError();
}

hipError_t launch_iteration(const DecodeDims& dm, const int32_t* A, const float* y,
                            float* x_hat, const Workspace& w, const ScoreTables& tb,
                            const IterParams& ip, const DebugOut& dbg, hipStream_t s,
                            hipEvent_t* ev_sweep) {
    (void)y;
    SweepArgs a;
    a.A = A;
    a.n = dm.n;
    a.r_buf0 = w.r_buf[0];
    a.r_buf1 = w.r_buf[1];
    a.x_hat = x_hat;
    a.tb = tb;
    a.ip = ip;
    a.cand_j = w.cand_j;
    a.cand_x = w.cand_x;
    a.st = w.st;
    a.dbg = dbg;
    if (ev_sweep) hipEventRecord(ev_sweep[0], s);
    hipError_t e = launch_sweep(dm.d, a, s);
    if (e != hipSuccess) return e;
    if (ev_sweep) hipEventRecord(ev_sweep[1], s);
    k_select<<<1, 1024, 0, s>>>(w.cand_j, w.cand_x, w.st, ip.it, dm.k);
    k_copy_ll<<<blocks(dm.m, 256), 256, 0, s>>>(w.Sy, w.S, dm.m, w.st);
    k_res_scatter<<<blocks(dm.n, 256), 256, 0, s>>>(A, dm.d, w.cand_j, w.cand_x, w.S, w.st, ip.it);
    k_res_finish<<<blocks(dm.m, 256), 256, 0, s>>>(w.S, w.r_buf[0], w.r_buf[1], dm.m, w.st, ip.it);
    k_decide<<<1, 1, 0, s>>>(w.st, ip.it, ip.n_iters, ip.tol_fx);
    k_commit<<<blocks(dm.n, 256), 256, 0, s>>>(w.cand_j, w.cand_x, x_hat, dbg.x_trial, w.st, ip.it);
    return hipGetLastError();
}

}  // namespace rl0
