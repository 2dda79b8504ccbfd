// HIP kernels of the Robust-l0 decoder for gfx950 (MI355X).
//
// One iteration of Alg. 1's loop is three kernels:
//   sweep         decides the previous iteration (accept/reject, stop test) from device
//                 state, makes the trial buffers equal to the current ones again, then runs
//                 the column loop: each column tests its rows against a 1-bit-per-row
//                 bitmask of the outer test held in LDS; only columns with a candidate row
//                 gather their exact residuals and run the noisy consensus test.  Columns in
//                 supp(x_hat) or updated join the candidate list of H_k.
//   select_apply  H_k: the k-th largest key (|x'_j| bits, then smaller j) by an 11-bit
//                 radix select started from the sweep's histogram; then the trial support
//                 and the exact integer change of the residual of every changed column.
//   finish_rows   r = fl32(2^-40 S) and ||r||_1 (an exact integer), and the outer-test
//                 bitmasks for the next iteration of both the trial and the current residual.
// Every launch is stream-ordered and the host never waits between iterations.
//
// Floating point follows a fixed contract so that results are bitwise reproducible:
// float32 operations in the written order, no contraction (-ffp-contract=off and the
// pragma below), IEEE division; residuals and ||r||_1 are integer sums.
#include "kernels.h"
#include "column_math.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#pragma clang fp contract(off)

namespace rl0 {

namespace {

constexpr int kTableStride = kTableStrideFloats;       // table_e starts 16-byte aligned
constexpr int kSweepBlock = 1024;
constexpr int kSweepCols = 4;                     // columns per sweep thread per chunk
constexpr int kSweepChunk = kSweepBlock * kSweepCols;
constexpr int kQueueRowInts = 7168;                 // 28 KiB of row indices of queued columns
constexpr int kBmLdsWords = 12288;                  // 48 KiB: bitmasks of m <= 393216 rows, or
                                                    // their 8-row summaries for m <= 3145728
constexpr int kBmPer = 4;                           // bitmask words per sweep thread held in registers
constexpr int kRowBlock = 1024;

// Checked builds (compiled with RL0_DEVICE_CHECKS=1 into a second copy of the library):
// RL0_CHK(i, n) tests a data-dependent index (one read from memory or from an atomic
// counter) against its range [0, n).  An index outside it records the source line of
// the first failed check in g_check_line (read back by device_check_read) and becomes 0,
// so that the access stays inside its buffer and the kernel runs to its end.  In normal
// builds RL0_CHK(i, n) is i and RL0_CHECK_ROWS does nothing.
#if RL0_DEVICE_CHECKS
__device__ unsigned g_check_line;

template <class I>
__device__ __forceinline__ I check_index(I i, long long n, unsigned line) {
    const long long v = static_cast<long long>(i);
    if (v >= 0 && v < n) return i;
    atomicCAS(&g_check_line, 0u, line);
    return static_cast<I>(0);
}
#define RL0_CHK(i, n) check_index((i), static_cast<long long>(n), __LINE__)
#define RL0_CHECK_ROWS(rows, m)                                                     \
    do {                                                                            \
        for (int q_ = 0; q_ < kSweepCols; ++q_)                                     \
            for (int p_ = 0; p_ < D; ++p_) rows[q_][p_] = RL0_CHK(rows[q_][p_], m); \
    } while (0)
#else
#define RL0_CHK(i, n) (i)
#define RL0_CHECK_ROWS(rows, m) \
    do {                        \
    } while (0)
#endif


template <int BLOCK>
__device__ __forceinline__ long long block_sum_ll(long long v, long long* sh) {
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

// Decision on iteration it-1 (Alg. 1: keep (x', r) iff ||r||_1 < ||r_hat||_1) and the
// stop test for iteration it ("while not converged and t > 0").  p = slot of iteration
// it-1, Lt = ||r||_1 of its trial iterate, err = the error flags.
__device__ __forceinline__ Slot decide_from(const Slot p, int err, int it, int n_iters, double tol_fx,
                                            long long Lt) {
    Slot s = p;
    if (p.pending) {
        const int acc = (Lt < p.L_hat) && (err == 0);
        if (acc) {
            s.L_hat = Lt;
            s.cur = p.cur ^ 1;
            s.accepted = p.accepted + 1;
        }
        s.accepted_last = acc;
        s.iterations = p.iterations + 1;
    }
    s.pending = 0;
    if (!s.done) s.done = (err != 0) || (static_cast<double>(s.L_hat) <= tol_fx) || (it >= n_iters);
    if (!s.done) s.pending = 1;
    return s;
}

__device__ __forceinline__ Slot decide(const DevState* st, int it, int n_iters, double tol_fx, long long Lt) {
    return decide_from(st->slot[(it & 1) ^ 1], st->err, it, n_iters, tol_fx, Lt);
}

// The per-iteration log's record of a decision d just taken on a pending iteration (its
// trial norm Lt): the iteration is the d.iterations-th executed one.
__device__ __forceinline__ void log_decision(DevState* st, const Slot& d, long long Lt) {
    const int q = d.iterations - 1;
    if (q < 0 || q >= kLogCap) return;
    IterLog& lg = st->log[q];
    lg.L_trial = Lt;
    lg.L_hat = d.L_hat;
    lg.accepted = d.accepted_last;
}

// trial_l1 computed by a whole workgroup (blockDim.x >= 64, a multiple of 64); the
// result is returned to every thread.  The partial sums were written by other CUs, so
// their loads are issued in parallel rather than one after another.
__device__ __forceinline__ long long trial_l1_block(const DevState* st, int par, long long* sh) {
    long long v = 0;
    for (int b = threadIdx.x; b < kRowGrid; b += blockDim.x) v += st->L_part[par][b];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    const int waves = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
    for (int w = 0; w < waves; ++w) t += sh[w];
    __syncthreads();
    return t;
}

// Sum of kRowBlock-thread block values; result valid in thread 0.
__device__ __forceinline__ long long block_sum_rows(long long v, long long* sh) {
    return block_sum_ll<kRowBlock>(v, sh);
}

// ------------------------------------------------------------------ small utilities

// The columns [j0, j0 + cnt) of A ([n][d] row indices) into LDS, with one 16-byte load
// per thread where the block's span is 16-byte aligned, all issued together.  (With d
// not known at compile time, a thread's own loop over its column's d indices waits for
// each load in turn.)  Every thread of the block must call.
__device__ __forceinline__ void stage_columns(const int32_t* __restrict__ A, int d, int j0, int cnt, int* cols) {
    const int total = cnt * d;
    const int32_t* __restrict__ src = A + static_cast<size_t>(j0) * d;
    if ((reinterpret_cast<uintptr_t>(src) & 15u) == 0u) {
        const int n4 = total >> 2;
        for (int i = threadIdx.x; i < n4; i += blockDim.x)
            reinterpret_cast<int4*>(cols)[i] = reinterpret_cast<const int4*>(src)[i];
        for (int i = (n4 << 2) + threadIdx.x; i < total; i += blockDim.x) cols[i] = src[i];
    } else {
        for (int i = threadIdx.x; i < total; i += blockDim.x) cols[i] = src[i];
    }
    __syncthreads();
}

constexpr int kStageBlock = 256;   // threads (and columns) per block of the staged kernels

__global__ __launch_bounds__(kStageBlock) void k_validate(const int32_t* __restrict__ A, int n, int m, int d,
                                                          int* err) {
    __shared__ __align__(16) int cols_sh[kStageBlock * kMaxD];
    const int j0 = blockIdx.x * kStageBlock;
    const int j = j0 + threadIdx.x;
    stage_columns(A, d, j0, min(kStageBlock, n - j0), cols_sh);
    if (j >= n) return;
    const int* col = cols_sh + threadIdx.x * d;
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

__global__ void k_zero_i32(int* __restrict__ p, long long count) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

__global__ void k_zero_f32(float* __restrict__ p, long long count) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0.0f;
}

__global__ void k_copy_f32(const float* __restrict__ src, float* __restrict__ dst, long long count) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i];
}

// Validates every column (rows strictly ascending in [0, m)) and scatters the nonzero
// ones: a malformed column flags kErrIndex and adds nothing, so no write leaves S.

__global__ __launch_bounds__(kStageBlock) void k_sketch_scatter(const int32_t* __restrict__ A, int n, int m, int d,
                                                                const float* __restrict__ x,
                                                                long long* __restrict__ S, int* err) {
    __shared__ __align__(16) int cols_sh[kStageBlock * kMaxD];
    const int j0 = blockIdx.x * kStageBlock;
    const int j = j0 + threadIdx.x;
    stage_columns(A, d, j0, min(kStageBlock, n - j0), cols_sh);
    if (j >= n) return;
    const int* col = cols_sh + threadIdx.x * d;
    const float xj = x[j];
    int prev = -1;
    bool bad = false;
    for (int p = 0; p < d; ++p) {
        const int r = col[p];
        bad |= (r <= prev) | (r >= m);
        prev = r;
    }
    if (bad) {
        atomicOr(err, kErrIndex);
        return;
    }
    if (xj == 0.0f) return;
    const long long fx = to_fx(xj, err);
    for (int p = 0; p < d; ++p)
        atomicAdd(reinterpret_cast<unsigned long long*>(S + col[p]), static_cast<unsigned long long>(fx));
}

// y = fl32(2^-40 S), unless the scatter flagged an error (then y is left unwritten).
__global__ void k_sketch_finish(const long long* __restrict__ S, float* __restrict__ y, int m, const int* err) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m && *err == 0) y[i] = from_fx(S[i]);
}

// ------------------------------------------------------------------ prepare

// the state a decode starts from: everything before the per-iteration log
constexpr int kStateWords = static_cast<int>(offsetof(DevState, log) / sizeof(int));

__global__ void k_prep_state(DevState* st) {
    int* p = reinterpret_cast<int*>(st);
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kStateWords; i += gridDim.x * blockDim.x) p[i] = 0;
}

// The starting support x0 as the candidate segments of the iteration before it0, in
// the workgroup that owns each column (kth_key of that parity stays 0: all kept).
__global__ void k_prep_support(const float* __restrict__ x0, int n, Workspace w, int slot) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float v = x0[j];
    if (v == 0.0f) return;
    const int seg = (j / kSweepChunk) % w.sweep_grid;
    const int o = atomicAdd(&w.st->seg_count[slot][seg], 1);
    const size_t ix = static_cast<size_t>(seg) * w.seg_cap + (w.seg_cap - 1 - RL0_CHK(o, w.seg_cap));   // back of the segment
    w.cand_j[slot][ix] = j;
    w.cand_x[slot][ix] = v;
    w.cand_h[slot][ix] = v;
}

// Sy = rint(2^40 y), S0 = Sy
__global__ void k_prep_rows(const float* __restrict__ y, long long* __restrict__ Sy, long long* __restrict__ S0,
                            long long* __restrict__ Dl, int m, DevState* st) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    Dl[i] = 0;
    const float yi = y[i];
    if (!isfinite(yi)) atomicOr(&st->err, kErrNonFinite);
    const long long s = to_fx(yi, &st->err);
    if (fx_inexact(yi)) atomicAdd(&st->inexact_y, 1);
    Sy[i] = s;
    S0[i] = s;
}

// S0 -= A x0 (columns with x0_j != 0)
__global__ void k_prep_scatter(const int32_t* __restrict__ A, int n, int d, const float* __restrict__ x0,
                               long long* __restrict__ S0, DevState* st) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n || st->err) return;
    const float v = x0[j];
    if (v == 0.0f) return;
    const long long fx = to_fx(v, &st->err);
    const int32_t* col = A + static_cast<size_t>(j) * d;
    for (int p = 0; p < d; ++p)
        atomicAdd(reinterpret_cast<unsigned long long*>(S0 + col[p]), static_cast<unsigned long long>(-fx));
}

// Bit g of the result: some bit of 8g .. 8g + 7 is set in b.
__device__ __forceinline__ uint8_t summary8(unsigned long long b) {
    uint32_t s = 0u;
#pragma unroll
    for (int g = 0; g < 8; ++g) s |= ((b >> (8 * g)) & 0xFFull) ? (1u << g) : 0u;
    return static_cast<uint8_t>(s);
}

// Bits of rows [base, base + 64) (base a multiple of 64) from a wave ballot.
__device__ __forceinline__ void store_bits(uint32_t* bm, int words, int base, unsigned long long b) {
    const int w0 = base >> 5;
    if (w0 < words) bm[w0] = static_cast<uint32_t>(b);
    if (w0 + 1 < words) bm[w0 + 1] = static_cast<uint32_t>(b >> 32);
}

// r0 = fl32(2^-40 S0), partial L(r0) into L_part[slot], outer-test bitmask of r0 (and,
// with bs0, its 8-row summary)
__global__ __launch_bounds__(kRowBlock) void k_prep_rows2(const long long* __restrict__ S0, float* __restrict__ r0,
                                                          uint32_t* __restrict__ bm0, uint8_t* __restrict__ bs0,
                                                          int m, uint32_t tau, DevState* st, int slot) {
    __shared__ long long sh[kRowBlock / 64];
    __shared__ unsigned flw[kRowBlock / 64];
    const int words = (m + 31) >> 5;
    long long l = 0;
    unsigned fl = 0u;
    for (int base = blockIdx.x * kRowBlock; base < m; base += gridDim.x * kRowBlock) {
        const int i = base + threadIdx.x;
        bool bit = false;
        if (i < m) {
            const float v = from_fx(S0[i]);
            r0[i] = v;
            l += l1_term(v);
            bit = abs_bits(v) >= tau;
        }
        const unsigned long long b = __ballot(bit);
        fl += static_cast<unsigned>(__popcll(b));
        if ((threadIdx.x & 63) == 0) {
            const int wb = base + (threadIdx.x & ~63);
            store_bits(bm0, words, wb, b);
            if (bs0 && wb < m) bs0[wb >> 6] = summary8(b);
        }
    }
    if ((threadIdx.x & 63) == 0) flw[threadIdx.x >> 6] = fl;
    const long long tot = block_sum_rows(l, sh);   // its barrier also publishes flw
    if (threadIdx.x == 0) {
        st->L_part[slot][blockIdx.x] = tot;
        unsigned f = 0u;
        for (int w = 0; w < kRowBlock / 64; ++w) f += flw[w];
        st->flag_part[slot][0][blockIdx.x] = f;
    }
}

__global__ __launch_bounds__(256) void k_prep_slot(DevState* st, int slot) {
    __shared__ long long red[4];
    const long long L0 = trial_l1_block(st, slot, red);
    if (threadIdx.x != 0) return;
    Slot& s = st->slot[slot];
    s.L_hat = L0;
    s.cur = 0;
    s.done = 0;
    s.pending = 0;
    s.accepted = 0;
    s.iterations = 0;
    s.accepted_last = 0;
    s.t_step = 0;
    s.last_par = slot;
}

// ------------------------------------------------------------------ H_k helpers

// The top 11 bits of hk_key(j, x) (x != 0): bits 30..20 of |x|.
__device__ __forceinline__ unsigned top_digit(float x) { return abs_bits(x) >> 20; }
static_assert(kHistBins == 2048, "H_k's radix digits are 11 bits");

// Within one workgroup of kRowBlock threads: the digit of the bucket (among 2048,
// highest first) that holds the `rem`-th largest of the counted keys, the count above it
// and the bucket's count.  Thread t holds digits 2047 - 2t and 2046 - 2t; the prefix
// counts come from wave scans and one exchange of the wave totals (scan: >= 16 entries).
__device__ void find_digit(const unsigned* hist, unsigned rem, unsigned* scan, int* digit_out,
                           unsigned* above_out, unsigned* bucket_out) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const unsigned hi = hist[2047 - 2 * tid], lo = hist[2046 - 2 * tid];
    unsigned incl = hi + lo;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned t = __shfl_up(incl, off);
        if (lane >= off) incl += t;
    }
    if (lane == 63) scan[wave] = incl;
    __syncthreads();
    for (int w = 0; w < wave; ++w) incl += scan[w];
    const unsigned before = incl - hi - lo;
    if (before < rem && rem <= before + hi) {
        *digit_out = 2047 - 2 * tid;
        *above_out = before;
        *bucket_out = hi;
    } else if (before + hi < rem && rem <= incl) {
        *digit_out = 2046 - 2 * tid;
        *above_out = before + hi;
        *bucket_out = lo;
    }
    __syncthreads();
}

// Within one workgroup: exclusive prefix sums of one int per segment (threads < nseg
// hold their value in v) by wave scans; returns the total.  start[] gets the sums.
__device__ __forceinline__ int segment_scan(int v, int nseg, int* start, int* wtot) {
    const int tid = threadIdx.x, lane = tid & 63;
    if (tid < kSweepGridMax) {
        int incl = tid < nseg ? v : 0;
        for (int off = 1; off < 64; off <<= 1) {
            const int t = __shfl_up(incl, off);
            if (lane >= off) incl += t;
        }
        start[tid] = incl - (tid < nseg ? v : 0);
        if (lane == 63) wtot[tid >> 6] = incl;
    }
    __syncthreads();
    int total = 0;
    for (int w = 0; w < kSweepGridMax / 64; ++w) total += wtot[w];
    if (tid < kSweepGridMax) {
        int add = 0;
        for (int w = 0; w < (tid >> 6); ++w) add += wtot[w];
        start[tid] += add;
    }
    __syncthreads();
    return total;
}

// Physical index of entry e (0 <= e < count) of a segment whose first `front` entries
// sit at its start and the rest at its end, backwards.
__device__ __forceinline__ size_t seg_phys(int seg, int cap, int front, int e) {
    return static_cast<size_t>(seg) * cap + (e < front ? e : cap - 1 - (e - front));
}

// ------------------------------------------------------------------ sweep

struct SweepArgs {
    const int32_t* A;
    int n, m;
    int chunks;      // ceil(n / kSweepChunk)
    int bm_lds;      // the outer-test bitmask fits in LDS
    int bs_lds;      // otherwise its 8-row summary does: a row's bit is read from global
                     // memory only where its group's summary bit is set
    Workspace w;
    ScoreTables tb;
    IterParams ip;
    DebugOut dbg;
    const float* learned;   // learned decisions per column (NaN: no update), or nullptr
    const uint4* Apk;       // packed A_cols (Packing<D>), or nullptr
};


// H_k's value of candidate j in an iteration whose k-th key was kth (zero if dropped).
__device__ __forceinline__ float hk_value(int j, float xp, unsigned long long kth) {
    return (xp != 0.0f && hk_key(j, xp) >= kth) ? xp : 0.0f;
}

// The support of x_hat is carried by the candidate segments rather than by a dense
// array: every column of supp(x_hat) is a candidate of every iteration, and sweep
// workgroup b writes only the columns it owns into segment b.  From its own previous
// segment and the accept decision a workgroup therefore knows x_hat on all its columns
// (the value H_k gave if the iteration was accepted, the value before it otherwise).
__device__ __forceinline__ float current_value(int accepted, int j, float xp, float xh, unsigned long long kth) {
    return accepted ? hk_value(j, xp, kth) : xh;
}

// Packed column indices: the d rows of a column in one 16-byte word, kField bits each
// (row p in bits [p kField, (p + 1) kField)), usable when m <= 2^kField.
template <int D>
struct Packing {
    static constexpr int kField = D <= 4 ? 32 : 128 / D;
};

template <int D>
__device__ __forceinline__ void unpack_rows(const uint4 w, int (&rows)[D]) {
    constexpr int F = Packing<D>::kField;
    const unsigned long long lo = (static_cast<unsigned long long>(w.y) << 32) | w.x;
    const unsigned long long hi = (static_cast<unsigned long long>(w.w) << 32) | w.z;
    constexpr unsigned long long mask = F >= 64 ? ~0ull : ((1ull << F) - 1ull);
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const int o = p * F;
        unsigned long long v;
        if (o + F <= 64)
            v = lo >> o;
        else if (o >= 64)
            v = hi >> (o - 64);
        else
            v = (lo >> o) | (hi << (64 - o));
        rows[p] = static_cast<int>(v & mask);
    }
}

// Row indices of the kSweepCols columns of thread tid in a chunk: column
// cbase + q kSweepBlock + tid for slot q (consecutive lanes, consecutive columns).
// issue_rows starts the loads (the packed words into w, or A_cols' rows into rows) and
// unpack_chunk turns packed words into rows; between the two the loads are in flight
// while other work goes on.  A column past n loads column n - 1 (n >= 1), so no per-lane
// branch separates the loads (a branch makes the compiler wait for each load before the
// next); every use of the rows checks the column against n.
template <int D, bool PACKED>
__device__ __forceinline__ void issue_rows(const int32_t* __restrict__ A, const uint4* __restrict__ Apk, int n,
                                           int cbase, int tid, uint4 (&w)[kSweepCols], int (&rows)[kSweepCols][D]) {
    if constexpr (PACKED) {
#pragma unroll
        for (int q = 0; q < kSweepCols; ++q) w[q] = Apk[min(cbase + q * kSweepBlock + tid, n - 1)];
    } else {
#pragma unroll
        for (int q = 0; q < kSweepCols; ++q) {
            const size_t jj = static_cast<size_t>(min(cbase + q * kSweepBlock + tid, n - 1));
#pragma unroll
            for (int p = 0; p < D; ++p) rows[q][p] = A[jj * D + p];
        }
    }
}

template <int D, bool PACKED>
__device__ __forceinline__ void unpack_chunk(const uint4 (&w)[kSweepCols], int (&rows)[kSweepCols][D],
                                             int n, int cbase, int tid) {
    if constexpr (PACKED) {
#pragma unroll
        for (int q = 0; q < kSweepCols; ++q) unpack_rows<D>(w[q], rows[q]);
    }
#pragma unroll
    for (int q = 0; q < kSweepCols; ++q) {
        const bool valid = cbase + q * kSweepBlock + tid < n;
#pragma unroll
        for (int p = 0; p < D; ++p) rows[q][p] = valid ? rows[q][p] : 0;
    }
}

// The packed form of A_cols (one 16-byte word per column).  With err, the columns are
// validated on the way (rows strictly ascending in [0, m)); with x_zero, x_zero[j] = 0.
template <int D>
__global__ void k_pack_cols(const int32_t* __restrict__ A, int n, int m, uint4* __restrict__ Apk, int* err,
                            float* __restrict__ x_zero) {
    // (the D loads of a thread's column are unrolled and issued together; staging the
    // block's columns through LDS, as the sketch does, measured slower here)
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    if (x_zero) x_zero[j] = 0.0f;
    constexpr int F = Packing<D>::kField;
    unsigned long long lo = 0ull, hi = 0ull;
    int prev = -1;
    bool bad = false;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        const int rp = A[static_cast<size_t>(j) * D + p];
        bad |= (rp <= prev) | (rp >= m);
        prev = rp;
        const unsigned long long r = static_cast<unsigned int>(rp);
        const int o = p * F;
        if (o + F <= 64) {
            lo |= r << o;
        } else if (o >= 64) {
            hi |= r << (o - 64);
        } else {
            lo |= r << o;
            hi |= r >> (64 - o);
        }
    }
    Apk[j] = make_uint4(static_cast<unsigned>(lo), static_cast<unsigned>(lo >> 32), static_cast<unsigned>(hi),
                        static_cast<unsigned>(hi >> 32));
    if (err && bad) atomicOr(err, kErrIndex);
}

// D[row] += rint(2^40 x_old) - rint(2^40 x_new) on the d rows of a column: the exact
// change of the fixed-point residual when the column's value goes from x_old to x_new.
template <int D>
__device__ __forceinline__ void add_change(long long* Dl, const int (&rows)[D], float x_old, float x_new, int* err) {
    const long long delta = (x_old != 0.0f ? to_fx(x_old, err) : 0) - (x_new != 0.0f ? to_fx(x_new, err) : 0);
    if (delta == 0) return;
#pragma unroll
    for (int p = 0; p < D; ++p)
        atomicAdd(reinterpret_cast<unsigned long long*>(Dl + rows[p]), static_cast<unsigned long long>(delta));
}

// The sweep: one workgroup per CU, each owning chunks of kSweepChunk columns (thread t
// takes the kSweepCols consecutive columns from kSweepCols * t) and one segment of the
// candidate list.  All loads that do not depend on the accept decision of the previous
// iteration are issued in one round before it: this workgroup's column indices, the
// score tables, the partial sums of ||r||_1, the previous segment, and both candidates
// for the outer-test bitmask and for the S copy (the decision picks one).  A second
// round gathers the exact residuals of the columns with a candidate row.  DENSE (used
// where the bitmask does not fit in LDS) adds the dense mode: when the row kernel counted
// enough flagged rows, every thread tests its own columns without the bitmask and queue.
// PACKED: the indices come from the packed words (a.Apk), else from A_cols.  Both are
// template parameters, so that no branch separates the index loads from the loads
// before them (the compiler then waits for all of them at the first use of any).
// The workgroup's place in the grid: its launch index, or the mirror of it when rev is set
// (every kernel of an iteration uses the same order; results do not depend on it).
__device__ __forceinline__ int wg_index(int rev) {
    return rev ? static_cast<int>(gridDim.x - 1 - blockIdx.x) : static_cast<int>(blockIdx.x);
}

// REV: the workgroups take their chunks and segments in reverse order (IterParams::wg_rev).
// A template parameter: the sweep uses every scalar register, and one more live value
// (the flag) made the compiler spill and wait for its load at the kernel's start.
template <int D, bool DENSE, bool PACKED, bool REV>
__global__ __launch_bounds__(kSweepBlock) void k_sweep(SweepArgs a) {
    constexpr int kQueueRows = kQueueRowInts / D;
    __shared__ uint32_t bml[kBmLdsWords];
    __shared__ float Tz[kTableStride];
    __shared__ float Te[kTableStride];
    __shared__ float supv[kSweepChunk];
    __shared__ int queue[kSweepChunk];
    __shared__ int qrows[kQueueRowInts];
    __shared__ int qn, seg_f, seg_b, seg_z, seg_upd, seg_inx;
    __shared__ unsigned lhist[kHistBins];   // this workgroup's nonzero candidates by top digit
    __shared__ Slot s_sh;
    __shared__ long long red[kSweepBlock / 64];
    __shared__ unsigned redf[kSweepBlock / 64][2];
    __shared__ bool dense_sh;
    const int it = a.ip.it, me = it & 1, pv = me ^ 1;
    const int tid = threadIdx.x;
    const unsigned wg = REV ? gridDim.x - 1 - blockIdx.x : blockIdx.x;
    const int seg = wg;
    const size_t seg_base = static_cast<size_t>(seg) * a.w.seg_cap;
    DevState* st = a.w.st;
    const int words = (a.m + 31) >> 5;
    const bool bm_regs = words <= kBmPer * kSweepBlock;

    // ---- round 1
    for (int b = threadIdx.x; b < kHistBins; b += kSweepBlock) lhist[b] = 0u;
    // the score tables (read only by the consensus test) are loaded first and stored to
    // LDS before the decision, so they hold no registers past it
    float4 tz4 = make_float4(0.f, 0.f, 0.f, 0.f), te4 = tz4;
    float tzl = 0.0f, tel = 0.0f;
    if (!a.tb.exact) {
        tz4 = reinterpret_cast<const float4*>(a.tb.Tz)[tid];
        te4 = reinterpret_cast<const float4*>(a.tb.Te)[tid];
        if (tid == 0) {
            tzl = a.tb.Tz[kTableN];
            tel = a.tb.Te[kTableN];
        }
    }
    Slot prev{};
    int err = 0;
    if (tid == 0) {
        prev = st->slot[pv];
        err = st->err;
    }
    const int pc = RL0_CHK(st->seg_count[pv][seg], a.w.seg_cap + 1);
    const int pf = RL0_CHK(st->seg_front[pv][seg], pc + 1);
    const unsigned long long kthp = st->kth_key[pv];
    long long lp = tid < kRowGrid ? st->L_part[pv][tid] : 0;
    // flagged-row counts exist only where the bitmask does not fit in LDS
    unsigned fp0 = (DENSE && tid < kRowGrid) ? st->flag_part[pv][0][tid] : 0u;
    unsigned fp1 = (DENSE && tid < kRowGrid) ? st->flag_part[pv][1][tid] : 0u;
    // the previous segment's first front and first back entry of this thread
    int pj = 0, qj = 0;
    float pxp = 0.0f, pxh = 0.0f, qxp = 0.0f, qxh = 0.0f;
    if (tid < a.w.seg_cap) {
        const size_t fb = seg_base + tid, bb = seg_base + (a.w.seg_cap - 1 - tid);
        pj = a.w.cand_j[pv][fb];
        pxp = a.w.cand_x[pv][fb];
        pxh = a.w.cand_h[pv][fb];
        qj = a.w.cand_j[pv][bb];
        qxp = a.w.cand_x[pv][bb];
        qxh = a.w.cand_h[pv][bb];
    }
    uint4 bw0 = make_uint4(0u, 0u, 0u, 0u), bw1 = bw0;
    if (bm_regs && kBmPer * tid < words) {
        bw0 = reinterpret_cast<const uint4*>(a.w.bm[0])[tid];
        bw1 = reinterpret_cast<const uint4*>(a.w.bm[1])[tid];
    }
    // the chunk's indices are loaded last: loads complete in order, so the table stores
    // and the decision below wait only for the loads before them
    int rows[kSweepCols][D];
    uint4 pw[kSweepCols];
    issue_rows<D, PACKED>(a.A, a.Apk, a.n, wg * kSweepChunk, tid, pw, rows);
    if (!a.tb.exact) {
        reinterpret_cast<float4*>(Tz)[tid] = tz4;
        reinterpret_cast<float4*>(Te)[tid] = te4;
        if (tid == 0) {
            Tz[kTableN] = tzl;
            Te[kTableN] = tel;
        }
    }
    for (int off = 32; off > 0; off >>= 1) lp += __shfl_down(lp, off);
    if (DENSE) {
        for (int off = 32; off > 0; off >>= 1) {
            fp0 += __shfl_down(fp0, off);
            fp1 += __shfl_down(fp1, off);
        }
        if ((tid & 63) == 0) {
            redf[tid >> 6][0] = fp0;
            redf[tid >> 6][1] = fp1;
        }
    }
    if ((tid & 63) == 0) red[tid >> 6] = lp;
    __syncthreads();
    if (tid == 0) {
        long long Lt = 0;
        unsigned f0 = 0u, f1 = 0u;
        for (int w = 0; w < kSweepBlock / 64; ++w) Lt += red[w];
        if (DENSE) {
            for (int w = 0; w < kSweepBlock / 64; ++w) {
                f0 += redf[w][0];
                f1 += redf[w][1];
            }
        }
        Slot d = decide_from(prev, err, it, a.ip.n_iters, a.ip.tol_fx, Lt);
        // rows flagged in the bitmask the decision selects
        if (DENSE) dense_sh = 4ull * (d.cur ? f1 : f0) >= static_cast<unsigned long long>(a.m);
        // an analytic retry has nothing to do when the iteration before it was accepted:
        // it only carries x_hat forward and leaves no decision pending
        if (a.ip.retry && d.pending && d.accepted_last)
            d.pending = 0;
        else if (d.pending)
            d.t_step = a.ip.step;
        if (!d.done) d.last_par = me;
        s_sh = d;
        seg_f = 0;
        seg_b = 0;
        seg_z = 0;
        seg_upd = 0;
        seg_inx = 0;
    }
    __syncthreads();
    const Slot s = s_sh;
    unpack_chunk<D, PACKED>(pw, rows, a.n, wg * kSweepChunk, tid);   // the first chunk's indices
    if (wg == 0 && tid == 0) st->slot[me] = s;
    if (s.done) return;
    // (malformed columns stop the loop above, before any of their rows is used)
    RL0_CHECK_ROWS(rows, a.m);
    const bool skip = !s.pending;   // a retry with nothing to retry
    const int c = s.cur;
    const int acc = s.accepted_last;
    // when a quarter of the rows or more pass the outer test, nearly every column has such
    // a row: then every thread tests its own columns directly, without the bitmask filter
    // and the queue (the consensus test recomputes the outer test from the residuals)
    const bool dense = DENSE && !a.learned && !skip && dense_sh;
    const float* __restrict__ r = a.w.r[c];
    const uint32_t* __restrict__ bmg = a.w.bm[c];
    int* __restrict__ out_j = a.w.cand_j[me] + seg_base;
    float* __restrict__ out_x = a.w.cand_x[me] + seg_base;
    float* __restrict__ out_h = a.w.cand_h[me] + seg_base;
    ScoreTables lt = a.tb;
    lt.Tz = Tz;
    lt.Te = Te;
    lt.quant = a.ip.quant;
    lt.qe_bits = a.ip.qe_bits;
    lt.qz_bits = a.ip.qz_bits;

    // ---- the decision picks: outer-test bitmask into LDS, S_trial = S_hat
    if (a.bm_lds) {
        if (bm_regs) {
            if (kBmPer * tid < words) {
                uint4 b;   // selected lane by lane, so the loads above need not complete first
                b.x = c ? bw1.x : bw0.x;
                b.y = c ? bw1.y : bw0.y;
                b.z = c ? bw1.z : bw0.z;
                b.w = c ? bw1.w : bw0.w;
                reinterpret_cast<uint4*>(bml)[tid] = b;
            }
        } else {
            for (int wi = tid; wi < words; wi += kSweepBlock) bml[wi] = bmg[wi];
        }
    } else if (a.bs_lds) {
        const uint32_t* __restrict__ bsg = a.w.bs[c];
        for (int wi = tid; wi < ((a.m + 255) >> 8); wi += kSweepBlock) bml[wi] = bsg[wi];
    }

    for (int chunk = wg; chunk < a.chunks; chunk += gridDim.x) {
        const int cbase = chunk * kSweepChunk;
        if (chunk != static_cast<int>(wg)) {
            issue_rows<D, PACKED>(a.A, a.Apk, a.n, cbase, tid, pw, rows);
            unpack_chunk<D, PACKED>(pw, rows, a.n, cbase, tid);
            RL0_CHECK_ROWS(rows, a.m);
        }
        reinterpret_cast<float4*>(supv)[tid] = make_float4(0.f, 0.f, 0.f, 0.f);
        if (tid == 0) qn = 0;
        __syncthreads();
        // x_hat on this chunk's columns, from the previous segment: its front part and its
        // back part, each walked from entry tid, whose values this thread loaded in round 1
        for (int o = tid; o < pf; o += kSweepBlock) {
            int j = pj;
            float xp = pxp, xh = pxh;
            if (o != tid) {
                const size_t ix = seg_base + RL0_CHK(o, a.w.seg_cap);
                j = a.w.cand_j[pv][ix];
                xp = a.w.cand_x[pv][ix];
                xh = a.w.cand_h[pv][ix];
            }
            const float v = current_value(acc, j, xp, xh, kthp);
            if (v != 0.0f && j >= cbase && j < cbase + kSweepChunk) supv[j - cbase] = v;
        }
        for (int o = tid; o < pc - pf; o += kSweepBlock) {
            int j = qj;
            float xp = qxp, xh = qxh;
            if (o != tid) {
                const size_t ix = seg_base + (a.w.seg_cap - 1 - RL0_CHK(o, a.w.seg_cap));
                j = a.w.cand_j[pv][ix];
                xp = a.w.cand_x[pv][ix];
                xh = a.w.cand_h[pv][ix];
            }
            const float v = current_value(acc, j, xp, xh, kthp);
            if (v != 0.0f && j >= cbase && j < cbase + kSweepChunk) supv[j - cbase] = v;
        }
        __syncthreads();
        float svq[kSweepCols];
#pragma unroll
        for (int q = 0; q < kSweepCols; ++q) svq[q] = supv[q * kSweepBlock + tid];
        if (a.learned || skip) {
            // the learned decision replaces the column test: x'_j = x_hat_j + value (a
            // skipped retry updates nothing and keeps the support)
#pragma unroll
            for (int q = 0; q < kSweepCols; ++q) {
                const int j = cbase + q * kSweepBlock + tid;
                if (j >= a.n) continue;
                const float lv = skip ? 0.0f : a.learned[j];
                const bool upd = !skip && lv == lv;
                if (a.dbg.updated) a.dbg.updated[j] = upd ? 1 : 0;
                if (a.dbg.omega) a.dbg.omega[j] = upd ? lv : 0.0f;
                if (upd) {
                    atomicAdd(&seg_upd, 1);
                    const float xp = svq[q] + lv;
                    const int o = RL0_CHK(atomicAdd(&seg_f, 1), a.w.seg_cap);
                    out_j[o] = j;
                    out_x[o] = xp;
                    out_h[o] = svq[q];
                    if (xp != 0.0f) {
                        atomicAdd(&seg_z, 1);
                        if (fx_inexact(xp)) atomicAdd(&seg_inx, 1);
                        atomicAdd(&lhist[top_digit(xp)], 1u);
                    }
                    add_change<D>(a.w.D, rows[q], svq[q], xp, &st->err);
                } else if (svq[q] != 0.0f) {
                    const int o = RL0_CHK(a.w.seg_cap - 1 - atomicAdd(&seg_b, 1), a.w.seg_cap);
                    out_j[o] = j;
                    out_x[o] = svq[q];
                    out_h[o] = svq[q];
                    atomicAdd(&lhist[top_digit(svq[q])], 1u);
                }
            }
            __syncthreads();
            continue;
        }
        if (dense) {
            // one column at a time, its rows picked by selects (one copy of the test's code)
#pragma unroll 1
            for (int q = 0; q < kSweepCols; ++q) {
                const int j = cbase + q * kSweepBlock + tid;
                if (j >= a.n) continue;
                int rq[D];
                float xhq = svq[0];
#pragma unroll
                for (int p = 0; p < D; ++p) rq[p] = rows[0][p];
#pragma unroll
                for (int qq = 1; qq < kSweepCols; ++qq) {
                    if (q == qq) {
#pragma unroll
                        for (int p = 0; p < D; ++p) rq[p] = rows[qq][p];
                        xhq = svq[qq];
                    }
                }
                float v[D];
#pragma unroll
                for (int p = 0; p < D; ++p) v[p] = r[rq[p]];
                unsigned int cm = 0u;
#pragma unroll
                for (int p = 0; p < D; ++p)
                    if (abs_bits(v[p]) >= a.ip.tau_bits) cm |= 1u << p;
                float om = 0.0f;
                bool upd = false;
                if (cm) {
                    upd = column_update<D>(v, cm, lt, a.ip.alpha, a.ip.l1_test, &om);
                    if (a.dbg.updated) a.dbg.updated[j] = upd ? 1 : 0;
                    if (a.dbg.omega) a.dbg.omega[j] = upd ? om : 0.0f;
                }
                if (upd) {
                    atomicAdd(&seg_upd, 1);
                    const float xp = xhq + om;
                    const int o = RL0_CHK(atomicAdd(&seg_f, 1), a.w.seg_cap);
                    out_j[o] = j;
                    out_x[o] = xp;
                    out_h[o] = xhq;
                    if (xp != 0.0f) {
                        atomicAdd(&seg_z, 1);
                        if (fx_inexact(xp)) atomicAdd(&seg_inx, 1);
                        atomicAdd(&lhist[top_digit(xp)], 1u);
                    }
                    add_change<D>(a.w.D, rq, xhq, xp, &st->err);
                } else if (xhq != 0.0f) {
                    const int o = RL0_CHK(a.w.seg_cap - 1 - atomicAdd(&seg_b, 1), a.w.seg_cap);
                    out_j[o] = j;
                    out_x[o] = xhq;
                    out_h[o] = xhq;
                    atomicAdd(&lhist[top_digit(xhq)], 1u);
                }
            }
            __syncthreads();
            continue;
        }
        // outer test of every row of my columns: one bit each from the bitmask
#pragma unroll
        for (int q = 0; q < kSweepCols; ++q) {
            const int j = cbase + q * kSweepBlock + tid;
            if (j >= a.n) continue;
            unsigned int cm = 0u;
            if (a.bm_lds) {
#pragma unroll
                for (int p = 0; p < D; ++p) {
                    const int row = rows[q][p];
                    cm |= ((bml[row >> 5] >> (row & 31)) & 1u) << p;
                }
            } else {
                // the column's bitmask words from global memory (only under a set summary
                // bit when the summary is in LDS), all loaded before any is used
                uint32_t word[D];
#pragma unroll
                for (int p = 0; p < D; ++p) {
                    const int row = rows[q][p];
                    const bool need = !a.bs_lds || ((bml[row >> 8] >> ((row >> 3) & 31)) & 1u);
                    word[p] = 0u;
                    if (need) word[p] = bmg[row >> 5];
                }
#pragma unroll
                for (int p = 0; p < D; ++p) cm |= ((word[p] >> (rows[q][p] & 31)) & 1u) << p;
            }
            if (cm) {
                const int qi = atomicAdd(&qn, 1);
                queue[RL0_CHK(qi, kSweepChunk)] = j;
                if (qi < kQueueRows) {
#pragma unroll
                    for (int p = 0; p < D; ++p) qrows[qi * D + p] = rows[q][p];
                }
            } else if (svq[q] != 0.0f) {
                // a support column with no candidate row keeps x'_j = x_hat_j: the back
                // of the segment holds the entries with x' = x_hat, the front the others
                const int o = RL0_CHK(a.w.seg_cap - 1 - atomicAdd(&seg_b, 1), a.w.seg_cap);
                out_j[o] = j;
                out_x[o] = svq[q];
                out_h[o] = svq[q];
                atomicAdd(&lhist[top_digit(svq[q])], 1u);
            }
        }
        __syncthreads();
        // ---- round 2: the noisy consensus test of the queued columns, spread over all
        // waves (entry e of a pass goes to wave e % 16, lane e / 16)
        const int nq = qn;
        for (int e0 = 0; e0 < nq; e0 += kSweepBlock) {
            const int e = e0 + (tid & 63) * (kSweepBlock / 64) + (tid >> 6);
            if (e >= nq) continue;
            const int jq = queue[e];
            int rr[D];
            if (e < kQueueRows) {
#pragma unroll
                for (int p = 0; p < D; ++p) rr[p] = qrows[e * D + p];
            } else {
                const int32_t* __restrict__ col = a.A + static_cast<size_t>(RL0_CHK(jq, a.n)) * D;
#pragma unroll
                for (int p = 0; p < D; ++p) rr[p] = RL0_CHK(col[p], a.m);
            }
            float v[D];
#pragma unroll
            for (int p = 0; p < D; ++p) v[p] = r[rr[p]];
            const float xhq = supv[RL0_CHK(jq - cbase, kSweepChunk)];
            unsigned int cm = 0u;
#pragma unroll
            for (int p = 0; p < D; ++p)
                if (abs_bits(v[p]) >= a.ip.tau_bits) cm |= 1u << p;
            float om = 0.0f;
            const bool upd = column_update<D>(v, cm, lt, a.ip.alpha, a.ip.l1_test, &om);
            if (a.dbg.updated) a.dbg.updated[jq] = upd ? 1 : 0;
            if (a.dbg.omega) a.dbg.omega[jq] = upd ? om : 0.0f;
            if (upd) atomicAdd(&seg_upd, 1);
            if (upd) {
                // an updated column goes to the front; its residual change is added at
                // once, as if H_k keeps it (the select kernel takes back what it drops)
                const float xp = xhq + om;
                const int o = RL0_CHK(atomicAdd(&seg_f, 1), a.w.seg_cap);
                out_j[o] = jq;
                out_x[o] = xp;
                out_h[o] = xhq;
                if (xp != 0.0f) {
                    atomicAdd(&seg_z, 1);
                    if (fx_inexact(xp)) atomicAdd(&seg_inx, 1);
                    atomicAdd(&lhist[top_digit(xp)], 1u);
                }
                add_change<D>(a.w.D, rr, xhq, xp, &st->err);
            } else if (xhq != 0.0f) {
                const int o = RL0_CHK(a.w.seg_cap - 1 - atomicAdd(&seg_b, 1), a.w.seg_cap);
                out_j[o] = jq;
                out_x[o] = xhq;
                out_h[o] = xhq;
                atomicAdd(&lhist[top_digit(xhq)], 1u);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        st->seg_count[me][seg] = seg_f + seg_b;
        st->seg_front[me][seg] = seg_f;
        st->seg_nz[me][seg] = seg_z + seg_b;
        st->seg_updates[me][seg] = seg_upd;
        if (seg_inx) atomicAdd(&st->inexact_x, seg_inx);
    }
    // H_k's first radix digit, counted for every workgroup at once
    for (int b = tid; b < kHistBins; b += kSweepBlock) {
        const unsigned v = lhist[b];
        if (v) atomicAdd(&st->hk_hist[me][wg % kHistCopies][b], v);
    }
}

// ------------------------------------------------------------------ H_k and residual change

// ------------------------------------------------------------------ H_k and the rows

struct FinishArgs {
    const int32_t* A;
    int d, k, m;
    Workspace w;
    int it;
    uint32_t tau_next;
    int summary;    // also write the 8-row summaries of both bitmasks
    int count_flags;   // also count the flagged rows of both bitmasks (the bitmask does not
                       // fit in the sweep's LDS; the counts select its dense mode)
    int pre;        // k_hk_classify ran before: drops below the boundary bucket are in D and
                    // the bucket's entries are listed in w.bkey / w.bx
    int log;        // record the iteration in the per-iteration log
    float t;        // the iteration's t (for that log)
    int wg_rev;     // workgroups take their row ranges in reverse order
    int n;          // columns
};


constexpr int kWinKeys = 12288;   // candidates a window of the row kernel maps in LDS
constexpr int kWinPer = kWinKeys / kRowBlock;   // their loads in flight per thread
constexpr int kShortSegs = 256;  // mean candidates per segment up to which a thread maps a segment
constexpr int kBucketCap = 4096;  // entries of H_k's boundary bucket kept in LDS
constexpr int kCorrRows = 8192;   // rows a correction window of the row kernel covers

// Calls fn(j, x'_j, ok) for every candidate of the iteration, in windows of kWinKeys: an
// entry -> segment map is written in LDS (by a thread per segment when segments are short,
// else thread t maps kWinPer consecutive entries from one binary search over the segments'
// starts), then every thread issues its kWinPer loads before it uses any.  Every lane of the workgroup calls fn the same number of times
// (ok = false past the count), so fn may use wave-wide operations.
template <class F>
__device__ __forceinline__ void for_candidates(int count, int nseg, int cap, const int* seg_start, const int* seg_cnt,
                                               const int* seg_frt, unsigned short* segmap, const int* __restrict__ cj,
                                               const float* __restrict__ cx, F&& fn) {
    const int tid = threadIdx.x;
    // short segments: a thread per segment writes its own entries; long ones would make
    // that serial, so then each thread maps a run of entries instead
    const bool per_segment = count <= kShortSegs * nseg;
    for (int w0 = 0; w0 < count; w0 += kWinKeys) {
        const int e_lo = w0 + tid * kWinPer;
        if (per_segment) {
            if (tid < nseg) {
                const int st0 = seg_start[tid], c = seg_cnt[tid];
                const int lo = max(0, w0 - st0), hi = min(c, w0 + kWinKeys - st0);
                for (int o = lo; o < hi; ++o) segmap[st0 + o - w0] = static_cast<unsigned short>(tid);
            }
        } else if (e_lo < count) {
            // the segment holding e_lo: the last one that starts at or before it (empty
            // segments share their start with the next one, which wins)
            int lo = 0, hi = nseg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (seg_start[mid] <= e_lo) lo = mid; else hi = mid - 1;
            }
            int sg = lo;
            for (int k = 0; k < kWinPer && e_lo + k < count; ++k) {
                while (sg + 1 < nseg && seg_start[sg + 1] <= e_lo + k) ++sg;
                segmap[e_lo + k - w0] = static_cast<unsigned short>(sg);
            }
        }
        __syncthreads();
        size_t ixs[kWinPer];
#pragma unroll
        for (int q = 0; q < kWinPer; ++q) {
            const int e = q * kRowBlock + tid;
            ixs[q] = 0;
            if (w0 + e < count) {
                const int sg = segmap[e];
                ixs[q] = seg_phys(sg, cap, seg_frt[sg], w0 + e - seg_start[sg]);
            }
        }
        float xs[kWinPer];
        int js[kWinPer];
#pragma unroll
        for (int q = 0; q < kWinPer; ++q) {
            xs[q] = cx[ixs[q]];
            js[q] = cj[ixs[q]];
        }
#pragma unroll
        for (int q = 0; q < kWinPer; ++q) fn(js[q], xs[q], w0 + q * kRowBlock + tid < count);
        __syncthreads();   // the map is rewritten by the next window
    }
}

// For m > kPreRows, H_k's first step runs once here instead of in every workgroup of the
// row kernel.  The boundary digit d1 of the first radix digit comes from the sweep's
// histogram.  Workgroup b takes a contiguous slice of the candidates.  A column below
// bucket d1 is dropped, and its change is taken back on all of its rows at once with 64-bit
// atomics on D (exact, so the order does not matter).  When bucket d1 is not kept whole,
// its entries are listed with their keys for the row kernel's later digits.
__global__ __launch_bounds__(kRowBlock) void k_hk_classify(FinishArgs a) {
    __shared__ unsigned hist[kHistBins];
    __shared__ unsigned scan[kRowBlock / 64];
    __shared__ int seg_start[kSweepGridMax];
    __shared__ int seg_frt[kSweepGridMax];
    __shared__ int wtot[kSweepGridMax / 64];
    __shared__ int digit;
    __shared__ unsigned above, bucket;
    __shared__ int nz_sh;
    const int me = a.it & 1;
    DevState* st = a.w.st;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nseg = a.w.sweep_grid;
    const int cap = a.w.seg_cap;
    const Slot s = st->slot[me];
    int myc = 0, myz = 0;
    if (tid < nseg) {
        myc = RL0_CHK(st->seg_count[me][tid], cap + 1);
        myz = st->seg_nz[me][tid];
        seg_frt[tid] = RL0_CHK(st->seg_front[me][tid], myc + 1);
    }
    if (tid == 0) nz_sh = 0;
    __syncthreads();
    if (s.done) return;
    if (tid < kSweepGridMax) {
        int z = myz;
        for (int off = 32; off > 0; off >>= 1) z += __shfl_down(z, off);
        if (lane == 0 && z) atomicAdd(&nz_sh, z);
    }
    __syncthreads();
    if (nz_sh <= a.k) return;   // every candidate is kept
    unsigned h_hi = 0u, h_lo = 0u;
#pragma unroll
    for (int cp = 0; cp < kHistCopies; ++cp) {
        h_hi += st->hk_hist[me][cp][tid];
        h_lo += st->hk_hist[me][cp][tid + kRowBlock];
    }
    hist[tid] = h_hi;
    hist[tid + kRowBlock] = h_lo;
    const int count = segment_scan(myc, nseg, seg_start, wtot);   // its barriers publish hist
    find_digit(hist, static_cast<unsigned>(a.k), scan, &digit, &above, &bucket);
    const unsigned d1 = static_cast<unsigned>(digit);
    const bool gather = static_cast<unsigned>(a.k) - above != bucket;
    const int* __restrict__ cj = a.w.cand_j[me];
    const float* __restrict__ cx = a.w.cand_x[me];
    const int per = (count + gridDim.x - 1) / gridDim.x;
    const int e0 = wg_index(a.wg_rev) * per, e1 = min(count, e0 + per);
    for (int base = e0; base < e1; base += kRowBlock) {
        const int e = base + tid;
        float x = 0.0f;
        int j = 0;
        if (e < e1) {
            int lo = 0, hi = nseg - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (seg_start[mid] <= e) lo = mid; else hi = mid - 1;
            }
            const size_t ix = seg_phys(lo, cap, seg_frt[lo], e - seg_start[lo]);
            x = cx[ix];
            j = cj[ix];
        }
        const unsigned dg = x != 0.0f ? top_digit(x) : 0u;
        if (x != 0.0f && dg < d1) {
            const long long delta = to_fx(x, &st->err);
            const int32_t* __restrict__ col = a.A + static_cast<size_t>(RL0_CHK(j, a.n)) * a.d;
            for (int p = 0; p < a.d; ++p)
                atomicAdd(reinterpret_cast<unsigned long long*>(&a.w.D[RL0_CHK(col[p], a.m)]),
                          static_cast<unsigned long long>(delta));
        }
        const bool put = gather && x != 0.0f && dg == d1;
        const int slot = wave_append(&st->bucket_n[me], put);
        if (put) {
            const int b = RL0_CHK(slot, static_cast<long long>(nseg) * cap);
            a.w.bkey[me][b] = hk_key(j, x);
            a.w.bx[me][b] = x;
        }
    }
}

// One kernel after the sweep.  H_k: when the nonzero candidates number at most k (the
// common case once the support has formed) every one is kept and the sweep has already
// added every residual change to D.  Otherwise every workgroup finds the k-th largest
// key (|x'_j| bits, then smaller j) by an 11-bit radix select over the candidates and
// takes back, on its own rows, the columns H_k drops (+rint(2^40 x'_j) per row).
// Then, on its rows: S_trial = S_hat + D (D cleared for the next iteration), the
// rounded residual r = fl32(2^-40 S), the partial sum of ||r||_1 and the outer-test
// bitmasks of the next threshold for both possible outcomes of the decision.
__global__ __launch_bounds__(kRowBlock) void k_finish_rows(FinishArgs a) {
    __shared__ unsigned short segmap[kWinKeys];
    __shared__ unsigned long long bkey[kBucketCap];
    __shared__ float bx[kBucketCap];
    __shared__ long long corr[kCorrRows];
    __shared__ unsigned hist[kHistBins];
    __shared__ unsigned scan[kRowBlock / 64];
    __shared__ int seg_cnt[kSweepGridMax];
    __shared__ int seg_frt[kSweepGridMax];
    __shared__ int seg_start[kSweepGridMax];
    __shared__ int wtot[kSweepGridMax / 64];
    __shared__ long long sh[kRowBlock / 64];
    __shared__ unsigned flw[kRowBlock / 64][2];
    __shared__ int digit;
    __shared__ unsigned above, bucket;
    __shared__ int nz_sh, upd_sh, bn;
    const int me = a.it & 1;
    DevState* st = a.w.st;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int nseg = a.w.sweep_grid;
    const int cap = a.w.seg_cap;
    const int words = (a.m + 31) >> 5;
    // rows of this workgroup: [row0, row1), whole multiples of the block
    const int per = ((a.m + gridDim.x * kRowBlock - 1) / (gridDim.x * kRowBlock)) * kRowBlock;
    const int wg = wg_index(a.wg_rev);
    const int row0 = wg * per;
    const int row1 = min(a.m, row0 + per);

    // the per-iteration log (workgroup 0): this iteration's record, and the decision on the
    // iteration before, which this iteration's sweep took (its trial norm is the sum of the
    // partial sums that iteration's row kernel left in L_part)
    const bool log_wg = a.log && wg == 0;
    const unsigned long long t_entry = (log_wg && tid == 0) ? wall_clock64() : 0ull;
    long long lt_prev = 0;
    if (log_wg && tid < 64)
        for (int b = tid; b < kRowGrid; b += 64) lt_prev += st->L_part[me ^ 1][b];
    // ---- round 1: slot, segment sizes and this workgroup's first rows
    const Slot s = st->slot[me];
    int myc = 0, myf = 0, myz = 0, myu = 0;
    if (tid < nseg) {
        myc = RL0_CHK(st->seg_count[me][tid], cap + 1);
        myf = RL0_CHK(st->seg_front[me][tid], myc + 1);
        myz = st->seg_nz[me][tid];
        if (wg == 0) myu = st->seg_updates[me][tid];
    }
    long long s0 = 0, s1 = 0, dl = 0;
    {
        const int i = row0 + tid;
        if (i < row1) {
            s0 = a.w.S[0][i];
            s1 = a.w.S[1][i];
            dl = a.w.D[i];
        }
    }
    // the next iteration's first-digit histograms are cleared here, a slice per workgroup
    for (int i = wg * kRowBlock + tid; i < kHistCopies * kHistBins; i += gridDim.x * kRowBlock)
        (&st->hk_hist[me ^ 1][0][0])[i] = 0u;
    if (wg == 0 && tid == 0) st->bucket_n[me ^ 1] = 0;
    if (tid == 0) {
        nz_sh = 0;
        upd_sh = 0;
    }
    if (tid < kSweepGridMax) {
        seg_cnt[tid] = myc;
        seg_frt[tid] = myf;
    }
    if (log_wg && tid < 64) {
        // recorded before the return below: the decision that stopped the loop is logged too
        for (int off = 32; off > 0; off >>= 1) lt_prev += __shfl_down(lt_prev, off);
        if (tid == 0 && st->slot[me ^ 1].pending) log_decision(st, s, lt_prev);
    }
    __syncthreads();
    if (s.done) return;
    const int c = s.cur, tr = c ^ 1;
    if (tid < kSweepGridMax) {
        int z = myz, u = myu;
        for (int off = 32; off > 0; off >>= 1) {
            z += __shfl_down(z, off);
            u += __shfl_down(u, off);
        }
        if (lane == 0) {
            if (z) atomicAdd(&nz_sh, z);
            if (u) atomicAdd(&upd_sh, u);
        }
    }
    __syncthreads();
    if (wg == 0 && tid == 0) {
        if (upd_sh) atomicAdd(&st->updates_total, upd_sh);
        if (log_wg) {
            if (s.pending && s.iterations < kLogCap) {
                IterLog& lg = st->log[s.iterations];
                lg.updates = upd_sh;
                lg.t = a.t;
                lg.it = a.it;
                lg.rows_start = t_entry;
            }
        }
    }
    const bool all_kept = nz_sh <= a.k;
    const int* __restrict__ cj = a.w.cand_j[me];
    const float* __restrict__ cx = a.w.cand_x[me];

    // ---- H_k, only when something is dropped.  The first radix digit's histogram is the
    // sweep's (summed over its copies).  Candidates below the boundary bucket are dropped
    // and those above it kept.  One pass over the candidates takes back the dropped ones on
    // the first correction window of rows and, when the bucket is not kept whole, collects
    // the bucket's entries in LDS; the later digits are then selected among them alone.
    unsigned long long kth = 1ull << 32;   // every nonzero entry is kept
    int count = 0;
    unsigned d1 = 0u;
    int nbk = 0;
    unsigned h_hi = 0u, h_lo = 0u;
    if (!all_kept) {
#pragma unroll
        for (int cp = 0; cp < kHistCopies; ++cp) {
            h_hi += st->hk_hist[me][cp][tid];
            h_lo += st->hk_hist[me][cp][tid + kRowBlock];
        }
    }
    // +rint(2^40 x'_j) on the rows [cb, ce) of a column H_k drops
    int cb = row0, ce = min(row1, row0 + kCorrRows);
    auto take_back = [&](int j, float x) {
        const long long delta = to_fx(x, &st->err);
        const int32_t* __restrict__ col = a.A + static_cast<size_t>(RL0_CHK(j, a.n)) * a.d;
        for (int p = 0; p < a.d; ++p) {
            const int row = col[p];
            if (row >= cb && row < ce)
                atomicAdd(reinterpret_cast<unsigned long long*>(&corr[row - cb]), static_cast<unsigned long long>(delta));
        }
    };
    if (!all_kept) {
        if (!a.pre) count = segment_scan(myc, nseg, seg_start, wtot);
        if (tid == 0) bn = 0;
        for (int i = tid; i < ce - cb; i += kRowBlock) corr[i] = 0;
        hist[tid] = h_hi;
        hist[tid + kRowBlock] = h_lo;
        __syncthreads();
        find_digit(hist, static_cast<unsigned>(a.k), scan, &digit, &above, &bucket);
        d1 = static_cast<unsigned>(digit);
        unsigned long long prefix = static_cast<unsigned long long>(d1) << 52;
        unsigned long long pmask = 0x7FFull << 52;
        unsigned rem = static_cast<unsigned>(a.k) - above;
        bool exact = (rem == bucket);
        const bool gather = !exact;
        if (a.pre) {
            // the columns below the bucket are already taken back; the bucket is listed
            nbk = gather ? RL0_CHK(st->bucket_n[me], static_cast<long long>(nseg) * cap + 1) : 0;
            if (nbk <= kBucketCap) {
                for (int e = tid; e < nbk; e += kRowBlock) {
                    bkey[e] = a.w.bkey[me][e];
                    bx[e] = a.w.bx[me][e];
                }
            }
            __syncthreads();
        } else {
            for_candidates(count, nseg, cap, seg_start, seg_cnt, seg_frt, segmap, cj, cx, [&](int j, float x, bool ok) {
                if (!ok || x == 0.0f) return;
                const unsigned dg = top_digit(x);
                if (dg < d1) {
                    take_back(j, x);
                } else if (gather && dg == d1) {
                    const int slot = atomicAdd(&bn, 1);
                    if (slot < kBucketCap) {
                        bkey[slot] = hk_key(j, x);
                        bx[slot] = x;
                    }
                }
            });
            nbk = bn;
        }
        for (int pass = 1; pass < 6 && !exact; ++pass) {
            const int sft = pass < 5 ? 52 - 11 * pass : 0;
            const unsigned dmask = pass < 5 ? 0x7FFu : 0xFFu;
            hist[tid] = 0u;
            hist[tid + kRowBlock] = 0u;
            __syncthreads();
            if (nbk <= kBucketCap) {
                for (int e0 = 0; e0 < nbk; e0 += kRowBlock) {
                    const int e = e0 + tid;
                    const unsigned long long key = e < nbk ? bkey[e] : 0ull;
                    hist_add(hist, static_cast<unsigned>((key >> sft) & dmask), e < nbk && (key & pmask) == prefix);
                }
                __syncthreads();
            } else if (a.pre) {
                // the bucket's list in global memory
                for (int e0 = 0; e0 < nbk; e0 += kRowBlock) {
                    const int e = e0 + tid;
                    const unsigned long long key = e < nbk ? a.w.bkey[me][e] : 0ull;
                    hist_add(hist, static_cast<unsigned>((key >> sft) & dmask), e < nbk && (key & pmask) == prefix);
                }
                __syncthreads();
            } else {
                // the bucket did not fit: the pass reads every candidate
                for_candidates(count, nseg, cap, seg_start, seg_cnt, seg_frt, segmap, cj, cx,
                               [&](int j, float x, bool ok) {
                                   const unsigned long long key = (ok && x != 0.0f) ? hk_key(j, x) : 0ull;
                                   hist_add(hist, static_cast<unsigned>((key >> sft) & dmask),
                                            key != 0ull && (key & pmask) == prefix);
                               });
            }
            find_digit(hist, rem, scan, &digit, &above, &bucket);
            prefix |= static_cast<unsigned long long>(digit) << sft;
            pmask |= static_cast<unsigned long long>(dmask) << sft;
            rem -= above;
            exact = (rem == bucket);
        }
        kth = prefix;
        // the bucket's dropped entries
        if (gather) {
            if (nbk <= kBucketCap) {
                for (int e = tid; e < nbk; e += kRowBlock) {
                    const unsigned long long key = bkey[e];
                    if (key < kth) take_back(static_cast<int>(0xFFFFFFFFu - static_cast<uint32_t>(key)), bx[e]);
                }
            } else if (a.pre) {
                for (int e = tid; e < nbk; e += kRowBlock) {
                    const unsigned long long key = a.w.bkey[me][e];
                    if (key < kth) take_back(static_cast<int>(0xFFFFFFFFu - static_cast<uint32_t>(key)), a.w.bx[me][e]);
                }
            } else {
                for_candidates(count, nseg, cap, seg_start, seg_cnt, seg_frt, segmap, cj, cx,
                               [&](int j, float x, bool ok) {
                                   if (ok && x != 0.0f && top_digit(x) == d1 && hk_key(j, x) < kth) take_back(j, x);
                               });
            }
        }
        __syncthreads();
    }
    if (wg == 0 && tid == 0) st->kth_key[me] = kth;

    // ---- the rows, a correction window of kCorrRows rows at a time
    long long l = 0;
    unsigned ft = 0u, fc = 0u;   // rows flagged in the two bitmasks (wave-uniform)
    for (; cb < row1; cb += kCorrRows) {
        ce = min(row1, cb + kCorrRows);
        if (!all_kept && cb != row0) {
            // a later window: the dropped columns' rows in it
            for (int i = tid; i < ce - cb; i += kRowBlock) corr[i] = 0;
            __syncthreads();
            const bool bucket_in_lds = nbk <= kBucketCap;
            if (!a.pre) {
                for_candidates(count, nseg, cap, seg_start, seg_cnt, seg_frt, segmap, cj, cx, [&](int j, float x, bool ok) {
                    if (!ok || x == 0.0f) return;
                    const unsigned dg = top_digit(x);
                    if (dg < d1 || (dg == d1 && !bucket_in_lds && hk_key(j, x) < kth)) take_back(j, x);
                });
            } else if (!bucket_in_lds) {
                for (int e = tid; e < nbk; e += kRowBlock) {
                    const unsigned long long key = a.w.bkey[me][e];
                    if (key < kth) take_back(static_cast<int>(0xFFFFFFFFu - static_cast<uint32_t>(key)), a.w.bx[me][e]);
                }
            }
            if (bucket_in_lds) {
                for (int e = tid; e < nbk; e += kRowBlock) {
                    const unsigned long long key = bkey[e];
                    if (key < kth) take_back(static_cast<int>(0xFFFFFFFFu - static_cast<uint32_t>(key)), bx[e]);
                }
            }
            __syncthreads();
        }
        for (int base = cb; base < ce; base += kRowBlock) {
            const int i = base + tid;
            // the next block's rows are loaded before this block's work (its values are
            // in s0, s1, dl: the first block's from round 1); a clamped row, no per-lane
            // branch, so the loads overlap this block rather than wait for it
            const int nb = base + kRowBlock;
            long long n0 = 0, n1 = 0, nd = 0;
            if (nb < row1) {
                const int ni = min(nb + tid, a.m - 1);
                n0 = a.w.S[0][ni];
                n1 = a.w.S[1][ni];
                nd = a.w.D[ni];
            }
            if (!all_kept && i < ce) dl += corr[i - cb];
            bool bt = false, bc = false;
            if (i < row1) {
                // the trial residual: the current one plus this iteration's changes
                const long long sc = c ? s1 : s0;
                const long long snew = sc + dl;
                a.w.S[tr][i] = snew;
                a.w.D[i] = 0;
                const float v = from_fx(snew);
                a.w.r[tr][i] = v;
                l += l1_term(v);
                bt = abs_bits(v) >= a.tau_next;
                bc = abs_bits(from_fx(sc)) >= a.tau_next;
            }
            const unsigned long long bmt = __ballot(bt);
            const unsigned long long bmc = __ballot(bc);
            if (a.count_flags) {
                ft += static_cast<unsigned>(__popcll(bmt));
                fc += static_cast<unsigned>(__popcll(bmc));
            }
            if (lane == 0) {
                const int wb = base + (tid & ~63);
                store_bits(a.w.bm[tr], words, wb, bmt);
                store_bits(a.w.bm[c], words, wb, bmc);
                if (a.summary && wb < a.m) {
                    // 8 summary bits for the wave's 64 rows, one byte
                    reinterpret_cast<uint8_t*>(a.w.bs[tr])[wb >> 6] = summary8(bmt);
                    reinterpret_cast<uint8_t*>(a.w.bs[c])[wb >> 6] = summary8(bmc);
                }
            }
            s0 = n0;
            s1 = n1;
            dl = nd;
        }
        if (!all_kept) __syncthreads();   // corr is reused by the next window
    }
    if (a.count_flags && lane == 0) {
        flw[tid >> 6][0] = ft;
        flw[tid >> 6][1] = fc;
    }
    const long long tot = block_sum_rows(l, sh);   // its barrier also publishes flw
    if (tid == 0) {
        st->L_part[me][wg] = tot;
        if (a.count_flags) {
            unsigned st_t = 0u, st_c = 0u;
            for (int w = 0; w < kRowBlock / 64; ++w) {
                st_t += flw[w][0];
                st_c += flw[w][1];
            }
            st->flag_part[me][tr][wg] = st_t;
            st->flag_part[me][c][wg] = st_c;
        }
        if (log_wg && s.pending && s.iterations < kLogCap) st->log[s.iterations].rows_end = wall_clock64();
    }
}

// ------------------------------------------------------------------ final decision

__global__ __launch_bounds__(256) void k_peek(DevState* st, int it, int n_iters, double tol_fx) {
    __shared__ long long red[4];
    const long long Lt = trial_l1_block(st, (it & 1) ^ 1, red);
    if (threadIdx.x == 0) {
        const Slot s = decide(st, it, n_iters, tol_fx, Lt);
        st->peek_cur = s.cur;
        st->peek_done = s.done;
        st->peek_acc = s.accepted_last;
        st->adapt_sum = 0;
    }
}

// adaptive_k: the sum over x_hat = H_k(x') of iteration it (segments of parity it & 1) of
// rint(2^30 fl32(1 - Tz(|x_hat_j|))).  One workgroup per segment; runs after k_peek.
__global__ __launch_bounds__(256) void k_adapt_sum(const Workspace w, ScoreTables tb, int it) {
    __shared__ long long red[4];
    const int par = it & 1;
    const int seg = blockIdx.x;
    const int cnt = RL0_CHK(w.st->seg_count[par][seg], w.seg_cap + 1);
    const int front = RL0_CHK(w.st->seg_front[par][seg], cnt + 1);
    const unsigned long long kth = w.st->kth_key[par];
    long long acc = 0;
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const size_t ix = static_cast<size_t>(seg) * w.seg_cap + (e < front ? e : w.seg_cap - 1 - (e - front));
        const int j = w.cand_j[par][ix];
        const float v = current_value(1, j, w.cand_x[par][ix], w.cand_h[par][ix], kth);
        if (v == 0.0f) continue;
        const float z = score(tb.Tz, tb.inv_h_z, tb.exact, fabsf(v));
        acc += __double2ll_rn(static_cast<double>(1.0f - z) * kTwo30);
    }
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const long long t = red[0] + red[1] + red[2] + red[3];
        if (t) atomicAdd(reinterpret_cast<unsigned long long*>(&w.st->adapt_sum), static_cast<unsigned long long>(t));
    }
}

// The outer-test bitmask of residual buffer b redone for threshold tau; for m past the LDS
// bitmask also its 8-row summary and the flagged-row counts the next sweep's dense mode
// reads (flag_part of parity it & 1, buffer b).
__global__ __launch_bounds__(kRowBlock) void k_rebuild_outer(const float* __restrict__ r, uint32_t* __restrict__ bm,
                                                             uint8_t* __restrict__ bs, int m, uint32_t tau,
                                                             unsigned* __restrict__ flags) {
    __shared__ unsigned flw[kRowBlock / 64];
    const int words = (m + 31) >> 5;
    unsigned fl = 0u;
    for (int base = blockIdx.x * kRowBlock; base < m; base += gridDim.x * kRowBlock) {
        const int i = base + threadIdx.x;
        const bool bit = i < m && abs_bits(r[i]) >= tau;
        const unsigned long long b = __ballot(bit);
        fl += static_cast<unsigned>(__popcll(b));
        if ((threadIdx.x & 63) == 0) {
            const int wb = base + (threadIdx.x & ~63);
            store_bits(bm, words, wb, b);
            if (bs && wb < m) bs[wb >> 6] = summary8(b);
        }
    }
    if ((threadIdx.x & 63) == 0) flw[threadIdx.x >> 6] = fl;
    __syncthreads();
    if (threadIdx.x == 0 && flags) {
        unsigned f = 0u;
        for (int w = 0; w < kRowBlock / 64; ++w) f += flw[w];
        flags[blockIdx.x] = f;
    }
}

__global__ __launch_bounds__(256) void k_decide_only(DevState* st, int it, int n_iters, double tol_fx, int log_on) {
    __shared__ long long red[4];
    const long long Lt = trial_l1_block(st, (it & 1) ^ 1, red);
    if (threadIdx.x == 0) {
        const Slot p = st->slot[(it & 1) ^ 1];
        const Slot d = decide_from(p, st->err, it, n_iters, tol_fx, Lt);
        st->slot[it & 1] = d;
        if (p.pending && log_on) log_decision(st, d, Lt);
    }
}

// x_out = x_hat (or, with trial = 1, H_k(x') of the last executed iteration) from the
// candidate segments of the last executed iteration; x_out holds zeros beforehand.  With decide = 1 every workgroup first takes the
// decision on the last iteration (it_end = n_iters) itself, and workgroup 0 records it.
__global__ __launch_bounds__(256) void k_copy_out(const Workspace w, float* __restrict__ x_out, int n, int it_end,
                                                  int trial, int decide_last, int n_iters, double tol_fx, int log_on) {
    __shared__ long long red[4];
    __shared__ Slot fin_sh;
    if (decide_last) {
        const long long Lt = trial_l1_block(w.st, (it_end & 1) ^ 1, red);
        if (threadIdx.x == 0) {
            const Slot p = w.st->slot[(it_end & 1) ^ 1];
            fin_sh = decide_from(p, w.st->err, it_end, n_iters, tol_fx, Lt);
            if (blockIdx.x == 0) {
                w.st->slot[it_end & 1] = fin_sh;
                if (p.pending && log_on) log_decision(w.st, fin_sh, Lt);
            }
        }
    } else if (threadIdx.x == 0) {
        fin_sh = w.st->slot[it_end & 1];
    }
    __syncthreads();
    const Slot fin = fin_sh;
    const int par = fin.last_par;   // the parity of it0 - 1 if nothing ran
    const int acc = trial ? 1 : fin.accepted_last;
    const unsigned long long kth = w.st->kth_key[par];
    const int seg = blockIdx.x;
    const int cnt = RL0_CHK(w.st->seg_count[par][seg], w.seg_cap + 1);
    const int front = RL0_CHK(w.st->seg_front[par][seg], cnt + 1);
    for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
        const size_t ix = static_cast<size_t>(seg) * w.seg_cap + (e < front ? e : w.seg_cap - 1 - (e - front));
        const int j = w.cand_j[par][ix];
        const float v = current_value(acc, j, w.cand_x[par][ix], w.cand_h[par][ix], kth);
        if (v != 0.0f) x_out[RL0_CHK(j, n)] = v;
    }
}

inline int blocks(long long n, int b) { return static_cast<int>((n + b - 1) / b); }

}  // namespace

hipError_t device_check_read(int* line, hipStream_t s) {
#if RL0_DEVICE_CHECKS
    unsigned v = 0u;
    hipError_t e = hipMemcpyFromSymbolAsync(&v, HIP_SYMBOL(g_check_line), sizeof(v), 0, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && v != 0u) {
        const unsigned zero = 0u;
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_check_line), &zero, sizeof(zero), 0, hipMemcpyHostToDevice, s);
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

namespace {

int sweep_grid(int n) {
    // one workgroup per CU, persistent over chunks of kSweepChunk columns
    const int chunks = blocks(n, kSweepChunk);
    return chunks < kSweepGridMax ? chunks : kSweepGridMax;
}

// Workgroups of the row kernel after the sweep: one per kRowBlock rows, at most kRowGrid
// (each holds a partial sum; the unused ones stay zero).  Every workgroup runs H_k's
// selection for itself, so fewer of them read the candidates fewer times.
int finish_grid(int m) {
    const int g = blocks(m, kRowBlock);
    return g < 1 ? 1 : (g > kRowGrid ? kRowGrid : g);
}

int seg_capacity(int n) {
    const int chunks = blocks(n, kSweepChunk);
    return blocks(chunks, sweep_grid(n)) * kSweepChunk;
}

// A launch with optional HIP events that take the dispatch's own start and end times.
template <class K, class Args>
hipError_t launch_timed(K kernel, int grid, int block, hipStream_t s, const hipEvent_t* ev, const Args& a) {
    if (ev) {
        hipExtLaunchKernelGGL(kernel, dim3(grid), dim3(block), 0, s, ev[0], ev[1], 0, a);
    } else {
        kernel<<<grid, block, 0, s>>>(a);
    }
    return hipGetLastError();
}

template <int D, bool DENSE, bool PACKED>
hipError_t launch_sweep_v(const SweepArgs& a, hipStream_t s, const hipEvent_t* ev) {
    if (a.ip.wg_rev) return launch_timed(k_sweep<D, DENSE, PACKED, true>, a.w.sweep_grid, kSweepBlock, s, ev, a);
    return launch_timed(k_sweep<D, DENSE, PACKED, false>, a.w.sweep_grid, kSweepBlock, s, ev, a);
}

template <int D>
hipError_t launch_sweep_d(const SweepArgs& a, hipStream_t s, const hipEvent_t* ev) {
    // the flagged-row counts exist where the bitmask does not fit in LDS; packing fits
    // such an m only for d <= 6 (18 bits a row or more)
    if (a.Apk) {
        if (a.bm_lds) return launch_sweep_v<D, false, true>(a, s, ev);
        if constexpr (D <= 6) return launch_sweep_v<D, true, true>(a, s, ev);
        return hipErrorInvalidValue;
    }
    if (a.bm_lds) return launch_sweep_v<D, false, false>(a, s, ev);
    return launch_sweep_v<D, true, false>(a, s, ev);
}

template <int D>
bool pack_fits(int m) {
    constexpr int F = Packing<D>::kField;
    return F >= 32 || static_cast<long long>(m) <= (1ll << F);
}

// The packed indices when they fit (d <= 16 and m <= 2^field); false if not.
template <int D>
bool launch_pack_d(const int32_t* A, int n, int m, uint4* Apk, int* err, float* x_zero, hipStream_t s) {
    if (!pack_fits<D>(m)) return false;
    k_pack_cols<D><<<blocks(n, 256), 256, 0, s>>>(A, n, m, Apk, err, x_zero);
    return true;
}

// Packs A_cols when its rows fit the packed fields (false otherwise: nothing ran), and
// validates it and zeroes x_zero on the way when those are given.
bool launch_pack(int d, const int32_t* A, int n, int m, uint4* Apk, int* err, float* x_zero, hipStream_t s) {
    switch (d) {
#define RL0_PK(D) \
    case D: return launch_pack_d<D>(A, n, m, Apk, err, x_zero, s);
        RL0_PK(1) RL0_PK(2) RL0_PK(3) RL0_PK(4) RL0_PK(5) RL0_PK(6) RL0_PK(7) RL0_PK(8)
        RL0_PK(9) RL0_PK(10) RL0_PK(11) RL0_PK(12) RL0_PK(13) RL0_PK(14) RL0_PK(15) RL0_PK(16)
#undef RL0_PK
        default: return false;
    }
}

bool pack_usable(int d, int m) {
    switch (d) {
#define RL0_PF(D) \
    case D: return pack_fits<D>(m);
        RL0_PF(1) RL0_PF(2) RL0_PF(3) RL0_PF(4) RL0_PF(5) RL0_PF(6) RL0_PF(7) RL0_PF(8)
        RL0_PF(9) RL0_PF(10) RL0_PF(11) RL0_PF(12) RL0_PF(13) RL0_PF(14) RL0_PF(15) RL0_PF(16)
#undef RL0_PF
        default: return false;
    }
}

hipError_t launch_sweep(int d, const SweepArgs& a, hipStream_t s, const hipEvent_t* ev = nullptr) {
    switch (d) {
        case 1: return launch_sweep_d<1>(a, s, ev);
        case 2: return launch_sweep_d<2>(a, s, ev);
        case 3: return launch_sweep_d<3>(a, s, ev);
        case 4: return launch_sweep_d<4>(a, s, ev);
        case 5: return launch_sweep_d<5>(a, s, ev);
        case 6: return launch_sweep_d<6>(a, s, ev);
        case 7: return launch_sweep_d<7>(a, s, ev);
        case 8: return launch_sweep_d<8>(a, s, ev);
        case 9: return launch_sweep_d<9>(a, s, ev);
        case 10: return launch_sweep_d<10>(a, s, ev);
        case 11: return launch_sweep_d<11>(a, s, ev);
        case 12: return launch_sweep_d<12>(a, s, ev);
        case 13: return launch_sweep_d<13>(a, s, ev);
        case 14: return launch_sweep_d<14>(a, s, ev);
        case 15: return launch_sweep_d<15>(a, s, ev);
        case 16: return launch_sweep_d<16>(a, s, ev);
        default: return hipErrorInvalidValue;
    }
}

size_t al(size_t b) { return (b + 255) & ~size_t(255); }

}  // namespace

// ------------------------------------------------------------------ workspace

size_t workspace_bytes(int n, int m) {
    const size_t wm = (static_cast<size_t>(m) + 31) / 32, wn = (static_cast<size_t>(n) + 31) / 32;
    const size_t cand = static_cast<size_t>(sweep_grid(n)) * seg_capacity(n);
    (void)wn;
    const size_t bucket = m > kPreRows ? 2 * (al(8 * cand) + al(4 * cand)) : 0;
    return 4 * al(8ull * m) + 2 * al(4ull * m) + 2 * al(4 * wm + 16) + 2 * al(4 * ((m + 255) / 256) + 16) +
           6 * al(4 * cand) + al(4ull * n) +
           al(8ull * n) + 2 * al(4ull * m) + al(4ull * m) + al(4ull * n) + al(16ull * n) + al(sizeof(DevState)) + bucket;
}

void carve_workspace(void* base, int n, int m, Workspace* w) {
    const size_t wm = (static_cast<size_t>(m) + 31) / 32, wn = (static_cast<size_t>(n) + 31) / 32;
    const size_t cand = static_cast<size_t>(sweep_grid(n)) * seg_capacity(n);
    char* p = static_cast<char*>(base);
    auto take = [&](size_t bytes) { char* q = p; p += al(bytes); return q; };
    w->Sy = reinterpret_cast<long long*>(take(8ull * m));
    for (int b = 0; b < 2; ++b) w->S[b] = reinterpret_cast<long long*>(take(8ull * m));
    w->D = reinterpret_cast<long long*>(take(8ull * m));
    for (int b = 0; b < 2; ++b) w->r[b] = reinterpret_cast<float*>(take(4ull * m));
    for (int b = 0; b < 2; ++b) w->bm[b] = reinterpret_cast<uint32_t*>(take(4 * wm + 16));
    for (int b = 0; b < 2; ++b) w->bs[b] = reinterpret_cast<uint32_t*>(take(4 * ((static_cast<size_t>(m) + 255) / 256) + 16));
    (void)wn;
    for (int b = 0; b < 2; ++b) {
        w->cand_j[b] = reinterpret_cast<int*>(take(4 * cand));
        w->cand_x[b] = reinterpret_cast<float*>(take(4 * cand));
        w->cand_h[b] = reinterpret_cast<float*>(take(4 * cand));
    }
    w->seg_cap = seg_capacity(n);
    w->sweep_grid = sweep_grid(n);
    w->learned = reinterpret_cast<float*>(take(4ull * n));
    w->lcache = reinterpret_cast<float*>(take(8ull * n));
    for (int b = 0; b < 2; ++b) w->reval[b] = reinterpret_cast<float*>(take(4ull * m));
    w->ystage = reinterpret_cast<float*>(take(4ull * m));
    w->xstage = reinterpret_cast<float*>(take(4ull * n));
    w->Apk = reinterpret_cast<uint4*>(take(16ull * n));
    w->st = reinterpret_cast<DevState*>(take(sizeof(DevState)));
    for (int b = 0; b < 2; ++b) {
        w->bkey[b] = m > kPreRows ? reinterpret_cast<unsigned long long*>(take(8 * cand)) : nullptr;
        w->bx[b] = m > kPreRows ? reinterpret_cast<float*>(take(4 * cand)) : nullptr;
    }
}

// ------------------------------------------------------------------ launchers

hipError_t launch_validate(const int32_t* A, int n, int m, int d, int* err, hipStream_t s) {
    if (n > 0) k_validate<<<blocks(n, kStageBlock), kStageBlock, 0, s>>>(A, n, m, d, err);
    return hipGetLastError();
}

hipError_t launch_sketch(const int32_t* A, int n, int m, int d, const float* x, float* y,
                         long long* S, int* err, hipStream_t s) {
    k_zero_ll<<<blocks(m, 256), 256, 0, s>>>(S, m);
    if (n > 0) k_sketch_scatter<<<blocks(n, kStageBlock), kStageBlock, 0, s>>>(A, n, m, d, x, S, err);
    k_sketch_finish<<<blocks(m, 256), 256, 0, s>>>(S, y, m, err);
    return hipGetLastError();
}

hipError_t launch_clear_state(DevState* st, hipStream_t s) {
    k_prep_state<<<(kStateWords + 1023) / 1024, 256, 0, s>>>(st);
    return hipGetLastError();
}

hipError_t launch_zero_i32(int* p, long long count, hipStream_t s) {
    if (count > 0) k_zero_i32<<<blocks(count, 256), 256, 0, s>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_zero_f32(float* p, long long count, hipStream_t s) {
    if (count > 0) k_zero_f32<<<blocks(count, 256), 256, 0, s>>>(p, count);
    return hipGetLastError();
}

hipError_t launch_copy_f32(const float* src, float* dst, long long count, hipStream_t s) {
    if (count > 0) k_copy_f32<<<blocks(count, 256), 256, 0, s>>>(src, dst, count);
    return hipGetLastError();
}

hipError_t launch_prepare(const DecodeDims& dm, const int32_t* A, bool validate, const float* y,
                          const float* x_hat0, const Workspace& w, const IterParams& ip0, hipStream_t s,
                          float* x_zero) {
    const int slot = (ip0.it & 1) ^ 1;   // the slot iteration it0 reads as "previous"
    k_prep_state<<<(kStateWords + 1023) / 1024, 256, 0, s>>>(w.st);
    if (x_hat0) k_prep_support<<<blocks(dm.n, 256), 256, 0, s>>>(x_hat0, dm.n, w, slot);
    k_prep_rows<<<blocks(dm.m, 256), 256, 0, s>>>(y, w.Sy, w.S[0], w.D, dm.m, w.st);
    // the packing pass validates the columns and clears x_zero; without packing they
    // run on their own
    if (!launch_pack(dm.d, A, dm.n, dm.m, w.Apk, validate ? &w.st->err : nullptr, x_zero, s)) {
        if (validate) k_validate<<<blocks(dm.n, kStageBlock), kStageBlock, 0, s>>>(A, dm.n, dm.m, dm.d, &w.st->err);
        if (x_zero) k_zero_f32<<<blocks(dm.n, 256), 256, 0, s>>>(x_zero, dm.n);
    }
    if (x_hat0) k_prep_scatter<<<blocks(dm.n, 256), 256, 0, s>>>(A, dm.n, dm.d, x_hat0, w.S[0], w.st);
    const bool summary = ((dm.m + 31) / 32) > kBmLdsWords && ((dm.m + 255) / 256) <= kBmLdsWords;
    k_prep_rows2<<<kRowGrid, kRowBlock, 0, s>>>(w.S[0], w.r[0], w.bm[0],
                                                summary ? reinterpret_cast<uint8_t*>(w.bs[0]) : nullptr, dm.m,
                                                ip0.tau_bits, w.st, slot);
    k_prep_slot<<<1, 256, 0, s>>>(w.st, slot);
    return hipGetLastError();
}

hipError_t launch_iteration(const DecodeDims& dm, const int32_t* A, const Workspace& w,
                            const ScoreTables& tb, const IterParams& ip, const DebugOut& dbg,
                            hipStream_t s, const hipEvent_t* ev, const float* learned) {
    SweepArgs a;
    a.A = A;
    a.n = dm.n;
    a.m = dm.m;
    a.chunks = blocks(dm.n, kSweepChunk);
    a.bm_lds = ((dm.m + 31) / 32) <= kBmLdsWords ? 1 : 0;
    a.bs_lds = (!a.bm_lds && ((dm.m + 255) / 256) <= kBmLdsWords) ? 1 : 0;
    a.w = w;
    a.tb = tb;
    a.ip = ip;
    a.dbg = dbg;
    a.learned = learned;
    a.Apk = pack_usable(dm.d, dm.m) ? w.Apk : nullptr;
    hipError_t e = launch_sweep(dm.d, a, s, ev ? ev : nullptr);
    if (e != hipSuccess) return e;
    const int pre = dm.m > kPreRows ? 1 : 0;
    const FinishArgs fa{A, dm.d, dm.k, dm.m, w, ip.it, ip.tau_next, a.bs_lds, !a.bm_lds, pre, ip.log, ip.t, ip.wg_rev,
                        dm.n};
    if (pre) {
        e = launch_timed(k_hk_classify, kRowGrid, kRowBlock, s, ev ? ev + 2 : nullptr, fa);
        if (e != hipSuccess) return e;
    }
    return launch_timed(k_finish_rows, finish_grid(dm.m), kRowBlock, s, ev ? ev + 4 : nullptr, fa);
}

hipError_t launch_peek(const Workspace& w, const IterParams& ip, hipStream_t s) {
    k_peek<<<1, 256, 0, s>>>(w.st, ip.it, ip.n_iters, ip.tol_fx);
    return hipGetLastError();
}

hipError_t launch_adapt_sum(const Workspace& w, const ScoreTables& tb, int it, hipStream_t s) {
    k_adapt_sum<<<w.sweep_grid, 256, 0, s>>>(w, tb, it);
    return hipGetLastError();
}

hipError_t launch_rebuild_outer(const DecodeDims& dm, const Workspace& w, int buf, uint32_t tau, int it,
                                hipStream_t s) {
    const bool summary = ((dm.m + 31) / 32) > kBmLdsWords && ((dm.m + 255) / 256) <= kBmLdsWords;
    const bool counts = ((dm.m + 31) / 32) > kBmLdsWords;
    k_rebuild_outer<<<kRowGrid, kRowBlock, 0, s>>>(w.r[buf], w.bm[buf],
                                                  summary ? reinterpret_cast<uint8_t*>(w.bs[buf]) : nullptr, dm.m, tau,
                                                  counts ? w.st->flag_part[it & 1][buf] : nullptr);
    return hipGetLastError();
}

hipError_t launch_finish(const DecodeDims& dm, const Workspace& w, const IterParams& ip_last,
                         float* x_out, hipStream_t s, bool x_zeroed) {
    if (!x_out) {
        k_decide_only<<<1, 256, 0, s>>>(w.st, ip_last.it, ip_last.n_iters, ip_last.tol_fx, ip_last.log);
        return hipGetLastError();
    }
    if (!x_zeroed) k_zero_f32<<<blocks(dm.n, 256), 256, 0, s>>>(x_out, dm.n);
    k_copy_out<<<w.sweep_grid, 256, 0, s>>>(w, x_out, dm.n, ip_last.it, 0, 1, ip_last.n_iters, ip_last.tol_fx,
                                            ip_last.log);
    return hipGetLastError();
}

hipError_t launch_trial_out(const DecodeDims& dm, const Workspace& w, int it_end, float* x_trial,
                            hipStream_t s) {
    k_zero_f32<<<blocks(dm.n, 256), 256, 0, s>>>(x_trial, dm.n);
    k_copy_out<<<w.sweep_grid, 256, 0, s>>>(w, x_trial, dm.n, it_end, 1, 0, 0, 0.0, 0);
    return hipGetLastError();
}

}  // namespace rl0
