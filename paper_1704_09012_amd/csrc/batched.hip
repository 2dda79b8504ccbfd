// Persistent batched Robust-l0 decoder for gfx950.
//
// One launch decodes many independent instances.  Every workgroup repeatedly takes the
// next instance from a queue (the host orders it largest first) and runs Alg. 1 for that
// instance alone, so the only synchronisation is the workgroup barrier and the launch
// drains when the queue is empty.  Per iteration a workgroup
//   1. writes the outer-test bitmask |r_i| >= tau_it of its instance into LDS (ballot),
//      and r = fl32(S) beside S, which the sweep gathers (4 bytes a row instead of 8);
//   2. sweeps its columns in tiles (the next tile's indices load while the current one is
//      tested): a column whose rows hit the bitmask gathers its exact residuals and runs
//      the consensus test; an update goes to x' and to the change list;
//   3. applies H_k: when x' has more than k nonzeros, the k-th largest key by a radix
//      select over x', and the dropped columns join the change list;
//   4. adds the exact fixed-point residual change of every changed column with 64-bit
//      atomics, accumulating the change of ||r||_1 from the values the atomics return
//      (the per-row differences telescope, whatever the order of the atomics);
//   5. accepts (x_hat <- x') or undoes the residual change.
// The arithmetic is the single-decode kernels' (column_math.h), so every instance's
// result is bit-identical to rl0_decode's on the same input.
#include "batched.h"

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <utility>

#include "column_math.h"

#pragma clang fp contract(off)

namespace rl0 {

namespace {

// Checked builds (compiled with RL0_DEVICE_CHECKS=1 into the second copy of the library):
// BCHK(i, n) tests a data-dependent index (a row read from A_cols, a slot taken from an
// append counter, a column read back from a list or decoded from a key) against [0, n).
// Outside it, the source line of the first failed check is recorded in
// g_batched_check_line (read back by batched_check_read) and the index becomes 0, so that
// the access stays inside its buffer and the decode runs to its end.  In normal builds
// BCHK(i, n) is i.
#if RL0_DEVICE_CHECKS
__device__ unsigned g_batched_check_line;

template <class I>
__device__ __forceinline__ I bchk(I i, long long n, unsigned line) {
    const long long v = static_cast<long long>(i);
    if (v >= 0 && v < n) return i;
    atomicCAS(&g_batched_check_line, 0u, line);
    return static_cast<I>(0);
}
#define BCHK(i, n) bchk((i), static_cast<long long>(n), __LINE__)
#else
#define BCHK(i, n) (i)
#endif

constexpr int kBins = 2048;
constexpr int kTabStride = kTableStrideFloats;   // floats from the start of Tz to Te in LDS

template <int BLOCK>
struct BatchShared {
    unsigned hist[kBins];
    int queue[BLOCK * 5];      // queued columns: fewer than BLOCK carried over plus one tile
    unsigned scan[BLOCK / 64];
    long long red[BLOCK / 64];
    int idx, nq, nchg, nupd, nzd, nkeys, err, digit;
    int ninx;                  // the sweep's updated x'_j != 0 whose conversion rounds
    int nflag[2];              // rows flagged by the outer test, by iteration parity
    unsigned above, bucket;
};

// Sum over the workgroup, returned to every thread.
template <int BLOCK>
__device__ __forceinline__ long long wg_sum(long long v, long long* red) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    long long t = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / 64; ++w) t += red[w];
    __syncthreads();
    return t;
}

// The digit (among kBins, highest first) of the bucket holding the rem-th largest of the
// counted keys, the count above that bucket and the bucket's own count.  Needs
// 1 <= rem <= total count.
template <int BLOCK>
__device__ void wg_find_digit(const unsigned* hist, unsigned rem, BatchShared<BLOCK>& sh) {
    constexpr int B = kBins / BLOCK;
    const int tid = threadIdx.x;
    unsigned c = 0;
#pragma unroll
    for (int i = 0; i < B; ++i) c += hist[kBins - 1 - tid * B - i];
    unsigned incl = c;
    for (int off = 1; off < 64; off <<= 1) {
        const unsigned t = __shfl_up(incl, off);
        if ((tid & 63) >= off) incl += t;
    }
    if ((tid & 63) == 63) sh.scan[tid >> 6] = incl;
    __syncthreads();
    unsigned before = incl - c;
    for (int w = 0; w < (tid >> 6); ++w) before += sh.scan[w];
    if (before < rem && rem <= before + c) {
        unsigned acc = before;
        for (int i = 0; i < B; ++i) {
            const int dg = kBins - 1 - tid * B - i;
            const unsigned h = hist[dg];
            if (rem <= acc + h) {
                sh.digit = dg;
                sh.above = acc;
                sh.bucket = h;
                break;
            }
            acc += h;
        }
    }
    __syncthreads();
}

constexpr int kU = 8;   // loads in flight per thread in the streaming loops

// H_k's threshold: the k-th largest key (|x'_j| bits, then smaller j) among the nonzero
// entries of x', which number more than k.  One pass over x' writes the nonzero keys to
// the key buffer (and their top-digit histogram); five radix passes over that buffer
// follow (11, ..., 11, 8 bits), stopping once the bucket is exactly the rest of H_k.
// Returns the number of keys in the buffer through *nkeys.
template <int BLOCK>
__device__ unsigned long long wg_select_kth(const BatchProblem& P, BatchShared<BLOCK>& sh, int* nkeys) {
    const int tid = threadIdx.x;
    for (int b = tid; b < kBins; b += BLOCK) sh.hist[b] = 0u;
    if (tid == 0) sh.nkeys = 0;
    __syncthreads();
    for (int base = 0; base < P.n; base += BLOCK * kU) {
        float v[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int j = base + u * BLOCK + tid;
            v[u] = j < P.n ? P.xp[j] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const bool nz = v[u] != 0.0f;
            const unsigned long long key = nz ? hk_key(base + u * BLOCK + tid, v[u]) : 0ull;
            const int slot = wave_append(&sh.nkeys, nz);
            if (nz) P.keys[BCHK(slot, P.n)] = key;
            hist_add(sh.hist, static_cast<unsigned>(key >> 52), nz);
        }
    }
    __syncthreads();
    const int nk = sh.nkeys;
    *nkeys = nk;
    unsigned long long prefix = 0ull, pmask = 0ull;
    unsigned rem = static_cast<unsigned>(P.k);
    for (int pass = 0; pass < 6; ++pass) {
        const int sft = pass < 5 ? 52 - 11 * pass : 0;
        const unsigned dmask = pass < 5 ? 0x7FFu : 0xFFu;
        if (pass > 0) {
            for (int b = tid; b < kBins; b += BLOCK) sh.hist[b] = 0u;
            __syncthreads();
            for (int base = 0; base < nk; base += BLOCK * kU) {
                unsigned long long kv[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int e = base + u * BLOCK + tid;
                    kv[u] = e < nk ? P.keys[BCHK(e, P.n)] : 0ull;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u)
                    hist_add(sh.hist, static_cast<unsigned>((kv[u] >> sft) & dmask),
                             kv[u] != 0ull && (kv[u] & pmask) == prefix);
            }
            __syncthreads();
        }
        wg_find_digit<BLOCK>(sh.hist, rem, sh);
        prefix |= static_cast<unsigned long long>(sh.digit) << sft;
        pmask |= static_cast<unsigned long long>(dmask) << sft;
        rem -= sh.above;
        const bool exact = (rem == sh.bucket);
        __syncthreads();
        if (exact) break;
    }
    return prefix;
}

template <int D, int C>
__device__ __forceinline__ void load_tile(const int32_t* __restrict__ A, int n, int j0, int (&rows)[C][D]) {
    if (C == 4 && j0 + C <= n) {
        // C * D ints from a 16-byte aligned start (j0 is a multiple of 4)
        const int4* __restrict__ p4 = reinterpret_cast<const int4*>(A + static_cast<size_t>(j0) * D);
        int flat[C * D];
#pragma unroll
        for (int k = 0; k < D; ++k) {
            const int4 t = p4[k];
            flat[4 * k] = t.x;
            flat[4 * k + 1] = t.y;
            flat[4 * k + 2] = t.z;
            flat[4 * k + 3] = t.w;
        }
#pragma unroll
        for (int q = 0; q < C; ++q)
#pragma unroll
            for (int p = 0; p < D; ++p) rows[q][p] = flat[q * D + p];
    } else {
#pragma unroll
        for (int q = 0; q < C; ++q)
#pragma unroll
            for (int p = 0; p < D; ++p) rows[q][p] = (j0 + q < n) ? A[static_cast<size_t>(j0 + q) * D + p] : 0;
    }
}

// Step 2 for one instance: the column sweep, C consecutive columns per thread per tile.
// A tile's columns test their rows against the bitmask and those with a candidate row
// join an LDS queue; the next tile's indices load while the queue is checked.  Once the
// queue holds a column per thread (or the sweep ends) it is worked off one column per
// thread, so the consensus test is balanced and its gathers are paid once per BLOCK
// queued columns rather than once per tile.  In the dense mode (a quarter of the rows
// or more flagged, so that nearly every column has a candidate row) there is no queue:
// each thread gathers the residuals of all its tile's rows at once, while the next tile's
// indices load, and tests its own columns.  The two modes propose the same updates; only
// the order of the change list differs, which nothing after the sweep depends on.
template <int D, int BLOCK, int C>
__device__ void wg_sweep(const BatchProblem& P, const ScoreTables& tb, const uint32_t* bm, int it,
                         BatchShared<BLOCK>& sh, int j_begin, int j_end, int* nchg, int* chg, bool dense,
                         const float* rs) {
    const int tid = threadIdx.x;
    const int n = j_end;   // the columns [j_begin, j_end); j_begin is a multiple of 4
    constexpr int kTile = BLOCK * C;
    int cur[C][D];
    load_tile<D, C>(P.A, n, j_begin + tid * C, cur);
    int nupd = 0, nzd = 0, ninx = 0;
    if (dense) {
        for (int base = j_begin; base < n; base += kTile) {
            const int j0 = base + tid * C;
            float v[C][D];
            unsigned cm[C];
#pragma unroll
            for (int q = 0; q < C; ++q) {
                cm[q] = 0u;
#pragma unroll
                for (int p = 0; p < D; ++p) {
                    const int r = BCHK(cur[q][p], P.m);   // 0 past the end: a valid row, left unused
                    v[q][p] = rs[r];
                    cm[q] |= ((bm[r >> 5] >> (r & 31)) & 1u) << p;
                }
                if (j0 + q >= n) cm[q] = 0u;
            }
            if (base + kTile < n) load_tile<D, C>(P.A, n, base + kTile + tid * C, cur);
#pragma unroll
            for (int q = 0; q < C; ++q) {
                const int j = j0 + q;
                bool upd = false;
                if (cm[q]) {
                    float om = 0.0f;
                    upd = column_update_pairs<D>(v[q], cm[q], tb, P.alpha, P.l1_test, &om);
                    if (upd) {
                        const float xh = P.x[j];
                        const float xn = xh + om;
                        P.xp[j] = xn;
                        P.stamp[j] = it;
                        ++nupd;
                        nzd += (xn != 0.0f ? 1 : 0) - (xh != 0.0f ? 1 : 0);
                        ninx += (xn != 0.0f && fx_inexact(xn)) ? 1 : 0;
                    }
                }
                const int slot = wave_append(nchg, upd);
                if (upd) chg[BCHK(slot, P.n)] = j;
            }
        }
        if (nupd) atomicAdd(&sh.nupd, nupd);
        if (nzd) atomicAdd(&sh.nzd, nzd);
        if (ninx) atomicAdd(&sh.ninx, ninx);
        return;
    }
    for (int base = j_begin; base < n; base += kTile) {
        const int j0 = base + tid * C;
#pragma unroll
        for (int q = 0; q < C; ++q) {
            unsigned hit = 0u;
            if (j0 + q < n) {
#pragma unroll
                for (int p = 0; p < D; ++p) {
                    const int r = BCHK(cur[q][p], P.m);
                    hit |= (bm[r >> 5] >> (r & 31)) & 1u;
                }
            }
            const int slot = wave_append(&sh.nq, hit != 0u);
            if (hit) sh.queue[BCHK(slot, BLOCK * 5)] = j0 + q;
        }
        const bool more = base + kTile < n;
        if (more) load_tile<D, C>(P.A, n, base + kTile + tid * C, cur);
        __syncthreads();
        const int nq = sh.nq;
        __syncthreads();   // every thread has read nq before the next tile appends
        if (nq < BLOCK && more) continue;
        for (int e0 = 0; e0 < nq; e0 += BLOCK) {
            const int e = e0 + tid;
            bool upd = false;
            int j = 0;
            if (e < nq) {
                j = BCHK(sh.queue[BCHK(e, BLOCK * 5)], n);
                const int32_t* __restrict__ col = P.A + static_cast<size_t>(j) * D;
                int rows[D];
#pragma unroll
                for (int p = 0; p < D; ++p) rows[p] = BCHK(col[p], P.m);
                float v[D];
#pragma unroll
                for (int p = 0; p < D; ++p) v[p] = rs[rows[p]];
                unsigned cm = 0u;
#pragma unroll
                for (int p = 0; p < D; ++p) cm |= ((bm[rows[p] >> 5] >> (rows[p] & 31)) & 1u) << p;
                float om = 0.0f;
                upd = column_update<D>(v, cm, tb, P.alpha, P.l1_test, &om);
                if (upd) {
                    const float xh = P.x[j];
                    const float xn = xh + om;
                    P.xp[j] = xn;
                    P.stamp[j] = it;
                    ++nupd;
                    nzd += (xn != 0.0f ? 1 : 0) - (xh != 0.0f ? 1 : 0);
                    ninx += (xn != 0.0f && fx_inexact(xn)) ? 1 : 0;
                }
            }
            const int slot = wave_append(nchg, upd);
            if (upd) chg[BCHK(slot, P.n)] = j;
        }
        if (tid == 0) sh.nq = 0;
        __syncthreads();
    }
    if (nupd) atomicAdd(&sh.nupd, nupd);
    if (nzd) atomicAdd(&sh.nzd, nzd);
    if (ninx) atomicAdd(&sh.ninx, ninx);
}

// The fixed-point residual change of changing column j from xh to xn (d rows); with
// `track`, the change of ||r||_1 that the atomics' returned values give.
template <int D>
__device__ __forceinline__ long long apply_change(const BatchProblem& P, int j, float xh, float xn, bool track,
                                                  int* err) {
    const long long delta = (xh != 0.0f ? to_fx(xh, err) : 0) - (xn != 0.0f ? to_fx(xn, err) : 0);
    if (delta == 0) return 0;
    const int32_t* __restrict__ col = P.A + static_cast<size_t>(j) * D;
    int rows[D];
#pragma unroll
    for (int p = 0; p < D; ++p) rows[p] = BCHK(col[p], P.m);
    long long dl = 0;
#pragma unroll
    for (int p = 0; p < D; ++p) {
        unsigned long long* a = reinterpret_cast<unsigned long long*>(P.S + rows[p]);
        const long long old = static_cast<long long>(atomicAdd(a, static_cast<unsigned long long>(delta)));
        if (track) dl += l1_term(from_fx(old + delta)) - l1_term(from_fx(old));
    }
    return dl;
}

template <int D, int BLOCK>
__device__ void decode_instance(const BatchProblem P, BatchResult* R, float* dyn, float* rs, BatchShared<BLOCK>& sh) {
    const unsigned long long t_start = wall_clock64();
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m;
    float* Tz = dyn;
    float* Te = dyn + kTabStride;
    uint32_t* bm = reinterpret_cast<uint32_t*>(dyn + 2 * kTabStride);
    if (!P.exact)
        for (int i = tid; i <= kTableN; i += BLOCK) {
            Tz[i] = P.Tz[i];
            Te[i] = P.Te[i];
        }
    if (tid == 0) sh.err = 0;
    __syncthreads();
    const ScoreTables tb{Tz, Te, P.inv_h_z, P.inv_h_e, P.exact, P.e_zero_bits};

    // ---- ingest: the columns (rows in range, strictly ascending), y, the state
    if (P.validate) {
        for (int j = tid; j < n; j += BLOCK) {
            const int32_t* __restrict__ col = P.A + static_cast<size_t>(j) * D;
            int prev = -1;
            bool bad = false;
#pragma unroll
            for (int p = 0; p < D; ++p) {
                const int r = col[p];
                bad = bad || r <= prev || r >= m;
                prev = r;
            }
            if (bad) atomicOr(&sh.err, kErrIndex);
        }
        __syncthreads();
    }
    for (int j = tid; j < n; j += BLOCK) {
        P.x[j] = 0.0f;
        P.xp[j] = 0.0f;
        P.stamp[j] = -1;
    }
    long long l = 0, ny = 0;
    for (int base = 0; base < m; base += BLOCK * kU) {
        float yv[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = base + u * BLOCK + tid;
            yv[u] = i < m ? P.y[i] : 0.0f;
        }
#pragma unroll
        for (int u = 0; u < kU; ++u) {
            const int i = base + u * BLOCK + tid;
            if (i >= m) continue;
            long long sfx = 0;
            if (!isfinite(yv[u]))
                atomicOr(&sh.err, kErrNonFinite);
            else
                sfx = to_fx(yv[u], &sh.err);
            ny += fx_inexact(yv[u]) ? 1 : 0;
            P.S[i] = sfx;
            l += l1_term(from_fx(sfx));
        }
    }
    if (tid == 0) {
        sh.nflag[0] = 0;
        sh.nflag[1] = 0;
    }
    long long L_hat = wg_sum<BLOCK>(l, sh.red);
    const int inexact_y = static_cast<int>(wg_sum<BLOCK>(ny, sh.red));

    int iters = 0, accepted = 0, updates = 0, supp = 0, inexact_x = 0;
    const int words = (m + 31) >> 5;
    for (int it = 0;; ++it) {
        if (sh.err != 0 || static_cast<double>(L_hat) <= P.tol_fx || it >= P.n_iters) break;
        // ---- 1. outer-test bitmask of this iteration's threshold
        const uint32_t tau = P.tau[it];
        int flagged = 0;
        for (int base = 0; base < words * 32; base += BLOCK * kU) {
            long long sv[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = base + u * BLOCK + tid;
                sv[u] = i < m ? P.S[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = base + u * BLOCK + tid;
                const float rv = from_fx(sv[u]);
                if (i < m) rs[i] = rv;   // (global: every member of a group writes the same values)
                const bool pred = i < m && abs_bits(rv) >= tau;
                const unsigned long long b = __ballot(pred);
                if ((tid & 63) == 0) {
                    const int w = i >> 5;
                    if (w < words) bm[w] = static_cast<uint32_t>(b);
                    if (w + 1 < words) bm[w + 1] = static_cast<uint32_t>(b >> 32);
                    flagged += __popcll(b);
                }
            }
        }
        if (flagged) atomicAdd(&sh.nflag[it & 1], flagged);
        if (tid == 0) {
            sh.nq = 0;
            sh.nchg = 0;
            sh.nupd = 0;
            sh.nzd = 0;
            sh.ninx = 0;
            sh.nflag[(it & 1) ^ 1] = 0;   // the next iteration's count
        }
        __syncthreads();
        const bool dense = 4ll * sh.nflag[it & 1] >= static_cast<long long>(m);
        // ---- 2. sweep (with this iteration's quantised-score thresholds)
        ScoreTables tbi = tb;
        if (P.quant) {
            tbi.quant = 1;
            tbi.qe_bits = P.qe[it];
            tbi.qz_bits = P.qz[it];
        }
        if (P.cols == 1)
            wg_sweep<D, BLOCK, 1>(P, tbi, bm, it, sh, 0, n, &sh.nchg, P.chg, dense, rs);
        else if (P.cols == 2)
            wg_sweep<D, BLOCK, 2>(P, tbi, bm, it, sh, 0, n, &sh.nchg, P.chg, dense, rs);
        else
            wg_sweep<D, BLOCK, 4>(P, tbi, bm, it, sh, 0, n, &sh.nchg, P.chg, dense, rs);
        __syncthreads();
        updates += sh.nupd;
        inexact_x += sh.ninx;
        // ---- 3. H_k
        if (supp + sh.nzd > P.k) {
            int nk = 0;
            const unsigned long long kth = wg_select_kth<BLOCK>(P, sh, &nk);
            // the dropped columns: keys below the threshold
            for (int e0 = 0; e0 < nk; e0 += BLOCK) {
                const int e = e0 + tid;
                bool add = false;
                int j = 0;
                if (e < nk) {
                    const unsigned long long key = P.keys[BCHK(e, P.n)];
                    if (key < kth) {
                        j = BCHK(static_cast<int>(0xFFFFFFFFu - static_cast<unsigned>(key & 0xFFFFFFFFull)), P.n);
                        P.xp[j] = 0.0f;
                        add = P.stamp[j] != it;
                        if (add) P.stamp[j] = it;
                    }
                }
                const int slot = wave_append(&sh.nchg, add);
                if (add) P.chg[BCHK(slot, P.n)] = j;
            }
            __syncthreads();
        }
        // ---- 4. exact residual change and ||r||_1 of the trial iterate
        const int nchg = sh.nchg;
        long long dl = 0, dsupp = 0;
        for (int base = 0; base < nchg; base += BLOCK * 4) {
            int jj[4];
            float xh[4], xn[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int c = base + u * BLOCK + tid;
                jj[u] = c < nchg ? BCHK(P.chg[BCHK(c, P.n)], P.n) : -1;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                xh[u] = jj[u] >= 0 ? P.x[jj[u]] : 0.0f;
                xn[u] = jj[u] >= 0 ? P.xp[jj[u]] : 0.0f;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (jj[u] < 0 || xh[u] == xn[u]) continue;
                dsupp += (xn[u] != 0.0f ? 1 : 0) - (xh[u] != 0.0f ? 1 : 0);
                dl += apply_change<D>(P, jj[u], xh[u], xn[u], true, &sh.err);
            }
        }
        const long long Lt = L_hat + wg_sum<BLOCK>(dl, sh.red);
        const long long ds = wg_sum<BLOCK>(dsupp, sh.red);
        // ---- 5. accept or undo
        const bool acc = (Lt < L_hat) && (sh.err == 0);
        ++iters;
        if (acc) {
            for (int c = tid; c < nchg; c += BLOCK) {
                const int j = BCHK(P.chg[BCHK(c, P.n)], P.n);
                P.x[j] = P.xp[j];
            }
            L_hat = Lt;
            supp += static_cast<int>(ds);
            ++accepted;
        } else {
            for (int c = tid; c < nchg; c += BLOCK) {
                const int j = BCHK(P.chg[BCHK(c, P.n)], P.n);
                const float xh = P.x[j], xn = P.xp[j];
                if (xh == xn) continue;
                P.xp[j] = xh;
                apply_change<D>(P, j, xn, xh, false, &sh.err);
            }
        }
        __syncthreads();
    }
    if (tid == 0) {
        R->L_hat = L_hat;
        R->iterations = iters;
        R->accepted = accepted;
        R->updates_total = updates;
        R->inexact_y = inexact_y;
        R->inexact_x = inexact_x;
        R->err = sh.err;
        R->t_start = t_start;
        R->t_end = wall_clock64();
    }
    __syncthreads();
}

// ---------------------------------------------------------------- groups of workgroups
//
// A large instance is decoded by G workgroups together.  Member p of the group sweeps the
// p-th slice of the columns and takes the p-th slice of each list (dropped keys, changed
// columns); everything the members need from each other goes through global memory (x',
// the change and key lists, S) and the group's BatchCtl, separated by group barriers.
// Every member builds the whole outer-test bitmask in its own LDS and runs H_k's radix
// passes over the whole key list itself, so those need no barrier and every member
// reaches the same threshold.  Sums are exact integers, so the result is the same bits as
// a decode by one workgroup whatever the members' order.

// Wall-clock ticks (100 MHz) a member waits at a group barrier before it gives up.  The
// other members of a group take their tickets as soon as a workgroup is free, and the
// host queues groups first, so a healthy barrier completes in microseconds.
constexpr unsigned long long kGroupWaitTicks = 500000000ull;   // 5 s

// Barrier of the group's G members (the `count`-th one of this decode).  Returns false when
// a member's wait timed out; then every member returns from the instance.
template <int BLOCK>
__device__ bool group_barrier(BatchCtl* c, int G, unsigned count, BatchShared<BLOCK>& sh) {
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();   // this workgroup's writes, before its arrival
        atomicAdd(&c->bar, 1u);
        const unsigned target = count * static_cast<unsigned>(G);
        const unsigned long long deadline = wall_clock64() + kGroupWaitTicks;
        int ok = 1;
        for (;;) {
            if (__hip_atomic_load(&c->bar, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= target) break;
            if (__hip_atomic_load(&c->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                ok = 0;
                break;
            }
            if (wall_clock64() > deadline) {
                __hip_atomic_store(&c->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                atomicOr(&c->err, kErrTimeout);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        __threadfence();   // the other members' writes, after the wait
        sh.digit = ok;
    }
    __syncthreads();
    const bool ok = sh.digit != 0;
    __syncthreads();
    return ok;
}

// A member left the instance after a timed-out wait: its result says so (every member
// that leaves writes the same).
__device__ __forceinline__ void group_failed(BatchResult* R) {
    if (threadIdx.x == 0) {
        R->L_hat = 0;
        R->iterations = 0;
        R->accepted = 0;
        R->updates_total = 0;
        R->inexact_y = 0;
        R->inexact_x = 0;
        R->err = kErrTimeout;
    }
}

// [lo, hi) of member p of G over count items, in multiples of `align`.
__device__ __forceinline__ void member_slice(int count, int p, int G, int align, int* lo, int* hi) {
    const int units = (count + align - 1) / align;
    const int per = (units + G - 1) / G;
    *lo = min(count, p * per * align);
    *hi = min(count, (p + 1) * per * align);
}

template <int D, int BLOCK>
__device__ __noinline__ void decode_instance_group(const BatchProblem P, int part, BatchResult* R, float* dyn, float* rs,
                                      BatchShared<BLOCK>& sh) {
    const unsigned long long t_start = wall_clock64();
    const int tid = threadIdx.x;
    const int n = P.n, m = P.m, G = P.group;
    BatchCtl* ctl = P.ctl;
    float* Tz = dyn;
    float* Te = dyn + kTabStride;
    uint32_t* bm = reinterpret_cast<uint32_t*>(dyn + 2 * kTabStride);
    if (!P.exact)
        for (int i = tid; i <= kTableN; i += BLOCK) {
            Tz[i] = P.Tz[i];
            Te[i] = P.Te[i];
        }
    if (tid == 0) sh.err = 0;
    __syncthreads();
    const ScoreTables tb{Tz, Te, P.inv_h_z, P.inv_h_e, P.exact, P.e_zero_bits};
    unsigned nbar = 0;
    int c_lo, c_hi;                                  // this member's columns
    member_slice(n, part, G, 64, &c_lo, &c_hi);
    int r_lo, r_hi;                                  // and rows
    member_slice(m, part, G, 64, &r_lo, &r_hi);

    // ---- ingest, each member on its slices
    if (P.validate) {
        for (int j = c_lo + tid; j < c_hi; j += BLOCK) {
            const int32_t* __restrict__ col = P.A + static_cast<size_t>(j) * D;
            int prev = -1;
            bool bad = false;
#pragma unroll
            for (int p = 0; p < D; ++p) {
                const int r = col[p];
                bad = bad || r <= prev || r >= m;
                prev = r;
            }
            if (bad) atomicOr(&sh.err, kErrIndex);
        }
    }
    for (int j = c_lo + tid; j < c_hi; j += BLOCK) {
        P.x[j] = 0.0f;
        P.xp[j] = 0.0f;
        P.stamp[j] = -1;
    }
    long long l = 0, ny = 0;
    for (int i = r_lo + tid; i < r_hi; i += BLOCK) {
        const float yv = P.y[i];
        long long sfx = 0;
        if (!isfinite(yv))
            atomicOr(&sh.err, kErrNonFinite);
        else
            sfx = to_fx(yv, &sh.err);
        ny += fx_inexact(yv) ? 1 : 0;
        P.S[i] = sfx;
        l += l1_term(from_fx(sfx));
    }
    if (tid == 0) {
        sh.nflag[0] = 0;
        sh.nflag[1] = 0;
    }
    l = wg_sum<BLOCK>(l, sh.red);
    ny = wg_sum<BLOCK>(ny, sh.red);
    if (tid == 0) {
        if (l) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->L0), static_cast<unsigned long long>(l));
        if (ny) atomicAdd(&ctl->inexact_y, static_cast<int>(ny));
        if (sh.err) atomicOr(&ctl->err, sh.err);
    }
    if (!group_barrier<BLOCK>(ctl, G, ++nbar, sh)) return group_failed(R);
    long long L_hat = __hip_atomic_load(&ctl->L0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    int iters = 0, accepted = 0, updates = 0, supp = 0;
    const int words = (m + 31) >> 5;
    for (int it = 0;; ++it) {
        const int par = it & 1, nxt = par ^ 1;
        const int err = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (err != 0 || static_cast<double>(L_hat) <= P.tol_fx || it >= P.n_iters) break;
        // ---- 1. the whole outer-test bitmask, in this member's LDS
        const uint32_t tau = P.tau[it];
        int flagged = 0;
        for (int base = 0; base < words * 32; base += BLOCK * kU) {
            long long sv[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = base + u * BLOCK + tid;
                sv[u] = i < m ? P.S[i] : 0;
            }
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                const int i = base + u * BLOCK + tid;
                const float rv = from_fx(sv[u]);
                if (i < m) rs[i] = rv;   // (global: every member of a group writes the same values)
                const bool pred = i < m && abs_bits(rv) >= tau;
                const unsigned long long b = __ballot(pred);
                if ((tid & 63) == 0) {
                    const int w = i >> 5;
                    if (w < words) bm[w] = static_cast<uint32_t>(b);
                    if (w + 1 < words) bm[w + 1] = static_cast<uint32_t>(b >> 32);
                    flagged += __popcll(b);
                }
            }
        }
        if (flagged) atomicAdd(&sh.nflag[it & 1], flagged);
        if (tid == 0) {
            sh.nq = 0;
            sh.nupd = 0;
            sh.nzd = 0;
            sh.ninx = 0;
            sh.nflag[(it & 1) ^ 1] = 0;   // the next iteration's count
        }
        __syncthreads();
        const bool dense = 4ll * sh.nflag[it & 1] >= static_cast<long long>(m);
        // the change list of this iteration: one of two, by parity, since a member may start
        // the next iteration while another still reads this one's list (after an accept)
        int* __restrict__ chg = par ? P.chg2 : P.chg;
        // ---- 2. sweep of this member's columns
        ScoreTables tbi = tb;
        if (P.quant) {
            tbi.quant = 1;
            tbi.qe_bits = P.qe[it];
            tbi.qz_bits = P.qz[it];
        }
        if (P.cols == 1)
            wg_sweep<D, BLOCK, 1>(P, tbi, bm, it, sh, c_lo, c_hi, &ctl->nchg[par], chg, dense, rs);
        else if (P.cols == 2)
            wg_sweep<D, BLOCK, 2>(P, tbi, bm, it, sh, c_lo, c_hi, &ctl->nchg[par], chg, dense, rs);
        else
            wg_sweep<D, BLOCK, 4>(P, tbi, bm, it, sh, c_lo, c_hi, &ctl->nchg[par], chg, dense, rs);
        __syncthreads();
        if (tid == 0) {
            if (sh.nupd) atomicAdd(&ctl->nupd[par], sh.nupd);
            if (sh.nzd) atomicAdd(&ctl->nzd[par], sh.nzd);
            if (sh.ninx) atomicAdd(&ctl->inexact_x, sh.ninx);   // a running total: read at the end
        }
        if (!group_barrier<BLOCK>(ctl, G, ++nbar, sh)) return group_failed(R);
        // the next iteration's counters: every member has passed the previous iteration's
        // last reads of them (they arrived here after it); the next barrier publishes
        if (part == 0 && tid == 0) {
            ctl->nchg[nxt] = 0;
            ctl->nupd[nxt] = 0;
            ctl->nzd[nxt] = 0;
            ctl->nkeys[nxt] = 0;
            ctl->dl[nxt] = 0;
            ctl->dsupp[nxt] = 0;
        }
        updates += __hip_atomic_load(&ctl->nupd[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int nzd = __hip_atomic_load(&ctl->nzd[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // ---- 3. H_k
        if (supp + nzd > P.k) {
            // the nonzero keys of this member's columns join the key list
            for (int base = c_lo; base < c_hi; base += BLOCK * kU) {
                float v[kU];
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const int j = base + u * BLOCK + tid;
                    v[u] = j < c_hi ? P.xp[j] : 0.0f;
                }
#pragma unroll
                for (int u = 0; u < kU; ++u) {
                    const bool nz = v[u] != 0.0f;
                    const int slot = wave_append(&ctl->nkeys[par], nz);
                    if (nz) P.keys[BCHK(slot, P.n)] = hk_key(base + u * BLOCK + tid, v[u]);
                }
            }
            if (!group_barrier<BLOCK>(ctl, G, ++nbar, sh)) return group_failed(R);
            const int nk = __hip_atomic_load(&ctl->nkeys[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // every member selects the k-th key over the whole list (radix passes in LDS)
            unsigned long long prefix = 0ull, pmask = 0ull;
            unsigned rem = static_cast<unsigned>(P.k);
            for (int pass = 0; pass < 6; ++pass) {
                const int sft = pass < 5 ? 52 - 11 * pass : 0;
                const unsigned dmask = pass < 5 ? 0x7FFu : 0xFFu;
                for (int b = tid; b < kBins; b += BLOCK) sh.hist[b] = 0u;
                __syncthreads();
                for (int base = 0; base < nk; base += BLOCK * kU) {
                    unsigned long long kv[kU];
#pragma unroll
                    for (int u = 0; u < kU; ++u) {
                        const int e = base + u * BLOCK + tid;
                        kv[u] = e < nk ? P.keys[BCHK(e, P.n)] : 0ull;
                    }
#pragma unroll
                    for (int u = 0; u < kU; ++u)
                        hist_add(sh.hist, static_cast<unsigned>((kv[u] >> sft) & dmask),
                                 kv[u] != 0ull && (kv[u] & pmask) == prefix);
                }
                __syncthreads();
                wg_find_digit<BLOCK>(sh.hist, rem, sh);
                prefix |= static_cast<unsigned long long>(sh.digit) << sft;
                pmask |= static_cast<unsigned long long>(dmask) << sft;
                rem -= sh.above;
                const bool exact = (rem == sh.bucket);
                __syncthreads();
                if (exact) break;
            }
            const unsigned long long kth = prefix;
            // the dropped columns of this member's slice of the key list
            int k_lo, k_hi;
            member_slice(nk, part, G, 1, &k_lo, &k_hi);
            for (int e0 = k_lo; e0 < k_hi; e0 += BLOCK) {
                const int e = e0 + tid;
                bool add = false;
                int j = 0;
                if (e < k_hi) {
                    const unsigned long long key = P.keys[BCHK(e, P.n)];
                    if (key < kth) {
                        j = BCHK(static_cast<int>(0xFFFFFFFFu - static_cast<unsigned>(key & 0xFFFFFFFFull)), P.n);
                        P.xp[j] = 0.0f;
                        add = P.stamp[j] != it;
                        if (add) P.stamp[j] = it;
                    }
                }
                const int slot = wave_append(&ctl->nchg[par], add);
                if (add) chg[BCHK(slot, P.n)] = j;
            }
            if (!group_barrier<BLOCK>(ctl, G, ++nbar, sh)) return group_failed(R);
        }
        // ---- 4. residual change of this member's slice of the change list
        const int nchg = __hip_atomic_load(&ctl->nchg[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        int h_lo, h_hi;
        member_slice(nchg, part, G, 1, &h_lo, &h_hi);
        long long dl = 0, dsupp = 0;
        for (int c = h_lo + tid; c < h_hi; c += BLOCK) {
            const int j = BCHK(chg[BCHK(c, P.n)], P.n);
            const float xh = P.x[j], xn = P.xp[j];
            if (xh == xn) continue;
            dsupp += (xn != 0.0f ? 1 : 0) - (xh != 0.0f ? 1 : 0);
            dl += apply_change<D>(P, j, xh, xn, true, &sh.err);
        }
        dl = wg_sum<BLOCK>(dl, sh.red);
        dsupp = wg_sum<BLOCK>(dsupp, sh.red);
        if (tid == 0) {
            if (dl) atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->dl[par]), static_cast<unsigned long long>(dl));
            if (dsupp)
                atomicAdd(reinterpret_cast<unsigned long long*>(&ctl->dsupp[par]), static_cast<unsigned long long>(dsupp));
            if (sh.err) atomicOr(&ctl->err, sh.err);
        }
        if (!group_barrier<BLOCK>(ctl, G, ++nbar, sh)) return group_failed(R);
        // ---- 5. accept or undo, each member on its slice of the change list
        const long long Lt = L_hat + __hip_atomic_load(&ctl->dl[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const long long ds = __hip_atomic_load(&ctl->dsupp[par], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int err2 = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const bool acc = (Lt < L_hat) && (err2 == 0);
        ++iters;
        if (acc) {
            // each member takes over x' on its own columns: the next iteration reads x
            // and x' there before any barrier, so no barrier is needed here (S is final
            // since the barrier above; the owners' writes are published by the next one)
            for (int c = tid; c < nchg; c += BLOCK) {
                const int j = BCHK(chg[BCHK(c, P.n)], P.n);
                if (j >= c_lo && j < c_hi) P.x[j] = P.xp[j];
            }
            L_hat = Lt;
            supp += static_cast<int>(ds);
            ++accepted;
        } else {
            for (int c = h_lo + tid; c < h_hi; c += BLOCK) {
                const int j = BCHK(chg[BCHK(c, P.n)], P.n);
                const float xh = P.x[j], xn = P.xp[j];
                if (xh == xn) continue;
                P.xp[j] = xh;
                apply_change<D>(P, j, xn, xh, false, &sh.err);
            }
            if (tid == 0 && sh.err) atomicOr(&ctl->err, sh.err);
            // the undo changed S, which every member's next bitmask reads
            if (!group_barrier<BLOCK>(ctl, G, ++nbar, sh)) return group_failed(R);
        }
        __syncthreads();
    }
    if (part == 0 && tid == 0) {
        R->L_hat = L_hat;
        R->iterations = iters;
        R->accepted = accepted;
        R->updates_total = updates;
        R->inexact_y = __hip_atomic_load(&ctl->inexact_y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        R->inexact_x = __hip_atomic_load(&ctl->inexact_x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        R->err = __hip_atomic_load(&ctl->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        R->t_start = t_start;
        R->t_end = wall_clock64();
    }
    __syncthreads();
}

template <int D, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_decode_batched(const BatchProblem* __restrict__ probs,
                                                          const int* __restrict__ order, int count,
                                                          BatchResult* __restrict__ res, int* __restrict__ counter,
                                                          int r_off, int r_rows) {
    extern __shared__ float dyn[];
    __shared__ BatchShared<BLOCK> sh;
    for (;;) {
        if (threadIdx.x == 0) sh.idx = atomicAdd(counter, 1);
        __syncthreads();
        // the instance index is uniform over the workgroup: keep it (and so the
        // descriptor loads) scalar
        const int q = __builtin_amdgcn_readfirstlane(sh.idx);
        __syncthreads();
        if (q >= count) return;
        const int ticket = __builtin_amdgcn_readfirstlane(order[q]);
        const int pi = ticket / kTicketParts, part = ticket % kTicketParts;
        const BatchProblem P = probs[pi];
        // the residual snapshot in LDS when the instance's rows fit the region
        float* rs = P.m <= r_rows ? dyn + r_off : P.r;
        if (P.group > 1)
            decode_instance_group<D, BLOCK>(P, part, res + pi, dyn, rs, sh);
        else
            decode_instance<D, BLOCK>(P, res + pi, dyn, rs, sh);
    }
}

__global__ void k_zero_counter(int* counter) { *counter = 0; }

__global__ void k_zero_words(int* __restrict__ w, long long count) {
    const long long i = static_cast<long long>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) w[i] = 0;
}

template <int D, int BLOCK>
hipError_t launch_db(const BatchLaunch& L, int grid, size_t lds, const BatchProblem* probs, const int* order,
                     int count, BatchResult* res, int* counter, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    if (e0) {
        hipExtLaunchKernelGGL(k_decode_batched<D, BLOCK>, dim3(grid), dim3(BLOCK), static_cast<uint32_t>(lds), s,
                              e0, e1, 0, probs, order, count, res, counter, L.r_off, L.r_rows);
    } else {
        k_decode_batched<D, BLOCK><<<grid, BLOCK, lds, s>>>(probs, order, count, res, counter, L.r_off, L.r_rows);
    }
    return hipGetLastError();
}

constexpr size_t kCuLds = 160 * 1024;   // LDS of one gfx950 compute unit

template <int D, int BLOCK>
size_t static_lds_db() {
    hipFuncAttributes a{};
    if (hipFuncGetAttributes(&a, reinterpret_cast<const void*>(&k_decode_batched<D, BLOCK>)) != hipSuccess) return 0;
    return a.sharedSizeBytes;
}

template <int D, int BLOCK>
hipError_t set_lds_limit() {
    const size_t st = static_lds_db<D, BLOCK>();
    if (st == 0 || st >= kCuLds) return hipErrorInvalidValue;
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_decode_batched<D, BLOCK>),
                               hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kCuLds - st));
}

template <int D>
hipError_t set_lds_limits_d() {
    hipError_t e = set_lds_limit<D, 256>();
    if (e == hipSuccess) e = set_lds_limit<D, 512>();
    if (e == hipSuccess) e = set_lds_limit<D, 1024>();
    return e;
}

template <int... Ds>
hipError_t set_lds_limits_all(std::integer_sequence<int, Ds...>) {
    hipError_t e = hipSuccess;
    ((e = (e == hipSuccess ? set_lds_limits_d<Ds + 1>() : e)), ...);
    return e;
}

template <int D, int BLOCK>
int max_resident_db(size_t lds) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_decode_batched<D, BLOCK>, BLOCK, lds) != hipSuccess)
        return 0;
    return nb;
}

template <int D>
int max_resident_d(int block, size_t lds) {
    switch (block) {
        case 256: return max_resident_db<D, 256>(lds);
        case 512: return max_resident_db<D, 512>(lds);
        case 1024: return max_resident_db<D, 1024>(lds);
        default: return 0;
    }
}

template <int... Ds>
int max_resident_any(int d, int block, size_t lds, std::integer_sequence<int, Ds...>) {
    int r = 0;
    ((r = (d == Ds + 1 ? max_resident_d<Ds + 1>(block, lds) : r)), ...);
    return r;
}

template <int D>
hipError_t launch_d(const BatchLaunch& L, int grid, size_t lds, const BatchProblem* probs, const int* order,
                    int count, BatchResult* res, int* counter, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    switch (L.block) {
        case 256: return launch_db<D, 256>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 512: return launch_db<D, 512>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 1024: return launch_db<D, 1024>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

template <int D>
size_t static_lds_d(int block) {
    switch (block) {
        case 256: return static_lds_db<D, 256>();
        case 512: return static_lds_db<D, 512>();
        case 1024: return static_lds_db<D, 1024>();
        default: return 0;
    }
}

template <int... Ds>
size_t static_lds_any(int d, int block, std::integer_sequence<int, Ds...>) {
    size_t r = 0;
    ((r = (d == Ds + 1 ? static_lds_d<Ds + 1>(block) : r)), ...);
    return r;
}

}  // namespace

hipError_t batched_check_read(int* line, hipStream_t s) {
#if RL0_DEVICE_CHECKS
    unsigned v = 0u;
    hipError_t e =
        hipMemcpyFromSymbolAsync(&v, HIP_SYMBOL(g_batched_check_line), sizeof(v), 0, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && v != 0u) {
        const unsigned zero = 0u;
        e = hipMemcpyToSymbolAsync(HIP_SYMBOL(g_batched_check_line), &zero, sizeof(zero), 0, hipMemcpyHostToDevice, s);
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

hipError_t batched_set_lds_limits() {
    return set_lds_limits_all(std::make_integer_sequence<int, kMaxD>{});
}

size_t batched_static_lds(int d, int block) {
    return static_lds_any(d, block, std::make_integer_sequence<int, kMaxD>{});
}

int batched_max_resident(int d, int block, size_t lds_bytes) {
    return max_resident_any(d, block, lds_bytes, std::make_integer_sequence<int, kMaxD>{});
}

size_t batched_lds_bytes(int max_m) {
    const size_t words = (static_cast<size_t>(max_m) + 31) / 32;
    return (2 * static_cast<size_t>(kTabStride)) * sizeof(float) + 4 * words;
}

hipError_t launch_zero_words(int* words, long long count, hipStream_t s) {
    if (count > 0) k_zero_words<<<static_cast<int>((count + 255) / 256), 256, 0, s>>>(words, count);
    return hipGetLastError();
}

hipError_t launch_batched(int d, const BatchLaunch& L, int grid, size_t lds, const BatchProblem* probs,
                          const int* order, int count, BatchResult* res, int* counter, hipStream_t s,
                          hipEvent_t e0, hipEvent_t e1) {
    k_zero_counter<<<1, 1, 0, s>>>(counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (d) {
        case 1: return launch_d<1>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 2: return launch_d<2>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 3: return launch_d<3>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 4: return launch_d<4>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 5: return launch_d<5>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 6: return launch_d<6>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 7: return launch_d<7>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 8: return launch_d<8>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 9: return launch_d<9>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 10: return launch_d<10>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 11: return launch_d<11>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 12: return launch_d<12>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 13: return launch_d<13>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 14: return launch_d<14>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 15: return launch_d<15>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        case 16: return launch_d<16>(L, grid, lds, probs, order, count, res, counter, s, e0, e1);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace rl0
