// C-ABI of librl0 (declared in include/rl0.h): argument checks, the cached constants
// and working memory, and the host-side order of kernel launches.
#include "../../include/rl0.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "constants.h"
#include "kernels.h"

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
    g_last_error = msg;
    return code;
}

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t e_ = (expr);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(RL0_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));  \
    } while (0)

std::mutex g_mu;

// ---------------------------------------------------------------- sweep timing

struct SweepProfile {
    bool enabled = false;
    std::vector<hipEvent_t> pool;   // per iteration: start and end of the sweep, select, finish
    double total_ms[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // all launched, then executed
    long long launches = 0, executed = 0;
};
SweepProfile g_prof;

hipEvent_t* profile_events(int it) {
    if (!g_prof.enabled) return nullptr;
    const size_t need = 6 * static_cast<size_t>(it + 1);
    while (g_prof.pool.size() < need) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        g_prof.pool.push_back(e);
    }
    return &g_prof.pool[6 * it];
}

// after a synchronised decode: add the kernels of the launched iterations (the first
// `executed` of which ran before the stopping condition)
void profile_collect(int launched, int executed) {
    if (!g_prof.enabled) return;
    for (int it = 0; it < launched && 6 * static_cast<size_t>(it) + 5 < g_prof.pool.size(); ++it) {
        float ms[3] = {0.0f, 0.0f, 0.0f};
        bool ok = true;
        for (int k = 0; k < 3; ++k)
            ok = ok && hipEventElapsedTime(&ms[k], g_prof.pool[6 * it + 2 * k], g_prof.pool[6 * it + 2 * k + 1]) == hipSuccess;
        if (!ok) continue;
        for (int k = 0; k < 3; ++k) g_prof.total_ms[k] += ms[k];
        g_prof.launches += 1;
        if (it < executed) {
            for (int k = 0; k < 3; ++k) g_prof.total_ms[3 + k] += ms[k];
            g_prof.executed += 1;
        }
    }
}

// ---------------------------------------------------------------- constants cache

struct DeviceConstants {
    rl0::HostConstants hc;
    float* d_tables = nullptr;  // table_z then table_e, kTableN + 1 each
};

using ConstKey = std::tuple<int, int, int, int, int, uint32_t, uint32_t, double, int, int>;
std::map<ConstKey, std::unique_ptr<DeviceConstants>> g_consts;

uint32_t fbits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

// Looks up (or builds and uploads) the constants of a problem; the device copy is
// written with a blocking copy, so it is ready before any later launch.
int get_constants(const rl0::Problem& pr, int device, DeviceConstants** out) {
    ConstKey key{device, pr.n, pr.m, pr.d, pr.k, fbits(static_cast<float>(pr.sigma)),
                 fbits(static_cast<float>(pr.sigma_s)), pr.c, pr.ell, pr.max_iters};
    auto it = g_consts.find(key);
    if (it != g_consts.end()) {
        *out = it->second.get();
        return RL0_OK;
    }
    auto dc = std::make_unique<DeviceConstants>();
    rl0::compute_constants(pr, &dc->hc);
    const size_t bytes = 2 * rl0::kTableStrideFloats * sizeof(float);
    if (hipMalloc(&dc->d_tables, bytes) != hipSuccess) return fail(RL0_ENOMEM, "hipMalloc(tables)");
    HIP_TRY(hipMemcpy(dc->d_tables, dc->hc.table_z, (rl0::kTableN + 1) * sizeof(float), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(dc->d_tables + rl0::kTableStrideFloats, dc->hc.table_e, (rl0::kTableN + 1) * sizeof(float),
                      hipMemcpyHostToDevice));
    *out = dc.get();
    g_consts.emplace(key, std::move(dc));
    return RL0_OK;
}

// ---------------------------------------------------------------- working memory

// A decode's whole launch sequence, captured once and replayed: one host call in place
// of ~4 + 3 * iterations launches.  Everything a launch bakes in is in the key.
struct DecodeKey {
    const void* A;
    const void* y;
    void* x;
    const void* dc;
    int32_t n, m, d;
    rl0_params p;
};

struct GraphEntry {
    DecodeKey key;
    hipGraphExec_t exec = nullptr;
    unsigned long long last_use = 0;
};

constexpr size_t kMaxGraphs = 16;   // per workspace; least recently used is dropped

struct Buffers {
    int cap_n = 0, cap_m = 0;
    void* block = nullptr;
    rl0::Workspace w{};
    rl0::DevState* st_host = nullptr;  // pinned copy of the device state
    hipStream_t capture = nullptr;     // private stream the launch sequence is captured on
    std::vector<GraphEntry> graphs;    // replayable decodes on this workspace
    unsigned long long uses = 0;
};

bool graphs_enabled() {
    static const bool on = [] {
        const char* e = std::getenv("RL0_GRAPHS");
        return !(e && e[0] == '0');
    }();
    return on;
}

void drop_graphs(Buffers* b) {
    for (GraphEntry& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

std::map<std::pair<int, hipStream_t>, std::unique_ptr<Buffers>> g_ws;

int get_workspace(int device, hipStream_t s, int n, int m, Buffers** out) {
    auto& slot = g_ws[{device, s}];
    if (!slot) slot = std::make_unique<Buffers>();
    Buffers* b = slot.get();
    if (b->cap_n < n || b->cap_m < m || !b->block) {
        if (b->block) {
            HIP_TRY(hipStreamSynchronize(s));
            drop_graphs(b);   // they point into the old block
            HIP_TRY(hipFree(b->block));
            b->block = nullptr;
        }
        const int cn = std::max(n, b->cap_n), cm = std::max(m, b->cap_m);
        if (hipMalloc(&b->block, rl0::workspace_bytes(cn, cm)) != hipSuccess)
            return fail(RL0_ENOMEM, "hipMalloc(workspace)");
        rl0::carve_workspace(b->block, cn, cm, &b->w);
        b->cap_n = cn;
        b->cap_m = cm;
    }
    if (!b->st_host) {
        if (hipHostMalloc(&b->st_host, sizeof(rl0::DevState), hipHostMallocDefault) != hipSuccess)
            return fail(RL0_ENOMEM, "hipHostMalloc(state)");
    }
    *out = b;
    return RL0_OK;
}

// ---------------------------------------------------------------- argument checks

int check_dims(int32_t n, int32_t m, int32_t d) {
    if (n < 1 || m < 1) return fail(RL0_EINVAL, "n and m must be >= 1");
    if (d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "d must be in [1, 16]");
    if (d > m) return fail(RL0_EINVAL, "d must be <= m");
    if (static_cast<long long>(n) * d > 0x7FFFFFFFLL * 4) return fail(RL0_EINVAL, "n*d too large");
    return RL0_OK;
}

int check_params(const rl0_params* p, int32_t n, int32_t m, int32_t d) {
    if (!p) return fail(RL0_EINVAL, "params is NULL");
    if (int rc = check_dims(n, m, d)) return rc;
    if (p->k < 1 || p->k >= m) return fail(RL0_EINVAL, "k must be in [1, m)");
    if (!(p->alpha > 1.0f && p->alpha <= static_cast<float>(d))) return fail(RL0_EINVAL, "alpha must be in (1, d]");
    if (!(p->c >= 0.0f && p->c < 1.0f)) return fail(RL0_EINVAL, "c must be in [0, 1) (0 = the paper's rule)");
    if (!(p->sigma >= 0.0f) || !std::isfinite(p->sigma)) return fail(RL0_EINVAL, "sigma must be finite and >= 0");
    if (!(p->sigma_signal > 0.0f) || !std::isfinite(p->sigma_signal))
        return fail(RL0_EINVAL, "sigma_signal must be finite and > 0");
    if (p->series_terms < 1 || p->series_terms > 30) return fail(RL0_EINVAL, "series_terms must be in [1, 30]");
    if (p->max_iters < 0) return fail(RL0_EINVAL, "max_iters must be >= 0");
    if (p->l1_test != 0 && p->l1_test != 1) return fail(RL0_EINVAL, "l1_test must be 0 or 1");
    if (p->posterior != 0 && p->posterior != 1) return fail(RL0_EINVAL, "posterior must be 0 or 1");
    if (p->posterior == 1 && !p->mlp) return fail(RL0_ENOWEIGHTS, "learned posterior requested without weights");
    if (p->posterior == 1) return fail(RL0_EINVAL, "learned posterior is not available in this build");
    return RL0_OK;
}

rl0::Problem problem_of(const rl0_params* p, int32_t n, int32_t m, int32_t d) {
    rl0::Problem pr;
    pr.n = n; pr.m = m; pr.d = d; pr.k = p->k;
    pr.sigma = static_cast<double>(p->sigma);
    pr.sigma_s = static_cast<double>(p->sigma_signal);
    pr.c = static_cast<double>(p->c);
    pr.ell = p->series_terms;
    pr.max_iters = p->max_iters;
    return pr;
}

int err_code_of(int flags) {
    if (flags & rl0::kErrIndex) return fail(RL0_EINDEX, "A_cols: index out of range or column not strictly ascending");
    if (flags & rl0::kErrNonFinite) return fail(RL0_EINVAL, "y holds a non-finite value");
    if (flags & rl0::kErrRange) return fail(RL0_ERANGE, "a value left the fixed-point range (|v| >= 2^22)");
    return RL0_OK;
}

// Launches the decode whose launches `issue` makes, from the workspace's graph cache;
// a key seen for the first time is captured on the private stream first.
template <class Issue>
int replay_decode(Buffers* b, const DecodeKey& key, hipStream_t s, Issue&& issue) {
    GraphEntry* hit = nullptr;
    for (GraphEntry& g : b->graphs)
        if (std::memcmp(&g.key, &key, sizeof(key)) == 0) hit = &g;
    if (!hit) {
        if (!b->capture) HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
        const int rc = issue(b->capture);
        hipGraph_t graph = nullptr;
        const hipError_t ec = hipStreamEndCapture(b->capture, &graph);
        if (rc != RL0_OK) {
            if (graph) (void)hipGraphDestroy(graph);
            return rc;
        }
        if (ec != hipSuccess) return fail(RL0_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
        hipGraphExec_t exec = nullptr;
        const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (ei != hipSuccess) return fail(RL0_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ei));
        if (b->graphs.size() >= kMaxGraphs) {
            // every decode on this workspace synchronises before returning: none in flight
            size_t lru = 0;
            for (size_t i = 1; i < b->graphs.size(); ++i)
                if (b->graphs[i].last_use < b->graphs[lru].last_use) lru = i;
            (void)hipGraphExecDestroy(b->graphs[lru].exec);
            b->graphs.erase(b->graphs.begin() + static_cast<std::ptrdiff_t>(lru));
        }
        GraphEntry g;
        g.key = key;
        g.exec = exec;
        b->graphs.push_back(g);
        hit = &b->graphs.back();
    }
    hit->last_use = ++b->uses;
    HIP_TRY(hipGraphLaunch(hit->exec, s));
    return RL0_OK;
}

rl0::ScoreTables tables_of(const DeviceConstants* dc) {
    rl0::ScoreTables tb;
    tb.Tz = dc->d_tables;
    tb.Te = dc->d_tables + rl0::kTableStrideFloats;
    tb.inv_h_z = dc->hc.inv_h_z;
    tb.inv_h_e = dc->hc.inv_h_e;
    tb.exact = dc->hc.exact ? 1 : 0;
    return tb;
}

rl0::IterParams iter_params(const DeviceConstants* dc, const rl0_params* p, int it) {
    rl0::IterParams ip;
    const int N = dc->hc.n_iters;
    ip.it = it;
    ip.t = it < N ? dc->hc.t[it] : static_cast<float>(1.0 - it * dc->hc.c);
    ip.tau_bits = it < N ? dc->hc.tau_bits[it] : 0x7F800000u;
    ip.tau_next = it + 1 < N ? dc->hc.tau_bits[it + 1] : 0x7F800000u;
    ip.alpha = p->alpha;
    ip.l1_test = p->l1_test;
    ip.n_iters = N;
    ip.tol_fx = dc->hc.tol * 1073741824.0;
    return ip;
}


}  // namespace

extern "C" {

const char* rl0_last_error(void) { return g_last_error.c_str(); }

int rl0_params_default(rl0_params* p, int32_t n, int32_t m, int32_t d, int32_t k, float sigma) {
    if (!p) return fail(RL0_EINVAL, "params is NULL");
    if (int rc = check_dims(n, m, d)) return rc;
    if (k < 1 || k >= m) return fail(RL0_EINVAL, "k must be in [1, m)");
    std::memset(p, 0, sizeof(*p));
    p->k = k;
    p->sigma = sigma;
    p->sigma_signal = 1.0f;
    p->alpha = 2.0f;
    p->c = 0.0f;  // the paper's rule, evaluated in double by the constants
    p->series_terms = 4;
    p->max_iters = 0;
    p->l1_test = 0;
    p->posterior = 0;
    p->mlp = nullptr;
    p->validate = 1;
    return RL0_OK;
}

int rl0_compute_constants(const rl0_params* p, int32_t n, int32_t m, int32_t d, rl0_constants* out,
                          float* t_h, float* tau_h) {
    if (int rc = check_params(p, n, m, d)) return rc;
    if (!out) return fail(RL0_EINVAL, "out is NULL");
    rl0::HostConstants hc;
    rl0::compute_constants(problem_of(p, n, m, d), &hc);
    out->n_iters = hc.n_iters;
    out->exact = hc.exact ? 1 : 0;
    out->c = hc.c;
    out->tol = hc.tol;
    out->range_z = hc.range_z;
    out->range_e = hc.range_e;
    out->inv_h_z = hc.inv_h_z;
    out->inv_h_e = hc.inv_h_e;
    std::memcpy(out->table_z, hc.table_z, sizeof(hc.table_z));
    std::memcpy(out->table_e, hc.table_e, sizeof(hc.table_e));
    for (int it = 0; it < hc.n_iters; ++it) {
        if (t_h) t_h[it] = hc.t[it];
        if (tau_h) { float f; std::memcpy(&f, &hc.tau_bits[it], 4); tau_h[it] = f; }
    }
    return RL0_OK;
}

int rl0_validate(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, void* stream) {
    if (int rc = check_dims(n, m, d)) return rc;
    if (!A_cols) return fail(RL0_EINVAL, "A_cols is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    Buffers* b = nullptr;
    if (int rc = get_workspace(dev, s, 1, 1, &b)) return rc;
    HIP_TRY(rl0::launch_clear_state(b->w.st, s));
    HIP_TRY(rl0::launch_validate(A_cols, n, m, d, &b->w.st->err, s));
    HIP_TRY(hipMemcpyAsync(b->st_host, b->w.st, sizeof(rl0::DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return err_code_of(b->st_host->err);
}

int rl0_sketch(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* x, float* y,
               void* stream) {
    if (int rc = check_dims(n, m, d)) return rc;
    if (!A_cols || !x || !y) return fail(RL0_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    Buffers* b = nullptr;
    if (int rc = get_workspace(dev, s, 1, m, &b)) return rc;
    HIP_TRY(rl0::launch_clear_state(b->w.st, s));
    HIP_TRY(rl0::launch_sketch(A_cols, n, m, d, x, y, b->w.S[0], &b->w.st->err, s));
    HIP_TRY(hipMemcpyAsync(b->st_host, b->w.st, sizeof(rl0::DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return err_code_of(b->st_host->err);
}

int rl0_decode(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* y,
               const rl0_params* p, float* x_out, rl0_stats* st_h, void* stream) {
    if (int rc = check_params(p, n, m, d)) return rc;
    if (!A_cols || !y || !x_out) return fail(RL0_EINVAL, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(A_cols) % 16) return fail(RL0_EINVAL, "A_cols must be 16-byte aligned");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DeviceConstants* dc = nullptr;
    if (int rc = get_constants(problem_of(p, n, m, d), dev, &dc)) return rc;
    Buffers* b = nullptr;
    if (int rc = get_workspace(dev, s, n, m, &b)) return rc;
    const rl0::DecodeDims dm{n, m, d, p->k};
    const rl0::ScoreTables tb = tables_of(dc);
    const int N = dc->hc.n_iters;
    auto issue = [&](hipStream_t q) -> int {
        HIP_TRY(rl0::launch_prepare(dm, A_cols, p->validate != 0, y, nullptr, b->w, iter_params(dc, p, 0), q));
        const rl0::DebugOut dbg{nullptr, nullptr};
        for (int it = 0; it < N; ++it)
            HIP_TRY(rl0::launch_iteration(dm, A_cols, b->w, tb, iter_params(dc, p, it), dbg, q, profile_events(it)));
        HIP_TRY(rl0::launch_finish(dm, b->w, iter_params(dc, p, N), 0, x_out, q));
        return RL0_OK;
    };
    // per-iteration timing events cannot be recorded into a captured graph: a profiled
    // decode launches eagerly
    if (graphs_enabled() && !g_prof.enabled) {
        DecodeKey key;
        std::memset(&key, 0, sizeof(key));
        key.A = A_cols;
        key.y = y;
        key.x = x_out;
        key.dc = dc;
        key.n = n;
        key.m = m;
        key.d = d;
        std::memcpy(&key.p, p, sizeof(*p));
        if (int rc = replay_decode(b, key, s, issue)) return rc;
    } else {
        if (int rc = issue(s)) return rc;
    }
    // the slots, counters and flags lead the device state
    HIP_TRY(hipMemcpyAsync(b->st_host, b->w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const rl0::DevState& ds = *b->st_host;
    const rl0::Slot& fin = ds.slot[N & 1];
    profile_collect(N, fin.iterations);
    if (st_h) {
        st_h->iterations = fin.iterations;
        st_h->accepted = fin.accepted;
        st_h->l1_final_fx = fin.L_hat;
        st_h->l1_final = static_cast<double>(fin.L_hat) / 1073741824.0;
        st_h->l1_tol = dc->hc.tol;
        st_h->converged = (static_cast<double>(fin.L_hat) <= dc->hc.tol * 1073741824.0) ? 1 : 0;
        st_h->updates_total = ds.updates_total;
        st_h->t_final = fin.iterations > 0 ? dc->hc.t[fin.iterations - 1] : 1.0f;
        st_h->error_flags = ds.err;
    }
    return err_code_of(ds.err);
}

int rl0_step(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* y,
             const rl0_params* p, int32_t it, float* x_hat, float* r_hat, int64_t* L_hat_h,
             int32_t* accepted_h, int32_t* updated, float* omega, float* x_trial, float* r_trial,
             void* stream) {
    if (int rc = check_params(p, n, m, d)) return rc;
    if (!A_cols || !y || !x_hat || !r_hat || !L_hat_h) return fail(RL0_EINVAL, "NULL pointer");
    if (reinterpret_cast<uintptr_t>(A_cols) % 16) return fail(RL0_EINVAL, "A_cols must be 16-byte aligned");
    if (it < 0) return fail(RL0_EINVAL, "it must be >= 0");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    DeviceConstants* dc = nullptr;
    if (int rc = get_constants(problem_of(p, n, m, d), dev, &dc)) return rc;
    Buffers* b = nullptr;
    if (int rc = get_workspace(dev, s, n, m, &b)) return rc;
    const rl0::DecodeDims dm{n, m, d, p->k};
    const rl0::Workspace& w = b->w;
    rl0::IterParams ip = iter_params(dc, p, it);
    ip.n_iters = it + 1;
    ip.tol_fx = -1.0;  // a single step never stops early
    rl0::IterParams ip_end = iter_params(dc, p, it + 1);
    ip_end.n_iters = it + 1;
    ip_end.tol_fx = -1.0;
    if (updated) HIP_TRY(rl0::launch_zero_i32(updated, n, s));
    if (omega) HIP_TRY(rl0::launch_zero_f32(omega, n, s));
    HIP_TRY(rl0::launch_prepare(dm, A_cols, p->validate != 0, y, x_hat, w, ip, s));
    const rl0::DebugOut dbg{updated, omega};
    HIP_TRY(rl0::launch_iteration(dm, A_cols, w, tables_of(dc), ip, dbg, s));
    HIP_TRY(rl0::launch_finish(dm, w, ip_end, it, x_hat, s));
    // the iteration ran from buffer 0; its trial iterate sits in buffer 1
    if (x_trial) HIP_TRY(rl0::launch_trial_out(dm, w, it + 1, it, x_trial, s));
    if (r_trial) HIP_TRY(rl0::launch_copy_f32(w.r[1], r_trial, m, s));
    HIP_TRY(hipMemcpyAsync(b->st_host, w.st, sizeof(rl0::DevState), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const rl0::DevState& ds = *b->st_host;
    if (int rc = err_code_of(ds.err)) return rc;
    const rl0::Slot& fin = ds.slot[(it + 1) & 1];
    if (accepted_h) *accepted_h = fin.accepted_last;
    *L_hat_h = fin.L_hat;
    HIP_TRY(rl0::launch_copy_f32(w.r[fin.cur], r_hat, m, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RL0_OK;
}

int rl0_profile_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof.enabled = enable != 0;
    for (double& t : g_prof.total_ms) t = 0.0;
    g_prof.launches = 0;
    g_prof.executed = 0;
    return RL0_OK;
}

int rl0_profile_read(double* sweep_ms_total_h, int64_t* sweep_launches_h) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (sweep_ms_total_h) *sweep_ms_total_h = g_prof.total_ms[0];
    if (sweep_launches_h) *sweep_launches_h = g_prof.launches;
    return RL0_OK;
}

int rl0_profile_read_kernels(double* ms_total_h, int64_t* counts_h) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!ms_total_h) return fail(RL0_EINVAL, "NULL pointer");
    for (int k = 0; k < 6; ++k) ms_total_h[k] = g_prof.total_ms[k];
    if (counts_h) {
        counts_h[0] = g_prof.launches;
        counts_h[1] = g_prof.executed;
    }
    return RL0_OK;
}

void rl0_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipDeviceSynchronize();
    for (auto& kv : g_ws) {
        drop_graphs(kv.second.get());
        if (kv.second->capture) hipStreamDestroy(kv.second->capture);
        if (kv.second->block) hipFree(kv.second->block);
        if (kv.second->st_host) hipHostFree(kv.second->st_host);
    }
    g_ws.clear();
    for (auto& kv : g_consts)
        if (kv.second->d_tables) hipFree(kv.second->d_tables);
    g_consts.clear();
    for (hipEvent_t e : g_prof.pool) hipEventDestroy(e);
    g_prof.pool.clear();
}

}  // extern "C"
