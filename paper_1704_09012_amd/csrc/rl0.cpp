// C-ABI of librl0 (declared in include/rl0.h): argument checks, the cached constants
// and working memory, and the host-side order of kernel launches.
#include "../../include/rl0.h"

#include <hip/hip_runtime.h>

#include <array>
#include <cerrno>
#include <cmath>
#include <cstddef>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <map>
#include <set>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <algorithm>
#include <tuple>
#include <vector>

#include <unistd.h>

#include "constants.h"
#include "kernels.h"
#include "batched.h"
#include "mlp.h"
#include "noalloc.h"

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
    std::vector<hipEvent_t> pool;   // per iteration: start and end of the sweep, H_k's classification
                                    // (large m only), the row kernel
    double total_ms[4] = {0.0, 0.0, 0.0, 0.0};   // sweep and row kernel: all launched, then executed
    long long launches = 0, executed = 0;
    hipEvent_t learned_ev[2] = {nullptr, nullptr};   // around the learned decision of rl0_step
    double learned_ms = 0.0;
    long long learned_launches = 0;
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
// `executed` of which ran before the stopping condition); with `pre` the row kernel's time
// includes H_k's classification kernel
void profile_collect(int launched, int executed, bool pre) {
    if (!g_prof.enabled) return;
    for (int it = 0; it < launched && 6 * static_cast<size_t>(it) + 5 < g_prof.pool.size(); ++it) {
        float ms[2] = {0.0f, 0.0f}, mc = 0.0f;
        const bool ok =
            hipEventElapsedTime(&ms[0], g_prof.pool[6 * it], g_prof.pool[6 * it + 1]) == hipSuccess &&
            hipEventElapsedTime(&ms[1], g_prof.pool[6 * it + 4], g_prof.pool[6 * it + 5]) == hipSuccess &&
            (!pre || hipEventElapsedTime(&mc, g_prof.pool[6 * it + 2], g_prof.pool[6 * it + 3]) == hipSuccess);
        if (!ok) continue;
        ms[1] += mc;
        for (int k = 0; k < 2; ++k) g_prof.total_ms[k] += ms[k];
        g_prof.launches += 1;
        if (it < executed) {
            for (int k = 0; k < 2; ++k) g_prof.total_ms[2 + k] += ms[k];
            g_prof.executed += 1;
        }
    }
}

// ---------------------------------------------------------------- constants cache

struct DeviceConstants {
    rl0::HostConstants hc;
    float* d_tables = nullptr;        // table_z, table_e (kTableStrideFloats apart), then tau
    const uint32_t* d_tau = nullptr;  // outer-test threshold bits per iteration
    const uint32_t* d_qe = nullptr;   // quantised-score thresholds per iteration (after tau)
    const uint32_t* d_qz = nullptr;
    size_t bytes = 0;                 // size of the d_tables allocation
};

using ConstKey = std::tuple<int, int, int, int, int, uint32_t, uint32_t, double, int, int, int, int, int, bool,
                            unsigned long long>;
std::map<ConstKey, std::unique_ptr<DeviceConstants>> g_consts;

uint32_t fbits(float f) { uint32_t u; std::memcpy(&u, &f, 4); return u; }

// Looks up (or builds and uploads) the constants of a problem; the device copy is
// written with a blocking copy, so it is ready before any later launch.
ConstKey key_of(const rl0::Problem& pr, int device) {
    return ConstKey{device, pr.n, pr.m, pr.d, pr.k, fbits(static_cast<float>(pr.sigma)),
                    fbits(static_cast<float>(pr.sigma_s)), pr.c, pr.ell, pr.max_iters, pr.variant,
                    pr.signal_law, pr.noise_law, pr.tables != nullptr, pr.tables_hash};
}

// Device copy of computed constants: both tables and the per-iteration thresholds (tau,
// then the quantised-score thresholds qe and qz) in one allocation, written with a
// blocking copy, so they are ready before any later launch.
int upload_constants(DeviceConstants* dc) {
    const size_t tab = 2 * rl0::kTableStrideFloats * sizeof(float);
    const size_t ntau = dc->hc.tau_bits.size();
    const size_t per = sizeof(uint32_t) * (ntau ? ntau : 1);
    std::vector<char> staging(tab + 3 * per, 0);
    std::memcpy(staging.data(), dc->hc.table_z, (rl0::kTableN + 1) * sizeof(float));
    std::memcpy(staging.data() + rl0::kTableStrideFloats * sizeof(float), dc->hc.table_e,
                (rl0::kTableN + 1) * sizeof(float));
    if (ntau) {
        std::memcpy(staging.data() + tab, dc->hc.tau_bits.data(), ntau * sizeof(uint32_t));
        std::memcpy(staging.data() + tab + per, dc->hc.qe_bits.data(), ntau * sizeof(uint32_t));
        std::memcpy(staging.data() + tab + 2 * per, dc->hc.qz_bits.data(), ntau * sizeof(uint32_t));
    }
    if (dc->bytes < staging.size()) {   // a constant set rewritten in place keeps a large enough block
        if (dc->d_tables) HIP_TRY(hipFree(dc->d_tables));
        dc->d_tables = nullptr;
        dc->bytes = 0;
        if (hipMalloc(&dc->d_tables, staging.size()) != hipSuccess) return fail(RL0_ENOMEM, "hipMalloc(tables)");
        dc->bytes = staging.size();
    }
    HIP_TRY(hipMemcpy(dc->d_tables, staging.data(), staging.size(), hipMemcpyHostToDevice));
    const char* base = reinterpret_cast<const char*>(dc->d_tables);
    dc->d_tau = reinterpret_cast<const uint32_t*>(base + tab);
    dc->d_qe = reinterpret_cast<const uint32_t*>(base + tab + per);
    dc->d_qz = reinterpret_cast<const uint32_t*>(base + tab + 2 * per);
    return RL0_OK;
}

// At most this many problems' constants are kept; past it the cache is emptied (rare:
// every distinct sigma of a problem size is an entry).
constexpr size_t kMaxConstants = 4096;
int drop_all_constants();   // after the working memory's definitions

// Looks up (or builds and uploads) the constants of a problem.
int get_constants(const rl0::Problem& pr, int device, DeviceConstants** out) {
    if (g_consts.size() >= kMaxConstants)
        if (int rc = drop_all_constants()) return rc;
    const ConstKey key = key_of(pr, device);
    auto it = g_consts.find(key);
    if (it != g_consts.end()) {
        *out = it->second.get();
        return RL0_OK;
    }
    auto dc = std::make_unique<DeviceConstants>();
    if (!rl0::compute_constants(pr, &dc->hc))
        return fail(RL0_EINVAL, "the posteriors of these signal and noise laws could not be tabulated");
    if (int rc = upload_constants(dc.get())) return rc;
    *out = dc.get();
    g_consts.emplace(key, std::move(dc));
    return RL0_OK;
}

// The same for many problems; the ones not cached yet are computed on host threads.
int get_constants_many(const std::vector<rl0::Problem>& prs, int device, std::vector<DeviceConstants*>* out) {
    if (g_consts.size() + prs.size() > kMaxConstants)
        if (int rc = drop_all_constants()) return rc;
    out->assign(prs.size(), nullptr);
    std::map<ConstKey, size_t> fresh_of;   // key -> index into fresh
    std::vector<size_t> fresh_src;          // a problem index per fresh entry
    for (size_t i = 0; i < prs.size(); ++i) {
        const ConstKey key = key_of(prs[i], device);
        auto it = g_consts.find(key);
        if (it != g_consts.end()) {
            (*out)[i] = it->second.get();
        } else if (!fresh_of.count(key)) {
            fresh_of.emplace(key, fresh_src.size());
            fresh_src.push_back(i);
        }
    }
    std::vector<std::unique_ptr<DeviceConstants>> fresh(fresh_src.size());
    for (auto& f : fresh) f = std::make_unique<DeviceConstants>();
    const size_t nt = std::min<size_t>(fresh.size(), std::max(1u, std::min(16u, std::thread::hardware_concurrency())));
    std::vector<std::thread> pool;
    std::vector<char> ok(fresh.size(), 1);
    for (size_t t = 0; t < nt; ++t)
        pool.emplace_back([&, t] {
            for (size_t f = t; f < fresh.size(); f += nt)
                ok[f] = rl0::compute_constants(prs[fresh_src[f]], &fresh[f]->hc) ? 1 : 0;
        });
    for (auto& th : pool) th.join();
    for (size_t f = 0; f < fresh.size(); ++f)
        if (!ok[f])
            return fail(RL0_EINVAL, "instance " + std::to_string(fresh_src[f]) +
                                        ": the posteriors of these signal and noise laws could not be tabulated");
    for (size_t f = 0; f < fresh.size(); ++f)
        if (int rc = upload_constants(fresh[f].get())) return rc;
    for (auto& kv : fresh_of) g_consts.emplace(kv.first, std::move(fresh[kv.second]));
    for (size_t i = 0; i < prs.size(); ++i)
        if (!(*out)[i]) (*out)[i] = g_consts.at(key_of(prs[i], device)).get();
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

constexpr size_t kMaxGraphs = 64;   // per workspace; least recently used is dropped

struct Buffers {
    int cap_n = 0, cap_m = 0;
    void* block = nullptr;
    rl0::Workspace w{};
    rl0::DevState* st_host = nullptr;  // pinned copy of the device state
    hipStream_t capture = nullptr;     // private stream the launch sequence is captured on
    hipEvent_t ev_call[2] = {nullptr, nullptr};   // start and end of a decode (rl0_stats.ms_total)
    std::vector<GraphEntry> graphs;    // replayable decodes on this workspace
    unsigned long long uses = 0;
    std::unique_ptr<DeviceConstants> adapted;   // adaptive_k: the decode's current constants
    int last_log_count = 0;            // executed iterations of the last decode (its log records)
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
    if (!b->ev_call[0]) {
        HIP_TRY(hipEventCreate(&b->ev_call[0]));
        HIP_TRY(hipEventCreate(&b->ev_call[1]));
    }
    *out = b;
    return RL0_OK;
}

// Frees every cached constant set.  Decode graphs bake their constants' device
// pointers, so they go too, once all work on every device that holds a workspace is done.
int drop_all_constants() {
    int cur = 0;
    HIP_TRY(hipGetDevice(&cur));
    std::set<int> devices;
    for (auto& kv : g_ws) devices.insert(kv.first.first);
    for (auto& kv : g_consts) devices.insert(std::get<0>(kv.first));
    for (int dev : devices) {
        HIP_TRY(hipSetDevice(dev));
        HIP_TRY(hipDeviceSynchronize());
    }
    HIP_TRY(hipSetDevice(cur));
    for (auto& kv : g_ws) drop_graphs(kv.second.get());
    for (auto& kv : g_consts)
        if (kv.second->d_tables) HIP_TRY(hipFree(kv.second->d_tables));
    g_consts.clear();
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
    if (p->posterior == 1 && d + 1 > rl0::kMlpMaxFeatures)
        return fail(RL0_EINVAL, "the learned posterior supports d <= 15");
    if (p->variant != 0 && p->variant != 1)
        return fail(RL0_EINVAL, "variant must be 0 (continuous scores) or 1 (quantised)");
    if (p->adaptive_k != 0 && p->adaptive_k != 1) return fail(RL0_EINVAL, "adaptive_k must be 0 or 1");
    if (p->adaptive_k == 1 && p->posterior == 1)
        return fail(RL0_EINVAL, "adaptive_k applies to the analytic posteriors only");
    if (p->log != 0 && p->log != 1) return fail(RL0_EINVAL, "log must be 0 or 1");
    if (p->wg_order != 0 && p->wg_order != 1) return fail(RL0_EINVAL, "wg_order must be 0 or 1");
    for (int32_t law : {p->signal_law, p->noise_law})
        if (law != RL0_LAW_GAUSSIAN && law != RL0_LAW_LAPLACE)
            return fail(RL0_EINVAL, "signal_law and noise_law must be RL0_LAW_GAUSSIAN or RL0_LAW_LAPLACE");
    if (p->adaptive_k == 1 && (p->tables || p->signal_law != RL0_LAW_GAUSSIAN || p->noise_law != RL0_LAW_GAUSSIAN))
        return fail(RL0_EINVAL, "adaptive_k rebuilds the Gaussian posteriors only (no other laws, no given tables)");
    if (p->tables) {
        const float* t = p->tables;
        for (int k = 0; k < 2; ++k) {
            const float* T = t + k * (RL0_TABLE_N + 1);
            if (T[0] != 1.0f) return fail(RL0_EINVAL, "tables: each table must start at 1");
            for (int i = 0; i <= RL0_TABLE_N; ++i) {
                if (!(T[i] >= 0.0f && T[i] <= 1.0f)) return fail(RL0_EINVAL, "tables: entries must lie in [0, 1]");
                if (i > 0 && T[i] > T[i - 1]) return fail(RL0_EINVAL, "tables: entries must be non-increasing");
            }
            const float ih = t[2 * (RL0_TABLE_N + 1) + k];
            if (!(ih > 0.0f) || !std::isfinite(ih)) return fail(RL0_EINVAL, "tables: inv_h must be finite and > 0");
        }
    }
    return RL0_OK;
}

// The parameters as part of a cache key (compared with memcmp): every field copied into
// *out after zeroing it, so that the padding between fields (whatever the caller's struct
// holds there) compares equal.
void params_key(const rl0_params* p, rl0_params* out) {
    rl0_params& k = *out;
    std::memset(out, 0, sizeof(*out));
    k.k = p->k;
    k.sigma = p->sigma;
    k.sigma_signal = p->sigma_signal;
    k.alpha = p->alpha;
    k.c = p->c;
    k.series_terms = p->series_terms;
    k.max_iters = p->max_iters;
    k.l1_test = p->l1_test;
    k.posterior = p->posterior;
    k.mlp = p->mlp;
    k.validate = p->validate;
    k.variant = p->variant;
    k.adaptive_k = p->adaptive_k;
    k.signal_law = p->signal_law;
    k.noise_law = p->noise_law;
    k.log = p->log;
    k.wg_order = p->wg_order;
    // given tables enter through the constants (their device copy is part of the key)
}

rl0::Problem problem_of(const rl0_params* p, int32_t n, int32_t m, int32_t d) {
    rl0::Problem pr;
    pr.n = n; pr.m = m; pr.d = d; pr.k = p->k;
    pr.sigma = static_cast<double>(p->sigma);
    pr.sigma_s = static_cast<double>(p->sigma_signal);
    pr.c = static_cast<double>(p->c);
    pr.ell = p->series_terms;
    pr.max_iters = p->max_iters;
    pr.variant = p->variant;
    pr.signal_law = p->signal_law;
    pr.noise_law = p->noise_law;
    if (p->tables) {
        // FNV-1a over the floats' bytes
        unsigned long long h = 1469598103934665603ull;
        const unsigned char* bytes = reinterpret_cast<const unsigned char*>(p->tables);
        for (size_t i = 0; i < sizeof(float) * RL0_TABLES_FLOATS; ++i) h = (h ^ bytes[i]) * 1099511628211ull;
        pr.tables = p->tables;
        pr.tables_hash = h;
    }
    return pr;
}

int err_code_of(int flags) {
    if (flags & rl0::kErrIndex) return fail(RL0_EINDEX, "A_cols: index out of range or column not strictly ascending");
    if (flags & rl0::kErrNonFinite) return fail(RL0_EINVAL, "y holds a non-finite value");
    if (flags & rl0::kErrRange) return fail(RL0_ERANGE, "a value left the fixed-point range (|v| >= 2^22)");
    if (flags & rl0::kErrTimeout) return fail(RL0_EHIP, "a bounded wait of a workgroup group timed out");
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

// The key with the buffers of y and x_out left out.
DecodeKey without_io(DecodeKey k) {
    k.y = nullptr;
    k.x = nullptr;
    return k;
}

// Replays a decode whose launches issue(q, y, x) makes.  A graph bakes the buffers it
// was captured with, so a call with other y / x_out buffers than the cached graph's
// (the same matrix and parameters otherwise) would capture and instantiate anew.  Such
// a call runs the graph captured once on the workspace's staging buffers instead: y is
// copied in before it and x copied out after it.
template <class Issue>
int replay_decode_io(Buffers* b, DecodeKey key, const float* y, float* x_out, int n, int m, hipStream_t s,
                     Issue&& issue) {
    key.y = y;
    key.x = x_out;
    const DecodeKey staged = without_io(key);
    bool direct = false, seen = false;
    for (const GraphEntry& g : b->graphs) {
        if (std::memcmp(&g.key, &key, sizeof(key)) == 0) direct = true;
        const DecodeKey gk = without_io(g.key);
        if (std::memcmp(&gk, &staged, sizeof(staged)) == 0) seen = true;
    }
    if (direct || !seen)
        return replay_decode(b, key, s, [&](hipStream_t q) { return issue(q, y, x_out); });
    HIP_TRY(hipMemcpyAsync(b->w.ystage, y, sizeof(float) * m, hipMemcpyDeviceToDevice, s));
    if (int rc = replay_decode(b, staged, s, [&](hipStream_t q) { return issue(q, b->w.ystage, b->w.xstage); }))
        return rc;
    HIP_TRY(hipMemcpyAsync(x_out, b->w.xstage, sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    return RL0_OK;
}

rl0::ScoreTables tables_of(const DeviceConstants* dc) {
    rl0::ScoreTables tb;
    tb.Tz = dc->d_tables;
    tb.Te = dc->d_tables + rl0::kTableStrideFloats;
    tb.inv_h_z = dc->hc.inv_h_z;
    tb.inv_h_e = dc->hc.inv_h_e;
    tb.exact = dc->hc.exact ? 1 : 0;
    tb.e_zero_bits = dc->hc.e_zero_bits;
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
    ip.quant = dc->hc.quant ? 1 : 0;
    ip.log = p->log;
    ip.wg_rev = p->wg_order;
    if (ip.quant && it < N) {
        ip.qe_bits = dc->hc.qe_bits[it];
        ip.qz_bits = dc->hc.qz_bits[it];
    }
    return ip;
}


// ---------------------------------------------------------------- batched decoding

struct BatchKey {
    int32_t count, d, block, per_cu, grid;
    size_t lds;
    const void* meta;
    uint64_t queue;   // hash of the launches' ticket ranges and grids
};

struct BatchGraph {
    BatchKey key;
    hipGraphExec_t exec = nullptr;
    unsigned long long last_use = 0;
};

// Working memory of batched decodes on one (device, stream).
struct BatchBuffers {
    void* block = nullptr;           // per-instance S, x', stamps, change lists
    size_t block_bytes = 0;
    void* meta = nullptr;            // descriptors, order, results, queue counter
    size_t meta_count = 0;
    void* host = nullptr;            // pinned staging of descriptors, order and results
    hipStream_t capture = nullptr;
    hipEvent_t ev[2] = {nullptr, nullptr};
    hipEvent_t ev_call[2] = {nullptr, nullptr};   // around a whole batched call (ms_total)
    std::vector<BatchGraph> graphs;
    unsigned long long uses = 0;
    std::vector<rl0::BatchResult> last_res;   // the last call's results (rl0_batch_timeline)
    std::vector<int> last_group;
    rl0::BatchProblem* desc_d() const { return static_cast<rl0::BatchProblem*>(meta); }
};

std::map<std::pair<int, hipStream_t>, std::unique_ptr<BatchBuffers>> g_bws;
std::map<int, rl0_batch_schedule> g_sched;
std::map<int, bool> g_lds_ready;

size_t meta_bytes(size_t count) {
    return rl0::al_host(count * sizeof(rl0::BatchProblem)) + rl0::al_host(count * rl0::kMaxGroup * sizeof(int)) +
           rl0::al_host(count * sizeof(rl0::BatchResult)) + rl0::al_host(count * sizeof(rl0::BatchCtl)) + 256;
}

struct MetaView {
    rl0::BatchProblem* desc;
    int* order;                 // tickets: instance * kTicketParts + part
    rl0::BatchResult* res;
    rl0::BatchCtl* ctl;         // one per instance (used by groups)
    int* counter;
};

MetaView meta_view(void* base, size_t count) {
    char* p = static_cast<char*>(base);
    MetaView v;
    v.desc = reinterpret_cast<rl0::BatchProblem*>(p);
    p += rl0::al_host(count * sizeof(rl0::BatchProblem));
    v.order = reinterpret_cast<int*>(p);
    p += rl0::al_host(count * rl0::kMaxGroup * sizeof(int));
    v.res = reinterpret_cast<rl0::BatchResult*>(p);
    p += rl0::al_host(count * sizeof(rl0::BatchResult));
    v.ctl = reinterpret_cast<rl0::BatchCtl*>(p);
    p += rl0::al_host(count * sizeof(rl0::BatchCtl));
    v.counter = reinterpret_cast<int*>(p);
    return v;
}

void drop_batch_graphs(BatchBuffers* b) {
    for (BatchGraph& g : b->graphs) (void)hipGraphExecDestroy(g.exec);
    b->graphs.clear();
}

int get_batch_buffers(int device, hipStream_t s, size_t block_bytes, size_t count, BatchBuffers** out) {
    auto& slot = g_bws[{device, s}];
    if (!slot) slot = std::make_unique<BatchBuffers>();
    BatchBuffers* b = slot.get();
    if (b->block_bytes < block_bytes) {
        HIP_TRY(hipStreamSynchronize(s));
        if (b->block) HIP_TRY(hipFree(b->block));
        b->block = nullptr;
        b->block_bytes = 0;
        if (hipMalloc(&b->block, block_bytes) != hipSuccess) return fail(RL0_ENOMEM, "hipMalloc(batch workspace)");
        b->block_bytes = block_bytes;
    }
    if (b->meta_count < count) {
        HIP_TRY(hipStreamSynchronize(s));
        drop_batch_graphs(b);   // they point into the old block
        if (b->meta) HIP_TRY(hipFree(b->meta));
        if (b->host) HIP_TRY(hipHostFree(b->host));
        b->meta = nullptr;
        b->host = nullptr;
        b->meta_count = 0;
        if (hipMalloc(&b->meta, meta_bytes(count)) != hipSuccess) return fail(RL0_ENOMEM, "hipMalloc(batch meta)");
        if (hipHostMalloc(&b->host, meta_bytes(count), hipHostMallocDefault) != hipSuccess)
            return fail(RL0_ENOMEM, "hipHostMalloc(batch meta)");
        b->meta_count = count;
    }
    if (!b->ev[0]) {
        HIP_TRY(hipEventCreate(&b->ev[0]));
        HIP_TRY(hipEventCreate(&b->ev[1]));
        HIP_TRY(hipEventCreate(&b->ev_call[0]));
        HIP_TRY(hipEventCreate(&b->ev_call[1]));
    }
    *out = b;
    return RL0_OK;
}

int size_class(int n) {
    int c = 0;
    while (c < RL0_SIZE_CLASSES - 1 && n >= (1 << (11 + c))) ++c;
    return c;
}

rl0_batch_schedule default_schedule() {
    // what the autotuner settles on for batches of uneven instances: one 1024-thread
    // workgroup per CU, which leaves the most LDS for the residual snapshot
    rl0_batch_schedule s;
    s.block = 1024;
    s.per_cu = 1;
    for (int c = 0; c < RL0_SIZE_CLASSES; ++c) {
        s.cols[c] = 4;
        s.group[c] = 4;   // the work estimate decides which instances are split (most are not)
    }
    return s;
}

int check_schedule(const rl0_batch_schedule& s) {
    if (s.block != 256 && s.block != 512 && s.block != 1024) return fail(RL0_EINVAL, "schedule: block must be 256, 512 or 1024");
    if (s.per_cu < 1 || s.per_cu > 8) return fail(RL0_EINVAL, "schedule: per_cu must be in [1, 8]");
    for (int c = 0; c < RL0_SIZE_CLASSES; ++c) {
        if (s.cols[c] != 1 && s.cols[c] != 2 && s.cols[c] != 4) return fail(RL0_EINVAL, "schedule: cols must be 1, 2 or 4");
        const int g = s.group[c];
        if (g != 1 && g != 2 && g != 4 && g != 8 && g != 16)
            return fail(RL0_EINVAL, "schedule: group must be 1, 2, 4, 8 or 16");
    }
    return RL0_OK;
}

rl0_batch_schedule& schedule_of(int device) {
    auto it = g_sched.find(device);
    if (it == g_sched.end()) it = g_sched.emplace(device, default_schedule()).first;
    return it->second;
}

// A batch checked, with its constants and working memory, ready to launch.
struct BatchPlan {
    int device = 0, count = 0, d = 0, max_m = 0;
    bool uniform_d = true;
    BatchBuffers* b = nullptr;
    std::vector<DeviceConstants*> dc;
    std::vector<size_t> offs;      // per instance: byte offset of its working memory
    std::vector<int> order;        // largest first
};

int plan_batch(const rl0_problem* probs, int count, hipStream_t s, BatchPlan* plan) {
    if (count < 0) return fail(RL0_EINVAL, "count must be >= 0");
    if (count > 0 && !probs) return fail(RL0_EINVAL, "probs_h is NULL");
    std::vector<rl0::Problem> prs(count);
    for (int i = 0; i < count; ++i) {
        const rl0_problem& q = probs[i];
        auto bad = [&](int rc) { return fail(rc, "instance " + std::to_string(i) + ": " + g_last_error); };
        if (int rc = check_params(&q.params, q.n, q.m, q.d)) return bad(rc);
        if (q.params.adaptive_k) return bad(fail(RL0_EINVAL, "adaptive_k is not supported by batched decodes"));
        if (q.params.posterior != 0)
            return bad(fail(RL0_EINVAL, "the learned posterior (posterior = 1) is not supported by batched decodes"));
        if (!q.A_cols || !q.y || !q.x_out) return fail(RL0_EINVAL, "instance " + std::to_string(i) + ": NULL pointer");
        if (reinterpret_cast<uintptr_t>(q.A_cols) % 16)
            return fail(RL0_EINVAL, "instance " + std::to_string(i) + ": A_cols must be 16-byte aligned");
        if (q.m > rl0::kBatchMaxRows)
            return fail(RL0_EINVAL, "instance " + std::to_string(i) + ": m exceeds RL0_BATCH_MAX_M");
        prs[i] = problem_of(&q.params, q.n, q.m, q.d);
    }
    plan->count = count;
    if (count == 0) return RL0_OK;
    HIP_TRY(hipGetDevice(&plan->device));
    if (int rc = get_constants_many(prs, plan->device, &plan->dc)) return rc;
    plan->offs.resize(count);
    size_t total = 0;
    plan->d = probs[0].d;
    for (int i = 0; i < count; ++i) {
        plan->offs[i] = total;
        total += rl0::al_host(8ull * probs[i].m) + rl0::al_host(4ull * probs[i].m) + 4 * rl0::al_host(4ull * probs[i].n) +
                 rl0::al_host(8ull * probs[i].n);
        plan->max_m = std::max(plan->max_m, probs[i].m);
        plan->uniform_d = plan->uniform_d && probs[i].d == plan->d;
    }
    plan->order.resize(count);
    for (int i = 0; i < count; ++i) plan->order[i] = i;
    // grouped by d (one launch each), largest first within a group
    std::stable_sort(plan->order.begin(), plan->order.end(), [&](int a, int c) {
        if (probs[a].d != probs[c].d) return probs[a].d < probs[c].d;
        return static_cast<long long>(probs[a].n) * probs[a].d > static_cast<long long>(probs[c].n) * probs[c].d;
    });
    if (!g_lds_ready[plan->device]) {
        HIP_TRY(rl0::batched_set_lds_limits());
        g_lds_ready[plan->device] = true;
    }
    return get_batch_buffers(plan->device, s, total, count, &plan->b);
}

size_t batch_lds(const BatchPlan& P);

// Workgroups of a persistent launch of column weight d that are resident at once under
// the schedule (its per_cu, capped by what the occupancy query says fits).
int batch_capacity(const BatchPlan& P, const rl0_batch_schedule& sc, int d) {
    hipDeviceProp_t prop;
    const int cus = hipGetDeviceProperties(&prop, P.device) == hipSuccess ? prop.multiProcessorCount : 256;
    const int fit = rl0::batched_max_resident(d, sc.block, batch_lds(P));
    const int per = fit > 0 ? std::min(sc.per_cu, fit) : sc.per_cu;
    return std::max(1, cus * per);
}

// The queue of one batched call: per instance its group size, the tickets (a group's
// consecutive), and per distinct d the range of tickets its launch takes and its grid.
struct BatchTickets {
    std::vector<int> group;       // per instance
    std::vector<int> tickets;
    struct Launch { int d, start, count, grid; };
    std::vector<Launch> launches;
};

// An instance's work, in arbitrary units, for the batch schedule.  A sweep's cost grows
// with the columns its consensus test queues, about n d / m columns per flagged row and
// flagged rows in proportion to the support, so n k / m per iteration (measured on one
// workgroup, the instance times follow n k / m more closely than n).
double instance_work(const rl0_problem& q, const DeviceConstants* dc) {
    const double per_it = static_cast<double>(q.n) * std::max(static_cast<double>(q.params.k) / q.m, 0.01);
    return per_it * dc->hc.n_iters;
}

// Group sizes and queue order of one launch (instances of one d).  An instance gets the
// smallest power-of-two group that brings its share of the work per member to half the
// average load of a resident workgroup (total work / resident workgroups), capped by the
// schedule's group for its size class, the resident grid and one member per 4096
// columns; so only the instances that would outlast the rest are split.  The queue then
// takes the instances by share per member, largest first (a group's tickets
// consecutive), so the long ones start at once.
BatchTickets make_tickets(const BatchPlan& P, const rl0_problem* probs, const rl0_batch_schedule& sc) {
    BatchTickets T;
    T.group.assign(P.count, 1);
    int start = 0;
    while (start < P.count) {
        const int d = probs[P.order[start]].d;
        const int cap = batch_capacity(P, sc, d);
        int end = start;
        double total = 0.0;
        for (; end < P.count && probs[P.order[end]].d == d; ++end) {
            const int i = P.order[end];
            total += instance_work(probs[i], P.dc[i]);
        }
        const double load = 0.5 * total / cap;
        std::vector<std::pair<double, int>> share;
        for (int e = start; e < end; ++e) {
            const int i = P.order[e];
            const double work = instance_work(probs[i], P.dc[i]);
            const int gmax = sc.group[size_class(probs[i].n)];
            int g = 1;
            while (g < gmax && 2 * g <= cap && static_cast<long long>(2 * g) * 4096 <= probs[i].n && work / g > load)
                g *= 2;
            T.group[i] = g;
            share.push_back({work / g, i});
        }
        std::stable_sort(share.begin(), share.end(), [](const auto& a, const auto& b) { return a.first > b.first; });
        const int t0 = static_cast<int>(T.tickets.size());
        for (const auto& sh : share)
            for (int p = 0; p < T.group[sh.second]; ++p) T.tickets.push_back(sh.second * rl0::kTicketParts + p);
        const int cnt = static_cast<int>(T.tickets.size()) - t0;
        T.launches.push_back({d, t0, cnt, std::max(1, std::min(cnt, cap))});
        start = end;
    }
    return T;
}

// Descriptors (with the schedule's columns per tile and group sizes) and the ticket queue
// to the device.
int upload_batch(const rl0_problem* probs, const BatchPlan& P, const rl0_batch_schedule& sc, hipStream_t s) {
    const MetaView h = meta_view(P.b->host, P.count);
    const MetaView dv = meta_view(P.b->meta, P.count);
    const BatchTickets T = make_tickets(P, probs, sc);
    char* ws = static_cast<char*>(P.b->block);
    for (int i = 0; i < P.count; ++i) {
        const rl0_problem& q = probs[i];
        const DeviceConstants* dc = P.dc[i];
        rl0::BatchProblem& B = h.desc[i];
        std::memset(&B, 0, sizeof(B));
        char* w = ws + P.offs[i];
        B.A = q.A_cols;
        B.y = q.y;
        B.x = q.x_out;
        B.S = reinterpret_cast<long long*>(w);
        w += rl0::al_host(8ull * q.m);
        B.r = reinterpret_cast<float*>(w);
        w += rl0::al_host(4ull * q.m);
        B.xp = reinterpret_cast<float*>(w);
        w += rl0::al_host(4ull * q.n);
        B.stamp = reinterpret_cast<int*>(w);
        w += rl0::al_host(4ull * q.n);
        B.chg = reinterpret_cast<int*>(w);
        w += rl0::al_host(4ull * q.n);
        B.chg2 = reinterpret_cast<int*>(w);
        w += rl0::al_host(4ull * q.n);
        B.keys = reinterpret_cast<unsigned long long*>(w);
        B.Tz = dc->d_tables;
        B.Te = dc->d_tables + rl0::kTableStrideFloats;
        B.tau = dc->d_tau;
        B.qe = dc->d_qe;
        B.qz = dc->d_qz;
        B.quant = dc->hc.quant ? 1 : 0;
        B.tol_fx = dc->hc.tol * 1073741824.0;
        B.n = q.n;
        B.m = q.m;
        B.d = q.d;
        B.k = q.params.k;
        B.alpha = q.params.alpha;
        B.inv_h_z = dc->hc.inv_h_z;
        B.inv_h_e = dc->hc.inv_h_e;
        B.exact = dc->hc.exact ? 1 : 0;
        B.e_zero_bits = dc->hc.e_zero_bits;
        B.l1_test = q.params.l1_test;
        B.validate = q.params.validate;
        B.n_iters = dc->hc.n_iters;
        B.cols = sc.cols[size_class(q.n)];
        B.group = T.group[i];
        B.ctl = dv.ctl + i;
    }
    std::memcpy(h.order, T.tickets.data(), sizeof(int) * T.tickets.size());
    HIP_TRY(hipMemcpyAsync(dv.desc, h.desc, sizeof(rl0::BatchProblem) * P.count, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(dv.order, h.order, sizeof(int) * T.tickets.size(), hipMemcpyHostToDevice, s));
    return RL0_OK;
}

size_t batch_lds(const BatchPlan& P) {
    // rounded up so that batches of similar sizes share a captured graph
    const int m = ((P.max_m + 32767) / 32768) * 32768;
    return rl0::batched_lds_bytes(std::min(m, rl0::kBatchMaxRows));
}

// The launch of a plan under a schedule: the LDS its per_cu workgroups per compute unit
// leave beside the tables and the bitmask holds the residual snapshot of instances with
// at most r_rows rows (the others gather it from global memory).  *lds_total <- the
// dynamic LDS per workgroup.
rl0::BatchLaunch batch_launch(const BatchPlan& P, const rl0_batch_schedule& sc, size_t* lds_total) {
    rl0::BatchLaunch L{sc.block, sc.per_cu};
    const size_t base = batch_lds(P);
    *lds_total = base;
    // the static LDS of the kernel, the largest over d (one launch per d shares this
    // dynamic size); queried once per block size (callers hold g_mu)
    static size_t st_cache[3] = {0, 0, 0};
    const int bi = sc.block == 256 ? 0 : sc.block == 512 ? 1 : sc.block == 1024 ? 2 : -1;
    if (bi < 0) return L;
    if (st_cache[bi] == 0) {
        size_t st = 0;
        for (int d = 1; d <= RL0_MAX_D; ++d) {
            const size_t sd = rl0::batched_static_lds(d, sc.block);
            if (sd == 0) return L;   // not queryable: no LDS snapshot
            st = std::max(st, sd);
        }
        st_cache[bi] = st;
    }
    const size_t st = st_cache[bi];
    const size_t share = (160u * 1024u) / static_cast<size_t>(std::max(1, sc.per_cu));
    long long rows = 0;
    if (share > st + base + 512) rows = static_cast<long long>((share - st - base - 512) / 4) & ~255ll;
    rows = std::min<long long>(rows, ((static_cast<long long>(P.max_m) + 255) / 256) * 256);
    if (rows < 1024) rows = 0;
    L.r_off = static_cast<int>(base / 4);
    L.r_rows = static_cast<int>(rows);
    *lds_total = base + 4 * static_cast<size_t>(rows);
    return L;
}

// Every launch of the plan (one per distinct d, in order), optionally timed; the groups'
// shared blocks are cleared first by a fill kernel.
int issue_batch(const BatchPlan& P, const rl0_batch_schedule& sc, const rl0_problem* probs, hipStream_t q,
                bool timed) {
    const MetaView dv = meta_view(P.b->meta, P.count);
    size_t lds = 0;
    const rl0::BatchLaunch L = batch_launch(P, sc, &lds);
    const BatchTickets T = make_tickets(P, probs, sc);
    HIP_TRY(rl0::launch_zero_words(reinterpret_cast<int*>(dv.ctl),
                                   static_cast<long long>(P.count) * (sizeof(rl0::BatchCtl) / sizeof(int)), q));
    for (size_t li = 0; li < T.launches.size(); ++li) {
        const BatchTickets::Launch& G = T.launches[li];
        HIP_TRY(rl0::launch_batched(G.d, L, G.grid, lds, dv.desc, dv.order + G.start, G.count, dv.res, dv.counter, q,
                                    timed && li == 0 ? P.b->ev[0] : nullptr,
                                    timed && li + 1 == T.launches.size() ? P.b->ev[1] : nullptr));
    }
    return RL0_OK;
}

int run_batch(const BatchPlan& P, const rl0_batch_schedule& sc, const rl0_problem* probs, hipStream_t s,
              bool timed) {
    if (timed || !P.uniform_d || !graphs_enabled()) return issue_batch(P, sc, probs, s, timed);
    BatchKey key;
    std::memset(&key, 0, sizeof(key));
    key.count = P.count;
    key.d = P.d;
    key.block = sc.block;
    key.per_cu = sc.per_cu;
    batch_launch(P, sc, &key.lds);
    key.meta = P.b->meta;
    {
        const BatchTickets T = make_tickets(P, probs, sc);
        uint64_t h = 1469598103934665603ull;   // FNV-1a over the launches
        for (const auto& G : T.launches)
            for (int v : {G.d, G.start, G.count, G.grid}) {
                h ^= static_cast<uint32_t>(v);
                h *= 1099511628211ull;
            }
        key.queue = h;
        key.grid = T.launches.empty() ? 0 : T.launches[0].grid;
    }
    BatchBuffers* b = P.b;
    BatchGraph* hit = nullptr;
    for (BatchGraph& g : b->graphs)
        if (std::memcmp(&g.key, &key, sizeof(key)) == 0) hit = &g;
    if (!hit) {
        if (!b->capture) HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeRelaxed));
        const int rc = issue_batch(P, sc, probs, b->capture, false);
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
            size_t lru = 0;
            for (size_t i = 1; i < b->graphs.size(); ++i)
                if (b->graphs[i].last_use < b->graphs[lru].last_use) lru = i;
            (void)hipGraphExecDestroy(b->graphs[lru].exec);
            b->graphs.erase(b->graphs.begin() + static_cast<std::ptrdiff_t>(lru));
        }
        BatchGraph g;
        g.key = key;
        g.exec = exec;
        b->graphs.push_back(g);
        hit = &b->graphs.back();
    }
    hit->last_use = ++b->uses;
    HIP_TRY(hipGraphLaunch(hit->exec, s));
    return RL0_OK;
}

// Results to the host (synchronising the stream) and into the stats; the first failed
// instance's code is returned.
int collect_batch(const rl0_problem* probs, const BatchPlan& P, rl0_stats* st, hipStream_t s) {
    const MetaView h = meta_view(P.b->host, P.count);
    const MetaView dv = meta_view(P.b->meta, P.count);
    HIP_TRY(hipMemcpyAsync(h.res, dv.res, sizeof(rl0::BatchResult) * P.count, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    P.b->last_res.assign(h.res, h.res + P.count);
    P.b->last_group.resize(P.count);
    for (int i = 0; i < P.count; ++i) P.b->last_group[i] = h.desc[i].group;
    float call_ms = -1.0f;
    if (st && hipEventElapsedTime(&call_ms, P.b->ev_call[0], P.b->ev_call[1]) != hipSuccess) {
        call_ms = -1.0f;
        (void)hipGetLastError();   // leave no error behind for the caller's next HIP call
    }
    int first_rc = RL0_OK;
    std::string first_msg;
    for (int i = 0; i < P.count; ++i) {
        const rl0::BatchResult& R = h.res[i];
        const DeviceConstants* dc = P.dc[i];
        if (st) {
            rl0_stats& o = st[i];
            o.iterations = R.iterations;
            o.accepted = R.accepted;
            o.l1_final_fx = R.L_hat;
            o.l1_final = static_cast<double>(R.L_hat) / 1073741824.0;
            o.l1_tol = dc->hc.tol;
            o.converged = (static_cast<double>(R.L_hat) <= dc->hc.tol * 1073741824.0) ? 1 : 0;
            o.updates_total = R.updates_total;
            o.t_final = R.iterations > 0 ? dc->hc.t[R.iterations - 1] : 1.0f;
            o.error_flags = R.err;
            o.ms_total = call_ms;   // the whole batched launch
            o.fx_inexact_y = R.inexact_y;
            o.fx_inexact_x = R.inexact_x;
            o.k_post = static_cast<double>(probs[i].params.k);
        }
        if (R.err && first_rc == RL0_OK) {
            first_rc = err_code_of(R.err);
            first_msg = "instance " + std::to_string(i) + ": " + g_last_error;
        }
    }
    if (first_rc != RL0_OK) return fail(first_rc, first_msg);
    return RL0_OK;
}

// Fills *st_h from a finished decode's device state (copied to the host) and the
// workspace's call events (both recorded on the decode's stream, now synchronised).
void fill_stats(rl0_stats* st_h, const rl0::DevState& ds, const rl0::Slot& fin, const DeviceConstants* dc,
                float t_final, Buffers* b, double k_post) {
    st_h->iterations = fin.iterations;
    st_h->accepted = fin.accepted;
    st_h->l1_final_fx = fin.L_hat;
    st_h->l1_final = static_cast<double>(fin.L_hat) / 1073741824.0;
    st_h->l1_tol = dc->hc.tol;
    st_h->converged = (static_cast<double>(fin.L_hat) <= dc->hc.tol * 1073741824.0) ? 1 : 0;
    st_h->updates_total = ds.updates_total;
    st_h->t_final = t_final;
    st_h->error_flags = ds.err;
    st_h->fx_inexact_y = ds.inexact_y;
    st_h->fx_inexact_x = ds.inexact_x;
    st_h->k_post = k_post;
    float ms = 0.0f;
    if (hipEventElapsedTime(&ms, b->ev_call[0], b->ev_call[1]) == hipSuccess) {
        st_h->ms_total = ms;
    } else {
        st_h->ms_total = -1.0f;
        (void)hipGetLastError();
    }
}

// ---------------------------------------------------------------- one iteration from x_hat

struct StepResult {
    int accepted = 0;
    int updates = 0;
    long long L_hat = 0;   // after the decision
    int cur = 0;           // buffer holding r_hat afterwards
};

// fl32(log(t / (1 - t))): the learned decision's threshold on the logit (+inf at t = 1).
float logit_threshold(float t) {
    if (!(t < 1.0f)) return INFINITY;
    return static_cast<float>(std::log(static_cast<double>(t) / (1.0 - static_cast<double>(t))));
}

// Iteration `it` of Alg. 1's loop from x_hat (device, updated in place when accepted):
// the residual is rebuilt from y and x_hat, the column decisions are the learned ones
// when `learned`, and the stream is synchronised.
int step_core(Buffers* b, const DeviceConstants* dc, const rl0::DecodeDims& dm, const int32_t* A, const float* y,
              const rl0_params* p, int it, bool learned, float* x_hat, const rl0::DebugOut& dbg, hipStream_t s,
              StepResult* out) {
    const rl0::Workspace& w = b->w;
    rl0::IterParams ip = iter_params(dc, p, it);
    ip.n_iters = it + 1;
    ip.tol_fx = -1.0;  // a single step never stops early
    rl0::IterParams ip_end = iter_params(dc, p, it + 1);
    ip_end.n_iters = it + 1;
    ip_end.tol_fx = -1.0;
    HIP_TRY(rl0::launch_prepare(dm, A, p->validate != 0, y, x_hat, w, ip, s));
    const float* lv = nullptr;
    if (learned) {
        rl0::LearnedCols lc{};
        lc.A = A;
        lc.n = dm.n;
        lc.m = dm.m;
        lc.d = dm.d;
        lc.r = w.r[0];
        lc.sigma = p->sigma;
        lc.logit_t = logit_threshold(ip.t);
        lc.w = static_cast<const float*>(p->mlp);
        lc.value = w.learned;
        const bool timed = g_prof.enabled;
        if (timed) {
            for (hipEvent_t& e : g_prof.learned_ev)
                if (!e) HIP_TRY(hipEventCreate(&e));
            HIP_TRY(hipEventRecord(g_prof.learned_ev[0], s));
        }
        HIP_TRY(rl0::launch_learned_cols(lc, s));
        if (timed) HIP_TRY(hipEventRecord(g_prof.learned_ev[1], s));
        lv = w.learned;
    }
    HIP_TRY(rl0::launch_iteration(dm, A, w, tables_of(dc), ip, dbg, s, nullptr, lv));
    HIP_TRY(rl0::launch_finish(dm, w, ip_end, x_hat, s));
    HIP_TRY(hipMemcpyAsync(b->st_host, w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (learned && g_prof.enabled) {
        float ms = 0.0f;
        HIP_TRY(hipEventElapsedTime(&ms, g_prof.learned_ev[0], g_prof.learned_ev[1]));
        g_prof.learned_ms += ms;
        g_prof.learned_launches += 1;
    }
    const rl0::DevState& ds = *b->st_host;
    if (int rc = err_code_of(ds.err)) return rc;
    const rl0::Slot& fin = ds.slot[(it + 1) & 1];
    b->last_log_count = p->log ? fin.iterations : 0;
    out->accepted = fin.accepted_last;
    out->L_hat = fin.L_hat;
    out->cur = fin.cur;
    out->updates = ds.updates_total;
    return RL0_OK;
}

// Alg. 1 with the learned column decision: at each t a learned iteration, and when it
// is not accepted, an iteration with the analytic decision at the same t.  The whole
// decode stays on the device: t-step j is sub-iteration 2j (learned) and 2j + 1 (the
// analytic retry, which the sweep skips when 2j was accepted).  The learned decisions
// of 2j need r_hat after the decision on 2j - 1, which a one-workgroup kernel evaluates
// ahead; the sweep of 2j takes the same decision again.
rl0::IterParams learned_sub_params(const DeviceConstants* dc, const rl0_params* p, int u) {
    const int N = dc->hc.n_iters;
    rl0::IterParams ip = iter_params(dc, p, u >> 1);
    ip.tau_next = iter_params(dc, p, (u + 1) >> 1).tau_bits;   // the next sweep's t
    ip.it = u;
    ip.n_iters = 2 * N;
    ip.step = u >> 1;
    ip.retry = u & 1;
    return ip;
}

int decode_learned(Buffers* b, const DeviceConstants* dc, const rl0::DecodeDims& dm, const int32_t* A,
                   const float* y, const rl0_params* p, float* x_out, rl0_stats* st_h, hipStream_t s) {
    const rl0::ScoreTables tb = tables_of(dc);
    const int N = dc->hc.n_iters;
    const rl0::Workspace& w = b->w;
    const float* mlp = static_cast<const float*>(p->mlp);
    auto issue = [&](hipStream_t q, const float* yq, float* xq) -> int {
        HIP_TRY(rl0::launch_prepare(dm, A, p->validate != 0, yq, nullptr, w, learned_sub_params(dc, p, 0), q, xq));
        const rl0::DebugOut dbg{nullptr, nullptr};
        for (int j = 0; j < N; ++j) {
            const rl0::IterParams ipl = learned_sub_params(dc, p, 2 * j);
            HIP_TRY(rl0::launch_peek(w, ipl, q));
            // columns whose residual entries are unchanged since the last t keep the
            // network's outputs of then
            rl0::LearnedCols lc{};
            lc.A = A;
            lc.n = dm.n;
            lc.m = dm.m;
            lc.d = dm.d;
            lc.r = w.r[0];
            lc.r1 = w.r[1];
            lc.pick = &w.st->peek_cur;
            lc.reval_in = j > 0 ? w.reval[(j + 1) & 1] : nullptr;
            lc.reval_out = w.reval[j & 1];
            lc.cache = w.lcache;
            lc.sigma = p->sigma;
            lc.logit_t = logit_threshold(ipl.t);
            lc.w = mlp;
            lc.value = w.learned;
            HIP_TRY(rl0::launch_learned_cols(lc, q));
            HIP_TRY(rl0::launch_iteration(dm, A, w, tb, ipl, dbg, q, nullptr, w.learned));
            HIP_TRY(rl0::launch_iteration(dm, A, w, tb, learned_sub_params(dc, p, 2 * j + 1), dbg, q));
        }
        HIP_TRY(rl0::launch_finish(dm, w, learned_sub_params(dc, p, 2 * N), xq, q, true));
        return RL0_OK;
    };
    if (st_h) HIP_TRY(hipEventRecord(b->ev_call[0], s));
    if (graphs_enabled()) {
        DecodeKey key;
        std::memset(&key, 0, sizeof(key));
        key.A = A;
        key.dc = dc;
        key.n = dm.n;
        key.m = dm.m;
        key.d = dm.d;
        params_key(p, &key.p);
        if (int rc = replay_decode_io(b, key, y, x_out, dm.n, dm.m, s, issue)) return rc;
    } else {
        if (int rc = issue(s, y, x_out)) return rc;
    }
    if (st_h) HIP_TRY(hipEventRecord(b->ev_call[1], s));
    HIP_TRY(hipMemcpyAsync(b->st_host, w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const rl0::DevState& ds = *b->st_host;
    const rl0::Slot& fin = ds.slot[0];   // sub-iteration 2N decides last
    b->last_log_count = p->log ? fin.iterations : 0;
    if (st_h) fill_stats(st_h, ds, fin, dc, fin.iterations > 0 ? dc->hc.t[fin.t_step] : 1.0f, b, p->k);
    return err_code_of(ds.err);
}

// ---------------------------------------------------------------- network training memory

// Alg. 1 with the adaptive_k branch.  After iteration it the decision on it (evaluated
// ahead by launch_peek) and sum_j rint(2^30 fl32(1 - Tz(|x_hat_j|))) over the x_hat that
// acceptance would give are read back; when accepted, the posteriors' sparsity becomes
// k_0 = max(k - 2^-30 sum, floor(m/100), 1) and the constants of every later iteration are
// recomputed with rho = k_0/m (the t-sweep and c stay, being functions of k).  The
// outer-test bitmask of the residual the next sweep starts from was built with the old
// threshold tau_{it+1}; it is redone with the new one.  The launches of it + 1 depend on a
// value read back after it, so the decode is launched eagerly, one host round trip per
// iteration.
int decode_adaptive(Buffers* b, const DeviceConstants* dc0, const rl0::Problem& pr0, const rl0::DecodeDims& dm,
                    const int32_t* A, const float* y, const rl0_params* p, float* x_out, rl0_stats* st_h,
                    hipStream_t s) {
    const rl0::Workspace& w = b->w;
    const int N = dc0->hc.n_iters;
    const rl0::DebugOut dbg{nullptr, nullptr};
    const DeviceConstants* dc = dc0;
    rl0::Problem pr = pr0;
    double k_post = static_cast<double>(p->k);
    const double k_floor = std::max(static_cast<double>(dm.m / 100), 1.0);
    if (st_h) HIP_TRY(hipEventRecord(b->ev_call[0], s));
    HIP_TRY(rl0::launch_prepare(dm, A, p->validate != 0, y, nullptr, w, iter_params(dc, p, 0), s, x_out));
    int it_end = N;
    for (int it = 0; it < N; ++it) {
        HIP_TRY(rl0::launch_iteration(dm, A, w, tables_of(dc), iter_params(dc, p, it), dbg, s, profile_events(it)));
        if (it + 1 == N) break;
        HIP_TRY(rl0::launch_peek(w, iter_params(dc, p, it + 1), s));
        HIP_TRY(rl0::launch_adapt_sum(w, tables_of(dc), it, s));
        HIP_TRY(hipMemcpyAsync(b->st_host, w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        const rl0::DevState& ds = *b->st_host;
        if (ds.peek_done) {   // stopped (converged, or an error flag): the decision is final
            it_end = it + 1;
            break;
        }
        if (!ds.peek_acc) continue;
        const double k0 = std::max(static_cast<double>(p->k) - static_cast<double>(ds.adapt_sum) * 0x1p-30, k_floor);
        if (k0 == k_post) continue;
        k_post = k0;
        pr.k_post = k0;
        const uint32_t tau_old = dc->hc.tau_bits[it + 1];
        if (!b->adapted) b->adapted = std::make_unique<DeviceConstants>();
        // every launch that read the previous constants has completed (the stream is
        // synchronised), so the one set is rewritten in place
        if (!rl0::compute_constants(pr, &b->adapted->hc)) return fail(RL0_EINVAL, "adaptive_k: constants failed");
        if (int rc = upload_constants(b->adapted.get())) return rc;
        dc = b->adapted.get();
        if (dc->hc.tau_bits[it + 1] != tau_old)
            HIP_TRY(rl0::launch_rebuild_outer(dm, w, ds.peek_cur, dc->hc.tau_bits[it + 1], it, s));
    }
    HIP_TRY(rl0::launch_finish(dm, w, iter_params(dc, p, it_end), x_out, s, true));
    if (st_h) HIP_TRY(hipEventRecord(b->ev_call[1], s));
    HIP_TRY(hipMemcpyAsync(b->st_host, w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const rl0::DevState& ds = *b->st_host;
    const rl0::Slot& fin = ds.slot[it_end & 1];
    b->last_log_count = p->log ? fin.iterations : 0;
    profile_collect(it_end, fin.iterations, dm.m > rl0::kPreRows);
    if (st_h) fill_stats(st_h, ds, fin, dc, fin.iterations > 0 ? dc->hc.t[fin.iterations - 1] : 1.0f, b, k_post);
    return err_code_of(ds.err);
}

struct MlpBuffers {
    float* grad = nullptr;
    float* losses = nullptr;
    float* part = nullptr;             // the gradient kernel's per-workgroup shares
    size_t cap_p = 0, cap_steps = 0, cap_part = 0;
    std::vector<float> host_losses;
};

std::map<std::pair<int, hipStream_t>, MlpBuffers> g_mlp;

// Gradient, per-step losses and the gradient kernel's scratch for column weight d.
int get_mlp_buffers(int device, hipStream_t s, int d, size_t steps, MlpBuffers** out) {
    MlpBuffers& mb = g_mlp[{device, s}];
    const size_t P = static_cast<size_t>(rl0::mlp_params(d)), part = rl0::mlp_grad_scratch_floats(d);
    if (mb.cap_p < P || mb.cap_steps < steps || mb.cap_part < part) {
        HIP_TRY(hipStreamSynchronize(s));
        const size_t np = std::max(P, mb.cap_p), ns = std::max<size_t>(std::max(steps, mb.cap_steps), 1),
                     nq = std::max(part, mb.cap_part);
        if (mb.grad) HIP_TRY(hipFree(mb.grad));
        mb.grad = nullptr;
        mb.cap_p = mb.cap_steps = mb.cap_part = 0;
        if (hipMalloc(&mb.grad, sizeof(float) * (np + ns + nq)) != hipSuccess) return fail(RL0_ENOMEM, "hipMalloc(mlp)");
        mb.losses = mb.grad + np;
        mb.part = mb.losses + ns;
        mb.cap_p = np;
        mb.cap_steps = ns;
        mb.cap_part = nq;
    }
    *out = &mb;
    return RL0_OK;
}

// Training checkpoints (rl0_mlp_save, rl0_mlp_load).
static_assert(__BYTE_ORDER__ == __ORDER_LITTLE_ENDIAN__, "the checkpoint layout is little-endian");

constexpr char kCkptMagic[8] = {'R', 'L', '0', 'M', 'L', 'P', 'C', 'K'};
constexpr uint32_t kCkptVersion = 1;
constexpr size_t kCkptHeader = 80;

// CRC-32 of IEEE 802.3 (reflected polynomial 0xEDB88320, initial and final complement),
// the checksum zlib computes.
uint32_t crc32_ieee(const unsigned char* p, size_t n) {
    static const std::array<uint32_t, 256> table = [] {
        std::array<uint32_t, 256> t{};
        for (uint32_t i = 0; i < 256; ++i) {
            uint32_t c = i;
            for (int b = 0; b < 8; ++b) c = (c & 1u) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
            t[i] = c;
        }
        return t;
    }();
    uint32_t crc = 0xFFFFFFFFu;
    for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xFFu] ^ (crc >> 8);
    return ~crc;
}

template <class T>
void put_le(unsigned char* b, size_t off, T v) { std::memcpy(b + off, &v, sizeof(T)); }

template <class T>
T get_le(const unsigned char* b, size_t off) {
    T v;
    std::memcpy(&v, b + off, sizeof(T));
    return v;
}

bool ckpt_cfg_ok(const rl0_train_cfg& c) {
    return std::isfinite(c.lr) && std::isfinite(c.beta1) && std::isfinite(c.beta2) && std::isfinite(c.eps) &&
           std::isfinite(c.lam) && c.batch >= 1;
}

int ckpt_fail(const char* path, const std::string& why) {
    return fail(RL0_EIO, std::string("checkpoint ") + path + ": " + why);
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
    if (!rl0::compute_constants(problem_of(p, n, m, d), &hc))
        return fail(RL0_EINVAL, "the posteriors of these signal and noise laws could not be tabulated");
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

int rl0_validate_host(const int32_t* A_cols_h, int32_t n, int32_t m, int32_t d) {
    if (int rc = check_dims(n, m, d)) return rc;
    if (!A_cols_h) return fail(RL0_EINVAL, "A_cols_h is NULL");
    for (int64_t j = 0; j < n; ++j) {
        int prev = -1;
        for (int p = 0; p < d; ++p) {
            const int r = A_cols_h[j * d + p];
            if (r <= prev || r >= m) return fail(RL0_EINDEX, "column " + std::to_string(j) + " is malformed");
            prev = r;
        }
    }
    return RL0_OK;
}

size_t rl0_workspace_bytes(int32_t n, int32_t m, int32_t d, int32_t k) {
    if (n < 1 || m < 1 || d < 1 || d > RL0_MAX_D || d > m || k < 1 || k >= m) return 0;
    return rl0::workspace_bytes(n, m);
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
    HIP_TRY(hipMemcpyAsync(b->st_host, b->w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
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
    // the flags lead the device state
    HIP_TRY(hipMemcpyAsync(b->st_host, b->w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return err_code_of(b->st_host->err);
}

int rl0_sketch_static(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* x, float* y,
                      void* stream) {
    static_assert(RL0_SKETCH_STATIC_MAX_M == rl0::kStaticSketchRows, "scratch rows");
    if (int rc = check_dims(n, m, d)) return rc;
    if (!A_cols || !x || !y) return fail(RL0_EINVAL, "NULL pointer");
    if (m > RL0_SKETCH_STATIC_MAX_M) return fail(RL0_EINVAL, "m exceeds RL0_SKETCH_STATIC_MAX_M");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    long long* scr = nullptr;
    HIP_TRY(rl0::static_scratch(&scr));
    int* err = reinterpret_cast<int*>(scr + rl0::kStaticSketchRows);
    HIP_TRY(rl0::launch_zero_i32(err, 1, s));   // the flags keep the last call's value
    HIP_TRY(rl0::launch_sketch(A_cols, n, m, d, x, y, scr, err, s));
    int flags = 0;
    HIP_TRY(hipMemcpyAsync(&flags, err, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return err_code_of(flags);
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
    if (p->posterior == 1) return decode_learned(b, dc, dm, A_cols, y, p, x_out, st_h, s);
    if (p->adaptive_k == 1 && !dc->hc.exact) return decode_adaptive(b, dc, problem_of(p, n, m, d), dm, A_cols, y, p, x_out, st_h, s);
    const rl0::ScoreTables tb = tables_of(dc);
    const int N = dc->hc.n_iters;
    auto issue = [&](hipStream_t q, const float* yq, float* xq) -> int {
        HIP_TRY(rl0::launch_prepare(dm, A_cols, p->validate != 0, yq, nullptr, b->w, iter_params(dc, p, 0), q, xq));
        const rl0::DebugOut dbg{nullptr, nullptr};
        for (int it = 0; it < N; ++it)
            HIP_TRY(rl0::launch_iteration(dm, A_cols, b->w, tb, iter_params(dc, p, it), dbg, q, profile_events(it)));
        HIP_TRY(rl0::launch_finish(dm, b->w, iter_params(dc, p, N), xq, q, true));
        return RL0_OK;
    };
    if (st_h) HIP_TRY(hipEventRecord(b->ev_call[0], s));
    // per-iteration timing events cannot be recorded into a captured graph: a profiled
    // decode launches eagerly
    if (graphs_enabled() && !g_prof.enabled) {
        DecodeKey key;
        std::memset(&key, 0, sizeof(key));
        key.A = A_cols;
        key.dc = dc;
        key.n = n;
        key.m = m;
        key.d = d;
        params_key(p, &key.p);
        if (int rc = replay_decode_io(b, key, y, x_out, n, m, s, issue)) return rc;
    } else {
        if (int rc = issue(s, y, x_out)) return rc;
    }
    if (st_h) HIP_TRY(hipEventRecord(b->ev_call[1], s));
    // the slots, counters and flags lead the device state
    HIP_TRY(hipMemcpyAsync(b->st_host, b->w.st, offsetof(rl0::DevState, seg_count), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    const rl0::DevState& ds = *b->st_host;
    const rl0::Slot& fin = ds.slot[N & 1];
    b->last_log_count = p->log ? fin.iterations : 0;
    profile_collect(N, fin.iterations, m > rl0::kPreRows);
    if (st_h) fill_stats(st_h, ds, fin, dc, fin.iterations > 0 ? dc->hc.t[fin.iterations - 1] : 1.0f, b, p->k);
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
    if (p->adaptive_k) return fail(RL0_EINVAL, "adaptive_k applies to whole decodes (rl0_decode)");
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
    if (updated) HIP_TRY(rl0::launch_zero_i32(updated, n, s));
    if (omega) HIP_TRY(rl0::launch_zero_f32(omega, n, s));
    const rl0::DebugOut dbg{updated, omega};
    StepResult r;
    if (int rc = step_core(b, dc, dm, A_cols, y, p, it, p->posterior == 1, x_hat, dbg, s, &r)) return rc;
    // the iteration ran from buffer 0; its trial iterate sits in buffer 1
    if (x_trial) HIP_TRY(rl0::launch_trial_out(dm, w, it + 1, x_trial, s));
    if (r_trial) HIP_TRY(rl0::launch_copy_f32(w.r[1], r_trial, m, s));
    if (accepted_h) *accepted_h = r.accepted;
    *L_hat_h = r.L_hat;
    HIP_TRY(rl0::launch_copy_f32(w.r[r.cur], r_hat, m, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RL0_OK;
}

int rl0_decode_batched(const rl0_problem* probs_h, int32_t count, rl0_stats* st_h, void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchPlan plan;
    if (int rc = plan_batch(probs_h, count, s, &plan)) return rc;
    if (count == 0) return RL0_OK;
    const rl0_batch_schedule sc = schedule_of(plan.device);
    if (int rc = upload_batch(probs_h, plan, sc, s)) return rc;
    HIP_TRY(hipEventRecord(plan.b->ev_call[0], s));
    if (int rc = run_batch(plan, sc, probs_h, s, false)) return rc;
    HIP_TRY(hipEventRecord(plan.b->ev_call[1], s));
    return collect_batch(probs_h, plan, st_h, s);
}

int rl0_batch_timeline(int32_t count, double* start_ms_h, double* end_ms_h, int32_t* group_h, void* stream) {
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto it = g_bws.find({dev, static_cast<hipStream_t>(stream)});
    if (it == g_bws.end() || !it->second) return fail(RL0_EINVAL, "no batched decode on this device and stream");
    const BatchBuffers& b = *it->second;
    if (count < 0 || static_cast<size_t>(count) > b.last_res.size())
        return fail(RL0_EINVAL, "count exceeds the last batch's instances");
    int khz = 0;
    HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
    const double ms_per_tick = khz > 0 ? 1.0 / khz : 1e-5;
    unsigned long long t0 = ~0ull;
    for (const auto& r : b.last_res) t0 = std::min(t0, r.t_start);
    for (int i = 0; i < count; ++i) {
        const rl0::BatchResult& r = b.last_res[i];
        if (start_ms_h) start_ms_h[i] = static_cast<double>(r.t_start - t0) * ms_per_tick;
        if (end_ms_h) end_ms_h[i] = static_cast<double>(r.t_end - t0) * ms_per_tick;
        if (group_h) group_h[i] = b.last_group[i];
    }
    return RL0_OK;
}

int rl0_batch_schedule_get(rl0_batch_schedule* out_h) {
    if (!out_h) return fail(RL0_EINVAL, "out_h is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    *out_h = schedule_of(dev);
    return RL0_OK;
}

int rl0_batch_schedule_set(const rl0_batch_schedule* s_h) {
    if (!s_h) return fail(RL0_EINVAL, "s_h is NULL");
    if (int rc = check_schedule(*s_h)) return rc;
    std::lock_guard<std::mutex> lk(g_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    schedule_of(dev) = *s_h;
    return RL0_OK;
}

int rl0_autotune_batched(const rl0_problem* probs_h, int32_t count, int32_t reps, rl0_batch_schedule* best_h,
                         double* ms_h, void* stream) {
    if (reps < 1) return fail(RL0_EINVAL, "reps must be >= 1");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    BatchPlan plan;
    if (int rc = plan_batch(probs_h, count, s, &plan)) return rc;
    if (count == 0) return fail(RL0_EINVAL, "nothing to tune on: count is 0");
    // median time of the persistent launches under a schedule
    auto time_of = [&](const rl0_batch_schedule& sc, double* ms) -> int {
        if (int rc = upload_batch(probs_h, plan, sc, s)) return rc;
        std::vector<double> t;
        for (int r = 0; r < reps; ++r) {
            if (int rc = run_batch(plan, sc, probs_h, s, true)) return rc;
            HIP_TRY(hipStreamSynchronize(s));
            float e = 0.0f;
            HIP_TRY(hipEventElapsedTime(&e, plan.b->ev[0], plan.b->ev[1]));
            t.push_back(e);
        }
        std::sort(t.begin(), t.end());
        *ms = t[t.size() / 2];
        return RL0_OK;
    };
    rl0_batch_schedule best = schedule_of(plan.device);
    double best_ms = 0.0;
    if (int rc = time_of(best, &best_ms)) return rc;
    // 1. launch shape, over the shapes the device can hold
    const size_t lds = batch_lds(plan);
    for (int block : {256, 512, 1024}) {
        const int fit = rl0::batched_max_resident(plan.d, block, lds);
        for (int per_cu : {1, 2, 3, 4, 6, 8}) {
            if (per_cu > fit) continue;
            rl0_batch_schedule c = best;
            c.block = block;
            c.per_cu = per_cu;
            if (c.block == best.block && c.per_cu == best.per_cu) continue;
            double ms = 0.0;
            if (int rc = time_of(c, &ms)) return rc;
            if (ms < best_ms) {
                best = c;
                best_ms = ms;
            }
        }
    }
    std::vector<long long> cls_cols(RL0_SIZE_CLASSES, 0);
    for (int i = 0; i < count; ++i) cls_cols[size_class(probs_h[i].n)] += probs_h[i].n;
    std::vector<int> cls;
    for (int c = 0; c < RL0_SIZE_CLASSES; ++c)
        if (cls_cols[c] > 0) cls.push_back(c);
    // 2. the cap on workgroups per instance (which instances are split, and how far, follows
    // from their work against the average load), first for every class at once, then
    // lowered class by class, the largest first
    for (int g : {2, 4, 8, 16}) {
        rl0_batch_schedule cand = best;
        for (int c = 0; c < RL0_SIZE_CLASSES; ++c) cand.group[c] = g;
        double ms = 0.0;
        if (int rc = time_of(cand, &ms)) return rc;
        if (ms < best_ms) {
            best = cand;
            best_ms = ms;
        }
    }
    for (int c = RL0_SIZE_CLASSES - 1; c >= 0; --c) {
        if (cls_cols[c] == 0 || best.group[c] == 1) continue;
        for (int g = best.group[c] / 2; g >= 1; g /= 2) {
            rl0_batch_schedule cand = best;
            cand.group[c] = g;
            double ms = 0.0;
            if (int rc = time_of(cand, &ms)) return rc;
            if (ms < best_ms) {
                best = cand;
                best_ms = ms;
            }
        }
    }
    // 3. columns per tile, size class by size class, the classes with most columns first
    std::stable_sort(cls.begin(), cls.end(), [&](int a, int b) { return cls_cols[a] > cls_cols[b]; });
    for (int c : cls) {
        for (int cols : {1, 2, 4}) {
            if (cols == best.cols[c]) continue;
            rl0_batch_schedule cand = best;
            cand.cols[c] = cols;
            double ms = 0.0;
            if (int rc = time_of(cand, &ms)) return rc;
            if (ms < best_ms) {
                best = cand;
                best_ms = ms;
            }
        }
    }
    schedule_of(plan.device) = best;
    if (best_h) *best_h = best;
    if (ms_h) *ms_h = best_ms;
    // leave every x_out holding the decode under the installed schedule
    if (int rc = upload_batch(probs_h, plan, best, s)) return rc;
    if (int rc = run_batch(plan, best, probs_h, s, false)) return rc;
    return collect_batch(probs_h, plan, nullptr, s);
}

int32_t rl0_mlp_num_params(int32_t d) { return d >= 1 && d <= RL0_MAX_D ? rl0::mlp_params(d) : -1; }

int rl0_mlp_pack_bf16(const float* w_h, int32_t d, uint16_t* packed_h) {
    if (!w_h || !packed_h) return fail(RL0_EINVAL, "NULL pointer");
    if (d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "d must be in [1, 16]");
    const int P = rl0::mlp_params(d);
    for (int i = 0; i < P; ++i) {
        uint32_t u;
        std::memcpy(&u, &w_h[i], 4);
        if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu)) {
            packed_h[i] = static_cast<uint16_t>((u >> 16) | 0x0040u);   // NaN stays NaN
        } else {
            const uint32_t lsb = (u >> 16) & 1u;   // round to nearest, ties to even
            packed_h[i] = static_cast<uint16_t>((u + 0x7FFFu + lsb) >> 16);
        }
    }
    return RL0_OK;
}

int rl0_mlp_init(float* w, int32_t d, uint64_t seed, void* stream) {
    if (!w) return fail(RL0_EINVAL, "w is NULL");
    if (d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "d must be in [1, 16]");
    const int F = d + 1, H = rl0::kHidden;
    std::vector<float> h(rl0::mlp_params(d), 0.0f);
    uint64_t st = seed;
    auto next = [&]() {   // SplitMix64
        uint64_t z = (st += 0x9E3779B97F4A7C15ull);
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    };
    size_t o = 0;
    const int shapes[3][2] = {{H, F}, {H, H}, {2, H}};
    for (const auto& sh : shapes) {
        const double bound = std::sqrt(3.0 / sh[1]);
        for (int i = 0; i < sh[0] * sh[1]; ++i) {
            const double u = static_cast<double>(next() >> 11) * (1.0 / 9007199254740992.0);
            h[o++] = static_cast<float>((2.0 * u - 1.0) * bound);
        }
        o += sh[0];   // biases stay 0
    }
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIP_TRY(hipMemcpyAsync(w, h.data(), sizeof(float) * h.size(), hipMemcpyHostToDevice, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RL0_OK;
}

int rl0_mlp_features(const int32_t* A_cols, int32_t n, int32_t m, int32_t d, const float* r, float sigma,
                     float* feats, void* stream) {
    if (int rc = check_dims(n, m, d)) return rc;
    if (!A_cols || !r || !feats) return fail(RL0_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    HIP_TRY(rl0::launch_mlp_features(A_cols, n, m, d, r, sigma, feats, static_cast<hipStream_t>(stream)));
    return RL0_OK;
}

int rl0_mlp_labels(const float* x_true, const float* x_hat, int32_t n, int32_t d, float sigma, float* labels,
                   void* stream) {
    if (n < 1 || d < 1) return fail(RL0_EINVAL, "n and d must be >= 1");
    if (!x_true || !x_hat || !labels) return fail(RL0_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    const double thr = 3.0 * static_cast<double>(sigma) / std::sqrt(static_cast<double>(d));
    HIP_TRY(rl0::launch_mlp_labels(x_true, x_hat, n, thr, labels, static_cast<hipStream_t>(stream)));
    return RL0_OK;
}

int rl0_mlp_grad(const float* feats, const float* labels, int32_t N, int32_t d, const float* w, float lam,
                 float* grad, float* loss_h, void* stream) {
    if (N < 1 || d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "N >= 1 and d in [1, 16] required");
    if (!feats || !labels || !w || !grad) return fail(RL0_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    MlpBuffers* mb = nullptr;
    if (int rc = get_mlp_buffers(dev, s, d, 1, &mb)) return rc;
    HIP_TRY(rl0::launch_mlp_grad(feats, labels, N, d, w, lam, grad, mb->losses, mb->part, s));
    float l = 0.0f;
    HIP_TRY(hipMemcpyAsync(&l, mb->losses, sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (loss_h) *loss_h = l;
    return RL0_OK;
}

int rl0_mlp_train(const float* feats, const float* labels, int64_t N, int32_t d, float* w, float* adam_m,
                  float* adam_v, const rl0_train_cfg* cfg, float* loss_h, void* stream) {
    if (!cfg) return fail(RL0_EINVAL, "cfg is NULL");
    if (d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "d must be in [1, 16]");
    if (cfg->batch < 1 || cfg->steps < 0 || cfg->t0 < 0 || N < cfg->batch)
        return fail(RL0_EINVAL, "need batch >= 1, steps >= 0, t0 >= 0 and N >= batch");
    if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
        !(cfg->eps > 0.0f))
        return fail(RL0_EINVAL, "Adam settings out of range");
    if (!feats || !labels || !w || !adam_m || !adam_v) return fail(RL0_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    const int F = d + 1;
    MlpBuffers* mb = nullptr;
    if (int rc = get_mlp_buffers(dev, s, d, cfg->steps, &mb)) return rc;
    const int64_t nb = N / cfg->batch;
    for (int i = 0; i < cfg->steps; ++i) {
        const int64_t blk = (static_cast<int64_t>(cfg->t0) + i) % nb;
        const size_t off = static_cast<size_t>(blk) * cfg->batch;
        const double t = static_cast<double>(cfg->t0) + i + 1;
        const float c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta1), t));
        const float c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta2), t));
        const rl0::AdamStep adam{w, adam_m, adam_v, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, c1, c2};
        HIP_TRY(rl0::launch_mlp_grad(feats + off * F, labels + off * 2, cfg->batch, d, w, cfg->lam, mb->grad,
                                     mb->losses + i, mb->part, s, &adam));
    }
    if (cfg->steps > 0) {
        mb->host_losses.resize(cfg->steps);
        HIP_TRY(hipMemcpyAsync(mb->host_losses.data(), mb->losses, sizeof(float) * cfg->steps, hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    if (loss_h) {
        const int tail = std::min(cfg->steps, 50);
        double acc = 0.0;
        for (int i = cfg->steps - tail; i < cfg->steps; ++i) acc += mb->host_losses[i];
        *loss_h = tail > 0 ? static_cast<float>(acc / tail) : 0.0f;
    }
    return RL0_OK;
}

int rl0_mlp_adam(float* w, const float* grad, float* adam_m, float* adam_v, int32_t d, int32_t t,
                 const rl0_train_cfg* cfg, void* stream) {
    if (!cfg) return fail(RL0_EINVAL, "cfg is NULL");
    if (d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "d must be in [1, 16]");
    if (t < 1) return fail(RL0_EINVAL, "t must be >= 1");
    if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) || !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) ||
        !(cfg->eps > 0.0f))
        return fail(RL0_EINVAL, "Adam settings out of range");
    if (!w || !grad || !adam_m || !adam_v) return fail(RL0_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    const float c1 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta1), static_cast<double>(t)));
    const float c2 = static_cast<float>(1.0 - std::pow(static_cast<double>(cfg->beta2), static_cast<double>(t)));
    HIP_TRY(rl0::launch_mlp_adam(w, grad, adam_m, adam_v, rl0::mlp_params(d), cfg->lr, cfg->beta1, cfg->beta2, cfg->eps,
                                 c1, c2, s));
    HIP_TRY(hipStreamSynchronize(s));
    return RL0_OK;
}

int rl0_mlp_forward(const float* feats, int32_t N, int32_t d, const float* w, float* out, int32_t bf16,
                    void* stream) {
    if (N < 1 || d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "N >= 1 and d in [1, 16] required");
    if (bf16 && d + 1 > rl0::kMlpMaxFeatures) return fail(RL0_EINVAL, "bf16 inference supports d <= 15");
    if (!feats || !w || !out) return fail(RL0_EINVAL, "NULL pointer");
    std::lock_guard<std::mutex> lk(g_mu);
    HIP_TRY(rl0::launch_mlp_forward(feats, N, d, w, out, bf16 ? 1 : 0, static_cast<hipStream_t>(stream)));
    return RL0_OK;
}

// ---------------------------------------------------------------- training checkpoints

int rl0_mlp_save(const char* path_h, const rl0_mlp_ckpt* info_h, const float* w, const float* adam_m,
                 const float* adam_v, void* stream) {
    if (!path_h || !info_h || !w || !adam_m || !adam_v) return fail(RL0_EINVAL, "NULL pointer");
    const int32_t d = info_h->d;
    if (d < 1 || d > RL0_MAX_D) return fail(RL0_EINVAL, "d must be in [1, 16]");
    if (info_h->step < 0) return fail(RL0_EINVAL, "step must be >= 0");
    const rl0_train_cfg& c = info_h->cfg;
    if (!ckpt_cfg_ok(c)) return fail(RL0_EINVAL, "cfg: finite hyper-parameters and batch >= 1 required");
    const size_t P = static_cast<size_t>(rl0::mlp_params(d));
    std::vector<unsigned char> buf(kCkptHeader + 12 * P, 0);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const float* arrays[3] = {w, adam_m, adam_v};
    for (int a = 0; a < 3; ++a)
        HIP_TRY(hipMemcpyAsync(buf.data() + kCkptHeader + a * 4 * P, arrays[a], 4 * P, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));

    unsigned char* h = buf.data();
    std::memcpy(h, kCkptMagic, 8);
    put_le<uint32_t>(h, 8, kCkptVersion);
    put_le<uint32_t>(h, 12, 0);
    put_le<int32_t>(h, 16, d);
    put_le<int32_t>(h, 20, c.batch);
    put_le<int64_t>(h, 24, static_cast<int64_t>(P));
    put_le<uint64_t>(h, 32, info_h->seed);
    put_le<int64_t>(h, 40, info_h->step);
    const float hp[5] = {c.lr, c.beta1, c.beta2, c.eps, c.lam};
    for (int i = 0; i < 5; ++i) put_le<float>(h, 48 + 4 * i, hp[i]);
    put_le<uint32_t>(h, 68, crc32_ieee(h + kCkptHeader, 12 * P));
    put_le<uint32_t>(h, 72, crc32_ieee(h, 72));

    const std::string tmp = std::string(path_h) + ".tmp";
    std::FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f) return ckpt_fail(path_h, "cannot open " + tmp + " for writing: " + std::strerror(errno));
    const size_t wrote = std::fwrite(buf.data(), 1, buf.size(), f);
    const bool flushed = std::fflush(f) == 0 && fsync(fileno(f)) == 0;
    const bool closed = std::fclose(f) == 0;
    if (wrote != buf.size() || !flushed || !closed) {
        std::remove(tmp.c_str());
        return ckpt_fail(path_h, "writing " + tmp + " failed");
    }
    if (std::rename(tmp.c_str(), path_h) != 0) {
        const std::string why = std::strerror(errno);
        std::remove(tmp.c_str());
        return ckpt_fail(path_h, "cannot rename " + tmp + ": " + why);
    }
    return RL0_OK;
}

int rl0_mlp_load(const char* path_h, rl0_mlp_ckpt* info_h, float* w, float* adam_m, float* adam_v, void* stream) {
    if (!path_h) return fail(RL0_EINVAL, "path is NULL");
    std::FILE* f = std::fopen(path_h, "rb");
    if (!f) return ckpt_fail(path_h, std::string("cannot open: ") + std::strerror(errno));
    std::unique_ptr<std::FILE, int (*)(std::FILE*)> guard(f, std::fclose);
    unsigned char h[kCkptHeader];
    if (std::fread(h, 1, kCkptHeader, f) != kCkptHeader) return ckpt_fail(path_h, "shorter than its 80-byte header");
    if (std::memcmp(h, kCkptMagic, 8) != 0) return ckpt_fail(path_h, "not a checkpoint (magic)");
    const uint32_t version = get_le<uint32_t>(h, 8);
    if (version != kCkptVersion) return ckpt_fail(path_h, "format version " + std::to_string(version) + " is not 1");
    if (get_le<uint32_t>(h, 72) != crc32_ieee(h, 72)) return ckpt_fail(path_h, "header checksum mismatch");
    if (get_le<uint32_t>(h, 76) != 0) return ckpt_fail(path_h, "reserved header bytes are not zero");
    if (get_le<uint32_t>(h, 12) != 0) return ckpt_fail(path_h, "dtype is not 0 (float32)");
    rl0_mlp_ckpt info{};
    info.d = get_le<int32_t>(h, 16);
    info.dtype = 0;
    info.P = get_le<int64_t>(h, 24);
    info.seed = get_le<uint64_t>(h, 32);
    info.step = get_le<int64_t>(h, 40);
    info.cfg.batch = get_le<int32_t>(h, 20);
    info.cfg.lr = get_le<float>(h, 48);
    info.cfg.beta1 = get_le<float>(h, 52);
    info.cfg.beta2 = get_le<float>(h, 56);
    info.cfg.eps = get_le<float>(h, 60);
    info.cfg.lam = get_le<float>(h, 64);
    info.cfg.steps = 0;
    if (info.d < 1 || info.d > RL0_MAX_D) return ckpt_fail(path_h, "d out of [1, 16]");
    if (info.P != rl0::mlp_params(info.d)) return ckpt_fail(path_h, "P does not match d");
    if (info.step < 0 || info.step > INT32_MAX) return ckpt_fail(path_h, "step out of [0, 2^31)");
    if (!ckpt_cfg_ok(info.cfg)) return ckpt_fail(path_h, "bad hyper-parameters or batch");
    info.cfg.t0 = static_cast<int32_t>(info.step);
    const size_t P = static_cast<size_t>(info.P);
    std::vector<unsigned char> payload(12 * P + 1);
    const size_t got = std::fread(payload.data(), 1, payload.size(), f);
    if (got < 12 * P) return ckpt_fail(path_h, "truncated payload");
    if (got > 12 * P) return ckpt_fail(path_h, "bytes after the payload");
    if (get_le<uint32_t>(h, 68) != crc32_ieee(payload.data(), 12 * P))
        return ckpt_fail(path_h, "payload checksum mismatch");
    const hipStream_t s = static_cast<hipStream_t>(stream);
    float* arrays[3] = {w, adam_m, adam_v};
    bool any = false;
    for (int a = 0; a < 3; ++a) {
        if (!arrays[a]) continue;
        HIP_TRY(hipMemcpyAsync(arrays[a], payload.data() + a * 4 * P, 4 * P, hipMemcpyHostToDevice, s));
        any = true;
    }
    if (any) HIP_TRY(hipStreamSynchronize(s));
    if (info_h) *info_h = info;
    return RL0_OK;
}

// rl0_device_check reports a line of the batched kernel's source as this base + line,
// and one of the learned-decision kernel's source as the second base + line.
constexpr int kBatchedLineBase = 100000;
constexpr int kLearnedLineBase = 200000;

int rl0_device_check(int32_t* line_h, void* stream) {
    if (!line_h) return fail(RL0_EINVAL, "line_h is NULL");
    std::lock_guard<std::mutex> lk(g_mu);
    int line = 0, bline = 0, mline = 0;
    HIP_TRY(rl0::device_check_read(&line, static_cast<hipStream_t>(stream)));
    HIP_TRY(rl0::batched_check_read(&bline, static_cast<hipStream_t>(stream)));
    HIP_TRY(rl0::mlp_check_read(&mline, static_cast<hipStream_t>(stream)));
    *line_h = line != 0 ? line
                        : (bline > 0 ? kBatchedLineBase + bline : (mline > 0 ? kLearnedLineBase + mline : 0));
    return RL0_OK;
}

int rl0_profile_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    g_prof.enabled = enable != 0;
    for (double& t : g_prof.total_ms) t = 0.0;
    g_prof.launches = 0;
    g_prof.executed = 0;
    g_prof.learned_ms = 0.0;
    g_prof.learned_launches = 0;
    return RL0_OK;
}

static_assert(sizeof(rl0_iter_log) == sizeof(rl0::IterLog), "rl0_iter_log mirrors the device record");

int rl0_last_log(rl0_iter_log* out_h, int32_t cap, int32_t* count_h, void* stream) {
    if (cap < 0 || (cap > 0 && !out_h)) return fail(RL0_EINVAL, "out_h is NULL or cap < 0");
    std::lock_guard<std::mutex> lk(g_mu);
    hipStream_t s = static_cast<hipStream_t>(stream);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    auto it = g_ws.find({dev, s});
    const int count = (it == g_ws.end() || !it->second->block) ? 0 : it->second->last_log_count;
    if (count_h) *count_h = count;
    const int take = std::min({count, cap, rl0::kLogCap});
    if (take > 0) {
        HIP_TRY(hipMemcpyAsync(out_h, it->second->w.st->log, sizeof(rl0::IterLog) * take, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    return RL0_OK;
}

int rl0_profile_read_learned(double* ms_total_h, int64_t* launches_h) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (ms_total_h) *ms_total_h = g_prof.learned_ms;
    if (launches_h) *launches_h = g_prof.learned_launches;
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
    for (int k = 0; k < 4; ++k) ms_total_h[k] = g_prof.total_ms[k];
    if (counts_h) {
        counts_h[0] = g_prof.launches;
        counts_h[1] = g_prof.executed;
    }
    return RL0_OK;
}

void rl0_release(void) {
    std::lock_guard<std::mutex> lk(g_mu);
    // teardown: errors are not reported (the handles are dropped either way)
    (void)hipDeviceSynchronize();
    for (auto& kv : g_ws) {
        Buffers* b = kv.second.get();
        drop_graphs(b);
        if (b->capture) (void)hipStreamDestroy(b->capture);
        for (hipEvent_t e : b->ev_call)
            if (e) (void)hipEventDestroy(e);
        if (b->block) (void)hipFree(b->block);
        if (b->st_host) (void)hipHostFree(b->st_host);
        if (b->adapted && b->adapted->d_tables) (void)hipFree(b->adapted->d_tables);
    }
    g_ws.clear();
    for (auto& kv : g_bws) {
        BatchBuffers* b = kv.second.get();
        drop_batch_graphs(b);
        if (b->capture) (void)hipStreamDestroy(b->capture);
        for (hipEvent_t e : b->ev)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : b->ev_call)
            if (e) (void)hipEventDestroy(e);
        if (b->block) (void)hipFree(b->block);
        if (b->meta) (void)hipFree(b->meta);
        if (b->host) (void)hipHostFree(b->host);
    }
    g_bws.clear();
    for (auto& kv : g_mlp)
        if (kv.second.grad) (void)hipFree(kv.second.grad);
    g_mlp.clear();
    for (auto& kv : g_consts)
        if (kv.second->d_tables) (void)hipFree(kv.second->d_tables);
    g_consts.clear();
    for (hipEvent_t e : g_prof.pool) (void)hipEventDestroy(e);
    g_prof.pool.clear();
    for (hipEvent_t& e : g_prof.learned_ev) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }
}

}  // extern "C"
