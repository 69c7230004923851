// C-ABI front end: argument checks, workspace sizing and path dispatch.
//
// Every check runs on the host before any device work (the paper keeps the
// host blind during elimination, Sec. 3.1 and 3.2; here the host decides only
// the launch sequence).  Kernels live in plain.hip, batched.hip and blocked.hip.
#include <stdio.h>
#include <string.h>

#include <stdlib.h>

#include <algorithm>
#include <mutex>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "internal.h"

using namespace linac;

hipError_t linac::side_stream(hipStream_t* out) {
    static std::mutex mu;
    static std::vector<hipStream_t> streams;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lock(mu);
    if ((int)streams.size() <= dev) streams.resize(dev + 1, nullptr);
    if (!streams[dev]) {
        e = hipStreamCreateWithFlags(&streams[dev], hipStreamNonBlocking);
        if (e != hipSuccess) {
            streams[dev] = nullptr;
            return e;
        }
    }
    *out = streams[dev];
    return hipSuccess;
}

namespace {

thread_local int g_last_hip = 0;

linac_status hip_fail(hipError_t e) {
    g_last_hip = (int)e;
    return LINAC_E_HIP;
}

// a^e mod n for n < 2^32 (host).
uint64_t pow_mod_u64(uint64_t a, uint64_t e, uint64_t n) {
    uint64_t r = 1 % n;
    a %= n;
    while (e) {
        if (e & 1) r = r * a % n;
        a = a * a % n;
        e >>= 1;
    }
    return r;
}

// Deterministic Miller-Rabin for n < 4 759 123 141 with bases 2, 7, 61
// (Jaeschke 1993).
bool is_prime_u32(uint32_t n) {
    if (n < 2) return false;
    static const uint32_t small[] = {2, 3, 5, 7, 11, 13, 61};
    for (uint32_t q : small)
        if (n % q == 0) return n == q;
    uint32_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    for (uint32_t a : {2u, 7u, 61u}) {
        uint64_t x = pow_mod_u64(a, d, n);
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int i = 1; i < s; ++i) {
            x = x * x % n;
            if (x == n - 1) {
                witness = false;
                break;
            }
        }
        if (witness) return false;
    }
    return true;
}

// a * b mod n for n < 2^64 (host, 128-bit product).
uint64_t mul_mod_u128(uint64_t a, uint64_t b, uint64_t n) {
    return (uint64_t)((unsigned __int128)a * b % n);
}

// Deterministic Miller-Rabin for n < 3.3e24 with the first twelve primes as
// bases (J. Sorenson and J. Webster, "Strong pseudoprimes to twelve prime
// bases", 2017).
bool is_prime_u64(uint64_t n) {
    static const uint64_t bases[] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2) return false;
    for (uint64_t q : bases)
        if (n % q == 0) return n == q;
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
    for (uint64_t a : bases) {
        uint64_t x = 1, b = a, e = d;
        while (e) {
            if (e & 1) x = mul_mod_u128(x, b, n);
            b = mul_mod_u128(b, b, n);
            e >>= 1;
        }
        if (x == 1 || x == n - 1) continue;
        bool witness = true;
        for (int i = 1; i < s; ++i) {
            x = mul_mod_u128(x, x, n);
            if (x == n - 1) {
                witness = false;
                break;
            }
        }
        if (witness) return false;
    }
    return true;
}

// Primes of the 64-bit column-step paths: 2 <= p < 2^63.
linac_status check_field64(uint64_t p) {
    if (p == 0 || p >= (1ull << 63)) return LINAC_E_UNSUPPORTED;
    return is_prime_u64(p) ? LINAC_OK : LINAC_E_NOT_PRIME;
}

template <typename W>
linac_status validate_range_t(const W* M, int64_t rows, int64_t cols, int64_t ld, W p, uint32_t* flag,
                              hipStream_t s) {
    if (rows * cols == 0) return LINAC_OK;
    uint32_t zero = 0, host = 0;
    hipError_t e = hipMemcpyAsync(flag, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = colstep_range<W>(M, rows, cols, ld, p, flag, s);
    if (e == hipSuccess) e = hipMemcpyAsync(&host, flag, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    return host ? LINAC_E_RANGE : LINAC_OK;
}

linac_status check_field(uint32_t p) {
    if (p == 0 || p >= 0x80000000u) return LINAC_E_UNSUPPORTED;
    return is_prime_u32(p) ? LINAC_OK : LINAC_E_NOT_PRIME;
}

// ---------------------------------------------------------------------------
// Tuning table.  Defaults are built in; linac_load_tuning replaces them with
// values measured by the autotuner.  Only choices that never change results
// are tuned: the plain/blocked crossover, the panel width per size bucket and
// the number of resident batched workgroups per compute unit.
// ---------------------------------------------------------------------------
struct PanelRule {
    int64_t n_max;
    int32_t panel;
};
struct Tuning {
    int64_t blocked_min = 1024;  // AUTO takes the blocked path from min(m, n) >= this
    int32_t batched_per_cu = 4;
    int32_t lookahead = 1;       // blocked int8: overlap the next panel with the trailing update
    int32_t rref_lanes = 4;      // linac_rref_batched: instances reduced concurrently
    int64_t forward_min = 12288; // solves on the blocked int8 path eliminate forward from min(m, n) >= this
    int32_t leaf_blocks = 2;     // 16-column blocks per workgroup of the int8 leaf product
    int32_t leaf_pipeline = 1;   // blocked int8: overlap each leaf's product with the next selection
    std::vector<PanelRule> panels{{1 << 30, 256}};
};
std::mutex g_tune_mu;
Tuning g_tune;

Tuning tuning() {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    return g_tune;
}

// A small JSON reader for the tuning file: objects, arrays, numbers, strings,
// true/false/null.  Values are collected as "path.to.key" -> number; arrays of
// objects are flattened with an index ("panel.0.n_max").
struct JsonReader {
    const char* s;
    bool ok = true;
    std::vector<std::pair<std::string, double>> out;
    void ws() {
        while (*s == ' ' || *s == '\n' || *s == '\t' || *s == '\r') ++s;
    }
    bool str(std::string& v) {
        ws();
        if (*s != '"') return false;
        ++s;
        v.clear();
        while (*s && *s != '"') {
            if (*s == '\\' && s[1]) ++s;
            v.push_back(*s++);
        }
        if (*s != '"') return false;
        ++s;
        return true;
    }
    bool value(const std::string& key) {
        ws();
        if (*s == '{') {
            ++s;
            ws();
            if (*s == '}') return ++s, true;
            for (;;) {
                std::string k;
                if (!str(k)) return false;
                ws();
                if (*s != ':') return false;
                ++s;
                if (!value(key.empty() ? k : key + "." + k)) return false;
                ws();
                if (*s == ',') { ++s; continue; }
                if (*s == '}') return ++s, true;
                return false;
            }
        }
        if (*s == '[') {
            ++s;
            ws();
            if (*s == ']') return ++s, true;
            for (int i = 0;; ++i) {
                if (!value(key + "." + std::to_string(i))) return false;
                ws();
                if (*s == ',') { ++s; continue; }
                if (*s == ']') return ++s, true;
                return false;
            }
        }
        if (*s == '"') {
            std::string v;
            return str(v);
        }
        if (!strncmp(s, "true", 4) || !strncmp(s, "null", 4)) return s += 4, true;
        if (!strncmp(s, "false", 5)) return s += 5, true;
        char* end = nullptr;
        double d = strtod(s, &end);
        if (end == s) return false;
        s = end;
        out.emplace_back(key, d);
        return true;
    }
};

linac_status parse_tuning(const char* json, Tuning* t) {
    JsonReader r{json};
    if (!r.value("")) return LINAC_E_INVALID_ARG;
    r.ws();
    if (*r.s) return LINAC_E_INVALID_ARG;
    Tuning nt;
    std::vector<PanelRule> rules;
    for (const auto& kv : r.out) {
        const std::string& k = kv.first;
        const double v = kv.second;
        if (k == "blocked_min") nt.blocked_min = (int64_t)v;
        else if (k == "batched_per_cu") nt.batched_per_cu = (int32_t)v;
        else if (k == "lookahead") nt.lookahead = (int32_t)v;
        else if (k == "rref_lanes") nt.rref_lanes = (int32_t)v;
        else if (k == "forward_min") nt.forward_min = (int64_t)v;
        else if (k == "leaf_blocks") nt.leaf_blocks = (int32_t)v;
        else if (k == "leaf_pipeline") nt.leaf_pipeline = (int32_t)v;
        else if (k.rfind("panel.", 0) == 0) {
            size_t dot = k.find('.', 6);
            if (dot == std::string::npos) return LINAC_E_INVALID_ARG;
            size_t idx = (size_t)atoi(k.c_str() + 6);
            if (rules.size() <= idx) rules.resize(idx + 1, PanelRule{0, 0});
            std::string field = k.substr(dot + 1);
            if (field == "n_max") rules[idx].n_max = (int64_t)v;
            else if (field == "panel") rules[idx].panel = (int32_t)v;
        }
    }
    for (const PanelRule& pr : rules)
        if (pr.n_max <= 0 || pr.panel < 32 || pr.panel > 512 || pr.panel % 32) return LINAC_E_INVALID_ARG;
    if (nt.blocked_min < 1 || nt.batched_per_cu < 1 || nt.batched_per_cu > 16 ||
        (nt.lookahead != 0 && nt.lookahead != 1) || nt.rref_lanes < 1 || nt.rref_lanes > 8 ||
        nt.forward_min < 0 || (nt.leaf_pipeline != 0 && nt.leaf_pipeline != 1) ||
        (nt.leaf_blocks != 2 && nt.leaf_blocks != 3 && nt.leaf_blocks != 6 && nt.leaf_blocks != 9))
        return LINAC_E_INVALID_ARG;
    std::sort(rules.begin(), rules.end(),
              [](const PanelRule& a, const PanelRule& b) { return a.n_max < b.n_max; });
    if (!rules.empty()) nt.panels = rules;
    *t = nt;
    return LINAC_OK;
}

// AUTO: the plain path for small systems, the int8-MFMA blocked path from the
// tuned crossover on.  Depends only on the shape so that the workspace query
// and the call agree.
int choose_path(const linac_opts* opts, int64_t m, int64_t n) {
    int path = opts ? opts->path : LINAC_PATH_AUTO;
    if (path != LINAC_PATH_AUTO) return path;
    return (m < n ? m : n) >= tuning().blocked_min ? LINAC_PATH_BLOCKED_INT8 : LINAC_PATH_PLAIN;
}

// Panel width: the caller's, else the tuned one for this size (the first rule
// whose n_max covers min(m, n)), else the last rule.
int32_t panel_width(const linac_opts* opts, int64_t m = 0, int64_t n = 0) {
    if (opts && opts->panel_width > 0) return opts->panel_width;
    const Tuning t = tuning();
    const int64_t sz = m < n ? m : n;
    for (const PanelRule& pr : t.panels)
        if (sz <= pr.n_max) return pr.panel;
    return t.panels.back().panel;
}

bool panel_ok(int32_t w) { return w >= 32 && w <= 512 && w % 32 == 0; }

linac_status path_workspace(int path, int64_t m, int64_t n, int64_t k, const linac_opts* opts,
                            size_t* bytes) {
    if (path == LINAC_PATH_PLAIN) {
        *bytes = plain_workspace(m, n, k);
        return LINAC_OK;
    }
    if (path == LINAC_PATH_BLOCKED_INT8 || path == LINAC_PATH_BLOCKED_FP64) {
        int32_t w = panel_width(opts, m, n);
        if (!panel_ok(w)) return LINAC_E_INVALID_ARG;
        *bytes = blocked_workspace(m, n, k, w);
        return LINAC_OK;
    }
    return LINAC_E_UNSUPPORTED;
}

// Elimination on an already prepared workspace; on return `a` describes the
// bookkeeping the extraction kernels read.
// allow_overlap = false keeps the blocked int8 path on the caller's stream (no
// side stream, no events: nothing is created).
// forward = true: a solve (only X, rank, pivots and consistency are read), so
// the blocked int8 path may eliminate forward and back-substitute; it does so
// from the tuned size forward_min on (below it Gauss-Jordan is faster: the
// leaf chain, not the trailing product, bounds the time, and back-substitution
// adds launches).
hipError_t run_path(int path, void* ws, int64_t m, int64_t n, int64_t k, PlainArgs& a,
                    const linac_opts* opts, hipStream_t s, bool allow_overlap = true,
                    bool forward = false) {
    if (path == LINAC_PATH_PLAIN) return plain_eliminate(a, opts, s);
    const Tuning t = tuning();
    forward = forward && (m < n ? m : n) >= t.forward_min;
    return blocked_eliminate(ws, m, n, k, panel_width(opts, m, n), path == LINAC_PATH_BLOCKED_FP64,
                             allow_overlap && t.lookahead != 0, forward, t.leaf_blocks,
                             t.leaf_pipeline != 0, a, opts, s);
}

bool size_ok(int64_t m, int64_t n, int64_t k) {
    // kernels index rows and columns with 32-bit values
    return m < (1LL << 31) - 64 && n + k < (1LL << 31) - 64;
}

// Host range check (optional, synchronous): runs a kernel that raises a flag
// in the workspace, then reads the flag back.
linac_status validate_range(const uint32_t* M, int64_t rows, int64_t cols, int64_t ld, uint32_t p,
                            uint32_t* flag, hipStream_t s) {
    if (rows * cols == 0) return LINAC_OK;
    uint32_t zero = 0, host = 0;
    hipError_t e = hipMemcpyAsync(flag, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);
    e = launch_range_check(M, rows, cols, ld, p, flag, s);
    if (e != hipSuccess) return hip_fail(e);
    e = hipMemcpyAsync(&host, flag, sizeof(host), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e);
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e);
    return host ? LINAC_E_RANGE : LINAC_OK;
}

// Streams of linac_rref_batched: kMaxLanes per device, created on first use
// (default priority), with one event per lane for the join and one for the fork.
constexpr int kMaxLanes = 8;
struct Lanes {
    hipStream_t st[kMaxLanes] = {};
    hipEvent_t done[kMaxLanes] = {};
    hipEvent_t fork = nullptr;
    std::mutex busy;  // one batched call per device at a time uses the lanes
};
std::mutex g_lanes_mu;
std::vector<Lanes*> g_lanes;

hipError_t lanes_for_device(int dev, Lanes** out) {
    std::lock_guard<std::mutex> lock(g_lanes_mu);
    if ((int)g_lanes.size() <= dev) g_lanes.resize(dev + 1, nullptr);
    if (!g_lanes[dev]) {
        Lanes* L = new Lanes();
        hipError_t e = hipEventCreateWithFlags(&L->fork, hipEventDisableTiming);
        for (int i = 0; i < kMaxLanes && e == hipSuccess; ++i) {
            e = hipStreamCreateWithFlags(&L->st[i], hipStreamNonBlocking);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&L->done[i], hipEventDisableTiming);
        }
        if (e != hipSuccess) return e;  // the partial set is kept for the process (never reused)
        g_lanes[dev] = L;
    }
    *out = g_lanes[dev];
    return hipSuccess;
}

// Checks of one matrix of a batched RREF (host only); *need receives its workspace.
linac_status check_rref_matrix(const linac_matrix& d, const linac_opts* opts,
                               std::vector<uint32_t>& primes_ok, size_t* need) {
    if (d.m < 0 || d.n < 0) return LINAC_E_INVALID_ARG;
    if (d.lda < (d.n > 0 ? d.n : 1)) return LINAC_E_INVALID_ARG;
    if (!d.rank) return LINAC_E_INVALID_ARG;
    if (d.m * d.n > 0 && !d.A) return LINAC_E_INVALID_ARG;
    if ((d.m < d.n ? d.m : d.n) > 0 && !d.pivots) return LINAC_E_INVALID_ARG;
    if (std::find(primes_ok.begin(), primes_ok.end(), d.p) == primes_ok.end()) {
        const linac_status st = check_field(d.p);
        if (st != LINAC_OK) return st;
        primes_ok.push_back(d.p);
    }
    if (!size_ok(d.m, d.n, 0)) return LINAC_E_NOMEM;
    const int path = choose_path(opts, d.m, d.n);
    if (path == LINAC_PATH_BLOCKED_FP64 && d.p >= (1u << 21)) return LINAC_E_UNSUPPORTED;
    return path_workspace(path, d.m, d.n, 0, opts, need);
}

// One RREF on a prepared workspace (the body of linac_rref after its checks).
hipError_t rref_on(const linac_matrix& d, void* ws, const linac_opts* opts, hipStream_t s,
                   bool allow_overlap) {
    const int path = choose_path(opts, d.m, d.n);
    PlainArgs a;
    plain_carve(ws, d.m, d.n, 0, a);
    a.F = make_field(d.p);
    hipError_t e = plain_prepare(a, d.A, d.lda, nullptr, 1, (int32_t)d.n, 0, s);
    if (e == hipSuccess) e = run_path(path, ws, d.m, d.n, 0, a, opts, s, allow_overlap);
    if (e == hipSuccess) e = plain_finish_rref(a, d.A, d.lda, d.rank, d.pivots, s);
    return e;
}

// Graphs of the batched launch (counter reset + persistent kernel), captured
// once per (device, workspace, count, grid, multiplier rows) and replayed
// afterwards.  The
// kernel arguments point into the workspace only, so a replay on the same
// workspace sees the descriptors uploaded by the current call.
struct BatchedGraph {
    int dev;
    void* ws;
    int32_t count;
    int32_t grid;
    int32_t mult_rows;
    hipGraphExec_t exec;
};
std::mutex g_graph_mu;
std::vector<BatchedGraph> g_graphs;

hipError_t batched_graph(int dev, void* ws, int32_t count, int32_t grid, int32_t mult_rows,
                         hipGraphExec_t* out) {
    std::lock_guard<std::mutex> lock(g_graph_mu);
    for (const BatchedGraph& g : g_graphs)
        if (g.dev == dev && g.ws == ws && g.count == count && g.grid == grid &&
            g.mult_rows == mult_rows) {
            *out = g.exec;
            return hipSuccess;
        }
    hipStream_t cap = nullptr;
    hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
    if (e != hipSuccess) return e;
    hipGraph_t graph = nullptr;
    e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        hipError_t le = batched_launch(ws, count, grid, mult_rows, cap);
        e = hipStreamEndCapture(cap, &graph);
        if (le != hipSuccess) e = le;
    }
    hipGraphExec_t exec = nullptr;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return e;
    if (g_graphs.size() >= 64) {  // bounded cache: drop the oldest
        (void)hipGraphExecDestroy(g_graphs.front().exec);
        g_graphs.erase(g_graphs.begin());
    }
    g_graphs.push_back({dev, ws, count, grid, mult_rows, exec});
    *out = exec;
    return hipSuccess;
}

template <typename W>
linac_status lup_t(W* A, int64_t m, int64_t n, int64_t lda, W p, int32_t* perm, int32_t* rank,
                          int32_t* pivots, void* ws, size_t ws_bytes, const linac_opts* opts,
                          hipStream_t s) {
    constexpr bool wide = sizeof(W) == 8;
    if (m < 0 || n < 0 || lda < (n > 0 ? n : 1) || !rank) return LINAC_E_INVALID_ARG;
    if (m * n > 0 && !A) return LINAC_E_INVALID_ARG;
    if (m > 0 && !perm) return LINAC_E_INVALID_ARG;
    if ((m < n ? m : n) > 0 && !pivots) return LINAC_E_INVALID_ARG;
    const linac_status st = wide ? check_field64((uint64_t)p) : check_field((uint32_t)p);
    if (st != LINAC_OK) return st;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    if (!ws || ws_bytes < colstep_workspace(m, n, 0, wide)) return LINAC_E_WORKSPACE;
    if (opts && opts->validate) {
        const linac_status vs = validate_range_t<W>(A, m, n, lda, p, (uint32_t*)ws, s);
        if (vs != LINAC_OK) return vs;
    }
    return hip_status(colstep_lup<W>(A, m, n, lda, p, perm, rank, pivots, ws, s));
}

}  // namespace

linac_status linac::hip_status(hipError_t e) {
    return e == hipSuccess ? LINAC_OK : hip_fail(e);
}

linac_status linac::solve_check(const uint32_t* A, int64_t m, int64_t n, int64_t lda,
                                const uint32_t* B, int64_t k, int64_t ldb, uint32_t p,
                                const uint32_t* X, int64_t ldx, const int32_t* rank,
                                const int32_t* pivots, const uint8_t* consistent,
                                const linac_opts* opts, int* path, size_t* need) {
    if (m < 0 || n < 0 || k < 0) return LINAC_E_INVALID_ARG;
    if (lda < (n > 0 ? n : 1) || ldb < (k > 0 ? k : 1) || ldx < (k > 0 ? k : 1))
        return LINAC_E_INVALID_ARG;
    if (!rank) return LINAC_E_INVALID_ARG;
    if (m * n > 0 && !A) return LINAC_E_INVALID_ARG;
    if (m * k > 0 && !B) return LINAC_E_INVALID_ARG;
    if (n * k > 0 && !X) return LINAC_E_INVALID_ARG;
    if (k > 0 && !consistent) return LINAC_E_INVALID_ARG;
    if ((m < n ? m : n) > 0 && !pivots) return LINAC_E_INVALID_ARG;
    linac_status st = check_field(p);
    if (st != LINAC_OK) return st;
    if (!size_ok(m, n, k)) return LINAC_E_NOMEM;
    *path = choose_path(opts, m, n);
    if (*path == LINAC_PATH_BLOCKED_FP64 && p >= (1u << 21)) return LINAC_E_UNSUPPORTED;
    return path_workspace(*path, m, n, k, opts, need);
}

linac_status linac::solve_launch(const uint32_t* A, int64_t m, int64_t n, int64_t lda,
                                 const uint32_t* B, int64_t k, int64_t ldb, uint32_t p, uint32_t* X,
                                 int64_t ldx, int32_t* rank, int32_t* pivots, uint8_t* consistent,
                                 void* ws, int path, const linac_opts* opts, hipStream_t s,
                                 bool allow_overlap, const char* name) {
    PlainArgs a;
    plain_carve(ws, m, n, k, a);
    a.F = make_field(p);
    if (opts && opts->validate) {
        linac_status st = validate_range(A, m, n, lda, p, (uint32_t*)a.state, s);
        if (st == LINAC_OK) st = validate_range(B, m, k, ldb, p, (uint32_t*)a.state, s);
        if (st != LINAC_OK) return st;
    }
    if (opts && opts->verbose)
        fprintf(stderr, "[linac] %s path=%d m=%lld n=%lld k=%lld p=%u ld=%lld panel=%d\n", name,
                path, (long long)m, (long long)n, (long long)k, p, (long long)a.ld,
                panel_width(opts, m, n));
    hipError_t e = plain_prepare(a, A, lda, B, ldb, (int32_t)n, (int32_t)k, s);
    if (e == hipSuccess) e = run_path(path, ws, m, n, k, a, opts, s, allow_overlap, true);
    if (e == hipSuccess) e = plain_finish_solve(a, (int32_t)n, (int32_t)k, X, ldx, rank, pivots,
                                                consistent, s);
    return e == hipSuccess ? LINAC_OK : hip_fail(e);
}

extern "C" {

int linac_version(void) { return 100; }

int linac_last_hip_error(void) { return g_last_hip; }

const char* linac_status_string(linac_status st) {
    switch (st) {
        case LINAC_OK: return "ok";
        case LINAC_E_INVALID_ARG: return "invalid argument";
        case LINAC_E_UNSUPPORTED: return "unsupported (p must be a prime below 2^31; path unavailable)";
        case LINAC_E_NOT_PRIME: return "modulus is not prime";
        case LINAC_E_RANGE: return "entry out of range [0, p)";
        case LINAC_E_WORKSPACE: return "workspace missing or too small";
        case LINAC_E_NOMEM: return "problem too large";
        case LINAC_E_HIP: return "HIP runtime error";
    }
    return "unknown status";
}

linac_status linac_check_prime(uint32_t p) { return check_field(p); }

linac_status linac_plan(int64_t m, int64_t n, const linac_opts* opts, int* path, int* panel) {
    if (!path || !panel || m < 0 || n < 0) return LINAC_E_INVALID_ARG;
    const int pth = choose_path(opts, m, n);
    if (pth != LINAC_PATH_PLAIN && pth != LINAC_PATH_BLOCKED_INT8 && pth != LINAC_PATH_BLOCKED_FP64)
        return LINAC_E_UNSUPPORTED;
    const int32_t w = pth == LINAC_PATH_PLAIN ? 0 : panel_width(opts, m, n);
    if (pth != LINAC_PATH_PLAIN && !panel_ok(w)) return LINAC_E_INVALID_ARG;
    *path = pth;
    *panel = w;
    return LINAC_OK;
}

linac_status linac_rref_workspace(int64_t m, int64_t n, const linac_opts* opts, size_t* bytes) {
    if (!bytes || m < 0 || n < 0) return LINAC_E_INVALID_ARG;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    return path_workspace(choose_path(opts, m, n), m, n, 0, opts, bytes);
}

linac_status linac_rref(uint32_t* A, int64_t m, int64_t n, int64_t lda, uint32_t p, int32_t* rank,
                        int32_t* pivots, void* ws, size_t ws_bytes, const linac_opts* opts,
                        hipStream_t s) {
    if (m < 0 || n < 0) return LINAC_E_INVALID_ARG;
    if (lda < (n > 0 ? n : 1)) return LINAC_E_INVALID_ARG;
    if (!rank) return LINAC_E_INVALID_ARG;
    if (m * n > 0 && !A) return LINAC_E_INVALID_ARG;
    if ((m < n ? m : n) > 0 && !pivots) return LINAC_E_INVALID_ARG;
    linac_status st = check_field(p);
    if (st != LINAC_OK) return st;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    int path = choose_path(opts, m, n);
    if (path == LINAC_PATH_BLOCKED_FP64 && p >= (1u << 21)) return LINAC_E_UNSUPPORTED;
    size_t need = 0;
    st = path_workspace(path, m, n, 0, opts, &need);
    if (st != LINAC_OK) return st;
    if (!ws || ws_bytes < need) return LINAC_E_WORKSPACE;

    PlainArgs a;
    plain_carve(ws, m, n, 0, a);
    a.F = make_field(p);
    if (opts && opts->validate) {
        st = validate_range(A, m, n, lda, p, (uint32_t*)a.state, s);
        if (st != LINAC_OK) return st;
    }
    if (opts && opts->verbose)
        fprintf(stderr, "[linac] rref path=%d m=%lld n=%lld p=%u ld=%lld panel=%d\n", path,
                (long long)m, (long long)n, p, (long long)a.ld, panel_width(opts, m, n));
    hipError_t e = plain_prepare(a, A, lda, nullptr, 1, (int32_t)n, 0, s);
    if (e == hipSuccess) e = run_path(path, ws, m, n, 0, a, opts, s);
    if (e == hipSuccess) e = plain_finish_rref(a, A, lda, rank, pivots, s);
    return e == hipSuccess ? LINAC_OK : hip_fail(e);
}

linac_status linac_solve_workspace(int64_t m, int64_t n, int64_t k, const linac_opts* opts,
                                   size_t* bytes) {
    if (!bytes || m < 0 || n < 0 || k < 0) return LINAC_E_INVALID_ARG;
    if (!size_ok(m, n, k)) return LINAC_E_NOMEM;
    return path_workspace(choose_path(opts, m, n), m, n, k, opts, bytes);
}

linac_status linac_solve(const uint32_t* A, int64_t m, int64_t n, int64_t lda, const uint32_t* B,
                         int64_t k, int64_t ldb, uint32_t p, uint32_t* X, int64_t ldx,
                         int32_t* rank, int32_t* pivots, uint8_t* consistent, void* ws,
                         size_t ws_bytes, const linac_opts* opts, hipStream_t s) {
    int path = 0;
    size_t need = 0;
    const linac_status st = solve_check(A, m, n, lda, B, k, ldb, p, X, ldx, rank, pivots,
                                        consistent, opts, &path, &need);
    if (st != LINAC_OK) return st;
    if (!ws || ws_bytes < need) return LINAC_E_WORKSPACE;
    return solve_launch(A, m, n, lda, B, k, ldb, p, X, ldx, rank, pivots, consistent, ws, path, opts,
                        s, true, "solve");
}

linac_status linac_solve_batched_workspace(const linac_system* sys, int32_t count,
                                           const linac_opts* opts, size_t* bytes) {
    if (!bytes || count < 0 || (count > 0 && !sys)) return LINAC_E_INVALID_ARG;
    (void)opts;
    for (int32_t i = 0; i < count; ++i) {
        const linac_system& d = sys[i];
        if (d.m < 0 || d.n < 0 || d.k < 0) return LINAC_E_INVALID_ARG;
        if (!batched_fits(d.m, d.n, d.k)) return LINAC_E_UNSUPPORTED;
    }
    *bytes = batched_workspace(sys, count);
    return LINAC_OK;
}

linac_status linac_solve_batched(const linac_system* sys, int32_t count, void* ws, size_t ws_bytes,
                                 const linac_opts* opts, hipStream_t s) {
    if (count < 0 || (count > 0 && !sys)) return LINAC_E_INVALID_ARG;
    if (count == 0) return LINAC_OK;
    std::vector<uint32_t> primes_ok;
    for (int32_t i = 0; i < count; ++i) {
        const linac_system& d = sys[i];
        if (d.m < 0 || d.n < 0 || d.k < 0) return LINAC_E_INVALID_ARG;
        if (d.lda < (d.n > 0 ? d.n : 1) || d.ldb < (d.k > 0 ? d.k : 1) ||
            d.ldx < (d.k > 0 ? d.k : 1))
            return LINAC_E_INVALID_ARG;
        if (!d.rank) return LINAC_E_INVALID_ARG;
        if ((int64_t)d.m * d.n > 0 && !d.A) return LINAC_E_INVALID_ARG;
        if ((int64_t)d.m * d.k > 0 && !d.B) return LINAC_E_INVALID_ARG;
        if ((int64_t)d.n * d.k > 0 && !d.X) return LINAC_E_INVALID_ARG;
        if (d.k > 0 && !d.consistent) return LINAC_E_INVALID_ARG;
        if ((d.m < d.n ? d.m : d.n) > 0 && !d.pivots) return LINAC_E_INVALID_ARG;
        if (!batched_fits(d.m, d.n, d.k)) return LINAC_E_UNSUPPORTED;
        if (std::find(primes_ok.begin(), primes_ok.end(), d.p) == primes_ok.end()) {
            linac_status st = check_field(d.p);
            if (st != LINAC_OK) return st;
            primes_ok.push_back(d.p);
        }
    }
    const size_t need = batched_workspace(sys, count);
    if (!ws || ws_bytes < need) return LINAC_E_WORKSPACE;
    if (opts && opts->validate) {
        // every system's A and B against its own prime; the flag borrows the
        // queue counter's word, which the launch resets before use
        uint32_t* flag = (uint32_t*)ws;
        uint32_t zero = 0, host = 0;
        hipError_t e = hipMemcpyAsync(flag, &zero, sizeof(zero), hipMemcpyHostToDevice, s);
        for (int32_t i = 0; i < count && e == hipSuccess; ++i) {
            const linac_system& d = sys[i];
            e = launch_range_check(d.A, d.m, d.n, d.lda, d.p, flag, s);
            if (e == hipSuccess) e = launch_range_check(d.B, d.m, d.k, d.ldb, d.p, flag, s);
        }
        if (e == hipSuccess) e = hipMemcpyAsync(&host, flag, sizeof(host), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e);
        if (host) return LINAC_E_RANGE;
    }

    // queue order: decreasing Gauss-Jordan cost m * n * (n + k)
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        const double ca = (double)sys[a].m * sys[a].n * (sys[a].n + sys[a].k);
        const double cb = (double)sys[b].m * sys[b].n * (sys[b].n + sys[b].k);
        return ca > cb;
    });
    std::vector<char> host(batched_desc_bytes() * (size_t)count);
    batched_describe(sys, count, ws, host.data(), order.data());
    // pageable source: the runtime stages it before returning
    hipError_t e = hipMemcpyAsync(batched_desc_ptr(ws), host.data(), host.size(),
                                  hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e);

    int dev = 0;
    e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    int cus = 0;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e);
    const int32_t per_cu = tuning().batched_per_cu;
    const int32_t grid = std::max(1, std::min(count, cus * per_cu));
    hipGraphExec_t exec = nullptr;
    e = batched_graph(dev, ws, count, grid, batched_mult_rows(sys, count), &exec);
    if (e != hipSuccess) return hip_fail(e);
    if (opts && opts->verbose)
        fprintf(stderr, "[linac] batched count=%d grid=%d ws=%p\n", count, grid, ws);
    if (opts && opts->ev_begin) {
        e = hipEventRecord(opts->ev_begin, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    LaunchTimer lt(opts, s);
    lt.before(LINAC_KERNEL_BATCHED);
    e = hipGraphLaunch(exec, s);
    lt.after();
    if (e != hipSuccess) return hip_fail(e);
    if (opts && opts->ev_end) {
        e = hipEventRecord(opts->ev_end, s);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (opts && opts->dominant_launches) *opts->dominant_launches = 1;
    return LINAC_OK;
}

linac_status linac_load_matrix(const uint32_t* bases, int64_t nrows, int64_t nbasis,
                               int64_t ldbases, const int32_t* lindices, int64_t ncols, int64_t d,
                               int64_t ldl, uint32_t p, uint32_t* A, int64_t lda, hipStream_t s) {
    if (nrows < 0 || nbasis < 0 || ncols < 0 || d < 0) return LINAC_E_INVALID_ARG;
    if (ldbases < (nbasis > 0 ? nbasis : 1) || ldl < (d > 0 ? d : 1) || lda < (ncols > 0 ? ncols : 1))
        return LINAC_E_INVALID_ARG;
    if (nrows * nbasis > 0 && !bases) return LINAC_E_INVALID_ARG;
    if (ncols * d > 0 && !lindices) return LINAC_E_INVALID_ARG;
    if (nrows * ncols > 0 && !A) return LINAC_E_INVALID_ARG;
    linac_status st = check_field(p);
    if (st != LINAC_OK) return st;
    if (nrows >= (1LL << 31) || ncols >= (1LL << 31) || nbasis >= (1LL << 31) - 1 ||
        d >= (1LL << 31))
        return LINAC_E_NOMEM;
    const hipError_t e = launch_load_matrix(bases, nrows, nbasis, ldbases, lindices, ncols, d, ldl,
                                            make_field(p), A, lda, s);
    return e == hipSuccess ? LINAC_OK : hip_fail(e);
}

linac_status linac_nullspace(const uint32_t* R, int64_t m, int64_t n, int64_t ldr,
                             const int32_t* rank, const int32_t* pivots, uint32_t p, uint32_t* K,
                             int64_t kcols, int64_t ldk, int32_t* free_cols, hipStream_t s) {
    if (m < 0 || n < 0 || kcols < 0 || kcols > n) return LINAC_E_INVALID_ARG;
    if (ldr < (n > 0 ? n : 1) || ldk < (kcols > 0 ? kcols : 1)) return LINAC_E_INVALID_ARG;
    if (!rank) return LINAC_E_INVALID_ARG;
    if ((m < n ? m : n) > 0 && (!R || !pivots)) return LINAC_E_INVALID_ARG;
    if (n * kcols > 0 && !K) return LINAC_E_INVALID_ARG;
    linac_status st = check_field(p);
    if (st != LINAC_OK) return st;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    const hipError_t e = launch_nullspace(R, m, n, ldr, rank, pivots, p, K, kcols, ldk, free_cols, s);
    return e == hipSuccess ? LINAC_OK : hip_fail(e);
}

linac_status linac_column_basis(const uint32_t* A, int64_t m, int64_t n, int64_t lda,
                                const int32_t* rank, const int32_t* pivots, uint32_t* C,
                                int64_t ccols, int64_t ldc, hipStream_t s) {
    if (m < 0 || n < 0 || ccols < 0 || ccols > (m < n ? m : n)) return LINAC_E_INVALID_ARG;
    if (lda < (n > 0 ? n : 1) || ldc < (ccols > 0 ? ccols : 1)) return LINAC_E_INVALID_ARG;
    if (!rank) return LINAC_E_INVALID_ARG;
    if ((m < n ? m : n) > 0 && (!A || !pivots)) return LINAC_E_INVALID_ARG;
    if (m * ccols > 0 && !C) return LINAC_E_INVALID_ARG;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    const hipError_t e = launch_column_basis(A, m, n, lda, rank, pivots, C, ccols, ldc, s);
    return e == hipSuccess ? LINAC_OK : hip_fail(e);
}

linac_status linac_rref_batched_workspace(const linac_matrix* mats, int32_t count,
                                          const linac_opts* opts, size_t* bytes) {
    if (!bytes || count < 0 || (count > 0 && !mats)) return LINAC_E_INVALID_ARG;
    size_t per = 0;
    for (int32_t i = 0; i < count; ++i) {
        const linac_matrix& d = mats[i];
        if (d.m < 0 || d.n < 0) return LINAC_E_INVALID_ARG;
        if (!size_ok(d.m, d.n, 0)) return LINAC_E_NOMEM;
        size_t need = 0;
        const linac_status st = path_workspace(choose_path(opts, d.m, d.n), d.m, d.n, 0, opts, &need);
        if (st != LINAC_OK) return st;
        per = std::max(per, (size_t)round_up((int64_t)need, 256));
    }
    const int32_t lanes = std::min<int32_t>(std::max<int32_t>(count, 1), tuning().rref_lanes);
    *bytes = per * (size_t)lanes;
    return LINAC_OK;
}

linac_status linac_rref_batched(const linac_matrix* mats, int32_t count, void* ws, size_t ws_bytes,
                                const linac_opts* opts, hipStream_t s) {
    if (count < 0 || (count > 0 && !mats)) return LINAC_E_INVALID_ARG;
    if (count == 0) return LINAC_OK;
    std::vector<uint32_t> primes_ok;
    size_t per = 0;
    for (int32_t i = 0; i < count; ++i) {
        size_t need = 0;
        const linac_status st = check_rref_matrix(mats[i], opts, primes_ok, &need);
        if (st != LINAC_OK) return st;
        per = std::max(per, (size_t)round_up((int64_t)need, 256));
    }
    const int32_t lanes = std::min<int32_t>(count, tuning().rref_lanes);
    if (!ws || ws_bytes < per * (size_t)lanes) return LINAC_E_WORKSPACE;
    if (opts && opts->validate) {
        uint32_t* flag = (uint32_t*)ws;  // the first lane's workspace, reinitialised by its first RREF
        for (int32_t i = 0; i < count; ++i) {
            const linac_matrix& d = mats[i];
            const linac_status st = validate_range(d.A, d.m, d.n, d.lda, d.p, flag, s);
            if (st != LINAC_OK) return st;
        }
    }
    // instance order: decreasing cost m n min(m, n), each to the lane that
    // frees first (longest processing time first)
    std::vector<int32_t> order(count);
    std::iota(order.begin(), order.end(), 0);
    auto cost = [&](int32_t i) {
        const double m = (double)mats[i].m, n = (double)mats[i].n;
        return m * n * std::min(m, n) + m * n;
    };
    std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return cost(a) > cost(b); });
    std::vector<std::vector<int32_t>> plan(lanes);
    std::vector<double> load(lanes, 0.0);
    for (int32_t i : order) {
        const int32_t l = (int32_t)(std::min_element(load.begin(), load.end()) - load.begin());
        plan[l].push_back(i);
        load[l] += cost(i);
    }
    // the lanes do not record per-launch timings; the caller's event pair
    // brackets the whole batch
    linac_opts lane_opts{};
    if (opts) {
        lane_opts = *opts;
        lane_opts.ev_begin = nullptr;
        lane_opts.ev_end = nullptr;
        lane_opts.dominant_launches = nullptr;
        lane_opts.launch_events = nullptr;
        lane_opts.launch_cap = 0;
        lane_opts.validate = 0;
    }
    const linac_opts* lo = opts ? &lane_opts : nullptr;

    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e);
    if (lanes == 1) {  // one lane: the caller's stream, look-ahead as in linac_rref
        if (opts && opts->ev_begin) (void)hipEventRecord(opts->ev_begin, s);
        for (int32_t i : plan[0]) {
            e = rref_on(mats[i], ws, lo, s, true);
            if (e != hipSuccess) return hip_fail(e);
        }
        if (opts && opts->ev_end) (void)hipEventRecord(opts->ev_end, s);
        if (opts && opts->dominant_launches) *opts->dominant_launches = count;
        return LINAC_OK;
    }
    Lanes* L = nullptr;
    e = lanes_for_device(dev, &L);
    if (e != hipSuccess) return hip_fail(e);
    std::lock_guard<std::mutex> busy(L->busy);
    if (opts && opts->ev_begin) (void)hipEventRecord(opts->ev_begin, s);
    e = hipEventRecord(L->fork, s);
    if (e != hipSuccess) return hip_fail(e);
    // one host thread per lane enqueues that lane's instances, so a lane whose
    // queue is full never holds back the others
    std::vector<hipError_t> err(lanes, hipSuccess);
    std::vector<std::thread> threads;
    threads.reserve(lanes);
    for (int32_t l = 0; l < lanes; ++l) {
        threads.emplace_back([&, l]() {
            hipError_t le = hipSetDevice(dev);
            hipStream_t st = L->st[l];
            if (le == hipSuccess) le = hipStreamWaitEvent(st, L->fork, 0);
            char* lws = (char*)ws + per * (size_t)l;
            for (size_t q = 0; q < plan[l].size() && le == hipSuccess; ++q)
                le = rref_on(mats[plan[l][q]], lws, lo, st, false);
            const hipError_t re = hipEventRecord(L->done[l], st);
            err[l] = le != hipSuccess ? le : re;
        });
    }
    for (std::thread& t : threads) t.join();
    for (int32_t l = 0; l < lanes; ++l) {
        if (err[l] != hipSuccess) return hip_fail(err[l]);
        e = hipStreamWaitEvent(s, L->done[l], 0);
        if (e != hipSuccess) return hip_fail(e);
    }
    if (opts && opts->ev_end) (void)hipEventRecord(opts->ev_end, s);
    if (opts && opts->dominant_launches) *opts->dominant_launches = count;
    return LINAC_OK;
}

linac_status linac_rref_u64_workspace(int64_t m, int64_t n, size_t* bytes) {
    if (!bytes || m < 0 || n < 0) return LINAC_E_INVALID_ARG;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    *bytes = colstep_workspace(m, n, 0, true);
    return LINAC_OK;
}

linac_status linac_rref_u64(uint64_t* A, int64_t m, int64_t n, int64_t lda, uint64_t p,
                            int32_t* rank, int32_t* pivots, void* ws, size_t ws_bytes,
                            const linac_opts* opts, hipStream_t s) {
    if (m < 0 || n < 0 || lda < (n > 0 ? n : 1) || !rank) return LINAC_E_INVALID_ARG;
    if (m * n > 0 && !A) return LINAC_E_INVALID_ARG;
    if ((m < n ? m : n) > 0 && !pivots) return LINAC_E_INVALID_ARG;
    const linac_status st = check_field64(p);
    if (st != LINAC_OK) return st;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    if (!ws || ws_bytes < colstep_workspace(m, n, 0, true)) return LINAC_E_WORKSPACE;
    if (opts && opts->validate) {
        const linac_status vs = validate_range_t<uint64_t>(A, m, n, lda, p, (uint32_t*)ws, s);
        if (vs != LINAC_OK) return vs;
    }
    return hip_status(colstep_rref<uint64_t>(A, m, n, lda, p, rank, pivots, ws, s));
}

linac_status linac_solve_u64_workspace(int64_t m, int64_t n, int64_t k, size_t* bytes) {
    if (!bytes || m < 0 || n < 0 || k < 0) return LINAC_E_INVALID_ARG;
    if (!size_ok(m, n, k)) return LINAC_E_NOMEM;
    *bytes = colstep_workspace(m, n, k, true);
    return LINAC_OK;
}

linac_status linac_solve_u64(const uint64_t* A, int64_t m, int64_t n, int64_t lda, const uint64_t* B,
                             int64_t k, int64_t ldb, uint64_t p, uint64_t* X, int64_t ldx,
                             int32_t* rank, int32_t* pivots, uint8_t* consistent, void* ws,
                             size_t ws_bytes, const linac_opts* opts, hipStream_t s) {
    if (m < 0 || n < 0 || k < 0) return LINAC_E_INVALID_ARG;
    if (lda < (n > 0 ? n : 1) || ldb < (k > 0 ? k : 1) || ldx < (k > 0 ? k : 1))
        return LINAC_E_INVALID_ARG;
    if (!rank) return LINAC_E_INVALID_ARG;
    if (m * n > 0 && !A) return LINAC_E_INVALID_ARG;
    if (m * k > 0 && !B) return LINAC_E_INVALID_ARG;
    if (n * k > 0 && !X) return LINAC_E_INVALID_ARG;
    if (k > 0 && !consistent) return LINAC_E_INVALID_ARG;
    if ((m < n ? m : n) > 0 && !pivots) return LINAC_E_INVALID_ARG;
    const linac_status st = check_field64(p);
    if (st != LINAC_OK) return st;
    if (!size_ok(m, n, k)) return LINAC_E_NOMEM;
    if (!ws || ws_bytes < colstep_workspace(m, n, k, true)) return LINAC_E_WORKSPACE;
    if (opts && opts->validate) {
        linac_status vs = validate_range_t<uint64_t>(A, m, n, lda, p, (uint32_t*)ws, s);
        if (vs == LINAC_OK) vs = validate_range_t<uint64_t>(B, m, k, ldb, p, (uint32_t*)ws, s);
        if (vs != LINAC_OK) return vs;
    }
    return hip_status(
        colstep_solve<uint64_t>(A, m, n, lda, B, k, ldb, p, X, ldx, rank, pivots, consistent, ws, s));
}

linac_status linac_lup_workspace(int64_t m, int64_t n, int wide, size_t* bytes) {
    if (!bytes || m < 0 || n < 0) return LINAC_E_INVALID_ARG;
    if (!size_ok(m, n, 0)) return LINAC_E_NOMEM;
    *bytes = colstep_workspace(m, n, 0, wide != 0);
    return LINAC_OK;
}

linac_status linac_lup(uint32_t* A, int64_t m, int64_t n, int64_t lda, uint32_t p, int32_t* perm,
                       int32_t* rank, int32_t* pivots, void* ws, size_t ws_bytes,
                       const linac_opts* opts, hipStream_t s) {
    return lup_t<uint32_t>(A, m, n, lda, p, perm, rank, pivots, ws, ws_bytes, opts, s);
}

linac_status linac_lup_u64(uint64_t* A, int64_t m, int64_t n, int64_t lda, uint64_t p, int32_t* perm,
                           int32_t* rank, int32_t* pivots, void* ws, size_t ws_bytes,
                           const linac_opts* opts, hipStream_t s) {
    return lup_t<uint64_t>(A, m, n, lda, p, perm, rank, pivots, ws, ws_bytes, opts, s);
}

linac_status linac_check_prime_u64(uint64_t p) { return check_field64(p); }

linac_status linac_load_tuning(const char* json) {
    Tuning t;
    if (json) {
        linac_status st = parse_tuning(json, &t);
        if (st != LINAC_OK) return st;
    }
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune = t;
    return LINAC_OK;
}

}  // extern "C"
