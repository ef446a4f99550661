// Exported C ABI: argument validation, workspace sizing, error state and
// optional kernel timing.  Everything numeric happens in knn.hip and
// graph.hip; this file only checks and dispatches.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rsc_internal.hpp"

namespace rsc {

namespace {
thread_local std::string g_error;

struct ProfileEntry {
    std::string name;
    hipEvent_t start, stop;
};

thread_local const char *g_timer_prefix = nullptr;

struct Profiler {
    std::mutex mu;
    bool enabled = false;
    std::vector<ProfileEntry> pending;
    std::vector<hipEvent_t> free_events;
    std::map<std::string, std::pair<double, int64_t>> totals;

    hipEvent_t take_event() {
        if (!free_events.empty()) {
            hipEvent_t e = free_events.back();
            free_events.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    // Resolve recorded pairs into totals (waits for them).
    void drain() {
        for (auto &p : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(p.stop) == hipSuccess && hipEventElapsedTime(&ms, p.start, p.stop) == hipSuccess) {
                auto &t = totals[p.name];
                t.first += ms;
                t.second += 1;
            }
            free_events.push_back(p.start);
            free_events.push_back(p.stop);
        }
        pending.clear();
    }
};

Profiler &profiler() {
    static Profiler *p = new Profiler();  // leaked on purpose: outlives static destructors
    return *p;
}
}  // namespace

void set_error(const std::string &msg) { g_error = msg; }
void clear_error() { g_error.clear(); }

int hip_status(hipError_t e, const char *what) {
    if (e == hipSuccess) return RSC_OK;
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return RSC_ERR_HIP;
}

int launch_status(const char *what) { return hip_status(hipGetLastError(), what); }

TimerPrefix::TimerPrefix(const char *prefix) : prev_(g_timer_prefix) { g_timer_prefix = prefix; }
TimerPrefix::~TimerPrefix() { g_timer_prefix = prev_; }

ScopedTimer::ScopedTimer(const char *name, hipStream_t stream)
    : name_(g_timer_prefix ? std::string(g_timer_prefix) + name : std::string(name)), stream_(stream),
      start_(nullptr) {
    Profiler &p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    if (!p.enabled) return;
    hipEvent_t e = p.take_event();
    if (e && hipEventRecord(e, stream) == hipSuccess) start_ = e;
}

ScopedTimer::~ScopedTimer() {
    if (!start_) return;
    Profiler &p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    hipEvent_t e = p.take_event();
    if (e && hipEventRecord(e, stream_) == hipSuccess)
        p.pending.push_back({name_, static_cast<hipEvent_t>(start_), e});
}

}  // namespace rsc

using namespace rsc;

namespace {

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

int check_ws(void *ws, size_t have, size_t need) {
    if (need > have) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes, got " + std::to_string(have));
        return RSC_ERR_WORKSPACE;
    }
    if (!ws || !aligned(ws, 256)) {
        set_error("workspace must be a non-null, 256-byte aligned device pointer");
        return RSC_ERR_WORKSPACE;
    }
    return RSC_OK;
}

}  // namespace

extern "C" {

int rsc_abi_version(void) { return RSC_ABI_VERSION; }

const char *rsc_last_error(void) { return g_error.c_str(); }

size_t rsc_knn_workspace_bytes(int64_t n_query, int64_t n_ref, int32_t d, int32_t k, const rsc_knn_opts *opts) {
    KnnPlan p;
    // the square and rectangular forms need the same workspace
    if (knn_plan(n_query, n_ref, d, k, opts, false, &p) != RSC_OK) return 0;
    return knn_workspace(p, nullptr, nullptr);
}

static int knn_common(const float *Q, int64_t nq, const float *R, int64_t nr, int32_t d, int32_t k,
                      const rsc_knn_opts *opts, bool self_mode, int32_t *out_idx, float *out_dist, void *ws,
                      size_t ws_bytes, void *stream) {
    clear_error();
    KnnPlan p;
    int st = knn_plan(nq, nr, d, k, opts, self_mode, &p);
    if (st != RSC_OK) return st;
    if (!R || (nq > 0 && (!Q || !out_idx || !out_dist))) {
        set_error("null device pointer");
        return RSC_ERR_INVALID_ARG;
    }
    if (!aligned(Q, 4) || !aligned(R, 4) || !aligned(out_idx, 4) || !aligned(out_dist, 4)) {
        set_error("arrays must be 4-byte aligned");
        return RSC_ERR_INVALID_ARG;
    }
    if ((st = check_ws(ws, ws_bytes, knn_workspace(p, nullptr, nullptr))) != RSC_OK)
        return st;
    return knn_run(p, Q, R, out_idx, out_dist, ws, static_cast<hipStream_t>(stream));
}

int rsc_knn(const float *X, int64_t n, int32_t d, int32_t k, int32_t *out_idx, float *out_dist, void *workspace,
            size_t workspace_bytes, void *stream) {
    return knn_common(X, n, X, n, d, k, nullptr, true, out_idx, out_dist, workspace, workspace_bytes, stream);
}

int rsc_knn_opt(const float *X, int64_t n, int32_t d, int32_t k, const rsc_knn_opts *opts, int32_t *out_idx,
                float *out_dist, void *workspace, size_t workspace_bytes, void *stream) {
    return knn_common(X, n, X, n, d, k, opts, true, out_idx, out_dist, workspace, workspace_bytes, stream);
}

int rsc_knn_ex(const float *Q, int64_t n_query, const float *R, int64_t n_ref, int32_t d, int32_t k,
               const rsc_knn_opts *opts, int32_t *out_idx, float *out_dist, void *workspace, size_t workspace_bytes,
               void *stream) {
    return knn_common(Q, n_query, R, n_ref, d, k, opts, false, out_idx, out_dist, workspace, workspace_bytes,
                      stream);
}

int rsc_knn_read_stats(const void *workspace, size_t workspace_bytes, rsc_knn_stats *out, void *stream) {
    clear_error();
    if (!workspace || !out || workspace_bytes < sizeof(KnnCounters)) {
        set_error("need a kNN workspace and an output struct");
        return RSC_ERR_INVALID_ARG;
    }
    KnnCounters c;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int st = hip_status(hipMemcpyAsync(&c, workspace, sizeof(c), hipMemcpyDeviceToHost, s), "read stats");
    if (st != RSC_OK) return st;
    if ((st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK) return st;
    out->escalated_rows = c.flagged;
    out->rescanned_rows = c.rescanned;
    uint32_t rb = c.max_ratio_bits, nb = c.max_norm_bits;
    std::memcpy(&out->max_err_ratio, &rb, 4);
    std::memcpy(&out->max_ref_norm, &nb, 4);
    return RSC_OK;
}

int rsc_knn_read_escalated(const void *workspace, size_t workspace_bytes, int64_t n_query, int64_t n_ref, int32_t d,
                           int32_t k, const rsc_knn_opts *opts, int32_t square, int32_t *rows, int64_t cap,
                           int64_t *count, void *stream) {
    clear_error();
    KnnPlan p;
    int st = knn_plan(n_query, n_ref, d, k, opts, square != 0, &p);
    if (st != RSC_OK) return st;
    if (!workspace || !count || (cap > 0 && !rows) || cap < 0) {
        set_error("need a kNN workspace, a count and a host row array of cap entries");
        return RSC_ERR_INVALID_ARG;
    }
    if (workspace_bytes < knn_workspace(p, nullptr, nullptr)) {
        set_error("workspace smaller than the plan of these sizes");
        return RSC_ERR_WORKSPACE;
    }
    KnnBuffers b;
    knn_workspace(p, const_cast<void *>(workspace), &b);
    KnnCounters c;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = hip_status(hipMemcpyAsync(&c, b.counters, sizeof(c), hipMemcpyDeviceToHost, s), "read counters")) !=
        RSC_OK)
        return st;
    if ((st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK) return st;
    const int64_t flagged = std::min<int64_t>(c.flagged, p.nq);
    const int64_t take = std::min<int64_t>(flagged, cap);
    if (take > 0) {
        if ((st = hip_status(hipMemcpyAsync(rows, b.flag1, sizeof(int32_t) * (size_t)take, hipMemcpyDeviceToHost, s),
                             "read escalated rows")) != RSC_OK)
            return st;
        if ((st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK) return st;
    }
    *count = flagged;
    return RSC_OK;
}

size_t rsc_knn_batched_workspace_bytes(const int64_t *offsets, int32_t S, int32_t d, int32_t k) {
    if (d < 1 || d > 128 || k < 1 || k > 63) return 0;
    return batched_workspace_bytes(offsets, S, d, k);
}

int rsc_knn_batched(const float *X, const int64_t *offsets, int32_t S, int32_t d, int32_t k, int32_t *out_idx,
                    float *out_dist, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (d < 1 || k < 1) {
        set_error("need d >= 1 and k >= 1");
        return RSC_ERR_INVALID_ARG;
    }
    if (d > 128 || k > 63) {
        set_error("d > 128 or k > 63 is not supported by this build");
        return RSC_ERR_UNSUPPORTED;
    }
    if (!aligned(X, 4) || !aligned(out_idx, 4) || !aligned(out_dist, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return batched_run(X, offsets, S, d, k, out_idx, out_dist, workspace, workspace_bytes,
                       static_cast<hipStream_t>(stream));
}

int rsc_knn_batched_autotune(const float *X, const int64_t *offsets, int32_t S, int32_t d, int32_t k,
                             void *workspace, size_t workspace_bytes, void *stream, int32_t *chosen,
                             float *times_ms) {
    clear_error();
    if (d < 1 || k < 1 || d > 128 || k > 63) {
        set_error("need 1 <= d <= 128 and 1 <= k <= 63");
        return RSC_ERR_INVALID_ARG;
    }
    if (!aligned(X, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return batched_autotune(X, offsets, S, d, k, workspace, workspace_bytes, static_cast<hipStream_t>(stream),
                            chosen, times_ms);
}

const char *rsc_batch_policy_name(int32_t policy) { return batched_policy_name(policy); }

const char *rsc_batch_trial_name(int32_t trial) { return batched_trial_name(trial); }

size_t rsc_connectivities_workspace_bytes(int64_t n, int32_t k) {
    if (n < 1 || k < 1 || k > n || n > INT32_MAX - 1) return 0;
    return graph_workspace_bytes(n, k);
}

// Checks shared by the connectivities entry points (sizes, pointers,
// alignment, CSR capacity).
static int check_conn_args(const int32_t *idx, const float *dist, int64_t n, int32_t k, const int64_t *indptr,
                           const int32_t *indices, const float *data, int64_t cap, const int64_t *nnz,
                           const double *rho, const double *sigma) {
    if (n < 1 || k < 1 || k > n) {
        set_error("need n >= 1 and 1 <= k <= n");
        return RSC_ERR_INVALID_ARG;
    }
    if (n > INT32_MAX - 1) {
        set_error("n above 2^31-2 cannot be indexed by int32");
        return RSC_ERR_OVERFLOW;
    }
    if (k > 256) {
        set_error("k > 256 is not supported by this build");
        return RSC_ERR_UNSUPPORTED;
    }
    if (!idx || !dist || !indptr || !nnz || (k > 1 && (!indices || !data))) {
        set_error("null pointer");
        return RSC_ERR_INVALID_ARG;
    }
    if (!aligned(idx, 4) || !aligned(dist, 4) || !aligned(indptr, 8) || !aligned(indices, 4) ||
        !aligned(data, 4) || !aligned(rho, 8) || !aligned(sigma, 8)) {
        set_error("misaligned array");
        return RSC_ERR_INVALID_ARG;
    }
    const int64_t need = 2 * n * (int64_t)(k - 1);
    if (cap < need) {
        set_error("CSR capacity must be at least 2 n (k-1) = " + std::to_string(need));
        return RSC_ERR_CAPACITY;
    }
    return RSC_OK;
}

int rsc_connectivities(const int32_t *idx, const float *dist, int64_t n, int32_t k, int64_t *indptr,
                       int32_t *indices, float *data, int64_t cap, int64_t *nnz, double *rho, double *sigma,
                       void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    int st = check_conn_args(idx, dist, n, k, indptr, indices, data, cap, nnz, rho, sigma);
    if (st != RSC_OK) return st;
    st = check_ws(workspace, workspace_bytes, graph_workspace_bytes(n, k));
    if (st != RSC_OK) return st;
    return graph_run(idx, dist, n, k, indptr, indices, data, nnz, rho, sigma, workspace,
                     static_cast<hipStream_t>(stream));
}

size_t rsc_connectivities_noalloc_max_bytes(void) { return graph_noalloc_max_bytes(); }

int rsc_connectivities_noalloc(const int32_t *idx, const float *dist, int64_t n, int32_t k, int64_t *indptr,
                               int32_t *indices, float *data, int64_t cap, int64_t *nnz, double *rho, double *sigma,
                               void *stream) {
    clear_error();
    const int st = check_conn_args(idx, dist, n, k, indptr, indices, data, cap, nnz, rho, sigma);
    if (st != RSC_OK) return st;
    return graph_run_noalloc(idx, dist, n, k, indptr, indices, data, nnz, rho, sigma,
                             static_cast<hipStream_t>(stream));
}

// Sample offsets of the batched calls: S >= 1, offsets[0] = 0, each sample at
// least k rows, total <= 2^31 - 2.  Returns the total row count or -1.
static int64_t check_batch_offsets(const int64_t *offsets, int32_t S, int32_t k) {
    if (!offsets || S < 1 || offsets[0] != 0) return -1;
    for (int32_t s = 0; s < S; ++s)
        if (offsets[s + 1] - offsets[s] < (int64_t)k) return -1;
    if (offsets[S] > (int64_t)INT32_MAX - 1) return -1;
    return offsets[S];
}

size_t rsc_connectivities_batched_workspace_bytes(const int64_t *offsets, int32_t S, int32_t k) {
    const int64_t n = check_batch_offsets(offsets, S, k);
    if (n < 1 || k < 1 || k > 256) return 0;
    return graph_workspace_bytes(n, k, S);
}

int rsc_connectivities_batched(const int32_t *idx, const float *dist, const int64_t *offsets, int32_t S, int32_t k,
                               int64_t *indptr, int32_t *indices, float *data, int64_t cap, int64_t *nnz,
                               void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (k < 1) {
        set_error("need k >= 1");
        return RSC_ERR_INVALID_ARG;
    }
    const int64_t n = check_batch_offsets(offsets, S, k);
    if (n < 0) {
        set_error("offsets must hold S + 1 >= 2 entries from 0, every sample at least k rows, at most 2^31 - 2 in all");
        return RSC_ERR_INVALID_ARG;
    }
    int st = check_conn_args(idx, dist, n, k, indptr, indices, data, cap, nnz, nullptr, nullptr);
    if (st != RSC_OK) return st;
    st = check_ws(workspace, workspace_bytes, graph_workspace_bytes(n, k, S));
    if (st != RSC_OK) return st;
    return graph_run_batched(idx, dist, n, k, offsets, S, indptr, indices, data, nnz, workspace,
                             static_cast<hipStream_t>(stream));
}

size_t rsc_leiden_workspace_bytes(int64_t n, int64_t nnz) {
    if (n < 1 || n > INT32_MAX - 1 || nnz < 0 || nnz > ((int64_t)1 << 40)) return 0;
    return leiden_workspace_bytes(n, nnz);
}

int rsc_leiden(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
               double gamma, int32_t *labels, rsc_leiden_stats *stats, void *workspace, size_t workspace_bytes,
               void *stream) {
    clear_error();
    if (n < 1 || nnz < 0) {
        set_error("need n >= 1 and nnz >= 0");
        return RSC_ERR_INVALID_ARG;
    }
    if (n > INT32_MAX - 1) {
        set_error("n above 2^31-2 cannot be indexed by int32");
        return RSC_ERR_OVERFLOW;
    }
    if (nnz > ((int64_t)1 << 40)) {
        set_error("nnz above 2^40 is not supported");
        return RSC_ERR_UNSUPPORTED;
    }
    if (!(gamma > 0.0) || !std::isfinite(gamma)) {
        set_error("the resolution gamma must be finite and > 0");
        return RSC_ERR_INVALID_ARG;
    }
    if (!indptr || !labels || (nnz > 0 && (!indices || !weights))) {
        set_error("null pointer");
        return RSC_ERR_INVALID_ARG;
    }
    if (!aligned(indptr, 8) || !aligned(indices, 4) || !aligned(weights, 4) || !aligned(labels, 4)) {
        set_error("misaligned array");
        return RSC_ERR_INVALID_ARG;
    }
    const size_t need = leiden_workspace_bytes(n, nnz);
    if (need == 0) {
        set_error("leiden: workspace size query failed");
        return RSC_ERR_HIP;
    }
    int st = check_ws(workspace, workspace_bytes, need);
    if (st != RSC_OK) return st;
    return leiden_run(indptr, indices, weights, n, nnz, gamma, labels, stats, workspace,
                      static_cast<hipStream_t>(stream));
}

size_t rsc_partition_kmeans_workspace_bytes(int64_t n, int32_t d, int32_t parts) {
    if (n > INT32_MAX - 1 || d > 128) return 0;
    return kmeans_workspace_bytes(n, d, parts);
}

int rsc_partition_kmeans(const float *X, int64_t n, int32_t d, int32_t parts, const int32_t *init_rows,
                         int32_t iters, float *centroids, int32_t *assign, int64_t *offsets, int32_t *perm,
                         int64_t *relocated, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(X, 4) || !aligned(init_rows, 4) || !aligned(centroids, 4) || !aligned(assign, 4) ||
        !aligned(offsets, 8) || !aligned(perm, 4)) {
        set_error("misaligned array");
        return RSC_ERR_INVALID_ARG;
    }
    return kmeans_run(X, n, d, parts, init_rows, iters, centroids, assign, offsets, perm, relocated, workspace,
                      workspace_bytes, static_cast<hipStream_t>(stream));
}

size_t rsc_partition_lists_workspace_bytes(int32_t parts) {
    return parts < 1 ? 0 : partition_lists_workspace_bytes(parts);
}

int rsc_partition_lists(const int32_t *labels, int64_t n, int32_t parts, int64_t *offsets, int32_t *perm,
                        void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(labels, 4) || !aligned(offsets, 8) || !aligned(perm, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return partition_lists(labels, n, parts, offsets, perm, workspace, workspace_bytes,
                           static_cast<hipStream_t>(stream));
}

int rsc_partition_labels(const int32_t *idx, int64_t n, int32_t k, const int32_t *assign, int64_t n_assign,
                         int32_t *labels, void *stream) {
    clear_error();
    if (!aligned(idx, 4) || !aligned(assign, 4) || !aligned(labels, 4)) {
        set_error("misaligned array");
        return RSC_ERR_INVALID_ARG;
    }
    return partition_labels(idx, n, k, assign, n_assign, labels, static_cast<hipStream_t>(stream));
}

int rsc_router_create(rsc_router **out, int32_t d, int32_t hidden, int32_t parts, uint64_t seed) {
    clear_error();
    return router_create(out, d, hidden, parts, seed);
}

void rsc_router_destroy(rsc_router *router) { router_destroy(router); }

int rsc_router_info(const rsc_router *router, int32_t *d, int32_t *hidden, int32_t *parts, int64_t *n_params,
                    int64_t *steps) {
    clear_error();
    int dd = 0, hh = 0, pp = 0;
    const int st = router_info(router, &dd, &hh, &pp, n_params, steps);
    if (st == RSC_OK) {
        if (d) *d = dd;
        if (hidden) *hidden = hh;
        if (parts) *parts = pp;
    }
    return st;
}

size_t rsc_router_train_workspace_bytes(const rsc_router *router, int32_t batch, int64_t n) {
    return router_train_workspace(router, batch, n);
}

int rsc_router_train(rsc_router *router, const float *X, int64_t n, const int32_t *labels, int32_t m,
                     int32_t epochs, int32_t batch, float lr, float *loss_log, void *workspace,
                     size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(labels, 4) || !aligned(workspace, 256)) {
        set_error("misaligned labels or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return router_train(router, X, n, labels, m, epochs, batch, lr, loss_log, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream));
}

size_t rsc_router_gradients_workspace_bytes(const rsc_router *router, int64_t n) {
    return router_gradients_workspace(router, n);
}

int rsc_router_gradients(const rsc_router *router, const float *X, int64_t n, const int32_t *labels, int32_t m,
                         float *grad, float *loss, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(labels, 4) || !aligned(grad, 4) || !aligned(loss, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return router_gradients(router, X, n, labels, m, grad, loss, workspace, workspace_bytes,
                            static_cast<hipStream_t>(stream));
}

size_t rsc_router_infer_workspace_bytes(const rsc_router *router) { return router_infer_workspace(router); }

int rsc_router_logits(const rsc_router *router, const float *X, int64_t n, float *logits, void *workspace,
                      size_t workspace_bytes, void *stream) {
    clear_error();
    if (!logits || !aligned(logits, 4) || !aligned(workspace, 256)) {
        set_error("need an aligned logits array and workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return router_infer(router, X, n, nullptr, logits, 0, nullptr, nullptr, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream));
}

int rsc_router_probe(const rsc_router *router, const float *X, int64_t n, int32_t probes, int32_t *parts,
                     float *mass, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(parts, 4) || !aligned(mass, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return router_infer(router, X, n, nullptr, nullptr, probes, parts, mass, workspace, workspace_bytes,
                        static_cast<hipStream_t>(stream));
}

int rsc_router_save(const rsc_router *router, const char *path) {
    clear_error();
    return router_save(router, path);
}

int rsc_router_load(rsc_router *router, const char *path) {
    clear_error();
    return router_load(router, path);
}

size_t rsc_knn_probed_workspace_bytes(int64_t n, int32_t d, int32_t k, int32_t parts, int32_t probes) {
    if (n > INT32_MAX - 1) return 0;
    return probed_workspace_bytes(n, d, k, parts, probes);
}

int rsc_knn_probed(const float *X, int64_t n, int32_t d, int32_t k, const int64_t *offsets, const int32_t *perm,
                   int32_t parts, const int32_t *probe_parts, int32_t probes, const uint8_t *exact_rows,
                   int32_t *out_idx, float *out_dist, uint8_t *out_route, rsc_routed_stats *stats,
                   void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(offsets, 8) || !aligned(perm, 4) || !aligned(probe_parts, 4) || !aligned(out_idx, 4)) {
        set_error("misaligned array");
        return RSC_ERR_INVALID_ARG;
    }
    return probed_run(X, n, d, k, offsets, perm, parts, probe_parts, probes, exact_rows, nullptr, 0.f, out_idx,
                      out_dist, out_route, stats, workspace, workspace_bytes, static_cast<hipStream_t>(stream));
}

// Routed workspace: the probed search, then the router's scratch, the probe
// lists (n x probes int32) and the masses (n float32).
static size_t routed_layout(const rsc_router *router, int64_t n, int32_t d, int32_t k, int32_t parts,
                            int32_t probes, void *ws, size_t *off_infer, size_t *off_parts, size_t *off_mass) {
    const size_t a = probed_workspace_bytes(n, d, k, parts, probes);
    const size_t b = router_infer_workspace(router);
    if (a == 0 || b == 0) return 0;
    Carver cv(ws);
    cv.take<char>(a);
    const size_t oi = cv.used;
    cv.take<char>(b);
    const size_t op = cv.used;
    cv.take<int32_t>((size_t)n * probes);
    const size_t om = cv.used;
    cv.take<float>((size_t)n);
    if (off_infer) *off_infer = oi;
    if (off_parts) *off_parts = op;
    if (off_mass) *off_mass = om;
    return cv.used;
}

size_t rsc_knn_routed_workspace_bytes(const rsc_router *router, int64_t n, int32_t d, int32_t k, int32_t parts,
                                      int32_t probes) {
    if (!router || n > INT32_MAX - 1) return 0;
    return routed_layout(router, n, d, k, parts, probes, nullptr, nullptr, nullptr, nullptr);
}

int rsc_knn_routed(const rsc_router *router, const float *X, int64_t n, int32_t d, int32_t k,
                   const int64_t *offsets, const int32_t *perm, int32_t parts, int32_t probes, float mass_threshold,
                   int32_t *out_idx, float *out_dist, uint8_t *out_route, rsc_routed_stats *stats, void *workspace,
                   size_t workspace_bytes, void *stream) {
    clear_error();
    int rd = 0, rp = 0;
    if (!router || router_shape(router, &rd, &rp) != RSC_OK || rd != d || rp != parts) {
        set_error("knn_routed: the router's input width and partition count must equal d and parts");
        return RSC_ERR_INVALID_ARG;
    }
    if (!aligned(offsets, 8) || !aligned(perm, 4) || !aligned(out_idx, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    if (!(mass_threshold >= 0.f && mass_threshold <= 1.f)) {
        set_error("knn_routed: mass_threshold must lie in [0, 1]");
        return RSC_ERR_INVALID_ARG;
    }
    size_t oi = 0, op = 0, om = 0;
    const size_t need = routed_layout(router, n, d, k, parts, probes, nullptr, &oi, &op, &om);
    if (need == 0) {
        set_error("knn_routed: unsupported size (need n >= k, d <= 128, k <= 63, parts <= 4096, probes <= 64)");
        return RSC_ERR_UNSUPPORTED;
    }
    int st = check_ws(workspace, workspace_bytes, need);
    if (st != RSC_OK) return st;
    char *base = static_cast<char *>(workspace);
    int32_t *parts_buf = reinterpret_cast<int32_t *>(base + op);
    float *mass_buf = reinterpret_cast<float *>(base + om);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if ((st = router_infer(router, X, n, nullptr, nullptr, probes, parts_buf, mass_buf, base + oi, op - oi, s)) !=
        RSC_OK)
        return st;
    return probed_run(X, n, d, k, offsets, perm, parts, parts_buf, probes, nullptr, mass_buf, mass_threshold,
                      out_idx, out_dist, out_route, stats, workspace, oi, s);
}

size_t rsc_edistance_groups_workspace_bytes(int64_t n, int64_t n_groups) {
    return edistance_groups_workspace_bytes(n, n_groups);
}

int rsc_edistance_groups(const int32_t *labels, int64_t n, int64_t n_groups, int64_t *offsets, int32_t *cells,
                         void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(labels, 4) || !aligned(offsets, 8) || !aligned(cells, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return edistance_groups(labels, n, n_groups, offsets, cells, workspace, workspace_bytes,
                            static_cast<hipStream_t>(stream));
}

size_t rsc_edistance_sums_workspace_bytes(int64_t n_groups, int64_t n_pairs, int64_t n_cells, int32_t d) {
    return edistance_sums_workspace_bytes(n_groups, n_pairs, n_cells, d);
}

int rsc_edistance_sums(const float *X, int64_t n, int32_t d, const int64_t *offsets, int64_t n_groups,
                       const int32_t *cells, const int32_t *pairs, int64_t n_pairs, double *sums, void *workspace,
                       size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(X, 4) || !aligned(cells, 4) || !aligned(sums, 8) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return edistance_sums(X, n, d, offsets, n_groups, cells, pairs, n_pairs, sums, workspace, workspace_bytes,
                          static_cast<hipStream_t>(stream));
}

size_t rsc_edistance_pairwise_workspace_bytes(int64_t n_groups, int64_t n_cells, int32_t d) {
    return edistance_pairwise_workspace_bytes(n_groups, n_cells, d);
}

int rsc_edistance_pairwise(const float *X, int64_t n, int32_t d, const int64_t *offsets, int64_t n_groups,
                           const int32_t *cells, double *E, double *D, void *workspace, size_t workspace_bytes,
                           void *stream) {
    clear_error();
    if (!aligned(X, 4) || !aligned(cells, 4) || !aligned(E, 8) || !aligned(D, 8) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return edistance_pairwise(X, n, d, offsets, n_groups, cells, E, D, workspace, workspace_bytes,
                              static_cast<hipStream_t>(stream));
}

size_t rsc_edistance_onesided_workspace_bytes(int64_t n_groups, int64_t n_cells, int32_t d) {
    return edistance_onesided_workspace_bytes(n_groups, n_cells, d);
}

int rsc_edistance_onesided(const float *X, int64_t n, int32_t d, const int64_t *offsets, int64_t n_groups,
                           const int32_t *cells, int64_t ref, double *E, void *workspace, size_t workspace_bytes,
                           void *stream) {
    clear_error();
    if (!aligned(X, 4) || !aligned(cells, 4) || !aligned(E, 8) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return edistance_onesided(X, n, d, offsets, n_groups, cells, ref, E, workspace, workspace_bytes,
                              static_cast<hipStream_t>(stream));
}

size_t rsc_pca_workspace_bytes(int64_t n, int32_t p, int32_t k) { return pca_workspace_bytes(n, p, k); }

int rsc_pca_covariance(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int32_t p,
                       double *mean, double *cov, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(indptr, 8) || !aligned(indices, 4) || !aligned(data, 4) || !aligned(mean, 8) || !aligned(cov, 8) ||
        !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return pca_covariance(indptr, indices, data, n, p, mean, cov, workspace, workspace_bytes,
                          static_cast<hipStream_t>(stream));
}

int rsc_pca(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int32_t p, int32_t k,
            double *mean, double *cov, double *evals, double *loadings, float *scores, void *workspace,
            size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(indptr, 8) || !aligned(indices, 4) || !aligned(data, 4) || !aligned(mean, 8) || !aligned(cov, 8) ||
        !aligned(evals, 8) || !aligned(loadings, 8) || !aligned(scores, 4) || !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return pca_run(indptr, indices, data, n, p, k, mean, cov, evals, loadings, scores, workspace, workspace_bytes,
                   static_cast<hipStream_t>(stream));
}

size_t rsc_umap_workspace_bytes(int64_t n, int64_t nnz, int32_t dim, int32_t neg) {
    return umap_workspace_bytes(n, nnz, dim, neg);
}

int rsc_umap_layout(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
                    int32_t dim, float *Y, int32_t n_epochs, double a, double b, double gamma, double alpha0,
                    int32_t neg, uint64_t seed, void *workspace, size_t workspace_bytes, void *stream) {
    clear_error();
    if (!aligned(indptr, 8) || !aligned(indices, 4) || !aligned(weights, 4) || !aligned(Y, 4) ||
        !aligned(workspace, 256)) {
        set_error("misaligned array or workspace");
        return RSC_ERR_INVALID_ARG;
    }
    return umap_layout(indptr, indices, weights, n, nnz, dim, Y, n_epochs, a, b, gamma, alpha0, neg, seed, workspace,
                       workspace_bytes, static_cast<hipStream_t>(stream));
}

int rsc_profile_enable(int enable) {
    Profiler &p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    p.enabled = enable != 0;
    return RSC_OK;
}

int rsc_profile_reset(void) {
    Profiler &p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    p.drain();
    p.totals.clear();
    return RSC_OK;
}

int rsc_profile_get(const char *name, double *total_ms, int64_t *launches) {
    clear_error();
    if (!name || !total_ms || !launches) {
        set_error("null argument");
        return RSC_ERR_INVALID_ARG;
    }
    Profiler &p = profiler();
    std::lock_guard<std::mutex> lock(p.mu);
    p.drain();
    auto it = p.totals.find(name);
    *total_ms = it == p.totals.end() ? 0.0 : it->second.first;
    *launches = it == p.totals.end() ? 0 : it->second.second;
    return RSC_OK;
}

}  // extern "C"
