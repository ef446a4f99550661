// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>

#include "../../include/rsc.h"

namespace rsc {

// Thread-local error message behind rsc_last_error().
void set_error(const std::string &msg);
void clear_error();

// Record a HIP failure (if any) and turn it into RSC_ERR_HIP.
int hip_status(hipError_t e, const char *what);
// Check the last launch error.
int launch_status(const char *what);

// Optional per-kernel event timing (rsc_profile_*).  When enabled, a
// ScopedTimer records one event before and one after the launches made in
// its scope on `stream` and files the pair under `name`.
class ScopedTimer {
  public:
    ScopedTimer(const char *name, hipStream_t stream);
    ~ScopedTimer();
    ScopedTimer(const ScopedTimer &) = delete;
    ScopedTimer &operator=(const ScopedTimer &) = delete;

  private:
    std::string name_;
    hipStream_t stream_;
    void *start_;
};

// While a TimerPrefix lives, the timers this thread starts file their pairs
// under prefix + name (a stage that runs a whole kNN call inside another
// call, such as k-means' assignments, keeps its kernels apart from the
// outer call's own).
class TimerPrefix {
  public:
    explicit TimerPrefix(const char *prefix);
    ~TimerPrefix();
    TimerPrefix(const TimerPrefix &) = delete;
    TimerPrefix &operator=(const TimerPrefix &) = delete;

  private:
    const char *prev_;
};

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

// Carves 256-byte aligned sub-buffers out of a workspace, or only counts.
struct Carver {
    char *base;
    size_t used = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        size_t off = used;
        used = align_up(used + count * sizeof(T));
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
};

// ---- kNN stages (knn.hip) -------------------------------------------------

// Device counters of one kNN call, at the start of the workspace.
struct KnnCounters {
    int32_t flagged;          // rows whose first certificate failed (escalated)
    uint32_t max_ratio_bits;  // float bits of the largest error ratio seen
    uint32_t max_norm_bits;   // float bits of max_j ||y_j||
    int32_t flagged2;         // escalated rows whose second certificate failed
    int32_t rescanned;        // rows recomputed exhaustively
    int32_t pad[3];
};

struct KnnPlan {
    int64_t nq, nr;
    int d, k, screen, half;  // screen width (32 or 64) = 2 x list length per contraction half
    int dh;                // half of the padded contraction length
    bool self_mode;        // queries are the references (self forced to slot 0)
    int64_t nblk;          // 32-row reference blocks
    int splits;            // reference ranges of the main screen
    int precision;         // rsc_precision of the screen
    int metric;            // rsc_metric
    int resid;             // FP8 residual variant: reference partitions (0 = off)
};

struct KnnBuffers {
    KnnCounters *counters;
    float *nrow, *packed, *norms;
    float *scal;      // FP8 per-dimension scales
    uint32_t *amax;   // FP8 per-dimension absmax bits
    int32_t *cand_idx;
    float *cand_key;
    int32_t *flag1, *flag2;
    int32_t *esc_idx;
    float *esc_key;
    float *qn, *rn;   // unit-normalised queries / references (cosine metric)
    // FP8 residual variant
    float *cent;          // partition centroids, resid x d
    int32_t *assign, *perm, *init, *map;
    int32_t *qcount;  // the number of queries screened through perm (device)
    void *order_ws;   // reduced-precision screens: workspace of the spatial query order
    int32_t *blk_part;    // partition of each packed block, 4 copies per block
    int64_t *poff, *pblk;
    void *kws;            // k-means workspace
    size_t kws_bytes;
};

// Arguments of the float64 rerank (knn.hip).
struct RerankArgs {
    const float *Q;
    int64_t nq;
    const int32_t *qlist;   // optional: slot -> row
    const int32_t *qcount;
    int qcap;
    const float *R;
    int d, k, S, KP, P;
    int self_mode;
    int certify;            // 0: approximate screen, never flag rows
    int metric;             // rsc_metric of the reported distances
    double cosine_eps;      // cosine: bound on |screened key - (2 D - 1)| for unit vectors
    const int32_t *cand_idx;
    const float *cand_key;
    double eps_coef;
    KnnCounters *counters;
    int32_t *flag_out;   // rows that fail the certificate
    int32_t *flag_count;
    int32_t *out_idx;
    float *out_dist;
};

// Fill a plan; returns RSC_OK or an error status (with message set).
int knn_plan(int64_t nq, int64_t nr, int d, int k, const rsc_knn_opts *opts, bool self_mode, KnnPlan *plan);
// Bytes of workspace for a plan; with ws != nullptr also carves the buffers.
size_t knn_workspace(const KnnPlan &p, void *ws, KnnBuffers *out);
// With qlist (device rows) the query slots are the first min(*qcount, p.nq)
// rows of the list; outputs are written at those rows.
int knn_run(const KnnPlan &p, const float *Q, const float *R, int32_t *out_idx, float *out_dist, void *ws,
            hipStream_t stream, const int32_t *qlist = nullptr, const int32_t *qcount = nullptr);

// Pieces of the exact path reused by the batched form (knn.hip).
double knn_eps_coefficient(int d);
// init counters, norms, FP32 packing (optionally per sample: blk_sample,
// boff, soff device arrays).
int knn_prep_fp32(const KnnPlan &p, const float *R, const KnnBuffers &b, const int32_t *blk_sample,
                  const int64_t *boff, const int64_t *soff, hipStream_t stream);
int knn_launch_rerank(const RerankArgs &ra, int64_t slots, const char *name, hipStream_t stream);
// exhaustive float64 rescan of the rows flagged in b (first certificate only
// when there was no escalation); soff/nsamples restrict each row to its sample.
// (uses p.metric for the distances)
int knn_launch_rescan(const KnnPlan &p, const float *Q, const float *R, const KnnBuffers &b, int esc_cap,
                      int32_t *out_idx, float *out_dist, const int64_t *soff, int nsamples, hipStream_t stream);

namespace scr {
struct ScreenArgs;
}
// Squared norms of R's rows into nrow and their maximum into counters
// (counters re-initialised).
int knn_norms(const float *R, int64_t nr, int d, float *nrow, KnnCounters *counters, hipStream_t stream);
// FP32 packing of nblk blocks whose packed row 32b + c is row_map[32b + c]
// of R (-1: padding with an infinite norm).
int knn_pack_mapped(int dh, const float *R, const float *nrow, int64_t nr, int d, int64_t nblk, float *packed,
                    float *norms, const int32_t *row_map, hipStream_t stream);
size_t knn_packed_floats(int dh, int64_t nblk);
int knn_launch_screen(int dh, const scr::ScreenArgs &a, unsigned gx, int half_width, const char *name,
                      hipStream_t s);
// Reduced-precision screens (knn_lowp.hip).
int lowp_steps(int precision, int d);
int lowp_qb(int precision, int d);
int lowp_queries_per_group(int precision, int d);
size_t lowp_packed_bytes(int precision, int64_t nblk, int d);
// Packs the references (rmap: packed slot -> row, or null for row order).
int lowp_prepare(const KnnPlan &p, const float *Q, const float *R, void *packed, float *norms, float *scal,
                 uint32_t *amax, const int32_t *rmap, hipStream_t stream);
int lowp_screen(const KnnPlan &p, const scr::ScreenArgs &a, unsigned gx, hipStream_t s);
// FP8 residual variant: partitions, residual scales and the partition-ordered
// packing (into b.packed / b.norms, with b.map and b.blk_part); then, after
// the screen, the candidates' packed rows turned back into row ids.
int lowp_prepare_resid(const KnnPlan &p, const float *R, const KnnBuffers &b, hipStream_t stream);
int lowp_unmap(const KnnPlan &p, const KnnBuffers &b, hipStream_t stream);
// Candidates from packed slots to rows through the packing's row map.
int lowp_unmap_rows(const KnnPlan &p, const KnnBuffers &b, const int32_t *rmap, hipStream_t stream);

// Spatial order of query rows (query_order.hip): perm = the rows sorted by a
// Morton code of their first three coordinates.
size_t query_order_workspace(int64_t nq);
int query_order_run(const float *Q, int64_t nq, int d, void *ws, int32_t *perm, hipStream_t s);

// Batched form (knn_batched.hip).
size_t batched_workspace_bytes(const int64_t *offsets, int S, int d, int k);
int batched_run(const float *X, const int64_t *offsets, int S, int d, int k, int32_t *out_idx, float *out_dist,
                void *ws, size_t ws_bytes, hipStream_t s);
int batched_autotune(const float *X, const int64_t *offsets, int S, int d, int k, void *ws, size_t ws_bytes,
                     hipStream_t s, int32_t *chosen, float *times_ms);
const char *batched_policy_name(int pol);
const char *batched_trial_name(int trial);

// ---- routed form (partition.hip, router.hip, routed.hip) -----------------

size_t kmeans_workspace_bytes(int64_t n, int d, int P);
int kmeans_run(const float *X, int64_t n, int d, int P, const int32_t *init_rows, int iters, float *C,
               int32_t *assign, int64_t *offsets, int32_t *perm, int64_t *relocated, void *ws, size_t ws_bytes,
               hipStream_t s);
size_t partition_lists_workspace_bytes(int P);
int partition_lists(const int32_t *assign, int64_t n, int P, int64_t *offsets, int32_t *perm, void *ws,
                    size_t ws_bytes, hipStream_t s);
int partition_labels(const int32_t *idx, int64_t n, int k, const int32_t *assign, int64_t n_assign, int32_t *labels,
                     hipStream_t s);

int router_create(rsc_router **out, int d, int hidden, int parts, uint64_t seed);
void router_destroy(rsc_router *R);
int router_info(const rsc_router *R, int *d, int *hidden, int *parts, int64_t *n_params, int64_t *step);
size_t router_train_workspace(const rsc_router *R, int batch, int64_t n);
int router_train(rsc_router *R, const float *X, int64_t n, const int32_t *labels, int m, int epochs, int batch,
                 float lr, float *loss_log, void *ws, size_t ws_bytes, hipStream_t s);
size_t router_gradients_workspace(const rsc_router *R, int64_t n);
int router_gradients(const rsc_router *R, const float *X, int64_t n, const int32_t *labels, int m, float *grad_out,
                     float *loss_out, void *ws, size_t ws_bytes, hipStream_t s);
size_t router_infer_workspace(const rsc_router *R);
// Logits (logits != nullptr) or the top `probes` partitions and their mass
// of n rows (rows of X, or X[list[i]]).
int router_infer(const rsc_router *R, const float *X, int64_t n, const int32_t *list, float *logits, int probes,
                 int32_t *parts, float *mass, void *ws, size_t ws_bytes, hipStream_t s);
int router_save(const rsc_router *R, const char *path);
int router_load(rsc_router *R, const char *path);
int router_shape(const rsc_router *R, int *d, int *parts);

size_t probed_workspace_bytes(int64_t n, int d, int k, int P, int probes);
// mass/threshold: rows whose mass is below the threshold go to exact search
// (instead of, or besides, exact_rows).
int probed_run(const float *X, int64_t n, int d, int k, const int64_t *offsets, const int32_t *perm, int P,
               const int32_t *probe_parts, int probes, const uint8_t *exact_rows, const float *mass,
               float threshold, int32_t *out_idx, float *out_dist, uint8_t *out_route, rsc_routed_stats *stats,
               void *ws, size_t ws_bytes, hipStream_t s);

// ---- energy distance (edistance.hip) -------------------------------------

size_t edistance_sums_workspace_bytes(int64_t G, int64_t npairs, int64_t ncells, int d);
size_t edistance_pairwise_workspace_bytes(int64_t G, int64_t ncells, int d);
size_t edistance_onesided_workspace_bytes(int64_t G, int64_t ncells, int d);
size_t edistance_groups_workspace_bytes(int64_t n, int64_t G);
int edistance_groups(const int32_t *labels, int64_t n, int64_t G, int64_t *offsets, int32_t *cells, void *ws,
                     size_t ws_bytes, hipStream_t s);
int edistance_sums(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G, const int32_t *cells,
                   const int32_t *pairs, int64_t npairs, double *sums, void *ws, size_t ws_bytes, hipStream_t s);
int edistance_pairwise(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G, const int32_t *cells,
                       double *E, double *D, void *ws, size_t ws_bytes, hipStream_t s);
int edistance_onesided(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G, const int32_t *cells,
                       int64_t ref, double *E, void *ws, size_t ws_bytes, hipStream_t s);

// ---- sparse PCA (pca.hip) -------------------------------------------------

size_t pca_workspace_bytes(int64_t n, int p, int k);
int pca_covariance(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int p, double *mean,
                   double *cov, void *ws, size_t ws_bytes, hipStream_t s);
int pca_run(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int p, int k, double *mean,
            double *cov, double *evals, double *loadings, float *Z, void *ws, size_t ws_bytes, hipStream_t s);

// ---- UMAP layout (umap.hip) -----------------------------------------------

size_t umap_workspace_bytes(int64_t n, int64_t nnz, int dim, int neg);
int umap_layout(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
                int dim, float *Y, int n_epochs, double a, double b, double gamma, double alpha0, int neg,
                uint64_t seed, void *ws, size_t ws_bytes, hipStream_t s);

// ---- graph stages (graph.hip) --------------------------------------------

// Workspace of a graph build over n rows of k slots; S > 0 adds room for
// the offsets of S samples (the batched form).
size_t graph_workspace_bytes(int64_t n, int k, int32_t S = 0);
int graph_run(const int32_t *idx, const float *dist, int64_t n, int k, int64_t *indptr, int32_t *indices,
              float *data, int64_t *nnz, double *rho, double *sigma, void *ws, hipStream_t stream);
// As graph_run, with every edge checked to stay inside its row's sample
// (seg_host: HOST int64 [S + 1] sample offsets, validated by the caller).
int graph_run_batched(const int32_t *idx, const float *dist, int64_t n, int k, const int64_t *seg_host, int32_t S,
                      int64_t *indptr, int32_t *indices, float *data, int64_t *nnz, void *ws, hipStream_t stream);
// As graph_run, with the workspace taken from a fixed device array of
// graph_noalloc_max_bytes() bytes instead of the caller (RSC_ERR_CAPACITY
// when the problem needs more).
size_t graph_noalloc_max_bytes();
int graph_run_noalloc(const int32_t *idx, const float *dist, int64_t n, int k, int64_t *indptr, int32_t *indices,
                      float *data, int64_t *nnz, double *rho, double *sigma, hipStream_t stream);

// ---- Leiden communities (leiden.hip) ----------------------------------------

size_t leiden_workspace_bytes(int64_t n, int64_t nnz);
int leiden_run(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
               double gamma, int32_t *labels, rsc_leiden_stats *stats, void *ws, hipStream_t s);

}  // namespace rsc
