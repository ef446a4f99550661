/*
 * rsc.h -- C ABI of the MI355X (gfx950) neighbourhood-graph library.
 *
 * The library builds the graph that the paper's single-cell workflow derives
 * from a cells x PCA-components embedding (Methods, "Dimensionality reduction
 * and graph analysis": k-nearest-neighbour graph construction, stored as the
 * sparse distance and connectivity matrices scanpy keeps in .obsp):
 *
 *   rsc_knn             exact k nearest neighbours (Euclidean; the squared
 *                       distance ||x_i - x_j||^2 of Methods, "Custom GPU
 *                       kernels"), ties broken towards the lower index;
 *   rsc_connectivities  the UMAP fuzzy simplicial set built on that kNN
 *                       result: per-cell rho and sigma (smooth-kNN
 *                       calibration to log2 k), directed weights
 *                       exp(-max(0, d - rho)/sigma), and their fuzzy union
 *                       a + b - a*b as a CSR matrix (Methods,
 *                       "Implementation": CSR for row access).
 *
 * Conventions shared by every call:
 *   - Array arguments are DEVICE pointers on the current HIP device, owned
 *     by the caller; the library never frees them.  Host pointers are named
 *     as such.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Every call only enqueues work on it, except where a call says it
 *     synchronises.
 *   - `workspace` is caller-owned device scratch of at least the size the
 *     matching *_workspace_bytes call returns, 256-byte aligned.  The
 *     library allocates no device memory in these calls.  Work enqueued by
 *     two calls that share a workspace must not overlap in time.
 *   - Matrices are row-major and C-contiguous.  Float inputs must be
 *     4-byte aligned; the embedding must hold finite values.
 *   - Every call returns an rsc_status.  Arguments are validated before
 *     anything is enqueued; on failure nothing is enqueued and
 *     rsc_last_error() describes the problem.  HIP errors reported by the
 *     runtime map to RSC_ERR_HIP.
 *   - Row counts are int64 but indices are int32: n must not exceed
 *     2^31 - 1 (RSC_ERR_OVERFLOW).  CSR row pointers are int64, so nnz is
 *     not limited to int32.
 */
#ifndef RSC_H
#define RSC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSC_ABI_VERSION 1

typedef enum {
    RSC_OK = 0,
    RSC_ERR_INVALID_ARG = -1, /* bad size, null pointer, misaligned buffer, bad option */
    RSC_ERR_HIP = -2,         /* a HIP runtime call or launch failed */
    RSC_ERR_NO_MEMORY = -3,   /* host-side allocation failed */
    RSC_ERR_CAPACITY = -4,    /* output capacity smaller than the call can need */
    RSC_ERR_OVERFLOW = -5,    /* a size exceeds what the int32 indices can address */
    RSC_ERR_UNSUPPORTED = -6, /* valid request outside what this build implements */
    RSC_ERR_WORKSPACE = -7,   /* workspace null, too small or misaligned */
    RSC_ERR_BAD_GRAPH = -8    /* kNN lists handed to rsc_connectivities are malformed */
} rsc_status;

/* ABI version of the loaded library (RSC_ABI_VERSION of its build). */
int rsc_abi_version(void);

/* Message for the last failing call on this host thread ("" if none).
 * Valid until the next call on the same thread. */
const char *rsc_last_error(void);

/* ---------------------------------------------------------------------- */
/* Exact kNN                                                               */
/* ---------------------------------------------------------------------- */

typedef enum { RSC_FP32 = 0, RSC_BF16 = 1, RSC_FP8_E4M3 = 2 } rsc_precision;

/*
 * Options of the screening stage.  A zero-initialised struct (or NULL)
 * selects the default: FP32 screen of width 32 (64 for k > 16) followed by
 * the exactness certificate and rescan, i.e. the exact result.
 *   precision  arithmetic of the distance screen on the matrix cores:
 *              RSC_FP32      exact result (certified, see rsc_knn);
 *              RSC_BF16      BF16 operands, FP32 accumulation;
 *              RSC_FP8_E4M3  OCP e4m3 operands with per-dimension absmax
 *                            scaling (s_t = max|y_t| / 448), FP32 accumulation.
 *              The reduced-precision forms keep the 64 smallest screened keys
 *              per query and re-rank them with float64 distances; they are
 *              approximate (no certificate): judge them by recall@k.
 *   screen     candidates kept per query: 32 or 64 for RSC_FP32 (must exceed
 *              k), 64 for the reduced-precision forms; 0 = default.
 */
typedef struct {
    int32_t precision;
    int32_t screen;
    int32_t reserved0;
    int32_t reserved1;
} rsc_knn_opts;

/* Counters a kNN call leaves in its workspace (read with rsc_knn_read_stats). */
typedef struct {
    int64_t escalated_rows; /* rows the first screen could not certify (screened again, wider) */
    int64_t rescanned_rows; /* rows no screen could certify (recomputed exhaustively in float64) */
    float max_err_ratio;    /* largest |screened key - exact key| / certificate bound seen */
    float max_ref_norm;     /* max_j ||y_j|| over the references, float32 */
} rsc_knn_stats;

/* Workspace bytes for rsc_knn (n_query = n_ref = n) or rsc_knn_ex. */
size_t rsc_knn_workspace_bytes(int64_t n_query, int64_t n_ref, int32_t d, int32_t k, const rsc_knn_opts *opts);

/*
 * k nearest neighbours of every row of X among the rows of X.
 *   X         device, n x d float32 embedding (cells x components).
 *   n, d, k   1 <= k <= n <= 2^31-1, 1 <= d <= 128, k <= 63.
 *   out_idx   device, n x k int32: row i lists i itself in column 0, then
 *             the k-1 nearest other rows ordered by (distance, index).
 *   out_dist  device, n x k float32 Euclidean distances (column 0 is 0),
 *             each the float64 distance from direct differences rounded
 *             once to float32.
 * Screening runs on the MFMA units in the chosen precision; candidates are
 * re-ranked with float64 distances, and rows whose screen cannot be proved
 * to contain the true neighbours are recomputed exhaustively, so the result
 * is exact for every row.
 */
int rsc_knn(const float *X, int64_t n, int32_t d, int32_t k, int32_t *out_idx, float *out_dist, void *workspace,
            size_t workspace_bytes, void *stream);

/* rsc_knn with screening options (precision forms of the same square
 * problem; opts may be NULL for the exact default). */
int rsc_knn_opt(const float *X, int64_t n, int32_t d, int32_t k, const rsc_knn_opts *opts, int32_t *out_idx,
                float *out_dist, void *workspace, size_t workspace_bytes, void *stream);

/*
 * Rectangular form: k nearest rows of R for every row of Q (no self
 * column: all k slots come from R, ordered by (distance, index)).
 *   Q  device n_query x d float32;  R  device n_ref x d float32.
 *   1 <= k <= n_ref, k <= 63.  opts may be NULL.
 */
int rsc_knn_ex(const float *Q, int64_t n_query, const float *R, int64_t n_ref, int32_t d, int32_t k,
               const rsc_knn_opts *opts, int32_t *out_idx, float *out_dist, void *workspace, size_t workspace_bytes,
               void *stream);

/* Copy the counters of the last kNN call that used `workspace` into host
 * memory `out`.  Synchronises `stream`. */
int rsc_knn_read_stats(const void *workspace, size_t workspace_bytes, rsc_knn_stats *out, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched exact kNN (many independent samples, one persistent launch)     */
/* ---------------------------------------------------------------------- */

/* Number of scheduling policies the batched autotuner measures. */
#define RSC_BATCH_POLICIES 6

/*
 * A batch is S samples stored back to back in one matrix X: sample s is rows
 * offsets[s] .. offsets[s+1]-1 (offsets is a HOST int64 array of S+1
 * entries, offsets[0] = 0, every sample at least k rows, total <= 2^31-2).
 * Each sample is its own exact kNN problem (the paper analyses large
 * collections chunk by chunk along the cell axis: Methods, "Memory
 * management and scaling"); results use global row ids, so the kNN graph is
 * block-diagonal and rsc_connectivities applied to the whole output gives the
 * per-sample connectivities at once.
 */
size_t rsc_knn_batched_workspace_bytes(const int64_t *offsets, int32_t S, int32_t d, int32_t k);

/* Exact kNN of every sample (same output layout and exactness as rsc_knn,
 * neighbours drawn from the row's own sample).  Uses the scheduling policy
 * the autotuner chose for this batch shape, else a default.  Synchronises
 * `stream` once (to upload the work list into the workspace). */
int rsc_knn_batched(const float *X, const int64_t *offsets, int32_t S, int32_t d, int32_t k, int32_t *out_idx,
                    float *out_dist, void *workspace, size_t workspace_bytes, void *stream);

/* Time every scheduling policy on this batch (screen only, HIP events) and
 * remember the fastest for batches of the same shape (device, d, k and the
 * histogram of log2 sample sizes); with RSC_AUTOTUNE_CACHE=<file> in the
 * environment the choice is also read from / written to that file.
 * chosen (host, may be NULL): the policy index; times_ms (host, may be NULL):
 * RSC_BATCH_POLICIES measured times.  Synchronises `stream`. */
int rsc_knn_batched_autotune(const float *X, const int64_t *offsets, int32_t S, int32_t d, int32_t k,
                             void *workspace, size_t workspace_bytes, void *stream, int32_t *chosen,
                             float *times_ms);

/* Human-readable description of a policy index ("" if out of range). */
const char *rsc_batch_policy_name(int32_t policy);

/* ---------------------------------------------------------------------- */
/* Connectivities (fuzzy simplicial set)                                   */
/* ---------------------------------------------------------------------- */

/* Workspace bytes for rsc_connectivities. */
size_t rsc_connectivities_workspace_bytes(int64_t n, int32_t k);

/*
 * Connectivities of a kNN result in the layout rsc_knn produces.
 *   idx, dist   device n x k (int32, float32); column 0 is the row itself
 *               and is ignored; columns 1..k-1 are distinct rows != i.
 *   rho, sigma  device float64 n, or NULL: per row, rho = smallest strictly
 *               positive neighbour distance (0 if none), sigma solves
 *               sum_{j=1..k-1} exp(-max(0, d_ij - rho)/sigma) = log2 k
 *               (bisection in float64); rows where no sigma > 0 reaches
 *               log2 k get sigma = 0 and weight 1 for d <= rho, else 0.
 *   indptr      device int64 n+1.
 *   indices     device int32 capacity `cap`; data device float32 `cap`.
 *               cap >= 2 n (k-1) is required (RSC_ERR_CAPACITY otherwise).
 *   nnz         HOST int64: the number of stored entries.
 * The CSR holds w_ij = a_ij + a_ji - a_ij a_ji (a missing direction is 0),
 * computed in float64 and rounded once to float32; columns ascend within a
 * row, no diagonal, no stored zeros; w_ij and w_ji are bitwise equal.
 * Synchronises `stream` (to read nnz and the input check).  Malformed lists
 * (index out of range, self or a repeated neighbour in columns 1..k-1) give
 * RSC_ERR_BAD_GRAPH after the call; outputs are then unspecified.
 */
int rsc_connectivities(const int32_t *idx, const float *dist, int64_t n, int32_t k, int64_t *indptr,
                       int32_t *indices, float *data, int64_t cap, int64_t *nnz, double *rho, double *sigma,
                       void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* Kernel timing (off by default)                                          */
/* ---------------------------------------------------------------------- */

/* Enable (1) or disable (0) timing of every kernel the library launches
 * with HIP events recorded on the launch stream.  Host-side state. */
int rsc_profile_enable(int enable);
/* Drop all recorded timings. */
int rsc_profile_reset(void);
/* Total milliseconds and launch count recorded for the kernel `name`
 * (host string, e.g. "screen_fp32").  Waits for the recorded events. */
int rsc_profile_get(const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* RSC_H */
