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

/* Distance of the neighbour search.  RSC_EUCLIDEAN: ||x - y||.
 * RSC_COSINE: 1 - x.y / (||x|| ||y||) (a row of zero norm is at distance 1
 * from every row); the screen runs on the unit-normalised rows and the
 * reported distances are float64 cosine distances of the original rows,
 * rounded once to float32. */
typedef enum { RSC_EUCLIDEAN = 0, RSC_COSINE = 1 } rsc_metric;

/*
 * Options of the screening stage.  A zero-initialised struct (or NULL)
 * selects the default: FP32 screen of width 32 (64 for k > 16) followed by
 * the exactness certificate and rescan, i.e. the exact result.
 *   precision  arithmetic of the distance screen on the matrix cores:
 *              RSC_FP32      exact result (certified, see rsc_knn);
 *              RSC_BF16      BF16 operands, FP32 accumulation;
 *              RSC_FP8_E4M3  OCP e4m3 operands with per-dimension absmax
 *                            scaling (s_t = max|y_t| / 448), FP32 accumulation.
 *              The reduced-precision forms keep the `screen` (default 64)
 *              smallest screened keys per query and re-rank them with float64
 *              distances; they are approximate (no certificate): measure them
 *              by recall@k.
 *   screen     candidates kept per query and reference range: 32 or 64 for
 *              RSC_FP32 (must exceed k when k < 64; 64 for larger k, where
 *              the references are split into about k / 32 ranges so that
 *              every range's list keeps spare room); 64 (default), 128, 256
 *              or 512 for the reduced-precision forms, which split the
 *              references into screen / 64 ranges of 64 candidates each;
 *              0 = default.
 *   metric     rsc_metric (0 = Euclidean).  The exactness guarantee of
 *              RSC_FP32 holds for both metrics.
 *   fp8_residual  0: the FP8 screen codes the rows themselves (the
 *              per-dimension absmax scaling above).  P in [2, 4096] (at most
 *              the reference count): the residual variant, a separate form --
 *              the references are split into P k-means partitions (4 Lloyd
 *              iterations from P evenly spaced rows, exact assignment) and
 *              each is coded as its residual y - c_p, scaled per dimension
 *              by the absmax of the residuals; a query is coded against each
 *              partition it meets as x - c_p, so the screen ranks by
 *              |x - c_p|^2 + |r~|^2 - 2 (x - c_p)~ . r~.  The partitioning is
 *              part of the call.  Only with RSC_FP8_E4M3 and the Euclidean
 *              metric (RSC_ERR_INVALID_ARG otherwise).
 */
typedef struct {
    int32_t precision;
    int32_t screen;
    int32_t metric;
    int32_t fp8_residual;
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
 *   n, d, k   1 <= k <= n <= 2^31-1; the exact (FP32-screened) path takes
 *             1 <= d <= 256 and k <= 255, the reduced-precision screens
 *             d <= 128 and k <= 63.
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
 *   1 <= k <= n_ref; d and k limits as for rsc_knn.  opts may be NULL.
 */
int rsc_knn_ex(const float *Q, int64_t n_query, const float *R, int64_t n_ref, int32_t d, int32_t k,
               const rsc_knn_opts *opts, int32_t *out_idx, float *out_dist, void *workspace, size_t workspace_bytes,
               void *stream);

/* Copy the counters of the last kNN call that used `workspace` into host
 * memory `out`.  Synchronises `stream`. */
int rsc_knn_read_stats(const void *workspace, size_t workspace_bytes, rsc_knn_stats *out, void *stream);

/* Rows of the last kNN call on `workspace` whose first certificate failed
 * (the escalated rows of rsc_knn_stats), in no particular order.  The sizes
 * and options must be those of that call (square = 1 for rsc_knn /
 * rsc_knn_opt, 0 for rsc_knn_ex).  rows: HOST int32 [cap]; the first
 * min(*count, cap) entries are written; *count (HOST) receives the number of
 * escalated rows.  Synchronises `stream`. */
int rsc_knn_read_escalated(const void *workspace, size_t workspace_bytes, int64_t n_query, int64_t n_ref, int32_t d,
                           int32_t k, const rsc_knn_opts *opts, int32_t square, int32_t *rows, int64_t cap,
                           int64_t *count, void *stream);

/* ---------------------------------------------------------------------- */
/* Batched exact kNN (many independent samples, one persistent launch)     */
/* ---------------------------------------------------------------------- */

/* Number of scheduling policies the batched autotuner measures. */
#define RSC_BATCH_POLICIES 6
/* Largest number of tile shapes one autotune call measures (the size of its
 * times_ms array). */
#define RSC_BATCH_TRIALS 32

/*
 * A batch is S samples stored back to back in one matrix X: sample s is rows
 * offsets[s] .. offsets[s+1]-1 (offsets is a HOST int64 array of S+1
 * entries, offsets[0] = 0, every sample at least k rows, total <= 2^31-2).
 * Each sample is its own exact kNN problem (the paper analyses large
 * collections chunk by chunk along the cell axis: Methods, "Memory
 * management and scaling"); results use global row ids, so the kNN graph is
 * block-diagonal; rsc_connectivities_batched builds the per-sample
 * connectivities of the whole output at once (and checks that no edge leaves
 * its sample).
 */
size_t rsc_knn_batched_workspace_bytes(const int64_t *offsets, int32_t S, int32_t d, int32_t k);

/* Exact kNN of every sample (same output layout and exactness as rsc_knn,
 * neighbours drawn from the row's own sample).  Uses the scheduling policy
 * the autotuner chose for this batch shape, else a default.  Synchronises
 * `stream` once (to upload the work list into the workspace). */
int rsc_knn_batched(const float *X, const int64_t *offsets, int32_t S, int32_t d, int32_t k, int32_t *out_idx,
                    float *out_dist, void *workspace, size_t workspace_bytes, void *stream);

/* Choose the tile shape and schedule of this batch by timing its screen
 * (HIP events) and remember the choice for batches of the same shape
 * (device, d, k and the histogram of log2 sample sizes); with
 * RSC_AUTOTUNE_CACHE=<file> in the environment the choice is also read from
 * / written to that file.  Trials, in order: every scheduling policy
 * (RSC_BATCH_POLICIES: item order and a default rule for cutting large
 * samples' references into 2 ranges); the best of them with the wider
 * screen tile (32 instead of 16 keys kept per query and contraction half,
 * when k <= 16); then, for each log2 sample-size class holding at least 5%
 * of the work (heaviest first), the tile's depth along the references: the
 * class's samples cut into 1, 2 or 4 reference ranges, on top of the best so
 * far.  chosen (host, may be NULL): the index of the chosen trial;
 * times_ms (host, may be NULL): RSC_BATCH_TRIALS entries, the measured
 * screen time of each trial (NaN past the last); rsc_batch_trial_name
 * describes each.  Synchronises `stream`. */
int rsc_knn_batched_autotune(const float *X, const int64_t *offsets, int32_t S, int32_t d, int32_t k,
                             void *workspace, size_t workspace_bytes, void *stream, int32_t *chosen,
                             float *times_ms);

/* Human-readable description of a policy index ("" if out of range). */
const char *rsc_batch_policy_name(int32_t policy);

/* Description of trial t of the last rsc_knn_batched_autotune call in this
 * process ("" if out of range); the chosen trial ends with its shape.  Valid
 * until the next autotune call. */
const char *rsc_batch_trial_name(int32_t trial);

/* ---------------------------------------------------------------------- */
/* Connectivities (fuzzy simplicial set)                                   */
/* ---------------------------------------------------------------------- */

/* Workspace bytes for rsc_connectivities. */
size_t rsc_connectivities_workspace_bytes(int64_t n, int32_t k);

/*
 * Connectivities of a kNN result in the layout rsc_knn produces.
 *   idx, dist   device n x k (int32, float32), 1 <= k <= 256; column 0 is
 *               the row itself and is ignored; columns 1..k-1 are distinct
 *               rows != i.
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

/*
 * rsc_connectivities for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation and output, bitwise, without a
 * workspace argument.  Its scratch is a fixed device array of
 * rsc_connectivities_noalloc_max_bytes() bytes (64 MiB) inside the library,
 * which every GPU the library runs on holds until the process ends; the
 * call allocates nothing.  A problem whose workspace
 * (rsc_connectivities_workspace_bytes(n, k)) exceeds it is rejected with
 * RSC_ERR_CAPACITY before anything is enqueued (at k = 15 about 190,000
 * rows fit).  Every call on one GPU shares that GPU's array: calls that
 * overlap in time on one GPU (two streams, two host threads) race and must
 * be serialised by the caller.  Arguments, output, validation and
 * synchronisation as for rsc_connectivities.
 */
size_t rsc_connectivities_noalloc_max_bytes(void);
int rsc_connectivities_noalloc(const int32_t *idx, const float *dist, int64_t n, int32_t k, int64_t *indptr,
                               int32_t *indices, float *data, int64_t cap, int64_t *nnz, double *rho, double *sigma,
                               void *stream);

/*
 * Connectivities of a batch of samples (the output of rsc_knn_batched):
 * each sample's fuzzy simplicial set on its own rows, the samples' graphs
 * side by side in one block-diagonal CSR with global row ids (the paper
 * analyses large collections sample by sample through offset tables:
 * Methods, "Perturbation distance computation" and "Memory management and
 * scaling").
 *   offsets  HOST int64 [S + 1]: sample s is rows offsets[s] ..
 *            offsets[s+1]-1; offsets[0] = 0, every sample at least k rows,
 *            offsets[S] = n <= 2^31 - 2 (RSC_ERR_INVALID_ARG otherwise).
 *            Copied during the call.
 *   idx, dist, indptr, indices, data, cap, nnz  as for rsc_connectivities
 *            over the n rows (cap >= 2 n (k-1)).
 * Every neighbour in columns 1..k-1 of a row must lie in the row's own
 * sample: an edge to another sample gives RSC_ERR_BAD_GRAPH after the call,
 * as do the malformed lists rsc_connectivities rejects.  Synchronises
 * `stream`.
 */
size_t rsc_connectivities_batched_workspace_bytes(const int64_t *offsets, int32_t S, int32_t k);
int rsc_connectivities_batched(const int32_t *idx, const float *dist, const int64_t *offsets, int32_t S, int32_t k,
                               int64_t *indptr, int32_t *indices, float *data, int64_t cap, int64_t *nnz,
                               void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* Routed form: coarse partitions, learned router, probed search           */
/* ---------------------------------------------------------------------- */
/*
 * The routed form answers a query from a few coarse partitions of the cells
 * instead of all of them (the paper's approximate-neighbour alternative,
 * Methods, "Dimensionality reduction and graph analysis", where cuVS serves
 * the neighbour search): a small network predicts which partitions hold a
 * cell's neighbours, the cell is compared exactly with the cells of its most
 * probable partitions, and cells the network is unsure of fall back to
 * exact brute force.
 */

/* Workspace bytes for rsc_partition_kmeans. */
size_t rsc_partition_kmeans_workspace_bytes(int64_t n, int32_t d, int32_t parts);

/*
 * Lloyd's k-means into `parts` partitions.
 *   X          device n x d float32 (1 <= d <= 128, parts <= n <= 2^31-2).
 *   init_rows  device int32 `parts` row ids: initial centroids are those rows.
 *   iters      iterations (>= 0).  Each assigns every row to its nearest
 *              centroid (float64 distance from direct differences, lower
 *              centroid index on ties) and moves every centroid to the mean
 *              of its rows (exact integer sum of the rows in fixed point,
 *              divided by the count in float64, rounded to float32).  A
 *              centroid left without rows takes the row farthest from its own
 *              centroid (largest distance, lower row index on ties), one row
 *              per empty centroid, in ascending centroid order.
 *   centroids  device parts x d float32 (output).
 *   assign     device int32 n (output): nearest centroid of each row for the
 *              final centroids (one more assignment pass after the last
 *              iteration).
 *   offsets    device int64 parts+1, perm device int32 n (outputs, may be
 *              NULL): inverted lists of `assign`: the rows of partition p are
 *              perm[offsets[p] .. offsets[p+1]) (order within a partition
 *              unspecified).
 *   relocated  HOST int64 (may be NULL): empty-centroid relocations made.
 * Synchronises `stream` once per iteration (to look for empty centroids).
 */
int rsc_partition_kmeans(const float *X, int64_t n, int32_t d, int32_t parts, const int32_t *init_rows,
                         int32_t iters, float *centroids, int32_t *assign, int64_t *offsets, int32_t *perm,
                         int64_t *relocated, void *workspace, size_t workspace_bytes, void *stream);

/* Label gather: labels[i*k + j] = assign[idx[i*k + j]] for an n x k kNN
 * result `idx` (device int32); labels device int32 n x k.  Entries of idx
 * outside [0, n_assign) give label -1. */
int rsc_partition_labels(const int32_t *idx, int64_t n, int32_t k, const int32_t *assign, int64_t n_assign,
                         int32_t *labels, void *stream);

/*
 * The router: a d -> hidden -> hidden -> parts perceptron (ReLU, softmax over
 * partitions) held by an opaque handle that owns its device memory (float32
 * master weights, Adam moments and bfloat16 copies).  Forward and backward
 * products run in bfloat16 on the matrix cores with float32 accumulation.
 * Weight layout (rsc_router_gradients, files): W1 [hidden x d], b1 [hidden],
 * W2 [hidden x hidden], b2, W3 [parts x hidden], b3 [parts], row-major,
 * concatenated (n_params floats).
 */
typedef struct rsc_router rsc_router;

/* Create a router with uniform(+-sqrt(6/(fan_in+fan_out))) weights drawn from
 * a counter-based SplitMix64 stream of `seed`, zero biases.  1 <= d <= 256;
 * hidden and parts multiples of 64, parts <= 4096.  Synchronises the device. */
int rsc_router_create(rsc_router **out, int32_t d, int32_t hidden, int32_t parts, uint64_t seed);
/* Free a router (NULL is ignored). */
void rsc_router_destroy(rsc_router *router);
/* Shape and progress of a router (host outputs, each may be NULL). */
int rsc_router_info(const rsc_router *router, int32_t *d, int32_t *hidden, int32_t *parts, int64_t *n_params,
                    int64_t *steps);

/* Workspace bytes for rsc_router_train with this batch and row count. */
size_t rsc_router_train_workspace_bytes(const rsc_router *router, int32_t batch, int64_t n);
/*
 * Train on n labelled rows for `epochs` passes in row order, one Adam step
 * (beta1 0.9, beta2 0.999, eps 1e-8, learning rate lr) per batch of `batch`
 * rows (a multiple of 64; the last batch may be partial).
 *   X        device n x d float32.
 *   labels   device n x m int32 partition ids: the target of row i puts
 *            weight 1/m on each listed partition (repeats add up; entries
 *            outside [0, parts) are skipped, their weight dropped); the loss
 *            is the soft-target cross-entropy averaged over the batch.
 *   loss_log HOST float32 `epochs` (may be NULL): mean batch loss per epoch
 *            (losses before each step); when given the call synchronises.
 */
int rsc_router_train(rsc_router *router, const float *X, int64_t n, const int32_t *labels, int32_t m,
                     int32_t epochs, int32_t batch, float lr, float *loss_log, void *workspace,
                     size_t workspace_bytes, void *stream);

/* Workspace bytes for rsc_router_gradients over n rows. */
size_t rsc_router_gradients_workspace_bytes(const rsc_router *router, int64_t n);
/* Gradient of the mean loss over n rows (n <= 65536) at the current weights,
 * without updating them: grad device float32 n_params (layout above), loss
 * device float32 1 (may be NULL). */
int rsc_router_gradients(const rsc_router *router, const float *X, int64_t n, const int32_t *labels, int32_t m,
                         float *grad, float *loss, void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for rsc_router_logits / rsc_router_probe. */
size_t rsc_router_infer_workspace_bytes(const rsc_router *router);
/* Logits of n rows: device n x parts float32. */
int rsc_router_logits(const rsc_router *router, const float *X, int64_t n, float *logits, void *workspace,
                      size_t workspace_bytes, void *stream);
/* The `probes` most probable partitions of each row, by descending logit
 * (lower index on ties): parts device int32 n x probes; mass device float32 n:
 * the softmax probability those partitions hold. */
int rsc_router_probe(const rsc_router *router, const float *X, int64_t n, int32_t probes, int32_t *parts,
                     float *mass, void *workspace, size_t workspace_bytes, void *stream);

/* Inverted lists of given labels (device int32 n, each in [0, parts)):
 * offsets device int64 parts+1, perm device int32 n as for
 * rsc_partition_kmeans.  Synchronises `stream` (labels outside [0, parts)
 * give RSC_ERR_INVALID_ARG). */
size_t rsc_partition_lists_workspace_bytes(int32_t parts);
int rsc_partition_lists(const int32_t *labels, int64_t n, int32_t parts, int64_t *offsets, int32_t *perm,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Save / load weights and optimizer state (host file; header of shape and
 * step count, then float32 arrays in the layout above).  Loading requires a
 * router of the same shape.  Synchronise the device. */
int rsc_router_save(const rsc_router *router, const char *path);
int rsc_router_load(rsc_router *router, const char *path);

/* How the rows of a routed or probed search were answered. */
typedef struct {
    int64_t routed_rows;      /* answered from their probed partitions */
    int64_t low_mass_rows;    /* exact search: marked (probed softmax mass below the threshold) */
    int64_t uncertified_rows; /* exact search: the screen of the probed partitions was not certified */
    int64_t escalated_rows;   /* exact-search rows screened again, wider */
    int64_t rescanned_rows;   /* exact-search rows recomputed exhaustively in float64 */
    double mean_probed_rows;  /* mean candidates per probed row (rows of its probed partitions) */
    double mean_screened_rows; /* mean rows streamed past a probed row (the partitions its tile probes) */
} rsc_routed_stats;

/* Workspace bytes for rsc_knn_probed / rsc_knn_routed. */
size_t rsc_knn_probed_workspace_bytes(int64_t n, int32_t d, int32_t k, int32_t parts, int32_t probes);

/*
 * kNN of every row of X restricted to the partitions it probes.
 *   X            device n x d float32; k, d as for rsc_knn.
 *   offsets,perm device inverted lists of the partitions (as produced by
 *                rsc_partition_kmeans: every row in exactly one partition).
 *   probe_parts  device int32 n x probes partition ids (repeats and -1
 *                entries ignored), 1 <= probes <= 64.
 *   exact_rows   device uint8 n or NULL: rows with a non-zero entry are
 *                answered by exact search over all rows.
 *   out_idx, out_dist  as for rsc_knn.  A probed row's answer is the exact
 *                k nearest (float64 distances, lower index on ties) among
 *                the rows of its probed partitions, self in column 0; fewer
 *                candidates than k-1 leave index -1 / distance +inf.
 *                Rows whose screen cannot be certified within their
 *                partitions are answered by exact search instead.
 *   out_route    device uint8 n or NULL: 0 probed, 1 exact (marked), 2 exact
 *                (not certified).
 *   stats        HOST, may be NULL.
 * Synchronises `stream` (to size the exact search).
 */
int rsc_knn_probed(const float *X, int64_t n, int32_t d, int32_t k, const int64_t *offsets, const int32_t *perm,
                   int32_t parts, const int32_t *probe_parts, int32_t probes, const uint8_t *exact_rows,
                   int32_t *out_idx, float *out_dist, uint8_t *out_route, rsc_routed_stats *stats,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for rsc_knn_routed. */
size_t rsc_knn_routed_workspace_bytes(const rsc_router *router, int64_t n, int32_t d, int32_t k, int32_t parts,
                                      int32_t probes);

/*
 * The routed form: the router's `probes` most probable partitions per row
 * (rsc_router_probe), rows whose probed softmax mass is below
 * `mass_threshold` marked for exact search, then rsc_knn_probed.  The router
 * must have been created with d and parts equal to these.
 */
int rsc_knn_routed(const rsc_router *router, const float *X, int64_t n, int32_t d, int32_t k,
                   const int64_t *offsets, const int32_t *perm, int32_t parts, int32_t probes, float mass_threshold,
                   int32_t *out_idx, float *out_dist, uint8_t *out_route, rsc_routed_stats *stats, void *workspace,
                   size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* Energy distance between groups of cells                                 */
/* ---------------------------------------------------------------------- */
/*
 * Methods, "Perturbation distance computation": for groups X, Y of cells,
 *   E(X, Y) = 2 mean ||X_i - Y_j|| - mean ||X_i - X_i'|| - mean ||Y_j - Y_j'||
 * with the cross mean over all n_X n_Y pairs and each within mean over the
 * n (n - 1) / 2 pairs of the upper triangle.  A group with fewer than two
 * cells is skipped: its within mean counts as 0.  A cross mean with an empty
 * group has no pairs and is NaN.
 *
 * Groups use the paper's category-index layout:
 *   offsets   HOST int64 [G + 1], offsets[0] = 0, non-decreasing; group g
 *             holds cells[offsets[g] .. offsets[g+1]).  Copied during the
 *             call (the host array may be reused when it returns).
 *   cells     DEVICE int32 [offsets[G]], row ids of X in [0, n); an id
 *             outside that range is read as no cell (the kernels never
 *             touch memory outside X), so such input gives wrong sums.
 *   X         DEVICE float32 [n][d], row-major, finite values; any d >= 1.
 * Distances are float64: dot products on the float64 matrix cores, norms
 * and square roots in float64; each distance is within
 * min(sqrt(e), e / dist) + 4 u dist of the exact one, with
 * e = 2 (d + 4) u (||x||^2 + ||y||^2) and u = 2^-53.
 * Each pair's sum is accumulated in 64-bit fixed point (scale from an upper
 * bound of the sum), so results do not depend on scheduling.
 * G <= 2^20 groups, offsets[G] <= 2^31 cells.  Work is queued on `stream`.
 * Errors: RSC_ERR_INVALID_ARG (null pointer, bad offsets, group id out of
 * range), RSC_ERR_WORKSPACE (workspace smaller than the *_workspace_bytes
 * figure), RSC_ERR_HIP.
 */

/* Workspace bytes for rsc_edistance_groups (0 for invalid sizes, or when
 * no device is available to size the sort). */
size_t rsc_edistance_groups_workspace_bytes(int64_t n, int64_t n_groups);

/*
 * The category-index layout of integer labels (DEVICE int32 [n], values in
 * [0, G)): offsets DEVICE int64 [G + 1] and cells DEVICE int32 [n], each
 * group's rows in ascending order (a stable radix sort of (label, row)).
 * Synchronises `stream` to report RSC_ERR_INVALID_ARG for a label outside
 * [0, G); copy offsets to the host for the calls below.
 */
int rsc_edistance_groups(const int32_t *labels, int64_t n, int64_t n_groups, int64_t *offsets, int32_t *cells,
                         void *workspace, size_t workspace_bytes, void *stream);

/* Workspace bytes for rsc_edistance_sums with n_pairs pairs over G groups
 * holding n_cells = offsets[G] cells of dimension d (0 for invalid sizes).
 * The workspace holds the grouped rows in group order (n_cells x d float32)
 * and their norms, so that a tile's rows are contiguous. */
size_t rsc_edistance_sums_workspace_bytes(int64_t n_groups, int64_t n_pairs, int64_t n_cells, int32_t d);

/*
 * Sums of distances for a list of group pairs.
 *   pairs   HOST int32 [n_pairs][2] (a, b); a == b gives the within sum
 *           over the upper triangle, a != b the sum over all n_a n_b pairs.
 *   sums    DEVICE float64 [n_pairs].
 */
int rsc_edistance_sums(const float *X, int64_t n, int32_t d, const int64_t *offsets, int64_t n_groups,
                       const int32_t *cells, const int32_t *pairs, int64_t n_pairs, double *sums, void *workspace,
                       size_t workspace_bytes, void *stream);

/* Workspace bytes for rsc_edistance_pairwise (G (G + 1) / 2 pairs). */
size_t rsc_edistance_pairwise_workspace_bytes(int64_t n_groups, int64_t n_cells, int32_t d);

/*
 * All energy distances: E DEVICE float64 [G][G] (symmetric, zero diagonal),
 * D DEVICE float64 [G][G] mean distances (may be NULL).  E[a][b] is
 * 2 D[a][b] - (D[a][a] + D[b][b]).
 */
int rsc_edistance_pairwise(const float *X, int64_t n, int32_t d, const int64_t *offsets, int64_t n_groups,
                           const int32_t *cells, double *E, double *D, void *workspace, size_t workspace_bytes,
                           void *stream);

/* Workspace bytes for rsc_edistance_onesided (2 G - 1 pairs). */
size_t rsc_edistance_onesided_workspace_bytes(int64_t n_groups, int64_t n_cells, int32_t d);

/*
 * Methods, "Perturbation distance computation" (one-sided distances): E from
 * the reference group `ref` to every group, computing only the cross pairs
 * (ref, g) and the within pairs.  E DEVICE float64 [G], E[ref] = 0.
 */
int rsc_edistance_onesided(const float *X, int64_t n, int32_t d, const int64_t *offsets, int64_t n_groups,
                           const int32_t *cells, int64_t ref, double *E, void *workspace, size_t workspace_bytes,
                           void *stream);

/* ---------------------------------------------------------------------- */
/* Sparse PCA: the embedding the graph is built on                         */
/* ---------------------------------------------------------------------- */
/*
 * Methods, "Principal component analysis": for a cells x genes CSR matrix X
 * (n x p), mu = X^T 1 / n, S = X^T X (upper triangle accumulated, then
 * copied), C = (S - n mu mu^T) / (n - 1) without centring X, the top-k
 * eigenpairs of C, and the scores Z = X V - 1 (mu^T V).
 *   indptr   DEVICE int64 [n + 1]; indices DEVICE int32 [nnz] (genes in
 *            [0, p), distinct within a row); data DEVICE float32 [nnz].
 *   mean     DEVICE float64 [p]; cov DEVICE float64 [p][p] (symmetric;
 *            may be NULL in rsc_pca).
 *   evals    DEVICE float64 [k], descending.
 *   loadings DEVICE float64 [p][k], column t = the t-th eigenvector, signed
 *            so that its largest-magnitude entry (lowest gene on ties) is
 *            positive.
 *   scores   DEVICE float32 [n][k] (sums in float64, rounded once).
 * 2 <= n, 1 <= p <= 16384, 1 <= k <= min(p, 64).  The Gram matrix is summed
 * in float64 on the matrix cores (float32 products are exact in float64) over
 * densified chunks of cells; the eigendecomposition is rocSOLVER's float64
 * symmetric solver, run on the caller's workspace.  The first call on a
 * device creates a rocBLAS handle that the library keeps until the process
 * ends.  Both calls synchronise `stream` (to report a gene index outside
 * [0, p) as RSC_ERR_INVALID_ARG, and the solver's status).
 */

/* Workspace bytes for rsc_pca (k >= 1; needs a device to size the solver)
 * or rsc_pca_covariance (k = 0). */
size_t rsc_pca_workspace_bytes(int64_t n, int32_t p, int32_t k);

/* mean and covariance only. */
int rsc_pca_covariance(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int32_t p,
                       double *mean, double *cov, void *workspace, size_t workspace_bytes, void *stream);

/* The whole PCA. */
int rsc_pca(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int32_t p, int32_t k,
            double *mean, double *cov, double *evals, double *loadings, float *scores, void *workspace,
            size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* UMAP layout of the graph                                                */
/* ---------------------------------------------------------------------- */
/*
 * The layout step of UMAP (the embedding method the paper runs on this
 * graph, its reference [15]): stochastic gradient descent over the graph's
 * edges on the cross-entropy between the weights and q(d2) = 1/(1 + a d2^b).
 * Deterministic reading: edge e (weight w_e) is due every w_max / w_e
 * epochs (never when w_e < w_max / n_epochs); in epoch t every move is
 * computed from the embedding at the start of t and vertex i sums the moves
 * of its own row's due edges in CSR order -- an attraction towards the
 * neighbour, then `neg` repulsions from vertices drawn by a counter-based
 * SplitMix64 (state seed + (t 2^40 + e 64 + p + 1) 0x9E3779B97F4A7C15,
 * k = (mix >> 11) mod n; the edge stride 64 is the largest neg, so no two
 * draws of an epoch share a counter; a draw of the vertex itself is
 * skipped) -- each coordinate clipped to [-4, 4] and scaled by
 * alpha0 (1 - t / n_epochs); attraction -2 a b d2^(b-1) / (a d2^b + 1),
 * repulsion 2 gamma b / ((0.001 + d2)(a d2^b + 1)), with d2^(b-1) and d2^b
 * each the correctly rounded power.  The embedding is kept in float64 and every operation is
 * rounded as written, so the layout is bitwise reproducible and equals that
 * of any sequential implementation of these steps.
 *   indptr, indices, weights  DEVICE CSR of the symmetric graph (the
 *            rsc_connectivities layout): int64 [n + 1], int32 [nnz], float32
 *            [nnz] with weights >= 0 (indices and weights may be NULL when
 *            nnz = 0).
 *   Y        DEVICE float32 [n][dim], the initial embedding in (finite,
 *            else RSC_ERR_INVALID_ARG), the layout out; 1 <= dim <= 8.
 *   a, b     the similarity curve (min_dist 0.5, spread 1: a = 0.58303,
 *            b = 1.33417, the least-squares fit of UMAP's target curve);
 *            gamma the repulsion strength (1), alpha0 the initial rate (1),
 *            neg the negative samples per due edge (5); a > 0 finite,
 *            0 < b <= 64, 0 <= neg <= 64, n_epochs >= 1, else
 *            RSC_ERR_INVALID_ARG.
 * Synchronises `stream` once, to report a malformed graph as
 * RSC_ERR_BAD_GRAPH before any epoch runs.  Supports n < 2^31 and
 * nnz < 2^32 - 1; the workspace (rsc_umap_workspace_bytes, 0 for an
 * unsupported shape) holds about 28 nnz + 16 n dim bytes (the sampling
 * schedule, the due-edge list and two float64 embeddings).
 */
size_t rsc_umap_workspace_bytes(int64_t n, int64_t nnz, int32_t dim, int32_t neg);
int rsc_umap_layout(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
                    int32_t dim, float *Y, int32_t n_epochs, double a, double b, double gamma, double alpha0,
                    int32_t neg, uint64_t seed, void *workspace, size_t workspace_bytes, void *stream);

/* ---------------------------------------------------------------------- */
/* Leiden communities of the graph                                         */
/* ---------------------------------------------------------------------- */
/*
 * Community detection on the neighbourhood graph (the paper clusters cells
 * by Leiden: Technical architecture; Methods, "Dimensionality reduction and
 * graph analysis"; it validates the clustering by the agreement of
 * partitions, Methods, "Numerical validation").  One deterministic reading of
 * Traag, Waltman and van Eck's algorithm, so that the labels are a function
 * of the graph alone:
 *   quality   modularity with resolution gamma; the gain of moving v into c
 *             is h = K(v, c) - ((gamma k_v) T(c)) / 2m in float64, each
 *             operation rounded as written (K: weight from v to c's other
 *             vertices, T: total degree of c without v, 2m: sum of degrees);
 *   weights   fixed point W = rint(w 2^S), S = 62 - ceil(log2 nnz) - e with
 *             w_max <= 2^e, so every sum of weights is an exact int64;
 *   moving    synchronous sweeps from the labels at the sweep start: a
 *             vertex takes the neighbouring community of largest gain if it
 *             is strictly above staying (ties: lowest label); odd sweeps
 *             move only to higher labels, even sweeps only to lower ones;
 *             two quiet sweeps in a row (or 64 sweeps) end the phase;
 *   refining  rounds inside each community C from singletons: a singleton
 *             v with K(v, C - v) >= gamma k_v (Tot(C) - k_v) / 2m may join
 *             the refined community R of a neighbour in C with a smaller
 *             label if E(R, C - R) >= gamma Tot(R) (Tot(C) - Tot(R)) / 2m and
 *             the gain is >= 0 (largest gain, ties: lowest label); a join
 *             into a singleton that moves in the same round is cancelled; a
 *             round without joins (or 64 rounds) ends the phase;
 *   aggregating  refined communities become the next level's vertices
 *             (numbered by their smallest vertex) with summed weights, each
 *             starting in the community that holds it, labelled by its
 *             smallest new id.
 * Levels end when moving moves nothing (or after 32 levels).
 *   indptr, indices, weights  DEVICE CSR (int64 [n + 1], int32 [nnz],
 *            float32 [nnz]) of a symmetric graph with weights >= 0 and
 *            finite (the rsc_connectivities output; a diagonal entry counts
 *            once in its vertex's degree); indices and weights may be NULL
 *            when nnz = 0.  Malformed input (row pointers not from 0 to nnz
 *            or decreasing, a column outside [0, n), a negative or
 *            non-finite weight) gives RSC_ERR_INVALID_ARG.
 *   gamma    resolution, finite and > 0 (1 = plain modularity).
 *   labels   DEVICE int32 [n]: community of each vertex, numbered from 0 in
 *            order of first appearance (vertex 0 is in community 0).
 *   stats    HOST rsc_leiden_stats or NULL: the modularity of the labels on
 *            the input graph (from the exact integer sums, communities in
 *            label order), the community count and the work done.
 * Synchronises `stream` (once per sweep, refinement round and level).
 * Workspace: rsc_leiden_workspace_bytes (about 100 nnz + 100 n bytes; 0 for
 * unsupported sizes: n outside [1, 2^31 - 2], nnz outside [0, 2^40]).
 */
typedef struct {
    double quality;        /* modularity of the labels on the input graph */
    int64_t n_communities; /* number of communities */
    int32_t levels;        /* local-moving phases run */
    int32_t sweeps;        /* local-moving sweeps, all levels */
    int32_t rounds;        /* refinement rounds, all levels */
    int32_t reserved;
    int64_t move_bytes;    /* algorithmic bytes of all sweeps: per sweep of a level with
                              N vertices and M entries, 16 M (column, fixed-point weight,
                              the neighbour's label) + 24 N (row pointer, degree, label
                              in and out) */
} rsc_leiden_stats;

size_t rsc_leiden_workspace_bytes(int64_t n, int64_t nnz);
int rsc_leiden(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
               double gamma, int32_t *labels, rsc_leiden_stats *stats, void *workspace, size_t workspace_bytes,
               void *stream);

/* ---------------------------------------------------------------------- */
/* Kernel timing (off by default)                                          */
/* ---------------------------------------------------------------------- */

/* Enable (1) or disable (0) timing of every kernel the library launches
 * with HIP events recorded on the launch stream.  Host-side state. */
int rsc_profile_enable(int enable);
/* Drop all recorded timings. */
int rsc_profile_reset(void);
/* Total milliseconds and launch count recorded for the kernel `name`
 * (host string, e.g. "screen_fp32").  The k-means assignments that run
 * inside a call (rsc_partition_kmeans, the routed index, the FP8 residual
 * form's partitioning) are filed as "kmeans_assign" (brute force, for
 * d <= 64 and at most 2048 parts) or else under "kmeans/" + the kNN stage's name
 * ("kmeans/screen_fp32", "kmeans/rerank").  Waits for the recorded
 * events. */
int rsc_profile_get(const char *name, double *total_ms, int64_t *launches);

#ifdef __cplusplus
}
#endif
#endif /* RSC_H */
