// Connectivities of a kNN result: UMAP's fuzzy simplicial set as CSR.
//
// The paper stores the neighbourhood graph the way scanpy does (Methods,
// "Dimensionality reduction and graph analysis"); scanpy's connectivities
// are UMAP's fuzzy simplicial set (UMAP is the embedding method named in
// "Technical architecture"):
//
//   rho_i    smallest strictly positive neighbour distance of row i;
//   sigma_i  solves sum_{j=1..k-1} exp(-max(0, d_ij - rho_i)/sigma_i) = log2 k
//            (float64 bisection: the target sits in the flat part of the
//            sum, so float32 cannot meet a 1e-6 residual);
//   a_ij     exp(-max(0, d_ij - rho_i)/sigma_i);
//   w_ij     a_ij + a_ji - a_ij a_ji over the union of both directions.
//
// Every stage is a bandwidth-bound pass over the n (k-1) directed edges:
//   smooth      one thread per row, distances in registers;
//   count       one thread per row: find the reverse edge in the neighbour's
//               list (k-1 int32, one cache line), compute the union weight
//               once, count kept entries; one-way edges add one entry to the
//               neighbour's row (atomic counter);
//   scan        int64 exclusive scan of the row lengths -> indptr;
//   fill        each row writes its own entries in list order and appends
//               the one-way reverse entries to the neighbour's row;
//   sort        one wave per row ranks the (unique) columns and scatters
//               them into ascending order, which also makes the output
//               independent of the atomic append order.
// Weights of a pair are computed from the same two float64 operands with
// commutative operations, so w_ij and w_ji are bitwise equal.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>

#include "rsc_internal.hpp"

namespace rsc {
namespace {

constexpr int kWave = 64;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;

struct GraphResult {
    int64_t nnz;
    int32_t error;  // bit 0: index out of range or self; bit 1: repeated neighbour
    int32_t degenerate;
};

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_fill_f64(double *p, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_init_result(GraphResult *r) {
    if (threadIdx.x == 0) {
        r->nnz = 0;
        r->error = 0;
        r->degenerate = 0;
    }
}

// Sum over the row's neighbour slots of exp(-max(0, d - rho)/sigma), in slot order.
template <int KM>
__device__ __forceinline__ double membership_sum(const double (&dd)[KM], int m, double rho, double sigma) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        if (j < m) {
            double g = dd[j] - rho;
            if (g < 0.0) g = 0.0;
            s = __dadd_rn(s, exp(-g / sigma));
        }
    }
    return s;
}

template <int KM>
__global__ __launch_bounds__(256) void k_smooth(const float *__restrict__ dist, int64_t n, int k,
                                                double *__restrict__ a, double *__restrict__ rho_out,
                                                double *__restrict__ sigma_out, GraphResult *__restrict__ res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = k - 1;
    double dd[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) dd[j] = j < m ? (double)dist[i * k + 1 + j] : 0.0;

    double rho = 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j)
        if (j < m && dd[j] > 0.0 && (rho == 0.0 || dd[j] < rho)) rho = dd[j];
    int at_rho = 0;
#pragma unroll
    for (int j = 0; j < KM; ++j)
        if (j < m && dd[j] <= rho) ++at_rho;
    const double target = log2((double)k);
    double sigma;
    double *ai = a + i * m;
    if ((double)at_rho >= target) {
        // No sigma > 0 reaches the target: weight 1 on the nearest ties, 0 elsewhere.
        sigma = 0.0;
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j < m) ai[j] = dd[j] <= rho ? 1.0 : 0.0;
        atomicAdd(&res->degenerate, 1);
    } else {
        sigma = 1.0;
        double lo = 0.0, hi = INFINITY;
        for (int it = 0; it < 200; ++it) {
            const double f = membership_sum<KM>(dd, m, rho, sigma);
            if (fabs(f - target) <= 1e-12 * target) break;
            if (f > target)
                hi = sigma;
            else
                lo = sigma;
            if (isinf(hi))
                sigma = sigma * 2.0;
            else
                sigma = (lo + hi) / 2.0;
            if (!isinf(hi) && hi - lo <= ldexp(hi, -52)) break;
        }
#pragma unroll
        for (int j = 0; j < KM; ++j) {
            if (j < m) {
                double g = dd[j] - rho;
                if (g < 0.0) g = 0.0;
                ai[j] = exp(-g / sigma);
            }
        }
    }
    if (rho_out) rho_out[i] = rho;
    if (sigma_out) sigma_out[i] = sigma;
}

// The same computation for rows with more than 64 neighbour slots: the
// distances are read from memory (in slot order, as above) instead of being
// held in registers.
__device__ __forceinline__ double membership_sum_mem(const float *dr, int m, double rho, double sigma) {
    double s = 0.0;
    for (int j = 0; j < m; ++j) {
        double g = (double)dr[j] - rho;
        if (g < 0.0) g = 0.0;
        s = __dadd_rn(s, exp(-g / sigma));
    }
    return s;
}

__global__ __launch_bounds__(256) void k_smooth_wide(const float *__restrict__ dist, int64_t n, int k,
                                                     double *__restrict__ a, double *__restrict__ rho_out,
                                                     double *__restrict__ sigma_out, GraphResult *__restrict__ res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = k - 1;
    const float *dr = dist + i * k + 1;
    double rho = 0.0;
    for (int j = 0; j < m; ++j) {
        const double v = (double)dr[j];
        if (v > 0.0 && (rho == 0.0 || v < rho)) rho = v;
    }
    int at_rho = 0;
    for (int j = 0; j < m; ++j)
        if ((double)dr[j] <= rho) ++at_rho;
    const double target = log2((double)k);
    double sigma;
    double *ai = a + i * m;
    if ((double)at_rho >= target) {
        sigma = 0.0;
        for (int j = 0; j < m; ++j) ai[j] = (double)dr[j] <= rho ? 1.0 : 0.0;
        atomicAdd(&res->degenerate, 1);
    } else {
        sigma = 1.0;
        double lo = 0.0, hi = INFINITY;
        for (int it = 0; it < 200; ++it) {
            const double f = membership_sum_mem(dr, m, rho, sigma);
            if (fabs(f - target) <= 1e-12 * target) break;
            if (f > target)
                hi = sigma;
            else
                lo = sigma;
            if (isinf(hi))
                sigma = sigma * 2.0;
            else
                sigma = (lo + hi) / 2.0;
            if (!isinf(hi) && hi - lo <= ldexp(hi, -52)) break;
        }
        for (int j = 0; j < m; ++j) {
            double g = (double)dr[j] - rho;
            if (g < 0.0) g = 0.0;
            ai[j] = exp(-g / sigma);
        }
    }
    if (rho_out) rho_out[i] = rho;
    if (sigma_out) sigma_out[i] = sigma;
}

// Union weight of each directed edge and the row lengths.
__global__ __launch_bounds__(256) void k_union_count(const int32_t *__restrict__ idx, const double *__restrict__ a,
                                                     int64_t n, int k, float *__restrict__ wf,
                                                     uint8_t *__restrict__ mutual, int32_t *__restrict__ own,
                                                     int32_t *__restrict__ rev_cnt, GraphResult *__restrict__ res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = k - 1;
    int kept = 0;
    for (int s = 0; s < m; ++s) {
        const int64_t e = i * m + s;
        const int32_t j = idx[i * k + 1 + s];
        if (j < 0 || j >= n || j == i) {
            atomicOr(&res->error, 1);
            wf[e] = 0.f;
            mutual[e] = 0;
            continue;
        }
        const int32_t *lj = idx + (int64_t)j * k + 1;
        int sp = -1;
        for (int t = 0; t < m; ++t) {
            if (lj[t] == (int32_t)i) {
                sp = t;
                break;
            }
        }
        const double x = a[e];
        double w = x;
        if (sp >= 0) {
            const double y = a[(int64_t)j * m + sp];
            w = __dsub_rn(__dadd_rn(x, y), __dmul_rn(x, y));
        }
        const float f = (float)w;
        wf[e] = f;
        mutual[e] = sp >= 0 ? 1 : 0;
        if (f != 0.f) {
            ++kept;
            if (sp < 0) atomicAdd(&rev_cnt[j], 1);
        }
    }
    own[i] = kept;
}

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// Block-local exclusive scan of row lengths (own + reverse) into indptr.
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int32_t *__restrict__ own,
                                                              const int32_t *__restrict__ rev, int64_t n,
                                                              int64_t *__restrict__ indptr,
                                                              int64_t *__restrict__ block_tot) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    int64_t v[kScanItems];
    int64_t tsum = 0;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = base + u;
        v[u] = i < n ? (int64_t)own[i] + rev[i] : 0;
        tsum += v[u];
    }
    const int64_t incl = wave_incl_scan(tsum, lane);
    if (lane == kWave - 1) wsum[wave] = incl;
    __syncthreads();
    if (wave == 0) {
        int64_t s = lane < kScanThreads / kWave ? wsum[lane] : 0;
        s = wave_incl_scan(s, lane);
        if (lane < kScanThreads / kWave) wsum[lane] = s;
    }
    __syncthreads();
    int64_t run = incl - tsum + (wave > 0 ? wsum[wave - 1] : 0);
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = base + u;
        if (i < n) indptr[i] = run;
        run += v[u];
    }
    if (tid == kScanThreads - 1) block_tot[blockIdx.x] = run;
}

// Exclusive scan of the block totals (one workgroup, chunked); writes nnz.
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int64_t *__restrict__ block_tot, int64_t nb,
                                                               GraphResult *__restrict__ res) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    __shared__ int64_t carry;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
        const int64_t i = c0 + tid;
        const int64_t x = i < nb ? block_tot[i] : 0;
        const int64_t incl = wave_incl_scan(x, lane);
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        if (wave == 0) {
            int64_t s = lane < kScanThreads / kWave ? wsum[lane] : 0;
            s = wave_incl_scan(s, lane);
            if (lane < kScanThreads / kWave) wsum[lane] = s;
        }
        __syncthreads();
        const int64_t excl = incl - x + (wave > 0 ? wsum[wave - 1] : 0) + carry;
        if (i < nb) block_tot[i] = excl;
        __syncthreads();
        if (tid == kScanThreads - 1) carry = excl + x;
        __syncthreads();
    }
    if (tid == 0) res->nnz = carry;
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t *__restrict__ indptr, int64_t n,
                                                  const int64_t *__restrict__ block_tot,
                                                  const GraphResult *__restrict__ res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) indptr[i] += block_tot[i / kScanTile];
    if (i == n) indptr[n] = res->nnz;
}

__global__ __launch_bounds__(256) void k_union_fill(const int32_t *__restrict__ idx, int64_t n, int k,
                                                    const float *__restrict__ wf, const uint8_t *__restrict__ mutual,
                                                    const int32_t *__restrict__ own, const int64_t *__restrict__ indptr,
                                                    int32_t *__restrict__ cursor, int32_t *__restrict__ tmp_col,
                                                    float *__restrict__ tmp_val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int m = k - 1;
    int64_t p = indptr[i];
    for (int s = 0; s < m; ++s) {
        const int64_t e = i * m + s;
        const float f = wf[e];
        if (f == 0.f) continue;  // dropped zero, or a rejected edge
        const int32_t j = idx[i * k + 1 + s];
        tmp_col[p] = j;
        tmp_val[p] = f;
        ++p;
        if (!mutual[e]) {
            const int c = atomicAdd(&cursor[j], 1);
            const int64_t q = indptr[j] + own[j] + c;
            tmp_col[q] = (int32_t)i;
            tmp_val[q] = f;
        }
    }
}

// One wave per row: rank every entry by column and scatter into place.
__global__ __launch_bounds__(256) void k_row_sort(const int64_t *__restrict__ indptr, int64_t n,
                                                  const int32_t *__restrict__ tmp_col,
                                                  const float *__restrict__ tmp_val, int32_t *__restrict__ indices,
                                                  float *__restrict__ data, GraphResult *__restrict__ res) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x / kWave);
    if (row >= n) return;
    const int64_t beg = indptr[row];
    const int64_t len = indptr[row + 1] - beg;
    for (int64_t e0 = 0; e0 < len; e0 += kWave) {
        const int64_t e = e0 + lane;
        const int32_t col = e < len ? tmp_col[beg + e] : INT_MAX;
        const float val = e < len ? tmp_val[beg + e] : 0.f;
        int64_t rank = 0;
        bool dup = false;
        for (int64_t c0 = 0; c0 < len; c0 += kWave) {
            const int32_t oc = c0 + lane < len ? tmp_col[beg + c0 + lane] : INT_MAX;
            const int lim = (int)((len - c0) < kWave ? (len - c0) : kWave);
            for (int t = 0; t < lim; ++t) {
                const int32_t x = __shfl(oc, t, kWave);
                rank += x < col;
                dup |= (x == col) && (c0 + t != e);
            }
        }
        if (e < len) {
            indices[beg + rank] = col;
            data[beg + rank] = val;
            if (dup) atomicOr(&res->error, 2);
        }
    }
}

struct GraphWs {
    GraphResult *res;
    double *a;
    float *wf;
    uint8_t *mutual;
    int32_t *own, *rev_cnt, *cursor;
    int64_t *block_tot;
    int32_t *tmp_col;
    float *tmp_val;
};

size_t carve_graph(int64_t n, int k, void *base, GraphWs *w) {
    Carver cv(base);
    const size_t ne = (size_t)n * (size_t)(k - 1);
    const size_t nb = (size_t)((n + kScanTile - 1) / kScanTile) + 1;
    GraphWs g;
    g.res = cv.take<GraphResult>(1);
    g.a = cv.take<double>(ne ? ne : 1);
    g.wf = cv.take<float>(ne ? ne : 1);
    g.mutual = cv.take<uint8_t>(ne ? ne : 1);
    g.own = cv.take<int32_t>((size_t)n + 1);
    g.rev_cnt = cv.take<int32_t>((size_t)n + 1);
    g.cursor = cv.take<int32_t>((size_t)n + 1);
    g.block_tot = cv.take<int64_t>(nb);
    g.tmp_col = cv.take<int32_t>(2 * ne + 1);
    g.tmp_val = cv.take<float>(2 * ne + 1);
    if (w) *w = g;
    return cv.used;
}

unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

}  // namespace

size_t graph_workspace_bytes(int64_t n, int k) { return carve_graph(n, k, nullptr, nullptr); }

int graph_run(const int32_t *idx, const float *dist, int64_t n, int k, int64_t *indptr, int32_t *indices,
              float *data, int64_t cap, int64_t *nnz, double *rho, double *sigma, void *ws, hipStream_t stream) {
    (void)cap;
    GraphWs w;
    carve_graph(n, k, ws, &w);
    int st;
    const int m = k - 1;
    {
        ScopedTimer t("graph_init", stream);
        hipLaunchKernelGGL(k_init_result, dim3(1), dim3(64), 0, stream, w.res);
        const unsigned g = std::min<unsigned>(grid_for(n + 1, 256), 4096u);
        hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(256), 0, stream, w.rev_cnt, n + 1, 0);
        hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(256), 0, stream, w.cursor, n + 1, 0);
        if ((st = launch_status("graph_init")) != RSC_OK) return st;
    }
    if (m > 0) {
        ScopedTimer t("smooth_knn", stream);
        const unsigned g = grid_for(n, 256);
        if (m <= 16)
            hipLaunchKernelGGL((k_smooth<16>), dim3(g), dim3(256), 0, stream, dist, n, k, w.a, rho, sigma, w.res);
        else if (m <= 32)
            hipLaunchKernelGGL((k_smooth<32>), dim3(g), dim3(256), 0, stream, dist, n, k, w.a, rho, sigma, w.res);
        else if (m <= 64)
            hipLaunchKernelGGL((k_smooth<64>), dim3(g), dim3(256), 0, stream, dist, n, k, w.a, rho, sigma, w.res);
        else
            hipLaunchKernelGGL(k_smooth_wide, dim3(g), dim3(256), 0, stream, dist, n, k, w.a, rho, sigma, w.res);
        if ((st = launch_status("smooth_knn")) != RSC_OK) return st;
    } else {
        // k == 1: no neighbours; rho = sigma = 0 (no positive root exists)
        const unsigned g = std::min<unsigned>(grid_for(n, 256), 4096u);
        if (rho) hipLaunchKernelGGL(k_fill_f64, dim3(g), dim3(256), 0, stream, rho, n, 0.0);
        if (sigma) hipLaunchKernelGGL(k_fill_f64, dim3(g), dim3(256), 0, stream, sigma, n, 0.0);
        if ((st = launch_status("rho_sigma_fill")) != RSC_OK) return st;
    }
    {
        ScopedTimer t("union_count", stream);
        if (m > 0)
            hipLaunchKernelGGL(k_union_count, dim3(grid_for(n, 256)), dim3(256), 0, stream, idx, w.a, n, k, w.wf,
                               w.mutual, w.own, w.rev_cnt, w.res);
        else
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, stream, w.own, n, 0);
        if ((st = launch_status("union_count")) != RSC_OK) return st;
    }
    {
        ScopedTimer t("csr_scan", stream);
        const int64_t nb = (n + kScanTile - 1) / kScanTile;
        hipLaunchKernelGGL(k_scan_local, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(kScanThreads), 0, stream,
                           w.own, w.rev_cnt, n, indptr, w.block_tot);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, stream, w.block_tot,
                           std::max<int64_t>(nb, 1), w.res);
        hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n + 1, 256)), dim3(256), 0, stream, indptr, n, w.block_tot,
                           w.res);
        if ((st = launch_status("csr_scan")) != RSC_OK) return st;
    }
    if (m > 0) {
        ScopedTimer t("union_fill", stream);
        hipLaunchKernelGGL(k_union_fill, dim3(grid_for(n, 256)), dim3(256), 0, stream, idx, n, k, w.wf, w.mutual,
                           w.own, indptr, w.cursor, w.tmp_col, w.tmp_val);
        if ((st = launch_status("union_fill")) != RSC_OK) return st;
    }
    if (m > 0) {
        ScopedTimer t("row_sort", stream);
        hipLaunchKernelGGL(k_row_sort, dim3(grid_for(n, 4)), dim3(256), 0, stream, indptr, n, w.tmp_col, w.tmp_val,
                           indices, data, w.res);
        if ((st = launch_status("row_sort")) != RSC_OK) return st;
    }
    GraphResult host;
    if ((st = hip_status(hipMemcpyAsync(&host, w.res, sizeof(host), hipMemcpyDeviceToHost, stream), "read nnz")) !=
        RSC_OK)
        return st;
    if ((st = hip_status(hipStreamSynchronize(stream), "synchronise")) != RSC_OK) return st;
    *nnz = host.nnz;
    if (host.error) {
        set_error(host.error & 1 ? "kNN lists hold an index out of range or the row itself in columns 1..k-1"
                                 : "kNN lists repeat a neighbour within a row");
        return RSC_ERR_BAD_GRAPH;
    }
    return RSC_OK;
}

}  // namespace rsc
