// Coarse partitions of the cells for the routed form: Lloyd's k-means, its
// inverted lists, and the partition labels of kNN results.
//
// Assignment is the exact rectangular kNN (k = 1) of the rows against the
// centroids: MFMA screen, float64 rerank and certificate, so every row gets
// its true nearest centroid with ties to the lower index.  Centroid sums are
// integer sums of the rows in fixed point (x * 2^S rounded to int64, S chosen
// from the data's largest magnitude so no sum can overflow): integer addition
// is associative, so the atomics give the same sums in any order and the
// result does not depend on scheduling.  Each centroid is the sum converted
// to float64, scaled back, divided by the count in float64 and rounded to
// float32.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "rsc_internal.hpp"
#include "screen_common.hpp"

namespace rsc {
namespace {

using scr::exact_d2;
using scr::kWave;

__global__ __launch_bounds__(256) void k_absmax_bits(const float *__restrict__ X, int64_t total,
                                                     uint32_t *__restrict__ out) {
    float m = 0.f;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, fabsf(X[e]));
    m = scr::wave_max(m);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(out, __float_as_uint(m));
}

__global__ __launch_bounds__(256) void k_gather_rows(const float *__restrict__ X, int64_t n, int d,
                                                     const int32_t *__restrict__ rows, int P, float *__restrict__ C,
                                                     int32_t *__restrict__ err) {
    const int64_t total = (int64_t)P * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(e / d), t = (int)(e % d);
        const int32_t r = rows[p];
        if (r < 0 || r >= n) {
            if (t == 0) atomicOr(err, 1);
            C[e] = 0.f;
        } else {
            C[e] = X[(int64_t)r * d + t];
        }
    }
}

// counts[0..P) = 0 and sums[0..nsums) = 0.
__global__ __launch_bounds__(256) void k_zero_sums(int32_t *__restrict__ counts, int P,
                                                   unsigned long long *__restrict__ sums, int64_t nsums) {
    const int64_t total = nsums > P ? nsums : (int64_t)P;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
        if (e < nsums) sums[e] = 0ull;
        if (e < P) counts[e] = 0;
    }
}

__device__ __forceinline__ long long fixed_point(float x, int S) { return llrint(ldexp((double)x, S)); }

// counts[p] = rows assigned to p; sums[p][t] = sum of fixed_point(x_t).
__global__ __launch_bounds__(256) void k_accumulate(const float *__restrict__ X, int64_t n, int d,
                                                    const int32_t *__restrict__ assign, int S,
                                                    int32_t *__restrict__ counts,
                                                    unsigned long long *__restrict__ sums) {
    const int64_t total = n * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / d;
        const int t = (int)(e - row * d);
        const int p = assign[row];
        atomicAdd(&sums[(int64_t)p * d + t], (unsigned long long)fixed_point(X[e], S));
        if (t == 0) atomicAdd(&counts[p], 1);
    }
}

// Exact squared distance of every row to its assigned centroid.
__global__ __launch_bounds__(256) void k_row_d2(const float *__restrict__ X, int64_t n, int d,
                                                const float *__restrict__ C, const int32_t *__restrict__ assign,
                                                double *__restrict__ d2) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
        d2[r] = exact_d2(X + r * d, C + (int64_t)assign[r] * d, d);
}

// Exact nearest centroid of every row by brute force, for d <= 64 and at
// most 2048 centroids: the row
// sits in registers as float64 (zero-padded to DMAX dimensions, which adds
// exact zeros to every sum), the centroids pass through LDS in tiles of
// kAssignTile rows, and every distance is exact_d2's (differences, squares
// and sums rounded as written, in dimension order); ties go to the lowest
// centroid index.  So the assignment is the exact k = 1 search's, at
// 3 DMAX P float64 operations per row.
constexpr int kAssignTile = 64;

template <int DMAX>
__global__ __launch_bounds__(256) void k_assign_exact(const float *__restrict__ X, int64_t n, int d,
                                                      const float *__restrict__ C, int P,
                                                      int32_t *__restrict__ assign) {
    __shared__ double ct[kAssignTile * DMAX];
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double x[DMAX];
#pragma unroll
    for (int t = 0; t < DMAX; ++t) x[t] = (r < n && t < d) ? (double)X[r * d + t] : 0.0;
    double best = INFINITY;
    int32_t bj = 0;
    for (int j0 = 0; j0 < P; j0 += kAssignTile) {
        const int nt = P - j0 < kAssignTile ? P - j0 : kAssignTile;
        __syncthreads();  // the previous tile is no longer read
        for (int e = threadIdx.x; e < kAssignTile * DMAX; e += blockDim.x) {
            const int jj = e / DMAX, t = e - jj * DMAX;
            ct[e] = (jj < nt && t < d) ? (double)C[(int64_t)(j0 + jj) * d + t] : 0.0;
        }
        __syncthreads();
        for (int jj = 0; jj < nt; ++jj) {
            const double *c = ct + jj * DMAX;  // the same address on every lane: broadcast reads
            double s = 0.0;
#pragma unroll
            for (int t = 0; t < DMAX; ++t) {
                const double diff = __dsub_rn(x[t], c[t]);
                s = __dadd_rn(s, __dmul_rn(diff, diff));
            }
            if (s < best) {
                best = s;
                bj = j0 + jj;
            }
        }
    }
    if (r < n) assign[r] = bj;
}

// (d2 desc, index asc): whether (da, ia) comes first.
__device__ __forceinline__ bool farther(double da, int64_t ia, double db, int64_t ib) {
    return da > db || (da == db && ia < ib);
}

// Stage 1 of the farthest-row search: best row of each block's stride
// (taken rows carry d2 = -1).
__global__ __launch_bounds__(256) void k_far_partial(const double *__restrict__ d2, int64_t n,
                                                     double *__restrict__ pd, int64_t *__restrict__ pi) {
    __shared__ double sd[256];
    __shared__ int64_t si[256];
    double bd = -2.0;
    int64_t bi = INT64_MAX;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        if (farther(d2[r], r, bd, bi)) {
            bd = d2[r];
            bi = r;
        }
    }
    sd[threadIdx.x] = bd;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && farther(sd[threadIdx.x + w], si[threadIdx.x + w], sd[threadIdx.x], si[threadIdx.x])) {
            sd[threadIdx.x] = sd[threadIdx.x + w];
            si[threadIdx.x] = si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        pd[blockIdx.x] = sd[0];
        pi[blockIdx.x] = si[0];
    }
}

// Stage 2: the overall farthest row becomes chosen[j] and is marked taken.
__global__ __launch_bounds__(256) void k_far_final(const double *__restrict__ pd, const int64_t *__restrict__ pi,
                                                   int nparts, double *__restrict__ d2, int32_t *__restrict__ chosen,
                                                   int j) {
    __shared__ double sd[256];
    __shared__ int64_t si[256];
    double bd = -2.0;
    int64_t bi = INT64_MAX;
    for (int b = threadIdx.x; b < nparts; b += blockDim.x) {
        if (farther(pd[b], pi[b], bd, bi)) {
            bd = pd[b];
            bi = pi[b];
        }
    }
    sd[threadIdx.x] = bd;
    si[threadIdx.x] = bi;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w && farther(sd[threadIdx.x + w], si[threadIdx.x + w], sd[threadIdx.x], si[threadIdx.x])) {
            sd[threadIdx.x] = sd[threadIdx.x + w];
            si[threadIdx.x] = si[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        chosen[j] = (int32_t)si[0];
        d2[si[0]] = -1.0;
    }
}

// Move chosen[j] into empty partition empties[j], j = 0..m-1 in order (one
// block, thread t handles dimension t).
__global__ __launch_bounds__(128) void k_relocate(const float *__restrict__ X, int d, int S,
                                                  const int32_t *__restrict__ chosen,
                                                  const int32_t *__restrict__ empties, int m,
                                                  int32_t *__restrict__ assign, int32_t *__restrict__ counts,
                                                  unsigned long long *__restrict__ sums) {
    const int t = threadIdx.x;
    for (int j = 0; j < m; ++j) {
        const int32_t r = chosen[j], e = empties[j];
        const int32_t old = assign[r];
        if (t < d) {
            const unsigned long long v = (unsigned long long)fixed_point(X[(int64_t)r * d + t], S);
            sums[(int64_t)old * d + t] -= v;
            sums[(int64_t)e * d + t] += v;
        }
        __syncthreads();
        if (t == 0) {
            counts[old] -= 1;
            counts[e] += 1;
            assign[r] = e;
        }
        __syncthreads();
    }
}

// Centroid = exact sum / count (float64), rounded to float32; partitions
// without rows keep their centroid.
__global__ __launch_bounds__(256) void k_update(const unsigned long long *__restrict__ sums,
                                                const int32_t *__restrict__ counts, int P, int d, int S,
                                                float *__restrict__ C) {
    const int64_t total = (int64_t)P * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int p = (int)(e / d);
        const int cnt = counts[p];
        if (cnt > 0) C[e] = (float)(ldexp((double)(long long)sums[e], -S) / (double)cnt);
    }
}

// Relocated centroids are their row, exactly.
__global__ __launch_bounds__(128) void k_set_relocated(const float *__restrict__ X, int d,
                                                       const int32_t *__restrict__ chosen,
                                                       const int32_t *__restrict__ empties, int m,
                                                       float *__restrict__ C) {
    for (int j = blockIdx.x; j < m; j += gridDim.x)
        for (int t = threadIdx.x; t < d; t += blockDim.x) C[(int64_t)empties[j] * d + t] = X[(int64_t)chosen[j] * d + t];
}

__global__ __launch_bounds__(256) void k_count(const int32_t *__restrict__ assign, int64_t n, int P,
                                               int32_t *__restrict__ counts, int32_t *__restrict__ err) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = assign[r];
        if (p < 0 || p >= P) {
            atomicOr(err, 1);
            continue;
        }
        atomicAdd(&counts[p], 1);
    }
}

// Exclusive scan of counts[0..P) into offsets[0..P] (one block of 1024).
__global__ __launch_bounds__(1024) void k_scan_counts(const int32_t *__restrict__ counts, int P,
                                                      int64_t *__restrict__ offsets, int32_t *__restrict__ cursor) {
    __shared__ int64_t part[1024];
    const int per = (P + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(P, lo + per);
    int64_t s = 0;
    for (int i = lo; i < hi; ++i) s += counts[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t v = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += v;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int i = lo; i < hi; ++i) {
        offsets[i] = run;
        if (cursor) cursor[i] = 0;
        run += counts[i];
    }
    if (threadIdx.x == 1023) offsets[P] = part[1023];
}

__global__ __launch_bounds__(256) void k_fill_lists(const int32_t *__restrict__ assign, int64_t n, int P,
                                                    const int64_t *__restrict__ offsets,
                                                    int32_t *__restrict__ cursor, int32_t *__restrict__ perm) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = assign[r];
        if (p < 0 || p >= P) continue;
        perm[offsets[p] + atomicAdd(&cursor[p], 1)] = (int32_t)r;
    }
}

__global__ __launch_bounds__(256) void k_labels(const int32_t *__restrict__ idx, int64_t total,
                                                const int32_t *__restrict__ assign, int64_t n_assign,
                                                int32_t *__restrict__ labels) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t j = idx[e];
        labels[e] = (j < 0 || j >= n_assign) ? -1 : assign[j];
    }
}

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 16384)); }
constexpr int kFarBlocks = 512;

struct KmeansBuffers {
    void *knn_ws;
    size_t knn_bytes;
    int32_t *counts, *chosen, *empties, *cursor, *err;
    unsigned long long *sums;
    double *d2, *far_d;
    int64_t *far_i;
    float *dist;
    uint32_t *absmax;
};

size_t carve_kmeans(int64_t n, int d, int P, void *ws, KmeansBuffers *out) {
    KnnPlan kp;
    if (knn_plan(n, P, d, 1, nullptr, false, &kp) != RSC_OK) return 0;
    Carver cv(ws);
    KmeansBuffers b;
    b.knn_bytes = knn_workspace(kp, nullptr, nullptr);
    b.knn_ws = cv.take<char>(b.knn_bytes);
    b.counts = cv.take<int32_t>(P);
    b.chosen = cv.take<int32_t>(P);
    b.empties = cv.take<int32_t>(P);
    b.cursor = cv.take<int32_t>(P);
    b.err = cv.take<int32_t>(1);
    b.sums = cv.take<unsigned long long>((size_t)P * d);
    b.d2 = cv.take<double>(n);
    b.far_d = cv.take<double>(kFarBlocks);
    b.far_i = cv.take<int64_t>(kFarBlocks);
    b.dist = cv.take<float>(n);
    b.absmax = cv.take<uint32_t>(1);
    if (out) *out = b;
    return cv.used;
}

int assign_pass(const float *X, int64_t n, int d, const float *C, int P, int32_t *assign, const KmeansBuffers &b,
                hipStream_t s) {
    // Brute force costs about 3 (d + 7) float64 operations per (row,
    // centroid) pair on the vector units; the kNN search pays 2 d FP32
    // flops per pair on the matrix cores plus a rerank per row, so it wins
    // once the centroids number a few thousand (measured: 1024 centroids
    // 11.5 against 26 ms per pass over 2M rows; 4096 over 5M rows, the kNN
    // search faster).
    if (d <= 64 && P <= 2048) {
        ScopedTimer t("kmeans_assign", s);
        const unsigned g = (unsigned)((n + 255) / 256);
        switch ((d + 7) / 8) {
            case 1: hipLaunchKernelGGL(k_assign_exact<8>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
            case 2: hipLaunchKernelGGL(k_assign_exact<16>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
            case 3: hipLaunchKernelGGL(k_assign_exact<24>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
            case 4: hipLaunchKernelGGL(k_assign_exact<32>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
            case 5: hipLaunchKernelGGL(k_assign_exact<40>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
            case 6: hipLaunchKernelGGL(k_assign_exact<48>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
            case 7: hipLaunchKernelGGL(k_assign_exact<56>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
            default: hipLaunchKernelGGL(k_assign_exact<64>, dim3(g), dim3(256), 0, s, X, n, d, C, P, assign); break;
        }
        return launch_status("kmeans assignment");
    }
    KnnPlan kp;
    int st = knn_plan(n, P, d, 1, nullptr, false, &kp);
    if (st != RSC_OK) return st;
    TimerPrefix tp("kmeans/");  // the assignment's own screen and rerank
    return knn_run(kp, X, C, assign, b.dist, b.knn_ws, s);
}

int build_lists(const int32_t *assign, int64_t n, int P, int64_t *offsets, int32_t *perm, int32_t *counts,
                int32_t *cursor, int32_t *err, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_sums, dim3(grid_for(P)), dim3(256), 0, s, counts, P, nullptr, 0);
    hipLaunchKernelGGL(k_count, dim3(grid_for(n)), dim3(256), 0, s, assign, n, P, counts, err);
    hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, counts, P, offsets, cursor);
    hipLaunchKernelGGL(k_fill_lists, dim3(grid_for(n)), dim3(256), 0, s, assign, n, P, offsets, cursor, perm);
    return launch_status("partition lists");
}

}  // namespace

size_t kmeans_workspace_bytes(int64_t n, int d, int P) {
    if (n < 1 || d < 1 || P < 1 || P > n) return 0;
    return carve_kmeans(n, d, P, nullptr, nullptr);
}

int kmeans_run(const float *X, int64_t n, int d, int P, const int32_t *init_rows, int iters, float *C,
               int32_t *assign, int64_t *offsets, int32_t *perm, int64_t *relocated, void *ws, size_t ws_bytes,
               hipStream_t s) {
    if (!X || !init_rows || !C || !assign || iters < 0 || (offsets == nullptr) != (perm == nullptr)) {
        set_error("partition_kmeans: null argument, or offsets and perm not given together");
        return RSC_ERR_INVALID_ARG;
    }
    if (n > INT32_MAX - 1) {
        set_error("partition_kmeans: more rows than int32 can index");
        return RSC_ERR_OVERFLOW;
    }
    if (n < 1 || d < 1 || d > 128 || P < 1 || P > n) {
        set_error("partition_kmeans: need 1 <= parts <= n and 1 <= d <= 128");
        return RSC_ERR_INVALID_ARG;
    }
    KmeansBuffers b;
    const size_t need = carve_kmeans(n, d, P, ws, &b);
    if (!ws || need == 0 || need > ws_bytes || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1))) {
        set_error("partition_kmeans: workspace too small or misaligned: need " + std::to_string(need) + " bytes");
        return RSC_ERR_WORKSPACE;
    }
    ScopedTimer timer("kmeans", s);
    int st;
    // fixed-point shift from the largest magnitude: n * max|x| * 2^S < 2^62
    hipLaunchKernelGGL(k_zero_sums, dim3(1), dim3(64), 0, s, b.err, 1, nullptr, 0);
    hipLaunchKernelGGL(k_zero_sums, dim3(1), dim3(64), 0, s, reinterpret_cast<int32_t *>(b.absmax), 1, nullptr, 0);
    hipLaunchKernelGGL(k_absmax_bits, dim3(grid_for(n * d)), dim3(256), 0, s, X, n * d, b.absmax);
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for((int64_t)P * d)), dim3(256), 0, s, X, n, d, init_rows, P, C, b.err);
    if ((st = launch_status("kmeans init")) != RSC_OK) return st;
    uint32_t host_bits = 0;
    int32_t host_err = 0;
    if ((st = hip_status(hipMemcpyAsync(&host_bits, b.absmax, 4, hipMemcpyDeviceToHost, s), "read max")) != RSC_OK ||
        (st = hip_status(hipMemcpyAsync(&host_err, b.err, 4, hipMemcpyDeviceToHost, s), "read check")) != RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (host_err) {
        set_error("partition_kmeans: init_rows holds a row id outside [0, n)");
        return RSC_ERR_INVALID_ARG;
    }
    float amax;
    std::memcpy(&amax, &host_bits, 4);
    if (!std::isfinite(amax)) {
        set_error("partition_kmeans: non-finite input");
        return RSC_ERR_INVALID_ARG;
    }
    int e_amax = 0;
    std::frexp(std::max(amax, 1e-30f), &e_amax);  // amax < 2^e_amax
    int e_n = 0;
    std::frexp((double)n, &e_n);                  // n < 2^e_n
    const int S = std::min(62 - e_amax - e_n, 1000);
    int64_t nrel = 0;
    std::vector<int32_t> counts(P), empties;
    for (int it = 0; it < iters; ++it) {
        if ((st = assign_pass(X, n, d, C, P, assign, b, s)) != RSC_OK) return st;
        hipLaunchKernelGGL(k_zero_sums, dim3(grid_for((int64_t)P * d)), dim3(256), 0, s, b.counts, P, b.sums,
                           (int64_t)P * d);
        hipLaunchKernelGGL(k_accumulate, dim3(grid_for(n * d)), dim3(256), 0, s, X, n, d, assign, S, b.counts, b.sums);
        if ((st = launch_status("kmeans accumulate")) != RSC_OK) return st;
        if ((st = hip_status(hipMemcpyAsync(counts.data(), b.counts, (size_t)P * 4, hipMemcpyDeviceToHost, s),
                             "read counts")) != RSC_OK ||
            (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
            return st;
        empties.clear();
        for (int p = 0; p < P; ++p)
            if (counts[p] == 0) empties.push_back(p);
        const int m = (int)empties.size();
        if (m > 0) {
            nrel += m;
            if ((st = hip_status(hipMemcpyAsync(b.empties, empties.data(), (size_t)m * 4, hipMemcpyHostToDevice, s),
                                 "upload empties")) != RSC_OK)
                return st;
            hipLaunchKernelGGL(k_row_d2, dim3(grid_for(n)), dim3(256), 0, s, X, n, d, C, assign, b.d2);
            for (int j = 0; j < m; ++j) {
                hipLaunchKernelGGL(k_far_partial, dim3(kFarBlocks), dim3(256), 0, s, b.d2, n, b.far_d, b.far_i);
                hipLaunchKernelGGL(k_far_final, dim3(1), dim3(256), 0, s, b.far_d, b.far_i, kFarBlocks, b.d2,
                                   b.chosen, j);
            }
            hipLaunchKernelGGL(k_relocate, dim3(1), dim3(128), 0, s, X, d, S, b.chosen, b.empties, m, assign,
                               b.counts, b.sums);
        }
        hipLaunchKernelGGL(k_update, dim3(grid_for((int64_t)P * d)), dim3(256), 0, s, b.sums, b.counts, P, d, S, C);
        if (m > 0)
            hipLaunchKernelGGL(k_set_relocated, dim3(std::min(m, 1024)), dim3(128), 0, s, X, d, b.chosen, b.empties,
                               m, C);
        if ((st = launch_status("kmeans update")) != RSC_OK) return st;
        // the host vector of empties must outlive the upload above
        if (m > 0 && (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK) return st;
    }
    if ((st = assign_pass(X, n, d, C, P, assign, b, s)) != RSC_OK) return st;
    if (offsets && (st = build_lists(assign, n, P, offsets, perm, b.counts, b.cursor, b.err, s)) != RSC_OK) return st;
    if (relocated) *relocated = nrel;
    return RSC_OK;
}

int partition_lists(const int32_t *assign, int64_t n, int P, int64_t *offsets, int32_t *perm, void *ws,
                     size_t ws_bytes, hipStream_t s) {
    if (!assign || !offsets || !perm || n < 0 || P < 1) {
        set_error("partition_lists: null argument or parts < 1");
        return RSC_ERR_INVALID_ARG;
    }
    if (n > INT32_MAX - 1) {
        set_error("partition_lists: more rows than int32 can index");
        return RSC_ERR_OVERFLOW;
    }
    Carver cv(ws);
    int32_t *counts = cv.take<int32_t>(P);
    int32_t *cursor = cv.take<int32_t>(P);
    int32_t *err = cv.take<int32_t>(1);
    if (!ws || cv.used > ws_bytes) {
        set_error("partition_lists: workspace too small: need " + std::to_string(cv.used) + " bytes");
        return RSC_ERR_WORKSPACE;
    }
    hipLaunchKernelGGL(k_zero_sums, dim3(1), dim3(64), 0, s, err, 1, nullptr, 0);
    int st = build_lists(assign, n, P, offsets, perm, counts, cursor, err, s);
    if (st != RSC_OK) return st;
    int32_t host_err = 0;
    if ((st = hip_status(hipMemcpyAsync(&host_err, err, 4, hipMemcpyDeviceToHost, s), "read check")) != RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (host_err) {
        set_error("partition_lists: a label outside [0, parts)");
        return RSC_ERR_INVALID_ARG;
    }
    return RSC_OK;
}

size_t partition_lists_workspace_bytes(int P) {
    Carver cv(nullptr);
    cv.take<int32_t>(P);
    cv.take<int32_t>(P);
    cv.take<int32_t>(1);
    return cv.used;
}

int partition_labels(const int32_t *idx, int64_t n, int k, const int32_t *assign, int64_t n_assign, int32_t *labels,
                     hipStream_t s) {
    if (!idx || !assign || !labels || n < 0 || k < 1 || n_assign < 1) {
        set_error("partition_labels: null argument or bad size");
        return RSC_ERR_INVALID_ARG;
    }
    hipLaunchKernelGGL(k_labels, dim3(grid_for(n * k)), dim3(256), 0, s, idx, n * k, assign, n_assign, labels);
    return launch_status("partition labels");
}

}  // namespace rsc
