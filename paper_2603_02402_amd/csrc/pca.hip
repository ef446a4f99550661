// Sparse PCA: the embedding the neighbourhood graph is built on (Methods,
// "Principal component analysis").
//
// For a cells x genes CSR matrix X (n x p):
//   mu = X^T 1 / n, S = X^T X (upper triangle), C = (S - n mu mu^T) / (n - 1)
//   top-k eigenpairs of C (float64), Z = X V - 1 (mu^T V).
//
// Gram.  The cells are taken in chunks; each chunk is densified into a
// row-major float32 buffer whose rows are padded to a multiple of 64 genes
// plus one extra column that is 1 for every cell, so that the column of S
// for that "gene" is X^T 1 (the means need no separate reduction).  The
// upper-triangle 64 x 64 tiles of S are accumulated on the float64 matrix
// cores (v_mfma_f64_16x16x4_f64: float32 products are exact in float64):
// a workgroup owns one tile and one range of the chunk's cells, stages 64
// cells of the two gene slices through LDS per step, and writes its float64
// partial; the partials of all ranges and chunks are added in a fixed order,
// so S is deterministic.  Centring and the copy of the upper triangle into
// the lower one are one elementwise kernel.
//
// Eigendecomposition: rocSOLVER's float64 symmetric solver (dsyevd) on the
// workspace, then the k largest pairs in descending order with each loading
// signed so that its largest-magnitude entry is positive.  Scores: one wave
// per cell, lane t sums x_cg V[g][t] over the row in float64.

#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <mutex>

#include "rsc_internal.hpp"

namespace rsc {
namespace {

constexpr int kWave = 64;
constexpr int kPT = 64;                  // genes per tile side
constexpr int kPK = 64;                  // cells staged per step
constexpr int kPStride = kPT + 1;        // LDS row stride (floats)
constexpr int kPThreads = 256;
constexpr int kMaxComponents = 64;
constexpr size_t kChunkBytes = size_t(1) << 31;  // dense chunk budget (2 GiB)

typedef double f64x4 __attribute__((ext_vector_type(4)));

// padded width of a dense row: p genes + the constant column, rounded up to 64
inline int padded(int p) { return (p + 1 + kPT - 1) / kPT * kPT; }

// Dense chunk: rows c0 .. c0 + rows - 1 of X into Xd (rows x P), the
// constant column p set to 1, everything else 0.  One thread per dense
// element for the fill, then one per stored entry for the scatter.
__global__ __launch_bounds__(256) void k_pca_fill(float *__restrict__ Xd, int64_t total, int P, int p) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x)
        Xd[e] = (int)(e % P) == p ? 1.f : 0.f;
}

__global__ __launch_bounds__(256) void k_pca_scatter(const int64_t *__restrict__ indptr,
                                                     const int32_t *__restrict__ indices,
                                                     const float *__restrict__ data, int64_t c0, int64_t rows, int P,
                                                     int p, float *__restrict__ Xd, int32_t *__restrict__ err) {
    // one wave per row
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t r = wave; r < rows; r += nw) {
        const int64_t lo = indptr[c0 + r], hi = indptr[c0 + r + 1];
        for (int64_t e = lo + lane; e < hi; e += kWave) {
            const int32_t g = indices[e];
            if (g < 0 || g >= p) {
                atomicOr(err, 1);
                continue;
            }
            Xd[r * P + g] = data[e];  // (the genes of a row are distinct)
        }
    }
}

// Upper-triangle tiles of S: blockIdx.x = tile (I <= J, row-major over the
// T x T tile grid), blockIdx.y = cell range of this chunk.  Partial tile of
// range s written to part[(s * ntiles + tile) * 4096].
__global__ __launch_bounds__(kPThreads, 2) void k_pca_gram(const float *__restrict__ Xd, int64_t rows, int P,
                                                           const int32_t *__restrict__ tile_i,
                                                           const int32_t *__restrict__ tile_j, int ntiles,
                                                           int64_t per, double *__restrict__ part) {
    __shared__ float As[kPK * kPStride];
    __shared__ float Bs[kPK * kPStride];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    const int tile = blockIdx.x;
    const int I0 = tile_i[tile] * kPT, J0 = tile_j[tile] * kPT;
    const int64_t r0 = (int64_t)blockIdx.y * per, r1 = std::min<int64_t>(rows, r0 + per);
    f64x4 c[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) c[b] = f64x4{0.0, 0.0, 0.0, 0.0};
    // staging: thread t copies 32 consecutive genes of cell (t % 128) / 2 of side t / 128
    const int side = tid >> 7, srow = (tid & 127) >> 1, half = tid & 1;
    float *dst = (side ? Bs : As) + srow * kPStride + half * 32;
    const int col0 = (side ? J0 : I0) + half * 32;
    for (int64_t k0 = r0; k0 < r1; k0 += kPK) {
        const int64_t cell = k0 + srow;
        float v[32];
        if (cell < r1) {
            const float4 *src = reinterpret_cast<const float4 *>(Xd + cell * P + col0);
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const float4 t = src[u];
                v[4 * u] = t.x;
                v[4 * u + 1] = t.y;
                v[4 * u + 2] = t.z;
                v[4 * u + 3] = t.w;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 32; ++u) v[u] = 0.f;
        }
        __syncthreads();  // the previous step's operand reads are done
#pragma unroll
        for (int u = 0; u < 32; ++u) dst[u] = v[u];
        __syncthreads();
        // A[i][k] = Xd[cell k][I0 + i], B[k][j] = Xd[cell k][J0 + j]; lane l gives
        // A[l % 16][l / 16] and B[l / 16][l % 16]
#pragma unroll 4
        for (int ks = 0; ks < kPK; ks += 4) {
            const float *ra = As + (ks + lk) * kPStride + wr * 32 + lr;
            const float *rb = Bs + (ks + lk) * kPStride + wc * 32 + lr;
            const double a0 = (double)ra[0], a1 = (double)ra[16];
            const double b0 = (double)rb[0], b1 = (double)rb[16];
            c[0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c[0], 0, 0, 0);
            c[1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c[1], 0, 0, 0);
            c[2] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c[2], 0, 0, 0);
            c[3] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c[3], 0, 0, 0);
        }
    }
    // output register q of block (bi, bj): row 4 q + lk, column lr
    double *out = part + ((int64_t)blockIdx.y * ntiles + tile) * (kPT * kPT);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
        const int bi = b >> 1, bj = b & 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = wr * 32 + bi * 16 + 4 * q + lk, j = wc * 32 + bj * 16 + lr;
            out[i * kPT + j] = c[b][q];
        }
    }
}

// S[tile] += sum over ranges of the partials (in range order).
__global__ __launch_bounds__(256) void k_pca_reduce(const double *__restrict__ part, int nsplit, int ntiles,
                                                    const int32_t *__restrict__ tile_i,
                                                    const int32_t *__restrict__ tile_j, int P,
                                                    double *__restrict__ S) {
    const int tile = blockIdx.x;
    const int I0 = tile_i[tile] * kPT, J0 = tile_j[tile] * kPT;
    for (int e = threadIdx.x; e < kPT * kPT; e += blockDim.x) {
        double s = 0.0;
        for (int r = 0; r < nsplit; ++r) s += part[((int64_t)r * ntiles + tile) * (kPT * kPT) + e];
        const int i = e / kPT, j = e % kPT;
        S[(int64_t)(I0 + i) * P + J0 + j] += s;
    }
}

__global__ __launch_bounds__(256) void k_pca_zero(double *__restrict__ x, int64_t m) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x)
        x[e] = 0.0;
}

// mu_j = S[j][p] / n; C[i][j] = C[j][i] = (S[i][j] - n mu_i mu_j) / (n - 1) for
// i <= j (the upper triangle of S holds the sums; copied without branches
// on the position).
__global__ __launch_bounds__(256) void k_pca_center(const double *__restrict__ S, int P, int p, int64_t n,
                                                    double *__restrict__ mu, double *__restrict__ C) {
    const double dn = (double)n, dn1 = (double)(n - 1);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)p * p;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e % p);
        const int lo = min(i, j), hi = max(i, j);
        const double mi = S[(int64_t)lo * P + p] / dn, mj = S[(int64_t)hi * P + p] / dn;
        C[e] = (S[(int64_t)lo * P + hi] - dn * (mi * mj)) / dn1;
        if (i == j) mu[i] = mi;
    }
}

// The k largest eigenpairs (dsyevd leaves them ascending, vectors as the
// columns of A in column-major order, i.e. rows of A seen row-major), each
// loading signed so that its largest-magnitude entry (lowest index on ties)
// is positive.  One wave per component.
__global__ __launch_bounds__(64) void k_pca_select(const double *__restrict__ A, const double *__restrict__ W, int p,
                                                   int k, double *__restrict__ evals, double *__restrict__ V) {
    const int t = blockIdx.x, lane = threadIdx.x;
    const int src = p - 1 - t;
    const double *v = A + (int64_t)src * p;
    double best = -1.0;
    int bi = INT_MAX;
    for (int i = lane; i < p; i += kWave) {
        const double m = fabs(v[i]);
        if (m > best) {
            best = m;
            bi = i;
        }
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {
        const double ob = __shfl_xor(best, o, kWave);
        const int oi = __shfl_xor(bi, o, kWave);
        if (ob > best || (ob == best && oi < bi)) {
            best = ob;
            bi = oi;
        }
    }
    const double sgn = v[bi] < 0.0 ? -1.0 : 1.0;
    for (int i = lane; i < p; i += kWave) V[(int64_t)i * k + t] = sgn * v[i];
    if (lane == 0) evals[t] = W[src];
}

// mv[t] = sum_g mu_g V[g][t] (genes in order).
__global__ __launch_bounds__(64) void k_pca_muv(const double *__restrict__ mu, const double *__restrict__ V, int p,
                                                int k, double *__restrict__ mv) {
    const int t = threadIdx.x;
    if (t >= k) return;
    double s = 0.0;
    for (int g = 0; g < p; ++g) s += mu[g] * V[(int64_t)g * k + t];
    mv[t] = s;
}

// Z[c][t] = sum over the row's entries of x_cg V[g][t] (in stored order) - mv[t].
__global__ __launch_bounds__(256) void k_pca_scores(const int64_t *__restrict__ indptr,
                                                    const int32_t *__restrict__ indices,
                                                    const float *__restrict__ data, int64_t n, int p, int k,
                                                    const double *__restrict__ V, const double *__restrict__ mv,
                                                    float *__restrict__ Z) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
    for (int64_t c = wave; c < n; c += nw) {
        double s = 0.0;
        const int64_t lo = indptr[c], hi = indptr[c + 1];
        for (int64_t e = lo; e < hi; ++e) {
            const int32_t g = indices[e];
            if (lane < k && g >= 0 && g < p) s += (double)data[e] * V[(int64_t)g * k + lane];
        }
        if (lane < k) Z[c * k + lane] = (float)(s - mv[lane]);
    }
}

// ---- host side ----------------------------------------------------------

struct PcaLayout {
    int P, T, ntiles, nsplit;
    int64_t chunk, per;
    size_t bytes;
    // offsets into the workspace
    size_t o_tile_i, o_tile_j, o_part, o_S, o_Xd, o_A, o_W, o_E, o_info, o_err, o_mv, o_solver;
};

// One rocBLAS handle per device, created on first use and kept for the
// process (the solver's own allocations stay with it).  Its stream and
// workspace are set per call, so calls on one device hold solver_lock()
// while they use it.
std::mutex &solver_lock() {
    static std::mutex m;
    return m;
}

rocblas_handle solver_handle() {
    static std::mutex mu;
    static rocblas_handle handles[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    std::lock_guard<std::mutex> g(mu);
    if (!handles[dev] && rocblas_create_handle(&handles[dev]) != rocblas_status_success) handles[dev] = nullptr;
    return handles[dev];
}

size_t solver_bytes(int p) {
    rocblas_handle h = solver_handle();
    if (!h) return 0;
    std::lock_guard<std::mutex> lock(solver_lock());
    size_t bytes = 0;
    if (rocblas_start_device_memory_size_query(h) != rocblas_status_success) return 0;
    rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, p, nullptr, p, nullptr, nullptr, nullptr);
    if (rocblas_stop_device_memory_size_query(h, &bytes) != rocblas_status_success) return 0;
    return bytes;
}

bool layout(int64_t n, int p, int k, bool eig, PcaLayout *L) {
    if (n < 2 || p < 1 || p > 16384 || k < 0 || k > std::min(p, kMaxComponents)) return false;
    L->P = padded(p);
    L->T = L->P / kPT;
    L->ntiles = L->T * (L->T + 1) / 2;
    L->chunk = std::max<int64_t>(kPK, std::min<int64_t>(n, (int64_t)(kChunkBytes / (sizeof(float) * L->P))));
    // enough cell ranges that tiles x ranges fills the chip (about 2048 workgroups)
    L->nsplit = (int)std::min<int64_t>(std::max<int64_t>(1, 2048 / L->ntiles), (L->chunk + kPK - 1) / kPK);
    L->per = ((L->chunk + L->nsplit - 1) / L->nsplit + kPK - 1) / kPK * kPK;
    Carver cv(nullptr);
    L->o_tile_i = cv.used; cv.take<int32_t>(L->ntiles);
    L->o_tile_j = cv.used; cv.take<int32_t>(L->ntiles);
    L->o_part = cv.used; cv.take<double>((size_t)L->nsplit * L->ntiles * kPT * kPT);
    L->o_S = cv.used; cv.take<double>((size_t)L->P * L->P);
    L->o_Xd = cv.used; cv.take<float>((size_t)L->chunk * L->P);
    L->o_A = cv.used; cv.take<double>((size_t)p * p);
    L->o_W = cv.used; cv.take<double>(p);
    L->o_E = cv.used; cv.take<double>(p);
    L->o_info = cv.used; cv.take<int32_t>(1);
    L->o_err = cv.used; cv.take<int32_t>(1);
    L->o_mv = cv.used; cv.take<double>(kMaxComponents);
    L->o_solver = cv.used;
    if (eig) {
        const size_t sb = solver_bytes(p);
        if (sb == 0) return false;
        cv.take<char>(sb);
    }
    L->bytes = cv.used;
    return true;
}

template <class T>
T *at(void *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

__global__ void k_pca_tiles(int T, int32_t *ti, int32_t *tj) {
    int t = 0;
    for (int i = 0; i < T; ++i)
        for (int j = i; j < T; ++j, ++t) {
            ti[t] = i;
            tj[t] = j;
        }
}

__global__ void k_pca_clear(int32_t *x) { *x = 0; }

int check(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int p) {
    if (!indptr || !indices || !data) {
        set_error("pca: null CSR array");
        return RSC_ERR_INVALID_ARG;
    }
    if (n < 2 || p < 1 || p > 16384) {
        set_error("pca: need n >= 2 cells and 1 <= p <= 16384 genes");
        return RSC_ERR_INVALID_ARG;
    }
    return RSC_OK;
}

// mean (p) and covariance (p x p) into mu and C (device).
int covariance(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int p, const PcaLayout &L,
               void *ws, double *mu, double *C, hipStream_t s) {
    int32_t *ti = at<int32_t>(ws, L.o_tile_i), *tj = at<int32_t>(ws, L.o_tile_j);
    double *part = at<double>(ws, L.o_part), *S = at<double>(ws, L.o_S);
    float *Xd = at<float>(ws, L.o_Xd);
    int32_t *err = at<int32_t>(ws, L.o_err);
    hipLaunchKernelGGL(k_pca_tiles, dim3(1), dim3(1), 0, s, L.T, ti, tj);
    hipLaunchKernelGGL(k_pca_clear, dim3(1), dim3(1), 0, s, err);
    hipLaunchKernelGGL(k_pca_zero, dim3(4096), dim3(256), 0, s, S, (int64_t)L.P * L.P);
    int st;
    if ((st = launch_status("pca setup")) != RSC_OK) return st;
    for (int64_t c0 = 0; c0 < n; c0 += L.chunk) {
        const int64_t rows = std::min<int64_t>(L.chunk, n - c0);
        {
            ScopedTimer t("pca_densify", s);
            hipLaunchKernelGGL(k_pca_fill, dim3(8192), dim3(256), 0, s, Xd, rows * L.P, L.P, p);
            hipLaunchKernelGGL(k_pca_scatter, dim3((unsigned)std::min<int64_t>(16384, (rows + 3) / 4)), dim3(256), 0,
                               s, indptr, indices, data, c0, rows, L.P, p, Xd, err);
        }
        const int nsplit = (int)std::min<int64_t>(L.nsplit, (rows + L.per - 1) / L.per);
        {
            ScopedTimer t("pca_gram", s);
            hipLaunchKernelGGL(k_pca_gram, dim3(L.ntiles, nsplit), dim3(kPThreads), 0, s, Xd, rows, L.P, ti, tj,
                               L.ntiles, L.per, part);
            hipLaunchKernelGGL(k_pca_reduce, dim3(L.ntiles), dim3(256), 0, s, part, nsplit, L.ntiles, ti, tj, L.P, S);
        }
        if ((st = launch_status("pca gram")) != RSC_OK) return st;
    }
    {
        ScopedTimer t("pca_center", s);
        hipLaunchKernelGGL(k_pca_center, dim3(4096), dim3(256), 0, s, S, L.P, p, n, mu, C);
    }
    if ((st = launch_status("pca center")) != RSC_OK) return st;
    int32_t host_err = 0;
    if ((st = hip_status(hipMemcpyAsync(&host_err, err, 4, hipMemcpyDeviceToHost, s), "read check")) != RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (host_err) {
        set_error("pca: a gene index outside [0, p)");
        return RSC_ERR_INVALID_ARG;
    }
    return RSC_OK;
}

}  // namespace

size_t pca_workspace_bytes(int64_t n, int p, int k) {
    PcaLayout L;
    return layout(n, p, k, k > 0, &L) ? L.bytes : 0;
}

int pca_covariance(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int p, double *mean,
                   double *cov, void *ws, size_t ws_bytes, hipStream_t s) {
    int st;
    if ((st = check(indptr, indices, data, n, p)) != RSC_OK) return st;
    if (!mean || !cov) {
        set_error("pca_covariance: null output");
        return RSC_ERR_INVALID_ARG;
    }
    PcaLayout L;
    if (!layout(n, p, 0, false, &L) || !ws || ws_bytes < L.bytes) {
        set_error("pca_covariance: workspace too small");
        return RSC_ERR_WORKSPACE;
    }
    return covariance(indptr, indices, data, n, p, L, ws, mean, cov, s);
}

int pca_run(const int64_t *indptr, const int32_t *indices, const float *data, int64_t n, int p, int k, double *mean,
            double *cov, double *evals, double *loadings, float *Z, void *ws, size_t ws_bytes, hipStream_t s) {
    int st;
    if ((st = check(indptr, indices, data, n, p)) != RSC_OK) return st;
    if (k < 1 || k > std::min(p, kMaxComponents) || !evals || !loadings || !Z) {
        set_error("pca: need 1 <= k <= min(p, 64) and evals, loadings, Z");
        return RSC_ERR_INVALID_ARG;
    }
    PcaLayout L;
    if (!layout(n, p, k, true, &L) || !ws || ws_bytes < L.bytes) {
        set_error("pca: workspace too small (or no device to size the eigensolver)");
        return RSC_ERR_WORKSPACE;
    }
    if (!mean) {
        set_error("pca: null mean (it centres the scores)");
        return RSC_ERR_INVALID_ARG;
    }
    double *A = at<double>(ws, L.o_A);
    double *mu = mean;
    if ((st = covariance(indptr, indices, data, n, p, L, ws, mu, A, s)) != RSC_OK) return st;
    if (cov && (st = hip_status(hipMemcpyAsync(cov, A, sizeof(double) * (size_t)p * p, hipMemcpyDeviceToDevice, s),
                                "copy covariance")) != RSC_OK)
        return st;
    rocblas_handle h = solver_handle();
    if (!h) {
        set_error("pca: cannot create the solver handle");
        return RSC_ERR_HIP;
    }
    double *W = at<double>(ws, L.o_W), *E = at<double>(ws, L.o_E);
    int32_t *info = at<int32_t>(ws, L.o_info);
    {
        ScopedTimer t("pca_eigh", s);
        std::lock_guard<std::mutex> lock(solver_lock());
        if (rocblas_set_stream(h, s) != rocblas_status_success ||
            rocblas_set_workspace(h, at<char>(ws, L.o_solver), L.bytes - L.o_solver) != rocblas_status_success) {
            set_error("pca: solver setup failed");
            return RSC_ERR_HIP;
        }
        const rocblas_status rs =
            rocsolver_dsyevd(h, rocblas_evect_original, rocblas_fill_upper, p, A, p, W, E, (rocblas_int *)info);
        rocblas_set_workspace(h, nullptr, 0);
        if (rs != rocblas_status_success) {
            set_error("pca: rocsolver_dsyevd failed");
            return RSC_ERR_HIP;
        }
    }
    {
        ScopedTimer t("pca_scores", s);
        hipLaunchKernelGGL(k_pca_select, dim3(k), dim3(64), 0, s, A, W, p, k, evals, loadings);
        double *mv = at<double>(ws, L.o_mv);
        hipLaunchKernelGGL(k_pca_muv, dim3(1), dim3(64), 0, s, mu, loadings, p, k, mv);
        hipLaunchKernelGGL(k_pca_scores, dim3((unsigned)std::min<int64_t>(16384, (n + 3) / 4)), dim3(256), 0, s,
                           indptr, indices, data, n, p, k, loadings, mv, Z);
    }
    if ((st = launch_status("pca scores")) != RSC_OK) return st;
    int32_t host_info = 0;
    if ((st = hip_status(hipMemcpyAsync(&host_info, info, 4, hipMemcpyDeviceToHost, s), "read info")) != RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (host_info != 0) {
        set_error("pca: the eigensolver did not converge");
        return RSC_ERR_HIP;
    }
    return RSC_OK;
}

}  // namespace rsc
