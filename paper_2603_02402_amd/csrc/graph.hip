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
// Stages (m = k - 1 directed edges per row, E = n m edges):
//   smooth   one thread per row: rho, the bisection for sigma, and the m
//            directed weights a (float64, row-major n x m);
//   probe    one lane per edge, whole rows per wave (64 / m rows): the lane
//            of edge i -> j loads j's m neighbour ids in one batch and looks
//            for i; the union weight is computed once from the two float64
//            weights, and the row's kept entries are counted with a ballot.
//            A kept one-way edge takes a slot among j's reverse entries from
//            an atomic counter and records it, so no later pass needs
//            another atomic;
//   scan     two int64 exclusive scans in one pass: row lengths (own kept
//            edges + reverse entries) -> indptr, and reverse counts -> the
//            start of each row's reverse entries;
//   fill     one lane per edge again: each kept one-way edge writes (i, w)
//            as one 8-byte record into its slot of j's reverse entries;
//   sort     one wave per row: the row's own edges (read from the edge
//            arrays in place) and its reverse entries are ranked by column
//            with lane broadcasts and written to their sorted positions in
//            the CSR, which also makes the output independent of the atomic
//            slot order.
// Weights of a pair are computed from the same two float64 operands with
// commutative operations, so w_ij and w_ji are bitwise equal.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <mutex>
#include <string>

#include "rsc_internal.hpp"

namespace rsc {
namespace {

constexpr int kWave = 64;
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kEdgeBlock = 256;  // threads per block of the per-edge kernels (4 waves)

struct GraphResult {
    int64_t nnz;
    int32_t error;  // bit 0: index out of range or self; bit 1: repeated neighbour; bit 2: edge leaves its sample
    int32_t degenerate;
    int32_t long_rows;  // rows of more than 64 entries, listed for the second sort kernel
    int32_t pad;
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
        r->long_rows = 0;
    }
}

// Sum over the row's neighbour slots of exp(-g_j * rinv) with g_j =
// max(0, d_j - rho), in slot order.  The bisection multiplies by the
// reciprocal of sigma (one division per step instead of one per slot); the
// weights themselves divide by sigma as the definition writes them.
template <int KM>
__device__ __forceinline__ double membership_sum(const double (&gg)[KM], int m, double rinv) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < KM; ++j)
        if (j < m) s = __dadd_rn(s, exp(-gg[j] * rinv));
    return s;
}

// Bisection for sigma from sigma = 1: double until the sum exceeds the
// target, then halve the bracket; stop when the sum is within 1e-12 of the
// target (relative), the bracket is one ulp wide, or after 200 steps.
template <class SumFn>
__device__ __forceinline__ double bisect_sigma(double target, SumFn sum_at) {
    double sigma = 1.0;
    double lo = 0.0, hi = INFINITY;
    for (int it = 0; it < 200; ++it) {
        const double f = sum_at(1.0 / sigma);
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
    return sigma;
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
    double gg[KM];
#pragma unroll
    for (int j = 0; j < KM; ++j) {
        if (j < m && dd[j] <= rho) ++at_rho;
        const double g = dd[j] - rho;
        gg[j] = g < 0.0 ? 0.0 : g;
    }
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
        sigma = bisect_sigma(target, [&](double rinv) { return membership_sum<KM>(gg, m, rinv); });
#pragma unroll
        for (int j = 0; j < KM; ++j)
            if (j < m) ai[j] = exp(-gg[j] / sigma);
    }
    if (rho_out) rho_out[i] = rho;
    if (sigma_out) sigma_out[i] = sigma;
}

// The same computation for rows with more than 64 neighbour slots: the
// distances are read from memory (in slot order, as above) instead of being
// held in registers.
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
        sigma = bisect_sigma(target, [&](double rinv) {
            double s = 0.0;
            for (int j = 0; j < m; ++j) {
                double g = (double)dr[j] - rho;
                if (g < 0.0) g = 0.0;
                s = __dadd_rn(s, exp(-g * rinv));
            }
            return s;
        });
        for (int j = 0; j < m; ++j) {
            double g = (double)dr[j] - rho;
            if (g < 0.0) g = 0.0;
            ai[j] = exp(-g / sigma);
        }
    }
    if (rho_out) rho_out[i] = rho;
    if (sigma_out) sigma_out[i] = sigma;
}

// Lane -> (row within the wave's group, slot) of the per-edge kernels.  A
// group is R = 64 / m whole rows when m <= 32 (a row's edges sit on
// consecutive lanes), else one row walked in chunks of 64 slots.
struct EdgeMap {
    int m, R;
    int64_t groups;
    __device__ EdgeMap(int64_t n, int m_) : m(m_), R(m_ <= 32 ? kWave / m_ : 1), groups((n + R - 1) / R) {}
};

// Sample bounds of row i: [seg[s], seg[s+1]) with seg ascending (S samples).
__device__ __forceinline__ void sample_of(const int64_t *__restrict__ seg, int S, int64_t i, int64_t *lo,
                                          int64_t *hi) {
    int a = 0, b = S;  // invariant: seg[a] <= i < seg[b]
    while (b - a > 1) {
        const int c = (a + b) >> 1;
        if (seg[c] <= i)
            a = c;
        else
            b = c;
    }
    *lo = seg[a];
    *hi = seg[b];
}

// ids[i * P + t] = row i's neighbour t (slots 1..k-1 of idx), -1 in the
// padding up to P (a multiple of 16): every row starts a 64-byte line, so the
// mutual-edge lookup of a row reads whole lines.
__global__ __launch_bounds__(256) void k_pad_ids(const int32_t *__restrict__ idx, int64_t n, int k, int P,
                                                 int4 *__restrict__ ids) {
    const int m = k - 1, q = P / 4;
    const int64_t total = n * q;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = t / q;
        const int c = 4 * (int)(t - i * q);
        const int32_t *src = idx + i * k + 1;
        int4 v;
        v.x = c < m ? src[c] : -1;
        v.y = c + 1 < m ? src[c + 1] : -1;
        v.z = c + 2 < m ? src[c + 2] : -1;
        v.w = c + 3 < m ? src[c + 3] : -1;
        ids[t] = v;
    }
}

// Union weight of every directed edge, the rows' kept counts and the slots
// of the one-way edges among their targets' reverse entries.
//   wf[e]   float32 union weight (0: dropped, or a rejected edge);
//   rs[e]   slot among row j's reverse entries (kept one-way edge), -1 for a
//           mutual edge, -2 for a dropped or rejected one.
__global__ __launch_bounds__(kEdgeBlock) void k_union_probe(const int32_t *__restrict__ idx,
                                                            const int32_t *__restrict__ ids, int P,
                                                            const double *__restrict__ a, int64_t n, int k,
                                                            const int64_t *__restrict__ seg, int S,
                                                            float *__restrict__ wf, int32_t *__restrict__ rs,
                                                            int32_t *__restrict__ own,
                                                            int32_t *__restrict__ rev_cnt,
                                                            GraphResult *__restrict__ res) {
    const int lane = threadIdx.x & (kWave - 1);
    const EdgeMap mp(n, k - 1);
    const int m = mp.m;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    int err = 0;
    for (int64_t g = wave0; g < mp.groups; g += waves) {
        const int64_t i0 = g * mp.R;
        int own_acc = 0;
        const int chunks = mp.R > 1 ? 1 : (m + kWave - 1) / kWave;
        for (int c = 0; c < chunks; ++c) {
            int r, s;
            if (mp.R > 1) {
                r = lane / m;
                s = lane - r * m;
            } else {
                r = 0;
                s = c * kWave + lane;
            }
            const int64_t i = i0 + r;
            const bool act = (mp.R > 1 ? r < mp.R : s < m) && i < n;
            float f = 0.f;
            if (act) {
                const int64_t e = i * m + s;
                const int32_t j = idx[i * k + 1 + s];
                const double x = a[e];  // loaded beside j, not after the lookup
                bool ok = j >= 0 && j < n && j != i;
                if (ok && seg) {
                    int64_t lo, hi;
                    sample_of(seg, S, i, &lo, &hi);
                    if (j < lo || j >= hi) err |= 4, ok = false;
                } else if (!ok) {
                    err |= 1;
                }
                int32_t slot = -2;
                if (ok) {
                    // position of i in j's list: its padded copy, 16 ids
                    // (one 64-byte line) per load batch
                    const int4 *lj = reinterpret_cast<const int4 *>(ids + (int64_t)j * P);
                    int sp = -1;
                    for (int t0 = 0; t0 < m && sp < 0; t0 += 16) {
                        int4 v[4];
#pragma unroll
                        for (int u = 0; u < 4; ++u) v[u] = lj[t0 / 4 + u];
#pragma unroll
                        for (int u = 0; u < 4; ++u) {
                            if (sp < 0 && v[u].x == (int32_t)i) sp = t0 + 4 * u;
                            if (sp < 0 && v[u].y == (int32_t)i) sp = t0 + 4 * u + 1;
                            if (sp < 0 && v[u].z == (int32_t)i) sp = t0 + 4 * u + 2;
                            if (sp < 0 && v[u].w == (int32_t)i) sp = t0 + 4 * u + 3;
                        }
                    }
                    double w = x;
                    if (sp >= 0) {
                        const double y = a[(int64_t)j * m + sp];
                        w = __dsub_rn(__dadd_rn(x, y), __dmul_rn(x, y));
                    }
                    f = (float)w;
                    if (sp >= 0)
                        slot = -1;
                    else if (f != 0.f)
                        slot = atomicAdd(&rev_cnt[j], 1);
                }
                wf[e] = f;
                rs[e] = slot;
            }
            const uint64_t kept = __ballot(act && f != 0.f);
            if (mp.R > 1) {
                const uint64_t row_mask = ((1ull << m) - 1ull) << (r * m);
                if (act && s == 0) own[i] = __popcll(kept & row_mask);
            } else {
                own_acc += __popcll(kept);
            }
        }
        if (mp.R == 1 && lane == 0 && i0 < n) own[i0] = own_acc;
    }
    if (err) atomicOr(&res->error, err);
}

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v, int lane) {
    for (int o = 1; o < kWave; o <<= 1) {
        const int64_t u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// Block-local exclusive scans of the row lengths (own + reverse) into indptr
// and of the reverse counts into rbase; block totals of both into tot.
__global__ __launch_bounds__(kScanThreads) void k_scan_local(const int32_t *__restrict__ own,
                                                              const int32_t *__restrict__ rev, int64_t n,
                                                              int64_t *__restrict__ indptr,
                                                              int64_t *__restrict__ rbase,
                                                              int64_t *__restrict__ tot) {
    __shared__ int64_t wsum[2][kScanThreads / kWave];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)tid * kScanItems;
    int64_t v[kScanItems], q[kScanItems];
    int64_t tsum = 0, qsum = 0;
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = base + u;
        q[u] = i < n ? (int64_t)rev[i] : 0;
        v[u] = i < n ? (int64_t)own[i] + q[u] : 0;
        tsum += v[u];
        qsum += q[u];
    }
    const int64_t incl = wave_incl_scan(tsum, lane);
    const int64_t qincl = wave_incl_scan(qsum, lane);
    if (lane == kWave - 1) {
        wsum[0][wave] = incl;
        wsum[1][wave] = qincl;
    }
    __syncthreads();
    if (wave < 2) {
        int64_t s = lane < kScanThreads / kWave ? wsum[wave][lane] : 0;
        s = wave_incl_scan(s, lane);
        if (lane < kScanThreads / kWave) wsum[wave][lane] = s;
    }
    __syncthreads();
    int64_t run = incl - tsum + (wave > 0 ? wsum[0][wave - 1] : 0);
    int64_t qrun = qincl - qsum + (wave > 0 ? wsum[1][wave - 1] : 0);
#pragma unroll
    for (int u = 0; u < kScanItems; ++u) {
        const int64_t i = base + u;
        if (i < n) {
            indptr[i] = run;
            rbase[i] = qrun;
        }
        run += v[u];
        qrun += q[u];
    }
    if (tid == kScanThreads - 1) {
        tot[2 * blockIdx.x] = run;
        tot[2 * blockIdx.x + 1] = qrun;
    }
}

// Exclusive scan of the block totals (one workgroup, chunked; pairs); writes nnz.
__global__ __launch_bounds__(kScanThreads) void k_scan_totals(int64_t *__restrict__ tot, int64_t nb,
                                                               GraphResult *__restrict__ res) {
    __shared__ int64_t wsum[kScanThreads / kWave];
    __shared__ int64_t carry;
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    for (int part = 0; part < 2; ++part) {
        if (tid == 0) carry = 0;
        __syncthreads();
        for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
            const int64_t i = c0 + tid;
            const int64_t x = i < nb ? tot[2 * i + part] : 0;
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
            if (i < nb) tot[2 * i + part] = excl;
            __syncthreads();
            if (tid == kScanThreads - 1) carry = excl + x;
            __syncthreads();
        }
        if (tid == 0 && part == 0) res->nnz = carry;
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t *__restrict__ indptr, int64_t *__restrict__ rbase,
                                                  int64_t n, const int64_t *__restrict__ tot,
                                                  const GraphResult *__restrict__ res) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int64_t b = i / kScanTile;
        indptr[i] += tot[2 * b];
        rbase[i] += tot[2 * b + 1];
    }
    if (i == n) indptr[n] = res->nnz;
}

// Each kept one-way edge i -> j writes (i, w) into its slot of j's reverse entries.
__global__ __launch_bounds__(kEdgeBlock) void k_rev_fill(const int32_t *__restrict__ idx, int64_t n, int k,
                                                         const float *__restrict__ wf,
                                                         const int32_t *__restrict__ rs,
                                                         const int64_t *__restrict__ rbase,
                                                         int2 *__restrict__ rev) {
    const int lane = threadIdx.x & (kWave - 1);
    const EdgeMap mp(n, k - 1);
    const int m = mp.m;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    for (int64_t g = wave0; g < mp.groups; g += waves) {
        const int64_t i0 = g * mp.R;
        const int chunks = mp.R > 1 ? 1 : (m + kWave - 1) / kWave;
        for (int c = 0; c < chunks; ++c) {
            int r, s;
            if (mp.R > 1) {
                r = lane / m;
                s = lane - r * m;
            } else {
                r = 0;
                s = c * kWave + lane;
            }
            const int64_t i = i0 + r;
            if (!((mp.R > 1 ? r < mp.R : s < m) && i < n)) continue;
            const int64_t e = i * m + s;
            // the edge's three loads are independent: issue them together
            const int32_t slot = rs[e];
            const int32_t j = idx[i * k + 1 + s];
            const float f = wf[e];
            if (slot < 0) continue;
            rev[rbase[j] + slot] = make_int2((int32_t)i, __float_as_int(f));
        }
    }
}

// Entry p of row i's unsorted list: its own slots first (dropped ones as
// column INT_MAX), then its reverse entries.
__device__ __forceinline__ void row_entry(const int32_t *__restrict__ idx, const float *__restrict__ wf,
                                          const int2 *__restrict__ rev, int64_t i, int k, int m, int64_t rb,
                                          int64_t p, int32_t *col, float *val) {
    if (p < m) {
        // both loads unconditional, so that they are in flight together
        const float f = wf[i * m + p];
        const int32_t c = idx[i * k + 1 + p];
        *val = f;
        *col = f != 0.f ? c : INT_MAX;
    } else {
        const int2 t = rev[rb + (p - m)];
        *col = t.x;
        *val = __int_as_float(t.y);
    }
}

__device__ __forceinline__ int64_t lane_i64(int64_t x, int src) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)x, src);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)((uint64_t)x >> 32), src);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Ascending sort of (col, val) by col over segments of W lanes (W = 32: each
// half of the wave sorts its own row; W = 64: the whole wave one row); x is
// the lane's index within its segment.  A bitonic network: log2(W) merge
// stages, each a compare-exchange with the lane x ^ j.
template <int W>
__device__ __forceinline__ void bitonic_sort(int32_t &col, float &val, int x) {
#pragma unroll
    for (int kk = 2; kk <= W; kk <<= 1) {
#pragma unroll
        for (int j = kk >> 1; j > 0; j >>= 1) {
            const int32_t oc = __shfl_xor(col, j, kWave);
            const float ov = __shfl_xor(val, j, kWave);
            const bool ascending = (x & kk) == 0;
            const bool lower = (x & j) == 0;
            if (ascending == lower ? oc < col : oc > col) {
                col = oc;
                val = ov;
            }
        }
    }
}

// Row i's entries sorted by column and written from out0 on; repeated
// columns set dup.
// Rows of up to kSortCap entries that do not fit a wave are sorted in LDS:
// their (column, weight) pairs are staged, padded with column INT_MAX to a
// power of two, and sorted by a bitonic network whose compare-exchanges the
// wave's lanes share, stage by stage.
constexpr int kSortCap = 1024;

__device__ __forceinline__ void sort_row_wave(const int32_t *__restrict__ idx, const float *__restrict__ wf,
                                              const int2 *__restrict__ rev, int64_t i, int k, int m, int64_t rb,
                                              int64_t len, int64_t out0, int32_t *__restrict__ indices,
                                              float *__restrict__ data, bool &dup) {
    const int lane = threadIdx.x & (kWave - 1);
    if (len <= kWave) {
        int32_t col = INT_MAX;
        float val = 0.f;
        if (lane < len) row_entry(idx, wf, rev, i, k, m, rb, lane, &col, &val);
        bitonic_sort<kWave>(col, val, lane);
        const int32_t next = __shfl_down(col, 1, kWave);
        if (col != INT_MAX) {
            dup |= lane < kWave - 1 && next == col;
            indices[out0 + lane] = col;
            data[out0 + lane] = val;
        }
        return;
    }
    // rows longer than kSortCap: rank every entry by lane broadcasts of 64-entry chunks
    for (int64_t e0 = 0; e0 < len; e0 += kWave) {
        const int64_t e = e0 + lane;
        int32_t col = INT_MAX;
        float val = 0.f;
        if (e < len) row_entry(idx, wf, rev, i, k, m, rb, e, &col, &val);
        int64_t rank = 0;
        for (int64_t c0 = 0; c0 < len; c0 += kWave) {
            int32_t oc = INT_MAX;
            float ov;
            if (c0 + lane < len) row_entry(idx, wf, rev, i, k, m, rb, c0 + lane, &oc, &ov);
            const int lim = (int)((len - c0) < kWave ? (len - c0) : kWave);
            for (int t = 0; t < lim; ++t) {
                const int32_t x = __builtin_amdgcn_readlane(oc, t);
                rank += x < col;
                dup |= x == col && c0 + t != e && col != INT_MAX;
            }
        }
        if (col != INT_MAX) {
            indices[out0 + rank] = col;
            data[out0 + rank] = val;
        }
    }
}

// Rows in pairs, one pair per wave: when both rows have at most 32 entries
// each half of the wave sorts one of them; otherwise the wave takes the two
// rows one after the other.  Dropped own slots carry column INT_MAX and sort
// behind the kept entries, which land at out0 + their sorted position.
__global__ __launch_bounds__(256) void k_row_sort(const int32_t *__restrict__ idx, const float *__restrict__ wf,
                                                  const int2 *__restrict__ rev, const int32_t *__restrict__ rev_cnt,
                                                  const int64_t *__restrict__ rbase,
                                                  const int64_t *__restrict__ indptr, int64_t n, int k,
                                                  int32_t *__restrict__ indices, float *__restrict__ data,
                                                  int32_t *__restrict__ long_list, GraphResult *__restrict__ res) {
    const int lane = threadIdx.x & (kWave - 1);
    const int half = lane >> 5, sub = lane & 31;
    const int m = k - 1;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    bool dup = false;
    // the next pair's row figures are loaded one iteration ahead
    int64_t len_n = 0, rb_n = 0, out_n = 0;
    auto fetch = [&](int64_t g) {
        const int64_t r = 2 * g + half;
        const bool ok = 2 * g < n && r < n;
        len_n = ok ? (int64_t)m + rev_cnt[r] : 0;
        rb_n = ok ? rbase[r] : 0;
        out_n = ok ? indptr[r] : 0;
    };
    fetch(wave0);
    for (int64_t g = wave0; 2 * g < n; g += waves) {
        const int64_t mine = 2 * g + half;
        const int64_t len = len_n, rb = rb_n, out0 = out_n;
        fetch(g + waves);
        if (__ballot(len > 32) == 0ull) {
            int32_t col = INT_MAX;
            float val = 0.f;
            if (sub < len) row_entry(idx, wf, rev, mine, k, m, rb, sub, &col, &val);
            bitonic_sort<32>(col, val, sub);
            const int32_t next = __shfl_down(col, 1, 32);
            if (col != INT_MAX) {
                dup |= sub < 31 && next == col;
                indices[out0 + sub] = col;
                data[out0 + sub] = val;
            }
            continue;
        }
        for (int r = 0; r < 2; ++r) {
            const int64_t i = 2 * g + r;
            if (i >= n) break;
            const int src = 32 * r;  // lane 0 holds row 2g's figures, lane 32 row 2g + 1's
            const int64_t li = lane_i64(len, src), ri = lane_i64(rb, src), oi = lane_i64(out0, src);
            if (li > kWave) {
                if (lane == 0) long_list[atomicAdd(&res->long_rows, 1)] = (int32_t)i;
                continue;
            }
            sort_row_wave(idx, wf, rev, i, k, m, ri, li, oi, indices, data, dup);
        }
    }
    if (dup) atomicOr(&res->error, 2);
}

// The rows listed by k_row_sort (more than 64 entries), one wave each:
// sorted in LDS when they hold at most kSortCap entries, else ranked by
// lane broadcasts.
__global__ __launch_bounds__(256) void k_row_sort_long(const int32_t *__restrict__ idx, const float *__restrict__ wf,
                                                       const int2 *__restrict__ rev,
                                                       const int32_t *__restrict__ rev_cnt,
                                                       const int64_t *__restrict__ rbase,
                                                       const int64_t *__restrict__ indptr, int k,
                                                       const int32_t *__restrict__ long_list,
                                                       int32_t *__restrict__ indices, float *__restrict__ data,
                                                       GraphResult *__restrict__ res) {
    __shared__ int32_t stage_col[256 / kWave][kSortCap];
    __shared__ float stage_val[256 / kWave][kSortCap];
    int32_t *lds_col = stage_col[threadIdx.x / kWave];
    float *lds_val = stage_val[threadIdx.x / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int m = k - 1;
    const int64_t wave0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t waves = ((int64_t)gridDim.x * blockDim.x) / kWave;
    const int64_t count = res->long_rows;
    bool dup = false;
    for (int64_t t0 = wave0; t0 < count; t0 += waves) {
        const int64_t i = long_list[t0];
        const int64_t len = (int64_t)m + rev_cnt[i], rb = rbase[i], out0 = indptr[i];
        if (len <= kSortCap) {
            const int n_ = (int)len;
            int P2 = 2 * kWave;
            while (P2 < n_) P2 <<= 1;
            for (int e = lane; e < P2; e += kWave) {
                int32_t c = INT_MAX;
                float v = 0.f;
                if (e < n_) row_entry(idx, wf, rev, i, k, m, rb, e, &c, &v);
                lds_col[e] = c;
                lds_val[e] = v;
            }
            for (int kk = 2; kk <= P2; kk <<= 1) {
                for (int j = kk >> 1; j > 0; j >>= 1) {
                    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
                    __builtin_amdgcn_wave_barrier();
                    for (int t = lane; t < P2 / 2; t += kWave) {
                        const int i0 = ((t & ~(j - 1)) << 1) | (t & (j - 1)), i1 = i0 + j;
                        const int32_t c0 = lds_col[i0], c1 = lds_col[i1];
                        if ((i0 & kk) == 0 ? c0 > c1 : c0 < c1) {
                            const float v0 = lds_val[i0], v1 = lds_val[i1];
                            lds_col[i0] = c1;
                            lds_col[i1] = c0;
                            lds_val[i0] = v1;
                            lds_val[i1] = v0;
                        }
                    }
                }
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
            __builtin_amdgcn_wave_barrier();
            for (int e = lane; e < n_; e += kWave) {
                const int32_t c = lds_col[e];
                if (c == INT_MAX) continue;
                dup |= e + 1 < n_ && lds_col[e + 1] == c;
                indices[out0 + e] = c;
                data[out0 + e] = lds_val[e];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // read out before the wave's next row
            __builtin_amdgcn_wave_barrier();
            continue;
        }
        sort_row_wave(idx, wf, rev, i, k, m, rb, len, out0, indices, data, dup);
    }
    if (dup) atomicOr(&res->error, 2);
}

struct GraphWs {
    GraphResult *res;
    double *a;
    float *wf;
    int32_t *rs;
    int32_t *own, *rev_cnt;
    int64_t *rbase;
    int64_t *tot;
    int64_t *seg;
    int2 *rev;
    int32_t *ids;  // padded neighbour lists, n x pad_ids(k) (64-byte aligned)
};

int pad_ids(int k) { return ((k - 1 + 15) / 16) * 16; }

size_t carve_graph(int64_t n, int k, int32_t S, void *base, GraphWs *w) {
    Carver cv(base);
    const size_t ne = (size_t)n * (size_t)(k - 1);
    const size_t nb = (size_t)((n + kScanTile - 1) / kScanTile) + 1;
    GraphWs g;
    g.res = cv.take<GraphResult>(1);
    g.a = cv.take<double>(ne ? ne : 1);
    g.wf = cv.take<float>(ne ? ne : 1);
    g.rs = cv.take<int32_t>(ne ? ne : 1);
    g.own = cv.take<int32_t>((size_t)n + 1);
    g.rev_cnt = cv.take<int32_t>((size_t)n + 1);
    g.rbase = cv.take<int64_t>((size_t)n + 1);
    g.tot = cv.take<int64_t>(2 * nb);
    g.seg = S > 0 ? cv.take<int64_t>((size_t)S + 1) : nullptr;
    g.rev = cv.take<int2>(ne ? ne : 1);
    g.ids = cv.take<int32_t>(ne ? (size_t)n * (size_t)pad_ids(k) : 1);
    if (w) *w = g;
    return cv.used;
}

unsigned grid_for(int64_t n, int per_block) { return (unsigned)((n + per_block - 1) / per_block); }

// Blocks of the per-edge and per-row wave loops: enough waves to fill the
// chip several times over, no more than the work needs.
unsigned wave_grid(int64_t wave_items) {
    const int64_t blocks = (wave_items + kEdgeBlock / kWave - 1) / (kEdgeBlock / kWave);
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(blocks, 256 * 64));
}

int graph_run_impl(const int32_t *idx, const float *dist, int64_t n, int k, const int64_t *seg_host, int32_t S,
                   int64_t *indptr, int32_t *indices, float *data, int64_t *nnz, double *rho, double *sigma,
                   void *ws, hipStream_t stream) {
    GraphWs w;
    carve_graph(n, k, S, ws, &w);
    int st;
    const int m = k - 1;
    {
        ScopedTimer t("graph_init", stream);
        hipLaunchKernelGGL(k_init_result, dim3(1), dim3(64), 0, stream, w.res);
        const unsigned g = std::min<unsigned>(grid_for(n + 1, 256), 4096u);
        hipLaunchKernelGGL(k_fill_i32, dim3(g), dim3(256), 0, stream, w.rev_cnt, n + 1, 0);
        if (w.seg) {
            st = hip_status(hipMemcpyAsync(w.seg, seg_host, sizeof(int64_t) * ((size_t)S + 1), hipMemcpyHostToDevice,
                                           stream),
                            "upload sample offsets");
            if (st != RSC_OK) return st;
        }
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
    const int R = m >= 1 && m <= 32 ? kWave / m : 1;
    const int64_t groups = (n + R - 1) / R;
    {
        ScopedTimer t("union_count", stream);
        if (m > 0) {
            const int P = pad_ids(k);
            hipLaunchKernelGGL(k_pad_ids, dim3((unsigned)std::min<int64_t>(grid_for(n * (P / 4), 256), 65536)),
                               dim3(256), 0, stream, idx, n, k, P, reinterpret_cast<int4 *>(w.ids));
            hipLaunchKernelGGL(k_union_probe, dim3(wave_grid(groups)), dim3(kEdgeBlock), 0, stream, idx, w.ids, P,
                               w.a, n, k, w.seg, S, w.wf, w.rs, w.own, w.rev_cnt, w.res);
        } else
            hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, stream, w.own, n, 0);
        if ((st = launch_status("union_count")) != RSC_OK) return st;
    }
    {
        ScopedTimer t("csr_scan", stream);
        const int64_t nb = (n + kScanTile - 1) / kScanTile;
        hipLaunchKernelGGL(k_scan_local, dim3((unsigned)std::max<int64_t>(nb, 1)), dim3(kScanThreads), 0, stream,
                           w.own, w.rev_cnt, n, indptr, w.rbase, w.tot);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, stream, w.tot, std::max<int64_t>(nb, 1),
                           w.res);
        hipLaunchKernelGGL(k_scan_add, dim3(grid_for(n + 1, 256)), dim3(256), 0, stream, indptr, w.rbase, n, w.tot,
                           w.res);
        if ((st = launch_status("csr_scan")) != RSC_OK) return st;
    }
    if (m > 0) {
        ScopedTimer t("union_fill", stream);
        hipLaunchKernelGGL(k_rev_fill, dim3(wave_grid(groups)), dim3(kEdgeBlock), 0, stream, idx, n, k, w.wf, w.rs,
                           w.rbase, w.rev);
        if ((st = launch_status("union_fill")) != RSC_OK) return st;
    }
    if (m > 0) {
        ScopedTimer t("row_sort", stream);
        // own (the kept counts) is spent once the scan has run: it holds the long-row list
        hipLaunchKernelGGL(k_row_sort, dim3(wave_grid((n + 1) / 2)), dim3(256), 0, stream, idx, w.wf, w.rev, w.rev_cnt,
                           w.rbase, indptr, n, k, indices, data, w.own, w.res);
        hipLaunchKernelGGL(k_row_sort_long, dim3((unsigned)std::min<int64_t>(1024, (n + 255) / 256)), dim3(256), 0,
                           stream, idx, w.wf, w.rev, w.rev_cnt, w.rbase, indptr, k, w.own, indices, data, w.res);
        if ((st = launch_status("row_sort")) != RSC_OK) return st;
    }
    GraphResult host;
    if ((st = hip_status(hipMemcpyAsync(&host, w.res, sizeof(host), hipMemcpyDeviceToHost, stream), "read nnz")) !=
        RSC_OK)
        return st;
    if ((st = hip_status(hipStreamSynchronize(stream), "synchronise")) != RSC_OK) return st;
    *nnz = host.nnz;
    if (host.error) {
        set_error(host.error & 1   ? "kNN lists hold an index out of range or the row itself in columns 1..k-1"
                  : host.error & 4 ? "kNN lists hold an edge to a row of another sample"
                                   : "kNN lists repeat a neighbour within a row");
        return RSC_ERR_BAD_GRAPH;
    }
    return RSC_OK;
}

// Scratch of the allocation-free entry point: a file-scope device array
// that every GPU the library runs on holds until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in for the symbol); it uses the device address looked up once per
// device below.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array, looked up on the first
// call made with the device current.
int scratch_address(void **out) {
    int dev = -1;
    int st = hip_status(hipGetDevice(&dev), "current device");
    if (st != RSC_OK) return st;
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device ordinal beyond the scratch table");
        return RSC_ERR_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        st = hip_status(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "scratch symbol address");
        if (st != RSC_OK) return st;
        if (!p) {
            set_error("scratch symbol address: null");
            return RSC_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return RSC_OK;
}

}  // namespace

size_t graph_workspace_bytes(int64_t n, int k, int32_t S) { return carve_graph(n, k, S, nullptr, nullptr); }

size_t graph_noalloc_max_bytes() { return kNoAllocScratchBytes; }

int graph_run_noalloc(const int32_t *idx, const float *dist, int64_t n, int k, int64_t *indptr, int32_t *indices,
                      float *data, int64_t *nnz, double *rho, double *sigma, hipStream_t stream) {
    const size_t need = graph_workspace_bytes(n, k);
    if (need > kNoAllocScratchBytes) {
        set_error("allocation-free connectivities: n = " + std::to_string(n) + ", k = " + std::to_string(k) +
                  " need " + std::to_string(need) + " bytes of scratch, above the fixed " +
                  std::to_string(kNoAllocScratchBytes));
        return RSC_ERR_CAPACITY;
    }
    void *ws = nullptr;
    const int st = scratch_address(&ws);
    if (st != RSC_OK) return st;
    return graph_run_impl(idx, dist, n, k, nullptr, 0, indptr, indices, data, nnz, rho, sigma, ws, stream);
}

int graph_run(const int32_t *idx, const float *dist, int64_t n, int k, int64_t *indptr, int32_t *indices,
              float *data, int64_t *nnz, double *rho, double *sigma, void *ws, hipStream_t stream) {
    return graph_run_impl(idx, dist, n, k, nullptr, 0, indptr, indices, data, nnz, rho, sigma, ws, stream);
}

int graph_run_batched(const int32_t *idx, const float *dist, int64_t n, int k, const int64_t *seg_host, int32_t S,
                      int64_t *indptr, int32_t *indices, float *data, int64_t *nnz, void *ws, hipStream_t stream) {
    return graph_run_impl(idx, dist, n, k, seg_host, S, indptr, indices, data, nnz, nullptr, nullptr, ws, stream);
}

}  // namespace rsc
