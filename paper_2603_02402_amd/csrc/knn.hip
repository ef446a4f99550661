// Exact kNN on gfx950: MFMA distance screen + float64 rerank + certificate.
//
// The paper's neighbour step needs, per cell, the k nearest cells of the
// PCA embedding under the squared Euclidean distance of Methods, "Custom
// GPU kernels" (d_ij = ||x_i - x_j||^2).  The work is a dense contraction
// (2 d flops per ordered pair), so the screen runs on the matrix cores:
//
//   key_ij = ||y_j||^2 - 2 x_i . y_j      (= d_ij - ||x_i||^2, same order per row)
//
// Data path of the screen (one wave = 32 queries, one workgroup = 4 waves):
//   * the query operand (-2 x) stays in VGPRs for the whole launch;
//   * references are repacked once into the MFMA A-operand order (one
//     float4 per lane per four contraction steps, 1 KiB per wave load, fully
//     coalesced) and streamed HBM/MALL/L2 -> VGPR, each float4 of the next
//     block loaded as soon as the current one has been consumed; no LDS and
//     no workgroup barrier;
//   * when the half-width leaves a spare contraction slot, ||y||^2 rides in
//     it (times 1 on the query side), so the MFMA chain produces the key;
//     otherwise the norm is added in the epilogue;
//   * each lane keeps, in registers, the sorted 16 (or 32) smallest keys of
//     the references its contraction half sees (every other group of four
//     rows); a key below the lane's current 16th enters by an unrolled
//     compare-and-shift, so the common case costs one compare per pair.
// A launch may split the references into P ranges (blockIdx.y) to give
// small problems enough workgroups; each range keeps its own heap.
//
// The float32 screen is not the answer.  Its rounding error is bounded per
// query, every candidate is re-ranked with float64 distances summed from
// direct differences in dimension order, and a row is certified exact when
// its m-th re-ranked distance is below the smallest key any range could
// have rejected, minus the bound.  Rows that fail go through a second,
// wider screen over many reference ranges (escalation) and, if they fail
// again, an exhaustive float64 scan.  Ties are broken towards the lower
// index throughout.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <climits>
#include <cmath>

#include "rsc_internal.hpp"
#include "screen_common.hpp"
#include "screen_fp32.hpp"

namespace rsc {

namespace {

using namespace scr;

constexpr int kMaxD = 256;       // exact FP32 path (reduced-precision screens: 128)
constexpr int kMaxK = 255;       // exact FP32 path (reduced-precision screens: 63)
constexpr int kMaxDLowp = 128;
constexpr int kMaxKLowp = 63;
constexpr int kEscalateCap = 8192;  // rows handled by the escalation screen
constexpr int kEscalateSplits = 16;
constexpr int kEscalateWidth = 64;

// Squared norms of the reference rows (float64 sum, rounded once) and the
// largest norm.  One wave per block of norm_rows(d) rows (64 for d <= 128):
// the rows (contiguous in memory) are copied into LDS with coalesced loads,
// then lane i sums row i.
constexpr int kNormRows = 64;
constexpr int kNormBuf = kNormRows * 128;  // floats staged per block
__host__ __device__ inline int norm_rows(int d) { return d <= 128 ? kNormRows : kNormBuf / d; }

__global__ __launch_bounds__(64) void k_norms(const float *__restrict__ R, int64_t nr, int d,
                                              float *__restrict__ nrow, uint32_t *__restrict__ max_norm_bits) {
    __shared__ float buf[kNormBuf];
    const int lane = threadIdx.x;
    const int nrb = norm_rows(d);
    const int64_t r0 = (int64_t)blockIdx.x * nrb;
    const int rows = (int)min<int64_t>(nrb, nr - r0);
    const float *src = R + r0 * d;
    for (int e = lane; e < rows * d; e += kWave) buf[e] = src[e];
    __syncthreads();
    float nf = 0.f;
    if (lane < rows) {
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
            const double x = (double)buf[lane * d + t];
            s += x * x;
        }
        nf = (float)s;
        nrow[r0 + lane] = nf;
    }
    const float m = wave_max(sqrtf(nf));
    if (lane == 0) atomicMax(max_norm_bits, __float_as_uint(m));
}

// Unit-normalised rows for the cosine screen: x / ||x|| with the norm summed
// in float64 and rounded once to float32, then one float32 division per
// element (each element within 2 units of roundoff of x_t / ||x||); a row of
// zero norm stays zero.  One wave per 64 rows, staged through LDS so that the
// loads and stores are coalesced.
__global__ __launch_bounds__(64) void k_normalize(const float *__restrict__ X, int64_t n, int d,
                                                  float *__restrict__ out) {
    __shared__ float buf[kNormBuf];
    const int lane = threadIdx.x;
    const int nrb = norm_rows(d);
    const int64_t r0 = (int64_t)blockIdx.x * nrb;
    const int rows = (int)min<int64_t>(nrb, n - r0);
    for (int e = lane; e < rows * d; e += kWave) buf[e] = X[r0 * d + e];
    __syncthreads();
    if (lane < rows) {
        double s = 0.0;
        for (int t = 0; t < d; ++t) {
            const double x = (double)buf[lane * d + t];
            s += x * x;
        }
        const float nrm = (float)sqrt(s);
        for (int t = 0; t < d; ++t) buf[lane * d + t] = nrm > 0.f ? buf[lane * d + t] / nrm : 0.f;
    }
    __syncthreads();
    for (int e = lane; e < rows * d; e += kWave) out[r0 * d + e] = buf[e];
}

// Packed reference layout for a contraction half-width DH.  Block b holds
// rows 32b..32b+31:
//   A[b][s4][lane] (float4): element u = step s = 4 s4 + u of lane (c, h).
//       With the norm folded, step 0 of half 0 is ||R[32b + c]||^2 (+inf
//       past the end; half 1 holds 0) and step 1 + t is R[32b + c][h DH + t];
//       otherwise step t is R[32b + c][h DH + t].  0 elsewhere.  Putting the
//       norm first keeps the partial sums of the key near its final size;
//   N[b][h][4g + j] (only when not folded): ||R[32b + 8g + 4h + j]||^2, the
//       accumulator order of the 32x32 output block (+inf past the end);
// so that MFMA step s of a wave reads 1 KiB of lane-contiguous data.
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ R, const float *__restrict__ nrow, int64_t nr,
                                              int d, int DH, int S4, int folded, int64_t nblk,
                                              f32x4 *__restrict__ Ap, float *__restrict__ Np,
                                              const int32_t *__restrict__ blk_sample, const int64_t *__restrict__ boff,
                                              const int64_t *__restrict__ soff, const int32_t *__restrict__ row_map) {
    const int64_t total = nblk * S4 * kWave;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(e % kWave);
        const int64_t bs = e / kWave;
        const int s4 = (int)(bs % S4);
        const int64_t b = bs / S4;
        // row of lane (c, h); batched: blocks of sample s start at boff[s] and
        // hold rows soff[s]..soff[s+1]-1 (the last block of a sample is padded)
        // routed form: packed row 32b + c holds row_map[32b + c] (-1: padding)
        int64_t row = 32 * b + (lane & 31), row_end = nr;
        if (blk_sample) {
            const int smp = blk_sample[b];
            row = soff[smp] + 32 * (b - boff[smp]) + (lane & 31);
            row_end = soff[smp + 1];
        }
        bool live = row < row_end;
        if (row_map) {
            row = row_map[32 * b + (lane & 31)];
            live = row >= 0;
        }
        const int h = lane >> 5;
        f32x4 v;
        const int off = folded ? 1 : 0;  // the norm occupies step 0 when folded
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = 4 * s4 + u;
            const int sd = s - off;        // dimension step
            const int t = h * DH + sd;
            float x = 0.f;
            if (folded && s == 0) {
                if (h == 0) x = live ? nrow[row] : INFINITY;
            } else if (sd < DH) {
                if (live && t < d) x = R[row * d + t];
            }
            v[u] = x;
        }
        Ap[e] = v;
        if (!folded && s4 == 0) {
            // lane (c, h) of block b also files the norm of row 32b + c into accumulator order
            if (h == 0) {
                const int i = lane & 31;
                const int g = i >> 3, hh = (i >> 2) & 1, j = i & 3;
                Np[b * 32 + hh * 16 + 4 * g + j] = live ? nrow[row] : INFINITY;
            }
        }
    }
}

__global__ void k_set_i32(int32_t *p, int32_t v) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = v;
}

__global__ void k_init_counters(KnnCounters *c) {
    if (threadIdx.x == 0) {
        c->flagged = 0;
        c->max_ratio_bits = 0u;
        c->max_norm_bits = 0u;
        c->flagged2 = 0;
        c->rescanned = 0;
    }
}

// ---------------------------------------------------------------------------
// Screen.
//
// Lane l handles query c = l % 32 of its wave and contraction half
// h = l / 32: a step of the MFMA chain multiplies dimension h*DH + t (plus
// the norm step, first, when folded).
// Output register v of the 32x32 block holds reference row 8(v/4) + 4h +
// (v%4), so each lane sees half of the references of every block and keeps
// its own sorted list of the L smallest keys of that half.
// Query slot i of the launch is row i, or row qlist[i] for i < min(*qcount,
// qcap) when a list is given (the escalation pass).
// Output: cand[(slot * 2P + 2p + h) * L + i], i-th smallest key of half h
// of range p (index -1 / key +inf where fewer than L were seen).
// ---------------------------------------------------------------------------
template <int DH, int L, int W>
__global__ __launch_bounds__(256, W) void k_screen_fp32(ScreenArgs a) {
    // Per-lane queue of keys that beat the lane's threshold (see LaneTopK).
    __shared__ float2 qbuf[kQueueCap * 256];
    constexpr int QG = kScreenWaves * 32;
    const int tid = threadIdx.x;
    const int wave = tid >> 6, c = tid & 31;
    const int p = blockIdx.y;
    const int64_t blk_per = (a.nblk + a.P - 1) / a.P;
    const int64_t blk0 = (int64_t)p * blk_per;
    const int64_t blk1 = std::min<int64_t>(a.nblk, blk0 + blk_per);
    const int64_t nslots = screen_slots(a);
    for (int64_t qblk = blockIdx.x; qblk * QG < nslots; qblk += gridDim.x) {
        const int64_t slot = qblk * QG + wave * 32 + c;
        int64_t row = -1;
        if (slot < nslots) row = a.qlist ? (int64_t)a.qlist[slot] : slot;
        screen_fp32_tile<DH, L>(a, slot < nslots ? slot : -1, row, blk0, blk1, p, 0, qbuf);
    }
}

// ---------------------------------------------------------------------------
// Rerank + certificate: one wave per query slot.  Candidates of all P ranges
// are streamed 64 at a time; the m best (d2, j) are kept sorted across the
// lanes (lane i = i-th smallest) by bitonic sort + merge.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void bitonic_sort64(double &d2, int &jj, int lane) {
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const double od = __shfl_xor(d2, stride, kWave);
            const int oj = __shfl_xor(jj, stride, kWave);
            const bool want_min = ((lane & stride) == 0) == ((lane & size) == 0);
            const bool other_first = lex_before(od, oj, d2, jj);
            if (want_min == other_first) {
                d2 = od;
                jj = oj;
            }
        }
    }
}

// Sort a bitonic 64-sequence (d2, jj) ascending in (d, j) order.
__device__ __forceinline__ void bitonic_clean64(double &d2, int &jj, int lane) {
#pragma unroll
    for (int stride = kWave >> 1; stride > 0; stride >>= 1) {
        const double xd = __shfl_xor(d2, stride, kWave);
        const int xj = __shfl_xor(jj, stride, kWave);
        const bool lower = (lane & stride) == 0;
        const bool other_first = lex_before(xd, xj, d2, jj);
        if (lower == other_first) {
            d2 = xd;
            jj = xj;
        }
    }
}

// The m smallest (d, j) seen so far, m <= 64 R, sorted across the wave:
// position p = 64 r + lane lives in register r of that lane (+inf / INT_MAX
// where fewer were seen).  A sorted 64-chunk is merged register by register:
// the 64 smallest of (register r, carry) stay in r, the rest carry on.
template <int R>
struct TopM {
    double d[R];
    int j[R];

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            d[r] = INFINITY;
            j[r] = INT_MAX;
        }
    }
    // (d, j) at position p (p wave-uniform)
    __device__ __forceinline__ void at(int p, double &pd, int &pj) const {
        double rd = d[0];
        int rj = j[0];
#pragma unroll
        for (int r = 1; r < R; ++r)
            if (p >> 6 == r) {
                rd = d[r];
                rj = j[r];
            }
        pd = __shfl(rd, p & (kWave - 1), kWave);
        pj = __shfl(rj, p & (kWave - 1), kWave);
    }
    // merge a sorted chunk (cd, cj), lane i = i-th smallest
    __device__ __forceinline__ void merge(double cd, int cj, int lane) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const double od = __shfl(cd, kWave - 1 - lane, kWave);
            const int oj = __shfl(cj, kWave - 1 - lane, kWave);
            const bool take = lex_before(od, oj, d[r], j[r]);
            const double hd = take ? d[r] : od;
            const int hj = take ? j[r] : oj;
            if (take) {
                d[r] = od;
                j[r] = oj;
            }
            bitonic_clean64(d[r], j[r], lane);
            if (r + 1 < R) {
                cd = hd;
                cj = hj;
                if (__ballot(cd < INFINITY) == 0ull) break;  // nothing left to carry
                bitonic_clean64(cd, cj, lane);
            }
        }
    }
};

// Candidate rows are staged through LDS 32 dimensions at a time: for each
// batch of 64 candidates (one per lane) the wave copies the rows' chunk with
// coalesced loads (two 128-byte row segments per instruction), then every
// lane continues its own float64 sum in dimension order from LDS, so the
// distances are those of exact_d2 bit for bit.
constexpr int kRerankChunk = 32;

template <int R>
__global__ __launch_bounds__(256) void k_rerank(RerankArgs a) {
    __shared__ float tile[4][kWave][kRerankChunk + 1];
    __shared__ float qrow[4][kMaxD];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x >> 6;
    const int64_t slot = (int64_t)blockIdx.x * (blockDim.x / kWave) + wave;
    int64_t nslots = a.nq;
    if (a.qlist) nslots = std::min<int64_t>(std::min<int64_t>(*a.qcount, a.qcap), a.nq);
    if (slot >= nslots) return;
    const int64_t row = a.qlist ? (int64_t)a.qlist[slot] : slot;
    const float *x = a.Q + row * a.d;
    float(*T)[kRerankChunk + 1] = tile[wave];
    float *xs = qrow[wave];
    for (int t = lane; t < a.d; t += kWave) xs[t] = x[t];

    // ||x||^2 in float64 (only feeds the certificate's margin)
    double xx = 0.0;
    for (int t = lane; t < a.d; t += kWave) xx += (double)x[t] * (double)x[t];
    xx = wave_sum(xx);
    const double xn = sqrt(xx) * (1.0 + 1e-12);
    const double ymax = (double)__uint_as_float(a.counters->max_norm_bits) * (1.0 + 1e-6);
    const bool cosine = a.metric == RSC_COSINE;
    // cosine: the query's squared norm summed in dimension order (as every
    // pair's distance below and the oracle compute it)
    double cxx = 0.0;
    if (cosine) {
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
        __builtin_amdgcn_wave_barrier();
        for (int t = 0; t < a.d; ++t) {
            const double v = (double)xs[t];
            cxx = __dadd_rn(cxx, __dmul_rn(v, v));
        }
    }

    // Smallest key any full range could have rejected.
    float tau = INFINITY;
    const int64_t cbase = slot * a.P * a.KP;
    for (int p = 0; p < a.P; ++p) {
        int j = -1;
        float key = -INFINITY;
        if (lane < a.S) {
            j = a.cand_idx[cbase + p * a.KP + lane];
            key = a.cand_key[cbase + p * a.KP + lane];
        }
        const bool full = __ballot(lane < a.S && j < 0) == 0ull;
        const float root = wave_max(key);
        if (full) tau = fminf(tau, root);
    }

    TopM<R> top;
    top.init();
    float ratio = 0.f;
    const int total = a.P * a.S;
    for (int c0 = 0; c0 < total; c0 += kWave) {
        const int ci = c0 + lane;
        int j = -1;
        float key = 0.f;
        if (ci < total) {
            const int p = ci / a.S, e = ci - (ci / a.S) * a.S;
            j = a.cand_idx[cbase + p * a.KP + e];
            key = a.cand_key[cbase + p * a.KP + e];
        }
        const bool valid = j >= 0 && !(a.self_mode && j == row);
        const int jl = valid ? j : 0;  // a row of R that exists, loaded (and ignored) for empty slots
        double s2 = 0.0, yy = 0.0, sxy = 0.0;
        for (int k0 = 0; k0 < a.d; k0 += kRerankChunk) {
            const int w = min(kRerankChunk, a.d - k0);
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // earlier reads of the tile are done
            __builtin_amdgcn_wave_barrier();
#pragma unroll 4
            for (int i = 0; i < kWave / 2; ++i) {
                const int r = 2 * i + (lane >> 5), cc = lane & (kRerankChunk - 1);
                const int jr = __shfl(jl, r, kWave);
                if (cc < w) T[r][cc] = a.R[(int64_t)jr * a.d + k0 + cc];
            }
            __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the tile is written
            __builtin_amdgcn_wave_barrier();
            if (cosine) {
                for (int t = 0; t < w; ++t) {
                    const double y = (double)T[lane][t];
                    sxy = __dadd_rn(sxy, __dmul_rn((double)xs[k0 + t], y));
                    yy = __dadd_rn(yy, __dmul_rn(y, y));
                }
            } else {
                for (int t = 0; t < w; ++t) {
                    const double y = (double)T[lane][t];
                    const double diff = __dsub_rn((double)xs[k0 + t], y);
                    s2 = __dadd_rn(s2, __dmul_rn(diff, diff));
                    yy += y * y;
                }
            }
        }
        double d2 = INFINITY;
        int jj = INT_MAX;
        if (valid) {
            jj = j;
            if (cosine) {
                // 1 - x.y / (||x|| ||y||); a row of zero norm is at distance 1
                const bool zero = cxx == 0.0 || yy == 0.0;
                d2 = zero ? 1.0 : __dsub_rn(1.0, __ddiv_rn(sxy, __dmul_rn(__dsqrt_rn(cxx), __dsqrt_rn(yy))));
                // the screen ranked 2 D - 1 (unit vectors) up to cosine_eps
                if (!zero) ratio = fmaxf(ratio, (float)(fabs((double)key - (2.0 * d2 - 1.0)) / a.cosine_eps));
            } else {
                d2 = s2;
                const double yn = sqrt(yy);
                const double err_bound = a.eps_coef * (2.0 * xn * yn + yy) + 1e-300;
                ratio = fmaxf(ratio, (float)(fabs((double)key - (d2 - xx)) / err_bound));
            }
        }
        bitonic_sort64(d2, jj, lane);
        top.merge(d2, jj, lane);
    }
    ratio = wave_max(ratio);
    if (lane == 0 && ratio > 0.f) atomicMax(&a.counters->max_ratio_bits, __float_as_uint(ratio));

    const int m = a.self_mode ? a.k - 1 : a.k;  // neighbours to certify
    bool ok = true;
    if (a.certify && m > 0 && tau < INFINITY && cosine) {
        // Unit vectors: a rejected reference y had a screened key >= tau, and
        // the key is 2 D_y - 1 up to cosine_eps, so D_y >= (tau + 1 - eps) / 2,
        // which must exceed D_m.  (A zero row's key may be far from its
        // D_y = 1 but never above it: the bound still holds for it.)
        double dm;
        int jm;
        top.at(m - 1, dm, jm);
        const double bound = ((double)tau + 1.0 - a.cosine_eps) * 0.5 - 1e-13;
        ok = dm < bound;
    } else if (a.certify && m > 0 && tau < INFINITY) {
        // A rejected reference y had a screened key >= tau.  If ||y|| > Y =
        // ||x|| + D_m it lies farther than D_m (triangle inequality); else its
        // float32 key is off by at most eps(Y), so its true key is >= tau -
        // eps(Y), which must exceed D_m^2 - ||x||^2.
        double dm;
        int jm;
        top.at(m - 1, dm, jm);
        const double Y = fmin(ymax, (xn + sqrt(dm)) * (1.0 + 1e-9));
        const double eps = a.eps_coef * (2.0 * xn * Y + Y * Y);
        const double bound = (double)tau + xx - eps - 1e-12 * (fabs((double)tau) + xx);
        ok = dm < bound;
    }

    int32_t *oi = a.out_idx + row * a.k;
    float *od = a.out_dist + row * a.k;
    const int off = a.self_mode ? 1 : 0;
    if (a.self_mode && lane == 0) {
        oi[0] = (int32_t)row;
        od[0] = 0.f;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int pos = r * kWave + lane;
        if (pos < m) {
            oi[off + pos] = top.j[r] == INT_MAX ? -1 : top.j[r];
            od[off + pos] = cosine ? (float)top.d[r] : (float)sqrt(top.d[r]);
        }
    }
    if (!ok && lane == 0) {
        const int pos = atomicAdd(a.flag_count, 1);
        a.flag_out[pos] = (int32_t)row;
    }
}

// ---------------------------------------------------------------------------
// Exhaustive float64 scan of the rows no screen could certify: rows
// list2[0..count2) and list1[cap..count1).  One wave per row: each step the
// 64 lanes compute the distances of 64 consecutive references; a step with
// a distance before the current m-th is sorted and merged into the row's
// wave-wide top-m (TopM).
// ---------------------------------------------------------------------------
template <int R>
__global__ __launch_bounds__(64) void k_rescan(const float *__restrict__ Q, const float *__restrict__ Rf, int64_t nr,
                                               int d, int k, int self_mode, const int32_t *__restrict__ list1,
                                               const int32_t *__restrict__ count1, int cap1,
                                               const int32_t *__restrict__ list2,
                                               const int32_t *__restrict__ count2, int32_t *__restrict__ out_idx,
                                               float *__restrict__ out_dist, KnnCounters *__restrict__ counters,
                                               const int64_t *__restrict__ soff, int nsamples, int metric) {
    const int lane = threadIdx.x;
    const int m = self_mode ? k - 1 : k;
    const int c2 = *count2;
    const int extra = std::max(0, *count1 - cap1);
    const int count = c2 + extra;
    if (blockIdx.x == 0 && lane == 0) counters->rescanned = count;
    for (int f = blockIdx.x; f < count; f += gridDim.x) {
        const int64_t q = f < c2 ? list2[f] : list1[cap1 + (f - c2)];
        const float *x = Q + q * d;
        // references: all rows, or the rows of q's own sample (batched form)
        int64_t j0 = 0, j1 = nr;
        if (soff) {
            int lo = 0, hi = nsamples - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) / 2;
                if (soff[mid] <= q) lo = mid; else hi = mid - 1;
            }
            j0 = soff[lo];
            j1 = soff[lo + 1];
        }
        double cxx = 0.0;  // cosine: the query's squared norm, dimensions in order
        if (metric == RSC_COSINE)
            for (int t = 0; t < d; ++t) cxx = __dadd_rn(cxx, __dmul_rn((double)x[t], (double)x[t]));
        TopM<R> top;
        top.init();
        for (int64_t jb = j0; jb < j1; jb += kWave) {
            const int64_t j = jb + lane;
            double v = INFINITY;
            int jj = INT_MAX;
            if (j < j1 && !(self_mode && j == q)) {
                const float *y = Rf + j * d;
                if (metric == RSC_COSINE) {
                    double sxy = 0.0, syy = 0.0;
                    for (int t = 0; t < d; ++t) {
                        sxy = __dadd_rn(sxy, __dmul_rn((double)x[t], (double)y[t]));
                        syy = __dadd_rn(syy, __dmul_rn((double)y[t], (double)y[t]));
                    }
                    v = (cxx == 0.0 || syy == 0.0)
                            ? 1.0
                            : __dsub_rn(1.0, __ddiv_rn(sxy, __dmul_rn(__dsqrt_rn(cxx), __dsqrt_rn(syy))));
                } else {
                    v = exact_d2(x, y, d);
                }
                jj = (int)j;
            }
            if (m < 1) continue;
            double md;
            int mj;
            top.at(m - 1, md, mj);
            if (__ballot(lex_before(v, jj, md, mj)) == 0ull) continue;
            bitonic_sort64(v, jj, lane);
            top.merge(v, jj, lane);
        }
        int32_t *oi = out_idx + q * k;
        float *od = out_dist + q * k;
        const int off = self_mode ? 1 : 0;
        if (self_mode && lane == 0) {
            oi[0] = (int32_t)q;
            od[0] = 0.f;
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int pos = r * kWave + lane;
            if (pos < m) {
                oi[off + pos] = top.j[r] == INT_MAX ? -1 : top.j[r];
                od[off + pos] = metric == RSC_COSINE ? (float)top.d[r] : (float)sqrt(top.d[r]);
            }
        }
    }
}

// Registers per lane of the running top-m list.
int topm_regs(int m) { return m <= 64 ? 1 : m <= 128 ? 2 : 4; }

// sparse: a grid with few active workgroups (the escalation)
template <int DH, int L>
int launch_screen(const ScreenArgs &a, unsigned gx, bool sparse, const char *name, hipStream_t stream) {
    ScopedTimer timer(name, stream);
    constexpr int WF = tile_screen_waves(DH, L), WS = screen_min_waves(DH, L);
    if (sparse && WS != WF)
        hipLaunchKernelGGL((k_screen_fp32<DH, L, WS>), dim3(gx, (unsigned)a.P), dim3(256), 0, stream, a);
    else
        hipLaunchKernelGGL((k_screen_fp32<DH, L, WF>), dim3(gx, (unsigned)a.P), dim3(256), 0, stream, a);
    return launch_status(name);
}

template <int L>
int dispatch_screen(int dh, const ScreenArgs &a, unsigned gx, bool sparse, const char *name, hipStream_t s) {
    switch (dh) {
        case 4: return launch_screen<4, L>(a, gx, sparse, name, s);
        case 8: return launch_screen<8, L>(a, gx, sparse, name, s);
        case 16: return launch_screen<16, L>(a, gx, sparse, name, s);
        case 25: return launch_screen<25, L>(a, gx, sparse, name, s);
        case 32: return launch_screen<32, L>(a, gx, sparse, name, s);
        case 48: return launch_screen<48, L>(a, gx, sparse, name, s);
        case 64: return launch_screen<64, L>(a, gx, sparse, name, s);
        case 96: return launch_screen<96, L>(a, gx, sparse, name, s);
        case 128: return launch_screen<128, L>(a, gx, sparse, name, s);
        default: set_error("internal: no screen kernel for this dimension"); return RSC_ERR_UNSUPPORTED;
    }
}

// One launch of the screen; `half_width` is the list length per contraction
// half; `sparse` marks a grid with few active workgroups.
int screen(int dh, const ScreenArgs &a, unsigned gx, int half_width, bool sparse, const char *name, hipStream_t s) {
    if (half_width == 16) return dispatch_screen<16>(dh, a, gx, sparse, name, s);
    return dispatch_screen<32>(dh, a, gx, sparse, name, s);
}

constexpr int kQueriesPerGroup = kScreenWaves * 32;

int pick_dh(int d) {
    const int half = (d + 1) / 2;
    const int opts[] = {4, 8, 16, 25, 32, 48, 64, 96, 128};
    for (int o : opts)
        if (half <= o) return o;
    return -1;
}

// Reference ranges for the main screen: enough workgroups to fill the chip
// (about 4 per CU) while every range keeps at least 8 blocks.
int pick_splits(int64_t nq, int64_t nblk, int qg) {
    const int64_t qblocks = (nq + qg - 1) / qg;
    const int64_t want = 1024;
    int64_t P = qblocks >= want ? 1 : (want + qblocks - 1) / qblocks;
    P = std::min<int64_t>(P, std::max<int64_t>(1, nblk / 8));
    P = std::min<int64_t>(P, 32);
    return (int)std::max<int64_t>(P, 1);
}

}  // namespace

// Error bound of the float32 key (the norm enters the MFMA sum or is added
// after it; norms rounded once from float64): 2 (d + 3) units of roundoff
// times (2 ||x|| ||y|| + ||y||^2).
double knn_eps_coefficient(int d) { return 2.0 * (d + 3) * std::ldexp(1.0, -24); }

int knn_prep_fp32(const KnnPlan &p, const float *R, const KnnBuffers &b, const int32_t *blk_sample,
                  const int64_t *boff, const int64_t *soff, hipStream_t stream) {
    const int s4 = packed_s4(p.dh);
    ScopedTimer timer("prep_pack", stream);
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, stream, b.counters);
    hipLaunchKernelGGL(k_norms, dim3((unsigned)((p.nr + norm_rows(p.d) - 1) / norm_rows(p.d))), dim3(kNormRows), 0, stream, R,
                       p.nr, p.d, b.nrow,
                       &b.counters->max_norm_bits);
    const int64_t tot = p.nblk * s4 * kWave;
    const unsigned g1 = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
    hipLaunchKernelGGL(k_pack, dim3(g1), dim3(256), 0, stream, R, b.nrow, p.nr, p.d, p.dh, s4,
                       norm_folded(p.dh) ? 1 : 0, p.nblk, reinterpret_cast<f32x4 *>(b.packed), b.norms, blk_sample,
                       boff, soff, nullptr);
    return launch_status("prep_pack");
}

int knn_norms(const float *R, int64_t nr, int d, float *nrow, KnnCounters *counters, hipStream_t stream) {
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, stream, counters);
    hipLaunchKernelGGL(k_norms, dim3((unsigned)((nr + norm_rows(d) - 1) / norm_rows(d))), dim3(kNormRows), 0, stream, R, nr,
                       d, nrow,
                       &counters->max_norm_bits);
    return launch_status("norms");
}

int knn_pack_mapped(int dh, const float *R, const float *nrow, int64_t nr, int d, int64_t nblk, float *packed,
                    float *norms, const int32_t *row_map, hipStream_t stream) {
    const int s4 = packed_s4(dh);
    ScopedTimer timer("prep_pack", stream);
    const int64_t tot = nblk * s4 * kWave;
    const unsigned g1 = (unsigned)std::max<int64_t>(1, std::min<int64_t>((tot + 255) / 256, 65536));
    hipLaunchKernelGGL(k_pack, dim3(g1), dim3(256), 0, stream, R, nrow, nr, d, dh, s4, norm_folded(dh) ? 1 : 0, nblk,
                       reinterpret_cast<f32x4 *>(packed), norms, nullptr, nullptr, nullptr, row_map);
    return launch_status("prep_pack");
}

size_t knn_packed_floats(int dh, int64_t nblk) { return (size_t)nblk * packed_s4(dh) * kWave * 4; }

int knn_launch_screen(int dh, const scr::ScreenArgs &a, unsigned gx, int half_width, const char *name,
                      hipStream_t s) {
    return screen(dh, a, gx, half_width, false, name, s);
}

int knn_launch_rerank(const RerankArgs &ra, int64_t slots, const char *name, hipStream_t stream) {
    ScopedTimer timer(name, stream);
    const dim3 grid((unsigned)((slots + 3) / 4));
    switch (topm_regs(ra.self_mode ? ra.k - 1 : ra.k)) {
        case 1: hipLaunchKernelGGL(k_rerank<1>, grid, dim3(256), 0, stream, ra); break;
        case 2: hipLaunchKernelGGL(k_rerank<2>, grid, dim3(256), 0, stream, ra); break;
        default: hipLaunchKernelGGL(k_rerank<4>, grid, dim3(256), 0, stream, ra); break;
    }
    return launch_status(name);
}

int knn_launch_rescan(const KnnPlan &p, const float *Q, const float *R, const KnnBuffers &b, int esc_cap,
                      int32_t *out_idx, float *out_dist, const int64_t *soff, int nsamples, hipStream_t stream) {
    ScopedTimer timer("rescan", stream);
    auto go = [&](auto kern) {
        hipLaunchKernelGGL(kern, dim3(1024), dim3(64), 0, stream, Q, R, p.nr, p.d, p.k, p.self_mode ? 1 : 0, b.flag1,
                           &b.counters->flagged, esc_cap, b.flag2, &b.counters->flagged2, out_idx, out_dist,
                           b.counters, soff, nsamples, p.metric);
    };
    switch (topm_regs(p.self_mode ? p.k - 1 : p.k)) {
        case 1: go(k_rescan<1>); break;
        case 2: go(k_rescan<2>); break;
        default: go(k_rescan<4>); break;
    }
    return launch_status("rescan");
}

int knn_plan(int64_t nq, int64_t nr, int d, int k, const rsc_knn_opts *opts, bool self_mode, KnnPlan *plan) {
    if (nq < 0 || nr < 1) {
        set_error("need n_query >= 0 and n_ref >= 1");
        return RSC_ERR_INVALID_ARG;
    }
    if (nq > INT32_MAX - 1 || nr > INT32_MAX - 1) {
        set_error("row counts above 2^31-2 cannot be indexed by int32");
        return RSC_ERR_OVERFLOW;
    }
    if (d < 1 || k < 1 || k > nr) {
        set_error("need d >= 1 and 1 <= k <= n_ref");
        return RSC_ERR_INVALID_ARG;
    }
    if (d > kMaxD) {
        set_error("d > 256 is not supported by this build");
        return RSC_ERR_UNSUPPORTED;
    }
    if (k > kMaxK) {
        set_error("k > 255 is not supported by this build");
        return RSC_ERR_UNSUPPORTED;
    }
    int precision = opts ? opts->precision : RSC_FP32;
    if (precision != RSC_FP32 && (d > kMaxDLowp || k > kMaxKLowp)) {
        set_error("reduced-precision screens support d <= 128 and k <= 63");
        return RSC_ERR_UNSUPPORTED;
    }
    int screen_w = opts ? opts->screen : 0;
    const int metric = opts ? opts->metric : RSC_EUCLIDEAN;
    if (metric != RSC_EUCLIDEAN && metric != RSC_COSINE) {
        set_error("unknown metric");
        return RSC_ERR_INVALID_ARG;
    }
    if (precision != RSC_FP32 && precision != RSC_BF16 && precision != RSC_FP8_E4M3) {
        set_error("unknown precision");
        return RSC_ERR_INVALID_ARG;
    }
    if (precision == RSC_FP32) {
        if (screen_w == 0) screen_w = k <= 16 ? 32 : 64;
        if ((screen_w != 32 && screen_w != 64) || (k < 64 && screen_w <= k) || (k >= 64 && screen_w != 64)) {
            set_error("screen width must be 32 or 64 and larger than k (64 for k >= 64)");
            return RSC_ERR_INVALID_ARG;
        }
    } else {
        if (screen_w == 0) screen_w = 64;
        if (screen_w != 64 && screen_w != 128 && screen_w != 256 && screen_w != 512) {
            set_error("reduced-precision screens keep 64, 128, 256 or 512 candidates per query");
            return RSC_ERR_INVALID_ARG;
        }
    }
    const int resid = opts ? opts->fp8_residual : 0;
    if (resid != 0) {
        if (precision != RSC_FP8_E4M3 || metric != RSC_EUCLIDEAN) {
            set_error("fp8_residual needs the FP8-e4m3 screen and the Euclidean metric");
            return RSC_ERR_INVALID_ARG;
        }
        if (resid < 2 || resid > 4096 || resid > nr) {
            set_error("fp8_residual: the partition count must lie in [2, min(4096, n_ref)]");
            return RSC_ERR_INVALID_ARG;
        }
    }
    const int lowp_ranges = precision == RSC_FP32 ? 1 : screen_w / 64;
    if (precision != RSC_FP32) screen_w = 64;  // per reference range; the ranges multiply it
    plan->nq = nq;
    plan->nr = nr;
    plan->d = d;
    plan->k = k;
    plan->screen = screen_w;
    plan->half = screen_w / 2;
    plan->dh = pick_dh(d);
    plan->self_mode = self_mode;
    plan->nblk = (nr + 31) / 32 + resid;  // residual variant: each partition's last block padded
    plan->precision = precision;
    plan->metric = metric;
    plan->resid = resid;
    plan->splits = pick_splits(nq, plan->nblk,
                               precision == RSC_FP32 ? kQueriesPerGroup : lowp_queries_per_group(precision, d));
    if (precision == RSC_FP32) {
        // enough (range, half) lists that the m nearest fill each to about half
        const int m = self_mode ? k - 1 : k;
        plan->splits = std::min(32, std::max(plan->splits, (m + plan->half - 1) / plan->half));
    } else {
        plan->splits = std::max(plan->splits, lowp_ranges);
    }
    return RSC_OK;
}

size_t knn_workspace(const KnnPlan &p, void *ws, KnnBuffers *out) {
    Carver cv(ws);
    KnnBuffers b{};
    const bool fp32 = p.precision == RSC_FP32;
    const int s4 = packed_s4(p.dh);
    const int64_t esc_rows = fp32 ? std::min<int64_t>(p.nq, kEscalateCap) : 0;
    b.counters = cv.take<KnnCounters>(1);
    if (fp32) {
        b.nrow = cv.take<float>((size_t)p.nr);
        b.packed = cv.take<float>((size_t)p.nblk * s4 * kWave * 4);
        b.norms = cv.take<float>(norm_folded(p.dh) ? 1 : (size_t)p.nblk * 32);
    } else {
        b.packed = reinterpret_cast<float *>(cv.take<char>(lowp_packed_bytes(p.precision, p.nblk, p.d)));
        b.norms = cv.take<float>((size_t)p.nblk * 32);
        b.scal = cv.take<float>(2 * 128 + 1);
        b.amax = cv.take<uint32_t>(256);
    }
    b.cand_idx = cv.take<int32_t>((size_t)p.nq * p.splits * p.screen);
    b.cand_key = cv.take<float>((size_t)p.nq * p.splits * p.screen);
    b.flag1 = cv.take<int32_t>((size_t)std::max<int64_t>(p.nq, 1));
    b.flag2 = cv.take<int32_t>((size_t)std::max<int64_t>(esc_rows, 1));
    b.esc_idx = cv.take<int32_t>((size_t)std::max<int64_t>(esc_rows, 1) * kEscalateSplits * kEscalateWidth);
    b.esc_key = cv.take<float>((size_t)std::max<int64_t>(esc_rows, 1) * kEscalateSplits * kEscalateWidth);
    if (p.metric == RSC_COSINE) {
        b.rn = cv.take<float>((size_t)p.nr * p.d);
        b.qn = p.self_mode ? b.rn : cv.take<float>((size_t)std::max<int64_t>(p.nq, 1) * p.d);
    }
    if (!fp32 && p.resid == 0 && p.nq > 0) {
        // spatial order of the queries (perm) and its sort
        b.perm = cv.take<int32_t>((size_t)p.nq);
        b.qcount = cv.take<int32_t>(1);
        b.order_ws = cv.take<char>(query_order_workspace(p.nq));
    }
    if (p.resid > 0) {
        b.cent = cv.take<float>((size_t)p.resid * p.d);
        b.assign = cv.take<int32_t>((size_t)p.nr);
        b.perm = cv.take<int32_t>((size_t)p.nr);
        b.init = cv.take<int32_t>((size_t)p.resid);
        b.poff = cv.take<int64_t>((size_t)p.resid + 1);
        b.pblk = cv.take<int64_t>((size_t)p.resid + 1);
        b.blk_part = cv.take<int32_t>((size_t)p.nblk * 4);
        b.map = cv.take<int32_t>((size_t)p.nblk * 32);
        b.qcount = cv.take<int32_t>(1);
        b.kws_bytes = kmeans_workspace_bytes(p.nr, p.d, p.resid);
        b.kws = cv.take<char>(b.kws_bytes ? b.kws_bytes : 1);
    }
    if (out) *out = b;
    return cv.used;
}

// Cosine metric: the screen's inputs are the unit-normalised rows.
int normalize_inputs(const KnnPlan &p, const float *Q, const float *R, const KnnBuffers &b, hipStream_t stream) {
    ScopedTimer timer("normalize", stream);
    hipLaunchKernelGGL(k_normalize, dim3((unsigned)((p.nr + norm_rows(p.d) - 1) / norm_rows(p.d))), dim3(kNormRows), 0, stream,
                       R, p.nr, p.d, b.rn);
    if (!p.self_mode && p.nq > 0)
        hipLaunchKernelGGL(k_normalize, dim3((unsigned)((p.nq + norm_rows(p.d) - 1) / norm_rows(p.d))), dim3(kNormRows), 0,
                           stream, Q, p.nq, p.d, b.qn);
    return launch_status("normalize");
}

// Bound on |screened key - (2 D - 1)| for the cosine screen: the float32
// key error of unit vectors (eps_coef (2 |x||y| + |y|^2) with norms within
// 4 units of 1) plus the normalisation: each unit vector is within 2 units of
// roundoff per element of the exact direction, which moves |y|^2 by at most
// 4 units and x.y by at most 4 units (doubled in the key), with a margin.
double cosine_eps(int d) { return 3.0001 * knn_eps_coefficient(d) + 16.0 * std::ldexp(1.0, -24); }

// Reduced-precision form: screen, then rerank without a certificate.
int knn_run_lowp(const KnnPlan &p, const float *Q, const float *R, int32_t *out_idx, float *out_dist,
                 const KnnBuffers &b, hipStream_t stream) {
    int st;
    hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, stream, b.counters);
    if ((st = launch_status("init_counters")) != RSC_OK) return st;
    const bool cosine = p.metric == RSC_COSINE;
    if (cosine && (st = normalize_inputs(p, Q, R, b, stream)) != RSC_OK) return st;
    const float *Qs = cosine ? b.qn : Q, *Rs = cosine ? b.rn : R;  // what the screen sees
    // The queries are screened in an order that keeps neighbours together,
    // so that the 32 queries of a wave tend to take keys from the same
    // blocks and share the selection's queue flushes: the residual variant
    // on one matrix uses its partition order, the other forms a Morton order
    // of the first coordinates (query_order.hip).  On one matrix screened as
    // a single reference range the latter also packs the references in that
    // order, and every query group starts its scan at its own rows: the
    // nearest references come first and tighten the thresholds before the
    // rest streams past.  (With several ranges, references packed in that
    // order would put a query's near rows into one range, whose 64
    // candidates are then all it keeps of them: fewer true neighbours
    // survive the noisier FP8 keys.)
    bool ordered = false, rotate = false;
    if (p.resid == 0 && b.order_ws && p.nq > 0) {
        if ((st = query_order_run(Qs, p.nq, p.d, b.order_ws, b.perm, stream)) != RSC_OK) return st;
        ordered = true;
        rotate = p.self_mode && p.splits == 1;
    }
    if (p.resid > 0)
        st = lowp_prepare_resid(p, R, b, stream);
    else
        st = lowp_prepare(p, Qs, Rs, b.packed, b.norms, b.scal, b.amax, rotate ? b.perm : nullptr, stream);
    if (st != RSC_OK) return st;
    if (p.nq == 0) return RSC_OK;
    if (p.resid > 0) ordered = p.self_mode;
    if (ordered) {
        hipLaunchKernelGGL(k_set_i32, dim3(1), dim3(64), 0, stream, b.qcount, (int32_t)p.nq);
        if ((st = launch_status("set query count")) != RSC_OK) return st;
    }
    ScreenArgs sa{};
    sa.Q = Qs;
    sa.nq = p.nq;
    sa.qlist = ordered ? b.perm : nullptr;
    sa.qcount = ordered ? b.qcount : nullptr;
    sa.qcap = (int)p.nq;
    sa.Ap = b.packed;
    sa.Np = b.norms;
    sa.qscale = b.scal;
    sa.blk_part = b.blk_part;
    sa.cent = b.cent;
    sa.nblk = p.nblk;
    sa.d = p.d;
    sa.P = p.splits;
    sa.rotate = rotate ? 1 : 0;
    sa.cand_idx = b.cand_idx;
    sa.cand_key = b.cand_key;
    const int qg = lowp_queries_per_group(p.precision, p.d);
    if ((st = lowp_screen(p, sa, (unsigned)((p.nq + qg - 1) / qg), stream)) != RSC_OK) return st;
    if (p.resid > 0 && (st = lowp_unmap(p, b, stream)) != RSC_OK) return st;
    if (rotate && (st = lowp_unmap_rows(p, b, b.perm, stream)) != RSC_OK) return st;
    RerankArgs ra{};
    ra.Q = Q;
    ra.nq = p.nq;
    ra.qlist = sa.qlist;
    ra.qcount = sa.qcount;
    ra.qcap = sa.qcap;
    ra.R = R;
    ra.d = p.d;
    ra.k = p.k;
    ra.S = p.half;
    ra.KP = p.half;
    ra.P = 2 * p.splits;
    ra.self_mode = p.self_mode ? 1 : 0;
    ra.certify = 0;
    ra.metric = p.metric;
    ra.cosine_eps = 1.0;
    ra.cand_idx = b.cand_idx;
    ra.cand_key = b.cand_key;
    ra.eps_coef = 1.0;
    ra.counters = b.counters;
    ra.flag_out = b.flag1;
    ra.flag_count = &b.counters->flagged;
    ra.out_idx = out_idx;
    ra.out_dist = out_dist;
    return knn_launch_rerank(ra, p.nq, "rerank", stream);
}

int knn_run(const KnnPlan &p, const float *Q, const float *R, int32_t *out_idx, float *out_dist, void *ws,
            hipStream_t stream, const int32_t *qlist, const int32_t *qcount) {
    KnnBuffers b;
    knn_workspace(p, ws, &b);
    if (p.precision != RSC_FP32) {
        if (qlist) {
            set_error("internal: row lists need the FP32 path");
            return RSC_ERR_UNSUPPORTED;
        }
        return knn_run_lowp(p, Q, R, out_idx, out_dist, b, stream);
    }
    int st;
    const bool cosine = p.metric == RSC_COSINE;
    if (cosine && (st = normalize_inputs(p, Q, R, b, stream)) != RSC_OK) return st;
    const float *Qs = cosine ? b.qn : Q;  // what the screen sees
    if ((st = knn_prep_fp32(p, cosine ? b.rn : R, b, nullptr, nullptr, nullptr, stream)) != RSC_OK) return st;
    if (p.nq == 0) return RSC_OK;

    const double eps_coef = knn_eps_coefficient(p.d);

    // Slots are rows 0..nq-1, or the first min(*qcount, nq) rows of qlist.
    ScreenArgs sa{};
    sa.Q = Qs;
    sa.nq = p.nq;
    sa.qlist = qlist;
    sa.qcount = qcount;
    sa.qcap = (int)p.nq;
    sa.Ap = b.packed;
    sa.Np = b.norms;
    sa.nblk = p.nblk;
    sa.d = p.d;
    sa.P = p.splits;
    sa.cand_idx = b.cand_idx;
    sa.cand_key = b.cand_key;
    const unsigned gq = (unsigned)((p.nq + kQueriesPerGroup - 1) / kQueriesPerGroup);
    if ((st = screen(p.dh, sa, gq, p.half, false, "screen_fp32", stream)) != RSC_OK) return st;

    // Each (range, half) list is one candidate group of width `half`.
    RerankArgs ra{};
    ra.Q = Q;
    ra.nq = p.nq;
    ra.qlist = qlist;
    ra.qcount = qcount;
    ra.qcap = (int)p.nq;
    ra.R = R;
    ra.d = p.d;
    ra.k = p.k;
    ra.S = p.half;
    ra.KP = p.half;
    ra.P = 2 * p.splits;
    ra.self_mode = p.self_mode ? 1 : 0;
    ra.certify = 1;
    ra.metric = p.metric;
    ra.cosine_eps = cosine_eps(p.d);
    ra.cand_idx = b.cand_idx;
    ra.cand_key = b.cand_key;
    ra.eps_coef = eps_coef;
    ra.counters = b.counters;
    ra.flag_out = b.flag1;
    ra.flag_count = &b.counters->flagged;
    ra.out_idx = out_idx;
    ra.out_dist = out_dist;
    if ((st = knn_launch_rerank(ra, p.nq, "rerank", stream)) != RSC_OK) return st;

    // Escalation: rows that failed, screened again 64 wide over many ranges.
    const int esc_cap = (int)std::min<int64_t>(p.nq, kEscalateCap);
    ScreenArgs se = sa;
    se.qlist = b.flag1;
    se.qcount = &b.counters->flagged;
    se.qcap = esc_cap;
    se.P = (int)std::min<int64_t>(kEscalateSplits, std::max<int64_t>(1, p.nblk));
    se.cand_idx = b.esc_idx;
    se.cand_key = b.esc_key;
    const unsigned ge = (unsigned)((esc_cap + kQueriesPerGroup - 1) / kQueriesPerGroup);
    if ((st = screen(p.dh, se, ge, kEscalateWidth / 2, true, "screen_escalate", stream)) != RSC_OK) return st;
    RerankArgs re = ra;
    re.qlist = b.flag1;
    re.qcount = &b.counters->flagged;
    re.qcap = esc_cap;
    re.S = kEscalateWidth / 2;
    re.KP = kEscalateWidth / 2;
    re.P = 2 * se.P;
    re.cand_idx = b.esc_idx;
    re.cand_key = b.esc_key;
    re.flag_out = b.flag2;
    re.flag_count = &b.counters->flagged2;
    if ((st = knn_launch_rerank(re, esc_cap, "rerank_escalate", stream)) != RSC_OK) return st;
    return knn_launch_rescan(p, Q, R, b, esc_cap, out_idx, out_dist, nullptr, 0, stream);
}

}  // namespace rsc
