// Exact kNN on gfx950: MFMA distance screen + float64 rerank + certificate.
//
// The paper's neighbour step needs, per cell, the k nearest cells of the
// PCA embedding under the squared Euclidean distance of Methods, "Custom
// GPU kernels" (d_ij = ||x_i - x_j||^2).  The work is a dense contraction
// (2 d flops per ordered pair), so the screen runs on the matrix cores:
//
//   key_ij = ||y_j||^2 - 2 x_i . y_j      (= d_ij - ||x_i||^2, same order per row)
//
// Data path of the screen (one wave = 64 queries, one workgroup = 4 waves):
//   * the query operand (-2 x) stays in VGPRs for the whole launch;
//   * references are repacked once into the MFMA A-operand order (one
//     float4 per lane per four contraction steps, 1 KiB per wave load, fully
//     coalesced) and streamed HBM/MALL/L2 -> VGPR with a one-block
//     register prefetch; no LDS staging and no workgroup barrier;
//   * ||y||^2 is loaded straight into the accumulator (the C input of the
//     first v_mfma_f32_32x32x2_f32 of a block), so the MFMA chain produces
//     the key itself;
//   * the epilogue is one compare per pair against the query's current
//     threshold; a key below it enters the query's max-heap of the S
//     smallest keys in LDS (rare after the first few blocks).
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

namespace rsc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWave = 64;
constexpr int kScreenWaves = 4;   // waves per screen workgroup
constexpr int kMaxD = 128;
constexpr int kMaxK = 63;
constexpr int kRescanMax = 64;    // list capacity of the exhaustive rescan
constexpr int kEscalateCap = 2048;  // rows handled by the escalation screen
constexpr int kEscalateSplits = 32;
constexpr int kEscalateWidth = 64;

// (d2, j) lexicographic order: smaller distance first, lower index on ties.
__device__ __forceinline__ bool lex_before(double da, int ja, double db, int jb) {
    return da < db || (da == db && ja < jb);
}

// Squared distance of two float32 rows in float64, dimensions in order,
// every product and sum rounded separately (no contraction).
__device__ __forceinline__ double exact_d2(const float *__restrict__ x, const float *__restrict__ y, int d) {
    double s = 0.0;
    for (int t = 0; t < d; ++t) {
        double diff = __dsub_rn((double)x[t], (double)y[t]);
        s = __dadd_rn(s, __dmul_rn(diff, diff));
    }
    return s;
}

__device__ __forceinline__ float wave_max(float v) {
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, kWave));
    return v;
}

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, kWave);
    return v;
}

// Packed reference layout for a contraction half-width DH (DHP = DH rounded
// up to 4).  Block b holds rows 32b..32b+31:
//   A[b][s4][lane] (float4): element u = R[32b + lane%32][(lane/32) DH + 4 s4 + u]
//   N[b][h][4g + j]        : ||R[32b + 8g + 4h + j]||^2   (+inf past the end)
// so that MFMA step s reads lane-contiguous data and the norms land in the
// accumulator registers in output order.
__global__ __launch_bounds__(256) void k_pack(const float *__restrict__ R, int64_t nr, int d, int DH, int DHP4,
                                              int64_t nblk, f32x4 *__restrict__ Ap) {
    const int64_t total = nblk * DHP4 * kWave;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(e % kWave);
        const int64_t bs = e / kWave;
        const int s4 = (int)(bs % DHP4);
        const int64_t b = bs / DHP4;
        const int64_t row = 32 * b + (lane & 31);
        const int h = lane >> 5;
        f32x4 v;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = 4 * s4 + u;
            const int t = h * DH + s;
            v[u] = (row < nr && s < DH && t < d) ? R[row * d + t] : 0.f;
        }
        Ap[e] = v;
    }
}

// Squared norms (float64 sum, rounded once) in the packed order, and the
// largest norm.
__global__ __launch_bounds__(256) void k_pack_norms(const float *__restrict__ R, int64_t nr, int d, int64_t nblk,
                                                    float *__restrict__ Np, uint32_t *__restrict__ max_norm_bits) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float nf = 0.f;
    if (r < nblk * 32) {
        float out = INFINITY;
        if (r < nr) {
            const float *x = R + r * d;
            double s = 0.0;
            for (int t = 0; t < d; ++t) s += (double)x[t] * (double)x[t];
            out = (float)s;
            nf = out;
        }
        const int64_t b = r >> 5;
        const int i = (int)(r & 31);
        const int g = i >> 3, h = (i >> 2) & 1, j = i & 3;
        Np[b * 32 + h * 16 + 4 * g + j] = out;
    }
    const float m = wave_max(sqrtf(nf));
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(max_norm_bits, __float_as_uint(m));
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
// Lane l handles query column c = l % 32 of each of its QB query blocks and
// contraction half h = l / 32: dimension h*DH + s feeds MFMA step s.  Output
// register v of a 32x32 block holds reference row 8(v/4) + 4h + (v%4).
// Query slot i of the launch is row i, or row qlist[i] for i < min(*qcount,
// qcap) when a list is given (the escalation pass).
// ---------------------------------------------------------------------------
struct ScreenArgs {
    const float *Q;
    int64_t nq;
    const int32_t *qlist;   // optional gather list
    const int32_t *qcount;  // its device-side length
    int qcap;
    const f32x4 *Ap;
    const float *Np;
    int64_t nblk;
    int d;
    int S;  // heap size (<= KP)
    int P;  // reference ranges (gridDim.y)
    int32_t *cand_idx;  // [slot][P][KP]
    float *cand_key;
};

template <int DH, int QB, int KP>
__global__ __launch_bounds__(256, 2) void k_screen_fp32(ScreenArgs a) {
    constexpr int QW = QB * 32;
    constexpr int QG = kScreenWaves * QW;
    constexpr int DHP = (DH + 3) & ~3;
    constexpr int S4 = DHP / 4;

    __shared__ float hk[KP * QG];
    __shared__ int hi[KP * QG];

    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    const int h = lane >> 5, c = lane & 31;
    const int p = blockIdx.y;
    const int64_t blk_per = (a.nblk + a.P - 1) / a.P;
    const int64_t blk0 = (int64_t)p * blk_per;
    const int64_t blk1 = std::min<int64_t>(a.nblk, blk0 + blk_per);
    const int S = a.S;

    int64_t nslots = a.nq;
    if (a.qlist) {
        const int cnt = *a.qcount;
        nslots = std::min<int64_t>(std::min<int64_t>(cnt, a.qcap), a.nq);
    }

    for (int64_t qblk = blockIdx.x; qblk * QG < nslots; qblk += gridDim.x) {
        const int64_t slot_wave = qblk * QG + wave * QW;

        // Query operand, resident for the whole range; -2 folded in (exact).
        float b[QB][DH];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const int64_t slot = slot_wave + qb * 32 + c;
            int64_t row = -1;
            if (slot < nslots) row = a.qlist ? (int64_t)a.qlist[slot] : slot;
#pragma unroll
            for (int s = 0; s < DH; ++s) {
                const int t = h * DH + s;
                b[qb][s] = (row >= 0 && t < a.d) ? -2.f * a.Q[row * a.d + t] : 0.f;
            }
        }

        // This wave's heaps: slots [wave*QW, wave*QW + QW) of every heap level.
        for (int e = lane; e < KP * QW; e += kWave) {
            const int lvl = e / QW, ql = e % QW;
            hk[lvl * QG + wave * QW + ql] = INFINITY;
            hi[lvl * QG + wave * QW + ql] = -1;
        }

        float thr[QB];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) thr[qb] = INFINITY;

        f32x4 an[S4], nn[4];
        auto fetch = [&](int64_t blk, f32x4 (&A)[S4], f32x4 (&N)[4]) {
            const f32x4 *src = a.Ap + blk * (S4 * kWave) + lane;
#pragma unroll
            for (int s4 = 0; s4 < S4; ++s4) A[s4] = src[s4 * kWave];
            const f32x4 *ns = reinterpret_cast<const f32x4 *>(a.Np + blk * 32 + h * 16);
#pragma unroll
            for (int g = 0; g < 4; ++g) N[g] = ns[g];
        };
        if (blk0 < blk1) fetch(blk0, an, nn);

        for (int64_t blk = blk0; blk < blk1; ++blk) {
            f32x4 ac[S4], nc[4];
#pragma unroll
            for (int s4 = 0; s4 < S4; ++s4) ac[s4] = an[s4];
#pragma unroll
            for (int g = 0; g < 4; ++g) nc[g] = nn[g];
            if (blk + 1 < blk1) fetch(blk + 1, an, nn);

            f32x16 init;
#pragma unroll
            for (int v = 0; v < 16; ++v) init[v] = nc[v >> 2][v & 3];
            f32x16 acc[QB];
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) acc[qb] = init;
#pragma unroll
            for (int s4 = 0; s4 < S4; ++s4) {
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int s = 4 * s4 + u;
                    if (s < DH) {
#pragma unroll
                        for (int qb = 0; qb < QB; ++qb)
                            acc[qb] = __builtin_amdgcn_mfma_f32_32x32x2f32(ac[s4][u], b[qb][s], acc[qb], 0, 0, 0);
                    }
                }
            }

            bool hit = false;
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
                float mn = acc[qb][0];
#pragma unroll
                for (int v = 1; v < 16; ++v) mn = fminf(mn, acc[qb][v]);
                hit |= mn < thr[qb];
            }
            if (__ballot(hit) != 0ull) {
                const int ref0 = (int)(blk * 32) + 4 * h;
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) {
                    const int ql = wave * QW + qb * 32 + c;
                    float *hkq = hk + ql;
                    int *hiq = hi + ql;
                    // The two halves of a query share its heap: take turns.
#pragma unroll
                    for (int hh = 0; hh < 2; ++hh) {
                        if (h == hh) {
#pragma unroll
                            for (int v = 0; v < 16; ++v) {
                                const float key = acc[qb][v];
                                if (key < thr[qb] && key < hkq[0]) {
                                    // replace the root (largest kept key) and sift down
                                    const int idx = ref0 + 8 * (v >> 2) + (v & 3);
                                    int pos = 0;
                                    while (true) {
                                        int ch = 2 * pos + 1;
                                        if (ch >= S) break;
                                        float kc = hkq[ch * QG];
                                        if (ch + 1 < S) {
                                            const float k1 = hkq[(ch + 1) * QG];
                                            if (k1 > kc) {
                                                kc = k1;
                                                ++ch;
                                            }
                                        }
                                        if (!(kc > key)) break;
                                        hkq[pos * QG] = kc;
                                        hiq[pos * QG] = hiq[ch * QG];
                                        pos = ch;
                                    }
                                    hkq[pos * QG] = key;
                                    hiq[pos * QG] = idx;
                                    thr[qb] = hkq[0];
                                }
                            }
                        }
                    }
                    thr[qb] = hkq[0];
                }
            }
        }

        // Candidates of this range: lane (c, h) writes slots h, h+2, ... of its queries.
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            const int64_t slot = slot_wave + qb * 32 + c;
            if (slot < nslots) {
                const int ql = wave * QW + qb * 32 + c;
                const int64_t base = (slot * a.P + p) * KP;
                for (int sl = h; sl < S; sl += 2) {
                    a.cand_key[base + sl] = hk[sl * QG + ql];
                    a.cand_idx[base + sl] = hi[sl * QG + ql];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Rerank + certificate: one wave per query slot.  Candidates of all P ranges
// are streamed 64 at a time; the m best (d2, j) are kept sorted across the
// lanes (lane i = i-th smallest) by bitonic sort + merge.
// ---------------------------------------------------------------------------
struct RerankArgs {
    const float *Q;
    int64_t nq;
    const int32_t *qlist;   // optional: slot -> row
    const int32_t *qcount;
    int qcap;
    const float *R;
    int d, k, S, KP, P;
    int self_mode;
    const int32_t *cand_idx;
    const float *cand_key;
    double eps_coef;
    KnnCounters *counters;
    int32_t *flag_out;   // rows that fail the certificate
    int32_t *flag_count;
    int32_t *out_idx;
    float *out_dist;
};

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

// Merge a sorted 64-list (d2, jj) into the running sorted list (rd, rj): keep
// the 64 smallest, sorted.
__device__ __forceinline__ void merge_sorted64(double &rd, int &rj, double d2, int jj, int lane) {
    const double od = __shfl(d2, kWave - 1 - lane, kWave);
    const int oj = __shfl(jj, kWave - 1 - lane, kWave);
    if (lex_before(od, oj, rd, rj)) {
        rd = od;
        rj = oj;
    }
    // (rd, rj) is now bitonic; sort it ascending
#pragma unroll
    for (int stride = kWave >> 1; stride > 0; stride >>= 1) {
        const double xd = __shfl_xor(rd, stride, kWave);
        const int xj = __shfl_xor(rj, stride, kWave);
        const bool lower = (lane & stride) == 0;
        const bool other_first = lex_before(xd, xj, rd, rj);
        if (lower == other_first) {
            rd = xd;
            rj = xj;
        }
    }
}

__global__ __launch_bounds__(256) void k_rerank(RerankArgs a) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t slot = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
    int64_t nslots = a.nq;
    if (a.qlist) nslots = std::min<int64_t>(std::min<int64_t>(*a.qcount, a.qcap), a.nq);
    if (slot >= nslots) return;
    const int64_t row = a.qlist ? (int64_t)a.qlist[slot] : slot;
    const float *x = a.Q + row * a.d;

    // ||x||^2 in float64 (only feeds the certificate's margin)
    double xx = 0.0;
    for (int t = lane; t < a.d; t += kWave) xx += (double)x[t] * (double)x[t];
    xx = wave_sum(xx);
    const float ymax_f = __uint_as_float(a.counters->max_norm_bits);
    const double ym = (double)ymax_f * (1.0 + 1e-6);
    const double eps = a.eps_coef * (2.0 * sqrt(xx) * ym + ym * ym);

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

    double rd = INFINITY;
    int rj = INT_MAX;
    float ratio = 0.f;
    const int total = a.P * a.S;
    for (int c0 = 0; c0 < total; c0 += kWave) {
        const int ci = c0 + lane;
        double d2 = INFINITY;
        int jj = INT_MAX;
        if (ci < total) {
            const int p = ci / a.S, e = ci - (ci / a.S) * a.S;
            const int j = a.cand_idx[cbase + p * a.KP + e];
            if (j >= 0 && !(a.self_mode && j == row)) {
                d2 = exact_d2(x, a.R + (int64_t)j * a.d, a.d);
                jj = j;
                const float key = a.cand_key[cbase + p * a.KP + e];
                ratio = fmaxf(ratio, (float)(fabs((double)key - (d2 - xx)) / eps));
            }
        }
        bitonic_sort64(d2, jj, lane);
        if (c0 == 0) {
            rd = d2;
            rj = jj;
        } else {
            merge_sorted64(rd, rj, d2, jj, lane);
        }
    }
    ratio = wave_max(ratio);
    if (lane == 0 && ratio > 0.f) atomicMax(&a.counters->max_ratio_bits, __float_as_uint(ratio));

    const int m = a.self_mode ? a.k - 1 : a.k;  // neighbours to certify
    bool ok = true;
    if (m > 0 && tau < INFINITY) {
        const double dm = __shfl(rd, m - 1, kWave);
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
    if (lane < m) {
        oi[off + lane] = rj == INT_MAX ? -1 : rj;
        od[off + lane] = (float)sqrt(rd);
    }
    if (!ok && lane == 0) {
        const int pos = atomicAdd(a.flag_count, 1);
        a.flag_out[pos] = (int32_t)row;
    }
}

// ---------------------------------------------------------------------------
// Exhaustive float64 scan of the rows no screen could certify: rows
// list2[0..count2) and list1[cap..count1).  One wave per row; each lane keeps
// a sorted list of its m best in LDS; the lists are merged by m rounds of a
// wave-wide lexicographic minimum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_rescan(const float *__restrict__ Q, const float *__restrict__ R, int64_t nr,
                                               int d, int k, int self_mode, const int32_t *__restrict__ list1,
                                               const int32_t *__restrict__ count1, int cap1,
                                               const int32_t *__restrict__ list2,
                                               const int32_t *__restrict__ count2, int32_t *__restrict__ out_idx,
                                               float *__restrict__ out_dist, KnnCounters *__restrict__ counters) {
    __shared__ double ld[kRescanMax * kWave];
    __shared__ int lj[kRescanMax * kWave];
    const int lane = threadIdx.x;
    const int m = self_mode ? k - 1 : k;
    const int c2 = *count2;
    const int extra = std::max(0, *count1 - cap1);
    const int count = c2 + extra;
    if (blockIdx.x == 0 && lane == 0) counters->rescanned = count;
    for (int f = blockIdx.x; f < count; f += gridDim.x) {
        const int64_t q = f < c2 ? list2[f] : list1[cap1 + (f - c2)];
        const float *x = Q + q * d;
        for (int s = 0; s < m; ++s) {
            ld[s * kWave + lane] = INFINITY;
            lj[s * kWave + lane] = INT_MAX;
        }
        for (int64_t j = lane; j < nr; j += kWave) {
            if (self_mode && j == q) continue;
            const double v = exact_d2(x, R + j * d, d);
            if (m > 0 && lex_before(v, (int)j, ld[(m - 1) * kWave + lane], lj[(m - 1) * kWave + lane])) {
                int p = m - 1;
                while (p > 0 && lex_before(v, (int)j, ld[(p - 1) * kWave + lane], lj[(p - 1) * kWave + lane])) {
                    ld[p * kWave + lane] = ld[(p - 1) * kWave + lane];
                    lj[p * kWave + lane] = lj[(p - 1) * kWave + lane];
                    --p;
                }
                ld[p * kWave + lane] = v;
                lj[p * kWave + lane] = (int)j;
            }
        }
        int head = 0;
        int32_t *oi = out_idx + q * k;
        float *od = out_dist + q * k;
        const int off = self_mode ? 1 : 0;
        if (self_mode && lane == 0) {
            oi[0] = (int32_t)q;
            od[0] = 0.f;
        }
        for (int s = 0; s < m; ++s) {
            double bd = head < m ? ld[head * kWave + lane] : INFINITY;
            int bj = head < m ? lj[head * kWave + lane] : INT_MAX;
            int owner = lane;
            for (int o = 32; o > 0; o >>= 1) {
                const double od2 = __shfl_xor(bd, o, kWave);
                const int oj = __shfl_xor(bj, o, kWave);
                const int oo = __shfl_xor(owner, o, kWave);
                if (lex_before(od2, oj, bd, bj)) {
                    bd = od2;
                    bj = oj;
                    owner = oo;
                }
            }
            if (lane == owner) ++head;
            if (lane == 0) {
                oi[off + s] = bj == INT_MAX ? -1 : bj;
                od[off + s] = (float)sqrt(bd);
            }
        }
    }
}

template <int DH, int QB, int KP>
int launch_screen(const ScreenArgs &a, unsigned gx, const char *name, hipStream_t stream) {
    ScopedTimer timer(name, stream);
    hipLaunchKernelGGL((k_screen_fp32<DH, QB, KP>), dim3(gx, (unsigned)a.P), dim3(256), 0, stream, a);
    return launch_status(name);
}

template <int QB, int KP>
int dispatch_screen(int dh, const ScreenArgs &a, unsigned gx, const char *name, hipStream_t s) {
    switch (dh) {
        case 4: return launch_screen<4, QB, KP>(a, gx, name, s);
        case 8: return launch_screen<8, QB, KP>(a, gx, name, s);
        case 16: return launch_screen<16, QB, KP>(a, gx, name, s);
        case 25: return launch_screen<25, QB, KP>(a, gx, name, s);
        case 32: return launch_screen<32, QB, KP>(a, gx, name, s);
        case 48: return launch_screen<48, 1, KP>(a, gx, name, s);
        case 64: return launch_screen<64, 1, KP>(a, gx, name, s);
        default: set_error("internal: no screen kernel for this dimension"); return RSC_ERR_UNSUPPORTED;
    }
}

int screen(const KnnPlan &p, const ScreenArgs &a, unsigned gx, int kp, const char *name, hipStream_t s) {
    if (kp == 32) return dispatch_screen<2, 32>(p.dh, a, gx, name, s);
    return dispatch_screen<1, 64>(p.dh, a, gx, name, s);
}

int queries_per_group(int dh, int kp) { return kScreenWaves * 32 * ((kp == 32 && dh <= 32) ? 2 : 1); }

int pick_dh(int d) {
    const int half = (d + 1) / 2;
    const int opts[] = {4, 8, 16, 25, 32, 48, 64};
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
        set_error("d > 128 is not supported by this build");
        return RSC_ERR_UNSUPPORTED;
    }
    if (k > kMaxK) {
        set_error("k > 63 is not supported by this build");
        return RSC_ERR_UNSUPPORTED;
    }
    int precision = opts ? opts->precision : RSC_FP32;
    int screen_w = opts ? opts->screen : 0;
    if (precision != RSC_FP32) {
        if (precision == RSC_BF16 || precision == RSC_FP8_E4M3) {
            set_error("reduced-precision screens are not implemented in this build");
            return RSC_ERR_UNSUPPORTED;
        }
        set_error("unknown precision");
        return RSC_ERR_INVALID_ARG;
    }
    if (screen_w == 0) screen_w = k <= 16 ? 32 : 64;
    if (screen_w <= k || screen_w > 64) {
        set_error("screen width must satisfy k < screen <= 64");
        return RSC_ERR_INVALID_ARG;
    }
    plan->nq = nq;
    plan->nr = nr;
    plan->d = d;
    plan->k = k;
    plan->screen = screen_w;
    plan->kp = screen_w <= 32 ? 32 : 64;
    plan->dh = pick_dh(d);
    plan->self_mode = self_mode;
    plan->nblk = (nr + 31) / 32;
    plan->splits = pick_splits(nq, plan->nblk, queries_per_group(plan->dh, plan->kp));
    return RSC_OK;
}

size_t knn_workspace(const KnnPlan &p, void *ws, KnnBuffers *out) {
    Carver cv(ws);
    KnnBuffers b;
    const int dhp4 = ((p.dh + 3) & ~3) / 4;
    const int64_t esc_rows = std::min<int64_t>(p.nq, kEscalateCap);
    b.counters = cv.take<KnnCounters>(1);
    b.packed = cv.take<float>((size_t)p.nblk * dhp4 * kWave * 4);
    b.norms = cv.take<float>((size_t)p.nblk * 32);
    b.cand_idx = cv.take<int32_t>((size_t)p.nq * p.splits * p.kp);
    b.cand_key = cv.take<float>((size_t)p.nq * p.splits * p.kp);
    b.flag1 = cv.take<int32_t>((size_t)std::max<int64_t>(p.nq, 1));
    b.flag2 = cv.take<int32_t>((size_t)std::max<int64_t>(esc_rows, 1));
    b.esc_idx = cv.take<int32_t>((size_t)std::max<int64_t>(esc_rows, 1) * kEscalateSplits * kEscalateWidth);
    b.esc_key = cv.take<float>((size_t)std::max<int64_t>(esc_rows, 1) * kEscalateSplits * kEscalateWidth);
    if (out) *out = b;
    return cv.used;
}

int knn_run(const KnnPlan &p, const float *Q, const float *R, int32_t *out_idx, float *out_dist, void *ws,
            hipStream_t stream) {
    KnnBuffers b;
    knn_workspace(p, ws, &b);
    int st;
    const int dhp4 = ((p.dh + 3) & ~3) / 4;
    {
        ScopedTimer timer("prep_pack", stream);
        hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, stream, b.counters);
        const int64_t tot = p.nblk * dhp4 * kWave;
        const unsigned g1 = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
        hipLaunchKernelGGL(k_pack, dim3(g1), dim3(256), 0, stream, R, p.nr, p.d, p.dh, dhp4, p.nblk,
                           reinterpret_cast<f32x4 *>(b.packed));
        const unsigned g2 = (unsigned)((p.nblk * 32 + 255) / 256);
        hipLaunchKernelGGL(k_pack_norms, dim3(g2), dim3(256), 0, stream, R, p.nr, p.d, p.nblk, b.norms,
                           &b.counters->max_norm_bits);
        if ((st = launch_status("prep_pack")) != RSC_OK) return st;
    }
    if (p.nq == 0) return RSC_OK;

    // Error bound of the float32 key (norm folded into the MFMA sum, norms
    // rounded once from float64): 2 (d + 3) units of roundoff times
    // (2 ||x|| max||y|| + max||y||^2).
    const double eps_coef = 2.0 * (p.d + 3) * std::ldexp(1.0, -24);

    ScreenArgs sa{};
    sa.Q = Q;
    sa.nq = p.nq;
    sa.Ap = reinterpret_cast<const f32x4 *>(b.packed);
    sa.Np = b.norms;
    sa.nblk = p.nblk;
    sa.d = p.d;
    sa.S = p.screen;
    sa.P = p.splits;
    sa.cand_idx = b.cand_idx;
    sa.cand_key = b.cand_key;
    const int qg = queries_per_group(p.dh, p.kp);
    if ((st = screen(p, sa, (unsigned)((p.nq + qg - 1) / qg), p.kp, "screen_fp32", stream)) != RSC_OK) return st;

    RerankArgs ra{};
    ra.Q = Q;
    ra.nq = p.nq;
    ra.R = R;
    ra.d = p.d;
    ra.k = p.k;
    ra.S = p.screen;
    ra.KP = p.kp;
    ra.P = p.splits;
    ra.self_mode = p.self_mode ? 1 : 0;
    ra.cand_idx = b.cand_idx;
    ra.cand_key = b.cand_key;
    ra.eps_coef = eps_coef;
    ra.counters = b.counters;
    ra.flag_out = b.flag1;
    ra.flag_count = &b.counters->flagged;
    ra.out_idx = out_idx;
    ra.out_dist = out_dist;
    {
        ScopedTimer timer("rerank", stream);
        hipLaunchKernelGGL(k_rerank, dim3((unsigned)((p.nq + 3) / 4)), dim3(256), 0, stream, ra);
        if ((st = launch_status("rerank")) != RSC_OK) return st;
    }

    // Escalation: rows that failed, screened again 64 wide over many ranges.
    const int esc_cap = (int)std::min<int64_t>(p.nq, kEscalateCap);
    KnnPlan pe = p;
    pe.screen = kEscalateWidth;
    pe.kp = 64;
    ScreenArgs se = sa;
    se.qlist = b.flag1;
    se.qcount = &b.counters->flagged;
    se.qcap = esc_cap;
    se.S = kEscalateWidth;
    se.P = (int)std::min<int64_t>(kEscalateSplits, std::max<int64_t>(1, p.nblk));
    se.cand_idx = b.esc_idx;
    se.cand_key = b.esc_key;
    const int qge = queries_per_group(p.dh, 64);
    if ((st = screen(pe, se, (unsigned)((esc_cap + qge - 1) / qge), 64, "screen_escalate", stream)) != RSC_OK)
        return st;
    RerankArgs re = ra;
    re.qlist = b.flag1;
    re.qcount = &b.counters->flagged;
    re.qcap = esc_cap;
    re.S = kEscalateWidth;
    re.KP = 64;
    re.P = se.P;
    re.cand_idx = b.esc_idx;
    re.cand_key = b.esc_key;
    re.flag_out = b.flag2;
    re.flag_count = &b.counters->flagged2;
    {
        ScopedTimer timer("rerank_escalate", stream);
        hipLaunchKernelGGL(k_rerank, dim3((unsigned)((esc_cap + 3) / 4)), dim3(256), 0, stream, re);
        if ((st = launch_status("rerank_escalate")) != RSC_OK) return st;
    }
    {
        ScopedTimer timer("rescan", stream);
        hipLaunchKernelGGL(k_rescan, dim3(1024), dim3(64), 0, stream, Q, R, p.nr, p.d, p.k, p.self_mode ? 1 : 0,
                           b.flag1, &b.counters->flagged, esc_cap, b.flag2, &b.counters->flagged2, out_idx,
                           out_dist, b.counters);
        if ((st = launch_status("rescan")) != RSC_OK) return st;
    }
    return RSC_OK;
}

}  // namespace rsc
