// Device pieces shared by the FP32 and the reduced-precision screens.
#pragma once

#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>
#include <cstdint>

namespace rsc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace scr {

constexpr int kWave = 64;
constexpr int kScreenWaves = 4;  // waves per screen workgroup
constexpr int kQueueCap = 16;    // default queue entries per lane and query block (a block adds at most 16)

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

__device__ __forceinline__ int wave_max_int(int v) {
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, kWave));
    return v;
}

// Arguments of a screen launch.  Query slot i of the launch is row i, or
// row qlist[i] for i < min(*qcount, qcap) when a list is given.
// Output: cand[(slot * 2P + 2p + h) * L + i] = i-th smallest key of
// contraction half h of reference range p (index -1 / key +inf where fewer
// than L were seen).
struct ScreenArgs {
    const float *Q;
    int64_t nq;
    const int32_t *qlist;   // optional gather list
    const int32_t *qcount;  // its device-side length
    int qcap;
    const void *Ap;         // packed references (layout depends on the precision)
    const float *Np;        // norms in accumulator order, where the layout needs them
    const float *qscale;    // per-dimension query scales (FP8 screen)
    const int32_t *blk_part;  // FP8 residual variant: partition of each packed block (4 copies per block)
    const float *cent;        // FP8 residual variant: partition centroids
    int64_t nblk;
    int d;
    int P;                  // reference ranges (gridDim.y)
    int rotate;             // reduced-precision screens on one matrix whose references are packed in the
                            // queries' order: each query group starts its scan at its own block
    int32_t *cand_idx;
    float *cand_key;
};

__device__ __forceinline__ int64_t screen_slots(const ScreenArgs &a) {
    if (!a.qlist) return a.nq;
    const int64_t cnt = *a.qcount;
    const int64_t m = cnt < a.qcap ? cnt : a.qcap;
    return m < a.nq ? m : a.nq;
}

// The L smallest keys (and their reference indices) one lane has seen, kept
// sorted in registers, plus this lane's queue of keys that beat the
// threshold of the last merge.  Keys enter the queue with one LDS write; all
// lanes of the wave merge their queues together when any queue could
// overflow, so the per-key cost stays a compare in the common case.
template <int L, int QCAP = kQueueCap>
struct LaneTopK {
    float lk[L];
    int li[L];
    float thr;  // lk[L-1] as of the last merge
    int count;  // queued entries

    __device__ __forceinline__ void init() {
#pragma unroll
        for (int i = 0; i < L; ++i) {
            lk[i] = INFINITY;
            li[i] = -1;
        }
        thr = INFINITY;
        count = 0;
    }

    // Unrolled compare-and-shift insertion that drops the largest entry.
    __device__ __forceinline__ void insert(float key, int idx) {
#pragma unroll
        for (int i = L - 1; i > 0; --i) {
            const bool shift = key < lk[i - 1];
            const bool here = key < lk[i];
            lk[i] = shift ? lk[i - 1] : (here ? key : lk[i]);
            li[i] = shift ? li[i - 1] : (here ? idx : li[i]);
        }
        if (key < lk[0]) {
            lk[0] = key;
            li[0] = idx;
        }
    }

    // queue entry e of this lane lives at q[e * stride]
    __device__ __forceinline__ void flush(const float2 *q, int stride) {
        const int maxc = wave_max_int(count);
        for (int e = 0; e < maxc; ++e) {
            if (e < count) {
                const float2 v = q[e * stride];
                if (v.x < lk[L - 1]) insert(v.x, __float_as_int(v.y));
            }
        }
        count = 0;
        thr = lk[L - 1];
    }

    // Offer the 16 keys of one 32x32 output block (register v holds
    // reference ref0 + 8 (v/4) + (v%4)).
    __device__ __forceinline__ void offer(const f32x16 &acc, int ref0, float2 *q, int stride) {
        float mn = acc[0];
#pragma unroll
        for (int v = 1; v < 16; ++v) mn = fminf(mn, acc[v]);
        if (__ballot(mn < thr) == 0ull) return;
        int hits = 0;
#pragma unroll
        for (int v = 0; v < 16; ++v) hits += acc[v] < thr ? 1 : 0;
        if (__ballot(count + hits > QCAP) != 0ull) {
            flush(q, stride);
            if constexpr (QCAP < 16) {
                hits = 0;
#pragma unroll
                for (int v = 0; v < 16; ++v) hits += acc[v] < thr ? 1 : 0;
                if (__ballot(hits > QCAP) != 0ull) {
                    // more keys than a queue holds (only while the lists fill up): insert directly
#pragma unroll
                    for (int v = 0; v < 16; ++v)
                        if (acc[v] < lk[L - 1]) insert(acc[v], ref0 + 8 * (v >> 2) + (v & 3));
                    thr = lk[L - 1];
                    return;
                }
            }
        }
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            if (acc[v] < thr) {
                q[count * stride] = make_float2(acc[v], __int_as_float(ref0 + 8 * (v >> 2) + (v & 3)));
                ++count;
            }
        }
    }

    __device__ __forceinline__ void store(const ScreenArgs &a, int64_t slot, int p, int h) const {
        const int64_t base = ((slot * a.P + p) * 2 + h) * L;
#pragma unroll
        for (int i = 0; i < L; ++i) {
            a.cand_key[base + i] = lk[i];
            a.cand_idx[base + i] = li[i];
        }
    }
};

}  // namespace scr
}  // namespace rsc
