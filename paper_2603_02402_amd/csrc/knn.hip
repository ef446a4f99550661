// Exact kNN on gfx950: MFMA distance screen + float64 rerank + certificate.
//
// The paper's neighbour step needs, per cell, the k nearest cells of the
// PCA embedding under the squared Euclidean distance of Methods, "Custom
// GPU kernels" (d_ij = ||x_i - x_j||^2).  The work is a dense contraction
// (2 d flops per ordered pair), so the screen runs on the matrix cores:
//
//   key_ij = ||y_j||^2 - 2 x_i . y_j      (= d_ij - ||x_i||^2, same order per row)
//
// with the query tile resident in VGPRs for the whole launch, reference
// tiles streamed HBM/L2 -> LDS (double buffered), one
// v_mfma_f32_32x32x2_f32 per pair of contraction indices, and a per-query
// max-heap of the S smallest keys kept in LDS.  A query's two lanes (one
// per contraction half) own disjoint halves of every 32x32 output block;
// the common case (no key below the heap root) costs one add and one
// compare per pair.
//
// The float32 screen is not the answer: its rounding error is bounded and
// every query's S candidates are re-ranked with float64 distances summed
// from direct differences in dimension order.  A row is certified exact
// when its (k-1)-th re-ranked distance is below the smallest key the screen
// could have rejected, minus the error bound; other rows are recomputed by
// an exhaustive float64 scan.  Ties are broken towards the lower index.

#include <hip/hip_runtime.h>

#include <cfloat>
#include <climits>
#include <cmath>

#include "rsc_internal.hpp"

namespace rsc {

typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

namespace {

constexpr int kWave = 64;
constexpr int kScreenWaves = 4;  // waves per screen workgroup
constexpr int kMaxD = 128;
constexpr int kMaxK = 63;
constexpr int kRescanMax = 64;  // list capacity of the exhaustive rescan

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

// ---------------------------------------------------------------------------
// Prep: float32 squared norms of the reference rows and the largest norm.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_row_norms(const float *__restrict__ X, int64_t n, int d,
                                                   float *__restrict__ norms, uint32_t *__restrict__ max_norm_bits) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    float s = 0.f;
    if (i < n) {
        const float *x = X + i * d;
        for (int t = 0; t < d; ++t) s = fmaf(x[t], x[t], s);
        norms[i] = s;
    }
    float m = wave_max(i < n ? sqrtf(s) : 0.f);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicMax(max_norm_bits, __float_as_uint(m));
}

__global__ void k_init_counters(KnnCounters *c) {
    if (threadIdx.x == 0) {
        c->flagged = 0;
        c->max_ratio_bits = 0u;
        c->max_norm_bits = 0u;
        c->pad = 0;
    }
}

// ---------------------------------------------------------------------------
// Screen.
//
// Workgroup = 4 waves; wave w owns QB blocks of 32 queries.  Lane l handles
// query column c = l % 32 of every block and contraction half h = l / 32:
// dimension h*DH + s feeds MFMA step s.  Output register v of a 32x32 block
// holds reference row 8*(v/4) + 4*h + (v%4) of the current 32-row block.
// ---------------------------------------------------------------------------
template <int DH, int QB, int KP>
struct ScreenCfg {
    static constexpr int RB = 1;                       // 32-row reference blocks per tile
    static constexpr int TR = RB * 32;                 // reference rows per tile
    static constexpr int QW = QB * 32;                 // queries per wave
    static constexpr int QG = kScreenWaves * QW;       // queries per workgroup
    static constexpr int DHP = (DH + 3) & ~3;          // padded half width (16-byte rows)
    static constexpr int RS0 = 2 * DHP;
    static constexpr int RS = ((RS0 / 4) % 2 == 0) ? RS0 + 4 : RS0;  // LDS row stride (floats)
    static constexpr int PF = (TR * 2 * DH + 255) / 256;             // prefetch registers per thread
};

template <int DH, int QB, int KP>
__global__ __launch_bounds__(256, 2) void k_screen_fp32(const float *__restrict__ Q, int64_t nq,
                                                         const float *__restrict__ R, int64_t nr, int d,
                                                         const float *__restrict__ rnorm, int S,
                                                         int32_t *__restrict__ cand_idx,
                                                         float *__restrict__ cand_key) {
    using C = ScreenCfg<DH, QB, KP>;
    constexpr int TR = C::TR, RS = C::RS, DHP = C::DHP, QG = C::QG, QW = C::QW, PF = C::PF;

    __shared__ __attribute__((aligned(16))) float sA[2][TR * RS];
    __shared__ __attribute__((aligned(16))) float sN[2][TR];
    __shared__ float hk[KP * QG];
    __shared__ int hi[KP * QG];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const int h = lane >> 5, c = lane & 31;
    const int64_t q_wave = (int64_t)blockIdx.x * QG + wave * QW;

    // Query operand, resident for the whole launch; -2 folded in (exact).
    float b[QB][DH];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const int64_t q = q_wave + qb * 32 + c;
#pragma unroll
        for (int s = 0; s < DH; ++s) {
            const int t = h * DH + s;
            b[qb][s] = (q < nq && t < d) ? -2.f * Q[q * d + t] : 0.f;
        }
    }

    for (int e = tid; e < KP * QG; e += 256) {
        hk[e] = INFINITY;
        hi[e] = -1;
    }
    for (int e = tid; e < 2 * TR * RS; e += 256) (&sA[0][0])[e] = 0.f;

    const int64_t T = (nr + TR - 1) / TR;
    const int tile_elems = TR * d;
    const int step_r = 256 / d, step_t = 256 % d;

    // Prefetch a tile into registers: element e = tid + 256 m of the tile's
    // contiguous TR x d block.
    float pf[PF];
    auto load_tile = [&](int64_t t) {
        const int64_t base_row = t * TR;
        const float *src = R + base_row * d;
        const int64_t rows_left = nr - base_row;
        int r = tid / d, tt = tid - (tid / d) * d;
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int e = tid + 256 * m;
            float v = 0.f;
            if (e < tile_elems && r < rows_left) v = src[e];
            pf[m] = v;
            r += step_r;
            tt += step_t;
            if (tt >= d) {
                tt -= d;
                ++r;
            }
        }
    };
    auto store_tile = [&](int64_t t, int buf) {
        int r = tid / d, tt = tid - (tid / d) * d;
#pragma unroll
        for (int m = 0; m < PF; ++m) {
            const int e = tid + 256 * m;
            if (e < tile_elems) {
                const int col = tt < DH ? tt : DHP + (tt - DH);
                sA[buf][r * RS + col] = pf[m];
            }
            r += step_r;
            tt += step_t;
            if (tt >= d) {
                tt -= d;
                ++r;
            }
        }
        if (tid < TR) {
            const int64_t row = t * TR + tid;
            sN[buf][tid] = row < nr ? rnorm[row] : INFINITY;
        }
    };

    __syncthreads();  // pad zeroing done before the first tile lands
    load_tile(0);
    store_tile(0, 0);
    __syncthreads();

    float thr[QB];
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) thr[qb] = INFINITY;

    for (int64_t t = 0; t < T; ++t) {
        const int cur = (int)(t & 1);
        if (t + 1 < T) load_tile(t + 1);

#pragma unroll
        for (int rb = 0; rb < C::RB; ++rb) {
            f32x16 acc[QB];
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) acc[qb] = f32x16{};
            const float *arow = &sA[cur][(rb * 32 + c) * RS + h * DHP];
#pragma unroll
            for (int s4 = 0; s4 < DHP / 4; ++s4) {
                const f32x4 a4 = *reinterpret_cast<const f32x4 *>(arow + 4 * s4);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int s = 4 * s4 + u;
                    if (s < DH) {
#pragma unroll
                        for (int qb = 0; qb < QB; ++qb)
                            acc[qb] = __builtin_amdgcn_mfma_f32_32x32x2f32(a4[u], b[qb][s], acc[qb], 0, 0, 0);
                    }
                }
            }
            // keys = ||y||^2 + acc; the lane's 16 reference rows come in 4 groups of 4
            f32x4 nv[4];
#pragma unroll
            for (int g = 0; g < 4; ++g)
                nv[g] = *reinterpret_cast<const f32x4 *>(&sN[cur][rb * 32 + 8 * g + 4 * h]);
            bool hit = false;
#pragma unroll
            for (int qb = 0; qb < QB; ++qb) {
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    acc[qb][v] = acc[qb][v] + nv[v >> 2][v & 3];
                    hit |= acc[qb][v] < thr[qb];
                }
            }
            if (__ballot(hit) != 0ull) {
                const int ref0 = (int)(t * TR) + rb * 32 + 4 * h;
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
                                    int p = 0;
                                    while (true) {
                                        int ch = 2 * p + 1;
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
                                        hkq[p * QG] = kc;
                                        hiq[p * QG] = hiq[ch * QG];
                                        p = ch;
                                    }
                                    hkq[p * QG] = key;
                                    hiq[p * QG] = idx;
                                    thr[qb] = hkq[0];
                                }
                            }
                        }
                    }
                    thr[qb] = hkq[0];
                }
            }
        }

        if (t + 1 < T) store_tile(t + 1, cur ^ 1);
        __syncthreads();
    }

    // Write the candidates: lane (c, h) writes slots h, h+2, ... of its queries.
#pragma unroll
    for (int qb = 0; qb < QB; ++qb) {
        const int64_t q = q_wave + qb * 32 + c;
        if (q < nq) {
            const int ql = wave * QW + qb * 32 + c;
            for (int sl = h; sl < S; sl += 2) {
                cand_key[q * KP + sl] = hk[sl * QG + ql];
                cand_idx[q * KP + sl] = hi[sl * QG + ql];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Rerank + certificate: one wave per query, lane e handles candidate e.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_rerank(const float *__restrict__ Q, int64_t nq,
                                                const float *__restrict__ R, int d, int k, int S, int KP,
                                                int self_mode, const int32_t *__restrict__ cand_idx,
                                                const float *__restrict__ cand_key, double eps_coef,
                                                KnnCounters *__restrict__ counters, int32_t *__restrict__ flag_list,
                                                int32_t *__restrict__ out_idx, float *__restrict__ out_dist) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t q = (int64_t)blockIdx.x * (blockDim.x / kWave) + (threadIdx.x >> 6);
    if (q >= nq) return;
    const float *x = Q + q * d;

    int j = -1;
    float key = INFINITY;
    if (lane < S) {
        j = cand_idx[q * KP + lane];
        key = cand_key[q * KP + lane];
    }
    const bool slot_empty = (lane < S) && (j < 0);
    const bool heap_full = __ballot(slot_empty) == 0ull;
    const bool valid = (j >= 0) && !(self_mode && j == q);
    double d2 = INFINITY;
    int jj = INT_MAX;
    if (valid) {
        d2 = exact_d2(x, R + (int64_t)j * d, d);
        jj = j;
    }

    // ||x||^2 in float64 (only feeds the certificate's margin)
    double xx = 0.0;
    for (int t = lane; t < d; t += kWave) xx += (double)x[t] * (double)x[t];
    xx = wave_sum(xx);

    // Certificate bound on |screened key - exact key| for this query.
    const float ymax_f = __uint_as_float(counters->max_norm_bits);
    const double ym = (double)ymax_f * (1.0 + 1e-5);
    const double eps = eps_coef * (2.0 * sqrt(xx) * ym + ym * ym);

    // Largest kept key (the heap root) and the largest observed error ratio.
    const float tau = wave_max(lane < S ? key : -INFINITY);
    float ratio = 0.f;
    if (valid) ratio = (float)(fabs((double)key - (d2 - xx)) / eps);
    ratio = wave_max(ratio);
    if (lane == 0 && ratio > 0.f) atomicMax(&counters->max_ratio_bits, __float_as_uint(ratio));

    // Bitonic sort of (d2, jj) ascending across the wave.
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

    const int m = self_mode ? k - 1 : k;  // neighbours to certify
    bool ok = true;
    if (m > 0 && heap_full) {
        const double dm = __shfl(d2, m - 1, kWave);
        const double bound = (double)tau + xx - eps - 1e-12 * (fabs((double)tau) + xx);
        ok = dm < bound;
    }

    int32_t *oi = out_idx + q * k;
    float *od = out_dist + q * k;
    if (self_mode) {
        if (lane == 0) {
            oi[0] = (int32_t)q;
            od[0] = 0.f;
        }
        if (lane < k - 1) {
            oi[1 + lane] = jj == INT_MAX ? -1 : jj;
            od[1 + lane] = (float)sqrt(d2);
        }
    } else if (lane < k) {
        oi[lane] = jj == INT_MAX ? -1 : jj;
        od[lane] = (float)sqrt(d2);
    }
    if (!ok && lane == 0) {
        const int pos = atomicAdd(&counters->flagged, 1);
        flag_list[pos] = (int32_t)q;
    }
}

// ---------------------------------------------------------------------------
// Exhaustive float64 rescan of the rows whose certificate failed.
// One wave per row, grid-stride over the flagged list.  Each lane keeps a
// sorted list of its m best (d2, j) in LDS; the lists are merged by m
// rounds of a wave-wide lexicographic minimum.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_rescan(const float *__restrict__ Q, const float *__restrict__ R, int64_t nr,
                                               int d, int k, int self_mode,
                                               const KnnCounters *__restrict__ counters,
                                               const int32_t *__restrict__ flag_list, int32_t *__restrict__ out_idx,
                                               float *__restrict__ out_dist) {
    __shared__ double ld[kRescanMax * kWave];
    __shared__ int lj[kRescanMax * kWave];
    const int lane = threadIdx.x;
    const int m = self_mode ? k - 1 : k;
    const int count = counters->flagged;
    for (int f = blockIdx.x; f < count; f += gridDim.x) {
        const int64_t q = flag_list[f];
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
int launch_screen(const KnnPlan &p, const float *Q, const float *R, const float *norms, int32_t *cand_idx,
                  float *cand_key, hipStream_t stream) {
    using C = ScreenCfg<DH, QB, KP>;
    const int64_t grid = (p.nq + C::QG - 1) / C::QG;
    ScopedTimer timer("screen_fp32", stream);
    hipLaunchKernelGGL((k_screen_fp32<DH, QB, KP>), dim3((unsigned)grid), dim3(256), 0, stream, Q, p.nq, R, p.nr,
                       p.d, norms, p.screen, cand_idx, cand_key);
    return launch_status("screen_fp32");
}

template <int KP>
int dispatch_screen(const KnnPlan &p, const float *Q, const float *R, const float *norms, int32_t *ci, float *ck,
                    hipStream_t s) {
    constexpr int QB = KP == 64 ? 1 : 2;
    switch (p.dh) {
        case 4: return launch_screen<4, QB, KP>(p, Q, R, norms, ci, ck, s);
        case 8: return launch_screen<8, QB, KP>(p, Q, R, norms, ci, ck, s);
        case 16: return launch_screen<16, QB, KP>(p, Q, R, norms, ci, ck, s);
        case 25: return launch_screen<25, QB, KP>(p, Q, R, norms, ci, ck, s);
        case 32: return launch_screen<32, QB, KP>(p, Q, R, norms, ci, ck, s);
        case 48: return launch_screen<48, 1, KP>(p, Q, R, norms, ci, ck, s);
        case 64: return launch_screen<64, 1, KP>(p, Q, R, norms, ci, ck, s);
        default: set_error("internal: no screen kernel for this dimension"); return RSC_ERR_UNSUPPORTED;
    }
}

int pick_dh(int d) {
    const int half = (d + 1) / 2;
    const int opts[] = {4, 8, 16, 25, 32, 48, 64};
    for (int o : opts)
        if (half <= o) return o;
    return -1;
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
    int screen = opts ? opts->screen : 0;
    if (precision != RSC_FP32) {
        if (precision == RSC_BF16 || precision == RSC_FP8_E4M3) {
            set_error("reduced-precision screens are not implemented in this build");
            return RSC_ERR_UNSUPPORTED;
        }
        set_error("unknown precision");
        return RSC_ERR_INVALID_ARG;
    }
    if (screen == 0) screen = k <= 16 ? 32 : 64;
    if (screen <= k || screen > 64) {
        set_error("screen width must satisfy k < screen <= 64");
        return RSC_ERR_INVALID_ARG;
    }
    plan->nq = nq;
    plan->nr = nr;
    plan->d = d;
    plan->k = k;
    plan->screen = screen;
    plan->kp = screen <= 32 ? 32 : 64;
    plan->dh = pick_dh(d);
    plan->self_mode = self_mode;
    return RSC_OK;
}

size_t knn_workspace(const KnnPlan &p, void *ws, KnnCounters **counters, float **norms, int32_t **cand_idx,
                     float **cand_key, int32_t **flag_list) {
    Carver cv(ws);
    KnnCounters *c = cv.take<KnnCounters>(1);
    float *nrm = cv.take<float>((size_t)p.nr);
    int32_t *ci = cv.take<int32_t>((size_t)p.nq * p.kp);
    float *ck = cv.take<float>((size_t)p.nq * p.kp);
    int32_t *fl = cv.take<int32_t>((size_t)(p.nq > 0 ? p.nq : 1));
    if (counters) *counters = c;
    if (norms) *norms = nrm;
    if (cand_idx) *cand_idx = ci;
    if (cand_key) *cand_key = ck;
    if (flag_list) *flag_list = fl;
    return cv.used;
}

int knn_run(const KnnPlan &p, const float *Q, const float *R, int32_t *out_idx, float *out_dist, void *ws,
            hipStream_t stream) {
    KnnCounters *counters;
    float *norms, *cand_key;
    int32_t *cand_idx, *flag_list;
    knn_workspace(p, ws, &counters, &norms, &cand_idx, &cand_key, &flag_list);
    int st;
    {
        ScopedTimer timer("prep_norms", stream);
        hipLaunchKernelGGL(k_init_counters, dim3(1), dim3(64), 0, stream, counters);
        if ((st = launch_status("init_counters")) != RSC_OK) return st;
        const unsigned g = (unsigned)((p.nr + 255) / 256);
        hipLaunchKernelGGL(k_row_norms, dim3(g), dim3(256), 0, stream, R, p.nr, p.d, norms,
                           &counters->max_norm_bits);
        if ((st = launch_status("row_norms")) != RSC_OK) return st;
    }
    if (p.nq == 0) return RSC_OK;
    st = p.kp == 32 ? dispatch_screen<32>(p, Q, R, norms, cand_idx, cand_key, stream)
                    : dispatch_screen<64>(p, Q, R, norms, cand_idx, cand_key, stream);
    if (st != RSC_OK) return st;
    {
        // Error bound of the float32 key: 4 (d + 2) units of roundoff times
        // (2 ||x|| max||y|| + max||y||^2); see the derivation in the notes.
        const double u = std::ldexp(1.0, -24);
        const double eps_coef = 4.0 * (p.d + 2) * u;
        ScopedTimer timer("rerank", stream);
        const unsigned g = (unsigned)((p.nq + 3) / 4);
        hipLaunchKernelGGL(k_rerank, dim3(g), dim3(256), 0, stream, Q, p.nq, R, p.d, p.k, p.screen, p.kp,
                           p.self_mode ? 1 : 0, cand_idx, cand_key, eps_coef, counters, flag_list, out_idx,
                           out_dist);
        if ((st = launch_status("rerank")) != RSC_OK) return st;
    }
    {
        ScopedTimer timer("rescan", stream);
        hipLaunchKernelGGL(k_rescan, dim3(1024), dim3(64), 0, stream, Q, R, p.nr, p.d, p.k, p.self_mode ? 1 : 0,
                           counters, flag_list, out_idx, out_dist);
        if ((st = launch_status("rescan")) != RSC_OK) return st;
    }
    return RSC_OK;
}

}  // namespace rsc
