// Reduced-precision distance screens (BF16, FP8-e4m3) on gfx950 MFMA.
//
// The precision form of the neighbour search: the distance contraction runs
// in BF16 (v_mfma_f32_32x32x16_bf16) or in OCP FP8-e4m3 with per-dimension
// scaling (v_mfma_scale_f32_32x32x64_f8f6f4, unit block scales), always
// accumulating in FP32.  Each query keeps its 64 smallest screened keys (32
// per contraction half), which are then re-ranked with float64 distances of
// the original float32 data by the same rerank kernel as the exact path.
// No certificate is attempted: the result is approximate by design and is
// measured by recall@k and distance error against exact search.
//
// Keys are ||y~||^2 - 2 x~ . y~ where y~, x~ are the rounded vectors, so the
// screen ranks by the exact distance between the rounded points:
//   BF16: the squared norm of the BF16-rounded reference, split into a BF16
//         high part and a BF16 low part that ride in two spare contraction
//         slots (the query side holds 1.0 there), so the MFMA chain yields
//         the key and the padding to a multiple of 16 costs nothing extra;
//   FP8:  reference codes q(y_t / s_t) with s_t = absmax_t / 448 (round to
//         nearest even, saturating at 448), query codes q(-2 G x_t s_t) with a
//         power-of-two G that fills the e4m3 range; the dequantised norm
//         G ||s . q(y/s)||^2 is the accumulator's initial value, so the chain
//         yields G times the key (same order).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "rsc_internal.hpp"
#include "screen_common.hpp"

namespace rsc {

namespace {

using namespace scr;

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef int i32x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr float kFp8Max = 448.f;  // largest finite e4m3 (OCP "fn") value
constexpr int kLowpQB = 1;        // query blocks (of 32) per wave

// float32 -> bfloat16 bits, round to nearest even (finite inputs; inf kept).
__device__ inline uint32_t bf16_bits(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return u >> 16;  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return u >> 16;
}
__device__ inline float bf16_value(uint32_t b) { return __uint_as_float(b << 16); }

// float32 -> OCP e4m3 ("fn": no infinities, 0x7f / 0xff are NaN) code,
// round to nearest even, saturating to +-448.
__device__ inline uint32_t e4m3_code(float x) {
    const uint32_t sign = (__float_as_uint(x) >> 24) & 0x80u;
    const float a = fabsf(x);
    if (!(a < kFp8Max)) return sign | 0x7eu;  // saturate (also catches inf)
    const uint32_t bits = __float_as_uint(a);
    const int e = (int)((bits >> 23) & 0xff) - 127;
    if (e < -6) {
        // subnormal range: multiples of 2^-9; rintf is round-half-even
        const uint32_t m = (uint32_t)rintf(a * 512.f);  // 0..8; 8 is the smallest normal
        return sign | m;
    }
    uint32_t mant = bits & 0x7fffffu;
    uint32_t r = mant >> 20;
    const uint32_t rem = mant & 0xfffffu;
    if (rem > 0x80000u || (rem == 0x80000u && (r & 1u))) ++r;
    int ee = e + 7;
    if (r == 8) {
        r = 0;
        ++ee;
    }
    uint32_t code = ((uint32_t)ee << 3) | r;
    if (code > 0x7eu) code = 0x7eu;
    return sign | code;
}

__device__ inline float e4m3_value(uint32_t code) {
    const float s = (code & 0x80u) ? -1.f : 1.f;
    const uint32_t e = (code >> 3) & 0xfu, m = code & 7u;
    if (e == 0) return s * (float)m * (1.f / 512.f);
    return s * ldexpf(1.f + (float)m * 0.125f, (int)e - 7);
}

// ---------------------------------------------------------------------------
// BF16 packing.  Block b, step s, lane (c, h): 8 bf16 for contraction index
// kk = 16 s + 8 h + e: dimension kk < d; kk == d: high part of the norm of
// the rounded row; kk == d + 1: its low part; 0 elsewhere.  Past the last
// row: 0, and +inf as the norm's high part.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_pack_bf16(const float *__restrict__ R, int64_t nr, int d, int KS,
                                                   int64_t nblk, const int32_t *__restrict__ rmap,
                                                   i32x4 *__restrict__ Ap) {
    const int64_t total = nblk * KS * kWave;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(e % kWave);
        const int64_t bs = e / kWave;
        const int s = (int)(bs % KS);
        const int64_t b = bs / KS;
        const int64_t slot = 32 * b + (lane & 31);
        const int64_t row = slot < nr && rmap ? (int64_t)rmap[slot] : slot;  // packed slot -> row
        const int h = lane >> 5;
        const int k0 = 16 * s + 8 * h;
        float nhi = 0.f, nlo = 0.f;
        if (k0 <= d + 1 && k0 + 8 > d) {  // this group holds a norm slot
            if (slot < nr) {
                double n = 0.0;
                for (int t = 0; t < d; ++t) {
                    const double v = bf16_value(bf16_bits(R[row * d + t]));
                    n += v * v;
                }
                const float nf = (float)n;
                nhi = bf16_value(bf16_bits(nf));
                nlo = bf16_value(bf16_bits(nf - nhi));
            } else {
                nhi = INFINITY;
            }
        }
        uint32_t w[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
            uint32_t two = 0;
#pragma unroll
            for (int q = 0; q < 2; ++q) {
                const int kk = k0 + 2 * p + q;
                float v = 0.f;
                if (kk < d) {
                    if (slot < nr) v = R[row * d + kk];
                } else if (kk == d) {
                    v = nhi;
                } else if (kk == d + 1) {
                    v = nlo;
                }
                two |= bf16_bits(v) << (16 * q);
            }
            w[p] = two;
        }
        Ap[e] = i32x4{(int)w[0], (int)w[1], (int)w[2], (int)w[3]};
    }
}

__global__ void k_fill_u32(uint32_t *p, int n, uint32_t v) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = v;
}

// ---------------------------------------------------------------------------
// FP8 scaling and packing.
// ---------------------------------------------------------------------------
// Per-dimension max |x| over the rows of X (float bits, atomic max).
__global__ __launch_bounds__(256) void k_absmax(const float *__restrict__ X, int64_t n, int d,
                                                uint32_t *__restrict__ amax_bits) {
    __shared__ uint32_t local[128];
    for (int t = threadIdx.x; t < d; t += blockDim.x) local[t] = 0u;
    __syncthreads();
    const int64_t total = n * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int t = (int)(e % d);
        atomicMax(&local[t], __float_as_uint(fabsf(X[e])));
    }
    __syncthreads();
    for (int t = threadIdx.x; t < d; t += blockDim.x) atomicMax(&amax_bits[t], local[t]);
}

// scal[0..d): reference scale s_t = absmax_t / 448 (1 for an all-zero
// dimension); scal[d..2d): query multiplier -2 G s_t; scal[2d]: G.
__global__ void k_fp8_scales(const uint32_t *__restrict__ amax_r, const uint32_t *__restrict__ amax_q, int d,
                             float *__restrict__ scal) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float m = 0.f;
    for (int t = 0; t < d; ++t) {
        const float ar = __uint_as_float(amax_r[t]);
        const float s = ar > 0.f ? ar / kFp8Max : 1.f;
        scal[t] = s;
        m = fmaxf(m, 2.f * __uint_as_float(amax_q[t]) * s);
    }
    float G = 1.f;
    if (m > 0.f) G = ldexpf(1.f, (int)floorf(log2f(kFp8Max / m)));
    for (int t = 0; t < d; ++t) scal[d + t] = -2.f * G * scal[t];
    scal[2 * d] = G;
}

// Block b, step s, lane (c, h): 32 e4m3 codes for kk = 64 s + 32 h + e
// (dimension kk < d, else 0), stored as two 16-byte halves 1 KiB apart
// (codes 0..15 of every lane, then codes 16..31), so that a wave reads
// each half with one conflict-free 16-byte load per lane.  Norms:
// G ||s . q(y/s)||^2 in accumulator order (+inf past the last row).
__global__ __launch_bounds__(256) void k_pack_fp8(const float *__restrict__ R, int64_t nr, int d, int KS,
                                                  int64_t nblk, const float *__restrict__ scal,
                                                  const int32_t *__restrict__ rmap, i32x4 *__restrict__ Ap,
                                                  float *__restrict__ Np) {
    const int64_t total = nblk * KS * kWave;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(e % kWave);
        const int64_t bs = e / kWave;
        const int s = (int)(bs % KS);
        const int64_t b = bs / KS;
        const int64_t slot = 32 * b + (lane & 31);
        const int64_t row = slot < nr && rmap ? (int64_t)rmap[slot] : slot;  // packed slot -> row
        const int h = lane >> 5;
        const int k0 = 64 * s + 32 * h;
        i32x8 w;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            uint32_t four = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = k0 + 4 * p + q;
                uint32_t code = 0;
                if (kk < d && slot < nr) code = e4m3_code(R[row * d + kk] / scal[kk]);
                four |= code << (8 * q);
            }
            w[p] = (int)four;
        }
        // e = (b KS + s) 64 + lane: halves at 2 (b KS + s) 64 + {0, 64} + lane
        Ap[2 * bs * kWave + lane] = i32x4{w[0], w[1], w[2], w[3]};
        Ap[2 * bs * kWave + kWave + lane] = i32x4{w[4], w[5], w[6], w[7]};
        if (s == 0 && h == 0) {
            float out = INFINITY;
            if (slot < nr) {
                double n = 0.0;
                for (int t = 0; t < d; ++t) {
                    const double v = (double)e4m3_value(e4m3_code(R[row * d + t] / scal[t])) * scal[t];
                    n += v * v;
                }
                out = (float)(n * scal[2 * d]);
            }
            const int i = lane & 31;
            const int g = i >> 3, hh = (i >> 2) & 1, j = i & 3;
            Np[b * 32 + hh * 16 + 4 * g + j] = out;
        }
    }
}

// ---------------------------------------------------------------------------
// FP8 residual variant.  The references are split into k-means partitions
// and packed partition by partition (a partition's last block padded, map[]
// turning a packed row back into a row id); each reference is stored as the
// e4m3 code of its residual y - c_p, scaled per dimension by the absmax of
// the residuals.  A query is coded against each partition it meets, as
// q = x - c_p: the screen recomputes its codes when the wave's block moves
// to another partition.  With both sides relative to c_p the key is
// G (|q|^2 + |r~|^2 - 2 q~ . r~) = G |x - y~|^2: |r~|^2 (the dequantised
// residual's norm) is packed with the codes and |q|^2 is added per lane.
// ---------------------------------------------------------------------------
__global__ void k_resid_init_rows(int32_t *__restrict__ init, int P, int64_t n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < P; i += gridDim.x * blockDim.x)
        init[i] = (int32_t)(((int64_t)i * n) / P);
}

// Block offsets of the partitions (each padded to whole blocks) and the
// partition of every packed block (blocks past the last partition: P - 1),
// stored four times per block so that one 16-byte load brings it into LDS.
__global__ __launch_bounds__(1024) void k_resid_blocks(const int64_t *__restrict__ poff, int P, int64_t nblk,
                                                       int64_t *__restrict__ pblk, int32_t *__restrict__ blk_part) {
    if (threadIdx.x == 0) {
        int64_t b = 0;
        for (int p = 0; p < P; ++p) {
            pblk[p] = b;
            b += (poff[p + 1] - poff[p] + 31) / 32;
        }
        pblk[P] = b;
    }
    __syncthreads();
    for (int64_t blk = threadIdx.x; blk < nblk; blk += blockDim.x) {
        int lo = 0, hi = P - 1;  // last partition p with pblk[p] <= blk
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (pblk[mid] <= blk)
                lo = mid;
            else
                hi = mid - 1;
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) blk_part[4 * blk + j] = lo;
    }
}

// map[packed slot] = row for every row (the map is -1 filled before).
__global__ __launch_bounds__(256) void k_resid_map(const int64_t *__restrict__ poff, const int32_t *__restrict__ perm,
                                                   int64_t n, int P, const int64_t *__restrict__ pblk,
                                                   int64_t map_cap, int32_t *__restrict__ map) {
    for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < n;
         pos += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = P - 1;  // partition with poff[p] <= pos < poff[p+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (poff[mid] <= pos)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int64_t slot = pblk[lo] * 32 + (pos - poff[lo]);
        if (slot >= 0 && slot < map_cap) map[slot] = perm[pos];
    }
}

// Per-dimension max |y - c_assign(y)| over the references (float bits).
__global__ __launch_bounds__(256) void k_resid_absmax(const float *__restrict__ R, int64_t n, int d,
                                                      const float *__restrict__ C,
                                                      const int32_t *__restrict__ assign,
                                                      uint32_t *__restrict__ amax_bits) {
    __shared__ uint32_t local[128];
    for (int t = threadIdx.x; t < d; t += blockDim.x) local[t] = 0u;
    __syncthreads();
    const int64_t total = n * d;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = e / d;
        const int t = (int)(e - row * d);
        const float r = R[e] - C[(int64_t)assign[row] * d + t];
        atomicMax(&local[t], __float_as_uint(fabsf(r)));
    }
    __syncthreads();
    for (int t = threadIdx.x; t < d; t += blockDim.x) atomicMax(&amax_bits[t], local[t]);
}

// scal[0..d): residual scale s_t = absmax_t / 448 (1 for an all-zero
// dimension); scal[d..2d): query multiplier -2 G s_t; scal[2d]: G, the power
// of two that puts a query residual of the references' absmax at a quarter
// to a half of the e4m3 range (a query near the partition fits without
// saturating).
__global__ void k_fp8_resid_scales(const uint32_t *__restrict__ amax, int d, float *__restrict__ scal) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    float m = 0.f;
    for (int t = 0; t < d; ++t) {
        const float a = __uint_as_float(amax[t]);
        const float s = a > 0.f ? a / kFp8Max : 1.f;
        scal[t] = s;
        m = fmaxf(m, 2.f * a * s);
    }
    float G = 1.f;
    if (m > 0.f) G = ldexpf(1.f, (int)floorf(log2f(kFp8Max / m)) - 1);
    for (int t = 0; t < d; ++t) scal[d + t] = -2.f * G * scal[t];
    scal[2 * d] = G;
}

// As k_pack_fp8, for packed slot (b, row lane) holding map[32 b + lane % 32]
// and its residual against the block's partition centroid.
__global__ __launch_bounds__(256) void k_pack_fp8_resid(const float *__restrict__ R, int d, int KS, int64_t nblk,
                                                        const float *__restrict__ scal,
                                                        const int32_t *__restrict__ map,
                                                        const int32_t *__restrict__ blk_part,
                                                        const float *__restrict__ C, i32x4 *__restrict__ Ap,
                                                        float *__restrict__ Np) {
    const int64_t total = nblk * KS * kWave;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int lane = (int)(e % kWave);
        const int64_t bs = e / kWave;
        const int s = (int)(bs % KS);
        const int64_t b = bs / KS;
        const int32_t row = map[32 * b + (lane & 31)];
        const float *c = C + (int64_t)blk_part[4 * b] * d;
        const int h = lane >> 5;
        const int k0 = 64 * s + 32 * h;
        i32x8 w;
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            uint32_t four = 0;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int kk = k0 + 4 * p + q;
                uint32_t code = 0;
                if (kk < d && row >= 0) code = e4m3_code((R[(int64_t)row * d + kk] - c[kk]) / scal[kk]);
                four |= code << (8 * q);
            }
            w[p] = (int)four;
        }
        Ap[2 * bs * kWave + lane] = i32x4{w[0], w[1], w[2], w[3]};
        Ap[2 * bs * kWave + kWave + lane] = i32x4{w[4], w[5], w[6], w[7]};
        if (s == 0 && h == 0) {
            float out = INFINITY;
            if (row >= 0) {
                double nr2 = 0.0;
                for (int t = 0; t < d; ++t) {
                    const double v =
                        (double)e4m3_value(e4m3_code((R[(int64_t)row * d + t] - c[t]) / scal[t])) * scal[t];
                    nr2 += v * v;
                }
                out = (float)(nr2 * scal[2 * d]);
            }
            const int i = lane & 31;
            const int g = i >> 3, hh = (i >> 2) & 1, j = i & 3;
            Np[b * 32 + hh * 16 + 4 * g + j] = out;
        }
    }
}

__global__ __launch_bounds__(256) void k_resid_fill_i32(int32_t *__restrict__ a, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        a[i] = v;
}

// The residual variant's query codes against one partition: the e4m3 codes
// of -2 G s_t (x_t - c_t) over this lane's contraction half, and G |x - c|^2.
// Kept out of line: it runs once per partition change, and inlined into the
// unrolled block loop it would be copied once per block of a phase.
template <int KS>
struct ResidCodes {
    i32x8 c[KS];
    float t;
};

template <int KS>
__device__ __noinline__ ResidCodes<KS> resid_query_codes(const float *__restrict__ Q, const float *__restrict__ cent,
                                                         const float *__restrict__ qscale, int d, int64_t row,
                                                         int part, int h) {
    ResidCodes<KS> out;
    const float *cp = cent + (int64_t)part * d;
    const float *x = Q + (row >= 0 ? row : 0) * d;
    float ss = 0.f;
    for (int s = 0; s < KS; ++s) {
        for (int w = 0; w < 8; ++w) {
            uint32_t four = 0;
            for (int q = 0; q < 4; ++q) {
                const int kk = 64 * s + 32 * h + 4 * w + q;
                uint32_t code = 0;
                if (row >= 0 && kk < d) {
                    const float qv = x[kk] - cp[kk];
                    ss += qv * qv;
                    code = e4m3_code(qv * qscale[d + kk]);
                }
                four |= code << (8 * q);
            }
            out.c[s][w] = (int)four;
        }
    }
    ss += __shfl_xor(ss, 32, kWave);  // the other contraction half's dimensions
    out.t = qscale[2 * d] * ss;
    return out;
}

// Candidate lists hold packed slots: turn them into row ids through the
// packing's row map (slots past the rows, never entered, and -1 stay).
__global__ __launch_bounds__(256) void k_rows_unmap(int32_t *__restrict__ cand, int64_t count,
                                                    const int32_t *__restrict__ rmap, int64_t nr) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = cand[i];
        if (v >= 0 && v < nr) cand[i] = rmap[v];
    }
}

// Candidate lists hold packed rows: turn them into row ids (-1 stays).
__global__ __launch_bounds__(256) void k_resid_unmap(int32_t *__restrict__ cand, int64_t count,
                                                     const int32_t *__restrict__ map) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = cand[i];
        if (v >= 0) cand[i] = map[v];
    }
}

// ---------------------------------------------------------------------------
// Screen.  Lane l handles query c = l % 32 of each of its QB query blocks
// and contraction half h = l / 32; output register v of a 32x32 block holds
// reference row 8(v/4) + 4h + (v%4).
// ---------------------------------------------------------------------------
template <int PREC>
struct LowpOp;
template <>
struct LowpOp<RSC_BF16> {
    using T = i32x4;
    __device__ static f32x16 mfma(T a, T b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                       c, 0, 0, 0);
    }
};
template <>
struct LowpOp<RSC_FP8_E4M3> {
    using T = i32x8;
    __device__ static f32x16 mfma(T a, T b, f32x16 c) {
        // format 0 = e4m3 for both operands; block scales 127 = 2^0
        return __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(a, b, c, 0, 0, 0, 127, 0, 127);
    }
};

// The references are shared by the four waves of a workgroup through a
// double-buffered LDS ring of PH blocks per phase, filled by asynchronous
// global->LDS loads (each wave issues a quarter of them) one phase ahead;
// one barrier per phase.
template <int PREC, int KS, bool RESID = false>
struct LowpRing {
    static constexpr int kBlockBytes = KS * kWave * (PREC == RSC_BF16 ? 16 : 32);
    static constexpr int kNormBytes = PREC == RSC_FP8_E4M3 ? 128 : 0;
    static constexpr int kPartBytes = RESID ? 16 : 0;  // the block's partition (residual variant)
    static constexpr int kSlotBytes = kBlockBytes + kNormBytes + kPartBytes;
    static constexpr int kLoads = kBlockBytes / 1024;  // 1 KiB wave loads per block
    static constexpr int kPhase = PREC == RSC_BF16 ? 4 : 8;  // blocks per phase
};

__device__ __forceinline__ void lds_load16(const void *gsrc, void *lds_base) {
    __builtin_amdgcn_global_load_lds(gsrc, (void __attribute__((address_space(3))) *)lds_base, 16, 0, 0);
}

template <int PREC, int KS, int L, int QB, bool RESID = false>
__global__ __launch_bounds__(256, 3) void k_screen_lowp(ScreenArgs a) {
    using Op = LowpOp<PREC>;
    using T = typename Op::T;
    using Ring = LowpRing<PREC, KS, RESID>;
    constexpr int QW = QB * 32;
    constexpr int QG = kScreenWaves * QW;
    constexpr int PH = Ring::kPhase;
    constexpr int SLOT = Ring::kSlotBytes;
    constexpr int QCAP = 8;  // 16 KiB of queue per workgroup: three workgroups fit a CU
    constexpr bool kNormInAcc = PREC == RSC_FP8_E4M3;

    // Two ring buffers as two LDS objects: the compiler can then tell that
    // the asynchronous loads into one never alias the reads of the other and
    // does not make the reads wait for them.
    __shared__ __attribute__((aligned(16))) char ring0[PH * SLOT];
    __shared__ __attribute__((aligned(16))) char ring1[PH * SLOT];
    __shared__ float2 qbuf[QB * QCAP * 256];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const int h = lane >> 5, c = lane & 31;
    const int p = blockIdx.y;
    const int64_t blk_per = (a.nblk + a.P - 1) / a.P;
    const int64_t blk0 = (int64_t)p * blk_per;
    const int64_t blk1 = std::min<int64_t>(a.nblk, blk0 + blk_per);
    const int64_t nslots = screen_slots(a);
    const char *Ab = static_cast<const char *>(a.Ap);
    const int64_t span = blk1 - blk0;  // blocks of this range
    int64_t rot = 0;                   // the query group's first block, relative to blk0

    // Block of logical position j (0 <= j < span) of this range's scan:
    // blk0 + (rot + j) mod span.
    auto phys = [&](int64_t j) -> int64_t {
        int64_t q = rot + j;
        if (q >= span) q -= span;
        return blk0 + q;
    };

    // Issue this wave's share of the loads of phase `ph` into ring buffer `buf`.
    auto issue = [&](int64_t ph, char *buf) {
        const int64_t b0 = ph * PH;
        constexpr int NA = PH * Ring::kLoads;
#pragma unroll
        for (int j = wave; j < NA; j += kScreenWaves) {
            const int pb = j / Ring::kLoads, q = j % Ring::kLoads;
            const int64_t blk = phys(std::min<int64_t>(b0 + pb, span - 1));  // clamp: always in bounds
            lds_load16(Ab + blk * Ring::kBlockBytes + q * 1024 + lane * 16, buf + pb * SLOT + q * 1024);
        }
        if constexpr (kNormInAcc) {
#pragma unroll
            for (int pb = wave; pb < PH; pb += kScreenWaves) {
                const int64_t blk = phys(std::min<int64_t>(b0 + pb, span - 1));
                // lanes 0..7: the 32 norms; lane 8 (residual variant): the
                // block's partition, landing right after them
                if constexpr (RESID) {
                    if (lane < 9)
                        lds_load16(lane < 8 ? (const void *)(a.Np + blk * 32 + lane * 4)
                                            : (const void *)(a.blk_part + blk * 4),
                                   buf + pb * SLOT + Ring::kBlockBytes);
                } else {
                    if (lane < 8) lds_load16(a.Np + blk * 32 + lane * 4, buf + pb * SLOT + Ring::kBlockBytes);
                }
            }
        }
    };

    for (int64_t qblk = blockIdx.x; qblk * QG < nslots; qblk += gridDim.x) {
        if (a.rotate && span > 0) {
            // references packed in the queries' order: the group's own rows
            // sit at packed slots qblk QG ..; start there (near references
            // first fill the lists and tighten the thresholds early)
            const int64_t own = qblk * QG / 32;
            rot = own < blk0 ? 0 : (own >= blk1 ? span - 1 : own - blk0);
        }
        int64_t slot[QB];
        int64_t qrow[QB];
        T bq[QB][KS];
        float tq[QB];  // residual variant: G |x - c_p|^2 of the current partition
        int cur_part = -1;
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            slot[qb] = qblk * QG + wave * QW + qb * 32 + c;
            int64_t row = -1;
            if (slot[qb] < nslots) row = a.qlist ? (int64_t)a.qlist[slot[qb]] : slot[qb];
            qrow[qb] = row;
            tq[qb] = 0.f;
            if constexpr (RESID) continue;  // coded per partition, at its first block
            const float *x = a.Q + (row >= 0 ? row : 0) * a.d;
#pragma unroll
            for (int s = 0; s < KS; ++s) {
                T v;
                if constexpr (PREC == RSC_BF16) {
#pragma unroll
                    for (int w = 0; w < 4; ++w) {
                        uint32_t two = 0;
#pragma unroll
                        for (int q = 0; q < 2; ++q) {
                            const int kk = 16 * s + 8 * h + 2 * w + q;
                            float f = 0.f;
                            if (row >= 0) f = kk < a.d ? -2.f * x[kk] : (kk <= a.d + 1 ? 1.f : 0.f);
                            two |= bf16_bits(f) << (16 * q);
                        }
                        v[w] = (int)two;
                    }
                } else {
#pragma unroll
                    for (int w = 0; w < 8; ++w) {
                        uint32_t four = 0;
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            const int kk = 64 * s + 32 * h + 4 * w + q;
                            uint32_t code = 0;
                            if (row >= 0 && kk < a.d) code = e4m3_code(x[kk] * a.qscale[a.d + kk]);
                            four |= code << (8 * q);
                        }
                        v[w] = (int)four;
                    }
                }
                bq[qb][s] = v;
            }
        }

        LaneTopK<L, QCAP> top[QB];
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) top[qb].init();

        // Residual variant: the query codes of q = x - c_p (wave-uniform call).
        auto code_partition = [&](int part) {
            if constexpr (PREC == RSC_FP8_E4M3) {
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) {
                    const ResidCodes<KS> rc = resid_query_codes<KS>(a.Q, a.cent, a.qscale, a.d, qrow[qb], part, h);
#pragma unroll
                    for (int s = 0; s < KS; ++s) bq[qb][s] = rc.c[s];
                    tq[qb] = rc.t;
                }
            }
        };

        const int64_t nph = (span + PH - 1) / PH;
        // One phase: wait until its blocks have landed in `cur`, start the
        // next phase's loads into `nxt`, then screen the blocks of `cur`.
        auto phase = [&](int64_t ph, const char *cur, char *nxt) {
            __builtin_amdgcn_s_waitcnt(0x0f70);  // vmcnt(0): this wave's loads of phase ph landed
            __syncthreads();                      // everyone's landed; phase ph-1 is fully consumed
            if (ph + 1 < nph) issue(ph + 1, nxt);
#pragma unroll
            for (int r = 0; r < PH; ++r) {
                if (ph * PH + r >= span) break;
                const int64_t blk = phys(ph * PH + r);
                const char *sl = cur + r * SLOT;
                if constexpr (RESID) {
                    const int part = *reinterpret_cast<const int *>(sl + Ring::kBlockBytes + Ring::kNormBytes);
                    if (part != cur_part) {
                        code_partition(part);
                        cur_part = part;
                    }
                }
                T A[KS];
#pragma unroll
                for (int s = 0; s < KS; ++s) {
                    if constexpr (PREC == RSC_BF16) {
                        A[s] = reinterpret_cast<const i32x4 *>(sl)[s * kWave + lane];
                    } else {
                        const i32x4 lo = reinterpret_cast<const i32x4 *>(sl)[2 * s * kWave + lane];
                        const i32x4 hi = reinterpret_cast<const i32x4 *>(sl)[(2 * s + 1) * kWave + lane];
                        A[s] = i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
                    }
                }
                f32x16 init = f32x16{};
                if constexpr (kNormInAcc) {
                    const f32x4 *ns = reinterpret_cast<const f32x4 *>(sl + Ring::kBlockBytes) + h * 4;
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        const f32x4 t = ns[g];
#pragma unroll
                        for (int j = 0; j < 4; ++j) init[4 * g + j] = t[j];
                    }
                }
                // all operand reads of the block are in flight before its first MFMA
                __builtin_amdgcn_sched_barrier(0);
                f32x16 acc[QB];
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) {
                    acc[qb] = init;
                    if constexpr (RESID) {
#pragma unroll
                        for (int v = 0; v < 16; ++v) acc[qb][v] += tq[qb];
                    }
                }
#pragma unroll
                for (int s = 0; s < KS; ++s) {
#pragma unroll
                    for (int qb = 0; qb < QB; ++qb) acc[qb] = Op::mfma(A[s], bq[qb][s], acc[qb]);
                }
                const int ref0 = (int)(blk * 32) + 4 * h;
#pragma unroll
                for (int qb = 0; qb < QB; ++qb) top[qb].offer(acc[qb], ref0, qbuf + qb * QCAP * 256 + tid, 256);
            }
        };
        __syncthreads();  // the ring is free (previous query block done with it)
        if (nph > 0) issue(0, ring0);
        for (int64_t ph = 0; ph < nph; ph += 2) {
            phase(ph, ring0, ring1);
            if (ph + 1 < nph) phase(ph + 1, ring1, ring0);
        }
#pragma unroll
        for (int qb = 0; qb < QB; ++qb) {
            top[qb].flush(qbuf + qb * QCAP * 256 + tid, 256);
            if (slot[qb] < nslots) top[qb].store(a, slot[qb], p, h);
        }
    }
}

template <int PREC, int KS, int L, int QB, bool RESID = false>
int launch_lowp(const ScreenArgs &a, unsigned gx, const char *name, hipStream_t stream) {
    ScopedTimer timer(name, stream);
    hipLaunchKernelGGL((k_screen_lowp<PREC, KS, L, QB, RESID>), dim3(gx, (unsigned)a.P), dim3(256), 0, stream, a);
    return launch_status(name);
}

}  // namespace

int lowp_steps(int precision, int d) {
    if (precision == RSC_BF16) return (d + 2 + 15) / 16;
    return (d + 63) / 64;
}

int lowp_qb(int precision, int d) {
    (void)precision;
    (void)d;
    return kLowpQB;
}

int lowp_queries_per_group(int precision, int d) { return scr::kScreenWaves * 32 * lowp_qb(precision, d); }

size_t lowp_packed_bytes(int precision, int64_t nblk, int d) {
    const int ks = lowp_steps(precision, d);
    return (size_t)nblk * ks * kWave * (precision == RSC_BF16 ? 16 : 32);
}

int lowp_prepare(const KnnPlan &p, const float *Q, const float *R, void *packed, float *norms, float *scal,
                 uint32_t *amax, const int32_t *rmap, hipStream_t stream) {
    const int ks = lowp_steps(p.precision, p.d);
    const int64_t tot = p.nblk * ks * kWave;
    const unsigned g1 = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
    ScopedTimer timer("prep_pack", stream);
    if (p.precision == RSC_BF16) {
        hipLaunchKernelGGL(k_pack_bf16, dim3(g1), dim3(256), 0, stream, R, p.nr, p.d, ks, p.nblk, rmap,
                           static_cast<i32x4 *>(packed));
        return launch_status("pack_bf16");
    }
    // FP8: per-dimension absmax of references (and of queries when distinct)
    uint32_t *amax_r = amax, *amax_q = amax + 128;
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, stream, amax, 256, 0u);
    const unsigned ga = (unsigned)std::min<int64_t>((p.nr * p.d + 255) / 256, 2048);
    hipLaunchKernelGGL(k_absmax, dim3(ga), dim3(256), 0, stream, R, p.nr, p.d, amax_r);
    if (!p.self_mode && p.nq > 0) {
        const unsigned gq = (unsigned)std::min<int64_t>((p.nq * p.d + 255) / 256, 2048);
        hipLaunchKernelGGL(k_absmax, dim3(gq), dim3(256), 0, stream, Q, p.nq, p.d, amax_q);
    } else {
        amax_q = amax_r;
    }
    hipLaunchKernelGGL(k_fp8_scales, dim3(1), dim3(64), 0, stream, amax_r, amax_q, p.d, scal);
    hipLaunchKernelGGL(k_pack_fp8, dim3(g1), dim3(256), 0, stream, R, p.nr, p.d, ks, p.nblk, scal, rmap,
                       static_cast<i32x4 *>(packed), norms);
    return launch_status("pack_fp8");
}

int lowp_prepare_resid(const KnnPlan &p, const float *R, const KnnBuffers &b, hipStream_t stream) {
    constexpr int kIters = 4;  // Lloyd iterations of the partitioning
    int st;
    {
        ScopedTimer timer("resid_partition", stream);
        hipLaunchKernelGGL(k_resid_init_rows, dim3(1), dim3(256), 0, stream, b.init, p.resid, p.nr);
        if ((st = launch_status("resid_init_rows")) != RSC_OK) return st;
        int64_t relocated = 0;
        if ((st = kmeans_run(R, p.nr, p.d, p.resid, b.init, kIters, b.cent, b.assign, b.poff, b.perm, &relocated,
                             b.kws, b.kws_bytes, stream)) != RSC_OK)
            return st;
    }
    const int ks = lowp_steps(p.precision, p.d);
    const int64_t tot = p.nblk * ks * kWave;
    const unsigned g1 = (unsigned)std::min<int64_t>((tot + 255) / 256, 65536);
    ScopedTimer timer("prep_pack", stream);
    hipLaunchKernelGGL(k_resid_blocks, dim3(1), dim3(1024), 0, stream, b.poff, p.resid, p.nblk, b.pblk, b.blk_part);
    hipLaunchKernelGGL(k_resid_fill_i32, dim3((unsigned)std::min<int64_t>((p.nblk * 32 + 255) / 256, 65536)),
                       dim3(256), 0, stream, b.map, p.nblk * 32, -1);
    const unsigned gm = (unsigned)std::min<int64_t>((p.nr + 255) / 256, 65536);
    hipLaunchKernelGGL(k_resid_map, dim3(gm), dim3(256), 0, stream, b.poff, b.perm, p.nr, p.resid, b.pblk,
                       p.nblk * 32, b.map);
    hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(256), 0, stream, b.amax, 256, 0u);
    const unsigned ga = (unsigned)std::min<int64_t>((p.nr * p.d + 255) / 256, 2048);
    hipLaunchKernelGGL(k_resid_absmax, dim3(ga), dim3(256), 0, stream, R, p.nr, p.d, b.cent, b.assign, b.amax);
    hipLaunchKernelGGL(k_fp8_resid_scales, dim3(1), dim3(64), 0, stream, b.amax, p.d, b.scal);
    hipLaunchKernelGGL(k_pack_fp8_resid, dim3(g1), dim3(256), 0, stream, R, p.d, ks, p.nblk, b.scal, b.map,
                       b.blk_part, b.cent, static_cast<i32x4 *>((void *)b.packed), b.norms);
    return launch_status("pack_fp8_resid");
}

int lowp_unmap_rows(const KnnPlan &p, const KnnBuffers &b, const int32_t *rmap, hipStream_t stream) {
    const int64_t count = p.nq * p.splits * p.screen;
    const unsigned g = (unsigned)std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_rows_unmap, dim3(g), dim3(256), 0, stream, b.cand_idx, count, rmap, p.nr);
    return launch_status("rows_unmap");
}

int lowp_unmap(const KnnPlan &p, const KnnBuffers &b, hipStream_t stream) {
    const int64_t count = p.nq * p.splits * p.screen;
    const unsigned g = (unsigned)std::min<int64_t>((count + 255) / 256, 65536);
    hipLaunchKernelGGL(k_resid_unmap, dim3(g), dim3(256), 0, stream, b.cand_idx, count, b.map);
    return launch_status("resid_unmap");
}

int lowp_screen(const KnnPlan &p, const scr::ScreenArgs &a, unsigned gx, hipStream_t s) {
    const int ks = lowp_steps(p.precision, p.d);
    if (p.precision == RSC_BF16) {
        switch (ks) {
            case 1: return launch_lowp<RSC_BF16, 1, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 2: return launch_lowp<RSC_BF16, 2, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 3: return launch_lowp<RSC_BF16, 3, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 4: return launch_lowp<RSC_BF16, 4, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 5: return launch_lowp<RSC_BF16, 5, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 6: return launch_lowp<RSC_BF16, 6, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 7: return launch_lowp<RSC_BF16, 7, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 8: return launch_lowp<RSC_BF16, 8, 32, kLowpQB>(a, gx, "screen_bf16", s);
            case 9: return launch_lowp<RSC_BF16, 9, 32, kLowpQB>(a, gx, "screen_bf16", s);
            default: break;
        }
    } else if (p.resid > 0) {
        switch (ks) {
            case 1: return launch_lowp<RSC_FP8_E4M3, 1, 32, kLowpQB, true>(a, gx, "screen_fp8_resid", s);
            case 2: return launch_lowp<RSC_FP8_E4M3, 2, 32, kLowpQB, true>(a, gx, "screen_fp8_resid", s);
            default: break;
        }
    } else {
        switch (ks) {
            case 1: return launch_lowp<RSC_FP8_E4M3, 1, 32, kLowpQB>(a, gx, "screen_fp8", s);
            case 2: return launch_lowp<RSC_FP8_E4M3, 2, 32, kLowpQB>(a, gx, "screen_fp8", s);
            default: break;
        }
    }
    set_error("internal: no reduced-precision screen for this dimension");
    return RSC_ERR_UNSUPPORTED;
}

}  // namespace rsc
