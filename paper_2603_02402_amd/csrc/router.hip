// The learned partition router: a d -> H -> H -> P perceptron with ReLU
// activations and a softmax over P coarse partitions, run in BF16 on the
// matrix cores (v_mfma_f32_32x32x16_bf16, FP32 accumulation) for both
// training and inference.  FP32 master weights and Adam moments live in the
// handle; BF16 copies (and transposed copies for the backward GEMMs) are
// refreshed after every optimizer step.
//
// Every contraction is one "NT" GEMM, C[M x N] = A[M x K] . B[N x K]^T with
// both operands K-contiguous, so each lane reads 16 contiguous bytes per
// MFMA step straight from global memory; the epilogues fuse bias, ReLU, the
// ReLU derivative mask and the BF16 rounding.  M and N are multiples of 64,
// K of 16 (the input width is padded to a multiple of 64 with zeros).
//
// Loss: soft-target cross-entropy; each training cell lists m partitions
// (those of its exact nearest neighbours) with weight 1/m each.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "rsc_internal.hpp"

struct rsc_router {
    int d, dp, H, P;
    uint64_t seed;
    int64_t step;
    size_t n_params;              // exported (unpadded) parameter count
    size_t n_padded;              // parameters in the device layout (W1 rows padded to dp)
    float *master, *m1, *m2;      // FP32 weights and Adam moments (flat layout below)
    uint16_t *w1b, *w2b, *w3b;    // BF16 copies: W1 [H x dp], W2 [H x H], W3 [P x H]
    uint16_t *w2tb, *w3tb;        // BF16 transposes: W2^T [H x H], W3^T [H x P]
};

namespace rsc {
namespace {

typedef int i32x4 __attribute__((ext_vector_type(4)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

constexpr int kWave = 64;

// Flat parameter layout: W1 [H x dp] | b1 [H] | W2 [H x H] | b2 [H] | W3 [P x H] | b3 [P].
struct Layout {
    size_t w1, b1, w2, b2, w3, b3, total;
    Layout(int dp, int H, int P) {
        w1 = 0;
        b1 = w1 + (size_t)H * dp;
        w2 = b1 + H;
        b2 = w2 + (size_t)H * H;
        w3 = b2 + H;
        b3 = w3 + (size_t)P * H;
        total = b3 + P;
    }
};

__device__ __forceinline__ uint16_t to_bf16(float x) {
    uint32_t u = __float_as_uint(x);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// ---------------------------------------------------------------------------
// NT GEMM.  Workgroup = 4 waves = 64 x 64 tile; wave (wm, wn) owns a 32 x 32
// sub-tile; lane (c, h) feeds row c of each operand with 8 contiguous K values
// per MFMA (h selects which 8 of the step's 16).  Output register v holds
// C[8(v/4) + 4h + v%4][c] of the sub-tile.
// ---------------------------------------------------------------------------
enum Epi { kStoreF32 = 0, kBiasReluBf16 = 1, kBiasF32 = 2, kMaskBf16 = 3 };

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt(const uint16_t *__restrict__ A, int lda,
                                                 const uint16_t *__restrict__ B, int ldb, void *__restrict__ C,
                                                 int ldc, const float *__restrict__ bias,
                                                 const uint16_t *__restrict__ mask, int K) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 31, h = lane >> 5;
    const int64_t m0 = (int64_t)blockIdx.y * 64 + (wave >> 1) * 32;
    const int64_t n0 = (int64_t)blockIdx.x * 64 + (wave & 1) * 32;
    const uint16_t *ap = A + (m0 + c) * lda + 8 * h;
    const uint16_t *bp = B + (n0 + c) * ldb + 8 * h;
    f32x16 acc = f32x16{};
    i32x4 a = *reinterpret_cast<const i32x4 *>(ap);
    i32x4 b = *reinterpret_cast<const i32x4 *>(bp);
    for (int k0 = 16; k0 <= K; k0 += 16) {
        i32x4 an = a, bn = b;
        if (k0 < K) {
            an = *reinterpret_cast<const i32x4 *>(ap + k0);
            bn = *reinterpret_cast<const i32x4 *>(bp + k0);
        }
        acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b),
                                                      acc, 0, 0, 0);
        a = an;
        b = bn;
    }
#pragma unroll
    for (int v = 0; v < 16; ++v) {
        const int64_t m = m0 + 8 * (v >> 2) + 4 * h + (v & 3);
        const int64_t n = n0 + c;
        float x = acc[v];
        if constexpr (EPI == kBiasReluBf16 || EPI == kBiasF32) x += bias[n];
        if constexpr (EPI == kBiasReluBf16) {
            static_cast<uint16_t *>(C)[m * ldc + n] = to_bf16(fmaxf(x, 0.f));
        } else if constexpr (EPI == kMaskBf16) {
            static_cast<uint16_t *>(C)[m * ldc + n] = mask[m * ldc + n] != 0 ? to_bf16(x) : (uint16_t)0;
        } else {
            static_cast<float *>(C)[m * ldc + n] = x;
        }
    }
}

// The same product with 128 x 128 workgroup tiles: wave (wm, wn) owns a
// 64 x 64 sub-tile of 2 x 2 MFMA blocks, so each 16-byte operand fragment
// feeds two MFMAs and the four waves of a workgroup share every row they
// load (L1).  Needs M and N multiples of 128.
template <int EPI>
__global__ __launch_bounds__(256) void k_gemm_nt128(const uint16_t *__restrict__ A, int lda,
                                                    const uint16_t *__restrict__ B, int ldb, void *__restrict__ C,
                                                    int ldc, const float *__restrict__ bias,
                                                    const uint16_t *__restrict__ mask, int K) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int c = lane & 31, h = lane >> 5;
    const int64_t m0 = (int64_t)blockIdx.y * 128 + (wave >> 1) * 64;
    const int64_t n0 = (int64_t)blockIdx.x * 128 + (wave & 1) * 64;
    const uint16_t *ap0 = A + (m0 + c) * lda + 8 * h;
    const uint16_t *ap1 = ap0 + (int64_t)32 * lda;
    const uint16_t *bp0 = B + (n0 + c) * ldb + 8 * h;
    const uint16_t *bp1 = bp0 + (int64_t)32 * ldb;
    f32x16 acc[2][2] = {{f32x16{}, f32x16{}}, {f32x16{}, f32x16{}}};
    i32x4 a0 = *reinterpret_cast<const i32x4 *>(ap0), a1 = *reinterpret_cast<const i32x4 *>(ap1);
    i32x4 b0 = *reinterpret_cast<const i32x4 *>(bp0), b1 = *reinterpret_cast<const i32x4 *>(bp1);
    for (int k0 = 16; k0 <= K; k0 += 16) {
        i32x4 na0 = a0, na1 = a1, nb0 = b0, nb1 = b1;
        if (k0 < K) {
            na0 = *reinterpret_cast<const i32x4 *>(ap0 + k0);
            na1 = *reinterpret_cast<const i32x4 *>(ap1 + k0);
            nb0 = *reinterpret_cast<const i32x4 *>(bp0 + k0);
            nb1 = *reinterpret_cast<const i32x4 *>(bp1 + k0);
        }
        const bf16x8 fa0 = __builtin_bit_cast(bf16x8, a0), fa1 = __builtin_bit_cast(bf16x8, a1);
        const bf16x8 fb0 = __builtin_bit_cast(bf16x8, b0), fb1 = __builtin_bit_cast(bf16x8, b1);
        acc[0][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0, fb0, acc[0][0], 0, 0, 0);
        acc[0][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa0, fb1, acc[0][1], 0, 0, 0);
        acc[1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1, fb0, acc[1][0], 0, 0, 0);
        acc[1][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fa1, fb1, acc[1][1], 0, 0, 0);
        a0 = na0;
        a1 = na1;
        b0 = nb0;
        b1 = nb1;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i) {
#pragma unroll
        for (int j = 0; j < 2; ++j) {
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int64_t m = m0 + 32 * i + 8 * (v >> 2) + 4 * h + (v & 3);
                const int64_t n = n0 + 32 * j + c;
                float x = acc[i][j][v];
                if constexpr (EPI == kBiasReluBf16 || EPI == kBiasF32) x += bias[n];
                if constexpr (EPI == kBiasReluBf16) {
                    static_cast<uint16_t *>(C)[m * ldc + n] = to_bf16(fmaxf(x, 0.f));
                } else if constexpr (EPI == kMaskBf16) {
                    static_cast<uint16_t *>(C)[m * ldc + n] = mask[m * ldc + n] != 0 ? to_bf16(x) : (uint16_t)0;
                } else {
                    static_cast<float *>(C)[m * ldc + n] = x;
                }
            }
        }
    }
}

// C[R x C] -> out[C x R] (BF16), 64 x 64 tiles through LDS.
__global__ __launch_bounds__(256) void k_transpose_bf16(const uint16_t *__restrict__ in, int rows, int cols,
                                                        uint16_t *__restrict__ out) {
    __shared__ uint16_t tile[64][65];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e / 64, cc = e % 64;
        tile[r][cc] = in[(int64_t)(r0 + r) * cols + c0 + cc];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int cc = e / 64, r = e % 64;
        out[(int64_t)(c0 + cc) * rows + r0 + r] = tile[r][cc];
    }
}

// FP32 master (rows x cols, row stride ld_in) -> BF16 transposed (cols x rows).
__global__ __launch_bounds__(256) void k_transpose_f32_bf16(const float *__restrict__ in, int rows, int cols,
                                                            uint16_t *__restrict__ out) {
    __shared__ float tile[64][65];
    const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int r = e / 64, cc = e % 64;
        tile[r][cc] = in[(int64_t)(r0 + r) * cols + c0 + cc];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 64 * 64; e += 256) {
        const int cc = e / 64, r = e % 64;
        out[(int64_t)(c0 + cc) * rows + r0 + r] = to_bf16(tile[r][cc]);
    }
}

// Column sums of a BF16 matrix (bias gradients) in two passes with a fixed
// order: partial[c][j] = sum of rows 256c .. 256c+255 of column j (a wave
// reads consecutive columns of one row: coalesced), then out[j] = sum over c.
constexpr int kColChunk = 256;

__global__ __launch_bounds__(256) void k_colsum_partial(const uint16_t *__restrict__ in, int rows, int cols,
                                                        float *__restrict__ partial) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (j >= cols) return;
    const int r1 = min(rows, (c + 1) * kColChunk);
    float s = 0.f;
    for (int r = c * kColChunk; r < r1; ++r) s += from_bf16(in[(int64_t)r * cols + j]);
    partial[(int64_t)c * cols + j] = s;
}

__global__ __launch_bounds__(256) void k_colsum_final(const float *__restrict__ partial, int chunks, int cols,
                                                      float *__restrict__ out) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= cols) return;
    float s = 0.f;
    for (int c = 0; c < chunks; ++c) s += partial[(int64_t)c * cols + j];
    out[j] = s;
}

// Rows [row0, row0 + nb) of X (n x d, float32), or rows list[row0 + i], as a
// zero-padded BF16 block [B x dp].
__global__ __launch_bounds__(256) void k_cast_input(const float *__restrict__ X, int d, const int32_t *__restrict__ list,
                                                    int64_t row0, int nb, int B, int dp, uint16_t *__restrict__ out) {
    const int64_t total = (int64_t)B * dp;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / dp), t = (int)(e % dp);
        float x = 0.f;
        if (r < nb && t < d) {
            const int64_t row = list ? (int64_t)list[row0 + r] : row0 + r;
            x = X[row * d + t];
        }
        out[e] = to_bf16(x);
    }
}

// Soft-target cross-entropy and its gradient, one wave per row.
//   loss_i = logsumexp(z_i) - (1/m) sum_j z_i[label_j]
//   dZ_i   = (softmax(z_i) - t_i) * scale        (rows >= nb: 0)
__global__ __launch_bounds__(256) void k_softmax_ce(const float *__restrict__ Z, int P, const int32_t *__restrict__ labels,
                                                    int m, int64_t lrow0, int nb, int B, float scale,
                                                    uint16_t *__restrict__ dZ, float *__restrict__ row_loss) {
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= B) return;
    const float *z = Z + (int64_t)r * P;
    uint16_t *g = dZ + (int64_t)r * P;
    if (r >= nb) {
        for (int p = lane; p < P; p += kWave) g[p] = 0;
        if (lane == 0) row_loss[r] = 0.f;
        return;
    }
    float mx = -INFINITY;
    for (int p = lane; p < P; p += kWave) mx = fmaxf(mx, z[p]);
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
    float se = 0.f;
    for (int p = lane; p < P; p += kWave) se += expf(z[p] - mx);
    for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o, kWave);
    const float lse = mx + logf(se);
    const int32_t *lab = labels + (lrow0 + r) * m;
    for (int p = lane; p < P; p += kWave) {
        float t = 0.f;
        for (int j = 0; j < m; ++j) t += lab[j] == p ? 1.f : 0.f;
        g[p] = to_bf16((expf(z[p] - lse) - t / (float)m) * scale);
    }
    if (lane == 0) {
        // -sum_p t_p log softmax(z)_p, labels outside [0, P) skipped
        float loss = 0.f;
        for (int j = 0; j < m; ++j)
            if (lab[j] >= 0 && lab[j] < P) loss += (lse - z[lab[j]]) / (float)m;
        row_loss[r] = loss;
    }
}

// Sum of the per-row losses of one batch (one block), times `scale`.
__global__ __launch_bounds__(256) void k_batch_loss(const float *__restrict__ row_loss, int nb, float scale,
                                                    float *__restrict__ out) {
    __shared__ float part[256];
    float s = 0.f;
    for (int r = threadIdx.x; r < nb; r += 256) s += row_loss[r];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = part[0] * scale;
}

// Adam on the flat FP32 parameters; writes the BF16 copies of the weights.
__global__ __launch_bounds__(256) void k_adam(float *__restrict__ w, float *__restrict__ m1, float *__restrict__ m2,
                                              const float *__restrict__ g, int64_t n, float lr, float b1, float b2,
                                              float eps, float c1, float c2, Layout L, uint16_t *__restrict__ w1b,
                                              uint16_t *__restrict__ w2b, uint16_t *__restrict__ w3b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m1[i] + (1.f - b1) * gi;
        const float vi = b2 * m2[i] + (1.f - b2) * gi * gi;
        m1[i] = mi;
        m2[i] = vi;
        const float wi = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
        w[i] = wi;
        const size_t u = (size_t)i;
        if (u < L.b1) w1b[u - L.w1] = to_bf16(wi);
        else if (u >= L.w2 && u < L.b2) w2b[u - L.w2] = to_bf16(wi);
        else if (u >= L.w3 && u < L.b3) w3b[u - L.w3] = to_bf16(wi);
    }
}

// BF16 copies of the weights from the masters (after init or load).
__global__ __launch_bounds__(256) void k_refresh_bf16(const float *__restrict__ w, Layout L, uint16_t *__restrict__ w1b,
                                                      uint16_t *__restrict__ w2b, uint16_t *__restrict__ w3b) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)L.total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const size_t u = (size_t)i;
        if (u < L.b1) w1b[u - L.w1] = to_bf16(w[u]);
        else if (u >= L.w2 && u < L.b2) w2b[u - L.w2] = to_bf16(w[u]);
        else if (u >= L.w3 && u < L.b3) w3b[u - L.w3] = to_bf16(w[u]);
    }
}

// SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
// generators", 2014): state += 0x9e3779b97f4a7c15, then two xor-shift-multiply
// rounds.  Counter-based here: the i-th value of a stream is mix(seed + i*gamma).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9e3779b97f4a7c15ull;
    x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
    x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
    return x ^ (x >> 31);
}

// Uniform(-lim, lim) weights (lim = sqrt(6 / (fan_in + fan_out))), zero
// biases and zero padded input columns.
__global__ __launch_bounds__(256) void k_init_params(float *__restrict__ w, Layout L, int d, int dp, int H, int P,
                                                     uint64_t seed) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)L.total;
         i += (int64_t)gridDim.x * blockDim.x) {
        const size_t u = (size_t)i;
        float lim = 0.f;
        bool zero = false;
        if (u < L.b1) {
            lim = sqrtf(6.f / (float)(d + H));
            zero = (int)((u - L.w1) % dp) >= d;
        } else if (u >= L.w2 && u < L.b2) {
            lim = sqrtf(6.f / (float)(2 * H));
        } else if (u >= L.w3 && u < L.b3) {
            lim = sqrtf(6.f / (float)(H + P));
        } else {
            zero = true;
        }
        const uint64_t r = splitmix64(seed + (uint64_t)i * 0x9e3779b97f4a7c15ull);
        const float uni = (float)(r >> 40) * (1.f / 16777216.f);  // 24 random bits in [0, 1)
        w[u] = zero ? 0.f : (2.f * uni - 1.f) * lim;
    }
}

// Top `probes` partitions per row by logit (ties: lower index) and the
// softmax mass they hold.  One wave per row: lane l holds columns l + 64 t
// in registers and keeps a sorted list of its 4 best not yet taken; each
// round the wave-wide best head (by value, then column) is taken and only
// its lane's list moves.  A lane whose list runs dry rebuilds it from the
// values that come after the last one it gave up (rare: a lane holds more
// than 4 of the winners only when they cluster in its columns).
__global__ __launch_bounds__(256) void k_top_probes(const float *__restrict__ Z, int P, int nb, int probes,
                                                    int32_t *__restrict__ parts, float *__restrict__ mass) {
    constexpr int T = 4096 / kWave;  // registers per lane (P <= 4096)
    constexpr int LL = 4;            // list length
    const int lane = threadIdx.x & 63;
    const int r = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= nb) return;
    const float *z = Z + (int64_t)r * P;
    float v[T];
    float mx = -INFINITY;
#pragma unroll
    for (int t = 0; t < T; ++t) {
        const int p = lane + kWave * t;
        v[t] = p < P ? z[p] : -INFINITY;
        mx = fmaxf(mx, v[t]);
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmaxf(mx, __shfl_xor(mx, o, kWave));
    float se = 0.f;
#pragma unroll
    for (int t = 0; t < T; ++t) se += lane + kWave * t < P ? expf(v[t] - mx) : 0.f;
    for (int o = 32; o > 0; o >>= 1) se += __shfl_xor(se, o, kWave);

    // (value desc, t asc) order within the lane; t = -1 marks an empty slot
    float lv[LL];
    int lt[LL];
    float fv = INFINITY;  // last value this lane gave up (floor); everything before it is taken
    int ft = -1;
    auto rebuild = [&]() {
#pragma unroll
        for (int i = 0; i < LL; ++i) {
            lv[i] = -INFINITY;
            lt[i] = -1;
        }
#pragma unroll
        for (int t = 0; t < T; ++t) {
            const float x = v[t];
            const bool after_floor = x < fv || (x == fv && t > ft);
            const bool real = lane + kWave * t < P;
            if (real && after_floor && (lt[LL - 1] < 0 || x > lv[LL - 1])) {
                // insert (t ascending, so equal values keep index order)
#pragma unroll
                for (int i = LL - 1; i > 0; --i) {
                    const bool shift = lt[i - 1] < 0 || x > lv[i - 1];
                    const bool here = lt[i] < 0 || x > lv[i];
                    lv[i] = shift ? lv[i - 1] : (here ? x : lv[i]);
                    lt[i] = shift ? lt[i - 1] : (here ? t : lt[i]);
                }
                if (lt[0] < 0 || x > lv[0]) {
                    lv[0] = x;
                    lt[0] = t;
                }
            }
        }
    };
    rebuild();
    float got = 0.f;
    for (int s = 0; s < probes; ++s) {
        float best = lt[0] >= 0 ? lv[0] : -INFINITY;
        int bi = lt[0] >= 0 ? lane + kWave * lt[0] : INT32_MAX;
        for (int o = 32; o > 0; o >>= 1) {
            const float ov = __shfl_xor(best, o, kWave);
            const int oi = __shfl_xor(bi, o, kWave);
            if (ov > best || (ov == best && oi < bi)) {
                best = ov;
                bi = oi;
            }
        }
        if (bi == INT32_MAX) {  // fewer columns than probes
            if (lane == 0) parts[(int64_t)r * probes + s] = -1;
            continue;
        }
        if ((bi & 63) == lane) {
            fv = lv[0];
            ft = lt[0];
#pragma unroll
            for (int i = 0; i < LL - 1; ++i) {
                lv[i] = lv[i + 1];
                lt[i] = lt[i + 1];
            }
            lv[LL - 1] = -INFINITY;
            lt[LL - 1] = -1;
            if (lt[0] < 0) rebuild();
        }
        if (lane == 0) parts[(int64_t)r * probes + s] = bi;
        got += expf(best - mx) / se;
    }
    if (lane == 0) mass[r] = got;
}

// Parameters in the exported layout (W1 without the zero padding of the
// input width): dst[...] from the padded src.
__global__ __launch_bounds__(256) void k_unpad_params(const float *__restrict__ src, Layout L, int d, int dp, int H,
                                                      float *__restrict__ dst) {
    const int64_t w1n = (int64_t)H * d;
    const int64_t total = w1n + (int64_t)(L.total - L.b1);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        if (i < w1n) {
            const int64_t h = i / d, t = i % d;
            dst[i] = src[L.w1 + h * dp + t];
        } else {
            dst[i] = src[L.b1 + (i - w1n)];
        }
    }
}

// Mean loss of one epoch from its per-batch sums (one block, fixed order).
__global__ __launch_bounds__(256) void k_epoch_loss(const float *__restrict__ batch_sum, int64_t nbatches, double inv_n,
                                                    float *__restrict__ out) {
    __shared__ double part[256];
    double acc = 0.0;
    for (int64_t b = threadIdx.x; b < nbatches; b += 256) acc += (double)batch_sum[b];
    part[threadIdx.x] = acc;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = (float)(part[0] * inv_n);
}

constexpr int kMaxEpochs = 1024;
constexpr int kInferChunk = 16384;  // rows per inference pass

struct TrainBuffers {
    uint16_t *a0, *h1, *h2, *dz, *dzt, *h2t, *dh2, *dh2t, *h1t, *dh1, *dh1t, *a0t;
    float *z, *grad, *row_loss, *batch_sum, *epoch_loss, *colsum;
};

size_t carve_train(const rsc_router *R, int B, int64_t nbatches, void *ws, TrainBuffers *t) {
    Carver cv(ws);
    TrainBuffers b;
    const int dp = R->dp, H = R->H, P = R->P;
    b.a0 = cv.take<uint16_t>((size_t)B * dp);
    b.h1 = cv.take<uint16_t>((size_t)B * H);
    b.h2 = cv.take<uint16_t>((size_t)B * H);
    b.dz = cv.take<uint16_t>((size_t)B * P);
    b.dzt = cv.take<uint16_t>((size_t)B * P);
    b.h2t = cv.take<uint16_t>((size_t)B * H);
    b.dh2 = cv.take<uint16_t>((size_t)B * H);
    b.dh2t = cv.take<uint16_t>((size_t)B * H);
    b.h1t = cv.take<uint16_t>((size_t)B * H);
    b.dh1 = cv.take<uint16_t>((size_t)B * H);
    b.dh1t = cv.take<uint16_t>((size_t)B * H);
    b.a0t = cv.take<uint16_t>((size_t)B * dp);
    b.z = cv.take<float>((size_t)B * P);
    b.grad = cv.take<float>(R->n_padded);
    b.row_loss = cv.take<float>((size_t)B);
    b.batch_sum = cv.take<float>((size_t)std::max<int64_t>(nbatches, 1));
    b.epoch_loss = cv.take<float>(kMaxEpochs);
    b.colsum = cv.take<float>((size_t)((B + kColChunk - 1) / kColChunk) * std::max(P, H));
    if (t) *t = b;
    return cv.used;
}

struct InferBuffers {
    uint16_t *a0, *h1, *h2;
    float *z;
};

size_t carve_infer(const rsc_router *R, void *ws, InferBuffers *t) {
    Carver cv(ws);
    InferBuffers b;
    b.a0 = cv.take<uint16_t>((size_t)kInferChunk * R->dp);
    b.h1 = cv.take<uint16_t>((size_t)kInferChunk * R->H);
    b.h2 = cv.take<uint16_t>((size_t)kInferChunk * R->H);
    b.z = cv.take<float>((size_t)kInferChunk * R->P);
    if (t) *t = b;
    return cv.used;
}

// C[M x N] = A[M x K] . B[N x K]^T with the fused epilogue; 128-wide tiles
// when the shape allows them and still gives the chip enough workgroups.
template <int EPI>
int gemm(const uint16_t *A, int lda, const uint16_t *B, int ldb, void *C, int ldc, const float *bias,
         const uint16_t *mask, int M, int N, int K, hipStream_t s) {
    if (M % 128 == 0 && N % 128 == 0 && (int64_t)(M / 128) * (N / 128) >= 512)
        hipLaunchKernelGGL((k_gemm_nt128<EPI>), dim3(N / 128, M / 128), dim3(256), 0, s, A, lda, B, ldb, C, ldc,
                           bias, mask, K);
    else
        hipLaunchKernelGGL((k_gemm_nt<EPI>), dim3(N / 64, M / 64), dim3(256), 0, s, A, lda, B, ldb, C, ldc, bias,
                           mask, K);
    return launch_status("router gemm");
}

int colsum(const uint16_t *in, int rows, int cols, float *scratch, float *out, hipStream_t s) {
    const int chunks = (rows + kColChunk - 1) / kColChunk;
    hipLaunchKernelGGL(k_colsum_partial, dim3((cols + 255) / 256, chunks), dim3(256), 0, s, in, rows, cols, scratch);
    hipLaunchKernelGGL(k_colsum_final, dim3((cols + 255) / 256), dim3(256), 0, s, scratch, chunks, cols, out);
    return launch_status("router bias gradient");
}

int transpose(const uint16_t *in, int rows, int cols, uint16_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_transpose_bf16, dim3(cols / 64, rows / 64), dim3(256), 0, s, in, rows, cols, out);
    return launch_status("router transpose");
}

int refresh_transposes(rsc_router *R, hipStream_t s) {
    const Layout L(R->dp, R->H, R->P);
    hipLaunchKernelGGL(k_transpose_f32_bf16, dim3(R->H / 64, R->H / 64), dim3(256), 0, s, R->master + L.w2, R->H, R->H,
                       R->w2tb);
    hipLaunchKernelGGL(k_transpose_f32_bf16, dim3(R->H / 64, R->P / 64), dim3(256), 0, s, R->master + L.w3, R->P, R->H,
                       R->w3tb);
    return launch_status("router weight transposes");
}

// Forward pass of B rows already cast into a0: logits in z.
int forward(const rsc_router *R, const uint16_t *a0, uint16_t *h1, uint16_t *h2, float *z, int B, hipStream_t s) {
    const Layout L(R->dp, R->H, R->P);
    int st;
    if ((st = gemm<kBiasReluBf16>(a0, R->dp, R->w1b, R->dp, h1, R->H, R->master + L.b1, nullptr, B, R->H, R->dp, s)) !=
        RSC_OK)
        return st;
    if ((st = gemm<kBiasReluBf16>(h1, R->H, R->w2b, R->H, h2, R->H, R->master + L.b2, nullptr, B, R->H, R->H, s)) !=
        RSC_OK)
        return st;
    return gemm<kBiasF32>(h2, R->H, R->w3b, R->H, z, R->P, R->master + L.b3, nullptr, B, R->P, R->H, s);
}

// Gradients of the mean loss of rows [row0, row0 + nb) into t.grad; the
// sum of their losses times loss_scale into *loss_out.
int backward(const rsc_router *R, const TrainBuffers &t, const int32_t *labels, int m, int64_t row0, int nb, int B,
             float loss_scale, float *loss_out, hipStream_t s) {
    const Layout L(R->dp, R->H, R->P);
    const int H = R->H, P = R->P, dp = R->dp;
    int st;
    hipLaunchKernelGGL(k_softmax_ce, dim3((B + 3) / 4), dim3(256), 0, s, t.z, P, labels, m, row0, nb, B,
                       1.f / (float)nb, t.dz, t.row_loss);
    if ((st = launch_status("softmax_ce")) != RSC_OK) return st;
    hipLaunchKernelGGL(k_batch_loss, dim3(1), dim3(256), 0, s, t.row_loss, nb, loss_scale, loss_out);
    // W3, b3
    if ((st = transpose(t.dz, B, P, t.dzt, s)) != RSC_OK) return st;
    if ((st = transpose(t.h2, B, H, t.h2t, s)) != RSC_OK) return st;
    if ((st = gemm<kStoreF32>(t.dzt, B, t.h2t, B, t.grad + L.w3, H, nullptr, nullptr, P, H, B, s)) != RSC_OK) return st;
    if ((st = colsum(t.dz, B, P, t.colsum, t.grad + L.b3, s)) != RSC_OK) return st;
    // back through W3 and the second ReLU
    if ((st = gemm<kMaskBf16>(t.dz, P, R->w3tb, P, t.dh2, H, nullptr, t.h2, B, H, P, s)) != RSC_OK) return st;
    // W2, b2
    if ((st = transpose(t.dh2, B, H, t.dh2t, s)) != RSC_OK) return st;
    if ((st = transpose(t.h1, B, H, t.h1t, s)) != RSC_OK) return st;
    if ((st = gemm<kStoreF32>(t.dh2t, B, t.h1t, B, t.grad + L.w2, H, nullptr, nullptr, H, H, B, s)) != RSC_OK) return st;
    if ((st = colsum(t.dh2, B, H, t.colsum, t.grad + L.b2, s)) != RSC_OK) return st;
    // back through W2 and the first ReLU
    if ((st = gemm<kMaskBf16>(t.dh2, H, R->w2tb, H, t.dh1, H, nullptr, t.h1, B, H, H, s)) != RSC_OK) return st;
    // W1, b1
    if ((st = transpose(t.dh1, B, H, t.dh1t, s)) != RSC_OK) return st;
    if ((st = transpose(t.a0, B, dp, t.a0t, s)) != RSC_OK) return st;
    if ((st = gemm<kStoreF32>(t.dh1t, B, t.a0t, B, t.grad + L.w1, dp, nullptr, nullptr, H, dp, B, s)) != RSC_OK)
        return st;
    return colsum(t.dh1, B, H, t.colsum, t.grad + L.b1, s);
}

int cast_rows(const rsc_router *R, const float *X, const int32_t *list, int64_t row0, int nb, int B, uint16_t *out,
              hipStream_t s) {
    const int64_t tot = (int64_t)B * R->dp;
    const unsigned g = (unsigned)std::min<int64_t>((tot + 255) / 256, 8192);
    hipLaunchKernelGGL(k_cast_input, dim3(g), dim3(256), 0, s, X, R->d, list, row0, nb, B, R->dp, out);
    return launch_status("router input cast");
}

void free_router(rsc_router *R) {
    if (!R) return;
    void *bufs[] = {R->master, R->m1, R->m2, R->w1b, R->w2b, R->w3b, R->w2tb, R->w3tb};
    for (void *b : bufs)
        if (b) (void)hipFree(b);
    delete R;
}

int check_x(const rsc_router *R, const float *X, int64_t n, const char *who) {
    if (!R) {
        set_error(std::string(who) + ": null router");
        return RSC_ERR_INVALID_ARG;
    }
    if (n < 0 || (n > 0 && !X) || (reinterpret_cast<uintptr_t>(X) & 3u) != 0) {
        set_error(std::string(who) + ": need n >= 0 and an aligned float32 input");
        return RSC_ERR_INVALID_ARG;
    }
    if (n > INT32_MAX - 1) {
        set_error(std::string(who) + ": more rows than int32 can index");
        return RSC_ERR_OVERFLOW;
    }
    return RSC_OK;
}

constexpr uint32_t kMagic = 0x52435352u;  // "RSCR"
constexpr uint32_t kVersion = 1;

}  // namespace

// ---- host API used by abi.hip --------------------------------------------

int router_create(rsc_router **out, int d, int hidden, int parts, uint64_t seed) {
    if (!out || d < 1 || d > 256 || hidden < 64 || hidden % 64 || parts < 64 || parts % 64 || parts > 4096) {
        set_error("router: need 1 <= d <= 256, hidden a multiple of 64, 64 <= parts <= 4096 a multiple of 64");
        return RSC_ERR_INVALID_ARG;
    }
    rsc_router *R = new (std::nothrow) rsc_router();
    if (!R) {
        set_error("router: out of host memory");
        return RSC_ERR_NO_MEMORY;
    }
    R->d = d;
    R->dp = (d + 63) / 64 * 64;
    R->H = hidden;
    R->P = parts;
    R->seed = seed;
    R->step = 0;
    const Layout L(R->dp, hidden, parts);
    R->n_padded = L.total;
    R->n_params = L.total - (size_t)hidden * (R->dp - d);
    int st = RSC_OK;
    auto alloc = [&](void **p, size_t bytes) {
        if (st == RSC_OK) st = hip_status(hipMalloc(p, bytes), "router allocation");
    };
    alloc((void **)&R->master, L.total * 4);
    alloc((void **)&R->m1, L.total * 4);
    alloc((void **)&R->m2, L.total * 4);
    alloc((void **)&R->w1b, (size_t)hidden * R->dp * 2);
    alloc((void **)&R->w2b, (size_t)hidden * hidden * 2);
    alloc((void **)&R->w3b, (size_t)parts * hidden * 2);
    alloc((void **)&R->w2tb, (size_t)hidden * hidden * 2);
    alloc((void **)&R->w3tb, (size_t)parts * hidden * 2);
    if (st == RSC_OK) {
        hipLaunchKernelGGL(k_init_params, dim3(1024), dim3(256), 0, nullptr, R->master, L, d, R->dp, hidden, parts,
                           seed);
        st = hip_status(hipMemset(R->m1, 0, L.total * 4), "router moments");
        if (st == RSC_OK) st = hip_status(hipMemset(R->m2, 0, L.total * 4), "router moments");
        if (st == RSC_OK) {
            hipLaunchKernelGGL(k_refresh_bf16, dim3(1024), dim3(256), 0, nullptr, R->master, L, R->w1b, R->w2b, R->w3b);
            st = refresh_transposes(R, nullptr);
        }
        if (st == RSC_OK) st = hip_status(hipDeviceSynchronize(), "router init");
    }
    if (st != RSC_OK) {
        free_router(R);
        return st;
    }
    *out = R;
    return RSC_OK;
}

void router_destroy(rsc_router *R) { free_router(R); }

int router_info(const rsc_router *R, int *d, int *hidden, int *parts, int64_t *n_params, int64_t *step) {
    if (!R) {
        set_error("router: null handle");
        return RSC_ERR_INVALID_ARG;
    }
    if (d) *d = R->d;
    if (hidden) *hidden = R->H;
    if (parts) *parts = R->P;
    if (n_params) *n_params = (int64_t)R->n_params;
    if (step) *step = R->step;
    return RSC_OK;
}

size_t router_train_workspace(const rsc_router *R, int batch, int64_t n) {
    if (!R || batch < 64 || batch % 64 || n < 1) return 0;
    return carve_train(R, batch, (n + batch - 1) / batch, nullptr, nullptr);
}

int router_train(rsc_router *R, const float *X, int64_t n, const int32_t *labels, int m, int epochs, int batch, float lr,
                 float *loss_log, void *ws, size_t ws_bytes, hipStream_t s) {
    int st = check_x(R, X, n, "router_train");
    if (st != RSC_OK) return st;
    if (!labels || n < 1 || m < 1 || epochs < 1 || epochs > kMaxEpochs || batch < 64 || batch % 64 ||
        !(lr > 0.f)) {
        set_error("router_train: need n >= 1, labels, m >= 1, 1 <= epochs <= 1024, batch a multiple of 64, lr > 0");
        return RSC_ERR_INVALID_ARG;
    }
    const int64_t nbatches = (n + batch - 1) / batch;
    TrainBuffers t;
    const size_t need = carve_train(R, batch, nbatches, ws, &t);
    if (!ws || need > ws_bytes) {
        set_error("router_train: workspace too small: need " + std::to_string(need) + " bytes");
        return RSC_ERR_WORKSPACE;
    }
    const Layout L(R->dp, R->H, R->P);
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    ScopedTimer timer("router_train", s);
    for (int e = 0; e < epochs; ++e) {
        for (int64_t bi = 0; bi < nbatches; ++bi) {
            const int64_t row0 = bi * batch;
            const int nb = (int)std::min<int64_t>(batch, n - row0);
            if ((st = cast_rows(R, X, nullptr, row0, nb, batch, t.a0, s)) != RSC_OK) return st;
            if ((st = forward(R, t.a0, t.h1, t.h2, t.z, batch, s)) != RSC_OK) return st;
            if ((st = backward(R, t, labels, m, row0, nb, batch, 1.f, t.batch_sum + bi, s)) != RSC_OK) return st;
            ++R->step;
            const float c1 = 1.f - powf(b1, (float)R->step), c2 = 1.f - powf(b2, (float)R->step);
            hipLaunchKernelGGL(k_adam, dim3(1024), dim3(256), 0, s, R->master, R->m1, R->m2, t.grad,
                               (int64_t)L.total, lr, b1, b2, eps, c1, c2, L, R->w1b, R->w2b, R->w3b);
            if ((st = refresh_transposes(R, s)) != RSC_OK) return st;
        }
        hipLaunchKernelGGL(k_epoch_loss, dim3(1), dim3(256), 0, s, t.batch_sum, nbatches, 1.0 / (double)n,
                           t.epoch_loss + e);
        if ((st = launch_status("router epoch loss")) != RSC_OK) return st;
    }
    if (loss_log) {
        if ((st = hip_status(hipMemcpyAsync(loss_log, t.epoch_loss, (size_t)epochs * 4, hipMemcpyDeviceToHost, s),
                             "read losses")) != RSC_OK)
            return st;
        return hip_status(hipStreamSynchronize(s), "synchronise");
    }
    return RSC_OK;
}

size_t router_gradients_workspace(const rsc_router *R, int64_t n) {
    if (!R || n < 1 || n > 65536) return 0;
    return carve_train(R, (int)((n + 63) / 64 * 64), 1, nullptr, nullptr);
}

int router_gradients(const rsc_router *R, const float *X, int64_t n, const int32_t *labels, int m, float *grad_out,
                     float *loss_out, void *ws, size_t ws_bytes, hipStream_t s) {
    int st = check_x(R, X, n, "router_gradients");
    if (st != RSC_OK) return st;
    if (!labels || !grad_out || n < 1 || m < 1 || n > 65536) {
        set_error("router_gradients: need 1 <= n <= 65536 rows, labels and an output buffer");
        return RSC_ERR_INVALID_ARG;
    }
    const int B = (int)((n + 63) / 64 * 64);
    TrainBuffers t;
    const size_t need = carve_train(R, B, 1, ws, &t);
    if (!ws || need > ws_bytes) {
        set_error("router_gradients: workspace too small: need " + std::to_string(need) + " bytes");
        return RSC_ERR_WORKSPACE;
    }
    if ((st = cast_rows(R, X, nullptr, 0, (int)n, B, t.a0, s)) != RSC_OK) return st;
    if ((st = forward(R, t.a0, t.h1, t.h2, t.z, B, s)) != RSC_OK) return st;
    if ((st = backward(R, t, labels, m, 0, (int)n, B, 1.f / (float)n, loss_out ? loss_out : t.batch_sum, s)) !=
        RSC_OK)
        return st;
    const Layout L(R->dp, R->H, R->P);
    hipLaunchKernelGGL(k_unpad_params, dim3(1024), dim3(256), 0, s, t.grad, L, R->d, R->dp, R->H, grad_out);
    return launch_status("router gradients");
}

size_t router_infer_workspace(const rsc_router *R) { return R ? carve_infer(R, nullptr, nullptr) : 0; }

// Logits (logits != nullptr) or top-probe selection of n rows (rows of X, or
// X[list[i]] when a list is given), kInferChunk rows at a time.
int router_infer(const rsc_router *R, const float *X, int64_t n, const int32_t *list, float *logits, int probes,
                 int32_t *parts, float *mass, void *ws, size_t ws_bytes, hipStream_t s) {
    int st = check_x(R, X, n, "router inference");
    if (st != RSC_OK) return st;
    if (!logits && (!parts || !mass || probes < 1 || probes > R->P || probes > 64)) {
        set_error("router_probe: need 1 <= probes <= min(parts, 64) and output arrays");
        return RSC_ERR_INVALID_ARG;
    }
    InferBuffers t;
    const size_t need = carve_infer(R, ws, &t);
    if (!ws || need > ws_bytes) {
        set_error("router inference: workspace too small: need " + std::to_string(need) + " bytes");
        return RSC_ERR_WORKSPACE;
    }
    ScopedTimer timer("router_infer", s);
    for (int64_t row0 = 0; row0 < n; row0 += kInferChunk) {
        const int nb = (int)std::min<int64_t>(kInferChunk, n - row0);
        const int B = (nb + 127) / 128 * 128;  // 128-row tiles for the products
        if ((st = cast_rows(R, X, list, row0, nb, B, t.a0, s)) != RSC_OK) return st;
        float *z = logits ? nullptr : t.z;
        if (logits) {
            // whole 128-row groups straight into the output; the ragged tail via the scratch
            const int full = nb / 128 * 128;
            if (full > 0 && (st = forward(R, t.a0, t.h1, t.h2, logits + row0 * R->P, full, s)) != RSC_OK) return st;
            if (full < nb) {
                if ((st = forward(R, t.a0 + (size_t)full * R->dp, t.h1, t.h2, t.z, 128, s)) != RSC_OK) return st;
                if ((st = hip_status(hipMemcpyAsync(logits + (row0 + full) * R->P, t.z,
                                                    (size_t)(nb - full) * R->P * 4, hipMemcpyDeviceToDevice, s),
                                     "copy logits")) != RSC_OK)
                    return st;
            }
            continue;
        }
        if ((st = forward(R, t.a0, t.h1, t.h2, z, B, s)) != RSC_OK) return st;
        hipLaunchKernelGGL(k_top_probes, dim3((nb + 3) / 4), dim3(256), 0, s, z, R->P, nb, probes,
                           parts + row0 * probes, mass + row0);
        if ((st = launch_status("top probes")) != RSC_OK) return st;
    }
    return RSC_OK;
}

// File: magic, version, d, hidden, parts (int32), step (int64), seed
// (uint64), then the weights in the exported layout, then the two Adam
// moments in the same layout (float32).
int router_save(const rsc_router *R, const char *path) {
    if (!R || !path) {
        set_error("router_save: null argument");
        return RSC_ERR_INVALID_ARG;
    }
    const Layout L(R->dp, R->H, R->P);
    std::vector<float> host(L.total * 3);
    int st = hip_status(hipMemcpy(host.data(), R->master, L.total * 4, hipMemcpyDeviceToHost), "read weights");
    if (st == RSC_OK) st = hip_status(hipMemcpy(host.data() + L.total, R->m1, L.total * 4, hipMemcpyDeviceToHost), "m1");
    if (st == RSC_OK)
        st = hip_status(hipMemcpy(host.data() + 2 * L.total, R->m2, L.total * 4, hipMemcpyDeviceToHost), "m2");
    if (st != RSC_OK) return st;
    FILE *f = std::fopen(path, "wb");
    if (!f) {
        set_error(std::string("router_save: cannot open ") + path);
        return RSC_ERR_INVALID_ARG;
    }
    const int32_t hdr[5] = {(int32_t)kMagic, (int32_t)kVersion, R->d, R->H, R->P};
    bool ok = std::fwrite(hdr, sizeof(hdr), 1, f) == 1 && std::fwrite(&R->step, 8, 1, f) == 1 &&
              std::fwrite(&R->seed, 8, 1, f) == 1;
    for (int part = 0; part < 3 && ok; ++part) {
        const float *base = host.data() + part * L.total;
        for (int h = 0; h < R->H && ok; ++h)
            ok = std::fwrite(base + L.w1 + (size_t)h * R->dp, 4, R->d, f) == (size_t)R->d;
        ok = ok && std::fwrite(base + L.b1, 4, L.total - L.b1, f) == L.total - L.b1;
    }
    ok = (std::fclose(f) == 0) && ok;
    if (!ok) {
        set_error("router_save: write failed");
        return RSC_ERR_INVALID_ARG;
    }
    return RSC_OK;
}

int router_load(rsc_router *R, const char *path) {
    if (!R || !path) {
        set_error("router_load: null argument");
        return RSC_ERR_INVALID_ARG;
    }
    FILE *f = std::fopen(path, "rb");
    if (!f) {
        set_error(std::string("router_load: cannot open ") + path);
        return RSC_ERR_INVALID_ARG;
    }
    int32_t hdr[5];
    int64_t step = 0;
    uint64_t seed = 0;
    bool ok = std::fread(hdr, sizeof(hdr), 1, f) == 1 && std::fread(&step, 8, 1, f) == 1 &&
              std::fread(&seed, 8, 1, f) == 1;
    if (!ok || hdr[0] != (int32_t)kMagic || hdr[1] != (int32_t)kVersion || hdr[2] != R->d || hdr[3] != R->H ||
        hdr[4] != R->P) {
        std::fclose(f);
        set_error("router_load: not a router file of this shape");
        return RSC_ERR_INVALID_ARG;
    }
    const Layout L(R->dp, R->H, R->P);
    std::vector<float> host(L.total * 3, 0.f);
    for (int part = 0; part < 3 && ok; ++part) {
        float *base = host.data() + part * L.total;
        for (int h = 0; h < R->H && ok; ++h)
            ok = std::fread(base + L.w1 + (size_t)h * R->dp, 4, R->d, f) == (size_t)R->d;
        ok = ok && std::fread(base + L.b1, 4, L.total - L.b1, f) == L.total - L.b1;
    }
    std::fclose(f);
    if (!ok) {
        set_error("router_load: truncated file");
        return RSC_ERR_INVALID_ARG;
    }
    int st = hip_status(hipMemcpy(R->master, host.data(), L.total * 4, hipMemcpyHostToDevice), "write weights");
    if (st == RSC_OK) st = hip_status(hipMemcpy(R->m1, host.data() + L.total, L.total * 4, hipMemcpyHostToDevice), "m1");
    if (st == RSC_OK)
        st = hip_status(hipMemcpy(R->m2, host.data() + 2 * L.total, L.total * 4, hipMemcpyHostToDevice), "m2");
    if (st != RSC_OK) return st;
    R->step = step;
    R->seed = seed;
    hipLaunchKernelGGL(k_refresh_bf16, dim3(1024), dim3(256), 0, nullptr, R->master, L, R->w1b, R->w2b, R->w3b);
    if ((st = refresh_transposes(R, nullptr)) != RSC_OK) return st;
    return hip_status(hipDeviceSynchronize(), "router load");
}

int router_shape(const rsc_router *R, int *d, int *parts) {
    if (!R) return RSC_ERR_INVALID_ARG;
    *d = R->d;
    *parts = R->P;
    return RSC_OK;
}

}  // namespace rsc
