// UMAP layout of the fuzzy graph: edge-sampled stochastic gradient descent
// on the cross-entropy between the graph's weights and the embedding's
// similarities q(d2) = 1 / (1 + a d2^b) (the layout step of UMAP, the
// embedding method the paper runs on this graph).
//
// Reading (deterministic by construction):
//   * edge e of weight w_e is due every w_max / w_e epochs (never if
//     w_e < w_max / n_epochs), first at epoch w_max / w_e;
//   * within an epoch every move is computed from the embedding at the start
//     of the epoch; vertex i sums the moves of the edges of its own CSR row,
//     in row order, and the sums are applied at the end of the epoch (the
//     symmetric graph holds each edge in both rows, so both ends move);
//   * a due edge (i, j) attracts i towards j by clip(g (y_i - y_j)) alpha_t
//     with g = -2 a b d2^(b-1) / (a d2^b + 1) (0 for d2 = 0), then draws `neg`
//     vertices k from a counter-based SplitMix64 (state seed + (t 2^40 + e 64
//     + p + 1) 0x9E3779B97F4A7C15; the edge stride is the largest neg) and
//     repels i from each (k != i) by clip(g' (y_i - y_k)) alpha_t,
//     g' = 2 gamma b / ((0.001 + d2)(a d2^b + 1)), or by 4 alpha_t per
//     coordinate when the points coincide;
//   * clip to [-4, 4]; alpha_t = alpha0 (1 - t / n_epochs).
// The embedding is kept in float64 and every sum runs in the order stated,
// with explicitly rounded operations (no fused multiply-adds), and the powers
// d2^b and d2^(b-1) are the correctly rounded ones (table-driven double-double
// evaluation, the tables made on the device by a table-free series), so the
// result is the same function of the inputs as any sequential implementation
// that follows these steps: the dynamics amplify a one-ulp difference in a
// power into visibly different layouts within tens of epochs.
//
// One epoch, edge-parallel where the work is:
//   1. count the due edges of each tile of 4096 edges (at epoch 0; later
//      epochs take the counts that the previous epoch's step 3 made);
//   2. exclusive scan of the tile counts (one block);
//   3. rank the due edges within each tile (wave ballots, in edge order) and
//      write the list of due edges in CSR order -- those of one vertex form
//      one contiguous range -- the position of every edge in that list, and
//      the due edges' next-sample epochs;
//   4. moves and sums, one wave per 64 consecutive vertices: the due edges of
//      those vertices form one range of the list, and each (due edge, draw)
//      slot -- the attraction and each negative sample -- one move.  Chunk by
//      chunk the lanes compute the range's moves (the powers and the random
//      gathers: nearly all of the arithmetic) into LDS, the attractions
//      first and then the negative samples, one slot per lane; then each lane
//      adds its own vertex's moves in row order, skipping the negative
//      samples that drew the vertex itself (marked in a flag per slot), and
//      writes the new position (float64 embeddings ping-pong between two
//      buffers).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "crpow.hpp"
#include "rsc_internal.hpp"

// Every product and sum below is rounded on its own, as written.
#pragma clang fp contract(off)

namespace rsc {
namespace {

constexpr int kMaxDim = 8;
constexpr int kMaxNeg = 64;
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr int kTileSteps = 16;                  // 256-edge steps per tile
constexpr int64_t kTile = 256 * kTileSteps;     // edges per tile of the compaction

__device__ __forceinline__ uint64_t sm64_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// x mod n for x < 2^53, n < 2^31, from inv_n = 1/n rounded: the float64
// quotient is within 3 of the true one, and the integer remainder is then
// moved into [0, n) (the same residue as an integer division gives).
__device__ __forceinline__ int64_t mod_n(uint64_t x, int64_t n, double inv_n) {
    const int64_t q = (int64_t)__builtin_floor(__dmul_rn((double)x, inv_n));
    int64_t r = (int64_t)x - q * n;
    while (r < 0) r += n;
    while (r >= n) r -= n;
    return r;
}

// Negative sample p of edge e in epoch t.
__device__ __forceinline__ int64_t negative(uint64_t seed, int t, int64_t e, int p, int64_t n, double inv_n) {
    const uint64_t st = seed + ((uint64_t)t * (1ull << 40) + (uint64_t)e * (uint64_t)kMaxNeg + (uint64_t)p + 1ull) * kGolden;
    return mod_n(sm64_mix(st) >> 11, n, inv_n);
}

__device__ __forceinline__ double clip4(double x) { return x > 4.0 ? 4.0 : (x < -4.0 ? -4.0 : x); }

// alpha0 (1 - t / n_epochs), each operation rounded to nearest (the file is
// compiled without contraction, on the host as on the device)
__host__ __device__ inline double epoch_alpha(double alpha0, int t, int n_epochs) {
    return alpha0 * (1.0 - (double)t / (double)n_epochs);
}

__global__ __launch_bounds__(256) void k_umap_wmax(const float *__restrict__ w, int64_t nnz,
                                                   uint32_t *__restrict__ max_bits) {
    __shared__ float part[4];
    float m = 0.f;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x)
        m = fmaxf(m, w[e]);
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0)  // weights are >= 0: their bit patterns order as the values
        atomicMax(max_bits, __float_as_uint(fmaxf(fmaxf(part[0], part[1]), fmaxf(part[2], part[3]))));
}

__global__ __launch_bounds__(256) void k_umap_init(const float *__restrict__ w, int64_t nnz,
                                                   const uint32_t *__restrict__ max_bits, int n_epochs,
                                                   double *__restrict__ eps, double *__restrict__ next,
                                                   const float *__restrict__ Yin, int64_t ny,
                                                   double *__restrict__ Y) {
    const double wmax = (double)__uint_as_float(*max_bits);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        const double we = (double)w[e];
        const double v = (we > 0.0 && we >= wmax / (double)n_epochs) ? wmax / we : -1.0;
        eps[e] = v;
        next[e] = v;
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ny; e += (int64_t)gridDim.x * blockDim.x)
        Y[e] = (double)Yin[e];
}

// The power's tables (double-doubles), made on the device by the table-free
// series: entry t < 64 is log c_t, entry 64 + k is 2^(k/64).
__global__ __launch_bounds__(128) void k_umap_tables(crp::PowTables *__restrict__ tb) {
    const int t = threadIdx.x;
    const crp::dd v = crp::pow_table_entry(t);
    if (t < crp::kPowCells)
        tb->logc[t] = v;
    else
        tb->exp2[t - crp::kPowCells] = v;
}

// Row of every edge (the vertex whose move it makes).
__global__ __launch_bounds__(256) void k_umap_rows(const int64_t *__restrict__ indptr, int64_t n,
                                                   uint32_t *__restrict__ erow) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) erow[e] = (uint32_t)i;
}

__device__ __forceinline__ bool is_due(const double *__restrict__ eps, const double *__restrict__ next, int64_t e,
                                       int64_t nnz, int t) {
    return e < nnz && !(eps[e] < 0.0) && !(next[e] > (double)t);
}

// Due edges of each tile.
__global__ __launch_bounds__(256) void k_umap_count(const double *__restrict__ eps, const double *__restrict__ next,
                                                    int64_t nnz, int t, uint32_t *__restrict__ tile_cnt) {
    __shared__ uint32_t part[4];
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t c = 0;
#pragma unroll 4
    for (int k = 0; k < kTileSteps; ++k) c += is_due(eps, next, base + k * 256 + threadIdx.x, nnz, t) ? 1u : 0u;
    for (int o = 32; o > 0; o >>= 1) c += __shfl_xor(c, o, 64);
    if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Exclusive scan of the T tile counts; one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_umap_tile_scan(const uint32_t *__restrict__ cnt, int64_t T,
                                                         uint32_t *__restrict__ off) {
    __shared__ uint32_t part[1024];
    const int tid = threadIdx.x;
    const int64_t per = (T + 1023) / 1024;
    const int64_t lo = std::min<int64_t>(T, tid * per), hi = std::min<int64_t>(T, lo + per);
    uint32_t sum = 0;
    for (int64_t i = lo; i < hi; ++i) sum += cnt[i];
    part[tid] = sum;
    __syncthreads();
    for (int d = 1; d < 1024; d <<= 1) {
        const uint32_t v = tid >= d ? part[tid - d] : 0u;
        __syncthreads();
        part[tid] += v;
        __syncthreads();
    }
    uint32_t run = part[tid] - sum;
    for (int64_t i = lo; i < hi; ++i) {
        off[i] = run;
        run += cnt[i];
    }
}

// Rank the due edges of a tile in edge order: pos[e] = due edges before e;
// list[pos[e]] = e for a due edge, whose next-sample epoch advances by eps.
// The last tile writes the total to pos[nnz].  The tile's due edges of the
// next epoch are counted on the way (into tile_cnt, already consumed by the
// scan of this epoch).
__global__ __launch_bounds__(256) void k_umap_scatter(const double *__restrict__ eps, double *__restrict__ next,
                                                      int64_t nnz, int t, const uint32_t *__restrict__ tile_off,
                                                      uint32_t *__restrict__ pos, uint32_t *__restrict__ list,
                                                      uint32_t *__restrict__ tile_cnt) {
    __shared__ uint32_t part[4];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    uint32_t off = tile_off[blockIdx.x];
    uint32_t due_next = 0;
    for (int k = 0; k < kTileSteps; ++k) {
        const int64_t e = base + k * 256 + threadIdx.x;
        double ee = -1.0, nx = 0.0;
        if (e < nnz) {
            ee = eps[e];
            nx = next[e];
        }
        const bool due = !(ee < 0.0) && !(nx > (double)t);
        const uint64_t mask = __ballot(due);
        if (lane == 0) part[wv] = (uint32_t)__popcll(mask);
        __syncthreads();
        uint32_t before = (uint32_t)__popcll(mask & ((1ull << lane) - 1ull)), step = 0;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            before += v < wv ? part[v] : 0u;
            step += part[v];
        }
        if (e < nnz) pos[e] = off + before;
        if (due) {
            list[off + before] = (uint32_t)e;
            nx = __dadd_rn(nx, ee);
            next[e] = nx;
        }
        due_next += (!(ee < 0.0) && !(nx > (double)(t + 1))) ? 1u : 0u;
        off += step;
        __syncthreads();  // part is rewritten by the next step
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) pos[nnz] = off;
    for (int o = 32; o > 0; o >>= 1) due_next += __shfl_xor(due_next, o, 64);
    if (lane == 0) part[wv] = due_next;
    __syncthreads();
    if (threadIdx.x == 0) tile_cnt[blockIdx.x] = part[0] + part[1] + part[2] + part[3];
}

// Epoch constants of the moves.
struct Moves {
    double alpha, a, b, bm1, ab2, gb2, inv_n;  // bm1 = b - 1, ab2 = -2 a b, gb2 = 2 gamma b
    int64_t n;
    int t, dim, per;
    uint64_t seed;
};

// Slot (due edge j, draw p) of the epoch: p = 0 the attraction along the
// edge, p >= 1 the negative sample p - 1.  slot_fetch gathers what the move
// needs (the two embedding rows); a negative sample that drew the vertex
// itself is marked and makes no move.
template <int DIMS>
struct SlotIn {
    double yi[DIMS], yo[DIMS];
    bool self;
};

template <int DIMS>
__device__ __forceinline__ void slot_fetch(const Moves &m, int64_t j, int p, const uint32_t *__restrict__ list,
                                           const uint32_t *__restrict__ erow, const int32_t *__restrict__ indices,
                                           const double *__restrict__ Y0, SlotIn<DIMS> &in) {
    const int64_t e = list[j];
    const int64_t i = erow[e];
    const int64_t other = p == 0 ? (int64_t)indices[e] : negative(m.seed, m.t, e, p - 1, m.n, m.inv_n);
    in.self = p > 0 && other == i;
#pragma unroll
    for (int c = 0; c < DIMS; ++c) {
        in.yi[c] = c < m.dim ? Y0[i * m.dim + c] : 0.0;
        in.yo[c] = c < m.dim ? Y0[other * m.dim + c] : 0.0;
    }
}

template <int DIMS>
__device__ __forceinline__ double slot_d2(const Moves &m, const SlotIn<DIMS> &in, double *df) {
    double d2 = 0.0;
#pragma unroll
    for (int c = 0; c < DIMS; ++c)
        if (c < m.dim) {
            df[c] = __dsub_rn(in.yi[c], in.yo[c]);
            d2 = __dadd_rn(d2, __dmul_rn(df[c], df[c]));
        }
    return d2;
}

// Attraction: g = -2 a b d2^(b-1) / (a d2^b + 1), 0 when the points coincide.
template <int DIMS>
__device__ __forceinline__ void attract_move(const Moves &m, const SlotIn<DIMS> &in, const crp::PowTables &tb,
                                             double *out) {
    double df[DIMS];
    const double d2 = slot_d2<DIMS>(m, in, df);
    double g = 0.0;
    if (d2 > 0.0) {
        double pbm1, pb;
        crp::pow2_rn_t(d2, m.bm1, m.b, tb, &pbm1, &pb);
        g = __ddiv_rn(__dmul_rn(m.ab2, pbm1), __dadd_rn(__dmul_rn(m.a, pb), 1.0));
    }
#pragma unroll
    for (int c = 0; c < DIMS; ++c)
        if (c < m.dim) out[c] = __dmul_rn(clip4(__dmul_rn(g, df[c])), m.alpha);
}

// Repulsion: g = 2 gamma b / ((0.001 + d2)(a d2^b + 1)); a push of 4 alpha
// per coordinate when the points coincide.
template <int DIMS>
__device__ __forceinline__ void repel_move(const Moves &m, const SlotIn<DIMS> &in, const crp::PowTables &tb,
                                           double *out) {
    double df[DIMS];
    const double d2 = slot_d2<DIMS>(m, in, df);
    if (!(d2 > 0.0)) {
#pragma unroll
        for (int c = 0; c < DIMS; ++c)
            if (c < m.dim) out[c] = __dmul_rn(4.0, m.alpha);
        return;
    }
    const double pb = crp::pow_rn_t(d2, m.b, tb);
    const double g = __ddiv_rn(m.gb2, __dmul_rn(__dadd_rn(0.001, d2), __dadd_rn(__dmul_rn(m.a, pb), 1.0)));
#pragma unroll
    for (int c = 0; c < DIMS; ++c)
        if (c < m.dim) out[c] = __dmul_rn(clip4(__dmul_rn(g, df[c])), m.alpha);
}

// One wave (block) per 64 consecutive vertices, lane L for vertex i0 + L.
// The due edges of vertex i are list[pos[indptr[i]] .. pos[indptr[i+1]]), in
// row order, and its slots [pos[indptr[i]] per, pos[indptr[i+1]] per), so the
// wave's due edges, and their slots, form one range.  Chunk by chunk (whole
// due edges), the lanes compute the moves into LDS -- first the attractions
// (one lane per due edge: two powers each), then the negative samples (one
// lane per draw: one power each), so that a wave's lanes evaluate the same
// kind of move together -- then each lane adds its own vertex's moves in
// slot order, skipping the draws marked as the vertex itself.
constexpr int kMoveLds = 1024;  // float64 moves per chunk (8 KiB)
constexpr int kSumUnroll = 8;   // moves read from LDS per round, then added in order

template <int DIMS>  // coordinates held in registers: dim <= DIMS
__global__ __launch_bounds__(64) void k_umap_epoch(const int64_t *__restrict__ indptr,
                                                   const uint32_t *__restrict__ pos,
                                                   const uint32_t *__restrict__ list,
                                                   const uint32_t *__restrict__ erow,
                                                   const int32_t *__restrict__ indices, const double *__restrict__ Y0,
                                                   double *__restrict__ Y1, Moves m,
                                                   const crp::PowTables *__restrict__ tables) {
    __shared__ crp::PowTables tb;
    __shared__ double buf[kMoveLds];
    __shared__ uint8_t selfd[kMoveLds];  // slot drew the vertex itself
    static_assert(sizeof(crp::PowTables) == 256 * sizeof(double), "four doubles per lane");
#pragma unroll
    for (int u = 0; u < 4; ++u)
        reinterpret_cast<double *>(&tb)[u * 64 + threadIdx.x] = reinterpret_cast<const double *>(tables)[u * 64 + threadIdx.x];
    __syncthreads();
    const int lane = threadIdx.x;
    const int dim = m.dim, per = m.per, neg = per - 1;
    const int64_t n = m.n;
    const int jchunk = std::max(1, kMoveLds / (per * dim));  // due edges per chunk (per * dim <= 520)
    // a lane fetches four of its slots (two when dim > 2) before computing
    // them, so that their dependent loads (list, edge, two embedding rows)
    // overlap; deeper groups raise the register count and cost more
    // occupancy than they hide
    constexpr int PFD = DIMS <= 2 ? 4 : 2;
    for (int64_t i0 = (int64_t)blockIdx.x * 64; i0 < n; i0 += (int64_t)gridDim.x * 64) {
        const int64_t i = i0 + lane;
        const int64_t J0 = pos[indptr[i0]];
        const int64_t J1 = pos[indptr[std::min<int64_t>(i0 + 64, n)]];
        int64_t lo = 0, hi = 0;
        if (i < n) {
            lo = (int64_t)pos[indptr[i]] * per;
            hi = (int64_t)pos[indptr[i + 1]] * per;
        }
        double mv[DIMS];
#pragma unroll
        for (int c = 0; c < DIMS; ++c) mv[c] = 0.0;
        for (int64_t j0 = J0; j0 < J1; j0 += jchunk) {
            const int nj = (int)std::min<int64_t>(jchunk, J1 - j0);
            // attractions: slot jj * per of the chunk
            for (int jb = lane; jb < nj; jb += PFD * 64) {
                SlotIn<DIMS> in[PFD];
#pragma unroll
                for (int u = 0; u < PFD; ++u)
                    if (jb + u * 64 < nj) slot_fetch<DIMS>(m, j0 + jb + u * 64, 0, list, erow, indices, Y0, in[u]);
#pragma unroll
                for (int u = 0; u < PFD; ++u) {
                    const int jj = jb + u * 64;
                    if (jj < nj) {
                        attract_move<DIMS>(m, in[u], tb, buf + jj * per * dim);
                        selfd[jj * per] = 0;
                    }
                }
            }
            // negative samples: draw q of the chunk is slot (q / neg) per + 1 + q mod neg
            const int nq = nj * neg;
            for (int qb = lane; qb < nq; qb += PFD * 64) {
                SlotIn<DIMS> in[PFD];
#pragma unroll
                for (int u = 0; u < PFD; ++u) {
                    const int q = qb + u * 64;
                    if (q < nq) {
                        const int jj = q / neg;
                        slot_fetch<DIMS>(m, j0 + jj, 1 + q - jj * neg, list, erow, indices, Y0, in[u]);
                    }
                }
#pragma unroll
                for (int u = 0; u < PFD; ++u) {
                    const int q = qb + u * 64;
                    if (q < nq) {
                        const int jj = q / neg;
                        const int sl = jj * per + 1 + q - jj * neg;
                        selfd[sl] = in[u].self ? 1 : 0;
                        if (!in[u].self) repel_move<DIMS>(m, in[u], tb, buf + sl * dim);
                    }
                }
            }
            __syncthreads();
            const int64_t c0 = j0 * per;
            const int64_t s1 = std::min<int64_t>(hi, (j0 + nj) * per);
            for (int64_t sb = std::max<int64_t>(lo, c0); sb < s1; sb += kSumUnroll) {
                double v[kSumUnroll][DIMS];
                bool skip[kSumUnroll];
#pragma unroll
                for (int u = 0; u < kSumUnroll; ++u) {
                    const bool in_range = sb + u < s1;
                    skip[u] = !in_range || selfd[in_range ? sb + u - c0 : 0] != 0;
                    const double *tm = buf + (sb + u - c0) * dim;
#pragma unroll
                    for (int c = 0; c < DIMS; ++c) v[u][c] = (in_range && c < dim) ? tm[c] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < kSumUnroll; ++u) {
                    if (skip[u]) continue;
#pragma unroll
                    for (int c = 0; c < DIMS; ++c)
                        if (c < dim) mv[c] = __dadd_rn(mv[c], v[u][c]);
                }
            }
            __syncthreads();  // buf is refilled by the next chunk
        }
        if (i < n) {
#pragma unroll
            for (int c = 0; c < DIMS; ++c)
                if (c < dim) Y1[i * dim + c] = __dadd_rn(Y0[i * dim + c], mv[c]);
        }
    }
}

__global__ __launch_bounds__(256) void k_umap_out(const double *__restrict__ Y, int64_t ny, float *__restrict__ out) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ny; e += (int64_t)gridDim.x * blockDim.x)
        out[e] = (float)Y[e];
}

__global__ void k_umap_zero(uint32_t *x, int32_t *err) {
    *x = 0u;
    *err = 0;
}

// indptr ascending from 0 to nnz, indices in [0, n), weights finite and >= 0.
__global__ __launch_bounds__(256) void k_umap_check(const int64_t *__restrict__ indptr,
                                                    const int32_t *__restrict__ indices,
                                                    const float *__restrict__ w, const float *__restrict__ Y,
                                                    int64_t n, int64_t nnz, int64_t ny, int32_t *__restrict__ err) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = indptr[i];
        if (v < 0 || v > nnz || (i == 0 && v != 0) || (i == n && v != nnz) || (i < n && indptr[i + 1] < v))
            atomicOr(err, 1);
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz; e += (int64_t)gridDim.x * blockDim.x) {
        if (indices[e] < 0 || indices[e] >= n) atomicOr(err, 2);
        if (!(w[e] >= 0.f) || isinf(w[e])) atomicOr(err, 4);
    }
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ny; e += (int64_t)gridDim.x * blockDim.x)
        if (!isfinite(Y[e])) atomicOr(err, 8);
}

struct Ws {
    crp::PowTables *tables;
    double *eps, *next, *Y0, *Y1;
    uint32_t *pos, *list, *erow, *tile_cnt, *tile_off, *maxb;
    int32_t *err;
};

int64_t n_tiles(int64_t nnz) { return std::max<int64_t>(1, (nnz + kTile - 1) / kTile); }

size_t carve(int64_t n, int64_t nnz, int dim, int neg, void *ws, Ws *w) {
    const size_t m = (size_t)std::max<int64_t>(nnz, 1);
    const size_t T = (size_t)n_tiles(nnz);
    Carver cv(ws);
    crp::PowTables *tables = cv.take<crp::PowTables>(1);
    double *eps = cv.take<double>(m);
    double *next = cv.take<double>(m);
    uint32_t *pos = cv.take<uint32_t>(m + 1);
    uint32_t *list = cv.take<uint32_t>(m);
    uint32_t *erow = cv.take<uint32_t>(m);
    double *Y0 = cv.take<double>((size_t)n * dim);
    double *Y1 = cv.take<double>((size_t)n * dim);
    uint32_t *tile_cnt = cv.take<uint32_t>(T);
    uint32_t *tile_off = cv.take<uint32_t>(T);
    uint32_t *maxb = cv.take<uint32_t>(1);
    int32_t *err = cv.take<int32_t>(1);
    if (w) *w = Ws{tables, eps, next, Y0, Y1, pos, list, erow, tile_cnt, tile_off, maxb, err};
    return cv.used;
}

unsigned grid(int64_t m) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(16384, (m + 255) / 256)); }

bool shape_ok(int64_t n, int64_t nnz, int dim, int neg) {
    return n >= 1 && n <= INT32_MAX && nnz >= 0 && nnz < (int64_t)UINT32_MAX && dim >= 1 && dim <= kMaxDim &&
           neg >= 0 && neg <= kMaxNeg;
}

}  // namespace

size_t umap_workspace_bytes(int64_t n, int64_t nnz, int dim, int neg) {
    if (!shape_ok(n, nnz, dim, neg)) return 0;
    return carve(n, nnz, dim, neg, nullptr, nullptr);
}

int umap_layout(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
                int dim, float *Y, int n_epochs, double a, double b, double gamma, double alpha0, int neg,
                uint64_t seed, void *ws, size_t ws_bytes, hipStream_t s) {
    if (!indptr || !Y || (nnz > 0 && (!indices || !weights))) {
        set_error("umap_layout: null argument");
        return RSC_ERR_INVALID_ARG;
    }
    if (n < 1 || nnz < 0 || dim < 1 || dim > kMaxDim || n_epochs < 1 || neg < 0 || neg > kMaxNeg ||
        !(a > 0.0) || !(b > 0.0) || !(b <= 64.0) || !(gamma >= 0.0) || !(alpha0 > 0.0) || !(a < INFINITY) ||
        !(gamma < INFINITY) || !(alpha0 < INFINITY)) {
        set_error("umap_layout: need n >= 1, 1 <= dim <= 8, n_epochs >= 1, 0 <= neg <= 64, 0 < b <= 64, "
                  "finite a, alpha0 > 0 and finite gamma >= 0");
        return RSC_ERR_INVALID_ARG;
    }
    if (!shape_ok(n, nnz, dim, neg) || n_epochs >= (1 << 23)) {
        set_error("umap_layout: supports n < 2^31, nnz < 2^32 - 1 and epochs < 2^23");
        return RSC_ERR_UNSUPPORTED;
    }
    Ws w;
    const size_t need = carve(n, nnz, dim, neg, nullptr, nullptr);
    if (need == 0 || !ws || ws_bytes < need) {
        set_error("umap_layout: workspace too small");
        return RSC_ERR_WORKSPACE;
    }
    carve(n, nnz, dim, neg, ws, &w);
    const int64_t ny = n * dim;
    int st;
    hipLaunchKernelGGL(k_umap_zero, dim3(1), dim3(1), 0, s, w.maxb, w.err);
    hipLaunchKernelGGL(k_umap_check, dim3(grid(std::max(std::max(nnz, n + 1), ny))), dim3(256), 0, s, indptr,
                       indices, weights, (const float *)Y, n, nnz, ny, w.err);
    int32_t host_err = 0;
    if ((st = launch_status("umap check")) != RSC_OK ||
        (st = hip_status(hipMemcpyAsync(&host_err, w.err, 4, hipMemcpyDeviceToHost, s), "read check")) != RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (host_err & 8) {
        set_error("umap_layout: a non-finite initial position");
        return RSC_ERR_INVALID_ARG;
    }
    if (host_err) {
        set_error(host_err & 1 ? "umap_layout: indptr is not an ascending list from 0 to nnz"
                               : host_err & 2 ? "umap_layout: a column index outside [0, n)"
                                              : "umap_layout: a negative or non-finite weight");
        return RSC_ERR_BAD_GRAPH;
    }
    {
        ScopedTimer tm("umap_init", s);
        hipLaunchKernelGGL(k_umap_wmax, dim3((unsigned)std::min<int64_t>(1024, (nnz + 255) / 256 + 1)), dim3(256), 0,
                           s, weights, nnz, w.maxb);
        hipLaunchKernelGGL(k_umap_init, dim3(grid(std::max(nnz, ny))), dim3(256), 0, s, weights, nnz,
                           (const uint32_t *)w.maxb, n_epochs, w.eps, w.next, (const float *)Y, ny, w.Y0);
        hipLaunchKernelGGL(k_umap_rows, dim3(grid(n)), dim3(256), 0, s, indptr, n, w.erow);
        hipLaunchKernelGGL(k_umap_tables, dim3(1), dim3(2 * crp::kPowCells), 0, s, w.tables);
    }
    if ((st = launch_status("umap init")) != RSC_OK) return st;
    const int64_t T = n_tiles(nnz);
    const unsigned g_epoch = (unsigned)std::min<int64_t>(32768, (n + 63) / 64);
    {
        ScopedTimer tm("umap_epochs", s);
        for (int t = 0; t < n_epochs; ++t) {
            {
                ScopedTimer td("umap_due", s);
                if (t == 0)  // later epochs' counts come from the previous scatter
                    hipLaunchKernelGGL(k_umap_count, dim3((unsigned)T), dim3(256), 0, s, (const double *)w.eps,
                                       (const double *)w.next, nnz, t, w.tile_cnt);
                hipLaunchKernelGGL(k_umap_tile_scan, dim3(1), dim3(1024), 0, s, (const uint32_t *)w.tile_cnt, T,
                                   w.tile_off);
                hipLaunchKernelGGL(k_umap_scatter, dim3((unsigned)T), dim3(256), 0, s, (const double *)w.eps, w.next,
                                   nnz, t, (const uint32_t *)w.tile_off, w.pos, w.list, w.tile_cnt);
            }
            {
                ScopedTimer tt("umap_moves", s);
                const Moves mv{epoch_alpha(alpha0, t, n_epochs), a, b, b - 1.0, (-2.0 * a) * b, (2.0 * gamma) * b,
                               1.0 / (double)n, n, t, dim, 1 + neg, seed};
                if (dim <= 2)
                    hipLaunchKernelGGL(k_umap_epoch<2>, dim3(g_epoch), dim3(64), 0, s, indptr, (const uint32_t *)w.pos,
                                       (const uint32_t *)w.list, (const uint32_t *)w.erow, indices,
                                       (const double *)w.Y0, w.Y1, mv, (const crp::PowTables *)w.tables);
                else
                    hipLaunchKernelGGL(k_umap_epoch<kMaxDim>, dim3(g_epoch), dim3(64), 0, s, indptr,
                                       (const uint32_t *)w.pos, (const uint32_t *)w.list, (const uint32_t *)w.erow,
                                       indices, (const double *)w.Y0, w.Y1, mv, (const crp::PowTables *)w.tables);
            }
            std::swap(w.Y0, w.Y1);
        }
    }
    if ((st = launch_status("umap epochs")) != RSC_OK) return st;
    hipLaunchKernelGGL(k_umap_out, dim3(grid(ny)), dim3(256), 0, s, (const double *)w.Y0, ny, Y);
    return launch_status("umap output");
}

}  // namespace rsc
