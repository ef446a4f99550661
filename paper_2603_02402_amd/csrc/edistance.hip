// Energy distance between groups of cells (Methods, "Perturbation distance
// computation").
//
// For groups a, b of cells (rows of an embedding X) the path needs the sums
// of Euclidean distances
//   S[a, b] = sum_{i in a, j in b} ||x_i - x_j||       (a != b)
//   S[a, a] = sum_{i < j in a} ||x_i - x_j||           (upper triangle)
// from which mean distances d = S / pair count and the energy distances
// E[a, b] = 2 d[a, b] - d[a, a] - d[b, b] follow.  Groups are given the way
// the paper stores them: category offsets and a cell-index array (group g
// holds rows cells[offsets[g] .. offsets[g+1])).
//
// Work decomposition.  Every listed pair is cut into 64 x 64 tiles of
// (cells of a) x (cells of b); a diagonal pair keeps only the tiles on or
// above the diagonal.  The tiles of all pairs form one flat list (per-pair
// counts, exclusive scan), and the persistent grid splits that list into
// contiguous runs, so work is balanced whatever the group sizes.  Runs are
// dealt so that each XCD takes a contiguous stretch of the list: tiles of the
// same pair, which reuse the same rows, share an L2.
//
// Arithmetic.  A tile's dot products x_i . x_j run on the float64 matrix
// cores (v_mfma_f64_16x16x4_f64; the float32 inputs are exact in float64),
// the squared norms are float64 sums over the staged rows, and
//   ||x_i - x_j||^2 = (||x_i||^2 + ||x_j||^2) - 2 x_i . x_j
// is evaluated in float64 and clamped at 0 before a float64 square root
// (within 4 units of float64 roundoff: see root()).
// Its error is a few units of float64 roundoff of ||x_i||^2 + ||x_j||^2, so
// every distance is within sqrt of that of the exact one (and within that
// over twice the distance for distances that are not tiny).  On this chip
// the float64 matrix rate equals the float64 vector rate, and the product
// form needs half the operations of direct differences.
//
// Determinism.  Each tile's float64 partial sum is rounded to a per-pair
// fixed point (an int64 with scale 2^e_p chosen from an upper bound of the
// pair's sum, so nothing can overflow) and added with an integer atomic:
// integer addition is associative, so the sums do not depend on the order
// in which tiles finish.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include <rocprim/device/device_radix_sort.hpp>

#include "rsc_internal.hpp"

namespace rsc {
namespace {

constexpr int kWave = 64;
constexpr int kEdRows = 64;            // cells per side of a tile
constexpr int kEdK = 64;               // dimensions staged per pass
constexpr int kEdStride = kEdK + 1;    // LDS row stride (odd: conflict-free row reads)
constexpr int kEdThreads = 256;        // 4 waves, one 32 x 32 quadrant each
constexpr int kScanBlock = 1024;
constexpr int64_t kMaxGroups = 1 << 20;

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct EdArgs {
    const float *X;
    int64_t n;
    int d;
    const int64_t *goff;     // G + 1 group offsets into cells
    int64_t G;
    const int32_t *cells;
    const float *Xs;         // grouped rows: Xs[c] = X[cells[c]] (zero for an invalid id)
    const double *nrm;       // ||Xs[c]||^2 in float64, -1 for an invalid id
    const int32_t *pairs;    // npairs x (a, b)
    int64_t npairs;
    int64_t *tile_off;       // npairs + 1 exclusive prefix of tiles per pair
    int32_t *scale_exp;      // npairs fixed-point exponents
    unsigned long long *acc; // npairs fixed-point sums
    unsigned long long *max_norm2_bits;  // float64 bits of the largest squared norm
};

__device__ __forceinline__ int64_t group_size(const int64_t *goff, int64_t g) { return goff[g + 1] - goff[g]; }

__device__ __forceinline__ int64_t tiles_of(int64_t m) { return (m + kEdRows - 1) / kEdRows; }

// Number of distances behind a pair's sum (float64, as the means use it).
__device__ __forceinline__ double pair_count(double na, double nb, bool diag) {
    return diag ? na * (na - 1.0) / 2.0 : na * nb;
}

// acc = 0, largest squared norm = 0.
__global__ __launch_bounds__(256) void k_ed_zero(unsigned long long *__restrict__ acc, int64_t npairs,
                                                 unsigned long long *__restrict__ max_bits) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < npairs) acc[i] = 0ull;
    if (i == 0) *max_bits = 0ull;
}

// Rows of the grouped cells in group order, Xs[c] = X[cells[c]], with their
// squared norms (float64, dimensions in order) and the largest of them
// (non-negative doubles order like their bit patterns).  One wave per row
// block: lanes read consecutive floats of a row.
__global__ __launch_bounds__(256) void k_ed_gather(const float *__restrict__ X, int64_t n, int d,
                                                   const int32_t *__restrict__ cells, int64_t ncells,
                                                   float *__restrict__ Xs, double *__restrict__ nrm,
                                                   unsigned long long *__restrict__ max_bits) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / kWave;
    double m = 0.0;
    for (int64_t c = wave; c < ncells; c += nwaves) {
        const int32_t r = cells[c];
        const bool ok = r >= 0 && r < n;
        double s = 0.0;
        for (int t0 = 0; t0 < d; t0 += kWave) {
            const int t = t0 + lane;
            const float v = (ok && t < d) ? X[(int64_t)r * d + t] : 0.f;
            if (t < d) Xs[c * d + t] = v;
            double sq = (double)v * (double)v;
            for (int o = kWave / 2; o > 0; o >>= 1) sq += __shfl_xor(sq, o, kWave);
            s += sq;
        }
        if (lane == 0) nrm[c] = ok ? s : -1.0;
        m = fmax(m, s);
    }
    if (lane == 0) atomicMax(max_bits, (unsigned long long)__double_as_longlong(m));
}

// Per pair: tiles (into tile_off[p], scanned afterwards) and the fixed-point
// exponent: the pair's sum is at most count x (2 max ||x||), so with
// bound < 2^ex the scaled sum stays below 2^61.
__global__ __launch_bounds__(256) void k_ed_count(EdArgs a) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p == 0) a.tile_off[a.npairs] = 0;  // scanned with the rest: becomes the total
    if (p >= a.npairs) return;
    const int32_t ga = a.pairs[2 * p], gb = a.pairs[2 * p + 1];
    const int64_t na = group_size(a.goff, ga), nb = group_size(a.goff, gb);
    const bool diag = ga == gb;
    const int64_t ta = tiles_of(na), tb = tiles_of(nb);
    int64_t tiles = diag ? (na < 2 ? 0 : ta * (ta + 1) / 2) : ta * tb;
    a.tile_off[p] = tiles;
    const double maxn = sqrt(__longlong_as_double((long long)*a.max_norm2_bits));
    const double bound = pair_count((double)na, (double)nb, diag) * 2.0 * maxn * (1.0 + 1e-6);
    int ex = 0;
    if (bound > 0.0) frexp(bound, &ex);
    a.scale_exp[p] = bound > 0.0 ? 61 - ex : 0;
}

// Exclusive scan of v[0..m) in blocks of kScanBlock; block totals to bsum.
__global__ __launch_bounds__(kScanBlock) void k_scan_local(int64_t *__restrict__ v, int64_t m,
                                                           int64_t *__restrict__ bsum) {
    __shared__ int64_t s[kScanBlock];
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    const int64_t x = i < m ? v[i] : 0;
    s[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
        const int64_t t = (int)threadIdx.x >= o ? s[threadIdx.x - o] : 0;
        __syncthreads();
        s[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < m) v[i] = s[threadIdx.x] - x;
    if (threadIdx.x == kScanBlock - 1) bsum[blockIdx.x] = s[kScanBlock - 1];
}

// Exclusive scan of the block totals (one block; each thread a contiguous span).
__global__ __launch_bounds__(kScanBlock) void k_scan_totals(int64_t *__restrict__ bsum, int64_t nb,
                                                            int64_t *__restrict__ total) {
    __shared__ int64_t part[kScanBlock];
    const int64_t per = (nb + kScanBlock - 1) / kScanBlock;
    const int64_t lo = threadIdx.x * per, hi = std::min<int64_t>(nb, lo + per);
    int64_t s = 0;
    for (int64_t i = lo; i < hi; ++i) s += bsum[i];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < kScanBlock; o <<= 1) {
        const int64_t t = (int)threadIdx.x >= o ? part[threadIdx.x - o] : 0;
        __syncthreads();
        part[threadIdx.x] += t;
        __syncthreads();
    }
    int64_t run = part[threadIdx.x] - s;
    for (int64_t i = lo; i < hi; ++i) {
        const int64_t x = bsum[i];
        bsum[i] = run;
        run += x;
    }
    if (threadIdx.x == kScanBlock - 1) *total = part[kScanBlock - 1];
}

__global__ __launch_bounds__(kScanBlock) void k_scan_add(int64_t *__restrict__ v, int64_t m,
                                                         const int64_t *__restrict__ bsum) {
    const int64_t i = (int64_t)blockIdx.x * kScanBlock + threadIdx.x;
    if (i < m) v[i] += bsum[blockIdx.x];
}

// Row index ti of item r among the ta (ta + 1) / 2 upper-triangle tiles of
// a diagonal pair (row t holds ta - t tiles).
__device__ __forceinline__ int64_t tri_row(int64_t r, int64_t ta) {
    const double b = 2.0 * (double)ta + 1.0;
    int64_t t = (int64_t)((b - sqrt(fmax(b * b - 8.0 * (double)r, 0.0))) * 0.5);
    t = std::max<int64_t>(0, std::min<int64_t>(t, ta - 1));
    auto before = [ta](int64_t u) { return u * ta - u * (u - 1) / 2; };
    while (t > 0 && before(t) > r) --t;
    while (t + 1 < ta && before(t + 1) <= r) ++t;
    return t;
}

// Contiguous run of items [i0, i1) of block b.  Blocks go to the 8 XCDs
// round-robin; the renumbering gives each XCD a contiguous stretch of runs,
// so neighbouring tiles (which share rows) meet in the same L2.  gridDim.x
// is a multiple of 8.
__device__ __forceinline__ void block_run(int64_t total, int64_t &i0, int64_t &i1) {
    const int nblocks = gridDim.x;
    const int logical = (blockIdx.x % 8) * (nblocks / 8) + blockIdx.x / 8;
    const int64_t per = (total + nblocks - 1) / nblocks;
    i0 = std::min<int64_t>(total, (int64_t)logical * per);
    i1 = std::min<int64_t>(total, i0 + per);
}

// Dot products of one tile: rows ra0 .. ra0 + va - 1 (side a) and rb0 ..
// rb0 + vb - 1 (side b) of the grouped rows Xs, kEdK dimensions per pass
// through LDS (zero-padded).  Staging: waves 0, 1 copy rows 0..31, 32..63 of
// a, waves 2, 3 those of b; one load instruction covers two rows, 32 lanes
// per row.  Wave w accumulates quadrant (w / 2, w % 2) as 2 x 2 blocks of
// 16 x 16 float64 MFMA; the operands of step k + 4 are read from LDS before
// the MFMAs of step k are issued.  Every thread of the block calls this.
__device__ __forceinline__ void tile_dots(const EdArgs &a, int64_t ra0, int va, int64_t rb0, int vb, float *As,
                                          float *Bs, f64x4 &c00, f64x4 &c01, f64x4 &c10, f64x4 &c11) {
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
    c00 = f64x4{0.0, 0.0, 0.0, 0.0};
    c01 = c00;
    c10 = c00;
    c11 = c00;
    const int half = lane >> 5, kk = lane & 31;
    const int side = wave >> 1;  // wave-uniform
    const int rows_valid = side ? vb : va;
    const int row0 = (wave & 1) * 32 + half;  // this lane's first row; then + 2 u
    float *lds = (side ? Bs : As) + row0 * kEdStride + kk;
    for (int k0 = 0; k0 < a.d; k0 += kEdK) {
        const int w = std::min(kEdK, a.d - k0);
        const float *base = a.Xs + (side ? rb0 : ra0) * a.d + k0;  // wave-uniform
        float v[16];
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            const int k = pass * 32 + kk;
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int row = row0 + 2 * u;
                v[u] = (k < w && row < rows_valid) ? base[row * a.d + k] : 0.f;
            }
            if (pass == 0) __syncthreads();  // earlier reads of the LDS tiles are done
#pragma unroll
            for (int u = 0; u < 16; ++u) lds[2 * u * kEdStride + pass * 32] = v[u];
        }
        __syncthreads();
        const int w4 = (w + 3) & ~3;
        const float *pa0 = As + (wr * 32 + lr) * kEdStride + lk;
        const float *pa1 = pa0 + 16 * kEdStride;
        const float *pb0 = Bs + (wc * 32 + lr) * kEdStride + lk;
        const float *pb1 = pb0 + 16 * kEdStride;
        float fa0 = pa0[0], fa1 = pa1[0], fb0 = pb0[0], fb1 = pb1[0];
        for (int ks = 0; ks < w4; ks += 4) {
            const double a0 = (double)fa0, a1 = (double)fa1, b0 = (double)fb0, b1 = (double)fb1;
            const int kn = ks + 4 < w4 ? ks + 4 : ks;
            fa0 = pa0[kn];
            fa1 = pa1[kn];
            fb0 = pb0[kn];
            fb1 = pb1[kn];
            c00 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b0, c00, 0, 0, 0);
            c01 = __builtin_amdgcn_mfma_f64_16x16x4f64(a0, b1, c01, 0, 0, 0);
            c10 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b0, c10, 0, 0, 0);
            c11 = __builtin_amdgcn_mfma_f64_16x16x4f64(a1, b1, c11, 0, 0, 0);
        }
    }
}

// Square root for the distances: a float32 reciprocal-root seed (relative
// error below 2^-23) refined by two float64 Newton steps on 1/sqrt(x), so the
// result is within a few units of float64 roundoff; far outside the float32
// range (where the seed would under- or overflow) the correctly rounded
// square root instead.  Uses fewer float64 operations than the correctly
// rounded routine, and float64 vector work competes with the float64 MFMAs.
__device__ __forceinline__ double root(double x) {
    if (__builtin_expect(x > 1e-30 && x < 1e30, 1)) {
        double y = (double)__frsqrt_rn((float)x);
        y = y * (1.5 - 0.5 * x * y * y);
        y = y * (1.5 - 0.5 * x * y * y);
        return x * y;
    }
    return sqrt(x);
}

// Distances of the 16 output elements of this lane: element e = 4 (2 bi +
// bj) + q of block (bi, bj) is row 32 wr + 16 bi + 4 q + lk, column 32 wc +
// 16 bj + lr (operands: lane l gives A[l % 16][l / 16] and B[l / 16][l % 16],
// output register q holds row 4 q + l / 16, column l % 16).  Invalid
// elements (a negative norm marks a missing row) and, on a diagonal tile,
// elements on or below the diagonal give 0.
__device__ __forceinline__ void tile_distances(const f64x4 (&c)[4], const double *An, const double *Bn, bool diag,
                                               double (&dv)[16]) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
        const int bi = blk >> 1, bj = blk & 1;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int i = wr * 32 + bi * 16 + 4 * q + lk;
            const int j = wc * 32 + bj * 16 + lr;
            const bool valid = An[i] >= 0.0 && Bn[j] >= 0.0 && (!diag || i < j);
            const double d2 = (An[i] + Bn[j]) - 2.0 * c[blk][q];
            dv[4 * blk + q] = valid ? root(fmax(d2, 0.0)) : 0.0;
        }
    }
}

// Block sum of one value per thread (4 waves); every thread gets the total.
__device__ __forceinline__ double block_sum4(double s, double *red) {
    for (int o = kWave / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, kWave);
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x >> 6;
    if (lane == 0) red[wave] = s;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// Listed pairs.  Persistent: block b takes a contiguous run of the flat tile
// list (tile_off); per tile the dot products, then the distances summed and
// the tile's total added to its pair in fixed point.
__global__ __launch_bounds__(kEdThreads, 4) void k_ed_tiles(EdArgs a) {
    __shared__ float As[kEdRows * kEdStride];
    __shared__ float Bs[kEdRows * kEdStride];
    __shared__ double An[kEdRows], Bn[kEdRows];
    __shared__ double red[kEdThreads / kWave];
    const int tid = threadIdx.x;

    int64_t i0, i1;
    block_run(a.tile_off[a.npairs], i0, i1);
    if (i0 >= i1) return;
    // pair of the first item: last p with tile_off[p] <= i0
    int64_t lo = 0, hi = a.npairs - 1;
    while (lo < hi) {
        const int64_t mid = (lo + hi + 1) / 2;
        if (a.tile_off[mid] <= i0) lo = mid; else hi = mid - 1;
    }
    int64_t p = lo;

    for (int64_t item = i0; item < i1; ++item) {
        while (a.tile_off[p + 1] <= item) ++p;
        const int32_t ga = a.pairs[2 * p], gb = a.pairs[2 * p + 1];
        const int64_t oa = a.goff[ga], na = a.goff[ga + 1] - oa;
        const int64_t ob = a.goff[gb], nb = a.goff[gb + 1] - ob;
        const bool diag = ga == gb;
        const int64_t r = item - a.tile_off[p];
        int64_t ti, tj;
        if (diag) {
            const int64_t ta = tiles_of(na);
            ti = tri_row(r, ta);
            tj = ti + (r - (ti * ta - ti * (ti - 1) / 2));
        } else {
            const int64_t tb = tiles_of(nb);
            ti = r / tb;
            tj = r - ti * tb;
        }
        const int64_t ra0 = oa + ti * kEdRows, rb0 = ob + tj * kEdRows;  // first grouped row of each side
        const int va = (int)std::min<int64_t>(kEdRows, na - ti * kEdRows);  // valid rows of each side
        const int vb = (int)std::min<int64_t>(kEdRows, nb - tj * kEdRows);
        // (the previous tile's reads of An / Bn ended at its block_sum4 barrier)
        if (tid < 2 * kEdRows) {
            const int side = tid / kEdRows, row = tid % kEdRows;
            (side ? Bn : An)[row] = row < (side ? vb : va) ? a.nrm[(side ? rb0 : ra0) + row] : -1.0;
        }
        f64x4 c[4];
        tile_dots(a, ra0, va, rb0, vb, As, Bs, c[0], c[1], c[2], c[3]);
        double dv[16];
        tile_distances(c, An, Bn, diag && ti == tj, dv);
        double sum = 0.0;
#pragma unroll
        for (int e = 0; e < 16; ++e) sum += dv[e];
        const double t = block_sum4(sum, red);
        if (tid == 0) atomicAdd(&a.acc[p], (unsigned long long)llrint(ldexp(t, a.scale_exp[p])));
        __syncthreads();  // red is reused by the next tile
    }
}

// Index of pair (a, b), a <= b, in the row-major list of all pairs.
__device__ __forceinline__ int64_t all_pairs_index(int64_t a, int64_t b, int64_t G) {
    const int64_t lo = a < b ? a : b, hi = a < b ? b : a;
    return lo * G - lo * (lo - 1) / 2 + (hi - lo);
}

// Group of every grouped position (binary search in the offsets).
__global__ __launch_bounds__(256) void k_ed_group_of(const int64_t *__restrict__ goff, int64_t G, int64_t ncells,
                                                     int32_t *__restrict__ grp) {
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncells;
         c += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = G - 1;  // last g with goff[g] <= c
        while (lo < hi) {
            const int64_t mid = (lo + hi + 1) / 2;
            if (goff[mid] <= c) lo = mid; else hi = mid - 1;
        }
        grp[c] = (int32_t)lo;
    }
}

constexpr int kBins = 4;  // group segments per tile side handled by the binned sum

// The full matrix.  Every pair of grouped positions i < j (the cells in group
// order) is one distance of exactly one pair sum: (group(i), group(j)), the
// upper triangle for a group with itself.  So the upper triangle of the
// ncells x ncells matrix is cut into 64 x 64 tiles with no padding between
// groups.  A tile spans a few groups on each side (contiguous position
// ranges); its distances are summed per (row group, column group) bin and
// each bin added to its pair.  A tile with more than kBins groups on a side
// adds every distance to its pair on its own.
__global__ __launch_bounds__(kEdThreads, 4) void k_ed_matrix(EdArgs a, const int32_t *__restrict__ grp,
                                                             int64_t ncells) {
    __shared__ float As[kEdRows * kEdStride];
    __shared__ float Bs[kEdRows * kEdStride];
    __shared__ double An[kEdRows], Bn[kEdRows];
    __shared__ int32_t Ag[kEdRows], Bg[kEdRows];
    __shared__ double red[kEdThreads / kWave][kBins * kBins];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int lr = lane & 15, lk = lane >> 4;

    const int64_t T = tiles_of(ncells);
    int64_t i0, i1;
    block_run(T * (T + 1) / 2, i0, i1);
    for (int64_t item = i0; item < i1; ++item) {
        const int64_t ti = tri_row(item, T);
        const int64_t tj = ti + (item - (ti * T - ti * (ti - 1) / 2));
        const int64_t ra0 = ti * kEdRows, rb0 = tj * kEdRows;
        const int va = (int)std::min<int64_t>(kEdRows, ncells - ra0);
        const int vb = (int)std::min<int64_t>(kEdRows, ncells - rb0);
        if (tid < 2 * kEdRows) {
            const int side = tid / kEdRows, row = tid % kEdRows;
            const bool ok = row < (side ? vb : va);
            const int64_t pos = (side ? rb0 : ra0) + row;
            (side ? Bn : An)[row] = ok ? a.nrm[pos] : -1.0;
            (side ? Bg : Ag)[row] = ok ? grp[pos] : 0;
        }
        f64x4 c[4];
        tile_dots(a, ra0, va, rb0, vb, As, Bs, c[0], c[1], c[2], c[3]);  // (its barriers publish An, Ag)
        double dv[16];
        tile_distances(c, An, Bn, ti == tj, dv);
        const int g0r = Ag[0], g0c = Bg[0];
        const int nsr = Ag[va - 1] - g0r + 1, nsc = Bg[vb - 1] - g0c + 1;  // groups spanned (block-uniform)
        if (nsr <= kBins && nsc <= kBins) {
            int rs[8], cs[2];
#pragma unroll
            for (int u = 0; u < 8; ++u) rs[u] = Ag[wr * 32 + (u >> 2) * 16 + 4 * (u & 3) + lk] - g0r;
#pragma unroll
            for (int u = 0; u < 2; ++u) cs[u] = Bg[wc * 32 + u * 16 + lr] - g0c;
            // per row group: the lane's two column partials (its columns 16 bj + lr),
            // then one select per column and bin before the wave sum
            for (int sr = 0; sr < nsr; ++sr) {
                double p0 = 0.0, p1 = 0.0;
#pragma unroll
                for (int e = 0; e < 16; ++e) {
                    const int blk = e >> 2, q = e & 3;
                    const double v = rs[(blk >> 1) * 4 + q] == sr ? dv[e] : 0.0;
                    if (blk & 1) p1 += v; else p0 += v;
                }
                for (int sc = 0; sc < nsc; ++sc) {
                    double sum = (cs[0] == sc ? p0 : 0.0) + (cs[1] == sc ? p1 : 0.0);
                    for (int o = kWave / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, kWave);
                    if (lane == 0) red[wave][sr * kBins + sc] = sum;
                }
            }
            __syncthreads();
            if (tid < nsr * nsc) {
                const int sr = tid / nsc, sc = tid % nsc;
                const int b = sr * kBins + sc;
                const double t = (red[0][b] + red[1][b]) + (red[2][b] + red[3][b]);
                const int64_t pi = all_pairs_index(g0r + sr, g0c + sc, a.G);
                if (t != 0.0) atomicAdd(&a.acc[pi], (unsigned long long)llrint(ldexp(t, a.scale_exp[pi])));
            }
        } else {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                const int blk = e >> 2, q = e & 3;
                const int i = wr * 32 + (blk >> 1) * 16 + 4 * q + lk, j = wc * 32 + (blk & 1) * 16 + lr;
                if (dv[e] != 0.0) {
                    const int64_t pi = all_pairs_index(Ag[i], Bg[j], a.G);
                    atomicAdd(&a.acc[pi], (unsigned long long)llrint(ldexp(dv[e], a.scale_exp[pi])));
                }
            }
        }
        __syncthreads();  // LDS (norms, groups, bins) is reused by the next tile
    }
}

__global__ __launch_bounds__(256) void k_ed_finalize(const unsigned long long *__restrict__ acc,
                                                     const int32_t *__restrict__ scale_exp, int64_t npairs,
                                                     double *__restrict__ sums) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < npairs) sums[p] = ldexp((double)(long long)acc[p], -scale_exp[p]);
}

// Pair list of the full matrix: (a, b), a <= b, row-major.
__global__ __launch_bounds__(256) void k_ed_pairs_all(int64_t G, int32_t *__restrict__ pairs) {
    const int64_t a = blockIdx.y;
    for (int64_t b = a + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < G; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t p = a * G - a * (a - 1) / 2 + (b - a);
        pairs[2 * p] = (int32_t)a;
        pairs[2 * p + 1] = (int32_t)b;
    }
}

// Pair list of a one-sided query: (ref, g) for every g, then (g, g) for g != ref.
__global__ __launch_bounds__(256) void k_ed_pairs_onesided(int64_t G, int64_t ref, int32_t *__restrict__ pairs) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    pairs[2 * g] = (int32_t)ref;
    pairs[2 * g + 1] = (int32_t)g;
    if (g != ref) {
        const int64_t p = G + (g < ref ? g : g - 1);
        pairs[2 * p] = (int32_t)g;
        pairs[2 * p + 1] = (int32_t)g;
    }
}

// Mean distance of a pair: the within mean of a group with fewer than two
// cells is 0 (skipped), a cross mean with an empty group is NaN.
__device__ __forceinline__ double pair_mean(double s, int64_t na, int64_t nb, bool diag) {
    const double cnt = pair_count((double)na, (double)nb, diag);
    if (cnt == 0.0) return diag ? 0.0 : __longlong_as_double(0x7ff8000000000000ll);
    return s / cnt;
}

// E (and D) of the full matrix from the pair sums.
__global__ __launch_bounds__(256) void k_ed_assemble_all(const int64_t *__restrict__ goff, int64_t G,
                                                         const double *__restrict__ sums, double *__restrict__ E,
                                                         double *__restrict__ D) {
    const int64_t a = blockIdx.y;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b < G; b += (int64_t)gridDim.x * blockDim.x) {
        const int64_t na = group_size(goff, a), nb = group_size(goff, b);
        const double m = pair_mean(sums[all_pairs_index(a, b, G)], na, nb, a == b);
        const double da = pair_mean(sums[all_pairs_index(a, a, G)], na, na, true);
        const double db = pair_mean(sums[all_pairs_index(b, b, G)], nb, nb, true);
        E[a * G + b] = 2.0 * m - (da + db);
        if (D) D[a * G + b] = m;
    }
}

// E(ref, g) for every g from the one-sided pair sums.
__global__ __launch_bounds__(256) void k_ed_assemble_onesided(const int64_t *__restrict__ goff, int64_t G,
                                                              int64_t ref, const double *__restrict__ sums,
                                                              double *__restrict__ E) {
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= G) return;
    const int64_t nr = group_size(goff, ref), ng = group_size(goff, g);
    const double cross = pair_mean(sums[g], nr, ng, g == ref);
    const double wref = pair_mean(sums[ref], nr, nr, true);
    const double wg = g == ref ? wref : pair_mean(sums[G + (g < ref ? g : g - 1)], ng, ng, true);
    E[g] = 2.0 * cross - (wg + wref);
}

struct EdBuffers {
    int64_t *goff;
    int32_t *pairs;
    int64_t *tile_off;
    int32_t *scale_exp;
    unsigned long long *acc;
    unsigned long long *max_bits;
    int64_t *bsum;
    float *Xs;     // grouped rows
    double *nrm;   // their squared norms
    int32_t *grp;  // group of every grouped position (full-matrix form)
    double *sums;  // pair sums (only for the matrix / one-sided calls)
};

int64_t scan_blocks(int64_t m) { return (m + kScanBlock - 1) / kScanBlock; }

size_t carve(int64_t G, int64_t npairs, int64_t ncells, int d, bool own_sums, void *ws, EdBuffers *out) {
    Carver cv(ws);
    EdBuffers b{};
    b.goff = cv.take<int64_t>((size_t)G + 1);
    b.pairs = cv.take<int32_t>((size_t)std::max<int64_t>(npairs, 1) * 2);
    b.tile_off = cv.take<int64_t>((size_t)npairs + 1);
    b.scale_exp = cv.take<int32_t>((size_t)std::max<int64_t>(npairs, 1));
    b.acc = cv.take<unsigned long long>((size_t)std::max<int64_t>(npairs, 1));
    b.max_bits = cv.take<unsigned long long>(1);
    b.bsum = cv.take<int64_t>((size_t)scan_blocks(npairs + 1) + 1);
    b.Xs = cv.take<float>((size_t)std::max<int64_t>(ncells, 1) * d);
    b.nrm = cv.take<double>((size_t)std::max<int64_t>(ncells, 1));
    b.grp = cv.take<int32_t>((size_t)std::max<int64_t>(ncells, 1));
    b.sums = own_sums ? cv.take<double>((size_t)std::max<int64_t>(npairs, 1)) : nullptr;
    if (out) *out = b;
    return cv.used;
}

int check_groups(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G, const int32_t *cells) {
    if (!X || !offsets || !cells) {
        set_error("edistance: null X, offsets or cells");
        return RSC_ERR_INVALID_ARG;
    }
    if (n < 1 || d < 1 || G < 1 || G > kMaxGroups) {
        set_error("edistance: need n >= 1, d >= 1 and 1 <= G <= 2^20 groups");
        return RSC_ERR_INVALID_ARG;
    }
    if (offsets[0] != 0) {
        set_error("edistance: offsets[0] must be 0");
        return RSC_ERR_INVALID_ARG;
    }
    for (int64_t g = 0; g < G; ++g)
        if (offsets[g + 1] < offsets[g]) {
            set_error("edistance: offsets must be non-decreasing");
            return RSC_ERR_INVALID_ARG;
        }
    if (offsets[G] > (int64_t)1 << 31) {
        set_error("edistance: more than 2^31 grouped cells");
        return RSC_ERR_INVALID_ARG;
    }
    return RSC_OK;
}

int grid_blocks() {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
            cus = 256;
    }
    // 4 resident tiles per CU (LDS-limited), a multiple of the 8 XCDs
    return ((cus * 4 + 7) / 8) * 8;
}

// The shared core: sums of the pairs already in b.pairs (device).
// With `matrix`, b.pairs is the row-major list of all pairs and the sums come
// from the full-matrix tiling; otherwise from the per-pair tiles.
int run_sums(const float *X, int64_t n, int d, int64_t G, int64_t ncells, const int32_t *cells, int64_t npairs,
             const EdBuffers &b, double *sums, bool matrix, hipStream_t s) {
    EdArgs a{};
    a.X = X;
    a.n = n;
    a.d = d;
    a.goff = b.goff;
    a.G = G;
    a.cells = cells;
    a.Xs = b.Xs;
    a.nrm = b.nrm;
    a.pairs = b.pairs;
    a.npairs = npairs;
    a.tile_off = b.tile_off;
    a.scale_exp = b.scale_exp;
    a.acc = b.acc;
    a.max_norm2_bits = b.max_bits;
    const unsigned pg = (unsigned)std::max<int64_t>(1, (npairs + 255) / 256);
    hipLaunchKernelGGL(k_ed_zero, dim3(pg), dim3(256), 0, s, b.acc, npairs, b.max_bits);
    {
        ScopedTimer t("ed_plan", s);
        const unsigned cg = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (ncells + 3) / 4));
        hipLaunchKernelGGL(k_ed_gather, dim3(cg), dim3(256), 0, s, X, n, d, cells, ncells, b.Xs, b.nrm, b.max_bits);
        hipLaunchKernelGGL(k_ed_count, dim3(pg), dim3(256), 0, s, a);
        if (matrix) {
            const unsigned gg = (unsigned)std::min<int64_t>(4096, std::max<int64_t>(1, (ncells + 255) / 256));
            hipLaunchKernelGGL(k_ed_group_of, dim3(gg), dim3(256), 0, s, b.goff, G, ncells, b.grp);
        }
    }
    if (!matrix) {
        ScopedTimer t("ed_plan", s);
        // exclusive scan of npairs + 1 entries (the last one is 0 and becomes the total)
        const int64_t m = npairs + 1;
        const int64_t nb = scan_blocks(m);
        hipLaunchKernelGGL(k_scan_local, dim3((unsigned)nb), dim3(kScanBlock), 0, s, b.tile_off, m, b.bsum);
        hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanBlock), 0, s, b.bsum, nb, b.bsum + nb);
        hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nb), dim3(kScanBlock), 0, s, b.tile_off, m, b.bsum);
    }
    int st;
    if ((st = launch_status("edistance plan")) != RSC_OK) return st;
    {
        ScopedTimer t("ed_tiles", s);
        if (matrix)
            hipLaunchKernelGGL(k_ed_matrix, dim3((unsigned)grid_blocks()), dim3(kEdThreads), 0, s, a,
                               (const int32_t *)b.grp, ncells);
        else
            hipLaunchKernelGGL(k_ed_tiles, dim3((unsigned)grid_blocks()), dim3(kEdThreads), 0, s, a);
    }
    if ((st = launch_status("edistance tiles")) != RSC_OK) return st;
    hipLaunchKernelGGL(k_ed_finalize, dim3(pg), dim3(256), 0, s, b.acc, b.scale_exp, npairs, sums);
    return launch_status("edistance finalize");
}

int upload_offsets(const int64_t *offsets, int64_t G, const EdBuffers &b, hipStream_t s) {
    return hip_status(hipMemcpyAsync(b.goff, offsets, (size_t)(G + 1) * sizeof(int64_t), hipMemcpyHostToDevice, s),
                      "upload group offsets");
}

bool sizes_ok(int64_t G, int64_t ncells, int d) { return G >= 1 && G <= kMaxGroups && ncells >= 0 && d >= 1; }

// ---- the group layout of integer labels -----------------------------------

__global__ void k_ed_clear_flag(int32_t *flag) { *flag = 0; }

__global__ __launch_bounds__(256) void k_ed_iota_check(const int32_t *__restrict__ labels, int64_t n, int64_t G,
                                                       int32_t *__restrict__ rows, int32_t *__restrict__ err) {
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x) {
        rows[r] = (int32_t)r;
        if (labels[r] < 0 || labels[r] >= G) atomicOr(err, 1);
    }
}

// offsets[g] = number of sorted labels below g, for g = 0 .. G.
__global__ __launch_bounds__(256) void k_ed_offsets(const uint32_t *__restrict__ sorted, int64_t n, int64_t G,
                                                    int64_t *__restrict__ offsets) {
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g <= G; g += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = n;  // first index with sorted[i] >= g
        while (lo < hi) {
            const int64_t mid = (lo + hi) / 2;
            if ((int64_t)sorted[mid] < g) lo = mid + 1; else hi = mid;
        }
        offsets[g] = lo;
    }
}

int radix_bits(int64_t G) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < G) ++b;
    return b;
}

size_t groups_sort_bytes(int64_t n, int64_t G) {
    size_t bytes = 0;
    if (rocprim::radix_sort_pairs(nullptr, bytes, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                  (const int32_t *)nullptr, (int32_t *)nullptr, (unsigned)n, 0, radix_bits(G),
                                  (hipStream_t)0) != hipSuccess)
        return 0;
    return bytes;
}

}  // namespace

size_t edistance_groups_workspace_bytes(int64_t n, int64_t G) {
    if (n < 1 || n > INT32_MAX || G < 1 || G > kMaxGroups) return 0;
    const size_t sort = groups_sort_bytes(n, G);
    if (sort == 0) return 0;
    Carver cv(nullptr);
    cv.take<int32_t>((size_t)n);   // row ids
    cv.take<uint32_t>((size_t)n);  // sorted labels
    cv.take<int32_t>(1);           // error flag
    cv.take<char>(sort);
    return cv.used;
}

int edistance_groups(const int32_t *labels, int64_t n, int64_t G, int64_t *offsets, int32_t *cells, void *ws,
                     size_t ws_bytes, hipStream_t s) {
    if (!labels || !offsets || !cells || n < 1 || n > INT32_MAX || G < 1 || G > kMaxGroups) {
        set_error("edistance_groups: null argument, or n outside [1, 2^31) or G outside [1, 2^20]");
        return RSC_ERR_INVALID_ARG;
    }
    size_t sort = groups_sort_bytes(n, G);
    Carver cv(ws);
    int32_t *rows = cv.take<int32_t>((size_t)n);
    uint32_t *keys = cv.take<uint32_t>((size_t)n);
    int32_t *err = cv.take<int32_t>(1);
    char *tmp = cv.take<char>(sort);
    if (sort == 0 || !ws || cv.used > ws_bytes) {
        set_error("edistance_groups: workspace too small");
        return RSC_ERR_WORKSPACE;
    }
    const unsigned g = (unsigned)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_ed_clear_flag, dim3(1), dim3(1), 0, s, err);
    hipLaunchKernelGGL(k_ed_iota_check, dim3(g), dim3(256), 0, s, labels, n, G, rows, err);
    int st;
    if ((st = launch_status("edistance groups")) != RSC_OK) return st;
    // stable: the cells of a group keep ascending row order
    if ((st = hip_status(rocprim::radix_sort_pairs(tmp, sort, reinterpret_cast<const uint32_t *>(labels), keys,
                                                   (const int32_t *)rows, cells, (unsigned)n, 0, radix_bits(G), s),
                         "radix sort of the labels")) != RSC_OK)
        return st;
    const unsigned go = (unsigned)std::min<int64_t>(4096, (G + 1 + 255) / 256);
    hipLaunchKernelGGL(k_ed_offsets, dim3(go), dim3(256), 0, s, keys, n, G, offsets);
    if ((st = launch_status("edistance group offsets")) != RSC_OK) return st;
    int32_t host_err = 0;
    if ((st = hip_status(hipMemcpyAsync(&host_err, err, 4, hipMemcpyDeviceToHost, s), "read check")) != RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (host_err) {
        set_error("edistance_groups: a label outside [0, G)");
        return RSC_ERR_INVALID_ARG;
    }
    return RSC_OK;
}

size_t edistance_sums_workspace_bytes(int64_t G, int64_t npairs, int64_t ncells, int d) {
    if (!sizes_ok(G, ncells, d) || npairs < 1) return 0;
    return carve(G, npairs, ncells, d, false, nullptr, nullptr);
}

size_t edistance_pairwise_workspace_bytes(int64_t G, int64_t ncells, int d) {
    if (!sizes_ok(G, ncells, d)) return 0;
    return carve(G, G * (G + 1) / 2, ncells, d, true, nullptr, nullptr);
}

size_t edistance_onesided_workspace_bytes(int64_t G, int64_t ncells, int d) {
    if (!sizes_ok(G, ncells, d)) return 0;
    return carve(G, 2 * G - 1, ncells, d, true, nullptr, nullptr);
}

int edistance_sums(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G, const int32_t *cells,
                   const int32_t *pairs, int64_t npairs, double *sums, void *ws, size_t ws_bytes, hipStream_t s) {
    int st;
    if ((st = check_groups(X, n, d, offsets, G, cells)) != RSC_OK) return st;
    if (!pairs || !sums || npairs < 1) {
        set_error("edistance_sums: need a host pair list of npairs >= 1 and a device output");
        return RSC_ERR_INVALID_ARG;
    }
    for (int64_t p = 0; p < npairs; ++p)
        if (pairs[2 * p] < 0 || pairs[2 * p] >= G || pairs[2 * p + 1] < 0 || pairs[2 * p + 1] >= G) {
            set_error("edistance_sums: group id out of range in the pair list");
            return RSC_ERR_INVALID_ARG;
        }
    const size_t need = carve(G, npairs, offsets[G], d, false, nullptr, nullptr);
    if (!ws || ws_bytes < need) {
        set_error("edistance_sums: workspace too small");
        return RSC_ERR_WORKSPACE;
    }
    EdBuffers b;
    carve(G, npairs, offsets[G], d, false, ws, &b);
    if ((st = upload_offsets(offsets, G, b, s)) != RSC_OK) return st;
    if ((st = hip_status(hipMemcpyAsync(b.pairs, pairs, (size_t)npairs * 2 * sizeof(int32_t), hipMemcpyHostToDevice,
                                        s), "upload pairs")) != RSC_OK)
        return st;
    return run_sums(X, n, d, G, offsets[G], cells, npairs, b, sums, false, s);
}

int edistance_pairwise(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G, const int32_t *cells,
                       double *E, double *D, void *ws, size_t ws_bytes, hipStream_t s) {
    int st;
    if ((st = check_groups(X, n, d, offsets, G, cells)) != RSC_OK) return st;
    if (!E) {
        set_error("edistance_pairwise: null E");
        return RSC_ERR_INVALID_ARG;
    }
    const int64_t npairs = G * (G + 1) / 2;
    const size_t need = carve(G, npairs, offsets[G], d, true, nullptr, nullptr);
    if (!ws || ws_bytes < need) {
        set_error("edistance_pairwise: workspace too small");
        return RSC_ERR_WORKSPACE;
    }
    EdBuffers b;
    carve(G, npairs, offsets[G], d, true, ws, &b);
    if ((st = upload_offsets(offsets, G, b, s)) != RSC_OK) return st;
    const unsigned gx = (unsigned)std::min<int64_t>(64, (G + 255) / 256);
    hipLaunchKernelGGL(k_ed_pairs_all, dim3(gx, (unsigned)G), dim3(256), 0, s, G, b.pairs);
    if ((st = launch_status("edistance pair list")) != RSC_OK) return st;
    if ((st = run_sums(X, n, d, G, offsets[G], cells, npairs, b, b.sums, true, s)) != RSC_OK) return st;
    hipLaunchKernelGGL(k_ed_assemble_all, dim3(gx, (unsigned)G), dim3(256), 0, s, b.goff, G, b.sums, E, D);
    return launch_status("edistance assemble");
}

int edistance_onesided(const float *X, int64_t n, int d, const int64_t *offsets, int64_t G, const int32_t *cells,
                       int64_t ref, double *E, void *ws, size_t ws_bytes, hipStream_t s) {
    int st;
    if ((st = check_groups(X, n, d, offsets, G, cells)) != RSC_OK) return st;
    if (!E || ref < 0 || ref >= G) {
        set_error("edistance_onesided: null E or reference group out of range");
        return RSC_ERR_INVALID_ARG;
    }
    const int64_t npairs = 2 * G - 1;
    const size_t need = carve(G, npairs, offsets[G], d, true, nullptr, nullptr);
    if (!ws || ws_bytes < need) {
        set_error("edistance_onesided: workspace too small");
        return RSC_ERR_WORKSPACE;
    }
    EdBuffers b;
    carve(G, npairs, offsets[G], d, true, ws, &b);
    if ((st = upload_offsets(offsets, G, b, s)) != RSC_OK) return st;
    const unsigned g1 = (unsigned)((G + 255) / 256);
    hipLaunchKernelGGL(k_ed_pairs_onesided, dim3(g1), dim3(256), 0, s, G, ref, b.pairs);
    if ((st = launch_status("edistance pair list")) != RSC_OK) return st;
    if ((st = run_sums(X, n, d, G, offsets[G], cells, npairs, b, b.sums, false, s)) != RSC_OK) return st;
    hipLaunchKernelGGL(k_ed_assemble_onesided, dim3(g1), dim3(256), 0, s, b.goff, G, ref, b.sums, E);
    return launch_status("edistance assemble");
}

}  // namespace rsc
