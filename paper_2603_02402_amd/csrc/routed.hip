// Probed and routed kNN: each query is compared with the cells of the
// partitions it probes, on the same FP32 MFMA screen, float64 rerank and
// certificate as the exact path, and rows that are marked (or whose screen
// cannot be certified inside their partitions) are answered by the exact
// path over all cells.
//
// Layout.  The cells are packed once in partition order: partition p owns
// the 32-row blocks [pblk[p], pblk[p+1]) of one packed array (its last block
// padded), and map[] turns a packed row back into a cell id.
//
// Work.  Probed queries are grouped by their own partition (cells of one
// partition probe nearly the same partitions) and cut into tiles of 32
// queries.  A persistent grid pops tiles from an atomic counter; a wave
// builds the union of its 32 queries' probe lists as a bitmap in LDS, walks
// the union's partitions in ascending order and streams their blocks through
// the MFMA chain once for all 32 queries.  Each lane walks its own query's
// sorted probe list alongside, and keys of partitions the query did not
// probe are dropped before selection, so a query's answer is exactly the
// nearest cells among its own probed partitions, whatever tile it lands in.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <string>

#include "morton.hpp"
#include "rsc_internal.hpp"
#include "screen_common.hpp"
#include "screen_fp32.hpp"

namespace rsc {
namespace {

using namespace scr;

constexpr int kMaxParts = 8192;   // partitions of a probed search (LDS bitmap of 1 KiB)
constexpr int kMaxProbes = 64;    // probes per query (one per lane when sorting)
constexpr int kTileQ = 32;        // queries per tile (one wave)
constexpr int kBitmapWords = kMaxParts / 32;
constexpr int64_t kExactSlack = 131072;  // see exact_plan

struct RoutedCounters {
    int32_t nconf;      // probed rows
    int32_t nfall;      // rows on the exact list
    int32_t nmark;      // marked rows (the first entries of the exact list)
    int32_t ntiles;
    int32_t tile_next;  // persistent-grid work counter
    int32_t bad;        // malformed partitions or probe lists
    int32_t pad[2];
    unsigned long long probed_cells;    // candidates over all probed rows
    unsigned long long screened_cells;  // rows streamed past each probed query (its tile's union)
};

struct RoutedBuffers {
    RoutedCounters *rc;
    KnnCounters *kc;
    float *nrow;
    int64_t *pblk;
    int32_t *map;
    float *packed, *norms;
    int32_t *own, *probes, *ccount, *cursor, *qperm, *fall;
    int64_t *coff, *toff;
    int2 *tiles;
    int32_t *cand_idx;
    float *cand_key;
    uint8_t *route;
    void *exact_ws;
    size_t exact_bytes;
};

int pick_dh_local(int d) {
    const int half = (d + 1) / 2;
    const int opts[] = {4, 8, 16, 25, 32, 48, 64};
    for (int o : opts)
        if (half <= o) return o;
    return -1;
}

// The exact search over the list of F rows: the plan of rsc_knn restricted to
// the list.  Its workspace is bounded for every F <= n by the plan with
// n + kExactSlack queries and one reference range (the range count of the
// exact path is at most ceil(1024 / ceil(F / 128)), so F times it stays below
// F + 131072).
int exact_plan(int64_t F, int64_t n, int d, int k, KnnPlan *p) { return knn_plan(F, n, d, k, nullptr, true, p); }

size_t exact_bound_bytes(int64_t n, int d, int k) {
    KnnPlan p;
    if (exact_plan(n, n, d, k, &p) != RSC_OK) return 0;
    p.nq = n + kExactSlack;
    p.splits = 1;
    return knn_workspace(p, nullptr, nullptr);
}

size_t carve_probed(int64_t n, int d, int k, int P, int probes, void *ws, RoutedBuffers *out) {
    const int dh = pick_dh_local(d);
    if (dh < 0) return 0;
    const int64_t nblk = n / 32 + P;  // >= sum over partitions of ceil(size / 32)
    const int screen_w = k <= 16 ? 32 : 64;
    Carver cv(ws);
    RoutedBuffers b;
    b.rc = cv.take<RoutedCounters>(1);
    b.kc = cv.take<KnnCounters>(1);
    b.nrow = cv.take<float>(n);
    b.pblk = cv.take<int64_t>(P + 1);
    b.map = cv.take<int32_t>((size_t)nblk * 32);
    b.packed = cv.take<float>(knn_packed_floats(dh, nblk));
    b.norms = cv.take<float>((size_t)nblk * 32);
    b.own = cv.take<int32_t>(n);
    b.probes = cv.take<int32_t>((size_t)n * probes);
    b.ccount = cv.take<int32_t>(P);
    b.cursor = cv.take<int32_t>(P);
    b.qperm = cv.take<int32_t>(n);
    b.fall = cv.take<int32_t>(n);
    b.coff = cv.take<int64_t>(P + 1);
    b.toff = cv.take<int64_t>(P + 1);
    b.tiles = cv.take<int2>((size_t)(n / kTileQ + P));
    b.cand_idx = cv.take<int32_t>((size_t)n * screen_w);
    b.cand_key = cv.take<float>((size_t)n * screen_w);
    b.route = cv.take<uint8_t>(n);
    b.exact_bytes = exact_bound_bytes(n, d, k);
    if (b.exact_bytes == 0) return 0;
    b.exact_ws = cv.take<char>(b.exact_bytes);
    if (out) *out = b;
    return cv.used;
}

unsigned grid_for(int64_t work) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 16384)); }

__global__ void k_routed_init(RoutedCounters *rc) {
    if (threadIdx.x == 0) {
        rc->nconf = 0;
        rc->nfall = 0;
        rc->nmark = 0;
        rc->ntiles = 0;
        rc->tile_next = 0;
        rc->bad = 0;
        rc->probed_cells = 0ull;
        rc->screened_cells = 0ull;
    }
}

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *__restrict__ p, int64_t n, int32_t v) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) p[e] = v;
}

// Exclusive scans (one block of 1024) of a per-partition quantity:
//   mode 0: ceil((offsets[p+1] - offsets[p]) / 32) -> out0 (packed blocks);
//   mode 1: cnt[p] -> out0 and ceil(cnt[p] / 32) -> out1 (queries, tiles);
// with out0[P] / out1[P] the totals (tiles total also into *total1).
__global__ __launch_bounds__(1024) void k_scan_parts(int mode, const int64_t *__restrict__ offsets,
                                                     const int32_t *__restrict__ cnt, int P,
                                                     int64_t *__restrict__ out0, int64_t *__restrict__ out1,
                                                     int32_t *__restrict__ total1, int32_t *__restrict__ bad) {
    __shared__ int64_t s0[1024], s1[1024];
    const int per = (P + 1023) / 1024;
    const int lo = threadIdx.x * per, hi = min(P, lo + per);
    auto val0 = [&](int p) -> int64_t {
        if (mode == 0) {
            const int64_t sz = offsets[p + 1] - offsets[p];
            if (sz < 0) atomicOr(bad, 1);
            return sz > 0 ? (sz + 31) / 32 : 0;
        }
        return cnt[p];
    };
    auto val1 = [&](int p) -> int64_t { return mode == 1 ? ((int64_t)cnt[p] + kTileQ - 1) / kTileQ : 0; };
    int64_t a = 0, c = 0;
    for (int p = lo; p < hi; ++p) {
        a += val0(p);
        c += val1(p);
    }
    s0[threadIdx.x] = a;
    s1[threadIdx.x] = c;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int64_t va = (int)threadIdx.x >= o ? s0[threadIdx.x - o] : 0;
        const int64_t vc = (int)threadIdx.x >= o ? s1[threadIdx.x - o] : 0;
        __syncthreads();
        s0[threadIdx.x] += va;
        s1[threadIdx.x] += vc;
        __syncthreads();
    }
    int64_t ra = s0[threadIdx.x] - a, rc = s1[threadIdx.x] - c;
    for (int p = lo; p < hi; ++p) {
        out0[p] = ra;
        ra += val0(p);
        if (mode == 1) {
            out1[p] = rc;
            rc += val1(p);
        }
    }
    if (threadIdx.x == 1023) {
        out0[P] = s0[1023];
        if (mode == 1) {
            out1[P] = s1[1023];
            *total1 = (int32_t)s1[1023];
        }
    }
}

// Packed slots of every cell and each cell's own partition.
// (Runs before the host has checked the layout: every write is bounds-checked.)
__global__ __launch_bounds__(256) void k_scatter_map(const int64_t *__restrict__ offsets,
                                                     const int32_t *__restrict__ perm, int64_t n, int P,
                                                     const int64_t *__restrict__ pblk, int64_t map_cap,
                                                     int32_t *__restrict__ map, int32_t *__restrict__ own,
                                                     int32_t *__restrict__ bad) {
    for (int64_t pos = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; pos < n;
         pos += (int64_t)gridDim.x * blockDim.x) {
        int lo = 0, hi = P - 1;  // partition p with offsets[p] <= pos < offsets[p+1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) / 2;
            if (offsets[mid] <= pos) lo = mid; else hi = mid - 1;
        }
        const int32_t row = perm[pos];
        if (row < 0 || row >= n || pos < offsets[lo] || pos >= offsets[lo + 1]) {
            atomicOr(bad, 2);
            continue;
        }
        const int64_t slot = pblk[lo] * 32 + (pos - offsets[lo]);
        if (slot < 0 || slot >= map_cap) {
            atomicOr(bad, 2);
            continue;
        }
        map[slot] = row;
        own[row] = lo;
    }
}

// Lexicographic sort of one int per lane across the wave (ascending).
__device__ __forceinline__ int wave_sort_int(int v, int lane) {
#pragma unroll
    for (int size = 2; size <= kWave; size <<= 1) {
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            const int o = __shfl_xor(v, stride, kWave);
            const bool want_min = ((lane & stride) == 0) == ((lane & size) == 0);
            v = want_min ? min(v, o) : max(v, o);
        }
    }
    return v;
}

// Probe lists sorted ascending without repeats, padded with INT_MAX (-1
// entries dropped; entries outside [-1, P) flagged and dropped).  One wave
// per row.
__global__ __launch_bounds__(256) void k_sort_probes(const int32_t *__restrict__ in, int64_t n, int np, int P,
                                                     int32_t *__restrict__ out, int32_t *__restrict__ bad) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (r >= n) return;
    int v = INT_MAX;
    if (lane < np) {
        v = in[r * np + lane];
        if (v < -1 || v >= P) {
            atomicOr(bad, 4);
            v = INT_MAX;
        } else if (v == -1) {
            v = INT_MAX;
        }
    }
    v = wave_sort_int(v, lane);
    const int left = __shfl_up(v, 1, kWave);
    if (lane > 0 && left == v) v = INT_MAX;
    v = wave_sort_int(v, lane);
    if (lane < np) out[r * np + lane] = v;
}

// Marked rows (exact_rows, or mass below the threshold, or a row without a
// partition) go to the exact list; the others are counted per own partition.
__global__ __launch_bounds__(256) void k_classify(int64_t n, const uint8_t *__restrict__ exact_rows,
                                                  const float *__restrict__ mass, float threshold,
                                                  const int32_t *__restrict__ own,
                                                  const int32_t *__restrict__ probes, int np,
                                                  const int64_t *__restrict__ offsets, RoutedCounters *rc,
                                                  int32_t *__restrict__ ccount, int32_t *__restrict__ fall,
                                                  uint8_t *__restrict__ route) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const int p = own[i];
        bool exact = (exact_rows && exact_rows[i] != 0) || (mass && !(mass[i] >= threshold));
        if (p < 0) {
            atomicOr(&rc->bad, 2);
            exact = true;
        }
        if (exact) {
            fall[atomicAdd(&rc->nfall, 1)] = (int32_t)i;
            atomicAdd(&rc->nmark, 1);
            route[i] = 1;
        } else {
            atomicAdd(&ccount[p], 1);
            atomicAdd(&rc->nconf, 1);
            route[i] = 0;
            unsigned long long c = 0;
            for (int j = 0; j < np; ++j) {
                const int q = probes[i * np + j];
                if (q == INT_MAX) break;
                c += (unsigned long long)(offsets[q + 1] - offsets[q]);
            }
            atomicAdd(&rc->probed_cells, c);
        }
    }
}

__global__ __launch_bounds__(256) void k_fill_conf(int64_t n, const uint8_t *__restrict__ route,
                                                   const int32_t *__restrict__ own,
                                                   const int64_t *__restrict__ coff, int32_t *__restrict__ cursor,
                                                   int32_t *__restrict__ qperm) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        if (route[i] != 0) continue;
        const int p = own[i];
        qperm[coff[p] + atomicAdd(&cursor[p], 1)] = (int32_t)i;
    }
}

// Order the probed queries of each partition along a Morton (Z-order)
// curve of their first three coordinates, each quantised to 10 bits over the
// bounding box of the partition's probed queries (then by row): the 32
// queries of a tile then lie close together, probe nearly the same
// partitions, and their union stays small.  One workgroup per partition,
// bitonic sort in LDS; a partition with more than kSegSort probed queries
// keeps its fill order.
constexpr int kSegSort = 4096;

__global__ __launch_bounds__(1024) void k_order_tiles(const float *__restrict__ X, int d,
                                                      const int64_t *__restrict__ coff,
                                                      const int32_t *__restrict__ ccount,
                                                      int32_t *__restrict__ qperm) {
    __shared__ int2 e[kSegSort];  // (key, row)
    __shared__ uint32_t lo[3], hi[3];  // the box, as ordered bits
    const int p = blockIdx.x;
    const int c = ccount[p];
    if (c <= kTileQ || c > kSegSort) return;
    const int64_t base = coff[p];
    int n2 = kTileQ;
    while (n2 < c) n2 <<= 1;
    const int D = d < 3 ? d : 3;
    if (threadIdx.x < 3) {
        lo[threadIdx.x] = 0xffffffffu;
        hi[threadIdx.x] = 0u;
    }
    __syncthreads();
    for (int i = threadIdx.x; i < c; i += blockDim.x) {
        const int64_t row = qperm[base + i];
        for (int t = 0; t < D; ++t) {
            const uint32_t u = ordered_bits(X[row * d + t]);
            atomicMin(&lo[t], u);
            atomicMax(&hi[t], u);
        }
    }
    __syncthreads();
    float x0[3], sc[3];
    for (int t = 0; t < 3; ++t) {
        x0[t] = t < D ? from_ordered(lo[t]) : 0.f;
        sc[t] = t < D ? scale10(x0[t], from_ordered(hi[t])) : 0.f;
    }
    for (int i = threadIdx.x; i < n2; i += blockDim.x) {
        if (i < c) {
            const int32_t row = qperm[base + i];
            uint32_t key = 0;
            for (int t = 0; t < D; ++t) key |= spread3(quantise10(X[(int64_t)row * d + t], x0[t], sc[t])) << (2 - t);
            e[i] = make_int2((int)key, row);
        } else {
            e[i] = make_int2(INT_MAX, INT_MAX);
        }
    }
    __syncthreads();
    for (int size = 2; size <= n2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int i = threadIdx.x; i < n2 / 2; i += blockDim.x) {
                const int lo = 2 * stride * (i / stride) + (i % stride), hi = lo + stride;
                const bool up = (lo & size) == 0;
                const int2 a = e[lo], b = e[hi];
                const bool gt = a.x > b.x || (a.x == b.x && a.y > b.y);
                if (gt == up) {
                    e[lo] = b;
                    e[hi] = a;
                }
            }
            __syncthreads();
        }
    }
    for (int i = threadIdx.x; i < c; i += blockDim.x) qperm[base + i] = e[i].y;
}

__global__ __launch_bounds__(256) void k_fill_tiles(int P, const int32_t *__restrict__ ccount,
                                                    const int64_t *__restrict__ coff,
                                                    const int64_t *__restrict__ toff, int2 *__restrict__ tiles) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const int c = ccount[p];
        for (int t = 0; t * kTileQ < c; ++t)
            tiles[toff[p] + t] = make_int2((int)(coff[p] + (int64_t)t * kTileQ), min(kTileQ, c - t * kTileQ));
    }
}

// Exact-list entries after the marked ones came from the certificate.
__global__ __launch_bounds__(256) void k_route_uncertified(const RoutedCounters *__restrict__ rc,
                                                           const int32_t *__restrict__ fall,
                                                           uint8_t *__restrict__ route) {
    const int nf = rc->nfall, nm = rc->nmark;
    for (int f = nm + blockIdx.x * blockDim.x + threadIdx.x; f < nf; f += gridDim.x * blockDim.x) route[fall[f]] = 2;
}

struct RoutedScreenArgs {
    ScreenArgs s;                // Q = X, Ap/Np = partition-ordered packing, P = 1 range
    const int64_t *pblk;         // first packed block of each partition (P + 1)
    const int32_t *probes;       // sorted probe lists, n x np
    int np;
    int nparts;
    const int32_t *qperm;        // probed rows grouped by own partition
    const int2 *tiles;           // (first slot, queries)
    const int32_t *ntiles;
    int32_t *tile_next;
    const int32_t *map;          // packed row -> cell
    unsigned long long *screened;  // statistics: union rows x tile queries
};

template <int DH, int L>
__global__ __launch_bounds__(256, screen_min_waves(DH, L)) void k_screen_routed(RoutedScreenArgs ra) {
    __shared__ float2 qbuf[kQueueCap * 256];
    __shared__ uint32_t bitmap[kScreenWaves][kBitmapWords];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1), wave = tid >> 6;
    const int c = lane & 31, h = lane >> 5;
    uint32_t *bm = bitmap[wave];
    float2 *q = qbuf + tid;
    const int nwords = (ra.nparts + 31) / 32;
    const int ntiles = *ra.ntiles;
    const ScreenArgs &a = ra.s;
    while (true) {
        int t = 0;
        if (lane == 0) t = atomicAdd(ra.tile_next, 1);
        t = __shfl(t, 0, kWave);
        if (t >= ntiles) break;
        const int2 tile = ra.tiles[t];
        const int64_t slot = c < tile.y ? (int64_t)tile.x + c : -1;
        const int64_t row = slot >= 0 ? (int64_t)ra.qperm[slot] : -1;
        const int32_t *pr = ra.probes + (row >= 0 ? row : 0) * ra.np;

        // union of the tile's probe lists (this wave's bitmap only)
        for (int w = lane; w < nwords; w += kWave) bm[w] = 0u;
        __builtin_amdgcn_wave_barrier();
        if (row >= 0) {
            for (int j = h; j < ra.np; j += 2) {
                const int p = pr[j];
                if (p != INT_MAX) atomicOr(&bm[p >> 5], 1u << (p & 31));
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");  // the ORs land before the bitmap is read
        __builtin_amdgcn_wave_barrier();

        Fp32Query<DH> qop;
        qop.load(a, row, h);
        LaneTopK<L> top;
        top.init();
        int ptr = 0;
        int nextp = row >= 0 ? pr[0] : INT_MAX;
        int64_t union_blocks = 0;
        // One continuous stream over the blocks of the union's partitions in
        // ascending order: the next block (possibly the first of the next
        // partition) is always in flight while the current one is screened.
        int w = 0;
        uint32_t bits = nwords > 0 ? __builtin_amdgcn_readfirstlane(bm[0]) : 0u;
        auto next_part = [&]() -> int {  // next union partition, or -1
            while (bits == 0u) {
                if (++w >= nwords) return -1;
                bits = __builtin_amdgcn_readfirstlane(bm[w]);
            }
            const int p = w * 32 + __builtin_ctz(bits);
            bits &= bits - 1;
            return p;
        };
        int p = next_part();
        int64_t b0 = 0, b1 = 0;
        while (p >= 0) {  // skip empty partitions
            b0 = ra.pblk[p];
            b1 = ra.pblk[p + 1];
            if (b0 < b1) break;
            if (nextp == p) {
                ++ptr;
                nextp = ptr < ra.np ? pr[ptr] : INT_MAX;
            }
            p = next_part();
        }
        f32x4 A[packed_s4(DH)] = {};
        if (p >= 0) load_block<DH>(a, A, b0);
        while (p >= 0) {
            // every probe of this query below p has been consumed, so the
            // query probed p exactly when its next probe is p
            const bool active = nextp == p;
            if (active) {
                ++ptr;
                nextp = ptr < ra.np ? pr[ptr] : INT_MAX;
            }
            union_blocks += b1 - b0;
            // the following non-empty partition and its first block
            int pn = next_part();
            int64_t c0 = 0, c1 = 0;
            while (pn >= 0) {
                c0 = ra.pblk[pn];
                c1 = ra.pblk[pn + 1];
                if (c0 < c1) break;
                if (nextp == pn) {
                    ++ptr;
                    nextp = ptr < ra.np ? pr[ptr] : INT_MAX;
                }
                pn = next_part();
            }
            for (int64_t blk = b0; blk < b1; ++blk) {
                const int64_t nxt = blk + 1 < b1 ? blk + 1 : (pn >= 0 ? c0 : blk);
                screen_block<DH, L, true>(a, qop, top, A, blk, nxt, 0, q, active);
            }
            p = pn;
            b0 = c0;
            b1 = c1;
        }
        top.flush(q, 256);
        if (lane == 0) atomicAdd(ra.screened, (unsigned long long)(union_blocks * 32 * tile.y));
        if (slot >= 0) {
            const int64_t base = (slot * 2 + h) * L;
#pragma unroll
            for (int i = 0; i < L; ++i) {
                const int id = top.li[i];
                a.cand_key[base + i] = top.lk[i];
                a.cand_idx[base + i] = id >= 0 ? ra.map[id] : -1;
            }
        }
    }
}

int device_slots(int dh) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus * screen_min_waves(dh, 16);
}

template <int DH>
int launch_routed_dh(const RoutedScreenArgs &ra, unsigned grid, int half, hipStream_t s) {
    if (half == 16)
        hipLaunchKernelGGL((k_screen_routed<DH, 16>), dim3(grid), dim3(256), 0, s, ra);
    else
        hipLaunchKernelGGL((k_screen_routed<DH, 32>), dim3(grid), dim3(256), 0, s, ra);
    return launch_status("screen_routed");
}

int launch_routed(int dh, const RoutedScreenArgs &ra, int half, int64_t max_tiles, hipStream_t s) {
    ScopedTimer timer("screen_routed", s);
    const unsigned grid =
        (unsigned)std::max<int64_t>(1, std::min<int64_t>(device_slots(dh), (max_tiles + kScreenWaves - 1) / kScreenWaves));
    switch (dh) {
        case 4: return launch_routed_dh<4>(ra, grid, half, s);
        case 8: return launch_routed_dh<8>(ra, grid, half, s);
        case 16: return launch_routed_dh<16>(ra, grid, half, s);
        case 25: return launch_routed_dh<25>(ra, grid, half, s);
        case 32: return launch_routed_dh<32>(ra, grid, half, s);
        case 48: return launch_routed_dh<48>(ra, grid, half, s);
        case 64: return launch_routed_dh<64>(ra, grid, half, s);
        default: set_error("internal: no screen kernel for this dimension"); return RSC_ERR_UNSUPPORTED;
    }
}

}  // namespace

size_t probed_workspace_bytes(int64_t n, int d, int k, int P, int probes) {
    if (n < 1 || d < 1 || d > 128 || k < 1 || k > 63 || k > n || P < 1 || P > kMaxParts || probes < 1 ||
        probes > kMaxProbes)
        return 0;
    return carve_probed(n, d, k, P, probes, nullptr, nullptr);
}

int probed_run(const float *X, int64_t n, int d, int k, const int64_t *offsets, const int32_t *perm, int P,
               const int32_t *probe_parts, int probes, const uint8_t *exact_rows, const float *mass,
               float threshold, int32_t *out_idx, float *out_dist, uint8_t *out_route, rsc_routed_stats *stats,
               void *ws, size_t ws_bytes, hipStream_t s) {
    if (!X || !offsets || !perm || !probe_parts || !out_idx || !out_dist) {
        set_error("probed kNN: null argument");
        return RSC_ERR_INVALID_ARG;
    }
    if (n > INT32_MAX - 1) {
        set_error("probed kNN: more rows than int32 can index");
        return RSC_ERR_OVERFLOW;
    }
    if (n < 1 || d < 1 || k < 1 || k > n || P < 1 || probes < 1) {
        set_error("probed kNN: need n >= 1, d >= 1, 1 <= k <= n, parts >= 1, probes >= 1");
        return RSC_ERR_INVALID_ARG;
    }
    if (d > 128 || k > 63 || P > kMaxParts || probes > kMaxProbes) {
        set_error("probed kNN: this build supports d <= 128, k <= 63, parts <= 8192, probes <= 64");
        return RSC_ERR_UNSUPPORTED;
    }
    if ((reinterpret_cast<uintptr_t>(X) & 3u) || (reinterpret_cast<uintptr_t>(out_dist) & 3u)) {
        set_error("probed kNN: float arrays must be 4-byte aligned");
        return RSC_ERR_INVALID_ARG;
    }
    RoutedBuffers b;
    const size_t need = carve_probed(n, d, k, P, probes, ws, &b);
    if (!ws || need == 0 || need > ws_bytes || (reinterpret_cast<uintptr_t>(ws) & (kAlign - 1))) {
        set_error("probed kNN: workspace too small or misaligned: need " + std::to_string(need) + " bytes");
        return RSC_ERR_WORKSPACE;
    }
    const int dh = pick_dh_local(d);
    const int half = k <= 16 ? 16 : 32;
    const int64_t nblk_cap = n / 32 + P;
    int st;
    {
        ScopedTimer timer("probed_prep", s);
        hipLaunchKernelGGL(k_routed_init, dim3(1), dim3(64), 0, s, b.rc);
        if ((st = knn_norms(X, n, d, b.nrow, b.kc, s)) != RSC_OK) return st;
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, s, 0, offsets, nullptr, P, b.pblk, nullptr, nullptr,
                           &b.rc->bad);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(nblk_cap * 32)), dim3(256), 0, s, b.map, nblk_cap * 32, -1);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(256), 0, s, b.own, n, -1);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(P)), dim3(256), 0, s, b.ccount, (int64_t)P, 0);
        hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(P)), dim3(256), 0, s, b.cursor, (int64_t)P, 0);
        hipLaunchKernelGGL(k_scatter_map, dim3(grid_for(n)), dim3(256), 0, s, offsets, perm, n, P, b.pblk,
                           nblk_cap * 32, b.map, b.own, &b.rc->bad);
        if ((st = launch_status("probed layout")) != RSC_OK) return st;
        // a partition layout inconsistent with n could overrun the packed
        // array: the pack covers the capacity, which every valid layout fits
        if ((st = knn_pack_mapped(dh, X, b.nrow, n, d, nblk_cap, b.packed, b.norms, b.map, s)) != RSC_OK) return st;
        hipLaunchKernelGGL(k_sort_probes, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, probe_parts, n, probes, P,
                           b.probes, &b.rc->bad);
        hipLaunchKernelGGL(k_classify, dim3(grid_for(n)), dim3(256), 0, s, n, exact_rows, mass, threshold, b.own,
                           b.probes, probes, offsets, b.rc, b.ccount, b.fall, b.route);
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(1024), 0, s, 1, nullptr, b.ccount, P, b.coff, b.toff,
                           &b.rc->ntiles, &b.rc->bad);
        hipLaunchKernelGGL(k_fill_conf, dim3(grid_for(n)), dim3(256), 0, s, n, b.route, b.own, b.coff, b.cursor,
                           b.qperm);
        hipLaunchKernelGGL(k_order_tiles, dim3(P), dim3(1024), 0, s, X, d, b.coff, b.ccount, b.qperm);
        hipLaunchKernelGGL(k_fill_tiles, dim3(grid_for(P)), dim3(256), 0, s, P, b.ccount, b.coff, b.toff, b.tiles);
        if ((st = launch_status("probed lists")) != RSC_OK) return st;
    }
    // The partition sizes must add up to n before anything indexes with them.
    int64_t total = -1;
    RoutedCounters hc{};
    if ((st = hip_status(hipMemcpyAsync(&total, offsets + P, 8, hipMemcpyDeviceToHost, s), "read offsets")) !=
            RSC_OK ||
        (st = hip_status(hipMemcpyAsync(&hc, b.rc, sizeof(hc), hipMemcpyDeviceToHost, s), "read counters")) !=
            RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (total != n || hc.bad) {
        set_error(hc.bad & 4 ? "probed kNN: a probe outside [-1, parts)"
                             : "probed kNN: offsets/perm are not a partition of the n rows");
        return RSC_ERR_INVALID_ARG;
    }

    ScreenArgs sa{};
    sa.Q = X;
    sa.nq = n;
    sa.Ap = b.packed;
    sa.Np = b.norms;
    sa.nblk = nblk_cap;
    sa.d = d;
    sa.P = 1;
    sa.cand_idx = b.cand_idx;
    sa.cand_key = b.cand_key;
    RoutedScreenArgs ra{};
    ra.s = sa;
    ra.pblk = b.pblk;
    ra.probes = b.probes;
    ra.np = probes;
    ra.nparts = P;
    ra.qperm = b.qperm;
    ra.tiles = b.tiles;
    ra.ntiles = &b.rc->ntiles;
    ra.tile_next = &b.rc->tile_next;
    ra.map = b.map;
    ra.screened = &b.rc->screened_cells;
    if (hc.ntiles > 0 && (st = launch_routed(dh, ra, half, hc.ntiles, s)) != RSC_OK) return st;

    RerankArgs rr{};
    rr.Q = X;
    rr.nq = n;
    rr.qlist = b.qperm;
    rr.qcount = &b.rc->nconf;
    rr.qcap = (int)n;
    rr.R = X;
    rr.d = d;
    rr.k = k;
    rr.S = half;
    rr.KP = half;
    rr.P = 2;
    rr.self_mode = 1;
    rr.certify = 1;
    rr.cand_idx = b.cand_idx;
    rr.cand_key = b.cand_key;
    rr.eps_coef = knn_eps_coefficient(d);
    rr.counters = b.kc;
    rr.flag_out = b.fall;  // uncertified rows join the exact list
    rr.flag_count = &b.rc->nfall;
    rr.out_idx = out_idx;
    rr.out_dist = out_dist;
    if (hc.nconf > 0 && (st = knn_launch_rerank(rr, hc.nconf, "rerank_probed", s)) != RSC_OK) return st;
    hipLaunchKernelGGL(k_route_uncertified, dim3(64), dim3(256), 0, s, b.rc, b.fall, b.route);
    if ((st = launch_status("probed routes")) != RSC_OK) return st;
    if ((st = hip_status(hipMemcpyAsync(&hc, b.rc, sizeof(hc), hipMemcpyDeviceToHost, s), "read counters")) !=
            RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;

    rsc_knn_stats es{};
    if (hc.nfall > 0) {
        KnnPlan ep;
        if ((st = exact_plan(hc.nfall, n, d, k, &ep)) != RSC_OK) return st;
        if (knn_workspace(ep, nullptr, nullptr) > b.exact_bytes) ep.splits = 1;
        if (knn_workspace(ep, nullptr, nullptr) > b.exact_bytes) {
            set_error("internal: exact-search workspace bound violated");
            return RSC_ERR_WORKSPACE;
        }
        if ((st = knn_run(ep, X, X, out_idx, out_dist, b.exact_ws, s, b.fall, &b.rc->nfall)) != RSC_OK) return st;
        if (stats) {
            KnnCounters kc{};
            if ((st = hip_status(hipMemcpyAsync(&kc, b.exact_ws, sizeof(kc), hipMemcpyDeviceToHost, s),
                                 "read exact counters")) != RSC_OK ||
                (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
                return st;
            es.escalated_rows = kc.flagged;
            es.rescanned_rows = kc.rescanned;
        }
    }
    if (out_route &&
        (st = hip_status(hipMemcpyAsync(out_route, b.route, (size_t)n, hipMemcpyDeviceToDevice, s), "copy routes")) !=
            RSC_OK)
        return st;
    if (stats) {
        stats->routed_rows = hc.nconf - (hc.nfall - hc.nmark);
        stats->low_mass_rows = hc.nmark;
        stats->uncertified_rows = hc.nfall - hc.nmark;
        stats->escalated_rows = es.escalated_rows;
        stats->rescanned_rows = es.rescanned_rows;
        stats->mean_probed_rows = hc.nconf > 0 ? (double)hc.probed_cells / (double)hc.nconf : 0.0;
        stats->mean_screened_rows = hc.nconf > 0 ? (double)hc.screened_cells / (double)hc.nconf : 0.0;
    }
    return RSC_OK;
}

}  // namespace rsc
