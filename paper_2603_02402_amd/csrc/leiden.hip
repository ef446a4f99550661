// Leiden communities of the connectivities graph.
//
// The paper clusters cells by Leiden on the neighbourhood graph (Technical
// architecture; Methods, "Dimensionality reduction and graph analysis") and
// validates the clustering by the agreement of partitions (Methods,
// "Numerical validation"), because the published algorithm visits vertices
// in random order.  This library computes one deterministic reading of the
// algorithm of Traag, Waltman and van Eck, so that its labels are a function
// of the graph alone:
//
//   quality   modularity with resolution gamma; a vertex v's gain for a
//             community c is h(v, c) = K(v, c) - ((gamma k_v) T(c)) / 2m in
//             float64, each operation rounded as written, with K(v, c) the
//             weight from v to c's other vertices and T(c) the total degree
//             of c without v;
//   weights   fixed point: W = rint(w 2^S), S = 62 - ceil(log2 nnz) -
//             e(w_max) (w_max <= 2^e), so that degrees, community totals and
//             aggregated weights are exact int64 sums whatever the order of
//             the atomics that form them;
//   moving    synchronous sweeps: every vertex reads the labels as they stood
//             at the start of the sweep and takes the neighbouring community
//             of largest gain if it beats staying (ties: the lowest label);
//             odd sweeps move only to higher labels, even sweeps only to
//             lower ones; two quiet sweeps in a row (or 64 sweeps) end it;
//   refining  rounds inside each community C: a singleton vertex that is
//             well connected to C may join the refined community R of a
//             neighbour in C with a smaller label when R is well connected to
//             C and the gain is >= 0 (largest gain, ties: the lowest label);
//             a join into a singleton that itself moves in the same round is
//             cancelled; a round without joins (or 64 rounds) ends it;
//   aggregating  the refined communities become the next level's vertices
//             (numbered by their smallest vertex), the weights between them
//             the sums of the weights between their members (own weight on
//             the diagonal), each starting in the community that holds it,
//             labelled by its smallest new vertex id.
// Levels end when moving moves nothing (or after 32 levels); the last labels
// are carried down and numbered by first appearance.
//
// Layout: one wave per vertex.  A row of up to 64 entries sits one entry per
// lane and each lane sums the weights of the lanes that share its community
// (lane broadcasts); a longer row is summed in an open-addressing table of
// twice its length in global memory (integer atomics, so the sums are exact).
// Aggregation sorts (new row, new column) keys with a radix sort and adds
// equal keys with a reduce-by-key.

#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_reduce_by_key.hpp>
#include <rocprim/device/device_scan.hpp>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <string>
#include <utility>

#include "rsc_internal.hpp"

namespace rsc {
namespace {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kMaxSweeps = 64;
constexpr int kMaxRounds = 64;
constexpr int kMaxLevels = 32;

struct LeidenState {
    int32_t error;       // bit 0: column out of range; bit 1: weight negative or not finite; bit 2: bad row pointers
    uint32_t wmax_bits;  // float bits of the largest weight (weights >= 0, so bits order like values)
    unsigned long long two_m;
    int32_t moved;
    int32_t joins;
    int32_t pad[2];
};

__device__ __forceinline__ double gain(int64_t K, double gamma, int64_t k, int64_t T, double two_m) {
    const double t = __dmul_rn(gamma, (double)k);
    const double u = __dmul_rn(t, (double)T);
    const double q = __ddiv_rn(u, two_m);
    return __dsub_rn((double)K, q);
}

// ((gamma a) b) / 2m, the well-connectedness threshold
__device__ __forceinline__ double need(double gamma, int64_t a, int64_t b, double two_m) {
    return __ddiv_rn(__dmul_rn(__dmul_rn(gamma, (double)a), (double)b), two_m);
}

__device__ __forceinline__ bool better(double h1, int32_t c1, double h2, int32_t c2) {
    return h1 > h2 || (h1 == h2 && c1 < c2);
}

__device__ __forceinline__ int64_t readlane64(int64_t x, int t) {
    const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)x, t);
    const int hi = __builtin_amdgcn_readlane((int)((uint64_t)x >> 32), t);
    return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// Wave-wide best (largest h, then smallest c); c < 0 marks no candidate.
__device__ __forceinline__ void wave_best(double &h, int32_t &c) {
    for (int o = 32; o > 0; o >>= 1) {
        const double h2 = __shfl_xor(h, o, kWave);
        const int32_t c2 = __shfl_xor(c, o, kWave);
        if (c2 >= 0 && (c < 0 || better(h2, c2, h, c))) {
            h = h2;
            c = c2;
        }
    }
}

__device__ __forceinline__ int32_t atomic_load_i32(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int64_t atomic_load_i64(const int64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Adds w under key c in the table [0, cap) (cap > number of distinct keys).
__device__ __forceinline__ void table_add(int32_t *hk, int64_t *hv, int64_t cap, int32_t c, int64_t w) {
    int64_t s = (int64_t)(((uint64_t)(uint32_t)c * 0x9E3779B97F4A7C15ull) >> 11) % cap;
    for (;;) {
        const int32_t prev = atomicCAS(&hk[s], -1, c);
        if (prev == -1 || prev == c) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&hv[s]), (unsigned long long)w);
            return;
        }
        s = s + 1 == cap ? 0 : s + 1;
    }
}

// A wave's table of distinct keys in LDS (open addressing, kLdsSlots slots).
// A row with more distinct keys than it can place within kLdsProbes probes
// falls back to the global table.
constexpr int kLdsSlots = 256;
constexpr int kLdsProbes = 32;
struct WaveTable {
    int32_t key[kLdsSlots];
    unsigned long long val[kLdsSlots];
};

// LDS writes of this wave are complete and visible to all of its lanes.
__device__ __forceinline__ void lds_wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// Adds w under key c; false when no free slot was found within kLdsProbes.
__device__ __forceinline__ bool lds_add(WaveTable *t, int32_t c, int64_t w) {
    uint32_t s = ((uint32_t)c * 0x9E3779B1u) >> 24;  // top 8 bits: kLdsSlots = 256
    for (int p = 0; p < kLdsProbes; ++p) {
        const int32_t prev = atomicCAS(&t->key[s], -1, c);
        if (prev == -1 || prev == c) {
            atomicAdd(&t->val[s], (unsigned long long)w);
            return true;
        }
        s = (s + 1) & (kLdsSlots - 1);
    }
    return false;
}

// The distinct keys of one wave's row and the summed weight of each.
// key_of(e, &key, &w) gives an entry's key (< 0: skip the entry) and weight.
// visit(valid, key, K) is called once per lane and chunk with the lane's
// (key, K) pair; a key can reach several lanes (with the same K) but every
// distinct key of the row reaches at least one.  b, e: the row's entry
// range; lt: the wave's LDS table (or null), used for rows of more than 32
// entries; hk, hv: the row's global table of 2 (e - b) slots, used for rows
// longer than a wave when the LDS table is absent or too small.
template <class KeyOf, class Visit>
__device__ __forceinline__ void row_groups(int64_t b, int64_t e, WaveTable *lt, int32_t *hk, int64_t *hv,
                                           KeyOf key_of, Visit visit) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t len = e - b;
    if (lt && len > 32) {
        for (int j = lane; j < kLdsSlots; j += kWave) {
            lt->key[j] = -1;
            lt->val[j] = 0ull;
        }
        lds_wave_sync();
        bool full = false;
        for (int64_t j = b + lane; j < e; j += kWave) {
            int32_t c;
            int64_t w;
            key_of(j, &c, &w);
            if (c >= 0 && !lds_add(lt, c, w)) full = true;
        }
        lds_wave_sync();
        const bool fits = __ballot(full) == 0ull;
        if (fits) {
            for (int s0 = 0; s0 < kLdsSlots; s0 += kWave) {
                const int32_t c = lt->key[s0 + lane];
                const int64_t K = c >= 0 ? (int64_t)lt->val[s0 + lane] : 0;
                visit(c >= 0, c, K);
            }
        }
        lds_wave_sync();  // read out before the wave's next row clears it
        if (fits) return;
    }
    if (len <= kWave) {
        int32_t c = -1;
        int64_t w = 0;
        if (lane < len) key_of(b + lane, &c, &w);
        int64_t K = 0;
        for (int t = 0; t < (int)len; ++t) {
            const int32_t ct = __builtin_amdgcn_readlane(c, t);
            const int64_t wt = readlane64(w, t);
            if (ct == c) K += wt;
        }
        visit(c >= 0, c, K);
        return;
    }
    const int64_t cap = 2 * len;
    for (int64_t j = lane; j < cap; j += kWave) {
        hk[j] = -1;
        hv[j] = 0;
    }
    __threadfence();
    for (int64_t j = b + lane; j < e; j += kWave) {
        int32_t c;
        int64_t w;
        key_of(j, &c, &w);
        if (c >= 0) table_add(hk, hv, cap, c, w);
    }
    __threadfence();
    for (int64_t j0 = 0; j0 < cap; j0 += kWave) {
        const int64_t j = j0 + lane;
        int32_t c = -1;
        int64_t K = 0;
        if (j < cap) {
            c = atomic_load_i32(&hk[j]);
            if (c >= 0) K = atomic_load_i64(&hv[j]);
        }
        visit(c >= 0, c, K);
    }
}

// ---- input checks and fixed point ----------------------------------------

__global__ void k_lv_init(LeidenState *st) {
    if (threadIdx.x == 0) {
        st->error = 0;
        st->wmax_bits = 0;
        st->two_m = 0;
        st->moved = 0;
        st->joins = 0;
    }
}

__global__ __launch_bounds__(kBlock) void k_lv_check(const int64_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ col,
                                                     const float *__restrict__ wf, int64_t n, int64_t nnz,
                                                     LeidenState *__restrict__ st) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int err = 0;
    uint32_t wmax = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) {
        const int32_t c = col[i];
        if (c < 0 || c >= n) err |= 1;
        const float w = wf[i];
        if (!(w >= 0.f) || isinf(w)) {
            err |= 2;
        } else {
            wmax = max(wmax, __float_as_uint(w));
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (ptr[i] > ptr[i + 1]) err |= 4;
    if (blockIdx.x == 0 && threadIdx.x == 0 && (ptr[0] != 0 || ptr[n] != nnz)) err |= 4;
    if (err) atomicOr(&st->error, err);
    if (wmax) atomicMax(&st->wmax_bits, wmax);
}

// Level 0's graph: the input columns and W = rint(w 2^S) (twice: the level
// graph is overwritten by later levels, w0 is kept for the modularity).
__global__ __launch_bounds__(kBlock) void k_lv_fixed(const int32_t *__restrict__ col, const float *__restrict__ wf,
                                                     int64_t nnz, int S, int32_t *__restrict__ gcol,
                                                     int64_t *__restrict__ gw, int64_t *__restrict__ w0) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz; i += stride) {
        gcol[i] = col[i];
        const int64_t W = (int64_t)rint(ldexp((double)wf[i], S));
        gw[i] = W;
        w0[i] = W;
    }
}

__global__ __launch_bounds__(kBlock) void k_lv_copy_ptr(const int64_t *__restrict__ src, int64_t n,
                                                        int64_t *__restrict__ dst) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) dst[i] = src[i];
}

__global__ __launch_bounds__(kBlock) void k_lv_iota(int32_t *__restrict__ a, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = (int32_t)i;
}

__global__ __launch_bounds__(kBlock) void k_lv_fill64(int64_t *__restrict__ a, int64_t n, int64_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}

__global__ __launch_bounds__(kBlock) void k_lv_fill32(int32_t *__restrict__ a, int64_t n, int32_t v) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}

// ---- per level -------------------------------------------------------------

// Degrees k_v (row sums, diagonal once) and 2m.
__global__ __launch_bounds__(kBlock) void k_lv_degree(const int64_t *__restrict__ ptr,
                                                      const int64_t *__restrict__ gw, int64_t N,
                                                      int64_t *__restrict__ kdeg, LeidenState *__restrict__ st) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    int64_t acc = 0;
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < N; v += waves) {
        int64_t s = 0;
        for (int64_t e = ptr[v] + lane; e < ptr[v + 1]; e += kWave) s += gw[e];
        s = wave_sum64(s);
        if (lane == 0) kdeg[v] = s;
        acc += s;
    }
    if (lane == 0 && acc) atomicAdd(&st->two_m, (unsigned long long)acc);
}

// tot[c] += k_v over the vertices labelled c (tot cleared before).
__global__ __launch_bounds__(kBlock) void k_lv_tot(const int32_t *__restrict__ lab, const int64_t *__restrict__ kdeg,
                                                   int64_t N, int64_t *__restrict__ tot) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
        if (kdeg[v]) atomicAdd(reinterpret_cast<unsigned long long *>(&tot[lab[v]]), (unsigned long long)kdeg[v]);
}

// One sweep of local moving: Lnext[v] from the labels L at the sweep start.
// A wave takes two consecutive vertices: when both rows have at most 32
// entries, each half of the wave holds one row (its weights summed per
// community by lane broadcasts within the half); otherwise the wave takes
// the two vertices one after the other, a whole wave per row.
__device__ __forceinline__ void move_one(int64_t v, const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                         const int64_t *__restrict__ gw, const int64_t *__restrict__ kdeg,
                                         const int64_t *__restrict__ tot, const int32_t *__restrict__ L,
                                         int32_t *__restrict__ Lnext, int up, double gamma, double two_m,
                                         WaveTable *lt, int32_t *__restrict__ hk, int64_t *__restrict__ hv,
                                         int &moved) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t b = ptr[v], e = ptr[v + 1];
    const int32_t a = L[v];
    const int64_t kv = kdeg[v];
    double best_h = 0.0;
    int32_t best_c = -1;
    int64_t Ka = 0;  // K(v, a), held by the lanes whose key is a
    bool has_a = false;
    row_groups(
        b, e, lt, hk + 2 * b, hv + 2 * b,
        [&](int64_t j, int32_t *c, int64_t *w) {
            const int32_t u = col[j];
            *c = u == (int32_t)v ? -1 : L[u];
            *w = gw[j];
        },
        [&](bool valid, int32_t c, int64_t K) {
            if (!valid) return;
            if (c == a) {
                Ka = K;
                has_a = true;
                return;
            }
            if (up ? c < a : c > a) return;
            const double h = gain(K, gamma, kv, tot[c], two_m);
            if (best_c < 0 || better(h, c, best_h, best_c)) {
                best_h = h;
                best_c = c;
            }
        });
    wave_best(best_h, best_c);
    // K(v, a): every lane that saw key a holds the same sum
    const uint64_t holders = __ballot(has_a);
    if (holders)
        Ka = readlane64(Ka, __builtin_ctzll(holders));
    else
        Ka = 0;
    const double stay = gain(Ka, gamma, kv, tot[a] - kv, two_m);
    const int32_t next = (best_c >= 0 && best_h > stay) ? best_c : a;
    if (lane == 0) {
        Lnext[v] = next;
        moved += next != a;
    }
}

__global__ __launch_bounds__(kBlock) void k_lv_move(const int64_t *__restrict__ ptr, const int32_t *__restrict__ col,
                                                    const int64_t *__restrict__ gw, int64_t N,
                                                    const int64_t *__restrict__ kdeg, const int64_t *__restrict__ tot,
                                                    const int32_t *__restrict__ L, int32_t *__restrict__ Lnext,
                                                    int up, double gamma, double two_m, int32_t *__restrict__ hk,
                                                    int64_t *__restrict__ hv, LeidenState *__restrict__ st) {
    __shared__ WaveTable tabs[kBlock / kWave];
    WaveTable *lt = &tabs[threadIdx.x / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int half = lane >> 5, sub = lane & 31;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    int moved = 0;
    for (int64_t g = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; 2 * g < N; g += waves) {
        const int64_t v = 2 * g + half;
        const bool vok = v < N;
        const int64_t b = vok ? ptr[v] : 0;
        const int len = vok ? (int)(ptr[v + 1] - b) : 0;
        const int len0 = __builtin_amdgcn_readlane(len, 0), len1 = __builtin_amdgcn_readlane(len, 32);
        if (len0 > 32 || len1 > 32) {
            move_one(2 * g, ptr, col, gw, kdeg, tot, L, Lnext, up, gamma, two_m, lt, hk, hv, moved);
            if (2 * g + 1 < N)
                move_one(2 * g + 1, ptr, col, gw, kdeg, tot, L, Lnext, up, gamma, two_m, lt, hk, hv, moved);
            continue;
        }
        const int32_t a = vok ? L[v] : -1;
        const int64_t kv = vok ? kdeg[v] : 0;
        int32_t c = -1;
        int64_t w = 0;
        if (sub < len) {
            const int32_t u = col[b + sub];
            c = u == (int32_t)v ? -1 : L[u];
            w = gw[b + sub];
        }
        // K(v, c) of this lane's community within its half's row
        const int tmax = len0 > len1 ? len0 : len1;
        int64_t K = 0;
        for (int t = 0; t < tmax; ++t) {
            const int32_t c0 = __builtin_amdgcn_readlane(c, t), c1 = __builtin_amdgcn_readlane(c, 32 + t);
            const int64_t w0 = readlane64(w, t), w1 = readlane64(w, 32 + t);
            if ((half ? c1 : c0) == c) K += half ? w1 : w0;
        }
        double best_h = 0.0;
        int32_t best_c = -1;
        const bool valid = c >= 0;
        const bool is_a = valid && c == a;
        if (valid && !is_a && !(up ? c < a : c > a)) {
            best_h = gain(K, gamma, kv, tot[c], two_m);
            best_c = c;
        }
        for (int o = 16; o > 0; o >>= 1) {  // best within the half
            const double h2 = __shfl_xor(best_h, o, kWave);
            const int32_t c2 = __shfl_xor(best_c, o, kWave);
            if (c2 >= 0 && (best_c < 0 || better(h2, c2, best_h, best_c))) {
                best_h = h2;
                best_c = c2;
            }
        }
        const uint64_t holders = __ballot(is_a);
        const uint32_t hold0 = (uint32_t)holders, hold1 = (uint32_t)(holders >> 32);
        const int64_t Ka0 = hold0 ? readlane64(K, __builtin_ctz(hold0)) : 0;
        const int64_t Ka1 = hold1 ? readlane64(K, 32 + __builtin_ctz(hold1)) : 0;
        if (vok && sub == 0) {
            const double stay = gain(half ? Ka1 : Ka0, gamma, kv, tot[a] - kv, two_m);
            const int32_t next = (best_c >= 0 && best_h > stay) ? best_c : a;
            Lnext[v] = next;
            moved += next != a;
        }
    }
    if ((lane & 31) == 0 && moved) atomicAdd(&st->moved, moved);
}

// After a sweep: the community totals follow the vertices that moved (integer
// sums, so tot stays exactly the sum of k over each label).
__global__ __launch_bounds__(kBlock) void k_lv_tot_delta(const int32_t *__restrict__ L,
                                                         const int32_t *__restrict__ Lnext,
                                                         const int64_t *__restrict__ kdeg, int64_t N,
                                                         int64_t *__restrict__ tot) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
        const int32_t a = L[v], b = Lnext[v];
        const int64_t kv = kdeg[v];
        if (a != b && kv) {
            atomicAdd(reinterpret_cast<unsigned long long *>(&tot[b]), (unsigned long long)kv);
            atomicAdd(reinterpret_cast<unsigned long long *>(&tot[a]), (unsigned long long)(-kv));
        }
    }
}

// Refinement set-up: kin[v] = K(v, C - v) and totC[c] = sum of k over c.
__global__ __launch_bounds__(kBlock) void k_lv_refine_prep(const int64_t *__restrict__ ptr,
                                                           const int32_t *__restrict__ col,
                                                           const int64_t *__restrict__ gw, int64_t N,
                                                           const int64_t *__restrict__ kdeg,
                                                           const int32_t *__restrict__ L, int64_t *__restrict__ kin,
                                                           int64_t *__restrict__ totC) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < N; v += waves) {
        const int32_t c = L[v];
        int64_t s = 0;
        for (int64_t e = ptr[v] + lane; e < ptr[v + 1]; e += kWave) {
            const int32_t u = col[e];
            if (u != (int32_t)v && L[u] == c) s += gw[e];
        }
        s = wave_sum64(s);
        if (lane == 0) {
            kin[v] = s;
            if (kdeg[v]) atomicAdd(reinterpret_cast<unsigned long long *>(&totC[c]), (unsigned long long)kdeg[v]);
        }
    }
}

// Per round: totR, size and extR = E(R, C - R) by refined label (cleared before).
__global__ __launch_bounds__(kBlock) void k_lv_refine_stats(const int64_t *__restrict__ ptr,
                                                            const int32_t *__restrict__ col,
                                                            const int64_t *__restrict__ gw, int64_t N,
                                                            const int64_t *__restrict__ kdeg,
                                                            const int32_t *__restrict__ L,
                                                            const int32_t *__restrict__ R,
                                                            int64_t *__restrict__ totR, int32_t *__restrict__ size,
                                                            int64_t *__restrict__ extR) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < N; v += waves) {
        const int32_t c = L[v], r = R[v];
        int64_t s = 0;
        for (int64_t e = ptr[v] + lane; e < ptr[v + 1]; e += kWave) {
            const int32_t u = col[e];
            if (L[u] == c && R[u] != r) s += gw[e];
        }
        s = wave_sum64(s);
        if (lane == 0) {
            if (kdeg[v]) atomicAdd(reinterpret_cast<unsigned long long *>(&totR[r]), (unsigned long long)kdeg[v]);
            atomicAdd(&size[r], 1);
            if (s) atomicAdd(reinterpret_cast<unsigned long long *>(&extR[r]), (unsigned long long)s);
        }
    }
}

// Per round: the refined community each well-connected singleton proposes to join (-1: none).
__global__ __launch_bounds__(kBlock) void k_lv_refine_propose(
    const int64_t *__restrict__ ptr, const int32_t *__restrict__ col, const int64_t *__restrict__ gw, int64_t N,
    const int64_t *__restrict__ kdeg, const int32_t *__restrict__ L, const int32_t *__restrict__ R,
    const int64_t *__restrict__ kin, const int64_t *__restrict__ totC, const int64_t *__restrict__ totR,
    const int32_t *__restrict__ size, const int64_t *__restrict__ extR, double gamma, double two_m,
    int32_t *__restrict__ prop, int32_t *__restrict__ hk, int64_t *__restrict__ hv) {
    __shared__ WaveTable tabs[kBlock / kWave];
    WaveTable *lt = &tabs[threadIdx.x / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < N; v += waves) {
        const int32_t C = L[v];
        const int64_t kv = kdeg[v];
        bool cand = R[v] == (int32_t)v && size[v] == 1;
        if (cand) cand = (double)kin[v] >= need(gamma, kv, totC[C] - kv, two_m);
        if (!cand) {
            if (lane == 0) prop[v] = -1;
            continue;
        }
        const int64_t tC = totC[C];
        double best_h = 0.0;
        int32_t best_r = -1;
        const int64_t b = ptr[v], e = ptr[v + 1];
        row_groups(
            b, e, lt, hk + 2 * b, hv + 2 * b,
            [&](int64_t j, int32_t *c, int64_t *w) {
                const int32_t u = col[j];
                *c = -1;
                *w = gw[j];
                if (u == (int32_t)v || L[u] != C) return;
                const int32_t r = R[u];
                if (r < (int32_t)v) *c = r;
            },
            [&](bool valid, int32_t r, int64_t K) {
                if (!valid) return;
                const int64_t tr = totR[r];
                if (!((double)extR[r] >= need(gamma, tr, tC - tr, two_m))) return;
                const double h = gain(K, gamma, kv, tr, two_m);
                if (!(h >= 0.0)) return;
                if (best_r < 0 || better(h, r, best_h, best_r)) {
                    best_h = h;
                    best_r = r;
                }
            });
        wave_best(best_h, best_r);
        if (lane == 0) prop[v] = best_r;
    }
}

__global__ __launch_bounds__(kBlock) void k_lv_refine_apply(const int32_t *__restrict__ prop,
                                                            const int32_t *__restrict__ size, int64_t N,
                                                            int32_t *__restrict__ R, LeidenState *__restrict__ st) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int joins = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride) {
        const int32_t t = prop[v];
        if (t < 0) continue;
        if (size[t] == 1 && prop[t] >= 0) continue;  // the target singleton moves away
        R[v] = t;
        ++joins;
    }
    if (joins) atomicAdd(&st->joins, joins);
}

// head[v] = 1 where v is the smallest vertex (the label) of its refined community
__global__ __launch_bounds__(kBlock) void k_lv_heads(const int32_t *__restrict__ R, int64_t N,
                                                     int32_t *__restrict__ head) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
        head[v] = R[v] == (int32_t)v ? 1 : 0;
}

// Keys (new row << 32 | new column) and weights of every entry of the level's graph.
__global__ __launch_bounds__(kBlock) void k_lv_edge_keys(const int64_t *__restrict__ ptr,
                                                         const int32_t *__restrict__ col,
                                                         const int64_t *__restrict__ gw, int64_t N,
                                                         const int32_t *__restrict__ R,
                                                         const int32_t *__restrict__ id, uint64_t *__restrict__ key,
                                                         int64_t *__restrict__ val) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < N; v += waves) {
        const uint64_t a = (uint64_t)(uint32_t)id[R[v]] << 32;
        for (int64_t e = ptr[v] + lane; e < ptr[v + 1]; e += kWave) {
            key[e] = a | (uint32_t)id[R[col[e]]];
            val[e] = gw[e];
        }
    }
}

// The aggregated graph from the unique sorted keys: columns, weights, row pointers.
__global__ __launch_bounds__(kBlock) void k_lv_unpack(const uint64_t *__restrict__ ukey,
                                                      const int64_t *__restrict__ agg,
                                                      const unsigned long long *__restrict__ count,
                                                      int32_t *__restrict__ ncol, int64_t *__restrict__ nw) {
    const int64_t m = (int64_t)*count;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < m; j += stride) {
        ncol[j] = (int32_t)(uint32_t)(ukey[j] & 0xffffffffull);
        nw[j] = agg[j];
    }
}

__global__ __launch_bounds__(kBlock) void k_lv_rowptr(const uint64_t *__restrict__ ukey,
                                                      const unsigned long long *__restrict__ count, int64_t K2,
                                                      int64_t *__restrict__ nptr) {
    const int64_t m = (int64_t)*count;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a <= K2; a += stride) {
        // first unique entry whose row is >= a
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(ukey[mid] >> 32) < a)
                lo = mid + 1;
            else
                hi = mid;
        }
        nptr[a] = lo;
    }
}

__global__ __launch_bounds__(kBlock) void k_lv_minid(const int32_t *__restrict__ L, const int32_t *__restrict__ R,
                                                     const int32_t *__restrict__ id, int64_t N,
                                                     int32_t *__restrict__ minid) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
        atomicMin(&minid[L[v]], id[R[v]]);
}

__global__ __launch_bounds__(kBlock) void k_lv_newlabels(const int32_t *__restrict__ L,
                                                         const int32_t *__restrict__ R,
                                                         const int32_t *__restrict__ id,
                                                         const int32_t *__restrict__ minid, int64_t N,
                                                         int32_t *__restrict__ L2) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < N; v += stride)
        if (R[v] == (int32_t)v) L2[id[v]] = minid[L[v]];
}

__global__ __launch_bounds__(kBlock) void k_lv_top(const int32_t *__restrict__ R, const int32_t *__restrict__ id,
                                                   int64_t n, int32_t *__restrict__ top) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) top[i] = id[R[top[i]]];
}

// ---- final labels and modularity -----------------------------------------

__global__ __launch_bounds__(kBlock) void k_lv_first(const int32_t *__restrict__ L, const int32_t *__restrict__ top,
                                                     int64_t n, int32_t *__restrict__ first) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        atomicMin(&first[L[top[i]]], (int32_t)i);
}

__global__ __launch_bounds__(kBlock) void k_lv_mark(const int32_t *__restrict__ L, const int32_t *__restrict__ top,
                                                    const int32_t *__restrict__ first, int64_t n,
                                                    int32_t *__restrict__ mark) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        mark[i] = first[L[top[i]]] == (int32_t)i ? 1 : 0;
}

__global__ __launch_bounds__(kBlock) void k_lv_labels(const int32_t *__restrict__ L, const int32_t *__restrict__ top,
                                                      const int32_t *__restrict__ first,
                                                      const int32_t *__restrict__ num, int64_t n,
                                                      int32_t *__restrict__ labels) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        labels[i] = num[first[L[top[i]]]];
}

// in[c] and tot[c] of the final labels on the input graph (fixed-point weights).
__global__ __launch_bounds__(kBlock) void k_lv_quality_sums(const int64_t *__restrict__ ptr,
                                                            const int32_t *__restrict__ col,
                                                            const int64_t *__restrict__ gw, int64_t n,
                                                            const int32_t *__restrict__ labels,
                                                            int64_t *__restrict__ in, int64_t *__restrict__ tot) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; v < n; v += waves) {
        const int32_t c = labels[v];
        int64_t s = 0, t = 0;
        for (int64_t e = ptr[v] + lane; e < ptr[v + 1]; e += kWave) {
            t += gw[e];
            if (labels[col[e]] == c) s += gw[e];
        }
        s = wave_sum64(s);
        t = wave_sum64(t);
        if (lane == 0) {
            if (s) atomicAdd(reinterpret_cast<unsigned long long *>(&in[c]), (unsigned long long)s);
            if (t) atomicAdd(reinterpret_cast<unsigned long long *>(&tot[c]), (unsigned long long)t);
        }
    }
}

// Q = sum over communities in label order of in/2m - (gamma tot/2m) tot/2m (one thread, in order).
__global__ void k_lv_quality(const int64_t *__restrict__ in, const int64_t *__restrict__ tot, int64_t ncomm,
                             double gamma, double two_m, double *__restrict__ q) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double Q = 0.0;
    for (int64_t c = 0; c < ncomm; ++c) {
        if (!tot[c]) continue;
        const double x = __ddiv_rn((double)tot[c], two_m);
        Q = __dadd_rn(Q, __dsub_rn(__ddiv_rn((double)in[c], two_m), __dmul_rn(__dmul_rn(gamma, x), x)));
    }
    *q = Q;
}

// ---- workspace -------------------------------------------------------------

struct LevelGraph {
    int64_t *ptr;
    int32_t *col;
    int64_t *w;
};

struct LeidenWs {
    LeidenState *st;
    LevelGraph g[2];
    int64_t *w0;  // fixed-point input weights (level 0 keeps them for the modularity)
    int64_t *kdeg, *tot, *kin, *totC, *totR, *extR;
    int32_t *L, *Lnext, *R, *prop, *size, *head, *id, *minid, *top, *first, *mark, *num;
    int32_t *hk;
    int64_t *hv;
    uint64_t *key, *key2, *ukey;
    int64_t *val, *val2, *agg;
    unsigned long long *ucount;
    int64_t *qin, *qtot;
    double *q;
    char *tmp;
    size_t tmp_bytes;
};

int key_bits(int64_t K) {
    int b = 1;
    while (b < 31 && ((int64_t)1 << b) < K) ++b;
    return b;
}

size_t temp_bytes(int64_t n, int64_t nnz) {
    const size_t m = (size_t)std::max<int64_t>(nnz, 1);
    size_t a = 0, b = 0, c = 0;
    if (rocprim::radix_sort_pairs(nullptr, a, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                  (const int64_t *)nullptr, (int64_t *)nullptr, m, 0, 64, (hipStream_t)0) !=
        hipSuccess)
        return 0;
    if (rocprim::reduce_by_key(nullptr, b, (const uint64_t *)nullptr, (const int64_t *)nullptr, m,
                               (uint64_t *)nullptr, (int64_t *)nullptr, (unsigned long long *)nullptr,
                               rocprim::plus<int64_t>(), rocprim::equal_to<uint64_t>(), (hipStream_t)0) !=
        hipSuccess)
        return 0;
    if (rocprim::exclusive_scan(nullptr, c, (const int32_t *)nullptr, (int32_t *)nullptr, (int32_t)0,
                                (size_t)std::max<int64_t>(n, 1), rocprim::plus<int32_t>(), (hipStream_t)0) !=
        hipSuccess)
        return 0;
    return std::max(a, std::max(b, c));
}

size_t carve_leiden(int64_t n, int64_t nnz, void *base, LeidenWs *out) {
    Carver cv(base);
    LeidenWs w{};
    const size_t N = (size_t)std::max<int64_t>(n, 1), E = (size_t)std::max<int64_t>(nnz, 1);
    w.st = cv.take<LeidenState>(1);
    for (int i = 0; i < 2; ++i) {
        w.g[i].ptr = cv.take<int64_t>(N + 1);
        w.g[i].col = cv.take<int32_t>(E);
        w.g[i].w = cv.take<int64_t>(E);
    }
    w.w0 = cv.take<int64_t>(E);
    w.kdeg = cv.take<int64_t>(N);
    w.tot = cv.take<int64_t>(N);
    w.kin = cv.take<int64_t>(N);
    w.totC = cv.take<int64_t>(N);
    w.totR = cv.take<int64_t>(N);
    w.extR = cv.take<int64_t>(N);
    w.L = cv.take<int32_t>(N);
    w.Lnext = cv.take<int32_t>(N);
    w.R = cv.take<int32_t>(N);
    w.prop = cv.take<int32_t>(N);
    w.size = cv.take<int32_t>(N);
    w.head = cv.take<int32_t>(N);
    w.id = cv.take<int32_t>(N);
    w.minid = cv.take<int32_t>(N);
    w.top = cv.take<int32_t>(N);
    w.first = cv.take<int32_t>(N);
    w.mark = cv.take<int32_t>(N);
    w.num = cv.take<int32_t>(N);
    w.hk = cv.take<int32_t>(2 * E);
    w.hv = cv.take<int64_t>(2 * E);
    w.key = cv.take<uint64_t>(E);
    w.key2 = cv.take<uint64_t>(E);
    w.ukey = cv.take<uint64_t>(E);
    w.val = cv.take<int64_t>(E);
    w.val2 = cv.take<int64_t>(E);
    w.agg = cv.take<int64_t>(E);
    w.ucount = cv.take<unsigned long long>(1);
    w.qin = cv.take<int64_t>(N);
    w.qtot = cv.take<int64_t>(N);
    w.q = cv.take<double>(1);
    w.tmp_bytes = temp_bytes(n, nnz);
    w.tmp = cv.take<char>(w.tmp_bytes ? w.tmp_bytes : 1);
    if (out) *out = w;
    return w.tmp_bytes ? cv.used : 0;
}

unsigned grid_items(int64_t items) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((items + kBlock - 1) / kBlock, 8192));
}
unsigned grid_waves(int64_t waves) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>((waves + kBlock / kWave - 1) / (kBlock / kWave), 65536));
}

template <class T>
int read_back(T *host, const T *dev, hipStream_t s, const char *what) {
    int st = hip_status(hipMemcpyAsync(host, dev, sizeof(T), hipMemcpyDeviceToHost, s), what);
    if (st != RSC_OK) return st;
    return hip_status(hipStreamSynchronize(s), "synchronise");
}

}  // namespace

size_t leiden_workspace_bytes(int64_t n, int64_t nnz) { return carve_leiden(n, nnz, nullptr, nullptr); }

int leiden_run(const int64_t *indptr, const int32_t *indices, const float *weights, int64_t n, int64_t nnz,
               double gamma, int32_t *labels, rsc_leiden_stats *stats, void *ws, hipStream_t s) {
    LeidenWs w;
    carve_leiden(n, nnz, ws, &w);
    int st;
    hipLaunchKernelGGL(k_lv_init, dim3(1), dim3(64), 0, s, w.st);
    hipLaunchKernelGGL(k_lv_check, dim3(grid_items(std::max(n, nnz))), dim3(kBlock), 0, s, indptr, indices, weights, n,
                       nnz, w.st);
    if ((st = launch_status("leiden input check")) != RSC_OK) return st;
    LeidenState hs;
    if ((st = hip_status(hipMemcpyAsync(&hs, w.st, sizeof(hs), hipMemcpyDeviceToHost, s), "read check")) != RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    if (hs.error) {
        set_error(hs.error & 4   ? "leiden: row pointers must start at 0, not decrease and end at nnz"
                  : hs.error & 1 ? "leiden: a column index outside [0, n)"
                                 : "leiden: a weight that is negative, NaN or infinite");
        return RSC_ERR_INVALID_ARG;
    }
    float wmax;
    std::memcpy(&wmax, &hs.wmax_bits, 4);
    // S = 62 - ceil(log2 nnz) - e, with wmax = f 2^e, f in [0.5, 1)
    int c = 0, e = 0;
    while (((int64_t)1 << c) < std::max<int64_t>(nnz, 1)) ++c;
    if (wmax > 0.f) std::frexp((double)wmax, &e);
    const int S = 62 - c - e;

    ScopedTimer timer("leiden", s);
    LevelGraph G = w.g[0];
    int gi = 0;
    hipLaunchKernelGGL(k_lv_copy_ptr, dim3(grid_items(n + 1)), dim3(kBlock), 0, s, indptr, n, G.ptr);
    if (nnz > 0)
        hipLaunchKernelGGL(k_lv_fixed, dim3(grid_items(nnz)), dim3(kBlock), 0, s, indices, weights, nnz, S, G.col, G.w,
                           w.w0);
    hipLaunchKernelGGL(k_lv_iota, dim3(grid_items(n)), dim3(kBlock), 0, s, w.top, n);
    hipLaunchKernelGGL(k_lv_iota, dim3(grid_items(n)), dim3(kBlock), 0, s, w.L, n);
    if ((st = launch_status("leiden set-up")) != RSC_OK) return st;

    int64_t N = n, M = nnz;
    int lv = 0, sweeps = 0, rounds = 0;
    int64_t move_bytes = 0;
    double two_m0 = 0.0;
    for (;;) {
        hipLaunchKernelGGL(k_lv_init, dim3(1), dim3(64), 0, s, w.st);
        hipLaunchKernelGGL(k_lv_degree, dim3(grid_waves(N)), dim3(kBlock), 0, s, G.ptr, G.w, N, w.kdeg, w.st);
        if ((st = launch_status("leiden degrees")) != RSC_OK) return st;
        if ((st = read_back(&hs, w.st, s, "read 2m")) != RSC_OK) return st;
        if (lv == 0) two_m0 = (double)(int64_t)hs.two_m;
        if (hs.two_m == 0) break;
        const double two_m = (double)(int64_t)hs.two_m;
        // 1. local moving
        int64_t moves = 0;
        int quiet = 0;
        // community totals of the level's starting labels; each sweep then
        // moves them along with the vertices that change label
        hipLaunchKernelGGL(k_lv_fill64, dim3(grid_items(N)), dim3(kBlock), 0, s, w.tot, N, (int64_t)0);
        hipLaunchKernelGGL(k_lv_tot, dim3(grid_items(N)), dim3(kBlock), 0, s, w.L, w.kdeg, N, w.tot);
        for (int sweep = 1; sweep <= kMaxSweeps && quiet < 2; ++sweep) {
            {
                ScopedTimer t("leiden_move", s);
                hipLaunchKernelGGL(k_lv_init, dim3(1), dim3(64), 0, s, w.st);
                hipLaunchKernelGGL(k_lv_move, dim3(grid_waves((N + 1) / 2)), dim3(kBlock), 0, s, G.ptr, G.col, G.w, N, w.kdeg,
                                   w.tot, w.L, w.Lnext, sweep % 2, gamma, two_m, w.hk, w.hv, w.st);
                hipLaunchKernelGGL(k_lv_tot_delta, dim3(grid_items(N)), dim3(kBlock), 0, s, w.L, w.Lnext, w.kdeg, N,
                                   w.tot);
            }
            if ((st = launch_status("leiden local moving")) != RSC_OK) return st;
            ++sweeps;
            move_bytes += 16 * M + 24 * N;
            std::swap(w.L, w.Lnext);
            if ((st = read_back(&hs, w.st, s, "read moves")) != RSC_OK) return st;
            moves += hs.moved;
            quiet = hs.moved ? 0 : quiet + 1;
        }
        ++lv;
        if (moves == 0 || lv >= kMaxLevels) break;
        // 2. refinement
        {
        ScopedTimer t_refine("leiden_refine", s);
        hipLaunchKernelGGL(k_lv_fill64, dim3(grid_items(N)), dim3(kBlock), 0, s, w.totC, N, (int64_t)0);
        hipLaunchKernelGGL(k_lv_iota, dim3(grid_items(N)), dim3(kBlock), 0, s, w.R, N);
        hipLaunchKernelGGL(k_lv_refine_prep, dim3(grid_waves(N)), dim3(kBlock), 0, s, G.ptr, G.col, G.w, N, w.kdeg,
                           w.L, w.kin, w.totC);
        if ((st = launch_status("leiden refinement set-up")) != RSC_OK) return st;
        for (int round = 1; round <= kMaxRounds; ++round) {
            hipLaunchKernelGGL(k_lv_fill64, dim3(grid_items(N)), dim3(kBlock), 0, s, w.totR, N, (int64_t)0);
            hipLaunchKernelGGL(k_lv_fill64, dim3(grid_items(N)), dim3(kBlock), 0, s, w.extR, N, (int64_t)0);
            hipLaunchKernelGGL(k_lv_fill32, dim3(grid_items(N)), dim3(kBlock), 0, s, w.size, N, 0);
            hipLaunchKernelGGL(k_lv_refine_stats, dim3(grid_waves(N)), dim3(kBlock), 0, s, G.ptr, G.col, G.w, N,
                               w.kdeg, w.L, w.R, w.totR, w.size, w.extR);
            hipLaunchKernelGGL(k_lv_refine_propose, dim3(grid_waves(N)), dim3(kBlock), 0, s, G.ptr, G.col, G.w, N,
                               w.kdeg, w.L, w.R, w.kin, w.totC, w.totR, w.size, w.extR, gamma, two_m, w.prop, w.hk,
                               w.hv);
            hipLaunchKernelGGL(k_lv_init, dim3(1), dim3(64), 0, s, w.st);
            hipLaunchKernelGGL(k_lv_refine_apply, dim3(grid_items(N)), dim3(kBlock), 0, s, w.prop, w.size, N, w.R,
                               w.st);
            if ((st = launch_status("leiden refinement")) != RSC_OK) return st;
            ++rounds;
            if ((st = read_back(&hs, w.st, s, "read joins")) != RSC_OK) return st;
            if (!hs.joins) break;
        }
        }
        // 3. aggregation
        ScopedTimer t_agg("leiden_aggregate", s);
        hipLaunchKernelGGL(k_lv_heads, dim3(grid_items(N)), dim3(kBlock), 0, s, w.R, N, w.head);
        if ((st = hip_status(rocprim::exclusive_scan(w.tmp, w.tmp_bytes, (const int32_t *)w.head, w.id, (int32_t)0,
                                                     (size_t)N, rocprim::plus<int32_t>(), s),
                             "scan of the refined communities")) != RSC_OK)
            return st;
        int32_t last_id = 0, last_head = 0;
        if ((st = hip_status(hipMemcpyAsync(&last_id, w.id + (N - 1), 4, hipMemcpyDeviceToHost, s), "read ids")) !=
                RSC_OK ||
            (st = hip_status(hipMemcpyAsync(&last_head, w.head + (N - 1), 4, hipMemcpyDeviceToHost, s),
                             "read ids")) != RSC_OK ||
            (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
            return st;
        const int64_t K2 = (int64_t)last_id + last_head;
        LevelGraph H = w.g[1 - gi];
        if (M > 0) {
            hipLaunchKernelGGL(k_lv_edge_keys, dim3(grid_waves(N)), dim3(kBlock), 0, s, G.ptr, G.col, G.w, N, w.R,
                               w.id, w.key, w.val);
            if ((st = launch_status("leiden aggregation keys")) != RSC_OK) return st;
            if ((st = hip_status(rocprim::radix_sort_pairs(w.tmp, w.tmp_bytes, (const uint64_t *)w.key, w.key2,
                                                           (const int64_t *)w.val, w.val2, (size_t)M, 0,
                                                           32 + key_bits(K2), s),
                                 "sort of the aggregated entries")) != RSC_OK)
                return st;
            if ((st = hip_status(rocprim::reduce_by_key(w.tmp, w.tmp_bytes, (const uint64_t *)w.key2,
                                                        (const int64_t *)w.val2, (size_t)M, w.ukey, w.agg, w.ucount,
                                                        rocprim::plus<int64_t>(), rocprim::equal_to<uint64_t>(), s),
                                 "sum of the aggregated entries")) != RSC_OK)
                return st;
            hipLaunchKernelGGL(k_lv_unpack, dim3(grid_items(M)), dim3(kBlock), 0, s, w.ukey, w.agg, w.ucount, H.col,
                               H.w);
            hipLaunchKernelGGL(k_lv_rowptr, dim3(grid_items(K2 + 1)), dim3(kBlock), 0, s, w.ukey, w.ucount, K2, H.ptr);
            unsigned long long m2 = 0;
            if ((st = read_back(&m2, w.ucount, s, "read aggregated size")) != RSC_OK) return st;
            M = (int64_t)m2;
        } else {
            hipLaunchKernelGGL(k_lv_fill64, dim3(grid_items(K2 + 1)), dim3(kBlock), 0, s, H.ptr, K2 + 1, (int64_t)0);
        }
        hipLaunchKernelGGL(k_lv_fill32, dim3(grid_items(N)), dim3(kBlock), 0, s, w.minid, N, INT_MAX);
        hipLaunchKernelGGL(k_lv_minid, dim3(grid_items(N)), dim3(kBlock), 0, s, w.L, w.R, w.id, N, w.minid);
        hipLaunchKernelGGL(k_lv_newlabels, dim3(grid_items(N)), dim3(kBlock), 0, s, w.L, w.R, w.id, w.minid, N,
                           w.Lnext);
        hipLaunchKernelGGL(k_lv_top, dim3(grid_items(n)), dim3(kBlock), 0, s, w.R, w.id, n, w.top);
        if ((st = launch_status("leiden aggregation")) != RSC_OK) return st;
        std::swap(w.L, w.Lnext);
        G = H;
        gi = 1 - gi;
        N = K2;
    }
    // carry the labels down, number them by first appearance
    hipLaunchKernelGGL(k_lv_fill32, dim3(grid_items(N)), dim3(kBlock), 0, s, w.first, N, INT_MAX);
    hipLaunchKernelGGL(k_lv_first, dim3(grid_items(n)), dim3(kBlock), 0, s, w.L, w.top, n, w.first);
    hipLaunchKernelGGL(k_lv_mark, dim3(grid_items(n)), dim3(kBlock), 0, s, w.L, w.top, w.first, n, w.mark);
    if ((st = launch_status("leiden numbering")) != RSC_OK) return st;
    if ((st = hip_status(rocprim::exclusive_scan(w.tmp, w.tmp_bytes, (const int32_t *)w.mark, w.num, (int32_t)0,
                                                 (size_t)n, rocprim::plus<int32_t>(), s),
                         "scan of the community heads")) != RSC_OK)
        return st;
    hipLaunchKernelGGL(k_lv_labels, dim3(grid_items(n)), dim3(kBlock), 0, s, w.L, w.top, w.first, w.num, n, labels);
    if ((st = launch_status("leiden labels")) != RSC_OK) return st;
    int32_t last_num = 0, last_mark = 0;
    if ((st = hip_status(hipMemcpyAsync(&last_num, w.num + (n - 1), 4, hipMemcpyDeviceToHost, s), "read count")) !=
            RSC_OK ||
        (st = hip_status(hipMemcpyAsync(&last_mark, w.mark + (n - 1), 4, hipMemcpyDeviceToHost, s), "read count")) !=
            RSC_OK ||
        (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
        return st;
    const int64_t ncomm = (int64_t)last_num + last_mark;
    {
        double q = 0.0;
        if (two_m0 > 0.0) {
            hipLaunchKernelGGL(k_lv_fill64, dim3(grid_items(ncomm)), dim3(kBlock), 0, s, w.qin, ncomm, (int64_t)0);
            hipLaunchKernelGGL(k_lv_fill64, dim3(grid_items(ncomm)), dim3(kBlock), 0, s, w.qtot, ncomm, (int64_t)0);
            hipLaunchKernelGGL(k_lv_quality_sums, dim3(grid_waves(n)), dim3(kBlock), 0, s, indptr, indices, w.w0, n,
                               labels, w.qin, w.qtot);
            hipLaunchKernelGGL(k_lv_quality, dim3(1), dim3(64), 0, s, w.qin, w.qtot, ncomm, gamma, two_m0, w.q);
            if ((st = launch_status("leiden modularity")) != RSC_OK) return st;
            if ((st = read_back(&q, w.q, s, "read modularity")) != RSC_OK) return st;
        }
        if (stats) {
            stats->quality = q;
            stats->n_communities = ncomm;
            stats->levels = lv;
            stats->sweeps = sweeps;
            stats->rounds = rounds;
            stats->reserved = 0;
            stats->move_bytes = move_bytes;
        }
    }
    return RSC_OK;
}

}  // namespace rsc
