// Batched exact kNN: many independent samples in one persistent launch.
//
// A batch is S samples stored one after another (rows offsets[s] ..
// offsets[s+1]-1); every sample is its own kNN problem, so the graph is
// block-diagonal.  The paper processes large collections by chunks of cells
// (Methods, "Memory management and scaling"); here the whole batch sits in
// HBM and one launch covers every sample:
//   * the references of every sample are packed into one array (each
//     sample's last 32-row block padded);
//   * the host builds work items (sample, 128-query tile, reference range)
//     and orders them by a policy; a persistent grid (one workgroup slot per
//     CU and occupancy level) pops items from an atomic counter and runs the
//     FP32 MFMA screen of the exact path on each;
//   * rerank, certificate and exhaustive fallback are those of the exact
//     path, the fallback restricted to the row's own sample.
// The tile shape and the schedule are chosen by a measuring autotuner and
// cached per batch shape: the schedule policy (item order, default split
// rule), the screen tile's width (16 or 32 keys kept per query and
// contraction half) and, per log2 sample-size class, the tile's depth along
// the references (a sample's references cut into 1, 2 or 4 ranges, each a
// work item of its own).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "rsc_internal.hpp"
#include "screen_common.hpp"
#include "screen_fp32.hpp"

namespace rsc {

namespace {

using namespace scr;

struct BatchItem {
    int64_t q0;        // first query row, or (with a row list) first list entry
    int64_t b0, b1;    // packed reference blocks [b0, b1)
    int64_t ref_base;  // reference row of packed row 0 for this sample
    int32_t nq;        // queries in the tile (<= 128)
    int32_t p;         // range index the lists are filed under
};

struct BatchArgs {
    ScreenArgs base;
    const BatchItem *items;
    int n_items;
    int32_t *counter;
    const int32_t *rows;  // optional: query i of an item is row rows[q0 + i], filed under slot q0 + i
};

template <int DH, int L>
__global__ __launch_bounds__(256, tile_screen_waves(DH, L)) void k_screen_batched(BatchArgs ba) {
    __shared__ float2 qbuf[kQueueCap * 256];
    __shared__ int item_sh;
    const int tid = threadIdx.x;
    const int qi = (tid >> 6) * 32 + (tid & 31);  // query of this lane within the tile
    while (true) {
        if (tid == 0) item_sh = atomicAdd(ba.counter, 1);
        __syncthreads();
        const int it = item_sh;
        __syncthreads();  // every wave has read the item before it is overwritten
        if (it >= ba.n_items) break;
        const BatchItem I = ba.items[it];
        const bool live = qi < I.nq;
        const int64_t slot = live ? I.q0 + qi : -1;
        const int64_t row = live ? (ba.rows ? (int64_t)ba.rows[slot] : slot) : -1;
        screen_fp32_tile<DH, L>(ba.base, slot, row, I.b0, I.b1, I.p, I.ref_base, qbuf);
    }
}

__global__ void k_batch_init(int32_t *counter, int32_t *cand_idx, float *cand_key, int64_t n) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *counter = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        cand_idx[i] = -1;
        cand_key[i] = INFINITY;
    }
}

// ---------------------------------------------------------------------------
// Policies and plans (host).
// ---------------------------------------------------------------------------
constexpr int kMaxSplits = 4;  // reference ranges per sample a tile shape may ask for
constexpr int kBuckets = 40;   // log2 sample-size classes

struct Policy {
    int min_rows_split;  // samples with at least this many rows get 2 reference ranges (0 = never)
    int lpt;             // 0: items grouped by sample, largest sample first; 1: all items by cost
    const char *name;
};

const Policy kPolicies[RSC_BATCH_POLICIES] = {
    {0, 0, "grouped, no split"},
    {65536, 0, "grouped, split >= 64k rows"},
    {16384, 0, "grouped, split >= 16k rows"},
    {0, 1, "by cost, no split"},
    {65536, 1, "by cost, split >= 64k rows"},
    {16384, 1, "by cost, split >= 16k rows"},
};
constexpr int kDefaultPolicy = 0;

// What the autotuner chooses.
struct Shape {
    int policy = kDefaultPolicy;  // schedule policy (item order, default split rule)
    int half = 0;                 // keys per query and contraction half (16 or 32); 0: from k
    int8_t split[kBuckets] = {};  // reference ranges per sample by log2 size class; 0: the policy's rule
};

int size_bucket(int64_t n) {
    int b = 0;
    while (b < kBuckets - 1 && ((int64_t)1 << (b + 1)) <= n) ++b;
    return b;
}

std::string shape_text(const Shape &sh) {
    std::string t = "p" + std::to_string(sh.policy) + "h" + std::to_string(sh.half);
    for (int b = 0; b < kBuckets; ++b)
        if (sh.split[b]) t += "s" + std::to_string(b) + ":" + std::to_string((int)sh.split[b]);
    return t;
}

bool parse_shape(const std::string &t, Shape *out) {
    Shape sh;
    int pos = 0, v = 0, nread = 0;
    if (std::sscanf(t.c_str(), "p%dh%d%n", &sh.policy, &sh.half, &nread) != 2) return false;
    if (sh.policy < 0 || sh.policy >= RSC_BATCH_POLICIES || (sh.half != 0 && sh.half != 16 && sh.half != 32))
        return false;
    pos = nread;
    int b = 0;
    while (pos < (int)t.size()) {
        if (std::sscanf(t.c_str() + pos, "s%d:%d%n", &b, &v, &nread) != 2) return false;
        if (b < 0 || b >= kBuckets || v < 1 || v > kMaxSplits) return false;
        sh.split[b] = (int8_t)v;
        pos += nread;
    }
    *out = sh;
    return true;
}

struct BatchPlan {
    KnnPlan kp;
    int S = 0;
    int ranges = 1;  // reference ranges the items use (the candidate lists per query)
    std::vector<int64_t> soff, boff;
    std::vector<int32_t> blk_sample;
    std::vector<BatchItem> items;
};

int build_plan(const int64_t *offsets, int S, int d, int k, const Shape &sh, BatchPlan *out) {
    const Policy &pol = kPolicies[sh.policy];
    BatchPlan bp;
    bp.S = S;
    bp.soff.assign(offsets, offsets + S + 1);
    bp.boff.resize(S + 1);
    bp.boff[0] = 0;
    for (int s = 0; s < S; ++s) bp.boff[s + 1] = bp.boff[s] + (bp.soff[s + 1] - bp.soff[s] + 31) / 32;
    const int64_t N = bp.soff[S];
    int st = knn_plan(N, N, d, k, nullptr, true, &bp.kp);
    if (st != RSC_OK) return st;
    bp.kp.nblk = bp.boff[S];
    bp.kp.splits = kMaxSplits;
    if (sh.half == 32 && bp.kp.half == 16) {  // the wider screen tile
        bp.kp.half = 32;
        bp.kp.screen = 64;
    }
    bp.blk_sample.resize(bp.kp.nblk);
    for (int s = 0; s < S; ++s)
        for (int64_t b = bp.boff[s]; b < bp.boff[s + 1]; ++b) bp.blk_sample[b] = s;
    constexpr int QG = kScreenWaves * 32;
    std::vector<int> order(S);
    for (int s = 0; s < S; ++s) order[s] = s;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
        return bp.soff[a + 1] - bp.soff[a] > bp.soff[b + 1] - bp.soff[b];
    });
    for (int s : order) {
        const int64_t n = bp.soff[s + 1] - bp.soff[s];
        const int64_t nb = bp.boff[s + 1] - bp.boff[s];
        const int tuned = sh.split[size_bucket(n)];
        const int P = tuned > 0 ? (int)std::min<int64_t>(tuned, nb)
                                : ((pol.min_rows_split > 0 && n >= pol.min_rows_split) ? 2 : 1);
        const int64_t per = (nb + P - 1) / P;
        for (int64_t q = 0; q < n; q += QG) {
            for (int p = 0; p < P; ++p) {
                BatchItem it;
                it.q0 = bp.soff[s] + q;
                it.nq = (int32_t)std::min<int64_t>(QG, n - q);
                it.b0 = bp.boff[s] + p * per;
                it.b1 = std::min<int64_t>(bp.boff[s + 1], it.b0 + per);
                it.ref_base = bp.soff[s] - 32 * bp.boff[s];
                it.p = p;
                if (it.b1 > it.b0) bp.items.push_back(it);
            }
        }
    }
    for (const BatchItem &it : bp.items) bp.ranges = std::max(bp.ranges, (int)it.p + 1);
    if (pol.lpt)
        std::stable_sort(bp.items.begin(), bp.items.end(),
                         [](const BatchItem &a, const BatchItem &b) { return a.b1 - a.b0 > b.b1 - b.b0; });
    *out = std::move(bp);
    return RSC_OK;
}

constexpr int kEscCap = 8192;     // rows of the escalation pass (the rest are rescanned)
constexpr int kEscRanges = 16;    // reference ranges per sample in the escalation pass
constexpr int kEscHalf = 32;      // list length per contraction half (64-wide screen)

struct BatchBuffers {
    KnnBuffers kb;
    BatchItem *items;
    int32_t *blk_sample;
    int64_t *boff, *soff;
    int32_t *counter;
    BatchItem *esc_items;
    int32_t *esc_rows, *esc_count;
};

// Workspace: the exact path's buffers for the concatenated problem, then the
// batch tables.  Sized for the worst case over all tile shapes (the widest
// screen tile, the most reference ranges).
size_t batch_workspace(const BatchPlan &bp, void *ws, BatchBuffers *out) {
    BatchBuffers b;
    KnnPlan widest = bp.kp;  // any tile shape fits the same carving
    widest.half = 32;
    widest.screen = 64;
    const size_t base = knn_workspace(widest, nullptr, nullptr);
    knn_workspace(bp.kp, ws, &b.kb);
    Carver cv(ws ? static_cast<char *>(ws) + base : nullptr);
    constexpr int QG = kScreenWaves * 32;
    size_t max_items = 0;
    for (int s = 0; s < bp.S; ++s) max_items += (size_t)((bp.soff[s + 1] - bp.soff[s] + QG - 1) / QG) * kMaxSplits;
    b.items = cv.take<BatchItem>(std::max<size_t>(max_items, 1));
    b.blk_sample = cv.take<int32_t>((size_t)std::max<int64_t>(bp.kp.nblk, 1));
    b.boff = cv.take<int64_t>((size_t)bp.S + 1);
    b.soff = cv.take<int64_t>((size_t)bp.S + 1);
    b.counter = cv.take<int32_t>(1);
    // escalation: at most one partial tile per sample beyond the full ones
    const size_t esc_items = ((size_t)kEscCap / QG + (size_t)bp.S) * kEscRanges;
    b.esc_items = cv.take<BatchItem>(esc_items);
    b.esc_rows = cv.take<int32_t>(kEscCap);
    b.esc_count = cv.take<int32_t>(1);
    if (out) *out = b;
    return base + cv.used;
}

int device_slots(int dh) {
    static int cus = 0;
    if (cus == 0) {
        int dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
            cus = 256;
    }
    return cus * tile_screen_waves(dh, 16);
}

template <int DH>
int launch_batched_dh(const BatchArgs &ba, unsigned grid, int half, hipStream_t s) {
    if (half == 16)
        hipLaunchKernelGGL((k_screen_batched<DH, 16>), dim3(grid), dim3(256), 0, s, ba);
    else
        hipLaunchKernelGGL((k_screen_batched<DH, 32>), dim3(grid), dim3(256), 0, s, ba);
    return launch_status("screen_batched");
}

int launch_batched(const BatchPlan &bp, const BatchArgs &ba, hipStream_t s, int half = 0,
                   const char *name = "screen_batched") {
    ScopedTimer timer(name, s);
    if (half == 0) half = bp.kp.half;
    const unsigned grid = (unsigned)std::max(1, std::min<int>(device_slots(bp.kp.dh), ba.n_items));
    switch (bp.kp.dh) {
        case 4: return launch_batched_dh<4>(ba, grid, half, s);
        case 8: return launch_batched_dh<8>(ba, grid, half, s);
        case 16: return launch_batched_dh<16>(ba, grid, half, s);
        case 25: return launch_batched_dh<25>(ba, grid, half, s);
        case 32: return launch_batched_dh<32>(ba, grid, half, s);
        case 48: return launch_batched_dh<48>(ba, grid, half, s);
        case 64: return launch_batched_dh<64>(ba, grid, half, s);
        default: set_error("internal: no screen kernel for this dimension"); return RSC_ERR_UNSUPPORTED;
    }
}

// Upload the plan's tables into the workspace (synchronises the stream, so
// the host vectors may go out of scope afterwards).
int upload_plan(const BatchPlan &bp, const BatchBuffers &b, hipStream_t s) {
    int st;
    if ((st = hip_status(hipMemcpyAsync(b.items, bp.items.data(), bp.items.size() * sizeof(BatchItem),
                                        hipMemcpyHostToDevice, s), "upload items")) != RSC_OK)
        return st;
    if ((st = hip_status(hipMemcpyAsync(b.blk_sample, bp.blk_sample.data(), bp.blk_sample.size() * sizeof(int32_t),
                                        hipMemcpyHostToDevice, s), "upload block map")) != RSC_OK)
        return st;
    if ((st = hip_status(hipMemcpyAsync(b.boff, bp.boff.data(), bp.boff.size() * sizeof(int64_t),
                                        hipMemcpyHostToDevice, s), "upload block offsets")) != RSC_OK)
        return st;
    if ((st = hip_status(hipMemcpyAsync(b.soff, bp.soff.data(), bp.soff.size() * sizeof(int64_t),
                                        hipMemcpyHostToDevice, s), "upload row offsets")) != RSC_OK)
        return st;
    return hip_status(hipStreamSynchronize(s), "synchronise after upload");
}

BatchArgs batch_args(const BatchPlan &bp, const BatchBuffers &b, const float *X) {
    BatchArgs ba{};
    ba.base.Q = X;
    ba.base.nq = bp.kp.nq;
    ba.base.Ap = b.kb.packed;
    ba.base.Np = b.kb.norms;
    ba.base.nblk = bp.kp.nblk;
    ba.base.d = bp.kp.d;
    ba.base.P = bp.ranges;
    ba.base.cand_idx = b.kb.cand_idx;
    ba.base.cand_key = b.kb.cand_key;
    ba.items = b.items;
    ba.n_items = (int)bp.items.size();
    ba.counter = b.counter;
    return ba;
}

int screen_only(const BatchPlan &bp, const BatchBuffers &b, const float *X, hipStream_t s) {
    const int64_t ncand = bp.kp.nq * bp.ranges * bp.kp.screen;
    const unsigned g = (unsigned)std::min<int64_t>((ncand + 255) / 256, 65536);
    hipLaunchKernelGGL(k_batch_init, dim3(g), dim3(256), 0, s, b.counter, b.kb.cand_idx, b.kb.cand_key, ncand);
    int st = launch_status("batch init");
    if (st != RSC_OK) return st;
    return launch_batched(bp, batch_args(bp, b, X), s);
}

// ---------------------------------------------------------------------------
// Policy cache: key = device, d, k and the histogram of log2 sample sizes.
// ---------------------------------------------------------------------------
std::mutex g_cache_mu;
std::map<std::string, Shape> g_cache;
bool g_cache_loaded = false;
std::vector<std::string> g_trial_names;  // the trials of the last autotune call

std::string batch_key(const int64_t *offsets, int S, int d, int k) {
    int dev = 0, cus = 0;
    // (a failed query leaves 0 in the key: the cache entry is then shared
    // by devices that could not be told apart, which only costs a retune)
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) cus = 0;
    int hist[40] = {0};
    for (int s = 0; s < S; ++s) {
        const int64_t n = offsets[s + 1] - offsets[s];
        int b = 0;
        while (b < 39 && ((int64_t)1 << (b + 1)) <= n) ++b;
        ++hist[b];
    }
    std::string key = "cu" + std::to_string(cus) + ":d" + std::to_string(d) + ":k" + std::to_string(k) + ":";
    for (int b = 0; b < 40; ++b)
        if (hist[b]) key += std::to_string(b) + "x" + std::to_string(hist[b]) + ",";
    return key;
}

void load_cache_file() {
    if (g_cache_loaded) return;
    g_cache_loaded = true;
    const char *path = std::getenv("RSC_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "r");
    if (!f) return;
    char key[1024], val[1024];
    while (std::fscanf(f, "%1023s %1023s", key, val) == 2) {
        Shape sh;
        if (parse_shape(val, &sh)) g_cache[key] = sh;
    }
    std::fclose(f);
}

void store_cache(const std::string &key, const Shape &sh) {
    g_cache[key] = sh;
    const char *path = std::getenv("RSC_AUTOTUNE_CACHE");
    if (!path) return;
    FILE *f = std::fopen(path, "w");
    if (!f) return;
    for (auto &kv : g_cache) std::fprintf(f, "%s %s\n", kv.first.c_str(), shape_text(kv.second).c_str());
    std::fclose(f);
}

int check_batch_args(const float *X, const int64_t *offsets, int S, int d, int k, int32_t *out_idx, float *out_dist) {
    if (S < 1 || !offsets) {
        set_error("need S >= 1 samples and host offsets");
        return RSC_ERR_INVALID_ARG;
    }
    if (offsets[0] != 0) {
        set_error("offsets[0] must be 0");
        return RSC_ERR_INVALID_ARG;
    }
    for (int s = 0; s < S; ++s) {
        if (offsets[s + 1] - offsets[s] < k) {
            set_error("every sample needs at least k rows (sample " + std::to_string(s) + ")");
            return RSC_ERR_INVALID_ARG;
        }
    }
    if (offsets[S] > INT32_MAX - 1) {
        set_error("total rows above 2^31-2 cannot be indexed by int32");
        return RSC_ERR_OVERFLOW;
    }
    if (!X || !out_idx || !out_dist) {
        set_error("null device pointer");
        return RSC_ERR_INVALID_ARG;
    }
    (void)d;
    return RSC_OK;
}

// Rows the first pass could not certify: the first kEscCap of them are
// screened again 64 wide over up to kEscRanges ranges of their own sample
// (tiles of one sample, built on the host from the flagged rows) and
// re-ranked; rows that fail again, and rows beyond the cap, are rescanned
// exhaustively within their sample.  Synchronises the stream once.
int escalate(const BatchPlan &bp, const BatchBuffers &b, const float *X, int32_t *out_idx, float *out_dist,
             const RerankArgs &ra, hipStream_t s) {
    int32_t flagged = 0;
    int st = hip_status(hipMemcpyAsync(&flagged, &b.kb.counters->flagged, 4, hipMemcpyDeviceToHost, s),
                        "read flagged count");
    if (st == RSC_OK) st = hip_status(hipStreamSynchronize(s), "synchronise");
    if (st != RSC_OK) return st;
    const int c = std::min(flagged, kEscCap);
    if (c > 0) {
        std::vector<int32_t> rows(c);
        if ((st = hip_status(hipMemcpyAsync(rows.data(), b.kb.flag1, (size_t)c * 4, hipMemcpyDeviceToHost, s),
                             "read flagged rows")) != RSC_OK ||
            (st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK)
            return st;
        std::sort(rows.begin(), rows.end());
        constexpr int QG = kScreenWaves * 32;
        std::vector<BatchItem> items;
        size_t i = 0;
        while (i < rows.size()) {
            const int smp = (int)(std::upper_bound(bp.soff.begin(), bp.soff.end(), (int64_t)rows[i]) -
                                  bp.soff.begin()) - 1;
            size_t e = i;
            while (e < rows.size() && e - i < (size_t)QG && rows[e] < bp.soff[smp + 1]) ++e;
            const int64_t nb = bp.boff[smp + 1] - bp.boff[smp];
            const int P = (int)std::max<int64_t>(1, std::min<int64_t>(kEscRanges, nb / 8));
            const int64_t per = (nb + P - 1) / P;
            for (int p = 0; p < P; ++p) {
                BatchItem it;
                it.q0 = (int64_t)i;
                it.nq = (int32_t)(e - i);
                it.b0 = bp.boff[smp] + p * per;
                it.b1 = std::min<int64_t>(bp.boff[smp + 1], it.b0 + per);
                it.ref_base = bp.soff[smp] - 32 * bp.boff[smp];
                it.p = p;
                if (it.b1 > it.b0) items.push_back(it);
            }
            i = e;
        }
        if ((st = hip_status(hipMemcpyAsync(b.esc_items, items.data(), items.size() * sizeof(BatchItem),
                                            hipMemcpyHostToDevice, s), "upload escalation items")) != RSC_OK ||
            (st = hip_status(hipMemcpyAsync(b.esc_rows, rows.data(), (size_t)c * 4, hipMemcpyHostToDevice, s),
                             "upload escalation rows")) != RSC_OK ||
            (st = hip_status(hipMemcpyAsync(b.esc_count, &c, 4, hipMemcpyHostToDevice, s), "upload count")) !=
                RSC_OK)
            return st;
        const int64_t ncand = (int64_t)c * kEscRanges * 2 * kEscHalf;
        const unsigned g = (unsigned)std::min<int64_t>((ncand + 255) / 256, 65536);
        hipLaunchKernelGGL(k_batch_init, dim3(g), dim3(256), 0, s, b.counter, b.kb.esc_idx, b.kb.esc_key, ncand);
        if ((st = launch_status("escalation init")) != RSC_OK) return st;
        BatchArgs ba = batch_args(bp, b, X);
        ba.base.P = kEscRanges;
        ba.base.cand_idx = b.kb.esc_idx;
        ba.base.cand_key = b.kb.esc_key;
        ba.items = b.esc_items;
        ba.n_items = (int)items.size();
        ba.rows = b.esc_rows;
        if ((st = launch_batched(bp, ba, s, kEscHalf, "screen_escalate")) != RSC_OK) return st;
        RerankArgs re = ra;
        re.qlist = b.esc_rows;
        re.qcount = b.esc_count;
        re.qcap = c;
        re.S = kEscHalf;
        re.KP = kEscHalf;
        re.P = 2 * kEscRanges;
        re.cand_idx = b.kb.esc_idx;
        re.cand_key = b.kb.esc_key;
        re.flag_out = b.kb.flag2;
        re.flag_count = &b.kb.counters->flagged2;
        if ((st = knn_launch_rerank(re, c, "rerank_escalate", s)) != RSC_OK) return st;
        // the upload of the host vectors must finish before they go out of scope
        if ((st = hip_status(hipStreamSynchronize(s), "synchronise")) != RSC_OK) return st;
    }
    return knn_launch_rescan(bp.kp, X, X, b.kb, c, out_idx, out_dist, b.soff, bp.S, s);
}

}  // namespace

size_t batched_workspace_bytes(const int64_t *offsets, int S, int d, int k) {
    if (S < 1 || !offsets || offsets[0] != 0) return 0;
    for (int s = 0; s < S; ++s)
        if (offsets[s + 1] - offsets[s] < k) return 0;
    BatchPlan bp;
    if (build_plan(offsets, S, d, k, Shape(), &bp) != RSC_OK) return 0;
    return batch_workspace(bp, nullptr, nullptr);
}

int batched_run(const float *X, const int64_t *offsets, int S, int d, int k, int32_t *out_idx, float *out_dist,
                void *ws, size_t ws_bytes, hipStream_t s) {
    int st = check_batch_args(X, offsets, S, d, k, out_idx, out_dist);
    if (st != RSC_OK) return st;
    Shape sh;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        load_cache_file();
        auto it = g_cache.find(batch_key(offsets, S, d, k));
        if (it != g_cache.end()) sh = it->second;
    }
    BatchPlan bp;
    if ((st = build_plan(offsets, S, d, k, sh, &bp)) != RSC_OK) return st;
    BatchBuffers b;
    const size_t need = batch_workspace(bp, ws, &b);
    if (!ws || need > ws_bytes) {
        set_error("workspace too small: need " + std::to_string(need) + " bytes");
        return RSC_ERR_WORKSPACE;
    }
    if ((st = upload_plan(bp, b, s)) != RSC_OK) return st;
    if ((st = knn_prep_fp32(bp.kp, X, b.kb, b.blk_sample, b.boff, b.soff, s)) != RSC_OK) return st;
    if ((st = screen_only(bp, b, X, s)) != RSC_OK) return st;
    RerankArgs ra{};
    ra.Q = X;
    ra.nq = bp.kp.nq;
    ra.R = X;
    ra.d = d;
    ra.k = k;
    ra.S = bp.kp.half;
    ra.KP = bp.kp.half;
    ra.P = 2 * bp.ranges;
    ra.self_mode = 1;
    ra.certify = 1;
    ra.cand_idx = b.kb.cand_idx;
    ra.cand_key = b.kb.cand_key;
    ra.eps_coef = knn_eps_coefficient(d);
    ra.counters = b.kb.counters;
    ra.flag_out = b.kb.flag1;
    ra.flag_count = &b.kb.counters->flagged;
    ra.out_idx = out_idx;
    ra.out_dist = out_dist;
    if ((st = knn_launch_rerank(ra, bp.kp.nq, "rerank", s)) != RSC_OK) return st;
    return escalate(bp, b, X, out_idx, out_dist, ra, s);
}

int batched_autotune(const float *X, const int64_t *offsets, int S, int d, int k, void *ws, size_t ws_bytes,
                     hipStream_t s, int32_t *chosen, float *times_ms) {
    float dummy_f = 0.f;
    int32_t dummy_i = 0;
    int st = check_batch_args(X, offsets, S, d, k, &dummy_i, &dummy_f);
    if (st != RSC_OK) return st;
    if (times_ms)
        for (int t = 0; t < RSC_BATCH_TRIALS; ++t) times_ms[t] = NAN;
    hipEvent_t e0, e1;
    if ((st = hip_status(hipEventCreate(&e0), "event")) != RSC_OK) return st;
    if ((st = hip_status(hipEventCreate(&e1), "event")) != RSC_OK) {
        (void)hipEventDestroy(e0);
        return st;
    }
    std::vector<std::string> names;
    bool prepared = false;
    // Time the screen of one tile shape (a warm run first for the first trial).
    auto trial = [&](const Shape &sh, const std::string &name, float *ms_out) -> int {
        BatchPlan bp;
        int r = build_plan(offsets, S, d, k, sh, &bp);
        if (r != RSC_OK) return r;
        BatchBuffers b;
        const size_t need = batch_workspace(bp, ws, &b);
        if (!ws || need > ws_bytes) {
            set_error("workspace too small: need " + std::to_string(need) + " bytes");
            return RSC_ERR_WORKSPACE;
        }
        if ((r = upload_plan(bp, b, s)) != RSC_OK) return r;
        if (!prepared) {
            // the packed references do not depend on the shape
            if ((r = knn_prep_fp32(bp.kp, X, b.kb, b.blk_sample, b.boff, b.soff, s)) != RSC_OK) return r;
            if ((r = screen_only(bp, b, X, s)) != RSC_OK) return r;  // warm
            prepared = true;
        }
        if ((r = hip_status(hipEventRecord(e0, s), "event")) != RSC_OK) return r;
        if ((r = screen_only(bp, b, X, s)) != RSC_OK) return r;
        if ((r = hip_status(hipEventRecord(e1, s), "event")) != RSC_OK) return r;
        if ((r = hip_status(hipEventSynchronize(e1), "event")) != RSC_OK) return r;
        if ((r = hip_status(hipEventElapsedTime(ms_out, e0, e1), "event time")) != RSC_OK) return r;
        if (times_ms && (int)names.size() < RSC_BATCH_TRIALS) times_ms[names.size()] = *ms_out;
        names.push_back(name);
        return RSC_OK;
    };
    Shape best;
    float best_ms = INFINITY;
    int best_trial = -1;
    auto consider = [&](const Shape &sh, const std::string &name) -> int {
        float ms = 0.f;
        const int r = trial(sh, name, &ms);
        if (r == RSC_OK && ms < best_ms) {
            best_ms = ms;
            best = sh;
            best_trial = (int)names.size() - 1;
        }
        return r;
    };
    // 1. the schedule policies (default tile)
    for (int pol = 0; pol < RSC_BATCH_POLICIES && st == RSC_OK; ++pol) {
        Shape sh;
        sh.policy = pol;
        st = consider(sh, std::string("policy: ") + kPolicies[pol].name);
    }
    // 2. the wider screen tile (32 keys per query and half), when k leaves the choice
    if (st == RSC_OK && k <= 16) {
        Shape sh = best;
        sh.half = 32;
        st = consider(sh, std::string("tile 32 keys/half, ") + kPolicies[best.policy].name);
    }
    // 3. the tile's depth per size class, heaviest classes first
    if (st == RSC_OK) {
        double work[kBuckets] = {0.0}, total = 0.0;
        for (int i = 0; i < S; ++i) {
            const double n = (double)(offsets[i + 1] - offsets[i]);
            work[size_bucket(offsets[i + 1] - offsets[i])] += n * n;
            total += n * n;
        }
        std::vector<int> order;
        for (int b = 0; b < kBuckets; ++b)
            if (work[b] >= 0.05 * total) order.push_back(b);
        std::sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
        for (int b : order) {
            const Shape base = best;
            for (int sp : {1, 2, 4}) {
                if (st != RSC_OK) break;
                Shape sh = base;
                sh.split[b] = (int8_t)sp;
                const bool same_as_base = base.split[b] == sp;
                if (same_as_base) continue;
                st = consider(sh, "size class 2^" + std::to_string(b) + ": " + std::to_string(sp) +
                                      " reference range(s) per sample, on top of the best so far");
            }
        }
    }
    const hipError_t d0 = hipEventDestroy(e0), d1 = hipEventDestroy(e1);
    if (st != RSC_OK) return st;
    if ((st = hip_status(d0 != hipSuccess ? d0 : d1, "event destroy")) != RSC_OK) return st;
    {
        std::lock_guard<std::mutex> lock(g_cache_mu);
        load_cache_file();
        store_cache(batch_key(offsets, S, d, k), best);
        g_trial_names = names;
        if (best_trial >= 0 && best_trial < (int)g_trial_names.size())
            g_trial_names[best_trial] += " [chosen: " + shape_text(best) + "]";
    }
    if (chosen) *chosen = best_trial;
    return RSC_OK;
}

const char *batched_trial_name(int t) {
    std::lock_guard<std::mutex> lock(g_cache_mu);
    if (t < 0 || t >= (int)g_trial_names.size()) return "";
    return g_trial_names[t].c_str();
}

const char *batched_policy_name(int pol) {
    if (pol < 0 || pol >= RSC_BATCH_POLICIES) return "";
    return kPolicies[pol].name;
}

}  // namespace rsc
