// Spatial order of the query rows for the reduced-precision screens.
//
// The screens keep, per lane, a queue of keys that beat the lane's threshold
// and merge all lanes' queues together whenever one of them could overflow.
// When the 32 queries of a wave lie close together, the references that
// enter one query's list tend to enter its neighbours' too, so the queues
// fill together and fewer merges and fewer blocks with any key below a
// threshold occur.  The order is a Morton (Z-order) code of the first three
// coordinates, each quantised to 10 bits over its range, sorted by rocPRIM's
// radix sort; the rows' results are written back in row order, so the order
// changes which candidates a screen keeps only through the threshold
// history, never the rows of the answer.

#include <hip/hip_runtime.h>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstdint>

#include "morton.hpp"
#include "rsc_internal.hpp"

namespace rsc {
namespace {

constexpr int kOrderDims = 3;
constexpr int kOrderBits = 10;  // per coordinate (quantise10): 30-bit keys

__global__ void k_qo_init(uint32_t *bounds) {
    if (threadIdx.x < kOrderDims) {
        bounds[2 * threadIdx.x] = 0xffffffffu;  // running minimum (ordered bits)
        bounds[2 * threadIdx.x + 1] = 0u;       // running maximum
    }
}

__global__ __launch_bounds__(256) void k_qo_bounds(const float *__restrict__ Q, int64_t nq, int d, int D,
                                                   uint32_t *__restrict__ bounds) {
    uint32_t lo[kOrderDims], hi[kOrderDims];
#pragma unroll
    for (int t = 0; t < kOrderDims; ++t) {
        lo[t] = 0xffffffffu;
        hi[t] = 0u;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
        for (int t = 0; t < kOrderDims; ++t) {
            if (t < D) {
                const uint32_t u = ordered_bits(Q[i * d + t]);
                lo[t] = min(lo[t], u);
                hi[t] = max(hi[t], u);
            }
        }
    }
#pragma unroll
    for (int t = 0; t < kOrderDims; ++t) {
        if (t < D) {
            atomicMin(&bounds[2 * t], lo[t]);
            atomicMax(&bounds[2 * t + 1], hi[t]);
        }
    }
}

__global__ __launch_bounds__(256) void k_qo_keys(const float *__restrict__ Q, int64_t nq, int d, int D,
                                                 const uint32_t *__restrict__ bounds, uint32_t *__restrict__ key,
                                                 int32_t *__restrict__ row) {
    float lo[kOrderDims], scale[kOrderDims];
#pragma unroll
    for (int t = 0; t < kOrderDims; ++t) {
        lo[t] = 0.f;
        scale[t] = 0.f;
        if (t < D) {
            const float a = from_ordered(bounds[2 * t]), b = from_ordered(bounds[2 * t + 1]);
            lo[t] = a;
            scale[t] = scale10(a, b);
        }
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += (int64_t)gridDim.x * blockDim.x) {
        uint32_t k = 0;
#pragma unroll
        for (int t = 0; t < kOrderDims; ++t) {
            if (t < D) {
                k |= spread3(quantise10(Q[i * d + t], lo[t], scale[t])) << (kOrderDims - 1 - t);
            }
        }
        key[i] = k;
        row[i] = (int32_t)i;
    }
}

struct OrderWs {
    uint32_t *bounds, *key, *key2;
    int32_t *row;
    void *tmp;
    size_t tmp_bytes;
};

size_t carve_order(int64_t nq, void *base, OrderWs *out) {
    const size_t m = (size_t)std::max<int64_t>(nq, 1);
    size_t tmp = 0;
    if (rocprim::radix_sort_pairs(nullptr, tmp, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                                  (const int32_t *)nullptr, (int32_t *)nullptr, m, 0, kOrderDims * kOrderBits,
                                  (hipStream_t)0) != hipSuccess)
        return 0;
    Carver cv(base);
    OrderWs w{};
    w.bounds = cv.take<uint32_t>(2 * kOrderDims);
    w.key = cv.take<uint32_t>(m);
    w.key2 = cv.take<uint32_t>(m);
    w.row = cv.take<int32_t>(m);
    w.tmp_bytes = tmp;
    w.tmp = cv.take<char>(tmp ? tmp : 1);
    if (out) *out = w;
    return cv.used;
}

}  // namespace

size_t query_order_workspace(int64_t nq) { return carve_order(nq, nullptr, nullptr); }

int query_order_run(const float *Q, int64_t nq, int d, void *ws, int32_t *perm, hipStream_t s) {
    if (nq <= 0) return RSC_OK;
    OrderWs w;
    if (!carve_order(nq, ws, &w)) {
        set_error("query order: rocPRIM sort sizing failed");
        return RSC_ERR_HIP;
    }
    ScopedTimer timer("query_order", s);
    const int D = std::min(d, kOrderDims);
    const unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nq + 255) / 256, 4096));
    hipLaunchKernelGGL(k_qo_init, dim3(1), dim3(64), 0, s, w.bounds);
    hipLaunchKernelGGL(k_qo_bounds, dim3(std::min(g, 1024u)), dim3(256), 0, s, Q, nq, d, D, w.bounds);
    hipLaunchKernelGGL(k_qo_keys, dim3(g), dim3(256), 0, s, Q, nq, d, D, w.bounds, w.key, w.row);
    int st = launch_status("query order keys");
    if (st != RSC_OK) return st;
    return hip_status(rocprim::radix_sort_pairs(w.tmp, w.tmp_bytes, (const uint32_t *)w.key, w.key2,
                                                (const int32_t *)w.row, perm, (size_t)nq, 0,
                                                kOrderDims * kOrderBits, s),
                      "sort of the query order");
}

}  // namespace rsc
