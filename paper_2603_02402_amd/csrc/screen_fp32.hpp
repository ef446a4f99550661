// The FP32 MFMA screen of one 128-query tile over a range of packed
// reference blocks, shared by the grid-mapped and the persistent (batched)
// launches.
#pragma once

#include "screen_common.hpp"

namespace rsc {
namespace scr {

// Whether the contraction half-width DH leaves a spare slot in its last
// float4 for the reference norm (the common d = 49, 50 case: DH = 25).
__host__ __device__ constexpr bool norm_folded(int DH) { return (DH % 4) != 0; }
__host__ __device__ constexpr int packed_s4(int DH) { return (DH + (norm_folded(DH) ? 1 : 0) + 3) / 4; }

// Occupancy target (waves per SIMD) that the register budget of a screen
// instantiation allows without spilling.
__host__ __device__ constexpr int screen_min_waves(int DH, int L) {
    return (DH <= 25 && L == 16) ? 3 : DH <= 64 ? 2 : 1;
}

// Occupancy target of the launches that run the tile code alone over a
// full grid (the grid-mapped screen and the persistent batched one): for
// d <= 50, 4 waves per SIMD with lists of 16, whose block loop fits 128
// registers (the few values the compiler spills are addresses used outside
// the loop), and 3 with lists of 32 (167 registers, no spills).  A sparse
// grid (the escalation's few rows) keeps screen_min_waves: built for more
// resident waves, the chain hides less latency when a wave runs alone.
__host__ __device__ constexpr int tile_screen_waves(int DH, int L) {
    return DH <= 25 ? (L == 16 ? 4 : 3) : screen_min_waves(DH, L);
}

// Load float4 group s4 of a packed block (wave-uniform base wb).  A partial
// last group (STEPS not a multiple of 4) is fetched with a narrower load so
// that no dead register half is left pending under a load.
template <int STEPS, int S4>
__device__ __forceinline__ void load_group(f32x4 (&A)[S4], const f32x4 *wb, int s4, int lane) {
    constexpr int REM = STEPS - 4 * (S4 - 1);
    if (s4 < S4 - 1 || REM >= 3) {
        A[s4] = wb[s4 * kWave + lane];
    } else if (REM == 2) {
        const float2 t = reinterpret_cast<const float2 *>(wb + s4 * kWave + lane)[0];
        A[s4][0] = t.x;
        A[s4][1] = t.y;
    } else {
        A[s4][0] = reinterpret_cast<const float *>(wb + s4 * kWave + lane)[0];
    }
}

// Screen.
//
// Lane l handles query c = l % 32 of its wave and contraction half
// h = l / 32: a step of the MFMA chain multiplies dimension h*DH + t (plus
// the norm step, first, when folded).  Output register v of the 32x32 block
// holds reference row 8(v/4) + 4h + (v%4), so each lane sees half of the
// references of every block and keeps its own sorted list of the L smallest
// keys of that half.

// Query operand of one lane: -2 x (exact scaling) over the lane's half of
// the contraction, plus the factor 1 of the folded norm step.
template <int DH>
struct Fp32Query {
    static constexpr bool NF = norm_folded(DH);
    static constexpr int STEPS = DH + (NF ? 1 : 0);
    float b[STEPS];

    __device__ __forceinline__ void load(const ScreenArgs &a, int64_t row, int h) {
        constexpr int OFF = NF ? 1 : 0;  // step 0 carries the norm when folded
#pragma unroll
        for (int s = 0; s < DH; ++s) {
            const int t = h * DH + s;
            b[OFF + s] = (row >= 0 && t < a.d) ? -2.f * a.Q[row * a.d + t] : 0.f;
        }
        if constexpr (NF) b[0] = (row >= 0 && h == 0) ? 1.f : 0.f;
    }
};

// Issue the loads of packed block `blk` into A (in group order).
template <int DH>
__device__ __forceinline__ void load_block(const ScreenArgs &a, f32x4 (&A)[packed_s4(DH)], int64_t blk) {
    constexpr int STEPS = DH + (norm_folded(DH) ? 1 : 0);
    constexpr int S4 = packed_s4(DH);
    const int lane = threadIdx.x & (kWave - 1);
    const f32x4 *wb0 = static_cast<const f32x4 *>(a.Ap) + blk * (S4 * kWave);
#pragma unroll
    for (int s4 = 0; s4 < S4; ++s4) {
        load_group<STEPS, S4>(A, wb0, s4, lane);
        __builtin_amdgcn_sched_barrier(0);  // issue in group order, as the block step does
    }
}

// One block of the chain: A holds block `blk`; its float4 groups are
// replaced by those of block `nxt` as soon as the MFMAs have consumed them
// (nxt may be blk itself at the end of a stream: always in bounds, so the
// loads need no branch and stay in flight across the MFMAs).  The keys are
// offered to `top` as rows ref_base + 32 blk + 8(v/4) + 4h + (v%4); with
// MASK, a lane whose `active` is false offers nothing.
template <int DH, int L, bool MASK>
__device__ __forceinline__ void screen_block(const ScreenArgs &a, const Fp32Query<DH> &qop, LaneTopK<L> &top,
                                             f32x4 (&A)[packed_s4(DH)], int64_t blk, int64_t nxt, int64_t ref_base,
                                             float2 *q, bool active) {
    constexpr bool NF = norm_folded(DH);
    constexpr int STEPS = DH + (NF ? 1 : 0);
    constexpr int S4 = packed_s4(DH);
    const int lane = threadIdx.x & (kWave - 1);
    const int h = lane >> 5;
    f32x4 nv[4];
    if constexpr (!NF) {
        const f32x4 *ns = reinterpret_cast<const f32x4 *>(a.Np + blk * 32 + h * 16);
#pragma unroll
        for (int g = 0; g < 4; ++g) nv[g] = ns[g];
    }
    const f32x4 *wb = static_cast<const f32x4 *>(a.Ap) + nxt * (S4 * kWave);
    f32x16 acc = f32x16{};
#pragma unroll
    for (int s4 = 0; s4 < S4; ++s4) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int s = 4 * s4 + u;
            if (s < STEPS) acc = __builtin_amdgcn_mfma_f32_32x32x2f32(A[s4][u], qop.b[s], acc, 0, 0, 0);
        }
        load_group<STEPS, S4>(A, wb, s4, lane);  // consumed: fetch its successor
        // keep each load right behind the MFMAs that freed its registers
        __builtin_amdgcn_sched_barrier(0);
    }
    if constexpr (!NF) {
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] += nv[v >> 2][v & 3];
    }
    if constexpr (MASK) {
#pragma unroll
        for (int v = 0; v < 16; ++v) acc[v] = active ? acc[v] : INFINITY;
    }
    top.offer(acc, (int)(ref_base + blk * 32) + 4 * h, q, 256);
}

// Stream packed blocks [blk0, blk1) through the MFMA chain and offer the
// keys to `top`.  Every lane of the wave calls this together.
template <int DH, int L>
__device__ __forceinline__ void scan_blocks(const ScreenArgs &a, const Fp32Query<DH> &qop, LaneTopK<L> &top,
                                            int64_t blk0, int64_t blk1, int64_t ref_base, float2 *q) {
    f32x4 A[packed_s4(DH)] = {};
    if (blk0 < blk1) load_block<DH>(a, A, blk0);
    for (int64_t blk = blk0; blk < blk1; ++blk) {
        const int64_t nxt = blk + 1 < blk1 ? blk + 1 : blk;
        screen_block<DH, L, false>(a, qop, top, A, blk, nxt, ref_base, q, true);
    }
}

// One tile: slot: this lane's output slot (or -1); row: its query row (or
// -1); blocks [blk0, blk1) of the packed array; p: the range index the lists
// are filed under; ref_base: reference row of packed row 0.
template <int DH, int L>
__device__ __forceinline__ void screen_fp32_tile(const ScreenArgs &a, int64_t slot, int64_t row, int64_t blk0,
                                                 int64_t blk1, int p, int64_t ref_base, float2 *qbuf) {
    const int tid = threadIdx.x;
    const int h = (tid & (kWave - 1)) >> 5;
    Fp32Query<DH> qop;
    qop.load(a, row, h);
    LaneTopK<L> top;
    top.init();
    float2 *q = qbuf + tid;
    scan_blocks<DH, L>(a, qop, top, blk0, blk1, ref_base, q);
    top.flush(q, 256);
    if (slot >= 0) top.store(a, slot, p, h);
}

}  // namespace scr
}  // namespace rsc
