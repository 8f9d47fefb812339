// Kernels of the host-driven multi-model level step, shared by the batch
// driver and the server: every unfinished model's current level is expanded
// in one launch (global tiles mapped to models by a prefix over their tile
// counts), roots are inserted per model, and discarded levels rolled back.
#pragma once

#include <algorithm>

#include "expand_device.h"
#include "internal.h"
#include "reach_internal.h"

namespace {

using namespace lhs;

// One model's expansion work of the current step.
struct BatchSlot {
    TableView t;
    ModelView m;
    const uint32_t *front;
    uint32_t *next;
    LevelCounters *lc;
    uint32_t n_front;
    uint32_t limit;
    uint32_t tile_begin;   // first global tile of this model in the step
    uint32_t pad;
};

__device__ __forceinline__ uint32_t find_slot_by_tile(const uint32_t *begin, uint32_t n, uint32_t g) {
    uint32_t lo = 0, hi = n;   // begin[lo] <= g < begin[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (begin[mid] <= g)
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

// ---- host-driven step ---------------------------------------------------
template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock) void k_expand_multi(const BatchSlot *__restrict__ slots,
                                                               const uint32_t *__restrict__ begin,
                                                               uint32_t n_slots, uint32_t total_tiles,
                                                               uint32_t tcap) {
    extern __shared__ uint32_t smem[];
    expand_begin();
    for (uint32_t g = blockIdx.x; g < total_tiles; g += gridDim.x) {
        const BatchSlot &s = slots[find_slot_by_tile(begin, n_slots, g)];
        const uint64_t base = (uint64_t)(g - s.tile_begin) * kExpandBlock;
        const uint32_t rows = (uint32_t)min<uint64_t>(kExpandBlock, s.n_front - base);
        expand_tile<G, LS>(smem, s.t, s.m, s.front, base, rows, s.next, s.lc, s.limit, tcap);
    }
}

[[maybe_unused]] __global__ void k_zero_levels(LevelCounters *lc, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        lc[i] = LevelCounters{0, 0, 0, 0};
}

// Insert each model's initial state (level 0): block b handles model b.
struct LdsRowB {
    const uint32_t *r;
    __device__ __forceinline__ uint32_t get(uint32_t i) const { return r[i]; }
};

template <uint32_t LS>
__global__ void k_insert_roots(const BatchSlot *slots, const uint32_t *roots, const uint32_t *root_off,
                               uint32_t n) {
    __shared__ uint32_t row[32];
    const uint32_t b = blockIdx.x;
    if (b >= n)
        return;
    const BatchSlot &s = slots[b];
    if (threadIdx.x < s.m.W)
        row[threadIdx.x] = roots[root_off[b] + threadIdx.x];
    __syncthreads();
    if (threadIdx.x < 64) {
        LaneCounters cnt;
        const LdsRowB v{row};
        const bool active = threadIdx.x == 0;
        uint32_t slot = kNoSlot, code = kFull;
        const uint64_t h = hash_vec(v, s.m.W, s.t.seed);
        find_or_put<1, LS>(s.t, v, h, active, slot, code, cnt);
        if (active)
            const_cast<uint32_t *>(s.front)[0] = slot;
    }
}

// Undo a discarded level of one model (see reach.hip).
[[maybe_unused]] __global__ void k_rollback_one(uint64_t *bucket, const uint32_t *next, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        bucket[next[i]] = 0;
}


// Insert the roots of slots[0, n) (every table has line width ls).
inline lhs_status launch_insert_roots(uint32_t ls, hipStream_t s, const BatchSlot *slots, const uint32_t *roots,
                                      const uint32_t *root_off, uint32_t n) {
    return with_line_slots(ls, [&](auto L) {
        hipLaunchKernelGGL((k_insert_roots<decltype(L)::value>), dim3(n), dim3(64), 0, s, slots, roots,
                           root_off, n);
        return LHS_OK;
    });
}

// tcap: LDS entries for transitions (max over the step's models that fit).
inline lhs_status launch_expand_multi(uint32_t tps, uint32_t ls, uint32_t tiles, uint32_t max_W, uint32_t tcap,
                                      hipStream_t s, const BatchSlot *slots, const uint32_t *begin, uint32_t n) {
    const dim3 grid(std::min<uint32_t>(std::max(tiles, 1u), 1u << 16));
    const size_t lds = (size_t)expand_lds_words(max_W, tcap, tps) * sizeof(uint32_t);
    return with_shape(tps, ls, [&](auto G, auto L) {
        hipLaunchKernelGGL((k_expand_multi<decltype(G)::value, decltype(L)::value>), grid, dim3(kExpandBlock),
                           lds, s, slots, begin, n, tiles, tcap);
        return LHS_OK;
    });
}

}  // namespace
