// Device view of a model and helpers shared by the reachability units.
#pragma once

#include <vector>

#include "internal.h"

// Packed transition table [P][L][K] of uint2:
//   x = target | guard_var << 16 | eff_var << 24   (0xFF = none)
//   y = guard_val | eff_val << 16
struct ModelView {
    const uint2 *trans;
    uint32_t P, L, S, K, W;
    uint32_t magic_PK;   // ceil(2^32 / (P*K)) for __umulhi division
    uint32_t magic_K;
    uint32_t pad;
    unsigned long long key;   // tells apart models whose transitions reuse one
                              // buffer (0 where every model has a buffer of its own)
};

// Segmented next frontiers of single-model levels (expand_device.h): the
// number of segments and the distance of their append cursors, in words.
constexpr uint32_t kSegs = 8;
constexpr uint32_t kSegStride = 32;
constexpr size_t kSegCursorBytes = kSegs * kSegStride * sizeof(uint32_t);

// What a level leaves for the host loop, written by one small kernel into
// pinned host memory: its counters, its segment counts and the table's
// status (one write, no copies).
struct LevelSummary {
    LevelCounters lc;
    uint32_t seg_n[kSegs];
    lhs::DevStatus st;
};

// Device-side state of a graph-driven exploration (REACH_F_GRAPH): the level
// loop's bookkeeping, advanced by a kernel after every level so that levels
// can be replayed from a captured graph without the host.
struct LevelCtl {
    unsigned long long total, edges, deadlocks, cap;
    unsigned long long *levels;    // [max_levels] level counts (levels[0] = 1)
    uint32_t cur, n_front, limit, n_levels, max_levels;
    uint32_t done, capped, overflow, rollback_n, pad;
};

// Everything the graph's kernels read: one device struct per table, so a
// captured graph stays valid for any model explored on that table.
struct GraphCtx {
    lhs::TableView t;
    ModelView m;
    uint32_t *fr[2];
    LevelCounters *lc;
    LevelCtl ctl;
    uint32_t *segs;              // append cursors of the next frontier
    uint32_t seg_size;           // entries per segment
    uint32_t front_n[kSegs];     // entries per segment of the current frontier
    uint32_t rb_n[kSegs];        // ... of a discarded level (k_rollback_graph)
};

// Shared state of an exploration without level barriers (REACH_F_ASYNC).
// Each counter sits on a 128-byte line of its own: all workgroups poll or
// update them.
struct alignas(128) AsyncCtl {
    unsigned long long work;   // states discovered and not yet expanded
    char pad0[120];
    uint32_t chunk;            // next queue chunk to hand out
    char pad1[124];
    uint32_t error;            // LHS_ESTALL when a bounded wait ran out
    char pad2[124];
};

namespace lhs {

lhs_status validate_model(const reach_model *m);
void pack_model(const reach_model *m, std::vector<uint2> &out);
ModelView model_view(const reach_model *m, const uint2 *d_trans);
size_t expand_lds_bytes(uint32_t W, uint32_t tcap, uint32_t tps);
lhs_status ensure_bfs_buffers(lhs_table *t);

// The first levels of a single-model BFS in one persistent launch (the batch
// kernel on one model), until a level exceeds kPrefixHandover states: small
// levels then cost a tile's latency each instead of a launch and a host
// round trip.  s0 must be frontier[0][0] and the level counters zero.
struct PrefixArea;
struct PrefixOut {
    std::vector<uint64_t> levels;   // counts of levels 1, 2, ...
    uint64_t total = 1, edges = 0, deadlocks = 0;
    uint32_t cur = 0;               // frontier buffer of the last level
    bool handed = false;            // stopped after a level above the threshold
    bool capped = false;
};
lhs_status explore_prefix(lhs_table *t, const TableView &tv, const ModelView &mv, uint64_t cap,
                          PrefixArea *d_area, PrefixArea *h_area, hipStream_t s, PrefixOut &out);
uint64_t auto_capacity(const reach_model *m);
// The view a BFS on t expands with: predecessor records when requested.
TableView bfs_view(lhs_table *t, bool parents);
// s0 (the first entry of frontier[0]) is its own predecessor; no deadlock
// recorded yet.
lhs_status begin_parents(lhs_table *t, hipStream_t s);
lhs_status explore_async(lhs_table *t, const reach_model *m, const uint2 *d_trans, hipStream_t s,
                         reach_result *r, const uint32_t *d_init, AsyncCtl *d_ctl, AsyncCtl *h_ctl,
                         bool parents);

}  // namespace lhs
