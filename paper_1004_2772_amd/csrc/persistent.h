// The persistent work queue shared by the batch driver (csrc/batch.hip) and
// the persistent server (csrc/serve.hip): a bounded ring of (model, tile)
// items and the per-model level state that the workgroup finishing a level's
// last tile advances (finalize_level).
#pragma once

#include "expand_device.h"
#include "internal.h"
#include "reach_internal.h"

namespace lhs {

constexpr uint32_t kBarrierSpinLimit = 1u << 24;   // bound on every queue wait

// ---- persistent driver: a device work queue, no grid-wide barriers ---------
//
// Items are (model, tile of the model's current level).  Workgroups take
// items from a bounded multi-producer multi-consumer ring (cells carry a
// sequence number: cell of position p is ready when seq == p + 1, free for
// the producer of position p + R when seq == p + R).  The workgroup that
// finishes the last tile of a model's level finalises that level (cap
// rollback, level count, frontier swap, counter reset) and enqueues the
// tiles of the model's next level, so every model advances at its own pace.
// Everything one workgroup hands to another goes through agent-scope
// (coherent) accesses, completed (vmcnt(0)) before the item or counter that
// announces it.  Every wait is bounded; on timeout the error flag is set and
// all workgroups leave.
//
// The workgroups need not all be resident at once (the launch is a plain
// one, sized to what fits): a workgroup only ever waits for a cell that a
// running workgroup fills (a finaliser, or in the server the workgroup that
// admits a query, each of which waits only for free cells, and the ring
// holds one full level of every model), so one that starts late takes its
// first item, or finds the batch finished, and leaves.  A workgroup runs a
// tile that is not a queue item (a finaliser's tile 0 of the next level)
// only when it holds no queue position: an item filled into a position its
// holder is not polling would wait, and the ring could wrap onto it.

struct QCell {
    unsigned long long seq;
    uint32_t model;
    uint32_t tile;
};

struct QueueState {
    unsigned long long head;    // next position to take
    unsigned long long tail;    // next position to fill
    uint32_t remaining;         // unfinished models
    uint32_t error;
    unsigned long long mask;    // ring size - 1
};

// Per-model level state (changes every level; coherent accesses only).
struct LevelState {
    unsigned long long front;   // uint32_t* of the current frontier
    unsigned long long next;    // uint32_t* of the next frontier
    uint32_t n_front;
    uint32_t limit;
    uint32_t tiles_total;
    uint32_t tiles_done;
    uint32_t tile_rows;         // frontier states per tile of this level
    uint32_t pad;
    unsigned long long key;     // the model's ModelView key (persistent server)
};

// Per-model constants (written by the host before the launch, read-only in
// the kernel, so plain loads are fine).
struct ModelState {
    TableView t;
    ModelView m;
    LevelCounters *lc;
    uint32_t *fr[2];
    unsigned long long *levels;   // [max_levels] level counts (coherent stores)
    unsigned long long cap;
    uint32_t max_levels;
    uint32_t handover;            // stop after a level of more states (0 = never)
};

// Per-model progress: updated by whichever workgroup finalises a level, so
// only ever accessed with coherent loads and stores.
struct ModelProgress {
    unsigned long long total, edges, deadlocks;
    uint32_t cur, n_levels, done, capped, overflow, error;
    uint32_t handed, pad;   // handed: stopped after a level above M.handover
};

// Called by thread 0 of the finalising workgroup once model i is finished
// and its final progress is stored (completed): nothing for the batch.
struct NoDoneHook {
    __device__ void operator()(uint32_t, uint32_t) const {}
};

__device__ __forceinline__ bool queue_failed(QueueState *qs) {
    return ld_coherent(&qs->error) != 0u;
}

// Append one item (one thread): reserve a position on the tail, wait for
// its cell to be free (bounded, as the finaliser's enqueue), fill it, and
// publish it once the fill and everything the caller wrote before have
// completed.
__device__ inline void enqueue_item(QueueState *qs, QCell *ring, uint32_t model, uint32_t tile) {
    const unsigned long long pos = atomicAdd(&qs->tail, 1ull);
    QCell *c = ring + (pos & qs->mask);
    uint32_t spins = 0;
    while (ld_coherent(&c->seq) != pos) {
        if (++spins > kBarrierSpinLimit || queue_failed(qs)) {
            atomicCAS(&qs->error, 0u, (uint32_t)LHS_ESTALL);
            break;
        }
        __builtin_amdgcn_s_sleep(2);
    }
    st_coherent(&c->model, model);
    st_coherent(&c->tile, tile);
    wait_vm_complete();
    st_coherent(&c->seq, pos + 1ull);
}

// Tile size of a level.  Once at most kFewModels models remain and at least
// half the workgroups wait on the queue with nothing to take, a level of at
// most kSmallLevel states is cut into tiles of down to kMinTileRows states,
// about one per waiting workgroup: the deepest models' narrow levels, run
// after the rest of the batch has finished, then spread over the idle GPU
// instead of one full tile's latency chain per workgroup.  Otherwise tiles
// stay full (less per-tile work while the GPU is busy).
constexpr uint32_t kSmallLevel = 32768;
constexpr uint32_t kMinTileRows = 32;
constexpr uint32_t kFewModels = 8;
__device__ __forceinline__ uint32_t level_tile_rows(QueueState *qs, uint32_t n_states) {
    if (n_states > kSmallLevel || ld_coherent(&qs->remaining) > kFewModels)
        return kExpandBlock;
    const unsigned long long h = ld_coherent(&qs->head), t = ld_coherent(&qs->tail);
    const uint32_t idle = h > t ? (uint32_t)min<unsigned long long>(h - t, 1u << 16) : 0u;
    if (idle < gridDim.x / 2)
        return kExpandBlock;
    uint32_t rows = kMinTileRows;
    while (rows < kExpandBlock && (uint64_t)rows * (idle + 1) < n_states)
        rows <<= 1;
    return rows;
}

// A single-model exploration's first levels, run in one persistent launch
// until a level exceeds a threshold (explore_prefix): its work queue, model
// constants, progress, level state and level counts, in one region (device,
// and its pinned mirror).
constexpr uint32_t kPrefixHandover = 1u << 16;   // states of a level the prefix still expands
constexpr uint32_t kPrefixLevels = 4096;
constexpr uint32_t kPrefixGrid = 256;
constexpr uint32_t kPrefixCells = 8192;   // > tiles of a level of kPrefixHandover states + kPrefixGrid
static_assert(kPrefixCells >= 2 * (kPrefixHandover / kMinTileRows + 1 + kPrefixGrid), "prefix ring");
struct PrefixArea {
    QueueState qs;
    ModelState ms;
    ModelProgress mp;
    LevelState lv;
    unsigned long long levels[kPrefixLevels];
    QCell ring[kPrefixCells];
};

// Finalise model i's level (M = its constants); block-wide.  Called by the workgroup that
// completed its last tile.  Returns (uniformly) true when the model has a
// next level: its tile 0 is then left to the caller, which expands it at
// once instead of queueing it (a model's narrow levels do not wait behind
// the queue); tiles 1.. go to the queue.  CHECK_ERR: a model whose table
// reports a device error (EFULL, ESTALL) ends with it (P.error); on_done(i,
// error) runs when the model is finished.
template <bool CHECK_ERR = false, class OnDone = NoDoneHook>
__device__ bool finalize_level(const ModelState &M, ModelProgress *mp, LevelState *lv, uint32_t i,
                               QueueState *qs, QCell *ring, OnDone on_done = OnDone()) {
    __shared__ uint32_t s_nt;
    __shared__ unsigned long long s_pos0;
    const uint32_t tid = threadIdx.x;
    ModelProgress &P = mp[i];
    LevelState &L = lv[i];
    LevelCounters *lc = M.lc;
    const uint32_t n_next = ld_coherent(&lc->n_next);
    const uint32_t limit = ld_coherent(&L.limit);
    uint32_t *next = reinterpret_cast<uint32_t *>(ld_coherent(&L.next));
    const uint32_t err = CHECK_ERR ? ld_coherent(&M.t.status->error) : 0u;
    const bool over = !err && M.cap && n_next > limit;
    if (over) {
        // discard the partial level: zero every slot it claimed
        for (uint32_t j = tid; j < n_next; j += kExpandBlock)
            st_coherent(M.t.bucket + ld_coherent(next + j), 0ull);
    }
    wait_vm_complete();
    __syncthreads();
    if (tid == 0) {
        uint32_t nt = 0, done = 0;
        if (err) {
            st_coherent(&P.error, err);
            done = 1;
        } else if (over) {
            st_coherent(&P.capped, 1u);
            done = 1;
        } else {
            st_coherent(&P.edges, ld_coherent(&P.edges) + ld_coherent(&lc->edges));
            st_coherent(&P.deadlocks, ld_coherent(&P.deadlocks) + ld_coherent(&lc->deadlocks));
            const uint32_t nl = ld_coherent(&P.n_levels);
            if (n_next == 0) {
                done = 1;
            } else if (nl == M.max_levels) {
                st_coherent(&P.overflow, 1u);
                done = 1;
            } else {
                st_coherent(M.levels + nl, (unsigned long long)n_next);
                st_coherent(&P.n_levels, nl + 1u);
                const unsigned long long total = ld_coherent(&P.total) + n_next;
                st_coherent(&P.total, total);
                const uint32_t cur = ld_coherent(&P.cur) ^ 1u;
                st_coherent(&P.cur, cur);
                if (M.handover && (n_next > M.handover || nl + 1u == M.max_levels)) {
                    // a level too wide (or one level array full): the
                    // caller expands it and the rest
                    st_coherent(&P.handed, 1u);
                    done = 1;
                }
            }
            if (!done) {
                const uint32_t cur = ld_coherent(&P.cur);
                const unsigned long long total = ld_coherent(&P.total);
                const uint32_t rows_per = level_tile_rows(qs, n_next);
                nt = (n_next + rows_per - 1) / rows_per;
                const uint64_t room = M.cap ? M.cap - total : 0xFFFFFFFFull;
                st_coherent(&L.front, (unsigned long long)M.fr[cur]);
                st_coherent(&L.next, (unsigned long long)M.fr[cur ^ 1u]);
                st_coherent(&L.n_front, n_next);
                st_coherent(&L.limit, (uint32_t)min<uint64_t>(room, 0xFFFFFFFFull));
                st_coherent(&L.tiles_total, nt);
                st_coherent(&L.tiles_done, 0u);
                st_coherent(&L.tile_rows, rows_per);
            }
        }
        if (done)
            st_coherent(&P.done, 1u);
        st_coherent(&lc->n_next, 0u);
        st_coherent(&lc->abort, 0u);
        st_coherent(&lc->edges, 0ull);
        st_coherent(&lc->deadlocks, 0ull);
        wait_vm_complete();
        if (done) {
            atomicSub(&qs->remaining, 1u);
            on_done(i, err);
        } else if (nt > 1)
            s_pos0 = atomicAdd(&qs->tail, (unsigned long long)(nt - 1));
        s_nt = nt;
    }
    __syncthreads();
    const uint32_t nt = s_nt;
    // enqueue tiles 1.. of the next level: wait for each cell to be free,
    // fill it, then publish it
    for (uint32_t k = 1 + tid; k < nt; k += kExpandBlock) {
        const unsigned long long pos = s_pos0 + (k - 1);
        QCell *c = ring + (pos & qs->mask);
        uint32_t spins = 0;
        while (ld_coherent(&c->seq) != pos) {
            if (++spins > kBarrierSpinLimit || queue_failed(qs)) {
                atomicCAS(&qs->error, 0u, (uint32_t)LHS_ESTALL);
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        st_coherent(&c->model, i);
        st_coherent(&c->tile, k);
        wait_vm_complete();
        st_coherent(&c->seq, pos + 1ull);
    }
    return nt != 0;
}

}  // namespace lhs
