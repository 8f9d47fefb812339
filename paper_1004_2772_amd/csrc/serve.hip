// Reachability server with continuous batching (reach_server_*).
//
// A worker thread owns the GPU side, in one of two modes.
//
// Persistent (the default).  One launch of resident workgroups serves every
// query on the GPU: a query is admitted, expanded level by level and retired
// inside the launch, and the host only readies slots, posts admissions and
// reads completion records (the protocol is described above k_serve below).
//
// Rounds (REACH_SERVER_F_ROUNDS).  The worker works in rounds of kRoundSteps
// BFS level steps; between rounds it
//   * admits queued queries, first come first served, while their tables fit
//     the device-memory budget (tables come from a resident pool keyed by
//     capacity and width; pooled tables of other shapes are freed when room
//     is needed), inserts their initial states, and
//   * retires the queries whose exploration ended, returning their tables to
//     the pool.
// A step is one launch: its workgroups expand the current level of every
// active query (tiles mapped to queries by a prefix), and the workgroup that
// finishes last does every query's level bookkeeping (level count, cap test,
// frontier swap, the next step's tile prefix), so a round runs without the
// host and a step costs one kernel boundary.  A capped level is not undone:
// the query ends there and its table is emptied when it is next handed out.
//
// In both modes a query that arrives while others are on the GPU joins them
// and its work overlaps theirs; its result is exactly the one reach_explore
// computes for it alone (same expansion, its own table).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_kernels.h"
#include "expand_device.h"
#include "internal.h"
#include "persistent.h"
#include "reach_internal.h"

using namespace lhs;

namespace {

constexpr uint64_t kDefaultBudget = 200ull << 30;
constexpr uint32_t kDefaultMaxActive = 1024;   // also the most a round can hold
constexpr uint32_t kRoundSteps = 4;

// Device-side bookkeeping of one active query during a round.
struct StepCtl {
    uint32_t *fr[2];
    unsigned long long cap, total, edges, deadlocks, wait_hits;
    unsigned long long lv[kRoundSteps];   // level counts found in this round
    uint32_t lv_n, cur, done, capped, error;
    uint32_t rollback_n;   // capped: entries of the discarded level in fr[cur ^ 1]
};

// Every query's level bookkeeping after a step, then the next step's tile
// prefix; run by the one workgroup that finished the step last (all other
// workgroups' counter updates are complete by then).  `scan` is LDS for
// kDefaultMaxActive words.
static_assert(expand_lds_words(1, 0, 1) >= kDefaultMaxActive, "the scan reuses the expansion's LDS");

__device__ void step_finalize(BatchSlot *slots, StepCtl *ctl, LevelCounters *lc, DevStatus *st,
                              uint32_t *begin, uint32_t n, uint32_t *scan) {
    constexpr uint32_t kPer = kDefaultMaxActive / kExpandBlock;   // queries per thread in the scan
    __shared__ uint32_t s_wtot[kExpandBlock / 64];
    const uint32_t tid = threadIdx.x;
    for (uint32_t a = tid; a < kDefaultMaxActive; a += kExpandBlock) {
        uint32_t tiles = 0;
        if (a < n) {
            StepCtl &C = ctl[a];
            BatchSlot &S = slots[a];
            if (!C.done) {
                // updated by other workgroups' atomics: read at the coherence point
                const uint32_t n_next = ld_coherent(&lc[a].n_next);
                const uint32_t err = ld_coherent(&st[a].error);
                C.wait_hits += ld_coherent(&st[a].wait_hits);
                if (err) {
                    C.error = err;
                    C.done = 1;
                } else if (C.cap && n_next > S.limit) {
                    C.capped = 1;
                    C.done = 1;
                    C.rollback_n = n_next;
                } else {
                    C.edges += ld_coherent(&lc[a].edges);
                    C.deadlocks += ld_coherent(&lc[a].deadlocks);
                    if (n_next == 0) {
                        C.done = 1;
                    } else {
                        C.lv[C.lv_n++] = n_next;
                        C.total += n_next;
                        C.cur ^= 1u;
                        S.front = C.fr[C.cur];
                        S.next = C.fr[C.cur ^ 1u];
                        S.n_front = n_next;
                        S.limit = C.cap ? (uint32_t)min<unsigned long long>(C.cap - C.total, 0xFFFFFFFFull)
                                        : 0xFFFFFFFFu;
                    }
                }
            }
            if (C.done)
                S.n_front = 0;
            lc[a] = LevelCounters{0, 0, 0, 0};
            st[a] = DevStatus{};
            tiles = (S.n_front + kExpandBlock - 1) / kExpandBlock;
        }
        scan[a] = tiles;
    }
    __syncthreads();
    // exclusive prefix of the tile counts: thread t owns kPer consecutive queries
    uint32_t local = 0;
    for (uint32_t k = 0; k < kPer; ++k)
        local += scan[tid * kPer + k];
    const uint32_t incl = wave_scan_incl(local);
    if (__lane_id() == 63)
        s_wtot[tid / 64] = incl;
    __syncthreads();
    uint32_t off = incl - local, total = 0;
    for (uint32_t w = 0; w < kExpandBlock / 64; ++w) {
        off += w < tid / 64 ? s_wtot[w] : 0u;
        total += s_wtot[w];
    }
    for (uint32_t k = 0; k < kPer; ++k) {
        const uint32_t a = tid * kPer + k, v = scan[a];
        if (a < n) {
            begin[a] = off;
            slots[a].tile_begin = off;
        }
        off += v;
    }
    if (tid == 0)
        begin[n] = total;
}

// One step: expand the current level of every active query (the tile
// prefix and its total come from device memory), then the last workgroup to
// finish does the level bookkeeping for the next step.  `arrived` counts the
// workgroups done with the step (zero at launch; reset by the last one).
template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock) void k_step(BatchSlot *slots, uint32_t *begin, uint32_t n,
                                                       uint32_t tcap, StepCtl *ctl, LevelCounters *lc,
                                                       DevStatus *st, uint32_t *arrived) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_last;
    expand_begin();
    const uint32_t tiles = begin[n];
    for (uint32_t g = blockIdx.x; g < tiles; g += gridDim.x) {
        const BatchSlot &s = slots[find_slot_by_tile(begin, n, g)];
        const uint64_t base = (uint64_t)(g - s.tile_begin) * kExpandBlock;
        const uint32_t rows = (uint32_t)min<uint64_t>(kExpandBlock, s.n_front - base);
        expand_tile<G, LS>(smem, s.t, s.m, s.front, base, rows, s.next, s.lc, s.limit, tcap);
    }
    // this workgroup's counter updates are complete before it checks in
    wait_vm_complete();
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = atomicAdd(arrived, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!s_last)
        return;
    step_finalize(slots, ctl, lc, st, begin, n, smem);
    if (threadIdx.x == 0)
        *arrived = 0;
}

// ---- persistent server ------------------------------------------------------
//
// One launch of resident workgroups serves every query: the batch's work
// queue (persistent.h) of (query slot, tile) items, whose last-tile
// finalisation advances a query's level, plus admission and completion.
//  * Admission.  The host readies a slot (the query's constants in ms[slot],
//    its s0 in roots[slot], its table emptied) with copies and a clearing
//    kernel on its upload stream, then appends the slot to box->admit_slot
//    and raises box->admit_tail, also by copies, in that order.  An idle
//    workgroup takes the admission, inserts s0 and queues level 0's tile
//    (it holds a queue position, so it keeps no tile for itself).
//  * Completion.  The workgroup that finishes a query posts (slot, error) to
//    a ring of records in pinned host memory (system scope, the sequence
//    word last, after the query's progress and level counts are complete).
//  * Work queue.  Each workgroup holds one queue position, taken with a
//    fetch-and-add, and polls its cell; between polls it takes admissions.
//  * Lifetime.  After a while without work, with no query admitted and
//    unfinished, a workgroup leaves and closes the launch to admissions
//    (box->closing); every other workgroup leaves once no query is left.
//    The host starts a new launch when work arrives and the last one has
//    ended (a query posted to a closing launch waits for the next); before
//    it, the positions the last launch held unfilled are given back.  A
//    query wider than the running launch's LDS rows closes it early (the
//    host sets box->closing) and waits for the next launch, with the
//    queries behind it.  The
//    launch leaves one workgroup's room per CU for the host's clearing
//    kernels.
// Slots, tables and transition buffers are reused while a launch runs, so
// everything the host writes is read past the caches (system scope), and
// slot lines are read with coherent loads (expand_tile's CL).
constexpr uint32_t kAdmitRing = 2048;      // admission entries (> 2 x max active)
constexpr uint32_t kDoneRing = 2048;       // completion records (> 2 x max active)
constexpr uint64_t kServeCells = 1ull << 23;   // work-queue cells (128 MiB)
constexpr uint32_t kServeMaxLevels = 1u << 16; // levels of one served query
constexpr uint32_t kIdleSleepMax = 8;      // back-off steps (~0.4 us each) of an idle workgroup
constexpr uint32_t kIdleLeave = 384;       // checks (~5 ms) finding no query on the GPU
                                           // before a workgroup leaves
constexpr uint32_t kStallPolls = 1u << 19; // idle polls (~2 s) without any level finished while
                                           // queries are unfinished: the launch has stalled

struct ServeBox {
    unsigned long long admit_tail;   // admissions posted (host copies)
    unsigned long long admit_head;   // admissions taken (workgroups)
    unsigned long long done_tail;    // completion records handed out
    uint32_t stop;                   // host copy: leave once idle
    uint32_t closing;                // set by the first workgroup to leave; the
                                     // host clears it before the next launch
    uint32_t beat;                   // levels finished (any launch)
    uint32_t pad;
    uint32_t admit_slot[kAdmitRing]; // slot of admission k, at k % kAdmitRing
};

struct DoneRec {
    unsigned long long seq;          // position + 1 once the record is complete
    uint32_t slot, error, n_levels, pad;
};

__device__ __forceinline__ unsigned long long ld_system(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint32_t ld_system(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// finalize_level's hook: post the finished query's completion record.
struct ServeDone {
    ServeBox *box;
    DoneRec *done;
    const ModelProgress *mp;
    __device__ void operator()(uint32_t slot, uint32_t err) const {
        const unsigned long long pos = atomicAdd(&box->done_tail, 1ull);
        DoneRec *r = done + (pos % kDoneRing);
        __hip_atomic_store(&r->slot, slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->error, err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->n_levels, ld_coherent(&mp[slot].n_levels), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_SYSTEM);
        __hip_atomic_store(&r->seq, pos + 1ull, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
    }
};

// The constants of slot i's query into LDS, read past every cache (the host
// rewrites them between queries); block-wide.
static_assert(sizeof(ModelState) % 8 == 0 && sizeof(ModelState) / 8 <= kExpandBlock, "model constants");
__device__ __forceinline__ void load_model_state(ModelState *dst, const ModelState *src) {
    constexpr uint32_t n = sizeof(ModelState) / 8;
    if (threadIdx.x < n)
        reinterpret_cast<unsigned long long *>(dst)[threadIdx.x] =
            ld_system(reinterpret_cast<const unsigned long long *>(src) + threadIdx.x);
    __syncthreads();
}

// Admit slot i's query (block-wide): progress and level 0, s0 inserted into
// its (emptied) table and listed as the first frontier.
template <uint32_t LS>
__device__ void admit_query(const ModelState &M, ModelProgress *mp, LevelState *lv, uint32_t i,
                            const uint32_t *roots) {
    __shared__ uint32_t row[32];
    const uint32_t tid = threadIdx.x;
    if (tid < M.m.W)
        row[tid] = ld_system(roots + 32u * i + tid);
    __syncthreads();
    if (tid < 64) {
        LaneCounters cnt;
        const LdsRowB v{row};
        const bool active = tid == 0;
        uint32_t slot = kNoSlot, code = kFull;
        const uint64_t h = hash_vec(v, M.m.W, M.t.seed);
        find_or_put<1, LS, LdsRowB, true>(M.t, v, h, active, slot, code, cnt);
        if (active) {
            ModelProgress &P = mp[i];
            LevelState &L = lv[i];
            LevelCounters *lc = M.lc;
            st_coherent(M.fr[0], slot);
            st_coherent(&P.total, 1ull);
            st_coherent(&P.edges, 0ull);
            st_coherent(&P.deadlocks, 0ull);
            st_coherent(&P.cur, 0u);
            st_coherent(&P.n_levels, 1u);
            st_coherent(&P.done, 0u);
            st_coherent(&P.capped, 0u);
            st_coherent(&P.overflow, 0u);
            st_coherent(&P.error, 0u);
            st_coherent(&P.handed, 0u);
            st_coherent(M.levels, 1ull);
            st_coherent(&lc->n_next, 0u);
            st_coherent(&lc->abort, 0u);
            st_coherent(&lc->edges, 0ull);
            st_coherent(&lc->deadlocks, 0ull);
            st_coherent(&L.front, (unsigned long long)M.fr[0]);
            st_coherent(&L.next, (unsigned long long)M.fr[1]);
            st_coherent(&L.n_front, 1u);
            st_coherent(&L.limit, M.cap ? (uint32_t)min<unsigned long long>(M.cap - 1, 0xFFFFFFFFull) : 0xFFFFFFFFu);
            st_coherent(&L.tiles_total, 1u);
            st_coherent(&L.tiles_done, 0u);
            st_coherent(&L.tile_rows, (uint32_t)kExpandBlock);
            st_coherent(&L.key, M.m.key);
        }
        wait_vm_complete();
    }
    __syncthreads();
}

template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock) void k_serve(const ModelState *ms, ModelProgress *mp, LevelState *lv,
                                                        QueueState *qs, QCell *ring, ServeBox *box, DoneRec *done,
                                                        const uint32_t *roots, uint32_t tcap) {
    extern __shared__ uint32_t smem[];
    __shared__ ModelState s_M;               // constants of slot s_M_slot's query
    __shared__ uint32_t s_act, s_slot, s_tile, s_fin, s_M_slot;
    enum : uint32_t { kNone = 0, kTile = 1, kAdmit = 2, kLeave = 3 };
    const uint32_t tid = threadIdx.x;
    expand_begin();
    if (tid == 0)
        s_M_slot = 0xFFFFFFFFu;
    bool kept = false;       // tile 0 of kept_slot's new level is this workgroup's
    uint32_t kept_slot = 0;
    // thread 0: the queue position this workgroup holds (taken with one
    // fetch-and-add, so workgroups never contend for an item), polls without
    // work, and idle polls without a beat
    bool holding = false;
    unsigned long long pos = 0;
    uint32_t idle = 0, quiet = 0, stall = 0, last_beat = 0;
    while (true) {
        __syncthreads();     // the last decision has been read by every thread
        if (tid == 0) {
            uint32_t act = kNone, slot = 0, tile = 0;
            if (queue_failed(qs)) {
                act = kLeave;
            } else if (kept) {
                act = kTile;
                slot = kept_slot;
            } else {
                if (!holding) {
                    pos = atomicAdd(&qs->head, 1ull);
                    holding = true;
                }
                QCell *c = ring + (pos & qs->mask);
                if (ld_coherent(&c->seq) == pos + 1ull) {
                    slot = ld_coherent(&c->model);
                    tile = ld_coherent(&c->tile);
                    wait_vm_complete();   // read before the cell is freed
                    st_coherent(&c->seq, pos + qs->mask + 1ull);
                    holding = false;
                    act = kTile;
                } else if (idle < 16 || (idle & 3u) == 0) {
                    // nothing at the held position yet: admissions, or leave
                    // once idle.  Leaving and admitting race, so each side
                    // announces itself before it looks at the other (both
                    // sequentially consistent): an admission counts itself in
                    // `remaining`, then checks `closing`; a workgroup about to
                    // leave sets `closing`, then checks `remaining`.  At
                    // least one sees the other, so no query is admitted to a
                    // launch whose workgroups have begun to leave.
                    const bool closing = ld_coherent(&box->closing) != 0u;
                    const unsigned long long ah = ld_coherent(&box->admit_head);
                    // acquire: the host's copies of the slot's constants,
                    // s0 and admission entry precede the tail it raised
                    if (!closing && ah < __hip_atomic_load(&box->admit_tail, __ATOMIC_ACQUIRE,
                                                           __HIP_MEMORY_SCOPE_SYSTEM)) {
                        __hip_atomic_fetch_add(&qs->remaining, 1u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
                        if (__hip_atomic_load(&box->closing, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT) == 0u &&
                            atomicCAS(&box->admit_head, ah, ah + 1ull) == ah) {
                            slot = ld_system(&box->admit_slot[ah % kAdmitRing]);
                            act = kAdmit;
                        } else {
                            atomicSub(&qs->remaining, 1u);
                        }
                    } else if (ld_coherent(&qs->remaining) != 0u) {
                        quiet = 0;
                    } else if (++quiet >= kIdleLeave || closing || ld_system(&box->stop) != 0u) {
                        // a read-modify-write even when closing is already
                        // seen set (the host may have set it): it takes part
                        // in the order the admissions see
                        __hip_atomic_exchange(&box->closing, 1u, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT);
                        // the held position is never filled: no query is
                        // left, and none can be admitted any more
                        if (__hip_atomic_load(&qs->remaining, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_AGENT) == 0u)
                            act = kLeave;
                    }
                }
                if (act == kNone) {
                    // bounded: with queries unfinished, some level
                    // finishes every few milliseconds at most
                    const uint32_t b = ld_coherent(&box->beat);
                    stall = b == last_beat ? stall + 1u : 0u;
                    last_beat = b;
                    if (stall > kStallPolls) {
                        atomicCAS(&qs->error, 0u, (uint32_t)LHS_ESTALL);
                        act = kLeave;
                    }
                    ++idle;
                    for (uint32_t k = 0; k < min(idle, kIdleSleepMax); ++k)
                        __builtin_amdgcn_s_sleep(16);
                }
            }
            if (act == kTile || act == kAdmit) {
                idle = 0;
                stall = 0;
            }
            s_act = act;
            s_slot = slot;
            s_tile = tile;
        }
        __syncthreads();
        const uint32_t act = s_act, i = s_slot, j = s_tile;
        if (act == kLeave)
            break;
        if (act == kNone)
            continue;
        if (act == kAdmit) {
            load_model_state(&s_M, ms + i);
            if (tid == 0)
                s_M_slot = i;
            admit_query<LS>(s_M, mp, lv, i, roots);
            // Tile 0 of the new query goes to the work queue like any other
            // tile.  This workgroup still holds the queue position it
            // reserved before admitting: were it to keep tiles for itself
            // now, the item that lands in that position would wait for its
            // whole chain of levels, and once the ring wrapped onto that
            // cell every producer would wait for it too (LHS_ESTALL).
            if (tid == 0)
                enqueue_item(qs, ring, i, 0u);
            continue;
        }
        kept = false;
        LevelState &L = lv[i];
        // the constants are read again only when the slot holds another query
        if (s_M_slot != i || s_M.m.key != ld_coherent(&L.key)) {
            __syncthreads();   // every thread has compared before s_M changes
            load_model_state(&s_M, ms + i);
            if (tid == 0)
                s_M_slot = i;
        }
        const uint32_t *front = reinterpret_cast<const uint32_t *>(ld_coherent(&L.front));
        uint32_t *next = reinterpret_cast<uint32_t *>(ld_coherent(&L.next));
        const uint32_t n_front = ld_coherent(&L.n_front);
        const uint32_t limit = ld_coherent(&L.limit);
        const uint32_t rows_per = ld_coherent(&L.tile_rows);
        const uint64_t base = (uint64_t)j * rows_per;
        const uint32_t rows = (uint32_t)min<uint64_t>(rows_per, n_front - base);
        expand_tile<G, LS, true, false, false, false, true>(smem, s_M.t, s_M.m, front, base, rows, next, s_M.lc,
                                                            limit, tcap);
        wait_vm_complete();
        __syncthreads();
        if (tid == 0) {
            const uint32_t total = ld_coherent(&L.tiles_total);
            wait_vm_complete();
            s_fin = atomicAdd(&L.tiles_done, 1u) + 1u == total;
            // progress for the idle workgroups' stall bound: one per level
            // (a level, even a query's deepest chain of one-tile levels,
            // ends well within the bound), not one per tile on a shared
            // address
            if (s_fin)
                atomicAdd(&box->beat, 1u);
        }
        __syncthreads();
        if (s_fin && finalize_level<true>(s_M, mp, lv, i, qs, ring, ServeDone{box, done, mp})) {
            kept = true;
            kept_slot = i;
        }
    }
}

// Before a launch: positions taken by the workgroups of the last launch and
// never filled are given back (every filled one was consumed: no query was
// left), and admissions reopen.
__global__ void k_serve_reopen(QueueState *qs, ServeBox *box) {
    qs->head = qs->tail;
    box->closing = 0;
}

// Work queue empty, every cell free, admission and completion counters at
// the host's positions.
__global__ void k_serve_init(QCell *ring, unsigned long long cells, QueueState *qs, ServeBox *box,
                             unsigned long long posted, unsigned long long done_head) {
    for (unsigned long long p = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; p < cells;
         p += (unsigned long long)gridDim.x * blockDim.x) {
        ring[p].seq = p;
        ring[p].model = 0;
        ring[p].tile = 0;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        qs->head = 0;
        qs->tail = 0;
        qs->remaining = 0;
        qs->error = 0;
        qs->mask = cells - 1;
        box->admit_tail = posted;
        box->admit_head = posted;
        box->done_tail = done_head;
        box->stop = 0;
        box->closing = 0;
        box->beat = 0;
        box->pad = 0;
    }
}

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

__global__ void k_zero_step(LevelCounters *lc, DevStatus *st, uint32_t n, uint32_t *arrived) {
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *arrived = 0;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        lc[i] = LevelCounters{0, 0, 0, 0};
        st[i] = DevStatus{};
    }
}

struct Query {
    uint64_t ticket = 0;
    std::vector<reach_trans> trans;
    std::vector<uint32_t> init;
    reach_model m{};
    uint32_t W = 0;
    uint64_t capacity = 0, bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    lhs_table *t = nullptr;
    lhs_table *caller = nullptr;   // the caller's table (reach_server_submit_ex)
    uint2 *d_trans = nullptr;
    uint32_t n_cur = 1, cur = 0, limit = 0;
    std::vector<uint64_t> levels;
    uint64_t total = 1, edges = 0, dead = 0, wait_hits = 0;
    int capped = 0;
    lhs_status status = LHS_OK;
    bool done = false;
    uint32_t slot = 0xFFFFFFFFu;   // persistent server: its slot while on the GPU
    uint64_t tiles_bound = 0;      // bound on its items in the work queue
};

// A query's items in the work queue at once: one level's tiles, full or cut
// small (persistent.h's level_tile_rows), plus one.
uint64_t queue_bound(const Query *q) {
    return std::max<uint64_t>(q->capacity / kExpandBlock, kSmallLevel / kMinTileRows) + 1;
}

// Worker-owned state of the persistent server.
struct Persist {
    hipStream_t up = nullptr;          // uploads, clearing kernels and read-backs
    hipEvent_t ev_end = nullptr;       // recorded after each launch
    bool running = false;
    uint32_t launch_W = 0;             // widest vector the running launch's LDS holds
    uint64_t launches = 0;
    ModelState *d_ms = nullptr;
    ModelProgress *d_mp = nullptr;
    LevelState *d_lv = nullptr;
    LevelCounters *d_lc = nullptr;
    QueueState *d_qs = nullptr;
    QCell *d_ring = nullptr;
    ServeBox *d_box = nullptr;
    uint32_t *d_roots = nullptr;                  // [slot][32]
    std::vector<unsigned long long *> d_levels;   // [slot] -> level counts, on first use
    DoneRec *h_done = nullptr;                    // pinned; written by the device
    DoneRec *h_done_dev = nullptr;                // ... its device address
    ModelProgress *h_prog = nullptr;              // pinned read-backs
    unsigned long long *h_lv = nullptr;
    DevStatus *h_tst = nullptr;
    QueueState *h_qs = nullptr;
    uint32_t *h_word = nullptr;                   // pinned {0, 1}: box flag values
    bool stop_sent = false;
    bool close_sent = false;                      // the running launch was asked to drain
    std::vector<Query *> slot_q;                  // query in each slot
    std::vector<uint32_t> free_slots;
    uint32_t live = 0;                            // posted and not yet completed
    uint64_t posted = 0, done_head = 0, outstanding = 0;
};

uint64_t table_bytes(uint64_t capacity, uint32_t W) {
    // slots + rows + two frontiers (+ counters)
    return capacity * (8ull + 4ull * W + 8ull) + 4096;
}

}  // namespace

struct reach_server {
    reach_server_opts opts{};
    lhs_config cfg{};           // shape of every query table (one launch serves all)
    int device = 0;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Query *> queue;
    std::unordered_map<uint64_t, Query *> tickets;
    // worker-owned
    std::vector<Query *> active;
    std::multimap<std::pair<uint64_t, uint32_t>, lhs_table *> pool;
    uint64_t bytes_alloc = 0;   // tables allocated (in use + pooled)
    // step buffers
    uint32_t cap_slots = 0;
    BatchSlot *d_slots = nullptr, *h_slots = nullptr;
    uint32_t *d_begin = nullptr, *h_begin = nullptr;
    LevelCounters *d_lc = nullptr, *h_lc = nullptr;
    DevStatus *d_st = nullptr, *h_st = nullptr;
    StepCtl *d_ctl = nullptr, *h_ctl = nullptr;
    uint32_t *d_roots = nullptr, *d_root_off = nullptr;
    uint32_t cap_roots = 0;
    // admission: pinned staging of packed models, roots and root slots, and
    // a pool of device transition buffers by power-of-two size class
    void *h_stage = nullptr;
    size_t cap_stage = 0;
    std::multimap<size_t, uint2 *> trans_pool;
    // persistent server (the default; REACH_SERVER_F_ROUNDS: host rounds)
    bool persistent = false;
    Persist ps;
    // stats (under mu)
    reach_server_stats stats{};
    double busy_s = 0;
    lhs_status fatal = LHS_OK;
};

namespace {

void free_step_buffers(reach_server *s) {
    (void)hipFree(s->d_slots);
    (void)hipFree(s->d_begin);
    (void)hipFree(s->d_lc);
    (void)hipFree(s->d_st);
    if (s->h_slots)
        (void)hipHostFree(s->h_slots);
    if (s->h_begin)
        (void)hipHostFree(s->h_begin);
    if (s->h_lc)
        (void)hipHostFree(s->h_lc);
    if (s->h_st)
        (void)hipHostFree(s->h_st);
    (void)hipFree(s->d_ctl);
    if (s->h_ctl)
        (void)hipHostFree(s->h_ctl);
    s->d_ctl = s->h_ctl = nullptr;
    s->d_slots = s->h_slots = nullptr;
    s->d_begin = s->h_begin = nullptr;
    s->d_lc = s->h_lc = nullptr;
    s->d_st = s->h_st = nullptr;
    s->cap_slots = 0;
}

lhs_status ensure_step_buffers(reach_server *s, uint32_t n) {
    if (n <= s->cap_slots)
        return LHS_OK;
    free_step_buffers(s);
    uint32_t c = 64;
    while (c < n)
        c <<= 1;
    if (hipMalloc(&s->d_slots, c * sizeof(BatchSlot)) != hipSuccess ||
        hipHostMalloc(&s->h_slots, c * sizeof(BatchSlot), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->d_begin, (c + 2) * sizeof(uint32_t)) != hipSuccess ||   // + step arrival count
        hipHostMalloc(&s->h_begin, (c + 1) * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->d_lc, c * sizeof(LevelCounters)) != hipSuccess ||
        hipHostMalloc(&s->h_lc, c * sizeof(LevelCounters), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->d_st, c * sizeof(DevStatus)) != hipSuccess ||
        hipHostMalloc(&s->h_st, c * sizeof(DevStatus), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->d_ctl, c * sizeof(StepCtl)) != hipSuccess ||
        hipHostMalloc(&s->h_ctl, c * sizeof(StepCtl), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        free_step_buffers(s);
        return LHS_ENOMEM;
    }
    s->cap_slots = c;
    return LHS_OK;
}

// Reserve a table for q (worker thread).  Returns false if it does not fit
// now.  Pooled tables of q's shape are reused; otherwise pooled tables are
// freed until a new one fits the budget.
bool acquire_table(reach_server *s, Query *q) {
    if (q->caller) {
        q->t = q->caller;
        return true;
    }
    auto key = std::make_pair(q->capacity, q->W);
    auto it = s->pool.find(key);
    if (it != s->pool.end()) {
        q->t = it->second;
        s->pool.erase(it);
        return true;
    }
    while (s->bytes_alloc + q->bytes > s->opts.budget_bytes && !s->pool.empty()) {
        auto victim = s->pool.begin();
        s->bytes_alloc -= table_bytes(victim->second->capacity, victim->second->W);
        lhs_destroy(victim->second);
        s->pool.erase(victim);
    }
    if (s->bytes_alloc + q->bytes > s->opts.budget_bytes)
        return false;
    lhs_table *t = nullptr;
    if (lhs_create_ex(q->capacity, q->W, &s->cfg, &t) != LHS_OK || ensure_bfs_buffers(t) != LHS_OK) {
        lhs_destroy(t);
        return false;
    }
    s->bytes_alloc += q->bytes;
    q->t = t;
    return true;
}

size_t trans_class(size_t bytes) {
    size_t c = 256;
    while (c < bytes)
        c <<= 1;
    return c;
}

void release_table(reach_server *s, Query *q) {
    if (q->t && !q->caller)
        s->pool.emplace(std::make_pair(q->t->capacity, q->t->W), q->t);
    q->t = nullptr;
    if (q->d_trans) {
        const size_t bytes = (size_t)q->m.n_procs * q->m.n_locals * q->m.trans_per_local * sizeof(uint2);
        s->trans_pool.emplace(trans_class(bytes), q->d_trans);
    }
    q->d_trans = nullptr;
}

// Set up newly admitted queries: clear tables, upload models, insert roots.
lhs_status start_queries(reach_server *s, const std::vector<Query *> &qs) {
    if (qs.empty())
        return LHS_OK;
    const uint32_t n = (uint32_t)qs.size();
    // pinned staging: [slots | root offsets | roots | packed models]
    Carve c;
    const size_t o_slots = c.take<BatchSlot>(n), o_off = c.take<uint32_t>(n);
    size_t n_roots = 0, n_trans = 0;
    for (Query *q : qs) {
        n_roots += q->W;
        n_trans += (size_t)q->m.n_procs * q->m.n_locals * q->m.trans_per_local;
    }
    const size_t o_roots = c.take<uint32_t>(n_roots), o_trans = c.take<uint2>(n_trans);
    if (c.off > s->cap_stage) {
        if (s->h_stage)
            (void)hipHostFree(s->h_stage);
        s->h_stage = nullptr;
        s->cap_stage = 0;
        size_t cap = 1 << 20;
        while (cap < c.off)
            cap <<= 1;
        if (hipHostMalloc(&s->h_stage, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s->h_stage = nullptr;
            return LHS_ENOMEM;
        }
        s->cap_stage = cap;
    }
    if (n_roots > s->cap_roots || n > s->cap_roots) {
        (void)hipFree(s->d_roots);
        (void)hipFree(s->d_root_off);
        s->cap_roots = 0;
        const uint32_t cap = (uint32_t)std::max<size_t>(1024, std::max<size_t>(n_roots, n) * 2);
        if (hipMalloc(&s->d_roots, cap * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&s->d_root_off, cap * sizeof(uint32_t)) != hipSuccess)
            return LHS_ENOMEM;
        s->cap_roots = cap;
    }
    // room for the whole next round now: growing the step buffers later
    // would free them under this admission's queued work
    lhs_status rc = ensure_step_buffers(s, (uint32_t)s->active.size() + n);
    if (rc != LHS_OK)
        return rc;
    BatchSlot *slots = at<BatchSlot>(s->h_stage, o_slots);
    uint32_t *off = at<uint32_t>(s->h_stage, o_off), *roots = at<uint32_t>(s->h_stage, o_roots);
    uint2 *trans = at<uint2>(s->h_stage, o_trans);
    size_t r_at = 0, t_at = 0;
    std::vector<uint2> packed;
    for (uint32_t i = 0; i < n; ++i) {
        Query *q = qs[i];
        pack_model(&q->m, packed);
        const size_t bytes = packed.size() * sizeof(uint2);
        auto it = s->trans_pool.find(trans_class(bytes));
        if (it != s->trans_pool.end()) {
            q->d_trans = it->second;
            s->trans_pool.erase(it);
        } else if (hipMalloc(&q->d_trans, trans_class(bytes)) != hipSuccess) {
            (void)hipGetLastError();
            q->d_trans = nullptr;
            return LHS_ENOMEM;
        }
        std::memcpy(trans + t_at, packed.data(), bytes);
        if (hipMemcpyAsync(q->d_trans, trans + t_at, bytes, hipMemcpyHostToDevice, s->stream) != hipSuccess)
            return LHS_EDEVICE;
        t_at += packed.size();
        q->t->last_stream = s->stream;
        if (lhs_clear(q->t, s->stream) != LHS_OK)
            return LHS_EDEVICE;
        BatchSlot &sl = slots[i];
        sl.t = view(q->t);
        sl.m = model_view(&q->m, q->d_trans);
        sl.front = q->t->frontier[0];
        sl.next = q->t->frontier[1];
        sl.lc = s->d_lc + i;
        sl.n_front = 1;
        sl.limit = q->limit;
        sl.tile_begin = 0;
        sl.pad = 0;
        off[i] = (uint32_t)r_at;
        std::memcpy(roots + r_at, q->init.data(), q->W * sizeof(uint32_t));
        r_at += q->W;
    }
    if (hipMemcpyAsync(s->d_roots, roots, n_roots * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess ||
        hipMemcpyAsync(s->d_root_off, off, n * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_slots, slots, n * sizeof(BatchSlot), hipMemcpyHostToDevice, s->stream) != hipSuccess)
        return LHS_EDEVICE;
    if (launch_insert_roots(s->cfg.line_slots, s->stream, s->d_slots, s->d_roots, s->d_root_off, n) != LHS_OK)
        return LHS_EDEVICE;
    // the staging buffer is rewritten only at the next admission, after the
    // next round's synchronisation: no wait here
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

// One round of kRoundSteps level steps over every active query, run on the
// device without the host; afterwards the queries whose exploration ended
// are returned in `finished`.
lhs_status step_queries(reach_server *s, std::vector<Query *> &finished) {
    const uint32_t na = (uint32_t)s->active.size();
    lhs_status rc = ensure_step_buffers(s, na);
    if (rc != LHS_OK)
        return rc;
    uint32_t tiles = 0, maxW = 1, tps = 0, tcap = 0;
    for (uint32_t a = 0; a < na; ++a) {
        Query *q = s->active[a];
        BatchSlot &sl = s->h_slots[a];
        sl.t = view(q->t);
        sl.t.status = s->d_st + a;
        sl.m = model_view(&q->m, q->d_trans);
        sl.front = q->t->frontier[q->cur];
        sl.next = q->t->frontier[q->cur ^ 1];
        sl.lc = s->d_lc + a;
        sl.n_front = q->n_cur;
        sl.limit = q->limit;
        sl.tile_begin = tiles;
        sl.pad = 0;
        StepCtl &c = s->h_ctl[a];
        std::memset(&c, 0, sizeof(c));
        c.fr[0] = q->t->frontier[0];
        c.fr[1] = q->t->frontier[1];
        c.cap = q->m.state_cap;
        c.total = q->total;
        c.edges = q->edges;
        c.deadlocks = q->dead;
        c.cur = q->cur;
        s->h_begin[a] = tiles;
        tiles += (q->n_cur + kExpandBlock - 1) / kExpandBlock;
        maxW = std::max(maxW, q->W);
        tcap = std::max(tcap, trans_lds_entries(q->m.n_procs, q->m.n_locals, q->m.trans_per_local));
    }
    tps = s->cfg.tps_expand ? s->cfg.tps_expand : kDefaultTpsExpand;
    s->h_begin[na] = tiles;
    if (hipMemcpyAsync(s->d_slots, s->h_slots, na * sizeof(BatchSlot), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess ||
        hipMemcpyAsync(s->d_ctl, s->h_ctl, na * sizeof(StepCtl), hipMemcpyHostToDevice, s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_begin, s->h_begin, (na + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess)
        return LHS_EDEVICE;
    uint32_t *d_arrived = s->d_begin + s->cap_slots + 1;
    hipLaunchKernelGGL(k_zero_step, dim3((na + 255) / 256), dim3(256), 0, s->stream, s->d_lc, s->d_st, na,
                       d_arrived);
    // workgroups for the expansion: enough for the round's first level four
    // times over (later levels loop), at most as many as are resident
    const size_t lds = (size_t)expand_lds_words(maxW, tcap, tps) * sizeof(uint32_t);
    rc = with_shape(tps, s->cfg.line_slots, [&](auto G, auto L) {
        const void *fn = (const void *)k_step<decltype(G)::value, decltype(L)::value>;
        int ncu = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
            per_cu < 1)
            return LHS_EDEVICE;
        const uint32_t grid = (uint32_t)std::min<uint64_t>((uint64_t)ncu * per_cu,
                                                           std::max<uint64_t>(64, 4ull * tiles));
        for (uint32_t k = 0; k < kRoundSteps; ++k)
            hipLaunchKernelGGL((k_step<decltype(G)::value, decltype(L)::value>), dim3(grid), dim3(kExpandBlock),
                               lds, s->stream, s->d_slots, s->d_begin, na, tcap, s->d_ctl, s->d_lc, s->d_st,
                               d_arrived);
        return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
    });
    if (rc != LHS_OK)
        return rc;
    if (hipMemcpyAsync(s->h_slots, s->d_slots, na * sizeof(BatchSlot), hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess ||
        hipMemcpyAsync(s->h_ctl, s->d_ctl, na * sizeof(StepCtl), hipMemcpyDeviceToHost, s->stream) != hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return LHS_EDEVICE;
    std::vector<Query *> keep;
    keep.reserve(na);
    bool rolled_back = false;
    for (uint32_t a = 0; a < na; ++a) {
        Query *q = s->active[a];
        const StepCtl &c = s->h_ctl[a];
        const BatchSlot &sl = s->h_slots[a];
        if (c.capped && q->caller && c.rollback_n) {
            // a caller's table keeps the result: undo the discarded level
            // (pooled tables are emptied when next handed out instead)
            hipLaunchKernelGGL(k_rollback_one, dim3(std::min<uint32_t>((c.rollback_n + 255) / 256, 4096)),
                               dim3(256), 0, s->stream, q->t->bucket, c.fr[c.cur ^ 1u], c.rollback_n);
            rolled_back = true;
        }
        q->wait_hits += c.wait_hits;
        q->levels.insert(q->levels.end(), c.lv, c.lv + c.lv_n);
        q->total = c.total;
        q->edges = c.edges;
        q->dead = c.deadlocks;
        q->cur = c.cur;
        q->n_cur = sl.n_front;
        q->limit = sl.limit;
        if (c.error)
            q->status = (lhs_status)c.error;
        q->capped = (int)c.capped;
        (c.done ? finished : keep).push_back(q);
    }
    s->active.swap(keep);
    if (rolled_back && (hipGetLastError() != hipSuccess || hipStreamSynchronize(s->stream) != hipSuccess))
        return LHS_EDEVICE;
    return LHS_OK;
}

// ---- persistent server: host side (worker thread) -------------------------
lhs_status persist_reset(reach_server *s) {
    Persist &P = s->ps;
    hipLaunchKernelGGL(k_serve_init, dim3(4096), dim3(256), 0, P.up, P.d_ring, (unsigned long long)kServeCells,
                       P.d_qs, P.d_box, (unsigned long long)P.posted, (unsigned long long)P.done_head);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(P.up) != hipSuccess)
        return LHS_EDEVICE;
    return LHS_OK;
}

lhs_status persist_init(reach_server *s) {
    Persist &P = s->ps;
    const uint32_t n = s->opts.max_active;
    if (hipStreamCreateWithFlags(&P.up, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&P.ev_end, hipEventDisableTiming) != hipSuccess)
        return LHS_EDEVICE;
    if (hipMalloc(&P.d_ms, n * sizeof(ModelState)) != hipSuccess ||
        hipMalloc(&P.d_mp, n * sizeof(ModelProgress)) != hipSuccess ||
        hipMalloc(&P.d_lv, n * sizeof(LevelState)) != hipSuccess ||
        hipMalloc(&P.d_lc, n * sizeof(LevelCounters)) != hipSuccess ||
        hipMalloc(&P.d_qs, sizeof(QueueState)) != hipSuccess ||
        hipMalloc(&P.d_ring, kServeCells * sizeof(QCell)) != hipSuccess ||
        hipMalloc(&P.d_box, sizeof(ServeBox)) != hipSuccess ||
        hipMalloc(&P.d_roots, (size_t)n * 32 * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc(&P.h_done, kDoneRing * sizeof(DoneRec), hipHostMallocCoherent) != hipSuccess ||
        hipHostMalloc(&P.h_prog, sizeof(ModelProgress), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&P.h_lv, kServeMaxLevels * sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&P.h_tst, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&P.h_qs, sizeof(QueueState), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(&P.h_word, 2 * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        return LHS_ENOMEM;
    }
    std::memset(P.h_done, 0, kDoneRing * sizeof(DoneRec));
    P.h_word[0] = 0;
    P.h_word[1] = 1;
    void *dev = nullptr;
    if (hipHostGetDevicePointer(&dev, P.h_done, 0) != hipSuccess)
        return LHS_EDEVICE;
    P.h_done_dev = static_cast<DoneRec *>(dev);
    P.slot_q.assign(n, nullptr);
    P.d_levels.assign(n, nullptr);
    for (uint32_t i = n; i-- > 0;)
        P.free_slots.push_back(i);
    return persist_reset(s);
}

void persist_free(reach_server *s) {
    Persist &P = s->ps;
    (void)hipFree(P.d_ms);
    (void)hipFree(P.d_mp);
    (void)hipFree(P.d_lv);
    (void)hipFree(P.d_lc);
    (void)hipFree(P.d_qs);
    (void)hipFree(P.d_ring);
    (void)hipFree(P.d_box);
    (void)hipFree(P.d_roots);
    for (auto p : P.d_levels)
        (void)hipFree(p);
    for (void *h : {(void *)P.h_done, (void *)P.h_prog, (void *)P.h_lv, (void *)P.h_tst, (void *)P.h_qs, (void *)P.h_word})
        if (h)
            (void)hipHostFree(h);
    if (P.ev_end)
        (void)hipEventDestroy(P.ev_end);
    if (P.up)
        (void)hipStreamDestroy(P.up);
}

// Ready the slots of newly admitted queries and post them to the running
// (or next) launch: transitions uploaded, tables emptied, each slot's
// constants and s0 written, then the admission entries, then the tail.
lhs_status persist_post(reach_server *s, const std::vector<Query *> &qs) {
    Persist &P = s->ps;
    if (qs.empty())
        return LHS_OK;
    const uint32_t n = (uint32_t)qs.size();
    Carve c;
    const size_t o_ms = c.take<ModelState>(n), o_roots = c.take<uint32_t>((size_t)n * 32),
                 o_adm = c.take<uint32_t>(n), o_tail = c.take<unsigned long long>(1);
    size_t n_trans = 0;
    for (Query *q : qs)
        n_trans += (size_t)q->m.n_procs * q->m.n_locals * q->m.trans_per_local;
    const size_t o_trans = c.take<uint2>(n_trans);
    if (c.off > s->cap_stage) {
        if (s->h_stage)
            (void)hipHostFree(s->h_stage);
        s->h_stage = nullptr;
        s->cap_stage = 0;
        size_t cap = 1 << 20;
        while (cap < c.off)
            cap <<= 1;
        if (hipHostMalloc(&s->h_stage, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            s->h_stage = nullptr;
            return LHS_ENOMEM;
        }
        s->cap_stage = cap;
    }
    ModelState *ms = at<ModelState>(s->h_stage, o_ms);
    uint32_t *roots = at<uint32_t>(s->h_stage, o_roots), *adm = at<uint32_t>(s->h_stage, o_adm);
    uint2 *trans = at<uint2>(s->h_stage, o_trans);
    std::memset(roots, 0, (size_t)n * 32 * sizeof(uint32_t));
    size_t t_at = 0;
    std::vector<uint2> packed;
    for (uint32_t k = 0; k < n; ++k) {
        Query *q = qs[k];
        const uint32_t slot = P.free_slots.back();
        P.free_slots.pop_back();
        P.slot_q[slot] = q;
        q->slot = slot;
        ++P.live;
        P.outstanding += q->tiles_bound;
        if (!P.d_levels[slot] &&
            hipMalloc(&P.d_levels[slot], kServeMaxLevels * sizeof(unsigned long long)) != hipSuccess) {
            (void)hipGetLastError();
            P.d_levels[slot] = nullptr;
            return LHS_ENOMEM;
        }
        pack_model(&q->m, packed);
        const size_t bytes = packed.size() * sizeof(uint2);
        auto it = s->trans_pool.find(trans_class(bytes));
        if (it != s->trans_pool.end()) {
            q->d_trans = it->second;
            s->trans_pool.erase(it);
        } else if (hipMalloc(&q->d_trans, trans_class(bytes)) != hipSuccess) {
            (void)hipGetLastError();
            q->d_trans = nullptr;
            return LHS_ENOMEM;
        }
        std::memcpy(trans + t_at, packed.data(), bytes);
        LHS_HIP(hipMemcpyAsync(q->d_trans, trans + t_at, bytes, hipMemcpyHostToDevice, P.up));
        t_at += packed.size();
        q->t->last_stream = P.up;
        if (lhs_clear(q->t, P.up) != LHS_OK)
            return LHS_EDEVICE;
        ModelState &M = ms[k];
        std::memset(&M, 0, sizeof(M));
        M.t = view(q->t);
        M.m = model_view(&q->m, q->d_trans);
        M.m.key = q->ticket;   // unique and nonzero: a later query may reuse this transition buffer
        M.lc = P.d_lc + slot;
        M.fr[0] = q->t->frontier[0];
        M.fr[1] = q->t->frontier[1];
        M.levels = P.d_levels[slot];
        M.cap = q->m.state_cap;
        M.max_levels = kServeMaxLevels;
        std::memcpy(roots + 32 * k, q->init.data(), q->W * sizeof(uint32_t));
        adm[k] = slot;
        LHS_HIP(hipMemcpyAsync(P.d_ms + slot, &M, sizeof(M), hipMemcpyHostToDevice, P.up));
        LHS_HIP(hipMemcpyAsync(P.d_roots + 32 * slot, roots + 32 * k, 32 * sizeof(uint32_t), hipMemcpyHostToDevice,
                               P.up));
        LHS_HIP(hipMemcpyAsync(&P.d_box->admit_slot[(P.posted + k) % kAdmitRing], adm + k, sizeof(uint32_t),
                               hipMemcpyHostToDevice, P.up));
    }
    // the tail last: a workgroup that sees it finds every entry below it
    P.posted += n;
    *at<unsigned long long>(s->h_stage, o_tail) = P.posted;
    LHS_HIP(hipMemcpyAsync(&P.d_box->admit_tail, at<unsigned long long>(s->h_stage, o_tail),
                           sizeof(unsigned long long), hipMemcpyHostToDevice, P.up));
    // the staging is reused by the next admission
    LHS_HIP(hipStreamSynchronize(P.up));
    return LHS_OK;
}

// Launch for the queries on the GPU: LDS for the widest of them, one
// workgroup's room per CU left for the host's clearing kernels.
lhs_status persist_launch(reach_server *s) {
    Persist &P = s->ps;
    uint32_t maxW = 1, tcap = 0;
    for (Query *q : P.slot_q)
        if (q) {
            maxW = std::max(maxW, q->W);
            tcap = std::max(tcap, trans_lds_entries(q->m.n_procs, q->m.n_locals, q->m.trans_per_local));
        }
    const uint32_t tps = s->cfg.tps_expand ? s->cfg.tps_expand : kDefaultTpsExpand;
    const size_t lds = (size_t)expand_lds_words(maxW, tcap, tps) * sizeof(uint32_t);
    const lhs_status rc = with_shape(tps, s->cfg.line_slots, [&](auto G, auto L) {
        const void *fn = (const void *)k_serve<decltype(G)::value, decltype(L)::value>;
        int ncu = 0, per_cu = 0;
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
            per_cu < 1)
            return LHS_EDEVICE;
        const uint32_t grid = (uint32_t)ncu * (uint32_t)std::max(1, per_cu - 1);
        hipLaunchKernelGGL(k_serve_reopen, dim3(1), dim3(1), 0, s->stream, P.d_qs, P.d_box);
        hipLaunchKernelGGL((k_serve<decltype(G)::value, decltype(L)::value>), dim3(grid), dim3(kExpandBlock), lds,
                           s->stream, (const ModelState *)P.d_ms, P.d_mp, P.d_lv, P.d_qs, P.d_ring, P.d_box,
                           P.h_done_dev, (const uint32_t *)P.d_roots, tcap);
        return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
    });
    if (rc != LHS_OK)
        return rc;
    LHS_HIP(hipEventRecord(P.ev_end, s->stream));
    P.running = true;
    P.close_sent = false;
    P.launch_W = maxW;
    ++P.launches;
    return LHS_OK;
}

// Collect the completion records the device has written.
lhs_status persist_collect(reach_server *s, std::vector<Query *> &finished) {
    Persist &P = s->ps;
    while (true) {
        DoneRec &r = P.h_done[P.done_head % kDoneRing];
        if (__atomic_load_n(&r.seq, __ATOMIC_ACQUIRE) != P.done_head + 1)
            break;
        const uint32_t slot = r.slot, err = r.error, nl = std::min(r.n_levels, kServeMaxLevels);
        ++P.done_head;
        if (slot >= P.slot_q.size() || !P.slot_q[slot])
            return LHS_EDEVICE;
        Query *q = P.slot_q[slot];
        LHS_HIP(hipMemcpyAsync(P.h_prog, P.d_mp + slot, sizeof(ModelProgress), hipMemcpyDeviceToHost, P.up));
        LHS_HIP(hipMemcpyAsync(P.h_lv, P.d_levels[slot], nl * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                               P.up));
        LHS_HIP(hipMemcpyAsync(P.h_tst, q->t->status, sizeof(DevStatus), hipMemcpyDeviceToHost, P.up));
        LHS_HIP(hipStreamSynchronize(P.up));
        const ModelProgress &M = *P.h_prog;
        q->levels.assign(P.h_lv, P.h_lv + nl);
        q->total = M.total;
        q->edges = M.edges;
        q->dead = M.deadlocks;
        q->capped = (int)M.capped;
        q->wait_hits = P.h_tst->wait_hits;
        q->status = err ? (lhs_status)err : (M.overflow ? LHS_EINVAL : LHS_OK);
        P.slot_q[slot] = nullptr;
        P.free_slots.push_back(slot);
        --P.live;
        P.outstanding -= q->tiles_bound;
        q->slot = 0xFFFFFFFFu;
        finished.push_back(q);
    }
    return LHS_OK;
}

// After a launch ended: a queue failure ends every query on the GPU and
// starts the device state afresh.
lhs_status persist_after_launch(reach_server *s, std::vector<Query *> &finished) {
    Persist &P = s->ps;
    P.running = false;
    lhs_status rc = persist_collect(s, finished);
    if (rc != LHS_OK)
        return rc;
    LHS_HIP(hipMemcpyAsync(P.h_qs, P.d_qs, sizeof(QueueState), hipMemcpyDeviceToHost, P.up));
    LHS_HIP(hipStreamSynchronize(P.up));
    if (!P.h_qs->error)
        return LHS_OK;
    const lhs_status err = (lhs_status)P.h_qs->error;
    for (uint32_t i = 0; i < P.slot_q.size(); ++i)
        if (Query *q = P.slot_q[i]) {
            q->status = err;
            P.slot_q[i] = nullptr;
            P.free_slots.push_back(i);
            finished.push_back(q);
        }
    P.live = 0;
    P.outstanding = 0;
    return persist_reset(s);
}

void persist_worker(reach_server *s) {
    (void)hipSetDevice(s->device);
    Persist &P = s->ps;
    double busy_since = 0;
    while (true) {
        std::vector<Query *> admitted, finished;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            while (s->queue.empty() && P.live == 0 && !P.running && !s->stop)
                s->cv_work.wait(lk);
            if (s->stop && s->queue.empty() && P.live == 0 && !P.running)
                return;
            // first come first served, while a slot, room in the work queue
            // and the budget allow; a query wider than the running launch's
            // LDS waits for the next launch (and holds the queries behind it)
            bool drain = false;
            while (!s->queue.empty() && admitted.size() < P.free_slots.size()) {
                Query *q = s->queue.front();
                if (P.running && q->W > P.launch_W) {
                    drain = true;
                    break;
                }
                q->tiles_bound = queue_bound(q);
                if (P.outstanding + q->tiles_bound > kServeCells / 2)
                    break;
                if (!acquire_table(s, q)) {
                    if (P.live == 0 && admitted.empty() && s->pool.empty()) {
                        s->queue.pop_front();
                        q->status = LHS_ENOMEM;
                        q->t_admit = q->t_done = now_s();
                        q->done = true;
                        s->stats.completed += 1;
                        s->cv_done.notify_all();
                        continue;
                    }
                    break;
                }
                s->queue.pop_front();
                q->t_admit = now_s();
                admitted.push_back(q);
            }
            s->stats.active = P.live + (uint32_t)admitted.size();
            s->stats.queued = (uint32_t)s->queue.size();
            s->stats.bytes_in_use = s->bytes_alloc;
            s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->bytes_alloc);
            if (P.live == 0 && !admitted.empty())
                busy_since = now_s();
            if (drain && !P.close_sent) {
                // the running launch admits no more queries and ends once
                // its queries are done; the next one has room for this one
                (void)hipMemcpyAsync(&P.d_box->closing, P.h_word + 1, sizeof(uint32_t), hipMemcpyHostToDevice,
                                     P.up);
                P.close_sent = true;
            }
        }
        bool progress = !admitted.empty();
        lhs_status rc = lhs::guard([&] { return persist_post(s, admitted); });
        if (rc != LHS_OK) {
            // the slots of the failed admissions are in an unknown state: end
            // every query on the GPU and start over
            for (Query *q : admitted)
                if (q->slot == 0xFFFFFFFFu) {
                    q->status = rc;
                    finished.push_back(q);
                }
        }
        if (rc == LHS_OK && !P.running && P.live > 0)
            rc = lhs::guard([&] { return persist_launch(s); });
        if (rc == LHS_OK) {
            const size_t before = finished.size();
            rc = lhs::guard([&] { return persist_collect(s, finished); });
            progress |= finished.size() > before;
        }
        if (rc == LHS_OK && P.running) {
            const hipError_t q = hipEventQuery(P.ev_end);
            if (q == hipSuccess)
                rc = lhs::guard([&] { return persist_after_launch(s, finished); });
            else if (q != hipErrorNotReady)
                rc = LHS_EDEVICE;
        }
        if (rc != LHS_OK) {
            // a device failure ends every query on the GPU
            if (P.running)
                (void)hipEventSynchronize(P.ev_end);
            P.running = false;
            for (uint32_t i = 0; i < P.slot_q.size(); ++i)
                if (Query *q = P.slot_q[i]) {
                    q->status = rc;
                    P.slot_q[i] = nullptr;
                    P.free_slots.push_back(i);
                    finished.push_back(q);
                }
            P.live = 0;
            P.outstanding = 0;
            (void)persist_reset(s);
        }
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (rc != LHS_OK)
                s->fatal = rc;
            for (Query *q : finished) {
                release_table(s, q);
                q->t_done = t1;
                q->done = true;
                s->stats.completed += 1;
                if (q->status == LHS_OK)
                    s->stats.states += q->total;
            }
            s->stats.steps = P.launches;
            if (!finished.empty() && P.live == 0) {
                s->busy_s += t1 - busy_since;
                busy_since = t1;
            }
            uint64_t pooled = 0;
            for (auto &e : s->pool)
                pooled += table_bytes(e.second->capacity, e.second->W);
            s->stats.bytes_pooled = pooled;
            if (!finished.empty())
                s->cv_done.notify_all();
            if (s->stop && s->queue.empty() && P.live == 0 && P.running && !P.stop_sent) {
                // let idle workgroups leave at once
                (void)hipMemcpyAsync(&P.d_box->stop, P.h_word + 1, sizeof(uint32_t), hipMemcpyHostToDevice, P.up);
                P.stop_sent = true;
            }
        }
        // completion records are polled while a launch runs
        if (!progress)
            std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
}

void worker_main(reach_server *s) {
    (void)hipSetDevice(s->device);
    while (true) {
        std::vector<Query *> admitted;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            while (true) {
                while (!s->queue.empty() && s->active.size() + admitted.size() < s->opts.max_active) {
                    Query *q = s->queue.front();
                    if (!acquire_table(s, q)) {
                        if (s->active.empty() && admitted.empty() && s->pool.empty()) {
                            // nothing will free memory: the allocation itself failed
                            s->queue.pop_front();
                            q->status = LHS_ENOMEM;
                            q->t_admit = q->t_done = now_s();
                            q->done = true;
                            s->stats.completed += 1;
                            s->cv_done.notify_all();
                            continue;
                        }
                        break;
                    }
                    s->queue.pop_front();
                    q->t_admit = now_s();
                    admitted.push_back(q);
                }
                if (!s->active.empty() || !admitted.empty())
                    break;
                if (s->stop && s->queue.empty())
                    return;
                s->cv_work.wait(lk);
            }
            s->stats.active = (uint32_t)(s->active.size() + admitted.size());
            s->stats.queued = (uint32_t)s->queue.size();
            s->stats.bytes_in_use = s->bytes_alloc;
            s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->bytes_alloc);
        }
        const double t0 = now_s();
        std::vector<Query *> finished;
        // an exception (a failed host allocation) ends the queries like a
        // device failure instead of the process
        lhs_status rc = lhs::guard([&] { return start_queries(s, admitted); });
        if (rc == LHS_OK) {
            s->active.insert(s->active.end(), admitted.begin(), admitted.end());
            rc = lhs::guard([&] { return step_queries(s, finished); });
        } else {
            for (Query *q : admitted) {
                q->status = rc;
                finished.push_back(q);
            }
        }
        if (rc != LHS_OK) {
            // a device failure ends every query on the GPU
            for (Query *q : s->active) {
                q->status = rc;
                finished.push_back(q);
            }
            s->active.clear();
        }
        const double t1 = now_s();
        std::lock_guard<std::mutex> lk(s->mu);
        s->busy_s += t1 - t0;
        s->stats.steps += 1;
        if (rc != LHS_OK)
            s->fatal = rc;
        for (Query *q : finished) {
            release_table(s, q);
            q->t_done = t1;
            q->done = true;
            s->stats.completed += 1;
            if (q->status == LHS_OK)
                s->stats.states += q->total;
        }
        uint64_t pooled = 0;
        for (auto &e : s->pool)
            pooled += table_bytes(e.second->capacity, e.second->W);
        s->stats.bytes_pooled = pooled;
        if (!finished.empty())
            s->cv_done.notify_all();
    }
}

lhs_status collect(reach_server *s, Query *q, reach_result *r, reach_query_times *t) {
    if (t) {
        t->submit_s = q->t_submit;
        t->admit_s = q->t_admit;
        t->done_s = q->t_done;
    }
    lhs_status rc = q->status;
    if (r) {
        std::memset(r, 0, sizeof(*r));
        if (rc == LHS_OK) {
            r->total_states = q->total;
            r->edges = q->edges;
            r->deadlocks = q->dead;
            r->capped = q->capped;
            r->wait_hits = q->wait_hits;
            r->n_levels = (uint32_t)q->levels.size();
            r->gpu_ms = (q->t_done - q->t_admit) * 1e3;
            r->level_counts = (uint64_t *)std::malloc(q->levels.size() * sizeof(uint64_t));
            if (!r->level_counts)
                rc = LHS_ENOMEM;
            else
                std::memcpy(r->level_counts, q->levels.data(), q->levels.size() * sizeof(uint64_t));
        }
    }
    if (q->caller) {
        // its work is complete (the round that ended the query was waited
        // for); hand it back on the null stream: the server's stream dies
        // with the server
        q->caller->last_stream = nullptr;
        q->caller->served_by = nullptr;
    }
    s->tickets.erase(q->ticket);
    delete q;
    // other threads waiting on this ticket see it gone
    s->cv_done.notify_all();
    return rc;
}

}  // namespace

extern "C" {

double reach_server_clock(void) { return now_s(); }

static lhs_status reach_server_create_impl(const reach_server_opts *o, reach_server **out) {
    if (!out)
        return LHS_EINVAL;
    *out = nullptr;
    reach_server *s = new (std::nothrow) reach_server();
    if (!s)
        return LHS_ENOMEM;
    if (o)
        s->opts = *o;
    if (!s->opts.budget_bytes)
        s->opts.budget_bytes = kDefaultBudget;
    if (!s->opts.max_active)
        s->opts.max_active = kDefaultMaxActive;
    if (s->opts.max_active > kDefaultMaxActive || (s->opts.flags & ~REACH_SERVER_F_ROUNDS)) {
        delete s;
        return LHS_EINVAL;
    }
    const lhs_config &c = s->opts.table;
    if (c.line_slots == 0 && c.probe == 0 && c.tps_find_or_put == 0 && c.tps_expand == 0) {
        s->cfg = tuned_config(LHS_TUNE_BATCH, 32, s->opts.capacity ? s->opts.capacity : (1ull << 21));
    } else {
        s->cfg = c;
        if (s->cfg.line_slots == 0)
            s->cfg.line_slots = 16;
    }
    if ((s->opts.capacity && (!is_pow2(s->opts.capacity) || s->opts.capacity < kLineSlots ||
                              s->opts.capacity > (1ull << 32))) ||
        !valid_line_slots(s->cfg.line_slots) || s->cfg.probe > LHS_PROBE_QUADRATIC ||
        !valid_tps(s->cfg.tps_find_or_put) || !valid_tps(s->cfg.tps_expand)) {
        delete s;
        return LHS_EINVAL;
    }
    if (hipGetDevice(&s->device) != hipSuccess || hipStreamCreate(&s->stream) != hipSuccess) {
        delete s;
        return LHS_EDEVICE;
    }
    s->persistent = !(s->opts.flags & REACH_SERVER_F_ROUNDS);
    lhs_status rc = s->persistent ? persist_init(s) : LHS_OK;
    if (rc == LHS_OK) {
        try {
            s->worker = std::thread(s->persistent ? persist_worker : worker_main, s);
        } catch (...) {
            rc = LHS_ENOMEM;
        }
    }
    if (rc != LHS_OK) {
        if (s->persistent)
            persist_free(s);
        (void)hipStreamDestroy(s->stream);
        delete s;
        return rc;
    }
    *out = s;
    return LHS_OK;
}

lhs_status reach_server_create(const reach_server_opts *o, reach_server **out) {
    return lhs::guard([&] { return reach_server_create_impl(o, out); });
}

static lhs_status reach_server_submit_impl(reach_server *s, const reach_model *m, lhs_table *table,
                                           uint64_t *ticket) {
    if (!s || !ticket || validate_model(m) != LHS_OK)
        return LHS_EINVAL;
    if (table) {
        // one launch serves every query: the table must have the server's
        // line width and live on the server's device, which is current
        int dev = -1;
        if (table->W != m->n_procs + m->n_shared || table->line_slots != s->cfg.line_slots ||
            table->device != s->device || hipGetDevice(&dev) != hipSuccess || dev != s->device ||
            (m->state_cap && m->state_cap >= table->capacity))
            return LHS_EINVAL;
    }
    // owned here until queued (freed on every early return or exception)
    std::unique_ptr<Query> q(new (std::nothrow) Query());
    if (!q)
        return LHS_ENOMEM;
    q->W = m->n_procs + m->n_shared;
    const uint64_t nt = (uint64_t)m->n_procs * m->n_locals * m->trans_per_local;
    q->trans.assign(m->trans, m->trans + nt);
    q->init.assign(m->init, m->init + q->W);
    q->m = *m;
    q->m.trans = q->trans.data();
    q->m.init = q->init.data();
    if (table) {
        // the caller's memory: not pooled and not counted against the budget
        q->caller = table;
        q->capacity = table->capacity;
        q->bytes = 0;
    } else {
        q->capacity = s->opts.capacity ? s->opts.capacity
                                       : (m->state_cap ? auto_capacity(m) : (1ull << 21));
        if (m->state_cap && m->state_cap >= q->capacity)
            return LHS_EINVAL;
        q->bytes = table_bytes(q->capacity, q->W);
        if (q->bytes > s->opts.budget_bytes)
            return LHS_EBUDGET;
    }
    q->limit = m->state_cap ? (uint32_t)std::min<uint64_t>(m->state_cap - 1, 0xFFFFFFFFull) : 0xFFFFFFFFu;
    // the persistent work queue holds a full level of every query on the GPU
    if (s->persistent && queue_bound(q.get()) > kServeCells / 2)
        return LHS_EINVAL;
    q->levels.push_back(1);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop)
        return LHS_EINVAL;
    if (table) {
        // a table serves one query at a time; its frontiers are allocated
        // here, on the caller's thread, before the worker sees the query
        const void *idle = nullptr;
        if (!table->served_by.compare_exchange_strong(idle, s))
            return LHS_EINVAL;
        if (ensure_bfs_buffers(table) != LHS_OK) {
            table->served_by = nullptr;
            return LHS_ENOMEM;
        }
    }
    q->ticket = s->next_ticket++;
    q->t_submit = now_s();
    s->tickets[q->ticket] = q.get();
    try {
        s->queue.push_back(q.get());
    } catch (...) {
        s->tickets.erase(q->ticket);
        if (table)
            table->served_by = nullptr;
        throw;
    }
    s->stats.submitted += 1;
    *ticket = q->ticket;
    q.release();
    s->cv_work.notify_one();
    return LHS_OK;
}

lhs_status reach_server_submit(reach_server *s, const reach_model *m, uint64_t *ticket) {
    return lhs::guard([&] { return reach_server_submit_impl(s, m, nullptr, ticket); });
}

lhs_status reach_server_submit_ex(reach_server *s, const reach_model *m, lhs_table *table, uint64_t *ticket) {
    return lhs::guard([&] { return reach_server_submit_impl(s, m, table, ticket); });
}

lhs_status reach_server_poll(reach_server *s, uint64_t ticket, reach_result *r, reach_query_times *t) {
    if (!s)
        return LHS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end())
        return LHS_ENOTFOUND;
    if (!it->second->done)
        return LHS_EAGAIN;
    return collect(s, it->second, r, t);
}

lhs_status reach_server_wait(reach_server *s, uint64_t ticket, reach_result *r, reach_query_times *t) {
    if (!s)
        return LHS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    // the ticket is looked up again on every wake-up: another thread waiting
    // on the same ticket may have collected (and freed) the query meanwhile
    auto it = s->tickets.find(ticket);
    s->cv_done.wait(lk, [&] {
        it = s->tickets.find(ticket);
        return it == s->tickets.end() || it->second->done;
    });
    if (it == s->tickets.end())
        return LHS_ENOTFOUND;
    return collect(s, it->second, r, t);
}

lhs_status reach_server_get_stats(reach_server *s, reach_server_stats *out) {
    if (!s || !out)
        return LHS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->busy_s = s->busy_s;
    out->queued = (uint32_t)s->queue.size();
    return LHS_OK;
}

lhs_status reach_server_destroy(reach_server *s) {
    if (!s)
        return LHS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable())
        s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto &e : s->pool)
        lhs_destroy(e.second);
    for (auto &e : s->tickets) {
        if (e.second->caller) {
            e.second->caller->last_stream = nullptr;
            e.second->caller->served_by = nullptr;
        }
        delete e.second;
    }
    if (s->persistent) {
        (void)hipStreamSynchronize(s->ps.up);
        persist_free(s);
    }
    free_step_buffers(s);
    (void)hipFree(s->d_roots);
    (void)hipFree(s->d_root_off);
    for (auto &e : s->trans_pool)
        (void)hipFree(e.second);
    if (s->h_stage)
        (void)hipHostFree(s->h_stage);
    (void)hipStreamDestroy(s->stream);
    const lhs_status rc = s->fatal;
    delete s;
    return rc;
}

}  // extern "C"
