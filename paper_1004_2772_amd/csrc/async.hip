// Reachability without level barriers (REACH_F_ASYNC) for one model.
//
// Algorithm 1 only needs the set of visited states to be shared; the order
// in which open states are expanded is free.  The paper's workers therefore
// drop strict BFS order for local queues or stacks and balance load by
// handing work to idle workers (section "Preliminaries", paragraph on load
// balancing; the conclusions name pseudo-BFS and pseudo-DFS).  On the GPU the
// workers are the resident workgroups of one persistent launch and the
// shared work pool is a FIFO of slot indices in HBM:
//
//   queue[0, capacity)  u32 slot of every state, in discovery order (each
//                       state is appended exactly once, when inserted, so
//                       the array never wraps); 0xFFFFFFFF = not written yet
//   lc->n_next          append cursor (states stored so far)
//   ctl->chunk          next 256-entry chunk to hand out
//   ctl->work           states discovered and not yet expanded
//
// A workgroup owns one chunk at a time and expands the chunk's entries as
// they are appended (all 256 at once in the common case, fewer while the
// open set is narrow), then takes the next chunk with one atomic add, so
// idle workgroups pick up new work as soon as it exists instead of at a
// level boundary.  The expansion itself is the BFS tile (expand_tile):
// LDS-staged rows, guarded successors, find-or-put, compaction of the new
// states into an LDS buffer.  The buffer is appended to the queue with one
// atomic when it nears full, when some workgroup owns a chunk that nothing
// has been appended to (it is waiting), and whenever its own chunk has no
// entry left to expand: held-back states never starve an idle GPU, and while
// every workgroup is busy they go out in bulk.
//
// Termination: after every tile a workgroup adds (states it discovered,
// appended or buffered - states it expanded) to ctl->work in one atomic, and
// an append in the middle of a tile first adds the states of that tile it
// makes visible (another workgroup may expand them, and subtract them,
// before the tile ends).  So work only reaches 0 when no state is open
// anywhere (queued, buffered or in a tile in flight); then no state can be
// discovered again and every workgroup leaves.  The order of expansion
// varies from run to run, so per-level counts are not defined; the
// reachable set, edges and deadlocks are (they do not depend on the order).
#include <algorithm>
#include <cstring>

#include "internal.h"
#include "reach_internal.h"
#include "expand_device.h"

using namespace lhs;

namespace {

constexpr uint32_t kNoEntry = 0xFFFFFFFFu;
constexpr uint32_t kChunk = kExpandBlock;
// Bound on polls without progress (each sleeps about 0.4 us): an idle
// workgroup gives up with LHS_ESTALL after roughly a second in which no
// state was appended anywhere.
constexpr uint32_t kStallPolls = 1u << 21;

__global__ void k_fill_queue(uint4 *q, uint64_t n4) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4;
         i += (uint64_t)gridDim.x * blockDim.x)
        q[i] = make_uint4(kNoEntry, kNoEntry, kNoEntry, kNoEntry);
}

// s0 is queue entry 0 (written by its insert): one state stored, one open.
__global__ void k_async_init(AsyncCtl *ctl, LevelCounters *lc) {
    ctl->work = 1;
    ctl->chunk = 0;
    ctl->error = 0;
    lc->n_next = 1;
    lc->abort = 0;
    lc->edges = 0;
    lc->deadlocks = 0;
}

template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock) void k_explore_async(TableView t, ModelView m, uint32_t *queue,
                                                                LevelCounters *lc, AsyncCtl *ctl,
                                                                uint32_t limit, uint32_t tcap) {
    extern __shared__ uint32_t smem[];
    expand_begin();
    enum : uint32_t { kStop = 0, kExpand = 1, kPublish = 2 };
    __shared__ uint32_t s_from, s_take, s_act;
    const uint32_t tid = threadIdx.x;
    uint32_t *nbuf = expand_nbuf<G>(smem, m.W, tcap);
    // thread 0: the owned chunk is queue[base, base + kChunk), its first
    // `used` entries already taken.  s_found = new states this workgroup has
    // discovered (appended or still buffered) that ctl->work holds
    uint64_t base = 0;
    uint32_t used = kChunk, polls = 0, last_tail = 0;
    if (tid == 0) {
        s_open = &ctl->work;
        s_found = 0;
    }
    while (true) {
        if (tid == 0) {
            uint32_t take = 0, act = kStop;
            while (true) {
                if (used == kChunk) {
                    base = (uint64_t)atomicAdd(&ctl->chunk, 1u) * kChunk;
                    used = 0;
                }
                const uint32_t tl = ld_coherent(&lc->n_next);
                const uint64_t end = min<uint64_t>(tl, base + kChunk);
                // some workgroup owns a chunk that nothing has been appended
                // to yet, i.e. is waiting: publish held-back states before
                // expanding more (only asked while the cursor is within a
                // quarter of the grid's chunks of this one, as it then can be)
                if (s_nnew && (uint64_t)tl < base + (uint64_t)(gridDim.x / 4 + 1) * kChunk &&
                    (uint64_t)tl < (uint64_t)ld_coherent(&ctl->chunk) * kChunk) {
                    act = kPublish;
                    break;
                }
                if (end > base + used) {
                    take = (uint32_t)(end - base - used);
                    act = kExpand;
                    break;
                }
                // nothing appended to this chunk yet: publish the states this
                // workgroup holds back first (others may be waiting for them)
                if (s_nnew) {
                    act = kPublish;
                    break;
                }
                if (ld_coherent(&ctl->work) == 0 || ld_coherent(&lc->abort) ||
                    ld_coherent(&t.status->error) || ld_coherent(&ctl->error))
                    break;
                if (tl != last_tail) {
                    last_tail = tl;
                    polls = 0;
                } else if (++polls > kStallPolls) {
                    atomicCAS(&ctl->error, 0u, (uint32_t)LHS_ESTALL);
                    break;
                }
                __builtin_amdgcn_s_sleep(16);
            }
            // entries below the cursor are below the capacity (< 2^32)
            s_from = (uint32_t)(base + used);
            s_take = take;
            s_act = act;
            used += take;
        }
        __syncthreads();
        const uint32_t act = s_act, from = s_from, n = s_take;
        if (act == kStop)
            break;
        if (act == kPublish) {
            // states held since the last tile: already counted
            flush_new_slots<true, true>(nbuf, queue, lc, limit);
            continue;
        }
        // new states stay buffered across tiles while this chunk has work
        const bool aborted =
            expand_tile<G, LS, true, true, true, true>(smem, t, m, queue, from, n, queue, lc, limit, tcap);
        if (tid == 0) {
            // discovered - expanded, after the discoveries are counted
            const uint32_t now = s_pushed + s_nnew;
            atomicAdd(&ctl->work, (unsigned long long)(now - s_found) - (unsigned long long)n);
            s_found = now;
        }
        if (aborted)
            break;
    }
    // counts kept in LDS over the launch (and, after an abort, the buffer)
    expand_end<G, true>(smem, m.W, tcap, queue, lc, limit);
}

}  // namespace

namespace lhs {

lhs_status explore_async(lhs_table *t, const reach_model *m, const uint2 *d_trans, hipStream_t s,
                         reach_result *r, const uint32_t *d_init, AsyncCtl *d_ctl, AsyncCtl *h_ctl,
                         bool parents) {
    // queue entries are slots and 0xFFFFFFFF marks an unwritten entry
    if (t->capacity >= (1ull << 32))
        return LHS_EINVAL;
    const ModelView mv = model_view(m, d_trans);
    const TableView tv = bfs_view(t, parents);
    uint32_t *queue = t->frontier[0];
    const uint64_t n4 = t->capacity / 4;
    hipLaunchKernelGGL(k_fill_queue, dim3((uint32_t)std::min<uint64_t>((n4 + 255) / 256, 8192)), dim3(256), 0,
                       s, reinterpret_cast<uint4 *>(queue), n4);
    LHS_HIP(hipGetLastError());
    // s0: inserted with the batched find-or-put, its slot becomes entry 0
    lhs_status rc = launch_find_or_put(t, d_init, 1, reinterpret_cast<uint8_t *>(t->frontier[1]), queue, s);
    if (rc != LHS_OK)
        return rc;
    if (parents && (rc = begin_parents(t, s)) != LHS_OK)
        return rc;
    hipLaunchKernelGGL(k_async_init, dim3(1), dim3(1), 0, s, d_ctl, t->level);
    LHS_HIP(hipGetLastError());
    const uint32_t limit =
        m->state_cap ? (uint32_t)std::min<uint64_t>(m->state_cap, 0xFFFFFFFFull) : 0xFFFFFFFFu;
    const uint32_t tc = trans_lds_entries(mv.P, mv.L, mv.K);
    const size_t lds = expand_lds_bytes(mv.W, tc, tps_expand(t));
    rc = with_shape(tps_expand(t), t->line_slots, [&](auto G, auto L) {
        const void *fn = (const void *)k_explore_async<decltype(G)::value, decltype(L)::value>;
        int ncu = 0, per_cu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
            per_cu < 1)
            return LHS_EDEVICE;
        // the resident workgroups; waits are bounded, so the protocol needs
        // no co-residency guarantee
        hipLaunchKernelGGL((k_explore_async<decltype(G)::value, decltype(L)::value>),
                           dim3(exploration_grid(t, (uint64_t)ncu * per_cu)),
                           dim3(kExpandBlock), lds, s, tv, mv, queue, t->level, d_ctl, limit, tc);
        return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
    });
    if (rc != LHS_OK)
        return rc;
    LHS_HIP(hipMemcpyAsync(t->level_host, t->level, sizeof(LevelCounters), hipMemcpyDeviceToHost, s));
    LHS_HIP(hipMemcpyAsync(t->status_host, t->status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    LHS_HIP(hipMemcpyAsync(h_ctl, d_ctl, sizeof(AsyncCtl), hipMemcpyDeviceToHost, s));
    LHS_HIP(hipStreamSynchronize(s));
    if (t->status_host->error)
        return (lhs_status)t->status_host->error;
    if (h_ctl->error)
        return (lhs_status)h_ctl->error;
    const LevelCounters lc = *t->level_host;
    if (!lc.abort && h_ctl->work != 0)
        return LHS_EDEVICE;   // left with open states and no cap reached
    r->total_states = lc.n_next;
    r->edges = lc.edges;
    r->deadlocks = lc.deadlocks;
    r->capped = lc.abort ? 1 : 0;
    r->n_levels = 0;
    r->level_counts = nullptr;
    return LHS_OK;
}

}  // namespace lhs
