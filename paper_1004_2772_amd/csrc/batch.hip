// Batched exploration of many models (reach_explore_batch).
//
// Every model keeps its own table region (slots, rows, two frontiers) and its
// own level counters; all models advance together, one BFS level per step.  A
// step expands the tiles of every unfinished model in the same launch, so
// small and large models, and models of different state widths, share the
// GPU.  Two drivers:
//   * persistent (default): one cooperative launch runs every level of every
//     model from a device work queue of (model, tile) items; each model
//     advances at its own pace, with no grid-wide barrier;
//   * host loop (REACH_F_HOST_LOOP): all models advance together, one launch
//     per level step covering the tiles of every unfinished model, the host
//     reading the per-model counters after each.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "batch_kernels.h"
#include "expand_device.h"
#include "internal.h"
#include "reach_internal.h"

using namespace lhs;

namespace {

constexpr uint32_t kMaxBatch = 1024;   // models per call (tile prefix lives in LDS)
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
    uint32_t max_levels, pad;
};

// Per-model progress: updated by whichever workgroup finalises a level, so
// only ever accessed with coherent loads and stores.
struct ModelProgress {
    unsigned long long total, edges, deadlocks;
    uint32_t cur, n_levels, done, capped, overflow, pad;
};

__device__ __forceinline__ bool queue_failed(QueueState *qs) {
    return ld_coherent(&qs->error) != 0u;
}

// Finalise model i's level; block-wide.  Called by the workgroup that
// completed its last tile.
__device__ void finalize_level(const ModelState *ms, ModelProgress *mp, LevelState *lv, uint32_t i,
                               QueueState *qs, QCell *ring) {
    __shared__ uint32_t s_nt;
    __shared__ unsigned long long s_pos0;
    const uint32_t tid = threadIdx.x;
    const ModelState &M = ms[i];
    ModelProgress &P = mp[i];
    LevelState &L = lv[i];
    LevelCounters *lc = M.lc;
    const uint32_t n_next = ld_coherent(&lc->n_next);
    const uint32_t limit = ld_coherent(&L.limit);
    uint32_t *next = reinterpret_cast<uint32_t *>(ld_coherent(&L.next));
    const bool over = M.cap && n_next > limit;
    if (over) {
        // discard the partial level: zero every slot it claimed
        for (uint32_t j = tid; j < n_next; j += kExpandBlock)
            st_coherent(M.t.bucket + ld_coherent(next + j), 0ull);
    }
    wait_vm_complete();
    __syncthreads();
    if (tid == 0) {
        uint32_t nt = 0, done = 0;
        if (over) {
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
                nt = (n_next + kExpandBlock - 1) / kExpandBlock;
                const uint64_t room = M.cap ? M.cap - total : 0xFFFFFFFFull;
                st_coherent(&L.front, (unsigned long long)M.fr[cur]);
                st_coherent(&L.next, (unsigned long long)M.fr[cur ^ 1u]);
                st_coherent(&L.n_front, n_next);
                st_coherent(&L.limit, (uint32_t)min<uint64_t>(room, 0xFFFFFFFFull));
                st_coherent(&L.tiles_total, nt);
                st_coherent(&L.tiles_done, 0u);
            }
        }
        if (done)
            st_coherent(&P.done, 1u);
        st_coherent(&lc->n_next, 0u);
        st_coherent(&lc->abort, 0u);
        st_coherent(&lc->edges, 0ull);
        st_coherent(&lc->deadlocks, 0ull);
        wait_vm_complete();
        if (done)
            atomicSub(&qs->remaining, 1u);
        else
            s_pos0 = atomicAdd(&qs->tail, (unsigned long long)nt);
        s_nt = nt;
    }
    __syncthreads();
    const uint32_t nt = s_nt;
    // enqueue the next level's tiles: wait for each cell to be free, fill it,
    // then publish it
    for (uint32_t k = tid; k < nt; k += kExpandBlock) {
        const unsigned long long pos = s_pos0 + k;
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
}

template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock) void k_batch_persistent(const ModelState *__restrict__ ms,
                                                                   ModelProgress *mp, LevelState *lv,
                                                                   QueueState *qs, QCell *ring,
                                                                   uint32_t tcap) {
    extern __shared__ uint32_t smem[];
    expand_begin();
    __shared__ uint32_t s_model, s_tile, s_exit, s_fin;
    const uint32_t tid = threadIdx.x;
    while (true) {
        if (tid == 0) {
            uint32_t ex = 0;
            const unsigned long long pos = atomicAdd(&qs->head, 1ull);
            QCell *c = ring + (pos & qs->mask);
            uint32_t spins = 0;
            while (ld_coherent(&c->seq) != pos + 1ull) {
                if (ld_coherent(&qs->remaining) == 0u || queue_failed(qs)) {
                    ex = 1;
                    break;
                }
                if (++spins > kBarrierSpinLimit) {
                    atomicCAS(&qs->error, 0u, (uint32_t)LHS_ESTALL);
                    ex = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(4);
            }
            if (!ex) {
                s_model = ld_coherent(&c->model);
                s_tile = ld_coherent(&c->tile);
                st_coherent(&c->seq, pos + qs->mask + 1ull);   // free for position pos + R
            }
            s_exit = ex;
        }
        __syncthreads();
        if (s_exit)
            break;
        const uint32_t i = s_model, j = s_tile;
        const ModelState &M = ms[i];
        LevelState &L = lv[i];
        const uint32_t *front = reinterpret_cast<const uint32_t *>(ld_coherent(&L.front));
        uint32_t *next = reinterpret_cast<uint32_t *>(ld_coherent(&L.next));
        const uint32_t n_front = ld_coherent(&L.n_front);
        const uint32_t limit = ld_coherent(&L.limit);
        const uint64_t base = (uint64_t)j * kExpandBlock;
        const uint32_t rows = (uint32_t)min<uint64_t>(kExpandBlock, n_front - base);
        expand_tile<G, LS, true>(smem, M.t, M.m, front, base, rows, next, M.lc, limit, tcap);
        // this workgroup's stores of the tile are complete before it counts
        // the tile as done
        wait_vm_complete();
        __syncthreads();
        if (tid == 0) {
            const uint32_t done = atomicAdd(&L.tiles_done, 1u) + 1u;
            s_fin = done == ld_coherent(&L.tiles_total);
        }
        __syncthreads();
        if (s_fin)
            finalize_level(ms, mp, lv, i, qs, ring);
    }
}

__global__ void k_init_ring(QCell *ring, unsigned long long cells, uint32_t n_models) {
    for (unsigned long long p = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; p < cells;
         p += (unsigned long long)gridDim.x * blockDim.x) {
        // positions 0..n_models-1 hold level 0 (tile 0) of every model
        ring[p].seq = p < n_models ? p + 1 : p;
        ring[p].model = p < n_models ? (uint32_t)p : 0u;
        ring[p].tile = 0;
    }
}

uint64_t batch_auto_capacity(const reach_model *m) {
    if (m->state_cap)
        return auto_capacity(m);
    return 1ull << 21;
}

struct BatchModel {
    const reach_model *m = nullptr;
    uint32_t W = 0;
    lhs_table *t = nullptr;
    bool own = false;
    uint2 *d_trans = nullptr;
    // host-loop state
    uint32_t n_cur = 1, cur = 0, limit = 0;
    std::vector<uint64_t> levels;
    uint64_t total = 1, edges = 0, dead = 0;
    int capped = 0, done = 0;
};

}  // namespace

extern "C" {

lhs_status reach_explore_batch(const reach_model *const *models, uint32_t n, const reach_opts *o,
                               lhs_table *const *tables, reach_result *results) {
    if (!models || !results || n == 0 || n > kMaxBatch)
        return LHS_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        std::memset(&results[i], 0, sizeof(reach_result));
        if (validate_model(models[i]) != LHS_OK)
            return LHS_EINVAL;
        if (tables && tables[i] && tables[i]->W != models[i]->n_procs + models[i]->n_shared)
            return LHS_EINVAL;
    }
    reach_opts opts{};
    if (o)
        opts = *o;
    const uint32_t max_levels = opts.max_levels ? opts.max_levels : (1u << 16);
    const bool host_loop = (opts.flags & REACH_F_HOST_LOOP) != 0;
    hipStream_t s = (hipStream_t)opts.hip_stream;

    std::vector<BatchModel> bm(n);
    lhs_status rc = LHS_OK;
    DevStatus *d_status = nullptr;
    LevelCounters *d_lc = nullptr, *h_lc = nullptr;
    BatchSlot *d_slots = nullptr, *h_slots = nullptr;
    uint32_t *d_begin = nullptr, *h_begin = nullptr, *d_roots = nullptr, *d_root_off = nullptr;
    ModelState *d_ms = nullptr;
    ModelProgress *d_mp = nullptr;
    LevelState *d_lv = nullptr;
    QueueState *d_qs = nullptr;
    QCell *d_ring = nullptr;
    uint64_t *d_levels = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    uint32_t max_W = 1, tcap = 0;
    uint32_t tps = 0, ls = 0;
    // shape of the internal tables: the tuned batch choice for the widest model
    uint32_t widest = 1;
    for (uint32_t i = 0; i < n; ++i)
        widest = std::max(widest, models[i]->n_procs + models[i]->n_shared);
    const lhs_config batch_cfg = tuned_config(LHS_TUNE_BATCH, widest, opts.capacity ? opts.capacity : (1ull << 21));

    // ---- set-up: tables, models, roots (outside the timed exploration) --
    for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
        BatchModel &b = bm[i];
        b.m = models[i];
        b.W = b.m->n_procs + b.m->n_shared;
        max_W = std::max(max_W, b.W);
        tcap = std::max(tcap, trans_lds_entries(b.m->n_procs, b.m->n_locals, b.m->trans_per_local));
        if (tables && tables[i]) {
            b.t = tables[i];
        } else {
            const uint64_t cap = opts.capacity ? opts.capacity : batch_auto_capacity(b.m);
            rc = lhs_create_ex(cap, b.W, &batch_cfg, &b.t);
            b.own = rc == LHS_OK;
        }
        if (rc != LHS_OK)
            break;
        if (b.m->state_cap && b.m->state_cap >= b.t->capacity) {
            rc = LHS_EINVAL;
            break;
        }
        if (i == 0) {
            tps = tps_expand(b.t);
            ls = b.t->line_slots;
        } else if (b.t->line_slots != ls) {
            rc = LHS_EINVAL;   // one launch serves every table: one line width
            break;
        }
        rc = ensure_bfs_buffers(b.t);
        if (rc != LHS_OK)
            break;
        std::vector<uint2> packed;
        pack_model(b.m, packed);
        if (hipMalloc(&b.d_trans, packed.size() * sizeof(uint2)) != hipSuccess ||
            hipMemcpy(b.d_trans, packed.data(), packed.size() * sizeof(uint2), hipMemcpyHostToDevice) !=
                hipSuccess)
            rc = LHS_EDEVICE;
        b.limit = b.m->state_cap ? (uint32_t)std::min<uint64_t>(b.m->state_cap - 1, 0xFFFFFFFFull)
                                 : 0xFFFFFFFFu;
        b.levels.push_back(1);
    }
    std::vector<uint32_t> roots, root_off(n);
    for (uint32_t i = 0; i < n; ++i) {
        root_off[i] = (uint32_t)roots.size();
        if (bm[i].m)
            roots.insert(roots.end(), bm[i].m->init, bm[i].m->init + bm[i].W);
    }
    if (rc == LHS_OK &&
        (hipMalloc(&d_status, sizeof(DevStatus)) != hipSuccess ||
         hipMalloc(&d_lc, n * sizeof(LevelCounters)) != hipSuccess ||
         hipHostMalloc(&h_lc, n * sizeof(LevelCounters), hipHostMallocDefault) != hipSuccess ||
         hipMalloc(&d_slots, n * sizeof(BatchSlot)) != hipSuccess ||
         hipHostMalloc(&h_slots, n * sizeof(BatchSlot), hipHostMallocDefault) != hipSuccess ||
         hipMalloc(&d_begin, (n + 1) * sizeof(uint32_t)) != hipSuccess ||
         hipHostMalloc(&h_begin, (n + 1) * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
         hipMalloc(&d_roots, roots.size() * sizeof(uint32_t)) != hipSuccess ||
         hipMalloc(&d_root_off, n * sizeof(uint32_t)) != hipSuccess ||
         hipMemcpy(d_roots, roots.data(), roots.size() * sizeof(uint32_t), hipMemcpyHostToDevice) !=
             hipSuccess ||
         hipMemcpy(d_root_off, root_off.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice) !=
             hipSuccess ||
         hipMemset(d_status, 0, sizeof(DevStatus)) != hipSuccess ||
         hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess))
        rc = LHS_ENOMEM;
    // all tables of the batch report into one status word
    for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
        BatchModel &b = bm[i];
        b.t->last_stream = s;
        rc = lhs_clear(b.t, s);
        BatchSlot &sl = h_slots[i];
        sl.t = view(b.t);
        sl.t.status = d_status;
        sl.m = model_view(b.m, b.d_trans);
        sl.front = b.t->frontier[0];
        sl.next = b.t->frontier[1];
        sl.lc = d_lc + i;
        sl.n_front = 1;
        sl.limit = b.limit;
        sl.tile_begin = 0;
        sl.pad = 0;
    }
    if (rc == LHS_OK) {
        if (hipMemcpyAsync(d_slots, h_slots, n * sizeof(BatchSlot), hipMemcpyHostToDevice, s) != hipSuccess)
            rc = LHS_EDEVICE;
        hipLaunchKernelGGL(k_zero_levels, dim3((n + 255) / 256), dim3(256), 0, s, d_lc, n);
        if (launch_insert_roots(ls, s, d_slots, d_roots, d_root_off, n) != LHS_OK ||
            hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            rc = LHS_EDEVICE;
    }
    const size_t lds = (size_t)expand_lds_words(max_W, tcap) * sizeof(uint32_t);

    // ---- exploration -------------------------------------------------------
    if (rc == LHS_OK && !host_loop) {
        std::vector<ModelState> hms(n);
        std::vector<ModelProgress> hmp(n);
        std::vector<LevelState> hlv(n);
        // ring: at most one level's tiles per model are pending at a time
        uint64_t pending = n;
        for (uint32_t i = 0; i < n; ++i)
            pending += bm[i].t->capacity / kExpandBlock + 1;
        uint64_t cells = 1024;
        while (cells < 2 * pending)
            cells <<= 1;
        QueueState hq{};
        hq.head = 0;
        hq.tail = n;
        hq.remaining = n;
        hq.error = 0;
        hq.mask = cells - 1;
        if (hipMalloc(&d_ms, n * sizeof(ModelState)) != hipSuccess ||
            hipMalloc(&d_mp, n * sizeof(ModelProgress)) != hipSuccess ||
            hipMalloc(&d_lv, n * sizeof(LevelState)) != hipSuccess ||
            hipMalloc(&d_qs, sizeof(QueueState)) != hipSuccess ||
            hipMalloc(&d_ring, cells * sizeof(QCell)) != hipSuccess ||
            hipMalloc(&d_levels, (uint64_t)n * max_levels * sizeof(uint64_t)) != hipSuccess)
            rc = LHS_ENOMEM;
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            ModelState &M = hms[i];
            std::memset(&M, 0, sizeof(M));
            M.t = h_slots[i].t;
            M.m = h_slots[i].m;
            M.lc = h_slots[i].lc;
            M.fr[0] = bm[i].t->frontier[0];
            M.fr[1] = bm[i].t->frontier[1];
            M.levels = reinterpret_cast<unsigned long long *>(d_levels + (uint64_t)i * max_levels);
            M.cap = bm[i].m->state_cap;
            M.max_levels = max_levels;
            ModelProgress &P = hmp[i];
            std::memset(&P, 0, sizeof(P));
            P.total = 1;
            P.n_levels = 1;
            LevelState &L = hlv[i];
            L.front = (unsigned long long)M.fr[0];
            L.next = (unsigned long long)M.fr[1];
            L.n_front = 1;
            L.limit = bm[i].limit;
            L.tiles_total = 1;
            L.tiles_done = 0;
        }
        std::vector<uint64_t> lvl_host((uint64_t)n * max_levels, 0);
        for (uint32_t i = 0; i < n; ++i)
            lvl_host[(uint64_t)i * max_levels] = 1;
        int dev = 0, ncu = 0, per_cu = 0;
        const void *fn = nullptr;
        (void)with_shape(tps, ls, [&](auto G, auto L) {
            fn = (const void *)k_batch_persistent<decltype(G)::value, decltype(L)::value>;
            return LHS_OK;
        });
        if (rc == LHS_OK &&
            (hipMemcpy(d_ms, hms.data(), n * sizeof(ModelState), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(d_mp, hmp.data(), n * sizeof(ModelProgress), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(d_lv, hlv.data(), n * sizeof(LevelState), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(d_qs, &hq, sizeof(hq), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(d_levels, lvl_host.data(), lvl_host.size() * sizeof(uint64_t),
                       hipMemcpyHostToDevice) != hipSuccess ||
             hipGetDevice(&dev) != hipSuccess ||
             hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
             hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
             per_cu < 1))
            rc = LHS_EDEVICE;
        if (rc == LHS_OK) {
            hipLaunchKernelGGL(k_init_ring, dim3((uint32_t)std::min<uint64_t>((cells + 255) / 256, 4096)),
                               dim3(256), 0, s, d_ring, (unsigned long long)cells, n);
            const uint32_t grid = (uint32_t)(ncu * per_cu);
            void *args[] = {&d_ms, &d_mp, &d_lv, &d_qs, &d_ring, &tcap};
            (void)hipEventRecord(e0, s);
            if (hipGetLastError() != hipSuccess ||
                hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kExpandBlock), args, lds, s) != hipSuccess)
                rc = LHS_EDEVICE;
            (void)hipEventRecord(e1, s);
            if (rc == LHS_OK && hipStreamSynchronize(s) != hipSuccess)
                rc = LHS_EDEVICE;
        }
        DevStatus st{};
        if (rc == LHS_OK &&
            (hipMemcpy(&hq, d_qs, sizeof(hq), hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(&st, d_status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(hmp.data(), d_mp, n * sizeof(ModelProgress), hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(lvl_host.data(), d_levels, lvl_host.size() * sizeof(uint64_t),
                       hipMemcpyDeviceToHost) != hipSuccess))
            rc = LHS_EDEVICE;
        if (rc == LHS_OK && (hq.error || st.error))
            rc = (lhs_status)(hq.error ? hq.error : st.error);
        float ms = 0;
        if (rc == LHS_OK)
            (void)hipEventElapsedTime(&ms, e0, e1);
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            const ModelProgress &M = hmp[i];
            if (M.overflow || !M.done) {
                rc = M.overflow ? LHS_EINVAL : LHS_EDEVICE;
                break;
            }
            reach_result &r = results[i];
            r.total_states = M.total;
            r.edges = M.edges;
            r.deadlocks = M.deadlocks;
            r.capped = (int32_t)M.capped;
            r.n_levels = M.n_levels;
            r.wait_hits = st.wait_hits;
            r.gpu_ms = ms;
            r.level_counts = (uint64_t *)std::malloc(M.n_levels * sizeof(uint64_t));
            if (!r.level_counts) {
                rc = LHS_ENOMEM;
                break;
            }
            std::memcpy(r.level_counts, lvl_host.data() + (uint64_t)i * max_levels,
                        M.n_levels * sizeof(uint64_t));
        }
    } else if (rc == LHS_OK) {
        (void)hipEventRecord(e0, s);
        std::vector<uint32_t> act;
        while (rc == LHS_OK) {
            act.clear();
            uint32_t tiles = 0;
            for (uint32_t i = 0; i < n; ++i) {
                BatchModel &b = bm[i];
                if (b.done)
                    continue;
                BatchSlot &sl = h_slots[act.size()];
                sl.t = view(b.t);
                sl.t.status = d_status;
                sl.m = model_view(b.m, b.d_trans);
                sl.front = b.t->frontier[b.cur];
                sl.next = b.t->frontier[b.cur ^ 1];
                sl.lc = d_lc + act.size();
                sl.n_front = b.n_cur;
                sl.limit = b.limit;
                sl.tile_begin = tiles;
                h_begin[act.size()] = tiles;
                tiles += (b.n_cur + kExpandBlock - 1) / kExpandBlock;
                act.push_back(i);
            }
            if (act.empty())
                break;
            const uint32_t na = (uint32_t)act.size();
            h_begin[na] = tiles;
            if (hipMemcpyAsync(d_slots, h_slots, na * sizeof(BatchSlot), hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(d_begin, h_begin, (na + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s) !=
                    hipSuccess) {
                rc = LHS_EDEVICE;
                break;
            }
            hipLaunchKernelGGL(k_zero_levels, dim3((na + 255) / 256), dim3(256), 0, s, d_lc, na);
            if (launch_expand_multi(tps, ls, tiles, max_W, tcap, s, d_slots, d_begin, na) != LHS_OK) {
                rc = LHS_EDEVICE;
                break;
            }
            DevStatus st{};
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(h_lc, d_lc, na * sizeof(LevelCounters), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(&st, d_status, sizeof(st), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = LHS_EDEVICE;
                break;
            }
            if (st.error) {
                rc = (lhs_status)st.error;
                break;
            }
            for (uint32_t a = 0; a < na; ++a) {
                BatchModel &b = bm[act[a]];
                const LevelCounters &lc = h_lc[a];
                if (b.m->state_cap && lc.n_next > b.limit) {
                    hipLaunchKernelGGL(k_rollback_one, dim3(std::min<uint32_t>((lc.n_next + 255) / 256, 4096)),
                                       dim3(256), 0, s, b.t->bucket, b.t->frontier[b.cur ^ 1], lc.n_next);
                    b.capped = 1;
                    b.done = 1;
                    continue;
                }
                b.edges += lc.edges;
                b.dead += lc.deadlocks;
                if (lc.n_next == 0) {
                    b.done = 1;
                    continue;
                }
                if (b.levels.size() >= max_levels) {
                    rc = LHS_EINVAL;
                    break;
                }
                b.levels.push_back(lc.n_next);
                b.total += lc.n_next;
                b.n_cur = lc.n_next;
                b.cur ^= 1;
                if (b.m->state_cap)
                    b.limit = (uint32_t)std::min<uint64_t>(b.m->state_cap - b.total, 0xFFFFFFFFull);
            }
        }
        (void)hipEventRecord(e1, s);
        float ms = 0;
        if (hipEventSynchronize(e1) == hipSuccess)
            (void)hipEventElapsedTime(&ms, e0, e1);
        DevStatus st{};
        (void)hipMemcpy(&st, d_status, sizeof(st), hipMemcpyDeviceToHost);
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            BatchModel &b = bm[i];
            reach_result &r = results[i];
            r.total_states = b.total;
            r.edges = b.edges;
            r.deadlocks = b.dead;
            r.capped = b.capped;
            r.n_levels = (uint32_t)b.levels.size();
            r.wait_hits = st.wait_hits;
            r.gpu_ms = ms;
            r.level_counts = (uint64_t *)std::malloc(b.levels.size() * sizeof(uint64_t));
            if (!r.level_counts) {
                rc = LHS_ENOMEM;
                break;
            }
            std::memcpy(r.level_counts, b.levels.data(), b.levels.size() * sizeof(uint64_t));
        }
    }

    // ---- tear-down ---------------------------------------------------------
    for (auto &b : bm) {
        (void)hipFree(b.d_trans);
        if (b.own)
            lhs_destroy(b.t);
    }
    (void)hipFree(d_status);
    (void)hipFree(d_lc);
    (void)hipFree(d_slots);
    (void)hipFree(d_begin);
    (void)hipFree(d_roots);
    (void)hipFree(d_root_off);
    (void)hipFree(d_ms);
    (void)hipFree(d_mp);
    (void)hipFree(d_lv);
    (void)hipFree(d_qs);
    (void)hipFree(d_ring);
    (void)hipFree(d_levels);
    if (h_lc)
        (void)hipHostFree(h_lc);
    if (h_slots)
        (void)hipHostFree(h_slots);
    if (h_begin)
        (void)hipHostFree(h_begin);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (rc != LHS_OK)
        for (uint32_t i = 0; i < n; ++i)
            reach_result_free(&results[i]);
    return rc;
}

}  // extern "C"
