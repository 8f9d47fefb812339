// Batched exploration of many models (reach_explore_batch).
//
// Every model keeps its own table region (slots, rows, two frontiers) and its
// own level counters; all models advance together, one BFS level per step.  A
// step expands the tiles of every unfinished model in the same launch, so
// small and large models, and models of different state widths, share the
// GPU.  Two drivers:
//   * persistent (default): one launch of resident workgroups runs every
//     level of every model from a device work queue of (model, tile) items;
//     each model advances at its own pace, with no grid-wide barrier;
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
#include "persistent.h"
#include "reach_internal.h"

using namespace lhs;

namespace {

constexpr uint32_t kMaxBatch = 1024;   // models per call (tile prefix lives in LDS)

// With 8-slot lines, at least four waves per SIMD (at most 128 VGPRs): four
// workgroups per CU, as the LDS layout allows.  Wider lines would spill.
template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock, LS == 8 ? 4 : 1) void k_batch_persistent(const ModelState *__restrict__ ms,
                                                                   ModelProgress *mp, LevelState *lv,
                                                                   QueueState *qs, QCell *ring,
                                                                   uint32_t tcap) {
    extern __shared__ uint32_t smem[];
    expand_begin();
    __shared__ uint32_t s_model, s_tile, s_exit, s_fin;
    const uint32_t tid = threadIdx.x;
    bool kept = false;   // tile 0 of s_model's new level is this workgroup's
    while (true) {
        if (tid == 0 && kept) {
            s_tile = 0;
            s_exit = queue_failed(qs) ? 1u : 0u;
        } else if (tid == 0) {
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
                // the item is read before the cell is freed: the store must
                // not be performed ahead of the loads (different addresses),
                // or the next producer could overwrite the item first
                wait_vm_complete();
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
        const uint32_t rows_per = ld_coherent(&L.tile_rows);
        const uint64_t base = (uint64_t)j * rows_per;
        const uint32_t rows = (uint32_t)min<uint64_t>(rows_per, n_front - base);
        expand_tile<G, LS, true>(smem, M.t, M.m, front, base, rows, next, M.lc, limit, tcap);
        // this workgroup's stores of the tile are complete before it counts
        // the tile as done
        wait_vm_complete();
        __syncthreads();
        if (tid == 0) {
            // the level's tile count, read while this tile still holds the
            // level open: once the count below reaches it, the finaliser
            // may already be writing the next level's count
            const uint32_t total = ld_coherent(&L.tiles_total);
            // the load and the add go to different addresses, which the
            // memory model does not order: the load completes first
            wait_vm_complete();
            const uint32_t done = atomicAdd(&L.tiles_done, 1u) + 1u;
            s_fin = done == total;
        }
        __syncthreads();
        kept = s_fin && finalize_level(M, mp, lv, i, qs, ring);
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

// One table to empty: its slots and its status word.
struct TableZero {
    uint4 *bucket;
    unsigned long long chunks;   // 16-byte chunks of the slot array
    DevStatus *status;
};

// Empty every table of the batch in one launch: blockIdx.y = table.
__global__ void k_clear_tables(const TableZero *z) {
    const TableZero tz = z[blockIdx.y];
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < tz.chunks;
         i += (unsigned long long)gridDim.x * blockDim.x)
        tz.bucket[i] = make_uint4(0, 0, 0, 0);
    if (blockIdx.x == 0 && threadIdx.x == 0)
        *tz.status = DevStatus{0, 0, 0, 0, 0};
}

// Copy levels 1 .. n_levels-1 of every model into one compact array, model
// after model (one workgroup; n <= kMaxBatch).
__global__ __launch_bounds__(1024) void k_gather_levels(const ModelState *ms, const ModelProgress *mp,
                                                        uint32_t n, unsigned long long *out) {
    __shared__ uint32_t off[kMaxBatch + 1];
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        uint32_t acc = 0;
        for (uint32_t i = 0; i < n; ++i) {
            off[i] = acc;
            acc += mp[i].n_levels - 1;
        }
        off[n] = acc;
    }
    __syncthreads();
    for (uint32_t i = tid; i < n; i += blockDim.x)
        for (uint32_t k = 1; k < mp[i].n_levels; ++k)
            out[off[i] + k - 1] = ms[i].levels[k];
}

struct BatchModel {
    const reach_model *m = nullptr;
    uint32_t W = 0;
    lhs_table *t = nullptr;
    bool own = false;
    size_t trans_off = 0;        // entries into the packed transition area
    // host-loop state
    uint32_t n_cur = 1, cur = 0, limit = 0;
    std::vector<uint64_t> levels;
    uint64_t total = 1, edges = 0, dead = 0;
    int capped = 0, done = 0;
};

}  // namespace

namespace lhs {

lhs_status explore_prefix(lhs_table *t, const TableView &tv, const ModelView &mv, uint64_t cap, PrefixArea *d,
                          PrefixArea *h, hipStream_t s, PrefixOut &out) {
    // level 0 (s0 at frontier[0][0]) is tile 0 of queue position 0
    const size_t head = offsetof(PrefixArea, levels);
    std::memset(h, 0, head);
    h->qs.tail = 1;
    h->qs.remaining = 1;
    h->qs.mask = kPrefixCells - 1;
    ModelState &M = h->ms;
    M.t = tv;
    M.m = mv;
    M.lc = t->level;
    M.fr[0] = t->frontier[0];
    M.fr[1] = t->frontier[1];
    M.levels = d->levels;
    M.cap = cap;
    M.max_levels = kPrefixLevels;
    M.handover = kPrefixHandover;
    h->mp.total = 1;
    h->mp.n_levels = 1;
    LevelState &L = h->lv;
    L.front = (unsigned long long)M.fr[0];
    L.next = (unsigned long long)M.fr[1];
    L.n_front = 1;
    L.limit = cap ? (uint32_t)std::min<uint64_t>(cap - 1, 0xFFFFFFFFull) : 0xFFFFFFFFu;
    L.tiles_total = 1;
    L.tile_rows = kExpandBlock;
    LHS_HIP(hipMemcpyAsync(d, h, head, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_init_ring, dim3(kPrefixCells / 256), dim3(256), 0, s, d->ring,
                       (unsigned long long)kPrefixCells, 1u);
    LHS_HIP(hipGetLastError());
    const uint32_t tps = tps_expand(t);
    const uint32_t tcap = trans_lds_entries(mv.P, mv.L, mv.K);
    const size_t lds = (size_t)expand_lds_words(mv.W, tcap, tps) * sizeof(uint32_t);
    lhs_status rc = with_shape(tps, t->line_slots, [&](auto G, auto LS) {
        const void *fn = (const void *)k_batch_persistent<decltype(G)::value, decltype(LS)::value>;
        int dev = 0, ncu = 0, per_cu = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
            per_cu < 1)
            return LHS_EDEVICE;
        // the workgroups that fit at once, at most kPrefixGrid: every one
        // holds a queue position while the levels are small
        const uint32_t grid =
            exploration_grid(t, std::min<uint64_t>((uint64_t)ncu * per_cu, kPrefixGrid));
        const ModelState *ms = &d->ms;
        ModelProgress *mp = &d->mp;
        LevelState *lv = &d->lv;
        QueueState *qs = &d->qs;
        QCell *ring = d->ring;
        uint32_t tc = tcap;
        void *args[] = {&ms, &mp, &lv, &qs, &ring, &tc};
        return hipLaunchKernel(fn, dim3(grid), dim3(kExpandBlock), args, lds, s) == hipSuccess ? LHS_OK
                                                                                                : LHS_EDEVICE;
    });
    if (rc != LHS_OK)
        return rc;
    LHS_HIP(hipMemcpyAsync(h, d, offsetof(PrefixArea, ring), hipMemcpyDeviceToHost, s));
    LHS_HIP(hipMemcpyAsync(t->status_host, t->status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    LHS_HIP(hipStreamSynchronize(s));
    if (h->qs.error)
        return (lhs_status)h->qs.error;
    if (t->status_host->error)
        return (lhs_status)t->status_host->error;
    const ModelProgress &P = h->mp;
    if (!P.done || P.overflow || P.n_levels > kPrefixLevels)
        return LHS_EDEVICE;
    out.levels.assign(h->levels + 1, h->levels + P.n_levels);
    out.total = P.total;
    out.edges = P.edges;
    out.deadlocks = P.deadlocks;
    out.cur = P.cur;
    out.handed = P.handed != 0;
    out.capped = P.capped != 0;
    return LHS_OK;
}

}  // namespace lhs

extern "C" {

static lhs_status reach_explore_batch_impl(const reach_model *const *models, uint32_t n, const reach_opts *o,
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
    if (opts.flags & REACH_F_ASYNC)
        return LHS_EINVAL;   // the batch keeps levels: its results carry level counts
    hipStream_t s = (hipStream_t)opts.hip_stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess)
        return LHS_EDEVICE;

    std::vector<BatchModel> bm(n);
    lhs_status rc = LHS_OK;
    uint32_t max_W = 1, tcap = 0, tps = 0, ls = 0;
    // shape of the internal tables: the tuned batch choice for the widest model
    uint32_t widest = 1;
    for (uint32_t i = 0; i < n; ++i)
        widest = std::max(widest, models[i]->n_procs + models[i]->n_shared);
    const lhs_config batch_cfg = tuned_config(LHS_TUNE_BATCH, widest, opts.capacity ? opts.capacity : (1ull << 21));

    // ---- tables and host-side packing (no device work yet) -----------------
    std::vector<uint2> trans_all;
    std::vector<uint32_t> roots, root_off(n);
    uint64_t pending = n;    // ring cells: at most one level's tiles per model
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
        b.trans_off = trans_all.size();
        trans_all.insert(trans_all.end(), packed.begin(), packed.end());
        root_off[i] = (uint32_t)roots.size();
        roots.insert(roots.end(), b.m->init, b.m->init + b.W);
        b.limit = b.m->state_cap ? (uint32_t)std::min<uint64_t>(b.m->state_cap - 1, 0xFFFFFFFFull)
                                 : 0xFFFFFFFFu;
        b.levels.push_back(1);
        // tiles of one level: full tiles, or small ones for small levels
        pending += std::max<uint64_t>(b.t->capacity / kExpandBlock, kSmallLevel / kMinTileRows) + 1;
    }
    uint64_t cells = 1024;
    while (cells < 2 * pending)
        cells <<= 1;

    // ---- one device region: [uploaded part | device-only part] -------------
    Carve c;
    const size_t o_status = c.take<DevStatus>(1), o_qs = c.take<QueueState>(1),
                 o_mp = c.take<ModelProgress>(n), o_lc = c.take<LevelCounters>(n),
                 o_slots = c.take<BatchSlot>(n), o_begin = c.take<uint32_t>(n + 1),
                 o_roots = c.take<uint32_t>(roots.size()), o_root_off = c.take<uint32_t>(n),
                 o_trans = c.take<uint2>(trans_all.size()), o_ms = c.take<ModelState>(n),
                 o_lv = c.take<LevelState>(n), o_zero = c.take<TableZero>(n);
    const size_t up_bytes = c.off;
    const size_t o_ring = host_loop ? 0 : c.take<QCell>(cells);
    const size_t o_levels = host_loop ? 0 : c.take<unsigned long long>((uint64_t)n * max_levels);
    const size_t o_clevels = host_loop ? 0 : c.take<unsigned long long>((uint64_t)n * max_levels);
    const size_t dev_bytes = c.off;
    // pinned host region: a mirror of the uploaded part, then host-loop buffers
    Carve hc;
    hc.off = up_bytes;
    const size_t h_lc_off = hc.take<LevelCounters>(n), h_slots_off = hc.take<BatchSlot>(n),
                 h_begin_off = hc.take<uint32_t>(n + 1);
    const size_t host_bytes = hc.off;

    Workspace &ws = workspace(dev);
    std::unique_lock<std::mutex> lock(ws.mu);
    if (rc == LHS_OK)
        rc = ws_reserve(ws, dev_bytes, host_bytes);
    if (rc != LHS_OK) {
        lock.unlock();
        for (auto &b : bm)
            if (b.own)
                lhs_destroy(b.t);
        return rc;
    }
    void *D = ws.dev, *H = ws.host;
    DevStatus *d_status = at<DevStatus>(D, o_status);
    QueueState *d_qs = at<QueueState>(D, o_qs);
    ModelProgress *d_mp = at<ModelProgress>(D, o_mp);
    LevelCounters *d_lc = at<LevelCounters>(D, o_lc);
    BatchSlot *d_slots = at<BatchSlot>(D, o_slots);
    uint32_t *d_begin = at<uint32_t>(D, o_begin);
    uint2 *d_trans = at<uint2>(D, o_trans);
    ModelState *d_ms = at<ModelState>(D, o_ms);
    LevelState *d_lv = at<LevelState>(D, o_lv);
    QCell *d_ring = at<QCell>(D, o_ring);
    unsigned long long *d_levels = at<unsigned long long>(D, o_levels);
    LevelCounters *h_lc = at<LevelCounters>(H, h_lc_off);
    BatchSlot *h_slots = at<BatchSlot>(H, h_slots_off);
    uint32_t *h_begin = at<uint32_t>(H, h_begin_off);

    // ---- fill the upload mirror ---------------------------------------------
    std::memset(H, 0, up_bytes);   // status, level counters: zero
    std::memcpy(at<void>(H, o_roots), roots.data(), roots.size() * sizeof(uint32_t));
    std::memcpy(at<void>(H, o_root_off), root_off.data(), n * sizeof(uint32_t));
    std::memcpy(at<void>(H, o_trans), trans_all.data(), trans_all.size() * sizeof(uint2));
    BatchSlot *u_slots = at<BatchSlot>(H, o_slots);
    TableZero *u_zero = at<TableZero>(H, o_zero);
    uint64_t max_chunks = 1;
    for (uint32_t i = 0; i < n; ++i) {
        BatchModel &b = bm[i];
        b.t->last_stream = s;
        BatchSlot &sl = u_slots[i];
        sl.t = view(b.t);
        sl.t.status = d_status;   // all tables of the batch report into one status word
        sl.m = model_view(b.m, d_trans + b.trans_off);
        sl.front = b.t->frontier[0];
        sl.next = b.t->frontier[1];
        sl.lc = d_lc + i;
        sl.n_front = 1;
        sl.limit = b.limit;
        sl.tile_begin = 0;
        sl.pad = 0;
        u_zero[i] = TableZero{reinterpret_cast<uint4 *>(b.t->bucket), b.t->capacity / 2, b.t->status};
        max_chunks = std::max<uint64_t>(max_chunks, b.t->capacity / 2);
    }
    if (!host_loop) {
        QueueState &q = *at<QueueState>(H, o_qs);
        q.head = 0;
        q.tail = n;
        q.remaining = n;
        q.error = 0;
        q.mask = cells - 1;
        for (uint32_t i = 0; i < n; ++i) {
            ModelState &M = at<ModelState>(H, o_ms)[i];
            M.t = u_slots[i].t;
            M.m = u_slots[i].m;
            M.lc = u_slots[i].lc;
            M.fr[0] = bm[i].t->frontier[0];
            M.fr[1] = bm[i].t->frontier[1];
            M.levels = d_levels + (uint64_t)i * max_levels;
            M.cap = bm[i].m->state_cap;
            M.max_levels = max_levels;
            ModelProgress &P = at<ModelProgress>(H, o_mp)[i];
            P.total = 1;
            P.n_levels = 1;
            LevelState &L = at<LevelState>(H, o_lv)[i];
            L.front = (unsigned long long)M.fr[0];
            L.next = (unsigned long long)M.fr[1];
            L.n_front = 1;
            L.limit = bm[i].limit;
            L.tiles_total = 1;
            L.tiles_done = 0;
            L.tile_rows = kExpandBlock;
            L.pad = 0;
        }
    }

    // ---- one upload, clear every table, insert the roots --------------------
    if (hipMemcpyAsync(D, H, up_bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        rc = LHS_EDEVICE;
    if (rc == LHS_OK) {
        const uint32_t gx = (uint32_t)std::min<uint64_t>((max_chunks + 255) / 256, 2048);
        hipLaunchKernelGGL(k_clear_tables, dim3(gx, n), dim3(256), 0, s, at<TableZero>(D, o_zero));
        if (hipGetLastError() != hipSuccess ||
            launch_insert_roots(ls, s, d_slots, at<uint32_t>(D, o_roots), at<uint32_t>(D, o_root_off), n) !=
                LHS_OK)
            rc = LHS_EDEVICE;
    }
    const size_t lds = (size_t)expand_lds_words(max_W, tcap, tps) * sizeof(uint32_t);

    // ---- exploration -------------------------------------------------------
    if (rc == LHS_OK && !host_loop) {
        int ncu = 0, per_cu = 0;
        const void *fn = nullptr;
        (void)with_shape(tps, ls, [&](auto G, auto L) {
            fn = (const void *)k_batch_persistent<decltype(G)::value, decltype(L)::value>;
            return LHS_OK;
        });
        if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
            per_cu < 1)
            rc = LHS_EDEVICE;
        float ms = 0;
        if (rc == LHS_OK) {
            hipLaunchKernelGGL(k_init_ring, dim3((uint32_t)std::min<uint64_t>((cells + 255) / 256, 4096)),
                               dim3(256), 0, s, d_ring, (unsigned long long)cells, n);
            const uint32_t grid = (uint32_t)(ncu * per_cu);
            void *args[] = {&d_ms, &d_mp, &d_lv, &d_qs, &d_ring, &tcap};
            (void)hipEventRecord(ws.ev[0], s);
            if (hipGetLastError() != hipSuccess ||
                hipLaunchKernel(fn, dim3(grid), dim3(kExpandBlock), args, lds, s) != hipSuccess)
                rc = LHS_EDEVICE;
            (void)hipEventRecord(ws.ev[1], s);
            if (rc == LHS_OK) {
                hipLaunchKernelGGL(k_gather_levels, dim3(1), dim3(1024), 0, s, d_ms, d_mp, n,
                                   at<unsigned long long>(D, o_clevels));
                // status, queue state and progress are the region's first bytes
                if (hipGetLastError() != hipSuccess ||
                    hipMemcpyAsync(H, D, o_lc, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess)
                    rc = LHS_EDEVICE;
            }
            if (rc == LHS_OK)
                (void)hipEventElapsedTime(&ms, ws.ev[0], ws.ev[1]);
        }
        const DevStatus &st = *at<DevStatus>(H, o_status);
        const QueueState &hq = *at<QueueState>(H, o_qs);
        const ModelProgress *hmp = at<ModelProgress>(H, o_mp);
        if (rc == LHS_OK && (hq.error || st.error))
            rc = (lhs_status)(hq.error ? hq.error : st.error);
        uint64_t n_lvl = 0;
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            if (hmp[i].overflow || !hmp[i].done)
                rc = hmp[i].overflow ? LHS_EINVAL : LHS_EDEVICE;
            n_lvl += hmp[i].n_levels - 1;
        }
        std::vector<uint64_t> lv(n_lvl);
        if (rc == LHS_OK && n_lvl &&
            hipMemcpy(lv.data(), at<void>(D, o_clevels), n_lvl * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
                hipSuccess)
            rc = LHS_EDEVICE;
        uint64_t at_lvl = 0;
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            const ModelProgress &M = hmp[i];
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
            r.level_counts[0] = 1;
            std::memcpy(r.level_counts + 1, lv.data() + at_lvl, (M.n_levels - 1) * sizeof(uint64_t));
            at_lvl += M.n_levels - 1;
        }
    } else if (rc == LHS_OK) {
        (void)hipEventRecord(ws.ev[0], s);
        std::vector<uint32_t> act;
        DevStatus *h_st = at<DevStatus>(H, o_status);
        while (rc == LHS_OK) {
            act.clear();
            uint32_t tiles = 0;
            for (uint32_t i = 0; i < n; ++i) {
                BatchModel &b = bm[i];
                if (b.done)
                    continue;
                BatchSlot &sl = h_slots[act.size()];
                sl = u_slots[i];
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
            if (hipGetLastError() != hipSuccess ||
                hipMemcpyAsync(h_lc, d_lc, na * sizeof(LevelCounters), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipMemcpyAsync(h_st, d_status, sizeof(DevStatus), hipMemcpyDeviceToHost, s) != hipSuccess ||
                hipStreamSynchronize(s) != hipSuccess) {
                rc = LHS_EDEVICE;
                break;
            }
            if (h_st->error) {
                rc = (lhs_status)h_st->error;
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
        (void)hipEventRecord(ws.ev[1], s);
        float ms = 0;
        if (hipEventSynchronize(ws.ev[1]) == hipSuccess)
            (void)hipEventElapsedTime(&ms, ws.ev[0], ws.ev[1]);
        if (hipMemcpy(h_st, d_status, sizeof(DevStatus), hipMemcpyDeviceToHost) != hipSuccess && rc == LHS_OK)
            rc = LHS_EDEVICE;
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            BatchModel &b = bm[i];
            reach_result &r = results[i];
            r.total_states = b.total;
            r.edges = b.edges;
            r.deadlocks = b.dead;
            r.capped = b.capped;
            r.n_levels = (uint32_t)b.levels.size();
            r.wait_hits = h_st->wait_hits;
            r.gpu_ms = ms;
            r.level_counts = (uint64_t *)std::malloc(b.levels.size() * sizeof(uint64_t));
            if (!r.level_counts) {
                rc = LHS_ENOMEM;
                break;
            }
            std::memcpy(r.level_counts, b.levels.data(), b.levels.size() * sizeof(uint64_t));
        }
    }
    // the workspace may be reused by the next call once this one's work is done
    if (hipStreamSynchronize(s) != hipSuccess && rc == LHS_OK)
        rc = LHS_EDEVICE;
    lock.unlock();

    // ---- tear-down ---------------------------------------------------------
    for (auto &b : bm)
        if (b.own)
            lhs_destroy(b.t);
    if (rc != LHS_OK)
        for (uint32_t i = 0; i < n; ++i)
            reach_result_free(&results[i]);
    return rc;
}

lhs_status reach_explore_batch(const reach_model *const *models, uint32_t n, const reach_opts *o,
                               lhs_table *const *tables, reach_result *results) {
    return lhs::guard([&] { return reach_explore_batch_impl(models, n, o, tables, results); });
}

}  // extern "C"
