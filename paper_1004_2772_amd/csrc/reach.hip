// Level-synchronous reachability on the GPU (Algorithm 1 as BFS levels) for
// one model: one launch of k_expand per level (tile body in expand_device.h),
// the host reading the level's counters after each launch.
#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "internal.h"
#include "reach_internal.h"
#include "expand_device.h"
#include "persistent.h"

using namespace lhs;

namespace {

// Tiles of a segmented frontier: every tile lies in one segment.
__host__ __device__ inline void seg_tiles(SegFront &f) {
    f.tiles[0] = 0;
    for (uint32_t k = 0; k < kSegs; ++k)
        f.tiles[k + 1] = f.tiles[k] + (f.n[k] + kExpandBlock - 1) / kExpandBlock;
}

__host__ __device__ inline uint64_t seg_total(const SegFront &f) {
    uint64_t n = 0;
    for (uint32_t k = 0; k < kSegs; ++k)
        n += f.n[k];
    return n;
}

// The frontier entries of tile `tile`: their address and count.
__device__ __forceinline__ const uint32_t *seg_tile(const SegFront &f, uint32_t tile, uint32_t &rows) {
    uint32_t t0 = f.tiles[0], nk = f.n[0];
    uint64_t at = 0;
#pragma unroll
    for (uint32_t q = 1; q < kSegs; ++q)
        if (tile >= f.tiles[q]) {
            t0 = f.tiles[q];
            nk = f.n[q];
            at = (uint64_t)q * f.size;
        }
    const uint32_t j = tile - t0;
    rows = min<uint32_t>(kExpandBlock, nk - j * kExpandBlock);
    return f.buf + at + (uint64_t)j * kExpandBlock;
}

// Expand one BFS level of one model: the frontier's tiles, new states
// appended to the segments of the next frontier.
template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock) void k_expand(TableView t, ModelView m, SegFront f, SegOut o,
                                                         LevelCounters *lc, uint32_t limit, uint32_t tcap) {
    extern __shared__ uint32_t smem[];
    expand_begin();
    const uint32_t n_tiles = f.tiles[kSegs];
    for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        uint32_t rows = 0;
        const uint32_t *front = seg_tile(f, tile, rows);
        if (expand_tile<G, LS, false, true, true, false, false, true>(smem, t, m, front, 0, rows, nullptr, lc,
                                                                      limit, tcap, o))
            break;
    }
    expand_end<G, false, true>(smem, m.W, tcap, nullptr, lc, limit, o);
}

// Undo the inserts of a discarded level: zero the slots listed in its
// segments.  Only slots claimed during that level are listed, and no earlier
// state's probe sequence runs through a slot claimed later, so the table is
// exactly the kept levels afterwards.
__device__ __forceinline__ void rollback_segments(uint64_t *bucket, const uint32_t *buf, uint32_t size,
                                                  const uint32_t *n) {
    for (uint32_t k = 0; k < kSegs; ++k)
        for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n[k]; i += gridDim.x * blockDim.x)
            bucket[buf[(uint64_t)k * size + i]] = 0;
}

__global__ void k_rollback(uint64_t *bucket, SegFront f) {
    rollback_segments(bucket, f.buf, f.size, f.n);
}

// ---- graph-driven levels (REACH_F_GRAPH) ----------------------------------
// One level = k_expand_graph, k_finalize_graph, k_rollback_graph, all reading
// the table's GraphCtx; once the exploration is done every kernel returns at
// once, so a replay may run past the last level.

template <int G, uint32_t LS>
__global__ __launch_bounds__(kExpandBlock) void k_expand_graph(const GraphCtx *ctx, uint32_t tcap) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_go, s_lim;
    __shared__ SegFront s_f;
    __shared__ SegOut s_o;
    if (threadIdx.x == 0) {
        s_go = !ctx->ctl.done;
        s_lim = ctx->ctl.limit;
        const uint32_t cur = ctx->ctl.cur;
        s_f.buf = ctx->fr[cur];
        s_f.size = ctx->seg_size;
        for (uint32_t k = 0; k < kSegs; ++k)
            s_f.n[k] = ctx->front_n[k];
        seg_tiles(s_f);
        s_o.buf = ctx->fr[cur ^ 1u];
        s_o.cur = ctx->segs;
        s_o.size = ctx->seg_size;
        s_o.status = ctx->t.status;
    }
    __syncthreads();
    if (!s_go)
        return;
    const TableView t = ctx->t;
    const ModelView m = ctx->m;
    const SegFront f = s_f;
    const SegOut o = s_o;
    LevelCounters *lc = ctx->lc;
    const uint32_t limit = s_lim;
    expand_begin();
    const uint32_t n_tiles = f.tiles[kSegs];
    for (uint32_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        uint32_t rows = 0;
        const uint32_t *front = seg_tile(f, tile, rows);
        if (expand_tile<G, LS, false, true, true, false, false, true>(smem, t, m, front, 0, rows, nullptr, lc,
                                                                      limit, tcap, o))
            break;
    }
    expand_end<G, false, true>(smem, m.W, tcap, nullptr, lc, limit, o);
}

// The host loop's per-level bookkeeping, on the device (one thread).
__global__ void k_finalize_graph(GraphCtx *ctx) {
    LevelCtl &c = ctx->ctl;
    LevelCounters *lc = ctx->lc;
    if (c.done) {
        c.rollback_n = 0;
        return;
    }
    uint32_t seg_n[kSegs];
    uint64_t next_total = 0;
    for (uint32_t k = 0; k < kSegs; ++k) {
        seg_n[k] = min(ctx->segs[k * kSegStride], ctx->seg_size);
        next_total += seg_n[k];
        ctx->segs[k * kSegStride] = 0;
    }
    const uint32_t n_next = (uint32_t)next_total;
    if (c.cap && n_next > c.limit) {
        c.rollback_n = n_next;      // k_rollback_graph discards the level
        for (uint32_t k = 0; k < kSegs; ++k)
            ctx->rb_n[k] = seg_n[k];
        c.capped = 1;
        c.done = 1;
    } else {
        c.edges += lc->edges;
        c.deadlocks += lc->deadlocks;
        if (n_next == 0) {
            c.done = 1;
        } else if (c.n_levels == c.max_levels) {
            c.overflow = 1;
            c.done = 1;
        } else {
            c.levels[c.n_levels++] = n_next;
            c.total += n_next;
            c.n_front = n_next;
            for (uint32_t k = 0; k < kSegs; ++k)
                ctx->front_n[k] = seg_n[k];
            c.cur ^= 1u;
            c.limit = c.cap ? (uint32_t)min<unsigned long long>(c.cap - c.total, 0xFFFFFFFFull) : 0xFFFFFFFFu;
        }
    }
    lc->n_next = 0;
    lc->abort = 0;
    lc->edges = 0;
    lc->deadlocks = 0;
}

__global__ void k_rollback_graph(const GraphCtx *ctx) {
    if (ctx->ctl.rollback_n)
        rollback_segments(ctx->t.bucket, ctx->fr[ctx->ctl.cur ^ 1u], ctx->seg_size, ctx->rb_n);
}

constexpr uint32_t kGraphLevels = 8;

// Start of a BFS with predecessor records: s0 is its own predecessor, no
// deadlock recorded yet.
__global__ void k_begin_parents(uint32_t *parent, const uint32_t *front, uint32_t *dead_rec) {
    parent[front[0]] = front[0];
    dead_rec[0] = 0;
}

// A level's counters, segment counts and the table's status to the host
// loop's pinned summary, then the counters and cursors cleared for the next
// level.
__global__ void k_level_done(LevelCounters *lc, uint32_t *segs, const DevStatus *st, LevelSummary *out) {
    if (threadIdx.x == 0) {
        out->lc = *lc;
        out->st = *st;
        *lc = LevelCounters{0, 0, 0, 0};
    }
    if (threadIdx.x < kSegs) {
        out->seg_n[threadIdx.x] = segs[threadIdx.x * kSegStride];
        segs[threadIdx.x * kSegStride] = 0;
    }
}

__global__ void k_zero_level(LevelCounters *lc, uint32_t *segs) {
    if (threadIdx.x == 0) {
        lc->n_next = 0;
        lc->abort = 0;
        lc->edges = 0;
        lc->deadlocks = 0;
    }
    if (threadIdx.x < kSegs)
        segs[threadIdx.x * kSegStride] = 0;
}

// ---- exploration without allocation (reach_explore_noalloc) ---------------
// Everything the level loop needs besides the caller's table lives in one
// file-scope device array, `scratch`, of a fixed size: the two frontiers of a
// table of at most LHS_NOALLOC_MAX_CAPACITY slots, the level counters, the
// root's seen byte, the initial state, and the model's transitions (as
// given, and packed by k_pack_trans).  Each device holds its own copy from
// module load until the process ends; host code reaches it only through the
// address hipGetSymbolAddress returned on that device.
constexpr size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr size_t kNaFront0 = 0;
constexpr size_t kNaFront1 = kNaFront0 + LHS_NOALLOC_MAX_CAPACITY * sizeof(uint32_t);
constexpr size_t kNaLevel = kNaFront1 + LHS_NOALLOC_MAX_CAPACITY * sizeof(uint32_t);
constexpr size_t kNaSegs = kNaLevel + align256(sizeof(LevelCounters));
constexpr size_t kNaSeen = kNaSegs + align256(kSegCursorBytes);
constexpr size_t kNaInit = kNaSeen + 256;
constexpr size_t kNaRaw = kNaInit + align256(32 * sizeof(uint32_t));
constexpr size_t kNaPacked = kNaRaw + align256(LHS_NOALLOC_MAX_TRANS * sizeof(reach_trans));
constexpr size_t kNaBytes = kNaPacked + LHS_NOALLOC_MAX_TRANS * sizeof(uint2);
static_assert(kNaBytes <= LHS_NOALLOC_SCRATCH_BYTES, "the header states the scratch size");
static_assert(sizeof(reach_trans) == 5 * sizeof(uint32_t), "transitions are five words");

static __device__ __align__(256) unsigned char scratch[kNaBytes];

constexpr int kNaMaxDevices = 64;
std::mutex g_na_mu;                    // serialises the calls (one scratch per device)
void *g_na_ptr[kNaMaxDevices] = {};    // device address of `scratch`, per device

// The host-side packing of the transition table (pack_model), on the
// device: x = target | guard_var << 16 | eff_var << 24 (0xFF = none),
// y = guard_val | eff_val << 16 (0 where the variable is none).
__global__ void k_pack_trans(const uint32_t *raw, uint2 *out, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const uint32_t *t = raw + 5ull * i;
        const bool g = t[1] != REACH_NONE, e = t[3] != REACH_NONE;
        out[i] = make_uint2(t[0] | ((g ? t[1] : 0xFFu) << 16) | ((e ? t[3] : 0xFFu) << 24),
                            (g ? t[2] : 0u) | ((e ? t[4] : 0u) << 16));
    }
}

}  // namespace

namespace lhs {

TableView bfs_view(lhs_table *t, bool parents) {
    TableView v = view(t);
    if (parents) {
        v.parent = t->parent;
        v.dead_rec = t->dead_rec;
    }
    return v;
}

lhs_status begin_parents(lhs_table *t, hipStream_t s) {
    hipLaunchKernelGGL(k_begin_parents, dim3(1), dim3(1), 0, s, t->parent, t->frontier[0], t->dead_rec);
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status validate_model(const reach_model *m) {
    if (!m || !m->trans || !m->init || m->n_procs == 0 || m->n_locals == 0 ||
        m->trans_per_local == 0 || m->trans_per_local > 16 || m->n_locals > 65535 ||
        m->n_shared > 254 || m->n_procs + m->n_shared > 32 || m->n_procs + m->n_shared < 1)
        return LHS_EINVAL;
    const uint64_t n = (uint64_t)m->n_procs * m->n_locals * m->trans_per_local;
    for (uint64_t i = 0; i < n; ++i) {
        const reach_trans &t = m->trans[i];
        if (t.target >= m->n_locals)
            return LHS_EINVAL;
        if (t.guard_var != REACH_NONE && (t.guard_var >= m->n_shared || t.guard_val > 0xFFFFu))
            return LHS_EINVAL;
        if (t.eff_var != REACH_NONE && (t.eff_var >= m->n_shared || t.eff_val > 0xFFFFu))
            return LHS_EINVAL;
    }
    return LHS_OK;
}

// Pack transitions: x = target | guard_var << 16 | eff_var << 24 (0xFF = none),
// y = guard_val | eff_val << 16.
void pack_model(const reach_model *m, std::vector<uint2> &out) {
    const uint64_t n = (uint64_t)m->n_procs * m->n_locals * m->trans_per_local;
    out.resize(n);
    for (uint64_t i = 0; i < n; ++i) {
        const reach_trans &t = m->trans[i];
        const uint32_t gv = t.guard_var == REACH_NONE ? 0xFFu : t.guard_var;
        const uint32_t ev = t.eff_var == REACH_NONE ? 0xFFu : t.eff_var;
        out[i].x = t.target | (gv << 16) | (ev << 24);
        out[i].y = (t.guard_var == REACH_NONE ? 0u : t.guard_val) |
                   ((t.eff_var == REACH_NONE ? 0u : t.eff_val) << 16);
    }
}

ModelView model_view(const reach_model *m, const uint2 *d_trans) {
    ModelView v;
    v.trans = d_trans;
    v.P = m->n_procs;
    v.L = m->n_locals;
    v.S = m->n_shared;
    v.K = m->trans_per_local;
    v.W = m->n_procs + m->n_shared;
    const uint32_t PK = v.P * v.K;
    v.magic_PK = PK == 1 ? 0u : (uint32_t)(((1ull << 32) + PK - 1) / PK);
    v.magic_K = v.K == 1 ? 0u : (uint32_t)(((1ull << 32) + v.K - 1) / v.K);
    v.pad = 0;
    v.key = 0;
    return v;
}

size_t expand_lds_bytes(uint32_t W, uint32_t tcap, uint32_t tps) {
    return (size_t)expand_lds_words(W, tcap, tps) * sizeof(uint32_t);
}

// The first frontier, s0 alone in segment 0 of buf; a frontier from the
// segment cursors a level left (host copy).
SegFront seg_root(const uint32_t *buf, uint32_t size) {
    SegFront f{};
    f.buf = buf;
    f.size = size;
    f.n[0] = 1;
    seg_tiles(f);
    return f;
}

SegFront seg_front(const uint32_t *buf, uint32_t size, const uint32_t *cursors, uint32_t stride) {
    SegFront f{};
    f.buf = buf;
    f.size = size;
    for (uint32_t k = 0; k < kSegs; ++k)
        f.n[k] = std::min(cursors[k * stride], size);
    seg_tiles(f);
    return f;
}

uint32_t seg_size(const lhs_table *t) { return (uint32_t)(t->capacity / kSegs); }

lhs_status launch_expand(lhs_table *t, const TableView &tv, const ModelView &mv, const SegFront &f,
                         const SegOut &o, LevelCounters *lc, uint32_t limit, hipStream_t s) {
    const uint64_t tiles = f.tiles[kSegs];
    const uint32_t tc = trans_lds_entries(mv.P, mv.L, mv.K);
    const size_t lds = expand_lds_bytes(mv.W, tc, tps_expand(t));
    const lhs_status rc = with_shape(tps_expand(t), t->line_slots, [&](auto G, auto L) {
        const void *fn = (const void *)k_expand<decltype(G)::value, decltype(L)::value>;
        // workgroups loop over tiles: as many as are resident at once, so that
        // each keeps its new-state buffer across many tiles
        int ncu = 0, per_cu = 0, dev = 0;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
            per_cu < 1)
            return LHS_EDEVICE;
        const uint32_t blocks = exploration_grid(t, std::min<uint64_t>(tiles, (uint64_t)ncu * per_cu));
        hipLaunchKernelGGL((k_expand<decltype(G)::value, decltype(L)::value>), dim3(blocks), dim3(kExpandBlock),
                           lds, s, tv, mv, f, o, lc, limit, tc);
        return LHS_OK;
    });
    if (rc != LHS_OK)
        return rc;
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status ensure_bfs_buffers(lhs_table *t) {
    if (t->frontier[0])
        return LHS_OK;
    if (hipMalloc(&t->frontier[0], t->capacity * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&t->frontier[1], t->capacity * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&t->level, 256 + kSegCursorBytes) != hipSuccess ||
        hipHostMalloc(&t->level_host, sizeof(LevelSummary), hipHostMallocMapped) != hipSuccess ||
        hipHostGetDevicePointer(&t->summary_dev, t->level_host, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(t->frontier[0]);
        (void)hipFree(t->frontier[1]);
        (void)hipFree(t->level);
        if (t->level_host)
            (void)hipHostFree(t->level_host);
        t->frontier[0] = t->frontier[1] = nullptr;
        t->level = nullptr;
        t->level_host = nullptr;
        return LHS_ENOMEM;
    }
    t->segs = reinterpret_cast<uint32_t *>(reinterpret_cast<char *>(t->level) + 256);
    LevelSummary *sum = reinterpret_cast<LevelSummary *>(t->level_host);
    t->seg_n_host = sum->seg_n;
    t->status_host = &sum->st;
    return LHS_OK;
}

uint64_t auto_capacity(const reach_model *m) {
    if (!m->state_cap)
        return 1ull << 24;
    uint64_t want = 2 * m->state_cap + (1ull << 16), c = 1024;
    while (c < want && c < (1ull << 32))
        c <<= 1;
    return c;
}

// A frontier of n entries stored densely from buf, as segments.
SegFront seg_dense(const uint32_t *buf, uint32_t size, uint64_t n) {
    SegFront f{};
    f.buf = buf;
    f.size = size;
    for (uint32_t k = 0; k < kSegs; ++k) {
        const uint64_t from = (uint64_t)k * size;
        f.n[k] = n > from ? (uint32_t)std::min<uint64_t>(n - from, size) : 0u;
    }
    seg_tiles(f);
    return f;
}

// Host-driven level loop on table t (already sized, W matching); with a
// prefix area, the first (small) levels run in one persistent launch.
lhs_status explore_host_loop(lhs_table *t, const reach_model *m, const uint2 *d_trans,
                             uint32_t max_levels, hipStream_t s, reach_result *r,
                             uint32_t *d_init, bool parents, PrefixArea *d_pre, PrefixArea *h_pre) {
    const ModelView mv = model_view(m, d_trans);
    const TableView tv = bfs_view(t, parents);
    std::vector<uint64_t> levels;
    // s0 is level 0: insert it with the batched find-or-put; its slot is the
    // first frontier (the seen byte lands in the other frontier buffer).
    lhs_status rc = launch_find_or_put(t, d_init, 1, reinterpret_cast<uint8_t *>(t->frontier[1]),
                                       t->frontier[0], s);
    if (rc != LHS_OK)
        return rc;
    if (parents && (rc = begin_parents(t, s)) != LHS_OK)
        return rc;
    levels.push_back(1);
    uint64_t total = 1, edges = 0, dead = 0;
    uint32_t cur = 0;
    const uint32_t size = seg_size(t);
    SegFront f = seg_root(t->frontier[0], size);
    int capped = 0;
    hipLaunchKernelGGL(k_zero_level, dim3(1), dim3(64), 0, s, t->level, t->segs);
    bool finished = false;
    if (d_pre) {
        PrefixOut pre;
        rc = explore_prefix(t, tv, mv, m->state_cap, d_pre, h_pre, s, pre);
        if (rc != LHS_OK)
            return rc;
        levels.insert(levels.end(), pre.levels.begin(), pre.levels.end());
        if (levels.size() > max_levels)
            return LHS_EINVAL;
        total = pre.total;
        edges = pre.edges;
        dead = pre.deadlocks;
        capped = pre.capped;
        cur = pre.cur;
        finished = !pre.handed;
        f = seg_dense(t->frontier[cur], size, levels.back());
    }
    while (!finished) {
        uint32_t limit = 0xFFFFFFFFu;
        if (m->state_cap)
            limit = (uint32_t)std::min<uint64_t>(m->state_cap - total, 0xFFFFFFFFull);
        const SegOut o{t->frontier[cur ^ 1], t->segs, size, t->status};
        rc = launch_expand(t, tv, mv, f, o, t->level, limit, s);
        if (rc != LHS_OK)
            return rc;
        // the level's summary lands in pinned memory (and the counters are
        // cleared for the next level) in one small launch
        hipLaunchKernelGGL(k_level_done, dim3(1), dim3(64), 0, s, t->level, t->segs, (const DevStatus *)t->status,
                           static_cast<LevelSummary *>(t->summary_dev));
        LHS_HIP(hipStreamSynchronize(s));
        if (t->status_host->error)
            return (lhs_status)t->status_host->error;
        const LevelCounters lc = *t->level_host;
        const SegFront next = seg_front(t->frontier[cur ^ 1], size, t->seg_n_host, 1);
        const uint64_t n_next = seg_total(next);
        if (m->state_cap && n_next > limit) {
            hipLaunchKernelGGL(k_rollback, dim3((uint32_t)std::min<uint64_t>((n_next + 255) / 256, 4096)),
                               dim3(256), 0, s, t->bucket, next);
            LHS_HIP(hipGetLastError());
            capped = 1;
            break;
        }
        edges += lc.edges;
        dead += lc.deadlocks;
        if (n_next == 0)
            break;
        if (levels.size() >= max_levels)
            return LHS_EINVAL;
        levels.push_back(n_next);
        total += n_next;
        f = next;
        cur ^= 1;
    }
    LHS_HIP(hipStreamSynchronize(s));
    r->total_states = total;
    r->edges = edges;
    r->deadlocks = dead;
    r->capped = capped;
    r->n_levels = (uint32_t)levels.size();
    r->level_counts = (uint64_t *)std::malloc(levels.size() * sizeof(uint64_t));
    if (!r->level_counts)
        return LHS_ENOMEM;
    std::memcpy(r->level_counts, levels.data(), levels.size() * sizeof(uint64_t));
    return LHS_OK;
}

// Graph-driven level loop (REACH_F_GRAPH) on table t: the levels run from a
// captured graph of kGraphLevels levels, replayed until the device-side
// level record says done.  h_ctx is pinned host memory for the record.
lhs_status explore_graph(lhs_table *t, const reach_model *m, const uint2 *d_trans, uint32_t max_levels,
                         hipStream_t s, reach_result *r, uint32_t *d_init, GraphCtx *h_ctx, bool parents) {
    if (!t->gctx && hipMalloc(&t->gctx, sizeof(GraphCtx)) != hipSuccess) {
        (void)hipGetLastError();
        t->gctx = nullptr;
        return LHS_ENOMEM;
    }
    if (t->glevels_cap < max_levels) {
        (void)hipFree(t->glevels);
        t->glevels_cap = 0;
        if (hipMalloc(&t->glevels, (size_t)max_levels * sizeof(unsigned long long)) != hipSuccess) {
            (void)hipGetLastError();
            t->glevels = nullptr;
            return LHS_ENOMEM;
        }
        t->glevels_cap = max_levels;
    }
    if (!t->gstream && hipStreamCreateWithFlags(&t->gstream, hipStreamNonBlocking) != hipSuccess)
        return LHS_EDEVICE;
    GraphCtx *d_ctx = static_cast<GraphCtx *>(t->gctx);
    const uint32_t tcap = trans_lds_entries(m->n_procs, m->n_locals, m->trans_per_local);
    const uint32_t W = m->n_procs + m->n_shared;

    // level 0 and the level record
    lhs_status rc = launch_find_or_put(t, d_init, 1, reinterpret_cast<uint8_t *>(t->frontier[1]),
                                       t->frontier[0], s);
    if (rc != LHS_OK)
        return rc;
    if (parents && (rc = begin_parents(t, s)) != LHS_OK)
        return rc;
    hipLaunchKernelGGL(k_zero_level, dim3(1), dim3(64), 0, s, t->level, t->segs);
    GraphCtx &h = *h_ctx;
    std::memset(&h, 0, sizeof(h));
    h.segs = t->segs;
    h.seg_size = seg_size(t);
    h.front_n[0] = 1;
    h.t = bfs_view(t, parents);
    h.m = model_view(m, d_trans);
    h.fr[0] = t->frontier[0];
    h.fr[1] = t->frontier[1];
    h.lc = t->level;
    h.ctl.total = 1;
    h.ctl.cap = m->state_cap;
    h.ctl.levels = t->glevels;
    h.ctl.n_front = 1;
    h.ctl.limit = m->state_cap ? (uint32_t)std::min<uint64_t>(m->state_cap - 1, 0xFFFFFFFFull) : 0xFFFFFFFFu;
    h.ctl.n_levels = 1;
    h.ctl.max_levels = max_levels;
    LHS_HIP(hipMemcpyAsync(d_ctx, &h, sizeof(h), hipMemcpyHostToDevice, s));

    // the captured graph depends on the table, its lanes per state, the LDS
    // layout (W is the table's) and the worker cap
    const uint32_t tps = tps_expand(t);
    const uint64_t key = ((uint64_t)t->workers << 32) | (tcap * 32u + tps);
    if (!t->gexec || t->gexec_tcap != key) {
        if (t->gexec) {
            (void)hipGraphExecDestroy(t->gexec);
            t->gexec = nullptr;
        }
        const size_t lds = expand_lds_bytes(W, tcap, tps);
        hipGraph_t g = nullptr;
        rc = with_shape(tps, t->line_slots, [&](auto G, auto L) {
            const void *fn = (const void *)k_expand_graph<decltype(G)::value, decltype(L)::value>;
            int ncu = 0, per_cu = 0, dev = 0;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
                hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
                per_cu < 1)
                return LHS_EDEVICE;
            if (hipStreamBeginCapture(t->gstream, hipStreamCaptureModeThreadLocal) != hipSuccess)
                return LHS_EDEVICE;
            for (uint32_t k = 0; k < kGraphLevels; ++k) {
                hipLaunchKernelGGL((k_expand_graph<decltype(G)::value, decltype(L)::value>),
                                   dim3(exploration_grid(t, (uint64_t)ncu * per_cu)), dim3(kExpandBlock), lds,
                                   t->gstream,
                                   (const GraphCtx *)d_ctx, tcap);
                hipLaunchKernelGGL(k_finalize_graph, dim3(1), dim3(1), 0, t->gstream, d_ctx);
                hipLaunchKernelGGL(k_rollback_graph, dim3((uint32_t)ncu * 4), dim3(256), 0, t->gstream,
                                   (const GraphCtx *)d_ctx);
            }
            const bool ok = hipStreamEndCapture(t->gstream, &g) == hipSuccess && g;
            return ok ? LHS_OK : LHS_EDEVICE;
        });
        if (rc == LHS_OK && hipGraphInstantiate(&t->gexec, g, nullptr, nullptr, 0) != hipSuccess) {
            t->gexec = nullptr;
            rc = LHS_EDEVICE;
        }
        if (g)
            (void)hipGraphDestroy(g);
        if (rc != LHS_OK) {
            (void)hipGetLastError();
            return rc;
        }
        t->gexec_tcap = key;
    }

    // replay until done; the host waits once per replay
    const uint64_t max_replays = (uint64_t)max_levels / kGraphLevels + 2;
    for (uint64_t rep = 0;; ++rep) {
        if (rep == max_replays)
            return LHS_EDEVICE;
        LHS_HIP(hipGraphLaunch(t->gexec, s));
        LHS_HIP(hipMemcpyAsync(&h.ctl, &d_ctx->ctl, sizeof(LevelCtl), hipMemcpyDeviceToHost, s));
        LHS_HIP(hipMemcpyAsync(t->status_host, t->status, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
        LHS_HIP(hipStreamSynchronize(s));
        if (t->status_host->error)
            return (lhs_status)t->status_host->error;
        if (h.ctl.done)
            break;
    }
    if (h.ctl.overflow)
        return LHS_EINVAL;
    r->total_states = h.ctl.total;
    r->edges = h.ctl.edges;
    r->deadlocks = h.ctl.deadlocks;
    r->capped = (int32_t)h.ctl.capped;
    r->n_levels = h.ctl.n_levels;
    r->level_counts = (uint64_t *)std::malloc(h.ctl.n_levels * sizeof(uint64_t));
    if (!r->level_counts)
        return LHS_ENOMEM;
    r->level_counts[0] = 1;
    if (h.ctl.n_levels > 1)
        LHS_HIP(hipMemcpy(r->level_counts + 1, t->glevels + 1, (h.ctl.n_levels - 1) * sizeof(uint64_t),
                          hipMemcpyDeviceToHost));
    return LHS_OK;
}

}  // namespace lhs

extern "C" {

static lhs_status reach_explore_impl(const reach_model *m, const reach_opts *o, reach_result *r) {
    if (!r)
        return LHS_EINVAL;
    std::memset(r, 0, sizeof(*r));
    lhs_status rc = validate_model(m);
    if (rc != LHS_OK)
        return rc;
    const uint32_t W = m->n_procs + m->n_shared;
    reach_opts opts{};
    if (o)
        opts = *o;
    const uint32_t max_levels = opts.max_levels ? opts.max_levels : (1u << 20);
    hipStream_t s = (hipStream_t)opts.hip_stream;
    const bool parents = (opts.flags & REACH_F_PARENTS) != 0;
    const bool async = (opts.flags & REACH_F_ASYNC) != 0;
    if (async && (opts.flags & REACH_F_GRAPH))
        return LHS_EINVAL;   // no levels to capture

    // host-side packing first: nothing to undo if it throws
    std::vector<uint2> packed;
    pack_model(m, packed);
    lhs_table *t = opts.table;
    bool own = false;
    if (parents && !t)
        return LHS_EINVAL;   // the records live in the caller's table
    if (t) {
        if (t->W != W)
            return LHS_EINVAL;
    } else {
        const uint64_t cap = opts.capacity ? opts.capacity : auto_capacity(m);
        rc = lhs_create(cap, W, &t);
        if (rc != LHS_OK)
            return rc;
        own = true;
    }
    if (m->state_cap && m->state_cap >= t->capacity) {
        if (own)
            lhs_destroy(t);
        return LHS_EINVAL;
    }
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        if (own)
            lhs_destroy(t);
        return LHS_EDEVICE;
    }
    // model upload through the device's workspace: one copy, no allocation
    Carve c;
    const size_t o_trans = c.take<uint2>(packed.size()), o_init = c.take<uint32_t>(W);
    const size_t upload = c.off, o_ctx = c.take<GraphCtx>(1), o_actl = c.take<AsyncCtl>(1),
                 o_pre = c.take<PrefixArea>(1);
    Workspace &ws = workspace(dev);
    std::unique_lock<std::mutex> lock(ws.mu);
    rc = ensure_bfs_buffers(t);
    if (rc == LHS_OK && parents && !t->parent &&
        (hipMalloc(&t->parent, t->capacity * sizeof(uint32_t)) != hipSuccess ||
         hipMalloc(&t->dead_rec, (1 + kDeadRecord) * sizeof(uint32_t)) != hipSuccess)) {
        (void)hipGetLastError();
        (void)hipFree(t->parent);
        t->parent = nullptr;
        rc = LHS_ENOMEM;
    }
    if (rc == LHS_OK)
        rc = ws_reserve(ws, c.off, c.off);
    uint2 *d_trans = at<uint2>(ws.dev, o_trans);
    uint32_t *d_init = at<uint32_t>(ws.dev, o_init);
    if (rc == LHS_OK) {
        std::memcpy(at<void>(ws.host, o_trans), packed.data(), packed.size() * sizeof(uint2));
        std::memcpy(at<void>(ws.host, o_init), m->init, W * sizeof(uint32_t));
        if (hipMemcpyAsync(ws.dev, ws.host, upload, hipMemcpyHostToDevice, s) != hipSuccess)
            rc = LHS_EDEVICE;
    }
    if (rc == LHS_OK) {
        t->last_stream = s;
        rc = lhs_clear(t, s);
    }
    if (rc == LHS_OK) {
        (void)hipEventRecord(ws.ev[0], s);
        if (async)
            rc = explore_async(t, m, d_trans, s, r, d_init, at<AsyncCtl>(ws.dev, o_actl),
                               at<AsyncCtl>(ws.host, o_actl), parents);
        else if (opts.flags & REACH_F_GRAPH)
            rc = explore_graph(t, m, d_trans, max_levels, s, r, d_init, at<GraphCtx>(ws.host, o_ctx), parents);
        else
            rc = explore_host_loop(t, m, d_trans, max_levels, s, r, d_init, parents, at<PrefixArea>(ws.dev, o_pre),
                                   at<PrefixArea>(ws.host, o_pre));
        (void)hipEventRecord(ws.ev[1], s);
        if (hipEventSynchronize(ws.ev[1]) == hipSuccess) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, ws.ev[0], ws.ev[1]);
            r->gpu_ms = ms;
        }
        if (rc == LHS_OK) {
            DevStatus st;
            if (read_status(t, &st) == LHS_OK)
                r->wait_hits = st.wait_hits;
        }
    }
    t->has_parents = parents && rc == LHS_OK;
    if (hipStreamSynchronize(s) != hipSuccess && rc == LHS_OK)
        rc = LHS_EDEVICE;
    lock.unlock();
    if (own)
        lhs_destroy(t);
    if (rc != LHS_OK)
        reach_result_free(r);
    return rc;
}

lhs_status reach_explore(const reach_model *m, const reach_opts *o, reach_result *r) {
    return lhs::guard([&] { return reach_explore_impl(m, o, r); });
}

static lhs_status reach_trace_impl(lhs_table *t, uint32_t slot, uint32_t *h_path, uint32_t *h_rows, uint32_t max_len,
                                   uint32_t *len) {
    if (!t || !len || !t->has_parents || slot >= t->capacity)
        return LHS_EINVAL;
    if (hipStreamSynchronize(t->last_stream) != hipSuccess)
        return LHS_EDEVICE;
    uint64_t word = 0;
    LHS_HIP(hipMemcpy(&word, t->bucket + slot, sizeof(word), hipMemcpyDeviceToHost));
    if ((word >> 62) != 3u)
        return LHS_EINVAL;   // no stored state in this slot
    // walk the predecessor records back to s0 (its own predecessor)
    std::vector<uint32_t> rev{slot};
    for (uint64_t hops = 0;; ++hops) {
        if (hops > t->capacity)
            return LHS_EDEVICE;   // not a chain to s0
        uint32_t p = 0;
        LHS_HIP(hipMemcpy(&p, t->parent + rev.back(), sizeof(p), hipMemcpyDeviceToHost));
        if (p == rev.back())
            break;
        if (p >= t->capacity)
            return LHS_EDEVICE;
        rev.push_back(p);
    }
    *len = (uint32_t)rev.size();
    if (rev.size() > max_len)
        return (h_path || h_rows) ? LHS_EINVAL : LHS_OK;
    for (size_t i = 0; i < rev.size(); ++i) {
        const uint32_t sl = rev[rev.size() - 1 - i];
        if (h_path)
            h_path[i] = sl;
        if (h_rows)
            LHS_HIP(hipMemcpy(h_rows + i * t->W, t->data + (uint64_t)sl * t->W, t->W * sizeof(uint32_t),
                              hipMemcpyDeviceToHost));
    }
    return LHS_OK;
}

lhs_status reach_trace(lhs_table *t, uint32_t slot, uint32_t *h_path, uint32_t *h_rows, uint32_t max_len,
                       uint32_t *len) {
    return lhs::guard([&] { return reach_trace_impl(t, slot, h_path, h_rows, max_len, len); });
}

lhs_status reach_deadlock_slots(lhs_table *t, uint32_t *h_slots, uint32_t max, uint32_t *n) {
    if (!t || !n || !t->has_parents)
        return LHS_EINVAL;
    if (hipStreamSynchronize(t->last_stream) != hipSuccess)
        return LHS_EDEVICE;
    uint32_t count = 0;
    LHS_HIP(hipMemcpy(&count, t->dead_rec, sizeof(count), hipMemcpyDeviceToHost));
    const uint32_t kept = std::min(count, kDeadRecord);
    *n = count;
    const uint32_t k = std::min(kept, max);
    if (h_slots && k)
        LHS_HIP(hipMemcpy(h_slots, t->dead_rec + 1, k * sizeof(uint32_t), hipMemcpyDeviceToHost));
    return LHS_OK;
}

static lhs_status reach_explore_noalloc_impl(const reach_model *m, lhs_table *t, uint64_t *h_level_counts,
                                             uint32_t max_levels, reach_result *r, void *hip_stream) {
    if (!r)
        return LHS_EINVAL;
    std::memset(r, 0, sizeof(*r));
    if (!t || !h_level_counts || max_levels == 0 || validate_model(m) != LHS_OK)
        return LHS_EINVAL;
    const uint32_t W = m->n_procs + m->n_shared;
    const uint64_t n_trans = (uint64_t)m->n_procs * m->n_locals * m->trans_per_local;
    if (t->W != W || (m->state_cap && m->state_cap >= t->capacity))
        return LHS_EINVAL;
    if (t->capacity > LHS_NOALLOC_MAX_CAPACITY || n_trans > LHS_NOALLOC_MAX_TRANS)
        return LHS_EBUDGET;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess)
        return LHS_EDEVICE;
    if (dev != t->device || dev < 0 || dev >= kNaMaxDevices)
        return LHS_EINVAL;
    std::lock_guard<std::mutex> lock(g_na_mu);
    if (!g_na_ptr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
            return LHS_EDEVICE;
        g_na_ptr[dev] = p;
    }
    char *base = static_cast<char *>(g_na_ptr[dev]);
    uint32_t *fr[2] = {reinterpret_cast<uint32_t *>(base + kNaFront0), reinterpret_cast<uint32_t *>(base + kNaFront1)};
    LevelCounters *lc = reinterpret_cast<LevelCounters *>(base + kNaLevel);
    uint32_t *segs = reinterpret_cast<uint32_t *>(base + kNaSegs);
    uint8_t *seen = reinterpret_cast<uint8_t *>(base + kNaSeen);
    uint32_t *d_init = reinterpret_cast<uint32_t *>(base + kNaInit);
    uint32_t *raw = reinterpret_cast<uint32_t *>(base + kNaRaw);
    uint2 *d_trans = reinterpret_cast<uint2 *>(base + kNaPacked);
    hipStream_t s = (hipStream_t)hip_stream;
    const auto t0 = std::chrono::steady_clock::now();

    // model and initial state, then level 0
    LHS_HIP(hipMemcpyAsync(raw, m->trans, n_trans * sizeof(reach_trans), hipMemcpyHostToDevice, s));
    LHS_HIP(hipMemcpyAsync(d_init, m->init, W * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_pack_trans, dim3((uint32_t)std::min<uint64_t>((n_trans + 255) / 256, 256)), dim3(256),
                       0, s, raw, d_trans, (uint32_t)n_trans);
    LHS_HIP(hipGetLastError());
    t->last_stream = s;
    lhs_status rc = lhs_clear(t, s);
    if (rc != LHS_OK)
        return rc;
    if ((rc = launch_find_or_put(t, d_init, 1, seen, fr[0], s)) != LHS_OK)
        return rc;
    const ModelView mv = model_view(m, d_trans);
    const TableView tv = bfs_view(t, false);
    h_level_counts[0] = 1;
    uint32_t n_levels = 1, cur = 0;
    uint64_t total = 1, edges = 0, dead = 0;
    const uint32_t size = seg_size(t);
    SegFront f = seg_root(fr[0], size);
    int capped = 0;
    LevelCounters h_lc{};
    uint32_t h_segs[kSegs * kSegStride];
    DevStatus h_st{};
    while (true) {
        const uint32_t limit =
            m->state_cap ? (uint32_t)std::min<uint64_t>(m->state_cap - total, 0xFFFFFFFFull) : 0xFFFFFFFFu;
        hipLaunchKernelGGL(k_zero_level, dim3(1), dim3(64), 0, s, lc, segs);
        const SegOut o{fr[cur ^ 1], segs, size, t->status};
        if ((rc = launch_expand(t, tv, mv, f, o, lc, limit, s)) != LHS_OK)
            return rc;
        LHS_HIP(hipMemcpyAsync(&h_lc, lc, sizeof(h_lc), hipMemcpyDeviceToHost, s));
        LHS_HIP(hipMemcpyAsync(h_segs, segs, kSegCursorBytes, hipMemcpyDeviceToHost, s));
        LHS_HIP(hipMemcpyAsync(&h_st, t->status, sizeof(h_st), hipMemcpyDeviceToHost, s));
        LHS_HIP(hipStreamSynchronize(s));
        if (h_st.error)
            return (lhs_status)h_st.error;
        const SegFront next = seg_front(fr[cur ^ 1], size, h_segs, kSegStride);
        const uint64_t n_next = seg_total(next);
        if (m->state_cap && n_next > limit) {
            // discard the level: zero the slots it claimed
            hipLaunchKernelGGL(k_rollback, dim3((uint32_t)std::min<uint64_t>((n_next + 255) / 256, 4096)),
                               dim3(256), 0, s, t->bucket, next);
            LHS_HIP(hipGetLastError());
            capped = 1;
            break;
        }
        edges += h_lc.edges;
        dead += h_lc.deadlocks;
        if (n_next == 0)
            break;
        if (n_levels == max_levels)
            return LHS_EINVAL;   // more levels than the caller's array holds
        h_level_counts[n_levels++] = n_next;
        total += n_next;
        f = next;
        cur ^= 1;
    }
    LHS_HIP(hipMemcpyAsync(&h_st, t->status, sizeof(h_st), hipMemcpyDeviceToHost, s));
    LHS_HIP(hipStreamSynchronize(s));
    r->total_states = total;
    r->edges = edges;
    r->deadlocks = dead;
    r->capped = capped;
    r->n_levels = n_levels;
    r->level_counts = nullptr;
    r->wait_hits = h_st.wait_hits;
    r->gpu_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return LHS_OK;
}

lhs_status reach_explore_noalloc(const reach_model *m, lhs_table *t, uint64_t *h_level_counts, uint32_t max_levels,
                                 reach_result *r, void *hip_stream) {
    return lhs::guard([&] { return reach_explore_noalloc_impl(m, t, h_level_counts, max_levels, r, hip_stream); });
}

void reach_result_free(reach_result *r) {
    if (!r)
        return;
    std::free(r->level_counts);
    r->level_counts = nullptr;
    r->n_levels = 0;
}

}  // extern "C"
