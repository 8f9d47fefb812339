// Batched exploration of many models (reach_explore_batch).
//
// Every model keeps its own table region (slots, rows, two frontiers) and its
// own level counters; all models advance together, one BFS level per step.  A
// step expands the tiles of every unfinished model in the same launch, so
// small and large models, and models of different state widths, share the
// GPU.  Two drivers:
//   * persistent (default): one cooperative launch runs every step of every
//     model; workgroups meet at grid barriers between the expansion and the
//     per-model finalisation of a level;
//   * host loop (REACH_F_HOST_LOOP): one launch per step, the host reading
//     the per-model counters after each.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "expand_device.h"
#include "internal.h"
#include "reach_internal.h"

using namespace lhs;

namespace {

constexpr uint32_t kMaxBatch = 1024;   // models per call (tile prefix lives in LDS)
constexpr uint32_t kBarrierSpinLimit = 1u << 24;

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

// Full per-model state of the persistent driver (device memory).
struct ModelState {
    BatchSlot s;
    uint32_t *fr[2];
    uint64_t *levels;      // [max_levels]
    uint64_t total, edges, deadlocks, cap;
    uint32_t cur, n_levels, max_levels, done;
    uint32_t capped, overflow, pad0, pad1;
};

struct PersistState {
    uint32_t bar_count;
    uint32_t bar_gen;
    uint32_t error;
    uint32_t steps;
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
template <int G>
__global__ __launch_bounds__(kExpandBlock) void k_expand_multi(const BatchSlot *__restrict__ slots,
                                                               const uint32_t *__restrict__ begin,
                                                               uint32_t n_slots, uint32_t total_tiles) {
    extern __shared__ uint32_t smem[];
    for (uint32_t g = blockIdx.x; g < total_tiles; g += gridDim.x) {
        const BatchSlot &s = slots[find_slot_by_tile(begin, n_slots, g)];
        const uint64_t base = (uint64_t)(g - s.tile_begin) * kExpandBlock;
        const uint32_t rows = (uint32_t)min<uint64_t>(kExpandBlock, s.n_front - base);
        expand_tile<G>(smem, s.t, s.m, s.front, base, rows, s.next, s.lc, s.limit);
    }
}

__global__ void k_zero_levels(LevelCounters *lc, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        lc[i] = LevelCounters{0, 0, 0, 0};
}

// Insert each model's initial state (level 0): block b handles model b.
struct LdsRowB {
    const uint32_t *r;
    __device__ __forceinline__ uint32_t get(uint32_t i) const { return r[i]; }
};

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
        find_or_put<1>(s.t, v, h, active, slot, code, cnt);
        if (active)
            const_cast<uint32_t *>(s.front)[0] = slot;
    }
}

// Undo a discarded level of one model (see reach.hip).
__global__ void k_rollback_one(uint64_t *bucket, const uint32_t *next, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        bucket[next[i]] = 0;
}

// ---- persistent driver ----------------------------------------------------

// Grid-wide barrier (all workgroups are co-resident: cooperative launch).
// Agent-scope fences make every workgroup's writes of the phase visible to
// the others.  The wait is bounded: on timeout the error flag is set and
// every workgroup leaves at its next barrier.  Returns false on error.
__device__ bool grid_barrier(PersistState *ps, uint32_t nblocks) {
    __shared__ uint32_t s_ok;
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t gen = __hip_atomic_load(&ps->bar_gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t arrived = atomicAdd(&ps->bar_count, 1u) + 1u;
        if (arrived == nblocks) {
            __hip_atomic_store(&ps->bar_count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&ps->bar_gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            uint32_t spins = 0;
            while (__hip_atomic_load(&ps->bar_gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (++spins > kBarrierSpinLimit) {
                    atomicCAS(&ps->error, 0u, (uint32_t)LHS_ESTALL);
                    break;
                }
                __builtin_amdgcn_s_sleep(8);
            }
        }
        __threadfence();
        s_ok = __hip_atomic_load(&ps->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0u;
    }
    __syncthreads();
    return s_ok != 0;
}

// All levels of all models in one launch.  Per step:
//   (1) every workgroup computes the tile prefix over unfinished models
//       (in LDS); no tiles left -> done;
//   (2) workgroups take global tiles g = blockIdx.x, + gridDim.x, ...;
//   (3) barrier; model i is finalised by workgroup i mod gridDim.x (cap
//       rollback, level count, frontier swap, counter reset); barrier.
template <int G>
__global__ __launch_bounds__(kExpandBlock) void k_batch_persistent(ModelState *__restrict__ ms, uint32_t n,
                                                                   PersistState *ps, uint32_t max_steps) {
    extern __shared__ uint32_t smem[];
    __shared__ uint32_t s_begin[kMaxBatch + 1];
    __shared__ uint32_t s_part[kExpandBlock];
    const uint32_t tid = threadIdx.x;
    for (uint32_t step = 0; step < max_steps; ++step) {
        // (1) tile prefix: thread t sums the tiles of models t, t+256, ...
        //     (contiguous chunks so the scan gives model order)
        const uint32_t per = (n + kExpandBlock - 1) / kExpandBlock;
        uint32_t local = 0;
        for (uint32_t i = tid * per; i < min(n, (tid + 1) * per); ++i) {
            const uint32_t nf = ms[i].done ? 0u : ms[i].s.n_front;
            s_begin[i] = (nf + kExpandBlock - 1) / kExpandBlock;   // tiles, prefix below
            local += s_begin[i];
        }
        s_part[tid] = local;
        __syncthreads();
        if (tid == 0) {
            uint32_t acc = 0;
            for (uint32_t w = 0; w < kExpandBlock; ++w) {
                const uint32_t v = s_part[w];
                s_part[w] = acc;
                acc += v;
            }
            s_begin[n] = acc;
        }
        __syncthreads();
        {
            uint32_t acc = s_part[tid];
            for (uint32_t i = tid * per; i < min(n, (tid + 1) * per); ++i) {
                const uint32_t v = s_begin[i];
                s_begin[i] = acc;
                acc += v;
            }
        }
        __syncthreads();
        const uint32_t total = s_begin[n];
        if (total == 0)
            break;
        // (2) expansion
        for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
            const uint32_t i = find_slot_by_tile(s_begin, n, g);
            const BatchSlot s = ms[i].s;
            const uint64_t base = (uint64_t)(g - s_begin[i]) * kExpandBlock;
            const uint32_t rows = (uint32_t)min<uint64_t>(kExpandBlock, s.n_front - base);
            expand_tile<G>(smem, s.t, s.m, s.front, base, rows, s.next, s.lc, s.limit);
        }
        if (!grid_barrier(ps, gridDim.x))
            return;
        // (3) per-model finalisation of the level
        for (uint32_t i = blockIdx.x; i < n; i += gridDim.x) {
            ModelState &M = ms[i];
            if (M.done)
                continue;
            LevelCounters *lc = M.s.lc;
            const uint32_t n_next = lc->n_next;
            const bool over = M.cap && n_next > M.s.limit;
            if (over) {
                // discard the partial level: zero every slot it claimed
                for (uint32_t j = tid; j < n_next; j += kExpandBlock)
                    M.s.t.bucket[M.s.next[j]] = 0;
            }
            __syncthreads();
            if (tid == 0) {
                if (over) {
                    M.capped = 1;
                    M.done = 1;
                } else {
                    M.edges += lc->edges;
                    M.deadlocks += lc->deadlocks;
                    if (n_next == 0) {
                        M.done = 1;
                    } else if (M.n_levels == M.max_levels) {
                        M.overflow = 1;
                        M.done = 1;
                    } else {
                        M.levels[M.n_levels++] = n_next;
                        M.total += n_next;
                        M.cur ^= 1u;
                        M.s.front = M.fr[M.cur];
                        M.s.next = M.fr[M.cur ^ 1u];
                        M.s.n_front = n_next;
                        const uint64_t room = M.cap ? M.cap - M.total : 0xFFFFFFFFull;
                        M.s.limit = (uint32_t)min<uint64_t>(room, 0xFFFFFFFFull);
                    }
                }
                lc->n_next = 0;
                lc->abort = 0;
                lc->edges = 0;
                lc->deadlocks = 0;
            }
            __syncthreads();
        }
        if (tid == 0 && blockIdx.x == 0)
            ps->steps = step + 1;
        if (!grid_barrier(ps, gridDim.x))
            return;
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
    PersistState *d_ps = nullptr;
    uint64_t *d_levels = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    uint32_t max_W = 1;
    uint32_t tps = 0;

    // ---- set-up: tables, models, roots (outside the timed exploration) --
    for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
        BatchModel &b = bm[i];
        b.m = models[i];
        b.W = b.m->n_procs + b.m->n_shared;
        max_W = std::max(max_W, b.W);
        if (tables && tables[i]) {
            b.t = tables[i];
        } else {
            const uint64_t cap = opts.capacity ? opts.capacity : batch_auto_capacity(b.m);
            rc = lhs_create(cap, b.W, &b.t);
            b.own = rc == LHS_OK;
        }
        if (rc != LHS_OK)
            break;
        if (b.m->state_cap && b.m->state_cap >= b.t->capacity) {
            rc = LHS_EINVAL;
            break;
        }
        if (i == 0)
            tps = tps_expand(b.t);
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
        hipLaunchKernelGGL(k_insert_roots, dim3(n), dim3(64), 0, s, d_slots, d_roots, d_root_off, n);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            rc = LHS_EDEVICE;
    }
    const size_t lds = (size_t)expand_lds_words(max_W) * sizeof(uint32_t);

    // ---- exploration -------------------------------------------------------
    if (rc == LHS_OK && !host_loop) {
        std::vector<ModelState> hms(n);
        if (hipMalloc(&d_ms, n * sizeof(ModelState)) != hipSuccess ||
            hipMalloc(&d_ps, sizeof(PersistState)) != hipSuccess ||
            hipMalloc(&d_levels, (uint64_t)n * max_levels * sizeof(uint64_t)) != hipSuccess ||
            hipMemset(d_ps, 0, sizeof(PersistState)) != hipSuccess)
            rc = LHS_ENOMEM;
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            ModelState &M = hms[i];
            std::memset(&M, 0, sizeof(M));
            M.s = h_slots[i];
            M.fr[0] = bm[i].t->frontier[0];
            M.fr[1] = bm[i].t->frontier[1];
            M.levels = d_levels + (uint64_t)i * max_levels;
            M.total = 1;
            M.cap = bm[i].m->state_cap;
            M.max_levels = max_levels;
            M.n_levels = 1;
        }
        // level 0 count = 1 for every model
        std::vector<uint64_t> ones((uint64_t)n * max_levels, 0);
        for (uint32_t i = 0; i < n; ++i)
            ones[(uint64_t)i * max_levels] = 1;
        int dev = 0, ncu = 0, per_cu = 0;
        const void *fn = nullptr;
        switch (tps) {
        case 1: fn = (const void *)k_batch_persistent<1>; break;
        case 4: fn = (const void *)k_batch_persistent<4>; break;
        case 8: fn = (const void *)k_batch_persistent<8>; break;
        default: fn = (const void *)k_batch_persistent<16>; break;
        }
        if (rc == LHS_OK &&
            (hipMemcpy(d_ms, hms.data(), n * sizeof(ModelState), hipMemcpyHostToDevice) != hipSuccess ||
             hipMemcpy(d_levels, ones.data(), ones.size() * sizeof(uint64_t), hipMemcpyHostToDevice) !=
                 hipSuccess ||
             hipGetDevice(&dev) != hipSuccess ||
             hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
             hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kExpandBlock, lds) != hipSuccess ||
             per_cu < 1))
            rc = LHS_EDEVICE;
        if (rc == LHS_OK) {
            const uint32_t grid = (uint32_t)(ncu * per_cu);
            uint32_t max_steps = max_levels + 1;
            void *args[] = {&d_ms, &n, &d_ps, &max_steps};
            (void)hipEventRecord(e0, s);
            if (hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kExpandBlock), args, lds, s) != hipSuccess)
                rc = LHS_EDEVICE;
            (void)hipEventRecord(e1, s);
            if (rc == LHS_OK && hipStreamSynchronize(s) != hipSuccess)
                rc = LHS_EDEVICE;
        }
        PersistState ps{};
        DevStatus st{};
        if (rc == LHS_OK &&
            (hipMemcpy(&ps, d_ps, sizeof(ps), hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(&st, d_status, sizeof(st), hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(hms.data(), d_ms, n * sizeof(ModelState), hipMemcpyDeviceToHost) != hipSuccess ||
             hipMemcpy(ones.data(), d_levels, ones.size() * sizeof(uint64_t), hipMemcpyDeviceToHost) !=
                 hipSuccess))
            rc = LHS_EDEVICE;
        if (rc == LHS_OK && (ps.error || st.error))
            rc = (lhs_status)(ps.error ? ps.error : st.error);
        float ms = 0;
        if (rc == LHS_OK)
            (void)hipEventElapsedTime(&ms, e0, e1);
        for (uint32_t i = 0; i < n && rc == LHS_OK; ++i) {
            const ModelState &M = hms[i];
            if (M.overflow || !M.done) {
                rc = LHS_EINVAL;
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
            std::memcpy(r.level_counts, ones.data() + (uint64_t)i * max_levels, M.n_levels * sizeof(uint64_t));
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
            const uint32_t grid = std::min<uint32_t>(tiles, 1u << 16);
            if (hipMemcpyAsync(d_slots, h_slots, na * sizeof(BatchSlot), hipMemcpyHostToDevice, s) != hipSuccess ||
                hipMemcpyAsync(d_begin, h_begin, (na + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s) !=
                    hipSuccess) {
                rc = LHS_EDEVICE;
                break;
            }
            hipLaunchKernelGGL(k_zero_levels, dim3((na + 255) / 256), dim3(256), 0, s, d_lc, na);
            switch (tps) {
            case 1: hipLaunchKernelGGL(k_expand_multi<1>, dim3(grid), dim3(kExpandBlock), lds, s, d_slots, d_begin, na, tiles); break;
            case 4: hipLaunchKernelGGL(k_expand_multi<4>, dim3(grid), dim3(kExpandBlock), lds, s, d_slots, d_begin, na, tiles); break;
            case 8: hipLaunchKernelGGL(k_expand_multi<8>, dim3(grid), dim3(kExpandBlock), lds, s, d_slots, d_begin, na, tiles); break;
            default: hipLaunchKernelGGL(k_expand_multi<16>, dim3(grid), dim3(kExpandBlock), lds, s, d_slots, d_begin, na, tiles); break;
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
    (void)hipFree(d_ps);
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
