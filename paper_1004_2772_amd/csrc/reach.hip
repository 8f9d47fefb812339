// Level-synchronous reachability on the GPU (Algorithm 1 as BFS levels).
//
// One level = one launch of k_expand over the current frontier:
//   frontier slot indices -> state rows staged in LDS -> guarded successor
//   enumeration -> find-or-put of every successor -> wave ballot/prefix
//   compaction of the new ones into the next frontier, plus edge and deadlock
//   counts.  Successors are never written to HBM: only new states reach the
//   table's data array, as the table's own insert.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"
#include "reach_internal.h"

using namespace lhs;

namespace {

constexpr int kBlock = 256;
constexpr uint32_t kQueue = 512;   // LDS successor ring (2 passes of 256)

// Successor of an LDS row: row with s[p] = target and, if ew != NONE,
// s[ew] = ev (ew already offset by P).  Descriptor: x = row word offset from
// the LDS base | p << 16 | ew << 24 (0xFF = no effect), y = target | ev << 16.
struct SuccVec {
    const uint32_t *row;
    uint32_t p, target, ew, ev;
    __device__ __forceinline__ uint32_t get(uint32_t i) const {
        uint32_t x = row[i];
        x = i == p ? target : x;
        x = i == ew ? ev : x;
        return x;
    }
    __device__ __forceinline__ static SuccVec decode(const uint32_t *smem, uint2 d) {
        const uint32_t ew = d.x >> 24;
        return SuccVec{smem + (d.x & 0xFFFFu), (d.x >> 16) & 0xFFu, d.y & 0xFFFFu,
                       ew == 0xFFu ? 0xFFFFFFFFu : ew, d.y >> 16};
    }
};

// LDS layout of k_expand (32-bit words):
//   tile     [kBlock][W|1]  frontier states of the current tile
//   queue    [kQueue]       enabled (state, process, transition) triples
//   succ_cnt [kBlock]       successors per tile state (edges, deadlocks)
//   hq       [kBlock] u64   hash of each successor of the current pass
//   d0, d1   [kBlock]       packed successor descriptors of the pass
__host__ __device__ constexpr uint32_t expand_lds_words(uint32_t W) {
    return kBlock * (W | 1u) + kQueue + kBlock + 2 * kBlock + 2 * kBlock;
}

// Expand frontier[0, n_front) (one BFS level).  Requires blockDim.x == kBlock.
// limit: the level aborts once more than `limit` new states were appended.
template <int G>
__global__ __launch_bounds__(kBlock) void k_expand(TableView t, ModelView m,
                                                   const uint32_t *__restrict__ front,
                                                   uint32_t n_front, uint32_t *__restrict__ next,
                                                   LevelCounters *lc, uint32_t limit) {
    extern __shared__ uint32_t smem[];
    const uint32_t W = m.W, stride = W | 1u;
    uint32_t *tile = smem;
    uint32_t *queue = tile + kBlock * stride;
    uint32_t *succ_cnt = queue + kQueue;
    uint64_t *hq = reinterpret_cast<uint64_t *>(succ_cnt + kBlock);   // 8-byte aligned
    uint32_t *d0 = reinterpret_cast<uint32_t *>(hq + kBlock);
    uint32_t *d1 = d0 + kBlock;
    __shared__ uint32_t s_tail, s_abort;

    constexpr uint32_t NG = kBlock / G;
    LaneCounters cnt;
    unsigned long long my_edges = 0, my_dead = 0;
    const uint32_t tid = threadIdx.x, gi = tid / G;
    const bool leader = (tid & (G - 1)) == 0;
    const uint32_t PK = m.P * m.K;

    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < n_front;
         base += (uint64_t)gridDim.x * kBlock) {
        const uint32_t rows = (uint32_t)min<uint64_t>(kBlock, n_front - base);
        __syncthreads();   // previous tile fully consumed
        if (tid == 0) {
            s_tail = 0;
            s_abort = __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        succ_cnt[tid] = 0;
        if (tid < rows) {
            // rows of earlier levels were published by earlier launches
            const uint64_t slot = front[base + tid];
            const uint32_t *src = t.data + slot * W;
            uint32_t *dst = tile + tid * stride;
            if ((W & 3u) == 0) {
                const uint4 *s4 = reinterpret_cast<const uint4 *>(src);
                for (uint32_t i = 0; i < W; i += 4) {
                    const uint4 x = s4[i >> 2];
                    dst[i] = x.x;
                    dst[i + 1] = x.y;
                    dst[i + 2] = x.z;
                    dst[i + 3] = x.w;
                }
            } else {
                for (uint32_t i = 0; i < W; ++i)
                    dst[i] = src[i];
            }
        }
        __syncthreads();
        if (s_abort)
            break;

        const uint32_t total_c = rows * PK;
        uint32_t c_pos = 0, head = 0, tail = 0;
        while (true) {
            // ---- enumerate guarded candidates into the LDS ring ----------
            while (c_pos < total_c && tail - head < (uint32_t)kBlock) {
                const uint32_t c = c_pos + tid;
                bool en = false;
                uint32_t entry = 0;
                if (c < total_c) {
                    const uint32_t st = __umulhi(c, m.magic_PK);
                    const uint32_t j = c - st * PK;
                    const uint32_t p = m.K == 1 ? j : __umulhi(j, m.magic_K);
                    const uint32_t k = j - p * m.K;
                    const uint32_t *row = tile + st * stride;
                    const uint32_t local = row[p];
                    if (local < m.L) {
                        const uint2 tr = m.trans[((uint64_t)p * m.L + local) * m.K + k];
                        const uint32_t gvar = (tr.x >> 16) & 0xFFu;
                        en = gvar == 0xFFu || row[m.P + gvar] == (tr.y & 0xFFFFu);
                    }
                    if (en) {
                        atomicAdd(&succ_cnt[st], 1u);
                        entry = st | (p << 8) | (k << 16);
                    }
                }
                const uint64_t mask = __ballot(en);
                uint32_t wbase = 0;
                if (__lane_id() == 0 && mask)
                    wbase = atomicAdd(&s_tail, (uint32_t)__popcll(mask));
                wbase = __shfl(wbase, 0, 64);
                if (en)
                    queue[(wbase + mbcnt(mask)) & (kQueue - 1)] = entry;
                c_pos += kBlock;
                __syncthreads();
                tail = s_tail;
                __syncthreads();
            }
            if (tail == head)
                break;
            // ---- one pass over up to kBlock successors ---------------------
            // (a) one lane per successor: decode and hash
            const uint32_t take = min(tail - head, (uint32_t)kBlock);
            if (tid < take) {
                const uint32_t e = queue[(head + tid) & (kQueue - 1)];
                const uint32_t st = e & 0xFFu, p = (e >> 8) & 0xFFu, k = e >> 16;
                const uint32_t *row = tile + st * stride;
                const uint2 tr = m.trans[((uint64_t)p * m.L + row[p]) * m.K + k];
                const uint32_t evar = tr.x >> 24;
                const uint32_t ew = evar == 0xFFu ? 0xFFu : m.P + evar;
                const SuccVec v{row, p, tr.x & 0xFFFFu, ew == 0xFFu ? 0xFFFFFFFFu : ew, tr.y >> 16};
                hq[tid] = hash_vec(v, W, t.seed);
                d0[tid] = (st * stride) | (p << 16) | (ew << 24);
                d1[tid] = (tr.x & 0xFFFFu) | ((tr.y >> 16) << 16);
            }
            __syncthreads();
            // (b) find-or-put of every successor (G == 1: one lane each with
            //     wavefront-cooperative memory accesses; G > 1: one group of
            //     G lanes each), then ballot/prefix compaction of the new ones
            //     into next[]
            for (uint32_t r = 0; r < G; ++r) {
                const uint32_t q = r * NG + gi;
                const bool active = q < take;
                const uint32_t o = active ? q : 0;
                const uint2 dsc = make_uint2(d0[o], d1[o]);
                uint32_t slot, code;
                if constexpr (G == 1) {
                    __shared__ WaveScratch ws[kBlock / 64];
                    find_or_put_wave<SuccVec>(t, &ws[tid / 64], smem, dsc, hq[o], active, slot, code,
                                              cnt);
                } else {
                    find_or_put<G>(t, SuccVec::decode(smem, dsc), hq[o], active, slot, code, cnt);
                }
                const bool is_new = active && leader && code == kNew;
                const uint64_t nm = __ballot(is_new);
                if (nm) {
                    uint32_t wbase = 0;
                    const uint32_t wn = (uint32_t)__popcll(nm);
                    if (__lane_id() == 0) {
                        wbase = atomicAdd(&lc->n_next, wn);
                        if ((uint64_t)wbase + wn > limit)
                            __hip_atomic_store(&lc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    }
                    wbase = __shfl(wbase, 0, 64);
                    if (is_new)
                        next[wbase + mbcnt(nm)] = slot;
                }
            }
            head += take;
            __syncthreads();
            if (tid == 0)
                s_abort = __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __syncthreads();
            if (s_abort)
                break;
        }
        if (s_abort)
            break;
        if (tid < rows) {
            my_edges += succ_cnt[tid];
            my_dead += succ_cnt[tid] == 0;
        }
    }
    // ---- per-wave reduction of the level counters ----------------------
    const uint32_t e32 = wave_sum((uint32_t)my_edges), d32 = wave_sum((uint32_t)my_dead);
    if (__lane_id() == 0) {
        if (e32)
            atomicAdd(&lc->edges, (unsigned long long)e32);
        if (d32)
            atomicAdd(&lc->deadlocks, (unsigned long long)d32);
    }
    flush_counters(t.status, cnt);
}

// Undo the inserts of a discarded level: zero the slots listed in next[].
// Only slots claimed during that level are listed, and no earlier state's
// probe sequence runs through a slot claimed later, so the table is exactly
// the kept levels afterwards.
__global__ void k_rollback(uint64_t *bucket, const uint32_t *next, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        bucket[next[i]] = 0;
}

__global__ void k_zero_level(LevelCounters *lc) {
    lc->n_next = 0;
    lc->abort = 0;
    lc->edges = 0;
    lc->deadlocks = 0;
}

}  // namespace

namespace lhs {

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
    return v;
}

size_t expand_lds_bytes(uint32_t W) {
    return (size_t)expand_lds_words(W) * sizeof(uint32_t);
}

lhs_status launch_expand(lhs_table *t, const TableView &tv, const ModelView &mv, const uint32_t *front,
                         uint32_t n_front, uint32_t *next, LevelCounters *lc, uint32_t limit,
                         hipStream_t s) {
    const uint32_t blocks = (uint32_t)std::min<uint64_t>((n_front + kBlock - 1) / kBlock, 1u << 16);
    const size_t lds = expand_lds_bytes(mv.W);
    const dim3 grid(std::max(blocks, 1u)), block(kBlock);
    switch (tps_expand(t)) {
    case 1: hipLaunchKernelGGL(k_expand<1>, grid, block, lds, s, tv, mv, front, n_front, next, lc, limit); break;
    case 4: hipLaunchKernelGGL(k_expand<4>, grid, block, lds, s, tv, mv, front, n_front, next, lc, limit); break;
    case 8: hipLaunchKernelGGL(k_expand<8>, grid, block, lds, s, tv, mv, front, n_front, next, lc, limit); break;
    case 16: hipLaunchKernelGGL(k_expand<16>, grid, block, lds, s, tv, mv, front, n_front, next, lc, limit); break;
    default: return LHS_EINVAL;
    }
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status ensure_bfs_buffers(lhs_table *t) {
    if (t->frontier[0])
        return LHS_OK;
    if (hipMalloc(&t->frontier[0], t->capacity * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&t->frontier[1], t->capacity * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&t->level, sizeof(LevelCounters)) != hipSuccess ||
        hipHostMalloc(&t->level_host, sizeof(LevelCounters), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipFree(t->frontier[0]);
        (void)hipFree(t->frontier[1]);
        (void)hipFree(t->level);
        t->frontier[0] = t->frontier[1] = nullptr;
        t->level = nullptr;
        return LHS_ENOMEM;
    }
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

// Host-driven level loop on table t (already sized, W matching).
lhs_status explore_host_loop(lhs_table *t, const reach_model *m, const uint2 *d_trans,
                             uint32_t max_levels, hipStream_t s, reach_result *r,
                             uint32_t *d_init) {
    const ModelView mv = model_view(m, d_trans);
    const TableView tv = view(t);
    std::vector<uint64_t> levels;
    // s0 is level 0: insert it with the batched find-or-put; its slot is the
    // first frontier (the seen byte lands in the other frontier buffer).
    lhs_status rc = launch_find_or_put(t, d_init, 1, reinterpret_cast<uint8_t *>(t->frontier[1]),
                                       t->frontier[0], s);
    if (rc != LHS_OK)
        return rc;
    levels.push_back(1);
    uint64_t total = 1, edges = 0, dead = 0;
    uint32_t n_cur = 1, cur = 0;
    int capped = 0;
    while (true) {
        uint32_t limit = 0xFFFFFFFFu;
        if (m->state_cap)
            limit = (uint32_t)std::min<uint64_t>(m->state_cap - total, 0xFFFFFFFFull);
        hipLaunchKernelGGL(k_zero_level, dim3(1), dim3(1), 0, s, t->level);
        rc = launch_expand(t, tv, mv, t->frontier[cur], n_cur, t->frontier[cur ^ 1], t->level, limit, s);
        if (rc != LHS_OK)
            return rc;
        LHS_HIP(hipMemcpyAsync(t->level_host, t->level, sizeof(LevelCounters), hipMemcpyDeviceToHost, s));
        LHS_HIP(hipStreamSynchronize(s));
        DevStatus st;
        LHS_HIP(hipMemcpy(&st, t->status, sizeof(st), hipMemcpyDeviceToHost));
        if (st.error)
            return (lhs_status)st.error;
        const LevelCounters lc = *t->level_host;
        if (m->state_cap && lc.n_next > limit) {
            hipLaunchKernelGGL(k_rollback, dim3(std::min<uint32_t>((lc.n_next + 255) / 256, 4096)),
                               dim3(256), 0, s, t->bucket, t->frontier[cur ^ 1], lc.n_next);
            LHS_HIP(hipGetLastError());
            capped = 1;
            break;
        }
        edges += lc.edges;
        dead += lc.deadlocks;
        if (lc.n_next == 0)
            break;
        if (levels.size() >= max_levels)
            return LHS_EINVAL;
        levels.push_back(lc.n_next);
        total += lc.n_next;
        n_cur = lc.n_next;
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

}  // namespace lhs

extern "C" {

lhs_status reach_explore(const reach_model *m, const reach_opts *o, reach_result *r) {
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

    lhs_table *t = opts.table;
    bool own = false;
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
    std::vector<uint2> packed;
    pack_model(m, packed);
    uint2 *d_trans = nullptr;
    uint32_t *d_init = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    rc = ensure_bfs_buffers(t);
    if (rc == LHS_OK) {
        if (hipMalloc(&d_trans, packed.size() * sizeof(uint2)) != hipSuccess ||
            hipMalloc(&d_init, W * sizeof(uint32_t)) != hipSuccess ||
            hipMemcpy(d_trans, packed.data(), packed.size() * sizeof(uint2), hipMemcpyHostToDevice) !=
                hipSuccess ||
            hipMemcpy(d_init, m->init, W * sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess ||
            hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
            rc = LHS_EDEVICE;
    }
    if (rc == LHS_OK) {
        t->last_stream = s;
        rc = lhs_clear(t, s);
    }
    if (rc == LHS_OK) {
        (void)hipEventRecord(e0, s);
        rc = explore_host_loop(t, m, d_trans, max_levels, s, r, d_init);
        (void)hipEventRecord(e1, s);
        if (hipEventSynchronize(e1) == hipSuccess) {
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            r->gpu_ms = ms;
        }
        if (rc == LHS_OK) {
            DevStatus st;
            if (read_status(t, &st) == LHS_OK)
                r->wait_hits = st.wait_hits;
        }
    }
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    (void)hipFree(d_trans);
    (void)hipFree(d_init);
    if (own)
        lhs_destroy(t);
    if (rc != LHS_OK)
        reach_result_free(r);
    return rc;
}

void reach_result_free(reach_result *r) {
    if (!r)
        return;
    std::free(r->level_counts);
    r->level_counts = nullptr;
    r->n_levels = 0;
}

}  // extern "C"
