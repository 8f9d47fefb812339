// BFS level expansion of one tile of frontier states, shared by the
// single-model kernel, the multi-model step kernel and the persistent batch
// kernel.
//
// One tile = up to 256 frontier states of one model:
//   frontier slot indices -> state rows staged in LDS -> guarded successor
//   enumeration by all lanes, compacted into an LDS ring -> hashing (one lane
//   per successor) -> find-or-put -> wave ballot/prefix compaction of the new
//   states into the next frontier, plus edge and deadlock counts.  Successors
//   never go to HBM except as the table's own inserts.
#pragma once

#include "internal.h"
#include "reach_internal.h"

namespace lhs {

constexpr int kExpandBlock = 256;
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

// Dynamic LDS of the expansion (32-bit words):
//   tile     [256][W|1]  frontier states of the current tile
//   queue    [kQueue]    enabled (state, process, transition) triples
//   succ_cnt [256]       successors per tile state (edges, deadlocks)
//   hq       [256] u64   hash of each successor of the current pass
//   d0, d1   [256]       successor descriptors of the pass
__host__ __device__ constexpr uint32_t expand_lds_words(uint32_t W) {
    return kExpandBlock * (W | 1u) + kQueue + kExpandBlock + 2 * kExpandBlock + 2 * kExpandBlock;
}

// Expand states front[base, base + rows) of one model (rows <= 256).  All
// 256 threads of the workgroup call it together.  Returns true (uniformly)
// if the level has been aborted, i.e. more than `limit` new states were
// appended to next[] (the cap); the tile then stops early.  Edges and
// deadlocks of a completed tile are added to lc (one atomic per wavefront),
// event counts to t.status.
//
// COHERENT: frontier indices and rows are read, and next[] is written, with
// agent-scope (cross-XCD coherent) accesses.  Needed when the previous level
// was produced inside the same launch by other workgroups (the persistent
// driver); across launches the kernel boundary already makes them visible.
template <int G, bool COHERENT = false>
__device__ __forceinline__ bool expand_tile(uint32_t *smem, const TableView &t, const ModelView &m,
                                            const uint32_t *__restrict__ front, uint64_t base,
                                            uint32_t rows, uint32_t *__restrict__ next,
                                            LevelCounters *lc, uint32_t limit) {
    constexpr uint32_t kBlock = kExpandBlock;
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
    const uint32_t tid = threadIdx.x, gi = tid / G;
    const bool leader = (tid & (G - 1)) == 0;
    const uint32_t PK = m.P * m.K;

    __syncthreads();   // the previous tile is fully consumed
    if (tid == 0) {
        s_tail = 0;
        s_abort = __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    succ_cnt[tid] = 0;
    if (tid < rows) {
        // rows of earlier levels were published before this level started
        const uint64_t slot = COHERENT ? ld_coherent(front + base + tid) : front[base + tid];
        const uint32_t *src = t.data + slot * W;
        uint32_t *dst = tile + tid * stride;
        if (COHERENT && (W & 1u) == 0) {
            const uint64_t *s2 = reinterpret_cast<const uint64_t *>(src);
            for (uint32_t i = 0; i < W; i += 2) {
                const uint64_t x = ld_coherent(s2 + (i >> 1));
                dst[i] = (uint32_t)x;
                dst[i + 1] = (uint32_t)(x >> 32);
            }
        } else if (COHERENT) {
            for (uint32_t i = 0; i < W; ++i)
                dst[i] = ld_coherent(src + i);
        } else if ((W & 3u) == 0) {
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
        return true;

    const uint32_t total_c = rows * PK;
    uint32_t c_pos = 0, head = 0, tail = 0;
    bool aborted = false;
    while (true) {
        // ---- enumerate guarded candidates into the LDS ring --------------
        while (c_pos < total_c && tail - head < kBlock) {
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
        // ---- one pass over up to 256 successors ---------------------------
        // (a) one lane per successor: decode and hash
        const uint32_t take = min(tail - head, kBlock);
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
        //     wavefront-cooperative memory accesses; G > 1: one group of G
        //     lanes each), then ballot/prefix compaction of the new ones into
        //     next[] with one atomic per wavefront
        for (uint32_t r = 0; r < G; ++r) {
            const uint32_t q = r * NG + gi;
            const bool active = q < take;
            const uint32_t o = active ? q : 0;
            const uint2 dsc = make_uint2(d0[o], d1[o]);
            uint32_t slot, code;
            if constexpr (G == 1) {
                __shared__ WaveScratch ws[kBlock / 64];
                find_or_put_wave<SuccVec>(t, &ws[tid / 64], smem, dsc, hq[o], active, slot, code, cnt);
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
                if (is_new) {
                    if (COHERENT)
                        st_coherent(next + wbase + mbcnt(nm), slot);
                    else
                        next[wbase + mbcnt(nm)] = slot;
                }
            }
        }
        head += take;
        __syncthreads();
        if (tid == 0)
            s_abort = __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __syncthreads();
        if (s_abort) {
            aborted = true;
            break;
        }
    }
    if (!aborted) {
        const uint32_t mine = tid < rows ? succ_cnt[tid] : 0u;
        const uint32_t e32 = wave_sum(mine), d32 = wave_sum(tid < rows && mine == 0);
        if (__lane_id() == 0) {
            if (e32)
                atomicAdd(&lc->edges, (unsigned long long)e32);
            if (d32)
                atomicAdd(&lc->deadlocks, (unsigned long long)d32);
        }
    }
    flush_counters(t.status, cnt);
    return aborted;
}

}  // namespace lhs
