// BFS level expansion of one tile of frontier states, shared by the
// single-model kernel, the graph-driven level kernel, the multi-model step
// kernel, the persistent batch kernel, the order-free kernel and the
// persistent server.
//
// One tile = up to 256 frontier states of one model:
//   frontier slot indices -> state rows staged in LDS -> guarded successor
//   enumeration by all lanes, in passes of 256 successors -> hashing (one
//   lane per successor) -> equal successors of the pass merged in LDS ->
//   find-or-put -> wave ballot/prefix compaction of the new states into the
//   next frontier, plus edge and deadlock counts.  Successors never go to
//   HBM except as the table's own inserts.
#pragma once

#include "internal.h"
#include "reach_internal.h"

namespace lhs {

constexpr int kExpandBlock = 256;
constexpr uint32_t kQueue = 512;   // LDS successor ring (2 passes of 256)

// A next frontier appended in segments (single-model levels): kSegs
// segments of `size` entries at buf + k * size, with append cursors
// cur[k * kSegStride] (a 128-byte line each).
struct SegOut {
    uint32_t *buf;
    uint32_t *cur;
    uint32_t size;
    DevStatus *status;   // EFULL if the segments cannot take a flush
};

// The frontier such a level produced, as the next level reads it: n[k]
// entries in segment k, tiles[k] = tiles (of kExpandBlock entries, never
// across segments) in the segments before k.
struct SegFront {
    const uint32_t *buf;
    uint32_t size;
    uint32_t n[kSegs];
    uint32_t tiles[kSegs + 1];
};

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

// Dynamic LDS of the expansion (32-bit words), for state width W and a
// transition-table area of `tcap` entries:
//   tile     [256][W|1]  frontier states of the current tile
//   tr       [tcap] u64  the model's packed transitions (when they fit)
//   pick     [256]       the (state, enabled pair) of each successor of the
//                        current pass (P*K <= 64), in the mask area
//   dedup    [512]       the pass's successors by hash (G = 1), behind pick
//     (queue [kQueue]    enabled (state, process, transition) when P*K > 64,
//                        in the same words)
//   succ_cnt [256]       successors per tile state (edges, deadlocks)
//   hq       [256] u64   hash of each successor of the current pass  } G > 1
//   d0, d1   [256]       successor descriptors of the pass          } only
//   nbuf     [kNewBuf]   slots of new states, flushed to next[] in bulk
// With one lane per operation (G = 1) the lane that stages a successor also
// runs its find-or-put, so hash and descriptor stay in its registers; the
// layout then fits four workgroups of a 16-word model per CU.
constexpr uint32_t kNewBuf = 1536;
constexpr uint32_t kEagerRoom = 1u << 22;
constexpr uint32_t kMaskArea = 2 * kExpandBlock + 258;
static_assert(kQueue <= kMaskArea, "queue shares the mask area");
constexpr uint32_t kDedupCells = 512;   // twice the successors of a pass
static_assert(kExpandBlock + kDedupCells <= kMaskArea, "pick and the dedup cells share the mask area");
__host__ __device__ constexpr uint32_t expand_lds_words(uint32_t W, uint32_t tcap, uint32_t G) {
    return kExpandBlock * (W | 1u) + 2 * tcap + kMaskArea + kExpandBlock +
           (G > 1 ? 4 * kExpandBlock : 0u) + kNewBuf;
}

// Transitions that fit this many LDS entries are staged in LDS.
constexpr uint32_t kTransLdsMax = 2048;

// LDS entries to reserve for a model's transitions (0 = read from HBM).
__host__ __device__ inline uint32_t trans_lds_entries(uint32_t P, uint32_t L, uint32_t K) {
    const uint64_t n = (uint64_t)P * L * K;
    return n <= kTransLdsMax ? (uint32_t)n : 0u;
}

// Which model's transitions are currently staged in this workgroup's LDS
// (buffer and key).
static __shared__ const uint2 *s_trans_staged;
static __shared__ unsigned long long s_trans_key;
// Edge / deadlock counts accumulated over tiles (deferred mode).
static __shared__ unsigned long long s_acc_edges, s_acc_dead;
// New-state buffer fill, its reserved base in next[], and the level's abort
// / near-the-cap flags as this workgroup last saw them.
static __shared__ uint32_t s_nnew, s_nbase, s_abort, s_eager;
// New states appended to next[] since the caller last reset it.
static __shared__ uint32_t s_pushed;
// Set when a wait for a frontier entry ran out (AWAIT): the launch stops.
static __shared__ uint32_t s_stall;
// Exploration without level barriers: its count of open states, and how
// many of this workgroup's new states (s_pushed + s_nnew) it already holds.
static __shared__ unsigned long long *s_open;
static __shared__ uint32_t s_found;
// Segmented appends (SEG): this workgroup's estimate of the level's new
// states so far, and the pieces of the segments its current flush fills.
static __shared__ uint32_t s_seg_est, s_seg_np;
static __shared__ uint32_t s_seg_pos[2 * kSegs + 1], s_seg_off[2 * kSegs + 1];

// Call once at kernel start, before the first expand_tile.
__device__ __forceinline__ void expand_begin() {
    if (threadIdx.x == 0) {
        s_trans_staged = nullptr;
        s_trans_key = 0;
        s_acc_edges = 0;
        s_acc_dead = 0;
        s_nnew = 0;
        s_abort = 0;
        s_eager = 0;
        s_pushed = 0;
        s_stall = 0;
        s_seg_est = 0;
    }
}

// The new-state buffer in the expansion's LDS layout.
template <int G>
__device__ __forceinline__ uint32_t *expand_nbuf(uint32_t *smem, uint32_t W, uint32_t tcap) {
    return smem + expand_lds_words(W, tcap, G) - kNewBuf;
}

// Append the buffered new slots to next[] with one atomic on the level's
// cursor (block-wide, uniform call).  Flags the level aborted when the cursor
// passes `limit`; within kEagerRoom of it the workgroup turns eager (flushes
// every pass and rereads the abort flag).
// COUNT_OPEN (exploration without level barriers): new states that *s_open
// does not hold yet, those found in the current tile, are added to it before
// their entries are written.  A workgroup that expands one of them subtracts
// it only after it has read the entry, so the count never reaches zero while
// a tile that appended states is still running.
template <bool COHERENT, bool COUNT_OPEN = false>
__device__ __forceinline__ void flush_new_slots(const uint32_t *nbuf, uint32_t *next, LevelCounters *lc,
                                                uint32_t limit) {
    __syncthreads();
    const uint32_t tid = threadIdx.x;
    const uint32_t nn = s_nnew;
    if (tid == 0) {
        if (nn) {
            if constexpr (COUNT_OPEN) {
                const uint32_t held = s_pushed + nn;
                if (held > s_found) {
                    atomicAdd(s_open, (unsigned long long)(held - s_found));
                    s_found = held;
                    wait_vm_complete();   // counted before any entry is written
                }
            }
            const uint32_t b = atomicAdd(&lc->n_next, nn);
            s_nbase = b;
            s_pushed += nn;
            if ((uint64_t)b + nn > limit) {
                __hip_atomic_store(&lc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                s_abort = 1;
            } else if (limit != 0xFFFFFFFFu && (uint64_t)b + nn + kEagerRoom > limit) {
                s_eager = 1;
            }
        }
        if (s_eager && !s_abort)
            s_abort = __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (nn) {
        const uint32_t b = s_nbase;
        for (uint32_t i = tid; i < nn; i += kExpandBlock) {
            if (COHERENT)
                st_coherent(next + b + i, nbuf[i]);
            else
                next[b + i] = nbuf[i];
        }
        __syncthreads();
        if (tid == 0)
            s_nnew = 0;
        __syncthreads();
    }
}

// Segmented appends: the buffered new slots go to one of kSegs segments of
// the next frontier, each with its own append cursor on a line of its own,
// so that the workgroups of the GPU spread their cursor atomics over kSegs
// addresses (one atomic address saturates at a few million operations per
// second, and a level appends far more often).  A workgroup starts at the
// segment of its XCD (workgroups are dealt to the XCDs in turn); a flush
// that does not fit its segment takes the rest from the following ones.
// The level's exact count is only needed near the cap: this workgroup keeps
// an estimate from its cursor (the segments fill evenly), turns eager when
// the estimate comes within kEagerRoom of `limit`, and then sums the
// cursors after every flush to set the abort flag.  Block-wide, uniform.
template <bool COHERENT>
__device__ __forceinline__ void flush_new_slots_seg(const uint32_t *nbuf, const SegOut &so, LevelCounters *lc,
                                                    uint32_t limit) {
    __syncthreads();
    const uint32_t tid = threadIdx.x;
    const uint32_t nn = s_nnew;
    if (tid == 0) {
        if (nn) {
            uint32_t k = blockIdx.x & (kSegs - 1), rem = nn, np = 0, off = 0, first = 0;
            // every segment visited twice at most: a visited one that is
            // full stays full, and the segments hold every slot of the table
            for (uint32_t tries = 0; rem && tries < 2 * kSegs; ++tries) {
                const uint32_t b = atomicAdd(so.cur + k * kSegStride, rem);
                if (tries == 0)
                    first = b;
                if (b < so.size) {
                    const uint32_t n = min(rem, so.size - b);
                    s_seg_pos[np] = k * so.size + b;
                    s_seg_off[np] = off;
                    ++np;
                    off += n;
                    rem -= n;
                }
                k = (k + 1) & (kSegs - 1);
            }
            s_seg_off[np] = off;
            s_seg_np = np;
            if (rem)   // more new slots than the table has slots: cannot happen
                set_error(so.status, 3u /* LHS_EFULL */);
            s_pushed += nn;
            s_seg_est = max(s_seg_est, (uint32_t)min<uint64_t>((uint64_t)kSegs * ((uint64_t)first + nn), 0xFFFFFFFFull));
            if (limit != 0xFFFFFFFFu && ((uint64_t)s_seg_est + kEagerRoom > limit || s_eager)) {
                s_eager = 1;
                uint64_t total = 0;
                for (uint32_t q = 0; q < kSegs; ++q)
                    total += min(ld_coherent(so.cur + q * kSegStride), so.size);
                if (total > limit) {
                    __hip_atomic_store(&lc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_abort = 1;
                }
            }
        }
        if (s_eager && !s_abort)
            s_abort = __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (nn) {
        const uint32_t np = s_seg_np, placed = s_seg_off[np];
        for (uint32_t i = tid; i < placed; i += kExpandBlock) {
            uint32_t p = 0;
            while (p + 1 < np && i >= s_seg_off[p + 1])
                ++p;
            const uint32_t pos = s_seg_pos[p] + (i - s_seg_off[p]);
            if (COHERENT)
                st_coherent(so.buf + pos, nbuf[i]);
            else
                so.buf[pos] = nbuf[i];
        }
        __syncthreads();
        if (tid == 0)
            s_nnew = 0;
        __syncthreads();
    }
}

// Deferred mode: append the workgroup's remaining new states and add its
// accumulated edge/deadlock counts to lc.  Call by all threads after the
// last expand_tile of the launch (also after an aborted tile: every claimed
// slot must be listed in next[] for the rollback).
template <int G, bool COHERENT = false, bool SEG = false>
__device__ __forceinline__ void expand_end(uint32_t *smem, uint32_t W, uint32_t tcap, uint32_t *next,
                                           LevelCounters *lc, uint32_t limit, const SegOut &so = SegOut{}) {
    if constexpr (SEG)
        flush_new_slots_seg<COHERENT>(expand_nbuf<G>(smem, W, tcap), so, lc, limit);
    else
        flush_new_slots<COHERENT>(expand_nbuf<G>(smem, W, tcap), next, lc, limit);
    if (threadIdx.x == 0) {
        if (s_acc_edges)
            atomicAdd(&lc->edges, s_acc_edges);
        if (s_acc_dead)
            atomicAdd(&lc->deadlocks, s_acc_dead);
    }
}

// One packed transition: a plain load, or (CL) a coherent one for buffers
// rewritten while the kernel runs.
template <bool CL>
__device__ __forceinline__ uint2 ld_trans(const uint2 *p) {
    if constexpr (CL) {
        const uint64_t x = __hip_atomic_load(reinterpret_cast<const uint64_t *>(p), __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_SYSTEM);
        return make_uint2((uint32_t)x, (uint32_t)(x >> 32));
    } else {
        return *p;
    }
}

__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x) {
    const uint32_t lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(x, d, 64);
        if (lane >= (uint32_t)d)
            x += y;
    }
    return x;
}

// Expand states front[base, base + rows) of one model (rows <= 256).  All
// 256 threads of the workgroup call it together.  Returns true (uniformly)
// if the level has been aborted, i.e. more than `limit` new states were
// appended to next[] (the cap); the tile then stops early.  Edge and
// deadlock counts go to lc (see DEFER), event counts to t.status.  tcap = LDS entries reserved for transitions.
//
// Successor enumeration (P*K <= 64): every lane evaluates all guards of its
// own state into a 64-bit mask of enabled (process, transition) pairs, read
// from the LDS copy of the transition table; a block prefix sum over the mask
// popcounts numbers the tile's successors.  Before each pass of 256, every
// state lane writes its successors that fall in the pass, in bit order, to
// their places in an LDS list, and lane q of the pass takes entry q.  With
// one lane per operation, successors of a pass that are the same state are
// merged in an LDS hash set before the table is probed (interleavings of
// independent moves make such diamonds common among neighbouring frontier
// states), so each distinct state of a pass costs one find-or-put.  Wider
// models (P*K > 64) enumerate candidates 256 at a time into an LDS ring.
//
// New states are compacted into LDS and appended to next[] with one atomic
// per workgroup and flush: the level's append cursor is a single address that
// every workgroup of the GPU shares, and atomics on it serialise.  Far from
// the cap a workgroup flushes once per tile (or when its buffer of kNewBuf
// slots is nearly full).  Within kEagerRoom of the cap it flushes after every
// pass of 256 successors and rereads the abort flag, so a discarded level
// overshoots the cap by at most one pass per resident workgroup, as with
// per-pass appends.  kEagerRoom exceeds resident workgroups x kNewBuf, so the
// lazily buffered states cannot cross the cap unseen.
//
// COHERENT: frontier indices and rows are read, and next[] is written, with
// agent-scope (cross-XCD coherent) accesses.  Needed when the previous level
// was produced inside the same launch by other workgroups (the persistent
// driver); across launches the kernel boundary already makes them visible.
// DEFER: new states stay buffered across tiles (flushed when the buffer
// nears full) and edge/deadlock counts stay in LDS until expand_end
// (single-model launches, whose workgroups run many tiles of one level);
// otherwise both go out at the end of every tile.  DEFER_COUNTS alone keeps
// only the counts in LDS.
// AWAIT (with COHERENT): a frontier entry may still be in flight; 0xFFFFFFFF
// marks one not yet written, which the staging lane waits for (bounded:
// LHS_ESTALL and an aborted tile).  Appends in the middle of the tile count
// their states as open first (flush_new_slots, COUNT_OPEN).
// CL: slot lines are read with coherent loads (tables reused within one
// launch, the persistent server).
template <int G, uint32_t LS, bool COHERENT = false, bool DEFER = false, bool DEFER_COUNTS = DEFER,
          bool AWAIT = false, bool CL = false, bool SEG = false>
__device__ __forceinline__ bool expand_tile(uint32_t *smem, const TableView &t, const ModelView &m,
                                            const uint32_t *__restrict__ front, uint64_t base,
                                            uint32_t rows, uint32_t *__restrict__ next,
                                            LevelCounters *lc, uint32_t limit, uint32_t tcap,
                                            const SegOut &so = SegOut{}) {
    constexpr uint32_t kBlock = kExpandBlock;
    const uint32_t W = m.W, stride = W | 1u;
    uint32_t *tile = smem;
    uint2 *tr_lds = reinterpret_cast<uint2 *>(tile + kBlock * stride);
    uint64_t *masks = reinterpret_cast<uint64_t *>(tr_lds + tcap);
    uint32_t *queue = reinterpret_cast<uint32_t *>(masks);     // wide models only
    uint32_t *succ_cnt = reinterpret_cast<uint32_t *>(masks) + kMaskArea;
    uint64_t *hq = reinterpret_cast<uint64_t *>(succ_cnt + kBlock);   // 8-byte aligned (G > 1)
    uint32_t *d0 = reinterpret_cast<uint32_t *>(hq + kBlock);
    uint32_t *d1 = d0 + kBlock;
    uint32_t *nbuf = G > 1 ? d1 + kBlock : succ_cnt + kBlock;
    uint64_t my_h = 0;           // G == 1: this lane's successor of the pass
    uint32_t my_d0 = 0, my_d1 = 0;
    __shared__ uint32_t s_tail, s_wtot[kBlock / 64];
    __shared__ WaveScratch<LS> ws[kBlock / 64];

    constexpr uint32_t NG = kBlock / G;
    LaneCounters cnt;
    const uint32_t tid = threadIdx.x, gi = tid / G;
    const bool leader = (tid & (G - 1)) == 0;
    const uint32_t PK = m.P * m.K;
    const uint32_t PLK = m.P * m.L * m.K;
    const bool tr_in_lds = PLK <= tcap;

    __syncthreads();   // the previous tile is fully consumed
    const bool restage = tr_in_lds && (s_trans_staged != m.trans || s_trans_key != m.key);
    if (tid == 0) {
        s_tail = 0;
        s_abort = __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        // SEG: the level's count is this workgroup's estimate (the cursors
        // are read only near the cap)
        const uint32_t nn = SEG ? s_seg_est : __hip_atomic_load(&lc->n_next, __ATOMIC_RELAXED,
                                                                __HIP_MEMORY_SCOPE_AGENT);
        s_eager = limit != 0xFFFFFFFFu && (uint64_t)nn + kEagerRoom > limit;
    }
    if (restage)
        for (uint32_t i = tid; i < PLK; i += kBlock)
            tr_lds[i] = ld_trans<CL>(m.trans + i);
    succ_cnt[tid] = 0;
    bool staged = tid < rows;
    uint64_t slot = 0;
    if (staged) {
        // rows of earlier levels were published before this level started
        slot = COHERENT ? ld_coherent(front + base + tid) : front[base + tid];
        if constexpr (AWAIT) {
            for (uint32_t spins = 0; slot == 0xFFFFFFFFu; ++spins) {
                // give up on an aborted launch (the writer may have stopped)
                // or after the bound (then also an error)
                const bool out = spins >= kSpinLimit;
                if (out || ((spins & 63u) == 63u &&
                            __hip_atomic_load(&lc->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))) {
                    if (out)
                        set_error(t.status, 4u /* LHS_ESTALL */);
                    __hip_atomic_store(&lc->abort, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    s_stall = 1;
                    staged = false;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                slot = ld_coherent(front + base + tid);
            }
        }
    }
    // plain loads of rows of W = 4, 8, 16 or 32 words: the wavefront loads
    // its 64 rows together, W/4 lanes per row with one 16-byte piece each,
    // so one load instruction moves 64/(W/4) whole rows
    const bool coop = !COHERENT && (W == 4 || W == 8 || W == 16 || W == 32);
    if (coop) {
        const uint32_t lane = __lane_id(), wrow = tid - lane;    // the wave's first row
        const uint32_t cs = W == 4 ? 0u : (W == 8 ? 1u : (W == 16 ? 2u : 3u));   // log2(W/4)
        const uint32_t c = lane & ((1u << cs) - 1u);
        const uint32_t my_slot = (uint32_t)slot;
        for (uint32_t r0 = 0; r0 < 64; r0 += 64u >> cs) {
            const uint32_t r = r0 + (lane >> cs);
            const uint32_t rs = (uint32_t)__shfl((int)my_slot, (int)r, 64);
            if (wrow + r < rows) {
                const uint4 x = reinterpret_cast<const uint4 *>(t.data + (uint64_t)rs * W)[c];
                uint32_t *dst = tile + (wrow + r) * stride + 4 * c;
                dst[0] = x.x;
                dst[1] = x.y;
                dst[2] = x.z;
                dst[3] = x.w;
            }
        }
    } else if (staged) {
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
    // the LDS copy lives behind this model's tile rows: a tile that does not
    // stage its transitions may overwrite another model's copy with its rows
    // and masks, so it forgets that copy
    if ((restage || !tr_in_lds) && tid == 0) {
        s_trans_staged = tr_in_lds ? m.trans : nullptr;
        s_trans_key = m.key;
    }
    if (s_abort || s_stall)
        return true;
    const uint2 *tr = tr_in_lds ? tr_lds : m.trans;
    // transition idx (CL and not staged: read past the caches)
    auto trans_at = [&](uint64_t idx) -> uint2 {
        if constexpr (CL) {
            if (!tr_in_lds)
                return ld_trans<true>(m.trans + idx);
        }
        return tr[idx];
    };

    auto flush_new = [&]() {
        if constexpr (SEG)
            flush_new_slots_seg<COHERENT>(nbuf, so, lc, limit);
        else
            flush_new_slots<COHERENT, AWAIT>(nbuf, next, lc, limit);
    };
    // ---- find-or-put of successors d0/d1/hq[0, take); new slots to nbuf ----
    // skip (G == 1): this lane's successor is another lane's in the same pass
    auto fop_pass = [&](uint32_t take, bool skip) {
        for (uint32_t r = 0; r < G; ++r) {
            const uint32_t q = r * NG + gi;
            const bool active = q < take && !(G == 1 && skip);
            uint32_t slot, code;
            if constexpr (G == 1) {
                find_or_put_wave<LS, SuccVec, CL>(t, &ws[tid / 64], smem, make_uint2(my_d0, my_d1), my_h,
                                                  active, slot, code, cnt);
            } else {
                const uint32_t o = active ? q : 0;
                find_or_put<G, LS, SuccVec, CL>(t, SuccVec::decode(smem, make_uint2(d0[o], d1[o])), hq[o], active,
                                                slot, code, cnt);
            }
            const bool is_new = active && leader && code == kNew;
            if (t.parent && is_new) {
                // predecessor record: the frontier slot of the expanded row
                const uint32_t row_off = (G == 1 ? my_d0 : d0[q]) & 0xFFFFu;
                const uint32_t *src = front + base + row_off / stride;
                t.parent[slot] = COHERENT ? ld_coherent(src) : *src;
            }
            const uint64_t nm = __ballot(is_new);
            if (nm) {
                uint32_t wbase = 0;
                if (__lane_id() == 0)
                    wbase = atomicAdd(&s_nnew, (uint32_t)__popcll(nm));
                wbase = __shfl(wbase, 0, 64);
                if (is_new)
                    nbuf[wbase + mbcnt(nm)] = slot;
            }
        }
        __syncthreads();
        if (s_eager || s_nnew > kNewBuf - kBlock)
            flush_new();
        return s_abort != 0;
    };
    // successor (p, k) of tile row st
    auto succ_of = [&](uint32_t st, uint32_t p, uint32_t k) -> SuccVec {
        const uint32_t *row = tile + st * stride;
        const uint2 x = trans_at(((uint64_t)p * m.L + row[p]) * m.K + k);
        const uint32_t evar = x.x >> 24;
        return SuccVec{row, p, x.x & 0xFFFFu, evar == 0xFFu ? 0xFFFFFFFFu : m.P + evar, x.y >> 16};
    };
    // decode successor (st, p, k) into hq/d0/d1[i] (G > 1) or this lane's
    // registers (G == 1, i == tid)
    auto stage_successor = [&](uint32_t i, uint32_t st, const SuccVec &v) {
        const uint32_t ew = v.ew == 0xFFFFFFFFu ? 0xFFu : v.ew;
        const uint64_t h = hash_vec(v, W, t.seed);
        const uint32_t e0 = (st * stride) | (v.p << 16) | (ew << 24);
        const uint32_t e1 = v.target | (v.ev << 16);
        if constexpr (G == 1) {
            my_h = h;
            my_d0 = e0;
            my_d1 = e1;
        } else {
            hq[i] = h;
            d0[i] = e0;
            d1[i] = e1;
        }
    };

    bool aborted = false;
    if (PK <= 64) {
        // ---- enabled-transition masks, one lane per state ------------------
        uint64_t mask = 0;
        if (tid < rows) {
            const uint32_t *row = tile + tid * stride;
            for (uint32_t p = 0; p < m.P; ++p) {
                const uint32_t local = row[p];
                if (local >= m.L)
                    continue;
                const uint64_t tb = ((uint64_t)p * m.L + local) * m.K;
                for (uint32_t k = 0; k < m.K; ++k) {
                    const uint2 x = trans_at(tb + k);
                    const uint32_t gvar = (x.x >> 16) & 0xFFu;
                    const bool en = gvar == 0xFFu || row[m.P + gvar] == (x.y & 0xFFFFu);
                    mask |= (uint64_t)en << (p * m.K + k);
                }
            }
        }
        const uint32_t c = (uint32_t)__popcll(mask);
        succ_cnt[tid] = c;
        const uint32_t incl = wave_scan_incl(c);
        if (__lane_id() == 63)
            s_wtot[tid / 64] = incl;
        __syncthreads();
        uint32_t woff = 0, total = 0;
        for (uint32_t w = 0; w < kBlock / 64; ++w) {
            woff += w < tid / 64 ? s_wtot[w] : 0u;
            total += s_wtot[w];
        }
        // this state's successors are numbered [nextq, nextq + c) in the tile
        uint32_t nextq = woff + incl - c;
        uint64_t rem = mask;
        // ---- passes of 256 successors -------------------------------------
        // Every state lane writes the (state, enabled pair) of its successors
        // that fall in the pass into `pick` (the mask area); lane q of the
        // pass then stages successor s0 + q.
        uint32_t *pick = reinterpret_cast<uint32_t *>(masks);
        uint32_t *dedup = pick + kBlock;
        auto pick_succ = [&](uint32_t e) -> SuccVec {
            const uint32_t j = e & 0xFFu;
            const uint32_t p = m.K == 1 ? j : __umulhi(j, m.magic_K);
            return succ_of(e >> 8, p, j - p * m.K);
        };
        for (uint32_t s0 = 0; s0 < total && !aborted; s0 += kBlock) {
            const uint32_t take = min(total - s0, kBlock);
            while (rem && nextq < s0 + kBlock) {
                pick[nextq - s0] = (tid << 8) | (uint32_t)__builtin_ctzll(rem);
                rem &= rem - 1;
                ++nextq;
            }
            if constexpr (G == 1)
                for (uint32_t i = tid; i < kDedupCells; i += kBlock)
                    dedup[i] = 0;
            __syncthreads();
            bool skip = false;
            if (tid < take) {
                const uint32_t e = pick[tid];
                const SuccVec v = pick_succ(e);
                stage_successor(tid, e >> 8, v);
                if (G == 1 && !(t.flags & kNoMerge)) {
                    // Successors of one pass that are the same state (two
                    // interleavings reaching it) go to the table once.  Each
                    // lane claims a cell of an LDS hash set keyed by its
                    // hash; a lane that meets its own hash tag in a cell
                    // stops there, and takes that lane's find-or-put as its
                    // own once the full rows compare equal (a tag that
                    // belongs to another state leaves it on its own).  The
                    // lane that claimed the cell never skips.  (kNarrowTags
                    // keeps one tag bit, so that most tag matches are other
                    // states: a check of that path.)
                    const uint32_t tag = ((uint32_t)(my_h >> 41) << 9) &
                                         ((t.flags & kNarrowTags) ? 1u << 9 : ~0u);
                    uint32_t c = (uint32_t)(my_h >> 32) & (kDedupCells - 1), other = 0;
                    for (;;) {
                        const uint32_t old = atomicCAS(&dedup[c], 0u, tag | (tid + 1));
                        if (old == 0)
                            break;
                        if ((old & ~511u) == tag) {
                            other = old & 511u;
                            break;
                        }
                        c = (c + 1) & (kDedupCells - 1);
                    }
                    if (other) {
                        // one compare per lane, its words loaded independently
                        const SuccVec o = pick_succ(pick[other - 1]);
                        uint32_t diff = 0, w = 0;
                        for (; w + 4 <= W; w += 4)
                            diff |= (v.get(w) ^ o.get(w)) | (v.get(w + 1) ^ o.get(w + 1)) |
                                    (v.get(w + 2) ^ o.get(w + 2)) | (v.get(w + 3) ^ o.get(w + 3));
                        for (; w < W; ++w)
                            diff |= v.get(w) ^ o.get(w);
                        skip = diff == 0;
                        cnt.merged += skip;
                    }
                }
            }
            __syncthreads();
            aborted = fop_pass(take, skip);
        }
    } else {
        // ---- wide models: candidates 256 at a time into the LDS ring ------
        const uint32_t total_c = rows * PK;
        uint32_t c_pos = 0, head = 0, tail = 0;
        while (true) {
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
                        const uint2 x = trans_at(((uint64_t)p * m.L + local) * m.K + k);
                        const uint32_t gvar = (x.x >> 16) & 0xFFu;
                        en = gvar == 0xFFu || row[m.P + gvar] == (x.y & 0xFFFFu);
                    }
                    if (en) {
                        atomicAdd(&succ_cnt[st], 1u);
                        entry = st | (p << 8) | (k << 16);
                    }
                }
                const uint64_t msk = __ballot(en);
                uint32_t wbase = 0;
                if (__lane_id() == 0 && msk)
                    wbase = atomicAdd(&s_tail, (uint32_t)__popcll(msk));
                wbase = __shfl(wbase, 0, 64);
                if (en)
                    queue[(wbase + mbcnt(msk)) & (kQueue - 1)] = entry;
                c_pos += kBlock;
                __syncthreads();
                tail = s_tail;
                __syncthreads();
            }
            if (tail == head)
                break;
            const uint32_t take = min(tail - head, kBlock);
            if (tid < take) {
                const uint32_t e = queue[(head + tid) & (kQueue - 1)];
                stage_successor(tid, e & 0xFFu, succ_of(e & 0xFFu, (e >> 8) & 0xFFu, e >> 16));
            }
            __syncthreads();
            head += take;
            if (fop_pass(take, false)) {
                aborted = true;
                break;
            }
        }
    }
    // a workgroup that runs several tiles of one level keeps its buffer
    if constexpr (!DEFER)
        flush_new();
    // ---- edge and deadlock counts of the tile -------------------------------
    const uint32_t mine = tid < rows ? succ_cnt[tid] : 0u;
    const uint32_t e32 = wave_sum(mine), d32 = wave_sum(tid < rows && mine == 0);
    if (t.dead_rec && tid < rows && mine == 0) {
        const uint32_t k = atomicAdd(t.dead_rec, 1u);
        if (k < kDeadRecord)
            t.dead_rec[1 + k] = COHERENT ? ld_coherent(front + base + tid) : front[base + tid];
    }
    if (__lane_id() == 0) {
        atomicAdd(&s_acc_edges, (unsigned long long)e32);
        atomicAdd(&s_acc_dead, (unsigned long long)d32);
    }
    if constexpr (!DEFER_COUNTS) {
        __syncthreads();
        if (tid == 0) {
            if (s_acc_edges)
                atomicAdd(&lc->edges, s_acc_edges);
            if (s_acc_dead)
                atomicAdd(&lc->deadlocks, s_acc_dead);
            s_acc_edges = 0;
            s_acc_dead = 0;
        }
    }
    flush_counters(t, cnt);
    return s_abort != 0;
}

}  // namespace lhs
