// Device-side core of the lockless table: slot encoding, the vector hash and
// find-or-put (Algorithm 3 with walking-the-line, Algorithm 4) executed by a
// group of G cooperating lanes per operation.
//
// Slot (64 bits): 0 = empty; bit 63 OCC = claimed; bit 62 DONE = the vector
// has been written to the data array; bits 61..0 = memoised hash (the low 62
// bits of h1).  A slot goes empty -> claimed(memo) -> done(memo) and never
// changes again (figure "State diagram of buckets"): a slot seen non-empty
// keeps its memo forever, which is what makes a stale snapshot of a line safe.
//
// Memory ordering on gfx950 (8 XCDs, one L2 each).  The paper's requirement
// (section on the algorithm's memory-model needs): the vector must not be
// written before its slot is claimed, and a reader that sees DONE must see
// the whole vector.  Here:
//  * the claim is a 64-bit agent-scope CAS; the row is written only by the
//    winner, after the CAS returned (control dependency);
//  * row words are written and read with agent-scope atomic accesses, which
//    are coherent across the XCDs' L2 caches (no write-back or invalidate of
//    whole caches is needed for them);
//  * the publisher waits for its row stores to complete (vmcnt(0)) before
//    storing DONE; a reader issues its row loads only after its load of the
//    slot returned DONE.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lhs {

constexpr uint64_t kOcc = 1ull << 63;
constexpr uint64_t kDone = 1ull << 62;
constexpr uint64_t kMemoMask = kDone - 1;
constexpr uint32_t kLineSlots = 16;          // default line: 128 bytes of 8-byte slots
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kSpinLimit = 1u << 22;    // bound on one wait (ESTALL)

enum : uint32_t { kNew = 0, kSeen = 1, kFull = 2, kStall = 3 };

// Counters and sticky error kept in device memory per table.
struct DevStatus {
    uint32_t error;          // first device error (lhs_status), 0 = none
    uint32_t pad;
    unsigned long long wait_hits;
    unsigned long long cas_failures;
    unsigned long long lines;   // lines probed (only while counted, see TableView::flags)
    unsigned long long merged;  // successors merged into an equal one of their pass (counted)
};

// TableView::flags: counters to keep, and how expansions merge equal
// successors of a pass (expand_tile)
enum : uint32_t { kCountLines = 1, kCountMerged = 2, kNoMerge = 4, kNarrowTags = 8 };

// Per-lane event counts, reduced per wavefront before touching DevStatus.
struct LaneCounters {
    uint32_t waits = 0;
    uint32_t cas_failures = 0;
    uint32_t lines = 0;
    uint32_t merged = 0;
};

// Probe sequence across lines (after the home line's walk).
enum : uint32_t { kProbeDouble = 0, kProbeLinear = 1, kProbeQuadratic = 2 };

struct TableView {
    uint64_t *bucket;
    uint32_t *data;
    uint64_t seed;
    uint32_t W;
    uint32_t line_mask;      // lines - 1
    uint32_t max_rounds;     // lines probed before EFULL
    uint32_t probe;          // kProbe*
    DevStatus *status;
    // BFS with predecessor records (else null): parent[slot] = the slot the
    // state was first generated from; dead_rec = [count, slots of the first
    // kDeadRecord deadlock states expanded]
    uint32_t *parent;
    uint32_t *dead_rec;
    uint32_t flags;          // kCount*, kNoMerge, kNarrowTags
};
constexpr uint32_t kDeadRecord = 1024;

// log2 of the line width in slots (8, 16 or 32).
template <uint32_t LS>
__host__ __device__ constexpr uint32_t line_shift() {
    static_assert(LS == 8 || LS == 16 || LS == 32, "line slots");
    return LS == 8 ? 3u : (LS == 16 ? 4u : 5u);
}

// Line-to-line step of a vector's probe sequence.  Double hashing: a
// constant odd step from the hash's high half; linear: the next line;
// quadratic: the k-th move goes k lines on (the lines visited are line0 +
// k(k+1)/2).  On 2^n lines each sequence visits every line once in its first
// 2^n rounds.
__device__ __forceinline__ uint32_t probe_step(uint64_t h, uint32_t probe) {
    return probe == kProbeLinear ? 1u : ((uint32_t)(h >> 32) | 1u);
}
__device__ __forceinline__ uint32_t next_line(uint32_t line, uint32_t rounds_done, uint32_t step,
                                              uint32_t probe, uint32_t line_mask) {
    return (line + (probe == kProbeQuadratic ? rounds_done : step)) & line_mask;
}

__device__ __forceinline__ uint32_t mbcnt(uint64_t mask) {
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// ---- coherent (agent-scope) accesses --------------------------------------
__device__ __forceinline__ uint64_t ld_coherent(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_coherent(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long ld_coherent(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coherent(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Wait until this wavefront's outstanding vector memory operations completed
// (s_waitcnt vmcnt(0)); the signal fences keep the compiler from moving
// memory accesses across it.
__device__ __forceinline__ void wait_vm_complete() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0x0F70);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}
// 16 bytes of a slot line: a plain load, or (CL) two coherent 8-byte loads,
// for callers whose tables may have been emptied while they run (another
// XCD's cache can still hold the line as it was before).
template <bool CL>
__device__ __forceinline__ uint4 ld_line16(const uint4 *p) {
    if constexpr (CL) {
        const uint64_t *q = reinterpret_cast<const uint64_t *>(p);
        const uint64_t a = ld_coherent(q), b = ld_coherent(q + 1);
        return make_uint4((uint32_t)a, (uint32_t)(a >> 32), (uint32_t)b, (uint32_t)(b >> 32));
    } else {
        return *p;
    }
}

// Compiler-level acquire after observing DONE (the hardware already orders
// the dependent loads after the observed load).
__device__ __forceinline__ void after_done_observed() {
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
}

__device__ __forceinline__ uint64_t rotl64(uint64_t x, int r) {
    return (x << r) | (x >> (64 - r));
}

// 64-bit vector hash: MurmurHash3 x64 block mixing over 64-bit pairs of
// words, closed by its fmix64 finaliser (A. Appleby, MurmurHash3, public
// domain).  `Vec` provides get(i) for word i.
template <class Vec>
__device__ __forceinline__ uint64_t hash_vec(const Vec &v, uint32_t W, uint64_t seed) {
    const uint64_t c1 = 0x87c37b91114253d5ull, c2 = 0x4cf5ad432745937full;
    uint64_t h = seed;
    uint32_t i = 0;
    for (; i + 1 < W; i += 2) {
        uint64_t k = (uint64_t)v.get(i) | ((uint64_t)v.get(i + 1) << 32);
        k *= c1;
        k = rotl64(k, 31);
        k *= c2;
        h ^= k;
        h = rotl64(h, 27);
        h = h * 5 + 0x52dce729ull;
    }
    if (i < W) {
        uint64_t k = v.get(i);
        k *= c1;
        k = rotl64(k, 31);
        k *= c2;
        h ^= k;
    }
    h ^= (uint64_t)W * 4u;
    h ^= h >> 33;
    h *= 0xff51afd7ed558ccdull;
    h ^= h >> 33;
    h *= 0xc4ceb9fe1a85ec53ull;
    h ^= h >> 33;
    return h;
}

__device__ __forceinline__ void set_error(DevStatus *st, uint32_t code) {
    atomicCAS(&st->error, 0u, code);
}

// rotate an LS-bit mask right by r (bit k of the result = bit (k + r) mod LS)
template <uint32_t LS>
__device__ __forceinline__ uint32_t rotr_line(uint32_t m, uint32_t r) {
    if constexpr (LS == 32)
        return __builtin_rotateright32(m, r);
    else
        return ((m >> r) | (m << (LS - r))) & ((1u << LS) - 1u);
}

// Spread the low 16 bits of x so that bit i lands on bit 2i.
__device__ __forceinline__ uint32_t spread2(uint32_t x) {
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    return (x | (x << 1)) & 0x55555555u;
}

// Lane geometry of a group of G consecutive lanes of a wavefront.
template <int G>
struct Group {
    uint32_t sub, gbase;
    __device__ __forceinline__ Group() {
        const uint32_t lane = __lane_id();
        sub = lane & (G - 1);
        gbase = lane - sub;
    }
    __device__ __forceinline__ bool leader() const { return sub == 0; }
    // this group's G bits of a wavefront ballot
    __device__ __forceinline__ uint32_t bits(uint64_t ballot) const {
        return (uint32_t)(ballot >> gbase) & (uint32_t)((1ull << G) - 1);
    }
    __device__ __forceinline__ bool all(bool x) const {
        if constexpr (G == 1)
            return x;
        return bits(__ballot(x)) == (uint32_t)((1ull << G) - 1);
    }
    __device__ __forceinline__ uint64_t from_leader(uint64_t v) const {
        if constexpr (G == 1)
            return v;
        const uint32_t lo = __shfl((uint32_t)v, (int)gbase, 64);
        const uint32_t hi = __shfl((uint32_t)(v >> 32), (int)gbase, 64);
        return ((uint64_t)hi << 32) | lo;
    }
};

// Snapshot of one line of LS slots: masks of empty slots and of slots whose
// memo equals `memo` (any status), bit i = slot i of the line.  The line is
// LS/2 16-byte chunks (two slots each); lane `sub` of a group of G loads
// chunks sub, sub + G, ..., so every load instruction of the group covers one
// contiguous 16*G-byte segment of the line.  With G >= LS every lane below
// LS loads one slot and the others only take part in the ballots.
template <int G, uint32_t LS, bool CL = false>
__device__ __forceinline__ void line_masks(const Group<G> &g, const uint64_t *line_ptr, uint64_t memo,
                                           uint32_t &empty, uint32_t &match) {
    constexpr uint32_t SPL = LS / G;
    uint32_t e = 0, m = 0;
    if constexpr (SPL <= 1) {
        const bool own = (uint32_t)G == LS || g.sub < LS;
        const uint64_t s0 = own ? (CL ? ld_coherent(line_ptr + g.sub) : line_ptr[g.sub]) : ~0ull;
        constexpr uint32_t lm = LS == 32 ? 0xFFFFFFFFu : (1u << LS) - 1u;
        e = g.bits(__ballot(own && s0 == 0)) & lm;
        m = g.bits(__ballot(own && (s0 & ~kDone) == memo)) & lm;
    } else {
        constexpr uint32_t Q = SPL / 2;          // chunks per lane
        const uint4 *p = reinterpret_cast<const uint4 *>(line_ptr);
        uint4 x[Q];
#pragma unroll
        for (uint32_t q = 0; q < Q; ++q)
            x[q] = ld_line16<CL>(p + q * G + g.sub);
#pragma unroll
        for (uint32_t q = 0; q < Q; ++q) {
            const uint64_t s0 = ((uint64_t)x[q].y << 32) | x[q].x;
            const uint64_t s1 = ((uint64_t)x[q].w << 32) | x[q].z;
            if constexpr (G == 1) {
                e |= ((uint32_t)(s0 == 0) | ((uint32_t)(s1 == 0) << 1)) << (2 * q);
                m |= ((uint32_t)((s0 & ~kDone) == memo) | ((uint32_t)((s1 & ~kDone) == memo) << 1))
                     << (2 * q);
            } else {
                // chunk q*G + sub holds slots 2(q*G + sub) and 2(q*G + sub) + 1
                e |= spread2(g.bits(__ballot(s0 == 0))) << (2 * q * G);
                e |= spread2(g.bits(__ballot(s1 == 0))) << (2 * q * G + 1);
                m |= spread2(g.bits(__ballot((s0 & ~kDone) == memo))) << (2 * q * G);
                m |= spread2(g.bits(__ballot((s1 & ~kDone) == memo))) << (2 * q * G + 1);
            }
        }
    }
    empty = e;
    match = m;
}

// Row write by the group: 64-bit coherent stores when W is even (rows are
// 8-byte aligned), 32-bit otherwise; lane `sub` takes every G-th piece.
template <int G, class Vec>
__device__ __forceinline__ void write_row(const Group<G> &g, uint32_t *row, const Vec &v, uint32_t W) {
    if ((W & 1u) == 0) {
        uint64_t *r2 = reinterpret_cast<uint64_t *>(row);
        for (uint32_t j = g.sub; j < W / 2; j += G)
            st_coherent(r2 + j, (uint64_t)v.get(2 * j) | ((uint64_t)v.get(2 * j + 1) << 32));
    } else {
        for (uint32_t i = g.sub; i < W; i += G)
            st_coherent(row + i, v.get(i));
    }
}

template <int G, class Vec>
__device__ __forceinline__ bool row_equals(const Group<G> &g, const uint32_t *row, const Vec &v,
                                           uint32_t W) {
    uint32_t diff = 0;
    if ((W & 1u) == 0) {
        const uint64_t *r2 = reinterpret_cast<const uint64_t *>(row);
        for (uint32_t j = g.sub; j < W / 2; j += G) {
            const uint64_t x = ld_coherent(r2 + j);
            diff |= ((uint32_t)x ^ v.get(2 * j)) | ((uint32_t)(x >> 32) ^ v.get(2 * j + 1));
        }
    } else {
        for (uint32_t i = g.sub; i < W; i += G)
            diff |= ld_coherent(row + i) ^ v.get(i);
    }
    return g.all(diff == 0);
}

// One find-or-put per group of G lanes (G = 1, 4, 8 or 16) on a table of
// LS-slot lines (LS = 8, 16 or 32: 64, 128 or 256 bytes).
//
// All lanes of the wavefront call this together; `active`, `v` and `h` are
// uniform within a group, and every decision below is taken from
// group-uniform values, so the G lanes of a group always run the same path.
//
// The probe sequence of a vector with hash h: home line
// (h >> log2 LS) & line_mask, start slot h & (LS-1) inside it; the line is
// examined in walk order start, start+1, ..., wrapping inside the line
// (Algorithm 4 with the start offset read as the line base); after a line,
// the next line follows the table's probe sequence (probe_step/next_line:
// double hashing by default), which visits distinct lines until every line
// was seen.  After max_rounds lines the operation reports EFULL.
//
// Per line one snapshot is taken.  Candidates are, in walk order, the
// snapshot's empty slots and the slots whose memo equals ours.  Slots that
// are claimed with another memo are skipped: they are immutable.
//  - empty candidate: the group leader CASes 0 -> OCC|memo.  Won: the group
//    writes the row, waits for the stores, and the leader stores
//    OCC|DONE|memo; result "new".  Lost: the CAS returned the slot's value;
//    if its memo is ours it becomes a match candidate, otherwise walk on.
//  - match candidate: load the slot until DONE (a bounded wait, the paper's
//    write-busy "lock"), then compare the stored row; equal means "seen",
//    otherwise walk on.
//
// SIMT forward progress: every loop iteration runs the claim phase (CAS,
// row write, publish) for all lanes before the wait phase of any lane, and
// nothing waits between a claim and its publish.  A group that waits on a
// slot claimed by a group of its own wavefront therefore finds it already
// published; a claim made by another wavefront is published without that
// wavefront waiting on anything first.
template <int G, uint32_t LS, class Vec, bool CL = false>
__device__ __forceinline__ void find_or_put(const TableView &t, const Vec &v, uint64_t h, bool active,
                                            uint32_t &out_slot, uint32_t &out_code,
                                            LaneCounters &cnt) {
    const Group<G> g;
    const uint64_t memo = kOcc | (h & kMemoMask);
    const uint32_t start = (uint32_t)h & (LS - 1);
    const uint32_t step = probe_step(h, t.probe);
    uint32_t line = (uint32_t)(h >> line_shift<LS>()) & t.line_mask;
    uint32_t rounds = 0;
    uint32_t cand = 0, empty = 0;  // walk-ordered: bit k <-> slot start+k (mod LS)
    bool have_line = false;
    out_slot = kNoSlot;
    out_code = kFull;
    if (!active)
        return;

    while (true) {
        if (!have_line) {
            if (rounds == t.max_rounds) {
                out_code = kFull;
                if (g.leader())
                    set_error(t.status, 3u /* LHS_EFULL */);
                break;
            }
            uint32_t e, m;
            line_masks<G, LS, CL>(g, t.bucket + (uint64_t)line * LS, memo, e, m);
            empty = rotr_line<LS>(e, start);
            cand = rotr_line<LS>(e | m, start);
            have_line = true;
            cnt.lines += g.leader();
        }
        if (cand == 0) {
            have_line = false;
            ++rounds;
            line = next_line(line, rounds, step, t.probe, t.line_mask);
            continue;
        }
        const uint32_t k = __builtin_ctz(cand);
        cand &= cand - 1;
        const uint32_t slot = line * LS + ((start + k) & (LS - 1));
        uint64_t *bp = t.bucket + slot;
        uint32_t *row = t.data + (uint64_t)slot * t.W;
        bool match = ((empty >> k) & 1u) == 0;
        bool finished = false;

        // ---- claim phase ------------------------------------------------
        if (!match) {
            uint64_t old = 0;
            if (g.leader())
                __hip_atomic_compare_exchange_strong(bp, &old, memo, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            old = g.from_leader(old);
            if (old == 0) {
                write_row<G>(g, row, v, t.W);
                wait_vm_complete();
                if (g.leader())
                    st_coherent(bp, memo | kDone);
                out_slot = slot;
                out_code = kNew;
                finished = true;
            } else {
                cnt.cas_failures += g.leader();
                match = (old & ~kDone) == memo;
            }
        }
        // ---- wait + compare phase --------------------------------------
        if (match && !finished) {
            uint64_t cur = ld_coherent(bp);
            if (!(cur & kDone)) {
                cnt.waits += g.leader();
                uint32_t spins = 0;
                while (!(cur & kDone) && ++spins < kSpinLimit) {
                    __builtin_amdgcn_s_sleep(2);
                    cur = ld_coherent(bp);
                }
            }
            if (!(cur & kDone)) {
                out_code = kStall;
                if (g.leader())
                    set_error(t.status, 4u /* LHS_ESTALL */);
                finished = true;
            } else {
                after_done_observed();
                if (row_equals<G>(g, row, v, t.W)) {
                    out_slot = slot;
                    out_code = kSeen;
                    finished = true;
                }
            }
        }
        if (finished)
            break;
    }
}

// ---------------------------------------------------------------------------
// One operation per lane with wavefront-cooperative memory accesses.
//
// Every lane owns one find-or-put (64 operations in flight per wavefront),
// but the random 128-byte slot lines and the vector rows are moved by the
// whole wavefront: the lanes that need a line (or a row) this iteration are
// compacted into a list in LDS, and LS/2 lanes serve each listed line (16
// bytes each, one coalesced access per line), eight lanes each row (8 bytes
// each).  Results
// come back through the same per-wavefront LDS area.  The helpers need the
// owner's vector: `Vec` has a two-word descriptor any lane can decode.

template <uint32_t LS>
struct WaveScratch {         // one per wavefront, in LDS
    uint64_t key[64];        // memo per rank (line snapshots)
    uint32_t idx[64];        // listed line / slot per rank
    uint32_t aux[64];        // second word (row descriptor y)
    uint32_t desc[64];       // row descriptor x per rank
    uint8_t res[64 * (LS / 2 > 8 ? LS / 2 : 8)];   // per (rank, helper lane) result bits
};

__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// Masks (bit i = slot i of the line) of empty, memo-matching and done slots
// for every lane with `need`; other lanes only help.  Wavefront-uniform call.
// C = LS/2 helper lanes per line, 64/C lines per load instruction, C rounds.
template <uint32_t LS, bool CL = false>
__device__ __forceinline__ void coop_line_masks(WaveScratch<LS> *ws, const uint64_t *bucket, bool need,
                                                uint32_t line, uint64_t memo, uint32_t &empty,
                                                uint32_t &match, uint32_t &done) {
    constexpr uint32_t C = LS / 2, CS = line_shift<LS>() - 1, LPQ = 64 / C;
    const uint32_t lane = __lane_id();
    const uint64_t nmask = __ballot(need);
    const uint32_t nn = (uint32_t)__popcll(nmask);
    const uint32_t rank = mbcnt(nmask);
    if (need) {
        ws->idx[rank] = line;
        ws->key[rank] = memo;
    }
    wave_lds_sync();
    const uint32_t c = lane & (C - 1);
    uint4 x[C];
#pragma unroll
    for (uint32_t q = 0; q < C; ++q) {
        const uint32_t i = q * LPQ + (lane >> CS);
        if (i < nn)
            x[q] = ld_line16<CL>(reinterpret_cast<const uint4 *>(bucket + (uint64_t)ws->idx[i] * LS) + c);
    }
#pragma unroll
    for (uint32_t q = 0; q < C; ++q) {
        const uint32_t i = q * LPQ + (lane >> CS);
        if (i < nn) {
            const uint64_t s0 = ((uint64_t)x[q].y << 32) | x[q].x;
            const uint64_t s1 = ((uint64_t)x[q].w << 32) | x[q].z;
            const uint64_t mk = ws->key[i];
            const uint32_t b = (uint32_t)(s0 == 0) | ((uint32_t)(s1 == 0) << 1) |
                               ((uint32_t)((s0 & ~kDone) == mk) << 2) |
                               ((uint32_t)((s1 & ~kDone) == mk) << 3) |
                               ((uint32_t)(s0 >> 62) & 1u) << 4 | (((uint32_t)(s1 >> 62) & 1u) << 5);
            ws->res[i * C + c] = (uint8_t)b;
        }
    }
    wave_lds_sync();
    if (need) {
        const uint32_t *r = reinterpret_cast<const uint32_t *>(ws->res) + rank * (C / 4);
        uint32_t e = 0, m = 0, d = 0;
#pragma unroll
        for (uint32_t k = 0; k < C; ++k) {
            const uint32_t b = (r[k >> 2] >> (8 * (k & 3))) & 0xFFu;
            e |= (b & 3u) << (2 * k);
            m |= ((b >> 2) & 3u) << (2 * k);
            d |= ((b >> 4) & 3u) << (2 * k);
        }
        empty = e;
        match = m;
        done = d;
    }
    wave_lds_sync();
}

// Write the rows of every lane with `go` (slot, descriptor); eight lanes per
// row, 64-bit coherent stores when W is even, 32-bit otherwise.
template <class Vec, class WS>
__device__ __forceinline__ void coop_write_rows(WS *ws, const uint32_t *smem, uint32_t *data,
                                                uint32_t W, bool go, uint32_t slot, uint2 d) {
    const uint32_t lane = __lane_id();
    const uint64_t gm = __ballot(go);
    const uint32_t ng = (uint32_t)__popcll(gm);
    const uint32_t rank = mbcnt(gm);
    if (go) {
        ws->idx[rank] = slot;
        ws->desc[rank] = d.x;
        ws->aux[rank] = d.y;
    }
    wave_lds_sync();
    const uint32_t c = lane & 7u;
    for (uint32_t i0 = 0; i0 < ng; i0 += 8) {
        const uint32_t i = i0 + (lane >> 3);
        if (i < ng) {
            const Vec v = Vec::decode(smem, make_uint2(ws->desc[i], ws->aux[i]));
            uint32_t *row = data + (uint64_t)ws->idx[i] * W;
            if ((W & 1u) == 0) {
                uint64_t *r2 = reinterpret_cast<uint64_t *>(row);
                for (uint32_t j = c; j < W / 2; j += 8)
                    st_coherent(r2 + j, (uint64_t)v.get(2 * j) | ((uint64_t)v.get(2 * j + 1) << 32));
            } else {
                for (uint32_t j = c; j < W; j += 8)
                    st_coherent(row + j, v.get(j));
            }
        }
    }
    wave_lds_sync();
}

// Compare the stored rows of every lane with `go` against its vector;
// returns equality for those lanes.  Same layout as coop_write_rows.
template <class Vec, class WS>
__device__ __forceinline__ bool coop_rows_equal(WS *ws, const uint32_t *smem,
                                                const uint32_t *data, uint32_t W, bool go,
                                                uint32_t slot, uint2 d) {
    const uint32_t lane = __lane_id();
    const uint64_t gm = __ballot(go);
    const uint32_t ng = (uint32_t)__popcll(gm);
    const uint32_t rank = mbcnt(gm);
    if (go) {
        ws->idx[rank] = slot;
        ws->desc[rank] = d.x;
        ws->aux[rank] = d.y;
    }
    wave_lds_sync();
    const uint32_t c = lane & 7u;
    for (uint32_t i0 = 0; i0 < ng; i0 += 8) {
        const uint32_t i = i0 + (lane >> 3);
        uint32_t diff = 0;
        if (i < ng) {
            const Vec v = Vec::decode(smem, make_uint2(ws->desc[i], ws->aux[i]));
            const uint32_t *row = data + (uint64_t)ws->idx[i] * W;
            if ((W & 1u) == 0) {
                const uint64_t *r2 = reinterpret_cast<const uint64_t *>(row);
                for (uint32_t j = c; j < W / 2; j += 8) {
                    const uint64_t x = ld_coherent(r2 + j);
                    diff |= ((uint32_t)x ^ v.get(2 * j)) | ((uint32_t)(x >> 32) ^ v.get(2 * j + 1));
                }
            } else {
                for (uint32_t j = c; j < W; j += 8)
                    diff |= ld_coherent(row + j) ^ v.get(j);
            }
            ws->res[i * 8 + c] = diff != 0;
        }
    }
    wave_lds_sync();
    bool eq = false;
    if (go) {
        const uint2 r = reinterpret_cast<const uint2 *>(ws->res)[rank];
        eq = (r.x | r.y) == 0;
    }
    wave_lds_sync();
    return eq;
}

// One find-or-put per lane, memory moved cooperatively (see above).  The
// probe sequence, walk order, claim/publish protocol and the SIMT
// forward-progress structure (claim phase, then publish, then waits, in every
// iteration) are those of the group variant.  Additionally a match candidate
// whose snapshot (or failed CAS) already showed DONE is compared without
// re-reading its slot: DONE never goes away, and the row loads are coherent
// and issued after that observation completed.
//
// All 64 lanes must call this together (inactive lanes only help).  `d` is
// the lane's vector descriptor (Vec::decode(smem, d) rebuilds it in any lane).
template <uint32_t LS, class Vec, bool CL = false>
__device__ __forceinline__ void find_or_put_wave(const TableView &t, WaveScratch<LS> *ws,
                                                 const uint32_t *smem, uint2 d, uint64_t h,
                                                 bool active, uint32_t &out_slot,
                                                 uint32_t &out_code, LaneCounters &cnt) {
    const uint64_t memo = kOcc | (h & kMemoMask);
    const uint32_t start = (uint32_t)h & (LS - 1);
    const uint32_t step = probe_step(h, t.probe);
    uint32_t line = (uint32_t)(h >> line_shift<LS>()) & t.line_mask;
    uint32_t rounds = 0, cand = 0, empty = 0, donem = 0;
    bool have_line = false, finished = !active;
    out_slot = kNoSlot;
    out_code = kFull;

    while (__ballot(!finished)) {
        // ---- line snapshots for the lanes that need one -------------------
        if (!finished && !have_line && rounds == t.max_rounds) {
            out_code = kFull;
            set_error(t.status, 3u /* LHS_EFULL */);
            finished = true;
        }
        const bool need = !finished && !have_line;
        if (__ballot(need)) {
            uint32_t e = 0, m = 0, dn = 0;
            coop_line_masks<LS, CL>(ws, t.bucket, need, line, memo, e, m, dn);
            if (need) {
                empty = rotr_line<LS>(e, start);
                cand = rotr_line<LS>(e | m, start);
                donem = rotr_line<LS>(dn, start);
                have_line = true;
                ++cnt.lines;
            }
        }
        // ---- next candidate in walk order ---------------------------------
        uint32_t kind = 0, slot = 0;     // kind: 0 none, 1 empty, 2 match
        bool known_done = false;
        if (!finished) {
            if (cand == 0) {
                have_line = false;
                ++rounds;
                line = next_line(line, rounds, step, t.probe, t.line_mask);
            } else {
                const uint32_t k = __builtin_ctz(cand);
                cand &= cand - 1;
                slot = line * LS + ((start + k) & (LS - 1));
                kind = ((empty >> k) & 1u) ? 1u : 2u;
                known_done = (donem >> k) & 1u;
            }
        }
        // ---- claim phase, with the compare of matches already seen DONE ----
        // Rows of slots the snapshot showed DONE are compared while the
        // claims are in flight: their loads are issued after that snapshot
        // completed, behind the acquire below, and DONE never goes away.
        const bool early = kind == 2 && known_done;
        const uint64_t em = __ballot(early);
        if (em)
            after_done_observed();
        bool won = false;
        uint64_t old = 0;
        if (kind == 1)
            __hip_atomic_compare_exchange_strong(t.bucket + slot, &old, memo, __ATOMIC_RELAXED,
                                                 __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (em) {
            const bool eq = coop_rows_equal<Vec>(ws, smem, t.data, t.W, early, slot, d);
            if (early) {
                if (eq) {
                    out_slot = slot;
                    out_code = kSeen;
                    finished = true;
                }
                kind = 0;   // a different row: the walk goes on
            }
        }
        if (kind == 1) {
            if (old == 0) {
                won = true;
            } else {
                ++cnt.cas_failures;
                kind = (old & ~kDone) == memo ? 2u : 0u;
                known_done = (old & kDone) != 0;
            }
        }
        if (__ballot(won)) {
            coop_write_rows<Vec>(ws, smem, t.data, t.W, won, slot, d);
            wait_vm_complete();
            if (won) {
                st_coherent(t.bucket + slot, memo | kDone);
                out_slot = slot;
                out_code = kNew;
                finished = true;
            }
        }
        // ---- wait phase (only slots not yet seen done) ----------------------
        if (kind == 2 && !known_done) {
            uint64_t cur = ld_coherent(t.bucket + slot);
            if (!(cur & kDone)) {
                ++cnt.waits;
                uint32_t spins = 0;
                while (!(cur & kDone) && ++spins < kSpinLimit) {
                    __builtin_amdgcn_s_sleep(2);
                    cur = ld_coherent(t.bucket + slot);
                }
            }
            if (!(cur & kDone)) {
                out_code = kStall;
                set_error(t.status, 4u /* LHS_ESTALL */);
                finished = true;
                kind = 0;
            }
        }
        // ---- compare phase --------------------------------------------------
        const bool cmp = kind == 2;
        if (__ballot(cmp)) {
            after_done_observed();
            const bool eq = coop_rows_equal<Vec>(ws, smem, t.data, t.W, cmp, slot, d);
            if (cmp && eq) {
                out_slot = slot;
                out_code = kSeen;
                finished = true;
            }
        }
    }
}

// Sum one value over the active lanes of the wavefront; lane-uniform result.
__device__ __forceinline__ uint32_t wave_sum(uint32_t x) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
        x += __shfl_xor(x, off, 64);
    return x;
}

// Flush lane counters into the table status: one atomic per wavefront.
// Must be called by all 64 lanes of the wavefront.
// Lines probed are added only when the table counts them (one more atomic
// per wavefront, on by request: see lhs_set_counters).
__device__ __forceinline__ void flush_counters(const TableView &t, const LaneCounters &c) {
    const uint32_t w = wave_sum(c.waits), f = wave_sum(c.cas_failures);
    const uint32_t l = (t.flags & kCountLines) ? wave_sum(c.lines) : 0u;
    const uint32_t mg = (t.flags & kCountMerged) ? wave_sum(c.merged) : 0u;
    if (__lane_id() == 0) {
        if (w)
            atomicAdd(&t.status->wait_hits, (unsigned long long)w);
        if (f)
            atomicAdd(&t.status->cas_failures, (unsigned long long)f);
        if (l)
            atomicAdd(&t.status->lines, (unsigned long long)l);
        if (mg)
            atomicAdd(&t.status->merged, (unsigned long long)mg);
    }
}

}  // namespace lhs
