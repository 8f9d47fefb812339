// Device-side core of the lockless table: slot encoding, the vector hash and
// the per-lane find-or-put (Algorithm 3 with walking-the-line, Algorithm 4).
//
// Slot (64 bits): 0 = empty; bit 63 OCC = claimed; bit 62 DONE = the vector
// has been written to the data array; bits 61..0 = memoised hash (the low 62
// bits of h1).  A slot goes empty -> claimed(memo) -> done(memo) and never
// changes again (figure "State diagram of buckets"): a slot seen non-empty
// keeps its memo forever, which is what makes a stale snapshot of a line safe.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lhs {

constexpr uint64_t kOcc = 1ull << 63;
constexpr uint64_t kDone = 1ull << 62;
constexpr uint64_t kMemoMask = kDone - 1;
constexpr uint32_t kLineSlots = 16;          // 128-byte line of 8-byte slots
constexpr uint32_t kNoSlot = 0xFFFFFFFFu;
constexpr uint32_t kSpinLimit = 1u << 22;    // bound on one wait (ESTALL)

enum : uint32_t { kNew = 0, kSeen = 1, kFull = 2, kStall = 3 };

// Counters and sticky error kept in device memory per table.
struct DevStatus {
    uint32_t error;          // first device error (lhs_status), 0 = none
    uint32_t pad;
    unsigned long long wait_hits;
    unsigned long long cas_failures;
};

// Per-lane event counts, reduced per wavefront before touching DevStatus.
struct LaneCounters {
    uint32_t waits = 0;
    uint32_t cas_failures = 0;
};

struct TableView {
    uint64_t *bucket;
    uint32_t *data;
    uint64_t seed;
    uint32_t W;
    uint32_t line_mask;      // lines - 1
    uint32_t max_rounds;     // lines probed before EFULL
    DevStatus *status;
};

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

// rotate a 16-bit mask right by r (bit k of the result = bit (k + r) mod 16)
__device__ __forceinline__ uint32_t rotr16(uint32_t m, uint32_t r) {
    return ((m >> r) | (m << (16 - r))) & 0xFFFFu;
}

template <class Vec>
__device__ __forceinline__ void write_row(uint32_t *row, const Vec &v, uint32_t W) {
    if ((W & 3u) == 0) {
        uint4 *r4 = reinterpret_cast<uint4 *>(row);
        for (uint32_t i = 0; i < W; i += 4)
            r4[i >> 2] = make_uint4(v.get(i), v.get(i + 1), v.get(i + 2), v.get(i + 3));
    } else {
        for (uint32_t i = 0; i < W; ++i)
            row[i] = v.get(i);
    }
}

template <class Vec>
__device__ __forceinline__ bool row_equals(const uint32_t *row, const Vec &v, uint32_t W) {
    uint32_t diff = 0;
    if ((W & 3u) == 0) {
        const uint4 *r4 = reinterpret_cast<const uint4 *>(row);
        for (uint32_t i = 0; i < W; i += 4) {
            const uint4 x = r4[i >> 2];
            diff |= (x.x ^ v.get(i)) | (x.y ^ v.get(i + 1)) | (x.z ^ v.get(i + 2)) |
                    (x.w ^ v.get(i + 3));
        }
    } else {
        for (uint32_t i = 0; i < W; ++i)
            diff |= row[i] ^ v.get(i);
    }
    return diff == 0;
}

// One find-or-put per lane.
//
// The probe sequence of a vector with hash h: home line (h >> 4) & line_mask,
// start slot h & 15 inside it; the line is examined in walk order
// start, start+1, ..., wrapping inside the line (Algorithm 4 with the start
// offset read as the line base); after a line, the next line is
// line + step (mod lines) with step = (h >> 32) | 1, odd, so successive
// rounds visit distinct lines until every line was seen (double hashing
// across lines).  After max_rounds lines the operation reports EFULL.
//
// Per line one 128-byte snapshot is taken.  Candidates are, in walk order, the
// snapshot's empty slots and the slots whose memo equals ours.  Slots that
// are claimed with another memo are skipped: they are immutable.
//  - empty candidate: CAS(0 -> OCC|memo).  Won: write the row, then publish
//    OCC|DONE|memo with release semantics; result "new".  Lost: the CAS
//    returned the slot's value; if its memo is ours it becomes a match
//    candidate, otherwise walk on.
//  - match candidate: acquire-load the slot until DONE (a bounded wait, the
//    paper's write-busy "lock"), then compare the stored row; equal means
//    "seen", otherwise walk on.
//
// SIMT forward progress: every loop iteration runs the claim phase (CAS,
// row write, publish) for all lanes before the wait phase of any lane, and
// nothing waits between a claim and its publish.  A lane that waits on a slot
// claimed by a lane of its own wavefront therefore finds it already
// published; a claim made by another wavefront is published without that
// wavefront waiting on anything first.
template <class Vec>
__device__ __forceinline__ void find_or_put(const TableView &t, const Vec &v, uint64_t h,
                                            uint32_t &out_slot, uint32_t &out_code,
                                            LaneCounters &cnt) {
    const uint64_t memo = kOcc | (h & kMemoMask);
    const uint32_t start = (uint32_t)h & (kLineSlots - 1);
    const uint32_t step = (uint32_t)(h >> 32) | 1u;
    uint32_t line = (uint32_t)(h >> 4) & t.line_mask;
    uint32_t rounds = 0;
    uint32_t cand = 0, empty = 0;  // walk-ordered: bit k <-> slot start+k (mod 16)
    bool have_line = false;
    out_slot = kNoSlot;
    out_code = kFull;

    while (true) {
        if (!have_line) {
            if (rounds == t.max_rounds) {
                out_code = kFull;
                set_error(t.status, 3u /* LHS_EFULL */);
                break;
            }
            const uint4 *lp = reinterpret_cast<const uint4 *>(t.bucket + (uint64_t)line * kLineSlots);
            uint32_t e = 0, m = 0;
#pragma unroll
            for (uint32_t q = 0; q < kLineSlots / 2; ++q) {
                const uint4 x = lp[q];
                const uint64_t s0 = ((uint64_t)x.y << 32) | x.x;
                const uint64_t s1 = ((uint64_t)x.w << 32) | x.z;
                e |= (uint32_t)(s0 == 0) << (2 * q);
                e |= (uint32_t)(s1 == 0) << (2 * q + 1);
                m |= (uint32_t)((s0 & ~kDone) == memo) << (2 * q);
                m |= (uint32_t)((s1 & ~kDone) == memo) << (2 * q + 1);
            }
            empty = rotr16(e, start);
            cand = rotr16(e | m, start);
            have_line = true;
        }
        if (cand == 0) {
            have_line = false;
            ++rounds;
            line = (line + step) & t.line_mask;
            continue;
        }
        const uint32_t k = __builtin_ctz(cand);
        cand &= cand - 1;
        const uint32_t slot = line * kLineSlots + ((start + k) & (kLineSlots - 1));
        uint64_t *bp = t.bucket + slot;
        bool match = ((empty >> k) & 1u) == 0;
        bool finished = false;

        // ---- claim phase ------------------------------------------------
        if (!match) {
            uint64_t expected = 0;
            if (__hip_atomic_compare_exchange_strong(bp, &expected, memo, __ATOMIC_RELAXED,
                                                     __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) {
                write_row(t.data + (uint64_t)slot * t.W, v, t.W);
                __hip_atomic_store(bp, memo | kDone, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                out_slot = slot;
                out_code = kNew;
                finished = true;
            } else {
                ++cnt.cas_failures;
                match = (expected & ~kDone) == memo;
            }
        }
        // ---- wait + compare phase --------------------------------------
        if (match && !finished) {
            uint64_t cur = __hip_atomic_load(bp, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
            if (!(cur & kDone)) {
                ++cnt.waits;
                uint32_t spins = 0;
                while (!(cur & kDone) && ++spins < kSpinLimit) {
                    __builtin_amdgcn_s_sleep(2);
                    cur = __hip_atomic_load(bp, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                }
            }
            if (!(cur & kDone)) {
                out_code = kStall;
                set_error(t.status, 4u /* LHS_ESTALL */);
                finished = true;
            } else if (row_equals(t.data + (uint64_t)slot * t.W, v, t.W)) {
                out_slot = slot;
                out_code = kSeen;
                finished = true;
            }
        }
        if (finished)
            break;
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
__device__ __forceinline__ void flush_counters(DevStatus *st, const LaneCounters &c) {
    const uint32_t w = wave_sum(c.waits), f = wave_sum(c.cas_failures);
    if (__lane_id() == 0) {
        if (w)
            atomicAdd(&st->wait_hits, (unsigned long long)w);
        if (f)
            atomicAdd(&st->cas_failures, (unsigned long long)f);
    }
}

}  // namespace lhs
