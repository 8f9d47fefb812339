// Multi-core CPU implementation of the paper's lockless shared hash table and
// of level-synchronous reachability over it: the method as the paper runs it
// on x86 cores, measured next to the GPU library as a fair multi-core CPU
// baseline.  It is neither the oracle (which is sequential and uses a library
// set) nor a fallback of the GPU path (nothing in the GPU library loads it).
//
// Table (section "A Lockless Hash Table", Algorithms 2-4):
//  * 2^n slots of 64 bits in lines of 8 slots = one 64-byte x86 cache line;
//    slot = 0 (empty) | bit 63 claimed | bit 62 written | 62-bit memo of the
//    vector's hash; vectors in a separate data array indexed by slot;
//  * find-or-put walks the home line from the home slot, wrapping inside the
//    line, then moves to the next line by double hashing (odd step), and
//    gives up (table full) after every line was probed;
//  * an empty slot is claimed with a 64-bit compare-and-swap of 0 -> memo;
//    the winner writes the vector, then publishes "written" with a release
//    store; a thread that meets its own memo on a claimed slot waits
//    (acquire loads) until it is written, then compares the vector.
// Reachability (Algorithm 1): level by level, threads take chunks of the
// frontier, generate successors (asynchronous interleaving of guarded
// transitions), find-or-put every successor (each one an edge) and keep the
// new ones in per-thread buffers that form the next frontier.  A state
// without successors is a deadlock.  Level-prefix cap: a level that would
// take the total past the cap is undone (its slots zeroed) and dropped.
//
// Hash: 64-bit word-pair mixing with multiply/xor-shift steps closed by the
// SplitMix64 finaliser (Steele, Lea, Flood 2014).
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstring>
#include <memory>
#include <new>
#include <thread>
#include <vector>

namespace {

constexpr uint64_t kOcc = 1ull << 63, kDone = 1ull << 62, kMemo = kDone - 1;
constexpr uint32_t kLine = 8;
constexpr uint32_t NONE = 0xFFFFFFFFu;

inline uint64_t fmix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

inline uint64_t hash_row(const uint32_t *v, uint32_t W) {
    uint64_t h = 0x243F6A8885A308D3ull ^ W;
    uint32_t i = 0;
    for (; i + 1 < W; i += 2) {
        const uint64_t k = (uint64_t)v[i] | ((uint64_t)v[i + 1] << 32);
        h = (h ^ fmix(k + 0x9E3779B97F4A7C15ull)) * 0xD6E8FEB86659FD93ull;
    }
    if (i < W)
        h = (h ^ fmix(v[i] + 0x9E3779B97F4A7C15ull)) * 0xD6E8FEB86659FD93ull;
    return fmix(h);
}

enum : int { kNew = 0, kSeen = 1, kFull = 2 };

struct Table {
    uint32_t W;
    uint64_t cap, lines;
    std::unique_ptr<std::atomic<uint64_t>[]> bucket;
    std::unique_ptr<uint32_t[]> data;

    // Allocate and touch every page with `threads` threads (outside any
    // timed region: first-touch page faults are not part of the method).
    Table(uint32_t W_, uint32_t log2cap, uint32_t threads)
        : W(W_), cap(1ull << log2cap), lines((1ull << log2cap) / kLine) {
        bucket.reset(new std::atomic<uint64_t>[cap]);
        data.reset(new uint32_t[cap * W]);
        std::vector<std::thread> pool;
        for (uint32_t id = 0; id < threads; ++id)
            pool.emplace_back([this, id, threads] {
                const uint64_t lo = cap * id / threads, hi = cap * (id + 1) / threads;
                for (uint64_t i = lo; i < hi; ++i)
                    bucket[i].store(0, std::memory_order_relaxed);
                std::memset(data.get() + lo * W, 0, (hi - lo) * W * sizeof(uint32_t));
            });
        for (auto &th : pool)
            th.join();
    }

    bool equal(uint64_t slot, const uint32_t *v) const {
        return std::memcmp(data.get() + slot * W, v, W * sizeof(uint32_t)) == 0;
    }

    // Algorithm 3 with the line walk of Algorithm 4; returns kNew/kSeen/kFull
    int find_or_put(const uint32_t *v, uint64_t &slot_out) {
        const uint64_t h = hash_row(v, W);
        const uint64_t memo = kOcc | (h & kMemo);
        const uint64_t step = (h >> 32) | 1ull;
        uint64_t line = (h >> 3) & (lines - 1);
        const uint32_t start = (uint32_t)h & (kLine - 1);
        for (uint64_t round = 0; round < lines; ++round) {
            std::atomic<uint64_t> *ln = &bucket[line * kLine];
            for (uint32_t i = 0; i < kLine; ++i) {
                const uint32_t k = (start + i) & (kLine - 1);
                uint64_t cur = ln[k].load(std::memory_order_acquire);
                if (cur == 0) {
                    uint64_t expect = 0;
                    if (ln[k].compare_exchange_strong(expect, memo, std::memory_order_acq_rel)) {
                        const uint64_t slot = line * kLine + k;
                        std::memcpy(data.get() + slot * W, v, W * sizeof(uint32_t));
                        ln[k].store(memo | kDone, std::memory_order_release);
                        slot_out = slot;
                        return kNew;
                    }
                    cur = expect;   // lost the race: examine the winner
                }
                if ((cur & ~kDone) == memo) {
                    while (!(cur & kDone)) {   // written status ("write-busy")
                        std::this_thread::yield();
                        cur = ln[k].load(std::memory_order_acquire);
                    }
                    const uint64_t slot = line * kLine + k;
                    if (equal(slot, v)) {
                        slot_out = slot;
                        return kSeen;
                    }
                }
            }
            line = (line + step) & (lines - 1);
        }
        return kFull;
    }
};

double seconds_since(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

template <class F>
void run_threads(uint32_t threads, F &&f) {
    std::vector<std::thread> pool;
    for (uint32_t t = 1; t < threads; ++t)
        pool.emplace_back(f, t);
    f(0u);
    for (auto &th : pool)
        th.join();
}

}  // namespace

extern "C" {

typedef struct cpu_summary {
    uint64_t total, edges, deadlocks;
    uint32_t n_levels;
    int32_t capped;
} cpu_summary;

// Batched find-or-put of rows [n][W] into a fresh 2^log2cap-slot table by
// `threads` threads (chunks of 4096 rows).  seen[k] = 1 if the vector was
// stored before operation k took effect, index[k] = its slot.  *seconds =
// time of the find-or-put phase.  Returns 0, or 1 if the table filled up.
int cpu_stream(const uint32_t *rows, uint64_t n, uint32_t W, uint32_t log2cap, uint32_t threads,
               uint8_t *seen, uint32_t *index, double *seconds) {
    if (!rows || !seen || W == 0 || W > 32 || log2cap < 3 || log2cap > 32 || threads == 0)
        return 2;
    Table t(W, log2cap, threads);
    std::atomic<uint64_t> next{0};
    std::atomic<int> full{0};
    const auto t0 = std::chrono::steady_clock::now();
    run_threads(threads, [&](uint32_t) {
        constexpr uint64_t kChunk = 4096;
        for (uint64_t lo = next.fetch_add(kChunk); lo < n; lo = next.fetch_add(kChunk)) {
            const uint64_t hi = lo + kChunk < n ? lo + kChunk : n;
            for (uint64_t k = lo; k < hi; ++k) {
                uint64_t slot = 0;
                const int r = t.find_or_put(rows + k * W, slot);
                if (r == kFull)
                    full.store(1);
                seen[k] = r == kSeen ? 1 : (r == kNew ? 0 : 0xFF);
                if (index)
                    index[k] = (uint32_t)slot;
            }
        }
    });
    if (seconds)
        *seconds = seconds_since(t0);
    return full.load() ? 1 : 0;
}

// Level-synchronous reachability of a guarded model (trans [P][L][K][5] of
// target, guard var, guard value, effect var, effect value; NONE = 0xFFFFFFFF)
// from init [P + S] with `threads` threads on a 2^log2cap-slot table.
// level_counts gets up to max_levels entries; rows_out (may be NULL) gets the
// stored vectors in level order when max_rows suffices.  *seconds = time of
// the exploration.  Returns 0, 1 (table full), 2 (bad argument) or 3 (more
// levels than max_levels).
int cpu_reach(const uint32_t *trans, uint32_t P, uint32_t L, uint32_t S, uint32_t K, const uint32_t *init,
              uint64_t cap, uint32_t log2cap, uint32_t threads, uint64_t *level_counts, uint32_t max_levels,
              uint32_t *rows_out, uint64_t max_rows, cpu_summary *out, double *seconds) {
    const uint32_t W = P + S;
    if (!trans || !init || !out || !level_counts || W == 0 || W > 32 || threads == 0 || log2cap < 3 ||
        log2cap > 32 || max_levels == 0)
        return 2;
    std::memset(out, 0, sizeof(*out));
    Table t(W, log2cap, threads);
    const auto t0 = std::chrono::steady_clock::now();
    uint64_t root = 0;
    if (t.find_or_put(init, root) != kNew)
        return 1;
    std::vector<uint32_t> frontier{(uint32_t)root}, order{(uint32_t)root};
    uint64_t total = 1, edges = 0, dead = 0;
    uint32_t n_levels = 1;
    level_counts[0] = 1;
    int capped = 0, rc = 0;
    struct alignas(64) Local {
        std::vector<uint32_t> next;
        uint64_t edges = 0, dead = 0;
        int full = 0;
    };
    std::vector<Local> loc(threads);
    while (!frontier.empty()) {
        std::atomic<uint64_t> at{0};
        for (auto &l : loc) {
            l.next.clear();
            l.edges = l.dead = 0;
            l.full = 0;
        }
        run_threads(threads, [&](uint32_t id) {
            Local &me = loc[id];
            std::vector<uint32_t> s(W), succ(W);
            constexpr uint64_t kChunk = 256;
            for (uint64_t lo = at.fetch_add(kChunk); lo < frontier.size(); lo = at.fetch_add(kChunk)) {
                const uint64_t hi = lo + kChunk < frontier.size() ? lo + kChunk : frontier.size();
                for (uint64_t f = lo; f < hi; ++f) {
                    std::memcpy(s.data(), t.data.get() + (uint64_t)frontier[f] * W, W * sizeof(uint32_t));
                    uint64_t count = 0;
                    for (uint32_t p = 0; p < P; ++p) {
                        const uint32_t *tp = trans + (((uint64_t)p * L + s[p]) * K) * 5;
                        for (uint32_t k = 0; k < K; ++k, tp += 5) {
                            if (tp[1] != NONE && s[P + tp[1]] != tp[2])
                                continue;
                            std::memcpy(succ.data(), s.data(), W * sizeof(uint32_t));
                            succ[p] = tp[0];
                            if (tp[3] != NONE)
                                succ[P + tp[3]] = tp[4];
                            ++count;
                            uint64_t slot = 0;
                            const int r = t.find_or_put(succ.data(), slot);
                            if (r == kNew)
                                me.next.push_back((uint32_t)slot);
                            else if (r == kFull)
                                me.full = 1;
                        }
                    }
                    me.edges += count;
                    me.dead += count == 0;
                }
            }
        });
        uint64_t n_next = 0, l_edges = 0, l_dead = 0;
        for (auto &l : loc) {
            n_next += l.next.size();
            l_edges += l.edges;
            l_dead += l.dead;
            if (l.full)
                rc = 1;
        }
        if (rc)
            break;
        if (cap && total + n_next > cap) {   // discard the level: undo its claims
            for (auto &l : loc)
                for (uint32_t slot : l.next)
                    t.bucket[slot].store(0, std::memory_order_relaxed);
            capped = 1;
            break;
        }
        edges += l_edges;
        dead += l_dead;
        if (n_next == 0)
            break;
        if (n_levels == max_levels) {
            rc = 3;
            break;
        }
        level_counts[n_levels++] = n_next;
        total += n_next;
        frontier.clear();
        for (auto &l : loc)
            frontier.insert(frontier.end(), l.next.begin(), l.next.end());
        order.insert(order.end(), frontier.begin(), frontier.end());
    }
    if (seconds)
        *seconds = seconds_since(t0);
    out->total = total;
    out->edges = edges;
    out->deadlocks = dead;
    out->n_levels = n_levels;
    out->capped = capped;
    if (rows_out && order.size() <= max_rows)
        for (uint64_t i = 0; i < order.size(); ++i)
            std::memcpy(rows_out + i * W, t.data.get() + (uint64_t)order[i] * W, W * sizeof(uint32_t));
    return rc;
}

}  // extern "C"
