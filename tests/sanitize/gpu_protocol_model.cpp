// CPU-thread model of the GPU kernels' synchronisation protocols, for
// ThreadSanitizer.  It plays the part that a model checker plays for the
// paper's Algorithm 3 (section "Algorithm": the authors checked the
// find-or-put algorithm with a model of it): threads stand for lanes and
// workgroups, and TSan checks that every access to shared payload is ordered
// by the protocol's announcements.
//
// Mapping from the kernels (csrc/lhs_device.h, expand_device.h, batch.hip):
//  * Payload -- vector rows, frontier entries, a level's state, the (model,
//    tile) of a ring cell, per-model progress -- is plain memory here, so
//    that TSan reports any access pair the protocol leaves unordered.
//  * Slot words, counters, ring sequence numbers and the tile count are
//    std::atomic.  A kernel access that is relaxed and unordered stays
//    relaxed.  Where the kernel waits for its earlier accesses to complete
//    (s_waitcnt vmcnt(0)) before an announcing store or atomic, the model
//    uses release.  Where the kernel issues its next accesses only after an
//    observed value returned (the value decides what it does next), the
//    model uses acquire.
//
// Part 1, find-or-put: slot = 0 (empty) -> OCC|memo (claimed, CAS) ->
// OCC|DONE|memo (published).  The CAS winner writes the row and only then
// publishes; a reader compares a row only after observing DONE, from the
// line snapshot, from a failed CAS, or by a bounded wait.  Lines are walked
// from the home slot and left by double hashing, as in the kernels.
//
// Part 2, the persistent batch: workers take (model, tile) items from a
// bounded ring of sequence-numbered cells; the worker that completes a
// level's last tile finalises it (rollback of a capped level, level count,
// frontier swap, next level's state), keeps tile 0 of the next level and
// enqueues the others.  Models are N independent cyclic L-state processes;
// results are checked against a sequential BFS.
//
// Part 4, the persistent server: a host thread posts queries (a slot's
// constants and table, then an admission entry, then the admission tail)
// to running workers and collects completion records; workers hold one ring
// position each (fetch-and-add) and take admissions between polls, queueing
// the admitted query's first tile (a worker keeps tiles for itself only
// when it holds no position); the
// launch ends when its workers leave after a quiet spell, or early when the
// host asks it to drain, and the host starts another for queries posted too
// late.  Leaving and admitting announce themselves before each looks at the
// other (sequentially consistent), and an admission checks that no worker
// of its launch has left.  Slots are reused by later queries.
//
// Part 5, the merge of equal successors of an expansion pass: lanes write
// their successors (the pass's list, plain memory), meet at the pass
// barrier, and each claims a cell of a hash set (atomics) with its hash tag
// and lane; a lane that meets its own tag stops there and takes that lane's
// find-or-put as its own once the two vectors compare equal, and the lane
// holding the cell always probes.  Checked per pass: every distinct vector
// keeps a lane that probes, every merged lane's lane holds an equal vector
// and probes, and with distinct hashes each vector probes exactly once.
// Hashes are full, cut to one tag bit, or forced to collide across vectors.
//
// Part 6, a level's new states appended to eight segments of the next
// frontier: workgroups buffer new states and flush them with one fetch-and-
// add on the cursor of their own segment, a flush that does not fit takes
// the rest from the following segments, and a flush that finds every
// segment full reports EFULL.  Each workgroup estimates the level's count as
// eight times its cursor, turns eager (a flush after every pass) within a
// margin of the cap, and from then on sums the eight cursors after each
// flush and raises the abort flag past the cap.  Workgroups take tiles in a
// grid stride and look at the abort flag at every tile.  Checked per level:
// the segments' first min(cursor, size) entries hold every appended state
// exactly once, EFULL is reported exactly when the states outnumber the
// segments' room, and the abort is never raised below the cap.  Workgroup
// counts that are not multiples of eight fill the segments unevenly.
//
// Part 7, exploration without level barriers: workers take 16-entry chunks
// of one queue of slots in discovery order with a fetch-and-add, wait for
// the chunk's entries to be written (unwritten entries hold 0xFFFFFFFF),
// expand them, buffer new states and append them in bulk (mid-tile when
// the buffer nears full, and when their own chunk runs dry or another
// worker waits), and after every tile add (states discovered, appended or
// buffered) - (states expanded) to a shared work count; states appended in
// the middle of a tile are added to it before their entries are written.  A
// worker leaves once its chunk is dry, it holds nothing back and the work
// count is zero.
// Checked per run: the queue lists the reachable set of a sequential BFS
// exactly once, every entry is expanded exactly once, the edges are all
// counted and the work count ends at zero.  With a cap inside the state
// space the append that passes it stops every worker (at its next tile, or
// in a wait for an entry), and then every stored state is listed once and
// is reachable.
//
// Planted mistakes (compile with -DPLANT=n) remove one ordering or check
// each; the test expects TSan (or a result check) to catch every one:
//   1 publish DONE before writing the row      2 publish DONE relaxed
//   3 compare a matching row without DONE      4 free a ring cell relaxed
//   5 count a finished tile relaxed            6 raise the admission tail relaxed
//   7 publish a completion record relaxed      8 fill a completion record after
//                                                publishing it
//   9 merge on a tag match without comparing  10 read another lane's successor
//     the vectors                                 without the pass barrier
//  11 place a flush past the end of a         12 abort on the workgroup's own
//     segment                                    estimate, without the cursors
//  13 write a queue entry relaxed             14 count held-back states as open
//                                                only once they are appended
//  15 count states appended in the middle of a tile only when the tile ends
//     (caught by the unsanitized repeated run of part 7: `model part7 N`)
//  16 a worker that admits a query keeps its first tile while it still holds
//     a ring position (part 4; unsanitized repeated runs, `model part4 N`,
//     stop with a producer waiting on that position's cell in about 1 run
//     of 20 to 500, depending on how busy the host is)
#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <random>
#include <set>
#include <thread>
#include <vector>

#ifndef PLANT
#define PLANT 0
#endif

namespace {

constexpr uint64_t kOcc = 1ull << 63, kDone = 1ull << 62, kMemo = kDone - 1;
constexpr uint32_t kSpin = 1u << 26;
enum Code { kNew, kSeen, kFull, kStall };

uint64_t mix64(uint64_t z) {   // SplitMix64 finaliser (Steele, Lea, Flood 2014)
    z ^= z >> 30;
    z *= 0xbf58476d1ce4e5b9ull;
    z ^= z >> 27;
    z *= 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}
uint64_t hash_row(const uint32_t *v, uint32_t W) {
    uint64_t h = 0x243f6a8885a308d3ull;
    for (uint32_t i = 0; i < W; ++i)
        h = mix64(h ^ v[i]);
    return h;
}

struct Table {
    uint32_t W, LS, lines;
    std::unique_ptr<std::atomic<uint64_t>[]> slot;
    std::vector<uint32_t> data;   // payload: rows, plain memory
    std::atomic<uint64_t> waits{0}, cas_fail{0};
    Table(uint32_t W_, uint32_t LS_, uint32_t cap) : W(W_), LS(LS_), lines(cap / LS_),
                                                     slot(new std::atomic<uint64_t>[cap]), data((size_t)cap * W_) {
        for (uint32_t i = 0; i < cap; ++i)
            slot[i].store(0, std::memory_order_relaxed);
    }
    uint32_t capacity() const { return lines * LS; }
};

bool row_equals(const Table &t, uint32_t s, const uint32_t *v) {
    return std::memcmp(&t.data[(size_t)s * t.W], v, t.W * 4u) == 0;   // plain reads of the row
}

// Algorithm 3 with walking the line; returns kNew / kSeen / kFull / kStall.
Code find_or_put(Table &t, const uint32_t *v, uint32_t &out) {
    const uint64_t h = hash_row(v, t.W);
    const uint64_t memo = kOcc | (h & kMemo);
    const uint32_t start = (uint32_t)h & (t.LS - 1);
    const uint32_t step = (uint32_t)(h >> 32) | 1u;
    uint32_t line = (uint32_t)(h >> 8) & (t.lines - 1);
    std::vector<uint64_t> snap(t.LS);
    for (uint32_t round = 0; round < t.lines; ++round, line = (line + step) & (t.lines - 1)) {
        // the line snapshot (the kernel compares rows of slots seen DONE
        // here without reading their slot again)
        for (uint32_t i = 0; i < t.LS; ++i)
            snap[i] = t.slot[line * t.LS + i].load(std::memory_order_acquire);
        for (uint32_t k = 0; k < t.LS; ++k) {
            const uint32_t s = line * t.LS + ((start + k) & (t.LS - 1));
            uint64_t cur = snap[(start + k) & (t.LS - 1)];
            if (cur == 0) {
                // claim: a CAS whose returned value the lane tests before
                // its next access (acquire; a failure may return DONE, and
                // the row is then compared at once).  C++ wants the success
                // order at least as strong as the failure order.
                uint64_t old = 0;
                if (t.slot[s].compare_exchange_strong(old, memo, std::memory_order_acquire,
                                                      std::memory_order_acquire)) {
                    // (the yield widens the write-busy window, as the GPU's
                    // row store and its completion wait do)
#if PLANT == 1
                    t.slot[s].store(memo | kDone, std::memory_order_release);
                    std::this_thread::yield();
                    std::memcpy(&t.data[(size_t)s * t.W], v, t.W * 4u);
#elif PLANT == 2
                    std::memcpy(&t.data[(size_t)s * t.W], v, t.W * 4u);
                    std::this_thread::yield();
                    t.slot[s].store(memo | kDone, std::memory_order_relaxed);
#else
                    // row stores, completed (vmcnt(0)) before the DONE store
                    std::memcpy(&t.data[(size_t)s * t.W], v, t.W * 4u);
                    std::this_thread::yield();
                    t.slot[s].store(memo | kDone, std::memory_order_release);
#endif
                    out = s;
                    return kNew;
                }
                t.cas_fail.fetch_add(1, std::memory_order_relaxed);
                cur = old;
            }
            if ((cur & ~kDone) != memo)
                continue;   // claimed with another memo: immutable, skip
#if PLANT != 3
            if (!(cur & kDone)) {
                // the writer's bounded wait (write-busy "lock")
                t.waits.fetch_add(1, std::memory_order_relaxed);
                uint32_t spins = 0;
                while (!((cur = t.slot[s].load(std::memory_order_acquire)) & kDone))
                    if (++spins > kSpin)
                        return kStall;
                    else
                        std::this_thread::yield();
            }
#endif
            if (row_equals(t, s, v)) {
                out = s;
                return kSeen;
            }
        }
    }
    return kFull;
}

// ---------------------------------------------------------------- part 1 ---
int part1() {
    // W = 5 rows from a small alphabet: many equal vectors, a small table
    // with 8-slot lines filled to 3/4 so that probes leave their home line
    const uint32_t W = 5, cap = 1u << 12, pool = 3000, threads = 8, ops = 6000;
    Table t(W, 8, cap);
    std::vector<uint32_t> rows((size_t)pool * W);
    uint64_t x = 0x9E3779B97F4A7C15ull;
    for (uint32_t i = 0; i < pool; ++i) {
        rows[(size_t)i * W] = i;
        for (uint32_t j = 1; j < W; ++j)
            rows[(size_t)i * W + j] = (uint32_t)((x = mix64(x + i * 31 + j)) % 3);
    }
    std::vector<std::vector<std::pair<uint32_t, uint32_t>>> res(threads);   // (row, slot) of new/seen
    std::vector<std::vector<uint8_t>> isnew(threads);
    std::vector<std::thread> th;
    std::atomic<int> bad{0};
    // every thread walks the pool in the same order from a nearby start, so
    // equal vectors are inserted by several threads at about the same time
    for (uint32_t w = 0; w < threads; ++w)
        th.emplace_back([&, w] {
            for (uint32_t k = 0; k < ops; ++k) {
                const uint32_t r = (k + 3 * w) % pool;
                uint32_t s = ~0u;
                const Code c = find_or_put(t, &rows[(size_t)r * W], s);
                if (c != kNew && c != kSeen)
                    bad.fetch_add(1);
                res[w].push_back({r, s});
                isnew[w].push_back(c == kNew);
            }
        });
    for (auto &h : th)
        h.join();
    // every value stored once: one "new" per distinct row, one slot per row,
    // distinct rows in distinct slots, and each slot holds its row
    std::map<uint32_t, uint32_t> slot_of, news;
    std::set<uint32_t> used;
    for (uint32_t w = 0; w < threads; ++w)
        for (size_t k = 0; k < res[w].size(); ++k) {
            const auto [r, s] = res[w][k];
            auto it = slot_of.find(r);
            if (it == slot_of.end())
                slot_of[r] = s;
            else if (it->second != s)
                bad.fetch_add(1);
            news[r] += isnew[w][k];
        }
    for (auto &[r, s] : slot_of) {
        if (news[r] != 1 || !used.insert(s).second || !row_equals(t, s, &rows[(size_t)r * W]))
            bad.fetch_add(1);
    }
    uint32_t done = 0;
    for (uint32_t i = 0; i < cap; ++i) {
        const uint64_t v = t.slot[i].load();
        if (v && !(v & kDone))
            bad.fetch_add(1);   // claimed but never published
        done += (v & kDone) != 0;
    }
    if (done != slot_of.size())
        bad.fetch_add(1);
    printf("part1: %zu distinct of %u ops, %u stored, %llu waits, %llu cas failures, errors %d\n",
           slot_of.size(), threads * ops, done, (unsigned long long)t.waits.load(),
           (unsigned long long)t.cas_fail.load(), bad.load());
    return bad.load();
}

// ---------------------------------------------------------------- part 2 ---
struct Cell {
    std::atomic<uint64_t> seq;
    uint32_t model, tile;   // payload
};

struct LevelState {     // payload, written by the finaliser of the level before
    uint32_t cur;       // announcing the level's tiles
    uint32_t n_front, limit, tiles_total, tile_rows;
    std::atomic<uint32_t> tiles_done{0};
};

struct Model {
    uint32_t N, L;      // N independent cyclic L-state processes, W = N
    uint64_t cap;       // level-prefix state cap (0 = none)
    std::unique_ptr<Table> t;
    std::vector<uint32_t> fr[2];                  // payload
    std::atomic<uint32_t> n_next{0}, abort{0};
    std::atomic<uint64_t> edges{0}, dead{0};
    LevelState lv;
    // progress (payload; only finalisers touch it, one level after another)
    uint64_t total = 1, p_edges = 0, p_dead = 0;
    std::vector<uint64_t> levels{1};
    bool capped = false;
};

struct Queue {
    std::atomic<uint64_t> head{0}, tail{0};
    std::atomic<uint32_t> remaining{0}, error{0};
    uint64_t mask = 0;
    std::unique_ptr<Cell[]> ring;
};

constexpr uint32_t kTileRows = 8;

// Fill ring position pos (reserved on the tail): wait for its cell to be
// free, write the item, publish it.  False if the wait ran out.
bool ring_put(Queue &q, uint64_t pos, uint32_t model, uint32_t tile) {
    Cell &c = q.ring[pos & q.mask];
    uint32_t spins = 0;
    while (c.seq.load(std::memory_order_acquire) != pos) {
        if (++spins > kSpin)
            return false;
        std::this_thread::yield();
    }
    c.model = model;
    c.tile = tile;
    c.seq.store(pos + 1, std::memory_order_release);   // after vmcnt(0)
    return true;
}

// Take ring position pos (reserved on the head): wait for its cell to be
// filled, read the item, free the cell for position pos + ring size.  False
// if give_up() said so, or the wait ran out (then *timed_out).
template <class GiveUp>
bool ring_take(Queue &q, uint64_t pos, uint32_t &model, uint32_t &tile, GiveUp give_up, bool &timed_out) {
    Cell &c = q.ring[pos & q.mask];
    uint32_t spins = 0;
    timed_out = false;
    while (c.seq.load(std::memory_order_acquire) != pos + 1) {
        if (give_up())
            return false;
        if (++spins > kSpin) {
            timed_out = true;
            return false;
        }
        std::this_thread::yield();
    }
    model = c.model;
    tile = c.tile;
#if PLANT == 4
    c.seq.store(pos + q.mask + 1, std::memory_order_relaxed);
#else
    // the item was read (vmcnt(0)) before the cell is freed
    c.seq.store(pos + q.mask + 1, std::memory_order_release);
#endif
    return true;
}

// Expand tile `j` of model m's current level; new states to next[].
void expand_tile(Model &m, uint32_t j, Queue &q) {
    const LevelState &L = m.lv;
    const uint32_t cur = L.cur, n_front = L.n_front, limit = L.limit, rows_per = L.tile_rows;
    const uint32_t base = j * rows_per, rows = std::min(rows_per, n_front - base);
    const uint32_t W = m.N;
    std::vector<uint32_t> fresh, s(W);
    uint64_t edges = 0, dead = 0;
    for (uint32_t i = 0; i < rows; ++i) {
        if (m.abort.load(std::memory_order_relaxed))
            break;
        const uint32_t slot = m.fr[cur][base + i];                    // frontier entry (payload)
        std::memcpy(s.data(), &m.t->data[(size_t)slot * W], W * 4u);  // row of an earlier level
        uint32_t n = 0;
        for (uint32_t p = 0; p < m.N; ++p) {
            std::vector<uint32_t> v = s;
            v[p] = (v[p] + 1) % m.L;
            uint32_t at = 0;
            const Code c = find_or_put(*m.t, v.data(), at);
            if (c == kNew)
                fresh.push_back(at);
            else if (c != kSeen)
                q.error.store(1, std::memory_order_relaxed);
            ++n;
        }
        edges += n;
        dead += n == 0;
    }
    // append: one reservation on the level's cursor, then the entries; the
    // level aborts once the cursor passes its limit
    if (!fresh.empty()) {
        const uint32_t b = m.n_next.fetch_add((uint32_t)fresh.size(), std::memory_order_relaxed);
        if ((uint64_t)b + fresh.size() > limit)
            m.abort.store(1, std::memory_order_relaxed);
        std::copy(fresh.begin(), fresh.end(), m.fr[cur ^ 1u].begin() + b);
    }
    m.edges.fetch_add(edges, std::memory_order_relaxed);
    m.dead.fetch_add(dead, std::memory_order_relaxed);
}

// Finalise model i's level (its last tile is done).  Returns true when the
// model has a next level, whose tile 0 the caller then expands; on_done(i)
// runs once the model is finished.
template <class OnDone>
bool finalize(std::vector<Model> &ms, uint32_t i, Queue &q, OnDone on_done) {
    Model &m = ms[i];
    LevelState &L = m.lv;
    const uint32_t n_next = m.n_next.load(std::memory_order_relaxed);
    bool done = false;
    uint32_t nt = 0;
    if (m.cap && n_next > L.limit) {
        for (uint32_t k = 0; k < n_next; ++k)   // discard the level: free its claims
            m.t->slot[m.fr[L.cur ^ 1u][k]].store(0, std::memory_order_relaxed);
        m.capped = true;
        done = true;
    } else {
        m.p_edges += m.edges.load(std::memory_order_relaxed);
        m.p_dead += m.dead.load(std::memory_order_relaxed);
        if (n_next == 0) {
            done = true;
        } else {
            m.levels.push_back(n_next);
            m.total += n_next;
            nt = (n_next + kTileRows - 1) / kTileRows;
            L.cur ^= 1u;
            L.n_front = n_next;
            L.limit = m.cap ? (uint32_t)std::min<uint64_t>(m.cap - m.total, 0xFFFFFFFFu) : 0xFFFFFFFFu;
            L.tiles_total = nt;
            L.tile_rows = kTileRows;
            L.tiles_done.store(0, std::memory_order_relaxed);
        }
    }
    m.n_next.store(0, std::memory_order_relaxed);
    m.abort.store(0, std::memory_order_relaxed);
    m.edges.store(0, std::memory_order_relaxed);
    m.dead.store(0, std::memory_order_relaxed);
    if (done) {
        q.remaining.fetch_sub(1, std::memory_order_release);
        on_done(i);
        return false;
    }
    if (nt > 1) {
        // enqueue tiles 1..: wait for each cell to be free, fill, publish
        const uint64_t pos0 = q.tail.fetch_add(nt - 1, std::memory_order_relaxed);
        for (uint32_t k = 1; k < nt; ++k)
            if (!ring_put(q, pos0 + k - 1, i, k)) {
                q.error.store(2, std::memory_order_relaxed);
                return false;
            }
    }
    return true;
}

void worker(std::vector<Model> &ms, Queue &q) {
    bool kept = false;
    uint32_t mi = 0, tile = 0;
    while (true) {
        if (kept) {
            tile = 0;
        } else {
            const uint64_t pos = q.head.fetch_add(1, std::memory_order_relaxed);
            bool timed_out = false;
            const bool got = ring_take(
                q, pos, mi, tile,
                [&] {
                    return q.remaining.load(std::memory_order_relaxed) == 0 ||
                           q.error.load(std::memory_order_relaxed) != 0;
                },
                timed_out);
            if (timed_out)
                q.error.store(3, std::memory_order_relaxed);
            if (!got)
                return;
        }
        Model &m = ms[mi];
        expand_tile(m, tile, q);
        // the tile's stores completed (vmcnt(0)), and the level's tile count
        // read, before the tile is counted as done
        const uint32_t total = m.lv.tiles_total;
#if PLANT == 5
        const uint32_t done = m.lv.tiles_done.fetch_add(1, std::memory_order_relaxed) + 1;
#else
        const uint32_t done = m.lv.tiles_done.fetch_add(1, std::memory_order_acq_rel) + 1;
#endif
        kept = done == total && finalize(ms, mi, q, [](uint32_t) {});
    }
}

// Sequential BFS of a cyclic model with the same level-prefix cap.
void bfs(uint32_t N, uint32_t L, uint64_t cap, std::vector<uint64_t> &levels, uint64_t &edges, bool &capped,
         std::set<std::vector<uint32_t>> &seen) {
    std::vector<std::vector<uint32_t>> cur{std::vector<uint32_t>(N, 0)};
    seen = {cur[0]};
    levels = {1};
    edges = 0;
    capped = false;
    while (true) {
        std::vector<std::vector<uint32_t>> next;
        for (auto &s : cur)
            for (uint32_t p = 0; p < N; ++p) {
                auto v = s;
                v[p] = (v[p] + 1) % L;
                if (seen.insert(v).second)
                    next.push_back(v);
            }
        if (cap && seen.size() > cap) {
            for (auto &v : next)
                seen.erase(v);
            capped = true;
            return;
        }
        edges += cur.size() * N;
        if (next.empty())
            return;
        levels.push_back(next.size());
        cur.swap(next);
    }
}

int part2() {
    // (N, L, cap): widths 2..6, some capped in the middle of a level
    const uint32_t spec[][3] = {{2, 9, 0},  {3, 7, 0},   {4, 5, 0},  {5, 4, 0},    {6, 3, 0},   {3, 12, 500},
                                {4, 6, 700}, {5, 5, 1000}, {2, 30, 0}, {6, 4, 2000}, {4, 7, 0}, {3, 3, 0}};
    const uint32_t n_models = sizeof(spec) / sizeof(spec[0]);
    std::vector<Model> ms(n_models);
    // expected results first; the ring holds one full level of every model
    // (as the kernel's does), so its cells are reused many times over
    std::vector<std::vector<uint64_t>> w_levels(n_models);
    std::vector<uint64_t> w_edges(n_models);
    std::vector<bool> w_capped(n_models);
    std::vector<std::set<std::vector<uint32_t>>> w_set(n_models);
    uint64_t pending = n_models;
    for (uint32_t i = 0; i < n_models; ++i) {
        bool c = false;
        bfs(spec[i][0], spec[i][1], spec[i][2], w_levels[i], w_edges[i], c, w_set[i]);
        w_capped[i] = c;
        // only kept levels are ever enqueued (a discarded one is not expanded)
        const uint64_t widest = *std::max_element(w_levels[i].begin(), w_levels[i].end());
        pending += (widest + kTileRows - 1) / kTileRows + 1;
    }
    for (uint32_t i = 0; i < n_models; ++i) {
        Model &m = ms[i];
        m.N = spec[i][0];
        m.L = spec[i][1];
        m.cap = spec[i][2];
        uint64_t states = 1;
        for (uint32_t p = 0; p < m.N; ++p)
            states *= m.L;
        uint32_t cap = 64;
        while (cap < 2 * states + 64)
            cap <<= 1;
        m.t.reset(new Table(m.N, 8, cap));
        m.fr[0].assign(cap, 0);
        m.fr[1].assign(cap, 0);
        // level 0: insert s0 (before the workers start)
        std::vector<uint32_t> s0(m.N, 0);
        uint32_t at = 0;
        if (find_or_put(*m.t, s0.data(), at) != kNew)
            return 1;
        m.fr[0][0] = at;
        m.lv.cur = 0;
        m.lv.n_front = 1;
        m.lv.limit = m.cap ? (uint32_t)(m.cap - 1) : 0xFFFFFFFFu;
        m.lv.tiles_total = 1;
        m.lv.tile_rows = kTileRows;
    }
    Queue q;
    uint64_t cells = 16;
    while (cells < pending)
        cells <<= 1;
    q.mask = cells - 1;
    q.ring.reset(new Cell[cells]);
    for (uint64_t p = 0; p < cells; ++p) {
        // positions 0..n-1 hold tile 0 of every model's level 0
        q.ring[p].seq.store(p < n_models ? p + 1 : p, std::memory_order_relaxed);
        q.ring[p].model = p < n_models ? (uint32_t)p : 0u;
        q.ring[p].tile = 0;
    }
    q.tail.store(n_models);
    q.remaining.store(n_models);
    std::vector<std::thread> th;
    for (int w = 0; w < 8; ++w)
        th.emplace_back(worker, std::ref(ms), std::ref(q));
    for (auto &h : th)
        h.join();
    int bad = q.error.load() ? 1 : 0;
    uint64_t items = 0;
    for (uint32_t i = 0; i < n_models; ++i) {
        Model &m = ms[i];
        const std::vector<uint64_t> &levels = w_levels[i];
        const uint64_t edges = w_edges[i];
        const bool capped = w_capped[i];
        const std::set<std::vector<uint32_t>> &want = w_set[i];
        for (uint64_t n : m.levels)
            items += (n + kTileRows - 1) / kTileRows;
        std::set<std::vector<uint32_t>> got;
        uint32_t claimed = 0;
        for (uint32_t s = 0; s < m.t->capacity(); ++s) {
            const uint64_t v = m.t->slot[s].load();
            if (v & kDone)
                got.insert(std::vector<uint32_t>(&m.t->data[(size_t)s * m.N], &m.t->data[(size_t)s * m.N] + m.N));
            else if (v)
                ++claimed;
        }
        const bool ok = levels == m.levels && edges == m.p_edges && capped == m.capped && got == want &&
                        claimed == 0 && m.total == want.size();
        bad += !ok;
        printf("part2: model %u (%u x %u, cap %llu): %llu states in %zu levels, %llu edges, capped %d %s\n", i, m.N,
               m.L, (unsigned long long)m.cap, (unsigned long long)m.total, m.levels.size(),
               (unsigned long long)m.p_edges, (int)m.capped, ok ? "ok" : "WRONG");
    }
    printf("part2: %llu tiles through a ring of %llu cells\n", (unsigned long long)items,
           (unsigned long long)cells);
    if (items <= cells)
        ++bad;   // the ring was never reused: the test would prove little
    return bad;
}

// ---------------------------------------------------------------- part 3 ---
// The ring alone, with no other synchronisation between its users: four
// producers reserve positions on the tail and fill them, four consumers
// reserve positions on the head and take them, through eight cells.  Every
// item must come out exactly once and intact.
int part3() {
    Queue q;
    q.mask = 7;
    q.ring.reset(new Cell[8]);
    for (uint64_t p = 0; p < 8; ++p) {
        q.ring[p].seq.store(p, std::memory_order_relaxed);
        q.ring[p].model = q.ring[p].tile = 0;
    }
    const uint32_t per = 4000, np = 4, nc = 4, total = per * np;
    std::vector<std::vector<uint32_t>> got(nc);
    std::atomic<int> bad{0};
    std::vector<std::thread> th;
    for (uint32_t w = 0; w < np; ++w)
        th.emplace_back([&, w] {
            for (uint32_t k = 0; k < per; ++k) {
                const uint32_t id = w * per + k;
                if (!ring_put(q, q.tail.fetch_add(1, std::memory_order_relaxed), id, id ^ 0x5A5A5A5Au))
                    bad.fetch_add(1);
            }
        });
    for (uint32_t w = 0; w < nc; ++w)
        th.emplace_back([&, w] {
            while (true) {
                const uint64_t pos = q.head.fetch_add(1, std::memory_order_relaxed);
                if (pos >= total)
                    return;
                uint32_t a = 0, b = 0;
                bool timed_out = false;
                if (!ring_take(q, pos, a, b, [] { return false; }, timed_out) || b != (a ^ 0x5A5A5A5Au))
                    bad.fetch_add(1);
                got[w].push_back(a);
            }
        });
    for (auto &h : th)
        h.join();
    std::vector<uint32_t> all;
    for (auto &g : got)
        all.insert(all.end(), g.begin(), g.end());
    std::sort(all.begin(), all.end());
    for (uint32_t i = 0; i < all.size(); ++i)
        if (all[i] != i)
            bad.fetch_add(1);
    if (all.size() != total)
        bad.fetch_add(1);
    printf("part3: %zu items through 8 cells, errors %d\n", all.size(), bad.load());
    return bad.load();
}

// ---------------------------------------------------------------- part 4 ---
constexpr uint32_t kSlots = 4, kAdmitRing = 8, kDoneRing = 8, kQuiet = 400, kStallPolls = 1u << 22;

struct DoneRec {
    std::atomic<uint64_t> seq{0};
    uint32_t slot = 0, n_levels = 0;   // payload
};

struct Server {
    std::vector<Model> ms{kSlots};             // per-slot query state (payload)
    Queue q;
    std::atomic<uint64_t> admit_tail{0}, admit_head{0}, done_tail{0};
    uint32_t admit_slot[kAdmitRing] = {};      // payload
    DoneRec done[kDoneRing];
    std::atomic<uint32_t> closing{0}, stop{0}, beat{0}, left{0}, alive{0};
};

// One worker of a launch: the kernel's decision loop.
void serve_worker(Server &S) {
    Queue &q = S.q;
    bool kept = false, holding = false;
    uint32_t mi = 0, tile = 0, quiet = 0, stall = 0, last_beat = 0;
    uint64_t pos = 0;
    auto on_done = [&S](uint32_t i) {
        const uint64_t p = S.done_tail.fetch_add(1, std::memory_order_relaxed);
        DoneRec &r = S.done[p % kDoneRing];
#if PLANT == 8
        r.seq.store(p + 1, std::memory_order_release);
        r.slot = i;
        r.n_levels = (uint32_t)S.ms[i].levels.size();
#else
        r.slot = i;
        r.n_levels = (uint32_t)S.ms[i].levels.size();
#if PLANT == 7
        r.seq.store(p + 1, std::memory_order_relaxed);
#else
        r.seq.store(p + 1, std::memory_order_release);   // system-scope release
#endif
#endif
    };
    while (true) {
        if (q.error.load(std::memory_order_relaxed))
            break;
        bool have = false, admit = false;
        if (kept) {
            tile = 0;
            have = true;
        } else {
            if (!holding) {
                pos = q.head.fetch_add(1, std::memory_order_relaxed);
                holding = true;
            }
            Cell &c = q.ring[pos & q.mask];
            if (c.seq.load(std::memory_order_acquire) == pos + 1) {
                mi = c.model;
                tile = c.tile;
                c.seq.store(pos + q.mask + 1, std::memory_order_release);
                holding = false;
                have = true;
            } else {
                const bool closing = S.closing.load(std::memory_order_relaxed) != 0;
                const uint64_t ah = S.admit_head.load(std::memory_order_relaxed);
                if (!closing && ah < S.admit_tail.load(std::memory_order_acquire)) {
                    q.remaining.fetch_add(1, std::memory_order_seq_cst);
                    uint64_t e = ah;
                    if (S.closing.load(std::memory_order_seq_cst) == 0 &&
                        S.admit_head.compare_exchange_strong(e, ah + 1, std::memory_order_relaxed)) {
                        if (S.left.load(std::memory_order_seq_cst) != 0)
                            q.error.store(5, std::memory_order_relaxed);   // admitted to a draining launch
                        mi = S.admit_slot[ah % kAdmitRing];
                        admit = true;
                    } else {
                        q.remaining.fetch_sub(1, std::memory_order_relaxed);
                    }
                } else if (q.remaining.load(std::memory_order_relaxed) != 0) {
                    quiet = 0;
                } else if (++quiet >= kQuiet || closing || S.stop.load(std::memory_order_relaxed)) {
                    S.closing.exchange(1, std::memory_order_seq_cst);
                    if (q.remaining.load(std::memory_order_seq_cst) == 0) {
                        S.left.fetch_add(1, std::memory_order_seq_cst);
                        break;
                    }
                }
                if (!admit) {
                    const uint32_t b = S.beat.load(std::memory_order_relaxed);
                    stall = b == last_beat ? stall + 1 : 0;
                    last_beat = b;
                    if (stall > kStallPolls) {
                        q.error.store(4, std::memory_order_relaxed);
                        break;
                    }
                    std::this_thread::yield();
                    continue;
                }
            }
        }
        stall = 0;
        Model &m = S.ms[mi];
        if (admit) {
            // the slot's constants and table come from the host; s0 and
            // level 0 are set up here, and tile 0 is this worker's
            m.levels.assign(1, 1);
            m.total = 1;
            m.p_edges = m.p_dead = 0;
            m.capped = false;
            m.n_next.store(0, std::memory_order_relaxed);
            m.abort.store(0, std::memory_order_relaxed);
            m.edges.store(0, std::memory_order_relaxed);
            m.dead.store(0, std::memory_order_relaxed);
            std::vector<uint32_t> s0(m.N, 0);
            uint32_t at = 0;
            if (find_or_put(*m.t, s0.data(), at) != kNew)
                q.error.store(6, std::memory_order_relaxed);
            m.fr[0][0] = at;
            m.lv.cur = 0;
            m.lv.n_front = 1;
            m.lv.limit = m.cap ? (uint32_t)(m.cap - 1) : 0xFFFFFFFFu;
            m.lv.tiles_total = 1;
            m.lv.tile_rows = kTileRows;
            m.lv.tiles_done.store(0, std::memory_order_relaxed);
#if PLANT == 16
            kept = true;
#else
            // tile 0 goes to the queue like any other tile: this worker still
            // holds the position it reserved before admitting, and a worker
            // that keeps tiles for itself while holding one leaves the item
            // that lands there waiting for its whole chain of levels, until
            // the ring wraps onto that cell and every producer stops
            if (!ring_put(q, q.tail.fetch_add(1, std::memory_order_relaxed), mi, 0)) {
                q.error.store(2, std::memory_order_relaxed);
                break;
            }
#endif
            continue;
        }
        expand_tile(m, tile, q);
        const uint32_t total = m.lv.tiles_total;
        const uint32_t done = m.lv.tiles_done.fetch_add(1, std::memory_order_acq_rel) + 1;
        S.beat.fetch_add(1, std::memory_order_relaxed);
        kept = done == total && finalize(S.ms, mi, q, on_done);
    }
    S.alive.fetch_sub(1, std::memory_order_release);
}

int part4() {
    // queries: cyclic models, some capped, each with its expected result
    struct Spec {
        uint32_t N, L;
        uint64_t cap;
    };
    const Spec specs[] = {{2, 9, 0}, {3, 5, 0}, {4, 4, 0}, {2, 20, 0}, {3, 6, 60}, {4, 3, 40}, {5, 3, 0}, {3, 4, 0}};
    const uint32_t n_specs = sizeof(specs) / sizeof(specs[0]);
    std::vector<std::vector<uint64_t>> w_levels(n_specs);
    std::vector<uint64_t> w_edges(n_specs);
    std::vector<bool> w_capped(n_specs);
    std::vector<std::set<std::vector<uint32_t>>> w_set(n_specs);
    uint64_t widest = 0;
    for (uint32_t k = 0; k < n_specs; ++k) {
        bool c = false;
        bfs(specs[k].N, specs[k].L, specs[k].cap, w_levels[k], w_edges[k], c, w_set[k]);
        w_capped[k] = c;
        widest = std::max(widest, *std::max_element(w_levels[k].begin(), w_levels[k].end()));
    }
    Server S;
    Queue &q = S.q;
    // the ring holds a full level of every slot plus one held position per worker
    const uint32_t workers = 4;
    uint64_t cells = 16;
    while (cells < kSlots * ((widest + kTileRows - 1) / kTileRows + 1) + workers)
        cells <<= 1;
    q.mask = cells - 1;
    q.ring.reset(new Cell[cells]);
    for (uint64_t p = 0; p < cells; ++p) {
        q.ring[p].seq.store(p, std::memory_order_relaxed);
        q.ring[p].model = q.ring[p].tile = 0;
    }
    const uint32_t n_queries = 160;
    std::vector<uint32_t> slot_spec(kSlots, 0), free_slots;
    for (uint32_t i = 0; i < kSlots; ++i)
        free_slots.push_back(i);
    std::vector<std::thread> launch;
    uint64_t posted = 0, done_head = 0, launches = 0, drains = 0;
    uint32_t live = 0, bad = 0, completed = 0, seed = 12345;
    auto rnd = [&seed] {
        seed = seed * 1103515245u + 12345u;
        return seed >> 16;
    };
    auto start_launch = [&] {
        // no worker of the last launch is alive (joined): positions it held
        // unfilled are given back, admissions reopen
        q.head.store(q.tail.load(std::memory_order_relaxed), std::memory_order_relaxed);
        S.closing.store(0, std::memory_order_relaxed);
        S.left.store(0, std::memory_order_relaxed);
        S.alive.store(workers, std::memory_order_relaxed);
        for (uint32_t w = 0; w < workers; ++w)
            launch.emplace_back(serve_worker, std::ref(S));
        ++launches;
    };
    auto join_launch = [&] {
        for (auto &t : launch)
            t.join();
        launch.clear();
    };
    auto collect = [&] {
        while (true) {
            DoneRec &r = S.done[done_head % kDoneRing];
            if (r.seq.load(std::memory_order_acquire) != done_head + 1)
                break;
            const uint32_t slot = r.slot, nl = r.n_levels;
            ++done_head;
            Model &m = S.ms[slot];
            const uint32_t k = slot_spec[slot];
            std::set<std::vector<uint32_t>> got;
            for (uint32_t s = 0; s < m.t->capacity(); ++s)
                if (m.t->slot[s].load(std::memory_order_relaxed) & kDone)
                    got.insert(std::vector<uint32_t>(&m.t->data[(size_t)s * m.N], &m.t->data[(size_t)s * m.N] + m.N));
            const bool ok = nl == m.levels.size() && m.levels == w_levels[k] && m.p_edges == w_edges[k] &&
                            m.capped == w_capped[k] && got == w_set[k];
            if (!ok) {
                ++bad;
                printf("part4: query on slot %u (model %u) WRONG\n", slot, k);
            }
            ++completed;
            --live;
            free_slots.push_back(slot);
        }
    };
    for (uint32_t n = 0; n < n_queries && !q.error.load();) {
        collect();
        if (S.alive.load(std::memory_order_acquire) == 0 && !launch.empty())
            join_launch();
        if (!free_slots.empty()) {
            // post: the slot's constants and a fresh table, the entry, then the tail
            const uint32_t slot = free_slots.back();
            free_slots.pop_back();
            const uint32_t k = rnd() % n_specs;
            Model &m = S.ms[slot];
            m.N = specs[k].N;
            m.L = specs[k].L;
            m.cap = specs[k].cap;
            uint64_t states = 1;
            for (uint32_t p = 0; p < m.N; ++p)
                states *= m.L;
            uint32_t cap = 64;
            while (cap < 2 * states + 64)
                cap <<= 1;
            m.t.reset(new Table(m.N, 8, cap));
            m.fr[0].assign(cap, 0);
            m.fr[1].assign(cap, 0);
            slot_spec[slot] = k;
            S.admit_slot[posted % kAdmitRing] = slot;
            ++posted;
#if PLANT == 6
            S.admit_tail.store(posted, std::memory_order_relaxed);
#else
            S.admit_tail.store(posted, std::memory_order_release);   // copies in stream order
#endif
            ++live;
            ++n;
            if (rnd() % 16 == 0 && !launch.empty()) {
                S.closing.store(1, std::memory_order_relaxed);      // drain for a wider query
                ++drains;
            }
        }
        if (launch.empty() && live > 0)
            start_launch();
        if (rnd() % 8 == 0)
            std::this_thread::sleep_for(std::chrono::microseconds(rnd() % 3000));   // quiet spells
        else
            std::this_thread::yield();
    }
    // the rest: wait for every query, relaunching for queries posted too late
    for (uint64_t spins = 0; live > 0 && !q.error.load(); ++spins) {
        collect();
        if (S.alive.load(std::memory_order_acquire) == 0 && !launch.empty())
            join_launch();
        if (launch.empty() && live > 0)
            start_launch();
        std::this_thread::yield();
        if (spins > kSpin) {
            ++bad;
            break;
        }
    }
    S.stop.store(1, std::memory_order_relaxed);
    join_launch();
    if (q.error.load()) {
        printf("part4: error %u\n", q.error.load());
        ++bad;
    }
    printf("part4: %u queries on %u slots in %llu launches (%llu drains asked), errors %u\n", completed, kSlots,
           (unsigned long long)launches, (unsigned long long)drains, bad);
    if (launches < 2 || completed != n_queries)
        ++bad;   // no relaunch was exercised, or a query was lost
    return (int)bad;
}


// ---------------------------------------------------------------- part 5 ---
// A reusable barrier for the lanes of one pass (the workgroup barrier).
struct PassBarrier {
    std::atomic<uint32_t> arrived{0}, phase{0};
    uint32_t n;
    explicit PassBarrier(uint32_t n_) : n(n_) {}
    void wait() {
        const uint32_t ph = phase.load(std::memory_order_acquire);
        if (arrived.fetch_add(1, std::memory_order_acq_rel) + 1 == n) {
            arrived.store(0, std::memory_order_relaxed);
            phase.store(ph + 1, std::memory_order_release);
        } else {
            while (phase.load(std::memory_order_acquire) == ph)
                std::this_thread::yield();
        }
    }
};

int part5() {
    constexpr uint32_t kLanes = 32, kCells = 2 * kLanes, W = 6;
    constexpr int kTrials = 60;
    enum HashMode { kFull, kOneBit, kCollide };
    std::mt19937_64 rnd(0x5EED5);
    unsigned bad = 0, merged_total = 0;
    for (int trial = 0; trial < 3 * kTrials; ++trial) {
        const HashMode mode = HashMode(trial % 3);
        // the pass's successors: drawn from a small pool, so that many repeat
        const uint32_t pool = 2 + (uint32_t)(rnd() % 12);
        std::vector<std::vector<uint32_t>> pool_rows(pool, std::vector<uint32_t>(W));
        for (auto &r : pool_rows)
            for (auto &w : r)
                w = (uint32_t)(rnd() % 4);
        std::vector<uint32_t> pick(kLanes);
        for (auto &x : pick)
            x = (uint32_t)(rnd() % pool);
        std::vector<uint32_t> succ((size_t)kLanes * W);   // payload: the pass's list
        std::unique_ptr<std::atomic<uint32_t>[]> cells(new std::atomic<uint32_t>[kCells]);
        for (uint32_t i = 0; i < kCells; ++i)
            cells[i].store(0, std::memory_order_relaxed);
        std::vector<uint8_t> skip(kLanes, 0);
        std::vector<uint32_t> rep(kLanes, 0);
        PassBarrier bar(kLanes);
        auto lane = [&](uint32_t l) {
            uint32_t *mine = &succ[(size_t)l * W];
            for (uint32_t w = 0; w < W; ++w)
                mine[w] = pool_rows[pick[l]][w];
#if PLANT != 10
            bar.wait();   // the list is complete (the pass barrier)
#endif
            uint64_t h = hash_row(mine, W);
            if (mode == kCollide)
                h = mix64(h & 3);      // four hashes for the whole pool
            uint32_t tag = (uint32_t)(h >> 41) << 9;
            if (mode == kOneBit)
                tag &= 1u << 9;
            uint32_t c = (uint32_t)(h >> 32) & (kCells - 1), other = 0;
            for (;;) {
                uint32_t old = 0;
                if (cells[c].compare_exchange_strong(old, tag | (l + 1), std::memory_order_relaxed))
                    break;
                if ((old & ~511u) == tag) {
                    other = old & 511u;
                    break;
                }
                c = (c + 1) & (kCells - 1);
            }
            if (other) {
                const uint32_t *o = &succ[(size_t)(other - 1) * W];
                bool eq = true;
#if PLANT != 9
                for (uint32_t w = 0; w < W; ++w)
                    eq = eq && mine[w] == o[w];
#endif
                skip[l] = eq;
                rep[l] = other - 1;
            }
        };
        std::vector<std::thread> th;
        for (uint32_t l = 0; l < kLanes; ++l)
            th.emplace_back(lane, l);
        for (auto &t : th)
            t.join();
        // per distinct vector: the lanes that probe the table
        std::map<std::vector<uint32_t>, uint32_t> probing;
        for (uint32_t l = 0; l < kLanes; ++l)
            probing[pool_rows[pick[l]]] += !skip[l];
        for (auto &kv : probing)
            if (kv.second == 0)
                ++bad;   // a state no lane puts into the table: lost
        std::set<uint64_t> hashes;
        for (auto &kv : probing)
            hashes.insert(hash_row(kv.first.data(), W));
        const bool distinct = hashes.size() == probing.size();
        for (uint32_t l = 0; l < kLanes; ++l) {
            if (!skip[l])
                continue;
            ++merged_total;
            if (skip[rep[l]] || pool_rows[pick[rep[l]]] != pool_rows[pick[l]])
                ++bad;   // merged into a lane that does not probe, or into another state
        }
        if (mode == kFull && distinct)
            for (auto &kv : probing)
                if (kv.second != 1)
                    ++bad;   // a repeat that the full hash should have merged
    }
    printf("part5: %d passes, %u successors merged, errors %u\n", 3 * kTrials, merged_total, bad);
    if (merged_total == 0)
        ++bad;
    return (int)bad;
}


// ---------------------------------------------------------------- part 6 ---
constexpr uint32_t kSegsM = 8;

struct SegLevel {
    uint32_t size;                                   // entries per segment
    std::unique_ptr<std::atomic<uint32_t>[]> cur;    // append cursors
    std::vector<uint32_t> buf;                       // payload: kSegsM * size entries
    std::atomic<uint32_t> abort{0}, efull{0};
    explicit SegLevel(uint32_t s) : size(s), cur(new std::atomic<uint32_t>[kSegsM]), buf((size_t)kSegsM * s, 0) {
        for (uint32_t k = 0; k < kSegsM; ++k)
            cur[k].store(0, std::memory_order_relaxed);
    }
};

// One workgroup's state across its tiles (the kernel's LDS scalars).
struct SegWorker {
    uint32_t b;                       // workgroup index
    uint32_t est = 0;                 // 8 x the largest cursor seen
    bool eager = false, aborted = false;
    std::vector<uint32_t> nbuf;       // buffered new states
};

void seg_flush(SegLevel &lv, SegWorker &w, uint32_t limit, uint32_t room) {
    const uint32_t nn = (uint32_t)w.nbuf.size();
    if (nn) {
        struct Piece { uint32_t pos, off, n; };
        Piece pc[2 * kSegsM];
        uint32_t k = w.b & (kSegsM - 1), rem = nn, np = 0, off = 0, first = 0;
        for (uint32_t tries = 0; rem && tries < 2 * kSegsM; ++tries) {
            const uint32_t b = lv.cur[k].fetch_add(rem, std::memory_order_relaxed);
            if (tries == 0)
                first = b;
#if PLANT == 11
            if (b < lv.size) {
                const uint32_t n = rem;
#else
            if (b < lv.size) {
                const uint32_t n = std::min(rem, lv.size - b);
#endif
                pc[np++] = Piece{k * lv.size + b, off, n};
                off += n;
                rem -= n;
            }
            k = (k + 1) & (kSegsM - 1);
        }
        if (rem)
            lv.efull.store(1, std::memory_order_relaxed);
        w.est = std::max<uint32_t>(w.est, (uint32_t)std::min<uint64_t>(8ull * ((uint64_t)first + nn), 0xFFFFFFFFull));
        if (limit != 0xFFFFFFFFu && ((uint64_t)w.est + room > limit || w.eager)) {
            w.eager = true;
            uint64_t total = 0;
#if PLANT == 12
            total = w.est;
#else
            for (uint32_t q = 0; q < kSegsM; ++q)
                total += std::min(lv.cur[q].load(std::memory_order_relaxed), lv.size);
#endif
            if (total > limit) {
                lv.abort.store(1, std::memory_order_relaxed);
                w.aborted = true;
            }
        }
        for (uint32_t p = 0; p < np; ++p)
            for (uint32_t i = 0; i < pc[p].n && pc[p].pos + i < lv.buf.size(); ++i)
                lv.buf[pc[p].pos + i] = w.nbuf[pc[p].off + i];
        w.nbuf.clear();
    }
    if (w.eager && !w.aborted)
        w.aborted = lv.abort.load(std::memory_order_relaxed) != 0;
}

int part6() {
    constexpr uint32_t kPass = 32, kBuf = 3 * kPass, kTileMax = 4 * kPass;
    std::mt19937_64 rnd(0x5E6);
    unsigned bad = 0, aborted_levels = 0, efull_levels = 0, uneven = 0;
    const uint32_t worker_counts[] = {1, 3, 8, 9, 13, 16};
    for (int trial = 0; trial < 48; ++trial) {
        const uint32_t nw = worker_counts[trial % 6];
        const uint32_t size = 64 + (uint32_t)(rnd() % 512);
        const uint32_t tiles = 8 + (uint32_t)(rnd() % 96);
        // new states per tile, each a distinct id: tile * kTileMax + i
        std::vector<uint32_t> out(tiles);
        uint64_t produced = 0;
        for (auto &o : out) {
            o = (uint32_t)(rnd() % (kTileMax + 1));
            produced += o;
        }
        const int kind = (trial / 6) % 4;   // no cap, cap inside, cap above, segments too small
        uint32_t limit = 0xFFFFFFFFu;
        if (kind == 1)
            limit = (uint32_t)(produced / 2);
        else if (kind == 2)
            limit = (uint32_t)(produced + 1);
        const uint32_t seg = kind == 3 ? std::max<uint32_t>(1u, (uint32_t)(produced / (kSegsM + 2))) : size;
        SegLevel lv(kind == 3 ? seg : std::max<uint32_t>(size, (uint32_t)(produced / kSegsM) + kTileMax));
        const uint32_t room = nw * kBuf + kPass;
        std::vector<uint64_t> pushed(nw, 0);
        auto worker = [&](uint32_t b) {
            SegWorker w;
            w.b = b;
            for (uint32_t t = b; t < tiles; t += nw) {
                if (lv.abort.load(std::memory_order_relaxed))
                    break;   // the tile's start
                for (uint32_t p0 = 0; p0 < out[t] && !w.aborted; p0 += kPass) {
                    for (uint32_t i = p0; i < std::min(out[t], p0 + kPass); ++i)
                        w.nbuf.push_back(t * kTileMax + i);
                    if (w.eager || w.nbuf.size() > kBuf - kPass) {
                        pushed[b] += w.nbuf.size();
                        seg_flush(lv, w, limit, room);
                    }
                }
                if (w.aborted)
                    break;
            }
            pushed[b] += w.nbuf.size();
            seg_flush(lv, w, limit, room);   // the end of the launch
        };
        std::vector<std::thread> th;
        for (uint32_t b = 0; b < nw; ++b)
            th.emplace_back(worker, b);
        for (auto &t : th)
            t.join();
        uint64_t total = 0, n_push = 0;
        std::vector<uint32_t> seen_id((size_t)tiles * kTileMax, 0);
        uint32_t lo = 0xFFFFFFFFu, hi = 0;
        for (uint32_t k = 0; k < kSegsM; ++k) {
            const uint32_t n = std::min(lv.cur[k].load(), lv.size);
            lo = std::min(lo, n);
            hi = std::max(hi, n);
            total += n;
            for (uint32_t i = 0; i < n; ++i) {
                const uint32_t id = lv.buf[(size_t)k * lv.size + i];
                if (id >= seen_id.size() || id % kTileMax >= out[id / kTileMax] || seen_id[id]++) {
                    ++bad;   // not a state of this level, or one listed twice
                    break;
                }
            }
        }
        for (auto x : pushed)
            n_push += x;
        const bool efull = lv.efull.load() != 0;
        uneven += hi > lo + kBuf;
        if (efull != (n_push > (uint64_t)kSegsM * lv.size)) {
            printf("part6: trial %d: EFULL %d with %llu states for %u entries\n", trial, (int)efull,
                   (unsigned long long)n_push, kSegsM * lv.size);
            ++bad;
        }
        if (!efull && total != n_push) {
            printf("part6: trial %d: %llu entries listed, %llu appended\n", trial, (unsigned long long)total,
                   (unsigned long long)n_push);
            ++bad;   // an appended state missing from the segments
        }
        if (!lv.abort.load() && !efull && n_push != produced)
            ++bad;   // a level that was not aborted lost states
        if (lv.abort.load()) {
            ++aborted_levels;
            if (total <= limit) {
                printf("part6: trial %d: abort with %llu states, cap %u\n", trial, (unsigned long long)total, limit);
                ++bad;   // aborted below the cap
            }
        }
        efull_levels += efull;
    }
    printf("part6: 48 levels, %u aborted, %u with EFULL, %u filled unevenly, errors %u\n", aborted_levels,
           efull_levels, uneven, bad);
    if (aborted_levels == 0 || efull_levels == 0 || uneven == 0)
        ++bad;   // a case the trials were meant to reach
    return (int)bad;
}


// ---------------------------------------------------------------- part 7 ---
constexpr uint32_t kNoEntryM = 0xFFFFFFFFu;
// polls without progress before a worker gives up (the kernel's bound is
// about a second; a lost entry must end a run here within seconds)
constexpr uint32_t kAsyncSpin = 1u << 20;

// The explored model: N cyclic L-state processes (W = N), or a broom (W = 2):
// a chain (a, 0) -> (a + 1, 0) for a < L whose last state (L, 0) has F
// successors (L, 1..F), each a deadlock.
struct AsyncModel {
    bool broom;
    uint32_t N, L, F;
    uint32_t W() const { return broom ? 2u : N; }
    void successors(const uint32_t *s, std::vector<std::vector<uint32_t>> &out) const {
        out.clear();
        if (!broom) {
            for (uint32_t p = 0; p < N; ++p) {
                std::vector<uint32_t> v(s, s + N);
                v[p] = (v[p] + 1) % L;
                out.push_back(v);
            }
        } else if (s[1] == 0 && s[0] < L) {
            out.push_back({s[0] + 1, 0});
        } else if (s[1] == 0) {
            for (uint32_t k = 1; k <= F; ++k)
                out.push_back({L, k});
        }
    }
};

struct AsyncRun {
    AsyncModel m;
    uint32_t nw;
    uint32_t chunk_size, buf_size, pass;   // entries per chunk, new-state buffer, successors per pass
    Table t;
    std::unique_ptr<std::atomic<uint32_t>[]> queue;      // slots; kNoEntryM = unwritten
    std::unique_ptr<std::atomic<uint8_t>[]> expanded;     // per entry, for the check
    std::atomic<uint32_t> n_next{1}, chunk{0}, error{0};
    std::atomic<uint64_t> work{1}, edges{0};
    uint32_t limit = 0xFFFFFFFFu;          // states stored before the run stops (the cap)
    std::atomic<uint32_t> abort{0};        // set by the append that passed it
    // the smallest cursor a leaving worker saw after deciding to leave: below
    // the final cursor, a worker left while states were still to be found
    std::atomic<uint32_t> left_at_min{0xFFFFFFFFu};
    AsyncRun(const AsyncModel &m_, uint32_t nw_, uint32_t chunk_, uint32_t buf_, uint32_t pass_, uint32_t cap)
        : m(m_), nw(nw_), chunk_size(chunk_), buf_size(buf_), pass(pass_), t(m_.W(), 8, cap),
          queue(new std::atomic<uint32_t>[cap]), expanded(new std::atomic<uint8_t>[cap]) {
        for (uint32_t i = 0; i < cap; ++i) {
            queue[i].store(kNoEntryM, std::memory_order_relaxed);
            expanded[i].store(0, std::memory_order_relaxed);
        }
    }
};

void async_worker(AsyncRun &r) {
    const uint32_t W = r.m.W(), kChunkM = r.chunk_size, kBufM = r.buf_size;
    uint64_t base = 0;
    uint32_t used = kChunkM, pushed = 0, found = 0, polls = 0, last_tail = 0;
    std::vector<uint32_t> nbuf;
    auto flush = [&]() {
#if PLANT != 15
        // states that become visible here and are not in the work count yet
        // (found in the current tile) are counted first: a worker that
        // expands one subtracts it only after reading its entry
        const uint32_t held = pushed + (uint32_t)nbuf.size();
        if (held > found) {
            r.work.fetch_add(held - found, std::memory_order_relaxed);
            found = held;
        }
#endif
        const uint32_t at = r.n_next.fetch_add((uint32_t)nbuf.size(), std::memory_order_relaxed);
        if ((uint64_t)at + nbuf.size() > r.limit)
            r.abort.store(1, std::memory_order_relaxed);   // past the cap: every worker stops
        for (uint32_t i = 0; i < nbuf.size(); ++i)
#if PLANT == 13
            r.queue[at + i].store(nbuf[i], std::memory_order_relaxed);
#else
            // the rows of these slots were written, and completed (vmcnt(0)),
            // by this worker's own inserts before the entries are stored
            r.queue[at + i].store(nbuf[i], std::memory_order_release);
#endif
        pushed += (uint32_t)nbuf.size();
        nbuf.clear();
    };
    std::vector<uint32_t> row(W);
    std::vector<std::vector<uint32_t>> succ;
    while (true) {
        enum { kStop, kExpand, kPublish } act = kStop;
        uint32_t take = 0;
        while (true) {
            if (used == kChunkM) {
                base = (uint64_t)r.chunk.fetch_add(1, std::memory_order_relaxed) * kChunkM;
                used = 0;
            }
            const uint32_t tl = r.n_next.load(std::memory_order_relaxed);
            const uint64_t end = std::min<uint64_t>(tl, base + kChunkM);
            if (!nbuf.empty() && (uint64_t)tl < base + (uint64_t)(r.nw / 4 + 1) * kChunkM &&
                (uint64_t)tl < (uint64_t)r.chunk.load(std::memory_order_relaxed) * kChunkM) {
                act = kPublish;   // another worker owns a chunk nothing was appended to
                break;
            }
            if (end > base + used) {
                take = (uint32_t)(end - base - used);
                act = kExpand;
                break;
            }
            if (!nbuf.empty()) {
                act = kPublish;   // this chunk is dry: hold nothing back
                break;
            }
            if (r.work.load(std::memory_order_relaxed) == 0 || r.abort.load(std::memory_order_relaxed) ||
                r.error.load(std::memory_order_relaxed))
                break;
            if (tl != last_tail) {
                last_tail = tl;
                polls = 0;
            } else if (++polls > kAsyncSpin) {
                r.error.store(4, std::memory_order_relaxed);
                break;
            }
            std::this_thread::yield();
        }
        const uint64_t from = base + used;
        used += take;
        if (act == kStop) {
            const uint32_t n = r.n_next.load(std::memory_order_relaxed);
            uint32_t m = r.left_at_min.load(std::memory_order_relaxed);
            while (n < m && !r.left_at_min.compare_exchange_weak(m, n, std::memory_order_relaxed)) {
            }
            break;
        }
        if (act == kPublish) {
            flush();
            continue;
        }
        if (r.abort.load(std::memory_order_relaxed))
            break;   // the tile's start: the run has passed its cap
        uint64_t edges = 0;
        bool stop = false;
        for (uint64_t e = from; e < from + take && !stop; ++e) {
            // the entry is below the cursor but may still be in flight
            uint32_t slot, spins = 0;
            while ((slot = r.queue[e].load(std::memory_order_acquire)) == kNoEntryM) {
                if (++spins > kAsyncSpin) {
                    r.error.store(4, std::memory_order_relaxed);
                    return;
                }
                if ((spins & 63u) == 0 && r.abort.load(std::memory_order_relaxed)) {
                    stop = true;   // the writer may have stopped
                    break;
                }
                std::this_thread::yield();
            }
            if (stop)
                break;
            r.expanded[e].fetch_add(1, std::memory_order_relaxed);
            std::memcpy(row.data(), &r.t.data[(size_t)slot * W], W * 4u);   // the row (payload)
            r.m.successors(row.data(), succ);
            for (auto &v : succ) {
                uint32_t at = 0;
                const Code c = find_or_put(r.t, v.data(), at);
                if (c == kNew)
                    nbuf.push_back(at);
                else if (c != kSeen)
                    r.error.store(1, std::memory_order_relaxed);
                // after every pass of successors: append when the buffer
                // nears full (in the middle of the tile)
                if (++edges % r.pass == 0 && nbuf.size() + r.pass > kBufM)
                    flush();
            }
        }
        r.edges.fetch_add(edges, std::memory_order_relaxed);
        // open states: discovered (appended or held back) - expanded
#if PLANT == 14
        const uint32_t now = pushed;
#else
        const uint32_t now = pushed + (uint32_t)nbuf.size();
#endif
        r.work.fetch_add((uint64_t)(now - found) - (uint64_t)take, std::memory_order_relaxed);
        found = now;
        if (stop)
            break;
    }
    // the end of the launch: states still held back are listed too (every
    // stored state is in the queue)
    if (!nbuf.empty())
        flush();
}

// Sequential BFS of the model: the reachable set and the edge count.
void async_reference(const AsyncModel &m, std::set<std::vector<uint32_t>> &seen, uint64_t &edges) {
    std::vector<std::vector<uint32_t>> stack{std::vector<uint32_t>(m.W(), 0)};
    std::vector<std::vector<uint32_t>> succ;
    seen = {stack[0]};
    edges = 0;
    while (!stack.empty()) {
        const auto s = stack.back();
        stack.pop_back();
        m.successors(s.data(), succ);
        edges += succ.size();
        for (auto &v : succ)
            if (seen.insert(v).second)
                stack.push_back(v);
    }
}

// One exploration; returns 1 on a wrong result, and sets `early` when a
// worker left while states were still to be found.
int async_run(const AsyncModel &m, uint32_t nw, uint32_t chunk, uint32_t buf, uint32_t pass, bool &early,
              uint32_t limit = 0xFFFFFFFFu) {
    std::set<std::vector<uint32_t>> want;
    uint64_t want_edges = 0;
    async_reference(m, want, want_edges);
    uint32_t cap = 64;
    while (cap < 4 * want.size())
        cap <<= 1;
    AsyncRun r(m, nw, chunk, buf, pass, cap);
    r.limit = limit;
    const uint32_t W = m.W();
    // s0 is entry 0, inserted before the launch
    std::vector<uint32_t> s0(W, 0);
    uint32_t slot0 = 0;
    if (find_or_put(r.t, s0.data(), slot0) != kNew)
        return 1;
    r.queue[0].store(slot0, std::memory_order_relaxed);
    std::vector<std::thread> th;
    for (uint32_t b = 0; b < nw; ++b)
        th.emplace_back(async_worker, std::ref(r));
    for (auto &t : th)
        t.join();
    const uint32_t n = r.n_next.load();
    std::set<std::vector<uint32_t>> got;
    unsigned once = 1;
    for (uint32_t e = 0; e < n; ++e) {
        const uint32_t s = r.queue[e].load();
        if (s == kNoEntryM)
            continue;
        got.insert(std::vector<uint32_t>(&r.t.data[(size_t)s * W], &r.t.data[(size_t)s * W] + W));
        once &= r.expanded[e].load() == 1;
    }
    early = r.left_at_min.load() < n;
    bool ok;
    if (want.size() <= limit) {
        ok = r.error.load() == 0 && !r.abort.load() && n == want.size() && got == want && once &&
             r.edges.load() == want_edges && r.work.load() == 0;
    } else {
        // past the cap: the run stopped; everything stored is listed once
        // and is reachable
        uint32_t stored = 0;
        for (uint32_t s = 0; s < r.t.capacity(); ++s)
            stored += (r.t.slot[s].load() & kDone) != 0;
        ok = r.error.load() == 0 && r.abort.load() && n > limit && got.size() == n && stored == n &&
             std::includes(want.begin(), want.end(), got.begin(), got.end());
        early = false;   // leaving at the cap is the point
    }
    if (!ok)
        printf("part7: %s N=%u L=%u F=%u workers=%u chunk=%u: %u entries, %zu distinct listed, %zu reachable, "
               "all expanded once %u, edges %llu of %llu, work %llu, error %u WRONG\n",
               m.broom ? "broom" : "cyclic", m.N, m.L, m.F, nw, chunk, n, got.size(), want.size(), once,
               (unsigned long long)r.edges.load(), (unsigned long long)want_edges, (unsigned long long)r.work.load(),
               r.error.load());
    return ok ? 0 : 1;
}

int part7() {
    const AsyncModel models[] = {{false, 1, 700, 0}, {false, 2, 30, 0}, {false, 3, 9, 0}, {false, 4, 6, 0},
                                 {false, 5, 4, 0},   {false, 6, 3, 0},  {true, 0, 40, 60}, {true, 0, 3, 200}};
    const uint32_t workers[] = {1, 3, 6};
    unsigned bad = 0, runs = 0, early = 0;
    // the kernel's proportions (16-entry chunks, a buffer of three chunks,
    // passes of a chunk), then 1-entry chunks with an append after every
    // pass of 2 successors: appends in the middle of tiles whose entries
    // other workers expand at once
    const uint32_t shapes[][3] = {{16, 48, 16}, {1, 2, 2}};
    for (const auto &sh : shapes)
        for (const AsyncModel &m : models)
            for (uint32_t nw : workers) {
                bool e = false;
                bad += async_run(m, nw, sh[0], sh[1], sh[2], e);
                early += e;
                ++runs;
            }
    // with a cap inside the state space: every worker stops, nothing
    // unreachable is listed, and every stored state is listed
    for (const auto &sh : shapes)
        for (uint32_t nw : workers)
            for (const auto &mc : {std::make_pair(models[0], 100u), std::make_pair(models[2], 300u),
                                   std::make_pair(models[6], 50u), std::make_pair(models[7], 120u)}) {
                bool e = false;
                bad += async_run(mc.first, nw, sh[0], sh[1], sh[2], e, mc.second);
                ++runs;
            }
    // the broom's fan again, many times: a worker that expands a state
    // appended in the middle of another's tile must never drive the work
    // count to zero while that tile is still open
    for (int rep = 0; rep < 40; ++rep)
        for (uint32_t nw : {3u, 6u}) {
            bool e = false;
            bad += async_run(models[7], nw, 1, 2, 2, e);
            early += e;
            ++runs;
        }
    printf("part7: %u explorations without levels, %u with a worker that left early, errors %u\n", runs, early,
           bad);
    return (int)(bad + early);
}

}  // namespace

int main(int argc, char **argv) {
    if (argc == 3 && (std::strcmp(argv[1], "part4") == 0 || std::strcmp(argv[1], "part7") == 0)) {
        // part 4 or 7 alone, repeated (built without a sanitizer, threads
        // interleave far more finely)
        const bool four = argv[1][4] == '4';
        int bad = 0;
        for (int i = 0, n = std::atoi(argv[2]); i < n; ++i)
            bad += four ? part4() : part7();
        printf("errors %d\n", bad);
        return bad ? 1 : 0;
    }
    const int a = part1();
    const int b = part2();
    const int c = part3();
    const int d = part4();
    const int e = part5();
    const int f = part6();
    const int g = part7();
    printf("errors %d\n", a + b + c + d + e + f + g);
    return a + b + c + d + e + f + g ? 1 : 0;
}
