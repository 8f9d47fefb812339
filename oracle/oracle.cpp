// CPU oracle for level-synchronous reachability and batched find-or-put.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
// calls this file: only the test-suite, the smoke check and the benchmark's
// CPU-baseline leg do.  It shares no code with the GPU library (no headers,
// no hash function, no table layout); both sides only read the arrays made
// by the input generators in gen/.
//
// Everything here is the plain definition, written sequentially:
//
//  * Reachability (Preliminaries section, Algorithm 1 "Reachability
//    analysis"): start from s0, take states from a work sequence, enumerate
//    next-state successors, count them, and keep the successors that the
//    visited set reports as new.  The work sequence here is a FIFO processed
//    level by level, so levels are exact BFS distances.  A state with zero
//    successors is a deadlock (the count == 0 test of Algorithm 1).
//    Reading adopted: a successor is queued when find-or-put reports it was
//    NOT seen before (Algorithm 3 returns `seen`; Algorithm 1's test has the
//    opposite polarity as printed).
//  * The visited set is a std::unordered_set (a library primitive); states
//    are kept in insertion order in one arena, so level d is a contiguous
//    range of the arena.
//  * Every emitted successor is an edge, duplicates and self-loops included:
//    the paper equates find-or-put calls with transitions (Shared Storage
//    Parameters section).
//  * Level-prefix state cap (reading adopted where the paper is silent):
//    the result is the longest prefix of BFS levels whose cumulative count is
//    <= cap.  When inserting level d+1 would push the total over the cap, the
//    partial level d+1 is discarded, level d is the last level kept, and
//    edges/deadlocks cover the expanded levels 0..d-1 only.
//  * Batched find-or-put as a sequential stream (Algorithm 3's contract,
//    Requirements on the State Storage section): seen[k] = 1 iff row k equals
//    an earlier row; id[k] = ordinal of the first occurrence of that row.
//
// Model semantics (asynchronous interleaving): for each process p and each of
// its K transitions t = trans[p][s[p]][k]: if t.guard_var is NONE or
// s[P + guard_var] == guard_val (guard read on the source state), emit a copy
// of s with s'[p] = t.target and, if eff_var is not NONE,
// s'[P + eff_var] = eff_val.
#include <cstdint>
#include <cstring>
#include <string_view>
#include <unordered_map>
#include <unordered_set>
#include <vector>

namespace {

constexpr uint32_t NONE = 0xFFFFFFFFu;

struct Arena {
    uint32_t W;
    std::vector<uint32_t> words;
    uint64_t rows() const { return words.size() / W; }
    const uint32_t *row(uint64_t id) const { return words.data() + id * W; }
};

struct RowHash {
    const Arena *a;
    size_t operator()(uint64_t id) const {
        return std::hash<std::string_view>{}(
            std::string_view(reinterpret_cast<const char *>(a->row(id)), a->W * 4u));
    }
};

struct RowEq {
    const Arena *a;
    bool operator()(uint64_t x, uint64_t y) const {
        return std::memcmp(a->row(x), a->row(y), a->W * 4u) == 0;
    }
};

struct Model {
    const uint32_t *trans;
    uint32_t P, L, S, K;
    // trans[p][l][k][5]
    const uint32_t *t(uint32_t p, uint32_t l, uint32_t k) const {
        return trans + ((static_cast<uint64_t>(p) * L + l) * K + k) * 5;
    }
};

// Enumerate the successors of `s` into `out` (rows of W words); returns the
// number of successors.  Locals outside [0, L) have no transitions.
uint32_t successors(const Model &m, const uint32_t *s, std::vector<uint32_t> &out) {
    const uint32_t W = m.P + m.S;
    out.clear();
    uint32_t n = 0;
    for (uint32_t p = 0; p < m.P; ++p) {
        if (s[p] >= m.L)
            continue;
        for (uint32_t k = 0; k < m.K; ++k) {
            const uint32_t *t = m.t(p, s[p], k);
            if (t[1] != NONE && s[m.P + t[1]] != t[2])
                continue;
            size_t o = out.size();
            out.insert(out.end(), s, s + W);
            out[o + p] = t[0];
            if (t[3] != NONE)
                out[o + m.P + t[3]] = t[4];
            ++n;
        }
    }
    return n;
}

// Oracle-side 64-bit digest of one row: FNV-1a over the words, then the
// SplitMix64 finaliser (Steele, Lea, Flood 2014).  Used only to compare sets
// without shipping them.
uint64_t row_digest(const uint32_t *r, uint32_t W) {
    uint64_t h = 0xcbf29ce484222325ull;
    for (uint32_t i = 0; i < W; ++i) {
        h ^= r[i];
        h *= 0x100000001b3ull;
    }
    h ^= h >> 30;
    h *= 0xbf58476d1ce4e5b9ull;
    h ^= h >> 27;
    h *= 0x94d049bb133111ebull;
    h ^= h >> 31;
    return h;
}

bool valid_model(const Model &m) {
    if (!m.trans || !m.P || !m.L || !m.K || m.P + m.S > 1024)
        return false;
    for (uint64_t i = 0; i < static_cast<uint64_t>(m.P) * m.L * m.K; ++i) {
        const uint32_t *t = m.trans + i * 5;
        if (t[1] != NONE && t[1] >= m.S)
            return false;
        if (t[3] != NONE && t[3] >= m.S)
            return false;
    }
    return true;
}

}  // namespace

extern "C" {

struct oracle_reach_summary {
    uint64_t total;
    uint64_t edges;
    uint64_t deadlocks;
    uint64_t digest_sum;
    uint64_t digest_xor;
    uint32_t n_levels;
    int32_t capped;
};

// Level-synchronous BFS reachability.
//   trans [P][L][K][5], init [P+S]; cap = 0 means no cap.
//   level_counts receives n_levels entries (max_levels available).
//   If states_out is non-null and has room for `total` rows, the reachable
//   states are written there in BFS order (level 0 first).
// Returns 0, -1 (bad arguments), -2 (more levels than max_levels).
int oracle_reach(const uint32_t *trans, uint32_t P, uint32_t L, uint32_t S, uint32_t K,
                 const uint32_t *init, uint64_t cap, uint64_t *level_counts,
                 uint32_t max_levels, uint32_t *states_out, uint64_t states_out_rows,
                 oracle_reach_summary *sum) {
    Model m{trans, P, L, S, K};
    if (!valid_model(m) || !init || !level_counts || !max_levels || !sum)
        return -1;
    const uint32_t W = P + S;
    Arena a{W, {}};
    std::unordered_set<uint64_t, RowHash, RowEq> V(1024, RowHash{&a}, RowEq{&a});
    if (cap) {
        V.reserve(cap + 1);
        a.words.reserve((cap + 1) * W);
    }

    a.words.assign(init, init + W);
    V.insert(0);
    std::memset(sum, 0, sizeof(*sum));
    level_counts[0] = 1;
    sum->n_levels = 1;

    uint64_t lvl_begin = 0, lvl_end = 1;
    std::vector<uint32_t> succ, s(W);
    while (true) {
        uint64_t lvl_edges = 0, lvl_dead = 0;
        bool abort = false;
        for (uint64_t id = lvl_begin; id < lvl_end && !abort; ++id) {
            // copy the source row: appending to the arena may reallocate it
            s.assign(a.row(id), a.row(id) + W);
            const uint32_t n = successors(m, s.data(), succ);
            for (uint32_t j = 0; j < n; ++j) {
                const uint64_t cand = a.rows();
                a.words.insert(a.words.end(), succ.begin() + j * W, succ.begin() + (j + 1) * W);
                if (!V.insert(cand).second) {
                    a.words.resize(cand * W);   // seen before: drop the copy
                } else if (cap && a.rows() > cap) {
                    abort = true;
                    break;
                }
            }
            lvl_edges += n;
            lvl_dead += (n == 0);
        }
        if (abort) {
            for (uint64_t id = lvl_end; id < a.rows(); ++id)
                V.erase(id);
            a.words.resize(lvl_end * W);
            sum->capped = 1;
            break;
        }
        sum->edges += lvl_edges;
        sum->deadlocks += lvl_dead;
        const uint64_t fresh = a.rows() - lvl_end;
        if (fresh == 0)
            break;
        if (sum->n_levels >= max_levels)
            return -2;
        level_counts[sum->n_levels++] = fresh;
        lvl_begin = lvl_end;
        lvl_end = a.rows();
    }
    sum->total = a.rows();
    for (uint64_t id = 0; id < a.rows(); ++id) {
        const uint64_t d = row_digest(a.row(id), W);
        sum->digest_sum += d;
        sum->digest_xor ^= d;
    }
    if (states_out && states_out_rows >= a.rows())
        std::memcpy(states_out, a.words.data(), a.words.size() * 4);
    return 0;
}

// Successors of one state (rows of W words, in (p, k) order) for sampled
// closure checks.  Returns the count, or -1 if out has fewer than
// max_rows rows for them.
int64_t oracle_successors(const uint32_t *trans, uint32_t P, uint32_t L, uint32_t S,
                          uint32_t K, const uint32_t *state, uint32_t *out,
                          uint64_t max_rows) {
    Model m{trans, P, L, S, K};
    std::vector<uint32_t> succ;
    const uint32_t n = successors(m, state, succ);
    if (n > max_rows)
        return -1;
    if (n)
        std::memcpy(out, succ.data(), succ.size() * 4);
    return n;
}

// Sequential find-or-put over a stream of n rows of W words.
//   seen[k] = 1 iff row k equals some row j < k;  id[k] = first-occurrence
//   ordinal of row k's value.  Returns the number of distinct rows.
uint64_t oracle_stream(const uint32_t *rows, uint64_t n, uint32_t W, uint8_t *seen,
                       uint32_t *id) {
    // Key: stream position of the first occurrence; rows are read in place.
    struct PosHash {
        const uint32_t *r;
        uint32_t W;
        size_t operator()(uint64_t k) const {
            return std::hash<std::string_view>{}(
                std::string_view(reinterpret_cast<const char *>(r + k * W), W * 4u));
        }
    };
    struct PosEq {
        const uint32_t *r;
        uint32_t W;
        bool operator()(uint64_t x, uint64_t y) const {
            return std::memcmp(r + x * W, r + y * W, W * 4u) == 0;
        }
    };
    std::unordered_map<uint64_t, uint32_t, PosHash, PosEq> first(n + 1, PosHash{rows, W},
                                                                 PosEq{rows, W});
    uint64_t distinct = 0;
    for (uint64_t k = 0; k < n; ++k) {
        auto it = first.find(k);
        if (it == first.end()) {
            first.emplace(k, static_cast<uint32_t>(distinct));
            seen[k] = 0;
            id[k] = static_cast<uint32_t>(distinct++);
        } else {
            seen[k] = 1;
            id[k] = it->second;
        }
    }
    return distinct;
}

// Order-independent set digest: count, wrapping sum and xor of row_digest.
// Duplicated rows are NOT removed (callers check uniqueness separately).
void oracle_digest(const uint32_t *rows, uint64_t n, uint32_t W, uint64_t *dsum,
                   uint64_t *dxor) {
    uint64_t s = 0, x = 0;
    for (uint64_t k = 0; k < n; ++k) {
        const uint64_t d = row_digest(rows + k * W, W);
        s += d;
        x ^= d;
    }
    *dsum = s;
    *dxor = x;
}

}  // extern "C"
