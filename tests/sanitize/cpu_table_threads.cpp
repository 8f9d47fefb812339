// Drives the multi-core lockless CPU table from 8 threads (a stream holding
// every vector four times, and reachability with and without a cap) so that
// a ThreadSanitizer build can check every access between threads.  Exit code
// 1 if a result is wrong.
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <algorithm>
#include <random>
#include <vector>
extern "C" {
typedef struct cpu_summary { uint64_t total, edges, deadlocks; uint32_t n_levels; int32_t capped; } cpu_summary;
int cpu_stream(const uint32_t *rows, uint64_t n, uint32_t W, uint32_t log2cap, uint32_t threads,
               uint8_t *seen, uint32_t *index, double *seconds);
int cpu_reach(const uint32_t *trans, uint32_t P, uint32_t L, uint32_t S, uint32_t K, const uint32_t *init,
              uint64_t cap, uint32_t log2cap, uint32_t threads, uint64_t *level_counts, uint32_t max_levels,
              uint32_t *rows_out, uint64_t max_rows, cpu_summary *out, double *seconds);
}
int main() {
    const uint32_t W = 6, nd = 1 << 14, copies = 4;
    std::mt19937 rng(7);
    std::vector<uint32_t> distinct(nd * W);
    for (auto &x : distinct) x = rng() % 5;
    for (uint32_t i = 0; i < nd; ++i) distinct[i * W] = i;   // rows distinct through their first word
    std::vector<uint32_t> rows;
    std::vector<uint32_t> order(nd * copies);
    for (uint32_t i = 0; i < nd * copies; ++i) order[i] = i % nd;
    std::shuffle(order.begin(), order.end(), rng);
    for (uint32_t o : order) rows.insert(rows.end(), distinct.begin() + o * W, distinct.begin() + o * W + W);
    std::vector<uint8_t> seen(order.size());
    std::vector<uint32_t> index(order.size());
    double sec;
    int rc = cpu_stream(rows.data(), order.size(), W, 16, 8, seen.data(), index.data(), &sec);
    uint64_t nnew = 0;
    for (auto s : seen) nnew += s == 0;
    printf("stream rc %d new %llu (expect %u)\n", rc, (unsigned long long)nnew, nd);
    if (rc != 0 || nnew != nd)
        return 1;
    // a guarded model: P processes, L locals, S shared vars, K transitions each
    const uint32_t P = 4, L = 6, S = 2, K = 2;
    std::vector<uint32_t> trans(P * L * K * 5);
    for (uint32_t p = 0; p < P; ++p)
        for (uint32_t l = 0; l < L; ++l)
            for (uint32_t k = 0; k < K; ++k) {
                uint32_t *t = &trans[((p * L + l) * K + k) * 5];
                t[0] = rng() % L;
                t[1] = rng() % 3 == 0 ? 0xFFFFFFFFu : rng() % S; t[2] = rng() % 3;
                t[3] = rng() % 2 ? 0xFFFFFFFFu : rng() % S; t[4] = rng() % 3;
            }
    std::vector<uint32_t> init(P + S, 0);
    std::vector<uint64_t> lv(4096);
    cpu_summary sum{};
    rc = cpu_reach(trans.data(), P, L, S, K, init.data(), 0, 16, 8, lv.data(), 4096, nullptr, 0, &sum, &sec);
    printf("reach rc %d total %llu levels %u edges %llu\n", rc, (unsigned long long)sum.total, sum.n_levels,
           (unsigned long long)sum.edges);
    if (rc != 0 || sum.capped != 0)
        return 1;
    rc = cpu_reach(trans.data(), P, L, S, K, init.data(), sum.total / 2, 16, 8, lv.data(), 4096, nullptr, 0, &sum, &sec);
    printf("capped reach rc %d total %llu capped %d\n", rc, (unsigned long long)sum.total, sum.capped);
    return rc == 0 && sum.capped == 1 ? 0 : 1;
}
