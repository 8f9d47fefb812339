// Reachability server with continuous batching (reach_server_*).
//
// A worker thread owns the GPU side.  Between every BFS level step it
//   * admits queued queries, first come first served, while their tables fit
//     the device-memory budget (tables come from a resident pool keyed by
//     capacity and width; pooled tables of other shapes are freed when room
//     is needed), inserts their initial states,
//   * expands the current level of every admitted, unfinished query in one
//     launch (the multi-model step of the batch driver), and
//   * retires the queries whose exploration ended, returning their tables to
//     the pool.
// A query that arrives while others are on the GPU therefore joins at the
// next level step and its work overlaps theirs; its result is exactly the one
// reach_explore computes for it alone (same kernels, its own table).
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "batch_kernels.h"
#include "expand_device.h"
#include "internal.h"
#include "reach_internal.h"

using namespace lhs;

namespace {

constexpr uint64_t kDefaultBudget = 200ull << 30;
constexpr uint32_t kDefaultMaxActive = 1024;

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

__global__ void k_zero_step(LevelCounters *lc, DevStatus *st, uint32_t n) {
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        lc[i] = LevelCounters{0, 0, 0, 0};
        st[i].error = 0;
        st[i].wait_hits = 0;
        st[i].cas_failures = 0;
    }
}

struct Query {
    uint64_t ticket = 0;
    std::vector<reach_trans> trans;
    std::vector<uint32_t> init;
    reach_model m{};
    uint32_t W = 0;
    uint64_t capacity = 0, bytes = 0;
    double t_submit = 0, t_admit = 0, t_done = 0;
    lhs_table *t = nullptr;
    uint2 *d_trans = nullptr;
    uint32_t n_cur = 1, cur = 0, limit = 0;
    std::vector<uint64_t> levels;
    uint64_t total = 1, edges = 0, dead = 0, wait_hits = 0;
    int capped = 0;
    lhs_status status = LHS_OK;
    bool done = false;
};

uint64_t table_bytes(uint64_t capacity, uint32_t W) {
    // slots + rows + two frontiers (+ counters)
    return capacity * (8ull + 4ull * W + 8ull) + 4096;
}

}  // namespace

struct reach_server {
    reach_server_opts opts{};
    lhs_config cfg{};           // shape of every query table (one launch serves all)
    int device = 0;
    hipStream_t stream = nullptr;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    uint64_t next_ticket = 1;
    std::deque<Query *> queue;
    std::unordered_map<uint64_t, Query *> tickets;
    // worker-owned
    std::vector<Query *> active;
    std::multimap<std::pair<uint64_t, uint32_t>, lhs_table *> pool;
    uint64_t bytes_alloc = 0;   // tables allocated (in use + pooled)
    // step buffers
    uint32_t cap_slots = 0;
    BatchSlot *d_slots = nullptr, *h_slots = nullptr;
    uint32_t *d_begin = nullptr, *h_begin = nullptr;
    LevelCounters *d_lc = nullptr, *h_lc = nullptr;
    DevStatus *d_st = nullptr, *h_st = nullptr;
    uint32_t *d_roots = nullptr, *d_root_off = nullptr;
    uint32_t cap_roots = 0;
    // stats (under mu)
    reach_server_stats stats{};
    double busy_s = 0;
    lhs_status fatal = LHS_OK;
};

namespace {

void free_step_buffers(reach_server *s) {
    (void)hipFree(s->d_slots);
    (void)hipFree(s->d_begin);
    (void)hipFree(s->d_lc);
    (void)hipFree(s->d_st);
    if (s->h_slots)
        (void)hipHostFree(s->h_slots);
    if (s->h_begin)
        (void)hipHostFree(s->h_begin);
    if (s->h_lc)
        (void)hipHostFree(s->h_lc);
    if (s->h_st)
        (void)hipHostFree(s->h_st);
    s->d_slots = s->h_slots = nullptr;
    s->d_begin = s->h_begin = nullptr;
    s->d_lc = s->h_lc = nullptr;
    s->d_st = s->h_st = nullptr;
    s->cap_slots = 0;
}

lhs_status ensure_step_buffers(reach_server *s, uint32_t n) {
    if (n <= s->cap_slots)
        return LHS_OK;
    free_step_buffers(s);
    uint32_t c = 64;
    while (c < n)
        c <<= 1;
    if (hipMalloc(&s->d_slots, c * sizeof(BatchSlot)) != hipSuccess ||
        hipHostMalloc(&s->h_slots, c * sizeof(BatchSlot), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->d_begin, (c + 1) * sizeof(uint32_t)) != hipSuccess ||
        hipHostMalloc(&s->h_begin, (c + 1) * sizeof(uint32_t), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->d_lc, c * sizeof(LevelCounters)) != hipSuccess ||
        hipHostMalloc(&s->h_lc, c * sizeof(LevelCounters), hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&s->d_st, c * sizeof(DevStatus)) != hipSuccess ||
        hipHostMalloc(&s->h_st, c * sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        free_step_buffers(s);
        return LHS_ENOMEM;
    }
    s->cap_slots = c;
    return LHS_OK;
}

// Reserve a table for q (worker thread).  Returns false if it does not fit
// now.  Pooled tables of q's shape are reused; otherwise pooled tables are
// freed until a new one fits the budget.
bool acquire_table(reach_server *s, Query *q) {
    auto key = std::make_pair(q->capacity, q->W);
    auto it = s->pool.find(key);
    if (it != s->pool.end()) {
        q->t = it->second;
        s->pool.erase(it);
        return true;
    }
    while (s->bytes_alloc + q->bytes > s->opts.budget_bytes && !s->pool.empty()) {
        auto victim = s->pool.begin();
        s->bytes_alloc -= table_bytes(victim->second->capacity, victim->second->W);
        lhs_destroy(victim->second);
        s->pool.erase(victim);
    }
    if (s->bytes_alloc + q->bytes > s->opts.budget_bytes)
        return false;
    lhs_table *t = nullptr;
    if (lhs_create_ex(q->capacity, q->W, &s->cfg, &t) != LHS_OK || ensure_bfs_buffers(t) != LHS_OK) {
        lhs_destroy(t);
        return false;
    }
    s->bytes_alloc += q->bytes;
    q->t = t;
    return true;
}

void release_table(reach_server *s, Query *q) {
    if (q->t)
        s->pool.emplace(std::make_pair(q->t->capacity, q->t->W), q->t);
    q->t = nullptr;
    (void)hipFree(q->d_trans);
    q->d_trans = nullptr;
}

// Set up newly admitted queries: clear tables, upload models, insert roots.
lhs_status start_queries(reach_server *s, const std::vector<Query *> &qs) {
    if (qs.empty())
        return LHS_OK;
    lhs_status rc = ensure_step_buffers(s, (uint32_t)qs.size());
    if (rc != LHS_OK)
        return rc;
    std::vector<uint32_t> roots, off;
    std::vector<std::vector<uint2>> packed_all(qs.size());   // alive until the sync below
    for (uint32_t i = 0; i < qs.size(); ++i) {
        Query *q = qs[i];
        std::vector<uint2> &packed = packed_all[i];
        pack_model(&q->m, packed);
        if (hipMalloc(&q->d_trans, packed.size() * sizeof(uint2)) != hipSuccess ||
            hipMemcpyAsync(q->d_trans, packed.data(), packed.size() * sizeof(uint2), hipMemcpyHostToDevice,
                           s->stream) != hipSuccess)
            return LHS_EDEVICE;
        q->t->last_stream = s->stream;
        if (lhs_clear(q->t, s->stream) != LHS_OK)
            return LHS_EDEVICE;
        BatchSlot &sl = s->h_slots[i];
        sl.t = view(q->t);
        sl.m = model_view(&q->m, q->d_trans);
        sl.front = q->t->frontier[0];
        sl.next = q->t->frontier[1];
        sl.lc = s->d_lc + i;
        sl.n_front = 1;
        sl.limit = q->limit;
        sl.tile_begin = 0;
        off.push_back((uint32_t)roots.size());
        roots.insert(roots.end(), q->init.begin(), q->init.end());
    }
    if (roots.size() > s->cap_roots) {
        (void)hipFree(s->d_roots);
        (void)hipFree(s->d_root_off);
        s->cap_roots = 0;
        const uint32_t c = (uint32_t)std::max<size_t>(1024, roots.size() * 2);
        if (hipMalloc(&s->d_roots, c * sizeof(uint32_t)) != hipSuccess ||
            hipMalloc(&s->d_root_off, c * sizeof(uint32_t)) != hipSuccess)
            return LHS_ENOMEM;
        s->cap_roots = c;
    }
    const uint32_t n = (uint32_t)qs.size();
    if (hipMemcpyAsync(s->d_roots, roots.data(), roots.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                       s->stream) != hipSuccess ||
        hipMemcpyAsync(s->d_root_off, off.data(), n * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess ||
        hipMemcpyAsync(s->d_slots, s->h_slots, n * sizeof(BatchSlot), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess)
        return LHS_EDEVICE;
    if (launch_insert_roots(s->cfg.line_slots, s->stream, s->d_slots, s->d_roots, s->d_root_off, n) != LHS_OK)
        return LHS_EDEVICE;
    // host buffers are reused by the next step: wait for the copies
    return (hipGetLastError() == hipSuccess && hipStreamSynchronize(s->stream) == hipSuccess) ? LHS_OK
                                                                                            : LHS_EDEVICE;
}

// One level step over every active query.  Returns the queries that ended.
lhs_status step_queries(reach_server *s, std::vector<Query *> &finished) {
    const uint32_t na = (uint32_t)s->active.size();
    lhs_status rc = ensure_step_buffers(s, na);
    if (rc != LHS_OK)
        return rc;
    uint32_t tiles = 0, maxW = 1, tps = 1, tcap = 0;
    for (uint32_t a = 0; a < na; ++a) {
        Query *q = s->active[a];
        BatchSlot &sl = s->h_slots[a];
        sl.t = view(q->t);
        sl.t.status = s->d_st + a;
        sl.m = model_view(&q->m, q->d_trans);
        sl.front = q->t->frontier[q->cur];
        sl.next = q->t->frontier[q->cur ^ 1];
        sl.lc = s->d_lc + a;
        sl.n_front = q->n_cur;
        sl.limit = q->limit;
        sl.tile_begin = tiles;
        s->h_begin[a] = tiles;
        tiles += (q->n_cur + kExpandBlock - 1) / kExpandBlock;
        maxW = std::max(maxW, q->W);
        tcap = std::max(tcap, trans_lds_entries(q->m.n_procs, q->m.n_locals, q->m.trans_per_local));
        tps = tps_expand(q->t);
    }
    s->h_begin[na] = tiles;
    if (hipMemcpyAsync(s->d_slots, s->h_slots, na * sizeof(BatchSlot), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess ||
        hipMemcpyAsync(s->d_begin, s->h_begin, (na + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, s->stream) !=
            hipSuccess)
        return LHS_EDEVICE;
    hipLaunchKernelGGL(k_zero_step, dim3((na + 255) / 256), dim3(256), 0, s->stream, s->d_lc, s->d_st, na);
    if (launch_expand_multi(tps, s->cfg.line_slots, tiles, maxW, tcap, s->stream, s->d_slots, s->d_begin, na) !=
            LHS_OK ||
        hipGetLastError() != hipSuccess ||
        hipMemcpyAsync(s->h_lc, s->d_lc, na * sizeof(LevelCounters), hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess ||
        hipMemcpyAsync(s->h_st, s->d_st, na * sizeof(DevStatus), hipMemcpyDeviceToHost, s->stream) !=
            hipSuccess ||
        hipStreamSynchronize(s->stream) != hipSuccess)
        return LHS_EDEVICE;
    std::vector<Query *> keep;
    keep.reserve(na);
    for (uint32_t a = 0; a < na; ++a) {
        Query *q = s->active[a];
        const LevelCounters &lc = s->h_lc[a];
        q->wait_hits += s->h_st[a].wait_hits;
        bool end = false;
        if (s->h_st[a].error) {
            q->status = (lhs_status)s->h_st[a].error;
            end = true;
        } else if (q->m.state_cap && lc.n_next > q->limit) {
            hipLaunchKernelGGL(k_rollback_one, dim3(std::min<uint32_t>((lc.n_next + 255) / 256, 4096)), dim3(256),
                               0, s->stream, q->t->bucket, q->t->frontier[q->cur ^ 1], lc.n_next);
            q->capped = 1;
            end = true;
        } else {
            q->edges += lc.edges;
            q->dead += lc.deadlocks;
            if (lc.n_next == 0) {
                end = true;
            } else {
                q->levels.push_back(lc.n_next);
                q->total += lc.n_next;
                q->n_cur = lc.n_next;
                q->cur ^= 1;
                if (q->m.state_cap)
                    q->limit = (uint32_t)std::min<uint64_t>(q->m.state_cap - q->total, 0xFFFFFFFFull);
            }
        }
        (end ? finished : keep).push_back(q);
    }
    s->active.swap(keep);
    if (!finished.empty() && hipStreamSynchronize(s->stream) != hipSuccess)
        return LHS_EDEVICE;
    return LHS_OK;
}

void worker_main(reach_server *s) {
    (void)hipSetDevice(s->device);
    while (true) {
        std::vector<Query *> admitted;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            while (true) {
                while (!s->queue.empty() && s->active.size() + admitted.size() < s->opts.max_active) {
                    Query *q = s->queue.front();
                    if (!acquire_table(s, q)) {
                        if (s->active.empty() && admitted.empty() && s->pool.empty()) {
                            // nothing will free memory: the allocation itself failed
                            s->queue.pop_front();
                            q->status = LHS_ENOMEM;
                            q->t_admit = q->t_done = now_s();
                            q->done = true;
                            s->stats.completed += 1;
                            s->cv_done.notify_all();
                            continue;
                        }
                        break;
                    }
                    s->queue.pop_front();
                    q->t_admit = now_s();
                    admitted.push_back(q);
                }
                if (!s->active.empty() || !admitted.empty())
                    break;
                if (s->stop && s->queue.empty())
                    return;
                s->cv_work.wait(lk);
            }
            s->stats.active = (uint32_t)(s->active.size() + admitted.size());
            s->stats.queued = (uint32_t)s->queue.size();
            s->stats.bytes_in_use = s->bytes_alloc;
            s->stats.peak_bytes = std::max(s->stats.peak_bytes, s->bytes_alloc);
        }
        const double t0 = now_s();
        std::vector<Query *> finished;
        lhs_status rc = start_queries(s, admitted);
        if (rc == LHS_OK) {
            s->active.insert(s->active.end(), admitted.begin(), admitted.end());
            rc = step_queries(s, finished);
        } else {
            for (Query *q : admitted) {
                q->status = rc;
                finished.push_back(q);
            }
        }
        if (rc != LHS_OK) {
            // a device failure ends every query on the GPU
            for (Query *q : s->active) {
                q->status = rc;
                finished.push_back(q);
            }
            s->active.clear();
        }
        const double t1 = now_s();
        std::lock_guard<std::mutex> lk(s->mu);
        s->busy_s += t1 - t0;
        s->stats.steps += 1;
        if (rc != LHS_OK)
            s->fatal = rc;
        for (Query *q : finished) {
            release_table(s, q);
            q->t_done = t1;
            q->done = true;
            s->stats.completed += 1;
            if (q->status == LHS_OK)
                s->stats.states += q->total;
        }
        uint64_t pooled = 0;
        for (auto &e : s->pool)
            pooled += table_bytes(e.second->capacity, e.second->W);
        s->stats.bytes_pooled = pooled;
        if (!finished.empty())
            s->cv_done.notify_all();
    }
}

lhs_status collect(reach_server *s, Query *q, reach_result *r, reach_query_times *t) {
    if (t) {
        t->submit_s = q->t_submit;
        t->admit_s = q->t_admit;
        t->done_s = q->t_done;
    }
    lhs_status rc = q->status;
    if (r) {
        std::memset(r, 0, sizeof(*r));
        if (rc == LHS_OK) {
            r->total_states = q->total;
            r->edges = q->edges;
            r->deadlocks = q->dead;
            r->capped = q->capped;
            r->wait_hits = q->wait_hits;
            r->n_levels = (uint32_t)q->levels.size();
            r->gpu_ms = (q->t_done - q->t_admit) * 1e3;
            r->level_counts = (uint64_t *)std::malloc(q->levels.size() * sizeof(uint64_t));
            if (!r->level_counts)
                rc = LHS_ENOMEM;
            else
                std::memcpy(r->level_counts, q->levels.data(), q->levels.size() * sizeof(uint64_t));
        }
    }
    s->tickets.erase(q->ticket);
    delete q;
    return rc;
}

}  // namespace

extern "C" {

double reach_server_clock(void) { return now_s(); }

lhs_status reach_server_create(const reach_server_opts *o, reach_server **out) {
    if (!out)
        return LHS_EINVAL;
    *out = nullptr;
    reach_server *s = new (std::nothrow) reach_server();
    if (!s)
        return LHS_ENOMEM;
    if (o)
        s->opts = *o;
    if (!s->opts.budget_bytes)
        s->opts.budget_bytes = kDefaultBudget;
    if (!s->opts.max_active)
        s->opts.max_active = kDefaultMaxActive;
    const lhs_config &c = s->opts.table;
    if (c.line_slots == 0 && c.probe == 0 && c.tps_find_or_put == 0 && c.tps_expand == 0) {
        s->cfg = tuned_config(LHS_TUNE_BATCH, 32, s->opts.capacity ? s->opts.capacity : (1ull << 21));
    } else {
        s->cfg = c;
        if (s->cfg.line_slots == 0)
            s->cfg.line_slots = 16;
    }
    if ((s->opts.capacity && (!is_pow2(s->opts.capacity) || s->opts.capacity < kLineSlots ||
                              s->opts.capacity > (1ull << 32))) ||
        !valid_line_slots(s->cfg.line_slots) || s->cfg.probe > LHS_PROBE_QUADRATIC ||
        !valid_tps(s->cfg.tps_find_or_put) || !valid_tps(s->cfg.tps_expand)) {
        delete s;
        return LHS_EINVAL;
    }
    if (hipGetDevice(&s->device) != hipSuccess || hipStreamCreate(&s->stream) != hipSuccess) {
        delete s;
        return LHS_EDEVICE;
    }
    s->worker = std::thread(worker_main, s);
    *out = s;
    return LHS_OK;
}

lhs_status reach_server_submit(reach_server *s, const reach_model *m, uint64_t *ticket) {
    if (!s || !ticket || validate_model(m) != LHS_OK)
        return LHS_EINVAL;
    Query *q = new (std::nothrow) Query();
    if (!q)
        return LHS_ENOMEM;
    q->W = m->n_procs + m->n_shared;
    const uint64_t nt = (uint64_t)m->n_procs * m->n_locals * m->trans_per_local;
    q->trans.assign(m->trans, m->trans + nt);
    q->init.assign(m->init, m->init + q->W);
    q->m = *m;
    q->m.trans = q->trans.data();
    q->m.init = q->init.data();
    q->capacity = s->opts.capacity ? s->opts.capacity
                                   : (m->state_cap ? auto_capacity(m) : (1ull << 21));
    if (m->state_cap && m->state_cap >= q->capacity) {
        delete q;
        return LHS_EINVAL;
    }
    q->bytes = table_bytes(q->capacity, q->W);
    if (q->bytes > s->opts.budget_bytes) {
        delete q;
        return LHS_EBUDGET;
    }
    q->limit = m->state_cap ? (uint32_t)std::min<uint64_t>(m->state_cap - 1, 0xFFFFFFFFull) : 0xFFFFFFFFu;
    q->levels.push_back(1);
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete q;
        return LHS_EINVAL;
    }
    q->ticket = s->next_ticket++;
    q->t_submit = now_s();
    s->queue.push_back(q);
    s->tickets[q->ticket] = q;
    s->stats.submitted += 1;
    *ticket = q->ticket;
    s->cv_work.notify_one();
    return LHS_OK;
}

lhs_status reach_server_poll(reach_server *s, uint64_t ticket, reach_result *r, reach_query_times *t) {
    if (!s)
        return LHS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end())
        return LHS_ENOTFOUND;
    if (!it->second->done)
        return LHS_EAGAIN;
    return collect(s, it->second, r, t);
}

lhs_status reach_server_wait(reach_server *s, uint64_t ticket, reach_result *r, reach_query_times *t) {
    if (!s)
        return LHS_EINVAL;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->tickets.find(ticket);
    if (it == s->tickets.end())
        return LHS_ENOTFOUND;
    Query *q = it->second;
    s->cv_done.wait(lk, [&] { return q->done; });
    return collect(s, q, r, t);
}

lhs_status reach_server_get_stats(reach_server *s, reach_server_stats *out) {
    if (!s || !out)
        return LHS_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->busy_s = s->busy_s;
    out->queued = (uint32_t)s->queue.size();
    return LHS_OK;
}

lhs_status reach_server_destroy(reach_server *s) {
    if (!s)
        return LHS_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    if (s->worker.joinable())
        s->worker.join();
    (void)hipStreamSynchronize(s->stream);
    for (auto &e : s->pool)
        lhs_destroy(e.second);
    for (auto &e : s->tickets)
        delete e.second;
    free_step_buffers(s);
    (void)hipFree(s->d_roots);
    (void)hipFree(s->d_root_off);
    (void)hipStreamDestroy(s->stream);
    const lhs_status rc = s->fatal;
    delete s;
    return rc;
}

}  // extern "C"
