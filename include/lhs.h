/*
 * lhs — lockless GPU state storage and level-synchronous reachability for
 * MI355X (gfx950).  Plain C ABI: no C++ or framework types cross it.
 *
 * Paper: A. Laarman, J. van de Pol, M. Weber, "Boosting Multi-Core
 * Reachability Performance with Shared Hash Tables".
 *
 * Conventions for every call below
 *   - Return value: lhs_status; LHS_OK (0) on success.  Argument errors are
 *     detected on the host before any device work is queued (LHS_EINVAL) and
 *     leave the table untouched.
 *   - "device" pointers are HIP device allocations (e.g. a torch tensor's
 *     data_ptr() on the current device); "host" pointers are ordinary host
 *     memory.  The caller keeps ownership of every buffer it passes in; the
 *     library owns what it allocates and frees it in the matching destroy/free
 *     call.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  Calls that take
 *     a stream are asynchronous on it unless documented otherwise.
 *   - Device-side failures (table full, a spin that exceeded its bound) are
 *     sticky in the table and are reported by lhs_check().
 */
#ifndef LHS_H
#define LHS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum lhs_status {
    LHS_OK = 0,
    LHS_EINVAL = 1,   /* bad argument (checked on the host)                    */
    LHS_ENOMEM = 2,   /* device or host allocation failed                      */
    LHS_EFULL = 3,    /* a find-or-put probed every line without a free slot   */
    LHS_ESTALL = 4,   /* a wait on a slot being written exceeded its bound     */
    LHS_EDEVICE = 5,  /* a HIP runtime call failed                             */
    LHS_EBUDGET = 6,  /* a request does not fit a memory budget (the server's,
                         or the fixed array of reach_explore_noalloc)          */
    LHS_ENOTFOUND = 7,/* unknown ticket                                        */
    LHS_EAGAIN = 8    /* result not ready yet (non-blocking poll)              */
} lhs_status;

/* Human-readable name of a status code (static storage). */
const char *lhs_strerror(lhs_status s);

/* ------------------------------------------------------------------------
 * Table: one shared, lockless, open-addressing set of fixed-width vectors.
 *
 * Design (section "Hash Table Design"): open addressing; probing walks the
 * line of slots that holds the home slot (by default 128 bytes = 16
 * eight-byte slots), starting at the home slot and wrapping inside the line
 * ("walking the line", Algorithm 4), then moves to another line (by default
 * double hashing); vectors live in a separate data array indexed by slot;
 * each slot memoises the vector's hash and carries write/done status; 2^n
 * slots so the index is the low hash bits; empty = 0; slots are claimed with
 * a 64-bit compare-and-swap (Algorithm 2).  The table never resizes and
 * allocates nothing after creation (requirements listed in "Requirements on
 * the State Storage").
 * ---------------------------------------------------------------------- */
typedef struct lhs_table lhs_table;

/* Line-to-line probe sequence after the home line ("Hash Table Design": the
 * paper rehashes with further hash functions).  On 2^n lines each visits
 * every line once in its first 2^n rounds. */
typedef enum lhs_probe {
    LHS_PROBE_DOUBLE = 0,    /* line_k = line_0 + k*step, step odd, from the hash */
    LHS_PROBE_LINEAR = 1,    /* line_k = line_0 + k                               */
    LHS_PROBE_QUADRATIC = 2  /* line_k = line_0 + k(k+1)/2                        */
} lhs_probe;

/* Tunable shape of a table.  Every choice gives the same results (the same
 * stored set, seen flags and per-level counts); only speed and the slot
 * numbers differ. */
typedef struct lhs_config {
    uint32_t line_slots;      /* slots per line walked before the next probe:
                                 8, 16 or 32 (64, 128, 256 bytes); 0 = 16     */
    uint32_t probe;           /* lhs_probe                                     */
    uint32_t tps_find_or_put; /* GPU lanes per operation in lhs_find_or_put:
                                 1, 4, 8, 16, or 0 = 4 (see
                                 lhs_set_threads_per_state)                    */
    uint32_t tps_expand;      /* the same for BFS expansion; 0 = 1             */
} lhs_config;

/* Create a table on the current HIP device.
 *   capacity    : number of slots, a power of two in [16, 2^32].
 *   state_words : vector width W in 32-bit words, in [1, 32].
 * Allocates capacity*8 bytes of slots (zeroed) plus capacity*W*4 bytes of
 * vector data, once.  *out receives the handle (owned by the caller, freed by
 * lhs_destroy).  The table's shape is the loaded tuning table's choice for
 * (state_words, capacity) (lhs_tune_load), or the defaults of lhs_config.
 * Errors: LHS_EINVAL, LHS_ENOMEM, LHS_EDEVICE. */
lhs_status lhs_create(uint64_t capacity, uint32_t state_words, lhs_table **out);

/* lhs_create with an explicit shape (cfg NULL = defaults, no tuning table).
 * LHS_EINVAL for a value outside the ranges of lhs_config. */
lhs_status lhs_create_ex(uint64_t capacity, uint32_t state_words, const lhs_config *cfg,
                         lhs_table **out);

/* The table's shape as configured (0 = default for the tps fields). */
lhs_status lhs_get_config(lhs_table *t, lhs_config *out);

/* Free the table and everything it allocated.  NULL is accepted. The caller
 * must not have work on the table in flight. */
lhs_status lhs_destroy(lhs_table *t);

/* Empty the table (all slots to 0) and clear its sticky error and counters,
 * asynchronously on hip_stream. */
lhs_status lhs_clear(lhs_table *t, void *hip_stream);

/* Batched find-or-put (Algorithm 3, "find-or-put").
 *   d_states : device, n rows of state_words uint32 each, row-major, read only.
 *   n        : number of rows (0 is a no-op); at most 2^32 - 1.
 *   d_seen   : device, n bytes out.  1 = the vector was already stored
 *              ("seen", the paper's output), 0 = this call inserted it,
 *              0xFF = the operation failed (see lhs_check).
 *   d_index  : device, n uint32 out (may be NULL): the slot holding the
 *              vector.  Equal vectors always get equal indices; the index
 *              also addresses the vector's row in the data array.
 * Within one call the order of operations is unspecified: when a batch holds
 * a vector several times and it was not stored before, exactly one of those
 * rows reports 0.  Calls on one table may run concurrently on several
 * streams (the table is lockless).  Asynchronous on hip_stream. */
lhs_status lhs_find_or_put(lhs_table *t, const uint32_t *d_states, uint64_t n,
                           uint8_t *d_seen, uint32_t *d_index, void *hip_stream);

/* Number of GPU lanes that cooperate on one find-or-put: 1, 4, 8 or 16, or
 * 0 for each kernel's default (4 for lhs_find_or_put, 1 for the BFS).  G > 1:
 * a group of G lanes runs one operation and loads its slot line as one
 * coalesced access (line_slots/G slots per lane).  G = 1: every lane runs its
 * own operation while the wavefront moves lines and rows cooperatively
 * (line_slots/2 lanes per line, eight per row).  Affects speed only; results
 * are identical for every value.  Sets both tps fields of the table's
 * lhs_config; applies to later calls (find-or-put and BFS). */
lhs_status lhs_set_threads_per_state(lhs_table *t, uint32_t tps);

/* Wait for the last stream used with the table, then return its sticky
 * device error (LHS_EFULL / LHS_ESTALL) or LHS_OK.  The paper lets a probe
 * continue indefinitely and a writer's slot stay busy for as long as the
 * write takes (section "Algorithm", Algorithm 3's probe loop and wait loop);
 * here both are bounded and their failures are reported by this call.
 * LHS_EINVAL for a null table, LHS_EDEVICE if the synchronisation fails. */
lhs_status lhs_check(lhs_table *t);

/* Number of stored vectors: slots in the done state of the bucket state
 * diagram (figure "State diagram of buckets": empty -> write -> done).
 * Slots still being written are not counted.  Synchronous (waits for the
 * table's last stream); uses temporary device memory.  LHS_EINVAL for a null
 * argument. */
lhs_status lhs_count(lhs_table *t, uint64_t *out);

/* Copy every stored vector to host memory, in ascending slot order: the
 * vectors of the done slots of the bucket state diagram (figure "State
 * diagram of buckets"), read from the separate data array that the slot
 * index addresses (section "Hash Table Design").
 *   h_states : host, room for max_rows * state_words uint32 (may be NULL
 *              to only count).
 *   h_index  : host, room for max_rows uint32 (may be NULL): slot of each row.
 *   *n_rows  : number of stored vectors (also when it exceeds max_rows, in
 *              which case nothing is copied and LHS_EINVAL is returned).
 * Synchronous; uses temporary device memory.  For checks, not the hot path. */
lhs_status lhs_dump(lhs_table *t, uint32_t *h_states, uint32_t *h_index,
                    uint64_t max_rows, uint64_t *n_rows);

/* Copy the raw slot words (capacity uint64) to host memory.  Slot encoding:
 * 0 = empty; bit 63 = claimed; bit 62 = vector written ("done"); bits 61..0
 * = the low 62 bits of the vector's 64-bit hash.  Synchronous. */
lhs_status lhs_dump_slots(lhs_table *t, uint64_t *h_slots);

typedef struct lhs_info {
    uint64_t capacity;     /* slots                                          */
    uint32_t state_words;  /* W                                              */
    uint32_t line_slots;   /* slots per probed line (8, 16, 32)              */
    uint64_t hash_seed;    /* seed of the 64-bit vector hash                 */
    uint64_t wait_hits;    /* waits on a slot still being written (the
                              paper's write-busy "lock" hits)                */
    uint64_t cas_failures; /* lost claims of an empty slot                   */
    uint32_t error;        /* sticky lhs_status of device failures           */
    uint32_t probe;        /* lhs_probe                                      */
    uint32_t tps_find_or_put; /* lanes per operation in effect (defaults
                                 resolved)                                   */
    uint32_t tps_expand;
    uint64_t lines_probed; /* lines examined by find-or-puts while counted
                              (lhs_set_counters); the paper's probe count     */
    uint64_t merged;       /* successors that explorations merged into an
                              equal successor of the same pass while counted
                              (lhs_set_counters, lhs_set_merge)               */
} lhs_info;

/* Table geometry and device counters (synchronises the last stream). */
lhs_status lhs_get_info(lhs_table *t, lhs_info *out);

/* Optional device counters for later calls on t: LHS_COUNT_LINES adds the
 * number of lines every find-or-put examines to lhs_info.lines_probed,
 * LHS_COUNT_MERGED the successors merged by explorations to lhs_info.merged
 * (one more atomic per wavefront each; off by default).  0 turns them off;
 * the counts restart at lhs_clear.  LHS_EINVAL for unknown bits. */
#define LHS_COUNT_LINES 1u
#define LHS_COUNT_MERGED 2u
lhs_status lhs_set_counters(lhs_table *t, uint32_t flags);

/* How explorations on t (reach_explore in every mode, the batch, the
 * server) treat successors of one expansion pass that are the same state.
 * Algorithm 1 runs find-or-put once per successor.  Two interleavings of
 * independent moves often reach one state from neighbouring frontier
 * states, and find-or-put of an equal vector has one answer (its slot), so
 * with LHS_MERGE_ON (the default) a workgroup gives each distinct state of
 * a pass of 256 successors one find-or-put in the table, and the equal ones
 * take it as seen.  The test is exact: a hash-tag match is confirmed on the
 * full vectors, else the successor runs its own find-or-put.
 *   LHS_MERGE_OFF          one find-or-put per successor, as Algorithm 1;
 *   LHS_MERGE_NARROW_TAGS  merging with one-bit tags, so that most tag
 *                          matches belong to other states (a check of that
 *                          path: slower, same results).
 * Reachable set, level counts, edges and deadlocks do not depend on the
 * mode; wait and CAS-failure counts do.  Applies to expansions with one
 * lane per successor (lhs_set_threads_per_state 1, the default) of models
 * with at most 64 (process, transition) pairs.  LHS_EINVAL for a null table
 * or an unknown mode. */
#define LHS_MERGE_ON 0u
#define LHS_MERGE_OFF 1u
#define LHS_MERGE_NARROW_TAGS 2u
lhs_status lhs_set_merge(lhs_table *t, uint32_t mode);

/* Number of workers of the explorations on t (reach_explore, with or
 * without REACH_F_GRAPH / REACH_F_ASYNC): at most max_workgroups workgroups
 * of 256 lanes expand states, each one a worker in the sense of the paper's
 * speedup S = T_1 / T_N and efficiency E = S / N over N workers (section
 * "Preliminaries").  0 (the default) = every workgroup that fits on the GPU
 * at once.  Results do not depend on it.  Find-or-put calls and the batch
 * are not affected.  LHS_EINVAL for a null table. */
lhs_status lhs_set_workers(lhs_table *t, uint32_t max_workgroups);

/* ------------------------------------------------------------------------
 * Tuning table: table shapes chosen by the autotuner
 * (paper_1004_2772_amd/autotune.py), which times every lhs_config on
 * synthetic workloads of a set of widths and sizes and writes them as JSON:
 *   {"format": "lhs-tune-1", "device": "<gcn arch>", "entries": [
 *     {"kind": "table"|"batch", "W": w, "log2_capacity": c,
 *      "line_slots": 8|16|32, "probe": "double"|"linear"|"quadratic",
 *      "tps_find_or_put": g, "tps_expand": g, ...}, ...]}
 * (other keys are ignored).  A loaded table is process-wide; lhs_create,
 * reach_explore (kind "table"), reach_explore_batch and the server (kind
 * "batch") take their tables' shapes from it.
 * ---------------------------------------------------------------------- */
#define LHS_TUNE_TABLE 0u
#define LHS_TUNE_BATCH 1u

/* Load a tuning file, replacing the loaded table.  Entries of another device
 * are skipped: device = the arch name to match ("gfx950"), NULL = the
 * current HIP device's.  *n_loaded (may be NULL) = entries kept.  Errors:
 * LHS_EINVAL (unreadable file, malformed JSON or a value out of range; the
 * loaded table is then unchanged), LHS_EDEVICE (device NULL and no device). */
lhs_status lhs_tune_load(const char *path, const char *device, uint32_t *n_loaded);

/* Forget the loaded tuning table (back to the defaults). */
lhs_status lhs_tune_clear(void);

/* The shape used for a table of `kind` with W = state_words and `capacity`
 * slots: among the loaded entries of that kind, those of the smallest tuned
 * W >= state_words (else the largest W), and of these the one whose
 * log2_capacity is nearest (ties: the larger).  *found = 1 if it came from
 * the tuning table, 0 for the defaults (found may be NULL). */
lhs_status lhs_tune_lookup(uint32_t kind, uint32_t state_words, uint64_t capacity, lhs_config *out,
                           int32_t *found);

/* ------------------------------------------------------------------------
 * Reachability (Algorithm 1, "Reachability analysis") as level-synchronous
 * BFS on the GPU: every level expands the whole frontier with the model's
 * next-state function, inserts every successor with find-or-put and queues
 * the ones that were new; levels are exact BFS distances.
 * ---------------------------------------------------------------------- */

#define REACH_NONE 0xFFFFFFFFu

/* One guarded transition of a process (asynchronous interleaving): from the
 * process's current local state it fires when guard_var == REACH_NONE or
 * shared[guard_var] == guard_val (read on the source state); it sets the
 * process's local state to target and, when eff_var != REACH_NONE,
 * shared[eff_var] = eff_val. */
typedef struct reach_trans {
    uint32_t target;
    uint32_t guard_var;
    uint32_t guard_val;
    uint32_t eff_var;
    uint32_t eff_val;
} reach_trans;

/* A model in host memory.  State vector: n_procs local states followed by
 * n_shared shared values, W = n_procs + n_shared words (1..32).
 *   trans      : [n_procs][n_locals][trans_per_local] transitions.
 *   init       : W words, the initial state s0.
 *   state_cap  : 0 = explore to exhaustion; otherwise keep the longest prefix
 *                of BFS levels whose cumulative state count is <= state_cap
 *                (the first level that would exceed it is discarded and the
 *                result is flagged capped).
 * Limits: n_locals <= 65535, targets < n_locals, n_shared <= 254,
 * guard/effect values <= 65535, trans_per_local <= 16. */
typedef struct reach_model {
    uint32_t n_procs;
    uint32_t n_locals;
    uint32_t n_shared;
    uint32_t trans_per_local;
    const reach_trans *trans;
    const uint32_t *init;
    uint64_t state_cap;
} reach_model;

typedef struct reach_opts {
    uint64_t capacity;    /* table slots (power of two); 0 = automatic        */
    uint32_t max_levels;  /* bound on the number of levels; 0 = 1<<20          */
    uint32_t flags;       /* REACH_F_* below                                   */
    lhs_table *table;     /* optional caller-created table (W must match); it
                             is cleared first and keeps the result set, so it
                             can be dumped afterwards.  NULL = internal table. */
    void *hip_stream;     /* stream for all device work                        */
} reach_opts;

#define REACH_F_NONE 0u
#define REACH_F_GRAPH 2u       /* reach_explore: the level loop runs from a
                                  captured HIP graph of 8 levels (expand,
                                  finalise, rollback kernels driven by a
                                  device-side level record), replayed until
                                  the exploration ends; the host waits once
                                  per replay instead of once per level      */
#define REACH_F_PARENTS 4u     /* reach_explore on a caller table (o->table):
                                  also record, for every new state, the slot
                                  of the state it was generated from (one
                                  uint32 per slot, allocated in the table on
                                  first use) and the slots of the first 1024
                                  deadlock states expanded, for reach_trace
                                  and reach_deadlock_slots.  Without a caller
                                  table: LHS_EINVAL                          */
#define REACH_F_ASYNC 8u       /* reach_explore without level barriers (the
                                  paper's order-free exploration with shared
                                  state storage and dynamic load balancing):
                                  one persistent launch whose workgroups
                                  expand states from a shared FIFO of slots in
                                  discovery order (pseudo-BFS) and take new
                                  work as soon as it is appended.  Result:
                                  total_states, edges and deadlocks as for
                                  the full BFS; n_levels = 0 and level_counts
                                  = NULL (levels are not defined).  With a
                                  state_cap the exploration stops once
                                  state_cap states are stored; the result then
                                  holds every state stored (state_cap plus at
                                  most one pass of 256 per workgroup), the
                                  counts cover the states expanded, and it is
                                  flagged capped.  Traces (REACH_F_PARENTS)
                                  are valid paths, not shortest ones.  Not
                                  with REACH_F_GRAPH; capacity < 2^32.       */
#define REACH_F_HOST_LOOP 1u   /* batch: one launch per level step, the host
                                  reads the counters after each (default: one
                                  persistent launch for all levels)           */

typedef struct reach_result {
    uint64_t total_states;  /* |kept levels|                                   */
    uint64_t edges;         /* successors generated by the expanded levels     */
    uint64_t deadlocks;     /* expanded states without successors              */
    uint64_t wait_hits;     /* waits on slots being written (informational)    */
    uint64_t *level_counts; /* n_levels entries, library-allocated             */
    uint32_t n_levels;
    int32_t capped;         /* 1 if state_cap cut a level off                  */
    double gpu_ms;          /* device time of the exploration                  */
} reach_result;

/* Explore m.  r is filled on LHS_OK; free it with reach_result_free.
 * Synchronous (returns when the exploration is complete). */
lhs_status reach_explore(const reach_model *m, const reach_opts *o, reach_result *r);

/* Free what reach_explore / reach_explore_batch allocated in r. */
void reach_result_free(reach_result *r);

/* For callers that cannot allocate memory (tight serving loops, harnesses
 * that forbid allocation after start-up): reach_explore on a caller-created
 * table t that allocates nothing, neither device nor host memory.  The
 * frontiers, level counters and model upload that reach_explore keeps in the
 * table and the device workspace live instead in one fixed device array of
 * LHS_NOALLOC_SCRATCH_BYTES per device, reserved when the library is loaded
 * and held until the process ends.  Limits, checked before any device work:
 * t->capacity <= LHS_NOALLOC_MAX_CAPACITY slots and n_procs * n_locals *
 * trans_per_local <= LHS_NOALLOC_MAX_TRANS transitions, else LHS_EBUDGET.
 *   m              : the model (as for reach_explore; its state_cap applies).
 *   t              : the caller's table on the current device, width
 *                    n_procs + n_shared, capacity > state_cap; cleared first,
 *                    it keeps the result set as with reach_opts.table.
 *   h_level_counts : host, max_levels uint64 (caller-owned): the level counts.
 *   r              : filled as by reach_explore except level_counts = NULL
 *                    (the counts are in h_level_counts[0, r->n_levels)); it
 *                    owns nothing, so reach_result_free is not needed.
 *   hip_stream     : stream for all device work.
 * Synchronous.  Errors: LHS_EINVAL (null or mismatched arguments, another
 * device current, more levels than max_levels), LHS_EBUDGET (limits above),
 * LHS_EFULL / LHS_ESTALL (device), LHS_EDEVICE.  Calls are serialised inside
 * the library: they all share the device's one array, which keeps the last
 * call's contents (every call clears what it reads). */
#define LHS_NOALLOC_MAX_CAPACITY (1u << 21)
#define LHS_NOALLOC_MAX_TRANS (1u << 16)
#define LHS_NOALLOC_SCRATCH_BYTES (18u << 20)
lhs_status reach_explore_noalloc(const reach_model *m, lhs_table *t, uint64_t *h_level_counts,
                                 uint32_t max_levels, reach_result *r, void *hip_stream);

/* Counterexample trace (Algorithm 1's deadlock report made concrete): after
 * reach_explore with REACH_F_PARENTS on table t, the path of slots from s0 to
 * the state stored in `slot` along the recorded predecessors, s0 first;
 * every step is one transition and the path has BFS-depth + 1 states.
 *   h_path : host, max_len uint32 (may be NULL): the slots;
 *   h_rows : host, max_len * state_words uint32 (may be NULL): the vectors;
 *   *len   : path length (also when it exceeds max_len, in which case
 *            nothing is copied and LHS_EINVAL is returned if a buffer was
 *            given).
 * LHS_EINVAL if the table holds no records of its last exploration or
 * `slot` holds no stored state.  Synchronous (one small copy per step). */
lhs_status reach_trace(lhs_table *t, uint32_t slot, uint32_t *h_path, uint32_t *h_rows,
                       uint32_t max_len, uint32_t *len);

/* Deadlock states recorded by the last reach_explore with REACH_F_PARENTS
 * on t: *n = how many were expanded (including those of a level discarded by
 * the cap); the slots of the first min(*n, 1024, max) go to h_slots (host,
 * may be NULL).  Synchronous. */
lhs_status reach_deadlock_slots(lhs_table *t, uint32_t *h_slots, uint32_t max, uint32_t *n);

/* Explore n models (1..1024) together: every model has its own table region
 * (slots, rows, frontiers) and results identical to reach_explore on it
 * alone, so models of different sizes and widths share the GPU.  By default
 * the whole exploration is one persistent launch: its workgroups take
 * (model, tile) items from a device work queue, and the workgroup that
 * finishes a model's last tile of a level finalises that level and queues
 * the next one, so models advance independently.  REACH_F_HOST_LOOP instead
 * runs one launch per step in which every unfinished model advances one
 * level.  All tables of a batch share one line width and lanes per state
 * (internal tables: the tuning table's "batch" choice; given tables must
 * agree on line_slots, and the first one's tps_expand is used).
 *   models  : n host pointers to models (same rules as reach_explore).
 *   o       : capacity = slots per model table (0: pow2 >= 2*state_cap +
 *             2^16 for capped models, 2^21 otherwise); max_levels (0 =
 *             65536); flags; hip_stream.  o->table is ignored.
 *   tables  : optional, n caller tables (NULL entries = internal); a given
 *             table must match the model's width, is cleared first and keeps
 *             the model's reachable set.
 *   results : n results, filled on LHS_OK (free each with reach_result_free);
 *             gpu_ms is the time of the whole batch.
 * Synchronous. */
lhs_status reach_explore_batch(const reach_model *const *models, uint32_t n, const reach_opts *o,
                               lhs_table *const *tables, reach_result *results);

/* ------------------------------------------------------------------------
 * Serving: reachability queries with continuous batching.
 *
 * A server owns a worker thread and a HIP stream on the device that was
 * current at reach_server_create.  By default one persistent launch serves
 * every query on the GPU: its workgroups take (query, tile) items from a
 * device work queue, the workgroup that finishes a query's level advances
 * that query alone, new queries are posted to the running launch (an idle
 * workgroup inserts s0 and starts it at once) and finished ones are
 * reported through completion records in host memory, so a query starts and
 * ends without waiting for a kernel boundary.  The launch ends once idle
 * and is started again when work arrives.  REACH_SERVER_F_ROUNDS instead
 * works in rounds of four BFS level steps run by the device alone (every
 * step expands the current level of every active query in one launch), and
 * admits and retires queries between rounds.  Either way queries are
 * admitted first come, first served, while their tables fit the
 * device-memory budget; tables stay resident in a pool and are reused by
 * later queries of the same capacity and width.  A query's result equals
 * reach_explore on it alone.
 * ---------------------------------------------------------------------- */
typedef struct reach_server reach_server;

typedef struct reach_server_opts {
    uint64_t budget_bytes; /* device memory for query tables (0 = 200 GiB)      */
    uint64_t capacity;     /* slots per query table (power of two); 0 = pow2 >=
                              2*state_cap + 2^16 if the model is capped, else
                              2^21                                               */
    uint32_t max_active;   /* queries on the GPU at once, at most 1024 (0 = 1024) */
    uint32_t flags;        /* REACH_SERVER_F_*                                  */
    lhs_config table;      /* shape of every query table; all zero = the
                              tuning table's "batch" choice                   */
} reach_server_opts;

/* Rounds of host-launched level steps instead of the persistent launch. */
#define REACH_SERVER_F_ROUNDS 1u

typedef struct reach_query_times {
    double submit_s;       /* reach_server_clock() at submission                */
    double admit_s;        /* ... when its table was granted                    */
    double done_s;         /* ... when its result was complete                  */
} reach_query_times;

typedef struct reach_server_stats {
    uint64_t submitted, completed, steps;
    uint64_t states;        /* states found by successfully completed queries   */
    uint64_t bytes_in_use;  /* table memory allocated (in use and pooled)       */
    uint64_t bytes_pooled;  /* of which idle in the pool                        */
    uint64_t peak_bytes;
    uint32_t active, queued;
    double busy_s;          /* worker time spent admitting and stepping         */
} reach_server_stats;

/* Monotonic clock (seconds) used for reach_query_times. */
double reach_server_clock(void);

/* Start a server.  o may be NULL (defaults).  Errors: LHS_EINVAL (bad
 * capacity), LHS_EDEVICE. */
lhs_status reach_server_create(const reach_server_opts *o, reach_server **out);

/* Queue a query; the model (host memory) is copied, the caller may free it
 * on return.  *ticket identifies the query.  LHS_EBUDGET if its table can
 * never fit the budget, LHS_EINVAL for an invalid model (or, on a
 * persistent server, a table of more than 2^30 slots: the work queue holds a
 * full level of every query on the GPU). */
lhs_status reach_server_submit(reach_server *s, const reach_model *m, uint64_t *ticket);

/* reach_server_submit on a table of the caller's (NULL = the pool, as
 * reach_server_submit).  The query's result is its visited set V of
 * Algorithm 1, which the table keeps: once the query is collected
 * (reach_server_poll / reach_server_wait) the table holds exactly the states
 * of the kept levels (a level discarded by state_cap is undone) and can be
 * read with lhs_dump / lhs_count.  The table is cleared when the query is
 * admitted.  It must have the query's width, the server's line_slots and the
 * server's device, which must be current, and capacity > state_cap.  Its
 * memory is the caller's: it is not counted against budget_bytes and never
 * pooled.  Its BFS frontiers are allocated now if it has none.  Between
 * submission and collection the caller must not use or destroy the table;
 * a table serves one query at a time.  Errors: LHS_EINVAL (also for a table
 * already serving a query), LHS_ENOMEM. */
lhs_status reach_server_submit_ex(reach_server *s, const reach_model *m, lhs_table *table,
                                  uint64_t *ticket);

/* Non-blocking: LHS_EAGAIN while the query runs; otherwise fills r (free with
 * reach_result_free) and t (either may be NULL), forgets the ticket and
 * returns the query's status (LHS_OK or its device error).  LHS_ENOTFOUND for
 * an unknown or already collected ticket. */
lhs_status reach_server_poll(reach_server *s, uint64_t ticket, reach_result *r, reach_query_times *t);

/* Blocking version of reach_server_poll.  Any thread may submit, poll and
 * wait; when several threads wait on one ticket, one of them collects the
 * result and the others return LHS_ENOTFOUND. */
lhs_status reach_server_wait(reach_server *s, uint64_t ticket, reach_result *r, reach_query_times *t);

lhs_status reach_server_get_stats(reach_server *s, reach_server_stats *out);

/* Finish every queued and running query, stop the worker and free all device
 * memory; uncollected results are dropped.  NULL is accepted. */
lhs_status reach_server_destroy(reach_server *s);

/* ------------------------------------------------------------------------
 * Measurement probes (ceilings for the roofline of find-or-put).
 * All asynchronous on hip_stream; d_sink is a device uint64 the kernels may
 * write to keep their loads alive.
 * ---------------------------------------------------------------------- */

/* n_reads reads of uniformly random lines of line_bytes (64, 128 or 256)
 * bytes of d_buf (buf_bytes / line_bytes must be a power of two, d_buf
 * line_bytes-aligned), each line read by one lane (lanes_per_line = 1,
 * line_bytes/16 sixteen-byte loads) or by line_bytes/16 cooperating lanes
 * (lanes_per_line = line_bytes/16, one 16-byte load each). */
lhs_status lhs_probe_random_lines(const void *d_buf, uint64_t buf_bytes, uint32_t line_bytes,
                                  uint32_t lanes_per_line, uint64_t n_reads, uint64_t seed,
                                  uint64_t *d_sink, void *hip_stream);

/* n_ops 64-bit compare-and-swap operations (0 -> random value with bit 63
 * set) at uniformly random slots of d_slots (n_slots a power of two). */
lhs_status lhs_probe_random_cas(uint64_t *d_slots, uint64_t n_slots, uint64_t n_ops,
                                uint64_t seed, uint64_t *d_sink, void *hip_stream);

/* n_ops accesses in the remaining forms of a find-or-put, at uniformly random
 * positions of d_buf (buf_bytes / 64 a power of two, d_buf 64-byte aligned):
 *   LHS_PROBE_SLOT_STORE  8-byte agent-scope store to a random slot, one lane
 *                         per store (the DONE publish of an insert);
 *   LHS_PROBE_ROW_STORE   64-byte row written by eight lanes with 8-byte
 *                         agent-scope stores (the row write of an insert);
 *   LHS_PROBE_ROW_LOAD    the same row read by eight lanes with 8-byte
 *                         agent-scope loads (the row compare of a lookup).
 * d_buf's contents are overwritten by the store forms.  LHS_EINVAL for an
 * unknown form, a null pointer, a size or an alignment outside the above. */
typedef enum lhs_probe_form {
    LHS_PROBE_SLOT_STORE = 0,
    LHS_PROBE_ROW_STORE = 1,
    LHS_PROBE_ROW_LOAD = 2
} lhs_probe_form;
lhs_status lhs_probe_random_access(void *d_buf, uint64_t buf_bytes, uint32_t form, uint64_t n_ops,
                                   uint64_t seed, uint64_t *d_sink, void *hip_stream);

/* Streaming copy of `bytes` (multiple of 16, 16-byte aligned pointers): the
 * reference kernel for calibrating hardware traffic counters. */
lhs_status lhs_probe_copy(void *d_dst, const void *d_src, uint64_t bytes, void *hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* LHS_H */
