// The lockless table: lifecycle, batched find-or-put and inspection.
//
// Memory layout in HBM (section "Hash Table Design": separated data, 2^n
// table, memoised hash, empty = 0):
//   bucket : uint64[capacity]            8 B/slot, 8/16/32 slots per line
//   data   : uint32[capacity][W]         row of slot i at data + i*W
//   status : DevStatus                   sticky error + counters
#include <algorithm>
#include <cstring>
#include <new>
#include <vector>

#include "internal.h"

using namespace lhs;

namespace {

constexpr int kBlock = 256;
constexpr uint64_t kDefaultSeed = 0x5851F42D4C957F2Dull;
constexpr uint32_t kMaxGrid = 1u << 19;

// A vector staged in LDS (row of W words); descriptor x = word offset of
// the row from the LDS base.
struct LdsRow {
    const uint32_t *r;
    __device__ __forceinline__ uint32_t get(uint32_t i) const { return r[i]; }
    __device__ __forceinline__ static LdsRow decode(const uint32_t *smem, uint2 d) {
        return LdsRow{smem + d.x};
    }
};

// Batched find-or-put.  A workgroup takes a tile of 256 consecutive input
// rows: it stages them into LDS with coalesced loads (rows padded to an odd
// stride so that lanes reading different rows hit different banks), hashes
// each row with one lane, then runs find-or-put.  G == 1: one operation per
// lane with wavefront-cooperative line and row accesses (256 operations in
// flight per workgroup); the lane keeps its hash and result in registers and
// writes seen/index itself (lane i <-> row i: coalesced).  G > 1: one group
// of G lanes per operation (256/G in flight, G rounds per tile); hashes and
// results go through LDS so that seen/index are written coalesced.
// One lane per operation with 8-slot lines (the tuned shape of large
// tables): at most 80 VGPRs, six waves per SIMD, as the LDS of a 16-word
// tile allows (measured 0.8 % faster than five).
template <int G, uint32_t LS>
__global__ __launch_bounds__(kBlock, (G == 1 && LS == 8) ? 6 : 1) void k_find_or_put(TableView t, const uint32_t *__restrict__ in,
                                                        uint64_t n, uint8_t *__restrict__ seen,
                                                        uint32_t *__restrict__ index,
                                                        uint32_t magicW) {
    extern __shared__ uint32_t smem[];
    const uint32_t W = t.W, stride = W | 1u;
    uint32_t *tile = smem;                                          // kBlock x stride
    uint64_t *hs = reinterpret_cast<uint64_t *>(tile + kBlock * stride);
    uint32_t *res_slot = reinterpret_cast<uint32_t *>(hs + kBlock);
    uint32_t *res_code = res_slot + kBlock;
    constexpr uint32_t NG = kBlock / G;
    const uint32_t tid = threadIdx.x, gi = tid / G;
    LaneCounters cnt;
    for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < n;
         base += (uint64_t)gridDim.x * kBlock) {
        const uint32_t rows = (uint32_t)min<uint64_t>(kBlock, n - base);
        const uint32_t words = rows * W;
        const uint32_t *src = in + base * W;
        __syncthreads();
        if ((W & 3u) == 0 && (reinterpret_cast<uintptr_t>(in) & 15u) == 0) {
            // rows of a multiple of four words, 16-byte aligned: 16-byte
            // loads, each inside one row
            typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
            const u32x4 *src4 = reinterpret_cast<const u32x4 *>(src);
            for (uint32_t f4 = tid; f4 < words / 4; f4 += kBlock) {
                const uint32_t f = 4 * f4, r = __umulhi(f, magicW);
                const u32x4 x = __builtin_nontemporal_load(src4 + f4);   // read once
                uint32_t *dst = tile + r * stride + (f - r * W);
                dst[0] = x.x;
                dst[1] = x.y;
                dst[2] = x.z;
                dst[3] = x.w;
            }
        } else {
            for (uint32_t f = tid; f < words; f += kBlock) {
                const uint32_t r = W == 1 ? f : __umulhi(f, magicW);
                tile[r * stride + (f - r * W)] = src[f];
            }
        }
        __syncthreads();
        uint64_t h = 0;
        if (tid < rows)
            h = hash_vec(LdsRow{tile + tid * stride}, W, t.seed);
        if constexpr (G > 1) {
            if (tid < rows)
                hs[tid] = h;
            __syncthreads();
        }
        if constexpr (G == 1) {
            __shared__ WaveScratch<LS> ws[kBlock / 64];
            const bool active = tid < rows;
            uint32_t slot, code;
            find_or_put_wave<LS, LdsRow>(t, &ws[tid / 64], smem, make_uint2(tid * stride, 0u), h, active,
                                         slot, code, cnt);
            if (active) {
                __builtin_nontemporal_store((uint8_t)(code == kSeen ? 1 : (code == kNew ? 0 : 0xFF)), seen + base + tid);
                if (index)
                    __builtin_nontemporal_store(slot, index + base + tid);
            }
        } else {
            for (uint32_t r = 0; r < G; ++r) {
                const uint32_t op = r * NG + gi;
                const bool active = op < rows;
                const uint32_t o = active ? op : 0;
                uint32_t slot, code;
                find_or_put<G, LS>(t, LdsRow{tile + o * stride}, hs[o], active, slot, code, cnt);
                if (active && (tid & (G - 1)) == 0) {
                    res_slot[op] = slot;
                    res_code[op] = code;
                }
            }
            __syncthreads();
            if (tid < rows) {
                const uint32_t code = res_code[tid];
                seen[base + tid] = code == kSeen ? 1 : (code == kNew ? 0 : 0xFF);
                if (index)
                    index[base + tid] = res_slot[tid];
            }
        }
    }
    flush_counters(t, cnt);
}

// Zero n 64-bit words (p 16-byte aligned): 16-byte stores, so one
// wavefront store instruction writes 1 KiB of whole lines.
__global__ void k_zero_u64(uint64_t *p, uint64_t n) {
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    u32x4 *q = reinterpret_cast<u32x4 *>(p);
    const uint64_t n2 = n / 2, stride = (uint64_t)gridDim.x * blockDim.x;
    const u32x4 z = {0u, 0u, 0u, 0u};
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n2; i += stride)
        __builtin_nontemporal_store(z, q + i);
    if ((n & 1) && blockIdx.x == 0 && threadIdx.x == 0)
        p[n - 1] = 0;
}

__global__ void k_zero_status(DevStatus *st) {
    *st = DevStatus{};
}

// Done slots are scanned in chunks of kLineSlots slots (any line width).
// Per-block count of done slots.  Block b covers chunks [b*256, b*256+256),
// thread i one chunk.
__global__ __launch_bounds__(kBlock) void k_count_done(const uint64_t *bucket, uint64_t lines,
                                                       uint32_t *block_counts) {
    __shared__ uint32_t part[kBlock / 64];
    const uint64_t line = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t c = 0;
    if (line < lines) {
        const uint4 *lp = reinterpret_cast<const uint4 *>(bucket + line * kLineSlots);
        for (uint32_t q = 0; q < kLineSlots / 2; ++q) {
            const uint4 x = lp[q];
            c += (x.y >> 30) == 3u;   // OCC and DONE
            c += (x.w >> 30) == 3u;
        }
    }
    c = wave_sum(c);
    if (__lane_id() == 0)
        part[threadIdx.x / 64] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (int w = 0; w < kBlock / 64; ++w)
            s += part[w];
        block_counts[blockIdx.x] = s;
    }
}

// Ordered gather of done slots: block b writes its rows starting at
// offsets[b], in ascending slot order.
__global__ __launch_bounds__(kBlock) void k_gather_done(const uint64_t *bucket, const uint32_t *data,
                                                        uint32_t W, uint64_t lines,
                                                        const uint64_t *offsets,
                                                        uint32_t *out_rows, uint32_t *out_idx) {
    __shared__ uint32_t scan[kBlock];
    const uint64_t line = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    uint32_t mask = 0;
    if (line < lines) {
        const uint4 *lp = reinterpret_cast<const uint4 *>(bucket + line * kLineSlots);
        for (uint32_t q = 0; q < kLineSlots / 2; ++q) {
            const uint4 x = lp[q];
            mask |= (uint32_t)((x.y >> 30) == 3u) << (2 * q);
            mask |= (uint32_t)((x.w >> 30) == 3u) << (2 * q + 1);
        }
    }
    // inclusive scan of per-thread counts (Hillis-Steele; small)
    scan[threadIdx.x] = __popc(mask);
    __syncthreads();
    for (uint32_t d = 1; d < kBlock; d <<= 1) {
        const uint32_t v = threadIdx.x >= d ? scan[threadIdx.x - d] : 0;
        __syncthreads();
        scan[threadIdx.x] += v;
        __syncthreads();
    }
    uint64_t pos = offsets[blockIdx.x] + scan[threadIdx.x] - __popc(mask);
    while (mask) {
        const uint32_t k = __builtin_ctz(mask);
        mask &= mask - 1;
        const uint64_t slot = line * kLineSlots + k;
        if (out_idx)
            out_idx[pos] = (uint32_t)slot;
        if (out_rows)
            for (uint32_t i = 0; i < W; ++i)
                out_rows[pos * W + i] = data[slot * W + i];
        ++pos;
    }
}

uint32_t grid_for(uint64_t items, uint32_t per_block) {
    const uint64_t b = (items + per_block - 1) / per_block;
    return (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(b, kMaxGrid));
}

// Per-block done counts and their exclusive prefix (host).  Returns total.
lhs_status done_offsets(lhs_table *t, std::vector<uint64_t> &offsets, uint32_t **d_counts_out,
                        uint64_t *total) {
    const uint64_t lines = t->capacity / kLineSlots;
    const uint32_t blocks = (uint32_t)((lines + kBlock - 1) / kBlock);
    uint32_t *d_counts = nullptr;
    LHS_HIP(hipMalloc(&d_counts, blocks * sizeof(uint32_t)));
    hipLaunchKernelGGL(k_count_done, dim3(blocks), dim3(kBlock), 0, t->last_stream, t->bucket, lines,
                       d_counts);
    std::vector<uint32_t> counts(blocks);
    if (hipMemcpyAsync(counts.data(), d_counts, blocks * sizeof(uint32_t), hipMemcpyDeviceToHost,
                       t->last_stream) != hipSuccess ||
        hipStreamSynchronize(t->last_stream) != hipSuccess) {
        (void)hipFree(d_counts);
        return LHS_EDEVICE;
    }
    offsets.resize(blocks);
    uint64_t acc = 0;
    for (uint32_t b = 0; b < blocks; ++b) {
        offsets[b] = acc;
        acc += counts[b];
    }
    *total = acc;
    if (d_counts_out)
        *d_counts_out = d_counts;
    else
        (void)hipFree(d_counts);
    return LHS_OK;
}

}  // namespace

namespace lhs {

lhs_status launch_find_or_put(lhs_table *t, const uint32_t *d_states, uint64_t n, uint8_t *d_seen,
                              uint32_t *d_index, hipStream_t s) {
    if (!n)
        return LHS_OK;
    // G == 1 needs only the row tile; G > 1 also hashes and results
    const uint32_t tps = tps_find_or_put(t);
    const size_t lds = (size_t)kBlock * ((t->W | 1u) + (tps > 1 ? 4u : 0u)) * sizeof(uint32_t);
    const dim3 grid(grid_for(n, kBlock)), block(kBlock);
    const TableView v = view(t);
    const uint32_t mw = div_magic(t->W);
    const lhs_status rc = with_shape(tps, t->line_slots, [&](auto G, auto L) {
        hipLaunchKernelGGL((k_find_or_put<decltype(G)::value, decltype(L)::value>), grid, block, lds, s,
                           v, d_states, n, d_seen, d_index, mw);
        return LHS_OK;
    });
    if (rc != LHS_OK)
        return rc;
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status launch_zero_u64(uint64_t *p, uint64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_u64, dim3(grid_for(n / 2 + 1, kBlock * 4)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status read_status(lhs_table *t, DevStatus *out) {
    LHS_HIP(hipStreamSynchronize(t->last_stream));
    LHS_HIP(hipMemcpy(out, t->status, sizeof(DevStatus), hipMemcpyDeviceToHost));
    return LHS_OK;
}

}  // namespace lhs

extern "C" {

const char *lhs_strerror(lhs_status s) {
    switch (s) {
    case LHS_OK: return "LHS_OK";
    case LHS_EINVAL: return "LHS_EINVAL: invalid argument";
    case LHS_ENOMEM: return "LHS_ENOMEM: out of memory";
    case LHS_EFULL: return "LHS_EFULL: table full (every line probed)";
    case LHS_ESTALL: return "LHS_ESTALL: wait on a slot being written exceeded its bound";
    case LHS_EDEVICE: return "LHS_EDEVICE: HIP runtime error";
    case LHS_EBUDGET: return "LHS_EBUDGET: request exceeds the memory budget";
    case LHS_ENOTFOUND: return "LHS_ENOTFOUND: unknown ticket";
    case LHS_EAGAIN: return "LHS_EAGAIN: not ready";
    }
    return "LHS_?: unknown status";
}

lhs_status lhs_create(uint64_t capacity, uint32_t state_words, lhs_table **out) {
    if (!out || state_words < 1 || state_words > 32)
        return LHS_EINVAL;
    const lhs_config cfg = tuned_config(LHS_TUNE_TABLE, state_words, capacity);
    return lhs_create_ex(capacity, state_words, &cfg, out);
}

lhs_status lhs_create_ex(uint64_t capacity, uint32_t state_words, const lhs_config *cfg,
                         lhs_table **out) {
    lhs_config c{16, LHS_PROBE_DOUBLE, 0, 0};
    if (cfg) {
        c = *cfg;
        if (c.line_slots == 0)
            c.line_slots = 16;
    }
    if (!out || !is_pow2(capacity) || capacity < kLineSlots || capacity > (1ull << 32) ||
        state_words < 1 || state_words > 32 || !valid_line_slots(c.line_slots) ||
        c.probe > LHS_PROBE_QUADRATIC || !valid_tps(c.tps_find_or_put) || !valid_tps(c.tps_expand) ||
        capacity < c.line_slots)
        return LHS_EINVAL;
    *out = nullptr;
    lhs_table *t = new (std::nothrow) lhs_table();
    if (!t)
        return LHS_ENOMEM;
    t->capacity = capacity;
    t->W = state_words;
    t->line_slots = c.line_slots;
    t->probe = c.probe;
    t->tps_fop = c.tps_find_or_put;
    t->tps_exp = c.tps_expand;
    t->lines = (uint32_t)(capacity / c.line_slots);
    // a find-or-put gives up (EFULL) only after its probe sequence has
    // visited every line, i.e. when the table has no empty slot
    t->max_rounds = t->lines;
    t->seed = kDefaultSeed;
    if (hipGetDevice(&t->device) != hipSuccess) {
        delete t;
        return LHS_EDEVICE;
    }
    if (hipMalloc(&t->bucket, capacity * sizeof(uint64_t)) != hipSuccess ||
        hipMalloc(&t->data, capacity * (uint64_t)state_words * sizeof(uint32_t)) != hipSuccess ||
        hipMalloc(&t->status, sizeof(DevStatus)) != hipSuccess) {
        (void)hipGetLastError();
        lhs_destroy(t);
        return LHS_ENOMEM;
    }
    if (lhs_clear(t, nullptr) != LHS_OK || hipStreamSynchronize(nullptr) != hipSuccess) {
        lhs_destroy(t);
        return LHS_EDEVICE;
    }
    *out = t;
    return LHS_OK;
}

lhs_status lhs_destroy(lhs_table *t) {
    if (!t)
        return LHS_OK;
    (void)hipDeviceSynchronize();
    (void)hipFree(t->bucket);
    (void)hipFree(t->data);
    (void)hipFree(t->status);
    (void)hipFree(t->frontier[0]);
    (void)hipFree(t->frontier[1]);
    (void)hipFree(t->level);
    if (t->level_host)
        (void)hipHostFree(t->level_host);
    (void)hipFree(t->parent);
    (void)hipFree(t->dead_rec);
    if (t->gexec)
        (void)hipGraphExecDestroy(t->gexec);
    if (t->gstream)
        (void)hipStreamDestroy(t->gstream);
    (void)hipFree(t->gctx);
    (void)hipFree(t->glevels);
    delete t;
    return LHS_OK;
}

lhs_status lhs_clear(lhs_table *t, void *hip_stream) {
    if (!t)
        return LHS_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    t->last_stream = s;
    t->has_parents = false;
    if (launch_zero_u64(t->bucket, t->capacity, s) != LHS_OK)
        return LHS_EDEVICE;
    hipLaunchKernelGGL(k_zero_status, dim3(1), dim3(1), 0, s, t->status);
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status lhs_find_or_put(lhs_table *t, const uint32_t *d_states, uint64_t n, uint8_t *d_seen,
                           uint32_t *d_index, void *hip_stream) {
    if (!t || n >= (1ull << 32) || (n && (!d_states || !d_seen)))
        return LHS_EINVAL;
    t->last_stream = (hipStream_t)hip_stream;
    return launch_find_or_put(t, d_states, n, d_seen, d_index, (hipStream_t)hip_stream);
}

lhs_status lhs_set_threads_per_state(lhs_table *t, uint32_t tps) {
    if (!t || !valid_tps(tps))
        return LHS_EINVAL;
    t->tps_fop = tps;
    t->tps_exp = tps;
    return LHS_OK;
}

lhs_status lhs_set_counters(lhs_table *t, uint32_t flags) {
    if (!t || (flags & ~(LHS_COUNT_LINES | LHS_COUNT_MERGED)))
        return LHS_EINVAL;
    t->counters = flags;
    return LHS_OK;
}

lhs_status lhs_set_merge(lhs_table *t, uint32_t mode) {
    if (!t || mode > LHS_MERGE_NARROW_TAGS)
        return LHS_EINVAL;
    t->merge = mode;
    return LHS_OK;
}

lhs_status lhs_set_workers(lhs_table *t, uint32_t max_workgroups) {
    if (!t)
        return LHS_EINVAL;
    t->workers = max_workgroups;
    return LHS_OK;
}

lhs_status lhs_get_config(lhs_table *t, lhs_config *out) {
    if (!t || !out)
        return LHS_EINVAL;
    out->line_slots = t->line_slots;
    out->probe = t->probe;
    out->tps_find_or_put = t->tps_fop;
    out->tps_expand = t->tps_exp;
    return LHS_OK;
}

lhs_status lhs_check(lhs_table *t) {
    if (!t)
        return LHS_EINVAL;
    DevStatus st;
    lhs_status rc = read_status(t, &st);
    if (rc != LHS_OK)
        return rc;
    return (lhs_status)st.error;
}

static lhs_status lhs_count_impl(lhs_table *t, uint64_t *out) {
    if (!t || !out)
        return LHS_EINVAL;
    std::vector<uint64_t> offsets;
    return done_offsets(t, offsets, nullptr, out);
}

lhs_status lhs_count(lhs_table *t, uint64_t *out) {
    return lhs::guard([&] { return lhs_count_impl(t, out); });
}

static lhs_status lhs_dump_impl(lhs_table *t, uint32_t *h_states, uint32_t *h_index, uint64_t max_rows,
                                uint64_t *n_rows) {
    if (!t || !n_rows)
        return LHS_EINVAL;
    std::vector<uint64_t> offsets;
    uint64_t total = 0;
    lhs_status rc = done_offsets(t, offsets, nullptr, &total);
    if (rc != LHS_OK)
        return rc;
    *n_rows = total;
    if (total > max_rows)
        return (h_states || h_index) ? LHS_EINVAL : LHS_OK;
    if (!total || (!h_states && !h_index))
        return LHS_OK;
    uint64_t *d_off = nullptr;
    uint32_t *d_rows = nullptr, *d_idx = nullptr;
    const uint64_t lines = t->capacity / kLineSlots;
    const uint32_t blocks = (uint32_t)offsets.size();
    hipStream_t s = t->last_stream;
    rc = LHS_EDEVICE;
    if (hipMalloc(&d_off, blocks * sizeof(uint64_t)) == hipSuccess &&
        (!h_states || hipMalloc(&d_rows, total * t->W * sizeof(uint32_t)) == hipSuccess) &&
        (!h_index || hipMalloc(&d_idx, total * sizeof(uint32_t)) == hipSuccess) &&
        hipMemcpyAsync(d_off, offsets.data(), blocks * sizeof(uint64_t), hipMemcpyHostToDevice, s) ==
            hipSuccess) {
        hipLaunchKernelGGL(k_gather_done, dim3(blocks), dim3(kBlock), 0, s, t->bucket, t->data, t->W,
                           lines, d_off, d_rows, d_idx);
        bool ok = hipGetLastError() == hipSuccess;
        if (ok && h_states)
            ok = hipMemcpyAsync(h_states, d_rows, total * t->W * sizeof(uint32_t),
                                hipMemcpyDeviceToHost, s) == hipSuccess;
        if (ok && h_index)
            ok = hipMemcpyAsync(h_index, d_idx, total * sizeof(uint32_t), hipMemcpyDeviceToHost, s) ==
                 hipSuccess;
        if (ok)
            ok = hipStreamSynchronize(s) == hipSuccess;
        rc = ok ? LHS_OK : LHS_EDEVICE;
    } else {
        (void)hipGetLastError();
        rc = LHS_ENOMEM;
    }
    (void)hipFree(d_off);
    (void)hipFree(d_rows);
    (void)hipFree(d_idx);
    return rc;
}

lhs_status lhs_dump(lhs_table *t, uint32_t *h_states, uint32_t *h_index, uint64_t max_rows,
                    uint64_t *n_rows) {
    return lhs::guard([&] { return lhs_dump_impl(t, h_states, h_index, max_rows, n_rows); });
}

lhs_status lhs_dump_slots(lhs_table *t, uint64_t *h_slots) {
    if (!t || !h_slots)
        return LHS_EINVAL;
    LHS_HIP(hipStreamSynchronize(t->last_stream));
    LHS_HIP(hipMemcpy(h_slots, t->bucket, t->capacity * sizeof(uint64_t), hipMemcpyDeviceToHost));
    return LHS_OK;
}

lhs_status lhs_get_info(lhs_table *t, lhs_info *out) {
    if (!t || !out)
        return LHS_EINVAL;
    DevStatus st;
    lhs_status rc = read_status(t, &st);
    if (rc != LHS_OK)
        return rc;
    std::memset(out, 0, sizeof(*out));
    out->capacity = t->capacity;
    out->state_words = t->W;
    out->line_slots = t->line_slots;
    out->probe = t->probe;
    out->tps_find_or_put = tps_find_or_put(t);
    out->tps_expand = tps_expand(t);
    out->hash_seed = t->seed;
    out->wait_hits = st.wait_hits;
    out->cas_failures = st.cas_failures;
    out->lines_probed = st.lines;
    out->merged = st.merged;
    out->error = st.error;
    return LHS_OK;
}

}  // extern "C"
