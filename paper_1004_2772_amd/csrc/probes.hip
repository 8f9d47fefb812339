// Roofline probes: the memory-system ceilings the find-or-put kernel is
// measured against.
//   random lines : uniformly random line-aligned lines (64, 128 or 256 bytes)
//                  of a large buffer, read either by one lane (16-byte loads,
//                  one after another) or by line/16 cooperating lanes (16 B
//                  each, one coalesced access: the find-or-put pattern).
//   random CAS   : 64-bit compare-and-swap at uniformly random slots.
//   random slot store, row store, row load: the other accesses of an insert
//                  or lookup (DONE publish, row write, row compare) in the
//                  form find-or-put issues them.
//   copy         : a plain streaming copy, the reference for hardware
//                  traffic counters.
// Indices come from the SplitMix64 output function applied to a counter
// (Steele, Lea, Flood, "Fast splittable pseudorandom number generators", 2014).
#include "internal.h"

namespace {

__device__ __forceinline__ uint64_t splitmix(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// C = 16-byte chunks per line (4, 8, 16).
template <uint32_t C>
__global__ __launch_bounds__(256) void k_probe_lines_lane(const uint4 *buf, uint64_t n_lines,
                                                          uint64_t n_reads, uint64_t seed,
                                                          uint64_t *sink) {
    uint32_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_reads;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t line = splitmix(seed ^ i) & (n_lines - 1);
        const uint4 *p = buf + line * C;
#pragma unroll
        for (uint32_t q = 0; q < C; ++q) {
            const uint4 x = p[q];
            acc ^= x.x ^ x.y ^ x.z ^ x.w;
        }
    }
    if (acc == 0x9E3779B9u)
        sink[0] = acc;
}

template <uint32_t C>
__global__ __launch_bounds__(256) void k_probe_lines_coop(const uint4 *buf, uint64_t n_lines,
                                                          uint64_t n_reads, uint64_t seed,
                                                          uint64_t *sink) {
    constexpr uint32_t CS = C == 4 ? 2u : (C == 8 ? 3u : 4u);
    uint32_t acc = 0;
    const uint32_t sub = threadIdx.x & (C - 1);
    for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> CS; i < n_reads;
         i += ((uint64_t)gridDim.x * blockDim.x) >> CS) {
        const uint64_t line = splitmix(seed ^ i) & (n_lines - 1);
        const uint4 x = buf[line * C + sub];
        acc ^= x.x ^ x.y ^ x.z ^ x.w;
    }
    if (acc == 0x9E3779B9u)
        sink[0] = acc;
}

__global__ __launch_bounds__(256) void k_probe_cas(uint64_t *slots, uint64_t n_slots, uint64_t n_ops,
                                                   uint64_t seed, uint64_t *sink) {
    uint32_t won = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops;
         i += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = splitmix(seed ^ i);
        uint64_t expected = 0;
        won += __hip_atomic_compare_exchange_strong(slots + (r & (n_slots - 1)), &expected,
                                                    r | (1ull << 63), __ATOMIC_RELAXED,
                                                    __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (won == 0xFFFFFFFFu)
        sink[0] = won;
}

// FORM 0: 8-byte agent-scope store to a random slot, one lane each.
// FORM 1 / 2: 64-byte row at a random row position, stored / loaded by eight
// lanes with 8-byte agent-scope accesses.  n_rows = 64-byte rows in buf.
template <uint32_t FORM>
__global__ __launch_bounds__(256) void k_probe_access(uint64_t *buf, uint64_t n_rows, uint64_t n_ops,
                                                      uint64_t seed, uint64_t *sink) {
    uint64_t acc = 0;
    if constexpr (FORM == 0) {
        for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_ops;
             i += (uint64_t)gridDim.x * blockDim.x) {
            const uint64_t r = splitmix(seed ^ i);
            __hip_atomic_store(buf + (r & (n_rows * 8 - 1)), r | 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    } else {
        const uint32_t sub = threadIdx.x & 7u;
        for (uint64_t i = ((uint64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3; i < n_ops;
             i += ((uint64_t)gridDim.x * blockDim.x) >> 3) {
            const uint64_t r = splitmix(seed ^ i);
            uint64_t *p = buf + (r & (n_rows - 1)) * 8 + sub;
            if constexpr (FORM == 1)
                __hip_atomic_store(p, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            else
                acc ^= __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    if (acc == 0x9E3779B97F4A7C15ull)
        sink[0] = acc;
}

__global__ __launch_bounds__(256) void k_probe_copy(uint4 *dst, const uint4 *src, uint64_t n) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

uint32_t probe_grid(uint64_t items) {
    const uint64_t b = (items + 255) / 256;
    return (uint32_t)(b < 8192 ? (b ? b : 1) : 8192);
}

}  // namespace

extern "C" {

lhs_status lhs_probe_random_lines(const void *d_buf, uint64_t buf_bytes, uint32_t line_bytes,
                                  uint32_t lanes_per_line, uint64_t n_reads, uint64_t seed,
                                  uint64_t *d_sink, void *hip_stream) {
    if (line_bytes != 64 && line_bytes != 128 && line_bytes != 256)
        return LHS_EINVAL;
    const uint64_t n_lines = buf_bytes / line_bytes;
    const uint32_t C = line_bytes / 16;
    if (!d_buf || !d_sink || !lhs::is_pow2(n_lines) || (lanes_per_line != 1 && lanes_per_line != C) ||
        ((uintptr_t)d_buf & (line_bytes - 1)))
        return LHS_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    const uint4 *b = (const uint4 *)d_buf;
    const uint32_t gl = probe_grid(n_reads), gc = probe_grid(n_reads * C);
    switch (C * (lanes_per_line == 1 ? 1 : 100)) {
    case 4: hipLaunchKernelGGL(k_probe_lines_lane<4>, dim3(gl), dim3(256), 0, s, b, n_lines, n_reads, seed, d_sink); break;
    case 8: hipLaunchKernelGGL(k_probe_lines_lane<8>, dim3(gl), dim3(256), 0, s, b, n_lines, n_reads, seed, d_sink); break;
    case 16: hipLaunchKernelGGL(k_probe_lines_lane<16>, dim3(gl), dim3(256), 0, s, b, n_lines, n_reads, seed, d_sink); break;
    case 400: hipLaunchKernelGGL(k_probe_lines_coop<4>, dim3(gc), dim3(256), 0, s, b, n_lines, n_reads, seed, d_sink); break;
    case 800: hipLaunchKernelGGL(k_probe_lines_coop<8>, dim3(gc), dim3(256), 0, s, b, n_lines, n_reads, seed, d_sink); break;
    default: hipLaunchKernelGGL(k_probe_lines_coop<16>, dim3(gc), dim3(256), 0, s, b, n_lines, n_reads, seed, d_sink); break;
    }
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status lhs_probe_random_cas(uint64_t *d_slots, uint64_t n_slots, uint64_t n_ops, uint64_t seed,
                                uint64_t *d_sink, void *hip_stream) {
    if (!d_slots || !d_sink || !lhs::is_pow2(n_slots))
        return LHS_EINVAL;
    hipLaunchKernelGGL(k_probe_cas, dim3(probe_grid(n_ops)), dim3(256), 0, (hipStream_t)hip_stream,
                       d_slots, n_slots, n_ops, seed, d_sink);
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status lhs_probe_random_access(void *d_buf, uint64_t buf_bytes, uint32_t form, uint64_t n_ops,
                                   uint64_t seed, uint64_t *d_sink, void *hip_stream) {
    const uint64_t n_rows = buf_bytes / 64;
    if (!d_buf || !d_sink || form > LHS_PROBE_ROW_LOAD || !lhs::is_pow2(n_rows) || ((uintptr_t)d_buf & 63))
        return LHS_EINVAL;
    hipStream_t s = (hipStream_t)hip_stream;
    uint64_t *b = (uint64_t *)d_buf;
    switch (form) {
    case LHS_PROBE_SLOT_STORE:
        hipLaunchKernelGGL(k_probe_access<0>, dim3(probe_grid(n_ops)), dim3(256), 0, s, b, n_rows, n_ops, seed, d_sink);
        break;
    case LHS_PROBE_ROW_STORE:
        hipLaunchKernelGGL(k_probe_access<1>, dim3(probe_grid(n_ops * 8)), dim3(256), 0, s, b, n_rows, n_ops, seed, d_sink);
        break;
    default:
        hipLaunchKernelGGL(k_probe_access<2>, dim3(probe_grid(n_ops * 8)), dim3(256), 0, s, b, n_rows, n_ops, seed, d_sink);
        break;
    }
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

lhs_status lhs_probe_copy(void *d_dst, const void *d_src, uint64_t bytes, void *hip_stream) {
    if (!d_dst || !d_src || (bytes & 15) || ((uintptr_t)d_dst & 15) || ((uintptr_t)d_src & 15))
        return LHS_EINVAL;
    const uint64_t n = bytes / 16;
    hipLaunchKernelGGL(k_probe_copy, dim3(probe_grid(n)), dim3(256), 0, (hipStream_t)hip_stream,
                       (uint4 *)d_dst, (const uint4 *)d_src, n);
    return hipGetLastError() == hipSuccess ? LHS_OK : LHS_EDEVICE;
}

}  // extern "C"
