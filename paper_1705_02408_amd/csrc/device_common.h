// Device helpers shared by the search and graph kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define MPAP_INF __builtin_inff()

// Label layout: float4 {c, d, m, meta}.  meta (as int32):
//   open  : bit 31 set, low 31 bits = parent label id + 1 (0 for the root)
//   closed: the label's own arena id (>= 0)
#define MPAP_OPEN_BIT 0x80000000u

__device__ __forceinline__ bool lab_open(const float4 &L) {
    return (__float_as_uint(L.w) & MPAP_OPEN_BIT) != 0u;
}
__device__ __forceinline__ int lab_parent(const float4 &L) {
    return (int)(__float_as_uint(L.w) & 0x7fffffffu) - 1;
}
// weak dominance a <= b in every objective (m is 0 for two objectives)
__device__ __forceinline__ bool lab_le(const float4 &a, const float4 &b) {
    return a.x <= b.x && a.y <= b.y && a.z <= b.z;
}
__device__ __forceinline__ bool lab_eq(const float4 &a, const float4 &b) {
    return a.x == b.x && a.y == b.y && a.z == b.z;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }
__device__ __forceinline__ uint64_t ballot64(bool p) { return (uint64_t)__ballot(p); }
__device__ __forceinline__ int lanes_below(uint64_t m) {
    return (int)__popcll(m & __lanemask_lt());
}

template <typename T>
__device__ __forceinline__ T wave_incl_scan_add(T v) {
    const int l = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        T u = __shfl_up(v, o, 64);
        if (l >= o) v += u;
    }
    return v;
}
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_min(float v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ int wave_max_i(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
    return v;
}

// Block-wide exclusive scan of one int per thread.  `scratch` holds at least
// blockDim.x/64 + 1 ints of LDS.  Returns the exclusive prefix; *total gets
// the block sum.  Must be called by every thread of the block.
__device__ __forceinline__ int block_excl_scan(int v, int *scratch, int *total) {
    const int l = lane_id();
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    int incl = wave_incl_scan_add(v);
    __syncthreads();
    if (l == 63) scratch[w] = incl;
    __syncthreads();
    int before = 0, all = 0;
    for (int i = 0; i < nw; ++i) {
        int s = scratch[i];
        if (i < w) before += s;
        all += s;
    }
    *total = all;
    __syncthreads();
    return before + incl - v;
}

__device__ __forceinline__ long long block_sum_ll(long long v, long long *scratch) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    long long s = 0;
    for (int i = 0; i < nw; ++i) s += scratch[i];
    __syncthreads();
    return s;
}

__device__ __forceinline__ long long block_min_ll(long long v, long long *scratch) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, (long long)__shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    long long s = scratch[0];
    for (int i = 1; i < nw; ++i) s = min(s, scratch[i]);
    __syncthreads();
    return s;
}

__device__ __forceinline__ float block_min(float v, float *scratch) {
    v = wave_min(v);
    const int w = threadIdx.x >> 6;
    const int nw = blockDim.x >> 6;
    __syncthreads();
    if (lane_id() == 0) scratch[w] = v;
    __syncthreads();
    float s = MPAP_INF;
    for (int i = 0; i < nw; ++i) s = fminf(s, scratch[i]);
    __syncthreads();
    return s;
}

// Grid-wide barrier for a cooperative launch.  `counter` is zeroed before the
// launch; every block must call it the same number of times.  The wait is
// bounded: after `spin_limit` polls the block records `timeout_flag` in
// *err and proceeds, so a broken launch still terminates.
//
// Cache maintenance is done once per workgroup, not once per wave: every wave
// first waits until its own global stores and atomics are acknowledged by the
// L2 of its XCD; after the workgroup barrier one thread writes that L2's dirty
// lines back (agent-scope release), arrives, polls the counter with relaxed
// loads (which leave the caches alone, so blocks still at work on the same
// XCD keep their L2 contents) and, once all blocks have arrived, drops stale
// lines (agent-scope acquire) before the workgroup goes on.  The waves of a
// workgroup share one CU and its L1, so the one invalidation serves them all.
__device__ __forceinline__ void grid_barrier(unsigned *counter, unsigned nblocks,
                                             unsigned &epoch, int *err, int timeout_flag,
                                             unsigned long long spin_limit) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);  // vmcnt, expcnt and lgkmcnt all zero
    __syncthreads();
    if (threadIdx.x == 0) {
        epoch += 1u;
        const unsigned target = epoch * nblocks;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned long long spins = 0;
        while (__hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(2);
            if (++spins > spin_limit) {
                atomicOr(err, timeout_flag);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

// float32 -> bfloat16 bits, round to nearest, ties to even (NaN stays NaN)
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }
