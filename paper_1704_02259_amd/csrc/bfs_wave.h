// Wavefront helpers shared by the single-root and batched kernels (gfx950,
// wave64).  Every cross-lane read here must run with all lanes active.
#pragma once

#include <hip/hip_runtime.h>

namespace hybfs {

#define AGENT __HIP_MEMORY_SCOPE_AGENT

static __device__ __forceinline__ unsigned long long ld_relaxed(unsigned long long *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, AGENT);
}

static __device__ __forceinline__ long long bcast64(long long x, int lane)
{
    int lo = __builtin_amdgcn_readlane((int)(x & 0xFFFFFFFFll), lane);
    int hi = __builtin_amdgcn_readlane((int)(x >> 32), lane);
    return ((long long)hi << 32) | (unsigned int)lo;
}

static __device__ __forceinline__ unsigned long long bcast_u64(unsigned long long x, int lane)
{
    return (unsigned long long)bcast64((long long)x, lane);
}

static __device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
    return x;
}

// Inclusive prefix sum across the wavefront.
static __device__ __forceinline__ long long wave_incl_scan(long long x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, (unsigned)o);
        if (lane >= o) x += y;
    }
    return x;
}

// Inclusive prefix sum of 32-bit values across the wavefront.
static __device__ __forceinline__ int wave_incl_scan32(int x)
{
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, (unsigned)o);
        if (lane >= o) x += y;
    }
    return x;
}

static __device__ __forceinline__ bool test_bit(const unsigned long long *bm, int v)
{
    return (bm[v >> 6] >> (v & 63)) & 1ull;
}

// Position of the k-th set bit (k from 0) of a 64-bit word.
static __device__ __forceinline__ int select_bit(unsigned long long x, int k)
{
    int pos = 0;
#pragma unroll
    for (int width = 32; width > 0; width >>= 1) {
        const unsigned long long low = x & ((1ull << width) - 1ull);
        const int c = __popcll(low);
        if (k >= c) {
            k -= c;
            x >>= width;
            pos += width;
        } else {
            x = low;
        }
    }
    return pos;
}

// Largest lane l whose (non-decreasing across lanes) value key_l is <= x.
static __device__ __forceinline__ int lane_search(int key, int x)
{
    int lo = 0;
#pragma unroll
    for (int step = 32; step > 0; step >>= 1) {
        const int c = lo + step;
        if (__shfl(key, c) <= x) lo = c;
    }
    return lo;
}

// End of a traversal, in the finisher's thread 0: a traversal that did not
// end normally or failed a device-side check is remembered for
// bfs_graph_sync when it was enqueued asynchronously (a synchronous run reads
// done and status itself).  Other kernels set status bits with device-scope
// atomics, so the flags are read at that scope.
template <class C_>
__device__ __forceinline__ void record_failure(C_ *C)
{
    const int dn = __hip_atomic_load(&C->done, __ATOMIC_RELAXED, AGENT);
    unsigned st = __hip_atomic_load((unsigned *)&C->status, __ATOMIC_RELAXED, AGENT);
    if (C->fail_injected) {
        st |= 0x200u;
        atomicOr((unsigned *)&C->status, 0x200u);
    }
    if (C->async_run && (dn != 1 || st != 0u)) {
        C->err_runs += 1u;
        C->err_bits |= st | (dn != 1 ? 0x100u : 0u);
    }
}

}  // namespace hybfs
