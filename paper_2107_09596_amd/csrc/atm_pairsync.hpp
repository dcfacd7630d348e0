// Device-coherent accesses for two workgroups that share one task (a pair): values one half writes
// and the other reads go through relaxed atomics at agent scope, which bypass the non-coherent
// caches, and a half waits for its own stores to complete before it raises its counter.
#pragma once
#include <hip/hip_runtime.h>

namespace atm {
namespace pair {

__device__ __forceinline__ void put(float* p, float v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float get(const float* p)
{
    return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void put(double* p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double get(const double* p)
{
    return __hip_atomic_load(const_cast<double*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// this thread's stores (and loads) have completed
__device__ __forceinline__ void drain()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    __builtin_amdgcn_s_waitcnt(0);
}

// Blocks b and b ^ 8 of a grid of 16 g blocks form pair ((b >> 4) << 3) | (b & 7): workgroups are
// dealt to the eight XCDs in turn, so the two halves of a pair share one L2.
__device__ __forceinline__ int pair_of(int b) { return ((b >> 4) << 3) | (b & 7); }
__device__ __forceinline__ int half_of(int b) { return (b >> 3) & 1; }

}  // namespace pair
}  // namespace atm
