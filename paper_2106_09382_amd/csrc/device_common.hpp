// Device helpers shared by the kernels: coherent loads/stores for data that
// crosses workgroups, the soft-threshold, and type traits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace concord {

// Data exchanged between workgroups lives in ordinary device memory and is
// only ever touched through agent-scope (device-coherent) loads and stores.
// On gfx950 these are plain global loads/stores with the sc1 bit: they are
// served from the device-coherent level, never from a stale line in another
// XCD's L2.  Relaxed order is enough because ordering is made explicit with
// `wait_stores()` before a workgroup signals, and by issuing the reads only
// after the signal has been observed.
template <typename T>
__device__ __forceinline__ T ld_dev(const T *p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T>
__device__ __forceinline__ void st_dev(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait until every vector memory operation this wave issued has completed
// (for agent-scope stores: reached the device-coherent level).
__device__ __forceinline__ void wait_stores() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

template <typename T>
struct FBits;
template <>
struct FBits<double> {
    using U = unsigned long long;
    static constexpr double eps = 2.220446049250313e-16;
};
template <>
struct FBits<float> {
    using U = unsigned int;
    static constexpr float eps = 1.1920929e-07f;
};

// Non-negative IEEE values order like their bit patterns read as unsigned,
// so a max over |x| can be taken with an unsigned atomic max.
__device__ __forceinline__ unsigned long long ord_bits(double x) { return __double_as_longlong(x); }
__device__ __forceinline__ unsigned long long ord_bits(float x) { return (unsigned long long)__float_as_uint(x); }
__device__ __forceinline__ double from_ord(unsigned long long u, double) { return __longlong_as_double((long long)u); }
__device__ __forceinline__ float from_ord(unsigned long long u, float) { return __uint_as_float((unsigned)u); }

// Soft_tau(x) = sign(x) max(|x| - tau, 0); |x| == tau gives +0; NaN stays NaN.
template <typename T>
__device__ __forceinline__ T soft_threshold(T x, T tau)
{
    T a = fabs(x) - tau;
    if (a <= T(0))
        return T(0);
    return x > T(0) ? a : -a;
}

}  // namespace concord
