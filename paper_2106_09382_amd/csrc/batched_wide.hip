// The batched persistent sweep in wide workgroups: up to wide_threads<T>()
// threads, one row of W per thread.  With two rows per thread a batch's
// problems, each served by few workgroups, fill most waves with rows; with
// one row per thread in wider workgroups their rows fill at most half of the
// waves in more problems, and the other waves rewrite rows in the background
// (the same solve body, the same bits).
#include "sweep_solve.hpp"

namespace concord {

template <typename T, int CPL, int BG>
__global__ void __launch_bounds__(wide_threads<T>())
    pcd_batched_wide_kernel(const SweepParams<T> *__restrict__ descs,
                            const int *__restrict__ wg_problem)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SweepParams<T> P = descs[wg_problem[blockIdx.x]];
    const int g = (int)blockIdx.x - P.g0, G = P.Gr * P.Gc;
    pcd_solve<T, false, 1, CPL, false, false, false, BG>(P, g, G, smem_raw);
}

template <typename T>
hipError_t launch_sweep_batched_wide(const SweepParams<T> *descs, const int *wg_problem, int G,
                                     size_t lds, int threads, int cpl, bool any_bg,
                                     hipStream_t stream)
{
    if ((cpl != 2 && cpl != 4) || threads <= 512 || threads > wide_threads<T>())
        return hipErrorInvalidValue;
    const void *fn = (cpl == 2) ? (any_bg ? (const void *)pcd_batched_wide_kernel<T, 2, 2>
                                          : (const void *)pcd_batched_wide_kernel<T, 2, 0>)
                                : (any_bg ? (const void *)pcd_batched_wide_kernel<T, 4, 2>
                                          : (const void *)pcd_batched_wide_kernel<T, 4, 0>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    void *args[] = {&descs, &wg_problem};
    if (G == 1)
        return hipLaunchKernel(fn, dim3(1), dim3(threads), args, lds, stream);
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(threads), args, (unsigned)lds, stream);
}

template hipError_t launch_sweep_batched_wide<float>(const SweepParams<float> *, const int *, int,
                                                     size_t, int, int, bool, hipStream_t);
template hipError_t launch_sweep_batched_wide<double>(const SweepParams<double> *, const int *,
                                                      int, size_t, int, int, bool, hipStream_t);

}  // namespace concord
