// Kernels and launchers of the persistent CONCORD-PCD sweep (the solve
// itself, shared with the joint two-population kernel, is in sweep_solve.hpp).
#include "sweep_solve.hpp"

namespace concord {

template <typename T>
size_t sweep_lds_bytes(const SweepParams<T> &P)
{
    const size_t nb = P.ovl ? 2 : 1;  // sets of pending lists
    size_t bytes = sizeof(T) * (nb * P.nr_max * P.depth + 16);
    if (P.w_lds)
        bytes += sizeof(T) * (size_t)P.nr_max * P.nc_max;
    bytes += sizeof(int) * (nb * P.nr_max * P.depth + nb * P.nr_max + 2 * (size_t)P.nr_max + 8);
    bytes += sizeof(unsigned) * 16;
    bytes += 8 + sizeof(double) * 16 + sizeof(unsigned long long) * 16;  // path summaries
    return bytes;
}

// BG: row rewrites right after each step (0) or in the background (1); the
// host picks the instantiation from P.ovl.
template <typename T, bool WLDS, int RPT, bool ADJ, bool TAB, int BG>
__global__ void __launch_bounds__(512) pcd_sweep_kernel(SweepParams<T> P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    pcd_solve<T, WLDS, RPT, 2, ADJ, TAB, false, BG>(P, blockIdx.x, gridDim.x, smem_raw);
}

// The same solve in workgroups of up to wide_threads<T>() threads (W in HBM,
// one row per thread); see wide_threads.
template <typename T, bool ADJ, bool TAB, int BG>
__global__ void __launch_bounds__(wide_threads<T>()) pcd_sweep_wide_kernel(SweepParams<T> P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    pcd_solve<T, false, 1, 2, ADJ, TAB, false, BG>(P, blockIdx.x, gridDim.x, smem_raw);
}

// Many independent problems in one launch: workgroup blockIdx.x serves
// problem wg_problem[blockIdx.x], as workgroup blockIdx.x - g0 of its Gr x Gc.
// W stays in HBM here (one code path keeps the register budget of the
// single-problem kernel; the problems of a batch are small enough for their
// W rows to stay in L2 and the last-level cache anyway).  A batch gives each
// problem few workgroups, so row rewrites are a large part of each colour
// step: by default they keep four columns per lane in flight (CPL) instead
// of two.  A problem's workgroups may also split its columns into slices
// (Gr x Gc per problem, from its descriptor).
// BG: 0 = every problem rewrites right after each step, 2 = each problem as
// its descriptor's ovl says.
template <typename T, int CPL, int BG>
__global__ void __launch_bounds__(512)
    pcd_batched_kernel(const SweepParams<T> *__restrict__ descs, const int *__restrict__ wg_problem)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SweepParams<T> P = descs[wg_problem[blockIdx.x]];
    const int g = (int)blockIdx.x - P.g0, G = P.Gr * P.Gc;
    pcd_solve<T, false, 2, CPL, false, false, false, BG>(P, g, G, smem_raw);
}

namespace {

// The schedule is a template argument: Algorithm 1's round robin computes
// partners in registers, a colouring table (forward solves only) loads them.
// Background rewrites exist only with W in HBM.
template <typename T, bool WLDS, bool ADJ, bool TAB>
const void *pick_kernel(int rpt, int ovl)
{
    if constexpr (!WLDS) {
        if (ovl)
            return rpt <= 1 ? (const void *)pcd_sweep_kernel<T, false, 1, ADJ, TAB, 1>
                            : (const void *)pcd_sweep_kernel<T, false, 2, ADJ, TAB, 1>;
    }
    if (rpt <= 1)
        return (const void *)pcd_sweep_kernel<T, WLDS, 1, ADJ, TAB, 0>;
    return (const void *)pcd_sweep_kernel<T, WLDS, 2, ADJ, TAB, 0>;
}

template <typename T, bool ADJ, bool TAB>
const void *pick_wide_kernel(int ovl)
{
    return ovl ? (const void *)pcd_sweep_wide_kernel<T, ADJ, TAB, 1>
               : (const void *)pcd_sweep_wide_kernel<T, ADJ, TAB, 0>;
}

}  // namespace

template <typename T>
hipError_t launch_sweep(const SweepParams<T> &P, int threads, hipStream_t stream)
{
    const size_t lds = sweep_lds_bytes(P);
    const int G = P.Gr * P.Gc;
    SweepParams<T> arg = P;
    void *args[] = {&arg};
    const void *fn;
    if (P.adj_g && P.part)
        return hipErrorInvalidValue;
    if (threads > 512) {
        if (P.w_lds || P.rpt > 1 || threads > wide_threads<T>())
            return hipErrorInvalidValue;
        fn = P.adj_g  ? pick_wide_kernel<T, true, false>(P.ovl)
             : P.part ? pick_wide_kernel<T, false, true>(P.ovl)
                      : pick_wide_kernel<T, false, false>(P.ovl);
    } else if (P.adj_g)
        fn = P.w_lds ? pick_kernel<T, true, true, false>(P.rpt, 0)
                     : pick_kernel<T, false, true, false>(P.rpt, P.ovl);
    else if (P.part)
        fn = P.w_lds ? pick_kernel<T, true, false, true>(P.rpt, 0)
                     : pick_kernel<T, false, false, true>(P.rpt, P.ovl);
    else
        fn = P.w_lds ? pick_kernel<T, true, false, false>(P.rpt, 0)
                     : pick_kernel<T, false, false, false>(P.rpt, P.ovl);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    if (G == 1)
        return hipLaunchKernel(fn, dim3(1), dim3(threads), args, lds, stream);
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(threads), args, (unsigned)lds, stream);
}

template <typename T>
hipError_t launch_sweep_batched(const SweepParams<T> *descs, const int *wg_problem, int G,
                                size_t lds, int threads, int cpl, bool any_bg, hipStream_t stream)
{
    if (cpl != 2 && cpl != 4)
        return hipErrorInvalidValue;
    const void *fn = (cpl == 2) ? (any_bg ? (const void *)pcd_batched_kernel<T, 2, 2>
                                          : (const void *)pcd_batched_kernel<T, 2, 0>)
                                : (any_bg ? (const void *)pcd_batched_kernel<T, 4, 2>
                                          : (const void *)pcd_batched_kernel<T, 4, 0>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    void *args[] = {&descs, &wg_problem};
    if (G == 1)
        return hipLaunchKernel(fn, dim3(1), dim3(threads), args, lds, stream);
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(threads), args, (unsigned)lds, stream);
}

template hipError_t launch_sweep_batched<float>(const SweepParams<float> *, const int *, int,
                                                size_t, int, int, bool, hipStream_t);
template hipError_t launch_sweep_batched<double>(const SweepParams<double> *, const int *, int,
                                                 size_t, int, int, bool, hipStream_t);
template size_t sweep_lds_bytes<float>(const SweepParams<float> &);
template size_t sweep_lds_bytes<double>(const SweepParams<double> &);
template hipError_t launch_sweep<float>(const SweepParams<float> &, int, hipStream_t);
template hipError_t launch_sweep<double>(const SweepParams<double> &, int, hipStream_t);

}  // namespace concord
