// Joint estimation of two precision matrices (Section 6 of arXiv 2106.09382):
// block coordinate descent over (omega^1_ij, omega^2_ij) on Algorithm 1's
// schedule.  Pairs of one colour share no vertex, so their blocks do not
// involve one another, exactly as single entries do in Lemma 2; the persistent
// sweep of sweep_solve.hpp runs both populations in one launch.
//
// Launch.  2 G workgroups: the first G solve population 0 (Gr x Gc as in a
// single solve), the next G population 1 with the same shape, so a row's
// published slot has the same index in both.  A workgroup keeps its own
// population's W block and pending row updates as in a single solve, plus a
// copy of the other population's omega for its rows.  In each colour step it
// polls the published numerator entries of both populations, evaluates the
// block update (population 1's operands first on both sides, so the two
// populations' workgroups compute the same bits) and applies its own
// population's change to its own W rows.  One grid barrier per sweep over all
// 2 G workgroups carries the convergence test on the change of both matrices.
#include "support.hpp"
#include "sweep_solve.hpp"

namespace concord {

// BG: row rewrites right after each step (0) or in the background (1).
template <typename T, bool WLDS, int RPT, int BG>
__global__ void __launch_bounds__(512) pcd_joint_kernel(SweepParams<T> P0, SweepParams<T> P1)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int G = (int)gridDim.x / 2;
    const int pop = (int)blockIdx.x >= G ? 1 : 0;
    // both joint kernels instantiate the same solve body for one row per
    // thread in HBM; inlined in each, as in every other kernel
    [[clang::always_inline]] pcd_solve<T, WLDS, RPT, 2, false, false, true, BG>(
        pop ? P1 : P0, (int)blockIdx.x - pop * G, G, smem_raw);
}

// The same in workgroups of up to kJointWideThreads threads, one row per
// thread, W in HBM: the waves beyond the rows rewrite in the background.  At
// 768 threads the kernel holds 168 VGPRs a wave and spills a few more in
// FP64, which measured cheaper than the five waves the 512-thread kernel
// leaves to the rewrites.
template <typename T, int BG>
__global__ void __launch_bounds__(kJointWideThreads)
    pcd_joint_wide_kernel(SweepParams<T> P0, SweepParams<T> P1)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const int G = (int)gridDim.x / 2;
    const int pop = (int)blockIdx.x >= G ? 1 : 0;
    [[clang::always_inline]] pcd_solve<T, false, 1, 2, false, false, true, BG>(
        pop ? P1 : P0, (int)blockIdx.x - pop * G, G, smem_raw);
}

template <typename T>
hipError_t launch_sweep_joint(const SweepParams<T> &P0, const SweepParams<T> &P1, int threads,
                              hipStream_t stream)
{
    if (P0.Gr != P1.Gr || P0.Gc != P1.Gc || P0.nr_max != P1.nr_max || P0.depth != P1.depth ||
        P0.w_lds != P1.w_lds || P0.rpt != P1.rpt || P0.p != P1.p || P0.pop != 0 || P1.pop != 1 ||
        P0.ovl != P1.ovl || (P0.ovl && P0.w_lds))
        return hipErrorInvalidValue;
    const size_t lds = sweep_lds_bytes(P0);
    const int G = P0.Gr * P0.Gc;
    SweepParams<T> a0 = P0, a1 = P1;
    void *args[] = {&a0, &a1};
    const void *fn;
    if (threads > 512) {
        if (P0.w_lds || P0.rpt > 1 || threads > kJointWideThreads)
            return hipErrorInvalidValue;
        fn = P0.ovl ? (const void *)pcd_joint_wide_kernel<T, 1>
                    : (const void *)pcd_joint_wide_kernel<T, 0>;
    } else if (P0.w_lds)
        fn = P0.rpt <= 1 ? (const void *)pcd_joint_kernel<T, true, 1, 0>
                         : (const void *)pcd_joint_kernel<T, true, 2, 0>;
    else if (P0.ovl)
        fn = P0.rpt <= 1 ? (const void *)pcd_joint_kernel<T, false, 1, 1>
                         : (const void *)pcd_joint_kernel<T, false, 2, 1>;
    else
        fn = P0.rpt <= 1 ? (const void *)pcd_joint_kernel<T, false, 1, 0>
                         : (const void *)pcd_joint_kernel<T, false, 2, 0>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    return hipLaunchCooperativeKernel(fn, dim3(2 * G), dim3(threads), args, (unsigned)lds, stream);
}

namespace {

constexpr int kSumThreads = 256;

// Over i <= j: acc += lam2 |omega^1_ij - omega^2_ij| (the fused term of the
// joint objective) and differ += [omega^1_ij != omega^2_ij] for i < j.
template <typename T>
__global__ void __launch_bounds__(kSumThreads)
    joint_summary_kernel(const T *__restrict__ o1, const T *__restrict__ o2, int p, T lam2,
                         double *__restrict__ acc, unsigned long long *__restrict__ differ)
{
    __shared__ double sred[kSumThreads / 64];
    __shared__ unsigned long long sn[kSumThreads / 64];
    const long long total = (long long)p * p;
    double part = 0.0;
    unsigned long long cnt = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e - (long long)i * p);
        if (j < i)
            continue;
        const T a = o1[e], b = o2[e];
        part += (double)lam2 * fabs((double)a - (double)b);
        cnt += (j > i && a != b) ? 1ull : 0ull;
    }
    for (int off = 32; off > 0; off >>= 1) {
        part += __shfl_xor(part, off, 64);
        cnt += __shfl_xor(cnt, off, 64);
    }
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        sred[wv] = part;
        sn[wv] = cnt;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        unsigned long long c = 0;
        for (int w = 0; w < kSumThreads / 64; ++w) {
            s += sred[w];
            c += sn[w];
        }
        atomicAdd(acc, s);
        atomicAdd(differ, c);
    }
}

}  // namespace

template <typename T>
hipError_t launch_joint_summary(const T *o1, const T *o2, int p, T lam2, double *acc,
                                unsigned long long *differ, hipStream_t st)
{
    const long long total = (long long)p * p;
    const int grid = (int)std::min<long long>(2048, (total + kSumThreads - 1) / kSumThreads);
    hipLaunchKernelGGL(joint_summary_kernel<T>, dim3(std::max(grid, 1)), dim3(kSumThreads), 0, st,
                       o1, o2, p, lam2, acc, differ);
    return hipGetLastError();
}

template hipError_t launch_sweep_joint<float>(const SweepParams<float> &,
                                              const SweepParams<float> &, int, hipStream_t);
template hipError_t launch_sweep_joint<double>(const SweepParams<double> &,
                                               const SweepParams<double> &, int, hipStream_t);
template hipError_t launch_joint_summary<float>(const float *, const float *, int, float,
                                                double *, unsigned long long *, hipStream_t);
template hipError_t launch_joint_summary<double>(const double *, const double *, int, double,
                                                 double *, unsigned long long *, hipStream_t);

}  // namespace concord
