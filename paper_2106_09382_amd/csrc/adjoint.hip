// Set-up and output kernels of the implicit gradient (the adjoint system the
// sweep kernel solves in its adjoint mode).
//
// At Omega-hat the free entries are the diagonal and the pairs i < j with
// omega_ij != 0.  For a loss with gradient C = dL/dOmega-hat the right-hand
// side is g_ii = C_ii and g_ij = C_ij + C_ji (omega_ij and omega_ji are one
// unknown).  The solution v, laid out as the symmetric matrix V (0 off the
// free pairs), gives
//   dL/dS   = -(Omega V + V Omega) / 2     (the symmetric gradient)
//   dL/dlam = -sum_{i<j, free} v_ij sign(omega_ij),
// because the stationarity residuals R_ij = W_ij + W_ji + lam sign(omega_ij)
// and R_ii = W_ii - 1/omega_ii depend on S only through W = Omega S.
#include "device_common.hpp"
#include "schedule.hpp"
#include "support.hpp"

namespace concord {

namespace {

constexpr int kThreads = 256;

inline int grid_for(long long work, int cap = 4096)
{
    long long g = (work + kThreads - 1) / kThreads;
    if (g < 1)
        g = 1;
    return (int)(g > cap ? cap : g);
}

// Starting point v = 0 and the right-hand side in the sweep layout: for
// workgroup g = a * Gc + b and its k-th row i = a + k Gr, colour r pairs i
// with j = partner_r(i); adj_g holds g_ij there when the pair is free, else
// NaN (the sweep then leaves v_ij at 0).  Per row: g_ii and S_ii + 1/omega_ii^2.
template <typename T>
__global__ void init_adjoint_kernel(const T *__restrict__ om, const T *__restrict__ C,
                                    const T *__restrict__ sd, int p, int Gr, int Gc, int NR,
                                    T *__restrict__ vp, T *__restrict__ vdp, T *__restrict__ adj_g,
                                    T *__restrict__ adj_gd, T *__restrict__ adj_hd,
                                    int *__restrict__ err)
{
    const Circle Cc = Circle::make(p);
    const int G = Gr * Gc;
    const long long offd = (long long)G * Cc.m * NR;
    const long long total = offd + (long long)G * NR;
    const T qnan = __builtin_nan("");
    int bad = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < offd) {
            const long long per = (long long)Cc.m * NR;
            const int g = (int)(e / per);
            const long long rem = e - (long long)g * per;
            const int r = (int)(rem / NR), k = (int)(rem - (long long)r * NR);
            const int i = g / Gc + k * Gr;
            T rhs = qnan;
            if (i < p) {
                const int j = Cc.partner(r, i);
                if (j >= 0) {
                    const T w = om[(size_t)i * p + j];
                    const T c = C[(size_t)i * p + j] + C[(size_t)j * p + i];
                    if (!isfinite(w) || !isfinite(c))
                        bad |= kErrNonFinite;
                    if (w != T(0))
                        rhs = c;
                }
            }
            vp[e] = T(0);
            adj_g[e] = rhs;
        } else {
            const long long e2 = e - offd;
            const int g = (int)(e2 / NR), k = (int)(e2 - (long long)g * NR);
            const int i = g / Gc + k * Gr;
            T gd = T(0), hd = T(1);
            if (i < p) {
                const T w = om[(size_t)i * p + i];
                gd = C[(size_t)i * p + i];
                if (!isfinite(w) || !isfinite(gd))
                    bad |= kErrNonFinite;
                if (!(w > T(0)))
                    bad |= kErrNotPD;
                hd = sd[i] + T(1) / (w * w);
            }
            vdp[e2] = T(0);
            adj_gd[e2] = gd;
            adj_hd[e2] = hd;
        }
    }
    if (bad)
        atomicOr(err, bad);
}

template <typename T>
__global__ void fill_kernel(T *__restrict__ x, long long n, T v)
{
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < n;
         e += (long long)gridDim.x * blockDim.x)
        x[e] = v;
}

// Dense symmetric V from the sweep layout (the copies of column slice 0).
template <typename T>
__global__ void gather_kernel(const T *__restrict__ vp, const T *__restrict__ vdp, int Gr, int Gc,
                              int NR, int p, T *__restrict__ V)
{
    const Circle Cc = Circle::make(p);
    const long long total = (long long)p * p;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e - (long long)i * p);
        const int lo = i < j ? i : j;
        const int g = (lo % Gr) * Gc, k = lo / Gr;
        V[e] = (i == j) ? vdp[(size_t)g * NR + k]
                        : vp[((size_t)g * Cc.m + Cc.colour(i, j)) * NR + k];
    }
}

// grad_S = -(M + M^T) / 2 with M = Omega V; acc[0] += -sum_{i<j} V_ij sign(omega_ij).
template <typename T>
__global__ void adjoint_output_kernel(const T *__restrict__ M, const T *__restrict__ V,
                                      const T *__restrict__ om, int p, T *__restrict__ gS,
                                      double *__restrict__ acc, int *__restrict__ err)
{
    __shared__ double sred[kThreads / 64];
    const long long total = (long long)p * p;
    double part = 0.0;
    int bad = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e - (long long)i * p);
        const T gv = -(M[e] + M[(size_t)j * p + i]) * T(0.5);
        if (!isfinite(gv))
            bad |= kErrNonFinite;
        gS[e] = gv;
        if (i < j) {
            const T w = om[e];
            if (w != T(0))
                part -= (double)V[e] * (w > T(0) ? 1.0 : -1.0);
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        part += __shfl_xor(part, off, 64);
    if ((threadIdx.x & 63) == 0)
        sred[threadIdx.x >> 6] = part;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2)
            s += sred[w2];
        atomicAdd(acc, s);
    }
    if (bad)
        atomicOr(err, bad);
}

}  // namespace

template <typename T>
hipError_t launch_init_adjoint(const T *om, const T *C, const T *sd, int p, int Gr, int Gc, int NR,
                               T *vp, T *vdp, T *adj_g, T *adj_gd, T *adj_hd, int *err,
                               hipStream_t st)
{
    const Circle Cc = Circle::make(p);
    const long long total = (long long)Gr * Gc * NR * (Cc.m + 1);
    hipLaunchKernelGGL(init_adjoint_kernel<T>, dim3(grid_for(total, 8192)), dim3(kThreads), 0, st,
                       om, C, sd, p, Gr, Gc, NR, vp, vdp, adj_g, adj_gd, adj_hd, err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_fill(T *x, long long n, T v, hipStream_t st)
{
    hipLaunchKernelGGL(fill_kernel<T>, dim3(grid_for(n, 8192)), dim3(kThreads), 0, st, x, n, v);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(const T *vp, const T *vdp, int Gr, int Gc, int NR, int p, T *V,
                         hipStream_t st)
{
    hipLaunchKernelGGL(gather_kernel<T>, dim3(grid_for((long long)p * p, 4096)), dim3(kThreads), 0,
                       st, vp, vdp, Gr, Gc, NR, p, V);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_output(const T *M, const T *V, const T *om, int p, T *gS, double *acc,
                                 int *err, hipStream_t st)
{
    hipLaunchKernelGGL(adjoint_output_kernel<T>, dim3(grid_for((long long)p * p, 2048)),
                       dim3(kThreads), 0, st, M, V, om, p, gS, acc, err);
    return hipGetLastError();
}

#define CONCORD_ADJOINT_INST(T)                                                                  \
    template hipError_t launch_init_adjoint<T>(const T *, const T *, const T *, int, int, int,  \
                                               int, T *, T *, T *, T *, T *, int *,             \
                                               hipStream_t);                                     \
    template hipError_t launch_fill<T>(T *, long long, T, hipStream_t);                        \
    template hipError_t launch_gather<T>(const T *, const T *, int, int, int, int, T *,        \
                                         hipStream_t);                                           \
    template hipError_t launch_adjoint_output<T>(const T *, const T *, const T *, int, T *,    \
                                                 double *, int *, hipStream_t);

CONCORD_ADJOINT_INST(float)
CONCORD_ADJOINT_INST(double)

}  // namespace concord
