// Set-up and output kernels around the persistent sweep: input checks, the
// starting state of Algorithm 1 (Omega^(0), W = Omega^(0) S, the first
// published numerator entries) and the dense output with its summary
// (|E-hat|, the objective of eq. (1) on the S scale).
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

template <typename T>
__device__ __forceinline__ bool finite_v(T x)
{
    return isfinite(x);
}

}  // namespace

// Scan S: every entry finite, every diagonal entry positive; copy diag(S).
// With no warm start also W = S (Omega^(0) = I gives W = S).
template <typename T>
__global__ void check_copy_kernel(const T *__restrict__ S, int p, T *__restrict__ W, int copy_w,
                                  T *__restrict__ sd, int *__restrict__ err)
{
    const long long total = (long long)p * p;
    int bad = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const T v = S[e];
        if (!finite_v(v))
            bad |= kErrNonFinite;
        if (copy_w)
            W[e] = v;
        const int i = (int)(e / p);
        if (e == (long long)i * p + i) {
            sd[i] = v;
            if (!(v > T(0)))
                bad |= kErrNotPD;
        }
    }
    if (bad)
        atomicOr(err, bad);
}

// Starting Omega in the sweep's layout: colour-major off-diagonals and the
// diagonal.  omega0 == nullptr means the identity.
template <typename T>
__global__ void init_omega_kernel(const T *__restrict__ omega0, int p, T *__restrict__ omc,
                                  T *__restrict__ omd, int *__restrict__ err)
{
    const Circle C = Circle::make(p);
    const long long slots = (long long)C.m * C.H;
    int bad = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < slots + p;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < slots) {
            const int r = (int)(e / C.H), q = (int)(e - (long long)r * C.H);
            int u, v;
            C.pair(r, q, &u, &v);
            T w = T(0);
            if (omega0 && u < p && v < p) {
                w = omega0[(size_t)u * p + v];
                if (!finite_v(w))
                    bad |= kErrNonFinite;
            }
            omc[e] = w;
        } else {
            const int i = (int)(e - slots);
            T w = omega0 ? omega0[(size_t)i * p + i] : T(1);
            if (!finite_v(w))
                bad |= kErrNonFinite;
            omd[i] = w;
        }
    }
    if (bad)
        atomicOr(err, bad);
}

// Clears the per-solve counters: barrier flags, sweep reductions, status
// words and the summary accumulators.
__global__ void clear_kernel(unsigned *__restrict__ flags, int nflags,
                             unsigned long long *__restrict__ red, int nred, int *__restrict__ out,
                             int nout, double *__restrict__ acc, int nacc)
{
    int n = nflags > nred ? nflags : nred;
    n = n > nout ? n : nout;
    n = n > nacc ? n : nacc;
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n; e += gridDim.x * blockDim.x) {
        if (e < nflags)
            flags[e] = 0u;
        if (e < nred)
            red[e] = 0ull;
        if (e < nout)
            out[e] = 0;
        if (e < nacc)
            acc[e] = 0.0;
    }
}

// First published numerator entries: pub[i] = W_{i, partner_0(i)} for the
// first colour step and pubd[i] = W_ii (read before the last colour).
template <typename T>
__global__ void init_publish_kernel(const T *__restrict__ W, int p, T *__restrict__ pub,
                                    T *__restrict__ pubd)
{
    const Circle C = Circle::make(p);
    for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < p; e += gridDim.x * blockDim.x) {
        const int j = C.partner(0, e);
        pub[e] = (j >= 0) ? W[(size_t)e * p + j] : T(0);
        pub[p + e] = T(0);
        pubd[e] = W[(size_t)e * p + e];
        pubd[p + e] = T(0);
    }
}

// Dense symmetric Omega from the sweep layout, plus the summary: nonzeros
// above the diagonal and F(Omega) = -sum log omega_ii + 1/2 sum_ij W_ij omega_ij
// + lam sum_{i<j} |omega_ij| (tr(Omega S Omega) = sum_ij (Omega S)_ij omega_ij).
template <typename T>
__global__ void finalize_kernel(const T *__restrict__ omc, const T *__restrict__ omd,
                                const T *__restrict__ W, int p, T lam, T *__restrict__ omega,
                                double *__restrict__ acc, unsigned long long *__restrict__ nnz,
                                int *__restrict__ err)
{
    __shared__ double sred[kThreads / 64];
    __shared__ unsigned long long sn[kThreads / 64];
    const Circle C = Circle::make(p);
    const long long total = (long long)p * p;
    double part = 0.0;
    unsigned long long cnt = 0;
    int bad = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(e / p), j = (int)(e - (long long)i * p);
        T w;
        if (i == j) {
            w = omd[i];
            part += -log((double)w);
        } else {
            const int r = C.colour(i, j);
            w = omc[(size_t)r * C.H + C.slot(r, i)];
            if (i < j) {
                part += (double)lam * fabs((double)w);
                cnt += (w != T(0));
            }
        }
        if (!finite_v(w))
            bad |= kErrNonFinite;
        part += 0.5 * (double)W[e] * (double)w;
        omega[e] = w;
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
        for (int w2 = 0; w2 < (int)(blockDim.x >> 6); ++w2) {
            s += sred[w2];
            c += sn[w2];
        }
        atomicAdd(acc, s);
        atomicAdd(nnz, c);
    }
    if (bad)
        atomicOr(err, bad);
}

template <typename T>
hipError_t launch_check_copy(const T *S, int p, T *W, bool copy_w, T *sd, int *err,
                             hipStream_t st)
{
    hipLaunchKernelGGL(check_copy_kernel<T>, dim3(grid_for((long long)p * p)), dim3(kThreads), 0,
                       st, S, p, W, copy_w ? 1 : 0, sd, err);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_omega(const T *omega0, int p, T *omc, T *omd, int *err, hipStream_t st)
{
    const Circle C = Circle::make(p);
    hipLaunchKernelGGL(init_omega_kernel<T>, dim3(grid_for((long long)C.m * C.H + p)),
                       dim3(kThreads), 0, st, omega0, p, omc, omd, err);
    return hipGetLastError();
}

hipError_t launch_clear(unsigned *flags, int nflags, unsigned long long *red, int nred, int *out,
                        int nout, double *acc, int nacc, hipStream_t st)
{
    int n = nflags > nred ? nflags : nred;
    n = n > nout ? n : nout;
    n = n > nacc ? n : nacc;
    hipLaunchKernelGGL(clear_kernel, dim3(grid_for(n)), dim3(kThreads), 0, st, flags, nflags, red,
                       nred, out, nout, acc, nacc);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_init_publish(const T *W, int p, T *pub, T *pubd, hipStream_t st)
{
    hipLaunchKernelGGL(init_publish_kernel<T>, dim3(grid_for(p)), dim3(kThreads), 0, st, W, p, pub,
                       pubd);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const T *omc, const T *omd, const T *W, int p, T lam, T *omega,
                           double *acc, unsigned long long *nnz, int *err, hipStream_t st)
{
    hipLaunchKernelGGL(finalize_kernel<T>, dim3(grid_for((long long)p * p, 2048)), dim3(kThreads),
                       0, st, omc, omd, W, p, lam, omega, acc, nnz, err);
    return hipGetLastError();
}

#define CONCORD_SUPPORT_INST(T)                                                                  \
    template hipError_t launch_check_copy<T>(const T *, int, T *, bool, T *, int *, hipStream_t); \
    template hipError_t launch_init_omega<T>(const T *, int, T *, T *, int *, hipStream_t);      \
    template hipError_t launch_init_publish<T>(const T *, int, T *, T *, hipStream_t);          \
    template hipError_t launch_finalize<T>(const T *, const T *, const T *, int, T, T *,         \
                                           double *, unsigned long long *, int *, hipStream_t);

CONCORD_SUPPORT_INST(float)
CONCORD_SUPPORT_INST(double)

}  // namespace concord
