// Set-up and output kernels around the persistent sweep: input checks, the
// starting state of Algorithm 1 (Omega^(0), W = Omega^(0) S, the first
// published numerator entries) and the dense output with its summary
// (|E-hat|, the objective of eq. (1) on the S scale).
#include "device_common.hpp"
#include "schedule.hpp"
#include "support.hpp"
#include "sweep.hpp"

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

// Starting Omega in the sweep's layout: every workgroup's own copy of
// omega_{i, partner_r(i)} for its rows and all colours, and of omega_ii.
// omega0 == nullptr means the identity.  part == nullptr: Algorithm 1's
// schedule; else the mt-colour table part[r * p + i].
template <typename T>
__global__ void init_omega_kernel(const T *__restrict__ omega0, int p, int Gr, int Gc, int NR,
                                  const int *__restrict__ part, int mt, T *__restrict__ omp,
                                  T *__restrict__ omdp, int *__restrict__ err)
{
    const Circle C = Circle::make(p);
    const int G = Gr * Gc;
    const int M = part ? mt : C.m;
    const long long offd = (long long)G * M * NR;
    const long long total = offd + (long long)G * NR;
    int bad = 0;
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < total;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < offd) {
            const long long per = (long long)M * NR;
            const int g = (int)(e / per);
            const long long rem = e - (long long)g * per;
            const int r = (int)(rem / NR), k = (int)(rem - (long long)r * NR);
            const int i = g / Gc + k * Gr;
            T w = T(0);
            if (omega0 && i < p) {
                const int j = part ? part[(size_t)r * p + i] : C.partner(r, i);
                if (j >= 0) {
                    w = omega0[(size_t)i * p + j];
                    if (!finite_v(w))
                        bad |= kErrNonFinite;
                }
            }
            omp[e] = w;
        } else {
            const long long e2 = e - offd;
            const int g = (int)(e2 / NR), k = (int)(e2 - (long long)g * NR);
            const int i = g / Gc + k * Gr;
            T w = T(1);
            if (omega0 && i < p) {
                w = omega0[(size_t)i * p + i];
                if (!finite_v(w))
                    bad |= kErrNonFinite;
            }
            omdp[e2] = w;
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

// First published numerator entries: pc[0][colour 0][slot(i)] = W_{i, partner_0(i)};
// every other slot of pc and pd holds the sentinel, except pd[0] when the
// first colour is also the last (m = 1), which reads W_ii directly.  Slots
// are group-major: row i at (i mod Gr) * NR + i / Gr, PS = Gr * NR per colour.
template <typename T>
__global__ void init_publish_kernel(const T *__restrict__ W, int p, int Gr, int NR,
                                    const int *__restrict__ part, int mt, T *__restrict__ pc,
                                    T *__restrict__ pd)
{
    using U = typename Sentinel<T>::U;
    const Circle C = Circle::make(p);
    const int M = part ? mt : C.m;
    const long long PS = (long long)Gr * NR;
    const long long npc = 2ll * M * PS;
    U *pcu = reinterpret_cast<U *>(pc);
    U *pdu = reinterpret_cast<U *>(pd);
    for (long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x; e < npc + 2 * PS;
         e += (long long)gridDim.x * blockDim.x) {
        if (e < PS) {
            const int i = (int)(e % NR) * Gr + (int)(e / NR);
            const int j = (i < p) ? (part ? part[i] : C.partner(0, i)) : -1;
            pc[e] = (j >= 0) ? W[(size_t)i * p + j] : T(0);
        } else if (e < npc) {
            pcu[e] = Sentinel<T>::bits;
        } else {
            const long long d = e - npc;
            const int i = (int)(d % NR) * Gr + (int)(d / NR);
            if (d < PS && M == 1 && i < p)
                pd[d] = W[(size_t)i * p + i];
            else
                pdu[d] = Sentinel<T>::bits;
        }
    }
}

// Dense symmetric Omega from the sweep layout (the copies held by the
// workgroups of column slice 0), plus the summary: nonzeros above the
// diagonal and F(Omega) = -sum log omega_ii + 1/2 sum_ij W_ij omega_ij
// + lam sum_{i<j} |omega_ij| (tr(Omega S Omega) = sum_ij (Omega S)_ij omega_ij).
template <typename T>
__global__ void finalize_kernel(const T *__restrict__ omp, const T *__restrict__ omdp, int Gr,
                                int Gc, int NR, const T *__restrict__ W, int p, T lam,
                                T *__restrict__ omega, double *__restrict__ acc,
                                unsigned long long *__restrict__ nnz, int *__restrict__ err)
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
        const int lo = i < j ? i : j;
        const int g = (lo % Gr) * Gc, k = lo / Gr;
        T w;
        if (i == j) {
            w = omdp[(size_t)g * NR + k];
            part += -log((double)w);
        } else {
            const int r = C.colour(i, j);
            w = omp[((size_t)g * C.m + r) * NR + k];
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
hipError_t launch_init_omega(const T *omega0, int p, int Gr, int Gc, int NR, T *omp, T *omdp,
                             int *err, hipStream_t st, const int *part, int mt)
{
    const Circle C = Circle::make(p);
    const long long total = (long long)Gr * Gc * NR * ((part ? mt : C.m) + 1);
    hipLaunchKernelGGL(init_omega_kernel<T>, dim3(grid_for(total, 8192)), dim3(kThreads), 0, st,
                       omega0, p, Gr, Gc, NR, part, mt, omp, omdp, err);
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
hipError_t launch_init_publish(const T *W, int p, int Gr, int NR, T *pc, T *pd, hipStream_t st,
                               const int *part, int mt)
{
    const Circle C = Circle::make(p);
    const long long PS = (long long)Gr * NR;
    const int M = part ? mt : C.m;
    hipLaunchKernelGGL(init_publish_kernel<T>, dim3(grid_for(2ll * M * PS + 2 * PS, 8192)),
                       dim3(kThreads), 0, st, W, p, Gr, NR, part, mt, pc, pd);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_finalize(const T *omp, const T *omdp, int Gr, int Gc, int NR, const T *W, int p,
                           T lam, T *omega, double *acc, unsigned long long *nnz, int *err,
                           hipStream_t st)
{
    hipLaunchKernelGGL(finalize_kernel<T>, dim3(grid_for((long long)p * p, 2048)), dim3(kThreads),
                       0, st, omp, omdp, Gr, Gc, NR, W, p, lam, omega, acc, nnz, err);
    return hipGetLastError();
}

#define CONCORD_SUPPORT_INST(T)                                                                  \
    template hipError_t launch_check_copy<T>(const T *, int, T *, bool, T *, int *, hipStream_t); \
    template hipError_t launch_init_omega<T>(const T *, int, int, int, int, T *, T *, int *,     \
                                             hipStream_t, const int *, int);                     \
    template hipError_t launch_init_publish<T>(const T *, int, int, int, T *, T *, hipStream_t,  \
                                               const int *, int);                                \
    template hipError_t launch_finalize<T>(const T *, const T *, int, int, int, const T *, int, T, \
                                           T *, double *, unsigned long long *, int *, hipStream_t);

CONCORD_SUPPORT_INST(float)
CONCORD_SUPPORT_INST(double)

}  // namespace concord
