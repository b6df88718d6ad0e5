// Set-up and output kernels around the persistent sweep.
#pragma once

#include <hip/hip_runtime.h>

namespace concord {

// Bits of the device error word.
constexpr int kErrNonFinite = 1;  // NaN/Inf in an input or in the result
constexpr int kErrNotPD = 2;      // some S_ii <= 0

template <typename T>
hipError_t launch_check_copy(const T *S, int p, T *W, bool copy_w, T *sd, int *err,
                             hipStream_t st);
template <typename T>
hipError_t launch_init_omega(const T *omega0, int p, int Gr, int Gc, int NR, T *omp, T *omdp,
                             int *err, hipStream_t st);
hipError_t launch_clear(unsigned *flags, int nflags, unsigned long long *red, int nred, int *out,
                        int nout, double *acc, int nacc, hipStream_t st);
template <typename T>
hipError_t launch_init_publish(const T *W, int p, int Gr, int NR, T *pc, T *pd, hipStream_t st);
template <typename T>
hipError_t launch_finalize(const T *omp, const T *omdp, int Gr, int Gc, int NR, const T *W, int p,
                           T lam, T *omega, double *acc, unsigned long long *nnz, int *err,
                           hipStream_t st);

// Adjoint system of the implicit gradient (adjoint.hip).
template <typename T>
hipError_t launch_init_adjoint(const T *om, const T *C, const T *sd, int p, int Gr, int Gc, int NR,
                               T *vp, T *vdp, T *adj_g, T *adj_gd, T *adj_hd, int *err,
                               hipStream_t st);
template <typename T>
hipError_t launch_fill(T *x, long long n, T v, hipStream_t st);
template <typename T>
hipError_t launch_gather(const T *vp, const T *vdp, int Gr, int Gc, int NR, int p, T *V,
                         hipStream_t st);
template <typename T>
hipError_t launch_adjoint_output(const T *M, const T *V, const T *om, int p, T *gS, double *acc,
                                 int *err, hipStream_t st);

}  // namespace concord
