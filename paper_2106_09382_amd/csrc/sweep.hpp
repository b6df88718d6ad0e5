// Shared host/device description of one persistent CONCORD-PCD solve.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace concord {

// Workspace of one solve (all device pointers).  The layout in HBM:
//   S     p x p row-major (read-only during the sweeps)
//   W     p x p row-major, the maintained product W = Omega S; workgroup (a, b)
//         owns rows i = a (mod Gr) restricted to column slice b
//   omc   colour-major off-diagonals: omc[r * H + q] = omega of slot q of colour r
//   omd   diagonal, p
//   sd    diag(S), p
//   pub   2 x p: pub[(s & 1) * p + i] = W_{i, partner_r(i)} for global step s
//   pubd  2 x p: pubd[(t & 1) * p + i] = W_ii just before the last colour of sweep t
//   flags one arrival word per workgroup (barrier epochs)
//   red   per sweep t, 4 words: [4t] max |change| (bits), [4t+1] max omega_ii (bits),
//         [4t+2] pairs that changed, [4t+3] diagonals that changed
//   out   [0] sweeps, [1] converged, [2] device wait failed, [3] abort flag,
//         [4] input error bits from the set-up kernels
template <typename T>
struct SweepParams {
    const T *S;
    const T *sd;
    T *W;
    T *omc;
    T *omd;
    T *pub;
    T *pubd;
    unsigned *flags;
    unsigned long long *red;
    int *out;
    int p;
    int Gr, Gc;        // row groups x column slices = workgroups
    int maxit;
    int w_lds;         // W block resident in LDS
    int nr_max;        // max rows per workgroup = ceil(p / Gr)
    int nc_max;        // max columns per workgroup
    T lam;
    T tol;
    T tol_coef;        // tol_eff = max(tol, tol_coef * max_i omega_ii)
    long long spin_limit;
};

// Column slice b of Gc over p columns: [slice_lo(b), slice_lo(b + 1)).
__host__ __device__ inline int slice_lo(int b, int Gc, int p) { return (int)(((long long)b * p) / Gc); }

template <typename T>
size_t sweep_lds_bytes(const SweepParams<T> &P, int threads);

template <typename T>
hipError_t launch_sweep(const SweepParams<T> &P, int threads, hipStream_t stream);

}  // namespace concord
