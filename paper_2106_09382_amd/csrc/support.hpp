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
// part == nullptr: Algorithm 1's schedule; else the mt-colour partner table.
template <typename T>
hipError_t launch_init_omega(const T *omega0, int p, int Gr, int Gc, int NR, T *omp, T *omdp,
                             int *err, hipStream_t st, const int *part = nullptr, int mt = 0);
hipError_t launch_clear(unsigned *flags, int nflags, unsigned long long *red, int nred, int *out,
                        int nout, double *acc, int nacc, hipStream_t st);
template <typename T>
hipError_t launch_init_publish(const T *W, int p, int Gr, int NR, T *pc, T *pd, hipStream_t st,
                               const int *part = nullptr, int mt = 0);
template <typename T>
hipError_t launch_finalize(const T *omp, const T *omdp, int Gr, int Gc, int NR, const T *W, int p,
                           T lam, T *omega, double *acc, unsigned long long *nnz, int *err,
                           hipStream_t st);

// Active-set sweeps (active.hip): the support of a dense Omega as an edge
// list (i < j, appended through an atomic counter, at most cap), and the
// dense Omega from the sweep layout of a colour table (omega zero-filled first).
template <typename T>
hipError_t launch_support_edges(const T *omega, int p, int *count, int *edges, long long cap,
                                hipStream_t st);
// The m x p partner table of a colouring of the edge list: part[c * p + v] =
// the partner of v in colour c, -1 where v has none; colour[e] is the colour
// of edge e = (edges[2 e], edges[2 e + 1]).
hipError_t launch_partner_table(const int *edges, const int *colour, int ne, int p, int m,
                                int *part, hipStream_t st);
template <typename T>
hipError_t launch_scatter_omega(const T *omp, const T *omdp, const int *part, int mt, int Gr,
                                int Gc, int NR, int p, T *omega, hipStream_t st);
// Algorithm 1's layout (omp, omdp) after sweeps over a colouring of the
// support: rewrite the ne listed pairs (edges[2 e], edges[2 e + 1]) and the
// diagonal from the dense omega, in every column slice's copy.
template <typename T>
hipError_t launch_refresh_layout(const T *omega, const int *edges, int ne, int p, int Gr, int Gc,
                                 int NR, T *omp, T *omdp, hipStream_t st);

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

// Joint estimation (joint.hip): over i <= j, acc += lam2 |omega^1_ij -
// omega^2_ij| and differ += [omega^1_ij != omega^2_ij] for i < j.
template <typename T>
hipError_t launch_joint_summary(const T *o1, const T *o2, int p, T lam2, double *acc,
                                unsigned long long *differ, hipStream_t st);

}  // namespace concord
