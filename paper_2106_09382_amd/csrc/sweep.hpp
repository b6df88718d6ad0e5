// Shared host/device description of one persistent CONCORD-PCD solve.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace concord {

// Workspace of one solve (all device pointers).  The layout in HBM:
//   S     p x p row-major (read-only during the sweeps)
//   W     p x p row-major, the maintained product W = Omega S; workgroup
//         g = a * Gc + b owns rows i = a (mod Gr) restricted to column slice b
//   omp   per-workgroup copies of omega: omp[(g * m + r) * nr_max + k] is
//         omega_{i, partner_r(i)} for the workgroup's k-th row i = a + k Gr
//   omdp  per-workgroup diagonals: omdp[g * nr_max + k] = omega_ii
//   sd    diag(S), p
//   pc    published numerator entries, two sweep-parity buffers of m colours
//         of PS = Gr * nr_max slots, row i at slot (i mod Gr) * nr_max + i / Gr
//         (a row group's slots are contiguous, and so, up to one wrap, are the
//         slots of its partners in any colour):
//         pc[(buf * m + r) * PS + slot(i)] = W_{i, partner_r(i)} as colour r reads it
//   pd    pd[buf * PS + slot(i)] = W_ii as the last colour reads it
//   flags one sweep-barrier word per workgroup (epochs)
//   red   per sweep t, 4 words: [4t] max |change| (bits), [4t+1] max omega_ii (bits),
//         [4t+2] pairs that changed, [4t+3] diagonals that changed
//   out   [0] sweeps, [1] converged, [2] a device wait failed, [3] abort flag,
//         [4] input error bits from the set-up kernels
// Entries of pc (colours >= 1) and pd are reset to a signalling-NaN sentinel
// one sweep before they are written; a reader polls until the sentinel is gone.
// Summary of one lambda of a path, written by the sweep kernel: the sweep
// count at which the lambda finished (counted from the start of the path),
// whether its convergence test passed, nonzeros above the diagonal, the
// objective of the Omega it left, and when it started and ended.
struct PathRec {
    unsigned long long nnz_upper;
    double objective;
    int t_end;
    int converged;
    unsigned long long clock_start, clock_end;  // device clock (100 MHz) around the lambda
};

template <typename T>
struct SweepParams {
    const T *S;
    const T *sd;
    T *W;
    T *omp;
    T *omdp;
    T *pc;
    T *pd;
    unsigned *flags;
    unsigned long long *red;
    int *out;
    int p;
    int Gr, Gc;        // row groups x column slices = workgroups
    int maxit;
    int w_lds;         // W block resident in LDS
    int nr_max;        // max rows per workgroup = ceil(p / Gr)
    int nc_max;        // max columns per workgroup
    int depth;         // pending row updates held before a row is flushed (>= 2)
    int rpt;           // rows per thread (1, 2 or 4)
    int ovl;           // row rewrites run on the waves without rows, during the next
                       // step, from a second set of pending lists (set_overlap)
    T lam;
    T tol;
    T tol_coef;        // tol_eff = max(tol, tol_coef * max_i omega_ii)
    long long spin_limit;
    unsigned long long *tstamp;  // optional: [G][tstamp_steps][3] device timestamps
    int tstamp_steps;
    // Lambda path (batched solves): L values lams[0..L-1] run one after the
    // other, each warm-started from the previous; red then holds L * maxit
    // sweeps.  omega_out[l] (device pointers) receives the dense Omega of
    // lambda l and rec[l] its summary.  L = 1 with lams, omega_out and rec
    // null is a single solve at lam.
    int L;
    const double *lams;
    T *const *omega_out;
    PathRec *rec;
    int g0;  // first workgroup of this problem in a batched launch
    // Schedule: null for Algorithm 1's round robin (closed form); else an
    // m_tab x p table, part[r * p + i] = partner of i in colour r (-1 idle),
    // every colour a matching and m_tab >= 2 (single solves only).
    const int *part;
    int m_tab;
    // Adjoint system of the implicit gradient (null for a solve): adj_g in
    // omp's layout holds g_ij of the free pairs (NaN elsewhere); adj_gd and
    // adj_hd, one per row like omdp, hold g_ii and S_ii + 1 / omega_ii^2.
    const T *adj_g;
    const T *adj_gd;
    const T *adj_hd;
    // Joint estimation of two populations (Section 6; null/0 otherwise): this
    // solve is population `pop` of two run in one launch with the same shape,
    // sharing flags, red and out.  jo_S, jo_sd, jo_pc and jo_pd are the other
    // population's S, diag(S) and published entries; jo_omp and jo_omdp hold
    // this population's workgroups' copies of the other omega (laid out like
    // omp and omdp); lam2 weighs the fused penalty.
    const T *jo_S;
    const T *jo_sd;
    const T *jo_pc;
    const T *jo_pd;
    T *jo_omp;
    T *jo_omdp;
    T lam2;
    int pop;
};

// Column slice b of Gc over p columns: [slice_lo(b), slice_lo(b + 1)).
__host__ __device__ inline int slice_lo(int b, int Gc, int p) { return (int)(((long long)b * p) / Gc); }

// Sentinel bit patterns (signalling NaNs: arithmetic never produces them).
template <typename T>
struct Sentinel;
template <>
struct Sentinel<double> {
    using U = unsigned long long;
    static constexpr U bits = 0x7FF4DEAD0000BEEFull;
};
template <>
struct Sentinel<float> {
    using U = unsigned int;
    static constexpr U bits = 0x7FA0BEEFu;
};

template <typename T>
size_t sweep_lds_bytes(const SweepParams<T> &P);

// Background row rewrites (P.ovl) need W in HBM, waves that hold no rows
// (rows are dealt to threads in order, so waves past ceil(nr_max / 64) hold
// none), room in LDS for the second set of pending lists, and lists of at
// least 4 entries.  A row takes at most two updates per step (its pair and,
// after the last colour, its diagonal), so with depth >= 4 a row that went
// on in its other set is not listed again in the very next step, while the
// background rewrite of its first set is still running.  The rows must also
// fill at most half of the waves: fewer rewrite waves than row waves fall
// behind the rewrites a step lists (measured on the two-population solve at
// 313 rows per workgroup: 917 ms in the background against 772 ms after
// each step).
template <typename T>
inline void set_overlap(SweepParams<T> &P, int threads, size_t lds_cap)
{
    P.ovl = 0;
    if (P.w_lds || P.depth < 4 || 2 * ((P.nr_max + 63) / 64) > threads / 64)
        return;
    P.ovl = 1;
    if (sweep_lds_bytes(P) > lds_cap)
        P.ovl = 0;
}

// Widest workgroup of the single-problem sweep kernel (W in HBM, one row per
// thread): the waves beyond the rows' rewrite rows in the background, and
// more of them finish a burst of rewrites sooner.  The width is the largest
// whose register budget holds the kernel with at most a few spilled words:
// 1024 threads leave 128 VGPRs a wave (FP32 needs about that), 768 leave 168
// (FP64).  Workgroups of at most 512 threads use the 512-thread kernel.
template <typename T>
constexpr int wide_threads()
{
    return sizeof(T) == 4 ? 1024 : 768;
}

// Widest workgroup of the joint (two-population) kernel, in both precisions:
// its row state is larger, and 768 threads (168 VGPRs a wave) is the widest
// at which it spills little.
constexpr int kJointWideThreads = 768;

// threads > 512 launches the wide kernel, which needs W in HBM, one row per
// thread and threads <= wide_threads<T>().
template <typename T>
hipError_t launch_sweep(const SweepParams<T> &P, int threads, hipStream_t stream);

// One cooperative launch over G workgroups serving several problems:
// descs (device) holds one SweepParams per problem, wg_problem (device, G
// entries) the problem of each workgroup; lds = the largest sweep_lds_bytes;
// cpl = columns per lane in row rewrites (2 or 4); any_bg = some problem's
// descriptor asks for background rewrites.
template <typename T>
hipError_t launch_sweep_batched(const SweepParams<T> *descs, const int *wg_problem, int G,
                                size_t lds, int threads, int cpl, bool any_bg, hipStream_t stream);

// The same over workgroups of 513..wide_threads<T>() threads, one row per
// thread (every descriptor's rpt is 1).
template <typename T>
hipError_t launch_sweep_batched_wide(const SweepParams<T> *descs, const int *wg_problem, int G,
                                     size_t lds, int threads, int cpl, bool any_bg,
                                     hipStream_t stream);

// Joint estimation: one cooperative launch of 2 G workgroups, population 0 on
// the first G (P0) and population 1 on the rest (P1); G = Gr * Gc of both.
template <typename T>
hipError_t launch_sweep_joint(const SweepParams<T> &P0, const SweepParams<T> &P1, int threads,
                              hipStream_t stream);

}  // namespace concord
