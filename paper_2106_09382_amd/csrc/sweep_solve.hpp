// Persistent CONCORD-PCD sweep kernel (Algorithm 1 of arXiv 2106.09382) for gfx950.
//
// Method.  For a pair (i, j) of colour r, eq. (3)'s numerator is
//   b_ij = sum_{u != j} omega_iu S_ju + sum_{u != i} omega_uj S_iu
//        = W_ij + W_ji - (S_ii + S_jj) omega_ij,           W = Omega S,
// because Omega and S are symmetric ((S Omega)_ij = W_ji).  Changing
// omega_ij = omega_ji by d changes only rows i and j of W: W_i. += d S_j. and
// W_j. += d S_i..  For the diagonal step, eq. (2)'s sum is
// c_i = W_ii - S_ii omega_ii, and changing omega_ii by d gives W_i. += d S_i..
// So each pair costs O(1) to evaluate plus a row update when it moves,
// instead of two length-p sums.
//
// Work split.  Workgroup g = a * Gc + b owns rows i = a (mod Gr) of W
// restricted to column slice b (in LDS when the block fits, else in HBM where
// only this workgroup touches it).  It keeps its own copy of omega for those
// rows (every workgroup of a row group computes the same changes from the
// same bits, so the copies stay identical).
//
// Synchronisation.  Colour r of a sweep needs, for pair (i, j), the entries
// W_ij and W_ji as they stand after colour r - 1.  The workgroup owning
// (row i, column j) publishes W_ij into a slot of `pc` as soon as its colour
// r - 1 change is known; the readers poll that slot until the sentinel is
// gone.  So colours are ordered by point-to-point waits, not by grid
// barriers; one grid barrier per sweep carries the convergence test.  The
// diagonal step is folded into the last colour: W_ii is published one colour
// early (slot `pd`) and every workgroup of the row group finishes c_i itself.
//
// Deferred row updates.  A change of row i only has to reach W_ik by the time
// W_ik is next published.  Each row keeps a list of pending (source row,
// change) updates; a published entry is the stored W_ik with the pending
// updates applied on the fly (same fused multiply-adds, same order), and the
// whole row segment is rewritten only when the list fills.  The results are
// bit-identical to applying every update at once; HBM traffic for W drops by
// the list depth.
//
// Convergence.  Each entry of Omega changes exactly once per sweep, so
// |Omega^(t) - Omega^(t-1)|_inf is the max |change| over the sweep; it is
// reduced with one atomic max per workgroup, and read by every workgroup
// after the sweep's grid barrier, so all agree on when to stop.
#pragma once

#include "device_common.hpp"
#include "schedule.hpp"
#include "sweep.hpp"

namespace concord {

// Everything here has internal linkage: every kernel file that includes
// this header gets its own instantiations.
namespace {

constexpr int kMaxDepth = 8;  // longest pending list (registers hold one S value per entry)

// Sweep barrier: workgroup g stores the epoch into flags[g]; wave 0 of every
// workgroup polls all flags.  Bounded: after spin_limit polls (or when any
// workgroup has raised the abort word) it gives up and reports failure.
template <typename T>
__device__ bool sweep_barrier(const SweepParams<T> &P, unsigned epoch, int *s_fail, int g, int G)
{
    wait_stores();
    __syncthreads();
    if (G > 1) {
        if (threadIdx.x == 0)
            st_dev(&P.flags[g], epoch);
        if (threadIdx.x < 64) {
            long long spins = 0;
            for (;;) {
                int ok = 1;
                for (int g = threadIdx.x; g < G; g += 64)
                    ok &= (ld_dev(&P.flags[g]) >= epoch) ? 1 : 0;
                if (__all(ok))
                    break;
                if (++spins > P.spin_limit || ld_dev(&P.out[3]) != 0) {
                    if (threadIdx.x == 0) {
                        st_dev(&P.out[3], 1);
                        *s_fail = 1;
                    }
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
        }
        __syncthreads();
    }
    return *s_fail == 0;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T *scratch)
{
    for (int off = 32; off > 0; off >>= 1) {
        T o = __shfl_xor(v, off, 64);
        v = (o > v || o != o) ? o : v;
    }
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
        scratch[wv] = v;
    __syncthreads();
    T r = scratch[0];
    for (int w = 1; w < nw; ++w)
        r = (scratch[w] > r || scratch[w] != scratch[w]) ? scratch[w] : r;
    __syncthreads();
    return r;
}

__device__ __forceinline__ unsigned block_sum(unsigned v, unsigned *scratch)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0)
        scratch[wv] = v;
    __syncthreads();
    unsigned r = 0;
    for (int w = 0; w < nw; ++w)
        r += scratch[w];
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ T as_value(typename Sentinel<T>::U u)
{
    T v;
    __builtin_memcpy(&v, &u, sizeof(T));
    return v;
}

// Block minimisers of the joint two-population objective (Section 6).  For a
// pair (i, j) the objective in (x_1, x_2) = (omega^1_ij, omega^2_ij) is
//   sum_m [a_m x_m^2 / 2 + b_m x_m + lam1 |x_m|] + lam2 |x_1 - x_2|,
// a_m = S^m_ii + S^m_jj and b_m the eq. (3) numerator of population m.  It is
// strictly convex; where its minimiser has x_1 > x_2 the fused term's
// subgradient is +lam2 and the coordinates separate, and a separated pair
// that keeps x_1 > x_2 is optimal.  So: try x_1 > x_2 (lam2 added to b_1,
// taken from b_2), then x_1 < x_2, else the fused value on the line x_1 = x_2.
// Both populations' workgroups evaluate this from the same bits in the same
// order, so they agree on both new values.
template <typename T>
__device__ __forceinline__ void joint_pair(T a1, T b1, T a2, T b2, T lam1, T lam2, T &x1, T &x2)
{
    const T u1 = soft_threshold(-(b1 + lam2), lam1) / a1;
    const T u2 = soft_threshold(-(b2 - lam2), lam1) / a2;
    if (u1 > u2) {
        x1 = u1;
        x2 = u2;
        return;
    }
    const T v1 = soft_threshold(-(b1 - lam2), lam1) / a1;
    const T v2 = soft_threshold(-(b2 + lam2), lam1) / a2;
    if (v1 < v2) {
        x1 = v1;
        x2 = v2;
        return;
    }
    x1 = x2 = soft_threshold(-(b1 + b2), T(2) * lam1) / (a1 + a2);
}

// Positive root of s y^2 + c y - k = 0 (k > 0); for c >= 0 written as
// 2k / (c + disc), the same root without cancellation.
template <typename T>
__device__ __forceinline__ T pos_root(T s, T c, T k)
{
    const T disc = sqrt(fma(c, c, T(4) * k * s));
    return (c >= T(0)) ? T(2) * k / (c + disc) : (disc - c) / (T(2) * s);
}

// The diagonal block (omega^1_ii, omega^2_ii): smooth part
// -log y_m + S^m_ii y_m^2 / 2 + c_m y_m (c_m the eq. (2) sum) plus
// lam2 |y_1 - y_2|, same case order as joint_pair; the fused value is the
// positive root of (S^1_ii + S^2_ii) t^2 + (c_1 + c_2) t - 2 = 0.
template <typename T>
__device__ __forceinline__ void joint_diag(T s1, T c1, T s2, T c2, T lam2, T &y1, T &y2)
{
    const T u1 = pos_root(s1, c1 + lam2, T(1)), u2 = pos_root(s2, c2 - lam2, T(1));
    if (u1 > u2) {
        y1 = u1;
        y2 = u2;
        return;
    }
    const T v1 = pos_root(s1, c1 - lam2, T(1)), v2 = pos_root(s2, c2 + lam2, T(1));
    if (v1 < v2) {
        y1 = v1;
        y2 = v2;
        return;
    }
    y1 = y2 = pos_root(s1 + s2, c1 + c2, T(2));
}

// Rewrites the segments of the listed rows with their pending updates:
// W_ic <- fma(d_e, S_{src_e, c}, ...) in list order, for c in the slice.
// An entry 2 k + s names row k and its set s of pending lists (the lists of
// set s start at pj + s * LB, pdl + s * LB and np + s * NR).  Work is cut into
// (row, 64 * CPL column chunk) units dealt out to waves wv0 and up; each lane
// handles CPL columns 64 apart (every load is one coalesced row segment), so
// CPL * (n + 1) loads are in flight per lane.
template <typename T, bool WLDS, int CPL>
__device__ void flush_rows(const int *rows, int nrows, const int *pj, const T *pdl,
                           const int *np, int LB, int NR, int D, int a, int Gr, int p, int c0,
                           int nc, const T *__restrict__ S, T *__restrict__ Wg, T *wblk,
                           int wv0 = 0)
{
    constexpr int CW = 64 * CPL;
    const int lane = threadIdx.x & 63, wv = (threadIdx.x >> 6) - wv0;
    const int nw = (blockDim.x >> 6) - wv0;
    const int chunks = (nc + CW - 1) / CW;
    const int units = nrows * chunks;
    for (int u = wv; u < units; u += nw) {
        const int fr = u / chunks, ch = u - fr * chunks;
        const int ks = rows[fr];
        const int k = ks >> 1, set = ks & 1;
        const int i = a + k * Gr;
        const int n = np[set * NR + k];
        const int *pjs = pj + (size_t)set * LB + (size_t)k * D;
        const T *pdls = pdl + (size_t)set * LB + (size_t)k * D;
        const int cl = ch * CW + lane;
        T sv[kMaxDepth][CPL];
#pragma unroll
        for (int e = 0; e < kMaxDepth; ++e) {
            if (e < n) {
                const T *row = S + (size_t)pjs[e] * p + c0;
#pragma unroll
                for (int q = 0; q < CPL; ++q)
                    sv[e][q] = (cl + 64 * q < nc) ? row[cl + 64 * q] : T(0);
            }
        }
        T *wr = WLDS ? &wblk[(size_t)k * nc] : &Wg[(size_t)i * p + c0];
        T v[CPL];
#pragma unroll
        for (int q = 0; q < CPL; ++q)
            v[q] = (cl + 64 * q < nc) ? wr[cl + 64 * q] : T(0);
#pragma unroll
        for (int e = 0; e < kMaxDepth; ++e) {
            if (e < n) {
                const T d = pdls[e];
#pragma unroll
                for (int q = 0; q < CPL; ++q)
                    v[q] = fma(d, sv[e][q], v[q]);
            }
        }
        // Every load of this unit has been consumed (so this wait costs
        // nothing); stating it lets the compiler's wait analysis see that no
        // load of the rewrite is still in flight after it, on any path.
        // Otherwise the first LDS read after the step's barrier waits for
        // every load in flight, including the next step's prefetched
        // operands.  (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their
        // maxima.)
        __builtin_amdgcn_s_waitcnt(0x0F70);
#pragma unroll
        for (int q = 0; q < CPL; ++q)
            if (cl + 64 * q < nc)
                wr[cl + 64 * q] = v[q];
    }
}

// Operands of one row's next colour step that do not depend on that step's
// change, loaded one step ahead so that their latency overlaps the previous
// step's synchronisation and row rewrites.
// Joint mode: the other population's omega_ij, omega_ii and S_ji (an empty
// base otherwise, so single solves keep their register layout).
template <typename T, bool JNT>
struct RowJoint {
    T wo, odo, s_jio;
    T sdo_lo, sdo_hi, sio;  // the other population's S_ii, S_jj and (last colour) S_ii
};
template <typename T>
struct RowJoint<T, false> {
};

template <typename T, bool JNT>
struct RowNext : RowJoint<T, JNT> {
    int j;        // partner in the step (-1: idle)
    int kn;       // column published by the step (-1: none in this slice)
    int n;        // pending entries the published values fold in ...
    int set;      // ... taken from this set of pending lists
    bool last;    // the step is the last colour (diagonal step follows)
    bool pubd;    // the step publishes W_ii for the following last colour
    T w, od, s_ji, s_jn, s_in;
    T wb;         // stored W_{i,kn}
    T wd;         // stored W_ii, when the step publishes it
    T sd_lo, sd_hi;  // S_ll and S_hh of the pair (l < h), whose sum is eq. (3)'s denominator
    T sii;        // S_ii, for the diagonal step after the last colour
    T g;          // adjoint mode: right-hand side of the pair (NaN: pair not free)
    T sv[kMaxDepth];
};

// `pj` is the start of the set of pending lists `set`, whose first n entries
// of row k the step's published values fold in.  With loadw false the stored
// W entries are not read here (a rewrite of the row may be running): the step
// reads them itself, after the barrier that ends the rewrite.
template <typename T, bool WLDS, bool TAB, bool JNT>
__device__ __forceinline__ void load_next(RowNext<T, JNT> &x, const Circle &C, const int *part, int mt,
                                          int r1, int i, int k, int n, int set, bool loadw,
                                          const int *pj, int D, int NR, int p, int c0,
                                          int c1, int nc, const T *__restrict__ S,
                                          const T *__restrict__ Wg, const T *wblk,
                                          const T *__restrict__ omp, const T *__restrict__ omdp,
                                          const T *__restrict__ adjg, const T *omp_o,
                                          const T *omdp_o, const T *So,
                                          const T *__restrict__ sd, const T *sdo)
{
    // the schedule: Algorithm 1's round robin, or a given colouring's table
    const int m = TAB ? mt : C.m;
    const int rn1 = (r1 + 1 == m) ? 0 : r1 + 1;
    int kn;
    if constexpr (TAB) {
        x.j = part[(size_t)r1 * p + i];
        kn = part[(size_t)rn1 * p + i];
    } else {
        x.j = C.partner(r1, i);
        kn = C.partner(rn1, i);
    }
    x.kn = (kn >= c0 && kn < c1) ? kn : -1;
    x.last = (r1 == m - 1);
    x.pubd = (rn1 == m - 1) && i >= c0 && i < c1;
    x.n = n;
    x.set = set;
    x.w = (x.j >= 0) ? omp[(size_t)r1 * NR + k] : T(0);
    x.g = (adjg && x.j >= 0) ? adjg[(size_t)r1 * NR + k] : T(0);
    x.od = x.last ? omdp[k] : T(0);
    x.s_ji = (x.j >= 0 && (x.last || x.pubd)) ? S[(size_t)x.j * p + i] : T(0);
    // the diagonal of S for the step's denominators: loaded here, summed after
    // the poll (a sum here would wait for these loads at the end of this step)
    const int lo = (x.j >= 0 && x.j < i) ? x.j : i, hi = (x.j >= 0 && x.j < i) ? i : x.j;
    x.sd_lo = (x.j >= 0) ? sd[lo] : T(0);
    x.sd_hi = (x.j >= 0) ? sd[hi] : T(0);
    x.sii = x.last ? sd[i] : T(0);
    if constexpr (JNT) {
        x.wo = (x.j >= 0) ? omp_o[(size_t)r1 * NR + k] : T(0);
        x.odo = x.last ? omdp_o[k] : T(0);
        x.s_jio = (x.j >= 0 && x.last) ? So[(size_t)x.j * p + i] : T(0);
        x.sdo_lo = (x.j >= 0) ? sdo[lo] : T(0);
        x.sdo_hi = (x.j >= 0) ? sdo[hi] : T(0);
        x.sio = x.last ? sdo[i] : T(0);
    }
    x.wd = (x.pubd && loadw) ? (WLDS ? wblk[(size_t)k * nc + (i - c0)] : Wg[(size_t)i * p + i])
                             : T(0);
    if (x.kn >= 0) {
        x.wb = loadw ? (WLDS ? wblk[(size_t)k * nc + (x.kn - c0)] : Wg[(size_t)i * p + x.kn])
                     : T(0);
#pragma unroll
        for (int e = 0; e < kMaxDepth; ++e)
            if (e < n)
                x.sv[e] = S[(size_t)pj[k * D + e] * p + x.kn];
        x.s_jn = (x.j >= 0) ? S[(size_t)x.j * p + x.kn] : T(0);
        x.s_in = x.last ? S[(size_t)i * p + x.kn] : T(0);
    }
}


// Applies every pending row update to the stored W block, in list order:
// first the rewrite still owed for the last step's rows (when rewrites run
// in the background, `owed` lists nf_owed of them), then each row's current
// set of lists.  `spare` is an flist half that no rewrite is reading.
// Afterwards every list is empty.
template <typename T, bool WLDS, int RPT, int CPL>
__device__ void flush_all(const SweepParams<T> &P, int a, int Gr, int nr, int NR, int D, int c0,
                          int nc, int *np, const int *pj, const T *pdl, const int *owed,
                          int &nf_owed, int *spare, int *ncount, const int (&cset)[RPT],
                          bool (&flushed)[RPT], T *wblk)
{
    const int tid = threadIdx.x, nthr = blockDim.x, p = P.p, LB = NR * D;
    __syncthreads();
    if (nf_owed > 0) {
        flush_rows<T, WLDS, CPL>(owed, nf_owed, pj, pdl, np, LB, NR, D, a, Gr, p, c0, nc, P.S,
                                 P.W, wblk);
        nf_owed = 0;
        __syncthreads();
    }
    if (tid == 0)
        *ncount = 0;
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int k = tid + u * nthr;
        if (k < nr) {
            if (flushed[u]) {  // rewritten after the last step (one set of lists)
                np[k] = 0;
                flushed[u] = false;
            }
            if (np[cset[u] * NR + k] > 0)
                spare[atomicAdd(ncount, 1)] = 2 * k + cset[u];
        }
    }
    __syncthreads();
    flush_rows<T, WLDS, CPL>(spare, *ncount, pj, pdl, np, LB, NR, D, a, Gr, p, c0, nc, P.S, P.W,
                             wblk);
    __syncthreads();
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int k = tid + u * nthr;
        if (k < nr)
            np[cset[u] * NR + k] = 0;
    }
}

// End of one lambda of a path: apply every pending row update to the stored
// W block (the caller has done so with flush_all), then write this
// workgroup's block of the dense Omega (rows i = a (mod Gr), columns of
// slice b) and add its share of |E-hat| and of the objective
// F(Omega) = -sum log omega_ii + 1/2 sum_ij omega_ij W_ij
// + lam sum_{i<j} |omega_ij| to the lambda's record.
template <typename T, bool WLDS, int RPT, int CPL>
__device__ void end_of_lambda(const SweepParams<T> &P, int l, T lam, const Circle &C, int a,
                              int Gr, int nr, int NR, int c0, int nc, T *wblk, const T *omp,
                              const T *omdp, double *dred, unsigned long long *nred)
{
    const int tid = threadIdx.x, nthr = blockDim.x, p = P.p;
    T *om = P.omega_out[l];
    double part = 0.0;
    unsigned long long cnt = 0;
    for (long e = tid; e < (long)nr * nc; e += nthr) {
        const int k = (int)(e / nc), c = (int)(e - (long)k * nc);
        const int i = a + k * Gr, j = c0 + c;
        const T wij = WLDS ? wblk[(size_t)k * nc + c] : P.W[(size_t)i * p + j];
        T w;
        if (i == j) {
            w = omdp[k];
            part -= log((double)w);
        } else {
            w = omp[(size_t)C.colour(i, j) * NR + k];
            if (i < j) {
                part += (double)lam * fabs((double)w);
                cnt += (w != T(0)) ? 1ull : 0ull;
            }
        }
        part += 0.5 * (double)w * (double)wij;
        om[(size_t)i * p + j] = w;
    }
    for (int off = 32; off > 0; off >>= 1) {
        part += __shfl_xor(part, off, 64);
        cnt += __shfl_xor(cnt, off, 64);
    }
    const int wv = tid >> 6, nw = nthr >> 6;
    if ((tid & 63) == 0) {
        dred[wv] = part;
        nred[wv] = cnt;
    }
    __syncthreads();
    if (tid == 0) {
        double sp = 0.0;
        unsigned long long sc = 0;
        for (int w2 = 0; w2 < nw; ++w2) {
            sp += dred[w2];
            sc += nred[w2];
        }
        atomicAdd(&P.rec[l].objective, sp);
        atomicAdd(&P.rec[l].nnz_upper, sc);
    }
    __syncthreads();
}

// One solve (a whole lambda path) by workgroup g of the G workgroups that
// share the problem described by P.  CPL: columns per lane in row rewrites.
//
// ADJ selects the adjoint system of the implicit gradient instead of the
// estimate.  At Omega-hat the stationarity conditions on the free entries
// (the diagonal, and the pairs with omega_ij != 0) have the symmetric Jacobian
//   (J v)_ij = U_ij + U_ji,   (J v)_ii = U_ii + v_ii / omega_ii^2,   U = V S,
// with V the symmetric matrix of the unknowns v (0 off the free pairs): the
// same structure as eqs. (2)-(3) with U in place of W.  Gauss-Seidel on
// J v = g in the colour order is therefore this same sweep with linear
// coordinate updates,
//   v_ij <- (g_ij - (U_ij + U_ji - (S_ii + S_jj) v_ij)) / (S_ii + S_jj),
//   v_ii <- (g_ii - (U_ii - S_ii v_ii)) / (S_ii + 1 / omega_ii^2),
// a pair outside the active set keeping v_ij = 0; pairs of one colour share
// no vertex, so they are independent as in Lemma 2.  The buffers W, omp and
// omdp then hold U and v; P.adj_g holds g_ij per colour in omp's layout (NaN
// for a pair that is not free) and P.adj_gd / P.adj_hd hold g_ii and
// S_ii + 1/omega_ii^2 per row.
//
// TAB takes the partners from the colouring table P.part (active-set sweeps)
// instead of Algorithm 1's closed form.  JNT runs population P.pop of a joint
// two-population solve (Section 6): each pair and diagonal entry is updated by
// the block minimisers joint_pair / joint_diag from both populations' published
// entries, and this workgroup also keeps its copy of the other omega.
// BG selects the rewrite mode: 0 = right after each step, 1 = in the
// background (the host has set P.ovl), 2 = as P.ovl says (one kernel for
// problems of both kinds, e.g. a batch).
template <typename T, bool WLDS, int RPT, int CPL, bool ADJ, bool TAB, bool JNT, int BG>
__device__ void pcd_solve(const SweepParams<T> &P, int g, int G, unsigned char *smem_raw)
{
    static_assert(!(JNT && (ADJ || TAB)), "joint mode runs Algorithm 1's forward sweeps only");
    using U = typename Sentinel<T>::U;
    constexpr U SENT = Sentinel<T>::bits;
    const Circle C = Circle::make(P.p);
    // colours per sweep: p_even - 1 for Algorithm 1's schedule, or those of
    // the given colouring (P.part[r * p + i] = partner of i in colour r, -1 idle)
    const int p = P.p, m = TAB ? P.m_tab : C.m;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int a = g / P.Gc, b = g % P.Gc;
    const int Gr = P.Gr;
    const int nr = (a < p) ? (p - a + Gr - 1) / Gr : 0;
    const int c0 = slice_lo(b, P.Gc, p), c1 = slice_lo(b + 1, P.Gc, p);
    const int nc = c1 - c0;
    const int NR = P.nr_max, D = P.depth;
    const int PS = Gr * NR;  // published slots per colour; row i sits at (i mod Gr) * NR + i / Gr

    // LDS carve-up (sizes fixed by the host in sweep_lds_bytes).  The pending
    // lists come in NB sets: with background rewrites a row whose lists are
    // being rewritten keeps appending to its other set.
    const bool ovl = (BG == 2) ? (P.ovl != 0) : (BG == 1);
    const int NB = ovl ? 2 : 1;
    const int LB = NR * D;                      // one set of lists
    T *pdl = reinterpret_cast<T *>(smem_raw);   // pending changes, NB x NR x D
    T *wred = pdl + (size_t)NB * LB;            // 16 wave partials
    T *wblk = wred + 16;                        // W block (LDS variant): NR x nc_max
    int *pj = reinterpret_cast<int *>(wblk + (WLDS ? (size_t)NR * P.nc_max : 0));  // NB x NR x D sources
    int *np = pj + (size_t)NB * LB;             // pending count per row and set, NB x NR
    int *flist = np + NB * NR;                  // rows to rewrite, 2 k + set, two halves by step parity
    int *nflush = flist + 2 * NR;               // [3] counters, by step mod 3; [3] spare
    int *s_fail = nflush + 4;
    int *sfail3 = s_fail + 1;                   // [3] a wait of the step failed, by step mod 3
    unsigned *ured = reinterpret_cast<unsigned *>(sfail3 + 3);  // 16 wave partials
    double *dred = reinterpret_cast<double *>(((uintptr_t)(ured + 16) + 7) & ~(uintptr_t)7);
    unsigned long long *nred = reinterpret_cast<unsigned long long *>(dred + 16);

    const T *__restrict__ S = P.S;
    const T *__restrict__ sd = P.sd;
    T *__restrict__ Wg = P.W;
    T *__restrict__ omp = P.omp + (size_t)g * m * NR;
    T *__restrict__ omdp = P.omdp + (size_t)g * NR;
    const T *__restrict__ adjg = ADJ ? P.adj_g + (size_t)g * m * NR : nullptr;
    // joint mode: this workgroup's copy of the other population's omega
    T *__restrict__ omp_o = JNT ? P.jo_omp + (size_t)g * m * NR : nullptr;
    T *__restrict__ omdp_o = JNT ? P.jo_omdp + (size_t)g * NR : nullptr;
    const T lam2 = JNT ? P.lam2 : T(0);

    for (int k = tid; k < NB * NR; k += nthr)
        np[k] = 0;
    if (tid == 0) {
        nflush[0] = 0;
        nflush[1] = 0;
        nflush[2] = 0;
        nflush[3] = 0;
        *s_fail = 0;
        sfail3[0] = 0;
        sfail3[1] = 0;
        sfail3[2] = 0;
    }
    if (WLDS) {
        for (long e = tid; e < (long)nr * nc; e += nthr) {
            const int k = (int)(e / nc), c = (int)(e - (long)k * nc);
            wblk[(size_t)k * nc + c] = Wg[(size_t)(a + k * Gr) * p + c0 + c];
        }
    }
    __syncthreads();

    T dloc = T(0), gloc = T(0);
    unsigned moved = 0, moved_d = 0;  // pairs / diagonals that changed (counted once each)
    int t = 0, converged = 0, failed = 0;
    // Per row: the set of lists it appends to; with one set, whether its list
    // was rewritten after the last step (it restarts at the next step); with
    // two, whether its other set is being rewritten during this step, and
    // whether the step must read its stored W entries itself.
    int cset[RPT];
    bool flushed[RPT], inflight[RPT], reload[RPT];
    RowNext<T, JNT> nx[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        cset[u] = 0;
        flushed[u] = inflight[u] = reload[u] = false;
        const int k = tid + u * nthr;
        if (k < nr)
            load_next<T, WLDS, TAB, JNT>(nx[u], C, P.part, m, 0, a + k * Gr, k, 0, 0, true, pj, D,
                                         NR, p, c0, c1, nc, S, Wg, wblk, omp, omdp, adjg, omp_o,
                                         omdp_o, P.jo_S, sd, P.jo_sd);
    }
    // Background rewrites: the waves from fw0 on hold no rows; during each
    // step they rewrite the rows the previous step listed (nf_owed of them).
    const int fw0 = (nr + 63) >> 6;
    const bool bg_wave = ovl && (tid >> 6) >= fw0;
    int nf_owed = 0;
    // adjoint mode: the diagonal right-hand side and denominator of each row
    T adj_gd[RPT], adj_hd[RPT];
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
        const int k = tid + u * nthr;
        adj_gd[u] = (ADJ && k < nr) ? P.adj_gd[(size_t)g * NR + k] : T(0);
        adj_hd[u] = (ADJ && k < nr) ? P.adj_hd[(size_t)g * NR + k] : T(1);
    }
    unsigned step = 0;

    // A set-up kernel that found bad input leaves its bits in out[4]; then
    // every workgroup skips the sweeps (the same word is read by all).
    const bool run = ld_dev(&P.out[4]) == 0;

    // Lambda path: lambda l runs until its own convergence test passes or
    // maxit sweeps, then the next starts from where it stopped (warm start:
    // Omega, W and the published entries carry over unchanged).
    const int L = P.L > 0 ? P.L : 1;
    int lidx = 0, tl = 0;
    T lam = P.lams ? (T)P.lams[0] : P.lam;
    if (P.rec && g == 0 && tid == 0)
        P.rec[0].clock_start = __builtin_amdgcn_s_memrealtime();

    while (run) {
        const int cur = t & 1, nxt = cur ^ 1;
        if (t >= 1) {
            // Reset to the sentinel the slots that sweep t + 1 reads after
            // they are written within that sweep: colours >= 1 of buffer nxt,
            // and pd[nxt] when the diagonal entry is published in-sweep (m >= 2).
            // Their last readers finished in sweep t - 1.
            const long long E = (long long)(m - 1) * PS + (m >= 2 ? PS : 0);
            const long long e0 = E * g / G, e1 = E * (g + 1) / G;
            U *pcb = reinterpret_cast<U *>(P.pc + ((size_t)nxt * m + 1) * PS);
            U *pdb = reinterpret_cast<U *>(P.pd + (size_t)nxt * PS);
            for (long long e = e0 + tid; e < e1; e += nthr) {
                if (e < (long long)(m - 1) * PS)
                    st_dev(&pcb[e], SENT);
                else
                    st_dev(&pdb[e - (long long)(m - 1) * PS], SENT);
            }
        }

        for (int r = 0; r < m && !failed; ++r) {
            const bool last = (r == m - 1);
            const int rn = last ? 0 : r + 1;
            const int bufn = last ? nxt : cur;   // buffer of the next colour step
            const int s3 = (int)(step % 3u);
            const U *pcu = reinterpret_cast<const U *>(P.pc + ((size_t)cur * m + r) * PS);
            const U *pdu = reinterpret_cast<const U *>(P.pd + (size_t)cur * PS);
            T *pcn = P.pc + ((size_t)bufn * m + rn) * PS;
            // The next step reads pd when it is the last colour; the buffer
            // is that step's sweep.
            T *pdn = P.pd + (size_t)(last ? nxt : cur) * PS;
            // joint mode: the other population's entries of this step
            const U *pco = JNT ? reinterpret_cast<const U *>(P.jo_pc + ((size_t)cur * m + r) * PS)
                               : nullptr;
            const U *pdo = JNT ? reinterpret_cast<const U *>(P.jo_pd + (size_t)cur * PS) : nullptr;
            int lfail = 0, marked = 0;
            // optional per-step timestamps (100 MHz clock): start, rows done, rewrites done
            unsigned long long *ts =
                (P.tstamp && tid == 0 && step < (unsigned)P.tstamp_steps)
                    ? P.tstamp + ((size_t)g * P.tstamp_steps + step) * 3
                    : nullptr;
            if (ts)
                ts[0] = __builtin_amdgcn_s_memrealtime();

            // ---- background rewrites: the waves without rows rewrite the rows
            // the previous step listed while the row waves run this step.  Those
            // rows append to their other set of lists meanwhile, and read their
            // stored W entries only after the barrier that ends this step.
            if (bg_wave && nf_owed > 0)
                flush_rows<T, WLDS, CPL>(flist + ((step - 1u) & 1u) * NR, nf_owed, pj, pdl, np, LB,
                                         NR, D, a, Gr, p, c0, nc, S, Wg, wblk, fw0);

#pragma unroll
            for (int u = 0; u < RPT; ++u) {
                const int k = tid + u * nthr;
                if (k >= nr || lfail)
                    continue;
                const int i = a + k * Gr;
                RowNext<T, JNT> &x = nx[u];
                const int j = x.j;

                // ---- stored W entries that the previous step could not read: a
                // background rewrite of this row was running then (or the lambda
                // ended and every row was rewritten).  Issued before the poll, so
                // that both round trips overlap.
                if (reload[u]) {
                    if (x.kn >= 0)
                        x.wb = WLDS ? wblk[(size_t)k * nc + (x.kn - c0)] : Wg[(size_t)i * p + x.kn];
                    if (x.pubd)
                        x.wd = WLDS ? wblk[(size_t)k * nc + (i - c0)] : Wg[(size_t)i * p + i];
                    reload[u] = false;
                }

                // ---- poll the published numerator entries of this colour.  The
                // first poll is issued before anything waits for the operands
                // prefetched last step: issued after that wait, the poll's round
                // trip would follow the prefetch's instead of overlapping it.
                U blo = 0, bhi = 0, bd = 0, clo = 0, chi = 0, cd = 0;
                // slots of row i (own, contiguous over k) and of its partner
                const int si = a * NR + k;
                const int sj = (j >= 0) ? (j % Gr) * NR + j / Gr : 0;
                const int lo = (j >= 0 && j < i) ? sj : si, hi = (j >= 0 && j < i) ? si : sj;
                const bool poll_d = last && m >= 2;
                auto issue_poll = [&]() {
                    if (j >= 0) {
                        blo = ld_dev(&pcu[lo]);
                        bhi = ld_dev(&pcu[hi]);
                        if constexpr (JNT) {
                            clo = ld_dev(&pco[lo]);
                            chi = ld_dev(&pco[hi]);
                        }
                    }
                    if (last) {
                        bd = ld_dev(&pdu[si]);
                        if constexpr (JNT)
                            cd = ld_dev(&pdo[si]);
                    }
                };
                auto polled = [&]() {
                    bool ok = true;
                    if (j >= 0) {
                        ok = (blo != SENT) && (bhi != SENT);
                        if constexpr (JNT)
                            ok = ok && (clo != SENT) && (chi != SENT);
                    }
                    if (last) {
                        ok = ok && (!poll_d || bd != SENT);
                        if constexpr (JNT)
                            ok = ok && (!poll_d || cd != SENT);
                    }
                    return ok;
                };
                issue_poll();

                // ---- stored entries plus pending updates, for what this step publishes
                const T *pdlx = pdl + (size_t)x.set * LB + (size_t)k * D;
                T vpre = T(0), vdpre = T(0);
                if (x.kn >= 0) {
                    vpre = x.wb;
#pragma unroll
                    for (int e = 0; e < kMaxDepth; ++e)
                        if (e < x.n)
                            vpre = fma(pdlx[e], x.sv[e], vpre);
                }
                // ---- wait for the polled entries, polling again until they are there
                {
                    long long spins = 0;
                    while (!polled()) {
                        ++spins;
                        if (spins > P.spin_limit ||
                            ((spins & 255) == 0 && ld_dev(&P.out[3]) != 0)) {
                            st_dev(&P.out[3], 1);
                            lfail = 1;
                            break;
                        }
                        __builtin_amdgcn_s_sleep(1);
                        issue_poll();
                    }
                }
                if (lfail) {
                    *s_fail = 1;
                    sfail3[s3] = 1;
                    continue;
                }

                // ---- with one set of lists, a row rewritten after the last step
                // starts a new list (its entries are still read by the folds of
                // this step, which take the list as it was).  The
                // once-per-sweep gathers of the W_ii fold come after the wait:
                // loads issued before the poll would hold up the poll's first
                // answer (a wave's loads complete in order).
                if (flushed[u]) {
                    np[k] = 0;
                    flushed[u] = false;
                }
                const int cs = cset[u];
                const int n0 = np[cs * NR + k];
                if (x.pubd) {
                    const int *pjx = pj + (size_t)x.set * LB + (size_t)k * D;
                    vdpre = x.wd;
                    for (int e = 0; e < x.n; ++e)
                        vdpre = fma(pdlx[e], S[(size_t)pjx[e] * p + i], vdpre);
                    // every load of this once-per-sweep fold is consumed; said
                    // explicitly so that the compiler's wait analysis does not
                    // carry them into the next step, whose first register
                    // writes would then wait for every load in flight
                    __builtin_amdgcn_s_waitcnt(0x0F70);  // vmcnt(0)
                }

                // ---- eq. (3) for the pair, eq. (2) after the last colour
                T del = T(0), dd = T(0);
                T del_o = T(0), dd_o = T(0);  // joint mode: the other population's changes
                if (j >= 0) {
                    const T sden = x.sd_lo + x.sd_hi;
                    const T bnum = fma(-sden, x.w, as_value<T>(blo) + as_value<T>(bhi));
                    T wn;
                    if constexpr (JNT) {
                        // the block update takes population 1's operands first on both sides
                        const T sden_o = x.sdo_lo + x.sdo_hi;
                        const T bnum_o = fma(-sden_o, x.wo, as_value<T>(clo) + as_value<T>(chi));
                        T x1, x2;
                        if (P.pop == 0)
                            joint_pair(sden, bnum, sden_o, bnum_o, lam, lam2, x1, x2);
                        else
                            joint_pair(sden_o, bnum_o, sden, bnum, lam, lam2, x1, x2);
                        wn = P.pop == 0 ? x1 : x2;
                        const T wno = P.pop == 0 ? x2 : x1;
                        del_o = wno - x.wo;
                        if (del_o != T(0))
                            omp_o[(size_t)r * NR + k] = wno;
                    } else if (ADJ) {
                        wn = (x.g == x.g) ? (x.g - bnum) / sden : x.w;
                    } else {
                        wn = soft_threshold(-bnum, lam) / sden;
                    }
                    del = wn - x.w;
                    if (del != T(0))
                        omp[(size_t)r * NR + k] = wn;
                }
                if (last) {
                    T wii = as_value<T>(bd);
                    if (del != T(0))
                        wii = fma(del, x.s_ji, wii);
                    const T sii = x.sii;
                    const T c = fma(-sii, x.od, wii);
                    T on;
                    if constexpr (JNT) {
                        T wio = as_value<T>(cd);
                        if (del_o != T(0))
                            wio = fma(del_o, x.s_jio, wio);
                        const T sio = x.sio;
                        const T co = fma(-sio, x.odo, wio);
                        T y1, y2;
                        if (P.pop == 0)
                            joint_diag(sii, c, sio, co, lam2, y1, y2);
                        else
                            joint_diag(sio, co, sii, c, lam2, y1, y2);
                        on = P.pop == 0 ? y1 : y2;
                        const T ono = P.pop == 0 ? y2 : y1;
                        dd_o = ono - x.odo;
                        if (dd_o != T(0))
                            omdp_o[k] = ono;
                        gloc = (ono > gloc || ono != ono) ? ono : gloc;
                    } else if (ADJ) {
                        on = (adj_gd[u] - c) / adj_hd[u];
                    } else {
                        const T disc = sqrt(fma(c, c, T(4) * sii));
                        // eq. (2); for c >= 0 the same root is 2 / (c + disc) without cancellation.
                        on = (c >= T(0)) ? T(2) / (c + disc) : (disc - c) / (T(2) * sii);
                    }
                    dd = on - x.od;
                    if (dd != T(0))
                        omdp[k] = on;
                    const T gv = ADJ ? fabs(on) : on;
                    gloc = (gv > gloc || gv != gv) ? gv : gloc;
                }

                // ---- record the changes as pending updates of row i
                int *pjc = pj + (size_t)cs * LB + (size_t)k * D;
                T *pdlc = pdl + (size_t)cs * LB + (size_t)k * D;
                int n = n0;
                if (del != T(0)) {
                    pjc[n] = j;
                    pdlc[n] = del;
                    ++n;
                }
                if (dd != T(0)) {
                    pjc[n] = i;
                    pdlc[n] = dd;
                    ++n;
                }
                np[cs * NR + k] = n;

                // ---- publish what the next colour reads from row i
                if (x.kn >= 0) {
                    T v = vpre;
                    if (del != T(0))
                        v = fma(del, x.s_jn, v);
                    if (dd != T(0))
                        v = fma(dd, x.s_in, v);
                    st_dev(&pcn[a * NR + k], v);
                }
                if (x.pubd) {
                    T v = vdpre;
                    if (del != T(0))
                        v = fma(del, x.s_ji, v);
                    if (dd != T(0))
                        v = fma(dd, sd[i], v);
                    st_dev(&pdn[a * NR + k], v);
                }
                const bool mark = n > D - 2;
                if (mark) {
                    flist[(step & 1u) * NR + atomicAdd(&nflush[s3], 1)] = 2 * k + cs;
                    marked = 1;
                }
                T ad = fabs(del) > fabs(dd) ? fabs(del) : fabs(dd);
                if constexpr (JNT) {
                    const T ao = fabs(del_o) > fabs(dd_o) ? fabs(del_o) : fabs(dd_o);
                    ad = (ao > ad || ao != ao) ? ao : ad;
                }
                dloc = (ad > dloc || ad != ad) ? ad : dloc;
                if (b == 0) {
                    moved += (j > i && del != T(0)) ? 1u : 0u;
                    moved_d += (dd != T(0)) ? 1u : 0u;
                }

                // ---- operands of the row's next step, which folds the n entries
                // of this list set.  The stored W entries read here are read
                // before any rewrite of this list (it starts after the barrier
                // below), so they go with all n entries.  While a background
                // rewrite of the row's other set runs (listed last step), its W
                // segment is not read here but at the start of the next step.
                const bool loadw = !(ovl && inflight[u]);
                reload[u] = !loadw;
                inflight[u] = ovl && mark;
                load_next<T, WLDS, TAB, JNT>(nx[u], C, P.part, m, rn, i, k, n, cs, loadw,
                                             pj + (size_t)cs * LB, D, NR, p, c0, c1, nc, S, Wg,
                                             wblk, omp, omdp, adjg, omp_o, omdp_o, P.jo_S, sd,
                                             P.jo_sd);
                if (mark) {
                    if (ovl) {
                        // the row goes on in its other set of lists, whose
                        // background rewrite has ended: with depth >= 4 (see
                        // set_overlap) a row is listed at most every other step
                        cset[u] = cs ^ 1;
                        np[(cs ^ 1) * NR + k] = 0;
                    } else {
                        flushed[u] = true;  // rewritten right after this step
                    }
                }
            }

            // ---- every row of the step is done; rewrite the rows whose lists are full.
            // The step's outcome (rows to rewrite, a failed wait) is in LDS words
            // kept by step mod 3, read after a plain barrier.  A block-wide vote
            // here would wait for every load the wave has in flight, i.e. for
            // the operands just prefetched for the next step, before the
            // rewrites could issue their own loads; this way the two overlap.
            __syncthreads();
            const int nf = nflush[s3];
            const int sf = sfail3[s3];
            if (tid == 0) {
                // the previous step's words, read by all by now
                nflush[(s3 + 2) % 3] = 0;
                sfail3[(s3 + 2) % 3] = 0;
            }
            if (ts)
                ts[1] = __builtin_amdgcn_s_memrealtime();
            if (sf) {
                failed = 1;
                break;
            }
            if (ovl) {
                nf_owed = nf;  // rewritten in the background during the next step
            } else if (nf > 0) {
                flush_rows<T, WLDS, CPL>(flist + (step & 1u) * NR, nf, pj, pdl, np, LB, NR, D, a,
                                         Gr, p, c0, nc, S, Wg, wblk);
                __syncthreads();
            }
            if (ts)
                ts[2] = __builtin_amdgcn_s_memrealtime();
            ++step;
        }
        if (failed)
            break;

        // ---- end of sweep t: reductions, then the sweep barrier
        const T dm = block_max(dloc, wred);
        const T gm = block_max(gloc, wred);
        const unsigned mv = block_sum(moved, ured);
        const unsigned mvd = block_sum(moved_d, ured);
        if (tid == 0) {
            unsigned long long *rt = P.red + 4 * (size_t)t;
            __hip_atomic_fetch_max(&rt[0], ord_bits(dm), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_fetch_max(&rt[1], ord_bits(gm), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (mv)
                __hip_atomic_fetch_add(&rt[2], (unsigned long long)mv, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
            if (mvd)
                __hip_atomic_fetch_add(&rt[3], (unsigned long long)mvd, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
        }
        dloc = T(0);
        gloc = T(0);
        moved = 0;
        moved_d = 0;
        if (!sweep_barrier(P, (unsigned)(t + 1), s_fail, JNT ? P.pop * G + g : g,
                           JNT ? 2 * G : G)) {
            failed = 1;
            break;
        }
        const T delta = from_ord(ld_dev(&P.red[4 * (size_t)t]), T(0));
        const T gmax = from_ord(ld_dev(&P.red[4 * (size_t)t + 1]), T(0));
        ++t;
        ++tl;
        T tol_eff = P.tol_coef * gmax;
        tol_eff = tol_eff > P.tol ? tol_eff : P.tol;
        const bool conv = delta < tol_eff;
        if (conv || tl >= P.maxit) {
            converged = conv ? 1 : 0;
            if (P.omega_out) {
                flush_all<T, WLDS, RPT, CPL>(P, a, Gr, nr, NR, D, c0, nc, np, pj, pdl,
                                             flist + ((step - 1u) & 1u) * NR, nf_owed,
                                             flist + (step & 1u) * NR, &nflush[3], cset, flushed,
                                             wblk);
                end_of_lambda<T, WLDS, RPT, CPL>(P, lidx, lam, C, a, Gr, nr, NR, c0, nc, wblk, omp,
                                                 omdp, dred, nred);
                // W now holds every update: the next step reads its stored
                // entries afresh and folds no list
#pragma unroll
                for (int u = 0; u < RPT; ++u) {
                    reload[u] = true;
                    inflight[u] = false;
                    nx[u].n = 0;
                }
            }
            if (P.rec && g == 0 && tid == 0) {
                const unsigned long long now = __builtin_amdgcn_s_memrealtime();
                P.rec[lidx].t_end = t;
                P.rec[lidx].converged = converged;
                P.rec[lidx].clock_end = now;
                if (lidx + 1 < L)
                    P.rec[lidx + 1].clock_start = now;
            }
            if (++lidx >= L)
                break;
            lam = (T)P.lams[lidx];
            tl = 0;
        }
    }

    // Apply every pending update so that the stored W is Omega S again.
    flush_all<T, WLDS, RPT, CPL>(P, a, Gr, nr, NR, D, c0, nc, np, pj, pdl,
                                 flist + ((step - 1u) & 1u) * NR, nf_owed, flist + (step & 1u) * NR,
                                 &nflush[3], cset, flushed, wblk);
    __syncthreads();
    if (WLDS) {
        for (long e = tid; e < (long)nr * nc; e += nthr) {
            const int k = (int)(e / nc), c = (int)(e - (long)k * nc);
            Wg[(size_t)(a + k * Gr) * p + c0 + c] = wblk[(size_t)k * nc + c];
        }
    }
    if (g == 0 && tid == 0 && (!JNT || P.pop == 0)) {
        P.out[0] = t;
        P.out[1] = converged;
        P.out[2] = failed;
    }
}

}  // namespace

}  // namespace concord
