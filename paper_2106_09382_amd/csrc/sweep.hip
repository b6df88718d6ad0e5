// Persistent CONCORD-PCD sweep kernel (Algorithm 1 of arXiv 2106.09382) for gfx950.
//
// Method.  For a pair (i, j) of colour r, eq. (3)'s numerator is
//   b_ij = sum_{u != j} omega_iu S_ju + sum_{u != i} omega_uj S_iu
//        = W_ij + W_ji - (S_ii + S_jj) omega_ij,           W = Omega S,
// because Omega and S are symmetric ((S Omega)_ij = W_ji).  Changing
// omega_ij = omega_ji by d changes only rows i and j of W: W_i. += d S_j. and
// W_j. += d S_i..  For the diagonal step, eq. (2)'s sum is
// c_i = W_ii - S_ii omega_ii, and changing omega_ii by d gives W_i. += d S_i..
// So each pair costs O(1) to evaluate plus an axpy of its two rows when it
// moves, instead of two length-p sums.
//
// Work split.  Workgroup (a, b), a < Gr, b < Gc, owns rows i = a (mod Gr) of W
// restricted to column slice b; its block stays in LDS when it fits, else in
// HBM (touched only by this workgroup, so ordinary cached accesses).  Per
// colour step every workgroup:
//   A. reads, for each own row i with partner j, the two published numerator
//      entries W_ij, W_ji and omega_ij, and evaluates eq. (3) (and, after the
//      last colour, eq. (2)).  Every workgroup of rows i's group and of j's
//      group evaluates the same pair from the same bits, so all agree on d.
//   B. publishes, for the next colour's partner k of row i when column k lies
//      in its slice, the updated W_ik (the row's entry that the next colour
//      reads), plus W_ii ahead of the last colour.
//   C. signals the grid barrier,
//   D. applies its share of the row axpys while the barrier settles,
//   E. waits for the barrier.
// The diagonal step needs no barrier of its own: every workgroup of row i's
// group recomputes c_i from the published W_ii.  So one sweep is m barriers.
//
// Convergence.  Each entry of Omega changes exactly once per sweep, so
// |Omega^(t) - Omega^(t-1)|_inf is the max |d| over the sweep; it is reduced
// with one atomic max per workgroup per sweep and read by every workgroup
// after the next barrier, so all agree on when to stop.
#include "device_common.hpp"
#include "schedule.hpp"
#include "sweep.hpp"

namespace concord {

namespace {

// Grid barrier: workgroup g stores the epoch into flags[g]; wave 0 of every
// workgroup polls all flags.  Bounded: after spin_limit polls (or when any
// workgroup has raised the abort word) it gives up and reports failure.
template <typename T>
__device__ __forceinline__ void grid_arrive(const SweepParams<T> &P, unsigned epoch)
{
    wait_stores();
    __syncthreads();
    if (gridDim.x > 1 && threadIdx.x == 0)
        st_dev(&P.flags[blockIdx.x], epoch);
}

template <typename T>
__device__ __forceinline__ bool grid_wait(const SweepParams<T> &P, unsigned epoch, int *s_fail)
{
    if (gridDim.x > 1 && threadIdx.x < 64) {
        const int G = gridDim.x;
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
    return *s_fail == 0;
}

template <typename T>
__device__ __forceinline__ T block_max(T v, T *scratch)
{
    // wave-level max via shuffles, then across waves through LDS
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

}  // namespace

template <typename T, bool WLDS>
__global__ void __launch_bounds__(1024) pcd_sweep_kernel(SweepParams<T> P)
{
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const Circle C = Circle::make(P.p);
    const int p = P.p, m = C.m, H = C.H;
    const int tid = threadIdx.x, nthr = blockDim.x;
    const int a = blockIdx.x / P.Gc, b = blockIdx.x % P.Gc;
    const int nr = (a < p) ? (p - a + P.Gr - 1) / P.Gr : 0;
    const int c0 = slice_lo(b, P.Gc, p), c1 = slice_lo(b + 1, P.Gc, p);
    const int nc = c1 - c0;
    const int NR = P.nr_max;

    // LDS carve-up (sizes fixed by the host in sweep_lds_bytes).
    T *rdel = reinterpret_cast<T *>(smem_raw);  // change of omega_{i, partner}
    T *rdd = rdel + NR;                         // change of omega_ii (last colour)
    T *rpend = rdd + NR;                        // new omega_{i, partner}, written one step late
    T *rpendd = rpend + NR;                     // new omega_ii, written one step late
    T *wred = rpendd + NR;                      // 16 wave partials
    T *wblk = wred + 16;                        // W block (LDS variant): NR x nc_max
    int *rj = reinterpret_cast<int *>(wblk + (WLDS ? (size_t)NR * P.nc_max : 0));
    int *act = rj + NR;                         // active row list
    int *nact = act + NR;                       // [2] counters by step parity
    int *s_fail = nact + 2;
    unsigned *ured = reinterpret_cast<unsigned *>(s_fail + 1);  // 16 wave partials

    const T *__restrict__ S = P.S;
    T *__restrict__ Wg = P.W;

    if (tid == 0) {
        nact[0] = 0;
        nact[1] = 0;
        *s_fail = 0;
    }
    if (WLDS) {
        for (long e = tid; e < (long)nr * nc; e += nthr) {
            int k = (int)(e / nc), c = (int)(e - (long)k * nc);
            wblk[(size_t)k * nc + c] = Wg[(size_t)(a + k * P.Gr) * p + c0 + c];
        }
    }
    __syncthreads();

    T dloc = T(0), gloc = T(0);
    unsigned moved = 0, moved_d = 0;  // pairs / diagonals that changed (counted once each)
    int t = 0, r = 0, converged = 0, failed = 0;
    unsigned long long s = 0;  // global colour-step counter

    // A set-up kernel that found bad input leaves its bits in out[4]; then
    // every workgroup skips the sweeps (the same word is read by all).
    const bool run = ld_dev(&P.out[4]) == 0;

    while (run) {
        const int par = (int)(s & 1);
        const bool last = (r == m - 1);
        const int tcur = (int)(s / (unsigned long long)m);
        if (tid == 0)
            nact[par ^ 1] = 0;

        // ---- A. evaluate eq. (3) for every own row (and eq. (2) after the last colour)
        for (int k = tid; k < nr; k += nthr) {
            const int i = a + k * P.Gr;
            const int j = C.partner(r, i);
            T del = T(0), dd = T(0);
            if (j >= 0) {
                const int lo = i < j ? i : j, hi = i < j ? j : i;
                const T wlo = ld_dev(&P.pub[(size_t)par * p + lo]);
                const T whi = ld_dev(&P.pub[(size_t)par * p + hi]);
                const T w = ld_dev(&P.omc[(size_t)r * H + C.slot(r, i)]);
                const T sden = P.sd[lo] + P.sd[hi];
                const T bnum = fma(-sden, w, wlo + whi);
                const T wn = soft_threshold(-bnum, P.lam) / sden;
                del = wn - w;
                rpend[k] = wn;
            }
            if (last) {
                T wii = ld_dev(&P.pubd[(size_t)(tcur & 1) * p + i]);
                if (j >= 0 && del != T(0))
                    wii = fma(del, S[(size_t)j * p + i], wii);
                const T od = ld_dev(&P.omd[i]);
                const T sii = P.sd[i];
                const T c = fma(-sii, od, wii);
                const T disc = sqrt(fma(c, c, T(4) * sii));
                // eq. (2); for c >= 0 the same root is 2 / (c + disc) without cancellation.
                const T on = (c >= T(0)) ? T(2) / (c + disc) : (disc - c) / (T(2) * sii);
                dd = on - od;
                rpendd[k] = on;
                gloc = (on > gloc || on != on) ? on : gloc;
            }
            rj[k] = j;
            rdel[k] = del;
            rdd[k] = dd;
            if (b == 0) {
                moved += (j > i && del != T(0)) ? 1u : 0u;
                moved_d += (dd != T(0)) ? 1u : 0u;
            }
            const T ad = fabs(del) > fabs(dd) ? fabs(del) : fabs(dd);
            dloc = (ad > dloc || ad != ad) ? ad : dloc;
            if (del != T(0) || dd != T(0)) {
                int slot = atomicAdd(&nact[par], 1);
                act[slot] = k;
            }
        }

        // ---- B. publish the next step's numerator entries of own rows
        const int rn = last ? 0 : r + 1;
        const int parn = par ^ 1;
        const int tnext = (int)((s + 1) / (unsigned long long)m);
        for (int k = tid; k < nr; k += nthr) {
            const int i = a + k * P.Gr;
            const int j = rj[k];
            const T del = rdel[k], dd = rdd[k];
            const int kn = C.partner(rn, i);
            if (kn >= c0 && kn < c1) {
                T v = WLDS ? wblk[(size_t)k * nc + (kn - c0)] : Wg[(size_t)i * p + kn];
                if (del != T(0))
                    v = fma(del, S[(size_t)j * p + kn], v);
                if (dd != T(0))
                    v = fma(dd, S[(size_t)i * p + kn], v);
                st_dev(&P.pub[(size_t)parn * p + i], v);
            }
            if (rn == m - 1 && i >= c0 && i < c1) {
                T v = WLDS ? wblk[(size_t)k * nc + (i - c0)] : Wg[(size_t)i * p + i];
                if (del != T(0))
                    v = fma(del, S[(size_t)j * p + i], v);
                if (dd != T(0))
                    v = fma(dd, S[(size_t)i * p + i], v);
                st_dev(&P.pubd[(size_t)(tnext & 1) * p + i], v);
            }
        }

        if (last) {
            const T dm = block_max(dloc, wred);
            const T gm = block_max(gloc, wred);
            const unsigned mv = block_sum(moved, ured);
            const unsigned mvd = block_sum(moved_d, ured);
            if (tid == 0) {
                unsigned long long *rt = P.red + 4 * (size_t)tcur;
                __hip_atomic_fetch_max(&rt[0], ord_bits(dm), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_fetch_max(&rt[1], ord_bits(gm), __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
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
        }

        // ---- C. signal
        const unsigned epoch = (unsigned)(s + 1);
        grid_arrive(P, epoch);

        // ---- D. row axpys on the owned block: W_i. += d S_j. (+ d_ii S_i.)
        {
            const int na = nact[par];
            const long total = (long)na * nc;
            for (long e = tid; e < total; e += nthr) {
                const int ai = (int)(e / nc);
                const int c = (int)(e - (long)ai * nc);
                const int k = act[ai];
                const int i = a + k * P.Gr;
                const int j = rj[k];
                const T del = rdel[k], dd = rdd[k];
                T *wp = WLDS ? &wblk[(size_t)k * nc + c] : &Wg[(size_t)i * p + c0 + c];
                T v = *wp;
                if (del != T(0))
                    v = fma(del, S[(size_t)j * p + c0 + c], v);
                if (dd != T(0))
                    v = fma(dd, S[(size_t)i * p + c0 + c], v);
                *wp = v;
            }
        }

        // ---- E. wait, then the deferred omega writes of this step
        if (!grid_wait(P, epoch, s_fail)) {
            failed = 1;
            break;
        }
        if (b == 0) {
            for (int k = tid; k < nr; k += nthr) {
                const int i = a + k * P.Gr;
                const int j = rj[k];
                if (j > i)
                    st_dev(&P.omc[(size_t)r * H + C.slot(r, i)], rpend[k]);
                if (last)
                    st_dev(&P.omd[i], rpendd[k]);
            }
        }
        ++s;
        if (last) {
            t = tcur + 1;
            const T delta = from_ord(ld_dev(&P.red[4 * (size_t)tcur]), T(0));
            const T gmax = from_ord(ld_dev(&P.red[4 * (size_t)tcur + 1]), T(0));
            T tol_eff = P.tol_coef * gmax;
            tol_eff = tol_eff > P.tol ? tol_eff : P.tol;
            if (delta < tol_eff) {
                converged = 1;
                break;
            }
            if (t >= P.maxit)
                break;
        }
        r = rn;
    }

    wait_stores();
    if (WLDS) {
        __syncthreads();
        for (long e = tid; e < (long)nr * nc; e += nthr) {
            int k = (int)(e / nc), c = (int)(e - (long)k * nc);
            Wg[(size_t)(a + k * P.Gr) * p + c0 + c] = wblk[(size_t)k * nc + c];
        }
    }
    if (blockIdx.x == 0 && tid == 0) {
        P.out[0] = t;
        P.out[1] = converged;
        P.out[2] = failed;
    }
}

template <typename T>
size_t sweep_lds_bytes(const SweepParams<T> &P, int threads)
{
    (void)threads;
    size_t b = sizeof(T) * (4 * (size_t)P.nr_max + 16);
    if (P.w_lds)
        b += sizeof(T) * (size_t)P.nr_max * P.nc_max;
    b += sizeof(int) * (2 * (size_t)P.nr_max + 3) + sizeof(unsigned) * 16;
    return b;
}

template <typename T>
hipError_t launch_sweep(const SweepParams<T> &P, int threads, hipStream_t stream)
{
    size_t lds = sweep_lds_bytes(P, threads);
    const int G = P.Gr * P.Gc;
    SweepParams<T> arg = P;
    void *args[] = {&arg};
    const void *fn = P.w_lds ? (const void *)pcd_sweep_kernel<T, true>
                             : (const void *)pcd_sweep_kernel<T, false>;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess)
        return e;
    if (G == 1)
        return hipLaunchKernel(fn, dim3(1), dim3(threads), args, lds, stream);
    return hipLaunchCooperativeKernel(fn, dim3(G), dim3(threads), args, (unsigned)lds, stream);
}

template size_t sweep_lds_bytes<float>(const SweepParams<float> &, int);
template size_t sweep_lds_bytes<double>(const SweepParams<double> &, int);
template hipError_t launch_sweep<float>(const SweepParams<float> &, int, hipStream_t);
template hipError_t launch_sweep<double>(const SweepParams<double> &, int, hipStream_t);

}  // namespace concord
