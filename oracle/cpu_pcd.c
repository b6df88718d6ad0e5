/*
 * CPU baseline for the benchmark: CONCORD-PCD (Algorithm 1 of arXiv
 * 2106.09382) with the maintained product W = Omega S, serial or with the
 * pairs of each colour spread over OpenMP threads.  TEST INFRASTRUCTURE
 * ONLY: the benchmark's CPU-baseline leg and the tests load it; the solver
 * never does, and it shares no code with the HIP path.
 *
 * Where the oracle (concord_oracle.c) evaluates eqs. (2)-(3) by direct sums,
 * this keeps W = Omega S: because Omega and S are symmetric,
 *   b_ij = sum_{u != j} omega_iu S_ju + sum_{u != i} omega_uj S_iu
 *        = W_ij + W_ji - (S_ii + S_jj) omega_ij,
 *   c_i  = sum_{j != i} omega_ij S_ij = W_ii - S_ii omega_ii,
 * and a change d of omega_ij = omega_ji adds d S_j. to row i of W and
 * d S_i. to row j (d S_i. to row i for a diagonal change).  Pairs of one
 * colour share no vertex (Lemma 2), so each pair reads and writes only its
 * own two rows: the pairs of a colour can be processed in any order or in
 * parallel and give the same bits as Algorithm 1's simultaneous update.
 * Every row is updated by one thread, in colour order, so the parallel run
 * gives the same bits as the serial one.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int oracle_round_robin(int p, int32_t *pairs);

static double soft_w(double x, double tau)
{
    double a = fabs(x) - tau;
    if (a <= 0.0)
        return 0.0;
    return x > 0.0 ? a : -a;
}

/*
 *   S, p, lam, tol, maxit  as for oracle_pcd (identity start)
 *   threads       OpenMP threads (0: the runtime's default)
 *   colour_limit  if > 0, stop after that many colour steps in total (a
 *                 bounded sample for timing)
 *   omega         out, p x p
 *   info          out [0] sweeps, [1] last delta, [2] converged,
 *                 [3] colour steps done, [4] pairs that changed,
 *                 [5] diagonals that changed, [6] threads used
 * Returns 0, -1 on invalid arguments, -3 when some S_ii <= 0, -4 when
 * memory runs out.
 */
int cpu_pcd_wform(const double *S, int p, double lam, double tol, int maxit, int threads,
                  long long colour_limit, double *omega, double *info)
{
    if (!S || !omega || p < 1 || !(lam >= 0.0) || !(tol > 0.0) || maxit < 1 || threads < 0)
        return -1;
    for (int i = 0; i < p; ++i)
        if (!(S[(size_t)i * p + i] > 0.0))
            return -3;
    const int pe = p + (p & 1), H = pe / 2, m = pe - 1;
    int32_t *tab = (int32_t *)malloc(sizeof(int32_t) * ((size_t)m * H * 2 + 2));
    double *W = (double *)malloc(sizeof(double) * (size_t)p * p);
    if (!tab || !W) {
        free(tab);
        free(W);
        return -4;
    }
    oracle_round_robin(p, tab);
    memcpy(W, S, sizeof(double) * (size_t)p * p);  /* W = I S */
    memset(omega, 0, sizeof(double) * (size_t)p * p);
    for (int i = 0; i < p; ++i)
        omega[(size_t)i * p + i] = 1.0;
    const int nt = threads > 0 ? threads : omp_get_max_threads();

    int t = 0, converged = 0, stopped = 0;
    double delta = 0.0;
    long long steps = 0, moved = 0, moved_d = 0;
    while (!stopped && t < maxit) {
        ++t;
        delta = 0.0;
        for (int k = 0; k < m; ++k) {
            const int32_t *pr = tab + (size_t)k * H * 2;
            double dk = 0.0;
            long long mk = 0;
#pragma omp parallel for num_threads(nt) schedule(dynamic, 4) reduction(max : dk) reduction(+ : mk)
            for (int q = 0; q < H; ++q) {
                const int i = pr[2 * q], j = pr[2 * q + 1];
                if (i == p || j == p)
                    continue;
                double *wi = W + (size_t)i * p, *wj = W + (size_t)j * p;
                const double *si = S + (size_t)i * p, *sj = S + (size_t)j * p;
                const double a = si[i] + sj[j];
                const double b = wi[j] + wj[i] - a * omega[(size_t)i * p + j];
                const double w = soft_w(-b, lam) / a;
                const double d = w - omega[(size_t)i * p + j];
                if (d != 0.0) {
                    for (int u = 0; u < p; ++u) {
                        wi[u] += d * sj[u];
                        wj[u] += d * si[u];
                    }
                    omega[(size_t)i * p + j] = w;
                    omega[(size_t)j * p + i] = w;
                    ++mk;
                }
                if (fabs(d) > dk)
                    dk = fabs(d);
            }
            if (dk > delta)
                delta = dk;
            moved += mk;
            ++steps;
            if (colour_limit > 0 && steps >= colour_limit) {
                stopped = 1;
                break;
            }
        }
        if (stopped)
            break;
        double dd = 0.0;
        long long md = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(max : dd) reduction(+ : md)
        for (int i = 0; i < p; ++i) {
            double *wi = W + (size_t)i * p;
            const double *si = S + (size_t)i * p;
            const double sii = si[i], oi = omega[(size_t)i * p + i];
            const double c = wi[i] - sii * oi;
            const double w = (-c + sqrt(c * c + 4.0 * sii)) / (2.0 * sii);
            const double d = w - oi;
            if (d != 0.0) {
                for (int u = 0; u < p; ++u)
                    wi[u] += d * si[u];
                omega[(size_t)i * p + i] = w;
                ++md;
            }
            if (fabs(d) > dd)
                dd = fabs(d);
        }
        if (dd > delta)
            delta = dd;
        moved_d += md;
        if (delta < tol) {
            converged = 1;
            break;
        }
    }
    if (info) {
        info[0] = t;
        info[1] = delta;
        info[2] = converged;
        info[3] = (double)steps;
        info[4] = (double)moved;
        info[5] = (double)moved_d;
        info[6] = nt;
    }
    free(tab);
    free(W);
    return 0;
}
