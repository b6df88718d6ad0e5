/*
 * CPU oracle for CONCORD-PCD.  TEST INFRASTRUCTURE ONLY: the tests, the smoke
 * check and the benchmark's CPU-baseline leg load this library; the solver
 * never does.  It shares no code with the HIP path.
 *
 * Plain, serial, double-precision restatement of the coordinate-descent
 * methods of Choi, Lee & Yu, "An efficient parallel block coordinate descent
 * algorithm for large-scale precision matrix estimation using graphics
 * processing units" (arXiv 2106.09382):
 *
 *   - CONCORD-CD (Section 2.1): diagonals by eq. (2), then every off-diagonal
 *     by eq. (3), one coordinate at a time, each using the latest values.
 *   - CONCORD-PCD (Section 3, Algorithm 1): the off-diagonals are visited in
 *     p_even - 1 parallel steps given by the circle-method round-robin table
 *     (Section 3.2, steps i-iv); all pairs of a step are updated from the same
 *     iterate; then all diagonals; then the convergence test.
 *   - The same over an arbitrary edge colouring (Section 4).
 *   - Joint estimation of two precision matrices with a fused penalty
 *     (Section 6), by block updates of (omega^1_ij, omega^2_ij) on
 *     Algorithm 1's schedule.
 *
 * Scale: every routine takes S = X^T X / n instead of T = X^T X.  Dividing
 * eqs. (2) and (3) by n gives the same updates with T -> S and the threshold
 * lambda -> lambda / n, so the lambda passed here is the threshold on the S
 * scale (the paper's lambda values 0.1 and 0.3 are on this scale).
 *
 * Numerators are direct sums over the current Omega, exactly as eqs. (2)-(3)
 * write them; there is no maintained product and no reordering of terms.
 *
 * Omega is a dense, symmetric, row-major p x p array; an off-diagonal update
 * writes both omega_ij and omega_ji.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Soft_tau(x) = sign(x) (|x| - tau)_+  (Section 2.1, below eq. (3)).
 * |x| == tau gives exactly zero. */
static double soft(double x, double tau)
{
    double a = fabs(x) - tau;
    if (a <= 0.0)
        return 0.0;
    return x > 0.0 ? a : -a;
}

/* Numerator of eq. (3) before the sign flip:
 *   b_ij = sum_{u != j} omega_iu S_ju + sum_{u != i} omega_uj S_iu.
 * Omega is symmetric, so omega_uj is read from row j. */
static double offdiag_sum(const double *S, const double *om, int p, int i, int j)
{
    const double *oi = om + (size_t)i * p, *oj = om + (size_t)j * p;
    const double *si = S + (size_t)i * p, *sj = S + (size_t)j * p;
    double b1 = 0.0, b2 = 0.0;
    for (int u = 0; u < j; ++u)
        b1 += oi[u] * sj[u];
    for (int u = j + 1; u < p; ++u)
        b1 += oi[u] * sj[u];
    for (int u = 0; u < i; ++u)
        b2 += oj[u] * si[u];
    for (int u = i + 1; u < p; ++u)
        b2 += oj[u] * si[u];
    return b1 + b2;
}

/* Eq. (3): omega_ij <- Soft_lambda(-b_ij) / (S_ii + S_jj). */
static double offdiag_new(const double *S, const double *om, int p, int i, int j, double lam)
{
    double b = offdiag_sum(S, om, p, i, j);
    return soft(-b, lam) / (S[(size_t)i * p + i] + S[(size_t)j * p + j]);
}

/* Eq. (2): with c = sum_{j != i} omega_ij S_ij,
 *   omega_ii <- (-c + sqrt(c^2 + 4 S_ii)) / (2 S_ii).
 * (T -> S turns 4 n T_ii into 4 S_ii after dividing by n^2 under the root.) */
static double diag_new(const double *S, const double *om, int p, int i)
{
    const double *oi = om + (size_t)i * p, *si = S + (size_t)i * p;
    double c = 0.0;
    for (int u = 0; u < i; ++u)
        c += oi[u] * si[u];
    for (int u = i + 1; u < p; ++u)
        c += oi[u] * si[u];
    double sii = si[i];
    return (-c + sqrt(c * c + 4.0 * sii)) / (2.0 * sii);
}

static int check_inputs(const double *S, int p, double lam, double tol, int maxit)
{
    if (!S || p < 1 || !(lam >= 0.0) || !(tol > 0.0) || maxit < 1)
        return -1;
    for (int i = 0; i < p; ++i)
        if (!(S[(size_t)i * p + i] > 0.0))
            return -3;
    return 0;
}

static void start_point(double *om, const double *omega0, int p)
{
    if (omega0) {
        memcpy(om, omega0, sizeof(double) * (size_t)p * p);
    } else {
        memset(om, 0, sizeof(double) * (size_t)p * p);
        for (int i = 0; i < p; ++i)
            om[(size_t)i * p + i] = 1.0;
    }
}

static long long count_upper(const double *om, int p)
{
    long long k = 0;
    for (int i = 0; i < p; ++i)
        for (int j = i + 1; j < p; ++j)
            k += om[(size_t)i * p + j] != 0.0;
    return k;
}

/* Exported single-coordinate updates, for spot checks of a solution. */
double oracle_offdiag_update(const double *S, const double *om, int p, int i, int j, double lam)
{
    return offdiag_new(S, om, p, i, j, lam);
}

double oracle_diag_update(const double *S, const double *om, int p, int i)
{
    return diag_new(S, om, p, i);
}

/*
 * Round-robin table of Section 3.2 / Algorithm 1, from the geometry of the
 * circle method.  The first index (vertex 0 here) stays at the centre; the
 * other m = pe - 1 vertices sit on a circle of m seats, vertex v on seat
 * v - 1 at the start.  The table pairs the centre with the vertex on the
 * seat that faces it (the axis), and every other vertex with its mirror
 * image across the axis.  Each step turns the circle by one seat, so the
 * axis moves one seat back: at step k it is seat c = m - 1 - k (mod m).
 * Slot 0 is (centre, axis vertex); slot q >= 1 is the mirror pair q seats
 * either side of the axis, the seat c + q first (the order in which the
 * target set of step (ii) lists its pairs).
 *
 * Output: pairs[(k * H + q) * 2 + {0,1}] for step k in [0, pe-1), slot q in
 * [0, pe/2), as 0-based vertex numbers.  For odd p the value p is the
 * paper's dummy index p+1 (a pair holding it is discarded, step iii).
 * Returns the number of steps, or -1 for p < 1.
 */
int oracle_round_robin(int p, int32_t *pairs)
{
    if (p < 1)
        return -1;
    int pe = p + (p & 1), H = pe / 2, m = pe - 1;
    /* seat[s] = vertex on seat s before any turn */
    int *seat = (int *)malloc(sizeof(int) * (m > 0 ? m : 1));
    for (int s = 0; s < m; ++s)
        seat[s] = s + 1;
    for (int k = 0; k < m; ++k) {
        int axis = ((m - 1 - k) % m + m) % m;
        int32_t *out = pairs + (size_t)k * H * 2;
        out[0] = 0;
        out[1] = seat[axis];
        for (int q = 1; q < H; ++q) {
            out[2 * q + 0] = seat[(axis + q) % m];
            out[2 * q + 1] = seat[(axis - q + m) % m];
        }
    }
    free(seat);
    return m;
}

/*
 * CONCORD-PCD, Algorithm 1.
 *
 *   S       p x p sample Gram matrix X^T X / n (symmetric, S_ii > 0)
 *   lam     threshold on the S scale
 *   tol     stop when delta < tol, delta = max |change| over all entries of
 *           the sweep (diagonal included), i.e. |Omega^(t) - Omega^(t-1)|_inf
 *   maxit   sweep limit
 *   omega0  start point (p x p) or NULL for the identity
 *   omega   out, p x p
 *   colour_limit  if > 0, stop after that many parallel off-diagonal steps in
 *           total (possibly mid-sweep, before that sweep's diagonal step); used
 *           to time a bounded sample and to watch the objective step by step
 *   serial  0: each step computes all its new values from the same iterate
 *           and then writes them (the parallel step of Algorithm 1);
 *           1: writes each pair as soon as it is computed, in slot order
 *   delta_trace  optional, maxit entries: delta of each sweep
 *   info    out [0] sweeps, [1] last delta, [2] converged (1/0),
 *           [3] nonzeros above the diagonal, [4] parallel steps done
 *
 * Returns 0 on success, -1 on invalid arguments, -3 when some S_ii <= 0.
 */
int oracle_pcd(const double *S, int p, double lam, double tol, int maxit,
               const double *omega0, double *omega, long long colour_limit,
               int serial, double *delta_trace, double *info)
{
    int rc = check_inputs(S, p, lam, tol, maxit);
    if (rc)
        return rc;
    int pe = p + (p & 1), H = pe / 2, m = pe - 1;
    int32_t *tab = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * H * 2 + 8);
    double *nv = (double *)malloc(sizeof(double) * (H + 1));
    double *od = (double *)malloc(sizeof(double) * p);
    start_point(omega, omega0, p);
    oracle_round_robin(p, tab);

    int t = 0, converged = 0;
    double delta = 0.0;
    long long steps = 0;
    int stopped = 0;
    while (!stopped && t < maxit) {
        ++t;
        delta = 0.0;
        for (int k = 0; k < m; ++k) {
            const int32_t *pr = tab + (size_t)k * H * 2;
            if (serial) {
                for (int q = 0; q < H; ++q) {
                    int a = pr[2 * q], b = pr[2 * q + 1];
                    if (a == p || b == p)
                        continue;
                    double w = offdiag_new(S, omega, p, a, b, lam);
                    double d = fabs(w - omega[(size_t)a * p + b]);
                    if (d > delta)
                        delta = d;
                    omega[(size_t)a * p + b] = w;
                    omega[(size_t)b * p + a] = w;
                }
            } else {
                for (int q = 0; q < H; ++q) {
                    int a = pr[2 * q], b = pr[2 * q + 1];
                    nv[q] = (a == p || b == p) ? 0.0 : offdiag_new(S, omega, p, a, b, lam);
                }
                for (int q = 0; q < H; ++q) {
                    int a = pr[2 * q], b = pr[2 * q + 1];
                    if (a == p || b == p)
                        continue;
                    double d = fabs(nv[q] - omega[(size_t)a * p + b]);
                    if (d > delta)
                        delta = d;
                    omega[(size_t)a * p + b] = nv[q];
                    omega[(size_t)b * p + a] = nv[q];
                }
            }
            ++steps;
            if (colour_limit > 0 && steps >= colour_limit) {
                stopped = 1;
                break;
            }
        }
        if (stopped)
            break;
        /* Diagonal step: every c_i is taken from the post-step Omega; the
         * diagonals do not enter one another's update, so one pass suffices. */
        for (int i = 0; i < p; ++i)
            od[i] = diag_new(S, omega, p, i);
        for (int i = 0; i < p; ++i) {
            double d = fabs(od[i] - omega[(size_t)i * p + i]);
            if (d > delta)
                delta = d;
            omega[(size_t)i * p + i] = od[i];
        }
        if (delta_trace)
            delta_trace[t - 1] = delta;
        if (delta < tol) {
            converged = 1;
            break;
        }
    }
    if (info) {
        info[0] = t;
        info[1] = delta;
        info[2] = converged;
        info[3] = (double)count_upper(omega, p);
        info[4] = (double)steps;
    }
    free(tab);
    free(nv);
    free(od);
    return 0;
}

/*
 * CONCORD-PCD over a given edge colouring (Section 4: the construction of
 * Theorem 2's update order extends to any edge colouring).  Colour c holds
 * the pairs pairs[2 e], pairs[2 e + 1] for e in [colour_start[c],
 * colour_start[c + 1]), 0-based, each colour a matching.  A sweep updates the
 * pairs of colour 0, 1, ..., ncol - 1 in that order, all pairs of a colour
 * from the same Omega (Lemma 2), then the diagonal step.  Pairs in no colour
 * keep their value.  delta, stopping rule, info and return codes as for
 * oracle_pcd (info[4] counts colour steps).
 */
int oracle_pcd_colouring(const double *S, int p, double lam, double tol, int maxit,
                         const double *omega0, double *omega, const int32_t *pairs,
                         const int32_t *colour_start, int ncol, double *delta_trace,
                         double *info)
{
    int rc = check_inputs(S, p, lam, tol, maxit);
    if (rc)
        return rc;
    if (ncol < 0 || (ncol > 0 && (!pairs || !colour_start)))
        return -1;
    int widest = 0;
    for (int c = 0; c < ncol; ++c) {
        int w = colour_start[c + 1] - colour_start[c];
        if (w < 0)
            return -1;
        if (w > widest)
            widest = w;
    }
    double *nv = (double *)malloc(sizeof(double) * (widest + 1));
    double *od = (double *)malloc(sizeof(double) * p);
    start_point(omega, omega0, p);
    int t = 0, converged = 0;
    double delta = 0.0;
    long long steps = 0;
    while (t < maxit) {
        ++t;
        delta = 0.0;
        for (int c = 0; c < ncol; ++c) {
            int e0 = colour_start[c], e1 = colour_start[c + 1];
            for (int e = e0; e < e1; ++e)
                nv[e - e0] = offdiag_new(S, omega, p, pairs[2 * e], pairs[2 * e + 1], lam);
            for (int e = e0; e < e1; ++e) {
                int a = pairs[2 * e], b = pairs[2 * e + 1];
                double d = fabs(nv[e - e0] - omega[(size_t)a * p + b]);
                if (d > delta)
                    delta = d;
                omega[(size_t)a * p + b] = nv[e - e0];
                omega[(size_t)b * p + a] = nv[e - e0];
            }
            ++steps;
        }
        for (int i = 0; i < p; ++i)
            od[i] = diag_new(S, omega, p, i);
        for (int i = 0; i < p; ++i) {
            double d = fabs(od[i] - omega[(size_t)i * p + i]);
            if (d > delta)
                delta = d;
            omega[(size_t)i * p + i] = od[i];
        }
        if (delta_trace)
            delta_trace[t - 1] = delta;
        if (delta < tol) {
            converged = 1;
            break;
        }
    }
    if (info) {
        info[0] = t;
        info[1] = delta;
        info[2] = converged;
        info[3] = (double)count_upper(omega, p);
        info[4] = (double)steps;
    }
    free(nv);
    free(od);
    return 0;
}

/*
 * CONCORD-CD (Section 2.1): each sweep updates the p diagonals by eq. (2),
 * then the p(p-1)/2 off-diagonals by eq. (3) in lexicographic order
 * (1,2), (1,3), ..., (p-1,p); every update uses the latest values.
 * Arguments and return codes as for oracle_pcd (no colour limit; info[4] is
 * the number of single-coordinate updates done).
 */
int oracle_cd(const double *S, int p, double lam, double tol, int maxit,
              const double *omega0, double *omega, double *delta_trace, double *info)
{
    int rc = check_inputs(S, p, lam, tol, maxit);
    if (rc)
        return rc;
    start_point(omega, omega0, p);
    int t = 0, converged = 0;
    double delta = 0.0;
    long long updates = 0;
    while (t < maxit) {
        ++t;
        delta = 0.0;
        for (int i = 0; i < p; ++i) {
            double w = diag_new(S, omega, p, i);
            double d = fabs(w - omega[(size_t)i * p + i]);
            if (d > delta)
                delta = d;
            omega[(size_t)i * p + i] = w;
            ++updates;
        }
        for (int i = 0; i < p; ++i) {
            for (int j = i + 1; j < p; ++j) {
                double w = offdiag_new(S, omega, p, i, j, lam);
                double d = fabs(w - omega[(size_t)i * p + j]);
                if (d > delta)
                    delta = d;
                omega[(size_t)i * p + j] = w;
                omega[(size_t)j * p + i] = w;
                ++updates;
            }
        }
        if (delta_trace)
            delta_trace[t - 1] = delta;
        if (delta < tol) {
            converged = 1;
            break;
        }
    }
    if (info) {
        info[0] = t;
        info[1] = delta;
        info[2] = converged;
        info[3] = (double)count_upper(omega, p);
        info[4] = (double)updates;
    }
    return 0;
}

/*
 * Joint estimation of two precision matrices (Section 6, the extension to
 * two populations): the objective, divided by n,
 *
 *   F(Omega_1, Omega_2) = sum_m [ -sum_i log omega^m_ii + 1/2 tr(Omega_m S_m Omega_m) ]
 *                         + lam1 sum_m sum_{i<j} |omega^m_ij|
 *                         + lam2 sum_{i<=j} |omega^1_ij - omega^2_ij|,
 *
 * minimised by block coordinate descent over (omega^1_ij, omega^2_ij).  As a
 * function of that block (every other entry fixed) the objective is, with
 * a_m = S^m_ii + S^m_jj and b_m the eq. (3) numerator of population m,
 *
 *   sum_m [ 1/2 a_m x_m^2 + b_m x_m + lam1 |x_m| ] + lam2 |x_1 - x_2|,
 *
 * strictly convex, so its minimiser is the one point where zero is a
 * subgradient.  If x_1 > x_2 there, the fused term's subgradient is +lam2 and
 * the two coordinates separate: x_1 = Soft_lam1(-(b_1 + lam2)) / a_1,
 * x_2 = Soft_lam1(-(b_2 - lam2)) / a_2; conversely, if these values satisfy
 * x_1 > x_2 they satisfy the optimality conditions.  The same holds for
 * x_1 < x_2 with lam2 negated.  Otherwise the minimiser has x_1 = x_2 = t and
 * minimises the objective along that line:
 * t = Soft_{2 lam1}(-(b_1 + b_2)) / (a_1 + a_2).
 *
 * The diagonal block (omega^1_ii, omega^2_ii) has the same structure with
 * the smooth part -log y_m + 1/2 S^m_ii y_m^2 + c_m y_m (c_m the eq. (2) sum)
 * and no lam1 term: a separated coordinate is the positive root of
 * S^m_ii y^2 + (c_m +- lam2) y - 1 = 0, and the fused value the positive root
 * of (S^1_ii + S^2_ii) t^2 + (c_1 + c_2) t - 2 = 0.
 */

/* Positive root of s y^2 + c y - 1 = 0 (eq. (2)'s formula). */
static double diag_root(double s, double c)
{
    return (-c + sqrt(c * c + 4.0 * s)) / (2.0 * s);
}

/* c_i = sum_{j != i} omega_ij S_ij (the sum of eq. (2)). */
static double diag_sum(const double *S, const double *om, int p, int i)
{
    const double *oi = om + (size_t)i * p, *si = S + (size_t)i * p;
    double c = 0.0;
    for (int u = 0; u < i; ++u)
        c += oi[u] * si[u];
    for (int u = i + 1; u < p; ++u)
        c += oi[u] * si[u];
    return c;
}

static void joint_pair(double a1, double b1, double a2, double b2, double lam1, double lam2,
                       double *x1, double *x2)
{
    double u1 = soft(-(b1 + lam2), lam1) / a1, u2 = soft(-(b2 - lam2), lam1) / a2;
    if (u1 > u2) {
        *x1 = u1;
        *x2 = u2;
        return;
    }
    double v1 = soft(-(b1 - lam2), lam1) / a1, v2 = soft(-(b2 + lam2), lam1) / a2;
    if (v1 < v2) {
        *x1 = v1;
        *x2 = v2;
        return;
    }
    double t = soft(-(b1 + b2), 2.0 * lam1) / (a1 + a2);
    *x1 = t;
    *x2 = t;
}

static void joint_diag(double s1, double c1, double s2, double c2, double lam2, double *y1,
                       double *y2)
{
    double u1 = diag_root(s1, c1 + lam2), u2 = diag_root(s2, c2 - lam2);
    if (u1 > u2) {
        *y1 = u1;
        *y2 = u2;
        return;
    }
    double v1 = diag_root(s1, c1 - lam2), v2 = diag_root(s2, c2 + lam2);
    if (v1 < v2) {
        *y1 = v1;
        *y2 = v2;
        return;
    }
    /* positive root of (s1 + s2) t^2 + (c1 + c2) t - 2 = 0 */
    double t = (-(c1 + c2) + sqrt((c1 + c2) * (c1 + c2) + 8.0 * (s1 + s2))) / (2.0 * (s1 + s2));
    *y1 = t;
    *y2 = t;
}

/* Exported block updates, for pins against brute force. */
void oracle_joint_pair(double a1, double b1, double a2, double b2, double lam1, double lam2,
                       double *out)
{
    joint_pair(a1, b1, a2, b2, lam1, lam2, &out[0], &out[1]);
}

void oracle_joint_diag(double s1, double c1, double s2, double c2, double lam2, double *out)
{
    joint_diag(s1, c1, s2, c2, lam2, &out[0], &out[1]);
}

/*
 * Joint CONCORD-PCD: Algorithm 1's schedule with the block update above in
 * place of eq. (3) and eq. (2).  Pairs of one step share no vertex, so their
 * blocks do not involve one another (the paper's remark on disjoint edge
 * indices) and every block of a step is computed from the same iterate; then
 * the diagonal blocks, every c taken from the post-step matrices.  delta is
 * the max |change| over both matrices and the whole sweep.
 *
 *   S1, S2          p x p Gram matrices of the two populations
 *   omega0_1/_2     start points or NULL (identity)
 *   omega1, omega2  out, p x p
 *   info            out [0] sweeps, [1] last delta, [2] converged,
 *                   [3] nonzeros above the diagonal of Omega_1, [4] of Omega_2,
 *                   [5] pairs i<j with omega^1_ij != omega^2_ij
 * Returns 0, -1 on invalid arguments, -3 when some S^m_ii <= 0.
 */
int oracle_joint_pcd(const double *S1, const double *S2, int p, double lam1, double lam2,
                     double tol, int maxit, const double *omega0_1, const double *omega0_2,
                     double *omega1, double *omega2, double *delta_trace, double *info)
{
    int rc = check_inputs(S1, p, lam1, tol, maxit);
    if (!rc)
        rc = check_inputs(S2, p, lam1, tol, maxit);
    if (rc)
        return rc;
    if (!(lam2 >= 0.0))
        return -1;
    int pe = p + (p & 1), H = pe / 2, m = pe - 1;
    int32_t *tab = (int32_t *)malloc(sizeof(int32_t) * (size_t)m * H * 2 + 8);
    double *nv = (double *)malloc(sizeof(double) * 2 * (H + 1));
    double *od = (double *)malloc(sizeof(double) * 2 * p);
    start_point(omega1, omega0_1, p);
    start_point(omega2, omega0_2, p);
    oracle_round_robin(p, tab);

    int t = 0, converged = 0;
    double delta = 0.0;
    while (t < maxit) {
        ++t;
        delta = 0.0;
        for (int k = 0; k < m; ++k) {
            const int32_t *pr = tab + (size_t)k * H * 2;
            for (int q = 0; q < H; ++q) {
                int i = pr[2 * q], j = pr[2 * q + 1];
                if (i == p || j == p)
                    continue;
                double a1 = S1[(size_t)i * p + i] + S1[(size_t)j * p + j];
                double a2 = S2[(size_t)i * p + i] + S2[(size_t)j * p + j];
                joint_pair(a1, offdiag_sum(S1, omega1, p, i, j), a2,
                           offdiag_sum(S2, omega2, p, i, j), lam1, lam2, &nv[2 * q],
                           &nv[2 * q + 1]);
            }
            for (int q = 0; q < H; ++q) {
                int i = pr[2 * q], j = pr[2 * q + 1];
                if (i == p || j == p)
                    continue;
                double d1 = fabs(nv[2 * q] - omega1[(size_t)i * p + j]);
                double d2 = fabs(nv[2 * q + 1] - omega2[(size_t)i * p + j]);
                if (d1 > delta)
                    delta = d1;
                if (d2 > delta)
                    delta = d2;
                omega1[(size_t)i * p + j] = omega1[(size_t)j * p + i] = nv[2 * q];
                omega2[(size_t)i * p + j] = omega2[(size_t)j * p + i] = nv[2 * q + 1];
            }
        }
        for (int i = 0; i < p; ++i)
            joint_diag(S1[(size_t)i * p + i], diag_sum(S1, omega1, p, i), S2[(size_t)i * p + i],
                       diag_sum(S2, omega2, p, i), lam2, &od[2 * i], &od[2 * i + 1]);
        for (int i = 0; i < p; ++i) {
            double d1 = fabs(od[2 * i] - omega1[(size_t)i * p + i]);
            double d2 = fabs(od[2 * i + 1] - omega2[(size_t)i * p + i]);
            if (d1 > delta)
                delta = d1;
            if (d2 > delta)
                delta = d2;
            omega1[(size_t)i * p + i] = od[2 * i];
            omega2[(size_t)i * p + i] = od[2 * i + 1];
        }
        if (delta_trace)
            delta_trace[t - 1] = delta;
        if (delta < tol) {
            converged = 1;
            break;
        }
    }
    if (info) {
        long long diff = 0;
        for (int i = 0; i < p; ++i)
            for (int j = i + 1; j < p; ++j)
                diff += omega1[(size_t)i * p + j] != omega2[(size_t)i * p + j];
        info[0] = t;
        info[1] = delta;
        info[2] = converged;
        info[3] = (double)count_upper(omega1, p);
        info[4] = (double)count_upper(omega2, p);
        info[5] = (double)diff;
    }
    free(tab);
    free(nv);
    free(od);
    return 0;
}
