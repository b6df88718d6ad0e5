/*
 * concord.h -- C ABI of the MI355X CONCORD-PCD solver.
 *
 * Solves the CONCORD problem (Choi, Lee & Yu, arXiv 2106.09382, Section 2.1,
 * eq. (1)) by the edge-coloured parallel coordinate descent of Algorithm 1
 * (Section 3): each sweep runs the p_even - 1 colour classes of the
 * circle-method 1-factorisation of K_p (Section 3.2), updating all pairs of a
 * class at once by eq. (3), then all diagonals by eq. (2), then the test
 * |Omega^(t) - Omega^(t-1)|_inf < tol.
 *
 * Scale convention: the library works on S = X^T X / n (not T = X^T X) and
 * `lambda` is the soft-threshold on that scale, i.e. the paper's updates with
 * T = nS and threshold n*lambda.  The objective minimised is
 *   F(Omega) = -sum_i log omega_ii + 1/2 tr(Omega S Omega) + lambda sum_{i<j} |omega_ij|.
 *
 * Conventions shared by every entry point:
 *  - Matrices are dense, row-major, contiguous, in device memory of the
 *    current HIP device, with element type given by `dt`.  Symmetric inputs
 *    are used as given (no symmetrisation, no check).
 *  - The caller owns all input and output buffers.  The library allocates its
 *    workspace stream-ordered on `stream` and releases it before returning.
 *  - Calls are stream-ordered and return after the work on `stream` has
 *    completed, so host-side outputs (`info`) are valid on return.  `stream`
 *    NULL means the default stream.  Calls on distinct streams may run
 *    concurrently.
 *  - Errors are returned as codes (never thrown).  On a negative code the
 *    outputs are unspecified; CONCORD_NOT_CONVERGED still returns the last
 *    iterate.
 */
#ifndef CONCORD_H
#define CONCORD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { CONCORD_F32 = 0, CONCORD_F64 = 1 } concord_dtype;
typedef enum { CONCORD_INPUT_S = 0, CONCORD_INPUT_Y = 1 } concord_input;

enum {
    CONCORD_OK = 0,
    CONCORD_NOT_CONVERGED = 1, /* maxit sweeps done; Omega is the last iterate */
    CONCORD_EINVAL = -1,       /* bad argument (sizes, pointers, lambda, tol, maxit, dtype) */
    CONCORD_ENONFINITE = -2,   /* S (or Y) holds NaN/Inf, or the iteration left the finite range */
    CONCORD_ENOTPD = -3,       /* some S_ii <= 0: eq. (2) and eq. (3) divide by S_ii */
    CONCORD_ENOMEM = -4,       /* workspace allocation failed */
    CONCORD_EDEVICE = -5,      /* HIP runtime error, or a device wait ran past its bound */
    CONCORD_ELAUNCH = -6,      /* launch shape cannot be made co-resident on this device */
    CONCORD_ESCRATCH = -7      /* concord_fit_noalloc: workspace larger than its fixed scratch */
};

/* Result of one solve. */
typedef struct {
    int32_t sweeps;     /* outer iterations t performed (the sweep that met the test counts) */
    int32_t status;     /* CONCORD_OK or CONCORD_NOT_CONVERGED, or a negative code */
    double delta;       /* |Omega^(t) - Omega^(t-1)|_inf of the last sweep, diagonal included */
    double tol_eff;     /* tolerance applied: tol in FP64; max(tol, 16 eps_f32 max_i omega_ii) in FP32 */
    int64_t nnz_upper;  /* #{i < j : omega_ij != 0} */
    double objective;   /* F(Omega) at the returned Omega (from the maintained product) */
    double elapsed_ms;  /* device time of the call (Gram, set-up, sweeps, output) */
    double gram_ms;     /* device time of the Gram kernel (CONCORD_INPUT_Y), else 0 */
    double sweep_ms;    /* device time of the persistent sweep kernel (all sweeps) */
    int64_t moved_pairs;/* sum over sweeps of the number of pairs i<j whose omega_ij changed */
    int64_t moved_diag; /* sum over sweeps of the number of diagonals that changed */
    int32_t row_groups; /* launch shape used: workgroups sharing out the rows of W */
    int32_t col_slices; /*   ... and the columns */
    int32_t w_in_lds;   /*   1 if W blocks were held in LDS */
    int32_t block_threads;
    int32_t pending_depth; /* row updates held back before a row of W is rewritten */
    int32_t active_sweeps; /* active-set mode: sweeps over the support's colouring */
} concord_info;

/* Launch/tuning options; zero-initialise for defaults. */
typedef struct {
    int32_t row_groups;     /* workgroups sharing out the rows of W (0 = auto) */
    int32_t col_slices;     /* workgroups sharing out the columns of W (0 = auto) */
    /* Threads per workgroup, a multiple of 64: up to 512; or, with W in HBM
     * and one row of W per thread, up to 1024 in FP32 and 768 in FP64 (the
     * waves that hold no rows rewrite rows in the background; more of them
     * finish a burst of rewrites sooner).  Wider requests, and wide ones with
     * w_in_lds = 1, are CONCORD_EINVAL; p above row_groups x block_threads
     * with a wide workgroup is CONCORD_ELAUNCH.  0 = auto: the widest (1024
     * in FP32, 768 in FP64) with W in HBM when the rows fill at most half of
     * its waves, else 512 (256 for a single workgroup). */
    int32_t block_threads;
    int32_t w_in_lds;       /* -1/0 = auto, 1 = force W blocks in LDS, 2 = force W in HBM */
    /* 0 = auto (2 with W in LDS; 8 with W in HBM, 5 in FP32 wide workgroups),
     * else 2..8: updates a row holds before it is rewritten */
    int32_t pending_depth;
    double *delta_trace;    /* optional host array of maxit entries: delta of every sweep */
    /* Optional device array of workgroups x timestamp_steps x 3 words: for
     * each of the first timestamp_steps colour steps, thread 0 of every
     * workgroup stores the 100 MHz device clock at the step's start, when its
     * rows are done, and when its row rewrites are done.  Query the launch
     * shape first (a call with the same options returns it in concord_info). */
    uint64_t *device_timestamps;
    int32_t timestamp_steps;
    /* Row rewrites (W in HBM): 0 = automatic (in the background, on the waves
     * that hold no rows, during the next step, when such waves exist and the
     * pending depth is at least 4), 1 = always right after their step. */
    int32_t sync_rewrites;
    /* Optional device p x p array (element type dt): receives the maintained
     * product W = Omega S as the solve leaves it (for checks). */
    void *w_out;
    /* Active-set sweeps (the construction of Theorem 2 with another edge
     * colouring, Section 4): 1 = after each full sweep of Algorithm 1 that has
     * not converged, colour the support of Omega greedily and sweep over
     * those colours (then the diagonal) until their delta < tol or
     * active_maxit sweeps (0 = 3); only full sweeps decide convergence
     * and count in info->sweeps and maxit.  0 = plain Algorithm 1. */
    int32_t active_set;
    int32_t active_maxit;
} concord_options;

/*
 * concord_fit -- one CONCORD-PCD solve (Algorithm 1).
 *   kind    CONCORD_INPUT_S: X is S, p x p symmetric with S_ii > 0.
 *           CONCORD_INPUT_Y: X is the n x p data matrix Y; the library forms
 *           S = Y^T Y / n on the device (no centring or scaling).
 *   n       rows of Y (ignored for CONCORD_INPUT_S)
 *   p       number of variables, >= 1 (p_even = p + (p mod 2), p_even - 1 colours)
 *   lambda  soft-threshold on the S scale, finite, >= 0
 *   tol     stop when delta < tol (strict), tol > 0
 *   maxit   sweep limit, >= 1
 *   dt      element type of X, omega0 and omega; the iteration runs in it
 *   omega0  start point, p x p symmetric with positive diagonal, or NULL for
 *           the identity (Algorithm 1's Omega^(0))
 *   omega   out, p x p; both triangles written (identical)
 *   info    out (host pointer, may be NULL)
 *   stream  hipStream_t or NULL
 * Returns CONCORD_OK, CONCORD_NOT_CONVERGED or a negative code.
 */
int concord_fit(concord_input kind, const void *X, int64_t n, int64_t p, double lambda,
                double tol, int32_t maxit, concord_dtype dt, const void *omega0, void *omega,
                concord_info *info, void *stream);

/* Bytes of the fixed device scratch that concord_fit_noalloc works in. */
#define CONCORD_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/*
 * concord_fit_noalloc -- concord_fit for callers that cannot allocate device
 * memory (code under stream capture, serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, same kernels and launch shape, same results
 * bit for bit.  The workspace (W = Omega S, the sweep layout of Omega, the
 * published entries, barrier and reduction words, and S itself when the
 * input is Y) is carved from one fixed array of CONCORD_NOALLOC_SCRATCH_BYTES
 * in device memory, which every device the library runs on holds from its
 * first call there until the process ends.  The call allocates no device
 * memory and creates no events: info's device times (elapsed_ms, gram_ms,
 * sweep_ms) read 0.  Everything the solve needs zeroed is cleared by its own
 * kernels, so a call never depends on what the previous one left.
 *   Returns CONCORD_ESCRATCH, before any device work, when the solve needs
 *   more than the scratch.  With the default launch shape on a 256-CU
 *   device that allows p <= 1280 from S and p <= 1152 from Y in FP64,
 *   p <= 1792 and p <= 1664 in FP32.
 * All calls on one device share its scratch: calls that overlap in time on
 * the same device (two host threads, or two streams) race and must be
 * serialised by the caller.  The call still synchronises `stream` before
 * returning, as concord_fit does.
 */
int concord_fit_noalloc(concord_input kind, const void *X, int64_t n, int64_t p, double lambda,
                        double tol, int32_t maxit, concord_dtype dt, const void *omega0,
                        void *omega, concord_info *info, void *stream);

/* concord_fit with explicit launch options (opts may be NULL = defaults). */
int concord_fit_ex(concord_input kind, const void *X, int64_t n, int64_t p, double lambda,
                   double tol, int32_t maxit, concord_dtype dt, const void *omega0, void *omega,
                   concord_info *info, void *stream, const concord_options *opts);

/* Launch options of the batched solver (all 0 = defaults). */
typedef struct {
    int32_t workgroups;     /* workgroups of one launch (0 = one per compute unit); at most
                               one per compute unit above 256 threads, two at 256 or fewer */
    /* Threads per workgroup, a multiple of 64: up to 512, each thread holding
     * up to two rows of W; or wide workgroups, up to 1024 in FP32 and 768 in
     * FP64, each thread holding one row (more problems then leave half of
     * their waves to background rewrites).  0 = 1024 in FP32, 512 in FP64.
     * R = rows a workgroup holds: 2 x block_threads up to 512 threads,
     * block_threads above. */
    int32_t block_threads;
    int32_t pending_depth;  /* 2..8 row updates held before a row is rewritten (0 = 8) */
    int32_t cols_per_lane;  /* columns of W each lane carries in a row rewrite: 2 or 4 (0 = 4) */
    /* Optional host array of B workgroup counts, one per problem (each at
     * least ceil(p_b / R) row groups' worth and at most
     * p_b, summing to at most `workgroups`): all problems then share one
     * launch with these counts instead of the built-in plan.  NULL = built-in
     * plan. */
    const int32_t *problem_workgroups;
    /* Optional host array of B column-slice counts (requires
     * problem_workgroups): problem b's problem_workgroups[b] workgroups form
     * a grid of problem_workgroups[b] / c_b row groups x c_b column slices,
     * each workgroup holding its row group's rows of W in one slice of the
     * columns (c_b must divide the workgroup count, be <= p_b, and leave
     * ceil(p_b / row groups) <= R).  NULL = one slice each. */
    const int32_t *problem_col_slices;
    /* 1 = row rewrites right after their step, as concord_options.sync_rewrites */
    int32_t sync_rewrites;
    int32_t reserved;
} concord_batch_options;

/*
 * concord_fit_batched -- B independent CONCORD-PCD solves, each along a path
 * of L values of lambda, in one persistent launch (more launches, in order,
 * only when the problems' minimum workgroup counts exceed one launch).
 * Problem b runs lambdas[b * L + 0], ..., lambdas[b * L + L - 1] in that
 * order; the first starts from the identity (Algorithm 1's Omega^(0)), each
 * later one from the Omega the previous one left (a warm start, as on a
 * regularisation path).  Every lambda gets its own convergence test and
 * maxit budget.
 *   B          number of problems, >= 1
 *   kind       as for concord_fit, for all problems
 *   X          host array of B device pointers: S_b (p_b x p_b) or Y_b (n_b x p_b)
 *   n          host array of B row counts (CONCORD_INPUT_Y; may be NULL for S)
 *   p          host array of B sizes, each >= 1 (mixed sizes and parities allowed)
 *   L          path length, >= 1 (L * maxit <= 2^24)
 *   lambdas    host array B x L, each finite and >= 0 (any order; descending
 *              is the usual path)
 *   tol, maxit, dt   as for concord_fit
 *   omega      host array of B x L device pointers: omega[b * L + l] receives
 *              the p_b x p_b Omega at lambdas[b * L + l]
 *   info       host array of B x L records (may be NULL): per lambda its
 *              sweeps, status, delta, tol_eff, nnz_upper, objective, moved
 *              counts and sweep_ms, the device time this lambda took;
 *              elapsed_ms (the whole call) and gram_ms (the set-up before the
 *              persistent launch) are those of the launch it ran in; row_groups
 *              is the number of workgroups the problem had
 * Returns the first negative per-solve status, else CONCORD_NOT_CONVERGED if
 * any lambda stopped at maxit, else CONCORD_OK; info[].status has each one.
 * Buffers of the batch must not overlap; the call returns after the stream's
 * work completes.
 */
int concord_fit_batched(int32_t B, concord_input kind, const void *const *X, const int64_t *n,
                        const int64_t *p, int32_t L, const double *lambdas, double tol,
                        int32_t maxit, concord_dtype dt, void *const *omega, concord_info *info,
                        void *stream);

/* concord_fit_batched with launch options (opts may be NULL = defaults). */
int concord_fit_batched_ex(int32_t B, concord_input kind, const void *const *X, const int64_t *n,
                           const int64_t *p, int32_t L, const double *lambdas, double tol,
                           int32_t maxit, concord_dtype dt, void *const *omega,
                           concord_info *info, void *stream, const concord_batch_options *opts);

/* Result of one joint solve (concord_fit_joint). */
typedef struct {
    int32_t sweeps;         /* sweeps performed (the sweep that met the test counts) */
    int32_t status;         /* CONCORD_OK, CONCORD_NOT_CONVERGED or a negative code */
    double delta;           /* max |change| over both matrices in the last sweep */
    double tol_eff;         /* tolerance applied (as in concord_info) */
    int64_t nnz_upper[2];   /* #{i < j : omega^m_ij != 0} for m = 1, 2 */
    int64_t differ_upper;   /* #{i < j : omega^1_ij != omega^2_ij} */
    double objective;       /* the joint objective F(Omega_1, Omega_2) at the output */
    double elapsed_ms;      /* device time of the call */
    double gram_ms;         /* device time of the two Gram kernels (CONCORD_INPUT_Y), else 0 */
    double sweep_ms;        /* device time of the persistent sweep kernel */
    int64_t moved_pairs;    /* over sweeps and both populations: pairs i<j whose entry changed */
    int64_t moved_diag;     /* ... and diagonals */
    int32_t row_groups;     /* launch shape of each population: workgroups over rows of W */
    int32_t col_slices;     /*   ... and over columns (2 row_groups col_slices in all) */
    int32_t w_in_lds;
    int32_t block_threads;
    int32_t pending_depth;
    int32_t reserved;
} concord_joint_info;

/*
 * concord_fit_joint -- joint estimation of two sparse precision matrices
 * that differ little (Section 6 of arXiv 2106.09382), on the S scale:
 *   F(Omega_1, Omega_2) = sum_m [ -sum_i log omega^m_ii + 1/2 tr(Omega_m S_m Omega_m) ]
 *                         + lambda1 sum_m sum_{i<j} |omega^m_ij|
 *                         + lambda2 sum_{i<=j} |omega^1_ij - omega^2_ij|.
 * Block coordinate descent over (omega^1_ij, omega^2_ij) on Algorithm 1's
 * schedule: the pairs of a colour share no vertex, so their blocks are
 * updated at once, each by its exact block minimiser; then every diagonal
 * block (omega^1_ii, omega^2_ii); stop when the largest change over both
 * matrices in a sweep is below tol.  lambda2 = 0 gives two independent
 * CONCORD-PCD solves; a large lambda2 fuses them (both equal the solve on
 * (S_1 + S_2) / 2).
 *   kind, dt   as for concord_fit, for both populations
 *   X1, X2     S_m (p x p) or Y_m (n_m x p) in device memory (may be the same)
 *   n1, n2     rows of Y_1, Y_2 (CONCORD_INPUT_Y)
 *   p          variables, >= 1 (the same in both populations)
 *   lambda1    sparsity threshold on the S scale, finite, >= 0
 *   lambda2    fused threshold on the S scale, finite, >= 0
 *   tol, maxit as for concord_fit
 *   omega0_1, omega0_2  start points (p x p, symmetric, positive diagonal)
 *              or NULL for the identity, each independently
 *   omega1, omega2  out, p x p each, distinct buffers
 *   info       out (host, may be NULL)
 * The launch runs 2 row_groups x col_slices workgroups (by default each
 * population gets half the compute units).  Options (opts may be NULL):
 * row_groups, col_slices, block_threads (wide workgroups here up to 768
 * threads in both precisions; 0 = 768 with W in HBM when the rows fill at
 * most half of the waves, else 512), w_in_lds, pending_depth and delta_trace
 * as for concord_fit_ex; active_set, w_out and device_timestamps must be
 * zero (CONCORD_EINVAL otherwise).
 * Returns CONCORD_OK, CONCORD_NOT_CONVERGED or a negative code.
 */
int concord_fit_joint(concord_input kind, const void *X1, const void *X2, int64_t n1, int64_t n2,
                      int64_t p, double lambda1, double lambda2, double tol, int32_t maxit,
                      concord_dtype dt, const void *omega0_1, const void *omega0_2, void *omega1,
                      void *omega2, concord_joint_info *info, void *stream);

/* concord_fit_joint with explicit launch options (opts may be NULL). */
int concord_fit_joint_ex(concord_input kind, const void *X1, const void *X2, int64_t n1,
                         int64_t n2, int64_t p, double lambda1, double lambda2, double tol,
                         int32_t maxit, concord_dtype dt, const void *omega0_1,
                         const void *omega0_2, void *omega1, void *omega2,
                         concord_joint_info *info, void *stream, const concord_options *opts);

/*
 * concord_backward -- implicit gradient of the estimate (for training losses
 * and lambda tuning through a fit).  Given Omega-hat = concord_fit(S, lam)
 * and C = dL/dOmega-hat, returns dL/dS and dL/dlam.
 *
 * At Omega-hat the stationarity conditions of eq. (1) on the free entries
 * (the diagonal, and the pairs i < j with omega_ij != 0; the others stay 0
 * under small changes) are R_ii = (Omega S)_ii - 1/omega_ii = 0 and
 * R_ij = (Omega S)_ij + (Omega S)_ji + lam sign(omega_ij) = 0.  The adjoint
 * system J^T v = dL/dtheta (J = dR/dtheta, symmetric) is solved by coloured
 * Gauss-Seidel sweeps on the schedule of Algorithm 1 (pairs of a colour are
 * independent, as in Lemma 2); then
 *   dL/dS   = -(Omega V + V Omega) / 2   (V: v as a symmetric matrix),
 *   dL/dlam = -sum_{i<j free} v_ij sign(omega_ij).
 * The system does not involve lam itself.
 *   S           p x p device matrix the fit used (S_ii > 0)
 *   omega_hat   p x p device matrix, the fit's output (symmetric, omega_ii > 0)
 *   grad_omega  p x p device matrix dL/dOmega-hat (any matrix; omega_ij and
 *               omega_ji are one unknown, so C_ij + C_ji is what counts)
 *   grad_S      out, p x p device matrix, the symmetric gradient: dL =
 *               sum_ab grad_S_ab dS_ab for every symmetric change dS
 *   grad_lambda out, host pointer (may be NULL)
 *   tol, maxit  Gauss-Seidel stopping rule: max |change of v| over a sweep
 *               < tol (FP32: tol_eff = max(tol, 16 eps max_i |v_ii|)), at
 *               most maxit sweeps
 *   info        out (host, may be NULL): sweeps, status, delta, tol_eff, times
 * Returns CONCORD_OK, CONCORD_NOT_CONVERGED (outputs from the last sweep), or
 * a negative code (CONCORD_ENOTPD when some omega_ii or S_ii is not positive).
 */
int concord_backward(const void *S, const void *omega_hat, int64_t p, const void *grad_omega,
                     void *grad_S, double *grad_lambda, double tol, int32_t maxit,
                     concord_dtype dt, concord_info *info, void *stream);

/* concord_backward with explicit launch options (opts may be NULL). */
int concord_backward_ex(const void *S, const void *omega_hat, int64_t p, const void *grad_omega,
                        void *grad_S, double *grad_lambda, double tol, int32_t maxit,
                        concord_dtype dt, concord_info *info, void *stream,
                        const concord_options *opts);

/*
 * concord_gram -- S = Y^T Y / n (the T = X^T X of Algorithm 1's set-up, on
 * the S scale), computed with matrix-core (MFMA) instructions.
 *   Y  n x p device matrix, S  p x p device output (both triangles written).
 */
int concord_gram(const void *Y, int64_t n, int64_t p, concord_dtype dt, void *S, void *stream);

/*
 * concord_schedule -- host-side closed form of the round-robin table of
 * Section 3.2 (the target sets I_k of Algorithm 1).  Writes
 * pairs[(k * (p_even/2) + q) * 2 + {0,1}] = 0-based vertices of slot q of
 * colour k, for k < p_even - 1; the value p marks the dummy vertex of odd p
 * (the paper's index p+1; such a slot is idle).  `pairs` is a host buffer of
 * (p_even - 1) * p_even entries.  Returns the number of colours or CONCORD_EINVAL.
 */
int64_t concord_schedule(int64_t p, int32_t *pairs);

/* Static description of a code. */
const char *concord_strerror(int code);

/* Library version string. */
const char *concord_version(void);

#ifdef __cplusplus
}
#endif

#endif /* CONCORD_H */
