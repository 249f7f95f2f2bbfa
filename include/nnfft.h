/*
 * nnfft.h - C ABI of the MI355X (gfx950) NNFFT / fast sinc transform library.
 *
 * Method: Kircheis, Potts, Tasche, "Nonuniform fast Fourier transforms with
 * nonequispaced spatial and frequency data and fast sinc transforms"
 * (arXiv 2107.02671).
 *
 *   NNFFT (Algorithm 2.2): approximates, for frequencies v_k and spatial nodes
 *   x_j in [-1/2, 1/2],
 *        y_j = f(x_j) = sum_{k=0}^{M1-1} f_k exp(-2 pi i N v_k x_j)    (1.2)
 *   by sinh-type window spreading (step 1, (2.12)), division by phi_hat_2
 *   (step 2), a length-N2 FFT (step 3), phi_2 interpolation (step 4) and the
 *   final division by phi_hat_1(N x_j) (Algorithm 2.2, output line).  The
 *   substitution N -> N* = N + ceil(2 m1 / sigma1) of Sec. 2 (after (2.7)) is
 *   always applied, so v_k may fill all of [-1/2, 1/2].
 *
 *   Fast sinc transform (Algorithm 6.1): approximates
 *        h_l = sum_{k=0}^{L1-1} c_k sinc(N pi (b_l - a_k))              (6.2)
 *   by the quadrature sinc(N pi x) = (1/2) int_{-1}^{1} e^{-pi i N t x} dt
 *   (Sec. 5), an NNFFT, a multiplication by the quadrature weights and a
 *   second NNFFT.
 *
 * Conventions for every entry point:
 *   - Complex arrays are interleaved (re, im): c64 = 2 x float, c128 = 2 x
 *     double.  NNFFT_FP32_COMP plans take and return c64, NNFFT_FP64_PLAIN
 *     plans c128.
 *   - Node arrays (v, x, a, b) are FP64 DEVICE pointers; coefficient and
 *     result arrays (f, y, c, h) are DEVICE pointers.  Index k of an array is
 *     the paper's label k - M/2 (any M >= 1 is accepted).
 *   - `stream` is a hipStream_t (NULL = the legacy default stream).  exec is
 *     asynchronous on that stream and never synchronizes the host; plan
 *     creation synchronizes `stream` once.
 *   - The caller owns every pointer it passes.  A plan copies what it needs
 *     from v and x; they may be freed once the plan call has returned.
 *   - A plan owns its device scratch, so one plan serves one exec at a time:
 *     two execs of the same plan on different streams race.
 *   - Errors are returned as nnfft_status; nothing throws across the ABI.
 *     nnfft_last_error() returns a thread-local message for the last failure.
 *   - Precision: NNFFT_FP64_PLAIN evaluates the windows exactly in FP64 and
 *     accumulates in FP64 (the plain comparator).  NNFFT_FP32_COMP streams,
 *     transforms and interpolates in FP32 with compensated (two-sum)
 *     accumulation of the grid cells; the correction factors phi_hat_1,
 *     phi_hat_2, the FFT twiddles and the quadrature nodes and weights are
 *     computed in FP64.
 */
#ifndef NNFFT_H
#define NNFFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nnfft_plan_s *nnfft_plan_t;
typedef struct sinc_plan_s *sinc_plan_t;
typedef struct nnfft_plan_s *nfft_plan_t;   /* NFFT plans (nfft_plan); not valid for nnfft_exec */

typedef enum {
    NNFFT_OK = 0,
    NNFFT_ERR_ARG = 1,          /* invalid size or parameter (see below)           */
    NNFFT_ERR_DOMAIN = 2,       /* a node outside [-1/2, 1/2] or not finite        */
    NNFFT_ERR_NOMEM = 3,        /* device or host allocation failed                */
    NNFFT_ERR_DEVICE = 4,       /* a HIP call failed                               */
    NNFFT_ERR_UNSUPPORTED = 5,  /* parameters outside what the kernels implement   */
    NNFFT_ERR_BUSY = 6          /* resource in use (serving layer)                 */
} nnfft_status;

typedef enum {
    NNFFT_FP64_PLAIN = 0,       /* FP64 windows, FP64 accumulation, FP64 FFT       */
    NNFFT_FP32_COMP = 1         /* FP32 data path, compensated grid accumulation   */
} nnfft_precision;

typedef enum {
    SINC_QUAD_GAUSS_LEGENDRE = 0,   /* n_quad Gauss-Legendre nodes (e.g. 2N)         */
    SINC_QUAD_CLENSHAW_CURTIS = 1   /* Chebyshev points, n_quad + 1 nodes, (5.4)     */
} sinc_quad;

/*
 * Window families of Example 2.1 (both windows of a plan are of one family):
 *   SINH       sinh(beta sqrt(1 - x^2)) / sinh(beta), beta_j = 2 pi m_j (1 - 1/(2 sigma_j));
 *   BSPLINE    B_2m(m x) / B_2m(0), B_2m the centred cardinal B-spline of order 2m,
 *              transform sinc(pi v / m)^(2m) / (m B_2m(0));
 *   ALGEBRAIC  (1 - x^2)^(beta - 1/2) on [-1, 1], beta_j = 3 m_j, transform
 *              pi (2 beta)! / (4^beta beta!) (pi v)^(-beta) J_beta(2 pi v); needs
 *              sigma_j > pi/3;
 * and the Kaiser-Bessel family of the comparison runs of Example 4.2, in its
 * continuous form, which belongs to the set Omega of Sec. 2:
 *   KAISER_BESSEL  (I_0(beta sqrt(1 - x^2)) - 1) / (I_0(beta) - 1) on [-1, 1],
 *              beta_j as for SINH, transform 2 / (I_0(beta) - 1) [sinh(z)/z -
 *              sin(2 pi v)/(2 pi v)], z = sqrt(beta^2 - 4 pi^2 v^2).
 */
typedef enum {
    NNFFT_WINDOW_SINH = 0,
    NNFFT_WINDOW_BSPLINE = 1,
    NNFFT_WINDOW_ALGEBRAIC = 2,
    NNFFT_WINDOW_KAISER_BESSEL = 3
} nnfft_window;

/* Derived sizes and diagnostics of a plan (host struct, filled by the library). */
typedef struct {
    int64_t N, N_star, N1, G1, N2;  /* bandwidth, N*, N1, G1 = N1 + 2 m1, FFT length */
    int64_t M1, M2;                 /* node counts                                   */
    int32_t m1, m2;                 /* truncation parameters                         */
    int32_t precision;              /* nnfft_precision                               */
    double sigma1, sigma2;          /* requested oversampling factors                */
    double sigma1_eff, sigma2_eff;  /* N1 / N*, N2 / G1 (used in beta and the bound) */
    double a;                       /* (2.6): 1 + 2 m1 / N1                          */
    double beta1, beta2;            /* sinh: 2 pi m_j (1 - 1/(2 sigma_j_eff));
                                       algebraic: 3 m_j; B-spline: 0               */
    double bound_thm41;             /* E(phi_sinh) of (4.2) at the effective sigmas
                                       (sinh windows; 0 for the others)             */
    int32_t thm41_applies;          /* 1 if sinh, sigma_eff in [5/4, 2], m2 >= m1    */
    int32_t window_degree;          /* FP32: degree of the per-tap window polynomials*/
    double window_fit_err;          /* FP32: max abs error of those polynomials      */
    int32_t corr_degree;            /* degree of the 1/phi_hat_1 Chebyshev series     */
    double corr_fit_err;            /* its max relative error                        */
    int64_t device_bytes;           /* device memory owned by the plan               */
    int64_t block_points;           /* points per node block (XCD locality unit)     */
    int32_t items_points;           /* max points per work item                      */
    int32_t spread_workgroups;      /* workgroups of the spreading launch            */
    int32_t interp_workgroups;      /* workgroups of the interpolation launch        */
    int32_t fft_n1, fft_n2;         /* FFT factorization N2 = n1 * n2 (n1 = 1: one WG)*/
    int32_t window;                 /* nnfft_window of both windows                  */
    int32_t reserved;
} nnfft_info_t;

/*
 * Parameter derivation only (no device work); used to size requests.
 * Sizes of Algorithm 2.2 with these readings: N* = N + ceil(2 m1/sigma1);
 * N1 = 2 ceil(sigma1 N* / 2); G1 = N1 + 2 m1; N2 = the largest even integer
 * with prime factors 2, 3, 5 not above sigma2 G1 (if that drops below
 * min(sigma2, 5/4) G1: the smallest such integer >= sigma2 G1);
 * beta_j from the effective sigmas.
 * Errors: NNFFT_ERR_ARG if N < 1, m < 2, sigma <= 1, 2 m1 >= N1 or
 * 2 m2 > (1 - 1/sigma1_eff) N2 (the requirement of Algorithm 2.2).
 */
nnfft_status nnfft_derive_params(int64_t N, double sigma1, double sigma2, int m1, int m2,
                                 nnfft_info_t *out);

/*
 * Creates a plan for Algorithm 2.2 (step 0 "precompute" and the node
 * preprocessing): node records (grid cell + fractional offset, computed in
 * FP64), a stable sort of the nodes into cell bins inside blocks of
 * consecutive indices, the work items and the workgroup schedule, the FP64
 * table 1/(N1 N2 phi_hat_2(l)), the FFT twiddles (FP64, rounded for FP32),
 * and for FP32 the Chebyshev fits of the window taps and of 1/phi_hat_1.
 *   v[M1], x[M2]  FP64 device arrays of frequencies and spatial nodes.
 * Errors: ARG (sizes as in nnfft_derive_params, M1 < 1, M2 < 1, M > 2^30),
 * DOMAIN (|v_k| > 1/2 or |x_j| > 1/2 or NaN), UNSUPPORTED (m > 16, FP32 with
 * m < 4, or a window / correction fit that misses its tolerance), NOMEM,
 * DEVICE.  On error *out is set to NULL.
 */
nnfft_status nnfft_plan(nnfft_plan_t *out, int64_t N, int64_t M1, int64_t M2,
                        double sigma1, double sigma2, int m1, int m2, nnfft_precision prec,
                        const double *v, const double *x, void *stream);

/*
 * nnfft_plan with windows of family `window` (Example 2.1; nnfft_plan uses
 * NNFFT_WINDOW_SINH).  Plans of every family run through nnfft_exec,
 * nnfft_exec_batch and the serving layer alike.  The FP32 path evaluates the
 * taps of every family from its per-tap Chebyshev series; the FP64 path
 * evaluates sinh and algebraic taps directly and B-spline taps from the exact
 * series of their polynomial pieces.  The error of Theorem 3.5 with these
 * windows is larger than with sinh windows of equal m (Sec. 4 compares them).
 * Errors: as nnfft_plan, plus ARG for an unknown family or an algebraic
 * window with sigma_eff <= pi/3.
 */
nnfft_status nnfft_plan_window(nnfft_plan_t *out, int64_t N, int64_t M1, int64_t M2,
                               double sigma1, double sigma2, int m1, int m2, nnfft_precision prec,
                               nnfft_window window, const double *v, const double *x, void *stream);

/*
 * Host-only dry run of nnfft_plan on HOST node arrays v[M1], x[M2]: the same
 * validations, tables and node layout, then a check of the layout invariants
 * the kernels rely on (every point in exactly one work item, record blocks,
 * spreading windows inside the grid, no two windows writing one partial
 * cell, merge lists).  No device work, no device memory.  *out receives the
 * plan's info, device_bytes included (its exact device footprint).
 * Errors: as nnfft_plan; ARG with an "internal:" message if an invariant fails.
 */
nnfft_status nnfft_plan_dry_run(int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2, int m1, int m2,
                                nnfft_precision prec, const double *v, const double *x, nnfft_info_t *out);

/* nnfft_plan_dry_run for windows of family `window` (as nnfft_plan_window). */
nnfft_status nnfft_plan_window_dry_run(int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2, int m1,
                                       int m2, nnfft_precision prec, nnfft_window window, const double *v,
                                       const double *x, nnfft_info_t *out);

/*
 * Layout digests (Algorithm 2.2 step 0).  nnfft_plan orders the nodes on the
 * device (cell/offset split in FP64, domain check, per-block bin counts and a
 * stable sort by (node block, cell)) and builds the work schedule on the host
 * from the bin counts; the dry run builds the same layout from host nodes on
 * the host alone.  Both digests hash, with 64-bit FNV-1a, the byte image of
 * the plan's tables, schedule and point records as the kernels read them, so
 * equal digests mean bit-for-bit equal layouts.
 *   nnfft_plan_digest           of a plan on the device (copies the image to
 *                               the host; synchronizes the device);
 *   nnfft_plan_window_dry_run_digest  of the layout the dry run builds from
 *                               host nodes v[M1], x[M2].
 * Errors: as nnfft_plan_dry_run; ARG (null argument), DEVICE.
 */
nnfft_status nnfft_plan_digest(nnfft_plan_t p, uint64_t *digest);
nnfft_status nnfft_plan_window_dry_run_digest(int64_t N, int64_t M1, int64_t M2, double sigma1, double sigma2,
                                              int m1, int m2, nnfft_precision prec, nnfft_window window,
                                              const double *v, const double *x, uint64_t *digest);

/*
 * Runs Algorithm 2.2 on `stream`: f[M1] -> y[M2] (c64 or c128 per the plan's
 * precision; y in the caller's node order).  f and y must not overlap.
 */
nnfft_status nnfft_exec(nnfft_plan_t p, const void *f, void *y, void *stream);

/*
 * For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid it): the
 * same transform as nnfft_exec on the same kernels, with the per-exec
 * working memory (window planes, FFT intermediate and consumed outputs) in a
 * static device array of the library, 64 MiB, one per GPU, held until the
 * process ends; this call allocates nothing and records no memset.  The
 * caller passes the plan, f and y as for nnfft_exec; the results are bitwise
 * those of nnfft_exec.  Every call on one GPU shares that GPU's array: calls
 * that overlap on one GPU (other streams, other threads) race and must be
 * ordered by the caller.  The array keeps the last call's contents; the call
 * clears what must start at zero itself.  Errors: ARG (null argument, an
 * NFFT plan, or a plan whose working memory exceeds 64 MiB: the message
 * states both sizes), DEVICE.
 */
nnfft_status nnfft_exec_noalloc(nnfft_plan_t p, const void *f, void *y, void *stream);

/*
 * Batched form (Algorithm 2.2 on many plans at once): runs n independent
 * plans of any sizes N, M1, M2, sigma, m with one launch per stage for all
 * plans of one precision -- spreading, FFT stage A (whole transforms of
 * short plans), FFT stage B, interpolation -- up to 32 plans per launch
 * (longer lists are cut into groups of 32).  FP32 and FP64 plans form
 * separate groups.  f[i], y[i] are the device arrays of plans[i] (c64 for
 * FP32 plans, c128 for FP64).  Each workgroup runs the same code on the same
 * data as nnfft_exec, so every y[i] is bitwise equal to nnfft_exec on that
 * plan.  Errors: ARG (n < 0, a null plan or array, or a plan listed twice:
 * plans own their scratch), DEVICE.  Asynchronous on `stream`.
 */
nnfft_status nnfft_exec_batch(int n, const nnfft_plan_t *plans, const void *const *f,
                              void *const *y, void *stream);

nnfft_status nnfft_info(nnfft_plan_t p, nnfft_info_t *out);

/*
 * Kernel timing (not part of the transform).  nnfft_profile_start makes the
 * next `max_execs` nnfft_exec calls on the plan launch each of their kernels
 * with a pair of HIP events attached to the kernel's dispatch
 * (hipExtLaunchKernel), so an event pair measures that kernel's execution
 * on the device, on the stream it runs on, without the gaps between
 * kernels.  The results are read once, by one of:
 *   nnfft_profile_stop     average duration (ms) of each stage over the
 *                          recorded execs in stage_ms[0..2] = {spreading,
 *                          FFT (with merge and deconvolution: the sum of its
 *                          kernels), interpolation}; count in *nexecs;
 *   nnfft_profile_kernels  per kernel in launch order (up to kcap entries,
 *                          count in *nkernels): name, stage, average,
 *                          minimum and maximum duration; per exec (up to
 *                          ecap values in exec_ms) the span from the start
 *                          of its first kernel to the end of its last; the
 *                          number of recorded execs in *nexecs.
 * Both wait for the last recorded exec and release the events; host arrays
 * are owned by the caller.  Errors: ARG, NOMEM, DEVICE.
 */
typedef struct {
    char name[32];     /* kernel name, e.g. "k_spread32" */
    int stage;         /* 0 spreading, 1 FFT, 2 interpolation */
    double avg_ms, min_ms, max_ms;
} nnfft_kernel_time_t;
nnfft_status nnfft_profile_start(nnfft_plan_t p, int max_execs);
nnfft_status nnfft_profile_stop(nnfft_plan_t p, double *stage_ms, int *nexecs);
nnfft_status nnfft_profile_kernels(nnfft_plan_t p, nnfft_kernel_time_t *kernels, int kcap, int *nkernels,
                                   double *exec_ms, int ecap, int *nexecs);
nnfft_status nnfft_destroy(nnfft_plan_t p);

/*
 * NFFT with equispaced frequencies: the special case v_k = k / N, k in I_N
 * (M1 = N, f indexed k + N/2) of (1.2), named in Sec. 2 as the building block
 * of the NNFFT and in Sec. 6 as the form one NNFFT of Algorithm 6.1 takes
 * when its nodes are equispaced, and its adjoint:
 *   nfft_exec     y_j = sum_{k in I_N} f_k exp(-2 pi i k x_j),   j in I_M
 *   nfft_adjoint  h_k = sum_{j in I_M} y_j exp(+2 pi i k x_j),   k in I_N
 * Steps (sinh-type window of Example 2.1, phi(t) = omega(n t / m)):
 *   forward: f_k / (n phi_hat(k)) zero-padded to length n, a length-n FFT,
 *            window interpolation at n x_j on the 1-periodic grid;
 *   adjoint: window spreading of y_j at n x_j, folded 1-periodically, a
 *            length-n transform with the + sign, division by n phi_hat(k).
 * n is the smallest even 2,3,5-smooth integer >= sigma N; beta =
 * 2 pi m (1 - N / (2 n)).  The two maps are exact transposes of each other.
 * The same precisions as the NNFFT (FP32: m >= 4).  x[M]: FP64 device nodes in
 * [-1/2, 1/2]; f, y, h: c64 (FP32) or c128 (FP64) device arrays, caller-owned.
 * nnfft_info reports N1 = N2 = n.  NFFT plans cannot be batched.
 * Errors: ARG (odd N, N < 2, sigma <= 1, m < 2, 2 m >= n, null arrays, an
 * NNFFT plan given to nfft_exec or the reverse), DOMAIN, UNSUPPORTED (m > 16,
 * FP32 with m < 4, n too long), NOMEM, DEVICE.
 */
nnfft_status nfft_plan(nfft_plan_t *out, int64_t N, int64_t M, double sigma, int m, nnfft_precision prec,
                       const double *x, void *stream);
nnfft_status nfft_exec(nfft_plan_t p, const void *f, void *y, void *stream);
nnfft_status nfft_adjoint(nfft_plan_t p, const void *y, void *h, void *stream);
nnfft_status nfft_destroy(nfft_plan_t p);

/* Host-only dry run of nfft_plan on HOST nodes x[M], with the layout checks
 * of nnfft_plan_dry_run.  No device work.  Errors: as nfft_plan. */
nnfft_status nfft_plan_dry_run(int64_t N, int64_t M, double sigma, int m, nnfft_precision prec, const double *x,
                               nnfft_info_t *out);

/*
 * Layout tuning.  A plan sorts each node side into blocks of consecutive
 * caller indices (one XCD's share of the gathers and scatters), bins of one
 * grid cell, work items of at most items_points points of one bin, and
 * workgroups of 64 items (one workgroup per launch slot).
 * These knobs change speed, and the summation order of the FP32 cell sums,
 * never the algorithm.  Plans take them from a process-wide table keyed by
 * precision and ceil(log2 M) of each side, else from a built-in rule.
 */
typedef struct {
    int32_t items_points;           /* max points per work item (FP64: <= 8)         */
    int32_t reserved;               /* 0                                             */
    int64_t block_points;           /* points per node block                         */
    double exec_ms;                 /* nnfft_autotune: measured exec time            */
    int32_t candidates;             /* nnfft_autotune: layouts timed                 */
    int32_t tuned;                  /* nnfft_get_tuning: 1 if from the table         */
} nnfft_tuning_t;

/*
 * Autotuner: times nnfft_exec of an N, M1 = M2 = M, m1 = m2 = m, sigma = 2
 * plan on synthetic uniform nodes (a fixed seed) for a set of candidate
 * layouts (items_points {4, 8, 16, 32} (FP64 {2, 4, 8}) x block_points
 * {2^13 .. 2^17}, after the clamping rules,
 * and the built-in rule's layout), `reps` timed execs each
 * after 2 untimed ones, on `stream`, and installs the fastest in the table
 * for M's size class and precision (it then applies to both sides of later
 * plans of that class).  Allocates and frees its own device memory; blocks
 * until done.  *best receives the layout and its time.
 * Errors: ARG, UNSUPPORTED (as nnfft_plan), NOMEM, DEVICE.
 */
nnfft_status nnfft_autotune(int64_t N, int64_t M, int m, nnfft_precision prec, int reps, void *stream,
                            nnfft_tuning_t *best);

/* Installs a layout for plans of precision prec whose side has M's size class
 * (ceil(log2 M)).  Errors: ARG for items_points < 1 or block_points < 1.
 * Out-of-range values are clamped when a plan uses them. */
nnfft_status nnfft_set_tuning(nnfft_precision prec, int64_t M, const nnfft_tuning_t *t);

/* The layout a spreading side of M nodes would use now (tuned = 1 if from the
 * table).  Without a table entry the rule takes 2^17-point blocks, 2^18 for
 * spreading sides above 2^20 points. */
nnfft_status nnfft_get_tuning(nnfft_precision prec, int64_t M, nnfft_tuning_t *out);

/* Empties the table (plans fall back to the built-in rule). */
nnfft_status nnfft_clear_tuning(void);

/*
 * Fast sinc transform plan (Algorithm 6.1).  Quadrature nodes z_j and weights
 * w_j (sum w_j = 1) are computed on the host in FP64: Gauss-Legendre with
 * n_quad nodes, or Clenshaw-Curtis (5.4) with n_quad + 1 Chebyshev points.
 * The first NNFFT uses v = a_k, x = z_j / 2, the second v = -z_j / 2,
 * x = b_l, both with bandwidth N and the given sigma, m, precision.
 * Equispaced nodes take the special cases of Sec. 6 (exact FP64 equality,
 * decided at plan time):
 *   a_k = k / L1 for k in I_L1 (a[i] = (i - L1/2) / L1, L1 even, N <= L1):
 *     step 1 is the NFFT of length L1 (nfft_plan) at the nodes N z_j / (2 L1);
 *   L2 = N and b_l = l / N for l in I_N: step 3 is the adjoint NFFT of
 *     length N at the nodes z_j / 2.
 * Those NFFTs use sigma1 and m1.
 *   a[L1], b[L2]: FP64 device arrays in [-1/2, 1/2].
 * Errors: as nnfft_plan, plus ARG for n_quad < 1 or an unknown rule.
 */
nnfft_status sinc_plan(sinc_plan_t *out, int64_t N, int64_t L1, int64_t L2, sinc_quad quad,
                       int64_t n_quad, double sigma1, double sigma2, int m1, int m2,
                       nnfft_precision prec, const double *a, const double *b, void *stream);

/* c[L1] -> h[L2] (complex, c64/c128 per precision); real c gives real h up to
 * the transform's error.  Asynchronous on `stream`. */
nnfft_status sinc_exec(sinc_plan_t p, const void *c, void *h, void *stream);

/* Info of the two plans inside (which = 0: step 1, which = 1: step 3); an
 * NFFT step reports N = N_star = its length, N1 = N2 = its FFT length and
 * M1 = M2 = the quadrature size. */
nnfft_status sinc_info(sinc_plan_t p, int which, nnfft_info_t *out);

/* Input length L1, output length L2, quadrature size, and which steps are
 * NFFTs (bit 0: step 1, bit 1: step 3).  Errors: ARG for null arguments. */
nnfft_status sinc_sizes(sinc_plan_t p, int64_t *L1, int64_t *L2, int64_t *n_nodes, int32_t *nfft_steps);
nnfft_status sinc_destroy(sinc_plan_t p);

/*
 * The middle of Algorithm 6.1 as one operator.  Between the two FFTs the
 * transform is linear in the first FFT's outputs h_s and depends on the
 * quadrature and the plan parameters only: the first plan's interpolation
 * (2.13) at x_j = z_j / 2 with its factors 1/phi_hat_1(N* x_j), the weights w_j
 * of step 2, and the second plan's spreading (2.12) from v_j = -z_j / 2 with
 * its deconvolution 1/phi_hat_2(l) (step 2 of Algorithm 2.2) compose to
 *   u_l = sum_s K[l][s] h_s,  l in I_G1,
 *   K[l][s] = sum_j phi_1(l/N1 - v*_j) w_j phi_2(x_j/sigma1 - s/N2)
 *             / (N1 N2 phi_hat_1(N* x_j) phi_hat_2(l)),
 * a band of about 2 (m1 + m2) labels s per row l.  sinc_plan builds K on
 * the host in FP64 with the exact windows when both steps are NNFFTs and the
 * rule has at most 2^16 nodes; sinc_exec then runs spreading + FFT of the
 * first plan, one launch of the band, FFT + interpolation of the second plan
 * (instead of the first plan's interpolation at the quadrature nodes and the
 * second plan's spreading from them).  The results agree with the two-kernel
 * form up to rounding.
 *   on = 1: sinc_exec uses the operator (the default where it was built);
 *   on = 0: the two-kernel form; any other value: no change.
 *   built, active (may be null): 1 if the plan has the operator / if
 *   sinc_exec uses it.
 * Errors: ARG for a null plan, UNSUPPORTED for on = 1 without the operator.
 */
nnfft_status sinc_middle(sinc_plan_t p, int on, int32_t *built, int32_t *active);

/*
 * Host-only: the middle operator sinc_plan would build for bandwidth N, the
 * quadrature (quad, n_quad) and sigma, m, precision (it does not depend on
 * the nodes a_k, b_l).  On return *G1 is the number of rows (labels
 * l = r - G1/2, r = 0..G1-1) and *Wb the band width; if K and lo are non-null
 * and cap >= G1 * Wb, K[b * G1 + r] receives entry b of row r (label
 * lo[r] + b of the first FFT's outputs) and lo[r] the row's first label.
 * Errors: ARG (as sinc_plan, or cap too small with K given), UNSUPPORTED if
 * the operator is not built for these parameters (more than 2^16 nodes or a
 * band wider than 256 labels).
 */
nnfft_status sinc_middle_dry_run(int64_t N, sinc_quad quad, int64_t n_quad, double sigma1, double sigma2, int m1,
                                 int m2, nnfft_precision prec, double *K, int32_t *lo, int64_t cap, int64_t *G1,
                                 int32_t *Wb);

/*
 * The quadrature rule sinc_plan uses, on the host (no device work):
 * z[n_nodes], w[n_nodes] HOST arrays with n_nodes = n_quad (Gauss-Legendre)
 * or n_quad + 1 (Clenshaw-Curtis); weights sum to 1 (sinc(N pi x) is half the
 * integral of e^{-pi i N t x} over [-1, 1], Sec. 5).  Gauss-Legendre by
 * Newton's method on the Legendre recurrence; Clenshaw-Curtis by Algorithm
 * 5.4 (DCT-I of length n_quad + 1).  Errors: ARG for n_quad < 1, an unknown
 * rule or null arrays.
 */
nnfft_status nnfft_quadrature(sinc_quad quad, int64_t n_quad, double *z, double *w);

/* Thread-local description of the last error in this thread ("" if none). */
const char *nnfft_last_error(void);

/* Library version string. */
const char *nnfft_version(void);

#ifdef __cplusplus
}
#endif

#endif /* NNFFT_H */
