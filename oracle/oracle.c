/*
 * FP64 CPU oracle for the NNFFT and the fast sinc transform of
 * Kircheis, Potts, Tasche, "Nonuniform fast Fourier transforms with
 * nonequispaced spatial and frequency data and fast sinc transforms"
 * (arXiv 2107.02671).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU library
 * shares no code, header, table or constant generator with it.
 *
 * Everything here is plain, slow and written to be checked against the paper
 * by eye: direct sums, the steps of Algorithm 2.2 in the paper's order with a
 * direct DFT in step 3, Algorithm 6.1 built from two calls of that NNFFT, and
 * the two quadrature rules.  All arithmetic is IEEE double.
 *
 * Complex arrays are interleaved (re, im) doubles.
 * Readings of points where the paper is silent are marked "Reading:".
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846264338327950288

typedef struct {
    long N;          /* nonharmonic bandwidth N                               */
    long N_star;     /* N* = N + ceil(2 m1 / sigma1)      (Sec. 2, after (2.7)) */
    long N1;         /* first oversampled length, even                        */
    long G1;         /* N1 + 2 m1 = a N1, length of the grid in step 1        */
    long N2;         /* FFT length of step 3                                  */
    int m1, m2;      /* truncation parameters                                 */
    double sigma1, sigma2;          /* requested oversampling factors         */
    double sigma1_eff, sigma2_eff;  /* N1 / N*,  N2 / G1                      */
    double a;                       /* (2.6): a = 1 + 2 m1 / N1               */
    double beta1, beta2;            /* shape parameters of the windows        */
    int window;                     /* ORC_WIN_* of both windows              */
} orc_params_t;

/* Window families of Example 2.1 */
#define ORC_WIN_SINH 0        /* sinh-type, beta = 2 pi m (1 - 1/(2 sigma))       */
#define ORC_WIN_BSPLINE 1     /* B_{2m}(m x) / B_{2m}(0)                           */
#define ORC_WIN_ALGEBRAIC 2   /* (1 - x^2)^(beta - 1/2), beta = 3m, sigma > pi/3   */
#define ORC_WIN_KAISER_BESSEL 3 /* (I_0(beta sqrt(1 - x^2)) - 1) / (I_0(beta) - 1),
                                   beta = 2 pi m (1 - 1/(2 sigma))                   */

double orc_sinc_pi(double d);
double orc_window(int kind, double x, int m, double beta);
double orc_window_hat(int kind, double v, int m, double beta);

/* ------------------------------------------------------------------------ */
/* Parameter derivation                                                      */
/* ------------------------------------------------------------------------ */

static long orc_ceil_tol(double x) { return (long)ceil(x - 1e-9); }

static int orc_is_smooth235(long n)
{
    if (n < 1) return 0;
    while (n % 2 == 0) n /= 2;
    while (n % 3 == 0) n /= 3;
    while (n % 5 == 0) n /= 5;
    return n == 1;
}

/*
 * Sizes of Algorithm 2.2 (its input list) with the N* substitution of
 * Sec. 2 (the paragraph after (2.7)).
 * Reading: N1 = sigma1 N* need not be an even integer, so N1 is rounded up to
 *   the next even integer and sigma1_eff = N1 / N* is used afterwards.
 * Reading: N2 = sigma2 (N1 + 2 m1) is taken as the largest even integer with
 *   prime factors 2, 3, 5 that does not exceed sigma2 G1; if that falls below
 *   min(sigma2, 5/4) G1 the smallest such integer >= sigma2 G1 is used.
 * Reading: beta_j of Example 2.1 / Sec. 4 uses the effective factors.
 * Returns 0 on success, 1 for invalid parameters.
 */
int orc_params(long N, double sigma1, double sigma2, int m1, int m2, orc_params_t *p)
{
    if (N < 1 || m1 < 2 || m2 < 2 || !(sigma1 > 1.0) || !(sigma2 > 1.0)) return 1;
    memset(p, 0, sizeof(*p));
    p->N = N; p->m1 = m1; p->m2 = m2; p->sigma1 = sigma1; p->sigma2 = sigma2;
    p->N_star = N + orc_ceil_tol(2.0 * m1 / sigma1);
    p->N1 = 2 * orc_ceil_tol(sigma1 * (double)p->N_star / 2.0);
    p->G1 = p->N1 + 2 * m1;
    {
        double target = sigma2 * (double)p->G1;
        long n = (long)floor(target + 1e-9);
        if (n % 2) n -= 1;
        while (n >= 2 && !orc_is_smooth235(n)) n -= 2;
        double lowest = (sigma2 < 1.25 ? sigma2 : 1.25) * (double)p->G1;
        if ((double)n < lowest - 1e-9 || n <= p->G1) {
            n = orc_ceil_tol(target);
            if (n % 2) n += 1;
            while (!orc_is_smooth235(n)) n += 2;
        }
        p->N2 = n;
    }
    p->sigma1_eff = (double)p->N1 / (double)p->N_star;
    p->sigma2_eff = (double)p->N2 / (double)p->G1;
    p->a = 1.0 + 2.0 * m1 / (double)p->N1;
    p->beta1 = 2.0 * ORC_PI * m1 * (1.0 - 1.0 / (2.0 * p->sigma1_eff));
    p->beta2 = 2.0 * ORC_PI * m2 * (1.0 - 1.0 / (2.0 * p->sigma2_eff));
    /* Algorithm 2.2 input: 2 m2 <= (1 - 1/sigma1) N2 */
    if (2.0 * m2 > (1.0 - 1.0 / p->sigma1_eff) * (double)p->N2 + 1e-9) return 1;
    if (2 * m1 >= p->N1) return 1;
    p->window = ORC_WIN_SINH;
    return 0;
}

/*
 * The same sizes for the windows of family `window` (Example 2.1): the
 * B-spline windows have no shape parameter (beta = 0); the algebraic windows
 * take beta_j = 3 m_j and need sigma_j > pi/3; the continuous Kaiser-Bessel
 * windows take the sinh windows' beta_j.
 */
int orc_params_window(long N, double sigma1, double sigma2, int m1, int m2, int window, orc_params_t *p)
{
    if (orc_params(N, sigma1, sigma2, m1, m2, p)) return 1;
    if (window == ORC_WIN_BSPLINE) {
        p->beta1 = p->beta2 = 0.0;
    } else if (window == ORC_WIN_ALGEBRAIC) {
        if (!(p->sigma1_eff > ORC_PI / 3.0) || !(p->sigma2_eff > ORC_PI / 3.0)) return 1;
        p->beta1 = 3.0 * m1;
        p->beta2 = 3.0 * m2;
    } else if (window != ORC_WIN_SINH && window != ORC_WIN_KAISER_BESSEL) {
        return 1;
    }
    p->window = window;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* sinh-type window and its Fourier transform (Example 2.1, Sec. 4)          */
/* ------------------------------------------------------------------------ */

/* omega_sinh(x) = sinh(beta sqrt(1 - x^2)) / sinh(beta) on [-1, 1], else 0 */
double orc_omega(double x, double beta)
{
    if (fabs(x) >= 1.0) return 0.0;
    return sinh(beta * sqrt((1.0 - x) * (1.0 + x))) / sinh(beta);
}

/* (beta^2 - 4 pi^2 v^2)^(-1/2) I_1(sqrt(.)) written as the power series
 * (1/2) sum_k y^k / (4^k k! (k+1)!) with y = beta^2 - 4 pi^2 v^2 >= 0
 * (the expansion stated after (2.1)).  All terms are positive. */
double orc_i1_over_z_series(double y)
{
    double term = 0.5, sum = 0.5;
    for (int k = 0; k < 400; k++) {
        term *= (y / 4.0) / ((double)(k + 1) * (double)(k + 2));
        sum += term;
        if (term < 1e-18 * sum && (double)k > sqrt(y)) break;
    }
    return sum;
}

/* (2.1): Fourier transform of omega_sinh, all three branches */
double orc_omega_hat(double v, double beta)
{
    double pre = ORC_PI * beta / sinh(beta);
    double y = beta * beta - 4.0 * ORC_PI * ORC_PI * v * v;
    if (y > 0.0) return pre * orc_i1_over_z_series(y);
    if (y == 0.0) return pre * 0.5;
    double z = sqrt(-y);
    return pre * j1(z) / z;
}

/* Scaled window transforms (4.1) and the scaling rule of Sec. 3 (proof of
 * Theorem 3.4): phi_hat_j(v) = (m_j / N_j) omega_hat_j(m_j v / N_j). */
static double orc_phi1_hat(const orc_params_t *p, double v)
{
    return (double)p->m1 / (double)p->N1 * orc_window_hat(p->window, p->m1 * v / (double)p->N1, p->m1, p->beta1);
}
static double orc_phi2_hat(const orc_params_t *p, double v)
{
    return (double)p->m2 / (double)p->N2 * orc_window_hat(p->window, p->m2 * v / (double)p->N2, p->m2, p->beta2);
}

/* ------------------------------------------------------------------------ */
/* B-spline and algebraic windows (Example 2.1)                               */
/* ------------------------------------------------------------------------ */

/* Cardinal B-spline M_n of order n (support [0, n]) by its recursion
 * M_1 = indicator of [0, 1),
 * M_k(y) = (y M_{k-1}(y) + (k - y) M_{k-1}(y - 1)) / (k - 1),
 * with M_k(y - i) tabulated for the shifts i the recursion reaches.  The
 * centred spline of the paper is B_n(x) = M_n(x + n/2). */
double orc_bspline_cardinal(int n, double y)
{
    double val[130];
    if (n < 1 || n > 128) return NAN;
    for (int i = 0; i < n; i++) val[i] = (y - i >= 0.0 && y - i < 1.0) ? 1.0 : 0.0;
    for (int k = 2; k <= n; k++)
        for (int i = 0; i <= n - k; i++) {
            double yi = y - i;
            val[i] = (yi * val[i] + ((double)k - yi) * val[i + 1]) / (double)(k - 1);
        }
    return val[0];
}

/* omega_B(x) = B_{2m}(m x) / B_{2m}(0) */
static double orc_omega_bspline(double x, int m)
{
    if (fabs(x) >= 1.0) return 0.0;
    return orc_bspline_cardinal(2 * m, m * x + m) / orc_bspline_cardinal(2 * m, (double)m);
}

/* omega_B_hat(v) = sinc(pi v / m)^(2m) / (m B_{2m}(0)) */
static double orc_omega_hat_bspline(double v, int m)
{
    double b0 = orc_bspline_cardinal(2 * m, (double)m);
    double s = orc_sinc_pi(v / m);
    return pow(s, 2.0 * m) / ((double)m * b0);
}

/* omega_alg(x) = (1 - x^2)^(beta - 1/2) on [-1, 1] */
static double orc_omega_algebraic(double x, double beta)
{
    if (fabs(x) >= 1.0) return 0.0;
    return pow((1.0 - x) * (1.0 + x), beta - 0.5);
}

/* omega_alg_hat(v) = pi (2 beta)! / (4^beta beta!) (pi v)^(-beta) J_beta(2 pi v)
 * for integer beta, with the Bessel power series
 * (pi v)^(-beta) J_beta(2 pi v) = sum_k (-1)^k (pi v)^(2k) / (k! (k + beta)!),
 * summed in long double (the alternating terms cancel a few digits; accurate to
 * ~1e-14 for |v| <= m/2, which covers the |v| <= m / (2 sigma) the NNFFT uses). */
static double orc_omega_hat_algebraic(double v, double beta)
{
    long double b = (long double)beta;
    long double lead = logl((long double)ORC_PI) + lgammal(2.0L * b + 1.0L) - b * logl(4.0L) -
                       2.0L * lgammal(b + 1.0L);
    long double term = expl(lead), sum = term;     /* k = 0: pi (2b)! / (4^b (b!)^2) */
    long double y = (long double)ORC_PI * (long double)v;
    y *= y;
    for (int k = 0; k < 2000; k++) {
        term *= -y / ((long double)(k + 1) * ((long double)(k + 1) + b));
        sum += term;
        if (fabsl(term) < 1e-22L * fabsl(sum) && (long double)k > sqrtl(y)) break;
    }
    return (double)sum;
}

/* ------------------------------------------------------------------------ */
/* Continuous Kaiser-Bessel window (the Kaiser-Bessel family of the paper's   */
/* comparison runs, Example 4.2, in the form that belongs to Omega)          */
/* ------------------------------------------------------------------------ */

/* I_0(z) - 1 = sum_{k >= 1} (z^2/4)^k / (k!)^2: the power series of the
 * modified Bessel function without its constant term (all terms positive). */
double orc_i0_minus_1(double z)
{
    double q = 0.25 * z * z, term = 1.0, sum = 0.0;
    for (int k = 1; k < 2000; k++) {
        term *= q / ((double)k * (double)k);
        sum += term;
        if (term <= 1e-18 * sum && (double)k > sqrt(q)) break;
    }
    return sum;
}

/* omega_KB(x) = (I_0(beta sqrt(1 - x^2)) - 1) / (I_0(beta) - 1) on [-1, 1]:
 * even, 1 at 0, decreasing on [0, 1], 0 at +-1 (continuous). */
static double orc_omega_kb(double x, double beta)
{
    if (fabs(x) >= 1.0) return 0.0;
    return orc_i0_minus_1(beta * sqrt((1.0 - x) * (1.0 + x))) / orc_i0_minus_1(beta);
}

/* Its Fourier transform.  int_{-1}^{1} I_0(beta sqrt(1 - x^2)) e^{-2 pi i v x} dx
 * = 2 sinh(sqrt(y)) / sqrt(y), y = beta^2 - 4 pi^2 v^2 (2 sin(sqrt(-y)) / sqrt(-y)
 * for y < 0, 2 at y = 0), and the constant 1 on [-1, 1] transforms to
 * 2 sin(2 pi v) / (2 pi v), so
 *   omega_KB_hat(v) = 2 / (I_0(beta) - 1) [sinh(sqrt(y))/sqrt(y) - sinc(2 pi v)]. */
static double orc_omega_hat_kb(double v, double beta)
{
    double y = beta * beta - 4.0 * ORC_PI * ORC_PI * v * v, s;
    if (y > 1e-8) s = sinh(sqrt(y)) / sqrt(y);
    else if (y < -1e-8) s = sin(sqrt(-y)) / sqrt(-y);
    else s = 1.0 + y / 6.0;
    return 2.0 / orc_i0_minus_1(beta) * (s - orc_sinc_pi(2.0 * v));
}

/* The window omega of family `kind` (sinh uses beta, B-spline m, algebraic beta). */
double orc_window(int kind, double x, int m, double beta)
{
    if (kind == ORC_WIN_BSPLINE) return orc_omega_bspline(x, m);
    if (kind == ORC_WIN_ALGEBRAIC) return orc_omega_algebraic(x, beta);
    if (kind == ORC_WIN_KAISER_BESSEL) return orc_omega_kb(x, beta);
    return orc_omega(x, beta);
}

/* Its Fourier transform omega_hat(v) = 2 int_0^1 omega(x) cos(2 pi v x) dx. */
double orc_window_hat(int kind, double v, int m, double beta)
{
    if (kind == ORC_WIN_BSPLINE) return orc_omega_hat_bspline(v, m);
    if (kind == ORC_WIN_ALGEBRAIC) return orc_omega_hat_algebraic(v, beta);
    if (kind == ORC_WIN_KAISER_BESSEL) return orc_omega_hat_kb(v, beta);
    return orc_omega_hat(v, beta);
}

/* ------------------------------------------------------------------------ */
/* Direct sums                                                               */
/* ------------------------------------------------------------------------ */

/* exp(-2 pi i t) with t reduced modulo 1 first */
static void orc_expm2pi(double t, double *c, double *s)
{
    double r = t - nearbyint(t);
    *c = cos(2.0 * ORC_PI * r);
    *s = -sin(2.0 * ORC_PI * r);
}

/* Neumaier compensated accumulation */
typedef struct { double s, c; } orc_acc_t;
static void orc_acc_add(orc_acc_t *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x;
    else a->c += (x - t) + a->s;
    a->s = t;
}

/* (1.2): y_j = sum_k f_k exp(-2 pi i N v_k x_j) */
int orc_direct(long N, long M1, const double *v, const double *f,
               long M2, const double *x, double *y)
{
    long j;
#pragma omp parallel for schedule(dynamic, 4)
    for (j = 0; j < M2; j++) {
        orc_acc_t re = {0, 0}, im = {0, 0};
        for (long k = 0; k < M1; k++) {
            double c, s;
            orc_expm2pi((double)N * v[k] * x[j], &c, &s);
            orc_acc_add(&re, f[2 * k] * c - f[2 * k + 1] * s);
            orc_acc_add(&im, f[2 * k] * s + f[2 * k + 1] * c);
        }
        y[2 * j] = re.s + re.c;
        y[2 * j + 1] = im.s + im.c;
    }
    return 0;
}

/* sin(pi d) / (pi d) with sinc(0) = 1  (5.2); the argument of sin is reduced
 * by an even integer first so that pi is multiplied by a number in [-1, 1]. */
double orc_sinc_pi(double d)
{
    if (d == 0.0) return 1.0;
    double r = d - 2.0 * nearbyint(0.5 * d);
    return sin(ORC_PI * r) / (ORC_PI * d);
}

/* (6.2): h(b_l) = sum_k c_k sinc(N pi (b_l - a_k)), complex c */
int orc_sinc_direct(long N, long L1, const double *a, const double *c,
                    long L2, const double *b, double *h)
{
    long l;
#pragma omp parallel for schedule(dynamic, 4)
    for (l = 0; l < L2; l++) {
        orc_acc_t re = {0, 0}, im = {0, 0};
        for (long k = 0; k < L1; k++) {
            double s = orc_sinc_pi((double)N * (b[l] - a[k]));
            orc_acc_add(&re, c[2 * k] * s);
            orc_acc_add(&im, c[2 * k + 1] * s);
        }
        h[2 * l] = re.s + re.c;
        h[2 * l + 1] = im.s + im.c;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 2.2 (NNFFT)                                                      */
/* ------------------------------------------------------------------------ */

/*
 * Computes y_j ~ f(x_j) of (1.2) for v_k, x_j in [-1/2, 1/2].
 * Optional outputs (may be NULL):
 *   g_out[G1]  complex g_l of (2.12), l = -G1/2 .. G1/2-1 stored at l + G1/2
 *   h_out[N2]  complex h_s of step 3,  s = -N2/2 .. N2/2-1 stored at s + N2/2
 * Both windows are of family `window` (ORC_WIN_*, Example 2.1).
 * Returns 0, 1 for invalid parameters, 2 for a node outside [-1/2, 1/2],
 * 3 for an allocation failure.
 */
int orc_nnfft_window(int window, long N, double sigma1, double sigma2, int m1, int m2,
                     long M1, const double *v, const double *f,
                     long M2, const double *x, double *y,
                     double *g_out, double *h_out)
{
    orc_params_t P;
    if (orc_params_window(N, sigma1, sigma2, m1, m2, window, &P)) return 1;
    for (long k = 0; k < M1; k++) if (!(fabs(v[k]) <= 0.5)) return 2;
    for (long j = 0; j < M2; j++) if (!(fabs(x[j]) <= 0.5)) return 2;
    const long G1 = P.G1, N1 = P.N1, N2 = P.N2, Ns = P.N_star;

    double *g = calloc((size_t)(2 * G1), sizeof(double));
    double *gh = calloc((size_t)(2 * G1), sizeof(double));
    double *h = calloc((size_t)(2 * N2), sizeof(double));
    double *tw = malloc(sizeof(double) * (size_t)(2 * N2));
    if (!g || !gh || !h || !tw) { free(g); free(gh); free(h); free(tw); return 3; }

    /* Step 1, (2.12) with the N* substitution: v*_k = N v_k / N*, so that
     * phi_1(l/N1 - v*_k) = omega_1((l - t_k)/m1) with t_k = N1 v*_k.
     * The nonzero terms are l = floor(t_k) - m1 + 1 .. floor(t_k) + m1;
     * all of them lie in I_{G1} because |t_k| < N1/2. */
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *gpriv = calloc((size_t)nthr * (size_t)(2 * G1), sizeof(double));
    if (!gpriv) { free(g); free(gh); free(h); free(tw); return 3; }
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *gp = gpriv + (size_t)tid * (size_t)(2 * G1);
        long k;
#pragma omp for schedule(static)
        for (k = 0; k < M1; k++) {
            double vstar = (double)N * v[k] / (double)Ns;
            double t = (double)N1 * vstar;
            long c = (long)floor(t);
            for (long l = c - m1 + 1; l <= c + m1; l++) {
                double w = orc_window(P.window, ((double)l - t) / m1, m1, P.beta1);
                long idx = l + G1 / 2;
                gp[2 * idx] += f[2 * k] * w;
                gp[2 * idx + 1] += f[2 * k + 1] * w;
            }
        }
    }
    for (int t = 0; t < nthr; t++)
        for (long i = 0; i < 2 * G1; i++) g[i] += gpriv[(size_t)t * (size_t)(2 * G1) + (size_t)i];
    free(gpriv);
    for (long i = 0; i < 2 * G1; i++) g[i] /= (double)N1;
    if (g_out) memcpy(g_out, g, sizeof(double) * (size_t)(2 * G1));

    /* Step 2: g_hat_l = g_l / phi_hat_2(l).
     * Reading: the argument is l (as in step 2 and in the proof of
     * Theorem 3.5), not l/a (as printed in step 0(i)). */
    for (long l = -G1 / 2; l < G1 / 2; l++) {
        double d = orc_phi2_hat(&P, (double)l);
        long i = l + G1 / 2;
        gh[2 * i] = g[2 * i] / d;
        gh[2 * i + 1] = g[2 * i + 1] / d;
    }

    /* Step 3: h_s = (1/N2) sum_{l in I_G1} g_hat_l exp(-2 pi i l s / N2),
     * s in I_N2, as a direct DFT.  The exponent only depends on
     * (l s) mod N2, which is reduced exactly in integers.  Step 4 reads h_s
     * only for the 2 m2 labels s next to each u_j, so only those are
     * formed (all of them once M2 covers the grid); each one is the same sum.
     * Without h_out the other entries stay unset and unread. */
    unsigned char *need = calloc((size_t)N2, 1);
    if (!need) { free(g); free(gh); free(h); free(tw); return 3; }
    if (h_out) memset(need, 1, (size_t)N2);
    for (long j = 0; j < M2; j++) {
        double u = (double)N2 * (double)Ns * x[j] / (double)N1;
        long c = (long)floor(u);
        for (long sv = c - m2 + 1; sv <= c + m2; sv++) {
            long o = ((sv % N2) + N2) % N2;
            long oi = (o >= N2 / 2) ? o - N2 : o;
            need[oi + N2 / 2] = 1;
        }
    }
    for (long q = 0; q < N2; q++) {
        tw[2 * q] = cos(2.0 * ORC_PI * (double)q / (double)N2);
        tw[2 * q + 1] = -sin(2.0 * ORC_PI * (double)q / (double)N2);
    }
    long s;
#pragma omp parallel for schedule(dynamic, 64)
    for (s = -N2 / 2; s < N2 / 2; s++) {
        if (!need[s + N2 / 2]) continue;
        double re = 0.0, im = 0.0;
        for (long l = -G1 / 2; l < G1 / 2; l++) {
            long q = ((l * s) % N2 + N2) % N2;
            long i = l + G1 / 2;
            re += gh[2 * i] * tw[2 * q] - gh[2 * i + 1] * tw[2 * q + 1];
            im += gh[2 * i] * tw[2 * q + 1] + gh[2 * i + 1] * tw[2 * q];
        }
        long o = s + N2 / 2;
        h[2 * o] = re / (double)N2;
        h[2 * o + 1] = im / (double)N2;
    }
    free(need);
    if (h_out) memcpy(h_out, h, sizeof(double) * (size_t)(2 * N2));

    /* Step 4 and output: s1(N x_j) = sum_{|s/N2 - x_j/sigma1| < m2/N2} h_s
     * phi_2(x_j/sigma1 - s/N2), then divide by phi_hat_1(N x_j).  With the N*
     * substitution sigma1 = N1/N*, so phi_2(x_j/sigma1 - s/N2) =
     * omega_2((u_j - s)/m2) with u_j = N2 N* x_j / N1.  Since
     * 2 m2 <= (1 - 1/sigma1) N2 the taps never wrap (Sec. 2, end). */
    long j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < M2; j++) {
        double u = (double)N2 * (double)Ns * x[j] / (double)N1;
        long c = (long)floor(u);
        double re = 0.0, im = 0.0;
        for (long sv = c - m2 + 1; sv <= c + m2; sv++) {
            double w = orc_window(P.window, (u - (double)sv) / m2, m2, P.beta2);
            long o = ((sv % N2) + N2) % N2;        /* periodic index */
            long oi = (o >= N2 / 2) ? o - N2 : o;  /* label in I_N2  */
            oi += N2 / 2;
            re += h[2 * oi] * w;
            im += h[2 * oi + 1] * w;
        }
        double corr = orc_phi1_hat(&P, (double)Ns * x[j]);
        y[2 * j] = re / corr;
        y[2 * j + 1] = im / corr;
    }
    free(g); free(gh); free(h); free(tw);
    return 0;
}

/* Algorithm 2.2 with the sinh-type windows */
int orc_nnfft(long N, double sigma1, double sigma2, int m1, int m2,
              long M1, const double *v, const double *f,
              long M2, const double *x, double *y,
              double *g_out, double *h_out)
{
    return orc_nnfft_window(ORC_WIN_SINH, N, sigma1, sigma2, m1, m2, M1, v, f, M2, x, y, g_out, h_out);
}

/* ------------------------------------------------------------------------ */
/* Quadrature rules for sinc(N pi x) = (1/2) int_{-1}^{1} e^{-pi i N t x} dt */
/* ------------------------------------------------------------------------ */

/*
 * Gauss-Legendre rule with n nodes on [-1, 1] (the rule of the reference
 * [GrLeIn06] cited in Sec. 5 and Sec. 6; the paper gives no formula).
 * Textbook method: Newton's iteration on P_n, evaluated by the three-term
 * recurrence (k+1) P_{k+1} = (2k+1) t P_k - k P_{k-1}, from the initial guess
 * cos(pi (i + 3/4) / (n + 1/2)).  Weights W_i = 2 / ((1 - t_i^2) P_n'(t_i)^2),
 * returned halved (w_i = W_i / 2) so that sum w_i = 1 as in (5.5).
 * Nodes are returned in decreasing order.
 */
int orc_gauss_legendre(long n, double *z, double *w)
{
    if (n < 1) return 1;
    for (long i = 0; i < (n + 1) / 2; i++) {
        double t = cos(ORC_PI * ((double)i + 0.75) / ((double)n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; it++) {
            double p0 = 1.0, p1 = t;
            for (long k = 1; k < n; k++) {
                double p2 = ((2.0 * k + 1.0) * t * p1 - (double)k * p0) / (double)(k + 1);
                p0 = p1; p1 = p2;
            }
            dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
            double dt = p1 / dp;
            t -= dt;
            if (fabs(dt) < 1e-16) break;
        }
        /* derivative at the converged node */
        {
            double p0 = 1.0, p1 = t;
            for (long k = 1; k < n; k++) {
                double p2 = ((2.0 * k + 1.0) * t * p1 - (double)k * p0) / (double)(k + 1);
                p0 = p1; p1 = p2;
            }
            dp = (double)n * (t * p1 - p0) / (t * t - 1.0);
        }
        double W = 2.0 / ((1.0 - t * t) * dp * dp);
        z[i] = t; z[n - 1 - i] = -t;
        w[i] = 0.5 * W; w[n - 1 - i] = 0.5 * W;
    }
    if (n % 2 == 1) z[n / 2] = 0.0;
    return 0;
}

/*
 * Clenshaw-Curtis rule: Chebyshev points z_k = cos(k pi / n), k = 0..n, and
 * the weights of (5.4) with eps_n(0) = eps_n(n) = sqrt(2)/2 and eps_n(j) = 1
 * otherwise.  Written out as the double sum (O(n^2)).
 */
int orc_clenshaw_curtis(long n, double *z, double *w)
{
    if (n < 1) return 1;
    const double r2 = sqrt(2.0) / 2.0;
    for (long k = 0; k <= n; k++) {
        double ek = (k == 0 || k == n) ? r2 : 1.0;
        double sum = 0.0;
        for (long j = 0; 2 * j <= n; j++) {
            double e2j = (2 * j == 0 || 2 * j == n) ? r2 : 1.0;
            /* cos(2 j k pi / n) with the integer 2jk reduced modulo 2n */
            long q = (2 * j * k) % (2 * n);
            sum += e2j * e2j * 2.0 / (1.0 - 4.0 * (double)j * (double)j)
                   * cos(ORC_PI * (double)q / (double)n);
        }
        w[k] = ek * ek * sum / (double)n;
        /* cos(k pi / n) written as sin(pi (n - 2k) / (2n)), which is the same
         * number but exactly odd in (n - 2k), so z_k = -z_{n-k} holds exactly */
        z[k] = sin(ORC_PI * (double)(n - 2 * k) / (2.0 * (double)n));
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Algorithm 6.1 (fast sinc transform)                                       */
/* ------------------------------------------------------------------------ */

/*
 * h~_l ~ sum_k c_k sinc(N pi (b_l - a_k)) for a_k, b_l in [-1/2, 1/2].
 * quad = 0: Gauss-Legendre with nq nodes; quad = 1: Clenshaw-Curtis with
 * n = nq, i.e. nq + 1 nodes.
 * Step 1: g_j = sum_k c_k exp(-pi i N z_j a_k) is (1.2) with frequencies
 *         v_k = a_k and spatial nodes x_j = z_j / 2.
 * Step 2: alpha_j = w_j g~_j.
 * Step 3: h^_l = sum_j alpha_j exp(pi i N z_j b_l) is (1.2) with frequencies
 *         v_j = -z_j / 2 and spatial nodes b_l.
 * Returns 0 on success, the NNFFT code otherwise, 3 on allocation failure.
 */
int orc_sinc_fast(long N, double sigma1, double sigma2, int m1, int m2,
                  int quad, long nq, long L1, const double *a, const double *c,
                  long L2, const double *b, double *h)
{
    long nn = (quad == 0) ? nq : nq + 1;
    double *z = malloc(sizeof(double) * (size_t)nn);
    double *w = malloc(sizeof(double) * (size_t)nn);
    double *xs = malloc(sizeof(double) * (size_t)nn);
    double *vs = malloc(sizeof(double) * (size_t)nn);
    double *g = malloc(sizeof(double) * (size_t)(2 * nn));
    if (!z || !w || !xs || !vs || !g) { free(z); free(w); free(xs); free(vs); free(g); return 3; }
    int rc = (quad == 0) ? orc_gauss_legendre(nq, z, w) : orc_clenshaw_curtis(nq, z, w);
    if (rc == 0) {
        for (long j = 0; j < nn; j++) { xs[j] = 0.5 * z[j]; vs[j] = -0.5 * z[j]; }
        rc = orc_nnfft(N, sigma1, sigma2, m1, m2, L1, a, c, nn, xs, g, NULL, NULL);
    }
    if (rc == 0) {
        for (long j = 0; j < nn; j++) { g[2 * j] *= w[j]; g[2 * j + 1] *= w[j]; }
        rc = orc_nnfft(N, sigma1, sigma2, m1, m2, nn, vs, g, L2, b, h, NULL, NULL);
    }
    free(z); free(w); free(xs); free(vs); free(g);
    return rc;
}

/* number of OpenMP threads the oracle uses */
int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* NFFT with equispaced frequencies (Sec. 2, the building block of the NNFFT; */
/* Sec. 6, the equispaced special cases of the fast sinc transform)          */
/* ------------------------------------------------------------------------ */

/*
 * The special case v_k = k / N, k in I_N, of (1.2), and its adjoint:
 *   forward  y_j = sum_{k in I_N} f_k exp(-2 pi i k x_j),       j in I_M
 *   adjoint  h_k = sum_{j in I_M} y_j exp(+2 pi i k x_j),       k in I_N
 * with the sinh-type window of Example 2.1 on an oversampled grid of length n:
 *   phi(t) = omega(n t / m),  phi_hat(k) = (m / n) omega_hat(m k / n).
 * Reading: the paper names the NFFT without listing its steps; these are the
 * standard ones (deconvolution, length-n DFT, window interpolation, and their
 * transposes).  n is the smallest even 2,3,5-smooth integer >= sigma N (as
 * for N2 of Algorithm 2.2), sigma_eff = n / N, beta = 2 pi m (1 - 1/(2 sigma_eff)).
 * Returns 0, 1 for invalid parameters (N < 2 odd, m < 2, sigma <= 1, 2m >= n),
 * 2 for a node outside [-1/2, 1/2], 3 for allocation failure.
 */
int orc_nfft_params(long N, double sigma, int m, long *n_out, double *beta_out)
{
    if (N < 2 || (N % 2) || m < 2 || !(sigma > 1.0)) return 1;
    long n = orc_ceil_tol(sigma * (double)N);
    if (n % 2) n++;
    while (!orc_is_smooth235(n)) n += 2;
    if (2 * m >= n) return 1;
    *n_out = n;
    *beta_out = 2.0 * ORC_PI * m * (1.0 - (double)N / (2.0 * (double)n));
    return 0;
}

/* l mod n in [0, n) */
static long orc_mod(long l, long n)
{
    long r = l % n;
    return r < 0 ? r + n : r;
}

int orc_nfft(long N, double sigma, int m, const double *f, long M, const double *x, double *y)
{
    long n;
    double beta;
    if (orc_nfft_params(N, sigma, m, &n, &beta)) return 1;
    for (long j = 0; j < M; j++) if (!(fabs(x[j]) <= 0.5)) return 2;
    double *g = calloc((size_t)(2 * n), sizeof(double));
    if (!g) return 3;
    /* deconvolution and the length-n DFT: g_l = sum_k f_k / (n phi_hat(k)) e^{-2 pi i k l / n} */
    long l;
#pragma omp parallel for schedule(static)
    for (l = 0; l < n; l++) {
        orc_acc_t re = {0, 0}, im = {0, 0};
        for (long k = -N / 2; k < N / 2; k++) {
            const double d = 1.0 / ((double)n * ((double)m / (double)n) * orc_omega_hat(m * (double)k / (double)n, beta));
            const double fr = f[2 * (k + N / 2)] * d, fi = f[2 * (k + N / 2) + 1] * d;
            double c, s;
            orc_expm2pi((double)orc_mod(k * l, n) / (double)n, &c, &s);
            orc_acc_add(&re, fr * c - fi * s);
            orc_acc_add(&im, fr * s + fi * c);
        }
        g[2 * l] = re.s + re.c;
        g[2 * l + 1] = im.s + im.c;
    }
    /* interpolation with the periodized window */
    long j;
#pragma omp parallel for schedule(static)
    for (j = 0; j < M; j++) {
        const double u = (double)n * x[j];
        const long c = (long)floor(u);
        double sr = 0.0, si = 0.0;
        for (long ll = c - m + 1; ll <= c + m; ll++) {
            const double w = orc_omega((u - (double)ll) / m, beta);
            const long q = orc_mod(ll, n);
            sr += g[2 * q] * w;
            si += g[2 * q + 1] * w;
        }
        y[2 * j] = sr;
        y[2 * j + 1] = si;
    }
    free(g);
    return 0;
}

int orc_nfft_adjoint(long N, double sigma, int m, long M, const double *x, const double *y, double *h)
{
    long n;
    double beta;
    if (orc_nfft_params(N, sigma, m, &n, &beta)) return 1;
    for (long j = 0; j < M; j++) if (!(fabs(x[j]) <= 0.5)) return 2;
    double *g = calloc((size_t)(2 * n), sizeof(double));
    if (!g) return 3;
    /* spreading with the periodized window (serial: plain and order-fixed) */
    for (long j = 0; j < M; j++) {
        const double u = (double)n * x[j];
        const long c = (long)floor(u);
        for (long ll = c - m + 1; ll <= c + m; ll++) {
            const double w = orc_omega((u - (double)ll) / m, beta);
            const long q = orc_mod(ll, n);
            g[2 * q] += y[2 * j] * w;
            g[2 * q + 1] += y[2 * j + 1] * w;
        }
    }
    /* length-n DFT with the + sign and the deconvolution */
    long k;
#pragma omp parallel for schedule(static)
    for (k = -N / 2; k < N / 2; k++) {
        orc_acc_t re = {0, 0}, im = {0, 0};
        for (long l = 0; l < n; l++) {
            double c, s;
            orc_expm2pi((double)orc_mod(k * l, n) / (double)n, &c, &s);
            s = -s;   /* exp(+2 pi i k l / n) */
            orc_acc_add(&re, g[2 * l] * c - g[2 * l + 1] * s);
            orc_acc_add(&im, g[2 * l] * s + g[2 * l + 1] * c);
        }
        const double d = 1.0 / ((double)n * ((double)m / (double)n) * orc_omega_hat(m * (double)k / (double)n, beta));
        h[2 * (k + N / 2)] = (re.s + re.c) * d;
        h[2 * (k + N / 2) + 1] = (im.s + im.c) * d;
    }
    free(g);
    return 0;
}
