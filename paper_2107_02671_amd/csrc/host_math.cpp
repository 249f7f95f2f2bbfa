// Host-side FP64 mathematics of the NNFFT plan.
#include "host_math.h"

#include <cmath>
#include <complex>
#include <cstring>

#include "internal.h"

namespace nnfft {

namespace {


int64_t ceil_with_slack(double x) { return (int64_t)std::ceil(x - 1e-9); }

bool only_235(int64_t n)
{
    if (n < 1) return false;
    for (int p : {2, 3, 5})
        while (n % p == 0) n /= p;
    return n == 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Sizes (Algorithm 2.2 input list, N* substitution of Sec. 2)
// ---------------------------------------------------------------------------
nnfft_status derive_params(int64_t N, double sigma1, double sigma2, int m1, int m2,
                           nnfft_info_t *out)
{
    std::memset(out, 0, sizeof(*out));
    if (N < 1 || m1 < 2 || m2 < 2 || !(sigma1 > 1.0) || !(sigma2 > 1.0) ||
        !std::isfinite(sigma1) || !std::isfinite(sigma2))
        return NNFFT_ERR_ARG;
    nnfft_info_t &P = *out;
    P.N = N;
    P.m1 = m1;
    P.m2 = m2;
    P.sigma1 = sigma1;
    P.sigma2 = sigma2;
    P.N_star = N + ceil_with_slack(2.0 * m1 / sigma1);
    P.N1 = 2 * ceil_with_slack(0.5 * sigma1 * (double)P.N_star);
    P.G1 = P.N1 + 2 * m1;
    // N2: even, only prime factors 2, 3, 5; largest not above sigma2 G1,
    // unless that leaves too little oversampling.
    const double want = sigma2 * (double)P.G1;
    int64_t down = (int64_t)std::floor(want + 1e-9) & ~(int64_t)1;
    while (down > 0 && !only_235(down)) down -= 2;
    const double floor_ok = std::min(sigma2, 1.25) * (double)P.G1;
    int64_t n2 = down;
    if (down <= P.G1 || (double)down < floor_ok - 1e-9) {
        int64_t up = ceil_with_slack(want);
        up += (up & 1);
        while (!only_235(up)) up += 2;
        n2 = up;
    }
    P.N2 = n2;
    P.sigma1_eff = (double)P.N1 / (double)P.N_star;
    P.sigma2_eff = (double)P.N2 / (double)P.G1;
    P.a = (double)P.G1 / (double)P.N1;
    P.beta1 = 2.0 * kPi * m1 * (1.0 - 0.5 / P.sigma1_eff);
    P.beta2 = 2.0 * kPi * m2 * (1.0 - 0.5 / P.sigma2_eff);
    if (2 * m1 >= P.N1) return NNFFT_ERR_ARG;
    if (2.0 * m2 > (1.0 - 1.0 / P.sigma1_eff) * (double)P.N2 + 1e-9) return NNFFT_ERR_ARG;
    // (4.2), Theorem 4.1, evaluated at the effective oversampling factors
    {
        const double s1 = P.sigma1_eff, s2 = P.sigma2_eff;
        const double a1 = (24.0 * std::pow((double)m1, 1.5) + 10.0);
        const double a2 = (24.0 * std::pow((double)m2, 1.5) + 10.0);
        const double e1 = std::exp(-2.0 * kPi * m1 * std::sqrt(1.0 - 1.0 / s1));
        const double grow = std::exp(2.0 * kPi * m1 * (1.0 - std::sqrt(1.0 - 1.0 / s1) - 0.5 / s1));
        const double e2 = std::exp(-2.0 * kPi * m2 * std::sqrt(1.0 - 1.0 / s2));
        P.bound_thm41 = a1 * e1 + a2 * (2.0 * P.N1 + 4.0 * m1) / std::sqrt(2.0 * m1 * kPi) * grow * e2;
        P.thm41_applies = (s1 >= 1.25 - 1e-12 && s1 <= 2.0 + 1e-12 && s2 >= 1.25 - 1e-12 &&
                           s2 <= 2.0 + 1e-12 && m2 >= m1) ? 1 : 0;
    }
    return NNFFT_OK;
}

// ---------------------------------------------------------------------------
// Window and window transform
// ---------------------------------------------------------------------------
double window_sinh(double u, double beta)
{
    const double q = (1.0 - u) * (1.0 + u);
    if (!(q > 0.0)) return 0.0;
    return std::sinh(beta * std::sqrt(q)) / std::sinh(beta);
}

// I_1(z)/z for y = z^2 >= 0 from its Taylor series (1/2) sum y^k/(4^k k!(k+1)!)
// evaluated in nested (Horner) form from the last kept term down.
// 1 / (k (k + 1)) for the nested series below
constexpr int kSeriesMax = 1000;   // terms of the I_1 series (enough for beta <= 2 pi 16)

static const double *inv_k_k1()
{
    static const std::vector<double> t = [] {
        std::vector<double> v(kSeriesMax + 2);
        v[0] = 0.0;
        for (int k = 1; k < (int)v.size(); ++k) v[k] = 1.0 / ((double)k * (double)(k + 1));
        return v;
    }();
    return t.data();
}

static double i1_over_z(double y)
{
    const double q = 0.25 * y;
    // the terms peak near k = sqrt(q); the tail past k = 20 + 2 sqrt(q) is
    // below 1e-18 of the sum for every q <= 2500 (beta <= 2 pi 16)
    const int K = std::min(kSeriesMax, 20 + (int)(2.0 * std::sqrt(q)));
    const double *r = inv_k_k1();
    double acc = 1.0;
    for (int k = K; k >= 1; --k) acc = 1.0 + acc * q * r[k];
    return 0.5 * acc;
}

double window_sinh_hat(double v, double beta)
{
    const double y = beta * beta - 4.0 * kPi * kPi * v * v;
    const double pre = kPi * beta / std::sinh(beta);
    if (y >= 0.0) return pre * i1_over_z(y);
    const double z = std::sqrt(-y);
    return pre * ::j1(z) / z;
}

// window_sinh_hat at n arguments, kLanes at a time: the nested I_1 series of
// the lanes run side by side (each lane from its own last term, so every
// value is bitwise the scalar one), which hides the latency of the series'
// dependent chain.
static void window_sinh_hat_many(const double *v, double *out, int64_t n, double beta)
{
    constexpr int kLanes = 8;
    const double pre = kPi * beta / std::sinh(beta);
    const double *r = inv_k_k1();
    for (int64_t i0 = 0; i0 < n; i0 += kLanes) {
        const int nl = (int)std::min<int64_t>(kLanes, n - i0);
        double q[kLanes], acc[kLanes];
        int K[kLanes], Kmax = 0;
        bool series = true;
        for (int l = 0; l < kLanes; ++l) {
            const double vl = v[i0 + std::min(l, nl - 1)];
            const double y = beta * beta - 4.0 * kPi * kPi * vl * vl;
            series = series && y >= 0.0;
            q[l] = 0.25 * y;
            K[l] = std::min(kSeriesMax, 20 + (int)(2.0 * std::sqrt(std::max(q[l], 0.0))));
            Kmax = std::max(Kmax, K[l]);
            acc[l] = 1.0;
        }
        if (!series) {   // an argument past the series' range: one at a time
            for (int l = 0; l < nl; ++l) out[i0 + l] = window_sinh_hat(v[i0 + l], beta);
            continue;
        }
        for (int k = Kmax; k >= 1; --k) {
            const double rk = r[k];
            for (int l = 0; l < kLanes; ++l) {
                const double nx = 1.0 + acc[l] * q[l] * rk;
                acc[l] = k <= K[l] ? nx : acc[l];
            }
        }
        for (int l = 0; l < nl; ++l) out[i0 + l] = pre * (0.5 * acc[l]);
    }
}

// I_0(z) - 1 = sum_{k >= 1} q^k / (k!)^2, q = z^2 / 4, nested from the last
// kept term down: q (1 + q/2^2 (1 + q/3^2 (1 + ...))).  The terms peak near
// k = sqrt(q); past k = 30 + 3 sqrt(q) the tail is below 1e-18 of the sum.
static double bessel_i0_minus_1(double z)
{
    const double q = 0.25 * z * z;
    const int K = 30 + (int)(3.0 * std::sqrt(q));
    double acc = 1.0;
    for (int k = K; k >= 2; --k) acc = 1.0 + acc * q / ((double)k * (double)k);
    return q * acc;
}

// ---------------------------------------------------------------------------
// Chebyshev fits
// ---------------------------------------------------------------------------
std::vector<double> cheb_nodes(int deg)
{
    std::vector<double> t(deg + 1);
    for (int j = 0; j <= deg; ++j) t[j] = std::cos(kPi * (j + 0.5) / (deg + 1));
    return t;
}

std::vector<double> cheb_fit(int deg, const std::vector<double> &f)
{
    // cos(pi k (j + 1/2) / (deg + 1)) depends on k (2j + 1) mod 4 (deg + 1)
    // only: one table of 4 (deg + 1) cosines
    const int P = 4 * (deg + 1);
    std::vector<double> ct((size_t)P);
    for (int e = 0; e < P; ++e) ct[(size_t)e] = std::cos(kPi * (0.5 * e) / (deg + 1));
    std::vector<double> c(deg + 1, 0.0);
    for (int k = 0; k <= deg; ++k) {
        double s = 0.0;
        for (int j = 0; j <= deg; ++j) s += f[j] * ct[(size_t)(((int64_t)k * (2 * j + 1)) % P)];
        c[k] = 2.0 * s / (deg + 1);
    }
    c[0] *= 0.5;
    return c;
}

double cheb_eval(const double *c, int deg, double t)
{
    double b1 = 0.0, b2 = 0.0;
    for (int k = deg; k >= 1; --k) {
        const double b0 = c[k] + 2.0 * t * b1 - b2;
        b2 = b1;
        b1 = b0;
    }
    return c[0] + t * b1 - b2;
}

// ---------------------------------------------------------------------------
// Window families of Example 2.1
// ---------------------------------------------------------------------------

// Cardinal B-spline of order n (support [0, n]) at z: with j = floor(z) and
// d = z - j, the n values M_n(d + i), i = 0..n-1, are built from M_1(d + i) =
// [i == 0] by M_{k+1}(y) = (y M_k(y) + (k + 1 - y) M_k(y - 1)) / k, and
// M_n(z) is the one with i = j.
static double bspline_cardinal(int n, double z)
{
    if (!(z > 0.0) || !(z < (double)n)) return 0.0;
    const int j = (int)std::floor(z);
    const double d = z - j;
    double val[2 * kMaxM + 1] = {1.0};
    for (int k = 1; k < n; ++k) {
        val[k] = 0.0;
        for (int i = k; i >= 0; --i) {
            const double y = d + i;
            val[i] = (y * val[i] + (i > 0 ? ((double)(k + 1) - y) * val[i - 1] : 0.0)) / (double)k;
        }
    }
    return val[j];
}

Window make_window(int kind, int m, double beta)
{
    Window w;
    w.kind = kind;
    w.m = m;
    w.beta = beta;
    if (kind == NNFFT_WINDOW_BSPLINE) w.norm = 1.0 / bspline_cardinal(2 * m, (double)m);
    return w;
}

double window_value(const Window &w, double u)
{
    switch (w.kind) {
    case NNFFT_WINDOW_BSPLINE:
        // B_2m(m u) / B_2m(0), B_2m(x) = M_2m(x + m)
        return std::fabs(u) < 1.0 ? bspline_cardinal(2 * w.m, w.m * (u + 1.0)) * w.norm : 0.0;
    case NNFFT_WINDOW_ALGEBRAIC: {
        const double q = (1.0 - u) * (1.0 + u);
        return q > 0.0 ? std::pow(q, w.beta - 0.5) : 0.0;
    }
    case NNFFT_WINDOW_KAISER_BESSEL: {
        const double q = (1.0 - u) * (1.0 + u);
        return q > 0.0 ? bessel_i0_minus_1(w.beta * std::sqrt(q)) / bessel_i0_minus_1(w.beta) : 0.0;
    }
    default:
        return window_sinh(u, w.beta);
    }
}

// log Gamma(x) through the reentrant form: the plain lgamma stores the sign
// in a process-wide variable, which races when planner threads run it at once.
static double log_gamma(double x)
{
    int sign = 0;
    return ::lgamma_r(x, &sign);
}

// (pi v)^(-b) J_b(2 pi v) for integer b (the algebraic window's b = 3 m): its
// power series where the argument is small against the order, else libm's jn.
static double bessel_ratio(double b, double v)
{
    const double a = kPi * std::fabs(v);
    if (a * a <= b + 1.0) {
        // sum_k (-1)^k a^(2k) / (k! (k + b)!), nested from the last kept term
        const int K = 40;
        double acc = 1.0;
        for (int k = K; k >= 1; --k) acc = 1.0 - acc * a * a / ((double)k * ((double)k + b));
        return acc * std::exp(-log_gamma(b + 1.0));
    }
    // libm's integer-order jn keeps no state (the C++ library's general-order
    // Bessel function calls the plain lgamma, which does), so threads may share it
    return ::jn((int)b, 2.0 * a) * std::exp(-b * std::log(a));
}

std::vector<double> kaiser_bessel_series(double beta)
{
    const double q = 0.25 * beta * beta, den = bessel_i0_minus_1(beta);
    std::vector<double> t;
    double term = 1.0 / den, sum = 0.0;
    for (int k = 1; k <= 1000; ++k) {
        term *= q / ((double)k * (double)k);
        t.push_back(term);
        sum += term;
        if ((double)k > std::sqrt(q) && term < 1e-18 * sum) break;
    }
    return t;
}

double window_hat(const Window &w, double v)
{
    switch (w.kind) {
    case NNFFT_WINDOW_KAISER_BESSEL: {
        // 2 / (I_0(beta) - 1) [sinh(z)/z - sin(2 pi v)/(2 pi v)], z^2 = beta^2 - 4 pi^2 v^2
        const double y = w.beta * w.beta - 4.0 * kPi * kPi * v * v;
        double s;
        if (y > 1e-8) s = std::sinh(std::sqrt(y)) / std::sqrt(y);
        else if (y < -1e-8) s = std::sin(std::sqrt(-y)) / std::sqrt(-y);
        else s = 1.0 + y / 6.0;
        const double a = 2.0 * kPi * v;
        const double c = std::fabs(a) < 1e-8 ? 1.0 - a * a / 6.0 : std::sin(a) / a;
        return 2.0 / bessel_i0_minus_1(w.beta) * (s - c);
    }
    case NNFFT_WINDOW_BSPLINE: {
        // sinc(pi v / m)^(2m) / (m B_2m(0))
        const double t = kPi * v / w.m;
        const double s = t == 0.0 ? 1.0 : std::sin(t) / t;
        return std::pow(s, 2.0 * w.m) * w.norm / (double)w.m;
    }
    case NNFFT_WINDOW_ALGEBRAIC: {
        // pi (2b)! / (4^b b!) (pi v)^(-b) J_b(2 pi v)
        const double b = w.beta;
        const double lc = std::log(kPi) + log_gamma(2.0 * b + 1.0) - b * std::log(4.0) - log_gamma(b + 1.0);
        return std::exp(lc) * bessel_ratio(b, v);
    }
    default:
        return window_sinh_hat(v, w.beta);
    }
}

void window_hat_many(const Window &w, const double *v, double *out, int64_t n)
{
    if (w.kind == NNFFT_WINDOW_SINH) {
        window_sinh_hat_many(v, out, n, w.beta);
        return;
    }
    for (int64_t i = 0; i < n; ++i) out[i] = window_hat(w, v[i]);
}

std::vector<double> fit_window_taps(const Window &w, int deg, double *max_err)
{
    const int m = w.m;
    std::vector<double> out((size_t)(2 * m) * (deg + 1));
    const std::vector<double> tn = cheb_nodes(deg);
    double worst = 0.0;
    for (int r = 0; r < 2 * m; ++r) {
        std::vector<double> f(deg + 1);
        for (int j = 0; j <= deg; ++j) {
            const double x = 0.5 * (tn[j] + 1.0);
            f[j] = window_value(w, (r - m + 1 - x) / m);
        }
        std::vector<double> c = cheb_fit(deg, f);
        for (int k = 0; k <= deg; ++k) out[(size_t)r * (deg + 1) + k] = c[k];
        // the error of the interpolant has deg + 1 lobes, denser toward the
        // ends: eight check points per lobe, uniform in the angle of t = 2x - 1
        const int G = 8 * (deg + 1);
        for (int i = 0; i <= G; ++i) {
            const double t = std::cos(kPi * i / G), x = 0.5 * (t + 1.0);
            const double e = std::fabs(cheb_eval(c.data(), deg, t) - window_value(w, (r - m + 1 - x) / m));
            worst = std::max(worst, e);
        }
    }
    *max_err = worst;
    return out;
}

std::vector<double> fit_inverse_phi1(const nnfft_info_t &P, double tol, int max_deg,
                                     double *max_rel_err)
{
    // phi_hat_1(N* x) = (m1/N1) omega_hat_1(m1 N* x / N1)
    const Window w1 = make_window(P.window, P.m1, P.beta1);
    // 1 / phi_hat_1(N* x) at the points x[0..n)
    auto inv_many = [&](const std::vector<double> &x, std::vector<double> &out) {
        std::vector<double> v(x.size());
        for (size_t i = 0; i < x.size(); ++i) v[i] = (double)P.m1 * (double)P.N_star * x[i] / (double)P.N1;
        out.resize(x.size());
        window_hat_many(w1, v.data(), out.data(), (int64_t)v.size());
        for (double &o : out) o = 1.0 / ((double)P.m1 / (double)P.N1 * o);
    };
    // reference values on the check grid, shared by every degree tried:
    // uniform in the angle of t = 8 x^2 - 1 (dense toward both ends, where
    // the error of a Chebyshev interpolant peaks)
    constexpr int kGrid = 400;
    std::vector<double> tg(kGrid + 1), xg(kGrid + 1), ref;
    for (int i = 0; i <= kGrid; ++i) {
        tg[i] = std::cos(kPi * i / kGrid);
        xg[i] = std::sqrt(std::max(0.0, (tg[i] + 1.0) / 8.0));
    }
    inv_many(xg, ref);
    std::vector<double> best;
    double best_err = 1e300;
    for (int deg = 4; deg <= max_deg; deg += 2) {
        const std::vector<double> tn = cheb_nodes(deg);
        std::vector<double> xn(deg + 1), f;
        for (int j = 0; j <= deg; ++j) xn[j] = std::sqrt((tn[j] + 1.0) / 8.0);
        inv_many(xn, f);
        std::vector<double> c = cheb_fit(deg, f);
        double err = 0.0;
        for (int i = 0; i <= kGrid; ++i) err = std::max(err, std::fabs(cheb_eval(c.data(), deg, tg[i]) / ref[i] - 1.0));
        if (err < best_err) {
            best_err = err;
            best = c;
        }
        if (err <= tol) break;
    }
    *max_rel_err = best_err;
    return best;
}

// ---------------------------------------------------------------------------
// Twiddles: exp(-2 pi i q / n), exact at multiples of a quarter turn
// ---------------------------------------------------------------------------
std::vector<double> twiddles(int64_t n)
{
    std::vector<double> tw((size_t)(2 * n));
    // cos and sin of (pi/2) r / n, r in [0, n): evaluated once per r <= n/2
    // and taken from the complementary angle (pi/2) (n - r) / n above that
    std::vector<double> cr((size_t)n / 2 + 1), sr((size_t)n / 2 + 1);
    std::vector<char> have((size_t)n / 2 + 1, 0);
    auto quarter = [&](int64_t r, double &c, double &s) {
        const bool mirror = 2 * r > n;
        const int64_t a = mirror ? n - r : r;
        if (!have[a]) {
            const double th = 0.5 * kPi * (double)a / (double)n;
            cr[a] = std::cos(th);
            sr[a] = std::sin(th);
            have[a] = 1;
        }
        c = mirror ? sr[a] : cr[a];
        s = mirror ? cr[a] : sr[a];
    };
    for (int64_t q = 0; q < n; ++q) {
        const int64_t q4 = 4 * q;
        const int64_t quad = q4 / n;          // 0..3
        const int64_t rem = q4 - quad * n;    // angle in the quadrant = (pi/2) rem / n
        double c, s;
        quarter(rem, c, s);
        // exp(-i (quad pi/2 + th))
        double re, im;
        switch (quad) {
        case 0: re = c; im = -s; break;
        case 1: re = -s; im = -c; break;
        case 2: re = -c; im = s; break;
        default: re = s; im = c; break;
        }
        tw[2 * q] = re;
        tw[2 * q + 1] = im;
    }
    return tw;
}

// ---------------------------------------------------------------------------
// Quadrature rules for sinc(N pi x) = (1/2) int e^{-pi i N t x} dt (Sec. 5)
// ---------------------------------------------------------------------------
void gauss_legendre_rule(int64_t n, std::vector<double> &z, std::vector<double> &w)
{
    // Newton's method on P_n from Tricomi's asymptotic node estimate, with
    // (1 - t^2) P_n'(t) = n (P_{n-1}(t) - t P_n(t)); the weight
    // W = 2 / ((1 - t^2) P_n'(t)^2) is evaluated with that derivative at the
    // final node, which keeps it accurate where 1 - t^2 is small.
    z.assign((size_t)n, 0.0);
    w.assign((size_t)n, 0.0);
    const double nn = (double)n;
    auto legendre = [&](double t, double &p, double &pm) {
        pm = 1.0;
        p = t;
        for (int64_t k = 2; k <= n; ++k) {
            const double pk = ((2.0 * k - 1.0) * t * p - (k - 1.0) * pm) / (double)k;
            pm = p;
            p = pk;
        }
    };
    for (int64_t i = 1; i <= (n + 1) / 2; ++i) {
        const double th = kPi * (4.0 * i - 1.0) / (4.0 * nn + 2.0);
        double t = (1.0 - (nn - 1.0) / (8.0 * nn * nn * nn)) * std::cos(th);
        double p, pm;
        // quadratic convergence: once a step is below 1e-14 of the node (or
        // of 1e-3 for nodes near 0), the node is at the rounding floor
        for (int it = 0; it < 60; ++it) {
            legendre(t, p, pm);
            const double dp = nn * (pm - t * p) / ((1.0 - t) * (1.0 + t));
            const double step = p / dp;
            t -= step;
            if (std::fabs(step) <= 1e-14 * std::max(std::fabs(t), 1e-3)) break;
        }
        legendre(t, p, pm);
        const double omt2 = (1.0 - t) * (1.0 + t);
        const double dp = nn * (pm - t * p) / omt2;
        const double W = 2.0 / (omt2 * dp * dp);
        z[(size_t)(i - 1)] = t;
        z[(size_t)(n - i)] = -t;
        w[(size_t)(i - 1)] = 0.5 * W;
        w[(size_t)(n - i)] = 0.5 * W;
    }
    if (n % 2) z[(size_t)(n / 2)] = 0.0;
}

namespace {
// in-place iterative radix-2 complex FFT (forward), n a power of two
void fft_pow2(std::vector<std::complex<double>> &a)
{
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const double ang = -2.0 * kPi / (double)len;
        for (size_t i = 0; i < n; i += len)
            for (size_t k = 0; k < len / 2; ++k) {
                const std::complex<double> wk(std::cos(ang * k), std::sin(ang * k));
                const std::complex<double> u = a[i + k], v = a[i + k + len / 2] * wk;
                a[i + k] = u + v;
                a[i + k + len / 2] = u - v;
            }
    }
}
}  // namespace

void clenshaw_curtis_rule(int64_t n, std::vector<double> &z, std::vector<double> &w)
{
    // Chebyshev points z_k = cos(k pi / n) and the weights of Algorithm 5.4:
    // a_{2j} = eps(2j) 2/(1 - 4 j^2), a_odd = 0; a_hat = C^I_{n+1} a (DCT-I);
    // w_k = eps(k) a_hat_k / sqrt(2n).  The DCT-I is done through a length-2n
    // FFT of the even extension when n is a power of two, directly otherwise.
    z.assign((size_t)(n + 1), 0.0);
    w.assign((size_t)(n + 1), 0.0);
    const double r2 = std::sqrt(0.5);
    auto eps = [&](int64_t j) { return (j == 0 || j == n) ? r2 : 1.0; };
    std::vector<double> a((size_t)(n + 1), 0.0);
    for (int64_t j = 0; 2 * j <= n; ++j)
        a[(size_t)(2 * j)] = eps(2 * j) * 2.0 / (1.0 - 4.0 * (double)j * (double)j);
    // b_j = eps(j) a_j ; DCT-I core: S_k = sum_j b_j cos(j k pi / n)
    std::vector<double> S((size_t)(n + 1), 0.0);
    if (n >= 2 && (n & (n - 1)) == 0) {
        std::vector<std::complex<double>> e((size_t)(2 * n));
        for (int64_t j = 0; j <= n; ++j) e[(size_t)j] = eps(j) * a[(size_t)j];
        for (int64_t j = 1; j < n; ++j) e[(size_t)(2 * n - j)] = e[(size_t)j];
        fft_pow2(e);
        // E_k = b_0 + (-1)^k b_n + 2 sum_{0<j<n} b_j cos(j k pi / n), so
        // S_k = (E_k + b_0 + (-1)^k b_n) / 2
        for (int64_t k = 0; k <= n; ++k)
            S[(size_t)k] = 0.5 * (e[(size_t)k].real() + eps(0) * a[0] +
                                  ((k % 2) ? -1.0 : 1.0) * eps(n) * a[(size_t)n]);
    } else {
        for (int64_t k = 0; k <= n; ++k) {
            double s = 0.0;
            for (int64_t j = 0; j <= n; ++j) {
                const int64_t q = (j * k) % (2 * n);
                s += eps(j) * a[(size_t)j] * std::cos(kPi * (double)q / (double)n);
            }
            S[(size_t)k] = s;
        }
    }
    const double scale = std::sqrt(2.0 / (double)n);
    for (int64_t k = 0; k <= n; ++k) {
        const double ahat = scale * eps(k) * S[(size_t)k];
        w[(size_t)k] = eps(k) * ahat / std::sqrt(2.0 * (double)n);
        z[(size_t)k] = std::sin(kPi * (double)(n - 2 * k) / (2.0 * (double)n));
    }
}

std::vector<int> radix_passes(int64_t n)
{
    std::vector<int> r;
    if (n < 1) return {};
    while (n % 8 == 0 && n > 4) { r.push_back(8); n /= 8; }
    while (n % 4 == 0) { r.push_back(4); n /= 4; }
    while (n % 2 == 0) { r.push_back(2); n /= 2; }
    while (n % 5 == 0) { r.push_back(5); n /= 5; }
    while (n % 3 == 0) { r.push_back(3); n /= 3; }
    if (n != 1) return {};
    return r;
}

}  // namespace nnfft
