// Host-side FP64 mathematics of the plan: sizes, window transforms,
// Chebyshev fits, twiddles and quadrature rules.
#pragma once

#include <cstdint>
#include <vector>

#include "../../include/nnfft.h"

namespace nnfft {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Sizes of Algorithm 2.2 (see nnfft_derive_params in nnfft.h for the readings).
nnfft_status derive_params(int64_t N, double sigma1, double sigma2, int m1, int m2,
                           nnfft_info_t *out);

// sinh-type window of Example 2.1: sinh(beta sqrt(1 - u^2)) / sinh(beta).
double window_sinh(double u, double beta);

// Its Fourier transform (2.1) for |v| <= beta / (2 pi) (the only branch the
// algorithm evaluates, see the remark after (2.1) and Sec. 4).
double window_sinh_hat(double v, double beta);

// Chebyshev interpolant of degree `deg` on [-1, 1] (nodes of the first kind).
std::vector<double> cheb_fit(int deg, const std::vector<double> &fvals_at_nodes);
std::vector<double> cheb_nodes(int deg);
double cheb_eval(const double *c, int deg, double t);

// A window of Example 2.1 (family nnfft_window) with its parameters.
struct Window {
    int kind = NNFFT_WINDOW_SINH;
    int m = 2;
    double beta = 0.0;    // sinh: shape parameter; algebraic: exponent parameter (3m)
    double norm = 1.0;    // B-spline: 1 / M_2m(m), the value at 0 of the unscaled spline
};
Window make_window(int kind, int m, double beta);
// omega(u) of the family, 0 for |u| >= 1.
double window_value(const Window &w, double u);
// Its Fourier transform for |v| <= m/2 (the algorithm needs |v| <= m/(2 sigma)).
double window_hat(const Window &w, double v);
// window_hat at v[0..n) into out[0..n), each value bitwise the scalar one
// (sinh windows: several series evaluated side by side).
void window_hat_many(const Window &w, const double *v, double *out, int64_t n);

// Continuous Kaiser-Bessel window as a power series in s = 1 - u^2:
// omega(u) = sum_{k >= 1} t_k s^k, t_k = (beta^2/4)^k / ((k!)^2 (I_0(beta) - 1));
// returns t_1 .. t_K with the tail past K below 1e-18 of the sum (the FP64
// kernels evaluate it by Horner's rule).
std::vector<double> kaiser_bessel_series(double beta);

// Tap r (0 <= r < 2m) of a point at fractional offset x in [0, 1) of its cell
// carries the weight omega((r - m + 1 - x) / m); as a function of t = 2x - 1
// it is fitted by a degree-`deg` Chebyshev series (FP32 path: degree kDeg;
// FP64 path with B-spline windows: degree 2m - 1, where each tap is one
// polynomial piece and the series is exact).  Returns the [2m][deg+1]
// coefficients and the max abs error on a fine grid.
std::vector<double> fit_window_taps(const Window &w, int deg, double *max_err);

// Chebyshev series of 1/phi_hat_1(N* x) in t = 8 x^2 - 1, |x| <= 1/2, of the
// smallest degree <= max_deg whose max relative error is <= tol (else the
// best found; *max_rel_err tells).  The window is P.window with m1, beta1.
std::vector<double> fit_inverse_phi1(const nnfft_info_t &P, double tol, int max_deg,
                                     double *max_rel_err);

// exp(-2 pi i q / n) for q = 0..n-1, interleaved (re, im).
std::vector<double> twiddles(int64_t n);

// Quadrature rules on [-1, 1] with weights scaled to sum 1.
void gauss_legendre_rule(int64_t n, std::vector<double> &z, std::vector<double> &w);
void clenshaw_curtis_rule(int64_t n, std::vector<double> &z, std::vector<double> &w);

// Radix factorization of n over {8, 4, 2, 5, 3}; empty if n has another prime.
std::vector<int> radix_passes(int64_t n);

}  // namespace nnfft
