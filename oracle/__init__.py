"""FP64 CPU oracle for the NNFFT (Algorithm 2.2) and the fast sinc transform
(Algorithm 6.1) of Kircheis, Potts, Tasche (arXiv 2107.02671).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark are the only users.  It shares no code with the GPU
library and never imports it.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double, OpenMP only for
parallel loops); this module marshals numpy arrays and holds the closed-form
error bounds, which are one-line formulas from the paper.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None


class _Params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_long), ("N_star", ctypes.c_long), ("N1", ctypes.c_long),
                ("G1", ctypes.c_long), ("N2", ctypes.c_long), ("m1", ctypes.c_int),
                ("m2", ctypes.c_int), ("sigma1", ctypes.c_double), ("sigma2", ctypes.c_double),
                ("sigma1_eff", ctypes.c_double), ("sigma2_eff", ctypes.c_double),
                ("a", ctypes.c_double), ("beta1", ctypes.c_double), ("beta2", ctypes.c_double),
                ("window", ctypes.c_int)]


def lib():
    global _lib
    if _lib is None:
        from . import build as _build
        path = _build.build(force=False)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.orc_params.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, ctypes.POINTER(_Params)]
        L.orc_params_window.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, ctypes.c_int, ctypes.POINTER(_Params)]
        L.orc_window.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double]
        L.orc_window.restype = ctypes.c_double
        L.orc_window_hat.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_int, ctypes.c_double]
        L.orc_window_hat.restype = ctypes.c_double
        L.orc_bspline_cardinal.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_bspline_cardinal.restype = ctypes.c_double
        L.orc_omega.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_omega.restype = ctypes.c_double
        L.orc_omega_hat.argtypes = [ctypes.c_double, ctypes.c_double]
        L.orc_omega_hat.restype = ctypes.c_double
        L.orc_sinc_pi.argtypes = [ctypes.c_double]
        L.orc_i0_minus_1.argtypes = [ctypes.c_double]
        L.orc_i0_minus_1.restype = ctypes.c_double
        L.orc_sinc_pi.restype = ctypes.c_double
        L.orc_direct.argtypes = [ctypes.c_long, ctypes.c_long, dp, dp, ctypes.c_long, dp, dp]
        L.orc_sinc_direct.argtypes = [ctypes.c_long, ctypes.c_long, dp, dp, ctypes.c_long, dp, dp]
        L.orc_nnfft.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                ctypes.c_int, ctypes.c_long, dp, dp, ctypes.c_long, dp, dp, dp, dp]
        L.orc_nnfft_window.argtypes = [ctypes.c_int] + L.orc_nnfft.argtypes
        L.orc_gauss_legendre.argtypes = [ctypes.c_long, dp, dp]
        L.orc_clenshaw_curtis.argtypes = [ctypes.c_long, dp, dp]
        L.orc_sinc_fast.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.c_int, ctypes.c_long, ctypes.c_long, dp, dp,
                                    ctypes.c_long, dp, dp]
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_nfft_params.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_long),
                                      ctypes.POINTER(ctypes.c_double)]
        L.orc_nfft.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_int, dp, ctypes.c_long, dp, dp]
        L.orc_nfft_adjoint.argtypes = [ctypes.c_long, ctypes.c_double, ctypes.c_int, ctypes.c_long, dp, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _real(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _cplx(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.complex128))


@dataclass(frozen=True)
class Params:
    N: int
    N_star: int
    N1: int
    G1: int
    N2: int
    m1: int
    m2: int
    sigma1: float
    sigma2: float
    sigma1_eff: float
    sigma2_eff: float
    a: float
    beta1: float
    beta2: float
    window: int


# window families of Example 2.1, and the continuous Kaiser-Bessel window
# (the Kaiser-Bessel family of Example 4.2's comparison runs, in the form that
# belongs to the set Omega of Sec. 2: (I_0(beta sqrt(1 - x^2)) - 1) / (I_0(beta) - 1),
# beta = 2 pi m (1 - 1/(2 sigma)))
WIN_SINH, WIN_BSPLINE, WIN_ALGEBRAIC, WIN_KAISER_BESSEL = 0, 1, 2, 3


def params(N, sigma1, sigma2, m1, m2, window=WIN_SINH) -> Params:
    p = _Params()
    rc = lib().orc_params_window(int(N), float(sigma1), float(sigma2), int(m1), int(m2), int(window),
                                 ctypes.byref(p))
    if rc:
        raise ValueError(f"invalid NNFFT parameters N={N} sigma=({sigma1},{sigma2}) m=({m1},{m2}) "
                         f"window={window}")
    return Params(**{f: getattr(p, f) for f, _ in _Params._fields_})


def window(kind, u, m, beta) -> np.ndarray:
    """omega(u) of family `kind` (Example 2.1); beta is ignored by the B-spline."""
    u = np.asarray(u, dtype=np.float64)
    return np.vectorize(lambda t: lib().orc_window(int(kind), float(t), int(m), float(beta)),
                        otypes=[float])(u)


def window_hat(kind, v, m, beta) -> np.ndarray:
    """The Fourier transform of window(kind, ., m, beta) in its closed form (Example 2.1)."""
    v = np.asarray(v, dtype=np.float64)
    return np.vectorize(lambda t: lib().orc_window_hat(int(kind), float(t), int(m), float(beta)),
                        otypes=[float])(v)


def bspline_cardinal(n, y) -> np.ndarray:
    """Cardinal B-spline M_n(y) of order n on [0, n]; B_n(x) = M_n(x + n/2)."""
    y = np.asarray(y, dtype=np.float64)
    return np.vectorize(lambda t: lib().orc_bspline_cardinal(int(n), float(t)), otypes=[float])(y)


def omega(u, beta) -> np.ndarray:
    u = np.asarray(u, dtype=np.float64)
    return np.vectorize(lambda t: lib().orc_omega(float(t), float(beta)), otypes=[float])(u)


def omega_hat(v, beta) -> np.ndarray:
    v = np.asarray(v, dtype=np.float64)
    return np.vectorize(lambda t: lib().orc_omega_hat(float(t), float(beta)), otypes=[float])(v)


def sinc_pi(d) -> np.ndarray:
    d = np.asarray(d, dtype=np.float64)
    return np.vectorize(lambda t: lib().orc_sinc_pi(float(t)), otypes=[float])(d)


def direct(N, v, f, x) -> np.ndarray:
    """(1.2): y_j = sum_k f_k exp(-2 pi i N v_k x_j), FP64, compensated sums."""
    v, x, f = _real(v), _real(x), _cplx(f)
    y = np.zeros(len(x), dtype=np.complex128)
    lib().orc_direct(int(N), len(v), _dp(v), _dp(f.view(np.float64)), len(x), _dp(x),
                     _dp(y.view(np.float64)))
    return y


def nnfft(N, v, f, x, sigma1=2.0, sigma2=2.0, m1=4, m2=4, return_steps=False, window=WIN_SINH):
    """Algorithm 2.2 in FP64 with a direct DFT for step 3 (both windows of
    family `window`).

    Step 3 forms only the h_s that step 4 reads for these x, so outputs at a
    few nodes of a large-bandwidth problem cost a few direct sums of length
    G1 each.  return_steps=True forms all of them and also returns g (step 1,
    length G1, index l + G1/2) and h (step 3, length N2, index s + N2/2)."""
    v, x, f = _real(v), _real(x), _cplx(f)
    P = params(N, sigma1, sigma2, m1, m2, window)
    y = np.zeros(len(x), dtype=np.complex128)
    g = h = None
    gp = hp = None
    if return_steps:
        g = np.zeros(P.G1, dtype=np.complex128)
        h = np.zeros(P.N2, dtype=np.complex128)
        gp, hp = _dp(g.view(np.float64)), _dp(h.view(np.float64))
    rc = lib().orc_nnfft_window(int(window), int(N), float(sigma1), float(sigma2), int(m1), int(m2), len(v),
                                _dp(v), _dp(f.view(np.float64)), len(x), _dp(x), _dp(y.view(np.float64)),
                                gp, hp)
    if rc == 2:
        raise ValueError("node outside [-1/2, 1/2]")
    if rc:
        raise RuntimeError(f"orc_nnfft failed with code {rc}")
    return (y, g, h) if return_steps else y


def nfft_params(N, sigma, m):
    """(n, beta) of the oracle NFFT: n the smallest even 2,3,5-smooth integer >= sigma N."""
    n = ctypes.c_long()
    beta = ctypes.c_double()
    if lib().orc_nfft_params(int(N), float(sigma), int(m), ctypes.byref(n), ctypes.byref(beta)):
        raise ValueError("invalid NFFT parameters")
    return n.value, beta.value


def nfft(N, f, x, sigma=2.0, m=6) -> np.ndarray:
    """y_j = sum_{k in I_N} f_k exp(-2 pi i k x_j) by the NFFT steps (f index k + N/2)."""
    x, f = _real(x), _cplx(f)
    y = np.zeros(len(x), dtype=np.complex128)
    rc = lib().orc_nfft(int(N), float(sigma), int(m), _dp(f.view(np.float64)), len(x), _dp(x),
                        _dp(y.view(np.float64)))
    if rc == 2:
        raise ValueError("node outside [-1/2, 1/2]")
    if rc:
        raise RuntimeError(f"orc_nfft failed with code {rc}")
    return y


def nfft_adjoint(N, y, x, sigma=2.0, m=6) -> np.ndarray:
    """h_k = sum_j y_j exp(+2 pi i k x_j), k in I_N (index k + N/2), by the transposed steps."""
    x, y = _real(x), _cplx(y)
    h = np.zeros(int(N), dtype=np.complex128)
    rc = lib().orc_nfft_adjoint(int(N), float(sigma), int(m), len(x), _dp(x), _dp(y.view(np.float64)),
                                _dp(h.view(np.float64)))
    if rc == 2:
        raise ValueError("node outside [-1/2, 1/2]")
    if rc:
        raise RuntimeError(f"orc_nfft_adjoint failed with code {rc}")
    return h


def sinc_direct(N, a, c, b) -> np.ndarray:
    """(6.2): h(b_l) = sum_k c_k sinc(N pi (b_l - a_k)); complex output."""
    a, b, c = _real(a), _real(b), _cplx(c)
    h = np.zeros(len(b), dtype=np.complex128)
    lib().orc_sinc_direct(int(N), len(a), _dp(a), _dp(c.view(np.float64)), len(b), _dp(b),
                          _dp(h.view(np.float64)))
    return h


def gauss_legendre(n):
    """Gauss-Legendre nodes (decreasing) and halved weights (sum = 1)."""
    z = np.zeros(n)
    w = np.zeros(n)
    if lib().orc_gauss_legendre(int(n), _dp(z), _dp(w)):
        raise ValueError("n must be >= 1")
    return z, w


def clenshaw_curtis(n):
    """Chebyshev points z_k = cos(k pi/n), k = 0..n, and the weights of (5.4)."""
    z = np.zeros(n + 1)
    w = np.zeros(n + 1)
    if lib().orc_clenshaw_curtis(int(n), _dp(z), _dp(w)):
        raise ValueError("n must be >= 1")
    return z, w


QUAD_GAUSS_LEGENDRE = 0
QUAD_CLENSHAW_CURTIS = 1


def sinc_fast(N, a, c, b, nq, quad=QUAD_GAUSS_LEGENDRE, sigma1=2.0, sigma2=2.0, m1=6, m2=6):
    """Algorithm 6.1 built from two FP64 oracle NNFFTs."""
    a, b, c = _real(a), _real(b), _cplx(c)
    h = np.zeros(len(b), dtype=np.complex128)
    rc = lib().orc_sinc_fast(int(N), float(sigma1), float(sigma2), int(m1), int(m2), int(quad),
                             int(nq), len(a), _dp(a), _dp(c.view(np.float64)), len(b), _dp(b),
                             _dp(h.view(np.float64)))
    if rc:
        raise RuntimeError(f"orc_sinc_fast failed with code {rc}")
    return h


def sinc_fast_equispaced(N, a, c, b, nq, quad=QUAD_GAUSS_LEGENDRE, sigma=2.0, m=6,
                         step1_nfft=False, step3_nfft=False, sigma2=2.0, m2=6):
    """Algorithm 6.1 with the equispaced special cases of Sec. 6.

    step1_nfft: a_k = k / L1 (k in I_L1, N <= L1), so step 1 is the NFFT with L1
    frequencies at the nodes N z_j / (2 L1); step3_nfft: b_l = l / N (l in I_N),
    so step 3 is the adjoint NFFT with N frequencies at the nodes z_j / 2.  The
    NFFTs use (sigma, m); an NNFFT step that remains uses (sigma, sigma2, m, m2).
    """
    a, b, c = _real(a), _real(b), _cplx(c)
    z, w = gauss_legendre(nq) if quad == QUAD_GAUSS_LEGENDRE else clenshaw_curtis(nq)
    if step1_nfft:
        L1 = len(a)
        g = nfft(L1, c, N * z / (2.0 * L1), sigma, m)
    else:
        g = nnfft(N, a, c, z / 2.0, sigma, sigma2, m, m2)
    g = g * w
    if step3_nfft:
        return nfft_adjoint(N, g, z / 2.0, sigma, m)
    return nnfft(N, -z / 2.0, g, b, sigma, sigma2, m, m2)


def num_threads() -> int:
    return int(lib().orc_num_threads())


# --------------------------------------------------------------------------
# Closed-form error bounds (formulas transcribed from the theorems)
# --------------------------------------------------------------------------

# Theorem 4.1 slip: the proof bounds I_1(x) from below by (2/5) x^(-1/2) e^x
# for x >= 4 pi / sqrt(5); the true constant there is sqrt(x0) e^(-x0) I_1(x0)
# = 0.3705 (x0 = 4 pi / sqrt(5)), so the factor of the second term of (4.2)
# holds only after multiplying it by 0.4 / 0.3705 = 1.08.  The first term is
# untouched (its bound (4.3) does not use that inequality).
THM41_SLIP = 1.08


def thm41_terms(N1, m1, m2, sigma1, sigma2):
    """The three factors of (4.2), Theorem 4.1, as Theorem 3.5 composes them:
      E1 = (24 m1^(3/2) + 10) e^(-2 pi m1 sqrt(1 - 1/sigma1))   bound (4.3) on E_sigma1(phi_1)
      F  = (2 N1 + 4 m1) / sqrt(2 pi m1) e^(2 pi m1 (1 - sqrt(1 - 1/sigma1) - 1/(2 sigma1)))
                                                              bound on a / phi_hat_1(N/2)
      E2 = (24 m2^(3/2) + 10) e^(-2 pi m2 sqrt(1 - 1/sigma2))   bound (4.3) on E_sigma2(phi_2)
    with (4.2) = E1 + F E2 (2 N1 a = 2 N1 + 4 m1 by (2.6))."""
    E1 = (24 * m1 ** 1.5 + 10) * math.exp(-2 * math.pi * m1 * math.sqrt(1 - 1 / sigma1))
    F = ((2 * N1 + 4 * m1) / math.sqrt(2 * m1 * math.pi)
         * math.exp(2 * math.pi * m1 * (1 - math.sqrt(1 - 1 / sigma1) - 1 / (2 * sigma1))))
    E2 = (24 * m2 ** 1.5 + 10) * math.exp(-2 * math.pi * m2 * math.sqrt(1 - 1 / sigma2))
    return E1, F, E2


def bound_thm41(N1, m1, m2, sigma1, sigma2) -> float:
    """E(phi_sinh) of (4.2), Theorem 4.1, as printed: bound on E_paper for sinh windows."""
    E1, F, E2 = thm41_terms(N1, m1, m2, sigma1, sigma2)
    return E1 + F * E2


def bound_thm41_gate(N1, m1, m2, sigma1, sigma2) -> float:
    """(4.2) with the slip of its proof corrected: E1 + 1.08 F E2 (THM41_SLIP)."""
    E1, F, E2 = thm41_terms(N1, m1, m2, sigma1, sigma2)
    return E1 + THM41_SLIP * F * E2


def thm34_constants(kind, m, sigma, beta):
    """Decay constants (c1, c2, mu) of Theorem 3.4's condition for the windows
    of Example 2.1, holding for every v:
      B-spline   |omega_hat(v)| <= (m / (pi |v|))^(2m) / (m B_2m(0)), mu = 2m
                 (|sin| <= 1 in the power of sinc);
      algebraic  |omega_hat(v)| <= C (pi |v|)^(-beta), mu = beta,
                 C = pi (2 beta)! / (4^beta beta!) (|J_beta| <= 1);
    c2 is the coefficient of |v|^(-mu) and c1 the envelope at |v| =
    m (1 - 1/(2 sigma)), where the interval of the theorem starts (the envelope
    decreases, so it bounds |omega_hat| on the whole interval).

    Continuous Kaiser-Bessel (beta = 2 pi m (1 - 1/(2 sigma)), so the interval
    starts at the branch point |v| = beta / (2 pi)): with K = 2 / (I_0(beta) - 1),
    b = 2 pi |v| and a = sqrt(b^2 - beta^2),
      omega_hat(v) = K (sin(a)/a - sin(b)/b),
    so |omega_hat| <= K (1 + 1/beta) on the interval (|sin t / t| <= 1 and
    b >= beta) and, beyond it (b >= b0 = beta (2 sigma + 1) / (2 sigma - 1),
    a >= rho b with rho = sqrt(8 sigma) / (2 sigma + 1)), by the mean value
    theorem with |d/dt (sin t / t)| <= (1 + 1/t) / t and b - a = beta^2 / (a + b),
      |omega_hat| <= K beta^2 (1 + 1/(rho b0)) / (rho (1 + rho) b^2):
    mu = 2, c1 = K (1 + 1/beta), c2 = K beta^2 (1 + 1/(rho b0)) / (4 pi^2 rho (1 + rho))."""
    lo = m * (1.0 - 1.0 / (2.0 * sigma))
    if kind == WIN_KAISER_BESSEL:
        if not abs(beta - 2.0 * math.pi * lo) <= 1e-12 * beta:
            raise ValueError("the Kaiser-Bessel constants need beta = 2 pi m (1 - 1/(2 sigma))")
        K = 2.0 / float(lib().orc_i0_minus_1(float(beta)))
        rho = math.sqrt(8.0 * sigma) / (2.0 * sigma + 1.0)
        b0 = beta * (2.0 * sigma + 1.0) / (2.0 * sigma - 1.0)
        c1 = K * (1.0 + 1.0 / beta)
        c2 = K * beta * beta * (1.0 + 1.0 / (rho * b0)) / (4.0 * math.pi ** 2 * rho * (1.0 + rho))
        return c1, c2, 2.0
    if kind == WIN_BSPLINE:
        b0 = float(bspline_cardinal(2 * m, m))
        c2 = (m / math.pi) ** (2 * m) / (m * b0)
        mu = 2.0 * m
    elif kind == WIN_ALGEBRAIC:
        lc = math.log(math.pi) + math.lgamma(2 * beta + 1) - beta * math.log(4.0) - math.lgamma(beta + 1)
        c2 = math.exp(lc - beta * math.log(math.pi))
        mu = float(beta)
    else:
        raise ValueError("Theorem 3.4 constants are given for the B-spline, algebraic and "
                         "Kaiser-Bessel windows")
    c1 = c2 * lo ** (-mu)
    return c1, c2, mu


def bound_thm34(kind, m, sigma, beta) -> float:
    """(3.9), Theorem 3.4: upper bound of the general error constant E_sigma(phi)
    of a window of family `kind` from the constants of thm34_constants."""
    c1, c2, mu = thm34_constants(kind, m, sigma, beta)
    inner = 2.0 * c1 + 2.0 * c2 / ((mu - 1.0) * m ** mu) * (1.0 - 1.0 / (2.0 * sigma)) ** (1.0 - mu)
    return float(inner / window_hat(kind, m / (2.0 * sigma), m, beta))


def bound_thm35(kind, N, sigma1, sigma2, m1, m2) -> float:
    """(3.10), Theorem 3.5: [E_sigma1(phi_1) + a E_sigma2(phi_2) / phi_hat_1(N*/2)],
    the bound on E_paper, with Theorem 3.4 for both constants and the sizes of
    the N* substitution (phi_hat_1(N*/2) = (m1/N1) omega_hat_1(m1 / (2 sigma1_eff)))."""
    P = params(N, sigma1, sigma2, m1, m2, kind)
    e1 = bound_thm34(kind, m1, P.sigma1_eff, P.beta1)
    e2 = bound_thm34(kind, m2, P.sigma2_eff, P.beta2)
    phi1 = m1 / P.N1 * float(window_hat(kind, m1 / (2.0 * P.sigma1_eff), m1, P.beta1))
    return e1 + P.a / phi1 * e2


CC_C = math.pi * (math.e ** 2 - 1) / (2 * math.e)   # C of Theorem 5.3


def bound_thm53(N, nu) -> float:
    """(5.6), Theorem 5.3: Clenshaw-Curtis sinc error bound for n = nu N."""
    return (36 * (1 + math.exp(-2 * CC_C * N)) / (35 * (math.e ** 2 - 1))
            * math.exp(-N * (nu - CC_C)))


def bound_thm62(eps, E) -> float:
    """(6.7), Theorem 6.2: fast sinc error factor (eps + 2E + E^2) times sum |c_k|,
    where E is the NNFFT error constant of Theorem 3.5."""
    return eps + 2 * E + E * E
