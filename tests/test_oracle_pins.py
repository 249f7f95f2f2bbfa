"""Pins for the FP64 CPU oracle, against facts that do not come from the oracle
itself: closed forms, library routines (numpy FFT, scipy quadrature, scipy
Bessel functions, scipy Gauss-Legendre), brute force on tiny inputs, the
error bounds of Theorems 4.1, 5.3 and 6.2, and numbers printed in the paper
(tests/golden/paper_values.json).

Each test is chosen so that a plausible slip in the oracle (a dropped factor,
a wrong sign or index, a transposed operand) makes it fail.
"""
import json
import math
import os

import numpy as np
import pytest
import scipy.fft
import scipy.integrate
import scipy.special

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")



def _rng(seed):
    return np.random.default_rng(seed)


def _cgauss(rng, n):
    return rng.standard_normal(n) + 1j * rng.standard_normal(n)


def _bound(P):
    # (4.2) with the slip of its proof corrected on the second term (1.08)
    return oracle.bound_thm41_gate(P.N1, P.m1, P.m2, P.sigma1_eff, P.sigma2_eff)


# --------------------------------------------------------------------------
# windows
# --------------------------------------------------------------------------

@pytest.mark.parametrize("beta", [9.42477796, 18.8495559, 28.2743339, 56.5486678])
def test_omega_closed_form_properties(beta):
    # Example 2.1: even, support [-1, 1], omega(0) = 1, decreasing on [0, 1]
    u = np.linspace(0, 1, 2001)
    w = oracle.omega(u, beta)
    assert w[0] == pytest.approx(1.0, abs=1e-15)
    assert w[-1] == 0.0
    assert np.all(np.diff(w) <= 1e-18)
    np.testing.assert_array_equal(oracle.omega(-u, beta), w)
    assert oracle.omega(np.array([1.5, -3.0]), beta).tolist() == [0.0, 0.0]
    ref = np.sinh(beta * np.sqrt(1 - u[:-1] ** 2)) / np.sinh(beta)
    np.testing.assert_allclose(w[:-1], ref, rtol=1e-13, atol=1e-300)


@pytest.mark.parametrize("beta", [9.42477796, 18.8495559, 28.2743339, 37.6991118, 56.5486678])
def test_omega_hat_matches_numerical_fourier_integral(beta):
    # (2.1) against 2 int_0^1 omega(x) cos(2 pi v x) dx by adaptive quadrature,
    # on both sides of the branch point v = beta / (2 pi).
    vb = beta / (2 * np.pi)
    for v in [0.0, 0.13 * vb, 0.5 * vb, 0.9 * vb, vb, 1.3 * vb, 2.1 * vb]:
        f = lambda x: 2 * np.sinh(beta * np.sqrt(1 - x * x)) / np.sinh(beta) * np.cos(2 * np.pi * v * x)
        ref, err = scipy.integrate.quad(f, 0, 1, epsabs=1e-15, epsrel=1e-13, limit=400)
        got = float(oracle.omega_hat(v, beta))
        scale = float(oracle.omega_hat(0.0, beta))
        assert abs(got - ref) <= 1e-11 * scale, (v, got, ref)


@pytest.mark.parametrize("beta", [9.42477796, 28.2743339, 56.5486678, 75.398])
def test_omega_hat_matches_scipy_bessel_i1(beta):
    v = np.linspace(0, 0.99 * beta / (2 * np.pi), 50)
    z = np.sqrt(beta ** 2 - 4 * np.pi ** 2 * v ** 2)
    ref = np.pi * beta / np.sinh(beta) * scipy.special.i1(z) / z
    np.testing.assert_allclose(oracle.omega_hat(v, beta), ref, rtol=5e-14)


# --------------------------------------------------------------------------
# parameter derivation (sizes worked out by hand from the readings)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,sigma,m,expect", [
    # N* = N + ceil(2m/sigma); N1 = 2 ceil(sigma N*/2); G1 = N1 + 2m;
    # N2 = largest even 2^p 3^q 5^r <= sigma G1.
    (64, 2.0, 4, (68, 136, 144, 288)),          # 64+4; 136; 144; 288 = 2^5 3^2
    (4096, 2.0, 6, (4102, 8204, 8216, 16384)),  # 16432 -> 16384 = 2^14
    (1024, 2.0, 6, (1030, 2060, 2072, 4096)),   # 4144 -> 4096
    (64, 2.0, 6, (70, 140, 152, 300)),          # 304 -> 300 = 2^2 3 5^2
    (8192, 2.0, 12, (8204, 16408, 16432, 32768)),
    (16384, 2.0, 8, (16392, 32784, 32800, 65536)),
    (1200, 1.25, 6, (1210, 1514, 1526, 1920)),  # N*=1200+ceil(9.6)=1210; 1.25*1210=1512.5 -> 1514
])
def test_param_sizes(N, sigma, m, expect):
    P = oracle.params(N, sigma, sigma, m, m)
    assert (P.N_star, P.N1, P.G1, P.N2) == expect
    assert P.a == pytest.approx(P.G1 / P.N1)
    assert P.beta1 == pytest.approx(2 * math.pi * m * (1 - 1 / (2 * P.N1 / P.N_star)))
    # Algorithm 2.2 input requirement 2 m2 <= (1 - 1/sigma1) N2
    assert 2 * m <= (1 - 1 / P.sigma1_eff) * P.N2


def test_param_rejects_invalid():
    for args in [(0, 2, 2, 4, 4), (64, 1.0, 2, 4, 4), (64, 2, 0.9, 4, 4), (64, 2, 2, 1, 4)]:
        with pytest.raises(ValueError):
            oracle.params(*args)


# --------------------------------------------------------------------------
# direct sum (1.2)
# --------------------------------------------------------------------------

def test_direct_single_exponential_closed_form():
    rng = _rng(11)
    N = 1000
    v = rng.uniform(-0.5, 0.5, 37)
    x = np.concatenate([rng.uniform(-0.5, 0.5, 50), [-0.5, 0.5, 0.0]])
    for k0 in [0, 17, 36]:
        f = np.zeros(37, complex)
        f[k0] = 0.7 - 0.2j
        y = oracle.direct(N, v, f, x)
        ref = f[k0] * np.exp(-2j * np.pi * N * v[k0] * x)
        np.testing.assert_allclose(y, ref, rtol=0, atol=2e-13)


def test_direct_equals_numpy_dft_on_equispaced_nodes():
    # v_k = k/n, x_j = j/n, N = n: exp(-2 pi i N v_k x_j) = exp(-2 pi i k j / n)
    n = 96
    lab = np.arange(-n // 2, n // 2)
    rng = _rng(12)
    f = _cgauss(rng, n)
    y = oracle.direct(n, lab / n, f, lab / n)
    Y = np.fft.fft(np.fft.ifftshift(f))       # index k mod n
    ref = Y[lab % n]
    np.testing.assert_allclose(y, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def test_direct_brute_force_tiny():
    rng = _rng(13)
    v = rng.uniform(-0.5, 0.5, 5)
    x = rng.uniform(-0.5, 0.5, 4)
    f = _cgauss(rng, 5)
    N = 7
    ref = [sum(f[k] * complex(math.cos(2 * math.pi * N * v[k] * x[j]),
                              -math.sin(2 * math.pi * N * v[k] * x[j])) for k in range(5))
           for j in range(4)]
    np.testing.assert_allclose(oracle.direct(N, v, f, x), ref, atol=1e-13)


# --------------------------------------------------------------------------
# NNFFT (Algorithm 2.2)
# --------------------------------------------------------------------------

@pytest.mark.parametrize("N,M1,M2,sigma,m", [
    (64, 256, 256, 2.0, 4),      # the smallest workload: checked against brute force
    (64, 256, 256, 2.0, 2),
    (64, 256, 256, 2.0, 6),
    (100, 333, 301, 1.5, 5),     # odd node counts, sigma1 N* not an integer
    (200, 500, 400, 1.25, 7),
    (128, 1000, 777, 2.0, 8),
])
def test_nnfft_within_theorem_4_1(N, M1, M2, sigma, m):
    rng = _rng(N + M1 + m)
    v = rng.uniform(-0.5, 0.5, M1)
    x = rng.uniform(-0.5, 0.5, M2)
    f = _cgauss(rng, M1)
    P = oracle.params(N, sigma, sigma, m, m)
    y = oracle.nnfft(N, v, f, x, sigma, sigma, m, m)
    ex = oracle.direct(N, v, f, x)
    e_paper = np.abs(y - ex).max() / np.abs(f).sum()
    assert e_paper <= _bound(P), (e_paper, _bound(P))


def test_nnfft_error_decays_exponentially_in_m():
    rng = _rng(21)
    N, M = 64, 256
    v = rng.uniform(-0.5, 0.5, M)
    x = rng.uniform(-0.5, 0.5, M)
    f = _cgauss(rng, M)
    ex = oracle.direct(N, v, f, x)
    errs = []
    for m in [2, 3, 4, 5, 6, 7]:
        y = oracle.nnfft(N, v, f, x, 2.0, 2.0, m, m)
        errs.append(np.abs(y - ex).max() / np.abs(f).sum())
    # each step in m gains more than a factor 10 (the bound (4.2) gains
    # e^{2 pi sqrt(1/2)} ~ 85 per step for sigma = 2)
    for a, b in zip(errs, errs[1:]):
        assert b < a / 10, errs
    assert errs[-1] < 1e-12


@pytest.mark.parametrize("v0", [0.0, 0.49, -0.5, 0.5, 0.123456789])
def test_nnfft_single_exponential(v0):
    rng = _rng(22)
    N = 80
    x = np.concatenate([rng.uniform(-0.5, 0.5, 300), [-0.5, 0.5]])
    for m in [4, 6]:
        P = oracle.params(N, 2.0, 2.0, m, m)
        y = oracle.nnfft(N, np.array([v0]), np.array([1.0 + 0j]), x, 2.0, 2.0, m, m)
        err = np.abs(y - np.exp(-2j * np.pi * N * v0 * x)).max()
        assert err <= _bound(P)


def test_nnfft_edge_nodes():
    rng = _rng(23)
    N = 64
    v = np.concatenate([[-0.5, 0.5, 0.0], rng.uniform(-0.5, 0.5, 60)])
    x = np.concatenate([[-0.5, 0.5, 0.0], rng.uniform(-0.5, 0.5, 40)])
    f = _cgauss(rng, len(v))
    P = oracle.params(N, 2.0, 2.0, 6, 6)
    y = oracle.nnfft(N, v, f, x, 2.0, 2.0, 6, 6)
    ex = oracle.direct(N, v, f, x)
    assert np.abs(y - ex).max() / np.abs(f).sum() <= _bound(P)


def test_nnfft_rejects_nodes_outside_domain():
    with pytest.raises(ValueError):
        oracle.nnfft(64, np.array([0.6]), np.array([1 + 0j]), np.array([0.0]))
    with pytest.raises(ValueError):
        oracle.nnfft(64, np.array([0.1]), np.array([1 + 0j]), np.array([-0.50001]))


def test_nnfft_step3_matches_numpy_fft():
    # step 3 of the oracle is a direct DFT; compare with numpy's FFT applied to
    # the deconvolved step-1 output.
    rng = _rng(24)
    N, m = 64, 4
    P = oracle.params(N, 2.0, 2.0, m, m)
    v = rng.uniform(-0.5, 0.5, 200)
    f = _cgauss(rng, 200)
    _, g, h = oracle.nnfft(N, v, f, np.array([0.0]), 2.0, 2.0, m, m, return_steps=True)
    ell = np.arange(P.G1) - P.G1 // 2
    phi2 = (P.m2 / P.N2) * oracle.omega_hat(P.m2 * ell / P.N2, P.beta2)
    X = np.zeros(P.N2, complex)
    X[ell % P.N2] = g / phi2
    Y = np.fft.fft(X) / P.N2
    s = np.arange(P.N2) - P.N2 // 2
    np.testing.assert_allclose(h, Y[s % P.N2], rtol=0, atol=1e-12 * np.abs(Y).max())


def test_nnfft_step1_total_mass():
    # sum_l phi_1(l/N1 - v) / N1 is a rectangular rule for int phi_1 = phi_1_hat(0)
    # (Sec. 2, (2.10) at x = 0); so sum_l g_l ~ phi_1_hat(0) sum_k f_k.
    rng = _rng(25)
    N, m = 64, 6
    P = oracle.params(N, 2.0, 2.0, m, m)
    v = rng.uniform(-0.5, 0.5, 50)
    f = _cgauss(rng, 50)
    _, g, _ = oracle.nnfft(N, v, f, np.array([0.0]), 2.0, 2.0, m, m, return_steps=True)
    phi1_hat0 = (P.m1 / P.N1) * float(oracle.omega_hat(0.0, P.beta1))
    np.testing.assert_allclose(g.sum(), phi1_hat0 * f.sum(), rtol=1e-8)


def test_nnfft_linearity():
    rng = _rng(26)
    N = 50
    v = rng.uniform(-0.5, 0.5, 90)
    x = rng.uniform(-0.5, 0.5, 70)
    f1, f2 = _cgauss(rng, 90), _cgauss(rng, 90)
    a, b = 0.3 - 1.1j, -2.0 + 0.5j
    lhs = oracle.nnfft(N, v, a * f1 + b * f2, x, 2, 2, 5, 5)
    rhs = a * oracle.nnfft(N, v, f1, x, 2, 2, 5, 5) + b * oracle.nnfft(N, v, f2, x, 2, 2, 5, 5)
    np.testing.assert_allclose(lhs, rhs, rtol=0, atol=1e-12 * np.abs(lhs).max())


def test_nnfft_outputs_at_node_subsets():
    # Each output of Algorithm 2.2 depends on its own node only, and step 3 of
    # the oracle forms just the h_s that step 4 reads: outputs at a subset of
    # the nodes (grid edges included) equal the full run's bit for bit, and a
    # few nodes at a large bandwidth still meet Theorem 4.1.  (With the step
    # outputs requested, every h_s is formed.)
    rng = _rng(27)
    N, m = 300, 6
    v = rng.uniform(-0.5, 0.5, 400)
    x = np.concatenate([[-0.5, 0.5, 0.0], rng.uniform(-0.5, 0.5, 300)])
    f = _cgauss(rng, 400)
    full = oracle.nnfft(N, v, f, x, 2.0, 2.0, m, m, return_steps=True)[0]     # every h_s formed
    idx = np.array([0, 1, 2, 17, 150, 302])
    np.testing.assert_array_equal(oracle.nnfft(N, v, f, x[idx], 2.0, 2.0, m, m), full[idx])
    N = 1 << 17
    P = oracle.params(N, 2.0, 2.0, m, m)
    v = rng.uniform(-0.5, 0.5, 2000)
    f = _cgauss(rng, 2000)
    xs = np.concatenate([[0.5, -0.5], rng.uniform(-0.5, 0.5, 6)])
    y = oracle.nnfft(N, v, f, xs, 2.0, 2.0, m, m)
    err = np.abs(y - oracle.direct(N, v, f, xs)).max() / np.abs(f).sum()
    assert err <= _bound(P)


# --------------------------------------------------------------------------
# quadrature rules
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [1, 2, 5, 64, 2048])
def test_gauss_legendre_matches_scipy(n):
    z, w = oracle.gauss_legendre(n)
    zr, wr = scipy.special.roots_legendre(n)
    order = np.argsort(-zr)
    np.testing.assert_allclose(z, zr[order], rtol=0, atol=1e-14)
    # scipy's weights lose ~1e-7 relative accuracy at the end nodes for large n
    np.testing.assert_allclose(w, wr[order] / 2, rtol=5e-7, atol=5e-15)
    assert w.sum() == pytest.approx(1.0, abs=1e-13)
    # independent recomputation in extended precision: Newton-polish the nodes
    # with the Legendre recurrence in long double and use W = 2/((1-t^2) P_n'^2)
    t = z.astype(np.longdouble)

    def legendre(t):
        p0, p1 = np.ones_like(t), t.copy()
        for k in range(1, n):
            p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
        return p1, n * (t * p1 - p0) / (t * t - 1)

    if n > 1:
        for _ in range(3):
            p, dp = legendre(t)
            t = t - p / dp
        p, dp = legendre(t)
        wl = (1 / ((1 - t * t) * dp * dp)).astype(np.float64)
        np.testing.assert_allclose(w, wl, rtol=1e-9)


def test_gauss_legendre_exact_on_polynomials():
    n = 9
    z, w = oracle.gauss_legendre(n)
    for p in range(2 * n):
        exact = 0.0 if p % 2 else 1.0 / (p + 1)   # (1/2) int_{-1}^{1} t^p dt
        assert np.dot(w, z ** p) == pytest.approx(exact, abs=1e-14)


def test_clenshaw_curtis_small_and_structure():
    z, w = oracle.clenshaw_curtis(2)
    np.testing.assert_allclose(w, [1 / 6, 2 / 3, 1 / 6], atol=1e-15)   # Simpson's rule, halved
    for n in [2, 3, 4, 8, 64, 1024]:
        z, w = oracle.clenshaw_curtis(n)
        assert w.sum() == pytest.approx(1.0, abs=1e-13)                # (5.5)
        np.testing.assert_array_equal(z, -z[::-1])                       # z_k = -z_{n-k}
        np.testing.assert_allclose(w, w[::-1], rtol=0, atol=1e-15)       # w_k = w_{n-k}
        assert np.all(w > 0)
        np.testing.assert_allclose(z, np.cos(np.arange(n + 1) * np.pi / n), atol=1e-15)


@pytest.mark.parametrize("n", [4, 16, 64])
def test_clenshaw_curtis_exact_on_polynomials(n):
    z, w = oracle.clenshaw_curtis(n)
    for p in range(n + 1):
        exact = 0.0 if p % 2 else 1.0 / (p + 1)
        assert np.dot(w, z ** p) == pytest.approx(exact, abs=1e-13)


@pytest.mark.parametrize("t", [2, 3, 6, 10])
def test_clenshaw_curtis_weights_match_algorithm_5_4(t):
    # Algorithm 5.4: the same weights from an orthogonal DCT-I (scipy.fft)
    n = 2 ** t
    eps = np.ones(n + 1)
    eps[0] = eps[n] = math.sqrt(2) / 2
    a = np.zeros(n + 1)
    j = np.arange(n // 2 + 1)
    a[2 * j] = eps[2 * j] * 2.0 / (1.0 - 4.0 * j * j)
    ahat = scipy.fft.dct(a, type=1, norm="ortho")
    w54 = eps * ahat / math.sqrt(2 * n)
    _, w = oracle.clenshaw_curtis(n)
    np.testing.assert_allclose(w, w54, rtol=0, atol=1e-15)


def test_theorem_5_3_printed_values():
    gold = json.load(open(os.path.join(GOLDEN, "paper_values.json")))
    c = gold["clenshaw_curtis_C"]
    assert oracle.CC_C == pytest.approx(c["value"], abs=c["abs_tol"])
    assert oracle.CC_C == pytest.approx(math.pi * math.sinh(1.0), rel=1e-15)
    g = gold["cc_eps_1e-8_nu_4_min_N"]
    nmin = g["value"]
    assert oracle.bound_thm53(nmin, g["nu"]) < g["eps"] < oracle.bound_thm53(nmin - 1, g["nu"])


@pytest.mark.parametrize("N", [16, 64, 200])
def test_clenshaw_curtis_sinc_error_within_theorem_5_3(N):
    nu = 4
    z, w = oracle.clenshaw_curtis(nu * N)
    x = np.linspace(-1, 1, 4001)
    approx = (w[None, :] * np.exp(-1j * np.pi * N * np.outer(x, z))).sum(axis=1)
    err = np.abs(approx - np.sinc(N * x)).max()
    assert err <= oracle.bound_thm53(N, nu) + 1e-14


@pytest.mark.parametrize("N", [64, 256, 1024])
def test_gauss_legendre_2N_sinc_error(N):
    # 2N Gauss-Legendre nodes integrate (1/2) e^{-pi i N t x} on [-1, 1] for
    # |x| <= 1 to better than 1e-11 once N >= 64 (at N = 16 the error is still
    # ~1e-4: the rule needs n well above pi N / 2 plus a margin that only
    # becomes small relative to N for larger N).
    z, w = oracle.gauss_legendre(2 * N)
    x = np.linspace(-1, 1, 3001)
    approx = (w[None, :] * np.exp(-1j * np.pi * N * np.outer(x, z))).sum(axis=1)
    assert np.abs(approx - np.sinc(N * x)).max() < 1e-11


# --------------------------------------------------------------------------
# discrete sinc transform (6.2) and Algorithm 6.1
# --------------------------------------------------------------------------

def test_sinc_direct_matches_numpy_sinc():
    rng = _rng(31)
    N = 128
    a = rng.uniform(-0.5, 0.5, 70)
    b = np.concatenate([rng.uniform(-0.5, 0.5, 60), a[:5]])   # include b = a (sinc(0) = 1)
    c = _cgauss(rng, 70)
    ref = (np.sinc(N * (b[:, None] - a[None, :])) * c[None, :]).sum(axis=1)
    np.testing.assert_allclose(oracle.sinc_direct(N, a, c, b), ref, rtol=0, atol=1e-12)


def test_sinc_direct_shannon_cardinality():
    # sinc(N pi (a0 + l/N - a0)) = delta_{l0}
    N = 64
    a0 = 0.0123
    ell = np.arange(-20, 21)
    b = a0 + ell / N
    h = oracle.sinc_direct(N, np.array([a0]), np.array([1.0 + 0j]), b)
    np.testing.assert_allclose(h, (ell == 0).astype(float), atol=1e-13)
    assert float(oracle.sinc_pi(0.0)) == 1.0


@pytest.mark.parametrize("quad,nq_of_N", [(oracle.QUAD_GAUSS_LEGENDRE, lambda N: 2 * N),
                                          (oracle.QUAD_CLENSHAW_CURTIS, lambda N: 4 * N)])
def test_sinc_fast_within_theorem_6_2(quad, nq_of_N):
    rng = _rng(32)
    N, m = 64, 6
    L1, L2 = 200, 180
    a = 0.5 * np.cos(rng.uniform(0, np.pi, L1))     # Chebyshev-distributed nodes
    b = 0.5 * np.cos(rng.uniform(0, np.pi, L2))
    c = rng.standard_normal(L1) + 0j
    h = oracle.sinc_fast(N, a, c, b, nq_of_N(N), quad, 2.0, 2.0, m, m)
    ref = oracle.sinc_direct(N, a, c, b)
    P = oracle.params(N, 2.0, 2.0, m, m)
    if quad == oracle.QUAD_CLENSHAW_CURTIS:
        eps = oracle.bound_thm53(N, 4)
    else:
        z, w = oracle.gauss_legendre(2 * N)
        xs = np.linspace(-1, 1, 4001)
        eps = np.abs((w[None, :] * np.exp(-1j * np.pi * N * np.outer(xs, z))).sum(1) - np.sinc(N * xs)).max()
    bound = oracle.bound_thm62(eps, _bound(P)) * np.abs(c).sum()
    err = np.abs(h - ref).max()
    assert err <= bound, (err, bound)
    assert err < 1e-6 * np.abs(ref).max()
    # real coefficients give a real transform
    assert np.abs(h.imag).max() < 1e-9 * np.abs(h).max()


# --------------------------------------------------------------------------
# NFFT with equispaced frequencies and its adjoint (the special case v_k = k/N
# of (1.2), Sec. 2; the equispaced cases of the fast sinc transform, Sec. 6)
# --------------------------------------------------------------------------

def _nfft_case(N, M, seed):
    rng = _rng(seed)
    x = rng.uniform(-0.5, 0.5, M)
    x[:3] = [-0.5, 0.5, 0.0]
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    y = rng.standard_normal(M) + 1j * rng.standard_normal(M)
    return x, f, y


def _nfft_gate(N, sigma, m):
    # the sinh-type window's NFFT error constant decays like
    # m^(3/2) exp(-2 pi m sqrt(1 - 1/sigma)); gate with the factor 24 (the
    # largest entry error of the fast map measured for sigma in [5/4, 2],
    # m in {4, 6, 8} is 6-14 times m^(3/2) exp(...)); rounding floor 1e-14
    n, _ = oracle.nfft_params(N, sigma, m)
    return 24.0 * m ** 1.5 * math.exp(-2 * math.pi * m * math.sqrt(1 - N / n)) + 1e-14


@pytest.mark.parametrize("N,M,sigma", [(64, 300, 2.0), (100, 257, 1.5), (250, 64, 2.0), (32, 500, 1.25)])
@pytest.mark.parametrize("m", [4, 6, 8])
def test_nfft_forward_and_adjoint_against_direct_sums(N, M, sigma, m):
    x, f, y = _nfft_case(N, M, N + M + m)
    k = np.arange(-N // 2, N // 2)
    yf = oracle.nfft(N, f, x, sigma, m)
    yd = oracle.direct(N, k / N, f, x)                      # (1.2) with v_k = k / N
    assert np.abs(yf - yd).max() <= _nfft_gate(N, sigma, m) * np.abs(f).sum()
    h = oracle.nfft_adjoint(N, y, x, sigma, m)
    hd = oracle.direct(1, -x, y, k.astype(float))           # sum_j y_j exp(+2 pi i k x_j)
    assert np.abs(h - hd).max() <= _nfft_gate(N, sigma, m) * np.abs(y).sum()


def test_nfft_pair_is_adjoint():
    # the two fast maps are transposes of each other: <A f, y> = <f, A^H y>
    for N, M, m in [(64, 300, 4), (128, 1000, 7)]:
        x, f, y = _nfft_case(N, M, 7 * m)
        lhs = np.vdot(y, oracle.nfft(N, f, x, 2.0, m))
        rhs = np.vdot(oracle.nfft_adjoint(N, y, x, 2.0, m), f)
        assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_nfft_equispaced_nodes_is_a_dft():
    N, m = 64, 8
    x = np.arange(-N // 2, N // 2) / N
    rng = _rng(3)
    f = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    # y_j = sum_k f_k exp(-2 pi i k j / N): numpy's FFT after moving index -N/2 to 0
    ref = np.fft.fftshift(np.fft.fft(np.fft.ifftshift(f)))
    np.testing.assert_allclose(oracle.nfft(N, f, x, 2.0, m), ref, atol=1e-12 * np.abs(f).sum())
    refa = np.fft.fftshift(np.fft.ifft(np.fft.ifftshift(f))) * N
    np.testing.assert_allclose(oracle.nfft_adjoint(N, f, x, 2.0, m), refa, atol=1e-12 * np.abs(f).sum())


def test_nfft_single_frequency_and_errors():
    N, m = 32, 8
    x = _rng(4).uniform(-0.5, 0.5, 50)
    f = np.zeros(N, dtype=complex)
    f[5 + N // 2] = 1.0
    np.testing.assert_allclose(oracle.nfft(N, f, x, 2.0, m), np.exp(-2j * np.pi * 5 * x), atol=1e-13)
    with pytest.raises(ValueError):
        oracle.nfft(N, f, np.array([0.7]), 2.0, m)
    with pytest.raises(ValueError):
        oracle.nfft_params(33, 2.0, 4)


def test_nfft_error_decays_exponentially_in_m():
    N, M = 64, 400
    x, f, _ = _nfft_case(N, M, 11)
    yd = oracle.direct(N, np.arange(-N // 2, N // 2) / N, f, x)
    errs = [np.abs(oracle.nfft(N, f, x, 2.0, m) - yd).max() / np.abs(f).sum() for m in (3, 4, 5, 6)]
    for a, b in zip(errs, errs[1:]):
        assert b < a / 30      # about exp(-2 pi sqrt(1/2)) = 1/85 per step of m


@pytest.mark.parametrize("s1,s3", [(True, False), (False, True), (True, True)])
@pytest.mark.parametrize("quad", [oracle.QUAD_GAUSS_LEGENDRE, oracle.QUAD_CLENSHAW_CURTIS])
def test_sinc_equispaced_special_cases_against_direct_sum(s1, s3, quad):
    # Sec. 6 after Algorithm 6.1: equispaced a_k = k / L1 turn step 1 into an
    # NFFT, b_l = l / N turn step 3 into an adjoint NFFT; the result is the
    # sinc sum (6.2) within Theorem 6.2 with the NFFT's error in place of E
    rng = _rng(41)
    N, m = 64, 8
    L1 = 96 if s1 else 150
    a = np.arange(-L1 // 2, L1 // 2) / L1 if s1 else 0.5 * np.cos(rng.uniform(0, np.pi, L1))
    b = np.arange(-N // 2, N // 2) / N if s3 else 0.5 * np.cos(rng.uniform(0, np.pi, 130))
    c = rng.standard_normal(L1) + 1j * rng.standard_normal(L1)
    nq = 2 * N if quad == oracle.QUAD_GAUSS_LEGENDRE else 4 * N
    h = oracle.sinc_fast_equispaced(N, a, c, b, nq, quad, 2.0, m, s1, s3, 2.0, m)
    ref = oracle.sinc_direct(N, a, c, b)
    if quad == oracle.QUAD_CLENSHAW_CURTIS:
        eps = oracle.bound_thm53(N, 4)
    else:
        z, w = oracle.gauss_legendre(nq)
        xs = np.linspace(-1, 1, 4001)
        eps = np.abs((w[None, :] * np.exp(-1j * np.pi * N * np.outer(xs, z))).sum(1) - np.sinc(N * xs)).max()
    E = max(_nfft_gate(L1 if s1 else N, 2.0, m), _nfft_gate(N, 2.0, m),
            _bound(oracle.params(N, 2.0, 2.0, m, m)))
    err = np.abs(h - ref).max()
    assert err <= oracle.bound_thm62(eps, E) * np.abs(c).sum(), err
    assert err < 1e-6 * np.abs(ref).max()
    # and it agrees with the general chain of two NNFFTs
    hg = oracle.sinc_fast(N, a, c, b, nq, quad, 2.0, 2.0, m, m)
    assert np.abs(h - hg).max() < 2e-6 * np.abs(ref).max()


# --------------------------------------------------------------------------
# B-spline and algebraic windows (Example 2.1) and the NNFFT with them
# --------------------------------------------------------------------------

@pytest.mark.parametrize("n", [2, 3, 4, 7, 12, 16, 32])
def test_bspline_against_scipy_and_partition_of_unity(n):
    from scipy.interpolate import BSpline
    ys = np.linspace(0.003, n - 0.003, 97)
    ref = np.nan_to_num(BSpline.basis_element(np.arange(n + 1), extrapolate=False)(ys))
    assert np.abs(oracle.bspline_cardinal(n, ys) - ref).max() < 1e-14
    # sum over integer shifts is 1
    y = 0.3721
    assert abs(sum(float(oracle.bspline_cardinal(n, y + j)) for j in range(-n, n + 1)) - 1.0) < 1e-14


def test_bspline_central_values():
    # B_4(0) = 2/3, B_6(0) = 11/20, B_8(0) = 151/315 (centred cardinal splines)
    for n, val in ((4, 2 / 3), (6, 11 / 20), (8, 151 / 315)):
        assert abs(float(oracle.bspline_cardinal(n, n / 2)) - val) < 1e-15


@pytest.mark.parametrize("kind,m", [(oracle.WIN_BSPLINE, 3), (oracle.WIN_BSPLINE, 8),
                                    (oracle.WIN_ALGEBRAIC, 2), (oracle.WIN_ALGEBRAIC, 6),
                                    (oracle.WIN_ALGEBRAIC, 12), (oracle.WIN_KAISER_BESSEL, 2),
                                    (oracle.WIN_KAISER_BESSEL, 6), (oracle.WIN_KAISER_BESSEL, 12)])
def test_window_transforms_against_quadrature(kind, m):
    beta = {oracle.WIN_ALGEBRAIC: 3.0 * m, oracle.WIN_KAISER_BESSEL: 1.5 * math.pi * m}.get(kind, 0.0)
    w = lambda x: float(oracle.window(kind, x, m, beta))
    assert w(0.0) == pytest.approx(1.0, abs=1e-15)
    assert w(1.0) == 0.0 and w(-1.0) == 0.0
    assert w(0.37) == pytest.approx(w(-0.37), abs=1e-15)
    # (Kaiser-Bessel at v = m/2, where the transform is 1e-6 of the integrand's
    # scale, is beyond quad's absolute accuracy: the mpmath pin below covers it)
    vs = (0.0, 0.25, 0.9, m / 2.5) + (() if kind == oracle.WIN_KAISER_BESSEL else (m / 2.0,))
    for v in vs:
        ref, _ = scipy.integrate.quad(lambda x: 2.0 * w(x) * math.cos(2 * math.pi * v * x), 0, 1,
                                      epsabs=1e-16, epsrel=1e-13, limit=400)
        got = float(oracle.window_hat(kind, v, m, beta))
        assert abs(got - ref) <= 1e-12 * abs(ref) + 1e-16, (v, got, ref)   # quad: epsabs 1e-16


@pytest.mark.parametrize("m", [2, 5, 8, 16])
def test_algebraic_transform_against_scipy_bessel(m):
    import scipy.special as sp
    beta = 3 * m
    C = math.pi * math.exp(math.lgamma(2 * beta + 1) - beta * math.log(4) - math.lgamma(beta + 1))
    assert float(oracle.window_hat(oracle.WIN_ALGEBRAIC, 0.0, m, beta)) == pytest.approx(
        C / math.factorial(beta), rel=1e-13)
    # the NNFFT evaluates the transform for |v| <= m / (2 sigma) < m / 2
    for v in np.linspace(0.05, m / 2, 9):
        ref = C * (math.pi * v) ** (-beta) * sp.jv(beta, 2 * math.pi * v)
        assert float(oracle.window_hat(oracle.WIN_ALGEBRAIC, v, m, beta)) == pytest.approx(ref, rel=1e-11)


@pytest.mark.parametrize("m,sigma", [(2, 1.25), (4, 2.0), (6, 1.5), (12, 2.0), (16, 2.0)])
def test_kaiser_bessel_window_closed_form(m, sigma):
    # (I_0(beta sqrt(1 - x^2)) - 1) / (I_0(beta) - 1) with scipy's i0; in the
    # set Omega: even, 1 at 0, 0 at +-1, decreasing on [0, 1]
    import scipy.special as sp
    beta = 2 * math.pi * m * (1 - 1 / (2 * sigma))
    xs = np.linspace(0.0, 0.999, 300)
    got = oracle.window(oracle.WIN_KAISER_BESSEL, xs, m, beta)
    ref = (sp.i0(beta * np.sqrt(1 - xs * xs)) - 1) / (sp.i0(beta) - 1)
    assert np.abs(got - ref).max() <= 1e-13
    assert np.all(np.diff(got) < 0)
    assert float(oracle.window(oracle.WIN_KAISER_BESSEL, 1.0, m, beta)) == 0.0
    assert float(oracle.window(oracle.WIN_KAISER_BESSEL, -0.3, m, beta)) == float(
        oracle.window(oracle.WIN_KAISER_BESSEL, 0.3, m, beta))
    # near the support ends the window vanishes like (beta^2/4)(1 - x^2) / (I_0(beta) - 1)
    x = 1 - 1e-9
    lead = beta * beta / 4 * (1 - x * x) / (sp.i0(beta) - 1)
    assert float(oracle.window(oracle.WIN_KAISER_BESSEL, x, m, beta)) == pytest.approx(lead, rel=1e-6)


@pytest.mark.parametrize("m,v", [(2, 1.6), (2, 5.3), (6, 4.6), (6, 9.25), (6, 40.1), (12, 6.0)])
def test_kaiser_bessel_transform_past_the_branch_point(m, v):
    # beyond |v| = beta / (2 pi) the transform is the sin branch, small and
    # oscillating: checked against 30-digit quadrature of the window (mpmath)
    import mpmath as mp
    mp.mp.dps = 30
    beta = 1.5 * math.pi * m            # sigma = 2
    i0b = mp.besseli(0, beta) - 1
    w = lambda x: (mp.besseli(0, beta * mp.sqrt(1 - x * x)) - 1) / i0b
    ref = 2 * mp.quad(lambda x: w(x) * mp.cos(2 * mp.pi * v * x), mp.linspace(0, 1, 40))
    got = float(oracle.window_hat(oracle.WIN_KAISER_BESSEL, v, m, beta))
    assert abs(got - float(ref)) <= 1e-12 * abs(float(ref)) + 1e-300, (got, float(ref))


def test_bspline_transform_is_a_power_of_sinc():
    for m in (2, 4, 7):
        b0 = float(oracle.bspline_cardinal(2 * m, m))
        for v in (0.0, 0.4, 1.7, m - 0.01):
            ref = np.sinc(v / m) ** (2 * m) / (m * b0)
            assert float(oracle.window_hat(oracle.WIN_BSPLINE, v, m, 0.0)) == pytest.approx(ref, rel=1e-13)


def test_window_family_parameters():
    P = oracle.params(100, 2.0, 2.0, 5, 7, oracle.WIN_ALGEBRAIC)
    assert (P.beta1, P.beta2, P.window) == (15.0, 21.0, oracle.WIN_ALGEBRAIC)
    assert oracle.params(100, 2.0, 2.0, 5, 7, oracle.WIN_BSPLINE).beta1 == 0.0
    S = oracle.params(100, 2.0, 2.0, 5, 7)
    assert oracle.params(100, 2.0, 2.0, 5, 7, oracle.WIN_BSPLINE).N2 == S.N2
    with pytest.raises(ValueError):      # the algebraic window needs sigma > pi/3
        oracle.params(100, 1.02, 2.0, 5, 5, oracle.WIN_ALGEBRAIC)
    K = oracle.params(100, 2.0, 1.5, 5, 7, oracle.WIN_KAISER_BESSEL)   # the sinh windows' beta
    S = oracle.params(100, 2.0, 1.5, 5, 7)
    assert (K.beta1, K.beta2, K.N2, K.window) == (S.beta1, S.beta2, S.N2, oracle.WIN_KAISER_BESSEL)


@pytest.mark.parametrize("kind", [oracle.WIN_BSPLINE, oracle.WIN_ALGEBRAIC, oracle.WIN_KAISER_BESSEL])
@pytest.mark.parametrize("sigma", [1.5, 2.0])
def test_nnfft_other_windows_against_direct_sum(kind, sigma):
    # Theorem 3.5 with Theorem 3.4's constants bounds the error; the error
    # decays geometrically in m and reaches 1e-9 at m = 12 (the Kaiser-Bessel
    # window at m = 6, and FP64 rounding, ~1e-14 of sum |f|, from m = 8 on)
    g = _rng(71)
    N, M1, M2 = 128, 700, 500
    v, x = g.uniform(-0.5, 0.5, M1), g.uniform(-0.5, 0.5, M2)
    f = g.standard_normal(M1) + 1j * g.standard_normal(M1)
    ex = oracle.direct(N, v, f, x)
    sf = np.abs(f).sum()
    errs = []
    ms = (2, 4, 6) if kind == oracle.WIN_KAISER_BESSEL else (4, 6, 8, 10, 12)
    for m in ms:
        y = oracle.nnfft(N, v, f, x, sigma, sigma, m, m, window=kind)
        e = np.abs(y - ex).max() / sf
        assert e <= oracle.bound_thm35(kind, N, sigma, sigma, m, m)
        errs.append(e)
    for a, b in zip(errs, errs[1:]):
        assert b < a / 3            # each step of 2 in m gains at least a factor 3
    assert errs[-1] < 1e-8
    if kind == oracle.WIN_KAISER_BESSEL:
        for m in (10, 12):
            y = oracle.nnfft(N, v, f, x, sigma, sigma, m, m, window=kind)
            assert np.abs(y - ex).max() / sf <= max(oracle.bound_thm35(kind, N, sigma, sigma, m, m), 2e-13)


@pytest.mark.parametrize("sigma,m", [(1.25, 4), (1.5, 6), (2.0, 4), (2.0, 8)])
def test_nnfft_kaiser_bessel_tracks_the_sinh_window(sigma, m):
    # the two windows are close relatives (both ~ exp(beta (sqrt(1 - x^2) - 1))
    # in the bulk, same beta): their NNFFT errors at the sizes of Example 4.2
    # agree within a factor 10
    g = _rng(73)
    N, M1, M2 = 1200, 2400, 1600
    v, x = g.uniform(-0.5, 0.5, M1), g.uniform(-0.5, 0.5, M2)
    f = g.standard_normal(M1) + 1j * g.standard_normal(M1)
    ex = oracle.direct(N, v, f, x)
    ek = np.abs(oracle.nnfft(N, v, f, x, sigma, sigma, m, m, window=oracle.WIN_KAISER_BESSEL) - ex).max()
    es = np.abs(oracle.nnfft(N, v, f, x, sigma, sigma, m, m) - ex).max()
    assert es / 10 <= ek <= es * 10, (ek, es)
