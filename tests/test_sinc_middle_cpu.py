"""The fast sinc transform's middle operator (sinc_middle_dry_run, host
only) against its definition built here from the oracle's windows.

Between the two FFTs, Algorithm 6.1 applies the first NNFFT's step 4 and
output scaling at x_j = z_j / 2 (Algorithm 2.2), multiplies by the weights
w_j (step 2 of Algorithm 6.1), and applies the second NNFFT's steps 1 and 2
from v_j = -z_j / 2.  For random first-FFT outputs h_s the operator's rows
u_l = sum_b K[b][l] h_{lo[l] + b} must equal that chain evaluated term by
term with the oracle's window, window transform and quadrature rules (the
FFT input convention of the library: u_l = g_l / (N1 N2 phi_hat_2(l)) with
g_l the unscaled spread sum), to FP64 rounding.
"""
import numpy as np
import pytest

import oracle
import paper_2107_02671_amd as P

GL, CC = P.SINC_QUAD_GAUSS_LEGENDRE, P.SINC_QUAD_CLENSHAW_CURTIS


def _reference(N, quad, nq, s1, s2, m, h):
    Pp = oracle.params(N, s1, s2, m, m)
    z, w = oracle.gauss_legendre(nq) if quad == GL else oracle.clenshaw_curtis(nq)
    N1, N2, Ns, G1 = Pp.N1, Pp.N2, Pp.N_star, Pp.G1
    # first NNFFT, step 4 and output at x_j = z_j / 2
    x = 0.5 * z
    u = N2 * Ns * x / N1
    cu = np.floor(u).astype(np.int64)
    y1 = np.zeros(len(z), dtype=np.complex128)
    for r in range(2 * m):
        s = cu - m + 1 + r
        y1 += oracle.window(0, (u - s) / m, m, Pp.beta2) * h[s + N2 // 2]
    phi1 = m / N1 * oracle.window_hat(0, m * Ns * x / N1, m, Pp.beta1)
    alpha = w * y1 / phi1
    # second NNFFT, steps 1 and 2 from v_j = -z_j / 2
    v = -0.5 * z
    t = N1 * (N * v / Ns)
    ct = np.floor(t).astype(np.int64)
    g = np.zeros(G1, dtype=np.complex128)
    for q in range(2 * m):
        l = ct - m + 1 + q
        np.add.at(g, l + G1 // 2, oracle.window(0, (l - t) / m, m, Pp.beta1) * alpha)
    labels = np.arange(G1) - G1 // 2
    phi2 = m / N2 * oracle.window_hat(0, m * labels / N2, m, Pp.beta2)
    return g / (N1 * N2 * phi2), Pp


@pytest.mark.parametrize("N,quad,nqf,s1,s2,m", [
    (64, GL, 2, 2.0, 2.0, 6),
    (100, CC, 2, 1.5, 2.0, 7),
    (333, GL, 3, 2.0, 1.5, 5),
    (1024, GL, 2, 2.0, 2.0, 6),
    (512, CC, 4, 2.0, 2.0, 8),
])
def test_middle_operator_matches_the_chain(N, quad, nqf, s1, s2, m):
    nq = nqf * N
    K, lo = P.sinc_middle_dry_run(N, quad, nq, s1, s2, m, m)
    Pp = oracle.params(N, s1, s2, m, m)
    # a row l gathers the nodes with t_j within m of l, whose u_j = -t_j / rho
    # (rho = N1^2 N / (N*^2 N2)) span 2 m / rho labels, plus the 2 m taps
    rho = Pp.N1 ** 2 * N / (Pp.N_star ** 2 * Pp.N2)
    assert K.shape[1] == Pp.G1 and K.shape[0] <= int(np.ceil(2 * m / rho)) + 2 * m + 2
    rng = np.random.default_rng(N + m)
    h = rng.standard_normal(Pp.N2) + 1j * rng.standard_normal(Pp.N2)   # label s at s + N2/2
    ref, _ = _reference(N, quad, nq, s1, s2, m, h)
    Wb = K.shape[0]
    idx = lo[None, :] + np.arange(Wb)[:, None] + Pp.N2 // 2
    assert idx.min() >= 0 and idx.max() < Pp.N2
    got = (K * h[idx]).sum(axis=0)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    assert err <= 1e-12, err


def test_middle_operator_refusals():
    with pytest.raises(P.NnfftError) as e:
        P.sinc_middle_dry_run(64, GL, 1 << 17, 2.0, 2.0, 6, 6)   # more quadrature nodes than it is built for
    assert e.value.status == P.binding.NNFFT_ERR_UNSUPPORTED
    with pytest.raises(P.NnfftError) as e:
        P.sinc_middle_dry_run(64, 7, 128, 2.0, 2.0, 6, 6)
    assert e.value.status == P.binding.NNFFT_ERR_ARG
