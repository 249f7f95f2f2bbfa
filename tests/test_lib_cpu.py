"""CPU checks of the HIP library: it loads, exports every entry point that
include/nnfft.h and include/nnfft_serve.h declare, and its host-side logic (size derivation, error
codes, quadrature rules) agrees with the oracle.  No device work."""
import ctypes

import numpy as np
import pytest

import oracle
import paper_2107_02671_amd as P
from paper_2107_02671_amd import binding


def test_library_loads_and_exports_header_symbols():
    L = binding.lib()
    names = binding.header_functions()
    assert len(names) >= 12
    assert {"nnfft_exec_batch", "nnfft_autotune", "nnfft_server_create", "nnfft_server_submit"} <= set(names)
    for n in names:
        assert hasattr(L, n), n
        assert ctypes.cast(getattr(L, n), ctypes.c_void_p).value
    assert "gfx950" in P.nnfft_version()


@pytest.mark.parametrize("N", [1, 2, 7, 64, 100, 1000, 1200, 4096, 8192, 16384])
@pytest.mark.parametrize("sig", [(2.0, 2.0), (1.25, 1.25), (1.5, 2.0), (1.7, 1.3), (3.0, 2.5)])
@pytest.mark.parametrize("m", [(2, 2), (4, 4), (6, 6), (6, 9), (12, 12)])
def test_derive_params_matches_oracle(N, sig, m):
    try:
        o = oracle.params(N, sig[0], sig[1], m[0], m[1])
    except ValueError:
        with pytest.raises(P.NnfftError) as e:
            P.nnfft_derive_params(N, sig[0], sig[1], m[0], m[1])
        assert e.value.status == binding.NNFFT_ERR_ARG
        return
    a = P.nnfft_derive_params(N, sig[0], sig[1], m[0], m[1])
    for key in ["N_star", "N1", "G1", "N2", "m1", "m2"]:
        assert a[key] == getattr(o, key), key
    for key in ["sigma1_eff", "sigma2_eff", "a", "beta1", "beta2"]:
        assert a[key] == pytest.approx(getattr(o, key), rel=1e-14), key
    assert a["bound_thm41"] == pytest.approx(
        oracle.bound_thm41(o.N1, m[0], m[1], o.sigma1_eff, o.sigma2_eff), rel=1e-12)


@pytest.mark.parametrize("args", [(0, 2, 2, 4, 4), (64, 1.0, 2, 4, 4), (64, 2, 1.0, 4, 4),
                                  (64, 2, 2, 1, 4), (64, 2, 2, 4, 1), (64, float("nan"), 2, 4, 4)])
def test_derive_params_rejects(args):
    with pytest.raises(P.NnfftError) as e:
        P.nnfft_derive_params(*args)
    assert e.value.status == binding.NNFFT_ERR_ARG
    assert "invalid" in P.nnfft_last_error()


@pytest.mark.parametrize("n", [1, 2, 3, 8, 64, 2048, 4096])
def test_gauss_legendre_rule_matches_oracle(n):
    z, w = P.nnfft_quadrature(P.SINC_QUAD_GAUSS_LEGENDRE, n)
    zo, wo = oracle.gauss_legendre(n)
    np.testing.assert_allclose(z, zo, rtol=0, atol=4e-16)
    np.testing.assert_allclose(w, wo, rtol=1e-11, atol=1e-16)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 8, 100, 1024, 8192])
def test_clenshaw_curtis_rule_matches_oracle(n):
    z, w = P.nnfft_quadrature(P.SINC_QUAD_CLENSHAW_CURTIS, n)
    zo, wo = oracle.clenshaw_curtis(n)
    np.testing.assert_array_equal(z, zo)
    np.testing.assert_allclose(w, wo, rtol=0, atol=1e-15)


def test_quadrature_rejects():
    with pytest.raises(P.NnfftError):
        P.nnfft_quadrature(P.SINC_QUAD_GAUSS_LEGENDRE, 0)
    with pytest.raises(P.NnfftError):
        P.nnfft_quadrature(7, 4)


# ---------------------------------------------------------------------------
# layout tuning table (host only)
# ---------------------------------------------------------------------------
def test_tuning_table_rule_set_clear():
    L = binding.lib()
    binding.nnfft_clear_tuning()
    FP32, FP64 = binding.NNFFT_FP32_COMP, binding.NNFFT_FP64_PLAIN
    r = binding.nnfft_get_tuning(FP32, 1 << 20)
    # built-in rule: 16 points per item at 2^20 nodes, 2^17-point blocks, no grid cap
    assert (r["items_points"], r["block_points"], r["tuned"]) == (16, 1 << 17, 0)
    r = binding.nnfft_get_tuning(FP64, 1 << 20)
    assert (r["items_points"], r["block_points"], r["tuned"]) == (4, 1 << 17, 0)
    # spreading sides above 2^20 points take 2^18-point blocks
    assert binding.nnfft_get_tuning(FP32, 1 << 22)["block_points"] == 1 << 18
    # small sides keep one block; 8 blocks once every XCD can get 2^14 points
    assert binding.nnfft_get_tuning(FP32, 1000)["block_points"] == 1000
    assert binding.nnfft_get_tuning(FP32, 8 << 14)["block_points"] == 1 << 14
    binding.nnfft_set_tuning(FP32, 1 << 20, 8, 1 << 16)
    r = binding.nnfft_get_tuning(FP32, 1 << 20)
    assert (r["items_points"], r["block_points"], r["tuned"]) == (8, 1 << 16, 1)
    r = binding.nnfft_get_tuning(FP32, (1 << 19) + 1)     # same size class ceil(log2 M) = 20
    assert (r["items_points"], r["tuned"]) == (8, 1)
    assert binding.nnfft_get_tuning(FP32, 1 << 19)["tuned"] == 0
    # FP64 kernels hold at most 8 points per item
    binding.nnfft_set_tuning(FP64, 1 << 20, 32, 1 << 16)
    r = binding.nnfft_get_tuning(FP64, 1 << 20)
    assert (r["items_points"], r["tuned"]) == (8, 1)
    with pytest.raises(binding.NnfftError):
        binding.nnfft_set_tuning(FP32, 1 << 20, 0, 1 << 16)
    binding.nnfft_clear_tuning()
    assert binding.nnfft_get_tuning(FP32, 1 << 20)["tuned"] == 0
    assert L is binding.lib()


# ---------------------------------------------------------------------------
# host-side plan construction: layout invariants (no device work)
# ---------------------------------------------------------------------------
DRY_CASES = [
    # N, M1, M2, sigma, m, prec, nodes
    (119, 11545, 18958, 2.0, 6, P.NNFFT_FP32_COMP, "uniform"),     # 2-point items, deep window overlap
    (179, 107085, 1217, 2.0, 12, P.NNFFT_FP64_PLAIN, "uniform"),
    (4096, 1 << 20, 1 << 20, 2.0, 6, P.NNFFT_FP32_COMP, "uniform"),
    (4096, 1 << 18, 1 << 18, 2.0, 6, P.NNFFT_FP64_PLAIN, "uniform"),
    (2048, 1 << 16, 1 << 16, 2.0, 8, P.NNFFT_FP32_COMP, "clustered"),
    (1024, 30000, 30000, 2.0, 6, P.NNFFT_FP64_PLAIN, "chebyshev"),
    (1200, 2400, 1600, 1.25, 6, P.NNFFT_FP32_COMP, "uniform"),
    (64, 1, 1, 2.0, 4, P.NNFFT_FP32_COMP, "uniform"),
    (64, 5000, 3, 2.0, 16, P.NNFFT_FP64_PLAIN, "edge"),
]


@pytest.mark.parametrize("case", DRY_CASES, ids=lambda c: f"N{c[0]}-M{c[1]}x{c[2]}-m{c[4]}-p{c[5]}-{c[6]}")
def test_plan_dry_run_layout_invariants(case):
    from paper_2107_02671_amd import workloads as W
    N, M1, M2, sig, m, prec, kind = case
    g = W.rng(M1 + M2)
    if kind == "edge":    # every node on the boundary or at 0: all points in three bins
        v = g.choice([-0.5, 0.0, 0.5], M1)
        x = g.choice([-0.5, 0.0, 0.5], M2)
    else:
        gen = {"uniform": W.uniform_nodes, "chebyshev": W.chebyshev_nodes, "clustered": W.clustered_nodes}[kind]
        v, x = gen(g, M1), gen(g, M2)
    info = binding.nnfft_plan_dry_run(N, v, x, sig, sig, m, m, prec)
    o = oracle.params(N, sig, sig, m, m)
    assert (info["N1"], info["G1"], info["N2"]) == (o.N1, o.G1, o.N2)
    assert info["M1"] == M1 and info["M2"] == M2
    assert info["device_bytes"] > 8 * (M1 + M2)    # at least one 8-byte record per point
    assert info["spread_workgroups"] >= (M1 + 64 * info["items_points"] - 1) // (64 * info["items_points"])


def test_plan_dry_run_errors():
    with pytest.raises(binding.NnfftError) as e:
        binding.nnfft_plan_dry_run(64, np.array([0.1, 0.7]), np.array([0.0]), 2.0, 2.0, 6, 6)
    assert e.value.status == binding.NNFFT_ERR_DOMAIN
    with pytest.raises(binding.NnfftError) as e:
        binding.nnfft_plan_dry_run(64, np.array([0.1]), np.array([0.0]), 2.0, 2.0, 3, 3, P.NNFFT_FP32_COMP)
    assert e.value.status == binding.NNFFT_ERR_UNSUPPORTED


@pytest.mark.parametrize("N,M,m,prec", [(64, 300, 6, P.NNFFT_FP32_COMP), (64, 300, 12, P.NNFFT_FP64_PLAIN),
                                        (1000, 50000, 6, P.NNFFT_FP32_COMP), (2048, 3, 8, P.NNFFT_FP64_PLAIN),
                                        (4096, 1 << 18, 8, P.NNFFT_FP32_COMP)])
def test_nfft_dry_run_layout_invariants(N, M, m, prec):
    from paper_2107_02671_amd import workloads as W
    g = W.rng(N + M)
    x = W.uniform_nodes(g, M)
    x[:min(3, M)] = [-0.5, 0.5, 0.0][:min(3, M)]   # both edges of the period and the centre
    info = binding.nfft_plan_dry_run(N, x, 2.0, m, prec)
    n, beta = oracle.nfft_params(N, 2.0, m)
    assert info["N1"] == n and info["N2"] == n and info["N"] == N
    assert abs(info["beta1"] - beta) <= 1e-12 * beta


def test_nfft_dry_run_errors():
    x = np.array([0.1, -0.2])
    for args, status in [((63, x), binding.NNFFT_ERR_ARG), ((64, np.array([0.6])), binding.NNFFT_ERR_DOMAIN)]:
        with pytest.raises(binding.NnfftError) as e:
            binding.nfft_plan_dry_run(*args, 2.0, 6, P.NNFFT_FP64_PLAIN)
        assert e.value.status == status
    with pytest.raises(binding.NnfftError) as e:
        binding.nfft_plan_dry_run(64, x, 2.0, 3, P.NNFFT_FP32_COMP)
    assert e.value.status == binding.NNFFT_ERR_UNSUPPORTED


@pytest.mark.parametrize("window", [P.NNFFT_WINDOW_BSPLINE, P.NNFFT_WINDOW_ALGEBRAIC, P.NNFFT_WINDOW_KAISER_BESSEL])
@pytest.mark.parametrize("prec", [P.NNFFT_FP64_PLAIN, P.NNFFT_FP32_COMP])
def test_window_plan_dry_run(window, prec):
    # plans of the B-spline and algebraic families (Example 2.1) and the
    # Kaiser-Bessel family: sizes as for the sinh family, shape parameters of
    # the family, layout invariants
    g = np.random.default_rng(17)
    v, x = g.uniform(-0.5, 0.5, 5000), g.uniform(-0.5, 0.5, 3000)
    for sig, m in ((2.0, 6), (1.5, 8), (1.25, 4)):
        i = binding.nnfft_plan_dry_run(300, v, x, sig, sig, m, m, prec, window=window)
        s = binding.nnfft_plan_dry_run(300, v, x, sig, sig, m, m, prec)
        assert i["window"] == window and s["window"] == P.NNFFT_WINDOW_SINH
        assert (i["N1"], i["G1"], i["N2"]) == (s["N1"], s["G1"], s["N2"])
        assert i["thm41_applies"] == 0 and i["bound_thm41"] == 0.0
        Po = oracle.params(300, sig, sig, m, m, window)
        assert (i["beta1"], i["beta2"]) == (Po.beta1, Po.beta2)
        assert i["corr_fit_err"] <= (1e-8 if prec == P.NNFFT_FP32_COMP else 1e-12)


def test_window_plan_errors():
    v = np.zeros(8)
    with pytest.raises(P.NnfftError):
        binding.nnfft_plan_dry_run(100, v, v, 1.02, 2.0, 4, 4, P.NNFFT_FP64_PLAIN, window=P.NNFFT_WINDOW_ALGEBRAIC)
    with pytest.raises(P.NnfftError):
        binding.nnfft_plan_dry_run(100, v, v, 2.0, 2.0, 4, 4, P.NNFFT_FP64_PLAIN, window=4)


@pytest.mark.parametrize("prec,qmax", [(P.NNFFT_FP32_COMP, 32), (P.NNFFT_FP64_PLAIN, 8)])
@pytest.mark.parametrize("kind", ["chebyshev", "clustered"])
def test_dense_node_sets_raise_the_item_size(prec, qmax, kind):
    # 2^18 dense nodes at N = 1024 (the sinc workload's first spreading side,
    # ~127 nodes per grid cell and far more at the crowded ends): the layout
    # raises the item size to the family's maximum, with or without a tuned
    # entry for that size class (tuned entries are timed on uniform nodes)
    from paper_2107_02671_amd import workloads as W
    g = W.rng(18)
    gen = W.chebyshev_nodes if kind == "chebyshev" else W.clustered_nodes
    v = gen(g, 1 << 18)
    x = W.uniform_nodes(g, 2048)
    try:
        binding.nnfft_clear_tuning()
        assert binding.nnfft_plan_dry_run(1024, v, x, 2.0, 2.0, 6, 6, prec)["items_points"] == qmax
        binding.nnfft_set_tuning(prec, 1 << 18, 4, 1 << 15)
        assert binding.nnfft_get_tuning(prec, 1 << 18)["tuned"] == 1
        assert binding.nnfft_plan_dry_run(1024, v, x, 2.0, 2.0, 6, 6, prec)["items_points"] == qmax
        # uniform nodes of the same size class keep the tuned item size
        u = W.uniform_nodes(g, 1 << 18)
        assert binding.nnfft_plan_dry_run(1024, u, x, 2.0, 2.0, 6, 6, prec)["items_points"] == 4
    finally:
        binding.nnfft_clear_tuning()
