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
    assert (r["items_points"], r["block_points"], r["grid_max"], r["tuned"]) == (16, 1 << 17, 0, 0)
    r = binding.nnfft_get_tuning(FP64, 1 << 20)
    assert (r["items_points"], r["block_points"], r["tuned"]) == (8, 1 << 16, 0)
    # small sides keep one block; 8 blocks once every XCD can get 2^14 points
    assert binding.nnfft_get_tuning(FP32, 1000)["block_points"] == 1000
    assert binding.nnfft_get_tuning(FP32, 8 << 14)["block_points"] == 1 << 14
    binding.nnfft_set_tuning(FP32, 1 << 20, 8, 1 << 16, 2048)
    r = binding.nnfft_get_tuning(FP32, (1 << 19) + 1)     # same size class ceil(log2 M) = 20
    assert (r["items_points"], r["grid_max"], r["tuned"]) == (8, 2048, 1)
    assert binding.nnfft_get_tuning(FP32, 1 << 19)["tuned"] == 0
    # FP64 kernels hold at most 8 points per item and never loop over slots
    binding.nnfft_set_tuning(FP64, 1 << 20, 32, 1 << 16, 512)
    r = binding.nnfft_get_tuning(FP64, 1 << 20)
    assert (r["items_points"], r["grid_max"], r["tuned"]) == (8, 0, 1)
    with pytest.raises(binding.NnfftError):
        binding.nnfft_set_tuning(FP32, 1 << 20, 0, 1 << 16)
    binding.nnfft_clear_tuning()
    assert binding.nnfft_get_tuning(FP32, 1 << 20)["tuned"] == 0
    assert L is binding.lib()
