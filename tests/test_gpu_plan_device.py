"""Node preparation on the device (Algorithm 2.2 step 0): nnfft_plan splits
the nodes into (cell, offset) in FP64, checks their domain, counts the bins
of every node block and sorts the nodes stably by (block, cell) on the GPU,
and builds the work schedule on the host from the counts alone.  The layout
image it leaves in the plan block (tables, schedule, point records) must be
bit for bit the one the dry run builds from host copies of the nodes on the
host: compared through 64-bit digests of the two images, on uniform,
clustered, Chebyshev-crowded and degenerate node sets, both precisions and
every window family.  Nodes outside [-1/2, 1/2] (or NaN) are refused by the
device check with NNFFT_ERR_DOMAIN.
"""
import sys
import time

import numpy as np
import pytest
import torch

import paper_2107_02671_amd as P
from paper_2107_02671_amd import binding as B
from paper_2107_02671_amd import workloads as W

pytestmark = pytest.mark.gpu

FP64, FP32 = P.NNFFT_FP64_PLAIN, P.NNFFT_FP32_COMP
DEV = "cuda:0"


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _sets():
    g = W.rng(1701)
    out = {
        "uniform": (4096, W.uniform_nodes(g, 1 << 18), W.uniform_nodes(g, 3 * (1 << 16) + 7)),
        "clustered": (16384, W.clustered_nodes(g, 1 << 16), W.clustered_nodes(g, 50001)),
        "chebyshev": (1024, W.chebyshev_nodes(g, 1 << 18), W.chebyshev_nodes(g, 4099)),
        "small": (64, W.uniform_nodes(g, 256), W.uniform_nodes(g, 255)),
        "one_node": (100, np.array([0.123]), np.array([-0.25])),
    }
    same = np.full(1 << 17, 0.1234567)
    out["identical"] = (1000, same, np.full(1 << 13, -0.37))
    # grid-point nodes (integer grid coordinates) and the interval ends
    N = 1000
    out["grid_points"] = (N, (np.arange(-2000, 2000) / 4100.0)[:4000], np.linspace(-0.5, 0.5, 3001))
    out["ends"] = (N, np.tile([-0.5, 0.5], 5000), np.tile([0.5, -0.5, 0.0], 3000))
    return out


SETS = _sets()


@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
@pytest.mark.parametrize("name", list(SETS))
def test_device_layout_equals_dry_run(name, prec):
    N, v, x = SETS[name]
    m = 6
    _say(f"[gpu] device plan layout {name} N={N} M=({len(v)},{len(x)}) prec={prec}")
    ref = B.nnfft_plan_dry_run_digest(N, v, x, 2.0, 2.0, m, m, prec)
    with P.Plan(N, torch.tensor(v, device=DEV), torch.tensor(x, device=DEV), 2.0, 2.0, m, m, prec) as pl:
        got = B.nnfft_plan_digest(pl.handle)
    assert got == ref, f"{name}: device layout digest {got:#x} != dry run {ref:#x}"


@pytest.mark.parametrize("window", [P.NNFFT_WINDOW_BSPLINE, P.NNFFT_WINDOW_ALGEBRAIC, P.NNFFT_WINDOW_KAISER_BESSEL])
@pytest.mark.parametrize("prec", [FP32, FP64], ids=["fp32", "fp64"])
def test_device_layout_other_windows_and_sigmas(window, prec):
    g = W.rng(1702)
    v, x = W.uniform_nodes(g, 20001), W.uniform_nodes(g, 7777)
    for s1, s2, m1, m2 in ((1.5, 2.0, 8, 10), (2.0, 1.5, 5, 4)):
        if prec == FP32 and min(m1, m2) < 4:
            continue
        ref = B.nnfft_plan_dry_run_digest(333, v, x, s1, s2, m1, m2, prec, window)
        with P.Plan(333, torch.tensor(v, device=DEV), torch.tensor(x, device=DEV), s1, s2, m1, m2, prec,
                    window=window) as pl:
            assert B.nnfft_plan_digest(pl.handle) == ref


@pytest.mark.parametrize("bad", [np.nan, 0.5000001, -0.75])
@pytest.mark.parametrize("side", ["v", "x"])
def test_device_domain_check(bad, side):
    g = W.rng(1703)
    v, x = W.uniform_nodes(g, 5000), W.uniform_nodes(g, 4000)
    (v if side == "v" else x)[1234] = bad
    with pytest.raises(P.NnfftError) as e:
        P.Plan(256, torch.tensor(v, device=DEV), torch.tensor(x, device=DEV), 2.0, 2.0, 6, 6, FP32)
    assert e.value.status == B.NNFFT_ERR_DOMAIN
    assert ("frequency" if side == "v" else "spatial") in str(e.value)


def test_plan_time_large():
    # N = 4096, M1 = M2 = 2^20 uniform nodes (the benchmark workload)
    N, v, x, f, w = W.nnfft_inputs("large")
    tv, tx = torch.tensor(v, device=DEV), torch.tensor(x, device=DEV)
    for prec in (FP32, FP64):
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            pl = P.Plan(N, tv, tx, 2.0, 2.0, 6, 6, prec)
            ts.append((time.perf_counter() - t0) * 1e3)
            pl.close()
        _say(f"    plan N={N} M=2^20 prec={prec}: {sorted(ts)[len(ts) // 2]:.2f} ms (median of 5)")
        assert min(ts) < 30.0
