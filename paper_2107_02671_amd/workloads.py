"""Seeded synthetic inputs (numpy PCG64), shared by the tests, the benchmark
and the serving driver.  Node and coefficient generators only: nothing here
computes any part of the transform.

Workloads (the paper's experiments use random nodes and coefficients; no
dataset is involved):
  small     N=64, M1=M2=256, uniform nodes, complex Gaussian f, sigma=2, m=4
  large     N=4096, M1=M2=2^20, uniform nodes, complex Gaussian f, sigma=2, m=6
  sinc      N=1024, L1=L2=2^18, Chebyshev-distributed nodes (cos of uniform
            angles, halved), real Gaussian c, 2N Gauss-Legendre nodes, m=6
  served    10,000 requests: N log-uniform in [64, 8192], M1, M2 log-uniform
            in [2^10, 2^20], Poisson arrivals, FP32 m=6 or FP64 m=12
  clustered N=16384, M1=M2=2^24, 32 Gaussian clusters (std 1e-3, centers
            uniform in [-0.45, 0.45]), m=8
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def uniform_nodes(g: np.random.Generator, n: int) -> np.ndarray:
    return g.uniform(-0.5, 0.5, n)


def chebyshev_nodes(g: np.random.Generator, n: int) -> np.ndarray:
    return 0.5 * np.cos(g.uniform(0.0, np.pi, n))


def clustered_nodes(g: np.random.Generator, n: int, nclusters: int = 32, std: float = 1e-3,
                    lo: float = -0.45, hi: float = 0.45) -> np.ndarray:
    centers = g.uniform(lo, hi, nclusters)
    pick = g.integers(0, nclusters, n)
    out = centers[pick] + g.normal(0.0, std, n)
    bad = (out < -0.5) | (out >= 0.5)
    while bad.any():
        out[bad] = centers[pick[bad]] + g.normal(0.0, std, int(bad.sum()))
        bad = (out < -0.5) | (out >= 0.5)
    return out


def complex_gaussian(g: np.random.Generator, n: int) -> np.ndarray:
    return g.standard_normal(n) + 1j * g.standard_normal(n)


WORKLOADS = {
    "small": dict(N=64, M1=256, M2=256, sigma=2.0, m=4, nodes="uniform", seed=1),
    "large": dict(N=4096, M1=1 << 20, M2=1 << 20, sigma=2.0, m=6, nodes="uniform", seed=2),
    "sinc": dict(N=1024, M1=1 << 18, M2=1 << 18, sigma=2.0, m=6, nodes="chebyshev", seed=3, n_quad=2048),
    "clustered": dict(N=16384, M1=1 << 24, M2=1 << 24, sigma=2.0, m=8, nodes="clustered", seed=5),
}


def nnfft_inputs(name: str, M1: int | None = None, M2: int | None = None):
    """(N, v, x, f, params) of a named workload; M1/M2 may be cut down."""
    w = dict(WORKLOADS[name])
    g = rng(w["seed"])
    M1 = M1 or w["M1"]
    M2 = M2 or w["M2"]
    gen = {"uniform": uniform_nodes, "chebyshev": chebyshev_nodes, "clustered": clustered_nodes}[w["nodes"]]
    v = gen(g, M1)
    x = gen(g, M2)
    if name == "sinc":
        f = g.standard_normal(M1) + 0j
    else:
        f = complex_gaussian(g, M1)
    return w["N"], v, x, f, w


def served_requests(n: int = 10000, seed: int = 4):
    """Request descriptors of the served workload (no node arrays: those are
    drawn per request from request_nodes)."""
    g = rng(seed)
    N = np.rint(np.exp(g.uniform(np.log(64), np.log(8192), n))).astype(np.int64)
    M1 = np.rint(np.exp(g.uniform(np.log(2 ** 10), np.log(2 ** 20), n))).astype(np.int64)
    M2 = np.rint(np.exp(g.uniform(np.log(2 ** 10), np.log(2 ** 20), n))).astype(np.int64)
    fp32 = g.random(n) < 0.5
    gaps = g.exponential(1.0, n)      # Poisson arrivals; scaled by the rate at run time
    return [dict(id=i, N=int(N[i]), M1=int(M1[i]), M2=int(M2[i]), fp32=bool(fp32[i]),
                 m=6 if fp32[i] else 12, gap=float(gaps[i])) for i in range(n)]


def request_nodes(req: dict, seed: int = 4):
    g = rng(seed * 1_000_003 + req["id"])
    return uniform_nodes(g, req["M1"]), uniform_nodes(g, req["M2"]), complex_gaussian(g, req["M1"])
