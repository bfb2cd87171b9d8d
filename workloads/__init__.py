"""Seeded synthetic workloads shared by the tests, the smoke check and the benchmark.

Only parameter recipes live here: lattice size, filling, disorder width, localization
length, hop cutoff, temperature, field, Philox seed and sample id per sample.  The
random configurations and disorder themselves are drawn inside each implementation
from the Philox streams keyed by (seed, sample id), so this module holds none of the
method's arithmetic.  Sizes and parameter ranges follow the paper's 2D runs
(nu = 1/2, xi = 1, W = 1, square tori with toroidal boundaries; section "Results for
the lattice model in two dimensions").
"""
from __future__ import annotations

from dataclasses import dataclass, asdict

import numpy as np


@dataclass(frozen=True)
class Sample:
    L: int
    n_e: int
    W: float
    xi: float
    rc: float
    T: float
    E: float
    seed: int
    sample_id: int
    dim: int = 2  # 2: square lattice (L^2 sites), 3: simple cubic (L^3 sites)
    pair: float = 0.0  # probability that a label proposes a pair hop (0: single hops only)
    M: int = 0  # the sample's parallel width (p = ceil(m / M)); 0: the run options' M

    def as_dict(self):
        return asdict(self)


def _half(L: int) -> int:
    return (L * L) // 2


def serial_small(seed: int = 1):
    """L=16 (N=256), half filling, W=1, xi=1, rc=6, T=0.1, E=0.01: the small case the
    oracle finishes in well under a second (10^4 hops)."""
    return [Sample(16, _half(16), 1.0, 1.0, 6.0, 0.1, 0.01, seed, 0)]


def fp64_single(seed: int = 2):
    """L=64 (N=4096), half filling, rc=8, T=0.05, E=0.01; FP64, M=1024."""
    return [Sample(64, _half(64), 1.0, 1.0, 8.0, 0.05, 0.01, seed, 0)]


def vrh_l128(n_samples: int = 32, seed: int = 3):
    """L=128 (N=16384), half filling, rc=10, T=0.02, E=0.005 (the variable-range-hopping
    case); M=8192, refresh every 4096 hops in the FP32 form.  Samples 0..n-1."""
    return [Sample(128, _half(128), 1.0, 1.0, 10.0, 0.02, 0.005, seed, b) for b in range(n_samples)]


def batched_l64(n_samples: int = 256, seed: int = 4):
    """256 samples at L=64, rc=8, E=0.01, T from {0.02,0.03,0.05,0.08,0.12} round-robin;
    M=2048, refresh every 2048 hops."""
    grid = (0.02, 0.03, 0.05, 0.08, 0.12)
    return [Sample(64, _half(64), 1.0, 1.0, 8.0, grid[b % 5], 0.01, seed, b) for b in range(n_samples)]


def uneven_batch(n_samples: int = 96, seed: int = 5):
    """96 samples, L uniform over {32,48,64,96,128,160}, T ~ U[0.015,0.1], E ~ U[0.001,0.02],
    W ~ U[0.5,2], xi=1, rc=10; run to simulated time 1e3."""
    rng = np.random.default_rng(seed)
    sizes = (32, 48, 64, 96, 128, 160)
    out = []
    for b in range(n_samples):
        L = int(sizes[rng.integers(len(sizes))])
        T = float(rng.uniform(0.015, 0.1))
        E = float(rng.uniform(0.001, 0.02))
        W = float(rng.uniform(0.5, 2.0))
        out.append(Sample(L, _half(L), W, 1.0, 10.0, T, E, seed, b))
    return out


def headline(n_samples: int = 256, seed: int = 3):
    """Benchmark batch: the L=128, T=0.02 parameters above in one launch, one sample per CU."""
    return vrh_l128(n_samples, seed)
