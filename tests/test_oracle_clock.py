"""The exact serial clock (Gamma(m, Gamma) increments) of the oracle: its sampler against
the Gamma distribution of the library routine scipy.stats.gamma, and its use in a run."""
import numpy as np
import pytest
from scipy import stats

import oracle


@pytest.mark.parametrize("m", [1, 2, 7, 100, 1500])
def test_gamma_increments_follow_the_gamma_law(m):
    # the waiting time of m proposals, each Exp(Gamma), is Gamma(shape m, rate Gamma)
    G = 3.5
    x = np.array([oracle.gamma_dt(11, 4, h, m, G) for h in range(20000)])
    ks = stats.kstest(x, stats.gamma(a=m, scale=1.0 / G).cdf)
    assert ks.pvalue > 1e-3, ks
    assert abs(x.mean() - m / G) < 5 * np.sqrt(m) / G / np.sqrt(len(x))
    # different hops, samples and seeds draw different values
    assert len(set(x[:100].tolist())) == 100
    assert oracle.gamma_dt(11, 5, 0, m, G) != oracle.gamma_dt(11, 4, 0, m, G)
    assert oracle.gamma_dt(12, 4, 0, m, G) != oracle.gamma_dt(11, 4, 0, m, G)


def test_exponential_case_and_a_wrong_shape_is_detected():
    # m = 1 is the exponential law; a sampler off by the 1/3 of d = m - 1/3 would fail this
    x = np.array([oracle.gamma_dt(2, 0, h, 1, 1.0) for h in range(20000)])
    assert stats.kstest(x, stats.expon().cdf).pvalue > 1e-3
    assert stats.kstest(x * (4.0 / 3.0), stats.expon().cdf).pvalue < 1e-6


def test_run_with_the_gamma_clock_adds_the_increments():
    o = oracle.Oracle(L=16, n_e=128, W=1.0, xi=1.0, rc=6.0, T=0.1, E=0.01, seed=3, sample_id=1, clock_mode=2)
    lab, _, _ = o.run(300)
    G = o.tower()["Gamma"]
    m = np.diff(np.concatenate([[0], lab.astype(np.int64)]))
    t = 0.0
    for h, mm in enumerate(m.tolist(), start=1):  # the clock streams index hops from 1
        t = t + oracle.gamma_dt(3, 1, h, mm, G)
    assert o.scalars()["t"] == t
