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


def _rates(o, run_to, t1, t2):
    run_to(o, t1)
    s0 = o.scalars()
    run_to(o, t2)
    s1 = o.scalars()
    dt = s1["t"] - s0["t"]
    return (s1["hops"] - s0["hops"]) / dt, (s1["P"] - s0["P"]) / dt


def test_naive_kmc_and_the_mixed_algorithm_share_the_time_axis():
    """The mixed algorithm with the exact Gamma(m) clock is equivalent to naive KMC (uniform
    pair proposals, clock +1 per N(N-1) proposals): over the same stretch of simulated time
    both execute the same mean number of hops and move the same mean dipole.  Paired by
    disorder (each seed gives both chains the same phi and initial configuration; their
    dynamics draw from different streams), 16 seeds, mean difference within 4 standard
    errors; the comparison resolves a 10% error in the clock."""
    kw = dict(L=8, n_e=32, W=1.0, xi=1.0, rc=2.5, T=0.25, E=0.1)
    t1, t2 = 100.0, 1100.0
    naive, mixed = [], []
    for seed in range(1, 17):
        naive.append(_rates(oracle.Oracle(seed=seed, **kw), lambda o, t: o.naive_run(t), t1, t2))
        mixed.append(_rates(oracle.Oracle(seed=seed, clock_mode=2, **kw),
                            lambda o, t: o.run(0, t_end=t, log_cap=0), t1, t2))
    d = np.array(naive) - np.array(mixed)
    se = d.std(axis=0, ddof=1) / np.sqrt(len(d))
    for k, what in ((0, "hops per unit time"), (1, "dipole per unit time")):
        assert abs(d[:, k].mean()) < 4 * se[k], (what, d[:, k].mean(), se[k])
    rate = np.array(mixed)[:, 0].mean()
    assert 0.1 * rate > 4 * se[0], (rate, se[0])
    assert np.array(mixed)[:, 1].mean() > 0  # the field drives a current along +x
