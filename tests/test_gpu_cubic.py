"""GPU parity of the simple cubic lattice (FP64 form, through the C ABI) against the 3D
oracle: initial state, hop-for-hop trajectories, energies, and the refused configurations."""
import numpy as np
import pytest

from oracle import observables as ob
from tests.gpu_util import oracle_of, require_gpu, say
from workloads import Sample

pytestmark = pytest.mark.gpu


def _batch(cg, samples, **opts):
    return cg.Batch(samples, cg.make_opts(**opts))


def _cubes():
    return [Sample(6, 108, 1.0, 1.0, 2.0, 0.1, 0.01, 61, 0, dim=3),
            Sample(8, 256, 1.0, 1.0, 3.0, 0.08, 0.01, 61, 1, dim=3),
            Sample(11, 665, 0.5, 0.8, 2.5, 0.15, 0.0, 61, 2, dim=3),
            Sample(16, 2048, 1.0, 1.0, 4.0, 0.05, 0.005, 61, 3, dim=3)]


def test_cubic_initial_state_matches_oracle():
    cg = require_gpu()
    samples = _cubes() + [Sample(24, 6912, 1.0, 1.0, 3.0, 0.05, 0.005, 61, 4, dim=3)]
    b = _batch(cg, samples, precision=cg.CG_FP64)
    for k, s in enumerate(samples):
        o = oracle_of(s)
        assert np.array_equal(b.occupation(k), o.occ())
        assert np.array_equal(b.phi(k), o.phi())
        assert float(np.abs(b.energies(k) - o.eps()).max()) <= 1e-12
        assert abs(b.stats(k)["H0"] - o.scalars()["H0"]) <= 1e-10 * abs(o.scalars()["H0"])
    say(f"cubic init: {len(samples)} samples equal to the oracle")


def test_cubic_hop_for_hop():
    """Labels, sites, energies, dipole, clock and energy equal to the oracle's over 2500 hops
    in a batch of L = 6, 8, 11, 16 (odd L and a partly filled last chunk of sites included)."""
    cg = require_gpu()
    samples = _cubes()
    hops = 2500
    b = _batch(cg, samples, precision=cg.CG_FP64, log_hops=hops)
    b.run_hops(hops)
    for k, s in enumerate(samples):
        o = oracle_of(s)
        ol = o.run(hops)
        gl = b.hop_log(k)
        n = min(len(gl[0]), len(ol[0]))
        same = (gl[0][:n] == ol[0][:n]) & (gl[1][:n] == ol[1][:n]) & (gl[2][:n] == ol[2][:n])
        first = n if same.all() else int(np.argmin(same))
        assert first == hops, (k, first)
        assert float(np.abs(b.energies(k) - o.eps()).max()) <= 1e-12
        st, sc = b.stats(k), o.scalars()
        assert st["P"] == sc["P"] and st["hops"] == hops and st["s_last"] == sc["s_last"]
        assert abs(st["t"] - sc["t"]) <= 1e-12 * sc["t"]
        assert abs(st["H0"] - sc["H0"]) <= 1e-9 * abs(sc["H0"])
        assert abs(st["H0"] - o.energy()) <= 1e-9 * abs(sc["H0"])
    say(f"cubic: {hops} hops x {len(samples)} samples equal to the oracle")


def test_cubic_large_sample_and_dos():
    """L = 24 (13824 sites, the largest cubic lattice): 800 hops equal to the oracle, and the
    density-of-states counts equal to the oracle's count of its own energies."""
    cg = require_gpu()
    s = Sample(24, 6912, 1.0, 1.0, 3.0, 0.05, 0.005, 62, 0, dim=3)
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=800)
    b.run_hops(800)
    o = oracle_of(s)
    ol = o.run(800)
    for x, y in zip(b.hop_log(0), ol):
        assert np.array_equal(x, y)
    occ, emp, below, above = b.dos(0, 1, -3.0, 3.0, 120)
    ro, re, rb, ra = ob.dos_counts(o.eps(), o.occ(), -3.0, 3.0, 120)
    assert np.array_equal(occ, ro) and np.array_equal(emp, re) and (below, above) == (rb, ra)


def test_cubic_refused_configurations():
    cg = require_gpu()
    ok = Sample(8, 256, 1.0, 1.0, 3.0, 0.08, 0.01, 61, 1, dim=3)
    for samples, kw in (([ok], dict(precision=cg.CG_FP32_REFRESH)),
                        ([ok], dict(precision=cg.CG_FP64, clock_mode=cg.CG_CLOCK_GAUSS)),
                        ([ok, Sample(16, 128, 1.0, 1.0, 6.0, 0.1, 0.01, 1, 0)], dict(precision=cg.CG_FP64)),
                        ([Sample(25, 7812, 1.0, 1.0, 3.0, 0.08, 0.01, 61, 1, dim=3)], dict(precision=cg.CG_FP64)),
                        ([Sample(8, 256, 1.0, 1.0, 4.0, 0.08, 0.01, 61, 1, dim=3)], dict(precision=cg.CG_FP64)),
                        ([Sample(8, 256, 1.0, 1.0, 3.0, 0.08, 0.01, 61, 1, dim=4)], dict(precision=cg.CG_FP64)),
                        ([ok], dict(precision=cg.CG_FP64, variant=3)),
                        ([ok], dict(precision=cg.CG_FP64, variant=6, use_graph=1))):
        with pytest.raises(cg.CgError):
            _batch(cg, samples, **kw)


@pytest.mark.parametrize("spread,pieces", [(1, [2500]), (5, [1, 700, 1799]), (0, [3, 2497])])
def test_cubic_label_parallel_hop_for_hop(spread, pieces):
    """The cubic label-parallel kernel (variant 6: a replica of each sample per workgroup,
    rounds of spread x 1024 labels, one sample after another) executes the oracle's hops for
    every spread, over launches of several sizes, in a batch of L = 6, 8, 11, 16."""
    cg = require_gpu()
    samples = _cubes()
    hops = sum(pieces)
    say(f"cubic label-parallel spread={spread}: {hops} hops in {len(pieces)} launches")
    b = _batch(cg, samples, precision=cg.CG_FP64, log_hops=hops, variant=6, spread=spread)
    for n in pieces:
        b.run_hops(n)
    for k, s in enumerate(samples):
        o = oracle_of(s)
        ol = o.run(hops)
        gl = b.hop_log(k)
        for x, y in zip(gl, ol):
            assert np.array_equal(x, y), k
        assert np.array_equal(b.occupation(k), o.occ())
        assert float(np.abs(b.energies(k) - o.eps()).max()) <= 1e-12
        st, sc = b.stats(k), o.scalars()
        assert st["P"] == sc["P"] and st["hops"] == hops and st["s_last"] == sc["s_last"]
        assert abs(st["t"] - sc["t"]) <= 1e-12 * sc["t"]
        assert abs(st["H0"] - sc["H0"]) <= 1e-9 * abs(sc["H0"])


def test_cubic_label_parallel_low_temperature_and_run_to_time():
    """At T = 0.01 (thousands of labels per hop) the label-parallel kernel still follows the
    oracle hop for hop, and run-to-time stops at the oracle's hop."""
    cg = require_gpu()
    s = Sample(12, 864, 1.0, 1.0, 3.0, 0.01, 0.001, 67, 0, dim=3)
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=600, variant=6)
    o = oracle_of(s)
    b.run_hops(300)
    ol = o.run(300)
    for x, y in zip(b.hop_log(0), ol):
        assert np.array_equal(x, y)
    t_end = o.scalars()["t"] * 1.5
    b.run_time(t_end)
    st = b.stats(0)
    assert st["t"] >= t_end and st["hops"] > 300
    # the oracle reaches the same stopping hop: run it hop by hop to the GPU's count
    o2 = oracle_of(s)
    o2.run(st["hops"] - 1)
    assert o2.scalars()["t"] < t_end
    o2.run(1)
    sc = o2.scalars()
    assert sc["t"] >= t_end and sc["s_last"] == st["s_last"]
    say(f"cubic label-parallel T=0.01: {st['hops']} hops, m_bar = {st['s_last'] / st['hops']:.0f}")
