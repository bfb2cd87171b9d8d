"""GPU parity: the HIP path through the C ABI against the serial FP64 oracle."""
import math

import numpy as np
import pytest

from tests.gpu_util import compare_logs, oracle_of, require_gpu, say
from workloads import Sample, fp64_single, serial_small

pytestmark = pytest.mark.gpu


def _batch(cg, samples, **opts):
    return cg.Batch(samples, cg.make_opts(**opts))


def test_init_matches_oracle():
    cg = require_gpu()
    samples = serial_small() + [Sample(15, 112, 0.5, 1.0, 4.0, 0.2, 0.02, 9, 3),
                                Sample(64, 2048, 1.0, 1.0, 8.0, 0.05, 0.01, 2, 0)]
    for prec in (cg.CG_FP64, cg.CG_FP32_REFRESH):
        b = _batch(cg, samples, precision=prec)
        for k, s in enumerate(samples):
            say(f"init parity precision={prec} sample={k} L={s.L}")
            o = oracle_of(s)
            assert np.array_equal(b.occupation(k), o.occ())
            assert np.array_equal(b.phi(k), o.phi())
            e = b.energies(k)
            if prec == cg.CG_FP64:
                assert np.array_equal(e, o.eps()), float(np.abs(e - o.eps()).max())
            else:
                assert np.array_equal(e, o.eps().astype(np.float32).astype(np.float64))
            st = b.stats(k)
            assert abs(st["H0"] - o.scalars()["H0"]) <= 1e-12 * max(1.0, abs(o.scalars()["H0"]))
            assert st["hops"] == 0 and st["s_last"] == 0


def _check_run(cg, b, k, s, o, hops):
    log = b.hop_log(k)
    ol = o.run(hops)
    agree = compare_logs(s, log, ol)
    if agree == hops:
        st, sc = b.stats(k), o.scalars()
        assert st["hops"] == sc["hops"] == hops
        assert st["s_last"] == sc["s_last"]
        assert st["P"] == sc["P"]
        assert st["t"] == sc["t"]
        assert abs(st["H0"] - sc["H0"]) <= 1e-9 * max(1.0, abs(sc["H0"]))
        assert np.array_equal(b.occupation(k), o.occ())
        d = float(np.abs(b.energies(k) - o.eps()).max())
        assert d <= 1e-12, d
    return agree


def test_fp64_hop_for_hop_small():
    cg = require_gpu()
    s = serial_small()[0]
    hops = 10_000
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=hops)
    say(f"FP64 L=16 {hops} hops")
    b.run_hops(hops)
    _check_run(cg, b, 0, s, oracle_of(s), hops)


@pytest.mark.parametrize("block,M", [(256, 256), (256, 2048), (512, 512), (1024, 1024), (1024, 8192)])
def test_trajectory_independent_of_M_and_block(block, M):
    cg = require_gpu()
    s = serial_small(seed=21)[0]
    hops = 3000
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=hops, block=block, M=M)
    say(f"M-independence block={block} M={M}")
    b.run_hops(hops)
    _check_run(cg, b, 0, s, oracle_of(s), hops)
    st = b.stats(0)
    # p = ceil(m / M) per hop
    lab = b.hop_log(0)[0].astype(np.int64)
    m = np.diff(np.concatenate([[0], lab]))
    assert st["sum_p"] == int(np.sum((m + M - 1) // M))


def test_fp64_l64_hop_for_hop():
    cg = require_gpu()
    s = fp64_single()[0]
    hops = 20_000
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=hops, M=1024)
    say(f"FP64 L=64 {hops} hops")
    b.run_hops(hops)
    _check_run(cg, b, 0, s, oracle_of(s), hops)


def test_mixed_batch_hop_for_hop():
    """One launch, samples of different L (odd, not multiples of 64), T, E, W, rc."""
    cg = require_gpu()
    samples = [Sample(16, 128, 1.0, 1.0, 6.0, 0.1, 0.01, 1, 0),
               Sample(15, 112, 0.5, 1.0, 4.0, 0.2, 0.02, 9, 3),
               Sample(24, 288, 2.0, 1.5, 7.0, 0.05, 0.0, 4, 7),
               Sample(33, 544, 1.0, 1.0, 10.0, 0.08, 0.005, 5, 1),
               Sample(40, 700, 1.0, 0.7, 5.0, 0.03, 0.01, 6, 2)]
    hops = 2500
    b = _batch(cg, samples, precision=cg.CG_FP64, log_hops=hops, block=512, M=1024)
    b.run_hops(hops)
    for k, s in enumerate(samples):
        say(f"mixed batch sample {k} L={s.L}")
        _check_run(cg, b, k, s, oracle_of(s), hops)


def test_run_time_matches_oracle():
    cg = require_gpu()
    s = serial_small(seed=5)[0]
    o = oracle_of(s)
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=20_000)
    for t_end in (5.0, 40.0):
        say(f"run_time t_end={t_end}")
        b.run_time(t_end)
        o.run(0, t_end=t_end, log_cap=0)
        st, sc = b.stats(0), o.scalars()
        assert st["hops"] == sc["hops"] and st["s_last"] == sc["s_last"]
        assert st["t"] == sc["t"] and st["t"] >= t_end
    o2 = oracle_of(s)
    compare_logs(s, b.hop_log(0), o2.run(int(b.stats(0)["hops"])))


def test_resume_is_exact():
    cg = require_gpu()
    s = serial_small(seed=8)[0]
    b1 = _batch(cg, [s], precision=cg.CG_FP64, log_hops=6000)
    b2 = _batch(cg, [s], precision=cg.CG_FP64, log_hops=6000)
    b1.run_hops(5555)
    b2.run_hops(1234)
    b2.run_hops(4321)
    for a, c in zip(b1.hop_log(0), b2.hop_log(0)):
        assert np.array_equal(a, c)
    assert np.array_equal(b1.energies(0), b2.energies(0))
    assert b1.stats(0)["s_last"] == b2.stats(0)["s_last"]


def test_gaussian_clock():
    cg = require_gpu()
    s = serial_small(seed=13)[0]
    hops = 5000
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=hops, clock_mode=cg.CG_CLOCK_GAUSS)
    b.run_hops(hops)
    o = oracle_of(s, clock_mode=1)
    agree = compare_logs(s, b.hop_log(0), o.run(hops))
    assert agree == hops
    t_gpu, t_or = b.stats(0)["t"], o.scalars()["t"]
    assert abs(t_gpu - t_or) <= 1e-9 * t_or, (t_gpu, t_or)


def test_fp32_refresh_drift_and_energies():
    cg = require_gpu()
    s = Sample(64, 2048, 1.0, 1.0, 8.0, 0.05, 0.01, 2, 0)
    K, hops = 512, 4096
    b = _batch(cg, [s], precision=cg.CG_FP32_REFRESH, K_refresh=K, log_hops=hops)
    b.run_hops(hops)
    st = b.stats(0)
    say(f"FP32 refresh: refreshes={st['refreshes']} max drift={st['max_drift']:.3g}")
    assert st["hops"] == hops and st["refreshes"] == hops // K
    assert 0.0 < st["max_drift"] <= 1e-5
    # right after a refresh the FP32 energies are the rounded FP64 recompute of the occupation
    b.refresh()
    o = oracle_of(s)
    o.set_occ(b.occupation(0))
    e64 = o.eps()
    assert np.array_equal(b.energies(0), e64.astype(np.float32).astype(np.float64))
    # charge conservation and a valid hop sequence
    lab, fr, to = b.hop_log(0)
    n = oracle_of(s).occ()
    for a, c in zip(fr.tolist(), to.tolist()):
        assert n[a] == 1 and n[c] == 0
        n[a], n[c] = 0, 1
    assert np.array_equal(n, b.occupation(0))
    assert int(n.sum()) == s.n_e
