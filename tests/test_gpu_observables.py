"""GPU density of states (cg_dos, through the C ABI) against the oracle's definition of the
counts on the oracle's own energies, and a short temperature sweep of the observables."""
import numpy as np
import pytest

from oracle import observables as ob
from tests.gpu_util import oracle_of, require_gpu, say
from workloads import Sample

pytestmark = pytest.mark.gpu


def _batch(cg, samples, **opts):
    return cg.Batch(samples, cg.make_opts(**opts))


@pytest.mark.parametrize("hops", [0, 3000])
def test_dos_matches_oracle_fp64(hops):
    """FP64 form: the counts of every bin, both occupations, and outside the range are
    equal to the oracle's count of its own energies (the trajectories are equal hop for hop)."""
    cg = require_gpu()
    samples = [Sample(48, 1152, 1.0, 1.0, 6.0, 0.08, 0.008, 21, b) for b in range(3)]
    b = _batch(cg, samples, precision=cg.CG_FP64)
    if hops:
        b.run_hops(hops)
    for (first, count, lo, hi, nb) in ((0, 1, -2.0, 2.0, 64), (1, 2, -1.3, 1.7, 4096), (0, 3, -0.5, 0.5, 7)):
        occ, emp, below, above = b.dos(first, count, lo, hi, nb)
        ro = np.zeros(nb, np.uint64)
        re = np.zeros(nb, np.uint64)
        rb = ra = 0
        for k in range(first, first + count):
            o = oracle_of(samples[k])
            if hops:
                o.run(hops)
            a, c, d, e = ob.dos_counts(o.eps(), o.occ(), lo, hi, nb)
            ro, re, rb, ra = ro + a, re + c, rb + d, ra + e
        assert np.array_equal(occ, ro) and np.array_equal(emp, re) and (below, above) == (rb, ra)
    say(f"DOS FP64 after {hops} hops equal to the oracle's")


def test_dos_fp32_within_edge_tolerance():
    """FP32 form: energies within the drift bound (1e-5) of the oracle's FP64 ones, so a bin
    can differ only by sites whose oracle energy lies within 1e-5 of one of its edges."""
    cg = require_gpu()
    samples = [Sample(64, 2048, 1.0, 1.0, 8.0, 0.05, 0.01, 2, 0)]
    b = _batch(cg, samples, precision=cg.CG_FP32_REFRESH, K_refresh=1024)
    b.run_hops(1500)
    lo, hi, nb = -2.0, 2.0, 200
    occ, emp, below, above = b.dos(0, 1, lo, hi, nb)
    o = oracle_of(samples[0])
    o.run(1500)
    eps = o.eps()
    a, c, d, e = ob.dos_counts(eps, o.occ(), lo, hi, nb)
    assert int(occ.sum() + emp.sum()) + below + above == 64 * 64
    edges = lo + (hi - lo) / nb * np.arange(nb + 1)
    near = np.abs(eps[:, None] - edges[None, :]).min(axis=1) < 1e-5
    allowed = int(near.sum())
    diff = int(np.abs(occ.astype(np.int64) - a.astype(np.int64)).sum() +
               np.abs(emp.astype(np.int64) - c.astype(np.int64)).sum())
    assert diff <= 2 * allowed, (diff, allowed)
    say(f"DOS FP32: {diff} bin differences, {allowed} oracle energies within 1e-5 of an edge")


def test_dos_rejects_bad_arguments():
    cg = require_gpu()
    b = _batch(cg, [Sample(16, 128, 1.0, 1.0, 6.0, 0.1, 0.01, 1, 0)], precision=cg.CG_FP64)
    for args in ((0, 1, -1.0, 1.0, 0), (0, 1, -1.0, 1.0, 4097), (0, 1, 1.0, 1.0, 8), (0, 2, -1.0, 1.0, 8),
                 (-1, 1, -1.0, 1.0, 8), (0, 0, -1.0, 1.0, 8)):
        with pytest.raises(cg.CgError):
            b.dos(*args)


def test_short_sweep_observables():
    """A short sweep at L=32: positive sigma_0 growing with T, the DOS counts every site, and
    the Coulomb gap: fewer states at eps ~ 0 than at |eps| ~ 0.5."""
    cg = require_gpu()
    from paper_1407_5026_amd import observables as lib

    res = lib.sweep(cg, 32, [0.1, 0.2], 64, 9, 1.0, 6, cg.CG_FP32_REFRESH)
    s = [r["sigma0"] for r in res["temps"]]
    assert s[0] > 0 and s[1] > s[0]
    for r in res["temps"]:
        g = np.array(r["dos_g"])
        c = np.array(r["dos_centres"])
        width = c[1] - c[0]
        inside = 64 * 32 * 32 - sum(r["dos_outside"])
        assert abs(g.sum() * width * 64 * 32 * 32 - inside) < 1e-6
        g0 = g[np.abs(c) < 0.05].mean()
        g5 = g[np.abs(np.abs(c) - 0.5) < 0.05].mean()
        assert g0 < g5
    say(f"sweep L=32: sigma0 = {s}")
