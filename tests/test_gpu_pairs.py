"""GPU parity of the pair-hop model (two electrons moving at once, the multi-electron
extension the paper names in sections "Code performance" and "Conclusions"; the reading is
stated in the kernel and the oracle): the pair-hop kernel through the C ABI against the
serial FP64 oracle with the same pair probability, hop for hop."""
import numpy as np
import pytest

from tests.gpu_util import oracle_of, require_gpu, say
from workloads import Sample

pytestmark = pytest.mark.gpu


def _compare(sample, gpu_log, or_log, tol=1e-12):
    """Entries (label, from, to) equal; a pair hop is two entries with one label.  The only
    allowed divergence is a flip at the first differing label where the oracle's
    |u - P_acc| < tol (single or pair proposal); returns the entries that agree."""
    gl, gi, gj = gpu_log
    ol, oi, oj = or_log
    n = min(len(gl), len(ol))
    same = (gl[:n] == ol[:n]) & (gi[:n] == oi[:n]) & (gj[:n] == oj[:n])
    if same.all():
        assert len(gl) == len(ol), (len(gl), len(ol))
        return n
    k = int(np.argmin(same))
    assert k == 0 or ol[k] != ol[k - 1], f"entry {k}: the two moves of the pair hop at label {ol[k]} differ"
    o = oracle_of(sample)
    hops_before = len(np.unique(ol[:k]))  # every label before entry k is a whole hop
    if hops_before:
        o.run(hops_before)
    s = int(min(gl[k], ol[k]))
    is_pair, i, v1, ve, v2, u = o.draw_label(s)
    p, dH = o.move_pair(i, v1, ve, v2) if is_pair else o.move(i, v1)
    assert abs(u - p) < tol, (f"entry {k}: gpu (label {gl[k]}, {gi[k]}->{gj[k]}) vs oracle (label {ol[k]}, "
                              f"{oi[k]}->{oj[k]}); label {s} pair={is_pair} u={u!r} P_acc={p!r} dH={dH!r}")
    say(f"allowed flip at entry {k}: label {s} |u - P_acc| = {abs(u - p):.3g}")
    return k


def _check(cg, b, k, s, hops, clock_mode=0):
    o = oracle_of(s, clock_mode=clock_mode)
    ol = o.run(hops)
    gl = b.hop_log(k)
    n_pair_entries = int(len(ol[0]) - len(np.unique(ol[0])))
    agree = _compare(s, gl, ol)
    if agree == len(ol[0]):
        st, sc = b.stats(k), o.scalars()
        assert st["hops"] == sc["hops"] == hops
        assert st["s_last"] == sc["s_last"] and st["P"] == sc["P"]
        if clock_mode == 0:
            assert st["t"] == sc["t"]
        else:
            assert abs(st["t"] - sc["t"]) <= 1e-12 * max(1.0, abs(sc["t"]))
        assert abs(st["H0"] - sc["H0"]) <= 1e-9 * max(1.0, abs(sc["H0"]))
        assert np.array_equal(b.occupation(k), o.occ())
        d = float(np.abs(b.energies(k) - o.eps()).max())
        assert d <= 1e-12, d
    return agree, n_pair_entries


@pytest.mark.parametrize("pair", [0.1, 0.5])
def test_pair_hops_hop_for_hop(pair):
    """A batch of lattices (L = 16, 24, 33 with odd L, 64) with the pair probability, and one
    sample with pair = 0 in the same launch (the paper's chain on the pair-hop kernel)."""
    cg = require_gpu()
    samples = [Sample(16, 128, 1.0, 1.0, 6.0, 0.1, 0.01, 41, 0, pair=pair),
               Sample(24, 250, 0.7, 1.3, 5.0, 0.07, 0.02, 42, 1, pair=pair),
               Sample(33, 544, 1.0, 1.0, 8.0, 0.05, 0.01, 43, 2, pair=pair),
               Sample(64, 2048, 1.0, 1.0, 8.0, 0.05, 0.01, 44, 3, pair=pair),
               Sample(16, 128, 1.0, 1.0, 6.0, 0.1, 0.01, 45, 4, pair=0.0)]
    hops = 3000
    b = cg.Batch(samples, cg.make_opts(precision=cg.CG_FP64, log_hops=2 * hops))
    # two calls: the state (labels, energies, clock) carries across launches
    b.run_hops(1200)
    b.run_hops(hops - 1200)
    for k, s in enumerate(samples):
        agree, npair = _check(cg, b, k, s, hops)
        say(f"pair={s.pair} L={s.L}: {agree} log entries agree ({npair} pair hops)")
        if s.pair > 0:
            assert npair > 0
        else:
            assert npair == 0
    b.close()


@pytest.mark.parametrize("clock_mode", [1, 2])
def test_pair_hops_stochastic_clocks_and_run_to_time(clock_mode):
    """The Gaussian and Gamma clocks run at the label rate Gamma / (1 - pair); run-to-time
    stops at the oracle's hop."""
    cg = require_gpu()
    s = Sample(32, 512, 1.0, 1.0, 8.0, 0.08, 0.01, 46, 0, pair=0.3)
    b = cg.Batch([s], cg.make_opts(precision=cg.CG_FP64, clock_mode=clock_mode, log_hops=8000))
    b.run_hops(1500)
    agree, _ = _check(cg, b, 0, s, 1500, clock_mode=clock_mode)
    assert agree == len(b.hop_log(0)[0])
    t_end = b.stats(0)["t"] * 1.7
    b.run_time(t_end)
    o = oracle_of(s, clock_mode=clock_mode)
    o.run(1500)
    o.run(0, t_end=t_end)
    st, sc = b.stats(0), o.scalars()
    assert st["hops"] == sc["hops"] and st["s_last"] == sc["s_last"]
    assert abs(st["t"] - sc["t"]) <= 1e-12 * sc["t"] and st["t"] >= t_end
    b.close()


def test_pair_hops_checkpoint_and_deterministic_run_to_time():
    cg = require_gpu()
    s = Sample(32, 512, 1.0, 1.0, 8.0, 0.06, 0.01, 47, 0, pair=0.2)
    b = cg.Batch([s], cg.make_opts(precision=cg.CG_FP64))
    b.run_hops(700)
    blob = b.save(0)
    b.run_hops(900)
    ref = (b.energies(0), b.occupation(0), b.stats(0))
    b2 = cg.Batch([s], cg.make_opts(precision=cg.CG_FP64))
    b2.load(0, blob)
    b2.run_hops(900)
    assert np.array_equal(b2.energies(0), ref[0]) and np.array_equal(b2.occupation(0), ref[1])
    assert b2.stats(0)["s_last"] == ref[2]["s_last"] and b2.stats(0)["t"] == ref[2]["t"]
    # a checkpoint of another pair probability is refused
    b3 = cg.Batch([Sample(32, 512, 1.0, 1.0, 8.0, 0.06, 0.01, 47, 0, pair=0.25)], cg.make_opts(precision=cg.CG_FP64))
    with pytest.raises(cg.CgError):
        b3.load(0, blob)
    # run to time with the deterministic clock t = s_last (1 - pair) / Gamma
    t_end = ref[2]["t"] * 1.5
    b2.run_time(t_end)
    o = oracle_of(s)
    o.run(1600)
    o.run(0, t_end=t_end)
    assert b2.stats(0)["hops"] == o.scalars()["hops"] and b2.stats(0)["t"] == o.scalars()["t"]
    for x in (b, b2, b3):
        x.close()
