"""GPU parity of the whole-GPU kernel: one sample on every workgroup of a cooperative launch
(FP64 form; L = 128 ... 2048), through the C ABI, against the serial FP64 oracle."""
import numpy as np
import pytest

from tests.gpu_util import compare_logs, lazy_oracle_of, oracle_of, require_gpu, say
from workloads import Sample

pytestmark = pytest.mark.gpu


def _batch(cg, samples, **opts):
    return cg.Batch(samples, cg.make_opts(**opts))


@pytest.mark.parametrize("M", [1024, 2048])
def test_whole_gpu_kernel_hop_for_hop_l128(M):
    """Forced onto 16 workgroups at L=128 (variant 4), the kernel executes the oracle's hops,
    labels and sites, hop for hop, and ends with its FP64 energies, dipole, clock and energy."""
    cg = require_gpu()
    s = Sample(128, 8192, 1.0, 1.0, 10.0, 0.05, 0.01, 41, 0)
    hops = 2500
    say(f"whole-GPU kernel L=128 M={M}: {hops} hops")
    b = _batch(cg, [s], precision=cg.CG_FP64, M=M, variant=4, log_hops=hops)
    b.run_hops(hops)
    o = oracle_of(s)
    agree = compare_logs(s, b.hop_log(0), o.run(hops))
    assert agree == hops
    assert float(np.abs(b.energies(0) - o.eps()).max()) <= 1e-12
    st, sc = b.stats(0), o.scalars()
    assert st["P"] == sc["P"] and st["hops"] == hops
    assert abs(st["t"] - sc["t"]) <= 1e-12 * sc["t"]
    assert abs(st["H0"] - sc["H0"]) <= 1e-9 * abs(sc["H0"])


def test_whole_gpu_kernel_hop_for_hop_l256_benched_shapes():
    """L = 256 at T = 0.05 (the large-lattice bench leg's parameters) on the grid the bench times
    (64 workgroups, one site per thread) and forced onto 16 workgroups (four sites per thread):
    both execute the full oracle's hops, labels and sites, hop for hop, over launches of several
    hops, and end with its FP64 energies (1e-12), occupation, dipole, clock and energy."""
    cg = require_gpu()
    s = Sample(256, 32768, 1.0, 1.0, 10.0, 0.05, 0.005, 7, 0)
    pieces = [700, 1, 299, 500]
    hops = sum(pieces)
    runs = {}
    for spread in (0, 16):
        say(f"whole-GPU kernel L=256 spread={spread}: {hops} hops")
        b = _batch(cg, [s], precision=cg.CG_FP64, M=1024, spread=spread, log_hops=hops)
        for n in pieces:
            b.run_hops(n)
        runs[spread] = b
    say("whole-GPU kernel L=256: oracle")
    o = oracle_of(s)
    ol = o.run(hops)
    sc = o.scalars()
    eps = o.eps()
    for spread, b in runs.items():
        say(f"whole-GPU kernel L=256 spread={spread}: compare")
        assert compare_logs(s, b.hop_log(0), ol) == hops
        assert np.array_equal(b.occupation(0), o.occ())
        assert float(np.abs(b.energies(0) - eps).max()) <= 1e-12
        st = b.stats(0)
        assert st["P"] == sc["P"] and st["hops"] == hops and st["s_last"] == sc["s_last"]
        assert abs(st["t"] - sc["t"]) <= 1e-12 * sc["t"]
        assert abs(st["H0"] - sc["H0"]) <= 1e-9 * abs(sc["H0"])


def test_whole_gpu_kernel_refuses_unknown_grids():
    cg = require_gpu()
    s = Sample(256, 32768, 1.0, 1.0, 10.0, 0.05, 0.005, 7, 0)
    for spread in (8, 32, 128):
        with pytest.raises(cg.CgError):
            _batch(cg, [s], precision=cg.CG_FP64, spread=spread)
    with pytest.raises(cg.CgError):  # the per-sample kernels take no workgroup count
        _batch(cg, [Sample(64, 2048, 1.0, 1.0, 8.0, 0.05, 0.01, 2, 0)], precision=cg.CG_FP64, spread=16)


def test_whole_gpu_kernel_odd_and_even_launches():
    """Within a launch the kernel alternates two copies of the occupation and the energy mirror
    (hop k reads copy k % 2) and returns to the first copy at the launch's end.  Launches of
    odd and even hop counts, interleaved with reads of the state, must still execute the
    oracle's hops: after every launch the occupation and energies equal the oracle's."""
    cg = require_gpu()
    s = Sample(128, 8192, 1.0, 1.0, 10.0, 0.05, 0.01, 47, 2)
    pieces = [1, 2, 3, 1, 7, 64, 13, 1, 1, 400, 5, 2, 33]
    hops = sum(pieces)
    say(f"whole-GPU kernel L=128: {len(pieces)} launches, {hops} hops")
    b = _batch(cg, [s], precision=cg.CG_FP64, M=1024, variant=4, log_hops=hops)
    o = oracle_of(s)
    logs = []
    for n in pieces:
        b.run_hops(n)
        logs.append(o.run(n))
        assert np.array_equal(b.occupation(0), o.occ())
        assert float(np.abs(b.energies(0) - o.eps()).max()) <= 1e-12
    ol = tuple(np.concatenate([x[k] for x in logs]) for k in range(3))
    assert compare_logs(s, b.hop_log(0), ol) == hops
    st, sc = b.stats(0), o.scalars()
    assert st["P"] == sc["P"] and st["hops"] == hops


def _signed_dx(a, c, L):
    d = (c % L) - (a % L)
    d = np.where(d > L // 2, d - L, d)
    return np.where(d < -(L // 2), d + L, d)


@pytest.mark.parametrize("L,hops", [(256, 400), (1024, 200), (2048, 60)])
def test_whole_gpu_kernel_large_lattice(L, hops):
    """Large lattices (beyond the full oracle): the initial occupation and disorder equal the
    oracle's, sampled initial energies equal its O(N) single-site sum bit for bit (same order);
    after hops every logged hop moves an electron to an empty site, the occupation replays,
    the dipole is the sum of the logged dx, and sampled energies (random sites and the sites of
    the last hops) agree with the single-site recompute to 1e-10."""
    cg = require_gpu()
    s = Sample(L, L * L // 2, 1.0, 1.0, 10.0, 0.05, 0.01, 43, 1)
    say(f"whole-GPU kernel L={L}: init")
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=hops)
    lazy = lazy_oracle_of(s)
    n0 = b.occupation(0)
    assert np.array_equal(n0, lazy.occ())
    assert np.array_equal(b.phi(0), lazy.phi())
    sites = np.random.default_rng(7).choice(L * L, 16, replace=False)
    e0 = b.energies(0)
    for l in sites.tolist():
        assert e0[l] == lazy.site_eps(l), l
    say(f"whole-GPU kernel L={L}: {hops} hops")
    b.run_hops(hops)
    lab, fr, to = b.hop_log(0)
    assert len(lab) == hops and np.all(np.diff(lab.astype(np.int64)) > 0)
    n = n0.copy()
    for a, c in zip(fr.tolist(), to.tolist()):
        assert n[a] == 1 and n[c] == 0
        n[a], n[c] = 0, 1
    assert np.array_equal(n, b.occupation(0))
    st = b.stats(0)
    assert st["hops"] == hops and st["P"] == int(_signed_dx(fr, to, L).sum())
    lazy.set_occ(n)
    e = b.energies(0)
    for l in np.concatenate([sites, fr[-4:], to[-4:]]).tolist():
        assert abs(e[l] - lazy.site_eps(l)) <= 1e-10, l


def test_whole_gpu_kernel_checkpoint():
    """cg_save / cg_load on a whole-GPU sample (L = 256): the energies, their mirror and the
    state come back, and the next hops are the ones the saved run executed."""
    cg = require_gpu()
    s = Sample(256, 32768, 1.0, 1.0, 10.0, 0.05, 0.005, 43, 0)
    say("whole-GPU checkpoint L=256")
    a = _batch(cg, [s], precision=cg.CG_FP64, log_hops=600)
    a.run_hops(300)
    blob = a.save(0)
    a.run_hops(300)
    b = _batch(cg, [s], precision=cg.CG_FP64, log_hops=600)
    b.run_hops(50)
    b.load(0, blob)
    b.run_hops(300)
    la, lb = a.hop_log(0), b.hop_log(0)
    for x, y in zip(la, lb):
        assert np.array_equal(x[300:600], y)
    assert np.array_equal(a.energies(0), b.energies(0))
    sa, sb = a.stats(0), b.stats(0)
    for k in ("hops", "s_last", "P", "t", "H0"):
        assert sa[k] == sb[k], k
