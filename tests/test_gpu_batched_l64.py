"""The batched temperature grid at its full size: 256 samples at L = 64 (seed 4, sample ids
0..255), rc = 8, E = 0.01, T round-robin over {0.02, 0.03, 0.05, 0.08, 0.12}, M = 2048, one
launch for the whole batch (one workgroup per sample, every sample at its own temperature).

* FP64 form: five samples spanning the grid (one per temperature) execute the oracle's hops
  hop for hop, with energies to 1e-12, dipole, clock and energy.
* FP32 form with its FP64 refresh every 2048 hops: the same five samples follow the oracle up
  to the first label the FP32 rounding can decide the other way; the full run of 2 x 10^5 hops
  per sample keeps the drift within 1e-5 at every refresh on all 256 samples, conserves charge,
  keeps the clock at s_last / Gamma, and ends with energies that a single-site FP64 recompute
  of the final occupation reproduces to 1e-5 at sampled sites."""
import numpy as np
import pytest

from tests.gpu_util import compare_logs, compare_logs_fp32, lazy_oracle_of, oracle_of, require_gpu, say
from workloads import batched_l64

pytestmark = pytest.mark.gpu

M, K = 2048, 2048
CHECKED = (0, 1, 2, 3, 4, 130, 254)  # T = 0.02, 0.03, 0.05, 0.08, 0.12, 0.02, 0.08


def test_batched_l64_fp64_hop_for_hop():
    cg = require_gpu()
    samples = batched_l64(256)
    hops = 3000
    say(f"batched L=64 FP64: 256 samples, {hops} hops")
    b = cg.Batch(samples, cg.make_opts(precision=cg.CG_FP64, M=M, log_hops=hops))
    b.run_hops(hops)
    for k in CHECKED:
        s = samples[k]
        o = oracle_of(s)
        say(f"batched L=64 FP64 sample {k} T={s.T}")
        assert compare_logs(s, b.hop_log(k), o.run(hops)) == hops
        assert float(np.abs(b.energies(k) - o.eps()).max()) <= 1e-12
        st, sc = b.stats(k), o.scalars()
        assert st["P"] == sc["P"] and st["s_last"] == sc["s_last"] and st["t"] == sc["t"]
        assert abs(st["H0"] - sc["H0"]) <= 1e-9 * max(1.0, abs(sc["H0"]))
        assert np.array_equal(b.occupation(k), o.occ())


def test_batched_l64_fp32_until_the_first_near_tie():
    cg = require_gpu()
    samples = batched_l64(256)
    hops = 3 * K
    say(f"batched L=64 FP32: 256 samples, {hops} hops")
    b = cg.Batch(samples, cg.make_opts(precision=cg.CG_FP32_REFRESH, M=M, K_refresh=K, log_hops=hops))
    b.run_hops(hops)
    for k in CHECKED:
        s = samples[k]
        o = oracle_of(s)
        eps_max = max(float(np.abs(o.eps()).max()), float(np.abs(b.energies(k)).max()))
        st = b.stats(k)
        assert st["refreshes"] == hops // K and st["max_drift"] <= 1e-5
        agree = compare_logs_fp32(s, b.hop_log(k), o.run(hops), st["max_drift"], eps_max)
        say(f"batched L=64 FP32 sample {k} T={s.T}: {agree} of {hops} hops identical to the oracle")
        # measured: every compared hop identical (6144 of 6144 for each checked sample); an FP32
        # near-tie within the first half would be a new finding to look at
        assert agree >= hops // 2


def test_batched_l64_fp32_full_run():
    cg = require_gpu()
    from tests.pins import disk_vectors

    samples = batched_l64(256)
    hops, step = 200_000, 8192
    say(f"batched L=64 FP32 full run: 256 samples x {hops} hops")
    b = cg.Batch(samples, cg.make_opts(precision=cg.CG_FP32_REFRESH, M=M, K_refresh=K))
    done = 0
    while done < hops:
        n = min(step, hops - done)
        b.run_hops(n)
        done += n
    s0 = samples[0]
    d = np.array(sorted(disk_vectors(s0.rc)), dtype=float)
    gamma = s0.L * s0.L * float(np.exp(-2.0 * np.sqrt((d * d).sum(1)) / s0.xi).sum())
    for k, s in enumerate(samples):
        st = b.stats(k)
        assert st["hops"] == hops and st["status"] == 0, k
        assert st["refreshes"] == hops // K, (k, st["refreshes"])
        assert st["max_drift"] <= 1e-5, (k, st["max_drift"])
        assert abs(st["t"] - st["s_last"] / gamma) <= 1e-14 * st["t"], k
        assert int(b.occupation(k).sum()) == s.n_e, k
    for k in CHECKED[:5]:
        s = samples[k]
        lazy = lazy_oracle_of(s)
        lazy.set_occ(b.occupation(k))
        e = b.energies(k)
        for l in np.random.default_rng(k).choice(s.L * s.L, 12, replace=False).tolist():
            assert abs(e[l] - lazy.site_eps(l)) <= 1e-5, (k, l)
