"""GPU parity of the label-parallel kernel (variant 6): one sample spread over G workgroups,
each with a replica, evaluating one round of G x 1024 U labels at a time, through the C ABI,
against the serial FP64 oracle.  The hops do not depend on G or U, so every case must match
the oracle hop for hop."""
import numpy as np
import pytest

from tests.gpu_util import compare_logs, oracle_of, require_gpu, say
from workloads import Sample

pytestmark = pytest.mark.gpu


def _batch(cg, samples, **opts):
    return cg.Batch(samples, cg.make_opts(**opts))


@pytest.mark.parametrize(
    "L,rc,T,spread,M,pieces",
    [
        (16, 6.0, 0.1, 3, 1024, [1, 2, 797]),          # N = 256 < 1024 threads
        (32, 8.0, 0.01, 1, 2048, [400, 401]),          # one workgroup, two labels per lane
        (64, 10.0, 0.001, 0, 1024, [1, 150, 49]),      # every CU: ~1e5 proposals per hop
        (64, 8.0, 0.05, 7, 2048, [3, 1500]),
        (128, 10.0, 0.02, 64, 1024, [5, 600]),         # energies in LDS, table in global memory
    ],
)
def test_label_parallel_kernel_hop_for_hop(L, rc, T, spread, M, pieces):
    cg = require_gpu()
    s = Sample(L, L * L // 2, 1.0, 1.0, rc, T, T / 10, 53, 1)
    hops = sum(pieces)
    say(f"label-parallel kernel L={L} T={T} spread={spread} M={M}: {hops} hops in {len(pieces)} launches")
    b = _batch(cg, [s], precision=cg.CG_FP64, M=M, variant=6, spread=spread, log_hops=hops)
    o = oracle_of(s)
    logs = []
    for n in pieces:
        b.run_hops(n)
        logs.append(o.run(n))
        assert np.array_equal(b.occupation(0), o.occ())
    ol = tuple(np.concatenate([x[k] for x in logs]) for k in range(3))
    assert compare_logs(s, b.hop_log(0), ol) == hops
    assert float(np.abs(b.energies(0) - o.eps()).max()) <= 1e-12
    st, sc = b.stats(0), o.scalars()
    assert st["hops"] == hops and st["P"] == sc["P"] and st["s_last"] == sc["s_last"]
    assert abs(st["t"] - sc["t"]) <= 1e-12 * sc["t"]
    assert abs(st["H0"] - sc["H0"]) <= 1e-9 * abs(sc["H0"])
    # every label up to the last hop was evaluated exactly once, some beyond it too
    assert st["evaluated"] >= st["s_last"]
    assert st["theta_pass"] <= st["evaluated"]


def test_label_parallel_kernel_clocks_and_run_to_time():
    """Gamma clock (stochastic increments drawn by every replica) and run-to-time: the hops,
    the clock and the stopping hop are the oracle's."""
    cg = require_gpu()
    s = Sample(64, 2048, 1.0, 1.0, 8.0, 0.03, 0.003, 59, 0)
    hops = 1200
    say("label-parallel kernel L=64: Gamma clock, run to time")
    b = _batch(cg, [s], precision=cg.CG_FP64, variant=6, spread=32, log_hops=4 * hops,
               clock_mode=cg.CG_CLOCK_GAMMA)
    b.run_hops(hops)
    o = oracle_of(s, clock_mode=2)
    assert compare_logs(s, b.hop_log(0), o.run(hops)) == hops
    t_gpu, t_or = b.stats(0)["t"], o.scalars()["t"]
    assert abs(t_gpu - t_or) <= 1e-12 * t_or
    t_end = t_or * 1.37
    b.run_time(t_end)
    o.run(0, t_end=t_end)
    assert b.stats(0)["hops"] == o.scalars()["hops"] > hops
    # deterministic clock: run to time stops after the hop that reaches t_end
    d = _batch(cg, [s], precision=cg.CG_FP64, variant=6, spread=5)
    od = oracle_of(s)
    d.run_hops(300)
    od.run(300)
    t_end = od.scalars()["t"] * 2.1
    d.run_time(t_end)
    od.run(0, t_end=t_end, log_cap=0)
    st, sc = d.stats(0), od.scalars()
    assert st["hops"] == sc["hops"] and st["s_last"] == sc["s_last"]


def test_label_parallel_kernel_batch_and_checkpoint():
    """Two samples of different L run one after the other on the whole GPU; a checkpoint of
    one of them resumes on a fresh context with the same next hops."""
    cg = require_gpu()
    a_s = Sample(32, 512, 1.0, 1.0, 8.0, 0.02, 0.002, 61, 0)
    b_s = Sample(64, 2048, 1.0, 1.0, 8.0, 0.02, 0.002, 61, 1)
    say("label-parallel kernel: batch of L=32 and L=64, checkpoint")
    x = _batch(cg, [a_s, b_s], precision=cg.CG_FP64, variant=6, log_hops=800)
    x.run_hops(400)
    for k, s in enumerate((a_s, b_s)):
        o = oracle_of(s)
        assert compare_logs(s, x.hop_log(k), o.run(400)) == 400
        assert float(np.abs(x.energies(k) - o.eps()).max()) <= 1e-12
    blob = x.save(1)
    x.run_hops(400)
    y = _batch(cg, [b_s], precision=cg.CG_FP64, variant=6, spread=16, log_hops=400)
    y.load(0, blob)
    y.run_hops(400)
    assert np.array_equal(x.hop_log(1)[0][400:800], y.hop_log(0)[0])
    assert np.array_equal(x.energies(1), y.energies(0))


def test_label_parallel_kernel_refusals():
    """FP32 form, L not a power of two in [16, 128], a spread beyond the co-resident
    workgroups, and a spread without variant 6 are refused with CG_EINVAL / CG_ENOSPC."""
    cg = require_gpu()
    s64 = Sample(64, 2048, 1.0, 1.0, 8.0, 0.05, 0.005, 3, 0)
    for samples, opts in [
        ([s64], dict(precision=cg.CG_FP32_REFRESH, variant=6)),
        ([Sample(48, 1152, 1.0, 1.0, 8.0, 0.05, 0.005, 3, 0)], dict(precision=cg.CG_FP64, variant=6)),
        ([Sample(256, 32768, 1.0, 1.0, 8.0, 0.05, 0.005, 3, 0)], dict(precision=cg.CG_FP64, variant=6)),
        ([s64], dict(precision=cg.CG_FP64, variant=1, spread=4)),
        ([s64], dict(precision=cg.CG_FP64, variant=6, spread=100000)),
    ]:
        with pytest.raises(cg.CgError):
            _batch(cg, samples, **opts)
