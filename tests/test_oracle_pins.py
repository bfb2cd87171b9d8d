"""Oracle pinned to closed forms, brute force, identities and invariants (CPU only)."""
import math

import numpy as np
import pytest

import oracle
from tests import pins


@pytest.mark.parametrize("rc,count", [(6.0, 112), (8.0, 196), (10.0, 316), (math.sqrt(2.0), 8)])
def test_displacement_set(rc, count):
    L = 3 if rc < 2 else 32
    o = oracle.Oracle(L=L, n_e=L * L // 2, rc=rc)
    ok, msg = pins.check_displacement_set(o, rc)
    assert ok, msg
    assert o.n_vec == count


@pytest.mark.parametrize("rc", [6.0, 10.0])
def test_proposal_symmetry(rc):
    o = oracle.Oracle(L=32, n_e=512, rc=rc)
    ok, msg = pins.check_proposal_symmetry(o)
    assert ok, msg


@pytest.mark.parametrize("L,xi,rc", [(16, 1.0, 6.0), (24, 1.5, 8.0), (3, 1.0, math.sqrt(2.0))])
def test_gamma_brute_force(L, xi, rc):
    o = oracle.Oracle(L=L, n_e=L * L // 2, xi=xi, rc=rc)
    ok, msg = pins.check_gamma_pairs(o, L, xi, rc)
    assert ok, msg


def test_displacement_draws():
    o = oracle.Oracle(L=16, n_e=128, rc=6.0, seed=3)
    ok, msg = pins.check_displacement_draws(o, 1.0)
    assert ok, msg


def test_site_and_u():
    o = oracle.Oracle(L=16, n_e=128, rc=6.0, seed=4)
    ok, msg = pins.check_site_and_u(o)
    assert ok, msg


def test_eps_closed_form_3x3():
    ok, msg = pins.check_eps_closed_form_3x3()
    assert ok, msg


@pytest.mark.parametrize("E", [0.0, 0.05])
def test_dh_identity(E):
    o = oracle.Oracle(L=8, n_e=32, rc=3.0, T=0.2, E=E, seed=9)
    o.run(50)
    ok, msg = pins.check_dh_identity(o)
    assert ok, msg


def test_incremental_eps_matches_recompute():
    o = oracle.Oracle(L=16, n_e=128, rc=6.0, T=0.1, E=0.01, seed=1)
    ok, msg = pins.check_incremental_eps(o, 20_000)
    assert ok, msg


@pytest.mark.parametrize("clock", [0, 1])
def test_invariants(clock):
    o = oracle.Oracle(L=16, n_e=128, rc=6.0, T=0.1, E=0.01, seed=2, clock_mode=clock)
    ok, msg = pins.check_invariants(o, 5000)
    assert ok, msg


def test_energy_total_tracks_eq1():
    """H0 updated by the executed dH stays equal to Eq. 1 of the current occupation."""
    o = oracle.Oracle(L=12, n_e=72, rc=5.0, T=0.1, E=0.01, seed=8)
    o.run(3000)
    H = pins.eq1_energy(12, o.occ(), o.phi())
    assert abs(o.scalars()["H0"] - H) < 1e-10


def test_boltzmann_exact_3x3():
    ok, msg = pins.check_boltzmann_exact_3x3()
    assert ok, msg


def test_boltzmann_sampled_3x3():
    ok, msg = pins.check_boltzmann_sampled_3x3()
    assert ok, msg


def test_geometric_m_and_pr_iterations():
    ok, msg = pins.check_geometric_m()
    assert ok, msg


def test_fig1a_reading():
    """m = (p-1) M + q with 1-based q reproduces the worked example of Fig. 1(a)."""
    import os

    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "fig1a.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = int(v)
    M, m = vals["M"], vals["m"]
    p = -(-m // M)
    q = m - (p - 1) * M
    assert (p, q) == (vals["p"], vals["q"])


def test_gaussian_clock_mean():
    """Step 3c: the Gaussian increment has mean m/Gamma, so t*Gamma ~ s_last over many hops."""
    o = oracle.Oracle(L=16, n_e=128, rc=6.0, T=0.1, E=0.01, seed=12, clock_mode=1)
    o.run(20_000)
    sc = o.scalars()
    # Var(dt) = m/Gamma^2 per hop -> sd(t Gamma) = sqrt(s_last)
    assert abs(sc["t"] * sc["Gamma"] - sc["s_last"]) < 5.0 * math.sqrt(sc["s_last"])


def test_philox_matches_torch_engine(tmp_path):
    """Library pin: the oracle's Philox4x32-10 equals PyTorch's host philox_engine
    (counter = (offset_lo, offset_hi, subsequence_lo, subsequence_hi), key = seed)."""
    import os
    import shutil
    import subprocess

    import torch

    inc = os.path.join(os.path.dirname(torch.__file__), "include")
    if not shutil.which("g++") or not os.path.exists(os.path.join(inc, "ATen/core/PhiloxRNGEngine.h")):
        pytest.skip("torch Philox header or g++ unavailable")
    src = tmp_path / "ph.cpp"
    src.write_text(
        "#include <ATen/core/PhiloxRNGEngine.h>\n#include <cstdio>\n#include <cstdlib>\n"
        "int main(int c,char**v){unsigned long long s=strtoull(v[1],0,0),q=strtoull(v[2],0,0),"
        "o=strtoull(v[3],0,0);at::philox_engine e(s,q,o);for(int k=0;k<4;k++)printf(\"%u \",e());}\n")
    exe = tmp_path / "ph"
    subprocess.run(["g++", "-std=c++17", "-O1", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    rng = np.random.default_rng(0)
    for _ in range(64):
        c = rng.integers(0, 2**32, size=4, dtype=np.uint64)
        k = rng.integers(0, 2**32, size=2, dtype=np.uint64)
        seed = int(k[0]) | (int(k[1]) << 32)
        sub = int(c[2]) | (int(c[3]) << 32)
        off = int(c[0]) | (int(c[1]) << 32)
        out = subprocess.run([str(exe), str(seed), str(sub), str(off)], capture_output=True,
                             text=True, check=True).stdout.split()
        want = np.array([int(w) for w in out], dtype=np.uint32)
        got = oracle.philox(c.astype(np.uint32), k.astype(np.uint32))
        assert np.array_equal(got, want), (c, k, got, want)


def test_lazy_oracle_and_site_energy():
    """The lazy oracle (no O(N^2) energies) draws the same occupation and disorder as the full
    one, and its O(N) single-site energy equals the full recompute at every site, before and
    after hops, bit for bit (same summation order); running a lazy state is refused."""
    import numpy as np

    import oracle

    kw = dict(L=16, n_e=128, W=1.0, xi=1.0, rc=6.0, T=0.1, E=0.01, seed=11, sample_id=3)
    full = oracle.Oracle(**kw)
    lazy = oracle.Oracle(lazy=True, **kw)
    assert np.array_equal(full.occ(), lazy.occ())
    assert np.array_equal(full.phi(), lazy.phi())
    e = full.eps()
    assert all(lazy.site_eps(l) == e[l] for l in range(full.N))
    full.run(300)
    lazy.set_occ(full.occ())
    e = full.recompute_eps()
    assert all(lazy.site_eps(l) == e[l] for l in range(full.N))
    with pytest.raises(ValueError):
        lazy.run(1)
