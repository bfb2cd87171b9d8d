"""The 3D (simple cubic) oracle pinned by counts, closed forms and brute force."""
import itertools
import math

import numpy as np

import oracle


def test_hop_vectors_are_the_lattice_points_of_the_ball():
    # integer points with 0 < x^2 + y^2 + z^2 <= 9 counted by brute force: 122
    o = oracle.Oracle3D(L=8, n_e=256, rc=3.0)
    t = o.tower()
    pts = {(x, y, z) for x, y, z in itertools.product(range(-3, 4), repeat=3) if 0 < x * x + y * y + z * z <= 9}
    vec = set(zip(t["dx"].tolist(), t["dy"].tolist(), t["dz"].tolist()))
    assert len(pts) == 122 and vec == pts and len(t["dx"]) == 122
    # orbit sizes of the cube group: (100) 6, (110) 12, (111) 8, (200) 6, (210) 24, (211) 24,
    # (220) 12, (221) 24, (300) 6
    assert t["size"].tolist() == [6, 12, 8, 6, 24, 24, 12, 24, 6]
    for o_, (f, n) in enumerate(zip(t["first"], t["size"])):
        r2 = {x * x + y * y + z * z for x, y, z in zip(t["dx"][f:f + n], t["dy"][f:f + n], t["dz"][f:f + n])}
        assert len(r2) == 1


def test_proposal_law_is_exp_minus_2r_over_xi():
    xi = 0.8
    o = oracle.Oracle3D(L=10, n_e=500, rc=3.0, xi=xi)
    t = o.tower()
    w = np.array([n * math.exp(-2 * math.sqrt(t["dx"][f] ** 2 + t["dy"][f] ** 2 + t["dz"][f] ** 2) / xi)
                  for f, n in zip(t["first"], t["size"])])
    p = w / w.sum()
    thr = t["thr"].astype(np.float64) * 2.0 ** -32
    q = np.diff(np.concatenate([[0.0], thr]))
    assert np.abs(q - p).max() < 2 ** -31
    # Gamma = N sum_d exp(-2|d|/xi)
    assert abs(t["Gamma"] - 1000 * w.sum()) < 1e-9 * t["Gamma"]


def test_members_of_an_orbit_are_drawn_uniformly():
    o = oracle.Oracle3D(L=8, n_e=256, rc=2.3)
    t = o.tower()
    counts = np.zeros(len(t["dx"]))
    for s in range(1, 60001):
        counts[o.draw(s)[1]] += 1
    for f, n in zip(t["first"], t["size"]):
        c = counts[f:f + n]
        chi2 = ((c - c.mean()) ** 2 / c.mean()).sum()
        assert chi2 < n - 1 + 6 * math.sqrt(2 * (n - 1)), (f, n, c)


def test_minimum_image_distances():
    o = oracle.Oracle3D(L=8, n_e=256, rc=2.0)
    assert o.invr(7, 0, 0) == 1.0 and o.invr(0, -7, 0) == 1.0
    assert o.invr(4, 4, 4) == 1.0 / math.sqrt(48.0)
    assert o.invr(0, 0, 0) == 0.0 and o.invr(8, 16, -8) == 0.0
    assert o.invr(1, 2, 3) == o.invr(-3, 1, -2) == 1.0 / math.sqrt(14.0)


def test_energies_and_energy_after_hops_match_the_definitions():
    o = oracle.Oracle3D(L=6, n_e=108, rc=2.2, T=0.2, E=0.05, seed=9, sample_id=2)
    lab, li, lj = o.run(1500)
    assert len(lab) == 1500 and int(o.occ().sum()) == 108
    # every executed hop moved an electron to an empty site
    n = o.occ()
    eps = o.eps()
    fresh = oracle.Oracle3D(L=6, n_e=108, rc=2.2, T=0.2, E=0.05, seed=9, sample_id=2)
    fresh.set_occ(n)
    assert np.abs(fresh.eps() - eps).max() < 1e-12
    assert abs(o.scalars()["H0"] - o.energy()) < 1e-10 * abs(o.energy())
    # brute-force eps of one site from the definition
    L, nu = 6, 108 / 216
    phi = o.phi()
    l = 77
    xl, yl, zl = l % L, (l // L) % L, l // (L * L)
    acc = phi[l]
    for m in range(216):
        if m != l:
            d = [min(abs(a - b) % L, L - abs(a - b) % L) for a, b in ((xl, m % L), (yl, (m // L) % L), (zl, m // (L * L)))]
            acc += (n[m] - nu) / math.sqrt(sum(x * x for x in d))
    assert abs(acc - eps[l]) < 1e-12


def test_initial_state_is_the_2d_one_for_the_same_site_count():
    # occupation and disorder depend only on the site index and N: L = 4 in 3D and L = 8 in 2D
    a = oracle.Oracle3D(L=4, n_e=32, W=1.3, rc=1.5, seed=5, sample_id=1)
    b = oracle.Oracle(L=8, n_e=32, W=1.3, rc=3.0, seed=5, sample_id=1)
    assert np.array_equal(a.occ(), b.occ()) and np.array_equal(a.phi(), b.phi())
