"""Pins of the oracle's pair hops (two electrons moving at once; the reading is stated in
oracle.c): the energy change against Eq. 1 by brute force, exact stationarity of the
Boltzmann law on the 3x3 torus, the invariants of a run, and the proposal law."""
import math

import oracle
from tests import pins


def test_pair_energy_change_is_eq1_difference():
    o = oracle.Oracle(L=8, n_e=32, rc=3.0, T=0.2, E=0.05, seed=9, pair=0.5)
    ok, msg = pins.check_pair_dh_identity(o)
    assert ok, msg


def test_pair_energy_change_after_hops():
    o = oracle.Oracle(L=10, n_e=40, rc=3.0, T=0.15, E=0.02, seed=3, pair=0.3)
    o.run(300)
    ok, msg = pins.check_pair_dh_identity(o, n_moves=80, seed=2)
    assert ok, msg


def test_pair_moves_keep_the_boltzmann_law_exactly():
    ok, msg = pins.check_pair_boltzmann_exact()
    assert ok, msg


def test_pair_moves_keep_the_boltzmann_law_at_low_temperature():
    ok, msg = pins.check_pair_boltzmann_exact(T=0.15, pair=0.8, seed=8)
    assert ok, msg


def test_pair_moves_keep_the_boltzmann_law_with_the_separation_filter():
    ok, msg = pins.check_pair_boltzmann_exact(L=4, n_e=3, rc=1.0, T=0.3, pair=0.5, seed=2)
    assert ok, msg


def test_pair_run_invariants():
    o = oracle.Oracle(L=12, n_e=72, rc=4.0, T=0.1, E=0.01, seed=2, pair=0.3)
    ok, msg = pins.check_pair_invariants(o, 3000)
    assert ok, msg


def test_pair_run_invariants_gaussian_clock_free():
    o = oracle.Oracle(L=16, n_e=100, rc=5.0, T=0.2, E=0.0, seed=4, pair=0.6)
    ok, msg = pins.check_pair_invariants(o, 1500)
    assert ok, msg


def test_pair_proposal_law():
    o = oracle.Oracle(L=16, n_e=128, rc=4.0, seed=3, pair=0.35)
    ok, msg = pins.check_pair_draws(o, 1.0)
    assert ok, msg


def test_zero_pair_fraction_is_the_single_hop_chain():
    a = oracle.Oracle(L=16, n_e=128, rc=6.0, T=0.1, E=0.01, seed=1, pair=0.0)
    b = oracle.Oracle(L=16, n_e=128, rc=6.0, T=0.1, E=0.01, seed=1)
    la, lb = a.run(2000), b.run(2000)
    assert all((x == y).all() for x, y in zip(la, lb))
    assert a.scalars()["Gamma_lab"] == a.scalars()["Gamma"]
    assert math.isclose(a.scalars()["t"], b.scalars()["t"], rel_tol=0, abs_tol=0)
