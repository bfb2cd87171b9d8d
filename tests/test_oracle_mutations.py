"""Plant known mistakes in the oracle (on the CPU) and show that its pins catch each one."""
import math

import pytest

import oracle
from tests import pins


def _dh_field():
    o = oracle.Oracle(L=8, n_e=32, rc=3.0, T=0.2, E=0.05, seed=9)
    return pins.check_dh_identity(o, n_moves=60)


def _incremental():
    o = oracle.Oracle(L=12, n_e=72, rc=5.0, T=0.1, E=0.01, seed=1)
    return pins.check_incremental_eps(o, 2000)


def _invariants():
    o = oracle.Oracle(L=12, n_e=72, rc=5.0, T=0.1, E=0.01, seed=2)
    return pins.check_invariants(o, 2000)


def _draws():
    o = oracle.Oracle(L=16, n_e=128, rc=6.0, seed=3)
    return pins.check_displacement_draws(o, 1.0, n=50_000)


def _symmetry():
    o = oracle.Oracle(L=16, n_e=128, rc=6.0, seed=3)
    return pins.check_proposal_symmetry(o)


def _gamma():
    o = oracle.Oracle(L=16, n_e=128, rc=6.0)
    return pins.check_gamma_pairs(o, 16, 1.0, 6.0)


# mutation id -> (what it plants, checks expected to catch it)
CASES = {
    1: ("field term sign flipped in dH", [_dh_field]),
    2: ("-1/r_ij dropped from dH", [_dh_field, pins.check_boltzmann_exact_3x3]),
    3: ("hop sites skipped by the energy update", [_incremental]),
    4: ("occupancy filter ignores n_j", [_invariants]),
    5: ("orbit member always the first", [_draws, pins.check_boltzmann_exact_3x3]),
    6: ("tunnelling weight exp(-r/xi)", [_gamma, _draws]),
    7: ("background nu dropped from eps", [pins.check_eps_closed_form_3x3]),
    8: ("Metropolis uses exp(-dH*T)", [pins.check_boltzmann_exact_3x3]),
    9: ("dipole sign flipped", [_invariants]),
    10: ("energy update sign flipped", [_incremental]),
}


@pytest.mark.parametrize("mut", sorted(CASES))
def test_planted_mistake_is_caught(mut):
    what, checks = CASES[mut]
    oracle.set_mutation(mut)
    try:
        results = []
        for chk in checks:
            try:
                ok, msg = chk()
            except Exception as e:  # a crash of the check also counts as detection
                ok, msg = False, f"raised {type(e).__name__}: {e}"
            results.append((chk.__name__, ok, msg))
    finally:
        oracle.set_mutation(0)
    assert any(not ok for _, ok, _ in results), f"mutation {mut} ({what}) not caught: {results}"


def test_unmutated_oracle_passes_the_same_checks():
    for _, checks in CASES.values():
        for chk in checks:
            ok, msg = chk()
            assert ok, (chk.__name__, msg)
