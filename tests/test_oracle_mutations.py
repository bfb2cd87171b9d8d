"""Plant known mistakes in copies of the oracle's source (on the CPU) and show that its pins
catch each one.  The shipped oracle.c carries no switch: each case below replaces one exact
piece of its source text, compiles the copy with the regular flags and runs the checks
against it.  A case whose text no longer occurs in oracle.c fails, so the cases follow the
source."""
import tempfile

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


def _pair_dh():
    o = oracle.Oracle(L=8, n_e=32, rc=3.0, T=0.2, E=0.05, seed=9, pair=0.5)
    return pins.check_pair_dh_identity(o, n_moves=60)


def _pair_exact_filter():
    return pins.check_pair_boltzmann_exact(L=4, n_e=3, rc=1.0, T=0.3, pair=0.5, seed=2)


def _pair_invariants():
    o = oracle.Oracle(L=12, n_e=72, rc=4.0, T=0.3, E=0.01, seed=2, pair=0.4)
    return pins.check_pair_invariants(o, 1500)


def _pair_draws():
    o = oracle.Oracle(L=16, n_e=128, rc=4.0, seed=3, pair=0.35)
    return pins.check_pair_draws(o, 1.0, n=30_000)


# case -> (what it plants, (original text, planted text), checks expected to catch it)
CASES = {
    1: ("field term sign flipped in dH",
        ("return ((st->eps[j] - st->eps[i]) - vij) - st->p.E * dx;",
         "return ((st->eps[j] - st->eps[i]) - vij) + st->p.E * dx;"),
        [_dh_field]),
    2: ("-1/r_ij dropped from dH",
        ("return ((st->eps[j] - st->eps[i]) - vij) - st->p.E * dx;",
         "return (st->eps[j] - st->eps[i]) - st->p.E * dx;"),
        [_dh_field, pins.check_boltzmann_exact_3x3]),
    3: ("hop sites skipped by the energy update",
        ("      st->eps[l] = st->eps[l] + (a - b);",
         "      if (l != i && l != j) st->eps[l] = st->eps[l] + (a - b);"),
        [_incremental]),
    4: ("occupancy filter ignores n_j",
        ("    if (!(st->n[i] == 1 && st->n[j] == 0)) continue;\n    st->theta_pass++;",
         "    if (!(st->n[i] == 1)) continue;\n    st->theta_pass++;"),
        [_invariants]),
    5: ("orbit member always the first",
        ("  uint32_t member = w[3] & (uint32_t)(st->orb_size[o] - 1);",
         "  uint32_t member = 0u;"),
        [_draws, pins.check_boltzmann_exact_3x3]),
    6: ("tunnelling weight exp(-r/xi)",
        ("    double w = (double)nu * exp(-2.0 * r / xi);",
         "    double w = (double)nu * exp(-1.0 * r / xi);"),
        [_gamma, _draws]),
    7: ("background nu dropped from eps",
        ("      double q = (double)st->n[m] - st->nu;",
         "      double q = (double)st->n[m];"),
        [pins.check_eps_closed_form_3x3]),
    8: ("Metropolis uses exp(-dH*T)",
        ("  return exp(-dH / st->p.T);",
         "  return exp(-dH * st->p.T);"),
        [pins.check_boltzmann_exact_3x3]),
    9: ("dipole sign flipped",
        ("    st->P += st->vec_dx[v];",
         "    st->P -= st->vec_dx[v];"),
        [_invariants]),
    10: ("energy update sign flipped",
         ("      st->eps[l] = st->eps[l] + (a - b);",
          "      st->eps[l] = st->eps[l] + (b - a);"),
         [_incremental]),
    11: ("pair interaction term with the wrong sign",
         ("  double hi = ((vsite(st, i, k) + vsite(st, j, l)) - vsite(st, i, l)) - vsite(st, j, k);",
          "  double hi = ((vsite(st, i, l) + vsite(st, j, k)) - vsite(st, i, k)) - vsite(st, j, l);"),
         [_pair_dh, _pair_exact_filter]),
    12: ("pair final-separation filter dropped",
         ("&& j != l && near;", "&& j != l;"),
         [_pair_exact_filter]),
    13: ("second electron of a pair not applied to the energies",
         ("      update_eps(st, k, l);\n", ""),
         [_pair_invariants]),
    14: ("pair dipole counts the first electron only",
         ("      st->P += st->vec_dx[v] + st->vec_dx[v2];", "      st->P += st->vec_dx[v];"),
         [_pair_invariants]),
    15: ("partner offset drawn from the tunnelling tower",
         ("  while (!((uint64_t)w[1] < st->thr_u[o])) ++o;", "  while (!((uint64_t)w[1] < st->thr[o])) ++o;"),
         [_pair_draws, _pair_exact_filter]),
}


def _planted(case: int) -> str:
    _, (old, new), _ = CASES[case]
    src = oracle.source()
    assert src.count(old) == 1, f"case {case}: the text it replaces occurs {src.count(old)} times in oracle.c"
    return src.replace(old, new)


@pytest.mark.parametrize("case", sorted(CASES))
def test_planted_mistake_is_caught(case):
    what, _, checks = CASES[case]
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build_copy(_planted(case), d)
        with oracle.using_build(path):
            results = []
            for chk in checks:
                try:
                    ok, msg = chk()
                except Exception as e:  # a crash of the check also counts as detection
                    ok, msg = False, f"raised {type(e).__name__}: {e}"
                results.append((chk.__name__, ok, msg))
    assert any(not ok for _, ok, _ in results), f"case {case} ({what}) not caught: {results}"


def test_unmodified_copy_passes_the_same_checks():
    """The copy mechanism itself plants nothing: an unmodified copy passes every check."""
    with tempfile.TemporaryDirectory() as d:
        path = oracle.build_copy(oracle.source(), d)
        with oracle.using_build(path):
            for _, _, checks in CASES.values():
                for chk in checks:
                    ok, msg = chk()
                    assert ok, (chk.__name__, msg)
