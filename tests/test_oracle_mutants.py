"""Every planted mistake in tests/oracle_mutants.py fails an oracle pin (CPU:
each mutant is a compiled copy of oracle.c, the pins run against it)."""
from oracle_mutants import MUTANTS, run_all


def test_every_planted_mistake_fails_a_pin():
    res = run_all(MUTANTS)
    missed = [(name, detail) for name, caught, detail in res if not caught]
    assert not missed, missed
    assert len(res) == len(MUTANTS) >= 21
