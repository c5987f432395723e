"""Every planted mistake in tests/oracle_mutants.py fails an oracle pin (CPU:
each traversal mutant is a compiled copy of oracle.c, each stroke mutant a
copy of oracle/stroke.py; the pins run against it)."""
from oracle_mutants import MUTANTS, STROKE_MUTANTS, run_all, run_all_stroke


def test_every_planted_traversal_mistake_fails_a_pin():
    res = run_all(MUTANTS)
    missed = [(name, detail) for name, caught, detail in res if not caught]
    assert not missed, missed
    assert len(res) == len(MUTANTS) >= 21


def test_every_planted_stroke_mistake_fails_a_pin():
    res = run_all_stroke(STROKE_MUTANTS)
    missed = [(name, detail) for name, caught, detail in res if not caught]
    assert not missed, missed
    assert len(res) == len(STROKE_MUTANTS) >= 13
