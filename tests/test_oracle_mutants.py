"""Each mutation build of the oracle plants one plausible mistake (no
injectivity check, tree edges only, a skipped root vertex, columns in search
order, descending sort, one orientation per edge, a cap off by one, a wrong
hash index, no sort, an induced check that skips the last vertex, a layout
cost without the root's vertex cost, a CSR export that drops its last offset
or shifts its lists).  Every one must be caught by at least one pin, which
shows that the pins constrain the oracle beyond its own code."""
import os

import pytest

import oracle
import pins

MUTANTS = {1: "no injectivity", 2: "tree edges only", 3: "skips last root vertex",
           4: "columns in search order", 5: "descending order", 6: "one orientation per edge",
           7: "cap off by one", 8: "hash index shifted", 9: "unsorted",
           10: "induced check skips the last vertex", 11: "cost skips the root vertex",
           12: "CSR export drops the last offset", 13: "CSR export shifts the lists"}


@pytest.mark.parametrize("mutant", sorted(MUTANTS), ids=lambda m: MUTANTS[m])
def test_mutant_is_caught(mutant, tmp_path):
    path = str(tmp_path / f"liboracle_m{mutant}.so")
    oracle.build(out=path, mutant=mutant)
    lib = oracle.load(path)
    assert lib.oracle_mutant_id() == mutant
    caught = []
    for pin in pins.ALL_PINS:
        try:
            pin(lib)
        except (AssertionError, oracle.OracleError, StopIteration):
            caught.append(pin.__name__)
    assert caught, f"mutant {mutant} ({MUTANTS[mutant]}) passed every pin"
    print(f"mutant {mutant}: caught by {caught}")
