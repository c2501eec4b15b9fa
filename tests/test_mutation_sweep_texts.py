"""The oracle's mutation sweep (oracle/mutation_sweep.py) plants each mistake
by replacing a piece of source text; every such text must still occur
exactly once in the current oracle sources, or the sweep stops at that
mutant.  (The sweep itself builds and tests every mutant and is run by
hand.)"""
import os

import pytest

import oracle.mutation_sweep as MS

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _cases():
    out = []
    for group, path in ((MS.MUTANTS, MS.SRC), (MS.RELAX_MUTANTS, MS.RELAX), (MS.PROJECT_MUTANTS, MS.PROJECT)):
        for name, edits in group:
            for old, new in edits:
                out.append((os.path.basename(path), name, path, old, new))
    return out


@pytest.mark.parametrize("fname,name,path,old,new", _cases(), ids=[f"{c[0]}: {c[1]}" for c in _cases()])
def test_mutated_text_occurs_once(fname, name, path, old, new):
    src = open(path).read()
    assert src.count(old) == 1, f"{name}: {src.count(old)} occurrences in {fname}"
    assert old != new
