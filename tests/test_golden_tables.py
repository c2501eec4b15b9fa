"""The values the paper prints in its two tables (fixtures under
tests/golden/, each with its citation) against every copy the code keeps:
Table 2's model constants in the relaxation oracle, the workloads' model
constants and the library's relaxation kernels; Table 1's sampling locations
in the probe module (point 10 by its documented reading)."""
import os
import re

import pytest

import oracle.relax as R
import workloads as W
from workloads import probes

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = os.path.join(ROOT, "tests", "golden")


def _read(name):
    rows = []
    for line in open(os.path.join(GOLD, name)):
        line = line.strip()
        if line and not line.startswith("#"):
            rows.append(line.split())
    return rows


@pytest.fixture(scope="module")
def table2():
    return {k: float(v) for k, v in _read("table2_constants.txt")}


def test_table2_in_the_relaxation_oracle(table2):
    for name, val in (("C1", R.C1), ("C2", R.C2), ("CT", R.CT), ("CL", R.CL), ("Ceta", R.CETA), ("Cv", R.CV),
                      ("gamma5", R.GAMMA5)):
        assert val == table2[name], name


def test_table2_in_the_workload_constants(table2):
    c = W.small_canyon(target=300, ppe=1, steps=1).constants
    for name, key in (("CT", "CT"), ("Cs", "Cs"), ("Ct", "Ct"), ("C3", "C3"), ("C4", "C4"), ("Comega1", "Cw1"),
                      ("Comega2", "Cw2")):
        assert c[key] == table2[name], name


def test_table2_in_the_relaxation_kernels(table2):
    src = open(os.path.join(ROOT, "paper_1003_4548_amd", "csrc", "pdf_relax.hpp")).read()
    m = re.search(r"constexpr double C1 = ([\d.]+), C2 = ([\d.]+), CT = ([\d.]+), CL = ([\d.]+), CETA = ([\d.]+), "
                  r"CV = ([\d.]+), GAMMA5 = ([\d.]+);", src)
    assert m, "the Table 2 line of pdf_relax.hpp"
    for name, val in zip(("C1", "C2", "CT", "CL", "Ceta", "Cv", "gamma5"), m.groups()):
        assert float(val) == table2[name], name


def test_table1_in_the_probe_module():
    rows = _read("table1_locations.txt")
    assert [int(r[0]) for r in rows] == list(range(1, 25))
    printed = [(float(r[1]), float(r[2])) for r in rows]
    assert len(probes.TABLE1) == 24
    for i, ((x, y), (px, py)) in enumerate(zip(printed, probes.TABLE1), start=1):
        if i == 10:
            assert (x, y) == (2.5, 0.5) and (px, py) == (2.0, 0.5)
        else:
            assert (px, py) == (x, y), i
