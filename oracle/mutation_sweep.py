"""Mutation sweep of the oracle's pins (CPU only).

Each entry plants one plausible mistake in a copy of ``orc.cpp`` (a dropped
term, a wrong sign, a swapped index, a transposed operand), builds that copy
to a temporary library and runs the pin tests against it through the
ORC_LIB override of ``oracle/__init__.py``; the entries for the Python
oracles of the elliptic-relaxation solve and of the mean-pressure projection
replace ``relax.py`` or ``project.py`` for their run.  A pin set is adequate when every
mutant fails at least one test.  Run: ``python oracle/mutation_sweep.py``
(a few minutes; prints one line per mutant and exits 1 if any survives).
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)
from oracle import CFLAGS, SRC  # noqa: E402

PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_physics.py", "tests/test_oracle_geometry.py"]
RELAX = os.path.join(HERE, "relax.py")
RELAX_PINS = ["tests/test_oracle_relax.py"]
PROJECT = os.path.join(HERE, "project.py")
PROJECT_PINS = ["tests/test_oracle_project.py"]

# (name, [(original text, planted text), ...])
MUTANTS = [
    ("sign of the mean pressure gradient (eq. 6)",
     [("std::fma(nu2, f[C_LAPU], -f[C_DPDX])", "std::fma(nu2, f[C_LAPU], f[C_DPDX])")]),
    ("swapped barycentric weights",
     [("lam[0] = orient_edge(c, e, 1, px, py) * ia;\n  lam[1] = orient_edge(c, e, 2, px, py) * ia;",
       "lam[0] = orient_edge(c, e, 2, px, py) * ia;\n  lam[1] = orient_edge(c, e, 1, px, py) * ia;")]),
    ("nu in place of 2 nu in the viscous drift",
     [("std::fma(nu2, f[C_LAPU], -f[C_DPDX])", "std::fma((T)p.nu, f[C_LAPU], -f[C_DPDX])")]),
    ("transposed velocity gradient in the laminar noise",
     [("T gu = std::fma(f[C_DUDY], dW2, f[C_DUDX] * dW1), gv = std::fma(f[C_DVDY], dW2, f[C_DVDX] * dW1);",
       "T gu = std::fma(f[C_DVDX], dW2, f[C_DUDX] * dW1), gv = std::fma(f[C_DVDY], dW2, f[C_DUDY] * dW1);")]),
    ("position and velocity with independent molecular increments",
     [("T xn = std::fma(s2nu, dW1, std::fma(u, dt, x));", "T xn = std::fma(s2nu, dWp1, std::fma(u, dt, x));")]),
    ("r0 in place of r0^2 in eq. (11)",
     [("newton_cbrt(r0 * r0 / eps)", "newton_cbrt(r0 / eps)")]),
    ("dropped C_t in eq. (11)",
     [("first = first + p.Ct * dist / Uc;", "first = first + dist / Uc;")]),
    ("minimum in place of maximum in the plateau of eq. (11)",
     [("std::max(k / eps, p.CT * std::sqrt(p.nu / eps))", "std::min(k / eps, p.CT * std::sqrt(p.nu / eps))")]),
    ("wrong L21 of the Cholesky factor",
     [("double L21 = R12 / L11;", "double L21 = R12 / std::sqrt(R22);")]),
    ("sign of the gamma_tau test (eq. 26)",
     [("double gamma_tau = prod > 0.0 ? 1.0 : 0.0;", "double gamma_tau = prod < 0.0 ? 1.0 : 0.0;")]),
    ("y_p dP/dx without its absolute value (eq. 25)",
     [("gamma_tau * std::fabs(p.yp * dPdx)", "gamma_tau * (p.yp * dPdx)")]),
    ("<U>_p^2 in place of <U>_p |<U>_p| (eq. 22)",
     [("Up * std::fabs(Up)", "Up * Up")]),
]


# mistakes planted in the Python oracle of the elliptic-relaxation solve
# (relax.py is replaced in place for the run and restored afterwards)
RELAX_MUTANTS = [
    ("sign of the gamma5/3 term of H (eq. 15)",
     [("- GAMMA5 / 3.0 * I[i, ll] * I[j, kk]", "+ GAMMA5 / 3.0 * I[i, ll] * I[j, kk]")]),
    ("sign of the b_ik term of H (eq. 15)",
     [("+ GAMMA5 * b[:, i, kk] * I[j, ll]", "- GAMMA5 * b[:, i, kk] * I[j, ll]")]),
    ("transposed mean velocity gradient in eq. (14)",
     [("acc = acc + H * grad[:, kk, ll]", "acc = acc + H * grad[:, ll, kk]")]),
    ("C_xi = 1.3 in eq. (18)", [("C_XI = 2.3", "C_XI = 1.3")]),
    ("L in place of L^2 in eq. (14)", [("L2=L * L", "L2=L")]),
    ("load with half the element area", [("S[:, c] * area / 3.0", "S[:, c] * area / 2.0")]),
    ("lumped diagonal of the mass matrix", [("(2.0 if a == b else 1.0)", "(1.0 if a == b else 1.0)")]),
    ("periodic seams not joined", [("parent[max(ra, rb)] = min(ra, rb)", "pass")]),
    ("wp in place of 2 wp in eq. (12)", [("G = (2.0 * w - eps * np.eye(3))", "G = (w - eps * np.eye(3))")]),
    ("factor 2 dropped in eq. (13)", [("C0 = -2.0 * np.sum(w * Rv[c])", "C0 = -np.sum(w * Rv[c])")]),
    ("C2 = 0.36 (Table 2)", [("C1, C2, CT, CL, CETA, CV, GAMMA5 = 1.85, 0.63,",
                              "C1, C2, CT, CL, CETA, CV, GAMMA5 = 1.85, 0.36,")]),
]


# the projection's Python oracle (project.py replaced in place for the run)
PROJECT_MUTANTS = [
    ("sign of the load", [("b, canon[mesh.tri[:, a]], area * (U[:, 0]", "b, canon[mesh.tri[:, a]], -area * (U[:, 0]")]),
    ("x and y gradients swapped in the load",
     [("(U[:, 0] * gx[:, a] + U[:, 1] * gy[:, a])", "(U[:, 0] * gy[:, a] + U[:, 1] * gx[:, a])")]),
    ("element area dropped from the load",
     [("b, canon[mesh.tri[:, a]], area * (U[:, 0]", "b, canon[mesh.tri[:, a]], (U[:, 0]")]),
    ("dt dropped from the load", [("U[:, 1] * gy[:, a]) / dt)", "U[:, 1] * gy[:, a]))")]),
    ("y gradient from the x weights", [("(p * gy).sum(axis=1)], axis=1)", "(p * gx).sum(axis=1)], axis=1)")]),
    ("unweighted vertex average",
     [("np.add.at(ws, canon[mesh.tri[:, a]], area)", "np.add.at(ws, canon[mesh.tri[:, a]], 1.0)"),
      ("np.add.at(gs, canon[mesh.tri[:, a]], area[:, None] * ge)", "np.add.at(gs, canon[mesh.tri[:, a]], ge)")]),
    ("sign of the velocity correction", [("- dt * ge[e, q]", "+ dt * ge[e, q]")]),
    ("fallback below eleven particles", [("use = stats[:, ST_N] >= N_MIN", "use = stats[:, ST_N] > N_MIN")]),
    ("frozen V in place of U", [("U = fc[:, F_U:F_U + 2].copy()", "U = fc[:, F_U + 1:F_U + 3].copy()")]),
]


def run_py_one(name, edits, path, pins):
    orig = open(path).read()
    src = orig
    for old, new in edits:
        if src.count(old) != 1:
            raise RuntimeError(f"{name}: the text to mutate occurs {src.count(old)} times")
        src = src.replace(old, new)
    try:
        with open(path, "w") as f:
            f.write(src)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins],
                           cwd=ROOT, capture_output=True, text=True)
    finally:
        with open(path, "w") as f:
            f.write(orig)
    failed = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return r.returncode != 0, failed


def run_one(name, edits, tmp):
    src = open(SRC).read()
    for old, new in edits:
        if src.count(old) != 1:
            raise RuntimeError(f"{name}: the text to mutate occurs {src.count(old)} times")
        src = src.replace(old, new)
    cpp = os.path.join(tmp, "orc_mut.cpp")
    lib = os.path.join(tmp, "liborc_mut.so")
    with open(cpp, "w") as f:
        f.write(src)
    subprocess.run(["g++", *CFLAGS, "-I", HERE, "-o", lib, cpp], check=True)
    env = dict(os.environ, ORC_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True)
    failed = [ln.split(" ")[1] for ln in r.stdout.splitlines() if ln.startswith("FAILED")]
    return r.returncode != 0, failed


def main() -> int:
    survivors = 0
    with tempfile.TemporaryDirectory() as tmp:
        for name, edits in MUTANTS:
            caught, failed = run_one(name, edits, tmp)
            survivors += 0 if caught else 1
            print(f"{'caught  ' if caught else 'SURVIVED'} {name}: {failed[0] if failed else '-'}", flush=True)
    for name, edits in RELAX_MUTANTS:
        caught, failed = run_py_one(name, edits, RELAX, RELAX_PINS)
        survivors += 0 if caught else 1
        print(f"{'caught  ' if caught else 'SURVIVED'} {name}: {failed[0] if failed else '-'}", flush=True)
    for name, edits in PROJECT_MUTANTS:
        caught, failed = run_py_one(name, edits, PROJECT, PROJECT_PINS)
        survivors += 0 if caught else 1
        print(f"{'caught  ' if caught else 'SURVIVED'} {name}: {failed[0] if failed else '-'}", flush=True)
    return 1 if survivors else 0


if __name__ == "__main__":
    sys.exit(main())
