"""Parity of the elliptic-relaxation solve (section 2.1, eqs. 12-18) on the
GPU against the oracle (oracle/relax.py: the same Galerkin system solved by a
sparse direct factorisation, G and C0 from eqs. 12-13).

Both sides start from the same particles: the GPU state and the oracle's are
bit-exact (the step parity tests), and each side takes its statistics records
from its own state.  The GPU solves by conjugate gradients to a relative
residual tol = 1e-12, so its solution is compared by
* the residual of the GPU solution in the oracle's system,
  ||b - A x_gpu|| <= 10 tol ||b|| (plus rounding of the products), and
* the error against the direct solution, ||x_gpu - x|| <= 10 kappa(A) tol ||x||
  (kappa from the extreme eigenvalues of the oracle's matrix);
then G and C0 eps per vertex, within the error that bound allows after the
division by 2k (k from the same records on both sides), and the number of
vertices whose C0 was clamped at zero.  Cases: the 2k-element canyon at 40
and at 8 particles per element (elements under 10 particles take the frozen
stresses), the float and the double state, the doubly periodic box (seams in
both directions, four copies of the corner vertex), and the 1M-particle,
10k-element canyon the benchmark times.  Then the step after a relaxation
uses the new table: one step of the GPU against the oracle stepping with its
own relaxed table (the tables agree to the bound above, not bit for bit, so
the comparison is to 1e-5), far from the oracle stepping with the frozen
table.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
import oracle.relax as R
import workloads as W

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    P.load_library()
    return P


def _cases():
    return {
        "canyon_40ppe_f32": lambda: W.small_canyon(target=2000, ppe=40, steps=5),
        "canyon_8ppe_f32": lambda: W.small_canyon(target=2000, ppe=8, steps=5),
        "canyon_40ppe_f64": lambda: W.small_canyon(target=2000, ppe=40, steps=5, precision="f64"),
        "periodic_box_f32": lambda: W.square_box(n=12, ppe=30, periodic_y=True, precision="f32", model=W.GLM,
                                                 dt=1e-3, steps=5),
        "canyon_1M_f32": lambda: W.config2(steps=3),
    }


def _extreme_condition(A):
    lmax = spla.eigsh(A, k=1, which="LA", return_eigenvectors=False)[0]
    lmin = spla.eigsh(A, k=1, sigma=0.0, which="LM", return_eigenvectors=False)[0]
    return lmax / lmin


def _oracle_side(wl, steps):
    orc = O.Oracle(wl)
    orc.step(steps)
    stats = orc.stats()
    wp, parts = R.solve(wl.mesh, wl.fields, stats, wl.nu)
    coef, neg = R.vertex_coefficients(wl.mesh, wl.fields, wp, parts)
    return orc, stats, wp, parts, coef, neg


def _check_solution(res, wl, stats, wp, parts, coef, neg, what):
    canon, nc = parts["canon"], parts["nc"]
    A = (parts["M"] + parts["K"]).tocsr()
    # the load vector of the oracle's system
    area = parts["area"]
    S = np.stack([parts["S"][:, i, j] for i, j in R.COMPONENTS], axis=1)
    b = np.zeros((nc, 5))
    for a in range(3):
        np.add.at(b, canon[wl.mesh.tri[:, a]], S * (area / 3.0)[:, None])
    # the GPU solution at the unknowns (every copy of a seam vertex holds it)
    xg = np.zeros((nc, 5))
    xg[canon] = res["wp"]
    for c in range(5):
        np.testing.assert_array_equal(res["wp"][:, c], xg[canon, c], err_msg=f"{what}: seam copies differ")
    kappa = _extreme_condition(A)
    print(f"[relax] {what}: unknowns {nc}, nonzeros {A.nnz}, kappa {kappa:.3g}, iterations {res['iterations']}, "
          f"resid {res['resid'].max():.2e}, clamped {res['clamped']} (oracle {neg}), "
          f"from statistics {res['from_stats']}", flush=True)
    assert res["converged"]
    assert (res["resid"] <= TOL).all(), res["resid"]
    assert res["from_stats"] == int((stats[:, O.ST_N] >= R.N_MIN).sum())
    rounding = 1e-14 * (abs(A).sum(axis=1).A.ravel().max()) * np.abs(wp).max(axis=0)
    err_bound = np.zeros(5)
    for c in range(5):
        r = b[:, c] - A @ xg[:, c]
        bn = np.linalg.norm(b[:, c])
        assert np.linalg.norm(r) <= 10 * TOL * bn + np.sqrt(nc) * rounding[c], (what, c)
        err = np.linalg.norm(xg[:, c] - wp[:, c])
        err_bound[c] = 10 * kappa * TOL * np.linalg.norm(wp[:, c])
        assert err <= err_bound[c], (what, c, err, err_bound[c])
    # G = (2 wp - eps) / 2k and C0 eps = -2 wp:R / 3k per vertex, with R and k
    # area-weighted over the elements around the vertex: a pointwise error of
    # wp under err_bound moves G by err_bound / k and C0 eps by
    # 2 sum |R| err_bound / 3k (plus rounding of the division)
    wsum = np.zeros(nc)
    Rs = np.zeros((nc, 3, 3))
    for a in range(3):
        np.add.at(wsum, canon[wl.mesh.tri[:, a]], area)
        np.add.at(Rs, canon[wl.mesh.tri[:, a]], area[:, None, None] * parts["R"])
    Rv = (Rs / wsum[:, None, None])[canon]
    kv = 0.5 * np.trace(Rv, axis1=1, axis2=2)
    atol_G = err_bound[None, :] / kv[:, None] + 1e-14 * np.abs(coef[:, :5])
    dG = np.abs(res["coef"][:, :5] - coef[:, :5])
    assert (dG <= atol_G).all(), (what, "G", float((dG / atol_G).max()))
    Rabs = np.stack([np.abs(Rv[:, i, j]) for i, j in R.COMPONENTS], axis=1)
    atol_C = 2.0 * (Rabs * err_bound[None, :]).sum(axis=1) / (3.0 * kv) + 1e-14 * np.abs(coef[:, 5])
    dC = np.abs(res["coef"][:, 5] - coef[:, 5])
    assert (dC <= atol_C).all(), (what, "C0 eps", float((dC / atol_C).max()))
    assert abs(res["clamped"] - neg) <= max(1, neg // 1000)


@pytest.mark.parametrize("case", list(_cases()))
def test_relaxation_matches_the_oracle(gpu, case):
    wl = _cases()[case]()
    steps = wl.steps
    print(f"[case] relaxation {case}: {wl.name} n={wl.n_total} elements={wl.mesh.nelem} steps={steps}", flush=True)
    sim = gpu.Simulation.from_workload(wl)
    sim.step(steps)
    sim.sync()
    res = sim.elliptic_relaxation(max_iters=20000, tol=TOL)
    sim.close()
    orc, stats, wp, parts, coef, neg = _oracle_side(wl, steps)
    del orc
    _check_solution(res, wl, stats, wp, parts, coef, neg, case)


def test_steps_use_the_relaxed_coefficients(gpu):
    wl = W.small_canyon(target=2000, ppe=40, steps=5)
    print(f"[case] step after relaxation: {wl.name} n={wl.n_total}", flush=True)
    sim = gpu.Simulation.from_workload(wl)
    sim.step(wl.steps)
    res = sim.elliptic_relaxation(max_iters=20000, tol=TOL)
    assert res["converged"]
    sim.step(1)
    sim.sync()
    g = sim.state()
    orc, stats, wp, parts, coef, neg = _oracle_side(wl, wl.steps)
    frozen = O.Oracle(wl)
    frozen.step(wl.steps + 1)
    orc.set_drift(coef)
    orc.step(1)
    o, f = orc.state(), frozen.state()
    scale = max(np.abs(o["u"]).max(), np.abs(o["v"]).max(), np.abs(o["w"]).max())
    d_relaxed = max(np.abs(g[q] - o[q]).max() for q in ("u", "v", "w"))
    d_frozen = max(np.abs(g[q] - f[q]).max() for q in ("u", "v", "w"))
    moved = int((g["elem"] != o["elem"]).sum())
    print(f"[relax] velocity difference after one step: relaxed table {d_relaxed:.2e}, frozen table "
          f"{d_frozen:.2e} (scale {scale:.3g}); elements differing {moved} of {len(g['elem'])}", flush=True)
    assert d_relaxed <= 1e-5 * scale
    assert d_frozen > 1e3 * d_relaxed
    assert moved <= 1e-4 * len(g["elem"]) + 1
    np.testing.assert_allclose(g["x"], o["x"], rtol=0, atol=1e-5)
    np.testing.assert_allclose(g["y"], o["y"], rtol=0, atol=1e-5)


def test_warm_start_and_iteration_limit(gpu):
    wl = W.small_canyon(target=2000, ppe=40, steps=5)
    print(f"[case] warm start and limit: {wl.name}", flush=True)
    sim = gpu.Simulation.from_workload(wl)
    sim.step(wl.steps)
    first = sim.elliptic_relaxation(max_iters=20000, tol=TOL)
    again = sim.elliptic_relaxation(max_iters=20000, tol=TOL)
    print(f"[relax] iterations: first {first['iterations']}, warm {again['iterations']}", flush=True)
    assert first["converged"] and again["converged"]
    assert again["iterations"] < first["iterations"] // 4
    scale = np.abs(first["wp"]).max(axis=0)
    assert (np.abs(again["wp"] - first["wp"]).max(axis=0) <= 1e-6 * scale).all()
    sim.step(2)
    short = sim.elliptic_relaxation(max_iters=1, tol=TOL, outputs=False)
    assert short["iterations"] == 1 and not short["converged"] and short["resid"].max() > TOL
    with pytest.raises(gpu.PdfError):
        sim.elliptic_relaxation(max_iters=0)
    with pytest.raises(gpu.PdfError):
        sim.elliptic_relaxation(tol=0.0)
    sim.close()
    slm = W.small_canyon(target=2000, ppe=10, steps=1, wallfn=True)
    s2 = gpu.Simulation.from_workload(slm)
    with pytest.raises(gpu.PdfError) as ei:
        s2.elliptic_relaxation()
    assert ei.value.code == -8
    s2.close()
