"""Parity of time averaging, point location and probes (section 3, eq. 29)
between the HIP library and the CPU oracle.

Bar: steps averaged, pooled counts and summed histograms exact (they follow
the bit-exact trajectories); pooled means and central second moments within
1e-5, scale-aware as for the per-step records; point location exact (the
same orientation predicate); probe rows as computed from the oracle's average.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads import probes

from test_gpu_parity import TOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1003_4548_amd as P
    P.load_library()
    return P


def _label(wl, extra=""):
    print(f"[case] average {wl.name} n={wl.n_total} ens={wl.nens} {wl.precision} {extra}", flush=True)


def assert_average_parity(ag, ao, hist, omega, what=""):
    np.testing.assert_array_equal(ag[:, O.AV_STEPS], ao[:, O.AV_STEPS], err_msg=what)
    np.testing.assert_array_equal(ag[:, O.AV_N], ao[:, O.AV_N], err_msg=what)
    m2 = ao[:, O.AV_M2:O.AV_M2 + 10]
    sig = np.sqrt(np.maximum(m2[:, [0, 4, 7, 9]], 0.0))
    lim = TOL * np.maximum(np.abs(ao[:, O.AV_MEAN:O.AV_MEAN + 4]), np.maximum(sig, 1e-30))
    err = np.abs(ag[:, O.AV_MEAN:O.AV_MEAN + 4] - ao[:, O.AV_MEAN:O.AV_MEAN + 4])
    assert (err <= lim).all(), f"{what}: pooled means, worst {np.max(err / lim)}"
    pairs = [(a, b) for a in range(4) for b in range(a, 4)]
    sc = np.stack([sig[:, a] * sig[:, b] for a, b in pairs], axis=1)
    lim2 = TOL * np.maximum(np.abs(m2), np.maximum(sc, 1e-30))
    err2 = np.abs(ag[:, O.AV_M2:O.AV_M2 + 10] - m2)
    assert (err2 <= lim2).all(), f"{what}: pooled moments, worst {np.max(err2 / lim2)}"
    if hist:
        np.testing.assert_array_equal(ag[:, O.AV_HIST:O.AV_HIST + hist], ao[:, O.AV_HIST:O.AV_HIST + hist],
                                      err_msg=what)
    if omega:
        sw = np.sqrt(np.maximum(ao[:, -1], 0.0))
        assert (np.abs(ag[:, -2] - ao[:, -2]) <= TOL * np.maximum(np.abs(ao[:, -2]), sw) + 1e-300).all(), what
        assert (np.abs(ag[:, -1] - ao[:, -1]) <= TOL * np.maximum(ao[:, -1], 1e-3 * ao[:, -2] ** 2) + 1e-300).all(), what


CASES = {
    "glm_f32": lambda: W.tiny_canyon(precision="f32", steps=0),
    "wallfn_m4_hist_omega": lambda: W.small_canyon(target=600, ppe=30, wallfn=True, moments=4, hist_bins=32,
                                                   steps=0, omega=True),
    "three_ensembles": lambda: W.tiny_canyon(precision="f32", nens=3, steps=0),
    "glm_f64": lambda: W.tiny_canyon(precision="f64", steps=0),
}


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("case", list(CASES))
def test_time_average_parity(gpu, case, graph):
    wl = CASES[case]()
    _label(wl, f"graph={graph}")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    run = sim.step_graph if graph else sim.step
    run(5)                      # before averaging
    orc.step(5)
    sim.average_attach()
    orc.average_start()
    run(13)
    orc.step(13)
    sim.sync()
    ag = sim.average()
    for en in range(wl.nens):
        assert_average_parity(ag[en], orc.average(en), wl.hist_bins, wl.omega, what=f"{case} ens {en}")
    assert (ag[:, :, O.AV_STEPS] == 13).all()


def test_detach_and_restart(gpu):
    wl = CASES["glm_f32"]()
    _label(wl, "detach/restart")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    sim.average_attach()
    orc.average_start()
    sim.step_graph(7)
    orc.step(7)
    sim.average_detach()
    orc.average_stop()
    sim.step_graph(6)
    orc.step(6)
    sim.sync()
    a1 = sim.average()
    assert (a1[0, :, O.AV_STEPS] == 7).all()
    assert_average_parity(a1[0], orc.average(), 0, False, what="after detach")
    sim.average_attach()          # restarts from zero
    orc.average_start()
    sim.step(4)
    orc.step(4)
    sim.sync()
    assert_average_parity(sim.average()[0], orc.average(), 0, False, what="restart")


@pytest.mark.parametrize("wallfn", [False, True])
def test_locate_parity(gpu, wallfn):
    wl = W.small_canyon(target=600, ppe=2, wallfn=wallfn, steps=0)
    _label(wl, "locate")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(9)
    pts = np.column_stack([rng.uniform(-0.1, 2.1, 500), rng.uniform(-0.1, 2.1, 500)])
    geo = wl.mesh.geometry
    pts = np.concatenate([pts, np.array(probes.table1_points(geo) + probes.cdf_points(geo)),
                          wl.mesh.vtx[:200]])          # vertices: on several elements at once
    got = sim.locate(pts)
    want = np.array([orc.locate(x, y) for x, y in pts])
    np.testing.assert_array_equal(got, want)
    assert (got[500:] >= 0).all()


def test_probes_and_cdf(gpu):
    wl = W.small_canyon(target=600, ppe=40, wallfn=True, moments=4, hist_bins=32, steps=0)
    wl.psi_init = W.PSI_LEFT_QUARTER      # scalar already at some sampling locations
    _label(wl, "probes")
    sim = gpu.Simulation.from_workload(wl)
    orc = O.Oracle(wl)
    sim.step_graph(12)
    orc.step(12)
    sim.average_attach()
    orc.average_start()
    sim.step_graph(24)
    orc.step(24)
    geo = wl.mesh.geometry
    pts = probes.table1_points(geo) + probes.cdf_points(geo)
    el = sim.locate(pts)
    rows = sim.probe(np.concatenate([el, [-1, wl.mesh.nelem]]))
    ao = orc.average()
    for i, e in enumerate(el):
        a = ao[e]
        assert rows[i, 0] == 24 and rows[i, 1] == a[O.AV_N] / 24
        np.testing.assert_allclose(rows[i, 2], a[O.AV_MEAN + 3], rtol=TOL, atol=TOL * np.sqrt(a[O.AV_M2 + 9]) + 1e-300)
        np.testing.assert_allclose(rows[i, 3], a[O.AV_M2 + 9], rtol=TOL, atol=1e-300)
        cdf = np.cumsum(a[O.AV_HIST:O.AV_HIST + 32]) / a[O.AV_N] if a[O.AV_N] > 0 else np.zeros(32)
        np.testing.assert_array_equal(rows[i, 4:], cdf)
        assert (np.diff(rows[i, 4:]) >= 0).all() and (a[O.AV_N] == 0 or rows[i, -1] == 1.0)
    assert np.isnan(rows[-2:]).all()
    # some locations see scalar, with a CDF strictly between 0 and 1 somewhere
    assert (rows[:len(el), 2] > 0).any()
    assert ((rows[:len(el), 4:-1] > 0) & (rows[:len(el), 4:-1] < 1)).any()
