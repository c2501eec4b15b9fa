"""Pins of the oracle's time averaging, point location and probe mapping
(section 3: statistics time-averaged once stationary, the sampling locations
of Table 1, the scalar CDF of eq. 29).

* Averaging one step returns that step's record.
* The time average equals the statistics of the pooled sample -- every
  particle of the element at the start of every averaged step -- computed by
  brute force with numpy (mean, population covariance, histogram), also for
  the turbulent frequency.
* The CDF at the histogram edges equals the pooled fraction below each edge.
* Point location agrees with an independent brute-force search; every
  sampling location lies in the flow of both canyon meshes.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads import probes


def _pooled(states, nelem, hist, omegas=None):
    """Brute-force pooled statistics per element over a list of states."""
    by = [[] for _ in range(nelem)]
    byw = [[] for _ in range(nelem)]
    for i, st in enumerate(states):
        vals = np.stack([st["u"], st["v"], st["w"], st["psi"]], axis=1)
        for e in range(nelem):
            m = st["elem"] == e
            by[e].append(vals[m])
            if omegas is not None:
                byw[e].append(omegas[i][m])
    out = []
    for e in range(nelem):
        v = np.concatenate(by[e]) if by[e] else np.zeros((0, 4))
        rec = {"n": len(v)}
        if len(v):
            rec["mean"] = v.mean(axis=0)
            c = np.cov(v.T, bias=True).reshape(4, 4)
            rec["m2"] = np.array([c[a, b] for a in range(4) for b in range(a, 4)])
            if hist:
                hb = np.clip(np.floor(v[:, 3] * hist), 0, hist - 1).astype(int)
                rec["hist"] = np.bincount(hb, minlength=hist)
                rec["psi"] = v[:, 3]
            if omegas is not None:
                w = np.concatenate(byw[e])
                rec["om"] = (w.mean(), w.var())
        out.append(rec)
    return out


def test_average_of_one_step_is_its_record():
    wl = W.small_canyon(target=600, ppe=30, wallfn=True, moments=4, hist_bins=32, omega=True, precision="f64")
    orc = O.Oracle(wl)
    orc.step(3)
    rec = orc.stats()
    orc.average_start()
    orc.step(1)
    av = orc.average()
    assert (av[:, O.AV_STEPS] == 1).all()
    np.testing.assert_array_equal(av[:, O.AV_N], rec[:, O.ST_N])
    np.testing.assert_allclose(av[:, O.AV_MEAN:O.AV_MEAN + 4], rec[:, O.ST_MEAN:O.ST_MEAN + 4], rtol=1e-15, atol=0)
    np.testing.assert_allclose(av[:, O.AV_M2:O.AV_M2 + 10], rec[:, O.ST_M2:O.ST_M2 + 10], rtol=1e-14, atol=1e-300)
    np.testing.assert_array_equal(av[:, O.AV_HIST:O.AV_HIST + 32], rec[:, O.NSTAT_4:O.NSTAT_4 + 32])
    np.testing.assert_allclose(av[:, -2], rec[:, -3], rtol=1e-15)
    np.testing.assert_allclose(av[:, -1], rec[:, -2], rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("omega", [False, True])
def test_average_is_the_pooled_sample(omega):
    wl = W.small_canyon(target=600, ppe=20, wallfn=True, moments=4, hist_bins=32, omega=omega, precision="f64")
    orc = O.Oracle(wl)
    orc.step(2)
    orc.average_start()
    states, oms = [], []
    for _ in range(6):
        states.append(orc.state())
        if omega:
            oms.append(orc.omega())
        orc.step(1)
    av = orc.average()
    ref = _pooled(states, wl.mesh.nelem, 32, omegas=oms if omega else None)
    nonempty = 0
    for e, r in enumerate(ref):
        a = av[e]
        assert a[O.AV_STEPS] == 6
        assert a[O.AV_N] == r["n"]
        if r["n"] == 0:
            continue
        nonempty += 1
        np.testing.assert_allclose(a[O.AV_MEAN:O.AV_MEAN + 4], r["mean"], rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(a[O.AV_M2:O.AV_M2 + 10], r["m2"], rtol=1e-9, atol=1e-14)
        np.testing.assert_array_equal(a[O.AV_HIST:O.AV_HIST + 32], r["hist"])
        # eq. (29) at the bin edges: the pooled fraction below each edge
        cdf = np.cumsum(a[O.AV_HIST:O.AV_HIST + 32]) / a[O.AV_N]
        edges = np.arange(1, 33) / 32.0
        frac = np.array([(r["psi"] < t).mean() for t in edges[:-1]] + [1.0])
        np.testing.assert_array_equal(cdf, frac)
        if omega:
            np.testing.assert_allclose(a[-2], r["om"][0], rtol=1e-12)
            np.testing.assert_allclose(a[-1], r["om"][1], rtol=1e-9, atol=1e-14)
    assert nonempty > 100


def test_restart_and_stop():
    wl = W.tiny_canyon(precision="f32")
    orc = O.Oracle(wl)
    orc.average_start()
    orc.step(3)
    assert (orc.average()[:, O.AV_STEPS] == 3).all()
    orc.average_stop()
    orc.step(2)
    assert (orc.average()[:, O.AV_STEPS] == 3).all()
    orc.average_start()
    orc.step(1)
    assert (orc.average()[:, O.AV_STEPS] == 1).all()


@pytest.mark.parametrize("wallfn", [False, True])
def test_locate_matches_brute_force(wallfn):
    wl = W.small_canyon(target=600, ppe=2, wallfn=wallfn)
    m = wl.mesh
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(4)
    pts = np.column_stack([rng.uniform(-0.1, 2.1, 600), rng.uniform(-0.1, 2.1, 600)])
    for p in pts:
        assert orc.locate(*p) == m.locate_brute(p)
    # centroids sit in their own element
    cen = m.vtx[m.tri].mean(axis=1)
    for e in range(0, m.nelem, 7):
        assert orc.locate(*cen[e]) == e


@pytest.mark.parametrize("wallfn", [False, True])
def test_sampling_locations_lie_in_the_flow(wallfn):
    wl = W.small_canyon(target=600, ppe=2, wallfn=wallfn)
    geo = wl.mesh.geometry
    orc = O.Oracle(wl, ensembles=[])
    pts = probes.table1_points(geo) + probes.cdf_points(geo)
    assert len(pts) == 26
    el = [orc.locate(x, y) for x, y in pts]
    assert min(el) >= 0
    t1 = probes.table1_points(geo)
    # roof points repeat one building period apart (periodic x)
    assert t1[0] == t1[21] and t1[1] == t1[22] and t1[2] == t1[23]
    # wall points sit on the wall lines of this geometry
    for i in list(range(4, 12)):
        assert t1[i][0] == geo.x_l
    for i in list(range(12, 20)):
        assert t1[i][0] == geo.x_r
    for i in (0, 1, 2, 3, 20, 21, 22, 23):
        assert t1[i][1] == geo.y_roof
