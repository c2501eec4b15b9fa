"""Pins of the oracle's stochastic turbulent frequency (eqs. 8-10, 27-28).

* The series exponential of the wall condition against numpy's exp.
* Frozen <omega> per element solves eq. (8) at the centroid (residual), and
  the estimated dissipation of a state built to carry the frozen stresses and
  <omega> returns the frozen eps (eq. 8 read the other way).
* S_omega (eq. 10) for simple shear, its transpose and plane strain, where
  the production reduces to the textbook forms.
* Eq. (9) under homogeneous fields, with <omega> = M the frozen value that
  also drives the velocity model: one Euler-Maruyama step from omega = M
  has mean M(1 - S_omega M dt) and variance 2 C3 C4 M^3 dt; from a sample
  of mean m and variance V the next has mean m - C3 M (m - M) dt -
  S_omega M m dt and variance (1 - (C3 + S_omega) M dt)^2 V +
  2 C3 C4 M^2 m dt; with S_omega = 0 the stationary law is the gamma
  distribution of the model (mean M, variance 2 C4 M^2 / (2 - C3 M dt)
  discretely, skewness 2 sqrt(C4)).
* Wall condition (eqs. 27-28): log(omega_R / omega_I) is linear in the
  incident wall-normal velocity with slope beta / (y_p <omega>_p), beta from
  Table 2 with C0 = 3.5; resolved walls and periodic seams leave omega alone.
"""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads.fields import F, NFIELD, uniform_fields
from workloads.mesh import EDGE

from test_oracle_physics import _wallfn_strip

C3, C4, CW1, CW2, CT = 5.0, 0.25, 0.5, 0.73, 6.0   # Table 2


def _ulp_diff(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ia = a.view(np.int64)
    ib = b.view(np.int64)
    return np.abs(ia - ib)


def test_exp_series_within_two_ulp():
    rng = np.random.default_rng(3)
    xs = np.concatenate([rng.uniform(-700, 700, 4000), rng.uniform(-1, 1, 4000),
                         rng.uniform(-1e-6, 1e-6, 200), [0.0, 1.0, -1.0, math.log(2), 0.5 * math.log(2)]])
    xs = np.concatenate([xs, np.arange(-20, 21) * math.log(2)])
    got = np.array([O.exp64(float(x)) for x in xs])
    assert _ulp_diff(got, np.exp(xs)).max() <= 2
    assert O.exp64(0.0) == 1.0


def _omega_box(fields=None, ppe=5000, dt=0.05, n=2, constants=None, seed=3):
    wl = W.configs.square_box(n=n, ppe=ppe, precision="f64", dt=dt, seed=seed, fields=fields)
    wl.omega = True
    wl.flags = 1                 # velocity and frequency only: particles keep their element
    if constants:
        wl.constants = dict(wl.constants, **constants)
    return wl


def test_frozen_mean_frequency_solves_eq8():
    wl = W.small_canyon(target=600, ppe=2, wallfn=True, precision="f64")
    wl.omega = True
    orc = O.Oracle(wl, ensembles=[])
    om0, sw, omw = orc.omega_fields()
    m, f = wl.mesh, wl.fields
    cen = f[m.tri].mean(axis=1)
    k = 0.5 * (cen[:, F["R11"]] + cen[:, F["R22"]] + cen[:, F["R33"]])
    eps = cen[:, F["eps"]]
    assert (om0 > 0).all()
    np.testing.assert_allclose(om0 * (k + wl.nu * CT * CT * om0), eps, rtol=1e-12)
    # wall-function edges: the fields at the edge midpoint
    e, q = np.nonzero(m.ekind == EDGE.WALLFN)
    assert len(e) > 10
    mid = 0.5 * (f[m.tri[e, q]] + f[m.tri[e, (q + 1) % 3]])
    kp = 0.5 * (mid[:, F["R11"]] + mid[:, F["R22"]] + mid[:, F["R33"]])
    w = omw[e, q]
    np.testing.assert_allclose(w * (kp + wl.nu * CT * CT * w), mid[:, F["eps"]], rtol=1e-12)
    rest = np.ones_like(omw, bool)
    rest[e, q] = False
    assert (omw[rest] == 0).all()


def test_estimated_dissipation_returns_frozen_eps():
    # two particles per element at U +- sqrt(R_ii) (population variance R_ii),
    # omega equal to the frozen <omega>: eq. (8) must give back eps
    wl = W.small_canyon(target=600, ppe=2, wallfn=True, precision="f64")
    wl.omega = True
    m, f = wl.mesh, wl.fields
    counts = np.full(m.nelem, 2, np.int64)
    wl.ensembles = [W.configs.Ensemble(counts=counts, seed=1)]
    orc = O.Oracle(wl)
    om0, _, _ = orc.omega_fields()
    st = orc.state()
    cen = f[m.tri].mean(axis=1)
    el = st["elem"]
    sgn = np.where(np.arange(len(el)) % 2 == 0, 1.0, -1.0)
    st["u"] = cen[el, F["U"]] + sgn * np.sqrt(cen[el, F["R11"]])
    st["v"] = cen[el, F["V"]] + sgn * np.sqrt(cen[el, F["R22"]])
    st["w"] = sgn * np.sqrt(cen[el, F["R33"]])
    orc.set_state(st)
    orc.set_omega(om0[el])
    s = orc.stats()
    assert s.shape[1] == orc.nstat
    np.testing.assert_allclose(s[:, -3], om0, rtol=1e-14)
    assert np.abs(s[:, -2]).max() < 1e-12 * om0.max() ** 2
    np.testing.assert_allclose(s[:, -1], cen[:, F["eps"]], rtol=1e-12)


@pytest.mark.parametrize("case", ["shear", "transpose", "strain"])
def test_somega_production_special_cases(case):
    g, uv, r11, r22 = 0.7, -0.03, 0.05, 0.02
    eps = 0.4

    def fields(mesh):
        f = uniform_fields(mesh.nvert, U=(0.0, 0.0), k=0.1, eps=eps)
        f[:, F["R11"]], f[:, F["R22"]], f[:, F["R12"]] = r11, r22, uv
        if case == "shear":
            f[:, F["dUdy"]] = g
        elif case == "transpose":
            f[:, F["dVdx"]] = g
        else:
            f[:, F["dUdx"]], f[:, F["dVdy"]] = g, -g
        return f

    wl = _omega_box(fields=fields, ppe=1)
    orc = O.Oracle(wl, ensembles=[])
    _, sw, _ = orc.omega_fields()
    prod = {"shear": -uv * g, "transpose": -uv * g, "strain": -(r11 - r22) * g}[case]
    np.testing.assert_allclose(sw, CW2 - CW1 * prod / eps, rtol=1e-13)


@pytest.mark.parametrize("eps", [1.0, 2.5])
def test_one_step_mean_and_variance_from_deterministic_state(eps):
    # k = 1, nu = 0: the frozen <omega> is eps / k
    wl = _omega_box(dt=0.05 / eps, fields=lambda mesh: uniform_fields(mesh.nvert, k=1.0, eps=eps))
    orc = O.Oracle(wl)
    om0, sw, _ = orc.omega_fields()
    m, s_om, dt = om0[0], sw[0], wl.dt
    assert m == pytest.approx(eps, rel=1e-14) and s_om == pytest.approx(CW2, rel=1e-14)
    w0 = orc.omega()
    np.testing.assert_array_equal(w0, m)
    orc.step(1)
    w = orc.omega()
    n = len(w)
    var1 = 2 * C3 * C4 * m ** 3 * dt
    mean1 = m * (1 - s_om * m * dt)
    assert abs(w.mean() - mean1) < 5 * math.sqrt(var1 / n)
    assert abs(w.var() - var1) < 5 * var1 * math.sqrt(2.0 / n)
    # the S_omega term is resolved: dropping it would be a 10 sigma miss
    assert abs(w.mean() - m) > 10 * math.sqrt(var1 / n)


def test_variance_recursion_per_element():
    wl = _omega_box(dt=0.05, ppe=5000)
    orc = O.Oracle(wl)
    om0, sw, _ = orc.omega_fields()
    dt = wl.dt
    orc.step(1)
    el = orc.state()["elem"]
    w1 = orc.omega()
    orc.step(1)
    w2 = orc.omega()
    rel = []
    for e in range(wl.mesh.nelem):
        a, b = w1[el == e], w2[el == e]
        m, v, M = a.mean(), a.var(), om0[e]
        pred_v = (1 - (C3 + sw[e]) * M * dt) ** 2 * v + 2 * C3 * C4 * M * M * m * dt
        pred_m = m - C3 * M * (m - M) * dt - sw[e] * M * m * dt
        rel.append(b.var() / pred_v - 1)
        assert abs(b.mean() - pred_m) < 5 * math.sqrt(2 * C3 * C4 * M * M * m * dt / len(b))
    rel = np.array(rel)
    # per-element sampling error ~ sqrt(2 / 5000) = 2 %
    assert abs(rel.mean()) < 0.03 and np.abs(rel).max() < 0.1
    # the statistics record carries the same mean and variance
    s = orc.stats()
    for e in range(wl.mesh.nelem):
        b = w2[el == e]
        assert s[e, -3] == pytest.approx(b.mean(), rel=1e-13)
        assert s[e, -2] == pytest.approx(b.var(), rel=1e-11)


def test_stationary_gamma_without_source():
    wl = _omega_box(dt=0.02, ppe=5000, constants=dict(Cw2=0.0))
    orc = O.Oracle(wl)
    om0, sw, _ = orc.omega_fields()
    np.testing.assert_array_equal(sw, 0.0)       # no production, no C_w2
    dt = wl.dt
    orc.step(200)                                # 20 relaxation times 1 / (C3 <omega>)
    el = orc.state()["elem"]
    w = orc.omega()
    ratios, z = [], []
    for e in range(wl.mesh.nelem):
        a = w[el == e]
        M = om0[e]
        ratios.append(a.var() / (2 * C4 * M * M / (2 - C3 * M * dt)))
        z.append((a - a.mean()) / a.std())
    ratios = np.array(ratios)
    z = np.concatenate(z)
    assert abs(ratios.mean() - 1) < 0.04
    # without a source the mean is M = 1, within a few standard errors
    assert abs(w.mean() - 1.0) < 0.02
    assert abs((z ** 3).mean() - 2 * math.sqrt(C4)) < 0.12
    assert w.min() > 0


def _street_hits(orc, m, yp, vel, om_in):
    rng = np.random.default_rng(5)
    out = []
    for _ in range(4000):
        e = int(rng.integers(m.nelem))
        s = m.vtx[m.tri[e]].mean(axis=0)
        if not (0.7 < s[0] < 1.3 and s[1] < yp + 0.05):
            continue
        t = np.array([s[0] + 0.003, yp - 0.002])
        r, tt, v2, nref, om = orc.walk(e, s, t, vel, om=om_in)
        assert nref == 1 and r >= 0
        out.append(om)
    return np.array(out)


def test_wall_function_frequency_condition():
    nu, yp = 1.0 / 12000.0, 13.0 / 256.0
    uhat = 0.05
    k_p = uhat ** 2 / math.sqrt(0.09)
    Ue = uhat / 0.41 * math.log(8.5 * yp * uhat / nu)
    wl = _wallfn_strip(U_p=Ue, v2_p=uhat ** 2, k_p=k_p, yp=yp, nu=nu)
    wl.omega = True
    orc = O.Oracle(wl, ensembles=[])
    m = wl.mesh
    _, _, omw = orc.omega_fields()
    w_p = omw[m.ekind == EDGE.WALLFN]
    np.testing.assert_allclose(w_p, w_p[0], rtol=1e-14)       # uniform fields
    w_p = w_p[0]
    # beta of eq. (28) with C0 = 3.5 and Table 2: -2 / 8.355
    beta = -0.23937761819269898
    slopes = []
    for vn in (-0.05, -0.2, -0.6):
        om = _street_hits(orc, m, yp, np.array([0.3, vn, 0.1]), 2.0)
        assert len(om) > 0
        lr = np.log(om / 2.0)
        np.testing.assert_allclose(lr, lr[0], rtol=0, atol=0)
        assert lr[0] > 0                         # the incident particle moves toward the wall
        slopes.append(lr[0] / vn)
    np.testing.assert_allclose(slopes, beta / (yp * w_p), rtol=1e-14)
    # the tangential and spanwise components do not enter
    a = _street_hits(orc, m, yp, np.array([0.3, -0.2, 0.1]), 2.0)
    b = _street_hits(orc, m, yp, np.array([-1.1, -0.2, 0.7]), 2.0)
    np.testing.assert_array_equal(a, b)
    # a grazing particle (V_I = 0) keeps its frequency
    c = _street_hits(orc, m, yp, np.array([0.3, 0.0, 0.1]), 2.0)
    np.testing.assert_array_equal(c, 2.0)


def test_resolved_walls_and_periodic_seams_keep_frequency():
    wl = W.tiny_canyon(precision="f64")
    wl.omega = True
    m = wl.mesh
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(16)
    for _ in range(1500):
        e = int(rng.integers(m.nelem))
        s = m.vtx[m.tri[e]].mean(axis=0)
        t = s + rng.normal(scale=0.2, size=2)
        r, tt, v2, nref, om = orc.walk(e, s, t, rng.normal(size=3), om=1.7)
        assert r >= 0
        assert om == 1.7


def test_omega_stays_bounded_over_1000_steps_on_the_large_wall_function_canyon():
    """The large wall-function canyon (the 10M-particle workload's mesh and
    fields, here at 5 particles per element) keeps every particle's omega
    finite and within a bounded factor of the frozen <omega> over 1000 steps.
    The wall condition (eqs. 27-28) multiplies omega by exp(beta V_I /
    (y_p <omega>)) per hit; the fields are built so that the statistics at
    y_p are those of a log layer (|alpha| <= 2 on every wall edge), without
    which alpha up to 17 pumped tangential speed that a corner turned into
    wall-normal speed, and single hits grew omega by e^5 - e^10."""
    wl = W.config3w(steps=1000, n=5 * 48618)
    orc = O.Oracle(wl)
    al = orc.wall_alpha()
    assert np.abs(al).max() <= 2.0 + 1e-9
    om0, _, _ = orc.omega_fields()
    worst = 0.0
    for _ in range(10):
        orc.step(100)
        om = orc.omega()
        e = orc.state()["elem"]
        assert np.isfinite(om).all() and (om >= 0).all()
        worst = max(worst, float((om / om0[e]).max()))
    assert worst < 1e3, worst
    assert orc.wallfn_hits() > 10000
