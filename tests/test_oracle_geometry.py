"""Pins of the oracle's particle tracking (closing summary of section 2.2: the grid tracks the
particles) and boundary conditions, against brute force and closed forms."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from workloads.mesh import EDGE


def _domain_contains(mesh, p):
    return mesh.locate_brute(p) >= 0


def _wall_segments(mesh):
    e, k = np.nonzero((mesh.ekind == EDGE.NOSLIP) | (mesh.ekind == EDGE.SLIP) | (mesh.ekind == EDGE.WALLFN))
    a = mesh.vtx[mesh.tri[e, k]]
    b = mesh.vtx[mesh.tri[e, (k + 1) % 3]]
    return a, b


def _segment_inside(mesh, a, b):
    """True when the segment a-b stays in the domain: both ends inside and no
    wall edge touched (closed-segment intersection test)."""
    if not (_domain_contains(mesh, a) and _domain_contains(mesh, b)):
        return False
    p, q = _wall_segments(mesh)
    def o(u, v, w):
        return (v[..., 0] - u[..., 0]) * (w[..., 1] - u[..., 1]) - (v[..., 1] - u[..., 1]) * (w[..., 0] - u[..., 0])
    d1 = o(p, q, a[None]); d2 = o(p, q, b[None])
    d3 = o(a[None], b[None], p); d4 = o(a[None], b[None], q)
    hit = (d1 * d2 <= 0) & (d3 * d4 <= 0)
    return not hit.any()


def _random_point_in(mesh, e, rng):
    v = mesh.vtx[mesh.tri[e]]
    s1, s2 = rng.uniform(), rng.uniform()
    if s1 + s2 > 1:
        s1, s2 = 1 - s1, 1 - s2
    return v[0] + s1 * (v[1] - v[0]) + s2 * (v[2] - v[0])


def _contains(mesh, e, p, tol=1e-12):
    a, b, c = mesh.vtx[mesh.tri[e]]
    def o(u, v):
        return (v[0] - u[0]) * (p[1] - u[1]) - (v[1] - u[1]) * (p[0] - u[0])
    return o(a, b) >= -tol and o(b, c) >= -tol and o(c, a) >= -tol


@pytest.mark.parametrize("wl_fn", [lambda: W.config1(), lambda: W.tiny_canyon(precision="f64")])
def test_walk_matches_brute_force_location(wl_fn):
    wl = wl_fn()
    wl.precision = "f64"
    m = wl.mesh
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(11)
    checked = 0
    for _ in range(3000):
        e = int(rng.integers(m.nelem))
        s = _random_point_in(m, e, rng)
        t = s + rng.normal(scale=0.08, size=2)
        if not _segment_inside(m, s, t):
            continue
        r, tt, vel, nref = orc.walk(e, s, t, [0.1, 0.2, 0.3])
        assert nref == 0
        assert tuple(tt) == (t[0], t[1])
        assert r >= 0 and _contains(m, r, t)
        checked += 1
    assert checked > 1000


def test_periodic_seam_shift_applied_once():
    wl = W.config1()
    m = wl.mesh
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(12)
    for _ in range(500):
        e = int(rng.integers(m.nelem))
        s = _random_point_in(m, e, rng)
        t = s + np.array([rng.uniform(-1.4, 1.4), 0.0])
        t[1] = s[1]
        r, tt, vel, nref = orc.walk(e, s, t, [1.0, 0.0, 0.0])
        expect_x = t[0] % 1.0
        assert abs(tt[0] - expect_x) < 1e-12 or abs(abs(tt[0] - expect_x) - 1.0) < 1e-12
        assert tt[1] == t[1]
        assert r >= 0 and _contains(m, r, tt)
        assert m.locate_brute(np.array(tt)) >= 0
        np.testing.assert_array_equal(vel, [1.0, 0.0, 0.0])


def test_slip_wall_specular_reflection():
    wl = W.config1()
    m = wl.mesh
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(13)
    for _ in range(300):
        e = int(rng.integers(m.nelem))
        s = _random_point_in(m, e, rng)
        dy = -s[1] - rng.uniform(0.001, 0.2)       # crosses y = 0
        t = np.array([s[0] + rng.uniform(-0.05, 0.05), s[1] + dy])
        if not (0.0 < t[0] < 1.0):
            continue
        vel = rng.normal(size=3)
        r, tt, v2, nref = orc.walk(e, s, t, vel)
        assert nref == 1
        assert tt[0] == t[0] and tt[1] == -t[1]        # mirror image about y = 0
        np.testing.assert_array_equal(v2, [vel[0], -vel[1], vel[2]])
        assert np.isclose(np.linalg.norm(v2), np.linalg.norm(vel), rtol=0, atol=0)
        assert r >= 0 and _contains(m, r, tt)
        # reflecting the mirror image again returns the original target (involution)
        r2, tt2, v3, _ = orc.walk(r, np.array(tt), np.array([tt[0], -tt[1]]), v2)
        assert tt2[1] == tt[1]


def test_noslip_wall_reverses_velocity():
    wl = W.tiny_canyon(precision="f64")
    m = wl.mesh
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(14)
    n_ok = 0
    for _ in range(2000):
        e = int(rng.integers(m.nelem))
        s = _random_point_in(m, e, rng)
        if not (0.6 < s[0] < 1.4 and s[1] < 0.1):
            continue
        t = np.array([s[0] + rng.uniform(-0.02, 0.02), -rng.uniform(0.0005, 0.05)])
        vel = rng.normal(size=3)
        r, tt, v2, nref = orc.walk(e, s, t, vel)
        assert nref == 1
        assert tt[1] == -t[1] and tt[0] == t[0]
        np.testing.assert_array_equal(v2, -vel)
        assert r >= 0 and _contains(m, r, tt)
        n_ok += 1
    assert n_ok > 20


def test_corner_reflections_stay_in_domain():
    wl = W.tiny_canyon(precision="f64")
    m = wl.mesh
    orc = O.Oracle(wl, ensembles=[])
    rng = np.random.default_rng(15)
    for _ in range(3000):
        e = int(rng.integers(m.nelem))
        s = _random_point_in(m, e, rng)
        t = s + rng.normal(scale=0.15, size=2)
        if max(s[1], t[1]) > 1.7:
            continue        # keep clear of the free-slip top, which flips only v
        vel = rng.normal(size=3)
        r, tt, v2, nref = orc.walk(e, s, t, vel)
        assert r >= 0, "walk lost the particle"
        assert _contains(m, r, tt)
        assert np.isclose(np.abs(v2), np.abs(vel)).all()   # no-slip reflections only flip signs
        if nref % 2 == 0:
            np.testing.assert_array_equal(v2, vel)
        else:
            np.testing.assert_array_equal(v2, -vel)


@pytest.mark.parametrize("wl_fn", [lambda: W.config1(steps=20), lambda: W.tiny_canyon(precision="f32")])
def test_steps_keep_particles_located(wl_fn):
    wl = wl_fn()
    orc = O.Oracle(wl)
    n0 = orc.count()
    for _ in range(wl.steps if wl.steps <= 20 else 20):
        orc.step(1)
        st = orc.state()
        assert len(st["x"]) == n0
        a = wl.mesh.vtx[wl.mesh.tri[st["elem"]]]
        p = np.stack([st["x"], st["y"]], axis=1)
        def o(u, v):
            return (v[:, 0] - u[:, 0]) * (p[:, 1] - u[:, 1]) - (v[:, 1] - u[:, 1]) * (p[:, 0] - u[:, 0])
        tol = -1e-12
        assert (o(a[:, 0], a[:, 1]) >= tol).all()
        assert (o(a[:, 1], a[:, 2]) >= tol).all()
        assert (o(a[:, 2], a[:, 0]) >= tol).all()


def test_seeding_uniform_in_triangles_and_element_major():
    wl = W.config1()
    orc = O.Oracle(wl)
    st = orc.state()
    assert (np.diff(st["elem"]) >= 0).all()                 # ids are element-major
    np.testing.assert_array_equal(np.bincount(st["elem"]), wl.ensembles[0].counts)
    m = wl.mesh
    v = m.vtx[m.tri[st["elem"]]]
    p = np.stack([st["x"], st["y"]], axis=1)
    area2 = ((v[:, 1, 0] - v[:, 0, 0]) * (v[:, 2, 1] - v[:, 0, 1]) - (v[:, 1, 1] - v[:, 0, 1]) * (v[:, 2, 0] - v[:, 0, 0]))
    lam0 = ((v[:, 1, 0] - p[:, 0]) * (v[:, 2, 1] - p[:, 1]) - (v[:, 1, 1] - p[:, 1]) * (v[:, 2, 0] - p[:, 0])) / area2
    # a uniform point in a triangle has barycentric marginal P(lambda <= t) = 1 - (1-t)^2
    from scipy import stats
    assert stats.kstest(lam0, lambda t: 1 - (1 - np.clip(t, 0, 1)) ** 2).pvalue > 1e-4
    # C1 seeding: velocity (1,0,0) + sqrt(2k/3) xi
    n = len(p)
    for comp, mean in (("u", 1.0), ("v", 0.0), ("w", 0.0)):
        assert abs(st[comp].mean() - mean) < 5 * np.sqrt(2 / 3 / n)
        assert abs(st[comp].var() - 2 / 3) < 5 * (2 / 3) * np.sqrt(2 / n)
    np.testing.assert_array_equal(st["psi"], (st["x"] < 0.25).astype(float))
