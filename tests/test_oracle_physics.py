"""Pins of the oracle's model equations against closed forms and invariants.

* Velocity (eq. 6, SLM eq. 19 and GLM eqs. 12-13): under homogeneous k and eps
  the Euler-Maruyama scheme is the discrete Ornstein-Uhlenbeck process
  u_{n+1} = A u_n + b xi; its covariance follows R_{n+1} = A R_n A^T + C0 eps
  dt I, solved in closed form (scalar case) or by scipy's discrete Lyapunov
  solver (anisotropic drift tensor).
* IECM (eq. 7): per (element, velocity bin) the scalar sum is unchanged and
  the centred sum of squares shrinks by (1 - r)^2 exactly; the scalar stays
  in [0, 1]; the global mean is conserved without a source.
* Micro-mixing time (eq. 11) and wall-function alpha (eqs. 22-26) special
  cases, and the source (section 3).
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from workloads.fields import F, NFIELD, uniform_fields


def _discrete_ou_variance(var0, a, b2, n):
    a2n = a ** (2 * n)
    return a2n * var0 + (1 - a2n) * b2 / (1 - a * a)


def test_slm_ornstein_uhlenbeck_variance_config1():
    wl = W.config1()
    orc = O.Oracle(wl)
    C0, eps, k, dt = 2.1, 1.0, 1.0, 0.01
    G = -(0.5 + 0.75 * C0) * eps / k               # = -2.075
    a, b2 = 1 + G * dt, C0 * eps * dt
    # the discrete stationary variance differs from the continuous one by ~1 %
    assert abs(b2 / (1 - a * a) - 0.5113291) < 1e-6
    n_part = orc.count()
    done = 0
    for n in (10, 50, 100):
        orc.step(n - done)
        done = n
        st = orc.state()
        ref = _discrete_ou_variance(2.0 / 3.0, a, b2, n)
        for comp in ("u", "v", "w"):
            var = st[comp].var()
            se = ref * math.sqrt(2.0 / n_part)
            assert abs(var - ref) < 4 * se, (n, comp, var, ref)
        assert abs(st["u"].mean() - 1.0) < 4 * math.sqrt(ref / n_part)
        assert abs(st["v"].mean()) < 4 * math.sqrt(ref / n_part)
    assert abs(_discrete_ou_variance(2.0 / 3.0, a, b2, 100) - 0.5136733) < 1e-6


def _box_with_wp(wp, k=1.0, eps=1.0, n=8, ppe=400, seed=21):
    """Doubly periodic box, no mean flow, isotropic stresses, given wp tensor."""
    def fields(m):
        f = uniform_fields(m.nvert, U=(0.0, 0.0), k=k, eps=eps)
        f[:, F["P11"]], f[:, F["P12"]], f[:, F["P21"]], f[:, F["P22"]], f[:, F["P33"]] = wp
        return f
    return W.configs.square_box(n=n, ppe=ppe, periodic_y=True, precision="f64", seed=seed,
                                model=W.GLM, dt=0.01, fields=fields)


def test_glm_isotropic_wp_reduces_to_rotta():
    # wp = 1/2 (1 - C1) k <omega> delta (eq. 14 without the rapid part):
    # G = -C1/2 <omega>, C0 = 2 (C1 - 1) / 3 (with nu = 0, eps = k <omega>)
    C1 = 1.85
    w = 0.5 * (1 - C1)
    wl = _box_with_wp((w, 0.0, 0.0, w, w))
    orc = O.Oracle(wl)
    coef = orc.coefficients()
    np.testing.assert_allclose(coef[:, 10], -C1 / 2, rtol=1e-15)
    np.testing.assert_allclose(coef[:, 13], -C1 / 2, rtol=1e-15)
    np.testing.assert_allclose(coef[:, 14], -C1 / 2, rtol=1e-15)
    np.testing.assert_array_equal(coef[:, 11], 0.0)
    np.testing.assert_allclose(coef[:, 15], 2 * (C1 - 1) / 3, rtol=1e-15)
    a, b2 = 1 - C1 / 2 * wl.dt, 2 * (C1 - 1) / 3 * wl.dt
    orc.step(150)
    st = orc.state()
    ref = _discrete_ou_variance(2 / 3, a, b2, 150)
    for comp in ("u", "v", "w"):
        assert abs(st[comp].var() - ref) < 4 * ref * math.sqrt(2 / len(st["u"]))


def test_glm_anisotropic_drift_matches_discrete_lyapunov():
    G2 = np.array([[-2.0, 0.6], [-0.3, -1.5]])
    G33 = -1.8
    # wp_ij = (2k G_ij + eps delta_ij) / 2 with k = eps = 1 (inverse of eq. 12)
    wp = (G2[0, 0] + 0.5, G2[0, 1], G2[1, 0], G2[1, 1] + 0.5, G33 + 0.5)
    wl = _box_with_wp(wp)
    orc = O.Oracle(wl)
    coef = orc.coefficients()[0]
    np.testing.assert_allclose(coef[10:15], [G2[0, 0], G2[0, 1], G2[1, 0], G2[1, 1], G33], rtol=1e-14)
    # eq. (13) with R = 2/3 I: C0 = -(4/9) tr(wp)
    C0 = -(4.0 / 9.0) * (wp[0] + wp[3] + wp[4])
    assert abs(coef[15] - C0) < 1e-14
    dt = wl.dt
    A = np.eye(3)
    A[:2, :2] += G2 * dt
    A[2, 2] += G33 * dt
    Q = C0 * dt * np.eye(3)
    R0 = 2.0 / 3.0 * np.eye(3)
    nsteps = 300
    R = R0
    for _ in range(nsteps):
        R = A @ R @ A.T + Q
    Rinf = scipy.linalg.solve_discrete_lyapunov(A, Q)
    assert np.abs(R - Rinf).max() < 0.02 * np.abs(Rinf).max()
    orc.step(nsteps)
    st = orc.state()
    X = np.stack([st["u"], st["v"], st["w"]])
    C = np.cov(X, bias=True)
    n = X.shape[1]
    se = np.sqrt((np.outer(np.diag(R), np.diag(R)) + R * R) / n)
    assert (np.abs(C - R) < 4.5 * se).all(), (C, R)


def _mix_only(wl):
    wl.flags = 4
    return wl


def test_iecm_conserves_bin_sums_and_contracts_variance():
    wl = _mix_only(W.config1())
    orc = O.Oracle(wl)
    st0 = orc.state()
    stats0 = orc.stats()
    orc.step(1)
    st1 = orc.state()
    # position and velocity untouched in the IECM-only step
    for k in ("x", "y", "u", "v", "w", "elem"):
        np.testing.assert_array_equal(st0[k], st1[k])
    e = st0["elem"]
    mean = stats0[e, 1:4]
    b = (st0["u"] > mean[:, 0]) * 1 + (st0["v"] > mean[:, 1]) * 2 + (st0["w"] > mean[:, 2]) * 4
    key = e * 8 + b
    r = orc.mix_rate()[e]
    np.testing.assert_allclose(r, wl.dt, rtol=1e-15)           # t_m = max(k/eps, ...) = 1 in C1
    s0 = np.bincount(key, weights=st0["psi"], minlength=8 * wl.mesh.nelem)
    s1 = np.bincount(key, weights=st1["psi"], minlength=8 * wl.mesh.nelem)
    np.testing.assert_allclose(s1, s0, rtol=0, atol=1e-13)
    cnt = np.bincount(key, minlength=8 * wl.mesh.nelem)
    m0 = np.divide(s0, cnt, out=np.zeros_like(s0), where=cnt > 0)[key]
    c0 = np.bincount(key, weights=(st0["psi"] - m0) ** 2, minlength=8 * wl.mesh.nelem)
    c1 = np.bincount(key, weights=(st1["psi"] - m0) ** 2, minlength=8 * wl.mesh.nelem)
    np.testing.assert_allclose(c1, (1 - wl.dt) ** 2 * c0, rtol=1e-11, atol=1e-15)


def test_scalar_bounded_and_globally_conserved_config1():
    wl = W.config1(steps=60)
    orc = O.Oracle(wl)
    total0 = orc.state()["psi"].sum()
    for _ in range(6):
        orc.step(10)
        psi = orc.state()["psi"]
        assert psi.min() >= 0.0 and psi.max() <= 1.0
        assert abs(psi.sum() - total0) < len(psi) * 1e-14
    # mixing makes the scalar variance decay
    assert orc.state()["psi"].var() < 0.75 * 0.1875


def test_mix_rate_special_cases():
    wl = W.tiny_canyon(precision="f64")
    orc = O.Oracle(wl)
    r = orc.mix_rate()
    assert (r > 0).all() and (r <= 1).all()
    # without a source t_m = max(k/eps, C_T sqrt(nu/eps)) everywhere
    en = wl.ensembles[0]
    nosrc = W.Ensemble(counts=en.counts, seed=en.seed, x0=en.x0, r0=0.0)
    orc2 = O.Oracle(wl, ensembles=[nosrc])
    r2 = orc2.mix_rate()
    m, f = wl.mesh, wl.fields
    kv = 0.5 * (f[:, F["R11"]] + f[:, F["R22"]] + f[:, F["R33"]])
    kc = kv[m.tri].mean(axis=1)
    ec = f[:, F["eps"]][m.tri].mean(axis=1)
    tm = np.maximum(kc / ec, 6.0 * np.sqrt(wl.nu / ec))
    np.testing.assert_allclose(r2, np.minimum(wl.dt / tm, 1.0), rtol=1e-12)
    # the source shortens the mixing time near it, never lengthens it
    assert (r >= r2 * (1 - 1e-12)).all()
    assert (r > r2 * (1 + 1e-9)).any()


def _wallfn_strip(U_p, v2_p, k_p, dPdx=0.0, uv=0.0, yp=13 / 256, nu=1 / 12000):
    """Stripped canyon with uniform fields chosen for the alpha special case."""
    wl = W.small_canyon(target=600, ppe=5, wallfn=True, precision="f64")
    f = np.zeros((wl.mesh.nvert, NFIELD))
    f[:, F["U"]] = U_p
    # stresses: wall-normal variance v2_p, k = k_p, no shear stress
    f[:, F["R11"]] = k_p
    f[:, F["R22"]] = v2_p
    f[:, F["R33"]] = 2 * k_p - k_p - v2_p
    f[:, F["R12"]] = uv
    f[:, F["dPdx"]] = dPdx
    f[:, F["eps"]] = 1.0
    wl.fields = f
    wl.nu = nu
    wl.yp = yp
    return wl


def test_wall_function_alpha_equilibrium_special_case():
    # With no pressure gradient u* = uhat = C_mu^(1/4) k^(1/2) (eq. 25); choosing
    # <U>_p equal to the log-law value U_e (eq. 24) and <v^2>_p = uhat^2 makes
    # alpha = 2 on a wall whose tangent points along +x (the street, eq. 22).
    nu, yp = 1.0 / 12000.0, 13.0 / 256.0
    uhat = 0.05
    k_p = uhat ** 2 / math.sqrt(0.09)
    Ue = uhat / 0.41 * math.log(8.5 * yp * uhat / nu)
    wl = _wallfn_strip(U_p=Ue, v2_p=uhat ** 2, k_p=k_p, yp=yp, nu=nu)
    orc = O.Oracle(wl, ensembles=[])
    al = orc.wall_alpha()
    m = wl.mesh
    from workloads.mesh import EDGE
    e, kk = np.nonzero(m.ekind == EDGE.WALLFN)
    a = m.vtx[m.tri[e, kk]]
    b = m.vtx[m.tri[e, (kk + 1) % 3]]
    street = (a[:, 1] == yp) & (b[:, 1] == yp)
    roof = (a[:, 1] == 1 + yp) & (b[:, 1] == 1 + yp)
    side = a[:, 0] == b[:, 0]
    assert street.any() and roof.any() and side.any()
    np.testing.assert_allclose(al[e[street], kk[street]], 2.0, rtol=1e-12)
    # roofs: the fluid is above as on the street, so the same frame and value
    np.testing.assert_allclose(al[e[roof], kk[roof]], 2.0, rtol=1e-12)
    # side walls: no tangential mean velocity, no slip correction
    np.testing.assert_array_equal(al[e[side], kk[side]], 0.0)
    assert (al[m.ekind != EDGE.WALLFN] == 0).all()


def test_wall_function_reflection_on_the_street():
    nu, yp = 1.0 / 12000.0, 13.0 / 256.0
    uhat = 0.05
    k_p = uhat ** 2 / math.sqrt(0.09)
    Ue = uhat / 0.41 * math.log(8.5 * yp * uhat / nu)
    wl = _wallfn_strip(U_p=Ue, v2_p=uhat ** 2, k_p=k_p, yp=yp, nu=nu)
    orc = O.Oracle(wl, ensembles=[])
    m = wl.mesh
    rng = np.random.default_rng(5)
    hits = 0
    for _ in range(4000):
        e = int(rng.integers(m.nelem))
        v = m.vtx[m.tri[e]]
        s = v.mean(axis=0)
        if not (0.7 < s[0] < 1.3 and s[1] < yp + 0.05):
            continue
        t = np.array([s[0] + 0.003, yp - 0.002])
        vel = np.array([0.3, -0.2, 0.1])
        r, tt, v2, nref = orc.walk(e, s, t, vel)
        assert nref == 1 and r >= 0
        # eqs. (20)-(21): V_R = -V_I, U_R = U_I + alpha V_I with alpha = 2
        np.testing.assert_allclose(v2, [0.3 + 2.0 * (-0.2), 0.2, 0.1], rtol=1e-15)
        assert abs(tt[1] - (2 * yp - t[1])) < 1e-15
        hits += 1
    assert hits > 0


def test_source_sets_unit_scalar():
    wl = W.small_canyon(target=600, ppe=30, precision="f32")
    orc = O.Oracle(wl)
    en = wl.ensembles[0]
    orc.step(3)
    st = orc.state()
    d2 = (st["x"] - en.x0[0]) ** 2 + (st["y"] - en.x0[1]) ** 2
    inside = d2 <= en.r0 ** 2
    assert inside.sum() > 5
    np.testing.assert_array_equal(st["psi"][inside], 1.0)
    assert st["psi"].min() >= 0 and st["psi"].max() <= 1
