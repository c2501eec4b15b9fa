"""Pins of the oracle parts that uniform-field runs cannot see.

* P1 interpolation (section 2: Eulerian statistics at the particle location)
  reproduces a linear field exactly, so one velocity step under a linear
  mean pressure gradient, with no drift, no diffusion and no viscosity, gives
  dU/dt = -dP/dx at the particle's own position (eq. 6, first term).
* The laminar terms of eq. (6): 2 nu lap<U> adds to the drift with that
  factor; (2 nu)^1/2 d<U_i>/dx_j dW_j shares its dW with the position
  increment of eq. (5), so the one-step cross-covariance of the position and
  velocity increments is 2 nu dt A^T (A_ij = d<U_i>/dx_j), and the stationary
  covariance solves the discrete Lyapunov equation with that extra noise.
* A uniform mean pressure gradient g with the SLM drift G = -a I moves the
  ensemble mean along U_inf + (M_0 - U_inf)(1 - a dt)^n, U_inf = <U> - g / a.
* Eq. (11) with a source: t_m = dt / r is affine in the centroid distance to
  the source (slope C_t / |<U>|, intercept C_s (r0^2 / eps)^(1/3)) up to the
  plateau max(k / eps, C_T (nu / eps)^1/2).
* Seeding with an anisotropic Reynolds stress: the seeded velocity
  covariance is the stress tensor (the Cholesky factor of the 2 x 2 block).
* Wall-function alpha (eqs. 22-26) away from equilibrium: the gamma_tau
  branch at a point where u* = 2 u_hat has the closed form alpha = 2; with
  gamma_tau = 0 the pressure gradient drops out exactly; alpha is invariant
  under (<uv>, dP/dx) -> (-<uv>, -dP/dx), odd in <U>_p and proportional to
  1 / <v^2>_p at fixed k_p.
"""
import math

import numpy as np
import pytest
import scipy.linalg

import oracle as O
import workloads as W
from workloads.fields import F, NFIELD, uniform_fields


def _zero_velocity(orc):
    st = orc.state()
    for k in ("u", "v", "w"):
        st[k] = np.zeros_like(st[k])
    orc.set_state(st)
    return orc.state()


def _linear_case(nu=0.0, lap=None):
    """Unstructured canyon mesh, no drift and no turbulent diffusion (eps = 0:
    <omega> = 0 in the SLM, so G = 0 and C0 eps = 0), linear mean pressure
    gradient, velocity sub-step only."""
    wl = W.tiny_canyon(precision="f64")
    m = wl.mesh
    x, y = m.vtx[:, 0], m.vtx[:, 1]
    f = uniform_fields(m.nvert, U=(0.0, 0.0), k=1.0, eps=0.0)
    f[:, F["dPdx"]] = 0.7 - 1.3 * x + 2.1 * y
    f[:, F["dPdy"]] = -0.4 + 0.9 * x + 1.7 * y
    if lap is not None:
        f[:, F["lapU"]] = lap[0] + lap[1] * x + lap[2] * y
        f[:, F["lapV"]] = lap[3] + lap[4] * x + lap[5] * y
    wl.fields = f
    wl.model = W.SLM
    wl.nu = nu
    wl.flags = 1
    wl.mix = False
    en = wl.ensembles[0]
    return wl, O.Oracle(wl, ensembles=[W.Ensemble(counts=en.counts, seed=3, r0=0.0)])


def test_interpolation_reproduces_a_linear_pressure_gradient():
    wl, orc = _linear_case()
    s0 = _zero_velocity(orc)
    orc.step(1)
    s1 = orc.state()
    np.testing.assert_array_equal(s1["x"], s0["x"])
    ex = -(0.7 - 1.3 * s0["x"] + 2.1 * s0["y"])
    ey = -(-0.4 + 0.9 * s0["x"] + 1.7 * s0["y"])
    scale = max(np.abs(ex).max(), np.abs(ey).max())
    assert np.abs(s1["u"] / wl.dt - ex).max() <= 1e-12 * scale
    assert np.abs(s1["v"] / wl.dt - ey).max() <= 1e-12 * scale
    np.testing.assert_array_equal(s1["w"], 0.0)
    # the fields vary enough over an element for a swapped weight to show
    assert np.ptp(ex) > 1.0 and np.ptp(ey) > 1.0


def test_viscous_drift_enters_with_twice_the_viscosity():
    nu = 0.01
    lap = (1.5, -2.0, 0.5, -0.8, 1.1, 2.4)
    wl, orc = _linear_case(nu=nu, lap=lap)
    s0 = _zero_velocity(orc)
    orc.step(1)
    s1 = orc.state()
    x, y = s0["x"], s0["y"]
    ex = -(0.7 - 1.3 * x + 2.1 * y) + 2 * nu * (lap[0] + lap[1] * x + lap[2] * y)
    ey = -(-0.4 + 0.9 * x + 1.7 * y) + 2 * nu * (lap[3] + lap[4] * x + lap[5] * y)
    scale = max(np.abs(ex).max(), np.abs(ey).max())
    assert np.abs(s1["u"] / wl.dt - ex).max() <= 1e-12 * scale
    assert np.abs(s1["v"] / wl.dt - ey).max() <= 1e-12 * scale
    # and the viscous part is far above that bar
    assert 2 * nu * 0.5 > 1e-6 * scale


def _box(fields, nu=0.0, flags=15, ppe=400, seed=21, C0=2.1, n=8):
    wl = W.configs.square_box(n=n, ppe=ppe, periodic_y=True, precision="f64", seed=seed, model=W.SLM,
                              dt=0.01, fields=fields, C0=C0)
    wl.nu = nu
    wl.flags = flags
    return wl


def test_uniform_pressure_gradient_moves_the_mean_to_its_closed_form():
    g = np.array([0.8, -0.5])
    Um = np.array([0.3, 0.2])

    def fields(m):
        f = uniform_fields(m.nvert, U=tuple(Um), k=1.0, eps=1.0)
        f[:, F["dPdx"]], f[:, F["dPdy"]] = g
        return f

    wl = _box(fields)
    orc = O.Oracle(wl)
    a = -orc.coefficients()[0, 10]             # SLM: G = -(1/2 + 3/4 C0) <omega> I
    assert abs(a - (0.5 + 0.75 * 2.1)) < 1e-14
    st = orc.state()
    M0 = np.array([st["u"].mean(), st["v"].mean()])
    Uinf = Um - g / a
    n_part = len(st["u"])
    done = 0
    for n in (20, 100):
        orc.step(n - done)
        done = n
        st = orc.state()
        M = np.array([st["u"].mean(), st["v"].mean()])
        pred = Uinf + (M0 - Uinf) * (1 - a * wl.dt) ** n
        se = np.sqrt(np.array([st["u"].var(), st["v"].var()]) / n_part)
        assert (np.abs(M - pred) < 4 * se).all(), (n, M, pred, se)
        assert abs(st["w"].mean()) < 4 * math.sqrt(st["w"].var() / n_part)
    # the pressure gradient has moved the mean by many standard errors
    assert (np.abs(M - M0) > 20 * se).all()


A_GRAD = np.array([[0.3, 1.2], [-0.4, 0.5]])      # A_ij = d<U_i>/dx_j, uniform


def _gradient_box(nu):
    def fields(m):
        f = uniform_fields(m.nvert, U=(0.0, 0.0), k=1.0, eps=1.0)
        f[:, F["dUdx"]], f[:, F["dUdy"]] = A_GRAD[0]
        f[:, F["dVdx"]], f[:, F["dVdy"]] = A_GRAD[1]
        return f
    return _box(fields, nu=nu, flags=3)


def _unwrap(d):
    return d - np.round(d)   # the doubly periodic unit box


def test_velocity_gradient_noise_shares_the_position_increment():
    nu = 0.05
    wl = _gradient_box(nu)
    orc = O.Oracle(wl)
    s0 = orc.state()
    orc.step(1)
    s1 = orc.state()
    dt = wl.dt
    dX = np.stack([_unwrap(s1["x"] - s0["x"]) - s0["u"] * dt, _unwrap(s1["y"] - s0["y"]) - s0["v"] * dt])
    dU = np.stack([s1["u"] - s0["u"], s1["v"] - s0["v"]])
    n = dX.shape[1]
    C = (dX - dX.mean(axis=1, keepdims=True)) @ (dU - dU.mean(axis=1, keepdims=True)).T / n
    expect = 2 * nu * dt * A_GRAD.T          # E[dX_i dU_j] = 2 nu dt A_ji
    vx = dX.var(axis=1)
    vu = dU.var(axis=1)
    se = np.sqrt(np.outer(vx, vu) / n)
    assert (np.abs(C - expect) < 4 * se).all(), (C, expect, se)
    # the position increment alone is the molecular diffusion, variance 2 nu dt
    np.testing.assert_allclose(vx, 2 * nu * dt, rtol=4 * math.sqrt(2 / n))
    # A and its transpose differ by many standard errors
    assert np.abs(expect - 2 * nu * dt * A_GRAD).max() > 20 * se.max()


def test_velocity_gradient_noise_in_the_stationary_covariance():
    nu = 0.2
    wl = _gradient_box(nu)
    orc = O.Oracle(wl)
    coef = orc.coefficients()[0]
    G, c0eps = coef[10], coef[15]
    dt = wl.dt
    Amat = np.eye(3) * (1 + G * dt)
    A3 = np.zeros((3, 2))
    A3[:2, :] = A_GRAD
    Q = c0eps * dt * np.eye(3) + 2 * nu * dt * A3 @ A3.T
    st = orc.state()
    R = np.cov(np.stack([st["u"], st["v"], st["w"]]), bias=True)
    nsteps = 600
    for _ in range(nsteps):
        R = Amat @ R @ Amat.T + Q
    Rinf = scipy.linalg.solve_discrete_lyapunov(Amat, Q)
    assert np.abs(R - Rinf).max() < 0.01 * np.abs(Rinf).max()
    orc.step(nsteps)
    st = orc.state()
    X = np.stack([st["u"], st["v"], st["w"]])
    C = np.cov(X, bias=True)
    n = X.shape[1]
    se = np.sqrt((np.outer(np.diag(R), np.diag(R)) + R * R) / n)
    assert (np.abs(C - R) < 4.5 * se).all(), (C, R)
    # without the gradient noise the u-v covariance would vanish
    assert abs(R[0, 1]) > 10 * se[0, 1]


def _rate_box(U, k, eps, nu, x0, r0):
    def fields(m):
        return uniform_fields(m.nvert, U=U, k=k, eps=eps)
    wl = W.configs.square_box(n=20, ppe=1, periodic_y=False, precision="f64", seed=1, model=W.SLM,
                              dt=1e-3, fields=fields)
    wl.nu = nu
    m = wl.mesh
    ens = [W.Ensemble(counts=np.ones(m.nelem, np.int64), seed=1, x0=x0, r0=r0)]
    orc = O.Oracle(wl, ensembles=ens)
    cen = m.vtx[m.tri].mean(axis=1)
    d = np.hypot(cen[:, 0] - x0[0], cen[:, 1] - x0[1])
    return wl, orc, d


def test_mixing_time_with_a_source_is_affine_in_the_distance():
    U, k, eps, nu = (0.6, 0.8), 1.0, 0.5, 1.0 / 12000.0
    x0, r0 = (0.5, 0.5), 0.05
    wl, orc, d = _rate_box(U, k, eps, nu, x0, r0)
    r = orc.mix_rate()
    assert (r < 1).all()
    tm = wl.dt / r
    plateau = max(k / eps, 6.0 * math.sqrt(nu / eps))
    below = tm < plateau * (1 - 1e-9)
    assert below.sum() > 100
    Amat = np.stack([np.ones(below.sum()), d[below]], axis=1)
    (c0, c1), *_ = np.linalg.lstsq(Amat, tm[below], rcond=None)
    Uc = math.hypot(*U)
    assert abs(c1 - 0.7 / Uc) < 1e-9 * (0.7 / Uc)
    assert abs(c0 - 0.02 * (r0 * r0 / eps) ** (1 / 3)) < 1e-9 * 0.02 * (r0 * r0 / eps) ** (1 / 3)
    assert np.abs(Amat @ np.array([c0, c1]) - tm[below]).max() < 1e-12 * tm[below].max()


def test_mixing_time_plateau_and_the_viscous_branch():
    # |<U>| small: the advection term exceeds the plateau everywhere but at
    # the source; nu large: C_T (nu / eps)^1/2 beats k / eps
    U, k, eps, nu = (0.003, 0.004), 0.1, 1.0, 1.0
    x0, r0 = (0.5, 0.5), 0.05
    wl, orc, d = _rate_box(U, k, eps, nu, x0, r0)
    tm = wl.dt / orc.mix_rate()
    plateau = 6.0 * math.sqrt(nu / eps)
    assert plateau > k / eps
    far = 0.02 * (r0 * r0 / eps) ** (1 / 3) + 0.7 * d / math.hypot(*U) > plateau
    assert far.sum() > 0.9 * len(d)
    np.testing.assert_allclose(tm[far], plateau, rtol=1e-14)
    assert (tm[~far] < plateau).all()
    # no mean velocity: the advection term is unbounded, the plateau everywhere
    wl, orc, d = _rate_box((0.0, 0.0), k, eps, nu, x0, r0)
    np.testing.assert_allclose(wl.dt / orc.mix_rate(), plateau, rtol=1e-14)


def test_seeding_with_an_anisotropic_reynolds_stress():
    Rm = np.array([[0.5, -0.2, 0.0], [-0.2, 0.3, 0.0], [0.0, 0.0, 0.4]])
    Um = np.array([0.7, -0.1, 0.0])

    def fields(m):
        f = uniform_fields(m.nvert, U=tuple(Um[:2]), k=1.0, eps=1.0)
        f[:, F["R11"]], f[:, F["R22"]], f[:, F["R33"]], f[:, F["R12"]] = Rm[0, 0], Rm[1, 1], Rm[2, 2], Rm[0, 1]
        return f

    wl = _box(fields, ppe=800)
    st = O.Oracle(wl).state()
    X = np.stack([st["u"], st["v"], st["w"]])
    n = X.shape[1]
    se_m = np.sqrt(np.diag(Rm) / n)
    assert (np.abs(X.mean(axis=1) - Um) < 4 * se_m).all()
    C = np.cov(X, bias=True)
    se = np.sqrt((np.outer(np.diag(Rm), np.diag(Rm)) + Rm * Rm) / n)
    assert (np.abs(C - Rm) < 4 * se).all(), (C, Rm)
    assert abs(Rm[0, 1]) > 50 * se[0, 1]


NU_WF, YP_WF, UHAT = 1.0 / 12000.0, 13.0 / 256.0, 0.05


def _log_law(ustar):
    return ustar / 0.41 * math.log(8.5 * YP_WF * ustar / NU_WF)


def _alpha_street_roof(U_p, v2_p, k_p, dPdx=0.0, uv=0.0):
    """alpha on the street and roof edges of the stripped canyon (tangent +x,
    fluid above) for uniform fields with the given wall statistics."""
    wl = W.small_canyon(target=600, ppe=5, wallfn=True, precision="f64")
    f = np.zeros((wl.mesh.nvert, NFIELD))
    f[:, F["U"]] = U_p
    f[:, F["R11"]] = k_p
    f[:, F["R22"]] = v2_p
    f[:, F["R33"]] = k_p - v2_p            # k = (R11 + R22 + R33) / 2 = k_p
    f[:, F["R12"]] = uv
    f[:, F["dPdx"]] = dPdx
    f[:, F["eps"]] = 1.0
    wl.fields = f
    wl.nu = NU_WF
    wl.yp = YP_WF
    orc = O.Oracle(wl, ensembles=[])
    al = orc.wall_alpha()
    m = wl.mesh
    from workloads.mesh import EDGE
    e, kk = np.nonzero(m.ekind == EDGE.WALLFN)
    a = m.vtx[m.tri[e, kk]]
    b = m.vtx[m.tri[e, (kk + 1) % 3]]
    flat = (a[:, 1] == b[:, 1]) & ((a[:, 1] == YP_WF) | (a[:, 1] == 1 + YP_WF))
    assert flat.sum() > 4
    return al[e[flat], kk[flat]]


def test_alpha_with_the_pressure_gradient_branch_at_a_closed_form_point():
    # gamma_tau = 1 (<uv> dP/dx > 0 in the edge frame) and y_p |dP/dx| = 3 u_hat^2
    # make u* = 2 u_hat (eq. 25); with <U>_p = U_e(u*) and <v^2>_p = u_hat^2,
    # eq. (22) gives alpha = 2
    k_p = UHAT ** 2 / math.sqrt(0.09)
    dPdx = 3 * UHAT ** 2 / YP_WF
    al = _alpha_street_roof(_log_law(2 * UHAT), UHAT ** 2, k_p, dPdx=dPdx, uv=0.01)
    np.testing.assert_allclose(al, 2.0, rtol=1e-12)
    # and without the branch (dP/dx of the opposite sign) the gradient drops
    # out: the value at dP/dx = 0, (U_e(2 u_hat) / U_e(u_hat))^2 times larger
    off = _alpha_street_roof(_log_law(2 * UHAT), UHAT ** 2, k_p, dPdx=-dPdx, uv=0.01)
    zero = _alpha_street_roof(_log_law(2 * UHAT), UHAT ** 2, k_p, dPdx=0.0, uv=0.01)
    np.testing.assert_array_equal(off, zero)
    np.testing.assert_allclose(zero, 2.0 * (_log_law(2 * UHAT) / _log_law(UHAT)) ** 2, rtol=1e-12)


def test_alpha_symmetries():
    k_p = UHAT ** 2 / math.sqrt(0.09)
    base = dict(U_p=0.9, v2_p=0.6 * k_p, k_p=k_p, dPdx=0.02, uv=0.004)
    a0 = _alpha_street_roof(**base)
    assert (a0 > 0).all()
    # (<uv>, dP/dx) -> (-<uv>, -dP/dx): gamma_tau and u* unchanged
    a1 = _alpha_street_roof(**dict(base, dPdx=-0.02, uv=-0.004))
    np.testing.assert_array_equal(a1, a0)
    # odd in <U>_p
    a2 = _alpha_street_roof(**dict(base, U_p=-0.9))
    np.testing.assert_array_equal(a2, -a0)
    # proportional to 1 / <v^2>_p at fixed k_p
    a3 = _alpha_street_roof(**dict(base, v2_p=0.3 * k_p))
    np.testing.assert_allclose(a3, 2.0 * a0, rtol=1e-14)
    # the branch is on here: the gradient lowers alpha against dP/dx = 0
    a4 = _alpha_street_roof(**dict(base, dPdx=0.0))
    assert (a0 < a4).all()
