"""Pins of the elliptic-relaxation oracle (section 2.1, eqs. 12-18).

* The Galerkin P1 solve converges at second order in the L2 norm to a
  manufactured solution: w = cos(2 pi x) cos(pi y) on the unit square,
  periodic in x with natural conditions at y = 0 and 1, solves
  w - L^2 lap w = (1 + 5 pi^2 L^2) w.
* With L = 0 and a uniform right-hand side the solution is that value at
  every unknown (the mass matrix reproduces constants).
* The system matrix is symmetric positive definite.
* Periodic seams: the unit square periodic in x has n (n + 1) unknowns, the
  doubly periodic box n^2.
* The right-hand side of eq. (14) for simple shear d<U>/dy = g: with
  isotropic stresses (b = 0, A_v = 1) it is k (C2 + gamma5/3) g in the 12
  component and -k gamma5/3 g in the 21 component, the slow term on the
  diagonal; with anisotropic stresses the b terms of eq. (15) add
  k gamma5 g (b_11, -b_22) to those and -k gamma5 g b_12, k gamma5 g b_21 to
  the 11 and 22 components.
* eq. (18): L from the turbulent length when it is the larger, from the
  Kolmogorov length otherwise.
* G and C0 of eqs. (12)-(13) from the isotropic slow term alone reduce to the
  Rotta model: G = -C1/2 <omega>, C0 = 2 (C1 - 1) / 3 (nu = 0).
"""
import math

import numpy as np
import pytest

import oracle.relax as R
import workloads as W

# Table 2 of the paper, written here independently of the oracle's copy
C1, C2, CL, CETA, CV, GAMMA5 = 1.85, 0.63, 0.134, 72.0, 1.4, 0.1
C_XI = 1.0 + 1.3 * 1.0          # eq. (18) with a unit wall normal
from workloads.fields import F, NFIELD, uniform_fields
from workloads.mesh import doubly_periodic_box, unit_square_mesh


def _manufactured_error(n, L):
    m = unit_square_mesh(n)
    cen = m.vtx[m.tri].mean(axis=1)
    exact = lambda x, y: np.cos(2 * math.pi * x) * np.cos(math.pi * y)
    S = (1 + 5 * math.pi ** 2 * L * L) * exact(cen[:, 0], cen[:, 1])
    w, parts = R.solve_with(m, np.full(m.nelem, L * L), S)
    canon, M = parts["canon"], parts["M"]
    ref = np.zeros(parts["nc"])
    ref[canon] = exact(m.vtx[:, 0], m.vtx[:, 1])
    e = w[:, 0] - ref
    return math.sqrt(e @ (M @ e))


def test_manufactured_solution_converges_at_second_order():
    L = 0.1
    errs = [_manufactured_error(n, L) for n in (8, 16, 32)]
    rates = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(1.8 < r < 2.3 for r in rates), (errs, rates)
    assert errs[-1] < 5e-3


def test_zero_length_and_uniform_source_give_the_source():
    m = W.tiny_canyon(precision="f64").mesh
    w, _ = R.solve_with(m, np.zeros(m.nelem), np.full(m.nelem, 0.37))
    np.testing.assert_allclose(w[:, 0], 0.37, rtol=1e-12)


def test_system_matrix_is_symmetric_positive_definite():
    m = W.tiny_canyon(precision="f64").mesh
    rng = np.random.default_rng(1)
    M, K, canon, nc, area = R.assemble(m, rng.uniform(0.0, 0.01, m.nelem))
    A = (M + K).toarray()
    assert np.abs(A - A.T).max() == 0.0
    assert np.linalg.eigvalsh(A).min() > 0.0
    # the stiffness part annihilates constants (natural conditions, seams joined)
    np.testing.assert_allclose(K @ np.ones(nc), 0.0, atol=1e-14)


def test_periodic_seams_share_unknowns():
    n = 6
    canon, nc = R.canonical_vertices(unit_square_mesh(n))
    assert nc == n * (n + 1)
    canon, nc = R.canonical_vertices(doubly_periodic_box(n))
    assert nc == n * n
    m = W.tiny_canyon(precision="f64").mesh
    canon, nc = R.canonical_vertices(m)
    on_seam = (m.vtx[:, 0] == 0.0) | (m.vtx[:, 0] == m.Lx)
    assert nc == m.nvert - on_seam.sum() // 2


def test_rhs_for_simple_shear():
    k, om, g = 0.3, 2.0, 1.7
    grad = np.zeros((1, 3, 3))
    grad[0, 0, 1] = g
    iso = np.eye(3)[None] * (2 * k / 3)
    S = R.rhs_tensor(np.array([k]), iso, np.array([om]), grad)[0]
    slow = 0.5 * (1 - C1) * k * om
    np.testing.assert_allclose(S[0, 1], k * (C2 + GAMMA5 / 3) * g, rtol=1e-14)
    np.testing.assert_allclose(S[1, 0], -k * GAMMA5 / 3 * g, rtol=1e-14)
    np.testing.assert_allclose(np.diag(S), slow, rtol=1e-14)
    assert S[0, 2] == S[2, 0] == S[1, 2] == S[2, 1] == 0.0
    # anisotropic: tr R = 2k with b = R / tr R - I/3
    Ran = np.array([[0.26, -0.05, 0.0], [-0.05, 0.16, 0.0], [0.0, 0.0, 0.18]])
    kk = 0.5 * np.trace(Ran)
    b = Ran / np.trace(Ran) - np.eye(3) / 3
    Av = min(1.0, CV * (2 * kk / 3) ** -3 * np.linalg.det(Ran))
    S = R.rhs_tensor(np.array([kk]), Ran[None], np.array([om]), grad)[0]
    slow = 0.5 * (1 - C1) * kk * om
    np.testing.assert_allclose(S[0, 1], kk * g * (C2 * Av + GAMMA5 / 3 + GAMMA5 * b[0, 0]), rtol=1e-13)
    np.testing.assert_allclose(S[1, 0], kk * g * (-GAMMA5 / 3 - GAMMA5 * b[1, 1]), rtol=1e-13)
    np.testing.assert_allclose(S[0, 0], slow - kk * g * GAMMA5 * b[0, 1], rtol=1e-13)
    np.testing.assert_allclose(S[1, 1], slow + kk * g * GAMMA5 * b[1, 0], rtol=1e-13)
    np.testing.assert_allclose(S[2, 2], slow, rtol=1e-13)


def _square_case(k=0.3, eps=0.5, nu=0.0, n=4):
    m = unit_square_mesh(n)
    f = uniform_fields(m.nvert, U=(0.0, 0.0), k=k, eps=eps)
    stats = np.zeros((m.nelem, 31))
    stats[:, 0] = 100
    r = 2 * k / 3
    stats[:, 5], stats[:, 9], stats[:, 12] = r, r, r        # u'u', v'v', w'w'
    return m, f, stats


def test_length_scale_branches():
    m, f, stats = _square_case(k=0.3, eps=0.5, nu=1e-5)
    ins = R.element_inputs(m, f, stats, 1e-5)
    np.testing.assert_allclose(np.sqrt(ins["L2"]), CL * C_XI * 0.3 ** 1.5 / 0.5, rtol=1e-13)
    m, f, stats = _square_case(k=1e-4, eps=0.5, nu=1e-2)
    ins = R.element_inputs(m, f, stats, 1e-2)
    np.testing.assert_allclose(np.sqrt(ins["L2"]), CL * CETA * (1e-6 / 0.5) ** 0.25, rtol=1e-13)


def test_coefficients_reduce_to_rotta_for_the_slow_term():
    m, f, stats = _square_case(k=0.3, eps=0.5, nu=0.0)
    wp, parts = R.solve(m, f, stats, 0.0)
    coef, neg = R.vertex_coefficients(m, f, wp, parts)
    om = 0.5 / 0.3
    np.testing.assert_allclose(coef[:, 0], -C1 / 2 * om, rtol=1e-12)
    np.testing.assert_allclose(coef[:, 3], -C1 / 2 * om, rtol=1e-12)
    np.testing.assert_allclose(coef[:, 4], -C1 / 2 * om, rtol=1e-12)
    np.testing.assert_allclose(coef[:, 1:3], 0.0, atol=1e-14)
    np.testing.assert_allclose(coef[:, 5], 2 * (C1 - 1) / 3 * 0.5, rtol=1e-12)
    assert neg == 0
